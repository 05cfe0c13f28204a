"""GPU parity of the batched form (one captured graph for many matrices of uneven size, each
with its own bounds, degree and probe seed) against per-matrix oracle runs."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._gpu import U32, U64, dev, floor_for, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ld():
    import torch

    assert torch.cuda.is_available()
    import paper_1503_06394_amd as pkg

    pkg.lib()
    return pkg


def _batch(count, storage, d_max=6000, seed0=300):
    mats = synth.random_batch(count, mseed0=seed0, d_min=20, d_max=d_max, n_min=3, n_max=40, storage=storage)
    return mats


@pytest.mark.parametrize("storage,tol,plain", [("f32", 1e-4, False), ("f64", 1e-10, False), ("bf16", 1e-4, False),
                                               ("f32", 1e-4, True), ("f64", 1e-10, True)])
def test_batched_parity(ld, oracle_lib, storage, tol, plain):
    mats = _batch(14, storage)
    bounds = [oracle_lib.gershgorin(B) for B in mats]
    a = [x[0] for x in bounds]
    b = [x[1] for x in bounds]
    ns = [B.meta["n"] for B in mats]
    M, seed = 32, 77
    D = [dev(B) for B in mats]
    say(f"batched {storage} count={len(mats)} plain={plain}")
    res = ld.ld_logdet_cheb_batched(D, a, b, ns, M, seed, plain=plain)
    for i, B in enumerate(mats):
        o = oracle_lib.logdet(B, a[i], b[i], ns[i], M, seed=seed + i)
        assert rel(res[i]["logdet"], o["gamma"], floor_for(a[i], b[i], ns[i], B.d, tol, U64 if tol < 1e-6 else U32)) <= tol, (i, res[i]["logdet"], o["gamma"])
        assert rel(res[i]["std_err"], o["std_err"]) <= max(1e-3, 100 * tol)
    # second call hits the cached graph and reproduces the result bit for bit
    say("batched replay")
    res2 = ld.ld_logdet_cheb_batched(D, a, b, ns, M, seed, plain=plain)
    assert [r["logdet"] for r in res2] == [r["logdet"] for r in res]


def test_batched_matches_single_calls(ld, oracle_lib):
    mats = _batch(5, "f32", seed0=900)
    ab = [oracle_lib.gershgorin(B) for B in mats]
    ns = [B.meta["n"] for B in mats]
    D = [dev(B) for B in mats]
    say("batched vs single")
    res = ld.ld_logdet_cheb_batched(D, [x[0] for x in ab], [x[1] for x in ab], ns, 16, 4, tile=64)
    for i in range(len(mats)):
        r = ld.ld_logdet_cheb(D[i], ab[i][0], ab[i][1], ns[i], 16, 4 + i, tile=64)
        assert rel(res[i]["logdet"], r["logdet"], floor_for(*ab[i], ns[i], mats[i].d, 1e-12)) <= 1e-12


def test_batched_new_bounds_new_graph(ld, oracle_lib):
    mats = _batch(3, "f64", seed0=50)
    ab = [oracle_lib.gershgorin(B) for B in mats]
    ns = [B.meta["n"] for B in mats]
    D = [dev(B) for B in mats]
    a = [x[0] * 0.9 for x in ab]
    b = [x[1] * 1.1 for x in ab]
    say("batched new bounds")
    res = ld.ld_logdet_cheb_batched(D, a, b, ns, 8, 1)
    for i, B in enumerate(mats):
        o = oracle_lib.logdet(B, a[i], b[i], ns[i], 8, seed=1 + i)
        assert rel(res[i]["logdet"], o["gamma"], floor_for(a[i], b[i], ns[i], B.d, 1e-10)) <= 1e-10
    ld.ld_clear_cache()


def test_batched_rejects_mixed_dtypes(ld):
    import torch

    m1 = dev(synth.random_sparse_spd(100, 2, 1, 1.0, "f32"))
    m2 = dev(synth.random_sparse_spd(100, 2, 2, 1.0, "f64"))
    with pytest.raises(ld.LogdetChebError):
        ld.ld_logdet_cheb_batched([m1, m2], [0.1, 0.1], [10.0, 10.0], [5, 5], 4, 0)
    assert torch.cuda.is_available()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_gershgorin_batched_bit_exact(ld, oracle_lib, storage):
    """One pass over a batch (members split into several work items, shifts included) gives the
    single-matrix and the oracle's Gershgorin intervals bit for bit."""
    mats = _batch(12, storage, d_max=20_000, seed0=410) + [synth.grid_laplacian_2d(90, storage)]
    shifts = [0.0] * 12 + [0.25]
    D = [dev(B, shift=s) for B, s in zip(mats, shifts)]
    say(f"batched gershgorin {storage}")
    a, b = ld.ld_gershgorin_batched(D)
    for i, B in enumerate(mats):
        assert (a[i], b[i]) == ld.ld_gershgorin(D[i])
        assert (a[i], b[i]) == oracle_lib.gershgorin(B, shifts[i])


def test_batched_default_bounds_are_gershgorin(ld, oracle_lib):
    mats = _batch(6, "f32", seed0=1200)
    ns = [B.meta["n"] for B in mats]
    D = [dev(B) for B in mats]
    say("batched with default bounds")
    r0 = ld.ld_logdet_cheb_batched(D, None, None, ns, 16, 3)
    ab = [oracle_lib.gershgorin(B) for B in mats]
    r1 = ld.ld_logdet_cheb_batched(D, [x[0] for x in ab], [x[1] for x in ab], ns, 16, 3)
    assert [r["logdet"] for r in r0] == [r["logdet"] for r in r1]


def test_graph_cache_evicts_least_recently_used(ld, oracle_lib):
    """Eleven bound sets pass through the cache of eight captured graphs; every result, also of a
    set whose graph was evicted and is captured again, matches the oracle."""
    mats = _batch(3, "f64", seed0=77)
    ns = [B.meta["n"] for B in mats]
    D = [dev(B) for B in mats]
    ab = [oracle_lib.gershgorin(B) for B in mats]
    ld.ld_clear_cache()
    for k in list(range(11)) + [0]:
        a = [x[0] * (1.0 - 0.01 * k) for x in ab]
        b = [x[1] * (1.0 + 0.01 * k) for x in ab]
        say(f"batched cache round {k}")
        res = ld.ld_logdet_cheb_batched(D, a, b, ns, 4, 2)
        for i, B in enumerate(mats):
            o = oracle_lib.logdet(B, a[i], b[i], ns[i], 4, seed=2 + i)
            assert rel(res[i]["logdet"], o["gamma"], floor_for(a[i], b[i], ns[i], B.d, 1e-10)) <= 1e-10
    ld.ld_clear_cache()


@pytest.mark.parametrize("M", [1, 4, 10, 24, 100, 300])
def test_batched_probe_counts(ld, oracle_lib, M):
    """Probe blocks of one lane, widened blocks (4, 10, 24 run as 8, 16, 32 probes, the extra ones
    dropped), one wide tile and several probe tiles per pass (M = 300)."""
    mats = _batch(4, "f32", d_max=3000, seed0=640)
    ab = [oracle_lib.gershgorin(B) for B in mats]
    ns = [B.meta["n"] for B in mats]
    D = [dev(B) for B in mats]
    say(f"batched M={M}")
    res = ld.ld_logdet_cheb_batched(D, [x[0] for x in ab], [x[1] for x in ab], ns, M, 9)
    for i, B in enumerate(mats):
        o = oracle_lib.logdet(B, ab[i][0], ab[i][1], ns[i], M, seed=9 + i)
        assert rel(res[i]["logdet"], o["gamma"], floor_for(*ab[i], ns[i], B.d, 1e-4, U32)) <= 1e-4, i
        if M > 1:  # one probe has no standard error
            assert rel(res[i]["std_err"], o["std_err"]) <= 1e-3, i


@pytest.mark.parametrize("ns", [[0], [0, 1, 2, 5], [1, 1], [7]])
def test_batched_low_degrees_and_single_member(ld, oracle_lib, ns):
    mats = [synth.random_sparse_spd(200 + 37 * i, 3, 50 + i, 1.0, "f64") for i in range(len(ns))]
    ab = [oracle_lib.gershgorin(B) for B in mats]
    D = [dev(B) for B in mats]
    say(f"batched degrees {ns}")
    res = ld.ld_logdet_cheb_batched(D, [x[0] for x in ab], [x[1] for x in ab], ns, 8, 5)
    for i, B in enumerate(mats):
        o = oracle_lib.logdet(B, ab[i][0], ab[i][1], ns[i], 8, seed=5 + i)
        assert rel(res[i]["logdet"], o["gamma"], floor_for(*ab[i], ns[i], B.d, 1e-10)) <= 1e-10, (i, ns[i])


@pytest.mark.parametrize("autotune", ["1", "0"])
def test_batched_autotuned_graph(ld, oracle_lib, monkeypatch, autotune):
    """A batch of more than 65536 rows in all is captured once per candidate shape and timed;
    whichever graph wins, every member matches the oracle and a replay reproduces it bit for
    bit (LD_AUTOTUNE=0 keeps the default shape)."""
    monkeypatch.setenv("LD_AUTOTUNE", autotune)
    mats = synth.random_batch(12, mseed0=4400, d_min=3000, d_max=20000, n_min=8, n_max=24, storage="f32")
    assert sum(B.d for B in mats) >= 65536
    ab = [oracle_lib.gershgorin(B) for B in mats]
    ns = [B.meta["n"] for B in mats]
    D = [dev(B) for B in mats]
    M, seed = 32, 61
    say(f"batched autotuned graph LD_AUTOTUNE={autotune}")
    ld.ld_clear_cache()
    res = ld.ld_logdet_cheb_batched(D, [x[0] for x in ab], [x[1] for x in ab], ns, M, seed)
    for i in (0, 5, 11):
        o = oracle_lib.logdet(mats[i], ab[i][0], ab[i][1], ns[i], M, seed=seed + i)
        assert rel(res[i]["logdet"], o["gamma"], floor_for(*ab[i], ns[i], mats[i].d, 1e-4, U32)) <= 1e-4
    res2 = ld.ld_logdet_cheb_batched(D, [x[0] for x in ab], [x[1] for x in ab], ns, M, seed)
    assert [r["logdet"] for r in res2] == [r["logdet"] for r in res]
