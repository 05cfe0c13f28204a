"""GPU parity of spanning-tree counting (Section 3.3): the device-built Laplacian minor against
the oracle's, bit for bit, and the log tau estimates against the oracle on the same probes."""
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


def _moved_hub(G, hub):
    """The same graph with the generator's hub (vertex 0) relabelled as `hub`."""
    perm = np.arange(G.d)
    perm[[0, hub]] = perm[[hub, 0]]
    rows = np.repeat(np.arange(G.d), np.diff(G.row_ptr))
    keep = rows < G.col
    return synth.graph_from_edges(G.d, perm[rows[keep]], perm[G.col[keep].astype(np.int64)])


CASES = [("wheel10", lambda: synth.wheel_graph(10), 0), ("hub5000_mid", lambda: _moved_hub(synth.hub_graph(5000, 4, 3), 2500), 2500),
         ("hub3000_last", lambda: _moved_hub(synth.hub_graph(3000, 2, 4), 2999), 2999), ("k2", lambda: synth.complete_graph(2), 1)]


@pytest.mark.parametrize("name,make,hub", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("f64", [False, True])
def test_minor_bit_exact(ld, oracle_lib, name, make, hub, f64):
    import torch

    G = make()
    say(f"laplacian minor {name} hub={hub} f64={f64}")
    Lg, dmax = ld.ld_laplacian_minor(dev(G), hub, torch.float64 if f64 else torch.float32)
    Lo, dmo = oracle_lib.laplacian_minor(G, hub)
    assert dmax == dmo
    assert np.array_equal(Lg.row_ptr.cpu().numpy(), Lo.row_ptr)
    assert np.array_equal(Lg.col.cpu().numpy(), Lo.col)
    assert np.array_equal(Lg.values.double().cpu().numpy(), Lo.val)


def test_minor_rejects_bad_graphs(ld):
    # vertex 0 misses vertex 5: not a hub
    W = synth.wheel_graph(6)
    rows = np.repeat(np.arange(W.d), np.diff(W.row_ptr))
    keep = ~(((rows == 0) & (W.col == 5)) | ((rows == 5) & (W.col == 0)))
    G = synth.graph_from_edges(W.d, rows[keep], W.col[keep].astype(np.int64))
    say("laplacian minor: hub of too small degree")
    with pytest.raises(ld.LogdetChebError, match="not adjacent"):
        ld.ld_laplacian_minor(dev(G), 0)
    # a self loop at vertex 3 in place of its edge to vertex 4 (hub degree still right)
    col = W.col.copy()
    seg = slice(int(W.row_ptr[3]), int(W.row_ptr[4]))
    c3 = col[seg]
    c3[c3 == 4] = 3
    col[seg] = np.sort(c3)
    bad = synth.CSR(W.d, W.row_ptr.copy(), col, W.val.copy(), "f32", {})
    say("laplacian minor: self loop")
    with pytest.raises(ld.LogdetChebError, match="self loop"):
        ld.ld_laplacian_minor(dev(bad), 0)
    say("laplacian minor: hub out of range")
    with pytest.raises(ld.LogdetChebError):
        ld.ld_laplacian_minor(dev(W), W.d)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("f64", [False, True])
def test_log_spanning_trees_parity(ld, oracle_lib, method, f64):
    G = _moved_hub(synth.hub_graph(3000, 3, 8), 1234)
    n, M, seed = 40, 16, 21
    say(f"log spanning trees d=3000 method={method} f64={f64}")
    r = ld.ld_log_spanning_trees(dev(G), 1234, n, M, seed, method=method, vec_f64=f64, want_probes=True)
    o = oracle_lib.log_spanning_trees(G, 1234, n, M, seed=seed, method=method)
    tol = 1e-10 if f64 else 1e-4
    assert rel(r["logdet"], o["gamma"], floor_for(1.0, (2.0 * o["delta_max"] - 1.0) ** (2 if method == 1 else 1), n, G.d, tol, U64 if f64 else U32)) <= tol
    for j in range(M):
        assert rel(r["s"][j], o["s"][j], floor_for(1.0, (2.0 * o["delta_max"] - 1.0) ** (2 if method == 1 else 1), n, G.d, tol, U64 if f64 else U32)) <= tol, j


def test_log_spanning_trees_star_is_zero(ld):
    nv = 9
    G = synth.graph_from_edges(nv, np.zeros(nv - 1, dtype=np.int64), np.arange(1, nv))
    say("log spanning trees: star")
    r = ld.ld_log_spanning_trees(dev(G), 0, 20, 8, 1, want_probes=True)
    assert r["logdet"] == 0.0 and np.all(r["s"] == 0.0)


@pytest.mark.parametrize("method", [0, 1])
def test_log_spanning_trees_wheel_accuracy(ld, method):
    """W_40 at degree 100: the estimate lies within 5 standard errors of log(L_80 - 2)."""
    import math

    a, b = 2, 1
    for _ in range(80):
        a, b = b, a + b
    say(f"log spanning trees: wheel 40 method={method}")
    r = ld.ld_log_spanning_trees(dev(synth.wheel_graph(40)), 0, 100, 512, 3, method=method, vec_f64=True)
    assert abs(r["logdet"] - math.log(a - 2)) < 5 * r["std_err"] + 1e-9
