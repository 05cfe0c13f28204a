"""Benchmark of the stochastic Chebyshev log-determinant hot path on one MI355X.

A step is one pass of the whole path over the workload with inputs resident in HBM: the
spectral interval (given, or Gershgorin bounds on the device), then the forward estimate and
its gradient on the sparsity pattern (ld_logdet_cheb_grad: forward recurrence with
checkpoints, adjoint recurrence fused with the SDDMM).

Default workload: the 2-D Dirichlet grid Laplacian 4096 x 4096 (d = 16,777,216, 83,869,696
stored entries) + 0.01 I, values stored in BF16 (exact) with the 0.01 shift kept in FP64, FP32
recurrence, M = 32 probes, degree n = 100, bounds [0.01, 8.01]: the largest configuration,
in the paper's tens-of-millions regime (Section 5.1).

`value` counts the sparse matrix-vector nonzeros of the products the method executes per
second of fwd+grad time: M * nnz per product, ceil(n/2) forward products (Chebyshev product
identities) plus ceil(n/2) - 1 adjoint products, recomputation from checkpoints excluded.
The count with the paper's n products per logdet is reported beside it.

Prints ONE JSON line.  Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
METRIC = "logdet fwd+grad matvec-nnz/s and HBM GB/s vs peak, at stated rel. error"
KERNEL_SRC = os.path.join(ROOT, "paper_1503_06394_amd", "csrc", "ld_kernels.hip")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------

def workload(name: str):
    import synth

    if name == "random1m":
        B = synth.random_sparse_spd(1_000_000, k_off=5, mseed=2, diag_add=1.0, storage="f32")
        return dict(B=B, shift=0.0, a=None, b=None, n=50, M=64, seed=2, grad=True,
                    desc="random sparse SPD d=1e6, ~11 nnz/row, U[-1,1] offdiag, diag=sum|off|+1, FP32, "
                         "M=64, n=50, Gershgorin bounds")
    if name == "grid32":
        B = synth.grid_laplacian_2d(32, "f64")
        return dict(B=B, shift=0.1, a=0.1, b=8.1, n=30, M=50, seed=1, grad=True,
                    desc="2D Dirichlet grid 32x32 + 0.1 I, FP64, M=50, n=30")
    if name == "gmrf128":
        B = synth.grid_laplacian_3d(128, "f32")
        kappa = 0.3
        return dict(B=B, shift=kappa ** 2, a=kappa ** 2, b=kappa ** 2 + 12.0, n=60, M=32, seed=3, grad=True,
                    desc="3D GMRF Q=tau(kappa^2 I+L) 128^3, tau=1, kappa=0.3, FP32, M=32, n=60")
    if name == "nonsingular1m":
        C = synth.random_nonsingular(1_000_000, per_row=8, mseed=6, diag_add=3.0, storage="f32")
        return dict(B=C, shift=0.0, a=None, b=None, n=100, M=32, seed=6, grad=False, nonsingular=True,
                    desc="general sparse d=1e6, 8 N(0,1) entries per row + 3 I, FP32, Algorithm 2 "
                         "(log|det C| = 1/2 log det C^T C), M=32, n=100, sigma bounds from a 300-step "
                         "Lanczos estimate on C^T C (smin^2 = 0.5 x lowest Ritz value, smax = 1.05 x sqrt(highest))")
    if name == "batch256":
        mats = synth.random_batch(256, mseed0=1000)
        return dict(B=None, mats=mats, shift=0.0, a=None, b=None, n=None, M=32, seed=4, grad=False,
                    desc="batch of 256 random sparse SPD matrices, d log-uniform in [1e3, 2e5], 5-20 nnz/row, "
                         "own Gershgorin bounds, n in [20, 80], M=32, FP32, one captured graph")
    if name == "gmrf5000":
        return dict(B=None, N=5000, rho0=-0.22, rhos=[round(-0.24 + 0.005 * i, 4) for i in range(9)], n=40, M=32, seed=2,
                    grad=False, desc="grid GMRF 5000x5000 (d=25M), J(rho) = I - rho A, FP32, exact draw at "
                                     "rho=-0.22; log-likelihood at 9 values of rho in [-0.24, -0.20], "
                                     "Algorithm 1 with Gershgorin bounds, M=32, n=40")
    if name == "sec51_3e7":
        return dict(B=None, d=30_000_000, n=15, M=10, seed=11, grad=False,
                    desc="Section 5.1's largest run: random symmetric C, d=3e7, 5 off-diagonals per row U[-1,1] "
                         "mirrored, diagonal = sum|off| + 1e-3 (about 3.3e8 nnz), FP32; Algorithm 2 with m=10, "
                         "n=15, sigma_min=1e-3, sigma_max=||C||_1")
    if name == "trees1m":
        return dict(B=None, nv=1_000_000, k_off=5, mseed=7, n=100, M=32, seed=8, grad=False,
                    desc="spanning trees of a hub graph with 1e6 vertices (vertex 0 joined to all, 5 random "
                         "neighbours drawn per vertex, edges mirrored): Laplacian minor L(hub) on the device, then "
                         "Algorithm 2 with sigma in [1, 2 Delta_max - 1] (Section 3.3), FP32, M=32, n=100")
    if name == "taylor4096":
        B = synth.grid_laplacian_2d(4096, "bf16")
        return dict(B=B, shift=0.01, a=0.01, b=8.01, n=100, M=32, seed=5, grad=False,
                    desc="Taylor-series comparator of Section 5.1 on the 2D Dirichlet grid 4096x4096 + 0.01 I "
                         "(BF16 values, FP32 vectors, M=32, n=100), beside the Chebyshev estimate with the same "
                         "probes; both against the closed-form log det")
    if name == "lanczos1m":
        B = synth.random_sparse_spd(1_000_000, k_off=5, mseed=2, diag_add=1.0, storage="f32")
        return dict(B=B, iters=300, seed=2, grad=False,
                    desc="spectral estimate (Section 3.2's bounds): 300 FP64 Lanczos steps on the random d=1e6 "
                         "matrix of the main workload, extreme Ritz values")
    if name == "grid4096":
        B = synth.grid_laplacian_2d(4096, "bf16")
        return dict(B=B, shift=0.01, a=0.01, b=8.01, n=100, M=32, seed=5, grad=True,
                    desc="2D Dirichlet grid 4096x4096 (d=16.8M) + 0.01 I, BF16 values (shift 0.01 in FP64), "
                         "FP32 recurrence, M=32, n=100, bounds [0.01, 8.01]: fwd+grad")
    raise SystemExit(f"unknown workload {name}")


# ----------------------------------------------------------------------------------------
# algorithmic bytes of the dominant kernels (per launch)
# ----------------------------------------------------------------------------------------

def csr_bytes(d: int, nnz: int, val_bytes: int) -> int:
    """The CSR matrix once: values, int32 columns and 4-byte row pointers (the compulsory-bytes count;
    the library's int64 row pointers add (d + 1) * 4 bytes, reported in `moved_bytes_per_launch`)."""
    return nnz * (val_bytes + 4) + (d + 1) * 4


def step_bytes(d: int, nnz: int, M: int, val_bytes: int, vec_bytes: int) -> int:
    """Algorithmic bytes of one recurrence step: the CSR matrix once, W_k read once, W_{k-1} read,
    W_{k+1} written.  Algorithm 2 splits a degree into T = C W_k (C, W_k gathered, T written) and
    W_{k+1} = alpha C^T T + beta W_k - W_{k-1} (C^T, T gathered, W_k and W_{k-1} read, W_{k+1}
    written): 2 + 4 vectors over two launches, the same three per launch on average."""
    return csr_bytes(d, nnz, val_bytes) + 3 * d * M * vec_bytes


def adjoint_bytes(d: int, nnz: int, M: int, val_bytes: int, vec_bytes: int, acc_bytes: int) -> int:
    """Algorithmic bytes of one adjoint step, the method's own work: the SpMM y_j = c_j v + 2 At y_{j+1}
    - y_{j+2} (the CSR matrix, y_{j+1} read once, y_{j+2} read, y_j written), w_j read once for the
    SDDMM, and the gradient accumulators read and written (2 * acc_bytes per stored entry)."""
    return csr_bytes(d, nnz, val_bytes) + 4 * d * M * vec_bytes + 2 * nnz * acc_bytes


def adjoint_moved_bytes(d: int, nnz: int, M: int, val_bytes: int, vec_bytes: int, acc_bytes: int,
                        form: str | None) -> int:
    """What the adjoint kernel moves, by the form that ran: the explicit seed of the product-identity
    form reads w_{j-1} and w_{j+1} as well (and int64 row pointers); the shifted form on staged
    stencil tiles reads four vector blocks and, in place of the CSR matrix, one packed entry (slot and
    value: 4 bytes for BF16 values, 8 for FP32) per stored entry, plus its accumulators (padding slots
    of the layout, under 0.3 % of the entries on the grids, not counted)."""
    alg = adjoint_bytes(d, nnz, M, val_bytes, vec_bytes, acc_bytes)
    if form == "shifted_staged":
        ent = {2: 4, 4: 8, 8: 16}[val_bytes]
        return alg - csr_bytes(d, nnz, val_bytes) + nnz * ent
    extra = 2 * d * M * vec_bytes if form in ("explicit_single", "explicit_two") else 0
    return alg + extra + (d + 1) * 4


def traffic_from_profiles(kernel_tag: str, workload_name: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when absent or
    when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{kernel_tag}_{workload_name}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t:
        return None
    cur = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if cur != m.group(1):
        return None
    return float(t.group(1))


# ----------------------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample
# ----------------------------------------------------------------------------------------

def host_cpu() -> dict:
    """The host CPU: model name and clock (/proc/cpuinfo, cpufreq), logical CPUs on the machine and
    the CPUs this process may run on."""
    model, mhz = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except (OSError, ValueError):
        pass
    max_mhz = None
    try:
        with open("/sys/devices/system/cpu/cpu0/cpufreq/cpuinfo_max_freq") as f:
            max_mhz = int(f.read().strip()) / 1000.0
    except (OSError, ValueError):
        pass
    return {"model": model, "mhz_now": mhz, "mhz_max": max_mhz, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(W: dict, a: float, b: float, gpu_probe_values) -> tuple:
    """The oracle as it stands, single-threaded FP64 C, on a bounded sample of the workload: whole
    probes on the full matrix, one at a time, until about 12 s of work.  The oracle's gradient keeps
    every w_k and y_k (2n + 3 vectors of d doubles), so at large d the sample runs at a reduced
    degree (at most 4 GB of vectors); the rate is per executed sparse product, the unit of `value`
    (the oracle applies B once per degree forward and once per degree backward)."""
    import numpy as np

    import oracle

    oracle.build()
    B, n, M = W["B"], W["n"], W["M"]
    ns = n
    if W["grad"]:
        ns = max(2, min(n, int(4e9 / (16.0 * (B.d + 1)) - 2)))
    secs, done = 0.0, 0
    while done < M and (secs < 12.0 or done == 0):
        t0 = time.perf_counter()
        if W.get("nonsingular"):
            oracle.logabsdet(B, a, b, ns, 1, seed=W["seed"], ids=np.array([done]))
        elif W["grad"]:
            oracle.logdet_grad(B, a, b, ns, 1, seed=W["seed"], ids=np.array([done]), shift=W["shift"])
        else:
            oracle.logdet(B, a, b, ns, 1, seed=W["seed"], ids=np.array([done]), shift=W["shift"])
        secs += time.perf_counter() - t0
        done += 1
    products = (2 * ns - 1) if W["grad"] else ns * (2 if W.get("nonsingular") else 1)
    kind = "fwd+grad" if W["grad"] else "fwd"
    base = {"value": done * products * B.nnz / secs, "unit": "matvec-nnz/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(),
            "sample": f"{kind} of probes 0..{done - 1} of {M} on the full matrix at degree {ns} (workload degree "
                      f"{n}), single-threaded FP64 C oracle, {secs:.1f} s; {products} sparse products per probe"}
    parity = None
    if gpu_probe_values is not None:
        t0 = time.perf_counter()
        if W.get("nonsingular"):
            r = oracle.logabsdet(B, a, b, n, 1, seed=W["seed"], ids=np.array([0]))
        else:
            r = oracle.logdet(B, a, b, n, 1, seed=W["seed"], ids=np.array([0]), shift=W["shift"])
        log(f"oracle probe 0 at degree {n}: {time.perf_counter() - t0:.1f} s")
        ref = float(r["s"][0])
        parity = abs(float(gpu_probe_values[0]) - ref) / abs(ref)
    return base, parity


# ----------------------------------------------------------------------------------------
# main
# ----------------------------------------------------------------------------------------

def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid4096",
                    choices=["random1m", "grid32", "gmrf128", "grid4096", "batch256", "nonsingular1m", "gmrf5000",
                             "trees1m", "taylor4096", "lanczos1m",
                             "sec51_3e7"])
    ap.add_argument("--compare-perprobe", action="store_true",
                    help="also time the plain per-probe forms (one probe per call, one product per degree, "
                         "FP64 and FP32) and the block form with the plain recurrence")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fwd-only", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=2 << 30,
                    help="first run the library's streaming copy kernel on this many bytes (what a streaming "
                         "kernel reaches on this GPU; 0 skips it)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (probes would shard "
              "across GPUs with one all-reduce of the moment table).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1503_06394_amd as ld

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    copy_gbps = None
    if args.copy_bytes:
        src = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        src.fill_(1)
        ts = [ld.ld_copy(dst, src) for _ in range(4)]
        copy_gbps = 2 * args.copy_bytes / (min(ts[1:]) / 1e3) / 1e9
        log(f"copy kernel: {args.copy_bytes} bytes, best {min(ts[1:]):.4f} ms, {copy_gbps:.1f} GB/s (read+write)")
        del src, dst
    log(f"building workload {args.workload}")
    W = workload(args.workload)
    if args.workload == "batch256":
        return bench_batch(args, W, copy_gbps)
    if args.workload == "gmrf5000":
        return bench_gmrf(args, W, copy_gbps)
    if args.workload == "sec51_3e7":
        return bench_sec51(args, W, copy_gbps)
    if args.workload == "trees1m":
        return bench_trees(args, W, copy_gbps)
    if args.workload == "taylor4096":
        return bench_taylor(args, W, copy_gbps)
    if args.workload == "lanczos1m":
        return bench_lanczos(args, W, copy_gbps)
    B = W["B"]
    d, nnz, M, n = B.d, B.nnz, W["M"], W["n"]
    D = ld.DeviceCSR.from_host(B, device="cuda:0", diag_shift=W["shift"])
    vec_f64 = B.storage == "f64"
    val_bytes = {"f64": 8, "f32": 4, "bf16": 2}[B.storage]
    vec_bytes = 8 if vec_f64 else 4
    do_grad = W["grad"] and not args.fwd_only
    log(f"d={d} nnz={nnz} M={M} n={n} storage={B.storage} grad={do_grad}")

    ws_fwd = torch.empty(ld.ld_workspace_bytes(D, n, M, 1 if W.get("nonsingular") else 0), dtype=torch.uint8,
                         device="cuda:0")
    ws_grad = torch.empty(ld.ld_workspace_bytes(D, n, M, 2), dtype=torch.uint8, device="cuda:0") if do_grad else None
    gdt = torch.float64 if vec_f64 else torch.float32

    nonsingular = W.get("nonsingular", False)
    if nonsingular:
        # estimated once per matrix, outside the timed region (the same for every evaluation)
        lo, hi = ld.ld_spectral_estimate(D, iters=300, gram=True, seed=W["seed"])
        W["a"], W["b"] = (0.5 * lo) ** 0.5, 1.05 * hi ** 0.5
        log(f"sigma bounds from Lanczos: smin={W['a']:.5g} smax={W['b']:.5g}")

    def bounds():
        if W["a"] is not None:
            return W["a"], W["b"]
        return ld.ld_gershgorin(D)

    def one_step(timing: bool):
        a, b = bounds()
        if nonsingular:
            return ld.ld_logabsdet_cheb(D, None, a, b, n, M, W["seed"], workspace=ws_fwd, timing=timing)
        if do_grad:
            r, g = ld.ld_logdet_cheb_grad(D, a, b, n, M, W["seed"], 1.0, grad_dtype=gdt, workspace=ws_grad,
                                          timing=timing)
            return r
        return ld.ld_logdet_cheb(D, a, b, n, M, W["seed"], workspace=ws_fwd, timing=timing)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps")
    step_ms = adj_ms = 0.0
    step_n = adj_n = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = one_step(True)
        step_ms += r["kernel_ms"]
        step_n += r["kernel_launches"]
        adj_ms += r["adjoint_ms"]
        adj_n += r["adjoint_launches"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # sparse products of the method per step: ceil(n/2) forward products with the product identities
    # (Algorithm 2: two per step, C and C^T), plus ceil(n/2) - 1 adjoint products with the gradient
    m_fwd = (n + 1) // 2
    products = m_fwd * (2 if nonsingular else 1) + (max(m_fwd - 1, 0) if do_grad else 0)
    value = M * nnz * products / (ms_per_step / 1e3)
    work = M * n * nnz * (2 if nonsingular else 1)  # the paper's count: n products per logdet

    # forward-only throughput on the same inputs (context)
    a, b = bounds()
    fwd_ms = None
    if do_grad:
        for _ in range(2):
            ld.ld_logdet_cheb(D, a, b, n, M, W["seed"], workspace=ws_fwd)
        torch.cuda.synchronize()
        tf0 = time.perf_counter()
        kf = max(3, args.steps)
        for _ in range(kf):
            rf = ld.ld_logdet_cheb(D, a, b, n, M, W["seed"], workspace=ws_fwd)
        torch.cuda.synchronize()
        fwd_ms = (time.perf_counter() - tf0) * 1e3 / kf
    if nonsingular:
        rp = ld.ld_logabsdet_cheb(D, None, a, b, n, M, W["seed"], workspace=ws_fwd, want_probes=True)
    else:
        rp = ld.ld_logdet_cheb(D, a, b, n, M, W["seed"], workspace=ws_fwd, want_probes=True)

    # dominant kernel: the larger of the summed step and adjoint kernel times
    sb = step_bytes(d, nnz, M, val_bytes, vec_bytes)
    ab_ = adjoint_bytes(d, nnz, M, val_bytes, vec_bytes, vec_bytes)
    if adj_ms > step_ms and adj_n > 0:
        tag, avg_ms, bytes_ = "adjoint", adj_ms / adj_n, ab_
        moved = adjoint_moved_bytes(d, nnz, M, val_bytes, vec_bytes, vec_bytes, r.get("adjoint_form"))
    else:
        tag, avg_ms, bytes_ = "step", step_ms / max(step_n, 1), sb
        moved = sb + (d + 1) * 4
    achieved = bytes_ / (avg_ms / 1e3) / 1e9
    traffic = traffic_from_profiles(tag, args.workload)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic, "kernel": f"{tag} kernel",
            "avg_launch_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": bytes_,
            "moved_bytes_per_launch": moved, "moved_GBps": round(moved / (avg_ms / 1e3) / 1e9, 1)}
    if tag == "adjoint":
        roof["adjoint_form"] = r.get("adjoint_form")
        roof["kernel"] = {"shifted_staged": "adjoint_stencil_kernel (shifted adjoint, LDS-staged stencil tiles)",
                          "explicit_single": "adjoint_kernel (explicit seed, single gather)"}.get(
                              r.get("adjoint_form"), "adjoint kernel")
    if traffic is not None:
        roof["traffic_GBps"] = round(traffic / (avg_ms / 1e3) / 1e9, 1)  # counted bytes at the live launch time
        roof["traffic_over_algorithmic"] = round(traffic / bytes_, 3)
    extra = {
        "step_kernel": {"avg_ms": round(step_ms / max(step_n, 1), 5), "launches_per_step": step_n // args.steps,
                        "algorithmic_GBps": round(sb / (step_ms / max(step_n, 1) / 1e3) / 1e9, 1)},
    }
    if adj_n:
        extra["adjoint_kernel"] = {"avg_ms": round(adj_ms / adj_n, 5), "launches_per_step": adj_n // args.steps,
                                   "algorithmic_GBps": round(ab_ / (adj_ms / adj_n / 1e3) / 1e9, 1)}
    if fwd_ms is not None:
        extra["forward_only"] = {"ms": round(fwd_ms, 3),
                                 "matvec_nnz_per_s": M * nnz * m_fwd * (2 if nonsingular else 1) / (fwd_ms / 1e3)}
    extra["paper_equivalent_matvec_nnz_per_s"] = work / (ms_per_step / 1e3)
    extra["products_per_step"] = products
    # sparse products the kernels actually executed (product identities: ceil(n/2) per forward; every
    # timed adjoint step runs the SpMM and the SDDMM, and each call closes with one more SDDMM),
    # per second of step time
    executed = nnz * M * (step_n + (2 * adj_n + args.steps if adj_n else 0))
    extra["executed_spmm_sddmm_nnz_ops_per_s"] = executed / args.steps / (ms_per_step / 1e3)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one probe)")
        cpu, parity = cpu_baseline(W, a, b, rp["s"])
    accuracy = {"logdet": r["logdet"], "std_err_rel": abs(r["std_err"] / r["logdet"]),
                "lemma7_bound_rel": abs(r["poly_bound"] / r["logdet"]),
                "oracle_parity_rel_probe0": parity, "parity_tolerance": 1e-10 if vec_f64 else 1e-4}

    out = {
        "metric": METRIC, "value": value, "unit": "matvec-nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if vec_f64 else "f32", "data": "synthetic",
        "config": {"workload": W["desc"], "d": d, "nnz": nnz, "M": M, "n": n, "values": B.storage,
                   "step": ("Algorithm 2 forward (sigma bounds estimated once, before timing)" if nonsingular
                            else ("gershgorin bounds + " if W["a"] is None else "")
                            + ("forward + gradient" if do_grad else "forward")),
                   "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu, "accuracy": accuracy, "kernels": extra,
    }
    if copy_gbps is not None:
        out["copy_kernel_GBps"] = round(copy_gbps, 1)
        out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / copy_gbps, 4)
    if args.compare_perprobe:
        log("plain per-probe forms and the plain block form")
        out["perprobe_fp64"] = perprobe([B], [a], [b], [n], M, W["seed"], W["shift"], "f64")
        out["perprobe_fp32"] = perprobe([B], [a], [b], [n], M, W["seed"], W["shift"], "f32")
        out["block_plain_forward_ms"] = block_plain_ms(D, a, b, n, M, W["seed"])
    print(json.dumps(out), flush=True)


def perprobe(mats, a, b, ns, M, seed, shift=0.0, dtype="f64") -> dict:
    """The plain per-probe form as Algorithm 1 states it: every probe is its own call with M = 1 and
    one sparse matrix-vector product per degree (plain recurrence), values and vectors in `dtype`.
    Probe j of matrix i uses seed (seed + i) * 100003 + j, so the estimator is statistically the
    same as the block form."""
    import numpy as np
    import torch

    import paper_1503_06394_amd as ld

    tdt = torch.float64 if dtype == "f64" else torch.float32
    devs = [ld.DeviceCSR.from_host(B, device="cuda:0", dtype=tdt, diag_shift=shift) for B in mats]
    ld.ld_logdet_cheb(devs[0], a[0], b[0], ns[0], 1, 0, plain=True)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est = []
    for i, D in enumerate(devs):
        s = [ld.ld_logdet_cheb(D, a[i], b[i], ns[i], 1, (seed + i) * 100003 + j, plain=True)["logdet"]
             for j in range(M)]
        est.append((float(np.mean(s)), float(np.std(s, ddof=1) / np.sqrt(M))))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    work = sum(M * ns[i] * mats[i].nnz for i in range(len(mats)))
    return {"ms": round(ms, 3), "matvec_nnz_per_s": work / (ms / 1e3),
            "std_err_rel_first": abs(est[0][1] / est[0][0]), "logdet_first": est[0][0]}


def block_plain_ms(D, a, b, n, M, seed, reps=3) -> float:
    """The block form with the plain recurrence (n products instead of ceil(n/2))."""
    import torch

    import paper_1503_06394_amd as ld

    ld.ld_logdet_cheb(D, a, b, n, M, seed, plain=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ld.ld_logdet_cheb(D, a, b, n, M, seed, plain=True)
    torch.cuda.synchronize()
    return round((time.perf_counter() - t0) * 1e3 / reps, 3)


def bench_batch(args, W, copy_gbps) -> None:
    import numpy as np
    import torch

    import paper_1503_06394_amd as ld

    mats, M, seed = W["mats"], W["M"], W["seed"]
    D = [ld.DeviceCSR.from_host(B, device="cuda:0") for B in mats]
    a, b = ld.ld_gershgorin_batched(D)
    ns = [B.meta["n"] for B in mats]
    work = sum(M * ns[i] * mats[i].nnz for i in range(len(mats)))
    log(f"batch: {len(mats)} matrices, sum d={sum(B.d for B in mats)}, sum nnz={sum(B.nnz for B in mats)}")
    for _ in range(max(1, args.warmup)):
        ld.ld_logdet_cheb_batched(D, a, b, ns, M, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gms = 0.0
    for _ in range(args.steps):
        ga, gb = ld.ld_gershgorin_batched(D)
        res = ld.ld_logdet_cheb_batched(D, ga, gb, ns, M, seed, timing=True)
        gms += res[0]["kernel_ms"]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    gms /= args.steps
    vec_bytes = 4
    steps = [(x + 1) // 2 for x in ns]  # product identities: ceil(n/2) sparse products per member
    alg = sum(steps[i] * (mats[i].nnz * 8 + (mats[i].d + 1) * 8 + 3 * mats[i].d * M * vec_bytes)
              for i in range(len(mats)))
    achieved = alg / (gms / 1e3) / 1e9
    traffic = traffic_from_profiles("step", args.workload)  # counted bytes of one whole graph replay
    cpu = None
    if not args.no_cpu_baseline:
        order = np.argsort([B.d for B in mats])
        i = int(order[len(order) // 2])
        import oracle

        oracle.build()
        t1 = time.perf_counter()
        o = oracle.logdet(mats[i], a[i], b[i], ns[i], M, seed=seed + i)
        secs = time.perf_counter() - t1
        cpu = {"value": M * ns[i] * mats[i].nnz / secs, "unit": "matvec-nnz/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"member {i} of the batch (d={mats[i].d}, n={ns[i]}, {M} probes), single-threaded FP64 "
                         f"C oracle, {secs:.1f} s"}
        parity = abs(res[i]["logdet"] - o["gamma"]) / max(abs(o["gamma"]), 1e-3 * mats[i].d)
    else:
        parity = None
    out = {
        "metric": METRIC, "value": work / (ms / 1e3), "unit": "matvec-nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": W["desc"], "count": len(mats), "sum_d": sum(B.d for B in mats),
                   "sum_nnz": sum(B.nnz for B in mats), "M": M, "step": "gershgorin bounds + batched forward graph",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic, "kernel": "batched graph",
                     "graph_ms": round(gms, 4), "algorithmic_bytes_per_launch": alg},
        "cpu_baseline": cpu,
        "accuracy": {"oracle_parity_rel_median_member": parity, "parity_tolerance": 1e-4,
                     "std_err_rel_first": abs(res[0]["std_err"] / res[0]["logdet"])},
    }
    if traffic is not None:
        out["roofline"]["traffic_over_algorithmic"] = round(traffic / alg, 3)
    if copy_gbps is not None:
        out["copy_kernel_GBps"] = round(copy_gbps, 1)
        out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / copy_gbps, 4)
    if args.compare_perprobe:
        log("plain per-probe FP64 form")
        out["perprobe_fp64"] = perprobe(mats, a, b, ns, M, seed, 0.0, "f64")
    print(json.dumps(out), flush=True)


def bench_gmrf(args, W, copy_gbps) -> None:
    """Log-likelihood curve of the 5000 x 5000 grid GMRF (Section 5.2): one step evaluates
    l(rho) = log det J(rho)/2 - x^T J(rho) x/2 at every rho of the sweep."""
    import numpy as np
    import torch

    import paper_1503_06394_amd as ld
    import synth
    from paper_1503_06394_amd.gmrf import GMRF

    N, n, M, seed, rhos = W["N"], W["n"], W["M"], W["seed"], W["rhos"]
    L = synth.grid_laplacian_2d(N, "f32")
    log("drawing the sample")
    x = synth.gmrf_sample(N, W["rho0"], seed=1)
    D = ld.DeviceCSR.from_host(L, device="cuda:0")
    g = GMRF(D.row_ptr, D.col)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda:0")
    d, nnz = L.d, L.nnz
    ws = torch.empty(ld.ld_workspace_bytes(g.precision(rhos[0]), n, M, 0), dtype=torch.uint8, device="cuda:0")

    def sweep(timing):
        out, kms, kn = [], 0.0, 0
        for rho in rhos:
            a, b = g.bounds(rho)
            J = g.precision(rho)
            r = ld.ld_logdet_cheb(J, a, b, n, M, seed, workspace=ws, timing=timing)
            q = ld.ld_quadratic_form(J, xt)
            out.append((rho, r["logdet"], q, 0.5 * r["logdet"] - 0.5 * q))
            kms += r["kernel_ms"]
            kn += r["kernel_launches"]
        return out, kms, kn

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        sweep(False)
    torch.cuda.synchronize()
    log(f"timing {args.steps} sweeps of {len(rhos)} values")
    kms = kn = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        curve, k1, k2 = sweep(True)
        kms += k1
        kn += k2
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    work = len(rhos) * M * n * nnz
    sb = step_bytes(d, nnz, M, 4, 4)
    avg = kms / max(kn, 1)
    achieved = sb / (avg / 1e3) / 1e9
    # accuracy against the closed-form spectrum of the grid
    t = np.pi * np.arange(1, N + 1) / (N + 1)
    lam = (2.0 * np.cos(t)[:, None] + 2.0 * np.cos(t)[None, :]).ravel()
    rows = L.row_of_entry()
    off = L.col != rows
    xax = float(np.sum(x[rows[off]] * x[L.col[off].astype(np.int64)]))
    xx = float(x @ x)
    exact_ld = [float(np.log1p(-r * lam).sum()) for r in rhos]
    exact = [0.5 * ld_ - 0.5 * (xx - r * xax) for r, ld_ in zip(rhos, exact_ld)]
    est_rho = max(curve, key=lambda c: c[3])[0]
    exact_rho = rhos[int(np.argmax(exact))]
    logdet_err = max(abs(c[1] - ld_) / abs(ld_) for c, ld_ in zip(curve, exact_ld))
    cpu = parity = None
    if not args.no_cpu_baseline:
        deg = 80  # about 10 s of oracle work on one core
        log(f"cpu baseline (oracle, probe 0 at degree {deg})")
        Jh = synth.gmrf_grid_precision(N, W["rho0"], "f32")
        a, b = g.bounds(W["rho0"])
        rg = ld.ld_logdet_cheb(g.precision(W["rho0"]), a, b, deg, M, seed, want_probes=True)
        import oracle

        oracle.build()
        t1 = time.perf_counter()
        o = oracle.logdet(Jh, a, b, deg, 1, seed=seed, ids=np.array([0]))
        secs = time.perf_counter() - t1
        cpu = {"value": deg * Jh.nnz / secs, "unit": "matvec-nnz/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"probe 0 at degree {deg} of J(-0.22) on the full grid, single-threaded FP64 C oracle, "
                         f"{secs:.1f} s"}
        parity = abs(rg["s"][0] - o["s"][0]) / max(abs(o["s"][0]), 1e-3 * d)
    out = {
        "metric": METRIC, "value": work / (ms / 1e3), "unit": "matvec-nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": W["desc"], "d": d, "nnz": nnz, "M": M, "n": n, "points": len(rhos),
                   "step": "log-likelihood at every rho of the sweep", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": "step kernel",
                     "avg_launch_ms": round(avg, 5), "algorithmic_bytes_per_launch": sb},
        "cpu_baseline": cpu,
        "accuracy": {"argmax_rho_estimated": est_rho, "argmax_rho_exact": exact_rho, "hidden_rho": W["rho0"],
                     "max_logdet_rel_err_vs_closed_form": logdet_err, "oracle_parity_rel_probe0_deg80": parity,
                     "parity_tolerance": 1e-4},
        "curve": [{"rho": c[0], "loglik": c[3]} for c in curve],
    }
    if copy_gbps is not None:
        out["copy_kernel_GBps"] = round(copy_gbps, 1)
        out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / copy_gbps, 4)
    print(json.dumps(out), flush=True)


# the paper's figure for this run: 500 s for m=10, n=15, Algorithm 2 (C and C^T per degree) on its
# 3e8 stored entries, i.e. 10 * 15 * 2 * 3e8 / 500 matvec-nnz/s on one CPU
SEC51_PAPER_RATE = 10 * 15 * 2 * 3e8 / 500.0


def bench_sec51(args, W, copy_gbps) -> None:
    """Replay of Section 5.1's largest timing point on one GPU: Algorithm 2 on a d = 3e7 random
    symmetric matrix.  C^T and the bounds are prepared once, outside the timed region."""
    import numpy as np
    import torch

    import paper_1503_06394_amd as ld
    import synth

    d, n, M, seed = W["d"], W["n"], W["M"], W["seed"]
    log("generating the matrix (about 1.5 minutes on the host)")
    C = synth.random_sparse_spd(d, 5, seed, 1e-3, "f32")
    nnz = C.nnz
    log(f"d={d} nnz={nnz}; uploading")
    D = ld.DeviceCSR.from_host(C, device="cuda:0")
    Ct = ld.ld_transpose(D)
    smin = 1e-3
    smax = ld.ld_gershgorin(D)[1]  # = ||C||_1: the diagonal is the absolute off-diagonal row sum plus 1e-3
    ws = torch.empty(ld.ld_workspace_bytes(D, n, M, 1), dtype=torch.uint8, device="cuda:0")
    log(f"sigma in [{smin}, {smax:.4g}]; warmup {args.warmup}")
    for _ in range(args.warmup):
        ld.ld_logabsdet_cheb(D, Ct, smin, smax, n, M, seed, workspace=ws)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    kms = kn = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ld.ld_logabsdet_cheb(D, Ct, smin, smax, n, M, seed, workspace=ws, timing=True)
        kms += r["kernel_ms"]
        kn += r["kernel_launches"]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    work = 2 * M * n * nnz
    value = work / (ms / 1e3)
    sb = step_bytes(d, nnz, M, 4, 4)
    avg = kms / max(kn, 1)
    achieved = sb / (avg / 1e3) / 1e9
    cpu = parity = None
    if not args.no_cpu_baseline:
        deg = 2  # about 10 s of oracle work on one core
        log(f"cpu baseline (oracle, probe 0 at degree {deg})")
        rg = ld.ld_logabsdet_cheb(D, Ct, smin, smax, deg, M, seed, want_probes=True)
        import oracle

        oracle.build()
        t1 = time.perf_counter()
        o = oracle.logabsdet(C, smin, smax, deg, 1, seed=seed, ids=np.array([0]))
        secs = time.perf_counter() - t1
        cpu = {"value": 2 * deg * nnz / secs, "unit": "matvec-nnz/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"probe 0 at degree {deg} of Algorithm 2 on the full matrix, single-threaded FP64 C oracle, "
                         f"{secs:.1f} s"}
        parity = abs(rg["s"][0] - o["s"][0]) / max(abs(o["s"][0]), 1e-3 * d)
    out = {
        "metric": METRIC, "value": value, "unit": "matvec-nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(value / SEC51_PAPER_RATE, 1), "dtype": "f32", "data": "synthetic",
        "config": {"workload": W["desc"], "d": d, "nnz": nnz, "M": M, "n": n,
                   "step": "Algorithm 2 forward (C^T and bounds prepared once, before timing)",
                   "parallelism": "single GPU",
                   "paper": "500 s on a 3.40 GHz Intel i7 for this run (3e8 stored entries); vs_baseline divides "
                            "by the rate that implies, 10*15*2*3e8/500 matvec-nnz/s"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": "step kernel",
                     "avg_launch_ms": round(avg, 5), "algorithmic_bytes_per_launch": sb},
        "cpu_baseline": cpu,
        "accuracy": {"log_abs_det": r["logdet"], "std_err_rel": abs(r["std_err"] / r["logdet"]),
                     "oracle_parity_rel_probe0_deg2": parity, "parity_tolerance": 1e-4},
    }
    if copy_gbps is not None:
        out["copy_kernel_GBps"] = round(copy_gbps, 1)
        out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / copy_gbps, 4)
    print(json.dumps(out), flush=True)


def _finish(out: dict, copy_gbps) -> None:
    if copy_gbps is not None:
        out["copy_kernel_GBps"] = round(copy_gbps, 1)
        out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / copy_gbps, 4)
    print(json.dumps(out), flush=True)


def _line(args, W, value, ms, dtype, config, achieved, avg_ms, bytes_, kernel, cpu, accuracy) -> dict:
    return {
        "metric": METRIC, "value": value, "unit": "matvec-nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": dict({"workload": W["desc"], "parallelism": "single GPU"}, **config),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": kernel,
                     "avg_launch_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": bytes_},
        "cpu_baseline": cpu, "accuracy": accuracy,
    }


def bench_trees(args, W, copy_gbps) -> None:
    """Spanning-tree counting (Section 3.3) on a hub graph with 1e6 vertices: each step builds the
    Laplacian minor on the device and runs Algorithm 2 on it."""
    import numpy as np
    import torch

    import paper_1503_06394_amd as ld
    import synth

    G = synth.hub_graph(W["nv"], W["k_off"], W["mseed"])
    D = ld.DeviceCSR.from_host(G, device="cuda:0")
    n, M, seed = W["n"], W["M"], W["seed"]
    dm, nnz_l = G.d - 1, G.nnz - (G.d - 1)  # the minor: hub row and column out, the diagonal in
    log(f"graph: {G.d} vertices, {G.nnz} adjacency entries; minor d={dm} nnz={nnz_l}")
    for _ in range(args.warmup):
        ld.ld_log_spanning_trees(D, 0, n, M, seed)
    torch.cuda.synchronize()
    kms = kn = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ld.ld_log_spanning_trees(D, 0, n, M, seed, timing=True, want_probes=True)
        kms += r["kernel_ms"]
        kn += r["kernel_launches"]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    value = 2 * M * n * nnz_l / (ms / 1e3)
    sb = step_bytes(dm, nnz_l, M, 4, 4)
    avg = kms / max(kn, 1)
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        deg = 4
        log(f"cpu baseline (oracle minor, then Algorithm 2 probe 0 at degree {deg})")
        L, dmax = oracle.laplacian_minor(G, 0)
        rg = ld.ld_log_spanning_trees(D, 0, deg, M, seed, want_probes=True)
        t1 = time.perf_counter()
        o = oracle.logabsdet(L, 1.0, 2.0 * dmax - 1.0, deg, 1, seed=seed, ids=np.array([0]))
        secs = time.perf_counter() - t1
        cpu = {"value": 2 * deg * nnz_l / secs, "unit": "matvec-nnz/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"probe 0 at degree {deg} of Algorithm 2 on the minor (built beforehand), single-threaded "
                         f"FP64 C oracle, {secs:.1f} s"}
        parity = abs(rg["s"][0] - o["s"][0]) / max(abs(o["s"][0]), 1e-3 * dm)
    out = _line(args, W, value, ms, "f32",
                {"d": G.d, "nnz": G.nnz, "M": M, "n": n, "minor_nnz": nnz_l,
                 "step": "Laplacian minor + Algorithm 2 (Section 3.3)"},
                sb / (avg / 1e3) / 1e9, avg, sb, "step kernel", cpu,
                {"log_spanning_trees": r["logdet"], "std_err_rel": abs(r["std_err"] / r["logdet"]),
                 "oracle_parity_rel_probe0_deg4": parity, "parity_tolerance": 1e-4})
    _finish(out, copy_gbps)


def bench_taylor(args, W, copy_gbps) -> None:
    """The Taylor-series comparator of Section 5.1 at scale, beside the Chebyshev estimate with the
    same probes and degree; both against the grid's closed-form log det."""
    import numpy as np
    import torch

    import paper_1503_06394_amd as ld

    B = W["B"]
    D = ld.DeviceCSR.from_host(B, device="cuda:0", diag_shift=W["shift"])
    a, b, n, M, seed = W["a"], W["b"], W["n"], W["M"], W["seed"]
    for _ in range(args.warmup):
        ld.ld_logdet_taylor(D, a, b, n, M, seed)
    torch.cuda.synchronize()
    kms = kn = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ld.ld_logdet_taylor(D, a, b, n, M, seed, timing=True, want_probes=True)
        kms += r["kernel_ms"]
        kn += r["kernel_launches"]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    rc = ld.ld_logdet_cheb(D, a, b, n, M, seed)
    N = 4096
    mu = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, N + 1) / (N + 1))
    exact = float(np.log((mu[:, None] + mu[None, :]).ravel() + W["shift"]).sum())
    value = M * n * B.nnz / (ms / 1e3)
    # a Taylor step W_{k+1} = A W_k reads the matrix and W_k once and writes W_{k+1}: two vector blocks
    sb = csr_bytes(B.d, B.nnz, 2) + 2 * B.d * M * 4
    avg = kms / max(kn, 1)
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        deg = 10
        log(f"cpu baseline (oracle Taylor comparator, probe 0 at degree {deg})")
        rg = ld.ld_logdet_taylor(D, a, b, deg, M, seed, want_probes=True)
        t1 = time.perf_counter()
        o = oracle.logdet_taylor(B, a, b, deg, 1, seed=seed, ids=np.array([0]), shift=W["shift"])
        secs = time.perf_counter() - t1
        cpu = {"value": deg * B.nnz / secs, "unit": "matvec-nnz/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"probe 0 at degree {deg} of the Taylor comparator on the full grid, single-threaded FP64 C "
                         f"oracle, {secs:.1f} s"}
        parity = abs(rg["s"][0] - o["s"][0]) / max(abs(o["s"][0]), 1e-3 * B.d)
    out = _line(args, W, value, ms, "f32",
                {"d": B.d, "nnz": B.nnz, "M": M, "n": n, "values": "bf16", "step": "Taylor comparator forward"},
                sb / (avg / 1e3) / 1e9, avg, sb, "step kernel", cpu,
                {"logdet_exact": exact, "taylor": r["logdet"], "taylor_rel_err": abs(r["logdet"] - exact) / abs(exact),
                 "taylor_truncation_bound_rel": abs(r["poly_bound"] / exact),
                 "chebyshev": rc["logdet"], "chebyshev_rel_err": abs(rc["logdet"] - exact) / abs(exact),
                 "oracle_parity_rel_probe0_deg10": parity, "parity_tolerance": 1e-4})
    _finish(out, copy_gbps)


def bench_lanczos(args, W, copy_gbps) -> None:
    """The spectral estimate that feeds the bounds (Section 3.2): FP64 Lanczos on the main
    workload's matrix, one product per step (M = 1)."""
    import numpy as np
    import torch

    import paper_1503_06394_amd as ld

    B, iters, seed = W["B"], W["iters"], W["seed"]
    D = ld.DeviceCSR.from_host(B, device="cuda:0")
    for _ in range(args.warmup):
        ld.ld_spectral_estimate(D, iters=iters, seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lo, hi = ld.ld_spectral_estimate(D, iters=iters, seed=seed)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    value = iters * B.nnz / (ms / 1e3)
    # per Lanczos step: the product (matrix, x gathered, y written) and three FP64 vector passes
    per_step = B.nnz * 8 + (B.d + 1) * 8 + 2 * B.d * 8 + 7 * B.d * 8
    achieved = per_step / (ms / iters / 1e3) / 1e9
    ga, gb = ld.ld_gershgorin(D)
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        k = 25
        log(f"cpu baseline (oracle Lanczos, {k} steps)")
        glo, ghi = ld.ld_spectral_estimate(D, iters=k, seed=seed)
        t1 = time.perf_counter()
        olo, ohi, _, _ = oracle.lanczos_extremes(B, k, seed=seed)
        secs = time.perf_counter() - t1
        cpu = {"value": k * B.nnz / secs, "unit": "matvec-nnz/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"{k} Lanczos steps on the full matrix, FP64 numpy oracle, {secs:.1f} s"}
        parity = max(abs(glo - olo) / abs(olo), abs(ghi - ohi) / abs(ohi))
    out = _line(args, W, value, ms, "f64",
                {"d": B.d, "nnz": B.nnz, "M": 1, "iters": iters, "step": "300 Lanczos steps and the tridiagonal's "
                 "extreme eigenvalues"},
                achieved, ms / iters, per_step, "one Lanczos step (product, dots, update)", cpu,
                {"ritz_lo": lo, "ritz_hi": hi, "gershgorin": [ga, gb],
                 "oracle_parity_rel_25_steps": parity, "parity_tolerance": 1e-9})
    _finish(out, copy_gbps)


if __name__ == "__main__":
    main()
