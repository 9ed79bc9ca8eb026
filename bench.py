#!/usr/bin/env python3
"""Benchmark of the fractional-Poisson hot path on one MI355X.

Workload (the headline configuration): 2D, Omega = (-1,1)^2, N = 512
(511^2 = 261,121 unknowns, embedding 1024^2), quadratic basis, alpha cycling
over {0.5, 1.0, 1.5}; each step solves one batch of 17 right-hand sides
(the manufactured right-hand side of u = (1-|x|^2)_+^{1+alpha/2} inside the
unit disk plus 16 U[-1,1] fields, seeds 0..15) to a relative residual of
1e-10 with FP64 PCG (fl_solve; `--path reliable` times the FP32 CG with FP64
reliable updates instead, which is otherwise reported beside it).
Operators (weights, symbol) are built before the timed region; inputs are
resident in HBM when it starts.

Printed: one JSON line with solves/s (right-hand sides solved per second),
p50/p99 latency of a batch, the FP64 one-at-a-time path for comparison,
the roofline of the dominant FFT-matvec kernel (HIP events inside the
library, on the stream the kernels run on), and the CPU oracle timed on a
bounded sample as a baseline.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# Vector ALU peak without packed FP32 math (which this build does not emit):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz; FP64 vector is the same.
VALU_PEAK_TFLOPS = 78.6

# HBM bytes per launch of the roofline kernels from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE runs of `bench.py --roofline-only`, each scaled by what the
# same counter reads for a device copy of known size in that run.  Keyed by
# (kernel, precision, nrhs); valid only for the kernel sources they were
# measured on (SHA-256 prefix of the files that define the transform kernels).
TRAFFIC = {
    ("axis0_fwd_r2c", "f64", 17): 109219917,
    ("last_axis_fwd_symbol_inv", "f64", 17): 145083958,
    ("axis0_inv_c2r", "f64", 17): 108995204,
    ("tau_axis0_sine", "f64", 17): 72937095,
    ("tau_last_axis_sine_mult_sine", "f64", 17): 73720767,
    ("tau_axis0_sine_back", "f64", 17): 72937095,
}
TRAFFIC_SRC = "058bdcb69e9add1e"


def pass_sources_hash():
    import hashlib
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2103_03658_amd", "csrc")
    h = hashlib.sha256()
    for fn in ("fl_device.h", "passes_impl.h"):
        with open(os.path.join(root, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, fp32, nrhs=17):
    key = (kernel, "f32" if fp32 else "f64", nrhs)
    if key not in TRAFFIC or TRAFFIC_SRC != pass_sources_hash():
        return None
    return TRAFFIC[key]
METRIC = ("CG solves/s + p50/p99 latency (2D 511², tol 1e-10); "
          "FFT-matvec HBM GB/s")


def progress(msg):
    """One line per finished phase on stderr (the JSON line goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=21,
                    help="timed batched solves (7 per alpha: p50/p99 over >= 20)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--degree", type=int, default=2)
    ap.add_argument("--nrand", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--path", choices=["reliable", "refine", "fp64"], default="fp64",
                    help="reliable: FP32 CG with FP64 reliable updates; refine: restarted FP32 "
                         "inner solves with FP64 refinement; fp64: FP64 CG")
    ap.add_argument("--mixed-steps", type=int, default=None,
                    help="timed batched solves of the mixed-precision path reported beside the "
                         "headline path, after the same warm-up (default: --steps; 0: skip)")
    ap.add_argument("--delta", type=float, default=None,
                    help="reliable path: residual reduction that triggers an FP64 update")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="refine path: relative tolerance of each FP32 inner solve")
    ap.add_argument("--fp64-single", type=int, default=2,
                    help="right-hand sides per alpha solved one at a time in FP64 for comparison")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle work for the CPU baseline (0: skip)")
    ap.add_argument("--profile-reps", type=int, default=20)
    ap.add_argument("--d2-reps", type=int, default=100,
                    help="back-to-back launches per pass in the large-working-set products")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch schedule")
    ap.add_argument("--tune-cache", action="store_true",
                    help="reuse / store tuned schedules in the tuner's JSON cache "
                         "(FL_SCHEDULE_CACHE), so a profiler run can skip the tuning launches")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="roofline-only: also run a device copy of this many MiB, three times "
                         "(the known-size kernel that scales the HBM byte counters)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only time the FFT-matvec kernels (for profiler runs)")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the serving stream (Poisson arrivals at 200/s; 0: skip)")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-graphs", type=int, default=1,
                    help="fl_set_graphs mode of the served operators (2: capture a CG chunk "
                         "when it runs a second time; 1: at its first run; 0: never)")
    ap.add_argument("--serve-fp64", type=int, default=1,
                    help="1: also serve the stream with FP64 PCG beside the mixed path")
    ap.add_argument("--serve-burst", type=int, default=512,
                    help="requests of the burst stream (six operators, arrivals at 4000/s; 0: skip)")
    ap.add_argument("--serve-sample", type=int, default=32,
                    help="requests of each stream re-solved alone and compared with the mix")
    ap.add_argument("--configs", type=int, default=1,
                    help="1: also measure the 1D, 2D 255^2, 3D 127^3 and tempered 1023^2 "
                         "workloads (a few seconds); 0: skip")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--general-n-only", action="store_true",
                    help="only the tau-vs-circulant comparison on grids whose 2N is not a "
                         "power of two (for profiler runs)")
    ap.add_argument("--d2-only", action="store_true",
                    help="only time the product on the large working sets (default and tuned "
                         "schedules; for profiler runs)")
    ap.add_argument("--d2", type=int, default=1,
                    help="1: report the large-working-set products in the bench line")
    return ap.parse_args()


def run_serving(n_requests, workers, tol, mixed=1, sample=32, burst=False, graphs=1):
    """Serving stream: d = 2, n in {63,127,255,511}, alpha ~ U(0.2, 1.9)
    rounded to 0.01, degree in {0,1,2}, 1-8 U[-1,1] right-hand sides,
    Poisson arrivals at 200 requests/s, solves to tol with the mixed path
    (mixed = 1) or FP64 PCG (mixed = 0); burst: the six-operator stream at
    4000 requests/s.  `sample` requests spread over the stream are solved
    again alone on fresh operators and compared with their result in the mix."""
    import torch
    import paper_2103_03658_amd as fl
    from paper_2103_03658_amd import inputs
    from paper_2103_03658_amd.serve import Request, Server
    if burst:
        spec = inputs.burst_stream(n_requests)
    else:
        spec = inputs.request_stream(n_requests, rate=200.0, seed=0)
    reqs = [Request(r["id"], 2, r["N"], r["alpha"], r["degree"],
                    torch.from_numpy(inputs.request_rhs(r)).cuda(), t_arrive=r["t_arrive"])
            for r in spec]
    torch.cuda.synchronize()
    step = max(1, n_requests // max(1, sample))
    keep = set(range(0, n_requests, step)[:sample])
    warm = sorted({(2, r["N"], r["degree"]) for r in spec})
    srv = Server(workers=workers, tol=tol, mixed=mixed, warm=warm, keep_solutions=keep,
                 graphs=graphs)
    st = srv.run(reqs, realtime=True)
    # alone against the mix: each sampled request on a fresh operator of its own
    same, worst = 0, 0.0
    for r in reqs:
        if r.id not in keep or r.u is None:
            continue
        op = fl.Operator(2, r.alpha, r.degree, N=r.N)
        u, _ = op.solve(r.f, tol=tol, mixed=mixed)
        same += int(torch.equal(u, r.u))
        worst = max(worst, float((u - r.u).abs().max() / u.abs().max()))
        op.close()
    st["alone_vs_mix"] = {"sampled": len(keep), "bitwise_equal": same,
                          "max_rel_linf_diff": worst}
    prec = "FP32 CG with FP64 reliable updates" if mixed else "FP64 PCG"
    if burst:
        st["stream"] = (f"{n_requests} requests, Poisson arrivals at 4000/s, d=2, n in "
                        "{127,255}, alpha in {0.5,1,1.5}, degree 1 (six operators), 1-8 U[-1,1] "
                        f"RHS each, {prec} to {tol:g}, {workers} worker streams")
    else:
        st["stream"] = (f"{n_requests} requests, Poisson arrivals at 200/s, d=2, "
                        "n in {63,127,255,511} (p=.4/.3/.2/.1), alpha~U(0.2,1.9) rounded to 0.01, "
                        f"degree in {{0,1,2}}, 1-8 U[-1,1] RHS each, {prec} "
                        f"to {tol:g}, {workers} worker streams, each warmed first by one solve "
                        "per (N, degree) of the stream (warmup_s)")
    st["precision"] = prec
    return st


def pass_bytes(d, N, nrhs, sr):
    """Algorithmic HBM bytes of each kernel of one batched product y = A u
    (2D: axis-0 forward, last-axis fused, axis-0 inverse).  Complex values
    are 2*sr bytes; the axis-0 frequency keeps rows 0..M/2 (Hermitian half)."""
    n, M = N - 1, 2 * N
    h = M // 2 + 1
    assert d == 2
    vec = n * n * sr * nrhs
    mid = h * n * 2 * sr * nrhs
    sym = (N + 1) ** 2 * sr
    return [vec + mid, 2 * mid + sym, mid + vec]


def pass_flops(d, N, nrhs):
    """Nominal flops of each kernel of one batched 2D product: 5 M log2 M per
    length-M complex transform, 2 per complex element for the symbol
    multiply, 6 per output pair for the Hermitian split / merge."""
    n, M = N - 1, 2 * N
    h = M // 2 + 1
    assert d == 2
    fft = 5.0 * M * math.log2(M)
    pairs = (n + 1) // 2
    col = pairs * (fft + 6.0 * h)
    mid = h * (2.0 * fft + 2.0 * M)
    return [col * nrhs, mid * nrhs, col * nrhs]


def pass_bytes_3d(N, nrhs, sr):
    """Algorithmic HBM bytes of the five kernels of one batched 3D product:
    axis-0 forward (n^3 real in, h n^2 complex out), axis-1 forward (h n^2
    in, h M n out), last axis (h M n complex in and out, plus the folded
    symbol), axis-1 inverse, axis-0 inverse (h = M/2 + 1, M = 2N)."""
    n, M = N - 1, 2 * N
    h = M // 2 + 1
    vec = n ** 3 * sr * nrhs
    t1 = h * n * n * 2 * sr * nrhs
    t2 = h * M * n * 2 * sr * nrhs
    sym = (N + 1) ** 3 * sr
    return [vec + t1, t1 + t2, 2 * t2 + sym, t2 + t1, t1 + vec]


def d2_shapes(dev, reps=20, use_cache=False):
    """The product on working sets far beyond the 256 MB Infinity Cache, with
    the default launch schedule and the tuned one: tempered 2D 1023^2 FP32 x
    64 right-hand sides, 3D 127^3 FP32 x 8 and FP64 x 4, and the headline 2D
    511^2 FP64 x 17 (0.64 GB, partly cache-resident).  Per kernel: HIP-event
    milliseconds (each kernel `reps` times back to back) and GB/s of the
    algorithmic bytes."""
    import torch
    import paper_2103_03658_amd as fl
    from paper_2103_03658_amd import inputs, tune
    shapes = [("C5_2d_1023_tempered_fp32_x64", 2, 1024, 1, 1.2, 1.0, 64, True),
              ("C3_3d_127_fp32_x8", 3, 128, 1, 1.0, 0.0, 8, True),
              ("C3_3d_127_fp64_x4", 3, 128, 1, 1.0, 0.0, 4, False),
              ("D1_2d_511_fp64_x17", 2, 512, 2, 1.5, 0.0, 17, False)]
    out = {}
    for name, d, N, p, a, lam, nrhs, fp32 in shapes:
        op = (fl.Operator(d, a, p, N=N, kernel="tempered", lam=lam) if lam
              else fl.Operator(d, a, p, N=N))
        dt = torch.float32 if fp32 else torch.float64
        u = torch.from_numpy(inputs.uniform_rhs(d, N, nrhs, seed=0)).to(dev).to(dt)
        sr = 4 if fp32 else 8
        by = pass_bytes_3d(N, nrhs, sr) if d == 3 else pass_bytes(2, N, nrhs, sr)
        res = {"bytes_per_product": sum(by), "nrhs": nrhs, "precision": "f32" if fp32 else "f64"}
        for label in ("default", "tuned"):
            if label == "tuned":
                tune.tune(op, nrhs, fp32, use_cache=use_cache)
            ms = op.profile_apply(u, reps=reps)
            res[label] = {"schedule": op.get_schedule(fp32), "ms_per_kernel": ms,
                          "GBs_per_kernel": [b / (t * 1e-3) / 1e9 for b, t in zip(by, ms)],
                          "matvec_ms": sum(ms), "GBs": sum(by) / (sum(ms) * 1e-3) / 1e9,
                          "frac_of_8TBs": sum(by) / (sum(ms) * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out[name] = res
        op.close()
        del u
        torch.cuda.empty_cache()
    return out


def precond_bytes(d, N, nrhs, sr):
    """Algorithmic HBM bytes of each kernel of one batched tau preconditioner
    application (2D: axis-0 sine pass, last-axis sine * multiplier * sine in
    place, axis-0 sine pass): every intermediate is real, n^2 per RHS."""
    n = N - 1
    assert d == 2
    vec = n * n * sr * nrhs
    sym = (N + 1) ** 2 * sr
    return [2 * vec, 2 * vec + sym, 2 * vec]


def precond_flops(d, N, nrhs):
    """Nominal flops of the tau passes: 5 M log2 M per length-M transform of
    a packed pair of odd-extended lines, 2 per element for the multiplier."""
    n, M = N - 1, 2 * N
    assert d == 2
    fft = 5.0 * M * math.log2(M)
    pairs = (n + 1) // 2
    col = pairs * fft
    mid = pairs * (2.0 * fft + 2.0 * M)
    return [col * nrhs, mid * nrhs, col * nrhs]


def run_configs(dev, tol, quick=False):
    """The other workloads of the method at their full sizes (not the headline
    metric): per config, solves/s or latency, iterations, true residuals; and
    FFT-matvec rates on the large-working-set shapes (tempered 1023^2 x 64
    RHS FP32, 3D 127^3 x 8 RHS FP32)."""
    import torch
    import paper_2103_03658_amd as fl
    from paper_2103_03658_amd import inputs, tune

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    out = {}
    # C1: 1D, N = 1024 (h = 1/512), alpha = 1.5, p = 1, FP64, tol 1e-12
    op = fl.Operator(1, 1.5, 1, N=1024)
    f = torch.from_numpy(np.stack([np.full(1023, math.gamma(2.5)),
                                   inputs.uniform_rhs(1, 1024, 1, seed=0)[0]])).to(dev)
    t, (u, inf) = timed(lambda: op.solve(f, tol=1e-12), 5)
    out["C1_1d_N1024"] = {"ms_per_batched_solve": 1e3 * t, "nrhs": 2,
                          "iters": [i["iters"] for i in inf],
                          "relres_true": [i["relres_true"] for i in inf]}
    op.close()
    # C2: 2D 255^2, p = 2, 17 RHS, FP64 PCG, tol 1e-10
    c2 = {}
    for a in (0.5, 1.0, 1.5):
        op = fl.Operator(2, a, 2, N=256)
        tune.tune(op, 17, False, use_cache=False)
        f = torch.from_numpy(np.concatenate([inputs.manufactured_rhs_disk(256, a)[None],
                                             inputs.uniform_rhs(2, 256, 16, seed=0)])).to(dev)
        t, (u, inf) = timed(lambda: op.solve(f, tol=tol), 3)
        c2[str(a)] = {"solves_per_s": 17 / t, "iters": max(i["iters"] for i in inf),
                      "max_relres_true": max(i["relres_true"] for i in inf)}
        op.close()
    out["C2_2d_255_fp64_17rhs"] = c2
    out["C2_h_sweep_p2"] = h_sweep(dev)
    # C3: 3D 127^3, alpha = 1, p = 1, N(0,1) seed 3, mixed precision; FP64 as reference
    op = fl.Operator(3, 1.0, 1, N=128)
    for fp32 in (True, False):
        tune.tune(op, 1, fp32, use_cache=False)
    f = torch.from_numpy(inputs.normal_rhs(3, 128, 1, seed=3)).to(dev)
    tm, (um, im) = timed(lambda: op.solve(f, tol=tol, mixed=1), 3)
    t6, (u6, i6) = timed(lambda: op.solve(f, tol=tol, mixed=0), 3)
    u8 = torch.from_numpy(inputs.normal_rhs(3, 128, 8, seed=3).astype(np.float32)).to(dev)
    ms3 = op.profile_apply(u8, reps=10)
    # per RHS: n^3 real in and out, and h n^2 (axis 0) and h M n (axis 1) complex
    # lines each written and read twice; the folded symbol once per product
    n3, M3 = 127, 256
    h3 = M3 // 2 + 1
    by3 = 8 * 4 * (2 * n3 ** 3 + 8 * (h3 * n3 * n3 + h3 * M3 * n3)) + 129 ** 3 * 4
    out["C3_3d_127"] = {"mixed_s_per_solve": tm, "fp64_s_per_solve": t6,
                        "mixed_iters": im[0]["iters"], "mixed_updates": im[0]["outer_iters"],
                        "fp64_iters": i6[0]["iters"], "relres_true_mixed": im[0]["relres_true"],
                        "mixed_vs_fp64_rel_linf": float((um - u6).abs().max() / u6.abs().max()),
                        "matvec_fp32_8rhs_ms": sum(ms3),
                        "matvec_fp32_8rhs_GBs": by3 / (sum(ms3) * 1e-3) / 1e9,
                        "matvec_ms_per_pass": ms3}
    op.close()
    # C5: tempered 2D 1023^2, alpha = 1.2, p = 1, 64 N(0,1) RHS per lambda, mixed to tol
    c5 = {}
    f = torch.from_numpy(inputs.normal_rhs(2, 1024, 64, seed=0)).to(dev)
    for lam in ((1.0,) if quick else (0.5, 1.0, 5.0)):
        op = fl.Operator(2, 1.2, 1, N=1024, kernel="tempered", lam=lam)
        best32, _ = tune.tune(op, 64, True, use_cache=False)
        tune.tune(op, 64, False, use_cache=False)
        t, (u, inf) = timed(lambda: op.solve(f, tol=tol, mixed=1), 1)
        t64, (u64, inf64) = timed(lambda: op.solve(f, tol=tol, mixed=0), 1)
        ms5 = op.profile_apply(f.to(torch.float32), reps=10)
        by5 = pass_bytes(2, 1024, 64, 4)
        c5[str(lam)] = {"mixed_solves_per_s": 64 / t, "fp64_solves_per_s": 64 / t64,
                        "mixed_iters": max(i["iters"] for i in inf),
                        "fp64_iters": max(i["iters"] for i in inf64),
                        "max_relres_true_mixed": max(i["relres_true"] for i in inf),
                        "schedule_f32": best32,
                        "matvec_fp32_64rhs_ms": sum(ms5),
                        "matvec_fp32_64rhs_GBs": sum(by5) / (sum(ms5) * 1e-3) / 1e9,
                        "per_pass_GBs": [b / (m * 1e-3) / 1e9 for b, m in zip(by5, ms5)]}
        op.close()
    out["C5_tempered_1023_64rhs"] = c5
    out["general_n_tau"] = general_n_tau(dev, tol)
    return out


def general_n_tau(dev, tol, reps=3):
    """Grids whose 2N is not a power of two (2D, p = 1, 4 U[-1,1] RHS):
    the tau preconditioner on mixed-radix sine passes (2N = 1200, 1400, 2000)
    against the restricted circulant inverse on the power-of-two embedding:
    iterations and ms per batched solve (FP64 and mixed), and the
    preconditioner's passes (HIP events, 10 back-to-back launches each)."""
    import torch
    import paper_2103_03658_amd as fl
    from paper_2103_03658_amd import inputs
    out = {}
    for N in (600, 700, 1000):
        for a in (0.5, 1.5):
            op = fl.Operator(2, a, 1, N=N)
            f = torch.from_numpy(inputs.uniform_rhs(2, N, 4, seed=1)).to(dev)
            res = {}
            for kind in (1, 2):
                op.set_preconditioner(kind)
                res[f"precond{kind}_us_per_pass"] = [1e3 * x for x in
                                                     op.profile_precond(f, reps=10)]
                for mixed in (0, 1):
                    op.solve(f, tol=tol, mixed=mixed)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        _, info = op.solve(f, tol=tol, mixed=mixed)
                    torch.cuda.synchronize()
                    res[f"kind{kind}_{'mixed' if mixed else 'fp64'}"] = {
                        "ms_per_batched_solve": 1e3 * (time.perf_counter() - t0) / reps,
                        "iters": max(i["iters"] for i in info),
                        "max_relres_true": max(i["relres_true"] for i in info)}
            out[f"N{N}_alpha{a}"] = res
            op.close()
    return out


def h_sweep(dev, Ns=(64, 128, 256, 512), alphas=(0.5, 1.0, 1.5)):
    """h-refinement of the 2D quadratic-basis operator (63^2 -> 511^2): the
    product on u = (1-|x|^2)_+^{4+alpha/2} (supported in the unit disk, so no
    exterior data) against its closed-form image at the points
    {-1/2, -1/4, 0, 1/4, 1/2}^2, where it is the terminating series
    2^alpha Gamma(1+alpha/2) Gamma(s+1)/Gamma(s+1-alpha/2) 2F1(1+alpha/2, -4; 1; |x|^2),
    s = 4 + alpha/2; the measured rate (the origin element caps the
    quadratic basis at 4 - alpha)."""
    import torch
    from scipy.special import hyp2f1
    import paper_2103_03658_amd as fl
    pts = (-0.5, -0.25, 0.0, 0.25, 0.5)
    out = {}
    for a in alphas:
        s_ = 4.0 + a / 2.0
        errs = []
        for N in Ns:
            op = fl.Operator(2, a, 2, N=N)
            x = -1.0 + (2.0 / N) * np.arange(1, N)
            X0, X1 = np.meshgrid(x, x, indexing="ij")
            u = np.maximum(1.0 - X0 * X0 - X1 * X1, 0.0) ** s_
            y = op.apply(torch.from_numpy(u[None].copy()).to(dev)).cpu().numpy()[0]
            idx = [int(round((v + 1.0) * N / 2.0)) - 1 for v in pts]
            got = y[np.ix_(idx, idx)]
            xs = np.array(pts)
            r2 = xs[:, None] ** 2 + xs[None, :] ** 2
            pref = (2.0 ** a * math.gamma(1.0 + a / 2.0) * math.gamma(s_ + 1.0)
                    / math.gamma(s_ + 1.0 - a / 2.0))
            ref = pref * hyp2f1(1.0 + a / 2.0, a / 2.0 - s_, 1.0, r2)
            errs.append(float(np.abs(got - ref).max()))
            op.close()
        out[str(a)] = {"N": list(Ns), "max_err": errs,
                       "rates": [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]}
    return out


def cpu_baseline(N, degree, alpha, tol, budget):
    """Time the oracle on this host: whole solves of one right-hand side by
    its preconditioned CG (dense block-Toeplitz product, no FFT, for A; the
    FFT form of the circulant inverse for P), repeated while the budget lasts."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    # BLAS threads: the host cores this process may use, capped at 16 (one
    # GPU's share of a multi-GPU host's cores); `cores` reports the count used
    cores = len(os.sched_getaffinity(0))
    cores = min(cores, 16)
    ctx = threadpool_limits(limits=cores) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        G = oracle.generator(2, alpha, degree, N)
        t_gen = time.perf_counter() - t0
        from paper_2103_03658_amd import inputs
        f = inputs.uniform_rhs(2, N, 1, seed=0)[0]
        pc = lambda v: oracle.precond_apply(G, v)
        ns, its = 0, []
        t0 = time.perf_counter()
        while True:
            _, it, rel = oracle.solve_cg(G, f, tol=tol, precond=pc)
            its.append(it)
            ns += 1
            el = time.perf_counter() - t0
            if el > budget or ns >= 20:
                break
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    t_s = el / ns
    return dict(value=1.0 / t_s, unit="solves/s", cores=cores, kind="oracle",
                sample=(f"{ns} oracle solves of one uniform RHS at {N - 1}^2, p={degree}, "
                        f"alpha={alpha}, tol {tol:g}: preconditioned CG on the dense "
                        f"block-Toeplitz product, {its[0]} iterations, {t_s:.2f} s per solve "
                        f"(final rel. residual {rel:.1e}); oracle generator {t_gen:.1f} s "
                        f"not included"),
                solve_s=t_s, iterations=its[0], generator_s=t_gen)


def serving_legs(args):
    """The serving stream with the mixed path (as configured), beside it the
    same stream with FP64 PCG, and the burst stream in which same-operator
    requests queue and are merged."""
    if args.serve_requests <= 0:
        return None
    kw = dict(sample=args.serve_sample, graphs=args.serve_graphs)
    out = run_serving(args.serve_requests, args.serve_workers, args.tol, mixed=1, **kw)
    progress("serving stream (mixed) done")
    if args.serve_fp64:
        out["fp64"] = run_serving(args.serve_requests, args.serve_workers, args.tol, mixed=0,
                                  **kw)
    if args.serve_burst > 0:
        out["burst"] = run_serving(args.serve_burst, args.serve_workers, args.tol, mixed=1,
                                   burst=True, **kw)
        if args.serve_fp64:
            # the same saturated stream in FP64 PCG: the batched serving path's
            # throughput in each precision when requests queue
            out["burst_fp64"] = run_serving(args.serve_burst, args.serve_workers, args.tol,
                                            mixed=0, burst=True, **kw)
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                          f"--gpus {args.gpus} (WORLD_SIZE {world}) is not supported"}))
        sys.exit(2)
    import torch
    import paper_2103_03658_amd as fl
    from paper_2103_03658_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serve_only:
        print(json.dumps({"serving": serving_legs(args)}))
        return
    if args.general_n_only:
        print(json.dumps({"general_n_tau": general_n_tau(dev, args.tol)}))
        return
    if args.d2_only:
        print(json.dumps({"d2": d2_shapes(dev, reps=args.d2_reps,
                                          use_cache=args.tune_cache)}))
        return
    N, p = args.N, args.degree
    alphas = [0.5, 1.0, 1.5]
    nrhs = 1 + args.nrand
    t0 = time.perf_counter()
    ops, rhs = {}, {}
    setup_s = {}
    for a in alphas:
        ts = time.perf_counter()
        ops[a] = fl.Operator(2, a, p, N=N)
        torch.cuda.synchronize()
        setup_s[a] = time.perf_counter() - ts
        f = np.concatenate([inputs.manufactured_rhs_disk(N, a)[None],
                            inputs.uniform_rhs(2, N, args.nrand, seed=0)])
        rhs[a] = torch.from_numpy(f).to(dev)
    out = torch.empty_like(rhs[alphas[0]])
    mixed = {"fp64": 0, "reliable": 1, "refine": 2}[args.path]
    if args.delta is not None or args.inner_tol is not None:
        for a in alphas:
            ops[a].set_refinement(delta=args.delta if args.delta is not None else 1e-5,
                                  inner_tol=args.inner_tol if args.inner_tol is not None else 1e-4)

    # launch schedules: tuned once per precision on one operator (same M for all)
    from paper_2103_03658_amd import tune as _tune
    sched = {"default_f32": ops[1.5].get_schedule(True), "default_f64": ops[1.5].get_schedule(False)}
    if not args.no_tune:
        t_tune = time.perf_counter()
        for fp32 in (True, False):
            best, _ = _tune.tune(ops[1.5], nrhs, fp32, use_cache=args.tune_cache)
            bestp = ops[1.5].get_schedule(fp32, precond=True)
            for a in alphas:
                ops[a].set_schedule(fp32, **best)
                ops[a].set_schedule(fp32, precond=True, **bestp)
        sched["tune_s"] = time.perf_counter() - t_tune
    sched["f32"] = ops[1.5].get_schedule(True)
    sched["f64"] = ops[1.5].get_schedule(False)
    sched["precond_f32"] = ops[1.5].get_schedule(True, precond=True)
    sched["precond_f64"] = ops[1.5].get_schedule(False, precond=True)

    if args.roofline_only:
        if args.calib_copy_mib > 0:
            nb = args.calib_copy_mib << 20
            src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        # the timed path's precision: FP64 unless a mixed path is selected
        fp32 = mixed != 0
        u_ = rhs[1.5].to(torch.float32).contiguous() if fp32 else rhs[1.5]
        acc = None
        for _ in range(max(1, args.steps)):
            m = ops[1.5].profile_apply(u_, reps=args.profile_reps)
            acc = m if acc is None else [x + y for x, y in zip(acc, m)]
        ms = [x / max(1, args.steps) for x in acc]
        by = pass_bytes(2, N, nrhs, 4 if fp32 else 8)
        acc = None
        for _ in range(max(1, args.steps)):
            m = ops[1.5].profile_precond(u_, reps=args.profile_reps)
            acc = m if acc is None else [x + y for x, y in zip(acc, m)]
        mp = [x / max(1, args.steps) for x in acc]
        bp = precond_bytes(2, N, nrhs, 4 if fp32 else 8)
        print(json.dumps({"roofline_only": True, "precision": "f32" if fp32 else "f64",
                          "ms_per_kernel": ms, "bytes_per_kernel": by,
                          "GBs": [b / (t * 1e-3) / 1e9 for b, t in zip(by, ms)],
                          "precond_ms_per_kernel": mp, "precond_bytes_per_kernel": bp,
                          "precond_GBs": [b / (t * 1e-3) / 1e9 for b, t in zip(bp, mp)],
                          "schedule": sched}))
        return

    def step(k):
        a = alphas[k % len(alphas)]
        _, info = ops[a].solve(rhs[a], tol=args.tol, mixed=mixed, out=out)
        return info

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    lat, infos = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        infos.append(step(k))
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    progress(f"headline: {args.steps * nrhs / total:.1f} solves/s")
    solves = args.steps * nrhs
    value = solves / total
    max_relres = max(i["relres_true"] for inf in infos for i in inf)
    iters = {alphas[k % 3]: [i["iters"] for i in infos[k]] for k in range(min(3, args.steps))}
    outers = {alphas[k % 3]: [i["outer_iters"] for i in infos[k]]
              for k in range(min(3, args.steps))}

    # FP64, one right-hand side at a time (the plain path), same operators
    fp64 = {}
    if args.fp64_single > 0:
        n1 = args.fp64_single
        tsum, cnt, it64 = 0.0, 0, {}
        for a in alphas:
            for j in range(n1):
                f1 = rhs[a][1 + j].contiguous()
                ops[a].solve(f1, tol=args.tol, mixed=False)  # warm
                torch.cuda.synchronize()
                ts = time.perf_counter()
                _, inf = ops[a].solve(f1, tol=args.tol, mixed=False)
                tsum += time.perf_counter() - ts
                cnt += 1
                it64.setdefault(a, []).append(inf[0]["iters"])
        fp64 = {"solves_per_s": cnt / tsum, "ms_per_solve": 1e3 * tsum / cnt,
                "iters": it64}
        # accuracy of the mixed path against the FP64 path (one RHS per alpha)
        diffs = []
        for a in alphas:
            f1 = rhs[a][1].contiguous()
            u64, _ = ops[a].solve(f1, tol=args.tol, mixed=False)
            umx, _ = ops[a].solve(f1, tol=args.tol, mixed=mixed or 1)
            diffs.append(float((umx - u64).abs().max() / u64.abs().max()))
        fp64["mixed_vs_fp64_rel_linf"] = max(diffs)

    # the mixed-precision path (FP32 CG, FP64 reliable updates) on the same batches
    # timed like the headline path: the same warm-up steps (every operator's
    # first mixed solve captures its graphs), then the same number of steps
    mixed_res = None
    msteps = args.steps if args.mixed_steps is None else args.mixed_steps
    if msteps > 0 and mixed != 1:
        def mstep(k):
            a = alphas[k % len(alphas)]
            return ops[a].solve(rhs[a], tol=args.tol, mixed=1, out=out)[1]
        for k in range(max(args.warmup, len(alphas))):
            mstep(k)
        torch.cuda.synchronize()
        mlat, minf = [], []
        t0m = time.perf_counter()
        for k in range(msteps):
            ts = time.perf_counter()
            minf.append(mstep(k))
            mlat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0m
        mixed_res = {"solves_per_s": msteps * nrhs / tm, "steps": msteps,
                     "p50_ms": float(np.percentile(np.array(mlat) * 1e3, 50)),
                     "p99_ms": float(np.percentile(np.array(mlat) * 1e3, 99)),
                     "max_relres_true": max(i["relres_true"] for inf in minf for i in inf),
                     "iters": {alphas[k % 3]: [i["iters"] for i in minf[k]]
                               for k in range(min(3, msteps))},
                     "outer_iters": {alphas[k % 3]: [i["outer_iters"] for i in minf[k]]
                                     for k in range(min(3, msteps))},
                     "vs_fp64_batched": msteps * nrhs / tm / value,
                     "path": "FP32 CG with FP64 reliable updates"}

    # roofline of the dominant kernel of the timed path: per-pass durations
    # (HIP events on the operator's stream, each pass back to back) of the
    # batched product in the timed precision, same operator and schedule
    a = 1.5
    names = ["axis0_fwd_r2c", "last_axis_fwd_symbol_inv", "axis0_inv_c2r"]

    def passes(fp32):
        u_ = rhs[a].to(torch.float32).contiguous() if fp32 else rhs[a]
        # mean over 5 measurements of `profile_reps` back-to-back launches (the
        # mean per dispatch, as a kernel trace's average reports it)
        runs = [ops[a].profile_apply(u_, reps=args.profile_reps) for _ in range(5)]
        ms_ = [float(np.mean([r[i] for r in runs])) for i in range(len(runs[0]))]
        by_ = pass_bytes(2, N, nrhs, 4 if fp32 else 8)
        fl_ = pass_flops(2, N, nrhs)
        return [{"kernel": nm, "ms": t, "bytes": b, "GBs": b / (t * 1e-3) / 1e9,
                 "flops": f, "TFLOPs": f / (t * 1e-3) / 1e12}
                for nm, t, b, f in zip(names, ms_, by_, fl_)]

    pk64, pk32 = passes(False), passes(True)
    progress("product passes timed")

    # the tau preconditioner's kernels (same operator, schedule and batch)
    pnames = ["tau_axis0_sine", "tau_last_axis_sine_mult_sine", "tau_axis0_sine_back"]

    def ppasses(fp32):
        u_ = rhs[a].to(torch.float32).contiguous() if fp32 else rhs[a]
        runs = [ops[a].profile_precond(u_, reps=args.profile_reps) for _ in range(5)]
        ms_ = [float(np.mean([r[i] for r in runs])) for i in range(len(runs[0]))]
        by_ = precond_bytes(2, N, nrhs, 4 if fp32 else 8)
        fl_ = precond_flops(2, N, nrhs)
        return [{"kernel": nm, "ms": t, "bytes": b, "GBs": b / (t * 1e-3) / 1e9,
                 "flops": f, "TFLOPs": f / (t * 1e-3) / 1e12}
                for nm, t, b, f in zip(pnames, ms_, by_, fl_)]

    pp64, pp32 = ppasses(False), ppasses(True)

    # a plain device copy of 4 GiB (read + write), HIP events on torch's stream
    src = torch.ones((4 << 30) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbs = 5 * 2 * (4 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    pk = pk32 if mixed else pk64
    dom = max(range(3), key=lambda i: pk[i]["ms"])
    kd = pk[dom]
    roof = {"bound": "hbm", "achieved": kd["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": kd["GBs"] / HBM_PEAK_GBS, "traffic": traffic_for(kd["kernel"], bool(mixed), nrhs),
            "kernel": kd["kernel"], "precision": "f32" if mixed else "f64", "nrhs": nrhs,
            "bytes_per_launch": kd["bytes"], "ms_per_launch": kd["ms"],
            "alu_TFLOPs": kd["TFLOPs"], "alu_peak_TFLOPs": VALU_PEAK_TFLOPS,
            "alu_frac": kd["TFLOPs"] / VALU_PEAK_TFLOPS,
            "copy_GBs": copy_gbs, "frac_of_copy": kd["GBs"] / copy_gbs,
            "per_kernel_f64": pk64, "per_kernel_f32": pk32,
            "matvec_ms_f64": sum(k["ms"] for k in pk64),
            "matvec_ms_f32": sum(k["ms"] for k in pk32),
            "precond_per_kernel_f64": pp64, "precond_per_kernel_f32": pp32,
            "precond_ms_f64": sum(k["ms"] for k in pp64),
            "precond_ms_f32": sum(k["ms"] for k in pp32),
            # time of each FP32 pass over its FP64 twin (0.5 = the byte ratio)
            "f32_over_f64": {k64["kernel"]: k32["ms"] / k64["ms"]
                             for k64, k32 in zip(pk64 + pp64, pk32 + pp32)}}

    configs = run_configs(dev, args.tol) if args.configs else None
    progress("configs done")
    d2 = d2_shapes(dev, reps=args.d2_reps) if args.d2 else None
    progress("large working sets done")

    serving = serving_legs(args)
    progress("serving done")

    cpu = None
    if args.cpu_budget > 0:
        cpu = cpu_baseline(N, p, 1.0, args.tol, args.cpu_budget)

    lat_ms = np.array(lat) * 1e3
    res = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": (f"2D fractional Poisson, {N - 1}^2 unknowns (N={N}, embedding "
                                f"{2 * N}^2), degree {p}, alpha cycling 0.5/1.0/1.5, "
                                f"{nrhs} RHS per batched solve, tol {args.tol:g}, "
                                + {0: "FP64 CG", 1: "FP32 CG with FP64 reliable updates",
                                   2: "FP32 inner CG + FP64 iterative refinement"}[mixed]),
                   "global_batch": nrhs, "grid": f"{N - 1}x{N - 1}", "degree": p,
                   "alphas": alphas, "tol": args.tol, "path": args.path},
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "latency_unit": "ms per batched solve (all RHS of the batch complete)",
        "max_relres_true": max_relres, "iters": iters, "outer_iters": outers,
        "setup_s": setup_s, "schedule": sched, "fp64_single": fp64, "mixed": mixed_res,
        "serving": serving, "configs": configs, "d2": d2,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
