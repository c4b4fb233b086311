"""Benchmark: -2logL evaluations per second on one MI355X.

Workload: n=4096 points in d=8 (Latin-hypercube-like design, smooth response
plus noise), p=1.95, nugget 1e-6, a batch of 128 thetas log-uniform on
[0.05, 20]^8.  One step = one gp_nll_batch call over the 128 thetas: the
whole hot path (correlation build, blocked Cholesky, log-determinant, solves
and reductions) with every input already resident in HBM.

Prints one JSON line.  `roofline` reports the dominant kernel (the FP64-MFMA
trailing SYRK/GEMM update): algorithmic FLOPs of its launches in the timed
steps over their summed HIP-event durations, recorded by the library on the
stream the kernels run on.  `cpu_baseline` times the plain C oracle (FP64,
one theta per thread) on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The request-server leg keeps up to 8 micro-batches in flight on as many
# streams, each with the library's two side streams; HIP maps a process's
# streams onto 4 hardware queues unless told otherwise (the usual environment
# says 4 explicitly), which serialises the excess.  At least 16, set before
# the HIP runtime starts (first device call).
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _hwq = 4
if _hwq < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "-2logL evals/sec at n=4096,d=8 (mixed vs FP64 GPU); p50/p99 request latency"
FP64_MFMA_PEAK = 78.6e12   # MI355X dense FP64 matrix peak, FLOP/s
HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
SYRK_SRC = os.path.join(ROOT, "paper_1203_1269_amd", "csrc", "chol.hip")

# HBM traffic of the rank-512 trailing update (syrk_update_kernel) on this
# workload, from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by
# what the same counters read for a 512 MiB device copy (bench.py
# --copy-calibration: FETCH_SIZE reads 0.5x the bytes copied, WRITE_SIZE 1.0x).
# Valid only for the kernel and launch loop it was taken on: reported as null
# once the sha256 of their source differs.
SYRK_TRAFFIC = {"kernel_sha256": "94579d149ba9a879048cbfe28f1b17c827a5963b4385b2c8d8b3d57c81dcade1",
                "bytes_per_launch": (2.0 * 4.80649e7 + 1.0 * 1.88089e7) / 13 * 1024}


def syrk_kernel_text():
    """Source of the trailing-update kernel and of the host loop that
    launches it (the launch shapes decide the per-launch traffic)."""
    with open(SYRK_SRC) as f:
        src = f.read()
    parts = [line for line in src.splitlines(keepends=True)
             if line.startswith(("#define SY_", "constexpr int SY_"))]
    for start in ("void syrk_update_kernel(", "void factor_batch("):
        i = src.index(start)
        parts.append(src[i:src.index("\n}\n", i) + 3])
    return "".join(parts)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision legs")
    ap.add_argument("--mixed-fast", action="store_true",
                    help="also run the FP32-update mixed mode (GP_MIXED_FAST; off by default: "
                         "at n=4096 it runs at 0.38x FP64, errors reported, not matched)")
    ap.add_argument("--no-mixed-fast", action="store_true",
                    help="leave out the FP32-update mixed mode (the default)")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-server leg")
    ap.add_argument("--no-large", action="store_true", help="skip the n=8192 leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient / L-BFGS leg")
    ap.add_argument("--no-predict", action="store_true", help="skip the prediction leg")
    ap.add_argument("--no-ga", action="store_true", help="skip the GA whole-fit leg")
    ap.add_argument("--no-conditioning", action="store_true",
                    help="skip the kappa_hat estimate of the benchmark thetas")
    ap.add_argument("--serving-requests", type=int, default=5000)
    ap.add_argument("--serving-arena-gb", type=float, default=16.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 512 MiB device-to-device copy first (counter calibration)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads (default: every core this process may run on)")
    ap.add_argument("--prof-steps", type=int, default=3,
                    help="instrumented steps (per-launch HIP events) after the timed ones")
    return ap.parse_args()


def cpu_baseline(w, threads):
    """Time the FP64 oracle on `threads` thetas of the same workload, one per
    thread (about 20-40 s of wall time at n=4096)."""
    import oracle
    oracle.build()
    th = w.theta[:threads]
    t0 = time.perf_counter()
    r = oracle.nll_batch(w.X, w.y, th, w.p, w.delta, nthreads=threads)
    dt = time.perf_counter() - t0
    assert (r.info == 0).all()
    return {"value": len(th) / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(th)} of the {w.B} thetas of the same n={w.n}, d={w.d} workload, "
                      f"one theta per thread, {dt:.1f} s wall"}


def cpu_lapack_baseline(w, threads, count=16):
    """Second CPU baseline: NumPy for R and SciPy/LAPACK (multi-threaded
    OpenBLAS on `threads` threads) for the Cholesky and the solves, one theta
    at a time; the theta-independent power terms are computed once for the
    sample and their time is included."""
    import numpy as np
    import scipy.linalg as sla
    from threadpoolctl import threadpool_limits
    th = w.theta[:count]
    n = w.n
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        D = np.empty((w.d, n, n))
        for k in range(w.d):
            np.power(np.abs(w.X[:, k, None] - w.X[None, :, k]), w.p, out=D[k])
        one = np.ones(n)
        nll = np.empty(len(th))
        for t in range(len(th)):
            R = np.exp(-np.tensordot(th[t], D, axes=1))
            R[np.diag_indices(n)] += w.delta
            L = sla.cholesky(R, lower=True, overwrite_a=True, check_finite=False)
            ab = sla.solve_triangular(L, np.stack([one, w.y], axis=1), lower=True,
                                      check_finite=False)
            a, b = ab[:, 0], ab[:, 1]
            mu = a @ b / (a @ a)
            Q = np.sum((b - mu * a) ** 2)
            nll[t] = 2 * np.sum(np.log(np.diag(L))) + n * np.log(Q / n)
        dt = time.perf_counter() - t0
    assert np.all(np.isfinite(nll))
    return {"value": len(th) / dt, "unit": "evals/s", "cores": threads, "kind": "lapack",
            "sample": f"{len(th)} of the {w.B} thetas of the same n={w.n}, d={w.d} workload, "
                      f"one theta at a time on {threads} BLAS threads, {dt:.1f} s wall"}


def syrk_traffic():
    import hashlib
    h = hashlib.sha256(syrk_kernel_text().encode()).hexdigest()
    if SYRK_TRAFFIC["kernel_sha256"] != h:
        return None
    return SYRK_TRAFFIC["bytes_per_launch"]


def conditioning(w, dev, chunk=32):
    """kappa_hat = (max_j L_jj / min_j L_jj)^2 of every theta of the workload
    (R from gp_corr_build, L from gp_cholesky_batch), in chunks of thetas."""
    import numpy as np
    import torch
    from paper_1203_1269_amd import binding
    ds = binding.Dataset(w.X, w.y, w.p, w.delta, device=dev)
    kap = []
    for c0 in range(0, w.B, chunk):
        R, info = binding.corr_build(ds, w.theta[c0:c0 + chunk])
        info2, _ = binding.cholesky_batch(R, w.n)
        dg = torch.diagonal(R, dim1=1, dim2=2)[:, :w.n]
        k = (dg.max(dim=1).values / dg.min(dim=1).values) ** 2
        k[(info != 0) | (info2 != 0)] = float("nan")
        kap.append(k.cpu().numpy())
        del R
    torch.cuda.empty_cache()
    kap = np.concatenate(kap)
    return {"kappa_hat_median": float(np.nanmedian(kap)), "kappa_hat_max": float(np.nanmax(kap)),
            "kappa_hat_over_1e8": int(np.sum(kap > 1e8))}


def multi_leg(args, dev, per=16):
    """The 64 serving datasets (uneven n and d), `per` thetas each, in one
    gp_nll_multi call per step; beside it the same work as one gp_nll_batch
    call per dataset on one stream."""
    import numpy as np
    import torch
    from paper_1203_1269_amd import binding, inputs
    sets = inputs.serving_datasets()
    ds = [binding.Dataset(s.X, s.y, s.p, s.delta, device=dev) for s in sets]
    rng = np.random.default_rng(9)
    th = [torch.as_tensor(inputs.log_uniform_theta(per, d.d, 0.05, 20.0, rng),
                          dtype=torch.float64, device=dev) for d in ds]
    ws = None
    binding.nll_multi(ds, th)
    torch.cuda.synchronize()
    steps = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = binding.nll_multi(ds, th)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ok = int(sum(int((r["info"] == 0).sum()) for r in res))
    wsb = max(binding.workspace_bytes(d.n, d.d, per) for d in ds)
    ws = binding.alloc_workspace(wsb, dev)
    t1 = time.perf_counter()
    for _ in range(steps):
        for d, t in zip(ds, th):
            binding.nll_batch(d, t, ws=ws)
    torch.cuda.synchronize()
    ds_ = (time.perf_counter() - t1) / steps
    del ws
    torch.cuda.empty_cache()
    total = per * len(ds)
    return {"datasets": len(ds), "thetas_per_dataset": per, "evaluations": total,
            "results_ok": ok, "ms_per_call": dt * 1e3, "evals_per_s": total / dt,
            "sequential_batches_ms": ds_ * 1e3, "sequential_evals_per_s": total / ds_}


def serving_leg(args, dev):
    """64 resident datasets (n uniform over multiples of 64 in [256, 6144],
    d in 2..12, p in {1.5, 1.95, 2}); for each form of micro-batch a
    closed-loop burst (one untimed pass, then two timed) measures the
    saturation throughput, then Poisson streams at 0.5x and 0.9x of it are replayed
    open-loop with per-request latency.  Forms: ragged (requests of up to 8 datasets of close orders in
    one ragged launch sequence), one dataset per micro-batch, and the latter
    launched as captured graphs (burst and 0.5x only)."""
    import numpy as np
    from paper_1203_1269_amd import binding, inputs, serving
    sets = inputs.serving_datasets()
    ds = [binding.Dataset(s.X, s.y, s.p, s.delta, device=dev) for s in sets]
    arena = int(args.serving_arena_gb * (1 << 30))
    N = args.serving_requests
    burst = inputs.serving_requests(sets, count=min(N, 1000), rate=1e9, seed=7)

    def run(fracs, **cfg):
        srv = serving.Server(ds, arena_bytes=arena, **cfg)
        # one untimed pass of the burst first (a new server's streams, their
        # side streams and staging buffers are set up on first use), then
        # two timed passes
        serving.replay(srv, [0.0] * len(burst), [r[2] for r in burst], [r[1] for r in burst])
        wall = 0.0
        for _ in range(2):
            wall += serving.replay(srv, [0.0] * len(burst), [r[2] for r in burst],
                                   [r[1] for r in burst])[3]
        sat = 2 * len(burst) / wall
        out = dict(cfg)
        out["saturation_evals_per_s"] = sat
        for frac in fracs:
            reqs = inputs.serving_requests(sets, count=N, rate=frac * sat, seed=8)
            lat, res, bsz, wall = serving.replay(srv, [r[0] for r in reqs], [r[2] for r in reqs],
                                                 [r[1] for r in reqs])
            summ = serving.latency_summary(lat, wall)
            summ["offered_rate"] = frac * sat
            summ["mean_batch"] = float(np.mean(bsz))
            summ["failed"] = int(sum(1 for r in res if r["info"] != 0))
            out[f"poisson_{frac}"] = summ
        srv.close()
        return out

    out = {"datasets": len(ds), "arena_gb": args.serving_arena_gb,
           "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")}
    out["ragged"] = run((0.5, 0.9), max_batch=128, nstreams=3, ragged=True)
    out["by_dataset"] = run((0.5, 0.9), max_batch=16, nstreams=8)
    out["by_dataset_graphs"] = run((0.5,), max_batch=16, nstreams=8, graphs=True)
    return out


PRECS = ("fp64", "mixed", "mixed_fast")


def time_batch(binding, torch, ds, theta, ws, prec, steps, warmup, profile=False):
    """`warmup` untimed then `steps` timed gp_nll_batch calls on the current
    stream; returns (seconds, per-kernel stats of the timed calls, results)."""
    B = theta.shape[0]
    out = torch.empty((B, 5), dtype=torch.float64, device=theta.device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        binding.nll_batch_raw(ds, theta, ws, out, prec=prec, stream=stream)
    torch.cuda.synchronize()
    if profile:   # the library records per-launch events on the same stream
        binding.profile_begin(max_launches=4000 * max(1, steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        binding.nll_batch_raw(ds, theta, ws, out, prec=prec, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kstats = binding.profile_end() if profile else {}
    res = {k: v.cpu().numpy().copy() for k, v in binding.unpack_results(out).items()}
    return dt, kstats, res


def rel_errs(res, ref, y):
    import numpy as np
    sc = {"logdet": 1.0, "nll": 1.0, "mu": float(np.std(y)), "sigma2": 0.0}
    ok = (res["info"] == 0) & (ref["info"] == 0)
    if not ok.any():
        return {k: None for k in sc}, ok
    return {k: float(np.max(np.abs(res[k][ok] - ref[k][ok]) /
                            np.maximum(np.abs(ref[k][ok]), sc[k]))) for k in sc}, ok


GOLDEN = os.path.join(ROOT, "tests", "golden")
FP64_FLOOR, MATCH_FLOOR = 1e-10, 1e-8


def load_golden(name):
    """Stored oracle values (80-bit and FP64 builds of the C oracle, LAPACK
    spread) for thetas of a full-size workload, written by
    tests/golden/make_expected.py; None when absent."""
    path = os.path.join(GOLDEN, f"{name}_expected.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def oracle_check(res, exp, y, floor):
    """Largest relative error per output against the stored 80-bit oracle
    values, and how many stored thetas lie within their bar
    max(floor, 10 x the FP64 rounding spread of that theta)."""
    import numpy as np
    if exp is None:
        return None
    sc = {"logdet": 1.0, "nll": 1.0, "mu": float(np.std(y)), "sigma2": 0.0}
    worst = {k: 0.0 for k in sc}
    n = within = 0
    for rec in exp["samples"]:
        t = rec["index"]
        n += 1
        ok = int(res["info"][t]) == rec["info"]
        if rec["info"] != 0:
            within += ok
            continue
        for k in sc:
            ref = rec["f80"][k]
            e = abs(float(res[k][t]) - ref) / max(abs(ref), sc[k])
            worst[k] = max(worst[k], e)
            tol = max(floor, 10 * max(rec["err64"][k], rec["err64_lapack"][k]))
            ok = ok and e <= tol
        within += ok
    return {"thetas": n, "max_rel_err": worst, "within_bar": within, "floor": floor}


def mixed_summary(prec, dt, kst, res, dt64, res64, w, steps, kst_steps=1):
    """A mixed mode's timing (dt over `steps` steps) against the FP64 path,
    its largest differences from the FP64 GPU results, and the kernel table
    of its instrumented pass (`kst` over `kst_steps` steps)."""
    errs, ok = rel_errs(res, res64, w.y)
    out = {"prec": prec, "value": w.B * steps / dt, "ms_per_step": dt / steps * 1e3,
           "speedup_vs_fp64": dt64 / dt, "max_rel_err_vs_fp64_gpu": errs,
           "results_ok": int((res["info"] == 0).sum()),
           "results_recomputed_fp64": int((res["ir_iters"] == -1).sum()),
           "matched_1e-8": bool(errs["nll"] is not None and errs["nll"] <= 1e-8 and ok.all()),
           "kernels_ms_per_step": {k: v["ms"] / kst_steps for k, v in kst.items()}}
    if prec == "mixed":
        # INT8 MFMA operations issued per FP64 product: one product per modulus
        from paper_1203_1269_amd import binding
        per = binding.header_constant("GP_MIXED_MODULI")
        sy = kst.get("syrk_update_crt", {"flops": 0.0, "ms": 1.0})
        out["int8_products_per_fp64_product"] = per
        out["trailing_update_fp64_equiv_tflops"] = sy["flops"] / (sy["ms"] * 1e-3) / 1e12
        out["trailing_update_int8_tops"] = per * sy["flops"] / (sy["ms"] * 1e-3) / 1e12
        out["trailing_update_frac_of_int8_peak"] = out["trailing_update_int8_tops"] / 5000.0
    else:
        sy = kst.get("syrk_update_f32", {"flops": 0.0, "ms": 1.0})
        out["trailing_update_tflops_fp32_mfma"] = sy["flops"] / (sy["ms"] * 1e-3) / 1e12
    return out


INT8_MFMA_PEAK = 5.0e15   # MI355X dense INT8 matrix peak, OP/s


def mixed_roofline(kst):
    """The matched mixed form's dominant kernel (the INT8 trailing update):
    INT8 operations it issues per launch (16 modular products of 2K
    operations per updated lower entry) over its event time, against the
    INT8 MFMA peak; the FP64-equivalent rate beside it."""
    if not kst or "syrk_update_crt" not in kst:
        return None
    sy = kst["syrk_update_crt"]
    ops = 16.0 * sy["flops"]
    achieved = ops / (sy["ms"] * 1e-3)
    return {"bound": "mfma", "kernel": "syrk_update_crt", "achieved": achieved / 1e12,
            "peak": INT8_MFMA_PEAK / 1e12, "unit": "TOP/s", "frac": achieved / INT8_MFMA_PEAK,
            "fp64_equivalent_tflops": sy["flops"] / (sy["ms"] * 1e-3) / 1e12,
            "launches": sy["launches"], "traffic": None}


def large_leg(args, dev):
    """n=8192, d=10, p=2, 32 thetas: FP64 and matched-accuracy mixed (and, with
    --mixed-fast, the FP32 mode), each against the stored oracle values of this
    workload."""
    import torch
    from paper_1203_1269_amd import binding, inputs
    w = inputs.mixed_at_scale()
    ds = binding.Dataset(w.X, w.y, w.p, w.delta, device=dev)
    theta = torch.as_tensor(w.theta, dtype=torch.float64, device=dev).contiguous()
    ws = binding.alloc_workspace(max(binding.workspace_bytes(w.n, w.d, w.B, p) for p in PRECS), dev)
    steps = max(1, args.steps // 3)
    gold = load_golden(w.name)
    dt64, _, r64 = time_batch(binding, torch, ds, theta, ws, "fp64", steps, 1)
    _, k64, _ = time_batch(binding, torch, ds, theta, ws, "fp64", 1, 0, profile=True)
    dtm, _, rm = time_batch(binding, torch, ds, theta, ws, "mixed", steps, 1)
    _, km, _ = time_batch(binding, torch, ds, theta, ws, "mixed", 1, 0, profile=True)
    fast = args.mixed_fast and not args.no_mixed_fast
    if fast:
        dtf, _, rf = time_batch(binding, torch, ds, theta, ws, "mixed_fast", 1, 1)
    del ws
    torch.cuda.empty_cache()
    sy = k64["syrk_update"]
    out = {"workload": w.name, "n": w.n, "d": w.d, "batch": w.B, "p": w.p, "delta": w.delta,
           "steps": steps, "fp64_evals_per_s": w.B * steps / dt64,
           "fp64_syrk_update_frac_of_peak": sy["flops"] / (sy["ms"] * 1e-3) / FP64_MFMA_PEAK,
           "fp64_factorization_frac_of_peak": w.n ** 3 / 3.0 * w.B * steps / dt64 / FP64_MFMA_PEAK,
           "fp64_results_ok": int((r64["info"] == 0).sum()),
           "fp64_vs_oracle": oracle_check(r64, gold, w.y, FP64_FLOOR),
           "mixed": mixed_summary("mixed", dtm, km, rm, dt64, r64, w, steps)}
    out["mixed"]["vs_oracle"] = oracle_check(rm, gold, w.y, MATCH_FLOOR)
    if fast:
        out["mixed_fast"] = mixed_summary("mixed_fast", dtf * steps, {}, rf, dt64, r64, w, steps)
        out["mixed_fast"]["vs_oracle"] = oracle_check(rf, gold, w.y, MATCH_FLOOR)
    return out


def gradient_leg(args, dev):
    """n=4096, d=6, p=2, 16 thetas: value + adjoint gradient per call
    (bordered factorisation), and 16 multi-start L-BFGS fits x 50 iterations."""
    import numpy as np
    import torch
    from paper_1203_1269_amd import binding, inputs, optim
    w = inputs.gradient_workload()
    ds = binding.Dataset(w.X, w.y, w.p, w.delta, device=dev)
    theta = torch.as_tensor(w.theta, dtype=torch.float64, device=dev).contiguous()
    ws = binding.alloc_workspace(binding.grad_workspace_bytes(w.n, w.d, w.B), dev)
    binding.nll_grad(ds, theta, ws)
    torch.cuda.synchronize()
    steps = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        res, g = binding.nll_grad(ds, theta, ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del ws
    torch.cuda.empty_cache()
    t1 = time.perf_counter()
    fit = optim.lbfgs_multistart(ds, w.theta, iters=50)
    torch.cuda.synchronize()
    dfit = time.perf_counter() - t1
    return {"workload": w.name, "n": w.n, "d": w.d, "batch": w.B,
            "value_and_grad_per_s": w.B * steps / dt, "ms_per_call": dt / steps * 1e3,
            "lbfgs_starts": int(w.B), "lbfgs_iters_max": 50, "lbfgs_seconds": dfit,
            "lbfgs_batched_calls": int(fit.evaluations), "lbfgs_best_nll": float(np.min(fit.nll))}


def prediction_leg(args, dev):
    """Fit + predict at a 1000-point test set (n=4096, d=8, 8 thetas in one
    call), with the SSPE of each fitted theta against the noiseless response;
    the same thetas through gp_nll_batch alone for the cost of the fit."""
    import numpy as np
    import torch
    from paper_1203_1269_amd import binding, inputs
    w = inputs.prediction_workload()
    ds = binding.Dataset(w.X, w.y, w.p, w.delta, device=dev)
    theta = torch.as_tensor(w.theta, dtype=torch.float64, device=dev).contiguous()
    Xs = torch.as_tensor(w.Xs, dtype=torch.float64, device=dev).contiguous()
    B, N = w.theta.shape[0], w.Xs.shape[0]
    ws = binding.alloc_workspace(binding.predict_workspace_bytes(ds.n, ds.d, B, N), dev)
    binding.predict(ds, theta, Xs, ws)
    torch.cuda.synchronize()
    steps = max(1, args.steps // 2)
    binding.profile_begin(max_launches=4000 * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fit, mean, mse = binding.predict(ds, theta, Xs, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kst = binding.profile_end()
    t1 = time.perf_counter()
    for _ in range(steps):
        binding.nll_batch(ds, theta, ws=ws)
    torch.cuda.synchronize()
    dfit = (time.perf_counter() - t1) / steps
    sspe = ((mean.cpu().numpy() - w.ys[None, :]) ** 2).sum(axis=1)
    nll = fit["nll"].cpu().numpy()
    best = int(np.nanargmin(nll))
    del ws
    torch.cuda.empty_cache()
    return {"workload": "pred_n4096_d8", "n": ds.n, "d": ds.d, "batch": B, "test_points": N,
            "p": w.p, "delta": w.delta, "ms_per_call": dt * 1e3,
            "predictions_per_s": B * N / dt, "fits_with_prediction_per_s": B / dt,
            "ms_fit_alone": dfit * 1e3,
            "sspe_best_nll_theta": float(sspe[best]), "sspe_median": float(np.median(sspe)),
            "mse_mean_best_nll_theta": float(mse[best].mean().item()),
            "kernels": {k: {"ms_per_call": v["ms"] / steps,
                            "gbyte_per_s": v["bytes"] / (v["ms"] * 1e-3) / 1e9,
                            "tflop_per_s": v["flops"] / (v["ms"] * 1e-3) / 1e12}
                        for k, v in kst.items() if v["ms"] > 0}}


# whole-fit wall times (s) the paper reports (10-replication averages; the
# CPU n=4064 fit ran once): Table 1 (d=2) and Table 2 (d=6), CPU and CUDA
PAPER_FIT_SECONDS = {
    (16, 2): (0.91, 2.26), (32, 2): (3.30, 4.94), (64, 2): (12.90, 5.50),
    (128, 2): (51.45, 7.25), (256, 2): (206.18, 9.88), (512, 2): (911.93, 20.75),
    (64, 6): (32.32, 9.45), (256, 6): (514.43, 16.58), (1024, 6): (13325.86, 96.19),
    (4064, 6): (161925.05, 1059.71),
}


def ga_leg(args, dev, reps=3):
    """Whole GP fits at the shapes of the paper's two examples: a genetic
    algorithm with population 100 over 20 generations (2000 -2logL
    evaluations, one gp_nll_batch call per generation), then prediction at a
    1000-point test set with the best theta; p = 1.95, no nugget, synthetic
    LHS-like designs with a noiseless sine response, `reps` replications."""
    import numpy as np
    import torch
    from paper_1203_1269_amd import binding, ga, inputs
    out = {}
    warm = inputs.ga_workload(64, 2, seed=99)
    ga.fit_ga(binding.Dataset(warm.X, warm.y, warm.p, warm.delta, device=dev), seed=0)
    for (n, d), (cpu_s, cuda_s) in PAPER_FIT_SECONDS.items():
        secs, nll, sspe, infeasible = [], [], [], []
        for r in range(reps):
            w = inputs.ga_workload(n, d, seed=1000 * d + n + r)
            ds = binding.Dataset(w.X, w.y, w.p, w.delta, device=dev)
            Xs = torch.as_tensor(w.Xs, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fit = ga.fit_ga(ds, seed=r, keep_history=True)
            _, mean, _ = binding.predict(ds, fit.theta[None, :], Xs)
            m = mean[0].cpu().numpy()
            secs.append(time.perf_counter() - t0)
            nll.append(fit.nll)
            sspe.append(float(((m - w.ys) ** 2).sum()))
            infeasible.append(int(sum(int(np.isinf(v).sum()) for v in fit.all_values)))
            del ds, Xs
        t = float(np.mean(secs))
        out[f"n{n}_d{d}"] = {
            "fit_seconds": t, "evals_per_s": 2000 / t, "best_nll_mean": float(np.mean(nll)),
            "best_nll_plus_n_ln_n_mean": float(np.mean(nll) + n * np.log(n)),
            "sspe_median": float(np.median(sspe)),
            "failed_evaluations_mean": float(np.mean(infeasible)),
            "paper_cpu_fit_seconds": cpu_s, "paper_cuda_fit_seconds": cuda_s,
            "ratio_vs_paper_cuda_fit": cuda_s / t}
    torch.cuda.empty_cache()
    return {"replications": reps, "population": 100, "generations": 20, "fits": out}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every evaluation is "
              "independent, so more GPUs would split the theta batch (not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1203_1269_amd import binding, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.fp64_at_scale(n=args.n, B=args.batch)
    ds = binding.Dataset(w.X, w.y, w.p, w.delta, device=dev)
    theta = torch.as_tensor(w.theta, dtype=torch.float64, device=dev).contiguous()
    fast = args.mixed_fast and not args.no_mixed_fast
    precs = ("fp64",) if args.no_mixed else (PRECS if fast else ("fp64", "mixed"))
    ws = binding.alloc_workspace(max(binding.workspace_bytes(w.n, w.d, w.B, p) for p in precs), dev)

    runs = {}
    for prec in reversed(precs):   # FP64 last
        # the FP32 mode is reported for its errors, not timed at length
        steps = args.steps if prec != "mixed_fast" else max(1, args.steps // 4)
        runs[prec] = time_batch(binding, torch, ds, theta, ws, prec, steps, args.warmup)
    # an instrumented pass after the timed steps: the library records HIP
    # events around every launch on the stream it runs on; these give the
    # per-kernel table and the roofline (the timed steps above run without)
    prof = {}
    for prec in precs:
        if prec != "mixed_fast":
            _, prof[prec], _ = time_batch(binding, torch, ds, theta, ws, prec, args.prof_steps, 0,
                                          profile=True)
    dt, _, res64 = runs["fp64"]
    kstats = prof["fp64"]
    gold = load_golden(w.name) if (args.n == 4096 and args.batch == 128) else None
    mixed = {}
    for p in precs:
        if p == "fp64":
            continue
        dtp, _, resp = runs[p]
        steps = args.steps if p != "mixed_fast" else max(1, args.steps // 4)
        mixed[p] = mixed_summary(p, dtp * args.steps / steps, prof.get(p, {}), resp, dt, res64, w,
                                 args.steps, args.prof_steps)
        mixed[p]["vs_oracle"] = oracle_check(resp, gold, w.y, MATCH_FLOOR)
        if p == "mixed" and mixed[p]["vs_oracle"] is not None:
            vo = mixed[p]["vs_oracle"]
            mixed[p]["matched_1e-8_vs_oracle"] = vo["within_bar"] == vo["thetas"]
    oracle64 = oracle_check(res64, gold, w.y, FP64_FLOOR)

    n_ok = int((res64["info"] == 0).sum())
    evals = w.B * args.steps / dt
    ms_step = dt / args.steps * 1e3

    sy = kstats["syrk_update"]
    achieved = sy["flops"] / (sy["ms"] * 1e-3)
    factor_flops = w.n ** 3 / 3.0
    # per kernel (instrumented pass): event time per step, algorithmic FLOPs
    # and bytes per step, and the rates they imply (bytes against the 8 TB/s
    # HBM peak); kernels of the factorisation overlap each other
    # (lookahead), so their event times include that sharing
    ps = args.prof_steps
    kernels = {k: {"ms_per_step": v["ms"] / ps, "launches_per_step": v["launches"] / ps,
                   "gflop_per_step": v["flops"] / ps / 1e9,
                   "gbyte_per_step": v["bytes"] / ps / 1e9,
                   "tflop_per_s": v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else None,
                   "gbyte_per_s": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None}
               for k, v in kstats.items()}
    mx = mixed.get("mixed")
    line = {
        "metric": METRIC,
        "value": evals,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "batch": w.B, "p": w.p,
                   "delta": w.delta, "prec": "fp64", "seed": w.seed},
        "mixed_value": mx["value"] if mx else None,
        "mixed_vs_fp64": mx["speedup_vs_fp64"] if mx else None,
        "oracle_fp64": oracle64,
        "oracle_mixed": mx["vs_oracle"] if mx else None,
        "roofline": {"bound": "mfma", "kernel": "syrk_update", "achieved": achieved / 1e12,
                     "peak": FP64_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK, "traffic": syrk_traffic(),
                     "traffic_unit": "bytes per launch",
                     "measured": f"HIP events around each launch, {ps} instrumented steps after "
                                 "the timed ones"},
        "roofline_mixed": mixed_roofline(prof.get("mixed")),
        "factorization_frac_of_fp64_peak": factor_flops * evals / FP64_MFMA_PEAK,
        "results_ok": n_ok,
        "kernels": kernels,
    }
    line.update(mixed)
    del ws
    torch.cuda.empty_cache()
    if not args.no_conditioning:
        line["conditioning"] = conditioning(w, dev)
    if not args.no_large:
        line["large_n8192"] = large_leg(args, dev)
    if not args.no_grad:
        line["gradient"] = gradient_leg(args, dev)
    if not args.no_predict:
        line["prediction"] = prediction_leg(args, dev)
    if not args.no_ga:
        line["ga_fit"] = ga_leg(args, dev)
    if not args.no_serving:
        line["multi_dataset"] = multi_leg(args, dev)
        line["serving"] = serving_leg(args, dev)
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or len(os.sched_getaffinity(0))
        line["cpu_baseline"] = cpu_baseline(w, threads)
        line["cpu_baseline"]["nproc"] = os.cpu_count()
        line["cpu_lapack"] = cpu_lapack_baseline(w, threads)
    # the headline comparison again at the end of the line, where a
    # truncated capture of the output still shows it
    line["summary"] = {
        "fp64_evals_per_s": evals,
        "mixed_evals_per_s": mx["value"] if mx else None,
        "mixed_vs_fp64": mx["speedup_vs_fp64"] if mx else None,
        "fp64_max_rel_err_vs_oracle": oracle64["max_rel_err"] if oracle64 else None,
        "mixed_max_rel_err_vs_oracle": (mx["vs_oracle"] or {}).get("max_rel_err") if mx else None,
        "mixed_matched_1e-8_vs_oracle": mx.get("matched_1e-8_vs_oracle") if mx else None,
        "n8192_mixed_vs_fp64": (line.get("large_n8192") or {}).get("mixed", {}).get(
            "speedup_vs_fp64"),
    }
    sv = line.get("serving")
    if sv:
        for form in ("ragged", "by_dataset"):
            f = sv[form]
            line["summary"][f"serving_{form}"] = {
                "saturation_evals_per_s": f["saturation_evals_per_s"],
                "p50_ms_at_0.9": f["poisson_0.9"]["p50_ms"],
                "p99_ms_at_0.9": f["poisson_0.9"]["p99_ms"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
