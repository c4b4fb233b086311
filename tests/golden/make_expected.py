"""Write oracle values for sampled thetas of the full-size workloads.

Calls only the CPU oracle (80-bit and FP64 builds, plus LAPACK on the
oracle's R to measure the FP64 rounding spread) on the seeded inputs of
paper_1203_1269_amd.inputs; the GPU path is not involved.  Usage:
    python tests/golden/make_expected.py fp64_n4096_d8 all
    python tests/golden/make_expected.py mixed_n8192_d10 all
    python tests/golden/make_expected.py grad_n4096_d6 all
    python tests/golden/make_expected.py pred_n4096_d8 2
("all": every theta of the workload; a number k: k sampled thetas.)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1203_1269_amd import inputs  # noqa: E402

sys.path.insert(0, os.path.dirname(HERE))
from parity_util import lapack_fp64, lapack_predict  # noqa: E402

WORKLOADS = {
    "fp64_n4096_d8": inputs.fp64_at_scale,
    "mixed_n8192_d10": inputs.mixed_at_scale,
    "grad_n4096_d6": inputs.gradient_workload,
}


def sample_indices(theta, k):
    """The theta with the smallest and the largest norm plus evenly spaced
    others; every theta when k covers the batch."""
    if k >= theta.shape[0]:
        return list(range(theta.shape[0]))
    norms = np.linalg.norm(np.log(theta), axis=1)
    idx = {int(np.argmin(np.sum(theta, axis=1))), int(np.argmax(np.sum(theta, axis=1)))}
    for q in np.linspace(0, theta.shape[0] - 1, k):
        if len(idx) >= k:
            break
        idx.add(int(q))
    _ = norms
    return sorted(idx)


def main_grad(name, k=2):
    """Oracle gradients (FP64 and 80-bit builds) for k sampled thetas."""
    w = WORKLOADS[name]()
    idx = sample_indices(w.theta, k)
    t0 = time.time()
    th = w.theta[idx]
    _, g64 = oracle.grad_batch(w.X, w.y, th, w.p, w.delta)
    _, g80 = oracle.grad_batch(w.X, w.y, th, w.p, w.delta, extended=True)
    samples = [{"index": t, "theta": th[q].tolist(), "grad_f64": g64[q].tolist(),
                "grad_f80": g80[q].tolist()} for q, t in enumerate(idx)]
    out = {"workload": name, "seed": w.seed, "n": w.n, "d": w.d, "p": w.p, "delta": w.delta,
           "samples": samples, "oracle_seconds": time.time() - t0}
    path = os.path.join(HERE, f"{name}_expected.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"])


def main_pred(name, k=2, points=16):
    """Oracle predictions (80-bit and FP64 builds, plus the LAPACK predictor)
    at `points` evenly spaced test points for k sampled thetas of the
    prediction workload."""
    w = inputs.prediction_workload()
    idx = sample_indices(w.theta, k)
    pts = np.unique(np.linspace(0, w.Xs.shape[0] - 1, points).astype(int))
    Xs = w.Xs[pts]
    t0 = time.time()
    samples = []
    for t in idx:
        m80, v80, f80 = oracle.predict(w.X, w.y, w.theta[t], w.p, w.delta, Xs, extended=True)
        m64, v64, _ = oracle.predict(w.X, w.y, w.theta[t], w.p, w.delta, Xs)
        ml, vl = lapack_predict(w.X, w.y, w.theta[t], w.p, w.delta, Xs)
        samples.append({"index": int(t), "theta": w.theta[t].tolist(), "points": pts.tolist(),
                        "sigma2_f80": float(f80.sigma2[0]), "mean_f80": m80.tolist(),
                        "mse_f80": v80.tolist(), "mean_f64": m64.tolist(),
                        "mse_f64": v64.tolist(), "mean_lapack": ml.tolist(),
                        "mse_lapack": vl.tolist()})
    out = {"workload": name, "n": w.X.shape[0], "d": w.X.shape[1], "B": w.theta.shape[0],
           "N": w.Xs.shape[0], "p": w.p, "delta": w.delta, "samples": samples,
           "oracle_seconds": time.time() - t0}
    path = os.path.join(HERE, f"{name}_expected.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"])


def main(name, k=4):
    if name.startswith("grad_"):
        return main_grad(name, k)
    if name.startswith("pred_"):
        return main_pred(name, k)
    w = WORKLOADS[name]()
    idx = sample_indices(w.theta, k)
    t0 = time.time()
    th = w.theta[idx]
    r64 = oracle.nll_batch(w.X, w.y, th, w.p, w.delta)
    r80 = oracle.nll_batch(w.X, w.y, th, w.p, w.delta, extended=True)
    lap = lapack_fp64(w.X, w.y, th, w.p, w.delta)
    sc = {"logdet": 1.0, "nll": 1.0, "mu": float(np.std(w.y)), "sigma2": 0.0}
    samples = []
    for q, t in enumerate(idx):
        rec = {"index": t, "theta": th[q].tolist(), "info": int(r80.info[q]), "f80": {}, "f64": {},
               "err64": {}, "err64_lapack": {}}
        for key in ("logdet", "mu", "sigma2", "nll"):
            a, b = float(getattr(r64, key)[q]), float(getattr(r80, key)[q])
            rec["f80"][key] = b
            rec["f64"][key] = a
            rec["err64"][key] = abs(a - b) / max(abs(b), sc[key])
            rec["err64_lapack"][key] = abs(float(lap[key][q]) - b) / max(abs(b), sc[key])
        samples.append(rec)
    out = {"workload": name, "seed": w.seed, "n": w.n, "d": w.d, "B": w.B, "p": w.p,
           "delta": w.delta, "samples": samples, "oracle_seconds": time.time() - t0}
    path = os.path.join(HERE, f"{name}_expected.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["oracle_seconds"])


if __name__ == "__main__":
    arg = sys.argv[2] if len(sys.argv) > 2 else "4"
    main(sys.argv[1], 1 << 30 if arg == "all" else int(arg))
