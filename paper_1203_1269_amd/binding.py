"""ctypes binding of libgpnll.so (argument marshalling only).

Every step of the likelihood runs inside the HIP library; this module only
turns torch device tensors into pointers, sizes the workspace and unpacks the
result records.  It fails loudly when the library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GPNLL_LIB") or os.path.join(HERE, "libgpnll.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gpnll.h")

GP_OK, GP_EINVAL, GP_EWORKSPACE, GP_ELAUNCH = 0, -1, -2, -3
PRECISIONS = {"fp64": 0, "mixed": 1, "mixed_fast": 2}
STATUS_NAMES = {0: "GP_OK", -1: "GP_EINVAL", -2: "GP_EWORKSPACE", -3: "GP_ELAUNCH"}


class GPResult(ctypes.Structure):
    _fields_ = [("logdet", ctypes.c_double), ("mu", ctypes.c_double),
                ("sigma2", ctypes.c_double), ("nll", ctypes.c_double),
                ("info", ctypes.c_int32), ("ir_iters", ctypes.c_int32)]


class GPDataset(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("d", ctypes.c_int32), ("p", ctypes.c_double), ("delta", ctypes.c_double),
                ("corr", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# gp_corr: correlation families
CORR = {"powexp": 0, "matern32": 1, "matern52": 2}


class GPKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("ms", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


RESULT_BYTES = ctypes.sizeof(GPResult)
assert RESULT_BYTES == 40


def header_constant(name: str) -> int:
    m = re.search(rf"#define\s+{name}\s+(\d+)", open(HEADER).read())
    return int(m.group(1))


def header_constant_expr(name: str) -> int:
    """A header constant written as a number or as (a << b), with an optional
    u suffix."""
    m = re.search(rf"#define\s+{name}\s+\(?\s*(\d+)u?\s*(?:<<\s*(\d+))?\s*\)?", open(HEADER).read())
    return int(m.group(1)) << int(m.group(2) or 0)


class GPError(RuntimeError):
    pass


class GPLbfgsConfig(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("m", ctypes.c_int32), ("max_ls", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("c1", ctypes.c_double), ("gtol", ctypes.c_double),
                ("theta_lo", ctypes.c_double), ("theta_hi", ctypes.c_double)]


class GPLbfgsSummary(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("evaluations", ctypes.c_int32)]


_lib = None


def lib():
    """Load libgpnll.so (built in-tree by paper_1203_1269_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1203_1269_amd/build.py "
                              "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        L.gp_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.gp_workspace_bytes.restype = sz
        L.gp_nll_batch.argtypes = [ctypes.POINTER(GPDataset), i32, vp, i32, vp, sz, vp, vp]
        L.gp_nll_batch.restype = ctypes.c_int
        L.gp_nll.argtypes = [ctypes.POINTER(GPDataset), vp, i32, vp, sz, vp, vp]
        L.gp_nll.restype = ctypes.c_int
        L.gp_corr_build.argtypes = [ctypes.POINTER(GPDataset), i32, vp, vp, i32, vp, vp]
        L.gp_corr_build.restype = ctypes.c_int
        L.gp_cholesky_ws_bytes.argtypes = [i32, i32]
        L.gp_cholesky_ws_bytes.restype = sz
        L.gp_cholesky_batch.argtypes = [i32, i32, vp, i32, vp, vp, vp, sz, vp]
        L.gp_cholesky_batch.restype = ctypes.c_int
        L.gp_grad_workspace_bytes.argtypes = [i32, i32, i32]
        L.gp_grad_workspace_bytes.restype = sz
        L.gp_nll_grad.argtypes = [ctypes.POINTER(GPDataset), i32, vp, i32, vp, sz, vp, vp, vp]
        L.gp_nll_grad.restype = ctypes.c_int
        L.gp_multi_workspace_bytes.argtypes = [ctypes.POINTER(GPDataset), i32, vp, i32]
        L.gp_multi_workspace_bytes.restype = sz
        L.gp_nll_multi.argtypes = [ctypes.POINTER(GPDataset), i32, vp, vp, i32, vp, sz, vp, vp]
        L.gp_nll_multi.restype = ctypes.c_int
        L.gp_predict_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.gp_predict_workspace_bytes.restype = sz
        L.gp_predict.argtypes = [ctypes.POINTER(GPDataset), i32, vp, vp, i32, i32, vp, sz, vp, vp,
                                 vp, vp]
        L.gp_predict.restype = ctypes.c_int
        L.gp_lbfgs_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.gp_lbfgs_workspace_bytes.restype = sz
        L.gp_lbfgs.argtypes = [ctypes.POINTER(GPDataset), i32, vp, ctypes.POINTER(GPLbfgsConfig),
                               vp, sz, vp, vp, vp, vp, ctypes.POINTER(GPLbfgsSummary), vp]
        L.gp_lbfgs.restype = ctypes.c_int
        L.gp_profile_begin.argtypes = [i32]
        L.gp_profile_begin.restype = ctypes.c_int
        L.gp_profile_end.argtypes = [ctypes.POINTER(GPKernelStat), i32]
        L.gp_profile_end.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != GP_OK:
        raise GPError(f"{what} returned {STATUS_NAMES.get(status, status)}")


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, device):
    t = torch.as_tensor(t, dtype=torch.float64)
    return t.to(device).contiguous()


def pad64(n: int) -> int:
    return (n + 63) // 64 * 64


class Dataset:
    """A dataset resident on the GPU: X (n x d, row-major) and y, plus p, delta
    and the correlation family ("powexp", "matern32", "matern52")."""

    def __init__(self, X, y, p: float, delta: float, device="cuda", corr: str = "powexp"):
        if corr not in CORR:
            raise ValueError(f"unknown correlation family {corr!r}")
        self.X = _dev_f64(X, device)
        self.y = _dev_f64(y, device).reshape(-1)
        self.n, self.d = self.X.shape
        self.p = float(p)
        self.delta = float(delta)
        self.corr = corr
        self.device = self.X.device
        self._c = GPDataset(self.X.data_ptr(), self.y.data_ptr(), self.n, self.d, self.p, self.delta,
                            CORR[corr], 0)

    @property
    def c(self):
        return ctypes.byref(self._c)


def workspace_bytes(n: int, d: int, batch: int, prec: str = "fp64") -> int:
    return int(lib().gp_workspace_bytes(n, d, batch, PRECISIONS[prec]))


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def unpack_results(raw: torch.Tensor):
    """raw: (B, 5) float64 device tensor holding gp_result records."""
    f = raw[:, :4]
    B = raw.shape[0]
    ints = raw.contiguous().reshape(-1).view(torch.int32).reshape(B, 10)[:, 8:10]
    return {"logdet": f[:, 0], "mu": f[:, 1], "sigma2": f[:, 2], "nll": f[:, 3],
            "info": ints[:, 0], "ir_iters": ints[:, 1]}


def nll_batch_raw(ds: Dataset, theta: torch.Tensor, ws: torch.Tensor, out: torch.Tensor,
                  prec: str = "fp64", stream=None) -> None:
    """gp_nll_batch on preallocated device buffers (no allocation, async)."""
    B = theta.shape[0]
    st = lib().gp_nll_batch(ds.c, B, ctypes.c_void_p(theta.data_ptr()), PRECISIONS[prec],
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _check(st, "gp_nll_batch")


def nll_batch(ds: Dataset, theta, prec: str = "fp64", ws: torch.Tensor | None = None):
    """Profile likelihood for each row of theta (B x d). Returns a dict of
    device tensors: logdet, mu, sigma2, nll (float64), info, ir_iters (int32)."""
    th = _dev_f64(theta, ds.device).reshape(-1, ds.d)
    B = th.shape[0]
    need = workspace_bytes(ds.n, ds.d, B, prec)
    if need == 0:
        raise GPError("gp_workspace_bytes rejected the sizes")
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, ds.device)
    out = torch.empty((B, 5), dtype=torch.float64, device=ds.device)
    nll_batch_raw(ds, th, ws, out, prec)
    return unpack_results(out)


def nll(ds: Dataset, theta, prec: str = "fp64"):
    th = _dev_f64(theta, ds.device).reshape(1, ds.d)
    need = workspace_bytes(ds.n, ds.d, 1, prec)
    ws = alloc_workspace(need, ds.device)
    out = torch.empty((1, 5), dtype=torch.float64, device=ds.device)
    st = lib().gp_nll(ds.c, ctypes.c_void_p(th.data_ptr()), PRECISIONS[prec],
                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out.data_ptr()),
                      _stream_ptr())
    _check(st, "gp_nll")
    return unpack_results(out)


def corr_build(ds: Dataset, theta):
    """R_delta for each theta: returns (R (B x np x np, column-major per matrix,
    i.e. R[b].T is the matrix in row-major view), info)."""
    th = _dev_f64(theta, ds.device).reshape(-1, ds.d)
    B = th.shape[0]
    np_ = pad64(ds.n)
    R = torch.zeros((B, np_, np_), dtype=torch.float64, device=ds.device)
    info = torch.empty(B, dtype=torch.int32, device=ds.device)
    st = lib().gp_corr_build(ds.c, B, ctypes.c_void_p(th.data_ptr()), ctypes.c_void_p(R.data_ptr()),
                             np_, ctypes.c_void_p(info.data_ptr()), _stream_ptr())
    _check(st, "gp_corr_build")
    return R, info


def cholesky_batch(A: torch.Tensor, n: int):
    """In-place blocked Cholesky of A (B x lda x lda, each matrix stored
    column-major, i.e. A[b].T in row-major view). Returns (info, logdet)."""
    B, lda, lda2 = A.shape
    assert lda == lda2 and A.dtype == torch.float64 and A.is_contiguous()
    info = torch.zeros(B, dtype=torch.int32, device=A.device)
    logdet = torch.empty(B, dtype=torch.float64, device=A.device)
    need = int(lib().gp_cholesky_ws_bytes(n, B))
    ws = alloc_workspace(need, A.device)
    st = lib().gp_cholesky_batch(n, B, ctypes.c_void_p(A.data_ptr()), lda,
                                 ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(logdet.data_ptr()),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr())
    _check(st, "gp_cholesky_batch")
    return info, logdet


def profile_begin(max_launches: int = 100000) -> None:
    """Start per-launch event timing inside the library."""
    _check(lib().gp_profile_begin(max_launches), "gp_profile_begin")


def profile_end() -> dict:
    """Stop timing; returns {kernel: {launches, ms, flops, bytes}} (waits for
    the recorded events)."""
    stats = (GPKernelStat * 32)()
    m = lib().gp_profile_end(stats, 32)
    if m < 0:
        _check(m, "gp_profile_end")
    return {stats[q].name.decode(): {"launches": stats[q].launches, "ms": stats[q].ms,
                                     "flops": stats[q].flops, "bytes": stats[q].bytes}
            for q in range(m)}


def grad_workspace_bytes(n: int, d: int, batch: int) -> int:
    return int(lib().gp_grad_workspace_bytes(n, d, batch))


def nll_multi(datasets, thetas, prec: str = "fp64", ws: torch.Tensor | None = None):
    """Uneven-n batching in one call (gp_nll_multi): thetas[k] (B_k x d_k)
    for datasets[k].  Returns a list of result dicts (device tensors), one
    per dataset, as nll_batch."""
    nds = len(datasets)
    assert nds == len(thetas) and nds > 0
    dev = datasets[0].device
    blocks = [_dev_f64(t, dev).reshape(-1, ds.d) for ds, t in zip(datasets, thetas)]
    counts = (ctypes.c_int32 * nds)(*[b.shape[0] for b in blocks])
    arr = (GPDataset * nds)(*[ds._c for ds in datasets])
    th = torch.cat([b.reshape(-1) for b in blocks]) if blocks else torch.empty(0)
    th = th.contiguous()
    need = int(lib().gp_multi_workspace_bytes(arr, nds, ctypes.cast(counts, ctypes.c_void_p),
                                              PRECISIONS[prec]))
    if need == 0:
        raise GPError("gp_multi_workspace_bytes rejected the sizes")
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, dev)
    total = sum(counts)
    out = torch.empty((max(total, 1), 5), dtype=torch.float64, device=dev)
    st = lib().gp_nll_multi(arr, nds, ctypes.cast(counts, ctypes.c_void_p),
                            ctypes.c_void_p(th.data_ptr()), PRECISIONS[prec],
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            ctypes.c_void_p(out.data_ptr()), _stream_ptr())
    _check(st, "gp_nll_multi")
    res, o = [], 0
    for c in counts:
        res.append(unpack_results(out[o:o + c]))
        o += c
    return res


def predict_workspace_bytes(n: int, d: int, batch: int, N: int) -> int:
    return int(lib().gp_predict_workspace_bytes(n, d, batch, N))


def predict(ds: Dataset, theta, Xstar, ws: torch.Tensor | None = None):
    """Predictions (mean and mean squared error) at the rows of Xstar (N x d)
    with the model fitted at each row of theta (B x d).  Returns (fit results
    dict as nll_batch, mean B x N, mse B x N), device tensors."""
    th = _dev_f64(theta, ds.device).reshape(-1, ds.d)
    Xs = _dev_f64(Xstar, ds.device).reshape(-1, ds.d)
    B, N = th.shape[0], Xs.shape[0]
    need = predict_workspace_bytes(ds.n, ds.d, B, N)
    if need == 0:
        raise GPError("gp_predict_workspace_bytes rejected the sizes")
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, ds.device)
    fit = torch.empty((B, 5), dtype=torch.float64, device=ds.device)
    mean = torch.empty((B, N), dtype=torch.float64, device=ds.device)
    mse = torch.empty((B, N), dtype=torch.float64, device=ds.device)
    st = lib().gp_predict(ds.c, B, ctypes.c_void_p(th.data_ptr()), ctypes.c_void_p(Xs.data_ptr()),
                          N, PRECISIONS["fp64"], ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                          ctypes.c_void_p(fit.data_ptr()), ctypes.c_void_p(mean.data_ptr()),
                          ctypes.c_void_p(mse.data_ptr()), _stream_ptr())
    _check(st, "gp_predict")
    return unpack_results(fit), mean, mse


def nll_grad(ds: Dataset, theta, ws: torch.Tensor | None = None):
    """Profile likelihood and its adjoint gradient for each row of theta.
    Returns (results dict as nll_batch, grad tensor B x d)."""
    th = _dev_f64(theta, ds.device).reshape(-1, ds.d)
    B = th.shape[0]
    need = grad_workspace_bytes(ds.n, ds.d, B)
    if need == 0:
        raise GPError("gp_grad_workspace_bytes rejected the sizes")
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, ds.device)
    out = torch.empty((B, 5), dtype=torch.float64, device=ds.device)
    grad = torch.empty((B, ds.d), dtype=torch.float64, device=ds.device)
    st = lib().gp_nll_grad(ds.c, B, ctypes.c_void_p(th.data_ptr()), PRECISIONS["fp64"],
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out.data_ptr()),
                           ctypes.c_void_p(grad.data_ptr()), _stream_ptr())
    _check(st, "gp_nll_grad")
    return unpack_results(out), grad


def lbfgs_workspace_bytes(n: int, d: int, starts: int, m: int) -> int:
    return int(lib().gp_lbfgs_workspace_bytes(n, d, starts, m))


def lbfgs(ds: Dataset, theta0, iters: int = 50, m: int = 10, c1: float = 1e-4,
          max_ls: int = 20, gtol: float = 1e-6, theta_bounds=(1e-4, 1e4),
          ws: torch.Tensor | None = None):
    """Batched multi-start L-BFGS (gp_lbfgs) from the rows of theta0
    (S x d).  Returns a dict of device tensors theta (S x d), nll, gnorm,
    iters, trace ((iterations + 1) x S) and the host counts iterations and
    evaluations."""
    th = _dev_f64(theta0, ds.device).reshape(-1, ds.d).clone()
    S = th.shape[0]
    need = lbfgs_workspace_bytes(ds.n, ds.d, S, m)
    if need == 0:
        raise GPError("gp_lbfgs_workspace_bytes rejected the sizes")
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, ds.device)
    dev = ds.device
    nll = torch.empty(S, dtype=torch.float64, device=dev)
    gnorm = torch.empty(S, dtype=torch.float64, device=dev)
    its = torch.empty(S, dtype=torch.int32, device=dev)
    trace = torch.empty((iters + 1, S), dtype=torch.float64, device=dev)
    cfg = GPLbfgsConfig(iters, m, max_ls, 0, c1, gtol, float(theta_bounds[0]),
                        float(theta_bounds[1]))
    summ = GPLbfgsSummary()
    st = lib().gp_lbfgs(ds.c, S, ctypes.c_void_p(th.data_ptr()), ctypes.byref(cfg),
                        ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                        ctypes.c_void_p(nll.data_ptr()), ctypes.c_void_p(gnorm.data_ptr()),
                        ctypes.c_void_p(its.data_ptr()), ctypes.c_void_p(trace.data_ptr()),
                        ctypes.byref(summ), _stream_ptr())
    _check(st, "gp_lbfgs")
    return {"theta": th, "nll": nll, "gnorm": gnorm, "iters": its,
            "trace": trace[:summ.iterations + 1], "iterations": summ.iterations,
            "evaluations": summ.evaluations}


class ProfileNLL(torch.autograd.Function):
    """nll(theta) for a batch of thetas (B x d) with the adjoint gradient
    computed by the library in the forward pass; backward scales it."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, ds: Dataset):
        res, grad = nll_grad(ds, theta.detach())
        ctx.save_for_backward(grad)
        return res["nll"].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out[:, None] * grad, None


def profile_nll(theta: torch.Tensor, ds: Dataset) -> torch.Tensor:
    return ProfileNLL.apply(theta, ds)
