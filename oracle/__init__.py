"""Plain FP64 (and 80-bit long double) CPU oracle for the GP profile likelihood.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares
no code with the GPU path.

The arithmetic lives in ``gp_oracle.c`` (plain C, compiled with gcc, no
``-ffast-math``, no ``-march`` so results are the same on every x86-64 host).
Each function below names the passage of Franey, Ranjan & Chipman (arXiv
1203.1269) it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NOUT = 8  # logdet, mu, sigma2, nll, nll_paper, Q, aa, ab


def build(force: bool = False) -> str:
    """Compile gp_oracle.c twice (double and long double) into liboracle.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    objs = []
    for real, sfx in (("double", "f64"), ("long double", "f80")):
        obj = os.path.join(_HERE, f"_oracle_{sfx}.o")
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-c", _SRC, "-o", obj,
               f"-DREAL={real}", f"-DSFX(name)=name##_{sfx}"]
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-shared", "-fopenmp", "-o", tmp] + objs + ["-lm"])
    os.replace(tmp, _LIB)
    for o in objs:
        os.remove(o)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("GP_ORACLE_LIB")  # planted-mistake tests only
        if not path:
            path = build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        for sfx in ("f64", "f80"):
            f = getattr(lib, f"orc_corr_{sfx}")
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int,
                          ctypes.c_double, dp]
            f.restype = ctypes.c_int
            f = getattr(lib, f"orc_cholesky_{sfx}")
            f.argtypes = [ctypes.c_int, dp, dp]
            f.restype = ctypes.c_int
            f = getattr(lib, f"orc_nll_batch_{sfx}")
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int, dp,
                          ctypes.c_double, ctypes.c_int, ctypes.c_double, dp, ip, ctypes.c_int]
            f.restype = ctypes.c_int
            f = getattr(lib, f"orc_grad_batch_{sfx}")
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int, dp,
                          ctypes.c_double, ctypes.c_int, ctypes.c_double, dp, ip, dp,
                          ctypes.c_int]
            f.restype = ctypes.c_int
            f = getattr(lib, f"orc_predict_{sfx}")
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int,
                          ctypes.c_double, ctypes.c_int, dp, dp, dp, dp]
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _sfx(extended: bool) -> str:
    return "f80" if extended else "f64"


# correlation families: the power exponential of eq. (2) (exponent p) and
# the Matern families with smoothness 3/2 and 5/2 that Sec. 2 names as the
# alternative (p is not used by them)
FAMILIES = {"powexp": 0, "matern32": 1, "matern52": 2}


def _fam(family: str) -> int:
    if family not in FAMILIES:
        raise ValueError(f"unknown correlation family {family!r}")
    return FAMILIES[family]


@dataclass
class OracleResult:
    logdet: np.ndarray
    mu: np.ndarray
    sigma2: np.ndarray
    nll: np.ndarray        # log|R_delta| + n ln(sigma2)
    nll_paper: np.ndarray  # literal eq. (4): log|R_delta| + n ln(Q) = nll + n ln n
    Q: np.ndarray
    aa: np.ndarray         # 1' R^-1 1
    ab: np.ndarray         # 1' R^-1 y
    info: np.ndarray


def corr(X, theta, p, delta, extended: bool = False, family: str = "powexp") -> np.ndarray:
    """R_delta of eq. (2) (or a Matern family) plus the nugget (Sec. 2):
    full symmetric n x n."""
    X = _c64(X)
    n, d = X.shape
    th = _c64(theta).reshape(d)
    R = np.empty((n, n))
    st = getattr(_load(), f"orc_corr_{_sfx(extended)}")(n, d, _dp(X), _dp(th), float(p),
                                                        _fam(family), float(delta), _dp(R))
    if st != 0:
        raise ValueError(f"oracle corr failed ({st})")
    return R


def cholesky(A, extended: bool = False):
    """Unblocked Cholesky (Sec. 2 / Sec. 3 CPU implementation). Returns (L, info)."""
    A = _c64(A)
    n = A.shape[0]
    L = np.empty_like(A)
    info = getattr(_load(), f"orc_cholesky_{_sfx(extended)}")(n, _dp(A), _dp(L))
    return L, int(info)


def nll_batch(X, y, theta, p, delta, extended: bool = False, nthreads: int = 0,
              family: str = "powexp") -> OracleResult:
    """Profile likelihood, eq. (3)-(4), for each row of theta (B x d)."""
    X = _c64(X)
    n, d = X.shape
    y = _c64(y).reshape(n)
    th = _c64(theta).reshape(-1, d)
    B = th.shape[0]
    out = np.empty((B, NOUT))
    info = np.empty(B, dtype=np.int32)
    st = getattr(_load(), f"orc_nll_batch_{_sfx(extended)}")(
        n, d, _dp(X), _dp(y), B, _dp(th), float(p), _fam(family), float(delta), _dp(out),
        info.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(nthreads))
    if st != 0:
        raise ValueError(f"oracle nll_batch failed ({st})")
    return OracleResult(*(out[:, q].copy() for q in range(NOUT)), info=info)


def grad_batch(X, y, theta, p, delta, extended: bool = False, nthreads: int = 0,
               family: str = "powexp"):
    """Gradient of nll w.r.t. theta (adjoint formula; see gp_oracle.c)."""
    X = _c64(X)
    n, d = X.shape
    y = _c64(y).reshape(n)
    th = _c64(theta).reshape(-1, d)
    B = th.shape[0]
    out = np.empty((B, NOUT))
    info = np.empty(B, dtype=np.int32)
    g = np.empty((B, d))
    st = getattr(_load(), f"orc_grad_batch_{_sfx(extended)}")(
        n, d, _dp(X), _dp(y), B, _dp(th), float(p), _fam(family), float(delta), _dp(out),
        info.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(g), int(nthreads))
    if st != 0:
        raise ValueError(f"oracle grad_batch failed ({st})")
    return OracleResult(*(out[:, q].copy() for q in range(NOUT)), info=info), g


def rel(x, ref, scale):
    """Relative error |x - ref| / max(|ref|, scale), elementwise."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(x - ref) / np.maximum(np.abs(ref), scale)


def predict(X, y, theta, p, delta, Xs, extended: bool = False, family: str = "powexp"):
    """Predictions at the rows of Xs with the model fitted at one theta: the
    best linear unbiased predictor and its mean squared error (Sec. 3 counts
    their solves; Sec. 4 scores them by the SSPE).  Returns (mean, mse,
    OracleResult of the fit for that theta)."""
    X = _c64(X)
    n, d = X.shape
    y = _c64(y).reshape(n)
    th = _c64(theta).reshape(d)
    Xs = _c64(Xs).reshape(-1, d)
    N = Xs.shape[0]
    fit = np.empty(NOUT)
    mean = np.empty(N)
    mse = np.empty(N)
    info = getattr(_load(), f"orc_predict_{_sfx(extended)}")(
        n, d, _dp(X), _dp(y), _dp(th), float(p), _fam(family), float(delta), N, _dp(Xs),
        _dp(fit), _dp(mean), _dp(mse))
    if info == -100 or info == -101:
        raise ValueError(f"oracle predict failed ({info})")
    res = OracleResult(*(np.array([fit[q]]) for q in range(NOUT)),
                       info=np.array([info], dtype=np.int32))
    return mean, mse, res
