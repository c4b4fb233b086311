"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/gpnll.h declares, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpnll.h")
LIB = os.path.join(ROOT, "paper_1203_1269_amd", "libgpnll.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:gp_status|size_t|int|void)\s+\**\s*(gp_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1203_1269_amd import build
        build.build()
    from paper_1203_1269_amd import binding
    return binding.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gp_nll", "gp_nll_batch", "gp_workspace_bytes", "gp_corr_build",
                     "gp_cholesky_batch", "gp_cholesky_ws_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(\w+)$", out, flags=re.M))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_result_struct_layout(tmp_path):
    from paper_1203_1269_amd import binding
    assert ctypes.sizeof(binding.GPResult) == 40
    assert ctypes.sizeof(binding.GPDataset) == 48
    assert binding.GPDataset.corr.offset == 40
    # the header's own layout, compiled on the host
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gpnll.h"\n'
                   'int main(void) { printf("%zu %zu %zu", sizeof(gp_dataset), '
                   'offsetof(gp_dataset, corr), sizeof(gp_result)); return 0; }\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include", "-I/opt/rocm/include",
                           str(src), "-o", str(exe)])
    assert subprocess.check_output([str(exe)]).decode().split() == ["48", "40", "40"]
    assert binding.header_constant("GP_NMAX") == 8192
    assert binding.header_constant("GP_DMAX") == 32


def test_workspace_sizing(lib):
    from paper_1203_1269_amd import binding
    ws = binding.workspace_bytes(4096, 8, 128)
    assert ws >= 128 * 4096 * 4096 * 8
    assert ws < 128 * 4096 * 4096 * 8 + (1 << 24)
    assert binding.workspace_bytes(200, 2, 64) >= 64 * 256 * 256 * 8
    assert lib.gp_workspace_bytes(1, 2, 1, 0) == 0        # n < 2
    assert lib.gp_workspace_bytes(8193, 2, 1, 0) == 0     # n > GP_NMAX
    assert lib.gp_workspace_bytes(100, 0, 1, 0) == 0      # d < 1
    assert lib.gp_workspace_bytes(100, 33, 1, 0) == 0     # d > GP_DMAX
    assert lib.gp_workspace_bytes(100, 2, 0, 0) == 0      # empty batch
    assert lib.gp_workspace_bytes(100, 2, 1, 7) == 0      # unknown precision
    # the matched-accuracy mixed mode adds the INT8 residues of the panel
    # rows (GP_MIXED_MODULI x GP_MIXED_RANK bytes per row, rows padded to a
    # multiple of 128), one exponent per row and a fallback flag per theta
    N = binding.header_constant("GP_MIXED_MODULI")
    K = binding.header_constant("GP_MIXED_RANK")
    assert (N, K) == (16, 768)
    mx = binding.workspace_bytes(4096, 8, 128, "mixed")
    assert mx >= ws + 128 * 4096 * (N * K + 4)
    assert mx < ws + 128 * 4096 * (N * K + 4) + (1 << 12)
    assert binding.workspace_bytes(4096, 8, 128, "mixed_fast") > ws
    bmax = binding.header_constant("GP_BATCH_MAX")
    assert lib.gp_workspace_bytes(100, 2, bmax, 0) > 0
    assert lib.gp_workspace_bytes(100, 2, bmax + 1, 0) == 0
    assert lib.gp_grad_workspace_bytes(100, 2, bmax + 1) == 0
    assert lib.gp_cholesky_ws_bytes(100, bmax + 1) == 0
    # predictions: 64 + 64 ceil(N / 64) extra rows below each matrix
    pw = binding.predict_workspace_bytes(4096, 8, 8, 1000)
    rows = 4096 + 64 + 1024
    assert 8 * rows * 4096 * 8 <= pw < 8 * rows * 4096 * 8 + (1 << 20)
    assert binding.predict_workspace_bytes(4096, 8, 8, 0) > 0
    assert binding.predict_workspace_bytes(4096, 8, 8, -1) == 0
    assert binding.predict_workspace_bytes(4096, 8, 8, (1 << 20) + 1) == 0
    assert binding.predict_workspace_bytes(4096, 33, 8, 10) == 0
    assert binding.predict_workspace_bytes(100, 2, bmax + 1, 10) == 0


def _ds(X=1 << 20, y=1 << 21, n=100, d=2, p=2.0, delta=1e-6, corr=0, reserved=0):
    from paper_1203_1269_amd import binding
    return binding.GPDataset(X, y, n, d, p, delta, corr, reserved)


@pytest.mark.parametrize("kw", [dict(n=1), dict(n=8193), dict(d=0), dict(d=33), dict(p=0.0),
                                dict(p=2.5), dict(p=float("nan")), dict(delta=-1e-9),
                                dict(delta=float("inf")), dict(X=0), dict(y=0), dict(corr=3),
                                dict(corr=-1), dict(reserved=1)])
def test_invalid_dataset_rejected_on_host(lib, kw):
    from paper_1203_1269_amd import binding
    ds = _ds(**kw)
    vp = ctypes.c_void_p
    st = lib.gp_nll_batch(ctypes.byref(ds), 4, vp(1 << 22), 0, vp(1 << 23), 1 << 40, vp(1 << 24), None)
    assert st == binding.GP_EINVAL
    st = lib.gp_corr_build(ctypes.byref(ds), 4, vp(1 << 22), vp(1 << 23), 256, vp(1 << 24), None)
    assert st == binding.GP_EINVAL


def test_invalid_call_arguments_rejected_on_host(lib):
    from paper_1203_1269_amd import binding
    ds = _ds()
    vp = ctypes.c_void_p
    need = lib.gp_workspace_bytes(100, 2, 4, 0)
    assert lib.gp_nll_batch(ctypes.byref(ds), 0, vp(1 << 22), 0, vp(1 << 23), need, vp(1 << 24), None) == binding.GP_EINVAL
    assert lib.gp_nll_batch(ctypes.byref(ds), 4, None, 0, vp(1 << 23), need, vp(1 << 24), None) == binding.GP_EINVAL
    assert lib.gp_nll_batch(ctypes.byref(ds), 4, vp(1 << 22), 0, None, need, vp(1 << 24), None) == binding.GP_EINVAL
    assert lib.gp_nll_batch(ctypes.byref(ds), 4, vp(1 << 22), 0, vp(1 << 23), need, None, None) == binding.GP_EINVAL
    assert lib.gp_nll_batch(ctypes.byref(ds), 4, vp(1 << 22), 5, vp(1 << 23), need, vp(1 << 24), None) == binding.GP_EINVAL
    assert lib.gp_nll_batch(ctypes.byref(ds), 4, vp(1 << 22), 0, vp((1 << 23) + 8), need, vp(1 << 24), None) == binding.GP_EINVAL
    assert lib.gp_nll_batch(ctypes.byref(ds), 4, vp(1 << 22), 0, vp(1 << 23), need - 1, vp(1 << 24), None) == binding.GP_EWORKSPACE
    assert lib.gp_nll_batch(None, 4, vp(1 << 22), 0, vp(1 << 23), need, vp(1 << 24), None) == binding.GP_EINVAL
    # Cholesky entry point
    assert lib.gp_cholesky_batch(100, 2, vp(1 << 22), 100, vp(1 << 23), vp(1 << 24), vp(1 << 25), 1 << 20, None) == binding.GP_EINVAL  # lda < 128
    assert lib.gp_cholesky_batch(100, 2, vp(1 << 22), 129, vp(1 << 23), vp(1 << 24), vp(1 << 25), 1 << 20, None) == binding.GP_EINVAL  # odd lda
    assert lib.gp_cholesky_batch(100, 2, vp(1 << 22), 128, vp(1 << 23), vp(1 << 24), vp(1 << 25), 0, None) == binding.GP_EWORKSPACE
    assert lib.gp_corr_build(ctypes.byref(ds), 4, vp(1 << 22), vp(1 << 23), 100, vp(1 << 24), None) == binding.GP_EINVAL  # ldr < 128
    assert lib.gp_nll_batch(ctypes.byref(ds), 65536, vp(1 << 22), 0, vp(1 << 23), 1 << 40, vp(1 << 24), None) == binding.GP_EINVAL  # batch > GP_BATCH_MAX
    # prediction entry point: FP64 only, test points and outputs needed when N > 0
    pneed = lib.gp_predict_workspace_bytes(100, 2, 4, 10)
    args = [ctypes.byref(ds), 4, vp(1 << 22), vp(1 << 21), 10, 0, vp(1 << 23), pneed, vp(1 << 24),
            vp(1 << 25), vp(1 << 26), None]

    def pred(**chg):
        a = list(args)
        for i, v in chg.items():
            a[int(i[1:])] = v
        return lib.gp_predict(*a)
    assert pred(a5=1) == binding.GP_EINVAL                     # not FP64
    assert pred(a3=None) == binding.GP_EINVAL                  # no test points
    assert pred(a9=None) == binding.GP_EINVAL                  # no mean
    assert pred(a10=None) == binding.GP_EINVAL                 # no mse
    assert pred(a8=None) == binding.GP_EINVAL                  # no fit
    assert pred(a4=-1) == binding.GP_EINVAL                    # N < 0
    assert pred(a6=vp((1 << 23) + 8)) == binding.GP_EINVAL     # unaligned workspace
    assert pred(a7=pneed - 1) == binding.GP_EWORKSPACE
    assert pred(a1=0) == binding.GP_EINVAL


def test_multi_dataset_call_checked_on_host(lib):
    from paper_1203_1269_amd import binding
    vp = ctypes.c_void_p
    arr = (binding.GPDataset * 3)(_ds(n=100, d=2), _ds(n=700, d=5), _ds(n=2, d=2, p=0.0))
    counts = (ctypes.c_int32 * 3)(4, 7, 0)
    need = lib.gp_multi_workspace_bytes(arr, 3, counts, 0)
    up = lambda x: (x + 255) // 256 * 256
    # FP64: one ragged batch of B = 11 matrices (orders 128 and 704): 32-byte
    # descriptors, the matrices back to back (per dataset, 256-byte aligned),
    # then per matrix at the largest order: log-det partials, info, the
    # 64 x 64 TRSM copy and the 2-vector solve state
    B, npmax = 11, 704
    ragged = (up(32 * B) + up(8 * (up(4 * 128 * 128 * 8) // 8 + 7 * 704 * 704)) +
              up(8 * (npmax // 64) * B) + up(4 * B) + up(8 * 64 * 64 * B) + up(16 * npmax * B))
    assert need == ragged            # dataset 2 has no work: its descriptor is not read
    # the mixed modes: one gp_nll_batch workspace per dataset with work
    a = lib.gp_workspace_bytes(100, 2, 4, 1)
    b = lib.gp_workspace_bytes(700, 5, 7, 1)
    assert lib.gp_multi_workspace_bytes(arr, 3, counts, 1) == up(a) + up(b)
    assert lib.gp_multi_workspace_bytes(arr, 3, (ctypes.c_int32 * 3)(4, -1, 0), 0) == 0
    assert lib.gp_multi_workspace_bytes(arr, 3, counts, 9) == 0
    assert lib.gp_multi_workspace_bytes(arr, 3, (ctypes.c_int32 * 3)(0, 0, 0), 0) == 256
    call = lambda arr_, n_, c_, ws_, wsb: lib.gp_nll_multi(arr_, n_, c_, vp(1 << 22), 0, ws_, wsb,
                                                           vp(1 << 24), None)
    assert call(arr, 0, counts, vp(1 << 23), need) == binding.GP_EINVAL
    assert call(arr, 3, counts, vp((1 << 23) + 8), need) == binding.GP_EINVAL
    assert call(arr, 3, counts, vp(1 << 23), need - 1) == binding.GP_EWORKSPACE
    assert call(arr, 3, (ctypes.c_int32 * 3)(4, 7, 1), vp(1 << 23), 1 << 40) == binding.GP_EINVAL
    assert call(arr, 3, (ctypes.c_int32 * 3)(4, 65536, 0), vp(1 << 23), 1 << 40) == binding.GP_EINVAL
    assert call(arr, 3, (ctypes.c_int32 * 3)(0, 0, 0), vp(1 << 23), 256) == binding.GP_OK


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1203_1269_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.lib()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    before touching a device."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_product_code_never_uses_the_oracle():
    """Only tests, smoke() and the bench's CPU baseline may call the oracle:
    the package itself must not import it."""
    import glob
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_1203_1269_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*.py"), recursive=True) + \
            glob.glob(os.path.join(pkg, "csrc", "*")):
        text = open(path, errors="replace").read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), path
        assert "liboracle" not in text and "gp_oracle" not in text, path


def test_lbfgs_call_checked_on_host(lib):
    """gp_lbfgs rejects bad arguments (and a short workspace) before it
    launches anything."""
    from paper_1203_1269_amd import binding
    vp = ctypes.c_void_p
    ds = _ds(n=300, d=3)
    need = lib.gp_lbfgs_workspace_bytes(300, 3, 4, 10)
    assert need > lib.gp_grad_workspace_bytes(300, 3, 4)
    assert lib.gp_lbfgs_workspace_bytes(300, 3, 0, 10) == 0        # no starts
    assert lib.gp_lbfgs_workspace_bytes(300, 3, 1025, 10) == 0     # too many starts
    assert lib.gp_lbfgs_workspace_bytes(300, 3, 4, 0) == 0         # no history
    assert lib.gp_lbfgs_workspace_bytes(300, 3, 4, 33) == 0
    assert lib.gp_lbfgs_workspace_bytes(300, 33, 4, 10) == 0       # d too large

    def call(S=4, cfg=None, ws=1 << 24, wsb=None, summ=True, ds_=ds, **kw):
        c = binding.GPLbfgsConfig(50, 10, 20, 0, 1e-4, 1e-6, 1e-4, 1e4)
        for k, v in kw.items():
            setattr(c, k, v)
        s = binding.GPLbfgsSummary()
        return lib.gp_lbfgs(ctypes.byref(ds_), S, vp(1 << 22), ctypes.byref(c), vp(ws),
                            need if wsb is None else wsb, vp(1 << 23), vp(1 << 23),
                            vp(1 << 23), None, ctypes.byref(s) if summ else None, None)
    assert call(wsb=need - 1) == binding.GP_EWORKSPACE
    assert call(ws=(1 << 24) + 8) == binding.GP_EINVAL              # unaligned workspace
    assert call(S=0) == binding.GP_EINVAL
    assert call(m=0) == binding.GP_EINVAL
    assert call(max_ls=0) == binding.GP_EINVAL
    assert call(iters=-1) == binding.GP_EINVAL
    assert call(c1=0.0) == binding.GP_EINVAL
    assert call(c1=1.0) == binding.GP_EINVAL
    assert call(gtol=float("nan")) == binding.GP_EINVAL
    assert call(theta_lo=0.0) == binding.GP_EINVAL
    assert call(theta_hi=1e-5) == binding.GP_EINVAL                 # below theta_lo
    assert call(theta_hi=float("inf")) == binding.GP_EINVAL
    assert call(reserved=1) == binding.GP_EINVAL
    assert call(summ=False) == binding.GP_EINVAL
    assert call(ds_=_ds(n=1)) == binding.GP_EINVAL


def test_server_config_checked_on_host(lib):
    """gp_server_create rejects a bad configuration before it creates any
    stream: ragged micro-batches are FP64 only and take no graphs."""
    from paper_1203_1269_amd import binding, serving
    L = serving._bind()
    vp = ctypes.c_void_p
    arr = (binding.GPDataset * 1)(_ds(n=300, d=3))
    h = vp()

    def create(**kw):
        c = dict(max_batch=8, nstreams=2, prec=0, graphs=0, ragged=0)
        c.update(kw)
        cfg = serving.GPServerConfig(c["max_batch"], c["nstreams"], c["prec"], c["graphs"],
                                     c["ragged"])
        return L.gp_server_create(arr, 1, vp(1 << 24), 1 << 30, ctypes.byref(cfg), ctypes.byref(h))
    assert create(ragged=1, prec=1) == binding.GP_EINVAL
    assert create(ragged=1, prec=2) == binding.GP_EINVAL
    assert create(ragged=1, graphs=1) == binding.GP_EINVAL
    assert create(ragged=2) == binding.GP_EINVAL
    assert create(graphs=2) == binding.GP_EINVAL
    assert create(max_batch=0) == binding.GP_EINVAL
    assert create(nstreams=65) == binding.GP_EINVAL
