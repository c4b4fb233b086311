"""Uneven-n batching in one call (gp_nll_multi): thetas for several datasets
of different n, d, p and correlation family evaluated together (FP64: one
ragged batch, every matrix at its own order in the same launches; mixed:
the per-dataset batches side by side on the library's stream pool).

Bar: every result bitwise the one gp_nll_batch gives for the same dataset
and theta (the per-theta arithmetic is the same), and, for the small
datasets, within the FP64 bar of the 80-bit oracle."""
import numpy as np
import pytest

import oracle
from paper_1203_1269_amd import inputs
from parity_util import compare, lapack_fp64, to_host, tolerances

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (n, d, p, family, count)
SETS = [(100, 2, 2.0, "powexp", 3), (257, 4, 1.95, "matern52", 0), (700, 6, 1.5, "powexp", 5),
        (1500, 8, 1.95, "powexp", 2), (2048, 3, 2.0, "matern32", 4), (64, 12, 1.0, "powexp", 1)]


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_1269_amd import binding
    binding.lib()
    return binding


def _make(gp):
    rng = np.random.default_rng(777)
    data, dsets, thetas = [], [], []
    for n, d, p, fam, c in SETS:
        X = inputs.lhs_design(n, d, rng)
        y = inputs.sine_response(X, rng)
        th = inputs.log_uniform_theta(c, d, 0.05, 20, rng)
        data.append((X, y, p, fam))
        dsets.append(gp.Dataset(X, y, p, 1e-6, corr=fam))
        thetas.append(th)
    return data, dsets, thetas


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_matches_per_dataset_batches(gp, prec):
    data, dsets, thetas = _make(gp)
    print(f"[parity] nll_multi {prec} over {len(SETS)} datasets", flush=True)
    got = [to_host(r) for r in gp.nll_multi(dsets, thetas, prec=prec)]
    for k, (ds, th) in enumerate(zip(dsets, thetas)):
        assert got[k]["nll"].shape[0] == th.shape[0]
        if th.shape[0] == 0:
            continue
        ref = to_host(gp.nll_batch(ds, th, prec=prec))
        for key in ("logdet", "mu", "sigma2", "nll", "info", "ir_iters"):
            assert np.array_equal(got[k][key], ref[key], equal_nan=True), (k, key)


def test_multi_against_oracle_and_repeatable(gp):
    data, dsets, thetas = _make(gp)
    print("[parity] nll_multi vs oracle", flush=True)
    a = [to_host(r) for r in gp.nll_multi(dsets, thetas)]
    b = [to_host(r) for r in gp.nll_multi(dsets, thetas)]
    for k in range(len(SETS)):
        for key in ("logdet", "nll", "info"):
            assert np.array_equal(a[k][key], b[k][key]), (k, key)
    for k in (0, 2, 5):
        X, y, p, fam = data[k]
        th = thetas[k]
        r64 = oracle.nll_batch(X, y, th, p, 1e-6, family=fam)
        r80 = oracle.nll_batch(X, y, th, p, 1e-6, extended=True, family=fam)
        tol = tolerances(r64, r80, y, lapack_fp64(X, y, th, p, 1e-6, family=fam))
        compare(a[k], r80, tol, y, f"multi dataset {k}")


def test_multi_ragged_serving_shapes(gp):
    """The 64 serving datasets (n from 256 to 6144, d 2..12, p in {1.5, 1.95,
    2}) with 1 to 3 thetas each in one ragged FP64 batch, one theta invalid
    (negative component): every result bitwise the per-dataset gp_nll_batch
    one, the invalid theta alone marked info = -3, and the small datasets
    within the FP64 bar of the 80-bit oracle."""
    sets = inputs.serving_datasets()
    rng = np.random.default_rng(778)
    dsets = [gp.Dataset(s.X, s.y, s.p, s.delta) for s in sets]
    thetas = [inputs.log_uniform_theta(1 + k % 3, s.X.shape[1], 0.05, 20, rng)
              for k, s in enumerate(sets)]
    thetas[5][0, 0] = -1.0
    print(f"[parity] ragged nll_multi over {len(sets)} serving datasets, "
          f"{sum(t.shape[0] for t in thetas)} thetas", flush=True)
    got = [to_host(r) for r in gp.nll_multi(dsets, thetas)]
    for k, (ds, th) in enumerate(zip(dsets, thetas)):
        ref = to_host(gp.nll_batch(ds, th))
        for key in ("logdet", "mu", "sigma2", "nll", "info", "ir_iters"):
            assert np.array_equal(got[k][key], ref[key], equal_nan=True), (k, key)
    assert got[5]["info"][0] == -3
    assert all(np.all(got[k]["info"] == 0) for k in range(len(sets)) if k != 5)
    small = [k for k, s in enumerate(sets) if s.X.shape[0] <= 640 and k != 5][:4]
    for k in small:
        s = sets[k]
        r64 = oracle.nll_batch(s.X, s.y, thetas[k], s.p, s.delta)
        r80 = oracle.nll_batch(s.X, s.y, thetas[k], s.p, s.delta, extended=True)
        tol = tolerances(r64, r80, s.y, lapack_fp64(s.X, s.y, thetas[k], s.p, s.delta))
        compare(got[k], r80, tol, s.y, f"ragged serving dataset {k}")
