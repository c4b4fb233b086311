"""The continuous-batching request server on the GPU: every request completes
exactly once, each result is bitwise the one the request gets alone and
within the FP64 bar of the 80-bit oracle, work of different datasets
overlaps (several micro-batches in flight), admission respects the arena
(HBM footprint) and a tiny arena queues instead of failing.  Both forms of
micro-batch: one dataset each, and ragged (requests of several datasets of
close orders in one launch sequence)."""
import numpy as np
import pytest

from paper_1203_1269_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_1269_amd import binding, serving
    sets = inputs.serving_datasets(seed=40, count=8, n_lo=256, n_hi=1536, d_lo=2, d_hi=12)
    ds = [binding.Dataset(s.X, s.y, s.p, s.delta) for s in sets]
    return binding, serving, sets, ds


def alone(binding, ds, k, th):
    r = binding.nll_batch(ds[k], np.asarray(th)[None])
    return {key: v.cpu().numpy()[0] for key, v in r.items()}


@pytest.mark.parametrize("ragged", [False, True])
def test_server_results_match_alone(env, ragged):
    binding, serving, sets, ds = env
    reqs = inputs.serving_requests(sets, count=300, rate=1e6, seed=41)
    print(f"[serving] alone-vs-served ragged={ragged}", flush=True)
    srv = serving.Server(ds, arena_bytes=2 << 30, max_batch=8, nstreams=6, ragged=ragged)
    lat, res, bsz, wall = serving.replay(srv, [r[0] for r in reqs], [r[2] for r in reqs],
                                         [r[1] for r in reqs], time_limit=120)
    assert srv.outstanding() == 0 and srv.arena_used() == 0
    srv.close()
    assert all(r is not None for r in res)
    assert bsz.max() > 1            # requests were batched
    for q in range(0, 300, 7):
        a = alone(binding, ds, reqs[q][1], reqs[q][2])
        for key in ("logdet", "mu", "sigma2", "nll"):
            assert res[q][key] == a[key], (q, key)
        assert res[q]["info"] == a["info"] == 0
    if ragged:   # micro-batches mixed datasets
        assert len({reqs[q][1] for q in range(8)}) > 1
    print(serving.latency_summary(lat, wall))


def test_ragged_servers_created_and_destroyed(env):
    """Servers made and closed one after another (each close releases the
    side streams the factorisation made for its streams; the next server's
    streams may reuse their handles): results stay bitwise the alone ones."""
    binding, serving, sets, ds = env
    reqs = inputs.serving_requests(sets, count=60, rate=1e9, seed=43)
    for rep in range(4):
        print(f"[serving] server {rep} of 4, ragged, created and destroyed", flush=True)
        srv = serving.Server(ds, arena_bytes=2 << 30, max_batch=16, nstreams=3, ragged=True)
        lat, res, bsz, wall = serving.replay(srv, [r[0] for r in reqs], [r[2] for r in reqs],
                                             [r[1] for r in reqs], time_limit=60)
        assert srv.outstanding() == 0 and srv.arena_used() == 0
        srv.close()
        for q in range(rep, 60, 13):
            a = alone(binding, ds, reqs[q][1], reqs[q][2])
            for key in ("logdet", "mu", "sigma2", "nll"):
                assert res[q][key] == a[key], (rep, q, key)


@pytest.mark.parametrize("ragged", [False, True])
def test_server_results_match_oracle(env, ragged):
    """Served results (uneven n, d and p across the datasets, requests batched
    and overlapped on several streams) against the 80-bit oracle: a sample of
    requests per dataset, every output within max(1e-10, 10 x the FP64
    rounding spread of two independent FP64 codes) for that theta."""
    import oracle
    from parity_util import compare, lapack_fp64, tolerances
    binding, serving, sets, ds = env
    reqs = inputs.serving_requests(sets, count=160, rate=1e6, seed=45)
    print(f"[serving] served-vs-oracle ragged={ragged}", flush=True)
    srv = serving.Server(ds, arena_bytes=2 << 30, max_batch=8, nstreams=6, ragged=ragged)
    lat, res, bsz, wall = serving.replay(srv, [r[0] for r in reqs], [r[2] for r in reqs],
                                         [r[1] for r in reqs], time_limit=120)
    srv.close()
    assert bsz.max() > 1
    checked = 0
    for k, s in enumerate(sets):
        qs = [q for q in range(len(reqs)) if reqs[q][1] == k][:3]
        if not qs:
            continue
        th = np.array([reqs[q][2] for q in qs])
        got = {key: np.array([res[q][key] for q in qs]) for key in
               ("logdet", "mu", "sigma2", "nll", "info")}
        print(f"[serving] dataset {k}: n={s.X.shape[0]} d={s.X.shape[1]} p={s.p}, {len(qs)} requests",
              flush=True)
        r64 = oracle.nll_batch(s.X, s.y, th, s.p, s.delta)
        r80 = oracle.nll_batch(s.X, s.y, th, s.p, s.delta, extended=True)
        tol = tolerances(r64, r80, s.y, lapack_fp64(s.X, s.y, th, s.p, s.delta))
        compare(got, r80, tol, s.y, f"served dataset {k}")
        checked += len(qs)
    assert checked >= 16


@pytest.mark.parametrize("ragged", [False, True])
def test_server_tiny_arena_queues(env, ragged):
    binding, serving, sets, ds = env
    # room for about one largest single request at a time
    need = max(binding.workspace_bytes(d.n, d.d, 1) for d in ds) + (1 << 20)
    reqs = inputs.serving_requests(sets, count=40, rate=1e6, seed=42)
    srv = serving.Server(ds, arena_bytes=need, max_batch=4, nstreams=4, ragged=ragged)
    lat, res, bsz, wall = serving.replay(srv, [r[0] for r in reqs], [r[2] for r in reqs],
                                         [r[1] for r in reqs], time_limit=120)
    assert all(r is not None and r["info"] == 0 for r in res)
    assert srv.arena_used() == 0
    srv.close()


def test_server_rejects_impossible_request(env):
    binding, serving, sets, ds = env
    srv = serving.Server(ds, arena_bytes=1 << 20, max_batch=4, nstreams=2)
    with pytest.raises(binding.GPError):
        srv.submit([(0, 0, np.ones(ds[0].d))])
    srv.close()
    # ragged micro-batches are FP64 only and take no graphs
    for kw in ({"prec": "mixed"}, {"graphs": True}):
        with pytest.raises(binding.GPError):
            serving.Server(ds, arena_bytes=1 << 24, max_batch=4, nstreams=2, ragged=True, **kw)


def test_server_mixed_matches_alone(env):
    """The server in the matched-accuracy mixed mode: each result bitwise the
    one the request gets alone in that mode."""
    binding, serving, sets, ds = env
    reqs = inputs.serving_requests(sets, count=120, rate=1e6, seed=44)
    srv = serving.Server(ds, arena_bytes=2 << 30, max_batch=8, nstreams=4, prec="mixed")
    lat, res, bsz, wall = serving.replay(srv, [r[0] for r in reqs], [r[2] for r in reqs],
                                         [r[1] for r in reqs], time_limit=120)
    assert srv.outstanding() == 0 and srv.arena_used() == 0
    srv.close()
    for q in range(0, 120, 5):
        k, th = reqs[q][1], reqs[q][2]
        r = binding.nll_batch(ds[k], np.asarray(th)[None], prec="mixed")
        a = {key: v.cpu().numpy()[0] for key, v in r.items()}
        for key in ("logdet", "mu", "sigma2", "nll"):
            assert res[q][key] == a[key], (q, key)
        assert res[q]["info"] == a["info"] == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_server_graphs_match_direct_launches(env, prec):
    """Micro-batches launched as captured graphs (kept per stream, updated in
    place when dataset and batch size repeat, instantiated anew otherwise):
    every result bitwise the same as with direct launches, with eager calls
    of the library between the server runs."""
    binding, serving, sets, ds = env
    reqs = inputs.serving_requests(sets, count=240, rate=1e6, seed=43)
    runs = []
    for graphs in (False, True, True):
        srv = serving.Server(ds, arena_bytes=2 << 30, max_batch=8, nstreams=6, prec=prec,
                             graphs=graphs)
        lat, res, bsz, wall = serving.replay(srv, [r[0] for r in reqs], [r[2] for r in reqs],
                                             [r[1] for r in reqs], time_limit=120)
        assert srv.outstanding() == 0 and srv.arena_used() == 0
        srv.close()
        assert all(r is not None for r in res)
        runs.append(res)
        alone(binding, ds, reqs[0][1], reqs[0][2])   # eager work between the runs
    for q in range(len(reqs)):
        for key in ("logdet", "mu", "sigma2", "nll", "info"):
            assert runs[1][q][key] == runs[0][q][key], (q, key)
            assert runs[2][q][key] == runs[0][q][key], (q, key)
