"""The continuous-batching request server on the GPU: every request completes
exactly once, each result is bitwise the one the request gets alone, work of
different datasets overlaps (several micro-batches in flight), admission
respects the arena (HBM footprint) and a tiny arena queues instead of
failing."""
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


def test_server_results_match_alone(env):
    binding, serving, sets, ds = env
    reqs = inputs.serving_requests(sets, count=300, rate=1e6, seed=41)
    srv = serving.Server(ds, arena_bytes=2 << 30, max_batch=8, nstreams=6)
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
    print(serving.latency_summary(lat, wall))


def test_server_tiny_arena_queues(env):
    binding, serving, sets, ds = env
    # room for about one largest single request at a time
    need = max(binding.workspace_bytes(d.n, d.d, 1) for d in ds) + (1 << 20)
    reqs = inputs.serving_requests(sets, count=40, rate=1e6, seed=42)
    srv = serving.Server(ds, arena_bytes=need, max_batch=4, nstreams=4)
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
