"""Python side of the continuous-batching request server (gp_server_* in the
C ABI): argument marshalling plus an open-loop driver that replays a stream
of timed requests and records per-request latency."""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import binding

DMAX = binding.header_constant("GP_DMAX")


class GPRequest(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("dataset", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("theta", ctypes.c_double * DMAX)]


class GPCompletion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("dataset", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("result", binding.GPResult)]


class GPServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("nstreams", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("graphs", ctypes.c_int32), ("ragged", ctypes.c_int32)]


_bound = False


def _bind():
    global _bound
    if _bound:
        return binding.lib()
    L = binding.lib()
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.gp_server_create.argtypes = [ctypes.POINTER(binding.GPDataset), i32, vp, ctypes.c_size_t,
                                   ctypes.POINTER(GPServerConfig), ctypes.POINTER(vp)]
    L.gp_server_create.restype = ctypes.c_int
    L.gp_server_submit.argtypes = [vp, ctypes.POINTER(GPRequest), i32]
    L.gp_server_submit.restype = ctypes.c_int
    L.gp_server_poll.argtypes = [vp, ctypes.POINTER(GPCompletion), i32]
    L.gp_server_poll.restype = ctypes.c_int32
    L.gp_server_outstanding.argtypes = [vp]
    L.gp_server_outstanding.restype = ctypes.c_int64
    L.gp_server_arena_used.argtypes = [vp]
    L.gp_server_arena_used.restype = ctypes.c_size_t
    L.gp_server_destroy.argtypes = [vp]
    L.gp_server_destroy.restype = ctypes.c_int
    _bound = True
    return L


class Server:
    """Resident datasets + a device arena (admission by HBM footprint) +
    `nstreams` concurrent micro-batches of at most `max_batch` thetas;
    `graphs` launches each micro-batch as a captured HIP graph; `ragged`
    (FP64) forms each micro-batch from the requests of up to 8 datasets (the
    oldest request's and those closest to it in order n) and runs it as one
    ragged batch."""

    def __init__(self, datasets, arena_bytes: int, max_batch: int = 16, nstreams: int = 8,
                 prec: str = "fp64", device="cuda", graphs: bool = False, ragged: bool = False):
        L = _bind()
        self.datasets = list(datasets)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        arr = (binding.GPDataset * len(self.datasets))(*[d._c for d in self.datasets])
        cfg = GPServerConfig(max_batch, nstreams, binding.PRECISIONS[prec], int(bool(graphs)),
                             int(bool(ragged)))
        h = ctypes.c_void_p()
        binding._check(L.gp_server_create(arr, len(self.datasets),
                                          ctypes.c_void_p(self.arena.data_ptr()), arena_bytes,
                                          ctypes.byref(cfg), ctypes.byref(h)), "gp_server_create")
        self.h = h
        self._out = (GPCompletion * 8192)()
        torch.cuda.synchronize()   # dataset uploads done before other streams read them

    def submit(self, reqs):
        """reqs: iterable of (id, dataset_index, theta)."""
        reqs = list(reqs)
        if not reqs:
            return
        arr = (GPRequest * len(reqs))()
        for q, (rid, k, th) in enumerate(reqs):
            arr[q].id = int(rid)
            arr[q].dataset = int(k)
            th = np.asarray(th, dtype=np.float64)
            for j, v in enumerate(th):
                arr[q].theta[j] = float(v)
        binding._check(_bind().gp_server_submit(self.h, arr, len(reqs)), "gp_server_submit")

    def poll(self):
        m = _bind().gp_server_poll(self.h, self._out, len(self._out))
        if m < 0:
            binding._check(m, "gp_server_poll")
        out = []
        for q in range(m):
            c = self._out[q]
            r = c.result
            out.append((c.id, c.dataset, c.batch, {"logdet": r.logdet, "mu": r.mu, "sigma2": r.sigma2,
                                                    "nll": r.nll, "info": r.info}))
        return out

    def outstanding(self) -> int:
        return int(_bind().gp_server_outstanding(self.h))

    def arena_used(self) -> int:
        return int(_bind().gp_server_arena_used(self.h))

    def close(self):
        if self.h:
            _bind().gp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server: Server, arrivals, thetas, datasets_idx, time_limit: float = 600.0):
    """Open-loop replay: request q arrives at arrivals[q] seconds (relative);
    it is submitted as soon as the host clock passes that time.  Returns
    (latency seconds per request, result dict per request, batch size per
    request, wall seconds)."""
    N = len(arrivals)
    order = np.argsort(arrivals, kind="stable")
    lat = np.full(N, np.nan)
    results = [None] * N
    bsz = np.zeros(N, dtype=int)
    t0 = time.perf_counter()
    nxt = 0
    done = 0
    while done < N:
        now = time.perf_counter() - t0
        if now > time_limit:
            raise TimeoutError(f"replay exceeded {time_limit} s ({done}/{N} done)")
        batch = []
        while nxt < N and arrivals[order[nxt]] <= now:
            q = int(order[nxt])
            batch.append((q, datasets_idx[q], thetas[q]))
            nxt += 1
        server.submit(batch)
        for rid, _k, b, res in server.poll():
            t = time.perf_counter() - t0
            lat[rid] = t - arrivals[rid]
            results[rid] = res
            bsz[rid] = b
            done += 1
    return lat, results, bsz, time.perf_counter() - t0


def latency_summary(lat: np.ndarray, wall: float) -> dict:
    return {"requests": int(lat.size), "evals_per_s": float(lat.size / wall),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(np.mean(lat) * 1e3), "max_ms": float(np.max(lat) * 1e3)}
