// Continuous-batching request server over resident datasets.
//
// Requests (dataset, theta) are queued on the host.  Each poll
//   1. retires finished micro-batches (their completion event has fired):
//      results are handed out, their arena block and stream are freed;
//   2. admits queued work while a stream and arena space are free: the
//      oldest queued request picks the dataset, up to max_batch queued
//      requests of that dataset (in arrival order) form one micro-batch, its
//      footprint (workspace + theta + results) is carved from the caller's
//      arena, and the batch is launched on its own stream (theta upload,
//      gp_nll_batch, result download, event).
// With `ragged` (FP64), a micro-batch mixes datasets and runs as one ragged
// batch (nll_ragged_impl), whose kernels advance every request of the batch
// together, each matrix at its own order.  It takes the requests (in arrival
// order) of at most RAGGED_DATASETS datasets: the oldest request's, then
// those closest to it in order n among the queued ones (choose_ragged_batch).
// When the queue is long this gathers several requests per dataset, whose
// correlation builds then share the |x_i - x_j|^p terms (one request per
// dataset shares nothing, and the build's pow() is then a large part of the
// work), and matrices of close orders, which finish together; when it is
// short the batch is just the queued requests.
// Micro-batches run concurrently on different streams,
// so requests that arrive while others are on the GPU start as soon as a
// stream and memory are free.  Every theta's arithmetic is independent of the
// rest of its batch and of the other streams, so a request's result is
// bitwise the one it gets alone.  Every micro-batch takes the oldest queued
// request, so no request starves.
//
// With graphs on, each micro-batch's kernel sequence is captured into a HIP
// graph and launched as one: the executable graph of a stream is kept and,
// when the next micro-batch on that stream has the same dataset and batch
// size (same launch sequence, new buffers), updated in place instead of
// instantiated again.  A stream's graph is only updated after its previous
// micro-batch retired.  No memset nodes are captured (every kernel writes
// what it needs).  Graphs are not used while per-launch profiling is on.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <vector>

#include "admission.hpp"
#include "arena.hpp"
#include "kernels.hpp"

using namespace gpk;

// Ragged micro-batches factor with the one-panel lookahead (side streams per
// server stream): the thin tail of a batch's largest matrices then overlaps
// the next panel.
constexpr bool RAGGED_LOOKAHEAD = true;
constexpr int RAGGED_DATASETS = 8;

struct gp_server {
    std::vector<gp_dataset> ds;
    char *arena_base = nullptr;
    Arena arena;
    int max_batch = 32;
    int prec = GP_FP64;
    bool graphs = false;
    bool ragged = false;
    std::deque<gp_request> pending;
    struct Stream {
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;
        double *h_theta = nullptr;      // pinned staging, max_batch * GP_DMAX
        gp_result *h_out = nullptr;     // pinned results, max_batch
        bool busy = false;
        bool failed = false;             // the micro-batch's launch failed
        int dataset = -1, B = 0;         // dataset: -1 for a ragged batch
        hipGraphExec_t exec = nullptr;   // kept executable graph (graphs on)
        int g_dataset = -1, g_B = 0;     // the launch sequence it holds
        size_t off = 0, bytes = 0;
        std::vector<int64_t> ids;
        std::vector<int32_t> dsets;      // dataset of each result (ragged batch)
    };
    std::vector<Stream> streams;
    int64_t in_flight = 0;
};

namespace {

size_t batch_bytes(const gp_dataset &d, int B, int prec, size_t &ws_bytes, size_t &theta_off,
                   size_t &out_off)
{
    ws_bytes = gp_workspace_bytes(d.n, d.d, B, prec);
    if (ws_bytes == 0) return 0;
    theta_off = Arena::round(ws_bytes);
    out_off = theta_off + Arena::round(sizeof(double) * (size_t)B * d.d);
    return out_off + Arena::round(sizeof(gp_result) * (size_t)B);
}

// One micro-batch's gp_nll_batch sequence as a graph on st.s.  Falls back to
// launching the kernels directly when capture or instantiation fails.
gp_status launch_captured(gp_server::Stream &st, int k, const gp_dataset &d, int B,
                          const double *d_theta, int prec, void *ws, size_t ws_bytes,
                          gp_result *d_out)
{
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(st.s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nll_batch_impl(&d, B, d_theta, prec, ws, ws_bytes, d_out, st.s, false);
    }
    const gp_status rc = nll_batch_impl(&d, B, d_theta, prec, ws, ws_bytes, d_out, st.s, false);
    const hipError_t e = hipStreamEndCapture(st.s, &g);
    if (e != hipSuccess || rc != GP_OK || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return nll_batch_impl(&d, B, d_theta, prec, ws, ws_bytes, d_out, st.s, false);
    }
    bool ok = false;
    if (st.exec && st.g_dataset == k && st.g_B == B) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res;
        ok = hipGraphExecUpdate(st.exec, g, &bad, &res) == hipSuccess &&
             res == hipGraphExecUpdateSuccess;
        (void)hipGetLastError();
    }
    if (!ok) {
        if (st.exec) (void)hipGraphExecDestroy(st.exec);
        st.exec = nullptr;
        st.g_dataset = -1;
        ok = hipGraphInstantiate(&st.exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (ok) {
            st.g_dataset = k;
            st.g_B = B;
        } else {
            st.exec = nullptr;
            (void)hipGetLastError();
        }
    }
    (void)hipGraphDestroy(g);
    if (!ok) return nll_batch_impl(&d, B, d_theta, prec, ws, ws_bytes, d_out, st.s, false);
    return hipGraphLaunch(st.exec, st.s) == hipSuccess ? GP_OK : GP_ELAUNCH;
}

bool launch_batch(gp_server *sv, gp_server::Stream &st, int k, std::vector<gp_request> &reqs)
{
    const gp_dataset &d = sv->ds[k];
    const int B = (int)reqs.size();
    size_t ws_bytes, theta_off, out_off;
    const size_t need = batch_bytes(d, B, sv->prec, ws_bytes, theta_off, out_off);
    size_t off;
    if (need == 0 || !sv->arena.alloc(need, off)) return false;
    char *base = sv->arena_base + off;
    for (int q = 0; q < B; ++q)
        memcpy(st.h_theta + (size_t)q * d.d, reqs[q].theta, sizeof(double) * d.d);
    double *d_theta = (double *)(base + theta_off);
    gp_result *d_out = (gp_result *)(base + out_off);
    (void)hipMemcpyAsync(d_theta, st.h_theta, sizeof(double) * (size_t)B * d.d,
                         hipMemcpyHostToDevice, st.s);
    // micro-batches already run side by side: no lookahead stream per call
    const gp_status rc =
        (sv->graphs && !prof_enabled())
            ? launch_captured(st, k, d, B, d_theta, sv->prec, base, ws_bytes, d_out)
            : nll_batch_impl(&d, B, d_theta, sv->prec, base, ws_bytes, d_out, st.s, false);
    (void)hipMemcpyAsync(st.h_out, d_out, sizeof(gp_result) * B, hipMemcpyDeviceToHost, st.s);
    (void)hipEventRecord(st.done, st.s);
    st.busy = true;
    st.dataset = k;
    st.B = B;
    st.off = off;
    st.bytes = need;
    st.ids.clear();
    for (const gp_request &r : reqs) st.ids.push_back(r.id);
    // arguments were validated at submit; a failed launch marks the results
    // at retirement (the copy into h_out queued above still lands first)
    st.failed = rc != GP_OK;
    return true;
}

// Footprint of a ragged micro-batch with counts[k] requests of dataset k:
// workspace, then the packed thetas, then the results.
size_t ragged_bytes(const gp_server *sv, const std::vector<int32_t> &counts, size_t &ws_bytes,
                    size_t &theta_off, size_t &out_off)
{
    const int nds = (int)sv->ds.size();
    ws_bytes = ragged_workspace_bytes(sv->ds.data(), nds, counts.data());
    if (ws_bytes == 0) return 0;
    size_t nth = 0, B = 0;
    for (int k = 0; k < nds; ++k) {
        nth += (size_t)counts[k] * sv->ds[k].d;
        B += counts[k];
    }
    theta_off = Arena::round(ws_bytes);
    out_off = theta_off + Arena::round(sizeof(double) * nth);
    return out_off + Arena::round(sizeof(gp_result) * B);
}

// Ragged micro-batch of the requests `reqs` (any datasets): they are grouped
// by dataset (stable) for the launch; results come back in that order.
bool launch_ragged(gp_server *sv, gp_server::Stream &st, std::vector<gp_request> &reqs)
{
    const int nds = (int)sv->ds.size();
    std::vector<int32_t> counts(nds, 0);
    for (const gp_request &r : reqs) ++counts[r.dataset];
    size_t ws_bytes, theta_off, out_off;
    const size_t need = ragged_bytes(sv, counts, ws_bytes, theta_off, out_off);
    if (need == 0) return false;
    const int B = (int)reqs.size();
    std::stable_sort(reqs.begin(), reqs.end(),
                     [](const gp_request &a, const gp_request &b) { return a.dataset < b.dataset; });
    size_t nth = 0;
    for (const gp_request &r : reqs) nth += sv->ds[r.dataset].d;
    size_t off;
    if (!sv->arena.alloc(need, off)) return false;
    char *base = sv->arena_base + off;
    size_t t = 0;
    for (const gp_request &r : reqs) {
        const int d = sv->ds[r.dataset].d;
        memcpy(st.h_theta + t, r.theta, sizeof(double) * d);
        t += d;
    }
    double *d_theta = (double *)(base + theta_off);
    gp_result *d_out = (gp_result *)(base + out_off);
    (void)hipMemcpyAsync(d_theta, st.h_theta, sizeof(double) * nth, hipMemcpyHostToDevice, st.s);
    const gp_status rc = nll_ragged_impl(sv->ds.data(), nds, counts.data(), d_theta, base,
                                         ws_bytes, d_out, st.s, RAGGED_LOOKAHEAD);
    (void)hipMemcpyAsync(st.h_out, d_out, sizeof(gp_result) * B, hipMemcpyDeviceToHost, st.s);
    (void)hipEventRecord(st.done, st.s);
    st.busy = true;
    st.dataset = -1;
    st.B = B;
    st.off = off;
    st.bytes = need;
    st.ids.clear();
    st.dsets.clear();
    for (const gp_request &r : reqs) {
        st.ids.push_back(r.id);
        st.dsets.push_back(r.dataset);
    }
    st.failed = rc != GP_OK;
    return true;
}

}  // namespace

extern "C" {

gp_status gp_server_create(const gp_dataset *datasets, int32_t ndatasets, void *arena,
                           size_t arena_bytes, const gp_server_config *cfg, gp_server **out)
{
    if (!datasets || ndatasets < 1 || !arena || !cfg || !out) return GP_EINVAL;
    if (cfg->max_batch < 1 || cfg->max_batch > 1024 || cfg->nstreams < 1 || cfg->nstreams > 64)
        return GP_EINVAL;
    if (cfg->prec != GP_FP64 && cfg->prec != GP_MIXED && cfg->prec != GP_MIXED_FAST)
        return GP_EINVAL;
    if (cfg->graphs != 0 && cfg->graphs != 1) return GP_EINVAL;
    if (cfg->ragged != 0 && cfg->ragged != 1) return GP_EINVAL;
    if (cfg->ragged == 1 && (cfg->prec != GP_FP64 || cfg->graphs != 0)) return GP_EINVAL;
    if (((uintptr_t)arena & 255) != 0) return GP_EINVAL;
    for (int k = 0; k < ndatasets; ++k) {
        const gp_dataset &d = datasets[k];
        if (!d.X || !d.y || d.n < 2 || d.n > GP_NMAX || d.d < 1 || d.d > GP_DMAX ||
            !gpk::family_ok(&d) || !(d.delta >= 0.0) || !std::isfinite(d.delta))
            return GP_EINVAL;
    }
    gp_server *sv = new gp_server();
    sv->ds.assign(datasets, datasets + ndatasets);
    sv->arena_base = (char *)arena;
    sv->arena.reset(arena_bytes);
    sv->max_batch = cfg->max_batch;
    sv->prec = cfg->prec;
    sv->graphs = cfg->graphs == 1;
    sv->ragged = cfg->ragged == 1;
    sv->streams.resize(cfg->nstreams);
    for (auto &st : sv->streams) {
        bool ok = hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&st.done, hipEventDisableTiming) == hipSuccess &&
                  hipHostMalloc((void **)&st.h_theta, sizeof(double) * cfg->max_batch * GP_DMAX,
                                hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc((void **)&st.h_out, sizeof(gp_result) * cfg->max_batch,
                                hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            gp_server_destroy(sv);
            return GP_ELAUNCH;
        }
    }
    *out = sv;
    return GP_OK;
}

gp_status gp_server_submit(gp_server *sv, const gp_request *reqs, int32_t count)
{
    if (!sv || (!reqs && count > 0) || count < 0) return GP_EINVAL;
    for (int q = 0; q < count; ++q) {
        const gp_request &r = reqs[q];
        if (r.dataset < 0 || r.dataset >= (int)sv->ds.size()) return GP_EINVAL;
        size_t a, b, c, one;
        if (sv->ragged) {
            std::vector<int32_t> counts(sv->ds.size(), 0);
            counts[r.dataset] = 1;
            one = ragged_bytes(sv, counts, a, b, c);
        } else {
            one = batch_bytes(sv->ds[r.dataset], 1, sv->prec, a, b, c);
        }
        if (one > sv->arena.size()) return GP_EWORKSPACE;   // would never fit
    }
    for (int q = 0; q < count; ++q) sv->pending.push_back(reqs[q]);
    sv->in_flight += count;
    return GP_OK;
}

int32_t gp_server_poll(gp_server *sv, gp_completion *out, int32_t max_out)
{
    if (!sv || max_out < 0 || (!out && max_out > 0)) return GP_EINVAL;
    // a micro-batch is reported whole: room for fewer than max_batch could
    // leave one unretired for ever
    if (max_out > 0 && max_out < sv->max_batch) return GP_EINVAL;
    int32_t m = 0;
    // 1. retire finished micro-batches
    for (auto &st : sv->streams) {
        if (!st.busy) continue;
        if (m + st.B > max_out) continue;   // no room to report it yet
        const hipError_t q = hipEventQuery(st.done);
        if (q == hipErrorNotReady) continue;
        for (int k = 0; k < st.B; ++k) {
            out[m].id = st.ids[k];
            out[m].dataset = st.dataset >= 0 ? st.dataset : st.dsets[k];
            out[m].batch = st.B;
            out[m].result = st.h_out[k];
            if (q != hipSuccess || st.failed) {
                gp_result &r = out[m].result;
                r.info = -4;
                r.logdet = r.mu = r.sigma2 = r.nll = NAN;
                r.ir_iters = 0;
            }
            ++m;
        }
        sv->arena.release(st.off, st.bytes);
        sv->in_flight -= st.B;
        st.busy = false;
    }
    // 2. admit queued work, oldest first
    auto dataset_of = [sv](size_t q) { return sv->pending[q].dataset; };
    for (auto &st : sv->streams) {
        if (st.busy) continue;
        if (sv->pending.empty()) break;
        if (sv->ragged) {
            std::vector<size_t> taken = choose_ragged_batch(
                sv->pending.size(), dataset_of, [sv](int k) { return sv->ds[k].n; },
                sv->max_batch, RAGGED_DATASETS);
            // shrunk (newest out) until its footprint fits
            bool launched = false;
            while (!taken.empty()) {
                std::vector<gp_request> batch;
                for (size_t q : taken) batch.push_back(sv->pending[q]);
                if (launch_ragged(sv, st, batch)) {
                    launched = true;
                    break;
                }
                taken.pop_back();
            }
            if (!launched) break;   // the oldest request waits for memory
            std::deque<gp_request> rest;
            size_t ti = 0;
            for (size_t q = 0; q < sv->pending.size(); ++q) {
                if (ti < taken.size() && taken[ti] == q) {
                    ++ti;
                    continue;
                }
                rest.push_back(sv->pending[q]);
            }
            sv->pending.swap(rest);
            continue;
        }
        const int k = sv->pending.front().dataset;
        std::vector<size_t> taken = choose_dataset_batch(sv->pending.size(), dataset_of,
                                                         sv->max_batch);
        std::vector<gp_request> batch;
        for (size_t q : taken) batch.push_back(sv->pending[q]);
        // shrink the batch until its footprint fits the free arena space
        bool launched = false;
        while (!batch.empty()) {
            if (launch_batch(sv, st, k, batch)) {
                launched = true;
                break;
            }
            batch.pop_back();
            taken.pop_back();
        }
        if (!launched) break;   // the oldest request waits for memory
        for (size_t q = taken.size(); q-- > 0;) sv->pending.erase(sv->pending.begin() + (long)taken[q]);
    }
    return m;
}

int64_t gp_server_outstanding(const gp_server *sv) { return sv ? sv->in_flight : -1; }

size_t gp_server_arena_used(const gp_server *sv) { return sv ? sv->arena.used() : 0; }

gp_status gp_server_destroy(gp_server *sv)
{
    if (!sv) return GP_EINVAL;
    for (auto &st : sv->streams) {
        if (st.s) (void)hipStreamSynchronize(st.s);
        if (st.exec) (void)hipGraphExecDestroy(st.exec);
        if (st.done) (void)hipEventDestroy(st.done);
        if (st.s) {
            release_side_streams(st.s);
            (void)hipStreamDestroy(st.s);
        }
        if (st.h_theta) (void)hipHostFree(st.h_theta);
        if (st.h_out) (void)hipHostFree(st.h_out);
    }
    delete sv;
    return GP_OK;
}

}  // extern "C"
