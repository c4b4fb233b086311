// Uneven-n batching in one call: thetas for several resident datasets (any
// n, d and correlation family).  The paper could run only one evaluation at
// a time (Sec. 3); here unrelated evaluations share the GPU.
//
// FP64: one ragged batch.  Every theta gets a matrix of its own order
// (n_pad of its dataset) packed one after the other in the workspace and a
// descriptor (RagMat) with its offset, order, n and y.  The correlation
// build runs per dataset (the |x_i - x_j|^p terms are shared by that
// dataset's thetas); then ONE launch sequence factors and solves every
// matrix, so the panel chains of all requests advance together in the same
// kernels.  The matrices are taken in order of decreasing order, so a launch
// at column c covers only the leading matrices that still reach past c; in
// the trailing updates each matrix's own tiles are shared out evenly over
// the XCDs.
// Mixed modes: the per-dataset batches are spread over a small pool of
// streams that fork from and join back into the caller's stream.
//
// The per-theta arithmetic is that of gp_nll_batch (every kernel works per
// theta, with the same tiles, blocking and order of operations for a matrix
// whatever the others in the launch), so each result is bitwise the one
// gp_nll_batch gives for that dataset and theta.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "kernels.hpp"

namespace gpk {
namespace {

constexpr int MULTI_LANES = 8;

// Lanes (streams) plus fork/join events for one caller stream, created on
// first use per (device, caller stream) and kept for the life of the
// process.  Default priority, non-blocking.  At most MULTI_CALLERS caller
// streams get lanes; calls on further streams run their groups on the
// caller's stream, so a caller that cycles through new streams does not make
// the library create streams without bound.
constexpr size_t MULTI_CALLERS = 32;
struct Lanes {
    hipStream_t s[MULTI_LANES] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[MULTI_LANES] = {};
    bool ok = false;
};

Lanes *lanes_for(hipStream_t caller)
{
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, Lanes> table;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(dev, caller);
    auto it = table.find(key);
    if (it != table.end()) return it->second.ok ? &it->second : nullptr;
    if (table.size() >= MULTI_CALLERS) return nullptr;
    Lanes L;
    bool ok = hipEventCreateWithFlags(&L.fork, hipEventDisableTiming) == hipSuccess;
    for (int l = 0; ok && l < MULTI_LANES; ++l)
        ok = hipStreamCreateWithFlags(&L.s[l], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&L.join[l], hipEventDisableTiming) == hipSuccess;
    L.ok = ok;   // on failure: remembered, the groups then run on the caller's stream
    table[key] = L;
    return ok ? &table[key] : nullptr;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct RagChunk {
    RagMat m[RAG_CHUNK];
};

__global__ void rag_fill_kernel(RagMat *__restrict__ dst, RagChunk src, int count)
{
    const int i = threadIdx.x;
    if (i < count) dst[i] = src.m[i];
}

// Workspace of a ragged FP64 batch: descriptors, the matrices (each of its
// own order, back to back), log-det partials, info, the TRSM diagonal
// copies and the solve state (the last three at the largest order).
struct RagLayout {
    int B = 0, npmax = 0;
    size_t rag, mat, lpart, info, lk, z, total;
    std::vector<size_t> goff;   // first matrix of dataset k, in doubles from mat
};

bool rag_layout(const gp_dataset *ds, int nds, const int32_t *counts, RagLayout &L)
{
    L.goff.assign(nds, 0);
    size_t dbl = 0;   // doubles of matrices
    long B = 0;
    for (int k = 0; k < nds; ++k) {
        if (counts[k] <= 0) continue;
        const int np = pad64(ds[k].n);
        L.goff[k] = dbl;
        dbl += (size_t)counts[k] * np * np;
        dbl = (dbl + 31) & ~(size_t)31;   // 256-byte aligned groups
        L.npmax = std::max(L.npmax, np);
        B += counts[k];
    }
    if (B < 1 || B > GP_BATCH_MAX) return false;
    L.B = (int)B;
    size_t off = 0;
    L.rag = off;
    off = align256(off + sizeof(RagMat) * B);
    L.mat = off;
    off = align256(off + sizeof(double) * dbl);
    L.lpart = off;
    off = align256(off + sizeof(double) * (size_t)(L.npmax / TB) * B);
    L.info = off;
    off = align256(off + sizeof(int32_t) * B);
    L.lk = off;
    off = align256(off + sizeof(double) * TB * TB * B);
    L.z = off;
    off = align256(off + sizeof(double) * 2 * (size_t)L.npmax * B);
    L.total = off;
    return true;
}

}  // namespace

void launch_rag_fill(RagMat *rag, const RagMat *src, int count, hipStream_t s)
{
    RagChunk c;
    memset(&c, 0, sizeof(c));
    memcpy(c.m, src, sizeof(RagMat) * count);
    rag_fill_kernel<<<1, RAG_CHUNK, 0, s>>>(rag, c, count);
}

size_t ragged_workspace_bytes(const gp_dataset *ds, int32_t nds, const int32_t *counts)
{
    RagLayout L;
    return rag_layout(ds, nds, counts, L) ? L.total : 0;
}

// One ragged FP64 batch: thetas packed per dataset in order (counts[k] of
// dataset k, d_k values each), results in the same order.  Arguments are
// checked by the caller.
gp_status nll_ragged_impl(const gp_dataset *ds, int32_t nds, const int32_t *counts,
                          const double *theta, void *ws, size_t ws_bytes, gp_result *out,
                          hipStream_t stream, bool lookahead)
{
    RagLayout L;
    if (!rag_layout(ds, nds, counts, L)) return GP_EINVAL;
    if (ws_bytes < L.total) return GP_EWORKSPACE;
    char *base = (char *)ws;
    RagMat *rag = (RagMat *)(base + L.rag);
    double *A = (double *)(base + L.mat);
    double *lpart = (double *)(base + L.lpart);
    int32_t *info = (int32_t *)(base + L.info);

    // caller order: dataset by dataset, theta offsets and result indices
    std::vector<size_t> toff(nds);
    std::vector<int> ooff(nds);
    std::vector<int> order;
    size_t t = 0;
    int o = 0;
    for (int k = 0; k < nds; ++k) {
        toff[k] = t;
        ooff[k] = o;
        t += (size_t)counts[k] * ds[k].d;
        o += counts[k];
        if (counts[k] > 0) order.push_back(k);
    }
    // launch order: datasets by decreasing n_pad (ties in dataset order)
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pad64(ds[a].n) > pad64(ds[b].n); });

    // descriptors, in chunks through kernel arguments, and the host copy of
    // the orders
    std::vector<int32_t> hlive;
    hlive.reserve(L.B);
    RagMat chunk[RAG_CHUNK];
    int filled = 0, q = 0;
    for (int k : order) {
        const int np = pad64(ds[k].n);
        for (int j = 0; j < counts[k]; ++j) {
            RagMat &m = chunk[q++];
            m.off = L.goff[k] + (size_t)j * np * np;
            m.lda = np;
            m.live = np;
            m.n = ds[k].n;
            m.dst = ooff[k] + j;
            m.y = ds[k].y;
            hlive.push_back(np);
            if (q == RAG_CHUNK) {
                launch_rag_fill(rag + filled, chunk, q, stream);
                filled += q;
                q = 0;
            }
        }
    }
    if (q) launch_rag_fill(rag + filled, chunk, q, stream);

    // theta checks and R_delta per dataset, each block homogeneous
    int first = 0;
    for (int k : order) {
        const gp_dataset &d = ds[k];
        const int np = pad64(d.n);
        launch_init(theta + toff[k], d.d, counts[k], info + first, stream);
        launch_corr_build(d.X, d.n, d.d, family_p(&d), d.delta, theta + toff[k], counts[k],
                          A + L.goff[k], np, (size_t)np * np, np, stream);
        first += counts[k];
    }
    SolvePlan plan{nullptr, 0, (double *)(base + L.z), out, rag};
    factor_batch(A, L.npmax, 0, L.npmax, L.B, info, lpart, (double *)(base + L.lk), stream,
                 GP_FP64, false, nullptr, nullptr, nullptr, lookahead, 0, &plan, rag,
                 hlive.data());
    return hipGetLastError() == hipSuccess ? GP_OK : GP_ELAUNCH;
}

}  // namespace gpk

using namespace gpk;

extern "C" {

size_t gp_multi_workspace_bytes(const gp_dataset *ds, int32_t nds, const int32_t *counts,
                                int32_t prec)
{
    if (!ds || !counts || nds < 1) return 0;
    if (prec == GP_FP64) {
        long B = 0;
        for (int k = 0; k < nds; ++k) {
            if (counts[k] < 0) return 0;
            if (counts[k] > 0 && gp_workspace_bytes(ds[k].n, ds[k].d, 1, prec) == 0) return 0;
            B += counts[k];
        }
        if (B == 0) return 256;
        return ragged_workspace_bytes(ds, nds, counts);
    }
    size_t total = 0;
    for (int k = 0; k < nds; ++k) {
        if (counts[k] < 0) return 0;
        if (counts[k] == 0) continue;
        const size_t b = gp_workspace_bytes(ds[k].n, ds[k].d, counts[k], prec);
        if (b == 0) return 0;
        total += align256(b);
    }
    return total ? total : 256;
}

gp_status gp_nll_multi(const gp_dataset *ds, int32_t nds, const int32_t *counts,
                       const double *theta, int32_t prec, void *ws, size_t ws_bytes,
                       gp_result *out, hipStream_t stream)
{
    if (!ds || !counts || nds < 1 || !ws || ((uintptr_t)ws & 255) != 0) return GP_EINVAL;
    long total = 0;
    for (int k = 0; k < nds; ++k) {
        if (counts[k] < 0 || counts[k] > GP_BATCH_MAX) return GP_EINVAL;
        if (counts[k] > 0 && !dataset_valid(&ds[k])) return GP_EINVAL;
        total += counts[k];
    }
    if (total > 0 && (!theta || !out)) return GP_EINVAL;
    const size_t need = gp_multi_workspace_bytes(ds, nds, counts, prec);
    if (need == 0) return GP_EINVAL;
    if (ws_bytes < need) return GP_EWORKSPACE;
    if (total == 0) return GP_OK;
    if (prec == GP_FP64)
        return nll_ragged_impl(ds, nds, counts, theta, ws, ws_bytes, out, stream, true);

    // largest work first, each onto the lane with the least work so far
    // (work ~ count * n^3); ties in order of the datasets
    std::vector<int> order;
    for (int k = 0; k < nds; ++k)
        if (counts[k] > 0) order.push_back(k);
    auto cost = [&](int k) { return (double)counts[k] * ds[k].n * ds[k].n * ds[k].n; };
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<size_t> woff(nds), toff(nds), ooff(nds);
    size_t w = 0, t = 0, o = 0;
    for (int k = 0; k < nds; ++k) {
        woff[k] = w;
        toff[k] = t;
        ooff[k] = o;
        if (counts[k] > 0) w += align256(gp_workspace_bytes(ds[k].n, ds[k].d, counts[k], prec));
        t += (size_t)counts[k] * ds[k].d;
        o += counts[k];
    }

    Lanes *L = lanes_for(stream);
    double load[MULTI_LANES] = {};
    bool used[MULTI_LANES] = {};
    if (L) {
        if (hipEventRecord(L->fork, stream) != hipSuccess) return GP_ELAUNCH;
    }
    gp_status rc = GP_OK;
    for (int k : order) {
        hipStream_t st = stream;
        if (L) {
            int lane = 0;
            for (int l = 1; l < MULTI_LANES; ++l)
                if (load[l] < load[lane]) lane = l;
            load[lane] += cost(k);
            if (!used[lane]) {
                (void)hipStreamWaitEvent(L->s[lane], L->fork, 0);
                used[lane] = true;
            }
            st = L->s[lane];
        }
        const gp_status r = nll_batch_impl(&ds[k], counts[k], theta + toff[k], prec,
                                           (char *)ws + woff[k],
                                           align256(gp_workspace_bytes(ds[k].n, ds[k].d,
                                                                       counts[k], prec)),
                                           out + ooff[k], st, false);
        if (r != GP_OK && rc == GP_OK) rc = r;
    }
    if (L) {
        for (int l = 0; l < MULTI_LANES; ++l)
            if (used[l]) {
                (void)hipEventRecord(L->join[l], L->s[l]);
                (void)hipStreamWaitEvent(stream, L->join[l], 0);
            }
    }
    return rc;
}

}  // extern "C"
