// Uneven-n batching in one call: thetas for several resident datasets (any
// n, d and correlation family) are evaluated as one batch per dataset, the
// per-dataset batches spread over a small pool of streams that fork from
// and join back into the caller's stream.  The paper could run only one
// evaluation at a time (Sec. 3); here unrelated evaluations share the GPU,
// so the short kernels of small problems fill the gaps of large ones.
//
// The per-theta arithmetic is that of gp_nll_batch (every kernel works per
// theta), so each result is bitwise the one gp_nll_batch gives for that
// dataset and theta.
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

}  // namespace
}  // namespace gpk

using namespace gpk;

extern "C" {

size_t gp_multi_workspace_bytes(const gp_dataset *ds, int32_t nds, const int32_t *counts,
                                int32_t prec)
{
    if (!ds || !counts || nds < 1) return 0;
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
