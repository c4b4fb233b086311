// Per-launch event timing behind gp_profile_begin / gp_profile_end.
// Not thread-safe: one host thread drives the library while profiling.
#include <string.h>

#include <vector>

#include "gpnll.h"
#include "profile.hpp"

namespace gpk {

const char *const kKindNames[K_NUM_KINDS] = {
    "init", "corr_build", "potrf_diag", "trsm_panel", "syrk_update", "syrk_panel",
    "syrk_update_f32", "solve_reduce", "pad_identity", "logdet_sum", "border_init", "alpha", "adjoint", "residual", "solve2",
    "pred_rows", "pred_reduce", "crt_split", "syrk_update_crt"};

namespace {

struct Rec {
    int kind;
    double flops, bytes;
    hipEvent_t e0, e1;
};

bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_used = 0;
size_t g_cap = 0;
bool g_overflow = false;

hipEvent_t take_event()
{
    if (g_used >= g_pool.size()) return nullptr;
    return g_pool[g_used++];
}

}  // namespace

bool prof_enabled() { return g_on; }

void prof_record_begin(int kind, double flops, double bytes, hipStream_t s)
{
    hipEvent_t e0 = take_event();
    if (!e0) { g_overflow = true; return; }
    (void)hipEventRecord(e0, s);
    g_recs.push_back(Rec{kind, flops, bytes, e0, nullptr});
}

void prof_record_end(hipStream_t s)
{
    if (g_recs.empty() || g_recs.back().e1 != nullptr || g_recs.back().e0 == nullptr) return;
    hipEvent_t e1 = take_event();
    if (!e1) { g_overflow = true; g_recs.pop_back(); return; }
    (void)hipEventRecord(e1, s);
    g_recs.back().e1 = e1;
}

}  // namespace gpk

using namespace gpk;

extern "C" {

gp_status gp_profile_begin(int32_t max_launches)
{
    if (max_launches < 1) return GP_EINVAL;
    for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
    g_pool.clear();
    g_recs.clear();
    g_recs.reserve(max_launches);
    g_pool.resize((size_t)2 * max_launches, nullptr);
    for (auto &e : g_pool)
        if (hipEventCreate(&e) != hipSuccess) return GP_ELAUNCH;
    g_used = 0;
    g_cap = g_pool.size();
    g_overflow = false;
    g_on = true;
    return GP_OK;
}

int32_t gp_profile_end(gp_kernel_stat *stats, int32_t max_stats)
{
    if (!g_on) return GP_EINVAL;
    g_on = false;
    gp_kernel_stat acc[K_NUM_KINDS];
    memset(acc, 0, sizeof(acc));
    for (int k = 0; k < K_NUM_KINDS; ++k) strncpy(acc[k].name, kKindNames[k], sizeof(acc[k].name) - 1);
    int32_t status = 0;
    for (const Rec &r : g_recs) {
        if (!r.e1) continue;
        if (hipEventSynchronize(r.e1) != hipSuccess) { status = GP_ELAUNCH; break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) { status = GP_ELAUNCH; break; }
        acc[r.kind].launches += 1;
        acc[r.kind].ms += ms;
        acc[r.kind].flops += r.flops;
        acc[r.kind].bytes += r.bytes;
    }
    for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
    g_pool.clear();
    g_recs.clear();
    if (status != 0) return status;
    if (g_overflow) return GP_EWORKSPACE;
    int32_t m = 0;
    for (int k = 0; k < K_NUM_KINDS && m < max_stats; ++k)
        if (acc[k].launches > 0 && stats) stats[m++] = acc[k];
    return m;
}

}  // extern "C"
