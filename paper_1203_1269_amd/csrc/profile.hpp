// Optional per-launch timing: when enabled with gp_profile_begin(), every
// kernel launch is bracketed by two hipEvents on its own stream and tagged
// with the algorithmic FLOPs and HBM bytes of that launch.  Disabled, the
// scope objects cost one branch.
#pragma once
#include <hip/hip_runtime.h>

namespace gpk {

enum KernelKind {
    K_INIT = 0,
    K_CORR_BUILD,
    K_POTRF_DIAG,
    K_TRSM_PANEL,
    K_SYRK_UPDATE,
    K_SYRK_PANEL,
    K_SYRK_UPDATE_F32,
    K_SOLVE_REDUCE,
    K_PAD,
    K_LOGDET_SUM,
    K_BORDER,
    K_ALPHA,
    K_ADJOINT,
    K_RESIDUAL,
    K_SOLVE2,
    K_PRED_ROWS,
    K_PRED_REDUCE,
    K_CRT_SPLIT,
    K_SYRK_UPDATE_CRT,
    K_NUM_KINDS
};

extern const char *const kKindNames[K_NUM_KINDS];

bool prof_enabled();
void prof_record_begin(int kind, double flops, double bytes, hipStream_t s);
void prof_record_end(hipStream_t s);

struct ProfScope {
    hipStream_t s;
    bool on;
    ProfScope(int kind, double flops, double bytes, hipStream_t st) : s(st), on(prof_enabled())
    {
        if (on) prof_record_begin(kind, flops, bytes, s);
    }
    ~ProfScope()
    {
        if (on) prof_record_end(s);
    }
};

}  // namespace gpk
