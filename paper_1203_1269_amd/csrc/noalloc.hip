// gp_nll_batch_noalloc: gp_nll_batch for callers that cannot allocate
// device memory (code under stream capture, tight serving loops).  The
// workspace is a fixed array in the library's own device memory instead of a
// caller buffer.
//
// `scratch` is a file-scope device array; the runtime gives each GPU its own
// copy when the code object is loaded there.  Its host-side name is only a
// symbol handle, so host code never passes it to a kernel: on the first call
// on a device (that device current) hipGetSymbolAddress yields the device
// address of that GPU's copy, which is kept per device and used for every
// launch.  Calls on one GPU share the array: calls that overlap on one GPU
// (on different streams, or from different host threads) race, and every
// call overwrites what the previous one left.  Nothing in it has to start at
// zero: every byte a call reads is written earlier in the same call (the
// matrices, per-theta state and residues), except residue rows past the
// matrix, which are read and never used.
#include <mutex>

#include "kernels.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[GP_NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;

// device address of `scratch` on the current device, nullptr on failure
void *scratch_ptr()
{
    static std::once_flag once[MAX_DEVICES];
    static void *ptr[MAX_DEVICES];
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::call_once(once[dev], [dev] {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) ptr[dev] = p;
    });
    return ptr[dev];
}

}  // namespace

extern "C" {

gp_status gp_nll_batch_noalloc(const gp_dataset *ds, int32_t batch, const double *theta,
                               int32_t prec, gp_result *out, hipStream_t stream)
{
    if (!gpk::dataset_valid(ds) || batch < 1 || batch > GP_BATCH_MAX || !theta || !out)
        return GP_EINVAL;
    const size_t need = gp_workspace_bytes(ds->n, ds->d, batch, prec);
    if (need == 0) return GP_EINVAL;
    if (need > (size_t)GP_NOALLOC_BYTES) return GP_EWORKSPACE;
    void *ws = scratch_ptr();
    if (!ws) return GP_ELAUNCH;
    // no lookahead: the factorisation then needs no library-created streams
    return gpk::nll_batch_impl(ds, batch, theta, prec, ws, (size_t)GP_NOALLOC_BYTES, out, stream,
                               false);
}

}  // extern "C"
