// Allocation-free variant of md_forces_lj for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// md_forces_lj keeps its per-block energy and virial partials (8 doubles per
// block of kBlock / kSlice = 32 atoms) in the caller's workspace.  Here they
// live in a file-scope device array, one copy per GPU, held until the
// process ends.  The array's host-side name is only a stand-in: its device
// address is taken once per device with hipGetSymbolAddress and only that
// address is handed to kernels.  No call allocates or frees memory.
#include <mutex>

#include "md_common.h"

namespace md {

constexpr int64_t kNoAllocRows = MD_NOALLOC_MAX_ATOMS / (kBlock / kSlice);   // partial rows

static __device__ __align__(256) double scratch[kNoAllocRows * 8];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first
// call on each device, with that device current).
int scratch_of_current_device(double **out)
{
    int dev = -1;
    MD_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MD_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return MD_ERR_HIP;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return MD_OK;
}

}  // namespace
}  // namespace md

using namespace md;

extern "C" int md_forces_lj_noalloc(const md_box_t *box, int64_t n, const double *x, const uint32_t *xs,
                                    int32_t row_cap, const int32_t *idx, const int32_t *count, const md_lj_t *lj,
                                    void *f, double *ev, int32_t flags, void *stream)
{
    if (int rc = lj_args_check(box, n, x, xs, row_cap, idx, count, lj, f, ev, flags)) return rc;
    if ((flags & MD_ENERGY) && n > MD_NOALLOC_MAX_ATOMS) return MD_ERR_ARG;
    double *part = nullptr;
    if (int rc = scratch_of_current_device(&part)) return rc;
    // every block of the force kernel writes its whole partial row before
    // the reduction reads it: nothing in the array has to start at zero
    return forces_lj_part(box, n, x, xs, row_cap, idx, count, lj, f, ev, flags, part, kNoAllocRows,
                          static_cast<hipStream_t>(stream));
}
