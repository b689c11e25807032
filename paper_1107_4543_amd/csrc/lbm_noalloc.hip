// Allocation-free FP64 diagnostics of a raw lattice state.
//
// lbm_diagnostics reduces over a lattice's state with per-workgroup partial
// sums held in the reduction scratch of the lattice's workspace.  This
// variant takes the raw state itself (the layout lbm_save_state writes) and
// keeps the partial sums in a fixed device array of this library instead, so
// a caller that cannot allocate -- code under HIP graph capture, a tight
// serving loop -- can reduce a state it already holds without creating a
// lattice or a workspace.  Results go to device memory and nothing waits.
//
// The array is `scratch` below; each GPU the library runs on holds its own
// copy at its own address until the process ends.  Host code never passes
// the array's name to a kernel (on the host it only stands for the
// symbol): on the first call on a device, with that device current, the
// device address of that device's copy is looked up once with
// hipGetSymbolAddress and kept per device; kernels receive that address.
#include <mutex>

#include "lbm_internal.hpp"

namespace {

// Partial rows of the fixed-grid two-pass reduction (lbm::kRedBlocks rows of
// four doubles for the diagnostics; the whole reduction block of a workspace
// is reserved).  The need does not grow with the lattice: every lattice the
// library accepts fits.
constexpr size_t kNoallocScratchBytes = lbm::kScratchBytes;
static_assert((size_t)lbm::kRedBlocks * 4 * sizeof(double) <= kNoallocScratchBytes,
              "diagnostics partials must fit the scratch array");

static __device__ __align__(256) char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];      // device address of each GPU's copy
std::mutex g_scratch_mu;

lbm_status noalloc_fail(lbm_status st, const char *msg)
{
    lbm::set_error_text(msg);
    return st;
}

// Device address of the current device's copy of `scratch` (looked up on
// the first call on each device).
lbm_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return noalloc_fail(LBM_E_HIP, "hipGetDevice failed");
    if (dev >= kMaxDevices) return noalloc_fail(LBM_E_INVAL, "device index beyond the supported 64 devices");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return noalloc_fail(LBM_E_HIP, "hipGetSymbolAddress(scratch) failed");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

// The collision-invariant sums in stored units times 2^-p (the count stays).
__global__ void k_unscale_sums(double *out, double inv_scale)
{
    if (threadIdx.x < 3) out[threadIdx.x] *= inv_scale;
}

}  // namespace

extern "C" lbm_status lbm_diagnostics_noalloc(const lbm_desc *desc, const void *dev_state, double *dev_out,
                                              void *stream)
{
    if (!desc || !dev_state || !dev_out) return noalloc_fail(LBM_E_INVAL, "NULL argument");
    lbm::View v;
    lbm_status st = lbm::view_of_state(desc, &v);
    if (st != LBM_OK) return st;
    void *ptr = nullptr;
    if ((st = scratch_address(&ptr)) != LBM_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    // the partial rows are all rewritten before they are summed: nothing to clear
    hipError_t e = lbm::launch_diagnostics(v, dev_state, (double *)ptr, dev_out, s);
    if (e == hipSuccess && v.inv_scale != 1.0) {
        hipLaunchKernelGGL(k_unscale_sums, dim3(1), dim3(64), 0, s, dev_out, v.inv_scale);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        lbm::set_error_text(hipGetErrorString(e));
        return LBM_E_HIP;
    }
    return LBM_OK;
}
