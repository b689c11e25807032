// Internal interface between the C ABI/runtime (lbm_api.hip) and the kernels
// (lbm_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {

// Everything a kernel launcher needs to know about one lattice.
struct View {
    int32_t nx, ny, pitch;
    int32_t storage, compute;
    int32_t scale_exp;
    int64_t plane;            // elements per population plane (= pitch * ny)
    double s_e, s_eps, s_q, s_nu;
    double rho0, j0x, j0y;    // base state (j0 = rho0 u0)
    double fbase[9];          // f^eq(rho0, j0), FP64
    double scale, inv_scale;  // 2^p, 2^-p
};

constexpr int kRedBlocks = 512;    // blocks of the two-pass reductions
constexpr int kRedWidth = 20;      // max doubles per block partial
constexpr size_t kScratchBytes = (size_t)kRedBlocks * kRedWidth * sizeof(double) + 64 * sizeof(double);

size_t storage_bytes(int32_t storage);
bool step_shape_supported(const View &v, const lbm_launch &cfg);

hipError_t launch_step(const View &v, const void *src, void *dst, const lbm_launch &cfg,
                       hipStream_t st);
// measure_only: compute max |g| (before scaling) into result[0], store nothing.
hipError_t launch_init(const View &v, const double *rho, const double *ux, const double *uy,
                       void *dst, double *partials, double *result, bool measure_only,
                       hipStream_t st);
hipError_t launch_moments(const View &v, const void *src, double *rho, double *ux, double *uy,
                          hipStream_t st);
hipError_t launch_read_populations(const View &v, const void *src, double *f, hipStream_t st);
hipError_t launch_write_populations(const View &v, const double *f, void *dst, hipStream_t st);
// result[0..3] = sum rho', sum jx', sum jy', non-finite count
hipError_t launch_diagnostics(const View &v, const void *src, double *partials, double *result,
                              hipStream_t st);
// out[0..17] = projection on mode (mx, my)
hipError_t launch_project(const View &v, const void *src, int32_t mx, int32_t my,
                          double *partials, double *out, hipStream_t st);

}  // namespace lbm
