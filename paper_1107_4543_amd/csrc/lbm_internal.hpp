// Internal interface between the C ABI/runtime (lbm_api.hip) and the kernels
// (lbm_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

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

constexpr int kWgHalo = 32;        // launch-flags bit of the workgroup-shared halo (variants 10-13)
constexpr int kWgMaxWaves = 4;     // waves per workgroup it supports
// With kWgHalo in a pool's T-step kernel: workgroups of two waves (strips of
// 128 - 2(T-1) columns, for the columns a member has left over after its
// four-wave strips); not a launch flag of a single lattice.
constexpr int kWgTwo = 64;
constexpr int kRedBlocks = 512;    // blocks of the two-pass reductions
constexpr int kRedWidth = 20;      // max doubles per block partial
constexpr size_t kScratchBytes = (size_t)kRedBlocks * kRedWidth * sizeof(double) + 64 * sizeof(double);

size_t storage_bytes(int32_t storage);
bool step_shape_supported(const View &v, const lbm_launch &cfg);
// Steps one launch of this shape advances (several-steps-per-pass variants).
int steps_per_launch(const lbm_launch &cfg);
// Output columns of a T-step strip run by `lanes` lanes (one wave: 64; a
// workgroup with the shared halo: 64 per wave) for a storage element of
// elem_bytes.
int multi_strip_cols(int T, int elem_bytes, int lanes = 64);

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

// Sets the pre-collision populations of cell (x, y) to f^eq(rho, rho u).
hipError_t launch_set_node(const View &v, void *dst, int32_t x, int32_t y, double rho, double ux, double uy,
                           hipStream_t st);

// ---- batched stepping (pool) --------------------------------------------------

// Storage/compute class of a lattice: storage * 2 + compute (8 values).
constexpr int kClasses = 8;
// The members of one class are split into kChains groups whose launches form
// independent chains in a recorded step loop (members never read each
// other's state), so one group's launch can start while another's is still
// ending.  Table range of a group: class * kChains + chain.
constexpr int kChains = 2;
constexpr int kRanges = kClasses * kChains;

// Device-resident member record.  t_done advances on the device (commit
// kernel) so that a recorded step loop stays valid while members come and go.
struct PoolMember {
    const void *buf[2];
    int32_t nx, ny, pitch, cur0;   // cur0: buffer holding the state when added
    int64_t plane;
    int64_t t_done, t_target;      // steps done since added / steps requested
    int64_t flips;                 // launches since added (buffer swaps)
    Relax<float> rf;
    Relax<double> rd;
    float scale, inv_scale;
    int32_t cls, pad;
};

// A tile of one member: rows y0 .. y0+nrows-1, columns x0 .. x0+ncols-1
// (whole rows when the lattice is narrower than the tile size, otherwise a
// segment of one row).  T-step strip tasks use the same record (one wave
// each, or with the shared halo one workgroup each).
struct PoolTile {
    int32_t member, y0, x0, nrows, ncols, pad0, pad1, pad2;
};

struct PoolHeader {
    int32_t begin[kRanges], end[kRanges];       // one-step tiles of each range
    int32_t mbegin[kRanges], mend[kRanges];     // T-step strip tasks of each range
    int32_t hbegin[kRanges], hend[kRanges];     // T-step two-wave strip tasks (kWgTwo) of each range
};

// Launch schedule of a recorded chunk of kk steps with T steps per T-step
// launch: floor(kk / T) T-step launches, then at most T - 1 one-step
// launches (as many as the members need; chunk_single_launches bounds it).  A
// member with rem steps left takes q = min(rem / T, kk / T) T-step launches
// and span - q T one-step launches, span = min(rem, kk): kk mod T (< T) if
// it stays, rem mod T (< T) if it finishes in the chunk.  Its source buffer
// alternates with every launch it takes.
__host__ __device__ inline int chunk_multi_launches(int kk, int T) { return T > 1 && kk >= T ? kk / T : 0; }
__host__ __device__ inline int chunk_single_launches(int kk, int T) { return T > 1 && kk >= T ? T - 1 : kk; }
__host__ __device__ inline int64_t member_multi(int64_t rem, int kk, int T)
{
    const int64_t a = rem / T, b = chunk_multi_launches(kk, T);
    return T > 1 ? (a < b ? a : b) : 0;
}

// Sets the text returned by lbm_last_error() on the calling thread.
void set_error_text(const char *msg);

// Compute units of the current device (256 on MI355X).
int device_cus();

// Fills *v for a raw state of the lattice that desc describes (validated as
// by lbm_create; 16-bit storage needs an explicit scale_exp).  Sets the
// error text on failure.
lbm_status view_of_state(const lbm_desc *desc, View *v);

Relax<float> relax_f32(const View &v);
Relax<double> relax_f64(const View &v);

// One-step launch i of a chunk of kk steps (schedule above) of every active
// member of class cls.
hipError_t launch_pool_step(int range, const PoolHeader *hdr, const PoolMember *mem, const PoolTile *tiles, int i,
                            int kk, int T, int grid, int block, hipStream_t st);
// T-step launch j of a chunk of every active member of table range `range`.
hipError_t launch_pool_multi(int range, int T, int flags, const PoolHeader *hdr, const PoolMember *mem,
                             const PoolTile *tiles, int j, int grid, int waves, hipStream_t st);
// t_done += span and flips += q + span - q T (schedule above) for members [0, nmem).
hipError_t launch_pool_commit(PoolMember *mem, int nmem, int kk, int T, hipStream_t st);
// Kernel entry points for graph nodes, by class (nullptr if not
// instantiated); their range argument selects the table range.
void *pool_step_kernel(int cls);
void *pool_multi_kernel(int cls, int T, int flags);
void *pool_commit_kernel();

}  // namespace lbm

struct lbm_pool;

// Host handle of one lattice (defined here so that the pool can drive it).
struct lbm_lattice {
    lbm::View v;
    lbm_desc desc;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    size_t buf_bytes = 0;      // bytes of one buffer (aligned)
    size_t state_bytes = 0;    // bytes of one buffer's planes (exact)
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    double *partials = nullptr;
    double *result = nullptr;
    hipStream_t stream = nullptr;
    int64_t t = 0;
    bool initialized = false;
    lbm_launch launch{};
    lbm_launch single{};       // one-step shape for the steps a multi-step shape leaves over
    lbm_pool *pool = nullptr;  // non-NULL while a pool advances this lattice
};
