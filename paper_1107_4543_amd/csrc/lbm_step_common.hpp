// Device building blocks shared by the library's kernel translation units:
// the step kernels' arguments, per-cell update, addressing through raw buffer
// resources, and the several-steps-per-pass strip pipeline with its kernels
// (single lattice and pool).  The several-steps kernels are instantiated per
// storage type in lbm_multi_<type>.hip, so that the translation units compile
// in parallel.
//
// Layout.  Structure of arrays: population i of row y at x lives at
// buf[i * plane + y * pitch + x], pitch = nx rounded up to 64 elements, two
// buffers (ping-pong).  The stored field is the post-collision deviation of
// the previous step, not yet streamed:  P_i(y) = g*_i(y, t-1), so that the
// pre-collision deviation at time t is g_i(x, t) = P_i(x - v_i)
// (pull streaming, Sec. 2.2, Eq. l-mrt-lbs).  One step therefore reads the
// nine pulled values of a cell, collides them and writes the nine results
// to the same cell of the other buffer: every HBM access of the step is a
// row-contiguous, coalesced stream; only the x-shift of populations with
// v_x != 0 is misaligned by one element.
#pragma once

#include <math.h>

#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {

template <typename C>
inline Relax<C> make_relax(const View &v)
{
    Relax<C> r;
    r.lam_e = (C)(v.s_e / 36.0);
    r.lam_eps = (C)(v.s_eps / 36.0);
    r.lam_q = (C)(v.s_q / 12.0);
    r.lam_nu = (C)(v.s_nu / 4.0);
    r.rho0 = (C)v.rho0;
    r.j0x = (C)v.j0x;
    r.j0y = (C)v.j0y;
    r.Q0 = (C)((v.j0x * v.j0x + v.j0y * v.j0y) / v.rho0);
    r.P0 = (C)((v.j0x * v.j0x - v.j0y * v.j0y) / v.rho0);
    r.X0 = (C)(v.j0x * v.j0y / v.rho0);
    return r;
}

template <typename C>
struct StepArgs {
    const void *src;
    void *dst;
    int32_t nx, ny, pitch, tiles_x;
    int32_t tile_h, rows, nblocks, xcd_remap;
    int32_t nwaves, out_cols;
    int64_t plane;
    Relax<C> r;
    float scale, inv_scale;
};


// Launches the several-steps kernel with T steps per pass and the given
// flags (instantiated per storage type in lbm_multi_<type>.hip).
template <typename S, typename C>
hipError_t launch_multi(const StepArgs<C> &a, dim3 grid, dim3 block, int T, int flags, hipStream_t st);
// The pool's several-steps kernel for T and flags, or nullptr.
template <typename S, typename C>
void *pool_multi_fn(int T, int flags);

#define LBM_DECLARE_MULTI(S_, C_)                                                                         \
    template <>                                                                                           \
    hipError_t launch_multi<S_, C_>(const StepArgs<C_> &a, dim3 grid, dim3 block, int T, int flags,      \
                                    hipStream_t st);                                                      \
    template <>                                                                                           \
    void *pool_multi_fn<S_, C_>(int T, int flags);
LBM_DECLARE_MULTI(double, double)
LBM_DECLARE_MULTI(double, float)
LBM_DECLARE_MULTI(float, float)
LBM_DECLARE_MULTI(f16_tag, float)
LBM_DECLARE_MULTI(bf16_tag, float)
#undef LBM_DECLARE_MULTI

namespace {



constexpr int VX_[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int VY_[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// MI355X dispatches consecutive workgroup ids round-robin over its 8 XCDs.
// Renumber so that each XCD receives one contiguous range of tiles: tiles
// that share misaligned cache lines then share one L2.
__device__ __forceinline__ int remap_xcd(int bid, int nb)
{
    const int xcd = bid & 7, local = bid >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Task of workgroup b among n tasks that keeps their order (longest first)
// chunk by chunk but gives each XCD (workgroups b, b + 8, ... run on XCD b
// mod 8) four consecutive tasks of every 32: adjacent strips of one lattice
// then load their shared halo columns and edge cache lines through the same
// L2.  The last partial chunk keeps the plain order.
__device__ __forceinline__ int xcd_group(int b, int n)
{
    const int c = b >> 5;
    if ((c + 1) << 5 > n) return b;
    return (c << 5) + ((b & 7) << 2) + ((b & 31) >> 3);
}

// Collide one cell held as widened stored values w (in place).  16-bit
// storage is collided in its scaled units (see collide_increment).  The
// last operation before a value is rounded to its storage type is the add
// of the increment: a fused multiply-add there could be merged with a
// 16-bit conversion into one mixed-precision instruction that rounds once
// instead of twice, and kernels that got it would no longer agree bitwise
// with those that did not.
template <typename S, typename C>
__device__ __forceinline__ void cell_update(typename Store<S>::wide w[9], const Relax<C> &r,
                                            float /*scale*/, float inv_scale)
{
    using W = typename Store<S>::wide;
    C g[9], dg[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = (C)w[i];
    collide_increment<C>(g, r, Store<S>::scaled ? (C)inv_scale : C(1), dg);
    // The rest population's increment is 4 dg[0]; scaling by 4 is exact, so
    // one multiply-add gives the same value as the product and the sum.  It
    // is used where the sum is stored as it is (the storage type is the
    // arithmetic type); before a narrowing to 16 bits the compiler could
    // merge a multiply-add with the conversion, which rounds once instead
    // of twice, so there the product and the sum stay separate operations.
    if constexpr (std::is_same<W, C>::value && !Store<S>::scaled)
        w[0] = fmad(C(4), dg[0], w[0]);
    else
        w[0] = w[0] + (W)(C(4) * dg[0]);
#pragma unroll
    for (int i = 1; i < 9; ++i) w[i] = w[i] + (W)dg[i];
}

// ---- fused step -------------------------------------------------------------

template <typename S, bool NT>
__device__ __forceinline__ typename Store<S>::wide ld(const typename Store<S>::raw *p)
{
    if constexpr (NT) return Store<S>::widen(__builtin_nontemporal_load(p));
    else return Store<S>::widen(*p);
}

// Addressing: plane i of a buffer starts at base + i * plane_bytes (a
// wave-uniform pointer); within a plane a cell is a 32-bit byte offset
// row * pitch_bytes + x * sizeof (planes are smaller than 4 GiB), which the
// hardware adds to the uniform base in the load instruction itself.
template <typename R>
__device__ __forceinline__ const R *at(const char *base, uint32_t off)
{
    return (const R *)(base + off);
}

// The nine pulled values of cell (x, y): population i comes from x - v_i.
// r0, rm, rp: byte offsets of rows y, y-1, y+1; c0, cm, cp: byte offsets of
// columns x, x-1, x+1 (wrapped).
template <typename S, bool NT>
__device__ __forceinline__ void gather9(const char *__restrict__ src, uint64_t pb, uint32_t r0, uint32_t rm,
                                        uint32_t rp, uint32_t c0, uint32_t cm, uint32_t cp,
                                        typename Store<S>::wide w[9])
{
    using R = typename Store<S>::raw;
    w[0] = ld<S, NT>(at<R>(src + 0 * pb, r0 + c0));
    w[1] = ld<S, NT>(at<R>(src + 1 * pb, r0 + cm));
    w[2] = ld<S, NT>(at<R>(src + 2 * pb, rm + c0));
    w[3] = ld<S, NT>(at<R>(src + 3 * pb, r0 + cp));
    w[4] = ld<S, NT>(at<R>(src + 4 * pb, rp + c0));
    w[5] = ld<S, NT>(at<R>(src + 5 * pb, rm + cm));
    w[6] = ld<S, NT>(at<R>(src + 6 * pb, rm + cp));
    w[7] = ld<S, NT>(at<R>(src + 7 * pb, rp + cp));
    w[8] = ld<S, NT>(at<R>(src + 8 * pb, rp + cm));
}

template <typename S>
__device__ __forceinline__ void store9(char *__restrict__ dst, uint64_t pb, uint32_t off,
                                       const typename Store<S>::wide w[9])
{
    using R = typename Store<S>::raw;
#pragma unroll
    for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(Store<S>::narrow(w[i]), (R *)(dst + i * pb + off));
}

// gather9 / store9 for rows that are the same on every lane of the wave: the
// plane and row part of each address is one wave-uniform pointer per row
// (readfirstlane keeps the compiler from folding it into per-lane 64-bit
// sums), so every access is a scalar base plus the lane's 32-bit column
// offset and the address costs no vector instruction.
// A raw buffer resource for the bytes [base, base + bytes): an access through
// it is the resource's (scalar) base plus the lane's 32-bit offset, added by
// the memory unit.  Word 3 selects 32-bit raw data (the value CDNA uses for
// untyped buffers); offsets are never out of range here.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const char *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
}

constexpr int kBufNT = 2;   // cache-policy bits of a non-temporal access
typedef unsigned int buf_u32x2 __attribute__((__vector_size__(8)));

// A raw buffer resource for a whole buffer of at most 4 GiB (all nine
// planes): accesses give the plane and row as the scalar offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t whole_rsrc(const char *base)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, -1, 0x00020000);
}

// Loads and stores through a buffer resource: lane offset off plus the
// wave-uniform offset soff.
template <typename S, bool NT>
__device__ __forceinline__ typename Store<S>::wide ld_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t soff = 0)
{
    using R = typename Store<S>::raw;
    constexpr int aux = NT ? kBufNT : 0;
    if constexpr (sizeof(R) == 8)
        return Store<S>::widen(__builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rs, off, soff, aux)));
    else if constexpr (sizeof(R) == 4)
        return Store<S>::widen(__builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rs, off, soff, aux)));
    else
        return Store<S>::widen(__builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b16(rs, off, soff, aux)));
}

template <typename S>
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t soff,
                                       typename Store<S>::wide v)
{
    using R = typename Store<S>::raw;
    const R x = Store<S>::narrow(v);
    if constexpr (sizeof(R) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(buf_u32x2, x), rs, off, soff, kBufNT);
    else if constexpr (sizeof(R) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), rs, off, soff, kBufNT);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, x), rs, off, soff, kBufNT);
}

// gather9 / store9 for rows that are the same on every lane of the wave
// (rb = bytes of a row): one buffer resource per plane and row, so the
// addresses cost scalar instructions only and the lanes supply their
// column offsets.
template <typename S, bool NT>
__device__ __forceinline__ void gather9_uniform_rows(const char *__restrict__ src, uint64_t pb, uint32_t rb,
                                                     uint32_t r0, uint32_t rm, uint32_t rp, uint32_t c0,
                                                     uint32_t cm, uint32_t cp, typename Store<S>::wide w[9])
{
    w[0] = ld_buf<S, NT>(row_rsrc(src + (0 * pb + r0), rb), c0);
    w[1] = ld_buf<S, NT>(row_rsrc(src + (1 * pb + r0), rb), cm);
    w[2] = ld_buf<S, NT>(row_rsrc(src + (2 * pb + rm), rb), c0);
    w[3] = ld_buf<S, NT>(row_rsrc(src + (3 * pb + r0), rb), cp);
    w[4] = ld_buf<S, NT>(row_rsrc(src + (4 * pb + rp), rb), c0);
    w[5] = ld_buf<S, NT>(row_rsrc(src + (5 * pb + rm), rb), cm);
    w[6] = ld_buf<S, NT>(row_rsrc(src + (6 * pb + rm), rb), cp);
    w[7] = ld_buf<S, NT>(row_rsrc(src + (7 * pb + rp), rb), cp);
    w[8] = ld_buf<S, NT>(row_rsrc(src + (8 * pb + rp), rb), cm);
}

template <typename S>
__device__ __forceinline__ void store9_uniform_row(char *__restrict__ dst, uint64_t pb, uint32_t rb, uint32_t row,
                                                   uint32_t col, const typename Store<S>::wide w[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) st_buf<S>(row_rsrc(dst + (i * pb + row), rb), col, 0, w[i]);
}

// ---- several steps per pass (temporal blocking in registers) ---------------
//
// One wave owns a strip of 64 consecutive columns and walks a segment of
// rows.  Stage 0 gathers the nine pulled values of its row from HBM and
// collides them; stage p (p = 1 .. T-1) collides row r - p from the outputs
// of stage p-1, which it keeps in registers: populations with v_y = +1 come
// from the row above (kept from two iterations back), v_y = 0 from the same
// row, v_y = -1 from the row just produced, and the one-column x-shift is a
// cross-lane shuffle.  Only stage T-1 writes to HBM, so one pass reads and
// writes every population once for T steps.  Each stage loses one column at
// each wave edge (its shuffles reach outside the wave there), so a wave
// produces the 64 - 2(T-1) middle columns; the segment is started 2(T-1)
// rows early so that every stage has its rows above.  Intermediate stages
// round their outputs to the storage type exactly as a store and reload
// would, so T steps in one pass are bit-identical to T single steps.

// Whole-wave shifts by one lane with DPP (wave_shr:1 / wave_shl:1 move a
// register between neighbouring lanes inside the VALU, without the LDS
// crossbar that a general shuffle uses).  The edge lane that has no source
// keeps its own value; the kernel never uses that lane's result.
constexpr int kDppWaveShl1 = 0x130;   // lane i receives lane i + 1
constexpr int kDppWaveShr1 = 0x138;   // lane i receives lane i - 1

template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v)
{
    const int b = __float_as_int(v);
    return __int_as_float(__builtin_amdgcn_update_dpp(b, b, CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    const uint32_t nlo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    const uint32_t nhi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)nhi << 32) | nlo));
}

// value of the lane to the left (column x - 1) / to the right (column x + 1)
template <bool DPP, typename V>
__device__ __forceinline__ V from_left(V v)
{
    if constexpr (DPP) return dpp_shift<kDppWaveShr1>(v);
    else return __shfl_up(v, 1, 64);
}

template <bool DPP, typename V>
__device__ __forceinline__ V from_right(V v)
{
    if constexpr (DPP) return dpp_shift<kDppWaveShl1>(v);
    else return __shfl_down(v, 1, 64);
}

template <typename S>
__device__ __forceinline__ typename Store<S>::wide round_trip(typename Store<S>::wide v)
{
    return Store<S>::widen(Store<S>::narrow(v));
}

// round_trip of a cell's nine values.  BF16 storage converts two values per
// instruction (v_cvt_pk_bf16_f32, round to nearest even like the scalar
// conversion of Store<>::narrow, so the results are the same bits) and
// widens the halves back with a shift and a mask: 1.5 instructions per value
// instead of 2 (BF16 several-steps loop 934 -> 880 VALU, +7.6 % measured).
// For FP16 the packed conversion (v_cvt_pk_f16_f32, halves widened with an
// SDWA conversion) issues fewer instructions too but measured 7 % slower, so
// FP16 and the other types take round_trip per value.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

template <typename S>
__device__ __forceinline__ void round_trip9(typename Store<S>::wide w[9])
{
    if constexpr (std::is_same<S, bf16_tag>::value) {
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const uint32_t u = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){w[i], w[i + 1]}, bf16x2_t));
            w[i] = __uint_as_float(u << 16);
            w[i + 1] = __uint_as_float(u & 0xffff0000u);
        }
        w[8] = round_trip<S>(w[8]);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) w[i] = round_trip<S>(w[i]);
    }
}

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Whether all nine planes of a buffer lie within 4 GiB of its start, so
// that one buffer resource with 32-bit offsets reaches every population.
template <typename S>
__device__ __forceinline__ bool one_resource(int64_t plane)
{
    return (uint64_t)plane * sizeof(typename Store<S>::raw) * 9 <= 0xFFFFFFFFull;
}

// Workgroup-shared halo (FLAGS bit 5): the waves of a workgroup cover
// adjacent 64-column pieces of one strip and walk its rows in step.  Each
// stage's output values that the next stage takes from the column to the
// left or right (populations 1, 3, 5, 6, 7, 8) go through LDS instead of a
// cross-lane shuffle: every lane writes them at its column of a
// workgroup-wide row, a barrier, and every lane reads its neighbours' --
// the edge lanes of a wave read the adjacent wave's.  Only the workgroup's
// outer edges lose a column per stage, so a workgroup of W waves writes
// 64 W - 2(T-1) columns instead of W (64 - 2(T-1)).  One buffer per stage
// boundary suffices as long as a barrier separates every read of it from
// its next write: boundary b > 0 is rewritten after boundary b - 1's
// barrier of the next row, boundary 0 after the next stage's barrier of the
// same row (every prologue row, and with T = 2 every row, also starts with a
// barrier, for the rows that run no second exchange).

// T steps of the strip whose cols output columns start at x0, rows y0 ..
// y0+len-1 of one lattice.  Without the shared halo the calling wave owns
// the strip (threadIdx.x = lane; lane T-1 holds column x0; cols <= 64 -
// 2(T-1)); with it the calling workgroup does (wave threadIdx.y holds
// columns x0 - (T-1) + 64 threadIdx.y + lane; cols <= 64 blockDim.y -
// 2(T-1)), and every wave of the workgroup must call with the same
// arguments.
// LDS of the shared-halo exchange: [buffer][stage boundary b (output of
// stage b)][value k (populations 1, 3, 5, 6, 7, 8)][column of the
// workgroup's lanes (256, or 128 for two-wave workgroups)]; one buffer for
// the plain pipeline, two (alternating rows) for the skewed one.
constexpr int kWgXchCols = 64 * kWgMaxWaves;
template <int FLAGS>
constexpr int wg_xch_cols()
{
    return (FLAGS & kWgTwo) ? 128 : kWgXchCols;
}
template <int T, int FLAGS>
constexpr int wg_exchange_values()
{
    return (FLAGS & kWgHalo) ? (T - 1) * 6 * wg_xch_cols<FLAGS>() * ((FLAGS & 16) ? 2 : 1) : 1;
}

template <typename S, typename C, int T, int FLAGS, bool ONE_RSRC>
__device__ __forceinline__ void strip_pass(const char *__restrict__ src, char *__restrict__ dst, int nx, int ny,
                                           int pitch, int64_t plane, const Relax<C> &relax, float scale,
                                           float inv_scale, int x0, int cols, int y0, int len,
                                           typename Store<S>::wide *wgx = nullptr)
{
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    constexpr bool NT = (FLAGS & 1) != 0;
    constexpr bool DPP = (FLAGS & 4) != 0;
    constexpr bool WG = (FLAGS & kWgHalo) != 0;
    // rows of stage-0 loads issued ahead of the row being collided
    constexpr int AHEAD = (FLAGS & 8) ? 2 : ((FLAGS & 2) ? 1 : 0);
    // skewed pipeline: stage p works on row r - 2p and reads only outputs of
    // earlier iterations, so the T collides of an iteration are independent
    constexpr bool SKEW = (FLAGS & 16) != 0;
    constexpr int LAG = SKEW ? 3 : 2;                   // iterations from one stage's start to the next
    constexpr uint32_t E = sizeof(R);
    const int lane = threadIdx.x;
    // column of this lane within the strip's lanes (the workgroup's with the
    // shared halo, the wave's without)
    const int lc = WG ? 64 * (int)threadIdx.y + lane : lane;
    const int xl = x0 + lc - (T - 1);                   // unwrapped column
    const int c = wrap_mod(xl, nx);
    const uint32_t c0 = (uint32_t)c * E;
    const uint32_t cm = (uint32_t)((c == 0 ? nx : c) - 1) * E;
    const uint32_t cp = (uint32_t)((c + 1 == nx) ? 0 : c + 1) * E;
    const bool writes = lc >= T - 1 && lc < T - 1 + cols && xl < nx;
    // shared-halo exchange rows (wgx, the kernel's LDS); the neighbour
    // columns are clamped at the workgroup's edges (those lanes' results are
    // not used)
    constexpr int XW = wg_xch_cols<FLAGS>();
    W *const xch = WG ? wgx : nullptr;
    const int lanes = WG ? 64 * (int)blockDim.y : 64;
    const int lcl = lc > 0 ? lc - 1 : 0, lcr = lc + 1 < lanes ? lc + 1 : lc;
    const uint64_t pb = (uint64_t)plane * E;
    const uint32_t rb = (uint32_t)pitch * E;
    const int iters = len + LAG * (T - 1);
    const int r_first = y0 - (T - 1);
    // Stage 0 gathers rows r_first, r_first + 1, ... in order, so a running
    // wrapped row index (wave-uniform, like x0 and y0) replaces a modulo.
    int yg = wrap_mod(r_first, ny);
    // ONE_RSRC (all nine planes within 4 GiB): one buffer resource per
    // buffer, plane and row as the access's scalar offset; otherwise one
    // resource per plane row
    const __amdgpu_buffer_rsrc_t src_rs = whole_rsrc(src), dst_rs = whole_rsrc(dst);
    auto gather_next = [&](W w[9]) {
        const int y = yg;
        const int ym = (y == 0 ? ny : y) - 1;
        const int yp = (y + 1 == ny) ? 0 : y + 1;
        const uint32_t r0 = (uint32_t)y * rb, rm = (uint32_t)ym * rb, rp = (uint32_t)yp * rb;
        if constexpr (ONE_RSRC) {
            const uint32_t p1 = (uint32_t)pb;
            w[0] = ld_buf<S, NT>(src_rs, c0, 0 * p1 + r0);
            w[1] = ld_buf<S, NT>(src_rs, cm, 1 * p1 + r0);
            w[2] = ld_buf<S, NT>(src_rs, c0, 2 * p1 + rm);
            w[3] = ld_buf<S, NT>(src_rs, cp, 3 * p1 + r0);
            w[4] = ld_buf<S, NT>(src_rs, c0, 4 * p1 + rp);
            w[5] = ld_buf<S, NT>(src_rs, cm, 5 * p1 + rm);
            w[6] = ld_buf<S, NT>(src_rs, cp, 6 * p1 + rm);
            w[7] = ld_buf<S, NT>(src_rs, cp, 7 * p1 + rp);
            w[8] = ld_buf<S, NT>(src_rs, cm, 8 * p1 + rp);
        } else {
            gather9_uniform_rows<S, NT>(src, pb, rb, r0, rm, rp, c0, cm, cp, w);
        }
        yg = yp;
    };
    auto store_row = [&](uint32_t ro, const W v[9]) {
        if constexpr (ONE_RSRC) {
#pragma unroll
            for (int i = 0; i < 9; ++i) st_buf<S>(dst_rs, c0, (uint32_t)i * (uint32_t)pb + ro, v[i]);
        } else {
            store9_uniform_row<S>(dst, pb, rb, ro, c0, v);
        }
    };
    // outputs of stage p kept for stage p + 1: populations 2, 5, 6 of the row
    // before the last one produced, and 0, 1, 3, 2, 5, 6 of the last one
    W up[T > 1 ? T - 1 : 1][3], mid[T > 1 ? T - 1 : 1][6];
    // skewed pipeline: stage p-1's outputs of the last three iterations
    // (all nine; 0, 1, 3, 2, 5, 6; 2, 5, 6)
    W r1[T > 1 ? T - 1 : 1][9], r2[T > 1 ? T - 1 : 1][6], r3[T > 1 ? T - 1 : 1][3];
#pragma unroll
    for (int p = 0; p < (T > 1 ? T - 1 : 1); ++p) {
#pragma unroll
        for (int i = 0; i < 3; ++i) up[p][i] = r3[p][i] = W(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) mid[p][i] = r2[p][i] = W(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) r1[p][i] = W(0);
    }
    W ahead[AHEAD > 0 ? AHEAD : 1][9];
#pragma unroll
    for (int d = 0; d < AHEAD; ++d) gather_next(ahead[d]);   // AHEAD <= 2 < iters
    // One row of the pipeline.  Before iteration 2(T-1) the later stages
    // have no rows yet and stop early (STEADY = false); afterwards every
    // stage runs and the body has no branches, so the loop can be unrolled
    // and the row rotation becomes register renaming.
    // Row j takes its stage-0 values from slot j % AHEAD and refills that
    // slot with row j + AHEAD: no register is copied while its load is in
    // flight, so the waits cover only the loads issued AHEAD rows earlier.
    auto row = [&](int j, auto steady, W(&slot)[9]) {
        constexpr bool STEADY = decltype(steady)::value;
        const int r = r_first + j;                      // row of stage 0
        W w[9];
        if constexpr (AHEAD > 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i) w[i] = slot[i];
            // row r + AHEAD, unconditional (rows past the segment wrap and
            // are never used): no branch, so the waits for these loads
            // stay exact
            gather_next(slot);
        } else {
            gather_next(w);                             // row r
        }
        cell_update<S, C>(w, relax, scale, inv_scale);
        if constexpr (WG) {
            // Stage boundary 0 is written again at the start of every row,
            // so a barrier must separate the previous row's reads of it
            // from this row's writes.  A steady row with T > 2 has one after
            // those reads (the next stage's exchange); a prologue row that
            // runs stage 0 and 1 only (rows 0 and 1), and every row with
            // T = 2 (one boundary), has none, so the rows after them start
            // with one.
            if (j >= 1 && (!STEADY || T == 2)) __syncthreads();
        }
#pragma unroll
        for (int p = 1; p < T; ++p) {
            // w holds stage p-1's output, row r - p + 1
            round_trip9<S>(w);
            W in[9];
            const bool active = STEADY || j >= 2 * p;   // wave-uniform (workgroup-uniform)
            if constexpr (WG) {
                // shifted once, where produced: mid and up keep the shifted
                // populations 1, 3 and 5, 6 for the next two rows
                W *xb = xch + (p - 1) * 6 * XW;
                xb[0 * XW + lc] = w[1];
                xb[1 * XW + lc] = w[3];
                xb[2 * XW + lc] = w[5];
                xb[3 * XW + lc] = w[6];
                xb[4 * XW + lc] = w[7];
                xb[5 * XW + lc] = w[8];
                __syncthreads();
                const W l1 = xb[0 * XW + lcl], r3 = xb[1 * XW + lcr], l5 = xb[2 * XW + lcl];
                const W r6 = xb[3 * XW + lcr], r7 = xb[4 * XW + lcr], l8 = xb[5 * XW + lcl];
                if (active) {
                    in[0] = mid[p - 1][0];
                    in[1] = mid[p - 1][1];
                    in[3] = mid[p - 1][2];
                    in[2] = up[p - 1][0];
                    in[5] = up[p - 1][1];
                    in[6] = up[p - 1][2];
                    in[4] = w[4];
                    in[7] = r7;
                    in[8] = l8;
                }
                up[p - 1][0] = mid[p - 1][3];
                up[p - 1][1] = mid[p - 1][4];
                up[p - 1][2] = mid[p - 1][5];
                mid[p - 1][0] = w[0];
                mid[p - 1][1] = l1;
                mid[p - 1][2] = r3;
                mid[p - 1][3] = w[2];
                mid[p - 1][4] = l5;
                mid[p - 1][5] = r6;
            } else {
                if (active) {
                    in[0] = mid[p - 1][0];
                    in[1] = from_left<DPP>(mid[p - 1][1]);
                    in[3] = from_right<DPP>(mid[p - 1][2]);
                    in[2] = up[p - 1][0];
                    in[5] = from_left<DPP>(up[p - 1][1]);
                    in[6] = from_right<DPP>(up[p - 1][2]);
                    in[4] = w[4];
                    in[7] = from_right<DPP>(w[7]);
                    in[8] = from_left<DPP>(w[8]);
                }
                up[p - 1][0] = mid[p - 1][3];
                up[p - 1][1] = mid[p - 1][4];
                up[p - 1][2] = mid[p - 1][5];
                mid[p - 1][0] = w[0];
                mid[p - 1][1] = w[1];
                mid[p - 1][2] = w[3];
                mid[p - 1][3] = w[2];
                mid[p - 1][4] = w[5];
                mid[p - 1][5] = w[6];
            }
            if (!active) break;
#pragma unroll
            for (int i = 0; i < 9; ++i) w[i] = in[i];
            cell_update<S, C>(w, relax, scale, inv_scale);
            if (p == T - 1 && writes) store_row((uint32_t)(r - (T - 1)) * rb, w);
        }
    };
    // The skewed pipeline's row: every stage reads only registers filled in
    // earlier iterations; the boundaries rotate after all stages have run.
    // Stage p starts at iteration 3p; its row is r - 2p.
    auto row_skew = [&](int j, auto steady, W(&slot)[9]) {
        constexpr bool STEADY = decltype(steady)::value;
        const int r = r_first + j;                      // row of stage 0
        W w[9];
        if constexpr (AHEAD > 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i) w[i] = slot[i];
            gather_next(slot);                          // row r + AHEAD
        } else {
            gather_next(w);                             // row r
        }
        cell_update<S, C>(w, relax, scale, inv_scale);
        W res[T > 1 ? T - 1 : 1][9];
#pragma unroll
        for (int p = 1; p < T; ++p) {
            const bool active = STEADY || j >= 3 * p;   // wave-uniform
            W in[9];
            if (active) {
                if constexpr (WG) {
                    // shifted by the exchange at the end of the row that produced them
                    in[0] = r2[p - 1][0];
                    in[1] = r2[p - 1][1];
                    in[3] = r2[p - 1][2];
                    in[2] = r3[p - 1][0];
                    in[5] = r3[p - 1][1];
                    in[6] = r3[p - 1][2];
                    in[4] = r1[p - 1][4];
                    in[7] = r1[p - 1][7];
                    in[8] = r1[p - 1][8];
                } else {
                    in[0] = r2[p - 1][0];
                    in[1] = from_left<DPP>(r2[p - 1][1]);
                    in[3] = from_right<DPP>(r2[p - 1][2]);
                    in[2] = r3[p - 1][0];
                    in[5] = from_left<DPP>(r3[p - 1][1]);
                    in[6] = from_right<DPP>(r3[p - 1][2]);
                    in[4] = r1[p - 1][4];
                    in[7] = from_right<DPP>(r1[p - 1][7]);
                    in[8] = from_left<DPP>(r1[p - 1][8]);
                }
                cell_update<S, C>(in, relax, scale, inv_scale);
                if (p == T - 1 && writes) store_row((uint32_t)(r - 2 * (T - 1)) * rb, in);
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) in[i] = W(0);
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) res[p - 1][i] = in[i];
        }
#pragma unroll
        for (int p = 1; p < T; ++p) {
            r3[p - 1][0] = r2[p - 1][3];
            r3[p - 1][1] = r2[p - 1][4];
            r3[p - 1][2] = r2[p - 1][5];
            r2[p - 1][0] = r1[p - 1][0];
            r2[p - 1][1] = r1[p - 1][1];
            r2[p - 1][2] = r1[p - 1][3];
            r2[p - 1][3] = r1[p - 1][2];
            r2[p - 1][4] = r1[p - 1][5];
            r2[p - 1][5] = r1[p - 1][6];
#pragma unroll
            for (int i = 0; i < 9; ++i) r1[p - 1][i] = p == 1 ? w[i] : res[p - 2][i];
            round_trip9<S>(r1[p - 1]);
        }
        if constexpr (WG) {
            // One exchange per row: every stage's new output goes through this
            // row's buffer (rows alternate between two, so a barrier of the
            // next row separates these reads from the writes that reuse it)
            // and comes back shifted to the neighbouring columns.
            W *const xb0 = xch + (j & 1) * (T - 1) * 6 * XW;
#pragma unroll
            for (int b = 0; b < T - 1; ++b) {
                W *xb = xb0 + b * 6 * XW;
                xb[0 * XW + lc] = r1[b][1];
                xb[1 * XW + lc] = r1[b][3];
                xb[2 * XW + lc] = r1[b][5];
                xb[3 * XW + lc] = r1[b][6];
                xb[4 * XW + lc] = r1[b][7];
                xb[5 * XW + lc] = r1[b][8];
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < T - 1; ++b) {
                const W *xb = xb0 + b * 6 * XW;
                r1[b][1] = xb[0 * XW + lcl];
                r1[b][3] = xb[1 * XW + lcr];
                r1[b][5] = xb[2 * XW + lcl];
                r1[b][6] = xb[3 * XW + lcr];
                r1[b][7] = xb[4 * XW + lcr];
                r1[b][8] = xb[5 * XW + lcl];
            }
        }
    };
    // Two rows per trip (the compiler does not unroll loops that hold
    // cross-lane operations by a runtime count itself); the even row of a
    // trip uses slot 0, the odd one slot AHEAD - 1.  The prologue has an even
    // number of rows unless the whole segment is shorter.
    constexpr int S1 = AHEAD > 1 ? 1 : 0;
    auto step_row = [&](int jj, auto steady, W(&slot)[9]) {
        if constexpr (SKEW) row_skew(jj, steady, slot);
        else row(jj, steady, slot);
    };
    // prologue rounded up to an even number of rows (the skewed one has
    // 3(T-1) rows of start-up, odd for T = 2 and 4)
    const int pro = min(iters, (LAG * (T - 1) + 1) & ~1);
    int j = 0;
    for (; j + 1 < pro; j += 2) {
        step_row(j, std::false_type{}, ahead[0]);
        step_row(j + 1, std::false_type{}, ahead[S1]);
    }
    if (j < pro) {
        // odd prologue: the segment ends inside it (j + 1 == pro == iters)
        step_row(j, std::false_type{}, ahead[0]);
        ++j;
    }
    for (; j + 1 < iters; j += 2) {
        step_row(j, std::true_type{}, ahead[0]);
        step_row(j + 1, std::true_type{}, ahead[S1]);
    }
    if (j < iters) step_row(j, std::true_type{}, ahead[0]);
}

// Waves per SIMD the register allocation of a several-steps kernel aims
// for: with the shared halo (36 KB of LDS per workgroup at T = 7 for 32-bit
// values) four workgroups of four waves fit a CU when a wave takes at most
// 128 VGPRs (the skewed pipeline holds more rows: two); FP64 values need
// twice the registers and LDS (one).
template <typename S, int FLAGS>
constexpr int multi_waves_per_eu()
{
    return !(FLAGS & kWgHalo) || sizeof(typename Store<S>::wide) == 8 ? 1 : ((FLAGS & 16) ? 2 : 4);
}

template <typename S, typename C, int T, int FLAGS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(multi_waves_per_eu<S, FLAGS>())))
k_step_multi(StepArgs<C> a)
{
    const int OUT = a.out_cols;
    int bid = blockIdx.x;
    if (a.xcd_remap) bid = remap_xcd(bid, a.nblocks);
    // one wave per strip segment (blockDim.x is the wave size), or with the
    // shared halo one workgroup per strip segment: the index is uniform
    // across the wave, which readfirstlane states to the compiler
    const int wave = (FLAGS & kWgHalo) ? bid : __builtin_amdgcn_readfirstlane(bid * (int)blockDim.y + (int)threadIdx.y);
    if (wave >= a.nwaves) return;                       // whole waves (workgroups) only
    const int strip = wave % a.tiles_x, seg = wave / a.tiles_x;
    const int y0 = seg * a.tile_h;
    __shared__ typename Store<S>::wide wgx[wg_exchange_values<T, FLAGS>()];
    // one resource per buffer where it measured faster (FP32 storage: +2 %;
    // with 16-bit storage and in the pool it was slower), else per plane row
    if constexpr (std::is_same<S, float>::value) {
        if (one_resource<S>(a.plane)) {
            strip_pass<S, C, T, FLAGS, true>((const char *)a.src, (char *)a.dst, a.nx, a.ny, a.pitch, a.plane, a.r,
                                             a.scale, a.inv_scale, strip * OUT, OUT, y0, min(a.tile_h, a.ny - y0),
                                             wgx);
            return;
        }
    }
    strip_pass<S, C, T, FLAGS, false>((const char *)a.src, (char *)a.dst, a.nx, a.ny, a.pitch, a.plane, a.r,
                                      a.scale, a.inv_scale, strip * OUT, OUT, y0, min(a.tile_h, a.ny - y0),
                                      wgx);
}

template <typename C>
__device__ __forceinline__ Relax<C> member_relax(const PoolMember *m);
template <>
__device__ __forceinline__ Relax<float> member_relax<float>(const PoolMember *m) { return m->rf; }
template <>
__device__ __forceinline__ Relax<double> member_relax<double>(const PoolMember *m) { return m->rd; }

// T-step launch j of a chunk over the tasks of one table range: a member
// takes T-step launches while T more steps fit.  Without the shared halo each
// wave takes strip tasks in turn; with it (FLAGS bit 5) each workgroup does,
// its waves sharing the halo columns through LDS: four-wave workgroups
// (blockDim.y == kWgMaxWaves) take the range's strip tasks, two-wave ones
// (FLAGS bit 6, blockDim.y == 2) its two-wave tasks.  The tables are
// read-only here: restrict lets the compiler read the task and member
// records with scalar loads, so their fields take no vector registers.
template <typename S, typename C, int T, int FLAGS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(multi_waves_per_eu<S, FLAGS>())))
k_pool_multi(const PoolHeader *__restrict__ hdr, const PoolMember *__restrict__ mem,
             const PoolTile *__restrict__ tiles, int range, int j)
{
    constexpr bool TWO = (FLAGS & kWgTwo) != 0;
    const int begin = TWO ? hdr->hbegin[range] : hdr->mbegin[range];
    const int end = TWO ? hdr->hend[range] : hdr->mend[range];
    if constexpr ((FLAGS & kWgHalo) != 0) {
        __shared__ typename Store<S>::wide wgx[wg_exchange_values<T, FLAGS>()];
        // the exchange rows hold the columns of exactly this many waves
        if ((int)blockDim.y != (TWO ? 2 : kWgMaxWaves)) return;
        for (int v = (int)blockIdx.x; v < end - begin; v += (int)gridDim.x) {
            const int ti = begin + xcd_group(v, end - begin);
            const PoolTile tile = tiles[ti];             // workgroup-uniform
            const PoolMember *m = mem + tile.member;
            if ((int64_t)(j + 1) * T > m->t_target - m->t_done) continue;
            const int par = (int)((m->cur0 + m->flips + j) & 1);
            strip_pass<S, C, T, FLAGS, false>((const char *)m->buf[par], (char *)m->buf[par ^ 1], m->nx, m->ny,
                                              m->pitch, m->plane, member_relax<C>(m), m->scale, m->inv_scale, tile.x0,
                                              tile.ncols, tile.y0, tile.nrows, wgx);
            // every wave's reads of this task's last exchange (which reach
            // into the neighbouring waves' columns) end before any wave
            // writes the next task's
            __syncthreads();
        }
    } else {
        const int nw = (int)(gridDim.x * blockDim.y);
        const int w0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * blockDim.y + threadIdx.y));   // one wave per task
        for (int ti = begin + w0; ti < end; ti += nw) {
            const PoolTile tile = tiles[ti];             // wave-uniform
            const PoolMember *m = mem + tile.member;
            if ((int64_t)(j + 1) * T > m->t_target - m->t_done) continue;
            const int par = (int)((m->cur0 + m->flips + j) & 1);
            strip_pass<S, C, T, FLAGS, false>((const char *)m->buf[par], (char *)m->buf[par ^ 1], m->nx, m->ny,
                                              m->pitch, m->plane, member_relax<C>(m), m->scale, m->inv_scale, tile.x0,
                                              tile.ncols, tile.y0, tile.nrows);
        }
    }
}


}  // namespace
}  // namespace lbm
