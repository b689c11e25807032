// Kernels of the D2Q9 MRT lattice Boltzmann library (gfx950, wave64).
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
#include <math.h>

#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {

namespace {

constexpr int VX_[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int VY_[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

template <typename C>
Relax<C> make_relax(const View &v)
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

// MI355X dispatches consecutive workgroup ids round-robin over its 8 XCDs.
// Renumber so that each XCD receives one contiguous range of tiles: tiles
// that share misaligned cache lines then share one L2.
__device__ __forceinline__ int remap_xcd(int bid, int nb)
{
    const int xcd = bid & 7, local = bid >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
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
#pragma unroll
    for (int i = 0; i < 9; ++i) w[i] = w[i] + (W)dg[i];
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

// One cell per lane: nine direct (possibly misaligned) loads.
// FLAGS bit 0: non-temporal loads; bit 1: the nine loads of the lane's next
// row are issued before the current row is collided and stored.
template <typename S, typename C, int FLAGS>
__global__ void __launch_bounds__(1024) k_step_v1(StepArgs<C> a)
{
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    constexpr bool NT = (FLAGS & 1) != 0;
    constexpr bool PIPE = (FLAGS & 2) != 0;
    constexpr uint32_t E = sizeof(R);
    int bid = blockIdx.x;
    if (a.xcd_remap) bid = remap_xcd(bid, a.nblocks);
    const int tile_x = bid % a.tiles_x, tile_y = bid / a.tiles_x;
    const int x = tile_x * blockDim.x + threadIdx.x;
    if (x >= a.nx) return;
    const uint32_t c0 = (uint32_t)x * E;
    const uint32_t cm = (uint32_t)((x == 0 ? a.nx : x) - 1) * E;
    const uint32_t cp = (uint32_t)((x + 1 == a.nx) ? 0 : x + 1) * E;
    const char *__restrict__ src = (const char *)a.src;
    char *__restrict__ dst = (char *)a.dst;
    const uint64_t pb = (uint64_t)a.plane * E;
    const uint32_t rb = (uint32_t)a.pitch * E;
    auto gather = [&](int y, W w[9]) {
        const int ym = (y == 0 ? a.ny : y) - 1;
        const int yp = (y + 1 == a.ny) ? 0 : y + 1;
        gather9<S, NT>(src, pb, (uint32_t)y * rb, (uint32_t)ym * rb, (uint32_t)yp * rb, c0, cm, cp, w);
    };
    int y = tile_y * a.tile_h + threadIdx.y;
    if (y >= a.ny) return;
    W w[9];
    gather(y, w);
    for (int rr = 0; rr < a.rows; ++rr) {
        const int yn = y + blockDim.y;
        const bool more = rr + 1 < a.rows && yn < a.ny;
        W nxt[9];
        if constexpr (PIPE) {
            if (more) gather(yn, nxt);
        }
        cell_update<S, C>(w, a.r, a.scale, a.inv_scale);
        store9<S>(dst, pb, (uint32_t)y * rb + c0, w);
        if (!more) return;
        if constexpr (PIPE) {
#pragma unroll
            for (int i = 0; i < 9; ++i) w[i] = nxt[i];
        } else {
            gather(yn, w);
        }
        y = yn;
    }
}

// Row strips: a workgroup owns whole rows and walks each one in chunks of
// blockDim.x cells.  The cache line that two neighbouring chunks of an
// x-shifted population share is then read twice by the same workgroup in
// quick succession (an L2 hit) instead of by two workgroups that may sit on
// different XCDs.  FLAGS as for k_step_v1 (bit 1 prefetches the next chunk).
template <typename S, typename C, int FLAGS>
__global__ void __launch_bounds__(1024) k_step_strip(StepArgs<C> a)
{
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    constexpr bool NT = (FLAGS & 1) != 0;
    constexpr bool PIPE = (FLAGS & 2) != 0;
    constexpr uint32_t E = sizeof(R);
    int bid = blockIdx.x;
    if (a.xcd_remap) bid = remap_xcd(bid, a.nblocks);
    const char *__restrict__ src = (const char *)a.src;
    char *__restrict__ dst = (char *)a.dst;
    const uint64_t pb = (uint64_t)a.plane * E;
    const uint32_t rb = (uint32_t)a.pitch * E;
    const int y0 = bid * a.tile_h + threadIdx.y;
    for (int rr = 0; rr < a.rows; ++rr) {
        const int y = y0 + rr * blockDim.y;
        if (y >= a.ny) return;
        const int ym = (y == 0 ? a.ny : y) - 1;
        const int yp = (y + 1 == a.ny) ? 0 : y + 1;
        const uint32_t r0 = (uint32_t)y * rb, rm = (uint32_t)ym * rb, rp = (uint32_t)yp * rb;
        auto gather = [&](int x, W w[9]) {
            const uint32_t cm = (uint32_t)((x == 0 ? a.nx : x) - 1) * E;
            const uint32_t cp = (uint32_t)((x + 1 == a.nx) ? 0 : x + 1) * E;
            gather9<S, NT>(src, pb, r0, rm, rp, (uint32_t)x * E, cm, cp, w);
        };
        int x = threadIdx.x;
        if (x >= a.nx) continue;
        W w[9];
        gather(x, w);
        while (true) {
            const int xn = x + blockDim.x;
            const bool more = xn < a.nx;
            W nxt[9];
            if constexpr (PIPE) {
                if (more) gather(xn, nxt);
            }
            cell_update<S, C>(w, a.r, a.scale, a.inv_scale);
            store9<S>(dst, pb, r0 + (uint32_t)x * E, w);
            if (!more) break;
            if constexpr (PIPE) {
#pragma unroll
                for (int i = 0; i < 9; ++i) w[i] = nxt[i];
            } else {
                gather(xn, w);
            }
            x = xn;
        }
    }
}

// VX consecutive cells per lane: aligned vector loads; the one-element
// x-shift of populations with v_x = +-1 is taken from the neighbouring lane
// (cross-lane shuffle), and only the first / last lane of a wave loads its
// edge element directly.  Needs nx % VX == 0 and blockDim.x % 64 == 0.
template <typename S, typename C, int VX, int FLAGS>
__global__ void __launch_bounds__(1024) k_step_vec(StepArgs<C> a)
{
    constexpr bool NT = (FLAGS & 1) != 0;
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    using V = typename VecOf<R, VX>::type;
    int bid = blockIdx.x;
    if (a.xcd_remap) bid = remap_xcd(bid, a.nblocks);
    const int tile_x = bid % a.tiles_x, tile_y = bid / a.tiles_x;
    const int lane = threadIdx.x & 63;
    const int xl = (tile_x * (int)blockDim.x + (int)threadIdx.x) * VX;
    if (xl - lane * VX >= a.nx) return;            // the whole wave is past the row end
    const bool active = xl < a.nx;
    const int x0 = active ? xl : 0;
    const int xleft = (x0 == 0 ? a.nx : x0) - 1;
    const int xright = (x0 + VX >= a.nx) ? 0 : x0 + VX;
    const bool edge_l = lane == 0;
    const bool edge_r = lane == 63 || xl + VX >= a.nx;
    const R *__restrict__ src = (const R *)a.src;
    R *__restrict__ dst = (R *)a.dst;
    const int64_t P = a.plane;
    int y = tile_y * a.tile_h + threadIdx.y;
    for (int rr = 0; rr < a.rows; ++rr, y += blockDim.y) {
        if (y >= a.ny) return;
        const int ym = (y == 0 ? a.ny : y) - 1;
        const int yp = (y + 1 == a.ny) ? 0 : y + 1;
        const int64_t rowoff[3] = {(int64_t)y * a.pitch, (int64_t)ym * a.pitch, (int64_t)yp * a.pitch};
        // source row of each population: 0 = own row, 1 = y-1 (v_y = +1), 2 = y+1 (v_y = -1)
        constexpr int ROW[9] = {0, 0, 1, 0, 2, 1, 1, 2, 2};
        W w[9][VX];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const R *row = src + i * P + rowoff[ROW[i]];
            V raw;
            if constexpr (NT) raw = __builtin_nontemporal_load((const V *)(row + x0));
            else raw = *(const V *)(row + x0);
            W vals[VX];
#pragma unroll
            for (int k = 0; k < VX; ++k) {
                if constexpr (VX == 1) vals[k] = Store<S>::widen(raw);
                else vals[k] = Store<S>::widen(raw[k]);
            }
            if (VX_[i] == 0) {
#pragma unroll
                for (int k = 0; k < VX; ++k) w[i][k] = vals[k];
            } else if (VX_[i] == 1) {                  // needs x0-1 .. x0+VX-2
                W left = __shfl_up(vals[VX - 1], 1, 64);
                if (edge_l) left = Store<S>::widen(row[xleft]);
                w[i][0] = left;
#pragma unroll
                for (int k = 1; k < VX; ++k) w[i][k] = vals[k - 1];
            } else {                                   // needs x0+1 .. x0+VX
                W right = __shfl_down(vals[0], 1, 64);
                if (edge_r) right = Store<S>::widen(row[xright]);
#pragma unroll
                for (int k = 0; k < VX - 1; ++k) w[i][k] = vals[k + 1];
                w[i][VX - 1] = right;
            }
        }
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            W c[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) c[i] = w[i][k];
            cell_update<S, C>(c, a.r, a.scale, a.inv_scale);
#pragma unroll
            for (int i = 0; i < 9; ++i) w[i][k] = c[i];
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                V out;
#pragma unroll
                for (int k = 0; k < VX; ++k) {
                    if constexpr (VX == 1) out = Store<S>::narrow(w[i][k]);
                    else out[k] = Store<S>::narrow(w[i][k]);
                }
                __builtin_nontemporal_store(out, (V *)(dst + i * P + rowoff[0] + x0));
            }
        }
    }
}

// VX consecutive cells per lane from overlapping aligned vector loads: a
// population with v_x = +1 needs x0-1 .. x0+VX-2, taken from the aligned
// vectors at x0-VX and x0; one with v_x = -1 needs x0+1 .. x0+VX, from the
// vectors at x0 and x0+VX (both wrap periodically).  The neighbouring
// vectors are the adjacent lanes' own vectors, so the extra loads are
// served by the cache; there is no cross-lane exchange and no divergent
// edge load.  Needs nx % VX == 0.
template <typename S, typename C, int VX, int FLAGS>
__global__ void __launch_bounds__(1024) k_step_wide(StepArgs<C> a)
{
    constexpr bool NT = (FLAGS & 1) != 0;
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    using V = typename VecOf<R, VX>::type;
    int bid = blockIdx.x;
    if (a.xcd_remap) bid = remap_xcd(bid, a.nblocks);
    const int tile_x = bid % a.tiles_x, tile_y = bid / a.tiles_x;
    const int x0 = (tile_x * (int)blockDim.x + (int)threadIdx.x) * VX;
    if (x0 >= a.nx) return;
    const int xl = (x0 == 0 ? a.nx : x0) - VX;           // previous vector (wrapped)
    const int xr = (x0 + VX == a.nx) ? 0 : x0 + VX;       // next vector (wrapped)
    const R *__restrict__ src = (const R *)a.src;
    R *__restrict__ dst = (R *)a.dst;
    const int64_t P = a.plane;
    auto vload = [&](const R *p) -> V {
        if constexpr (NT) return __builtin_nontemporal_load((const V *)p);
        else return *(const V *)p;
    };
    auto el = [](const V &v, int k) -> R {
        if constexpr (VX == 1) return v;
        else return v[k];
    };
    int y = tile_y * a.tile_h + threadIdx.y;
    for (int rr = 0; rr < a.rows; ++rr, y += blockDim.y) {
        if (y >= a.ny) return;
        const int ym = (y == 0 ? a.ny : y) - 1;
        const int yp = (y + 1 == a.ny) ? 0 : y + 1;
        const int64_t rowoff[3] = {(int64_t)y * a.pitch, (int64_t)ym * a.pitch, (int64_t)yp * a.pitch};
        constexpr int ROW[9] = {0, 0, 1, 0, 2, 1, 1, 2, 2};
        W w[9][VX];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const R *row = src + i * P + rowoff[ROW[i]];
            const V cur = vload(row + x0);
            if (VX_[i] == 0) {
#pragma unroll
                for (int k = 0; k < VX; ++k) w[i][k] = Store<S>::widen(el(cur, k));
            } else if (VX_[i] == 1) {
                const V prev = vload(row + xl);
                w[i][0] = Store<S>::widen(el(prev, VX - 1));
#pragma unroll
                for (int k = 1; k < VX; ++k) w[i][k] = Store<S>::widen(el(cur, k - 1));
            } else {
                const V next = vload(row + xr);
#pragma unroll
                for (int k = 0; k < VX - 1; ++k) w[i][k] = Store<S>::widen(el(cur, k + 1));
                w[i][VX - 1] = Store<S>::widen(el(next, 0));
            }
        }
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            W c[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) c[i] = w[i][k];
            cell_update<S, C>(c, a.r, a.scale, a.inv_scale);
#pragma unroll
            for (int i = 0; i < 9; ++i) w[i][k] = c[i];
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            V out;
#pragma unroll
            for (int k = 0; k < VX; ++k) {
                if constexpr (VX == 1) out = Store<S>::narrow(w[i][k]);
                else out[k] = Store<S>::narrow(w[i][k]);
            }
            __builtin_nontemporal_store(out, (V *)(dst + i * P + rowoff[0] + x0));
        }
    }
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

// T steps of the strip whose cols output columns start at x0 (cols <=
// 64 - 2(T-1)), rows y0 .. y0+len-1 of one lattice, by the calling wave
// (threadIdx.x = lane; lane T-1 holds column x0).
template <typename S, typename C, int T, int FLAGS, bool ONE_RSRC>
__device__ __forceinline__ void strip_pass(const char *__restrict__ src, char *__restrict__ dst, int nx, int ny,
                                           int pitch, int64_t plane, const Relax<C> &relax, float scale,
                                           float inv_scale, int x0, int cols, int y0, int len)
{
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    constexpr bool NT = (FLAGS & 1) != 0;
    constexpr bool DPP = (FLAGS & 4) != 0;
    // rows of stage-0 loads issued ahead of the row being collided
    constexpr int AHEAD = (FLAGS & 8) ? 2 : ((FLAGS & 2) ? 1 : 0);
    // skewed pipeline: stage p works on row r - 2p and reads only outputs of
    // earlier iterations, so the T collides of an iteration are independent
    constexpr bool SKEW = (FLAGS & 16) != 0;
    constexpr int LAG = SKEW ? 3 : 2;                   // iterations from one stage's start to the next
    constexpr uint32_t E = sizeof(R);
    const int lane = threadIdx.x;
    const int xl = x0 + lane - (T - 1);                 // unwrapped column
    const int c = wrap_mod(xl, nx);
    const uint32_t c0 = (uint32_t)c * E;
    const uint32_t cm = (uint32_t)((c == 0 ? nx : c) - 1) * E;
    const uint32_t cp = (uint32_t)((c + 1 == nx) ? 0 : c + 1) * E;
    const bool writes = lane >= T - 1 && lane < T - 1 + cols && xl < nx;
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
#pragma unroll
        for (int p = 1; p < T; ++p) {
            // w holds stage p-1's output, row r - p + 1
#pragma unroll
            for (int i = 0; i < 9; ++i) w[i] = round_trip<S>(w[i]);
            W in[9];
            const bool active = STEADY || j >= 2 * p;   // wave-uniform
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
                in[0] = r2[p - 1][0];
                in[1] = from_left<DPP>(r2[p - 1][1]);
                in[3] = from_right<DPP>(r2[p - 1][2]);
                in[2] = r3[p - 1][0];
                in[5] = from_left<DPP>(r3[p - 1][1]);
                in[6] = from_right<DPP>(r3[p - 1][2]);
                in[4] = r1[p - 1][4];
                in[7] = from_right<DPP>(r1[p - 1][7]);
                in[8] = from_left<DPP>(r1[p - 1][8]);
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
            for (int i = 0; i < 9; ++i) r1[p - 1][i] = round_trip<S>(p == 1 ? w[i] : res[p - 2][i]);
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

template <typename S, typename C, int T, int FLAGS>
__global__ void __launch_bounds__(256) k_step_multi(StepArgs<C> a)
{
    const int OUT = a.out_cols;
    int bid = blockIdx.x;
    if (a.xcd_remap) bid = remap_xcd(bid, a.nblocks);
    // one wave per strip segment (blockDim.x is the wave size): the index
    // is uniform across the wave, which readfirstlane states to the compiler
    const int wave = __builtin_amdgcn_readfirstlane(bid * (int)blockDim.y + (int)threadIdx.y);
    if (wave >= a.nwaves) return;                       // whole waves only
    const int strip = wave % a.tiles_x, seg = wave / a.tiles_x;
    const int y0 = seg * a.tile_h;
    // one resource per buffer where it measured faster (FP32 storage: +2 %;
    // with 16-bit storage and in the pool it was slower), else per plane row
    if constexpr (std::is_same<S, float>::value) {
        if (one_resource<S>(a.plane)) {
            strip_pass<S, C, T, FLAGS, true>((const char *)a.src, (char *)a.dst, a.nx, a.ny, a.pitch, a.plane, a.r,
                                             a.scale, a.inv_scale, strip * OUT, OUT, y0, min(a.tile_h, a.ny - y0));
            return;
        }
    }
    strip_pass<S, C, T, FLAGS, false>((const char *)a.src, (char *)a.dst, a.nx, a.ny, a.pitch, a.plane, a.r,
                                      a.scale, a.inv_scale, strip * OUT, OUT, y0, min(a.tile_h, a.ny - y0));
}

// ---- batched step over a pool of lattices ----------------------------------------
//
// A one-step launch advances every active member of one storage class by
// one step, a T-step launch by T steps.  The grid is persistent (a fixed
// number of workgroups strides over the tile table), so the same launch
// serves any membership.  A one-step tile is a rectangle of one member
// (whole rows of a narrow lattice, a row segment of a wide one) whose cells
// are walked as a flattened (row, column) index so narrow lattices still
// fill whole waves; a T-step task is one strip segment of one member, taken
// by one wave.  Which launches of a recorded chunk a member takes, and hence
// which of its buffers is the source, follows from its remaining step count
// (chunk schedule in lbm_internal.hpp).  The per-cell work is the same
// gather9 / cell_update / store9 and strip_pass as the single-lattice
// kernels, so a lattice gives bit-identical results alone or in a pool.

template <typename C>
__device__ __forceinline__ Relax<C> member_relax(const PoolMember *m);
template <>
__device__ __forceinline__ Relax<float> member_relax<float>(const PoolMember *m) { return m->rf; }
template <>
__device__ __forceinline__ Relax<double> member_relax<double>(const PoolMember *m) { return m->rd; }

template <typename S, typename C>
__global__ void __launch_bounds__(1024) k_pool_step(const PoolHeader *hdr, const PoolMember *mem,
                                                     const PoolTile *tiles, int cls, int i, int kk, int T)
{
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    const int begin = hdr->begin[cls], end = hdr->end[cls];
    for (int ti = begin + (int)blockIdx.x; ti < end; ti += (int)gridDim.x) {
        const PoolTile tile = tiles[ti];
        const PoolMember *m = mem + tile.member;
        const int64_t rem = m->t_target - m->t_done;
        const int64_t span = rem < kk ? rem : kk;
        const int64_t q = member_multi(rem, kk, T);
        if (i >= span - q * T) continue;                 // not one of its one-step launches
        const int par = (int)((m->cur0 + m->flips + q + i) & 1);
        const char *__restrict__ src = (const char *)m->buf[par];
        char *__restrict__ dst = (char *)m->buf[par ^ 1];
        const int nx = m->nx, ny = m->ny;
        constexpr uint32_t E = sizeof(R);
        const uint64_t pb = (uint64_t)m->plane * E;
        const uint32_t rb = (uint32_t)m->pitch * E;
        const Relax<C> r = member_relax<C>(m);
        const float scale = m->scale, inv_scale = m->inv_scale;
        const int ncols = tile.ncols;
        const int ncell = tile.nrows * ncols;
        for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
            const int dy = c / ncols;
            const int x = tile.x0 + (c - dy * ncols);
            const int y = tile.y0 + dy;
            const uint32_t cm = (uint32_t)((x == 0 ? nx : x) - 1) * E;
            const uint32_t cp = (uint32_t)((x + 1 == nx) ? 0 : x + 1) * E;
            const int ym = (y == 0 ? ny : y) - 1;
            const int yp = (y + 1 == ny) ? 0 : y + 1;
            const uint32_t r0 = (uint32_t)y * rb;
            W w[9];
            gather9<S, false>(src, pb, r0, (uint32_t)ym * rb, (uint32_t)yp * rb, (uint32_t)x * E, cm, cp, w);
            cell_update<S, C>(w, r, scale, inv_scale);
            store9<S>(dst, pb, r0 + (uint32_t)x * E, w);
        }
    }
}

// T-step launch j of a chunk: each wave takes strip tasks of the class in
// turn; a member takes T-step launches while T more steps fit.
template <typename S, typename C, int T, int FLAGS>
__global__ void __launch_bounds__(256) k_pool_multi(const PoolHeader *hdr, const PoolMember *mem,
                                                    const PoolTile *tiles, int cls, int j)
{
    const int begin = hdr->mbegin[cls], end = hdr->mend[cls];
    const int nw = (int)(gridDim.x * blockDim.y);
    const int w0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * blockDim.y + threadIdx.y));   // one wave per task
    for (int ti = begin + w0; ti < end; ti += nw) {
        const PoolTile tile = tiles[ti];                 // wave-uniform
        const PoolMember *m = mem + tile.member;
        if ((int64_t)(j + 1) * T > m->t_target - m->t_done) continue;
        const int par = (int)((m->cur0 + m->flips + j) & 1);
        strip_pass<S, C, T, FLAGS, false>((const char *)m->buf[par], (char *)m->buf[par ^ 1], m->nx, m->ny, m->pitch,
                                          m->plane, member_relax<C>(m), m->scale, m->inv_scale, tile.x0, tile.ncols,
                                          tile.y0, tile.nrows);
    }
}

__global__ void k_pool_commit(PoolMember *mem, int nmem, int kk, int T)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nmem) return;
    const int64_t rem = mem[i].t_target - mem[i].t_done;
    if (rem > 0) {
        const int64_t span = rem < kk ? rem : (int64_t)kk;
        const int64_t q = member_multi(rem, kk, T);
        mem[i].t_done += span;
        mem[i].flips += q + span - q * T;
    }
}

// ---- block reductions (fixed order, deterministic) ---------------------------

template <int N>
__device__ __forceinline__ void block_sum_to(double (&acc)[N], double *out)
{
    __shared__ double red[16][N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[k] = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[wave][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < N; ++k) {
            double s = 0.0;
            for (int wv = 0; wv < nw; ++wv) s += red[wv][k];
            out[k] = s;
        }
    }
}

__device__ __forceinline__ void block_max_to(double v, double *out)
{
    __shared__ double red[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0;
        for (int wv = 0; wv < nw; ++wv) s = fmax(s, red[wv]);
        *out = s;
    }
}

// Sums `width` columns of nb partial rows in a fixed order (one block).
// mode 0: out[k] = sum * mul; mode 1: max.
__global__ void __launch_bounds__(256) k_final(const double *partials, int nb, int width,
                                               double mul, int mode, double *out)
{
    __shared__ double red[256];
    for (int k = 0; k < width; ++k) {
        double s = 0.0;
        for (int j = threadIdx.x; j < nb; j += blockDim.x) {
            const double v = partials[(size_t)j * width + k];
            s = mode == 1 ? fmax(s, v) : s + v;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h)
                red[threadIdx.x] = mode == 1 ? fmax(red[threadIdx.x], red[threadIdx.x + h])
                                             : red[threadIdx.x] + red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = mode == 1 ? red[0] : red[0] * mul;
        __syncthreads();
    }
}

// ---- initialisation, readback, diagnostics ------------------------------------

struct CellArgs {
    int32_t nx, ny, pitch, pad;
    int64_t plane;
    double scale, inv_scale;
    Relax<double> r;
    double fbase[9];
};

CellArgs make_cell_args(const View &v)
{
    CellArgs c;
    c.nx = v.nx;
    c.ny = v.ny;
    c.pitch = v.pitch;
    c.pad = 0;
    c.plane = v.plane;
    c.scale = v.scale;
    c.inv_scale = v.inv_scale;
    c.r = make_relax<double>(v);
    for (int i = 0; i < 9; ++i) c.fbase[i] = v.fbase[i];
    return c;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// g(x) = M^{-1} dmeq(rho - rho0, rho u - j0), FP64; stored at P_i(x - v_i).
template <typename S>
__global__ void __launch_bounds__(256) k_init(CellArgs a, const double *rho, const double *ux,
                                              const double *uy, typename Store<S>::raw *dst,
                                              double *partials, int measure_only)
{
    using W = typename Store<S>::wide;
    const int64_t n = (int64_t)a.nx * a.ny;
    double mx = 0.0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
        const double r = rho[c];
        double dm[9], g[9];
        delta_meq<double>(r - a.r.rho0, r * ux[c] - a.r.j0x, r * uy[c] - a.r.j0y, a.r, dm);
        back_transform<double>(dm, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) mx = fmax(mx, fabs(g[i]));
        if (!measure_only) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int xs = wrap(x - VX_[i], a.nx), ys = wrap(y - VY_[i], a.ny);
                dst[i * a.plane + (int64_t)ys * a.pitch + xs] = Store<S>::narrow((W)(g[i] * a.scale));
            }
        }
    }
    if (measure_only) block_max_to(mx, partials + blockIdx.x);
}

// rho, u of the pre-collision state, FP64.
template <typename S>
__global__ void __launch_bounds__(256) k_moments(CellArgs a, const typename Store<S>::raw *src,
                                                 double *rho, double *ux, double *uy)
{
    const int64_t n = (int64_t)a.nx * a.ny;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
        double r = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int xs = wrap(x - VX_[i], a.nx), ys = wrap(y - VY_[i], a.ny);
            const double g = (double)Store<S>::widen(src[i * a.plane + (int64_t)ys * a.pitch + xs]) * a.inv_scale;
            r += g;
            jx += VX_[i] * g;
            jy += VY_[i] * g;
        }
        const double rr = a.r.rho0 + r;
        rho[c] = rr;
        ux[c] = (a.r.j0x + jx) / rr;
        uy[c] = (a.r.j0y + jy) / rr;
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_read_pop(CellArgs a, const typename Store<S>::raw *src, double *f)
{
    const int64_t n = (int64_t)a.nx * a.ny;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int xs = wrap(x - VX_[i], a.nx), ys = wrap(y - VY_[i], a.ny);
            const double g = (double)Store<S>::widen(src[i * a.plane + (int64_t)ys * a.pitch + xs]) * a.inv_scale;
            f[i * n + c] = a.fbase[i] + g;
        }
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_write_pop(CellArgs a, const double *f, typename Store<S>::raw *dst)
{
    using W = typename Store<S>::wide;
    const int64_t n = (int64_t)a.nx * a.ny;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int xs = wrap(x - VX_[i], a.nx), ys = wrap(y - VY_[i], a.ny);
            dst[i * a.plane + (int64_t)ys * a.pitch + xs] = Store<S>::narrow((W)((f[i * n + c] - a.fbase[i]) * a.scale));
        }
    }
}

// Global sums of the collision invariants (aligned reads: a global sum does
// not need the pull shift) and the count of non-finite stored values.
template <typename S>
__global__ void __launch_bounds__(256) k_diag(CellArgs a, const typename Store<S>::raw *src, double *partials)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t n = (int64_t)a.nx * a.ny;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
        double r = 0.0, jx = 0.0, jy = 0.0;
        int bad = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double g = (double)Store<S>::widen(src[i * a.plane + (int64_t)y * a.pitch + x]);
            bad += !isfinite(g);
            r += g;
            jx += VX_[i] * g;
            jy += VY_[i] * g;
        }
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += bad;
    }
    block_sum_to<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// sum_y P_i(y) e^{-i k.y}; the pull shift e^{-i k.v_i} is applied afterwards.
template <typename S>
__global__ void __launch_bounds__(256) k_project(CellArgs a, const typename Store<S>::raw *src, int mx,
                                                 int my, double *partials)
{
    double acc[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) acc[k] = 0.0;
    const int64_t n = (int64_t)a.nx * a.ny;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / a.nx), x = (int)(c - (int64_t)y * a.nx);
        // exact phase fraction: ((mx x) mod nx)/nx + ((my y) mod ny)/ny
        int64_t px = ((int64_t)mx * x) % a.nx, py = ((int64_t)my * y) % a.ny;
        if (px < 0) px += a.nx;
        if (py < 0) py += a.ny;
        const double frac = (double)px / a.nx + (double)py / a.ny;
        double sn, cs;
        sincospi(2.0 * frac, &sn, &cs);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double g = (double)Store<S>::widen(src[i * a.plane + (int64_t)y * a.pitch + x]);
            acc[2 * i] += g * cs;
            acc[2 * i + 1] -= g * sn;
        }
    }
    block_sum_to<18>(acc, partials + (size_t)blockIdx.x * 18);
}

__global__ void k_project_finish(const double *sums, int mx, int my, int nx, int ny, double inv_scale,
                                 double *out)
{
    const int i = threadIdx.x;
    if (i >= 9) return;
    int64_t px = ((int64_t)mx * VX_[i]) % nx, py = ((int64_t)my * VY_[i]) % ny;
    if (px < 0) px += nx;
    if (py < 0) py += ny;
    double sn, cs;
    sincospi(2.0 * ((double)px / nx + (double)py / ny), &sn, &cs);
    const double re = sums[2 * i] * inv_scale, im = sums[2 * i + 1] * inv_scale;
    out[2 * i] = re * cs + im * sn;          // (re + i im)(cs - i sn)
    out[2 * i + 1] = im * cs - re * sn;
}

int grid_for(int64_t n, int block, int cap)
{
    int64_t b = (n + block - 1) / block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

template <template <typename> class F, typename... Args>
hipError_t dispatch_storage(int storage, Args &&...args)
{
    switch (storage) {
    case LBM_STORE_F64: return F<double>::run(args...);
    case LBM_STORE_F32: return F<float>::run(args...);
    case LBM_STORE_F16: return F<f16_tag>::run(args...);
    case LBM_STORE_BF16: return F<bf16_tag>::run(args...);
    default: return hipErrorInvalidValue;
    }
}

template <typename S, typename C>
hipError_t launch_step_typed(const View &v, const void *src, void *dst, const lbm_launch &cfg, hipStream_t st)
{
    StepArgs<C> a;
    a.src = src;
    a.dst = dst;
    a.nx = v.nx;
    a.ny = v.ny;
    a.pitch = v.pitch;
    const int vx = cfg.variant <= 3 ? 1 << cfg.variant : (cfg.variant >= 5 ? 1 << (cfg.variant - 4) : 1);
    const int tile_w = cfg.block_x * vx;
    a.tiles_x = cfg.variant == 4 ? 1 : (v.nx + tile_w - 1) / tile_w;
    a.tile_h = cfg.block_y * cfg.rows;
    a.rows = cfg.rows;
    const int tiles_y = (v.ny + a.tile_h - 1) / a.tile_h;
    a.nblocks = a.tiles_x * tiles_y;
    a.xcd_remap = cfg.xcd_remap;
    a.plane = v.plane;
    a.r = make_relax<C>(v);
    a.scale = (float)v.scale;
    a.inv_scale = (float)v.inv_scale;
    a.nwaves = 0;
    a.out_cols = 0;
    if (cfg.variant >= 8) {
        // strips of multi_strip_cols output columns, segments of `rows` rows, one wave each
        const int T = cfg.variant - 6;
        a.out_cols = multi_strip_cols(T, (int)sizeof(typename Store<S>::raw));
        a.tiles_x = (v.nx + a.out_cols - 1) / a.out_cols;
        a.tile_h = cfg.rows;
        const int segs = (v.ny + cfg.rows - 1) / cfg.rows;
        a.nwaves = a.tiles_x * segs;
        a.nblocks = (a.nwaves + cfg.block_y - 1) / cfg.block_y;
    }
    const dim3 grid(a.nblocks), block(cfg.block_x, cfg.block_y);
    if (cfg.variant >= 8) {
        switch ((cfg.variant - 8) * 32 + cfg.flags) {
#define LBM_MULTI(T_, F_)                                                                    \
    case (T_ - 2) * 32 + F_: hipLaunchKernelGGL((k_step_multi<S, C, T_, F_>), grid, block, 0, st, a); break;
#define LBM_MULTI_T(T_) LBM_MULTI(T_, 0) LBM_MULTI(T_, 1) LBM_MULTI(T_, 2) LBM_MULTI(T_, 3) \
                        LBM_MULTI(T_, 4) LBM_MULTI(T_, 5) LBM_MULTI(T_, 6) LBM_MULTI(T_, 7) \
                        LBM_MULTI(T_, 8) LBM_MULTI(T_, 9) LBM_MULTI(T_, 12) LBM_MULTI(T_, 13)
        LBM_MULTI_T(2)
        LBM_MULTI_T(3)
        LBM_MULTI_T(4)
        // skewed pipeline (bit 4), T = 3 and 4
        LBM_MULTI(3, 16) LBM_MULTI(3, 18) LBM_MULTI(3, 20) LBM_MULTI(3, 22) LBM_MULTI(3, 24) LBM_MULTI(3, 28)
        LBM_MULTI(4, 16) LBM_MULTI(4, 18) LBM_MULTI(4, 20) LBM_MULTI(4, 22) LBM_MULTI(4, 24) LBM_MULTI(4, 28)
        // T = 5 and 6, loads not non-temporal
#define LBM_MULTI_E(T_) LBM_MULTI(T_, 0) LBM_MULTI(T_, 2) LBM_MULTI(T_, 4) LBM_MULTI(T_, 6) LBM_MULTI(T_, 8) \
                        LBM_MULTI(T_, 12) LBM_MULTI(T_, 16) LBM_MULTI(T_, 18) LBM_MULTI(T_, 20) LBM_MULTI(T_, 28)
        LBM_MULTI_E(5)
        LBM_MULTI_E(6)
        // T = 7: plain pipeline only
        LBM_MULTI(7, 0) LBM_MULTI(7, 2) LBM_MULTI(7, 4) LBM_MULTI(7, 6) LBM_MULTI(7, 8) LBM_MULTI(7, 12)
#undef LBM_MULTI_E
#undef LBM_MULTI_T
#undef LBM_MULTI
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const bool nt = cfg.flags & 1, pipe = cfg.flags & 2;
    switch (cfg.variant * 4 + (pipe ? 2 : 0) + (nt ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_step_v1<S, C, 0>), grid, block, 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_step_v1<S, C, 1>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_step_v1<S, C, 2>), grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_step_v1<S, C, 3>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_step_vec<S, C, 2, 0>), grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_step_vec<S, C, 2, 1>), grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_step_vec<S, C, 4, 0>), grid, block, 0, st, a); break;
    case 9: hipLaunchKernelGGL((k_step_vec<S, C, 4, 1>), grid, block, 0, st, a); break;
    case 12: hipLaunchKernelGGL((k_step_vec<S, C, 8, 0>), grid, block, 0, st, a); break;
    case 13: hipLaunchKernelGGL((k_step_vec<S, C, 8, 1>), grid, block, 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_step_strip<S, C, 0>), grid, block, 0, st, a); break;
    case 17: hipLaunchKernelGGL((k_step_strip<S, C, 1>), grid, block, 0, st, a); break;
    case 18: hipLaunchKernelGGL((k_step_strip<S, C, 2>), grid, block, 0, st, a); break;
    case 19: hipLaunchKernelGGL((k_step_strip<S, C, 3>), grid, block, 0, st, a); break;
    case 20: hipLaunchKernelGGL((k_step_wide<S, C, 2, 0>), grid, block, 0, st, a); break;
    case 21: hipLaunchKernelGGL((k_step_wide<S, C, 2, 1>), grid, block, 0, st, a); break;
    case 24: hipLaunchKernelGGL((k_step_wide<S, C, 4, 0>), grid, block, 0, st, a); break;
    case 25: hipLaunchKernelGGL((k_step_wide<S, C, 4, 1>), grid, block, 0, st, a); break;
    case 28: hipLaunchKernelGGL((k_step_wide<S, C, 8, 0>), grid, block, 0, st, a); break;
    case 29: hipLaunchKernelGGL((k_step_wide<S, C, 8, 1>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S>
struct InitF {
    static hipError_t run(const View &v, const double *rho, const double *ux, const double *uy, void *dst,
                          double *partials, double *result, bool measure, hipStream_t st)
    {
        const CellArgs a = make_cell_args(v);
        const int64_t n = (int64_t)v.nx * v.ny;
        const int g = measure ? kRedBlocks : grid_for(n, 256, 65536);
        hipLaunchKernelGGL(k_init<S>, dim3(g), dim3(256), 0, st, a, rho, ux, uy,
                           (typename Store<S>::raw *)dst, partials, (int)measure);
        if (measure) hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partials, g, 1, 1.0, 1, result);
        return hipGetLastError();
    }
};

template <typename S>
struct MomentsF {
    static hipError_t run(const View &v, const void *src, double *rho, double *ux, double *uy, hipStream_t st)
    {
        const CellArgs a = make_cell_args(v);
        const int g = grid_for((int64_t)v.nx * v.ny, 256, 65536);
        hipLaunchKernelGGL(k_moments<S>, dim3(g), dim3(256), 0, st, a,
                           (const typename Store<S>::raw *)src, rho, ux, uy);
        return hipGetLastError();
    }
};

template <typename S>
struct ReadPopF {
    static hipError_t run(const View &v, const void *src, double *f, hipStream_t st)
    {
        const CellArgs a = make_cell_args(v);
        const int g = grid_for((int64_t)v.nx * v.ny, 256, 65536);
        hipLaunchKernelGGL(k_read_pop<S>, dim3(g), dim3(256), 0, st, a, (const typename Store<S>::raw *)src, f);
        return hipGetLastError();
    }
};

template <typename S>
struct WritePopF {
    static hipError_t run(const View &v, const double *f, void *dst, hipStream_t st)
    {
        const CellArgs a = make_cell_args(v);
        const int g = grid_for((int64_t)v.nx * v.ny, 256, 65536);
        hipLaunchKernelGGL(k_write_pop<S>, dim3(g), dim3(256), 0, st, a, f, (typename Store<S>::raw *)dst);
        return hipGetLastError();
    }
};

template <typename S>
struct DiagF {
    static hipError_t run(const View &v, const void *src, double *partials, double *result, hipStream_t st)
    {
        const CellArgs a = make_cell_args(v);
        const int g = grid_for((int64_t)v.nx * v.ny, 256, kRedBlocks);
        hipLaunchKernelGGL(k_diag<S>, dim3(g), dim3(256), 0, st, a, (const typename Store<S>::raw *)src, partials);
        hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partials, g, 4, 1.0, 0, result);
        return hipGetLastError();
    }
};

template <typename S>
struct ProjectF {
    static hipError_t run(const View &v, const void *src, int32_t mx, int32_t my, double *partials,
                          double *out, hipStream_t st)
    {
        const CellArgs a = make_cell_args(v);
        const int g = grid_for((int64_t)v.nx * v.ny, 256, kRedBlocks);
        double *sums = partials + (size_t)kRedBlocks * 18;
        hipLaunchKernelGGL(k_project<S>, dim3(g), dim3(256), 0, st, a, (const typename Store<S>::raw *)src,
                           (int)mx, (int)my, partials);
        hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partials, g, 18, 1.0, 0, sums);
        hipLaunchKernelGGL(k_project_finish, dim3(1), dim3(64), 0, st, sums, (int)mx, (int)my, v.nx, v.ny,
                           v.inv_scale, out);
        return hipGetLastError();
    }
};

}  // namespace

size_t storage_bytes(int32_t storage)
{
    switch (storage) {
    case LBM_STORE_F64: return 8;
    case LBM_STORE_F32: return 4;
    case LBM_STORE_F16:
    case LBM_STORE_BF16: return 2;
    default: return 0;
    }
}

int steps_per_launch(const lbm_launch &cfg) { return cfg.variant >= 8 && cfg.variant <= 13 ? cfg.variant - 6 : 1; }

// Output columns of a strip: 64 - 2(T-1) lanes see all their neighbours for
// T stages.  The count is rounded down to a whole number of 32-byte (else
// 16-byte) pieces of a stored row when that costs at most two columns, so
// that neighbouring strips' row stores meet on sector boundaries (measured:
// 58 -> 56 columns at T = 4 is +17 % for FP32 and FP64 storage; larger cuts
// cost more lanes than they gain).
int multi_strip_cols(int T, int elem_bytes)
{
    const int raw = 64 - 2 * (T - 1);
    for (int bytes : {32, 16}) {
        const int a = elem_bytes >= bytes ? 1 : bytes / elem_bytes;
        const int aligned = raw - raw % a;
        if (raw - aligned <= 2) return aligned;
    }
    return raw;
}

bool step_shape_supported(const View &v, const lbm_launch &cfg)
{
    if (cfg.variant >= 8 && cfg.variant <= 13) {
        // several steps per pass: one wave per strip and segment
        if (cfg.variant >= 11 && (cfg.flags & 1)) return false;   // T = 5, 6, 7: no non-temporal loads
        if (cfg.variant == 13 && (cfg.flags & 16)) return false;  // T = 7: plain pipeline only
        return cfg.block_x == 64 && cfg.block_y >= 1 && cfg.block_y <= 4 && cfg.rows >= 1 &&
               cfg.rows <= 4096 && (cfg.xcd_remap == 0 || cfg.xcd_remap == 1) && cfg.flags >= 0 &&
               cfg.flags <= 29 && !((cfg.flags & 8) && (cfg.flags & 2)) &&
               // skewed pipeline: T = 3 and 4, no non-temporal loads
               (!(cfg.flags & 16) || (cfg.variant >= 9 && !(cfg.flags & 1)));
    }
    if (cfg.variant < 0 || cfg.variant > 7) return false;
    if (cfg.block_x < 1 || cfg.block_y < 1 || cfg.rows < 1 || cfg.rows > 64) return false;
    if (cfg.block_x * cfg.block_y > 1024 || cfg.block_x * cfg.block_y < 64) return false;
    if (cfg.block_x % 64 != 0 && cfg.block_x * cfg.block_y % 64 != 0) return false;
    if (cfg.xcd_remap != 0 && cfg.xcd_remap != 1) return false;
    if (cfg.flags < 0 || cfg.flags > 3) return false;
    if ((cfg.flags & 2) && cfg.variant != 0 && cfg.variant != 4) return false;   // pipelining: one-cell kernels
    if (cfg.variant >= 1 && cfg.variant <= 3) {
        const int vx = 1 << cfg.variant;
        if (cfg.block_x % 64 != 0 || v.nx % vx != 0) return false;
    }
    if (cfg.variant >= 5 && v.nx % (1 << (cfg.variant - 4)) != 0) return false;
    return true;
}

hipError_t launch_step(const View &v, const void *src, void *dst, const lbm_launch &cfg, hipStream_t st)
{
    if (v.compute == LBM_COMPUTE_F64) {
        if (v.storage == LBM_STORE_F64) return launch_step_typed<double, double>(v, src, dst, cfg, st);
        return hipErrorInvalidValue;
    }
    switch (v.storage) {
    case LBM_STORE_F64: return launch_step_typed<double, float>(v, src, dst, cfg, st);
    case LBM_STORE_F32: return launch_step_typed<float, float>(v, src, dst, cfg, st);
    case LBM_STORE_F16: return launch_step_typed<f16_tag, float>(v, src, dst, cfg, st);
    case LBM_STORE_BF16: return launch_step_typed<bf16_tag, float>(v, src, dst, cfg, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(const View &v, const double *rho, const double *ux, const double *uy, void *dst,
                       double *partials, double *result, bool measure_only, hipStream_t st)
{
    return dispatch_storage<InitF>(v.storage, v, rho, ux, uy, dst, partials, result, measure_only, st);
}

hipError_t launch_moments(const View &v, const void *src, double *rho, double *ux, double *uy, hipStream_t st)
{
    return dispatch_storage<MomentsF>(v.storage, v, src, rho, ux, uy, st);
}

hipError_t launch_read_populations(const View &v, const void *src, double *f, hipStream_t st)
{
    return dispatch_storage<ReadPopF>(v.storage, v, src, f, st);
}

hipError_t launch_write_populations(const View &v, const double *f, void *dst, hipStream_t st)
{
    return dispatch_storage<WritePopF>(v.storage, v, f, dst, st);
}

hipError_t launch_diagnostics(const View &v, const void *src, double *partials, double *result, hipStream_t st)
{
    return dispatch_storage<DiagF>(v.storage, v, src, partials, result, st);
}

hipError_t launch_project(const View &v, const void *src, int32_t mx, int32_t my, double *partials, double *out,
                          hipStream_t st)
{
    return dispatch_storage<ProjectF>(v.storage, v, src, mx, my, partials, out, st);
}

Relax<float> relax_f32(const View &v) { return make_relax<float>(v); }
Relax<double> relax_f64(const View &v) { return make_relax<double>(v); }

void *pool_step_kernel(int cls)
{
    switch (cls) {
    case LBM_STORE_F64 * 2 + LBM_COMPUTE_F64: return reinterpret_cast<void *>(&k_pool_step<double, double>);
    case LBM_STORE_F64 * 2 + LBM_COMPUTE_F32: return reinterpret_cast<void *>(&k_pool_step<double, float>);
    case LBM_STORE_F32 * 2 + LBM_COMPUTE_F32: return reinterpret_cast<void *>(&k_pool_step<float, float>);
    case LBM_STORE_F16 * 2 + LBM_COMPUTE_F32: return reinterpret_cast<void *>(&k_pool_step<f16_tag, float>);
    case LBM_STORE_BF16 * 2 + LBM_COMPUTE_F32: return reinterpret_cast<void *>(&k_pool_step<bf16_tag, float>);
    default: return nullptr;
    }
}

void *pool_commit_kernel() { return reinterpret_cast<void *>(&k_pool_commit); }

namespace {
template <typename S, typename C>
void *pool_multi_typed(int T, int flags)
{
#define LBM_PM(T_, F_) \
    if (T == T_ && flags == F_) return reinterpret_cast<void *>(&k_pool_multi<S, C, T_, F_>);
#define LBM_PM_T(T_) LBM_PM(T_, 0) LBM_PM(T_, 2) LBM_PM(T_, 4) LBM_PM(T_, 12)
    LBM_PM_T(2)
    LBM_PM_T(3)
    LBM_PM_T(4)
    LBM_PM_T(5)
    LBM_PM_T(6)
    LBM_PM_T(7)
#undef LBM_PM_T
#undef LBM_PM
    return nullptr;
}
}  // namespace

void *pool_multi_kernel(int cls, int T, int flags)
{
    switch (cls) {
    case LBM_STORE_F64 * 2 + LBM_COMPUTE_F64: return pool_multi_typed<double, double>(T, flags);
    case LBM_STORE_F64 * 2 + LBM_COMPUTE_F32: return pool_multi_typed<double, float>(T, flags);
    case LBM_STORE_F32 * 2 + LBM_COMPUTE_F32: return pool_multi_typed<float, float>(T, flags);
    case LBM_STORE_F16 * 2 + LBM_COMPUTE_F32: return pool_multi_typed<f16_tag, float>(T, flags);
    case LBM_STORE_BF16 * 2 + LBM_COMPUTE_F32: return pool_multi_typed<bf16_tag, float>(T, flags);
    default: return nullptr;
    }
}

hipError_t launch_pool_step(int cls, const PoolHeader *hdr, const PoolMember *mem, const PoolTile *tiles, int i,
                            int kk, int T, int grid, int block, hipStream_t st)
{
    void *f = pool_step_kernel(cls);
    if (!f) return hipErrorInvalidValue;
    void *args[] = {(void *)&hdr, (void *)&mem, (void *)&tiles, (void *)&cls, (void *)&i, (void *)&kk, (void *)&T};
    return hipLaunchKernel(f, dim3(grid), dim3(block), args, 0, st);
}

hipError_t launch_pool_multi(int cls, int T, int flags, const PoolHeader *hdr, const PoolMember *mem,
                             const PoolTile *tiles, int j, int grid, int waves, hipStream_t st)
{
    void *f = pool_multi_kernel(cls, T, flags);
    if (!f) return hipErrorInvalidValue;
    void *args[] = {(void *)&hdr, (void *)&mem, (void *)&tiles, (void *)&cls, (void *)&j};
    return hipLaunchKernel(f, dim3(grid), dim3(64, waves), args, 0, st);
}

hipError_t launch_pool_commit(PoolMember *mem, int nmem, int kk, int T, hipStream_t st)
{
    hipLaunchKernelGGL(k_pool_commit, dim3((nmem + 255) / 256), dim3(256), 0, st, mem, nmem, kk, T);
    return hipGetLastError();
}

}  // namespace lbm
