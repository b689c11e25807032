// Kernels of the D2Q9 MRT lattice Boltzmann library (gfx950, wave64): one
// step per launch, the pool's one-step kernel, initialisation, readback,
// reductions, and the launch dispatch (the several-steps kernels live in
// lbm_step_common.hpp and are instantiated in lbm_multi_<type>.hip).
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

#include "lbm_step_common.hpp"

namespace lbm {

namespace {

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

template <typename S, typename C>
__global__ void __launch_bounds__(1024) k_pool_step(const PoolHeader *hdr, const PoolMember *mem,
                                                     const PoolTile *tiles, int range, int i, int kk, int T)
{
    using R = typename Store<S>::raw;
    using W = typename Store<S>::wide;
    const int begin = hdr->begin[range], end = hdr->end[range];
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
        // strips of multi_strip_cols output columns, segments of `rows` rows,
        // one wave each (with the shared halo: one workgroup of block_y
        // waves each, strips as wide as its lanes allow)
        const int T = cfg.variant - 6;
        const bool wg = (cfg.flags & kWgHalo) != 0;
        a.out_cols = multi_strip_cols(T, (int)sizeof(typename Store<S>::raw), wg ? 64 * cfg.block_y : 64);
        a.tiles_x = (v.nx + a.out_cols - 1) / a.out_cols;
        a.tile_h = cfg.rows;
        const int segs = (v.ny + cfg.rows - 1) / cfg.rows;
        a.nwaves = a.tiles_x * segs;
        a.nblocks = wg ? a.nwaves : (a.nwaves + cfg.block_y - 1) / cfg.block_y;
    }
    const dim3 grid(a.nblocks), block(cfg.block_x, cfg.block_y);
    if (cfg.variant >= 8) return launch_multi<S, C>(a, grid, block, cfg.variant - 6, cfg.flags, st);
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
int multi_strip_cols(int T, int elem_bytes, int lanes)
{
    const int raw = lanes - 2 * (T - 1);
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
        // T = 7 with one wave per strip: plain pipeline only
        if (cfg.variant == 13 && (cfg.flags & 16) && !(cfg.flags & kWgHalo)) return false;
        if (cfg.flags & kWgHalo) {
            // shared halo: T = 4 .. 7, flags 32, 34 or 40 (no shuffles,
            // loads one or two rows ahead or none), plain or skewed
            // pipeline (+16); FP64 storage only T = 6, 7, plain
            if (cfg.variant < 10) return false;
            const int f = cfg.flags & ~16;      // bit 4: the skewed pipeline, one exchange per row
            if (f != kWgHalo && f != (kWgHalo | 2) && f != (kWgHalo | 8)) return false;
            // FP64 storage: T = 6 and 7, plain pipeline
            if (v.storage == LBM_STORE_F64 && (cfg.variant < 12 || (cfg.flags & 16))) return false;
            return cfg.block_x == 64 && cfg.block_y >= 1 && cfg.block_y <= kWgMaxWaves && cfg.rows >= 1 &&
                   cfg.rows <= 4096 && (cfg.xcd_remap == 0 || cfg.xcd_remap == 1);
        }
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

void *pool_multi_kernel(int cls, int T, int flags)
{
    switch (cls) {
    case LBM_STORE_F64 * 2 + LBM_COMPUTE_F64: return pool_multi_fn<double, double>(T, flags);
    case LBM_STORE_F64 * 2 + LBM_COMPUTE_F32: return pool_multi_fn<double, float>(T, flags);
    case LBM_STORE_F32 * 2 + LBM_COMPUTE_F32: return pool_multi_fn<float, float>(T, flags);
    case LBM_STORE_F16 * 2 + LBM_COMPUTE_F32: return pool_multi_fn<f16_tag, float>(T, flags);
    case LBM_STORE_BF16 * 2 + LBM_COMPUTE_F32: return pool_multi_fn<bf16_tag, float>(T, flags);
    default: return nullptr;
    }
}

hipError_t launch_pool_step(int range, const PoolHeader *hdr, const PoolMember *mem, const PoolTile *tiles, int i,
                            int kk, int T, int grid, int block, hipStream_t st)
{
    void *f = pool_step_kernel(range / kChains);
    if (!f) return hipErrorInvalidValue;
    void *args[] = {(void *)&hdr, (void *)&mem, (void *)&tiles, (void *)&range, (void *)&i, (void *)&kk, (void *)&T};
    return hipLaunchKernel(f, dim3(grid), dim3(block), args, 0, st);
}

hipError_t launch_pool_multi(int range, int T, int flags, const PoolHeader *hdr, const PoolMember *mem,
                             const PoolTile *tiles, int j, int grid, int waves, hipStream_t st)
{
    void *f = pool_multi_kernel(range / kChains, T, flags);
    if (!f) return hipErrorInvalidValue;
    void *args[] = {(void *)&hdr, (void *)&mem, (void *)&tiles, (void *)&range, (void *)&j};
    return hipLaunchKernel(f, dim3(grid), dim3(64, waves), args, 0, st);
}

hipError_t launch_pool_commit(PoolMember *mem, int nmem, int kk, int T, hipStream_t st)
{
    hipLaunchKernelGGL(k_pool_commit, dim3((nmem + 255) / 256), dim3(256), 0, st, mem, nmem, kk, T);
    return hipGetLastError();
}

}  // namespace lbm
