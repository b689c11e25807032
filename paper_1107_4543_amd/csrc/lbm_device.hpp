// Device-side building blocks of the D2Q9 MRT lattice Boltzmann step for gfx950.
//
// State representation.  The library stores the fluctuation of the
// populations about the uniform equilibrium of the base state (rho0, j0):
//     g_i = (f_i - f^eq_i(rho0, j0)) * 2^p
// (the mean/fluctuation split of Sec. 4.1, Eq. perturb-f).  A uniform
// equilibrium is a fixed point of both collision and streaming, so g obeys
// the same update as f.  Storing g instead of f keeps the stored numbers at
// the size of the acoustic fluctuation, which is what makes FP32 and 16-bit
// storage usable for small-amplitude acoustics.
//
// Collision in increment form.  With Lambda = M^{-1} S M (Sec. 2.1) and
// M^{-1} = M^T D^{-1}, D = diag(9,6,6,36,36,12,12,4,4) (the rows of M are
// orthogonal), one collision is
//     g*_i = g_i + sum_{k=3..8} M_ki (s_k / D_k) (dmeq_k - m'_k),
// where m' = M g and dmeq = m^eq(rho0 + rho', j0 + j') - m^eq(rho0, j0) is
// the equilibrium (Sec. 2.3) written without cancellation:
//     dQ = |j|^2/rho - |j0|^2/rho0 = (2 j0.j' + |j'|^2 - Q0 rho') / rho
//     dP = (jx^2 - jy^2)/rho - P0 ,  dX = jx jy / rho - X0   (same pattern)
// with Q0 = |j0|^2/rho0, P0 = (j0x^2 - j0y^2)/rho0, X0 = j0x j0y/rho0.
// M and M^T have integer entries, so both transforms are add/sub chains
// (small integer multiples go into fused multiply-adds); besides the
// quadratic terms of the equilibrium, the only multiplications are by the
// per-lattice constants s_k / D_k, and the only division is 1/rho.
//
// Velocity order: v_0=(0,0) v_1=(1,0) v_2=(0,1) v_3=(-1,0) v_4=(0,-1)
//                 v_5=(1,1) v_6=(-1,1) v_7=(-1,-1) v_8=(1,-1).
// Moment order (rows of M): rho, jx, jy, e, eps, qx, qy, pxx, pxy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Per-lattice constants of the collision, in the compute type T.
template <typename T>
struct Relax {
    T lam_e, lam_eps, lam_q, lam_nu;   // s_k / D_k: s_e/36, s_eps/36, s_q/12, s_nu/4
    T rho0, j0x, j0y;                  // base state
    T Q0, P0, X0;                      // |j0|^2/rho0, (j0x^2-j0y^2)/rho0, j0x j0y/rho0
};

// Equilibrium moment deviation dmeq(rho', j') about (rho0, j0), Sec. 2.3.
template <typename T>
__host__ __device__ __forceinline__ void delta_meq(T rho, T jx, T jy, const Relax<T> &r, T dm[9])
{
    const T inv = T(1) / (r.rho0 + rho);
    const T dQ = (T(2) * (r.j0x * jx + r.j0y * jy) + jx * jx + jy * jy - r.Q0 * rho) * inv;
    const T dP = (T(2) * (r.j0x * jx - r.j0y * jy) + jx * jx - jy * jy - r.P0 * rho) * inv;
    const T dX = (r.j0x * jy + r.j0y * jx + jx * jy - r.X0 * rho) * inv;
    dm[0] = rho;
    dm[1] = jx;
    dm[2] = jy;
    dm[3] = T(-2) * rho + T(3) * dQ;
    dm[4] = rho - T(3) * dQ;
    dm[5] = -jx;
    dm[6] = -jy;
    dm[7] = dP;
    dm[8] = dX;
}

// f = M^{-1} m = M^T D^{-1} m, folded.
template <typename T>
__host__ __device__ __forceinline__ void back_transform(const T m[9], T f[9])
{
    const T r = m[0] / T(9);
    const T ex = m[1] / T(6), ey = m[2] / T(6);
    const T ea = -m[3] / T(36) - m[4] / T(18);   // axis directions
    const T ed = m[3] / T(18) + m[4] / T(36);    // diagonal directions
    const T qx = m[5] / T(6), qy = m[6] / T(6);
    const T qxd = m[5] / T(12), qyd = m[6] / T(12);
    const T pxx = m[7] / T(4), pxy = m[8] / T(4);
    f[0] = r - m[3] / T(9) + m[4] / T(9);
    f[1] = r + ex + ea - qx + pxx;
    f[2] = r + ey + ea - qy - pxx;
    f[3] = r - ex + ea + qx + pxx;
    f[4] = r - ey + ea + qy - pxx;
    f[5] = r + ex + ey + ed + qxd + qyd + pxy;
    f[6] = r - ex + ey + ed - qxd + qyd - pxy;
    f[7] = r - ex - ey + ed - qxd - qyd + pxy;
    f[8] = r + ex - ey + ed + qxd - qyd - pxy;
}

// Fused multiply-add written out (the library is built without automatic
// contraction, so every kernel evaluates exactly these operations).
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/x: the hardware reciprocal (about 1 ulp) in FP32; in FP64 the hardware
// estimate refined by two Newton-Raphson steps r <- r + r (1 - x r), each
// of which squares the relative error (x is a density near rho0: positive
// and normal, so the special cases of a full division do not arise).
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// The collision increment dg = g* - g of one cell in the compute type T.
//
// g may hold the deviations multiplied by 2^p (16-bit storage); t = 2^-p is
// then applied only where the equilibrium is not homogeneous of degree one
// (the |j|^2 terms and the density in the denominator), so that every
// intermediate value is exactly 2^p times its unscaled counterpart and dg
// comes out scaled by 2^p with the same rounding.
//
// The relaxation terms a_k = (s_k / D_k)(dmeq_k - m'_k) are written in the
// populations' partial sums, with the conserved moments substituted
// (a = axis sum, b = diagonal sum, rho' = g_0 + a + b):
//     a_e   = lam_e   (2 g_0 - a - 4 b + 3 dQ)
//     a_eps = 3 lam_eps (a - g_0 - dQ)
//     a_qx  = lam_q   (dx1 - 2 dxd)      (dx1 = g_1 - g_3, dxd = sum_diag c_x g)
//     a_pxx = lam_nu  (dP - pxx),  a_pxy = lam_nu (dX - pxy)
// with dQ, dP, dX numerators N over rho = rho0 + t rho':
//     N_Q = ax + ay - Q0 rho',  N_P = ax - ay - P0 rho',  ax = jx (t jx + 2 j0x)
//     N_X = jy (t jx + j0x) + j0y jx - X0 rho'
// (the same quantities as the equilibrium above, in fewer operations; the
// kinetic moments e, eps, q are never formed).  The q terms enter M^T a
// through lam_q directly (dg_1 = A + lam_pxx - 2 lam_q x_5, dg_5 = B + lam_pxy
// + lam_q (x_5 + x_6), ...).
template <typename T>
__device__ __forceinline__ void collide_increment(const T g[9], const Relax<T> &r, T t, T dg[9])
{
    // partial sums of the populations
    const T s13 = g[1] + g[3], s24 = g[2] + g[4];
    const T s57 = g[5] + g[7], s68 = g[6] + g[8];
    const T a = s13 + s24;                              // axis sum
    const T b = s57 + s68;                              // diagonal sum
    const T rho = g[0] + a + b;
    const T dx1 = g[1] - g[3], dy1 = g[2] - g[4];
    const T d57 = g[5] - g[7], d86 = g[8] - g[6];
    const T dxd = d57 + d86;                            // sum_diag c_x g
    const T dyd = d57 - d86;                            // sum_diag c_y g
    const T jx = dx1 + dxd, jy = dy1 + dyd;
    const T pxx = s13 - s24;
    const T pxy = s57 - s68;
    // equilibrium numerators (Sec. 2.3) about (rho0, j0), one reciprocal
    const T inv = recip(fmad(t, rho, r.rho0));
    const T ax = jx * fmad(t, jx, T(2) * r.j0x);
    const T ay = jy * fmad(t, jy, T(2) * r.j0y);
    const T nQ = fmad(-r.Q0, rho, ax) + ay;
    const T nP = fmad(-r.P0, rho, ax) - ay;
    const T nX = fmad(-r.X0, rho, fmad(r.j0y, jx, jy * fmad(t, jx, r.j0x)));
    // relaxation terms a_k, k = 3..8
    const T a3 = r.lam_e * fmad(nQ, T(3) * inv, fmad(T(-4), b, fmad(T(2), g[0], -a)));
    const T a4 = (T(3) * r.lam_eps) * fmad(-nQ, inv, a - g[0]);
    const T x5 = fmad(T(-2), dxd, dx1);
    const T x6 = fmad(T(-2), dyd, dy1);
    const T x7 = fmad(nP, inv, -pxx);
    const T x8 = fmad(nX, inv, -pxy);
    // dg = M^T a
    const T A = fmad(T(-2), a4, -a3);
    const T B = fmad(T(2), a3, a4);
    const T A7 = fmad(r.lam_nu, x7, A), Am7 = fmad(-r.lam_nu, x7, A);
    const T B8 = fmad(r.lam_nu, x8, B), Bm8 = fmad(-r.lam_nu, x8, B);
    const T q2 = T(2) * r.lam_q;
    const T s56 = x5 + x6, d56 = x5 - x6;
    dg[0] = a4 - a3;                                    // a quarter of the rest population's increment
    dg[1] = fmad(-q2, x5, A7);
    dg[2] = fmad(-q2, x6, Am7);
    dg[3] = fmad(q2, x5, A7);
    dg[4] = fmad(q2, x6, Am7);
    dg[5] = fmad(r.lam_q, s56, B8);
    dg[6] = fmad(-r.lam_q, d56, Bm8);
    dg[7] = fmad(-r.lam_q, s56, B8);
    dg[8] = fmad(r.lam_q, d56, Bm8);
}

// ---- storage types ---------------------------------------------------------
//
// A storage tag S selects the type held in HBM (raw), the type the stored
// value is widened to (wide: double for FP64 storage, float otherwise) and the
// rounding back (round to nearest even).  16-bit storage carries the
// per-lattice power-of-two scale.

struct f16_tag {};
struct bf16_tag {};

template <typename S>
struct Store;

template <>
struct Store<double> {
    using raw = double;
    using wide = double;
    static constexpr bool scaled = false;
    __device__ static __forceinline__ double widen(double v) { return v; }
    __device__ static __forceinline__ double narrow(double v) { return v; }
};

template <>
struct Store<float> {
    using raw = float;
    using wide = float;
    static constexpr bool scaled = false;
    __device__ static __forceinline__ float widen(float v) { return v; }
    __device__ static __forceinline__ float narrow(float v) { return v; }
};

template <>
struct Store<f16_tag> {
    using raw = _Float16;
    using wide = float;
    static constexpr bool scaled = true;
    __device__ static __forceinline__ float widen(_Float16 v) { return (float)v; }
    __device__ static __forceinline__ _Float16 narrow(float v) { return (_Float16)v; }
};

template <>
struct Store<bf16_tag> {
    using raw = uint16_t;
    using wide = float;
    static constexpr bool scaled = true;
    __device__ static __forceinline__ float widen(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
    // the hardware conversion (round to nearest even; NaN stays NaN)
    __device__ static __forceinline__ uint16_t narrow(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
};

// N consecutive raw values as one naturally aligned vector (one wide load or
// store instruction).
template <typename R, int N>
struct VecOf {
    typedef R type __attribute__((ext_vector_type(N)));
};
template <typename R>
struct VecOf<R, 1> {
    typedef R type;
};

}  // namespace lbm
