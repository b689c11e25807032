/*
 * FP64 CPU oracle for the D2Q9 multi-relaxation-time lattice Boltzmann step
 * (Xu & Sagaut, "Optimal low-dispersion low-dissipation LBM schemes for
 * computational aeroacoustics").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow and obviously correct evaluation of the scheme.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * The step is written in the paper's absolute variables and order, unfused:
 *   1. moments            m = M f                          (Sec. 2.1, Eq. q-macro)
 *   2. conserved moments  W = (m_0, m_1, m_2) = (rho, j_x, j_y)
 *                                                          (Sec. 2.1, Eq. eq_conservative)
 *   3. equilibrium        m^eq(W) of the D2Q9 model        (Sec. 2.3, first display)
 *   4. relaxation         m*_k = m_k + s_k (m^eq_k - m_k), k = 3..8,
 *                         with S = diag(0,0,0,s_e,s_eps,s_q,s_q,s_nu,s_nu)
 *                                                          (Sec. 2.1, Eq. eq_noconservative;
 *                                                           Sec. 2.3, relaxation rates)
 *   5. back-transform     f* = M^{-1} m*                   (Sec. 2.1, Lambda = M^{-1} S M)
 *   6. streaming          f_i(x + v_i, t + 1) = f*_i(x)    (Sec. 2.1, Eq. blbs), periodic lattice
 *                                                          (Sec. 5.1, periodic boundaries)
 *
 * Readings of points the paper leaves open (they are listed with reasons in
 * the design notes of the repository):
 *   - velocity order: v_0=(0,0), v_1=(1,0), v_2=(0,1), v_3=(-1,0), v_4=(0,-1),
 *     v_5=(1,1), v_6=(-1,1), v_7=(-1,-1), v_8=(1,-1);
 *   - rows of M beyond rho and j (not printed): the Lallemand-Luo polynomial
 *     moments 1, c_x, c_y, -4+3|c|^2, 4-(21/2)|c|^2+(9/2)|c|^4,
 *     (-5+3|c|^2)c_x, (-5+3|c|^2)c_y, c_x^2-c_y^2, c_x c_y, which reproduce
 *     the printed equilibrium and the printed linearised collision Psi;
 *   - M^{-1} is obtained by a general Gauss-Jordan inverse, not from any
 *     closed form;
 *   - the state at integer t is the pre-collision f(t).
 *
 * Layout of every population array: f[i][y][x], i = 0..8, x fastest.
 * Compile with -O2 -fopenmp -ffp-contract=off (no FMA contraction, no
 * fast-math).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define Q 9

static const int VX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int VY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Copies the velocity set (its order fixes the population layout). */
void oracle_velocities(int32_t *cx, int32_t *cy)
{
    for (int i = 0; i < Q; ++i) {
        cx[i] = VX[i];
        cy[i] = VY[i];
    }
}

/* M[k][j] = k-th moment polynomial evaluated at velocity v_j.
 * Rows 0..2 are fixed by M_0j = 1, M_alpha j = v_j^alpha (Sec. 2.1). */
void oracle_build_M(double *M)
{
    for (int j = 0; j < Q; ++j) {
        const double cx = VX[j], cy = VY[j];
        const double c2 = cx * cx + cy * cy;
        M[0 * Q + j] = 1.0;
        M[1 * Q + j] = cx;
        M[2 * Q + j] = cy;
        M[3 * Q + j] = -4.0 + 3.0 * c2;
        M[4 * Q + j] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
        M[5 * Q + j] = (-5.0 + 3.0 * c2) * cx;
        M[6 * Q + j] = (-5.0 + 3.0 * c2) * cy;
        M[7 * Q + j] = cx * cx - cy * cy;
        M[8 * Q + j] = cx * cy;
    }
}

/* General n x n inverse by Gauss-Jordan elimination with partial pivoting.
 * Returns 0 on success, -1 if the matrix is singular. */
int oracle_invert(const double *A, double *Ainv, int n)
{
    double a[Q * 2 * Q];
    if (n > Q) return -1;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            a[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r * 2 * n + col]) > fabs(a[piv * 2 * n + col])) piv = r;
        if (a[piv * 2 * n + col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = a[col * 2 * n + c];
                a[col * 2 * n + c] = a[piv * 2 * n + c];
                a[piv * 2 * n + c] = t;
            }
        const double d = a[col * 2 * n + col];
        for (int c = 0; c < 2 * n; ++c) a[col * 2 * n + c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double fct = a[r * 2 * n + col];
            if (fct == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) a[r * 2 * n + c] -= fct * a[col * 2 * n + c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = a[r * 2 * n + n + c];
    return 0;
}

/* Equilibrium moments of the D2Q9 MRT model as functions of the conserved
 * moments (rho, j_x, j_y)  (Sec. 2.3, first display). */
void oracle_meq(double rho, double jx, double jy, double *meq)
{
    const double jj = jx * jx + jy * jy;
    meq[0] = rho;
    meq[1] = jx;
    meq[2] = jy;
    meq[3] = -2.0 * rho + 3.0 / rho * jj;
    meq[4] = rho - 3.0 / rho * jj;
    meq[5] = -jx;
    meq[6] = -jy;
    meq[7] = (jx * jx - jy * jy) / rho;
    meq[8] = jx * jy / rho;
}

/* Relaxation rates S_k for k = 0..8 from (s_e, s_eps, s_q, s_nu)
 * (Sec. 2.3: s_0=s_1=s_2=0, s_3=s_e, s_4=s_eps, s_5=s_6=s_q, s_7=s_8=s_nu). */
static void rates(const double *s4, double *S)
{
    S[0] = S[1] = S[2] = 0.0;
    S[3] = s4[0];
    S[4] = s4[1];
    S[5] = S[6] = s4[2];
    S[7] = S[8] = s4[3];
}

static void matvec(const double *A, const double *x, double *y)
{
    for (int r = 0; r < Q; ++r) {
        double acc = 0.0;
        for (int c = 0; c < Q; ++c) acc += A[r * Q + c] * x[c];
        y[r] = acc;
    }
}

/* Equilibrium initialisation: f(x, 0) = M^{-1} m^eq(rho, rho u). */
int oracle_init(int32_t nx, int32_t ny, const double *rho, const double *ux,
                const double *uy, double *f)
{
    double M[Q * Q], Minv[Q * Q];
    const size_t n = (size_t)nx * (size_t)ny;
    oracle_build_M(M);
    if (oracle_invert(M, Minv, Q)) return -1;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)n; ++c) {
        double meq[Q], fe[Q];
        oracle_meq(rho[c], rho[c] * ux[c], rho[c] * uy[c], meq);
        matvec(Minv, meq, fe);
        for (int i = 0; i < Q; ++i) f[(size_t)i * n + c] = fe[i];
    }
    return 0;
}

/* Collision of n independent cells: f* = M^{-1} (m + S (m^eq - m)), m = M f.
 * f and fstar are [9][n]. */
int oracle_collide(int64_t n, const double *s4, const double *f, double *fstar)
{
    double M[Q * Q], Minv[Q * Q], S[Q];
    oracle_build_M(M);
    if (oracle_invert(M, Minv, Q)) return -1;
    rates(s4, S);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)n; ++c) {
        double fl[Q], m[Q], meq[Q], ms[Q], fs[Q];
        for (int i = 0; i < Q; ++i) fl[i] = f[(size_t)i * n + c];
        matvec(M, fl, m);
        oracle_meq(m[0], m[1], m[2], meq);
        for (int k = 0; k < Q; ++k) ms[k] = m[k] + S[k] * (meq[k] - m[k]);
        matvec(Minv, ms, fs);
        for (int i = 0; i < Q; ++i) fstar[(size_t)i * n + c] = fs[i];
    }
    return 0;
}

/* Streaming on the periodic nx x ny lattice: f_i((x + v_i) mod L) = f*_i(x). */
void oracle_stream(int32_t nx, int32_t ny, const double *fstar, double *f)
{
    const size_t n = (size_t)nx * (size_t)ny;
    for (int i = 0; i < Q; ++i) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            const int yd = ((y + VY[i]) % ny + ny) % ny;
            for (int x = 0; x < nx; ++x) {
                const int xd = ((x + VX[i]) % nx + nx) % nx;
                f[(size_t)i * n + (size_t)yd * nx + xd] = fstar[(size_t)i * n + (size_t)y * nx + x];
            }
        }
    }
}

/* Advances the pre-collision state f by nsteps steps (collide everywhere,
 * then stream).  work must hold 9*nx*ny doubles. */
int oracle_run(int32_t nx, int32_t ny, const double *s4, double *f, int64_t nsteps, double *work)
{
    const int64_t n = (int64_t)nx * (int64_t)ny;
    for (int64_t t = 0; t < nsteps; ++t) {
        if (oracle_collide(n, s4, f, work)) return -1;
        oracle_stream(nx, ny, work, f);
    }
    return 0;
}

/* Macroscopic fields: rho = sum_i f_i, j = sum_i v_i f_i, u = j / rho
 * (Sec. 2.1, Eq. q-macro, rows 0..2 of M). */
void oracle_moments(int32_t nx, int32_t ny, const double *f, double *rho, double *ux, double *uy)
{
    const size_t n = (size_t)nx * (size_t)ny;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)n; ++c) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double v = f[(size_t)i * n + c];
            r += v;
            jx += VX[i] * v;
            jy += VY[i] * v;
        }
        rho[c] = r;
        ux[c] = jx / r;
        uy[c] = jy / r;
    }
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads for the following calls (ignored
 * without OpenMP); the arithmetic does not depend on it. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
