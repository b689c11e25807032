// C ABI and host runtime of the D2Q9 MRT lattice Boltzmann library.
//
// The library owns only host-side handles.  Every device byte it touches is
// carved from the caller's workspace:
//   [ buffer 0 : 9 planes ][ buffer 1 : 9 planes ][ reduction scratch ]
// each part 256-byte aligned.  Kernels are enqueued on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lbm_device.hpp"
#include "lbm_internal.hpp"

using lbm::View;

namespace lbm {

// Compute units of the current device (queried once per device; 256 on
// MI355X).
int device_cus()
{
    static int cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

}  // namespace lbm

namespace {

using lbm::device_cus;

thread_local std::string g_err;

lbm_status fail(lbm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

lbm_status busy(const lbm_lattice *L)
{
    return fail(LBM_E_STATE, "lattice is being advanced by a pool (remove it or poll it first)");
}

lbm_status hip_fail(hipError_t e, const char *what)
{
    return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool rate_ok(double s) { return isfinite(s) && s > 0.0 && s <= 2.0; }

lbm_status validate(const lbm_desc *d)
{
    if (!d) return fail(LBM_E_INVAL, "desc is NULL");
    if (d->nx < 1 || d->ny < 1) return fail(LBM_E_INVAL, "nx, ny must be >= 1 (got %d, %d)", d->nx, d->ny);
    const int64_t pitch = ((int64_t)d->nx + 63) / 64 * 64;
    if (pitch * (int64_t)d->ny >= ((int64_t)1 << 31))
        return fail(LBM_E_INVAL, "lattice too large: pitch * ny must be < 2^31");
    if (lbm::storage_bytes(d->storage) == 0) return fail(LBM_E_INVAL, "unknown storage %d", d->storage);
    if ((uint64_t)pitch * (uint64_t)d->ny * lbm::storage_bytes(d->storage) >= ((uint64_t)1 << 32))
        return fail(LBM_E_INVAL, "lattice too large: one population plane must be smaller than 4 GiB");
    if (d->compute != LBM_COMPUTE_F64 && d->compute != LBM_COMPUTE_F32)
        return fail(LBM_E_INVAL, "unknown compute %d", d->compute);
    if (d->compute == LBM_COMPUTE_F64 && d->storage != LBM_STORE_F64)
        return fail(LBM_E_INVAL, "FP64 compute requires FP64 storage");
    if (!rate_ok(d->s_e) || !rate_ok(d->s_eps) || !rate_ok(d->s_q) || !rate_ok(d->s_nu))
        return fail(LBM_E_INVAL, "relaxation rates must lie in (0, 2] (s_e=%g s_eps=%g s_q=%g s_nu=%g)", d->s_e,
                    d->s_eps, d->s_q, d->s_nu);
    if (!isfinite(d->rho0) || d->rho0 <= 0.0) return fail(LBM_E_INVAL, "rho0 must be finite and > 0");
    if (!isfinite(d->u0x) || !isfinite(d->u0y)) return fail(LBM_E_INVAL, "u0 must be finite");
    if (d->scale_exp != LBM_SCALE_AUTO && (d->scale_exp < -60 || d->scale_exp > 60))
        return fail(LBM_E_INVAL, "scale_exp must be in [-60, 60] or LBM_SCALE_AUTO");
    if (d->flags != 0) return fail(LBM_E_INVAL, "flags must be 0");
    return LBM_OK;
}

void layout(const lbm_desc *d, int32_t *pitch, int64_t *plane, size_t *state_bytes, size_t *buf_bytes)
{
    *pitch = (d->nx + 63) / 64 * 64;
    *plane = (int64_t)*pitch * d->ny;
    *state_bytes = (size_t)9 * (size_t)*plane * lbm::storage_bytes(d->storage);
    *buf_bytes = align256(*state_bytes);
}

void set_scale(View &v, int p)
{
    v.scale_exp = p;
    v.scale = ldexp(1.0, p);
    v.inv_scale = ldexp(1.0, -p);
}

// One-step shape (also used for the steps a multi-step shape leaves over).
lbm_launch default_single(const View &)
{
    lbm_launch c{};
    c.variant = 0;
    c.block_x = 64;
    c.block_y = 4;
    c.rows = 1;
    c.xcd_remap = 1;
    return c;
}

// Segment rows of a shared-halo shape (T steps, waves per workgroup) that
// give about per_cu workgroups per compute unit in one round: strips of
// multi_strip_cols columns, as many segments as the resident workgroups
// allow, each as tall as the lattice then needs.  Taller segments repeat
// fewer of the pipeline's 2(T-1) start-up rows; one round keeps every
// compute unit equally loaded.
int wg_rows(const View &v, int T, int waves, int per_cu)
{
    const int cols = lbm::multi_strip_cols(T, (int)lbm::storage_bytes(v.storage), 64 * waves);
    const int tiles_x = (v.nx + cols - 1) / cols;
    const int segs = std::max(1, per_cu * device_cus() / tiles_x);
    return std::max(1, std::min(4096, (v.ny + segs - 1) / segs));
}

// Several steps per launch with the shape measured fastest for the storage
// type on the 4096^2 wave workload: for 32- and 16-bit storage the
// workgroup-shared halo with four waves per workgroup -- FP32: T = 7, loads
// not ahead (flags 32), segments for three workgroups per compute unit (92
// rows on 4096^2); FP16: T = 6, one row ahead (34), BF16: T = 6, two rows
// ahead (40), four per compute unit (69 rows); FP64: T = 7, loads not ahead
// (32), two per compute unit (137 rows; a wave then holds about 250
// registers).  This from 2^19 cells, with segments of at least 8 rows: on
// small lattices the segments that give that workgroup count are short and
// the pipeline's start-up rows weigh more, yet the several-steps kernel
// measured 1.3-2.7x the one-step kernel from 640^2 to 2048 x 1024 (FP32,
// FP64), and for 16-bit storage 1.2x (FP16) and even (BF16) at 768^2, 1.4-1.5x
// at 1024^2 and 2x at 1448^2.  Smaller lattices keep the one-step shape.
lbm_launch default_launch(const View &v)
{
    if ((int64_t)v.nx * v.ny < ((int64_t)1 << 19)) return default_single(v);
    lbm_launch c{};
    c.block_x = 64;
    c.xcd_remap = 1;
    switch (v.storage) {
    case LBM_STORE_F32: c.variant = 13; c.block_y = 4; c.flags = 32; c.rows = wg_rows(v, 7, 4, 3); break;
    case LBM_STORE_F16: c.variant = 12; c.block_y = 4; c.flags = 34; c.rows = wg_rows(v, 6, 4, 4); break;
    case LBM_STORE_BF16: c.variant = 12; c.block_y = 4; c.flags = 40; c.rows = wg_rows(v, 6, 4, 4); break;
    default: c.variant = 13; c.block_y = 4; c.flags = 32; c.rows = wg_rows(v, 7, 4, 2); break;
    }
    c.rows = std::max(c.rows, 8);
    return c;
}

// Tuner stage 1: workgroup shapes of the one-cell kernel.
std::vector<lbm_launch> shape_candidates(const View &v)
{
    std::vector<lbm_launch> out;
    const int shapes[][2] = {{64, 1}, {64, 2}, {64, 4}, {64, 8}, {128, 1}, {128, 2}, {128, 4},
                             {256, 1}, {256, 2}, {256, 4}, {512, 1}, {512, 2}, {1024, 1}};
    for (const auto &sh : shapes)
        for (int r : {1, 2, 4})
            for (int remap = 0; remap < 2; ++remap) {
                lbm_launch c{};
                c.variant = 0;
                c.block_x = sh[0];
                c.block_y = sh[1];
                c.rows = r;
                c.xcd_remap = remap;
                c.flags = 0;
                if (lbm::step_shape_supported(v, c)) out.push_back(c);
            }
    return out;
}

// Tuner stage 2: kernel variants and flags around the best shape.
std::vector<lbm_launch> variant_candidates(const View &v, const lbm_launch &best)
{
    std::vector<lbm_launch> out;
    for (int var = 0; var < 8; ++var)
        for (int flags = 0; flags < 4; ++flags)
            for (int rows : {best.rows, 2 * best.rows}) {
                lbm_launch c = best;
                c.variant = var;
                c.flags = flags;
                c.rows = rows;
                if (var > 0 && c.block_x % 64 != 0) c.block_x = 64 * ((c.block_x + 63) / 64);
                if (lbm::step_shape_supported(v, c)) out.push_back(c);
            }
    return out;
}

// Tuner stage 3: shapes that advance several steps per launch (one wave
// per strip, and the workgroup-shared halo with segments sized for two to
// four workgroups per compute unit).
std::vector<lbm_launch> multi_candidates(const View &v)
{
    std::vector<lbm_launch> out;
    for (int var = 10; var <= 13; ++var)
        for (int flags : {32, 34, 40, 48, 50})
            for (int per_cu : {1, 2, 3, 4}) {
                lbm_launch c{};
                c.variant = var;
                c.block_x = 64;
                c.block_y = 4;
                c.rows = wg_rows(v, var - 6, 4, per_cu);
                c.xcd_remap = 1;
                c.flags = flags;
                if (lbm::step_shape_supported(v, c)) out.push_back(c);
            }
    for (int var = 8; var <= 13; ++var)
        for (int by : {1, 4})
            for (int rows : {32, 64, 168, 176, 256})
                for (int flags : {0, 2, 4, 12, 18, 20}) {
                    lbm_launch c{};
                    c.variant = var;
                    c.block_x = 64;
                    c.block_y = by;
                    c.rows = rows;
                    c.xcd_remap = 1;
                    c.flags = flags;
                    if (rows <= 2 * v.ny && lbm::step_shape_supported(v, c)) out.push_back(c);
                }
    return out;
}

lbm_status time_shape(lbm_lattice *L, const lbm_launch &c, int reps, double *us)
{
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    lbm_status st = LBM_OK;
    // Every launch reads the current buffer and writes the other one, so
    // the state is unchanged and the other buffer ends as the next step.
    for (int k = 0; k < 2 && st == LBM_OK; ++k)
        if ((e = lbm::launch_step(L->v, L->buf[L->cur], L->buf[L->cur ^ 1], c, L->stream)) != hipSuccess)
            st = hip_fail(e, "step launch");
    if (st == LBM_OK && (e = hipEventRecord(e0, L->stream)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
    for (int k = 0; k < reps && st == LBM_OK; ++k)
        if ((e = lbm::launch_step(L->v, L->buf[L->cur], L->buf[L->cur ^ 1], c, L->stream)) != hipSuccess)
            st = hip_fail(e, "step launch");
    if (st == LBM_OK && (e = hipEventRecord(e1, L->stream)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
    if (st == LBM_OK && (e = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    if (st == LBM_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) st = hip_fail(e, "hipEventElapsedTime");
    if (st == LBM_OK) *us = 1000.0 * ms / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

void lbm::set_error_text(const char *msg) { g_err = msg; }

// View of a raw state described by desc alone (no handle, no workspace):
// validation and layout as for lbm_create; scale_exp must be explicit for
// 16-bit storage (the scale of a saved state is the lattice's, see
// lbm_get_desc).
lbm_status lbm::view_of_state(const lbm_desc *desc, View *v)
{
    lbm_status st = validate(desc);
    if (st != LBM_OK) return st;
    if (desc->scale_exp == LBM_SCALE_AUTO &&
        (desc->storage == LBM_STORE_F16 || desc->storage == LBM_STORE_BF16))
        return fail(LBM_E_INVAL, "16-bit storage needs an explicit scale_exp (the lattice's, from lbm_get_desc)");
    *v = View{};
    v->nx = desc->nx;
    v->ny = desc->ny;
    v->storage = desc->storage;
    v->compute = desc->compute;
    size_t sb, bb;
    layout(desc, &v->pitch, &v->plane, &sb, &bb);
    v->s_e = desc->s_e;
    v->s_eps = desc->s_eps;
    v->s_q = desc->s_q;
    v->s_nu = desc->s_nu;
    v->rho0 = desc->rho0;
    v->j0x = desc->rho0 * desc->u0x;
    v->j0y = desc->rho0 * desc->u0y;
    set_scale(*v, desc->scale_exp == LBM_SCALE_AUTO ? 0 : desc->scale_exp);
    return LBM_OK;
}

extern "C" {

const char *lbm_status_string(lbm_status s)
{
    switch (s) {
    case LBM_OK: return "ok";
    case LBM_E_INVAL: return "invalid argument";
    case LBM_E_NOMEM: return "workspace too small";
    case LBM_E_HIP: return "HIP runtime error";
    case LBM_E_NONFINITE: return "non-finite populations";
    case LBM_E_STATE: return "call out of order";
    default: return "unknown status";
    }
}

const char *lbm_last_error(void) { return g_err.c_str(); }

double lbm_s_from_nu(double nu)
{
    if (!(nu >= 0.0) || !isfinite(nu)) return NAN;
    return 1.0 / (3.0 * nu + 0.5);
}

size_t lbm_workspace_bytes(const lbm_desc *desc)
{
    if (validate(desc) != LBM_OK) return 0;
    int32_t pitch;
    int64_t plane;
    size_t sb, bb;
    layout(desc, &pitch, &plane, &sb, &bb);
    return 2 * bb + align256(lbm::kScratchBytes);
}

lbm_status lbm_create(const lbm_desc *desc, void *dev_ws, size_t ws_bytes, void *stream, lbm_lattice **out)
{
    if (!out) return fail(LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    lbm_status st = validate(desc);
    if (st != LBM_OK) return st;
    if (!dev_ws || ((uintptr_t)dev_ws & 255u)) return fail(LBM_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
    const size_t need = lbm_workspace_bytes(desc);
    if (ws_bytes < need) return fail(LBM_E_NOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);

    lbm_lattice *L = new (std::nothrow) lbm_lattice();
    if (!L) return fail(LBM_E_NOMEM, "host allocation failed");
    L->desc = *desc;
    View &v = L->v;
    v.nx = desc->nx;
    v.ny = desc->ny;
    v.storage = desc->storage;
    v.compute = desc->compute;
    size_t sb, bb;
    layout(desc, &v.pitch, &v.plane, &sb, &bb);
    v.s_e = desc->s_e;
    v.s_eps = desc->s_eps;
    v.s_q = desc->s_q;
    v.s_nu = desc->s_nu;
    v.rho0 = desc->rho0;
    v.j0x = desc->rho0 * desc->u0x;
    v.j0y = desc->rho0 * desc->u0y;
    // f^eq(rho0, j0) = M^{-1} m^eq(rho0, j0): the deviation formula about a zero base.
    lbm::Relax<double> zero{};
    double m[9];
    lbm::delta_meq<double>(v.rho0, v.j0x, v.j0y, zero, m);
    lbm::back_transform<double>(m, v.fbase);
    set_scale(v, desc->scale_exp == LBM_SCALE_AUTO ? 0 : desc->scale_exp);
    L->ws = (char *)dev_ws;
    L->ws_bytes = ws_bytes;
    L->buf_bytes = bb;
    L->state_bytes = sb;
    L->buf[0] = L->ws;
    L->buf[1] = L->ws + bb;
    L->partials = (double *)(L->ws + 2 * bb);
    L->result = L->partials + (size_t)lbm::kRedBlocks * lbm::kRedWidth;
    L->stream = (hipStream_t)stream;
    L->launch = default_launch(v);
    L->single = default_single(v);
    *out = L;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_lattice *lat)
{
    if (!lat) return fail(LBM_E_INVAL, "lattice is NULL");
    if (lat->pool) return busy(lat);
    delete lat;
    return LBM_OK;
}

lbm_status lbm_set_stream(lbm_lattice *lat, void *stream)
{
    if (!lat) return fail(LBM_E_INVAL, "lattice is NULL");
    lat->stream = (hipStream_t)stream;
    return LBM_OK;
}

lbm_status lbm_get_desc(const lbm_lattice *lat, lbm_desc *out)
{
    if (!lat || !out) return fail(LBM_E_INVAL, "NULL argument");
    *out = lat->desc;
    if (lat->initialized || lat->desc.scale_exp != LBM_SCALE_AUTO) out->scale_exp = lat->v.scale_exp;
    return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_lattice *lat, const double *rho, const double *ux, const double *uy)
{
    if (!lat || !rho || !ux || !uy) return fail(LBM_E_INVAL, "NULL argument");
    if (lat->pool) return busy(lat);
    hipError_t e;
    const bool sixteen = lat->v.storage == LBM_STORE_F16 || lat->v.storage == LBM_STORE_BF16;
    if (lat->desc.scale_exp == LBM_SCALE_AUTO) {
        int p = 0;
        if (sixteen) {
            if ((e = lbm::launch_init(lat->v, rho, ux, uy, nullptr, lat->partials, lat->result, true, lat->stream)) !=
                hipSuccess)
                return hip_fail(e, "init (measure)");
            double mx = 0.0;
            if ((e = hipMemcpyAsync(&mx, lat->result, sizeof(double), hipMemcpyDeviceToHost, lat->stream)) !=
                hipSuccess)
                return hip_fail(e, "hipMemcpyAsync");
            if ((e = hipStreamSynchronize(lat->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            if (!isfinite(mx)) return fail(LBM_E_INVAL, "initial fields are not finite");
            if (mx > 0.0) p = (int)floor(log2(8192.0 / mx));
            p = std::max(-60, std::min(60, p));
        }
        set_scale(lat->v, p);
    }
    if ((e = lbm::launch_init(lat->v, rho, ux, uy, lat->buf[0], lat->partials, lat->result, false, lat->stream)) !=
        hipSuccess)
        return hip_fail(e, "init");
    lat->cur = 0;
    lat->t = 0;
    lat->initialized = true;
    return LBM_OK;
}

namespace {

// The r < T steps left after the T-step launches of lbm_step: one launch of
// the current shape with r steps per pass when r >= 2 (then T > 2 and the
// current shape is a several-steps one) and that shape is supported (*ok);
// a shared-halo shape whose r-step version does not exist (r < 4) takes
// r steps with one wave per strip, loads one row ahead (flags 2); else r
// one-step launches.
lbm_launch remainder_shape(const lbm_lattice *lat, int r, bool *ok)
{
    lbm_launch c = lat->launch;
    c.variant = 6 + r;
    *ok = r >= 2 && lbm::step_shape_supported(lat->v, c);
    if (!*ok && r >= 2 && (c.flags & lbm::kWgHalo)) {
        c.flags = 2;
        *ok = lbm::step_shape_supported(lat->v, c);
    }
    return c;
}

}  // namespace

lbm_status lbm_step(lbm_lattice *lat, int64_t n)
{
    if (!lat) return fail(LBM_E_INVAL, "lattice is NULL");
    if (n < 0) return fail(LBM_E_INVAL, "n must be >= 0");
    if (!lat->initialized) return fail(LBM_E_STATE, "lbm_step before lbm_init_equilibrium");
    if (lat->pool) return busy(lat);
    const int T = lbm::steps_per_launch(lat->launch);
    auto launch = [&](const lbm_launch &c, int steps) -> lbm_status {
        hipError_t e = lbm::launch_step(lat->v, lat->buf[lat->cur], lat->buf[lat->cur ^ 1], c, lat->stream);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        lat->cur ^= 1;
        lat->t += steps;
        return LBM_OK;
    };
    lbm_status st;
    for (int64_t k = 0; k < n / T; ++k)
        if ((st = launch(lat->launch, T)) != LBM_OK) return st;
    const int r = (int)(n % T);
    bool ok;
    const lbm_launch rest = remainder_shape(lat, r, &ok);
    if (ok) return launch(rest, r);
    for (int k = 0; k < r; ++k)
        if ((st = launch(lat->single, 1)) != LBM_OK) return st;
    return LBM_OK;
}

int64_t lbm_step_launches(const lbm_lattice *lat, int64_t n)
{
    if (!lat || n < 0) return -1;
    const int T = lbm::steps_per_launch(lat->launch);
    const int r = (int)(n % T);
    bool ok;
    (void)remainder_shape(lat, r, &ok);
    return n / T + (ok ? 1 : r);
}

lbm_status lbm_read_moments(lbm_lattice *lat, double *rho, double *ux, double *uy)
{
    if (!lat || !rho || !ux || !uy) return fail(LBM_E_INVAL, "NULL argument");
    if (!lat->initialized) return fail(LBM_E_STATE, "read before init");
    if (lat->pool) return busy(lat);
    hipError_t e = lbm::launch_moments(lat->v, lat->buf[lat->cur], rho, ux, uy, lat->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "moments");
}

lbm_status lbm_diagnostics(lbm_lattice *lat, double out[4])
{
    if (!lat || !out) return fail(LBM_E_INVAL, "NULL argument");
    if (!lat->initialized) return fail(LBM_E_STATE, "diagnostics before init");
    if (lat->pool) return busy(lat);
    hipError_t e = lbm::launch_diagnostics(lat->v, lat->buf[lat->cur], lat->partials, lat->result, lat->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics");
    double h[4];
    if ((e = hipMemcpyAsync(h, lat->result, sizeof h, hipMemcpyDeviceToHost, lat->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(lat->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (int k = 0; k < 3; ++k) out[k] = h[k] * lat->v.inv_scale;
    out[3] = h[3];
    if (h[3] > 0.0) return fail(LBM_E_NONFINITE, "%.0f non-finite stored values at t=%lld", h[3], (long long)lat->t);
    return LBM_OK;
}

lbm_status lbm_project(lbm_lattice *lat, int32_t mx, int32_t my, double *dev_out)
{
    if (!lat || !dev_out) return fail(LBM_E_INVAL, "NULL argument");
    if (!lat->initialized) return fail(LBM_E_STATE, "project before init");
    if (lat->pool) return busy(lat);
    hipError_t e = lbm::launch_project(lat->v, lat->buf[lat->cur], mx, my, lat->partials, dev_out, lat->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "project");
}

lbm_status lbm_read_populations(lbm_lattice *lat, double *dev_f)
{
    if (!lat || !dev_f) return fail(LBM_E_INVAL, "NULL argument");
    if (!lat->initialized) return fail(LBM_E_STATE, "read before init");
    if (lat->pool) return busy(lat);
    hipError_t e = lbm::launch_read_populations(lat->v, lat->buf[lat->cur], dev_f, lat->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "read populations");
}

lbm_status lbm_write_populations(lbm_lattice *lat, const double *dev_f)
{
    if (!lat || !dev_f) return fail(LBM_E_INVAL, "NULL argument");
    if (lat->pool) return busy(lat);
    if (!lat->initialized && lat->desc.scale_exp == LBM_SCALE_AUTO &&
        (lat->v.storage == LBM_STORE_F16 || lat->v.storage == LBM_STORE_BF16))
        return fail(LBM_E_STATE, "16-bit storage with automatic scale: init before writing populations");
    hipError_t e = lbm::launch_write_populations(lat->v, dev_f, lat->buf[lat->cur], lat->stream);
    if (e != hipSuccess) return hip_fail(e, "write populations");
    lat->initialized = true;
    return LBM_OK;
}

lbm_status lbm_set_node_equilibrium(lbm_lattice *lat, int32_t x, int32_t y, double rho, double ux, double uy)
{
    if (!lat) return fail(LBM_E_INVAL, "lattice is NULL");
    if (!lat->initialized) return fail(LBM_E_STATE, "set node before init");
    if (lat->pool) return busy(lat);
    if (x < 0 || y < 0 || x >= lat->v.nx || y >= lat->v.ny) return fail(LBM_E_INVAL, "node (%d, %d) outside the lattice", x, y);
    if (!isfinite(rho) || rho <= 0.0 || !isfinite(ux) || !isfinite(uy)) return fail(LBM_E_INVAL, "rho must be finite and > 0, u finite");
    hipError_t e = lbm::launch_set_node(lat->v, lat->buf[lat->cur], x, y, rho, ux, uy, lat->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "set node");
}

size_t lbm_state_bytes(const lbm_lattice *lat) { return lat ? lat->state_bytes : 0; }

lbm_status lbm_save_state(lbm_lattice *lat, void *dev_dst)
{
    if (!lat || !dev_dst) return fail(LBM_E_INVAL, "NULL argument");
    if (!lat->initialized) return fail(LBM_E_STATE, "save before init");
    if (lat->pool) return busy(lat);
    hipError_t e = hipMemcpyAsync(dev_dst, lat->buf[lat->cur], lat->state_bytes, hipMemcpyDeviceToDevice, lat->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "hipMemcpyAsync");
}

lbm_status lbm_load_state(lbm_lattice *lat, const void *dev_src, int64_t t)
{
    if (!lat || !dev_src) return fail(LBM_E_INVAL, "NULL argument");
    if (t < 0) return fail(LBM_E_INVAL, "t must be >= 0");
    if (lat->pool) return busy(lat);
    if (!lat->initialized && lat->desc.scale_exp == LBM_SCALE_AUTO &&
        (lat->v.storage == LBM_STORE_F16 || lat->v.storage == LBM_STORE_BF16))
        return fail(LBM_E_STATE, "16-bit storage with automatic scale: init before loading a state");
    hipError_t e = hipMemcpyAsync(lat->buf[lat->cur], dev_src, lat->state_bytes, hipMemcpyDeviceToDevice, lat->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    lat->t = t;
    lat->initialized = true;
    return LBM_OK;
}

int64_t lbm_time(const lbm_lattice *lat) { return lat ? lat->t : -1; }

lbm_status lbm_get_launch(const lbm_lattice *lat, lbm_launch *out)
{
    if (!lat || !out) return fail(LBM_E_INVAL, "NULL argument");
    *out = lat->launch;
    return LBM_OK;
}

lbm_status lbm_set_launch(lbm_lattice *lat, const lbm_launch *cfg)
{
    if (!lat || !cfg) return fail(LBM_E_INVAL, "NULL argument");
    if (!lbm::step_shape_supported(lat->v, *cfg))
        return fail(LBM_E_INVAL, "launch shape (variant %d, %dx%d, rows %d) not supported for nx=%d", cfg->variant,
                    cfg->block_x, cfg->block_y, cfg->rows, lat->v.nx);
    lat->launch = *cfg;
    if (lbm::steps_per_launch(*cfg) == 1) lat->single = *cfg;
    return LBM_OK;
}

int32_t lbm_steps_per_launch(const lbm_launch *cfg) { return cfg ? lbm::steps_per_launch(*cfg) : 0; }

lbm_status lbm_time_launches(lbm_lattice *lat, int32_t n, double *avg_us)
{
    if (!lat || !avg_us || n < 1) return fail(LBM_E_INVAL, "bad argument");
    if (!lat->initialized) return fail(LBM_E_STATE, "time before init");
    if (lat->pool) return busy(lat);
    return time_shape(lat, lat->launch, n, avg_us);
}

lbm_status lbm_tune(lbm_lattice *lat, int32_t reps, lbm_launch *best, double *best_us)
{
    if (!lat || reps < 1) return fail(LBM_E_INVAL, "bad argument");
    if (!lat->initialized) return fail(LBM_E_STATE, "tune before init");
    if (lat->pool) return busy(lat);
    struct Timed {
        double us;
        lbm_launch c;
    };
    // shapes are ranked by time per step
    auto per_step = [&](const lbm_launch &c, int r, double *us) -> lbm_status {
        lbm_status st = time_shape(lat, c, r, us);
        if (st == LBM_OK) *us /= lbm::steps_per_launch(c);
        return st;
    };
    auto sweep = [&](const std::vector<lbm_launch> &cands, int r, std::vector<Timed> &out) -> lbm_status {
        for (const lbm_launch &c : cands) {
            double us;
            lbm_status st = per_step(c, r, &us);
            if (st != LBM_OK) return st;
            out.push_back({us, c});
        }
        std::sort(out.begin(), out.end(), [](const Timed &a, const Timed &b) { return a.us < b.us; });
        return LBM_OK;
    };
    auto same = [](const lbm_launch &a, const lbm_launch &b) {
        return a.variant == b.variant && a.block_x == b.block_x && a.block_y == b.block_y && a.rows == b.rows &&
               a.xcd_remap == b.xcd_remap && a.flags == b.flags;
    };
    // stage 1: workgroup shapes of the one-cell kernel
    std::vector<Timed> s1;
    lbm_status st = sweep(shape_candidates(lat->v), reps, s1);
    if (st != LBM_OK) return st;
    // stage 2: every variant and flag combination around the three best shapes
    std::vector<lbm_launch> c2;
    for (size_t k = 0; k < s1.size() && k < 3; ++k)
        for (const lbm_launch &c : variant_candidates(lat->v, s1[k].c)) {
            bool dup = false;
            for (const lbm_launch &d : c2) dup = dup || same(c, d);
            if (!dup) c2.push_back(c);
        }
    std::vector<Timed> s2 = s1;
    if ((st = sweep(c2, reps, s2)) != LBM_OK) return st;
    // the best one-step shape also serves the steps a multi-step shape leaves over
    const lbm_launch best_single = s2.front().c;
    // stage 3: several steps per launch
    if ((st = sweep(multi_candidates(lat->v), reps, s2)) != LBM_OK) return st;
    // final: re-time the six best with more launches, twice, keep the minimum
    std::vector<Timed> fin;
    for (size_t k = 0; k < s2.size() && fin.size() < 6; ++k) {
        bool dup = false;
        for (const Timed &d : fin) dup = dup || same(s2[k].c, d.c);
        if (dup) continue;
        double a, b;
        if ((st = per_step(s2[k].c, 4 * reps, &a)) != LBM_OK) return st;
        if ((st = per_step(s2[k].c, 4 * reps, &b)) != LBM_OK) return st;
        fin.push_back({std::min(a, b), s2[k].c});
    }
    std::sort(fin.begin(), fin.end(), [](const Timed &a, const Timed &b) { return a.us < b.us; });
    lat->launch = fin.front().c;
    lat->single = best_single;
    if (best) *best = fin.front().c;
    if (best_us) *best_us = fin.front().us;
    return LBM_OK;
}

}  // extern "C"
