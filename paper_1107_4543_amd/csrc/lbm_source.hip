// Imposed equilibrium at one node: the acoustic point source of Sec. 5.1,
// where the density of one node is prescribed every step with zero velocity.
//
// The pre-collision populations of cell (x, y) are stored at P_i(x - v_i)
// (pull layout, see lbm_kernels.hip), so setting f(x, y) = f^eq(rho, u)
// writes one value into each of the nine neighbouring storage cells.
#include "lbm_internal.hpp"

namespace lbm {

namespace {

constexpr int SVX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int SVY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

struct NodeArgs {
    void *dst;
    int32_t nx, ny, pitch, x, y, pad;
    int64_t plane;
    double scale;
    double g[9];              // (f^eq(rho, u) - f^eq(rho0, u0)), FP64
};

template <typename S>
__global__ void k_set_node(NodeArgs a)
{
    const int i = threadIdx.x;
    if (i >= 9) return;
    using W = typename Store<S>::wide;
    int xs = a.x - SVX[i], ys = a.y - SVY[i];
    xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
    ys = ys < 0 ? ys + a.ny : (ys >= a.ny ? ys - a.ny : ys);
    typename Store<S>::raw *d = (typename Store<S>::raw *)a.dst;
    d[i * a.plane + (int64_t)ys * a.pitch + xs] = Store<S>::narrow((W)(a.g[i] * a.scale));
}

}  // namespace

hipError_t launch_set_node(const View &v, void *dst, int32_t x, int32_t y, double rho, double ux, double uy,
                           hipStream_t st)
{
    NodeArgs a;
    a.dst = dst;
    a.nx = v.nx;
    a.ny = v.ny;
    a.pitch = v.pitch;
    a.x = x;
    a.y = y;
    a.pad = 0;
    a.plane = v.plane;
    a.scale = v.scale;
    Relax<double> base{};
    base.rho0 = v.rho0;
    base.j0x = v.j0x;
    base.j0y = v.j0y;
    base.Q0 = (v.j0x * v.j0x + v.j0y * v.j0y) / v.rho0;
    base.P0 = (v.j0x * v.j0x - v.j0y * v.j0y) / v.rho0;
    base.X0 = v.j0x * v.j0y / v.rho0;
    double dm[9];
    delta_meq<double>(rho - v.rho0, rho * ux - v.j0x, rho * uy - v.j0y, base, dm);
    back_transform<double>(dm, a.g);
    switch (v.storage) {
    case LBM_STORE_F64: hipLaunchKernelGGL(k_set_node<double>, dim3(1), dim3(64), 0, st, a); break;
    case LBM_STORE_F32: hipLaunchKernelGGL(k_set_node<float>, dim3(1), dim3(64), 0, st, a); break;
    case LBM_STORE_F16: hipLaunchKernelGGL(k_set_node<f16_tag>, dim3(1), dim3(64), 0, st, a); break;
    case LBM_STORE_BF16: hipLaunchKernelGGL(k_set_node<bf16_tag>, dim3(1), dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
