// Several-steps-per-pass kernels (single lattice and pool) for BF16 storage (FP32 collide).
// The kernels are defined in lbm_step_common.hpp; this unit instantiates
// the supported (T, flags) pairs and launches them.
#include "lbm_step_common.hpp"

namespace lbm {

namespace {

template <typename S, typename C>
hipError_t launch_multi_impl(const StepArgs<C> &a, dim3 grid, dim3 block, int T, int flags, hipStream_t st)
{
    switch ((T - 2) * 64 + flags) {
#define LBM_MULTI(T_, F_)                                                                    \
    case (T_ - 2) * 64 + F_: hipLaunchKernelGGL((k_step_multi<S, C, T_, F_>), grid, block, 0, st, a); break;
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
        // workgroup-shared halo (bit 5), T = 4 .. 7
#define LBM_MULTI_WG(T_) LBM_MULTI(T_, 32) LBM_MULTI(T_, 34) LBM_MULTI(T_, 40) \
                         LBM_MULTI(T_, 48) LBM_MULTI(T_, 50) LBM_MULTI(T_, 56)
        LBM_MULTI_WG(4)
        LBM_MULTI_WG(5)
        LBM_MULTI_WG(6)
        LBM_MULTI_WG(7)
#undef LBM_MULTI_WG
#undef LBM_MULTI_E
#undef LBM_MULTI_T
#undef LBM_MULTI
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S, typename C>
void *pool_multi_impl(int T, int flags)
{
#define LBM_PM(T_, F_) \
    if (T == T_ && flags == F_) return reinterpret_cast<void *>(&k_pool_multi<S, C, T_, F_>);
#define LBM_PM_T(T_) LBM_PM(T_, 0) LBM_PM(T_, 2) LBM_PM(T_, 4) LBM_PM(T_, 12) LBM_PM(T_, 32) LBM_PM(T_, 34) \
                     LBM_PM(T_, 96) LBM_PM(T_, 98)
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

template <>
hipError_t launch_multi<bf16_tag, float>(const StepArgs<float> &a, dim3 grid, dim3 block, int T, int flags, hipStream_t st)
{
    return launch_multi_impl<bf16_tag, float>(a, grid, block, T, flags, st);
}

template <>
void *pool_multi_fn<bf16_tag, float>(int T, int flags)
{
    return pool_multi_impl<bf16_tag, float>(T, flags);
}

}  // namespace lbm
