// sweeps.hip -- single-grid sweep kernels: thin wrappers around the bodies in
// sweep_body.h, and their launchers.
#include "claw_launch.h"
#include "sweep_body.h"

namespace claw {

// LIMK: limiter fixed at compile time (the MC kernels) or LIM_RUNTIME.
// FP32 row sweeps of the built-in systems are held to 80 VGPRs (6 wavefronts
// per SIMD).
template <typename R, int SYS>
constexpr int row_waves_per_eu() { return sizeof(R) == 4 && !is_plugin(SYS) ? 6 : 1; }
template <typename R, int SYS, int MEQN, int CPL, bool SPEEDS, int LIMK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(row_waves_per_eu<R, SYS>())))
void k_sweep_row(SweepArgs<R> a) {
    const int by = (int)(blockIdx.y + blockIdx.z * gridDim.y);
    row_body<R, SYS, MEQN, CPL, SPEEDS, LIMK, row_rpw_single<R>()>(a, (int)blockIdx.x, by,
                                              blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0);
}

template <typename R, int SYS, int MEQN, int NRM, int PF, bool SPEEDS, int LIMK>
__global__ __launch_bounds__(256) void k_sweep_col(SweepArgs<R> a) {
    col_body<R, SYS, MEQN, NRM, PF, SPEEDS, LIMK>(a, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z,
                                                  blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

template <typename R, int SYS, int MEQN, bool SPEEDS, int LIMK>
static hipError_t launch_row(const SweepArgs<R>& a, hipStream_t s) {
    constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
    const int segs = ceil_div(a.nx, 62 * CPL);
    const int groups = ceil_div(a.nrows, 4 * row_rpw_single<R>());
    const int gy = groups < 32768 ? groups : 32768;
    const int gz = ceil_div(groups, gy);
    hipLaunchKernelGGL((k_sweep_row<R, SYS, MEQN, CPL, SPEEDS, LIMK>), dim3(segs, gy, gz), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R, int SYS, int MEQN, int NRM, bool SPEEDS, int LIMK>
static hipError_t launch_col(const SweepArgs<R>& a, hipStream_t s) {
    constexpr int PF = 4;
    const dim3 grid(ceil_div(ceil_div(a.nx, 64), 4), ceil_div(a.m, a.chunk), a.nlines_o);
    hipLaunchKernelGGL((k_sweep_col<R, SYS, MEQN, NRM, PF, SPEEDS, LIMK>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// whether a system has a z sweep: 3D acoustics, plug-ins that allow 3D
template <typename R, int SYS, int MEQN>
constexpr bool has_z() {
    if constexpr (is_plugin(SYS)) return Plug<R, SYS>::NDIM_MAX == 3;
    else return MEQN == 4;
}

template <typename R, int SYS, int MEQN, bool SPEEDS, int LIMK>
static hipError_t launch_dir(const SweepArgs<R>& a, hipStream_t s) {
    if (a.dir == 0) return launch_row<R, SYS, MEQN, SPEEDS, LIMK>(a, s);
    if (a.dir == 1) return launch_col<R, SYS, MEQN, 2, SPEEDS, LIMK>(a, s);
    if constexpr (has_z<R, SYS, MEQN>()) return launch_col<R, SYS, MEQN, 3, SPEEDS, LIMK>(a, s);
    return hipErrorInvalidValue;
}

// The MC limiter (the default) runs kernels specialised for it; the others
// share kernels that read the limiter from the arguments.  Speed passes form
// no correction.
template <typename R, int SYS, int MEQN>
static hipError_t launch_kind(const SweepArgs<R>& a, bool speeds, hipStream_t s) {
    if (speeds) return launch_dir<R, SYS, MEQN, true, LIM_RUNTIME>(a, s);
    if (a.limiter == LIM_MC) return launch_dir<R, SYS, MEQN, false, LIM_MC>(a, s);
    return launch_dir<R, SYS, MEQN, false, LIM_RUNTIME>(a, s);
}

template <typename R>
hipError_t launch_sweep(const SweepArgs<R>& a, int sys, int meqn, bool speeds, hipStream_t s) {
    if (sys == SYS_SW && meqn == 3) return launch_kind<R, SYS_SW, 3>(a, speeds, s);
    if (sys == SYS_AC && meqn == 3) return launch_kind<R, SYS_AC, 3>(a, speeds, s);
    if (sys == SYS_AC && meqn == 4) return launch_kind<R, SYS_AC, 4>(a, speeds, s);
    if (sys == SYS_ACV && meqn == 3) return launch_kind<R, SYS_ACV, 3>(a, speeds, s);
    if (sys == SYS_ACV && meqn == 4) return launch_kind<R, SYS_ACV, 4>(a, speeds, s);
#define CLAW_PLUGIN_LAUNCH(id, P) \
    if (sys == id && meqn == P<R>::MEQN) return launch_kind<R, id, P<R>::MEQN>(a, speeds, s);
    CLAW_PLUGINS(CLAW_PLUGIN_LAUNCH)
#undef CLAW_PLUGIN_LAUNCH
    return hipErrorInvalidValue;
}

template hipError_t launch_sweep<float>(const SweepArgs<float>&, int, int, bool, hipStream_t);
template hipError_t launch_sweep<double>(const SweepArgs<double>&, int, int, bool, hipStream_t);

}  // namespace claw
