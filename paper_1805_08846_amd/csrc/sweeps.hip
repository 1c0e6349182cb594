// sweeps.hip -- single-grid sweep kernels: thin wrappers around the bodies in
// sweep_body.h, and their launchers.
#include <stdlib.h>

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

// Whole-row x sweep of acoustics rows of exactly 64 CPL cells with
// extrapolation at both ends (256-cell FP32 rows: the 256^3 workload): one
// wavefront per row, every lane updates its CPL cells, so there are no halo
// lanes and no packed row tails, and a wavefront reads and writes exactly its
// row's cache lines.  The ghost cells equal the end cells, so the end faces
// carry no waves: lane 0 takes its own first cell as its left neighbour (face
// 0 solves two equal states), and the shifts that fetch a neighbour face or
// contribution give lane 0 and lane 63 zeros, which is exactly a face without
// waves (faces -1 and nx, nx + 1).  The end faces' speeds are the end cells'
// sound speeds, which faces 1 and nx - 1 carry as well, so the speed maximum
// is the one over faces 0 .. nx.  Same arithmetic per face as the row body.
template <typename R, int SYS, int MEQN, int CPL, bool SPEEDS, int LIMK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(row_waves_per_eu<R, SYS>())))
void k_sweep_row_whole(SweepArgs<R> a) {
    static_assert(SYS == SYS_AC || SYS == SYS_ACV, "whole-row sweeps are for acoustics");
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    typedef typename VecOf<R, CPL>::type V;
    constexpr int nrm = 1, tng = 2;
    constexpr int NC = contrib_width<SYS>();
    const int by = (int)(blockIdx.y + blockIdx.z * gridDim.y);
    const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0;
    if (by * 4 >= a.nrows) return;  // a block past the last row (whole block)
    if constexpr (SPEEDS) {
        if (a.auto_dt && a.ctrl->st[a.parity].dt_next > 0.0) return;  // next step already known
    }
    const int cur_guess = predicted_cur(a);
    const int lane = threadIdx.x & 63;
    const int row = by * 4 + wave_uniform((int)(threadIdx.x >> 6));
    const bool active = row < a.nrows;
    const unsigned fbytes = (unsigned)a.ncell * (unsigned)sizeof(R);
    const unsigned voff = ((unsigned)(active ? row : 0) * (unsigned)a.nx + (unsigned)(lane * CPL)) * (unsigned)sizeof(R);
    R q[CPL][MEQN];
    R zc[CPL][2];
    auto load = [&](const R* __restrict__ src) {
#pragma unroll
        for (int e = 0; e < MEQN; ++e) {
            V v = buf_load16<V>(field_rsrc(src + (size_t)e * (unsigned)a.ncell, fbytes), voff);
#pragma unroll
            for (int c = 0; c < CPL; ++c) q[c][e] = v[c];
        }
        if constexpr (SYS == SYS_ACV) {
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                V v = buf_load16<V>(field_rsrc(a.zc + (size_t)f * (unsigned)a.ncell, fbytes), voff);
#pragma unroll
                for (int c = 0; c < CPL; ++c) zc[c][f] = v[c];
            }
        }
    };
    load(pick_buf(a, (cur_guess + a.src_off) % 3));
    const Trial<R> tr = open_trial(a, 0, lead);
    if (tr.done && !SPEEDS) return;
    const R* __restrict__ src = pick_buf(a, (tr.cur + a.src_off) % 3);
    if (tr.cur != cur_guess) load(src);
    R* __restrict__ dst = pick_buf(a, (tr.cur + a.dst_off) % 3);
    const R nu = tr.nu;
    const R inv2Z = ac_inv2Z<R, SYS>(a);

    bool bad = false;
    C cell[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) make_cell<R, SYS, MEQN>(q[c], zc[c], nrm, tng, a.sqrt_grav, bad, cell[c]);
    C left;
    cell_prev(cell[CPL - 1], left);
    if (lane == 0) left = cell[0];  // ghost cell -1 = cell 0 (extrapolation)
    I f[CPL];
    solve_iface<R, SYS, 0>(left, cell[0], a, inv2Z, f[0]);
#pragma unroll
    for (int c = 1; c < CPL; ++c) solve_iface<R, SYS, 0>(cell[c - 1], cell[c], a, inv2Z, f[c]);
    R sm = iface_smax(f[0]);
#pragma unroll
    for (int c = 1; c < CPL; ++c) sm = rmax(sm, iface_smax(f[c]));
    if (!active) {
        sm = R(0);
        bad = false;
    }
    if constexpr (!SPEEDS) {
        I fprev, fnext;
        iface_prev(f[CPL - 1], fprev);  // lane 0: zeros, face -1 without waves
        iface_next(f[0], fnext);        // lane 63: zeros, face nx without waves
        Contrib<R, NC> k[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const I& km = c == 0 ? fprev : f[c - 1];
            const I& kp = c == CPL - 1 ? fnext : f[c + 1];
            limit_contrib(f[c], km, kp, nu, limiter_of<LIMK>(a), k[c]);
        }
        R Lnext[NC];
#pragma unroll
        for (int n = 0; n < NC; ++n) Lnext[n] = lane_next(k[0].L[n]);  // lane 63: face nx contributes 0
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (c < CPL - 1) apply_update<R, SYS, MEQN>(q[c], k[c].Rr, k[c + 1].L, nu, nrm, tng);
            else apply_update<R, SYS, MEQN>(q[c], k[c].Rr, Lnext, nu, nrm, tng);
        }
        if (active) {
#pragma unroll
            for (int e = 0; e < MEQN; ++e) {
                V v;
#pragma unroll
                for (int c = 0; c < CPL; ++c) v[c] = q[c][e];
                buf_store16<V>(field_rsrc(dst + (size_t)e * (unsigned)a.ncell, fbytes), voff, v);
            }
        }
    }
    block_finish(a, 0, sm, bad, lead);
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

// Whole-row sweeps on (CLAW_ROW_WHOLE=0 in the environment turns them off).
static bool row_whole_enabled() {
    static const bool on = [] {
        const char* e = getenv("CLAW_ROW_WHOLE");
        return !(e && e[0] == '0');
    }();
    return on;
}

template <typename R, int SYS, int MEQN, bool SPEEDS, int LIMK>
static hipError_t launch_row(const SweepArgs<R>& a, hipStream_t s) {
    constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
    if constexpr (SYS == SYS_AC || SYS == SYS_ACV) {
        if (a.nx == 64 * CPL && a.bc_lo == BC_EXTRAP && a.bc_hi == BC_EXTRAP && row_whole_enabled()) {
            const int groups = ceil_div(a.nrows, 4);
            const int gy = groups < 32768 ? groups : 32768;
            const int gz = ceil_div(groups, gy);
            hipLaunchKernelGGL((k_sweep_row_whole<R, SYS, MEQN, CPL, SPEEDS, LIMK>), dim3(1, gy, gz), dim3(256), 0,
                               s, a);
            return hipGetLastError();
        }
    }
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
