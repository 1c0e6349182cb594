// fused.hip -- one kernel per split step of 2D shallow water: the x sweep and
// the y sweep of equation LW-update fused through LDS (the paper kept them as
// separate kernels, section 5.2, because a unified kernel did not fit Fermi's
// registers and shared memory).
//
// A workgroup owns a strip of W = 62 * CPL columns and a chunk of rows
// [y0, y1), and marches down the chunk four rows at a time.  In iteration t
// each wavefront x-sweeps one row of the sequence y0 - 2, y0 - 1, ..., y1 + 1
// (row y0 - 2 + 4 t + wavefront: the row body's arithmetic, CPL cells per
// lane, DPP neighbour exchange, each interface solved once) and writes that
// row of Q* into one of two four-row LDS buffers; then, after one barrier,
// every lane marches its column of the strip through those four rows of Q*
// with the column body's rolling register window and writes Q^{n+1}.  The
// state is read once and written once per step; only the four halo rows of
// a chunk are x-swept twice.  The next row's loads are issued before the
// current row is computed, so their latency overlaps the sweeps.
//
// Ghost rows of Q* (y boundaries) are the x sweeps of their source rows under
// the y boundary rule, with the normal momentum negated for a wall (the x
// sweep commutes with that sign change), so every y boundary rule runs here.
// The step state is prepared by k_open (decision of the previous trial, fresh
// speed slots) before the fused kernel, which then publishes both
// directions' speed maxima.
#include "claw_launch.h"
#include "sweep_body.h"

namespace claw {

namespace {

constexpr int FR = 4;  // rows per iteration: one x-swept row per wavefront
#ifndef FUSED_WPE
#define FUSED_WPE 4
#endif

// Decides the previous trial (copy p ^ 1), writes the step state this trial
// runs with into copy p (an adaptive run's result buffer planned so that its
// last step ends in buffer 0) and clears copy p's speed slots.
__global__ void k_open(Ctrl* c, int p, int fp32) {
    StepState S;
    decide(c, p ^ 1, fp32 != 0, S);
    S.pending = S.done ? 0 : 1;
    if (S.mode == MODE_ADAPT && !S.done) S.result_off = planned_result_off(S.cur, S.target - S.accepted);
    c->st[p] = S;
    clear_speeds(c, p);
    c->nonphys[p] = 0;
}

template <typename R>
__device__ __forceinline__ void block_finish2(const SweepArgs<R>& a, R vx, R vy, bool bad) {
    __shared__ R red[2][4];
    __shared__ int redbad[4];
    vx = wave_max(vx);
    vy = wave_max(vy);
    const int anybad = __any(bad) ? 1 : 0;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = vx;
        red[1][w] = vy;
        redbad[w] = anybad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        R mx = R(0), my = R(0);
        int b = 0;
        for (int i = 0; i < 4; ++i) {
            mx = rmax(mx, red[0][i]);
            my = rmax(my, red[1][i]);
            b |= redbad[i];
        }
        publish_smax(a.ctrl, a.parity, 0, smax_slot(), mx);
        publish_smax(a.ctrl, a.parity, 1, smax_slot(), my);
        if (b) atomicOr(&a.ctrl->nonphys[a.parity], 1);
    }
}

template <typename R, int CPL, int LIMK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FUSED_WPE)))
void k_step2d(FusedArgs<R> F) {
#define STEP2D_BX blockIdx.x
#define STEP2D_BY blockIdx.y
#include "step2d_body.inc"
#undef STEP2D_BX
#undef STEP2D_BY
}

// Batched 2D steps: workgroup i runs block (x, y) of instance inst of the table.
template <typename R, int CPL, int LIMK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FUSED_WPE)))
void k_batch_step2d(BatchFusedLaunch<R> L) {
    const BatchBlock bb = L.blocks[blockIdx.x];
    FusedArgs<R> F = L.args[bb.inst];
    F.a.parity = L.parity;
#define STEP2D_BX bb.x
#define STEP2D_BY bb.y
#include "step2d_body.inc"
#undef STEP2D_BX
#undef STEP2D_BY
}

// ---------------------------------------------------------------------------
// 3D acoustics: x and y sweeps of one z plane fused
// ---------------------------------------------------------------------------
// Neither the x nor the y sweep couples z planes, so each plane's pair of
// sweeps is a 2D fused step.  The rows are exactly 64 CPL cells with
// extrapolation at both ends, so a wavefront x-sweeps a whole row with no halo
// lanes (the ghost cells equal the end cells: lane 0 takes its own first cell
// as its left neighbour, and the shifted neighbour faces and contributions
// that lanes 0 and 63 receive as zeros are faces without waves), and the four
// wavefronts' lanes are the row's columns in the y march.  Phase A writes p
// and the y velocity of Q*, with Z and c of per-cell coefficients, into the
// LDS rows; the x velocity of Q* and the z velocity go straight to the
// destination (the y sweep leaves both unchanged).  Phase B marches p and v
// down the columns.  Same arithmetic per interface as the x and y sweeps.
// Step control as in the split sweeps: this kernel opens the trial (every
// workgroup decides the previous trial, workgroup (0, 0) records the state)
// and the z sweep closes it (it clears the other parity's speed slots), so a
// trial needs no opening kernel of its own.
template <typename R, int SYS, int CPL, int LIMK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FUSED_WPE)))
void k_step_xy3(Fused3Args<R> F) {
    static_assert(SYS == SYS_AC || SYS == SYS_ACV, "the 3D fused step is for acoustics");
    constexpr int MEQN = 4;
    constexpr int NX = 64 * CPL;                 // cells per row
    constexpr int NL = SYS == SYS_ACV ? 4 : 2;   // LDS fields: p, v (, Z, c)
    constexpr int NC = contrib_width<SYS>();
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    typedef typename VecOf<R, CPL>::type V;
    __shared__ R ring[2][FR][NL][NX];

    const SweepArgs<R>& a = F.a;
    StepState S;
    decide(a.ctrl, a.parity ^ 1, sizeof(R) == 4, S);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        S.pending = S.done ? 0 : 1;
        a.ctrl->st[a.parity] = S;
    }
    if (wave_uniform(S.done)) return;  // the whole grid skips
    const int cur = wave_uniform(S.cur);
    const R nux = wave_uniform(state_nu<R>(S, 0)), nuy = wave_uniform(state_nu<R>(S, 1));
    const R* __restrict__ src = pick_buf(a, cur);
    R* __restrict__ dst = pick_buf(a, (cur + 1) % 3);
    const R inv2Z = ac_inv2Z<R, SYS>(a);

    const int lane = threadIdx.x & 63, wave = wave_uniform((int)(threadIdx.x >> 6));
    const int ny = F.ny;
    const int y0 = blockIdx.x * F.chunk;
    const int y1 = y0 + F.chunk < ny ? y0 + F.chunk : ny;
    const unsigned plane = (unsigned)blockIdx.y * (unsigned)ny * (unsigned)NX;  // first cell of the plane
    const int nt = (y1 - y0 + FR - 1) / FR + 1;  // iterations (the first only fills the window)
    const unsigned fbytes = (unsigned)a.ncell * (unsigned)sizeof(R);
    const unsigned xoff = (unsigned)(lane * CPL);

    // ---- x sweep of one whole row per wavefront (phase A) ------------------
    // loads the lane's cells of virtual row v (a ghost row loads its source row)
    auto row_base = [&](int v, bool& fy) { return plane + (unsigned)(ghost_idx(v, ny, F.bcy_lo, F.bcy_hi, fy) * NX); };
    auto load_row = [&](int v, R (&q)[CPL][MEQN], R (&zc)[CPL][2]) {
        bool fy;
        const unsigned voff = (row_base(v, fy) + xoff) * (unsigned)sizeof(R);
#pragma unroll
        for (int e = 0; e < MEQN; ++e) {
            V vv = buf_load16<V>(field_rsrc(src + (size_t)e * (unsigned)a.ncell, fbytes), voff);
#pragma unroll
            for (int c = 0; c < CPL; ++c) q[c][e] = vv[c];
        }
        if constexpr (SYS == SYS_ACV) {
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                V vv = buf_load16<V>(field_rsrc(a.zc + (size_t)f * (unsigned)a.ncell, fbytes), voff);
#pragma unroll
                for (int c = 0; c < CPL; ++c) zc[c][f] = vv[c];
            }
        }
    };
    R smx = R(0);
    bool bad = false;
    auto sweep_row = [&](int v, R (&q)[CPL][MEQN], const R (&zc)[CPL][2], R (*out)[NX]) {
        constexpr int nrm = 1, tng = 2;
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
        const bool real = v >= y0 && v < y1;  // uniform: a row of this chunk (each row counts once)
        if (real) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) smx = rmax(smx, iface_smax(f[c]));
        }
        I fprev, fnext;
        iface_prev(f[CPL - 1], fprev);  // lane 0: zeros, face -1 without waves
        iface_next(f[0], fnext);        // lane 63: zeros, face nx without waves
        Contrib<R, NC> k[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const I& km = c == 0 ? fprev : f[c - 1];
            const I& kp = c == CPL - 1 ? fnext : f[c + 1];
            limit_contrib(f[c], km, kp, nux, limiter_of<LIMK>(a), k[c]);
        }
        R Lnext[NC];
#pragma unroll
        for (int n = 0; n < NC; ++n) Lnext[n] = lane_next(k[0].L[n]);  // lane 63: face nx contributes 0
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (c < CPL - 1) apply_update<R, SYS, MEQN>(q[c], k[c].Rr, k[c + 1].L, nux, nrm, tng);
            else apply_update<R, SYS, MEQN>(q[c], k[c].Rr, Lnext, nux, nrm, tng);
        }
        // a wall ghost row of Q* is its source row with the y velocity negated
        bool fy;
        const unsigned base = row_base(v, fy);
        V vp, vv;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            vp[c] = q[c][0];
            vv[c] = fy ? -q[c][2] : q[c][2];
        }
        *reinterpret_cast<V*>(&out[0][xoff]) = vp;
        *reinterpret_cast<V*>(&out[1][xoff]) = vv;
        if constexpr (SYS == SYS_ACV) {
            V vz, vc;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                vz[c] = zc[c][0];
                vc[c] = zc[c][1];
            }
            *reinterpret_cast<V*>(&out[2][xoff]) = vz;
            *reinterpret_cast<V*>(&out[3][xoff]) = vc;
        }
        if (real) {  // the x and z velocities of Q** are those of Q*
            const unsigned voff = (base + xoff) * (unsigned)sizeof(R);
#pragma unroll
            for (int e = 1; e < MEQN; e += 2) {
                V vo;
#pragma unroll
                for (int c = 0; c < CPL; ++c) vo[c] = q[c][e];
                buf_store16<V>(field_rsrc(dst + (size_t)e * (unsigned)a.ncell, fbytes), voff, vo);
            }
        }
    };

    // ---- y march of one column per lane (phase B) --------------------------
    // the column's cells carry p and v in a two-field state (normal field 1)
    constexpr int NRM = 1, TNG = 0;
    const int lc = (int)threadIdx.x;
    const bool xin = lc < NX;  // FP64 rows (128 cells) leave wavefronts 2 and 3 idle here
    const int lcc = xin ? lc : 0;
    struct YC {
        R q[2];
        R zc[2];
    };
    auto ld = [&](R (*row)[NX], YC& o) {
        o.q[0] = row[0][lcc];
        o.q[1] = row[1][lcc];
        if constexpr (SYS == SYS_ACV) {
            o.zc[0] = row[2][lcc];
            o.zc[1] = row[3][lcc];
        } else {
            o.zc[0] = R(0);
            o.zc[1] = R(0);
        }
    };
    auto mk = [&](const YC& w, C& c) { make_cell<R, SYS, 2>(w.q, w.zc, NRM, TNG, a.sqrt_grav, bad, c); };
    const Rsrc rp = field_rsrc(dst, fbytes);
    const Rsrc rv = field_rsrc(dst + (size_t)2 * (unsigned)a.ncell, fbytes);
    YC w0, w1;
    C c1;
    I fb, fc;
    R Rb[NC];
    R smy = R(0);

    R qa[CPL][MEQN], qn[CPL][MEQN];
    R za[CPL][2] = {}, zn[CPL][2] = {};
    load_row(y0 - 2 + wave, qa, za);
    for (int t = 0; t < nt; ++t) {
        const int v = y0 - 2 + FR * t + wave;
        if (t + 1 < nt) load_row(v + FR, qn, zn);  // the next row's loads overlap this iteration
        R (*slot)[NL][NX] = ring[t & 1];
        if (v <= y1 + 1) sweep_row(v, qa, za, slot[wave]);
        __syncthreads();
        if (t == 0) {
            // window of rows y0 - 2 .. y0 + 1
            YC wm2, wm1;
            C cm2, cm1, c0;
            ld(slot[0], wm2);
            ld(slot[1], wm1);
            ld(slot[2], w0);
            ld(slot[3], w1);
            mk(wm2, cm2);
            mk(wm1, cm1);
            mk(w0, c0);
            mk(w1, c1);
            I fa;
            solve_iface<R, SYS, 1>(cm2, cm1, a, inv2Z, fa);
            solve_iface<R, SYS, 1>(cm1, c0, a, inv2Z, fb);
            solve_iface<R, SYS, 1>(c0, c1, a, inv2Z, fc);
            if (y0 == 0) smy = iface_smax(fb);
            Contrib<R, NC> kb;
            limit_contrib(fb, fa, fc, nuy, limiter_of<LIMK>(a), kb);
#pragma unroll
            for (int i = 0; i < NC; ++i) Rb[i] = kb.Rr[i];
        } else {
            // rows past the chunk (only in the last iteration) march on a copy of
            // the last row this iteration swept (row y1 + 1) and are neither
            // stored nor counted
            const int klast = y1 + 1 - (y0 - 2 + FR * t);  // uniform
#pragma unroll
            for (int k = 0; k < FR; ++k) {
                const int yy = y0 + FR * (t - 1) + k;
                const bool live = yy < y1;  // uniform
                YC w2;
                ld(slot[live ? k : klast], w2);  // row yy + 2
                C c2;
                mk(w2, c2);
                I fd;
                solve_iface<R, SYS, 1>(c1, c2, a, inv2Z, fd);
                smy = live ? rmax(smy, iface_smax(fc)) : smy;
                Contrib<R, NC> kc;
                limit_contrib(fc, fb, fd, nuy, limiter_of<LIMK>(a), kc);
                apply_update<R, SYS, 2>(w0.q, Rb, kc.L, nuy, NRM, TNG);
                if (xin && live) {
                    const unsigned off = (plane + (unsigned)(yy * NX + lc)) * (unsigned)sizeof(R);
                    buf_store(rp, off, 0u, w0.q[0]);
                    buf_store(rv, off, 0u, w0.q[1]);
                }
#pragma unroll
                for (int i = 0; i < NC; ++i) Rb[i] = kc.Rr[i];
                fb = fc;
                fc = fd;
                w0 = w1;
                w1 = w2;
                c1 = c2;
            }
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
#pragma unroll
            for (int e = 0; e < MEQN; ++e) qa[c][e] = qn[c][e];
#pragma unroll
            for (int f = 0; f < 2; ++f) za[c][f] = zn[c][f];
        }
    }
    if (!xin) smy = R(0);
    block_finish2(a, smx, smy, bad);
}

}  // namespace

int fused_rows_per_iteration() { return FR; }

hipError_t launch_open(Ctrl* c, int p, bool fp32, hipStream_t s) {
    hipLaunchKernelGGL(k_open, dim3(1), dim3(1), 0, s, c, p, fp32 ? 1 : 0);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_step2d(const FusedArgs<R>& F, hipStream_t s) {
    constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
    const int W = 62 * CPL;
    if (F.chunk < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((F.a.nx + W - 1) / W), (unsigned)((F.ny + F.chunk - 1) / F.chunk));
    if (F.a.limiter == LIM_MC) hipLaunchKernelGGL((k_step2d<R, CPL, LIM_MC>), grid, dim3(256), 0, s, F);
    else hipLaunchKernelGGL((k_step2d<R, CPL, LIM_RUNTIME>), grid, dim3(256), 0, s, F);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_step_xy3(const Fused3Args<R>& F, int sys, hipStream_t s) {
    constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
    if (F.chunk < 1 || F.a.nx != 64 * CPL || F.nz < 1 || F.nz > 65535 || (sys != SYS_AC && sys != SYS_ACV))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((F.ny + F.chunk - 1) / F.chunk), (unsigned)F.nz);
    const bool mc = F.a.limiter == LIM_MC;
    if (sys == SYS_ACV) {
        if (mc) hipLaunchKernelGGL((k_step_xy3<R, SYS_ACV, CPL, LIM_MC>), grid, dim3(256), 0, s, F);
        else hipLaunchKernelGGL((k_step_xy3<R, SYS_ACV, CPL, LIM_RUNTIME>), grid, dim3(256), 0, s, F);
    } else {
        if (mc) hipLaunchKernelGGL((k_step_xy3<R, SYS_AC, CPL, LIM_MC>), grid, dim3(256), 0, s, F);
        else hipLaunchKernelGGL((k_step_xy3<R, SYS_AC, CPL, LIM_RUNTIME>), grid, dim3(256), 0, s, F);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_step2d(const BatchFusedLaunch<R>& L, int nblocks, hipStream_t s) {
    constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
    if (nblocks < 1) return hipErrorInvalidValue;
    if (L.limiter == LIM_MC) hipLaunchKernelGGL((k_batch_step2d<R, CPL, LIM_MC>), dim3(nblocks), dim3(256), 0, s, L);
    else hipLaunchKernelGGL((k_batch_step2d<R, CPL, LIM_RUNTIME>), dim3(nblocks), dim3(256), 0, s, L);
    return hipGetLastError();
}

template hipError_t launch_step2d<float>(const FusedArgs<float>&, hipStream_t);
template hipError_t launch_step2d<double>(const FusedArgs<double>&, hipStream_t);
template hipError_t launch_step_xy3<float>(const Fused3Args<float>&, int, hipStream_t);
template hipError_t launch_batch_step2d<float>(const BatchFusedLaunch<float>&, int, hipStream_t);
template hipError_t launch_batch_step2d<double>(const BatchFusedLaunch<double>&, int, hipStream_t);
template hipError_t launch_step_xy3<double>(const Fused3Args<double>&, int, hipStream_t);

}  // namespace claw
