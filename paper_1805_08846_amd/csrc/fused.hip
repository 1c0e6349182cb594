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
// runs with into copy p and clears copy p's speed slots.
__global__ void k_open(Ctrl* c, int p, int fp32) {
    StepState S;
    decide(c, p ^ 1, fp32 != 0, S);
    S.pending = S.done ? 0 : 1;
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
    constexpr int SYS = SYS_SW;
    constexpr int MEQN = 3;
    constexpr int W = 62 * CPL;
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    using CC = ColCell<R, SYS, MEQN>;
    typedef typename VecOf<R, CPL>::type V;
    __shared__ R ring[2][FR][MEQN][W];

    const SweepArgs<R>& a = F.a;
    const StepState& S = a.ctrl->st[a.parity];
    if (S.done) return;  // the whole grid skips
    const int cur = wave_uniform(S.cur);
    const R nux = wave_uniform(state_nu<R>(S, 0)), nuy = wave_uniform(state_nu<R>(S, 1));
    const R* __restrict__ src = pick_buf(a, cur);
    R* __restrict__ dst = pick_buf(a, (cur + 1) % 3);

    const int lane = threadIdx.x & 63, wave = wave_uniform((int)(threadIdx.x >> 6));
    const int nx = a.nx, ny = F.ny;
    const int x0 = blockIdx.x * W;
    const int y0 = blockIdx.y * F.chunk;
    const int y1 = y0 + F.chunk < ny ? y0 + F.chunk : ny;
    const int nt = (y1 - y0 + FR - 1) / FR + 1;  // iterations (the first only fills the window)
    const unsigned fbytes = (unsigned)a.ncell * (unsigned)sizeof(R);
    bool bad = false;

    // ---- x sweep of one row per wavefront (phase A) ------------------------
    constexpr int nrm = 1, tng = 2;
    const int xl = x0 - CPL + lane * CPL;
    const bool interior = (nx % CPL) == 0 && (a.ncell % CPL) == 0 && xl >= 0 && xl + CPL <= nx;
    const bool useful = lane >= 1 && lane <= 62;
    // loads the lane's cells of virtual row v (a ghost row loads its source row)
    auto load_row = [&](int v, R (&q)[CPL][MEQN]) {
        bool fy;
        const unsigned base = (unsigned)(ghost_idx(v, ny, F.bcy_lo, F.bcy_hi, fy) * nx);
        if (interior) {
            const unsigned voff = (base + (unsigned)xl) * (unsigned)sizeof(R);
#pragma unroll
            for (int e = 0; e < MEQN; ++e) {
                V vv = buf_load16<V>(field_rsrc(src + (size_t)e * (unsigned)a.ncell, fbytes), voff);
#pragma unroll
                for (int c = 0; c < CPL; ++c) q[c][e] = vv[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                bool flip;
                const unsigned sidx = base + (unsigned)ghost_idx(xl + c, nx, a.bc_lo, a.bc_hi, flip);
                CLAW_CHECK(sidx < (unsigned)a.ncell);
#pragma unroll
                for (int e = 0; e < MEQN; ++e) q[c][e] = src[(size_t)e * (unsigned)a.ncell + sidx];
                if (flip) q[c][nrm] = -q[c][nrm];
            }
        }
    };
    R smx = R(0);
    auto sweep_row = [&](int v, R (&q)[CPL][MEQN], R (*out)[W]) {
        C cell[CPL];
        const R zc0[2] = {R(0), R(0)};
#pragma unroll
        for (int c = 0; c < CPL; ++c) make_cell<R, SYS, MEQN>(q[c], zc0, nrm, tng, a.sqrt_grav, bad, cell[c]);
        C left;
        cell_prev(cell[CPL - 1], left);
        I f[CPL];
        riemann(left, cell[0], a.Z0, a.c0, R(0), a.grav, a.efix, f[0]);
#pragma unroll
        for (int c = 1; c < CPL; ++c) riemann(cell[c - 1], cell[c], a.Z0, a.c0, R(0), a.grav, a.efix, f[c]);
        if (interior) {
            R m = iface_smax(f[0]);
#pragma unroll
            for (int c = 1; c < CPL; ++c) m = rmax(m, iface_smax(f[c]));
            if (useful) smx = rmax(smx, m);
        } else {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int j = xl + c;
                const bool own = (useful && j >= 0 && j <= nx) || (lane == 63 && c == 0 && j == nx);
                if (own) smx = rmax(smx, iface_smax(f[c]));
            }
        }
        I fprev, fnext;
        iface_prev(f[CPL - 1], fprev);
        iface_next(f[0], fnext);
        Contrib<R> k[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const I& km = c == 0 ? fprev : f[c - 1];
            const I& kp = c == CPL - 1 ? fnext : f[c + 1];
            limit_contrib(f[c], km, kp, nux, limiter_of<LIMK>(a), k[c]);
        }
        R Lnext[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) Lnext[i] = lane_next(k[0].L[i]);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (c < CPL - 1) apply_update<R, SYS, MEQN>(q[c], k[c].Rr, k[c + 1].L, nux, nrm, tng);
            else apply_update<R, SYS, MEQN>(q[c], k[c].Rr, Lnext, nux, nrm, tng);
        }
        // a wall ghost row of Q* is its source row with the y momentum negated
        bool fy;
        (void)ghost_idx(v, ny, F.bcy_lo, F.bcy_hi, fy);
        if (useful) {
            const int col = (lane - 1) * CPL;  // = xl - x0
            if (xl + CPL <= nx) {
#pragma unroll
                for (int e = 0; e < MEQN; ++e) {
                    V vv;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) vv[c] = (fy && e == 2) ? -q[c][e] : q[c][e];
                    *reinterpret_cast<V*>(&out[e][col]) = vv;
                }
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (xl + c < nx) {
#pragma unroll
                        for (int e = 0; e < MEQN; ++e) out[e][col + c] = (fy && e == 2) ? -q[c][e] : q[c][e];
                    }
            }
        }
    };

    // ---- y march of one column per lane (phase B) --------------------------
    constexpr int NRM = 2, TNG = 1;
    const int lc = wave * 62 + lane;  // FP64 strips (W = 124) leave wavefronts 2 and 3 idle here
    const int x = x0 + lc;
    const bool xin = lane < 62 && lc < W && x < nx;
    const int lcc = xin ? lc : 0;  // column 0 of the strip always holds data
    const R zc0[2] = {R(0), R(0)};
    auto ld = [&](R (*row)[W], CC& o) {
#pragma unroll
        for (int e = 0; e < MEQN; ++e) o.q[e] = row[e][lcc];
    };
    CC w0, w1;
    C c1;
    I fb, fc;
    R Rb[3];
    R smy = R(0);

    R qa[CPL][MEQN], qn[CPL][MEQN];
    load_row(y0 - 2 + wave, qa);
    for (int t = 0; t < nt; ++t) {
        const int v = y0 - 2 + FR * t + wave;
        if (t + 1 < nt) load_row(v + FR, qn);  // the next row's loads overlap this iteration
        R (*slot)[MEQN][W] = ring[t & 1];
        if (v <= y1 + 1) sweep_row(v, qa, slot[wave]);
        __syncthreads();
        if (t == 0) {
            // window of rows y0 - 2 .. y0 + 1
            CC wm2, wm1;
            C cm2, cm1, c0;
            ld(slot[0], wm2);
            ld(slot[1], wm1);
            ld(slot[2], w0);
            ld(slot[3], w1);
            make_cell<R, SYS, MEQN>(wm2.q, zc0, NRM, TNG, a.sqrt_grav, bad, cm2);
            make_cell<R, SYS, MEQN>(wm1.q, zc0, NRM, TNG, a.sqrt_grav, bad, cm1);
            make_cell<R, SYS, MEQN>(w0.q, zc0, NRM, TNG, a.sqrt_grav, bad, c0);
            make_cell<R, SYS, MEQN>(w1.q, zc0, NRM, TNG, a.sqrt_grav, bad, c1);
            I fa;
            riemann(cm2, cm1, a.Z0, a.c0, R(0), a.grav, a.efix, fa);
            riemann(cm1, c0, a.Z0, a.c0, R(0), a.grav, a.efix, fb);
            riemann(c0, c1, a.Z0, a.c0, R(0), a.grav, a.efix, fc);
            if (y0 == 0) smy = iface_smax(fb);
            Contrib<R> kb;
            limit_contrib(fb, fa, fc, nuy, limiter_of<LIMK>(a), kb);
#pragma unroll
            for (int i = 0; i < 3; ++i) Rb[i] = kb.Rr[i];
        } else {
            // rows past the chunk (only in the last iteration) march on a copy of
            // the last row this iteration swept (row y1 + 1) and are neither
            // stored nor counted: a march with no early exit keeps the window in
            // the same registers step to step
            const int klast = y1 + 1 - (y0 - 2 + FR * t);  // uniform
#pragma unroll
            for (int k = 0; k < FR; ++k) {
                const int yy = y0 + FR * (t - 1) + k;
                const bool live = yy < y1;  // uniform
                CC w2;
                ld(slot[live ? k : klast], w2);  // row yy + 2
                C c2;
                bool rb = false;
                make_cell<R, SYS, MEQN>(w2.q, zc0, NRM, TNG, a.sqrt_grav, rb, c2);
                bad = bad || (live && rb);
                I fd;
                riemann(c1, c2, a.Z0, a.c0, R(0), a.grav, a.efix, fd);
                smy = live ? rmax(smy, iface_smax(fc)) : smy;
                Contrib<R> kc;
                limit_contrib(fc, fb, fd, nuy, limiter_of<LIMK>(a), kc);
                apply_update<R, SYS, MEQN>(w0.q, Rb, kc.L, nuy, NRM, TNG);
                if (xin && live) {
                    const unsigned off = (unsigned)(yy * nx + x);
                    CLAW_CHECK(off < (unsigned)a.ncell);
#pragma unroll
                    for (int e = 0; e < MEQN; ++e) dst[(size_t)e * (unsigned)a.ncell + off] = w0.q[e];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) Rb[i] = kc.Rr[i];
                fb = fc;
                fc = fd;
                w0 = w1;
                w1 = w2;
                c1 = c2;
            }
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int e = 0; e < MEQN; ++e) qa[c][e] = qn[c][e];
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

template hipError_t launch_step2d<float>(const FusedArgs<float>&, hipStream_t);
template hipError_t launch_step2d<double>(const FusedArgs<double>&, hipStream_t);

}  // namespace claw
