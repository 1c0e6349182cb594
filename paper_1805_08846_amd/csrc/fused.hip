// fused.hip -- one kernel per split step of 2D shallow water: the x sweep and
// the y sweep of equation LW-update fused through LDS (the paper kept them as
// separate kernels, section 5.2, because a unified kernel did not fit Fermi's
// registers and shared memory).
//
// A workgroup owns a tile of W = 62 * CPL columns and TY rows.  Phase A runs
// the x sweep (the row body's arithmetic: CPL cells per lane, DPP neighbour
// exchange, each interface solved once) over the tile's rows plus two rows
// above and below, and keeps Q* in LDS.  Phase B marches the tile's columns
// along y through Q* in LDS and writes Q^{n+1}.  The state is read once and
// written once per step; the halo rows are swept twice (by this tile and by
// its neighbour), (TY + 4) / TY of the x-sweep work.
//
// Ghost rows of Q* (y boundaries) are mirrored or copied from the tile, so
// reflecting and extrapolation boundaries in y are supported here; periodic y
// takes the two-kernel path.  The step state is prepared by k_open (decision
// of the previous trial, fresh speed slots) before the fused kernel, which then
// publishes both directions' speed maxima.
#include "claw_launch.h"
#include "sweep_body.h"

namespace claw {

namespace {

constexpr int TY = 8;           // rows a workgroup updates
constexpr int ROWS = TY + 4;    // rows swept in x (two halo rows each side)
constexpr int RPW = ROWS / 4;   // x-swept rows per wavefront
static_assert(ROWS % 4 == 0, "rows split evenly over the four wavefronts");

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

template <typename R, int CPL>
__global__ __launch_bounds__(256) void k_step2d(FusedArgs<R> F) {
    constexpr int SYS = SYS_SW;
    constexpr int MEQN = 3;
    constexpr int W = 62 * CPL;
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    using CC = ColCell<R, SYS, MEQN>;
    typedef typename VecOf<R, CPL>::type V;
    __shared__ R tile[ROWS][MEQN][W];

    const SweepArgs<R>& a = F.a;
    const StepState& S = a.ctrl->st[a.parity];
    if (S.done) return;  // the whole grid skips
    const R nux = state_nu<R>(S, 0), nuy = state_nu<R>(S, 1);
    const R* __restrict__ src = pick_buf(a, S.cur);
    R* __restrict__ dst = pick_buf(a, (S.cur + 1) % 3);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nx = a.nx, ny = F.ny;
    const int x0 = blockIdx.x * W;
    const int y0 = blockIdx.y * TY;
    const int ylo = y0 - 2 > 0 ? y0 - 2 : 0;
    const int yhi = y0 + TY + 2 < ny ? y0 + TY + 2 : ny;
    bool bad = false;

    // ---- phase A: x sweep of rows [ylo, yhi) into the tile -------------------
    R smx = R(0);
    {
        constexpr int nrm = 1, tng = 2;
        const int xl = x0 - CPL + lane * CPL;
        const bool interior = (nx % CPL) == 0 && xl >= 0 && xl + CPL <= nx;
        // all of this wavefront's rows are loaded first, so their latencies overlap
        R qa[RPW][CPL][MEQN];
#pragma unroll
        for (int rk = 0; rk < RPW; ++rk) {
            const int r = ylo + wave + 4 * rk;
            const unsigned base = (unsigned)((r < yhi ? r : ylo) * nx);
            if (interior) {
#pragma unroll
                for (int e = 0; e < MEQN; ++e) {
                    V v = *reinterpret_cast<const V*>(src + (size_t)e * a.ncell + base + (unsigned)xl);
#pragma unroll
                    for (int c = 0; c < CPL; ++c) qa[rk][c][e] = v[c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    bool flip;
                    const unsigned sidx = base + (unsigned)ghost_idx(xl + c, nx, a.bc_lo, a.bc_hi, flip);
#pragma unroll
                    for (int e = 0; e < MEQN; ++e) qa[rk][c][e] = src[(size_t)e * a.ncell + sidx];
                    if (flip) qa[rk][c][nrm] = -qa[rk][c][nrm];
                }
            }
        }
#pragma unroll
        for (int rk = 0; rk < RPW; ++rk) {
            const int r = ylo + wave + 4 * rk;
            if (r >= yhi) break;  // uniform across the wavefront
            R (&q)[CPL][MEQN] = qa[rk];
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
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int j = xl + c;
                const bool own = (lane >= 1 && lane <= 62 && j >= 0 && j <= nx) || (lane == 63 && c == 0 && j == nx);
                if (own) smx = rmax(smx, iface_smax(f[c]));
            }
            I fprev, fnext;
            iface_prev(f[CPL - 1], fprev);
            iface_next(f[0], fnext);
            Contrib<R> k[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const I& km = c == 0 ? fprev : f[c - 1];
                const I& kp = c == CPL - 1 ? fnext : f[c + 1];
                limit_contrib(f[c], km, kp, nux, a.limiter, k[c]);
            }
            R Lnext[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) Lnext[i] = lane_next(k[0].L[i]);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                if (c < CPL - 1) apply_update<R, SYS, MEQN>(q[c], k[c].Rr, k[c + 1].L, nux, nrm, tng);
                else apply_update<R, SYS, MEQN>(q[c], k[c].Rr, Lnext, nux, nrm, tng);
            }
            if (lane >= 1 && lane <= 62) {
                const int col = (lane - 1) * CPL;  // = xl - x0
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (xl + c < nx) {
#pragma unroll
                        for (int e = 0; e < MEQN; ++e) tile[r - ylo][e][col + c] = q[c][e];
                    }
            }
        }
    }
    __syncthreads();

    // ---- phase B: y sweep of the tile's columns from Q* in LDS ----------------
    R smy = R(0);
    {
        constexpr int NRM = 2, TNG = 1;
        const int lc = wave * 62 + lane;  // FP64 tiles (W = 124) leave waves 2 and 3 idle here
        const int x = x0 + lc;
        const bool xin = lane < 62 && lc < W && x < nx;
        const int lcc = xin ? lc : 0;  // column 0 of the tile always holds data
        const int y1 = y0 + TY < ny ? y0 + TY : ny;
        const R zc0[2] = {R(0), R(0)};
        auto load = [&](int j, CC& out) {
            bool flip;
            const int rr = ghost_idx(j, ny, F.bcy_lo, F.bcy_hi, flip) - ylo;
#pragma unroll
            for (int e = 0; e < MEQN; ++e) out.q[e] = tile[rr][e][lcc];
            if (flip) out.q[NRM] = -out.q[NRM];
        };
        CC w0, w1;
        C c1;
        I fb, fc;
        R Rb[3];
        {
            CC wm2, wm1;
            C cm2, cm1, c0;
            load(y0 - 2, wm2);
            load(y0 - 1, wm1);
            load(y0, w0);
            load(y0 + 1, w1);
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
            limit_contrib(fb, fa, fc, nuy, a.limiter, kb);
#pragma unroll
            for (int i = 0; i < 3; ++i) Rb[i] = kb.Rr[i];
        }
        for (int yy = y0; yy < y1; ++yy) {
            CC w2;
            load(yy + 2, w2);
            C c2;
            make_cell<R, SYS, MEQN>(w2.q, zc0, NRM, TNG, a.sqrt_grav, bad, c2);
            I fd;
            riemann(c1, c2, a.Z0, a.c0, R(0), a.grav, a.efix, fd);
            smy = rmax(smy, iface_smax(fc));
            Contrib<R> kc;
            limit_contrib(fc, fb, fd, nuy, a.limiter, kc);
            apply_update<R, SYS, MEQN>(w0.q, Rb, kc.L, nuy, NRM, TNG);
            if (xin) {
                const unsigned off = (unsigned)(yy * nx + x);
#pragma unroll
                for (int e = 0; e < MEQN; ++e) dst[(size_t)e * a.ncell + off] = w0.q[e];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) Rb[i] = kc.Rr[i];
            fb = fc;
            fc = fd;
            w0 = w1;
            w1 = w2;
            c1 = c2;
        }
        if (!xin) smy = R(0);
    }
    block_finish2(a, smx, smy, bad);
}

}  // namespace

int fused_tile_rows() { return TY; }

hipError_t launch_open(Ctrl* c, int p, bool fp32, hipStream_t s) {
    hipLaunchKernelGGL(k_open, dim3(1), dim3(1), 0, s, c, p, fp32 ? 1 : 0);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_step2d(const FusedArgs<R>& F, hipStream_t s) {
    constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
    const int W = 62 * CPL;
    const dim3 grid((unsigned)((F.a.nx + W - 1) / W), (unsigned)((F.ny + TY - 1) / TY));
    hipLaunchKernelGGL((k_step2d<R, CPL>), grid, dim3(256), 0, s, F);
    return hipGetLastError();
}

template hipError_t launch_step2d<float>(const FusedArgs<float>&, hipStream_t);
template hipError_t launch_step2d<double>(const FusedArgs<double>&, hipStream_t);

}  // namespace claw
