// sweeps.hip -- the directional sweep kernels of the split wave-propagation
// step (equation LW-update): Riemann solve at every interface, wave limiter,
// correction flux, single-stage cell update and the fused wave-speed maximum.
//
// Row kernel (x sweep, the contiguous direction).  A wavefront owns a row
// segment: every lane holds CPL consecutive cells loaded with one 16-byte
// vector load per field, solves the CPL interfaces at the left faces of its
// cells and exchanges the missing neighbours (left cell, neighbouring waves,
// the next lane's left-cell contribution) with the adjacent lanes, so each
// interface is solved once.  The first and last lane of a wave only supply
// halo interfaces; neighbouring waves overlap by 2 * CPL cells.
//
// Column kernel (y and z sweeps).  A wavefront owns 64 adjacent columns (one
// per lane, coalesced rows) and marches along the sweep direction over a
// chunk of rows with a rolling register window, so each interface is solved
// once per chunk; rows are prefetched PF rows ahead.
//
// Ghost cells are never stored: a cell index outside the grid is mapped to its
// source cell by the boundary rule (section 4.1) when it is loaded.
#include "claw_device.h"
#include "claw_launch.h"

namespace claw {

template <typename R, int CPL>
struct VecOf {
    typedef R type __attribute__((ext_vector_type(CPL)));
};

// Loads the MEQN fields (plus derived coefficients for SYS_ACV) of the cells
// xl .. xl+CPL-1 of a row into q / zc with ghost mapping at the row ends.
template <typename R, int SYS, int MEQN, int CPL>
__device__ __forceinline__ void row_load(const R* __restrict__ src, const R* __restrict__ zcg,
                                         int64_t ncell, int64_t base, int64_t xl, int64_t nx,
                                         int bc_lo, int bc_hi, bool vec_ok, R (&q)[CPL][MEQN],
                                         R (&zc)[CPL][2]) {
    if (vec_ok && xl >= 0 && xl + CPL <= nx) {
        typedef typename VecOf<R, CPL>::type V;
#pragma unroll
        for (int e = 0; e < MEQN; ++e) {
            V v = *reinterpret_cast<const V*>(src + e * ncell + base + xl);
#pragma unroll
            for (int c = 0; c < CPL; ++c) q[c][e] = v[c];
        }
        if constexpr (SYS == SYS_ACV) {
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                V v = *reinterpret_cast<const V*>(zcg + f * ncell + base + xl);
#pragma unroll
                for (int c = 0; c < CPL; ++c) zc[c][f] = v[c];
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            bool flip;
            int64_t s = ghost_src(xl + c, nx, bc_lo, bc_hi, flip);
#pragma unroll
            for (int e = 0; e < MEQN; ++e) q[c][e] = src[e * ncell + base + s];
            if (flip) q[c][1] = -q[c][1];
            if constexpr (SYS == SYS_ACV) {
                zc[c][0] = zcg[base + s];
                zc[c][1] = zcg[ncell + base + s];
            }
        }
    }
}

template <typename R, int SYS, int MEQN>
__device__ __forceinline__ void make_cell(const R (&q)[MEQN], const R (&zc)[2], int nrm, int tng,
                                          R g, bool& bad, Cell<R, SYS>& c) {
    if constexpr (SYS == SYS_SW) {
        c.h = q[0];
        c.mn = q[nrm];
        c.mt = q[tng];
        c.derive(g, bad);
    } else if constexpr (SYS == SYS_ACV) {
        c.p = q[0];
        c.un = q[nrm];
        c.Z = zc[0];
        c.c = zc[1];
    } else {
        c.p = q[0];
        c.un = q[nrm];
    }
}

template <typename R, int SYS>
__device__ __forceinline__ void cell_prev(const Cell<R, SYS>& in, Cell<R, SYS>& out) {
    if constexpr (SYS == SYS_SW) {
        out.h = lane_prev(in.h);
        out.mn = lane_prev(in.mn);
        out.mt = lane_prev(in.mt);
        out.u = lane_prev(in.u);
        out.v = lane_prev(in.v);
        out.sqh = lane_prev(in.sqh);
        out.c = lane_prev(in.c);
    } else if constexpr (SYS == SYS_ACV) {
        out.p = lane_prev(in.p);
        out.un = lane_prev(in.un);
        out.Z = lane_prev(in.Z);
        out.c = lane_prev(in.c);
    } else {
        out.p = lane_prev(in.p);
        out.un = lane_prev(in.un);
    }
}

// Applies the two contributions to a cell's fields (normal frame -> fields).
template <typename R, int SYS, int MEQN>
__device__ __forceinline__ void apply_update(R (&q)[MEQN], const R (&Rl)[3], const R (&Lr)[3],
                                             R nu, int nrm, int tng) {
    if constexpr (SYS == SYS_SW) {
        q[0] = q[0] - nu * (Rl[0] + Lr[0]);
        q[nrm] = q[nrm] - nu * (Rl[1] + Lr[1]);
        q[tng] = q[tng] - nu * (Rl[2] + Lr[2]);
    } else {
        q[0] = q[0] - nu * (Rl[0] + Lr[0]);
        q[nrm] = q[nrm] - nu * (Rl[1] + Lr[1]);
    }
}

// ---------------------------------------------------------------------------
// Row kernel: x sweep
// ---------------------------------------------------------------------------
template <typename R, int SYS, int MEQN, int CPL, bool SPEEDS>
__global__ __launch_bounds__(256) void k_sweep_row(SweepArgs<R> a) {
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    Ctrl* ctrl = a.ctrl;
    if (ctrl->done) return;
    const int cur = ctrl->cur;
    const R* __restrict__ src = a.buf[(cur + a.src_off) % 3];
    R* __restrict__ dst = a.buf[(cur + a.dst_off) % 3];
    const R nu = ctrl_nu<R>(ctrl, 0);
    const int lane = threadIdx.x & 63;
    const int64_t P = 62 * CPL;
    const int64_t nx = a.nx;
    const int64_t segs = (nx + P - 1) / P;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const bool active = gw < a.nrows * segs;
    const int64_t row = active ? gw / segs : 0;
    const int64_t seg = active ? gw % segs : 0;
    const int64_t x0 = seg * P;
    const int64_t xl = x0 - CPL + (int64_t)lane * CPL;
    const int64_t base = row * nx;
    const bool vec_ok = (nx % CPL) == 0 && (a.ncell % CPL) == 0;
    constexpr int nrm = 1, tng = 2;

    R q[CPL][MEQN];
    R zc[CPL][2];
    row_load<R, SYS, MEQN, CPL>(src, a.zc, a.ncell, base, xl, nx, a.bc_lo, a.bc_hi, vec_ok, q, zc);

    bool bad = false;
    C cell[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) make_cell<R, SYS, MEQN>(q[c], zc[c], nrm, tng, a.grav, bad, cell[c]);
    if (!active) bad = false;

    // interfaces at the left face of each cell of this lane
    C left;
    cell_prev(cell[CPL - 1], left);
    I f[CPL];
    riemann(left, cell[0], a.Z0, a.c0, a.grav, a.efix, f[0]);
#pragma unroll
    for (int c = 1; c < CPL; ++c) riemann(cell[c - 1], cell[c], a.Z0, a.c0, a.grav, a.efix, f[c]);

    // largest speed over the interfaces j = x, 0 <= j <= nx, owned by lanes 1..62
    R sm = R(0);
    if (active) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int64_t j = xl + c;
            const bool own = (lane >= 1 && lane <= 62 && j >= 0 && j <= nx) ||
                             (lane == 63 && c == 0 && j == nx);
            if (own) sm = rmax(sm, iface_smax(f[c]));
        }
    }

    if constexpr (!SPEEDS) {
        I fprev, fnext;
        iface_prev(f[CPL - 1], fprev);
        iface_next(f[0], fnext);
        Contrib<R> k[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const I& km = c == 0 ? fprev : f[c - 1];
            const I& kp = c == CPL - 1 ? fnext : f[c + 1];
            limit_contrib(f[c], km, kp, nu, a.limiter, k[c]);
        }
        R Lnext[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) Lnext[i] = lane_next(k[0].L[i]);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (c < CPL - 1) apply_update<R, SYS, MEQN>(q[c], k[c].Rr, k[c + 1].L, nu, nrm, tng);
            else apply_update<R, SYS, MEQN>(q[c], k[c].Rr, Lnext, nu, nrm, tng);
        }
        if (active && lane >= 1 && lane <= 62) {
            if (vec_ok && xl + CPL <= nx) {
                typedef typename VecOf<R, CPL>::type V;
#pragma unroll
                for (int e = 0; e < MEQN; ++e) {
                    V v;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) v[c] = q[c][e];
                    *reinterpret_cast<V*>(dst + e * a.ncell + base + xl) = v;
                }
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    if (xl + c < nx) {
#pragma unroll
                        for (int e = 0; e < MEQN; ++e) dst[e * a.ncell + base + xl + c] = q[c][e];
                    }
                }
            }
        }
    }
    block_publish_smax(ctrl, 0, sm, bad);
}

// ---------------------------------------------------------------------------
// Column kernel: y and z sweeps
// ---------------------------------------------------------------------------
template <typename R, int SYS, int MEQN>
struct ColCell {
    R q[MEQN];
    R zc[2];
};

template <typename R, int SYS, int MEQN, int NRM>
__device__ __forceinline__ void col_load(const R* __restrict__ src, const R* __restrict__ zcg,
                                         int64_t ncell, int64_t colbase, int64_t y, int64_t m,
                                         int64_t stride, int bc_lo, int bc_hi,
                                         ColCell<R, SYS, MEQN>& out) {
    bool flip;
    const int64_t s = ghost_src(y, m, bc_lo, bc_hi, flip);
    const int64_t off = colbase + s * stride;
#pragma unroll
    for (int e = 0; e < MEQN; ++e) out.q[e] = src[e * ncell + off];
    if (flip) out.q[NRM] = -out.q[NRM];
    if constexpr (SYS == SYS_ACV) {
        out.zc[0] = zcg[off];
        out.zc[1] = zcg[ncell + off];
    }
}

template <typename R, int SYS, int MEQN, int NRM, int PF, bool SPEEDS>
__global__ __launch_bounds__(256) void k_sweep_col(SweepArgs<R> a) {
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    using CC = ColCell<R, SYS, MEQN>;
    constexpr int TNG = SYS == SYS_SW ? 3 - NRM : 0;
    Ctrl* ctrl = a.ctrl;
    if (ctrl->done) return;
    const int cur = ctrl->cur;
    const R* __restrict__ src = a.buf[(cur + a.src_off) % 3];
    R* __restrict__ dst = a.buf[(cur + a.dst_off) % 3];
    const int dir = a.dir;
    const R nu = ctrl_nu<R>(ctrl, dir);
    const int lane = threadIdx.x & 63;
    const int64_t nx = a.nx, m = a.m, chunk = a.chunk;
    const int64_t nstrip = (nx + 63) / 64;
    const int64_t nchunk = (m + chunk - 1) / chunk;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const bool active = gw < nstrip * nchunk * a.nlines_o;
    const int64_t strip = active ? gw % nstrip : 0;
    const int64_t t = active ? gw / nstrip : 0;
    const int64_t ck = t % nchunk;
    const int64_t o = t / nchunk;
    const int64_t x = strip * 64 + lane;
    const bool xin = active && x < nx;
    const int64_t colbase = o * a.ostride + (x < nx ? x : nx - 1);
    const int64_t y0 = ck * chunk;
    const int64_t y1 = active ? (y0 + chunk < m ? y0 + chunk : m) : y0;

    bool bad = false;
    R sm = R(0);
    CC w0, w1;  // cells y and y+1 of the window
    C c0, c1;
    I fb, fc;   // interfaces j = y and j = y + 1
    R Rb[3];    // right-cell contribution of interface j = y
    {
        CC wm2, wm1;
        C cm2, cm1;
        col_load<R, SYS, MEQN, NRM>(src, a.zc, a.ncell, colbase, y0 - 2, m, a.stride, a.bc_lo, a.bc_hi, wm2);
        col_load<R, SYS, MEQN, NRM>(src, a.zc, a.ncell, colbase, y0 - 1, m, a.stride, a.bc_lo, a.bc_hi, wm1);
        col_load<R, SYS, MEQN, NRM>(src, a.zc, a.ncell, colbase, y0, m, a.stride, a.bc_lo, a.bc_hi, w0);
        col_load<R, SYS, MEQN, NRM>(src, a.zc, a.ncell, colbase, y0 + 1, m, a.stride, a.bc_lo, a.bc_hi, w1);
        make_cell<R, SYS, MEQN>(wm2.q, wm2.zc, NRM, TNG, a.grav, bad, cm2);
        make_cell<R, SYS, MEQN>(wm1.q, wm1.zc, NRM, TNG, a.grav, bad, cm1);
        make_cell<R, SYS, MEQN>(w0.q, w0.zc, NRM, TNG, a.grav, bad, c0);
        make_cell<R, SYS, MEQN>(w1.q, w1.zc, NRM, TNG, a.grav, bad, c1);
        I fa;
        riemann(cm2, cm1, a.Z0, a.c0, a.grav, a.efix, fa);
        riemann(cm1, c0, a.Z0, a.c0, a.grav, a.efix, fb);
        riemann(c0, c1, a.Z0, a.c0, a.grav, a.efix, fc);
        if (xin && y0 == 0) sm = rmax(sm, iface_smax(fb));
        if constexpr (!SPEEDS) {
            Contrib<R> kb;
            limit_contrib(fb, fa, fc, nu, a.limiter, kb);
#pragma unroll
            for (int i = 0; i < 3; ++i) Rb[i] = kb.Rr[i];
        }
    }

    // prefetch ring: pre[k] holds row y + 2 + k at the top of each group
    CC pre[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        if (y0 + 2 + k < y1 + 2)
            col_load<R, SYS, MEQN, NRM>(src, a.zc, a.ncell, colbase, y0 + 2 + k, m, a.stride, a.bc_lo, a.bc_hi, pre[k]);
    }

    for (int64_t y = y0; y < y1; y += PF) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int64_t yy = y + k;
            if (yy < y1) {
                CC w2 = pre[k];
                if (yy + 2 + PF < y1 + 2)
                    col_load<R, SYS, MEQN, NRM>(src, a.zc, a.ncell, colbase, yy + 2 + PF, m, a.stride, a.bc_lo, a.bc_hi, pre[k]);
                C c2;
                make_cell<R, SYS, MEQN>(w2.q, w2.zc, NRM, TNG, a.grav, bad, c2);
                I fd;
                riemann(c1, c2, a.Z0, a.c0, a.grav, a.efix, fd);
                if (xin) sm = rmax(sm, iface_smax(fc));
                if constexpr (!SPEEDS) {
                    Contrib<R> kc;
                    limit_contrib(fc, fb, fd, nu, a.limiter, kc);
                    apply_update<R, SYS, MEQN>(w0.q, Rb, kc.L, nu, NRM, TNG);
                    if (xin) {
                        const int64_t off = colbase + yy * a.stride;
#pragma unroll
                        for (int e = 0; e < MEQN; ++e) dst[e * a.ncell + off] = w0.q[e];
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) Rb[i] = kc.Rr[i];
                }
                fb = fc;
                fc = fd;
                w0 = w1;
                w1 = w2;
                c1 = c2;
            }
        }
    }
    if (!active) bad = false;
    block_publish_smax(ctrl, dir, sm, bad);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename R, int SYS, int MEQN, bool SPEEDS>
static hipError_t launch_row(const SweepArgs<R>& a, hipStream_t s) {
    constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
    const int64_t P = 62 * CPL;
    const int64_t waves = a.nrows * ceil_div(a.nx, P);
    const int64_t blocks = ceil_div(waves, 4);
    hipLaunchKernelGGL((k_sweep_row<R, SYS, MEQN, CPL, SPEEDS>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R, int SYS, int MEQN, int NRM, bool SPEEDS>
static hipError_t launch_col(const SweepArgs<R>& a, hipStream_t s) {
    constexpr int PF = 4;
    const int64_t waves = ceil_div(a.nx, 64) * ceil_div(a.m, a.chunk) * a.nlines_o;
    const int64_t blocks = ceil_div(waves, 4);
    hipLaunchKernelGGL((k_sweep_col<R, SYS, MEQN, NRM, PF, SPEEDS>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R, int SYS, int MEQN, bool SPEEDS>
static hipError_t launch_dir(const SweepArgs<R>& a, hipStream_t s) {
    if (a.dir == 0) return launch_row<R, SYS, MEQN, SPEEDS>(a, s);
    if (a.dir == 1) return launch_col<R, SYS, MEQN, 2, SPEEDS>(a, s);
    if constexpr (MEQN == 4) return launch_col<R, SYS, MEQN, 3, SPEEDS>(a, s);
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_sweep(const SweepArgs<R>& a, int sys, int meqn, bool speeds_only, hipStream_t s) {
    if (sys == SYS_SW) {
        if (meqn != 3) return hipErrorInvalidValue;
        return speeds_only ? launch_dir<R, SYS_SW, 3, true>(a, s) : launch_dir<R, SYS_SW, 3, false>(a, s);
    }
    if (sys == SYS_AC) {
        if (meqn == 3) return speeds_only ? launch_dir<R, SYS_AC, 3, true>(a, s) : launch_dir<R, SYS_AC, 3, false>(a, s);
        if (meqn == 4) return speeds_only ? launch_dir<R, SYS_AC, 4, true>(a, s) : launch_dir<R, SYS_AC, 4, false>(a, s);
        return hipErrorInvalidValue;
    }
    if (sys == SYS_ACV) {
        if (meqn == 3) return speeds_only ? launch_dir<R, SYS_ACV, 3, true>(a, s) : launch_dir<R, SYS_ACV, 3, false>(a, s);
        if (meqn == 4) return speeds_only ? launch_dir<R, SYS_ACV, 4, true>(a, s) : launch_dir<R, SYS_ACV, 4, false>(a, s);
    }
    return hipErrorInvalidValue;
}

template hipError_t launch_sweep<float>(const SweepArgs<float>&, int, int, bool, hipStream_t);
template hipError_t launch_sweep<double>(const SweepArgs<double>&, int, int, bool, hipStream_t);

}  // namespace claw
