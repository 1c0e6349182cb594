// sweep_body.h -- bodies of the directional sweep kernels (equation
// LW-update), shared by the single-grid kernels (sweeps.hip) and the batched
// ensemble kernels (batch.hip).  A body works on one workgroup's share of a
// grid given its logical block coordinates.
//
// The directional sweeps of the split wave-propagation
// step (equation LW-update): Riemann solve at every interface, wave limiter,
// correction flux, single-stage cell update and the fused wave-speed maximum.
//
// Row kernel (x sweep, the contiguous direction).  A wavefront owns a row
// segment: every lane holds CPL consecutive cells loaded with one 16-byte
// vector load per field, solves the CPL interfaces at the left faces of its
// cells and takes what it misses (left neighbour cell, neighbouring waves,
// the next lane's left-cell contribution) from the adjacent lanes with DPP
// wave shifts, so each interface is solved once.  The first and last lane
// of a wave only supply halo interfaces; neighbouring waves overlap by
// 2 * CPL cells.  The cells left at the end of each row are packed several
// rows to a wavefront (row_tail), and a wavefront may sweep several rows in
// turn (RPW; the batched kernels use 8).
//
// Column kernel (y and z sweeps).  A wavefront owns 64 adjacent columns (one
// per lane, coalesced rows) and marches along the sweep direction over a
// chunk of cells with a rolling register window, so each interface is solved
// once per chunk; rows are prefetched PF rows ahead.
//
// Step control needs no kernel of its own: the first sweep of every trial
// decides the previous trial from its speed maxima (open_trial / decide) and
// the last sweep clears the speed slots of the other parity.
//
// Ghost cells are never stored: a cell index outside the grid is mapped to its
// source cell by the boundary rule (section 4.1) when it is loaded.
#pragma once

#include "claw_device.h"

namespace claw {

template <typename R, int CPL>
struct VecOf {
    typedef R type __attribute__((ext_vector_type(CPL)));
};

// Field of a plug-in's state that holds frame component f (0 <= f < MEQN) in
// the frame of direction dir: the vector's components are rotated so that
// its normal component comes first.
template <typename P>
__device__ __forceinline__ constexpr int frame_field(int f, int dir) {
    if constexpr (P::VEC < 0) {
        return f;
    } else {
        return (f < P::VEC || f >= P::VEC + P::NVEC) ? f : P::VEC + (f - P::VEC + dir) % P::NVEC;
    }
}

// Field negated in a wall ghost cell of direction dir (-1: none): the normal
// velocity / momentum, which is field dir + 1 for the built-in systems.
template <int SYS>
__device__ __forceinline__ constexpr int wall_field(int dir) {
    if constexpr (is_plugin(SYS)) {
        using P = Plug<float, SYS>;
        return P::VEC < 0 ? -1 : P::VEC + dir;
    } else {
        return dir + 1;
    }
}
template <int SYS, typename R, int MEQN>
__device__ __forceinline__ void wall_flip(R (&q)[MEQN], int dir) {
    const int f = wall_field<SYS>(dir);
#pragma unroll
    for (int e = 0; e < MEQN; ++e)
        if (e == f) q[e] = -q[e];
}

// Riemann problem between cells l and r of a sweep in direction DIR.
template <typename R, int SYS, int DIR>
__device__ __forceinline__ void solve_iface(const Cell<R, SYS>& l, const Cell<R, SYS>& r,
                                            const SweepArgs<R>& a, R inv2Z, Iface<R, SYS>& o) {
    if constexpr (is_plugin(SYS)) {
        Plug<R, SYS>::template solve<DIR>(l.q, r.q, a.prm, o.W, o.s, o.amdq, o.apdq);
    } else {
        riemann(l, r, a.Z0, a.c0, inv2Z, a.grav, a.efix, o);
    }
}

// nrm, tng: the normal and tangential fields of the sweep (nrm = dir + 1).
template <typename R, int SYS, int MEQN>
__device__ __forceinline__ void make_cell(const R (&q)[MEQN], const R (&zc)[2], int nrm, int tng,
                                          R sg, bool& bad, Cell<R, SYS>& c) {
    if constexpr (is_plugin(SYS)) {
        using P = Plug<R, SYS>;
#pragma unroll
        for (int f = 0; f < MEQN; ++f) c.q[f] = q[frame_field<P>(f, nrm - 1)];
        bad = bad || !P::admissible(c.q);
    } else if constexpr (SYS == SYS_SW) {
        c.h = q[0];
        c.mn = q[nrm];
        c.mt = q[tng];
        c.derive(sg, bad);
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
    if constexpr (is_plugin(SYS)) {
#pragma unroll
        for (int f = 0; f < Plug<R, SYS>::MEQN; ++f) out.q[f] = lane_prev(in.q[f]);
    } else if constexpr (SYS == SYS_SW) {
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
template <typename R, int SYS, int MEQN, int NC>
__device__ __forceinline__ void apply_update(R (&q)[MEQN], const R (&Rl)[NC], const R (&Lr)[NC],
                                             R nu, int nrm, int tng) {
    if constexpr (is_plugin(SYS)) {
#pragma unroll
        for (int f = 0; f < MEQN; ++f) {
            const int e = frame_field<Plug<R, SYS>>(f, nrm - 1);
            q[e] = q[e] - nu * (Rl[f] + Lr[f]);
        }
    } else {
        q[0] = q[0] - nu * (Rl[0] + Lr[0]);
        q[nrm] = q[nrm] - nu * (Rl[1] + Lr[1]);
        if constexpr (SYS == SYS_SW) q[tng] = q[tng] - nu * (Rl[2] + Lr[2]);
    }
}

// Limiter of a sweep: fixed at compile time (LIMK >= 0: the kernel is
// specialised for it and every limiter branch folds) or read from the
// arguments (LIM_RUNTIME).
enum { LIM_RUNTIME = -1 };
template <int LIMK, typename R>
__device__ __forceinline__ int limiter_of(const SweepArgs<R>& a) {
    if constexpr (LIMK >= 0) return LIMK;
    else return a.limiter;
}

template <typename R, int SYS>
__device__ __forceinline__ R ac_inv2Z(const SweepArgs<R>& a) {
    if constexpr (SYS == SYS_AC) return frcp(a.Z0 + a.Z0);
    return R(0);
}

// ---------------------------------------------------------------------------
// Row kernel: x sweep
// ---------------------------------------------------------------------------
// bx: segment of the row (bx = nx / (62 CPL): the packed row tails, see
// row_tail); by: group of four wavefronts; lead: block (0, 0, 0).  Each
// wavefront sweeps RPW rows (RPW * S with packed tails) one after the other,
// so the work that opens a wavefront (argument loads, the step decision) is
// paid once per RPW rows.
template <typename R, int SYS, int MEQN, int CPL, bool SPEEDS, int LIMK = LIM_RUNTIME, int RPW = 1>
__device__ __forceinline__ void row_body(const SweepArgs<R>& a, int bx, int by, bool lead) {
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    typedef typename VecOf<R, CPL>::type V;
    const int nx = a.nx;
    // tail blocks: each wavefront takes the tails of S rows at a time
    const bool tail_blk = bx >= nx / (62 * CPL);
    const RowTail tg = row_tail(nx, CPL);
    const int width = tail_blk ? tg.width : 64;
    const int S = tail_blk ? tg.rows : 1;
    if (by * 4 * RPW * S >= a.nrows) return;  // a block past the last row (whole block)
    if constexpr (SPEEDS) {
        if (a.auto_dt && a.ctrl->st[a.parity].dt_next > 0.0) return;  // next step already known
    }
    // The buffer of this trial is known before the previous trial is decided
    // unless that trial gets reverted: load from the predicted buffer first so
    // the decision's latency overlaps the loads, and reload on a mismatch.
    const int cur_guess = predicted_cur(a);
    const int lane = threadIdx.x & 63;
    // sub-segment and lane within it: lane / width by a multiply (exact for
    // lane < 64 and width <= 64)
    const int sub = (int)(((unsigned)lane * (65536u / (unsigned)width + 1u)) >> 16);
    const int l = lane - sub * width;
    // rows of this lane: row0 + i S, i < RPW
    const int row0 = (by * 4 + wave_uniform((int)(threadIdx.x >> 6))) * RPW * S + sub;
    const int x0 = bx * (62 * CPL);
    const int xl = x0 - CPL + l * CPL;
    // lane roles: useful (updates its cells), right halo of its sub-segment
    const bool useful = l >= 1 && l <= width - 2;
    const bool rhalo = l == width - 1;
    const bool vec_ok = (nx % CPL) == 0 && (a.ncell % CPL) == 0;
    const bool interior = vec_ok && xl >= 0 && xl + CPL <= nx;
    const R inv2Z = ac_inv2Z<R, SYS>(a);
    constexpr int nrm = 1, tng = 2;
    constexpr int NC = contrib_width<SYS>();

    // load the lane's cells of the row starting at base (ghost cells
    // synthesised at the row ends)
    R q[CPL][MEQN];
    R zc[CPL][2];
    // interior lanes: one 16-byte load per field through the field's buffer
    // resource at byte offset (base + xl) sizeof(R)
    const unsigned fbytes = (unsigned)a.ncell * (unsigned)sizeof(R);
    auto load_cells = [&](const R* __restrict__ src, unsigned base) {
        if (interior) {
            const unsigned voff = (base + (unsigned)xl) * (unsigned)sizeof(R);
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
        } else {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                bool flip;
                const unsigned sidx = base + (unsigned)ghost_idx(xl + c, nx, a.bc_lo, a.bc_hi, flip);
                CLAW_CHECK(sidx < (unsigned)a.ncell);
#pragma unroll
                for (int e = 0; e < MEQN; ++e) q[c][e] = src[(size_t)e * a.ncell + sidx];
                if (flip) wall_flip<SYS>(q[c], 0);
                if constexpr (SYS == SYS_ACV) {
                    zc[c][0] = a.zc[sidx];
                    zc[c][1] = a.zc[(size_t)a.ncell + sidx];
                }
            }
        }
    };
    auto base_of = [&](int row) { return (unsigned)((row < a.nrows ? row : 0) * nx); };
    load_cells(pick_buf(a, (cur_guess + a.src_off) % 3), base_of(row0));

    const Trial<R> tr = open_trial(a, 0, lead);
    if (tr.done && !SPEEDS) return;
    const R* __restrict__ src = pick_buf(a, (tr.cur + a.src_off) % 3);
    if (tr.cur != cur_guess) load_cells(src, base_of(row0));
    R* __restrict__ dst = pick_buf(a, (tr.cur + a.dst_off) % 3);
    const R nu = tr.nu;

    bool bad = false;
    R sm = R(0);
    for (int i = 0; i < RPW; ++i) {
        const int row = row0 + i * S;
        const bool active = row < a.nrows && sub < S;
        const unsigned base = base_of(row);
        if (i > 0) load_cells(src, base);

        bool rbad = false;
        C cell[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) make_cell<R, SYS, MEQN>(q[c], zc[c], nrm, tng, a.sqrt_grav, rbad, cell[c]);
        bad = bad || (active && rbad);

        // interfaces at the left face of each cell of this lane
        C left;
        cell_prev(cell[CPL - 1], left);
        I f[CPL];
        solve_iface<R, SYS, 0>(left, cell[0], a, inv2Z, f[0]);
#pragma unroll
        for (int c = 1; c < CPL; ++c) solve_iface<R, SYS, 0>(cell[c - 1], cell[c], a, inv2Z, f[c]);

        // largest speed over the interfaces j = x, 0 <= j <= nx, owned by the
        // useful lanes 1..width-2 (and by the right halo lane for j = nx when
        // the row ends exactly at its first cell)
        if (active) {
            if (interior) {  // faces xl .. xl + CPL - 1, all inside the row
                R m = iface_smax(f[0]);
#pragma unroll
                for (int c = 1; c < CPL; ++c) m = rmax(m, iface_smax(f[c]));
                if (useful) sm = rmax(sm, m);
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int j = xl + c;
                    const bool own = (useful && j >= 0 && j <= nx) || (rhalo && c == 0 && j == nx);
                    if (own) sm = rmax(sm, iface_smax(f[c]));
                }
            }
        }

        if constexpr (!SPEEDS) {
            I fprev, fnext;
            iface_prev(f[CPL - 1], fprev);
            iface_next(f[0], fnext);
            Contrib<R, NC> k[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const I& km = c == 0 ? fprev : f[c - 1];
                const I& kp = c == CPL - 1 ? fnext : f[c + 1];
                limit_contrib(f[c], km, kp, nu, limiter_of<LIMK>(a), k[c]);
            }
            R Lnext[NC];
#pragma unroll
            for (int n = 0; n < NC; ++n) Lnext[n] = lane_next(k[0].L[n]);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                if (c < CPL - 1) apply_update<R, SYS, MEQN>(q[c], k[c].Rr, k[c + 1].L, nu, nrm, tng);
                else apply_update<R, SYS, MEQN>(q[c], k[c].Rr, Lnext, nu, nrm, tng);
            }
            if (active && useful) {
                if (interior) {
                    const unsigned voff = (base + (unsigned)xl) * (unsigned)sizeof(R);
#pragma unroll
                    for (int e = 0; e < MEQN; ++e) {
                        V v;
#pragma unroll
                        for (int c = 0; c < CPL; ++c) v[c] = q[c][e];
                        buf_store16<V>(field_rsrc(dst + (size_t)e * (unsigned)a.ncell, fbytes), voff, v);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        if (xl + c < nx) {
#pragma unroll
                            for (int e = 0; e < MEQN; ++e) {
                                CLAW_CHECK(base + (unsigned)(xl + c) < (unsigned)a.ncell);
                                dst[(size_t)e * a.ncell + base + (unsigned)(xl + c)] = q[c][e];
                            }
                        }
                    }
                }
            }
        }
    }
    block_finish(a, 0, sm, bad, lead);
}

// ---------------------------------------------------------------------------
// Column kernel: y and z sweeps
// ---------------------------------------------------------------------------
template <typename R, int SYS, int MEQN>
struct ColCell {
    R q[MEQN];
    R zc[2];
};

// Buffer resources of the fields a column sweep reads and writes.
template <typename R, int MEQN>
struct ColRes {
    Rsrc src[MEQN], dst[MEQN], zc[2];
};

// Loads row y (a ghost row is mapped by the boundary rule) of the wavefront's
// 64 columns.  plane_b: byte offset of the wavefront's outer plane (the same
// for every lane); lane_byte: byte offset of the lane's column in a row.
template <typename R, int SYS, int MEQN, int NRM>
__device__ __forceinline__ void col_load(const ColRes<R, MEQN>& res, const SweepArgs<R>& a, unsigned plane_b,
                                         unsigned lane_byte, int y, ColCell<R, SYS, MEQN>& out) {
    bool flip;
    const unsigned soff =
        plane_b + (unsigned)(ghost_idx(y, a.m, a.bc_lo, a.bc_hi, flip) * a.stride) * (unsigned)sizeof(R);
#pragma unroll
    for (int e = 0; e < MEQN; ++e) out.q[e] = buf_load(res.src[e], lane_byte, soff, R(0));
    if (flip) wall_flip<SYS>(out.q, NRM - 1);
    if constexpr (SYS == SYS_ACV) {
        out.zc[0] = buf_load(res.zc[0], lane_byte, soff, R(0));
        out.zc[1] = buf_load(res.zc[1], lane_byte, soff, R(0));
    }
}

// bx: group of four 64-column strips; by: chunk along the sweep; bz: outer
// plane; lead: block (0, 0, 0).
template <typename R, int SYS, int MEQN, int NRM, int PF, bool SPEEDS, int LIMK = LIM_RUNTIME>
__device__ __forceinline__ void col_body(const SweepArgs<R>& a, int bx, int by, int bz, bool lead) {
    using C = Cell<R, SYS>;
    using I = Iface<R, SYS>;
    using CC = ColCell<R, SYS, MEQN>;
    constexpr int TNG = SYS == SYS_SW ? 3 - NRM : 0;
    constexpr int dir = NRM - 1;  // the normal component of direction d is q[d + 1]
    constexpr int NC = contrib_width<SYS>();
    if constexpr (SPEEDS) {
        if (a.auto_dt && a.ctrl->st[a.parity].dt_next > 0.0) return;  // next step already known
    }
    const Trial<R> tr = open_trial(a, dir, lead);
    if (tr.done && !SPEEDS) return;
    const R* __restrict__ src = pick_buf(a, (tr.cur + a.src_off) % 3);
    R* __restrict__ dst = pick_buf(a, (tr.cur + a.dst_off) % 3);
    const R nu = tr.nu;
    const R inv2Z = ac_inv2Z<R, SYS>(a);
    const int lane = threadIdx.x & 63;
    const int nx = a.nx, m = a.m;
    const int nstrip = (nx + 63) >> 6;
    const int strip = wave_uniform(bx * 4 + (int)(threadIdx.x >> 6));
    const bool sactive = strip < nstrip;
    const int x = strip * 64 + lane;
    const bool xin = sactive && x < nx;
    const unsigned plane_b = (unsigned)(bz * a.ostride) * (unsigned)sizeof(R);
    const unsigned lane_byte = (unsigned)(x < nx ? x : nx - 1) * (unsigned)sizeof(R);
    const unsigned fbytes = (unsigned)a.ncell * (unsigned)sizeof(R);
    ColRes<R, MEQN> res;
#pragma unroll
    for (int e = 0; e < MEQN; ++e) {
        res.src[e] = field_rsrc(src + (size_t)e * (unsigned)a.ncell, fbytes);
        res.dst[e] = field_rsrc(dst + (size_t)e * (unsigned)a.ncell, fbytes);
    }
    if constexpr (SYS == SYS_ACV) {
        res.zc[0] = field_rsrc(a.zc, fbytes);
        res.zc[1] = field_rsrc(a.zc + (size_t)(unsigned)a.ncell, fbytes);
    }
    const int y0 = by * a.chunk;
    const int y1 = sactive ? (y0 + a.chunk < m ? y0 + a.chunk : m) : y0;

    bool bad = false;
    R sm = R(0);
    CC w0, w1;  // cells y and y+1 of the window
    C c1;
    I fb, fc;   // interfaces j = y and j = y + 1
    R Rb[NC];   // right-cell contribution of interface j = y
    {
        CC wm2, wm1;
        C cm2, cm1, c0;
        col_load<R, SYS, MEQN, NRM>(res, a, plane_b, lane_byte, y0 - 2, wm2);
        col_load<R, SYS, MEQN, NRM>(res, a, plane_b, lane_byte, y0 - 1, wm1);
        col_load<R, SYS, MEQN, NRM>(res, a, plane_b, lane_byte, y0, w0);
        col_load<R, SYS, MEQN, NRM>(res, a, plane_b, lane_byte, y0 + 1, w1);
        make_cell<R, SYS, MEQN>(wm2.q, wm2.zc, NRM, TNG, a.sqrt_grav, bad, cm2);
        make_cell<R, SYS, MEQN>(wm1.q, wm1.zc, NRM, TNG, a.sqrt_grav, bad, cm1);
        make_cell<R, SYS, MEQN>(w0.q, w0.zc, NRM, TNG, a.sqrt_grav, bad, c0);
        make_cell<R, SYS, MEQN>(w1.q, w1.zc, NRM, TNG, a.sqrt_grav, bad, c1);
        I fa;
        solve_iface<R, SYS, dir>(cm2, cm1, a, inv2Z, fa);
        solve_iface<R, SYS, dir>(cm1, c0, a, inv2Z, fb);
        solve_iface<R, SYS, dir>(c0, c1, a, inv2Z, fc);
        if (y0 == 0) sm = iface_smax(fb);
        if constexpr (!SPEEDS) {
            Contrib<R, NC> kb;
            limit_contrib(fb, fa, fc, nu, limiter_of<LIMK>(a), kb);
#pragma unroll
            for (int i = 0; i < NC; ++i) Rb[i] = kb.Rr[i];
        }
    }

    // prefetch ring: pre[k] holds row y + 2 + k at the top of each group;
    // refills past the last needed row (y1 + 1) reload that row instead
    const int ylast = y1 + 1;
    CC pre[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int r = y0 + 2 + k;
        col_load<R, SYS, MEQN, NRM>(res, a, plane_b, lane_byte, r < ylast ? r : ylast, pre[k]);
    }

    // one row of the march: cell yy is finished, the window moves down by one
    auto step = [&](int yy, CC& slot) {
        CC w2 = slot;
        const int r = yy + 2 + PF;
        col_load<R, SYS, MEQN, NRM>(res, a, plane_b, lane_byte, r < ylast ? r : ylast, slot);
        C c2;
        make_cell<R, SYS, MEQN>(w2.q, w2.zc, NRM, TNG, a.sqrt_grav, bad, c2);
        I fd;
        solve_iface<R, SYS, dir>(c1, c2, a, inv2Z, fd);
        sm = rmax(sm, iface_smax(fc));
        if constexpr (!SPEEDS) {
            Contrib<R, NC> kc;
            limit_contrib(fc, fb, fd, nu, limiter_of<LIMK>(a), kc);
            apply_update<R, SYS, MEQN>(w0.q, Rb, kc.L, nu, NRM, TNG);
            if (xin) {
                const unsigned soff = plane_b + (unsigned)(yy * a.stride) * (unsigned)sizeof(R);
#pragma unroll
                for (int e = 0; e < MEQN; ++e) buf_store(res.dst[e], lane_byte, soff, w0.q[e]);
            }
#pragma unroll
            for (int i = 0; i < NC; ++i) Rb[i] = kc.Rr[i];
        }
        fb = fc;
        fc = fd;
        w0 = w1;
        w1 = w2;
        c1 = c2;
    };

    int y = y0;
    for (; y + PF <= y1; y += PF) {
#pragma unroll
        for (int k = 0; k < PF; ++k) step(y + k, pre[k]);
    }
    if (y < y1) {  // ragged end of the last chunk
#pragma unroll
        for (int k = 0; k < PF; ++k)
            if (y + k < y1) step(y + k, pre[k]);
    }
    if (!xin) {
        bad = false;
        sm = R(0);
    }
    block_finish(a, dir, sm, bad, lead);
}

}  // namespace claw
