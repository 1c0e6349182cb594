// claw_device.h -- device-side building blocks of the split wave-propagation
// sweeps for gfx950: control block, boundary index maps, the point-wise
// Riemann solvers (section 4.2 of the CUDACLAW paper), the wave limiter and the
// per-interface update contributions of equation LW-update.
//
// Compact wave form.  A wave is W^p = alpha_p r_p with r_p the eigenvector of
// the local linearisation, so an interface is stored as strengths alpha_p,
// speeds s_p, left-going speed shares a_p (A-dQ = sum_p a_p alpha_p r_p,
// A+dQ = sum_p (s_p - a_p) alpha_p r_p) and the two numbers e0, e1 that fix
// the eigenvectors:
//   shallow water (h, m_n, m_t):  r_1 = (1, s_1, e0), r_2 = (0, 0, 1),
//                                 r_3 = (1, s_3, e0), e0 = Roe tangential
//                                 velocity;
//   acoustics (p, u_n):           r_1 = (-e0, 1), r_2 = (e1, 1), e0 = Z left,
//                                 e1 = Z right (impedances).
// With the limited strength phi_p and c_p = 1/2 |s_p| (1 - dt/dx |s_p|) the
// interface hands its left cell  L = A-dQ + F~ = sum (a_p + c_p phi_p) alpha_p r_p
// and its right cell  R = A+dQ - F~ = sum (s_p - a_p - c_p phi_p) alpha_p r_p,
// and every cell is updated once: Q_k -= dt/dx (R_{k-1/2} + L_{k+1/2})
// (single-stage update, section 5.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace claw {

enum { BC_EXTRAP = 0, BC_WALL = 1, BC_PERIODIC = 2 };
enum { LIM_MC = 0, LIM_NONE = 1, LIM_FIRST = 2 };
// system kinds as compiled: constant-coefficient acoustics, acoustics with
// per-cell coefficients, shallow water
enum { SYS_AC = 0, SYS_ACV = 1, SYS_SW = 2 };

// Device control block: step-control state that lives on the GPU so that a
// captured graph can run many steps without the host.
struct alignas(256) Ctrl {
    double t;          // simulation time of the current state
    double dt;         // time step of the trial in flight
    double dt_next;    // proposal for the next trial
    double cfl;        // Courant number of the last trial
    double dtdx[3];    // dt / dx_d of the trial in flight
    float dtdx_f[3];   // the same rounded once to FP32
    int32_t mode;      // control mode of the run in flight
    double dx[3];
    double cfl_desired, cfl_max, dt_max;
    unsigned long long smax64[3];  // per-direction max |s| (FP64 bit pattern)
    unsigned int smax32[3];        // per-direction max |s| (FP32 bit pattern)
    int32_t cur;       // rotation buffer holding the current state
    int32_t done;      // nonzero: the requested steps are complete (sweeps skip)
    int32_t nonphys;   // set by a sweep that met depth <= 0 or NaN
    int32_t err;       // claw_status of a failure that stopped the run
    int32_t last_accepted;
    int32_t ndim;
    long long accepted, rejected, target, consecutive, trials;
};

// Per-launch arguments of a sweep kernel (passed by value).
template <typename R>
struct SweepArgs {
    R* buf[3];          // rotation buffers (buf[0] is the caller's q)
    const R* zc;        // derived coefficients: Z field then c field (SYS_ACV)
    Ctrl* ctrl;
    int64_t ncell;      // field stride
    int64_t nx;         // cells along x (the contiguous direction)
    int64_t m;          // cells along the sweep direction
    int64_t stride;     // element stride along the sweep direction
    int64_t nlines_o;   // column kernels: number of outer planes
    int64_t ostride;    // column kernels: element stride between outer planes
    int64_t nrows;      // row kernel: number of x-lines
    int32_t dir;        // 0, 1, 2
    int32_t src_off;    // source buffer = (cur + src_off) % 3
    int32_t dst_off;    // destination buffer = (cur + dst_off) % 3
    int32_t bc_lo, bc_hi;
    int32_t limiter;
    int32_t efix;
    int32_t speeds_only;
    int64_t chunk;      // column kernels: rows per wave
    R grav;
    R Z0, c0;           // constant-coefficient acoustics
};

// ---------------------------------------------------------------------------
// Precision helpers.  FP64 keeps correctly rounded division and square root;
// FP32 uses the hardware reciprocal and square root (about 1 ulp).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ double frcp(double a) { return 1.0 / a; }
__device__ __forceinline__ double fsqrt(double a) { return __builtin_sqrt(a); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float frcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ float fsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }

template <typename R>
__device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }
template <typename R>
__device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }
template <typename R>
__device__ __forceinline__ R rabs(R a) { return a < R(0) ? -a : a; }

// Source index of cell i (possibly a ghost, -2 <= i < m + 2) along a line of
// m cells; flip = the normal component changes sign (wall).
__device__ __forceinline__ int64_t ghost_src(int64_t i, int64_t m, int bc_lo, int bc_hi,
                                             bool& flip) {
    flip = false;
    if (i < 0) {
        if (bc_lo == BC_EXTRAP) return 0;
        if (bc_lo == BC_WALL) {
            flip = true;
            int64_t r = -1 - i;
            return r > m - 1 ? m - 1 : r;
        }
        int64_t r = i % m;
        return r < 0 ? r + m : r;
    }
    if (i >= m) {
        if (bc_hi == BC_EXTRAP) return m - 1;
        if (bc_hi == BC_WALL) {
            flip = true;
            int64_t r = 2 * m - 1 - i;
            return r < 0 ? 0 : r;
        }
        return i % m;
    }
    return i;
}

// ---------------------------------------------------------------------------
// Cells and interfaces
// ---------------------------------------------------------------------------
template <typename R, int SYS>
struct Cell;

// acoustics: pressure and normal velocity; tangential components are copied
// through by the caller (a normal sweep never changes them)
template <typename R>
struct Cell<R, SYS_AC> {
    R p, un;
    __device__ void derive(R, bool&) {}
};
template <typename R>
struct Cell<R, SYS_ACV> {
    R p, un, Z, c;
    __device__ void derive(R, bool&) {}
};
// shallow water: depth, normal and tangential momentum plus derived per-cell
// values shared by both interfaces of the cell
template <typename R>
struct Cell<R, SYS_SW> {
    R h, mn, mt;
    R u, v, sqh, c;
    __device__ void derive(R g, bool& bad) {
        bool ok = h > R(0);  // false for NaN too
        bad = bad || !ok;
        R hh = ok ? h : R(1);
        R ih = frcp(hh);
        u = mn * ih;
        v = mt * ih;
        sqh = fsqrt(hh);
        c = fsqrt(g * hh);
    }
};

template <typename R, int SYS>
struct Iface {
    static constexpr int MW = SYS == SYS_SW ? 3 : 2;
    R alpha[MW];
    R s[MW];
    R am[MW];  // left-going speed share a_p
    R e0, e1;
};

template <typename R>
__device__ __forceinline__ void riemann(const Cell<R, SYS_AC>& l, const Cell<R, SYS_AC>& r,
                                        R Z, R c, R, int, Iface<R, SYS_AC>& o) {
    R dp = r.p - l.p;
    R du = r.un - l.un;
    R inv = frcp(Z + Z);
    o.alpha[0] = (-dp + Z * du) * inv;
    o.alpha[1] = (dp + Z * du) * inv;
    o.s[0] = -c;
    o.s[1] = c;
    o.am[0] = -c;
    o.am[1] = R(0);
    o.e0 = Z;
    o.e1 = Z;
}

template <typename R>
__device__ __forceinline__ void riemann(const Cell<R, SYS_ACV>& l, const Cell<R, SYS_ACV>& r,
                                        R, R, R, int, Iface<R, SYS_ACV>& o) {
    R dp = r.p - l.p;
    R du = r.un - l.un;
    R inv = frcp(l.Z + r.Z);
    o.alpha[0] = (-dp + r.Z * du) * inv;
    o.alpha[1] = (dp + l.Z * du) * inv;
    o.s[0] = -l.c;
    o.s[1] = r.c;
    o.am[0] = -l.c;
    o.am[1] = R(0);
    o.e0 = l.Z;
    o.e1 = r.Z;
}

// Roe solver with arithmetic-mean depth and sqrt(h)-weighted velocities plus
// the Harten-Hyman entropy fix on the 1- and 3-waves.  The transonic test of
// the fix, lambda_r = m/h - sqrt(g h) > 0 in the middle state, is taken as
// m > 0 and m^2 > g h^3 so that the division and square root are only paid in
// the (rare) transonic case; the split it selects is continuous across the
// test's boundary.
template <typename R>
__device__ __forceinline__ void riemann(const Cell<R, SYS_SW>& l, const Cell<R, SYS_SW>& r,
                                        R, R, R g, int efix, Iface<R, SYS_SW>& o) {
    R hbar = R(0.5) * (l.h + r.h);
    R inv = frcp(l.sqh + r.sqh);
    R uhat = (l.sqh * l.u + r.sqh * r.u) * inv;
    R vhat = (l.sqh * l.v + r.sqh * r.v) * inv;
    R chat = fsqrt(g * hbar);
    R dh = r.h - l.h;
    R dn = r.mn - l.mn;
    R dt = r.mt - l.mt;
    R i2c = frcp(chat + chat);
    R s1 = uhat - chat;
    R s3 = uhat + chat;
    R a1 = (s3 * dh - dn) * i2c;
    R a2 = dt - vhat * dh;
    R a3 = (dn - s1 * dh) * i2c;
    R am1 = rmin(s1, R(0));
    R am3 = rmin(s3, R(0));
    if (efix) {
        R lam_l = l.u - l.c;
        R hm = l.h + a1;
        R mm = l.mn + a1 * s1;
        if (lam_l < R(0) && hm > R(0) && mm > R(0) && mm * mm > g * hm * hm * hm) {
            R lam_r = fdiv(mm, hm) - fsqrt(g * hm);
            if (lam_r > R(0)) am1 = fdiv(lam_l * (lam_r - s1), lam_r - lam_l);
        }
        R lam_r3 = r.u + r.c;
        R hm3 = r.h - a3;
        R mm3 = r.mn - a3 * s3;
        if (lam_r3 > R(0) && hm3 > R(0) && mm3 < R(0) && mm3 * mm3 > g * hm3 * hm3 * hm3) {
            R lam_l3 = fdiv(mm3, hm3) + fsqrt(g * hm3);
            if (lam_l3 < R(0)) am3 = fdiv(lam_l3 * (lam_r3 - s3), lam_r3 - lam_l3);
        }
    }
    o.alpha[0] = a1;
    o.alpha[1] = a2;
    o.alpha[2] = a3;
    o.s[0] = s1;
    o.s[1] = uhat;
    o.s[2] = s3;
    o.am[0] = am1;
    o.am[1] = rmin(uhat, R(0));
    o.am[2] = am3;
    o.e0 = vhat;
    o.e1 = R(0);
}

// r_p(this) . r_p(other) for the limiter's wave-projection ratio
template <typename R>
__device__ __forceinline__ R rdot(const Iface<R, SYS_SW>& a, const Iface<R, SYS_SW>& b, int p) {
    if (p == 1) return R(1);
    return R(1) + a.s[p] * b.s[p] + a.e0 * b.e0;
}
template <typename R, int SYS>
__device__ __forceinline__ R rdot(const Iface<R, SYS>& a, const Iface<R, SYS>& b, int p) {
    return p == 0 ? R(1) + a.e0 * b.e0 : R(1) + a.e1 * b.e1;
}

template <typename R>
__device__ __forceinline__ R phi_mc(R theta) {
    return rmax(R(0), rmin(R(0.5) * (R(1) + theta), rmin(R(2), theta + theta)));
}

// Output of one limited interface: contributions to its left and right cell
// in the interface's normal frame.  Shallow water: (h, m_n, m_t); acoustics:
// (p, u_n) in slots 0, 1.
template <typename R>
struct Contrib {
    R L[3];
    R Rr[3];
};

// Limits interface k with its neighbours km (k - 1) and kp (k + 1) and forms
// the contributions.  nu = dt / dx.
template <typename R, int SYS>
__device__ __forceinline__ void limit_contrib(const Iface<R, SYS>& k, const Iface<R, SYS>& km,
                                              const Iface<R, SYS>& kp, R nu, int limiter,
                                              Contrib<R>& out) {
    constexpr int MW = Iface<R, SYS>::MW;
    R kl[MW], kr[MW];
#pragma unroll
    for (int p = 0; p < MW; ++p) {
        R sp = k.s[p];
        R as = rabs(sp);
        R beta = R(0);
        // a wave whose squared length is zero (underflow included) gets no
        // correction; any other wave has a normal-range divisor below
        if (limiter != LIM_FIRST && k.alpha[p] * k.alpha[p] != R(0)) {
            R phi = R(1);
            if (limiter == LIM_MC) {
                // upwind neighbour by the sign of the speed
                const Iface<R, SYS>& up = sp > R(0) ? km : kp;
                R num = up.alpha[p] * rdot(up, k, p);
                R den = k.alpha[p] * rdot(k, k, p);
                phi = phi_mc(fdiv(num, den));
            }
            beta = R(0.5) * as * (R(1) - nu * as) * phi;
        }
        R a = k.am[p] + beta;
        kl[p] = a * k.alpha[p];
        kr[p] = (sp - a) * k.alpha[p];
    }
    if constexpr (SYS == SYS_SW) {
        R l13 = kl[0] + kl[2];
        R r13 = kr[0] + kr[2];
        out.L[0] = l13;
        out.L[1] = kl[0] * k.s[0] + kl[2] * k.s[2];
        out.L[2] = l13 * k.e0 + kl[1];
        out.Rr[0] = r13;
        out.Rr[1] = kr[0] * k.s[0] + kr[2] * k.s[2];
        out.Rr[2] = r13 * k.e0 + kr[1];
    } else {
        out.L[0] = -kl[0] * k.e0 + kl[1] * k.e1;
        out.L[1] = kl[0] + kl[1];
        out.Rr[0] = -kr[0] * k.e0 + kr[1] * k.e1;
        out.Rr[1] = kr[0] + kr[1];
        out.L[2] = R(0);
        out.Rr[2] = R(0);
    }
}

template <typename R, int SYS>
__device__ __forceinline__ R iface_smax(const Iface<R, SYS>& k) {
    R m = R(0);
#pragma unroll
    for (int p = 0; p < Iface<R, SYS>::MW; ++p) m = rmax(m, rabs(k.s[p]));
    return m;
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T lane_prev(T v) {  // value of lane - 1
    return __shfl_up(v, 1, 64);
}
template <typename T>
__device__ __forceinline__ T lane_next(T v) {  // value of lane + 1
    return __shfl_down(v, 1, 64);
}

template <typename R, int SYS>
__device__ __forceinline__ void iface_prev(const Iface<R, SYS>& in, Iface<R, SYS>& out) {
#pragma unroll
    for (int p = 0; p < Iface<R, SYS>::MW; ++p) {
        out.alpha[p] = lane_prev(in.alpha[p]);
        out.s[p] = lane_prev(in.s[p]);
    }
    out.e0 = lane_prev(in.e0);
    out.e1 = lane_prev(in.e1);
}
template <typename R, int SYS>
__device__ __forceinline__ void iface_next(const Iface<R, SYS>& in, Iface<R, SYS>& out) {
#pragma unroll
    for (int p = 0; p < Iface<R, SYS>::MW; ++p) {
        out.alpha[p] = lane_next(in.alpha[p]);
        out.s[p] = lane_next(in.s[p]);
    }
    out.e0 = lane_next(in.e0);
    out.e1 = lane_next(in.e1);
}

template <typename R>
__device__ __forceinline__ R wave_max(R v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = rmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Per-direction speed maximum: non-negative IEEE values order like their bit
// patterns, so an unsigned atomic max is exact and order independent.
__device__ __forceinline__ void publish_smax(Ctrl* c, int dir, float v) {
    unsigned int bits = __float_as_uint(v);
    if (bits > __atomic_load_n(&c->smax32[dir], __ATOMIC_RELAXED)) atomicMax(&c->smax32[dir], bits);
}
__device__ __forceinline__ void publish_smax(Ctrl* c, int dir, double v) {
    unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    if (bits > __atomic_load_n(&c->smax64[dir], __ATOMIC_RELAXED)) atomicMax(&c->smax64[dir], bits);
}

template <typename R>
__device__ __forceinline__ R ctrl_nu(const Ctrl* c, int dir);
template <>
__device__ __forceinline__ float ctrl_nu<float>(const Ctrl* c, int dir) { return c->dtdx_f[dir]; }
template <>
__device__ __forceinline__ double ctrl_nu<double>(const Ctrl* c, int dir) { return c->dtdx[dir]; }

// Block-wide max of v published once per workgroup (blockDim.x a multiple of 64).
template <typename R>
__device__ __forceinline__ void block_publish_smax(Ctrl* c, int dir, R v, bool bad) {
    __shared__ R red[16];
    __shared__ int redbad[16];
    v = wave_max(v);
    int anybad = __any(bad) ? 1 : 0;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = v;
        redbad[w] = anybad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        R m = R(0);
        int b = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            m = rmax(m, red[i]);
            b |= redbad[i];
        }
        publish_smax(c, dir, m);
        if (b) atomicOr(&c->nonphys, 1);
    }
}

}  // namespace claw
