// plugins.h -- point-wise Riemann solvers supplied through the plug-in
// interface (section 4.2 of the CUDACLAW paper: the user writes the Riemann
// solver of one interface; the framework runs it at every interface of every
// sweep and supplies boundary conditions, the wave limiter, the correction
// flux, the update and the CFL reduction).
//
// Contract.  A plug-in is a class template P<R> (R = float or double) with
//   static constexpr int MEQN;      fields per cell (1..4)
//   static constexpr int MWAVES;    waves per interface (1..3)
//   static constexpr int VEC;       first field of the vector (velocity or
//                                   momentum) that rotates with the sweep
//                                   direction, -1 if none
//   static constexpr int NVEC;      its number of components (0 if VEC < 0)
//   static constexpr int NDIM_MAX;  2 or 3
//   static const char* name();
//   __device__ static bool admissible(const R (&q)[MEQN]);
//   template <int DIR>
//   __device__ static void solve(const R (&ql)[MEQN], const R (&qr)[MEQN],
//                                const R (&prm)[4], R (&W)[MWAVES][MEQN],
//                                R (&s)[MWAVES], R (&amdq)[MEQN], R (&apdq)[MEQN]);
// solve() receives the left and right cell in the sweep's normal frame: field
// VEC + k holds component (DIR + k) mod NVEC of the vector, so field VEC is the
// normal component; it returns the waves W^p, their speeds s^p and the
// fluctuations A-dQ, A+dQ in the same frame.  DIR is the sweep direction
// (0 = x, 1 = y, 2 = z) as a compile-time constant; prm are the four
// parameters of the problem description.  admissible() is false for a state
// the solver cannot take (the step then fails as non-physical).  A wall
// boundary negates field VEC of the mirrored ghost cells (a plug-in without a
// vector is mirrored unchanged).
//
// The framework limits each wave by phi(theta) with theta the projection
// W_up . W / W . W of the same-family wave at the upwind interface (chosen by
// the sign of s^p), forms F~ = 1/2 sum_p |s^p| (1 - dt/dx |s^p|) phi W^p and
// updates Q_k -= dt/dx (A+dQ_{k-1/2} - F~_{k-1/2} + A-dQ_{k+1/2} + F~_{k+1/2}).
// The largest |s^p| enters the CFL reduction.
//
// Registering a plug-in: add its class template here and one X(id, name)
// entry to CLAW_PLUGINS (ids from 16 up); the library then accepts that id as
// claw_desc.riemann and compiles row and column sweep kernels for it.
#pragma once

namespace claw {

// Scalar Burgers-type law q_t + sum_d (c_d q^2 / 2)_{x_d} = 0 with c_d =
// prm[d]: one wave (the jump) at the Rankine-Hugoniot speed c (ql + qr) / 2.
// Entropy fix: a transonic rarefaction (c ql < 0 < c qr) passes the flux
// difference through q = 0 (f(0) = 0): A-dQ = -f(ql), A+dQ = f(qr)
// (LeVeque 2002, sections 11.8 and 12.2).
template <typename R>
struct BurgersPlugin {
    static constexpr int MEQN = 1, MWAVES = 1, VEC = -1, NVEC = 0, NDIM_MAX = 3;
    static const char* name() { return "burgers"; }
    __device__ static bool admissible(const R (&q)[1]) {
        return (q[0] - q[0]) == R(0);  // false for NaN and infinities
    }
    template <int DIR>
    __device__ static void solve(const R (&ql)[1], const R (&qr)[1], const R (&prm)[4],
                                 R (&W)[1][1], R (&s)[1], R (&amdq)[1], R (&apdq)[1]) {
        const R c = prm[DIR];
        const R l = ql[0], r = qr[0];
        W[0][0] = r - l;
        s[0] = R(0.5) * (c * (l + r));
        if (c * l < R(0) && c * r > R(0)) {
            amdq[0] = -(R(0.5) * (c * l * l));
            apdq[0] = R(0.5) * (c * r * r);
        } else {
            amdq[0] = rmin(s[0], R(0)) * W[0][0];
            apdq[0] = rmax(s[0], R(0)) * W[0][0];
        }
    }
};

// Shallow water (h, m_n, m_t) through the plug-in path: Roe linearisation with
// arithmetic-mean depth and sqrt(h)-weighted velocities and the Harten-Hyman
// entropy fix on the 1- and 3-waves (prm[0] = g, prm[1] != 0 turns the fix
// on).  It computes what the specialised shallow-water sweep computes, written
// plainly with full wave vectors, as a multi-wave example of the interface.
template <typename R>
struct ShallowWaterPlugin {
    static constexpr int MEQN = 3, MWAVES = 3, VEC = 1, NVEC = 2, NDIM_MAX = 2;
    static const char* name() { return "shallow_water_generic"; }
    __device__ static bool admissible(const R (&q)[3]) { return q[0] > R(0); }
    template <int DIR>
    __device__ static void solve(const R (&ql)[3], const R (&qr)[3], const R (&prm)[4],
                                 R (&W)[3][3], R (&s)[3], R (&amdq)[3], R (&apdq)[3]) {
        const R g = prm[0];
        // an inadmissible state has been flagged already; keep the arithmetic finite
        const R hl = ql[0] > R(0) ? ql[0] : R(1);
        const R hr = qr[0] > R(0) ? qr[0] : R(1);
        const R ul = fdiv(ql[1], hl), vl = fdiv(ql[2], hl);
        const R ur = fdiv(qr[1], hr), vr = fdiv(qr[2], hr);
        const R shl = fsqrt(hl), shr = fsqrt(hr);
        const R hbar = R(0.5) * (hl + hr);
        const R uhat = fdiv(shl * ul + shr * ur, shl + shr);
        const R vhat = fdiv(shl * vl + shr * vr, shl + shr);
        const R chat = fsqrt(g * hbar);
        const R dh = qr[0] - ql[0], dn = qr[1] - ql[1], dt = qr[2] - ql[2];
        const R a1 = fdiv((uhat + chat) * dh - dn, R(2) * chat);
        const R a2 = dt - vhat * dh;
        const R a3 = fdiv(dn - (uhat - chat) * dh, R(2) * chat);
        s[0] = uhat - chat;
        s[1] = uhat;
        s[2] = uhat + chat;
        W[0][0] = a1;
        W[0][1] = a1 * s[0];
        W[0][2] = a1 * vhat;
        W[1][0] = R(0);
        W[1][1] = R(0);
        W[1][2] = a2;
        W[2][0] = a3;
        W[2][1] = a3 * s[2];
        W[2][2] = a3 * vhat;
        R am[3];
        for (int p = 0; p < 3; ++p) am[p] = rmin(s[p], R(0));
        if (prm[1] != R(0)) {
            const R lam_l = ul - fsqrt(g * hl);
            const R hm = hl + W[0][0];
            const R mm = ql[1] + W[0][1];
            if (hm > R(0)) {
                const R lam_r = fdiv(mm, hm) - fsqrt(g * hm);
                if (lam_l < R(0) && lam_r > R(0)) am[0] = fdiv(lam_l * (lam_r - s[0]), lam_r - lam_l);
            }
            const R lam_r3 = ur + fsqrt(g * hr);
            const R hm3 = hr - W[2][0];
            const R mm3 = qr[1] - W[2][1];
            if (hm3 > R(0)) {
                const R lam_l3 = fdiv(mm3, hm3) + fsqrt(g * hm3);
                if (lam_l3 < R(0) && lam_r3 > R(0)) am[2] = fdiv(lam_l3 * (lam_r3 - s[2]), lam_r3 - lam_l3);
            }
        }
        for (int i = 0; i < 3; ++i) {
            amdq[i] = am[0] * W[0][i] + am[1] * W[1][i] + am[2] * W[2][i];
            apdq[i] = s[0] * W[0][i] + s[1] * W[1][i] + s[2] * W[2][i] - amdq[i];
        }
    }
};

// id, class template
#define CLAW_PLUGINS(X)          \
    X(16, BurgersPlugin)         \
    X(17, ShallowWaterPlugin)

#define CLAW_PLUGIN_MAP(id, P)                  \
    template <>                                 \
    struct PluginOf<id> {                       \
        template <typename R>                   \
        using type = P<R>;                      \
    };
CLAW_PLUGINS(CLAW_PLUGIN_MAP)
#undef CLAW_PLUGIN_MAP

}  // namespace claw
