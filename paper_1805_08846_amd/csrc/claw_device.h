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
// With the limited strength phi_p alpha_p and c_p = 1/2 |s_p| (1 - dt/dx |s_p|)
// the interface hands its left cell  L = A-dQ + F~ = sum (a_p alpha_p + c_p
// phi_p alpha_p) r_p and its right cell  R = A+dQ - F~ = sum (s_p alpha_p) r_p
// - L, and every cell is updated once: Q_k -= dt/dx (R_{k-1/2} + L_{k+1/2})
// (single-stage update, section 5.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace claw {

// Debug builds (compiled with CLAW_DEBUG, as libclaw_debug.so): every buffer
// load and store checks its byte range against the extent of the field it
// addresses, and the boundary index map checks the cell it resolves.  A
// failed check adds one to a device counter of its translation unit and
// records the source line of the first failure; the kernel then carries on as
// a release build would (a buffer access out of range reads zero and drops the
// store), so a wrong index shows up as a count instead of a silent zero.
// claw_debug_take reads and clears the counters.  Release builds compile the
// checks away.
#ifdef CLAW_DEBUG
typedef unsigned (*DebugTake)(unsigned* first_line);
void debug_register(DebugTake take);  // collects every translation unit's reader (runtime.hip)
namespace {
__device__ unsigned dbg_word[2];  // failed checks, source line of the first
__device__ __noinline__ void dbg_fail(unsigned line) {
    atomicAdd(&dbg_word[0], 1u);
    atomicCAS(&dbg_word[1], 0u, line);
}
unsigned dbg_take(unsigned* first_line) {
    unsigned w[2] = {0u, 0u};
    if (hipMemcpyFromSymbol(w, HIP_SYMBOL(dbg_word), sizeof w, 0, hipMemcpyDeviceToHost) != hipSuccess) return 0u;
    const unsigned z[2] = {0u, 0u};
    (void)hipMemcpyToSymbol(HIP_SYMBOL(dbg_word), z, sizeof z, 0, hipMemcpyHostToDevice);
    if (first_line) *first_line = w[1];
    return w[0];
}
struct DbgRegistrar {
    DbgRegistrar() { debug_register(dbg_take); }
};
DbgRegistrar dbg_registrar;
}  // namespace
#define CLAW_CHECK(cond)                              \
    do {                                              \
        if (!(cond)) ::claw::dbg_fail(__LINE__);      \
    } while (0)
#else
#define CLAW_CHECK(cond) \
    do {                 \
    } while (0)
#endif

enum { BC_EXTRAP = 0, BC_WALL = 1, BC_PERIODIC = 2 };
enum { LIM_MC = 0, LIM_NONE = 1, LIM_FIRST = 2, LIM_MINMOD = 3, LIM_SUPERBEE = 4, LIM_VANLEER = 5 };
// system kinds as compiled: constant-coefficient acoustics, acoustics with
// per-cell coefficients, shallow water; ids from SYS_PLUGIN up name
// point-wise solvers of the plug-in interface (plugins.h)
enum { SYS_AC = 0, SYS_ACV = 1, SYS_SW = 2, SYS_PLUGIN = 16 };
constexpr bool is_plugin(int sys) { return sys >= SYS_PLUGIN; }
// PluginOf<id>::type<R> is the plug-in class of id (specialised in plugins.h)
template <int SYS>
struct PluginOf;
template <typename R, int SYS>
using Plug = typename PluginOf<SYS>::template type<R>;

// Step state a trial step runs with.  The control block keeps one copy per
// trial parity: the first sweep of trial k decides trial k-1 from copy
// (k-1)&1 and the speed maxima of trial k-1, and writes the result to copy k&1
// for the remaining sweeps of trial k (section 4.1: the CFL number of the
// previous step decides accept / revert and the next time step).
struct StepState {
    double t;          // simulation time of the current state
    double dt;         // time step of this trial
    double dt_next;    // min(dt_max, cfl_desired / sigma) of the last decided trial
    double cfl;        // Courant number of the last decided trial
    double dtdx[3];    // dt / dx_d
    float dtdx_f[3];   // the same rounded once to FP32
    int32_t cur;       // rotation buffer holding the current state
    int32_t done;      // nonzero: the requested steps are complete (sweeps skip)
    int32_t err;       // claw_status of a failure that stopped the run
    int32_t last_accepted;
    int32_t pending;   // 1: this trial ran and is not decided yet
    int32_t mode;      // MODE_* of the trial
    int32_t result_off;  // buffer offset of the trial's result
    int32_t pad;
    long long accepted, rejected, target, consecutive, trials;
    long long base_accepted, base_rejected;  // counts when the current target was set
};

// Per parity and direction the largest |s| is kept in SMAX_SLOTS slots on
// separate 128-byte lines (a workgroup publishes into slot = its index mod
// SMAX_SLOTS), so workgroups that publish rising maxima one after another do
// not all serialise their atomics on one address; a decision takes the max
// over the slots.
constexpr int SMAX_SLOTS = 16;
struct alignas(128) SmaxSlot {
    unsigned long long v64;  // FP64 kernels: bits of max |s|
    unsigned int v32;        // FP32 kernels: bits of max |s|
    unsigned int pad[29];
};

// Device control block: step-control state that lives on the GPU so that a
// captured graph can run many steps without the host.
struct alignas(256) Ctrl {
    StepState st[2];
    SmaxSlot smax[2][4][SMAX_SLOTS];  // per parity, direction and slot
    int32_t nonphys[2];               // per parity: a sweep met depth <= 0 or NaN
    int32_t ndim;
    int32_t pad;
    double dx[3];
    double inv_dx[3];   // 1 / dx_d, so a decision costs one division
    double sweep_frac[3];  // fraction of dt each direction's sweeps take (Strang: 1/2 but the last)
    double cfl_desired, cfl_max, dt_max;
};

// Per-launch arguments of a sweep kernel (passed by value).  Element
// offsets fit in 32 bits (the runtime rejects larger grids).
template <typename R>
struct SweepArgs {
    R* buf[3];          // rotation buffers (buf[0] is the caller's q)
    const R* zc;        // derived coefficients: Z field then c field (SYS_ACV)
    Ctrl* ctrl;
    int32_t ncell;      // field stride
    int32_t nx;         // cells along x (the contiguous direction)
    int32_t m;          // cells along the sweep direction
    int32_t stride;     // element stride along the sweep direction
    int32_t nlines_o;   // column kernels: number of outer planes
    int32_t ostride;    // column kernels: element stride between outer planes
    int32_t nrows;      // row kernel: number of x-lines
    int32_t chunk;      // column kernels: cells along the sweep per wavefront
    int32_t dir;        // 0, 1, 2
    int32_t src_off;    // source buffer = (cur + src_off) % 3
    int32_t dst_off;    // destination buffer = (cur + dst_off) % 3
    int32_t bc_lo, bc_hi;
    int32_t limiter;
    int32_t efix;
    int32_t parity;     // trial parity: step-state copy and speed slots in use
    int32_t first;      // this sweep opens a trial (decides the previous one)
    int32_t last;       // this sweep closes a trial (clears the other parity's slots)
    int32_t auto_dt;    // speed pass of an adaptive start: skipped when the step
                        // state already holds a next step (dt_next > 0)
    R grav;
    R sqrt_grav;
    R Z0, c0;           // constant-coefficient acoustics
    R prm[4];           // plug-in solvers: the problem's parameters
};

// Row sweep geometry.  A wavefront covers 62 * cpl cells of a row (lanes 1..62;
// lanes 0 and 63 only supply halos).  The cells left at the end of every row
// (tail < 62 * cpl) are packed: one wavefront takes the tails of `rows` rows,
// each in a sub-segment of `width` lanes (its useful lanes plus two halo lanes),
// so short tails do not cost a whole wavefront per row.
struct RowTail {
    int width;
    int rows;
};
__host__ __device__ inline RowTail row_tail(int nx, int cpl) {
    const int seg = 62 * cpl;
    const int tail = nx - (nx / seg) * seg;
    RowTail t{64, 1};
    if (tail > 0) {
        t.width = (tail + cpl - 1) / cpl + 2;
        t.rows = 64 / t.width;
    }
    return t;
}

// A value every lane of the wavefront holds alike, moved into a scalar
// register (the compiler cannot prove that on its own for values read from
// memory or derived from the wavefront index): addresses built from it then
// stay scalar, and the per-lane part is a 32-bit offset.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float wave_uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// Buffer resource of one field: raw, byte addressed, offsets below 2^32 (the
// runtime keeps every field under 4 GiB).  A load or store then takes a
// per-lane byte offset and a scalar byte offset and costs no vector address
// arithmetic; the resource lives in scalar registers.
#ifdef CLAW_DEBUG
struct Rsrc {
    __amdgpu_buffer_rsrc_t r;
    unsigned bytes;
};
__device__ __forceinline__ Rsrc field_rsrc(const void* base, unsigned bytes) {
    return Rsrc{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000), bytes};
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t hw(Rsrc r) { return r.r; }
__device__ __forceinline__ void check_range(Rsrc r, unsigned voff, unsigned soff, unsigned size) {
    CLAW_CHECK((unsigned long long)voff + soff + size <= r.bytes);
}
#else
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc field_rsrc(const void* base, unsigned bytes) {
    // word 3: 32-bit data format, the value gfx9-family raw buffer access takes
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ Rsrc hw(Rsrc r) { return r; }
__device__ __forceinline__ void check_range(Rsrc, unsigned, unsigned, unsigned) {}
#endif
__device__ __forceinline__ float buf_load(Rsrc r, unsigned voff, unsigned soff, float) {
    check_range(r, voff, soff, 4);
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(hw(r), (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double buf_load(Rsrc r, unsigned voff, unsigned soff, double) {
    check_range(r, voff, soff, 8);
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(hw(r), (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_store(Rsrc r, unsigned voff, unsigned soff, float v) {
    check_range(r, voff, soff, 4);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), hw(r), (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_store(Rsrc r, unsigned voff, unsigned soff, double v) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    check_range(r, voff, soff, 8);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), hw(r), (int)voff, (int)soff, 0);
}

// 16-byte vector loads and stores through a field resource (a row lane's
// cells: four FP32 or two FP64 values).
typedef unsigned U4 __attribute__((ext_vector_type(4)));
template <typename V>
__device__ __forceinline__ V buf_load16(Rsrc r, unsigned voff) {
    static_assert(sizeof(V) == 16, "16-byte vectors only");
    check_range(r, voff, 0, 16);
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(hw(r), (int)voff, 0, 0));
}
template <typename V>
__device__ __forceinline__ void buf_store16(Rsrc r, unsigned voff, V v) {
    static_assert(sizeof(V) == 16, "16-byte vectors only");
    check_range(r, voff, 0, 16);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), hw(r), (int)voff, 0, 0);
}

// Rotation buffer i (0..2) chosen by selects rather than by indexing the
// array: a dynamic index into a SweepArgs held in registers would force the
// whole struct into private memory.
template <typename R>
__device__ __forceinline__ R* pick_buf(const SweepArgs<R>& a, int i) {
    return i == 0 ? a.buf[0] : (i == 1 ? a.buf[1] : a.buf[2]);
}

// ---------------------------------------------------------------------------
// Precision helpers.  FP64 divisions and square roots off the hot path (the
// entropy fix's transonic branch, plug-in solvers) are correctly rounded; the
// hot path's reciprocals and reciprocal square roots are Newton-refined
// hardware approximations.  FP32 uses the hardware reciprocal and square root
// (about 1 ulp).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ double fsqrt(double a) { return __builtin_sqrt(a); }
// FP64 reciprocal and reciprocal square root on the hot path: the hardware
// approximations refined by two Newton-Raphson steps (each about doubles the
// correct bits), within a few ulp instead of correctly rounded, for a
// fraction of the instructions of IEEE division and square root.
__device__ __forceinline__ double frcp(double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ double frsq(double a) {
    double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    y = y * __builtin_fma(-h * y, y, 1.5);  // y (3 - a y^2) / 2
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y;
}
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float frcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ float fsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ float frsq(float a) { return __builtin_amdgcn_rsqf(a); }

// min / max / abs as single VALU instructions (operands are never NaN on the
// paths that use them; a NaN state is caught by the depth check)
__device__ __forceinline__ float rmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float rmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ float rabs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ float rsign1(float a) { return __builtin_copysignf(1.0f, a); }
__device__ __forceinline__ double rmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double rmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double rabs(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ double rsign1(double a) { return __builtin_copysign(1.0, a); }

// Source index of cell i along a line of m cells under the boundary rules;
// only -2 <= i <= m + 1 matter, other indices are clamped into that range
// first.  flip = the normal component changes sign (wall).
__device__ __forceinline__ int ghost_idx_of(int i, int m, int bc_lo, int bc_hi, bool& flip) {
    i = i < -2 ? -2 : (i > m + 1 ? m + 1 : i);
    flip = false;
    if (i < 0) {
        if (bc_lo == BC_WALL) {
            flip = true;
            int r = -1 - i;
            return r > m - 1 ? m - 1 : r;
        }
        if (bc_lo == BC_PERIODIC) {
            int r = i + m;
            return r < 0 ? r + m : r;
        }
        return 0;
    }
    if (i >= m) {
        if (bc_hi == BC_WALL) {
            flip = true;
            int r = 2 * m - 1 - i;
            return r < 0 ? 0 : r;
        }
        if (bc_hi == BC_PERIODIC) {
            int r = i - m;
            return r >= m ? r - m : r;
        }
        return m - 1;
    }
    return i;
}
__device__ __forceinline__ int ghost_idx(int i, int m, int bc_lo, int bc_hi, bool& flip) {
    const int r = ghost_idx_of(i, m, bc_lo, bc_hi, flip);
    CLAW_CHECK(r >= 0 && r < m);
    return r;
}

// ---------------------------------------------------------------------------
// Cells and interfaces
// ---------------------------------------------------------------------------
// Plug-in systems: the fields in the sweep's normal frame.
template <typename R, int SYS>
struct Cell {
    R q[Plug<R, SYS>::MEQN];
};

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
__device__ __forceinline__ void sw_cell_derive(double h, double sg, double& ih, double& sqh, double& c) {
    const double r = frsq(h);  // 1/sqrt(h): sqrt(h) = h r, 1/h = r r
    ih = r * r;
    sqh = h * r;
    c = sg * sqh;
}
__device__ __forceinline__ void sw_cell_derive(float h, float sg, float& ih, float& sqh, float& c) {
    float r = frsq(h);  // 1/sqrt(h): sqrt(h) = h r, 1/h = r r
    ih = r * r;
    sqh = h * r;
    c = sg * sqh;
}
template <typename R>
struct Cell<R, SYS_SW> {
    R h, mn, mt;
    R u, v, sqh, c;
    __device__ void derive(R sg, bool& bad) {
        bool ok = h > R(0);  // false for NaN too
        bad = bad || !ok;
        R hh = ok ? h : R(1);
        R ih;
        sw_cell_derive(hh, sg, ih, sqh, c);
        u = mn * ih;
        v = mt * ih;
    }
};

// Built-in systems: the compact wave form above.
template <typename R, int NW>
struct CompactIface {
    static constexpr int MW = NW;
    R alpha[MW];
    R s[MW];
    R am[MW];  // left-going speed share a_p
    R e0, e1;
};
// Plug-in systems: full waves, speeds and fluctuations as the solver returns them.
template <typename R, int SYS>
struct Iface {
    static constexpr int MW = Plug<R, SYS>::MWAVES;
    static constexpr int ME = Plug<R, SYS>::MEQN;
    R W[MW][ME];
    R s[MW];
    R amdq[ME];
    R apdq[ME];
};
template <typename R>
struct Iface<R, SYS_AC> : CompactIface<R, 2> {};
template <typename R>
struct Iface<R, SYS_ACV> : CompactIface<R, 2> {};
template <typename R>
struct Iface<R, SYS_SW> : CompactIface<R, 3> {};

template <typename R>
__device__ __forceinline__ void riemann(const Cell<R, SYS_AC>& l, const Cell<R, SYS_AC>& r,
                                        R Z, R c, R inv2Z, R, int, Iface<R, SYS_AC>& o) {
    R dp = r.p - l.p;
    R du = r.un - l.un;
    o.alpha[0] = (-dp + Z * du) * inv2Z;
    o.alpha[1] = (dp + Z * du) * inv2Z;
    o.s[0] = -c;
    o.s[1] = c;
    o.am[0] = -c;
    o.am[1] = R(0);
    o.e0 = Z;
    o.e1 = Z;
}

template <typename R>
__device__ __forceinline__ void riemann(const Cell<R, SYS_ACV>& l, const Cell<R, SYS_ACV>& r,
                                        R, R, R, R, int, Iface<R, SYS_ACV>& o) {
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

// Roe speed of sound c^ = sqrt(g hbar) and 1 / (2 c^)
__device__ __forceinline__ void roe_c(double x, double& c, double& i2c) {
    const double r = frsq(x);
    c = x * r;
    i2c = 0.5 * r;
}
__device__ __forceinline__ void roe_c(float x, float& c, float& i2c) {
    float r = frsq(x);
    c = x * r;
    i2c = 0.5f * r;
}

// Roe solver with arithmetic-mean depth and sqrt(h)-weighted velocities plus
// the Harten-Hyman entropy fix on the 1- and 3-waves.  The transonic test of
// the fix, lambda_r = m/h - sqrt(g h) > 0 in the middle state, is taken as
// h > 0, m > 0 and m^2 > g h^3 so that the division and square root are only
// paid in the (rare) transonic case; the split it selects is continuous
// across the test's boundary.  A middle state of depth <= 0 takes no fix.
template <typename R>
__device__ __forceinline__ void riemann(const Cell<R, SYS_SW>& l, const Cell<R, SYS_SW>& r,
                                        R, R, R, R g, int efix, Iface<R, SYS_SW>& o) {
    R inv = frcp(l.sqh + r.sqh);
    R uhat = (l.sqh * l.u + r.sqh * r.u) * inv;
    R vhat = (l.sqh * l.v + r.sqh * r.v) * inv;
    R chat, i2c;
    roe_c((l.h + r.h) * (R(0.5) * g), chat, i2c);  // c^2 = g hbar, hbar = (h_l + h_r) / 2
    R dh = r.h - l.h;
    R dn = r.mn - l.mn;
    R dt = r.mt - l.mt;
    R s1 = uhat - chat;
    R s3 = uhat + chat;
    R a1 = (s3 * dh - dn) * i2c;
    R a2 = dt - vhat * dh;
    R a3 = (dn - s1 * dh) * i2c;
    R am1 = rmin(s1, R(0));
    R am3 = rmin(s3, R(0));
    if (efix) {
        // lambda_l = u_l - c_l < 0 is u_l < c_l; lambda_r3 = u_r + c_r > 0 is
        // u_r > -c_r (the differences are only formed in the transonic case)
        R hm = l.h + a1;
        R mm = l.mn + a1 * s1;
        if (l.u < l.c && hm > R(0) && mm > R(0) && mm * mm > g * hm * hm * hm) {
            R lam_l = l.u - l.c;
            R lam_r = fdiv(mm, hm) - fsqrt(g * hm);
            if (lam_r > R(0)) am1 = fdiv(lam_l * (lam_r - s1), lam_r - lam_l);
        }
        R hm3 = r.h - a3;
        R mm3 = r.mn - a3 * s3;
        if (r.u > -r.c && hm3 > R(0) && mm3 < R(0) && mm3 * mm3 > g * hm3 * hm3 * hm3) {
            R lam_r3 = r.u + r.c;
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

// Largest |s| of an interface (shallow water: |u^| <= max(|u^ - c^|, |u^ + c^|)).
template <typename R>
__device__ __forceinline__ R iface_smax(const Iface<R, SYS_SW>& k) {
    return rmax(rabs(k.s[0]), rabs(k.s[2]));
}
template <typename R, int SYS>
__device__ __forceinline__ R iface_smax(const Iface<R, SYS>& k) {
    if constexpr (is_plugin(SYS)) {
        R m = rabs(k.s[0]);
#pragma unroll
        for (int p = 1; p < Iface<R, SYS>::MW; ++p) m = rmax(m, rabs(k.s[p]));
        return m;
    } else {
        return rmax(rabs(k.s[0]), rabs(k.s[1]));
    }
}

// Half the limited wave strength, phi(theta) alpha / 2, of the MC limiter
// without forming theta = beta / alpha, beta = n / |r|^2 (n = alpha_up (r_up .
// r), the projection of the upwind wave).  phi(theta) alpha equals the
// minmod of the three values (alpha + beta) / 2, 2 alpha, 2 beta (all of one
// sign: the one nearest zero; else 0) in real arithmetic, and vanishes with
// alpha; halved, that is minmod((alpha + beta) / 4, alpha, beta).  In FP32 a
// two-value minmod is med3(x, y, 0), so the whole limiter is two v_med3_f32.
__device__ __forceinline__ float mc_half(float alpha, float beta) {
    const float m = __builtin_amdgcn_fmed3f(alpha, beta, 0.0f);
    return __builtin_amdgcn_fmed3f(0.25f * (alpha + beta), m, 0.0f);
}
__device__ __forceinline__ double mc_half(double alpha, double beta) {
    const double sg = rsign1(alpha);
    const double a = rabs(alpha);
    const double b = sg * beta;
    return sg * rmax(0.0, rmin(0.25 * (a + b), rmin(a, b)));
}

// phi(theta) * alpha for the other limiters, with a = |alpha| and b = theta |alpha|
// (theta never formed): minmod max(0, min(a, b)); superbee
// max(0, min(a, 2b), min(2a, b)); van Leer (b + |b|) a / (a + |b|).  The
// limiter is uniform, so callers branch once per interface and MC keeps its
// straight-line path.
template <typename R>
__device__ __forceinline__ R wave_limited(R alpha, R n_over_r2, int lim) {
    const R sg = rsign1(alpha);
    const R a = rabs(alpha);
    const R b = sg * n_over_r2;
    R m;
    if (lim == LIM_MINMOD) {
        m = rmax(R(0), rmin(a, b));
    } else if (lim == LIM_SUPERBEE) {
        m = rmax(R(0), rmax(rmin(a, b + b), rmin(a + a, b)));
    } else {  // van Leer
        const R ab = rabs(b);
        const R den = a + ab;
        m = den > R(0) ? (b + ab) * a * frcp(den) : R(0);
    }
    return sg * m;
}

// Output of one limited interface: contributions to its left and right cell
// in the interface's normal frame.  Shallow water: (h, m_n, m_t); acoustics:
// (p, u_n) in slots 0, 1; plug-ins: their MEQN fields.
template <typename R, int N = 3>
struct Contrib {
    R L[N];
    R Rr[N];
};
template <int SYS>
constexpr int contrib_width() {
    if constexpr (is_plugin(SYS)) return Plug<float, SYS>::MEQN;
    else return 3;
}

// phi(theta) of a limiter for theta = n / d (d = |W|^2 > 0), the classical
// forms (LeVeque 2002, section 6.12); used by plug-in systems, whose waves
// are general vectors.
template <typename R>
__device__ __forceinline__ R phi_of_ratio(R n, R d, int lim) {
    if (!(d > R(0))) return R(0);  // a wave of zero length has no correction
    const R th = fdiv(n, d);
    if (lim == LIM_MC) return rmax(R(0), rmin(R(0.5) * (R(1) + th), rmin(R(2), th + th)));
    if (lim == LIM_MINMOD) return rmax(R(0), rmin(R(1), th));
    if (lim == LIM_SUPERBEE) return rmax(R(0), rmax(rmin(R(1), th + th), rmin(R(2), th)));
    if (lim == LIM_VANLEER) {
        const R a = rabs(th);
        return fdiv(th + a, R(1) + a);
    }
    return R(1);  // LIM_NONE
}

// Plug-in interface k with neighbours km, kp: L = A-dQ + F~, Rr = A+dQ - F~.
template <typename R, int SYS, int N>
__device__ __forceinline__ void plugin_contrib(const Iface<R, SYS>& k, const Iface<R, SYS>& km,
                                               const Iface<R, SYS>& kp, R nu, int limiter,
                                               Contrib<R, N>& out) {
    constexpr int MW = Iface<R, SYS>::MW, ME = Iface<R, SYS>::ME;
    static_assert(N == ME, "contribution width is the plug-in's field count");
#pragma unroll
    for (int i = 0; i < ME; ++i) {
        out.L[i] = k.amdq[i];
        out.Rr[i] = k.apdq[i];
    }
    if (limiter == LIM_FIRST) return;
#pragma unroll
    for (int p = 0; p < MW; ++p) {
        const bool right = k.s[p] > R(0);  // upwind interface: k - 1 for s > 0, else k + 1
        R d = R(0), n = R(0);
#pragma unroll
        for (int i = 0; i < ME; ++i) {
            const R w = k.W[p][i];
            d += w * w;
            n += (right ? km.W[p][i] : kp.W[p][i]) * w;
        }
        const R phi = limiter == LIM_NONE ? R(1) : phi_of_ratio(n, d, limiter);
        const R as = rabs(k.s[p]);
        const R cw = R(0.5) * as * (R(1) - nu * as) * phi;
#pragma unroll
        for (int i = 0; i < ME; ++i) {
            const R f = cw * k.W[p][i];
            out.L[i] += f;
            out.Rr[i] -= f;
        }
    }
}

// Half the limited wave strengths, phi_p alpha_p / 2, of interface k given
// its neighbours km (k - 1) and kp (k + 1).
template <typename R>
__device__ __forceinline__ R half_limited(R alpha, R beta, int limiter) {
    if (limiter == LIM_MC) return mc_half(alpha, beta);
    return R(0.5) * wave_limited(alpha, beta, limiter);
}
template <typename R>
__device__ __forceinline__ void limited(const Iface<R, SYS_SW>& k, const Iface<R, SYS_SW>& km,
                                        const Iface<R, SYS_SW>& kp, int limiter, R (&w)[3]) {
    if (limiter == LIM_NONE) {
        w[0] = R(0.5) * k.alpha[0];
        w[1] = R(0.5) * k.alpha[1];
        w[2] = R(0.5) * k.alpha[2];
        return;
    }
    // |r_1|^2 and |r_3|^2 share one reciprocal
    const R r1 = R(1) + k.s[0] * k.s[0] + k.e0 * k.e0;
    const R r3 = R(1) + k.s[2] * k.s[2] + k.e0 * k.e0;
    const R t = frcp(r1 * r3);
    const R ir1 = t * r3, ir3 = t * r1;
    // upwind neighbour by the sign of each speed
    const bool p1 = k.s[0] > R(0), p2 = k.s[1] > R(0), p3 = k.s[2] > R(0);
    const R a1u = p1 ? km.alpha[0] : kp.alpha[0];
    const R s1u = p1 ? km.s[0] : kp.s[0];
    const R v1u = p1 ? km.e0 : kp.e0;
    const R a3u = p3 ? km.alpha[2] : kp.alpha[2];
    const R s3u = p3 ? km.s[2] : kp.s[2];
    const R v3u = p3 ? km.e0 : kp.e0;
    const R a2u = p2 ? km.alpha[1] : kp.alpha[1];
    const R n1 = a1u * (R(1) + s1u * k.s[0] + v1u * k.e0);
    const R n3 = a3u * (R(1) + s3u * k.s[2] + v3u * k.e0);
    w[0] = half_limited(k.alpha[0], n1 * ir1, limiter);
    w[1] = half_limited(k.alpha[1], a2u, limiter);
    w[2] = half_limited(k.alpha[2], n3 * ir3, limiter);
}

// Acoustics: wave 1 moves left (upwind neighbour k + 1), wave 2 right (k - 1).
template <typename R>
__device__ __forceinline__ void limited(const Iface<R, SYS_AC>& k, const Iface<R, SYS_AC>& km,
                                        const Iface<R, SYS_AC>& kp, int limiter, R (&w)[2]) {
    if (limiter == LIM_NONE) {
        w[0] = R(0.5) * k.alpha[0];
        w[1] = R(0.5) * k.alpha[1];
        return;
    }
    // constant coefficients: r_p is the same at every interface
    w[0] = half_limited(k.alpha[0], kp.alpha[0], limiter);
    w[1] = half_limited(k.alpha[1], km.alpha[1], limiter);
}
template <typename R>
__device__ __forceinline__ void limited(const Iface<R, SYS_ACV>& k, const Iface<R, SYS_ACV>& km,
                                        const Iface<R, SYS_ACV>& kp, int limiter, R (&w)[2]) {
    if (limiter == LIM_NONE) {
        w[0] = R(0.5) * k.alpha[0];
        w[1] = R(0.5) * k.alpha[1];
        return;
    }
    // r_1 = (-Z_l, 1), r_2 = (Z_r, 1)
    const R r1 = R(1) + k.e0 * k.e0;
    const R r2 = R(1) + k.e1 * k.e1;
    const R t = frcp(r1 * r2);
    const R n1 = kp.alpha[0] * (R(1) + kp.e0 * k.e0);
    const R n2 = km.alpha[1] * (R(1) + km.e1 * k.e1);
    w[0] = half_limited(k.alpha[0], n1 * (t * r2), limiter);
    w[1] = half_limited(k.alpha[1], n2 * (t * r1), limiter);
}

// Limits interface k and forms its contributions to the left cell
// (A-dQ + F~) and the right cell (A+dQ - F~).  nu = dt / dx.
template <typename R, int SYS, int N>
__device__ __forceinline__ void compact_contrib(const Iface<R, SYS>& k, const Iface<R, SYS>& km,
                                                const Iface<R, SYS>& kp, R nu, int limiter,
                                                Contrib<R, N>& out) {
    constexpr int MW = Iface<R, SYS>::MW;
    R w[MW];
    if (limiter == LIM_FIRST) {
#pragma unroll
        for (int p = 0; p < MW; ++p) w[p] = R(0);
    } else {
        limited(k, km, kp, limiter, w);
    }
    // w holds phi_p alpha_p / 2, so the F~ share of wave p is
    // |s| (1 - nu |s|) w = (|s| - nu |s| |s|) w; the left share adds the A-dQ
    // share a_p alpha_p, and the right share is the rest of s_p alpha_p.
    R kl[MW], kr[MW];
#pragma unroll
    for (int p = 0; p < MW; ++p) {
        const R sp = k.s[p];
        const R as = rabs(sp);
        const R cw = (as - (nu * as) * as) * w[p];
        kl[p] = k.am[p] * k.alpha[p] + cw;
        kr[p] = sp * k.alpha[p] - kl[p];
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

template <typename R, int SYS, int N>
__device__ __forceinline__ void limit_contrib(const Iface<R, SYS>& k, const Iface<R, SYS>& km,
                                              const Iface<R, SYS>& kp, R nu, int limiter,
                                              Contrib<R, N>& out) {
    if constexpr (is_plugin(SYS)) plugin_contrib(k, km, kp, nu, limiter, out);
    else compact_contrib(k, km, kp, nu, limiter, out);
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
// DPP wave shifts: lane_prev gives lane i the value of lane i - 1, lane_next
// the value of lane i + 1 (lane 0 / lane 63 receive 0).
__device__ __forceinline__ int dpp_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_shl1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(dpp_shr1(__float_as_int(v))); }
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(dpp_shl1(__float_as_int(v))); }
__device__ __forceinline__ double lane_prev(double v) {
    return __hiloint2double(dpp_shr1(__double2hiint(v)), dpp_shr1(__double2loint(v)));
}
__device__ __forceinline__ double lane_next(double v) {
    return __hiloint2double(dpp_shl1(__double2hiint(v)), dpp_shl1(__double2loint(v)));
}

// neighbour data a limiter needs: strengths, speeds and eigenvector numbers
template <typename R, int SYS>
__device__ __forceinline__ void iface_prev(const Iface<R, SYS>& in, Iface<R, SYS>& out) {
    if constexpr (is_plugin(SYS)) {
#pragma unroll
        for (int p = 0; p < Iface<R, SYS>::MW; ++p) {
            out.s[p] = lane_prev(in.s[p]);
#pragma unroll
            for (int i = 0; i < Iface<R, SYS>::ME; ++i) out.W[p][i] = lane_prev(in.W[p][i]);
        }
    } else {
#pragma unroll
        for (int p = 0; p < Iface<R, SYS>::MW; ++p) {
            out.alpha[p] = lane_prev(in.alpha[p]);
            if constexpr (SYS == SYS_SW) out.s[p] = lane_prev(in.s[p]);
        }
        if constexpr (SYS != SYS_AC) out.e0 = lane_prev(in.e0);
        if constexpr (SYS == SYS_ACV) out.e1 = lane_prev(in.e1);
    }
}
template <typename R, int SYS>
__device__ __forceinline__ void iface_next(const Iface<R, SYS>& in, Iface<R, SYS>& out) {
    if constexpr (is_plugin(SYS)) {
#pragma unroll
        for (int p = 0; p < Iface<R, SYS>::MW; ++p) {
            out.s[p] = lane_next(in.s[p]);
#pragma unroll
            for (int i = 0; i < Iface<R, SYS>::ME; ++i) out.W[p][i] = lane_next(in.W[p][i]);
        }
    } else {
#pragma unroll
        for (int p = 0; p < Iface<R, SYS>::MW; ++p) {
            out.alpha[p] = lane_next(in.alpha[p]);
            if constexpr (SYS == SYS_SW) out.s[p] = lane_next(in.s[p]);
        }
        if constexpr (SYS != SYS_AC) out.e0 = lane_next(in.e0);
        if constexpr (SYS == SYS_ACV) out.e1 = lane_next(in.e1);
    }
}

__device__ __forceinline__ float lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Wavefront maximum of non-negative values (speeds): DPP prefix maxima within
// each 16-lane row (shifts 1, 2, 4, 8), then row broadcasts 15 and 31, which
// leave the maximum in lane 63.  Lanes without a source read 0, the identity
// of max on non-negative values.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
// FP32: non-negative values order like their bit patterns, so an unsigned
// integer max does it (no canonicalising of the float operands)
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_max_step(float v) {
    const unsigned a = (unsigned)__float_as_int(v);
    const unsigned b = (unsigned)dpp_move<CTRL, ROWS>(__float_as_int(v));
    return __int_as_float((int)(a > b ? a : b));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_max_step(double v) {
    const double o = __hiloint2double(dpp_move<CTRL, ROWS>(__double2hiint(v)),
                                      dpp_move<CTRL, ROWS>(__double2loint(v)));
    return rmax(v, o);
}
template <typename R>
__device__ __forceinline__ R wave_max(R v) {
    v = dpp_max_step<0x111, 0xf>(v);  // row_shr:1
    v = dpp_max_step<0x112, 0xf>(v);  // row_shr:2
    v = dpp_max_step<0x114, 0xf>(v);  // row_shr:4
    v = dpp_max_step<0x118, 0xf>(v);  // row_shr:8
    v = dpp_max_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return lane63(v);
}

// Per-direction speed maximum: non-negative IEEE values order like their bit
// patterns, so an unsigned atomic max is exact and order independent.  A
// cached read first skips the atomic when a larger value is already known
// (a stale read only costs an unneeded atomic).
__device__ __forceinline__ void publish_smax(Ctrl* c, int par, int dir, int slot, float v) {
    const unsigned bits = __float_as_uint(v);
    unsigned* p = &c->smax[par][dir][slot].v32;
    if (bits > __atomic_load_n(p, __ATOMIC_RELAXED)) atomicMax(p, bits);
}
__device__ __forceinline__ void publish_smax(Ctrl* c, int par, int dir, int slot, double v) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    unsigned long long* p = &c->smax[par][dir][slot].v64;
    if (bits > __atomic_load_n(p, __ATOMIC_RELAXED)) atomicMax(p, bits);
}
// slot of the calling workgroup
__device__ __forceinline__ int smax_slot() {
    return (int)((blockIdx.x + blockIdx.y + blockIdx.z) % SMAX_SLOTS);
}
// max |s| of parity q, direction d over the slots (bits of a non-negative value)
__device__ __forceinline__ unsigned smax32_of(const Ctrl* c, int q, int d) {
    unsigned m = 0u;
    for (int k = 0; k < SMAX_SLOTS; ++k) m = c->smax[q][d][k].v32 > m ? c->smax[q][d][k].v32 : m;
    return m;
}
__device__ __forceinline__ unsigned long long smax64_of(const Ctrl* c, int q, int d) {
    unsigned long long m = 0ull;
    for (int k = 0; k < SMAX_SLOTS; ++k) m = c->smax[q][d][k].v64 > m ? c->smax[q][d][k].v64 : m;
    return m;
}
// zeroes the speed slots of parity q (one thread)
__device__ __forceinline__ void clear_speeds(Ctrl* c, int q) {
    for (int d = 0; d < 4; ++d)
        for (int k = 0; k < SMAX_SLOTS; ++k) {
            c->smax[q][d][k].v32 = 0u;
            c->smax[q][d][k].v64 = 0ull;
        }
}

template <typename R>
__device__ __forceinline__ R state_nu(const StepState& s, int dir);
template <>
__device__ __forceinline__ float state_nu<float>(const StepState& s, int dir) {
    return dir == 0 ? s.dtdx_f[0] : (dir == 1 ? s.dtdx_f[1] : s.dtdx_f[2]);
}
template <>
__device__ __forceinline__ double state_nu<double>(const StepState& s, int dir) {
    return dir == 0 ? s.dtdx[0] : (dir == 1 ? s.dtdx[1] : s.dtdx[2]);
}

enum { MODE_ADAPT = 0, MODE_STEP = 1, MODE_FIXED = 2 };

// ---------------------------------------------------------------------------
// Step control (section 4.1; equation CFL-condition): Courant number from the
// per-direction speed maxima, accept or revert, next trial step.  decide() is
// a pure function of the control block, evaluated identically by every
// wavefront of the sweep that opens the next trial (and by a one-thread
// commit kernel at the end of a host call).  It multiplies by 1/dx instead of
// dividing by dx (a last-bit difference in sigma and dt/dx) so that the
// decision costs one FP64 division.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void set_trial_dt(const Ctrl* c, StepState& s, double dt) {
    s.dt = dt;
    for (int d = 0; d < 3; ++d) {
        const double v = d < c->ndim ? dt * c->inv_dx[d] * c->sweep_frac[d] : 0.0;
        s.dtdx[d] = v;
        s.dtdx_f[d] = (float)v;
    }
}

__device__ __forceinline__ double sigma_of(const Ctrl* c, int q, bool fp32) {
    double sigma = 0.0;
    for (int d = 0; d < c->ndim; ++d) {
        const double sm = fp32 ? (double)__uint_as_float(smax32_of(c, q, d))
                               : __longlong_as_double((long long)smax64_of(c, q, d));
        const double v = sm * c->inv_dx[d];
        if (v > sigma) sigma = v;
    }
    return sigma;
}

// next trial step min(dt_max, cfl_desired / sigma); false if none exists
__device__ __forceinline__ bool next_dt(const Ctrl* c, double sigma, double* dt) {
    if (sigma > 0.0) {
        const double v = c->cfl_desired / sigma;
        *dt = v < c->dt_max ? v : c->dt_max;
        return true;
    }
    if (__builtin_isfinite(c->dt_max)) {
        *dt = c->dt_max;
        return true;
    }
    return false;
}

// N = state after deciding the trial recorded in copy q (unchanged if none pending).
__device__ __forceinline__ void decide(const Ctrl* c, int q, bool fp32, StepState& N) {
    N = c->st[q];
    if (!N.pending) return;
    N.pending = 0;
    if (N.done) return;
    const double sigma = sigma_of(c, q, fp32);
    const double cfl = N.dt * sigma;
    N.cfl = cfl;
    N.trials += 1;
    if (c->nonphys[q]) {  // the state stays Q^n
        N.err = 5;
        N.done = 1;
        N.last_accepted = 0;
        N.rejected += 1;
        return;
    }
    const bool accept = N.mode == MODE_FIXED ? true : (cfl <= c->cfl_max);
    if (accept) {
        N.cur = (N.cur + N.result_off) % 3;
        N.t += N.dt;
        N.accepted += 1;
        N.consecutive = 0;
    } else {
        N.rejected += 1;
        N.consecutive += 1;
        if (N.consecutive > 64) {
            N.err = 6;
            N.done = 1;
        }
    }
    N.last_accepted = accept ? 1 : 0;
    double dtn = 0.0;
    if (!next_dt(c, sigma, &dtn)) {
        N.err = 6;
        N.done = 1;
        return;
    }
    N.dt_next = dtn;
    if (N.mode == MODE_ADAPT) {
        set_trial_dt(c, N, dtn);
        if (N.accepted >= N.target) N.done = 1;
    }
}

// What a sweep needs of its trial: buffer index, skip flag, dt/dx.
template <typename R>
struct Trial {
    int cur;
    int done;
    R nu;
};

// Buffer index a trial will use if the previous trial is accepted (or the
// committed one if nothing is pending): readable before the decision.
template <typename R>
__device__ __forceinline__ int predicted_cur(const SweepArgs<R>& a) {
    if (!a.first) return wave_uniform(a.ctrl->st[a.parity].cur);
    const StepState& P = a.ctrl->st[a.parity ^ 1];
    return wave_uniform((P.pending && !P.done) ? (P.cur + P.result_off) % 3 : P.cur);
}

// lead: this workgroup is block (0, 0, 0) of its grid (it records the state).
template <typename R>
__device__ __forceinline__ Trial<R> open_trial(const SweepArgs<R>& a, int dir, bool lead) {
    Ctrl* c = a.ctrl;
    Trial<R> t;
    if (a.first) {
        StepState S;
        decide(c, a.parity ^ 1, sizeof(R) == 4, S);
        if (lead && threadIdx.x == 0) {
            S.pending = S.done ? 0 : 1;
            c->st[a.parity] = S;
        }
        t.cur = S.cur;
        t.done = S.done;
        t.nu = state_nu<R>(S, dir);
    } else {
        const StepState& S = c->st[a.parity];
        t.cur = S.cur;
        t.done = S.done;
        t.nu = state_nu<R>(S, dir);
    }
    // every lane read or decided the same step state
    t.cur = wave_uniform(t.cur);
    t.done = wave_uniform(t.done);
    t.nu = wave_uniform(t.nu);
    return t;
}

// Block-wide max of v published once per workgroup (blockDim.x a multiple of
// 64) into the trial's speed slot; the sweep that closes a trial also clears
// the other parity's slots for the trial after next.
template <typename R>
__device__ __forceinline__ void block_finish(const SweepArgs<R>& a, int dir, R v, bool bad, bool lead) {
    __shared__ R red[16];
    __shared__ int redbad[16];
    Ctrl* c = a.ctrl;
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
        publish_smax(c, a.parity, dir, smax_slot(), m);
        if (b) atomicOr(&c->nonphys[a.parity], 1);
        if (a.last && lead) {
            const int o = a.parity ^ 1;
            clear_speeds(c, o);
            c->nonphys[o] = 0;
        }
    }
}

}  // namespace claw

#include "plugins.h"
