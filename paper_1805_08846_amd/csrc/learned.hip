// learned.hip -- the learned coarse-grid flux correction: a 12-64-64-3 ReLU
// network evaluated on every interior interface of a shallow-water grid with
// BF16 matrix-core products (FP32 accumulation), its fused forward/backward
// pass for training, Adam on FP32 master weights, the fallback and conservative
// application of the corrections, and the 2 x 2 coarsening of a fine state.
//
// The correction enters the update only as a flux difference, like every flux
// of the method's conservative update (section 3, equation LW-update):
//   Q^{n+1} = S(Q^n) - nu_x (dF_{i+1/2} - dF_{i-1/2}) - nu_y (dG_{j+1/2} - dG_{j-1/2})
// with S the plain split step; wall faces carry no correction, so every
// field's sum changes by rounding only.
//
// Interface frame: a face along direction d sees (h, m_n, m_t) = depth,
// momentum along d, momentum across d; stencil cells k-2 .. k+1 around face
// k - 1/2, mirrored across a wall with m_n negated.  Features per channel c
// (level, slope, curvature, third difference, each over its own scale):
// ((b + e)/2 - mu_c)/sl_c, (e - b)/sd1_c, ((a + f) - (b + e))/sd2_c,
// ((f - a) - 3 (e - b))/sd3_c, formed in FP64 before the rounding to BF16.
//
// Matrix-core layout (v_mfma_f32_16x16x16_bf16, 64 lanes, lane = n + 16 kb):
//   A[i][k]  lane i + 16 (k/4), element k%4
//   B[k][j]  lane j + 16 (k/4), element k%4
//   D[i][j]  lane j + 16 (i/4), element i%4
// The network runs transposed, Z^T = W Z_prev^T, with 16 faces as the N
// dimension: the D tile of a layer is then exactly the B operand of the next
// layer, so activations never leave registers.  Weight gradients need the
// faces on the K dimension and go through a per-wavefront LDS transpose.
//
// The forward pass takes gfx950's v_mfma_f32_16x16x32_bf16 for the two
// 64-wide products: a lane holds 8 K values.  Lane group kb joins the D
// elements of two consecutive 16-unit tiles, so K block s (units 32 s ..
// 32 s + 31) gives lane group kb units 32 s + 4 kb + {0..3} and
// 32 s + 16 + 4 kb + {0..3}; the weight operands use the same K order (a
// product sums over K, any order shared by both operands gives the same
// sum).  The BF16 weight copies are stored in exactly these operand layouts
// (w1_slot, w2_slot, w3_slot), so every lane loads its operands with 8- and
// 16-byte loads.
#include "claw_launch.h"

namespace claw {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 hbf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(hbf16x8, a), __builtin_bit_cast(hbf16x8, b),
                                                   c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 join(bf16x4 lo, bf16x4 hi) {
    return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// Slots of the BF16 operand copies (one network): W1 as the A operand of
// the 16x16x16 product per unit tile t, W2 and W3 as the A operands of the
// 16x16x32 products per unit tile t and K block s.  Slots no weight maps to
// (features 12 .. 15, output rows 3 .. 15) hold zeros.
__device__ __forceinline__ int kblock_lane(int v, int& e) {  // unit v within its K block -> lane group, element
    const int w = v & 31;
    e = (w & 3) + (w & 16 ? 4 : 0);
    return (w & 15) >> 2;
}
__device__ __forceinline__ int w1_slot(int u, int f) {
    return ((u >> 4) * 64 + (u & 15) + 16 * (f >> 2)) * 4 + (f & 3);
}
__device__ __forceinline__ int w2_slot(int u, int v) {
    int e;
    const int kb = kblock_lane(v, e);
    return (((u >> 4) * 2 + (v >> 5)) * 64 + (u & 15) + 16 * kb) * 8 + e;
}
__device__ __forceinline__ int w3_slot(int o, int v) {
    int e;
    const int kb = kblock_lane(v, e);
    return ((v >> 5) * 64 + o + 16 * kb) * 8 + e;
}

// FP32 -> BF16, round to nearest even (gfx950's v_cvt_pk_bf16_f32 under the
// default rounding mode; the same bits as adding 0x7FFF plus the kept lowest
// bit and truncating, for finite inputs).
__device__ __forceinline__ short to_bf16(float x) { return __builtin_bit_cast(short, (__bf16)x); }

__device__ __forceinline__ bf16x4 pack4(f32x4 v) {
    bf16x4 r;
    r[0] = to_bf16(v[0]);
    r[1] = to_bf16(v[1]);
    r[2] = to_bf16(v[2]);
    r[3] = to_bf16(v[3]);
    return r;
}
// ReLU as a signed integer max with 0 on the FP32 bit patterns (one
// v_max_i32 per value, no NaN canonicalisation): a value with its sign bit
// set, -0 included, is a negative integer and becomes +0, the same bits as
// v > 0 ? v : 0 for every non-NaN v.
__device__ __forceinline__ f32x4 relu4(f32x4 v) {
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    return __builtin_bit_cast(f32x4, __builtin_elementwise_max(__builtin_bit_cast(i32x4, v), i32x4{0, 0, 0, 0}));
}
__device__ __forceinline__ bf16x4 relu_pack4(f32x4 v) { return pack4(relu4(v)); }

constexpr int WAVES = 4;  // wavefronts per workgroup

// FP32 arithmetic of the fallback, no contraction: its decisions must not
// depend on how the compiler fuses the products.
__device__ __forceinline__ float fmul(float x, float y) { return __fmul_rn(x, y); }
__device__ __forceinline__ float fsub(float x, float y) { return __fsub_rn(x, y); }
__device__ __forceinline__ float fadd(float x, float y) { return __fadd_rn(x, y); }

// Fallback indicator of one face: the depth jump at most tau times the
// smaller depth, and each correction component d[c] at most bound[c].
__device__ __forceinline__ bool indicator_ok(float hl, float hr, float tau, const float d[3], const float bound[3]) {
    const float lo = hl < hr ? hl : hr;
    bool ok = fabsf(fsub(hr, hl)) <= fmul(tau, lo);
    for (int c = 0; c < 3; ++c) ok = ok && (fabsf(d[c]) <= bound[c]);
    return ok;
}

// Geometry of one face tile of 64 consecutive faces along a line.
struct FaceTile {
    int axis;   // 0: x faces (face k between cells k-1, k of row j); 1: y faces
    int line;   // x: row j; y: face row k (between rows k-1 and k)
    int first;  // x: first face k; y: first column i
};

__device__ __forceinline__ float* pick3(float* b0, float* b1, float* b2, int i) {
    return i == 0 ? b0 : (i == 1 ? b1 : b2);
}

__device__ __forceinline__ FaceTile tile_of(const LcNet& a, int t) {
    FaceTile ft;
    if (t < a.ntiles_x) {
        ft.axis = 0;
        ft.line = t / a.tpr_x;
        ft.first = 1 + (t - ft.line * a.tpr_x) * 64;
    } else {
        const int u = t - a.ntiles_x;
        ft.axis = 1;
        ft.line = 1 + u / a.tpr_y;
        ft.first = (u - (ft.line - 1) * a.tpr_y) * 64;
    }
    return ft;
}

// Field of frame channel c on faces of `axis`: x (h, hu, hv), y (h, hv, hu).
__device__ __forceinline__ int frame_field(int axis, int c) { return (axis == 0 || c == 0) ? c : 3 - c; }

// Stencil value s (0..3 = cells k-2 .. k+1) of channel c for face `pos` of
// tile ft (pos: x face index k, y column i), with the wall mirror.
__device__ __forceinline__ float stencil(const LcNet& a, const float* __restrict__ q, const FaceTile& ft,
                                         int pos, int c, int s) {
    const int f = frame_field(ft.axis, c);
    const int n = ft.axis == 0 ? a.nx : a.ny;
    int idx = (ft.axis == 0 ? pos : ft.line) - 2 + s;
    float sign = 1.0f;
    if (idx < 0) {
        idx = -1 - idx;
        if (c == 1) sign = -1.0f;
    } else if (idx >= n) {
        idx = 2 * n - 1 - idx;
        if (c == 1) sign = -1.0f;
    }
    const int cell = ft.axis == 0 ? ft.line * a.nx + idx : idx * a.nx + pos;
    CLAW_CHECK(idx >= 0 && idx < n && cell >= 0 && cell < a.ncell);
    return sign * q[(size_t)f * a.ncell + cell];
}

// Weights of one wavefront in operand registers.
struct NetRegs {
    bf16x4 A1[4];      // W1 tiles (units 16t.., features)
    bf16x4 A2[4][4];   // W2 tiles [t][s]
    bf16x4 A3[4];      // W3 (outputs, units 16s..)
    f32x4 B1[4], B2[4], B3;
};

// Network of sweep direction `axis`.
struct NetPtr {
    const float* theta;
    const unsigned short *w1b, *w2b, *w3b;
};
__device__ __forceinline__ NetPtr net_of(const LcNet& a, int axis) {
    NetPtr n;
    n.theta = a.theta + axis * LC_NET;
    n.w1b = a.w1b + axis * LC_W1B;
    n.w2b = a.w2b + axis * LC_W2B;
    n.w3b = a.w3b + axis * LC_W3B;
    return n;
}

__device__ __forceinline__ void load_net(const NetPtr& N, int lane, NetRegs& R) {
    const int i = lane & 15, kb = lane >> 4;
    for (int t = 0; t < 4; ++t) {
        for (int e = 0; e < 4; ++e) {
            R.A1[t][e] = (short)N.w1b[w1_slot(16 * t + i, 4 * kb + e)];
            R.B1[t][e] = N.theta[LC_OFF_B1 + 16 * t + 4 * kb + e];
            R.B2[t][e] = N.theta[LC_OFF_B2 + 16 * t + 4 * kb + e];
            R.A3[t][e] = (short)N.w3b[w3_slot(i, 16 * t + 4 * kb + e)];
        }
        for (int s = 0; s < 4; ++s)
            for (int e = 0; e < 4; ++e) R.A2[t][s][e] = (short)N.w2b[w2_slot(16 * t + i, 16 * s + 4 * kb + e)];
    }
    for (int e = 0; e < 4; ++e) {
        const int o = 4 * kb + e;
        R.B3[e] = o < 3 ? N.theta[LC_OFF_B3 + o] : 0.0f;
    }
}

// Face tiles of launch direction blockIdx.y: [first, end) of the tile index.
__device__ __forceinline__ void axis_tiles(const LcNet& a, int axis, int& first, int& end) {
    first = axis == 0 ? 0 : a.ntiles_x;
    end = axis == 0 ? a.ntiles_x : a.ntiles;
}

// Channel kb's feature scales and their FP64 reciprocals (lane group kb;
// lane group 3 carries no channel).
struct FeatScale {
    double s[4], r[4], mu;
};
__device__ __forceinline__ FeatScale feat_scale(const LcNet& a, int kb) {
    FeatScale F;
    const int c = kb < 3 ? kb : 0;
    F.s[0] = a.nm.sl[c];
    F.s[1] = a.nm.sd1[c];
    F.s[2] = a.nm.sd2[c];
    F.s[3] = a.nm.sd3[c];
    for (int k = 0; k < 4; ++k) F.r[k] = __ddiv_rn(1.0, F.s[k]);
    F.mu = kb == 0 ? (double)a.nm.mu_h : 0.0;
    return F;
}

// A tile whose every face has its four stencil cells inside the grid (no
// wall mirror): x faces first .. first + 63 need first >= 2 and
// first + 63 <= nx - 2, a y face row k needs 2 <= k <= ny - 2 (its columns
// past nx - 1, in the row's last tile, are clamped by face_pos).
__device__ __forceinline__ bool tile_interior(const LcNet& a, const FaceTile& ft) {
    return ft.axis == 0 ? (ft.first >= 2 && ft.first + 63 <= a.nx - 2) : (ft.line >= 2 && ft.line <= a.ny - 2);
}

// Stencil values (cells k-2 .. k+1) of channel kb < 3 around face `pos`.
__device__ __forceinline__ void stencil_vals(const LcNet& a, const float* __restrict__ q, const FaceTile& ft, int pos,
                                             int kb, bool interior, float (&v)[4]) {
    if (interior) {
        const int f = frame_field(ft.axis, kb);
        const float* p = q + (size_t)f * a.ncell;
        if (ft.axis == 0) {
            CLAW_CHECK(pos >= 2 && pos + 1 < a.nx && ft.line < a.ny);
            p += (size_t)ft.line * a.nx + pos - 2;
            for (int k = 0; k < 4; ++k) v[k] = p[k];
        } else {
            CLAW_CHECK(ft.line >= 2 && ft.line + 1 < a.ny && pos < a.nx);
            p += (size_t)(ft.line - 2) * a.nx + pos;
            for (int k = 0; k < 4; ++k) v[k] = p[(size_t)k * a.nx];
        }
    } else {
        for (int k = 0; k < 4; ++k) v[k] = stencil(a, q, ft, pos, kb, k);
    }
}

// The four features of one channel as the B operand elements of lane group
// kb (zeros for kb = 3).  They are formed in FP64 (the higher differences
// cancel; FP32 would round them coarsely) and rounded FP64 -> FP32 -> BF16.
__device__ __forceinline__ bf16x4 feat_of(const float (&s)[4], int kb, const FeatScale& F) {
    bf16x4 x = {0, 0, 0, 0};
    if (kb < 3) {
        const double v0 = s[0], v1 = s[1], v2 = s[2], v3 = s[3];
        const double jump = __dsub_rn(v2, v1);
        const double mid = __dadd_rn(v1, v2);
        const double lvl = __builtin_fma(mid, 0.5, -F.mu);  // mid / 2 is exact
        const double curv = __dsub_rn(__dadd_rn(v0, v3), mid);
        const double third = __builtin_fma(-3.0, jump, __dsub_rn(v3, v0));
        // divisions by the scales as products with their reciprocals: a last-bit
        // difference in FP64 at most, gone after the rounding to FP32 and BF16
        // except in rare ties
        x[0] = to_bf16((float)__dmul_rn(lvl, F.r[0]));
        x[1] = to_bf16((float)__dmul_rn(jump, F.r[1]));
        x[2] = to_bf16((float)__dmul_rn(curv, F.r[2]));
        x[3] = to_bf16((float)__dmul_rn(third, F.r[3]));
    }
    return x;
}

// Inputs of 16 faces (group g of the tile) as the B operand: lane n + 16 kb
// holds the four features of channel kb; lane group 0 also returns the
// depths on either side of its face.
__device__ __forceinline__ bf16x4 features(const LcNet& a, const float* __restrict__ q, const FaceTile& ft,
                                           int pos, int lane, bool interior, const FeatScale& F, float& hl,
                                           float& hr) {
    const int kb = lane >> 4;
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (kb < 3) stencil_vals(a, q, ft, pos, kb, interior, v);
    hl = v[1];
    hr = v[2];
    return feat_of(v, kb, F);
}

struct Acts {
    bf16x4 h1[4], h2[4];
    f32x4 y;
};

__device__ __forceinline__ void net_forward(const NetRegs& R, bf16x4 x, Acts& A) {
    for (int t = 0; t < 4; ++t) A.h1[t] = relu_pack4(mma(R.A1[t], x, R.B1[t]));
    for (int t = 0; t < 4; ++t) {
        f32x4 z = R.B2[t];
        for (int s = 0; s < 4; ++s) z = mma(R.A2[t][s], A.h1[s], z);
        A.h2[t] = relu_pack4(z);
    }
    f32x4 y = R.B3;
    for (int s = 0; s < 4; ++s) y = mma(R.A3[s], A.h2[s], y);
    A.y = y;
}

// Face position of lane n in group g, clamped into the line; valid flag.
// (x tiles: faces 1 .. nx-1; y tiles: columns 0 .. nx-1 -- the same last index)
__device__ __forceinline__ int face_pos(const LcNet& a, const FaceTile& ft, int g, int n, bool& valid) {
    const int pos = ft.first + 16 * g + n;
    valid = pos <= a.nx - 1;
    return valid ? pos : a.nx - 1;
}

// A trial that ran and is not decided yet, with no failure and no
// non-physical state flagged by its sweeps (the learned step's kernels run
// between a fixed-dt trial and its decision, which accepts it).
__device__ __forceinline__ bool trial_ok(const Ctrl* c, int q) {
    const StepState& s = c->st[q];
    return s.pending && !s.done && !s.err && !c->nonphys[q];
}

__device__ __forceinline__ const float* resolve_state(const LcNet& a, bool& skip) {
    skip = false;
    if (!a.ctrl) return a.q;
    if (!trial_ok(a.ctrl, a.cq)) {
        skip = true;
        return a.q;
    }
    return pick3(a.buf0, a.buf1, a.buf2, (a.ctrl->st[a.cq].cur + a.qsel) % 3);
}

// Forward pass over every interior face: corrections dF (3, ny, nx+1) and
// dG (3, ny+1, nx) in state component order; wall faces written as zero.
// Per 16 faces: 4 products of 16x16x16 (layer 1, K = 12 features padded to
// 16) and 8 + 2 of 16x16x32 (layers 2 and 3, K = 64 in two blocks).
__global__ __launch_bounds__(256) void k_lc_forward(LcNet a) {
    bool skip;
    const float* __restrict__ q = resolve_state(a, skip);
    if (skip) return;
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, kb = lane >> 4;
    const int axis = blockIdx.y;
    const NetPtr N = net_of(a, axis);
    bf16x4 A1[4];
    bf16x8 A2[4][2], A3[2];
    f32x4 B1[4], B2[4], B3;
    for (int t = 0; t < 4; ++t) {
        A1[t] = *reinterpret_cast<const bf16x4*>(N.w1b + (t * 64 + lane) * 4);
        for (int s = 0; s < 2; ++s) A2[t][s] = *reinterpret_cast<const bf16x8*>(N.w2b + ((t * 2 + s) * 64 + lane) * 8);
        for (int e = 0; e < 4; ++e) {
            B1[t][e] = N.theta[LC_OFF_B1 + 16 * t + 4 * kb + e];
            B2[t][e] = N.theta[LC_OFF_B2 + 16 * t + 4 * kb + e];
        }
    }
    for (int s = 0; s < 2; ++s) A3[s] = *reinterpret_cast<const bf16x8*>(N.w3b + (s * 64 + lane) * 8);
    for (int e = 0; e < 4; ++e) {
        const int o = 4 * kb + e;
        B3[e] = o < 3 ? N.theta[LC_OFF_B3 + o] : 0.0f;
    }
    const FeatScale F = feat_scale(a, kb);
    const float so[3] = {a.nm.s_out[0], a.nm.s_out[1], a.nm.s_out[2]};
    const float bound[3] = {fmul(a.kappa, so[0]), fmul(a.kappa, so[1]), fmul(a.kappa, so[2])};
    const int wave = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * WAVES;
    const size_t fx = (size_t)a.ny * (a.nx + 1), fy = (size_t)(a.ny + 1) * a.nx;
    int t0, t1;
    axis_tiles(a, axis, t0, t1);
    // the network on 16 faces and the store of their corrections
    auto run_group = [&](const FaceTile& ft, int pos, bool valid, bf16x4 x, float hl, float hr) {
        bf16x4 h1[4], h2[4];
        for (int u = 0; u < 4; ++u) h1[u] = relu_pack4(mma(A1[u], x, B1[u]));
        const bf16x8 k0 = join(h1[0], h1[1]), k1 = join(h1[2], h1[3]);
        for (int u = 0; u < 4; ++u) h2[u] = relu_pack4(mma32(A2[u][1], k1, mma32(A2[u][0], k0, B2[u])));
        const f32x4 y = mma32(A3[1], join(h2[2], h2[3]), mma32(A3[0], join(h2[0], h2[1]), B3));
        if (kb == 0 && valid) {
            float v[3];
            for (int c = 0; c < 3; ++c) v[c] = so[c] * y[c];
            const bool drop = a.mask && !indicator_ok(hl, hr, a.tau, v, bound);
            for (int c = 0; c < 3; ++c) {
                const int f = frame_field(ft.axis, c);
                const float w = drop ? 0.0f : v[c];
                CLAW_CHECK(ft.axis == 0 ? (pos <= a.nx && ft.line < a.ny) : (pos < a.nx && ft.line <= a.ny));
                if (ft.axis == 0)
                    a.dF[f * fx + (size_t)ft.line * (a.nx + 1) + pos] = w;
                else
                    a.dG[f * fy + (size_t)ft.line * a.nx + pos] = w;
            }
        }
    };
    for (int t = t0 + wave; t < t1; t += nwaves) {
        const FaceTile ft = tile_of(a, t);
        if (tile_interior(a, ft)) {
            // every load of the tile first (no wall mirror: the stencils lie
            // inside the grid; faces past the end of a y-face row are clamped
            // onto its last column and not stored)
            float sv[4][4];
            int pos[4];
            bool valid[4];
            for (int g = 0; g < 4; ++g) {
                pos[g] = face_pos(a, ft, g, n, valid[g]);
                for (int k = 0; k < 4; ++k) sv[g][k] = 0.0f;
            }
            if (kb < 3)
                for (int g = 0; g < 4; ++g) stencil_vals(a, q, ft, pos[g], kb, true, sv[g]);
            for (int g = 0; g < 4; ++g) run_group(ft, pos[g], valid[g], feat_of(sv[g], kb, F), sv[g][1], sv[g][2]);
        } else {
            for (int g = 0; g < 4; ++g) {
                bool valid;
                const int pos = face_pos(a, ft, g, n, valid);
                float hl, hr;
                const bf16x4 x = features(a, q, ft, pos, lane, false, F, hl, hr);
                run_group(ft, pos, valid, x, hl, hr);
            }
        }
        // wall faces: x faces 0 and nx of this row; y face rows 0 and ny
        if (ft.axis == 0 && ft.first == 1 && lane < 6) {
            const int c = lane % 3;
            const int k = lane < 3 ? 0 : a.nx;
            a.dF[c * fx + (size_t)ft.line * (a.nx + 1) + k] = 0.0f;
        }
        if (ft.axis == 1 && (ft.line == 1 || ft.line == a.ny - 1)) {
            const int i = ft.first + lane;
            if (i < a.nx)
                for (int c = 0; c < 3; ++c) {
                    if (ft.line == 1) a.dG[c * fy + i] = 0.0f;
                    if (ft.line == a.ny - 1) a.dG[c * fy + (size_t)a.ny * a.nx + i] = 0.0f;
                }
        }
    }
}

// LDS transpose area of one wavefront, BF16, feature/unit-major [row][16 faces].
struct WaveLds {
    short x[16 * 16];
    short h1[64 * 16], h2[64 * 16], z1[64 * 16], z2[64 * 16];
    short y[16 * 16];
};

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Store a D-layout tile (lane n + 16 kb, element e -> row 16 t + 4 kb + e, face n).
__device__ __forceinline__ void put_tile(short* base, int t, int lane, bf16x4 v) {
    const int n = lane & 15, kb = lane >> 4;
    for (int e = 0; e < 4; ++e) base[(16 * t + 4 * kb + e) * 16 + n] = v[e];
}
// Operand with rows 16 t + (lane & 15) and the four faces 4 kb .. 4 kb + 3.
__device__ __forceinline__ bf16x4 get_rows(const short* base, int t, int lane) {
    const int i = lane & 15, kb = lane >> 4;
    const short* p = base + (16 * t + i) * 16 + 4 * kb;
    bf16x4 r;
    r[0] = p[0];
    r[1] = p[1];
    r[2] = p[2];
    r[3] = p[3];
    return r;
}

// Fused training pass: forward again, output gradient from the cell
// gradients g (dL/dF_{k-1/2} = nu (g_k - g_{k-1})), backward through the
// network, and per-wavefront partial parameter gradients.
__global__ __launch_bounds__(256) void k_lc_backward(LcNet a) {
    __shared__ WaveLds lds_all[WAVES];
    WaveLds& L = lds_all[threadIdx.x >> 6];
    const float* __restrict__ q = a.q;
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, kb = lane >> 4;
    const int axis = blockIdx.y;
    const NetPtr N = net_of(a, axis);
    NetRegs R;
    load_net(N, lane, R);
    // transposed weights for the backward products
    bf16x4 T3[4], T2[4][4];
    for (int t = 0; t < 4; ++t) {
        for (int e = 0; e < 4; ++e) {
            const int o = 4 * kb + e;
            T3[t][e] = o < 3 ? (short)N.w3b[w3_slot(o, 16 * t + n)] : (short)0;
        }
        for (int s = 0; s < 4; ++s)
            for (int e = 0; e < 4; ++e) T2[t][s][e] = (short)N.w2b[w2_slot(16 * s + 4 * kb + e, 16 * t + n)];
    }
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 acc1[4], acc2[4][4], acc3[4], sb1[4], sb2[4];
    float sb3[3] = {0.0f, 0.0f, 0.0f};
    for (int t = 0; t < 4; ++t) {
        acc1[t] = zero;
        acc3[t] = zero;
        sb1[t] = zero;
        sb2[t] = zero;
        for (int s = 0; s < 4; ++s) acc2[t][s] = zero;
    }
    const int wave = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * WAVES;
    int t0, t1;
    axis_tiles(a, axis, t0, t1);
    const FeatScale F = feat_scale(a, kb);
    for (int t = t0 + wave; t < t1; t += nwaves) {
        const FaceTile ft = tile_of(a, t);
        const bool interior = tile_interior(a, ft);
        const float nu = ft.axis == 0 ? a.nux : a.nuy;
        for (int grp = 0; grp < 4; ++grp) {
            bool valid;
            const int pos = face_pos(a, ft, grp, n, valid);
            float hl, hr;
            const bf16x4 x = features(a, q, ft, pos, lane, interior, F, hl, hr);
            Acts A;
            net_forward(R, x, A);
            // output gradient (lanes kb = 0 hold the three channels of face n)
            float dy[3] = {0.0f, 0.0f, 0.0f};
            if (kb == 0 && valid) {
                for (int c = 0; c < 3; ++c) {
                    const int f = frame_field(ft.axis, c);
                    const float* gf = a.g + (size_t)f * a.ncell;
                    float gr, gl;
                    if (ft.axis == 0) {
                        gr = gf[ft.line * a.nx + pos];
                        gl = gf[ft.line * a.nx + pos - 1];
                    } else {
                        gr = gf[ft.line * a.nx + pos];
                        gl = gf[(ft.line - 1) * a.nx + pos];
                    }
                    dy[c] = a.nm.s_out[c] * (nu * (gr - gl));
                }
            }
            for (int c = 0; c < 3; ++c) sb3[c] += dy[c];
            bf16x4 dyb = {0, 0, 0, 0};
            if (kb == 0) {
                dyb[0] = to_bf16(dy[0]);
                dyb[1] = to_bf16(dy[1]);
                dyb[2] = to_bf16(dy[2]);
            }
            bf16x4 dz2b[4], dz1b[4];
            for (int t2 = 0; t2 < 4; ++t2) {
                f32x4 d = mma(T3[t2], dyb, zero);
                for (int e = 0; e < 4; ++e) d[e] = A.h2[t2][e] > 0 ? d[e] : 0.0f;  // bf16 > 0 as an integer
                sb2[t2] += d;
                dz2b[t2] = pack4(d);
            }
            for (int t1 = 0; t1 < 4; ++t1) {
                f32x4 d = zero;
                for (int s = 0; s < 4; ++s) d = mma(T2[t1][s], dz2b[s], d);
                for (int e = 0; e < 4; ++e) d[e] = A.h1[t1][e] > 0 ? d[e] : 0.0f;
                sb1[t1] += d;
                dz1b[t1] = pack4(d);
            }
            // transposes through LDS: rows are units / features / outputs, columns faces
            put_tile(L.x, 0, lane, x);
            for (int t4 = 0; t4 < 4; ++t4) {
                put_tile(L.h1, t4, lane, A.h1[t4]);
                put_tile(L.h2, t4, lane, A.h2[t4]);
                put_tile(L.z1, t4, lane, dz1b[t4]);
                put_tile(L.z2, t4, lane, dz2b[t4]);
            }
            put_tile(L.y, 0, lane, dyb);
            lds_sync();
            const bf16x4 xr = get_rows(L.x, 0, lane);
            bf16x4 yr = get_rows(L.y, 0, lane);
            if (n >= 3) yr = bf16x4{0, 0, 0, 0};
            for (int tk = 0; tk < 4; ++tk) {
                const bf16x4 h1r = get_rows(L.h1, tk, lane);
                const bf16x4 h2r = get_rows(L.h2, tk, lane);
                acc3[tk] = mma(yr, h2r, acc3[tk]);
                for (int tu = 0; tu < 4; ++tu) acc2[tu][tk] = mma(get_rows(L.z2, tu, lane), h1r, acc2[tu][tk]);
            }
            for (int tu = 0; tu < 4; ++tu) acc1[tu] = mma(get_rows(L.z1, tu, lane), xr, acc1[tu]);
            lds_sync();
        }
    }
    // partial gradients of this wavefront for its direction's network
    float* P = a.partial + ((size_t)axis * nwaves + wave) * LC_NET;
    for (int tu = 0; tu < 4; ++tu)
        for (int e = 0; e < 4; ++e) {
            const int u = 16 * tu + 4 * kb + e;
            if (n < 12) P[LC_OFF_W1 + u * 12 + n] = acc1[tu][e];
            for (int tk = 0; tk < 4; ++tk) P[LC_OFF_W2 + u * 64 + 16 * tk + n] = acc2[tu][tk][e];
        }
    if (kb == 0)
        for (int tk = 0; tk < 4; ++tk)
            for (int e = 0; e < 3; ++e) P[LC_OFF_W3 + e * 64 + 16 * tk + n] = acc3[tk][e];
    // bias gradients: sum over the 16 faces (lanes) of each row group
    for (int t = 0; t < 4; ++t)
        for (int e = 0; e < 4; ++e) {
            float v1 = sb1[t][e], v2 = sb2[t][e];
            for (int m = 1; m < 16; m <<= 1) {
                v1 += __shfl_xor(v1, m);
                v2 += __shfl_xor(v2, m);
            }
            if (n == 0) {
                P[LC_OFF_B1 + 16 * t + 4 * kb + e] = v1;
                P[LC_OFF_B2 + 16 * t + 4 * kb + e] = v2;
            }
        }
    for (int c = 0; c < 3; ++c) {
        float v = sb3[c];
        for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m);
        if (lane == 0) P[LC_OFF_B3 + c] = v;
    }
}

// Cell gradients of the loss  sum w_f (p - r)^2 / (3N),  p the correction's
// flux difference and r = target - plain; per-block partial sums
// (loss numerator, sum r_f^2) in FP64.
__global__ __launch_bounds__(256) void k_lc_cellgrad(LcCell a) {
    __shared__ double red[4][256];
    const int tid = threadIdx.x;
    double acc[4] = {0, 0, 0, 0};
    const size_t fx = (size_t)a.ny * (a.nx + 1), fy = (size_t)(a.ny + 1) * a.nx;
    for (int c = blockIdx.x * 256 + tid; c < a.ncell; c += gridDim.x * 256) {
        const int j = c / a.nx, i = c - j * a.nx;
        for (int f = 0; f < 3; ++f) {
            const float* F = a.dF + f * fx + (size_t)j * (a.nx + 1);
            const float* G = a.dG + f * fy;
            const float p = -a.nux * (F[i + 1] - F[i]) - a.nuy * (G[(size_t)(j + 1) * a.nx + i] - G[(size_t)j * a.nx + i]);
            const float r = a.target[(size_t)f * a.ncell + c] - a.plain[(size_t)f * a.ncell + c];
            const float d = p - r;
            a.g[(size_t)f * a.ncell + c] = a.gscale[f] * d;
            acc[0] += (double)a.w[f] * (double)d * (double)d;
            acc[1 + f] += (double)r * (double)r;
        }
    }
    for (int k = 0; k < 4; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + s];
        __syncthreads();
    }
    if (tid < 4) a.loss_part[blockIdx.x * 4 + tid] = red[tid][0];
}

// Sum of the per-wavefront partial gradients (fixed order; nparts
// wavefronts per direction) into grad, and of the loss partials into
// loss[0..3] (the first block's first four wavefronts).  A block sums 64 parameters:
// its 16 wavefronts take every 16th partial each, eight independent running
// sums per lane (so eight loads are in flight), combined in a fixed order.
constexpr int RED_PARTS = 16;
__global__ __launch_bounds__(64 * RED_PARTS) void k_lc_reduce(const float* __restrict__ partial, int nparts,
                                                              float* grad, const double* __restrict__ loss_part,
                                                              int nloss, double inv3n, double* loss) {
    __shared__ float red[RED_PARTS][64];
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 64 + lane;
    const int part = threadIdx.x >> 6;
    float s = 0.0f;
    if (p < LC_NPARAM) {
        const int axis = p / LC_NET, local = p - axis * LC_NET;
        const float* base = partial + (size_t)axis * nparts * LC_NET + local;
        float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int w = part;
        for (; w + 7 * RED_PARTS < nparts; w += 8 * RED_PARTS)
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += base[(size_t)(w + k * RED_PARTS) * LC_NET];
#pragma unroll
        for (int k = 0; k < 7; ++k)
            if (w + k * RED_PARTS < nparts) acc[k] += base[(size_t)(w + k * RED_PARTS) * LC_NET];
        s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    }
    red[part][lane] = s;
    __syncthreads();
    if (part == 0 && p < LC_NPARAM) {
        float t = 0.0f;
        for (int k = 0; k < RED_PARTS; ++k) t += red[k][lane];
        grad[p] = t;
    }
    if (blockIdx.x == 0 && part < 4 && loss) {  // wavefront `part` sums loss component `part`
        double v = 0.0;
        for (int b = lane; b < nloss; b += 64) v += loss_part[b * 4 + part];
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        if (lane == 0) loss[part] = part == 0 ? v * inv3n : v;
    }
}

__device__ __forceinline__ void emit_bf16(LcParams a, int p, float v) {
    const int axis = p / LC_NET, r = p - axis * LC_NET;
    if (r < LC_OFF_B1) {
        a.w1b[axis * LC_W1B + w1_slot(r / 12, r % 12)] = (unsigned short)to_bf16(v);
    } else if (r >= LC_OFF_W2 && r < LC_OFF_B2) {
        const int k = r - LC_OFF_W2;
        a.w2b[axis * LC_W2B + w2_slot(k / 64, k % 64)] = (unsigned short)to_bf16(v);
    } else if (r >= LC_OFF_W3 && r < LC_OFF_B3) {
        const int k = r - LC_OFF_W3;
        a.w3b[axis * LC_W3B + w3_slot(k / 64, k % 64)] = (unsigned short)to_bf16(v);
    }
}

// Zero the moments and the BF16 padding, then emit the BF16 weight copies.
__global__ void k_lc_init(LcParams a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < 2 * LC_W1B) a.w1b[p] = 0;
    if (p < 2 * LC_W3B) a.w3b[p] = 0;
    if (p < LC_NPARAM) {
        a.m[p] = 0.0f;
        a.v[p] = 0.0f;
    }
}
__global__ void k_lc_emit(LcParams a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < LC_NPARAM) emit_bf16(a, p, a.theta[p]);
}

// Adam on the FP32 masters (c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t)),
// then the BF16 copy of the new weight.
__global__ void k_lc_adam(LcParams a, const float* __restrict__ grad, float lr, float beta1, float beta2, float eps,
                          float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= LC_NPARAM) return;
    const float g = grad[p];
    const float m = beta1 * a.m[p] + (1.0f - beta1) * g;
    const float v = beta2 * a.v[p] + (1.0f - beta2) * g * g;
    a.m[p] = m;
    a.v[p] = v;
    const float th = a.theta[p] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    a.theta[p] = th;
    emit_bf16(a, p, th);
}

// ---------------------------------------------------------------------------
// Fallback and application (FP32, no contraction: the decisions must not
// depend on how the compiler fuses the products).
// ---------------------------------------------------------------------------

struct ApplyState {
    const float* qn;
    const float* plain;
    float* out;
};

__device__ __forceinline__ bool resolve_apply(const LcApply& a, ApplyState& S) {
    S.qn = a.qn;
    S.plain = a.plain;
    S.out = a.out;
    if (!a.ctrl) return true;
    if (!trial_ok(a.ctrl, a.cq)) return false;
    const int cur = a.ctrl->st[a.cq].cur;
    S.qn = pick3(a.buf0, a.buf1, a.buf2, (cur + a.qsel) % 3);
    S.out = pick3(a.buf0, a.buf1, a.buf2, (cur + a.rsel) % 3);
    S.plain = S.out;  // in place: each cell reads only its own plain values
    return true;
}

// Indicator test of x face k of row j (1 <= k <= nx-1) or y face row k of column i.
// bound[c]: kappa times the output scale of state component c on this face's axis.
__device__ __forceinline__ bool face_ok(const LcApply& a, float hl, float hr, const float* __restrict__ d,
                                        size_t stride, const float* bound) {
    const float dd[3] = {d[0], d[stride], d[2 * stride]};
    return indicator_ok(hl, hr, a.tau, dd, bound);
}

struct FaceKeep {
    bool l, r, b, t;
};

__device__ __forceinline__ FaceKeep keep_of(const LcApply& a, const float* __restrict__ h, int i, int j) {
    const size_t fx = (size_t)a.ny * (a.nx + 1), fy = (size_t)(a.ny + 1) * a.nx;
    const int nx = a.nx, ny = a.ny;
    FaceKeep k;
    if (a.premasked) {  // the forward pass zeroed the faces that fail the test
        k.l = i > 0;
        k.r = i < nx - 1;
        k.b = j > 0;
        k.t = j < ny - 1;
        return k;
    }
    const float hc = h[j * nx + i];
    // x faces: components (h, hu, hv) are frame (h, m_n, m_t); y faces (h, m_t, m_n)
    const float bx[3] = {fmul(a.kappa, a.s_out[0]), fmul(a.kappa, a.s_out[1]), fmul(a.kappa, a.s_out[2])};
    const float by[3] = {bx[0], bx[2], bx[1]};
    k.l = i > 0 && face_ok(a, h[j * nx + i - 1], hc, a.dF + (size_t)j * (nx + 1) + i, fx, bx);
    k.r = i < nx - 1 && face_ok(a, hc, h[j * nx + i + 1], a.dF + (size_t)j * (nx + 1) + i + 1, fx, bx);
    k.b = j > 0 && face_ok(a, h[(j - 1) * nx + i], hc, a.dG + (size_t)j * nx + i, fy, by);
    k.t = j < ny - 1 && face_ok(a, hc, h[(j + 1) * nx + i], a.dG + (size_t)(j + 1) * nx + i, fy, by);
    return k;
}

__device__ __forceinline__ float corrected(const LcApply& a, float plain, int f, int i, int j, const FaceKeep& k) {
    const size_t fx = (size_t)a.ny * (a.nx + 1), fy = (size_t)(a.ny + 1) * a.nx;
    const float* F = a.dF + f * fx + (size_t)j * (a.nx + 1);
    const float* G = a.dG + f * fy;
    const float Fl = k.l ? F[i] : 0.0f, Fr = k.r ? F[i + 1] : 0.0f;
    const float Gb = k.b ? G[(size_t)j * a.nx + i] : 0.0f, Gt = k.t ? G[(size_t)(j + 1) * a.nx + i] : 0.0f;
    const float cx = fmul(a.nux, fsub(Fr, Fl));
    const float cy = fmul(a.nuy, fsub(Gt, Gb));
    return fsub(plain, fadd(cx, cy));
}

// Pass 1: cells whose depth could fall below half the plain depth, or to zero
// or below: the depth from only those indicator-kept faces that lower it
// (outflow through the right / top face, inflow through the left / bottom
// face taken as negative).  This worst case bounds the depth after any subset
// of the faces is dropped in pass 2, so no cell ends below it.
__global__ __launch_bounds__(256) void k_lc_apply1(LcApply a) {
    ApplyState S;
    if (!resolve_apply(a, S)) return;
    for (int j = blockIdx.y; j < a.ny; j += gridDim.y)
    for (int i = blockIdx.x * 256 + threadIdx.x; i < a.nx; i += gridDim.x * 256) {
        const int c = j * a.nx + i;
        const FaceKeep k = keep_of(a, S.qn, i, j);
        const float p = S.plain[c];
        const float* F = a.dF + (size_t)j * (a.nx + 1);
        const float Fl = k.l ? F[i] : 0.0f, Fr = k.r ? F[i + 1] : 0.0f;
        const float Gb = k.b ? a.dG[(size_t)j * a.nx + i] : 0.0f;
        const float Gt = k.t ? a.dG[(size_t)(j + 1) * a.nx + i] : 0.0f;
        const float tl = fmul(a.nux, Fl), tr = fmul(a.nux, Fr);
        const float tb = fmul(a.nuy, Gb), tt = fmul(a.nuy, Gt);
        const float lower = fadd(fsub(fmaxf(tr, 0.0f), fminf(tl, 0.0f)), fsub(fmaxf(tt, 0.0f), fminf(tb, 0.0f)));
        const float worst = fsub(p, lower);
        a.bad[c] = (worst < fmul(0.5f, p) || worst <= 0.0f) ? 1 : 0;
    }
}

// Pass 2: faces next to a bad cell are dropped; every field is updated.
__global__ __launch_bounds__(256) void k_lc_apply2(LcApply a) {
    ApplyState S;
    if (!resolve_apply(a, S)) return;
    const int nx = a.nx;
    for (int j = blockIdx.y; j < a.ny; j += gridDim.y)
    for (int i = blockIdx.x * 256 + threadIdx.x; i < nx; i += gridDim.x * 256) {
        const int c = j * nx + i;
        FaceKeep k = keep_of(a, S.qn, i, j);
        const bool me = a.bad[c] != 0;
        k.l = k.l && !me && !a.bad[c - 1 + (i == 0)];
        k.r = k.r && !me && !a.bad[c + 1 - (i == nx - 1)];
        k.b = k.b && !me && !a.bad[c - (j > 0 ? nx : 0)];
        k.t = k.t && !me && !a.bad[c + (j < a.ny - 1 ? nx : 0)];
        float o[3];
        for (int f = 0; f < 3; ++f) o[f] = corrected(a, S.plain[(size_t)f * a.ncell + c], f, i, j, k);
        for (int f = 0; f < 3; ++f) S.out[(size_t)f * a.ncell + c] = o[f];
        if (a.keep_x) {
            if (i == 0) a.keep_x[(size_t)j * (nx + 1)] = 0;
            a.keep_x[(size_t)j * (nx + 1) + i + 1] = k.r ? 1 : 0;
        }
        if (a.keep_y) {
            if (j == 0) a.keep_y[i] = 0;
            a.keep_y[(size_t)(j + 1) * nx + i] = k.t ? 1 : 0;
        }
    }
}

// 2 x 2 averages: coarse (3, ny, nx) from fine (3, 2ny, 2nx).
__global__ __launch_bounds__(256) void k_lc_coarsen(const float* __restrict__ fine, float* __restrict__ coarse,
                                                    int nx, int ny) {
    const int ncell = nx * ny;
    for (int c = blockIdx.x * 256 + threadIdx.x; c < 3 * ncell; c += gridDim.x * 256) {
        const int f = c / ncell, r = c - f * ncell;
        const int j = r / nx, i = r - j * nx;
        const float* F = fine + (size_t)f * 4 * ncell + (size_t)(2 * j) * (2 * nx) + 2 * i;
        coarse[c] = 0.25f * ((F[0] + F[1]) + (F[2 * nx] + F[2 * nx + 1]));
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): a counter-based generator, ten rounds of the
// 4x32 Philox S-box with the published multipliers and Weyl key increments.
struct Philox4 {
    unsigned v[4];
};
__device__ __forceinline__ Philox4 philox4x32_10(unsigned c0, unsigned c1, unsigned c2, unsigned c3, unsigned k0,
                                                 unsigned k1) {
    const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)M0 * c0;
        const unsigned long long p1 = (unsigned long long)M1 * c2;
        const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
        const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
        const unsigned n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    Philox4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// out = q + sigma_f * N(0, 1) per value (field f = index / ncell).  Value i
// draws from counter (i / 2, call, 0, 0) with key (seed, 0): two uniforms
// u = (x + 0.5) / 2^32 from the first two output words, and Box-Muller
// (sqrt(-2 ln u0) cos / sin (2 pi u1)) gives values 2k and 2k + 1.
__global__ __launch_bounds__(256) void k_lc_perturb(const float* __restrict__ q, float* __restrict__ out, int ncell,
                                                    float s0, float s1, float s2, unsigned seed, unsigned call) {
    const int n = 3 * ncell;
    for (int k = blockIdx.x * 256 + threadIdx.x; 2 * k < n; k += gridDim.x * 256) {
        const Philox4 r = philox4x32_10((unsigned)k, call, 0u, 0u, seed, 0u);
        const float u0 = ((float)r.v[0] + 0.5f) * 2.3283064365386963e-10f;
        const float u1 = ((float)r.v[1] + 0.5f) * 2.3283064365386963e-10f;
        const float rad = sqrtf(-2.0f * logf(u0));
        const float ang = 6.283185307179586f * u1;
        const float z[2] = {rad * cosf(ang), rad * sinf(ang)};
        for (int e = 0; e < 2; ++e) {
            const int i = 2 * k + e;
            if (i < n) {
                const int f = i / ncell;
                const float sg = f == 0 ? s0 : (f == 1 ? s1 : s2);
                out[i] = q[i] + sg * z[e];
            }
        }
    }
}

int blocks_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

// Wavefronts per direction of a network launch: one per face tile of the
// larger direction, at most `cap`, rounded up to whole workgroups (the
// training pass writes one partial per wavefront and direction).
int lc_net_waves(const LcNet& a, int cap) {
    const int ny_tiles = a.ntiles - a.ntiles_x;
    const int most = a.ntiles_x > ny_tiles ? a.ntiles_x : ny_tiles;
    const int w = most < cap ? most : cap;
    return ((w + WAVES - 1) / WAVES) * WAVES;
}

hipError_t launch_lc_forward(const LcNet& a, hipStream_t s) {
    const int w = lc_net_waves(a, 2048);
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lc_forward, dim3(w / WAVES, 2), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lc_backward(const LcNet& a, hipStream_t s) {
    const int w = lc_net_waves(a, 512);
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lc_backward, dim3(w / WAVES, 2), dim3(256), 0, s, a);
    return hipGetLastError();
}

int lc_cell_blocks(int64_t ncell) { return blocks_for(ncell) < 1024 ? blocks_for(ncell) : 1024; }

hipError_t launch_lc_cellgrad(const LcCell& a, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_cellgrad, dim3(lc_cell_blocks(a.ncell)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lc_reduce(const float* partial, int nparts, float* grad, const double* loss_part, int nloss,
                            double inv3n, double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_reduce, dim3((LC_NPARAM + 63) / 64), dim3(64 * RED_PARTS), 0, s, partial, nparts, grad,
                       loss_part, nloss, inv3n, loss);
    return hipGetLastError();
}

hipError_t launch_lc_init(const LcParams& a, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_init, dim3((LC_NPARAM + 255) / 256), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lc_emit, dim3((LC_NPARAM + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lc_adam(const LcParams& a, const float* grad, float lr, float beta1, float beta2, float eps,
                          float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_adam, dim3((LC_NPARAM + 255) / 256), dim3(256), 0, s, a, grad, lr, beta1, beta2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_lc_apply(const LcApply& a, hipStream_t s) {
    // one row of cells per block row (up to 256 columns per block, rows strided beyond 65535)
    const dim3 b((unsigned)((a.nx + 255) / 256), (unsigned)(a.ny < 65535 ? a.ny : 65535));
    hipLaunchKernelGGL(k_lc_apply1, b, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lc_apply2, b, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lc_perturb(const float* q, float* out, int ncell, const float* sigma, unsigned seed,
                             unsigned call, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_perturb, dim3(blocks_for((3 * (int64_t)ncell + 1) / 2)), dim3(256), 0, s, q, out,
                       ncell, sigma[0], sigma[1], sigma[2], seed, call);
    return hipGetLastError();
}

hipError_t launch_lc_coarsen(const float* fine, float* coarse, int nx, int ny, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_coarsen, dim3(blocks_for(3LL * nx * ny)), dim3(256), 0, s, fine, coarse, nx, ny);
    return hipGetLastError();
}

}  // namespace claw
