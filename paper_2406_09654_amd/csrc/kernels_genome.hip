// Genome kernels: CPPN -> network weights (HyperNEAT, System Design), the
// parameter scatter of coralai_set_genomes, debug weight packing, and
// radiation -> mutation (Fig. 1, panel C).
//
// CPPN: inputs z = (x1, y1, x2, y2, 1), 8 hidden nodes phi_k(A_k . z) with
// phi = sin, gauss (exp(-s^2)), tanh, identity for k mod 4 = 0..3, two linear
// outputs (weight, bias) = B h, evaluated in FP64 for FP32 networks.  Neuron j of layer l sits at
// (-1 + 2j/(L_l - 1), -1 + 2l/n); W_l[o][j] = CPPN_w(x_j, y_l, x_o, y_{l+1}) /
// sqrt(L_l) and b_l[o] = CPPN_b(0, y_l, x_o, y_{l+1}).  One thread per weight
// element, combining a per-column and a per-row table of node-input parts
// (built once per genome), written straight into the MFMA fragment order of
// the act kernel.
//
// Radiation: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
// (seed, 0); the block at counter (k, step, 0, 0) gives cells 4k..4k+3 one
// word each, and a cell is hit when its word is below floor(rate 2^64).  Hits are ranked in ascending cell order and take the
// free slots (zero count) in ascending order; the new genome is the parent's
// CPPN plus sigma * N(0,1) from Box-Muller on the Philox blocks
// (i, step, 1 + b, 0), b = 0..13, and its network is regenerated at once.
//
// Merging (NEAT crossover applied through the physics): a candidate cell
// (counter (k, step, 0, 1), otherwise as the radiation hit test) merges with
// the neighbour it faces when the two hold different genomes; the merges
// take free slots in cell order like radiation hits, and the child inherits
// gene m from the partner when bit m of word 0 of block (i, step, 0, 2) is
// set, from its own genome otherwise.
#include <type_traits>

#include <algorithm>

#include "coralai_internal.h"

namespace coralai {

// T = double for FP32 worlds (weights then rounded once to FP32), float for
// BF16 worlds (whose weights are rounded to bf16, 2^-9 relative, so the
// hardware sin / exp / reciprocal, accurate to ~1e-6 here, suffice).
//
// The FP64 node functions are written for the arguments a CPPN produces
// (a x1 + c x2 + base with |x| <= 1): Cody-Waite reduction by pi/2 or ln 2,
// split into parts that are each the double nearest to what the previous
// parts leave of the constant, then the Taylor series of sin, cos or exp on
// the reduced interval (|r| <= pi/4: the first omitted sin term is below
// 1e-19; |r| <= ln2/2: the first omitted exp term is below 5e-18).  Each
// result is within a few 2^-53 of its own scale, against the 2^-24 of the
// rounding to FP32 that follows.  sin falls back to the library beyond
// |s| = 2^20, where the three-part pi/2 would no longer suffice.
template <int N>
__device__ __forceinline__ constexpr double inv_factorial() {
    double f = 1.0;
    for (int k = 2; k <= N; ++k) f *= k;
    return 1.0 / f;
}

// e^x = 2^k (1 + r q(r)), q(r) = 1 + r/2! + r^2/3! + ...; returns r q(r) and k
__device__ __forceinline__ double exp_reduced(double x, int* k_out) {  // x in [-746, 60]
    const double k = rint(x * 0x1.71547652b82fep+0);                     // x / ln 2
    double r = fma(-k, 0x1.62e42fefa39efp-1, x);                         // ln 2, first part
    r = fma(-k, 0x1.abc9e3b39803fp-56, r);                                // ln 2, second part
    double q = inv_factorial<13>();
    q = fma(q, r, inv_factorial<12>());
    q = fma(q, r, inv_factorial<11>());
    q = fma(q, r, inv_factorial<10>());
    q = fma(q, r, inv_factorial<9>());
    q = fma(q, r, inv_factorial<8>());
    q = fma(q, r, inv_factorial<7>());
    q = fma(q, r, inv_factorial<6>());
    q = fma(q, r, inv_factorial<5>());
    q = fma(q, r, inv_factorial<4>());
    q = fma(q, r, inv_factorial<3>());
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    *k_out = (int)k;
    return r * q;
}

__device__ __forceinline__ void node_sincos(double s, double* sn_out, double* cs_out) {
    if (!(fabs(s) < 0x1p20)) {
        *sn_out = sin(s);
        *cs_out = cos(s);
        return;
    }
    const double k = rint(s * 0x1.45f306dc9c883p-1);  // s / (pi / 2)
    double r = fma(-k, 0x1.921fb54442d18p+0, s);     // pi / 2, three parts
    r = fma(-k, 0x1.1a62633145c07p-54, r);
    r = fma(-k, -0x1.f1976b7ed8fbcp-110, r);
    const double z = r * r;
    double ps = -inv_factorial<17>();
    ps = fma(ps, -z, inv_factorial<15>());
    ps = fma(ps, -z, inv_factorial<13>());
    ps = fma(ps, -z, inv_factorial<11>());
    ps = fma(ps, -z, inv_factorial<9>());
    ps = fma(ps, -z, inv_factorial<7>());
    ps = fma(ps, -z, inv_factorial<5>());
    ps = fma(ps, -z, inv_factorial<3>());
    ps = fma(ps, -z, 1.0);
    const double sn = ps * r;
    double pc = inv_factorial<18>();
    pc = fma(pc, -z, inv_factorial<16>());
    pc = fma(pc, -z, inv_factorial<14>());
    pc = fma(pc, -z, inv_factorial<12>());
    pc = fma(pc, -z, inv_factorial<10>());
    pc = fma(pc, -z, inv_factorial<8>());
    pc = fma(pc, -z, inv_factorial<6>());
    pc = fma(pc, -z, inv_factorial<4>());
    pc = fma(pc, -z, 0.5);
    const double cs = fma(pc, -z, 1.0);
    const int qd = (int)(int64_t)k & 3;  // quadrant: (sin, cos)(r + q pi/2)
    double so = (qd & 1) ? cs : sn, co = (qd & 1) ? -sn : cs;
    if (qd & 2) {
        so = -so;
        co = -co;
    }
    *sn_out = so;
    *cs_out = co;
}

__device__ __forceinline__ double node_gauss(double s) {
    const double x = -s * s;
    if (x < -746.0) return 0.0;  // NaN passes through
    int k;
    const double rq = exp_reduced(x, &k);
    return ldexp(1.0 + rq, k);
}

__device__ __forceinline__ double node_tanh(double s) {
    // tanh a = t / (t + 2) with t = e^2a - 1, which keeps its relative
    // accuracy for small a (k = 0: t = r q(r)); beyond a = 20 tanh is 1 in FP64
    const double a = fabs(s);
    int k;
    const double rq = exp_reduced(2.0 * (a > 20.0 ? 20.0 : a), &k);  // NaN passes through
    const double t = k == 0 ? rq : ldexp(1.0 + rq, k) - 1.0;
    return copysign(a > 20.0 ? 1.0 : t / (t + 2.0), s);
}

__device__ __forceinline__ void node_sincos(float s, float* sn, float* cs) {
    *sn = __sinf(s);
    *cs = __cosf(s);
}
__device__ __forceinline__ float node_gauss(float s) { return __expf(-s * s); }
__device__ __forceinline__ float node_tanh(float s) {
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * s) + 1.0f);
}

// The CPPN at (x1, y_l, x2, y_l+1): node k's input is A_k . (x1, y_l, x2,
// y_l+1, 1) = (a_k x1 + base_k) + c_k x2, a column part plus a row part, where
// base_k = b_k y_l + d_k y_l+1 + e_k depends only on the genome and the layer.
// Per genome, each layer's columns and rows get a table entry; with
// sin(A + B) = sin A cos B + cos A sin B and
// tanh(A + B) = 1 - 2 / (e^2A e^2B + 1), a weight then costs two FMAs per sin
// node, one exponential per gaussian and one reciprocal per tanh node.
// Entry of a column (A_k) or row (B_k) part:
enum : int { kTA1, kTA3, kTA5, kTA7, kTS0, kTC0, kTS4, kTC4, kTE2, kTE6, kTA2, kTA6, kTab };

// e^2v, or -1 where the product of a column and a row value could leave the
// finite range (|v| above 40 in FP32, 300 in FP64): tanh is then evaluated
// directly on A + B
__device__ __forceinline__ float exp2v_guarded(float v) { return fabsf(v) <= 40.0f ? __expf(2.0f * v) : -1.0f; }
__device__ __forceinline__ double exp2v_guarded(double v) {
    if (!(fabs(v) <= 300.0)) return -1.0;
    int k;
    const double rq = exp_reduced(2.0 * v, &k);
    return ldexp(1.0 + rq, k);
}

// off = 0: column part a_k x + base_k; off = 2 (base null): row part c_k x.
// Returns whether a tanh part is out of the exponential's range.
template <typename T>
__device__ __forceinline__ bool fill_entry(T* e, const float* p, int off, const T* base, T x) {
    T v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = T(p[5 * k + off]) * x + (base ? base[k] : T(0));
    e[kTA1] = v[1];
    e[kTA3] = v[3];
    e[kTA5] = v[5];
    e[kTA7] = v[7];
    e[kTA2] = v[2];
    e[kTA6] = v[6];
    node_sincos(v[0], &e[kTS0], &e[kTC0]);
    node_sincos(v[4], &e[kTS4], &e[kTC4]);
    e[kTE2] = exp2v_guarded(v[2]);
    e[kTE6] = exp2v_guarded(v[6]);
    return e[kTE2] < T(0) || e[kTE6] < T(0);
}

// GUARD: some part of this genome's tables is out of the exponential's range
template <bool GUARD>
__device__ __forceinline__ float tanh_sum(float e, float f, float a, float b) {
    if (GUARD && (e < 0.0f || f < 0.0f)) return node_tanh(a + b);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e * f + 1.0f);
}
template <bool GUARD>
__device__ __forceinline__ double tanh_sum(double e, double f, double a, double b) {
    if (GUARD && (e < 0.0 || f < 0.0)) return node_tanh(a + b);
    return 1.0 - 2.0 / (e * f + 1.0);
}

// Output `out` (0 weight, 1 bias) of the CPPN at a column entry c and a row
// entry r: sum over the nodes of B_out,k phi_k(A_k + B_k), in node order.
template <typename T, bool GUARD>
__device__ __forceinline__ T cppn_eval(const float* __restrict__ p, const T* __restrict__ c, const T* __restrict__ r,
                                       int out) {
    const float* po = p + 40 + 8 * out;
    T s = T(po[0]) * (c[kTS0] * r[kTC0] + c[kTC0] * r[kTS0]);
    s += T(po[1]) * node_gauss(c[kTA1] + r[kTA1]);
    s += T(po[2]) * tanh_sum<GUARD>(c[kTE2], r[kTE2], c[kTA2], r[kTA2]);
    s += T(po[3]) * (c[kTA3] + r[kTA3]);
    s += T(po[4]) * (c[kTS4] * r[kTC4] + c[kTC4] * r[kTS4]);
    s += T(po[5]) * node_gauss(c[kTA5] + r[kTA5]);
    s += T(po[6]) * tanh_sum<GUARD>(c[kTE6], r[kTE6], c[kTA6], r[kTA6]);
    s += T(po[7]) * (c[kTA7] + r[kTA7]);
    return s;
}

// NEAT structural genes (System Design: NEAT's operators), a bounded
// superset of the CPPN: direct connections input m -> output o (weight
// xw[5 o + m], bit 5 o + m of conn) and added nodes N_k, k = 2 j + o, that
// split the connection hidden j -> output o (bit k of node; activation bits
// 2k..2k+1 of act: sin, gauss, tanh, identity; in weight xw[10 + k], out
// weight xw[26 + k]); while N_k is enabled it replaces B[o][j].
template <typename T>
__device__ __forceinline__ T node_fn(uint32_t f, T s) {
    switch (f & 3u) {
        case 0: { T sn, cs; node_sincos(s, &sn, &cs); return sn; }
        case 1: return node_gauss(s);
        case 2: return node_tanh(s);
        default: return s;
    }
}
struct ExtGenes {
    uint32_t conn, node, act;
    const float* w;  // 42 weights (LDS)
};
// Output `out` of the CPPN with structural genes, at substrate inputs z =
// (z0, z1, z2, z3, 1) and the same column and row entries: the node values,
// then the output sum in node order, then the direct connections.
template <typename T, bool GUARD>
__device__ __forceinline__ T cppn_eval_x(const float* __restrict__ p, const T* __restrict__ c,
                                         const T* __restrict__ r, int out, const ExtGenes& x, T z0, T z1, T z2,
                                         T z3) {
    T h[8];
    h[0] = c[kTS0] * r[kTC0] + c[kTC0] * r[kTS0];
    h[1] = node_gauss(c[kTA1] + r[kTA1]);
    h[2] = tanh_sum<GUARD>(c[kTE2], r[kTE2], c[kTA2], r[kTA2]);
    h[3] = c[kTA3] + r[kTA3];
    h[4] = c[kTS4] * r[kTC4] + c[kTC4] * r[kTS4];
    h[5] = node_gauss(c[kTA5] + r[kTA5]);
    h[6] = tanh_sum<GUARD>(c[kTE6], r[kTE6], c[kTA6], r[kTA6]);
    h[7] = c[kTA7] + r[kTA7];
    const float* po = p + 40 + 8 * out;
    T s = T(0);
    for (int j = 0; j < 8; ++j) {
        const int k = 2 * j + out;
        if ((x.node >> k) & 1u) s += T(x.w[26 + k]) * node_fn<T>(x.act >> (2 * k), T(x.w[10 + k]) * h[j]);
        else s += T(po[j]) * h[j];
    }
    const T z[5] = {z0, z1, z2, z3, T(1)};
    for (int m = 0; m < 5; ++m)
        if ((x.conn >> (5 * out + m)) & 1u) s += T(x.w[5 * out + m]) * z[m];
    return s;
}

// Layer heights y_l = -1 + l * (2 / NL) and the stored scale factors of
// stored_row_scale / stored_col_scale, in T: for T = float the products are
// the same as the FP64 ones rounded once (the factors differ by powers of 2).
template <typename T, int NL>
__device__ __forceinline__ T layer_y(int l) { return T(-1) + T(l) * (T(2) / T(NL)); }
template <typename T>
__device__ __forceinline__ T row_scale(int nl, int layer, int row) {
    if (layer < nl - 1) return T(kTanhScale);
    return row < 6 ? T(-kLog2e) : (row < kNOut ? T(kLog2e) : T(1));
}
template <typename T, int PREC>
__device__ __forceinline__ T col_scale(int layer, int col) {
    if (layer > 0) return hidden_input_is_r(PREC) ? T(-2) : T(1);
    return col % 6 < 2 ? T(0x1p-24) : T(1);
}

// Stored value of a weight / bias of a network with NL weight layers and HID
// hidden units: the generated value times the stored scale factors, then
// one rounding to FP32 or bf16.  Neuron j of a layer of L sits at
// x = -1 + j * (2 / (L - 1)): with the shape fixed at compile time every
// divisor is a constant, folded into a multiplier.
template <typename T, int NL, int HID>
__device__ __forceinline__ T col_x(int layer, int col) {
    return T(-1) + T(col) * (layer == 0 ? T(2) / T(kNIn - 1) : T(2) / T(HID - 1));
}
template <typename T, int NL, int HID>
__device__ __forceinline__ T row_x(int layer, int row) {
    return T(-1) + T(row) * (layer == NL - 1 ? T(2) / T(kNOut - 1) : T(2) / T(HID - 1));
}

template <typename T, int NL, int HID, int PREC, bool GUARD, bool EXT>
__device__ __forceinline__ float cppn_weight(const float* p, const T* ce, const T* re, int layer, int row, int col,
                                             const ExtGenes& x) {
    const T rs = layer == 0 ? T(1) / sqrt(T(kNIn)) : T(1) / sqrt(T(HID));  // 1 / sqrt(fan-in)
    const T sc = row_scale<T>(NL, layer, row) * col_scale<T, PREC>(layer, col);
    if constexpr (EXT)
        return (float)(cppn_eval_x<T, GUARD>(p, ce, re, 0, x, col_x<T, NL, HID>(layer, col), layer_y<T, NL>(layer),
                                             row_x<T, NL, HID>(layer, row), layer_y<T, NL>(layer + 1)) *
                       rs * sc);
    return (float)(cppn_eval<T, GUARD>(p, ce, re, 0) * rs * sc);
}

// biases: the CPPN at x1 = 0, second output
template <typename T, int NL, int HID, bool GUARD, bool EXT>
__device__ __forceinline__ float cppn_bias(const float* p, const T* ce0, const T* re, int layer, int row,
                                           const ExtGenes& x) {
    if constexpr (EXT)
        return (float)(cppn_eval_x<T, GUARD>(p, ce0, re, 1, x, T(0), layer_y<T, NL>(layer), row_x<T, NL, HID>(layer, row),
                                             layer_y<T, NL>(layer + 1)) *
                       row_scale<T>(NL, layer, row));
    return (float)(cppn_eval<T, GUARD>(p, ce0, re, 1) * row_scale<T>(NL, layer, row));
}

// Layer geometry of a bias element index.
__device__ __forceinline__ void bias_coord(int nl, int hid, int bidx, int* layer, int* row) {
    if (bidx < hid) { *layer = 0; *row = bidx; return; }
    if (nl == 3 && bidx < 2 * hid) { *layer = 1; *row = bidx - hid; return; }
    *layer = nl - 1;
    *row = bidx - (nl == 3 ? 2 * hid : hid);
}

__device__ __forceinline__ int layer_in(int nl, int hid, int l) { return l == 0 ? kNIn : hid; }
__device__ __forceinline__ int layer_out(int nl, int hid, int l) { return l == nl - 1 ? kNOut : hid; }

// Offset of W_l and b_l in the flat layout [W_0, b_0, W_1, b_1, ...].
__device__ __forceinline__ int flat_w_offset(int nl, int hid, int l) {
    int o = 0;
    for (int k = 0; k < l; ++k) o += layer_out(nl, hid, k) * layer_in(nl, hid, k) + layer_out(nl, hid, k);
    return o;
}

// ------------------------------------------------------------------ Philox

// 64 x 64 -> 128-bit product from four 32 x 32 -> 64-bit multiply-adds
// (none of the partial sums can overflow 64 bits)
__device__ __forceinline__ void mul_128(uint64_t a, uint64_t b, uint64_t* lo, uint64_t* hi) {
    const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
    const uint64_t p00 = a0 * b0;
    const uint64_t t = a0 * b1 + (p00 >> 32);
    const uint64_t u = a1 * b0 + (uint32_t)t;
    *lo = (u << 32) | (uint32_t)p00;
    *hi = a1 * b1 + (t >> 32) + (u >> 32);
}

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t lo0, hi0, lo1, hi1;
        mul_128(M0, c[0], &lo0, &hi0);
        mul_128(M1, c[2], &lo1, &hi1);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

// Odd multiple of 2^-24 from the top 23 bits: exact in FP32, inside (0, 1).
__device__ __forceinline__ float philox_uniform(uint64_t o) {
    return (float)(2u * (uint32_t)(o >> 41) + 1u) * 0x1p-24f;
}

// One block per genome: its 56 parameters are read once into LDS, then the
// block's threads walk the genome's weight and bias elements.
// from_radiation = 0: the n_host slots listed by coralai_set_genomes;
// 1: the slots the last radiation call assigned, 2: those the last merging
// call assigned (counts on the device).  A radiation genome is first
// mutated here: its parameters are the parent's
// plus sigma * N(0, 1), four normals per lane 0..13 from Box-Muller on the
// Philox block (cell, step, 1 + lane, 0); they are stored and go straight
// to the block's LDS.
template <int NL, int HID, int PREC>
__global__ __launch_bounds__(256) void k_cppn(const WorldDev* __restrict__ w, int from_radiation,
                                              int n_host, uint64_t step, float sigma) {
    using T = typename std::conditional<PREC == kPrecBF16, float, double>::type;
    constexpr bool bf = PREC == kPrecBF16;
    constexpr int ew = net_frags(NL, HID, PREC) * net_frag_elems(PREC);
    constexpr int eb = net_bias_floats(NL, HID);
    __shared__ float sp[kNParam];
    __shared__ T sbase[NL][8];  // per layer and node: b y_l + d y_l+1 + e
    // per layer: column entries of the 64 columns and of x1 = 0 (biases, index
    // 64), row entries of the 64 rows
    __shared__ T stc[NL][65][kTab];
    __shared__ T str[NL][64][kTab];
    __shared__ float sxw[kNExtW];  // structural genes: weights, then masks
    __shared__ uint32_t sxm[3];
    __shared__ float szx[44];      // radiation: normals of the structural weights
    static_assert(HID <= 64 && kNIn <= 64, "one table entry per column and row");
    const int n = from_radiation ? w->ctl->n_new : n_host;
    const int32_t* __restrict__ slots = from_radiation ? w->new_slots : w->stage_slots;
    for (int si = blockIdx.x; si < n; si += gridDim.x) {
        const int slot = uniform_i32(slots[si]);
        const int parent = from_radiation == 1 ? uniform_i32(((const int32_t*)w->stage_params)[si]) : -1;
        if (parent >= 0) {  // radiation: hit list (cell, parent) in the staging buffers
            if (threadIdx.x < 14) {
                const int lane = threadIdx.x;
                const int i = w->stage_slots[si];
                const float* pp = w->params + (int64_t)parent * kNParam;
                float* np = w->params + (int64_t)slot * kNParam;
                uint64_t c[4] = {(uint64_t)i, step, (uint64_t)(1 + lane), 0ull};
                philox4x64_10(c, w->seed, 0ull);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float u1 = philox_uniform(c[2 * h]), u2 = philox_uniform(c[2 * h + 1]);
                    const float rr = sqrtf(-2.0f * logf(u1));
                    float sn, cs;
                    sincospif(2.0f * u2, &sn, &cs);
                    const int m = 4 * lane + 2 * h;
                    const float v0 = pp[m] + sigma * (rr * cs), v1 = pp[m + 1] + sigma * (rr * sn);
                    np[m] = v0;
                    np[m + 1] = v1;
                    sp[m] = v0;
                    sp[m + 1] = v1;
                }
            }
            // the structural genes: the parent's; when it has any or structural
            // mutation is on, the enabled genes' weights drift with the same
            // sigma (normal m from the Philox blocks (cell, step, 16 + m / 4,
            // 0), four per lane 14..24) and the block (cell, step, 15, 0)
            // decides NEAT's structural mutations: word 0 below t_conn adds the
            // direct connection (word 2 & 0xffff) mod 10 with weight sigma times
            // its normal; word 1 below t_node adds the node (word 2 >> 16 &
            // 0xffff) mod 16 with activation word 3 & 3, in weight 1 and out
            // weight the child's B[o][j], which it replaces
            if (threadIdx.x >= 64 && threadIdx.x < 64 + kNExtW)
                sxw[threadIdx.x - 64] = w->ext_w[(int64_t)parent * kNExtW + threadIdx.x - 64];
            if (threadIdx.x >= 128 && threadIdx.x < 131)
                sxm[threadIdx.x - 128] = w->ext_mask[(int64_t)parent * 4 + threadIdx.x - 128];
            __syncthreads();
            const bool grow = (w->t_conn | w->t_node) != 0ull;
            if ((sxm[0] | sxm[1]) != 0u || grow) {  // block-uniform
                if (threadIdx.x >= 14 && threadIdx.x < 25) {
                    const int lane = threadIdx.x - 14;
                    const int i = w->stage_slots[si];
                    uint64_t c[4] = {(uint64_t)i, step, (uint64_t)(16 + lane), 0ull};
                    philox4x64_10(c, w->seed, 0ull);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float u1 = philox_uniform(c[2 * h]), u2 = philox_uniform(c[2 * h + 1]);
                        const float rr = sqrtf(-2.0f * logf(u1));
                        float sn, cs;
                        sincospif(2.0f * u2, &sn, &cs);
                        szx[4 * lane + 2 * h] = rr * cs;
                        szx[4 * lane + 2 * h + 1] = rr * sn;
                    }
                }
                __syncthreads();
                if (threadIdx.x < kNExtW) {
                    const int m = threadIdx.x;
                    const uint32_t on = m < 10 ? (sxm[0] >> m) & 1u : (sxm[1] >> (m < 26 ? m - 10 : m - 26)) & 1u;
                    if (on) sxw[m] = sxw[m] + sigma * szx[m];
                }
                __syncthreads();
                if (threadIdx.x == 0 && grow) {
                    const int i = w->stage_slots[si];
                    uint64_t c[4] = {(uint64_t)i, step, 15ull, 0ull};
                    philox4x64_10(c, w->seed, 0ull);
                    if (c[0] < w->t_conn) {
                        const int cc = (int)((c[2] & 0xffffull) % 10ull);
                        if (!((sxm[0] >> cc) & 1u)) {
                            sxm[0] |= 1u << cc;
                            sxw[cc] = sigma * szx[cc];
                        }
                    }
                    if (c[1] < w->t_node) {
                        const int k = (int)(((c[2] >> 16) & 0xffffull) % 16ull);
                        if (!((sxm[1] >> k) & 1u)) {
                            sxm[1] |= 1u << k;
                            sxm[2] = (sxm[2] & ~(3u << (2 * k))) | ((uint32_t)(c[3] & 3ull) << (2 * k));
                            sxw[10 + k] = 1.0f;
                            sxw[26 + k] = sp[40 + 8 * (k & 1) + (k >> 1)];
                        }
                    }
                }
                __syncthreads();
            }
            if (threadIdx.x < kNExtW) w->ext_w[(int64_t)slot * kNExtW + threadIdx.x] = sxw[threadIdx.x];
            if (threadIdx.x < 3) w->ext_mask[(int64_t)slot * 4 + threadIdx.x] = sxm[threadIdx.x];
        } else {
            if (threadIdx.x < kNParam) sp[threadIdx.x] = w->params[(int64_t)slot * kNParam + threadIdx.x];
            if (threadIdx.x >= 64 && threadIdx.x < 64 + kNExtW)
                sxw[threadIdx.x - 64] = w->ext_w[(int64_t)slot * kNExtW + threadIdx.x - 64];
            if (threadIdx.x >= 128 && threadIdx.x < 131)
                sxm[threadIdx.x - 128] = w->ext_mask[(int64_t)slot * 4 + threadIdx.x - 128];
        }
        __syncthreads();
        if (threadIdx.x < NL * 8) {
            const int l = threadIdx.x >> 3, k = threadIdx.x & 7;
            sbase[l][k] = T(sp[5 * k + 1]) * layer_y<T, NL>(l) + T(sp[5 * k + 3]) * layer_y<T, NL>(l + 1) +
                          T(sp[5 * k + 4]);
        }
        __syncthreads();
        bool out_of_range = false;
        for (int t = threadIdx.x; t < NL * (65 + 64); t += 256) {
            if (t < NL * 65) {
                const int l = t / 65, c = t - 65 * l;
                out_of_range |= fill_entry<T>(stc[l][c], sp, 0, sbase[l], c == 64 ? T(0) : col_x<T, NL, HID>(l, c));
            } else {
                const int l = (t - NL * 65) / 64, r = (t - NL * 65) - 64 * l;
                out_of_range |= fill_entry<T>(str[l][r], sp, 2, nullptr, row_x<T, NL, HID>(l, r));
            }
        }
        // block-uniform: only a genome with a part out of range takes the
        // element loop with the direct tanh fallback
        const bool guard = __syncthreads_or(out_of_range);
        const ExtGenes xg{sxm[0], sxm[1], sxm[2], sxw};
        const bool ext = (xg.conn | xg.node) != 0u;  // block-uniform
        uint8_t* dst = w->wfrag + (int64_t)slot * w->wfrag_stride;
        float* bdst = w->bias + (int64_t)slot * w->bias_stride;
        uint32_t bad = 0;
        auto elements = [&](auto guard_c, auto ext_c) {
            constexpr bool GUARD = decltype(guard_c)::value;
            constexpr bool EXT = decltype(ext_c)::value;
            for (int e = threadIdx.x; e < ew + eb; e += 256) {
                float v = 0.0f;
                if (e < ew) {
                    const FragCoord fc = frag_coord(NL, HID, PREC, e);
                    const int lin = fc.layer == 0 ? kNIn : HID, lout = fc.layer == NL - 1 ? kNOut : HID;
                    if (fc.row < lout && fc.col < lin)
                        v = cppn_weight<T, NL, HID, PREC, GUARD, EXT>(sp, stc[fc.layer][fc.col],
                                                                      str[fc.layer][fc.row], fc.layer, fc.row,
                                                                      fc.col, xg);
                } else {
                    int layer, row;
                    bias_coord(NL, HID, e - ew, &layer, &row);
                    if (row < (layer == NL - 1 ? kNOut : HID))
                        v = cppn_bias<T, NL, HID, GUARD, EXT>(sp, stc[layer][64], str[layer][row], layer, row, xg);
                }
                if (!__builtin_isfinite(v)) { bad = kErrNonFinite; v = 0.0f; }
                if (e < ew) {
                    if constexpr (bf) ((__bf16*)dst)[e] = (__bf16)v;
                    else ((float*)dst)[e] = v;
                } else {
                    bdst[e - ew] = v;
                }
            }
        };
        using TrueC = std::integral_constant<bool, true>;
        using FalseC = std::integral_constant<bool, false>;
        if (ext) {
            if (guard) elements(TrueC{}, TrueC{});
            else elements(FalseC{}, TrueC{});
        } else {
            if (guard) elements(TrueC{}, FalseC{});
            else elements(FalseC{}, FalseC{});
        }
        if (bad) atomicOr(&w->ctl->err, bad);
        __syncthreads();  // sp is rewritten for the next genome
    }
}

// Debug: natural flat layout <-> fragment layout of one slot (the stored
// values carry the stored scale factors; the flat layout does not).
__global__ __launch_bounds__(256) void k_pack(const WorldDev* __restrict__ w, int slot,
                                              const float* __restrict__ flat, int unpack,
                                              float* __restrict__ out) {
    const int nl = w->NL, hid = w->HID, prec = w->prec;
    const int ew = net_frags(nl, hid, prec) * net_frag_elems(prec);
    const int eb = net_bias_floats(nl, hid);
    const bool bf = prec == kPrecBF16;
    uint8_t* dst = w->wfrag + (int64_t)slot * w->wfrag_stride;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < ew + eb; e += gridDim.x * 256) {
        if (e < ew) {
            const FragCoord fc = frag_coord(nl, hid, prec, e);
            const int lin = layer_in(nl, hid, fc.layer), lout = layer_out(nl, hid, fc.layer);
            const bool ok = fc.row < lout && fc.col < lin;
            const int fi = flat_w_offset(nl, hid, fc.layer) + fc.row * lin + fc.col;
            const double sc = stored_row_scale(nl, fc.layer, fc.row) * stored_col_scale(prec, fc.layer, fc.col);
            if (!unpack) {
                const float v = ok ? (float)((double)flat[fi] * sc) : 0.0f;
                if (bf) ((__bf16*)dst)[e] = (__bf16)v;
                else ((float*)dst)[e] = v;
            } else if (ok) {
                out[fi] = (float)((bf ? (double)(float)((const __bf16*)dst)[e] : (double)((const float*)dst)[e]) / sc);
            }
        } else {
            int layer, row;
            bias_coord(nl, hid, e - ew, &layer, &row);
            const int lin = layer_in(nl, hid, layer), lout = layer_out(nl, hid, layer);
            const bool ok = row < lout;
            const int fi = flat_w_offset(nl, hid, layer) + lout * lin + row;
            const double sc = stored_row_scale(nl, layer, row);
            float* bp = w->bias + (int64_t)slot * w->bias_stride + (e - ew);
            if (!unpack) *bp = ok ? (float)((double)flat[fi] * sc) : 0.0f;
            else if (ok) out[fi] = (float)((double)*bp / sc);
        }
    }
    if (!unpack && blockIdx.x == 0 && threadIdx.x == 0) w->slot_set[slot] = 1;
}

__global__ __launch_bounds__(256) void k_scatter_params(const WorldDev* __restrict__ w, int n) {
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n * kNParam; e += gridDim.x * 256) {
        const int k = e / kNParam, m = e - k * kNParam;
        const int slot = w->stage_slots[k];
        w->params[(int64_t)slot * kNParam + m] = w->stage_params[e];
        if (m == 0) {
            w->slot_set[slot] = 1;
            // a genome the caller sets is a root of the phylogeny
            w->lineage_parent[slot] = -1;
            w->lineage_parent2[slot] = -1;
            w->lineage_birth[slot] = w->ctl->steps;
        }
        // and has no structural genes until coralai_set_genome_ext adds some
        if (m < kNExtW) w->ext_w[(int64_t)slot * kNExtW + m] = 0.0f;
        if (m < 4) w->ext_mask[(int64_t)slot * 4 + m] = 0u;
    }
}

// coralai_set_genome_ext: n records of 46 words (4 mask words, 42 weights)
// staged in stage_params, for the slots in stage_slots.
__global__ __launch_bounds__(256) void k_scatter_ext(const WorldDev* __restrict__ w, int n) {
    const uint32_t* rec = (const uint32_t*)w->stage_params;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n * 46; e += gridDim.x * 256) {
        const int k = e / 46, m = e - k * 46;
        const int slot = w->stage_slots[k];
        if (m < 4) w->ext_mask[(int64_t)slot * 4 + m] = m < 3 ? rec[e] : 0u;
        else w->ext_w[(int64_t)slot * kNExtW + (m - 4)] = __builtin_bit_cast(float, rec[e]);
    }
}

// NEAT's compatibility distance (genetic similarity) of two genomes:
// c1 E / N + c2 D / N + c3 W.  Genes are numbered by innovation: the 56
// base genes (always present), direct connection q at 56 + q, added node q's
// in and out connections at 66 + 2q, 67 + 2q (present while enabled).
// Matching genes are those both hold; of the others, those beyond the
// smaller of the two highest innovation numbers are excess (E), the rest
// disjoint (D); W is the mean absolute weight difference of the matching
// genes and N the larger genome's gene count.  Without structural genes all
// 56 genes match and the distance is c3 times their mean difference.
__device__ __forceinline__ int top_gene(uint32_t conn, uint32_t node) {
    return node ? 67 + 2 * (31 - __builtin_clz(node)) : (conn ? 56 + (31 - __builtin_clz(conn)) : 55);
}
__global__ __launch_bounds__(256) void k_genetic_distance(const WorldDev* __restrict__ w,
                                                          const int32_t* __restrict__ slots, int na, int nb,
                                                          float c1, float c2, float c3, float* __restrict__ out) {
    const int64_t total = (int64_t)na * nb;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / nb), j = (int)(e - (int64_t)i * nb);
        const int sa = slots[i], sb = slots[na + j];
        const float* pa = w->params + (int64_t)sa * kNParam;
        const float* pb = w->params + (int64_t)sb * kNParam;
        float acc = 0.0f;
#pragma unroll 8
        for (int m = 0; m < kNParam; ++m) acc += fabsf(pa[m] - pb[m]);
        const uint32_t ca = w->ext_mask[(int64_t)sa * 4], cb = w->ext_mask[(int64_t)sb * 4];
        const uint32_t da = w->ext_mask[(int64_t)sa * 4 + 1], db = w->ext_mask[(int64_t)sb * 4 + 1];
        int match = kNParam;
        if ((ca | cb | da | db) == 0u) {
            out[e] = c3 * (acc * (1.0f / kNParam));
            continue;
        }
        const float* xa = w->ext_w + (int64_t)sa * kNExtW;
        const float* xb = w->ext_w + (int64_t)sb * kNExtW;
        const int lim = min(top_gene(ca, da), top_gene(cb, db));
        int E = 0, D = 0;
        for (int q = 0; q < 10; ++q) {
            const bool ha = (ca >> q) & 1u, hb = (cb >> q) & 1u;
            if (ha && hb) { acc += fabsf(xa[q] - xb[q]); ++match; }
            else if (ha || hb) { if (56 + q > lim) ++E; else ++D; }
        }
        for (int q = 0; q < 16; ++q) {
            const bool ha = (da >> q) & 1u, hb = (db >> q) & 1u;
            if (ha && hb) {
                acc += fabsf(xa[10 + q] - xb[10 + q]) + fabsf(xa[26 + q] - xb[26 + q]);
                match += 2;
            } else if (ha || hb) {
                E += (66 + 2 * q > lim) + (67 + 2 * q > lim);
                D += (66 + 2 * q <= lim) + (67 + 2 * q <= lim);
            }
        }
        const int na_g = kNParam + __builtin_popcount(ca) + 2 * __builtin_popcount(da);
        const int nb_g = kNParam + __builtin_popcount(cb) + 2 * __builtin_popcount(db);
        const float N = (float)max(na_g, nb_g);
        out[e] = c1 * ((float)E / N) + c2 * ((float)D / N) + c3 * (acc / (float)match);
    }
}

void launch_genetic_distance(const WorldDev* wdev, const int32_t* slots, int na, int nb, float c1, float c2,
                             float c3, float* out, int n_cu, hipStream_t s) {
    const int64_t total = (int64_t)na * nb;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, (int64_t)n_cu * 8);
    if (blocks > 0)
        hipLaunchKernelGGL(k_genetic_distance, dim3(blocks), dim3(256), 0, s, wdev, slots, na, nb, c1, c2, c3, out);
}

void launch_scatter_ext(const WorldDev* wdev, int n, hipStream_t s) {
    const int blocks = max(1, min(1024, (n * 46 + 255) / 256));
    hipLaunchKernelGGL(k_scatter_ext, dim3(blocks), dim3(256), 0, s, wdev, n);
}

// ------------------------------------------------------------------ radiation

// The neighbour cell i faces (direction R[i]) on the torus.
__device__ __forceinline__ int facing_cell(const WorldDev* __restrict__ w, const uint8_t* __restrict__ R, int i) {
    const int y = i / w->W, x = i - y * w->W, d = R[i] & 7;
    return wrap(y + dir_dy(d), w->H) * w->W + wrap(x + dir_dx(d), w->W);
}

// Hit bits of radiation (MERGE = false, counter word 3 = 0) or of merging
// (word 3 = 1; a candidate is kept only if the cell it faces holds another
// genome), 16 cells per thread, and the count per block.
template <bool MERGE>
__global__ __launch_bounds__(256) void k_rad_hits(const WorldDev* __restrict__ w, uint64_t T,
                                                  uint64_t step) {
    __shared__ int s_cnt;
    const int N = w->N;
    const int32_t* __restrict__ G = w->G[w->ctl->cur];
    const uint8_t* __restrict__ R = w->R[w->ctl->cur];
    for (int blk = blockIdx.x; blk < w->n_rad_blocks; blk += gridDim.x) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const int64_t base = (int64_t)blk * kRadBlockCells + 16 * threadIdx.x;
        uint32_t bits = 0;  // base is a multiple of 16: four whole Philox blocks
#pragma unroll
        for (int q = 0; q < 4; ++q) {  // four independent multiply chains interleave
            const int64_t i0 = base + 4 * q;
            uint64_t c[4] = {(uint64_t)(i0 >> 2), step, 0ull, MERGE ? 1ull : 0ull};
            philox4x64_10(c, w->seed, 0ull);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i0 + k < N && c[k] < T) bits |= 1u << (4 * q + k);
        }
        if (MERGE) {
            for (uint32_t m = bits; m; m &= m - 1) {
                const int j = __builtin_ctz(m);
                const int i = (int)base + j;
                if (G[i] == G[facing_cell(w, R, i)]) bits &= ~(1u << j);
            }
        }
        w->hit_bits[(int64_t)blk * 256 + threadIdx.x] = (uint16_t)bits;
        if (bits) atomicAdd(&s_cnt, __popc(bits));
        __syncthreads();
        if (threadIdx.x == 0) w->blk_hits[blk] = s_cnt;
        __syncthreads();
    }
}

template <int NT>
__device__ __forceinline__ int block_scan_excl(int v, int* total, int* s_tmp) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int y = lane < NT / 64 ? s_tmp[lane] : 0;
#pragma unroll
        for (int o = 1; o < NT / 64; o <<= 1) {
            int z = __shfl_up(y, o, 64);
            if (lane >= o) y += z;
        }
        if (lane < NT / 64) s_tmp[lane] = y;
    }
    __syncthreads();
    const int before = wid > 0 ? s_tmp[wid - 1] : 0;
    *total = s_tmp[NT / 64 - 1];
    __syncthreads();
    return before + x - v;
}

// Hit ranks: exclusive scan of the per-block hit counts.
__global__ __launch_bounds__(1024) void k_rad_scan(const WorldDev* __restrict__ w) {
    __shared__ int s_tmp[16];
    const int nb = w->n_rad_blocks;
    const int per = (nb + 1023) / 1024;
    const int beg = min(nb, (int)threadIdx.x * per), end = min(nb, beg + per);
    int c = 0;
    for (int k = beg; k < end; ++k) c += w->blk_hits[k];
    int tot;
    int o = block_scan_excl<1024>(c, &tot, s_tmp);
    for (int k = beg; k < end; ++k) {
        w->blk_ofs[k] = o;
        o += w->blk_hits[k];
    }
    if (threadIdx.x == 0) {
        w->blk_ofs[nb] = tot;
        Ctl* ctl = w->ctl;
        const int nn = min(tot, ctl->n_free);
        ctl->hits = tot;
        ctl->n_new = nn;
        ctl->dropped = tot - nn;
        ctl->hits_pub = tot;  // the call's published statistics
        ctl->dropped_pub = tot - nn;
    }
}

// The k-th hit (cells in ascending order) takes the k-th free slot: the
// cell's genome becomes the slot, and the hit's cell and parent are listed
// for the mutation kernel.
__global__ __launch_bounds__(256) void k_rad_assign(const WorldDev* __restrict__ w, uint64_t step) {
    __shared__ int s_tmp[4];
    const Ctl* ctl = w->ctl;
    const int cur = ctl->cur;
    const int n_new = ctl->n_new;
    int32_t* G = w->G[cur];
    int32_t* hit_cell = w->stage_slots;                   // free during radiation
    int32_t* hit_parent = (int32_t*)w->stage_params;      // free during radiation
    for (int blk = blockIdx.x; blk < w->n_rad_blocks; blk += gridDim.x) {
        if (w->blk_hits[blk] == 0) continue;  // block-uniform
        const uint32_t bits = w->hit_bits[(int64_t)blk * 256 + threadIdx.x];
        int tot;
        int rank = w->blk_ofs[blk] + block_scan_excl<256>(__popc(bits), &tot, s_tmp);
        for (int j = 0; j < 16; ++j) {
            if (!((bits >> j) & 1u)) continue;
            const int i = blk * kRadBlockCells + 16 * threadIdx.x + j;
            const int parent = G[i];
            if (rank < n_new) w->new_slots[rank] = w->free_list[rank];  // every listed slot is valid
            if (parent < 0 || parent >= w->cap) {  // invalid id: flagged, never dereferenced
                atomicOr(&w->ctl->err, kErrGenomeRange);
                if (rank < n_new) hit_parent[rank] = -1;
            } else if (rank < n_new) {
                const int slot = w->free_list[rank];
                hit_cell[rank] = i;
                hit_parent[rank] = parent;
                hit_parent[w->cap + rank] = -1;  // one parent
                G[i] = slot;
                w->slot_set[slot] = 1;
                w->lineage_parent[slot] = parent;  // the phylogeny's edge
                w->lineage_parent2[slot] = -1;
                w->lineage_birth[slot] = (int64_t)step;
                // the stripe counts stay current
                const int cy = i / w->W, cx = i - cy * w->W;
                int32_t* sc = w->stripe_counts + (int64_t)cell_stripe(cx, cy, w->btiles_x) * w->cap;
                atomicAdd(sc + parent, -1);
                atomicAdd(sc + slot, 1);
            }
            ++rank;
        }
    }
}


// ------------------------------------------------------------------ merging

// The k-th merge (cells in ascending order) is listed with its cell and its
// two parents, read from the genome map before any merge of the call
// changes it (the commit kernel runs after this one).
__global__ __launch_bounds__(256) void k_merge_pairs(const WorldDev* __restrict__ w) {
    __shared__ int s_tmp[4];
    const Ctl* ctl = w->ctl;
    const int cur = ctl->cur;
    const int n_new = ctl->n_new;
    const int32_t* __restrict__ G = w->G[cur];
    const uint8_t* __restrict__ R = w->R[cur];
    int32_t* hit_cell = w->stage_slots;                   // free during merging
    int32_t* hit_a = (int32_t*)w->stage_params;           // [cap] own genome
    int32_t* hit_b = hit_a + w->cap;                      // [cap] the partner's
    for (int blk = blockIdx.x; blk < w->n_rad_blocks; blk += gridDim.x) {
        if (w->blk_hits[blk] == 0) continue;  // block-uniform
        const uint32_t bits = w->hit_bits[(int64_t)blk * 256 + threadIdx.x];
        int tot;
        int rank = w->blk_ofs[blk] + block_scan_excl<256>(__popc(bits), &tot, s_tmp);
        for (uint32_t m = bits; m; m &= m - 1, ++rank) {
            if (rank >= n_new) break;
            const int i = blk * kRadBlockCells + 16 * threadIdx.x + __builtin_ctz(m);
            const int a = G[i], b = G[facing_cell(w, R, i)];
            w->new_slots[rank] = w->free_list[rank];  // every listed slot is valid
            hit_cell[rank] = i;
            if (a < 0 || a >= w->cap || b < 0 || b >= w->cap) {  // invalid id: flagged, never dereferenced
                atomicOr(&w->ctl->err, kErrGenomeRange);
                hit_a[rank] = -1;
                hit_b[rank] = -1;
            } else {
                hit_a[rank] = a;
                hit_b[rank] = b;
            }
        }
    }
}

// One thread per listed merge: the child's parameters (gene m from the
// partner where bit m of the mask word is set), its cell's genome, the
// phylogeny (both parents) and the stripe counts.  Children take free slots
// and parents are live, so no thread reads a slot another one writes.
__global__ __launch_bounds__(256) void k_merge_commit(const WorldDev* __restrict__ w, uint64_t step) {
    const int n_new = w->ctl->n_new;
    int32_t* G = w->G[w->ctl->cur];
    const int32_t* hit_a = (const int32_t*)w->stage_params;
    const int32_t* hit_b = hit_a + w->cap;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n_new; k += gridDim.x * 256) {
        const int a = hit_a[k], b = hit_b[k];
        if (a < 0) continue;
        const int i = w->stage_slots[k], slot = w->new_slots[k];
        uint64_t c[4] = {(uint64_t)i, step, 0ull, 2ull};
        philox4x64_10(c, w->seed, 0ull);
        const uint64_t mask = c[0];
        const float* pa = w->params + (int64_t)a * kNParam;
        const float* pb = w->params + (int64_t)b * kNParam;
        float* pc = w->params + (int64_t)slot * kNParam;
        for (int m = 0; m < kNParam; ++m) pc[m] = ((mask >> m) & 1ull) ? pb[m] : pa[m];
        // structural genes: each direct-connection position (bit of word 1)
        // and added-node position (bit of word 2) whole from b or from a
        const uint32_t* ma = w->ext_mask + (int64_t)a * 4;
        const uint32_t* mb = w->ext_mask + (int64_t)b * 4;
        const float* xa = w->ext_w + (int64_t)a * kNExtW;
        const float* xb = w->ext_w + (int64_t)b * kNExtW;
        float* xc = w->ext_w + (int64_t)slot * kNExtW;
        uint32_t conn = 0u, node = 0u, act = 0u;
        for (int q = 0; q < 10; ++q) {
            const bool fb = (c[1] >> q) & 1ull;
            conn |= (fb ? mb[0] : ma[0]) & (1u << q);
            xc[q] = fb ? xb[q] : xa[q];
        }
        for (int q = 0; q < 16; ++q) {
            const bool fb = (c[2] >> q) & 1ull;
            node |= (fb ? mb[1] : ma[1]) & (1u << q);
            act |= (fb ? mb[2] : ma[2]) & (3u << (2 * q));
            xc[10 + q] = fb ? xb[10 + q] : xa[10 + q];
            xc[26 + q] = fb ? xb[26 + q] : xa[26 + q];
        }
        uint32_t* mc = w->ext_mask + (int64_t)slot * 4;
        mc[0] = conn;
        mc[1] = node;
        mc[2] = act;
        mc[3] = 0u;
        G[i] = slot;
        w->slot_set[slot] = 1;
        w->lineage_parent[slot] = a;
        w->lineage_parent2[slot] = b;
        w->lineage_birth[slot] = (int64_t)step;
        const int cy = i / w->W, cx = i - cy * w->W;
        int32_t* sc = w->stripe_counts + (int64_t)cell_stripe(cx, cy, w->btiles_x) * w->cap;
        atomicAdd(sc + a, -1);
        atomicAdd(sc + slot, 1);
    }
}

template <int NL, int HID, int PREC>
static void launch_cppn_t(const WorldDev* wdev, int from_radiation, int n_host, uint64_t step, float sigma,
                          int n_cu, hipStream_t s) {
    // one block per genome (the count of a radiation call is known on the device only)
    hipLaunchKernelGGL((k_cppn<NL, HID, PREC>), dim3(n_cu * 16), dim3(256), 0, s, wdev, from_radiation, n_host,
                       step, sigma);
}

void launch_cppn(const WorldDev* wdev, int nl, int hid, int prec, int from_radiation, int n_host, uint64_t step,
                 float sigma, int n_cu, hipStream_t s) {
    const bool bf = prec == kPrecBF16;
    auto go = [&](auto fn) { fn(wdev, from_radiation, n_host, step, sigma, n_cu, s); };
    if (nl == 2 && hid == 32) bf ? go(launch_cppn_t<2, 32, kPrecBF16>) : go(launch_cppn_t<2, 32, kPrecFP32>);
    else if (nl == 2) bf ? go(launch_cppn_t<2, 64, kPrecBF16>) : go(launch_cppn_t<2, 64, kPrecFP32>);
    else if (hid == 32) bf ? go(launch_cppn_t<3, 32, kPrecBF16>) : go(launch_cppn_t<3, 32, kPrecFP32>);
    else bf ? go(launch_cppn_t<3, 64, kPrecBF16>) : go(launch_cppn_t<3, 64, kPrecFP32>);
}

void launch_scatter_params(const WorldDev* wdev, int n, hipStream_t s) {
    const int blocks = max(1, min(1024, (n * kNParam + 255) / 256));
    hipLaunchKernelGGL(k_scatter_params, dim3(blocks), dim3(256), 0, s, wdev, n);
}

void launch_pack_weights(const WorldDev* wdev, int slot, const float* flat, int unpack, float* out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(64), dim3(256), 0, s, wdev, slot, flat, unpack, out);
}

void launch_radiate(const BatchDev* bdev, const WorldDev* wdev, const LaunchShape& ls, int nl, int hid,
                    int prec, int n_rad_blocks, uint64_t T, float sigma, uint64_t step, hipStream_t s,
                    int recount) {
    // free slots of the current state (the completed step's result), listed by
    // the slot scan; the counting pass inside runs only if the counts are not
    // current (right after a step they are)
    launch_hist_only(bdev, ls, s, 1, recount);
    const int hb = max(1, min(n_rad_blocks, ls.n_cu * 8));
    // the hit test is a chain of 64-bit multiplies per cell: as many waves as fit
    const int hh = max(1, min(n_rad_blocks, ls.n_cu * 32));
    hipLaunchKernelGGL(k_rad_hits<false>, dim3(hh), dim3(256), 0, s, wdev, T, step);
    hipLaunchKernelGGL(k_rad_scan, dim3(1), dim3(1024), 0, s, wdev);
    hipLaunchKernelGGL(k_rad_assign, dim3(hb), dim3(256), 0, s, wdev, step);
    launch_cppn(wdev, nl, hid, prec, 1, 0, step, sigma, ls.n_cu, s);  // mutation, then the networks
}

void launch_merge(const BatchDev* bdev, const WorldDev* wdev, const LaunchShape& ls, int nl, int hid, int prec,
                  int n_rad_blocks, uint64_t T, uint64_t step, hipStream_t s, int recount) {
    launch_hist_only(bdev, ls, s, 1, recount);  // free slots of the current state
    const int hb = max(1, min(n_rad_blocks, ls.n_cu * 8));
    const int hh = max(1, min(n_rad_blocks, ls.n_cu * 32));
    hipLaunchKernelGGL(k_rad_hits<true>, dim3(hh), dim3(256), 0, s, wdev, T, step);
    hipLaunchKernelGGL(k_rad_scan, dim3(1), dim3(1024), 0, s, wdev);
    hipLaunchKernelGGL(k_merge_pairs, dim3(hb), dim3(256), 0, s, wdev);
    hipLaunchKernelGGL(k_merge_commit, dim3(max(1, ls.n_cu)), dim3(256), 0, s, wdev, step);
    launch_cppn(wdev, nl, hid, prec, 2, 0, step, 0.0f, ls.n_cu, s);  // the children's networks
}

}  // namespace coralai
