// Sense -> act: the per-cell network of the cell's genome, run as a grouped
// GEMM on MFMA, followed by the actuator epilogue (System Design: each cell
// sends its Kernel neighbourhood of Sensor channels to its network and
// receives Actuator values; Experiment: invest / liquidate, sigmoid
// communication, explore actuators one per kernel offset).
//
// Work unit: 64 cells of one genome taken from the bucket order (one
// wavefront).  Each wavefront owns a contiguous range of units, so it keeps
// its genome's weights in registers across units and reloads them only at
// genome boundaries.  Per unit:
//   1. every lane gathers its cell's 54 sensor values (rotation-ordered 3x3
//      Moore kernel, periodic) straight from HBM/L2 and writes them to the
//      wavefront's LDS stage as one row (bf16 or fp32);
//   2. the cells are the MFMA B operand (16 per column group), the weights
//      the A operand; hidden layers stay in registers because the MFMA
//      output layout is reused as the next layer's B layout (tanh in FP32,
//      then RNE to bf16 in the BF16 form);
//   3. the 14 actuators go through LDS back to one cell per lane, and the
//      epilogue computes the ledger conversion, the sigmoid communication,
//      the quantised softmax flow plan and the argmax exploration, writing
//      C' and the boundary record: E1 and I1 as one ledger pair, and the 8
//      flows, each tagged with whether it is the explored direction, as one
//      32-byte record in direction order.  Every store of a cell is 16 or 32
//      contiguous bytes, so a 16-cell row of a unit writes whole cache lines.
#include <type_traits>

#include "coralai_internal.h"

namespace coralai {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int NL, int HID, int PREC>
struct Net {
    static constexpr bool kBF = PREC == kPrecBF16;
    static constexpr int MT = HID / 16;
    static constexpr int KS0 = net_ks0(PREC);
    static constexpr int KSH = net_ksh(HID, PREC);
    static constexpr int F0 = MT * KS0;
    static constexpr int F1 = NL == 3 ? MT * KSH : 0;
    static constexpr int FRAG_BYTES = net_frag_bytes(PREC);
    static constexpr int STAGE_ROW = kBF ? 144 : 272;  // bytes per cell row (padded)
    static constexpr int BIAS_BYTES = 4 * net_bias_floats(NL, HID);
    static constexpr int STAGE_BYTES = 64 * STAGE_ROW + BIAS_BYTES;  // stage, then the biases
    static constexpr int ACT_ROW = 80;                 // 16 floats + 4 pad, conflict free
    using frag_t = typename std::conditional<kBF, bf16x8, float>::type;
};

// Hidden activation r = 1 / (2^y + 1) = (1 - tanh(x)) / 2 on y = 2 log2(e) x:
// one exp2 and one reciprocal, exact limits.  The stored weights carry the
// argument scale.  BF16 networks feed r to the next layer, whose weights
// carry the -2 and the row-sum bias correction that turn r back into tanh;
// FP32 networks feed tanh = 1 - 2r.
__device__ __forceinline__ float tanh_r(float y) {
    return __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f);
}
// tanh itself, from the odd symmetry: 1 - 2r on |y| (r <= 1/2), sign of y.
// r below 1/2 keeps the absolute error of 1 - 2r at the rounding of r, where
// r near 1 (tanh near -1) would carry the rounding of 1 into it.
__device__ __forceinline__ float tanh_t(float y) {
    return __builtin_copysignf(__builtin_fmaf(-2.0f, tanh_r(__builtin_fabsf(y)), 1.0f), y);
}

// sigmoid on an actuator stored times -log2(e): 1 / (1 + 2^x)
__device__ __forceinline__ float sigmoid_s(float x) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(x));
}

__device__ __forceinline__ floatx4 mfma(const bf16x8& a, const bf16x8& b, const floatx4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma(float a, float b, const floatx4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS hand-off between lanes of one wavefront: LDS operations of a wave
// complete in order, so waiting for the LDS counter alone (not for vector
// memory, whose counter also holds outstanding global stores) suffices.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt / expcnt unconstrained
    __builtin_amdgcn_wave_barrier();
}

// Flow plan helpers of the physics variants.  A budget split by the softmax
// weights ex / sum (inv = 1 / sum) with a running clamp, in kernel-position
// order; or all of it to the maximal position.
__device__ __forceinline__ void split_soft(uint32_t budget, const float (&ex)[8], float inv, uint32_t (&out)[8]) {
    const float per = inv * (float)budget;
    uint32_t used = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        uint32_t f = (uint32_t)(ex[t] * per);  // >= 0 and finite: truncation is the floor
        const uint32_t rem = budget - used;
        f = f < rem ? f : rem;
        used += f;
        out[t] = f;
    }
}
__device__ __forceinline__ void split_hard(uint32_t budget, int best, uint32_t (&out)[8]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) out[t] = t == best ? budget : 0u;
}
// Kernel position t + 1 points at direction (r + offset) & 7: the words in
// offset order, then rotated by r, one conditional rotation per bit of r.
__device__ __forceinline__ void to_directions(const uint32_t (&fs)[8], int r, uint32_t (&dst)[8]) {
    uint32_t wd[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) wd[kernel_offset(t + 1)] = fs[t];
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1) {
        const bool on = (r & bit) != 0;
        uint32_t nw[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) nw[d] = on ? wd[(d - bit) & 7] : wd[d];
#pragma unroll
        for (int d = 0; d < 8; ++d) wd[d] = nw[d];
    }
#pragma unroll
    for (int d = 0; d < 8; ++d) dst[d] = wd[d];
}

// floor(max(x, 0)) as a 64-bit integer, for x below 2^63: the high word is
// floor(x 2^-32) and the low word the exact remainder (both conversions of
// integral non-negative values)
__device__ __forceinline__ int64_t floor_nonneg_i64(float x) {
    const float v = __builtin_floorf(__builtin_fmaxf(x, 0.0f));
    const float hi = __builtin_floorf(v * 0x1p-32f);
    const uint32_t h = (uint32_t)hi, l = (uint32_t)__builtin_fmaf(hi, -0x1p32f, v);
    return (int64_t)(((uint64_t)h << 32) | l);
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NL, int HID, int PREC, int CGI, int WAVES, bool DEBUG, bool VARIANTS>
__global__ __launch_bounds__(256, WAVES) void k_act(
    const BatchDev* __restrict__ b, float* __restrict__ dbg, int seg_force) {
    using NT = Net<NL, HID, PREC>;
    using frag_t = typename NT::frag_t;
    constexpr int MT = NT::MT, KS0 = NT::KS0, KSH = NT::KSH;
    constexpr int MT1 = NL == 3 ? MT : 1;
    static_assert(4 % CGI == 0, "column groups per pass must divide 4");
    static_assert(hidden_input_is_r(PREC) == NT::kBF, "BF16 layers read r, FP32 layers read tanh");

    __shared__ __attribute__((aligned(16))) uint8_t smem[4 * NT::STAGE_BYTES];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane >> 4, n16 = lane & 15;
    uint8_t* stage = smem + wv * NT::STAGE_BYTES;
    // the current genome's biases live in LDS: reading them must not wait on
    // the vector-memory counter, which also covers the previous unit's stores
    float* sbias = (float*)(stage + 64 * NT::STAGE_ROW);

    const int nworlds = cld(&b->n_worlds);
    if (nworlds <= 0) return;
    const int total = cld(b->group_prefix + (nworlds));
    // chunks of ceil(total / waves) units: a small job keeps fewer waves busy,
    // each with more units, which pays each wave's run setup (genome lookup,
    // weights, biases) fewer times than one unit per wave would.  A large job
    // is cut into nseg equal segments and a wave takes one chunk from each:
    // the units of one-cell genomes (which radiation puts in the lowest free
    // slots, mostly past the initial genomes) then spread over all waves
    // instead of loading the waves at the end of the list.  (FP32 networks,
    // with twice the weight bytes per run start, keep one segment.)
    const int nwaves = gridDim.x * 4;
    const int nseg = seg_force > 0 ? seg_force : (NT::kBF && total >= 64 * nwaves ? 4 : 1);
    const int seglen = (total + nseg - 1) / nseg;
    const int per = (seglen + nwaves - 1) / nwaves;
    const int wid = xcd_block() * 4 + wv;
    int seg = 0;
    int u = 0, uend = 0;
    auto enter_segment = [&]() {
        u = uniform_i32(min(total, seg * seglen + wid * per));
        uend = uniform_i32(min(min(total, (seg + 1) * seglen), u + per));
    };
    enter_segment();
    while (u >= uend && seg + 1 < nseg) {
        ++seg;
        enter_segment();
    }
    if (u >= uend) return;  // no block-wide barriers below: waves are independent

    frag_t w0[MT][KS0];
    frag_t w1[MT1][KSH];
    frag_t wo[KSH];

    int wi = uniform_i32(find_world(b->group_prefix, nworlds, u));
    int world_lo = 0, world_hi = -1;
    int g = -1, g_lo = 0, g_hi = -1;
    int64_t acc_mass = 0;
    uint32_t err = 0;
    // the next unit's perm entry (cell index | rotation), loaded while this unit computes
    bool have_pf = false;
    int e_pf = 0;
    // Stores of a unit are issued after the next unit's loads: one counter
    // tracks vector loads and stores in issue order, so a load issued after
    // a store could not be waited for without waiting for the store too.
    bool st_pending = false;
    int st_i = -1;
    uint32_t st_c[4] = {0u, 0u, 0u, 0u}, st_f[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    uint32_t st_e[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    int64_t st_E1 = 0, st_I1 = 0;

    // world fields kept in scalar registers
    int Wd = 0, Hd = 0, Nd = 0, cap = 0;
    uint32_t w_magic = 1u;
    int w_shift = 0;
    float rho_i = 0.f, rho_l = 0.f, kappa = 0.f;
    // physics variants in one scalar (bit 0: hard-max exploration, bit 1:
    // energy transport), in the kernel compiled with VARIANTS only; their
    // parameters are read from the world's table where used
    int variant = 0;
    __amdgpu_buffer_rsrc_t rEI, rC, rP, wC, wEI1, wFlow;
    const int32_t *counts = nullptr, *offsets = nullptr, *gofs = nullptr;
    const uint8_t* wfrag = nullptr;
    const float* bias = nullptr;
    const float* gbias = sbias + 4 * q;  // this lane's rows of the current genome's biases
    int64_t wstride = 0;
    int bstride = 0;
    Ctl* ctl = nullptr;

    auto flush = [&]() {
        // each lane's exact partial, then the FP64 sum over lanes and waves
        const double mf = wave_sum_f64((double)acc_mass);
        const int64_t m = wave_sum_i64(acc_mass);
        if (lane == 0 && ctl != nullptr) {
            atomicAdd((unsigned long long*)&ctl->acc_mass, (unsigned long long)m);
            atomicAdd(&ctl->acc_mass_f64, mf);
        }
        if (err && ctl != nullptr) atomicOr(&ctl->err, err);
        acc_mass = 0;
        err = 0;
    };

    // A lane with nothing to store (st_i < 0) stores at the end of each
    // buffer, where a raw buffer store is discarded: the stores are issued by
    // every lane of every unit, so the wait counts around them are exact.
    auto store_results = [&]() {
        const uint32_t ofs = st_i >= 0 ? 4u * (uint32_t)st_i : 4u * (uint32_t)Nd;
        // the results are read by the physics kernel, not here: streaming stores
        buf_st_f32x4<kCpolNT>(coralai_f32x4{__builtin_bit_cast(float, st_c[0]), __builtin_bit_cast(float, st_c[1]),
                                   __builtin_bit_cast(float, st_c[2]), __builtin_bit_cast(float, st_c[3])},
                     wC, 4 * ofs);
        __builtin_amdgcn_raw_buffer_store_b128(coralai_u32x4{st_f[0], st_f[1], st_f[2], st_f[3]}, wFlow, 8 * ofs, 0, kCpolNT);
        __builtin_amdgcn_raw_buffer_store_b128(coralai_u32x4{st_f[4], st_f[5], st_f[6], st_f[7]}, wFlow, 8 * ofs + 16, 0, kCpolNT);
        buf_st_i64x2<kCpolNT>(i64x2{st_E1, st_I1}, wEI1, 4 * ofs);
        if (VARIANTS && (variant & 2)) {  // world-uniform: energy transport records
            const __amdgpu_buffer_rsrc_t wEflow = buf_rsrc(world_at(b, wi)->eflow, 32u * (uint32_t)Nd);
            __builtin_amdgcn_raw_buffer_store_b128(coralai_u32x4{st_e[0], st_e[1], st_e[2], st_e[3]}, wEflow, 8 * ofs, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b128(coralai_u32x4{st_e[4], st_e[5], st_e[6], st_e[7]}, wEflow, 8 * ofs + 16, 0, 0);
        }
        st_i = -1;
        st_pending = false;
    };

    // One loop over the wave's units.  A unit that starts a run of a new
    // genome looks the genome up, issues its gather and then the genome's
    // weight loads; the bias and row-sum set-up follows the conversion of the
    // gathered values.  Weights stay in registers for the rest of the run.
    int run_end = -1;  // first unit past the current run
    int gcount = 0, goff = 0;
    floatx4 bias_ld = {0.f, 0.f, 0.f, 0.f};
    while (u < uend) {
        if (u >= world_hi) {
            if (st_pending) store_results();  // the buffers below change with the world
            flush();
            while (cld(b->group_prefix + (wi + 1)) <= u) ++wi;
            wi = uniform_i32(wi);
            world_lo = cld(b->group_prefix + (wi));
            world_hi = cld(b->group_prefix + (wi + 1));
            const auto* W = world_at(b, wi);
            Wd = W->W; Hd = W->H; Nd = W->N; cap = W->cap;
            w_magic = W->w_magic; w_shift = W->w_shift;
            rho_i = W->rho_i; rho_l = W->rho_l; kappa = W->kappa;
            if constexpr (VARIANTS)
                variant = (W->explore_mode == 1 ? 1 : 0) | (W->eflow != nullptr && W->kappa_e > 0.f ? 2 : 0);
            ctl = W->ctl;
            const int cur = ctl_cur(ctl), nxt = cur ^ 1;
            const uint32_t n4 = 4u * (uint32_t)Nd;
            rEI = buf_rsrc(W->EI[cur], 4u * n4);
            rC = buf_rsrc(W->C[cur], 4u * n4);
            rP = buf_rsrc(W->perm, n4);
            wC = buf_rsrc(W->C[nxt], 4u * n4);
            wEI1 = buf_rsrc(W->EI1, 4u * n4);
            wFlow = buf_rsrc(W->flow, 8u * n4);
            counts = W->counts; offsets = W->offsets; gofs = W->gofs;
            wfrag = W->wfrag; bias = W->bias; wstride = W->wfrag_stride; bstride = W->bias_stride;
            g = -1;
            run_end = -1;
            have_pf = false;
        }
        const bool new_run = u >= run_end;
        if (new_run) {
            const int k0 = u - world_lo;
            // the run's genome: short linear probe, else binary search over gofs
            int gn = -1;
            if (g >= 0) {
#pragma unroll 1
                for (int t = g + 1; t < min(cap, g + 5); ++t)
                    if (cld(gofs + t + 1) > k0) { gn = t; break; }
            }
            if (gn < 0) {
                // the largest g with gofs[g] <= k0, by a 64-way search: each lane
                // probes one of 64 evenly spaced slots of [lo, hi], and the
                // probes at or below k0 are a prefix (gofs does not decrease)
                int lo = 0, hi = cap - 1;
                while (lo < hi) {
                    const int step = (hi - lo + 63) / 64;
                    const int pos = min(hi, lo + (lane + 1) * step);
                    const int nle = (int)__popcll(__ballot(cld(gofs + pos) <= k0));
                    const int nlo = nle > 0 ? min(hi, lo + nle * step) : lo;
                    hi = nle < 64 ? min(hi, lo + (nle + 1) * step) - 1 : hi;
                    lo = uniform_i32(nlo);
                    hi = uniform_i32(hi);
                }
                gn = lo;
            }
            g = uniform_i32(gn);
            g_lo = cld(gofs + g);
            g_hi = cld(gofs + g + 1);
            run_end = min(uend, world_lo + g_hi);
            gcount = cld(counts + g);
            goff = cld(offsets + g);
        }
        const int j = u - world_lo - g_lo;
        const int cell0 = goff + j * kGroupCells;
        const int cnt = min(kGroupCells, gcount - j * kGroupCells);
        const bool valid = lane < cnt;
        // a prefetched entry of a lane past the unit's cells is replaced by
        // lane 0's, so that such lanes gather the addresses lane 0 gathers.
        // Each branch waits for its own load (the empty asm uses the value),
        // so the prefetched path does not wait for the stores issued after it.
        int entry;
        if (have_pf) {
            const int e0 = __builtin_amdgcn_readfirstlane(e_pf);
            entry = valid ? e_pf : e0;
        } else {
            entry = (int)__builtin_amdgcn_raw_buffer_load_b32(rP, 4 * (cell0 + (valid ? lane : 0)), 0, 0);
            asm volatile("" : "+v"(entry));
        }
        const int i = entry & kPermIndexMask, r = (entry >> kPermRotShift) & 7;
        // ---- 1. sense: rotation-ordered 3x3 Moore kernel, 6 channels.
        // The 8 neighbours in direction order from the wrapped columns and
        // row bases, then rotated by r (one conditional rotation per bit of
        // r): kernel position p reads direction (r + offset(p)) & 7.
        const int y = cell_row(i, w_magic, w_shift), x = i - y * Wd;
        const int xm = (x == 0 ? Wd : x) - 1, xp = x + 1 == Wd ? 0 : x + 1;
        const int r0 = i - x, rm = (y == 0 ? Nd : r0) - Wd, rp = y + 1 == Hd ? 0 : r0 + Wd;
        int dn[8] = {r0 + xp, rm + xp, rm + x, rm + xm, r0 + xm, rp + xm, rp + x, rp + xp};
#pragma unroll
        for (int sh = 0; sh < 3; ++sh) {
            // an all-ones or all-zeros lane mask, opaque to the compiler so
            // that each stage stays one bitfield select per entry
            int m = -((r >> sh) & 1);
            asm volatile("" : "+v"(m));
            int nd[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) nd[k] = (dn[(k + (1 << sh)) & 7] & m) | (dn[k] & ~m);
#pragma unroll
            for (int k = 0; k < 8; ++k) dn[k] = nd[k];
        }
        int nidx[9];
        nidx[0] = i;
#pragma unroll
        for (int p = 1; p < 9; ++p) nidx[p] = dn[kernel_offset(p)];
        int64_t gE[9], gI[9];
        float gC[9][4];
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const i64x2 ei = buf_ld_i64x2(rEI, 16 * nidx[p]);
            gE[p] = ei[0];
            gI[p] = ei[1];
            const coralai_f32x4 cv = buf_ld_f32x4(rC, 16 * nidx[p]);
#pragma unroll
            for (int c = 0; c < 4; ++c) gC[p][c] = cv[c];
        }
        // Loads in issue order: the gather, a new run's weights, the next
        // unit's cell indices; then the previous unit's stores.  One counter
        // covers them all and they complete in order, so each wait below
        // leaves what was issued after its operand in flight.
        if (new_run) {
            // weights of genome g -> registers, with the non-temporal hint (each
            // run reads them once; the gather's lines are the ones worth keeping)
            const uint8_t* wb = wfrag + (int64_t)g * wstride + lane * (NT::FRAG_BYTES / 64);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int s = 0; s < KS0; ++s)
                    w0[mt][s] = __builtin_nontemporal_load((const frag_t*)(wb + (mt * KS0 + s) * NT::FRAG_BYTES));
            if constexpr (NL == 3) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int s = 0; s < KSH; ++s)
                        w1[mt][s] = __builtin_nontemporal_load((const frag_t*)(wb + (NT::F0 + mt * KSH + s) * NT::FRAG_BYTES));
            }
#pragma unroll
            for (int s = 0; s < KSH; ++s)
                wo[s] = __builtin_nontemporal_load((const frag_t*)(wb + (NT::F0 + NT::F1 + s) * NT::FRAG_BYTES));
            static_assert(net_bias_floats(NL, HID) / 4 <= 64, "one bias load per lane");
            if (lane < net_bias_floats(NL, HID) / 4)
                bias_ld = gld((const floatx4*)(bias + (int64_t)g * bstride + 4 * lane));
        }
        // the next unit's cell indices: within the run, or the first unit of
        // the next run, whose genome's cells follow this genome's in the
        // world's perm (reads past the buffer return 0)
        // (issued by every unit, used only when have_pf)
        have_pf = u + 1 < uend && u + 1 < world_hi;
        {
            const bool same = u + 1 < run_end;
            const int next0 = same ? cell0 + kGroupCells : goff + gcount;
            const int cnt_n = same ? min(kGroupCells, gcount - (j + 1) * kGroupCells) : kGroupCells;
            e_pf = (int)__builtin_amdgcn_raw_buffer_load_b32(rP, 4 * (next0 + (lane < cnt_n ? lane : 0)), 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        store_results();  // the previous unit's results (past the buffers if none)
        __builtin_amdgcn_sched_barrier(0);
        const int64_t e_own = gE[0], i_own = gI[0];
        float uvec[kNIn];
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            uvec[6 * p + 0] = i64_to_f32(gE[p]);  // the 2^-24 quantum is in the weights
            uvec[6 * p + 1] = i64_to_f32(gI[p]);
#pragma unroll
            for (int c = 0; c < 4; ++c) uvec[6 * p + 2 + c] = gC[p][c];
        }
        if constexpr (NT::kBF) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                bf16x8 row;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int kk = 8 * t + e;
                    row[e] = (__bf16)(kk < kNIn ? uvec[kk] : 0.0f);
                }
                *(bf16x8*)(stage + lane * NT::STAGE_ROW + 16 * t) = row;
            }
        } else {
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                floatx4 v[4];
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    const int kk = 4 * s + qq;
                    v[s >> 2][s & 3] = (s < 14 && kk < kNIn) ? uvec[kk] : 0.0f;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    *(floatx4*)(stage + lane * NT::STAGE_ROW + qq * 64 + 16 * t) = v[t];
            }
        }
        wave_lds_sync();

        if (new_run) {
            if (lane < net_bias_floats(NL, HID) / 4) *(floatx4*)(sbias + 4 * lane) = bias_ld;
            wave_lds_sync();
            // BF16: layers after a hidden layer read r = (1 - tanh) / 2
            // through weights stored times -2: their biases gain -1/2 of the
            // stored row sums (an MFMA against a ones operand)
            if constexpr (hidden_input_is_r(PREC)) {
                frag_t ones;
                if constexpr (NT::kBF) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;
                } else {
                    ones = 1.0f;
                }
                if constexpr (NL == 3) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        floatx4 rs = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int s = 0; s < KSH; ++s) rs = mfma(w1[mt][s], ones, rs);
                        if (n16 == 0) {
                            floatx4* bp = (floatx4*)(sbias + HID + 16 * mt + 4 * q);
                            *bp = *bp - 0.5f * rs;
                        }
                    }
                }
                floatx4 rs = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < KSH; ++s) rs = mfma(wo[s], ones, rs);
                if (n16 == 0) {
                    floatx4* bp = (floatx4*)(sbias + (NL == 3 ? 2 * HID : HID) + 4 * q);
                    *bp = *bp - 0.5f * rs;
                }
                wave_lds_sync();
            }
        }
        // ---- 2. the network, G column groups of 16 cells per pass (pass cb
        // covers groups cb G .. cb G + G - 1)
        floatx4 outv[4];
        auto pass = [&](auto g_const, int cb) __attribute__((always_inline)) {
            constexpr int G = decltype(g_const)::value;
            floatx4 acc[G][MT];
            floatx4 bv0[MT];  // the biases enter as the first MFMA's accumulator
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) bv0[mt] = *(const floatx4*)(gbias + 16 * mt);
            if constexpr (NT::kBF) {
                bf16x8 xin[G][KS0];
#pragma unroll
                for (int cc = 0; cc < G; ++cc)
#pragma unroll
                    for (int s = 0; s < KS0; ++s)
                        xin[cc][s] = *(const bf16x8*)(stage + (16 * (cb * G + cc) + n16) * NT::STAGE_ROW +
                                                      (16 * q + 8 * s) * 2);
#pragma unroll
                for (int s = 0; s < KS0; ++s)
#pragma unroll
                    for (int cc = 0; cc < G; ++cc)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            acc[cc][mt] = mfma(w0[mt][s], xin[cc][s], s == 0 ? bv0[mt] : acc[cc][mt]);
            } else {
                float xin[G][16];
#pragma unroll
                for (int cc = 0; cc < G; ++cc)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const floatx4 v = *(const floatx4*)(stage + (16 * (cb * G + cc) + n16) * NT::STAGE_ROW +
                                                            q * 64 + 16 * t);
                        xin[cc][4 * t + 0] = v[0]; xin[cc][4 * t + 1] = v[1];
                        xin[cc][4 * t + 2] = v[2]; xin[cc][4 * t + 3] = v[3];
                    }
#pragma unroll
                for (int s = 0; s < KS0; ++s)
#pragma unroll
                    for (int cc = 0; cc < G; ++cc)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            acc[cc][mt] = mfma(w0[mt][s], xin[cc][s], s == 0 ? bv0[mt] : acc[cc][mt]);
            }
            // hidden layers
#pragma unroll
            for (int layer = 1; layer < NL; ++layer) {
                const bool last = layer == NL - 1;
                const float* lb = gbias + (last ? (NL == 3 ? 2 * HID : HID) : HID);
                if constexpr (NT::kBF) {
                    bf16x8 h[G][KSH];
#pragma unroll
                    for (int cc = 0; cc < G; ++cc)
#pragma unroll
                        for (int s = 0; s < KSH; ++s)
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                h[cc][s][t] = (__bf16)tanh_r(acc[cc][2 * s][t]);  // r is rounded
                                h[cc][s][4 + t] = (__bf16)tanh_r(acc[cc][2 * s + 1][t]);
                            }
                    if (last) {
                        const floatx4 bv = *(const floatx4*)lb;
#pragma unroll
                        for (int cc = 0; cc < G; ++cc) {
                            floatx4 o = mfma(wo[0], h[cc][0], bv);
#pragma unroll
                            for (int s = 1; s < KSH; ++s) o = mfma(wo[s], h[cc][s], o);
                            outv[cb * G + cc] = o;
                        }
                    } else {
                        floatx4 bvh[MT];
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) bvh[mt] = *(const floatx4*)(lb + 16 * mt);
#pragma unroll
                        for (int s = 0; s < KSH; ++s)
#pragma unroll
                            for (int cc = 0; cc < G; ++cc)
#pragma unroll
                                for (int mt = 0; mt < MT; ++mt)
                                    acc[cc][mt] = mfma(w1[mt % MT1][s], h[cc][s], s == 0 ? bvh[mt] : acc[cc][mt]);
                    }
                } else {
                    float h[G][MT][4];
#pragma unroll
                    for (int cc = 0; cc < G; ++cc)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                            for (int t = 0; t < 4; ++t) h[cc][mt][t] = tanh_t(acc[cc][mt][t]);
                    if (last) {
                        const floatx4 bv = *(const floatx4*)lb;
#pragma unroll
                        for (int cc = 0; cc < G; ++cc) {
                            floatx4 o = mfma(wo[0], h[cc][0][0], bv);
#pragma unroll
                            for (int s = 1; s < KSH; ++s) o = mfma(wo[s], h[cc][s >> 2][s & 3], o);
                            outv[cb * G + cc] = o;
                        }
                    } else {
                        floatx4 bvh[MT];
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) bvh[mt] = *(const floatx4*)(lb + 16 * mt);
#pragma unroll
                        for (int s = 0; s < KSH; ++s)
#pragma unroll
                            for (int cc = 0; cc < G; ++cc)
#pragma unroll
                                for (int mt = 0; mt < MT; ++mt)
                                    acc[cc][mt] = mfma(w1[mt % MT1][s], h[cc][s >> 2][s & 3],
                                                       s == 0 ? bvh[mt] : acc[cc][mt]);
                    }
                }
            }
        };
        // passes whose groups hold no valid cell are skipped (only invalid
        // lanes read their actuator rows): with one group per pass, a unit of
        // at most 16 cells, such as the one-cell genomes radiation creates,
        // takes a quarter of the network work
#pragma unroll
        for (int cb = 0; cb < 4 / CGI; ++cb)
            if (16 * CGI * cb < cnt) pass(std::integral_constant<int, CGI>{}, cb);
        wave_lds_sync();  // all stage reads done before the actuator rows overwrite them
#pragma unroll
        for (int c = 0; c < 4; ++c)
            *(floatx4*)(stage + (16 * c + n16) * NT::ACT_ROW + 16 * q) = outv[c];
        wave_lds_sync();
        float a[16];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const floatx4 v = *(const floatx4*)(stage + lane * NT::ACT_ROW + 16 * t);
            a[4 * t] = v[0]; a[4 * t + 1] = v[1]; a[4 * t + 2] = v[2]; a[4 * t + 3] = v[3];
        }
        wave_lds_sync();  // actuator rows read before the next unit's stage writes

        // ---- 3. epilogue: one cell per lane, results held for the stores
        st_i = valid ? i : -1;
        st_pending = true;
        if (valid) {
            if constexpr (DEBUG) {  // the actuators without their stored scale
                constexpr float kLn2 = 0.69314718055994531f;
#pragma unroll
                for (int t = 0; t < kNOut; ++t) dbg[(int64_t)i * kNOut + t] = a[t] * (t < 6 ? -kLn2 : kLn2);
            }
            bool finite = true;
#pragma unroll
            for (int t = 0; t < kNOut; ++t) finite = finite && __builtin_isfinite(a[t]);
            if (!finite) {
                err |= kErrNonFinite;
#pragma unroll
                for (int t = 0; t < kNOut; ++t) a[t] = __builtin_isfinite(a[t]) ? a[t] : 0.0f;
            }
            if (e_own < 0 || i_own < 0) err |= kErrLedger;
            // invest / liquidate: sigmoid-gated fractions of the pre-step stocks
            const float se = sigmoid_s(a[0]), sl = sigmoid_s(a[1]);
            // (negative stocks are flagged above; the transfers then stay
            // within [0, stock] or are zero, and the ledger still balances)
            int64_t xi = floor_nonneg_i64(rho_i * se * i64_to_f32(e_own));
            int64_t xl = floor_nonneg_i64(rho_l * sl * i64_to_f32(i_own));
            xi = xi > e_own ? e_own : xi;
            xl = xl > i_own ? i_own : xl;
            xi = xi < 0 ? 0 : xi;
            xl = xl < 0 ? 0 : xl;
            const int64_t E1 = e_own - xi + xl, I1 = i_own + xi - xl;
            st_E1 = E1;
            st_I1 = I1;
            // communication: sigmoid of the comm actuators
#pragma unroll
            for (int c = 0; c < 4; ++c) st_c[c] = __builtin_bit_cast(uint32_t, sigmoid_s(a[2 + c]));
            // exploration: softmax split of the flow budget, argmax explore
            float m = a[6];
            int best = 0;
#pragma unroll
            for (int t = 1; t < 8; ++t)
                if (a[6 + t] > m) { m = a[6 + t]; best = t; }
            float ex[8], ssum = 0.0f;
#pragma unroll
            // flow logits are stored times log2(e): exp(a - max) = 2^(a' - max')
            for (int t = 0; t < 8; ++t) { ex[t] = __builtin_amdgcn_exp2f(a[6 + t] - m); ssum += ex[t]; }
            const float inv = __builtin_amdgcn_rcpf(ssum);
            // flow budget below 2^31 quanta: each flow word carries the
            // explored flag in its low bit
            // floor(kappa I1) >= 0, clamped to 2^31 - 1 (the conversion
            // saturates at 2^32 - 1 beyond 32 bits)
            const float fF = __builtin_floorf(__builtin_fmaxf(kappa * i64_to_f32(I1), 0.0f));
            if (fF >= 0x1p31f) err |= kErrLedger;
            uint32_t Fu = (uint32_t)fF;
            Fu = Fu < 0x7fffffffu ? Fu : 0x7fffffffu;
            // all amounts are below 2^31: 32-bit integers suffice, and the
            // truncating conversion of a non-negative float is its floor
            if constexpr (!VARIANTS) {
                const float per = inv * (float)Fu;  // budget per unit of softmax weight
                const uint32_t onehot = 1u << best;   // the explored position's flag
                uint32_t used = 0, fs[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const float share = ex[t] * per;  // >= 0 and finite
                    uint32_t f = (uint32_t)share;
                    const uint32_t rem = Fu - used;
                    f = f < rem ? f : rem;
                    used += f;
                    fs[t] = (f << 1) | ((onehot >> t) & 1u);
                }
                // kernel position t + 1 points at direction (r + offset) & 7: put
                // the words in offset order (fixed), then rotate by r, one
                // conditional rotation per bit of r
                uint32_t wd[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) wd[kernel_offset(t + 1)] = fs[t];
#pragma unroll
                for (int bit = 1; bit < 8; bit <<= 1) {
                    const bool on = (r & bit) != 0;
                    uint32_t nw[8];
#pragma unroll
                    for (int d = 0; d < 8; ++d) nw[d] = on ? wd[(d - bit) & 7] : wd[d];
#pragma unroll
                    for (int d = 0; d < 8; ++d) wd[d] = nw[d];
                }
#pragma unroll
                for (int d = 0; d < 8; ++d) st_f[d] = wd[d];
            } else {
                // physics variants: the budget's split (softmax shares with a
                // running clamp, or with hard max all to the maximal explore
                // actuator), then the same for the energy budget
                uint32_t fs[8];
                if (variant & 1) split_hard(Fu, best, fs);
                else split_soft(Fu, ex, inv, fs);
#pragma unroll
                for (int t = 0; t < 8; ++t) fs[t] = (fs[t] << 1) | (uint32_t)(t == best);
                to_directions(fs, r, st_f);
                if (variant & 2) {
                    // energy transport: floor(kappa_e E1) along the same directions
                    const float kappa_e = cld(&world_at(b, wi)->kappa_e);
                    int64_t FE = (int64_t)floorf(kappa_e * i64_to_f32(E1));
                    if (FE < 0) FE = 0;
                    if (FE > 0x7fffffffll) { err |= kErrLedger; FE = 0x7fffffffll; }
                    uint32_t es[8];
                    if (variant & 1) split_hard((uint32_t)FE, best, es);
                    else split_soft((uint32_t)FE, ex, inv, es);
#pragma unroll
                    for (int t = 0; t < 8; ++t) es[t] <<= 1;
                    to_directions(es, r, st_e);
                }
            }
            acc_mass += E1;
        }
        ++u;
        // the next segment's chunk starts a new run
        while (u >= uend && seg + 1 < nseg) {
            ++seg;
            enter_segment();
            run_end = -1;
            g = -1;
            have_pf = false;
        }
    }
    if (st_pending) store_results();
    flush();
}

// Persistent grid: as many blocks as the kernel keeps resident.
template <typename K>
static int resident_blocks(K kernel, int n_cu) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return n_cu * per_cu;
}

template <int NL, int HID, int PREC, int CGI, int WAVES, bool DEBUG, bool VARIANTS>
static void launch_act_v(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s, float* dbg) {
    static int blocks = 0;
    if (blocks == 0) blocks = resident_blocks(k_act<NL, HID, PREC, CGI, WAVES, DEBUG, VARIANTS>, ls.n_cu);
    hipLaunchKernelGGL((k_act<NL, HID, PREC, CGI, WAVES, DEBUG, VARIANTS>), dim3(blocks), dim3(256), 0, s, bdev,
                       dbg, ls.act_segments);
}

template <int NL, int HID, int PREC, int CGI, int WAVES, bool DEBUG>
static void launch_act_c(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s, float* dbg) {
    if (ls.act_variants) launch_act_v<NL, HID, PREC, CGI, WAVES, DEBUG, true>(bdev, ls, s, dbg);
    else launch_act_v<NL, HID, PREC, CGI, WAVES, DEBUG, false>(bdev, ls, s, dbg);
}

// act_cells: column groups of 16 cells processed together (1, 2, 4);
// act_waves: 0 = fewer waves per SIMD with more registers each, 1 = more waves.
template <int NL, int HID, int PREC, bool DEBUG>
static void launch_act_t(const BatchDev* bdev, const LaunchShape& ls, int act_cells, int act_waves,
                         hipStream_t s, float* dbg) {
    constexpr int LO = PREC == kPrecBF16 ? 2 : 1, HI = LO + 1;
    if (act_waves) {
        switch (act_cells) {
            case 1: launch_act_c<NL, HID, PREC, 1, HI, DEBUG>(bdev, ls, s, dbg); break;
            case 2: launch_act_c<NL, HID, PREC, 2, HI, DEBUG>(bdev, ls, s, dbg); break;
            default: launch_act_c<NL, HID, PREC, 4, HI, DEBUG>(bdev, ls, s, dbg); break;
        }
    } else {
        switch (act_cells) {
            case 1: launch_act_c<NL, HID, PREC, 1, LO, DEBUG>(bdev, ls, s, dbg); break;
            case 2: launch_act_c<NL, HID, PREC, 2, LO, DEBUG>(bdev, ls, s, dbg); break;
            default: launch_act_c<NL, HID, PREC, 4, LO, DEBUG>(bdev, ls, s, dbg); break;
        }
    }
}

template <bool DEBUG>
static void launch_act_d(const BatchDev* bdev, const LaunchShape& ls, int NL, int HID, int prec,
                         int act_cells, int act_waves, hipStream_t s, float* dbg) {
    if (prec == kPrecBF16) {
        if (NL == 2 && HID == 32) launch_act_t<2, 32, kPrecBF16, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
        else if (NL == 2 && HID == 64) launch_act_t<2, 64, kPrecBF16, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
        else if (NL == 3 && HID == 32) launch_act_t<3, 32, kPrecBF16, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
        else launch_act_t<3, 64, kPrecBF16, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
    } else {
        if (NL == 2 && HID == 32) launch_act_t<2, 32, kPrecFP32, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
        else if (NL == 2 && HID == 64) launch_act_t<2, 64, kPrecFP32, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
        else if (NL == 3 && HID == 32) launch_act_t<3, 32, kPrecFP32, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
        else launch_act_t<3, 64, kPrecFP32, DEBUG>(bdev, ls, act_cells, act_waves, s, dbg);
    }
}

void launch_act_only(const BatchDev* bdev, const LaunchShape& ls, int NL, int HID, int prec,
                     int act_cells, int act_waves, hipStream_t s, float* debug_act) {
    if (debug_act) launch_act_d<true>(bdev, ls, NL, HID, prec, act_cells, act_waves, s, debug_act);
    else launch_act_d<false>(bdev, ls, NL, HID, prec, act_cells, act_waves, s, nullptr);
}

}  // namespace coralai
