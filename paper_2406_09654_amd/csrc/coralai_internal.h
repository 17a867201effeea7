// Internal structures of the gfx950 Coralai library: the device-resident
// world table, the per-world control block, and small device helpers.
// Everything here is plain data shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace coralai {

constexpr int kNParam = 56;   // CPPN parameters: A (8x5) then B (2x8)
constexpr int kNExtW = 42;    // structural-gene weights: 10 direct connections, 16 added nodes x (in, out)
constexpr int kNIn = 54;      // 9 kernel positions x 6 sensor channels
constexpr int kNOut = 14;     // invest, liquidate, 4 comm, 8 flow logits
// perm entries: cell index in bits 0..25 (W*H <= 2^26), rotation in 26..28
constexpr int kPermRotShift = 26;
constexpr int kPermIndexMask = (1 << kPermRotShift) - 1;
constexpr int kGroupCells = 64;   // cells per network work unit (one wavefront)
constexpr int kBucketTile = 64;   // bucketing tile: 64 x 64 cells
constexpr int kBucketGroup = 4;   // tiles per bucketing unit (one block)
constexpr int kStripes = 8;       // genome counts and cursors split by bucketing unit (unit mod 8)
constexpr int kSlotBlock = 512;   // genome slots per scan block (<= 8192 blocks at 2^22 slots)
constexpr int kFuseSlotBlocks = 1024;  // up to this many slot blocks the scan takes two passes, not three
constexpr int kRadBlockCells = 4096;  // cells per radiation hit block (256 x 16)
constexpr int kPrecFP32 = 0;
constexpr int kPrecBF16 = 1;

constexpr uint32_t kErrGenomeRange = 1u, kErrGenomeUnset = 2u, kErrLedger = 4u,
                   kErrNonFinite = 8u, kErrMass = 16u;

// Per-world control block (device memory, inside the world's arena).
struct Ctl {
    int32_t cur;            // index (0/1) of the current state buffer
    int32_t total_groups;   // network work units of this step
    int32_t live;           // genomes with a nonzero count in the current state
    int32_t n_free;         // free slots (radiation)
    int32_t hits;           // radiation hits of the last call
    int32_t n_new;          // hits that received a slot
    int32_t dropped;        // hits beyond the free slots
    uint32_t err;           // sticky CORALAI_ERR_* bits
    int32_t counts_valid;   // counts[] is the histogram of the current state's genomes
    int32_t pad_ctl;
    int64_t acc_mass;       // step accumulators
    double acc_mass_f64;
    int64_t acc_takeovers;
    int64_t mass;           // published after each step
    double mass_f64;
    int64_t steps;
    int32_t takeovers;
    int32_t live_pub;
    int32_t hits_pub;
    int32_t dropped_pub;
    // day / night energy ledger: this step's accumulators, the last step's
    // totals and the running totals since creation (quanta)
    int64_t acc_injected;
    int64_t acc_removed;
    int64_t injected_pub;
    int64_t removed_pub;
    int64_t injected_total;
    int64_t removed_total;
    int32_t mass_valid;     // `mass` is the sum of the current state (the next step checks against it)
    int32_t pad_ctl2;
};

// One world as the kernels see it (device memory).  All planes are
// row-major over the W x H torus.
struct WorldDev {
    int32_t W, H, N, cap;
    int32_t NL, HID, prec, n_rad_blocks;
    // row of a cell: y = (i * w_magic) >> w_shift (64-bit product) for every
    // i < 2^26, with w_shift = 26 + ceil(log2 W), w_magic = ceil(2^w_shift / W)
    uint32_t w_magic;
    int32_t w_shift;
    float rho_i, rho_l, kappa;
    int32_t day_period;   // day / night cycle length in steps (0 = no cycle)
    uint64_t seed;
    int64_t day_inject;   // energy quanta a cell receives per step at noon
    int32_t night_num;    // at midnight a cell loses night_num / 65536 of its energy per step
    int32_t explore_mode; // 0: softmax split of the exploration budget, 1: all to the maximal actuator
    float kappa_e;        // > 0: floor(kappa_e E1) of a cell's energy moves along its flow directions
    int32_t pad_pv;
    uint32_t* eflow;      // [N][8] energy flow words (amount << 1), only with CORALAI_WORLD_ENERGY_FLOWS
    int64_t* EI[2];       // [N][2]: energy and infrastructure quanta of a cell together
    float* C[2];          // [N][4]: the 4 communication channels of a cell together
    int32_t* G[2];
    uint8_t* R[2];
    uint32_t* flow;       // [N][8]: word k of a cell = (its outflow toward direction k) << 1
                          // | (k is its explored direction); one 32-byte record per cell
    int64_t* EI1;         // [N][2]: energy and infrastructure after invest / liquidate
    int32_t* perm;        // cells grouped by genome
    int32_t* counts;      // [cap] cells per genome (sum of the stripes)
    int32_t* offsets;     // [cap + 1]
    int32_t* stripe_counts; // [kStripes][cap] cells per genome in the units of each stripe
                            // (kept current by physics and radiation)
    int32_t* cursor;      // [kStripes][cap] next free position of each stripe's range (scatter)
    int32_t* gofs;        // [cap + 1] exclusive prefix of network units per genome
    uint8_t* slot_set;    // [cap]
    float* params;        // [cap][56]
    // NEAT structural genes per slot (the bounded superset of the CPPN):
    // ext_w [cap][42] = direct connection weights (10), added nodes' in
    // weights (16), out weights (16); ext_mask [cap][4] = direct connections
    // enabled, added nodes enabled, added nodes' activations (2 bits each)
    float* ext_w;
    uint32_t* ext_mask;
    uint64_t t_conn;      // radiation: add-connection threshold (floor(p 2^64))
    uint64_t t_node;      // radiation: add-node threshold
    int32_t* lineage_parent;  // [cap] slot the genome was mutated or merged from (-1: set by the caller)
    int32_t* lineage_parent2; // [cap] a merge's second parent (the partner's genome), else -1
    int64_t* lineage_birth;   // [cap] steps completed when the genome was created
    uint8_t* wfrag;       // [cap][wfrag_stride] weights in MFMA fragment order
    float* bias;          // [cap][bias_stride]
    int64_t wfrag_stride;
    int32_t bias_stride;
    int32_t pad1;
    uint16_t* hit_bits;   // [n_rad_blocks * 256]
    int32_t* blk_hits;    // [n_rad_blocks]
    int32_t* blk_ofs;     // [n_rad_blocks + 1]
    int32_t* free_list;   // [cap]
    int32_t* new_slots;   // [cap]
    int32_t* stage_slots; // [cap] slot list for set_genomes
    float* stage_params;  // [cap][56]
    int32_t* scan_part;   // [n_slot_blocks * 4] per slot-block partial sums / prefixes
    int32_t n_slot_blocks;
    int32_t btiles_x;     // bucketing tiles per row
    int32_t btiles;       // bucketing tiles of the world
    Ctl* ctl;
};

// A batch of worlds sharing one launch sequence (device memory).
struct BatchDev {
    int32_t n_worlds;
    int32_t pad;
    WorldDev* worlds;         // [max_worlds]
    int64_t* chunk_prefix;    // [max_worlds + 1] bucketing units (kBucketGroup tiles of 64 x 64)
    int64_t* slot_prefix;     // [max_worlds + 1] genome-slot scan blocks
    int64_t* tile_prefix;     // [max_worlds + 1] physics tiles
    int32_t* group_prefix;    // [max_worlds + 1] network units (device computed)
    int32_t* tiles_x;         // [max_worlds] physics tiles per row
};

// Network fragment geometry.  Weights are stored per genome in the order
// the MFMA A operand is loaded: fragment f = (layer, 16-row tile, K-step),
// 64 lanes x (8 bf16 | 1 float).  BF16 uses v_mfma_f32_16x16x32_bf16
// (K-step 32), FP32 uses v_mfma_f32_16x16x4_f32 (K-step 4).  The 54 inputs
// take 2 bf16 K-steps or 14 fp32 K-steps (inputs 54, 55 are zero padding).
__host__ __device__ constexpr int net_mt(int hid) { return hid / 16; }
__host__ __device__ constexpr int net_ks0(int prec) { return prec == kPrecBF16 ? 2 : 14; }
__host__ __device__ constexpr int net_ksh(int hid, int prec) {
    return prec == kPrecBF16 ? hid / 32 : hid / 4;
}
__host__ __device__ constexpr int net_frags(int nl, int hid, int prec) {
    return net_mt(hid) * net_ks0(prec) + (nl == 3 ? net_mt(hid) * net_ksh(hid, prec) : 0) +
           net_ksh(hid, prec);
}
__host__ __device__ constexpr int net_frag_bytes(int prec) { return prec == kPrecBF16 ? 1024 : 256; }
__host__ __device__ constexpr int net_frag_elems(int prec) { return prec == kPrecBF16 ? 512 : 64; }
// bias block per genome: [layer 0 rows (hid)] [layer 1 rows (hid), 3 layers only] [16 out rows]
__host__ __device__ constexpr int net_bias_floats(int nl, int hid) {
    return hid + (nl == 3 ? hid : 0) + 16;
}
// Flat (natural) network size: per layer W (out x in) then b (out).
__host__ __device__ constexpr int net_flat_size(int nl, int hid) {
    return nl == 2 ? hid * kNIn + hid + kNOut * hid + kNOut
                   : hid * kNIn + hid + hid * hid + hid + kNOut * hid + kNOut;
}

// Stored network weights are the generated ones times factors that move
// arithmetic out of the network kernel (one rounding of the product):
//  * rows of hidden layers carry kTanhScale = 2 log2(e): the kernel computes
//    r = 1 / (2^y + 1) on y = 2 log2(e) x, and tanh(x) = 1 - 2r;
//  * BF16 networks: layers after a hidden layer take r as input (r is what
//    gets rounded to bf16): their columns carry -2, and the kernel adds -1/2
//    of each stored row's sum to its bias when it loads a genome
//    (sum_j w_j tanh_j = sum_j w_j - 2 sum_j w_j r_j).  FP32 networks take
//    tanh = 1 - 2r itself (one FMA): in FP32 the row-sum correction and the
//    r-weighted sum cancel to the final value, which loses about a factor 2
//    of accuracy on the actuators against tanh, while in BF16 the operand
//    rounding dominates either way;
//  * output rows 0..5 (sigmoid actuators) carry -log2(e) and rows 6..13 (flow
//    logits) +log2(e): sigmoid and softmax then need one exp2 each;
//  * layer-0 columns of the energy and infrastructure channels carry 2^-24,
//    so the ledger quanta enter the network unscaled.
// Biases carry their row's factor.  The debug weight hooks undo all of it.
constexpr double kTanhScale = 2.8853900817779268;
constexpr double kLog2e = 1.4426950408889634;
__host__ __device__ inline double stored_row_scale(int nl, int layer, int row) {
    if (layer < nl - 1) return kTanhScale;
    return row < 6 ? -kLog2e : (row < kNOut ? kLog2e : 1.0);
}
// layers after a hidden layer read r = (1 - tanh) / 2 (BF16) or tanh (FP32)
__host__ __device__ constexpr bool hidden_input_is_r(int prec) { return prec == kPrecBF16; }
__host__ __device__ inline double stored_col_scale(int prec, int layer, int col) {
    if (layer > 0) return hidden_input_is_r(prec) ? -2.0 : 1.0;
    return col % 6 < 2 ? 0x1p-24 : 1.0;
}

struct FragCoord {
    int layer, row, col;
};

// Which weight W_layer[row][col] the fragment element e of a genome holds.
// Layer 0 columns: bf16 (K-step s, lane group q, element i) -> 16q + 8s + i,
// fp32 (s, q) -> 4s + q.  Hidden-input layers follow the MFMA output layout
// (lane group q holds rows 4q..4q+3 of each 16-row tile), so the previous
// layer's accumulators feed the next MFMA without data movement:
// bf16 -> 16(2s + i/4) + 4q + i%4, fp32 -> 16(s/4) + 4q + s%4.
__host__ __device__ inline FragCoord frag_coord(int nl, int hid, int prec, int e) {
    const bool bf = prec == kPrecBF16;
    const int epl = bf ? 8 : 1;
    const int f = e / (64 * epl), r = e % (64 * epl);
    const int lane = r / epl, i = r % epl;
    const int q = lane >> 4, m = lane & 15;
    const int MT = net_mt(hid), KS0 = net_ks0(prec), KSH = net_ksh(hid, prec);
    const int F0 = MT * KS0, F1 = nl == 3 ? MT * KSH : 0;
    int layer, mt, s;
    if (f < F0) {
        layer = 0; mt = f / KS0; s = f % KS0;
    } else if (f < F0 + F1) {
        layer = 1; mt = (f - F0) / KSH; s = (f - F0) % KSH;
    } else {
        layer = nl - 1; mt = 0; s = f - F0 - F1;
    }
    int col;
    if (layer == 0) col = bf ? 16 * q + 8 * s + i : 4 * s + q;
    else col = bf ? 16 * (2 * s + (i >> 2)) + 4 * q + (i & 3) : 16 * (s >> 2) + 4 * q + (s & 3);
    return {layer, 16 * mt + m, col};
}

// Direction d points 45*d degrees counter-clockwise from +x, y pointing down.
__device__ __forceinline__ int dir_dx(int d) { return (int)((0x440052u >> (d * 3)) & 7) - 1; }
__device__ __forceinline__ int dir_dy(int d) { return (int)((0x491001u >> (d * 3)) & 7) - 1; }
// Kernel position p (1..8) of rotation r points at direction r + offset(p):
// offsets {0, +1, -1, +2, -2, +3, -3, +4}, packed as (off & 7) in 3 bits.
__host__ __device__ constexpr int kernel_offset(int p) { return (int)((0x95e5c8u >> (p * 3 - 3)) & 7); }
__device__ __forceinline__ int kernel_dir(int r, int p) { return (r + kernel_offset(p)) & 7; }

// Stripe of a cell: its bucketing unit (kBucketGroup consecutive 64 x 64
// tiles in row-major tile order) mod kStripes.
__device__ __forceinline__ int cell_stripe(int x, int y, int btiles_x) {
    return ((y / kBucketTile * btiles_x + x / kBucketTile) / kBucketGroup) & (kStripes - 1);
}

__device__ __forceinline__ int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Block index remapped so that each XCD (blocks are dealt round-robin over
// the 8 XCDs) owns a contiguous range of work: neighbouring tiles then share
// an L2.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    if (nb & 7) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Contiguous share [begin, end) of `total` items for logical part `part` of
// `parts`: every part gets floor or ceil of total / parts.  With fewer items
// than parts the non-empty shares are spread evenly over the part ids, so a
// small job still reaches every XCD.
__device__ __forceinline__ void balanced_share(int64_t total, int64_t part, int64_t parts, int64_t* begin,
                                               int64_t* end) {
    *begin = part * total / parts;
    *end = (part + 1) * total / parts;
}

// First item of a block's strided loop over `total` items: XCD-contiguous
// when the job fills the grid, else the hardware order (round robin over
// the XCDs).
__device__ __forceinline__ int64_t spread_block(int64_t total) {
    return total >= (int64_t)gridDim.x ? (int64_t)xcd_block() : (int64_t)blockIdx.x;
}

// Scalar (constant address space) load of data that is invariant while the
// kernel runs: prefix tables, counters written by earlier kernels.
template <typename T>
__device__ __forceinline__ T cld(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

template <typename T>
__device__ __forceinline__ int find_world(const T* prefix, int n, T u) {
    // largest w in [0, n) with prefix[w] <= u
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cld(prefix + mid) <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Row of cell i < 2^26 of a world of width W, by the multiplier of WorldDev:
// with m = (2^k + e) / W, 0 <= e < W, and i = y W + x, i m / 2^k is
// y + x / W + i e / (W 2^k), and i e < 2^26 W <= 2^k keeps the last two
// terms below 1.
inline void row_magic(int32_t W, uint32_t* magic, int32_t* shift) {
    int lg = 0;
    while ((1ll << lg) < W) ++lg;
    const int k = 26 + lg;
    *shift = k;
    *magic = (uint32_t)(((1ull << k) + (uint64_t)W - 1) / (uint64_t)W);
}
__device__ __forceinline__ int cell_row(int i, uint32_t magic, int shift) {
    return (int)(((uint64_t)(uint32_t)i * magic) >> shift);
}

// Loads and stores through the global address space.  Pointers read from the
// device-side world table are generic; casting them lets the compiler emit
// global_load / global_store instead of flat accesses (which would also tie
// up the LDS counter).
#define CORALAI_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gld(const T* p) { return *(const CORALAI_GLOBAL T*)p; }
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) { *(CORALAI_GLOBAL T*)p = v; }

// The world table and the control block do not change while a kernel runs:
// reading them through the constant address space gives scalar loads, so the
// world's pointers and sizes stay in SGPRs.
#define CORALAI_CONST __attribute__((address_space(4)))
__device__ __forceinline__ const CORALAI_CONST WorldDev* world_at(const BatchDev* b, int wi) {
    return (const CORALAI_CONST WorldDev*)(b->worlds + wi);
}
__device__ __forceinline__ int ctl_cur(const Ctl* c) { return ((const CORALAI_CONST Ctl*)c)->cur; }

// Buffer resources over one plane or plane group (< 4 GiB: worlds have at
// most 2^26 cells).  Buffer accesses take 32-bit offsets next to an SGPR
// descriptor, and reads outside the range return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

typedef unsigned int coralai_u32x2 __attribute__((__vector_size__(8)));
__device__ __forceinline__ int64_t buf_ld_i64(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(int64_t, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st_i64(int64_t v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(coralai_u32x2, v), r, off, 0, 0);
}
typedef unsigned int coralai_u32x4 __attribute__((__vector_size__(16)));
typedef long long i64x2 __attribute__((__vector_size__(16)));
__device__ __forceinline__ i64x2 buf_ld_i64x2(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(i64x2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
// Cache-policy operand of buffer memory instructions: the non-temporal
// (streaming) hint, for data this kernel writes and does not read again.
constexpr int kCpolNT = 2;
template <int CPOL = 0>
__device__ __forceinline__ void buf_st_i64x2(i64x2 v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(coralai_u32x4, v), r, off, 0, CPOL);
}
typedef float coralai_f32x4 __attribute__((__vector_size__(16)));
__device__ __forceinline__ coralai_f32x4 buf_ld_f32x4(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(coralai_f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <int CPOL = 0>
__device__ __forceinline__ void buf_st_f32x4(coralai_f32x4 v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(coralai_u32x4, v), r, off, 0, CPOL);
}

// int64 -> float with at most one extra rounding for values >= 2^32 (exact
// conversion for the common |v| < 2^24, correctly rounded below 2^32).
__device__ __forceinline__ float i64_to_f32(int64_t v) {
    return __builtin_fmaf((float)(int32_t)(v >> 32), 4294967296.0f, (float)(uint32_t)v);
}

// Day / night cycle (Experiment: energy is added to and removed from the
// substrate in a day / night cycle).  With period P and q = s mod P for the
// step s (steps completed before it), the daylight is the triangle wave
// L = P - 4 min(q, P - q) in [-P, P] (P at noon, q = 0; -P at midnight,
// q = P / 2).  In the physics pass every cell's energy becomes
//   E2 = E1 + floor(A max(L, 0) / P) - floor(floor(E1 num / 2^16) max(-L, 0) / P),
// all in int64 (E1 < 2^40 quanta, A < 2^40), so every side of the
// computation gets the same integers and the mass ledger moves by exactly
// the injected minus the removed quanta.
struct DayNight {
    int64_t inject;  // quanta per cell this step
    int64_t night;   // max(-L, 0)
    int64_t period;
    int64_t num;
};
__device__ __forceinline__ DayNight day_night(int32_t period, int64_t day_inject, int32_t night_num,
                                               int64_t steps_done) {
    DayNight dn{0, 0, 1, 0};
    if (period <= 0) return dn;
    const int64_t P = period, q = steps_done % P;
    const int64_t L = P - 4 * (q < P - q ? q : P - q);
    dn.period = P;
    dn.inject = L > 0 ? day_inject * L / P : 0;
    dn.night = L < 0 ? -L : 0;
    dn.num = night_num;
    return dn;
}
// Energy after the cycle's source and sink; adds this cell's injected and
// removed quanta to the accumulators.
__device__ __forceinline__ int64_t day_night_energy(int64_t e1, const DayNight& dn, int64_t& inj,
                                                    int64_t& rem, uint32_t& err) {
    int64_t ec = e1;
    if (ec >= (1ll << 40)) {
        err |= kErrLedger;
        ec = (1ll << 40) - 1;
    }
    const int64_t r = dn.night > 0 ? ((ec * dn.num) >> 16) * dn.night / dn.period : 0;
    inj += dn.inject;
    rem += r;
    return e1 + dn.inject - r;
}

// Host-side launch shapes ----------------------------------------------------

struct LaunchShape {
    int n_cu;
    int act_blocks;
    int phys_blocks;
    int chunk_blocks;
    int misc_blocks;
    int max_worlds;
    int max_cap;
    // segments of the unit list the network kernel deals out to its waves:
    // 0 = automatic (4 for BF16 networks on large jobs, else 1); k >= 1
    // forces k (a test hook: results do not depend on it)
    int act_segments;
    // bit 0: some world of the launch uses a physics variant (hard-max
    // exploration or energy transport), so the network kernel compiled with
    // the variants' code runs (else the kernel without it); bit 1: some world
    // uses energy transport, so the physics kernel that loads the energy
    // records with the rest of the tile runs
    int act_variants;
    // 1: every world of the launch has at most kFuseSlotBlocks slot blocks,
    // so the scan's write pass forms the prefix of the slot blocks' partials
    // itself (no separate pass over them)
    int scan_fused;
};

// Launchers implemented in the kernel translation units.
void launch_step_kernels(const BatchDev* bdev, const LaunchShape& ls, int NL, int HID, int prec,
                         int act_cells, int act_waves, int phys_tile, hipStream_t s,
                         float* debug_act, int recount = 1);
// recount = 0 skips the genome histogram (k_prep, k_count): only valid when
// every world of the launch has counts that describe its current state.
void launch_bucket_only(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s, int recount = 1);
void launch_act_only(const BatchDev* bdev, const LaunchShape& ls, int NL, int HID, int prec,
                     int act_cells, int act_waves, hipStream_t s, float* debug_act);
void launch_physics_only(const BatchDev* bdev, const LaunchShape& ls, int phys_tile,
                         hipStream_t s);
void launch_finalize(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s);
void launch_hist_only(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s, int free_only, int recount = 1);
void launch_cppn(const WorldDev* wdev, int nl, int hid, int prec, int from_radiation, int n_host, uint64_t step,
                 float sigma, int n_cu, hipStream_t s);
void launch_scatter_params(const WorldDev* wdev, int n, hipStream_t s);
// NEAT compatibility distance of genome pairs (slots: device list of the na
// slots of A, then the nb of B) into out[na][nb] (device).
void launch_genetic_distance(const WorldDev* wdev, const int32_t* slots, int na, int nb, float c1, float c2,
                             float c3, float* out, int n_cu, hipStream_t s);
// structural genes of the slots listed in stage_slots, 46-word records in stage_params
void launch_scatter_ext(const WorldDev* wdev, int n, hipStream_t s);
void launch_radiate(const BatchDev* bdev, const WorldDev* wdev, const LaunchShape& ls, int nl, int hid,
                    int prec, int n_rad_blocks, uint64_t T, float sigma, uint64_t step, hipStream_t s,
                    int recount = 1);
// Merging (NEAT crossover through the physics) after step `step`: candidates
// below T on Philox counter (k, step, 0, 1) that face another genome.
void launch_merge(const BatchDev* bdev, const WorldDev* wdev, const LaunchShape& ls, int nl, int hid, int prec,
                  int n_rad_blocks, uint64_t T, uint64_t step, hipStream_t s, int recount = 1);
void launch_pack_weights(const WorldDev* wdev, int slot, const float* flat, int unpack, float* out,
                         hipStream_t s);
void launch_flip(const BatchDev* bdev, hipStream_t s);
// communication channels: planar [4][N] (the C ABI's layout) <-> interleaved
// [N][4] (the device layout: one 16-byte load per cell)
void launch_comm_layout(const float* src, float* dst, int64_t n, int to_interleaved, hipStream_t s);
// ledger pairs: dst[2i] = e[i * e_stride], dst[2i+1] = v[i * v_stride]
void launch_ledger_pack(const int64_t* e, int e_stride, const int64_t* v, int v_stride, int64_t* dst,
                        int64_t n, hipStream_t s);
// and back: e[i] = src[2i], v[i] = src[2i+1] (either may be null)
void launch_ledger_unpack(const int64_t* src, int64_t* e, int64_t* v, int64_t n, hipStream_t s);

int phys_tile_w(int t);
// cells per 256-thread unit of the streaming physics: 4 per thread when the
// width is a multiple of 4 (aligned 16-byte plane loads), else 1
inline int phys_stream_cells(int W) { return (W & 3) == 0 ? 1024 : 256; }
int phys_tile_h(int t);

}  // namespace coralai
