// Per-step bookkeeping kernels: genome bucketing (histogram, exclusive scan,
// compaction), the cross-world prefix of network work units, and the step
// finalisation that publishes the conservation sums and swaps buffers.
//
// Bucketing groups cells by GenomeIndex (System Design: the GenomeIndex
// channel locates the cell's network parameters) so that each genome's
// cells run through its network as one grouped GEMM.
//
// A block owns a 64 x 64 tile; each wavefront takes one 64-cell tile row at
// a time and run-length encodes it with a lane shuffle and a ballot, so every
// run of equal genomes is handled by its first lane, all runs in parallel.
// Per-genome counts are aggregated in an LDS hash table first, so the global counters see one
// atomic per (tile, genome): Voronoi patches put ~20 genomes in a tile, and
// a genome owning a sixth of the world costs one atomic per tile instead of
// one per wavefront.  A genome that finds the table full falls back to
// direct global atomics (fragmented populations), with identical results.
// The scan over genome slots is reduce-then-scan over 512-slot blocks with
// coalesced loads, in two passes (three for capacities beyond 1024 blocks);
// it also lists the free (zero-count) slots in ascending order for radiation.
#include "coralai_internal.h"

namespace coralai {

constexpr int kHashSlots = 2048;
constexpr int kHashProbes = 64;

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

// Exclusive scan of one int per thread over a block of NT threads.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int* total, int* s_tmp) {
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

// Zero every world's genome histogram unless its counts already describe
// the current state (physics and radiation keep them current; only a new
// state from the host does not).  Launched, with k_count, only when the host
// has made some world's counts stale.
__global__ __launch_bounds__(256) void k_prep(const BatchDev* __restrict__ b) {
    const int wi = blockIdx.y;
    if (wi >= b->n_worlds) return;
    const auto& w = *world_at(b, wi);
    if (!w.ctl->counts_valid)
        for (int g = blockIdx.x * 256 + threadIdx.x; g < kStripes * w.cap; g += gridDim.x * 256)
            w.stripe_counts[g] = 0;
}

// LDS hash of genome -> slot index (NSLOT = 2^LOG slots); returns -1 when
// the table has no room.
template <int LOG>
__device__ __forceinline__ int hash_find_n(int* s_key, int g, bool insert) {
    constexpr int NSLOT = 1 << LOG;
    int h = (int)(((uint32_t)g * 2654435761u) >> (32 - LOG));
    for (int p = 0; p < kHashProbes; ++p) {
        const int k = s_key[h];
        if (k == g) return h;
        if (k == -1) {
            if (!insert) return -1;
            const int old = atomicCAS(&s_key[h], -1, g);
            if (old == -1 || old == g) return h;
        }
        h = (h + 1) & (NSLOT - 1);
    }
    return -1;
}
__device__ __forceinline__ int hash_find(int* s_key, int g, bool insert) {
    static_assert(kHashSlots == 2048, "hash_find indexes 2^11 slots");
    return hash_find_n<11>(s_key, g, insert);
}

// Genome histogram.  A block takes a unit of kBucketGroup consecutive tiles
// and aggregates its counts over all of them before touching global memory:
// one atomic per (unit, genome).  Genome ids are checked here (out of range,
// unset slot).  Skipped while the counts are current: the scan sets the
// flag, physics and radiation keep the counts current, set_state clears it.
__global__ __launch_bounds__(256) void k_count(const BatchDev* __restrict__ b) {
    __shared__ int s_key[kHashSlots];
    __shared__ int s_cnt[kHashSlots];
    constexpr int ROWS = kBucketTile / 4;  // tile rows per wavefront
    const int n = cld(&b->n_worlds);
    if (n <= 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t total = cld(b->chunk_prefix + (n));
    for (int64_t u = spread_block(total); u < total; u += gridDim.x) {
        const int wi = find_world(b->chunk_prefix, n, u);
        const auto& w = *world_at(b, wi);
        const int cur = ctl_cur(w.ctl);
        const int64_t unit = u - cld(b->chunk_prefix + (wi));
        if (w.ctl->counts_valid) continue;  // block-uniform: nothing to count
        int32_t* scount = w.stripe_counts + (int64_t)(unit & (kStripes - 1)) * w.cap;
        const int32_t* G = w.G[cur];
        // the world's fields in registers: the atomics below would otherwise
        // make the compiler reload them from memory at every use
        const int Wd = w.W, Hd = w.H, btiles = w.btiles, btiles_x = w.btiles_x, capw = w.cap;
        const uint8_t* const slot_set = w.slot_set;
        for (int k = threadIdx.x; k < kHashSlots; k += 256) { s_key[k] = -1; s_cnt[k] = 0; }
        __syncthreads();
        uint32_t bad = 0;
        // the wavefront's rows of the unit's tiles, loaded up front, all
        // issued before any is used (an invalid lane reads cell 0, and the
        // slot flags of out-of-range ids are read at slot 0)
        int gv[kBucketGroup][ROWS];
        int tx[kBucketGroup], ty[kBucketGroup];
        bool tile_ok[kBucketGroup];
#pragma unroll
        for (int tg = 0; tg < kBucketGroup; ++tg) {
            const int tile = (int)unit * kBucketGroup + tg;
            tile_ok[tg] = tile < btiles;
            ty[tg] = tile / btiles_x;
            tx[tg] = tile - ty[tg] * btiles_x;
            const int x = tx[tg] * kBucketTile + lane;
#pragma unroll
            for (int it = 0; it < ROWS; ++it) {
                const int y = ty[tg] * kBucketTile + wv + 4 * it;
                const bool valid = tile_ok[tg] && x < Wd && y < Hd;
                gv[tg][it] = gld(G + (valid ? (int64_t)y * Wd + x : 0));
            }
        }
#pragma unroll
        for (int tg = 0; tg < kBucketGroup; ++tg) {
            const int x = tx[tg] * kBucketTile + lane;
            uint8_t set[ROWS];
#pragma unroll
            for (int it = 0; it < ROWS; ++it) {
                const int g = gv[tg][it];
                set[it] = gld(slot_set + ((g < 0 || g >= capw) ? 0 : g));
            }
#pragma unroll
            for (int it = 0; it < ROWS; ++it) {
                const int y = ty[tg] * kBucketTile + wv + 4 * it;
                const bool valid = tile_ok[tg] && x < Wd && y < Hd;
                const int g = gv[tg][it];
                const bool in_range = g >= 0 && g < capw;
                if (valid && !in_range) bad |= kErrGenomeRange;
                if (valid && in_range && !set[it]) bad |= kErrGenomeUnset;
                gv[tg][it] = (valid && in_range) ? g : 0;
            }
        }
        // 1. per-genome counts of the unit (LDS, global on table overflow).
        // Each tile row is run-length encoded across the wavefront: the first
        // lane of each run of equal genomes updates the table for the whole
        // run, all runs of the row at once.  Valid lanes form a prefix.
#pragma unroll
        for (int tg = 0; tg < kBucketGroup; ++tg) {
            const int x = tx[tg] * kBucketTile + lane;
#pragma unroll
            for (int it = 0; it < ROWS; ++it) {
                const int y = ty[tg] * kBucketTile + wv + 4 * it;
                const bool valid = tile_ok[tg] && x < Wd && y < Hd;
                const int g = gv[tg][it];
                const int prev = __shfl_up(g, 1, 64);
                const bool start = valid && (lane == 0 || prev != g);
                const uint64_t starts = __ballot(start);
                const int nvalid = (int)__popcll(__ballot(valid));
                if (start) {
                    const uint64_t later = starts & ~((2ull << lane) - 1ull);
                    const int len = (later ? __ffsll((unsigned long long)later) - 1 : nvalid) - lane;
                    const int h = hash_find(s_key, g, true);
                    if (h >= 0) atomicAdd(&s_cnt[h], len);
                    else atomicAdd(scount + g, len);
                }
            }
        }
        if (bad) atomicOr(&w.ctl->err, bad);
        __syncthreads();
        // 2. one global atomic per (unit, genome)
        for (int k = threadIdx.x; k < kHashSlots; k += 256) {
            const int g = s_key[k];
            if (g < 0) continue;
            atomicAdd(scount + g, s_cnt[k]);
        }
        __syncthreads();  // the table is cleared for the next unit
    }
}

// Compaction into perm, one 64 x 64 tile per block and one wavefront per
// 16-column strip of it.  A wavefront walks its strip four rows per
// instruction, so that a genome's cells of the tile come strip by strip: the
// network kernel's 64-cell groups are then compact 16 x 4 blocks of a patch,
// whose neighbourhoods overlap.  Each run of equal genomes in a 16-cell row
// segment takes its rank inside the strip's share of its genome with one LDS
// atomic on the wavefront's own counter (after a hash insert); every cell
// keeps (slot, rank) in a register.  Then per genome: the strips' shares are
// laid out one after another behind one global atomic on the unit's stripe
// cursor, and the cells are written with no second lookup.  A genome that
// finds the table full takes its run's positions straight from the cursor.
// Perm entries carry the cell's rotation in the high bits.  (Sixteen
// dependent steps per wavefront and a small register and LDS footprint keep
// many tiles in flight.)
// 256 slots: a tile holds a few dozen genomes (up to about a hundred late in
// a long run); a larger table costs its clearing and its scan in every tile
// (1024 slots: +17 us per 4096^2 step)
constexpr int kScatterHashLog = 8;
constexpr int kScatterHash = 1 << kScatterHashLog;
static_assert(kBucketTile == 64, "four 16-column strips per tile");
__global__ __launch_bounds__(256) void k_scatter(const BatchDev* __restrict__ b) {
    constexpr int SW = 16, RPI = 4, NIT = 16;  // strip width, rows per instruction, instructions
    __shared__ int s_key[kScatterHash];
    __shared__ int s_cnt[4][kScatterHash];  // per strip: cells so far, then the strip's base
    constexpr uint32_t kAbs = 0x80000000u;  // bits 0..25 hold an absolute position
    // packed per cell: kAbs | position, or slot << 12 | rank in the strip
    const int n = cld(&b->n_worlds);
    if (n <= 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane % SW, rsub = lane / SW;
    const uint64_t segmask = ((1ull << SW) - 1ull) << (SW * rsub);
    const int64_t total = cld(b->chunk_prefix + (n)) * kBucketGroup;  // tiles
    for (int64_t tt = spread_block(total); tt < total; tt += gridDim.x) {
        const int64_t u = tt / kBucketGroup;
        const int wi = find_world(b->chunk_prefix, n, u);
        const auto& w = *world_at(b, wi);
        // the world's fields in registers: the atomics below would otherwise
        // make the compiler reload them from memory at every use
        const int Wd = w.W, Hd = w.H, btiles = w.btiles, btiles_x = w.btiles_x, capw = w.cap;
        int32_t* const permp = w.perm;
        const int cur = ctl_cur(w.ctl);
        const int64_t unit = u - cld(b->chunk_prefix + (wi));
        const int32_t* G = w.G[cur];
        const uint8_t* Rc = w.R[cur];
        int32_t* scur = w.cursor + (int64_t)(unit & (kStripes - 1)) * capw;
        for (int k = threadIdx.x; k < kScatterHash; k += 256) {
            s_key[k] = -1;
#pragma unroll
            for (int t = 0; t < 4; ++t) s_cnt[t][k] = 0;
        }
        __syncthreads();
        const int tile = (int)unit * kBucketGroup + (int)(tt - u * kBucketGroup);
        const bool tile_ok = tile < btiles;
        const int ty = tile / btiles_x, tx = tile - ty * btiles_x;
        const int x = tx * kBucketTile + SW * wv + col;  // this wavefront's strip
        uint32_t pk[NIT];
        {
            // every load is issued before any is used: an invalid lane reads
            // cell 0 (a conditional load would be a branch, and each branch a
            // wait for the loads before it)
            int gv[NIT];
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int y = ty * kBucketTile + RPI * it + rsub;
                const bool valid = tile_ok && x < Wd && y < Hd;
                gv[it] = gld(G + (valid ? (int64_t)y * Wd + x : 0));
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int y = ty * kBucketTile + RPI * it + rsub;
                const bool valid = tile_ok && x < Wd && y < Hd;
                const int graw = gv[it];
                const int g = (!valid || graw < 0 || graw >= capw) ? 0 : graw;  // ids were checked when counted
                const int prev = __shfl_up(g, 1, 64);
                // runs of equal genomes inside each 16-cell row segment (valid lanes are a
                // prefix of their segment)
                const bool start = valid && (col == 0 || prev != g);
                const uint64_t starts = __ballot(start);
                const uint64_t vmask = __ballot(valid);
                uint32_t mine = 0;
                if (start) {
                    const uint64_t later = starts & ~((2ull << lane) - 1ull) & segmask;
                    const int seg_end = SW * rsub + (int)__popcll(vmask & segmask);
                    const int len = (later ? __ffsll((unsigned long long)later) - 1 : seg_end) - lane;
                    const int h = hash_find_n<kScatterHashLog>(s_key, g, true);
                    mine = h >= 0 ? ((uint32_t)h << 12) | (uint32_t)atomicAdd(&s_cnt[wv][h], len)
                                  : kAbs | (uint32_t)atomicAdd(scur + g, len);
                }
                const uint64_t upto = starts & ((2ull << lane) - 1ull);
                const int rs = upto ? 63 - __clzll((unsigned long long)upto) : 0;
                pk[it] = __shfl(mine, rs, 64) + (uint32_t)(lane - rs);
            }
        }
        __syncthreads();
        // the rotations, loaded while the global atomics below are in flight
        // (not earlier: fewer registers live through the ranking above)
        uint8_t rv[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int y = ty * kBucketTile + RPI * it + rsub;
            const bool valid = tile_ok && x < Wd && y < Hd;
            rv[it] = gld(Rc + (valid ? (int64_t)y * Wd + x : 0));
        }
        // per genome: one global atomic; the strips' shares laid out in strip
        // order.  A thread's atomics are issued together, then their results
        // used, so their latencies overlap.
        {
            // (the strips' counts are read again from LDS once the bases are
            // back rather than held in registers meanwhile)
            constexpr int KP = (kScatterHash + 255) / 256;
            int gk[KP], base[KP];
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                const int k = threadIdx.x + 256 * j;
                gk[j] = k < kScatterHash ? s_key[k] : -1;
                const int tot = gk[j] >= 0 ? s_cnt[0][k] + s_cnt[1][k] + s_cnt[2][k] + s_cnt[3][k] : 0;
                base[j] = gk[j] >= 0 ? atomicAdd(scur + gk[j], tot) : 0;
            }
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                if (gk[j] < 0) continue;
                const int k = threadIdx.x + 256 * j;
                int bj = base[j];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = s_cnt[t][k];
                    s_cnt[t][k] = bj;
                    bj += c;
                }
            }
        }
        __syncthreads();
        // Every load and atomic of this tile has returned by now (the bases
        // above waited for the atomics, issued after the rotation loads).  An
        // explicit full wait tells the compiler so: otherwise it keeps them
        // pending along the branches above and waits for all earlier stores
        // before each store below.
        __builtin_amdgcn_s_waitcnt(0);
        int pos[NIT];
        uint32_t ent[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int y = ty * kBucketTile + RPI * it + rsub;
            const uint32_t v = pk[it];
            const int base = s_cnt[wv][(v >> 12) & 0x3ffu];
            pos[it] = (v & kAbs) ? (int)(v & (uint32_t)kPermIndexMask) : base + (int)(v & 0xfffu);
            ent[it] = (uint32_t)(y * Wd + x) | ((uint32_t)(rv[it] & 7u) << kPermRotShift);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int y = ty * kBucketTile + RPI * it + rsub;
            if (tile_ok && x < Wd && y < Hd) gst(permp + pos[it], (int)ent[it]);
        }
        __syncthreads();  // the table is cleared for the next tile
    }
}

// Scan over genome slots, pass A: per kSlotBlock-slot block, the number of
// cells (summing the stripe counters into counts), of 64-cell network units,
// of live genomes and of free slots.  Each world's first block also resets
// the world's step accumulators.
__global__ __launch_bounds__(256) void k_scan_reduce(const BatchDev* __restrict__ b) {
    __shared__ int s_red[4][4];
    const int n = cld(&b->n_worlds);
    if (n <= 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t total = cld(b->slot_prefix + (n));
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        const int wi = find_world(b->slot_prefix, n, u);
        const auto& w = *world_at(b, wi);
        const int sb = (int)(u - cld(b->slot_prefix + (wi)));
        if (sb == 0 && threadIdx.x == 0) {  // the step accumulators start from zero
            w.ctl->acc_mass = 0;
            w.ctl->acc_mass_f64 = 0.0;
            w.ctl->acc_takeovers = 0;
            w.ctl->acc_injected = 0;
            w.ctl->acc_removed = 0;
        }
        int c = 0, gsum = 0, live = 0, fr = 0;
        for (int k = 0; k < kSlotBlock / 256; ++k) {
            const int g = sb * kSlotBlock + k * 256 + threadIdx.x;
            if (g < w.cap) {
                int v = 0;
#pragma unroll
                for (int q = 0; q < kStripes; ++q) v += gld(w.stripe_counts + q * w.cap + g);
                gst(w.counts + g, v);
                c += v;
                gsum += (v + kGroupCells - 1) / kGroupCells;
                live += v > 0;
                fr += v == 0;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            c += __shfl_xor(c, o, 64);
            gsum += __shfl_xor(gsum, o, 64);
            live += __shfl_xor(live, o, 64);
            fr += __shfl_xor(fr, o, 64);
        }
        if (lane == 0) { s_red[wv][0] = c; s_red[wv][1] = gsum; s_red[wv][2] = live; s_red[wv][3] = fr; }
        __syncthreads();
        if (threadIdx.x < 4) {
            const int f = threadIdx.x;
            gst(w.scan_part + sb * 4 + f, s_red[0][f] + s_red[1][f] + s_red[2][f] + s_red[3][f]);
        }
        __syncthreads();
    }
}

// Pass B (only when some world has more than kFuseSlotBlocks slot blocks):
// per world, exclusive prefix of the block partials (in place) and the
// world totals.
__global__ __launch_bounds__(1024) void k_scan_blocks(const BatchDev* __restrict__ b) {
    __shared__ int s_tmp[16];
    const int wi = blockIdx.y;
    if (wi >= b->n_worlds) return;
    const auto& w = *world_at(b, wi);
    const int nb = w.n_slot_blocks;
    const int t = threadIdx.x;
    // n_slot_blocks <= 8192: up to 8 consecutive partials per thread
    const int per = (nb + 1023) / 1024;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    int tot[4];
    for (int f = 0; f < 4; ++f) {
        int sum = 0;
        for (int k = b0; k < b1; ++k) sum += gld(w.scan_part + k * 4 + f);
        int run = block_exclusive_scan<1024>(sum, &tot[f], s_tmp);
        for (int k = b0; k < b1; ++k) {
            const int v = gld(w.scan_part + k * 4 + f);
            gst(w.scan_part + k * 4 + f, run);
            run += v;
        }
    }
    if (t == 0) {
        w.ctl->counts_valid = 1;
        w.offsets[w.cap] = tot[0];
        w.gofs[w.cap] = tot[1];
        w.ctl->total_groups = tot[1];
        w.ctl->live = tot[2];
        w.ctl->n_free = tot[3];
        if (b->n_worlds == 1) {  // the prefix over worlds (k_world_prefix) of a lone world
            b->group_prefix[0] = 0;
            b->group_prefix[1] = tot[1];
        }
    }
}

// Pass C: per slot block, the exclusive scans themselves (block-wide scan
// of each thread's serial sums), the partial ranges of each genome laid out
// one after another, plus the free-slot list.
// free_only: just the free-slot list (radiation), not the step's ranges.
// FUSED (every world has at most kFuseSlotBlocks slot blocks): pass B is not
// run; each block sums the raw partials of the world's earlier blocks itself,
// and the world's last block publishes the totals.
template <bool FUSED>
__global__ __launch_bounds__(256) void k_scan_write(const BatchDev* __restrict__ b, int free_only) {
    __shared__ int s_tmp[4];
    __shared__ int s_red[4][4];
    const int n = cld(&b->n_worlds);
    if (n <= 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t total = cld(b->slot_prefix + (n));
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        const int wi = find_world(b->slot_prefix, n, u);
        const auto& w = *world_at(b, wi);
        const int sb = (int)(u - cld(b->slot_prefix + (wi)));
        // the exclusive prefix of the block partials (cells, units, live, free)
        int pre[4];
        if constexpr (FUSED) {
            int p[4] = {0, 0, 0, 0};
            for (int k = threadIdx.x; k < sb; k += 256) {
#pragma unroll
                for (int f = 0; f < 4; ++f) p[f] += gld(w.scan_part + k * 4 + f);
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) {
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) p[f] += __shfl_xor(p[f], o, 64);
            }
            if (lane == 0) {
#pragma unroll
                for (int f = 0; f < 4; ++f) s_red[wv][f] = p[f];
            }
            __syncthreads();
#pragma unroll
            for (int f = 0; f < 4; ++f) pre[f] = s_red[0][f] + s_red[1][f] + s_red[2][f] + s_red[3][f];
            __syncthreads();
            if (sb == w.n_slot_blocks - 1 && threadIdx.x == 0) {  // the world's totals
                int tot[4];
#pragma unroll
                for (int f = 0; f < 4; ++f) tot[f] = pre[f] + gld(w.scan_part + sb * 4 + f);
                w.ctl->counts_valid = 1;
                w.offsets[w.cap] = tot[0];
                w.gofs[w.cap] = tot[1];
                w.ctl->total_groups = tot[1];
                w.ctl->live = tot[2];
                w.ctl->n_free = tot[3];
                if (n == 1) {  // the prefix over worlds (k_world_prefix) of a lone world
                    b->group_prefix[0] = 0;
                    b->group_prefix[1] = tot[1];
                }
            }
        } else {
#pragma unroll
            for (int f = 0; f < 4; ++f) pre[f] = gld(w.scan_part + sb * 4 + f);
        }
        // each thread owns kSlotBlock / 256 consecutive slots: serial sums,
        // one block-wide scan per quantity, then serial writes
        constexpr int PER = kSlotBlock / 256;
        const int g0 = sb * kSlotBlock + threadIdx.x * PER;
        int sc = 0, sg = 0, sf = 0;
        for (int k = 0; k < PER; ++k) {
            const int g = g0 + k;
            const int v = g < w.cap ? gld(w.counts + g) : 0;
            sc += v;
            sg += (v + kGroupCells - 1) / kGroupCells;
            sf += g < w.cap && v == 0;
        }
        int tc, tg, tf;
        int oc = pre[0] + block_exclusive_scan<256>(sc, &tc, s_tmp);
        int og = pre[1] + block_exclusive_scan<256>(sg, &tg, s_tmp);
        int of = pre[3] + block_exclusive_scan<256>(sf, &tf, s_tmp);
        for (int k = 0; k < PER; ++k) {
            const int g = g0 + k;
            if (g >= w.cap) break;
            const int v = gld(w.counts + g);
            if (free_only) {
                if (v == 0) gst(w.free_list + of++, g);
                continue;
            }
            gst(w.offsets + g, oc);
            int pos = oc;
#pragma unroll
            for (int q = 0; q < kStripes; ++q) {
                gst(w.cursor + q * w.cap + g, pos);
                pos += gld(w.stripe_counts + q * w.cap + g);
            }
            gst(w.gofs + g, og);
            if (v == 0) gst(w.free_list + of++, g);
            oc += v;
            og += (v + kGroupCells - 1) / kGroupCells;
        }
    }
}

// Exclusive prefix over worlds of their network work units.
__global__ __launch_bounds__(1024) void k_world_prefix(const BatchDev* __restrict__ b) {
    __shared__ int s_tmp[16];
    const int n = b->n_worlds;
    const int per = (n + 1023) / 1024;
    const int beg = min(n, (int)threadIdx.x * per), end = min(n, beg + per);
    int s = 0;
    for (int k = beg; k < end; ++k) s += b->worlds[k].ctl->total_groups;
    int tot;
    int o = block_exclusive_scan<1024>(s, &tot, s_tmp);
    for (int k = beg; k < end; ++k) {
        b->group_prefix[k] = o;
        o += b->worlds[k].ctl->total_groups;
    }
    if (threadIdx.x == 0) b->group_prefix[n] = tot;
}

// Publish the step's sums and swap the state buffers.
__global__ void k_finalize(const BatchDev* __restrict__ b) {
    const int wi = blockIdx.y * blockDim.x + threadIdx.x;
    if (wi >= b->n_worlds) return;
    Ctl* c = b->worlds[wi].ctl;
    // conservation check against the previous step: the sum moves by exactly
    // the cycle's injected minus removed quanta (zero without the cycle)
    if (c->mass_valid && c->acc_mass != c->mass + c->acc_injected - c->acc_removed) c->err |= kErrMass;
    c->mass = c->acc_mass;
    c->mass_f64 = c->acc_mass_f64;
    c->mass_valid = 1;
    c->injected_pub = c->acc_injected;
    c->removed_pub = c->acc_removed;
    c->injected_total += c->acc_injected;
    c->removed_total += c->acc_removed;
    c->takeovers = (int32_t)c->acc_takeovers;
    c->live_pub = c->live;
    c->steps += 1;
    c->cur ^= 1;
}

__global__ void k_flip(const BatchDev* __restrict__ b) {
    const int wi = blockIdx.x * blockDim.x + threadIdx.x;
    if (wi >= b->n_worlds) return;
    b->worlds[wi].ctl->cur ^= 1;
}

static void launch_scan(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s, int free_only) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(ls.misc_blocks), dim3(256), 0, s, bdev);
    if (ls.scan_fused) {
        hipLaunchKernelGGL(k_scan_write<true>, dim3(ls.misc_blocks), dim3(256), 0, s, bdev, free_only);
    } else {
        hipLaunchKernelGGL(k_scan_blocks, dim3(1, ls.max_worlds), dim3(1024), 0, s, bdev);
        hipLaunchKernelGGL(k_scan_write<false>, dim3(ls.misc_blocks), dim3(256), 0, s, bdev, free_only);
    }
}

void launch_hist_only(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s, int free_only, int recount) {
    if (recount) {
        const int cap_blocks = min(256, max(1, (kStripes * ls.max_cap + 255) / 256));
        hipLaunchKernelGGL(k_prep, dim3(cap_blocks, ls.max_worlds), dim3(256), 0, s, bdev);
        hipLaunchKernelGGL(k_count, dim3(ls.chunk_blocks), dim3(256), 0, s, bdev);
    }
    launch_scan(bdev, ls, s, free_only);
}

void launch_bucket_only(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s, int recount) {
    launch_hist_only(bdev, ls, s, 0, recount);
    // a single world's prefix is written by the scan
    if (ls.max_worlds > 1) hipLaunchKernelGGL(k_world_prefix, dim3(1), dim3(1024), 0, s, bdev);
    hipLaunchKernelGGL(k_scatter, dim3(ls.n_cu * 16), dim3(256), 0, s, bdev);
}

void launch_finalize(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1, (ls.max_worlds + 63) / 64), dim3(64), 0, s, bdev);
}

void launch_flip(const BatchDev* bdev, hipStream_t s) {
    hipLaunchKernelGGL(k_flip, dim3(64), dim3(64), 0, s, bdev);
}

}  // namespace coralai
