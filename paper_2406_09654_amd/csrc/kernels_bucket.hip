// Per-step bookkeeping kernels: genome bucketing (histogram, exclusive scan,
// compaction), the cross-world prefix of network work units, and the step
// finalisation that publishes the conservation sums and swaps buffers.
//
// Bucketing groups cells by GenomeIndex (System Design: the GenomeIndex
// channel locates the cell's network parameters) so that each genome's
// cells can run through its network as one grouped GEMM.  Cells are taken
// 64 at a time (one wavefront, raster order); inside a wavefront the
// distinct genomes are found with ballots, so each (wavefront, genome) pair
// costs one atomic on the genome's counter: with spatially clustered genomes
// that is 1-3 atomics per 64 cells.
#include "coralai_internal.h"

namespace coralai {

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

// Zero the genome histogram and the step accumulators of every world.
__global__ __launch_bounds__(256) void k_prep(const BatchDev* __restrict__ b) {
    const int wi = blockIdx.y;
    if (wi >= b->n_worlds) return;
    const WorldDev& w = b->worlds[wi];
    for (int g = blockIdx.x * 256 + threadIdx.x; g < w.cap; g += gridDim.x * 256) w.counts[g] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.ctl->acc_mass = 0;
        w.ctl->acc_mass_f64 = 0.0;
        w.ctl->acc_takeovers = 0;
    }
}

// Histogram (scatter = 0) or stable-per-wavefront compaction (scatter = 1)
// of the current GenomeIndex plane.  Cells naming a genome outside
// [0, cap) are counted under genome 0 and flagged; cells naming a slot
// without parameters are flagged.
__global__ __launch_bounds__(256) void k_bucket(const BatchDev* __restrict__ b, int scatter) {
    const int n = b->n_worlds;
    if (n <= 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t total = b->chunk_prefix[n];
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t u = (int64_t)xcd_block() * 4 + (threadIdx.x >> 6); u < total; u += nwaves) {
        const int wi = find_world(b->chunk_prefix, n, u);
        const WorldDev& w = b->worlds[wi];
        const int cur = w.ctl->cur;
        const int64_t i = (u - b->chunk_prefix[wi]) * kChunkCells + lane;
        const bool valid = i < w.N;
        int g = valid ? w.G[cur][i] : 0;
        uint32_t bad = 0;
        if (valid) {
            if (g < 0 || g >= w.cap) {
                bad = kErrGenomeRange;
                g = 0;
            } else if (!w.slot_set[g]) {
                bad = kErrGenomeUnset;
            }
        }
        if (!scatter) {
            const uint64_t anybad = __ballot(bad != 0);
            if (anybad && lane == __ffsll((unsigned long long)anybad) - 1) atomicOr(&w.ctl->err, bad);
        }
        uint64_t active = __ballot(valid);
        while (active) {
            const int leader = __ffsll((unsigned long long)active) - 1;
            const int g0 = __builtin_amdgcn_readlane(g, leader);
            const uint64_t m = __ballot(g == g0) & active;
            if (!scatter) {
                if (lane == leader) atomicAdd(&w.counts[g0], (int)__popcll(m));
            } else {
                int base = 0;
                if (lane == leader) base = atomicAdd(&w.cursor[g0], (int)__popcll(m));
                base = __builtin_amdgcn_readlane(base, leader);
                if ((m >> lane) & 1ull) w.perm[base + __popcll(m & lanemask_lt(lane))] = (int)i;
            }
            active &= ~m;
        }
    }
}

// Per world: offsets = exclusive scan of counts, cursor = offsets, gofs =
// exclusive scan of the number of 64-cell network units per genome.
// One 1024-thread block per world; each thread owns a contiguous slot range.
__global__ __launch_bounds__(1024) void k_scan(const BatchDev* __restrict__ b) {
    const int wi = blockIdx.y;
    if (wi >= b->n_worlds) return;
    __shared__ int s_tmp[16];
    const WorldDev& w = b->worlds[wi];
    const int cap = w.cap;
    const int per = (cap + 1023) / 1024;
    const int beg = min(cap, (int)threadIdx.x * per), end = min(cap, beg + per);
    int sc = 0, sg = 0, live = 0;
    for (int g = beg; g < end; ++g) {
        const int c = w.counts[g];
        sc += c;
        sg += (c + kGroupCells - 1) / kGroupCells;
        live += c > 0;
    }
    int tc, tg, tl;
    int oc = block_exclusive_scan<1024>(sc, &tc, s_tmp);
    int og = block_exclusive_scan<1024>(sg, &tg, s_tmp);
    block_exclusive_scan<1024>(live, &tl, s_tmp);
    for (int g = beg; g < end; ++g) {
        const int c = w.counts[g];
        w.offsets[g] = oc;
        w.cursor[g] = oc;
        w.gofs[g] = og;
        oc += c;
        og += (c + kGroupCells - 1) / kGroupCells;
    }
    if (threadIdx.x == 0) {
        w.offsets[cap] = tc;
        w.gofs[cap] = tg;
        w.ctl->total_groups = tg;
        w.ctl->live = tl;
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
    c->mass = c->acc_mass;
    c->mass_f64 = c->acc_mass_f64;
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

void launch_bucket_only(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s) {
    const int cap_blocks = min(64, max(1, (ls.max_cap + 255) / 256));
    hipLaunchKernelGGL(k_prep, dim3(cap_blocks, ls.max_worlds), dim3(256), 0, s, bdev);
    hipLaunchKernelGGL(k_bucket, dim3(ls.chunk_blocks), dim3(256), 0, s, bdev, 0);
    hipLaunchKernelGGL(k_scan, dim3(1, ls.max_worlds), dim3(1024), 0, s, bdev);
    hipLaunchKernelGGL(k_world_prefix, dim3(1), dim3(1024), 0, s, bdev);
    hipLaunchKernelGGL(k_bucket, dim3(ls.chunk_blocks), dim3(256), 0, s, bdev, 1);
}

void launch_hist_only(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s) {
    const int cap_blocks = min(64, max(1, (ls.max_cap + 255) / 256));
    hipLaunchKernelGGL(k_prep, dim3(cap_blocks, ls.max_worlds), dim3(256), 0, s, bdev);
    hipLaunchKernelGGL(k_bucket, dim3(ls.chunk_blocks), dim3(256), 0, s, bdev, 0);
}

void launch_finalize(const BatchDev* bdev, const LaunchShape& ls, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1, (ls.max_worlds + 63) / 64), dim3(64), 0, s, bdev);
}

void launch_flip(const BatchDev* bdev, hipStream_t s) {
    hipLaunchKernelGGL(k_flip, dim3(64), dim3(64), 0, s, bdev);
}

}  // namespace coralai
