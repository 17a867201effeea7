// Physics: exploration and takeover (Experiment: explore actuators spread
// infrastructure to the neighbour of the maximal actuator; if the exploring
// infrastructure exceeds the explored cell's, that cell adopts the explorer's
// genome and the rotation of the exploration, otherwise the infrastructure is
// absorbed; among several explorers the maximal investment wins).
//
// Pull form on an LDS-staged halo tile: every target t reads, for each
// direction d, the flow its neighbour n = nbr(t, d) sent toward (d+4) mod 8,
// and n's explore direction; I2 = I1 - sum(own flows) + sum(inflows); the
// candidate explorers are the neighbours exploring toward t, the largest
// investment wins (lowest d on ties) and takes t over when it strictly
// exceeds I1(t).  The tile loads (TW+2) x (TH+2) cells of the 8 flow planes,
// explore directions and genomes with coalesced row loads; inflows, takeover
// and the block's share of the total-mass reduction (int64 exact and FP64)
// follow from LDS.  Pure integer work: bit-exact by construction.
#include "coralai_internal.h"

namespace coralai {

template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_physics(const BatchDev* __restrict__ b) {
    constexpr int NT = TW * TH;
    constexpr int LW = TW + 2, LH = TH + 2, LN = LW * LH;
    __shared__ uint32_t s_flow[8][LN];
    __shared__ int32_t s_g[LN];
    __shared__ uint8_t s_x[LN];
    __shared__ int64_t s_red_m[NT / 64];
    __shared__ double s_red_f[NT / 64];
    __shared__ int s_red_t[NT / 64];

    const int nworlds = b->n_worlds;
    if (nworlds <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t total = b->tile_prefix[nworlds];
    const int blk = xcd_block();
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    int64_t tile = (int64_t)blk * per;
    const int64_t tend = min(total, tile + per);

    int wi = -1;
    int64_t world_hi = -1;
    int64_t acc_m = 0;
    double acc_f = 0.0;
    int acc_t = 0;
    Ctl* ctl = nullptr;

    auto flush = [&]() {
        // block-wide: every thread of the block walks the same tiles
        int64_t m = acc_m;
        double f = acc_f;
        int t = acc_t;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            m += __shfl_xor(m, o, 64);
            f += __shfl_xor(f, o, 64);
            t += __shfl_xor(t, o, 64);
        }
        if (lane == 0) { s_red_m[wid] = m; s_red_f[wid] = f; s_red_t[wid] = t; }
        __syncthreads();
        if (tid == 0 && ctl != nullptr) {
            int64_t sm = 0;
            double sf = 0.0;
            int st = 0;
            for (int k = 0; k < NT / 64; ++k) { sm += s_red_m[k]; sf += s_red_f[k]; st += s_red_t[k]; }
            atomicAdd((unsigned long long*)&ctl->acc_mass, (unsigned long long)sm);
            atomicAdd(&ctl->acc_mass_f64, sf);
            atomicAdd((unsigned long long*)&ctl->acc_takeovers, (unsigned long long)(int64_t)st);
        }
        __syncthreads();
        acc_m = 0;
        acc_f = 0.0;
        acc_t = 0;
    };

    int Wd = 0, Hd = 0, Nd = 0, tx_n = 1;
    int64_t world_lo = 0;
    const uint32_t* flow = nullptr;
    const int64_t* I1p = nullptr;
    const uint8_t* Xp = nullptr;
    const int32_t* Gc = nullptr;
    const uint8_t* Rc = nullptr;
    int64_t* In = nullptr;
    int32_t* Gn = nullptr;
    uint8_t* Rn = nullptr;

    for (; tile < tend; ++tile) {
        if (tile >= world_hi) {
            if (wi >= 0) flush();
            wi = find_world(b->tile_prefix, nworlds, tile);
            world_lo = b->tile_prefix[wi];
            world_hi = b->tile_prefix[wi + 1];
            const WorldDev* W = &b->worlds[wi];
            Wd = W->W; Hd = W->H; Nd = W->N;
            tx_n = b->tiles_x[wi];
            ctl = W->ctl;
            const int cur = ctl->cur, nxt = cur ^ 1;
            flow = W->flow; I1p = W->I1; Xp = W->X;
            Gc = W->G[cur]; Rc = W->R[cur];
            In = W->I[nxt]; Gn = W->G[nxt]; Rn = W->R[nxt];
        }
        const int64_t lt = tile - world_lo;
        const int ty = (int)(lt / tx_n), tx = (int)(lt - (int64_t)ty * tx_n);
        const int x0 = tx * TW, y0 = ty * TH;

        // stage the halo tile
        for (int idx = tid; idx < LN; idx += NT) {
            const int ly = idx / LW, lx = idx - ly * LW;
            const int gx = wrap(x0 + lx - 1, Wd), gy = wrap(y0 + ly - 1, Hd);
            const int n = gy * Wd + gx;
#pragma unroll
            for (int k = 0; k < 8; ++k) s_flow[k][idx] = flow[(int64_t)k * Nd + n];
            s_g[idx] = Gc[n];
            s_x[idx] = Xp[n];
        }
        __syncthreads();

        const int lx = tid % TW + 1, ly = tid / TW + 1;
        const int gx = x0 + lx - 1, gy = y0 + ly - 1;
        if (gx < Wd && gy < Hd) {
            const int t = gy * Wd + gx;
            const int own = ly * LW + lx;
            int64_t out = 0, in = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) out += s_flow[k][own];
            int win = -1;
            int64_t vbest = -1;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int back = (d + 4) & 7;
                const int nb = (ly + dir_dy(d)) * LW + (lx + dir_dx(d));
                const int64_t v = s_flow[back][nb];
                in += v;
                if (s_x[nb] == back && v > vbest) { vbest = v; win = d; }
            }
            const int64_t i1 = I1p[t];
            const int64_t i2 = i1 - out + in;
            int32_t g2 = Gc[t];
            uint8_t r2 = Rc[t];
            if (win >= 0 && vbest > i1) {
                g2 = s_g[(ly + dir_dy(win)) * LW + (lx + dir_dx(win))];
                r2 = (uint8_t)((win + 4) & 7);
                acc_t += 1;
            }
            In[t] = i2;
            Gn[t] = g2;
            Rn[t] = r2;
            acc_m += i2;
            acc_f += (double)i2;
        }
        __syncthreads();  // LDS reused by the next tile
    }
    if (wi >= 0) flush();
}

int phys_tile_w(int t) { return t == 1 ? 32 : (t == 2 ? 16 : 64); }
int phys_tile_h(int t) { return t == 1 ? 8 : (t == 2 ? 16 : 4); }

void launch_physics_only(const BatchDev* bdev, const LaunchShape& ls, int phys_tile,
                         hipStream_t s) {
    switch (phys_tile) {
        case 1: hipLaunchKernelGGL((k_physics<32, 8>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev); break;
        case 2: hipLaunchKernelGGL((k_physics<16, 16>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev); break;
        default: hipLaunchKernelGGL((k_physics<64, 4>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev); break;
    }
}

void launch_step_kernels(const BatchDev* bdev, const LaunchShape& ls, int NL, int HID, int prec,
                         int act_cells, int phys_tile, hipStream_t s, float* debug_act) {
    launch_bucket_only(bdev, ls, s);
    launch_act_only(bdev, ls, NL, HID, prec, act_cells, s, debug_act);
    launch_physics_only(bdev, ls, phys_tile, s);
    launch_finalize(bdev, ls, s);
}

}  // namespace coralai
