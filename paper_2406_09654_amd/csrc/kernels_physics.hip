// Physics: exploration and takeover (Experiment: explore actuators spread
// infrastructure to the neighbour of the maximal actuator; if the exploring
// infrastructure exceeds the explored cell's, that cell adopts the explorer's
// genome and the rotation of the exploration, otherwise the infrastructure is
// absorbed; among several explorers the maximal investment wins).
//
// Pull form on an LDS-staged halo tile: every target t reads, for each
// direction d, the flow its neighbour n = nbr(t, d) sent toward (d+4) mod 8
// (word (d+4) mod 8 of n's 8-word flow record), and n's explore direction;
// I2 = I1 - sum(own flows) + sum(inflows); the
// candidate explorers are the neighbours exploring toward t, the largest
// investment wins (lowest d on ties) and takes t over when it strictly
// exceeds I1(t).  The next state's ledger pair is (E2, I2): energy does not
// move between cells, and E2 = E1 plus the day / night cycle's source and
// sink (exact integers, see day_night).  Each flow word is (amount << 1) | explored, so one read per
// direction gives both the inflow and the candidacy.  The tile loads the
// flow records and genomes of (TW+2) x (TH+2) cells with coalesced row
// loads; outflows, inflows, takeover and the block's share of the total-mass
// reduction (int64 exact and FP64) follow from LDS.  Pure integer work:
// bit-exact by construction.
#include "coralai_internal.h"

namespace coralai {

// counts[g] += d for every lane with `on`, one atomic per distinct index of
// the wavefront (index = stripe * capacity + genome): takeovers cluster on a
// few genomes (early steps from a random state take over a large share of
// the grid), and per-lane atomics on one address would serialise.  Call with
// the whole wavefront converged.
__device__ __forceinline__ void wave_count_add(int32_t* counts, int g, int d, bool on) {
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(on);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int gl = __shfl(g, leader, 64);
        const uint64_t same = __ballot(on && g == gl) & pending;
        if (lane == leader) atomicAdd(counts + gl, d * (int)__popcll(same));
        pending &= ~same;
    }
}

// Energy transport (physics variant): the net energy a cell gains, the words
// (d+4) mod 8 of its 8 neighbours' energy records (what each sends toward it)
// minus the sum of its own record, read through the caches.  Each word is
// (amount << 1).
__device__ __forceinline__ int64_t energy_moved(const uint32_t* __restrict__ eflow, int x, int y, int W, int H) {
    const int64_t t = (int64_t)y * W + x;
    const coralai_u32x4 a = gld((const coralai_u32x4*)(eflow + 8 * t));
    const coralai_u32x4 c = gld((const coralai_u32x4*)(eflow + 8 * t) + 1);
    int64_t net = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) net -= (int64_t)(a[k] >> 1) + (int64_t)(c[k] >> 1);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        int nx = x + dir_dx(d), ny = y + dir_dy(d);
        nx = nx < 0 ? nx + W : (nx >= W ? nx - W : nx);
        ny = ny < 0 ? ny + H : (ny >= H ? ny - H : ny);
        net += (int64_t)(gld(eflow + 8 * ((int64_t)ny * W + nx) + ((d + 4) & 7)) >> 1);
    }
    return net;
}

// Adds a wavefront's injected and removed quanta and error bits to the
// world's step accumulators (one atomic each from the first lane holding a
// nonzero sum; the cycle is off in most worlds).
__device__ __forceinline__ void day_night_flush(Ctl* ctl, int64_t inj, int64_t rem, uint32_t err, int lane) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        inj += __shfl_xor(inj, o, 64);
        rem += __shfl_xor(rem, o, 64);
        err |= __shfl_xor(err, o, 64);
    }
    if (lane == 0 && ctl != nullptr) {
        if (inj) atomicAdd((unsigned long long*)&ctl->acc_injected, (unsigned long long)inj);
        if (rem) atomicAdd((unsigned long long*)&ctl->acc_removed, (unsigned long long)rem);
        if (err) atomicOr(&ctl->err, err);
    }
}

// ENERGY: the instantiation launched while energy transport is on in some
// world of the launch; it loads the energy records with the tile's other
// loads.  The other one reads them per cell (correct, slower) if it meets a
// world with energy transport on.
template <int TW, int TH, bool ENERGY>
__global__ __launch_bounds__(256) void k_physics(const BatchDev* __restrict__ b) {
    constexpr int NT = 256, CPT = TW * TH / NT;  // threads, cells per thread
    static_assert(TW * TH % NT == 0, "a tile is a whole number of cells per thread");
    constexpr int LW = TW + 2, LH = TH + 2, LN = LW * LH;
    __shared__ uint32_t s_flow[8][LN];
    __shared__ int32_t s_g[LN];
    __shared__ int64_t s_red_m[NT / 64];
    __shared__ double s_red_f[NT / 64];
    __shared__ int s_red_t[NT / 64];

    const int nworlds = cld(&b->n_worlds);
    if (nworlds <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t total = cld(b->tile_prefix + (nworlds));
    int64_t tile, tend;
    balanced_share(total, xcd_block(), gridDim.x, &tile, &tend);

    int wi = -1;
    int64_t world_hi = -1;
    int64_t acc_m = 0, acc_inj = 0, acc_rem = 0;
    double acc_f = 0.0;
    int acc_t = 0;
    uint32_t err = 0;
    Ctl* ctl = nullptr;
    DayNight dn{0, 0, 1, 0};

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
        day_night_flush(ctl, acc_inj, acc_rem, err, lane);
        acc_m = 0;
        acc_f = 0.0;
        acc_t = 0;
        acc_inj = 0;
        acc_rem = 0;
        err = 0;
    };

    int Wd = 0, Hd = 0, Nd = 0, tx_n = 1;
    int64_t world_lo = 0;
    const uint32_t* flow = nullptr;
    const uint32_t* eflow = nullptr;  // non-null: energy transport
    const int64_t* EI1p = nullptr;
    const int32_t* Gc = nullptr;
    const uint8_t* Rc = nullptr;
    int64_t* EIn = nullptr;
    int32_t* Gn = nullptr;
    uint8_t* Rn = nullptr;
    int32_t* cnt = nullptr;  // stripe counts
    int capw = 0, btx = 1;

    for (; tile < tend; ++tile) {
        if (tile >= world_hi) {
            if (wi >= 0) flush();
            wi = find_world(b->tile_prefix, nworlds, tile);
            world_lo = cld(b->tile_prefix + (wi));
            world_hi = cld(b->tile_prefix + (wi + 1));
            const auto* W = world_at(b, wi);
            Wd = W->W; Hd = W->H; Nd = W->N;
            tx_n = cld(b->tiles_x + (wi));
            ctl = W->ctl;
            dn = day_night(W->day_period, W->day_inject, W->night_num, cld(&ctl->steps));
            const int cur = ctl_cur(ctl), nxt = cur ^ 1;
            flow = W->flow; EI1p = W->EI1;
            eflow = W->kappa_e > 0.f ? W->eflow : nullptr;
            Gc = W->G[cur]; Rc = W->R[cur];
            EIn = W->EI[nxt]; Gn = W->G[nxt]; Rn = W->R[nxt];
            cnt = W->stripe_counts;
            capw = W->cap;
            btx = W->btiles_x;
        }
        const int64_t lt = tile - world_lo;
        const int ty = (int)(lt / tx_n), tx = (int)(lt - (int64_t)ty * tx_n);
        const int x0 = tx * TW, y0 = ty * TH;

        // Every load of the tile is issued before any is used: the thread's
        // own cells (tile cells tid + NT k; a cell outside the world reads
        // cell 0) and its share of the halo tile, staged through registers.
        // (Loads under a branch, or a loop that writes each load to LDS
        // before the next, compile to a wait for every load before it.)
        int cx[CPT], cy[CPT], ct[CPT];
        bool mine[CPT];
        i64x2 ei1[CPT];
        uint8_t r_own[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int cc = tid + NT * k;
            cx[k] = cc % TW + 1;
            cy[k] = cc / TW + 1;
            const int gx = x0 + cx[k] - 1, gy = y0 + cy[k] - 1;
            mine[k] = gx < Wd && gy < Hd;
            ct[k] = mine[k] ? gy * Wd + gx : 0;
            ei1[k] = gld((const i64x2*)EI1p + ct[k]);
            r_own[k] = gld(Rc + ct[k]);
        }
        // energy transport: each own cell's record and the word its 8
        // neighbours send toward it
        int64_t emoved[CPT];
        coralai_u32x4 ea[CPT], ec[CPT];
        uint32_t en[CPT][8];
        if constexpr (ENERGY) {
            if (eflow) {
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const int x = (x0 + cx[k] - 1 < Wd) ? x0 + cx[k] - 1 : 0;
                    const int y = (y0 + cy[k] - 1 < Hd) ? y0 + cy[k] - 1 : 0;
                    const int64_t t = (int64_t)y * Wd + x;
                    ea[k] = gld((const coralai_u32x4*)(eflow + 8 * t));
                    ec[k] = gld((const coralai_u32x4*)(eflow + 8 * t) + 1);
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        int nx = x + dir_dx(d), ny = y + dir_dy(d);
                        nx = nx < 0 ? nx + Wd : (nx >= Wd ? nx - Wd : nx);
                        ny = ny < 0 ? ny + Hd : (ny >= Hd ? ny - Hd : ny);
                        en[k][d] = gld(eflow + 8 * ((int64_t)ny * Wd + nx) + ((d + 4) & 7));
                    }
                }
            }
        }
        constexpr int HIT = (LN + NT - 1) / NT;  // halo entries per thread
        const bool small = Wd < TW + 2 || Hd < TH + 2;  // tiny worlds wrap more than once
        coralai_u32x4 fa[HIT], fb[HIT];
        int32_t gh[HIT];
#pragma unroll
        for (int j = 0; j < HIT; ++j) {
            const int idx = (tid + NT * j < LN) ? tid + NT * j : 0;
            const int ly = idx / LW, lx = idx - ly * LW;
            int gx = x0 + lx - 1, gy = y0 + ly - 1;
            if (small) {
                gx = wrap(gx, Wd);
                gy = wrap(gy, Hd);
            } else {
                gx = gx < 0 ? gx + Wd : (gx >= Wd ? gx - Wd : gx);
                gy = gy < 0 ? gy + Hd : (gy >= Hd ? gy - Hd : gy);
            }
            const int n = gy * Wd + gx;
            fa[j] = gld((const coralai_u32x4*)(flow + 8 * (int64_t)n));
            fb[j] = gld((const coralai_u32x4*)(flow + 8 * (int64_t)n) + 1);
            gh[j] = gld(Gc + n);
        }
        // Everything issued so far is needed now (own cells and halo; the
        // previous tile's stores went out before them).  A full wait here
        // costs nothing and tells the compiler so: otherwise the halo loads
        // whose LDS write a thread skips stay pending in its bookkeeping, and
        // the first reuse of their registers waits for every store after them.
        __builtin_amdgcn_s_waitcnt(0);
        if constexpr (ENERGY) {
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                int64_t net = 0;
                if (eflow) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) net -= (int64_t)(ea[k][q] >> 1) + (int64_t)(ec[k][q] >> 1);
#pragma unroll
                    for (int d = 0; d < 8; ++d) net += (int64_t)(en[k][d] >> 1);
                }
                emoved[k] = net;
            }
        }
#pragma unroll
        for (int j = 0; j < HIT; ++j) {
            const int idx = tid + NT * j;
            if (idx < LN) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    s_flow[k][idx] = fa[j][k];
                    s_flow[4 + k][idx] = fb[j][k];
                }
                s_g[idx] = gh[j];
            }
        }
        __syncthreads();

        bool took[CPT];
        int32_t g_from[CPT], g_to[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int lx = cx[k], ly = cy[k];
            took[k] = false;
            g_from[k] = 0;
            g_to[k] = 0;
            if (mine[k]) {
                const int t = ct[k];
                const int own = ly * LW + lx;
                int64_t out = 0, in = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) out += s_flow[q][own] >> 1;
                int win = -1;
                int64_t vbest = -1;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int back = (d + 4) & 7;
                    const int nb = (ly + dir_dy(d)) * LW + (lx + dir_dx(d));
                    const uint32_t word = s_flow[back][nb];
                    const int64_t v = word >> 1;
                    in += v;
                    if ((word & 1u) && v > vbest) { vbest = v; win = d; }
                }
                const int64_t e1 = ei1[k][0], i1 = ei1[k][1];
                const int64_t i2 = i1 - out + in;
                int32_t g2 = s_g[own];
                uint8_t r2 = r_own[k];
                if (win >= 0 && vbest > i1) {
                    const int so = cell_stripe(x0 + lx - 1, y0 + ly - 1, btx) * capw;
                    g_from[k] = so + g2;
                    g2 = s_g[(ly + dir_dy(win)) * LW + (lx + dir_dx(win))];
                    r2 = (uint8_t)((win + 4) & 7);
                    acc_t += 1;
                    took[k] = true;
                    g_to[k] = so + g2;
                }
                int64_t em = e1;
                if constexpr (ENERGY) em += emoved[k];
                else if (eflow) em += energy_moved(eflow, x0 + lx - 1, y0 + ly - 1, Wd, Hd);
                const int64_t e2 = day_night_energy(em, dn, acc_inj, acc_rem, err);
                // the next state, read by the next step's kernels and not
                // here: stores with the non-temporal hint
                __builtin_nontemporal_store(i64x2{e2, i2}, (i64x2*)EIn + t);
                __builtin_nontemporal_store(g2, Gn + t);
                __builtin_nontemporal_store(r2, Rn + t);
                // the network kernel added E1; the energy moved, the cycle's change and I2 complete the sum
                acc_m += i2 + (e2 - e1);
                acc_f += (double)(i2 + (e2 - e1));
            }
        }
        // the genome counts follow the takeovers (the next step and radiation
        // use them); after all the tile's stores, and skipped by a wavefront
        // with no takeover (the common case)
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            if (__ballot(took[k])) {
                wave_count_add(cnt, g_from[k], -1, took[k]);
                wave_count_add(cnt, g_to[k], 1, took[k]);
            }
        }
        __syncthreads();  // LDS reused by the next tile
    }
    if (wi >= 0) flush();
}

// Streaming variant, no LDS.  The inflow from direction d is word (d+4) mod 8
// of the neighbour's flow record; each word is read by exactly one target,
// and the cell's outflow total is the sum of its own record.  Buffer loads
// keep the offsets in 32 bits (the records are < 2 GiB) and return 0 outside
// a buffer.

__global__ __launch_bounds__(256) void k_physics_stream(const BatchDev* __restrict__ b) {
    __shared__ int64_t s_red_m[4];
    __shared__ double s_red_f[4];
    __shared__ int s_red_t[4];
    const int nworlds = cld(&b->n_worlds);
    if (nworlds <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t total = cld(b->tile_prefix + (nworlds));
    int wi = -1;
    int64_t world_hi = -1, world_lo = 0;
    int64_t acc_m = 0, acc_inj = 0, acc_rem = 0;
    double acc_f = 0.0;
    int acc_t = 0;
    uint32_t err = 0;
    Ctl* ctl = nullptr;
    DayNight dn{0, 0, 1, 0};
    int Wd = 0, Hd = 0, Nd = 0;
    __amdgpu_buffer_rsrc_t rflow, rei1, rg, rr;
    int32_t* cnt = nullptr;  // stripe counts
    int capw = 0, btx = 1;
    int64_t* EIn = nullptr;
    int32_t* Gn = nullptr;
    uint8_t* Rn = nullptr;
    const uint32_t* eflow = nullptr;  // non-null: energy transport
    auto flush = [&]() {
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
            atomicAdd((unsigned long long*)&ctl->acc_mass,
                      (unsigned long long)(s_red_m[0] + s_red_m[1] + s_red_m[2] + s_red_m[3]));
            atomicAdd(&ctl->acc_mass_f64, s_red_f[0] + s_red_f[1] + s_red_f[2] + s_red_f[3]);
            atomicAdd((unsigned long long*)&ctl->acc_takeovers,
                      (unsigned long long)(int64_t)(s_red_t[0] + s_red_t[1] + s_red_t[2] + s_red_t[3]));
        }
        __syncthreads();
        day_night_flush(ctl, acc_inj, acc_rem, err, lane);
        acc_m = 0;
        acc_f = 0.0;
        acc_t = 0;
        acc_inj = 0;
        acc_rem = 0;
        err = 0;
    };
    int64_t unit, uend;
    balanced_share(total, xcd_block(), gridDim.x, &unit, &uend);
    for (; unit < uend; ++unit) {
        if (unit >= world_hi) {
            if (wi >= 0) flush();
            wi = find_world(b->tile_prefix, nworlds, unit);
            world_lo = cld(b->tile_prefix + (wi));
            world_hi = cld(b->tile_prefix + (wi + 1));
            const auto* W = world_at(b, wi);
            Wd = W->W; Hd = W->H; Nd = W->N;
            ctl = W->ctl;
            dn = day_night(W->day_period, W->day_inject, W->night_num, cld(&ctl->steps));
            const int cur = ctl_cur(ctl), nxt = cur ^ 1;
            const uint32_t n4 = 4u * (uint32_t)Nd;
            rflow = buf_rsrc(W->flow, 8u * n4);
            rei1 = buf_rsrc(W->EI1, 4u * n4);
            rg = buf_rsrc(W->G[cur], n4);
            rr = buf_rsrc(W->R[cur], (uint32_t)Nd);
            EIn = W->EI[nxt]; Gn = W->G[nxt]; Rn = W->R[nxt];
            cnt = W->stripe_counts;
            capw = W->cap;
            btx = W->btiles_x;
            eflow = W->kappa_e > 0.f ? W->eflow : nullptr;
        }
        if ((Wd & 3) == 0) {
            // four consecutive cells of one row per thread: their own flow
            // records (aligned 16-byte loads) give the outflows and, within
            // the row, the east / west inflows; the other inflow words are
            // single words of the records in rows y-1 and y+1 (wrapping
            // around the row at the group's edges).
            const int t0 = (int)((unit - world_lo) * 1024) + 4 * tid;
            bool took[4] = {false, false, false, false};
            int32_t g_from[4] = {0, 0, 0, 0}, g_to[4] = {0, 0, 0, 0};
            if (t0 < Nd) {
                const int y = t0 / Wd, x0 = t0 - y * Wd;
                const int row[3] = {(y == 0 ? Hd - 1 : y - 1) * Wd, y * Wd, (y == Hd - 1 ? 0 : y + 1) * Wd};
                const int xl = x0 == 0 ? Wd - 1 : x0 - 1, xr = x0 + 4 == Wd ? 0 : x0 + 4;
                uint32_t ow[4][8];  // own flow records
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const coralai_u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rflow, 32 * (t0 + j), 0, 0);
                    const coralai_u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(rflow, 32 * (t0 + j) + 16, 0, 0);
#pragma unroll
                    for (int k = 0; k < 4; ++k) { ow[j][k] = a[k]; ow[j][4 + k] = c[k]; }
                }
                uint32_t fw[8][4];
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int dx = dir_dx(d), dy = dir_dy(d), back = (d + 4) & 7, base = row[dy + 1];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int c = j + dx;  // column within the group, -1..4
                        if (dy == 0 && c >= 0 && c < 4) {
                            fw[d][j] = ow[c][back];
                        } else {
                            const int x = c < 0 ? xl : (c > 3 ? xr : x0 + c);
                            fw[d][j] = __builtin_amdgcn_raw_buffer_load_b32(rflow, 32 * (base + x) + 4 * back, 0, 0);
                        }
                    }
                }
                i64x2 ei1[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) ei1[j] = buf_ld_i64x2(rei1, 16 * (t0 + j));
                uint32_t outs[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    uint32_t o = 0;
#pragma unroll
                    for (int k = 0; k < 8; ++k) o += ow[j][k] >> 1;
                    outs[j] = o;
                }
                coralai_u32x4 gs = __builtin_amdgcn_raw_buffer_load_b128(rg, 4 * t0, 0, 0);
                uint32_t rs = __builtin_amdgcn_raw_buffer_load_b32(rr, t0, 0, 0);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int64_t in = 0, vbest = -1;
                    int win = -1;
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        const uint32_t word = fw[d][j];
                        const int64_t v = word >> 1;
                        in += v;
                        if ((word & 1u) && v > vbest) { vbest = v; win = d; }
                    }
                    const int64_t e1 = ei1[j][0], i1 = ei1[j][1];
                    const int64_t i2 = i1 - (int64_t)outs[j] + in;
                    if (win >= 0 && vbest > i1) {
                        const int x = x0 + j;
                        int nx = x + dir_dx(win);
                        nx = nx < 0 ? nx + Wd : (nx >= Wd ? nx - Wd : nx);
                        const int n = row[dir_dy(win) + 1] + nx;
                        const int so = cell_stripe(x, y, btx) * capw;
                        g_from[j] = so + (int32_t)gs[j];
                        gs[j] = __builtin_amdgcn_raw_buffer_load_b32(rg, 4 * n, 0, 0);
                        g_to[j] = so + (int32_t)gs[j];
                        rs = (rs & ~(0xffu << (8 * j))) | ((uint32_t)((win + 4) & 7) << (8 * j));
                        took[j] = true;
                        acc_t += 1;
                    }
                    const int64_t em = eflow ? e1 + energy_moved(eflow, x0 + j, y, Wd, Hd) : e1;
                    const int64_t e2 = day_night_energy(em, dn, acc_inj, acc_rem, err);
                    __builtin_nontemporal_store(i64x2{e2, i2}, (i64x2*)EIn + t0 + j);
                    acc_m += i2 + (e2 - e1);
                    acc_f += (double)(i2 + (e2 - e1));
                }
                __builtin_nontemporal_store(gs, (coralai_u32x4*)Gn + t0 / 4);
                __builtin_nontemporal_store(rs, (uint32_t*)Rn + t0 / 4);
            }
            // the genome counts follow the takeovers (the next step and radiation use them)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                wave_count_add(cnt, g_from[j], -1, took[j]);
                wave_count_add(cnt, g_to[j], 1, took[j]);
            }
            continue;
        }
        const int t = (int)((unit - world_lo) * 256) + tid;
        bool took = false;
        int32_t g_from = 0, g_to = 0;
        if (t < Nd) {  // (no divergent continue: the world fields must stay uniform)
            const int y = t / Wd, x = t - y * Wd;
            const i64x2 ei1 = buf_ld_i64x2(rei1, 16 * t);
            const int64_t e1 = ei1[0], i1 = ei1[1];
            const coralai_u32x4 oa = __builtin_amdgcn_raw_buffer_load_b128(rflow, 32 * t, 0, 0);
            const coralai_u32x4 ob = __builtin_amdgcn_raw_buffer_load_b128(rflow, 32 * t + 16, 0, 0);
            uint32_t out = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) out += (oa[k] >> 1) + (ob[k] >> 1);
            int32_t g2 = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rg, 4 * t, 0, 0);
            uint8_t r2 = __builtin_amdgcn_raw_buffer_load_b8(rr, t, 0, 0);
            int64_t in = 0, vbest = -1;
            int win = -1, wn = 0;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                int nx = x + dir_dx(d), ny = y + dir_dy(d);
                nx = nx < 0 ? nx + Wd : (nx >= Wd ? nx - Wd : nx);
                ny = ny < 0 ? ny + Hd : (ny >= Hd ? ny - Hd : ny);
                const int n = ny * Wd + nx;
                const uint32_t word = __builtin_amdgcn_raw_buffer_load_b32(rflow, 32 * n + 4 * ((d + 4) & 7), 0, 0);
                const int64_t v = word >> 1;
                in += v;
                if ((word & 1u) && v > vbest) { vbest = v; win = d; wn = n; }
            }
            const int64_t i2 = i1 - (int64_t)out + in;
            if (win >= 0 && vbest > i1) {
                const int so = cell_stripe(x, y, btx) * capw;
                g_from = so + g2;
                g2 = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rg, 4 * wn, 0, 0);
                r2 = (uint8_t)((win + 4) & 7);
                acc_t += 1;
                took = true;
                g_to = so + g2;
            }
            const int64_t em = eflow ? e1 + energy_moved(eflow, x, y, Wd, Hd) : e1;
            const int64_t e2 = day_night_energy(em, dn, acc_inj, acc_rem, err);
            __builtin_nontemporal_store(i64x2{e2, i2}, (i64x2*)EIn + t);
            __builtin_nontemporal_store(g2, Gn + t);
            __builtin_nontemporal_store(r2, Rn + t);
            acc_m += i2 + (e2 - e1);
            acc_f += (double)(i2 + (e2 - e1));
        }
        // the genome counts follow the takeovers (the next step and radiation use them)
        wave_count_add(cnt, g_from, -1, took);
        wave_count_add(cnt, g_to, 1, took);
    }
    if (wi >= 0) flush();
}

int phys_tile_w(int t) { return t == 1 ? 32 : 64; }
int phys_tile_h(int t) { return t == 1 ? 8 : (t == 2 ? 8 : 16); }

void launch_physics_only(const BatchDev* bdev, const LaunchShape& ls, int phys_tile,
                         hipStream_t s) {
    const bool e = (ls.act_variants & 2) != 0;  // energy transport on in some world
    switch (phys_tile) {
        case 3: hipLaunchKernelGGL(k_physics_stream, dim3(ls.phys_blocks), dim3(256), 0, s, bdev); break;
        case 1:
            if (e) hipLaunchKernelGGL((k_physics<32, 8, true>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev);
            else hipLaunchKernelGGL((k_physics<32, 8, false>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev);
            break;
        case 2:
            if (e) hipLaunchKernelGGL((k_physics<64, 8, true>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev);
            else hipLaunchKernelGGL((k_physics<64, 8, false>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev);
            break;
        default:
            if (e) hipLaunchKernelGGL((k_physics<64, 16, true>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev);
            else hipLaunchKernelGGL((k_physics<64, 16, false>), dim3(ls.phys_blocks), dim3(256), 0, s, bdev);
            break;
    }
}

void launch_step_kernels(const BatchDev* bdev, const LaunchShape& ls, int NL, int HID, int prec,
                         int act_cells, int act_waves, int phys_tile, hipStream_t s,
                         float* debug_act, int recount) {
    launch_bucket_only(bdev, ls, s, recount);
    launch_act_only(bdev, ls, NL, HID, prec, act_cells, act_waves, s, debug_act);
    launch_physics_only(bdev, ls, phys_tile, s);
    launch_finalize(bdev, ls, s);
}

// Communication channels between the C ABI's planar layout and the device's
// interleaved one (set_state / get_state only).
__global__ __launch_bounds__(256) void k_comm_layout(const float* __restrict__ src, float* __restrict__ dst,
                                                     int64_t n, int to_interleaved) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (to_interleaved) {
            float4 v;
            v.x = src[i]; v.y = src[n + i]; v.z = src[2 * n + i]; v.w = src[3 * n + i];
            reinterpret_cast<float4*>(dst)[i] = v;
        } else {
            const float4 v = reinterpret_cast<const float4*>(src)[i];
            dst[i] = v.x; dst[n + i] = v.y; dst[2 * n + i] = v.z; dst[3 * n + i] = v.w;
        }
    }
}

__global__ __launch_bounds__(256) void k_ledger_pack(const int64_t* __restrict__ e, int e_stride,
                                                     const int64_t* __restrict__ v, int v_stride,
                                                     int64_t* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        reinterpret_cast<i64x2*>(dst)[i] = i64x2{e[i * e_stride], v[i * v_stride]};
}

__global__ __launch_bounds__(256) void k_ledger_unpack(const int64_t* __restrict__ src, int64_t* __restrict__ e,
                                                       int64_t* __restrict__ v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const i64x2 p = reinterpret_cast<const i64x2*>(src)[i];
        if (e) e[i] = p[0];
        if (v) v[i] = p[1];
    }
}

static int layout_blocks(int64_t n) {
    const int64_t want = (n + 255) / 256;
    return (int)(want < 4096 ? want : 4096);
}

void launch_ledger_pack(const int64_t* e, int e_stride, const int64_t* v, int v_stride, int64_t* dst,
                        int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ledger_pack, dim3(layout_blocks(n)), dim3(256), 0, s, e, e_stride, v, v_stride, dst, n);
}

void launch_ledger_unpack(const int64_t* src, int64_t* e, int64_t* v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ledger_unpack, dim3(layout_blocks(n)), dim3(256), 0, s, src, e, v, n);
}

void launch_comm_layout(const float* src, float* dst, int64_t n, int to_interleaved, hipStream_t s) {
    if (n <= 0) return;
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_comm_layout, dim3(blocks), dim3(256), 0, s, src, dst, n, to_interleaved);
}

}  // namespace coralai
