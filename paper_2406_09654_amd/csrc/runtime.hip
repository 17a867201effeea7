// Host runtime and C ABI of the gfx950 Coralai library: arena carving,
// world and batch objects, launch orchestration (direct launches or a
// captured HIP graph of persistent kernels), the autotuner, stats and error
// reporting, and the parity hooks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/coralai.h"
#include "coralai_internal.h"

using namespace coralai;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(CORALAI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    size_t EI[2], C[2], G[2], R[2];
    size_t flow, EI1, perm;
    size_t counts, offsets, stripe_counts, cursor, gofs, slot_set, params, ext_w, ext_mask, wfrag, bias;
    size_t hit_bits, blk_hits, blk_ofs, free_list, new_slots, stage_slots, stage_params;
    size_t eflow;  // 0: not reserved
    size_t lineage_parent, lineage_parent2, lineage_birth;
    size_t scan_part, ctl, wdev, bdev, chunk_prefix, slot_prefix, tile_prefix, group_prefix, tiles_x;
    int n_slot_blocks;
    size_t total;
    int64_t wfrag_stride;
    int bias_stride;
    int n_rad_blocks;
};

bool desc_valid(const coralai_world_desc* d, std::string* why) {
    auto bad = [&](const char* m) { if (why) *why = m; return false; };
    if (!d) return bad("desc is NULL");
    if (d->width < 1 || d->height < 1) return bad("width and height must be >= 1");
    if ((int64_t)d->width * d->height > (1ll << 26)) return bad("W*H must be <= 2^26");
    if (d->n_weight_layers != 2 && d->n_weight_layers != 3) return bad("n_weight_layers must be 2 or 3");
    if (d->hidden != 32 && d->hidden != 64) return bad("hidden must be 32 or 64");
    if (d->genome_capacity < 1 || d->genome_capacity > (1 << 22)) return bad("genome_capacity must be in [1, 2^22]");
    if (d->precision != CORALAI_FP32 && d->precision != CORALAI_BF16) return bad("precision must be CORALAI_FP32 or CORALAI_BF16");
    if (d->flags & ~CORALAI_WORLD_ENERGY_FLOWS) return bad("unknown flags");
    for (float v : {d->rho_invest, d->rho_liquidate, d->kappa_flow})
        if (!(v >= 0.0f && v <= 1.0f)) return bad("rho_invest, rho_liquidate, kappa_flow must be in [0, 1]");
    return true;
}

Layout make_layout(const coralai_world_desc* d) {
    Layout L{};
    const size_t N = (size_t)d->width * d->height, cap = (size_t)d->genome_capacity;
    size_t off = 0;
    auto take = [&](size_t bytes) { off = align_up(off, kAlign); size_t o = off; off += bytes; return o; };
    for (int k = 0; k < 2; ++k) {
        L.EI[k] = take(16 * N);
        L.C[k] = take(16 * N);
        L.G[k] = take(4 * N);
        L.R[k] = take(N);
    }
    L.flow = take(32 * N);
    L.eflow = (d->flags & CORALAI_WORLD_ENERGY_FLOWS) ? take(32 * N) : 0;
    L.EI1 = take(16 * N);
    L.perm = take(4 * N);
    L.counts = take(4 * cap);
    L.offsets = take(4 * (cap + 1));
    L.stripe_counts = take(4 * kStripes * cap);
    L.cursor = take(4 * kStripes * cap);
    L.gofs = take(4 * (cap + 1));
    L.slot_set = take(cap);
    L.params = take(4 * kNParam * cap);
    L.ext_w = take(4 * kNExtW * cap);
    L.ext_mask = take(16 * cap);
    L.lineage_parent = take(4 * cap);
    L.lineage_parent2 = take(4 * cap);
    L.lineage_birth = take(8 * cap);
    L.wfrag_stride = (int64_t)net_frags(d->n_weight_layers, d->hidden, d->precision) *
                     net_frag_bytes(d->precision);
    L.wfrag = take((size_t)L.wfrag_stride * cap);
    L.bias_stride = net_bias_floats(d->n_weight_layers, d->hidden);
    L.bias = take(4 * (size_t)L.bias_stride * cap);
    L.n_rad_blocks = (int)((N + kRadBlockCells - 1) / kRadBlockCells);
    L.hit_bits = take(2 * 256 * (size_t)L.n_rad_blocks);
    L.blk_hits = take(4 * (size_t)L.n_rad_blocks);
    L.blk_ofs = take(4 * ((size_t)L.n_rad_blocks + 1));
    L.free_list = take(4 * cap);
    L.new_slots = take(4 * cap);
    L.stage_slots = take(4 * cap);
    L.stage_params = take(4 * kNParam * cap);
    L.n_slot_blocks = (int)((cap + kSlotBlock - 1) / kSlotBlock);
    L.scan_part = take(16 * (size_t)L.n_slot_blocks);
    L.ctl = take(sizeof(Ctl));
    L.wdev = take(sizeof(WorldDev));
    L.bdev = take(sizeof(BatchDev));
    L.chunk_prefix = take(16);
    L.slot_prefix = take(16);
    L.tile_prefix = take(16);
    L.group_prefix = take(8);
    L.tiles_x = take(4);
    L.total = align_up(off, kAlign);
    return L;
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

LaunchShape make_shape(int max_worlds, int max_cap) {
    LaunchShape ls{};
    ls.n_cu = device_cus();
    ls.act_blocks = ls.n_cu * 2;
    ls.phys_blocks = ls.n_cu * 16;
    ls.chunk_blocks = ls.n_cu * 4;
    ls.misc_blocks = ls.n_cu;
    ls.max_worlds = max_worlds;
    ls.max_cap = max_cap;
    ls.scan_fused = (max_cap + kSlotBlock - 1) / kSlotBlock <= kFuseSlotBlocks ? 1 : 0;
    return ls;
}

struct BusyGuard {
    std::atomic<int>* flag;
    bool ok;
    explicit BusyGuard(std::atomic<int>* f) : flag(f) {
        int expect = 0;
        ok = flag->compare_exchange_strong(expect, 1);
    }
    ~BusyGuard() { if (ok) flag->store(0); }
};

}  // namespace

struct coralai_world {
    coralai_world_desc desc;
    Layout L;
    int device = 0;      // current device at creation: the arena's and the stream's
    hipStream_t stream;
    uint8_t* base;
    WorldDev host;       // the device table entry, host copy
    WorldDev* wdev;
    BatchDev* bdev;
    LaunchShape ls;
    int act_cells = 2;
    int act_waves = 0;
    int phys_tile = 2;
    hipGraphExec_t graph = nullptr;     // the step
    int graph_key = -1;
    hipGraphExec_t graph_rc = nullptr;  // the step with the genome recount first
    int graph_rc_key = -1;
    // the device counts may not describe the current state (a new state, the
    // autotuner's trials, a debug hook): the next bucketing recounts
    bool counts_stale = true;
    Ctl* pinned = nullptr;
    // live phase timing
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double prof_ms[CORALAI_PHASES] = {0, 0, 0, 0, 0};
    int64_t prof_n[CORALAI_PHASES] = {0, 0, 0, 0, 0};
    std::atomic<int> busy{0};
};

struct coralai_batch {
    int max_worlds;
    hipStream_t stream;
    uint8_t* base;
    BatchDev* bdev;
    WorldDev* table;
    int64_t* chunk_prefix;
    int64_t* slot_prefix;
    int64_t* tile_prefix;
    int32_t* group_prefix;
    int32_t* tiles_x;
    int n = 0;
    int NL = 0, HID = 0, prec = 0;
    int act_cells = 2, act_waves = 0, phys_tile = 2;
    LaunchShape ls;
    hipGraphExec_t graph = nullptr;
    int graph_key = -1;
    hipGraphExec_t graph_rc = nullptr;  // with the genome recount first
    int graph_rc_key = -1;
    // orders work between the batch's stream and its worlds' own streams
    hipEvent_t ev_order = nullptr;
    std::vector<coralai_world*> worlds;
    std::atomic<int> busy{0};
};

namespace {

int tiles_for(int W, int H, int phys_tile, int* tx) {
    if (phys_tile == 3) {  // streaming physics: linear units of 256 threads
        *tx = 0;
        const int64_t cells = (int64_t)W * H, per = phys_stream_cells(W);
        return (int)((cells + per - 1) / per);
    }
    const int tw = phys_tile_w(phys_tile), th = phys_tile_h(phys_tile);
    *tx = (W + tw - 1) / tw;
    return *tx * ((H + th - 1) / th);
}

int write_world_tables(coralai_world* w) {
    // single-world batch: table = the world itself
    int tx = 0;
    const int64_t tiles = tiles_for(w->desc.width, w->desc.height, w->phys_tile, &tx);
    const int64_t chunks = (w->host.btiles + kBucketGroup - 1) / kBucketGroup;
    int64_t cp[2] = {0, chunks}, tp[2] = {0, tiles}, sp[2] = {0, w->host.n_slot_blocks};
    BatchDev hb{};
    hb.n_worlds = 1;
    hb.worlds = w->wdev;
    hb.chunk_prefix = (int64_t*)(w->base + w->L.chunk_prefix);
    hb.slot_prefix = (int64_t*)(w->base + w->L.slot_prefix);
    hb.tile_prefix = (int64_t*)(w->base + w->L.tile_prefix);
    hb.group_prefix = (int32_t*)(w->base + w->L.group_prefix);
    hb.tiles_x = (int32_t*)(w->base + w->L.tiles_x);
    HIP_TRY(hipMemcpyAsync(w->wdev, &w->host, sizeof(WorldDev), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(w->bdev, &hb, sizeof(BatchDev), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(hb.chunk_prefix, cp, sizeof cp, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(hb.slot_prefix, sp, sizeof sp, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(hb.tile_prefix, tp, sizeof tp, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(hb.tiles_x, &tx, sizeof tx, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int read_ctl(coralai_world* w) {
    HIP_TRY(hipMemcpyAsync(w->pinned, w->host.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int report_errors(coralai_world* w, uint32_t* word_out) {
    int rc = read_ctl(w);
    if (rc) return rc;
    const uint32_t e = w->pinned->err;
    if (word_out) *word_out = e;
    if (e) {
        HIP_TRY(hipMemsetAsync(&w->host.ctl->err, 0, sizeof(uint32_t), w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        if (e & (CORALAI_ERR_GENOME_RANGE | CORALAI_ERR_GENOME_UNSET))
            return fail(CORALAI_E_GENOME, "a cell names a genome slot outside [0, capacity) or without parameters (error word 0x%x)", e);
        if (e & CORALAI_ERR_MASS)
            return fail(CORALAI_E_NUMERIC, "the total mass changed by other than the injected minus the removed quanta (error word 0x%x)", e);
        return fail(CORALAI_E_NUMERIC, "non-finite network output / CPPN weight or ledger overflow (error word 0x%x)", e);
    }
    return CORALAI_OK;
}

void fill_stats(const Ctl& c, coralai_stats* out) {
    out->mass_quanta = c.mass;
    out->mass_fp64 = c.mass_f64;
    out->steps = c.steps;
    out->live_genomes = c.live_pub;
    out->takeovers = c.takeovers;
    out->hits = c.hits_pub;
    out->dropped_hits = c.dropped_pub;
    out->error_word = c.err;
    out->reserved = 0;
}

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CORALAI_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return CORALAI_OK;
}

// The device genome counts no longer describe the current state (new state
// from the host, or trial launches that ran physics without committing it).
// The state changed outside a step (new state, a debug hook, the
// autotuner's trials): the genome counts must be recounted, and the next
// step has no previous total mass to check against.
int invalidate_counts(coralai_world* w) {
    w->counts_stale = true;
    HIP_TRY(hipMemsetAsync(&w->host.ctl->counts_valid, 0, sizeof(int32_t), w->stream));
    HIP_TRY(hipMemsetAsync(&w->host.ctl->mass_valid, 0, sizeof(int32_t), w->stream));
    return CORALAI_OK;
}

int current_buffer(coralai_world* w, int* cur) {
    int rc = read_ctl(w);
    if (rc) return rc;
    *cur = w->pinned->cur & 1;
    return CORALAI_OK;
}

int take_event(coralai_world* w, hipEvent_t* e) {
    if (!w->ev_pool.empty()) {
        *e = w->ev_pool.back();
        w->ev_pool.pop_back();
        return CORALAI_OK;
    }
    HIP_TRY(hipEventCreate(e));
    return CORALAI_OK;
}

// Harvest finished phase timings into the sums and recycle their events.
int harvest_profile(coralai_world* w) {
    if (w->ev_pending.empty()) return CORALAI_OK;
    HIP_TRY(hipStreamSynchronize(w->stream));
    for (auto& r : w->ev_pending) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.second.first, r.second.second));
        w->prof_ms[r.first] += ms;
        w->prof_n[r.first] += 1;
        w->ev_pool.push_back(r.second.first);
        w->ev_pool.push_back(r.second.second);
    }
    w->ev_pending.clear();
    return CORALAI_OK;
}

// Run fn between two events recorded on the world's stream (phase timing).
template <typename F>
int timed_phase(coralai_world* w, int phase, F&& fn) {
    if (!w->profiling) { fn(); return CORALAI_OK; }
    if (w->ev_pending.size() >= 512) {
        int rc = harvest_profile(w);
        if (rc) return rc;
    }
    hipEvent_t a, b;
    int rc = take_event(w, &a);
    if (!rc) rc = take_event(w, &b);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(a, w->stream));
    fn();
    HIP_TRY(hipEventRecord(b, w->stream));
    w->ev_pending.push_back({phase, {a, b}});
    return CORALAI_OK;
}

void destroy_graph(hipGraphExec_t* g) {
    if (*g) { (void)hipGraphExecDestroy(*g); *g = nullptr; }
}

// Capture the step sequence once; every size it needs is read on the device.
int tuning_key(int act_cells, int act_waves, int phys_tile, const LaunchShape& ls) {
    return (ls.scan_fused ? 0 : 10000) + ls.act_variants * 1000 + act_cells * 100 + act_waves * 10 + phys_tile;
}

int capture_step(hipStream_t s, const BatchDev* bdev, const LaunchShape& ls, int NL, int HID,
                 int prec, int act_cells, int act_waves, int phys_tile, int recount, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    launch_step_kernels(bdev, ls, NL, HID, prec, act_cells, act_waves, phys_tile, s, nullptr, recount);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return fail(CORALAI_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CORALAI_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    return CORALAI_OK;
}

}  // namespace

extern "C" {

const char* coralai_last_error(void) { return g_last_error.c_str(); }
const char* coralai_version(void) { return "coralai-gfx950 1.0"; }

size_t coralai_world_bytes(const coralai_world_desc* desc) {
    if (!desc_valid(desc, nullptr)) return 0;
    return make_layout(desc).total + kAlign;
}

int coralai_world_create(const coralai_world_desc* desc, void* dev_arena, size_t arena_bytes,
                         void* hip_stream, coralai_world** out) {
    std::string why;
    if (!out) return fail(CORALAI_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!desc_valid(desc, &why)) return fail(CORALAI_E_INVALID, "invalid world description: %s", why.c_str());
    if (!dev_arena) return fail(CORALAI_E_INVALID, "dev_arena is NULL");
    const size_t need = coralai_world_bytes(desc);
    if (arena_bytes < need)
        return fail(CORALAI_E_NOMEM, "arena of %zu bytes is smaller than the %zu bytes the world needs", arena_bytes, need);
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(CORALAI_E_HIP, "hipGetDevice failed");
    coralai_world* w = new coralai_world();
    w->device = device;
    w->desc = *desc;
    w->L = make_layout(desc);
    w->stream = (hipStream_t)hip_stream;
    w->base = (uint8_t*)align_up((uintptr_t)dev_arena, kAlign);
    if (hipHostMalloc((void**)&w->pinned, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        delete w;
        return fail(CORALAI_E_HIP, "hipHostMalloc of the stats block failed");
    }
    const Layout& L = w->L;
    uint8_t* b = w->base;
    WorldDev& h = w->host;
    memset(&h, 0, sizeof h);
    h.W = desc->width; h.H = desc->height; h.N = desc->width * desc->height; h.cap = desc->genome_capacity;
    row_magic(h.W, &h.w_magic, &h.w_shift);
    h.NL = desc->n_weight_layers; h.HID = desc->hidden; h.prec = desc->precision;
    h.n_rad_blocks = L.n_rad_blocks;
    h.rho_i = desc->rho_invest; h.rho_l = desc->rho_liquidate; h.kappa = desc->kappa_flow;
    h.seed = desc->seed;
    for (int k = 0; k < 2; ++k) {
        h.EI[k] = (int64_t*)(b + L.EI[k]);
        h.C[k] = (float*)(b + L.C[k]);
        h.G[k] = (int32_t*)(b + L.G[k]);
        h.R[k] = (uint8_t*)(b + L.R[k]);
    }
    h.flow = (uint32_t*)(b + L.flow);
    h.eflow = L.eflow ? (uint32_t*)(b + L.eflow) : nullptr;
    h.EI1 = (int64_t*)(b + L.EI1);
    h.perm = (int32_t*)(b + L.perm);
    h.counts = (int32_t*)(b + L.counts);
    h.offsets = (int32_t*)(b + L.offsets);
    h.stripe_counts = (int32_t*)(b + L.stripe_counts);
    h.cursor = (int32_t*)(b + L.cursor);
    h.gofs = (int32_t*)(b + L.gofs);
    h.slot_set = (uint8_t*)(b + L.slot_set);
    h.params = (float*)(b + L.params);
    h.ext_w = (float*)(b + L.ext_w);
    h.ext_mask = (uint32_t*)(b + L.ext_mask);
    h.lineage_parent = (int32_t*)(b + L.lineage_parent);
    h.lineage_parent2 = (int32_t*)(b + L.lineage_parent2);
    h.lineage_birth = (int64_t*)(b + L.lineage_birth);
    h.wfrag = (uint8_t*)(b + L.wfrag);
    h.bias = (float*)(b + L.bias);
    h.wfrag_stride = L.wfrag_stride;
    h.bias_stride = L.bias_stride;
    h.hit_bits = (uint16_t*)(b + L.hit_bits);
    h.blk_hits = (int32_t*)(b + L.blk_hits);
    h.blk_ofs = (int32_t*)(b + L.blk_ofs);
    h.free_list = (int32_t*)(b + L.free_list);
    h.new_slots = (int32_t*)(b + L.new_slots);
    h.stage_slots = (int32_t*)(b + L.stage_slots);
    h.stage_params = (float*)(b + L.stage_params);
    h.scan_part = (int32_t*)(b + L.scan_part);
    h.n_slot_blocks = L.n_slot_blocks;
    h.btiles_x = (h.W + kBucketTile - 1) / kBucketTile;
    h.btiles = h.btiles_x * ((h.H + kBucketTile - 1) / kBucketTile);
    h.ctl = (Ctl*)(b + L.ctl);
    w->wdev = (WorldDev*)(b + L.wdev);
    w->bdev = (BatchDev*)(b + L.bdev);
    w->ls = make_shape(1, h.cap);
    int rc = CORALAI_OK;
    if (hipMemsetAsync(b, 0, L.total, w->stream) != hipSuccess) rc = fail(CORALAI_E_HIP, "arena clear failed");
    if (!rc) rc = write_world_tables(w);
    if (rc) {
        (void)hipHostFree(w->pinned);
        delete w;
        return rc;
    }
    *out = w;
    return CORALAI_OK;
}

int coralai_world_destroy(coralai_world* w) {
    if (!w) return fail(CORALAI_E_INVALID, "world is NULL");
    BusyGuard g(&w->busy);
    if (!g.ok) return fail(CORALAI_E_BUSY, "world is in use");
    (void)hipStreamSynchronize(w->stream);
    destroy_graph(&w->graph);
    destroy_graph(&w->graph_rc);
    for (auto& r : w->ev_pending) { (void)hipEventDestroy(r.second.first); (void)hipEventDestroy(r.second.second); }
    for (hipEvent_t e : w->ev_pool) (void)hipEventDestroy(e);
    (void)hipHostFree(w->pinned);
    g.ok = false;
    delete w;
    return CORALAI_OK;
}

#define WORLD_GUARD(w)                                                            \
    if (!(w)) return fail(CORALAI_E_INVALID, "world is NULL");                    \
    BusyGuard guard_(&(w)->busy);                                                 \
    if (!guard_.ok) return fail(CORALAI_E_BUSY, "world is in use by another thread")

int coralai_set_state(coralai_world* w, const int64_t* e_q, const int64_t* i_q, const float* comm4,
                      const int32_t* genome, const uint8_t* rotation, int on_device) {
    WORLD_GUARD(w);
    {
        const int irc = invalidate_counts(w);
        if (irc) return irc;
    }
    if (!e_q || !i_q || !comm4 || !genome || !rotation) return fail(CORALAI_E_INVALID, "a state array is NULL");
    int cur = 0, rc = current_buffer(w, &cur);
    if (rc) return rc;
    const size_t N = (size_t)w->host.N;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    // e_q, i_q are planes; the device keeps [N][2] ledger pairs.  Host data is
    // staged through the flow planes (32N bytes), which hold nothing between
    // steps; each staging copy is ordered on the stream after the kernel
    // that consumed the previous one.
    {
        const int64_t *es = e_q, *is = i_q;
        if (!on_device) {
            int64_t* st = (int64_t*)w->host.flow;
            HIP_TRY(hipMemcpyAsync(st, e_q, 8 * N, hipMemcpyHostToDevice, w->stream));
            HIP_TRY(hipMemcpyAsync(st + N, i_q, 8 * N, hipMemcpyHostToDevice, w->stream));
            es = st;
            is = st + N;
        }
        launch_ledger_pack(es, 1, is, 1, w->host.EI[cur], (int64_t)N, w->stream);
    }
    // comm4 is planar; the device keeps [N][4].  Host data is staged through
    // the flow planes, which hold nothing between steps.
    const float* csrc = comm4;
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(w->host.flow, comm4, 16 * N, hipMemcpyHostToDevice, w->stream));
        csrc = (const float*)w->host.flow;
    }
    launch_comm_layout(csrc, w->host.C[cur], (int64_t)N, 1, w->stream);
    HIP_TRY(hipMemcpyAsync(w->host.G[cur], genome, 4 * N, k, w->stream));
    HIP_TRY(hipMemcpyAsync(w->host.R[cur], rotation, N, k, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_get_state(coralai_world* w, int64_t* e_q, int64_t* i_q, float* comm4, int32_t* genome,
                      uint8_t* rotation, int on_device) {
    WORLD_GUARD(w);
    int cur = 0, rc = current_buffer(w, &cur);
    if (rc) return rc;
    const size_t N = (size_t)w->host.N;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (e_q || i_q) {
        if (on_device) {
            launch_ledger_unpack(w->host.EI[cur], e_q, i_q, (int64_t)N, w->stream);
        } else {
            int64_t* st = (int64_t*)w->host.flow;
            launch_ledger_unpack(w->host.EI[cur], st, st + N, (int64_t)N, w->stream);
            if (e_q) HIP_TRY(hipMemcpyAsync(e_q, st, 8 * N, hipMemcpyDeviceToHost, w->stream));
            if (i_q) HIP_TRY(hipMemcpyAsync(i_q, st + N, 8 * N, hipMemcpyDeviceToHost, w->stream));
        }
    }
    if (comm4) {
        if (on_device) {
            launch_comm_layout(w->host.C[cur], comm4, (int64_t)N, 0, w->stream);
        } else {
            launch_comm_layout(w->host.C[cur], (float*)w->host.flow, (int64_t)N, 0, w->stream);
            HIP_TRY(hipMemcpyAsync(comm4, w->host.flow, 16 * N, hipMemcpyDeviceToHost, w->stream));
        }
    }
    if (genome) HIP_TRY(hipMemcpyAsync(genome, w->host.G[cur], 4 * N, k, w->stream));
    if (rotation) HIP_TRY(hipMemcpyAsync(rotation, w->host.R[cur], N, k, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_set_genomes(coralai_world* w, int32_t n, const int32_t* slot_ids, const float* cppn_params) {
    WORLD_GUARD(w);
    if (n < 0 || n > w->host.cap) return fail(CORALAI_E_INVALID, "n must be in [0, capacity]");
    if (n == 0) return CORALAI_OK;
    if (!slot_ids || !cppn_params) return fail(CORALAI_E_INVALID, "slot_ids / cppn_params is NULL");
    for (int k = 0; k < n; ++k)
        if (slot_ids[k] < 0 || slot_ids[k] >= w->host.cap)
            return fail(CORALAI_E_INVALID, "slot id %d outside [0, %d)", slot_ids[k], w->host.cap);
    HIP_TRY(hipMemcpyAsync(w->host.stage_slots, slot_ids, 4 * (size_t)n, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(w->host.stage_params, cppn_params, 4 * (size_t)kNParam * n, hipMemcpyHostToDevice, w->stream));
    launch_scatter_params(w->wdev, n, w->stream);
    launch_cppn(w->wdev, w->host.NL, w->host.HID, w->host.prec, 0, n, 0, 0.0f, w->ls.n_cu, w->stream);
    int rc = check_launch();
    if (rc) return rc;
    // the staging area held the last births: there are none to report now
    HIP_TRY(hipMemsetAsync(&w->host.ctl->n_new, 0, sizeof(int32_t), w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return report_errors(w, nullptr);
}

int coralai_set_genome_ext(coralai_world* w, int32_t n, const int32_t* slot_ids, const coralai_genome_ext* ext) {
    WORLD_GUARD(w);
    static_assert(sizeof(coralai_genome_ext) == 46 * 4, "46-word records");
    if (n < 0 || n > w->host.cap) return fail(CORALAI_E_INVALID, "n must be in [0, capacity]");
    if (n == 0) return CORALAI_OK;
    if (!slot_ids || !ext) return fail(CORALAI_E_INVALID, "slot_ids / ext is NULL");
    for (int k = 0; k < n; ++k) {
        if (slot_ids[k] < 0 || slot_ids[k] >= w->host.cap)
            return fail(CORALAI_E_INVALID, "slot id %d outside [0, %d)", slot_ids[k], w->host.cap);
        if ((ext[k].conn_mask >> 10) != 0u || (ext[k].node_mask >> 16) != 0u)
            return fail(CORALAI_E_INVALID, "conn_mask has 10 bits, node_mask 16");
        for (int m = 0; m < 10; ++m)
            if (!std::isfinite(ext[k].conn_w[m])) return fail(CORALAI_E_INVALID, "non-finite weight");
        for (int m = 0; m < 16; ++m)
            if (!std::isfinite(ext[k].node_in[m]) || !std::isfinite(ext[k].node_out[m]))
                return fail(CORALAI_E_INVALID, "non-finite weight");
    }
    HIP_TRY(hipMemcpyAsync(w->host.stage_slots, slot_ids, 4 * (size_t)n, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(w->host.stage_params, ext, sizeof(coralai_genome_ext) * (size_t)n, hipMemcpyHostToDevice,
                           w->stream));
    launch_scatter_ext(w->wdev, n, w->stream);
    launch_cppn(w->wdev, w->host.NL, w->host.HID, w->host.prec, 0, n, 0, 0.0f, w->ls.n_cu, w->stream);
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipMemsetAsync(&w->host.ctl->n_new, 0, sizeof(int32_t), w->stream));  // the staging area is reused
    HIP_TRY(hipStreamSynchronize(w->stream));
    return report_errors(w, nullptr);
}

int coralai_get_genome_ext(coralai_world* w, int32_t n, const int32_t* slot_ids, coralai_genome_ext* out) {
    WORLD_GUARD(w);
    if (n < 0 || (n > 0 && (!slot_ids || !out))) return fail(CORALAI_E_INVALID, "bad arguments");
    for (int k = 0; k < n; ++k) {
        if (slot_ids[k] < 0 || slot_ids[k] >= w->host.cap)
            return fail(CORALAI_E_INVALID, "slot id %d outside [0, %d)", slot_ids[k], w->host.cap);
        uint32_t* rec = (uint32_t*)(out + k);
        HIP_TRY(hipMemcpyAsync(rec, w->host.ext_mask + (size_t)slot_ids[k] * 4, 16, hipMemcpyDeviceToHost, w->stream));
        HIP_TRY(hipMemcpyAsync(rec + 4, w->host.ext_w + (size_t)slot_ids[k] * kNExtW, 4 * kNExtW,
                               hipMemcpyDeviceToHost, w->stream));
    }
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_set_structural_mutation(coralai_world* w, double p_conn, double p_node) {
    WORLD_GUARD(w);
    if (!(p_conn >= 0.0 && p_conn <= 1.0 && p_node >= 0.0 && p_node <= 1.0))
        return fail(CORALAI_E_INVALID, "probabilities must be in [0, 1]");
    auto thr = [](double p) -> uint64_t {
        if (p <= 0.0) return 0;
        if (p >= 1.0) return UINT64_MAX;
        return (uint64_t)std::floor(p * 18446744073709551616.0);
    };
    w->host.t_conn = thr(p_conn);
    w->host.t_node = thr(p_node);
    return write_world_tables(w);
}

int coralai_get_genomes(coralai_world* w, int32_t n, const int32_t* slot_ids, float* out) {
    WORLD_GUARD(w);
    if (n < 0) return fail(CORALAI_E_INVALID, "n < 0");
    for (int k = 0; k < n; ++k) {
        if (slot_ids[k] < 0 || slot_ids[k] >= w->host.cap)
            return fail(CORALAI_E_INVALID, "slot id %d outside [0, %d)", slot_ids[k], w->host.cap);
        HIP_TRY(hipMemcpyAsync(out + (size_t)k * kNParam, w->host.params + (size_t)slot_ids[k] * kNParam,
                               4 * kNParam, hipMemcpyDeviceToHost, w->stream));
    }
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_step(coralai_world* w, int32_t n_steps, coralai_stats* out) {
    WORLD_GUARD(w);
    if (n_steps < 0) return fail(CORALAI_E_INVALID, "n_steps < 0");
    const bool use_graph = w->stream != nullptr && !w->profiling;
    const int key = tuning_key(w->act_cells, w->act_waves, w->phys_tile, w->ls);
    const bool stale = w->counts_stale && n_steps > 0;  // the first step recounts
    if (use_graph && (w->graph == nullptr || w->graph_key != key)) {
        destroy_graph(&w->graph);
        int rc = capture_step(w->stream, w->bdev, w->ls, w->host.NL, w->host.HID, w->host.prec,
                              w->act_cells, w->act_waves, w->phys_tile, 0, &w->graph);
        if (rc) return rc;
        w->graph_key = key;
    }
    if (use_graph && stale && (w->graph_rc == nullptr || w->graph_rc_key != key)) {
        destroy_graph(&w->graph_rc);
        int rc = capture_step(w->stream, w->bdev, w->ls, w->host.NL, w->host.HID, w->host.prec,
                              w->act_cells, w->act_waves, w->phys_tile, 1, &w->graph_rc);
        if (rc) return rc;
        w->graph_rc_key = key;
    }
    for (int k = 0; k < n_steps; ++k) {
        const bool recount = stale && k == 0;
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(recount ? w->graph_rc : w->graph, w->stream));
        } else {
            const WorldDev& h = w->host;
            int rc = timed_phase(w, 0, [&] { launch_bucket_only(w->bdev, w->ls, w->stream, recount); });
            if (!rc) rc = timed_phase(w, 1, [&] {
                launch_act_only(w->bdev, w->ls, h.NL, h.HID, h.prec, w->act_cells, w->act_waves,
                                w->stream, nullptr);
            });
            if (!rc) rc = timed_phase(w, 2, [&] { launch_physics_only(w->bdev, w->ls, w->phys_tile, w->stream); });
            if (!rc) rc = timed_phase(w, 3, [&] { launch_finalize(w->bdev, w->ls, w->stream); });
            if (rc) return rc;
        }
    }
    if (n_steps > 0) w->counts_stale = false;
    int rc = check_launch();
    if (rc) return rc;
    if (out) {
        uint32_t word = 0;
        rc = report_errors(w, &word);
        fill_stats(*w->pinned, out);
        out->error_word = word;
        return rc;
    }
    return CORALAI_OK;
}

int coralai_radiate(coralai_world* w, double rate, float sigma, uint64_t step_index, coralai_stats* out) {
    WORLD_GUARD(w);
    if (!(rate >= 0.0 && rate <= 1.0)) return fail(CORALAI_E_INVALID, "rate must be in [0, 1]");
    if (!(sigma >= 0.0f) || !std::isfinite(sigma)) return fail(CORALAI_E_INVALID, "sigma must be finite and >= 0");
    uint64_t T;
    if (rate <= 0.0) T = 0;
    else if (rate >= 1.0) T = UINT64_MAX;
    else T = (uint64_t)std::floor(rate * 18446744073709551616.0);
    int rc = timed_phase(w, 4, [&] {
        launch_radiate(w->bdev, w->wdev, w->ls, w->host.NL, w->host.HID, w->host.prec, w->L.n_rad_blocks, T, sigma,
                       step_index, w->stream, w->counts_stale ? 1 : 0);
    });
    w->counts_stale = false;
    if (rc) return rc;
    rc = check_launch();
    if (rc) return rc;
    if (out) {
        uint32_t word = 0;
        rc = report_errors(w, &word);
        fill_stats(*w->pinned, out);
        out->error_word = word;
        return rc;
    }
    return CORALAI_OK;
}

int coralai_merge(coralai_world* w, double rate, uint64_t step_index, coralai_stats* out) {
    WORLD_GUARD(w);
    if (!(rate >= 0.0 && rate <= 1.0)) return fail(CORALAI_E_INVALID, "rate must be in [0, 1]");
    uint64_t T;
    if (rate <= 0.0) T = 0;
    else if (rate >= 1.0) T = UINT64_MAX;
    else T = (uint64_t)std::floor(rate * 18446744073709551616.0);
    int rc = timed_phase(w, 4, [&] {
        launch_merge(w->bdev, w->wdev, w->ls, w->host.NL, w->host.HID, w->host.prec, w->L.n_rad_blocks, T,
                     step_index, w->stream, w->counts_stale ? 1 : 0);
    });
    w->counts_stale = false;
    if (rc) return rc;
    rc = check_launch();
    if (rc) return rc;
    if (out) {
        uint32_t word = 0;
        rc = report_errors(w, &word);
        fill_stats(*w->pinned, out);
        out->error_word = word;
        return rc;
    }
    return CORALAI_OK;
}

int coralai_set_step_count(coralai_world* w, int64_t steps) {
    WORLD_GUARD(w);
    if (steps < 0) return fail(CORALAI_E_INVALID, "steps must be >= 0");
    HIP_TRY(hipMemcpyAsync(&w->host.ctl->steps, &steps, sizeof(int64_t), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_sync(coralai_world* w) {
    WORLD_GUARD(w);
    HIP_TRY(hipStreamSynchronize(w->stream));
    return report_errors(w, nullptr);
}

int coralai_get_stats(coralai_world* w, coralai_stats* out) {
    WORLD_GUARD(w);
    if (!out) return fail(CORALAI_E_INVALID, "out is NULL");
    uint32_t word = 0;
    int rc = report_errors(w, &word);
    fill_stats(*w->pinned, out);
    out->error_word = word;
    return rc;
}

int coralai_set_profiling(coralai_world* w, int on) {
    WORLD_GUARD(w);
    int rc = harvest_profile(w);
    if (rc) return rc;
    w->profiling = on != 0;
    for (int k = 0; k < CORALAI_PHASES; ++k) { w->prof_ms[k] = 0.0; w->prof_n[k] = 0; }
    return CORALAI_OK;
}

int coralai_get_profile(coralai_world* w, double* ms_sum, int64_t* launches) {
    WORLD_GUARD(w);
    int rc = harvest_profile(w);
    if (rc) return rc;
    for (int k = 0; k < CORALAI_PHASES; ++k) {
        if (ms_sum) ms_sum[k] = w->prof_ms[k];
        if (launches) launches[k] = w->prof_n[k];
    }
    return CORALAI_OK;
}

int coralai_set_tuning(coralai_world* w, int32_t act_cells, int32_t act_waves, int32_t phys_tile) {
    WORLD_GUARD(w);
    if (act_cells != 1 && act_cells != 2 && act_cells != 4) return fail(CORALAI_E_INVALID, "act_cells must be 1, 2 or 4");
    if (act_waves != 0 && act_waves != 1) return fail(CORALAI_E_INVALID, "act_waves must be 0 or 1");
    if (phys_tile < 0 || phys_tile > 3) return fail(CORALAI_E_INVALID, "phys_tile must be 0, 1, 2 or 3");
    w->act_cells = act_cells;
    w->act_waves = act_waves;
    w->phys_tile = phys_tile;
    return write_world_tables(w);
}

}  // extern "C"

namespace {

// Times every network-kernel variant and every physics variant on the
// current state (the kernels only write the next buffers and the record, so
// repeating them leaves the state unchanged) and returns the fastest.
template <typename SetTile>
int autotune_run(hipStream_t st, const BatchDev* bdev, const LaunchShape& ls, int NL, int HID, int prec,
                 SetTile&& set_tile, int* act_cells, int* act_waves, int* phys_tile) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto timed = [&](auto&& fn) -> float {
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, st);
            fn();
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        return best;
    };
    launch_bucket_only(bdev, ls, st);
    float best_act = 1e30f;
    for (int wv : {0, 1})
        for (int c : {1, 2, 4}) {
            float t = timed([&] { launch_act_only(bdev, ls, NL, HID, prec, c, wv, st, nullptr); });
            if (t < best_act) { best_act = t; *act_cells = c; *act_waves = wv; }
        }
    float best_phys = 1e30f;
    for (int t = 0; t < 4; ++t) {
        int rc = set_tile(t);
        if (rc) return rc;
        float ms = timed([&] { launch_physics_only(bdev, ls, t, st); });
        if (ms < best_phys) { best_phys = ms; *phys_tile = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return set_tile(*phys_tile);
}

}  // namespace

extern "C" {

int coralai_autotune(coralai_world* w, int32_t* act_cells_out, int32_t* act_waves_out,
                     int32_t* phys_tile_out) {
    WORLD_GUARD(w);
    int ac = 2, aw = 0, pt = 0;
    int rc = autotune_run(w->stream, w->bdev, w->ls, w->host.NL, w->host.HID, w->host.prec,
                          [&](int t) { w->phys_tile = t; return write_world_tables(w); }, &ac, &aw, &pt);
    if (rc) return rc;
    // the trial physics launches moved the genome counts off the state
    rc = invalidate_counts(w);
    if (rc) return rc;
    w->act_cells = ac;
    w->act_waves = aw;
    rc = check_launch();
    if (rc) return rc;
    if (act_cells_out) *act_cells_out = ac;
    if (act_waves_out) *act_waves_out = aw;
    if (phys_tile_out) *phys_tile_out = pt;
    return report_errors(w, nullptr);
}

// ------------------------------------------------------------------ batches

size_t coralai_batch_bytes(int32_t max_worlds) {
    if (max_worlds < 1 || max_worlds > (1 << 16)) return 0;
    const size_t m = (size_t)max_worlds;
    size_t off = 0;
    auto take = [&](size_t bytes) { off = align_up(off, kAlign); off += bytes; };
    take(sizeof(BatchDev));
    take(sizeof(WorldDev) * m);
    take(8 * (m + 1));
    take(8 * (m + 1));
    take(8 * (m + 1));
    take(4 * (m + 1));
    take(4 * m);
    return align_up(off, kAlign) + kAlign;
}

int coralai_batch_create(int32_t max_worlds, void* dev_arena, size_t arena_bytes, void* hip_stream,
                         coralai_batch** out) {
    if (!out) return fail(CORALAI_E_INVALID, "out is NULL");
    *out = nullptr;
    const size_t need = coralai_batch_bytes(max_worlds);
    if (!need) return fail(CORALAI_E_INVALID, "max_worlds must be in [1, 65536]");
    if (!dev_arena) return fail(CORALAI_E_INVALID, "dev_arena is NULL");
    if (arena_bytes < need) return fail(CORALAI_E_NOMEM, "batch arena of %zu bytes < %zu", arena_bytes, need);
    coralai_batch* b = new coralai_batch();
    b->max_worlds = max_worlds;
    b->stream = (hipStream_t)hip_stream;
    b->base = (uint8_t*)align_up((uintptr_t)dev_arena, kAlign);
    const size_t m = (size_t)max_worlds;
    size_t off = 0;
    auto take = [&](size_t bytes) { off = align_up(off, kAlign); size_t o = off; off += bytes; return b->base + o; };
    b->bdev = (BatchDev*)take(sizeof(BatchDev));
    b->table = (WorldDev*)take(sizeof(WorldDev) * m);
    b->chunk_prefix = (int64_t*)take(8 * (m + 1));
    b->slot_prefix = (int64_t*)take(8 * (m + 1));
    b->tile_prefix = (int64_t*)take(8 * (m + 1));
    b->group_prefix = (int32_t*)take(4 * (m + 1));
    b->tiles_x = (int32_t*)take(4 * m);
    b->ls = make_shape(max_worlds, 1 << 10);  // kernels stride over larger capacities
    BatchDev hb{};
    hb.n_worlds = 0;
    hb.worlds = b->table;
    hb.chunk_prefix = b->chunk_prefix;
    hb.slot_prefix = b->slot_prefix;
    hb.tile_prefix = b->tile_prefix;
    hb.group_prefix = b->group_prefix;
    hb.tiles_x = b->tiles_x;
    if (hipEventCreateWithFlags(&b->ev_order, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(CORALAI_E_HIP, "event creation failed");
    }
    if (hipMemcpyAsync(b->bdev, &hb, sizeof hb, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        (void)hipEventDestroy(b->ev_order);
        delete b;
        return fail(CORALAI_E_HIP, "batch table upload failed");
    }
    *out = b;
    return CORALAI_OK;
}

}  // extern "C"
namespace {
int batch_upload(coralai_batch* b, coralai_world* const* worlds, int32_t n);
}
extern "C" {

int coralai_batch_set_worlds(coralai_batch* b, coralai_world* const* worlds, int32_t n) {
    if (!b) return fail(CORALAI_E_INVALID, "batch is NULL");
    BusyGuard guard_(&b->busy);
    if (!guard_.ok) return fail(CORALAI_E_BUSY, "batch is in use");
    return batch_upload(b, worlds, n);
}

int coralai_batch_autotune(coralai_batch* b, int32_t* act_cells_out, int32_t* act_waves_out,
                           int32_t* phys_tile_out) {
    if (!b) return fail(CORALAI_E_INVALID, "batch is NULL");
    BusyGuard guard_(&b->busy);
    if (!guard_.ok) return fail(CORALAI_E_BUSY, "batch is in use");
    if (b->n == 0) return fail(CORALAI_E_INVALID, "the batch has no worlds");
    std::vector<coralai_world*> ws = b->worlds;
    int ac = 2, aw = 0, pt = 0;
    int rc = autotune_run(b->stream, b->bdev, b->ls, b->NL, b->HID, b->prec,
                          [&](int t) { b->phys_tile = t; return batch_upload(b, ws.data(), (int)ws.size()); },
                          &ac, &aw, &pt);
    if (rc) return rc;
    // the trial physics launches moved the worlds' genome counts off their states
    for (coralai_world* w : ws) {
        w->counts_stale = true;
        HIP_TRY(hipMemsetAsync(&w->host.ctl->counts_valid, 0, sizeof(int32_t), b->stream));
    }
    b->act_cells = ac;
    b->act_waves = aw;
    if (act_cells_out) *act_cells_out = ac;
    if (act_waves_out) *act_waves_out = aw;
    if (phys_tile_out) *phys_tile_out = pt;
    return check_launch();
}

int coralai_batch_set_tuning(coralai_batch* b, int32_t act_cells, int32_t act_waves, int32_t phys_tile) {
    if (!b) return fail(CORALAI_E_INVALID, "batch is NULL");
    BusyGuard guard_(&b->busy);
    if (!guard_.ok) return fail(CORALAI_E_BUSY, "batch is in use");
    if (act_cells != 1 && act_cells != 2 && act_cells != 4) return fail(CORALAI_E_INVALID, "act_cells must be 1, 2 or 4");
    if (act_waves != 0 && act_waves != 1) return fail(CORALAI_E_INVALID, "act_waves must be 0 or 1");
    if (phys_tile < 0 || phys_tile > 3) return fail(CORALAI_E_INVALID, "phys_tile must be 0, 1, 2 or 3");
    b->act_cells = act_cells;
    b->act_waves = act_waves;
    b->phys_tile = phys_tile;
    std::vector<coralai_world*> ws = b->worlds;
    return batch_upload(b, ws.data(), (int)ws.size());
}

}  // extern "C"
namespace {
int batch_upload(coralai_batch* b, coralai_world* const* worlds, int32_t n) {
    if (n < 0 || n > b->max_worlds) return fail(CORALAI_E_INVALID, "n must be in [0, max_worlds]");
    if (n > 0 && !worlds) return fail(CORALAI_E_INVALID, "worlds is NULL");
    std::vector<WorldDev> tab(n);
    std::vector<int64_t> cp(n + 1, 0), tp(n + 1, 0), sp(n + 1, 0);
    std::vector<int32_t> tx(std::max(n, 1), 0);
    int variants = 0, max_slot_blocks = 0;
    for (int k = 0; k < n; ++k) {
        coralai_world* w = worlds[k];
        if (!w) return fail(CORALAI_E_INVALID, "world %d is NULL", k);
        variants |= w->ls.act_variants;
        max_slot_blocks = std::max(max_slot_blocks, w->host.n_slot_blocks);
        if (k == 0) { b->NL = w->host.NL; b->HID = w->host.HID; b->prec = w->host.prec; }
        if (w->host.NL != b->NL || w->host.HID != b->HID || w->host.prec != b->prec)
            return fail(CORALAI_E_INVALID, "world %d: a batch needs one network shape and precision", k);
        tab[k] = w->host;
        cp[k + 1] = cp[k] + (w->host.btiles + kBucketGroup - 1) / kBucketGroup;
        sp[k + 1] = sp[k] + w->host.n_slot_blocks;
        int t = 0;
        tp[k + 1] = tp[k] + tiles_for(w->host.W, w->host.H, b->phys_tile, &t);
        tx[k] = t;
    }
    // work already queued on a world's own stream (state upload, genomes)
    // completes before the batch's next step touches the world
    for (int k = 0; k < n; ++k) {
        if (worlds[k]->stream == b->stream) continue;
        HIP_TRY(hipEventRecord(b->ev_order, worlds[k]->stream));
        HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_order, 0));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (n > 0) {
        HIP_TRY(hipMemcpyAsync(b->table, tab.data(), sizeof(WorldDev) * n, hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->tiles_x, tx.data(), 4 * (size_t)n, hipMemcpyHostToDevice, b->stream));
    }
    HIP_TRY(hipMemcpyAsync(b->chunk_prefix, cp.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->slot_prefix, sp.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->tile_prefix, tp.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(&b->bdev->n_worlds, &n, sizeof n, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->n = n;
    b->worlds.assign(worlds, worlds + n);
    b->ls.act_variants = variants;  // part of the graph key: the step is recaptured when it changes
    b->ls.scan_fused = max_slot_blocks <= kFuseSlotBlocks ? 1 : 0;  // likewise
    return CORALAI_OK;
}
}  // namespace
extern "C" {

int coralai_batch_step(coralai_batch* b, int32_t n_steps) {
    if (!b) return fail(CORALAI_E_INVALID, "batch is NULL");
    BusyGuard guard_(&b->busy);
    if (!guard_.ok) return fail(CORALAI_E_BUSY, "batch is in use");
    if (n_steps < 0) return fail(CORALAI_E_INVALID, "n_steps < 0");
    if (b->n == 0 || n_steps == 0) return CORALAI_OK;
    const bool use_graph = b->stream != nullptr;
    const int key = tuning_key(b->act_cells, b->act_waves, b->phys_tile, b->ls);
    bool stale = false;  // some world's counts are stale: the first step recounts
    for (coralai_world* w : b->worlds) stale = stale || w->counts_stale;
    if (use_graph && (b->graph == nullptr || b->graph_key != key)) {
        destroy_graph(&b->graph);
        int rc = capture_step(b->stream, b->bdev, b->ls, b->NL, b->HID, b->prec, b->act_cells,
                              b->act_waves, b->phys_tile, 0, &b->graph);
        if (rc) return rc;
        b->graph_key = key;
    }
    if (use_graph && stale && (b->graph_rc == nullptr || b->graph_rc_key != key)) {
        destroy_graph(&b->graph_rc);
        int rc = capture_step(b->stream, b->bdev, b->ls, b->NL, b->HID, b->prec, b->act_cells,
                              b->act_waves, b->phys_tile, 1, &b->graph_rc);
        if (rc) return rc;
        b->graph_rc_key = key;
    }
    for (int k = 0; k < n_steps; ++k) {
        const bool recount = stale && k == 0;
        if (use_graph) HIP_TRY(hipGraphLaunch(recount ? b->graph_rc : b->graph, b->stream));
        else launch_step_kernels(b->bdev, b->ls, b->NL, b->HID, b->prec, b->act_cells, b->act_waves,
                                 b->phys_tile, b->stream, nullptr, recount ? 1 : 0);
    }
    for (coralai_world* w : b->worlds) w->counts_stale = false;
    int rc = check_launch();
    if (rc) return rc;
    // later calls on a world's own stream (get_state, step, ...) wait for these steps
    bool other = false;
    for (coralai_world* w : b->worlds) other = other || w->stream != b->stream;
    if (other) {
        HIP_TRY(hipEventRecord(b->ev_order, b->stream));
        for (coralai_world* w : b->worlds)
            if (w->stream != b->stream) HIP_TRY(hipStreamWaitEvent(w->stream, b->ev_order, 0));
    }
    return CORALAI_OK;
}

int coralai_batch_sync(coralai_batch* b) {
    if (!b) return fail(CORALAI_E_INVALID, "batch is NULL");
    HIP_TRY(hipStreamSynchronize(b->stream));
    return CORALAI_OK;
}

int coralai_batch_destroy(coralai_batch* b) {
    if (!b) return fail(CORALAI_E_INVALID, "batch is NULL");
    (void)hipStreamSynchronize(b->stream);
    destroy_graph(&b->graph);
    destroy_graph(&b->graph_rc);
    if (b->ev_order) (void)hipEventDestroy(b->ev_order);
    delete b;
    return CORALAI_OK;
}

// ------------------------------------------------------------------ parity hooks

int coralai_debug_buckets(coralai_world* w, int32_t* counts, int32_t* offsets, int32_t* perm) {
    WORLD_GUARD(w);
    {
        const int irc = invalidate_counts(w);
        if (irc) return irc;
    }
    launch_bucket_only(w->bdev, w->ls, w->stream);
    int rc = check_launch();
    if (rc) return rc;
    const size_t cap = (size_t)w->host.cap, N = (size_t)w->host.N;
    if (counts) HIP_TRY(hipMemcpyAsync(counts, w->host.counts, 4 * cap, hipMemcpyDeviceToHost, w->stream));
    if (offsets) HIP_TRY(hipMemcpyAsync(offsets, w->host.offsets, 4 * (cap + 1), hipMemcpyDeviceToHost, w->stream));
    if (perm) HIP_TRY(hipMemcpyAsync(perm, w->host.perm, 4 * N, hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (perm)  // drop the rotation bits the network kernel reads with each index
        for (size_t k = 0; k < N; ++k) perm[k] &= kPermIndexMask;
    return report_errors(w, nullptr);
}

int coralai_debug_actuators(coralai_world* w, float* act) {
    WORLD_GUARD(w);
    {
        const int irc = invalidate_counts(w);
        if (irc) return irc;
    }
    if (!act) return fail(CORALAI_E_INVALID, "act is NULL");
    const size_t N = (size_t)w->host.N;
    float* d = nullptr;
    HIP_TRY(hipMalloc((void**)&d, 4 * kNOut * N));
    launch_bucket_only(w->bdev, w->ls, w->stream);
    launch_act_only(w->bdev, w->ls, w->host.NL, w->host.HID, w->host.prec, w->act_cells, w->act_waves,
                    w->stream, d);
    int rc = check_launch();
    if (!rc && hipMemcpyAsync(act, d, 4 * kNOut * N, hipMemcpyDeviceToHost, w->stream) != hipSuccess)
        rc = fail(CORALAI_E_HIP, "actuator copy failed");
    if (!rc && hipStreamSynchronize(w->stream) != hipSuccess) rc = fail(CORALAI_E_HIP, "sync failed");
    (void)hipFree(d);
    if (rc) return rc;
    return report_errors(w, nullptr);
}

int coralai_debug_set_weights(coralai_world* w, int32_t slot, const float* flat) {
    WORLD_GUARD(w);
    if (slot < 0 || slot >= w->host.cap || !flat) return fail(CORALAI_E_INVALID, "bad slot or NULL weights");
    const size_t n = (size_t)net_flat_size(w->host.NL, w->host.HID);
    float* d = nullptr;
    HIP_TRY(hipMalloc((void**)&d, 4 * n));
    int rc = CORALAI_OK;
    if (hipMemcpyAsync(d, flat, 4 * n, hipMemcpyHostToDevice, w->stream) != hipSuccess) rc = fail(CORALAI_E_HIP, "copy failed");
    if (!rc) {
        launch_pack_weights(w->wdev, slot, d, 0, nullptr, w->stream);
        rc = check_launch();
    }
    if (!rc && hipStreamSynchronize(w->stream) != hipSuccess) rc = fail(CORALAI_E_HIP, "sync failed");
    (void)hipFree(d);
    return rc;
}

int coralai_debug_get_weights(coralai_world* w, int32_t slot, float* flat) {
    WORLD_GUARD(w);
    if (slot < 0 || slot >= w->host.cap || !flat) return fail(CORALAI_E_INVALID, "bad slot or NULL output");
    const size_t n = (size_t)net_flat_size(w->host.NL, w->host.HID);
    float* d = nullptr;
    HIP_TRY(hipMalloc((void**)&d, 4 * n));
    launch_pack_weights(w->wdev, slot, nullptr, 1, d, w->stream);
    int rc = check_launch();
    if (!rc && hipMemcpyAsync(flat, d, 4 * n, hipMemcpyDeviceToHost, w->stream) != hipSuccess) rc = fail(CORALAI_E_HIP, "copy failed");
    if (!rc && hipStreamSynchronize(w->stream) != hipSuccess) rc = fail(CORALAI_E_HIP, "sync failed");
    (void)hipFree(d);
    return rc;
}

}  // extern "C"

namespace {

// Staging buffer of coralai_debug_set_weights_noalloc, one copy per device,
// held until the process ends.  In host code the array's name is only a
// host-side stand-in: kernels get the device address that
// hipGetSymbolAddress returns for the device (noalloc_scratch), never the
// name.  Every call on a device shares that device's copy.
constexpr int kNoAllocScratchFloats = 16384;  // 64 KiB; the largest network (54-64-64-14) has 8590 floats
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];

// The device address of this device's scratch, looked up once per device
// with that device current.
int noalloc_scratch(int device, float** out) {
    static std::mutex mu;
    static std::unordered_map<int, float*> ptrs;
    std::lock_guard<std::mutex> lock(mu);
    auto it = ptrs.find(device);
    if (it != ptrs.end()) {
        *out = it->second;
        return CORALAI_OK;
    }
    int prev = -1;
    HIP_TRY(hipGetDevice(&prev));
    if (prev != device) HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || p == nullptr)
        return fail(CORALAI_E_HIP, "hipGetSymbolAddress of the staging buffer failed on device %d: %s", device,
                    hipGetErrorString(e));
    ptrs[device] = (float*)p;
    *out = (float*)p;
    return CORALAI_OK;
}

}  // namespace

extern "C" {

int coralai_debug_set_weights_noalloc(coralai_world* w, int32_t slot, const float* flat) {
    WORLD_GUARD(w);
    if (slot < 0 || slot >= w->host.cap || !flat) return fail(CORALAI_E_INVALID, "bad slot or NULL weights");
    const size_t n = (size_t)net_flat_size(w->host.NL, w->host.HID);
    if (n > (size_t)kNoAllocScratchFloats)
        return fail(CORALAI_E_INVALID, "a network of %zu floats exceeds the %d-float staging buffer", n,
                    kNoAllocScratchFloats);
    float* d = nullptr;
    int rc = noalloc_scratch(w->device, &d);
    if (rc) return rc;
    // every one of the n staged floats is written before the kernel reads it
    HIP_TRY(hipMemcpyAsync(d, flat, 4 * n, hipMemcpyHostToDevice, w->stream));
    launch_pack_weights(w->wdev, slot, d, 0, nullptr, w->stream);
    rc = check_launch();
    if (rc) return rc;
    // the next call on this device may overwrite the staging buffer
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_set_daylight(coralai_world* w, int32_t period, int64_t inject_quanta, int32_t remove_num) {
    WORLD_GUARD(w);
    if (period != 0 && period < 2) return fail(CORALAI_E_INVALID, "period must be 0 (no cycle) or >= 2 steps");
    if (inject_quanta < 0 || inject_quanta >= (1ll << 40)) return fail(CORALAI_E_INVALID, "inject_quanta must be in [0, 2^40)");
    if (remove_num < 0 || remove_num > 65536) return fail(CORALAI_E_INVALID, "remove_num must be in [0, 65536]");
    (void)hipStreamSynchronize(w->stream);
    w->host.day_period = period;
    w->host.day_inject = period ? inject_quanta : 0;
    w->host.night_num = period ? remove_num : 0;
    return write_world_tables(w);
}

int coralai_set_physics_variant(coralai_world* w, int32_t explore_mode, float kappa_energy) {
    WORLD_GUARD(w);
    if (explore_mode != 0 && explore_mode != 1) return fail(CORALAI_E_INVALID, "explore_mode must be 0 or 1");
    if (!(kappa_energy >= 0.0f && kappa_energy <= 1.0f)) return fail(CORALAI_E_INVALID, "kappa_energy must be in [0, 1]");
    if (kappa_energy > 0.0f && w->host.eflow == nullptr)
        return fail(CORALAI_E_INVALID, "energy transport needs a world created with CORALAI_WORLD_ENERGY_FLOWS");
    (void)hipStreamSynchronize(w->stream);
    w->host.explore_mode = explore_mode;
    w->host.kappa_e = kappa_energy;
    // the network kernel with the variants' code runs only while one is on,
    // the physics kernel that loads the energy records only with transport
    w->ls.act_variants = ((explore_mode != 0 || kappa_energy > 0.0f) ? 1 : 0) | (kappa_energy > 0.0f ? 2 : 0);
    return write_world_tables(w);
}

int coralai_get_energy_ledger(coralai_world* w, int64_t* injected_last, int64_t* removed_last,
                              int64_t* injected_total, int64_t* removed_total) {
    WORLD_GUARD(w);
    const int rc = read_ctl(w);
    if (rc) return rc;
    const Ctl& c = *w->pinned;
    if (injected_last) *injected_last = c.injected_pub;
    if (removed_last) *removed_last = c.removed_pub;
    if (injected_total) *injected_total = c.injected_total;
    if (removed_total) *removed_total = c.removed_total;
    return CORALAI_OK;
}

int coralai_get_lineage(coralai_world* w, int32_t n, const int32_t* slot_ids, int32_t* parents,
                        int32_t* parents2, int64_t* birth_steps) {
    WORLD_GUARD(w);
    if (n < 0 || (n > 0 && !slot_ids)) return fail(CORALAI_E_INVALID, "bad slot list");
    for (int k = 0; k < n; ++k) {
        if (slot_ids[k] < 0 || slot_ids[k] >= w->host.cap)
            return fail(CORALAI_E_INVALID, "slot id %d outside [0, %d)", slot_ids[k], w->host.cap);
        if (parents)
            HIP_TRY(hipMemcpyAsync(parents + k, w->host.lineage_parent + slot_ids[k], 4, hipMemcpyDeviceToHost, w->stream));
        if (parents2)
            HIP_TRY(hipMemcpyAsync(parents2 + k, w->host.lineage_parent2 + slot_ids[k], 4, hipMemcpyDeviceToHost, w->stream));
        if (birth_steps)
            HIP_TRY(hipMemcpyAsync(birth_steps + k, w->host.lineage_birth + slot_ids[k], 8, hipMemcpyDeviceToHost, w->stream));
    }
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_get_births(coralai_world* w, int32_t max_births, int32_t* cells, int32_t* parents, int32_t* parents2,
                       int32_t* slots, int32_t* n_births) {
    WORLD_GUARD(w);
    if (max_births < 0 || !n_births) return fail(CORALAI_E_INVALID, "bad arguments");
    int rc = read_ctl(w);
    if (rc) return rc;
    const int n = std::min(max_births, std::max(0, w->pinned->n_new));
    *n_births = std::max(0, w->pinned->n_new);
    if (n > 0) {
        if (cells) HIP_TRY(hipMemcpyAsync(cells, w->host.stage_slots, 4 * (size_t)n, hipMemcpyDeviceToHost, w->stream));
        if (parents) HIP_TRY(hipMemcpyAsync(parents, w->host.stage_params, 4 * (size_t)n, hipMemcpyDeviceToHost, w->stream));
        if (parents2)
            HIP_TRY(hipMemcpyAsync(parents2, (const int32_t*)w->host.stage_params + w->host.cap, 4 * (size_t)n,
                                   hipMemcpyDeviceToHost, w->stream));
        if (slots) HIP_TRY(hipMemcpyAsync(slots, w->host.new_slots, 4 * (size_t)n, hipMemcpyDeviceToHost, w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
    }
    return CORALAI_OK;
}

int coralai_genetic_distance(coralai_world* w, int32_t na, const int32_t* slots_a, int32_t nb,
                             const int32_t* slots_b, float c1, float c2, float c3, float* out_device) {
    WORLD_GUARD(w);
    if (na < 0 || nb < 0 || (na > 0 && !slots_a) || (nb > 0 && !slots_b)) return fail(CORALAI_E_INVALID, "bad slot lists");
    if ((int64_t)na + nb > (int64_t)(kNParam - 2) * w->host.cap)
        return fail(CORALAI_E_INVALID, "na + nb must be <= 54 x the genome capacity");
    if (na == 0 || nb == 0) return CORALAI_OK;
    if (!out_device) return fail(CORALAI_E_INVALID, "out_device is NULL");
    for (int k = 0; k < na + nb; ++k) {
        const int sl = k < na ? slots_a[k] : slots_b[k - na];
        if (sl < 0 || sl >= w->host.cap) return fail(CORALAI_E_INVALID, "slot id %d outside [0, %d)", sl, w->host.cap);
    }
    // the slot lists go through the parameter staging area of set_genomes
    // (56 x capacity words, free between calls) past its first 2 x capacity
    // words, which hold the last radiation or merging call's births
    int32_t* staged = (int32_t*)w->host.stage_params + 2 * (int64_t)w->host.cap;
    HIP_TRY(hipMemcpyAsync(staged, slots_a, 4 * (size_t)na, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(staged + na, slots_b, 4 * (size_t)nb, hipMemcpyHostToDevice, w->stream));
    launch_genetic_distance(w->wdev, staged, na, nb, c1, c2, c3, out_device, w->ls.n_cu, w->stream);
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

int coralai_debug_set_act_segments(coralai_world* w, int32_t n_segments) {
    WORLD_GUARD(w);
    if (n_segments < 0 || n_segments > 64) return fail(CORALAI_E_INVALID, "n_segments must be in [0, 64]");
    (void)hipStreamSynchronize(w->stream);
    w->ls.act_segments = n_segments;
    destroy_graph(&w->graph);  // recaptured with the new launch argument at the next step
    destroy_graph(&w->graph_rc);
    return CORALAI_OK;
}

int coralai_debug_physics(coralai_world* w, const int64_t* i1, const uint32_t* flows8, const uint8_t* explore_dir) {
    WORLD_GUARD(w);
    {
        const int irc = invalidate_counts(w);
        if (irc) return irc;
    }
    if (!i1 || !flows8 || !explore_dir) return fail(CORALAI_E_INVALID, "a record array is NULL");
    if (w->host.kappa_e > 0.0f) return fail(CORALAI_E_INVALID, "debug_physics takes infrastructure flows only (energy transport is on)");
    int cur = 0, rc = current_buffer(w, &cur);
    if (rc) return rc;
    const size_t N = (size_t)w->host.N;
    // the record as the act kernel writes it: per cell, 8 flow words
    // (amount << 1 | explored) in direction order
    std::vector<uint32_t> words(8 * N);
    for (size_t i = 0; i < N; ++i) {
        uint64_t tot = 0;
        for (int k = 0; k < 8; ++k) {
            const uint32_t f = flows8[i * 8 + k];
            if (f > 0x7fffffffu) return fail(CORALAI_E_INVALID, "flow amounts must be < 2^31");
            words[i * 8 + k] = (f << 1) | (uint32_t)((explore_dir[i] & 7) == k);
            tot += f;
        }
        if (tot > 0xffffffffull) return fail(CORALAI_E_INVALID, "a cell's outflow must be < 2^32");
    }
    const int nxt = cur ^ 1;
    HIP_TRY(hipMemcpyAsync(w->host.flow, words.data(), 4 * 8 * N, hipMemcpyHostToDevice, w->stream));
    // boundary ledger pairs: the current energy (no conversion) and the given I1,
    // staged through the next state's ledger, which physics overwrites
    HIP_TRY(hipMemcpyAsync(w->host.EI[nxt], i1, 8 * N, hipMemcpyHostToDevice, w->stream));
    launch_ledger_pack(w->host.EI[cur], 2, w->host.EI[nxt], 1, w->host.EI1, (int64_t)N, w->stream);
    HIP_TRY(hipMemcpyAsync(w->host.C[nxt], w->host.C[cur], 16 * N, hipMemcpyDeviceToDevice, w->stream));
    launch_physics_only(w->bdev, w->ls, w->phys_tile, w->stream);
    launch_flip(w->bdev, w->stream);
    rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CORALAI_OK;
}

}  // extern "C"
