/*
 * coralai.h -- C ABI of the MI355X (gfx950) per-step ecosystem update of
 * Coralai (Barbieux & Canaan, "Coralai: Intrinsic Evolution of Embodied
 * Neural Cellular Automata Ecosystems", ALIFE 2024).
 *
 * The operation (System Design): every cell of a W x H substrate gathers the
 * Kernel neighbourhood of its Sensor channels, runs the dense network that
 * its integer GenomeIndex selects -- weights and biases generated per genome
 * by a CPPN, HyperNEAT style -- and the Physics turns the Actuator outputs
 * into substrate change (Experiment: invest / liquidate, sigmoid
 * communication, exploration with takeover).  Radiation mutates CPPN genomes
 * and regenerates their weights (Fig. 1, panel C).
 *
 * Substrate representation (row-major, cell index i = y*W + x, y pointing
 * down, periodic in both axes):
 *   E, I   int64  mass ledger in quanta of 2^-24 mass units (energy,
 *                 infrastructure); sum(E+I) is conserved exactly by a step;
 *   C      float  4 communication planes, plane c at offset c*W*H;
 *   G      int32  GenomeIndex, a slot id in [0, genome_capacity);
 *   R      uint8  Rotation in 0..7 (multiples of 45 degrees counter-clockwise
 *                 from +x).
 * CPPN parameters: 56 floats per genome, A (8x5 row-major) then B (2x8).
 *
 * Conventions for every entry point:
 *   - returns CORALAI_OK (0) or a negative CORALAI_E_* code; the message of
 *     the last failure on the calling thread is coralai_last_error();
 *   - host pointers are borrowed for the duration of the call only;
 *   - device pointers are HIP device addresses on the world's device;
 *   - work is enqueued on the stream given at creation; a call that returns
 *     data to the host (stats, get_*) waits for that stream;
 *   - a world is used by one thread at a time; a concurrent call on the same
 *     world returns CORALAI_E_BUSY;
 *   - device-side faults in the data (genome id out of range or naming a
 *     slot with no parameters, ledger overflow, non-finite network output)
 *     set bits of an error word that the next call returning stats reports
 *     as CORALAI_E_GENOME / CORALAI_E_NUMERIC (and then clears).
 */
#ifndef CORALAI_H
#define CORALAI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct coralai_world coralai_world; /* opaque; owns no device memory */
typedef struct coralai_batch coralai_batch; /* opaque; owns no device memory */

enum { CORALAI_FP32 = 0, CORALAI_BF16 = 1 };

enum {
    CORALAI_OK = 0,
    CORALAI_E_INVALID = -1, /* bad argument; nothing was enqueued */
    CORALAI_E_NOMEM = -2,   /* arena smaller than coralai_world_bytes() */
    CORALAI_E_GENOME = -3,  /* a cell named an out-of-range or unset genome slot */
    CORALAI_E_NUMERIC = -4, /* non-finite network output or ledger overflow */
    CORALAI_E_HIP = -5,     /* a HIP runtime call failed */
    CORALAI_E_BUSY = -6     /* the world is in use by another thread */
};

/* Bits of coralai_stats.error_word. */
enum {
    CORALAI_ERR_GENOME_RANGE = 1u,
    CORALAI_ERR_GENOME_UNSET = 2u,
    CORALAI_ERR_LEDGER = 4u,    /* negative stock or a flow budget >= 2^31 quanta */
    CORALAI_ERR_NONFINITE = 8u, /* network output or CPPN weight not finite */
    CORALAI_ERR_MASS = 16u      /* a step changed the total mass by other than the
                                   day / night cycle's injected minus removed quanta */
};

/* World description.  The physics constants are the recorded readings of
 * the Experiment section (which names the actuators but not their rates):
 * invest / liquidate move floor(rho * sigmoid(a) * stock) quanta, the
 * exploration budget is floor(kappa * I1) quanta. */
typedef struct {
    int32_t width, height;    /* >= 1 each; W*H <= 2^26 (8192 x 8192) */
    int32_t n_weight_layers;  /* 2: 54-h-14, 3: 54-h-h-14 */
    int32_t hidden;           /* 32 or 64 */
    int32_t genome_capacity;  /* slot ids in [0, capacity), 1 .. 2^22 */
    int32_t precision;        /* CORALAI_FP32 or CORALAI_BF16 (network GEMMs only) */
    uint64_t seed;            /* Philox key word 0 for radiation */
    float rho_invest;         /* default 0.1 */
    float rho_liquidate;      /* default 0.1 */
    float kappa_flow;         /* default 0.25 */
    int32_t flags;            /* CORALAI_WORLD_* bits, 0 by default */
} coralai_world_desc;

/* coralai_world_desc.flags: reserve the 32-byte-per-cell energy flow records
 * that energy transport (coralai_set_physics_variant) needs. */
enum { CORALAI_WORLD_ENERGY_FLOWS = 1 };

/* Per-world statistics, as of the last completed step or radiation call. */
typedef struct {
    int64_t mass_quanta;     /* exact sum(E+I) after the last step */
    double mass_fp64;        /* the same sum reduced in FP64 on the GPU */
    int64_t steps;           /* steps completed since creation */
    int32_t live_genomes;    /* distinct genomes in the state the last step read */
    int32_t takeovers;       /* cells that changed genome in the last step */
    int32_t hits;            /* radiation hits in the last radiate call */
    int32_t dropped_hits;    /* hits that found no free slot */
    uint32_t error_word;     /* CORALAI_ERR_* bits since the last report */
    int32_t reserved;
} coralai_stats;

/* HBM bytes a world of this description needs (0 if the description is
 * invalid).  Used for admission by footprint. */
size_t coralai_world_bytes(const coralai_world_desc* desc);

/* Create a world inside a caller-owned device arena of at least
 * coralai_world_bytes(desc) bytes (any alignment is accepted; the library
 * aligns internally).  hip_stream is a hipStream_t (NULL = default stream).
 * The state is zeroed, no genome slot is set.  The arena must outlive the
 * world; destroy frees only the host handle. */
int coralai_world_create(const coralai_world_desc* desc, void* dev_arena, size_t arena_bytes,
                         void* hip_stream, coralai_world** out);
int coralai_world_destroy(coralai_world* w);

/* Copy a whole state in (set) or out (get).  Arrays as described above, each
 * of W*H elements (comm4: 4*W*H).  on_device = 1: the pointers are device
 * addresses (copied device-to-device); 0: host memory.  Rotation values are
 * taken mod 8; genome ids are checked at the next step. */
int coralai_set_state(coralai_world* w, const int64_t* e_q, const int64_t* i_q, const float* comm4,
                      const int32_t* genome, const uint8_t* rotation, int on_device);
int coralai_get_state(coralai_world* w, int64_t* e_q, int64_t* i_q, float* comm4,
                      int32_t* genome, uint8_t* rotation, int on_device);

/* HyperNEAT (System Design): store n genomes' CPPN parameters (host, n x 56
 * floats) in slots slot_ids[0..n) and generate each one's dense network on
 * the GPU: W_l[o][j] = CPPN_w(x_{l,j}, y_l, x_{l+1,o}, y_{l+1}) / sqrt(L_l),
 * b_l[o] = CPPN_b(0, y_l, x_{l+1,o}, y_{l+1}), neuron j of layer l at
 * x = -1 + 2j/(L_l - 1), y_l = -1 + 2l/n_weight_layers.  Marks the slots set.
 * Returns after the weights are generated. */
int coralai_set_genomes(coralai_world* w, int32_t n, const int32_t* slot_ids,
                        const float* cppn_params);
int coralai_get_genomes(coralai_world* w, int32_t n, const int32_t* slot_ids,
                        float* cppn_params_out);

/* NEAT's structural genes (System Design: Coralai applies NEAT's mutation
 * and crossover operators), over a bounded superset of the CPPN above.
 * Innovation numbers are positions: the 56 base genes are 0..55; the
 * direct connection input m -> output o (m over x1, y1, x2, y2, 1; o = 0
 * weight, 1 bias) is gene 56 + 5 o + m, enabled by bit 5 o + m of
 * conn_mask, weight conn_w[5 o + m]; the added node N_k, k = 2 j + o, which
 * splits the connection hidden j -> output o (NEAT's add-node), has its in
 * connection (weight node_in[k], gene 66 + 2 k) and out connection (weight
 * node_out[k], gene 67 + 2 k), is enabled by bit k of node_mask and applies
 * activation bits 2k..2k+1 of node_act (0 sin, 1 gauss, 2 tanh, 3 identity);
 * while N_k is enabled it replaces B[o][j].  CPPN output o is then
 *   sum over j of (N_{2j+o} ? node_out phi(node_in h_j) : B[o][j] h_j)
 *   + sum over enabled direct connections of conn_w z_m.
 * coralai_set_genomes gives a slot no structural genes.
 * coralai_set_genome_ext replaces n slots' structural genes (host records;
 * 10 and 16 mask bits, finite weights) and regenerates their networks;
 * coralai_get_genome_ext reads them back.  Both wait for the stream. */
typedef struct {
    uint32_t conn_mask, node_mask, node_act, reserved;
    float conn_w[10];
    float node_in[16];
    float node_out[16];
} coralai_genome_ext;
int coralai_set_genome_ext(coralai_world* w, int32_t n, const int32_t* slot_ids, const coralai_genome_ext* ext);
int coralai_get_genome_ext(coralai_world* w, int32_t n, const int32_t* slot_ids, coralai_genome_ext* out);

/* Structural mutation in radiation (NEAT's add-connection and add-node).
 * Every hit's child also carries its parent's structural genes; the
 * weights of the enabled ones get sigma * N(0,1) like the base genes (weight
 * m, in the order conn_w, node_in, node_out, from Box-Muller on the Philox
 * block (i, step_index, 16 + m / 4, 0)), disabled ones keep theirs.  Then
 * the block (i, step_index, 15, 0): word 0 below floor(p_conn 2^64) adds
 * direct connection c = (word 2 & 0xffff) mod 10 with weight sigma times
 * its normal; word 1 below floor(p_node 2^64)
 * adds node k = ((word 2 >> 16) & 0xffff) mod 16 with activation word 3 & 3,
 * in weight 1 and out weight the child's B[o][j].  Adding a gene already
 * present changes nothing.  Both 0 by default.  p in [0, 1]. */
int coralai_set_structural_mutation(coralai_world* w, double p_conn, double p_node);

/* n_steps updates (System Design; Fig. 1 A and B): bucket cells by genome,
 * sense the rotation-ordered 3x3 Moore kernel, run the genome's network,
 * apply invest / liquidate / communication / exploration, then the
 * exploration-and-takeover physics, and reduce the total mass.  Asynchronous
 * when out is NULL; otherwise waits and fills *out. */
int coralai_step(coralai_world* w, int32_t n_steps, coralai_stats* out);

/* Radiation after step step_index (Fig. 1 C): cell i is hit when word i mod 4
 * of Philox4x64-10(counter (floor(i / 4), step_index, 0, 0), key (seed, 0))
 * is below floor(rate * 2^64); the k-th hit in ascending i takes the k-th free
 * slot (ascending slot ids whose genome count is zero), whose CPPN
 * parameters become the parent's plus sigma * N(0,1) (Box-Muller on Philox
 * blocks (i, step_index, 1+b, 0), b = 0..13) and whose network is
 * regenerated; G[i] becomes that slot.  Hits beyond the free slots are
 * dropped and counted.  rate in [0, 1], sigma >= 0.  Waits when out != NULL. */
int coralai_radiate(coralai_world* w, double rate, float sigma, uint64_t step_index,
                    coralai_stats* out);

/* Merging after step step_index (Abstract: organisms evolve through
 * survival, merging and mutation; System Design: NEAT's crossover operator,
 * applied through the physics).  Cell i is a candidate when word i mod 4 of
 * Philox4x64-10(counter (floor(i / 4), step_index, 0, 1), key (seed, 0)) is
 * below floor(rate * 2^64); it merges with the neighbour it faces (direction
 * R[i]) when the two cells hold different genomes a = G[i] and
 * b = G[neighbour], both read from the map as it was before the call.  The
 * k-th merge in ascending i takes the k-th free slot (ascending slot ids
 * whose genome count is zero); the new genome is the NEAT crossover of a and
 * b: base gene m (of the 56 parameters) comes from b when bit m of word 0 of
 * the Philox block (i, step_index, 0, 2) is set, from a otherwise; each
 * structural-gene position (see coralai_genome_ext) is taken whole from b
 * where bit c of word 1 (direct connection c) or bit k of word 2 (added
 * node k) is set, from a otherwise, so a gene both hold comes from either
 * parent and a gene one holds is kept with probability 1/2 (NEAT's rule for
 * parents of equal fitness; the ecosystem assigns none).  Its network is
 * regenerated and G[i] becomes the slot.  Merges beyond the free slots are
 * dropped.  The stats count merges as hits (stats.hits, stats.dropped).
 * rate in [0, 1].  Waits when out != NULL. */
int coralai_merge(coralai_world* w, double rate, uint64_t step_index, coralai_stats* out);

/* Day / night cycle (Experiment: energy is added to and removed from the
 * substrate in a day / night cycle).  period = 0 switches it off (the
 * default); otherwise, for the step s (steps completed before it, as in
 * coralai_stats.steps) and q = s mod period, the daylight is the triangle
 * wave L = period - 4 min(q, period - q) (period at noon, -period at
 * midnight), and the physics pass sets every cell's energy to
 *   E2 = E1 + floor(inject_quanta * max(L, 0) / period)
 *           - floor(floor(E1 * remove_num / 65536) * max(-L, 0) / period)
 * in exact int64 arithmetic: inject_quanta in [0, 2^40) quanta per cell per
 * step at noon, remove_num in [0, 65536] (the fraction of a cell's energy
 * removed per step at midnight, over 65536).  A cell's energy must stay below
 * 2^40 quanta (else CORALAI_ERR_LEDGER).  Each step then checks on the device
 * that the total mass moved by exactly the injected minus the removed quanta
 * (CORALAI_ERR_MASS otherwise).  Takes effect from the next step of the
 * world; a world that is in a batch takes it at the batch's next
 * coralai_batch_set_worlds. */
int coralai_set_daylight(coralai_world* w, int32_t period, int64_t inject_quanta, int32_t remove_num);

/* Physics variants (Experiment: an explore actuator spreads infrastructure
 * to the neighbour of the maximal actuator; which quantity moves is a
 * reading).  explore_mode 0 (default): the exploration budget
 * floor(kappa_flow * I1) is split over the 8 neighbours by the softmax of
 * the explore actuators; 1 (hard max): all of it goes to the neighbour of the
 * maximal explore actuator (lowest kernel position on ties).
 * kappa_energy > 0: a cell also sends floor(kappa_energy * E1) of its energy
 * along the same directions in the same proportions, so energy moves with
 * the infrastructure; 0 (default): energy stays.  kappa_energy > 0 needs a
 * world created with CORALAI_WORLD_ENERGY_FLOWS.  Per-cell budgets must stay
 * below 2^31 quanta (else CORALAI_ERR_LEDGER).  Takes effect from the next
 * step (a world in a batch: at the batch's next coralai_batch_set_worlds). */
int coralai_set_physics_variant(coralai_world* w, int32_t explore_mode, float kappa_energy);

/* Phylogeny (Discussion: the framework tracks phylogeny).  Every genome slot
 * records the slot it was mutated from, or for a merge its own genome a and
 * its partner's b (parent -1 for a genome set by coralai_set_genomes; second
 * parent -1 unless the slot was born by merging), and the number of steps
 * completed when it was created (the step_index of its radiation or merging
 * call).  A slot that becomes free and is reused records its new genome;
 * coralai_get_births returns the birth events of the last radiation or
 * merging call, so a caller that reads them after each call keeps the whole
 * tree.
 * coralai_get_lineage: parents, second parents and birth steps of n slots
 * (host arrays, any may be NULL).
 * coralai_get_births: the last radiation or merging call's births in the
 * order of their cells: cell index, parent slot, second parent slot (-1
 * after radiation), new slot (host arrays of max_births, any may be NULL);
 * *n_births receives the number of births (which may exceed max_births: the
 * first max_births are copied).  Valid until the next radiation or merging
 * call or coralai_set_genomes (after which there are none). */
int coralai_get_lineage(coralai_world* w, int32_t n, const int32_t* slot_ids, int32_t* parents,
                        int32_t* parents2, int64_t* birth_steps);
int coralai_get_births(coralai_world* w, int32_t max_births, int32_t* cells, int32_t* parents,
                       int32_t* parents2, int32_t* slots, int32_t* n_births);

/* NEAT's measure of genetic similarity (Discussion; Stanley and Miikkulainen's
 * compatibility distance c1 E / N + c2 D / N + c3 W) over the genes above:
 * matching genes are those both genomes hold; of the others, those beyond
 * the smaller of the two highest innovation numbers are excess (E), the
 * rest disjoint (D); W is the mean absolute weight difference of the
 * matching genes, N the larger genome's gene count.  Without structural
 * genes all 56 genes match and the distance is c3 times their mean
 * absolute difference.  Computes the na x nb matrix
 * out_device[i * nb + j] = distance(slots_a[i], slots_b[j]) on the GPU into a
 * caller-owned device buffer of na * nb floats (host slot lists,
 * na + nb <= 54 x genome_capacity).  Waits for the stream. */
int coralai_genetic_distance(coralai_world* w, int32_t na, const int32_t* slots_a, int32_t nb,
                             const int32_t* slots_b, float c1, float c2, float c3, float* out_device);

/* The cycle's energy ledger in quanta: injected and removed by the last step,
 * and in total since the world was created.  Waits for the stream; any
 * pointer may be NULL. */
int coralai_get_energy_ledger(coralai_world* w, int64_t* injected_last, int64_t* removed_last,
                              int64_t* injected_total, int64_t* removed_total);

/* Set the count of completed steps (coralai_stats.steps), which sets the
 * day / night cycle's phase and the birth step of genomes set afterwards:
 * with coralai_set_state and coralai_set_genomes it resumes a world from a
 * checkpoint (coralai_get_state, coralai_get_genomes of the live slots and
 * the stats' step count).  steps >= 0.  Waits for the stream. */
int coralai_set_step_count(coralai_world* w, int64_t steps);

/* Wait for the world's stream; report (and clear) device error bits. */
int coralai_sync(coralai_world* w);
int coralai_get_stats(coralai_world* w, coralai_stats* out);

/* Batched form: many worlds advanced together by one captured HIP graph of
 * persistent kernels over a device-side world table.  All worlds of a batch
 * share one device, one network shape (layers, hidden) and one precision;
 * the batch's stream is used for the whole step.  The table holds up to
 * max_worlds entries; set_worlds may change the set between steps without a
 * new graph.  The batch's arena (coralai_batch_bytes) is caller-owned.
 * Worlds may live on streams other than the batch's: set_worlds makes the
 * batch's stream wait for work already queued on each world's stream, and
 * batch_step makes each world's stream wait for the steps it queued, so a
 * later call on a world (get_state, step) sees their result.  A world must
 * leave the batch (set_worlds without it) before coralai_world_destroy. */
size_t coralai_batch_bytes(int32_t max_worlds);
int coralai_batch_create(int32_t max_worlds, void* dev_arena, size_t arena_bytes,
                         void* hip_stream, coralai_batch** out);
int coralai_batch_set_worlds(coralai_batch* b, coralai_world* const* worlds, int32_t n);
int coralai_batch_step(coralai_batch* b, int32_t n_steps);
int coralai_batch_sync(coralai_batch* b);
int coralai_batch_destroy(coralai_batch* b);

/* Launch tuning.  coralai_autotune times the candidate configurations on the
 * world's current state (without advancing it) and keeps the fastest;
 * coralai_set_tuning forces one.  act_cells: column groups of 16 cells the
 * network kernel processes together in one pass (1, 2 or 4; a pass holding
 * none of a 64-cell unit's cells is skipped); act_waves: 0 = fewer
 * wavefronts per SIMD with more registers each, 1 = more wavefronts;
 * phys_tile: LDS halo tiles 0 = 64x16, 1 = 32x8, 2 = 64x8, or 3 = streaming
 * without LDS (one thread per four cells of a row when the width is a
 * multiple of 4, else per cell).  The batch versions tune the batch's
 * single captured step over its current worlds.  Defaults before any call:
 * act_cells 2, act_waves 0, phys_tile 2. */
int coralai_autotune(coralai_world* w, int32_t* act_cells_out, int32_t* act_waves_out,
                     int32_t* phys_tile_out);
int coralai_set_tuning(coralai_world* w, int32_t act_cells, int32_t act_waves, int32_t phys_tile);
int coralai_batch_autotune(coralai_batch* b, int32_t* act_cells_out, int32_t* act_waves_out,
                           int32_t* phys_tile_out);
int coralai_batch_set_tuning(coralai_batch* b, int32_t act_cells, int32_t act_waves,
                             int32_t phys_tile);

/* Live phase timing.  While profiling is on, coralai_step, coralai_radiate and coralai_merge
 * launch their kernels directly (no graph) with HIP events recorded on the
 * world's stream between the phases; coralai_get_profile waits for the
 * stream and returns, per phase, the summed milliseconds and the number of
 * timed launches since profiling was switched on.  Phases:
 * 0 bucketing (histogram, scans, compaction), 1 sense+act (network),
 * 2 physics, 3 step finalisation, 4 radiation or merging (incl. weight
 * regeneration). */
enum { CORALAI_PHASES = 5 };
int coralai_set_profiling(coralai_world* w, int on);
int coralai_get_profile(coralai_world* w, double* ms_sum, int64_t* launches);

const char* coralai_last_error(void);
const char* coralai_version(void);

/* Parity hooks (tests).  All wait for the stream.
 *  debug_buckets:   genome counts [capacity], exclusive offsets [capacity+1]
 *                   and the bucket order perm [W*H] of the current state
 *                   (cells grouped by genome; order inside a genome is not
 *                   specified);
 *  debug_actuators: raw network outputs [W*H x 14] for the current state;
 *  debug_set_weights / debug_get_weights: one slot's network in the flat
 *                   layout [W_0 (h x 54) row-major, b_0, W_1, b_1, ...] as
 *                   float; set marks the slot set;
 *  debug_physics:   run the physics alone from given records -- I1 [W*H]
 *                   int64, flows [W*H x 8] uint32 (< 2^31) toward absolute
 *                   directions 0..7, explore direction [W*H] uint8 -- on the current G,
 *                   R; the result becomes the current state with E and C
 *                   unchanged (infrastructure flows only: an error while
 *                   energy transport is on);
 *  debug_set_act_segments: the number of segments of the genome-ordered
 *                   unit list from which each wavefront of the network kernel
 *                   takes one chunk (0 = automatic: 4 for BF16 networks on
 *                   jobs of at least 64 units per wavefront, else 1); results
 *                   do not depend on it, which the tests check. */
int coralai_debug_buckets(coralai_world* w, int32_t* counts, int32_t* offsets, int32_t* perm);
int coralai_debug_actuators(coralai_world* w, float* act);
int coralai_debug_set_weights(coralai_world* w, int32_t slot, const float* flat);
int coralai_debug_get_weights(coralai_world* w, int32_t slot, float* flat);
int coralai_debug_physics(coralai_world* w, const int64_t* i1, const uint32_t* flows8,
                          const uint8_t* explore_dir);
int coralai_debug_set_act_segments(coralai_world* w, int32_t n_segments);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as coralai_debug_set_weights, staged through a fixed 64 KiB
 * buffer in the library's device data (one per device, kept until the
 * process ends) instead of a buffer allocated per call.  Calls no hipMalloc
 * or hipFree.  Networks larger than 16384 floats are rejected with
 * CORALAI_E_INVALID (every shape the world description allows fits: the
 * largest, 54-64-64-14, has 8590).  Waits for the world's stream before it
 * returns; calls that overlap on one device (from several threads) race on
 * the shared buffer. */
int coralai_debug_set_weights_noalloc(coralai_world* w, int32_t slot, const float* flat);

#ifdef __cplusplus
}
#endif
#endif /* CORALAI_H */
