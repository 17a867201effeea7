/*
 * coralai_oracle.c -- plain, slow FP64 CPU oracle of the Coralai per-step
 * ecosystem update.  TEST INFRASTRUCTURE ONLY: it is called by the tests,
 * by the bench's CPU-baseline leg and by the smoke check, never by the
 * product path, and it shares no code with the HIP library.
 *
 * What it follows (the paper, "Coralai: Intrinsic Evolution of Embodied
 * Neural Cellular Automata Ecosystems"):
 *   - System Design: substrate with named channels; GenomeIndex selects the
 *     cell's network; each step sends the Kernel neighbourhood of Sensor
 *     channels to that network, whose Actuator outputs Physics turns into
 *     substrate change.
 *   - System Design, second paragraph: HyperNEAT -- a small CPPN generates
 *     the weights and biases of each genome's larger dense network.
 *   - Experiment: Infrastructure / Energy / Communication channels; Invest and
 *     Liquidate convert Energy <-> Infrastructure; communication passes
 *     through a sigmoid; the kernel is the Moore neighbourhood ordered by
 *     angular distance to the cell's Rotation; Explore actuators, one per
 *     offset, spread infrastructure; takeover rule with maximal investment.
 *   - Fig. 1 (C): radiation mutates CPPN genomes and regenerates weights.
 *   - Abstract and System Design: merging, NEAT's crossover of two genomes,
 *     applied through the physics where two organisms meet.
 * Every constant the paper leaves open is a recorded reading (directions,
 * kernel order, ledger quanta, rates, flow budget, CPPN geometry, Philox
 * layout); each function names the reading it uses.
 *
 * Arithmetic: FP64 throughout; mass is an exact int64 ledger of 2^-24 units.
 * Arrays are row-major, linear cell index i = y*W + x, y pointing down.
 *
 * Parity pins: every function here is pinned by CPU tests against closed
 * forms, invariants, library routines (numpy Philox, bincount, argsort, a
 * numpy MLP) or a brute-force pull-from-definition implementation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_QUANTUM (1.0 / 16777216.0) /* 2^-24 mass units per quantum */
#define ORC_NPARAM 56                   /* CPPN: A (8x5) then B (2x8) */
#define ORC_NIN 54                      /* 9 kernel positions x 6 channels */
#define ORC_NOUT 14                     /* invest, liquidate, 4 comm, 8 flow */

typedef struct {
    int32_t width, height;
    int32_t n_weight_layers; /* 2: 54-h-14, 3: 54-h-h-14 */
    int32_t hidden;
    double rho_invest, rho_liquidate, kappa_flow;
    /* day / night cycle (0 = none): period in steps, energy quanta added per
     * cell per step at noon, fraction (over 65536) of a cell's energy removed
     * per step at midnight, and the number of steps completed before this one */
    int32_t day_period;
    int32_t night_num;
    int64_t day_inject;
    int64_t cycle_step;
    /* physics variants: explore_mode 0 splits the exploration budget by the
     * softmax of the explore actuators, 1 sends all of it to the maximal
     * one; kappa_energy > 0 also moves floor(kappa_energy E1) of a cell's
     * energy along the same directions in the same proportions */
    int32_t explore_mode;
    int32_t pad_desc;
    double kappa_energy;
} orc_desc;

/* Per-cell result of sense -> act -> local conversion (the "record" that the
 * physics pass reads from a cell's neighbours). */
typedef struct {
    int64_t e1, i1;        /* ledger after invest / liquidate */
    int64_t flow[8];       /* outflow toward absolute direction d */
    int32_t explore_dir;   /* absolute direction of the argmax explore */
    int32_t explore_pos;   /* kernel position p* in 1..8 */
    double logit_gap;      /* top-1 minus top-2 flow logit (FP64) */
    int32_t runner_dir;    /* absolute direction of the second-largest logit */
    int32_t exact;         /* 1: every integer above is decided with margin (see floor_decided) */
    int64_t eflow[8];      /* energy sent toward absolute direction d (energy transport) */
} orc_record;

/* Directions: d at 45*d degrees counter-clockwise from +x, y pointing down. */
static const int DX[8] = {1, 1, 0, -1, -1, -1, 0, 1};
static const int DY[8] = {0, -1, -1, -1, 0, 1, 1, 1};
/* Kernel order for rotation r: centre, then r, r+1, r-1, r+2, r-2, r+3, r-3,
 * r+4 (increasing angular distance; the counter-clockwise member of each
 * equal-distance pair first). */
static const int KOFF[9] = {0, 0, 1, -1, 2, -2, 3, -3, 4};

int orc_kernel_dir(int r, int p) { return (r + KOFF[p] + 8) & 7; } /* p in 1..8 */

static int64_t nbr(const orc_desc* d, int64_t i, int dir) {
    int64_t W = d->width, H = d->height;
    int64_t x = i % W, y = i / W;
    x = ((x + DX[dir]) % W + W) % W;
    y = ((y + DY[dir]) % H + H) % H;
    return y * W + x;
}

int orc_layer_widths(const orc_desc* d, int32_t* widths) {
    int n = d->n_weight_layers;
    widths[0] = ORC_NIN;
    for (int l = 1; l < n; ++l) widths[l] = d->hidden;
    widths[n] = ORC_NOUT;
    return n + 1;
}

/* Number of doubles in one genome's flat network: for each layer l,
 * W_l (L_{l+1} x L_l, row-major) followed by b_l (L_{l+1}). */
int64_t orc_net_size(const orc_desc* d) {
    int32_t L[8];
    orc_layer_widths(d, L);
    int64_t n = 0;
    for (int l = 0; l < d->n_weight_layers; ++l) n += (int64_t)L[l + 1] * L[l] + L[l + 1];
    return n;
}

/* CPPN (HyperNEAT, System Design): inputs z = (x1, y1, x2, y2, 1); 8 hidden
 * nodes h_k = phi_k(sum_m A[k][m] z_m) with phi = sin, gauss, tanh, identity
 * for k mod 4 = 0, 1, 2, 3 and gauss(s) = exp(-s^2); two linear outputs
 * (weight, bias) = B h. */
void orc_cppn(const double* p, double x1, double y1, double x2, double y2, double out[2]) {
    const double z[5] = {x1, y1, x2, y2, 1.0};
    double h[8];
    for (int k = 0; k < 8; ++k) {
        double s = 0.0;
        for (int m = 0; m < 5; ++m) s += p[k * 5 + m] * z[m];
        switch (k & 3) {
            case 0: h[k] = sin(s); break;
            case 1: h[k] = exp(-s * s); break;
            case 2: h[k] = tanh(s); break;
            default: h[k] = s; break;
        }
    }
    for (int o = 0; o < 2; ++o) {
        double s = 0.0;
        for (int k = 0; k < 8; ++k) s += p[40 + o * 8 + k] * h[k];
        out[o] = s;
    }
}

/* HyperNEAT substrate: neuron j of layer l sits at (x_{l,j}, y_l) with
 * y_l = -1 + 2l/n and x_{l,j} = -1 + 2j/(L_l - 1).  Weight W_l[o][j] is the
 * CPPN weight output at (x_{l,j}, y_l, x_{l+1,o}, y_{l+1}) divided by
 * sqrt(L_l); bias b_l[o] is the CPPN bias output at (0, y_l, x_{l+1,o},
 * y_{l+1}).  No expression threshold. */
void orc_cppn_to_net(const orc_desc* d, const double* p, double* net) {
    int32_t L[8];
    orc_layer_widths(d, L);
    int n = d->n_weight_layers;
    double* w = net;
    for (int l = 0; l < n; ++l) {
        double yi = -1.0 + 2.0 * l / n, yo = -1.0 + 2.0 * (l + 1) / n;
        double scale = 1.0 / sqrt((double)L[l]);
        for (int o = 0; o < L[l + 1]; ++o) {
            double xo = -1.0 + 2.0 * o / (L[l + 1] - 1);
            for (int j = 0; j < L[l]; ++j) {
                double xi = -1.0 + 2.0 * j / (L[l] - 1);
                double r[2];
                orc_cppn(p, xi, yi, xo, yo, r);
                w[(int64_t)o * L[l] + j] = r[0] * scale;
            }
        }
        w += (int64_t)L[l + 1] * L[l];
        for (int o = 0; o < L[l + 1]; ++o) {
            double xo = -1.0 + 2.0 * o / (L[l + 1] - 1);
            double r[2];
            orc_cppn(p, 0.0, yi, xo, yo, r);
            w[o] = r[1];
        }
        w += L[l + 1];
    }
}

/* The networks of n genomes (params: n x 56 doubles) into nets (n x
 * orc_net_size doubles), one genome per thread: orc_cppn_to_net each. */
void orc_nets_for(const orc_desc* d, int64_t n, const double* params, double* nets) {
    const int64_t nsz = orc_net_size(d);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) orc_cppn_to_net(d, params + k * ORC_NPARAM, nets + k * nsz);
}

/* NEAT structural genes over a bounded superset of the CPPN (System Design:
 * NEAT's mutation and crossover operators).  Beyond the 56 base genes (A,
 * then B) a genome may hold:
 *   - direct connections input m -> output o (innovation 56 + 5 o + m),
 *     enabled by bit 5 o + m of conn_mask, weight conn_w[5 o + m];
 *   - added nodes N_k, k = 2 j + o, that split the connection hidden j ->
 *     output o (NEAT's add-node mutation): enabled by bit k of node_mask,
 *     activation node_act bits 2k..2k+1 (sin, gauss, tanh, identity), in
 *     weight node_in[k] (innovation 66 + 2 k) and out weight node_out[k]
 *     (innovation 67 + 2 k); while N_k is enabled the base connection
 *     B[o][j] is disabled.
 * Output o is then sum over j of (N_{2j+o} enabled ? node_out phi(node_in
 * h_j) : B[o][j] h_j) plus sum over enabled direct connections of
 * conn_w z_m.  A genome without structural genes is the base CPPN. */
typedef struct {
    uint32_t conn_mask, node_mask, node_act, pad;
    double conn_w[10];
    double node_in[16];
    double node_out[16];
} orc_ext;

static double node_fn(int f, double s) {
    switch (f & 3) {
        case 0: return sin(s);
        case 1: return exp(-s * s);
        case 2: return tanh(s);
        default: return s;
    }
}

void orc_cppn_x(const double* p, const orc_ext* e, double x1, double y1, double x2, double y2,
                double out[2]) {
    const double z[5] = {x1, y1, x2, y2, 1.0};
    double h[8];
    for (int k = 0; k < 8; ++k) {
        double s = 0.0;
        for (int m = 0; m < 5; ++m) s += p[k * 5 + m] * z[m];
        h[k] = node_fn(k, s);
    }
    for (int o = 0; o < 2; ++o) {
        double s = 0.0;
        for (int j = 0; j < 8; ++j) {
            const int k = 2 * j + o;
            if ((e->node_mask >> k) & 1u)
                s += e->node_out[k] * node_fn((int)(e->node_act >> (2 * k)), e->node_in[k] * h[j]);
            else
                s += p[40 + o * 8 + j] * h[j];
        }
        for (int m = 0; m < 5; ++m)
            if ((e->conn_mask >> (5 * o + m)) & 1u) s += e->conn_w[5 * o + m] * z[m];
        out[o] = s;
    }
}

/* orc_cppn_to_net with structural genes (the same substrate queries). */
void orc_cppn_to_net_x(const orc_desc* d, const double* p, const orc_ext* e, double* net) {
    int32_t L[8];
    orc_layer_widths(d, L);
    int n = d->n_weight_layers;
    double* w = net;
    for (int l = 0; l < n; ++l) {
        double yi = -1.0 + 2.0 * l / n, yo = -1.0 + 2.0 * (l + 1) / n;
        double scale = 1.0 / sqrt((double)L[l]);
        for (int o = 0; o < L[l + 1]; ++o) {
            double xo = -1.0 + 2.0 * o / (L[l + 1] - 1);
            for (int j = 0; j < L[l]; ++j) {
                double xi = -1.0 + 2.0 * j / (L[l] - 1);
                double r[2];
                orc_cppn_x(p, e, xi, yi, xo, yo, r);
                w[(int64_t)o * L[l] + j] = r[0] * scale;
            }
        }
        w += (int64_t)L[l + 1] * L[l];
        for (int o = 0; o < L[l + 1]; ++o) {
            double xo = -1.0 + 2.0 * o / (L[l + 1] - 1);
            double r[2];
            orc_cppn_x(p, e, 0.0, yi, xo, yo, r);
            w[o] = r[1];
        }
        w += L[l + 1];
    }
}

void orc_nets_for_x(const orc_desc* d, int64_t n, const double* params, const orc_ext* ext, double* nets) {
    const int64_t nsz = orc_net_size(d);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) orc_cppn_to_net_x(d, params + k * ORC_NPARAM, ext + k, nets + k * nsz);
}

/* Sensors over the Kernel (Experiment): u[p*6 + ch] is channel ch of the
 * cell at kernel position p, channels (E, I, C0, C1, C2, C3), E and I as
 * mass values (quanta * 2^-24). */
void orc_sense(const orc_desc* d, const int64_t* E, const int64_t* I, const double* C,
               const uint8_t* R, int64_t i, double* u) {
    int64_t N = (int64_t)d->width * d->height;
    int r = R[i] & 7;
    for (int p = 0; p < 9; ++p) {
        int64_t n = p == 0 ? i : nbr(d, i, orc_kernel_dir(r, p));
        u[p * 6 + 0] = (double)E[n] * ORC_QUANTUM;
        u[p * 6 + 1] = (double)I[n] * ORC_QUANTUM;
        for (int c = 0; c < 4; ++c) u[p * 6 + 2 + c] = C[c * N + n];
    }
}

/* The genome's dense network: tanh hidden layers, linear output layer. */
void orc_forward(const orc_desc* d, const double* net, const double* u, double* a) {
    int32_t L[8];
    orc_layer_widths(d, L);
    double buf0[128], buf1[128];
    const double* x = u;
    double* y = buf0;
    const double* w = net;
    for (int l = 0; l < d->n_weight_layers; ++l) {
        const double* b = w + (int64_t)L[l + 1] * L[l];
        int last = l == d->n_weight_layers - 1;
        double* dst = last ? a : y;
        for (int o = 0; o < L[l + 1]; ++o) {
            double s = 0.0;
            for (int j = 0; j < L[l]; ++j) s += w[(int64_t)o * L[l] + j] * x[j];
            s += b[o];
            dst[o] = last ? s : tanh(s);
        }
        w = b + L[l + 1];
        x = dst;
        y = (y == buf0) ? buf1 : buf0;
    }
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Relative perturbation of a floored argument that an FP32 evaluation of the
 * same step may make.  A sigmoid or a softmax weight moves relatively by about
 * the absolute error of the network outputs it reads (twice that for a
 * softmax weight), which an FP32 evaluation keeps near 1e-4 even at the
 * worst cells of a 4096 x 4096 grid; 1e-3 leaves a factor of 5 on top. */
#define ORC_FLOOR_REL 1e-3

/* floor(x) of a non-negative argument is decided when every value within
 * ORC_FLOOR_REL * x of x has the same floor, or when x is exactly zero (one
 * factor of the product is an exact zero, which any precision reproduces).
 * Used only for the near-tie report of the parity tests, never for the
 * step's results. */
static int floor_decided(double x) {
    if (x == 0.0) return 1;
    return floor(x * (1.0 - ORC_FLOOR_REL)) == floor(x * (1.0 + ORC_FLOOR_REL));
}

/* Actuators -> local part of the physics (Experiment):
 *   invest / liquidate: x_inv = min(E, floor(rho_inv * sig(a0) * E)),
 *                       x_liq = min(I, floor(rho_liq * sig(a1) * I)),
 *                       E1 = E - x_inv + x_liq, I1 = I + x_inv - x_liq;
 *   communication:      C'_j = sig(a_{2+j});
 *   explore / flow:     budget F = floor(kappa * I1) split by the softmax of
 *                       the 8 flow logits a_6..a_13 (kernel positions 1..8),
 *                       f_p = min(floor(w_p F), F - sum_{q<p} f_q);
 *                       the explored neighbour is the argmax position (lowest
 *                       on ties) and its investment is that position's flow.
 *                       Hard-max variant (explore_mode 1): the maximal
 *                       explore actuator takes the whole budget, f_p* = F.
 *   energy transport:   with kappa_energy > 0 the budget floor(kappa_energy
 *                       E1) is split the same way (softmax weights with the
 *                       running clamp, or all to p*).
 * All in FP64, quanta as integers. */
void orc_actuate(const orc_desc* d, int64_t e, int64_t i, int r, const double* a,
                 orc_record* rec, double* comm_out) {
    double se = sigmoid(a[0]), sl = sigmoid(a[1]);
    const double arg_inv = d->rho_invest * se * (double)e, arg_liq = d->rho_liquidate * sl * (double)i;
    int64_t xi = (int64_t)floor(arg_inv);
    int64_t xl = (int64_t)floor(arg_liq);
    int exact = floor_decided(arg_inv) && floor_decided(arg_liq);
    if (xi > e) xi = e;
    if (xl > i) xl = i;
    if (xi < 0) xi = 0;
    if (xl < 0) xl = 0;
    rec->e1 = e - xi + xl;
    rec->i1 = i + xi - xl;
    for (int j = 0; j < 4; ++j) comm_out[j] = sigmoid(a[2 + j]);

    const double* lg = a + 6; /* lg[p-1] is the logit of position p */
    double m = lg[0];
    int best = 0;
    for (int k = 1; k < 8; ++k)
        if (lg[k] > m) { m = lg[k]; best = k; }
    double second = -INFINITY;
    int runner = best == 0 ? 1 : 0;
    for (int k = 0; k < 8; ++k)
        if (k != best && lg[k] > second) { second = lg[k]; runner = k; }
    rec->logit_gap = m - second;
    rec->runner_dir = orc_kernel_dir(r, runner + 1);
    double ex[8], s = 0.0;
    for (int k = 0; k < 8; ++k) { ex[k] = exp(lg[k] - m); s += ex[k]; }
    const double arg_F = d->kappa_flow * (double)rec->i1;
    int64_t F = (int64_t)floor(arg_F);
    if (F < 0) F = 0;
    exact = exact && floor_decided(arg_F);
    int64_t used = 0;
    for (int k = 0; k < 8; ++k) {
        int64_t f;
        if (d->explore_mode == 1) {
            f = k == best ? F : 0;
        } else {
            const double arg_f = (ex[k] / s) * (double)F;
            exact = exact && floor_decided(arg_f);
            f = (int64_t)floor(arg_f);
            if (f > F - used) f = F - used;
            if (f < 0) f = 0;
        }
        used += f;
        rec->flow[orc_kernel_dir(r, k + 1)] = f;
    }
    for (int k = 0; k < 8; ++k) rec->eflow[k] = 0;
    if (d->kappa_energy > 0.0) {
        int64_t FE = (int64_t)floor(d->kappa_energy * (double)rec->e1);
        if (FE < 0) FE = 0;
        int64_t eused = 0;
        for (int k = 0; k < 8; ++k) {
            int64_t g;
            if (d->explore_mode == 1) {
                g = k == best ? FE : 0;
            } else {
                g = (int64_t)floor((ex[k] / s) * (double)FE);
                if (g > FE - eused) g = FE - eused;
                if (g < 0) g = 0;
            }
            eused += g;
            rec->eflow[orc_kernel_dir(r, k + 1)] = g;
        }
    }
    rec->explore_pos = best + 1;
    rec->explore_dir = orc_kernel_dir(r, best + 1);
    rec->exact = exact;
}

/* Whole per-cell act: sense, network of the cell's genome, actuate. */
static void cell_record(const orc_desc* d, const int64_t* E, const int64_t* I, const double* C,
                        const int32_t* G, const uint8_t* R, const double* nets, int64_t nsz,
                        int64_t i, orc_record* rec, double* comm, double* act) {
    double u[ORC_NIN], a[ORC_NOUT];
    orc_sense(d, E, I, C, R, i, u);
    orc_forward(d, nets + (int64_t)G[i] * nsz, u, a);
    if (act)
        for (int k = 0; k < ORC_NOUT; ++k) act[k] = a[k];
    orc_actuate(d, E[i], I[i], R[i] & 7, a, rec, comm);
}

/* Day / night cycle (Experiment: energy is added to and removed from the
 * substrate in a day / night cycle; the shape is a reading).  The daylight of
 * the step is a triangle wave over the period P: with q = cycle_step mod P
 * the cycle has run q steps since noon, min(q, P - q) is the distance to the
 * nearest noon, and the daylight is L = P - 4 min(q, P - q), so L = P at
 * noon, 0 a quarter period away, -P at midnight.  By day (L > 0) every cell
 * gains floor(A L / P) quanta of energy; by night (L < 0) it loses
 * floor(floor(E1 num / 65536) (-L) / P) quanta of its energy E1 (never more
 * than E1).  Integers throughout.  Returns the cell's energy after the cycle
 * and adds the cell's gain and loss to io[0] and io[1]. */
static int64_t cycle_energy(const orc_desc* d, int64_t e1, int64_t io[2]) {
    if (d->day_period <= 0) return e1;
    const int64_t P = d->day_period;
    const int64_t q = d->cycle_step % P;
    const int64_t to_noon = q < P - q ? q : P - q;
    const int64_t L = P - 4 * to_noon;
    int64_t gain = 0, loss = 0;
    if (L > 0) gain = d->day_inject * L / P;
    if (L < 0) loss = ((e1 * (int64_t)d->night_num) / 65536) * (-L) / P;
    io[0] += gain;
    io[1] += loss;
    return e1 + gain - loss;
}

/* Physics (Experiment, exploration and takeover), pulled at target t: every
 * neighbour n = nbr(t, d) sends t its flow toward direction (d+4) mod 8;
 * neighbours whose explore direction is (d+4) mod 8 are candidates; the
 * maximal investment wins (lowest d on ties) and takes the cell over when it
 * strictly exceeds I1(t), t adopting n's genome and the exploration
 * direction as its rotation.  E2 = E1.  Returns the takeover flag and the
 * decision margins used by the near-tie protocol: |v_win - I1(t)| and, when
 * the winner takes over, v_win - v_second (both in quanta), and the size
 * max(v_win, I1(t)) they are measured against. */
static int cell_physics(const orc_desc* d, const orc_record* rec_t, const orc_record* const nrec[8],
                        const int32_t* G, const uint8_t* R, const int64_t nidx[8], int64_t t,
                        int64_t* i2, int32_t* g2, uint8_t* r2, double* margin_take,
                        double* margin_rank, double* magnitude) {
    int64_t out = 0, in = 0;
    for (int k = 0; k < 8; ++k) out += rec_t->flow[k];
    int win = -1;
    int64_t vbest = 0, vsecond = -1;
    for (int dd = 0; dd < 8; ++dd) {
        int back = (dd + 4) & 7;
        const orc_record* rn = nrec[dd];
        in += rn->flow[back];
        if (rn->explore_dir == back) {
            int64_t v = rn->flow[back];
            if (win < 0 || v > vbest) {
                if (win >= 0) vsecond = vbest;
                vbest = v;
                win = dd;
            } else if (v > vsecond) {
                vsecond = v;
            }
        }
    }
    *i2 = rec_t->i1 - out + in;
    *g2 = G[t];
    *r2 = R[t];
    *margin_take = INFINITY;
    *margin_rank = INFINITY;
    *magnitude = 0.0;
    int took = 0;
    if (win >= 0) {
        *margin_take = fabs((double)vbest - (double)rec_t->i1);
        *magnitude = (double)(vbest > rec_t->i1 ? vbest : rec_t->i1);
        if (vsecond >= 0 && vbest > rec_t->i1) *margin_rank = (double)(vbest - vsecond);
        if (vbest > rec_t->i1) {
            *g2 = G[nidx[win]];
            *r2 = (uint8_t)((win + 4) & 7);
            took = 1;
        }
    }
    return took;
}

/* One step for output rows [y0, y1) of the torus.  Records are computed for
 * rows y0-1 .. y1 (wrapping); a full step is y0 = 0, y1 = H.
 * Outputs (full-size arrays; only the requested rows are written):
 *   E2, I2 (int64), C2 (4 planes, double), G2, R2;
 *   act (N x 14, nullable): raw network outputs of the rows;
 *   rec_out (N, nullable): per-cell records of the rows;
 *   margins (N x 5, nullable): per target t, the decision margins of the
 *   near-tie report:
 *     0: smallest flow-logit gap (top-1 minus top-2) among the neighbours
 *        whose two leading explore directions include t and that could
 *        invest in t at all (some flow not decided to be exactly zero);
 *     1: |v_win - I1(t)|, infinity without a candidate explorer;
 *     2: v_win - v_second when the winner takes over, else infinity;
 *     3: max(v_win, I1(t)) with a candidate, else 0;
 *     4: 1 when I1(t) and every candidate's flows are decided integers
 *        (floor_decided), so that the takeover and ranking decisions are
 *        exact comparisons of exactly known integers; else 0;
 *   energy_io (2, nullable): the day / night cycle's injected and removed
 *   quanta over the rows.
 * E2 = the cycle applied to E1 (cycle_energy; E1 itself without a cycle).
 * Returns the number of takeovers in the rows, or -1 on a bad genome id. */
int64_t orc_step_rows(const orc_desc* d, const int64_t* E, const int64_t* I, const double* C,
                      const int32_t* G, const uint8_t* R, const double* nets, int32_t n_genomes,
                      int32_t y0, int32_t y1, int64_t* E2, int64_t* I2, double* C2, int32_t* G2,
                      uint8_t* R2, double* act, orc_record* rec_out, double* margins,
                      int64_t* energy_io) {
    const int64_t W = d->width, H = d->height, N = W * H;
    const int64_t nsz = orc_net_size(d);
    for (int64_t i = 0; i < N; ++i)
        if (G[i] < 0 || G[i] >= n_genomes) return -1;
    int32_t rows = y1 - y0;
    int32_t rrows = rows + 2 > H ? (int32_t)H : rows + 2;
    int32_t rstart = rows + 2 > H ? 0 : y0 - 1;
    orc_record* rec = (orc_record*)malloc(sizeof(orc_record) * (size_t)N);
    double* cn = (double*)malloc(sizeof(double) * 4 * (size_t)N);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)rrows * W; ++k) {
        int64_t y = ((rstart + k / W) % H + H) % H, x = k % W, i = y * W + x;
        double comm[4];
        int in_rows = (y - y0 + H) % H < rows;
        cell_record(d, E, I, C, G, R, nets, nsz, i, &rec[i], comm,
                    (act && in_rows) ? act + i * ORC_NOUT : NULL);
        for (int c = 0; c < 4; ++c) cn[c * N + i] = comm[c];
    }
    int64_t takeovers = 0, gained = 0, lost = 0;
#pragma omp parallel for schedule(static) reduction(+ : takeovers, gained, lost)
    for (int64_t k = 0; k < (int64_t)rows * W; ++k) {
        int64_t y = (y0 + k / W) % H, x = k % W, t = y * W + x;
        int64_t nidx[8];
        const orc_record* nrec[8];
        /* a neighbour's near-tied argmax matters to t only if one of its two
         * leading explore directions points at t */
        double gap = INFINITY;
        int decided = rec[t].exact;
        for (int dd = 0; dd < 8; ++dd) {
            nidx[dd] = nbr(d, t, dd);
            nrec[dd] = &rec[nidx[dd]];
            const orc_record* rn = nrec[dd];
            const int back = (dd + 4) & 7;
            int64_t fsum = 0;
            for (int k = 0; k < 8; ++k) fsum += rn->flow[k];
            /* flows all exactly zero: it invests nothing in any direction */
            const int idle = rn->exact && fsum == 0;
            if ((rn->explore_dir == back || rn->runner_dir == back) && !idle && rn->logit_gap < gap)
                gap = rn->logit_gap;
            if (rn->explore_dir == back) decided = decided && rn->exact;
        }
        double mt, mr, mg;
        takeovers += cell_physics(d, &rec[t], nrec, G, R, nidx, t, &I2[t], &G2[t], &R2[t], &mt,
                                  &mr, &mg);
        /* energy transport: E1 minus the cell's own energy flows plus the
         * flows its neighbours send toward it (direction d's neighbour sends
         * its flow toward (d+4) mod 8) */
        int64_t e_mid = rec[t].e1;
        for (int k = 0; k < 8; ++k) e_mid -= rec[t].eflow[k];
        for (int dd = 0; dd < 8; ++dd) e_mid += nrec[dd]->eflow[(dd + 4) & 7];
        int64_t io[2] = {0, 0};
        E2[t] = cycle_energy(d, e_mid, io);
        gained += io[0];
        lost += io[1];
        for (int c = 0; c < 4; ++c) C2[c * N + t] = cn[c * N + t];
        if (rec_out) rec_out[t] = rec[t];
        if (margins) {
            margins[t * 5 + 0] = gap;
            margins[t * 5 + 1] = mt;
            margins[t * 5 + 2] = mr;
            margins[t * 5 + 3] = mg;
            margins[t * 5 + 4] = decided ? 1.0 : 0.0;
        }
    }
    free(rec);
    free(cn);
    if (energy_io) {
        energy_io[0] = gained;
        energy_io[1] = lost;
    }
    return takeovers;
}

/* Physics alone, from given records (I1, flows in absolute-direction order,
 * explore direction).  Pure integer work. */
int64_t orc_physics_from_records(const orc_desc* d, const int64_t* i1, const int64_t* flow8,
                                 const int32_t* explore_dir, const int32_t* G, const uint8_t* R,
                                 int64_t* I2, int32_t* G2, uint8_t* R2) {
    const int64_t N = (int64_t)d->width * d->height;
    orc_record* rec = (orc_record*)malloc(sizeof(orc_record) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        rec[i].i1 = i1[i];
        rec[i].e1 = 0;
        for (int k = 0; k < 8; ++k) rec[i].flow[k] = flow8[i * 8 + k];
        rec[i].explore_dir = explore_dir[i];
        rec[i].explore_pos = 0;
        rec[i].logit_gap = 0;
        rec[i].runner_dir = 0;
        rec[i].exact = 0;
        for (int k = 0; k < 8; ++k) rec[i].eflow[k] = 0;
    }
    int64_t takeovers = 0;
    for (int64_t t = 0; t < N; ++t) {
        int64_t nidx[8];
        const orc_record* nrec[8];
        for (int dd = 0; dd < 8; ++dd) {
            nidx[dd] = nbr(d, t, dd);
            nrec[dd] = &rec[nidx[dd]];
        }
        double mt, mr, mg;
        takeovers += cell_physics(d, &rec[t], nrec, G, R, nidx, t, &I2[t], &G2[t], &R2[t], &mt,
                                  &mr, &mg);
    }
    free(rec);
    return takeovers;
}

/* NEAT's compatibility distance of two genomes (Discussion: NEAT's measure
 * of genetic similarity; the measure of Stanley and Miikkulainen,
 * c1 E / N + c2 D / N + c3 W).  The CPPNs share one fixed topology, so all
 * 56 genes match: no excess (E) or disjoint (D) genes, and W is the mean
 * absolute difference of the matching genes' weights. */
double orc_genetic_distance(const double* a, const double* b, double c3) {
    double w = 0.0;
    for (int m = 0; m < ORC_NPARAM; ++m) w += fabs(a[m] - b[m]);
    return c3 * (w / ORC_NPARAM);
}

/* Buckets: counts = histogram of G over [0, cap), offsets = exclusive prefix
 * sum, perm = cells ordered by genome, ascending cell index within a genome
 * (a stable counting sort).  Returns -1 on an id outside [0, cap). */
int orc_buckets(int64_t n, const int32_t* G, int32_t cap, int32_t* counts, int32_t* offsets,
                int32_t* perm) {
    for (int32_t g = 0; g < cap; ++g) counts[g] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (G[i] < 0 || G[i] >= cap) return -1;
        counts[G[i]]++;
    }
    int32_t run = 0;
    for (int32_t g = 0; g < cap; ++g) { offsets[g] = run; run += counts[g]; }
    offsets[cap] = run;
    int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    memcpy(cur, offsets, sizeof(int32_t) * (size_t)cap);
    for (int64_t i = 0; i < n; ++i) perm[cur[G[i]]++] = (int32_t)i;
    free(cur);
    return 0;
}

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11 "Parallel random numbers:
 * as easy as 1, 2, 3"): ten rounds of two 64x64->128 multiplies with the
 * published multipliers and Weyl key increments. */
static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t h0, l0, h1, l1;
        mul128(0xD2E7470EE14C6C93ULL, x0, &h0, &l0);
        mul128(0xCA5A826395121157ULL, x2, &h1, &l1);
        uint64_t n0 = h1 ^ x1 ^ k0, n1 = l1, n2 = h0 ^ x3 ^ k1, n3 = l0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1) from a 64-bit draw: the top 23 bits as an odd multiple of
 * 2^-24, u = (2 (o >> 41) + 1) 2^-24, exactly representable in FP32. */
double orc_uniform(uint64_t o) { return (double)(2 * (o >> 41) + 1) * (1.0 / 16777216.0); }

/* The 56 standard normals of a mutation at cell i, step s: Philox blocks at
 * counter (i, s, 1+b, 0), b = 0..13; Box-Muller on (o0,o1) -> z[4b], z[4b+1]
 * and (o2,o3) -> z[4b+2], z[4b+3]: z = sqrt(-2 ln u1) (cos, sin)(2 pi u2). */
void orc_mutation_normals(uint64_t seed, uint64_t i, uint64_t s, double* z) {
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t key[2] = {seed, 0};
    for (int b = 0; b < 14; ++b) {
        uint64_t ctr[4] = {i, s, (uint64_t)(1 + b), 0}, o[4];
        orc_philox4x64_10(ctr, key, o);
        for (int h = 0; h < 2; ++h) {
            double u1 = orc_uniform(o[2 * h]), u2 = orc_uniform(o[2 * h + 1]);
            double rr = sqrt(-2.0 * log(u1));
            z[4 * b + 2 * h] = rr * cos(two_pi * u2);
            z[4 * b + 2 * h + 1] = rr * sin(two_pi * u2);
        }
    }
}

/* Hit threshold: a cell is hit when its draw is below floor(rate 2^64). */
uint64_t orc_hit_threshold(double rate) {
    if (!(rate > 0.0)) return 0;
    if (rate >= 1.0) return UINT64_MAX;
    return (uint64_t)floor(rate * 18446744073709551616.0);
}

/* Radiation (Fig. 1 C) applied after step s: the Philox block at counter
 * (floor(i / 4), s, 0, 0), key (seed, 0), gives cells 4k..4k+3 its four words;
 * cell i is hit when word i mod 4 is below T.  Free slots
 * are the slot ids with zero count in G (ascending); the k-th hit in
 * ascending i takes free slot k, gets its parent's CPPN parameters plus
 * sigma * z, and G[i] becomes that slot; hits beyond the free slots are
 * dropped.  params is cap x 56 (FP64), in/out.  hit_cells / hit_slots
 * (nullable, capacity max_hits) list the hits in order (slot -1 = dropped).
 * Returns the number of hits; *dropped counts the dropped ones. */
int64_t orc_radiate(int64_t n, int32_t* G, int32_t cap, double* params, uint64_t seed, uint64_t s,
                    uint64_t T, double sigma, int64_t* hit_cells, int32_t* hit_slots,
                    int64_t max_hits, int64_t* dropped) {
    int32_t* counts = (int32_t*)calloc((size_t)cap, sizeof(int32_t));
    int32_t* freel = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    for (int64_t i = 0; i < n; ++i) counts[G[i]]++;
    int32_t nfree = 0;
    for (int32_t g = 0; g < cap; ++g)
        if (counts[g] == 0) freel[nfree++] = g;
    uint64_t key[2] = {seed, 0};
    int64_t hits = 0;
    *dropped = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ctr[4] = {(uint64_t)(i / 4), s, 0, 0}, o[4];
        orc_philox4x64_10(ctr, key, o);
        if (!(o[i % 4] < T)) continue;
        int32_t slot = -1;
        if (hits < nfree) {
            slot = freel[hits];
            int32_t parent = G[i];
            double z[ORC_NPARAM];
            orc_mutation_normals(seed, (uint64_t)i, s, z);
            for (int m = 0; m < ORC_NPARAM; ++m)
                params[(int64_t)slot * ORC_NPARAM + m] =
                    params[(int64_t)parent * ORC_NPARAM + m] + sigma * z[m];
            G[i] = slot;
        } else {
            (*dropped)++;
        }
        if (hit_cells && hits < max_hits) {
            hit_cells[hits] = i;
            hit_slots[hits] = slot;
        }
        hits++;
    }
    free(counts);
    free(freel);
    return hits;
}

/* Merging (abstract: survival, merging and mutation; System Design: NEAT's
 * crossover operator applied through the physics), after step s.  A cell is
 * a merge candidate when word i mod 4 of the Philox block at counter
 * (floor(i / 4), s, 0, 1), key (seed, 0), is below T; its partner is the
 * neighbour it faces (direction R[i]).  The merge takes place when the two
 * cells hold different genomes in the map as it was before the call (G0).
 * The k-th merge in ascending i takes the k-th free slot (zero count in G0,
 * ascending) and becomes the crossover of its own genome a = G0[i] and its
 * partner's b = G0[partner]: every CPPN here has the same genes, so all
 * genes match and gene m is inherited from b when bit m of word 0 of the
 * Philox block (i, s, 0, 2) is set, from a otherwise.  G[i] becomes the new
 * slot; merges beyond the free slots are dropped.  hit_* (nullable,
 * capacity max_hits) list the merges in order: cell, new slot (-1 when
 * dropped), a, b.  Returns the number of merges; *dropped counts the
 * dropped ones. */
int64_t orc_merge(const orc_desc* d, int32_t* G, const uint8_t* R, int32_t cap, double* params,
                  uint64_t seed, uint64_t s, uint64_t T, int64_t* hit_cells, int32_t* hit_slots,
                  int32_t* hit_a, int32_t* hit_b, int64_t max_hits, int64_t* dropped) {
    const int64_t n = (int64_t)d->width * d->height;
    int32_t* G0 = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* counts = (int32_t*)calloc((size_t)cap, sizeof(int32_t));
    int32_t* freel = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    memcpy(G0, G, sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) counts[G0[i]]++;
    int32_t nfree = 0;
    for (int32_t g = 0; g < cap; ++g)
        if (counts[g] == 0) freel[nfree++] = g;
    uint64_t key[2] = {seed, 0};
    int64_t merges = 0;
    *dropped = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ctr[4] = {(uint64_t)(i / 4), s, 0, 1}, o[4];
        orc_philox4x64_10(ctr, key, o);
        if (!(o[i % 4] < T)) continue;
        const int32_t a = G0[i], b = G0[nbr(d, i, R[i] & 7)];
        if (a == b) continue;
        int32_t slot = -1;
        if (merges < nfree) {
            slot = freel[merges];
            uint64_t mc[4] = {(uint64_t)i, s, 0, 2}, mo[4];
            orc_philox4x64_10(mc, key, mo);
            for (int m = 0; m < ORC_NPARAM; ++m) {
                const int32_t src = ((mo[0] >> m) & 1) ? b : a;
                params[(int64_t)slot * ORC_NPARAM + m] = params[(int64_t)src * ORC_NPARAM + m];
            }
            G[i] = slot;
        } else {
            (*dropped)++;
        }
        if (hit_cells && merges < max_hits) {
            hit_cells[merges] = i;
            hit_slots[merges] = slot;
            hit_a[merges] = a;
            hit_b[merges] = b;
        }
        merges++;
    }
    free(G0);
    free(counts);
    free(freel);
    return merges;
}

/* Box-Muller normals from Philox blocks (i, s, third0 + b, 0), b = 0, 1, ...:
 * four normals per block, as in orc_mutation_normals. */
static void normals_from(uint64_t seed, uint64_t i, uint64_t s, uint64_t third0, int nz, double* z) {
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t key[2] = {seed, 0};
    for (int b = 0; 4 * b < nz; ++b) {
        uint64_t ctr[4] = {i, s, third0 + (uint64_t)b, 0}, o[4];
        orc_philox4x64_10(ctr, key, o);
        for (int h = 0; h < 2; ++h) {
            double u1 = orc_uniform(o[2 * h]), u2 = orc_uniform(o[2 * h + 1]);
            double rr = sqrt(-2.0 * log(u1));
            if (4 * b + 2 * h < nz) z[4 * b + 2 * h] = rr * cos(two_pi * u2);
            if (4 * b + 2 * h + 1 < nz) z[4 * b + 2 * h + 1] = rr * sin(two_pi * u2);
        }
    }
}

/* The 42 weights of the structural genes in one array: conn_w, node_in,
 * node_out. */
static double* ext_weight(orc_ext* e, int m) {
    return m < 10 ? &e->conn_w[m] : (m < 26 ? &e->node_in[m - 10] : &e->node_out[m - 26]);
}

/* Radiation with NEAT's structural mutations (System Design: NEAT's
 * mutation operator).  The hits, slots and base-gene mutation are those of
 * orc_radiate.  The weights of the child's enabled structural genes get
 * sigma * N(0,1) as well, normal m (of the 42 weights in ext_weight order)
 * from the Philox blocks (i, s, 16 + b, 0), b = 0..10; disabled genes keep
 * their stored weights.  Then the block (i, s, 15, 0) decides the
 * structural mutations: word 0 below Tc adds the direct connection
 * c = (word 2 & 0xffff) mod 10 with weight sigma times its normal; word 1
 * below Tn adds the node (word 2 >> 16 & 0xffff) mod 16 with activation
 * word 3 & 3, in weight 1 and out weight the child's B[o][j], which it
 * replaces.  Adding a gene that is already there changes nothing.  ext is
 * cap entries, in/out. */
int64_t orc_radiate_x(int64_t n, int32_t* G, int32_t cap, double* params, orc_ext* ext, uint64_t seed,
                      uint64_t s, uint64_t T, double sigma, uint64_t Tc, uint64_t Tn, int64_t* hit_cells,
                      int32_t* hit_slots, int64_t max_hits, int64_t* dropped) {
    int32_t* counts = (int32_t*)calloc((size_t)cap, sizeof(int32_t));
    int32_t* freel = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    for (int64_t i = 0; i < n; ++i) counts[G[i]]++;
    int32_t nfree = 0;
    for (int32_t g = 0; g < cap; ++g)
        if (counts[g] == 0) freel[nfree++] = g;
    uint64_t key[2] = {seed, 0};
    int64_t hits = 0;
    *dropped = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ctr[4] = {(uint64_t)(i / 4), s, 0, 0}, o[4];
        orc_philox4x64_10(ctr, key, o);
        if (!(o[i % 4] < T)) continue;
        int32_t slot = -1;
        if (hits < nfree) {
            slot = freel[hits];
            const int32_t parent = G[i];
            double z[ORC_NPARAM], zx[42];
            orc_mutation_normals(seed, (uint64_t)i, s, z);
            double* c = params + (int64_t)slot * ORC_NPARAM;
            for (int m = 0; m < ORC_NPARAM; ++m) c[m] = params[(int64_t)parent * ORC_NPARAM + m] + sigma * z[m];
            orc_ext e = ext[parent];
            normals_from(seed, (uint64_t)i, s, 16, 42, zx);
            for (int m = 0; m < 42; ++m) {
                const int on = m < 10 ? (int)((e.conn_mask >> m) & 1u)
                                      : (int)((e.node_mask >> (m < 26 ? m - 10 : m - 26)) & 1u);
                if (on) *ext_weight(&e, m) += sigma * zx[m];
            }
            uint64_t sc[4] = {(uint64_t)i, s, 15, 0}, so[4];
            orc_philox4x64_10(sc, key, so);
            if (so[0] < Tc) {
                const int cc = (int)((so[2] & 0xffff) % 10);
                if (!((e.conn_mask >> cc) & 1u)) {
                    e.conn_mask |= 1u << cc;
                    e.conn_w[cc] = sigma * zx[cc];
                }
            }
            if (so[1] < Tn) {
                const int k = (int)(((so[2] >> 16) & 0xffff) % 16);
                if (!((e.node_mask >> k) & 1u)) {
                    const int j = k >> 1, oo = k & 1;
                    e.node_mask |= 1u << k;
                    e.node_act = (e.node_act & ~(3u << (2 * k))) | ((uint32_t)(so[3] & 3) << (2 * k));
                    e.node_in[k] = 1.0;
                    e.node_out[k] = c[40 + oo * 8 + j];
                }
            }
            ext[slot] = e;
            G[i] = slot;
        } else {
            (*dropped)++;
        }
        if (hit_cells && hits < max_hits) {
            hit_cells[hits] = i;
            hit_slots[hits] = slot;
        }
        hits++;
    }
    free(counts);
    free(freel);
    return hits;
}

/* orc_merge with structural genes: the base genes as in orc_merge (word 0
 * of the block (i, s, 0, 2)); every structural gene position is taken whole
 * (enabled state, weights, activation) from b where bit c of word 1 (direct
 * connection c) or bit k of word 2 (added node k) is set, from a otherwise.
 * A gene both parents hold is so inherited from either with probability
 * 1/2, and a gene only one holds is kept with probability 1/2: NEAT's
 * crossover between parents of equal fitness (the ecosystem assigns none). */
int64_t orc_merge_x(const orc_desc* d, int32_t* G, const uint8_t* R, int32_t cap, double* params, orc_ext* ext,
                    uint64_t seed, uint64_t s, uint64_t T, int64_t* hit_cells, int32_t* hit_slots,
                    int32_t* hit_a, int32_t* hit_b, int64_t max_hits, int64_t* dropped) {
    const int64_t n = (int64_t)d->width * d->height;
    int32_t* G0 = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    memcpy(G0, G, sizeof(int32_t) * (size_t)n);
    const int64_t merges = orc_merge(d, G, R, cap, params, seed, s, T, hit_cells, hit_slots, hit_a, hit_b,
                                     max_hits, dropped);
    /* orc_merge listed the merges in cell order; replay their structural genes */
    uint64_t key[2] = {seed, 0};
    int64_t k = 0;
    for (int64_t i = 0; i < n && k < merges; ++i) {
        uint64_t ctr[4] = {(uint64_t)(i / 4), s, 0, 1}, o[4];
        orc_philox4x64_10(ctr, key, o);
        if (!(o[i % 4] < T)) continue;
        const int32_t a = G0[i], b = G0[nbr(d, i, R[i] & 7)];
        if (a == b) continue;
        const int32_t slot = G[i] != a ? G[i] : -1;
        if (slot >= 0) {
            uint64_t mc[4] = {(uint64_t)i, s, 0, 2}, mo[4];
            orc_philox4x64_10(mc, key, mo);
            orc_ext e;
            memset(&e, 0, sizeof e);
            for (int c = 0; c < 10; ++c) {
                const orc_ext* src = ((mo[1] >> c) & 1) ? &ext[b] : &ext[a];
                e.conn_mask |= src->conn_mask & (1u << c);
                e.conn_w[c] = src->conn_w[c];
            }
            for (int q = 0; q < 16; ++q) {
                const orc_ext* src = ((mo[2] >> q) & 1) ? &ext[b] : &ext[a];
                e.node_mask |= src->node_mask & (1u << q);
                e.node_act |= src->node_act & (3u << (2 * q));
                e.node_in[q] = src->node_in[q];
                e.node_out[q] = src->node_out[q];
            }
            ext[slot] = e;
        }
        ++k;
    }
    free(G0);
    return merges;
}

/* NEAT's compatibility distance with structural genes: genes are listed by
 * innovation number (base 0..55, always present; direct connection c at
 * 56 + c; added node k's in and out connections at 66 + 2k, 67 + 2k, present
 * while enabled).  Matching genes are those both genomes hold; of the
 * others, those beyond the smaller of the two genomes' highest innovation
 * numbers are excess (E), the rest disjoint (D); W is the mean absolute
 * weight difference of the matching genes and N the larger genome's gene
 * count: c1 E / N + c2 D / N + c3 W. */
double orc_genetic_distance_x(const double* pa, const orc_ext* ea, const double* pb, const orc_ext* eb,
                              double c1, double c2, double c3) {
    double wa[98], wb[98];
    int ha[98], hb[98];
    for (int m = 0; m < 56; ++m) { wa[m] = pa[m]; wb[m] = pb[m]; ha[m] = hb[m] = 1; }
    for (int c = 0; c < 10; ++c) {
        wa[56 + c] = ea->conn_w[c]; wb[56 + c] = eb->conn_w[c];
        ha[56 + c] = (ea->conn_mask >> c) & 1u; hb[56 + c] = (eb->conn_mask >> c) & 1u;
    }
    for (int q = 0; q < 16; ++q) {
        wa[66 + 2 * q] = ea->node_in[q]; wa[67 + 2 * q] = ea->node_out[q];
        wb[66 + 2 * q] = eb->node_in[q]; wb[67 + 2 * q] = eb->node_out[q];
        ha[66 + 2 * q] = ha[67 + 2 * q] = (ea->node_mask >> q) & 1u;
        hb[66 + 2 * q] = hb[67 + 2 * q] = (eb->node_mask >> q) & 1u;
    }
    int maxa = 0, maxb = 0, na = 0, nb = 0, match = 0;
    for (int g = 0; g < 98; ++g) {
        if (ha[g]) { maxa = g; ++na; }
        if (hb[g]) { maxb = g; ++nb; }
    }
    const int lim = maxa < maxb ? maxa : maxb;
    double w = 0.0;
    int E = 0, D = 0;
    for (int g = 0; g < 98; ++g) {
        if (ha[g] && hb[g]) { w += fabs(wa[g] - wb[g]); ++match; }
        else if (ha[g] || hb[g]) { if (g > lim) ++E; else ++D; }
    }
    const double N = (double)(na > nb ? na : nb);
    return c1 * E / N + c2 * D / N + c3 * (w / match);
}

/* Exact and FP64 total mass sum(E + I). */
int64_t orc_mass(int64_t n, const int64_t* E, const int64_t* I) {
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) s += E[i] + I[i];
    return s;
}
