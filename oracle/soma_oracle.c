/*
 * soma_oracle.c -- CPU reference of the single-chain-in-mean-field (SCMF)
 * Monte-Carlo sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent, plain and slow
 * oracle that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never links, imports or calls it, and it shares no code,
 * header, table or helper with the GPU library.
 *
 * What it follows
 *   Sec. 2 (Overview, SOMA paragraph): SOMA propagates a soft, coarse-grained
 *     polymer model with the SCMF algorithm; non-bonded interactions act
 *     through quasi-instantaneous fields, so chains move independently while
 *     the fields stay frozen.
 *   Sec. 2.2 (SOMA Optimization): the two dominant kernels perform trial
 *     moves with energy evaluations, and rebuild the particle density
 *     fields; bead coordinates are generated at initialisation.
 *   The paper gives no formulas for the model.  The readings used here are:
 *     bonds      harmonic, E_b/kT = (k/2) sum |r_{i+1}-r_i|^2, k = 3(N-1)/Re^2
 *     H_nb/kT    (rho0 dV / N) sum_cells f(phiA, phiB) with
 *                Helfand form  f = (kN/2)(phiA+phiB-1)^2 - (chiN/4)(phiA-phiB)^2
 *                or            f = chiN phiA phiB + (kN/2)(phiA+phiB-1)^2
 *     phi_t      n_t(c) * M / B (mean of phiA+phiB is one)
 *     omega_t    dH_nb/dn_t(c)
 *     moves      uniform in a cube of half-width delta, Metropolis, even
 *                beads first, then odd beads, fields frozen for the sweep;
 *                or, when smc_A > 0, bond-force-biased ("smart") moves
 *                (Sec. 2 names them as SOMA's move; Rossky, Doll and
 *                Friedman, J. Chem. Phys. 69, 4628 (1978)): displacement
 *                A F + sqrt(2A) xi with F the bond force and xi standard
 *                normal, accepted with the Metropolis-Hastings ratio of the
 *                Gaussian proposal densities
 *     density    nearest-grid-point, cell = floor(x / cell edge) mod n, the
 *                quotient exact, with the cell edge box/grid rounded to FP32
 *     RNG        Philox4x32-10 keyed by (seed) with counter
 *                (bead, chain, sweep, system)
 *
 * Position modes
 *   0  FP64 positions (reference for observables and precision errors)
 *   1  positions stored as FP32; all energies in FP64
 *   2  positions stored as int32 cell + FP32 offset: a new position in
 *      [0, cell edge), after trial moves anywhere in [-edge, 2 edge) (a cell
 *      step only when the offset leaves that window); all energies in FP64
 * Modes 1 and 2 reproduce the storage rounding of the GPU representation so
 * that single-sweep decisions and density histograms can be compared one by
 * one; they take every rounding step explicitly with C float arithmetic.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 * No function here is parity-unpinned; the pins live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random       */
/* numbers: as easy as 1, 2, 3").  Four 32-bit counter words, two key words, */
/* ten rounds; the key is bumped by the Weyl constants between rounds.       */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* System description                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_chains;
    int32_t N;
    int32_t n_chains_a;       /* chains [0, n_chains_a) use pattern_a */
    int32_t ham_form;         /* 0 Helfand, 1 chiN phiA phiB */
    const uint8_t *pattern_a; /* [N]: 0 = A, 1 = B */
    const uint8_t *pattern_b; /* [N] */
    double chiN, kappaN, Re;
    double box[3];
    int32_t grid[3];
    double move_halfwidth;
    uint32_t sys_id;
    double smc_A;             /* > 0: smart moves with this A (Re^2); 0: uniform moves */
    double umb_lambda;        /* umbrella strength lambda (kT); 0: no umbrella */
    const double *umb_target; /* [2][M] target phi_A, phi_B (umbrella and placement) */
    int32_t wall[2];          /* walls at the z-cell faces wall[0] < wall[1]; wall[1] == 0: none */
    int32_t zone[2];          /* z-cell widths of the conversion zones at the lower, upper wall */
} orc_system;

typedef struct {
    int32_t mode;    /* 0, 1 or 2 (see header) */
    double *x;       /* mode 0: [3][B] */
    float *xf;       /* mode 1: [3][B] */
    int32_t *cell;   /* mode 2: [3][B] */
    float *off;      /* mode 2: [3][B] */
    uint8_t *chain_class; /* [n_chains]: 0 = pattern_a, 1 = pattern_b; NULL: by n_chains_a */
    uint64_t conv[2];     /* chains converted to class a (lower zone) and to class b (upper zone) */
} orc_state;

static int64_t n_beads(const orc_system *s) { return (int64_t)s->n_chains * s->N; }
static int64_t n_cells(const orc_system *s) { return (int64_t)s->grid[0] * s->grid[1] * s->grid[2]; }

/* Chain class: which block pattern a chain carries.  Chains start as
 * [0, n_chains_a) -> a and the rest -> b; conversion zones change it. */
static int chain_class(const orc_system *s, const orc_state *st, int64_t chain)
{
    if (st && st->chain_class) return st->chain_class[chain];
    return chain < s->n_chains_a ? 0 : 1;
}

static int bead_type(const orc_system *s, const orc_state *st, int64_t chain, int i)
{
    return chain_class(s, st, chain) == 0 ? s->pattern_a[i] : s->pattern_b[i];
}

static int has_walls(const orc_system *s) { return s->wall[1] > s->wall[0]; }

static double cell_edge(const orc_system *s, int d) { return s->box[d] / (double)s->grid[d]; }

/* Spring constant in kT/Re^2: the Boltzmann weight of a harmonic bond with
 * k = 3(N-1)/Re^2 gives bond components N(0, Re^2/(3(N-1))), hence
 * <Re^2> = Re^2 for the ideal chain. */
static double spring_k(const orc_system *s) { return 3.0 * (double)(s->N - 1) / (s->Re * s->Re); }

/* ------------------------------------------------------------------------ */
/* Positions in FP64 from the stored representation                          */
/* ------------------------------------------------------------------------ */
static double get_pos(const orc_system *s, const orc_state *st, int d, int64_t b)
{
    int64_t B = n_beads(s);
    switch (st->mode) {
    case 0: return st->x[d * B + b];
    case 1: return (double)st->xf[d * B + b];
    default: {
        float edge = (float)cell_edge(s, d);
        return (double)st->cell[d * B + b] * (double)edge + (double)st->off[d * B + b];
    }
    }
}

/* Mode 2, canonical form of a new position: the offset in [0, edge), by
 * moving whole cells.  Every step is one FP32 rounding, and an offset that
 * rounds up to exactly one edge goes to offset 0 of the next cell. */
static void renorm_cell(int32_t *c, float *o, float edge)
{
    while (*o < 0.0f) { *o = *o + edge; *c -= 1; }
    while (*o >= edge) { *o = *o - edge; *c += 1; }
}

/* Mode 2, after a trial move (the paper does not describe the storage; this
 * is the representation's own rule): the offset may lie anywhere in the
 * window [-edge, 2 edge); an offset that
 * leaves it moves one whole cell, one FP32 rounding (a trial move is below
 * one edge, so one step brings it back).  The stored (cell, offset) pair
 * still names the same point c e + o. */
static void renorm_window(int32_t *c, float *o, float edge)
{
    if (*o < -edge) { *o = *o + edge; *c -= 1; }
    else if (*o >= 2.0f * edge) { *o = *o - edge; *c += 1; }
}

/* Mode 2: unwrapped NGP index along axis d of the stored pair: floor((c e + o) / e)
 * = c + floor(o / e) exactly, which for o in [-e, 2e) is c - 1, c or c + 1. */
static int64_t cell_index(int32_t c, float o, float edge)
{
    return (int64_t)c + (o >= edge ? 1 : 0) - (o < 0.0f ? 1 : 0);
}

/* Quantise FP64 positions into the state's representation. */
void orc_set_positions(const orc_system *s, orc_state *st, const double *xyz)
{
    int64_t B = n_beads(s);
    for (int d = 0; d < 3; ++d) {
        float edge = (float)cell_edge(s, d);
        for (int64_t b = 0; b < B; ++b) {
            double x = xyz[d * B + b];
            if (st->mode == 0) {
                st->x[d * B + b] = x;
            } else if (st->mode == 1) {
                st->xf[d * B + b] = (float)x;
            } else {
                double c = floor(x / (double)edge);
                int32_t ci = (int32_t)c;
                float o = (float)(x - c * (double)edge);
                renorm_cell(&ci, &o, edge);
                st->cell[d * B + b] = ci;
                st->off[d * B + b] = o;
            }
        }
    }
}

void orc_get_positions(const orc_system *s, const orc_state *st, double *xyz)
{
    int64_t B = n_beads(s);
    for (int d = 0; d < 3; ++d)
        for (int64_t b = 0; b < B; ++b)
            xyz[d * B + b] = get_pos(s, st, d, b);
}

/* ------------------------------------------------------------------------ */
/* Nearest-grid-point cell of a bead (unwrapped coordinates, periodic box)   */
/* ------------------------------------------------------------------------ */
static int64_t wrap_index(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* Unwrapped NGP index along axis d: the largest integer k with k * e <= x,
 * for the cell edge e = box/grid rounded to FP32 (the edge of the stored
 * representation, shared by every mode).  The FP64 quotient can round to
 * the wrong side of an integer, so k is checked with products k * e that
 * are exact in FP64 (|k| < 2^29 and e has a 24-bit significand). */
static int64_t ngp_index(const orc_system *s, int d, double x)
{
    double e = (double)(float)cell_edge(s, d);
    double k = floor(x / e);
    while (k * e > x) k -= 1.0;
    while ((k + 1.0) * e <= x) k += 1.0;
    return (int64_t)k;
}

static int64_t cell_of(const orc_system *s, const orc_state *st, int64_t b)
{
    int64_t B = n_beads(s);
    int64_t idx[3];
    for (int d = 0; d < 3; ++d) {
        int64_t i;
        if (st->mode == 2)
            i = cell_index(st->cell[d * B + b], st->off[d * B + b], (float)cell_edge(s, d));
        else
            i = ngp_index(s, d, get_pos(s, st, d, b));
        idx[d] = wrap_index(i, s->grid[d]);
    }
    return (idx[0] * s->grid[1] + idx[1]) * s->grid[2] + idx[2];
}

/* Density histogram: counts[t * M + cell] = number of type-t beads in cell. */
void orc_density(const orc_system *s, const orc_state *st, uint32_t *counts)
{
    int64_t M = n_cells(s);
    memset(counts, 0, sizeof(uint32_t) * 2 * (size_t)M);
    for (int64_t c = 0; c < s->n_chains; ++c)
        for (int i = 0; i < s->N; ++i) {
            int64_t b = c * s->N + i;
            counts[(int64_t)bead_type(s, st, c, i) * M + cell_of(s, st, b)] += 1u;
        }
}

/* ------------------------------------------------------------------------ */
/* Non-bonded free energy and the quasi-instantaneous fields                 */
/* ------------------------------------------------------------------------ */
static double f_nb(const orc_system *s, double pa, double pb)
{
    double inc = pa + pb - 1.0;
    if (s->ham_form == 1)
        return s->chiN * pa * pb + 0.5 * s->kappaN * inc * inc;
    return 0.5 * s->kappaN * inc * inc - 0.25 * s->chiN * (pa - pb) * (pa - pb);
}

/* Umbrella potential toward target concentration fields (Sec. 3.2,
 * "Coupling": placed molecules are equilibrated under an umbrella
 * potential).  Per cell (lambda/2) [(phiA - tA)^2 + (phiB - tB)^2], in the
 * same units as f_nb, so its field is lambda (phi_t - t_t) / N. */
static int has_umbrella(const orc_system *s) { return s->umb_lambda > 0.0 && s->umb_target != NULL; }

static double f_umb(const orc_system *s, int64_t c, double pa, double pb)
{
    int64_t M = n_cells(s);
    double da = pa - s->umb_target[c], db = pb - s->umb_target[M + c];
    return 0.5 * s->umb_lambda * (da * da + db * db);
}

/* H_nb / kT of the whole system from the counts. */
double orc_energy_nb(const orc_system *s, const uint32_t *counts)
{
    int64_t M = n_cells(s);
    double B = (double)n_beads(s);
    double phi_per_count = (double)M / B;
    double sum = 0.0, comp = 0.0;   /* Neumaier */
    for (int64_t c = 0; c < M; ++c) {
        double pa = counts[c] * phi_per_count, pb = counts[M + c] * phi_per_count;
        double v = f_nb(s, pa, pb);
        if (has_umbrella(s)) v += f_umb(s, c, pa, pb);
        double t = sum + v;
        if (fabs(sum) >= fabs(v)) comp += (sum - t) + v; else comp += (v - t) + sum;
        sum = t;
    }
    return (B / (double)M) / (double)s->N * (sum + comp);
}

/* omega[t * M + c] = dH/dn_t(c) in kT (non-bonded energy plus umbrella). */
void orc_fields(const orc_system *s, const uint32_t *counts, double *omega)
{
    int64_t M = n_cells(s);
    double phi_per_count = (double)M / (double)n_beads(s);
    for (int64_t c = 0; c < M; ++c) {
        double pa = counts[c] * phi_per_count, pb = counts[M + c] * phi_per_count;
        double inc = s->kappaN * (pa + pb - 1.0);
        double wa, wb;
        if (s->ham_form == 1) {
            wa = s->chiN * pb + inc;
            wb = s->chiN * pa + inc;
        } else {
            wa = inc - 0.5 * s->chiN * (pa - pb);
            wb = inc + 0.5 * s->chiN * (pa - pb);
        }
        if (has_umbrella(s)) {
            wa += s->umb_lambda * (pa - s->umb_target[c]);
            wb += s->umb_lambda * (pb - s->umb_target[M + c]);
        }
        omega[c] = wa / (double)s->N;
        omega[M + c] = wb / (double)s->N;
    }
}

/* ------------------------------------------------------------------------ */
/* Random numbers of one trial move                                          */
/* ------------------------------------------------------------------------ */
/* The top 24 bits of each word are used.  Words 0-2 give the displacement
 * d = fl32(delta * ((w >> 8) - 2^23) * 2^-23) in [-delta, delta), one FP32
 * multiply of exact operands; word 3 gives u = (w >> 8) * 2^-24 in [0, 1). */
static void move_draw(const orc_system *s, uint64_t seed, uint32_t sweep, int64_t chain, int i,
                      float d[3], double *u)
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)chain, sweep, s->sys_id};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    float delta = (float)s->move_halfwidth;
    for (int k = 0; k < 3; ++k) {
        float t = (float)((int32_t)(w[k] >> 8) - 8388608) * 0x1p-23f;
        d[k] = delta * t;
    }
    *u = (double)((float)(w[3] >> 8) * 0x1p-24f);
}

/* Random numbers of one smart move: three standard normals by Box-Muller on
 * the block with counter (bead, chain, sweep, system) -- words 0 and 1 give
 * the first two, words 2 and 3 the third -- and the acceptance variate from
 * word 0 of the block with counter (bead + 256, chain, sweep, system).  Beads
 * are numbered below 128, so the second block never meets a first one.
 * The uniforms of Box-Muller are ((w >> 8) + 1/2) 2^-24 (never zero, for the
 * logarithm) and (w >> 8) 2^-24, as in the initial walks. */
void orc_smc_draw(uint64_t seed, uint32_t sweep, uint32_t chain, uint32_t i, uint32_t sys_id,
                  double xi[3], double *u)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {i, chain, sweep, sys_id};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u1 = ((double)(w[0] >> 8) + 0.5) * 0x1p-24;
    double u2 = (double)(w[1] >> 8) * 0x1p-24;
    double u3 = ((double)(w[2] >> 8) + 0.5) * 0x1p-24;
    double u4 = (double)(w[3] >> 8) * 0x1p-24;
    double rad1 = sqrt(-2.0 * log(u1)), rad2 = sqrt(-2.0 * log(u3));
    xi[0] = rad1 * cos(two_pi * u2);
    xi[1] = rad1 * sin(two_pi * u2);
    xi[2] = rad2 * cos(two_pi * u4);
    uint32_t ctr2[4] = {i + 256u, chain, sweep, sys_id};
    orc_philox4x32_10(ctr2, key, w);
    *u = (double)((float)(w[0] >> 8) * 0x1p-24f);
}

/* ------------------------------------------------------------------------ */
/* Boundary zones: molecular type conversion (Sec. 3.2, "Coupling")         */
/* ------------------------------------------------------------------------ */
static int has_zones(const orc_system *s) { return has_walls(s) && (s->zone[0] > 0 || s->zone[1] > 0); }

/* Unwrapped z cell of bead b in the stored representation. */
static int64_t z_cell(const orc_system *s, const orc_state *st, int64_t b)
{
    if (st->mode == 2)
        return cell_index(st->cell[2 * n_beads(s) + b], st->off[2 * n_beads(s) + b], (float)cell_edge(s, 2));
    return ngp_index(s, 2, get_pos(s, st, 2, b));
}

/* After the moves of a sweep, a chain whose binned centre -- the mean of its
 * beads' z-cell indexes -- lies in the lower conversion zone [wall[0],
 * wall[0] + zone[0]) becomes a chain of pattern a; in the upper zone
 * [wall[1] - zone[1], wall[1]) one of pattern b.  conv[] counts the
 * conversions (the particle flux through each boundary zone).  The sum of
 * integer indexes makes the decision exact. */
void orc_convert(const orc_system *s, orc_state *st)
{
    if (!st->chain_class) return;
    const int N = s->N;
    const int64_t lo = (int64_t)N * (s->wall[0] + s->zone[0]);
    const int64_t hi = (int64_t)N * (s->wall[1] - s->zone[1]);
    for (int64_t c = 0; c < s->n_chains; ++c) {
        int64_t sum = 0;
        for (int i = 0; i < N; ++i) sum += z_cell(s, st, c * N + i);
        if (s->zone[0] > 0 && sum < lo && st->chain_class[c] != 0) {
            st->chain_class[c] = 0;
            st->conv[0] += 1;
        } else if (s->zone[1] > 0 && sum >= hi && st->chain_class[c] != 1) {
            st->chain_class[c] = 1;
            st->conv[1] += 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* One MC sweep with frozen fields                                           */
/* ------------------------------------------------------------------------ */
/* omega: [2][M] fields, read only during the sweep.  accepted: optional
 * per-bead decisions (1 accepted, 0 rejected).  Returns accepted count.
 * With conversion zones the sweep ends with the conversion step. */
uint64_t orc_sweep(const orc_system *s, orc_state *st, uint64_t seed, uint32_t sweep,
                   const double *omega, uint8_t *accepted)
{
    const int64_t B = n_beads(s), M = n_cells(s);
    const int N = s->N;
    const double k = spring_k(s);
    uint64_t n_acc = 0;

    for (int parity = 0; parity < 2; ++parity) {
#pragma omp parallel for schedule(static) reduction(+ : n_acc)
        for (int64_t c = 0; c < s->n_chains; ++c) {
            for (int i = parity; i < N; i += 2) {
                int64_t b = c * N + i;
                float d[3];
                double u;
                /* smart move: bond force at the current position (the
                 * neighbours hold still during this bead's move) */
                double F[3] = {0.0, 0.0, 0.0};
                int n_nb = 0;
                int smart = s->smc_A > 0.0;
                if (smart) {
                    double xi[3];
                    orc_smc_draw(seed, sweep, (uint32_t)c, (uint32_t)i, s->sys_id, xi, &u);
                    double sum[3] = {0.0, 0.0, 0.0};
                    for (int side = -1; side <= 1; side += 2) {
                        int j = i + side;
                        if (j < 0 || j >= N) continue;
                        ++n_nb;
                        for (int a = 0; a < 3; ++a)
                            sum[a] += get_pos(s, st, a, c * N + j) - get_pos(s, st, a, b);
                    }
                    int inside = 1;
                    for (int a = 0; a < 3; ++a) {
                        F[a] = k * sum[a];
                        d[a] = (float)(s->smc_A * F[a] + sqrt(2.0 * s->smc_A) * xi[a]);
                        /* displacements of 0.99 cell edges or more are
                         * rejected outright: a condition symmetric in r and
                         * r', so the chain keeps detailed balance */
                        if (!(fabsf(d[a]) < (float)(0.99 * cell_edge(s, a)))) inside = 0;
                    }
                    if (!inside) {
                        if (accepted) accepted[b] = 0;
                        continue;
                    }
                } else {
                    move_draw(s, seed, sweep, c, i, d, &u);
                }

                /* Old and proposed position in FP64, proposed state stored
                 * in the mode's representation. */
                double r_old[3], r_new[3];
                float xf_new[3];
                int32_t c_new[3];
                float o_new[3];
                for (int a = 0; a < 3; ++a) {
                    r_old[a] = get_pos(s, st, a, b);
                    if (st->mode == 0) {
                        r_new[a] = r_old[a] + (double)d[a];
                    } else if (st->mode == 1) {
                        xf_new[a] = st->xf[a * B + b] + d[a];
                        r_new[a] = (double)xf_new[a];
                    } else {
                        float edge = (float)cell_edge(s, a);
                        c_new[a] = st->cell[a * B + b];
                        o_new[a] = st->off[a * B + b] + d[a];
                        renorm_window(&c_new[a], &o_new[a], edge);
                        r_new[a] = (double)c_new[a] * (double)edge + (double)o_new[a];
                    }
                }
                double de[3] = {r_new[0] - r_old[0], r_new[1] - r_old[1], r_new[2] - r_old[2]};

                /* Bond energy change in displacement form:
                 * (k/2) sum_j [ |r'-r_j|^2 - |r-r_j|^2 ] = (k/2) sum_j [2 d.(r-r_j) + |d|^2]. */
                double dE = 0.0;
                double dd = de[0] * de[0] + de[1] * de[1] + de[2] * de[2];
                for (int side = -1; side <= 1; side += 2) {
                    int j = i + side;
                    if (j < 0 || j >= N) continue;
                    int64_t bj = c * N + j;
                    double dot = 0.0;
                    for (int a = 0; a < 3; ++a)
                        dot += de[a] * (r_old[a] - get_pos(s, st, a, bj));
                    dE += 0.5 * k * (2.0 * dot + dd);
                }

                /* Field energy change: omega of the bead's type at the new
                 * cell minus at the old cell. */
                int t = bead_type(s, st, c, i);
                int64_t cell_old = cell_of(s, st, b);
                /* cell of the proposal: evaluate it through a temporary state */
                int64_t idx[3];
                int outside = 0;
                for (int a = 0; a < 3; ++a) {
                    int64_t ia;
                    if (st->mode == 2)
                        ia = cell_index(c_new[a], o_new[a], (float)cell_edge(s, a));
                    else
                        ia = ngp_index(s, a, r_new[a]);
                    /* walls (Sec. 3.2, wall confinement): a trial position whose
                     * z cell lies outside [wall[0], wall[1]) is rejected */
                    if (a == 2 && has_walls(s) && (ia < s->wall[0] || ia >= s->wall[1])) outside = 1;
                    idx[a] = wrap_index(ia, s->grid[a]);
                }
                int64_t cell_new = (idx[0] * s->grid[1] + idx[1]) * s->grid[2] + idx[2];
                dE += omega[(int64_t)t * M + cell_new] - omega[(int64_t)t * M + cell_old];
                if (smart) {
                    /* log of q(r'->r)/q(r->r') for the Gaussian proposal
                     * q(r->r') ~ exp(-|r'-r-A F(r)|^2/(4A)); F(r') = F(r) - k n_nb d */
                    double A = s->smc_A, fwd = 0.0, rev = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double f = de[a] - A * F[a];
                        double r = de[a] + A * (F[a] - k * (double)n_nb * de[a]);
                        fwd += f * f;
                        rev += r * r;
                    }
                    dE -= (fwd - rev) / (4.0 * A);
                }

                int acc = !outside && u < exp(-dE);
                if (accepted) accepted[b] = (uint8_t)acc;
                if (acc) {
                    n_acc += 1;
                    for (int a = 0; a < 3; ++a) {
                        if (st->mode == 0) {
                            st->x[a * B + b] = r_new[a];
                        } else if (st->mode == 1) {
                            st->xf[a * B + b] = xf_new[a];
                        } else {
                            st->cell[a * B + b] = c_new[a];
                            st->off[a * B + b] = o_new[a];
                        }
                    }
                }
            }
        }
    }
    if (has_zones(s)) orc_convert(s, st);
    return n_acc;
}

/* Full SCMF sweeps: moves with frozen fields, then the density histogram,
 * then the field refresh.  counts [2][M] and omega [2][M] must hold the
 * current state on entry and hold it again on return.  If refresh is zero
 * the fields stay frozen (external-field runs). */
uint64_t orc_run(const orc_system *s, orc_state *st, uint64_t seed, uint32_t first_sweep,
                 int32_t n_sweeps, uint32_t *counts, double *omega, int32_t refresh)
{
    uint64_t acc = 0;
    for (int32_t k = 0; k < n_sweeps; ++k) {
        acc += orc_sweep(s, st, seed, first_sweep + (uint32_t)k, omega, NULL);
        orc_density(s, st, counts);
        if (refresh) orc_fields(s, counts, omega);
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Initial configuration: Gaussian random walks                              */
/* ------------------------------------------------------------------------ */
/* Initial streams use counter word 3 = system id with the top bit set, so
 * they never meet a move draw; counter word 2 names the stream and the
 * attempt j (walls only): 4j initial walks, 4j + 1 placement targets,
 * 4j + 2 placement walks. */
static void init_block(const orc_system *s, uint64_t seed, uint32_t w0, uint32_t chain, uint32_t stream,
                       uint32_t w[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {w0, chain, stream, s->sys_id | 0x80000000u};
    orc_philox4x32_10(ctr, key, w);
}

static double top24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

/* One bond of a Gaussian walk: each component N(0, sigma^2) by Box-Muller
 * on words (0,1) and (2,3). */
static void gauss_bond(const uint32_t w[4], double sigma, double b[3])
{
    const double two_pi = 6.283185307179586476925286766559;
    double u1 = ((double)(w[0] >> 8) + 0.5) * 0x1p-24;
    double u2 = top24(w[1]);
    double u3 = ((double)(w[2] >> 8) + 0.5) * 0x1p-24;
    double u4 = top24(w[3]);
    double rad1 = sqrt(-2.0 * log(u1)), rad2 = sqrt(-2.0 * log(u3));
    b[0] = sigma * rad1 * cos(two_pi * u2);
    b[1] = sigma * rad1 * sin(two_pi * u2);
    b[2] = sigma * rad2 * cos(two_pi * u4);
}

#define ORC_MAX_ATTEMPTS 64

/* Walls: a generated chain is kept only if every bead's z lies in
 * [wall[0] e + e/128, wall[1] e - e/128] (e the FP32 cell edge): a margin of
 * 1/128 edge keeps the stored representation's z cell inside the walls
 * whatever the rounding (|z| < 2^15 edges).  Otherwise the chain is drawn
 * again from the next attempt's counters. */
static int chain_fits(const orc_system *s, const double *z, int N)
{
    if (!has_walls(s)) return 1;
    double e = (double)(float)cell_edge(s, 2);
    double lo = (double)s->wall[0] * e + e / 128.0, hi = (double)s->wall[1] * e - e / 128.0;
    for (int i = 0; i < N; ++i)
        if (!(z[i] >= lo && z[i] <= hi)) return 0;
    return 1;
}

/* Bead 0 uniform in the box (in z between the walls when there are walls)
 * from the top 24 bits of words 0-2; every bond component
 * N(0, Re^2/(3(N-1))).  Written in FP64.  Returns 0, or -2 when a chain did
 * not fit between the walls in ORC_MAX_ATTEMPTS attempts. */
int orc_init_walks(const orc_system *s, uint64_t seed, double *xyz)
{
    const int64_t B = n_beads(s);
    const int N = s->N;
    const double sigma = s->Re / sqrt(3.0 * (double)(N > 1 ? N - 1 : 1));
    double *r = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    int rc = 0;
    for (int64_t c = 0; c < s->n_chains && rc == 0; ++c) {
        int ok = 0;
        for (int j = 0; j < ORC_MAX_ATTEMPTS && !ok; ++j) {
            for (int i = 0; i < N; ++i) {
                uint32_t w[4];
                init_block(s, seed, (uint32_t)i, (uint32_t)c, 4u * (uint32_t)j, w);
                if (i == 0) {
                    for (int a = 0; a < 3; ++a) r[a * N] = s->box[a] * top24(w[a]);
                    if (has_walls(s)) {
                        double e = (double)(float)cell_edge(s, 2);
                        double lo = (double)s->wall[0] * e, hi = (double)s->wall[1] * e;
                        r[2 * N] = lo + (hi - lo) * top24(w[2]);
                    }
                } else {
                    double b[3];
                    gauss_bond(w, sigma, b);
                    for (int a = 0; a < 3; ++a) r[a * N + i] = r[a * N + i - 1] + b[a];
                }
            }
            ok = chain_fits(s, r + 2 * N, N);
        }
        if (!ok) rc = -2;
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < N; ++i) xyz[a * B + c * N + i] = r[a * N + i];
    }
    free(r);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Placement from target concentration fields (Sec. 3.2, "Coupling")        */
/* ------------------------------------------------------------------------ */
/* Every molecule starts with its centre of mass at most Re/2 (half the
 * ideal end-to-end distance) from a target position drawn from the supplied
 * concentration fields:
 *   1. chains of class k (pattern a or b, with A fraction f_k) draw a target
 *      cell with probability proportional to the integer weight
 *      w_k(c) = floor(2^20 (f_k tA(c) + (1 - f_k) tB(c)) + 1/2), through the
 *      exact inclusive prefix sum W_k: the cell is the first c with
 *      W_k(c) > t, t = floor(v T_k / 2^64), v the 64-bit word (w0 << 32 | w1)
 *      of block (0, chain, 4j + 1) and T_k the total weight;
 *   2. the target point is uniform in that cell (words w2, w3 of that block
 *      and w0 of block (1, chain, 4j + 1));
 *   3. the chain's centre of mass goes uniformly into the ball of radius
 *      Re/2 around it: radius (Re/2) cbrt(u1), cos(theta) = 2 u2 - 1,
 *      azimuth 2 pi u3 (words w1-w3 of block (1, chain, 4j + 1));
 *   4. the conformation is a Gaussian walk (bonds from blocks
 *      (i, chain, 4j + 2)), shifted to that centre.
 * t_k = umb_target ([2][M]).  targets (or NULL): [3][n_chains] target points;
 * cells (or NULL): [n_chains] target cells.  Returns 0, -1 for a negative
 * or non-finite target or a class with zero total weight, -2 when a chain
 * did not fit between the walls in ORC_MAX_ATTEMPTS attempts. */
int orc_place_from_fields(const orc_system *s, const orc_state *st, uint64_t seed, double *xyz, double *targets,
                          int64_t *cells)
{
    const int64_t B = n_beads(s), M = n_cells(s);
    const int N = s->N;
    const double sigma = s->Re / sqrt(3.0 * (double)(N > 1 ? N - 1 : 1));
    const double two_pi = 6.283185307179586476925286766559;
    if (!s->umb_target) return -1;
    for (int64_t c = 0; c < 2 * M; ++c)
        if (!(s->umb_target[c] >= 0.0 && s->umb_target[c] <= 4096.0)) return -1;
    uint64_t *W = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)M);
    double *r = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    for (int k = 0; k < 2; ++k) {
        const uint8_t *pat = k == 0 ? s->pattern_a : s->pattern_b;
        int na = 0;
        for (int i = 0; i < N; ++i) na += pat[i] == 0;
        double fa = (double)na / (double)N, fb = (double)(N - na) / (double)N;
        uint64_t run = 0;
        for (int64_t c = 0; c < M; ++c) {
            double v = fa * s->umb_target[c] + fb * s->umb_target[M + c];
            run += (uint64_t)floor(1048576.0 * v + 0.5);
            W[k * M + c] = run;
        }
    }
    int rc = 0;
    for (int64_t ch = 0; ch < s->n_chains && rc == 0; ++ch) {
        const int k = chain_class(s, st, ch);
        const uint64_t *Wk = W + k * M;
        const uint64_t T = Wk[M - 1];
        if (T == 0) { rc = -1; break; }
        int ok = 0;
        double tp[3] = {0, 0, 0};
        int64_t cell = 0;
        for (int j = 0; j < ORC_MAX_ATTEMPTS && !ok; ++j) {
            uint32_t w[4], q[4];
            init_block(s, seed, 0u, (uint32_t)ch, 4u * (uint32_t)j + 1u, w);
            init_block(s, seed, 1u, (uint32_t)ch, 4u * (uint32_t)j + 1u, q);
            uint64_t v = ((uint64_t)w[0] << 32) | w[1];
            uint64_t t = (uint64_t)(((unsigned __int128)v * T) >> 64);
            int64_t lo = 0, hi = M - 1;          /* first c with Wk[c] > t */
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (Wk[mid] > t) hi = mid; else lo = mid + 1;
            }
            cell = lo;
            int64_t ix = cell / ((int64_t)s->grid[1] * s->grid[2]);
            int64_t iy = (cell / s->grid[2]) % s->grid[1];
            int64_t iz = cell % s->grid[2];
            double u3[3] = {top24(w[2]), top24(w[3]), top24(q[0])};
            int64_t ic[3] = {ix, iy, iz};
            for (int a = 0; a < 3; ++a) tp[a] = ((double)ic[a] + u3[a]) * cell_edge(s, a);
            double rad = 0.5 * s->Re * cbrt(top24(q[1]));
            double ct = 2.0 * top24(q[2]) - 1.0;
            double stt = sqrt(fmax(0.0, 1.0 - ct * ct));
            double ph = two_pi * top24(q[3]);
            double centre[3] = {tp[0] + rad * stt * cos(ph), tp[1] + rad * stt * sin(ph), tp[2] + rad * ct};
            double com[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a) r[a * N] = 0.0;
            for (int i = 1; i < N; ++i) {
                uint32_t g[4];
                double b[3];
                init_block(s, seed, (uint32_t)i, (uint32_t)ch, 4u * (uint32_t)j + 2u, g);
                gauss_bond(g, sigma, b);
                for (int a = 0; a < 3; ++a) r[a * N + i] = r[a * N + i - 1] + b[a];
            }
            for (int a = 0; a < 3; ++a) {
                for (int i = 0; i < N; ++i) com[a] += r[a * N + i];
                com[a] /= (double)N;
            }
            for (int a = 0; a < 3; ++a)
                for (int i = 0; i < N; ++i) r[a * N + i] = centre[a] + (r[a * N + i] - com[a]);
            ok = chain_fits(s, r + 2 * N, N);
        }
        if (!ok) { rc = -2; break; }
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < N; ++i) xyz[a * B + ch * N + i] = r[a * N + i];
        if (targets)
            for (int a = 0; a < 3; ++a) targets[a * s->n_chains + ch] = tp[a];
        if (cells) cells[ch] = cell;
    }
    free(W);
    free(r);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Observables (FP64, compensated sums)                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double Re2, Re2_err, Rg2, Rg2_err, Ebond_per_chain, Enb_per_chain;
} orc_obs;

typedef struct { double s, c; } nsum;
static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v; else a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_val(const nsum *a) { return a->s + a->c; }

/* Neumaier's improved Kahan summation, exposed for its own pin. */
double orc_neumaier_sum(const double *v, int64_t n)
{
    nsum a = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nsum_add(&a, v[i]);
    return nsum_val(&a);
}

/* Per-chain Re^2, Rg^2 and bond energy; per_chain may be NULL, else [3][n_chains]. */
void orc_observables(const orc_system *s, const orc_state *st, const uint32_t *counts,
                     orc_obs *out, double *per_chain)
{
    const int N = s->N;
    const double k = spring_k(s);
    nsum re = {0, 0}, re2 = {0, 0}, rg = {0, 0}, rg2 = {0, 0}, eb = {0, 0};
    for (int64_t c = 0; c < s->n_chains; ++c) {
        double r0[3], rl[3], cm[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
            r0[a] = get_pos(s, st, a, c * N);
            rl[a] = get_pos(s, st, a, c * N + N - 1);
        }
        double e2e = 0.0;
        for (int a = 0; a < 3; ++a) e2e += (rl[a] - r0[a]) * (rl[a] - r0[a]);
        for (int i = 0; i < N; ++i)
            for (int a = 0; a < 3; ++a) cm[a] += get_pos(s, st, a, c * N + i);
        for (int a = 0; a < 3; ++a) cm[a] /= (double)N;
        double g = 0.0, bond = 0.0;
        for (int i = 0; i < N; ++i)
            for (int a = 0; a < 3; ++a) {
                double v = get_pos(s, st, a, c * N + i) - cm[a];
                g += v * v;
                if (i + 1 < N) {
                    double bv = get_pos(s, st, a, c * N + i + 1) - get_pos(s, st, a, c * N + i);
                    bond += bv * bv;
                }
            }
        g /= (double)N;
        bond *= 0.5 * k;
        nsum_add(&re, e2e); nsum_add(&re2, e2e * e2e);
        nsum_add(&rg, g); nsum_add(&rg2, g * g);
        nsum_add(&eb, bond);
        if (per_chain) {
            per_chain[c] = e2e;
            per_chain[s->n_chains + c] = g;
            per_chain[2 * s->n_chains + c] = bond;
        }
    }
    double n = (double)s->n_chains;
    double mre = nsum_val(&re) / n, mrg = nsum_val(&rg) / n;
    double vre = nsum_val(&re2) / n - mre * mre, vrg = nsum_val(&rg2) / n - mrg * mrg;
    out->Re2 = mre;
    out->Re2_err = sqrt(fmax(vre, 0.0) / n);
    out->Rg2 = mrg;
    out->Rg2_err = sqrt(fmax(vrg, 0.0) / n);
    out->Ebond_per_chain = nsum_val(&eb) / n;
    out->Enb_per_chain = counts ? orc_energy_nb(s, counts) / n : 0.0;
}
