/*
 * soma.h -- C-ABI of the MI355X single-chain-in-mean-field (SCMF)
 * Monte-Carlo sweep library (libsoma_mi355x.so, HIP for gfx950).
 *
 * The method (Sec. 2, SOMA paragraph, and Sec. 2.2 of the paper): soft,
 * coarse-grained polymer chains are propagated by Monte-Carlo moves; the
 * non-bonded interactions act through quasi-instantaneous fields that stay
 * frozen while all chains move, so chains move independently.  One sweep is
 *   1. a Metropolis trial move of every bead (harmonic bonds plus the field
 *      of its type in its grid cell), even beads first, then odd beads;
 *   2. the nearest-grid-point (NGP) density histogram of every species;
 *   3. the field refresh from the new densities with chiN and kappaN.
 * The paper states the model in words only; the formulas used are:
 *   bonds    E_b/kT = (k/2) sum_i |r_{i+1} - r_i|^2, k = 3(N-1)/Re^2
 *   phi_t(c) = n_t(c) * M / B      (M cells, B beads of the system)
 *   Helfand  omega_A = [kN(phiA+phiB-1) - (chiN/2)(phiA-phiB)] / N,
 *            omega_B = [kN(phiA+phiB-1) + (chiN/2)(phiA-phiB)] / N
 *   chi-AB   omega_A = [chiN phiB + kN(phiA+phiB-1)] / N, omega_B symmetric
 *   move     r' = r + d, d uniform in [-delta, delta)^3; accept iff
 *            u < exp(-dE) with u uniform in [0, 1); or, per system, the
 *            bond-force-biased move of SOMA (Sec. 2): d = A F + sqrt(2A) xi,
 *            accept iff u < exp(-dE) q(r'->r) / q(r->r') with
 *            q(r->r') ~ exp(-|r'-r-A F(r)|^2 / (4A)) (see smc_A)
 *   RNG      Philox4x32-10, key = seed, counter = (bead, chain, sweep, system)
 *   NGP      cell = floor(x / edge) mod n (unwrapped x, periodic box);
 *            linear cell index (ix * ny + iy) * nz + iz
 *
 * Conventions for every call
 *   - Every call returns an int status (soma_status); no exception or abort
 *     crosses the ABI.  soma_last_error() gives text for the last failure.
 *   - Host pointers are read or written before the call returns unless the
 *     call says otherwise.  Device pointers must be in the device memory of
 *     the context's GPU.
 *   - Work is enqueued on the HIP stream given at creation.  Calls that
 *     return data to the host synchronise that stream.
 *   - Device-side failures (count overflow, cell index overflow, an
 *     internal consistency check) are latched in a status word and reported by the next
 *     synchronising call; after that the context only accepts
 *     soma_destroy and returns SOMA_ESTATE otherwise.
 *   - One context per stream; calls on one context are not thread-safe.
 */
#ifndef SOMA_MI355X_H
#define SOMA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct soma_ctx soma_ctx;

typedef enum {
    SOMA_OK = 0,
    SOMA_EINVAL = -1,      /* invalid argument */
    SOMA_ENOMEM = -2,      /* workspace too small */
    SOMA_EDEVICE = -3,     /* HIP runtime error */
    SOMA_EOVERFLOW = -4,   /* a density count exceeded its width, or a cell index left int32 range */
    SOMA_ENONFINITE = -5,  /* a field value passed in is not finite */
    SOMA_ESTATE = -6       /* the context latched an earlier error */
} soma_status;

/* Position representations. */
enum {
    SOMA_POS_F32 = 0,      /* unwrapped FP32 coordinates, 12 B per bead */
    SOMA_POS_CELL_F32 = 1  /* int32 unwrapped cell + FP32 offset (in [-edge, 2 edge)), 24 B per bead */
};
/* Density count widths. */
enum {
    SOMA_COUNT_U16 = 0,    /* A and B counts packed as two uint16 in one uint32 per cell */
    SOMA_COUNT_U32 = 1     /* uint32 A and B counts, interleaved per cell */
};
/* Non-bonded functional. */
enum { SOMA_HAM_HELFAND = 0, SOMA_HAM_CHI_AB = 1 };

/* One independent system.  Chains [0, n_chains_a) carry the bead types of
 * pattern_a, chains [n_chains_a, n_chains) those of pattern_b (0 = A,
 * 1 = B): a diblock or triblock melt sets n_chains_a = n_chains, an A/B
 * homopolymer blend an all-A pattern_a and an all-B pattern_b.  A chain's
 * pattern is its class (a or b); boundary zones and soma_set_classes change
 * classes.
 * Limits: 2 <= N <= 128; 1 <= grid[d] <= 32768 with grid[0] * grid[1] <= 2^24;
 * move_halfwidth below 0.99 cell edges box[d]/grid[d]; smc_A zero, or
 * positive with sqrt(2 smc_A) at most half a cell edge.
 *
 * Walls and boundary zones (Sec. 3.2, "Coupling": the particle subdomain
 * holds the fluxes across its edges by confining beads with walls and by
 * changing the type of molecules in zones next to them): walls = {lo, hi} with 0 <= lo < hi <= grid[2] puts hard
 * walls at the z-cell faces lo and hi -- a trial move whose z cell leaves
 * [lo, hi) is rejected, and initial walks and placements draw chains again
 * until every bead lies between the walls (64 attempts, else SOMA_EINVAL);
 * {0, 0} means periodic z.  zones = {w_lo, w_hi} (cells, with walls only,
 * lo + w_lo <= hi - w_hi) are conversion zones at the walls: after the moves
 * of every sweep a chain whose mean z-cell index is below lo + w_lo becomes
 * class a, at or above hi - w_hi class b; soma_observables counts the
 * conversions (the molecular flux through each zone).  Systems with zones
 * need density mode 0 or 1 (a conversion changes a cell's species). */
typedef struct {
    int32_t n_chains;
    int32_t N;                 /* beads per chain */
    int32_t n_chains_a;
    int32_t ham_form;          /* SOMA_HAM_* */
    const uint8_t *pattern_a;  /* host, [N] */
    const uint8_t *pattern_b;  /* host, [N] */
    double chiN, kappaN;
    double Re;                 /* end-to-end distance of the ideal chain (length unit) */
    double box[3];             /* periodic box, Re units */
    int32_t grid[3];           /* cells per direction */
    double move_halfwidth;     /* delta, Re units */
    double smc_A;              /* 0: uniform trial moves in the cube of half-width delta.
                                  > 0: bond-force-biased ("smart") moves, Sec. 2: displacement
                                  A F + sqrt(2A) xi (F the bond force in kT/Re, xi standard
                                  normal), accepted with the Metropolis-Hastings ratio of the
                                  Gaussian proposal densities; a displacement of 0.99 cell edges
                                  or more is rejected.  Requires sqrt(2A) <= 0.5 cell edge. */
    int32_t walls[2];          /* z-cell faces of the walls {lo, hi}; {0, 0}: periodic z */
    int32_t zones[2];          /* widths in z cells of the conversion zones at the lower and upper wall */
} soma_system_desc;

typedef struct {
    uint64_t seed;             /* Philox key */
    int32_t pos_repr;          /* SOMA_POS_* */
    int32_t count_width;       /* SOMA_COUNT_* */
    int32_t use_graph;         /* nonzero: soma_mc_sweep replays a captured hipGraph per sweep count */
    int32_t density_mode;      /* how accepted cell changes reach the counts (merged per
                                  wave, then device atomics):
                                  0: -1/+1 on the old and new cell's words of a delta buffer,
                                     folded into the counts by a streaming kernel after each
                                     sweep;
                                  1: the same words, folded inside the next sweep's kernel,
                                     whose gathers then read base + previous delta (two base,
                                     three delta buffers);
                                  2: face fluxes (one word per crossed cell face, so a
                                     one-axis move costs one atomic instead of two), folded
                                     by a kernel that adds each cell's flux divergence;
                                  3: mirrored counts: a sweep gathers one of two identical
                                     count buffers and adds its -1/+1 words straight into the
                                     other, then a copy kernel makes them equal again (half
                                     the upkeep traffic of mode 0; packed 16-bit overflow is
                                     caught by an exact check of the total bead count after
                                     each batch of sweeps) */
    int32_t reorder_every;     /* >0: spatially sort chains every this many sweeps; 0: never */
    int32_t waves_per_block;   /* 1..16 waves per workgroup; 0: library default */
    int32_t waves_per_cu;      /* >0: sweep grid of this many waves per compute unit, each wave
                                  moving a contiguous range of tiles; 0: one tile per wave */
    int32_t sys_id_base;       /* system k draws with Philox counter word sys_id_base + k (< 2^31);
                                  a system run alone with sys_id_base = k repeats its batched run */
    int32_t launch_order;      /* 0: workgroups remapped so that each XCD gets a contiguous
                                  tile range; 1: tiles in launch order */
    void *hip_stream;          /* hipStream_t, NULL for the null stream */
    int32_t coupling;          /* nonzero: reserve workspace for target concentration fields
                                  (soma_place_from_fields, soma_set_umbrella): 8 B per cell
                                  plus 16 B per cell of the largest system */
    int32_t packed_tiles;      /* 0: G = floor(64/P) whole chains per wave (P = ceil(N/2) lanes
                                  per chain).
                                  1: each workgroup moves floor(64 W / P) whole chains packed
                                  over its W waves, so fewer lanes idle when 64 is not a
                                  multiple of P; chains spanning two waves exchange their
                                  boundary beads through LDS.  No conversion zones.
                                  2: stream tiles: a system's lanes in chain order, 62 owned
                                  lanes per wave, so chains cross wave boundaries and no lane
                                  idles but in a system's last wave; a wave also takes the
                                  lane before and the lane after its own (from a copy made
                                  before the sweep) and repeats the even move of the bead
                                  after its last lane (same decision as that bead's own
                                  wave).  Uniform moves without walls, zones, umbrella or
                                  caller-set classes (otherwise the sweep takes wave tiles).
                                  1 and 2 need waves_per_cu = 0. */
} soma_options;

typedef struct {
    double Re2, Re2_err;       /* mean |r_{N-1} - r_0|^2 over chains and its standard error */
    double Rg2, Rg2_err;       /* mean radius of gyration squared and its standard error */
    double Ebond_per_chain;    /* (k/2) sum |b|^2 per chain, kT */
    double Enb_per_chain;      /* H_nb/kT per chain from the current counts */
    double accept_ratio;       /* accepted / attempted moves of the sweeps run on this context
                                  (a resumed checkpoint counts from the resume) */
    uint64_t n_moves, n_accepted;
    uint64_t sweep;            /* sweeps done since creation */
    uint64_t converted_to_a;   /* chains converted to class a in the lower zone since creation */
    uint64_t converted_to_b;   /* chains converted to class b in the upper zone since creation */
} soma_obs;

typedef struct {
    int32_t n_systems;
    int32_t n_tiles;           /* wave tiles per sweep launch */
    int64_t n_beads;           /* sum over systems */
    int64_t n_cells;           /* sum over systems */
    uint64_t sweep;            /* sweeps done */
    int64_t bytes_per_sweep;   /* algorithmic HBM bytes of one sweep (positions, counts) */
    int32_t density_mode;      /* the variant in use */
    int32_t waves_per_block;   /* launch shape in use (see soma_autotune) */
    int32_t waves_per_cu;
    int32_t xcd_remap;
    int32_t packed_tiles;      /* tiling in use: 0 wave tiles, 1 block tiles, 2 stream tiles */
} soma_info;

/* Bytes of device workspace that soma_create needs for these systems. */
int soma_workspace_size(const soma_system_desc *sys, int32_t n_sys, const soma_options *opt,
                        size_t *bytes);

/* Create a context over caller-owned device memory `workspace` (at least
 * soma_workspace_size bytes, 256-byte aligned).  The library never frees
 * it; it must outlive the context.  Initialises every system with Gaussian
 * random walks (first bead uniform in the box, bond components
 * N(0, Re^2/(3(N-1))); the init stream of Sec. 2.2 moved to the GPU), then
 * builds the density and fields, so a sweep can follow.  Returns
 * SOMA_EINVAL for bad descriptors, SOMA_ENOMEM for a short workspace. */
int soma_create(const soma_system_desc *sys, int32_t n_sys, const soma_options *opt,
                void *workspace, size_t workspace_bytes, soma_ctx **out);

/* Release the context (not the workspace).  Synchronises its stream. */
int soma_destroy(soma_ctx *ctx);

/* Enqueue n_sweeps >= 0 full SCMF sweeps of every system.  Defined by the
 * paper's SOMA paragraph (Sec. 2: chains move independently by Monte-Carlo
 * under quasi-instantaneous fields frozen for the sweep) and by Sec. 2.2,
 * which names the two kernels of a time step: trial moves with energy
 * evaluation (mc_polymer_iteration) and the rebuild of the particle density
 * fields (update_density_fields).  One sweep here is: every bead makes one
 * trial move (even beads, then odd beads) against its bonds and the frozen
 * field of its type in its cell; the NGP counts are brought to the new
 * positions; the fields follow from the counts (formulas at the top).
 * Asynchronous on the context's stream; no host memory is touched.
 * Returns SOMA_EINVAL for n_sweeps < 0, SOMA_ESTATE after a latched error,
 * SOMA_EDEVICE if a launch fails.  Count overflow and cell-range errors
 * raised by the kernels are reported by the next synchronising call. */
int soma_mc_sweep(soma_ctx *ctx, int32_t n_sweeps);

/* Wait for the stream and report latched device errors. */
int soma_sync(soma_ctx *ctx);

/* Density counts of system `sys` after the last sweep: the particle
 * density fields that Sec. 2.2's update_density_fields kernel rebuilds each
 * step, here as exact nearest-grid-point bead counts per cell and species.
 * Layout uint32 [2][nx][ny][nz] (A then B), linear cell (ix*ny + iy)*nz + iz.
 * dst (2*nx*ny*nz words, owned by the caller) is device memory of the
 * context's GPU if dst_on_device, else host memory.  Synchronises the
 * stream and reports latched device errors (SOMA_EOVERFLOW, ...).
 * SOMA_EINVAL for a bad system index or a null dst. */
int soma_density(soma_ctx *ctx, int32_t sys, uint32_t *dst, int32_t dst_on_device);

/* Fields omega_A, omega_B of system `sys` in kT: the quasi-instantaneous
 * fields of the SCMF algorithm (Sec. 2, SOMA paragraph), through which the
 * non-bonded interactions act and which stay frozen during the next sweep;
 * computed from the current counts with chiN and kappaN (formulas at the
 * top), or the frozen array after soma_set_fields.  Layout float
 * [2][nx][ny][nz] (A then B); dst (caller-owned, 2*nx*ny*nz floats) is
 * device memory if dst_on_device, else host memory.  Synchronises; errors
 * as soma_density. */
int soma_fields(soma_ctx *ctx, int32_t sys, float *dst, int32_t dst_on_device);

/* FP64 observables of system `sys`: the validation quantities that Sec. 2.2
 * moved to the GPU (initialisation and validation went from 235 s to under
 * 2 s).  Per chain from the unwrapped positions: Re^2, Rg^2 and the bond
 * energy; H_nb per chain from the counts; the acceptance ratio of the moves
 * since creation (or the last soma_set_sweep).  Chain sums are Neumaier-
 * compensated FP64 block sums, the only FP64 arithmetic on the GPU; the
 * standard errors are sqrt(Var/n) over the n chains of the snapshot.
 * `out` is host memory owned by the caller.  Synchronises; SOMA_EINVAL for a
 * bad index or null out, latched device errors as soma_density. */
int soma_observables(soma_ctx *ctx, int32_t sys, soma_obs *out);

/* soma_observables for callers that cannot allocate memory -- code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc:
 * the same results, bit for bit, computed by the same kernels, with the
 * partial sums in a static device array of the library (1 MiB per GPU, held
 * until the process ends) instead of the context's workspace.  Makes no
 * device or host allocation.  Limit: ceil(n_chains/256) + ceil(n_cells/256)
 * <= 10922 for the system (SOMA_EINVAL beyond).  The context's device must
 * be current (SOMA_EINVAL otherwise).  Calls on one GPU share the array:
 * calls that overlap in time on one GPU (other threads, other streams) race
 * and must be serialised by the caller.  Synchronises the context's stream;
 * errors as soma_observables. */
int soma_observables_noalloc(soma_ctx *ctx, int32_t sys, soma_obs *out);

/* Unwrapped FP64 positions of system `sys` as host double [3][n_chains*N]
 * (chain-major, Re units).  Synchronises. */
int soma_get_positions(soma_ctx *ctx, int32_t sys, double *xyz);

/* Set the positions of system `sys` from host double [3][n_chains*N]
 * (finite, |x| < 2^22 cell edges; SOMA_EINVAL otherwise),
 * rounded to the context's representation (FP32: round to nearest; cell:
 * floor(x/edge) and the FP32 offset), then rebuild its density.  Leaves
 * the system's frozen/unfrozen field state as it was. */
int soma_set_positions(soma_ctx *ctx, int32_t sys, const double *xyz);

/* Raw stored state of system `sys`, for exact checkpoints.
 * SOMA_POS_F32: f32 = float [3][n_chains*N], cell = NULL.
 * SOMA_POS_CELL_F32: cell = int32 [3][n_chains*N], f32 = float offsets
 * [3][n_chains*N]; a bead sits at cell * edge + offset.  A new position
 * has its offset in [0, edge); a trial move keeps the offset anywhere in
 * [-edge, 2 edge) and steps the cell only when it leaves that window (so a
 * sweep rewrites few cell words); the NGP cell is floor(offset / edge) +
 * cell.  soma_set_state takes offsets in [-edge, 2 edge) (SOMA_EINVAL
 * otherwise).  Host memory.  soma_set_state rebuilds the density. */
int soma_get_state(soma_ctx *ctx, int32_t sys, float *f32, int32_t *cell);
int soma_set_state(soma_ctx *ctx, int32_t sys, const float *f32, const int32_t *cell);

/* Freeze the fields of system `sys` to host float [2][nx][ny][nz]: later
 * sweeps move against them and still rebuild the density, but never
 * refresh them.  Returns SOMA_ENONFINITE for a non-finite value. */
int soma_set_fields(soma_ctx *ctx, int32_t sys, const float *omega);

/* Return system `sys` to fields derived from its density each sweep. */
int soma_release_fields(soma_ctx *ctx, int32_t sys);

/* Place the chains of system `sys` so that they reproduce target
 * concentration fields, the start of a SOMA run in the coupled workflow
 * (Sec. 3.2, "Coupling": each molecule starts near a target position, at
 * most half the mean end-to-end distance away).  phi_target: host float
 * [2][nx][ny][nz] (phi_A then phi_B, each in [0, 4096]).  A chain of class k
 * (A fraction f_k of its pattern) draws a target cell with probability
 * proportional to the integer weight floor(2^20 (f_k phi_A + (1 - f_k) phi_B)
 * + 1/2) through an exact inverse prefix sum, a target point uniform in the
 * cell, its centre of mass uniform in the ball of radius Re/2 around that
 * point, and a Gaussian-walk conformation (Philox streams of the initial
 * configuration).  The targets stay on the device for soma_set_umbrella;
 * the density is rebuilt.  Needs opts.coupling.  SOMA_EINVAL for a bad
 * value, for a class with chains but zero total weight, or when chains do not
 * fit between the walls (which latches the context). */
int soma_place_from_fields(soma_ctx *ctx, int32_t sys, const float *phi_target);

/* Umbrella potential toward the target fields of soma_place_from_fields,
 * used to equilibrate the placed molecules (Sec. 3.2, "Coupling"): adds
 * (lambda/2) sum_cells sum_t (phi_t - target_t)^2, in the units of H_nb, to
 * the energy, so omega_t gains lambda (phi_t - target_t) / N.  lambda >= 0;
 * 0 switches it off.  Applies to fields derived from the counts (not to
 * frozen fields).  SOMA_EINVAL for a bad lambda or no stored target. */
int soma_set_umbrella(soma_ctx *ctx, int32_t sys, double lambda);

/* Chain classes of system `sys` in logical chain order (host uint8
 * [n_chains], 0 = pattern_a, 1 = pattern_b), for checkpoints of runs with
 * conversion zones.  soma_set_classes rebuilds the density and makes the
 * classes authoritative for the system. */
int soma_get_classes(soma_ctx *ctx, int32_t sys, uint8_t *cls);
int soma_set_classes(soma_ctx *ctx, int32_t sys, const uint8_t *cls);

/* Set the sweep counter (the Philox counter word of the next sweep) for a
 * resumed checkpoint, and rebuild every system's density for it. */
int soma_set_sweep(soma_ctx *ctx, uint64_t sweep);

int soma_get_info(soma_ctx *ctx, soma_info *out);

/* Launch-shape autotuning, the "adjusting launch configurations" step of
 * the SOMA optimisation (Sec. 2.2).  For every candidate shape -- waves per
 * workgroup in {1, 2, 4, 8, 16}; one tile per wave, a resident grid of 8 or
 * 32 waves per compute unit walking tile ranges, one block tile per
 * workgroup, or stream tiles (uniform moves without coupling only);
 * XCD-aware block order on or off; density mode 0, 1, 2 or 3 (not 2 with
 * conversion zones) -- times `trial_sweeps` sweeps (1..1000) after a
 * warm-up batch of as many; the four fastest are timed twice more, and the
 * one with the lowest median of its three times is kept for every later
 * sweep.  The trial sweeps are undone: positions, counts, acceptance
 * counters, the status word and the sweep counter are restored, so the
 * trajectory is exactly the one of an untuned context (launch shapes never
 * change results).  The choice is cached per process (see
 * soma_tune_cache_clear).  Synchronises; out may be NULL.  SOMA_EINVAL for a
 * bad trial count. */
typedef struct {
    int32_t waves_per_block;   /* chosen shape */
    int32_t waves_per_cu;      /* 0: one tile per wave */
    int32_t xcd_remap;
    int32_t density_mode;      /* chosen density update */
    int32_t n_candidates;
    double us_per_sweep;       /* trial time of the chosen shape (0 when from_cache) */
    double us_per_sweep_before;/* trial time of the shape in use at the call (0 when from_cache) */
    int32_t from_cache;        /* 1: the shape came from the process-wide cache, nothing was timed */
    int32_t packed_tiles;      /* chosen tiling (see soma_options.packed_tiles) */
} soma_tune;
int soma_autotune(soma_ctx *ctx, int32_t trial_sweeps, soma_tune *out);

/* Empty the process-wide autotune cache.  soma_autotune first looks up the
 * context's key -- representation, count width, move kinds, graph use,
 * reorder on/off, compute units, and buckets of the number of systems (1,
 * 2-16, 17-128, more), of the total bead count (powers of two) and of the
 * largest and the bead-weighted mean chain length (16, 32, 64, 128) -- and
 * applies a cached shape without timing; otherwise it tunes and stores the
 * result.  Thread-safe. */
void soma_tune_cache_clear(void);

/* Per-kernel durations, the launch-configuration evidence of Sec. 2.2's
 * profiling: runs n_sweeps (1..1000) real sweeps -- they advance the
 * trajectory exactly like soma_mc_sweep -- launched eagerly with HIP events
 * on the context's stream before and after each sweep kernel and after each
 * fold kernel, and reports the average durations.  Synchronises.
 * SOMA_EINVAL for a bad count or a null out. */
typedef struct {
    int32_t n_sweeps;
    int32_t density_mode;      /* the density update in use */
    double sweep_kernel_us;    /* k_sweep: moves and the density delta */
    double fold_kernel_us;     /* the fold after it (0 launches in density mode 1) */
    double sweep_us;           /* their sum */
} soma_ktimes;
int soma_time_kernels(soma_ctx *ctx, int32_t n_sweeps, soma_ktimes *out);

/* Text of the last error of ctx (or of the last failed soma_create when
 * ctx is NULL).  Valid until the next call on the context. */
const char *soma_last_error(const soma_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SOMA_MI355X_H */
