// soma_launch.hpp -- kernel argument blocks and launchers of libsoma_mi355x.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "soma_types.hpp"

namespace soma {

// Stream tiles: owned lanes per wave (lanes 1..62; lanes 0 and 63 hold the
// neighbouring stream lanes).
constexpr int kStreamLanes = 62;

struct SweepArgs {
    const DevSys *systems;
    const Tile *tiles;
    int n_tiles;
    const Tile *ptiles;            // block tiles (chains packed over the waves of a block)
    int n_ptiles;
    int packed;                    // 1: one block tile per block; 2: stream tiles, one per wave
                                   // (only with max_blocks == 0)
    int waves_per_block;
    int max_blocks;                // 0: one tile per wave; else the grid size (waves loop over tiles)
    int xcd_remap;
    const uint32_t *chain_id;      // logical chain id (within its system) per chain slot
    float *P0, *P1, *P2;           // coordinates (F32) or offsets (CELL)
    int *C0, *C1, *C2;             // cells (CELL only)
    uint32_t *base;                // two count buffers of count_words words each
    uint32_t *delta;               // three delta buffers of count_words words each
    int64_t count_words;           // uint32 words per buffer
    int density_mode;              // 0: counts in base[0], delta in delta[0], folded by k_fold;
                                   // 1: rotation, the sweep kernel folds the previous delta;
                                   // 2: face fluxes in flux buffer s mod 2, folded by k_fold_faces;
                                   // 3: mirrored counts: gathers from base[s mod 2], atomics into
                                   //    base[(s+1) mod 2], then k_mirror copies it back
    uint32_t *flux;                // mode 2: two buffers of three count_words-word arrays
    int smc;                       // some system uses bond-force-biased moves
    int cpl;                       // some system uses walls, zones, the umbrella or caller-set classes
    const float2 *omega;           // frozen fields, per cell (A, B)
    const uint64_t *sweep_ctr;     // sweeps done before this graph / launch sequence
    uint32_t rel;                  // sweep index relative to *sweep_ctr
    uint64_t seed;
    unsigned long long *accept;    // [n_sys][kAcceptSlots][kAcceptStride]
    uint32_t *status;
    uint8_t *chain_class;          // per logical chain: 0 = pattern a, 1 = pattern b
    const float2 *tgt;             // umbrella target (phi_A, phi_B) per cell
    unsigned long long *conv;      // [n_sys][2]: chains converted to class a, to class b
    uint2 *halo;                   // stream tiles: boundary bead pairs, see halo_index
    int64_t halo_cap;              // stream tile entries per halo array
    unsigned long long *acc_tile;  // accepted moves per tile (see counts_per_tile), or null
};

// The one-tile-per-wave kernels for uniform moves without coupling (wave
// tiles and stream tiles) count accepted moves per tile: the wave that owns
// tile t in a sweep reads acc_tile[t] with its positions and writes back the
// sum after the moves, a plain load and store instead of a device atomic per
// wave.  The host folds acc_tile into the per-system counters (and clears
// it) before the tiling changes and before the counters are read; every
// other kernel adds to the per-system counters with atomics.
inline bool counts_per_tile(const SweepArgs &a)
{
    return !a.cpl && !a.smc && a.max_blocks == 0 && a.packed != 1;
}

// Stream tiles read the bead pairs of their two overlap lanes, which other
// waves own and rewrite during the same sweep, from a copy taken before the
// sweep: halo buffer (s mod 2) holds, for every stream tile and both of its
// end lanes (side 0: first owned lane, side 1: last owned lane), the pair as
// it stands when sweep s starts, one 8-byte pair per position array
// (component 0..2: coordinates or offsets, 3..5: cells).  A tile's entry is
// one 128-byte line (two sides of eight pair slots), so a wave reads one
// line of each neighbour and writes one line.  Sweep s writes buffer
// (s + 1) mod 2 as its owners finish; the host refills buffer (s mod 2)
// before a batch of sweeps and after a chain reorder.
constexpr int kHaloComps = 6;
constexpr int kHaloSlots = 8;      // pair slots per side (kHaloComps used)
__host__ __device__ inline int64_t halo_index(int buf, int comp, int64_t tile, int side, int64_t cap)
{
    return (((int64_t)buf * cap + tile) * 2 + side) * kHaloSlots + comp;
}
struct HaloArgs {
    const DevSys *systems;
    const Tile *ptiles;
    int n_ptiles;
    float *P0, *P1, *P2;           // read only
    int *C0, *C1, *C2;
    uint2 *halo;
    int64_t halo_cap;
    int buf;
};

struct DensityArgs {
    const DevSys *systems;
    const Tile *tiles;
    const uint32_t *chain_id;
    int tile_begin, tile_end;
    float *P0, *P1, *P2;
    int *C0, *C1, *C2;
    uint32_t *counts;              // the target buffer (zeroed by the caller)
    uint32_t *status;
    const uint8_t *chain_class;
};

struct ReorderArgs {
    const DevSys *systems;
    const Tile *tiles;
    int n_tiles;
    int64_t total_chains, total_cells;
    float *P0, *P1, *P2;           // live positions
    int *C0, *C1, *C2;
    float *Q0, *Q1, *Q2;           // scratch positions (same layout)
    int *D0, *D1, *D2;
    uint32_t *chain_id, *chain_id2;
    uint32_t *keys;                // per chain: context-wide cell of bead 0
    uint32_t *hist;                // per cell: count, then exclusive offsets
    uint32_t *bsum;                // scan block sums
    uint32_t *perm;                // perm[new] = old
    uint32_t *status;
};

struct FieldArgs {
    const DevSys *systems;
    int sys;
    int64_t n_cells;
    const uint32_t *counts;        // current counts
    const float2 *omega;
    const float2 *tgt;             // umbrella targets
    float *out;                    // [2][n_cells]
};

struct InitArgs {
    int repr;
    int n_chains, N, stride;
    int64_t slot_off;
    uint32_t sys_id;
    uint64_t seed;
    double box[3];
    float edge[3];
    double sigma;                  // Re / sqrt(3 (N - 1))
    float *P0, *P1, *P2;
    int *C0, *C1, *C2;
    int walls, wall_lo, wall_hi;   // chains are drawn again until they fit between the walls
    uint32_t *status;
};

// Placement from target concentration fields (one system).
struct PlaceArgs {
    InitArgs ia;                   // representation, stream, walls, output arrays
    const DevSys *sys;             // the system's table entry
    const uint32_t *chain_id;      // logical chain id per slot of the context
    const uint8_t *chain_class;    // per logical chain of the context
    int64_t chain_off, cell_off, n_cells;
    int grid[3];
    double edge64[3];              // box / grid in FP64 (target points)
    double Re;
    const float2 *tgt;             // target (phi_A, phi_B) per cell of the context
    unsigned long long *W;         // [2][n_cells] inclusive prefix sums of the class weights
    int na[2];                     // A beads of pattern a, b
};

struct ObsArgs {
    int repr;
    int n_chains, N, stride;
    int64_t slot_off;
    float edge[3];
    double k_half;
    const float *P0, *P1, *P2;
    const int *C0, *C1, *C2;
    const uint32_t *counts;        // current counts
    int64_t cell_off, n_cells;
    double phi_per_count;          // M / B
    double chiN, kappaN;
    int ham_form;
    double umb_lambda;             // umbrella strength (0: off)
    const float2 *tgt;             // umbrella targets per cell of the context
    double *partials;
    int block_base;
};

hipError_t launch_sweep(int repr, int cw, const SweepArgs &a, hipStream_t st);
hipError_t launch_stream_halo(int repr, const HaloArgs &a, hipStream_t st);
// Add acc_tile[t] to the acceptance counters of tile t's system and clear it
// (stream: the tiles are stream tiles, whose system is the low 24 bits).
hipError_t launch_acc_fold(const Tile *tiles, int n_tiles, bool stream, unsigned long long *acc_tile,
                           unsigned long long *accept, hipStream_t st);
hipError_t launch_density(int repr, int cw, const DensityArgs &a, hipStream_t st);
hipError_t launch_fields(int cw, const FieldArgs &a, hipStream_t st);
hipError_t launch_unpack_counts(int cw, const uint32_t *counts, int64_t cell_off, int64_t n_cells,
                                uint32_t *out, hipStream_t st);
// Density mode 2: the fold of one sweep's face fluxes, one block per chunk
// of kFoldChunk cells of one system.
constexpr int kFoldChunk = 2048;
struct FoldChunk {
    uint32_t sys;                  // index into the system table
    uint32_t pad;
    int64_t first;                 // first cell of the chunk within its system
};
struct FoldFacesArgs {
    const DevSys *systems;
    const FoldChunk *chunks;
    uint32_t *counts;              // base[0]
    uint32_t *flux;
    int64_t count_words;
    const uint64_t *sweep_ctr;
    uint32_t rel;
    uint32_t *status;
};
hipError_t launch_fold_faces(int cw, const FoldFacesArgs &a, int n_chunks, hipStream_t st);
hipError_t launch_fold(int cw, const uint32_t *counts_in, uint32_t *delta, uint32_t *counts_out, int64_t n,
                       uint32_t *status, hipStream_t st);
// Density mode 3: after sweep s, copy base[(s+1) mod 2] (the counts the
// sweep's atomics produced) into base[s mod 2]; for packed 16-bit counts
// also check that the halves sum to the number of beads: each copy block
// adds the sum of the halves it copied to its entry of `part`, and after
// the last sweep of a batch a one-block kernel compares the total with
// (sweeps of the batch) x (beads) and clears `part` for the next batch.
constexpr int kMirrorBlocks = 32768;
constexpr int kMirrorUnroll = 4;   // 16-byte words per thread per step
struct MirrorArgs {
    uint32_t *base;                // two count buffers of count_words words each
    int64_t count_words;           // a multiple of 4
    const uint64_t *sweep_ctr;
    uint32_t rel;
    unsigned long long *part;      // kMirrorBlocks running sums of the count halves (zero between batches)
    unsigned long long beads;      // beads of the context
    uint32_t *status;
};
hipError_t launch_mirror(int cw, const MirrorArgs &a, hipStream_t st);
// After n_sweeps mirrors of a batch (packed 16-bit counts only).
hipError_t launch_mirror_check(int cw, const MirrorArgs &a, uint32_t n_sweeps, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_advance(uint64_t *ctr, uint32_t n, hipStream_t st);
hipError_t launch_init(const InitArgs &a, hipStream_t st);
hipError_t launch_iota_chains(const ReorderArgs &a, hipStream_t st);
hipError_t launch_reorder(int repr, const ReorderArgs &a, hipStream_t st);
int64_t reorder_bsum_words(int64_t total_cells);
hipError_t launch_observables(int cw, const ObsArgs &a, double *out, hipStream_t st);
hipError_t launch_place(const PlaceArgs &a, unsigned long long *scan_bsum, hipStream_t st);
int64_t place_bsum_words(int64_t n_cells);

}  // namespace soma
