// soma_types.hpp -- device-side tables of the SCMF sweep library.
//
// Shared by the kernels and the host runtime of libsoma_mi355x only.
#pragma once
#include <stdint.h>

namespace soma {

constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kMaxN = 128;             // beads per chain handled by one wave (2 beads per lane)
constexpr int kPatternWords = kMaxN / 32;

// Accepted-move counters: each system owns kAcceptSlots 64-bit counters one
// cache line apart; wave w of a launch adds to slot (w mod kAcceptSlots), so
// no single address takes more than 1/kAcceptSlots of the updates.
constexpr int kAcceptSlots = 128;
constexpr int kAcceptStride = 8;          // uint64 words between slots (64 B)

enum Repr : int { REPR_F32 = 0, REPR_CELL = 1 };
enum CountW : int { COUNT_U16 = 0, COUNT_U32 = 1 };

// Device status bits, latched by the kernels and read at synchronising calls.
// (Fields are never non-finite on the device: they are affine in integer
// counts, and a frozen field array is checked on the host when it is set.)
enum StatusBits : uint32_t {
    ST_COUNT_OVERFLOW = 1u,
    ST_CELL_OVERFLOW = 4u,
    ST_INTERNAL = 8u,
    ST_PLACEMENT = 16u,     // a chain did not fit between the walls (initial walks, placement)
};

// Attempts of the initial walks and of the placement to draw a chain that
// fits between walls.
constexpr int kMaxAttempts = 64;

// One system, as the kernels see it.  Offsets are in elements of the flat
// arrays shared by all systems of a context.
struct alignas(16) DevSys {
    int64_t slot_off;      // first bead slot (chains stored with an even stride 2P)
    int64_t cell_off;      // first cell of the count / field arrays
    int64_t chain_off;     // first chain of the context-wide chain arrays
    int32_t n_chains;
    int32_t N;             // beads per chain
    int32_t P;             // bead pairs per chain = ceil(N/2); lane p holds beads 2p, 2p+1
    int32_t G;             // chains per wave tile = 64 / P
    int32_t n_chains_a;    // chains [0, n_chains_a) use pat_a
    uint32_t sys_id;       // Philox counter word 3
    int32_t n[3];          // grid
    int32_t frozen;        // 1: fields come from the frozen array, else from the counts
    int32_t edge_dyadic;   // 1: every cell edge is a power of two (x * (1/edge) is exact)
    float inv_n[3];        // 1 / n, for the periodic wrap
    float edge[3];         // cell edge (FP32)
    float inv_edge[3];     // 1 / edge (FP32)
    float k_half;          // k/2 = 3(N-1)/(2 Re^2)
    float delta;           // move half-width
    float inv_P;           // 1 / P
    // omega_A = cAA nA + cAB nB + c0, omega_B = cBA nA + cBB nB + c0
    float cAA, cAB, cBA, cBB, c0;
    int64_t n_cells;
    // bond-force-biased moves (smc != 0): displacement A F + sqrt(2A) xi in
    // FP64, rejected at 0.99 cell edges; the acceptance ratio in FP32
    int32_t smc;
    float smc_Af;          // A
    float smc_inv4A;       // 1 / (4 A)
    float k_f;             // k = 3(N-1)/Re^2
    float dmax[3];         // 0.99 cell edge
    double smc_A;          // A
    double smc_s2A;        // sqrt(2 A)
    double k_spring;       // k in FP64 (the force of the proposal)
    // Coupling (Sec. 3.2): umbrella potential toward target concentration
    // fields, hard walls at z-cell faces, molecular-type conversion zones.
    int32_t umb;           // 1: omega_t gains -umb_coef * target_t(c) (the lambda phi_t/N part is in the cXX)
    float umb_coef;        // lambda / N
    int32_t walls;         // 1: trial positions outside z cells [wall_lo, wall_hi) are rejected
    int32_t wall_lo, wall_hi;
    int32_t zones;         // 1: conversion zones at the walls
    int32_t cls_array;     // 1: chain classes come from the class array (zones, or classes set by
                           //    the caller); 0: chains [0, n_chains_a) are class a
    int32_t zone_a, zone_b;            // lower / upper zone present
    int32_t zone_a_lim, zone_b_lim;    // N (wall_lo + lower width), N (wall_hi - upper width)
    alignas(16) uint32_t pat_a[kPatternWords];   // bit i: type of bead i (0 = A, 1 = B)
    alignas(16) uint32_t pat_b[kPatternWords];
};

struct Tile {
    uint32_t sys;          // index into the system table (not the Philox system id)
    uint32_t chain0;       // first chain of the tile within its system
};

}  // namespace soma
