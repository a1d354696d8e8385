// soma_kernels.hip -- HIP kernels of the SCMF Monte-Carlo sweep for gfx950.
//
// The method (Sec. 2, SOMA paragraph, and Sec. 2.2 of the paper): chains
// move independently under frozen quasi-instantaneous fields; each sweep
// performs biased/Metropolis trial moves with energy evaluations, then
// rebuilds the particle density fields, then refreshes the fields.
//
// Mapping onto CDNA4
//   * One wavefront owns a tile of whole chains: lane p of a chain holds the
//     bead pair (2p, 2p+1), so a chain of N <= 128 beads fits one wave and
//     the bond neighbours of a bead sit in the same lane or the adjacent
//     lane (cross-lane exchange with ds_bpermute; no barrier).
//   * Positions are SoA with chains stored at an even stride, so each lane
//     reads and writes one 8-byte pair per coordinate: fully coalesced.
//   * The even pass moves bead 2p of every lane, the odd pass bead 2p+1;
//     beads of one parity share no bond, so all lanes move at once.
//   * The fields are never stored: omega of a cell is an affine function of
//     its two counts, evaluated where a moved bead needs it (only when the
//     trial move leaves the bead's cell).
//   * The density is updated, not rebuilt: a sweep reads frozen counts (for
//     the fields) and adds -1/+1 atomically only for accepted moves that
//     change cell (about a fifth of the beads), not one atomic per bead; a
//     wave first merges its updates in LDS.  Four placements of those
//     atomics (density modes): a delta folded by a streaming kernel after
//     the sweep (0); a delta folded by the next sweep's own threads, which
//     read B[s-1] + D[s-1] (1); face fluxes, folded as their divergence
//     (2); or the second of two identical count buffers, which no gather of
//     the sweep reads, copied back afterwards (3).
//   * Tilings: wave tiles (whole chains on the lanes of one wave), block
//     tiles (whole chains packed over the waves of a workgroup) and stream
//     tiles (a system's lanes in chain order, 62 owned lanes per wave plus
//     two overlap lanes whose pairs come from a halo copy).
//   * Accepted moves are counted per tile by the wave- and stream-tile
//     kernels (a plain load and store per wave), per system with one atomic
//     per wave by the others.
//   * Philox4x32-10 is counter based: one 128-bit block per (bead, logical
//     chain, sweep, system); no RNG state lives in memory.
//   * Per system, the trial move is uniform in a cube or bond-force biased
//     ("smart", SOMA's move): the biased move draws FP64 Box-Muller normals
//     and needs the moved even beads before the odd proposals.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "soma_launch.hpp"
#include "soma_types.hpp"

namespace soma {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies with the key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        // three-input XOR in one instruction (truth table 0x96)
        const uint32_t nx = __builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), c.y, k0, 0x96);
        const uint32_t nz = __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), c.w, k1, 0x96);
        c.y = (uint32_t)m1;
        c.w = (uint32_t)m0;
        c.x = nx;
        c.z = nz;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

struct Draw {
    float dx, dy, dz, u;
};

// Top 24 bits of each word: displacement = delta * ((w >> 8) - 2^23) * 2^-23
// (one FP32 multiply of exact operands), acceptance variate u = (w >> 8) 2^-24.
// delta_s = delta * 2^-23 (exact), so delta_s * m rounds exactly like
// delta * (m * 2^-23): one FP32 rounding of the same real product.
__device__ __forceinline__ Draw move_draw(uint32_t bead, uint32_t chain, uint32_t sweep,
                                          uint32_t sys, uint32_t k0, uint32_t k1, float delta_s)
{
    const uint4 w = philox4x32_10(make_uint4(bead, chain, sweep, sys), k0, k1);
    Draw d;
    d.dx = delta_s * (float)((int)(w.x >> 8) - 8388608);
    d.dy = delta_s * (float)((int)(w.y >> 8) - 8388608);
    d.dz = delta_s * (float)((int)(w.z >> 8) - 8388608);
    d.u = (float)(w.w >> 8) * 0x1p-24f;
    return d;
}

// Periodic wrap of an unwrapped cell index into [0, n); exact for |i| < 2^23
// (24-bit multiply: |q| < 2^23, n < 2^15).
__device__ __forceinline__ int wrap_cell(int i, int n, float inv_n)
{
    const int q = (int)floorf((float)i * inv_n);
    int r = i - __mul24(q, n);
    r = r < 0 ? r + n : r;
    r = r >= n ? r - n : r;
    return r;
}

// Wrap of i in [-n, 2n) into [0, n): exactly one of i, i + n, i - n lies in
// [0, n), and read as unsigned it is the smallest of the three (the others
// are >= n or negative).  For i outside [-n, 2n) all three are >= n, so the
// result is >= n exactly when i was out of that range.
__device__ __forceinline__ int wrap_step(int i, int n)
{
    const uint32_t u = (uint32_t)i, m = (uint32_t)n;
    return (int)min(min(u, u + m), u - m);
}

__device__ __forceinline__ bool wrapped(int w, int n) { return (uint32_t)w < (uint32_t)n; }

// ---------------------------------------------------------------------------
// Position representations
// ---------------------------------------------------------------------------
struct SysView {            // the per-system scalars a wave needs (SGPR resident)
    int n0, n1, n2;
    float inv_n0, inv_n1, inv_n2;
    float e0, e1, e2;
    float ie0, ie1, ie2;
    bool dyadic;            // every edge a power of two: x * (1/edge) is the exact quotient
};

// floor(x / e) of the exact quotient for the FP32 cell edge e.  The product
// with the rounded reciprocal can be one off next to a face when e is not a
// power of two; the sign of x - k e, exact after one FMA rounding, corrects
// it (|x / e| < 2^22, so the product is within one of the quotient).
__device__ __forceinline__ float floor_div(float x, float e, float ie, bool dyadic)
{
    float k = floorf(x * ie);
    if (!dyadic) {
        if (fmaf(-k, e, x) < 0.0f) k -= 1.0f;
        else if (fmaf(-(k + 1.0f), e, x) >= 0.0f) k += 1.0f;
    }
    return k;
}

struct BeadF32 {
    float x, y, z;
};
struct BeadCell {
    int cx, cy, cz;
    float ox, oy, oz;
};

// Unwrapped cell indexes must stay where the float-reciprocal wrap is exact
// (|i| < 2^24); beyond 2^23 the bead is flagged and counted in cell 0.
constexpr int kCellLimit = 1 << 23;

__device__ __forceinline__ float3 bond(const BeadF32 &a, const BeadF32 &b, const SysView &)
{
    return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
// (the product of a small cell difference and the edge is exact, so the
// fused form rounds exactly like the separate multiply and add)
__device__ __forceinline__ float3 bond(const BeadCell &a, const BeadCell &b, const SysView &v)
{
    return make_float3(fmaf((float)(a.cx - b.cx), v.e0, a.ox - b.ox),
                       fmaf((float)(a.cy - b.cy), v.e1, a.oy - b.oy),
                       fmaf((float)(a.cz - b.cz), v.e2, a.oz - b.oz));
}

__device__ __forceinline__ BeadF32 propose(const BeadF32 &a, const Draw &d, const SysView &)
{
    return BeadF32{a.x + d.dx, a.y + d.dy, a.z + d.dz};
}

// Keep the offset in [0, edge) by whole-cell steps, each one FP32 rounding;
// an offset that rounds up to exactly one edge moves to offset 0 of the next cell.
__device__ __forceinline__ void renorm(int &c, float &o, float e)
{
    while (o < 0.0f) { o = o + e; c -= 1; }
    while (o >= e) { o = o - e; c += 1; }
}

// Lazy renormalisation of a trial offset o + d (|d| < 0.99 edge): the
// offset may lie anywhere in the window [-e, 2e); only an offset that leaves
// it moves one whole cell (one FP32 rounding), which brings it back inside.
// A bead's cell index therefore changes only after a net displacement of
// about one edge, so a sweep rewrites few cell words (renorm, which keeps
// offsets in [0, e), gives the canonical form of a new position).
__device__ __forceinline__ void renorm_window(int &c, float &o, float e)
{
    const bool lo = o < -e;
    const bool hi = o >= 2.0f * e;
    o = lo ? o + e : (hi ? o - e : o);
    c += (int)hi - (int)lo;
}

// NGP index of a bead along one axis: floor((c e + o) / e) = c + floor(o / e)
// exactly, with o in [-e, 2e).
__device__ __forceinline__ int ngp(int c, float o, float e) { return c + (int)(o >= e) - (int)(o < 0.0f); }

__device__ __forceinline__ BeadCell propose(const BeadCell &a, const Draw &d, const SysView &v)
{
    BeadCell n{a.cx, a.cy, a.cz, a.ox + d.dx, a.oy + d.dy, a.oz + d.dz};
    renorm_window(n.cx, n.ox, v.e0);
    renorm_window(n.cy, n.oy, v.e1);
    renorm_window(n.cz, n.oz, v.e2);
    return n;
}

// NGP cell of a bead: wrapped cell coordinates and, for FP32 positions, the
// unwrapped floors (to step to the cell of a trial position; for cell +
// offset positions fz alone, the unwrapped z index).  `bad` is set
// when the unwrapped index leaves the range the wrap handles (or the
// coordinate is not finite); the bead is then counted in cell 0.
struct CellPos {
    int x, y, z;
    float fx, fy, fz;
};

// Beads almost always lie within one image of the box, where wrap_step is
// the wrap; the general form (and the range check) runs only for the lanes
// that need it.
__device__ __forceinline__ CellPos locate(const BeadF32 &a, const SysView &v, bool &bad)
{
    CellPos c;
    c.fx = floor_div(a.x, v.e0, v.ie0, v.dyadic);
    c.fy = floor_div(a.y, v.e1, v.ie1, v.dyadic);
    c.fz = floor_div(a.z, v.e2, v.ie2, v.dyadic);
    const float lim = (float)kCellLimit;
    c.x = wrap_step((int)c.fx, v.n0);
    c.y = wrap_step((int)c.fy, v.n1);
    c.z = wrap_step((int)c.fz, v.n2);
    // (a non-finite coordinate fails the magnitude test)
    if (!(wrapped(c.x, v.n0) && wrapped(c.y, v.n1) && wrapped(c.z, v.n2) && fabsf(c.fx) < lim &&
          fabsf(c.fy) < lim && fabsf(c.fz) < lim)) {
        if (!(fabsf(c.fx) < lim && fabsf(c.fy) < lim && fabsf(c.fz) < lim)) {
            bad = true;
            c.x = c.y = c.z = 0;
            c.fx = c.fy = c.fz = 0.0f;
            return c;
        }
        c.x = wrap_cell((int)c.fx, v.n0, v.inv_n0);
        c.y = wrap_cell((int)c.fy, v.n1, v.inv_n1);
        c.z = wrap_cell((int)c.fz, v.n2, v.inv_n2);
    }
    return c;
}
// (cell mode: fz carries the unwrapped z index, for walls and zones)
__device__ __forceinline__ CellPos locate(const BeadCell &a, const SysView &v, bool &bad)
{
    const int kx = ngp(a.cx, a.ox, v.e0), ky = ngp(a.cy, a.oy, v.e1), kz = ngp(a.cz, a.oz, v.e2);
    CellPos c{wrap_step(kx, v.n0), wrap_step(ky, v.n1), wrap_step(kz, v.n2), 0.0f, 0.0f, (float)kz};
    if (!(wrapped(c.x, v.n0) && wrapped(c.y, v.n1) && wrapped(c.z, v.n2))) {
        if (kx <= -kCellLimit || kx >= kCellLimit || ky <= -kCellLimit || ky >= kCellLimit ||
            kz <= -kCellLimit || kz >= kCellLimit) {
            bad = true;
            c.x = c.y = c.z = 0;
            c.fz = 0.0f;
            return c;
        }
        c.x = wrap_cell(kx, v.n0, v.inv_n0);
        c.y = wrap_cell(ky, v.n1, v.inv_n1);
        c.z = wrap_cell(kz, v.n2, v.inv_n2);
    }
    return c;
}

// Cell of a trial position.  The move half-width is below 0.99 cell edges,
// so the unwrapped index changes by at most one per axis (clamped so that a
// non-finite coordinate still yields an in-range cell).
__device__ __forceinline__ int clamp1(int k) { return max(-1, min(k, 1)); }

__device__ __forceinline__ CellPos step(const CellPos &o, const BeadF32 &, const BeadF32 &n, const SysView &v)
{
    CellPos c;
    c.fx = floor_div(n.x, v.e0, v.ie0, v.dyadic);
    c.fy = floor_div(n.y, v.e1, v.ie1, v.dyadic);
    c.fz = floor_div(n.z, v.e2, v.ie2, v.dyadic);
    c.x = wrap_step(o.x + clamp1((int)(c.fx - o.fx)), v.n0);
    c.y = wrap_step(o.y + clamp1((int)(c.fy - o.fy)), v.n1);
    c.z = wrap_step(o.z + clamp1((int)(c.fz - o.fz)), v.n2);
    return c;
}
__device__ __forceinline__ CellPos step(const CellPos &o, const BeadCell &ob, const BeadCell &n, const SysView &v)
{
    // (a trial move is shorter than one cell edge, so the NGP index changes
    // by -1, 0 or 1 per axis)
    const int dz = ngp(n.cz, n.oz, v.e2) - ngp(ob.cz, ob.oz, v.e2);
    CellPos c{0, 0, 0, 0.0f, 0.0f, o.fz + (float)dz};
    c.x = wrap_step(o.x + (ngp(n.cx, n.ox, v.e0) - ngp(ob.cx, ob.ox, v.e0)), v.n0);
    c.y = wrap_step(o.y + (ngp(n.cy, n.oy, v.e1) - ngp(ob.cy, ob.oy, v.e1)), v.n1);
    c.z = wrap_step(o.z + dz, v.n2);
    return c;
}

// Linear index (x * ny + y) * nz + z with 24-bit multiplies (nx * ny <= 2^24).
__device__ __forceinline__ int lin(const CellPos &c, const SysView &v)
{
    return (int)__umul24((uint32_t)(__umul24((uint32_t)c.x, (uint32_t)v.n1) + c.y), (uint32_t)v.n2) + c.z;
}

template <class Bead>
__device__ __forceinline__ int cell_of(const Bead &a, const SysView &v, bool &bad)
{
    return lin(locate(a, v, bad), v);
}

__device__ __forceinline__ BeadF32 shfl_up1(const BeadF32 &a)
{
    return BeadF32{__shfl_up(a.x, 1), __shfl_up(a.y, 1), __shfl_up(a.z, 1)};
}
__device__ __forceinline__ BeadF32 shfl_down1(const BeadF32 &a)
{
    return BeadF32{__shfl_down(a.x, 1), __shfl_down(a.y, 1), __shfl_down(a.z, 1)};
}
__device__ __forceinline__ BeadCell shfl_up1(const BeadCell &a)
{
    return BeadCell{__shfl_up(a.cx, 1), __shfl_up(a.cy, 1), __shfl_up(a.cz, 1),
                    __shfl_up(a.ox, 1), __shfl_up(a.oy, 1), __shfl_up(a.oz, 1)};
}
__device__ __forceinline__ BeadCell shfl_down1(const BeadCell &a)
{
    return BeadCell{__shfl_down(a.cx, 1), __shfl_down(a.cy, 1), __shfl_down(a.cz, 1),
                    __shfl_down(a.ox, 1), __shfl_down(a.oy, 1), __shfl_down(a.oz, 1)};
}

// Bond neighbours of a lane's bead pair: the odd bead of the lane before
// (left) and the even bead of the lane after (right).  In block tiles a
// wave's first and last lanes take them from the neighbouring waves through
// LDS; every thread of the block calls these (they hold a barrier).
template <bool BT, class Bead>
__device__ __forceinline__ Bead left_neighbour(const Bead &b1)
{
    Bead l = shfl_up1(b1);
    if constexpr (BT) {
        __shared__ Bead edge[16];
        const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
        if (lane == 63) edge[w] = b1;
        __syncthreads();
        if (lane == 0 && w > 0) l = edge[w - 1];
    }
    return l;
}
template <bool BT, class Bead>
__device__ __forceinline__ Bead right_neighbour(const Bead &b0)
{
    Bead r = shfl_down1(b0);
    if constexpr (BT) {
        __shared__ Bead edge[16];
        const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
        if (lane == 0) edge[w] = b0;
        __syncthreads();
        if (lane == 63 && w + 1 < (int)(blockDim.x >> 6)) r = edge[w + 1];
    }
    return r;
}

// Positions: F32 keeps coordinates in P0..P2; CELL keeps offsets in P0..P2
// and cells in C0..C2.  `slot` is even, so pairs are 8-byte aligned.
struct PosArrays {
    float *P0, *P1, *P2;
    int *C0, *C1, *C2;
};

// Position lines stay in the caches between a wave's loads and its stores:
// most stored lines are partial (only changed pairs are written back) and are
// completed in the L2 from the loaded data before they reach memory.
// (Non-temporal loads or stores, which keep lines out of the caches, made the
// sweep slower.)
__device__ __forceinline__ float2 ld2(const float *p) { return *reinterpret_cast<const float2 *>(p); }
__device__ __forceinline__ int2 ld2(const int *p) { return *reinterpret_cast<const int2 *>(p); }
__device__ __forceinline__ void st2(float *p, float x, float y) { *reinterpret_cast<float2 *>(p) = make_float2(x, y); }
__device__ __forceinline__ void st2(int *p, int x, int y) { *reinterpret_cast<int2 *>(p) = make_int2(x, y); }

__device__ __forceinline__ void load_pair(const PosArrays &A, int64_t slot, BeadF32 &a, BeadF32 &b)
{
    const float2 x = ld2(A.P0 + slot);
    const float2 y = ld2(A.P1 + slot);
    const float2 z = ld2(A.P2 + slot);
    a = BeadF32{x.x, y.x, z.x};
    b = BeadF32{x.y, y.y, z.y};
}
__device__ __forceinline__ void store_pair(const PosArrays &A, int64_t slot, const BeadF32 &a,
                                           const BeadF32 &b)
{
    st2(A.P0 + slot, a.x, b.x);
    st2(A.P1 + slot, a.y, b.y);
    st2(A.P2 + slot, a.z, b.z);
}
// Store what a sweep changed: nothing for a pair whose two moves were
// rejected; in cell mode, each cell word only when a bead of the pair left
// its cell along that axis (a few percent of the beads), so most cell
// sectors are never written back.
__device__ __forceinline__ void store_moved(const PosArrays &A, int64_t slot, const BeadF32 &a, const BeadF32 &b,
                                            const BeadF32 &, const BeadF32 &, bool moved)
{
    if (moved) store_pair(A, slot, a, b);
}
__device__ __forceinline__ void store_moved(const PosArrays &A, int64_t slot, const BeadCell &a, const BeadCell &b,
                                            const BeadCell &oa, const BeadCell &ob, bool moved)
{
    if (!moved) return;
    if (a.cx != oa.cx || b.cx != ob.cx) st2(A.C0 + slot, a.cx, b.cx);
    if (a.cy != oa.cy || b.cy != ob.cy) st2(A.C1 + slot, a.cy, b.cy);
    if (a.cz != oa.cz || b.cz != ob.cz) st2(A.C2 + slot, a.cz, b.cz);
    st2(A.P0 + slot, a.ox, b.ox);
    st2(A.P1 + slot, a.oy, b.oy);
    st2(A.P2 + slot, a.oz, b.oz);
}

__device__ __forceinline__ void load_pair(const PosArrays &A, int64_t slot, BeadCell &a, BeadCell &b)
{
    const int2 cx = ld2(A.C0 + slot);
    const int2 cy = ld2(A.C1 + slot);
    const int2 cz = ld2(A.C2 + slot);
    const float2 x = ld2(A.P0 + slot);
    const float2 y = ld2(A.P1 + slot);
    const float2 z = ld2(A.P2 + slot);
    a = BeadCell{cx.x, cy.x, cz.x, x.x, y.x, z.x};
    b = BeadCell{cx.y, cy.y, cz.y, x.y, y.y, z.y};
}
__device__ __forceinline__ void store_pair(const PosArrays &A, int64_t slot, const BeadCell &a,
                                           const BeadCell &b)
{
    st2(A.C0 + slot, a.cx, b.cx);
    st2(A.C1 + slot, a.cy, b.cy);
    st2(A.C2 + slot, a.cz, b.cz);
    st2(A.P0 + slot, a.ox, b.ox);
    st2(A.P1 + slot, a.oy, b.oy);
    st2(A.P2 + slot, a.oz, b.oz);
}

// ---------------------------------------------------------------------------
// Counts and fields
// ---------------------------------------------------------------------------
// U16: one uint32 per cell, A in the low half, B in the high half.
// U32: two uint32 per cell (A, B) interleaved.
template <int CW>
__device__ __forceinline__ uint2 load_counts(const uint32_t *cnt, int64_t cell)
{
    if constexpr (CW == COUNT_U16) {
        const uint32_t w = cnt[cell];
        return make_uint2(w & 0xFFFFu, w >> 16);
    } else {
        return *reinterpret_cast<const uint2 *>(cnt + 2 * cell);
    }
}

// Raw count words of one cell (and, when the fold runs inside the sweep, the
// words of the previous delta), loaded without being combined so that
// several gathers can be in flight before the first use.
struct RawCount {
    uint32_t w0, w1, d0, d1;
};

template <int CW, bool FI>
__device__ __forceinline__ RawCount load_raw(const uint32_t *cnt, const uint32_t *dprev, int64_t cell)
{
    RawCount r{0u, 0u, 0u, 0u};
    if constexpr (CW == COUNT_U16) {
        r.w0 = cnt[cell];
        if constexpr (FI) r.d0 = dprev[cell];
    } else {
        const uint2 w = *reinterpret_cast<const uint2 *>(cnt + 2 * cell);
        r.w0 = w.x;
        r.w1 = w.y;
        if constexpr (FI) {
            const uint2 d = *reinterpret_cast<const uint2 *>(dprev + 2 * cell);
            r.d0 = d.x;
            r.d1 = d.y;
        }
    }
    return r;
}

// Counts of the cell: base plus delta in modular uint32 arithmetic; for U16
// the packed sum equals nA + 2^16 nB whenever both true counts fit 16 bits.
template <int CW>
__device__ __forceinline__ uint2 counts_of(const RawCount &r)
{
    if constexpr (CW == COUNT_U16) {
        const uint32_t w = r.w0 + r.d0;
        return make_uint2(w & 0xFFFFu, w >> 16);
    } else {
        return make_uint2(r.w0 + r.d0, r.w1 + r.d1);
    }
}

// Per-wave aggregation of the density delta in LDS before the device
// atomics.  Device-scope atomics are executed at the memory side at a fixed
// rate; updates of one chain often hit the same count word (a chain carries
// a count along: one bead leaves a cell that another bead of the same chain
// enters), so merging a wave's updates first removes about a fifth of them.
// Open addressing over SLOTS slots: key = word index + 1 (0 = empty).  A
// wave makes at most 4 updates per lane with cell words (256 in all) and at
// most 6 with face fluxes (384), so with 256 or 512 slots a slot is always
// found and the probe loop ends.
constexpr int kAggSlotsCells = 256;
constexpr int kAggSlotsFaces = 512;

// Multiplicative hash of the low 24 bits of the key.  The product is taken
// with the full-rate 24-bit multiply (left to itself the compiler narrows the
// constant and emits the quarter-rate 32-bit multiply).
template <int SLOTS>
__device__ __forceinline__ uint32_t agg_hash(uint32_t key)
{
    uint32_t p;
    asm("v_mul_u32_u24 %0, 0x9e3779, %1" : "=v"(p) : "v"(key));
    return (p >> 10) & (SLOTS - 1);
}

template <int SLOTS>
__device__ __forceinline__ void agg_insert(uint32_t *keys, uint32_t *vals, uint32_t key, uint32_t v, bool on)
{
    uint32_t h = agg_hash<SLOTS>(key);
    bool pending = on;
    while (__ballot(pending) != 0) {
        if (pending) {
            const uint32_t old = atomicCAS(keys + h, 0u, key);
            if (old == 0u || old == key) {
                atomicAdd(vals + h, v);
                pending = false;
            } else {
                h = (h + 1u) & (SLOTS - 1);
            }
        }
    }
}

// Empty the wave's table (each lane clears SLOTS / 64 keys and values).
template <int SLOTS>
__device__ __forceinline__ void agg_clear(uint32_t *keys, uint32_t *vals)
{
    const int lane = (int)(threadIdx.x & 63);
    for (int k = lane; k < SLOTS; k += 64) {
        keys[k] = 0u;
        vals[k] = 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Word index and packed increment of one bead of type t in a cell.
template <int CW>
__device__ __forceinline__ uint32_t count_word(int64_t cell, int t)
{
    return CW == COUNT_U16 ? (uint32_t)cell : (uint32_t)(2 * cell + t);
}
template <int CW>
__device__ __forceinline__ uint32_t count_inc(int t)
{
    return CW == COUNT_U16 ? (t ? 0x10000u : 1u) : 1u;
}

// Fold one word: counts' = counts + delta in modular uint32 arithmetic (for
// U16 the packed sum is exact whenever both true counts fit 16 bits); returns
// true if a true count left its range (below zero, or above 65535 for packed
// 16-bit counts).
template <int CW>
__device__ __forceinline__ bool fold_word(uint32_t b, uint32_t d, uint32_t &out)
{
    out = b + d;
    if constexpr (CW == COUNT_U16) {
        const int dA = (int)(int16_t)(d & 0xFFFFu);
        const int dB = (int)(int16_t)((d - (uint32_t)dA) >> 16);
        const int nA = (int)(b & 0xFFFFu) + dA, nB = (int)(b >> 16) + dB;
        return nA < 0 || nA > 0xFFFF || nB < 0 || nB > 0xFFFF;
    } else {
        return (int)d >= 0 ? out < b : out > b;
    }
}

// Adds one bead of type t; returns true if the count overflowed its width.
template <int CW>
__device__ __forceinline__ bool scatter_count(uint32_t *cnt, int64_t cell, int t)
{
    if constexpr (CW == COUNT_U16) {
        const uint32_t old = atomicAdd(cnt + cell, t ? 0x10000u : 1u);
        return ((old >> (t ? 16 : 0)) & 0xFFFFu) == 0xFFFFu;
    } else {
        const uint32_t old = atomicAdd(cnt + 2 * cell + t, 1u);
        return old == 0xFFFFFFFFu;
    }
}

struct FieldCoef {
    float aa, ab, ba, bb, c0;
};

// omega_t of a cell from its counts (affine in the counts).  The same
// function produces the fields the sweep uses and the ones soma_fields reports.
__device__ __forceinline__ float omega_of(const FieldCoef &f, uint2 n, int t)
{
    const float a = (float)n.x, b = (float)n.y;
    return t ? fmaf(f.ba, a, fmaf(f.bb, b, f.c0)) : fmaf(f.aa, a, fmaf(f.ab, b, f.c0));
}

template <int CW>
__device__ __forceinline__ float omega_at(bool frozen, const float2 *omega, const uint32_t *cnt,
                                          int64_t cell_off, int cell, int t, const FieldCoef &f)
{
    if (frozen) {
        const float2 w = omega[cell_off + cell];
        return t ? w.y : w.x;
    }
    return omega_of(f, load_counts<CW>(cnt, cell_off + cell), t);
}

// Bead type from the system's 128-bit pattern.  All pattern words are loaded
// as values and selected by value: a per-lane choice between word addresses
// compiled (gfx950, -O3) into divergent branches that left the address of
// the fourth word unset for beads 96..127.
__device__ __forceinline__ int pattern_type(const DevSys &S, int cls, int i)
{
    const uint4 pa = *reinterpret_cast<const uint4 *>(S.pat_a);
    const uint4 pb = *reinterpret_cast<const uint4 *>(S.pat_b);
    const bool use_a = cls == 0;
    const uint32_t x = use_a ? pa.x : pb.x, y = use_a ? pa.y : pb.y;
    const uint32_t z = use_a ? pa.z : pb.z, w = use_a ? pa.w : pb.w;
    const int k = i >> 5;
    const uint32_t lo = (k & 1) ? y : x, hi = (k & 1) ? w : z;
    const uint32_t word = (k & 2) ? hi : lo;
    return (int)((word >> (i & 31)) & 1u);
}

// Class of a chain (which pattern it carries): from the class array when
// conversion zones (or the caller) change classes, else chains
// [0, n_chains_a) are class a.
template <bool CPL = true>
__device__ __forceinline__ int chain_cls(const DevSys &S, const uint8_t *cc, uint32_t clog)
{
    if constexpr (CPL)
        if (S.cls_array) return (int)cc[S.chain_off + clog];
    return (int)clog < S.n_chains_a ? 0 : 1;
}

// Unwrapped z cell of a bead, as computed by locate/step.
__device__ __forceinline__ int zcell(const CellPos &c, const BeadF32 &) { return (int)c.fz; }
__device__ __forceinline__ int zcell(const CellPos &c, const BeadCell &) { return (int)c.fz; }

// Types of beads i (even) and i + 1, from one pattern word.
__device__ __forceinline__ void pattern_pair(const DevSys &S, int cls, int i, int &t0, int &t1)
{
    const uint4 pa = *reinterpret_cast<const uint4 *>(S.pat_a);
    const uint4 pb = *reinterpret_cast<const uint4 *>(S.pat_b);
    const bool use_a = cls == 0;
    const uint32_t x = use_a ? pa.x : pb.x, y = use_a ? pa.y : pb.y;
    const uint32_t z = use_a ? pa.z : pb.z, w = use_a ? pa.w : pb.w;
    const int k = i >> 5;
    const uint32_t lo = (k & 1) ? y : x, hi = (k & 1) ? w : z;
    const uint32_t word = ((k & 2) ? hi : lo) >> (i & 31);
    t0 = (int)(word & 1u);
    t1 = (int)((word >> 1) & 1u);
}

__device__ __forceinline__ int wave_tile(int waves_per_block, int xcd_remap)
{
    int bid = (int)blockIdx.x;
    if (xcd_remap) {
        // Workgroups are dispatched round-robin over the 8 XCDs; give each
        // XCD a contiguous range of tiles so its L2 sees a compact cell range.
        const int nb = (int)gridDim.x;
        const int full = nb & ~7;
        if (bid < full) bid = (bid & 7) * (full >> 3) + (bid >> 3);
    }
    // wave-uniform by construction; readfirstlane lets the tile and system
    // tables be read with scalar loads
    return __builtin_amdgcn_readfirstlane(bid * waves_per_block + (int)(threadIdx.x >> 6));
}

// Block tiles: workgroup b takes tile b (the same XCD-aware remap as wave
// tiles); a block tile packs whole chains across all waves of the block.
__device__ __forceinline__ int block_tile(int xcd_remap)
{
    int bid = (int)blockIdx.x;
    if (xcd_remap) {
        const int nb = (int)gridDim.x;
        const int full = nb & ~7;
        if (bid < full) bid = (bid & 7) * (full >> 3) + (bid >> 3);
    }
    return __builtin_amdgcn_readfirstlane(bid);
}

// Tiling of the sweep.  Wave tiles (BT = false): a tile is G = floor(64/P)
// whole chains on the lanes of one wave.  Block tiles (BT = true): a tile is
// floor(64 W / P) whole chains packed over the 64 W lanes of a block, so a
// chain may span two waves (fewer idle lanes when 64 is not a multiple of
// P); bond neighbours across a wave boundary go through LDS.
template <bool BT>
__device__ __forceinline__ const Tile *tile_table(const SweepArgs &a) { return BT ? a.ptiles : a.tiles; }
template <bool BT>
__device__ __forceinline__ int tile_lane() { return BT ? (int)threadIdx.x : (int)(threadIdx.x & 63); }
// chains per tile; (64 W + 1/2) / P is at least 1/(2P) from an integer
template <bool BT>
__device__ __forceinline__ int tile_capacity(const DevSys &S)
{
    return BT ? (int)(((float)blockDim.x + 0.5f) * S.inv_P) : S.G;
}

__device__ __forceinline__ SysView make_view(const DevSys &S)
{
    SysView v;
    v.n0 = S.n[0]; v.n1 = S.n[1]; v.n2 = S.n[2];
    v.inv_n0 = S.inv_n[0]; v.inv_n1 = S.inv_n[1]; v.inv_n2 = S.inv_n[2];
    v.e0 = S.edge[0]; v.e1 = S.edge[1]; v.e2 = S.edge[2];
    v.ie0 = S.inv_edge[0]; v.ie1 = S.inv_edge[1]; v.ie2 = S.inv_edge[2];
    v.dyadic = S.edge_dyadic != 0;
    return v;
}

__device__ __forceinline__ float dot3(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ float3 add3(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }

// ---------------------------------------------------------------------------
// The sweep kernel: even pass, odd pass, density update (and, in density
// mode 1, the fold of the previous delta).  One launch per sweep for every
// system.
// ---------------------------------------------------------------------------
// Load the positions of one wave tile (lane p of chain g holds beads 2p and
// 2p+1).
template <bool BT, class Bead>
__device__ __forceinline__ void tile_load(const SweepArgs &a, int tile, Bead &b0, Bead &b1, uint32_t &clog)
{
    const Tile T = tile_table<BT>(a)[tile];
    const DevSys &S = a.systems[T.sys];
    const int P = S.P;
    const int lane = tile_lane<BT>();
    const int g = (int)(((float)lane + 0.5f) * S.inv_P);
    const int p = lane - g * P;
    const int nin = min(tile_capacity<BT>(S), S.n_chains - (int)T.chain0);
    const bool active = g < nin;
    // the logical chain id keys the random numbers: load it with the
    // positions, so the draws do not wait for a second memory round trip
    clog = a.chain_id[S.chain_off + (int)T.chain0 + (active ? g : 0)];
    b0 = Bead{};
    b1 = Bead{};
    if (active) {
        const int64_t slot = S.slot_off + (int64_t)((int)T.chain0 + g) * (2 * P) + 2 * p;
        load_pair(PosArrays{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2}, slot, b0, b1);
    }
}

// One wave tile of the sweep: the even pass, the odd pass and the density
// delta of up to G whole chains, from positions already loaded by tile_load.
// Face fluxes of one bead that moved from cell o to cell n (wrapped
// coordinates, at most one step per axis): the move is taken axis by axis,
// x, y, then z, and each step adds the bead to the flux through one face:
// F_a(c) counts the beads that crossed from c to c + e_a, so a step -1 from
// c subtracts one from F_a(c - e_a).  Flux word of face (a, c) for type t:
// a W + word(c, t).
template <int CW>
__device__ __forceinline__ void emit_faces(uint32_t *keys, uint32_t *vals, int64_t W, int64_t cell_off,
                                           CellPos o, const CellPos &n, int t, bool on, const SysView &v)
{
    const uint32_t inc = count_inc<CW>(t);
    // x
    {
        const int k = n.x == o.x ? 0 : (n.x == wrap_step(o.x + 1, v.n0) ? 1 : -1);
        CellPos f = o;
        if (k < 0) f.x = n.x;
        agg_insert<kAggSlotsFaces>(keys, vals, (uint32_t)count_word<CW>(cell_off + lin(f, v), t) + 1u,
                                   k > 0 ? inc : 0u - inc, on && k != 0);
        o.x = n.x;
    }
    // y
    {
        const int k = n.y == o.y ? 0 : (n.y == wrap_step(o.y + 1, v.n1) ? 1 : -1);
        CellPos f = o;
        if (k < 0) f.y = n.y;
        agg_insert<kAggSlotsFaces>(keys, vals, (uint32_t)(W + count_word<CW>(cell_off + lin(f, v), t)) + 1u,
                                   k > 0 ? inc : 0u - inc, on && k != 0);
        o.y = n.y;
    }
    // z
    {
        const int k = n.z == o.z ? 0 : (n.z == wrap_step(o.z + 1, v.n2) ? 1 : -1);
        CellPos f = o;
        if (k < 0) f.z = n.z;
        agg_insert<kAggSlotsFaces>(keys, vals, (uint32_t)(2 * W + count_word<CW>(cell_off + lin(f, v), t)) + 1u,
                                   k > 0 ? inc : 0u - inc, on && k != 0);
    }
}

// End of a tile: the density change of the beads whose (cell, type)
// changed -- cell words (density modes 0, 1, 3) or face fluxes (mode 2) --
// merged per wave in LDS, then one device atomic per distinct word with a
// nonzero sum; the acceptance count (into the tile's own counter when
// a.acc_tile is set: acc_prev + this sweep's count) and the cell-range
// status.  Bead j moved from cell o_j with type t_j to cell f_j with type u_j
// (u_j != t_j only for a chain converted in a boundary zone, never in mode
// 2); m_j says that something changed.
template <int CW, int DM>
__device__ __forceinline__ void tile_finish(const SweepArgs &a, int wave, uint32_t sys, int64_t cell_off,
                                            const SysView &v, uint32_t *dcur, uint32_t *agg_keys,
                                            uint32_t *agg_vals, bool m0, const CellPos &o0, const CellPos &f0,
                                            int t0, int u0, bool m1, const CellPos &o1, const CellPos &f1, int t1,
                                            int u1, bool acc0, bool acc1, bool bad, unsigned long long acc_prev)
{
    constexpr int SLOTS = DM == 2 ? kAggSlotsFaces : kAggSlotsCells;
    const int lane = (int)(threadIdx.x & 63);
    if constexpr (DM == 2) {
        emit_faces<CW>(agg_keys, agg_vals, a.count_words, cell_off, o0, f0, t0, m0, v);
        emit_faces<CW>(agg_keys, agg_vals, a.count_words, cell_off, o1, f1, t1, m1, v);
    } else {
        agg_insert<SLOTS>(agg_keys, agg_vals, count_word<CW>(cell_off + lin(o0, v), t0) + 1u, 0u - count_inc<CW>(t0), m0);
        agg_insert<SLOTS>(agg_keys, agg_vals, count_word<CW>(cell_off + lin(f0, v), u0) + 1u, count_inc<CW>(u0), m0);
        agg_insert<SLOTS>(agg_keys, agg_vals, count_word<CW>(cell_off + lin(o1, v), t1) + 1u, 0u - count_inc<CW>(t1), m1);
        agg_insert<SLOTS>(agg_keys, agg_vals, count_word<CW>(cell_off + lin(f1, v), u1) + 1u, count_inc<CW>(u1), m1);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int k = lane; k < SLOTS; k += 64) {
        const uint32_t key = agg_keys[k], v = agg_vals[k];
        if (key != 0u && v != 0u)
            __hip_atomic_fetch_add(dcur + (key - 1u), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    const uint64_t nacc = __popcll(__ballot(acc0)) + __popcll(__ballot(acc1));
    const bool any_bad = __ballot(bad) != 0;
    if (lane == 0) {
        if (nacc && a.acc_tile)   // this wave owns tile `wave` for the sweep
            a.acc_tile[wave] = acc_prev + nacc;
        else if (nacc)
            atomicAdd(a.accept + ((int64_t)sys * kAcceptSlots + (wave % kAcceptSlots)) * kAcceptStride,
                      (unsigned long long)nacc);
        if (any_bad) atomicOr(a.status, ST_CELL_OVERFLOW);
    }
}

// Boundary-zone conversion (Sec. 3.2, "Coupling"), after the moves of a
// sweep: a chain whose binned centre -- the mean of its beads' z-cell
// indexes, compared as the exact integer sum -- lies in the lower zone
// becomes class a, in the upper zone class b.  zf0, zf1: the final z cells of
// this lane's beads.  Returns the chain's new class; the chain's first lane
// stores it and the wave counts the conversions.
__device__ __forceinline__ int zone_convert(const SweepArgs &a, const DevSys &S, uint32_t sys, uint32_t clog,
                                            int cls, bool active, int p, int P, bool has1, int zf0, int zf1)
{
    const int lane = (int)(threadIdx.x & 63);
    int z = active ? zf0 + (has1 ? zf1 : 0) : 0;
    // segmented sum over the chain's P lanes: lane p ends with the sum over
    // [p, P) of its chain, so the chain's first lane holds the total
    for (int o = 1; o < 64; o <<= 1) {
        const int w = __shfl_down(z, o);
        if (p + o < P) z += w;
    }
    const int sum = __shfl(z, lane - p);
    int nc = cls;
    if (S.zone_a && sum < S.zone_a_lim) nc = 0;
    else if (S.zone_b && sum >= S.zone_b_lim) nc = 1;
    const bool conv = active && p == 0 && nc != cls;
    if (conv) a.chain_class[S.chain_off + clog] = (uint8_t)nc;
    const uint64_t to_a = __popcll(__ballot(conv && nc == 0)), to_b = __popcll(__ballot(conv && nc == 1));
    if (lane == 0) {
        if (to_a) atomicAdd(a.conv + 2 * sys, (unsigned long long)to_a);
        if (to_b) atomicAdd(a.conv + 2 * sys + 1, (unsigned long long)to_b);
    }
    return active ? nc : cls;
}

// Trial position outside the walls (z cell outside [wall_lo, wall_hi)).
__device__ __forceinline__ bool outside_walls(const DevSys &S, int zc)
{
    return S.walls && (zc < S.wall_lo || zc >= S.wall_hi);
}

// Umbrella part of the field difference of a bead of type t between its
// trial and its old cell: -lambda/N (target_t(new) - target_t(old)).
__device__ __forceinline__ float umb_step(float coef, float2 tn, float2 to, int t)
{
    return coef * (t ? to.y - tn.y : to.x - tn.x);
}

template <int R, int CW, int DM, bool CPL, bool BT, class Bead>
__device__ __forceinline__ void sweep_tile(const SweepArgs &a, int wave, uint64_t s, const uint32_t *cin,
                                           const uint32_t *dprev, uint32_t *dcur, uint32_t *agg_keys,
                                           uint32_t *agg_vals, Bead b0, Bead b1, uint32_t clog,
                                           unsigned long long acc_prev = 0ull)
{
    const Tile T = tile_table<BT>(a)[wave];
    const DevSys &S = a.systems[T.sys];
    // per-system scalars, read once at the top so that divergent code below
    // keeps them in SGPRs instead of re-reading the table
    const SysView v = make_view(S);
    const FieldCoef fc{S.cAA, S.cAB, S.cBA, S.cBB, S.c0};
    const bool frozen = S.frozen != 0;
    const int64_t cell_off = S.cell_off;
    const int N = S.N, P = S.P;
    const int lane = tile_lane<BT>();
    // lane / P: (lane + 1/2) / P is at least 1/(2P) from an integer, far more
    // than the FP32 error of the product
    const int g = (int)(((float)lane + 0.5f) * S.inv_P);
    const int p = lane - g * P;
    const int nin = min(tile_capacity<BT>(S), S.n_chains - (int)T.chain0);
    const bool active = g < nin;
    const int chain = (int)T.chain0 + (active ? g : 0);
    const int i0 = 2 * p, i1 = 2 * p + 1;
    const bool has1 = active && i1 < N;
    const int64_t slot = S.slot_off + (int64_t)chain * (2 * P) + i0;
    const PosArrays A{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2};
    const Bead ob0 = b0, ob1 = b1;   // the stored state, to write back only what changes

    // logical chain id: keys the random numbers and picks the species, so
    // results do not depend on where a chain sits in memory
    const int cls = chain_cls<CPL>(S, a.chain_class, clog);
    int t0, t1;
    pattern_pair(S, cls, i0, t0, t1);
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const float delta_s = S.delta * 0x1p-23f;
    const Draw d0 = move_draw((uint32_t)i0, clog, (uint32_t)s, S.sys_id, k0, k1, delta_s);
    const Draw d1 = move_draw((uint32_t)i1, clog, (uint32_t)s, S.sys_id, k0, k1, delta_s);
    bool bad = false;
    const CellPos c0 = locate(b0, v, bad);
    const CellPos c1 = locate(b1, v, bad);
    const int old0 = lin(c0, v);
    const int old1 = lin(c1, v);

    // Both trial positions are known before either pass (the odd bead's
    // proposal does not depend on the even pass), so the fields of all four
    // cells are gathered together: one memory latency instead of two.
    const Bead n0 = propose(b0, d0, v);
    const Bead n1 = propose(b1, d1, v);
    const CellPos s0 = step(c0, b0, n0, v), s1 = step(c1, b1, n1, v);
    const int nc0 = lin(s0, v);
    const int nc1 = lin(s1, v);
    // walls: a trial position outside the slab is rejected (and needs no field)
    const bool out0 = CPL && outside_walls(S, zcell(s0, n0)), out1 = CPL && outside_walls(S, zcell(s1, n1));
    const bool g0 = active && nc0 != old0 && !out0, g1 = has1 && nc1 != old1 && !out1;
    float dw0 = 0.0f, dw1 = 0.0f;
    if (frozen) {
        float2 wn0{0.f, 0.f}, wo0{0.f, 0.f}, wn1{0.f, 0.f}, wo1{0.f, 0.f};
        if (g0) { wn0 = a.omega[cell_off + nc0]; wo0 = a.omega[cell_off + old0]; }
        if (g1) { wn1 = a.omega[cell_off + nc1]; wo1 = a.omega[cell_off + old1]; }
        dw0 = t0 ? wn0.y - wo0.y : wn0.x - wo0.x;
        dw1 = t1 ? wn1.y - wo1.y : wn1.x - wo1.x;
    } else {
        RawCount rn0{0u, 0u, 0u, 0u}, ro0{0u, 0u, 0u, 0u}, rn1{0u, 0u, 0u, 0u}, ro1{0u, 0u, 0u, 0u};
        if (g0) {
            rn0 = load_raw<CW, DM == 1>(cin, dprev, cell_off + nc0);
            ro0 = load_raw<CW, DM == 1>(cin, dprev, cell_off + old0);
        }
        if (g1) {
            rn1 = load_raw<CW, DM == 1>(cin, dprev, cell_off + nc1);
            ro1 = load_raw<CW, DM == 1>(cin, dprev, cell_off + old1);
        }
        float2 un0{0.f, 0.f}, uo0{0.f, 0.f}, un1{0.f, 0.f}, uo1{0.f, 0.f};
        const bool umb = CPL && S.umb != 0;
        if (umb) {
            if (g0) { un0 = a.tgt[cell_off + nc0]; uo0 = a.tgt[cell_off + old0]; }
            if (g1) { un1 = a.tgt[cell_off + nc1]; uo1 = a.tgt[cell_off + old1]; }
        }
        if (g0) dw0 = omega_of(fc, counts_of<CW>(rn0), t0) - omega_of(fc, counts_of<CW>(ro0), t0);
        if (g1) dw1 = omega_of(fc, counts_of<CW>(rn1), t1) - omega_of(fc, counts_of<CW>(ro1), t1);
        if (umb) {
            dw0 += umb_step(S.umb_coef, un0, uo0, t0);
            dw1 += umb_step(S.umb_coef, un1, uo1, t1);
        }
    }
    const float kh = S.k_half;

    // even pass: bead 2p, neighbours 2p-1 (previous lane's odd bead) and 2p+1.
    // dE_b = (k/2) sum_j [2 d.(r - r_j) + |d|^2] = (k/2) [2 d.sum_j (r - r_j) + n_j |d|^2]
    bool acc0;
    {
        const Bead left = left_neighbour<BT>(b1);
        const float3 de = bond(n0, b0, v);
        const float3 zero = make_float3(0.0f, 0.0f, 0.0f);
        const float3 bl = p > 0 ? bond(b0, left, v) : zero, br = i1 < N ? bond(b0, b1, v) : zero;
        const float nj = (p > 0 ? 1.0f : 0.0f) + (i1 < N ? 1.0f : 0.0f);
        const float dE = fmaf(fmaf(2.0f, dot3(de, add3(bl, br)), nj * dot3(de, de)), kh, dw0);
        acc0 = active && !out0 && (d0.u < __expf(-dE));
        if (acc0) b0 = n0;
    }
    // odd pass: bead 2p+1, neighbours 2p (this lane, updated) and 2p+2 (next lane)
    bool acc1;
    {
        const Bead right = right_neighbour<BT>(b0);
        const float3 de = bond(n1, b1, v);
        const float3 br = i1 + 1 < N ? bond(b1, right, v) : make_float3(0.0f, 0.0f, 0.0f);
        const float nj = i1 + 1 < N ? 2.0f : 1.0f;
        const float dE = fmaf(fmaf(2.0f, dot3(de, add3(bond(b1, b0, v), br)), nj * dot3(de, de)), kh, dw1);
        acc1 = has1 && !out1 && (d1.u < __expf(-dE));
        if (acc1) b1 = n1;
    }
    if (active) store_moved(A, slot, b0, b1, ob0, ob1, acc0 || acc1);
    // final cells: without coupling a change implies an accepted move, so the
    // trial cells serve (and the selection costs no registers)
    const CellPos f0 = CPL ? (acc0 ? s0 : c0) : s0, f1 = CPL ? (acc1 ? s1 : c1) : s1;
    int u0 = t0, u1 = t1;
    if (CPL && !BT && S.zones) {   // (the host never packs contexts with zones)
        const int ncls = zone_convert(a, S, T.sys, clog, cls, active, p, P, has1, zcell(f0, b0), zcell(f1, b1));
        pattern_pair(S, ncls, i0, u0, u1);
    }
    tile_finish<CW, DM>(a, BT ? wave * 16 + (int)(threadIdx.x >> 6) : wave, T.sys, cell_off, v, dcur, agg_keys, agg_vals,
                        active && ((acc0 && nc0 != old0) || u0 != t0), c0, f0, t0, u0,
                        has1 && ((acc1 && nc1 != old1) || u1 != t1), c1, f1, t1, u1, acc0, acc1, active && bad, acc_prev);
}

// ---------------------------------------------------------------------------
// Stream tiles (uniform moves, no coupling)
// ---------------------------------------------------------------------------
// The lanes of a system form one stream in chain order (chain c holds lanes
// [c P, (c + 1) P)), so chains run across wave boundaries and no lane idles
// but in a system's last wave.  Wave w moves the 62 stream lanes
// [62 w, 62 w + 62) on its lanes 1..62; lane 0 holds the stream lane before
// them and lane 63 the one after, which take every step of the sweep but
// store nothing, update no count and count no acceptance.  Lane 1's even
// bead reads lane 0's odd bead (unmoved in the even pass), and lane 62's odd
// bead reads lane 63's even bead after lane 63 has made that bead's even move
// with the same draw, stored state, frozen counts and arithmetic as the wave
// that owns it, so the same decision.  The owners of the two overlap lanes
// rewrite them during the same sweep, so the overlap lanes read them from
// the halo copy taken before the sweep (halo_index): tile w - 1's last and
// tile w + 1's first owned lane.  A stream tile names its system (low 24
// bits), the pair index of its first owned lane within that lane's chain
// (high 8 bits) and that chain.
__device__ __forceinline__ uint32_t stile_sys(const Tile &T) { return T.sys & 0xFFFFFFu; }

struct StreamLane {
    int chain, p;
    bool valid;     // a bead pair of the system: takes every step
    bool own;       // and belongs to this wave: stores and counts
};

__device__ __forceinline__ StreamLane stream_lane(const Tile &T, const DevSys &S, int lane)
{
    const int P = S.P;
    // stream lane 62 w - 1 + lane, as (chain0 - 1 + gr, q - gr P) with q >= 0
    const int q = (int)(T.sys >> 24) + lane - 1 + P;            // < 2 P + 63
    const int gr = (int)(((float)q + 0.5f) * S.inv_P);
    StreamLane L;
    L.chain = (int)T.chain0 - 1 + gr;
    L.p = q - gr * P;
    L.valid = L.chain >= 0 && L.chain < S.n_chains;
    L.own = L.valid && lane >= 1 && lane <= kStreamLanes;
    return L;
}

// One bead pair in the halo: component k of both beads in one 8-byte word,
// the components of one side contiguous (16-byte accesses).
__device__ __forceinline__ void halo_put(uint2 *h, int buf, int64_t tile, int side, int64_t cap, const BeadF32 &a,
                                         const BeadF32 &b)
{
    uint2 *e = h + halo_index(buf, 0, tile, side, cap);
    *reinterpret_cast<uint4 *>(e) = make_uint4(__float_as_uint(a.x), __float_as_uint(b.x), __float_as_uint(a.y),
                                               __float_as_uint(b.y));
    e[2] = make_uint2(__float_as_uint(a.z), __float_as_uint(b.z));
}
__device__ __forceinline__ void halo_put(uint2 *h, int buf, int64_t tile, int side, int64_t cap, const BeadCell &a,
                                         const BeadCell &b)
{
    uint4 *e = reinterpret_cast<uint4 *>(h + halo_index(buf, 0, tile, side, cap));
    e[0] = make_uint4(__float_as_uint(a.ox), __float_as_uint(b.ox), __float_as_uint(a.oy), __float_as_uint(b.oy));
    e[1] = make_uint4(__float_as_uint(a.oz), __float_as_uint(b.oz), (uint32_t)a.cx, (uint32_t)b.cx);
    e[2] = make_uint4((uint32_t)a.cy, (uint32_t)b.cy, (uint32_t)a.cz, (uint32_t)b.cz);
}
__device__ __forceinline__ void halo_get(const uint2 *h, int buf, int64_t tile, int side, int64_t cap, BeadF32 &a,
                                         BeadF32 &b)
{
    const uint2 *e = h + halo_index(buf, 0, tile, side, cap);
    const uint4 xy = *reinterpret_cast<const uint4 *>(e);
    const uint2 z = e[2];
    a = BeadF32{__uint_as_float(xy.x), __uint_as_float(xy.z), __uint_as_float(z.x)};
    b = BeadF32{__uint_as_float(xy.y), __uint_as_float(xy.w), __uint_as_float(z.y)};
}
__device__ __forceinline__ void halo_get(const uint2 *h, int buf, int64_t tile, int side, int64_t cap, BeadCell &a,
                                         BeadCell &b)
{
    const uint4 *e = reinterpret_cast<const uint4 *>(h + halo_index(buf, 0, tile, side, cap));
    const uint4 u = e[0], v = e[1], w = e[2];
    a = BeadCell{(int)v.z, (int)w.x, (int)w.z, __uint_as_float(u.x), __uint_as_float(u.z), __uint_as_float(v.x)};
    b = BeadCell{(int)v.w, (int)w.y, (int)w.w, __uint_as_float(u.y), __uint_as_float(u.w), __uint_as_float(v.y)};
}

// Owned lanes load their pairs from the position arrays; the overlap lanes
// (valid only next to a tile of the same system: lane 0 when the tile does
// not start its system's stream, lane 63 when the stream goes on) load them
// from halo buffer s mod 2.
template <class Bead>
__device__ __forceinline__ void stream_load(const SweepArgs &a, int tile, uint64_t s, Bead &b0, Bead &b1,
                                            uint32_t &clog)
{
    const Tile T = a.ptiles[tile];
    const DevSys &S = a.systems[stile_sys(T)];
    const int lane = (int)(threadIdx.x & 63);
    const StreamLane L = stream_lane(T, S, lane);
    clog = a.chain_id[S.chain_off + (L.valid ? L.chain : (int)T.chain0)];
    b0 = Bead{};
    b1 = Bead{};
    if (L.own)
        load_pair(PosArrays{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2}, S.slot_off + (int64_t)L.chain * (2 * S.P) + 2 * L.p,
                  b0, b1);
    else if (L.valid)
        halo_get(a.halo, (int)(s & 1), lane == 0 ? tile - 1 : tile + 1, lane == 0 ? 1 : 0, a.halo_cap, b0, b1);
}

template <int R, int CW, int DM, class Bead>
__device__ __forceinline__ void sweep_tile_stream(const SweepArgs &a, int wave, uint64_t s, const uint32_t *cin,
                                                  const uint32_t *dprev, uint32_t *dcur, uint32_t *agg_keys,
                                                  uint32_t *agg_vals, Bead b0, Bead b1, uint32_t clog,
                                                  unsigned long long acc_prev)
{
    const Tile T = a.ptiles[wave];
    const uint32_t sys = stile_sys(T);
    const DevSys &S = a.systems[sys];
    const SysView v = make_view(S);
    const FieldCoef fc{S.cAA, S.cAB, S.cBA, S.cBB, S.c0};
    const bool frozen = S.frozen != 0;
    const int64_t cell_off = S.cell_off;
    const int N = S.N, P = S.P;
    const StreamLane L = stream_lane(T, S, (int)(threadIdx.x & 63));
    const bool valid = L.valid, own = L.own;
    const int p = L.p;
    const int i0 = 2 * p, i1 = 2 * p + 1;
    const bool has1 = valid && i1 < N;
    const int64_t slot = S.slot_off + (int64_t)(valid ? L.chain : 0) * (2 * P) + 2 * p;
    const PosArrays A{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2};
    const Bead ob0 = b0, ob1 = b1;

    const int cls = chain_cls<false>(S, a.chain_class, clog);
    int t0, t1;
    pattern_pair(S, cls, i0, t0, t1);
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const float delta_s = S.delta * 0x1p-23f;
    const Draw d0 = move_draw((uint32_t)i0, clog, (uint32_t)s, S.sys_id, k0, k1, delta_s);
    const Draw d1 = move_draw((uint32_t)i1, clog, (uint32_t)s, S.sys_id, k0, k1, delta_s);
    bool bad = false;
    const CellPos c0 = locate(b0, v, bad);
    const CellPos c1 = locate(b1, v, bad);
    const int old0 = lin(c0, v), old1 = lin(c1, v);
    const Bead n0 = propose(b0, d0, v);
    const Bead n1 = propose(b1, d1, v);
    const CellPos s0 = step(c0, b0, n0, v), s1 = step(c1, b1, n1, v);
    const int nc0 = lin(s0, v), nc1 = lin(s1, v);
    const bool g0 = valid && nc0 != old0, g1 = has1 && nc1 != old1;
    float dw0 = 0.0f, dw1 = 0.0f;
    if (frozen) {
        float2 wn0{0.f, 0.f}, wo0{0.f, 0.f}, wn1{0.f, 0.f}, wo1{0.f, 0.f};
        if (g0) { wn0 = a.omega[cell_off + nc0]; wo0 = a.omega[cell_off + old0]; }
        if (g1) { wn1 = a.omega[cell_off + nc1]; wo1 = a.omega[cell_off + old1]; }
        dw0 = t0 ? wn0.y - wo0.y : wn0.x - wo0.x;
        dw1 = t1 ? wn1.y - wo1.y : wn1.x - wo1.x;
    } else {
        RawCount rn0{0u, 0u, 0u, 0u}, ro0{0u, 0u, 0u, 0u}, rn1{0u, 0u, 0u, 0u}, ro1{0u, 0u, 0u, 0u};
        if (g0) {
            rn0 = load_raw<CW, DM == 1>(cin, dprev, cell_off + nc0);
            ro0 = load_raw<CW, DM == 1>(cin, dprev, cell_off + old0);
        }
        if (g1) {
            rn1 = load_raw<CW, DM == 1>(cin, dprev, cell_off + nc1);
            ro1 = load_raw<CW, DM == 1>(cin, dprev, cell_off + old1);
        }
        if (g0) dw0 = omega_of(fc, counts_of<CW>(rn0), t0) - omega_of(fc, counts_of<CW>(ro0), t0);
        if (g1) dw1 = omega_of(fc, counts_of<CW>(rn1), t1) - omega_of(fc, counts_of<CW>(ro1), t1);
    }
    const float kh = S.k_half;
    const float3 zero = make_float3(0.0f, 0.0f, 0.0f);

    // even pass: bead 2p, neighbours 2p-1 (previous lane) and 2p+1
    bool acc0;
    {
        const Bead left = left_neighbour<false>(b1);
        const float3 de = bond(n0, b0, v);
        const float3 bl = p > 0 ? bond(b0, left, v) : zero, br = i1 < N ? bond(b0, b1, v) : zero;
        const float nj = (p > 0 ? 1.0f : 0.0f) + (i1 < N ? 1.0f : 0.0f);
        const float dE = fmaf(fmaf(2.0f, dot3(de, add3(bl, br)), nj * dot3(de, de)), kh, dw0);
        acc0 = valid && (d0.u < __expf(-dE));
        if (acc0) b0 = n0;
    }
    // odd pass: bead 2p+1, neighbours 2p (this lane, updated) and 2p+2 (next lane)
    bool acc1;
    {
        const Bead right = right_neighbour<false>(b0);
        const float3 de = bond(n1, b1, v);
        const float3 br = i1 + 1 < N ? bond(b1, right, v) : zero;
        const float nj = i1 + 1 < N ? 2.0f : 1.0f;
        const float dE = fmaf(fmaf(2.0f, dot3(de, add3(bond(b1, b0, v), br)), nj * dot3(de, de)), kh, dw1);
        acc1 = has1 && (d1.u < __expf(-dE));
        if (acc1) b1 = n1;
    }
    const bool own1 = own && has1;
    if (own) store_moved(A, slot, b0, b1, ob0, ob1, acc0 || acc1);
    // the end lanes' pairs for the overlap lanes of the next sweep
    const int lane = (int)(threadIdx.x & 63);
    if (own && (lane == 1 || lane == kStreamLanes))
        halo_put(a.halo, (int)((s + 1) & 1), wave, lane == 1 ? 0 : 1, a.halo_cap, b0, b1);
    tile_finish<CW, DM>(a, wave, sys, cell_off, v, dcur, agg_keys, agg_vals, own && acc0 && nc0 != old0, c0, s0, t0,
                        t0, own1 && acc1 && nc1 != old1, c1, s1, t1, t1, own && acc0, own1 && acc1, own && bad, acc_prev);
}

// Fill halo buffer a.buf from the position arrays: one thread per stream
// tile and end lane (side 0: lane 1, side 1: lane 62), for the lanes that
// belong to their system.
template <class Bead>
__global__ __launch_bounds__(256) void k_stream_halo(HaloArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * (int64_t)a.n_ptiles) return;
    const int64_t tile = i >> 1;
    const int side = (int)(i & 1);
    const Tile T = a.ptiles[tile];
    const DevSys &S = a.systems[stile_sys(T)];
    const StreamLane L = stream_lane(T, S, side == 0 ? 1 : kStreamLanes);
    if (!L.own) return;
    Bead b0, b1;
    load_pair(PosArrays{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2}, S.slot_off + (int64_t)L.chain * (2 * S.P) + 2 * L.p,
              b0, b1);
    halo_put(a.halo, a.buf, tile, side, a.halo_cap, b0, b1);
}

// ---------------------------------------------------------------------------
// Bond-force-biased ("smart") moves (Sec. 2; Rossky, Doll and Friedman 1978)
// ---------------------------------------------------------------------------
// Three standard normals by Box-Muller (FP64) on the Philox block with counter
// (bead, chain, sweep, system): words 0, 1 give the first two, words 2, 3 the
// third; the acceptance variate is word 0 of the block with counter
// (bead + 256, chain, sweep, system) (beads are numbered below 128).
__device__ __forceinline__ void smc_draw(uint32_t bead, uint32_t chain, uint32_t sweep, uint32_t sys,
                                         uint32_t k0, uint32_t k1, double xi[3], float &u)
{
    const double two_pi = 6.283185307179586476925286766559;
    const uint4 w = philox4x32_10(make_uint4(bead, chain, sweep, sys), k0, k1);
    const double u1 = ((double)(w.x >> 8) + 0.5) * 0x1p-24;
    const double u2 = (double)(w.y >> 8) * 0x1p-24;
    const double u3 = ((double)(w.z >> 8) + 0.5) * 0x1p-24;
    const double u4 = (double)(w.w >> 8) * 0x1p-24;
    const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    xi[0] = r1 * cos(two_pi * u2);
    xi[1] = r1 * sin(two_pi * u2);
    xi[2] = r2 * cos(two_pi * u4);
    const uint4 w2 = philox4x32_10(make_uint4(bead + 256u, chain, sweep, sys), k0, k1);
    u = (float)(w2.x >> 8) * 0x1p-24f;
}

// Position in FP64 from the stored representation (exact for FP32; cell
// mode: cell * edge + offset with the FP32 edge).
__device__ __forceinline__ double3 pos64(const BeadF32 &a, const SysView &)
{
    return make_double3((double)a.x, (double)a.y, (double)a.z);
}
__device__ __forceinline__ double3 pos64(const BeadCell &a, const SysView &v)
{
    return make_double3((double)a.cx * (double)v.e0 + (double)a.ox, (double)a.cy * (double)v.e1 + (double)a.oy,
                        (double)a.cz * (double)v.e2 + (double)a.oz);
}

// One smart move of bead b with neighbours nl (if hl) and nr (if hr), which
// hold still.  Returns the trial state and whether the displacement stays
// below 0.99 cell edges; F gets the bond force at b (FP64).
template <class Bead>
__device__ __forceinline__ Bead smc_propose(const Bead &b, const Bead &nl, bool hl, const Bead &nr, bool hr,
                                            const DevSys &S, const SysView &v, const double xi[3], double3 &F,
                                            bool &inside)
{
    const double3 r = pos64(b, v);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (hl) {
        const double3 q = pos64(nl, v);
        fx += q.x - r.x; fy += q.y - r.y; fz += q.z - r.z;
    }
    if (hr) {
        const double3 q = pos64(nr, v);
        fx += q.x - r.x; fy += q.y - r.y; fz += q.z - r.z;
    }
    F = make_double3(S.k_spring * fx, S.k_spring * fy, S.k_spring * fz);
    Draw d;
    d.dx = (float)(S.smc_A * F.x + S.smc_s2A * xi[0]);
    d.dy = (float)(S.smc_A * F.y + S.smc_s2A * xi[1]);
    d.dz = (float)(S.smc_A * F.z + S.smc_s2A * xi[2]);
    d.u = 0.0f;
    // a displacement of 0.99 cell edges or more is rejected: the condition is
    // symmetric in r and r', so detailed balance holds, and a kept trial move
    // changes each cell index by at most one
    inside = fabsf(d.dx) < S.dmax[0] && fabsf(d.dy) < S.dmax[1] && fabsf(d.dz) < S.dmax[2];
    if (!inside) d.dx = d.dy = d.dz = 0.0f;
    return propose(b, d, v);
}

// log of q(r'->r) / q(r->r') for q(r->r') ~ exp(-|r'-r-A F(r)|^2 / (4A)),
// with de the stored displacement and F(r') = F(r) - k n_nb de (FP32).
__device__ __forceinline__ float smc_log_ratio(const DevSys &S, float3 de, double3 F, int n_nb)
{
    const float A = S.smc_Af, kn = S.k_f * (float)n_nb;
    const float fx = (float)F.x, fy = (float)F.y, fz = (float)F.z;
    const float3 f = make_float3(de.x - A * fx, de.y - A * fy, de.z - A * fz);
    const float3 r = make_float3(de.x + A * (fx - kn * de.x), de.y + A * (fy - kn * de.y), de.z + A * (fz - kn * de.z));
    return (dot3(f, f) - dot3(r, r)) * S.smc_inv4A;
}

// Field difference between a trial cell and the old cell of one bead.
template <int CW, int DM>
__device__ __forceinline__ float field_step(const SweepArgs &a, bool frozen, const FieldCoef &fc,
                                            const uint32_t *cin, const uint32_t *dprev, int64_t cell_off,
                                            int nc, int old, int t, bool gather, bool umb, float umb_coef)
{
    float dw = 0.0f;
    if (frozen) {
        float2 wn{0.f, 0.f}, wo{0.f, 0.f};
        if (gather) { wn = a.omega[cell_off + nc]; wo = a.omega[cell_off + old]; }
        dw = t ? wn.y - wo.y : wn.x - wo.x;
    } else {
        RawCount rn{0u, 0u, 0u, 0u}, ro{0u, 0u, 0u, 0u};
        if (gather) {
            rn = load_raw<CW, DM == 1>(cin, dprev, cell_off + nc);
            ro = load_raw<CW, DM == 1>(cin, dprev, cell_off + old);
            float2 un{0.f, 0.f}, uo{0.f, 0.f};
            if (umb) { un = a.tgt[cell_off + nc]; uo = a.tgt[cell_off + old]; }
            dw = omega_of(fc, counts_of<CW>(rn), t) - omega_of(fc, counts_of<CW>(ro), t);
            if (umb) dw += umb_step(umb_coef, un, uo, t);
        }
    }
    return dw;
}

// One wave tile with smart moves.  The odd bead's proposal depends on the
// even pass (its bond force uses the moved even beads), so the two passes
// gather their fields one after the other.
template <int R, int CW, int DM, bool CPL, bool BT, class Bead>
__device__ __forceinline__ void sweep_tile_smc(const SweepArgs &a, int wave, uint64_t s, const uint32_t *cin,
                                               const uint32_t *dprev, uint32_t *dcur, uint32_t *agg_keys,
                                               uint32_t *agg_vals, Bead b0, Bead b1, uint32_t clog)
{
    const Tile T = tile_table<BT>(a)[wave];
    const DevSys &S = a.systems[T.sys];
    const SysView v = make_view(S);
    const FieldCoef fc{S.cAA, S.cAB, S.cBA, S.cBB, S.c0};
    const bool frozen = S.frozen != 0;
    const int64_t cell_off = S.cell_off;
    const int N = S.N, P = S.P;
    const int lane = tile_lane<BT>();
    const int g = (int)(((float)lane + 0.5f) * S.inv_P);
    const int p = lane - g * P;
    const int nin = min(tile_capacity<BT>(S), S.n_chains - (int)T.chain0);
    const bool active = g < nin;
    const int chain = (int)T.chain0 + (active ? g : 0);
    const int i0 = 2 * p, i1 = 2 * p + 1;
    const bool has1 = active && i1 < N;
    const int64_t slot = S.slot_off + (int64_t)chain * (2 * P) + i0;
    const PosArrays A{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2};
    const Bead ob0 = b0, ob1 = b1;   // the stored state, to write back only what changes
    const int cls = chain_cls<CPL>(S, a.chain_class, clog);
    const int t0 = pattern_type(S, cls, i0);
    const int t1 = pattern_type(S, cls, i1 < N ? i1 : i0);
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const float kh = S.k_half;
    const bool umb = CPL && S.umb != 0;
    const float umb_coef = S.umb_coef;
    bool bad = false;
    const CellPos c0 = locate(b0, v, bad);
    const CellPos c1 = locate(b1, v, bad);
    const int old0 = lin(c0, v);
    const int old1 = lin(c1, v);

    // even pass: bead 2p, neighbours 2p-1 (previous lane's odd bead) and 2p+1
    bool acc0;
    int nc0;
    CellPos s0;
    {
        double xi[3];
        float u;
        smc_draw((uint32_t)i0, clog, (uint32_t)s, S.sys_id, k0, k1, xi, u);
        const Bead left = left_neighbour<BT>(b1);
        const bool hl = p > 0, hr = i1 < N;
        double3 F;
        bool inside;
        const Bead n0 = smc_propose(b0, left, hl, b1, hr, S, v, xi, F, inside);
        s0 = step(c0, b0, n0, v);
        nc0 = lin(s0, v);
        if (CPL) inside = inside && !outside_walls(S, zcell(s0, n0));
        const float dw = field_step<CW, DM>(a, frozen, fc, cin, dprev, cell_off, nc0, old0, t0,
                                            active && inside && nc0 != old0, umb, umb_coef);
        const float3 de = bond(n0, b0, v);
        const float dd = dot3(de, de);
        float dE = 0.0f;
        if (hl) dE += 2.0f * dot3(de, bond(b0, left, v)) + dd;
        if (hr) dE += 2.0f * dot3(de, bond(b0, b1, v)) + dd;
        dE = dE * kh + dw - smc_log_ratio(S, de, F, (hl ? 1 : 0) + (hr ? 1 : 0));
        acc0 = active && inside && (u < __expf(-dE));
        if (acc0) b0 = n0;
    }
    // odd pass: bead 2p+1, neighbours 2p (this lane, moved) and 2p+2 (next lane)
    bool acc1;
    int nc1;
    CellPos s1;
    {
        double xi[3];
        float u;
        smc_draw((uint32_t)i1, clog, (uint32_t)s, S.sys_id, k0, k1, xi, u);
        const Bead right = right_neighbour<BT>(b0);
        const bool hr = i1 + 1 < N;
        double3 F;
        bool inside;
        const Bead n1 = smc_propose(b1, b0, true, right, hr, S, v, xi, F, inside);
        s1 = step(c1, b1, n1, v);
        nc1 = lin(s1, v);
        if (CPL) inside = inside && !outside_walls(S, zcell(s1, n1));
        const float dw = field_step<CW, DM>(a, frozen, fc, cin, dprev, cell_off, nc1, old1, t1,
                                            has1 && inside && nc1 != old1, umb, umb_coef);
        const float3 de = bond(n1, b1, v);
        const float dd = dot3(de, de);
        float dE = 2.0f * dot3(de, bond(b1, b0, v)) + dd;
        if (hr) dE += 2.0f * dot3(de, bond(b1, right, v)) + dd;
        dE = dE * kh + dw - smc_log_ratio(S, de, F, 1 + (hr ? 1 : 0));
        acc1 = has1 && inside && (u < __expf(-dE));
        if (acc1) b1 = n1;
    }
    if (active) store_moved(A, slot, b0, b1, ob0, ob1, acc0 || acc1);
    // final cells: without coupling a change implies an accepted move, so the
    // trial cells serve (and the selection costs no registers)
    const CellPos f0 = CPL ? (acc0 ? s0 : c0) : s0, f1 = CPL ? (acc1 ? s1 : c1) : s1;
    int u0 = t0, u1 = t1;
    if (CPL && !BT && S.zones) {   // (the host never packs contexts with zones)
        const int ncls = zone_convert(a, S, T.sys, clog, cls, active, p, P, has1, zcell(f0, b0), zcell(f1, b1));
        u0 = pattern_type(S, ncls, i0);
        u1 = pattern_type(S, ncls, i1 < N ? i1 : i0);
    }
    tile_finish<CW, DM>(a, BT ? wave * 16 + (int)(threadIdx.x >> 6) : wave, T.sys, cell_off, v, dcur, agg_keys, agg_vals,
                        active && ((acc0 && nc0 != old0) || u0 != t0), c0, f0, t0, u0,
                        has1 && ((acc1 && nc1 != old1) || u1 != t1), c1, f1, t1, u1, acc0, acc1, active && bad, 0ull);
}

// The sweep kernel: one launch per sweep for every system.  With one tile
// per wave (the default) wave w moves tile w; with a resident grid (fewer
// waves) the waves walk the tiles grid-stride, each prefetching its next
// tile's positions.  One tile's state is live at a
// time, which keeps the register count (and so the occupancy) of the
// one-tile case.  With FI every thread also folds count words of the
// previous sweep: the first word's loads are issued before the move work
// and its stores after it, so they overlap.
template <int R, int CW, bool LOOP, int DM, bool SMC, bool CPL, bool BT, bool ST = false>
__device__ __forceinline__ void sweep_body(const SweepArgs &a)
{
    using Bead = typename std::conditional<R == REPR_F32, BeadF32, BeadCell>::type;
    constexpr bool FI = DM == 1;
    constexpr int SLOTS = DM == 2 ? kAggSlotsFaces : kAggSlotsCells;
    const uint64_t s = *a.sweep_ctr + a.rel;
    const int64_t W = a.count_words;
    // mode 1: counts of sweep s are B[s-1] + D[s-1]; this sweep adds to D[s],
    // writes B[s] and clears D[s+1] (last read by sweep s-1).  Mode 2: the
    // face fluxes of sweep s go to flux buffer s mod 2 (three W-word arrays).
    // Mode 3: the counts are B[s mod 2]; the changes go straight into its
    // mirror B[(s+1) mod 2], which holds the same counts when the sweep
    // starts and is read by no gather of this sweep.
    const uint32_t *cin = FI ? a.base + ((s + 1) & 1) * W : (DM == 3 ? a.base + (s & 1) * W : a.base);
    const uint32_t *dprev = FI ? a.delta + ((s + 2) % 3) * W : nullptr;
    uint32_t *dcur = FI ? a.delta + (s % 3) * W
                        : (DM == 2 ? a.flux + (s & 1) * 3 * W : (DM == 3 ? a.base + ((s + 1) & 1) * W : a.delta));
    const int wave = BT ? block_tile(a.xcd_remap) : wave_tile(a.waves_per_block, a.xcd_remap);
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // this wave's aggregation table (2 SLOTS words of dynamic LDS per wave)
    HIP_DYNAMIC_SHARED(uint32_t, agg_lds)
    uint32_t *agg_keys = agg_lds + (threadIdx.x >> 6) * (2 * SLOTS);
    uint32_t *agg_vals = agg_keys + SLOTS;
    uint32_t fb = 0u, fd = 0u;
    if constexpr (FI) {
        if (gtid < W) {
            fb = cin[gtid];
            fd = dprev[gtid];
        }
    }
    if constexpr (LOOP) {
        // Resident waves walk the tiles grid-stride (wave, wave + n_waves,
        // ...), so the tiles in flight at any time are neighbours in the
        // spatial chain order and their field gathers share the L2.  Software
        // pipeline: the positions of a wave's next tile are loaded before
        // the current tile's field gathers, so their latency overlaps the
        // current tile's work.
        const int n_waves = (int)gridDim.x * a.waves_per_block;
        Bead nb0, nb1;
        uint32_t nclog = 0u;
        if (wave < a.n_tiles) tile_load<false>(a, wave, nb0, nb1, nclog);
        for (int t = wave; t < a.n_tiles; t += n_waves) {
            const Bead b0 = nb0, b1 = nb1;
            const uint32_t clog = nclog;
            if (t + n_waves < a.n_tiles) tile_load<false>(a, t + n_waves, nb0, nb1, nclog);
            agg_clear<SLOTS>(agg_keys, agg_vals);
            if (SMC && a.systems[a.tiles[t].sys].smc)
                sweep_tile_smc<R, CW, DM, CPL, false>(a, t, s, cin, dprev, dcur, agg_keys, agg_vals, b0, b1, clog);
            else
                sweep_tile<R, CW, DM, CPL, false>(a, t, s, cin, dprev, dcur, agg_keys, agg_vals, b0, b1, clog);
        }
    } else {
        // block tiles: the test is uniform over the block, so every thread
        // of a working block reaches the barriers of the tile
        // the tile's acceptance count is read with its positions (see
        // counts_per_tile; a.acc_tile is null for the other kernels)
        if constexpr (ST) {
            if (wave < a.n_ptiles) {
                Bead b0, b1;
                uint32_t clog;
                stream_load(a, wave, s, b0, b1, clog);
                const unsigned long long accp = a.acc_tile ? a.acc_tile[wave] : 0ull;
                agg_clear<SLOTS>(agg_keys, agg_vals);
                sweep_tile_stream<R, CW, DM>(a, wave, s, cin, dprev, dcur, agg_keys, agg_vals, b0, b1, clog, accp);
            }
        } else if (wave < (BT ? a.n_ptiles : a.n_tiles)) {
            Bead b0, b1;
            uint32_t clog;
            tile_load<BT>(a, wave, b0, b1, clog);
            const unsigned long long accp = !BT && a.acc_tile ? a.acc_tile[wave] : 0ull;
            agg_clear<SLOTS>(agg_keys, agg_vals);
            if (SMC && a.systems[tile_table<BT>(a)[wave].sys].smc)
                sweep_tile_smc<R, CW, DM, CPL, BT>(a, wave, s, cin, dprev, dcur, agg_keys, agg_vals, b0, b1, clog);
            else
                sweep_tile<R, CW, DM, CPL, BT>(a, wave, s, cin, dprev, dcur, agg_keys, agg_vals, b0, b1, clog, accp);
        }
    }
    if constexpr (FI) {
        uint32_t *bcur = a.base + (s & 1) * W;
        uint32_t *dnext = a.delta + ((s + 1) % 3) * W;
        const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
        bool ovf = false;
        if (gtid < W) {
            uint32_t w;
            ovf |= fold_word<CW>(fb, fd, w);
            bcur[gtid] = w;
            dnext[gtid] = 0u;
        }
        for (int64_t i = gtid + nthreads; i < W; i += nthreads) {
            uint32_t w;
            ovf |= fold_word<CW>(cin[i], dprev[i], w);
            bcur[i] = w;
            dnext[i] = 0u;
        }
        if (ovf) atomicOr(a.status, ST_COUNT_OVERFLOW);
    }
    if constexpr (DM == 2) {
        // clear the flux buffer of sweep s + 1 (folded after sweep s - 1);
        // its 3 W words are a multiple of 4 and 16-byte aligned
        uint4 *fn = reinterpret_cast<uint4 *>(a.flux + ((s + 1) & 1) * 3 * W);
        const int64_t n4 = 3 * W / 4, nthreads = (int64_t)gridDim.x * blockDim.x;
        for (int64_t i = gtid; i < n4; i += nthreads) fn[i] = make_uint4(0u, 0u, 0u, 0u);
    }
}

template <int R, int CW, bool LOOP, int DM, bool SMC, bool CPL, bool BT>
__global__ __launch_bounds__(1024) void k_sweep(SweepArgs a)
{
    sweep_body<R, CW, LOOP, DM, SMC, CPL, BT>(a);
}

// The plain one-tile-per-wave sweep (uniform moves, no coupling) fits in 64
// VGPRs: it asks for eight waves per SIMD, the most a SIMD holds (the SGPRs
// beyond that budget live in VGPR lanes).  The sweep waits on memory, and
// the eighth wave hides enough of it to pay for those moves.
template <int R, int CW, int DM>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sweep_plain(SweepArgs a)
{
    sweep_body<R, CW, false, DM, false, false, false, false>(a);
}

// Stream tiles, with the same register budget.
template <int R, int CW, int DM>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sweep_stream(SweepArgs a)
{
    sweep_body<R, CW, false, DM, false, false, false, true>(a);
}

// Density mode 2: counts += divergence of the face fluxes of sweep s, per
// cell c of one system: n(c) += sum_a F_a(c - e_a) - F_a(c) (modular uint32,
// both species at once for packed counts), with the range check of the
// other folds.  (The sweep kernel of sweep s + 1 clears these fluxes.)  One
// block per chunk of kFoldChunk cells of one system.
template <int CW>
__global__ __launch_bounds__(256) void k_fold_faces(FoldFacesArgs a)
{
    const FoldChunk ch = a.chunks[blockIdx.x];
    const DevSys &S = a.systems[ch.sys];
    const uint64_t s = *a.sweep_ctr + a.rel;
    const int64_t W = a.count_words;
    const uint32_t *F = a.flux + (s & 1) * 3 * W;
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int64_t M = S.n_cells;
    const int64_t end = ch.first + kFoldChunk < M ? ch.first + kFoldChunk : M;
    constexpr int WPC = CW == COUNT_U16 ? 1 : 2;
    // cell -> (ix, iy, iz) by FP64 reciprocals with one correction step
    // (exact: cells < 2^31), not by integer division
    const double inz = 1.0 / (double)nz, iny = 1.0 / (double)ny;
    bool ovf = false;
    for (int64_t c = ch.first + threadIdx.x; c < end; c += blockDim.x) {
        const int ci = (int)c;
        int r = (int)((double)ci * inz);
        int iz = ci - r * nz;
        if (iz < 0) { iz += nz; --r; } else if (iz >= nz) { iz -= nz; ++r; }
        int ix = (int)((double)r * iny);
        int iy = r - ix * ny;
        if (iy < 0) { iy += ny; --ix; } else if (iy >= ny) { iy -= ny; ++ix; }
        const int64_t cxm = ((int64_t)(ix == 0 ? nx - 1 : ix - 1) * ny + iy) * nz + iz;
        const int64_t cym = ((int64_t)ix * ny + (iy == 0 ? ny - 1 : iy - 1)) * nz + iz;
        const int64_t czm = ((int64_t)ix * ny + iy) * nz + (iz == 0 ? nz - 1 : iz - 1);
        for (int j = 0; j < WPC; ++j) {
            const int64_t w = WPC * (S.cell_off + c) + j;
            const int64_t wx = WPC * (S.cell_off + cxm) + j, wy = WPC * (S.cell_off + cym) + j,
                          wz = WPC * (S.cell_off + czm) + j;
            const uint32_t d = (F[wx] - F[w]) + (F[W + wy] - F[W + w]) + (F[2 * W + wz] - F[2 * W + w]);
            uint32_t out;
            ovf |= fold_word<CW>(a.counts[w], d, out);
            a.counts[w] = out;
        }
    }
    if (ovf) atomicOr(a.status, ST_COUNT_OVERFLOW);
}

// Fold a density delta into counts and clear it: out = in + delta (out may
// be in), with 16-byte accesses (the arrays are 256-byte aligned), then the
// words past the last full quadruple.
template <int CW>
__global__ __launch_bounds__(256) void k_fold(const uint32_t *in, uint32_t *delta, uint32_t *counts, int64_t n,
                                              uint32_t *status)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = n >> 2;
    const uint4 *i4 = reinterpret_cast<const uint4 *>(in);
    uint4 *c4 = reinterpret_cast<uint4 *>(counts);
    uint4 *d4 = reinterpret_cast<uint4 *>(delta);
    bool ovf = false;
    for (int64_t i = tid; i < n4; i += stride) {
        const uint4 b = i4[i], d = d4[i];
        uint4 w;
        ovf |= fold_word<CW>(b.x, d.x, w.x);
        ovf |= fold_word<CW>(b.y, d.y, w.y);
        ovf |= fold_word<CW>(b.z, d.z, w.z);
        ovf |= fold_word<CW>(b.w, d.w, w.w);
        c4[i] = w;
        d4[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    for (int64_t i = 4 * n4 + tid; i < n; i += stride) {
        uint32_t w;
        ovf |= fold_word<CW>(in[i], delta[i], w);
        counts[i] = w;
        delta[i] = 0u;
    }
    if (ovf) atomicOr(status, ST_COUNT_OVERFLOW);
}

// Density mode 3: copy the counts the sweep's atomics produced,
// B[(s+1) mod 2], into B[s mod 2], so both hold them for the next sweep (16-byte
// accesses; the buffers are 256-byte aligned and W is a multiple of 4).
// Packed 16-bit counts: every change of a sweep is a device atomic add of
// +-1 or +-2^16 on the word, and a true count never goes below zero during
// the sweep (a bead leaves only a cell it was counted in at the start), so
// the word is exact unless a count passed 65535: then its carry moves into
// the other half or out of the word, which lowers the sum of all halves, and
// the error stays in the counts.  So each block adds the sum of the halves
// it copied to its running entry of a.part (the same block index copies the
// same words every sweep), and k_mirror_check, once after the last sweep of
// a batch, compares the total with (sweeps) x (beads).  (Plain stores and a
// second kernel instead of a last-block reduction: a device-scope fence per
// block would write back the L2 each time.)
template <int CW>
__global__ __launch_bounds__(256) void k_mirror(MirrorArgs a)
{
    const uint64_t s = *a.sweep_ctr + a.rel;
    const int64_t W = a.count_words;
    const uint4 *src = reinterpret_cast<const uint4 *>(a.base + ((s + 1) & 1) * W);
    uint4 *dst = reinterpret_cast<uint4 *>(a.base + (s & 1) * W);
    const int64_t n4 = W >> 2;
    // four 16-byte loads in flight per thread before the stores
    constexpr int U = kMirrorUnroll;
    const int64_t step = (int64_t)gridDim.x * (256 * U);
    uint64_t sum = 0;
    for (int64_t b = (int64_t)blockIdx.x * (256 * U) + threadIdx.x; b < n4; b += step) {
        uint4 w[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (b + 256 * k < n4) w[k] = src[b + 256 * k];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (b + 256 * k < n4) {
                dst[b + 256 * k] = w[k];
                if constexpr (CW == COUNT_U16)
                    sum += (uint64_t)((w[k].x & 0xFFFFu) + (w[k].x >> 16) + (w[k].y & 0xFFFFu) + (w[k].y >> 16)) +
                           (uint64_t)((w[k].z & 0xFFFFu) + (w[k].z >> 16) + (w[k].w & 0xFFFFu) + (w[k].w >> 16));
            }
    }
    if constexpr (CW == COUNT_U16) {
        __shared__ unsigned long long part[4];
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
        __syncthreads();
        if (threadIdx.x == 0) a.part[blockIdx.x] += part[0] + part[1] + part[2] + part[3];
    }
}

// Running half sums of the copy blocks against (sweeps) x (beads); clears
// them for the next batch (one block; each thread clears what it read).
__global__ __launch_bounds__(1024) void k_mirror_check(unsigned long long *part, int n_part,
                                                       unsigned long long expected, uint32_t *status)
{
    __shared__ unsigned long long red[16];
    unsigned long long sum = 0;
    for (int i = threadIdx.x; i < n_part; i += blockDim.x) {
        sum += part[i];
        part[i] = 0ull;
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
        if (t != expected) atomicOr(status, ST_COUNT_OVERFLOW);
    }
}

template <int R, int CW>
__global__ __launch_bounds__(256) void k_density(DensityArgs a)
{
    using Bead = typename std::conditional<R == REPR_F32, BeadF32, BeadCell>::type;
    const int wave = __builtin_amdgcn_readfirstlane(
        a.tile_begin + (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    if (wave >= a.tile_end) return;
    const Tile T = a.tiles[wave];
    const DevSys &S = a.systems[T.sys];
    const SysView v = make_view(S);
    const int N = S.N, P = S.P;
    const int lane = (int)(threadIdx.x & 63);
    const int g = (int)(((float)lane + 0.5f) * S.inv_P);
    const int p = lane - g * P;
    const int nin = min(S.G, S.n_chains - (int)T.chain0);
    const bool active = g < nin;
    if (!active) return;
    const int chain = (int)T.chain0 + g;
    const int i0 = 2 * p, i1 = 2 * p + 1;
    const int64_t slot = S.slot_off + (int64_t)chain * (2 * P) + i0;
    const PosArrays A{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2};
    Bead b0, b1;
    load_pair(A, slot, b0, b1);
    bool bad = false, ovf = false;
    const int c0 = cell_of(b0, v, bad);
    const int cls = chain_cls(S, a.chain_class, a.chain_id[S.chain_off + chain]);
    ovf |= scatter_count<CW>(a.counts, S.cell_off + c0, pattern_type(S, cls, i0));
    if (i1 < N) {
        const int c1 = cell_of(b1, v, bad);
        ovf |= scatter_count<CW>(a.counts, S.cell_off + c1, pattern_type(S, cls, i1));
    }
    if (ovf) atomicOr(a.status, ST_COUNT_OVERFLOW);
    if (bad) atomicOr(a.status, ST_CELL_OVERFLOW);
}

// Fields of one system as float [2][M] (A then B), from its counts or its
// frozen array.
template <int CW>
__global__ __launch_bounds__(256) void k_fields(FieldArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_cells) return;
    const DevSys &S = a.systems[a.sys];
    float wa, wb;
    if (S.frozen) {
        const float2 w = a.omega[S.cell_off + c];
        wa = w.x;
        wb = w.y;
    } else {
        const FieldCoef fc{S.cAA, S.cAB, S.cBA, S.cBB, S.c0};
        const uint2 n = load_counts<CW>(a.counts, S.cell_off + c);
        wa = omega_of(fc, n, 0);
        wb = omega_of(fc, n, 1);
        if (S.umb) {
            const float2 t = a.tgt[S.cell_off + c];
            wa -= S.umb_coef * t.x;
            wb -= S.umb_coef * t.y;
        }
    }
    a.out[c] = wa;
    a.out[a.n_cells + c] = wb;
}

// Counts of one system as uint32 [2][M].
template <int CW>
__global__ __launch_bounds__(256) void k_unpack_counts(const uint32_t *counts, int64_t cell_off, int64_t n_cells,
                                                       uint32_t *out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const uint2 n = load_counts<CW>(counts, cell_off + c);
    out[c] = n.x;
    out[n_cells + c] = n.y;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_advance(uint64_t *ctr, uint32_t n) { *ctr += n; }

// ---------------------------------------------------------------------------
// Spatial chain reorder: chains are sorted by the cell of their first bead
// (a counting sort over the context-wide cell index, which keeps every system
// inside its own chain range), so that the waves of one XCD work on a compact
// slab whose counts stay in that XCD's L2.  Logical chain ids move with the
// chains, so the sweep's results do not change.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void k_reorder_keys(ReorderArgs a)
{
    using Bead = typename std::conditional<R == REPR_F32, BeadF32, BeadCell>::type;
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    if (wave >= a.n_tiles) return;
    const Tile T = a.tiles[wave];
    const DevSys &S = a.systems[T.sys];
    const SysView v = make_view(S);
    const int P = S.P;
    const int lane = (int)(threadIdx.x & 63);
    const int g = (int)(((float)lane + 0.5f) * S.inv_P);
    const int p = lane - g * P;
    const int nin = min(S.G, S.n_chains - (int)T.chain0);
    if (g >= nin || p != 0) return;
    const int chain = (int)T.chain0 + g;
    const int64_t slot = S.slot_off + (int64_t)chain * (2 * P);
    Bead b0, b1;
    load_pair(PosArrays{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2}, slot, b0, b1);
    bool bad = false;
    const uint32_t key = (uint32_t)(S.cell_off + cell_of(b0, v, bad));
    a.keys[S.chain_off + chain] = key;
    atomicAdd(a.hist + key, 1u);
}

// Exclusive scan of hist[0, n) in place: block sums, a scan of the block
// sums by one block, then the block-local scans plus offsets.
constexpr int kScanBlock = 1024, kScanPer = 4, kScanTile = kScanBlock * kScanPer;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const uint32_t x = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    total = sh[kScanBlock - 1];
    const uint32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_partials(const uint32_t *hist, int64_t n, uint32_t *bsum)
{
    __shared__ uint32_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t v = 0;
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) v += hist[base + k];
    uint32_t total;
    (void)block_exclusive_scan(v, sh, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_bsum(uint32_t *bsum, int nb)
{
    __shared__ uint32_t sh[kScanBlock];
    uint32_t carry = 0;
    for (int start = 0; start < nb; start += kScanBlock) {
        const int i = start + (int)threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, sh, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(uint32_t *hist, int64_t n, const uint32_t *bsum)
{
    __shared__ uint32_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t vals[kScanPer];
    uint32_t v = 0;
    for (int k = 0; k < kScanPer; ++k) {
        vals[k] = base + k < n ? hist[base + k] : 0u;
        v += vals[k];
    }
    uint32_t total;
    uint32_t run = bsum[blockIdx.x] + block_exclusive_scan(v, sh, total);
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) {
            hist[base + k] = run;
            run += vals[k];
        }
}

// perm[new] = old: each chain takes the next free place of its key.
__global__ __launch_bounds__(256) void k_reorder_scatter(ReorderArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.total_chains) return;
    const uint32_t pos = atomicAdd(a.hist + a.keys[c], 1u);
    if (pos < (uint64_t)a.total_chains) a.perm[pos] = (uint32_t)c;
    else atomicOr(a.status, ST_INTERNAL);
}

// Move chain perm[new] into place `new` (scratch copy), with its logical id.
template <int R>
__global__ __launch_bounds__(256) void k_reorder_permute(ReorderArgs a)
{
    using Bead = typename std::conditional<R == REPR_F32, BeadF32, BeadCell>::type;
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    if (wave >= a.n_tiles) return;
    const Tile T = a.tiles[wave];
    const DevSys &S = a.systems[T.sys];
    const int P = S.P;
    const int lane = (int)(threadIdx.x & 63);
    const int g = (int)(((float)lane + 0.5f) * S.inv_P);
    const int p = lane - g * P;
    const int nin = min(S.G, S.n_chains - (int)T.chain0);
    if (g >= nin) return;
    const int chain = (int)T.chain0 + g;
    const int64_t old = (int64_t)a.perm[S.chain_off + chain] - S.chain_off;
    if (old < 0 || old >= S.n_chains) {           // a chain left its system: never expected
        atomicOr(a.status, ST_INTERNAL);
        return;
    }
    Bead b0, b1;
    load_pair(PosArrays{a.P0, a.P1, a.P2, a.C0, a.C1, a.C2}, S.slot_off + old * (2 * P) + 2 * p, b0, b1);
    store_pair(PosArrays{a.Q0, a.Q1, a.Q2, a.D0, a.D1, a.D2}, S.slot_off + (int64_t)chain * (2 * P) + 2 * p, b0, b1);
    if (p == 0) a.chain_id2[S.chain_off + chain] = a.chain_id[S.chain_off + old];
}

// Logical chain ids in system order (identity within each system).
__global__ __launch_bounds__(256) void k_iota_chains(ReorderArgs a)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    if (wave >= a.n_tiles) return;
    const Tile T = a.tiles[wave];
    const DevSys &S = a.systems[T.sys];
    const int lane = (int)(threadIdx.x & 63);
    const int chain = (int)T.chain0 + lane;
    if (lane < S.G && chain < S.n_chains) a.chain_id[S.chain_off + chain] = (uint32_t)chain;
}

// ---------------------------------------------------------------------------
// Initial configuration: Gaussian random walks on the GPU (Sec. 2.2 moved
// the generation of bead coordinates to the GPU).  One thread per chain,
// FP64 accumulation along the chain, then rounding to the representation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_init(const InitArgs &a, int64_t slot, double x, double y,
                                           double z)
{
    if (a.repr == REPR_F32) {
        a.P0[slot] = (float)x;
        a.P1[slot] = (float)y;
        a.P2[slot] = (float)z;
        return;
    }
    const double r[3] = {x, y, z};
    float *P[3] = {a.P0, a.P1, a.P2};
    int *C[3] = {a.C0, a.C1, a.C2};
    for (int d = 0; d < 3; ++d) {
        const float e = a.edge[d];
        const double cf = floor(r[d] / (double)e);
        int c = (int)cf;
        float o = (float)(r[d] - cf * (double)e);
        renorm(c, o, e);
        C[d][slot] = c;
        P[d][slot] = o;
    }
}

// Initial streams: counter word 3 = system id with the top bit set (never a
// move draw); word 2 names the stream and the attempt j (walls only):
// 4j initial walks, 4j + 1 placement targets, 4j + 2 placement walks.
__device__ __forceinline__ uint4 init_block(uint32_t w0, uint32_t chain, uint32_t stream, uint32_t sys_id,
                                            uint64_t seed)
{
    return philox4x32_10(make_uint4(w0, chain, stream, sys_id | 0x80000000u), (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

__device__ __forceinline__ double top24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

// One Gaussian bond, each component N(0, sigma^2), Box-Muller on words (0,1), (2,3).
__device__ __forceinline__ double3 gauss_bond(uint4 w, double sigma)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double u1 = ((double)(w.x >> 8) + 0.5) * 0x1p-24;
    const double u2 = top24(w.y);
    const double u3 = ((double)(w.z >> 8) + 0.5) * 0x1p-24;
    const double u4 = top24(w.w);
    const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    return make_double3(sigma * r1 * cos(two_pi * u2), sigma * r1 * sin(two_pi * u2), sigma * r2 * cos(two_pi * u4));
}

// Walls: the z range a drawn chain must stay in, with a margin of 1/128 cell
// edge so that the stored representation's z cell is inside whatever the
// rounding (|z| < 2^15 edges).
__device__ __forceinline__ void wall_range(const InitArgs &a, double &lo, double &hi)
{
    const double e = (double)a.edge[2];
    lo = (double)a.wall_lo * e + e / 128.0;
    hi = (double)a.wall_hi * e - e / 128.0;
}

// Bead 0 uniform in the box (in z between the walls when there are walls),
// bonds Gaussian; with walls a chain that leaves the slab is drawn again
// from the next attempt's counters (kMaxAttempts at most, else the status
// bit).  One thread per chain, FP64 along the chain, then rounding to the
// representation (the last attempt's chain is the one stored).
__global__ __launch_bounds__(256) void k_init_walks(InitArgs a)
{
    const int chain = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (chain >= a.n_chains) return;
    const int64_t base = a.slot_off + (int64_t)chain * a.stride;
    double zlo = 0.0, zhi = 0.0;
    if (a.walls) wall_range(a, zlo, zhi);
    bool ok = false;
    for (int j = 0; j < kMaxAttempts && !ok; ++j) {
        ok = true;
        double x = 0, y = 0, z = 0;
        for (int i = 0; i < a.N; ++i) {
            const uint4 w = init_block((uint32_t)i, (uint32_t)chain, 4u * (uint32_t)j, a.sys_id, a.seed);
            if (i == 0) {
                x = a.box[0] * top24(w.x);
                y = a.box[1] * top24(w.y);
                z = a.box[2] * top24(w.z);
                if (a.walls) {
                    const double e = (double)a.edge[2];
                    const double lo = (double)a.wall_lo * e, hi = (double)a.wall_hi * e;
                    z = lo + (hi - lo) * top24(w.z);
                }
            } else {
                const double3 b = gauss_bond(w, a.sigma);
                x += b.x;
                y += b.y;
                z += b.z;
            }
            if (a.walls && !(z >= zlo && z <= zhi)) ok = false;
            store_init(a, base + i, x, y, z);
        }
        if (!a.walls) break;
    }
    if (!ok) atomicOr(a.status, ST_PLACEMENT);
    for (int i = a.N; i < a.stride; ++i) store_init(a, base + i, 0.0, 0.0, 0.0);   // padding slot
}

// ---------------------------------------------------------------------------
// Placement from target concentration fields (Sec. 3.2, "Coupling"): each
// molecule's centre ends up at most Re/2 (half the ideal end-to-end
// distance) from a target position drawn from the supplied fields.
//   1. Class k (pattern a or b, A fraction f_k) weighs cell c by the integer
//      w_k(c) = floor(2^20 (f_k tA(c) + (1 - f_k) tB(c)) + 1/2) (FP64, exact
//      as the same operations on any IEEE machine); W_k is its exact
//      inclusive prefix sum (uint64).
//   2. A chain of class k takes t = floor(v T_k / 2^64) for the 64-bit word
//      v of its block (0, chain, 4j + 1) and the first cell with W_k > t.
//   3. Target point uniform in that cell; centre of mass uniform in the ball
//      of radius Re/2 around it; conformation a Gaussian walk (blocks
//      (i, chain, 4j + 2)) shifted to that centre.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_place_weights(PlaceArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_cells) return;
    const int N = a.ia.N;
    const float2 t = a.tgt[a.cell_off + c];
    for (int k = 0; k < 2; ++k) {
        const double fa = (double)a.na[k] / (double)N, fb = (double)(N - a.na[k]) / (double)N;
        const double v = fa * (double)t.x + fb * (double)t.y;
        a.W[k * a.n_cells + c] = (unsigned long long)floor(1048576.0 * v + 0.5);
    }
}

// Inclusive scan of 64-bit words in place (block sums, a one-block scan of
// the sums, then block-local scans plus offsets), as for the reorder.
constexpr int kScan64Block = 256, kScan64Per = 8, kScan64Tile = kScan64Block * kScan64Per;

__device__ __forceinline__ unsigned long long block_scan64(unsigned long long v, unsigned long long *sh,
                                                           unsigned long long &total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScan64Block; off <<= 1) {
        const unsigned long long x = t >= off ? sh[t - off] : 0ull;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    total = sh[kScan64Block - 1];
    const unsigned long long incl = sh[t];
    __syncthreads();
    return incl - v;          // exclusive
}

__global__ __launch_bounds__(kScan64Block) void k_scan64_partials(const unsigned long long *x, int64_t n,
                                                                  unsigned long long *bsum)
{
    __shared__ unsigned long long sh[kScan64Block];
    const int64_t base = (int64_t)blockIdx.x * kScan64Tile + (int64_t)threadIdx.x * kScan64Per;
    unsigned long long v = 0;
    for (int k = 0; k < kScan64Per; ++k)
        if (base + k < n) v += x[base + k];
    unsigned long long total;
    (void)block_scan64(v, sh, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScan64Block) void k_scan64_bsum(unsigned long long *bsum, int nb)
{
    __shared__ unsigned long long sh[kScan64Block];
    unsigned long long carry = 0;
    for (int start = 0; start < nb; start += kScan64Block) {
        const int i = start + (int)threadIdx.x;
        const unsigned long long v = i < nb ? bsum[i] : 0ull;
        unsigned long long total;
        const unsigned long long ex = block_scan64(v, sh, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kScan64Block) void k_scan64_apply(unsigned long long *x, int64_t n,
                                                               const unsigned long long *bsum)
{
    __shared__ unsigned long long sh[kScan64Block];
    const int64_t base = (int64_t)blockIdx.x * kScan64Tile + (int64_t)threadIdx.x * kScan64Per;
    unsigned long long vals[kScan64Per];
    unsigned long long v = 0;
    for (int k = 0; k < kScan64Per; ++k) {
        vals[k] = base + k < n ? x[base + k] : 0ull;
        v += vals[k];
    }
    unsigned long long total;
    unsigned long long run = bsum[blockIdx.x] + block_scan64(v, sh, total);
    for (int k = 0; k < kScan64Per; ++k)
        if (base + k < n) {
            run += vals[k];
            x[base + k] = run;      // inclusive
        }
}

// One thread per chain slot of the system: the chain with that slot's
// logical id is placed into it.
__global__ __launch_bounds__(256) void k_place_chains(PlaceArgs a)
{
    const int slot_chain = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const InitArgs &ia = a.ia;
    if (slot_chain >= ia.n_chains) return;
    const uint32_t chain = a.chain_id[a.chain_off + slot_chain];
    const int k = (int)a.chain_class[a.chain_off + chain];
    const unsigned long long *Wk = a.W + k * a.n_cells;
    const unsigned long long T = Wk[a.n_cells - 1];
    const int64_t base = ia.slot_off + (int64_t)slot_chain * ia.stride;
    const int N = ia.N;
    const double two_pi = 6.283185307179586476925286766559;
    double zlo = 0.0, zhi = 0.0;
    if (ia.walls) wall_range(ia, zlo, zhi);
    bool ok = false;
    for (int j = 0; j < kMaxAttempts && !ok && T > 0; ++j) {
        const uint4 w = init_block(0u, chain, 4u * (uint32_t)j + 1u, ia.sys_id, ia.seed);
        const uint4 q = init_block(1u, chain, 4u * (uint32_t)j + 1u, ia.sys_id, ia.seed);
        const unsigned long long v = ((unsigned long long)w.x << 32) | w.y;
        const unsigned long long t = __umul64hi(v, T);
        int64_t lo = 0, hi = a.n_cells - 1;     // first cell with Wk > t
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (Wk[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        const int64_t nyz = (int64_t)a.grid[1] * a.grid[2];
        const int64_t ix = lo / nyz, iy = (lo / a.grid[2]) % a.grid[1], iz = lo % a.grid[2];
        const double tx = ((double)ix + top24(w.z)) * a.edge64[0];
        const double ty = ((double)iy + top24(w.w)) * a.edge64[1];
        const double tz = ((double)iz + top24(q.x)) * a.edge64[2];
        const double rad = 0.5 * a.Re * cbrt(top24(q.y));
        const double ct = 2.0 * top24(q.z) - 1.0;
        const double stt = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double ph = two_pi * top24(q.w);
        const double cx = tx + rad * stt * cos(ph), cy = ty + rad * stt * sin(ph), cz = tz + rad * ct;
        // centre of mass of the walk (bead 0 at the origin), then the beads
        double sx = 0, sy = 0, sz = 0, x = 0, y = 0, z = 0;
        for (int i = 1; i < N; ++i) {
            const double3 b = gauss_bond(init_block((uint32_t)i, chain, 4u * (uint32_t)j + 2u, ia.sys_id, ia.seed),
                                         ia.sigma);
            x += b.x;
            y += b.y;
            z += b.z;
            sx += x;
            sy += y;
            sz += z;
        }
        const double mx = sx / (double)N, my = sy / (double)N, mz = sz / (double)N;
        ok = true;
        x = y = z = 0;
        for (int i = 0; i < N; ++i) {
            if (i > 0) {
                const double3 b = gauss_bond(
                    init_block((uint32_t)i, chain, 4u * (uint32_t)j + 2u, ia.sys_id, ia.seed), ia.sigma);
                x += b.x;
                y += b.y;
                z += b.z;
            }
            const double pz = cz + (z - mz);
            if (ia.walls && !(pz >= zlo && pz <= zhi)) ok = false;
            store_init(ia, base + i, cx + (x - mx), cy + (y - my), pz);
        }
        if (!ia.walls) break;
    }
    if (!ok) atomicOr(ia.status, ST_PLACEMENT);
}

// ---------------------------------------------------------------------------
// Observables: FP64 per chain, compensated (Neumaier) block sums.  These are
// the only FP64 operations on the GPU.
// ---------------------------------------------------------------------------
struct NSum {
    double s, c;
};
__device__ __forceinline__ void nadd(NSum &a, double v)
{
    const double t = a.s + v;
    a.c += fabs(a.s) >= fabs(v) ? (a.s - t) + v : (v - t) + a.s;
    a.s = t;
}
__device__ __forceinline__ void nmerge(NSum &a, const NSum &b)
{
    nadd(a, b.s);
    a.c += b.c;
}

constexpr int kObsQ = 6;   // Re2, Re2^2, Rg2, Rg2^2, Ebond, Enb

__device__ __forceinline__ double pos_f64(const ObsArgs &a, int d, int64_t slot)
{
    const float *P = d == 0 ? a.P0 : d == 1 ? a.P1 : a.P2;
    if (a.repr == REPR_F32) return (double)P[slot];
    const int *C = d == 0 ? a.C0 : d == 1 ? a.C1 : a.C2;
    return (double)C[slot] * (double)a.edge[d] + (double)P[slot];
}

// Block-level deterministic tree reduction of kObsQ Neumaier sums.
__device__ void block_reduce_store(NSum (&q)[kObsQ], double *partials, int block)
{
    __shared__ double sh_s[kObsQ][256];
    __shared__ double sh_c[kObsQ][256];
    const int t = threadIdx.x;
    for (int k = 0; k < kObsQ; ++k) {
        sh_s[k][t] = q[k].s;
        sh_c[k][t] = q[k].c;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            for (int k = 0; k < kObsQ; ++k) {
                NSum x{sh_s[k][t], sh_c[k][t]};
                nmerge(x, NSum{sh_s[k][t + w], sh_c[k][t + w]});
                sh_s[k][t] = x.s;
                sh_c[k][t] = x.c;
            }
        }
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < kObsQ; ++k) {
            partials[(int64_t)block * 2 * kObsQ + 2 * k] = sh_s[k][0];
            partials[(int64_t)block * 2 * kObsQ + 2 * k + 1] = sh_c[k][0];
        }
}

__global__ __launch_bounds__(256) void k_obs_chains(ObsArgs a)
{
    NSum q[kObsQ];
    for (int k = 0; k < kObsQ; ++k) q[k] = NSum{0.0, 0.0};
    const int chain = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (chain < a.n_chains) {
        const int64_t base = a.slot_off + (int64_t)chain * a.stride;
        const int N = a.N;
        double cm[3] = {0, 0, 0}, e2e = 0, bond = 0;
        for (int d = 0; d < 3; ++d) {
            const double r0 = pos_f64(a, d, base), rl = pos_f64(a, d, base + N - 1);
            e2e += (rl - r0) * (rl - r0);
            double prev = r0;
            cm[d] = r0;
            for (int i = 1; i < N; ++i) {
                const double r = pos_f64(a, d, base + i);
                bond += (r - prev) * (r - prev);
                cm[d] += r;
                prev = r;
            }
            cm[d] /= (double)N;
        }
        double g = 0;
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < N; ++i) {
                const double r = pos_f64(a, d, base + i) - cm[d];
                g += r * r;
            }
        g /= (double)N;
        bond *= a.k_half;
        nadd(q[0], e2e);
        nadd(q[1], e2e * e2e);
        nadd(q[2], g);
        nadd(q[3], g * g);
        nadd(q[4], bond);
    }
    block_reduce_store(q, a.partials, blockIdx.x);
}

// f(phiA, phiB) per cell; sum over cells times (B / M) / N gives H_nb / kT.
template <int CW>
__global__ __launch_bounds__(256) void k_obs_cells(ObsArgs a)
{
    NSum q[kObsQ];
    for (int k = 0; k < kObsQ; ++k) q[k] = NSum{0.0, 0.0};
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < a.n_cells) {
        const uint2 n = load_counts<CW>(a.counts, a.cell_off + c);
        const double pa = (double)n.x * a.phi_per_count, pb = (double)n.y * a.phi_per_count;
        const double inc = pa + pb - 1.0;
        double f;
        if (a.ham_form == 1)
            f = a.chiN * pa * pb + 0.5 * a.kappaN * inc * inc;
        else
            f = 0.5 * a.kappaN * inc * inc - 0.25 * a.chiN * (pa - pb) * (pa - pb);
        if (a.umb_lambda > 0.0) {
            // umbrella toward the target fields: (lambda/2) sum_t (phi_t - target_t)^2
            const float2 t = a.tgt[a.cell_off + c];
            const double da = pa - (double)t.x, db = pb - (double)t.y;
            f += 0.5 * a.umb_lambda * (da * da + db * db);
        }
        nadd(q[5], f);
    }
    block_reduce_store(q, a.partials, a.block_base + blockIdx.x);
}

__global__ __launch_bounds__(256) void k_obs_finalize(const double *partials, int n_blocks, double *out)
{
    __shared__ double sh_s[256], sh_c[256];
    const int t = threadIdx.x;
    for (int k = 0; k < kObsQ; ++k) {
        NSum acc{0.0, 0.0};
        for (int b = t; b < n_blocks; b += 256)
            nmerge(acc, NSum{partials[(int64_t)b * 2 * kObsQ + 2 * k], partials[(int64_t)b * 2 * kObsQ + 2 * k + 1]});
        sh_s[t] = acc.s;
        sh_c[t] = acc.c;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) {
                NSum x{sh_s[t], sh_c[t]};
                nmerge(x, NSum{sh_s[t + w], sh_c[t + w]});
                sh_s[t] = x.s;
                sh_c[t] = x.c;
            }
            __syncthreads();
        }
        if (t == 0) out[k] = sh_s[0] + sh_c[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int R, int CW, int DM, bool SMC>
static void launch_sweep_d(const SweepArgs &a, int blocks, hipStream_t st)
{
    const dim3 g(blocks), b(64 * a.waves_per_block);
    const size_t lds = sizeof(uint32_t) * 2 * (DM == 2 ? kAggSlotsFaces : kAggSlotsCells) * a.waves_per_block;
    // contexts without walls, zones, umbrella or caller-set classes launch
    // kernels built without that code (fewer registers)
    // block tiles: one tile per block (never with conversion zones, whose
    // chain sums stay within a wave)
    // only the plain and stream kernels count acceptances per tile
    SweepArgs o = a;
    if (!counts_per_tile(a)) o.acc_tile = nullptr;
    if (o.cpl) {
        if (o.max_blocks > 0) hipLaunchKernelGGL((k_sweep<R, CW, true, DM, SMC, true, false>), g, b, lds, st, o);
        else if (o.packed == 1) hipLaunchKernelGGL((k_sweep<R, CW, false, DM, SMC, true, true>), g, b, lds, st, o);
        else hipLaunchKernelGGL((k_sweep<R, CW, false, DM, SMC, true, false>), g, b, lds, st, o);
    } else {
        if (o.max_blocks > 0) hipLaunchKernelGGL((k_sweep<R, CW, true, DM, SMC, false, false>), g, b, lds, st, o);
        else if (o.packed == 1) hipLaunchKernelGGL((k_sweep<R, CW, false, DM, SMC, false, true>), g, b, lds, st, o);
        else if (!SMC && o.packed == 2) hipLaunchKernelGGL((k_sweep_stream<R, CW, DM>), g, b, lds, st, o);
        else if (!SMC) hipLaunchKernelGGL((k_sweep_plain<R, CW, DM>), g, b, lds, st, o);
        else hipLaunchKernelGGL((k_sweep<R, CW, false, DM, SMC, false, false>), g, b, lds, st, o);
    }
}

template <int R, int CW, bool SMC>
static hipError_t launch_sweep_s(const SweepArgs &a, int blocks, hipStream_t st)
{
    if (a.density_mode == 1) launch_sweep_d<R, CW, 1, SMC>(a, blocks, st);
    else if (a.density_mode == 2) launch_sweep_d<R, CW, 2, SMC>(a, blocks, st);
    else if (a.density_mode == 3) launch_sweep_d<R, CW, 3, SMC>(a, blocks, st);
    else launch_sweep_d<R, CW, 0, SMC>(a, blocks, st);
    return hipGetLastError();
}

// Contexts with smart moves use the kernels that carry both move kinds (the
// kind is chosen per wave tile); the others keep the smaller uniform-only ones.
template <int R, int CW>
static hipError_t launch_sweep_t(const SweepArgs &a, int blocks, hipStream_t st)
{
    return a.smc ? launch_sweep_s<R, CW, true>(a, blocks, st) : launch_sweep_s<R, CW, false>(a, blocks, st);
}

hipError_t launch_sweep(int repr, int cw, const SweepArgs &a, hipStream_t st)
{
    int blocks = (a.n_tiles + a.waves_per_block - 1) / a.waves_per_block;
    if (a.max_blocks > 0 && blocks > a.max_blocks) blocks = a.max_blocks;
    if (a.packed == 1 && a.max_blocks == 0) blocks = a.n_ptiles;
    // stream tiles only for uniform moves without coupling (the launch below
    // takes wave tiles otherwise)
    if (a.packed == 2 && a.max_blocks == 0 && !a.cpl && !a.smc)
        blocks = (a.n_ptiles + a.waves_per_block - 1) / a.waves_per_block;
    if (blocks <= 0) return hipErrorInvalidConfiguration;   // the tile tables are empty
    if (repr == REPR_F32)
        return cw == COUNT_U16 ? launch_sweep_t<REPR_F32, COUNT_U16>(a, blocks, st)
                               : launch_sweep_t<REPR_F32, COUNT_U32>(a, blocks, st);
    return cw == COUNT_U16 ? launch_sweep_t<REPR_CELL, COUNT_U16>(a, blocks, st)
                           : launch_sweep_t<REPR_CELL, COUNT_U32>(a, blocks, st);
}

hipError_t launch_density(int repr, int cw, const DensityArgs &a, hipStream_t st)
{
    const int n = a.tile_end - a.tile_begin;
    if (n <= 0) return hipSuccess;
    const int blocks = (n + 3) / 4;
    if (repr == REPR_F32) {
        if (cw == COUNT_U16) hipLaunchKernelGGL((k_density<REPR_F32, COUNT_U16>), dim3(blocks), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_density<REPR_F32, COUNT_U32>), dim3(blocks), dim3(256), 0, st, a);
    } else {
        if (cw == COUNT_U16) hipLaunchKernelGGL((k_density<REPR_CELL, COUNT_U16>), dim3(blocks), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_density<REPR_CELL, COUNT_U32>), dim3(blocks), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_fields(int cw, const FieldArgs &a, hipStream_t st)
{
    const int blocks = (int)((a.n_cells + 255) / 256);
    if (blocks == 0) return hipSuccess;
    if (cw == COUNT_U16) hipLaunchKernelGGL((k_fields<COUNT_U16>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_fields<COUNT_U32>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_unpack_counts(int cw, const uint32_t *counts, int64_t cell_off, int64_t n_cells,
                                uint32_t *out, hipStream_t st)
{
    const int blocks = (int)((n_cells + 255) / 256);
    if (blocks == 0) return hipSuccess;
    if (cw == COUNT_U16) hipLaunchKernelGGL((k_unpack_counts<COUNT_U16>), dim3(blocks), dim3(256), 0, st, counts, cell_off, n_cells, out);
    else hipLaunchKernelGGL((k_unpack_counts<COUNT_U32>), dim3(blocks), dim3(256), 0, st, counts, cell_off, n_cells, out);
    return hipGetLastError();
}

hipError_t launch_fold_faces(int cw, const FoldFacesArgs &a, int n_chunks, hipStream_t st)
{
    if (n_chunks <= 0) return hipSuccess;
    if (cw == COUNT_U16) hipLaunchKernelGGL((k_fold_faces<COUNT_U16>), dim3(n_chunks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_fold_faces<COUNT_U32>), dim3(n_chunks), dim3(256), 0, st, a);
    return hipGetLastError();
}

static int64_t mirror_blocks(int64_t count_words)
{
    const int64_t blocks = (count_words / 4 + 256 * kMirrorUnroll - 1) / (256 * kMirrorUnroll);
    return blocks > kMirrorBlocks ? kMirrorBlocks : blocks;
}

hipError_t launch_mirror(int cw, const MirrorArgs &a, hipStream_t st)
{
    if (a.count_words <= 0) return hipSuccess;
    const int64_t blocks = mirror_blocks(a.count_words);
    if (cw == COUNT_U16)
        hipLaunchKernelGGL((k_mirror<COUNT_U16>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_mirror<COUNT_U32>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mirror_check(int cw, const MirrorArgs &a, uint32_t n_sweeps, hipStream_t st)
{
    if (a.count_words <= 0 || cw != COUNT_U16 || n_sweeps == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mirror_check, dim3(1), dim3(1024), 0, st, a.part, (int)mirror_blocks(a.count_words),
                       a.beads * (unsigned long long)n_sweeps, a.status);
    return hipGetLastError();
}

hipError_t launch_stream_halo(int repr, const HaloArgs &a, hipStream_t st)
{
    if (a.n_ptiles <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((2 * (int64_t)a.n_ptiles + 255) / 256);
    if (repr == REPR_F32)
        hipLaunchKernelGGL((k_stream_halo<BeadF32>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_stream_halo<BeadCell>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_acc_fold(const Tile *tiles, int n_tiles, int stream,
                                                  unsigned long long *acc_tile, unsigned long long *accept)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= n_tiles) return;
    const unsigned long long v = acc_tile[t];
    if (v == 0ull) return;
    const uint32_t sys = stream ? stile_sys(tiles[t]) : tiles[t].sys;
    atomicAdd(accept + ((int64_t)sys * kAcceptSlots + (t % kAcceptSlots)) * kAcceptStride, v);
    acc_tile[t] = 0ull;
}

hipError_t launch_acc_fold(const Tile *tiles, int n_tiles, bool stream, unsigned long long *acc_tile,
                           unsigned long long *accept, hipStream_t st)
{
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_acc_fold, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, st, tiles, n_tiles,
                       stream ? 1 : 0, acc_tile, accept);
    return hipGetLastError();
}

hipError_t launch_fold(int cw, const uint32_t *counts_in, uint32_t *delta, uint32_t *counts_out, int64_t n,
                       uint32_t *status, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = ((n + 3) / 4 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (cw == COUNT_U16)
        hipLaunchKernelGGL((k_fold<COUNT_U16>), dim3((unsigned)blocks), dim3(256), 0, st, counts_in, delta, counts_out, n, status);
    else
        hipLaunchKernelGGL((k_fold<COUNT_U32>), dim3((unsigned)blocks), dim3(256), 0, st, counts_in, delta, counts_out, n, status);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_advance(uint64_t *ctr, uint32_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, st, ctr, n);
    return hipGetLastError();
}

hipError_t launch_iota_chains(const ReorderArgs &a, hipStream_t st)
{
    const int blocks = (a.n_tiles + 3) / 4;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota_chains, dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reorder(int repr, const ReorderArgs &a, hipStream_t st)
{
    const int tblocks = (a.n_tiles + 3) / 4;
    if (tblocks == 0) return hipSuccess;
    hipError_t e = launch_fill_u32(a.hist, a.total_cells, 0u, st);
    if (e != hipSuccess) return e;
    if (repr == REPR_F32) hipLaunchKernelGGL((k_reorder_keys<REPR_F32>), dim3(tblocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_reorder_keys<REPR_CELL>), dim3(tblocks), dim3(256), 0, st, a);
    const int nb = (int)((a.total_cells + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kScanBlock), 0, st, a.hist, a.total_cells, a.bsum);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(kScanBlock), 0, st, a.bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanBlock), 0, st, a.hist, a.total_cells, a.bsum);
    const int cblocks = (int)((a.total_chains + 255) / 256);
    hipLaunchKernelGGL(k_reorder_scatter, dim3(cblocks), dim3(256), 0, st, a);
    if (repr == REPR_F32) hipLaunchKernelGGL((k_reorder_permute<REPR_F32>), dim3(tblocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_reorder_permute<REPR_CELL>), dim3(tblocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

int64_t reorder_bsum_words(int64_t total_cells) { return (total_cells + kScanTile - 1) / kScanTile; }

hipError_t launch_init(const InitArgs &a, hipStream_t st)
{
    const int blocks = (a.n_chains + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_walks, dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

int64_t place_bsum_words(int64_t n_cells) { return (n_cells + kScan64Tile - 1) / kScan64Tile; }

hipError_t launch_place(const PlaceArgs &a, unsigned long long *bsum, hipStream_t st)
{
    if (a.n_cells <= 0 || a.ia.n_chains <= 0) return hipSuccess;
    const int cb = (int)((a.n_cells + 255) / 256);
    hipLaunchKernelGGL(k_place_weights, dim3(cb), dim3(256), 0, st, a);
    const int nb = (int)place_bsum_words(a.n_cells);
    for (int k = 0; k < 2; ++k) {
        unsigned long long *x = a.W + k * a.n_cells;
        hipLaunchKernelGGL(k_scan64_partials, dim3(nb), dim3(kScan64Block), 0, st, x, a.n_cells, bsum);
        hipLaunchKernelGGL(k_scan64_bsum, dim3(1), dim3(kScan64Block), 0, st, bsum, nb);
        hipLaunchKernelGGL(k_scan64_apply, dim3(nb), dim3(kScan64Block), 0, st, x, a.n_cells, bsum);
    }
    hipLaunchKernelGGL(k_place_chains, dim3((a.ia.n_chains + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_observables(int cw, const ObsArgs &a, double *out, hipStream_t st)
{
    const int bc = (a.n_chains + 255) / 256;
    const int bm = (int)((a.n_cells + 255) / 256);
    ObsArgs b = a;
    hipLaunchKernelGGL(k_obs_chains, dim3(bc), dim3(256), 0, st, b);
    b.block_base = bc;
    if (cw == COUNT_U16) hipLaunchKernelGGL((k_obs_cells<COUNT_U16>), dim3(bm), dim3(256), 0, st, b);
    else hipLaunchKernelGGL((k_obs_cells<COUNT_U32>), dim3(bm), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_obs_finalize, dim3(1), dim3(256), 0, st, a.partials, bc + bm, out);
    return hipGetLastError();
}

}  // namespace soma
