// Product path guiding (Sec. 3.6): two-level sampling of a radiance field
// times an 8 x 8 BSDF table, one wave per query.
//
// Upper level: the N x N field summed to 8 x 8 cells (cell C = 8 V + U holds
// the s x s fine bins u in [U s, U s + s), v in [V s, V s + s), s = N / 8),
// each cell value F_C multiplied by the table entry f_C; lane C of the wave
// owns cell C. Lower level: the fine bin inside the chosen cell, sampled from
// the field restricted to that cell. The pdf of fine bin b in cell C is
// P_C / sum(P) * L_b / F_C * N^2 / (4 pi).
//
// Selection rule (rows, then columns, at both levels): the first entry whose
// inclusive CDF exceeds the target; if none does (a target rounded up to the
// total), the last entry with positive mass. A product whose total is zero or
// not finite (a zero or non-finite normal) is replaced by f = 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "march_core.h"

namespace wfpg {
namespace prod {

constexpr int kCells = 8;   // the upper level is kCells x kCells

// Inclusive scan over groups of W consecutive lanes (W a power of two <= 64).
template <int W>
__device__ __forceinline__ float group_scan(float v, int lane)
{
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
        const float t = __shfl_up(v, d, W);
        if ((lane & (W - 1)) >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ int lowest(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
__device__ __forceinline__ int highest(uint64_t m) { return 63 - __builtin_clzll(m); }

// Table entry of cell `lane` for query i: row i of `bsdf` (n x 64, row-major
// [V][U]) when given, else the Lambertian cosine factor max(0, n . d_C) of the
// normal (SoA planes of stride ps) with the cell-centre direction d_C (the
// N = 8 bin-centre table), as (n_x d_x + n_y d_y) + n_z d_z in FP32.
__device__ __forceinline__ float table_entry(const float *nrm, const float *bsdf, int64_t i, int64_t ps,
                                             const float *tab8, int lane)
{
    float x;
    if (bsdf) {
        x = bsdf[i * 64 + lane];
    } else {
        x = core::dot3(nrm[i], nrm[ps + i], nrm[2 * ps + i], tab8[3 * lane], tab8[3 * lane + 1],
                       tab8[3 * lane + 2]);
    }
    return x > 0.f ? x : 0.f;   // negative, zero and NaN entries count as 0
}

// The upper level of one query (wave-wide; lane = cell).
struct Upper {
    float F;       // this lane's cell sum
    float P;       // this lane's product
    float R;       // inclusive CDF of this lane's row up to this cell
    float rs;      // lanes 0..7: row sums of the product
    float M;       // lanes 0..7: inclusive marginal CDF
    float total;   // sum of the product (wave-uniform)
};

__device__ __forceinline__ void upper_level(float F, float f, int lane, Upper &q)
{
    q.F = F;
    for (int pass = 0; pass < 2; ++pass) {   // pass 1 only when the product is degenerate
        q.P = pass ? F : F * f;
        q.R = group_scan<kCells>(q.P, lane);
        const float t = __shfl(q.R, (lane & 7) * kCells + kCells - 1);
        q.rs = lane < kCells ? t : 0.f;
        q.M = group_scan<kCells>(q.rs, lane);
        q.total = __shfl(q.M, kCells - 1);
        if (q.total > 0.f && q.total < INFINITY) break;
    }
}

// Cell from the product with uniforms w1 (row) and w2 (column); returns C.
__device__ __forceinline__ int pick_cell(const Upper &q, float w1, float w2, int lane)
{
    const float tv = w1 * q.total;
    const uint64_t bv = __ballot(lane < kCells && tv < q.M);
    int V;
    if (bv) {
        V = lowest(bv);
    } else {
        const uint64_t bp = __ballot(lane < kCells && q.rs > 0.f);
        V = bp ? highest(bp) : kCells - 1;
    }
    const float rowsum = __shfl(q.rs, V);
    const float tu = w2 * rowsum;
    const bool in_row = (lane >> 3) == V;
    const uint64_t bu = __ballot(in_row && tu < q.R);
    int U;
    if (bu) {
        U = lowest(bu) - V * kCells;
    } else {
        const uint64_t bp = __ballot(in_row && q.P > 0.f);
        U = bp ? highest(bp) - V * kCells : kCells - 1;
    }
    return V * kCells + U;
}

// Fine bin inside cell (U, V): `ld(dv, du)` loads the field value of fine bin
// (V s + dv, U s + du). Uniforms u1 (row) and u2 (column). Returns the value
// of the chosen bin; dv, du its offsets in the cell (wave-uniform).
template <int S, typename Load>
__device__ __forceinline__ float pick_fine(Load ld, float u1, float u2, int lane, int &dv, int &du)
{
    constexpr int SS = S * S;
    constexpr int R = SS > 64 ? SS / 64 : 1;   // registers per lane
    constexpr int G = 64 / S;                  // block rows per register
    float v[R], c[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int t = r * 64 + lane;
        v[r] = t < SS ? ld(t / S, t % S) : 0.f;
        c[r] = group_scan<S>(v[r], lane);
    }
    float rs = 0.f;   // lanes 0..S-1: row sums
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float t = __shfl(c[r], (lane % G) * S + S - 1);
        if (lane / G == r) rs = t;
    }
    if (lane >= S) rs = 0.f;
    const float M = group_scan<S>(rs, lane);
    const float tot = __shfl(M, S - 1);
    const float tv = u1 * tot;
    const uint64_t bv = __ballot(lane < S && tv < M);
    if (bv) {
        dv = lowest(bv);
    } else {
        const uint64_t bp = __ballot(lane < S && rs > 0.f);
        dv = bp ? highest(bp) : S - 1;
    }
    const int jr = dv / G, gr = dv % G;
    float cj = c[0], vj = v[0];
#pragma unroll
    for (int r = 1; r < R; ++r)
        if (r == jr) { cj = c[r]; vj = v[r]; }
    const float rowsum = __shfl(rs, dv);
    const float tu = u2 * rowsum;
    const bool in_row = lane / S == gr;
    const uint64_t bu = __ballot(in_row && tu < cj);
    if (bu) {
        du = lowest(bu) - gr * S;
    } else {
        const uint64_t bp = __ballot(in_row && vj > 0.f);
        du = bp ? highest(bp) - gr * S : S - 1;
    }
    return __shfl(vj, gr * S + du);
}

}  // namespace prod
}  // namespace wfpg
