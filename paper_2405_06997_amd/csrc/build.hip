// SVO generation on the GPU (Sec. 3.2): voxelization of axis-aligned
// rectangles into a dense leaf bitmap, bottom-up OR reduction to the coarser
// levels, rank (popcount prefix) arrays that give every node its index,
// sorted key lists, and the k = 2 k-means normals of Fig. 2.
//
// No sort is needed: the Morton-ordered bitmaps already hold every level's
// keys in sorted order, so "sort fragments by Morton code" becomes "set bits,
// then compact".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "wfpg_internal.h"

namespace wfpg {
namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;  // words per block

__device__ __forceinline__ uint32_t part1by2(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}

// Cell of fragment f (one leaf cell of one rectangle).
__device__ __forceinline__ uint32_t frag_key(const RectCells *rc, const int64_t *foff,
                                             int64_t n_rects, int64_t f, int32_t *rect_out)
{
    int64_t lo = 0, hi = n_rects - 1;
    while (lo < hi) {  // last rect with foff[r] <= f
        int64_t mid = (lo + hi + 1) >> 1;
        if (foff[mid] <= f) lo = mid; else hi = mid - 1;
    }
    const RectCells r = rc[lo];
    int64_t local = f - foff[lo];
    int64_t nb = (int64_t)(r.b1 - r.b0 + 1);
    uint32_t p = (uint32_t)(r.a0 + local / nb), q = (uint32_t)(r.b0 + local % nb);
    uint32_t c[3];
    int j0 = r.axis == 0 ? 1 : 0, j1 = r.axis == 2 ? 1 : 2;
    c[r.axis] = (uint32_t)r.ca;
    c[j0] = p;
    c[j1] = q;
    *rect_out = (int32_t)lo;
    return morton3(c[0], c[1], c[2]);
}

__global__ void k_vox(const RectCells *rc, const int64_t *foff, int64_t n_rects, int64_t n_frag,
                      uint64_t *bits_leaf)
{
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n_frag;
         f += (int64_t)gridDim.x * blockDim.x) {
        int32_t r;
        uint32_t k = frag_key(rc, foff, n_rects, f, &r);
        atomicOr((unsigned long long *)&bits_leaf[k >> 6], 1ull << (k & 63));
    }
}

// Parent bit k is set iff child byte k is nonzero.
__global__ void k_reduce(const uint64_t *child, uint64_t child_words, uint64_t *parent,
                         uint64_t parent_words)
{
    uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (w >= parent_words) return;
    uint64_t out = 0;
    for (int i = 0; i < 8; ++i) {
        uint64_t cw = 8 * w + i;
        if (cw >= child_words) break;
        uint64_t v = child[cw];
        for (int b = 0; b < 8; ++b)
            if ((v >> (8 * b)) & 0xffull) out |= 1ull << (8 * i + b);
    }
    parent[w] = out;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive block scan of per-thread values; returns the block total.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *excl, uint32_t *sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[wv] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < wv) base += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *excl = base + inc - v;
    return tot;
}

__global__ void k_scan_reduce(const uint64_t *words, uint64_t n, uint32_t *bsum)
{
    __shared__ uint32_t sh[SCAN_THREADS / 64];
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        uint64_t w = base + (uint64_t)threadIdx.x * SCAN_ITEMS + i;
        if (w < n) s += __popcll(words[w]);
    }
    uint32_t ex;
    uint32_t tot = block_excl_scan(s, &ex, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb block sums in place; total to *total.
__global__ void k_scan_blocks(uint32_t *bsum, uint32_t nb, int64_t *total)
{
    __shared__ uint32_t sh[1024 / 64];
    uint32_t carry = 0;
    for (uint32_t start = 0; start < nb; start += blockDim.x) {
        uint32_t i = start + threadIdx.x;
        uint32_t v = i < nb ? bsum[i] : 0;
        uint32_t ex;
        uint32_t tot = block_excl_scan(v, &ex, sh);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_final(const uint64_t *words, uint64_t n, const uint32_t *bsum,
                             uint32_t base, uint32_t *rank)
{
    __shared__ uint32_t sh[SCAN_THREADS / 64];
    uint64_t b0 = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t c[SCAN_ITEMS];
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        c[i] = (b0 + i < n) ? (uint32_t)__popcll(words[b0 + i]) : 0u;
        s += c[i];
    }
    uint32_t ex;
    block_excl_scan(s, &ex, sh);
    uint32_t run = base + bsum[blockIdx.x] + ex;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (b0 + i < n) rank[b0 + i] = run;
        run += c[i];
    }
}

__global__ void k_keys(const uint64_t *words, const uint32_t *rank, uint64_t n, uint32_t *keys)
{
    uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (w >= n) return;
    uint64_t v = words[w];
    uint32_t r = rank[w];
    while (v) {
        int b = __ffsll((unsigned long long)v) - 1;
        keys[r++] = (uint32_t)(w * 64 + b);
        v &= v - 1;
    }
}

__device__ __forceinline__ uint32_t node_index(const uint64_t *bits, const uint32_t *rank,
                                               uint64_t woff, uint32_t key)
{
    uint64_t w = bits[woff + (key >> 6)];
    uint64_t m = (key & 63) ? (w & ((1ull << (key & 63)) - 1)) : 0ull;
    return rank[woff + (key >> 6)] + (uint32_t)__popcll(m);
}

// Per-leaf histogram of fragment normal classes and the smallest rectangle
// index (the k-means seed fragment).
__global__ void k_leaf_hist(const RectCells *rc, const int64_t *foff, int64_t n_rects,
                            int64_t n_frag, const uint64_t *bits, const uint32_t *rank,
                            uint64_t woffD, int64_t noffD, uint32_t *hist, uint32_t *seed)
{
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n_frag;
         f += (int64_t)gridDim.x * blockDim.x) {
        int32_t r;
        uint32_t k = frag_key(rc, foff, n_rects, f, &r);
        int64_t leaf = (int64_t)node_index(bits, rank, woffD, k) - noffD;
        int cls = rc[r].cls;
        atomicAdd(&hist[6 * leaf + cls], 1u);
        atomicMin(&seed[leaf], ((uint32_t)r << 3) | (uint32_t)cls);
    }
}

__device__ __forceinline__ float dot3(const float *a, const float *b)
{
    return __fadd_rn(__fadd_rn(__fmul_rn(a[0], b[0]), __fmul_rn(a[1], b[1])), __fmul_rn(a[2], b[2]));
}

// k-means (k = 2) of a leaf's fragment normals, computed from the class
// histogram: every fragment normal is +-e_axis, so its dot products with a
// mean are +-mean[axis] exactly and the cluster sums are integers, exact in
// FP32 whatever the summation order. The result equals clustering the
// fragments one by one in rectangle order.
__global__ void k_leaf_kmeans(const uint32_t *hist, const uint32_t *seed, int64_t nleaf,
                              int64_t noffD, float4 *nrm)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    uint32_t h[6];
    for (int c = 0; c < 6; ++c) h[c] = hist[6 * i + c];
    int sc = (int)(seed[i] & 7u);
    float muA[3] = {0.f, 0.f, 0.f}, muB[3] = {0.f, 0.f, 0.f};
    muA[sc >> 1] = (sc & 1) ? 1.f : -1.f;
    muB[sc >> 1] = (sc & 1) ? -1.f : 1.f;
    // the seed normal's other components are +0 in muA; in muB they are -0
    for (int k = 0; k < 3; ++k)
        if (k != (sc >> 1)) muB[k] = -0.f;
    int asg[6] = {-1, -1, -1, -1, -1, -1};
    for (int it = 0; it < 16; ++it) {
        bool changed = false;
        for (int c = 0; c < 6; ++c) {
            if (!h[c]) continue;
            float s = (c & 1) ? 1.f : -1.f;
            int ax = c >> 1;
            int a = (s * muA[ax] >= s * muB[ax]) ? 0 : 1;
            if (a != asg[c]) changed = true;
            asg[c] = a;
        }
        if (!changed) break;
        int sA[3] = {0, 0, 0}, sB[3] = {0, 0, 0};
        uint32_t nA = 0, nB = 0;
        for (int c = 0; c < 6; ++c) {
            if (!h[c]) continue;
            int v = (c & 1) ? (int)h[c] : -(int)h[c];
            if (asg[c] == 0) { sA[c >> 1] += v; nA += h[c]; }
            else { sB[c >> 1] += v; nB += h[c]; }
        }
        if (nA) {
            float f[3] = {(float)sA[0], (float)sA[1], (float)sA[2]};
            float len = __builtin_sqrtf(dot3(f, f));
            for (int k = 0; k < 3; ++k) muA[k] = __fdiv_rn(f[k], len);
        }
        if (nB) {
            float f[3] = {(float)sB[0], (float)sB[1], (float)sB[2]};
            float len = __builtin_sqrtf(dot3(f, f));
            for (int k = 0; k < 3; ++k) muB[k] = __fdiv_rn(f[k], len);
        }
    }
    nrm[noffD + i] = make_float4(muA[0], muA[1], muA[2], 0.f);
}

// Inner-node normal: k-means (k = 2) over the occupied children's normals in
// octant order, seeded with the first child, one item at a time in FP32.
__global__ void k_inner_kmeans(const uint64_t *bits, const uint32_t *rank, const uint32_t *keys,
                               int64_t nnode, int64_t noffL, uint64_t woffC, float4 *nrm)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nnode) return;
    uint32_t key = keys[noffL + i];
    uint64_t cw = bits[woffC + (key >> 3)];
    int sh = (int)(key & 7u) * 8;
    uint32_t mask = (uint32_t)((cw >> sh) & 0xffull);
    uint32_t base = rank[woffC + (key >> 3)] + (uint32_t)__popcll(sh ? (cw & ((1ull << sh) - 1)) : 0ull);
    int m = __popc(mask);
    float v[8][3];
    for (int t = 0; t < 8; ++t) {
        if (t < m) {
            float4 c = nrm[base + t];
            v[t][0] = c.x; v[t][1] = c.y; v[t][2] = c.z;
        }
    }
    float muA[3] = {v[0][0], v[0][1], v[0][2]};
    float muB[3] = {-v[0][0], -v[0][1], -v[0][2]};
    int asg[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    for (int it = 0; it < 16; ++it) {
        bool changed = false;
        for (int t = 0; t < 8; ++t) {
            if (t >= m) break;
            int a = dot3(v[t], muA) >= dot3(v[t], muB) ? 0 : 1;
            if (a != asg[t]) changed = true;
            asg[t] = a;
        }
        if (!changed) break;
        float sA[3] = {0.f, 0.f, 0.f}, sB[3] = {0.f, 0.f, 0.f};
        int nA = 0, nB = 0;
        for (int t = 0; t < 8; ++t) {
            if (t >= m) break;
            float *s = asg[t] == 0 ? sA : sB;
            for (int k = 0; k < 3; ++k) s[k] = __fadd_rn(s[k], v[t][k]);
            if (asg[t] == 0) ++nA; else ++nB;
        }
        if (nA) {
            float len = __builtin_sqrtf(dot3(sA, sA));
            for (int k = 0; k < 3; ++k) muA[k] = __fdiv_rn(sA[k], len);
        }
        if (nB) {
            float len = __builtin_sqrtf(dot3(sB, sB));
            for (int k = 0; k < 3; ++k) muB[k] = __fdiv_rn(sB[k], len);
        }
    }
    nrm[noffL + i] = make_float4(muA[0], muA[1], muA[2], 0.f);
}

inline unsigned nblocks(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

#define HIP_TRY(x) WFPG_HIP_TRY(x)

hipError_t launch_build(wfpg_svo *svo, const RectCells *d_rects, const int64_t *d_foff,
                        int64_t n_rects, int64_t n_frag, hipStream_t s)
{
    const int D = svo->depth;
    uint64_t *bits = svo->d_bits;
    int cus = device_cu_count();
    unsigned grid_frag = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n_frag + 255) / 256),
                                                     (int64_t)cus * 64);
    if (n_frag > 0)
        hipLaunchKernelGGL(k_vox, dim3(grid_frag), dim3(256), 0, s, d_rects, d_foff, n_rects,
                           n_frag, bits + level_woff(D));
    for (int l = D - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_reduce, dim3(nblocks(level_words(l), 256)), dim3(256), 0, s,
                           bits + level_woff(l + 1), level_words(l + 1), bits + level_woff(l),
                           level_words(l));
    HIP_TRY(hipGetLastError());
    // rank: block sums per level, then one readback of the level totals
    std::vector<uint64_t> boff(D + 2, 0);
    for (int l = 0; l <= D; ++l) boff[l + 1] = boff[l] + nblocks(level_words(l), SCAN_TILE);
    uint32_t *d_bsum = nullptr;
    int64_t *d_tot = nullptr;
    HIP_TRY(hipMalloc((void **)&d_bsum, boff[D + 1] * sizeof(uint32_t)));
    HIP_TRY(hipMalloc((void **)&d_tot, (D + 1) * sizeof(int64_t)));
    for (int l = 0; l <= D; ++l) {
        uint32_t nb = nblocks(level_words(l), SCAN_TILE);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_THREADS), 0, s,
                           bits + level_woff(l), level_words(l), d_bsum + boff[l]);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, d_bsum + boff[l], nb, d_tot + l);
    }
    HIP_TRY(hipGetLastError());
    int64_t tot[WFPG_MAXD + 1];
    HIP_TRY(hipMemcpyAsync(tot, d_tot, (D + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    svo->noff[0] = 0;
    for (int l = 0; l <= D; ++l) {
        svo->n[l] = tot[l];
        svo->noff[l + 1] = svo->noff[l] + tot[l];
    }
    for (int l = D + 1; l < WFPG_MAXD + 2; ++l) svo->noff[l] = svo->noff[D + 1];
    svo->total_nodes = svo->noff[D + 1];
    for (int l = 0; l <= D; ++l)
        hipLaunchKernelGGL(k_scan_final, dim3(nblocks(level_words(l), SCAN_TILE)),
                           dim3(SCAN_THREADS), 0, s, bits + level_woff(l), level_words(l),
                           d_bsum + boff[l], (uint32_t)svo->noff[l], svo->d_rank + level_woff(l));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(d_bsum));
    HIP_TRY(hipFree(d_tot));
    // per-node arrays
    const int64_t NT = std::max<int64_t>(svo->total_nodes, 1);
    const int64_t L = std::max<int64_t>(svo->n[D], 1);
    HIP_TRY(hipMalloc((void **)&svo->d_keys, NT * sizeof(uint32_t)));
    HIP_TRY(hipMalloc((void **)&svo->d_nrm, NT * sizeof(float4)));
    HIP_TRY(hipMalloc((void **)&svo->d_e32, NT * sizeof(float2)));
    HIP_TRY(hipMalloc((void **)&svo->d_e16, NT * sizeof(uint32_t)));
    HIP_TRY(hipMalloc((void **)&svo->d_sum, L * sizeof(float2)));
    HIP_TRY(hipMalloc((void **)&svo->d_cnt, L * sizeof(uint2)));
    HIP_TRY(hipMemsetAsync(svo->d_e32, 0, NT * sizeof(float2), s));
    HIP_TRY(hipMemsetAsync(svo->d_e16, 0, NT * sizeof(uint32_t), s));
    HIP_TRY(hipMemsetAsync(svo->d_sum, 0, L * sizeof(float2), s));
    HIP_TRY(hipMemsetAsync(svo->d_cnt, 0, L * sizeof(uint2), s));
    for (int l = 0; l <= D; ++l)
        hipLaunchKernelGGL(k_keys, dim3(nblocks(level_words(l), 256)), dim3(256), 0, s,
                           bits + level_woff(l), svo->d_rank + level_woff(l), level_words(l),
                           svo->d_keys);
    HIP_TRY(hipGetLastError());
    if (svo->n[D] > 0) {
        uint32_t *d_hist = nullptr, *d_seed = nullptr;
        HIP_TRY(hipMalloc((void **)&d_hist, L * 6 * sizeof(uint32_t)));
        HIP_TRY(hipMalloc((void **)&d_seed, L * sizeof(uint32_t)));
        HIP_TRY(hipMemsetAsync(d_hist, 0, L * 6 * sizeof(uint32_t), s));
        HIP_TRY(hipMemsetAsync(d_seed, 0xff, L * sizeof(uint32_t), s));
        hipLaunchKernelGGL(k_leaf_hist, dim3(grid_frag), dim3(256), 0, s, d_rects, d_foff, n_rects,
                           n_frag, bits, svo->d_rank, level_woff(D), svo->noff[D], d_hist, d_seed);
        hipLaunchKernelGGL(k_leaf_kmeans, dim3(nblocks(svo->n[D], 256)), dim3(256), 0, s, d_hist,
                           d_seed, svo->n[D], svo->noff[D], svo->d_nrm);
        for (int l = D - 1; l >= 0; --l)
            if (svo->n[l] > 0)
                hipLaunchKernelGGL(k_inner_kmeans, dim3(nblocks(svo->n[l], 256)), dim3(256), 0, s,
                                   bits, svo->d_rank, svo->d_keys, svo->n[l], svo->noff[l],
                                   level_woff(l + 1), svo->d_nrm);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(d_hist));
        HIP_TRY(hipFree(d_seed));
    }
    return hipGetLastError();
}

}  // namespace wfpg
