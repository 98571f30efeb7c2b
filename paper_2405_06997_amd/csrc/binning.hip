// Positional binning and per-bin guiding on gfx950 (Alg. 2 Partition-S, then
// Alg. 3 with one field per bin): queries are counted into the deepest SVO
// node that holds them, totals are summed bottom-up over the occupancy
// pyramid, nodes with at least c_ray queries (or on level l_min) are marked,
// every query takes its deepest marked ancestor as its bin, each bin draws
// one member as its origin (SelectOrigin), the guide kernel marches one
// N x N field per bin origin, and every member samples its bin's field with
// its own uniforms.
//
// Node identity is the global node index (rank + popcount over the level's
// occupancy bitmap), so all per-node state is a flat array over the SVO's
// nodes; no sort or partition of the queue is needed: members read their
// bin's CDF in place.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "march_core.h"
#include "product_core.h"
#include "antialias_core.h"
#include "wfpg_internal.h"

// Smallest field resolution generated one workgroup per bin (smaller ones go
// through the guide kernel over the list of bin origins).
#ifndef WFPG_BIN_FIELD_MIN_N
#define WFPG_BIN_FIELD_MIN_N 16
#endif

namespace wfpg {
namespace {

using core::woff;

// 16-bit storage formats of the exitance and the field bins (as the guide
// kernels store them): RNE rounding and unpacking.
__device__ __forceinline__ float round16_bin(float f, int fmt)
{
    if (fmt == WFPG_FP16) return __half2float(__float2half_rn(f));
    uint32_t u = __float_as_uint(f);
    return __uint_as_float(((u + 0x7fffu + ((u >> 16) & 1u)) >> 16) << 16);
}
__device__ __forceinline__ float unpack16_bin(uint32_t v, int side, int fmt)
{
    const uint32_t h = side ? (v >> 16) : (v & 0xffffu);
    if (fmt == WFPG_FP16) return __half2float(__ushort_as_half((unsigned short)h));
    return __uint_as_float(h << 16);
}

__device__ __forceinline__ bool node_index(const SvoView &sv, int l, uint32_t key, int64_t &g)
{
    const uint32_t wi = woff(l) + (key >> 6);
    const uint64_t w = sv.bits[wi];
    const uint32_t b = key & 63u;
    if (!((w >> b) & 1ull)) return false;
    const uint64_t below = b ? (w & ((1ull << b) - 1ull)) : 0ull;
    g = (int64_t)sv.rank[wi] + __popcll(below);
    return true;
}

// Level of a global node index (levels are contiguous ranges of noff).
__device__ __forceinline__ int level_of(const SvoView &sv, int64_t g)
{
    int l = 0;
    while (l < sv.depth && g >= sv.noff[l + 1]) ++l;
    return l;
}

// DescendLeaf + AtomicAdd: the deepest existing node holding the quantized
// position (its leaf when occupied); node_of[i] = its global index, or -1
// for an empty SVO.
__global__ void k_bin_count(SvoView sv, const float *__restrict__ pos, int64_t n, int32_t *node_of,
                            uint32_t *count)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int D = sv.depth;
    const uint32_t O0 = core::quantize_pos(pos[i]), O1 = core::quantize_pos(pos[n + i]),
                   O2 = core::quantize_pos(pos[2 * n + i]);
    uint32_t key = core::morton3(O0 >> (WFPG_FINE - D), O1 >> (WFPG_FINE - D), O2 >> (WFPG_FINE - D));
    int64_t g = -1;
    for (int l = D; l >= 0; --l, key >>= 3)
        if (node_index(sv, l, key, g)) break;
    node_of[i] = (int32_t)g;
    if (g >= 0) atomicAdd(&count[g], 1u);
}

// Totals of level l (children's totals added to the node's own count, level
// l + 1 already final) and the marks: T >= c_ray or l == l_min.
__global__ void k_bin_level(SvoView sv, int l, int l_min, uint32_t c_ray, uint32_t *count, uint8_t *mark)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t g = sv.noff[l] + j;
    if (g >= sv.noff[l + 1]) return;
    uint32_t T = count[g];
    if (l < sv.depth) {
        const uint32_t key = sv.keys[g];
        const uint32_t wi = woff(l + 1) + (key >> 3);
        const uint64_t w = sv.bits[wi];
        const uint32_t sh = 8u * (key & 7u);
        const uint32_t kids = (uint32_t)((w >> sh) & 0xffull);
        const int64_t base = (int64_t)sv.rank[wi] + (sh ? __popcll(w & ((1ull << sh) - 1ull)) : 0);
        for (int c = 0; c < __popc(kids); ++c) T += count[base + c];
        count[g] = T;
    }
    mark[g] = (T >= c_ray || l == l_min) ? 1 : 0;
}

// AscendAndFindMarked: bin = deepest marked node on the path from the query's
// node up to level l_min (the node itself when it lies above l_min); the
// bin's origin is the member with the smallest (hash, index). Neighbouring
// queue entries mostly share a bin, so each wave first folds the keys of equal
// bins (every partial minimum is over members of one bin, so any subset is
// correct) and only the first lane of each run of equal bins issues the
// atomic; the run head's fold covers its whole run.
__global__ void __launch_bounds__(256) k_bin_assign(SvoView sv, int l_min, int64_t n, uint64_t seed,
                                                    uint32_t bounce, const int32_t *node_of, const uint8_t *mark,
                                                    int32_t *bin_of, unsigned long long *origin_key)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int32_t bin = -1;
    unsigned long long key = ~0ull;
    if (i < n) {
        const int32_t g0 = node_of[i];
        if (g0 >= 0) {
            const int l0 = level_of(sv, g0);
            const uint32_t k0 = sv.keys[g0];
            int64_t b = g0;
            for (int m = l0; m >= l_min; --m) {
                int64_t g = -1;
                if (!node_index(sv, m, k0 >> (3 * (l0 - m)), g)) continue;   // (ancestors of a node exist)
                if (mark[g]) {
                    b = g;
                    break;
                }
            }
            bin = (int32_t)b;
            uint32_t c[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), bounce, 1u};
            core::philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
            key = ((unsigned long long)c[0] << 32) | (unsigned long long)(uint32_t)i;
        }
        bin_of[i] = bin;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t lo = __shfl_down((uint32_t)key, off);
        const uint32_t hi = __shfl_down((uint32_t)(key >> 32), off);
        const int32_t ob = __shfl_down(bin, off);
        const unsigned long long ok = ((unsigned long long)hi << 32) | lo;
        if (lane + off < 64 && ob == bin && ok < key) key = ok;
    }
    const int32_t prev = __shfl_up(bin, 1);
    if (bin >= 0 && (lane == 0 || prev != bin)) atomicMin(&origin_key[bin], key);
}

// One slot per used bin, the slot's origin position (SoA, plane stride cap).
__global__ void k_bin_slots(int64_t nodes, const unsigned long long *origin_key, const float *__restrict__ pos,
                            int64_t n, int32_t *slot_of, int32_t *nbins, float *opos, int64_t cap)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nodes) return;
    const unsigned long long k = origin_key[g];
    if (k == ~0ull) return;
    const int32_t s = atomicAdd(nbins, 1);
    slot_of[g] = s;
    if (s >= cap) return;   // never: cap bounds the used bins
    const int64_t o = (int64_t)(uint32_t)(k & 0xffffffffull);
    opos[s] = pos[o];
    opos[cap + s] = pos[n + o];
    opos[2 * cap + s] = pos[2 * n + o];
}

// Row CDFs (inclusive prefix within each field row v) and the marginal
// (inclusive prefix of the row sums) of every bin's pdf; one thread per
// (bin, row) for the rows, then the marginal from the row totals.
template <int N>
__global__ void k_bin_cdf(const float *__restrict__ pdf, const int32_t *nbins, float *rcdf)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t b = t / N;
    const int v = (int)(t % N);
    if (b >= *nbins) return;
    const float *p = pdf + b * N * N + v * N;
    float *r = rcdf + b * N * N + v * N;
    float acc = 0.f;
    for (int u = 0; u < N; ++u) {
        acc += p[u];
        r[u] = acc;
    }
}

// Marginal CDF of each bin over its rows: the row sums are the last entries
// of the row CDFs (the same sequential FP32 sums), accumulated in row order.
template <int N>
__global__ void k_bin_marg(const float *__restrict__ rcdf, const int32_t *nbins, float *mcdf)
{
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= *nbins) return;
    float m = 0.f;
    for (int v = 0; v < N; ++v) {
        m += rcdf[b * N * N + v * N + N - 1];
        mcdf[b * N + v] = m;
    }
}

// First k in [0, N) with t < cdf[k] (cdf non-decreasing), N - 1 if none.
template <int N>
__device__ __forceinline__ int upper_index(const float *cdf, float t)
{
    int lo = 0, hi = N - 1;   // the answer lies in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t < cdf[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ void oct_decode_f(float x, float y, float &dx, float &dy, float &dz)
{
    const float a = 2.f * x - 1.f, bb = 2.f * y - 1.f;
    const float aa = fabsf(a), ab = fabsf(bb);
    const float d = 1.f - (aa + ab);
    const float r = 1.f - fabsf(d);
    const float phi = r == 0.f ? 0.f : ((ab - aa) / r + 1.f) * 0.78539816339744831f;
    const float z = (d >= 0.f ? 1.f : -1.f) * (1.f - r * r);
    const float s = r * sqrtf(2.f - r * r);
    float sn, cs;
    sincosf(phi, &sn, &cs);
    dx = (a >= 0.f ? cs : -cs) * s;
    dy = (bb >= 0.f ? sn : -sn) * s;
    dz = z;
}

// Every member samples its bin's field with its own uniforms (counter = its
// queue index): row v = first with u1 * M[N-1] < M[v], column u = first with
// u2 * R_v[N-1] < R_v[u] (clamped to N-1), direction = octahedral decode of
// ((u + u3)/N, (v + u4)/N), pdf = the bin's pdf_b.
template <int N>
__global__ void k_bin_sample(int64_t n, uint64_t seed, uint32_t bounce, const int32_t *bin_of,
                             const int32_t *slot_of, const float *__restrict__ pdf, const float *__restrict__ rcdf,
                             const float *__restrict__ mcdf, float *dir_out, float *pdf_out, int32_t *bin_out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t bin = bin_of[i];
    if (bin_out) bin_out[i] = bin;
    if (bin < 0) {
        dir_out[i] = 0.f;
        dir_out[n + i] = 0.f;
        dir_out[2 * n + i] = 0.f;
        pdf_out[i] = 0.f;
        return;
    }
    const int64_t s = slot_of[bin];
    uint32_t c[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), bounce, 0u};
    core::philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u1 = (float)(c[0] >> 8) * 5.9604644775390625e-8f;
    const float u2 = (float)(c[1] >> 8) * 5.9604644775390625e-8f;
    const float u3 = (float)(c[2] >> 8) * 5.9604644775390625e-8f;
    const float u4 = (float)(c[3] >> 8) * 5.9604644775390625e-8f;
    const float *M = mcdf + s * N;
    const int v = upper_index<N>(M, u1 * M[N - 1]);
    const float *R = rcdf + s * N * N + v * N;
    const int u = upper_index<N>(R, u2 * R[N - 1]);
    const float inv = 1.f / (float)N;
    float ox, oy, oz;
    oct_decode_f((float)u * inv + u3 * inv, (float)v * inv + u4 * inv, ox, oy, oz);
    dir_out[i] = ox;
    dir_out[n + i] = oy;
    dir_out[2 * n + i] = oz;
    pdf_out[i] = pdf[s * N * N + v * N + u];
}

// Upper-level cell sums of every bin field for product guiding (thread per
// (bin, cell)), rows dv outer and columns du inner as the per-vertex path.
template <int N>
__global__ void k_bin_coarse(const float *__restrict__ pdf, const int32_t *nbins, float *coarse)
{
    constexpr int SB = N / prod::kCells;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t b = t >> 6;
    if (b >= *nbins) return;
    const int c = (int)(t & 63), V = c >> 3, U = c & 7;
    const float *p = pdf + b * N * N + (V * SB) * N + U * SB;
    float F = 0.f;
    for (int dv = 0; dv < SB; ++dv)
        for (int du = 0; du < SB; ++du) F += p[dv * N + du];
    coarse[t] = F;
}

// Product sample of every member (Sec. 3.6), a wave per member at a time as
// the paper gives a warp to a ray: lane C takes cell C's sum of the member's
// bin field and the member's table entry, the wave picks the cell, then the
// fine bin inside it from the bin field. A wave owns 64 consecutive members:
// lane m draws member m's uniforms and loads its bin and normal up front,
// the wave then walks the members one by one, and all 64 directions are
// decoded and written together at the end. Grid-stride over member batches.
template <int N>
__global__ void __launch_bounds__(256) k_bin_product(int64_t n, uint64_t seed, uint32_t bounce,
                                                     const int32_t *bin_of, const int32_t *slot_of,
                                                     const float *__restrict__ pdf, const float *__restrict__ coarse,
                                                     const float *nrm, const float *bsdf, const float *tab8,
                                                     float scale, float *dir_out, float *pdf_out, int32_t *bin_out)
{
    constexpr int SB = N / prod::kCells;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const float tx = tab8[3 * lane], ty = tab8[3 * lane + 1], tz = tab8[3 * lane + 2];   // cell centre
    for (int64_t base = ((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6) * 64; base < n; base += waves * 64) {
        const int64_t im = base + lane;   // this lane's member
        const bool valid = im < n;
        const int32_t bin = valid ? bin_of[im] : -1;
        if (valid && bin_out) bin_out[im] = bin;
        const int32_t sl = bin >= 0 ? slot_of[bin] : -1;
        float nx = 0.f, ny = 0.f, nz = 0.f;
        if (valid && !bsdf) {
            nx = nrm[im];
            ny = nrm[n + im];
            nz = nrm[2 * n + im];
        }
        uint32_t w[4] = {(uint32_t)(uint64_t)im, (uint32_t)((uint64_t)im >> 32), bounce, 2u};
        core::philox(w, (uint32_t)seed, (uint32_t)(seed >> 32));
        uint32_t r[4] = {(uint32_t)(uint64_t)im, (uint32_t)((uint64_t)im >> 32), bounce, 0u};
        core::philox(r, (uint32_t)seed, (uint32_t)(seed >> 32));
        const float w1 = (float)(w[0] >> 8) * 5.9604644775390625e-8f, w2 = (float)(w[1] >> 8) * 5.9604644775390625e-8f;
        const float u1 = (float)(r[0] >> 8) * 5.9604644775390625e-8f, u2 = (float)(r[1] >> 8) * 5.9604644775390625e-8f;
        int my_u = 0, my_v = 0;
        float my_pdf = 0.f;
        const int cnt = (int)min((int64_t)64, n - base);
        for (int m = 0; m < cnt; ++m) {   // wave-uniform
            const int32_t slm = __shfl(sl, m);
            if (slm < 0) continue;
            float x;
            if (bsdf) {
                x = bsdf[(base + m) * 64 + lane];
            } else {
                x = core::dot3(__shfl(nx, m), __shfl(ny, m), __shfl(nz, m), tx, ty, tz);
            }
            prod::Upper q;
            prod::upper_level(coarse[(int64_t)slm * 64 + lane], x > 0.f ? x : 0.f, lane, q);
            const int c = prod::pick_cell(q, __shfl(w1, m), __shfl(w2, m), lane);
            const int V = c >> 3, U = c & 7;
            const float *blk = pdf + (int64_t)slm * N * N + (V * SB) * N + U * SB;
            int dv = 0, du = 0;
            const float Lb = prod::pick_fine<SB>([&](int y, int xx) { return blk[y * N + xx]; }, __shfl(u1, m),
                                                 __shfl(u2, m), lane, dv, du);
            const float Pc = __shfl(q.P, c), Fc = __shfl(q.F, c);
            if (lane == m) {
                my_u = U * SB + du;
                my_v = V * SB + dv;
                my_pdf = (Pc / q.total) * (Lb / Fc) * scale;
            }
        }
        if (valid) {
            float ox = 0.f, oy = 0.f, oz = 0.f;
            if (sl >= 0) {
                const float inv = 1.f / (float)N;
                const float u3 = (float)(r[2] >> 8) * 5.9604644775390625e-8f;
                const float u4 = (float)(r[3] >> 8) * 5.9604644775390625e-8f;
                oct_decode_f((float)my_u * inv + u3 * inv, (float)my_v * inv + u4 * inv, ox, oy, oz);
            }
            dir_out[im] = ox;
            dir_out[n + im] = oy;
            dir_out[2 * n + im] = oz;
            pdf_out[im] = my_pdf;
        }
    }
}

// Queue index of each query's bin origin (-1 without a bin).
__global__ void k_origin_of(int64_t n, const int32_t *bin_of, const unsigned long long *origin_key, int32_t *out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = bin_of[i];
    out[i] = b < 0 ? -1 : (int32_t)(uint32_t)(origin_key[b] & 0xffffffffull);
}

// Per-bin fields of N >= 32 (up to the paper's depth-1 128 x 128): one
// workgroup of min(N*N, 1024) threads per bin, as the paper's block per bin.
// Threads march cones c = tid + B j from the bin's origin with the exact
// march, take the
// footprint node, side and exitance as the guide kernels do, keep their
// values in registers, reduce the field total over the block (pairwise: lane
// sums, wave butterflies, then the 16 wave totals) and write
// pdf_c = (L_c / total) * N^2 / (4 pi).
template <int N>
constexpr int bin_field_threads() { return N * N < 1024 ? N * N : 1024; }

template <int N>
__global__ void __launch_bounds__(bin_field_threads<N>()) k_bin_field(
    SvoView sv, const float *__restrict__ opos, int64_t cap, const int32_t *nbins, const float *__restrict__ dirtab,
    float eps, float omega, float pdf_scale, int blur, float *pdf, int32_t *err)
{
    constexpr int NN = N * N, B = bin_field_threads<N>(), PER = NN / B;
    extern __shared__ float L[];   // the bin's field values (first the cones' hit records)
    uint32_t *Lrec = reinterpret_cast<uint32_t *>(L);
    __shared__ float wsum[16];
    const int64_t b = blockIdx.x;
    if (b >= *nbins) return;   // uniform over the block
    const uint64_t *gbits = sv.bits;
    auto bits = [gbits](int, uint32_t wi) -> uint64_t { return gbits[wi]; };   // cached global reads
    const int D = sv.depth, fmt = sv.fmt;
    const uint32_t O[3] = {core::quantize_pos(opos[b]), core::quantize_pos(opos[cap + b]),
                           core::quantize_pos(opos[2 * cap + b])};
    const uint32_t okey = core::morton3(O[0] >> (WFPG_FINE - D), O[1] >> (WFPG_FINE - D), O[2] >> (WFPG_FINE - D));
    const bool occ = (bits(D, woff(D) + (okey >> 6)) >> (okey & 63)) & 1ull;
    // lanes march cones one after another, a few occupancy tests at a time;
    // a lane that finishes takes the block's next unmarched cone (one LDS
    // atomic per wave and refill), so lanes stay busy until the bin's cones
    // run out instead of waiting for the lane with the longest share
    __shared__ int s_next;
    if (threadIdx.x == 0) s_next = B;   // cones 0..B-1 start on their thread
    __syncthreads();
    const int lane = threadIdx.x & 63;
    int cur = threadIdx.x, it = 0;
    bool act = false, more = true;
    float dx = 0.f, dy = 0.f, dz = 0.f;
    core::MicroState st;
    float local = 0.f;
    while (true) {
        if (!act && more) {
            dx = dirtab[3 * cur];
            dy = dirtab[3 * cur + 1];
            dz = dirtab[3 * cur + 2];
            uint32_t a0, a1, a2;
            int s0, s1, s2;
            core::split_dir(core::quantize_dir(dx), a0, s0);
            core::split_dir(core::quantize_dir(dy), a1, s1);
            core::split_dir(core::quantize_dir(dz), a2, s2);
            int vis = 0;
            core::micro_begin(st, O, okey, occ, a0, a1, a2, s0, s1, s2, D, 0, vis);
            act = true;
            it = 0;
        }
        if (__ballot(act) == 0ull) break;   // no cone left for this wave
        int res = core::STEP_CONTINUE;
        core::Hit h = {-1, 0u, 0u};
        if (act) {
            int vis = 0;
            for (int m = 0; m < 4; ++m) {
                res = core::micro_step(st, D, bits, 0, vis, h);
                if (res != core::STEP_CONTINUE) break;
            }
            if (res == core::STEP_CONTINUE && (it += 4) >= core::kMaxTests) {
                atomicOr(err, 1);
                res = core::STEP_MISS;
            }
        }
        if (act && res != core::STEP_CONTINUE) {
            // the cone footprint (Eq. 7) is decided here; its node's value is read in
            // one pass after the march, so a finishing lane never stalls the wave
            // on dependent loads: record = 1 << 3*level | node key (0: a miss)
            uint32_t rv = 0u;
            if (res == core::STEP_HIT) {
                const float dsel = h.axis == 0 ? dx : (h.axis == 1 ? dy : dz);
                const int k = core::footprint_levels(h.delta, fabsf(dsel), D, omega);
                rv = (1u << (3 * (D - k))) | (h.key >> (3 * k));
            }
            Lrec[cur] = rv;
            act = false;
        }
        const uint64_t want = __ballot(!act && more);
        if (want) {
            const int first = __ffsll((unsigned long long)want) - 1;
            int base = 0;
            if (lane == first) base = atomicAdd(&s_next, __popcll(want));
            base = __shfl(base, first);
            if (!act && more) {
                const uint64_t below = want & ((1ull << lane) - 1ull);
                cur = base + __popcll(below);
                more = cur < NN;
            }
        }
    }
    __syncthreads();   // every record of the bin is written
    // values of this thread's cones: footprint node, side, exitance + eps
    for (int q = 0; q < PER; ++q) {
        const int c = threadIdx.x + B * q;
        const uint32_t r = Lrec[c];
        float val = fmt == WFPG_FP32 ? eps : round16_bin(eps, fmt);
        if (r) {
            const int lf = (31 - __builtin_clz(r)) / 3;
            const uint32_t node = r ^ (1u << (3 * lf));
            int64_t g = -1;
            node_index(sv, lf, node, g);   // the footprint node is an ancestor of the hit leaf
            const float4 Nn = sv.nrm[g];
            const int side =
                core::dot3(Nn.x, Nn.y, Nn.z, dirtab[3 * c], dirtab[3 * c + 1], dirtab[3 * c + 2]) < 0.f ? 0 : 1;
            if (fmt == WFPG_FP32) {
                const float2 e = sv.e32[g];
                val = (side ? e.y : e.x) + eps;
            } else {
                const uint32_t pk = sv.e16[g];
                val = round16_bin(unpack16_bin(pk, side, fmt) + eps, fmt);
            }
        }
        L[c] = val;   // in place over the thread's own record
        local += val;
    }
    if (blur) {   // uniform over the block: blur the whole field, then re-total
        float t[PER];
        __syncthreads();
        for (int q = 0; q < PER; ++q) {
            const int c = threadIdx.x + B * q;
            t[q] = aa::blur_at(N, c % N, c / N, [&](int k) { return L[k]; });
        }
        __syncthreads();
        local = 0.f;
        for (int q = 0; q < PER; ++q) {
            L[threadIdx.x + B * q] = t[q];
            local += t[q];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) local += __shfl_xor(local, d);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
    __syncthreads();
    float total = 0.f;
    if (B / 64 == 1) {
        total = wsum[0];
    } else {
        for (int w = 0; w < B / 64; w += 2) total += wsum[w] + wsum[w + 1];
    }
    for (int q = 0; q < PER; ++q) {
        const int c = threadIdx.x + B * q;
        pdf[b * NN + c] = (L[c] / total) * pdf_scale;
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned nblk(int64_t n, unsigned t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

hipError_t grow(void *&p, size_t &have, size_t want)
{
    if (have >= want) return hipSuccess;
    if (p) {
        const hipError_t e = hipFree(p);
        if (e != hipSuccess) return e;
    }
    p = nullptr;
    have = 0;
    const hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) have = want;
    return e;
}

}  // namespace

// Scratch of the binning path, owned by the SVO (grown on demand).
struct BinWork {
    void *count = nullptr, *mark = nullptr, *okey = nullptr, *slot = nullptr, *node_of = nullptr,
         *bin_of = nullptr, *nbins = nullptr, *opos = nullptr, *pdf = nullptr, *rcdf = nullptr,
         *mcdf = nullptr, *coarse = nullptr, *jtab = nullptr;
    size_t s_count = 0, s_mark = 0, s_okey = 0, s_slot = 0, s_node = 0, s_bin = 0, s_nbins = 0, s_opos = 0,
           s_pdf = 0, s_rcdf = 0, s_mcdf = 0, s_coarse = 0, s_jtab = 0;
};

// One workgroup per bin: the field of each bin origin into W->pdf.
template <int N>
void launch_bin_field(int32_t nb, size_t lds, hipStream_t s, const SvoView &v, const BinWork *W, int64_t cap,
                      const float *tab, const wfpg_bin_opts *o, float omega, float scale,
                      const wfpg_svo *svo)
{
    hipLaunchKernelGGL(k_bin_field<N>, dim3((unsigned)nb), dim3(bin_field_threads<N>()), lds, s, v,
                       (const float *)W->opos, cap, (const int32_t *)W->nbins, tab, o->eps, omega, scale,
                       (int)o->blur, (float *)W->pdf, svo->d_err);
}

void destroy_bin_work(void *w)
{
    BinWork *b = (BinWork *)w;
    if (!b) return;
    void *ps[] = {b->count, b->mark, b->okey, b->slot, b->node_of, b->bin_of, b->nbins, b->opos, b->pdf,
                  b->rcdf, b->mcdf, b->coarse, b->jtab};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete b;
}

// Partition-S on the device: bin_of (global node index per query) and the
// origin keys; returns the number of used bins through *nbins_host when it is
// not null (synchronizes then).
hipError_t bin_partition(const wfpg_svo *svo, const float *pos, int64_t n, int c_ray, int l_min,
                         uint64_t seed, uint32_t bounce, hipStream_t s, BinWork *&W)
{
    W = (BinWork *)svo->bin_work;
    if (!W) {
        W = new (std::nothrow) BinWork();
        if (!W) return hipErrorOutOfMemory;
        svo->bin_work = W;
    }
    const int64_t nodes = std::max<int64_t>(1, svo->total_nodes);
    hipError_t e = grow(W->count, W->s_count, nodes * 4);
    if (e == hipSuccess) e = grow(W->mark, W->s_mark, nodes);
    if (e == hipSuccess) e = grow(W->okey, W->s_okey, nodes * 8);
    if (e == hipSuccess) e = grow(W->slot, W->s_slot, nodes * 4);
    if (e == hipSuccess) e = grow(W->node_of, W->s_node, n * 4);
    if (e == hipSuccess) e = grow(W->bin_of, W->s_bin, n * 4);
    if (e == hipSuccess) e = grow(W->nbins, W->s_nbins, 4);
    if (e != hipSuccess) return e;
    const SvoView v = svo->view();
    uint32_t *count = (uint32_t *)W->count;
    hipLaunchKernelGGL(k_fill_u32, dim3(nblk(nodes, 256)), dim3(256), 0, s, count, nodes, 0u);
    hipLaunchKernelGGL(k_fill_u64, dim3(nblk(nodes, 256)), dim3(256), 0, s, (unsigned long long *)W->okey, nodes,
                       ~0ull);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t *)W->nbins, (int64_t)1, 0u);
    hipLaunchKernelGGL(k_bin_count, dim3(nblk(n, 256)), dim3(256), 0, s, v, pos, n, (int32_t *)W->node_of, count);
    for (int l = svo->depth; l >= l_min; --l) {
        const int64_t m = svo->n[l];
        if (m == 0) continue;
        hipLaunchKernelGGL(k_bin_level, dim3(nblk(m, 256)), dim3(256), 0, s, v, l, l_min, (uint32_t)c_ray, count,
                           (uint8_t *)W->mark);
    }
    hipLaunchKernelGGL(k_bin_assign, dim3(nblk(n, 256)), dim3(256), 0, s, v, l_min, n, seed, bounce,
                       (const int32_t *)W->node_of, (const uint8_t *)W->mark, (int32_t *)W->bin_of,
                       (unsigned long long *)W->okey);
    return hipGetLastError();
}

}  // namespace wfpg

using namespace wfpg;

namespace {

bool valid_bin_opts(const wfpg_svo *svo, const wfpg_bin_opts *o)
{
    return o && (o->N == 8 || o->N == 16 || o->N == 32 || o->N == 64 || o->N == 128) && std::isfinite(o->eps) &&
           o->eps > 0.f && o->c_ray >= 1 && o->l_min >= 0 && o->l_min <= svo->depth &&
           (o->jitter == 0 || o->jitter == 1) && (o->blur == 0 || o->blur == 1);
}

wfpg_status st_of(hipError_t e, int line)
{
    if (e == hipSuccess) return WFPG_OK;
    (void)note_error(e, __FILE__, line);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? WFPG_ENOMEM : WFPG_EDEVICE;
}

template <int N>
void launch_cdf_sample(int64_t cap, int64_t n, uint64_t seed, uint32_t bounce, BinWork *W, float *dir_out,
                       float *pdf_out, int32_t *bin_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_cdf<N>, dim3(nblk(cap * N, 256)), dim3(256), 0, s, (const float *)W->pdf,
                       (const int32_t *)W->nbins, (float *)W->rcdf);
    hipLaunchKernelGGL(k_bin_marg<N>, dim3(nblk(cap, 256)), dim3(256), 0, s, (const float *)W->rcdf,
                       (const int32_t *)W->nbins, (float *)W->mcdf);
    hipLaunchKernelGGL(k_bin_sample<N>, dim3(nblk(n, 256)), dim3(256), 0, s, n, seed, bounce,
                       (const int32_t *)W->bin_of, (const int32_t *)W->slot, (const float *)W->pdf,
                       (const float *)W->rcdf, (const float *)W->mcdf, dir_out, pdf_out, bin_out);
}

template <int N>
void launch_product(int64_t m, int64_t n, uint64_t seed, uint32_t bounce, const BinWork *W, const float *nrm,
                    const float *bsdf, const float *tab8, float *dir_out, float *pdf_out, int32_t *bin_out,
                    hipStream_t s)
{
    const double pi = 3.14159265358979323846;
    hipLaunchKernelGGL(k_bin_coarse<N>, dim3(nblk(m * 64, 256)), dim3(256), 0, s, (const float *)W->pdf,
                       (const int32_t *)W->nbins, (float *)W->coarse);
    const int64_t blocks = std::min<int64_t>(nblk(n, 256), (int64_t)1 << 20);   // 64 members per wave
    hipLaunchKernelGGL(k_bin_product<N>, dim3((unsigned)blocks), dim3(256), 0, s, n, seed, bounce,
                       (const int32_t *)W->bin_of, (const int32_t *)W->slot, (const float *)W->pdf,
                       (const float *)W->coarse, nrm, bsdf, tab8, (float)((double)(N * N) / (4.0 * pi)), dir_out,
                       pdf_out, bin_out);
}

// Partition-S, bin slots and one field per used bin (normalized pdf values in
// W->pdf, slot-major); m = max(1, used bins). Synchronizes once.
hipError_t binned_fields(const wfpg_svo *svo, const float *pos, int64_t n, uint64_t seed, uint32_t bounce,
                         const wfpg_bin_opts *opts, hipStream_t s, BinWork *&W, int64_t &m)
{
    hipError_t e = bin_partition(svo, pos, n, opts->c_ray, opts->l_min, seed, bounce, s, W);
    int32_t nb = 0;
    // bins are nodes used by at least one query: at most min(n, nodes)
    const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(n, svo->total_nodes));
    const int N = opts->N, NN = N * N;
    if (e == hipSuccess) e = grow(W->opos, W->s_opos, cap * 3 * 4);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_bin_slots, dim3(nblk(std::max<int64_t>(1, svo->total_nodes), 256)), dim3(256), 0, s,
                           svo->total_nodes, (const unsigned long long *)W->okey, pos, n, (int32_t *)W->slot,
                           (int32_t *)W->nbins, (float *)W->opos, cap);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&nb, W->nbins, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && (nb < 0 || nb > cap)) e = hipErrorUnknown;
    m = std::max<int32_t>(nb, 1);
    if (e == hipSuccess) e = grow(W->pdf, W->s_pdf, m * NN * 4);
    if (e == hipSuccess && nb > 0 && N >= WFPG_BIN_FIELD_MIN_N) {   // one workgroup per bin field
        const double pi = 3.14159265358979323846;
        const float *tab = device_dirtab(N);
        if (opts->jitter && tab) {   // this call's jittered cone directions, once, into the bin scratch
            e = grow(W->jtab, W->s_jtab, (size_t)NN * 3 * 4);
            if (e == hipSuccess) e = launch_jitter_table(N, opts->jitter_key, (float *)W->jtab, s);
            tab = e == hipSuccess ? (const float *)W->jtab : nullptr;
        }
        const size_t lds = (size_t)NN * 4;   // the field
        const SvoView v = svo->view();
        const float omega = (float)(4.0 * pi / (double)NN), scale = (float)((double)NN / (4.0 * pi));
        if (!tab) e = hipErrorOutOfMemory;
        else if (N == 16) launch_bin_field<16>(nb, lds, s, v, W, cap, tab, opts, omega, scale, svo);
        else if (N == 32) launch_bin_field<32>(nb, lds, s, v, W, cap, tab, opts, omega, scale, svo);
        else if (N == 64) launch_bin_field<64>(nb, lds, s, v, W, cap, tab, opts, omega, scale, svo);
        else launch_bin_field<128>(nb, lds, s, v, W, cap, tab, opts, omega, scale, svo);
        if (e == hipSuccess) e = hipGetLastError();
    } else if (e == hipSuccess && nb > 0) {   // one field per bin origin (plane stride cap)
        GuideArgs a;
        std::memset(&a, 0, sizeof a);
        const double pi = 3.14159265358979323846;
        a.pos = (const float *)W->opos;
        a.n = nb;
        a.stride = cap;
        a.eps = opts->eps;
        a.omega = (float)(4.0 * pi / (double)NN);
        a.pdf_scale = (float)((double)NN / (4.0 * pi));
        a.dirtab = device_dirtab(N);
        a.err = svo->d_err;
        a.pdf_out = (float *)W->pdf;
        a.jitter = opts->jitter;
        a.jitter_key = opts->jitter_key;
        a.blur = opts->blur;
        e = a.dirtab ? launch_guide(svo, N, MODE_PDF, a, choose_tile(svo, N), s) : hipErrorOutOfMemory;
    }
    return e;
}

}  // namespace

extern "C" {

wfpg_bin_opts wfpg_default_bin_opts(void)
{
    wfpg_bin_opts o;
    o.N = 16;
    o.eps = 0.01f;
    o.c_ray = 512;
    o.l_min = 5;
    o.jitter = 0;
    o.jitter_key = 0;
    o.blur = 0;
    return o;
}

wfpg_status wfpg_partition(const wfpg_svo *svo, const float *pos, int64_t n, int32_t c_ray, int32_t l_min,
                           uint64_t seed, uint32_t bounce, int32_t *bin_out, int32_t *origin_out,
                           void *hip_stream)
{
    if (!svo || n < 0 || n > 0x7fffffffLL || c_ray < 1 || l_min < 0 || l_min > svo->depth ||
        (n > 0 && (!pos || !bin_out)))
        return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    BinWork *W = nullptr;
    hipError_t e = bin_partition(svo, pos, n, c_ray, l_min, seed, bounce, s, W);
    if (e == hipSuccess) e = hipMemcpyAsync(bin_out, W->bin_of, n * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && origin_out) {
        hipLaunchKernelGGL(k_origin_of, dim3(nblk(n, 256)), dim3(256), 0, s, n, (const int32_t *)W->bin_of,
                           (const unsigned long long *)W->okey, origin_out);
        e = hipGetLastError();
    }
    return st_of(e, __LINE__);
}

wfpg_status guide_sample_binned(const wfpg_svo *svo, const float *pos, int64_t n, uint64_t seed,
                                uint32_t bounce, const wfpg_bin_opts *opts, float *dir_out, float *pdf_out,
                                int32_t *bin_out, void *hip_stream)
{
    if (!svo || n < 0 || n > 0x7fffffffLL || !valid_bin_opts(svo, opts) ||
        (n > 0 && (!pos || !dir_out || !pdf_out)))
        return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    BinWork *W = nullptr;
    int64_t m = 1;
    const int N = opts->N;
    hipError_t e = binned_fields(svo, pos, n, seed, bounce, opts, s, W, m);
    if (e == hipSuccess) e = grow(W->rcdf, W->s_rcdf, m * N * N * 4);
    if (e == hipSuccess) e = grow(W->mcdf, W->s_mcdf, m * N * 4);
    if (e == hipSuccess) {
        switch (N) {
        case 8: launch_cdf_sample<8>(m, n, seed, bounce, W, dir_out, pdf_out, bin_out, s); break;
        case 16: launch_cdf_sample<16>(m, n, seed, bounce, W, dir_out, pdf_out, bin_out, s); break;
        case 32: launch_cdf_sample<32>(m, n, seed, bounce, W, dir_out, pdf_out, bin_out, s); break;
        case 64: launch_cdf_sample<64>(m, n, seed, bounce, W, dir_out, pdf_out, bin_out, s); break;
        default: launch_cdf_sample<128>(m, n, seed, bounce, W, dir_out, pdf_out, bin_out, s); break;
        }
        e = hipGetLastError();
    }
    return st_of(e, __LINE__);
}

wfpg_status guide_sample_binned_product(const wfpg_svo *svo, const float *pos, const float *nrm,
                                        const float *bsdf, int64_t n, uint64_t seed, uint32_t bounce,
                                        const wfpg_bin_opts *opts, float *dir_out, float *pdf_out,
                                        int32_t *bin_out, void *hip_stream)
{
    if (!svo || n < 0 || n > 0x7fffffffLL || !valid_bin_opts(svo, opts) ||
        (n > 0 && (!pos || !dir_out || !pdf_out || (nrm != nullptr) == (bsdf != nullptr))))
        return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    BinWork *W = nullptr;
    int64_t m = 1;
    const int N = opts->N;
    const float *tab8 = device_dirtab(8);
    if (!tab8) return WFPG_ENOMEM;
    hipError_t e = binned_fields(svo, pos, n, seed, bounce, opts, s, W, m);
    if (e == hipSuccess) e = grow(W->coarse, W->s_coarse, m * 64 * 4);
    if (e == hipSuccess) {
        switch (N) {
        case 8: launch_product<8>(m, n, seed, bounce, W, nrm, bsdf, tab8, dir_out, pdf_out, bin_out, s); break;
        case 16: launch_product<16>(m, n, seed, bounce, W, nrm, bsdf, tab8, dir_out, pdf_out, bin_out, s); break;
        case 32: launch_product<32>(m, n, seed, bounce, W, nrm, bsdf, tab8, dir_out, pdf_out, bin_out, s); break;
        case 64: launch_product<64>(m, n, seed, bounce, W, nrm, bsdf, tab8, dir_out, pdf_out, bin_out, s); break;
        default: launch_product<128>(m, n, seed, bounce, W, nrm, bsdf, tab8, dir_out, pdf_out, bin_out, s); break;
        }
        e = hipGetLastError();
    }
    return st_of(e, __LINE__);
}

}  // extern "C"
