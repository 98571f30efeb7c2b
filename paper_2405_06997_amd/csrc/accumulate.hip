// UpdateExitance (Alg. 1; Sec. 3.2 after Eq. 5): splat path-vertex radiance
// estimates into their SVO leaves, then average bottom-up (Sec. 3.2).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wfpg_internal.h"

namespace wfpg {
namespace {

__device__ __forceinline__ uint32_t part1by2(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz)
{
    return __fadd_rn(__fadd_rn(__fmul_rn(ax, bx), __fmul_rn(ay, by)), __fmul_rn(az, bz));
}

__device__ __forceinline__ uint32_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;   // RNE; inputs are finite
}
__device__ __forceinline__ uint32_t to_f16(float f)
{
    return (uint32_t)__half_as_ushort(__float2half_rn(f));
}

// One splat (position p, outgoing direction w, rgb c): luminance y =
// (0.2126 r + 0.7152 g) + 0.0722 b in FP32; the leaf of p; side 0 iff
// dot(N_leaf, w) >= 0; FP32/uint32 atomic accumulation. Returns false for an
// invalid or unplaceable splat (counted as dropped by the caller).
__device__ __forceinline__ bool splat_one(const SvoView &sv, const float p[3], const float w[3], const float c[3],
                                          float2 *sum, uint2 *cnt)
{
    const int D = sv.depth;
    const float R = (float)(1 << D);
    const uint64_t woffD = level_woff(D);
    bool ok = true;
    for (int k = 0; k < 3; ++k) ok = ok && isfinite(p[k]) && isfinite(w[k]) && isfinite(c[k]);
    const float y = __fadd_rn(__fadd_rn(__fmul_rn(0.2126f, c[0]), __fmul_rn(0.7152f, c[1])),
                              __fmul_rn(0.0722f, c[2]));
    ok = ok && (y >= 0.f) && isfinite(y);
    uint32_t cell[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        ok = ok && p[k] >= 0.f && p[k] <= 1.f;
        const int v = ok ? (int)floorf(__fmul_rn(p[k], R)) : 0;
        cell[k] = (uint32_t)min(v, (1 << D) - 1);
    }
    if (!ok) return false;
    const uint32_t key = part1by2(cell[0]) | (part1by2(cell[1]) << 1) | (part1by2(cell[2]) << 2);
    const uint64_t word = sv.bits[woffD + (key >> 6)];
    if (!((word >> (key & 63)) & 1ull)) return false;
    const uint64_t m = (key & 63) ? (word & ((1ull << (key & 63)) - 1)) : 0ull;
    const int64_t g = (int64_t)sv.rank[woffD + (key >> 6)] + __popcll(m);
    const int64_t leaf = g - sv.noff[D];
    const float4 N = sv.nrm[g];
    const int side = dot3(N.x, N.y, N.z, w[0], w[1], w[2]) >= 0.f ? 0 : 1;
    unsafeAtomicAdd(side ? &sum[leaf].y : &sum[leaf].x, y);
    atomicAdd(side ? &cnt[leaf].y : &cnt[leaf].x, 1u);
    return true;
}

// One thread per splat.
__global__ void k_splat(SvoView sv, const float *__restrict__ pos, const float *__restrict__ wo,
                        const float *__restrict__ rgb, int64_t n, float2 *sum, uint2 *cnt,
                        unsigned long long *dropped)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool drop = false;
    if (i < n) {
        float p[3], w[3], c[3];
        for (int k = 0; k < 3; ++k) {
            p[k] = pos[k * n + i];
            w[k] = wo[k * n + i];
            c[k] = rgb[k * n + i];
        }
        drop = !splat_one(sv, p, w, c, sum, cnt);
    }
    const uint64_t b = __ballot(drop);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(dropped, (unsigned long long)__popcll(b));
}

// Exitance extraction (Eq. 5), one thread per (depth k, path i), depth-major
// so a wave reads consecutive paths of one depth plane: when path i reached an
// emitter at depth n = hit[i] (1..d) with radiance Le toward p_{n-1}, every
// k <= n splats (T_n / T_k) Le (per channel, FP32; 0 where T_k is 0) at p_k
// with outgoing direction p_{k-1} - p_k (p_0 = the path's eye point).
__global__ void k_splat_paths(SvoView sv, const float *__restrict__ pos, const float *__restrict__ T,
                              const float *__restrict__ eye, const int32_t *__restrict__ hit,
                              const float *__restrict__ Le, int64_t P, int d, bool place, float2 *sum,
                              uint2 *cnt, unsigned long long *dropped)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool drop = false;
    if (t < P * d) {
        const int k = (int)(t / P) + 1;
        const int64_t i = t - (int64_t)(k - 1) * P;
        const int n = hit[i];
        if (n >= 1 && n <= d && k <= n) {
            const float *pk = pos + (int64_t)(k - 1) * 3 * P;
            const float *pp = k > 1 ? pos + (int64_t)(k - 2) * 3 * P : eye;
            const float *Tk = T + (int64_t)(k - 1) * 3 * P;
            const float *Tn = T + (int64_t)(n - 1) * 3 * P;
            float p[3], w[3], c[3];
            for (int q = 0; q < 3; ++q) {
                p[q] = pk[q * P + i];
                w[q] = __fsub_rn(pp[q * P + i], p[q]);
                const float tk = Tk[q * P + i];
                const float ratio = tk == 0.f ? 0.f : __fdiv_rn(Tn[q * P + i], tk);
                c[q] = __fmul_rn(ratio, Le[q * P + i]);
            }
            drop = !place || !splat_one(sv, p, w, c, sum, cnt);   // an SVO without leaves places none
        }
    }
    const uint64_t b = __ballot(drop);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(dropped, (unsigned long long)__popcll(b));
}

__device__ __forceinline__ void store16(uint32_t *e16, int64_t g, float2 e, int fmt)
{
    if (fmt == WFPG_FP16) e16[g] = to_f16(e.x) | (to_f16(e.y) << 16);
    else if (fmt == WFPG_BF16) e16[g] = to_bf16(e.x) | (to_bf16(e.y) << 16);
}

// Leaf exitance: mean of the splats of each side (0 without splats).
__global__ void k_prop_leaf(const float2 *sum, const uint2 *cnt, int64_t nleaf, int64_t noffD,
                            float2 *e32, uint32_t *e16, int fmt)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    float2 s = sum[i];
    uint2 c = cnt[i];
    float2 e;
    e.x = c.x ? __fdiv_rn(s.x, (float)c.x) : 0.f;
    e.y = c.y ? __fdiv_rn(s.y, (float)c.y) : 0.f;
    e32[noffD + i] = e;
    store16(e16, noffD + i, e, fmt);
}

// Inner exitance: per side, the FP32 mean in octant order over the occupied
// children of the child side facing the same way (swapped when the child
// normal points away from the parent's).
__global__ void k_prop_inner(SvoView sv, int64_t nnode, int64_t noffL, uint64_t woffC,
                             float2 *e32, uint32_t *e16, int fmt)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nnode) return;
    int64_t g = noffL + i;
    uint32_t key = sv.keys[g];
    uint64_t cw = sv.bits[woffC + (key >> 3)];
    int sh = (int)(key & 7u) * 8;
    uint32_t mask = (uint32_t)((cw >> sh) & 0xffull);
    uint32_t base = sv.rank[woffC + (key >> 3)] + (uint32_t)__popcll(sh ? (cw & ((1ull << sh) - 1)) : 0ull);
    int m = __popc(mask);
    float4 P = sv.nrm[g];
    float a0 = 0.f, a1 = 0.f;
    for (int t = 0; t < m; ++t) {
        float4 Cn = sv.nrm[base + t];
        float2 ce = e32[base + t];
        bool flip = !(dot3(Cn.x, Cn.y, Cn.z, P.x, P.y, P.z) >= 0.f);
        a0 = __fadd_rn(a0, flip ? ce.y : ce.x);
        a1 = __fadd_rn(a1, flip ? ce.x : ce.y);
    }
    float2 e;
    e.x = __fdiv_rn(a0, (float)m);
    e.y = __fdiv_rn(a1, (float)m);
    e32[g] = e;
    store16(e16, g, e, fmt);
}

__global__ void k_add_dropped(unsigned long long *dropped, unsigned long long n)
{
    atomicAdd(dropped, n);
}

inline unsigned nblocks(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_accumulate(wfpg_svo *svo, const float *pos, const float *wo, const float *rgb,
                             int64_t n, hipStream_t s)
{
    if (n > 0 && svo->n[svo->depth] > 0) {
        hipLaunchKernelGGL(k_splat, dim3(nblocks(n, 256)), dim3(256), 0, s, svo->view(), pos, wo,
                           rgb, n, svo->d_sum, svo->d_cnt, svo->d_dropped);
    } else if (n > 0) {
        // an SVO without leaves places no splat: all are dropped
        hipLaunchKernelGGL(k_add_dropped, dim3(1), dim3(1), 0, s, svo->d_dropped,
                           (unsigned long long)n);
    }
    return hipGetLastError();
}

hipError_t launch_accumulate_paths(wfpg_svo *svo, const float *pos, const float *T, const float *eye,
                                   const int32_t *hit, const float *Le, int64_t P, int d, hipStream_t s)
{
    if (P > 0 && d > 0)
        hipLaunchKernelGGL(k_splat_paths, dim3(nblocks(P * d, 256)), dim3(256), 0, s, svo->view(), pos, T, eye, hit,
                           Le, P, d, svo->n[svo->depth] > 0, svo->d_sum, svo->d_cnt, svo->d_dropped);
    return hipGetLastError();
}

hipError_t launch_propagate(wfpg_svo *svo, hipStream_t s)
{
    const int D = svo->depth;
    if (svo->n[D] == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prop_leaf, dim3(nblocks(svo->n[D], 256)), dim3(256), 0, s, svo->d_sum,
                       svo->d_cnt, svo->n[D], svo->noff[D], svo->d_e32, svo->d_e16, svo->fmt);
    for (int l = D - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_prop_inner, dim3(nblocks(svo->n[l], 256)), dim3(256), 0, s,
                           svo->view(), svo->n[l], svo->noff[l], level_woff(l + 1), svo->d_e32,
                           svo->d_e16, svo->fmt);
    return hipGetLastError();
}

}  // namespace wfpg
