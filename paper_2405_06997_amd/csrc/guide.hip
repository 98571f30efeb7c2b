// Per-vertex guiding on gfx950 (Alg. 3: ConeTrace for every direction patch,
// GeneratePDF-CDF, sampling; Sec. 3.3-3.5).
//
// One wave64 owns one query vertex; lane l marches bins b = j*64 + l
// (j < N*N/64) with the exact SVO march of march_core.h. Rows of the N x N
// field are runs of N consecutive lanes, so the row CDFs are segmented wave
// scans and the marginal CDF is one more scan over N lanes; sampling is a
// ballot + find-first-set over the CDF.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "march_core.h"
#include "product_core.h"
#include "antialias_core.h"
#include "wfpg_internal.h"

namespace wfpg {
namespace {

using core::Hit;
using core::woff;

__device__ __forceinline__ float round16(float f, int fmt)
{
    if (fmt == WFPG_FP16) return __half2float(__float2half_rn(f));
    uint32_t u = __float_as_uint(f);
    return __uint_as_float(((u + 0x7fffu + ((u >> 16) & 1u)) >> 16) << 16);
}
__device__ __forceinline__ float unpack16(uint32_t v, int side, int fmt)
{
    uint32_t h = side ? (v >> 16) : (v & 0xffffu);
    if (fmt == WFPG_FP16) return __half2float(__ushort_as_half((unsigned short)h));
    return __uint_as_float(h << 16);
}

// Equal-area concentric octahedral map (Clarberg 2008), FP32.
__device__ __forceinline__ void oct_decode(float x, float y, float &dx, float &dy, float &dz)
{
    const float a = 2.f * x - 1.f, b = 2.f * y - 1.f;
    const float aa = fabsf(a), ab = fabsf(b);
    const float d = 1.f - (aa + ab);
    const float r = 1.f - fabsf(d);
    const float phi = r == 0.f ? 0.f : ((ab - aa) / r + 1.f) * 0.78539816339744831f;
    const float z = (d >= 0.f ? 1.f : -1.f) * (1.f - r * r);
    const float s = r * sqrtf(2.f - r * r);
    float sn, cs;
    sincosf(phi, &sn, &cs);
    dx = (a >= 0.f ? cs : -cs) * s;
    dy = (b >= 0.f ? sn : -sn) * s;
    dz = z;
}
__device__ __forceinline__ void oct_encode(float dx, float dy, float dz, float &x, float &y)
{
    const float r = sqrtf(fmaxf(1.f - fabsf(dz), 0.f));
    const float phi = atan2f(fabsf(dy), fabsf(dx));
    const float t = r * phi * 0.63661977236758134f;
    float aa = r - t, ab = t;
    if (dz < 0.f) {
        const float na = 1.f - ab, nb = 1.f - aa;
        aa = na;
        ab = nb;
    }
    x = ((dx >= 0.f ? aa : -aa) + 1.f) * 0.5f;
    y = ((dy >= 0.f ? ab : -ab) + 1.f) * 0.5f;
}

template <int N>
__device__ __forceinline__ float seg_scan(float v, int lane)
{
#pragma unroll
    for (int d = 1; d < N; d <<= 1) {
        const float t = __shfl_up(v, d, N);
        if ((lane & (N - 1)) >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// March steps each lane makes between the wave's bookkeeping points (with
// the prepass taking the short rays, the pool's rays are long: 8 steps
// measured faster than 4, 6, 10, 12 or 16).
constexpr int kMicro = 8;

constexpr uint32_t kMissRec = 0xffffffffu;
constexpr int kChunk = 4;   // vertices taken from a queue counter at a time (8 and 16 were slower)

// Per-vertex finalization (wave-wide): footprint level, node, side and value
// of every bin from the hit records in `rec`, then the row / marginal CDFs
// and the mode's output for vertex i. Returns the number of hit bins of this
// lane (for the count mode).
template <int N, int MODE, bool BLUR, bool R24>
__device__ __forceinline__ void finalize(const SvoView &sv, const GuideArgs &a, const float *ldir,
                                         uint32_t *rec, float *field, int64_t i, int64_t ps, int lane,
                                         int vis_lane)
{
    constexpr int NN = N * N;
    constexpr int BPL = NN / 64;
    constexpr int G = 64 / N;
    const int D = sv.depth;
    const int fmt = sv.fmt;
    float L[BPL];
    int hit_sum = 0;
#pragma unroll
    for (int j = 0; j < BPL; ++j) {
        const int b = j * 64 + lane;
        float val = fmt == WFPG_FP32 ? a.eps : round16(a.eps, fmt);
        bool hit;
        int lf = 0, k = 0, axis = 0;
        uint32_t node = 0, key = 0;
        const float dx = ldir[3 * b], dy = ldir[3 * b + 1], dz = ldir[3 * b + 2];
        if constexpr (MODE == MODE_DEBUG) {   // raw record: key | axis << 30, |B - O|
            const uint32_t r = rec[2 * b];
            hit = r != kMissRec;
            if (hit) {
                axis = (int)(r >> 30);
                key = r & 0x3fffffffu;
                const float dsel = axis == 0 ? dx : (axis == 1 ? dy : dz);
                k = core::footprint_levels(rec[2 * b + 1], fabsf(dsel), D, a.omega);
                lf = D - k;
                node = key >> (3 * k);
            }
        } else if constexpr (R24) {           // footprint node's index + 1 (0: miss), 16 + 8 bits
            const uint32_t r = (uint32_t)reinterpret_cast<const uint16_t *>(rec)[b] |
                               ((uint32_t)reinterpret_cast<const uint8_t *>(rec)[2 * NN + b] << 16);
            hit = r != 0u;
            node = r - 1u;
        } else {                              // footprint node: 1 << 3*lf | key (0: miss)
            const uint32_t r = rec[b];
            hit = r != 0u;
            if (hit) {
                lf = (31 - __builtin_clz(r)) / 3;
                node = r ^ (1u << (3 * lf));
            }
        }
        if (hit) {
            int64_t g;
            if constexpr (R24) {
                g = (int64_t)node;
            } else {
                const uint32_t wi = woff(lf) + (node >> 6);
                const uint64_t w = sv.bits[wi];
                const uint64_t msk = (node & 63) ? (w & ((1ull << (node & 63)) - 1)) : 0ull;
                g = (int64_t)sv.rank[wi] + __popcll(msk);
            }
            const float4 Nn = sv.nrm[g];
            const int side = core::dot3(Nn.x, Nn.y, Nn.z, dx, dy, dz) < 0.f ? 0 : 1;
            if (fmt == WFPG_FP32) {
                const float2 e = sv.e32[g];
                val = (side ? e.y : e.x) + a.eps;
            } else {
                val = round16(unpack16(sv.e16[g], side, fmt) + a.eps, fmt);
            }
            ++hit_sum;
            if constexpr (MODE == MODE_DEBUG) {
                int32_t *o = a.dbg_out + ((size_t)i * NN + b) * 8;
                o[0] = 1; o[1] = axis; o[2] = (int32_t)key; o[3] = (int32_t)rec[2 * b + 1];
                o[4] = k; o[5] = (int32_t)node; o[6] = (int32_t)(g - sv.noff[lf]); o[7] = side;
            }
        } else if constexpr (MODE == MODE_DEBUG) {
            int32_t *o = a.dbg_out + ((size_t)i * NN + b) * 8;
            o[0] = 0; o[1] = -1; o[2] = -1; o[3] = -1; o[4] = -1; o[5] = -1; o[6] = -1; o[7] = 0;
        }
        L[j] = val;
    }
    if constexpr (MODE == MODE_DEBUG) return;
    if constexpr (MODE == MODE_COUNT) {
        int vt = vis_lane;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            vt += __shfl_xor(vt, d);
            hit_sum += __shfl_xor(hit_sum, d);
        }
        if (lane == 0) {
            a.dbg_out[2 * i] = vt;
            a.dbg_out[2 * i + 1] = hit_sum;
        }
        return;
    }
    if constexpr (BLUR) {   // the slot's records are consumed: its LDS (or the field buffer) holds the field
        float *lv = R24 ? field : reinterpret_cast<float *>(rec);
#pragma unroll
        for (int j = 0; j < BPL; ++j) lv[j * 64 + lane] = L[j];
        wave_lds_fence();
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            const int b = j * 64 + lane;
            L[j] = aa::blur_at(N, b % N, b / N, [&](int k) { return lv[k]; });
        }
        wave_lds_fence();
    }
    if constexpr (MODE == MODE_PRODUCT || MODE == MODE_PEVAL) {
        // the slot's records are consumed: its LDS holds the field for the two levels
        constexpr int SB = N / prod::kCells;
        float *lv = R24 ? field : reinterpret_cast<float *>(rec);
#pragma unroll
        for (int j = 0; j < BPL; ++j) lv[j * 64 + lane] = L[j];
        wave_lds_fence();
        const int cv = lane >> 3, cu = lane & 7;
        float F = 0.f;
#pragma unroll
        for (int dv = 0; dv < SB; ++dv)
#pragma unroll
            for (int du = 0; du < SB; ++du) F += lv[(cv * SB + dv) * N + cu * SB + du];
        prod::Upper q;
        prod::upper_level(F, prod::table_entry(a.nrm_in, a.bsdf_in, i, ps, a.dirtab8, lane), lane, q);
        int c, fu, fv;
        float Lb;
        if constexpr (MODE == MODE_PRODUCT) {
            uint32_t w[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), a.bounce, 2u};
            core::philox(w, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
            c = prod::pick_cell(q, (float)(w[0] >> 8) * 5.9604644775390625e-8f,
                                (float)(w[1] >> 8) * 5.9604644775390625e-8f, lane);
            uint32_t r[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), a.bounce, 0u};
            core::philox(r, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
            const float u1 = (float)(r[0] >> 8) * 5.9604644775390625e-8f;
            const float u2 = (float)(r[1] >> 8) * 5.9604644775390625e-8f;
            const int V = c >> 3, U = c & 7;
            int dv = 0, du = 0;
            Lb = prod::pick_fine<SB>([&](int y, int x) { return lv[(V * SB + y) * N + U * SB + x]; }, u1, u2,
                                     lane, dv, du);
            fu = U * SB + du;
            fv = V * SB + dv;
            if (lane == 0) {
                const float inv = 1.f / (float)N;
                const float u3 = (float)(r[2] >> 8) * 5.9604644775390625e-8f;
                const float u4 = (float)(r[3] >> 8) * 5.9604644775390625e-8f;
                float ox, oy, oz;
                oct_decode((float)fu * inv + u3 * inv, (float)fv * inv + u4 * inv, ox, oy, oz);
                a.dir_out[i] = ox;
                a.dir_out[ps + i] = oy;
                a.dir_out[2 * ps + i] = oz;
            }
        } else {
            float ex, ey;
            oct_encode(a.dir_in[i], a.dir_in[ps + i], a.dir_in[2 * ps + i], ex, ey);
            fu = min(max((int)floorf(ex * (float)N), 0), N - 1);
            fv = min(max((int)floorf(ey * (float)N), 0), N - 1);
            c = (fv / SB) * prod::kCells + fu / SB;
            Lb = lv[fv * N + fu];
        }
        const float Pc = __shfl(q.P, c), Fc = __shfl(q.F, c);
        if (lane == 0) a.pdf_out[i] = (Pc / q.total) * (Lb / Fc) * a.pdf_scale;
        return;
    }
    // row CDFs (segmented inclusive scans), marginal CDF over the row sums
    float S[BPL];
#pragma unroll
    for (int j = 0; j < BPL; ++j) S[j] = seg_scan<N>(L[j], lane);
    float rs = 0.f;
#pragma unroll
    for (int j = 0; j < BPL; ++j) {
        const float t = __shfl(S[j], (lane % G) * N + N - 1);
        if (lane / G == j) rs = t;
    }
    if (lane >= N) rs = 0.f;
    const float M = seg_scan<N>(rs, lane);
    const float total = __shfl(M, N - 1);

    if constexpr (MODE == MODE_PDF) {
#pragma unroll
        for (int j = 0; j < BPL; ++j)
            a.pdf_out[(size_t)i * NN + j * 64 + lane] = (L[j] / total) * a.pdf_scale;
    } else if constexpr (MODE == MODE_SAMPLE) {
        uint32_t c[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), a.bounce, 0u};
        core::philox(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        const float u1 = (float)(c[0] >> 8) * 5.9604644775390625e-8f;
        const float u2 = (float)(c[1] >> 8) * 5.9604644775390625e-8f;
        const float u3 = (float)(c[2] >> 8) * 5.9604644775390625e-8f;
        const float u4 = (float)(c[3] >> 8) * 5.9604644775390625e-8f;
        const float tv = u1 * total;
        const uint64_t bv = __ballot(lane < N && tv < M);
        const int v = bv ? (__ffsll((unsigned long long)bv) - 1) : N - 1;
        const int jv = v / G, gv = v % G;
        float Sj = S[0], Lj = L[0];
#pragma unroll
        for (int j = 1; j < BPL; ++j)
            if (j == jv) { Sj = S[j]; Lj = L[j]; }
        const float rowsum = __shfl(Sj, gv * N + N - 1);
        const float tu = u2 * rowsum;
        const bool in_row = (lane / N) == gv;
        const uint64_t bu = __ballot(in_row && tu < Sj);
        const int u = bu ? (__ffsll((unsigned long long)bu) - 1 - gv * N) : N - 1;
        const float Lb = __shfl(Lj, gv * N + u);
        if (lane == 0) {
            const float inv = 1.f / (float)N;
            float ox, oy, oz;
            oct_decode((float)u * inv + u3 * inv, (float)v * inv + u4 * inv, ox, oy, oz);
            a.dir_out[i] = ox;
            a.dir_out[ps + i] = oy;
            a.dir_out[2 * ps + i] = oz;
            a.pdf_out[i] = (Lb / total) * a.pdf_scale;
        }
    } else if constexpr (MODE == MODE_EVAL) {
        float ex, ey;
        oct_encode(a.dir_in[i], a.dir_in[ps + i], a.dir_in[2 * ps + i], ex, ey);
        const int u = min(max((int)floorf(ex * (float)N), 0), N - 1);
        const int v = min(max((int)floorf(ey * (float)N), 0), N - 1);
        const int jv = v / G, gv = v % G;
        float Lj = L[0];
#pragma unroll
        for (int j = 1; j < BPL; ++j)
            if (j == jv) Lj = L[j];
        const float Lb = __shfl(Lj, gv * N + u);
        if (lane == 0) a.pdf_out[i] = (Lb / total) * a.pdf_scale;
    }
}

// Wave-uniform values, marked so for the compiler (kept in scalar registers).
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t shfl64(int64_t v, int src)
{
    const uint32_t lo = __shfl((uint32_t)(uint64_t)v, src);
    const uint32_t hi = __shfl((uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// LDS layout of a block: [N*N*3 bin directions]
// [N*N*3 quantized directions |q| | sign << 31][per wave: S vertex slots x
// N*N hit records][per wave: S node-test counters (count mode)][per wave: S
// unfinished-bin counts][per wave: S x N*N/64 pending-bin masks][per wave:
// 64-entry exchange][per wave: S slot vertices][per wave: the fed vertex's
// origin]. A hit record is the node the cone footprint selects, as
// 1 << 3*level | key (0 for a miss), or with R24 that node's index + 1 in a
// 16-bit and an 8-bit array; the debug mode keeps the raw traversal record
// {key | axis << 30, |B - O|} instead.
//
// A wave keeps up to S = guide_slots(N, R24) query vertices in flight. Idle
// lanes take the next unmarched bin of the vertex being fed; when it has no
// bins left a free slot is opened for the next vertex of the queue (taken
// kChunk at a time from the counter of one of kQueueRanges contiguous ranges
// of the queue, the workgroup's XCD's first), so lanes rarely wait for another
// vertex's longest rays. A slot whose bins are all finished is finalized by
// the whole wave (values, CDF, sample) and freed. Slot bookkeeping is
// wave-uniform; the per-slot arrays in registers are only ever indexed by
// unrolled constants.
// BLUR: the field is blurred before its CDF (a variant of its own: the blur's
// registers would lower the occupancy of the unblurred kernel).
// At N = 16 the register allocation is held to six waves per SIMD (80 VGPRs;
// a few bytes of spills): left free it takes one register more and five.
template <int N, int MODE, bool BLUR, bool R24>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(N == 16 ? 6 : 1)))
k_guide(SvoView sv, GuideArgs a)
{
    constexpr int NN = N * N;
    constexpr int BPL = NN / 64;
    constexpr bool FIELD = guide_field_buffer(MODE, BLUR, R24);
    constexpr int S = guide_slots(N, R24, FIELD);
    static_assert(!R24 || (N == 16 && MODE != MODE_DEBUG && MODE != MODE_COUNT),
                  "3-byte records: N = 16, not the debug or counting modes");
    extern __shared__ uint64_t smem[];
    if (a.gate && *a.gate == 0) return;   // uniform: every thread reads the same flag
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int D = sv.depth;
    float *ldir = reinterpret_cast<float *>(smem);
    uint32_t *lq = reinterpret_cast<uint32_t *>(ldir + 3 * NN);
    constexpr int SW = guide_slot_words(N, MODE, R24);   // 32-bit words of one slot's records
    const int nw = blockDim.x / 64;
    uint32_t *recs = lq + 3 * NN + (size_t)wave * S * SW;
    uint32_t *svis = lq + 3 * NN + (size_t)nw * S * SW + (size_t)wave * S;
    // per wave: the bins each slot has not finished yet (-1: the slot is free)
    int *srem = reinterpret_cast<int *>(lq + 3 * NN + (size_t)nw * S * SW + (size_t)nw * S) + (size_t)wave * S;
    // per wave: the bins each slot still has to march, one 64-bit mask per
    // 64 bins (bit l of mask j: bin 64 j + l), and a 64-entry exchange buffer
    // through which the hand-out passes bins to idle lanes
    uint64_t *pmask = reinterpret_cast<uint64_t *>(lq + 3 * NN + (size_t)nw * S * (SW + 2)) +
                      (size_t)wave * S * BPL;
    uint64_t *pm_end = reinterpret_cast<uint64_t *>(lq + 3 * NN + (size_t)nw * S * (SW + 2)) + (size_t)nw * S * BPL;
    uint16_t *xch = reinterpret_cast<uint16_t *>(pm_end) + (size_t)wave * 64;
    // per wave: the vertex of each slot and the fed vertex's origin (x, y, z,
    // leaf key | occupied << 31)
    int64_t *svert = reinterpret_cast<int64_t *>(reinterpret_cast<uint16_t *>(pm_end) + (size_t)nw * 64) +
                     (size_t)wave * S;
    uint32_t *sfeed_all = reinterpret_cast<uint32_t *>(reinterpret_cast<int64_t *>(reinterpret_cast<uint16_t *>(pm_end) +
                                                                                  (size_t)nw * 64) + (size_t)nw * S);
    uint32_t *sfeed = sfeed_all + (size_t)wave * 4;
    // per wave (blur and product modes with 3-byte records): the field buffer
    float *sfield = FIELD ? reinterpret_cast<float *>(sfeed_all + (size_t)nw * 4) + (size_t)wave * NN : nullptr;
    // The per-vertex finalization reads its arguments from an LDS copy: held
    // in scalar registers across the march loop they overflowed the scalar
    // file and were spilled into vector lanes (two lane moves per use); read
    // from LDS at each finalization they cost a few loads per vertex.
    __shared__ SvoView s_sv;
    __shared__ GuideArgs s_a;
    static_assert(sizeof(SvoView) + sizeof(GuideArgs) + 64 <= kGuideStaticLds, "static LDS over its reserve");
    if (threadIdx.x == 0) {
        s_sv = sv;
        s_a = a;
    }
    for (int t = threadIdx.x; t < NN; t += blockDim.x) {
        float d[3];
        if (a.jitter) {
            aa::jitter_dir(N, t, a.jitter_key, d[0], d[1], d[2]);
        } else {
            d[0] = a.dirtab[3 * t];
            d[1] = a.dirtab[3 * t + 1];
            d[2] = a.dirtab[3 * t + 2];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ldir[3 * t + k] = d[k];
            const int q = core::quantize_dir(d[k]);
            lq[3 * t + k] = (uint32_t)(q < 0 ? -q : q) | (q < 0 ? 0x80000000u : 0u);
        }
    }
    __syncthreads();

    const int64_t n = a.n_dev ? *a.n_dev : a.n;
    const int64_t ps = a.stride ? a.stride : n;   // SoA plane stride
    // every occupancy test is a plain global load: the top levels stay hot in
    // the L1/L2 caches (staging them in LDS made the loads flat loads through
    // a pointer select, which measured slower)
    const uint32_t *gbits = reinterpret_cast<const uint32_t *>(sv.bits);   // 32-bit words
    auto bits = [gbits](int, uint32_t wi) -> uint32_t { return gbits[wi]; };
    const uint64_t *gbits64 = sv.bits;
    auto bits64 = [gbits64](uint32_t wi) -> uint64_t { return gbits64[wi]; };

    // wave-uniform stream and slot state
    int64_t chunk_next = 0;
    int chunk_left = 0;
    bool exhausted = false;
    // the queue range taken from (this workgroup's XCD's first) and how many
    // ranges were found exhausted
    int xr = (int)(blockIdx.x % (unsigned)kQueueRanges), xdone = 0;
    // the bins each slot has not finished, the slots' vertices and the fed
    // vertex's origin live in LDS (scalar registers are the kernel's scarcest
    // resource); a finishing lane takes its bin off its slot's count
    if (lane < S) srem[lane] = -1;
    wave_lds_fence();
    int feed = -1, nxt = BPL;            // slot being handed out and its mask of bins being handed out
    // per-lane march state
    int lslot = 0, lbin = -1, vis = 0, iters = 0;
    core::MicroState st;

    // the record of a finished march (res: STEP_HIT or STEP_MISS) of bin b
    // of slot k whose vertex is v, with its node-test count pv
    auto finish_hit = [&](int res, const Hit &h, int k, int b, int64_t v, int pv) {
        uint32_t *rec = recs + k * SW;
        if constexpr (MODE == MODE_DEBUG) {
            rec[2 * b] = res == core::STEP_HIT ? (h.key | ((uint32_t)h.axis << 30)) : kMissRec;
            rec[2 * b + 1] = h.delta;
            if (a.dbg_visits) a.dbg_visits[(size_t)v * NN + b] = pv;
        } else {
            // cone footprint (Eq. 7) decided here: the record is the node it selects
            uint32_t rv = 0u;
            if (res == core::STEP_HIT) {
                const float dsel = ldir[3 * b + h.axis];
                const int kk = core::footprint_levels(h.delta, fabsf(dsel), D, a.omega);
                rv = (1u << (3 * (D - kk))) | (h.key >> (3 * kk));
                if constexpr (R24) {   // the node's index + 1
                    const uint32_t node = h.key >> (3 * kk);
                    const uint32_t wi = woff(D - kk) + (node >> 6);
                    const uint64_t w = gbits64[wi];
                    const uint64_t msk = (node & 63) ? (w & ((1ull << (node & 63)) - 1)) : 0ull;
                    rv = __builtin_launder(&s_sv)->rank[wi] + (uint32_t)__popcll(msk) + 1u;
                }
            }
            if constexpr (R24) {
                reinterpret_cast<uint16_t *>(rec)[b] = (uint16_t)rv;
                reinterpret_cast<uint8_t *>(rec)[2 * NN + b] = (uint8_t)(rv >> 16);
            } else {
                rec[b] = rv;
            }
        }
        if constexpr (MODE == MODE_COUNT) atomicAdd(&svis[k], (uint32_t)pv);
    };
    auto finish = [&](const core::MicroState &ms, int res, int k, int b, int64_t v, int pv) {
        finish_hit(res, res == core::STEP_HIT ? core::hit_of(ms, D) : Hit{-1, 0u, 0u}, k, b, v, pv);
    };

    while (true) {
        // finalize every slot whose bins are all finished
        while (true) {
            int64_t vd = 0;
            const uint64_t zr = __ballot(lane < S && srem[lane] == 0);
            if (zr == 0ull) break;
            const int done = uni((int)__builtin_ctzll(zr));
            vd = uni(svert[done]);
            const int vl = MODE == MODE_COUNT && lane == 0 ? (int)svis[done] : 0;
            finalize<N, MODE, BLUR, R24>(*__builtin_launder(&s_sv), *__builtin_launder(&s_a), ldir, recs + done * SW, sfield,
                                    vd, ps, lane, vl);
            wave_lds_fence();
            if (lane == 0) srem[done] = -1;
            wave_lds_fence();
        }
        // hand out bins to idle lanes
        uint64_t idle = __ballot(lbin < 0);
        while (idle) {
            if (feed < 0 || nxt >= BPL) {
                const uint64_t fr = __ballot(lane < S && srem[lane] < 0);
                if (fr == 0ull || exhausted) break;
                const int f = uni((int)__builtin_ctzll(fr));
                if (chunk_left == 0) {
                    int64_t b = 0, hi = 0;
                    for (;;) {   // the next chunk of range xr, else of the next range
                        const int64_t lo = n * xr / kQueueRanges;
                        hi = n * (xr + 1) / kQueueRanges;
                        if (lane == 0)
                            b = (int64_t)atomicAdd(__builtin_launder(&s_a)->queue_ctr + xr * kQueueStride, (unsigned long long)kChunk);
                        b = uni(shfl64(b, 0)) + lo;
                        if (b < hi || ++xdone == kQueueRanges) break;
                        xr = (xr + 1) % kQueueRanges;
                    }
                    if (b >= hi) { exhausted = true; break; }
                    chunk_next = b;
                    chunk_left = uni((int)min((int64_t)kChunk, hi - b));
                }
                const int64_t vi = chunk_next++;
                --chunk_left;
                uint32_t O[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) O[k] = core::quantize_pos(__builtin_launder(&s_a)->pos[k * ps + vi]);
                const uint32_t okey = core::morton3(O[0] >> (WFPG_FINE - D), O[1] >> (WFPG_FINE - D),
                                                    O[2] >> (WFPG_FINE - D));
                const bool oc = core::occupied(bits, D, okey);
                if (lane == 0) {
                    sfeed[0] = O[0];
                    sfeed[1] = O[1];
                    sfeed[2] = O[2];
                    sfeed[3] = okey | (oc ? 0x80000000u : 0u);
                    svert[f] = vi;
                }
                if constexpr (MODE == MODE_COUNT) {
                    if (lane == 0) svis[f] = 0u;
                    wave_lds_fence();
                }
                // First step of every bin of the new vertex by the whole wave,
                // whatever ray a lane is marching (about four rays in five end
                // there: they enter an occupied face neighbour of the origin's
                // leaf, or leave the cube); the others are marked for the
                // hand-out. Without node-test counts, a vertex whose leaf is
                // occupied takes it from the leaf's six face neighbours (lane
                // 2j + up reads the one along axis j: its key, whether it lies
                // in the cube, whether it is occupied), read once for all its
                // bins, and the exit crossing of each bin, with no march state;
                // with an empty leaf every bin starts in the hand-out.
                constexpr bool kNbrStep = MODE != MODE_DEBUG && MODE != MODE_COUNT;
                int npend = 0;
                if constexpr (kNbrStep) {
                    const bool nbr_step = uni((int)oc) != 0;
                    uint32_t nkey = 0u;
                    bool nin = false, non = false;
                    if (lane < 6) {
                        const int ax = lane >> 1;
                        uint32_t c0 = O[0] >> (WFPG_FINE - D), c1 = O[1] >> (WFPG_FINE - D),
                                 c2 = O[2] >> (WFPG_FINE - D);
                        const uint32_t cj = ax == 0 ? c0 : (ax == 1 ? c1 : c2);
                        const uint32_t nj = (lane & 1) ? cj + 1u : cj - 1u;   // wraps below 0
                        c0 = ax == 0 ? nj : c0;
                        c1 = ax == 1 ? nj : c1;
                        c2 = ax == 2 ? nj : c2;
                        nin = nj < (1u << D);
                        nkey = core::morton3(c0, c1, c2);
                        non = nin && core::occupied(bits, D, nkey);
                    }
                    const uint32_t inm = (uint32_t)__ballot(nin), onm = (uint32_t)__ballot(non);
                    core::FirstLeaf fl = core::first_leaf(O, D);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {   // the same on every lane
                        fl.up[k] = uni(fl.up[k]);
                        fl.dn[k] = uni(fl.dn[k]);
                    }
#pragma unroll 1
                    for (int j = 0; j < BPL; ++j) {
                        const int b = j * 64 + lane;
                        const uint32_t w0 = lq[3 * b], w1 = lq[3 * b + 1], w2 = lq[3 * b + 2];
                        const uint32_t a0 = w0 & 0x7fffffffu, a1 = w1 & 0x7fffffffu, a2 = w2 & 0x7fffffffu;
                        int e;
                        bool up;
                        uint32_t delta;
                        core::first_exit(fl, a0, a1, a2, a0 && (w0 >> 31), a1 && (w1 >> 31), a2 && (w2 >> 31), e, up,
                                         delta);
                        const int idx = 2 * e + (up ? 1 : 0);
                        const uint32_t hkey = (uint32_t)__shfl((int)nkey, idx);
                        const int r1 = !nbr_step ? core::STEP_CONTINUE
                                                 : (((inm >> idx) & 1u) == 0u ? core::STEP_MISS
                                                                              : (((onm >> idx) & 1u) != 0u
                                                                                     ? core::STEP_HIT
                                                                                     : core::STEP_CONTINUE));
                        if (r1 != core::STEP_CONTINUE) finish_hit(r1, Hit{e, hkey, delta}, f, b, vi, 0);
                        const uint64_t pm = __ballot(r1 == core::STEP_CONTINUE);
                        if (lane == 0) pmask[f * BPL + j] = pm;
                        npend += (int)__popcll(pm);
                    }
                } else {
#pragma unroll 1
                    for (int j = 0; j < BPL; ++j) {
                        const int b = j * 64 + lane;
                        const uint32_t w0 = lq[3 * b], w1 = lq[3 * b + 1], w2 = lq[3 * b + 2];
                        const uint32_t a0 = w0 & 0x7fffffffu, a1 = w1 & 0x7fffffffu, a2 = w2 & 0x7fffffffu;
                        core::MicroState ms;
                        int pv = 0;
                        core::micro_begin(ms, O, okey, oc, a0, a1, a2, a0 ? ((w0 >> 31) ? -1 : 1) : 0,
                                          a1 ? ((w1 >> 31) ? -1 : 1) : 0, a2 ? ((w2 >> 31) ? -1 : 1) : 0, D, 5, pv);
                        const int r1 = core::micro_step(ms, D, bits64, 5, pv);
                        if (r1 != core::STEP_CONTINUE) finish(ms, r1, f, b, vi, pv);
                        const uint64_t pm = __ballot(r1 == core::STEP_CONTINUE);
                        if (lane == 0) pmask[f * BPL + j] = pm;
                        npend += (int)__popcll(pm);
                    }
                }
                if (lane == 0) srem[f] = npend;
                wave_lds_fence();
                feed = f;
                nxt = 0;
            }
            // the next bins of the feed slot's current mask go to the idle lanes
            // in order, through the exchange buffer
            const uint64_t avail = (uint64_t)uni((int64_t)pmask[feed * BPL + nxt]);
            if (avail == 0ull) {
                nxt = uni(nxt + 1);
                continue;
            }
            const int nidle = (int)__popcll(idle), left = (int)__popcll(avail);
            const int take = nidle < left ? nidle : left;   // (integer min: the mixed-type min was FP64)
            const int kr = lanes_below(avail);
            const bool give = ((avail >> lane) & 1ull) && kr < take;
            if (give) xch[kr] = (uint16_t)(nxt * 64 + lane);
            const uint64_t given = __ballot(give);
            wave_lds_fence();
            const int r = lanes_below(idle);
            const bool mine = ((idle >> lane) & 1ull) && r < take;
            if (mine) {
                lslot = feed;
                lbin = xch[r];
                const uint32_t O[3] = {sfeed[0], sfeed[1], sfeed[2]};
                const uint32_t Fk = sfeed[3];
                const uint32_t w0 = lq[3 * lbin], w1 = lq[3 * lbin + 1], w2 = lq[3 * lbin + 2];
                const uint32_t a0 = w0 & 0x7fffffffu, a1 = w1 & 0x7fffffffu, a2 = w2 & 0x7fffffffu;
                vis = 0;
                iters = 0;
                core::micro_begin(st, O, Fk & 0x7fffffffu, (Fk >> 31) != 0u, a0, a1, a2, a0 ? ((w0 >> 31) ? -1 : 1) : 0,
                                  a1 ? ((w1 >> 31) ? -1 : 1) : 0, a2 ? ((w2 >> 31) ? -1 : 1) : 0, D, 5, vis);
            }
            idle &= ~__ballot(mine);
            wave_lds_fence();   // the exchange buffer is read before it is written again
            if (lane == 0) pmask[feed * BPL + nxt] = avail & ~given;
            wave_lds_fence();
        }
        if (__ballot(lbin >= 0) == 0ull) {
            const int rk = lane < S ? srem[lane] : -1;
            const bool any = __ballot(rk >= 0) != 0ull, ready = __ballot(rk == 0) != 0ull;
            if (!any) break;
            if (!ready) {
                atomicOr(__builtin_launder(&s_a)->err, 2);   // no progress possible (never expected)
                break;
            }
            continue;
        }
        int res = core::STEP_CONTINUE;
        if (lbin >= 0) {
            // unrolled: the steps run as one straight sequence, a lane that finished
            // masked out of the rest
#pragma unroll
            for (int m = 0; m < kMicro; ++m) {
                res = core::micro_step(st, D, bits64, 5, vis);
                if (res != core::STEP_CONTINUE) break;
            }
            if (res == core::STEP_CONTINUE && (iters += kMicro) >= core::kMaxTests) {
                atomicOr(__builtin_launder(&s_a)->err, 1);
                res = core::STEP_MISS;
            }
        }
        const bool fin = lbin >= 0 && res != core::STEP_CONTINUE;
        if (fin) {
            const int64_t vl = MODE == MODE_DEBUG ? svert[lslot] : 0;
            finish(st, res, lslot, lbin, vl, vis);
            lbin = -1;
        }
        if (fin) atomicSub(&srem[lslot], 1);
        wave_lds_fence();
    }
}

__global__ void k_reset_counter(unsigned long long *ctr)
{
    if (threadIdx.x < kQueueRanges) ctr[threadIdx.x * kQueueStride] = 0ull;
}

template <int N>
hipError_t launch_n(const wfpg_svo *svo, int mode, const GuideArgs &a0, const TileConfig &tc,
                    hipStream_t s)
{
    GuideArgs a = a0;
    if (!a.queue_ctr)
        a.queue_ctr = svo->d_ctr + (size_t)kQueueRanges * kQueueStride * (svo->ctr_next.fetch_add(1u) % (unsigned)kCounterPool);
    const bool blur = a.blur != 0 && mode != MODE_DEBUG && mode != MODE_COUNT;
    const bool r24 = guide_use_r24(N, mode, svo->total_nodes);
    TileConfig t = tc;   // debug records are twice as large: shrink the workgroup if needed
    while (t.waves_per_block > 1 && guide_lds_bytes(N, t, mode, r24, blur) > guide_max_lds()) --t.waves_per_block;
    const int W = t.waves_per_block;
    const int64_t want = a.n_dev ? INT64_MAX : ((a.n + kChunk - 1) / kChunk + W - 1) / W;
    const int64_t cap = (int64_t)device_cu_count() * t.blocks_per_cu;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, cap));
    const size_t lds = guide_lds_bytes(N, t, mode, r24, blur);
    if (lds > guide_max_lds()) return hipErrorInvalidValue;
    const dim3 blk(64 * W);
    const wfpg::SvoView v = svo->view();
    const void *fn = nullptr;
#define WFPG_PICK(M)                                                                      \
    fn = blur ? (const void *)&k_guide<N, M, true, false> : (const void *)&k_guide<N, M, false, false>
#define WFPG_PICK24(M)                                                                    \
    if constexpr (N == 16) {                                                              \
        if (r24)                                                                          \
            fn = blur ? (const void *)&k_guide<N, M, true, true> : (const void *)&k_guide<N, M, false, true>; \
    }
    switch (mode) {
    case MODE_SAMPLE: WFPG_PICK(MODE_SAMPLE); WFPG_PICK24(MODE_SAMPLE); break;
    case MODE_PDF: WFPG_PICK(MODE_PDF); WFPG_PICK24(MODE_PDF); break;
    case MODE_EVAL: WFPG_PICK(MODE_EVAL); WFPG_PICK24(MODE_EVAL); break;
    case MODE_PRODUCT: WFPG_PICK(MODE_PRODUCT); WFPG_PICK24(MODE_PRODUCT); break;
    case MODE_PEVAL: WFPG_PICK(MODE_PEVAL); WFPG_PICK24(MODE_PEVAL); break;
    case MODE_COUNT: fn = (const void *)&k_guide<N, MODE_COUNT, false, false>; break;
    default: fn = (const void *)&k_guide<N, MODE_DEBUG, false, false>; break;
    }
#undef WFPG_PICK
#undef WFPG_PICK24
    if (lds > 64 * 1024) {   // opt in to the device's whole LDS once per kernel
        static std::atomic<bool> opted[4 * MODE_COUNT_OF_MODES];
        const int m = ((mode < 0 || mode >= MODE_COUNT_OF_MODES ? MODE_DEBUG : mode) * 2 + (blur ? 1 : 0)) * 2 +
                      (r24 ? 1 : 0);
        if (!opted[m].load()) {
            const hipError_t e =
                hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)guide_max_lds());
            if (e != hipSuccess) return e;
            opted[m].store(true);
        }
    }
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, a.queue_ctr);
    void *args[] = {(void *)&v, (void *)&a};
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), blk, args, lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_guide(const wfpg_svo *svo, int N, int mode, const GuideArgs &a,
                        const TileConfig &tc, hipStream_t s)
{
    switch (N) {
    case 8: return launch_n<8>(svo, mode, a, tc, s);
    case 16: return launch_n<16>(svo, mode, a, tc, s);
    case 32: return launch_n<32>(svo, mode, a, tc, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace wfpg
