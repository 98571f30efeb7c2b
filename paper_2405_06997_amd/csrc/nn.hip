// Learned stand-in for the march (not part of the paper, which surveys neural
// guiding only as related work, Sec. 2.1): a multiresolution hash encoding
// of the position (Mueller et al. 2022) plus the normal feeds a ReLU MLP
// 35 -> 64 -> 64 -> 64 -> 64 -> 256 whose softmax is a distribution over the
// 16 x 16 direction bins. Trained on the GPU by cross-entropy against the
// march's PDFs; the march judges it on probe vertices and replaces it when
// the probes' mean KL exceeds a bound.
//
// Matrix products run on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16:
// BF16 operands, FP32 accumulation) through one generic tiled GEMM with
// fused epilogues. Activation rows are padded to a multiple of 64 (pad rows
// are zero on input and never read back), so tiles need no bounds checks.
// BF16 rounding points: hash-table entries, encoded inputs, weights, hidden
// activations, the logit gradient and the hidden pre-activation gradients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "march_core.h"
#include "wfpg_internal.h"

namespace wfpg {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);   // RNE (finite inputs)
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ GEMM ---
// C[M x N] = A[M x K] * B[K x N]; A stored row-major [M][K] (AT = false) or
// as [K][M] (AT = true); B stored row-major [K][N] (BT = false) or as [N][K]
// (BT = true). M, N multiples of 64, K a multiple of 32 (split-K chunks of
// k_chunk rows, a multiple of 32).
enum Epi {
    EPI_F32 = 0,          // C = acc + bias (bias may be null), FP32
    EPI_BIAS_RELU = 1,    // Cb = bf16(relu(acc + bias))
    EPI_MASK = 2,         // v = mask > 0 ? acc : 0; Cb = bf16(v); colsum += v
    EPI_ATOMIC = 3,       // C += acc (atomic, split-K)
};

struct GemmArgs {
    const uint16_t *A;
    int64_t lda;
    const uint16_t *B;
    int64_t ldb;
    int M, N, K, k_chunk;
    float *C;
    uint16_t *Cb;
    int64_t ldc;
    const float *bias;
    const uint16_t *mask;   // EPI_MASK: bf16 activations, same layout as C
    float *colsum;          // EPI_MASK: column sums (bias gradient), atomic
};

constexpr int TS = 64, TK = 32, LDK = TK + 8;   // LDS rows padded against bank conflicts

template <bool AT, bool BT, int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[TS * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TS * LDK];
    __shared__ float csum[TS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * TS, n0 = blockIdx.y * TS;
    const int kb = blockIdx.z * g.k_chunk;
    const int ke = min(g.K, kb + g.k_chunk);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (EPI == EPI_MASK && tid < TS) csum[tid] = 0.f;
    for (int k0 = kb; k0 < ke; k0 += TK) {
        if (!AT) {   // 64 rows x 32 k: thread = (row tid/4, 8 k at (tid%4)*8)
            const int m = tid >> 2, k = (tid & 3) * 8;
            const uint4 v = *reinterpret_cast<const uint4 *>(g.A + (int64_t)(m0 + m) * g.lda + k0 + k);
            *reinterpret_cast<uint4 *>(&As[m * LDK + k]) = v;
        } else {     // memory [K][M]: thread = (k tid/8, 8 m at (tid%8)*8)
            const int k = tid >> 3, m = (tid & 7) * 8;
            const uint4 v = *reinterpret_cast<const uint4 *>(g.A + (int64_t)(k0 + k) * g.lda + m0 + m);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
            for (int t = 0; t < 8; ++t) As[(m + t) * LDK + k] = e[t];
        }
        if (BT) {    // memory [N][K]
            const int n = tid >> 2, k = (tid & 3) * 8;
            const uint4 v = *reinterpret_cast<const uint4 *>(g.B + (int64_t)(n0 + n) * g.ldb + k0 + k);
            *reinterpret_cast<uint4 *>(&Bs[n * LDK + k]) = v;
        } else {     // memory [K][N]
            const int k = tid >> 3, n = (tid & 7) * 8;
            const uint4 v = *reinterpret_cast<const uint4 *>(g.B + (int64_t)(k0 + k) * g.ldb + n0 + n);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
            for (int t = 0; t < 8; ++t) Bs[(n + t) * LDK + k] = e[t];
        }
        __syncthreads();
        bf16x8 af[2], bfr[2];
        for (int a = 0; a < 2; ++a)
            af[a] = *reinterpret_cast<const bf16x8 *>(&As[(wm + 16 * a + (lane & 15)) * LDK + 8 * (lane >> 4)]);
        for (int b = 0; b < 2; ++b)
            bfr[b] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn + 16 * b + (lane & 15)) * LDK + 8 * (lane >> 4)]);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // epilogue: lane holds D[4*(lane/16) + r][lane % 16] of each 16 x 16 tile
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int n = n0 + wn + 16 * b + (lane & 15);
            float colpart = 0.f;
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * a + 4 * (lane >> 4) + r;
                const int64_t o = (int64_t)m * g.ldc + n;
                float v = acc[a][b][r];
                if (EPI == EPI_F32) {
                    g.C[o] = g.bias ? v + g.bias[n] : v;
                } else if (EPI == EPI_BIAS_RELU) {
                    v = v + g.bias[n];
                    g.Cb[o] = f2bf(v > 0.f ? v : 0.f);
                } else if (EPI == EPI_MASK) {
                    v = bf2f(g.mask[o]) > 0.f ? v : 0.f;
                    g.Cb[o] = f2bf(v);
                    colpart += v;
                } else {
                    unsafeAtomicAdd(&g.C[o], v);
                }
            }
            if (EPI == EPI_MASK) atomicAdd(&csum[n - n0], colpart);
        }
    if (EPI == EPI_MASK) {
        __syncthreads();
        if (tid < TS) unsafeAtomicAdd(&g.colsum[n0 + tid], csum[tid]);
    }
}

// MLP parameters: FP32 master -> BF16 copy in the padded GEMM layout (W0 is
// stored [64][64] with zero columns 35..63).
struct MlpLayout {
    int64_t woff[5], boff[5];   // offsets in the FP32 parameter vector
    int fin[5], fout[5];
    int64_t bw[5];              // offsets of the BF16 weight copies
};

// --------------------------------------------------------- hash encoding ---
struct Grid {
    int32_t res[16];
    int log2T;
};

__device__ __forceinline__ uint32_t corner_index(uint32_t x, uint32_t y, uint32_t z, int32_t R, int log2T)
{
    const uint64_t side = (uint64_t)R + 1;
    if (side * side * side <= (1ull << log2T)) return (uint32_t)(x + side * (y + side * z));
    return (x * 1u ^ y * 2654435761u ^ z * 805459861u) & ((1u << log2T) - 1u);
}

// Cell and FP32 fractions of position p at resolution R.
__device__ __forceinline__ void cell_of(const float p[3], int32_t R, uint32_t c[3], float fr[3])
{
    for (int k = 0; k < 3; ++k) {
        const float x = p[k] * (float)R;
        float fl = floorf(x);
        fl = fminf(fmaxf(fl, 0.f), (float)(R - 1));
        c[k] = (uint32_t)fl;
        fr[k] = x - fl;
    }
}

// The two BF16 features of level l at position p (low half: feature 0):
// trilinear interpolation, FP32 weights (wx * wy) * wz, corners x fastest,
// FP32 sums in that order, rounded once to BF16.
__device__ __forceinline__ uint32_t encode_level(const Grid &gr, const uint16_t *__restrict__ table, const float p[3],
                                                 int l)
{
    uint32_t c[3];
    float fr[3];
    cell_of(p, gr.res[l], c, fr);
    const uint64_t T = 1ull << gr.log2T;
    float a0 = 0.f, a1 = 0.f;
    for (int q = 0; q < 8; ++q) {
        const float wx = (q & 1) ? fr[0] : 1.f - fr[0];
        const float wy = (q & 2) ? fr[1] : 1.f - fr[1];
        const float wz = (q & 4) ? fr[2] : 1.f - fr[2];
        const float w = (wx * wy) * wz;
        const uint32_t id = corner_index(c[0] + (q & 1), c[1] + ((q >> 1) & 1), c[2] + ((q >> 2) & 1),
                                         gr.res[l], gr.log2T);
        const uint32_t pr = *reinterpret_cast<const uint32_t *>(table + ((uint64_t)l * T + id) * 2);
        a0 = a0 + w * bf2f((uint16_t)(pr & 0xffffu));
        a1 = a1 + w * bf2f((uint16_t)(pr >> 16));
    }
    return (uint32_t)f2bf(a0) | ((uint32_t)f2bf(a1) << 16);
}

// X[v][0..63] = bf16(features of 16 levels x 2, then the normal, then zeros).
// One thread per (vertex, level); rows >= n (padding) are zeroed.
__global__ void k_encode(Grid gr, const uint16_t *__restrict__ table, const float *__restrict__ pos,
                         const float *__restrict__ nrm, int64_t n, int64_t stride, int64_t rows,
                         uint16_t *X)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t v = t >> 4;
    const int l = (int)(t & 15);
    if (v >= rows) return;
    uint16_t *x = X + v * 64;
    if (v >= n) {
        for (int k = 0; k < 4; ++k) x[4 * l + k] = 0;
        return;
    }
    const float p[3] = {pos[v], pos[stride + v], pos[2 * stride + v]};
    const uint32_t pair = encode_level(gr, table, p, l);
    x[2 * l] = (uint16_t)(pair & 0xffffu);
    x[2 * l + 1] = (uint16_t)(pair >> 16);
    if (l == 0) {
        x[32] = f2bf(nrm ? nrm[v] : 0.f);
        x[33] = f2bf(nrm ? nrm[stride + v] : 0.f);
        x[34] = f2bf(nrm ? nrm[2 * stride + v] : 0.f);
    }
    if (l >= 3) {   // zero the padding columns 35..63 (29 columns over 13 threads)
        const int c0 = 35 + (l - 3) * 3;
        for (int k = c0; k < c0 + 3 && k < 64; ++k) x[k] = 0;
    } else if (l == 2) {
        x[62] = 0; x[63] = 0;
    }
}

// Table gradient: grad[l][corner][f] += w * dX[v][2l + f] (FP32 atomics).
__global__ void k_hash_scatter(Grid gr, const float *__restrict__ pos, int64_t n, int64_t stride,
                               const float *__restrict__ dX, float *gtable)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t v = t >> 4;
    const int l = (int)(t & 15);
    if (v >= n) return;
    const float p[3] = {pos[v], pos[stride + v], pos[2 * stride + v]};
    uint32_t c[3];
    float fr[3];
    cell_of(p, gr.res[l], c, fr);
    const uint64_t T = 1ull << gr.log2T;
    const float g0 = dX[v * 64 + 2 * l], g1 = dX[v * 64 + 2 * l + 1];
    for (int q = 0; q < 8; ++q) {
        const float wx = (q & 1) ? fr[0] : 1.f - fr[0];
        const float wy = (q & 2) ? fr[1] : 1.f - fr[1];
        const float wz = (q & 4) ? fr[2] : 1.f - fr[2];
        const float w = (wx * wy) * wz;
        const uint32_t id = corner_index(c[0] + (q & 1), c[1] + ((q >> 1) & 1), c[2] + ((q >> 2) & 1),
                                         gr.res[l], gr.log2T);
        float *gp = gtable + ((uint64_t)l * T + id) * 2;
        unsafeAtomicAdd(gp, w * g0);
        unsafeAtomicAdd(gp + 1, w * g1);
    }
}

// ------------------------------------------------- softmax, loss, judge ---
__device__ __forceinline__ float wave_sum(float v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d));
    return v;
}

// One wave per row (grid-stride over the padded batch): p = softmax(z);
// target t = march pdf renormalized to sum 1; dZ = (p - t) * inv_b (BF16 for
// the products; rows >= n get 0); loss = -sum t ln p * inv_b. The output-bias
// gradient (FP32, unrounded) and the loss are summed per lane across the
// wave's rows, then across the block in LDS, and added with one atomic per
// bin and block.
__global__ void __launch_bounds__(256) k_softmax_xent(const float *__restrict__ Z, const float *__restrict__ tpdf,
                                                      int64_t n, int64_t rows, float inv_b, uint16_t *dZ,
                                                      float *db, float *loss)
{
    __shared__ float sdb[4][256];
    __shared__ float sloss[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    float lacc = 0.f;
    const int64_t wstride = (int64_t)gridDim.x * 4;
    for (int64_t v = blockIdx.x * 4 + wave; v < rows; v += wstride) {
        if (v >= n) {
            for (int j = 0; j < 4; ++j) dZ[v * 256 + j * 64 + lane] = 0;
            continue;
        }
        float z[4], t[4];
        for (int j = 0; j < 4; ++j) {
            z[j] = Z[v * 256 + j * 64 + lane];
            t[j] = tpdf[v * 256 + j * 64 + lane];
        }
        const float mx = wave_max(fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3])));
        float e[4], s = 0.f, ts = 0.f;
        for (int j = 0; j < 4; ++j) {
            e[j] = expf(z[j] - mx);
            s += e[j];
            ts += t[j];
        }
        s = wave_sum(s);
        ts = wave_sum(ts);
        const float ls = logf(s);
        float l = 0.f;
        for (int j = 0; j < 4; ++j) {
            const float p = e[j] / s, tt = t[j] / ts;
            const float g = (p - tt) * inv_b;
            dZ[v * 256 + j * 64 + lane] = f2bf(g);
            acc[j] += g;
            if (tt > 0.f) l -= tt * (z[j] - mx - ls);
        }
        lacc += l;
    }
    for (int j = 0; j < 4; ++j) sdb[wave][j * 64 + lane] = acc[j];
    lacc = wave_sum(lacc);
    if (lane == 0) sloss[wave] = lacc;
    __syncthreads();
    const int b = threadIdx.x;   // 256 threads: one output bin each
    const float sum = (sdb[0][b] + sdb[1][b]) + (sdb[2][b] + sdb[3][b]);
    unsafeAtomicAdd(&db[b], sum);
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, ((sloss[0] + sloss[1]) + (sloss[2] + sloss[3])) * inv_b);
}

// KL(p_march || p_net) of probe rows: tpdf (march pdfs), Z (net logits of the
// same rows). Adds sum over rows of KL to *acc.
__global__ void k_probe_kl(const float *__restrict__ Z, const float *__restrict__ tpdf, int64_t n,
                           float *acc)
{
    const int lane = threadIdx.x & 63;
    const int64_t v = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (v >= n) return;
    float z[4], t[4];
    for (int j = 0; j < 4; ++j) {
        z[j] = Z[v * 256 + j * 64 + lane];
        t[j] = tpdf[v * 256 + j * 64 + lane];
    }
    const float mx = wave_max(fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3])));
    float s = 0.f, ts = 0.f;
    for (int j = 0; j < 4; ++j) {
        s += expf(z[j] - mx);
        ts += t[j];
    }
    s = wave_sum(s);
    ts = wave_sum(ts);
    const float lse = mx + logf(s);
    float kl = 0.f;
    for (int j = 0; j < 4; ++j) {
        const float tt = t[j] / ts;
        if (tt > 0.f) kl += tt * (logf(tt) - (z[j] - lse));
    }
    kl = wave_sum(kl);
    if (lane == 0) unsafeAtomicAdd(acc, kl);
}

// judge[0] = 1 (fall back to the march) iff mean probe KL > bound; also
// records the mean in judge_kl.
__global__ void k_judge(const float *kl_sum, int64_t n_probe, float bound, int32_t *fallback,
                        float *judge_kl, unsigned long long *fallback_count)
{
    const float m = n_probe > 0 ? *kl_sum / (float)n_probe : 0.f;
    const int fb = !(m <= bound);
    *fallback = fb;
    *judge_kl = m;
    if (fb) atomicAdd(fallback_count, 1ull);
}

__global__ void k_gather_rows(const float *__restrict__ src, int64_t n, int64_t stride, int64_t step,
                              int64_t m, float *dst)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t s = i * step;
    for (int k = 0; k < 3; ++k) dst[k * m + i] = src[k * stride + s];
}

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

// Whole network fused with the softmax and its use (inference only). One
// wave takes 16 rows (vertices): it encodes them into a BF16 tile in LDS,
// runs the four hidden layers and the output layer on the matrix cores with
// the weights staged once per block in LDS (16-byte chunks XOR-swizzled by
// row), with the same MFMA sequence, bias add, ReLU and BF16 rounding as the
// unfused encode + GEMM path (so the logits are bit-identical to it), and
// keeps the logits in registers: lane l holds, for rows 4*(l/16) + r (r < 4),
// the logits of bins 16*c + l%16 (c < 16), i.e. field row v = c and column
// u = l%16. Per row: softmax; then either the probabilities (PROB) or
// inverse-CDF sampling with the march path's uniforms and row/column rule,
// the octahedral decode of ((u + u3)/16, (v + u4)/16) and
// pdf = p_b * 256 / (4 pi) (SAMPLE). Activations never reach HBM.
enum { OUT_SAMPLE = 0, OUT_PROB = 1 };

// Reductions and scans over the 16 lanes of a DPP row, all in VALU data-
// parallel primitives (no LDS crossbar): the butterfly uses quad_perm
// [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror and row_mirror, so every
// lane ends with the same bits (each step adds two equal partial sums in
// either order); the inclusive scan is Hillis-Steele over row_shr 1, 2, 4, 8
// (lanes shifted in from outside the row read 0).
template <int CTRL>
__device__ __forceinline__ float dppf(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float row16_sum(float v)
{
    v += dppf<0xB1>(v);
    v += dppf<0x4E>(v);
    v += dppf<0x141>(v);
    v += dppf<0x140>(v);
    return v;
}
__device__ __forceinline__ float row16_max(float v)
{
    v = fmaxf(v, dppf<0xB1>(v));
    v = fmaxf(v, dppf<0x4E>(v));
    v = fmaxf(v, dppf<0x141>(v));
    v = fmaxf(v, dppf<0x140>(v));
    return v;
}
__device__ __forceinline__ float row16_scan(float v)
{
    v += dppf<0x111>(v);
    v += dppf<0x112>(v);
    v += dppf<0x114>(v);
    v += dppf<0x118>(v);
    return v;
}

__device__ __forceinline__ int swz64(int row, int chunk) { return row * 64 + ((chunk ^ (row & 7)) << 3); }

// LDS element index of column e of a swizzled [rows][64] BF16 tile.
__device__ __forceinline__ int swz_el(int row, int e) { return swz64(row, e >> 3) + (e & 7); }

__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct InferArgs {
    Grid gr;
    const uint16_t *table;     // BF16 hash table [16][T][2]
    const uint16_t *wbf;       // BF16 weights, layer k at bw[k], [out][64]
    const float *params;       // FP32 parameters (biases)
    MlpLayout lay;
    const float *pos, *nrm;    // 3 x n SoA
    int64_t n;
    uint64_t seed;
    uint32_t bounce;
    float pdf_scale;
    float *dir_out, *pdf_out, *prob_out;
};

constexpr int kInferWaves = 4;

template <int MODE>
__global__ void __launch_bounds__(64 * kInferWaves) k_nn_infer(InferArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t Wh[4][64 * 64];
    __shared__ __attribute__((aligned(16))) uint16_t Ws[256 * 64];
    __shared__ float bh[4][64];
    __shared__ float bs[256];
    __shared__ __attribute__((aligned(16))) uint16_t act[kInferWaves][16 * 64];
    for (int t = threadIdx.x; t < 4 * 64 * 8; t += blockDim.x) {
        const int k = t >> 9, row = (t >> 3) & 63, ch = t & 7;
        *reinterpret_cast<uint4 *>(&Wh[k][swz64(row, ch)]) =
            *reinterpret_cast<const uint4 *>(A.wbf + A.lay.bw[k] + (int64_t)row * 64 + ch * 8);
    }
    for (int t = threadIdx.x; t < 256 * 8; t += blockDim.x) {
        const int row = t >> 3, ch = t & 7;
        *reinterpret_cast<uint4 *>(&Ws[swz64(row, ch)]) =
            *reinterpret_cast<const uint4 *>(A.wbf + A.lay.bw[4] + (int64_t)row * 64 + ch * 8);
    }
    for (int t = threadIdx.x; t < 256; t += blockDim.x) {
        bh[t >> 6][t & 63] = A.params[A.lay.boff[t >> 6] + (t & 63)];
        bs[t] = A.params[A.lay.boff[4] + t];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, g = lane >> 4, u = lane & 15;
    uint16_t *X = act[wave];
    const int64_t n = A.n;
    const int64_t tiles = (n + 15) / 16;
    const int64_t wstride = (int64_t)gridDim.x * kInferWaves;
    for (int64_t tile = blockIdx.x * (int64_t)kInferWaves + wave; tile < tiles; tile += wstride) {
        wave_fence();   // the previous tile's reads of X are done (also keeps LDS loads in the loop)
        const int64_t r0 = tile * 16;
        // encode: item j of a lane is row 4j + g, level u; lanes 0..15 also
        // write the normal and the zero padding of row u
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 4 * j + g;
            const int64_t v = min(r0 + row, n - 1);
            const float p[3] = {A.pos[v], A.pos[n + v], A.pos[2 * n + v]};
            const uint32_t pair = r0 + row < n ? encode_level(A.gr, A.table, p, u) : 0u;
            *reinterpret_cast<uint32_t *>(&X[swz_el(row, 2 * u)]) = pair;
        }
        if (lane < 16) {
            const int64_t v = min(r0 + lane, n - 1);
            const bool ok = r0 + lane < n;
            uint32_t w4[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) w4[k] = 0u;
            if (ok) {
                w4[0] = (uint32_t)f2bf(A.nrm[v]) | ((uint32_t)f2bf(A.nrm[n + v]) << 16);
                w4[1] = (uint32_t)f2bf(A.nrm[2 * n + v]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)   // columns 32..63: chunks 4..7
                *reinterpret_cast<uint4 *>(&X[swz64(lane, 4 + k)]) =
                    make_uint4(w4[4 * k], w4[4 * k + 1], w4[4 * k + 2], w4[4 * k + 3]);
        }
        wave_fence();
        // hidden layers: H = bf16(relu(X W^T + b)), written back over the tile
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(&X[swz64(u, g)]);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(&X[swz64(u, 4 + g)]);
            floatx4 hc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int row = 16 * c + u;
                const bf16x8 w0 = *reinterpret_cast<const bf16x8 *>(&Wh[k][swz64(row, g)]);
                const bf16x8 w1 = *reinterpret_cast<const bf16x8 *>(&Wh[k][swz64(row, 4 + g)]);
                hc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, w0, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                hc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, w1, hc[c], 0, 0, 0);
            }
            wave_fence();   // every lane has read its A fragments
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = hc[c][r] + bh[k][16 * c + u];
                    X[swz_el(4 * g + r, 16 * c + u)] = f2bf(v > 0.f ? v : 0.f);
                }
            wave_fence();
        }
        const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(&X[swz64(u, g)]);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(&X[swz64(u, 4 + g)]);
        floatx4 acc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int row = 16 * c + u;
            const bf16x8 w0 = *reinterpret_cast<const bf16x8 *>(&Ws[swz64(row, g)]);
            const bf16x8 w1 = *reinterpret_cast<const bf16x8 *>(&Ws[swz64(row, 4 + g)]);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, w0, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, w1, acc[c], 0, 0, 0);
        }
        // uniforms of row r0 + (lane % 16), fetched per row below
        uint32_t cu[4] = {0u, 0u, A.bounce, 0u};
        if (MODE == OUT_SAMPLE) {
            const uint64_t i = (uint64_t)(r0 + u);
            cu[0] = (uint32_t)i;
            cu[1] = (uint32_t)(i >> 32);
            core::philox(cu, (uint32_t)A.seed, (uint32_t)(A.seed >> 32));
        }
#pragma unroll 1
        for (int r = 0; r < 4; ++r) {   // one row of the lane group at a time (register pressure)
            const int64_t row = r0 + 4 * g + r;
            float e[16];
            float mx = -3.4e38f;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const floatx4 a4 = acc[c];
                const float x = r == 0 ? a4[0] : (r == 1 ? a4[1] : (r == 2 ? a4[2] : a4[3]));
                e[c] = x + bs[16 * c + u];
                mx = fmaxf(mx, e[c]);
            }
            mx = row16_max(mx);
#pragma unroll
            for (int c = 0; c < 16; ++c) e[c] = expf(e[c] - mx);
            if (MODE == OUT_PROB) {
                float sum = 0.f;
#pragma unroll
                for (int c = 0; c < 16; ++c) sum += e[c];
                sum = row16_sum(sum);
                if (row < n) {
#pragma unroll
                    for (int c = 0; c < 16; ++c) A.prob_out[row * 256 + 16 * c + u] = e[c] / sum;
                }
            } else {
                // marginal CDF over field rows (row sums reduced over the 16 lanes)
                float M[16];
                float run = 0.f;
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    run += row16_sum(e[c]);
                    M[c] = run;
                }
                const float total = M[15];
                const int src = 4 * g + r;   // a lane holding this row's uniforms
                const uint32_t b1 = __shfl(cu[0], src), b2 = __shfl(cu[1], src);
                const uint32_t b3 = __shfl(cu[2], src), b4u = __shfl(cu[3], src);
                const float u1 = (float)(b1 >> 8) * 5.9604644775390625e-8f;
                const float u2 = (float)(b2 >> 8) * 5.9604644775390625e-8f;
                const float tv = u1 * total;
                int v = 15;
#pragma unroll
                for (int c = 14; c >= 0; --c)
                    if (tv < M[c]) v = c;
                float ev = e[0];
#pragma unroll
                for (int c = 1; c < 16; ++c)
                    if (c == v) ev = e[c];
                const float S = row16_scan(ev);   // inclusive scan of field row v over its 16 columns
                const float rowsum = __shfl(S, 16 * g + 15);
                const uint64_t bal = __ballot(u2 * rowsum < S);
                const uint32_t mine = (uint32_t)(bal >> (16 * g)) & 0xffffu;
                const int col = mine ? __ffs(mine) - 1 : 15;
                const float Lb = __shfl(ev, 16 * g + col);
                if (u == 0 && row < n) {
                    const float inv = 1.f / 16.f;
                    const float u3 = (float)(b3 >> 8) * 5.9604644775390625e-8f;
                    const float u4 = (float)(b4u >> 8) * 5.9604644775390625e-8f;
                    float ox, oy, oz;
                    oct_decode((float)col * inv + u3 * inv, (float)v * inv + u4 * inv, ox, oy, oz);
                    A.dir_out[row] = ox;
                    A.dir_out[n + row] = oy;
                    A.dir_out[2 * n + row] = oz;
                    A.pdf_out[row] = (Lb / total) * A.pdf_scale;
                }
            }
        }
    }
}

// ----------------------------------------------------------------- Adam ----

__global__ void k_adam(float *p, float *m, float *v, const float *g, int64_t count, float lr,
                       float b1, float b2, float eps, float c1, float c2, int64_t mlp_count,
                       MlpLayout lay, uint16_t *wbf, int64_t table_off, uint16_t *tbf)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    const float pi = p[i] - upd;
    p[i] = pi;
    if (i >= table_off) {
        tbf[i - table_off] = f2bf(pi);
    } else {
        for (int k = 0; k < 5; ++k) {
            if (i >= lay.woff[k] && i < lay.woff[k] + (int64_t)lay.fin[k] * lay.fout[k]) {
                const int64_t r = (i - lay.woff[k]) / lay.fin[k], c = (i - lay.woff[k]) % lay.fin[k];
                wbf[lay.bw[k] + r * 64 + c] = f2bf(pi);
            }
        }
    }
}

// Deterministic initialization: weights U(-s, s) with s = sqrt(6 / fan_in),
// biases 0, table U(-1e-4, 1e-4), from a counter-based hash of the index.
__global__ void k_init(float *p, int64_t count, MlpLayout lay, int64_t table_off, uint64_t seed)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint32_t c[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), 0x5eedu, 0u};
    core::philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u = (float)(c[0] >> 8) * 5.9604644775390625e-8f * 2.f - 1.f;   // [-1, 1)
    float val = 0.f;
    if (i >= table_off) {
        val = 1e-4f * u;
    } else {
        for (int k = 0; k < 5; ++k)
            if (i >= lay.woff[k] && i < lay.woff[k] + (int64_t)lay.fin[k] * lay.fout[k])
                val = sqrtf(6.f / (float)lay.fin[k]) * u;
    }
    p[i] = val;
}

}  // namespace nn
}  // namespace wfpg

// ============================================================= host side ===
namespace wfpg {
namespace nn {

constexpr int kIn = 35, kH = 64, kOut = 256;

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

static hipError_t ensure(Buf &b, size_t bytes)
{
    if (b.bytes >= bytes) return hipSuccess;
    if (b.p) { hipError_t e = hipFree(b.p); if (e != hipSuccess) return e; }
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.bytes = bytes;
    return e;
}

struct Model {
    int log2T = 19, n_min = 16, n_max = 1024;
    Grid grid;
    int64_t count = 0, mlp = 0, table_off = 0;
    MlpLayout lay;
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;   // FP32 master, Adam, grads
    uint16_t *wbf = nullptr, *tbf = nullptr;                         // BF16 copies
    float *gW = nullptr, *gB = nullptr;                              // padded MLP grads
    int64_t steps_done = 0;
    bool trained = false;
    // scratch (rows padded to 64)
    Buf X, H[4], Z, dZ, dA[2], dX, tpdf, ppos, pnrm, Zp, tp, stats;
    float *d_loss = nullptr, *d_klsum = nullptr, *d_judge_kl = nullptr;
    int32_t *d_fallback = nullptr;
    unsigned long long *d_fallback_count = nullptr;

    int64_t bw_total() const { return lay.bw[4] + (int64_t)kOut * 64; }
    int64_t bias_off(int k) const { return lay.boff[k]; }
};

static void make_layout(Model &M)
{
    const int fin[5] = {kIn, kH, kH, kH, kH}, fout[5] = {kH, kH, kH, kH, kOut};
    int64_t off = 0, bw = 0;
    for (int k = 0; k < 5; ++k) {
        M.lay.fin[k] = fin[k];
        M.lay.fout[k] = fout[k];
        M.lay.woff[k] = off;
        off += (int64_t)fin[k] * fout[k];
        M.lay.boff[k] = off;
        off += fout[k];
        M.lay.bw[k] = bw;
        bw += (int64_t)fout[k] * 64;
    }
    M.mlp = off;
    M.table_off = off;
    M.count = off + 16ll * (1ll << M.log2T) * 2;
    const double b = std::exp((std::log((double)M.n_max) - std::log((double)M.n_min)) / 15.0);
    for (int l = 0; l < 16; ++l) M.grid.res[l] = (int32_t)std::floor((double)M.n_min * std::pow(b, (double)l));
    M.grid.log2T = M.log2T;
}

// FP32 master -> padded BF16 copies (after init or an explicit parameter set).
__global__ void k_refresh_bf16(const float *p, int64_t count, MlpLayout lay, int64_t table_off,
                               uint16_t *wbf, uint16_t *tbf)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = p[i];
    if (i >= table_off) {
        tbf[i - table_off] = f2bf(v);
        return;
    }
    for (int k = 0; k < 5; ++k)
        if (i >= lay.woff[k] && i < lay.woff[k] + (int64_t)lay.fin[k] * lay.fout[k]) {
            const int64_t r = (i - lay.woff[k]) / lay.fin[k], c = (i - lay.woff[k]) % lay.fin[k];
            wbf[lay.bw[k] + r * 64 + c] = f2bf(v);
        }
}

// Padded MLP gradients -> the flat gradient vector (same order as the
// parameters).
__global__ void k_pack_grads(const float *gW, const float *gB, MlpLayout lay, float *g, int64_t mlp)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= mlp) return;
    int64_t boff_acc = 0;
    for (int k = 0; k < 5; ++k) {
        const int64_t nw = (int64_t)lay.fin[k] * lay.fout[k];
        if (i >= lay.woff[k] && i < lay.woff[k] + nw) {
            const int64_t r = (i - lay.woff[k]) / lay.fin[k], c = (i - lay.woff[k]) % lay.fin[k];
            g[i] = gW[lay.bw[k] + r * 64 + c];
            return;
        }
        if (i >= lay.boff[k] && i < lay.boff[k] + lay.fout[k]) {
            g[i] = gB[boff_acc + (i - lay.boff[k])];
            return;
        }
        boff_acc += lay.fout[k];
    }
}

__global__ void k_fill(float *p, int64_t n, float v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static inline unsigned nb(int64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }
static inline int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

static hipError_t fill(float *p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nb(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <bool AT, bool BT, int EPI>
static hipError_t gemm(const GemmArgs &g, int splits, hipStream_t s)
{
    hipLaunchKernelGGL((k_gemm<AT, BT, EPI>), dim3(g.M / TS, g.N / TS, splits), dim3(256), 0, s, g);
    return hipGetLastError();
}

static GemmArgs gargs(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, int M, int N, int K)
{
    GemmArgs g;
    std::memset(&g, 0, sizeof g);
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.M = M; g.N = N; g.K = K; g.k_chunk = K;
    return g;
}

// Hidden activations H0..H3 [rows][64] of n positions (SoA with plane
// stride `stride`), rows padded to a multiple of 64; keeps X for a backward
// pass.
static hipError_t forward_hidden(Model &M, const float *pos, const float *nrm, int64_t n, int64_t stride,
                                 hipStream_t s)
{
    const int64_t rows = pad64(std::max<int64_t>(n, 1));
    hipError_t e = ensure(M.X, rows * 64 * 2);
    for (int k = 0; k < 4 && e == hipSuccess; ++k) e = ensure(M.H[k], rows * 64 * 2);
    if (e != hipSuccess) return e;
    uint16_t *X = (uint16_t *)M.X.p;
    hipLaunchKernelGGL(k_encode, dim3(nb(rows * 16, 256)), dim3(256), 0, s, M.grid, M.tbf, pos, nrm, n,
                       stride, rows, X);
    const uint16_t *in = X;
    for (int k = 0; k < 4; ++k) {
        GemmArgs g = gargs(in, 64, M.wbf + M.lay.bw[k], 64, (int)rows, 64, 64);
        g.Cb = (uint16_t *)M.H[k].p;
        g.ldc = 64;
        g.bias = M.p + M.lay.boff[k];
        e = gemm<false, true, EPI_BIAS_RELU>(g, 1, s);
        if (e != hipSuccess) return e;
        in = (const uint16_t *)M.H[k].p;
    }
    return hipSuccess;
}

// Logits Z [rows][256] (training and the judge's probes).
static hipError_t forward(Model &M, const float *pos, const float *nrm, int64_t n, int64_t stride,
                          hipStream_t s)
{
    const int64_t rows = pad64(std::max<int64_t>(n, 1));
    hipError_t e = forward_hidden(M, pos, nrm, n, stride, s);
    if (e == hipSuccess) e = ensure(M.Z, rows * 256 * 4);
    if (e != hipSuccess) return e;
    GemmArgs g = gargs((const uint16_t *)M.H[3].p, 64, M.wbf + M.lay.bw[4], 64, (int)rows, 256, 64);
    g.C = (float *)M.Z.p;
    g.ldc = 256;
    g.bias = M.p + M.lay.boff[4];
    return gemm<false, true, EPI_F32>(g, 1, s);
}

// Gradients of the mean cross-entropy of the last forward pass against the
// march pdfs tpdf ([rows][256]); writes the flat gradient vector M.g.
static hipError_t backward(Model &M, const float *pos, int64_t n, int64_t stride, const float *tpdf,
                           hipStream_t s)
{
    const int64_t rows = pad64(std::max<int64_t>(n, 1));
    hipError_t e = ensure(M.dZ, rows * 256 * 2);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = ensure(M.dA[k], rows * 64 * 2);
    if (e == hipSuccess) e = ensure(M.dX, rows * 64 * 4);
    if (e != hipSuccess) return e;
    e = fill(M.gW, M.bw_total(), 0.f, s);
    if (e == hipSuccess) e = fill(M.gB, 4 * kH + kOut, 0.f, s);
    if (e == hipSuccess) e = fill(M.g + M.table_off, M.count - M.table_off, 0.f, s);
    if (e == hipSuccess) e = fill(M.d_loss, 1, 0.f, s);
    if (e != hipSuccess) return e;
    uint16_t *dZ = (uint16_t *)M.dZ.p;
    hipLaunchKernelGGL(k_softmax_xent, dim3((unsigned)std::min<int64_t>(nb(rows, 4), (int64_t)device_cu_count() * 4)),
                       dim3(256), 0, s, (const float *)M.Z.p, tpdf, n,
                       rows, 1.f / (float)n, dZ, M.gB + 4 * kH, M.d_loss);
    const int ksplit = 2048;   // vertices per split-K chunk of the weight gradients
    const int splits = (int)((rows + ksplit - 1) / ksplit);
    // output layer
    {
        GemmArgs g = gargs(dZ, 256, (const uint16_t *)M.H[3].p, 64, 256, 64, (int)rows);
        g.k_chunk = ksplit;
        g.C = M.gW + M.lay.bw[4];
        g.ldc = 64;
        e = gemm<true, false, EPI_ATOMIC>(g, splits, s);
        if (e != hipSuccess) return e;
        GemmArgs h = gargs(dZ, 256, M.wbf + M.lay.bw[4], 64, (int)rows, 64, 256);
        h.Cb = (uint16_t *)M.dA[0].p;
        h.ldc = 64;
        h.mask = (const uint16_t *)M.H[3].p;
        h.colsum = M.gB + 3 * kH;
        e = gemm<false, false, EPI_MASK>(h, 1, s);
        if (e != hipSuccess) return e;
    }
    int cur = 0;
    for (int k = 3; k >= 1; --k) {
        const uint16_t *dA = (const uint16_t *)M.dA[cur].p;
        GemmArgs g = gargs(dA, 64, (const uint16_t *)M.H[k - 1].p, 64, 64, 64, (int)rows);
        g.k_chunk = ksplit;
        g.C = M.gW + M.lay.bw[k];
        g.ldc = 64;
        e = gemm<true, false, EPI_ATOMIC>(g, splits, s);
        if (e != hipSuccess) return e;
        GemmArgs h = gargs(dA, 64, M.wbf + M.lay.bw[k], 64, (int)rows, 64, 64);
        h.Cb = (uint16_t *)M.dA[cur ^ 1].p;
        h.ldc = 64;
        h.mask = (const uint16_t *)M.H[k - 1].p;
        h.colsum = M.gB + (k - 1) * kH;
        e = gemm<false, false, EPI_MASK>(h, 1, s);
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    {
        const uint16_t *dA = (const uint16_t *)M.dA[cur].p;
        GemmArgs g = gargs(dA, 64, (const uint16_t *)M.X.p, 64, 64, 64, (int)rows);
        g.k_chunk = ksplit;
        g.C = M.gW + M.lay.bw[0];
        g.ldc = 64;
        e = gemm<true, false, EPI_ATOMIC>(g, splits, s);
        if (e != hipSuccess) return e;
        GemmArgs h = gargs(dA, 64, M.wbf + M.lay.bw[0], 64, (int)rows, 64, 64);
        h.C = (float *)M.dX.p;
        h.ldc = 64;
        e = gemm<false, false, EPI_F32>(h, 1, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_hash_scatter, dim3(nb(n * 16, 256)), dim3(256), 0, s, M.grid, pos, n, stride,
                       (const float *)M.dX.p, M.g + M.table_off);
    hipLaunchKernelGGL(k_pack_grads, dim3(nb(M.mlp, 256)), dim3(256), 0, s, M.gW, M.gB, M.lay, M.g, M.mlp);
    return hipGetLastError();
}

// Network distribution of n positions, sampled (dir_out, pdf_out) or written
// out (prob_out), through the fused output kernel.
static hipError_t infer(Model &M, const float *pos, const float *nrm, int64_t n, int mode, uint64_t seed,
                        uint32_t bounce, float *dir_out, float *pdf_out, float *prob_out, hipStream_t s)
{
    const double pi = 3.14159265358979323846;
    InferArgs A;
    A.gr = M.grid;
    A.table = M.tbf;
    A.wbf = M.wbf;
    A.params = M.p;
    A.lay = M.lay;
    A.pos = pos;
    A.nrm = nrm;
    A.n = n;
    A.seed = seed;
    A.bounce = bounce;
    A.pdf_scale = (float)(256.0 / (4.0 * pi));
    A.dir_out = dir_out;
    A.pdf_out = pdf_out;
    A.prob_out = prob_out;
    const int64_t tiles = (n + 15) / 16;
    const unsigned grid = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((tiles + kInferWaves - 1) / kInferWaves, (int64_t)device_cu_count() * 2));
    if (mode == OUT_SAMPLE)
        hipLaunchKernelGGL(k_nn_infer<OUT_SAMPLE>, dim3(grid), dim3(64 * kInferWaves), 0, s, A);
    else
        hipLaunchKernelGGL(k_nn_infer<OUT_PROB>, dim3(grid), dim3(64 * kInferWaves), 0, s, A);
    return hipGetLastError();
}

static void free_model(Model *M)
{
    if (!M) return;
    void *ptrs[] = {M->p, M->m, M->v, M->g, M->wbf, M->tbf, M->gW, M->gB, M->d_loss, M->d_klsum,
                    M->d_judge_kl, M->d_fallback, M->d_fallback_count};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    Buf *bufs[] = {&M->X, &M->H[0], &M->H[1], &M->H[2], &M->H[3], &M->Z, &M->dZ, &M->dA[0], &M->dA[1],
                   &M->dX, &M->tpdf, &M->ppos, &M->pnrm, &M->Zp, &M->tp, &M->stats};
    for (Buf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    delete M;
}

static hipError_t create_model(Model *&out, int log2T, int n_min, int n_max, uint64_t seed, hipStream_t s)
{
    Model *M = new (std::nothrow) Model();
    if (!M) return hipErrorOutOfMemory;
    M->log2T = log2T;
    M->n_min = n_min;
    M->n_max = n_max;
    make_layout(*M);
    hipError_t e = hipMalloc((void **)&M->p, M->count * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->m, M->count * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->v, M->count * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->g, M->count * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->wbf, M->bw_total() * 2);
    if (e == hipSuccess) e = hipMalloc((void **)&M->tbf, (M->count - M->table_off) * 2);
    if (e == hipSuccess) e = hipMalloc((void **)&M->gW, M->bw_total() * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->gB, (4 * kH + kOut) * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->d_loss, 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->d_klsum, 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->d_judge_kl, 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->d_fallback, 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->d_fallback_count, 8);
    if (e == hipSuccess) e = hipMemsetAsync(M->m, 0, M->count * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(M->v, 0, M->count * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(M->wbf, 0, M->bw_total() * 2, s);
    if (e == hipSuccess) e = hipMemsetAsync(M->d_fallback_count, 0, 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(M->d_judge_kl, 0, 4, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_init, dim3(nb(M->count, 256)), dim3(256), 0, s, M->p, M->count, M->lay,
                           M->table_off, seed);
        hipLaunchKernelGGL(k_refresh_bf16, dim3(nb(M->count, 256)), dim3(256), 0, s, M->p, M->count,
                           M->lay, M->table_off, M->wbf, M->tbf);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        free_model(M);
        return e;
    }
    out = M;
    return hipSuccess;
}

}  // namespace nn

void destroy_model(void *m) { nn::free_model((nn::Model *)m); }

}  // namespace wfpg

// ================================================================ C ABI ====
using namespace wfpg;
using wfpg::nn::Model;

namespace {

wfpg_status st_of(hipError_t e, int line)
{
    if (e == hipSuccess) return WFPG_OK;
    (void)note_error(e, __FILE__, line);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? WFPG_ENOMEM : WFPG_EDEVICE;
}

Model *model_of(const wfpg_svo *svo) { return (Model *)svo->nn_model; }

hipError_t get_model(wfpg_svo *svo, const wfpg_train_cfg *c, hipStream_t s, Model *&M)
{
    M = model_of(svo);
    if (M) return hipSuccess;
    const int n_max = c->n_max > 0 ? c->n_max : (1 << svo->depth);
    hipError_t e = nn::create_model(M, c->log2_table, c->n_min, n_max, c->seed, s);
    if (e == hipSuccess) svo->nn_model = M;
    return e;
}

bool valid_cfg(const wfpg_train_cfg *c)
{
    return c && c->log2_table >= 10 && c->log2_table <= 24 && c->n_min >= 2 && c->n_max >= 0 &&
           (c->n_max == 0 || c->n_max > c->n_min) && c->batch >= 64 && c->batch <= (1 << 22) &&
           c->steps >= 0 && std::isfinite(c->lr_mlp) && std::isfinite(c->lr_table) &&
           c->lr_mlp >= 0 && c->lr_table >= 0 && c->beta1 >= 0 && c->beta1 < 1 && c->beta2 >= 0 &&
           c->beta2 < 1 && c->adam_eps > 0 && std::isfinite(c->target_eps) && c->target_eps > 0 &&
           (c->target_blur == 0 || c->target_blur == 1);
}

// The march's pdf at N = 16 of n vertices (SoA planes of stride `stride`):
// the field with the given eps, optional jitter key and blur (Sec. 4), as
// guide_pdf computes it.
hipError_t march_pdf(const wfpg_svo *svo, const float *pos, int64_t n, int64_t stride, float eps,
                     int jitter, uint32_t jitter_key, int blur, float *out, hipStream_t s)
{
    GuideArgs a;
    std::memset(&a, 0, sizeof a);
    const double pi = 3.14159265358979323846;
    a.pos = pos;
    a.n = n;
    a.stride = stride;
    a.eps = eps;
    a.jitter = jitter;
    a.jitter_key = jitter_key;
    a.blur = blur;
    a.omega = (float)(4.0 * pi / 256.0);
    a.pdf_scale = (float)(256.0 / (4.0 * pi));
    a.dirtab = device_dirtab(16);
    a.err = svo->d_err;
    a.pdf_out = out;
    if (!a.dirtab) return hipErrorOutOfMemory;
    return launch_guide(svo, 16, MODE_PDF, a, choose_tile(svo, 16), s);
}

}  // namespace

extern "C" {

wfpg_train_cfg wfpg_default_train_cfg(void)
{
    wfpg_train_cfg c;
    c.log2_table = 19;
    c.n_min = 16;
    c.n_max = 0;
    c.batch = 65536;
    c.steps = 100;
    c.lr_mlp = 2e-3f;
    c.lr_table = 1e-2f;
    c.beta1 = 0.9f;
    c.beta2 = 0.99f;
    c.adam_eps = 1e-15f;
    c.seed = 1;
    c.target_eps = 0.01f;
    c.target_blur = 0;
    return c;
}

wfpg_status guide_train(wfpg_svo *svo, const float *pos, const float *nrm, int64_t n,
                        const wfpg_train_cfg *cfg, float *mean_loss, void *hip_stream)
{
    if (!svo || !valid_cfg(cfg) || n <= 0 || !pos || !nrm) return WFPG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    Model *M = nullptr;
    hipError_t e = get_model(svo, cfg, s, M);
    if (e != hipSuccess) return st_of(e, __LINE__);
    const int64_t b = std::min<int64_t>(cfg->batch, n);
    e = nn::ensure(M->tpdf, nn::pad64(b) * 256 * 4);
    if (e != hipSuccess) return st_of(e, __LINE__);
    float loss_acc = 0.f;
    int loss_n = 0;
    for (int st = 0; st < cfg->steps; ++st) {
        int64_t off = (int64_t)(((uint64_t)M->steps_done * (uint64_t)b) % (uint64_t)n);
        if (off + b > n) off = n - b;
        e = march_pdf(svo, pos + off, b, n, cfg->target_eps, 0, 0u, cfg->target_blur, (float *)M->tpdf.p, s);
        if (e == hipSuccess) e = nn::forward(*M, pos + off, nrm + off, b, n, s);
        if (e == hipSuccess) e = nn::backward(*M, pos + off, b, n, (const float *)M->tpdf.p, s);
        if (e != hipSuccess) return st_of(e, __LINE__);
        const int64_t t = M->steps_done + 1;
        const float c1 = 1.f - (float)std::pow((double)cfg->beta1, (double)t);
        const float c2 = 1.f - (float)std::pow((double)cfg->beta2, (double)t);
        // two launches: MLP part and table part use their own learning rates
        hipLaunchKernelGGL(nn::k_adam, dim3(nn::nb(M->mlp, 256)), dim3(256), 0, s, M->p, M->m, M->v, M->g,
                           M->mlp, cfg->lr_mlp, cfg->beta1, cfg->beta2, cfg->adam_eps, c1, c2, M->mlp,
                           M->lay, M->wbf, M->table_off, M->tbf);
        hipLaunchKernelGGL(nn::k_adam, dim3(nn::nb(M->count - M->table_off, 256)), dim3(256), 0, s,
                           M->p + M->table_off, M->m + M->table_off, M->v + M->table_off,
                           M->g + M->table_off, M->count - M->table_off, cfg->lr_table, cfg->beta1,
                           cfg->beta2, cfg->adam_eps, c1, c2, (int64_t)0, M->lay, M->wbf, (int64_t)0, M->tbf);
        e = hipGetLastError();
        if (e != hipSuccess) return st_of(e, __LINE__);
        M->steps_done = t;
        if (mean_loss && st >= cfg->steps - 10) {
            float l = 0.f;
            e = hipMemcpyAsync(&l, M->d_loss, 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return st_of(e, __LINE__);
            loss_acc += l;
            ++loss_n;
        }
    }
    M->trained = true;
    if (mean_loss) *mean_loss = loss_n ? loss_acc / loss_n : 0.f;
    return WFPG_OK;
}

wfpg_status wfpg_nn_params(wfpg_svo *svo, float *host, int64_t count, int32_t set, void *hip_stream)
{
    if (!svo || !host || (set != 0 && set != 1)) return WFPG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    Model *M = model_of(svo);
    if (!M && set) {
        wfpg_train_cfg c = wfpg_default_train_cfg();
        hipError_t e = get_model(svo, &c, s, M);
        if (e != hipSuccess) return st_of(e, __LINE__);
    }
    if (!M) return WFPG_ESTATE;
    if (count != M->count) return WFPG_EINVAL;
    hipError_t e;
    if (set) {
        e = hipMemcpyAsync(M->p, host, count * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(nn::k_refresh_bf16, dim3(nn::nb(M->count, 256)), dim3(256), 0, s, M->p,
                               M->count, M->lay, M->table_off, M->wbf, M->tbf);
            e = hipGetLastError();
        }
        M->trained = true;
    } else {
        e = hipMemcpyAsync(host, M->p, count * 4, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return st_of(e, __LINE__);
}

int64_t wfpg_nn_param_count(const wfpg_svo *svo)
{
    const Model *M = svo ? model_of(svo) : nullptr;
    return M ? M->count : -1;
}

wfpg_status wfpg_nn_forward(wfpg_svo *svo, const float *pos, const float *nrm, int64_t n,
                            float *prob_out, void *hip_stream)
{
    if (!svo || n < 0 || (n > 0 && (!pos || !nrm || !prob_out))) return WFPG_EINVAL;
    Model *M = model_of(svo);
    if (!M) return WFPG_ESTATE;
    if (n == 0) return WFPG_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    const hipError_t e = nn::infer(*M, pos, nrm, n, nn::OUT_PROB, 0, 0, nullptr, nullptr, prob_out, s);
    return st_of(e, __LINE__);
}

wfpg_status wfpg_nn_grad(wfpg_svo *svo, const float *pos, const float *nrm, const float *target,
                         int64_t n, float *grad_out, float *loss_out, void *hip_stream)
{
    if (!svo || n <= 0 || !pos || !nrm || !target || !grad_out) return WFPG_EINVAL;
    Model *M = model_of(svo);
    if (!M) return WFPG_ESTATE;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = nn::ensure(M->tpdf, nn::pad64(n) * 256 * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(M->tpdf.p, target, n * 256 * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = nn::forward(*M, pos, nrm, n, n, s);
    if (e == hipSuccess) e = nn::backward(*M, pos, n, n, (const float *)M->tpdf.p, s);
    if (e == hipSuccess) e = hipMemcpyAsync(grad_out, M->g, M->count * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && loss_out) {
        e = hipMemcpyAsync(loss_out, M->d_loss, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    return st_of(e, __LINE__);
}

wfpg_status wfpg_learned_stats(const wfpg_svo *svo, float *last_probe_kl, int64_t *fallbacks)
{
    if (!svo) return WFPG_EINVAL;
    const Model *M = model_of(svo);
    if (!M) return WFPG_ESTATE;
    float kl = 0.f;
    unsigned long long fb = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&kl, M->d_judge_kl, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&fb, M->d_fallback_count, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return st_of(e, __LINE__);
    if (last_probe_kl) *last_probe_kl = kl;
    if (fallbacks) *fallbacks = (int64_t)fb;
    return WFPG_OK;
}

}  // extern "C"

namespace wfpg {

// guide_sample with the learned model: network sample for every vertex;
// every probe_stride-th vertex is also marched and the network judged by the
// probes' mean KL(p_march || p_net); a march kernel gated by that judgment
// overwrites the outputs when the bound is exceeded. No host synchronization.
wfpg_status learned_sample(const wfpg_svo *svo, const float *pos, const float *nrm, int64_t n,
                           uint64_t seed, uint32_t bounce, const wfpg_opts *o, float *dir_out,
                           float *pdf_out, hipStream_t s)
{
    Model *M = model_of(svo);
    if (!M || !M->trained) return WFPG_ESTATE;
    if (o->N != 16 || !nrm || o->probe_stride < 1 || !std::isfinite(o->kl_bound)) return WFPG_EINVAL;
    const double pi = 3.14159265358979323846;
    hipError_t e = nn::infer(*M, pos, nrm, n, nn::OUT_SAMPLE, seed, bounce, dir_out, pdf_out, nullptr, s);
    const int64_t step = o->probe_stride;
    const int64_t m = (n + step - 1) / step;
    if (e == hipSuccess) e = nn::ensure(M->ppos, m * 3 * 4);
    if (e == hipSuccess) e = nn::ensure(M->pnrm, m * 3 * 4);
    if (e == hipSuccess) e = nn::ensure(M->tp, nn::pad64(m) * 256 * 4);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(nn::k_gather_rows, dim3(nn::nb(m, 256)), dim3(256), 0, s, pos, n, n, step, m,
                           (float *)M->ppos.p);
        hipLaunchKernelGGL(nn::k_gather_rows, dim3(nn::nb(m, 256)), dim3(256), 0, s, nrm, n, n, step, m,
                           (float *)M->pnrm.p);
        e = hipGetLastError();
    }
    // the probes' targets are the field the fallback march samples (same eps,
    // jitter and blur), so the judge measures the network against its output
    if (e == hipSuccess)
        e = march_pdf(svo, (const float *)M->ppos.p, m, m, o->eps, o->jitter, o->jitter_key, o->blur,
                      (float *)M->tp.p, s);
    if (e == hipSuccess) e = nn::forward(*M, (const float *)M->ppos.p, (const float *)M->pnrm.p, m, m, s);
    if (e == hipSuccess) e = nn::fill(M->d_klsum, 1, 0.f, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(nn::k_probe_kl, dim3(nn::nb(m, 4)), dim3(256), 0, s, (const float *)M->Z.p,
                           (const float *)M->tp.p, m, M->d_klsum);
        hipLaunchKernelGGL(nn::k_judge, dim3(1), dim3(1), 0, s, (const float *)M->d_klsum, m, o->kl_bound,
                           M->d_fallback, M->d_judge_kl, M->d_fallback_count);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        GuideArgs a;
        std::memset(&a, 0, sizeof a);
        a.pos = pos;
        a.n = n;
        a.eps = o->eps;
        a.jitter = o->jitter;
        a.jitter_key = o->jitter_key;
        a.blur = o->blur;
        a.omega = (float)(4.0 * pi / 256.0);
        a.pdf_scale = (float)(256.0 / (4.0 * pi));
        a.seed = seed;
        a.bounce = bounce;
        a.dir_out = dir_out;
        a.pdf_out = pdf_out;
        a.dirtab = device_dirtab(16);
        a.err = svo->d_err;
        a.gate = M->d_fallback;
        e = a.dirtab ? launch_guide(svo, 16, MODE_SAMPLE, a, choose_tile(svo, 16), s) : hipErrorOutOfMemory;
    }
    return st_of(e, __LINE__);
}

}  // namespace wfpg
