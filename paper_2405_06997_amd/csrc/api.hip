// C ABI of the path-guiding library: argument validation, device memory
// ownership and kernel dispatch. Declarations and contracts: include/wfpg.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "antialias_core.h"
#include "wfpg_internal.h"

using namespace wfpg;

namespace wfpg {

namespace {
thread_local char g_last_error[256] = "";
}

hipError_t note_error(hipError_t e, const char *file, int line)
{
    if (e != hipSuccess) {
        const char *base = std::strrchr(file, '/');
        std::snprintf(g_last_error, sizeof g_last_error, "%s (%s:%d)", hipGetErrorName(e),
                      base ? base + 1 : file, line);
    }
    return e;
}

int device_cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
            cu = 256;
        cached[dev] = cu;
    }
    return cached[dev];
}

// Bin-centre directions of the N x N field: the equal-area concentric
// octahedral map (Clarberg 2008, the projection named in Sec. 4) evaluated in
// FP64 at ((u + 1/2)/N, (v + 1/2)/N) and rounded to FP32.
void host_dir_table(int N, float *out)
{
    const double quarter_pi = std::atan(1.0);
    for (int v = 0; v < N; ++v) {
        for (int u = 0; u < N; ++u) {
            const double a = 2.0 * ((u + 0.5) / N) - 1.0;
            const double b = 2.0 * ((v + 0.5) / N) - 1.0;
            const double aa = std::fabs(a), ab = std::fabs(b);
            const double d = 1.0 - (aa + ab);
            const double r = 1.0 - std::fabs(d);
            const double phi = (r == 0.0) ? 0.0 : ((ab - aa) / r + 1.0) * quarter_pi;
            const double s = r * std::sqrt(2.0 - r * r);
            float *o = out + 3 * (v * N + u);
            o[0] = (float)((a >= 0.0 ? 1.0 : -1.0) * std::cos(phi) * s);
            o[1] = (float)((b >= 0.0 ? 1.0 : -1.0) * std::sin(phi) * s);
            o[2] = (float)((d >= 0.0 ? 1.0 : -1.0) * (1.0 - r * r));
        }
    }
}

const float *device_dirtab(int N)
{
    static std::mutex mu;
    static float *tabs[64][5] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    int slot = -1;   // N = 8, 16, 32, 64, 128
    for (int k = 0; k < 5; ++k)
        if (N == (8 << k)) slot = k;
    if (slot < 0) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    if (!tabs[dev][slot]) {
        std::vector<float> h((size_t)N * N * 3);
        host_dir_table(N, h.data());
        float *d = nullptr;
        if (hipMalloc((void **)&d, h.size() * sizeof(float)) != hipSuccess) return nullptr;
        if (hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return nullptr;
        }
        tabs[dev][slot] = d;
    }
    return tabs[dev][slot];
}

}  // namespace wfpg

namespace {

// The jittered cone directions the kernels use for one key (FP32, 3 per bin).
__global__ void k_jitter_table(int N, uint32_t key, float *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N * N) return;
    wfpg::aa::jitter_dir(N, b, key, out[3 * b], out[3 * b + 1], out[3 * b + 2]);
}

wfpg_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return WFPG_OK;
    if (!g_last_error[0]) (void)note_error(e, "api", 0);
    if (e == hipErrorOutOfMemory) return WFPG_ENOMEM;
    return WFPG_EDEVICE;
}

// Cell range of [lo, hi] along one axis under the half-open rule.
void cell_range(float lo, float hi, int D, int32_t &i0, int32_t &i1)
{
    const int R = 1 << D;
    const float R_f = (float)R;
    int32_t a = (int32_t)std::floor(lo * R_f);
    int32_t b = (int32_t)std::ceil(hi * R_f) - 1;
    if (b < a) b = a;
    a = std::min(std::max(a, 0), R - 1);
    b = std::min(std::max(b, 0), R - 1);
    i0 = a;
    i1 = b;
}

bool valid_opts(const wfpg_opts *o)
{
    if (!o) return false;
    if (o->N != 8 && o->N != 16 && o->N != 32) return false;
    if (!std::isfinite(o->eps) || !(o->eps > 0.f)) return false;
    if (o->mode != 0 && o->mode != 1) return false;
    if ((o->jitter != 0 && o->jitter != 1) || (o->blur != 0 && o->blur != 1)) return false;
    return true;
}

// Kernel arguments common to the guide entry points; the bin-direction table
// is the library's (uploaded on first use) unless with_table is false.
GuideArgs base_args(const wfpg_svo *svo, const wfpg_opts *o, bool with_table = true)
{
    GuideArgs a;
    std::memset(&a, 0, sizeof a);
    const double pi = 3.14159265358979323846;
    a.eps = o->eps;
    a.omega = (float)(4.0 * pi / (double)(o->N * o->N));
    a.pdf_scale = (float)((double)(o->N * o->N) / (4.0 * pi));
    a.dirtab = with_table ? device_dirtab(o->N) : nullptr;
    a.err = svo->d_err;
    a.jitter = o->jitter;
    a.jitter_key = o->jitter_key;
    a.blur = o->blur;
    return a;
}

void free_svo(wfpg_svo *s)
{
    if (!s) return;
    void *ptrs[] = {s->d_bits, s->d_rank, s->d_keys, s->d_nrm, s->d_e32, s->d_e16,
                    s->d_sum, s->d_cnt, s->d_dropped, s->d_err, s->d_ctr};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s->nn_model) destroy_model(s->nn_model);
    if (s->bin_work) destroy_bin_work(s->bin_work);
    delete s;
}

}  // namespace

extern "C" {

wfpg_opts wfpg_default_opts(void)
{
    wfpg_opts o;
    o.N = 16;
    o.eps = 0.01f;
    o.mode = 0;
    o.kl_bound = 0.05f;
    o.probe_stride = 256;
    o.jitter = 0;
    o.jitter_key = 0;
    o.blur = 0;
    return o;
}

const char *wfpg_status_string(wfpg_status s)
{
    switch (s) {
    case WFPG_OK: return "ok";
    case WFPG_EINVAL: return "invalid argument";
    case WFPG_ENOMEM: return "out of memory";
    case WFPG_EDEVICE: return "device error";
    case WFPG_ESTATE: return "invalid state";
    case WFPG_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

wfpg_status svo_build(const wfpg_rect *rects, int64_t n_rects, int32_t depth, int32_t exitance_fmt,
                      void *hip_stream, wfpg_svo **out)
{
    if (!out) return WFPG_EINVAL;
    *out = nullptr;
    if (depth < 1 || depth > WFPG_MAXD || n_rects < 0 || (n_rects > 0 && !rects)) return WFPG_EINVAL;
    if (exitance_fmt != WFPG_FP32 && exitance_fmt != WFPG_FP16 && exitance_fmt != WFPG_BF16)
        return WFPG_EINVAL;
    if (n_rects >= (1ll << 29)) return WFPG_EINVAL;
    std::vector<RectCells> rc((size_t)n_rects);
    std::vector<int64_t> foff((size_t)n_rects + 1, 0);
    for (int64_t i = 0; i < n_rects; ++i) {
        const wfpg_rect &r = rects[i];
        if (r.axis < 0 || r.axis > 2 || (r.sign != 1 && r.sign != -1)) return WFPG_EINVAL;
        const float v[5] = {r.c, r.lo[0], r.lo[1], r.hi[0], r.hi[1]};
        for (float x : v)
            if (!std::isfinite(x)) return WFPG_EINVAL;
        if (r.lo[0] > r.hi[0] || r.lo[1] > r.hi[1]) return WFPG_EINVAL;
        RectCells &c = rc[(size_t)i];
        int32_t dummy;
        c.axis = r.axis;
        cell_range(r.c, r.c, depth, c.ca, dummy);
        cell_range(r.lo[0], r.hi[0], depth, c.a0, c.a1);
        cell_range(r.lo[1], r.hi[1], depth, c.b0, c.b1);
        c.cls = r.axis * 2 + (r.sign > 0 ? 1 : 0);
        c.emissive = r.emissive;
        foff[(size_t)i + 1] = foff[(size_t)i] + (int64_t)(c.a1 - c.a0 + 1) * (c.b1 - c.b0 + 1);
    }
    const int64_t n_frag = foff[(size_t)n_rects];
    hipStream_t s = (hipStream_t)hip_stream;
    wfpg_svo *svo = new (std::nothrow) wfpg_svo();
    if (!svo) return WFPG_ENOMEM;
    svo->depth = depth;
    svo->fmt = exitance_fmt;
    (void)hipGetDevice(&svo->device);
    svo->total_words = level_woff(depth + 1);
#define NOTE(x) note_error((x), __FILE__, __LINE__)
    hipError_t e = NOTE(hipMalloc((void **)&svo->d_bits, svo->total_words * sizeof(uint64_t)));
    if (e == hipSuccess) e = NOTE(hipMalloc((void **)&svo->d_rank, svo->total_words * sizeof(uint32_t)));
    if (e == hipSuccess) e = NOTE(hipMalloc((void **)&svo->d_dropped, 2 * sizeof(unsigned long long)));
    if (e == hipSuccess) e = NOTE(hipMalloc((void **)&svo->d_err, sizeof(int32_t)));
    if (e == hipSuccess)
        e = NOTE(hipMalloc((void **)&svo->d_ctr, (size_t)kCounterPool * kQueueRanges * kQueueStride * sizeof(unsigned long long)));
    if (e == hipSuccess) e = NOTE(hipMemsetAsync(svo->d_bits, 0, svo->total_words * sizeof(uint64_t), s));
    if (e == hipSuccess) e = NOTE(hipMemsetAsync(svo->d_dropped, 0, 2 * sizeof(unsigned long long), s));
    if (e == hipSuccess) e = NOTE(hipMemsetAsync(svo->d_err, 0, sizeof(int32_t), s));
    RectCells *d_rc = nullptr;
    int64_t *d_foff = nullptr;
    if (e == hipSuccess && n_rects > 0) {
        e = hipMalloc((void **)&d_rc, rc.size() * sizeof(RectCells));
        if (e == hipSuccess) e = hipMalloc((void **)&d_foff, foff.size() * sizeof(int64_t));
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_rc, rc.data(), rc.size() * sizeof(RectCells), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_foff, foff.data(), foff.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = launch_build(svo, d_rc, d_foff, n_rects, n_frag, s);
    if (e == hipSuccess) e = NOTE(hipStreamSynchronize(s));
#undef NOTE
    if (d_rc) (void)hipFree(d_rc);
    if (d_foff) (void)hipFree(d_foff);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_svo(svo);
        return from_hip(e);
    }
    *out = svo;
    return WFPG_OK;
}

void svo_destroy(wfpg_svo *svo)
{
    if (!svo) return;
    (void)hipDeviceSynchronize();
    free_svo(svo);
}

wfpg_status svo_accumulate(wfpg_svo *svo, const float *pos, const float *wo, const float *rgb,
                           int64_t n, void *hip_stream)
{
    if (!svo || n < 0 || (n > 0 && (!pos || !wo || !rgb))) return WFPG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = launch_accumulate(svo, pos, wo, rgb, n, s);
    if (e == hipSuccess) e = launch_propagate(svo, s);
    return from_hip(e);
}

wfpg_status svo_accumulate_paths(wfpg_svo *svo, const float *pos, const float *T, const float *eye,
                                 const int32_t *hit, const float *Le, int64_t P, int32_t d, void *hip_stream)
{
    if (!svo || P < 0 || d < 1 || d > 64 || (P > 0 && (!pos || !T || !eye || !hit || !Le))) return WFPG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = launch_accumulate_paths(svo, pos, T, eye, hit, Le, P, d, s);
    if (e == hipSuccess) e = launch_propagate(svo, s);
    return from_hip(e);
}

static wfpg_status guide_common(const wfpg_svo *svo, int mode, const wfpg_opts *o, GuideArgs &a,
                                void *hip_stream)
{
    if (!a.dirtab) return WFPG_ENOMEM;
    return from_hip(launch_guide(svo, o->N, mode, a, choose_tile(svo, o->N), (hipStream_t)hip_stream));
}

wfpg_status guide_pdf(const wfpg_svo *svo, const float *pos, int64_t n, const wfpg_opts *opts,
                      float *pdf_out, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || (n > 0 && (!pos || !pdf_out))) return WFPG_EINVAL;
    if (opts->mode != 0) return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    GuideArgs a = base_args(svo, opts);
    a.pos = pos;
    a.n = n;
    a.pdf_out = pdf_out;
    return guide_common(svo, MODE_PDF, opts, a, hip_stream);
}

wfpg_status guide_sample(const wfpg_svo *svo, const float *pos, const float *nrm, int64_t n,
                         uint64_t seed, uint32_t bounce, const wfpg_opts *opts, float *dir_out,
                         float *pdf_out, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || (n > 0 && (!pos || !dir_out || !pdf_out)))
        return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    if (opts->mode == 1)
        return learned_sample(svo, pos, nrm, n, seed, bounce, opts, dir_out, pdf_out, (hipStream_t)hip_stream);
    GuideArgs a = base_args(svo, opts);
    a.pos = pos;
    a.n = n;
    a.seed = seed;
    a.bounce = bounce;
    a.dir_out = dir_out;
    a.pdf_out = pdf_out;
    return guide_common(svo, MODE_SAMPLE, opts, a, hip_stream);
}

wfpg_status pdf_eval(const wfpg_svo *svo, const float *pos, const float *dir, int64_t n,
                     const wfpg_opts *opts, float *pdf_out, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || (n > 0 && (!pos || !dir || !pdf_out))) return WFPG_EINVAL;
    if (opts->mode != 0) return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    GuideArgs a = base_args(svo, opts);
    a.pos = pos;
    a.dir_in = dir;
    a.n = n;
    a.pdf_out = pdf_out;
    return guide_common(svo, MODE_EVAL, opts, a, hip_stream);
}

// Exactly one BSDF source: normals (Lambertian table) or explicit tables.
static bool one_table(const float *nrm, const float *bsdf) { return (nrm != nullptr) != (bsdf != nullptr); }

wfpg_status guide_sample_product(const wfpg_svo *svo, const float *pos, const float *nrm, const float *bsdf,
                                 int64_t n, uint64_t seed, uint32_t bounce, const wfpg_opts *opts, float *dir_out,
                                 float *pdf_out, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || opts->mode != 0 ||
        (n > 0 && (!pos || !dir_out || !pdf_out || !one_table(nrm, bsdf))))
        return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    GuideArgs a = base_args(svo, opts);
    a.pos = pos;
    a.n = n;
    a.seed = seed;
    a.bounce = bounce;
    a.dir_out = dir_out;
    a.pdf_out = pdf_out;
    a.nrm_in = nrm;
    a.bsdf_in = bsdf;
    a.dirtab8 = device_dirtab(8);
    if (!a.dirtab8) return WFPG_ENOMEM;
    return guide_common(svo, MODE_PRODUCT, opts, a, hip_stream);
}

wfpg_status pdf_eval_product(const wfpg_svo *svo, const float *pos, const float *nrm, const float *bsdf,
                             const float *dir, int64_t n, const wfpg_opts *opts, float *pdf_out, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || opts->mode != 0 ||
        (n > 0 && (!pos || !dir || !pdf_out || !one_table(nrm, bsdf))))
        return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    GuideArgs a = base_args(svo, opts);
    a.pos = pos;
    a.dir_in = dir;
    a.n = n;
    a.pdf_out = pdf_out;
    a.nrm_in = nrm;
    a.bsdf_in = bsdf;
    a.dirtab8 = device_dirtab(8);
    if (!a.dirtab8) return WFPG_ENOMEM;
    return guide_common(svo, MODE_PEVAL, opts, a, hip_stream);
}

wfpg_status wfpg_debug_march(const wfpg_svo *svo, const float *pos, int64_t n, const wfpg_opts *opts,
                             int32_t *out, int32_t *visits, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || (n > 0 && (!pos || !out))) return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    GuideArgs a = base_args(svo, opts);
    a.pos = pos;
    a.n = n;
    a.dbg_out = out;
    a.dbg_visits = visits;
    return guide_common(svo, MODE_DEBUG, opts, a, hip_stream);
}

wfpg_status wfpg_march_counts(const wfpg_svo *svo, const float *pos, int64_t n, const wfpg_opts *opts,
                              int32_t *counts, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || (n > 0 && (!pos || !counts))) return WFPG_EINVAL;
    if (n == 0) return WFPG_OK;
    GuideArgs a = base_args(svo, opts);
    a.pos = pos;
    a.n = n;
    a.dbg_out = counts;
    return guide_common(svo, MODE_COUNT, opts, a, hip_stream);
}

wfpg_status svo_stats(const wfpg_svo *svo, int64_t *leaves, int64_t *nodes, int64_t *dropped_splats,
                      int32_t *error_flags)
{
    if (!svo) return WFPG_EINVAL;
    hipError_t e = hipDeviceSynchronize();
    unsigned long long d[2] = {0, 0};
    int32_t err = 0;
    if (e == hipSuccess) e = hipMemcpy(d, svo->d_dropped, sizeof d, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&err, svo->d_err, sizeof err, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    if (leaves) *leaves = svo->n[svo->depth];
    if (nodes) *nodes = svo->total_nodes;
    if (dropped_splats) *dropped_splats = (int64_t)(d[0] + d[1]);
    if (error_flags) *error_flags = err;
    return WFPG_OK;
}

int64_t svo_level_size(const wfpg_svo *svo, int32_t level)
{
    if (!svo || level < 0 || level > svo->depth) return -1;
    return svo->n[level];
}

wfpg_status svo_export_level(const wfpg_svo *svo, int32_t level, uint32_t *keys, float *normals,
                             float *exitance, void *hip_stream)
{
    if (!svo || level < 0 || level > svo->depth) return WFPG_EINVAL;
    const int64_t m = svo->n[level], off = svo->noff[level];
    if (m == 0) return WFPG_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
    if (keys) e = hipMemcpyAsync(keys, svo->d_keys + off, m * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    std::vector<float4> nb;
    if (e == hipSuccess && normals) {
        nb.resize((size_t)m);
        e = hipMemcpyAsync(nb.data(), svo->d_nrm + off, m * sizeof(float4), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess && exitance)
        e = hipMemcpyAsync(exitance, svo->d_e32 + off, m * sizeof(float2), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && normals)
        for (int64_t i = 0; i < m; ++i) {
            normals[3 * i] = nb[(size_t)i].x;
            normals[3 * i + 1] = nb[(size_t)i].y;
            normals[3 * i + 2] = nb[(size_t)i].z;
        }
    return from_hip(e);
}

wfpg_status svo_export_accum(const wfpg_svo *svo, float *sums, uint32_t *counts, void *hip_stream)
{
    if (!svo) return WFPG_EINVAL;
    const int64_t L = svo->n[svo->depth];
    if (L == 0) return WFPG_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
    if (sums) e = hipMemcpyAsync(sums, svo->d_sum, L * sizeof(float2), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && counts)
        e = hipMemcpyAsync(counts, svo->d_cnt, L * sizeof(uint2), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return from_hip(e);
}

const char *wfpg_last_error(void)
{
    return g_last_error;
}

wfpg_status wfpg_dir_table(int32_t N, float *out)
{
    if (!out || (N != 8 && N != 16 && N != 32 && N != 64 && N != 128)) return WFPG_EINVAL;
    host_dir_table(N, out);
    return WFPG_OK;
}

wfpg_status wfpg_dir_table_jitter(int32_t N, uint32_t jitter_key, float *out)
{
    if (!out || (N != 8 && N != 16 && N != 32 && N != 64 && N != 128)) return WFPG_EINVAL;
    const size_t bytes = (size_t)N * N * 3 * sizeof(float);
    float *d = nullptr;
    hipError_t e = hipMalloc((void **)&d, bytes);
    if (e != hipSuccess) return from_hip(e);
    e = wfpg::launch_jitter_table(N, jitter_key, d, 0);
    if (e == hipSuccess) e = hipMemcpy(out, d, bytes, hipMemcpyDeviceToHost);
    const hipError_t f = hipFree(d);
    return from_hip(e != hipSuccess ? e : f);
}

}  // extern "C"

// ----------------------------------------------------------------------------
// guide_sample without allocation. Its scratch is a file-scope device array:
// the bin-direction tables of N = 8, 16 and 32 (FP32, three per bin, as
// host_dir_table computes them) and the vertex-queue counter of the guide
// kernel. Host code never passes the array's name to the device; it uses the
// address hipGetSymbolAddress returns, taken once per device.
namespace {

constexpr size_t kNaTabFloats[3] = {8 * 8 * 3, 16 * 16 * 3, 32 * 32 * 3};
constexpr size_t kNaTabOff[3] = {0, 8 * 8 * 3, 8 * 8 * 3 + 16 * 16 * 3};   // floats
constexpr size_t kNaCounterOff = 16384;                                  // bytes (tables: 16128)
constexpr size_t kNaScratchBytes = kNaCounterOff + kQueueRanges * kQueueStride * 8;
static_assert((kNaTabOff[2] + kNaTabFloats[2]) * sizeof(float) <= kNaCounterOff, "tables overlap the counters");

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

std::mutex g_na_mu;
unsigned char *g_na_ptr[64] = {};   // device address of `scratch`, per device
float g_na_host[(kNaTabOff[2] + kNaTabFloats[2])];

// Device address of the scratch array on the current device; on the first
// call for a device, looks it up and uploads the direction tables
// (synchronously, with that device current).
hipError_t noalloc_scratch(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return note_error(e, __FILE__, __LINE__);
        for (int k = 0; k < 3; ++k) host_dir_table(8 << k, g_na_host + kNaTabOff[k]);
        e = hipMemcpy(ptr, g_na_host, sizeof g_na_host, hipMemcpyHostToDevice);
        if (e != hipSuccess) return note_error(e, __FILE__, __LINE__);
        g_na_ptr[dev] = (unsigned char *)ptr;
    }
    *out = g_na_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" wfpg_status guide_sample_noalloc(const wfpg_svo *svo, const float *pos, int64_t n, uint64_t seed,
                                            uint32_t bounce, const wfpg_opts *opts, float *dir_out,
                                            float *pdf_out, void *hip_stream)
{
    if (!svo || n < 0 || !valid_opts(opts) || (n > 0 && (!pos || !dir_out || !pdf_out)))
        return WFPG_EINVAL;
    if (opts->mode != 0) return WFPG_EUNSUPPORTED;   // the learned form keeps working buffers
    if (n == 0) return WFPG_OK;
    unsigned char *sp = nullptr;
    const hipError_t e = noalloc_scratch(&sp);
    if (e != hipSuccess) return from_hip(e);
    GuideArgs a = base_args(svo, opts, false);
    const int k = opts->N == 8 ? 0 : (opts->N == 16 ? 1 : 2);
    a.dirtab = reinterpret_cast<const float *>(sp) + kNaTabOff[k];
    a.queue_ctr = reinterpret_cast<unsigned long long *>(sp + kNaCounterOff);   // the counters, reset by the launch
    a.pos = pos;
    a.n = n;
    a.seed = seed;
    a.bounce = bounce;
    a.dir_out = dir_out;
    a.pdf_out = pdf_out;
    return from_hip(launch_guide(svo, opts->N, MODE_SAMPLE, a, choose_tile(svo, opts->N),
                                 (hipStream_t)hip_stream));
}

namespace wfpg {

hipError_t launch_jitter_table(int N, uint32_t key, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_jitter_table, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, s, N, key, out);
    return hipGetLastError();
}

}  // namespace wfpg
