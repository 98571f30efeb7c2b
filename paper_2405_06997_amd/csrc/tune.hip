// Autotuner of the guide kernel's launch shape (waves per block, persistent
// grid size), cached per (device, N, depth, format).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "wfpg_internal.h"

namespace wfpg {
namespace {

using Key = std::tuple<int, int, int, int>;   // device, N, depth, fmt
std::mutex g_mu;
std::map<Key, TileConfig> g_cache;

Key key_of(const wfpg_svo *svo, int N)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    return Key(dev, N, svo->depth, svo->fmt);
}

TileConfig default_tile(int N, int depth)
{
    // the tuner's usual picks on the frame-scale room: 24 waves per CU (six
    // per SIMD, what the guide kernel's registers allow); at N = 16 in two
    // blocks, whose two copies of the direction tables leave the LDS for
    // five vertex slots per wave
    TileConfig t;
    t.waves_per_block = N == 16 ? 12 : 4;
    t.blocks_per_cu = N == 16 ? 2 : (N == 32 ? 4 : 6);
    return legalize_tile(t, N, depth);
}

}  // namespace

size_t guide_max_lds()
{
    static std::mutex mu;
    static std::map<int, size_t> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 64 * 1024;
    // dynamic LDS only: the guide kernel's static LDS (its argument copies)
    // must fit beside it
    const size_t dyn = (size_t)v - kGuideStaticLds;
    cache[dev] = dyn;
    return dyn;
}

TileConfig legalize_tile(TileConfig t, int N, int depth)
{
    t.waves_per_block = std::min(std::max(t.waves_per_block, 1), 16);
    t.blocks_per_cu = std::min(std::max(t.blocks_per_cu, 1), 64);
    (void)depth;
    while (t.waves_per_block > 1 && guide_lds_bytes(N, t) > guide_max_lds()) --t.waves_per_block;
    return t;
}

TileConfig choose_tile(const wfpg_svo *svo, int N)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_cache.find(key_of(svo, N));
    if (it != g_cache.end()) return it->second;
    return default_tile(N, svo->depth);
}

}  // namespace wfpg

using namespace wfpg;

extern "C" {

wfpg_status wfpg_get_tile(const wfpg_svo *svo, int32_t N, wfpg_tile *out)
{
    if (!svo || !out || (N != 8 && N != 16 && N != 32)) return WFPG_EINVAL;
    const TileConfig t = choose_tile(svo, N);
    out->waves_per_block = t.waves_per_block;
    out->blocks_per_cu = t.blocks_per_cu;
    return WFPG_OK;
}

wfpg_status wfpg_set_tile(const wfpg_svo *svo, int32_t N, const wfpg_tile *tile)
{
    if (!svo || !tile || (N != 8 && N != 16 && N != 32)) return WFPG_EINVAL;
    TileConfig t;
    t.waves_per_block = tile->waves_per_block;
    t.blocks_per_cu = tile->blocks_per_cu;
    if (t.waves_per_block < 1 || t.waves_per_block > 16 || t.blocks_per_cu < 1 || t.blocks_per_cu > 64 ||
        guide_lds_bytes(N, t) > guide_max_lds())
        return WFPG_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    g_cache[key_of(svo, N)] = t;
    return WFPG_OK;
}

wfpg_status wfpg_autotune(wfpg_svo *svo, const float *pos, int64_t n, int32_t N, int32_t reps,
                          void *hip_stream, wfpg_tile *best_out, float *best_ms)
{
    if (!svo || !pos || n <= 0 || reps < 1 || (N != 8 && N != 16 && N != 32)) return WFPG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    float *d_dir = nullptr, *d_pdf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&d_dir, (size_t)n * 3 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&d_pdf, (size_t)n * sizeof(float));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const float *tab = device_dirtab(N);
    TileConfig best = default_tile(N, svo->depth);
    float best_t = 1e30f;
    if (e == hipSuccess && tab) {
        GuideArgs a;
        std::memset(&a, 0, sizeof a);
        const double pi = 3.14159265358979323846;
        a.pos = pos;
        a.n = n;
        a.eps = 0.01f;
        a.omega = (float)(4.0 * pi / (double)(N * N));
        a.pdf_scale = (float)((double)(N * N) / (4.0 * pi));
        a.dirtab = tab;
        a.err = svo->d_err;
        a.dir_out = d_dir;
        a.pdf_out = d_pdf;
        const int waves[] = {1, 2, 3, 4, 6, 8, 12, 16};
        const int bpcu[] = {1, 2, 3, 4, 6, 8, 12, 16};
        std::vector<TileConfig> cand;
        for (int w : waves)
            for (int b : bpcu) {
                TileConfig t;
                t.waves_per_block = w;
                t.blocks_per_cu = b;
                // at least 4 and at most 32 waves per CU: fewer cannot hide the
                // march's memory latency, more cannot be resident
                if (guide_lds_bytes(N, t) > guide_max_lds() || w * b > 32 || w * b < 4) continue;
                cand.push_back(t);
            }
        for (const TileConfig &t : cand) {
            e = launch_guide(svo, N, MODE_SAMPLE, a, t, s);   // warm-up
            if (e != hipSuccess) break;
            std::vector<float> ts;
            for (int r = 0; r < reps && e == hipSuccess; ++r) {
                e = hipEventRecord(e0, s);
                if (e == hipSuccess) e = launch_guide(svo, N, MODE_SAMPLE, a, t, s);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                ts.push_back(ms);
            }
            if (e != hipSuccess) break;
            std::sort(ts.begin(), ts.end());
            const float med = ts[ts.size() / 2];
            if (std::getenv("WFPG_TUNE_VERBOSE"))
                std::fprintf(stderr, "tune N=%d waves=%d blocks/CU=%d: %.3f ms\n", N, t.waves_per_block,
                             t.blocks_per_cu, med);
            if (med < best_t) { best_t = med; best = t; }
        }
    }
    if (d_dir) (void)hipFree(d_dir);
    if (d_pdf) (void)hipFree(d_pdf);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return note_error(e, __FILE__, __LINE__) == hipErrorOutOfMemory ? WFPG_ENOMEM : WFPG_EDEVICE;
    if (!tab) return WFPG_ENOMEM;
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_cache[key_of(svo, N)] = best;
    }
    if (best_out) {
        best_out->waves_per_block = best.waves_per_block;
        best_out->blocks_per_cu = best.blocks_per_cu;
    }
    if (best_ms) *best_ms = best_t;
    return WFPG_OK;
}

wfpg_status wfpg_autotune_n(wfpg_svo *svo, const float *pos, int64_t n, int32_t reps,
                            float budget_ns_per_vertex, void *hip_stream, int32_t *N_out,
                            wfpg_tile *tile_out, float *ms_per_N)
{
    if (!svo || !pos || n <= 0 || reps < 1 || !N_out || !(budget_ns_per_vertex >= 0.f))
        return WFPG_EINVAL;
    const int Ns[3] = {8, 16, 32};
    float ms[3];
    wfpg_tile tiles[3];
    for (int k = 0; k < 3; ++k) {
        const wfpg_status st = wfpg_autotune(svo, pos, n, Ns[k], reps, hip_stream, &tiles[k], &ms[k]);
        if (st != WFPG_OK) return st;
        if (ms_per_N) ms_per_N[k] = ms[k];
    }
    int pick = 0;   // the finest field whose time per vertex fits the budget, else the coarsest
    for (int k = 2; k >= 0; --k)
        if ((double)ms[k] * 1e6 / (double)n <= (double)budget_ns_per_vertex) { pick = k; break; }
    *N_out = Ns[pick];
    if (tile_out) *tile_out = tiles[pick];
    return WFPG_OK;
}

}  // extern "C"
