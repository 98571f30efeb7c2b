// Batched bounces (the per-depth loop of Alg. 1 over a wavefront): one
// guide_sample per bounce over queues whose lengths live in device memory,
// captured once into a HIP graph and replayed. The guide kernels are
// persistent (grid sized to the GPU) and read their queue length when they
// run, so a replay after the lengths changed needs no re-instantiation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "wfpg_internal.h"

using namespace wfpg;

struct wfpg_bounce_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long *d_ctr = nullptr;   // the queue counters of each bounce
};

namespace {
void free_graph(wfpg_bounce_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->d_ctr) (void)hipFree(g->d_ctr);
    delete g;
}
}  // namespace

extern "C" {

wfpg_status wfpg_graph_create(const wfpg_svo *svo, int32_t n_bounces, const float *const *pos,
                              const int64_t *capacity, const int64_t *n_dev, const int32_t *N,
                              uint64_t seed, float eps, float *const *dir_out,
                              float *const *pdf_out, void *hip_stream, wfpg_bounce_graph **out)
{
    if (!out) return WFPG_EINVAL;
    *out = nullptr;
    if (!svo || n_bounces < 1 || n_bounces > 64 || !pos || !capacity || !n_dev || !N || !dir_out ||
        !pdf_out || !std::isfinite(eps) || !(eps > 0.f))
        return WFPG_EINVAL;
    for (int b = 0; b < n_bounces; ++b) {
        if (!pos[b] || !dir_out[b] || !pdf_out[b] || capacity[b] < 0) return WFPG_EINVAL;
        if (N[b] != 8 && N[b] != 16 && N[b] != 32) return WFPG_EINVAL;
        if (!device_dirtab(N[b])) return WFPG_ENOMEM;   // allocate before capture
    }
    wfpg_bounce_graph *g = new (std::nothrow) wfpg_bounce_graph();
    if (!g) return WFPG_ENOMEM;
    hipStream_t user = (hipStream_t)hip_stream;
    hipStream_t cs = nullptr;
    hipError_t e = hipMalloc((void **)&g->d_ctr, (size_t)n_bounces * kQueueRanges * kQueueStride * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamSynchronize(user);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const double pi = 3.14159265358979323846;
        for (int b = 0; b < n_bounces && e == hipSuccess; ++b) {
            GuideArgs a;
            std::memset(&a, 0, sizeof a);
            a.pos = pos[b];
            a.n = 0;
            a.n_dev = n_dev + b;
            a.stride = capacity[b];
            a.eps = eps;
            a.omega = (float)(4.0 * pi / (double)(N[b] * N[b]));
            a.pdf_scale = (float)((double)(N[b] * N[b]) / (4.0 * pi));
            a.seed = seed;
            a.bounce = (uint32_t)b;
            a.dir_out = dir_out[b];
            a.pdf_out = pdf_out[b];
            a.dirtab = device_dirtab(N[b]);
            a.err = svo->d_err;
            a.queue_ctr = g->d_ctr + (size_t)kQueueRanges * kQueueStride * b;
            e = launch_guide(svo, N[b], MODE_SAMPLE, a, choose_tile(svo, N[b]), cs);
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
        g->graph = graph;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        (void)note_error(e, __FILE__, __LINE__);
        (void)hipGetLastError();
        free_graph(g);
        return e == hipErrorOutOfMemory ? WFPG_ENOMEM : WFPG_EDEVICE;
    }
    *out = g;
    return WFPG_OK;
}

wfpg_status wfpg_graph_launch(wfpg_bounce_graph *g, void *hip_stream)
{
    if (!g || !g->exec) return WFPG_EINVAL;
    const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
        (void)note_error(e, __FILE__, __LINE__);
        return WFPG_EDEVICE;
    }
    return WFPG_OK;
}

void wfpg_graph_destroy(wfpg_bounce_graph *g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();
    free_graph(g);
}

}  // extern "C"
