// Internal declarations of the wavefront path-guiding library (gfx950).
//
// SVO layout in device memory (depth D <= 10):
//  * occupancy: one dense bitmap per level l, 8^l bits in Morton order, packed
//    into 64-bit words (a word is one 4x4x4 brick of level l, i.e. two levels
//    of the tree below one level-(l-2) node). Level l starts at word
//    woff(l) of one shared array; levels 0..2 take one word each.
//  * rank: per word, the global index of the first node stored in that word
//    (level node offset + popcount of all earlier words of the level). The
//    index of node `key` at level l is rank[woff(l) + key/64] +
//    popcount(word & ((1 << key%64) - 1)). Nodes of all levels share one
//    index space, level 0 first.
//  * per node: keys (uint32 Morton), normal (float4, w unused), exitance
//    (float2, FP32 value of side 0 / side 1) and, for 16-bit storage, the two
//    sides packed into one uint32 (side 0 in the low half).
//  * per leaf: splat sums (float2) and counts (uint2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "../../include/wfpg.h"

#define WFPG_MAXD 10
#define WFPG_FINE 30

namespace wfpg {

// Word offset of level l in the shared bitmap/rank arrays.
__host__ __device__ constexpr uint64_t level_words(int l)
{
    return l <= 2 ? 1ull : (1ull << (3 * l - 6));
}
__host__ __device__ constexpr uint64_t level_woff(int l)
{
    uint64_t o = 0;
    for (int m = 0; m < l; ++m) o += level_words(m);
    return o;
}

// Read-only view of an SVO handed to kernels by value.
struct SvoView {
    const uint64_t *bits;
    const uint32_t *rank;
    const uint32_t *keys;
    const float4 *nrm;
    const float2 *e32;
    const uint32_t *e16;
    int64_t noff[WFPG_MAXD + 2];  // first node index of each level
    int depth;
    int fmt;
};

struct RectCells {   // voxelized extent of one rectangle (host computed)
    int32_t axis, ca;       // plane axis and its cell index
    int32_t a0, a1, b0, b1; // inclusive cell ranges along the two other axes
    int32_t cls;            // normal class: axis * 2 + (sign > 0)
    int32_t emissive;
};

// Launchers (one translation unit each, enqueued on `s`).
hipError_t launch_build(struct ::wfpg_svo *svo, const RectCells *d_rects, const int64_t *d_foff,
                        int64_t n_rects, int64_t n_frag, hipStream_t s);
hipError_t launch_accumulate(struct ::wfpg_svo *svo, const float *pos, const float *wo,
                             const float *rgb, int64_t n, hipStream_t s);
hipError_t launch_accumulate_paths(struct ::wfpg_svo *svo, const float *pos, const float *T, const float *eye,
                                   const int32_t *hit, const float *Le, int64_t P, int d, hipStream_t s);
hipError_t launch_propagate(struct ::wfpg_svo *svo, hipStream_t s);

enum GuideMode {
    MODE_SAMPLE = 0, MODE_PDF = 1, MODE_EVAL = 2, MODE_DEBUG = 3, MODE_COUNT = 4,
    MODE_PRODUCT = 5,   // product guiding sample (Sec. 3.6)
    MODE_PEVAL = 6,     // product guiding pdf of given directions
    MODE_COUNT_OF_MODES = 7
};

struct GuideArgs {
    const float *pos;
    const float *dir_in;      // MODE_EVAL
    int64_t n;                // queue length (ignored when n_dev != NULL)
    const int64_t *n_dev;     // optional device-resident queue length
    int64_t stride;           // distance between SoA planes (0: the queue length)
    float eps;
    float omega;              // fp32(4*pi/N^2)
    float pdf_scale;          // fp32(N^2/(4*pi))
    uint64_t seed;
    uint32_t bounce;
    float *dir_out;
    float *pdf_out;
    int32_t *dbg_out;
    int32_t *dbg_visits;
    const float *dirtab;      // N*N*3 FP32 bin centres
    int32_t *err;             // device error flags
    unsigned long long *queue_ctr;   // kQueueRanges vertex-queue counters (reset before each launch)
    const int32_t *gate;             // optional: the kernel does nothing unless *gate != 0
    const float *nrm_in;      // product modes: SoA normals (Lambertian table) or NULL
    const float *bsdf_in;     // product modes: n x 64 BSDF tables or NULL
    const float *dirtab8;     // product modes: the 8 x 8 cell-centre directions
    int32_t jitter;           // cone directions jittered in their bins (key jitter_key)
    uint32_t jitter_key;
    int32_t blur;             // Gaussian blur of the field before the CDF
};

struct TileConfig {          // launch shape chosen by the autotuner
    int waves_per_block;     // 1 .. 16
    int blocks_per_cu;       // persistent grid size factor
};

hipError_t launch_guide(const struct ::wfpg_svo *svo, int N, int mode, const GuideArgs &a,
                        const TileConfig &tc, hipStream_t s);

// LDS bytes of one guide block: bin directions and the per-wave hit records.
// Query vertices a wave keeps in flight (hit records of each in LDS). A slot
// stays taken until the last ray of its vertex ends, so with few slots a wave
// runs out of bins to hand out while its slots drain; as many as the LDS holds
// at six waves per SIMD (1 KiB of records per slot at N = 16, 256 B at N = 8;
// 768 B at N = 16 with 3-byte records, one slot fewer where the wave also
// holds a field buffer).
__host__ __device__ constexpr int guide_slots(int N, bool r24 = false, bool field = false)
{
    return N >= 32 ? 2 : (N == 16 ? (r24 ? (field ? 6 : 7) : 5) : 8);
}

// With 3-byte records a slot cannot hold the field the blur and the product
// modes build in the finalization (N*N floats): those take a per-wave field
// buffer of their own (32-bit words).
__host__ __device__ constexpr bool guide_field_buffer(int mode, bool blur, bool r24)
{
    return r24 && (blur || mode == MODE_PRODUCT || mode == MODE_PEVAL);
}

// 32-bit words of one bin's hit record: the debug mode keeps the raw
// traversal record, every other mode the footprint node only.
__host__ __device__ constexpr int guide_rec_words(int mode) { return mode == MODE_DEBUG ? 2 : 1; }

// 32-bit words of one slot's records: with r24 a record is the footprint
// node's index + 1 (0: miss) in 3 bytes, a 16-bit and an 8-bit array of NN.
__host__ __device__ constexpr int guide_slot_words(int N, int mode, bool r24)
{
    return r24 ? 3 * N * N / 4 : guide_rec_words(mode) * N * N;
}

// 3-byte records: at N = 16 in every mode but debug and counting, for SVOs
// whose node indices + 1 fit 24 bits.
inline bool guide_use_r24(int N, int mode, int64_t total_nodes)
{
    return N == 16 && mode != MODE_DEBUG && mode != MODE_COUNT && total_nodes < (int64_t)0xffffff;
}

inline size_t guide_lds_bytes(int N, const TileConfig &tc, int mode = MODE_SAMPLE, bool r24 = false,
                              bool blur = false)
{
    const bool field = guide_field_buffer(mode, blur, r24);
    const size_t S = (size_t)guide_slots(N, r24, field), NN = (size_t)N * N;
    return NN * 3 * 4 * 2 +
           (size_t)tc.waves_per_block * (S * ((size_t)guide_slot_words(N, mode, r24) * 4 + 8) +   // records, counts
                                         S * (NN / 64) * 8 + 64 * 2 +                            // bin masks, exchange
                                         S * 8 + 4 * 4 +                                         // slot vertices, origin
                                         (field ? NN * 4 : 0));                                  // field buffer
}
// Dynamic LDS a guide workgroup may use on the current device (all modes but
// debug): the device's per-workgroup LDS less kGuideStaticLds, a bound on the
// kernel's static LDS (checked at compile time in the kernel's source).
constexpr size_t kGuideStaticLds = 1024;
size_t guide_max_lds();
constexpr int kCounterPool = 64;   // concurrent guide launches per SVO with distinct counters
// The guide kernel splits its vertex queue into this many contiguous ranges,
// one per XCD (workgroups are dispatched to the XCDs round robin, so
// workgroup b runs on XCD b mod 8), each with its own counter: the vertices
// one XCD works on at a time are neighbours in the queue (neighbouring
// pixels of a camera queue), whose rays read the same occupancy words, so
// its L2 and its CUs' L1s see a narrow front of the queue instead of a
// slice of every XCD's. A workgroup takes from its own range first, then
// from the others in turn; results do not depend on the order. The counters
// sit kQueueStride words apart, each on its own 128-byte line (sharing one
// line, the XCDs' atomics on it contended).
constexpr int kQueueRanges = 8;
constexpr int kQueueStride = 16;

// Tile chosen for (device, N, depth, format): the autotuned one if present.
TileConfig choose_tile(const struct ::wfpg_svo *svo, int N);
TileConfig legalize_tile(TileConfig t, int N, int depth);

int device_cu_count();
void destroy_model(void *model);
void destroy_bin_work(void *work);
wfpg_status learned_sample(const struct ::wfpg_svo *svo, const float *pos, const float *nrm, int64_t n,
                           uint64_t seed, uint32_t bounce, const wfpg_opts *o, float *dir_out,
                           float *pdf_out, hipStream_t s);
// Records a failing HIP call (thread-local) for wfpg_last_error().
hipError_t note_error(hipError_t e, const char *file, int line);
#define WFPG_HIP_TRY(x)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) return ::wfpg::note_error(e_, __FILE__, __LINE__);             \
    } while (0)
const float *device_dirtab(int N);   // uploaded once per N per device
// The jittered cone directions of key `key` (N*N*3 FP32, device), on `s`.
hipError_t launch_jitter_table(int N, uint32_t key, float *out, hipStream_t s);
void host_dir_table(int N, float *out);

}  // namespace wfpg

// Host-side object behind the opaque handle.
struct wfpg_svo {
    int depth = 0, fmt = 0, device = 0;
    int64_t n[WFPG_MAXD + 1] = {};
    int64_t noff[WFPG_MAXD + 2] = {};
    int64_t total_nodes = 0;
    uint64_t total_words = 0;
    uint64_t *d_bits = nullptr;
    uint32_t *d_rank = nullptr;
    uint32_t *d_keys = nullptr;
    float4 *d_nrm = nullptr;
    float2 *d_e32 = nullptr;
    uint32_t *d_e16 = nullptr;
    float2 *d_sum = nullptr;
    uint2 *d_cnt = nullptr;
    unsigned long long *d_dropped = nullptr;
    int32_t *d_err = nullptr;
    unsigned long long *d_ctr = nullptr;   // pool of vertex-queue counters
    void *nn_model = nullptr;              // learned stand-in (nn.hip), created on demand
    mutable void *bin_work = nullptr;      // scratch of the binned path (binning.hip)
    mutable std::atomic<unsigned> ctr_next{0};   // round-robin slot of the pool
    wfpg::SvoView view() const
    {
        wfpg::SvoView v;
        v.bits = d_bits; v.rank = d_rank; v.keys = d_keys; v.nrm = d_nrm;
        v.e32 = d_e32; v.e16 = d_e16; v.depth = depth; v.fmt = fmt;
        for (int i = 0; i < WFPG_MAXD + 2; ++i) v.noff[i] = noff[i];
        return v;
    }
};
