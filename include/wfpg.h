/*
 * wfpg.h -- C ABI of the wavefront path-guiding library for AMD Instinct
 * MI355X (gfx950).
 *
 * The library implements the guiding hot path of Yalciner & Akyuz, "Path
 * Guiding for Wavefront Path Tracing: A Memory Efficient Approach for GPU Path
 * Tracers" (2024): a sparse voxel octree (SVO) caches radiant exitance
 * (Sec. 3.2); at a path vertex an N x N field of equal solid-angle directions
 * (Sec. 3.3) is traced through the SVO, turned into a piecewise-constant PDF
 * and CDF (Sec. 3.5, Alg. 3) and sampled.
 *
 * Conventions shared by every entry point:
 *  - World space is the unit cube [0,1]^3. Positions outside it are invalid
 *    for guiding and are dropped by svo_accumulate.
 *  - Device arrays are caller-owned, FP32, structure-of-arrays: a "3 x n"
 *    array holds n x-values, then n y-values, then n z-values, contiguous.
 *  - Every call validates its arguments synchronously and returns a negative
 *    wfpg_status on error, without touching any device memory. Work is
 *    enqueued asynchronously on the given HIP stream (NULL = default stream);
 *    a device fault surfaces as WFPG_EDEVICE from a later call or from
 *    svo_stats. n == 0 is a no-op that returns WFPG_OK. No C++ exception
 *    crosses this interface. No function keeps a caller pointer after it
 *    returns.
 *  - Directions are unit vectors in world space: the field is omnidirectional
 *    (Sec. 3.7 / Fig. 5 discussion), mapped to the square by the equal-area
 *    concentric octahedral map (Sec. 4, "Radiance field projection"), square
 *    centre = +z. Bin (u, v) covers x in [u/N, (u+1)/N), y in [v/N, (v+1)/N);
 *    rows are v and the flat bin index is b = v*N + u.
 *  - Returned pdfs are solid-angle densities in 1/sr (Eq. 2).
 *  - Concurrency: guide_pdf, guide_sample (mode 0), pdf_eval and
 *    wfpg_debug_march only read the SVO and may run concurrently;
 *    svo_accumulate mutates it, and guide_train, the wfpg_nn_* calls and
 *    guide_sample in mode 1 use the model's working buffers: the caller
 *    orders those (stream order).
 */
#ifndef WFPG_H
#define WFPG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wfpg_svo wfpg_svo; /* opaque; owns all of its device memory */
typedef int32_t wfpg_status;

enum {
    WFPG_OK = 0,
    WFPG_EINVAL = -1,      /* invalid argument */
    WFPG_ENOMEM = -2,      /* device or host allocation failed */
    WFPG_EDEVICE = -3,     /* HIP runtime error or device-side fault */
    WFPG_ESTATE = -4,      /* call not valid in the object's current state */
    WFPG_EUNSUPPORTED = -5 /* valid request the library does not support */
};

/* Storage format of the exitance and of the field bins (the CDF and pdf are
 * always accumulated in FP32). */
enum { WFPG_FP32 = 0, WFPG_FP16 = 1, WFPG_BF16 = 2 };

/* Axis-aligned rectangle: the plane x[axis] == c, spanning [lo[k], hi[k]]
 * along the other two axes taken in increasing order; normal sign * e_axis.
 * emissive != 0 marks light sources (used only for statistics). */
typedef struct {
    int32_t axis;   /* 0, 1 or 2 */
    float c;
    float lo[2], hi[2];
    int32_t sign;   /* +1 or -1 */
    int32_t emissive;
} wfpg_rect;

/* Per-call guiding options.
 *  N        -- bins per side of the direction field: 8, 16 or 32.
 *  eps      -- value added to every bin (Sec. 4, "PDF domains": the field
 *              starts at a nonzero value so the pdf is positive wherever
 *              radiance may arrive); finite and > 0. Default 0.01.
 *  mode     -- 0: SVO march. 1: learned model with march fallback
 *              (requires guide_train first).
 *  kl_bound -- fallback threshold in nats for mode 1 (default 0.05).
 *  probe_stride -- every probe_stride-th vertex is also marched to judge the
 *              learned model in mode 1 (default 256).
 *  jitter, jitter_key -- field antialiasing (Sec. 4, "aliasing"): with
 *              jitter = 1 the cone of bin b = v*N + u runs along the decode
 *              of ((u + j_u)/N, (v + j_v)/N) instead of the bin centre, with
 *              (j_u, j_v) = words 0 and 1 of Philox-4x32-10 at counter
 *              (b, 0, 0, 3), key (jitter_key, 0), each (bits >> 8) * 2^-24,
 *              decoded in FP64 and rounded to FP32. The caller picks a new
 *              key on the iterations it jitters; pdf_eval with the same
 *              options regenerates the same field. 0 or 1 (default 0).
 *  blur     -- 1: the field L (eps included) is blurred before the CDF with
 *              the 3 x 3 binomial kernel (1/4, 1/2, 1/4) per axis over the
 *              bins, in FP32, rows outer; neighbours across the edge of the
 *              octahedral square are the mirrored bins ((N, v) is
 *              (N - 1, N - 1 - v), (u, N) is (N - 1 - u, N - 1)), as the map
 *              joins them on the sphere. 0 or 1 (default 0).
 *  In mode 1 the judge's probes and the fallback march both use eps, jitter
 *  and blur as given here, so the judge measures the network against the
 *  very field the fallback would sample. */
typedef struct {
    int32_t N;
    float eps;
    int32_t mode;
    float kl_bound;
    int32_t probe_stride;
    int32_t jitter;
    uint32_t jitter_key;
    int32_t blur;
} wfpg_opts;

/* Default options {16, 0.01f, 0, 0.05f, 256, 0, 0, 0}. */
wfpg_opts wfpg_default_opts(void);

const char *wfpg_status_string(wfpg_status s);

/* ---------------------------------------------------------------------
 * svo_build -- SVO generation (Sec. 3.2: conservative voxelization of the
 * scene, a hierarchy from Morton-sorted voxel keys, and two normals per node
 * from k-means with k = 2, Fig. 2).
 *
 * rects, n_rects: HOST array of rectangles (read during the call only).
 * depth: leaf level D in [1, 10]; leaves are cells of size 2^-D.
 * exitance_fmt: WFPG_FP32, WFPG_FP16 or WFPG_BF16 (storage of the exitance
 *   read by the march and of the field bins).
 * Voxelization is half-open: along an in-plane axis a rectangle covers the
 *   cells whose [i, i+1) * 2^-D extent meets the open interval (lo, hi) (the
 *   single cell holding lo when lo == hi); along its plane axis the cell
 *   floor(c * 2^D), clamped to 2^D - 1.
 * Leaf normal: k-means (k = 2) over the fragment normals of the cell in
 *   rectangle order, seeded with the first fragment's normal and its
 *   opposite; inner-node normal: the same over the occupied children's
 *   normals in octant order. The node stores N and -N implicitly.
 * Errors: EINVAL for depth out of range, n_rects < 0, rects == NULL with
 *   n_rects > 0, axis not in {0,1,2}, sign not +-1, non-finite or lo > hi
 *   coordinates, an unknown format, out == NULL. ENOMEM if the device
 *   arrays cannot be allocated. On success *out owns the device memory;
 *   the call synchronizes the stream before returning.
 * ------------------------------------------------------------------- */
wfpg_status svo_build(const wfpg_rect *rects, int64_t n_rects, int32_t depth,
                      int32_t exitance_fmt, void *hip_stream, wfpg_svo **out);

/* Frees the SVO and its device memory (synchronizes the device). NULL is a
 * no-op. */
void svo_destroy(wfpg_svo *svo);

/* ---------------------------------------------------------------------
 * svo_accumulate -- UpdateExitance (Alg. 1; Sec. 3.2 after Eq. 5): each
 * path-vertex splat is mapped to its leaf and its local radiance estimate is
 * accumulated; then the exitance is averaged bottom-up through the tree.
 *
 * pos, wo, rgb: DEVICE 3 x n FP32 (SoA). pos in [0,1]^3; wo the unit
 *   direction the radiance leaves in (toward the previous path vertex); rgb
 *   the local radiance estimate (e.g. T_n/T_k * L_e, Eq. 5).
 * Per splat: y = Rec.709 luminance (0.2126 r + 0.7152 g) + 0.0722 b in FP32;
 *   leaf = cell of pos; side 0 iff dot(N_leaf, wo) >= 0 else 1; the leaf
 *   side's sum += y and count += 1 (FP32 / uint32 atomics, so sums of
 *   several splats depend on arrival order within FP32 rounding). Splats
 *   with a non-finite component, y < 0, or a position outside [0,1]^3 or in
 *   an empty leaf are dropped and counted (svo_stats). Sums persist across
 *   calls (progressive learning).
 * Then every node is rewritten: leaf side value = sum/count (0 with no
 *   splats); inner side value = mean, in octant order, over the occupied
 *   children of the child side facing the same way (child sides swapped
 *   when dot(N_child, N_parent) < 0), in FP32; stored rounded once (RNE) to
 *   the SVO's exitance format.
 * n == 0 still recomputes the averages.
 * Errors: EINVAL for NULL svo, n < 0, or NULL arrays with n > 0.
 * ------------------------------------------------------------------- */
wfpg_status svo_accumulate(wfpg_svo *svo, const float *pos, const float *wo,
                           const float *rgb, int64_t n, void *hip_stream);

/* ---------------------------------------------------------------------
 * svo_accumulate_paths -- UpdateExitance from path memory (Eq. 5): the
 * local radiance at every depth of the paths that reached an emitter,
 * splatted as svo_accumulate does, then averaged bottom-up.
 *
 * A wavefront of P paths stores, for each depth k = 1..d, the path vertex
 * p_k and the throughput T_k of its first k vertices (RGB):
 *   pos, T: DEVICE d planes of 3 x P FP32 SoA (plane k-1 at offset
 *           (k-1) * 3 * P);
 *   eye:    DEVICE 3 x P, p_0 of each path (its camera point);
 *   hit:    DEVICE P int32, the depth n in 1..d at which the path reached
 *           an emitter (any other value: no emitter, no splat);
 *   Le:     DEVICE 3 x P, the radiance that emitter sends toward p_{n-1}.
 * For k = 1..n the splat is: position p_k; outgoing direction
 * p_{k-1} - p_k (FP32, only its sign against the leaf normal matters);
 * rgb = (T_n / T_k) * Le per channel, FP32 correctly rounded, 0 where the
 * channel of T_k is 0. Drop rules, accumulation and propagation as
 * svo_accumulate. A path that reaches several emitters is passed once per
 * emitter.
 * Errors: EINVAL for NULL svo, P < 0, d < 1 or d > 64, or NULL arrays with
 * P > 0.
 * ------------------------------------------------------------------- */
wfpg_status svo_accumulate_paths(wfpg_svo *svo, const float *pos, const float *T, const float *eye,
                                 const int32_t *hit, const float *Le, int64_t P, int32_t d,
                                 void *hip_stream);

/* ---------------------------------------------------------------------
 * guide_pdf -- the per-vertex guiding PDF (Alg. 3, ConeTrace for every
 * direction patch, then GeneratePDF-CDF), written out in full.
 *
 * For vertex i (pos DEVICE 3 x n) and bin b with centre direction d_b:
 *  - quantize: O = clamp(rint(p * 2^30), 0, 2^30 - 1), q = rint(d_b * 2^23);
 *  - march: the first occupied leaf, other than the one holding p, met by
 *    the exact 6-connected traversal of the ray (crossings compared exactly,
 *    ties stepping the lowest axis first); leaving the cube is a miss;
 *  - footprint (Eq. 7): r = distance to the hit leaf's entry point in leaf
 *    units (FP32), A = r^2 * 4*pi/N^2, ascend k = #{j in 1..D : A >
 *    2.5 * 4^(j-1)} levels to the node whose area is closest to A;
 *  - value: side 0 iff dot(N_node, d_b) < 0 (FP32, fixed order), L_b =
 *    E[node][side] + eps; a miss gives eps;
 *  - pdf_b = L_b / sum_b' L_b' * N^2 / (4*pi).
 * pdf_out: DEVICE n * N * N FP32, row-major [i][v][u].
 * Errors: EINVAL for NULL svo/pos/opts/pdf_out with n > 0, n < 0, N not in
 *   {8, 16, 32}, eps not finite and > 0, mode != 0.
 * ------------------------------------------------------------------- */
wfpg_status guide_pdf(const wfpg_svo *svo, const float *pos, int64_t n,
                      const wfpg_opts *opts, float *pdf_out, void *hip_stream);

/* ---------------------------------------------------------------------
 * guide_sample -- one guided direction per vertex (Alg. 3 sampling step;
 * inverse-CDF sampling of the piecewise-constant 2D field, Sec. 3.5).
 *
 * The field of vertex i is built as in guide_pdf (never written to memory);
 * uniforms (u1..u4) come from Philox-4x32-10 with counter (i mod 2^32,
 * i >> 32, bounce, 0) and key (seed mod 2^32, seed >> 32), u = (bits >> 8)
 * * 2^-24. Row v: first with u1 * total < M_v (M: inclusive prefix of the
 * row sums); column u: first with u2 * rowsum_v < R_v[u] (R_v: inclusive
 * prefix of row v); both clamped to N - 1. Direction = octahedral decode of
 * ((u + u3)/N, (v + u4)/N); its pdf = pdf_b of bin (u, v).
 * nrm: DEVICE 3 x n surface normals; may be NULL unless opts->mode == 1.
 * dir_out: DEVICE 3 x n FP32; pdf_out: DEVICE n FP32.
 * Errors: as guide_pdf; mode 1 without a trained model is ESTATE.
 * ------------------------------------------------------------------- */
wfpg_status guide_sample(const wfpg_svo *svo, const float *pos, const float *nrm,
                         int64_t n, uint64_t seed, uint32_t bounce,
                         const wfpg_opts *opts, float *dir_out, float *pdf_out,
                         void *hip_stream);

/* ---------------------------------------------------------------------
 * guide_sample_noalloc -- guide_sample (mode 0) for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. It calls no hipMalloc, hipFree or
 * allocating library routine; the caller passes inputs and outputs as for
 * guide_sample and gets the same results bit for bit (same kernels).
 *
 * Its scratch is one static device array of 17,408 bytes per GPU, held
 * until the process ends: the bin-direction tables of N = 8, 16 and 32 and
 * the vertex-queue counters. The first call on a device, with that device
 * current, looks the array up and uploads the tables synchronously (make
 * that first call before capturing a graph); later calls only enqueue a
 * counter reset (a kernel, not a memset) and the guide kernel on the stream.
 * Every call on a GPU shares that array: calls that overlap on one GPU
 * (concurrent streams) race on the counters and must be ordered by the
 * caller.
 * Errors: as guide_sample; EINVAL for N beyond the tables (not 8, 16 or
 * 32); EUNSUPPORTED for mode 1 (the learned form keeps working buffers).
 * ------------------------------------------------------------------- */
wfpg_status guide_sample_noalloc(const wfpg_svo *svo, const float *pos, int64_t n, uint64_t seed,
                                 uint32_t bounce, const wfpg_opts *opts, float *dir_out,
                                 float *pdf_out, void *hip_stream);

/* ---------------------------------------------------------------------
 * pdf_eval -- guiding pdf of given directions (needed to weight guided
 * samples against BSDF and light samples with MIS, Sec. 4): the direction
 * is encoded with the octahedral map, its bin taken, and pdf_b returned;
 * the vertex's field is regenerated (nothing is stored between calls).
 * pos, dir: DEVICE 3 x n; pdf_out: DEVICE n.
 * Errors: as guide_pdf.
 * ------------------------------------------------------------------- */
wfpg_status pdf_eval(const wfpg_svo *svo, const float *pos, const float *dir,
                     int64_t n, const wfpg_opts *opts, float *pdf_out,
                     void *hip_stream);

/* ---------------------------------------------------------------------
 * guide_sample_product -- product path guiding (Sec. 3.6): the vertex's
 * field (as guide_pdf, never written to memory) times an 8 x 8 BSDF table,
 * sampled in two levels after the hierarchical product sampler the paper
 * adopts (Estevez and Kulla).
 *
 *  - Upper level: cell C = 8 V + U (rows V, the same octahedral square cut
 *    into 8 x 8) holds the s x s fine bins u in [U s, U s + s), v in
 *    [V s, V s + s), s = N / 8; F_C = their sum; P_C = F_C * f_C.
 *  - Table f_C: row i of bsdf (DEVICE n x 64 FP32, row-major [i][V][U]), or,
 *    when bsdf is NULL, the Lambertian cosine factor max(0, n_i . d_C) of the
 *    normal nrm (DEVICE 3 x n) and the cell-centre direction d_C (the N = 8
 *    bin centres), computed in FP32 as (n_x d_x + n_y d_y) + n_z d_z. Entries
 *    that are not > 0 count as 0. The normal should face the side the path
 *    continues on; it need not be unit length.
 *  - Uniforms: w1, w2 = words 0 and 1 of Philox-4x32-10 at counter (i_lo,
 *    i_hi, bounce, 2); u1..u4 as guide_sample (counter word 0).
 *  - Cell: row V from the product's row sums (target w1 * total), column U
 *    within the row (target w2 * rowsum); then the fine row dv and column du
 *    inside the cell from the field values (targets u1 * cell sum, u2 *
 *    row sum); each pick is the first entry whose inclusive CDF exceeds the
 *    target, else the last entry with positive mass. Direction = decode of
 *    ((U s + du + u3)/N, (V s + dv + u4)/N).
 *  - pdf = P_C / sum(P) * L_b / F_C * N^2 / (4 pi) (1/sr), the normalized
 *    product of the field with the table held constant over each cell.
 *  - A product whose total is 0 or not finite (zero or non-finite normal,
 *    all-zero table) is sampled with f = 1: plain guiding.
 * Exactly one of nrm, bsdf is given. dir_out DEVICE 3 x n, pdf_out DEVICE n.
 * Errors: as guide_pdf; EINVAL when both or neither of nrm, bsdf is given.
 * ------------------------------------------------------------------- */
wfpg_status guide_sample_product(const wfpg_svo *svo, const float *pos, const float *nrm,
                                 const float *bsdf, int64_t n, uint64_t seed, uint32_t bounce,
                                 const wfpg_opts *opts, float *dir_out, float *pdf_out,
                                 void *hip_stream);

/* pdf_eval_product -- the product pdf of given directions (for MIS): the
 * direction's fine bin (u, v), its cell C = (u / s, v / s), and the pdf of
 * guide_sample_product for that bin (bit-identical to what that call
 * returns for a direction it sampled). Arguments and errors as
 * guide_sample_product and pdf_eval. */
wfpg_status pdf_eval_product(const wfpg_svo *svo, const float *pos, const float *nrm,
                             const float *bsdf, const float *dir, int64_t n,
                             const wfpg_opts *opts, float *pdf_out, void *hip_stream);

/* ------------------------------------------------------------ auxiliaries */

/* Occupied leaves, all nodes and dropped splats so far; error_flags != 0
 * means a kernel hit an internal limit (the last results are invalid).
 * Any pointer may be NULL. Synchronizes the device. */
wfpg_status svo_stats(const wfpg_svo *svo, int64_t *leaves, int64_t *nodes,
                      int64_t *dropped_splats, int32_t *error_flags);

/* Number of nodes at a level (0 = root .. depth = leaves); -1 on error. */
int64_t svo_level_size(const wfpg_svo *svo, int32_t level);

/* Copies one level to HOST arrays (any may be NULL): sorted Morton keys
 * (x in bit 3i, y in 3i+1, z in 3i+2), normals (3 floats per node, AoS) and
 * the exitance of side 0 and 1 (2 floats per node, FP32 values before the
 * storage rounding). Synchronizes the stream. */
wfpg_status svo_export_level(const wfpg_svo *svo, int32_t level, uint32_t *keys,
                             float *normals, float *exitance, void *hip_stream);

/* Copies the leaf accumulators to HOST arrays (either may be NULL): per leaf
 * 2 FP32 sums and 2 uint32 counts (side 0, side 1). */
wfpg_status svo_export_accum(const wfpg_svo *svo, float *sums, uint32_t *counts,
                             void *hip_stream);

/* Name and source location of the last failing HIP call seen by the library
 * on this thread ("" if none); the string stays valid until the next failure
 * on the thread. */
const char *wfpg_last_error(void);

/* Host copy of the FP32 bin-centre direction table the kernels use for
 * resolution N in {8, 16, 32, 64, 128} (N*N*3 floats, AoS, bin b = v*N + u). */
wfpg_status wfpg_dir_table(int32_t N, float *out);

/* Host copy of the jittered cone directions the kernels compute for
 * jitter_key (see wfpg_opts.jitter), same layout as wfpg_dir_table.
 * Synchronizes the device. */
wfpg_status wfpg_dir_table_jitter(int32_t N, uint32_t jitter_key, float *out);

/* Test-only: the traversal record of every (vertex, bin) pair, for
 * bit-exact comparison with an independent implementation.
 * out: DEVICE n * N*N * 8 int32 = {hit, entry axis, leaf key, |B - O| of
 * the entry crossing (2^-30 units), footprint ascent k, node key, node index
 * within its level, side}; for a miss every field after hit is -1 except
 * side (0). visits: DEVICE n * N*N int32 (may be NULL): occupancy tests at
 * levels >= 5 of the traversal. */
wfpg_status wfpg_debug_march(const wfpg_svo *svo, const float *pos, int64_t n,
                             const wfpg_opts *opts, int32_t *out, int32_t *visits,
                             void *hip_stream);

/* ---------------------------------------------------------------------
 * Launch shape of the guide kernels and its autotuner. A tile is the number
 * of waves per workgroup (each wave keeps up to four vertices in flight) and
 * the persistent grid size in workgroups per compute unit. Tiles are cached
 * per (device, N, SVO depth, exitance format); guide_pdf, guide_sample,
 * pdf_eval use the cached tile or a default. Results never depend on the
 * tile.
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t waves_per_block;
    int32_t blocks_per_cu;
} wfpg_tile;

/* Current tile for resolution N. EINVAL for bad arguments. */
wfpg_status wfpg_get_tile(const wfpg_svo *svo, int32_t N, wfpg_tile *out);

/* Force a tile for resolution N (EINVAL if it exceeds the kernel's limits:
 * 1..16 waves, 1..64 blocks per CU, the device's LDS per workgroup less 1 KiB: 159 KiB
 * on MI355X). */
wfpg_status wfpg_set_tile(const wfpg_svo *svo, int32_t N, const wfpg_tile *tile);

/* Sweep candidate tiles for resolution N on the given DEVICE queue pos
 * (3 x n), time guide_sample with HIP events (median of reps), cache and
 * return the fastest (best_out, best_ms may be NULL). Allocates its own
 * scratch outputs; synchronizes the stream. */
wfpg_status wfpg_autotune(wfpg_svo *svo, const float *pos, int64_t n, int32_t N, int32_t reps,
                          void *hip_stream, wfpg_tile *best_out, float *best_ms);

/* Pick the field resolution for a queue: tunes the tile of every N in
 * {8, 16, 32} on the DEVICE queue pos (3 x n) as wfpg_autotune does, then
 * returns in *N_out the largest N whose best time per vertex is within
 * budget_ns_per_vertex (N = 8 if none is), its tile in tile_out (may be NULL)
 * and the best times of N = 8, 16, 32 in ms_per_N[3] (HOST, may be NULL).
 * Finer fields resolve the incident radiance better (Sec. 3.3) at a cost that
 * grows with N^2; the budget states what a bounce may spend per vertex. */
wfpg_status wfpg_autotune_n(wfpg_svo *svo, const float *pos, int64_t n, int32_t reps,
                            float budget_ns_per_vertex, void *hip_stream, int32_t *N_out,
                            wfpg_tile *tile_out, float *ms_per_N);

/* ---------------------------------------------------------------------
 * Batched bounces: the per-depth guiding of Alg. 1 for a whole wavefront
 * (one guide_sample per bounce), captured once into a HIP graph of
 * persistent kernels that read each bounce's queue length from device memory
 * at replay time, so lengths may change between replays without
 * re-instantiation.
 *  n_bounces in [1, 64]; the arrays below are HOST arrays of n_bounces.
 *  pos[b]: DEVICE 3 x capacity[b] SoA positions (plane stride capacity[b]).
 *  n_dev: DEVICE int64[n_bounces], current length of each queue
 *         (0 <= n_dev[b] <= capacity[b]; read when the graph runs).
 *  N[b] in {8, 16, 32}; eps as in wfpg_opts.
 *  dir_out[b] (3 x capacity[b], same stride), pdf_out[b] (capacity[b]):
 *         DEVICE outputs. Vertex i of bounce b draws its uniforms from
 *         Philox counter (i, bounce = b) and key seed, exactly as
 *         guide_sample(..., seed, b, ...) would.
 * The graph keeps the pointers; the caller keeps every buffer alive (and
 * the SVO unchanged in structure) until wfpg_graph_destroy. Replays that
 * overlap on the same graph race; launch them in stream order.
 * ------------------------------------------------------------------- */
typedef struct wfpg_bounce_graph wfpg_bounce_graph;

wfpg_status wfpg_graph_create(const wfpg_svo *svo, int32_t n_bounces, const float *const *pos,
                              const int64_t *capacity, const int64_t *n_dev, const int32_t *N,
                              uint64_t seed, float eps, float *const *dir_out,
                              float *const *pdf_out, void *hip_stream, wfpg_bounce_graph **out);

/* Replay the captured bounces on a stream. */
wfpg_status wfpg_graph_launch(wfpg_bounce_graph *g, void *hip_stream);

/* Free the graph (synchronizes the device). NULL is a no-op. */
void wfpg_graph_destroy(wfpg_bounce_graph *g);

/* Per-vertex work counts of the march, for measurement: counts (DEVICE
 * n x 2 int32) = {occupancy tests at levels >= 5 summed over the vertex's
 * N*N bins, number of bins that hit}. The same traversal as guide_sample. */
wfpg_status wfpg_march_counts(const wfpg_svo *svo, const float *pos, int64_t n,
                              const wfpg_opts *opts, int32_t *counts, void *hip_stream);

/* ---------------------------------------------------------------------
 * Positional binning and per-bin fields (Alg. 2 Partition-S, Sec. 3.4; Alg. 3
 * GuideRays with SelectOrigin). One field is generated per bin of nearby
 * queries instead of one per query.
 *  Partition-S: each query descends to the deepest existing SVO node that
 *  holds its quantized position (its leaf when occupied) and adds one to
 *  that node's count; bottom-up from the leaves to level l_min, a node's
 *  total T is its own count plus its children's totals, and the node is
 *  marked when T >= c_ray or it lies on level l_min (the leaf level takes
 *  part with T = its own count). A query's bin is the deepest marked node on
 *  its path to the root, the node itself included (a query whose node lies
 *  above l_min is its own bin).
 *  SelectOrigin: a random member of the bin, drawn as the member i with the
 *  smallest (h_i, i), h_i = first word of Philox-4x32-10 at counter (i_lo,
 *  i_hi, bounce, 1) and key (seed_lo, seed_hi).
 *  The N x N field of the bin is generated at its origin exactly as
 *  guide_pdf does for a vertex, and every member samples it with its own
 *  uniforms (counter (i_lo, i_hi, bounce, 0)) by the guide_sample rule.
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t N;       /* 8, 16, 32, 64 or 128 (16); 64 and 128 as the paper's per-bin fields */
    float eps;       /* as wfpg_opts (0.01) */
    int32_t c_ray;   /* queries that make a bin, >= 1 (512) */
    int32_t l_min;   /* coarsest bin level, 0..depth (5) */
    int32_t jitter;       /* as wfpg_opts: jittered cone directions of every bin field (0) */
    uint32_t jitter_key;  /* (0) */
    int32_t blur;         /* as wfpg_opts: blur every bin field before its CDF (0) */
} wfpg_bin_opts;

wfpg_bin_opts wfpg_default_bin_opts(void);

/* The bins alone: bin_out DEVICE n int32 = global node index of each query's
 * bin (levels are consecutive ranges of svo_level_size; -1 for an empty
 * SVO); origin_out DEVICE n int32 (may be NULL) = queue index of the bin's
 * origin. n < 2^31. Uses the SVO's binning scratch (calls on one SVO must be
 * stream-ordered). */
wfpg_status wfpg_partition(const wfpg_svo *svo, const float *pos, int64_t n, int32_t c_ray,
                           int32_t l_min, uint64_t seed, uint32_t bounce, int32_t *bin_out,
                           int32_t *origin_out, void *hip_stream);

/* Binned guide_sample: pos DEVICE 3 x n; dir_out DEVICE 3 x n, pdf_out DEVICE
 * n (pdf of the sampled direction under the member's bin field, 1/sr; 0 and
 * a zero direction for a query without a bin); bin_out DEVICE n int32 (may
 * be NULL) as wfpg_partition. Never waits for the device: the per-bin
 * fields are sized by a bound on the bins a call can use (every bin is a node
 * at a level up to l_min, or a deeper node holding at least c_ray queries:
 * at most n / c_ray per level) and the kernels read the used count on the
 * device, so the call can be captured in a HIP graph. It uses the SVO's
 * binning scratch, which grows on first use: calls on one SVO must be
 * stream-ordered, and a caller capturing a graph makes one call of the same
 * n and N first. Errors: EINVAL for bad arguments, n >= 2^31. */
wfpg_status guide_sample_binned(const wfpg_svo *svo, const float *pos, int64_t n, uint64_t seed,
                                uint32_t bounce, const wfpg_bin_opts *opts, float *dir_out,
                                float *pdf_out, int32_t *bin_out, void *hip_stream);

/* Binned product guiding (Sec. 3.6 over the bins of Alg. 2): every member
 * draws a product sample (as guide_sample_product) from its bin's field,
 * generated once at the bin origin, and its own table (nrm DEVICE 3 x n or
 * bsdf DEVICE n x 64; exactly one). One wave per member, as the paper
 * assigns one warp to a ray. Outputs and errors as guide_sample_binned;
 * EINVAL when both or neither of nrm, bsdf is given. */
wfpg_status guide_sample_binned_product(const wfpg_svo *svo, const float *pos, const float *nrm,
                                        const float *bsdf, int64_t n, uint64_t seed, uint32_t bounce,
                                        const wfpg_bin_opts *opts, float *dir_out, float *pdf_out,
                                        int32_t *bin_out, void *hip_stream);

/* ---------------------------------------------------------------------
 * Learned stand-in for the march (guide_sample with opts->mode == 1).
 *
 * A multiresolution hash-grid encoding of the position (16 levels, 2^log2_table
 * entries of 2 features per level; level l has resolution
 * floor(n_min * b^l), b chosen so level 15 reaches n_max; a level whose
 * (R+1)^3 corner grid fits the table is indexed densely, otherwise by the
 * spatial hash x*1 ^ y*2654435761 ^ z*805459861 mod 2^log2_table; trilinear
 * interpolation) is concatenated with the surface normal (3 values) and fed to
 * a ReLU MLP 35 -> 64 -> 64 -> 64 -> 64 -> 256 whose softmax over the 256
 * logits is a 16 x 16 bin distribution on the same octahedral field the march
 * uses (Sec. 3.3). Table, inputs, weights and activations are BF16, products
 * accumulate in FP32 (MFMA); master parameters and Adam moments are FP32.
 * It is trained on pdfs the march itself produces (guide_pdf at N = 16 with
 * eps = target_eps and, with target_blur = 1, the blurred field) by
 * minimising the mean cross-entropy -sum_b t_b log q_b.
 *
 * Parameter vector order (FP32): W0[64][35], b0[64], W1[64][64], b1, W2, b2,
 * W3, b3, W4[256][64], b4[256], then the table [16][2^log2_table][2]
 * (31424 MLP parameters + 32 * 2^log2_table table entries).
 * The model belongs to the SVO: created by the first guide_train or
 * wfpg_nn_params(set = 1), freed by svo_destroy.
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t log2_table;  /* entries per level = 2^log2_table, 10..24 (19) */
    int32_t n_min;       /* coarsest resolution, >= 2 (16) */
    int32_t n_max;       /* finest resolution; 0 = 2^depth of the SVO */
    int32_t batch;       /* vertices per step, 64..2^22 (65536) */
    int32_t steps;       /* Adam steps this call, >= 0 (100) */
    float lr_mlp;        /* Adam step size of the MLP (2e-3) */
    float lr_table;      /* Adam step size of the hash table (1e-2) */
    float beta1, beta2;  /* Adam moment decays (0.9, 0.99) */
    float adam_eps;      /* Adam denominator guard (1e-15) */
    uint64_t seed;       /* initialisation seed, used when the model is created */
    float target_eps;    /* eps of the march fields the model is trained on, finite > 0 (0.01) */
    int32_t target_blur; /* 1: the training targets are the blurred fields (Sec. 4), 0 or 1 (0) */
} wfpg_train_cfg;

wfpg_train_cfg wfpg_default_train_cfg(void);

/* Run cfg->steps Adam steps. Step t takes the batch of cfg->batch consecutive
 * vertices of the DEVICE queue pos/nrm (3 x n SoA each) starting at
 * ((t - 1) * batch) mod n (clamped to end at n), marches their targets, and
 * updates the model. The model configuration (log2_table, n_min, n_max, seed)
 * is fixed when the model is created; later calls continue training it
 * (steps = 0 only creates the model). Step counts t are global over calls.
 * mean_loss (HOST, may be NULL): mean cross-entropy over the last 10 steps
 * (synchronizes). Errors: EINVAL for bad arguments or configuration. */
wfpg_status guide_train(wfpg_svo *svo, const float *pos, const float *nrm, int64_t n,
                        const wfpg_train_cfg *cfg, float *mean_loss, void *hip_stream);

/* Number of FP32 parameters of the attached model, -1 if none. */
int64_t wfpg_nn_param_count(const wfpg_svo *svo);

/* Copy the FP32 parameters to (set = 0) or from (set = 1) the HOST array
 * host[count]; count must equal wfpg_nn_param_count. set = 1 creates a model
 * with the default configuration if none exists and marks it trained.
 * Synchronizes the stream. ESTATE: get without a model. */
wfpg_status wfpg_nn_params(wfpg_svo *svo, float *host, int64_t count, int32_t set,
                           void *hip_stream);

/* Network distribution (softmax of the logits) of each vertex:
 * prob_out DEVICE n x 256 FP32, row-major, bin b = v*16 + u. */
wfpg_status wfpg_nn_forward(wfpg_svo *svo, const float *pos, const float *nrm, int64_t n,
                            float *prob_out, void *hip_stream);

/* Test-only: the gradient of the mean cross-entropy against DEVICE targets
 * target[n][256] (rows summing to 1), written to DEVICE grad_out[count] in
 * parameter order, and the loss to HOST *loss_out (may be NULL; synchronizes).
 * Parameters are not changed. */
wfpg_status wfpg_nn_grad(wfpg_svo *svo, const float *pos, const float *nrm, const float *target,
                         int64_t n, float *grad_out, float *loss_out, void *hip_stream);

/* Judge of the learned path: in mode 1, guide_sample marches every
 * probe_stride-th vertex and computes the mean over those probes of
 * KL(p_march || q_net) in nats (bins weighted by the marched pdf). If it
 * exceeds kl_bound, the call's outputs are those of the march (mode 0) for
 * every vertex. Last judged KL and the number of calls that fell back.
 * Synchronizes the device. */
wfpg_status wfpg_learned_stats(const wfpg_svo *svo, float *last_probe_kl, int64_t *fallbacks);

#ifdef __cplusplus
}
#endif
#endif /* WFPG_H */
