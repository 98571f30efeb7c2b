// Exact SVO march and cone footprint, shared by the gfx950 kernels and by a
// host build used in the CPU test suite (same source, compiled by g++).
//
// The ray is O + t*q: O is the query position on a 2^30 grid per unit length
// and q = rint(d * 2^23) the bin direction. Crossing parameters are compared
// exactly as |B_a - O_a| * |q_b| vs |B_b - O_b| * |q_a| in 64-bit integers
// (each factor < 2^31 and < 2^24). The result is the first occupied leaf,
// other than the origin's, of the 6-connected leaf traversal whose ties step
// the lowest axis first; leaving the unit cube is a miss. This replaces the
// hardware ray cast of the paper (Sec. 3.3) with a march of the SVO itself.
//
// The walk is top-down with empty-space skipping. After each step only the
// levels below the deepest ancestor shared with the previous cell are
// tested, down to the first empty level or the leaf. An empty cell at any
// level is left through its first exit crossing; descending into an occupied
// cell picks the child by comparing each mid-plane's crossing parameter with
// the current one (equal parameters: the plane counts as crossed iff its axis
// is not above the axis of the current crossing).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define WFPG_HD __host__ __device__ __forceinline__
#define WFPG_UNROLL _Pragma("unroll")
#else
#define WFPG_HD inline
#define WFPG_UNROLL
#endif

namespace wfpg {
namespace core {

constexpr int kFine = 30;

// Word offset of level l in the concatenated occupancy bitmaps (levels 0..2
// take one 64-bit word each, level l >= 3 takes 8^l / 64 words).
WFPG_HD uint32_t woff(int l)
{
    return l <= 3 ? (uint32_t)l : 3u + ((0x09249249u & ((1u << (3 * l - 9)) - 1u)) << 3);
}

WFPG_HD uint32_t part1by2(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
WFPG_HD uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}

// Position and direction quantization. Positions are clamped to the grid in
// integers (2^30 - 1 is not an FP32 value).
WFPG_HD uint32_t quantize_pos(float p)
{
    const float o = __builtin_rintf(p * 1073741824.0f);   // exact scaling, ties to even
    if (!(o > 0.0f)) return 0u;         // also NaN
    if (o >= 1073741824.0f) return 1073741823u;
    return (uint32_t)o;
}
WFPG_HD int quantize_dir(float d)
{
    return (int)__builtin_rintf(d * 8388608.0f);   // exact scaling, |q| <= 2^23
}

struct Hit {
    int axis;          // axis of the crossing that entered the hit leaf
    uint32_t key;      // hit leaf key
    uint32_t delta;    // |B - O| of that crossing, 2^-30 units
};

enum { STEP_CONTINUE = 0, STEP_HIT = 1, STEP_MISS = 2 };

// Which half of a cell the ray is in along one axis just after the current
// crossing (tn/td, ta): the mid-plane M counts as crossed iff its crossing
// parameter is smaller, or equal with an axis not above ta.
WFPG_HD uint32_t upper_half(uint32_t M, uint32_t O, uint32_t aq, int sg, int j, uint32_t tn,
                            uint32_t td, int ta)
{
    if (sg == 0) return O >= M ? 1u : 0u;
    int32_t dl = (int32_t)(M - O);
    if (sg < 0) dl = -dl;
    const int64_t lhs = (int64_t)dl * (int64_t)td - (int64_t)((uint64_t)tn * aq);
    const bool crossed = lhs < (int64_t)(j <= ta) || (sg > 0 && dl == 0);
    return (crossed != (sg < 0)) ? 1u : 0u;
}

// Distance (2^-30 units) from O to the far face of [lo, lo + size) along
// the ray's direction on one axis (1 when the axis is not crossed).
WFPG_HD uint32_t far_face(uint32_t lo, uint32_t size, uint32_t O, int sg)
{
    return sg > 0 ? lo + size - O : (sg < 0 ? O - lo : 1u);
}

WFPG_HD void split_dir(int q, uint32_t &aq, int &sg)
{
    aq = (uint32_t)(q < 0 ? -q : q);
    sg = (q > 0) - (q < 0);
}

// The traversal is a machine that performs exactly one occupancy test per
// call, so that the lanes of a wave, each on its own ray, advance in lockstep
// one test at a time instead of waiting for the longest ancestor walk or
// descent of the wave. Phases:
//  PH_ADVANCE  the state is an empty cell (or the origin's leaf): leave it
//              through its first exit crossing, then test the first unshared
//              ancestor of the cell entered (same call);
//  PH_PATH     key/lo/lvl hold the cell entered; its ancestors from level l
//              down are tested one per call (levels above l are occupied);
//  PH_DESCEND  key/lo/lvl hold an occupied cell; each call tests the child the
//              ray is in (mid-plane comparisons).
enum { PH_ADVANCE = 0, PH_PATH = 1, PH_DESCEND = 2 };
constexpr int kMaxTests = 1 << 17;   // > worst-case occupancy tests of a depth-10 ray

struct MicroState {
    uint32_t O0, O1, O2;      // origin, 2^-30 units
    uint32_t aq0, aq1, aq2;   // |q|
    int sg0, sg1, sg2;        // sign(q)
    int lvl, ta, l, phase;
    uint32_t key, tn, td;
    uint32_t lo0, lo1, lo2;
};

// Start at the origin's cell. When the origin's leaf is occupied it is the
// cell to leave (never a hit) and the ancestors the top-down walk would test
// are counted; otherwise the origin's path is tested from the root down.
WFPG_HD void micro_begin(MicroState &s, const uint32_t O[3], uint32_t origin_key, bool origin_occupied,
                         uint32_t aq0, uint32_t aq1, uint32_t aq2, int sg0, int sg1, int sg2, int D,
                         int count_from, int &vis)
{
    s.O0 = O[0]; s.O1 = O[1]; s.O2 = O[2];
    s.aq0 = aq0; s.aq1 = aq1; s.aq2 = aq2;
    s.sg0 = sg0; s.sg1 = sg1; s.sg2 = sg2;
    s.ta = -1; s.tn = 0; s.td = 1;
    const uint32_t mk = ~((1u << (kFine - D)) - 1u);
    s.lvl = D;
    s.key = origin_key;
    s.lo0 = O[0] & mk; s.lo1 = O[1] & mk; s.lo2 = O[2] & mk;
    s.l = 0;
    if (origin_occupied) {
        s.phase = PH_ADVANCE;
        vis += D + 1 - (count_from < D ? count_from : D);   // levels count_from..D
    } else {
        s.phase = PH_PATH;
    }
}

// OPAQUE_SIGNS: hide the ray's signs from the optimizer at every step, so the
// sign tests stay in the loop as vector compares. For a caller whose scalar
// registers are already full (the guide kernel's queue and slot bookkeeping),
// the loop-invariant lane masks the compiler would otherwise hoist are spilled
// into vector lanes and cost two lane moves per use; elsewhere the hoisted
// masks are the cheaper form.
template <bool OPAQUE_SIGNS = false, class Bits>
WFPG_HD int micro_step(MicroState &s, int D, const Bits &bits, int count_from, int &vis, Hit &h)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (OPAQUE_SIGNS) asm volatile("" : "+v"(s.sg0), "+v"(s.sg1), "+v"(s.sg2));
#endif
    if (s.phase == PH_ADVANCE) {
        const uint32_t size = 1u << (kFine - s.lvl);
        const uint32_t dl0 = far_face(s.lo0, size, s.O0, s.sg0);
        const uint32_t dl1 = far_face(s.lo1, size, s.O1, s.sg1);
        const uint32_t dl2 = far_face(s.lo2, size, s.O2, s.sg2);
        const uint32_t c1 = (uint64_t)dl1 * s.aq0 < (uint64_t)dl0 * s.aq1 ? 0xffffffffu : 0u;
        const uint32_t D01 = (dl1 & c1) | (dl0 & ~c1), Q01 = (s.aq1 & c1) | (s.aq0 & ~c1);
        const uint32_t c2 = (uint64_t)dl2 * Q01 < (uint64_t)D01 * s.aq2 ? 0xffffffffu : 0u;
        const uint32_t m0 = ~c1 & ~c2, m1 = c1 & ~c2, m2 = c2;
        const int e = (int)((m1 & 1u) | (m2 & 2u));
        const uint32_t De = (dl2 & m2) | (D01 & ~m2);
        const uint32_t Qe = (s.aq2 & m2) | (Q01 & ~m2);
        const int sgn = (int)(((uint32_t)s.sg0 & m0) | ((uint32_t)s.sg1 & m1) | ((uint32_t)s.sg2 & m2));
        const uint32_t le = (s.lo0 & m0) | (s.lo1 & m1) | (s.lo2 & m2);
        const int64_t nl = (int64_t)le + (int64_t)sgn * (int64_t)size;
        if (nl < 0 || nl >= (1ll << kFine)) return STEP_MISS;
        const uint32_t nlu = (uint32_t)nl;
        const uint32_t oldc = le >> (kFine - s.lvl), newc = nlu >> (kFine - s.lvl);
        const uint32_t m = 0x09249249u << e;
        s.key = sgn > 0 ? ((((s.key | ~m) + 1u) & m) | (s.key & ~m)) : ((((s.key & m) - 1u) & m) | (s.key & ~m));
        s.lo0 = (nlu & m0) | (s.lo0 & ~m0);
        s.lo1 = (nlu & m1) | (s.lo1 & ~m1);
        s.lo2 = (nlu & m2) | (s.lo2 & ~m2);
        s.tn = De;
        s.td = Qe;
        s.ta = e;
        s.l = s.lvl - (31 - __builtin_clz(oldc ^ newc));   // first level not shared with the cell left
        s.phase = PH_PATH;
    }
    // the cell to test: an ancestor of the entered cell, or the child the ray is in
    int tl;
    uint32_t tk, n0 = s.lo0, n1 = s.lo1, n2 = s.lo2;
    if (s.phase == PH_PATH) {
        tl = s.l;
        tk = s.key >> (3 * (s.lvl - s.l));
    } else {
        const uint32_t half = 1u << (29 - s.lvl);
        const uint32_t oct = upper_half(s.lo0 + half, s.O0, s.aq0, s.sg0, 0, s.tn, s.td, s.ta) |
                             (upper_half(s.lo1 + half, s.O1, s.aq1, s.sg1, 1, s.tn, s.td, s.ta) << 1) |
                             (upper_half(s.lo2 + half, s.O2, s.aq2, s.sg2, 2, s.tn, s.td, s.ta) << 2);
        tk = (s.key << 3) | oct;
        n0 += (oct & 1u) ? half : 0u;
        n1 += (oct & 2u) ? half : 0u;
        n2 += (oct & 4u) ? half : 0u;
        tl = s.lvl + 1;
    }
    const uint64_t w = bits(tl, woff(tl) + (tk >> 6));
    vis += (tl >= count_from);
    if (!((w >> (tk & 63)) & 1ull)) {   // empty: the cell to leave next
        const uint32_t mk = ~((1u << (kFine - tl)) - 1u);
        s.lvl = tl;
        s.key = tk;
        s.lo0 = n0 & mk;
        s.lo1 = n1 & mk;
        s.lo2 = n2 & mk;
        s.phase = PH_ADVANCE;
        return STEP_CONTINUE;
    }
    if (s.phase == PH_PATH) {
        if (tl < s.lvl) {
            s.l = tl + 1;
            return STEP_CONTINUE;
        }
        s.phase = PH_DESCEND;   // the entered cell is occupied
    } else {
        s.lvl = tl;
        s.key = tk;
        s.lo0 = n0;
        s.lo1 = n1;
        s.lo2 = n2;
    }
    if (s.lvl == D) {
        h.axis = s.ta;
        h.key = s.key;
        h.delta = s.tn;
        return STEP_HIT;
    }
    return STEP_CONTINUE;
}

// Whole march: 1 on a hit, 0 on a miss, -1 if the iteration bound is
// exceeded (never expected).
template <class Bits>
WFPG_HD int march(const uint32_t O[3], int q0, int q1, int q2, int D, const Bits &bits,
                  int count_from, int &vis, Hit &h)
{
    MicroState s;
    uint32_t aq0, aq1, aq2;
    int sg0, sg1, sg2;
    split_dir(q0, aq0, sg0);
    split_dir(q1, aq1, sg1);
    split_dir(q2, aq2, sg2);
    const uint32_t ok = morton3(O[0] >> (kFine - D), O[1] >> (kFine - D), O[2] >> (kFine - D));
    const bool occ = (bits(D, woff(D) + (ok >> 6)) >> (ok & 63)) & 1ull;
    micro_begin(s, O, ok, occ, aq0, aq1, aq2, sg0, sg1, sg2, D, count_from, vis);
    for (int it = 0; it < kMaxTests; ++it) {
        const int st = micro_step(s, D, bits, count_from, vis, h);
        if (st == STEP_HIT) return 1;
        if (st == STEP_MISS) return 0;
    }
    return -1;
}

// Cone footprint (Eq. 7): A = r^2 * omega, r = ((float)delta * 2^-(30-D)) /
// |d_axis| the distance to the hit leaf's entry point in leaf units (FP32,
// every operation rounded); the node whose area side^2 is closest to A lies
// k = #{ j in 1..D : A > 2.5 * 4^(j-1) } levels above the leaf.
WFPG_HD int footprint_levels(uint32_t delta, float dabs, int D, float omega)
{
    float scale = 1.0f;
    WFPG_UNROLL
    for (int i = 0; i < kFine; ++i)                         // exact 2^-(30-D)
        if (i < kFine - D) scale *= 0.5f;
    const float dist = ((float)delta * scale) / dabs;
    const float sq = dist * dist;
    const float A = sq * omega;
    int k = 0;
    float thr = 2.5f;
    WFPG_UNROLL
    for (int j = 1; j <= 10; ++j) {
        if (j > D) break;
        k += A > thr ? 1 : 0;
        thr *= 4.0f;
    }
    return k;
}

// Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), the counter-based
// generator of every random draw of the library: ten rounds of two 32 x 32
// -> 64-bit products with a Weyl key schedule.
WFPG_HD void philox(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    WFPG_UNROLL
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
    }
}

// dot(N, d) in FP32 as (x*x' + y*y') + z*z', each product rounded.
WFPG_HD float dot3(float ax, float ay, float az, float bx, float by, float bz)
{
    const float px = ax * bx;
    const float py = ay * by;
    const float pz = az * bz;
    const float s = px + py;
    return s + pz;
}

}  // namespace core
}  // namespace wfpg
