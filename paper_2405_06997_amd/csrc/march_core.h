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
#else
#define WFPG_HD inline
#endif

namespace wfpg {
namespace core {

constexpr int kFine = 30;
constexpr int kMaxIt = 1 << 15;   // > worst-case steps of a depth-10 ray

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

struct Ray {
    uint32_t O[3];    // origin, 2^-30 units
    uint32_t aq[3];   // |q|
    int sg[3];        // sign(q)
};

WFPG_HD void make_ray(const uint32_t O[3], int q0, int q1, int q2, Ray &r)
{
    const int q[3] = {q0, q1, q2};
    for (int k = 0; k < 3; ++k) {
        r.O[k] = O[k];
        r.aq[k] = (uint32_t)(q[k] < 0 ? -q[k] : q[k]);
        r.sg[k] = (q[k] > 0) - (q[k] < 0);
    }
}

struct Hit {
    int axis;          // axis of the crossing that entered the hit leaf
    uint32_t key;      // hit leaf key
    uint32_t delta;    // |B - O| of that crossing, 2^-30 units
};

// Bits(level, word_index) -> uint64 occupancy word. Returns 1 on a hit, 0 on
// a miss and -1 if the iteration bound is exceeded (never expected).
template <class Bits>
WFPG_HD int march(const Ray &r, int D, uint32_t origin_key, const Bits &bits, int count_from,
                  int &vis, Hit &h)
{
    int lvl = 0;
    uint32_t key = 0;
    uint32_t lo0 = 0, lo1 = 0, lo2 = 0;
    int tlvl = 0;
    uint32_t tkey = 0;
    uint32_t tn = 0, td = 1;
    int ta = -1;
    for (int it = 0; it < kMaxIt; ++it) {
        const uint64_t w = bits(lvl, woff(lvl) + (key >> 6));
        vis += (lvl >= count_from);
        if ((w >> (key & 63)) & 1ull) {
            if (lvl == D) {
                if (key != origin_key) {
                    h.axis = ta;
                    h.key = key;
                    h.delta = tn;
                    return 1;
                }
            } else {
                const uint32_t half = 1u << (29 - lvl);
                uint32_t oct;
                if (lvl < tlvl) {
                    oct = (tkey >> (3 * (tlvl - lvl - 1))) & 7u;
                } else {
                    oct = 0;
                    const uint32_t lo[3] = {lo0, lo1, lo2};
                    for (int j = 0; j < 3; ++j) {
                        const uint32_t M = lo[j] + half;
                        bool up;
                        if (r.sg[j] == 0) {
                            up = r.O[j] >= M;
                        } else {
                            int32_t dl = (int32_t)(M - r.O[j]);
                            if (r.sg[j] < 0) dl = -dl;
                            const int64_t lhs = (int64_t)dl * (int64_t)td -
                                                (int64_t)((uint64_t)tn * r.aq[j]);
                            const bool crossed =
                                lhs < (int64_t)(j <= ta) || (r.sg[j] > 0 && dl == 0);
                            up = crossed != (r.sg[j] < 0);
                        }
                        oct |= (uint32_t)up << j;
                    }
                }
                key = (key << 3) | oct;
                lo0 += (oct & 1u) ? half : 0u;
                lo1 += (oct & 2u) ? half : 0u;
                lo2 += (oct & 4u) ? half : 0u;
                ++lvl;
                continue;
            }
        }
        // leave the current cell (empty, or the origin's leaf)
        const uint32_t size = 1u << (kFine - lvl);
        const uint32_t dl0 = r.sg[0] > 0 ? lo0 + size - r.O[0] : (r.sg[0] < 0 ? r.O[0] - lo0 : 1u);
        const uint32_t dl1 = r.sg[1] > 0 ? lo1 + size - r.O[1] : (r.sg[1] < 0 ? r.O[1] - lo1 : 1u);
        const uint32_t dl2 = r.sg[2] > 0 ? lo2 + size - r.O[2] : (r.sg[2] < 0 ? r.O[2] - lo2 : 1u);
        int e = 0;
        uint32_t De = dl0, Qe = r.aq[0];
        if ((uint64_t)dl1 * Qe < (uint64_t)De * r.aq[1]) { e = 1; De = dl1; Qe = r.aq[1]; }
        if ((uint64_t)dl2 * Qe < (uint64_t)De * r.aq[2]) { e = 2; De = dl2; Qe = r.aq[2]; }
        const int s = e == 0 ? r.sg[0] : (e == 1 ? r.sg[1] : r.sg[2]);
        const uint32_t le = e == 0 ? lo0 : (e == 1 ? lo1 : lo2);
        const int64_t nl = (int64_t)le + (int64_t)s * (int64_t)size;
        if (nl < 0 || nl >= (1ll << kFine)) return 0;
        const uint32_t oldc = le >> (kFine - lvl), newc = (uint32_t)nl >> (kFine - lvl);
        if (e == 0) lo0 = (uint32_t)nl; else if (e == 1) lo1 = (uint32_t)nl; else lo2 = (uint32_t)nl;
        const uint32_t m = 0x09249249u << e;
        key = s > 0 ? ((((key | ~m) + 1u) & m) | (key & ~m)) : ((((key & m) - 1u) & m) | (key & ~m));
        tn = De;
        td = Qe;
        ta = e;
        tlvl = lvl;
        tkey = key;
        const int p = 31 - __builtin_clz(oldc ^ newc);
        lvl -= p;
        key >>= 3 * p;
        const uint32_t mk = ~((1u << (kFine - lvl)) - 1u);
        lo0 &= mk;
        lo1 &= mk;
        lo2 &= mk;
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
    for (int i = 0; i < kFine - D; ++i) scale *= 0.5f;     // exact 2^-(30-D)
    const float dist = ((float)delta * scale) / dabs;
    const float sq = dist * dist;
    const float A = sq * omega;
    int k = 0;
    float thr = 2.5f;
    for (int j = 1; j <= D; ++j) {
        k += A > thr ? 1 : 0;
        thr *= 4.0f;
    }
    return k;
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
