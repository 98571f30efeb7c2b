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
    const uint32_t t = 3u * ((uint32_t)l & 15u) - 9u;   // wraps for l < 3, where l is returned
    const uint32_t f = 3u + ((0x09249249u & ((1u << (t & 31u)) - 1u)) << 3);
    return l <= 3 ? (uint32_t)l : f;
}

// Occupancy bit of cell `key` at level l, read as 32-bit words: bit key & 31
// of word 2 woff(l) + key / 32 (the bitmaps are little-endian 64-bit words).
// bits(l, i) returns 32-bit word i.
template <class Bits>
WFPG_HD bool occupied(const Bits &bits, int l, uint32_t key)
{
    return (bits(l, 2u * woff(l) + (key >> 5)) >> (key & 31u)) & 1u;
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

WFPG_HD void split_dir(int q, uint32_t &aq, int &sg)
{
    aq = (uint32_t)(q < 0 ? -q : q);
    sg = (q > 0) - (q < 0);
}

// Lane conditions of the march step held as 32-bit masks (all ones or zero)
// in ordinary registers, made from the sign of a difference, and combined and
// selected with one three-input bitwise operation each: on gfx950 an add, a
// logic op, a right shift and v_bitop3_b32 issue at twice the rate of a
// select on a condition register, a compare, a left shift or a min/max.
// bop3<F>(a, b, c): bit i of the result is bit (a_i << 2 | b_i << 1 | c_i)
// of the truth table F (the host build evaluates the table).
template <unsigned F>
WFPG_HD uint32_t bop3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, F);
#else
    uint32_t r = 0;
    for (unsigned i = 0; i < 8; ++i)
        if ((F >> i) & 1u) r |= ((i & 4u) ? a : ~a) & ((i & 2u) ? b : ~b) & ((i & 1u) ? c : ~c);
    return r;
#endif
}
// A value the compiler may not reason about: an empty statement that keeps
// it in a vector register, so that a sign mask stays a shift (not a compare
// and a select) and a sum keeps the grouping it is written in.
template <class T>
WFPG_HD T opaque(T x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    __asm__("" : "+v"(x));
#endif
    return x;
}
WFPG_HD uint32_t msel(uint32_t m, uint32_t a, uint32_t b) { return bop3<0xCA>(m, a, b); }   // m ? a : b
WFPG_HD uint32_t neg_mask(int32_t x) { return (uint32_t)(opaque(x) >> 31); }               // x < 0
WFPG_HD uint32_t neg_mask64(int64_t x) { return neg_mask((int32_t)(uint32_t)((uint64_t)x >> 32)); }

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

// The march runs in a frame mirrored on every axis the ray descends
// (x -> 2^30 - x), so that it always moves towards larger coordinates:
// cell planes map to cell planes and crossing parameters are unchanged, and a
// mirrored cell's key is the original key with that axis's bits complemented.
// Only the membership of points lying exactly on a plane differs between the
// frames; the mid-plane test below keeps the original rule for it.
struct MicroState {
    uint32_t O0, O1, O2;      // origin in the mirrored frame, 2^-30 units
    uint32_t aq0, aq1, aq2;   // |q|
    uint32_t mir;             // bit j: axis j is mirrored (q_j < 0); bit 3 + j: q_j = 0
    uint32_t flip;            // key bits of the mirrored axes, all levels
    int lvl, ta, l, phase;
    uint32_t key, tn, td;     // key in the mirrored frame
    uint32_t lo0, lo1, lo2;   // cell corner in the mirrored frame
};

// Start at the origin's cell. When the origin's leaf is occupied it is the
// cell to leave (never a hit) and the ancestors the top-down walk would test
// are counted; otherwise the origin's path is tested from the root down.
WFPG_HD void micro_begin(MicroState &s, const uint32_t O[3], uint32_t origin_key, bool origin_occupied,
                         uint32_t aq0, uint32_t aq1, uint32_t aq2, int sg0, int sg1, int sg2, int D,
                         int count_from, int &vis)
{
    const uint32_t leaf = 1u << (kFine - D), mk = ~(leaf - 1u);
    const bool n0 = sg0 < 0, n1 = sg1 < 0, n2 = sg2 < 0;
    s.O0 = n0 ? (1u << kFine) - O[0] : O[0];
    s.O1 = n1 ? (1u << kFine) - O[1] : O[1];
    s.O2 = n2 ? (1u << kFine) - O[2] : O[2];
    s.lo0 = n0 ? (1u << kFine) - (O[0] & mk) - leaf : O[0] & mk;
    s.lo1 = n1 ? (1u << kFine) - (O[1] & mk) - leaf : O[1] & mk;
    s.lo2 = n2 ? (1u << kFine) - (O[2] & mk) - leaf : O[2] & mk;
    s.aq0 = aq0; s.aq1 = aq1; s.aq2 = aq2;
    // bits 0-2: mirrored axes; bits 3-5: axes without motion (|q| = 0)
    s.mir = (n0 ? 1u : 0u) | (n1 ? 2u : 0u) | (n2 ? 4u : 0u) | (aq0 == 0u ? 8u : 0u) | (aq1 == 0u ? 16u : 0u) |
            (aq2 == 0u ? 32u : 0u);
    s.flip = (n0 ? 0x09249249u : 0u) | (n1 ? 0x12492492u : 0u) | (n2 ? 0x24924924u : 0u);
    s.ta = -1; s.tn = 0; s.td = 1;
    s.lvl = D;
    s.key = origin_key ^ (s.flip >> (kFine - 3 * D));
    s.l = 0;
    if (origin_occupied) {
        s.phase = PH_ADVANCE;
        vis += D + 1 > count_from ? D + 1 - count_from : 0;   // levels count_from..D
    } else {
        s.phase = PH_PATH;
    }
}

// One 64-bit occupancy load per call, with no branch that depends on the
// lane: every lane computes the exit step of PH_ADVANCE and both candidate
// cells (the ancestor of PH_PATH, the child of PH_DESCEND) and keeps what its
// phase selects, so a wave whose lanes sit in different phases runs one
// straight sequence with every lane active instead of each phase's code under
// its own lane mask.
//
// A 64-bit word of level L (the cells of one level-(L-2) cell, Morton order)
// answers three levels at once: level L-2 (the word is not zero), level L-1
// (one of its bytes) and level L (one bit). A path descent therefore tests
// up to three ancestors of the entered cell per call -- the window [l, T],
// T = min(l + 2, lvl) -- and stops at the first empty one, exactly the tests
// of the top-down walk one at a time; a child descent tests one level. The
// node tests counted are those of the walk (levels >= count_from).
// bits64(wi) returns 64-bit word wi of the concatenated bitmaps. On STEP_HIT
// the hit is hit_of(s, D).
// The first exit crossing of the cell s holds, through its upper face on
// every axis: along axis e (c1: axis 1 before axis 0, c2: axis 2 before
// both, as masks), at parameter tn / td. The cell entered has corner nlu
// along e (2^30 when the crossing leaves the cube) and key akey. An axis the
// ray does not cross (|q| = 0) has lo + size - O >= 1, which only ever meets
// its zero |q| in the comparisons.
struct Exit {
    uint32_t c1, c2, le, nlu, akey, tn, td;
    int e;
};
WFPG_HD Exit exit_crossing(const MicroState &s, uint32_t size)
{
    Exit x;
    const uint32_t dl0 = s.lo0 + size - s.O0;
    const uint32_t dl1 = s.lo1 + size - s.O1;
    const uint32_t dl2 = s.lo2 + size - s.O2;
    // axis 1 before axis 0 iff dl1 |q0| - dl0 |q1| < 0 (dl <= 2^30, |q| <= 2^23:
    // the difference is exact in 64 bits)
    x.c1 = neg_mask64((int64_t)((uint64_t)dl1 * s.aq0) + (int64_t)(int32_t)dl0 * (int64_t)(0 - (int32_t)s.aq1));
    const uint32_t D01 = msel(x.c1, dl1, dl0), Q01 = msel(x.c1, s.aq1, s.aq0);
    x.c2 = neg_mask64((int64_t)((uint64_t)dl2 * Q01) + (int64_t)(int32_t)D01 * (int64_t)(0 - (int32_t)s.aq2));
    x.e = (int)(bop3<0x58>(x.c2, x.c1, 1u) & 3u);   // c2 ? 2 : (c1 ? 1 : 0)
    x.le = msel(x.c2, s.lo2, msel(x.c1, s.lo1, s.lo0));
    // one cell up along the crossed axis (|q| > 0); leaving the cube reaches 2^30
    x.nlu = x.le + size;
    const uint32_t m = 0x24924924u >> (2 - x.e);   // the key bits of axis e: add one to them
    x.akey = msel(m, bop3<0xF3>(s.key, m, m) + 1u, s.key);   // (key | ~m) + 1 on those bits
    x.tn = msel(x.c2, dl2, D01);
    x.td = msel(x.c2, s.aq2, Q01);
    return x;
}

template <class Bits64>
WFPG_HD int micro_step(MicroState &s, int D, const Bits64 &bits64, int count_from, int &vis)
{
    const uint32_t advm = neg_mask(s.phase - PH_PATH);    // PH_ADVANCE
    const uint32_t pathm = neg_mask(s.phase - PH_DESCEND);  // PH_ADVANCE or PH_PATH
    const uint32_t size = (1u << kFine) >> s.lvl;
    // PH_DESCEND candidate (taken from the state before the advance below,
    // which leaves a descending lane's state as it is, so that the two are
    // independent): the child the ray is in just after the current crossing
    // tn/td. Along axis j the mid-plane M counts as crossed iff its
    // parameter is smaller, or equal with j not above ta: with d = M - O,
    // iff d td < tn |q_j| + k (k = 1 when j is not above ta), i.e. iff
    // P = tn |q_j| + k - d td > 0, iff tn |q_j| + (k - 1) - d td >= 0: one
    // 32 x 32 + 64 product-add and one signed one (td < 2^24), the sign of the
    // sum giving the mask of the lower half; a plane behind the origin (d < 0)
    // gives P > 0. A point on the plane (d = 0) of an axis that is not
    // mirrored is in the upper half (the half-open cells of the original
    // frame); that decides only where tn |q_j| = 0 (at the origin, or with no
    // motion along j, where O >= M is the whole rule), and there k = 1 gives it.
    const uint32_t half = size >> 1;
    const int32_t nd0 = (int32_t)(s.O0 - s.lo0 - half);   // -d
    const int32_t nd1 = (int32_t)(s.O1 - s.lo1 - half);
    const int32_t nd2 = (int32_t)(s.O2 - s.lo2 - half);
    const int64_t td = (int64_t)(int32_t)s.td;
    // k_j as bits: bit j of K (j not above ta: the low ta + 1 bits; an axis
    // without motion; a non-mirrored axis while tn = 0, tn <= 2^30)
    const uint32_t K = bop3<0xFE>(7u >> (2 - s.ta), s.mir >> 3, bop3<0x20>(neg_mask((int32_t)s.tn - 1), s.mir, 7u));
    // -d td + (k_j - 1) (k_j - 1 is 0 or -1), then + tn |q_j|: the mask of
    // the lower half (the plane not crossed) on each axis
    auto lower = [&](int32_t nd, uint32_t kbit, uint32_t aq) {
        const int64_t a = opaque((int64_t)nd * td + (int64_t)(int32_t)neg_mask((int32_t)kbit - 1));
        return neg_mask64((int64_t)((uint64_t)s.tn * aq + (uint64_t)a));
    };
    const uint32_t lo0m = lower(nd0, K & 1u, s.aq0);
    const uint32_t lo1m = lower(nd1, K & 2u, s.aq1);
    const uint32_t lo2m = lower(nd2, K & 4u, s.aq2);
    // the child key: bit j set where the plane is crossed
    const uint32_t dk = (s.key << 3) | (bop3<0xB1>(bop3<0x1B>(lo0m, lo1m, 1u), lo2m, 3u) & 7u);

    // PH_ADVANCE: leave the current cell through its first exit crossing.
    const Exit x = exit_crossing(s, size);
    const uint32_t missm = advm & neg_mask((int32_t)((1u << kFine) - 1u - x.nlu));   // nlu < 2^31
    // first level not shared with the cell left: le and nlu differ first in
    // bit 30 - al (at level lvl or above, so al <= lvl)
    const int cz = __builtin_clz(x.le ^ x.nlu);   // al = cz - 1
    s.lo0 = msel(bop3<0x10>(advm, x.c1, x.c2), x.nlu, s.lo0);   // adv & ~c1 & ~c2
    s.lo1 = msel(bop3<0x40>(advm, x.c1, x.c2), x.nlu, s.lo1);   // adv & c1 & ~c2
    s.lo2 = msel(advm & x.c2, x.nlu, s.lo2);
    s.key = msel(advm, x.akey, s.key);
    s.tn = msel(advm, x.tn, s.tn);
    s.td = msel(advm, x.td, s.td);
    s.ta = (int)msel(advm, (uint32_t)x.e, (uint32_t)s.ta);
    const int l = (int)msel(advm, (uint32_t)(cz - 1), (uint32_t)s.l);

    // The levels tested: the window [ws, T] of the path (ancestors of the
    // entered cell at level lvl, l <= lvl, T = min(l + 2, lvl) = lvl - dsh),
    // or the child's level. A lane that left the cube tests the root instead
    // (its stepped key is out of range).
    const int dp = (int)msel(advm, (uint32_t)(s.lvl - 1 - cz), (uint32_t)(s.lvl - 2 - s.l));
    const uint32_t dsh = (uint32_t)(dp > 0 ? dp : 0) & 15u;   // levels are < 16
    const int Tp = s.lvl - (int)dsh;
    const int T = (int)bop3<0x20>(msel(pathm, (uint32_t)Tp, (uint32_t)(s.lvl + 1)), missm, 15u);   // & ~miss & 15
    const uint32_t pnm = bop3<0x30>(pathm, missm, missm);   // path & ~miss
    const int ws = (int)msel(pnm, (uint32_t)l, (uint32_t)T);   // ws <= T
    const uint32_t tk = msel(pnm, s.key >> ((3 * dsh) & 31), bop3<0x30>(dk, missm, missm));
    // the word of level wl = max(T, 2) holding the cell (original frame;
    // level D itself on SVOs of depth 1), read as two 32-bit halves
    const int w2 = D < 2 ? D : 2;
    const int wl = (T < w2 ? w2 : T) & 15;
    const uint32_t ko = (tk ^ (s.flip >> (kFine - 3 * T))) << (3 * ((wl - T) & 3));
    const uint64_t W = bits64(woff(wl) + (ko >> 6));
    const uint32_t wlo = (uint32_t)W, whi = (uint32_t)(W >> 32);
    const uint32_t wh = msel(((ko >> 5) & 1u) - 1u, wlo, whi);   // the half holding the cell
    // occupancy of levels wl - 2 (the word), wl - 1 (its byte) and wl (its
    // bit) as 0 / 1; each implies the one before, so the first empty level of
    // the three is wl - 2 + o0 + o1 + o2 (wl + 1: none)
    const uint32_t ow = wlo | whi;
    const uint32_t o0 = ((0u - ow) | ow) >> 31;
    const uint32_t o1 = ((opaque(wh >> (ko & 0x18u)) & 0xffu) + 0xffu) >> 8;
    const uint32_t o2 = opaque(wh >> (ko & 31u)) & 1u;
    // the first empty level of the window [ws, T] (-1: all occupied)
    const int fe = wl - 2 + (int)(o0 + o1 + o2);
    const int c = fe > ws ? fe : ws;
    const uint32_t fullm = neg_mask(T - fe);   // T < c, as ws <= T
    const int ee = (int)((uint32_t)c | fullm);
    const int last = ee >= 0 ? ee : T;
    const int from = ws > count_from ? ws : count_from;
    vis += (missm == 0u && last >= from) ? last - from + 1 : 0;

    // The new cell: on the path the ancestor at the first empty level (the
    // entered cell itself when the window is all occupied); in a descent the
    // child. Its corner: the old corner cut to its level, with the child's
    // half added on each axis for a child.
    const int nl = (int)msel(pathm, msel(fullm, (uint32_t)s.lvl, (uint32_t)c), (uint32_t)(s.lvl + 1));
    const uint32_t MK = 0u - ((1u << kFine) >> nl);
    s.lo0 = bop3<0xEA>(s.lo0, MK, bop3<0x10>(half, pathm, lo0m));   // (lo & MK) | (half & ~path & ~lower)
    s.lo1 = bop3<0xEA>(s.lo1, MK, bop3<0x10>(half, pathm, lo1m));
    s.lo2 = bop3<0xEA>(s.lo2, MK, bop3<0x10>(half, pathm, lo2m));
    s.key = msel(pathm, s.key >> ((3 * ((s.lvl - nl) & 15)) & 31), dk);
    // the window did not reach the cell itself (path lanes only; a descent has T = lvl + 1)
    const uint32_t shortm = neg_mask(T - s.lvl);
    const int lvl0 = s.lvl;
    s.lvl = nl;
    s.phase = (int)(bop3<0x90>(fullm, shortm, 1u) & 3u);   // full ? (short ? PH_PATH : PH_DESCEND) : PH_ADVANCE
    s.l = T + 1;
    // STEP_MISS, else STEP_HIT where the full window reached the leaf (the
    // new level of a full window is lvl on the path, lvl + 1 in a descent)
    const uint32_t hitm = bop3<0x10>(fullm, shortm, neg_mask((int)msel(pathm, (uint32_t)lvl0, (uint32_t)(lvl0 + 1)) - D));
    return (int)(bop3<0x58>(missm, hitm, 1u) & 3u);   // miss ? 2 : (hit ? 1 : 0)
}

// The first step from an occupied origin leaf (the state micro_begin leaves),
// for callers that need the march's result but not its node-test count: the
// leaf's first exit crossing and the face neighbour it enters. nbr(j, up)
// returns whether the neighbour leaf along axis j (up: towards larger
// coordinates of the original frame) is occupied. STEP_MISS when the
// crossing leaves the cube; STEP_HIT when the neighbour is occupied -- the
// hit micro_step reaches from the same state, since the neighbour's
// ancestors are occupied too and the leaf is entered by this crossing (on
// STEP_HIT the hit is hit_of(s, D)); STEP_CONTINUE otherwise, with s no
// longer a valid march state. The kernels take the state-free form below;
// this one, built on the march state, is its reference in the host tests.
template <class Nbr>
WFPG_HD int first_step(MicroState &s, int D, const Nbr &nbr)
{
    const Exit x = exit_crossing(s, 1u << (kFine - D));
    if (x.nlu >= (1u << kFine)) return STEP_MISS;
    s.key = x.akey;
    s.tn = x.tn;
    s.td = x.td;
    s.ta = x.e;
    return nbr(x.e, ((s.mir >> x.e) & 1u) == 0u) ? STEP_HIT : STEP_CONTINUE;
}

// The same first step from per-origin and per-direction quantities, with no
// march state: first_leaf gives, per origin, the distance from O to the
// leaf's upper face (up) and lower face (dn) on each axis (2^-30 units);
// first_exit, per direction (|q| and q < 0 per axis), the exit axis e,
// whether the crossing goes towards larger coordinates, and |B - O| along e
// -- the values first_step computes in its mirrored frame (the lower face of
// a mirrored axis is its upper face there), by the same comparisons.
struct FirstLeaf {
    uint32_t up[3], dn[3];
};
WFPG_HD FirstLeaf first_leaf(const uint32_t O[3], int D)
{
    const uint32_t leaf = 1u << (kFine - D), mk = ~(leaf - 1u);
    FirstLeaf f;
    WFPG_UNROLL
    for (int j = 0; j < 3; ++j) {
        f.up[j] = (O[j] & mk) + leaf - O[j];
        f.dn[j] = O[j] - (O[j] & mk);
    }
    return f;
}
WFPG_HD void first_exit(const FirstLeaf &f, uint32_t aq0, uint32_t aq1, uint32_t aq2, bool n0, bool n1, bool n2,
                        int &e, bool &up, uint32_t &delta)
{
    const uint32_t dl0 = n0 ? f.dn[0] : f.up[0];
    const uint32_t dl1 = n1 ? f.dn[1] : f.up[1];
    const uint32_t dl2 = n2 ? f.dn[2] : f.up[2];
    const bool c1 = (uint64_t)dl1 * aq0 < (uint64_t)dl0 * aq1;   // axis 1 before axis 0
    const uint32_t d01 = c1 ? dl1 : dl0, q01 = c1 ? aq1 : aq0;
    const bool c2 = (uint64_t)dl2 * q01 < (uint64_t)d01 * aq2;   // axis 2 before both
    e = c2 ? 2 : (c1 ? 1 : 0);
    delta = c2 ? dl2 : d01;
    up = !(c2 ? n2 : (c1 ? n1 : n0));
}

// The hit of a march whose last step returned STEP_HIT: the crossing axis, the
// leaf key in the original frame, and |B - O| of the crossing.
WFPG_HD Hit hit_of(const MicroState &s, int D)
{
    Hit h;
    h.axis = s.ta;
    h.key = s.key ^ (s.flip >> (kFine - 3 * D));
    h.delta = s.tn;
    return h;
}

// Whole march: 1 on a hit, 0 on a miss, -1 if the iteration bound is
// exceeded (never expected).
template <class Bits, class Bits64>
WFPG_HD int march(const uint32_t O[3], int q0, int q1, int q2, int D, const Bits &bits, const Bits64 &bits64,
                  int count_from, int &vis, Hit &h)
{
    MicroState s;
    uint32_t aq0, aq1, aq2;
    int sg0, sg1, sg2;
    split_dir(q0, aq0, sg0);
    split_dir(q1, aq1, sg1);
    split_dir(q2, aq2, sg2);
    const uint32_t ok = morton3(O[0] >> (kFine - D), O[1] >> (kFine - D), O[2] >> (kFine - D));
    const bool occ = occupied(bits, D, ok);
    micro_begin(s, O, ok, occ, aq0, aq1, aq2, sg0, sg1, sg2, D, count_from, vis);
    for (int it = 0; it < kMaxTests; ++it) {
        const int st = micro_step(s, D, bits64, count_from, vis);
        if (st == STEP_HIT) {
            h = hit_of(s, D);
            return 1;
        }
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
    const float scale = __builtin_ldexpf(1.0f, D - kFine);   // exactly 2^-(30-D)
    const float dist = ((float)delta * scale) / dabs;
    const float sq = dist * dist;
    const float A = sq * omega;
    // The thresholds 2.5 * 4^(j-1) are 1.25 * 2^(2j-1): with A = m 2^e,
    // m in [1, 2), A exceeds the j-th iff 2j - 1 < e, or 2j - 1 = e and
    // m > 1.25, so k = floor(e / 2) plus one when e is odd and m > 1.25,
    // capped at D (the same count as comparing with each threshold in turn).
    if (!(A > 2.5f)) return 0;                 // also NaN
    if (A > 3.40282347e38f) return D;          // infinity
    int e;
    const float m = __builtin_frexpf(A, &e);   // A = m 2^e, m in [0.5, 1)
    --e;
    const int k = (e >> 1) + (((e & 1) != 0) && m > 0.625f ? 1 : 0);
    return k < D ? k : D;
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
