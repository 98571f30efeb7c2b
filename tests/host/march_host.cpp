// Host build of the library's traversal core (paper_2405_06997_amd/csrc/
// march_core.h) for the CPU test suite: the same source the gfx950 kernels
// run, driven here over arrays the test builds from the oracle's SVO.
#include <stdint.h>

#include "../../paper_2405_06997_amd/csrc/march_core.h"

using namespace wfpg::core;

extern "C" void host_debug_march(const uint64_t *bits, const uint32_t *rank, const int64_t *noff,
                                 const float *nrm, int D, const float *pos, int64_t n,
                                 const float *dirtab, int N, float omega, int32_t *out,
                                 int32_t *visits)
{
    const int NN = N * N;
    const uint32_t *bits32 = reinterpret_cast<const uint32_t *>(bits);   // 32-bit words
    auto load = [&](int, uint32_t wi) -> uint32_t { return bits32[wi]; };
    auto load64 = [&](uint32_t wi) -> uint64_t { return bits[wi]; };
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t O[3];
        for (int k = 0; k < 3; ++k) O[k] = quantize_pos(pos[k * n + i]);
        for (int b = 0; b < NN; ++b) {
            const float *d = dirtab + 3 * b;
            int vis = 0;
            Hit h = {-1, 0u, 0u};
            const int res = march(O, quantize_dir(d[0]), quantize_dir(d[1]), quantize_dir(d[2]), D,
                                  load, load64, 5, vis, h);
            int32_t *o = out + ((int64_t)i * NN + b) * 8;
            o[0] = res > 0;
            o[1] = res > 0 ? h.axis : -1;
            o[2] = res > 0 ? (int32_t)h.key : -1;
            o[3] = res > 0 ? (int32_t)h.delta : -1;
            o[4] = -1; o[5] = -1; o[6] = -1; o[7] = 0;
            if (res > 0) {
                const float da = d[h.axis] < 0 ? -d[h.axis] : d[h.axis];
                const int k = footprint_levels(h.delta, da, D, omega);
                const int lf = D - k;
                const uint32_t node = h.key >> (3 * k);
                const uint32_t wi = woff(lf) + (node >> 6);
                const uint64_t w = bits[wi];
                const uint64_t m = (node & 63) ? (w & ((1ull << (node & 63)) - 1)) : 0ull;
                const int64_t g = (int64_t)rank[wi] + __builtin_popcountll(m);
                const float *nn = nrm + 3 * g;
                o[4] = k;
                o[5] = (int32_t)node;
                o[6] = (int32_t)(g - noff[lf]);
                o[7] = dot3(nn[0], nn[1], nn[2], d[0], d[1], d[2]) < 0.f ? 0 : 1;
            }
            visits[(int64_t)i * NN + b] = res < 0 ? -1 : vis;
        }
    }
}

// One march per (point, direction) pair for arbitrary directions (axis-aligned
// and other directions with zero components included): out = {hit, axis, key,
// delta} per pair, point-major.
extern "C" void host_march_dirs(const uint64_t *bits, int D, const float *pos, int64_t n, const float *dirs,
                                int nd, int64_t *out)
{
    const uint32_t *bits32 = reinterpret_cast<const uint32_t *>(bits);
    auto load = [&](int, uint32_t wi) -> uint32_t { return bits32[wi]; };
    auto load64 = [&](uint32_t wi) -> uint64_t { return bits[wi]; };
    for (int64_t i = 0; i < n; ++i) {
        uint32_t O[3];
        for (int k = 0; k < 3; ++k) O[k] = quantize_pos(pos[k * n + i]);
        for (int b = 0; b < nd; ++b) {
            const float *d = dirs + 3 * b;
            int vis = 0;
            Hit h = {-1, 0u, 0u};
            const int res = march(O, quantize_dir(d[0]), quantize_dir(d[1]), quantize_dir(d[2]), D, load, load64, 0,
                                  vis, h);
            int64_t *o = out + (i * nd + b) * 4;
            o[0] = res;
            o[1] = res > 0 ? h.axis : -1;
            o[2] = res > 0 ? (int64_t)h.key : -1;
            o[3] = res > 0 ? (int64_t)h.delta : -1;
        }
    }
}

// Footprint level of the library for given (delta, |d_axis|, D, omega).
extern "C" int host_footprint_levels(uint32_t delta, float dabs, int D, float omega)
{
    return footprint_levels(delta, dabs, D, omega);
}

// The first step from an occupied origin leaf taken from the occupancy of the
// leaf's face neighbours (first_step), per (point, direction) pair: out =
// {result, axis, key, delta} with result 1 hit, 2 miss, 0 continue (axis, key
// and delta then those of the crossing into the empty neighbour), -1 when the
// origin leaf is empty (no first step taken), -2 when the same step taken with
// no march state (first_leaf, first_exit) disagrees.
extern "C" void host_first_step_dirs(const uint64_t *bits, int D, const float *pos, int64_t n, const float *dirs,
                                     int nd, int64_t *out)
{
    const uint32_t *bits32 = reinterpret_cast<const uint32_t *>(bits);
    auto load = [&](int, uint32_t wi) -> uint32_t { return bits32[wi]; };
    for (int64_t i = 0; i < n; ++i) {
        uint32_t O[3];
        for (int k = 0; k < 3; ++k) O[k] = quantize_pos(pos[k * n + i]);
        const uint32_t c[3] = {O[0] >> (kFine - D), O[1] >> (kFine - D), O[2] >> (kFine - D)};
        const uint32_t ok = morton3(c[0], c[1], c[2]);
        const bool occ = occupied(load, D, ok);
        auto nbr = [&](int ax, bool up) {
            uint32_t cc[3] = {c[0], c[1], c[2]};
            cc[ax] = up ? cc[ax] + 1u : cc[ax] - 1u;
            return cc[ax] < (1u << D) && occupied(load, D, morton3(cc[0], cc[1], cc[2]));
        };
        for (int b = 0; b < nd; ++b) {
            int64_t *o = out + (i * nd + b) * 4;
            if (!occ) {
                o[0] = -1; o[1] = -1; o[2] = -1; o[3] = -1;
                continue;
            }
            const float *d = dirs + 3 * b;
            uint32_t aq[3];
            int sg[3];
            for (int k = 0; k < 3; ++k) split_dir(quantize_dir(d[k]), aq[k], sg[k]);
            MicroState s;
            int vis = 0;
            micro_begin(s, O, ok, true, aq[0], aq[1], aq[2], sg[0], sg[1], sg[2], D, 0, vis);
            const int r = first_step(s, D, nbr);
            const Hit h = hit_of(s, D);
            o[0] = r == STEP_HIT ? 1 : (r == STEP_MISS ? 2 : 0);
            o[1] = r == STEP_MISS ? -1 : h.axis;
            o[2] = r == STEP_MISS ? -1 : (int64_t)h.key;
            o[3] = r == STEP_MISS ? -1 : (int64_t)h.delta;
            // the same step with no march state (first_leaf, first_exit) must agree
            int e;
            bool up;
            uint32_t delta;
            first_exit(first_leaf(O, D), aq[0], aq[1], aq[2], sg[0] < 0, sg[1] < 0, sg[2] < 0, e, up, delta);
            uint32_t cc[3] = {c[0], c[1], c[2]};
            cc[e] = up ? cc[e] + 1u : cc[e] - 1u;
            const bool inside = cc[e] < (1u << D);
            const uint32_t nk = morton3(cc[0], cc[1], cc[2]);
            const int r2 = !inside ? STEP_MISS : (occupied(load, D, nk) ? STEP_HIT : STEP_CONTINUE);
            if (r2 != r || (r != STEP_MISS && (e != h.axis || nk != h.key || delta != h.delta))) o[0] = -2;
        }
    }
}
