// Field antialiasing (Sec. 4): directional jitter of the cone directions and
// a Gaussian blur of the field over the octahedral square.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "march_core.h"

namespace wfpg {
namespace aa {

// Cone direction of bin b = v N + u under jitter key `key`: the map's decode of
// ((u + j_u) / N, (v + j_v) / N), (j_u, j_v) = the first two words of
// Philox-4x32-10 at counter (b, 0, 0, 3), key (key, 0), each (bits >> 8) *
// 2^-24. Decoded in FP64 and rounded to FP32, as the bin-centre table is.
__device__ inline void jitter_dir(int N, int b, uint32_t key, float &x, float &y, float &z)
{
    uint32_t c[4] = {(uint32_t)b, 0u, 0u, 3u};
    core::philox(c, key, 0u);
    const int u = b % N, v = b / N;
    const double ju = (double)(c[0] >> 8) * (1.0 / 16777216.0);
    const double jv = (double)(c[1] >> 8) * (1.0 / 16777216.0);
    const double a = 2.0 * (((double)u + ju) / N) - 1.0;
    const double bb = 2.0 * (((double)v + jv) / N) - 1.0;
    const double aa = fabs(a), ab = fabs(bb);
    const double d = 1.0 - (aa + ab);
    const double r = 1.0 - fabs(d);
    const double phi = (r == 0.0) ? 0.0 : ((ab - aa) / r + 1.0) * 0.78539816339744830962;
    const double s = r * sqrt(2.0 - r * r);
    x = (float)((a >= 0.0 ? 1.0 : -1.0) * cos(phi) * s);
    y = (float)((bb >= 0.0 ? 1.0 : -1.0) * sin(phi) * s);
    z = (float)((d >= 0.0 ? 1.0 : -1.0) * (1.0 - r * r));
}

// Neighbours across the square's edges: the map sends (1, b) and (1, -b)
// (and likewise on the other edges) to one direction, so bin (N, v) is bin
// (N - 1, N - 1 - v) and bin (u, N) is bin (N - 1 - u, N - 1); corners fold
// twice.
__device__ __forceinline__ void fold_bin(int N, int &u, int &v)
{
    if (u < 0) { u = 0; v = N - 1 - v; }
    else if (u >= N) { u = N - 1; v = N - 1 - v; }
    if (v < 0) { v = 0; u = N - 1 - u; }
    else if (v >= N) { v = N - 1; u = N - 1 - u; }
}

// Blurred value of bin (u, v): the 3 x 3 binomial kernel (1/4, 1/2, 1/4) in
// each direction, rows dy outer and columns dx inner, FP32; ld(k) returns the
// field value of bin k.
template <typename Load>
__device__ __forceinline__ float blur_at(int N, int u, int v, Load ld)
{
    float acc = 0.f;
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {   // rolled: the nine taps stay off the register budget
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        int uu = u + dx, vv = v + dy;
        fold_bin(N, uu, vv);
        const float w = (dx == 0 ? 0.5f : 0.25f) * (dy == 0 ? 0.5f : 0.25f);
        acc += w * ld(vv * N + uu);
    }
    return acc;
}

}  // namespace aa
}  // namespace wfpg
