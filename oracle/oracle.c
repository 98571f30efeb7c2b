/*
 * CPU oracle for wavefront path guiding with an exitance SVO
 * (Yalciner & Akyuz, "Path Guiding for Wavefront Path Tracing", 2024).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * GPU library is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header, table
 * or constant generator with the GPU library, and the library never calls it.
 *
 * Precision: values that the method leaves free (PDF, CDF, exitance "truth")
 * are FP64. Decisions that pick an integer (voxel normal clustering, footprint
 * level, exitance side) are taken in FP32 with a fixed operation order and no
 * fused multiply-add, because the paper keeps its field in FP32 (Sec. 3.4,
 * 64 KiB for a 128x128 field) and both sides must take such decisions in the
 * same precision. Build with -ffp-contract=off.
 *
 * Readings of the paper that this file fixes (each one is stated where it is
 * used): half-open voxelization, deterministic k-means seed, first occupied
 * leaf by an exact 6-connected DDA, linear "closest area" level, side selection
 * by the sign of the normal/direction dot product, additive epsilon, mean
 * exitance per leaf, side-aligned bottom-up averaging, Philox-4x32-10 uniforms.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 10
#define MAXN 128 /* largest field resolution (bins per side) */
#define FINE 30 /* positions are quantized to 2^30 steps per unit length */

typedef struct {
    int32_t axis;
    float c;
    float lo[2], hi[2];
    int32_t sign;
    int32_t emissive;
} orc_rect;

typedef struct {
    int depth;
    int64_t n[MAXD + 1];
    uint32_t *keys[MAXD + 1];   /* sorted Morton keys per level */
    float *nrm[MAXD + 1];       /* 3 per node */
    float *e32[MAXD + 1];       /* 2 per node, FP32 computed in the stated order */
    double *e64[MAXD + 1];      /* 2 per node, FP64 "truth" */
    int32_t *leaf_xyz;          /* 3 per leaf */
    uint8_t *leaf_emissive;
    float *s32;                 /* 2 per leaf: FP32 splat sums (splat order) */
    double *s64;
    int64_t *cnt;               /* 2 per leaf */
    int64_t dropped;
    int fmt;                    /* 0 FP32, 1 FP16, 2 BF16: storage of E and L_b */
} orc_svo;

/* ---------------------------------------------------------------- Morton -- */
/* Interleave bits: x in bit 3i, y in bit 3i+1, z in bit 3i+2. Written as a
 * plain loop over bits. */
uint32_t orc_morton(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t k = 0;
    for (int i = 0; i < 10; i++) {
        k |= ((x >> i) & 1u) << (3 * i);
        k |= ((y >> i) & 1u) << (3 * i + 1);
        k |= ((z >> i) & 1u) << (3 * i + 2);
    }
    return k;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

static int64_t find_key(const uint32_t *keys, int64_t n, uint32_t k)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (keys[mid] == k) return mid;
        if (keys[mid] < k) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ----------------------------------------------------- FP32 helpers ------ */
/* dot = (x*x' + y*y') + z*z' in FP32, each product rounded, no FMA. */
static float dot3f(const float *a, const float *b)
{
    float px = a[0] * b[0];
    float py = a[1] * b[1];
    float pz = a[2] * b[2];
    float s = px + py;
    return s + pz;
}

/* Round FP32 to bfloat16, round-to-nearest-even (NaN kept quiet). */
static uint16_t f32_to_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
static float bf16_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* Round FP32 to IEEE binary16, round-to-nearest-even, with subnormals and
 * overflow to infinity. Written from the format definition. */
static uint16_t f32_to_f16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t sign = (u >> 16) & 0x8000u;
    uint32_t ex = (u >> 23) & 0xffu;
    uint32_t man = u & 0x7fffffu;
    if (ex == 0xff) return (uint16_t)(sign | 0x7c00u | (man ? 0x200u : 0));
    int e = (int)ex - 127;            /* unbiased exponent */
    if (e > 15) return (uint16_t)(sign | 0x7c00u);
    if (e >= -14) {                   /* normal half */
        uint32_t m = man | 0x800000u; /* 24-bit significand */
        uint32_t keep = m >> 13, rest = m & 0x1fffu;
        if (rest > 0x1000u || (rest == 0x1000u && (keep & 1u))) keep++;
        uint32_t he = (uint32_t)(e + 15);
        if (keep == 0x800u) { keep = 0x400u; he++; }
        if (he >= 31) return (uint16_t)(sign | 0x7c00u);
        return (uint16_t)(sign | (he << 10) | (keep & 0x3ffu));
    }
    /* subnormal half: value = m * 2^(e-23), target unit 2^-24 */
    if (ex == 0) return (uint16_t)sign;  /* FP32 subnormals round to zero */
    uint32_t m = man | 0x800000u;
    int shift = -e - 1;               /* = (-14 - e) + 13 */
    if (shift > 24) return (uint16_t)sign;
    uint32_t keep = m >> shift;
    uint32_t rest = m & ((1u << shift) - 1u);
    uint32_t half = 1u << (shift - 1);
    if (rest > half || (rest == half && (keep & 1u))) keep++;
    return (uint16_t)(sign | keep);   /* keep may carry into the exponent: fine */
}
static float f16_to_f32(uint16_t h)
{
    uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    float v;
    if (e == 0) v = ldexpf((float)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexpf((float)(m | 0x400u), (int)e - 25);
    uint32_t u;
    memcpy(&u, &v, 4);
    u |= sign;
    memcpy(&v, &u, 4);
    return v;
}
float orc_round_fmt(float f, int fmt)
{
    if (fmt == 1) return f16_to_f32(f32_to_f16(f));
    if (fmt == 2) return bf16_to_f32(f32_to_bf16(f));
    return f;
}

/* ------------------------------------------------- concentric octahedral -- */
/* Equal-area concentric octahedral map (Clarberg 2008), cited by the paper for
 * projecting the radiance field to a square (Sec. 4, "Radiance field
 * projection"). Square coordinates (x, y) in [0,1]^2; a = 2x-1, b = 2y-1;
 * the square's centre maps to +z and its corners to -z. FP64. */
void orc_oct_decode(double x, double y, double *out)
{
    double a = 2.0 * x - 1.0, b = 2.0 * y - 1.0;
    double aa = fabs(a), ab = fabs(b);
    double d = 1.0 - (aa + ab);
    double r = 1.0 - fabs(d);
    double phi = (r == 0.0) ? 0.0 : ((ab - aa) / r + 1.0) * (M_PI / 4.0);
    double z = (d >= 0.0 ? 1.0 : -1.0) * (1.0 - r * r);
    double s = r * sqrt(2.0 - r * r);
    out[0] = (a >= 0.0 ? 1.0 : -1.0) * cos(phi) * s;
    out[1] = (b >= 0.0 ? 1.0 : -1.0) * sin(phi) * s;
    out[2] = z;
}

void orc_oct_encode(double dx, double dy, double dz, double *xy)
{
    double r = sqrt(1.0 - fabs(dz));
    double phi = atan2(fabs(dy), fabs(dx));
    double t = 2.0 * r * phi / M_PI;
    double aa = r - t, ab = t;
    if (dz < 0.0) {
        double na = 1.0 - ab, nb = 1.0 - aa;
        aa = na;
        ab = nb;
    }
    double a = (dx >= 0.0 ? aa : -aa), b = (dy >= 0.0 ? ab : -ab);
    xy[0] = (a + 1.0) * 0.5;
    xy[1] = (b + 1.0) * 0.5;
}

/* Direction of every bin centre, bins b = v*N + u (rows are v), rounded to
 * FP32 from the FP64 decode. Equal-area map => each bin spans 4*pi/N^2 sr,
 * the paper's "equal solid angle patches" (Sec. 3.3). */
void orc_dir_table(int N, float *out)
{
    for (int v = 0; v < N; v++)
        for (int u = 0; u < N; u++) {
            double d[3];
            orc_oct_decode((u + 0.5) / N, (v + 0.5) / N, d);
            for (int k = 0; k < 3; k++) out[3 * (v * N + u) + k] = (float)d[k];
        }
}

/* --------------------------------------------------------- Philox ------- */
/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplications with a Weyl-sequence key schedule. */
void orc_philox(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out)
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four uniforms in [0,1) for query i of a bounce: counter (i_lo, i_hi,
 * bounce, 0), key (seed_lo, seed_hi), u = (bits >> 8) * 2^-24. */
static void uniforms(uint64_t seed, uint32_t bounce, int64_t i, double u[4])
{
    uint32_t ctr[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), bounce, 0};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox(ctr, key, o);
    for (int k = 0; k < 4; k++) u[k] = (double)(o[k] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------ build ----- */
typedef struct { uint32_t key; int32_t rect; } frag_t;
static int cmp_frag(const void *a, const void *b)
{
    const frag_t *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->rect > y->rect) - (x->rect < y->rect);
}

/* k-means with k = 2 over unit vectors v[0..m) (Sec. 3.2, Fig. 2). The paper
 * seeds with a random member and its opposite; here the seed is member 0 so
 * that both sides agree. Assignment to A iff dot(v, muA) >= dot(v, muB);
 * a mean is the normalized sum of its members in order; an empty cluster
 * keeps its mean; at most 16 rounds; the result is cluster A's mean. */
static void kmeans2(const float *v, int m, float *out)
{
    float muA[3] = {v[0], v[1], v[2]};
    float muB[3] = {-v[0], -v[1], -v[2]};
    int *asg = malloc(sizeof(int) * (size_t)m);
    for (int i = 0; i < m; i++) asg[i] = -1;
    for (int it = 0; it < 16; it++) {
        int changed = 0;
        for (int i = 0; i < m; i++) {
            int a = dot3f(v + 3 * i, muA) >= dot3f(v + 3 * i, muB) ? 0 : 1;
            if (a != asg[i]) changed = 1;
            asg[i] = a;
        }
        if (!changed) break;
        float sA[3] = {0, 0, 0}, sB[3] = {0, 0, 0};
        int nA = 0, nB = 0;
        for (int i = 0; i < m; i++) {
            float *s = asg[i] == 0 ? sA : sB;
            for (int k = 0; k < 3; k++) s[k] = s[k] + v[3 * i + k];
            if (asg[i] == 0) nA++; else nB++;
        }
        if (nA) {
            float len = sqrtf(dot3f(sA, sA));
            for (int k = 0; k < 3; k++) muA[k] = sA[k] / len;
        }
        if (nB) {
            float len = sqrtf(dot3f(sB, sB));
            for (int k = 0; k < 3; k++) muB[k] = sB[k] / len;
        }
    }
    free(asg);
    out[0] = muA[0]; out[1] = muA[1]; out[2] = muA[2];
}

/* Leaf index range of a rectangle along one axis. Half-open reading of the
 * paper's conservative voxelization (Sec. 3.2): the cells whose half-open
 * extent meets the open interval (lo, hi), or the single cell holding lo when
 * lo == hi. Along the plane axis the single cell floor(c * 2^D). */
static void cell_range(float lo, float hi, int D, int *i0, int *i1)
{
    int R = 1 << D;
    float sl = lo * (float)R, sh = hi * (float)R;   /* exact scalings */
    int a = (int)floorf(sl);
    int b = (int)ceilf(sh) - 1;
    if (b < a) b = a;
    if (a < 0) a = 0;
    if (b > R - 1) b = R - 1;
    if (a > R - 1) a = R - 1;
    if (b < 0) b = 0;
    *i0 = a;
    *i1 = b;
}

void orc_free(orc_svo *s);

/* Build the SVO (Sec. 3.2): voxelize, sort fragments by Morton key (Karras
 * 2012 hierarchy from sorted keys), unique keys per level, k-means normals.
 * status: 0 ok, -1 bad argument, -2 out of memory. */
orc_svo *orc_build(const orc_rect *rects, int64_t nr, int32_t depth, int32_t *status)
{
    *status = -1;
    if (depth < 1 || depth > MAXD || nr < 0) return NULL;
    for (int64_t i = 0; i < nr; i++) {
        const orc_rect *r = rects + i;
        if (r->axis < 0 || r->axis > 2) return NULL;
        if (!isfinite(r->c) || !isfinite(r->lo[0]) || !isfinite(r->lo[1]) ||
            !isfinite(r->hi[0]) || !isfinite(r->hi[1])) return NULL;
        if (r->lo[0] > r->hi[0] || r->lo[1] > r->hi[1]) return NULL;
        if (r->sign != 1 && r->sign != -1) return NULL;
    }
    *status = -2;
    orc_svo *s = calloc(1, sizeof(orc_svo));
    if (!s) return NULL;
    s->depth = depth;
    int D = depth, R = 1 << D;
    /* fragments */
    int64_t nf = 0;
    for (int64_t i = 0; i < nr; i++) {
        int a0, a1, b0, b1;
        cell_range(rects[i].lo[0], rects[i].hi[0], D, &a0, &a1);
        cell_range(rects[i].lo[1], rects[i].hi[1], D, &b0, &b1);
        nf += (int64_t)(a1 - a0 + 1) * (b1 - b0 + 1);
    }
    frag_t *fr = malloc(sizeof(frag_t) * (size_t)(nf ? nf : 1));
    if (!fr) { free(s); return NULL; }
    int64_t f = 0;
    for (int64_t i = 0; i < nr; i++) {
        const orc_rect *r = rects + i;
        int ax = r->axis, j0 = ax == 0 ? 1 : 0, j1 = ax == 2 ? 1 : 2;
        int a0, a1, b0, b1, ca;
        cell_range(r->lo[0], r->hi[0], D, &a0, &a1);
        cell_range(r->lo[1], r->hi[1], D, &b0, &b1);
        cell_range(r->c, r->c, D, &ca, &ca);
        for (int p = a0; p <= a1; p++)
            for (int q = b0; q <= b1; q++) {
                uint32_t c[3];
                c[ax] = (uint32_t)ca; c[j0] = (uint32_t)p; c[j1] = (uint32_t)q;
                fr[f].key = orc_morton(c[0], c[1], c[2]);
                fr[f].rect = (int32_t)i;
                f++;
            }
    }
    qsort(fr, (size_t)nf, sizeof(frag_t), cmp_frag);
    /* leaves */
    int64_t L = 0;
    for (int64_t i = 0; i < nf; i++)
        if (i == 0 || fr[i].key != fr[i - 1].key) L++;
    s->n[D] = L;
    s->keys[D] = malloc(sizeof(uint32_t) * (size_t)(L ? L : 1));
    int64_t *off = malloc(sizeof(int64_t) * (size_t)(L + 1));
    s->leaf_xyz = calloc((size_t)(3 * L + 1), sizeof(int32_t));
    s->leaf_emissive = calloc((size_t)(L + 1), 1);
    {
        int64_t l = -1;
        for (int64_t i = 0; i < nf; i++) {
            if (i == 0 || fr[i].key != fr[i - 1].key) {
                l++;
                s->keys[D][l] = fr[i].key;
                off[l] = i;
            }
            if (rects[fr[i].rect].emissive) s->leaf_emissive[l] = 1;
        }
        off[L] = nf;
    }
    for (int64_t l = 0; l < L; l++) {
        uint32_t k = s->keys[D][l], x = 0, y = 0, z = 0;
        for (int i = 0; i < D; i++) {
            x |= ((k >> (3 * i)) & 1u) << i;
            y |= ((k >> (3 * i + 1)) & 1u) << i;
            z |= ((k >> (3 * i + 2)) & 1u) << i;
        }
        s->leaf_xyz[3 * l] = (int32_t)x;
        s->leaf_xyz[3 * l + 1] = (int32_t)y;
        s->leaf_xyz[3 * l + 2] = (int32_t)z;
    }
    (void)R;
    /* inner levels: unique parents */
    for (int lv = D - 1; lv >= 0; lv--) {
        int64_t nc = s->n[lv + 1], np = 0;
        uint32_t *pk = malloc(sizeof(uint32_t) * (size_t)(nc ? nc : 1));
        for (int64_t i = 0; i < nc; i++) {
            uint32_t p = s->keys[lv + 1][i] >> 3;
            if (np == 0 || pk[np - 1] != p) pk[np++] = p;
        }
        s->n[lv] = np;
        s->keys[lv] = pk;
    }
    /* leaf normals from fragment normals, fragments in rectangle order */
    s->nrm[D] = malloc(sizeof(float) * (size_t)(3 * L + 3));
    {
        float *buf = NULL;
        int64_t cap = 0;
        for (int64_t l = 0; l < L; l++) {
            int64_t m = off[l + 1] - off[l];
            if (m > cap) { cap = m; buf = realloc(buf, sizeof(float) * (size_t)(3 * cap)); }
            for (int64_t i = 0; i < m; i++) {
                const orc_rect *r = rects + fr[off[l] + i].rect;
                buf[3 * i] = buf[3 * i + 1] = buf[3 * i + 2] = 0.0f;
                buf[3 * i + r->axis] = (float)r->sign;
            }
            kmeans2(buf, (int)m, s->nrm[D] + 3 * l);
        }
        free(buf);
    }
    /* inner normals: the same clustering over the children's normals in
     * octant order, seeded with the first child (the paper stores two normals
     * per node but does not say how inner ones are formed). */
    for (int lv = D - 1; lv >= 0; lv--) {
        int64_t np = s->n[lv];
        s->nrm[lv] = malloc(sizeof(float) * (size_t)(3 * np + 3));
        int64_t c = 0;
        for (int64_t p = 0; p < np; p++) {
            float buf[24];
            int m = 0;
            while (c < s->n[lv + 1] && (s->keys[lv + 1][c] >> 3) == s->keys[lv][p]) {
                memcpy(buf + 3 * m, s->nrm[lv + 1] + 3 * c, 3 * sizeof(float));
                m++;
                c++;
            }
            kmeans2(buf, m, s->nrm[lv] + 3 * p);
        }
    }
    for (int lv = 0; lv <= D; lv++) {
        s->e32[lv] = calloc((size_t)(2 * s->n[lv] + 2), sizeof(float));
        s->e64[lv] = calloc((size_t)(2 * s->n[lv] + 2), sizeof(double));
    }
    s->s32 = calloc((size_t)(2 * L + 2), sizeof(float));
    s->s64 = calloc((size_t)(2 * L + 2), sizeof(double));
    s->cnt = calloc((size_t)(2 * L + 2), sizeof(int64_t));
    free(off);
    free(fr);
    *status = 0;
    return s;
}

void orc_free(orc_svo *s)
{
    if (!s) return;
    for (int l = 0; l <= MAXD; l++) {
        free(s->keys[l]); free(s->nrm[l]); free(s->e32[l]); free(s->e64[l]);
    }
    free(s->leaf_xyz); free(s->leaf_emissive);
    free(s->s32); free(s->s64); free(s->cnt);
    free(s);
}

int32_t orc_depth(const orc_svo *s) { return s->depth; }
int64_t orc_level_size(const orc_svo *s, int32_t l) { return s->n[l]; }
void orc_level_keys(const orc_svo *s, int32_t l, uint32_t *out)
{
    memcpy(out, s->keys[l], sizeof(uint32_t) * (size_t)s->n[l]);
}
void orc_level_normals(const orc_svo *s, int32_t l, float *out)
{
    memcpy(out, s->nrm[l], sizeof(float) * (size_t)(3 * s->n[l]));
}
void orc_level_exitance(const orc_svo *s, int32_t l, float *e32, double *e64)
{
    if (e32) memcpy(e32, s->e32[l], sizeof(float) * (size_t)(2 * s->n[l]));
    if (e64) memcpy(e64, s->e64[l], sizeof(double) * (size_t)(2 * s->n[l]));
}
void orc_leaf_info(const orc_svo *s, int32_t *xyz, uint8_t *emissive)
{
    int64_t L = s->n[s->depth];
    if (xyz) memcpy(xyz, s->leaf_xyz, sizeof(int32_t) * (size_t)(3 * L));
    if (emissive) memcpy(emissive, s->leaf_emissive, (size_t)L);
}
void orc_leaf_accum(const orc_svo *s, float *s32, double *s64, int64_t *cnt)
{
    int64_t L = s->n[s->depth];
    if (s32) memcpy(s32, s->s32, sizeof(float) * (size_t)(2 * L));
    if (s64) memcpy(s64, s->s64, sizeof(double) * (size_t)(2 * L));
    if (cnt) memcpy(cnt, s->cnt, sizeof(int64_t) * (size_t)(2 * L));
}
int64_t orc_dropped(const orc_svo *s) { return s->dropped; }

/* Overwrite the stored exitance of every node of every level with value v on
 * both sides (test helper for closed-form checks). */
void orc_set_uniform_exitance(orc_svo *s, float v)
{
    for (int l = 0; l <= s->depth; l++)
        for (int64_t i = 0; i < 2 * s->n[l]; i++) { s->e32[l][i] = v; s->e64[l][i] = v; }
}

/* ---------------------------------------------- UpdateExitance / splat ---- */
/* Leaf cell of a position: c = min(floor(p * 2^D), 2^D - 1) per axis; the
 * point must lie in [0,1]^3. Returns 0 if outside. */
static int leaf_cell(const float *p, int D, uint32_t *c)
{
    for (int k = 0; k < 3; k++) {
        if (!(p[k] >= 0.0f && p[k] <= 1.0f)) return 0;
        int v = (int)floorf(p[k] * (float)(1 << D));
        if (v > (1 << D) - 1) v = (1 << D) - 1;
        c[k] = (uint32_t)v;
    }
    return 1;
}

/* Splat exitance estimates into the leaves (Sec. 3.2, "UpdateExitance", after
 * Eq. 5): the path vertex is mapped to its leaf and its local radiance
 * estimate is accumulated. Colour -> scalar by Rec. 709 luminance (reading;
 * the paper is silent). The side is the one whose normal faces the outgoing
 * direction: 0 iff dot(N_leaf, wo) >= 0. Inputs that are not finite, have
 * negative luminance or fall outside the occupied leaves are dropped and
 * counted. SoA inputs (3 planes of n). Returns the number dropped. */
int64_t orc_accumulate(orc_svo *s, const float *pos, const float *wo, const float *rgb, int64_t n)
{
    int D = s->depth;
    int64_t L = s->n[D], dropped = 0;
    for (int64_t i = 0; i < n; i++) {
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        float w[3] = {wo[i], wo[n + i], wo[2 * n + i]};
        float c3[3] = {rgb[i], rgb[n + i], rgb[2 * n + i]};
        int ok = 1;
        for (int k = 0; k < 3; k++)
            if (!isfinite(p[k]) || !isfinite(w[k]) || !isfinite(c3[k])) ok = 0;
        float t0 = 0.2126f * c3[0];
        float t1 = 0.7152f * c3[1];
        float t2 = 0.0722f * c3[2];
        float y = (t0 + t1) + t2;
        if (!(y >= 0.0f) || !isfinite(y)) ok = 0;
        uint32_t c[3];
        int64_t leaf = -1;
        if (ok && leaf_cell(p, D, c)) leaf = find_key(s->keys[D], L, orc_morton(c[0], c[1], c[2]));
        if (leaf < 0) { dropped++; continue; }
        int side = dot3f(s->nrm[D] + 3 * leaf, w) >= 0.0f ? 0 : 1;
        s->s32[2 * leaf + side] = s->s32[2 * leaf + side] + y;
        s->s64[2 * leaf + side] += (double)y;
        s->cnt[2 * leaf + side] += 1;
    }
    s->dropped += dropped;
    return dropped;
}

/* Bottom-up averaging (Sec. 3.2): a leaf side's exitance is the mean of its
 * splats (0 without splats); an inner node side is the mean over its occupied
 * children, in octant order, of the child side that faces the same way
 * (child side flipped when dot(N_child, N_parent) < 0). FP32 in that order
 * (e32) and FP64 (e64). fmt selects the storage format of the field. */
void orc_propagate(orc_svo *s, int32_t fmt)
{
    int D = s->depth;
    s->fmt = fmt;
    for (int64_t l = 0; l < s->n[D]; l++)
        for (int k = 0; k < 2; k++) {
            int64_t c = s->cnt[2 * l + k];
            s->e32[D][2 * l + k] = c > 0 ? s->s32[2 * l + k] / (float)c : 0.0f;
            s->e64[D][2 * l + k] = c > 0 ? s->s64[2 * l + k] / (double)c : 0.0;
        }
    for (int lv = D - 1; lv >= 0; lv--) {
        int64_t c = 0;
        for (int64_t p = 0; p < s->n[lv]; p++) {
            float a32[2] = {0.0f, 0.0f};
            double a64[2] = {0.0, 0.0};
            int m = 0;
            while (c < s->n[lv + 1] && (s->keys[lv + 1][c] >> 3) == s->keys[lv][p]) {
                int flip = dot3f(s->nrm[lv + 1] + 3 * c, s->nrm[lv] + 3 * p) >= 0.0f ? 0 : 1;
                for (int k = 0; k < 2; k++) {
                    a32[k] = a32[k] + s->e32[lv + 1][2 * c + (k ^ flip)];
                    a64[k] += s->e64[lv + 1][2 * c + (k ^ flip)];
                }
                m++;
                c++;
            }
            for (int k = 0; k < 2; k++) {
                s->e32[lv][2 * p + k] = a32[k] / (float)m;
                s->e64[lv][2 * p + k] = a64[k] / (double)m;
            }
        }
    }
}

/* ------------------------------------------------------------- march ---- */
/* Quantized ray: O = clamp(rint(p * 2^30), 0, 2^30-1), q = rint(d * 2^23). */
typedef struct { int64_t O[3], q[3]; } qray;

static void quantize(const float *p, const float *d, qray *r)
{
    for (int k = 0; k < 3; k++) {
        double o = rint((double)p[k] * 1073741824.0);
        if (o < 0) o = 0;
        if (o > 1073741823.0) o = 1073741823.0;
        r->O[k] = (int64_t)o;
        r->q[k] = (int64_t)rint((double)d[k] * 8388608.0);
    }
}

typedef struct {
    int hit;
    int axis;          /* axis of the crossing that entered the hit leaf */
    uint32_t key;      /* hit leaf key */
    int64_t delta;     /* |B_axis - O_axis| of that crossing, fine units */
    int64_t visits;    /* occupancy tests at levels >= lds_levels (hier only) */
} march_out;

static int occupied(const orc_svo *s, int l, uint32_t key)
{
    return find_key(s->keys[l], s->n[l], key) >= 0;
}

/* The definition of the march (replaces the paper's hardware ray cast against
 * triangles, Sec. 3.3): visit leaf cells in order of exact entry parameter
 * starting from the origin's leaf (never a hit); the next crossing on axis a
 * lies on B_a = (c_a + [q_a > 0]) << (30 - D); crossings are compared exactly
 * by |B_a - O_a| * |q_b| vs |B_b - O_b| * |q_a|; ties step the lowest axis
 * first; the first occupied leaf other than the origin's is the hit; leaving
 * [0, 2^D)^3 is a miss. */
static march_out march_flat(const orc_svo *s, const qray *r)
{
    int D = s->depth, sh = FINE - D;
    int64_t c[3];
    march_out mo = {0, -1, 0, 0, 0};
    for (int k = 0; k < 3; k++) c[k] = r->O[k] >> sh;
    for (;;) {
        int a = -1;
        int64_t da = 0, qa = 1;
        for (int k = 0; k < 3; k++) {
            if (r->q[k] == 0) continue;
            int64_t B = (c[k] + (r->q[k] > 0)) << sh;
            int64_t dk = llabs(B - r->O[k]), qk = llabs(r->q[k]);
            if (a < 0 || (__int128)dk * qa < (__int128)da * qk) { a = k; da = dk; qa = qk; }
        }
        if (a < 0) return mo;
        c[a] += r->q[a] > 0 ? 1 : -1;
        if (c[a] < 0 || c[a] >= (1 << D)) return mo;
        uint32_t key = orc_morton((uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]);
        if (occupied(s, D, key)) {
            mo.hit = 1; mo.axis = a; mo.key = key; mo.delta = da;
            return mo;
        }
    }
}

/* Leaf cell occupied by the ray just after the crossing event (t = tn/td on
 * axis ta; ta = -1 and tn = 0 at the start), counting every axis-j leaf
 * boundary crossed at an earlier parameter, or at the same parameter with
 * j <= ta. Exact integer arithmetic. */
static void leaf_at(const qray *r, int D, int64_t tn, int64_t td, int ta, int64_t *c)
{
    int sh = FINE - D;
    __int128 S = (__int128)1 << sh;
    for (int j = 0; j < 3; j++) {
        if (r->q[j] == 0) { c[j] = r->O[j] >> sh; continue; }
        __int128 num = (__int128)r->O[j] * td + (r->q[j] > 0 ? 1 : -1) * (__int128)tn * llabs(r->q[j]);
        __int128 den = (__int128)td * S;   /* X_j / S = num / den */
        __int128 k = num / den, rem = num % den;
        if (rem < 0) { k -= 1; rem += den; }
        if (rem != 0) { c[j] = (int64_t)k; continue; }
        /* exactly on the boundary k*S */
        if (r->q[j] > 0) {
            int ahead = (k * S > r->O[j]);       /* the plane is crossed at t > 0 */
            c[j] = (int64_t)((ahead && j > ta) ? k - 1 : k);
        } else {
            c[j] = (int64_t)((j <= ta) ? k - 1 : k);
        }
    }
}

/* The same march as a top-down walk with empty-space skipping (the SVO
 * traversal the GPU performs). At every step only the levels below the
 * deepest ancestor shared with the previous cell are tested, down to the
 * first empty level or the leaf; an empty cell at level l is left through
 * its first exit crossing. Used to prove equivalence with march_flat and to
 * count the node tests at levels >= lds_levels. */
static march_out march_hier(const orc_svo *s, const qray *r, int lds_levels)
{
    int D = s->depth;
    march_out mo = {0, -1, 0, 0, 0};
    int64_t cc[3] = {0, 0, 0};
    int l = 0, ta = -1;
    int64_t tn = 0, td = 1;
    int64_t o[3];
    for (int k = 0; k < 3; k++) o[k] = r->O[k] >> (FINE - D);
    uint32_t origin = orc_morton((uint32_t)o[0], (uint32_t)o[1], (uint32_t)o[2]);
    if (s->n[0] == 0) return mo;
    for (;;) {
        if (l >= lds_levels) mo.visits++;
        uint32_t key = orc_morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]);
        int occ = occupied(s, l, key);
        if (occ && l < D) {
            int64_t lc[3];
            leaf_at(r, D, tn, td, ta, lc);
            l++;
            for (int k = 0; k < 3; k++) cc[k] = lc[k] >> (D - l);
            continue;
        }
        if (occ && l == D && key != origin) {
            mo.hit = 1; mo.axis = ta; mo.key = key; mo.delta = tn;
            return mo;
        }
        /* leave the (empty, or origin) cell */
        int sh = FINE - l, e = -1;
        int64_t de = 0, qe = 1;
        for (int k = 0; k < 3; k++) {
            if (r->q[k] == 0) continue;
            int64_t F = (cc[k] + (r->q[k] > 0)) << sh;
            int64_t dk = llabs(F - r->O[k]), qk = llabs(r->q[k]);
            if (e < 0 || (__int128)dk * qe < (__int128)de * qk) { e = k; de = dk; qe = qk; }
        }
        if (e < 0) return mo;
        int64_t old = cc[e];
        cc[e] += r->q[e] > 0 ? 1 : -1;
        if (cc[e] < 0 || cc[e] >= ((int64_t)1 << l)) return mo;
        tn = de; td = qe; ta = e;
        uint64_t x = (uint64_t)(old ^ cc[e]);
        int p = 63 - __builtin_clzll(x);
        l -= p;
        for (int k = 0; k < 3; k++) cc[k] >>= p;
    }
}

/* ------------------------------------------------- footprint and value --- */
typedef struct {
    int hit, axis, k, side;
    uint32_t leaf, node;
    int64_t node_index, delta, visits;
    float value;      /* stored exitance value used (before epsilon) */
    double truth;     /* FP64 exitance of the same node/side */
} bin_out;

/* Cone footprint (Eq. 7): A = r^2 * omega with omega = 4*pi/N^2, r the
 * distance to the hit leaf's entry point in leaf units, computed in FP32 as
 * ((float)delta * 2^-(30-D)) / |d_axis|. The node whose area (side^2, leaf
 * units) is closest to A: k = #{ j in 1..D : A > 2.5 * 4^(j-1) } levels above
 * the leaf (linear-area midpoints; ties go to the finer level). The exitance
 * side is selected by the sign of N_node . d (Sec. 3.3): side 0 (the N side,
 * facing the origin) iff the dot product is negative. */
static bin_out eval_bin(const orc_svo *s, const float *p, const float *d, int N, int lds_levels, int hier)
{
    bin_out bo;
    memset(&bo, 0, sizeof bo);
    qray r;
    quantize(p, d, &r);
    march_out mo = hier ? march_hier(s, &r, lds_levels) : march_flat(s, &r);
    bo.visits = mo.visits;
    if (!mo.hit) return bo;
    int D = s->depth;
    bo.hit = 1;
    bo.axis = mo.axis;
    bo.leaf = mo.key;
    bo.delta = mo.delta;
    float omega = (float)(4.0 * M_PI / (double)(N * N));
    float dist = ((float)mo.delta * ldexpf(1.0f, -(FINE - D))) / fabsf(d[mo.axis]);
    float A = (dist * dist) * omega;
    int k = 0;
    for (int j = 1; j <= D; j++)
        if (A > 2.5f * ldexpf(1.0f, 2 * (j - 1))) k++;
    bo.k = k;
    bo.node = mo.key >> (3 * k);
    int lv = D - k;
    int64_t ni = find_key(s->keys[lv], s->n[lv], bo.node);
    bo.node_index = ni;
    float cdot = dot3f(s->nrm[lv] + 3 * ni, d);
    bo.side = cdot < 0.0f ? 0 : 1;
    bo.value = s->e32[lv][2 * ni + bo.side];
    bo.truth = s->e64[lv][2 * ni + bo.side];
    return bo;
}

/* Per (vertex, bin) traversal record for bit-exact comparison with the GPU:
 * out[8*(i*NN+b) + ...] = {hit, axis, leaf key, delta, k, node key,
 * node index, side}; visits[i*NN+b] = node tests at levels >= lds_levels of
 * the top-down walk (NULL to skip); hier selects the walk used for the record. */
void orc_debug_march(const orc_svo *s, const float *pos, int64_t n, int32_t N,
                     int32_t lds_levels, int32_t hier, int64_t *out, int64_t *visits)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN);
    orc_dir_table(N, tab);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        for (int b = 0; b < NN; b++) {
            bin_out bo = eval_bin(s, p, tab + 3 * b, N, lds_levels, hier);
            int64_t *o = out + 8 * (i * NN + b);
            o[0] = bo.hit; o[1] = bo.hit ? bo.axis : -1; o[2] = bo.leaf; o[3] = bo.delta;
            o[4] = bo.k; o[5] = bo.node; o[6] = bo.hit ? bo.node_index : -1; o[7] = bo.side;
            if (visits) {
                if (hier) visits[i * NN + b] = bo.visits;
                else {
                    qray r;
                    quantize(p, tab + 3 * b, &r);
                    visits[i * NN + b] = march_hier(s, &r, lds_levels).visits;
                }
            }
        }
    }
    free(tab);
}

/* Radiance field of one vertex (Alg. 3, ConeTrace for all patches): L_b =
 * E[node][side] + eps (eps added to every bin, "initial value" of Sec. 4);
 * a miss gives eps. With 16-bit storage (fmt 1/2) the stored E is already
 * rounded and L_b is rounded once more to the 16-bit format, as the GPU
 * stores its bins. L (FP64 of the FP32/16-bit field) and Lt (FP64 truth:
 * unrounded FP64 exitance + eps) may be NULL. */
static void field_one(const orc_svo *s, const float *p, int N, float eps, const float *tab,
                      double *L, double *Lt)
{
    int NN = N * N;
    for (int b = 0; b < NN; b++) {
        bin_out bo = eval_bin(s, p, tab + 3 * b, N, 0, 0);
        float e = bo.hit ? orc_round_fmt(bo.value, s->fmt) : 0.0f;
        double v;
        if (s->fmt == 0) v = (double)e + (double)eps;
        else v = (double)orc_round_fmt(bo.hit ? e + eps : eps, s->fmt);
        if (L) L[b] = v;
        if (Lt) Lt[b] = (bo.hit ? bo.truth : 0.0) + (double)eps;
    }
}

void orc_field(const orc_svo *s, const float *pos, int64_t n, int32_t N, float eps,
               double *L, double *Lt)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN);
    orc_dir_table(N, tab);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        field_one(s, p, N, eps, tab, L ? L + i * NN : NULL, Lt ? Lt + i * NN : NULL);
    }
    free(tab);
}

/* Piecewise-constant PDF over the equal-area bins (Sec. 3.5): pdf_b =
 * L_b / sum(L) * N^2 / (4*pi), a solid-angle density. */
static void pdf_from_field(const double *L, int N, double *pdf)
{
    int NN = N * N;
    double tot = 0.0;
    for (int b = 0; b < NN; b++) tot += L[b];
    for (int b = 0; b < NN; b++) pdf[b] = L[b] / tot * (double)NN / (4.0 * M_PI);
}

void orc_guide_pdf(const orc_svo *s, const float *pos, int64_t n, int32_t N, float eps,
                   double *pdf, double *pdf_truth)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN);
    orc_dir_table(N, tab);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double *L = malloc(sizeof(double) * 2 * (size_t)NN), *Lt = L + NN;
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        field_one(s, p, N, eps, tab, L, Lt);
        if (pdf) pdf_from_field(L, N, pdf + i * NN);
        if (pdf_truth) pdf_from_field(Lt, N, pdf_truth + i * NN);
        free(L);
    }
    free(tab);
}

/* One sample of the field L (N x N, rows v) for query i with RNG counter
 * ctr; see orc_guide_sample. Writes entry i of the n-long outputs. */
static void sample_field(const double *L, int N, uint64_t seed, uint32_t bounce, int64_t ctr, int64_t n,
                         int64_t i, double *dir, double *pdf, int32_t *bin, double *margin)
{
    int NN = N * N;
    double M[MAXN] = {0}, rows[MAXN] = {0}, R[MAXN] = {0};
    double tot = 0.0;
    for (int v = 0; v < N; v++) {
        double rs = 0.0;
        for (int u = 0; u < N; u++) rs += L[v * N + u];
        rows[v] = rs;
        tot += rs;
        M[v] = tot;
    }
    double u4[4];
    uniforms(seed, bounce, ctr, u4);
    double tv = u4[0] * tot;
    int v = 0;
    while (v < N - 1 && !(tv < M[v])) v++;
    double acc = 0.0;
    for (int u = 0; u < N; u++) { acc += L[v * N + u]; R[u] = acc; }
    double tu = u4[1] * rows[v];
    int u = 0;
    while (u < N - 1 && !(tu < R[u])) u++;
    double d[3];
    orc_oct_decode((u + u4[2]) / N, (v + u4[3]) / N, d);
    for (int k = 0; k < 3; k++) dir[k * n + i] = d[k];
    pdf[i] = L[v * N + u] / tot * (double)NN / (4.0 * M_PI);
    bin[2 * i] = u;
    bin[2 * i + 1] = v;
    if (margin) {
        double lo = v > 0 ? M[v - 1] : 0.0, hi = M[v];
        margin[2 * i + 1] = fmin(tv - lo, hi - tv) / tot;
        double lo2 = u > 0 ? R[u - 1] : 0.0, hi2 = R[u];
        margin[2 * i] = fmin(tu - lo2, hi2 - tu) / rows[v];
    }
}

/* Inverse-CDF sampling of the piecewise-constant 2D field (Sec. 3.5): the
 * row v is the first with u1 * total < M_v (M = inclusive prefix of the row
 * sums, rows are v), the column u the first with u2 * rowsum_v < R_v[u]
 * (inclusive prefix within the row); both clamped to N-1. The direction is
 * the octahedral decode of ((u + u3)/N, (v + u4)/N); its pdf is pdf_b.
 * margin[2i], margin[2i+1]: distance of the row / column target to the
 * nearest CDF boundary, relative to the total / row sum (for the tolerance
 * band of the GPU comparison). counter[i] (NULL: i) is the RNG counter of
 * vertex i, i.e. its index in the caller's full queue. */
void orc_guide_sample(const orc_svo *s, const float *pos, int64_t n, uint64_t seed,
                      uint32_t bounce, int32_t N, float eps, const int64_t *counter, double *dir,
                      double *pdf, int32_t *bin, double *margin)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN);
    orc_dir_table(N, tab);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double *L = malloc(sizeof(double) * (size_t)NN);
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        field_one(s, p, N, eps, tab, L, NULL);
        sample_field(L, N, seed, bounce, counter ? counter[i] : i, n, i, dir, pdf, bin, margin);
        free(L);
    }
    free(tab);
}

/* pdf of arbitrary directions (needed by MIS, Sec. 4): encode the direction,
 * take its bin, re-generate the vertex's field and return pdf_b. bin[2i] =
 * (u, v) and edge[i] = distance of x*N or y*N to the nearest bin edge. */
void orc_pdf_eval(const orc_svo *s, const float *pos, const float *dir, int64_t n, int32_t N,
                  float eps, double *pdf, int32_t *bin, double *edge)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN);
    orc_dir_table(N, tab);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double *L = malloc(sizeof(double) * (size_t)NN), xy[2];
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        orc_oct_encode(dir[i], dir[n + i], dir[2 * n + i], xy);
        int u = (int)floor(xy[0] * N), v = (int)floor(xy[1] * N);
        if (u > N - 1) u = N - 1;
        if (v > N - 1) v = N - 1;
        if (u < 0) u = 0;
        if (v < 0) v = 0;
        field_one(s, p, N, eps, tab, L, NULL);
        double tot = 0.0;
        for (int b = 0; b < NN; b++) tot += L[b];
        pdf[i] = L[v * N + u] / tot * (double)NN / (4.0 * M_PI);
        if (bin) { bin[2 * i] = u; bin[2 * i + 1] = v; }
        if (edge) {
            double fx = xy[0] * N, fy = xy[1] * N;
            double ex = fabs(fx - rint(fx)), ey = fabs(fy - rint(fy));
            edge[i] = fmin(ex, ey);
        }
        free(L);
    }
    free(tab);
}

/* Single-ray helpers for tests: out = {hit, axis, key, delta, visits}. */
void orc_march_one(const orc_svo *s, const float *p, const float *d, int32_t hier,
                   int32_t lds_levels, int64_t *out)
{
    qray r;
    quantize(p, d, &r);
    march_out mo = hier ? march_hier(s, &r, lds_levels) : march_flat(s, &r);
    out[0] = mo.hit; out[1] = mo.axis; out[2] = mo.key; out[3] = mo.delta; out[4] = mo.visits;
}

void orc_quantize(const float *p, const float *d, int64_t *O, int64_t *q)
{
    qray r;
    quantize(p, d, &r);
    for (int k = 0; k < 3; k++) { O[k] = r.O[k]; q[k] = r.q[k]; }
}

void orc_round_fmt_array(const float *in, float *out, int64_t n, int32_t fmt)
{
    for (int64_t i = 0; i < n; i++) out[i] = orc_round_fmt(in[i], fmt);
}

/* One (vertex, direction) evaluation for tests: out = {hit, axis, leaf, delta,
 * k, node, node_index, side}; val = {stored exitance used, FP32 distance r}. */
void orc_eval_one(const orc_svo *s, const float *p, const float *d, int32_t N, int64_t *out,
                  double *val)
{
    bin_out bo = eval_bin(s, p, d, N, 0, 0);
    out[0] = bo.hit; out[1] = bo.hit ? bo.axis : -1; out[2] = bo.leaf; out[3] = bo.delta;
    out[4] = bo.k; out[5] = bo.node; out[6] = bo.hit ? bo.node_index : -1; out[7] = bo.side;
    val[0] = bo.value;
    val[1] = bo.hit ? (double)(((float)bo.delta * ldexpf(1.0f, -(FINE - s->depth))) /
                               fabsf(d[bo.axis])) : 0.0;
}

/* Vectorized map helpers for tests: dirs/points are SoA (3 resp. 2 planes). */
void orc_oct_encode_many(const double *d, int64_t n, double *xy)
{
    for (int64_t i = 0; i < n; i++) {
        double o[2];
        orc_oct_encode(d[i], d[n + i], d[2 * n + i], o);
        xy[i] = o[0];
        xy[n + i] = o[1];
    }
}
void orc_oct_decode_many(const double *xy, int64_t n, double *d)
{
    for (int64_t i = 0; i < n; i++) {
        double o[3];
        orc_oct_decode(xy[i], xy[n + i], o);
        d[i] = o[0]; d[n + i] = o[1]; d[2 * n + i] = o[2];
    }
}

/* Number of OpenMP threads the parallel loops above use. */
/* Threads of the parallel loops from now on (the CPU baseline's single-thread leg). */
void orc_set_num_threads(int32_t n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

int32_t orc_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}

/* ------------------------------------------- positional binning (Alg. 2) - */
/* Partition-S. Each query descends to the deepest existing node that holds
 * its quantized position (its leaf when occupied) and adds one to that node's
 * count. Bottom-up from the leaves to level l_min, a node's total T is its own
 * count plus its children's totals, and the node is marked when T >= c_ray or
 * when it lies on level l_min (reading: the leaf level takes part with T = its
 * own count). A query's bin is the deepest marked node on the path from its
 * node to the root, the node itself included; a query whose node lies above
 * l_min is its own bin. Output: the bin's level and index within the level. */
void orc_partition(const orc_svo *s, const float *pos, int64_t n, int32_t c_ray, int32_t l_min,
                   int32_t *bin_level, int64_t *bin_index)
{
    int D = s->depth;
    int64_t *T[MAXD + 1];
    for (int l = 0; l <= D; l++) T[l] = calloc((size_t)(s->n[l] ? s->n[l] : 1), sizeof(int64_t));
    int32_t *nl = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *ni = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; i++) {   /* DescendLeaf + AtomicAdd */
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]}, d0[3] = {0, 0, 0};
        qray r;
        quantize(p, d0, &r);
        uint32_t key = orc_morton((uint32_t)(r.O[0] >> (FINE - D)), (uint32_t)(r.O[1] >> (FINE - D)),
                                  (uint32_t)(r.O[2] >> (FINE - D)));
        int l = D;
        int64_t idx = find_key(s->keys[l], s->n[l], key);
        while (idx < 0 && l > 0) {
            l--;
            key >>= 3;
            idx = find_key(s->keys[l], s->n[l], key);
        }
        nl[i] = idx < 0 ? -1 : l;
        ni[i] = idx;
        if (idx >= 0) T[l][idx] += 1;
    }
    uint8_t *mark[MAXD + 1];
    for (int l = 0; l <= D; l++) mark[l] = calloc((size_t)(s->n[l] ? s->n[l] : 1), 1);
    for (int l = D; l >= l_min && l >= 0; l--) {   /* bottom-up totals and marks */
        if (l < D) {
            for (int64_t c = 0; c < s->n[l + 1]; c++) {
                int64_t par = find_key(s->keys[l], s->n[l], s->keys[l + 1][c] >> 3);
                T[l][par] += T[l + 1][c];
            }
        }
        for (int64_t k = 0; k < s->n[l]; k++) mark[l][k] = (T[l][k] >= c_ray) || (l == l_min);
    }
    for (int64_t i = 0; i < n; i++) {   /* AscendAndFindMarked */
        int l = nl[i];
        int64_t idx = ni[i];
        if (l < 0) { bin_level[i] = -1; bin_index[i] = -1; continue; }
        int bl = l;
        int64_t bi = idx;
        uint32_t key = s->keys[l][idx];
        for (int m = l; m >= l_min && m >= 0; m--) {
            int64_t k = find_key(s->keys[m], s->n[m], key >> (3 * (l - m)));
            if (mark[m][k]) { bl = m; bi = k; break; }
        }
        bin_level[i] = bl;
        bin_index[i] = bi;
    }
    for (int l = 0; l <= D; l++) { free(T[l]); free(mark[l]); }
    free(nl);
    free(ni);
}

/* Origin choice of a bin (SelectOrigin, Alg. 3; a random member of the bin,
 * Sec. 4): the member minimizing (h_i, i) with h_i the first word of
 * Philox-4x32-10 at counter (i_lo, i_hi, bounce, 1), key (seed_lo, seed_hi).
 * The counter's last word keeps this stream apart from the sampling
 * uniforms (which use 0). */
static uint32_t origin_hash(uint64_t seed, uint32_t bounce, int64_t i)
{
    uint32_t ctr[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), bounce, 1};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox(ctr, key, o);
    return o[0];
}

static void product_table(const float *nrm, const float *bsdf, int64_t n, int64_t i, const float *tab8,
                          double *f);
static void product_one(const double *L, int N, const double *f, uint64_t seed, uint32_t bounce, int64_t ctr,
                        int64_t n, int64_t i, double *dir, double *pdf, int32_t *bin, double *margin);

void orc_jitter_table(int32_t N, uint32_t jitter_key, float *out);
void orc_blur(const double *L, int32_t N, double *out);

/* Binned guiding (Alg. 2 then Alg. 3): partition the queue, take each bin's
 * origin, generate the N x N field once per bin at its origin (as
 * orc_guide_pdf does for a vertex), and sample every member from its bin's
 * field with the member's own uniforms (counter = its index i). Outputs as
 * orc_guide_sample, plus the bin (level, index) and the queue index of the
 * bin's origin per member. Queries without a bin (empty SVO) get pdf 0.
 * With nrm or bsdf given, every member draws a product sample (below) from
 * its bin's field and its own BSDF table, as the paper's product variant does
 * per ray over the shared bin field. jitter/jitter_key/blur: the field
 * antialiasing options of orc_field_aa, applied to every bin field. */
void orc_binned_sample(const orc_svo *s, const float *pos, int64_t n, int32_t c_ray, int32_t l_min,
                       uint64_t seed, uint32_t bounce, int32_t N, float eps, double *dir, double *pdf,
                       int32_t *bin, double *margin, int32_t *bin_level, int64_t *bin_index,
                       int64_t *origin, const float *nrm, const float *bsdf, int32_t jitter,
                       uint32_t jitter_key, int32_t blur)
{
    int D = s->depth, NN = N * N;
    orc_partition(s, pos, n, c_ray, l_min, bin_level, bin_index);
    /* origin per bin: argmin over members of (h, i) */
    int64_t *best[MAXD + 1];
    uint32_t *besth[MAXD + 1];
    for (int l = 0; l <= D; l++) {
        size_t m = (size_t)(s->n[l] ? s->n[l] : 1);
        best[l] = malloc(sizeof(int64_t) * m);
        besth[l] = malloc(sizeof(uint32_t) * m);
        for (size_t k = 0; k < m; k++) best[l][k] = -1;
    }
    for (int64_t i = 0; i < n; i++) {
        int l = bin_level[i];
        if (l < 0) continue;
        int64_t k = bin_index[i];
        uint32_t h = origin_hash(seed, bounce, i);
        if (best[l][k] < 0 || h < besth[l][k] || (h == besth[l][k] && i < best[l][k])) {
            best[l][k] = i;
            besth[l][k] = h;
        }
    }
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN);
    if (jitter) orc_jitter_table(N, jitter_key, tab);
    else orc_dir_table(N, tab);
    /* the field of each bin, once, at its origin */
    int64_t nb = 0;
    int64_t *slot[MAXD + 1];
    for (int l = 0; l <= D; l++) {
        size_t m = (size_t)(s->n[l] ? s->n[l] : 1);
        slot[l] = malloc(sizeof(int64_t) * m);
        for (size_t k = 0; k < m; k++) slot[l][k] = best[l][k] >= 0 ? nb++ : -1;
    }
    double *fields = malloc(sizeof(double) * (size_t)(nb ? nb : 1) * (size_t)NN);
    int64_t *forig = malloc(sizeof(int64_t) * (size_t)(nb ? nb : 1));
    for (int l = 0; l <= D; l++)
        for (int64_t k = 0; k < s->n[l]; k++)
            if (slot[l][k] >= 0) forig[slot[l][k]] = best[l][k];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nb; b++) {
        int64_t o = forig[b];
        float p[3] = {pos[o], pos[n + o], pos[2 * n + o]};
        field_one(s, p, N, eps, tab, fields + b * NN, NULL);
        if (blur) {
            double *t = malloc(sizeof(double) * (size_t)NN);
            orc_blur(fields + b * NN, N, t);
            memcpy(fields + b * NN, t, sizeof(double) * (size_t)NN);
            free(t);
        }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        int l = bin_level[i];
        if (l < 0) {
            origin[i] = -1;
            pdf[i] = 0.0;
            for (int k = 0; k < 3; k++) dir[k * n + i] = 0.0;
            bin[2 * i] = bin[2 * i + 1] = -1;
            if (margin) margin[2 * i] = margin[2 * i + 1] = 0.0;
            continue;
        }
        origin[i] = best[l][bin_index[i]];
        if (nrm || bsdf) {   /* product guiding: the member's own table times its bin's field */
            double f[64];
            float tab8[3 * 64];
            orc_dir_table(8, tab8);
            product_table(nrm, bsdf, n, i, tab8, f);
            product_one(fields + slot[l][bin_index[i]] * NN, N, f, seed, bounce, i, n, i, dir, pdf, bin, margin);
        } else {
            sample_field(fields + slot[l][bin_index[i]] * NN, N, seed, bounce, i, n, i, dir, pdf, bin, margin);
        }
    }
    free(tab);
    free(fields);
    free(forig);
    for (int l = 0; l <= D; l++) { free(best[l]); free(besth[l]); free(slot[l]); }
}

/* ------------------------------------------------ product guiding ------- */
/* Product path guiding (Sec. 3.6, after the two-level product sampler of
 * Estevez and Kulla that the paper adopts). The upper level is the N x N field
 * subsampled to the 8 x 8 resolution of the BSDF table: cell C = (U, V) holds
 * the s x s fine bins u in [U s, U s + s), v in [V s, V s + s), s = N / 8, and
 * its value F_C is their sum (rows dv outer, columns du inner). The BSDF
 * table f_C lives on the same octahedral 8 x 8 cells; it is either given per
 * query or, for a Lambertian surface with normal n, the cosine factor
 * max(0, n . d_C) at the cell centre d_C (the N = 8 bin-centre table). That
 * dot product decides which cells can be sampled, so it is taken in FP32 as
 * (n_x d_x + n_y d_y) + n_z d_z without contraction; a table entry that is
 * not > 0 (negative, zero, NaN) counts as 0.
 *
 * Sampling: the cell from the product P_C = F_C f_C (marginal over rows V,
 * then the row's CDF over U; uniforms w1, w2 = the first two words of
 * Philox-4x32-10 at counter (i_lo, i_hi, bounce, 2)), then the fine bin inside
 * the cell from the field restricted to it (row dv, column du; uniforms u1, u2
 * of the plain sampler, counter word 0), then the in-bin offset (u3, u4).
 * pdf = P_C / sum(P) * L_b / F_C * N^2 / (4 pi), i.e. the normalized product of
 * the field with the table held constant over each cell. A row or column is
 * the first whose inclusive CDF exceeds the target; if none does (a target
 * rounded up to the total), the last one with positive mass. A product that
 * sums to zero or to a non-finite value (zero or non-finite normal) is
 * replaced by f = 1, which is plain guiding. */
#define PCELLS 8

static void product_uniforms(uint64_t seed, uint32_t bounce, int64_t i, double w[2])
{
    uint32_t ctr[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), bounce, 2};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox(ctr, key, o);
    for (int k = 0; k < 2; k++) w[k] = (double)(o[k] >> 8) * (1.0 / 16777216.0);
}

/* f[64] of query i: table row i of bsdf (n x 64) or the cosine factor of the
 * normal (SoA 3 x n); tab8 = the FP32 bin-centre table of N = 8. */
static void product_table(const float *nrm, const float *bsdf, int64_t n, int64_t i, const float *tab8,
                          double *f)
{
    for (int c = 0; c < PCELLS * PCELLS; c++) {
        float x;
        if (bsdf) {
            x = bsdf[i * 64 + c];
        } else {
            float nv[3] = {nrm[i], nrm[n + i], nrm[2 * n + i]};
            x = dot3f(nv, tab8 + 3 * c);
        }
        f[c] = x > 0.0f ? (double)x : 0.0;
    }
}

typedef struct {
    double F[64], P[64], rows[8], M[8], total;
} product_upper;

static void product_upper_level(const double *L, int N, const double *f, product_upper *q)
{
    int s = N / PCELLS;
    for (int V = 0; V < PCELLS; V++)
        for (int U = 0; U < PCELLS; U++) {
            double F = 0.0;
            for (int dv = 0; dv < s; dv++)
                for (int du = 0; du < s; du++) F += L[(V * s + dv) * N + U * s + du];
            q->F[V * PCELLS + U] = F;
        }
    for (int pass = 0; pass < 2; pass++) {
        double tot = 0.0;
        for (int V = 0; V < PCELLS; V++) {
            double rs = 0.0;
            for (int U = 0; U < PCELLS; U++) {
                int c = V * PCELLS + U;
                q->P[c] = q->F[c] * (pass ? 1.0 : f[c]);
                rs += q->P[c];
            }
            q->rows[V] = rs;
            tot += rs;
            q->M[V] = tot;
        }
        q->total = tot;
        if (tot > 0.0 && isfinite(tot)) break;   /* else: f = 1 (plain guiding) */
    }
}

/* first k with t < cdf[k]; else the last k with mass[k] > 0; else m - 1 */
static int pick(const double *cdf, const double *mass, int m, double t)
{
    for (int k = 0; k < m; k++)
        if (t < cdf[k]) return k;
    for (int k = m - 1; k >= 0; k--)
        if (mass[k] > 0.0) return k;
    return m - 1;
}

static double rel_margin(const double *cdf, int k, double t, double scale)
{
    double lo = k > 0 ? cdf[k - 1] : 0.0, hi = cdf[k];
    return fmin(fabs(t - lo), fabs(hi - t)) / scale;
}

static void product_one(const double *L, int N, const double *f, uint64_t seed, uint32_t bounce, int64_t ctr,
                        int64_t n, int64_t i, double *dir, double *pdf, int32_t *bin, double *margin)
{
    int s = N / PCELLS, NN = N * N;
    product_upper q;
    product_upper_level(L, N, f, &q);
    double w[2], u[4];
    product_uniforms(seed, bounce, ctr, w);
    uniforms(seed, bounce, ctr, u);
    /* upper level: the cell */
    double tv = w[0] * q.total;
    int V = pick(q.M, q.rows, PCELLS, tv);
    double R[PCELLS], acc = 0.0;
    for (int U = 0; U < PCELLS; U++) { acc += q.P[V * PCELLS + U]; R[U] = acc; }
    double tu = w[1] * q.rows[V];
    int U = pick(R, q.P + V * PCELLS, PCELLS, tu);
    int c = V * PCELLS + U;
    /* lower level: the fine bin inside the cell */
    double br[MAXN / PCELLS] = {0}, BM[MAXN / PCELLS] = {0}, bt = 0.0;
    for (int dv = 0; dv < s; dv++) {
        double rs = 0.0;
        for (int du = 0; du < s; du++) rs += L[(V * s + dv) * N + U * s + du];
        br[dv] = rs;
        bt += rs;
        BM[dv] = bt;
    }
    double t2 = u[0] * bt;
    int dv = pick(BM, br, s, t2);
    double BR[MAXN / PCELLS], bv[MAXN / PCELLS];
    acc = 0.0;
    for (int du = 0; du < s; du++) {
        bv[du] = L[(V * s + dv) * N + U * s + du];
        acc += bv[du];
        BR[du] = acc;
    }
    double t3 = u[1] * br[dv];
    int du = pick(BR, bv, s, t3);
    int fu = U * s + du, fv = V * s + dv;
    double d[3];
    orc_oct_decode((fu + u[2]) / N, (fv + u[3]) / N, d);
    for (int k = 0; k < 3; k++) dir[k * n + i] = d[k];
    pdf[i] = q.P[c] / q.total * (L[fv * N + fu] / q.F[c]) * (double)NN / (4.0 * M_PI);
    bin[2 * i] = fu;
    bin[2 * i + 1] = fv;
    if (margin) {
        margin[2 * i] = fmin(rel_margin(q.M, V, tv, q.total), rel_margin(R, U, tu, q.rows[V]));
        margin[2 * i + 1] = fmin(rel_margin(BM, dv, t2, bt), rel_margin(BR, du, t3, br[dv]));
    }
}

static double product_pdf_one(const double *L, int N, const double *f, int fu, int fv)
{
    int s = N / PCELLS;
    product_upper q;
    product_upper_level(L, N, f, &q);
    int c = (fv / s) * PCELLS + fu / s;
    return q.P[c] / q.total * (L[fv * N + fu] / q.F[c]) * (double)(N * N) / (4.0 * M_PI);
}

static void dir_bin(double dx, double dy, double dz, int N, int *u, int *v, double *edge)
{
    double xy[2];
    orc_oct_encode(dx, dy, dz, xy);
    int a = (int)floor(xy[0] * N), b = (int)floor(xy[1] * N);
    *u = a < 0 ? 0 : (a > N - 1 ? N - 1 : a);
    *v = b < 0 ? 0 : (b > N - 1 ? N - 1 : b);
    if (edge) {
        double fx = xy[0] * N, fy = xy[1] * N;
        *edge = fmin(fabs(fx - rint(fx)), fabs(fy - rint(fy)));
    }
}

/* Product sampling from given fields: query i uses L + i * lstride (N*N,
 * rows v; lstride 0 shares one field); nrm (SoA 3 x n) or bsdf (n x 64)
 * gives each query's table. Outputs as orc_guide_sample. */
void orc_product_fields(const double *L, int64_t lstride, int64_t n, int32_t N, const float *nrm,
                        const float *bsdf,
                        uint64_t seed, uint32_t bounce, const int64_t *counter, double *dir, double *pdf,
                        int32_t *bin, double *margin)
{
    float tab8[3 * 64];
    orc_dir_table(PCELLS, tab8);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double f[64];
        product_table(nrm, bsdf, n, i, tab8, f);
        product_one(L + i * lstride, N, f, seed, bounce, counter ? counter[i] : i, n, i, dir, pdf, bin, margin);
    }
}

/* Product pdf of directions dir (SoA 3 x n) under fields L (n x N*N). */
void orc_product_pdf_fields(const double *L, int64_t n, int32_t N, const float *nrm, const float *bsdf,
                            const double *dir, double *pdf)
{
    float tab8[3 * 64];
    orc_dir_table(PCELLS, tab8);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double f[64];
        int u, v;
        product_table(nrm, bsdf, n, i, tab8, f);
        dir_bin(dir[i], dir[n + i], dir[2 * n + i], N, &u, &v, NULL);
        pdf[i] = product_pdf_one(L + i * (int64_t)N * N, N, f, u, v);
    }
}

/* Product guiding of a queue: each vertex's own field (as orc_guide_sample),
 * then the two-level product sample above. */
void orc_product_sample(const orc_svo *s, const float *pos, const float *nrm, const float *bsdf, int64_t n,
                        uint64_t seed, uint32_t bounce, int32_t N, float eps, double *dir, double *pdf,
                        int32_t *bin, double *margin)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN), tab8[3 * 64];
    orc_dir_table(N, tab);
    orc_dir_table(PCELLS, tab8);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double *L = malloc(sizeof(double) * (size_t)NN), f[64];
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        field_one(s, p, N, eps, tab, L, NULL);
        product_table(nrm, bsdf, n, i, tab8, f);
        product_one(L, N, f, seed, bounce, i, n, i, dir, pdf, bin, margin);
        free(L);
    }
    free(tab);
}

/* Product pdf of arbitrary directions at the queue's vertices (MIS). */
void orc_product_pdf_eval(const orc_svo *s, const float *pos, const float *nrm, const float *bsdf,
                          const float *dir, int64_t n, int32_t N, float eps, double *pdf, int32_t *bin,
                          double *edge)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN), tab8[3 * 64];
    orc_dir_table(N, tab);
    orc_dir_table(PCELLS, tab8);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double *L = malloc(sizeof(double) * (size_t)NN), f[64];
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        int u, v;
        dir_bin(dir[i], dir[n + i], dir[2 * n + i], N, &u, &v, edge ? edge + i : NULL);
        field_one(s, p, N, eps, tab, L, NULL);
        product_table(nrm, bsdf, n, i, tab8, f);
        pdf[i] = product_pdf_one(L, N, f, u, v);
        if (bin) { bin[2 * i] = u; bin[2 * i + 1] = v; }
        free(L);
    }
    free(tab);
}

/* ------------------------------------------- field antialiasing (Sec. 4) - */
/* Directional jitter: instead of the bin centre, the cone of bin b = v N + u
 * runs along the decode of ((u + j_u) / N, (v + j_v) / N), with (j_u, j_v) the
 * first two words of Philox-4x32-10 at counter (b, 0, 0, 3) and key
 * (jitter_key, 0), each as (bits >> 8) * 2^-24. The caller draws a new key
 * on the iterations it jitters. Decoded in FP64, rounded to FP32 (as the
 * bin-centre table). */
void orc_jitter_table(int32_t N, uint32_t jitter_key, float *out)
{
    for (int v = 0; v < N; v++)
        for (int u = 0; u < N; u++) {
            int b = v * N + u;
            uint32_t ctr[4] = {(uint32_t)b, 0, 0, 3}, key[2] = {jitter_key, 0}, o[4];
            orc_philox(ctr, key, o);
            double ju = (double)(o[0] >> 8) * (1.0 / 16777216.0), jv = (double)(o[1] >> 8) * (1.0 / 16777216.0);
            double d[3];
            orc_oct_decode((u + ju) / N, (v + jv) / N, d);
            for (int k = 0; k < 3; k++) out[3 * b + k] = (float)d[k];
        }
}

/* Neighbour bins across the edge of the octahedral square: the map sends the
 * points (1, b) and (1, -b) of the edge a = 1 to the same direction (and
 * likewise on the other three edges), so bin (N, v) is bin (N - 1, N - 1 - v)
 * and bin (u, N) is bin (N - 1 - u, N - 1); a corner folds twice. */
static void fold_bin(int N, int *u, int *v)
{
    if (*u < 0) { *u = 0; *v = N - 1 - *v; }
    else if (*u >= N) { *u = N - 1; *v = N - 1 - *v; }
    if (*v < 0) { *v = 0; *u = N - 1 - *u; }
    else if (*v >= N) { *v = N - 1; *u = N - 1 - *u; }
}

/* Gaussian blur of a field (Sec. 4, "to make the generated radiance field
 * plausible for all the rays in the bin"): the 3 x 3 binomial kernel
 * (1/4, 1/2, 1/4) in each direction over the bins, neighbours folded across
 * the square's edges. FP64. */
void orc_blur(const double *L, int32_t N, double *out)
{
    static const double w[3] = {0.25, 0.5, 0.25};
    for (int v = 0; v < N; v++)
        for (int u = 0; u < N; u++) {
            double acc = 0.0;
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int uu = u + dx, vv = v + dy;
                    fold_bin(N, &uu, &vv);
                    acc += w[dy + 1] * w[dx + 1] * L[vv * N + uu];
                }
            out[v * N + u] = acc;
        }
}

/* Fields with the antialiasing options: the cone directions of the jittered
 * table when jitter != 0, then the blur when blur != 0. L: n x N*N. */
void orc_field_aa(const orc_svo *s, const float *pos, int64_t n, int32_t N, float eps, int32_t jitter,
                  uint32_t jitter_key, int32_t blur, double *L)
{
    int NN = N * N;
    float *tab = malloc(sizeof(float) * 3 * (size_t)NN);
    if (jitter) orc_jitter_table(N, jitter_key, tab);
    else orc_dir_table(N, tab);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        double *Li = L + i * NN;
        field_one(s, p, N, eps, tab, Li, NULL);
        if (blur) {
            double *t = malloc(sizeof(double) * (size_t)NN);
            orc_blur(Li, N, t);
            memcpy(Li, t, sizeof(double) * (size_t)NN);
            free(t);
        }
    }
    free(tab);
}

/* Plain guide_sample rule on given fields (query i uses L + i * lstride). */
void orc_sample_fields(const double *L, int64_t lstride, int64_t n, int32_t N, uint64_t seed, uint32_t bounce,
                       const int64_t *counter, double *dir, double *pdf, int32_t *bin, double *margin)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++)
        sample_field(L + i * lstride, N, seed, bounce, counter ? counter[i] : i, n, i, dir, pdf, bin, margin);
}

/* ------------------------------------ exitance extraction (Eq. 5) ------ */
/* Local radiance along a path (Sec. 3.2, Eq. 5): a path stores, for every
 * depth k = 1..d, its vertex p_k and the throughput T_k of its first k
 * vertices (RGB); p_0 is its eye point. When the path reaches an emitter at
 * depth n with emitted radiance L_e toward p_{n-1}, the radiance leaving p_k
 * toward p_{k-1} is (T_n / T_k) L_e for every k = 1..n (k = n: L_e itself).
 * Each becomes one splat: position p_k, outgoing direction p_{k-1} - p_k
 * (only its sign against the leaf normal is used), rgb (T_n / T_k) L_e per
 * channel in FP32 (a zero T_k channel gives 0: T_n is then 0 as well).
 * Layout: pos, T = d planes of 3 x P SoA, plane k-1 at offset (k-1) * 3 * P;
 * eye, Le = 3 x P; hit[i] = n (1..d), anything else = no emitter. The splats
 * come out depth-major (k outer, path inner), at most d * P of them; returns
 * their number. */
int64_t orc_path_splats(const float *pos, const float *T, const float *eye, const int32_t *hit, const float *Le,
                        int64_t P, int32_t d, float *spos, float *swo, float *srgb, int64_t cap)
{
    int64_t m = 0;
    for (int k = 1; k <= d; k++)
        for (int64_t i = 0; i < P; i++) {
            int n = hit[i];
            if (n < 1 || n > d || k > n) continue;
            const float *pk = pos + (int64_t)(k - 1) * 3 * P, *pp = k > 1 ? pos + (int64_t)(k - 2) * 3 * P : eye;
            const float *Tk = T + (int64_t)(k - 1) * 3 * P, *Tn = T + (int64_t)(n - 1) * 3 * P;
            if (m >= cap) return -1;
            for (int c = 0; c < 3; c++) {
                float tk = Tk[c * P + i], tn = Tn[c * P + i];
                float ratio = tk == 0.0f ? 0.0f : tn / tk;
                spos[c * cap + m] = pk[c * P + i];
                swo[c * cap + m] = pp[c * P + i] - pk[c * P + i];
                srgb[c * cap + m] = ratio * Le[c * P + i];
            }
            m++;
        }
    return m;
}
