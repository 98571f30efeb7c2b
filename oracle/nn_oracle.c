/*
 * CPU oracle of the learned stand-in for the march (test infrastructure
 * only; see oracle.c's header). Not part of the paper, which only surveys
 * neural guiding as related work (Sec. 2.1); the network follows the
 * multiresolution hash encoding of Mueller et al. 2022 (written from that
 * paper) feeding a small ReLU MLP whose softmax is a distribution over the
 * N x N direction bins, trained by cross-entropy against the march's PDFs.
 *
 * Two modes:
 *  mode 0: FP64 throughout (the mathematical network; pinned by finite
 *          differences).
 *  mode 1: BF16-faithful: every value the GPU kernels round to BF16 (hash
 *          table entries, encoded inputs, weights, hidden activations, the
 *          logit and hidden-layer gradients fed to matrix products) is rounded
 *          here at the same point (RNE); the hash interpolation follows the
 *          kernels' FP32 operation order; sums are FP64.
 *
 * Parameter vector (FP32, this order): W0[64][35], b0[64], W1[64][64], b1,
 * W2, b2, W3, b3, W4[256][64], b4[256], table[L][T][F].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NN_IN 35
#define NN_H 64
#define NN_OUT 256
#define NN_L 16
#define NN_F 2

typedef struct {
    int32_t log2_table;   /* T = 2^log2_table entries per level */
    int32_t n_min, n_max; /* coarsest and finest grid resolution */
} orc_nn_cfg;

static float bf16r(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return f;
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return f;
}

int64_t orc_nn_mlp_params(void)
{
    return (int64_t)NN_H * NN_IN + NN_H + 3 * ((int64_t)NN_H * NN_H + NN_H) +
           (int64_t)NN_OUT * NN_H + NN_OUT;
}
int64_t orc_nn_num_params(const orc_nn_cfg *c)
{
    return orc_nn_mlp_params() + (int64_t)NN_L * ((int64_t)1 << c->log2_table) * NN_F;
}

/* Grid resolution of every level: floor(n_min * b^l) with
 * b = exp((ln n_max - ln n_min) / (L - 1)), in FP64. */
void orc_nn_resolutions(const orc_nn_cfg *c, int32_t *res)
{
    double b = exp((log((double)c->n_max) - log((double)c->n_min)) / (NN_L - 1));
    for (int l = 0; l < NN_L; l++) res[l] = (int32_t)floor((double)c->n_min * pow(b, (double)l));
}

/* Table slot of grid corner (x, y, z) at resolution R: dense while
 * (R + 1)^3 <= T, else the spatial hash x*1 ^ y*2654435761 ^ z*805459861
 * (32-bit products) modulo T. */
static uint32_t corner_index(uint32_t x, uint32_t y, uint32_t z, int32_t R, int log2T)
{
    uint64_t T = (uint64_t)1 << log2T;
    uint64_t side = (uint64_t)R + 1;
    if (side * side * side <= T) return (uint32_t)(x + side * (y + side * z));
    return (x * 1u ^ y * 2654435761u ^ z * 805459861u) & (uint32_t)(T - 1);
}

typedef struct {
    uint32_t idx[NN_L][8];
    double w[NN_L][8];
} enc_info;

/* Hash-grid encoding of one position: per level, the 8 cell corners (bit 0
 * of the corner number = +x, bit 1 = +y, bit 2 = +z) and trilinear weights;
 * the scaled position p*R and the fractions are FP32 (the cell choice is an
 * integer decision taken in the kernels' precision). */
static void encode(const float *p, const int32_t *res, const orc_nn_cfg *c, const float *table,
                   int mode, double *feat, enc_info *ei)
{
    uint64_t T = (uint64_t)1 << c->log2_table;
    for (int l = 0; l < NN_L; l++) {
        int32_t R = res[l];
        uint32_t cell[3];
        float fr[3];
        for (int k = 0; k < 3; k++) {
            float x = p[k] * (float)R;
            float fl = floorf(x);
            if (fl > (float)(R - 1)) fl = (float)(R - 1);
            if (fl < 0.0f) fl = 0.0f;
            cell[k] = (uint32_t)fl;
            fr[k] = x - fl;
        }
        float acc32[NN_F] = {0.0f, 0.0f};
        double acc64[NN_F] = {0.0, 0.0};
        for (int q = 0; q < 8; q++) {
            uint32_t cx = cell[0] + (q & 1), cy = cell[1] + ((q >> 1) & 1), cz = cell[2] + ((q >> 2) & 1);
            float wx = (q & 1) ? fr[0] : 1.0f - fr[0];
            float wy = (q & 2) ? fr[1] : 1.0f - fr[1];
            float wz = (q & 4) ? fr[2] : 1.0f - fr[2];
            float w32 = (wx * wy) * wz;
            double w64 = (double)wx * (double)wy * (double)wz;
            uint32_t id = corner_index(cx, cy, cz, R, c->log2_table);
            if (ei) { ei->idx[l][q] = id; ei->w[l][q] = mode ? (double)w32 : w64; }
            for (int f = 0; f < NN_F; f++) {
                float t = table[((uint64_t)l * T + id) * NN_F + f];
                if (mode) acc32[f] = acc32[f] + w32 * bf16r(t);
                else acc64[f] += w64 * (double)t;
            }
        }
        for (int f = 0; f < NN_F; f++)
            feat[2 * l + f] = mode ? (double)bf16r(acc32[f]) : acc64[f];
    }
}

typedef struct {
    double x[NN_IN];
    double a[4][NN_H];   /* pre-activations of the hidden layers */
    double h[4][NN_H];   /* post-ReLU hidden activations (rounded in mode 1) */
    double z[NN_OUT];
    double p[NN_OUT];
    enc_info ei;
} fwd_state;

static double wv(const float *w, int64_t i, int mode)
{
    return mode ? (double)bf16r(w[i]) : (double)w[i];
}

static void forward_one(const float *par, const int32_t *res, const orc_nn_cfg *c, const float *p,
                        const float *n, int mode, fwd_state *s)
{
    const float *W[5], *B[5];
    int64_t off = 0;
    int fin[5] = {NN_IN, NN_H, NN_H, NN_H, NN_H}, fout[5] = {NN_H, NN_H, NN_H, NN_H, NN_OUT};
    for (int k = 0; k < 5; k++) {
        W[k] = par + off; off += (int64_t)fout[k] * fin[k];
        B[k] = par + off; off += fout[k];
    }
    const float *table = par + off;
    encode(p, res, c, table, mode, s->x, &s->ei);
    for (int k = 0; k < 3; k++) s->x[2 * NN_L + k] = mode ? (double)bf16r(n[k]) : (double)n[k];
    const double *in = s->x;
    for (int k = 0; k < 4; k++) {
        for (int j = 0; j < NN_H; j++) {
            double acc = 0.0;
            for (int i = 0; i < fin[k]; i++) acc += wv(W[k], (int64_t)j * fin[k] + i, mode) * in[i];
            acc += (double)B[k][j];
            s->a[k][j] = acc;
            double h = acc > 0.0 ? acc : 0.0;
            s->h[k][j] = mode ? (double)bf16r((float)h) : h;
        }
        in = s->h[k];
    }
    double zmax = -1e300;
    for (int j = 0; j < NN_OUT; j++) {
        double acc = 0.0;
        for (int i = 0; i < NN_H; i++) acc += wv(W[4], (int64_t)j * NN_H + i, mode) * in[i];
        acc += (double)B[4][j];
        s->z[j] = acc;
        if (acc > zmax) zmax = acc;
    }
    double sum = 0.0;
    for (int j = 0; j < NN_OUT; j++) { s->p[j] = exp(s->z[j] - zmax); sum += s->p[j]; }
    for (int j = 0; j < NN_OUT; j++) s->p[j] /= sum;
}

/* Softmax probabilities (n x 256) and logits (may be NULL) of n vertices
 * (pos and nrm SoA, 3 planes of n). */
void orc_nn_forward(const float *par, const orc_nn_cfg *c, const float *pos, const float *nrm,
                    int64_t n, int32_t mode, double *prob, double *logit)
{
    int32_t res[NN_L];
    orc_nn_resolutions(c, res);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        fwd_state *s = malloc(sizeof(fwd_state));
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        float q[3] = {nrm[i], nrm[n + i], nrm[2 * n + i]};
        forward_one(par, res, c, p, q, mode, s);
        for (int j = 0; j < NN_OUT; j++) {
            if (prob) prob[i * NN_OUT + j] = s->p[j];
            if (logit) logit[i * NN_OUT + j] = s->z[j];
        }
        free(s);
    }
}

/* Gradient of the mean cross-entropy -1/n sum_i sum_b t_ib log p_ib over
 * all parameters (target rows t sum to one). dlogit = (p - t)/n; in mode 1
 * the logit gradient and the hidden pre-activation gradients are rounded to
 * BF16 before they enter the next product, as the kernels do. Returns the
 * loss. */
double orc_nn_grad(const float *par, const orc_nn_cfg *c, const float *pos, const float *nrm,
                   const double *target, int64_t n, int32_t mode, double *grad)
{
    int32_t res[NN_L];
    orc_nn_resolutions(c, res);
    int64_t np = orc_nn_num_params(c);
    memset(grad, 0, sizeof(double) * (size_t)np);
    const float *W[5];
    int64_t woff[5], boff[5], off = 0;
    int fin[5] = {NN_IN, NN_H, NN_H, NN_H, NN_H}, fout[5] = {NN_H, NN_H, NN_H, NN_H, NN_OUT};
    for (int k = 0; k < 5; k++) {
        woff[k] = off; W[k] = par + off; off += (int64_t)fout[k] * fin[k];
        boff[k] = off; off += fout[k];
    }
    int64_t toff = off;
    uint64_t T = (uint64_t)1 << c->log2_table;
    double loss = 0.0;
    fwd_state *s = malloc(sizeof(fwd_state));
    for (int64_t i = 0; i < n; i++) {
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        float q[3] = {nrm[i], nrm[n + i], nrm[2 * n + i]};
        forward_one(par, res, c, p, q, mode, s);
        double dz[NN_OUT], dzr[NN_OUT];
        for (int j = 0; j < NN_OUT; j++) {
            double t = target[i * NN_OUT + j];
            if (t > 0.0) loss -= t * log(s->p[j]) / (double)n;
            dz[j] = (s->p[j] - t) / (double)n;
            dzr[j] = mode ? (double)bf16r((float)dz[j]) : dz[j];
        }
        /* output layer */
        double dh[NN_H], dhr[NN_H];
        for (int j = 0; j < NN_OUT; j++) {
            grad[boff[4] + j] += dz[j];
            for (int k2 = 0; k2 < NN_H; k2++) grad[woff[4] + (int64_t)j * NN_H + k2] += dzr[j] * s->h[3][k2];
        }
        for (int k2 = 0; k2 < NN_H; k2++) {
            double acc = 0.0;
            for (int j = 0; j < NN_OUT; j++) acc += wv(W[4], (int64_t)j * NN_H + k2, mode) * dzr[j];
            dh[k2] = acc;
        }
        /* hidden layers 3..0 */
        for (int k = 3; k >= 0; k--) {
            double da[NN_H], dar[NN_H];
            for (int j = 0; j < NN_H; j++) {
                da[j] = s->a[k][j] > 0.0 ? dh[j] : 0.0;
                dar[j] = mode ? (double)bf16r((float)da[j]) : da[j];
                grad[boff[k] + j] += da[j];
            }
            const double *in = k == 0 ? s->x : s->h[k - 1];
            for (int j = 0; j < NN_H; j++)
                for (int i2 = 0; i2 < fin[k]; i2++) grad[woff[k] + (int64_t)j * fin[k] + i2] += dar[j] * in[i2];
            for (int i2 = 0; i2 < fin[k]; i2++) {
                double acc = 0.0;
                for (int j = 0; j < NN_H; j++) acc += wv(W[k], (int64_t)j * fin[k] + i2, mode) * dar[j];
                dhr[i2] = acc;
            }
            for (int i2 = 0; i2 < fin[k]; i2++) dh[i2] = dhr[i2];
        }
        /* hash table: d feature(l, f) / d entry = trilinear weight of the corner */
        for (int l = 0; l < NN_L; l++)
            for (int qq = 0; qq < 8; qq++)
                for (int f = 0; f < NN_F; f++)
                    grad[toff + ((int64_t)l * (int64_t)T + s->ei.idx[l][qq]) * NN_F + f] +=
                        s->ei.w[l][qq] * dh[2 * l + f];
    }
    free(s);
    return loss;
}

/* KL(p || q) = sum_b p_b (ln p_b - ln q_b) in nats, rows of n x 256. */
void orc_kl_rows(const double *p, const double *q, int64_t n, double *kl)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int j = 0; j < NN_OUT; j++) {
            double a = p[i * NN_OUT + j], b = q[i * NN_OUT + j];
            if (a > 0.0) s += a * (log(a) - log(b));
        }
        kl[i] = s;
    }
}

/* Table slots and FP32 trilinear weights of one position (tests). */
void orc_nn_encode_info(const orc_nn_cfg *c, const float *p, uint32_t *idx, double *w)
{
    int32_t res[NN_L];
    orc_nn_resolutions(c, res);
    enc_info ei;
    double feat[2 * NN_L];
    /* a zero table: only the indices and weights are of interest */
    uint64_t T = (uint64_t)1 << c->log2_table;
    float *table = calloc((size_t)(NN_L * T * NN_F), sizeof(float));
    encode(p, res, c, table, 1, feat, &ei);
    free(table);
    memcpy(idx, ei.idx, sizeof ei.idx);
    memcpy(w, ei.w, sizeof ei.w);
}

/* Network inputs (n x 35: the 32 encoded features, then the normal) in the
 * given mode (tests). */
void orc_nn_inputs(const float *par, const orc_nn_cfg *c, const float *pos, const float *nrm, int64_t n,
                   int32_t mode, double *x)
{
    int32_t res[NN_L];
    orc_nn_resolutions(c, res);
    fwd_state *s = malloc(sizeof(fwd_state));
    for (int64_t i = 0; i < n; i++) {
        float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        float q[3] = {nrm[i], nrm[n + i], nrm[2 * n + i]};
        forward_one(par, res, c, p, q, mode, s);
        for (int k = 0; k < NN_IN; k++) x[i * NN_IN + k] = s->x[k];
    }
    free(s);
}

/*
 * Parity bounds of the GPU's arithmetic against the BF16-faithful mode
 * (mode 1), for element-wise comparison. Both sides round the same
 * quantities to BF16 at the same points, but the GPU sums its products in
 * FP32 (matrix cores, in an order of their own) where this oracle sums in
 * FP64. Every FP32 sum of K terms is taken to lie within 2 K u sum |terms| of
 * its exact value (u = 2^-24; first order, any order of the additions; the
 * factor 2 also covers an accumulation that rounds toward zero). Where such
 * an interval contains a BF16 rounding boundary (or, before a ReLU, zero),
 * the GPU may round to another BF16 value than the oracle ("flip"). The
 * bounds follow every value of the network as an interval centred on the
 * oracle's own mode-1 value: the radius of a sum is the sum of its terms'
 * radii (|w| r for a weight times an interval, |a| r_b + r_a |b| + r_a r_b for
 * a product of intervals) plus the accumulation bound; a BF16 rounding maps
 * [v - r, v + r] to the BF16 values it may round to, the radius the larger
 * distance of those from the oracle's rounded value; an ambiguous ReLU mask
 * widens a gradient interval to contain 0.
 *  - pe[i][b]: bound of |p_gpu - p| / p for every bin (logit radii, the
 *    shift by the maximum, expf within 2 ulp, the FP32 sum of 256 terms,
 *    the division).
 *  - gr[k] (given target, batch scale inv_b): radius of the interval around
 *    the oracle's mode-1 gradient that the GPU's gradient lies in: the sum
 *    over the rows of each contribution's radius, plus 2 m u sum |terms| for
 *    the FP32 sum of its m terms (rows for the MLP; rows times trilinear
 *    corners for the table). The logit gradient is (p - t) inv_b with p's
 *    bound and the target renormalized in FP32 (16 u).
 * Rows beyond first-order validity are not singled out: all bounds are
 * first order in u (terms of order u^2 and of the squared radii dropped
 * except in products of intervals).
 */
#define ORC_U (1.0 / 16777216.0)

typedef struct {
    const float *par;
    const orc_nn_cfg *c;
    int32_t res[NN_L];
    const float *W[5];
    int64_t woff[5], boff[5], toff;
    uint64_t T;
} netv;

static void netv_init(netv *v, const float *par, const orc_nn_cfg *c)
{
    int fin[5] = {NN_IN, NN_H, NN_H, NN_H, NN_H}, fout[5] = {NN_H, NN_H, NN_H, NN_H, NN_OUT};
    int64_t off = 0;
    v->par = par;
    v->c = c;
    orc_nn_resolutions(c, v->res);
    for (int k = 0; k < 5; k++) {
        v->woff[k] = off; v->W[k] = par + off; off += (int64_t)fout[k] * fin[k];
        v->boff[k] = off; off += fout[k];
    }
    v->toff = off;
    v->T = (uint64_t)1 << c->log2_table;
}

/* BF16 rounding of an FP32 value within [v - r, v + r] (v the oracle's
 * value): the radius around bf16(v) of the values it may take. */
static double bf16_radius(double v, double r, int relu)
{
    double lo = v - r, hi = v + r, own = v;
    if (relu) {
        lo = lo > 0.0 ? lo : 0.0;
        hi = hi > 0.0 ? hi : 0.0;
        own = own > 0.0 ? own : 0.0;
    }
    const double c = (double)bf16r((float)own);
    const double a = c - (double)bf16r((float)lo), b = (double)bf16r((float)hi) - c;
    return a > b ? a : b;
}

typedef struct {
    double x[NN_IN];
    double h[4][NN_H], hr[4][NN_H];   /* mode-1 activations and their radii */
    double a[4][NN_H];                /* mode-1 pre-activations */
    double p[NN_OUT], pe[NN_OUT];
    enc_info ei;
} ival_state;

static void fwd_ival(const netv *v, const float *p, const float *q, ival_state *s)
{
    const double u = ORC_U;
    const int fin[5] = {NN_IN, NN_H, NN_H, NN_H, NN_H};
    encode(p, v->res, v->c, v->par + v->toff, 1, s->x, &s->ei);   /* the kernels' FP32 order: exact */
    for (int k = 0; k < 3; k++) s->x[2 * NN_L + k] = (double)bf16r(q[k]);
    static const double zero[NN_H] = {0};
    const double *in = s->x, *inr = zero;
    for (int k = 0; k < 4; k++) {
        for (int j = 0; j < NN_H; j++) {
            const double b = (double)v->par[v->boff[k] + j];
            double acc = b, rad = 0.0, sa = fabs(b);
            for (int i = 0; i < fin[k]; i++) {
                const double w = wv(v->W[k], (int64_t)j * fin[k] + i, 1);
                acc += w * in[i];
                rad += fabs(w) * inr[i];
                sa += fabs(w) * (fabs(in[i]) + inr[i]);
            }
            rad += 2.0 * (64 + 1) * u * sa;   /* padded fan-in 64, plus the bias */
            s->a[k][j] = acc;
            s->h[k][j] = (double)bf16r((float)(acc > 0.0 ? acc : 0.0));
            s->hr[k][j] = bf16_radius(acc, rad, 1);
        }
        in = s->h[k];
        inr = s->hr[k];
    }
    double z[NN_OUT], zr[NN_OUT], zmax = -1e300, rmax = 0.0;
    for (int j = 0; j < NN_OUT; j++) {
        const double b = (double)v->par[v->boff[4] + j];
        double acc = b, rad = 0.0, sa = fabs(b);
        for (int i = 0; i < NN_H; i++) {
            const double w = wv(v->W[4], (int64_t)j * NN_H + i, 1);
            acc += w * s->h[3][i];
            rad += fabs(w) * s->hr[3][i];
            sa += fabs(w) * (fabs(s->h[3][i]) + s->hr[3][i]);
        }
        z[j] = acc;
        zr[j] = rad + 2.0 * (64 + 1) * u * sa;
        if (acc > zmax) zmax = acc;
        if (zr[j] > rmax) rmax = zr[j];
    }
    double sum = 0.0;
    for (int j = 0; j < NN_OUT; j++) { s->p[j] = exp(z[j] - zmax); sum += s->p[j]; }
    for (int j = 0; j < NN_OUT; j++) {
        s->p[j] /= sum;
        /* ln(p'/p) within zr_j + max zr (the softmax of perturbed logits),
         * plus the FP32 shift, expf, sum and division */
        const double d = zr[j] + rmax + u * fabs(z[j] - zmax) + (4.0 + 2.0 * NN_OUT + 2.0) * u;
        s->pe[j] = expm1(d);
    }
}

/* Radii of one row's contributions to every parameter's gradient: mr (MLP
 * parameters, by index), tr and tc (table contributions of the row's
 * [level][corner][feature]: radius and |centre|), and ma, |centre| + radius of
 * each MLP contribution (for the accumulation bound). */
static void bwd_ival(const netv *v, const ival_state *s, const double *t, double inv_b, double *mr, double *ma,
                     double *tr, double *tc)
{
    const double u = ORC_U;
    const int fin[5] = {NN_IN, NN_H, NN_H, NN_H, NN_H};
    double dc[NN_OUT], dr[NN_OUT];
    for (int j = 0; j < NN_OUT; j++) {
        const double g = (s->p[j] - t[j]) * inv_b;
        const double eg = (s->pe[j] * s->p[j] + 16.0 * u * t[j] + u * fabs(s->p[j] - t[j])) * inv_b + u * fabs(g);
        mr[v->boff[4] + j] = eg;   /* the bias takes the unrounded FP32 value */
        ma[v->boff[4] + j] = fabs(g) + eg;
        dc[j] = (double)bf16r((float)g);
        dr[j] = bf16_radius(g, eg, 0);
        for (int k2 = 0; k2 < NN_H; k2++) {
            const double hc = s->h[3][k2], hr = s->hr[3][k2];
            const int64_t k = v->woff[4] + (int64_t)j * NN_H + k2;
            mr[k] = fabs(dc[j]) * hr + dr[j] * fabs(hc) + dr[j] * hr;
            ma[k] = fabs(dc[j] * hc) + mr[k];
        }
    }
    double gc[NN_H], grd[NN_H];   /* gradient of a layer's input: centre, radius */
    for (int k2 = 0; k2 < NN_H; k2++) {
        double c = 0.0, r = 0.0, sa = 0.0;
        for (int j = 0; j < NN_OUT; j++) {
            const double w = wv(v->W[4], (int64_t)j * NN_H + k2, 1);
            c += w * dc[j];
            r += fabs(w) * dr[j];
            sa += fabs(w) * (fabs(dc[j]) + dr[j]);
        }
        gc[k2] = c;
        grd[k2] = r + 2.0 * NN_OUT * u * sa;
    }
    for (int k = 3; k >= 0; k--) {
        double ac[NN_H], ar[NN_H];
        for (int j = 0; j < NN_H; j++) {
            const int on = s->h[k][j] > 0.0;
            const int sure = s->hr[k][j] == 0.0 || (on && s->h[k][j] - s->hr[k][j] > 0.0);
            const double c = on ? gc[j] : 0.0;
            const double r = sure ? (on ? grd[j] : 0.0) : fabs(gc[j]) + grd[j];   /* mask may differ */
            mr[v->boff[k] + j] = r;   /* unrounded FP32 */
            ma[v->boff[k] + j] = fabs(c) + r;
            ac[j] = (double)bf16r((float)c);
            ar[j] = bf16_radius(c, r, 0);
        }
        const double *in = k == 0 ? s->x : s->h[k - 1];
        for (int j = 0; j < NN_H; j++)
            for (int i = 0; i < fin[k]; i++) {
                const double ir = k == 0 ? 0.0 : s->hr[k - 1][i];
                const int64_t kk = v->woff[k] + (int64_t)j * fin[k] + i;
                mr[kk] = fabs(ac[j]) * ir + ar[j] * fabs(in[i]) + ar[j] * ir;
                ma[kk] = fabs(ac[j] * in[i]) + mr[kk];
            }
        for (int i = 0; i < fin[k]; i++) {
            double c = 0.0, r = 0.0, sa = 0.0;
            for (int j = 0; j < NN_H; j++) {
                const double w = wv(v->W[k], (int64_t)j * fin[k] + i, 1);
                c += w * ac[j];
                r += fabs(w) * ar[j];
                sa += fabs(w) * (fabs(ac[j]) + ar[j]);
            }
            gc[i] = c;
            grd[i] = r + 2.0 * NN_H * u * sa;
        }
    }
    for (int l = 0; l < NN_L; l++)
        for (int q = 0; q < 8; q++)
            for (int f = 0; f < NN_F; f++) {
                const int k = (l * 8 + q) * NN_F + f;
                const double w = fabs(s->ei.w[l][q]);
                const double c = w * fabs(gc[2 * l + f]);
                tr[k] = w * grd[2 * l + f] + u * (c + w * grd[2 * l + f]);   /* FP32 product */
                tc[k] = c;
            }
}

void orc_nn_parity_bounds(const float *par, const orc_nn_cfg *c, const float *pos, const float *nrm,
                          const double *target, int64_t n, double inv_b, double *pe, double *gr)
{
    netv v;
    netv_init(&v, par, c);
    const int64_t mlp = v.toff, np = orc_nn_num_params(c);
    const int64_t ntab = (int64_t)NN_L * (int64_t)v.T * NN_F;
    const int grad = target && gr;
    double *R = NULL, *A = NULL, *mr = NULL, *ma = NULL;
    int64_t *cnt = NULL;
    if (grad) {
        R = calloc((size_t)np, sizeof(double));
        A = calloc((size_t)np, sizeof(double));
        cnt = calloc((size_t)ntab, sizeof(int64_t));
        mr = malloc(sizeof(double) * (size_t)mlp);
        ma = malloc(sizeof(double) * (size_t)mlp);
    }
    ival_state *s = malloc(sizeof(ival_state));
    for (int64_t i = 0; i < n; i++) {
        const float p[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        const float q[3] = {nrm[i], nrm[n + i], nrm[2 * n + i]};
        fwd_ival(&v, p, q, s);
        if (pe)
            for (int j = 0; j < NN_OUT; j++) pe[i * NN_OUT + j] = s->pe[j];
        if (!grad) continue;
        double tr[NN_L * 8 * NN_F], tc[NN_L * 8 * NN_F];
        bwd_ival(&v, s, target + i * NN_OUT, inv_b, mr, ma, tr, tc);
        for (int64_t k = 0; k < mlp; k++) { R[k] += mr[k]; A[k] += ma[k]; }
        for (int l = 0; l < NN_L; l++)
            for (int qq = 0; qq < 8; qq++)
                for (int f = 0; f < NN_F; f++) {
                    const int k = (l * 8 + qq) * NN_F + f;
                    const int64_t e = ((int64_t)l * (int64_t)v.T + s->ei.idx[l][qq]) * NN_F + f;
                    R[mlp + e] += tr[k];
                    A[mlp + e] += tc[k] + tr[k];
                    cnt[e] += 1;
                }
    }
    if (grad) {
        for (int64_t k = 0; k < np; k++) {
            const double m = k < mlp ? (double)n : (double)cnt[k - mlp];
            gr[k] = R[k] + 2.0 * m * ORC_U * A[k];
        }
        free(R); free(A); free(cnt); free(mr); free(ma);
    }
    free(s);
}
