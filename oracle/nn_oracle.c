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
