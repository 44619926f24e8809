/*
 * mlp_ref.c -- FP64 CPU oracle of the learned eddy-viscosity closure.
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_ref.c).  Shares no code with the HIP
 * library; it parses the same closure blob format independently.
 *
 * The paper uses the Smagorinsky model (Sec. 2.2) and names other SGS models
 * as future work (Sec. 6).  The learned closure replaces nu_t of Sec. 2.2 by
 * a small network; everything here is a design choice of this project, fixed
 * identically on both sides:
 *
 *   features (9): with P = Pi_neq / (rho c_s^2) and n = e_y (wall normal),
 *     x1 = tr P, x2 = tr P^2, x3 = tr P^3, x4 = n.P.n, x5 = n.P^2.n,
 *     x6 = sqrt(tr P^2), x7 = y / h, x8 = LAD(y), x9 = filter width (= 1)
 *   standardisation z_i = (x_i - mean_i) / std_i
 *   network 9-64-64-1: h1 = gelu(W1 z + b1), h2 = gelu(W2 h1 + b2),
 *     o = w3 . h2 + b3, nu_t = s * softplus(o)
 *   gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))
 *   fallback: if any raw feature lies outside [lo_i, hi_i], nu_t is the
 *     Smagorinsky value.  The bounds are FP32 numbers and the test is taken
 *     in FP32 on the feature rounded to FP32: a yes/no decision that a
 *     floating-point comparison makes is made in the same precision on both
 *     sides (the kernel's; the bounds come from the training data, where
 *     the extreme values, such as the LAD of the densest row, are the
 *     bounds themselves).
 *   loss for training: mean over the batch of (softplus(o) - y)^2, with y the
 *     target nu_t / s.
 *
 * Closure blob (little-endian), 10184 bytes:
 *     0  char  magic[4] = "LBMC"
 *     4  u32   version = 1
 *     8  u32   n_in = 9, n_h1 = 64, n_h2 = 64, reserved = 0
 *    24  f32   mean[9], std[9], lo[9], hi[9]
 *   168  f32   out_scale s, canopy_h, pad, pad
 *   184  f32   b1[64], b2[64], b3, pad[3]
 *   712  bf16  W1[64][9] (row = hidden unit), W2[64][64], w3[64]
 *
 * Flat parameter order used by the gradient routine (4865 values):
 *   W1[64][9], b1[64], W2[64][64], b2[64], w3[64], b3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NIN 9
#define NH1 64
#define NH2 64
#define NPARAM (NH1 * NIN + NH1 + NH2 * NH1 + NH2 + NH2 + 1)
#define BLOB_BYTES 10184

struct mlp_ref {
    double mean[NIN], std[NIN], lo[NIN], hi[NIN];
    double scale, canopy_h;
    double p[NPARAM];
};

static const double PI_D = 3.14159265358979323846;

static double bf16_to_double(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double f32_at(const unsigned char *b, size_t off) {
    float f;
    memcpy(&f, b + off, 4);
    return (double)f;
}

int ref_mlp_nparams(void) { return NPARAM; }

/* parse a blob; NULL if its shape or version is wrong */
void *ref_mlp_load(const void *blob, size_t nbytes) {
    const unsigned char *b = (const unsigned char *)blob;
    if (!b || nbytes != BLOB_BYTES || memcmp(b, "LBMC", 4) != 0) return NULL;
    uint32_t hdr[5];
    memcpy(hdr, b + 4, sizeof(hdr));
    if (hdr[0] != 1 || hdr[1] != NIN || hdr[2] != NH1 || hdr[3] != NH2) return NULL;
    struct mlp_ref *m = (struct mlp_ref *)calloc(1, sizeof(struct mlp_ref));
    for (int i = 0; i < NIN; ++i) {
        m->mean[i] = f32_at(b, 24 + 4 * i);
        m->std[i] = f32_at(b, 24 + 36 + 4 * i);
        m->lo[i] = f32_at(b, 24 + 72 + 4 * i);
        m->hi[i] = f32_at(b, 24 + 108 + 4 * i);
    }
    m->scale = f32_at(b, 168);
    m->canopy_h = f32_at(b, 172);
    double *W1 = m->p, *b1 = W1 + NH1 * NIN, *W2 = b1 + NH1, *b2 = W2 + NH2 * NH1,
           *w3 = b2 + NH2, *b3 = w3 + NH2;
    for (int i = 0; i < NH1; ++i) b1[i] = f32_at(b, 184 + 4 * i);
    for (int i = 0; i < NH2; ++i) b2[i] = f32_at(b, 184 + 256 + 4 * i);
    *b3 = f32_at(b, 184 + 512);
    const unsigned char *w = b + 712;
    uint16_t v;
    for (int i = 0; i < NH1 * NIN; ++i) { memcpy(&v, w, 2); w += 2; W1[i] = bf16_to_double(v); }
    for (int i = 0; i < NH2 * NH1; ++i) { memcpy(&v, w, 2); w += 2; W2[i] = bf16_to_double(v); }
    for (int i = 0; i < NH2; ++i) { memcpy(&v, w, 2); w += 2; w3[i] = bf16_to_double(v); }
    return m;
}

void ref_mlp_free(void *m) { free(m); }

double ref_mlp_canopy_h(const void *m) { return ((const struct mlp_ref *)m)->canopy_h; }

double ref_gelu(double x) {
    return 0.5 * x * (1.0 + tanh(sqrt(2.0 / PI_D) * (x + 0.044715 * x * x * x)));
}

static double gelu_grad(double x) {
    double k = sqrt(2.0 / PI_D);
    double a = k * (x + 0.044715 * x * x * x);
    double t = tanh(a);
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * k * (1.0 + 3.0 * 0.044715 * x * x);
}

double ref_softplus(double x) {
    /* log(1 + e^x), written to stay finite for large |x| */
    return (x > 0.0) ? x + log1p(exp(-x)) : log1p(exp(x));
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* network on one standardised input; returns o (before softplus) and, if
 * asked, the pre-activations of both hidden layers */
static double net(const double *p, const double *z, double *a1, double *a2) {
    const double *W1 = p, *b1 = W1 + NH1 * NIN, *W2 = b1 + NH1, *b2 = W2 + NH2 * NH1,
                 *w3 = b2 + NH2, *b3 = w3 + NH2;
    double h1[NH1], h2[NH2], pre1[NH1], pre2[NH2];
    for (int r = 0; r < NH1; ++r) {
        double s = b1[r];
        for (int i = 0; i < NIN; ++i) s += W1[r * NIN + i] * z[i];
        pre1[r] = s;
        h1[r] = ref_gelu(s);
    }
    for (int r = 0; r < NH2; ++r) {
        double s = b2[r];
        for (int i = 0; i < NH1; ++i) s += W2[r * NH1 + i] * h1[i];
        pre2[r] = s;
        h2[r] = ref_gelu(s);
    }
    double o = *b3;
    for (int i = 0; i < NH2; ++i) o += w3[i] * h2[i];
    if (a1) memcpy(a1, pre1, sizeof(pre1));
    if (a2) memcpy(a2, pre2, sizeof(pre2));
    return o;
}

/* o for n standardised inputs Z[n][9] with flat parameters p */
void ref_mlp_apply(const double *p, const double *Z, int64_t n, double *o) {
    for (int64_t s = 0; s < n; ++s) o[s] = net(p, Z + NIN * s, NULL, NULL);
}

/* loss = (1/n) sum (softplus(o_s) - y_s)^2 and its gradient w.r.t. the flat
 * parameters (backpropagation through the network above) */
double ref_mlp_loss_grad(const double *p, const double *Z, const double *y, int64_t n,
                         double *grad) {
    const double *W2 = p + NH1 * NIN + NH1, *w3 = W2 + NH2 * NH1 + NH2;
    double *gW1 = grad, *gb1 = gW1 + NH1 * NIN, *gW2 = gb1 + NH1, *gb2 = gW2 + NH2 * NH1,
           *gw3 = gb2 + NH2, *gb3 = gw3 + NH2;
    memset(grad, 0, NPARAM * sizeof(double));
    double loss = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const double *z = Z + NIN * s;
        double pre1[NH1], pre2[NH2], h1[NH1], h2[NH2];
        double o = net(p, z, pre1, pre2);
        for (int i = 0; i < NH1; ++i) h1[i] = ref_gelu(pre1[i]);
        for (int i = 0; i < NH2; ++i) h2[i] = ref_gelu(pre2[i]);
        double e = ref_softplus(o) - y[s];
        loss += e * e;
        double go = 2.0 * e * sigmoid(o) / (double)n; /* d loss / d o */
        *gb3 += go;
        double g2[NH2];
        for (int i = 0; i < NH2; ++i) {
            gw3[i] += go * h2[i];
            g2[i] = go * w3[i] * gelu_grad(pre2[i]); /* d loss / d pre2 */
            gb2[i] += g2[i];
        }
        double g1[NH1];
        for (int c = 0; c < NH1; ++c) {
            double s1 = 0.0;
            for (int r = 0; r < NH2; ++r) {
                gW2[r * NH1 + c] += g2[r] * h1[c];
                s1 += W2[r * NH1 + c] * g2[r];
            }
            g1[c] = s1 * gelu_grad(pre1[c]);
        }
        for (int r = 0; r < NH1; ++r) {
            gb1[r] += g1[r];
            for (int i = 0; i < NIN; ++i) gW1[r * NIN + i] += g1[r] * z[i];
        }
    }
    return loss / (double)n;
}

/* raw features of one cell (see the header) */
int ref_mlp_features(const struct mlp_ref *m, double tau0, double rho, const double *Pineq,
                     double yh, double lad, double *x) {
    (void)m;
    (void)tau0;
    double P[9], P2[9];
    for (int k = 0; k < 9; ++k) P[k] = Pineq[k] / (rho / 3.0);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += P[3 * a + c] * P[3 * c + b];
            P2[3 * a + b] = s;
        }
    double tr1 = P[0] + P[4] + P[8];
    double tr2 = P2[0] + P2[4] + P2[8];
    double tr3 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) tr3 += P2[3 * a + c] * P[3 * c + a];
    x[0] = tr1;
    x[1] = tr2;
    x[2] = tr3;
    x[3] = P[4];  /* n.P.n with n = e_y */
    x[4] = P2[4]; /* n.P^2.n */
    x[5] = sqrt(tr2);
    x[6] = yh;
    x[7] = lad;
    x[8] = 1.0;
    return 0;
}

/* nu_t of the learned closure, or the Smagorinsky value when any feature is
 * outside the stored range */
double ref_mlp_closure_nut(const struct mlp_ref *m, const double *x, int *used_fallback,
                           double smag_nut) {
    for (int i = 0; i < NIN; ++i) {
        const float xf = (float)x[i];
        if (!(xf >= (float)m->lo[i] && xf <= (float)m->hi[i])) {
            *used_fallback = 1;
            return smag_nut;
        }
    }
    double z[NIN];
    for (int i = 0; i < NIN; ++i) z[i] = (x[i] - m->mean[i]) / m->std[i];
    double o = net(m->p, z, NULL, NULL);
    *used_fallback = 0;
    return m->scale * ref_softplus(o);
}

/* raw-feature entry point for tests: nu_t for n cells given raw features */
void ref_mlp_predict(const void *mp, const double *X, int64_t n, const double *smag_nut,
                     double *nut, int *fallback) {
    const struct mlp_ref *m = (const struct mlp_ref *)mp;
    for (int64_t s = 0; s < n; ++s) {
        int fb = 0;
        nut[s] = ref_mlp_closure_nut(m, X + NIN * s, &fb, smag_nut ? smag_nut[s] : 0.0);
        if (fallback) fallback[s] = fb;
    }
}
