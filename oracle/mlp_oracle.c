/*
 * mlp_oracle.c -- plain FP64 CPU oracle of the learned warm start: a
 * multilayer perceptron 16 -> 64 -> GELU -> 64 -> GELU -> 16 that predicts a
 * marker's initial forcing from 12 (zero-padded to 16) standardised
 * features, its loss gradient and the Adam update.  The learned warm start is
 * not part of the paper; its definition (sizes, BF16 weights with FP32
 * accumulation, exact-erf GELU, MSE on standardised targets, Adam) is the
 * library's and is written out here as the reference.
 *
 * TEST INFRASTRUCTURE ONLY (see prs_oracle.c).
 *
 * Parameter vector (flat, double), row-major, out x in:
 *   W1[64][16], b1[64], W2[64][64], b2[64], W3[16][64], b3[16]   (6288 values)
 * With emulate_bf16 != 0 the values that the device multiplies in BF16 --
 * weights, inputs, hidden activations and back-propagated errors -- are
 * rounded to BF16 (round to nearest even, via FP32) before use; sums stay in
 * FP64.  With emulate_bf16 == 0 everything is plain FP64 (for the
 * finite-difference check).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define NI 16
#define NH 64
#define NO 16
#define NOUT 3

enum {
    OFF_W1 = 0,
    OFF_B1 = OFF_W1 + NH * NI,
    OFF_W2 = OFF_B1 + NH,
    OFF_B2 = OFF_W2 + NH * NH,
    OFF_W3 = OFF_B2 + NH,
    OFF_B3 = OFF_W3 + NO * NH,
    NPARAM = OFF_B3 + NO
};

int or_mlp_nparam(void) { return NPARAM; }

/* FP32 value of x rounded to the nearest BF16 (ties to even). */
double or_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    memcpy(&f, &u, 4);
    return (double)f;
}

static double E(double x, int emu) { return emu ? or_bf16(x) : x; }

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

static double gelu_d(double z)
{
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
}

typedef struct {
    double xb[NI], z1[NH], a1[NH], z2[NH], a2[NH], y[NO];
} fwd_t;

static void forward_one(const double *P, const double *x, int emu, fwd_t *s)
{
    for (int k = 0; k < NI; ++k)
        s->xb[k] = E(x[k], emu);
    for (int i = 0; i < NH; ++i) {
        double acc = 0.0;
        for (int k = 0; k < NI; ++k)
            acc += E(P[OFF_W1 + i * NI + k], emu) * s->xb[k];
        s->z1[i] = acc + P[OFF_B1 + i];
        s->a1[i] = E(gelu(s->z1[i]), emu);
    }
    for (int i = 0; i < NH; ++i) {
        double acc = 0.0;
        for (int k = 0; k < NH; ++k)
            acc += E(P[OFF_W2 + i * NH + k], emu) * s->a1[k];
        s->z2[i] = acc + P[OFF_B2 + i];
        s->a2[i] = E(gelu(s->z2[i]), emu);
    }
    for (int o = 0; o < NO; ++o) {
        double acc = 0.0;
        for (int k = 0; k < NH; ++k)
            acc += E(P[OFF_W3 + o * NH + k], emu) * s->a2[k];
        s->y[o] = acc + P[OFF_B3 + o];
    }
}

/* Y[b][0..15] = network output for X[b][0..15]. */
void or_mlp_forward(const double *P, int32_t B, const double *X, double *Y, int32_t emu)
{
    fwd_t s;
    for (int b = 0; b < B; ++b) {
        forward_one(P, &X[NI * b], emu, &s);
        for (int o = 0; o < NO; ++o)
            Y[NO * b + o] = s.y[o];
    }
}

/* Loss L = (1/(3B)) sum_b sum_{o<3} (Y[b][o] - T[b][o])^2 and its gradient
 * with respect to the parameter vector (grad must hold NPARAM values). */
double or_mlp_loss_grad(const double *P, int32_t B, const double *X, const double *T,
                        double *grad, int32_t emu)
{
    memset(grad, 0, sizeof(double) * NPARAM);
    double loss = 0.0;
    fwd_t s;
    for (int b = 0; b < B; ++b) {
        forward_one(P, &X[NI * b], emu, &s);
        double dy[NO], dyb[NO], da2[NH], dz2[NH], dz2b[NH], da1[NH], dz1[NH], dz1b[NH];
        for (int o = 0; o < NO; ++o) {
            double e = o < NOUT ? s.y[o] - T[NOUT * b + o] : 0.0;
            if (o < NOUT)
                loss += e * e;
            dy[o] = o < NOUT ? 2.0 * e / (3.0 * B) : 0.0;
            dyb[o] = E(dy[o], emu);
        }
        for (int o = 0; o < NO; ++o) {
            for (int k = 0; k < NH; ++k)
                grad[OFF_W3 + o * NH + k] += dyb[o] * s.a2[k];
            grad[OFF_B3 + o] += dy[o];
        }
        for (int k = 0; k < NH; ++k) {
            double acc = 0.0;
            for (int o = 0; o < NO; ++o)
                acc += E(P[OFF_W3 + o * NH + k], emu) * dyb[o];
            da2[k] = acc;
            dz2[k] = da2[k] * gelu_d(s.z2[k]);
            dz2b[k] = E(dz2[k], emu);
        }
        for (int i = 0; i < NH; ++i) {
            for (int k = 0; k < NH; ++k)
                grad[OFF_W2 + i * NH + k] += dz2b[i] * s.a1[k];
            grad[OFF_B2 + i] += dz2[i];
        }
        for (int k = 0; k < NH; ++k) {
            double acc = 0.0;
            for (int i = 0; i < NH; ++i)
                acc += E(P[OFF_W2 + i * NH + k], emu) * dz2b[i];
            da1[k] = acc;
            dz1[k] = da1[k] * gelu_d(s.z1[k]);
            dz1b[k] = E(dz1[k], emu);
        }
        for (int i = 0; i < NH; ++i) {
            for (int k = 0; k < NI; ++k)
                grad[OFF_W1 + i * NI + k] += dz1b[i] * s.xb[k];
            grad[OFF_B1 + i] += dz1[i];
        }
    }
    return loss / (3.0 * B);
}

/* One Adam update (bias-corrected, step t >= 1) of n parameters. */
void or_mlp_adam(double *P, double *m, double *v, const double *g, int32_t n, int32_t t,
                 double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        P[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
