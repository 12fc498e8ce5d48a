/*
 * mlp.c -- plain FP64 reference of the per-pair learned potential: a small
 * MLP that maps a pair distance r to the exchange J(r) and the mechanical
 * pair energy phi(r), with its derivative d/dr and the gradients of a
 * training loss with respect to every weight.
 *
 * TEST INFRASTRUCTURE ONLY (like oracle.c): no product code calls it.
 *
 * Network (5378 parameters):
 *   b_k(r)  = exp(-((r - mu_k)/sigma)^2),  mu_k = k * 5/15 A, k = 0..15
 *   a1      = silu(W1 b + c1)      W1: 64 x 16
 *   a2      = silu(W2 a1 + c2)     W2: 64 x 64
 *   y       = W3 a2 + c3           W3:  2 x 64
 *   J(r)    = sJ * y0(r) for r < ex_rc, else 0          (Heaviside cut as
 *             the analytic exchange)
 *   phi(r)  = sP * [y1(r) - y1(rc) - (r - rc) y1'(rc)] for r < rc, else 0
 *             (shifted force at the mechanical cutoff rc)
 * silu(z) = z / (1 + e^{-z}).
 * Parameter vector layout: W1 (row-major 64x16), c1[64], W2 (64x64), c2[64],
 * W3 (2x64), c3[2].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mlp.h"

#define NB 16
#define NH 64
#define NO 2
#define NPARAM (NH * NB + NH + NH * NH + NH + NO * NH + NO)

int mlp_nparam(void) { return NPARAM; }

static double sig(double z) { return 1.0 / (1.0 + exp(-z)); }
static double silu(double z) { return z * sig(z); }
static double dsilu(double z) { double s = sig(z); return s * (1.0 + z * (1.0 - s)); }
static double d2silu(double z)
{
    double s = sig(z);
    double ds = s * (1.0 - s);
    return ds * (2.0 + z * (1.0 - 2.0 * s));
}

/* Forward value and r-tangent of the raw outputs y(r), y'(r), keeping the
 * intermediates for the reverse pass. */
typedef struct {
    double b[NB], db[NB];
    double z1[NH], a1[NH], dz1[NH], da1[NH];
    double z2[NH], a2[NH], dz2[NH], da2[NH];
    double y[NO], dy[NO];
} mlp_tape;

static void raw_forward(const mlp_cfg *c, const double *p, double r, mlp_tape *t)
{
    const double *W1 = p, *c1 = W1 + NH * NB, *W2 = c1 + NH, *c2 = W2 + NH * NH;
    const double *W3 = c2 + NH, *c3 = W3 + NO * NH;
    for (int k = 0; k < NB; ++k) {
        double x = (r - k * c->mu_step) / c->sigma;
        t->b[k] = exp(-x * x);
        t->db[k] = t->b[k] * (-2.0 * x / c->sigma);
    }
    for (int h = 0; h < NH; ++h) {
        double z = c1[h], dz = 0.0;
        for (int k = 0; k < NB; ++k) {
            z += W1[h * NB + k] * t->b[k];
            dz += W1[h * NB + k] * t->db[k];
        }
        t->z1[h] = z; t->dz1[h] = dz;
        t->a1[h] = silu(z); t->da1[h] = dsilu(z) * dz;
    }
    for (int h = 0; h < NH; ++h) {
        double z = c2[h], dz = 0.0;
        for (int k = 0; k < NH; ++k) {
            z += W2[h * NH + k] * t->a1[k];
            dz += W2[h * NH + k] * t->da1[k];
        }
        t->z2[h] = z; t->dz2[h] = dz;
        t->a2[h] = silu(z); t->da2[h] = dsilu(z) * dz;
    }
    for (int o = 0; o < NO; ++o) {
        double y = c3[o], dy = 0.0;
        for (int k = 0; k < NH; ++k) {
            y += W3[o * NH + k] * t->a2[k];
            dy += W3[o * NH + k] * t->da2[k];
        }
        t->y[o] = y; t->dy[o] = dy;
    }
}

/* Reverse pass: given adjoints ybar = dL/dy and dybar = dL/dy' of the raw
 * outputs at one r, accumulate dL/dparams into g. */
static void raw_backward(const double *p, const mlp_tape *t, const double ybar[NO],
                         const double dybar[NO], double *g)
{
    const double *W1 = p, *c1 = W1 + NH * NB, *W2 = c1 + NH, *c2 = W2 + NH * NH;
    const double *W3 = c2 + NH;
    (void)c1; (void)c2;
    double *gW1 = g, *gc1 = gW1 + NH * NB, *gW2 = gc1 + NH, *gc2 = gW2 + NH * NH;
    double *gW3 = gc2 + NH, *gc3 = gW3 + NO * NH;
    double a2b[NH], da2b[NH], z2b[NH], dz2b[NH];
    for (int k = 0; k < NH; ++k) {
        a2b[k] = 0.0; da2b[k] = 0.0;
        for (int o = 0; o < NO; ++o) {
            gW3[o * NH + k] += ybar[o] * t->a2[k] + dybar[o] * t->da2[k];
            a2b[k] += W3[o * NH + k] * ybar[o];
            da2b[k] += W3[o * NH + k] * dybar[o];
        }
    }
    for (int o = 0; o < NO; ++o) gc3[o] += ybar[o];
    /* da2 = silu'(z2) dz2;  a2 = silu(z2) */
    for (int h = 0; h < NH; ++h) {
        dz2b[h] = dsilu(t->z2[h]) * da2b[h];
        z2b[h] = d2silu(t->z2[h]) * t->dz2[h] * da2b[h] + dsilu(t->z2[h]) * a2b[h];
    }
    double a1b[NH], da1b[NH], z1b[NH], dz1b[NH];
    for (int k = 0; k < NH; ++k) { a1b[k] = 0.0; da1b[k] = 0.0; }
    for (int h = 0; h < NH; ++h) {
        gc2[h] += z2b[h];
        for (int k = 0; k < NH; ++k) {
            gW2[h * NH + k] += z2b[h] * t->a1[k] + dz2b[h] * t->da1[k];
            a1b[k] += W2[h * NH + k] * z2b[h];
            da1b[k] += W2[h * NH + k] * dz2b[h];
        }
    }
    for (int h = 0; h < NH; ++h) {
        dz1b[h] = dsilu(t->z1[h]) * da1b[h];
        z1b[h] = d2silu(t->z1[h]) * t->dz1[h] * da1b[h] + dsilu(t->z1[h]) * a1b[h];
    }
    for (int h = 0; h < NH; ++h) {
        gc1[h] += z1b[h];
        for (int k = 0; k < NB; ++k) gW1[h * NB + k] += z1b[h] * t->b[k] + dz1b[h] * t->db[k];
    }
}

/* J, phi and their r-derivatives at r (physical outputs, eV and eV/A). */
void mlp_eval(const mlp_cfg *c, const double *p, double r, double out[4])
{
    mlp_tape t, tc;
    raw_forward(c, p, r, &t);
    raw_forward(c, p, c->rc, &tc);
    double J = 0.0, dJ = 0.0, P = 0.0, dP = 0.0;
    if (r < c->ex_rc) { J = c->sJ * t.y[0]; dJ = c->sJ * t.dy[0]; }
    if (r < c->rc) {
        P = c->sP * (t.y[1] - tc.y[1] - (r - c->rc) * tc.dy[1]);
        dP = c->sP * (t.dy[1] - tc.dy[1]);
    }
    out[0] = J; out[1] = dJ; out[2] = P; out[3] = dP;
}

void mlp_raw(const mlp_cfg *c, const double *p, double r, double y[2], double dy[2])
{
    mlp_tape t;
    raw_forward(c, p, r, &t);
    y[0] = t.y[0]; y[1] = t.y[1];
    dy[0] = t.dy[0]; dy[1] = t.dy[1];
}

/* Gradient of a linear functional of the physical outputs at a set of
 * distances: L = sum_q (aJ_q J(r_q) + adJ_q J'(r_q) + aP_q phi(r_q) +
 * adP_q phi'(r_q)). The shifted-force terms of phi bring in y1(rc) and
 * y1'(rc), whose adjoints are summed over all q. */
void mlp_grad_linear(const mlp_cfg *c, const double *p, int n, const double *r,
                     const double *aJ, const double *adJ, const double *aP,
                     const double *adP, double *g)
{
    memset(g, 0, NPARAM * sizeof(double));
    double yc_bar = 0.0, dyc_bar = 0.0;
    mlp_tape t;
    for (int q = 0; q < n; ++q) {
        raw_forward(c, p, r[q], &t);
        double ybar[NO] = {0.0, 0.0}, dybar[NO] = {0.0, 0.0};
        if (r[q] < c->ex_rc) {
            ybar[0] = aJ[q] * c->sJ;
            dybar[0] = adJ[q] * c->sJ;
        }
        if (r[q] < c->rc) {
            ybar[1] = aP[q] * c->sP;
            dybar[1] = adP[q] * c->sP;
            /* phi = sP (y1 - y1c - (r - rc) y1c'); phi' = sP (y1' - y1c') */
            yc_bar += -aP[q] * c->sP;
            dyc_bar += -aP[q] * c->sP * (r[q] - c->rc) - adP[q] * c->sP;
        }
        raw_backward(p, &t, ybar, dybar, g);
    }
    raw_forward(c, p, c->rc, &t);
    double ybar[NO] = {0.0, yc_bar}, dybar[NO] = {0.0, dyc_bar};
    raw_backward(p, &t, ybar, dybar, g);
}

/* ------------------------------------------------------------------------
 * Training loss of one snapshot with the MLP standing in for J and phi.
 * Unordered pairs (pi[q] < pj[q]) within the list radius; minimum image
 * in the box L. With e_ij = (r_i - r_j)/r:
 *   E    = sum_q [phi(r_q) - J(r_q) s_i.s_j]
 *   F_i  = sum_j [-phi'(r) + J'(r) s_i.s_j] e_ij
 *   hw_i = sum_j J(r_ij) s_j            (exchange part of hbar omega_i)
 *   loss = wE ((E - Eref)/N)^2 + wF |F - Fref|^2/(3N) + wW |hw - hwref|^2/(3N)
 * The gradient follows from the per-pair adjoints of J, J', phi, phi'.
 * Returns the loss; g (may be NULL) receives dloss/dparams.
 */
double mlp_loss_grad(const mlp_cfg *c, const double *p, int N, const double L[3],
                     const double *r, const double *s, int npair, const int *pi,
                     const int *pj, double Eref, const double *Fref, const double *Wref,
                     const double w[3], double *g)
{
    double *rr = (double *)malloc((size_t)(npair > 0 ? npair : 1) * sizeof(double));
    double *e = (double *)malloc((size_t)(npair > 0 ? npair : 1) * 3 * sizeof(double));
    double *val = (double *)malloc((size_t)(npair > 0 ? npair : 1) * 4 * sizeof(double));
    double *F = (double *)calloc((size_t)N * 3, sizeof(double));
    double *Wv = (double *)calloc((size_t)N * 3, sizeof(double));
    double E = 0.0;
    for (int q = 0; q < npair; ++q) {
        int i = pi[q], j = pj[q];
        double d[3];
        for (int a = 0; a < 3; ++a) {
            double x = r[3 * i + a] - r[3 * j + a];
            d[a] = x - L[a] * nearbyint(x / L[a]);
        }
        double rq = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        rr[q] = rq;
        for (int a = 0; a < 3; ++a) e[3 * q + a] = d[a] / rq;
        mlp_eval(c, p, rq, val + 4 * q);
        double sij = s[3 * i] * s[3 * j] + s[3 * i + 1] * s[3 * j + 1] + s[3 * i + 2] * s[3 * j + 2];
        E += val[4 * q + 2] - val[4 * q] * sij;
        double cf = -val[4 * q + 3] + val[4 * q + 1] * sij;
        for (int a = 0; a < 3; ++a) {
            F[3 * i + a] += cf * e[3 * q + a];
            F[3 * j + a] -= cf * e[3 * q + a];
            Wv[3 * i + a] += val[4 * q] * s[3 * j + a];
            Wv[3 * j + a] += val[4 * q] * s[3 * i + a];
        }
    }
    double eres = (E - Eref) / N;
    double loss = w[0] * eres * eres;
    double lf = 0.0, lw = 0.0;
    for (int k = 0; k < 3 * N; ++k) {
        lf += (F[k] - Fref[k]) * (F[k] - Fref[k]);
        lw += (Wv[k] - Wref[k]) * (Wv[k] - Wref[k]);
    }
    loss += w[1] * lf / (3.0 * N) + w[2] * lw / (3.0 * N);
    if (g) {
        double *aJ = (double *)calloc((size_t)(npair > 0 ? npair : 1), sizeof(double));
        double *adJ = (double *)calloc((size_t)(npair > 0 ? npair : 1), sizeof(double));
        double *aP = (double *)calloc((size_t)(npair > 0 ? npair : 1), sizeof(double));
        double *adP = (double *)calloc((size_t)(npair > 0 ? npair : 1), sizeof(double));
        double dE = 2.0 * w[0] * eres / N;
        for (int q = 0; q < npair; ++q) {
            int i = pi[q], j = pj[q];
            double sij = s[3 * i] * s[3 * j] + s[3 * i + 1] * s[3 * j + 1] + s[3 * i + 2] * s[3 * j + 2];
            aP[q] += dE;
            aJ[q] += -dE * sij;
            double dc = 0.0;
            for (int a = 0; a < 3; ++a) {
                double gi = 2.0 * w[1] * (F[3 * i + a] - Fref[3 * i + a]) / (3.0 * N);
                double gj = 2.0 * w[1] * (F[3 * j + a] - Fref[3 * j + a]) / (3.0 * N);
                dc += (gi - gj) * e[3 * q + a];
                double hi = 2.0 * w[2] * (Wv[3 * i + a] - Wref[3 * i + a]) / (3.0 * N);
                double hj = 2.0 * w[2] * (Wv[3 * j + a] - Wref[3 * j + a]) / (3.0 * N);
                aJ[q] += hi * s[3 * j + a] + hj * s[3 * i + a];
            }
            adP[q] += -dc;
            adJ[q] += dc * sij;
        }
        mlp_grad_linear(c, p, npair, rr, aJ, adJ, aP, adP, g);
        free(aJ); free(adJ); free(aP); free(adP);
    }
    free(rr); free(e); free(val); free(F); free(Wv);
    return loss;
}
