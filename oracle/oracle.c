/*
 * oracle.c -- plain serial FP64 CPU reference of the coupled spin-lattice
 * Suzuki-Trotter (ST) step of Tranchida, Plimpton, Thibaudeau and Thompson,
 * "Massively parallel symplectic algorithm for coupled magnetic spin dynamics
 * and molecular dynamics" (J. Comput. Phys. 2018, arXiv:1801.10233).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path. It shares no
 * code with the HIP library.
 *
 * Everything is written for a reader who checks it against the paper:
 * no blocking, no fusion, no reordering beyond what the equations state.
 * Where the paper is silent or garbled, the reading taken is stated at the
 * place it is used (constants, pair counting, truncation, noise amplitude,
 * colouring, rebuild rule, Philox layout).
 */
#include "oracle.h"
#include "mlp.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXC 64   /* colours tracked by the greedy colouring */

struct orc_sys {
    int N;
    double L[3];
    int frozen;
    double skin;
    uint64_t seed;
    uint32_t replica;
    int ordering;
    int sect[3];
    orc_pot pot;

    double *r, *v, *s, *m;     /* [N][3], [N][3], [N][3], [N] */
    int64_t step;

    /* neighbour list (CSR; spin entries first in each row) */
    int *off, *idx, *nspin;
    long cap;
    int have_list, user_list;
    double *rbuild;
    int nrebuild;

    /* colouring */
    int *colour;
    int K;
    int have_colour;
    int kbase;                   /* colours of the last full colouring */

    /* forces at the current positions and spins */
    double *F;
    int have_F;

    /* terms of the rebuild predictor taken at the previous step boundary:
     * largest displacement since the build, largest speed, closest
     * same-colour spin pair, and |dt| of the step that followed it */
    double disp_prev, vmax_prev, wmin_prev, adt_prev;
    int have_D;

    /* learned pair potential standing in for J and V (NULL: analytic) */
    mlp_cfg mcfg;
    double *mparams;

    /* scratch */
    double *w_tmp;
    double *rho;           /* embedded-atom densities of the current state */
    int *cls, *cls_off;
    int ncls;
};

/* ------------------------------------------------------------------------
 * Interaction functions.
 * ---------------------------------------------------------------------- */

/* Bethe-Slater exchange (appendix on the exchange parametrisation, Eq.
 * BSfunction): J(r) = 4 alpha u (1 - gamma u) exp(-u), u = (r/delta)^2, cut
 * by a Heaviside step at R_c. dJ/dr = (8 alpha r/delta^2) exp(-u)
 * (1 - (1+2 gamma) u + gamma u^2) inside the cutoff. */
static double bs_exchange(const orc_pot *p, double r, double *dJdr)
{
    double u = (r / p->ex_delta) * (r / p->ex_delta);
    double e = exp(-u);
    *dJdr = 8.0 * p->ex_alpha * r / (p->ex_delta * p->ex_delta) * e *
            (1.0 - (1.0 + 2.0 * p->ex_gamma) * u + p->ex_gamma * u * u);
    return 4.0 * p->ex_alpha * u * (1.0 - p->ex_gamma * u) * e;
}

/* The printed cut leaves a step of J(R_c) in the pair energy, which a
 * symplectic integrator cannot follow: each crossing of R_c changes the
 * total energy by J(R_c) s_i.s_j. With ex_shift set the exchange is
 * shifted in r^2 inside the cutoff,
 *   J(r) - J(R_c) - (r^2 - R_c^2) J'(R_c) / (2 R_c),
 * which vanishes at R_c together with its derivative J'(r) - r J'(R_c)/R_c
 * (the Morse rule in r, written in r^2 so that it needs no square root). */
double orc_J(const orc_pot *p, double r, double *dJdr)
{
    if (!(r < p->ex_rc) || p->ex_alpha == 0.0) {
        if (dJdr) *dJdr = 0.0;
        return 0.0;
    }
    double dJ;
    double J = bs_exchange(p, r, &dJ);
    if (p->ex_shift) {
        double dJc;
        const double rc = p->ex_rc;
        double Jc = bs_exchange(p, rc, &dJc);
        J -= Jc + (r * r - rc * rc) * dJc / (2.0 * rc);
        dJ -= r * dJc / rc;
    }
    if (dJdr) *dJdr = dJ;
    return J;
}

/* The three-parameter Bethe-Slater radial form 4 a u (1 - g u) e^{-u},
 * u = (r/d)^2, cut at rc, and its derivative: the exchange J(r) above, and
 * also the Neel function g1(r) (appendix A, spin-orbit coupling) and the
 * magnitude of the Dzyaloshinskii-Moriya vector. */
static double bethe_slater(double a, double g, double dl, double rc, double r, double *dfdr)
{
    if (!(r < rc) || a == 0.0) {
        *dfdr = 0.0;
        return 0.0;
    }
    double u = (r / dl) * (r / dl);
    double e = exp(-u);
    *dfdr = 8.0 * a * r / (dl * dl) * e * (1.0 - (1.0 + 2.0 * g) * u + g * u * u);
    return 4.0 * a * u * (1.0 - g * u) * e;
}

/* Morse pair potential M(r) = D (exp(-2 a (r-r0)) - 2 exp(-a (r-r0))) and
 * its derivative. */
static double morse_raw(const orc_pot *p, double r, double *dM)
{
    double e = exp(-p->morse_alpha * (r - p->morse_r0));
    if (dM) *dM = -2.0 * p->morse_alpha * p->morse_D * (e * e - e);
    return p->morse_D * (e * e - 2.0 * e);
}

/* Mechanical pair potential V(r). The workloads give Morse with a 5 A cutoff
 * but no truncation rule; we take the shifted-force form
 * V(r) = M(r) - M(rc) - (r - rc) M'(rc) for r < rc (continuous V and V'),
 * or the plain cut M(r) when morse_shift == 0. */
double orc_V(const orc_pot *p, double r, double *dVdr)
{
    if (!p->morse_on || !(r < p->morse_rc)) {
        if (dVdr) *dVdr = 0.0;
        return 0.0;
    }
    double dM, dMc;
    double M = morse_raw(p, r, &dM);
    if (!p->morse_shift) {
        if (dVdr) *dVdr = dM;
        return M;
    }
    double Mc = morse_raw(p, p->morse_rc, &dMc);
    if (dVdr) *dVdr = dM - dMc;
    return M - Mc - (r - p->morse_rc) * dMc;
}

/* J(r), J'(r), V(r), V'(r) of one pair: the analytic forms, or the learned
 * pair potential when one is set (it replaces both the exchange and the
 * mechanical pair term). */
static void pair_terms(const orc_sys *S, double r, double *J, double *dJ, double *V, double *dV)
{
    if (S->mparams) {
        double o[4];
        mlp_eval(&S->mcfg, S->mparams, r, o);
        *J = o[0]; *dJ = o[1]; *V = o[2]; *dV = o[3];
        if (S->pot.ex_shift && r < S->mcfg.ex_rc) {
            /* the shift of orc_J on the learned J = sJ y0 */
            double yc[2], dyc[2];
            const double rc = S->mcfg.ex_rc;
            mlp_raw(&S->mcfg, S->mparams, rc, yc, dyc);
            *J -= S->mcfg.sJ * (yc[0] + (r * r - rc * rc) * dyc[0] / (2.0 * rc));
            *dJ -= S->mcfg.sJ * r * dyc[0] / rc;
        }
        return;
    }
    *J = orc_J(&S->pot, r, dJ);
    *V = orc_V(&S->pot, r, dV);
}

/* Minimum-image displacement d = r_i - r_j in an orthorhombic periodic box. */
static void min_image(const double L[3], const double *ri, const double *rj,
                      double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double x = ri[a] - rj[a];
        d[a] = x - L[a] * nearbyint(x / L[a]);
    }
}

static double norm3(const double d[3])
{
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ------------------------------------------------------------------------
 * Single-spin propagator (Sec. 3, Omelyan's closed-form rotation):
 * s' = [s + h W x s + (h^2/4)(2 W (W.s) - |W|^2 s)] / (1 + h^2 |W|^2 / 4).
 * ---------------------------------------------------------------------- */
void orc_cayley(const double s[3], const double W[3], double h, double out[3])
{
    double wxs[3];
    cross3(W, s, wxs);
    double ws = dot3(W, s);
    double w2 = dot3(W, W);
    double den = 1.0 + h * h * w2 / 4.0;
    for (int a = 0; a < 3; ++a)
        out[a] = (s[a] + h * wxs[a] + h * h / 4.0 * (2.0 * W[a] * ws - w2 * s[a])) / den;
}

/* ------------------------------------------------------------------------
 * Counter-based random numbers: Philox4x32 with 10 rounds (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 * A round multiplies counter words 0 and 2 by two fixed odd constants,
 * takes 32x32->64 products, and mixes the high halves with the other two
 * counter words and the round key; the key is bumped by two Weyl constants
 * between rounds.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normals for one spin update. Counter = (atom id, step low,
 * step high, replica<<2 | sub-update), key = (seed low, seed high). Uniforms
 * u = (x + 1/2) 2^-32 in (0,1); Box-Muller on (u0,u1) gives two normals and
 * on (u2,u3) one more. */
void orc_gauss3(uint64_t seed, uint32_t atom_id, int64_t step,
                uint32_t replica, int sub, double out[3])
{
    uint32_t ctr[4] = {atom_id, (uint32_t)((uint64_t)step & 0xffffffffu),
                       (uint32_t)((uint64_t)step >> 32),
                       (replica << 2) | (uint32_t)(sub & 3)};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const double two32inv = 1.0 / 4294967296.0;
    const double twopi = 6.283185307179586;
    double u0 = ((double)x[0] + 0.5) * two32inv;
    double u1 = ((double)x[1] + 0.5) * two32inv;
    double u2 = ((double)x[2] + 0.5) * two32inv;
    double u3 = ((double)x[3] + 0.5) * two32inv;
    double ra = sqrt(-2.0 * log(u0));
    double rb = sqrt(-2.0 * log(u2));
    out[0] = ra * cos(twopi * u1);
    out[1] = ra * sin(twopi * u1);
    out[2] = rb * cos(twopi * u3);
}

/* ------------------------------------------------------------------------
 * Lifecycle and state.
 * ---------------------------------------------------------------------- */
orc_sys *orc_create(int N, const double L[3], int frozen, double skin,
                    uint64_t seed, uint32_t replica)
{
    if (N < 0) return NULL;
    orc_sys *S = (orc_sys *)calloc(1, sizeof(orc_sys));
    S->N = N;
    for (int a = 0; a < 3; ++a) S->L[a] = L[a];
    S->frozen = frozen;
    S->skin = frozen ? 0.0 : skin;
    S->seed = seed;
    S->replica = replica;
    S->ordering = ORC_COLOUR;
    S->sect[0] = S->sect[1] = S->sect[2] = 1;
    size_t n3 = (size_t)(N > 0 ? N : 1) * 3;
    S->r = (double *)calloc(n3, sizeof(double));
    S->v = (double *)calloc(n3, sizeof(double));
    S->s = (double *)calloc(n3, sizeof(double));
    S->F = (double *)calloc(n3, sizeof(double));
    S->rbuild = (double *)calloc(n3, sizeof(double));
    S->w_tmp = (double *)calloc(n3, sizeof(double));
    S->rho = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    S->m = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    S->off = (int *)calloc((size_t)N + 1, sizeof(int));
    S->nspin = (int *)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
    S->colour = (int *)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
    S->cls = (int *)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
    S->cls_off = (int *)calloc((size_t)N + 2 + MAXC, sizeof(int));
    S->cap = 0;
    S->idx = NULL;
    return S;
}

void orc_set_mlp(orc_sys *S, const mlp_cfg *c, const double *params)
{
    free(S->mparams);
    S->mparams = NULL;
    if (params) {
        int n = mlp_nparam();
        S->mparams = (double *)malloc((size_t)n * sizeof(double));
        memcpy(S->mparams, params, (size_t)n * sizeof(double));
        S->mcfg = *c;
    }
    S->have_F = 0;
}

void orc_destroy(orc_sys *S)
{
    if (!S) return;
    free(S->mparams);
    free(S->r); free(S->v); free(S->s); free(S->F); free(S->rbuild); free(S->rho);
    free(S->w_tmp); free(S->m); free(S->off); free(S->idx); free(S->nspin);
    free(S->colour); free(S->cls); free(S->cls_off);
    free(S);
}

int orc_set_state(orc_sys *S, const double *r, const double *v,
                  const double *s, const double *mass)
{
    size_t n3 = (size_t)S->N * 3;
    if (r) memcpy(S->r, r, n3 * sizeof(double));
    if (v) memcpy(S->v, v, n3 * sizeof(double));
    if (s) memcpy(S->s, s, n3 * sizeof(double));
    if (mass) memcpy(S->m, mass, (size_t)S->N * sizeof(double));
    S->have_F = 0;
    S->have_D = 0;
    if (!S->user_list) S->have_list = 0;
    S->have_colour = 0;
    return 0;
}

void orc_get_state(const orc_sys *S, double *r, double *v, double *s)
{
    size_t n3 = (size_t)S->N * 3;
    if (r) memcpy(r, S->r, n3 * sizeof(double));
    if (v) memcpy(v, S->v, n3 * sizeof(double));
    if (s) memcpy(s, S->s, n3 * sizeof(double));
}

/* New interactions may change the cutoffs: the Verlet list (unless given by
 * the user) is rebuilt at the next use and the predictor is dropped; the
 * colouring is kept and repaired at that rebuild. */
void orc_set_potential(orc_sys *S, const orc_pot *p)
{
    S->pot = *p;
    S->have_F = 0;
    if (!S->user_list) S->have_list = 0;
    S->have_D = 0;
}

void orc_set_ordering(orc_sys *S, int ordering, const int sect_grid[3])
{
    S->ordering = ordering;
    if (sect_grid)
        for (int a = 0; a < 3; ++a) S->sect[a] = sect_grid[a] > 0 ? sect_grid[a] : 1;
}

void orc_set_step_counter(orc_sys *S, int64_t step) { S->step = step; }
int64_t orc_get_step_counter(const orc_sys *S) { return S->step; }
int orc_num_rebuilds(const orc_sys *S) { return S->nrebuild; }

/* ------------------------------------------------------------------------
 * Neighbour list. Rows hold every j != i closer than the list radius under
 * the minimum image; entries closer than the spin radius come first
 * (nspin[i] of them). The spin radius is the exchange cutoff plus the skin;
 * the list radius adds the skin to the largest cutoff in use.
 * ---------------------------------------------------------------------- */
static double spin_radius(const orc_sys *S) { return S->pot.ex_rc + S->skin; }

static double list_radius(const orc_sys *S)
{
    double rc = S->pot.ex_rc;
    if (!S->frozen && S->pot.morse_on && S->pot.morse_rc > rc) rc = S->pot.morse_rc;
    if (!S->frozen && S->pot.eam_on) {
        if (S->pot.eam_d > rc) rc = S->pot.eam_d;
        if (S->pot.eam_c > rc) rc = S->pot.eam_c;
    }
    return rc + S->skin;
}

/* Two spins conflict (may not share a colour) when their distance at
 * colouring time is below the exchange cutoff plus a third of the skin. A
 * same-colour pair farther apart is watched instead: the list is rebuilt
 * before it can come within the exchange cutoff (see orc_step). With a user
 * list there is no rebuild, so every spin-segment entry conflicts. */
static double colour_radius(const orc_sys *S) { return S->pot.ex_rc + S->skin / 3.0; }

static int conflict(const orc_sys *S, int i, int j)
{
    if (S->user_list) return 1;
    double d[3];
    min_image(S->L, S->r + 3 * i, S->r + 3 * j, d);
    double rc = colour_radius(S);
    return dot3(d, d) < rc * rc;
}

static void ensure_cap(orc_sys *S, long need)
{
    if (need <= S->cap) return;
    long c = S->cap ? S->cap : 1024;
    while (c < need) c *= 2;
    S->idx = (int *)realloc(S->idx, (size_t)c * sizeof(int));
    S->cap = c;
}

/* Candidates of atom i: all j with a minimum-image distance below rl.
 * Uses a linked-cell search when every side holds at least three cells,
 * otherwise all pairs. */
typedef struct {
    int nc[3];
    int *head, *next;
} cells_t;

static void cells_build(const orc_sys *S, double rl, cells_t *C)
{
    C->head = NULL;
    C->next = NULL;
    for (int a = 0; a < 3; ++a) {
        C->nc[a] = (int)floor(S->L[a] / rl);
        if (C->nc[a] < 3) { C->nc[0] = 0; return; }
    }
    int ncell = C->nc[0] * C->nc[1] * C->nc[2];
    C->head = (int *)malloc((size_t)ncell * sizeof(int));
    C->next = (int *)malloc((size_t)(S->N > 0 ? S->N : 1) * sizeof(int));
    for (int c = 0; c < ncell; ++c) C->head[c] = -1;
    for (int i = S->N - 1; i >= 0; --i) {
        int ci[3];
        for (int a = 0; a < 3; ++a) {
            double x = S->r[3 * i + a] - S->L[a] * floor(S->r[3 * i + a] / S->L[a]);
            int k = (int)(x / S->L[a] * C->nc[a]);
            if (k >= C->nc[a]) k = C->nc[a] - 1;
            if (k < 0) k = 0;
            ci[a] = k;
        }
        int c = (ci[2] * C->nc[1] + ci[1]) * C->nc[0] + ci[0];
        C->next[i] = C->head[c];
        C->head[c] = i;
    }
}

static int cell_of(const orc_sys *S, const cells_t *C, int i, int ci[3])
{
    for (int a = 0; a < 3; ++a) {
        double x = S->r[3 * i + a] - S->L[a] * floor(S->r[3 * i + a] / S->L[a]);
        int k = (int)(x / S->L[a] * C->nc[a]);
        if (k >= C->nc[a]) k = C->nc[a] - 1;
        if (k < 0) k = 0;
        ci[a] = k;
    }
    return 0;
}

static int build_list(orc_sys *S)
{
    int N = S->N;
    double rs = spin_radius(S), rl = list_radius(S);
    if (rs > rl) rl = rs;
    cells_t C;
    cells_build(S, rl, &C);
    int *tmp_s = (int *)malloc(4096 * sizeof(int));
    int *tmp_f = (int *)malloc(4096 * sizeof(int));
    long pos = 0;
    S->off[0] = 0;
    for (int i = 0; i < N; ++i) {
        int ns = 0, nf = 0;
        const double *ri = S->r + 3 * i;
        if (C.nc[0] > 0) {
            int ci[3];
            cell_of(S, &C, i, ci);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int cx = (ci[0] + dx + C.nc[0]) % C.nc[0];
                        int cy = (ci[1] + dy + C.nc[1]) % C.nc[1];
                        int cz = (ci[2] + dz + C.nc[2]) % C.nc[2];
                        for (int j = C.head[(cz * C.nc[1] + cy) * C.nc[0] + cx];
                             j >= 0; j = C.next[j]) {
                            if (j == i) continue;
                            double d[3];
                            min_image(S->L, ri, S->r + 3 * j, d);
                            double r = norm3(d);
                            if (r < rs) tmp_s[ns++] = j;
                            else if (r < rl) tmp_f[nf++] = j;
                            if (ns >= 4096 || nf >= 4096) goto overflow;
                        }
                    }
        } else {
            for (int j = 0; j < N; ++j) {
                if (j == i) continue;
                double d[3];
                min_image(S->L, ri, S->r + 3 * j, d);
                double r = norm3(d);
                if (r < rs) tmp_s[ns++] = j;
                else if (r < rl) tmp_f[nf++] = j;
                if (ns >= 4096 || nf >= 4096) goto overflow;
            }
        }
        ensure_cap(S, pos + ns + nf);
        memcpy(S->idx + pos, tmp_s, (size_t)ns * sizeof(int));
        memcpy(S->idx + pos + ns, tmp_f, (size_t)nf * sizeof(int));
        S->nspin[i] = ns;
        pos += ns + nf;
        S->off[i + 1] = (int)pos;
    }
    free(tmp_s); free(tmp_f);
    free(C.head); free(C.next);
    memcpy(S->rbuild, S->r, (size_t)N * 3 * sizeof(double));
    S->have_list = 1;
    return 0;
overflow:
    free(tmp_s); free(tmp_f);
    free(C.head); free(C.next);
    return -4;
}

int orc_set_neighbor_list(orc_sys *S, const int *offsets, const int *idx)
{
    int N = S->N;
    double rs = spin_radius(S);
    long tot = offsets[N];
    ensure_cap(S, tot > 0 ? tot : 1);
    /* stable partition of each row: spin-radius entries first */
    for (int i = 0; i < N; ++i) {
        int a = offsets[i], b = offsets[i + 1], w = a;
        for (int k = a; k < b; ++k) {
            double d[3];
            min_image(S->L, S->r + 3 * i, S->r + 3 * idx[k], d);
            if (norm3(d) < rs) S->idx[w++] = idx[k];
        }
        S->nspin[i] = w - a;
        for (int k = a; k < b; ++k) {
            double d[3];
            min_image(S->L, S->r + 3 * i, S->r + 3 * idx[k], d);
            if (!(norm3(d) < rs)) S->idx[w++] = idx[k];
        }
        S->off[i] = a;
    }
    S->off[N] = (int)tot;
    memcpy(S->rbuild, S->r, (size_t)N * 3 * sizeof(double));
    S->have_list = 1;
    S->user_list = 1;
    return 0;
}

long orc_get_neighbor_list(orc_sys *S, int *nspin, int *nall, int *idx, long cap)
{
    long tot = S->off[S->N];
    if (nspin) memcpy(nspin, S->nspin, (size_t)S->N * sizeof(int));
    if (nall)
        for (int i = 0; i < S->N; ++i) nall[i] = S->off[i + 1] - S->off[i];
    if (idx && cap >= tot) memcpy(idx, S->idx, (size_t)tot * sizeof(int));
    return tot;
}

long orc_brute_pairs(int N, const double L[3], const double *r, double rcut,
                     int *pi, int *pj, long cap)
{
    long n = 0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            if (i == j) continue;
            double d[3];
            min_image(L, r + 3 * i, r + 3 * j, d);
            if (norm3(d) < rcut) {
                if (n < cap) { pi[n] = i; pj[n] = j; }
                ++n;
            }
        }
    return n;
}

/* ------------------------------------------------------------------------
 * Colour classes. The paper makes sectors -- groups of spins that do not
 * interact -- and updates each group in turn (Sec. 5.1, Eq.
 * spin_ST_sectoring). Here a group is a colour class of the spin graph
 * (edges: spin-segment entries closer than the colour radius at colouring
 * time, see conflict()). The colouring is
 * first-fit greedy in ascending lexicographic key (z, y, x) of the wrapped
 * position at colouring time, ties broken by atom id. At later rebuilds a
 * colouring is kept where valid: for every edge whose ends share a colour,
 * the end with the later key is uncoloured; so is every atom whose colour
 * lies outside the palette of the last full colouring (an atom moved there
 * by an earlier repair goes back as soon as its conflict is gone). The
 * uncoloured atoms are recoloured first-fit in ascending key order. More
 * than 32 colours triggers a full recolouring.
 * ---------------------------------------------------------------------- */
typedef struct { double z, y, x; int id; } key_t_;

static int key_cmp(const void *pa, const void *pb)
{
    const key_t_ *a = (const key_t_ *)pa, *b = (const key_t_ *)pb;
    if (a->z != b->z) return a->z < b->z ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

static void make_keys(const orc_sys *S, key_t_ *k)
{
    for (int i = 0; i < S->N; ++i) {
        double w[3];
        for (int a = 0; a < 3; ++a)
            w[a] = S->r[3 * i + a] - S->L[a] * floor(S->r[3 * i + a] / S->L[a]);
        k[i].x = w[0]; k[i].y = w[1]; k[i].z = w[2]; k[i].id = i;
    }
}

static int first_free(const orc_sys *S, int i)
{
    int used[MAXC];
    memset(used, 0, sizeof(used));
    for (int k = S->off[i]; k < S->off[i] + S->nspin[i]; ++k) {
        if (!conflict(S, i, S->idx[k])) continue;
        int c = S->colour[S->idx[k]];
        if (c >= 0 && c < MAXC) used[c] = 1;
    }
    int c = 0;
    while (c < MAXC && used[c]) ++c;
    return c;
}

static void colour_greedy(orc_sys *S, const key_t_ *sorted)
{
    for (int i = 0; i < S->N; ++i) S->colour[i] = -1;
    int K = 0;
    for (int t = 0; t < S->N; ++t) {
        int i = sorted[t].id;
        S->colour[i] = first_free(S, i);
        if (S->colour[i] + 1 > K) K = S->colour[i] + 1;
    }
    S->kbase = K;
}

static void colour_update(orc_sys *S)
{
    int N = S->N;
    key_t_ *keys = (key_t_ *)malloc((size_t)(N > 0 ? N : 1) * sizeof(key_t_));
    key_t_ *sorted = (key_t_ *)malloc((size_t)(N > 0 ? N : 1) * sizeof(key_t_));
    make_keys(S, keys);
    memcpy(sorted, keys, (size_t)N * sizeof(key_t_));
    qsort(sorted, (size_t)N, sizeof(key_t_), key_cmp);
    if (!S->have_colour) {
        colour_greedy(S, sorted);
    } else {
        int *drop = (int *)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
        for (int i = 0; i < N; ++i) {
            if (S->colour[i] >= S->kbase) drop[i] = 1;
            for (int k = S->off[i]; k < S->off[i] + S->nspin[i]; ++k) {
                int j = S->idx[k];
                if (S->colour[j] == S->colour[i] && key_cmp(&keys[j], &keys[i]) < 0 &&
                    conflict(S, i, j))
                    drop[i] = 1;
            }
        }
        for (int i = 0; i < N; ++i)
            if (drop[i]) S->colour[i] = -1;
        for (int t = 0; t < N; ++t) {
            int i = sorted[t].id;
            if (S->colour[i] < 0) S->colour[i] = first_free(S, i);
        }
        free(drop);
        int K = 0;
        for (int i = 0; i < N; ++i) if (S->colour[i] + 1 > K) K = S->colour[i] + 1;
        if (K > 32) colour_greedy(S, sorted);
    }
    int K = 0;
    for (int i = 0; i < N; ++i) if (S->colour[i] + 1 > K) K = S->colour[i] + 1;
    S->K = K;
    S->have_colour = 1;
    free(keys); free(sorted);
}

int orc_set_coloring(orc_sys *S, const int *colour)
{
    int K = 0;
    for (int i = 0; i < S->N; ++i) {
        if (colour[i] < 0 || colour[i] >= MAXC) return -1;
        if (colour[i] + 1 > K) K = colour[i] + 1;
    }
    memcpy(S->colour, colour, (size_t)S->N * sizeof(int));
    S->K = K;
    S->kbase = K;
    S->have_colour = 1;
    return 0;
}

int orc_get_coloring(const orc_sys *S, int *colour)
{
    if (colour) memcpy(colour, S->colour, (size_t)S->N * sizeof(int));
    return S->have_colour ? S->K : 0;
}

static int rebuild(orc_sys *S)
{
    int rc = build_list(S);
    if (rc) return rc;
    if (S->ordering == ORC_COLOUR) colour_update(S);
    S->nrebuild++;
    return 0;
}

int orc_build_now(orc_sys *S)
{
    if (S->user_list) {
        if (S->ordering == ORC_COLOUR && !S->have_colour) colour_update(S);
        return 0;
    }
    return rebuild(S);
}

/* ------------------------------------------------------------------------
 * Precession vector and forces.
 * omega_i = -(1/hbar) dH/ds_i (Sec. 2) for
 *   H = -sum_{i<j} J(r_ij) s_i.s_j - sum_i g mu_B B.s_i - sum_i K (s_i.n)^2
 * i.e. omega_i = (1/hbar)[sum_j J(r_ij) s_j + g mu_B B + 2 K (s_i.n) n].
 * Each unordered pair enters the energy once (the paper writes ordered-pair
 * sums but its force equation has no factor two).
 * ---------------------------------------------------------------------- */
/* Spin-orbit pair terms of one pair (appendix A), with d = r_i - r_j:
 *   Neel:  E = -g1(r) [(e.s_i)(e.s_j) - s_i.s_j/3]   (any sign of e)
 *   DMI:   E = D_ij . (s_i x s_j),  D_ij = dm(r) (n x e_ij), e_ij = -d/r.
 * Each unordered pair counts once (as the exchange, G4 reading). soc_field
 * adds -dE/ds_i (the pair's share of hbar omega_i), soc_force adds -dE/dr_i,
 * soc_pair_energy returns (E_Neel, E_DMI). */
static void soc_radial(const orc_pot *p, double r, double *g1, double *dg1, double *dm, double *ddm)
{
    *g1 = bethe_slater(p->neel_alpha, p->neel_gamma, p->neel_delta, p->neel_rc, r, dg1);
    *dm = bethe_slater(p->dmi_alpha, p->dmi_gamma, p->dmi_delta, p->dmi_rc, r, ddm);
}

static void soc_field(const orc_pot *p, const double d[3], const double *sj, double acc[3])
{
    double r = norm3(d), g1, dg1, dm, ddm;
    soc_radial(p, r, &g1, &dg1, &dm, &ddm);
    double e[3] = {-d[0] / r, -d[1] / r, -d[2] / r};
    double es = dot3(e, sj);
    double D[3], Dxs[3];
    cross3(p->dmi_n, e, D);
    for (int a = 0; a < 3; ++a) D[a] *= dm;
    cross3(D, sj, Dxs);            /* -d/ds_i [D.(s_i x s_j)] = D x s_j */
    for (int a = 0; a < 3; ++a)
        acc[a] += g1 * (es * e[a] - sj[a] / 3.0) + Dxs[a];
}

static void soc_force(const orc_pot *p, const double d[3], const double *si, const double *sj,
                      double f[3])
{
    double r = norm3(d), g1, dg1, dm, ddm;
    soc_radial(p, r, &g1, &dg1, &dm, &ddm);
    double a = dot3(si, d), b = dot3(sj, d), c = dot3(si, sj), r2 = r * r;
    /* Neel: E = -g1 (a b / r^2 - c/3) */
    for (int k = 0; k < 3; ++k)
        f[k] += dg1 * (d[k] / r) * (a * b / r2 - c / 3.0) +
                g1 * ((si[k] * b + sj[k] * a) / r2 - 2.0 * a * b * d[k] / (r2 * r2));
    /* DMI: E = -(dm/r) d.Y with Y = (s_i x s_j) x n */
    double X[3], Y[3];
    cross3(si, sj, X);
    cross3(X, p->dmi_n, Y);
    double dY = dot3(d, Y);
    for (int k = 0; k < 3; ++k)
        f[k] += (ddm / r - dm / r2) * dY * d[k] / r + dm / r * Y[k];
}

static void soc_pair_energy(const orc_pot *p, const double d[3], const double *si,
                            const double *sj, double *en, double *ed)
{
    double r = norm3(d), g1, dg1, dm, ddm;
    soc_radial(p, r, &g1, &dg1, &dm, &ddm);
    double e[3] = {-d[0] / r, -d[1] / r, -d[2] / r};
    *en = -g1 * (dot3(e, si) * dot3(e, sj) - dot3(si, sj) / 3.0);
    double D[3], X[3];
    cross3(p->dmi_n, e, D);
    cross3(si, sj, X);
    *ed = dm * dot3(D, X);
}

static int soc_on(const orc_pot *p)
{
    return p->neel_alpha != 0.0 || p->dmi_alpha != 0.0;
}

static void omega_i(const orc_sys *S, int i, double w[3])
{
    const orc_pot *p = &S->pot;
    double acc[3] = {0.0, 0.0, 0.0};
    const int soc = soc_on(p);
    for (int k = S->off[i]; k < S->off[i] + S->nspin[i]; ++k) {
        int j = S->idx[k];
        double d[3];
        min_image(S->L, S->r + 3 * i, S->r + 3 * j, d);
        double r = norm3(d);
        double J, dJ, V, dV;
        pair_terms(S, r, &J, &dJ, &V, &dV);
        for (int a = 0; a < 3; ++a) acc[a] += J * S->s[3 * j + a];
        if (soc) soc_field(p, d, S->s + 3 * j, acc);
    }
    const double *si = S->s + 3 * i;
    double sn = dot3(si, p->aniso_n);
    for (int a = 0; a < 3; ++a)
        w[a] = (acc[a] + p->zeeman_g * ORC_MUB * p->B[a] +
                2.0 * p->aniso_K * sn * p->aniso_n[a]) / ORC_HBAR;
}

void orc_omega_all(orc_sys *S, double *w)
{
    if (!S->have_list) orc_build_now(S);
    for (int i = 0; i < S->N; ++i) omega_i(S, i, w + 3 * i);
}

/* Force on atom i (Eq. p_advance): F_i = sum_j [-V'(r) + J'(r) s_i.s_j] e_ij
 * with e_ij = (r_i - r_j)/r_ij, so that F_i = -dH/dr_i. */
/* Embedded-atom terms of the Finnis-Sinclair form (the paper's mechanical
 * model is an EAM, Sec. 2 and the mechanical-potential appendix; its tables
 * are not available, so an analytic form of the same two-pass structure
 * stands in): the density function f(r), the pair term phi(r), the
 * embedding F(rho) = -A sqrt(rho), each with its derivative. */
static double eam_f(const orc_pot *p, double r, double *df)
{
    if (!(r < p->eam_d)) { *df = 0.0; return 0.0; }
    double x = r - p->eam_d;
    *df = 2.0 * x + 3.0 * p->eam_beta * x * x / p->eam_d;
    return x * x + p->eam_beta * x * x * x / p->eam_d;
}

static double eam_phi(const orc_pot *p, double r, double *dphi)
{
    if (!(r < p->eam_c)) { *dphi = 0.0; return 0.0; }
    double x = r - p->eam_c;
    double q = p->eam_c0 + p->eam_c1 * r + p->eam_c2 * r * r;
    *dphi = 2.0 * x * q + x * x * (p->eam_c1 + 2.0 * p->eam_c2 * r);
    return x * x * q;
}

static double eam_embed(const orc_pot *p, double rho, double *dF)
{
    if (!(rho > 0.0)) { *dF = 0.0; return 0.0; }
    double sq = sqrt(rho);
    *dF = -0.5 * p->eam_A / sq;
    return -p->eam_A * sq;
}

static int eam_active(const orc_sys *S) { return S->pot.eam_on && !S->frozen; }

/* First pass: rho_i over the whole list. */
static void eam_density(orc_sys *S)
{
    for (int i = 0; i < S->N; ++i) {
        double rho = 0.0;
        for (int k = S->off[i]; k < S->off[i + 1]; ++k) {
            double d[3], df;
            min_image(S->L, S->r + 3 * i, S->r + 3 * S->idx[k], d);
            rho += eam_f(&S->pot, norm3(d), &df);
        }
        S->rho[i] = rho;
    }
}

static void forces(orc_sys *S)
{
    const int eam = eam_active(S);
    if (eam) eam_density(S);
    for (int i = 0; i < S->N; ++i) {
        double f[3] = {0.0, 0.0, 0.0};
        for (int k = S->off[i]; k < S->off[i + 1]; ++k) {
            int j = S->idx[k];
            double d[3];
            min_image(S->L, S->r + 3 * i, S->r + 3 * j, d);
            double r = norm3(d);
            double J, dJ, V, dV;
            pair_terms(S, r, &J, &dJ, &V, &dV);
            double c = -dV + dJ * dot3(S->s + 3 * i, S->s + 3 * j);
            if (eam) {
                /* second pass: -[phi'(r) + (F'(rho_i) + F'(rho_j)) f'(r)] */
                double df, dphi, dFi, dFj;
                (void)eam_f(&S->pot, r, &df);
                (void)eam_phi(&S->pot, r, &dphi);
                (void)eam_embed(&S->pot, S->rho[i], &dFi);
                (void)eam_embed(&S->pot, S->rho[j], &dFj);
                c -= dphi + (dFi + dFj) * df;
            }
            for (int a = 0; a < 3; ++a) f[a] += c * d[a] / r;
            if (soc_on(&S->pot) && k < S->off[i] + S->nspin[i])
                soc_force(&S->pot, d, S->s + 3 * i, S->s + 3 * j, f);
        }
        for (int a = 0; a < 3; ++a) S->F[3 * i + a] = f[a];
    }
    S->have_F = 1;
}

void orc_force_all(orc_sys *S, double *F)
{
    if (!S->have_list) orc_build_now(S);
    forces(S);
    memcpy(F, S->F, (size_t)S->N * 3 * sizeof(double));
}

/* ------------------------------------------------------------------------
 * Stochastic spin update (Sec. 4.1, Eq. sLLG):
 * ds/dt = [(omega + eta) x s + lambda s x (omega x s)] / (1 + lambda^2)
 *       = W x s,  W = (omega + eta + lambda s x omega) / (1 + lambda^2).
 * The white noise has <eta_a eta_b> = 2 D_S delta_ab delta(t-t'). We read the
 * fluctuation-dissipation amplitude as D_S = lambda (1 + lambda^2) k_B T /
 * hbar, the value for which exp(-H/k_B T) is stationary for this equation
 * (the printed 2 pi mixes h and hbar). Over one update of length h the noise
 * is held constant at eta = sqrt(2 D_S / |h|) xi (mid-point Stratonovich:
 * the Cayley rotation with a fixed eta is the implicit mid-point rule for
 * the eta x s term). omega and the damping term are taken at the spin's
 * value before the update.
 * ---------------------------------------------------------------------- */
static void update_spin(orc_sys *S, int i, double h, int sub, const double w[3])
{
    const orc_pot *p = &S->pot;
    double *si = S->s + 3 * i;
    double W[3];
    if (p->aniso_split && p->aniso_K != 0.0 && !(p->lambda > 0.0)) {
        /* Symmetric split of the single-spin propagator: A(h/2) X(h) A(h/2).
         * A is the flow of the anisotropy alone, ds/dt = (2K/hbar)(s.n) n x s:
         * a rotation about n that keeps s.n, so its rate is fixed by the spin
         * it starts from and A(-h/2) undoes A(h/2) exactly. X rotates about
         * omega without its anisotropy term, which does not depend on s_i.
         * The composition is time-reversible; taking the whole omega at the
         * spin's value before the update is not, and loses exactly
         * K (delta s.n)^2 of energy per update. */
        double sn = dot3(si, p->aniso_n);
        double Wx[3], Wa[3], out[3];
        for (int a = 0; a < 3; ++a)
            Wx[a] = w[a] - 2.0 * p->aniso_K * sn * p->aniso_n[a] / ORC_HBAR;
        for (int a = 0; a < 3; ++a) Wa[a] = 2.0 * p->aniso_K * sn * p->aniso_n[a] / ORC_HBAR;
        orc_cayley(si, Wa, 0.5 * h, out);
        orc_cayley(out, Wx, h, si);
        sn = dot3(si, p->aniso_n);
        for (int a = 0; a < 3; ++a) Wa[a] = 2.0 * p->aniso_K * sn * p->aniso_n[a] / ORC_HBAR;
        orc_cayley(si, Wa, 0.5 * h, out);
        for (int a = 0; a < 3; ++a) si[a] = out[a];
        return;
    }
    if (p->lambda > 0.0) {
        double lam = p->lambda;
        double DS = lam * (1.0 + lam * lam) * ORC_KB * p->temperature / ORC_HBAR;
        double amp = sqrt(2.0 * DS / fabs(h));
        double xi[3];
        orc_gauss3(S->seed, (uint32_t)i, S->step, S->replica, sub, xi);
        double sxw[3];
        cross3(si, w, sxw);
        for (int a = 0; a < 3; ++a)
            W[a] = (w[a] + amp * xi[a] + lam * sxw[a]) / (1.0 + lam * lam);
    } else {
        for (int a = 0; a < 3; ++a) W[a] = w[a];
    }
    double out[3];
    orc_cayley(si, W, h, out);
    for (int a = 0; a < 3; ++a) si[a] = out[a];
}

/* Classes for the sectoring ordering: the box is split into sect[0] x
 * sect[1] x sect[2] processor subdomains, each bisected once per dimension
 * into 8 sectors (Sec. 5.1); class k = sector k on every subdomain, atoms
 * in subdomain order then id order. Assigned from the positions at the
 * start of the step. */
static void sect_classes(orc_sys *S)
{
    int N = S->N;
    int *sec = (int *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int));
    int *prc = (int *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int));
    for (int i = 0; i < N; ++i) {
        int pidx[3], bit[3];
        for (int a = 0; a < 3; ++a) {
            double x = S->r[3 * i + a] - S->L[a] * floor(S->r[3 * i + a] / S->L[a]);
            double f = x / S->L[a] * S->sect[a];
            int pi = (int)floor(f);
            if (pi >= S->sect[a]) pi = S->sect[a] - 1;
            pidx[a] = pi;
            bit[a] = (f - pi) >= 0.5;
        }
        sec[i] = bit[0] + 2 * bit[1] + 4 * bit[2];
        prc[i] = pidx[0] + S->sect[0] * (pidx[1] + S->sect[1] * pidx[2]);
    }
    int np = S->sect[0] * S->sect[1] * S->sect[2];
    int t = 0;
    S->cls_off[0] = 0;
    for (int k = 0; k < 8; ++k) {
        for (int q = 0; q < np; ++q)
            for (int i = 0; i < N; ++i)
                if (sec[i] == k && prc[i] == q) S->cls[t++] = i;
        S->cls_off[k + 1] = t;
    }
    S->ncls = 8;
    free(sec); free(prc);
}

static void colour_classes(orc_sys *S)
{
    int t = 0;
    S->cls_off[0] = 0;
    for (int c = 0; c < S->K; ++c) {
        for (int i = 0; i < S->N; ++i)
            if (S->colour[i] == c) S->cls[t++] = i;
        S->cls_off[c + 1] = t;
    }
    S->ncls = S->K;
}

/* One sweep of dt/4 updates: classes 1..K with atoms in order (forward), or
 * classes K..1 with atoms in reverse order (backward); omega_i is computed
 * right before s_i is rotated (Eqs. spin_ST_decomposition and
 * spin_ST_sectoring). SEQ: one atom per class (the serial decomposition).
 * JACOBI: every spin rotated at once from the old state -- not the paper's
 * method; kept only as a negative control for the independence of classes. */
static void sweep(orc_sys *S, double h, int backward, int sub)
{
    int N = S->N;
    if (S->ordering == ORC_JACOBI) {
        for (int i = 0; i < N; ++i) omega_i(S, i, S->w_tmp + 3 * i);
        for (int i = 0; i < N; ++i) update_spin(S, i, h, sub, S->w_tmp + 3 * i);
        return;
    }
    if (S->ordering == ORC_SEQ) {
        for (int t = 0; t < N; ++t) {
            int i = backward ? N - 1 - t : t;
            double w[3];
            omega_i(S, i, w);
            update_spin(S, i, h, sub, w);
        }
        return;
    }
    int K = S->ncls;
    for (int q = 0; q < K; ++q) {
        int c = backward ? K - 1 - q : q;
        int a = S->cls_off[c], b = S->cls_off[c + 1];
        for (int t = 0; t < b - a; ++t) {
            int i = backward ? S->cls[b - 1 - t] : S->cls[a + t];
            double w[3];
            omega_i(S, i, w);
            update_spin(S, i, h, sub, w);
        }
    }
}

static void prepare_classes(orc_sys *S)
{
    if (S->ordering == ORC_COLOUR) colour_classes(S);
    else if (S->ordering == ORC_SECT) sect_classes(S);
}

/* ------------------------------------------------------------------------
 * One step (Eq. general_ST_decomposition):
 *   exp(L_p dt/2) exp(L_s dt/2) exp(L_r dt) exp(L_s dt/2) exp(L_p dt/2),
 * each exp(L_s dt/2) being a forward then a backward sweep of dt/4 updates,
 * so every spin is rotated four times per step (Sec. 3 and Sec. 5.1); the
 * two dt/4 rotations of the last class are never merged. The frozen
 * lattice keeps only the four sweeps.
 *
 * Verlet rebuild rule (the paper uses the host code's defaults, unstated):
 * at the boundary before step k the list is rebuilt when
 *   D_{k-1} = max_i |r_i - r_i^build| + 2 a max_i |v_i| >= skin/2 - 0.01 A,
 * with the displacement and speed taken at the previous boundary (after that
 * boundary's own rebuild, if any) and a = max(|dt_{k-1}|, |dt_k|), the
 * larger of the two step lengths involved (they differ only when a call
 * changes dt). The extra 2 a max|v| covers the two drifts that can happen
 * before the next decision. It is also rebuilt when
 *   W_{k-1} = min |r_i - r_j| - 4 a max|v| < ex_rc + 0.01 A
 * over same-colour pairs of spin-segment entries at the previous boundary:
 * such a pair must not come within the exchange cutoff before the next
 * decision (each of the two ends moves at most 2 a max|v|). A boundary that
 * rebuilt takes the colour radius for the closest pair (after a colouring
 * no same-colour pair is closer). The classes are frozen for the step.
 * ---------------------------------------------------------------------- */
static double watch_min(const orc_sys *S)
{
    double m = 1e300;
    for (int i = 0; i < S->N; ++i)
        for (int k = S->off[i]; k < S->off[i] + S->nspin[i]; ++k) {
            int j = S->idx[k];
            if (S->colour[j] != S->colour[i]) continue;
            double d[3];
            min_image(S->L, S->r + 3 * i, S->r + 3 * j, d);
            double r = norm3(d);
            if (r < m) m = r;
        }
    return m;
}

static double max_disp(const orc_sys *S)
{
    double m = 0.0;
    for (int i = 0; i < S->N; ++i) {
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = S->r[3 * i + a] - S->rbuild[3 * i + a];
        double x = norm3(d);
        if (x > m) m = x;
    }
    return m;
}

static double max_speed(const orc_sys *S)
{
    double m = 0.0;
    for (int i = 0; i < S->N; ++i) {
        double x = norm3(S->v + 3 * i);
        if (x > m) m = x;
    }
    return m;
}

/* Drift of one step. Without a lattice bath: r += dt v. With the bath of
 * Eq. p_advance_T (friction -gamma_L p/m and a white-noise force whose
 * strength follows from the Einstein relation, D_L = 2 gamma_L k_B T_L),
 * the friction-plus-noise part is an Ornstein-Uhlenbeck process in v that
 * is integrated exactly over |dt| and placed between two half drifts:
 *   r += (dt/2) v;  v = c v + sqrt((1 - c^2) k_B T_L / m) xi;  r += (dt/2) v
 * with c = exp(-gamma_L |dt| / m) and xi three standard normals from the
 * Philox stream keyed by seed XOR ORC_LATTICE_KEY_TAG, counter (atom id,
 * step, replica, 0). k_B T / m in eV/amu becomes (A/ps)^2 through 1/ORC_MVV2E. */
static void drift(orc_sys *S, double dt)
{
    const orc_pot *p = &S->pot;
    if (!(p->lat_gamma > 0.0)) {
        for (int i = 0; i < 3 * S->N; ++i) S->r[i] += dt * S->v[i];
        return;
    }
    const uint64_t key = S->seed ^ ORC_LATTICE_KEY_TAG;
    for (int i = 0; i < S->N; ++i) {
        double *ri = S->r + 3 * i, *vi = S->v + 3 * i;
        const double c = exp(-p->lat_gamma * fabs(dt) / S->m[i]);
        const double sig = sqrt((1.0 - c * c) * ORC_KB * p->lat_temperature / S->m[i] / ORC_MVV2E);
        double xi[3];
        orc_gauss3(key, (uint32_t)i, S->step, S->replica, 0, xi);
        for (int a = 0; a < 3; ++a) {
            ri[a] += 0.5 * dt * vi[a];
            vi[a] = c * vi[a] + sig * xi[a];
            ri[a] += 0.5 * dt * vi[a];
        }
    }
}

int orc_step(orc_sys *S, int64_t n, double dt)
{
    const double ftm2v = 1.0 / ORC_MVV2E;
    double h = dt / 4.0;
    for (int64_t it = 0; it < n; ++it) {
        if (S->frozen) {
            if (!S->have_list) { int rc = orc_build_now(S); if (rc) return rc; }
            if (S->ordering == ORC_COLOUR && !S->have_colour) colour_update(S);
            prepare_classes(S);
            sweep(S, h, 0, 0);
            sweep(S, h, 1, 1);
            sweep(S, h, 0, 2);
            sweep(S, h, 1, 3);
            S->step++;
            continue;
        }
        int rebuilt = 0;
        if (!S->have_list) {
            int rc = orc_build_now(S); if (rc) return rc;
            rebuilt = 1;
        } else if (!S->user_list && S->have_D) {
            const double a = fmax(S->adt_prev, fabs(dt));
            const double D = S->disp_prev + 2.0 * a * S->vmax_prev;
            const double W = S->wmin_prev - 4.0 * a * S->vmax_prev;
            if (D >= S->skin / 2.0 - 0.01 ||
                (S->ordering == ORC_COLOUR && W < S->pot.ex_rc + 0.01)) {
                int rc = rebuild(S); if (rc) return rc;
                rebuilt = 1;
            }
        }
        if (S->ordering == ORC_COLOUR && !S->have_colour) colour_update(S);
        S->vmax_prev = max_speed(S);
        S->disp_prev = max_disp(S);
        S->wmin_prev = S->ordering != ORC_COLOUR ? 1e300
                       : (rebuilt ? colour_radius(S) : watch_min(S));
        S->adt_prev = fabs(dt);
        S->have_D = 1;
        prepare_classes(S);
        if (!S->have_F) forces(S);
        for (int i = 0; i < S->N; ++i)
            for (int a = 0; a < 3; ++a)
                S->v[3 * i + a] += dt / 2.0 * S->F[3 * i + a] / S->m[i] * ftm2v;
        sweep(S, h, 0, 0);
        sweep(S, h, 1, 1);
        drift(S, dt);
        sweep(S, h, 0, 2);
        sweep(S, h, 1, 3);
        forces(S);
        for (int i = 0; i < S->N; ++i)
            for (int a = 0; a < 3; ++a)
                S->v[3 * i + a] += dt / 2.0 * S->F[3 * i + a] / S->m[i] * ftm2v;
        S->step++;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Observables.
 * ---------------------------------------------------------------------- */
void orc_energy(orc_sys *S, double e[6])
{
    if (!S->have_list) orc_build_now(S);
    const orc_pot *p = &S->pot;
    double kin = 0.0, pair = 0.0, ex = 0.0, zee = 0.0, an = 0.0;
    const int eam = eam_active(S);
    if (eam) eam_density(S);
    for (int i = 0; i < S->N; ++i) {
        const double *vi = S->v + 3 * i;
        kin += 0.5 * S->m[i] * dot3(vi, vi) * ORC_MVV2E;
        if (eam) {
            double dF;
            pair += eam_embed(p, S->rho[i], &dF);
        }
        for (int k = S->off[i]; k < S->off[i + 1]; ++k) {
            int j = S->idx[k];
            if (j <= i) continue;     /* each unordered pair once */
            double d[3];
            min_image(S->L, S->r + 3 * i, S->r + 3 * j, d);
            double r = norm3(d);
            double J, dJ, V, dV;
            pair_terms(S, r, &J, &dJ, &V, &dV);
            if (!S->frozen) pair += V;
            if (eam) {
                double dphi;
                pair += eam_phi(p, r, &dphi);
            }
            ex -= J * dot3(S->s + 3 * i, S->s + 3 * j);
            if (soc_on(p) && k < S->off[i] + S->nspin[i]) {
                double en, ed;
                soc_pair_energy(p, d, S->s + 3 * i, S->s + 3 * j, &en, &ed);
                ex += en + ed;
            }
        }
        const double *si = S->s + 3 * i;
        zee -= p->zeeman_g * ORC_MUB * dot3(p->B, si);
        double sn = dot3(si, p->aniso_n);
        an -= p->aniso_K * sn * sn;
    }
    e[0] = kin; e[1] = pair; e[2] = ex; e[3] = zee; e[4] = an;
    e[5] = kin + pair + ex + zee + an;
}

void orc_soc_energy(orc_sys *S, double *neel, double *dmi)
{
    if (!S->have_list) orc_build_now(S);
    double a = 0.0, b = 0.0;
    for (int i = 0; i < S->N; ++i)
        for (int k = S->off[i]; k < S->off[i] + S->nspin[i]; ++k) {
            int j = S->idx[k];
            if (j <= i) continue;
            double d[3], en, ed;
            min_image(S->L, S->r + 3 * i, S->r + 3 * j, d);
            soc_pair_energy(&S->pot, d, S->s + 3 * i, S->s + 3 * j, &en, &ed);
            a += en;
            b += ed;
        }
    *neel = a;
    *dmi = b;
}

void orc_magnetization(const orc_sys *S, double M[3])
{
    M[0] = M[1] = M[2] = 0.0;
    for (int i = 0; i < S->N; ++i)
        for (int a = 0; a < 3; ++a) M[a] += S->s[3 * i + a];
}

/* Lattice temperature (Eq. lattice_temperature) and the spin temperature of
 * Nurdin et al. (Eq. spin_temperature):
 * T_S = (hbar / 2 k_B) sum |s x omega|^2 / sum s.omega. */
void orc_temperatures(orc_sys *S, double *T_lattice, double *T_spin)
{
    double kin = 0.0;
    for (int i = 0; i < S->N; ++i)
        kin += 0.5 * S->m[i] * dot3(S->v + 3 * i, S->v + 3 * i) * ORC_MVV2E;
    if (T_lattice) *T_lattice = S->N > 0 ? 2.0 * kin / (3.0 * S->N * ORC_KB) : 0.0;
    if (T_spin) {
        if (!S->have_list) orc_build_now(S);
        double num = 0.0, den = 0.0;
        for (int i = 0; i < S->N; ++i) {
            double w[3], c[3];
            omega_i(S, i, w);
            cross3(S->s + 3 * i, w, c);
            num += dot3(c, c);
            den += dot3(S->s + 3 * i, w);
        }
        *T_spin = ORC_HBAR / (2.0 * ORC_KB) * num / den;
    }
}
