/*
 * oracle.h -- plain serial FP64 CPU reference of the coupled spin-lattice
 * Suzuki-Trotter step (Tranchida, Plimpton, Thibaudeau, Thompson 2018).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or
 * call this library; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do. It shares no code with the HIP library.
 *
 * State is kept in user atom order, arrays are AoS double[N][3].
 * Units: A, ps, eV, amu, K, T; spins are unit vectors.
 */
#ifndef SPINLAT_ORACLE_H
#define SPINLAT_ORACLE_H

#include <stdint.h>

#include "mlp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Physical constants (CODATA 2018). */
#define ORC_HBAR  6.582119569e-4     /* eV ps            */
#define ORC_KB    8.617333262e-5     /* eV / K           */
#define ORC_MUB   5.7883818060e-5    /* eV / T           */
#define ORC_MVV2E 1.0364269652680506e-4  /* eV per amu A^2/ps^2 */

typedef struct {
    int morse_on;
    double morse_D, morse_alpha, morse_r0, morse_rc;
    int morse_shift;             /* 1: shifted-force truncation, 0: plain cut */
    double ex_alpha, ex_gamma, ex_delta, ex_rc;   /* Bethe-Slater J(r) */
    double zeeman_g;
    double B[3];                 /* tesla */
    double aniso_K;              /* eV */
    double aniso_n[3];           /* unit axis */
    double lambda;               /* transverse spin damping */
    double temperature;          /* spin bath temperature, K */
    double lat_gamma;            /* lattice friction gamma_L, amu/ps (0: no bath) */
    double lat_temperature;      /* lattice bath temperature, K */
    /* Neel pseudo-dipolar pair anisotropy, g1(r) of Bethe-Slater form */
    double neel_alpha, neel_gamma, neel_delta, neel_rc;
    /* Dzyaloshinskii-Moriya pair term, D_ij = d(r) (dmi_n x e_ij) with d(r)
     * of Bethe-Slater form and e_ij = (r_j - r_i)/r_ij */
    double dmi_alpha, dmi_gamma, dmi_delta, dmi_rc;
    double dmi_n[3];
    /* embedded-atom mechanical potential of the Finnis-Sinclair form:
     * E = sum_i F(rho_i) + sum_{i<j} phi(r_ij), rho_i = sum_j f(r_ij),
     * F(rho) = -A sqrt(rho), f(r) = (r-d)^2 + beta (r-d)^3/d (r < d),
     * phi(r) = (r-c)^2 (c0 + c1 r + c2 r^2) (r < c) */
    int eam_on;
    double eam_A, eam_d, eam_beta, eam_c, eam_c0, eam_c1, eam_c2;
    /* optional readings where the paper's literal form breaks exact energy
     * conservation (both off by default):
     * ex_shift = 1: J(r) shifted in r^2,
     *   J(r) - J(rc) - (r^2 - rc^2) J'(rc)/(2 rc) for r < rc, so J and J'
     *   are continuous at the cutoff (the learned J likewise);
     * aniso_split = 1: without a spin bath, each single-spin update splits
     *   the uniaxial anisotropy off symmetrically, A(h/2) X(h) A(h/2), A the
     *   rotation about n of the anisotropy flow (s.n conserved) and X the
     *   rotation about the rest of omega (which does not depend on s_i). */
    int ex_shift;
    int aniso_split;
} orc_pot;

/* Key tag of the lattice-noise Philox stream: key = seed XOR this value. */
#define ORC_LATTICE_KEY_TAG 0x6C61747469636521ull

enum { ORC_COLOUR = 0, ORC_SEQ = 1, ORC_SECT = 2, ORC_JACOBI = 3 };

typedef struct orc_sys orc_sys;

/* Lifecycle. skin = Verlet skin (A); frozen = 1 keeps positions fixed. */
orc_sys *orc_create(int N, const double L[3], int frozen, double skin,
                    uint64_t seed, uint32_t replica);
void orc_destroy(orc_sys *S);

int  orc_set_state(orc_sys *S, const double *r, const double *v,
                   const double *s, const double *mass);
void orc_get_state(const orc_sys *S, double *r, double *v, double *s);
void orc_set_potential(orc_sys *S, const orc_pot *p);
void orc_set_ordering(orc_sys *S, int ordering, const int sect_grid[3]);
void orc_set_step_counter(orc_sys *S, int64_t step);
int64_t orc_get_step_counter(const orc_sys *S);

/* User CSR list (offsets[N+1], idx): spin entries must be first in each row
 * and are identified by distance at use time; disables rebuilds. */
int orc_set_neighbor_list(orc_sys *S, const int *offsets, const int *idx);
/* Current list: counts per atom (spin, total) and rows; returns total size,
 * or the needed size when cap is too small. */
long orc_get_neighbor_list(orc_sys *S, int *nspin, int *nall, int *idx,
                           long cap);
int orc_build_now(orc_sys *S);      /* forced (re)build at the current state */
int orc_set_coloring(orc_sys *S, const int *colour);
int orc_get_coloring(const orc_sys *S, int *colour);   /* returns K */
int orc_num_rebuilds(const orc_sys *S);

int orc_step(orc_sys *S, int64_t n, double dt);

/* Observables of the current state. e = {kin, pair, exchange, zeeman, aniso,
 * total} in eV; M = sum_i s_i. */
void orc_energy(orc_sys *S, double e[6]);
/* The Neel and DMI parts of the magnetic pair energy (both are included in
 * e[2] of orc_energy). */
void orc_soc_energy(orc_sys *S, double *neel, double *dmi);
void orc_magnetization(const orc_sys *S, double M[3]);
void orc_temperatures(orc_sys *S, double *T_lattice, double *T_spin);
void orc_omega_all(orc_sys *S, double *w);     /* conservative omega, rad/ps */
void orc_force_all(orc_sys *S, double *F);     /* eV/A */

/* Pure functions. */
double orc_J(const orc_pot *p, double r, double *dJdr);
double orc_V(const orc_pot *p, double r, double *dVdr);
void orc_cayley(const double s[3], const double W[3], double h, double out[3]);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
void orc_gauss3(uint64_t seed, uint32_t atom_id, int64_t step,
                uint32_t replica, int sub, double out[3]);

/* Use the FP64 learned pair potential for J and V (params NULL: analytic). */
void orc_set_mlp(orc_sys *S, const mlp_cfg *c, const double *params);

/* Brute-force O(N^2) neighbour sets for pinning the cell-list build. */
long orc_brute_pairs(int N, const double L[3], const double *r, double rcut,
                     int *pi, int *pj, long cap);

#ifdef __cplusplus
}
#endif
#endif
