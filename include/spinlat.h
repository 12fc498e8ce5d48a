/*
 * spinlat.h -- C ABI of the MI355X (gfx950) spin-lattice library.
 *
 * One call of sl_step advances a periodic system of N atoms, each carrying
 * a position r_i, a velocity v_i and a unit spin s_i, with the symplectic
 * Suzuki-Trotter splitting of Tranchida, Plimpton, Thibaudeau and Thompson
 * (J. Comput. Phys. 2018; Sec. 3, Eq. general_ST_decomposition):
 *   half kick, spin half-step, drift, spin half-step, half kick,
 * where each spin half-step is a forward then a backward sweep over
 * classes of non-interacting spins (Sec. 5.1, Eq. spin_ST_sectoring) and
 * each spin update is the closed-form rotation of Sec. 3 about the
 * precession vector omega_i (Sec. 2) gathered right before the update.
 *
 * Conventions shared by every entry point:
 *  - Units: A, ps, eV, amu, K, T. Spins are unit vectors.
 *  - Arrays cross the ABI as AoS double[N][3] (or double[N], int[N]) in the
 *    caller's atom order ("user order"); the library keeps its own
 *    structure-of-arrays copies, reordered by colour class and cell.
 *  - `where` is SL_HOST (host pointer) or SL_DEVICE (device pointer on the
 *    system's stream, e.g. a torch tensor's data_ptr()). Caller memory is
 *    copied in or out during the call and never retained.
 *  - The library owns every device buffer it allocates.
 *  - Every function returns 0 (SL_OK) or a negative SL_E_* code; nothing
 *    throws or aborts across the ABI. sl_last_error() gives the message.
 *  - sl_step is asynchronous on the system's stream except for one host
 *    wait per step on the previous step's completion (the neighbour-list
 *    rebuild decision) and a synchronisation at each rebuild. Errors seen
 *    on the device (list overflow, non-finite values) are sticky and are
 *    returned by the next sl_step or sl_get_* call.
 *  - A handle is not thread-safe; separate handles are independent.
 */
#ifndef SPINLAT_H
#define SPINLAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SL_OK               0
#define SL_E_ARG           -1  /* invalid argument or unnormalised spin     */
#define SL_E_BOX           -2  /* box side below twice the list radius      */
#define SL_E_NONFINITE     -3  /* NaN/Inf in the input or in the trajectory */
#define SL_E_NBR_OVERFLOW  -4  /* more neighbours than max_nbr/max_spin_nbr  */
#define SL_E_COLOR         -5  /* two interacting spins share a colour      */
#define SL_E_HIP           -6  /* HIP runtime error                         */
#define SL_E_STATE         -7  /* call out of order (e.g. step before state) */
#define SL_E_NOMEM         -8  /* device allocation failed                  */

#define SL_HOST   0
#define SL_DEVICE 1

#define SL_FP64   0            /* every quantity in FP64                     */
#define SL_FP32   1            /* spins, omega, forces and rotations in FP32;
                                  positions, velocities and reductions FP64 */

typedef struct sl_system sl_system;

/* Creation parameters. */
typedef struct {
    int64_t n_atoms;       /* N >= 1                                        */
    double box[3];         /* orthorhombic periodic box sides, A            */
    int precision;         /* SL_FP64 or SL_FP32                            */
    int frozen;            /* 1: positions fixed, spin dynamics only        */
    double skin;           /* Verlet skin, A (ignored when frozen)          */
    int max_nbr;           /* list row capacity (0: default 80)             */
    int max_spin_nbr;      /* spin-segment capacity (0: default 32)         */
    uint64_t seed;         /* Philox key of the spin bath                   */
    uint32_t replica;      /* replica index folded into the Philox counter  */
    int thermo_every;      /* record E and M every n steps (0: never)       */
    void *stream;          /* hipStream_t to run on; NULL: own stream       */
} sl_params;

/* Interaction parameters.
 *  - Mechanical pair potential: Morse M(r) = D (e^{-2a(r-r0)} - 2 e^{-a(r-r0)})
 *    for r < morse_rc; morse_shift = 1 uses the shifted-force form
 *    M(r) - M(rc) - (r - rc) M'(rc) so V and V' are continuous at rc.
 *  - Exchange (appendix A.1, Eq. BSfunction): Bethe-Slater
 *    J(r) = 4 ex_alpha u (1 - ex_gamma u) e^{-u}, u = (r/ex_delta)^2, for
 *    r < ex_rc; enters H as -sum_{i<j} J(r_ij) s_i.s_j (each pair once).
 *  - Zeeman (Sec. 2, Eq. s_hamiltonian): -sum_i g mu_B B.s_i.
 *  - Uniaxial anisotropy (appendix A.2): -sum_i K (s_i.n)^2.
 *  - Spin bath (Sec. 4.1, Eq. sLLG): transverse damping lambda and white
 *    noise at temperature T with D_S = lambda (1 + lambda^2) k_B T / hbar.
 *  - Lattice bath (Sec. 4.2, Eq. p_advance_T): friction -lat_gamma p/m
 *    (lat_gamma in amu/ps; 0 = no bath) and white noise at lat_temperature
 *    with D_L = 2 lat_gamma k_B T (Einstein relation). The friction and
 *    noise are integrated exactly over |dt| (an Ornstein-Uhlenbeck step,
 *    v <- c v + sqrt((1 - c^2) k_B T/m) xi, c = exp(-lat_gamma |dt|/m)) in
 *    the middle of each drift: half drift, bath, half drift. The normals
 *    come from Philox4x32-10 keyed by seed XOR 0x6C61747469636521 with
 *    counter (atom id, step low, step high, replica << 2), Box-Muller as
 *    for the spin noise. Ignored on a frozen lattice.
 *  - Spin-orbit pair terms (appendix A), each unordered pair once, with
 *    g1(r) and d(r) of the Bethe-Slater form above (neel_* and dmi_*
 *    parameters, each cut at its own rc, which must not exceed ex_rc: the
 *    exchange cutoff is the radius of every magnetic pair term):
 *      Neel pseudo-dipolar: -sum_{i<j} g1(r) [(e.s_i)(e.s_j) - s_i.s_j/3]
 *      Dzyaloshinskii-Moriya: sum_{i<j} D_ij.(s_i x s_j),
 *        D_ij = d(r) (dmi_n x e_ij), e_ij = (r_j - r_i)/r_ij, |dmi_n| = 1.
 *    Available with the analytic exchange only (not with a learned pair
 *    potential); their field on s_i depends on s_j only, so the colour
 *    sweeps keep their exact properties.
 *  - Embedded-atom mechanical term (Sec. 2; the paper's tabulated EAM is
 *    replaced by the analytic Finnis-Sinclair form), added to the Morse
 *    term when both are on: sum_i F(rho_i) + sum_{i<j} phi(r_ij) with
 *    rho_i = sum_j f(r_ij), F(rho) = -eam_A sqrt(rho),
 *    f(r) = (r - eam_d)^2 + eam_beta (r - eam_d)^3 / eam_d for r < eam_d,
 *    phi(r) = (r - eam_c)^2 (eam_c0 + eam_c1 r + eam_c2 r^2) for r < eam_c.
 *    Forces take two passes (densities, then the gather with
 *    F'(rho_i) + F'(rho_j)); the list radius covers eam_d and eam_c. Its
 *    energy is reported in `pair`. Not with a learned pair potential.
 *  - Optional smooth forms (both 0 by default, the paper's literal form):
 *    ex_shift = 1 shifts the exchange in r^2,
 *    J(r) - J(ex_rc) - (r^2 - ex_rc^2) J'(ex_rc) / (2 ex_rc) for r < ex_rc,
 *    so J and J' are continuous at the cutoff (Eq. BSfunction cuts J with a step, which
 *    changes the energy by J(ex_rc) s_i.s_j at every crossing); a learned J
 *    takes the same rule. aniso_split = 1 applies each single-spin update
 *    without a spin bath as A(h/2) X(h) A(h/2): A rotates about n by the
 *    anisotropy's own flow (s.n is constant under it), X about the rest of
 *    omega_i. Taking the whole omega_i at the spin's value before the update
 *    (the default) loses exactly K (delta s.n)^2 of energy per update; the
 *    split form is time-reversible and keeps the energy without drift.
 *    With the spin bath on, the anisotropy stays in omega_i. */
typedef struct {
    int morse_on;
    double morse_D, morse_alpha, morse_r0, morse_rc;
    int morse_shift;
    double ex_alpha, ex_gamma, ex_delta, ex_rc;
    double zeeman_g;
    double B[3];
    double aniso_K;
    double aniso_n[3];
    double lambda;
    double temperature;
    double lat_gamma;
    double lat_temperature;
    double neel_alpha, neel_gamma, neel_delta, neel_rc;
    double dmi_alpha, dmi_gamma, dmi_delta, dmi_rc;
    double dmi_n[3];
    int eam_on;
    double eam_A, eam_d, eam_beta, eam_c, eam_c0, eam_c1, eam_c2;
    int ex_shift;
    int aniso_split;
} sl_potential;

/* Energies in eV: kinetic sum_i m v^2/2, pair, exchange (the magnetic pair
 * energy: exchange plus the Neel and DMI terms when set), Zeeman,
 * anisotropy. */
typedef struct {
    double kin, pair, exchange, zeeman, aniso, total;
} sl_energy;

typedef struct {
    int64_t step;            /* step counter (Philox counter word)          */
    int64_t rebuilds;        /* neighbour-list rebuilds so far              */
    int n_colours;           /* current number of colour classes K         */
    int jp_rounds;           /* colouring rounds of the last rebuild        */
    int max_spin_nbr_seen;   /* largest spin segment of the last build      */
    int max_nbr_seen;        /* largest row of the last build               */
} sl_stats;

/* Create a system. Fails with SL_E_ARG (bad sizes or precision) or SL_E_BOX
 * (a box side shorter than twice the largest list radius, which would make
 * the minimum image ambiguous; checked again at sl_set_potential). */
int sl_create(const sl_params *p, sl_system **out);

/* Destroy a system and free its device memory. NULL is allowed. */
int sl_destroy(sl_system *sys);

/* Set the state in user order (Sec. 3: X = (r, p, s); velocities here).
 * r: double[N][3] unwrapped positions (may be NULL to keep the current);
 * v: double[N][3] (NULL: keep); s: double[N][3] with ||s_i| - 1| <= 1e-12
 * (otherwise SL_E_ARG; NULL: keep); mass: double[N] in amu, > 0 (NULL:
 * keep). Any NaN/Inf gives SL_E_NONFINITE. Invalidates the forces, the
 * neighbour list (unless user-supplied) and the colouring. */
int sl_set_state(sl_system *sys, const double *r, const double *v,
                 const double *s, const double *mass, int where);

/* Copy the state out in user order; NULL outputs are skipped. Synchronises. */
int sl_get_state(sl_system *sys, double *r, double *v, double *s, int where);

/* Set the interactions (see sl_potential). Invalidates the list. */
int sl_set_potential(sl_system *sys, const sl_potential *pot);

/* Device cell-list neighbour build with Verlet skin `skin` and row capacity
 * max_nbr (0 keeps the current values). Rows hold every j closer than
 * max(cutoffs) + skin, the entries closer than ex_rc + skin first (the
 * spin segment). Two spins may not share a colour class (Sec. 5.1: spins
 * updated together must not interact) when they are closer than
 * ex_rc + skin/3 at colouring time; same-class pairs of the spin segment
 * that are farther apart are watched instead.
 * Rebuild rule: before step k the list is rebuilt when, at the boundary
 * before step k-1,
 *   max_i |r_i - r_i^build| + 2a max_i |v_i| >= skin/2 - 0.01 A, or
 *   min over watched pairs |r_i - r_j| - 4a max_i |v_i| < ex_rc + 0.01 A
 * with a = max(|dt| of step k-1, |dt| of step k), the two differing only
 * across calls that change dt (a boundary that rebuilt counts its build
 * positions and the colour radius ex_rc + skin/3 instead). A rebuild keeps the colouring where
 * valid: ends of conflicting edges with the later key (z, y, x, id), and
 * atoms outside the palette of the last full colouring, are recoloured
 * first-fit in key order. */
int sl_set_neighbor(sl_system *sys, double skin, int max_nbr);

/* Order of the entries inside each of the two segments of a list row
 * (a memory-layout choice: the physics is unchanged up to summation-order
 * roundoff). quantum = 0 (default): cell-loop order. quantum > 0 (A): each
 * segment sorted by the neighbour's displacement r_j - r_i rounded to a grid
 * of that step, (z, y, x) lexicographic, ties by internal index. In a
 * crystal whose neighbour displacements are multiples of the grid step (half
 * the cubic lattice constant for bcc and fcc) slot k of every row then holds
 * the neighbour at the same lattice offset, so a wavefront of spatially
 * sorted atoms gathers slot k from a short contiguous range of memory.
 * A segment of more than 64 entries keeps the cell-loop order (the sort
 * holds a segment's keys in LDS).
 * Applies from the next automatic list build (the list is invalidated);
 * user-supplied lists keep their order. SL_E_ARG if quantum < 0 or not
 * finite. */
int sl_set_row_order(sl_system *sys, double quantum);

/* User-supplied full list in CSR form over user ids: offsets[N+1], idx[].
 * Each row is split (stably) into entries closer than ex_rc + skin first.
 * Disables automatic rebuilds. */
int sl_set_neighbor_list(sl_system *sys, const int *offsets, const int *idx,
                         int where);

/* Current list in user ids: nspin[N], nall[N] and rows concatenated in idx
 * (row order as stored). Returns the total number of entries (>= 0) or an
 * error; when cap is smaller than the total only the counts are written. */
int64_t sl_get_neighbor_list(sl_system *sys, int *nspin, int *nall, int *idx,
                             int64_t cap);

/* Override the colouring (colour[N] in user order, values 0..63); validated
 * against the colouring graph (spin-segment entries closer than
 * ex_rc + skin/3; every spin-segment entry for a user list), SL_E_COLOR on
 * conflict. Its palette becomes the base palette of later repairs. */
int sl_set_coloring(sl_system *sys, const int *colour, int where);

/* Colouring in user order and the class count K. Synchronises. */
int sl_get_coloring(sl_system *sys, int *colour, int *K);

/* Set the step counter (used as a Philox counter word). */
int sl_set_step(sl_system *sys, int64_t step);

/* Advance n >= 0 steps of length dt (dt < 0 runs backwards). */
int sl_step(sl_system *sys, int64_t n, double dt);

/* Spin update order of the spin half-steps.
 *  - SL_ORDER_COLOUR (default): colour classes of the spin graph, every
 *    class updated in parallel (the GPU form of the sectors of Sec. 5.1).
 *  - SL_ORDER_SECTORS: the paper's own order (Sec. 5.1, Eq.
 *    spin_ST_sectoring). The box is split into grid[0] x grid[1] x grid[2]
 *    subdomains (the processors of the paper), each bisected once per
 *    dimension into 8 sectors, from the wrapped positions at the start of
 *    every step. Class k is sector k of every subdomain: subdomains run in
 *    parallel, and the atoms of one subdomain's sector are updated one after
 *    another in id order (reversed on backward sweeps). A sector must be at
 *    least the spin radius (ex_rc + skin) wide, else SL_E_ARG. Slow on a GPU
 *    by nature (the sequential chains are a sector's atom count long); meant
 *    for ordering studies.
 *  - SL_ORDER_SERIAL: the serial order of Eq. spin_ST_decomposition (every
 *    spin in id order, one thread); small systems only.
 * The rebuild rule's watched-pair term applies to the colour ordering only.
 * grid is read for SL_ORDER_SECTORS only. Batches always use colours. */
enum { SL_ORDER_COLOUR = 0, SL_ORDER_SECTORS = 1, SL_ORDER_SERIAL = 2 };
int sl_set_ordering(sl_system *sys, int ordering, const int grid[3]);

/* Energy of the current state (computed now). Synchronises. */
int sl_get_energy(sl_system *sys, sl_energy *out);

/* M = sum_i s_i of the current state. Synchronises. */
int sl_get_magnetization(sl_system *sys, double M[3]);

/* Temperatures of the current state (Sec. 4.2), in K: the kinetic lattice
 * temperature T_L = (2 / 3 N k_B) sum_i m_i v_i^2 / 2 (Eq.
 * lattice_temperature) and the spin temperature of Nurdin et al.
 * T_S = (hbar / 2 k_B) sum_i |s_i x omega_i|^2 / sum_i s_i.omega_i (Eq.
 * spin_temperature) with the conservative omega_i (exchange, Zeeman and
 * anisotropy). Either pointer may be NULL. Both are deterministic device
 * reductions. Synchronises. */
int sl_get_temperatures(sl_system *sys, double *T_lattice, double *T_spin);

/* Samples recorded every thermo_every steps since the last call: up to max
 * entries of (step, energy, M[3]); *count receives the number written. */
int sl_get_thermo(sl_system *sys, int max, int64_t *steps, sl_energy *e,
                  double *M, int *count);

int sl_get_stats(sl_system *sys, sl_stats *out);

/* Wait for the system's stream; returns any sticky device error. */
int sl_synchronize(sl_system *sys);

/* Launch shape of the per-step kernels. Changes speed only: the results
 * differ at most by summation-order roundoff. lanes = 1, 2, 4 or 8
 * consecutive wavefront lanes cooperate on one atom (0 = default: 2 for
 * the spin phase, 1 for forces).
 * Runs of consecutive colour classes of at most small_class atoms each are
 * applied by one single-workgroup launch (0 = default 128, -1 = never). */
typedef struct {
    int spin_lanes;
    int force_lanes;
    int small_class;
    int jcache;       /* exchange-coefficient cache (analytic potential and
                         the spline form of a learned one): J(r_ij) of every
                         spin-segment entry is evaluated once per drift and
                         read by the spin phases; 0 = default (on for the
                         FP32 form, off for FP64, as measured on MI355X),
                         1 on, -1 off */
    int overlap;      /* split force (analytic potentials, 1 or 2 force
                         lanes): the spin-independent pair terms of a step's
                         closing force run on a second stream of the library
                         while the spins update, and the closing force launch
                         adds the spin-dependent terms; 0 = default (off),
                         1 on, -1 off. Not changed by the autotuner. */
} sl_tuning;

int sl_set_tuning(sl_system *sys, const sl_tuning *t);
int sl_get_tuning(sl_system *sys, sl_tuning *t);

/* Autotuner. Runs windows of `steps` steps of length dt under each
 * candidate launch shape (spin lanes 1, 2, 4, 8; force lanes 1, 2; the
 * exchange-coefficient cache on or off) on a scratch copy of the system
 * (same parameters, interactions, learned potential, user list, state and
 * step counter; its own stream and memory, freed before returning), times
 * each whole window with HIP events on the copy's stream (a window with a
 * list rebuild in it is run again; four rounds in rotating order, best
 * window per shape),
 * and sets the fastest shape on sys (returned in *chosen if not NULL). sys is
 * not advanced, and its later results change at most by summation-order
 * roundoff (the shape only splits neighbour sums across lanes); colouring,
 * skin and rebuild rule are never touched. When the environment variable
 * SL_TUNE_CACHE names a file, results are looked up there first (one JSON
 * object per line, keyed by the GPU architecture and the system's shape)
 * and appended after tuning. */
int sl_autotune(sl_system *sys, int steps, double dt, sl_tuning *chosen);

/* Per-kernel timing with HIP events on the system's stream. With on = 1
 * every launch of the spin-phase, force, rebuild and table kernels inside
 * the steps of sl_step is timed; with on = N > 1 only the launches of the
 * second step of each sl_step call (the first when the call has one step)
 * and of every N-th step after it are (the event packets themselves cost a
 * few microseconds of GPU time each); 0 stops. A run of consecutive
 * spin-phase launches is bracketed by one pair of events and counted as its
 * number of launches; every other launch by a pair of its own. Launches outside whole steps
 * (the force launch that opens a call, sl_get_energy and the like) are
 * never timed, so the totals are those of whole steps. sl_get_profile
 * returns, per kernel kind, the launch count, the summed event time in ms
 * and the work items since profiling was last switched on (switching it off
 * keeps the totals readable). Kinds and their work items: 0 spin phase
 * (atom updates: a launch that applies two successive updates to a class
 * counts its atoms twice), 1 force (atoms), 2 neighbour rebuild (atoms),
 * 3 pair-coefficient table (exchange cache: atoms; per-pair learned
 * potential: pairs), 4 pair pass of the split force (atoms; its events are
 * on the library's second stream). */
int sl_set_profiling(sl_system *sys, int on);
int sl_get_profile(sl_system *sys, int kind, int64_t *launches, double *ms,
                   double *work_items);

/* ------------------------------------------------------------------------
 * Learned pair potential: a per-pair MLP that stands in for the exchange
 * J(r) (appendix A.1) and the mechanical pair energy phi(r) of
 * Eq. sl_hamiltonian. r -> 16 Gaussian radial basis functions
 * b_k = exp(-((r - k mu_step)/sigma)^2) -> silu(64) -> silu(64) -> (y0, y1);
 * J(r) = sJ y0 for r < ex_rc, phi(r) = sP [y1(r) - y1(rc) - (r - rc) y1'(rc)]
 * for r < rc. Evaluated on BF16 matrix cores with FP32 accumulation; the
 * r-derivatives go through the network as a forward-mode tangent.
 * Parameters (FP32 master copy, SL_MLP_NPARAM values): W1[64][16], c1[64],
 * W2[64][64], c2[64], W3[2][64], c3[2], row-major.
 */
#define SL_MLP_NPARAM 5378

typedef struct sl_mlp sl_mlp;

typedef struct {
    double sigma;     /* RBF width, A (0: 0.4)                          */
    double mu_step;   /* RBF centre spacing, A (0: 5/15)                */
    double sJ, sP;    /* output scales of J and phi, eV (0: 0.01, 1)    */
    double ex_rc;     /* exchange cutoff, A (0: 3.5)                    */
    double rc;        /* mechanical cutoff, A (0: 5)                    */
    void *stream;     /* hipStream_t; NULL: own stream                  */
} sl_mlp_spec;

int sl_mlp_create(const sl_mlp_spec *spec, sl_mlp **out);
int sl_mlp_destroy(sl_mlp *m);
/* Copy in/out the FP32 master parameters (n must be SL_MLP_NPARAM). */
int sl_mlp_set_weights(sl_mlp *m, const float *params, int n, int where);
int sl_mlp_get_weights(sl_mlp *m, float *params, int n, int where);
/* out[P][4] = (J, dJ/dr, phi, dphi/dr) at the P distances r (tests). */
int sl_mlp_eval(sl_mlp *m, const double *r, int64_t P, double *out, int where);
const char *sl_mlp_last_error(const sl_mlp *m);

/* sl_mlp_eval without any device allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same arguments, output layout and
 * results (bit for bit) as sl_mlp_eval, for P <= SL_MLP_EVAL_STATIC_MAX
 * distances (SL_E_ARG beyond). Its staging lives in one library-owned static
 * device array per GPU (52 bytes per distance, about 1.7 MB), held from the
 * first call on that GPU until the process ends; no call allocates or frees
 * device memory. Every call on a GPU reuses that GPU's array: calls that
 * overlap on one GPU (from other threads or on other streams) race on it.
 * The handle's device must be the current one (SL_E_ARG otherwise). With
 * where = SL_DEVICE the call only enqueues work on the handle's stream (r
 * must be ready on that stream; out is valid once the stream has reached the
 * end of the call); with SL_HOST it synchronises the stream before
 * returning. */
#define SL_MLP_EVAL_STATIC_MAX 32768
int sl_mlp_eval_static(sl_mlp *m, const double *r, int64_t P, double *out, int where);

/* Use the learned potential for J and the mechanical pair energy of this
 * system (replacing Morse and Bethe-Slater; Zeeman, anisotropy and the bath
 * are kept); NULL restores the analytic potential. FP32 form only. The
 * evaluation follows sl_set_mlp_mode. The handle must outlive its use; its
 * weights may be changed between sl_step calls. */
int sl_set_mlp(sl_system *sys, sl_mlp *m);

/* How a system evaluates the learned potential.
 *   SL_MLP_SPLINE (default): the network's raw outputs and r-derivatives
 *     are tabulated once per weight update (4096 points on [0.5 A, rc], the
 *     FP32 master weights evaluated in FP64) and every pair takes a cubic
 *     Hermite interpolant of them; the force is the exact derivative of
 *     the interpolated energy, so the dynamics conserve the energy that is
 *     reported.
 *   SL_MLP_PAIRWISE: after every drift the network itself is evaluated
 *     once per unordered pair of the list (BF16 MFMA, FP32 accumulation;
 *     value and r-tangent streams) and the kernels read that table. */
enum { SL_MLP_PAIRWISE = 0, SL_MLP_SPLINE = 1 };
int sl_set_mlp_mode(sl_system *sys, int mode);

/* Per-atom force F_i = sum_j [-phi'(r) + J'(r) s_i.s_j] e_ij (Eq. p_advance)
 * and exchange part of hbar omega_i = sum_j J(r_ij) s_j (Sec. 2) of the
 * current state, double[N][3] each in user order (NULL: skipped), from the
 * analytic potential or the learned one. Synchronises. */
int sl_get_fields(sl_system *sys, double *F, double *hw, int where);

/* Training data: S snapshots of one N-atom periodic box, host arrays.
 * Labels come from the analytic path: E = pair + exchange energy, F the
 * force and hw the exchange part of hbar omega (see sl_get_fields). */
typedef struct {
    int n_snapshots;
    int64_t n_atoms;
    double box[3];
    const double *r;     /* [S][N][3] positions, A           */
    const double *s;     /* [S][N][3] unit spins             */
    const double *E;     /* [S] pair + exchange energy, eV   */
    const double *F;     /* [S][N][3] forces, eV/A           */
    const double *hw;    /* [S][N][3] exchange hbar omega, eV */
} sl_dataset;

/* Loss of one snapshot (learned potential in place of J and phi):
 *   w_E ((E - E_ref)/N)^2 + w_F |F - F_ref|^2/(3N) + w_W |hw - hw_ref|^2/(3N)
 * and its gradient with respect to the SL_MLP_NPARAM master parameters
 * (grad may be NULL), by the BF16-MFMA forward/tangent and reverse kernels
 * with FP32 accumulation. */
int sl_mlp_loss_grad(sl_mlp *m, const sl_dataset *d, int snapshot, const double w[3],
                     double *loss, float *grad);

typedef struct {
    int epochs;                  /* passes over the snapshots              */
    double lr, beta1, beta2, eps;/* Adam (0: 1e-3, 0.9, 0.999, 1e-8)       */
    double w_E, w_F, w_W;        /* loss weights                           */
    uint64_t seed;               /* snapshot order                         */
} sl_train_opts;

typedef struct {
    double loss_first, loss_last;   /* mean loss of the first / last epoch */
    int64_t updates;
} sl_train_log;

/* Adam on the FP32 master parameters, one update per snapshot. */
int sl_mlp_train(sl_mlp *m, const sl_dataset *d, const sl_train_opts *o, sl_train_log *log);

/* ------------------------------------------------------------------------
 * Batched replicas: R independent coupled systems (each with its own box,
 * size, list, colouring, Philox key/replica index, bath temperature and
 * field) advanced together. A step of every replica is the step of
 * sl_step, with the same rebuild rule per replica. Two execution modes
 * (sl_batch_set_mode): one persistent kernel launch (replayed from a
 * captured hipGraph) with one workgroup per replica, which stops a replica
 * before a step that needs a neighbour-list rebuild, the library rebuilding
 * it and replaying the launch until every replica has done n steps; or one
 * launch per colour phase over all replicas. Results per replica equal
 * those of a single sl_system up to summation order. All replicas share
 * one precision; frozen lattices are not batched.
 */
typedef struct sl_batch sl_batch;

/* params[R], pots[R]: per-replica creation parameters and interactions
 * (params[r].stream is ignored: the batch owns one stream). */
int sl_batch_create(int R, const sl_params *params, const sl_potential *pots,
                    sl_batch **out);
int sl_batch_destroy(sl_batch *b);
/* State of replica r (same contract as sl_set_state / sl_get_state). */
int sl_batch_set_state(sl_batch *b, int r, const double *x, const double *v,
                       const double *s, const double *mass, int where);
int sl_batch_get_state(sl_batch *b, int r, double *x, double *v, double *s,
                       int where);
int sl_batch_get_energy(sl_batch *b, int r, sl_energy *out);
/* Temperatures of replica r (same contract as sl_get_temperatures). */
int sl_batch_get_temperatures(sl_batch *b, int r, double *T_lattice, double *T_spin);
/* n steps of length dt for every replica. */
int sl_batch_step(sl_batch *b, int64_t n, double dt);

/* Execution mode of sl_batch_step; both give the same trajectories for the
 * same lanes setting (they share the per-atom device code).
 *   SL_BATCH_PERSISTENT: one workgroup per replica runs all its steps in
 *     one launch, replayed from a captured hipGraph (suits many small
 *     replicas: no launch per phase);
 *   SL_BATCH_PHASED: one launch per colour phase and per force pass over
 *     all replicas at once (grid = tiles x replicas), the host deciding
 *     rebuilds one step ahead (suits replicas too large for one CU).
 * Default SL_BATCH_PHASED (5x faster than the persistent launch for 64
 * replicas of 1k-28k atoms on MI355X). */
enum { SL_BATCH_PERSISTENT = 0, SL_BATCH_PHASED = 1 };
int sl_batch_set_mode(sl_batch *b, int mode);
int sl_batch_get_mode(sl_batch *b, int *mode);

/* Batch autotuner: times `steps` steps of a scratch copy of the batch
 * under each (mode, lanes) pair (phased with 1, 2, 4 lanes; persistent
 * with 1, 2) and keeps the fastest on b; b is not advanced. Same cache as
 * sl_autotune. */
int sl_batch_autotune(sl_batch *b, int steps, double dt, int *mode, int *lanes);
/* Lanes per atom inside the persistent kernel (1, 2 or 4; speed only). */
int sl_batch_set_lanes(sl_batch *b, int lanes);
/* sl_set_row_order on every replica (one grid step for all; SL_E_ARG if
 * negative or not finite). */
int sl_batch_set_row_order(sl_batch *b, double quantum);
int sl_batch_get_stats(sl_batch *b, int64_t *launches, int64_t *rebuilds, int *lanes);
const char *sl_batch_last_error(const sl_batch *b);

/* Message of the last failed call on this handle (or of the last failed
 * sl_create when sys is NULL). Never NULL. */
const char *sl_last_error(const sl_system *sys);

#ifdef __cplusplus
}
#endif
#endif
