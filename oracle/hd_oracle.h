/*
 * FP64 CPU oracle for the hyperdynamics-for-sliding hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, obviously
 * correct reference for what the GPU path computes.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What it computes (Kim & Falk, "Accelerated molecular dynamics simulation
 * of low-velocity frictional sliding"):
 *   - Lennard-Jones pair potential with a type table (eq. 9; parameters of
 *     Sec. 3.1.1 and Sec. 3.2.1), energy-shifted at the cutoff rc;
 *   - the slider drive on the rigid top layer (Sec. 3.1.1), lateral force
 *     F_R = k (x_S - x_T) (eq. 10);
 *   - everything about the basin minimum r_O, over the generalised position
 *     vector;
 *   - the local variables d (eq. 7), slope g = grad V . s (eq. 5),
 *     curvature kappa = d2V/ds2 = u.Hu/d^2 (eq. 6) and the eigenvalue
 *     variable of eq. 15 (the lowest Hessian eigenvalue, tracked as the
 *     Rayleigh quotient lambda = q^T H q along a mode estimate q that turns
 *     towards the lowest mode by one gradient step per time step), any one
 *     or two of them as bias variables: each through the switch of eq. 14
 *     (eq. 15's form), two combined by eq. 13; the bias force from the
 *     chain rule, with grad g = (Hu - F - g u/d)/d,
 *     grad kappa = (2 Hu + T[u,u])/d^2 - 2 kappa u/d^2 (T[u,u]: third
 *     derivatives of V contracted twice with u), grad d = u/d and
 *     grad lambda = T[q,q] at fixed q;
 *   - the boosted clock t_hyper = sum dt exp(dV/kT) (eq. 3 as a time average;
 *     eq. 8 fixes what it means for stepped sliding);
 *   - a Langevin BAOAB step, or the paper's Nose-Hoover chain thermostat
 *     (Sec. 3.1.1) with velocity Verlet, the chain integrated by the
 *     Trotter splitting of Martyna, Tuckerman, Tobias and Klein (Mol. Phys.
 *     87, 1117, 1996);
 *   - Philox4x32-10 + Box-Muller normals;
 *   - a FIRE minimiser for r_O.
 *
 * Parity unpinned: none of the functions below; each is pinned by tests
 * (closed forms, finite differences, invariants, brute force, limits).
 *
 * Units: reduced LJ units.  Arrays are SoA: x[k*n + i] is component k of
 * atom i.  Roles: 0 mobile, 1 fixed, 2 rigid.  Types: 0 substrate, 1 tip.
 */
#ifndef HD_ORACLE_H
#define HD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim, n;
    double box[3];
    int32_t periodic[3];
    double mass;
    double eps[2][2], sig[2][2], rc, skin;
    double dt, gamma, kT;
    uint64_t seed;
    double k_spring, f_normal, x_slider, v_slider;
    int32_t bias_on, m_b;
    double dv_max, g_lo, g_hi;
    /* harmonic tip bonds (eq. 12): when tip_bonds, a tip-tip pair closer
     * than r_bond_cut is a spring 1/2 k_bond (r - r_bond)^2 and farther
     * tip-tip pairs do not interact */
    int32_t tip_bonds, pad_tb;
    double k_bond, r_bond, r_bond_cut;
    /* bias variables: bias_var1 enters dV1 (thresholds g_lo, g_hi) and
     * bias_var2 (-1 = none) dV2 (thresholds b2_lo, b2_hi), combined by
     * eq. 13.  0 = slope (eq. 5), 1 = curvature (eq. 6), 2 = distance
     * (eq. 7).  A switch is full on the g_hi side and zero on the g_lo
     * side, whichever of the two is larger. */
    int32_t bias_var1, bias_var2;
    double b2_lo, b2_hi;
    /* thermostat: 0 Langevin (BAOAB, gamma), 1 Nose-Hoover chain of nhc_len
     * (1..4) thermostats with relaxation time nhc_tau: masses
     * Q_1 = N_f kT tau^2, Q_j = kT tau^2, N_f = dim (n_mobile + 1 if the
     * model has a rigid layer) */
    int32_t thermostat, nhc_len;
    double nhc_tau;
    /* eigenvalue bias variable (3): the Rayleigh quotient of the reduced
     * Hessian along the system's mode estimate q; after every step q takes
     * one rotation step q <- q - mode_alpha (H q - lambda q) (normalised
     * over the degrees of freedom at the next evaluation) */
    double mode_alpha;
} orc_params;

typedef struct {
    double e_lj, v_drive, e_pot, e_kin;
    double d, g, dv, dvp;
    double x_slider, x_tip, f_lat;
    double t_md, t_hyper;
    int64_t step;
    int32_t flags, pad_f;
    double kappa;         /* curvature along s (eq. 6); 0 when d ~ 0 */
    double dv1, dv2;      /* the two switches of eq. 13 */
    /* Nose-Hoover chain energy sum_j Q_j xi_j^2 / 2 + N_f kT eta_1
     * + kT sum_{j>1} eta_j: with e_kin + e_pot + dv it is conserved */
    double e_nhc;
    /* the eigenvalue variable lambda = q^T H q along the unit mode estimate
     * (systems biased on it; 0 otherwise) */
    double lambda;
} orc_scalars;

/* Opaque simulation state for one system. */
typedef struct orc_sys orc_sys;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Four standard normals from counter (step, particle, tag) and the seed,
 * via (w + 0.5) 2^-32 uniforms and the Box-Muller transform. */
void orc_normals(uint64_t seed, int64_t step, uint32_t particle, uint32_t tag, double z[4]);

/* Pairs (i<j) with r^2 < rl^2, excluding fixed-fixed and rigid-rigid pairs
 * when exclude != 0.  Brute force over all pairs.  Returns the count; writes
 * at most cap pairs as (i, j) into ij. */
int64_t orc_pairs_brute(const orc_params *p, const double *x, const uint8_t *role,
                        double rl, int exclude, int32_t *ij, int64_t cap);
/* Same set via the oracle's own cell list. */
int64_t orc_pairs_cells(const orc_params *p, const double *x, const uint8_t *role,
                        double rl, int exclude, int32_t *ij, int64_t cap);

orc_sys *orc_create(const orc_params *p, const double *x, const uint8_t *type,
                    const uint8_t *role, const double *rO);
void orc_destroy(orc_sys *s);
void orc_set_params(orc_sys *s, const orc_params *p);
void orc_set_positions(orc_sys *s, const double *x);
void orc_set_velocities(orc_sys *s, const double *v);
void orc_set_reference(orc_sys *s, const double *rO);
/* Maxwell-Boltzmann velocities from the seed (tag 1, step 0). */
void orc_init_velocities(orc_sys *s);
/* 0 = cell list (default), 1 = brute force over all pairs. */
void orc_set_pair_method(orc_sys *s, int brute);

/* Evaluate energy, forces, Hu and the bias at the current positions.  Does not
 * advance the clock.  Outputs (any may be NULL): f_lj = -grad V (LJ + drive
 * share), hu = H u, f_b = bias force, f_tot = f_lj + f_b, e_atom = per-atom
 * half pair energies. */
void orc_compute(orc_sys *s, double *f_lj, double *hu, double *f_b, double *f_tot,
                 double *e_atom, orc_scalars *out);
/* Nose-Hoover chain state: thermostat velocities xi and positions eta (4
 * each; entries beyond nhc_len unused). */
void orc_get_nhc(const orc_sys *s, double xi[4], double eta[4]);
void orc_set_nhc(orc_sys *s, const double xi[4], const double eta[4]);
/* T[u,u] of the last evaluation: the gradient of u.H(r)u at fixed u (for
 * a system biased on the eigenvalue variable, T[q,q] along its unit mode). */
void orc_get_tuu(const orc_sys *s, double *t);
/* Mode estimate of the eigenvalue variable, atom layout [dim][n]: mobile
 * atoms' components, the rigid body's (read from its first atom) and zero
 * for fixed atoms; orc_get_mode returns it normalised over the degrees of
 * freedom. */
void orc_set_mode(orc_sys *s, const double *q);
void orc_get_mode(const orc_sys *s, double *q);
/* Evaluate at the current positions and take one rotation step of the mode
 * (what a time step does after its force evaluation), without moving. */
void orc_rotate_mode(orc_sys *s);
/* Advance nsteps BAOAB steps (bias included when enabled). */
void orc_step(orc_sys *s, int64_t nsteps);
void orc_get_positions(const orc_sys *s, double *x);
void orc_get_velocities(const orc_sys *s, double *v);
void orc_get_scalars(const orc_sys *s, orc_scalars *out);
/* Rigid body state: centre of mass X_R, velocity V_R, initial X_R(0). */
void orc_get_rigid(const orc_sys *s, double XR[3], double VR[3], double XR0[3]);
/* Relax positions with FIRE (bias off) until max |F| < ftol on integrated
 * degrees of freedom.  Returns iterations used (negative if not converged).
 * The relaxed positions become the current positions. */
int64_t orc_fire(orc_sys *s, double ftol, int64_t maxit);

#ifdef __cplusplus
}
#endif
#endif
