/*
 * hd.h -- C ABI of libhd.so, the MI355X (gfx950) hot path of hyperdynamics
 * for driven frictional sliding (Kim & Falk, "Accelerated molecular dynamics
 * simulation of low-velocity frictional sliding").
 *
 * One context holds a batch of independent AFM tip/substrate models, each at
 * its own slider position (the parallel slider-position scheme of Sec. 2.3:
 * the transition probabilities at different stepped slider positions are
 * independent, so the positions can run at the same time).  Every step of
 * every system runs in HIP kernels on the GPU:
 *   - Lennard-Jones energy and forces with a type table (eq. 9; parameters of
 *     Sec. 3.1.1 / Sec. 3.2.1), energy-shifted at rc, over cell-binned Verlet
 *     neighbour lists with a skin; optionally harmonic tip bonds (eq. 12) for
 *     the conical-tip model of Sec. 3.2.1;
 *   - the slider drive on the rigid top tip layer: spring k to the slider
 *     along x, anchor of stiffness k along y in 3D, normal load F_N pushing
 *     down (Sec. 3.1.1, Sec. 3.2.1); lateral force F_R = k (x_S - x_T) (eq. 10);
 *   - the bias of Sec. 2.2: the distance d (eq. 7), the slope
 *     g = grad V . s (eq. 5), the curvature kappa (eq. 6) and the lowest
 *     Hessian eigenvalue (the variable of eq. 15), one or two of them through
 *     the switch of eq. 14 and combined by eq. 13 (the slope alone by
 *     default), with the bias force -grad dV by the chain rule;
 *   - the boosted clock t_hyper = sum dt exp(dV/kT) (eq. 3, eq. 8);
 *   - a Langevin BAOAB step with Philox4x32-10 normals, or the paper's
 *     Nose-Hoover chain with velocity Verlet (Sec. 3.1.1), per system;
 *   - the FIRE quench that gives the basin minimum r_O and the
 *     quench-and-compare transition check of Sec. 2.3.
 *
 * Conventions
 *   - Every call returns hd_status; nothing throws across the ABI.  On
 *     failure hd_last_error(ctx) gives a message.  After HD_E_HIP the context
 *     is poisoned and only hd_destroy is valid.
 *   - Host arrays are owned by the caller and copied during the call.  Per-atom
 *     arrays are SoA float64 of shape [dim][n_atoms] (component k of atom i at
 *     k*n_atoms + i).  Device pointers (the *_device calls) must hold the same
 *     layout and stay valid until the call returns.
 *   - Device memory is owned by the context (hd_finalize allocates it,
 *     hd_destroy frees it), except for fields the caller binds to its own
 *     device storage with hd_bind_device.  Work is ordered on the context's
 *     HIP stream; the hd_read_* calls synchronise that stream before
 *     returning.
 *   - Systems are added before hd_finalize; per-system parameters (slider,
 *     bias, thermostat) may change afterwards.
 *   - One context per host thread.
 */
#ifndef HD_H
#define HD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HD_OK = 0,
    HD_E_ARG = -1,       /* invalid argument (null pointer, bad index, bad size) */
    HD_E_OOM = -2,       /* device or host allocation failed */
    HD_E_HIP = -3,       /* HIP runtime error; the context is poisoned */
    HD_E_STATE = -4,     /* call not valid in the current lifecycle state */
    HD_E_UNSTABLE = -5,  /* every system has been frozen as unstable */
    HD_E_NOGPU = -6      /* no usable gfx950 device */
} hd_status;

/* Arithmetic of the pair pass.  Positions, velocities, reductions, the bias
 * scalars and the clock are float64 in both. */
typedef enum {
    HD_FP64 = 0,   /* float64 pair arithmetic */
    HD_FP32C = 1   /* float32 pair arithmetic, per-atom sums in float64;
                      displacements and the cutoff decision in float64; the
                      Langevin normals formed in float32 from the same Philox
                      words (relative error ~1e-7) */
} hd_precision;

/* How hd_step schedules the batch.  BATCHED runs small systems in one
 * persistent launch per chunk of steps (one workgroup per system, state in
 * LDS) and large systems on the grid kernels, concurrently (see
 * hd_set_launch).  GRID runs a short sequence of kernels per step over all
 * systems, replayed from a HIP graph.  SEQUENTIAL is GRID applied to one
 * system at a time (the plain single-system path). */
typedef enum { HD_EXEC_BATCHED = 0, HD_EXEC_GRID = 1, HD_EXEC_SEQUENTIAL = 2 } hd_exec;

/* Per-atom roles and types. */
enum { HD_ROLE_MOBILE = 0, HD_ROLE_FIXED = 1, HD_ROLE_RIGID = 2 };
enum { HD_TYPE_SUBSTRATE = 0, HD_TYPE_TIP = 1 };

typedef struct hd_ctx hd_ctx;

/* Geometry of one model.  dim is 2 or 3.  box[k] is the periodic length on
 * axes with periodic[k] != 0 (it must be at least 2 (rc + skin)); open axes
 * ignore box[k].  pos is SoA [dim][n_atoms]; type and role have n_atoms
 * entries.  Atoms with role RIGID move together as one body of mass
 * n_rigid * mass; atoms with role FIXED never move. */
typedef struct {
    int32_t dim;
    int32_t n_atoms;
    double box[3];
    int32_t periodic[3];
    const double *pos;
    const uint8_t *type;
    const uint8_t *role;
    double mass;
} hd_system_desc;

/* Lennard-Jones table indexed [type_a][type_b] (eq. 9), energy-shifted at rc;
 * skin is the Verlet-list margin (lists are rebuilt when an atom has moved
 * more than skin/2 since the last build). */
typedef struct { double eps[2][2], sig[2][2], rc, skin; } hd_lj_params;

/* Langevin thermostat: time step, friction, temperature, 64-bit seed of the
 * Philox stream (key = seed; counter = step, particle, tag). */
typedef struct { double dt, gamma, kT; uint64_t seed; } hd_thermo_params;

/* Slider drive: spring stiffness k, normal load F_N, slider position x_S and
 * slider velocity (v_slider = 0: stepped sliding at fixed x_S; otherwise
 * x_S(step) = x_slider + v_slider * step * dt). */
typedef struct { double k_spring, f_normal, x_slider, v_slider; } hd_drive_params;

/* Bias of eq. 14: dV_max, thresholds g_lo < g_hi, integer exponent m_b >= 1.
 * The switch acts on the slope g unless hd_set_bias_variables picks another
 * variable (for the distance, g_lo > g_hi).  enabled = 0 turns the bias (and
 * its force) off. */
typedef struct { int32_t enabled, m_b; double dv_max, g_lo, g_hi; } hd_bias_params;

/* Per-system scalars after the last evaluation. */
typedef struct {
    double e_pot;     /* LJ energy + drive energy */
    double e_kin;     /* mobile atoms + rigid body */
    double dv;        /* bias dV */
    double dvp;       /* d dV / d g */
    double g;         /* slope, eq. 5 */
    double d;         /* distance from r_O, eq. 7 */
    double t_md;      /* elapsed MD time */
    double t_hyper;   /* boosted time sum dt exp(dV/kT) */
    double x_slider;  /* slider position at the last evaluation */
    double x_tip;     /* tip position X_R,x - X_R,x(0) */
    double f_lat;     /* lateral force k (x_S - x_T), eq. 10 */
    int64_t step;     /* steps taken */
    int32_t flags;    /* HD_FLAG_* bits */
    int32_t n_rebuilds;
    double kappa;     /* curvature u.Hu/d^2 along s, eq. 6 (systems biased on
                         it; 0 otherwise) */
    double dv1, dv2;  /* the two switches combined by eq. 13 (dv2 = 0 with
                         one variable) */
    double e_nhc;     /* Nose-Hoover chain energy (0 under Langevin): with
                         e_pot + e_kin + dv it is conserved */
    double lambda;    /* the eigenvalue variable (eq. 15): the Rayleigh
                         quotient along the mode estimate (systems biased on
                         it; 0 otherwise) */
} hd_scalars;

enum { HD_FLAG_UNSTABLE = 1, HD_FLAG_NBR_OVERFLOW = 2 };

/* Which per-atom force hd_read_forces returns. */
/* HD_TUU: T[u,u], the gradient of u.H(r)u at fixed u (third derivatives of
 * V contracted twice with u), kept for systems biased on the curvature; for
 * systems biased on the eigenvalue T[w,w] along the unit mode estimate of
 * the last evaluation (the eigenvalue variable's gradient). */
enum { HD_FORCE_TOTAL = 0, HD_FORCE_LJ = 1, HD_FORCE_BIAS = 2, HD_HU = 3, HD_TUU = 4 };

/* Bias variables (eq. 5-7, eq. 15). */
enum { HD_BIAS_SLOPE = 0, HD_BIAS_CURVATURE = 1, HD_BIAS_DISTANCE = 2, HD_BIAS_EIGENVALUE = 3 };

/* Create a context on HIP device `device`.  hip_stream is a hipStream_t to
 * order work on (for example torch.cuda.current_stream().cuda_stream) or NULL
 * for a stream owned by the context. */
hd_status hd_create(hd_precision prec, int device, void *hip_stream, hd_ctx **out);

/* Choose the scheduler before hd_finalize (default HD_EXEC_BATCHED). */
hd_status hd_set_exec(hd_ctx *ctx, hd_exec exec);

/* Tuning knobs before hd_finalize: threads per workgroup of the grid tiles and
 * of the one-workgroup global kernel (64..1024, multiple of 64; 0 =
 * automatic), the neighbour-slot capacity per atom (0 = automatic: 32 in 2D,
 * 128 in 3D), and HD_LAUNCH_* flags.  Under HD_EXEC_BATCHED, systems that fit
 * one workgroup's LDS (at most 1024 atoms) run in the LDS-resident persistent
 * kernel when HD_LAUNCH_LDS is set (the default); the others run on the grid
 * kernels over the whole chip, concurrently, or on the persistent
 * one-workgroup global kernel when HD_LAUNCH_PERSISTENT_LARGE is set. */
enum { HD_LAUNCH_LDS = 1, HD_LAUNCH_PERSISTENT_LARGE = 2 };
hd_status hd_set_launch(hd_ctx *ctx, int32_t block_threads, int32_t max_neighbors, int32_t flags);

/* Append one model.  Copies every array.  Returns its index in *sys_id.  The
 * basin reference r_O defaults to the given positions; velocities start at 0;
 * the bias starts disabled. */
hd_status hd_add_system(hd_ctx *ctx, const hd_system_desc *desc, const hd_lj_params *lj,
                        const hd_thermo_params *thermo, const hd_drive_params *drive,
                        int32_t *sys_id);

/* Harmonic tip bonds (eq. 12) for system sys: with enabled, a pair of tip
 * atoms (type 1) closer than r_cut is a spring k_bond (r - r_bond)^2 / 2 and
 * farther tip pairs do not interact (tip-substrate and substrate pairs stay
 * LJ); without, tip pairs are LJ.  The cut lies between the tip lattice's
 * first and second neighbour shells (bonds follow the lattice and, stiff,
 * do not reach it).  HD_E_ARG unless k_bond >= 0, r_bond > 0 and
 * 0 < r_cut <= rc; HD_E_STATE after hd_finalize.  Off by default.  Such
 * systems run on the grid kernels (never LDS-resident). */
hd_status hd_set_tip_bonds(hd_ctx *ctx, int32_t sys, int32_t enabled, double k_bond, double r_bond,
                           double r_cut);

/* Bias variables of system `sys` (Sec. 2.2): var1 is the variable the switch
 * of hd_bias_params acts on, var2 (-1: none) a second one with its own
 * critical values lo2, hi2 (same dV_max and m_b), the two combined by
 * eq. 13: dV = dV1 + dV2 - dV1 dV2 / dV_max.  Variables: HD_BIAS_SLOPE
 * g = grad V . s (eq. 5), HD_BIAS_CURVATURE kappa = d2V/ds2 = u.Hu/d^2
 * (eq. 6), HD_BIAS_DISTANCE d = |r - r_O| (eq. 7), HD_BIAS_EIGENVALUE the
 * lowest Hessian eigenvalue of eq. 15 (see hd_set_min_mode).  A switch is
 * dV_max at or beyond its upper value and zero at or beyond its lower one;
 * for the slope, the curvature and the eigenvalue lower < upper, for the
 * distance lower > upper (the bias is full near r_O and vanishes as d
 * grows).  The bias force is -grad dV by the chain rule, with
 * grad g = (Hu - F - g u/d)/d, grad kappa = (2 Hu + T[u,u])/d^2
 * - 2 kappa u/d^2, grad d = u/d and grad lambda = T[w,w].
 * Default: the slope alone.  Before hd_finalize only (HD_E_STATE after);
 * HD_E_ARG for an unknown variable, var2 == var1, the curvature with the
 * eigenvalue, and, while the bias is enabled, for critical values in the
 * wrong order (also those set by hd_set_bias, which checks the same against
 * the current variables) or, with two variables, dv_max = 0.  Systems with
 * any other choice than the slope alone run on the grid kernels (never
 * LDS-resident). */
hd_status hd_set_bias_variables(hd_ctx *ctx, int32_t sys, int32_t var1, int32_t var2, double lo2, double hi2);

/* The eigenvalue variable of eq. 15 along the trajectory.  The paper biases
 * on the lowest eigenvalue of the Hessian but does not say how it follows
 * it; here each system carries a mode estimate q over its degrees of
 * freedom (mobile atoms' coordinates and the rigid body's), the variable is
 * the Rayleigh quotient lambda = w.Hw of the unbiased potential's Hessian
 * along w = P q/|q| (the mode spread over the atoms: each rigid atom moves
 * with the rigid body, fixed atoms stay; the drive's Hessian included), its
 * gradient at fixed q is T[w,w] (third derivatives of V contracted twice
 * with w, from the same pair pass), and after every step's force
 * evaluation q takes one gradient step on the Rayleigh quotient,
 * q <- w - alpha (P^T H w - lambda w), which turns it towards the lowest mode
 * (at a fixed configuration the steps converge to it when alpha is below
 * 1 / the largest eigenvalue).  mode: host [dim][n], hd_min_mode's layout
 * (mobile atoms' components, the rigid body's read from its first rigid
 * atom, fixed atoms ignored); any nonzero length (it is stored normalised
 * over the degrees of freedom).  Before or after
 * hd_finalize; HD_E_STATE unless the system is biased on the eigenvalue
 * (hd_set_bias_variables first); HD_E_ARG for alpha < 0.  Without a mode
 * (all zero) lambda is 0 and exerts no force. */
hd_status hd_set_min_mode(hd_ctx *ctx, int32_t sys, const double *mode, double alpha);
/* The current mode estimate, normalised over the degrees of freedom, into
 * out [dim][n] (rigid atoms: the rigid body's component; fixed atoms 0).
 * HD_E_STATE unless the system is biased on the eigenvalue. */
hd_status hd_read_min_mode(hd_ctx *ctx, int32_t sys, double *out);

/* Thermostat of system `sys`: chain_len = 0 keeps Langevin BAOAB (the
 * default, friction gamma of hd_thermo_params); 1..4 selects the paper's
 * Nose-Hoover chain (Sec. 3.1.1) of that many thermostats with relaxation
 * time tau: masses Q_1 = N_f kT tau^2 and Q_j = kT tau^2, N_f the mobile
 * atoms' coordinates plus the rigid body's.  A step is the chain over dt/2,
 * velocity Verlet (half kick, full drift, forces, half kick), the chain over
 * dt/2, with the Trotter splitting of Martyna, Tuckerman, Tobias and Klein
 * (1996); gamma is then unused.  The chain starts at rest.  Before
 * hd_finalize only (HD_E_STATE after); HD_E_ARG for chain_len outside 0..4,
 * tau <= 0 or kT <= 0.  Such systems run on the grid kernels. */
hd_status hd_set_nose_hoover(hd_ctx *ctx, int32_t sys, int32_t chain_len, double tau);

/* Basin minimum r_O (eq. 7), SoA [dim][n]. */
hd_status hd_set_reference(hd_ctx *ctx, int32_t sys, const double *rO);
hd_status hd_set_bias(hd_ctx *ctx, int32_t sys, const hd_bias_params *bias);
/* Stepped slider position x_S (Sec. 2.3). */
hd_status hd_set_slider(hd_ctx *ctx, int32_t sys, double x_slider);
hd_status hd_set_thermo(hd_ctx *ctx, int32_t sys, const hd_thermo_params *thermo);
/* Maxwell-Boltzmann velocities v = sqrt(kT/m) z from the seed (Philox tag 1,
 * step 0; the rigid body draws with particle index n_atoms and its mass). */
hd_status hd_init_velocities(hd_ctx *ctx, int32_t sys);
/* Replace positions: mobile and fixed atoms are copied; the rigid body moves
 * by the minimum-image displacement of its first atom and its atoms are
 * re-placed at X_R + c_i. */
hd_status hd_set_positions(hd_ctx *ctx, int32_t sys, const double *pos);
/* Replace velocities: mobile atoms copied, fixed atoms zero, the rigid body
 * takes the mean of its atoms' velocities. */
hd_status hd_set_velocities(hd_ctx *ctx, int32_t sys, const double *vel);

/* Lay out the batch in device memory, upload it and evaluate forces at the
 * initial positions. */
hd_status hd_finalize(hd_ctx *ctx);

/* Advance every system by n_steps BAOAB steps (asynchronous on the context
 * stream).  A system whose energy becomes non-finite, or one of whose atoms
 * feels a force above 1e6 eps/sigma (or a non-finite one), is frozen
 * (HD_FLAG_UNSTABLE) while the others continue; hd_set_positions or
 * hd_set_state revive it.  The energies read after the call are those of
 * the last step (the grid kernels evaluate the pair energy only on the last
 * step of each replayed sequence of steps, the call's last among them, and
 * test stability by the forces elsewhere); the LDS-resident kernel
 * evaluates the pair energy on that step only, so a system frozen earlier
 * within a launch reports a pair
 * energy of zero for its last step: its e_pot is the
 * drive energy alone and stays finite (test the flags, not isfinite(e_pot)).
 * A system frozen by an evaluation (hd_finalize, hd_compute) keeps that
 * evaluation's energies and its step count.  Returns HD_E_UNSTABLE when the
 * last hd_sync found every system frozen. */
hd_status hd_step(hd_ctx *ctx, int64_t n_steps);
/* Evaluate forces, energy, H u and the bias at the current positions without
 * stepping or advancing the clock; rebuilds every neighbour list. */
hd_status hd_compute(hd_ctx *ctx);
/* Wait for the context stream; returns HD_E_UNSTABLE if every system is
 * frozen. */
hd_status hd_sync(hd_ctx *ctx);

/* Host read-outs (synchronising).  out holds dim*n_atoms doubles. */
hd_status hd_read_forces(hd_ctx *ctx, int32_t sys, int32_t which, double *out);
hd_status hd_read_positions(hd_ctx *ctx, int32_t sys, double *out);
hd_status hd_read_velocities(hd_ctx *ctx, int32_t sys, double *out);
hd_status hd_read_scalars(hd_ctx *ctx, int32_t sys, hd_scalars *out);
/* The scalars of systems first .. first + count - 1 in one device-to-host
 * copy (out holds count entries; count 0 reads nothing).  HD_E_ARG for a
 * range outside the context's systems. */
hd_status hd_read_scalars_batch(hd_ctx *ctx, int32_t first, int32_t count, hd_scalars *out);
/* Device-to-device copy of a system's positions / forces into a caller
 * buffer of dim*n_atoms doubles (stream-ordered, not synchronising). */
hd_status hd_copy_positions_device(hd_ctx *ctx, int32_t sys, double *dev_out);
hd_status hd_copy_forces_device(hd_ctx *ctx, int32_t sys, int32_t which, double *dev_out);

/* Checkpoint of one system's run state: positions, velocities, the
 * reference r_O, the list build positions, the last total forces, the rigid
 * body, the step count, both clocks, the last scalars and the Nose-Hoover
 * chain's state.  The seed, the slider position and every parameter are not
 * part of it: they stay with the system the state is restored into, so a
 * state copied into several systems (the redistribution of Sec. 2.3)
 * continues there with each system's own noise stream and slider; when the
 * target's potential, drive or bias parameters differ from the source's,
 * its forces are re-evaluated before the next step, as after a parameter
 * change.  With buf == NULL, *bytes receives the size needed.  Philox is
 * counter based, so a state restored into the system it came from (or one
 * with the same seed and parameters) continues bit-identically. */
hd_status hd_get_state(hd_ctx *ctx, int32_t sys, void *buf, size_t *bytes);
hd_status hd_set_state(hd_ctx *ctx, int32_t sys, const void *buf, size_t bytes);

/* Zero-copy binding of a batch field to caller-owned device memory, for
 * example a torch tensor's storage (the boundary of Sec. 2.3's parallel
 * algorithm, where positions and forces feed other device code).  The batch
 * stores each field as float64 [3][ntot]: component k of atom i of system s
 * at k*ntot + offset(s) + i (hd_batch_layout gives offset and ntot; the
 * third row of a 2D system is unused).  sys must be HD_ALL_SYSTEMS.
 * field: HD_FIELD_POSITIONS, HD_FIELD_VELOCITIES, HD_FIELD_FORCES (total),
 * HD_FIELD_FORCES_LJ (LJ + drive), HD_FIELD_FORCES_BIAS or HD_FIELD_HU.
 * dev_ptr: 3*ntot doubles of device memory on the context's device, 8-byte
 * aligned, kept alive by the caller until it is unbound or the context is
 * destroyed.  The field's current contents are copied into it and from then
 * on every kernel reads and writes the field there; the caller may read it
 * between calls (stream-ordered on the context stream), and changes
 * positions or velocities only through hd_set_positions, hd_set_velocities
 * or hd_set_state.  dev_ptr == NULL unbinds: the contents are copied back
 * into the context's own storage.  After HD_OK the previous storage is no
 * longer used.  HD_E_STATE before hd_finalize; HD_E_ARG for another sys, an
 * unknown field, or a pointer that is not aligned device memory of the
 * context's device. */
#define HD_ALL_SYSTEMS (-1)
enum { HD_FIELD_POSITIONS = 0, HD_FIELD_VELOCITIES = 1, HD_FIELD_FORCES = 2, HD_FIELD_FORCES_LJ = 3,
       HD_FIELD_FORCES_BIAS = 4, HD_FIELD_HU = 5 };
hd_status hd_bind_device(hd_ctx *ctx, int32_t sys, int32_t field, void *dev_ptr);
/* Where system sys lives in the batch arrays: *offset = its first atom,
 * *ntot = atoms in the batch (after hd_finalize). */
hd_status hd_batch_layout(hd_ctx *ctx, int32_t sys, int64_t *offset, int64_t *ntot);

/* Neighbour pairs (i < j, system-local indices) of the current list, i.e.
 * pairs with r^2 < (rc + skin)^2 at the last build, without fixed-fixed and
 * rigid-rigid pairs.  Writes up to cap pairs into ij[2*k], ij[2*k+1] and the
 * total count into *n_pairs. */
hd_status hd_debug_pairs(hd_ctx *ctx, int32_t sys, int32_t *ij, int64_t cap, int64_t *n_pairs);

/* Number of systems, and the atom count / dimension of one. */
hd_status hd_system_info(hd_ctx *ctx, int32_t sys, int32_t *dim, int32_t *n_atoms);
int32_t hd_num_systems(const hd_ctx *ctx);

/* Launch shape of the schedule (after hd_finalize).  lds_resident: systems
 * that fit one workgroup run in the LDS-resident persistent kernel;
 * small_block: its workgroup size (256, 512 or 1024, one thread per atom,
 * raised to cover the largest system); persistent_large: the remaining
 * systems run on the one-workgroup global kernel (1) or on the grid kernels
 * (0); large_block: threads per grid tile or per workgroup of that kernel;
 * small_half_lists: under HD_FP32C the LDS-resident pair pass visits each
 * pair once and adds the partner's share with float64 LDS atomics (1), or
 * visits it from both atoms (0); always 0 under HD_FP64;
 * ms_per_step: the time hd_autotune measured for this shape (0 otherwise). */
typedef struct {
    int32_t lds_resident;
    int32_t small_block;
    int32_t persistent_large;
    int32_t large_block;
    int32_t small_half_lists;
    double ms_per_step;
} hd_schedule;

/* Current launch shape. */
hd_status hd_get_schedule(hd_ctx *ctx, hd_schedule *out);

/* Switch to a launch shape (after hd_finalize; for instance one that
 * hd_autotune chose earlier for the same kind of batch).  The state of every
 * system is kept; neighbour lists are rebuilt from their recorded build
 * positions, so the run continues bit for bit as a run that used this shape
 * from the start would.  HD_E_ARG for block sizes outside the ranges above,
 * HD_E_STATE under HD_EXEC_SEQUENTIAL. */
hd_status hd_set_schedule(hd_ctx *ctx, const hd_schedule *shape);

/* Autotuner (after hd_finalize, HD_EXEC_BATCHED or HD_EXEC_GRID): times every
 * candidate launch shape on the context's own batch and keeps the fastest.
 * Each candidate is rebuilt, warmed up, and timed with HIP events over runs
 * of 8, 32, 128, ... steps until one lasts at least min_ms milliseconds or
 * reaches max_steps steps (a candidate more than three times slower than the
 * best so far is dropped after its first run).  Every system's state is
 * checkpointed before and restored after each trial, so the tuning leaves
 * every system's state (positions, velocities, step, clocks) exactly where
 * it was, and the run continues as one that used the chosen shape from the
 * start.  The trials are written to trials[0..cap) (may be
 * NULL) and their count to *n_trials; the chosen shape is then current.
 * Returns HD_E_UNSTABLE if a trial froze every system (the state is restored
 * and the previous shape kept). */
hd_status hd_autotune(hd_ctx *ctx, double min_ms, int64_t max_steps, hd_schedule *trials, int32_t cap,
                      int32_t *n_trials);

/* Energy minimisation (the basin minimum r_O of eq. 7, and the quench-and-
 * compare transition check of the parallel slider-position algorithm, §2.3):
 * FIRE (Bitzek et al., PRL 97, 170201, 2006; dt_max = 10 dt, alpha_0 = 0.1,
 * f_inc = 1.1, f_dec = 0.5, f_alpha = 0.99, N_min = 5) on the unbiased
 * potential (LJ plus the drive at each system's slider position), from each
 * listed system's current positions, starting at rest.  Mobile atoms and the
 * rigid body move (semi-implicit Euler, first step dt); fixed atoms stay.
 * Converged when the largest force on a degree of freedom is below ftol
 * (iters 0: already at the start).  LDS-resident systems run the whole
 * quench in one launch of the LDS kernel (iterations and evaluations in
 * LDS); the others iterate grid kernels, evaluations and the FIRE step, the
 * convergence read back every 32 iterations.  Every system's run state (positions, velocities, forces, clock, lists) is
 * restored afterwards, so stepping continues exactly as without the call.
 *   systems[0..count): distinct system indices (after hd_finalize);
 *   mode HD_QUENCH_CHECK: max_disp[k] = the largest atom displacement
 *     (minimum image) of system k's minimum from its r_O -- a transition
 *     when above a threshold of the caller's choosing;
 *   mode HD_QUENCH_SET_REFERENCE: the minimum becomes the system's r_O;
 *     max_disp[k] = the largest displacement from the starting positions;
 *   iters[k] = iterations used, or -max_iters when not converged;
 *   x_min (may be NULL): host buffer of sum_k dim_k * n_k doubles, receiving
 *     each listed system's minimum ([dim][n], in list order).
 * HD_E_ARG for bad arguments (max_iters >= 1, ftol > 0), HD_E_STATE for a
 * system frozen as unstable.  Allocates its own device scratch. */
#define HD_QUENCH_CHECK 0
#define HD_QUENCH_SET_REFERENCE 1
hd_status hd_quench(hd_ctx *ctx, const int32_t *systems, int32_t count, double ftol, int64_t max_iters,
                    int32_t mode, int64_t *iters, double *max_disp, double *x_min);

/* hd_quench without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same minimisation, arguments, results and error
 * codes as hd_quench, but the FIRE state, the system list and the reduction
 * partials live in a static device array of 1 MiB that each device holds
 * for the life of the process, and the read-out arrays (LJ and bias forces,
 * H u) are evaluated again at the restored positions
 * instead of being saved.  It needs 4 count and 64 count bytes, each
 * rounded up to a multiple of 256, plus 32 count ceil(n_max / 2048) bytes,
 * n_max the largest listed system; HD_E_ARG (with the sizes in the message)
 * beyond 1 MiB.  Calls on one device share
 * the array: calls that overlap on one device (several contexts on several
 * host threads) race.  Host memory is still used for the checkpoints of
 * every system. */
hd_status hd_quench_noalloc(hd_ctx *ctx, const int32_t *systems, int32_t count, double ftol, int64_t max_iters,
                            int32_t mode, int64_t *iters, double *max_disp, double *x_min);

/* Lowest eigenvalue of the Hessian of the unbiased potential over system
 * sys's degrees of freedom (its mobile atoms' coordinates and the rigid
 * body's), the variable of the eigenvalue bias (§2.2, eq. 15), at the
 * current positions: Lanczos with full reorthogonalisation from a random
 * start (seed), each Hessian-vector product one evaluation of the pair pass's
 * H u with r_O moved so that u is the Lanczos vector; the rigid body's row
 * collects its atoms' rows (and the drive's Hessian).  Stops when the
 * smallest Ritz value changes by less than tol (relative, at least absolute
 * tol) or after max_iter products (at most the number of degrees of
 * freedom).  *eps = that Ritz value; *iters = products used (negative: not
 * converged); mode (may be NULL): host [dim][n] doubles receiving its Ritz
 * vector (unit norm over the degrees of freedom; fixed atoms 0, rigid atoms
 * the body's component).  The run state is restored afterwards.  Float32
 * contexts give H u in float32 (eigenvalue to ~1e-6). */
hd_status hd_min_mode(hd_ctx *ctx, int32_t sys, int32_t max_iter, double tol, uint64_t seed, double *eps,
                      int32_t *iters, double *mode);

/* Gradient of the lowest eigenvalue eps over the degrees of freedom, what
 * the eigenvalue bias of eq. 13 and eq. 15 differentiates: for a simple
 * eigenvalue with unit eigenvector q, d eps = q^T dH q, the third
 * derivatives of V contracted twice with the atom displacement w = P q.
 * One GPU evaluation of the pair pass with u = w that also accumulates
 * T[u,u] (the kernels of the curvature bias), projected by P^T.
 * mode: hd_min_mode's output layout, [dim][n] host doubles (read: mobile
 * atoms and the first rigid atom; normalised here over the degrees of
 * freedom).  grad: [dim][n] host doubles, written: each mobile atom's
 * derivative, on every rigid atom the rigid body's (the sum over its atoms),
 * fixed atoms 0.  The run state is restored afterwards.  HD_E_STATE before
 * hd_finalize or when the system does not run on the grid kernels
 * (HD_EXEC_GRID puts every system there); HD_E_ARG for a zero mode. */
hd_status hd_min_mode_gradient(hd_ctx *ctx, int32_t sys, const double *mode, double *grad);

/* Per-kernel timing of the last hd_step, measured with HIP events on the
 * context stream: total milliseconds and launches. */
hd_status hd_last_step_timing(hd_ctx *ctx, double *ms, int64_t *launches);

const char *hd_last_error(const hd_ctx *ctx);
void hd_destroy(hd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HD_H */
