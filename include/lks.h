/*
 * lks.h -- C ABI of the MI355X (gfx950) library for the unsteady Lattice
 * Kinetic Scheme with a rigidly moving Brinkman body and its adjoint.
 *
 * Paper: Tanabe, Yaji, Ushijima, "4D topology optimization of moving rigid
 * bodies in fluid flows".  The library computes, on one GPU:
 *   - the motion prelude: temporal filter, bounds and time derivatives of the
 *     motion design variables (Sec. 2.4, Eqs. chi_filtered, x_g, u_g,
 *     psi_filtered, theta, omega);
 *   - kappa_ref(gamma) on the design grid (Sec. 2.3, Eq. kappa_ref);
 *   - the per-step rigid transform and design -> analysis transfer of kappa and
 *     the body velocity (Sec. 2.3, Eqs. kappa, u_s, rigid_body_position,
 *     rigid_body_velocity);
 *   - the LKS step: velocity gradient, Inamuro equilibrium, neighbour gather
 *     and Brinkman correction (Sec. 2.2, Eqs. p_tmp, u_tmp, p, u), with wall
 *     nodes whose p and u are imposed;
 *   - the objective J1 = E - phi V over a target box (Sec. 2.6, Eq. objective1);
 *   - the exact discrete adjoint of that march and the shape / motion
 *     sensitivities (Sec. 2.5, Eqs. dJdgamma, dJdchi, dJdpsi and the
 *     multipliers u~^G, omega~), with checkpoint-every-K recomputation.
 *
 * Units: lattice units (dx = dt = 1).  kappa is the lattice product dx*kappa.
 *
 * Layouts (all row-major, x fastest):
 *   - analysis state: planes [d+1][N] of the state type (float when
 *     precision = LKS_FP32, double when LKS_FP64).  Plane 0 holds the
 *     pressure OFFSET p - 1/3, planes 1..d the velocity components.  The
 *     pressure of a wall node is defined by the wall rule (a copy of its
 *     nearest interior node); states returned by the library satisfy it.
 *   - adjoint state: planes [d+1][N] of the state type, dJ/dp then dJ/du.
 *   - gamma: [m2][m1][m0] doubles in [0,1] (inner design points, no margin).
 *   - chi: [nt][3] doubles (component z ignored when d = 2); psi: [nt] doubles,
 *     or [nt][3] with rot = LKS_ROT_EULER.
 *   - motion table: [nt][8] doubles per step: xg[3], ug[3], theta, omega; with
 *     rot = LKS_ROT_EULER [nt][12]: xg[3], ug[3], th[3], om[3].
 *   - kappa_ref: [D2][D1][D0] of the state type, D = m + 2 * margin.
 *
 * Ownership: every buffer belongs to the caller.  The library never allocates
 * device memory; the caller provides a workspace of the size reported by
 * lks_plan_create and keeps it alive between lks_forward and lks_adjoint.
 * A plan owns only host objects.
 *
 * Calls are asynchronous on `stream` unless noted.  Pointers are DEVICE
 * pointers unless marked (host).  Every call returns an lks_status; on error
 * lks_last_error() returns a message (thread-local).  LKS_EDOMAIN and
 * LKS_EUNSTABLE are found by a short device-to-host read inside the call
 * (the call then synchronises `stream`).
 */
#ifndef LKS_H
#define LKS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LKS_OK = 0,
  LKS_EINVAL = 1,     /* bad argument or unsupported problem */
  LKS_EDOMAIN = 2,    /* the body's kernel support reaches a wall node */
  LKS_EUNSTABLE = 3,  /* non-finite or |u| >= 0.5 seen during the march */
  LKS_EHIP = 4        /* a HIP runtime call failed */
} lks_status;

enum { LKS_FP32 = 0, LKS_FP64 = 1 };

typedef struct lks_problem {
  int32_t d;               /* 2 -> D2Q9, 3 -> D3Q15 */
  int32_t precision;       /* state type: LKS_FP32 or LKS_FP64; sums are FP64 */
  int32_t n[3];            /* analysis nodes per axis incl. wall nodes; n[2] = 1 in 2D */
  int32_t bc[3];           /* per axis: 0 periodic, 1 wall nodes at index 0 and n-1
                              (3D: z must be periodic) */
  double u_wall[3][2][3];  /* imposed wall velocity [axis][lo, hi][component];
                              a node on several walls takes the highest axis' value */
  double nu;               /* lattice viscosity; A = 3/4 - 9 nu / 2 (Sec. 2.2) */
  double kappa_max, q;     /* Eq. kappa_ref parameters */
  int32_t m[3];            /* inner design points per axis */
  int32_t margin;          /* fluid margin width around the design grid (>= 0) */
  double xg_min[3], xg_max[3]; /* admissible centre range (Eq. x_g) */
  double th_min, th_max;   /* admissible rotation range about z (Eq. theta) */
  int32_t nt;              /* time steps */
  int32_t r_t, r_w;        /* temporal filter radii in steps (>= 1; 1 = identity) */
  int32_t tgt_lo[3], tgt_hi[3]; /* objective target box [lo, hi) */
  double ndir[3];          /* flow direction n of J1 */
  double phi;              /* J1 = E - phi V */
  int32_t ckpt_k;          /* checkpoint interval K (1..nt); 0 means nt */
  int32_t body_tape;       /* body fields (kappa, u_s) kept for the reverse sweep:
                              1 every step's, written by the forward march, so the
                              segment recompute skips the map; -1 only the segment
                              being reversed (the recompute maps again); 0 the
                              former when it takes at most LKS_BODY_TAPE_AUTO_MAX
                              bytes, else the latter.  Results are the same. */
  int32_t scheme;          /* reverse sweep of lks_adjoint: LKS_ADJ_EXACT, the exact
                              discrete adjoint of the march (the true gradient), or
                              LKS_ADJ_ALKS, the paper's adjoint lattice kinetic
                              scheme (Sec. 2.5), an approximation of it */
  int32_t objective;       /* LKS_OBJ_J1: Eq. objective1 (flow through the target
                              box, target box, ndir and phi used); LKS_OBJ_J2:
                              Eq. objective2 (2D only), the propulsive force F_L,
                              drag work F_D and torque work T of the force density
                              kappa_ref (u_ref - u_S_ref) on the design points,
                              J2 = F_L + w_d F_D + w_t T.  Inside the body this
                              density is a small difference of nearly equal
                              velocities, so with an FP32 state the 2D transfer,
                              its transpose and the pull-back u_ref take their
                              weights and sums in FP64 (J2 then agrees with the
                              FP64 state to about 2e-6 on the oar workload) */
  double w_d, w_t;         /* J2 weights of F_D and T */
  double l_m;              /* J2 moment arm in T's normalisation 2 pi l_m (> 0);
                              F_D is normalised by xg_max[1] - xg_min[1] (> 0) */
  int32_t rot;             /* LKS_ROT_Z: one rotation angle, about z (Sec. 2.4, Eqs.
                              psi_filtered, theta, omega); LKS_ROT_EULER (3D only):
                              three angles th1, th2, th3 about x, y, z, each from its
                              own design series through the same filter, with
                              R = Rz(th3) Ry(th2) Rx(th1) in Eq. rigid_body_position
                              and u_ref = sum_k om_k (dR/dth_k) r + u^G (the Euler
                              angles the closing remark of Sec. 2.4 names).  psi and
                              dJ_dpsi are then [nt][3], motion rows hold 12 values */
  double tilt_min[2], tilt_max[2]; /* LKS_ROT_EULER: ranges of th1 (about x) and th2
                              (about y); th3 (about z) keeps th_min, th_max */
} lks_problem;

#define LKS_ADJ_EXACT 0
#define LKS_ADJ_ALKS 1
#define LKS_OBJ_J1 0
#define LKS_OBJ_J2 1
#define LKS_ROT_Z 0
#define LKS_ROT_EULER 1

#define LKS_BODY_TAPE_AUTO_MAX (96ull << 30)

typedef struct lks_plan lks_plan;

/* Validate `prob` (host) and build a plan.  *workspace_bytes receives the
 * device workspace size the caller must allocate (256-byte aligned).
 * Errors: LKS_EINVAL for inconsistent sizes (e.g. a wall axis with fewer
 * than 4 nodes, design grid larger than a periodic extent) and for grids
 * above 2^29 nodes, or in 3D whose (p, u) state reaches 4 GiB (2^28 nodes in
 * FP32, 2^27 in FP64). */
lks_status lks_plan_create(const lks_problem* prob, lks_plan** out, size_t* workspace_bytes);
lks_status lks_plan_destroy(lks_plan* plan);

/* Graph replay of the time loops (default on).  With it on, lks_forward and
 * lks_adjoint capture their time loop into a hipGraph on first use for a
 * workspace (on a private stream of the plan) and replay it afterwards;
 * per-step data are read from device tables, so replays see new inputs.
 * While lks_profile_enable is on, loops run eagerly (per-launch events). */
lks_status lks_plan_set_graphs(lks_plan* plan, int32_t on);

/* Tuning: z planes per block segment of the 3D step kernels (0 = automatic,
 * sized to fill every CU).  Smaller values mean more blocks and more halo
 * planes re-read per segment.  Ignored in 2D. */
lks_status lks_plan_set_zseg(lks_plan* plan, int32_t zseg);

/* Forward march (Algorithm 1, state loop; Sec. 2.2-2.4, 2.6).
 * state0: initial state (nullable: p = 1/3, u = 0 everywhere; the wall
 *   nodes' given p is used for the first step as is).
 * state_final: receives the state after nt steps (nullable); with state0
 *   this supports the periodic approximation of Sec. 3.3.
 * J_out: 3 doubles: (J, E, V) for J1, (J2, F_L, F_D) for J2.
 * Leaves motion, kappa_ref, checkpoints and E in the workspace for
 * lks_adjoint.  Returns LKS_EDOMAIN (before the march) if an inner design
 * point's kernel support reaches a wall node at some step, LKS_EUNSTABLE if
 * the march blew up. */
lks_status lks_forward(lks_plan* plan, const double* gamma, const double* chi,
                       const double* psi, const void* state0, void* state_final,
                       void* workspace, double* J_out, hipStream_t stream);

/* Reverse sweep of the forward march with the same inputs (Sec. 2.5): the
 * exact discrete adjoint, or with scheme = LKS_ADJ_ALKS the paper's adjoint
 * lattice kinetic scheme (adjoint equilibrium, Eqs. ap_tmp .. as, and the
 * sensitivities of Eqs. dJdgamma, dJdchi, dJdpsi), which approximates it.
 * dJ: 1 double, the seed (dJ/dJ; usually 1).
 * adj_terminal: adjoint state added at step nt (nullable; periodic
 *   approximation of Sec. 3.3).
 * adj_initial: receives dJ/d(state0) (nullable).
 *   Both are [d+1][N] (state type) with the exact adjoint.  With the ALKS
 *   they are [(d+1) + 1 + d + d(d+1)/2][N]: the scheme's estimate of
 *   dJ/d(state0) ([d+1][N]), then the ALKS state itself, p~ [N], u~ [d][N]
 *   and the symmetric components of s~ ((xx, yy, xy) in 2D, (xx, yy, zz,
 *   xy, xz, yz) in 3D), in the paper's sign.  adj_terminal reads only that
 *   state: as Algorithm 1's periodic approximation prescribes, p~(t1) =
 *   p~(t0) of an earlier run and likewise u~ and s~; it takes the place of
 *   the moments of the last level (before that level's sources), whose
 *   adjoint equilibrium is then formed with this run's own velocity at t1.
 *   A run's adj_initial can be passed as the next run's adj_terminal.
 * dJ_dgamma [m2][m1][m0], dJ_dchi [nt][3], dJ_dpsi [nt] ([nt][3] with
 *   LKS_ROT_EULER): gradients of J (the paper maximises J; these are +grad J).
 * Recomputes each K-step segment from its checkpoint. */
lks_status lks_adjoint(lks_plan* plan, const double* gamma, const double* chi,
                       const double* psi, void* workspace, const double* dJ,
                       const void* adj_terminal, void* adj_initial, double* dJ_dgamma,
                       double* dJ_dchi, double* dJ_dpsi, hipStream_t stream);

/* Design prelude of the optimisation loop (Sec. 3.1, Algorithm 1), for a
 * caller's optimiser: gamma [m2][m1][m0] (the design variables, device)
 * -> the density filter of radius `radius` (Eq. filtering: cone weights
 * (R - |x_i - x_j|) / R on the inner design grid, spacing 1, normalised
 * per point) -> the Heaviside projection with steepness beta and threshold
 * eta (Eq. projection; beta <= 0 skips it) -> gamma_phys [M] (device), the
 * field lks_forward takes as gamma.  FP64.  LKS_EINVAL unless
 * 0 < radius <= 64 and 0 <= eta <= 1. */
lks_status lks_design_filter(lks_plan* plan, const double* gamma, double radius, double beta,
                             double eta, double* gamma_phys, hipStream_t stream);

/* Chain rule of lks_design_filter: dJ_dphys [M] (e.g. lks_adjoint's
 * dJ_dgamma) -> dJ_dgamma [M] w.r.t. the design variables.  work: M
 * doubles of device scratch owned by the caller. */
lks_status lks_design_filter_adjoint(lks_plan* plan, const double* gamma, double radius,
                                     double beta, double eta, const double* dJ_dphys,
                                     double* work, double* dJ_dgamma, hipStream_t stream);

/* lks_design_filter_adjoint for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid
 * allocation): the same chain rule with its M-double scratch in a fixed
 * device array of the library (LKS_NOALLOC_MAX_POINTS doubles, 16 MiB, held
 * on every device the library runs on until the process ends) instead of a
 * caller-owned `work`.  Allocates nothing.  Every call on a device shares that
 * device's array, so calls that overlap on one device race; calls in order
 * on one stream are safe.  LKS_EINVAL when the plan has more than
 * LKS_NOALLOC_MAX_POINTS inner design points, and as lks_design_filter_adjoint. */
#define LKS_NOALLOC_MAX_POINTS (1ll << 21)
lks_status lks_design_filter_adjoint_noalloc(lks_plan* plan, const double* gamma, double radius,
                                             double beta, double eta, const double* dJ_dphys,
                                             double* dJ_dgamma, hipStream_t stream);

/* Constraint functionals of Sec. 2.6 and their gradients (device arrays):
 *   G_out[0] = G1 = sum(gamma_phys) / (vmax M) - 1      (Eq. constraint1)
 *   G_out[1] = G2 = sum(1 - gamma_phys) / (vmax M) - 1  (Eq. constraint2)
 *   G_out[2] = G3 = (sum_n |omega_n / omega_max|^p)^(1/p) - 1 over the steps
 *              n = 1..nt, omega from chi, psi by the motion prelude
 *              (Eq. constraint3).
 * dG1, dG2 [M] w.r.t. gamma_phys, dG3_dpsi [nt] (each nullable; G3 does not
 * depend on chi or gamma).  workspace: the plan's; this call writes only a
 * motion table of its own and the epilogue's scratch (which every
 * lks_sensitivities call rebuilds), so what lks_forward and lks_adjoint
 * leave for later calls stays intact.  LKS_EINVAL unless vmax > 0,
 * omega_max > 0 and p >= 1. */
lks_status lks_constraints(lks_plan* plan, void* workspace, const double* gamma_phys,
                           const double* chi, const double* psi, double vmax, double omega_max,
                           double p_omega, double* G_out, double* dG1, double* dG2,
                           double* dG3_dpsi, hipStream_t stream);

/* ---- the optimisation loop (Algorithm 1, Secs. 3.2-3.4) ---- */

/* What the driver hands the caller's optimiser step after each iteration's
 * sensitivities (device pointers unless marked). */
typedef struct lks_opt_state {
  int32_t level;           /* continuation level l, 0-based */
  int32_t iter;            /* iteration k within the level, 0-based */
  int32_t total;           /* iterations so far, this one included */
  double beta;             /* projection steepness of the level */
  double J;                /* (host) objective of this iteration */
  double G[3];             /* (host) G1, G2, G3 of this iteration (Sec. 2.6) */
  double* gamma;           /* design variables [M], [nt][3], [nt] or [nt][3]: */
  double* chi;             /*   the caller's arrays, to be updated in place */
  double* psi;
  const double* dJ_dgamma; /* [M]: gradient of J w.r.t. gamma itself (through */
  const double* dJ_dchi;   /*   filter and projection); [nt][3]; as psi */
  const double* dJ_dpsi;
  const double* dG1_dgamma; /* [M] each: G1, G2 w.r.t. gamma (filter chain applied) */
  const double* dG2_dgamma;
  const double* dG3_dpsi;  /* as psi (G3 depends on psi only) */
} lks_opt_state;

/* The optimiser step (MMA in the paper, Sec. 3.4; the caller's choice):
 * reads the state and writes new design variables into st->gamma, st->chi,
 * st->psi on `stream`.  Returns 0 to go on, anything else to stop the loop. */
typedef int32_t (*lks_update_fn)(void* user, const lks_opt_state* st, hipStream_t stream);

typedef struct lks_opt_options {
  int32_t n_cont;          /* continuation levels N_cont (Sec. 3.2) */
  const double* beta;      /* (host) [n_cont]: beta of each level, e.g. 1, 2, 4, ..., 32 */
  int32_t n_opt;           /* most iterations per level N_opt */
  double radius, eta;      /* density filter radius, projection threshold (Sec. 3.1) */
  double tol;              /* stopping criterion |J^(k+1) - J^k| / |J^k| <= tol (1e-6) */
  double vmax, omega_max, p_omega; /* constraint parameters (Eqs. constraint1..3) */
  int32_t g_active;        /* bit j-1: G_j <= 0 is required before a level may stop */
  int32_t periodic;        /* 1: periodic approximation (Sec. 3.3): each march starts
                              from the previous march's final state and each reverse
                              sweep from the previous sweep's adj_initial */
} lks_opt_options;

typedef struct lks_opt_result {
  int32_t iterations;      /* forward marches run */
  int32_t levels;          /* continuation levels entered */
  int32_t stopped;         /* 0 ran out of levels; 1 the callback stopped the loop */
  double J_last;           /* objective of the last march */
} lks_opt_result;

/* Device scratch lks_optimize needs (bytes, 256-aligned). */
size_t lks_optimize_scratch_bytes(const lks_plan* plan);

/* Algorithm 1: for each continuation level l (beta = beta[l]) and iteration
 * k < n_opt: filter and project gamma (lks_design_filter), march
 * (lks_forward; periodic: from the previous final state), J and G1-G3
 * (lks_constraints); the level ends when k > 0 and
 * |J^k - J^(k-1)| / |J^(k-1)| <= tol with every active G_j <= 0 (Sec. 3.2:
 * J of consecutive iterations of the level); otherwise the reverse sweep
 * (lks_adjoint; periodic: from the previous sweep's adj_initial), the chain
 * rule back to gamma (lks_design_filter_adjoint) for J, G1 and G2, and the
 * caller's update.  gamma, chi, psi: device, read and updated in place.
 * history (host, nullable): [n_cont * n_opt][4] rows (J, G1, G2, G3) of the
 * iterations run, in order.  The call synchronises `stream` once per
 * iteration (J and G go to the host).  Errors of the stages are returned as
 * they occur. */
lks_status lks_optimize(lks_plan* plan, void* workspace, const lks_opt_options* opt,
                        double* gamma, double* chi, double* psi, void* scratch,
                        lks_update_fn update, void* user, double* history,
                        lks_opt_result* result, hipStream_t stream);

/* Design -> analysis transfer for one time step (Sec. 2.3, Eqs. kappa, u_s):
 * kappa_ref [D2][D1][D0] (state type), motion8 = one motion row, (xg[3],
 * ug[3], theta, omega) doubles (12 with LKS_ROT_EULER: xg, ug, th[3], om[3])
 * -> kappa [N] and u_s [d][N] (state type).  Wall nodes receive 0.
 * workspace: the plan's workspace (3D keeps a z-fastest copy of kappa_ref
 * there; the checkpoints left by lks_forward are not touched and a later
 * lks_adjoint rebuilds its copy).  Reads motion8 back to
 * the host (synchronises `stream`).  Returns LKS_EINVAL if the body's
 * support does not fit a periodic extent. */
lks_status lks_map_design_to_grid(lks_plan* plan, const void* kappa_ref, const double* motion8,
                                  void* kappa, void* u_s, void* workspace, hipStream_t stream);

/* Sensitivity epilogue (Algorithm 1, "compute design sensitivity" and
 * "unfilter"): from the raw accumulators left in the workspace by
 * lks_adjoint (dJ/dkappa_ref per design point and the per-step motion
 * partials) to dJ/dgamma, dJ/dchi, dJ/dpsi, through Eq. kappa_ref, the
 * time differences of Eqs. u_g and omega, the bound maps and the transposed
 * temporal filter.  lks_adjoint calls it; exported for reuse and testing. */
lks_status lks_sensitivities(lks_plan* plan, const double* gamma, const void* workspace,
                             double* dJ_dgamma, double* dJ_dchi, double* dJ_dpsi,
                             hipStream_t stream);

/* ---- single-stage entry points (used by tests; same kernels as above) ---- */

/* Motion prelude only: chi, psi -> motion [nt][8] doubles (Sec. 2.4), or
 * [nt][12] with LKS_ROT_EULER. */
lks_status lks_motion(lks_plan* plan, const double* chi, const double* psi, double* motion,
                      hipStream_t stream);

/* kappa_ref(gamma) incl. margin (Eq. kappa_ref), state type. */
lks_status lks_kappa_ref(lks_plan* plan, const double* gamma, void* kappa_ref,
                         hipStream_t stream);

/* One LKS step (Sec. 2.2) with given body fields kappa [N], u_s [d][N]
 * (state type): state_in -> state_out (both [d+1][N]; must not alias).
 * state_in's wall-node pressures are used as given. */
lks_status lks_step(lks_plan* plan, const void* state_in, const void* kappa, const void* u_s,
                    void* state_out, hipStream_t stream);

/* Transpose of lks_step: lam = dJ/d(state_out) -> lam_prev = dJ/d(state_in),
 * kbar = dJ/dkappa [N], usbar = dJ/du_s [d][N] (state type).  Always the
 * exact transpose, whatever the plan's scheme. */
lks_status lks_step_adjoint(lks_plan* plan, const void* state_in, const void* state_out,
                            const void* kappa, const void* u_s, const void* lam,
                            void* lam_prev, void* kbar, void* usbar, hipStream_t stream);

/* Transpose of lks_map_design_to_grid at one step: kbar [N], usbar [d][N]
 * (state type) -> kref_bar [Mtot] doubles (OVERWRITTEN) and motion_bar8
 * (first W doubles, W = 8 or 12 the motion row width: the partials of the
 * row's entries, xg_bar[3], ug_bar[3], then the angles' and rates'; the
 * buffer must hold W * (lks_map_adjoint_blocks(plan) + 1) doubles, the rest
 * is scratch for the fixed-order block reduction). */
lks_status lks_map_adjoint(lks_plan* plan, const void* kappa_ref, const double* motion8,
                           const void* kbar, const void* usbar, double* kref_bar,
                           double* motion_bar8, hipStream_t stream);

/* ---- batching: independent instances in one captured graph ---- */

/* Runs forward + adjoint for `count` independent problems (a parameter
 * study: the instances may differ in every lks_problem field) as one hipGraph
 * launched on `stream`.  2D J1 instances with a common step count, checkpoint
 * interval, precision, body-tape mode and adjoint scheme share every launch:
 * each kernel runs once per step for up to 16 of them, instance k owning a
 * block range.  Other mixes run as parallel branches of the graph, so their
 * kernels may run concurrently.
 *   plans, gamma, chi, psi, workspace, J_out, dJ_dgamma, dJ_dchi, dJ_dpsi:
 *     (host) arrays of `count` entries, each entry as for lks_forward /
 *     lks_adjoint of that instance (device pointers, caller-owned).  Plans and
 *     workspaces must be distinct.  Every instance starts from the rest state
 *     (p = 1/3, u = 0).
 *   dJ: device array of `count` objective seeds, or NULL for 1 each.
 * The per-instance preludes (with their LKS_EDOMAIN checks) run eagerly
 * first; the graph is captured on the first call and replayed while the
 * pointer tables are unchanged (it is kept by plans[0]).  The call
 * synchronises `stream` at its end and returns LKS_EUNSTABLE if any instance
 * became unstable; lks_last_error names the instance.  After the call each
 * workspace holds its instance's forward data as after lks_forward. */
lks_status lks_batch_run(int32_t count, lks_plan* const* plans, const double* const* gamma,
                         const double* const* chi, const double* const* psi,
                         void* const* workspace, double* const* J_out, const double* dJ,
                         double* const* dJ_dgamma, double* const* dJ_dchi,
                         double* const* dJ_dpsi, hipStream_t stream);

/* Number of per-block partial slots the stand-alone map transpose uses:
 * motion_bar8 of lks_map_adjoint must hold W * (blocks + 1) doubles (W = 8,
 * or 12 with LKS_ROT_EULER). */
int32_t lks_map_adjoint_blocks(lks_plan* plan);

/* ---- introspection ---- */

/* Per-kernel-class HIP event timing of the calls made while enabled.
 * lks_profile_enable(1) resets and enables; lks_profile_read fills up to
 * `cap` entries (host arrays) after synchronising the recorded streams and
 * returns the number of classes. */
lks_status lks_profile_enable(int32_t on);
int32_t lks_profile_read(const char** names, double* total_ms, int64_t* launches, int32_t cap);

const char* lks_last_error(void);

/* SHA-256 (hex) of the sources the library was built from, as computed by
 * the build; "unknown" for a build that did not supply it.  The Python
 * binding refuses a library whose digest differs from its sources. */
const char* lks_source_digest(void);

#ifdef __cplusplus
}
#endif
#endif
