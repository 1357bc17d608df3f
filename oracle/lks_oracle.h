/*
 * lks_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU reference of the Lattice Kinetic Scheme
 * (LKS) time march with a rigidly moving Brinkman body, the objectives J1 and
 * J2, the exact discrete adjoint of that march and the paper's ALKS (shape and
 * motion sensitivities), and the optimiser-side filter, projection and
 * constraints.
 * It exists to check the GPU library; only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no source with the
 * GPU library.
 *
 * Paper: Tanabe, Yaji, Ushijima, "4D topology optimization of moving rigid
 * bodies in fluid flows".  Sections cited: 2.2 (LKS), 2.3 (grid separation),
 * 2.4 (motion representation), 2.5 (sensitivities), 2.6 (objectives and
 * constraints), 3.1 (filter and projection).
 *
 * Conventions (lattice units, dx = dt = 1):
 *   - analysis fields are stored as planes [d+1][N]: plane 0 is the pressure p
 *     itself, planes 1..d the velocity components; x is fastest, then y, z.
 *   - motion table per time step n = 1..nt (row n-1): xg[3], ug[3], theta, omega
 *     (8 values); with rot = 1: xg[3], ug[3], th[3], om[3] (12 values), and
 *     psi, dJ/dpsi are [nt][3] instead of [nt]; the motion partials likewise.
 *   - design grid (incl. margin) is [Dz][Dy][Dx], Dx = m[0] + 2*margin, ...;
 *     gamma covers only the inner m[0] x m[1] x m[2] block, margin gamma = 0.
 * All functions return 0 on success and a negative value on bad arguments.
 */
#ifndef LKS_ORACLE_H
#define LKS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_problem {
  int32_t d;               /* 2 -> D2Q9, 3 -> D3Q15 */
  int32_t n[3];            /* analysis nodes per axis (n[2] = 1 when d = 2) */
  int32_t bc[3];           /* per axis: 0 periodic, 1 wall nodes at both ends */
  double u_wall[3][2][3];  /* wall velocity [axis][lo, hi][component] */
  double dp_seam[3];       /* pressure drop across a periodic axis (test mode) */
  double nu;               /* lattice kinematic viscosity */
  double kappa_max, q;     /* Brinkman interpolation parameters (lattice units) */
  int32_t m[3];            /* design points per axis, margin excluded */
  int32_t margin;          /* margin width in design points */
  double xg_min[3], xg_max[3]; /* admissible centre range per axis */
  double th_min, th_max;   /* admissible rotation range (about z) */
  int32_t nt, r_t, r_w;    /* time steps, temporal filter radii (steps) */
  int32_t tgt_lo[3], tgt_hi[3]; /* objective target box [lo, hi) */
  double ndir[3];          /* flow direction n */
  double phi;              /* J1 = E - phi * V */
  int32_t objective;       /* 0: J1 (Eq. objective1); 1: J2 (Eq. objective2, 2D) */
  double w_d, w_t, l_m;    /* J2 weights w_D, w_T and moment arm l_m */
  int32_t rot;             /* 0: one angle about z (Eqs. psi_filtered, theta, omega);
                              1 (3D only): three angles, R = Rz(th3) Ry(th2) Rx(th1),
                              the Euler-angle extension closing Sec. 2.4 */
  double tilt_min[2], tilt_max[2]; /* rot = 1: ranges of th1 (about x), th2 (about y);
                                      th3 (about z) keeps th_min, th_max */
} orc_problem;

/* Motion prelude (Sec. 2.4): chi [nt][3], psi [nt] -> motion [nt][8]. */
int orc_motion(const orc_problem* p, const double* chi, const double* psi, double* motion);

/* Brinkman coefficient on the design grid incl. margin (Eq. kappa_ref). */
int orc_kappa_ref(const orc_problem* p, const double* gamma, double* kappa_ref);

/* Design -> analysis transfer for one time step (Eqs. kappa, u_s, rigid motion):
 * kappa [N], us [d][N].  Wall nodes receive 0. */
int orc_map(const orc_problem* p, const double* kappa_ref, const double* motion8,
            double* kappa, double* us);

/* Transpose of orc_map at one step: given dJ/dkappa [N] and dJ/dus [d][N],
 * ADD dJ/dkappa_ref into kref_bar [Mtot] and WRITE the step's motion partials
 * motion_bar8 = (xg_bar[3], ug_bar[3], theta_bar, omega_bar). */
int orc_map_adjoint(const orc_problem* p, const double* kappa_ref, const double* motion8,
                    const double* kbar, const double* usbar, double* kref_bar,
                    double* motion_bar8);

/* One LKS step (Sec. 2.2) from state_in to state_out with given body fields. */
int orc_step(const orc_problem* p, const double* state_in, const double* kappa,
             const double* us, double* state_out);

/* Transpose of orc_step.  lam = dJ/d(state_out) (total), state_in/state_out as
 * in orc_step.  Writes lam_prev = dJ/d(state_in) through this step,
 * kbar = dJ/dkappa, usbar = dJ/dus. */
int orc_step_adjoint(const orc_problem* p, const double* state_in, const double* state_out,
                     const double* kappa, const double* us, const double* lam,
                     double* lam_prev, double* kbar, double* usbar);

/* Full forward march.  state0 nullable (p = 1/3, u = 0); state_final, traj
 * nullable; traj receives [(nt+1)][d+1][N].  J_out = (J, E, V) for J1 and
 * (J, F_L, F_D) for J2. */
int orc_forward(const orc_problem* p, const double* gamma, const double* chi,
                const double* psi, const double* state0, double* state_final,
                double* J_out, double* traj);

/* Full discrete adjoint.  dJ = seed scalar; adj_terminal nullable ([d+1][N],
 * added to dJ/d(state at nt)); adj_initial nullable (receives dJ/d(state0)).
 * kref_bar [Mtot] and motion_bar [nt][8] nullable (raw accumulators). */
int orc_adjoint(const orc_problem* p, const double* gamma, const double* chi,
                const double* psi, const double* state0, double dJ,
                const double* adj_terminal, double* adj_initial, double* dJ_dgamma,
                double* dJ_dchi, double* dJ_dpsi, double* kref_bar, double* motion_bar);

/* Paper-literal ALKS backward (Sec. 2.5): the continuous-adjoint lattice
 * kinetic scheme with the adjoint equilibrium and Eqs. ap_tmp .. as, run from
 * the last step to the first, and the sensitivities of Eqs. dJdgamma, dJdchi,
 * dJdpsi.  Outputs as orc_adjoint.  adj_initial (nullable,
 * [(d+1) + 1 + d + d(d+1)/2][N]): the scheme's estimate of dJ/d(state0)
 * ([d+1][N]) followed by the ALKS state of level 0: p~ [N], u~ [d][N] and
 * the symmetric components of s~ (xx, yy, xy in 2D; xx, yy, zz, xy, xz, yz
 * in 3D).  adj_terminal (nullable, same layout; the first d+1 planes are not
 * read): the state carried from an earlier run's adj_initial for the
 * periodic approximation (Sec. 3.3, Algorithm 1), p~(t1) = p~(t0) of the
 * earlier run and likewise u~, s~; it stands for the moments of the last
 * level before that level's sources. */
int orc_alks_adjoint(const orc_problem* p, const double* gamma, const double* chi,
                     const double* psi, const double* state0, double dJ,
                     const double* adj_terminal, double* adj_initial, double* dJ_dgamma,
                     double* dJ_dchi, double* dJ_dpsi, double* kref_bar, double* motion_bar);

/* Vector of the adjoint equilibrium f~eq_i = p~ + c_i . V of one ALKS level
 * (Sec. 2.5): carry = (p~ [N], u~ [d][N], symmetric s~ [d(d+1)/2][N]) as in
 * the ALKS carried state, u [d][N] the level's velocity -> V [d][N],
 * V = 3 (u~ + 3 s~ u - p~ u) - A d_b (s~_ab + s~_ba). */
int orc_alks_vector(const orc_problem* p, const double* carry, const double* u, double* V);

/* Objective J2 (Eq. objective2) step sums of one state, unnormalised: with
 * f = kappa_ref (u_ref - u_S_ref) on the design points, sums3 receives
 * (sum f_1, u^G_2 sum f_2, omega sum (v_1 f_2 - v_2 f_1)), v = x_ref - x^G;
 * u [2][N] is the fluid velocity, motion8 the step's motion row.  2D only. */
int orc_j2_sums(const orc_problem* p, const double* kappa_ref, const double* motion8,
                const double* u, double* sums3);

/* One ALKS level without sources: multipliers (p~ [N], u~ [d][N], s~ [9][N],
 * s~_ab in plane 3a+b) of level t+1 and that level's velocity u [d][N] ->
 * the gathered moments p~*, u~*, s~* of level t (same layout). */
int orc_alks_gather(const orc_problem* p, const double* fields_next, const double* u_next,
                    double* fields_out);

/* Design prelude of the optimisation loop (Sec. 3.1, Algorithm 1): the
 * density filter of radius R (Eq. filtering) on the inner design grid, then
 * the Heaviside projection (Eq. projection; beta <= 0 means none).
 * gamma, phys [M]. */
int orc_design_prelude(const orc_problem* p, const double* gamma, double radius, double beta,
                       double eta, double* phys);
/* Its chain rule: dJ/dphys [M] -> dJ/dgamma [M]. */
int orc_design_prelude_adjoint(const orc_problem* p, const double* gamma, double radius,
                               double beta, double eta, const double* dJ_dphys,
                               double* dJ_dgamma);
/* Constraints (Sec. 2.6, Eqs. constraint1 .. constraint3): G_out = (G1, G2,
 * G3) and the gradients dG1, dG2 [M] w.r.t. the projected density and
 * dG3/dpsi [nt] (each nullable). */
int orc_constraints(const orc_problem* p, const double* phys, const double* chi,
                    const double* psi, double vmax, double omega_max, double p_omega,
                    double* G_out, double* dG1, double* dG2, double* dG3_dpsi);

/* Sensitivity epilogue alone: raw accumulators -> dJ/dgamma, dJ/dchi, dJ/dpsi. */
int orc_sensitivities(const orc_problem* p, const double* gamma, const double* kref_bar,
                      const double* motion_bar, const double* motion, double* dJ_dgamma,
                      double* dJ_dchi, double* dJ_dpsi);

/* Complex-step variants (re, im pairs) used to pin the adjoint.  Null imaginary
 * parts mean zero. */
int orc_forward_cs(const orc_problem* p, const double* gamma_re, const double* gamma_im,
                   const double* chi_re, const double* chi_im, const double* psi_re,
                   const double* psi_im, const double* state0_re, const double* state0_im,
                   double* J_re, double* J_im);
int orc_step_cs(const orc_problem* p, const double* s_re, const double* s_im,
                const double* k_re, const double* k_im, const double* us_re,
                const double* us_im, double* out_re, double* out_im);
int orc_map_cs(const orc_problem* p, const double* kref_re, const double* kref_im,
               const double* mot_re, const double* mot_im, double* k_re, double* k_im,
               double* us_re, double* us_im);

#ifdef __cplusplus
}
#endif
#endif
