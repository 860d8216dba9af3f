/*
 * mfm_oracle.h -- FP64 CPU oracle for the neighbour loops of the mesh-less
 * finite-volume (MFV) and finite-mass (MFM) hydro scheme of Alonso Asensio,
 * Dalla Vecchia, Potter & Stadel (arXiv 2211.12243).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker that the GPU path is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the product path never links or calls it.  It
 * shares no code, header or table with the HIP library.
 *
 * Conventions (all arrays are plain host memory owned by the caller):
 *   - n particles, structure of arrays, FP64.
 *   - B (inverse of the E matrix) is stored as 6 arrays of n: xx,xy,xz,yy,yz,zz.
 *   - grad is stored as 15 arrays of n: for q in (rho, vx, vy, vz, P) the
 *     three components d/dx, d/dy, d/dz, i.e. grad[(3*q + k)*n + i].
 *   - dQ and its scale are 5 arrays of n: (mass, px, py, pz, energy).
 *   - box[k] > 0 makes axis k periodic with that side; box[k] == 0 on all axes
 *     makes the domain open (used by the linear-field test).
 * Every function returns 0 on success and a negative code on bad arguments.
 */
#ifndef MFM_ORACLE_H
#define MFM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t scheme;        /* 0 = MFV, 1 = MFM (sec. 2.3.3, face velocity) */
  int32_t limiter;       /* bit0: conditioned BJ slope limiter; bit1: pairwise face limiter (sec. 2.3.6) */
  int32_t max_boosts;    /* times N_NGB may be multiplied by ngb_boost per particle (sec. 2.3.5) */
  int32_t h_maxit;       /* iteration cap of the smoothing-length solve */
  int32_t riemann_maxit; /* Newton cap of the exact Riemann solver */
  int32_t pad0;
  double gamma;          /* adiabatic index */
  double n_ngb;          /* target neighbour number N_NGB (sec. 2.3.5) */
  double ncond_max;      /* condition-number threshold, 100 in the paper */
  double ngb_boost;      /* N_NGB growth factor on failure, 1.2 in the paper */
  double h_tol;          /* relative tolerance of the H solve */
  double c_cfl;          /* CFL factor (sec. 2.3.10) */
  double psi1, psi2;     /* pairwise limiter constants, 0.5 and 0.25 in the paper */
  double riemann_tol;    /* relative Newton step tolerance of the Riemann solve */
  double alpha1;         /* dual-energy switch constant alpha_1 = 1/100 (sec. 2.3.7) */
  double box[3];         /* periodic box sides (0 = open) */
  double alpha2, alpha3; /* entropy switch constants alpha_2, alpha_3 = 1/1000 (sec. 2.3.7) */
  int32_t entropy_switch;/* 1: criterion (ii) of sec. 2.3.7 is on */
  int32_t pad1;
} orc_params;

/* Source terms of one step (sec. 2.3.7-2.3.9); all optional. */
typedef struct {
  const double *accel;   /* 3n: external gravitational acceleration, a[k*n + i] (NULL: none) */
  double inv_a;          /* comoving integration: 1/a, the factor of the fluxes and of the
                            drift (1 = physical coordinates) */
  double hubble_n, hubble_np1; /* Hubble rate at the start and at the end of the step */
  double *S;             /* n: extensive entropy m P / rho^gamma (in/out; NULL: switch off) */
  int32_t *emode;        /* n: 1 where the next density pass takes the pressure from S */
} orc_sources;

typedef struct {
  int64_t h_noconv;      /* smoothing-length solves that hit the iteration cap */
  int64_t ncond_boosts;  /* N_NGB boosts applied */
  int64_t ncond_fail;    /* particles still above ncond_max after all boosts */
  int64_t h_fallback;    /* particles whose candidate radius had to be widened */
  int64_t grad_pairs;    /* ordered gradient interactions: sum_i #{j != i : r_ij < H_i} */
  int64_t faces;         /* unordered flux pairs: #{i<j : r_ij < max(H_i, H_j)} */
  int64_t riemann_iters; /* total Newton iterations of the Riemann solves */
  int64_t riemann_maxit; /* Riemann solves that hit the iteration cap */
  int64_t vacuum;        /* faces with vacuum generation (zero flux) */
  int64_t positivity;    /* faces that fell back to first-order states */
  int64_t neg_mass;      /* MFV particles whose mass became non-positive */
  int64_t singular_e;    /* particles with a singular E matrix */
  int64_t u_guard;       /* particles whose new internal energy was not positive (kept) */
} orc_counters;

/* The cubic-spline kernel W(r, H) with compact support H (sec. 2.3.2). */
double orc_kernel_W(double r, double H);

/* All j with |x_j - x_i| < R_i (minimum image), including j == i.
 * Two-pass CSR: call with idx == NULL to get counts into start[0..n] (start[n]
 * = total), then again with idx of that length.  use_grid = 0 forces brute
 * force O(N^2), 1 lets the oracle use its own uniform grid (periodic boxes). */
int orc_neighbours(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *R, int use_grid, int64_t *start,
                   int32_t *idx);

/* Density loop (sec. 2.3.2, 2.3.5): solve the smoothing-length equation per
 * particle starting from H, apply the condition-number check with N_NGB boosts,
 * then V_i = 1/sum_j W(r_ij, H_i) (self included).
 * In: x,y,z,H (start value).  Out: H (converged), V, ncond (unweighted, from
 * the final neighbour set), nngb (effective N_NGB after boosts). */
int orc_density(const orc_params *p, int64_t n, const double *x, const double *y,
                const double *z, double *H, double *V, double *ncond, double *nngb,
                orc_counters *cnt);

/* The same for the nq particles idx[0..nq) only, with every particle a
 * candidate (a sample of a large set).  In: x,y,z, H0 (start values, all n).
 * Out: H, V, ncond, nngb of particle idx[q] at entry q (nq entries each). */
int orc_density_at(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *H0, int64_t nq, const int64_t *idx,
                   double *H, double *V, double *ncond, double *nngb, orc_counters *cnt);

/* Gradient loop (sec. 2.3.3, 2.3.6) and time-step loop (sec. 2.3.10).
 * In: x,y,z,H,V,m,vx,vy,vz,U.  Out: rho, P, c, B[6n], grad[15n] (already
 * multiplied by the limiter), alpha[5n] (limiter factors), ncond (weighted E),
 * dt_i. */
int orc_gradients(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, const double *H, const double *V, const double *m,
                  const double *vx, const double *vy, const double *vz, const double *U,
                  double *rho, double *P, double *c, double *B, double *grad, double *alpha,
                  double *ncond, double *dt_i, orc_counters *cnt);

/* Exact Riemann solver (Toro's pressure function, Newton iteration).
 * Returns 0 on convergence, 1 for vacuum generation, 2 when the cap was hit. */
int orc_riemann(double gamma, double rhoL, double uL, double PL, double rhoR, double uR,
                double PR, double tol, int maxit, double *pstar, double *ustar, int *iters);

/* The Newton iteration's starting value: Toro's adaptive choice (the
 * primitive-variable estimate when the states are close, else the
 * two-rarefaction or two-shock estimate), floored at 1e-10 (P_L + P_R) / 2.
 * branch (optional): 0, 1 or 2 for the primitive-variable, two-rarefaction
 * or two-shock estimate. */
double orc_riemann_guess(double gamma, double rhoL, double uL, double PL, double rhoR, double uR,
                         double PR, int *branch);

/* Sample the exact solution at speed xi = x/t (Toro's sampling). */
int orc_riemann_sample(double gamma, double rhoL, double uL, double PL, double rhoR, double uR,
                       double PR, double pstar, double ustar, double xi, double *rho, double *u,
                       double *P);

/* Pairwise limiter of a face value qf extrapolated from the own side (value
 * qo) towards the other side (value qn), sec. 2.3.6 with psi_1, psi_2. */
double orc_pair_limit(double qf, double qo, double qn, double psi1, double psi2);

/* The flux of one face (i, j) as the oracle computes it: contribution vector
 * c = |A_ij| F_ij (5 components) oriented from i (left) to j (right). */
int orc_face(const orc_params *p, int64_t n, int64_t i, int64_t j, const double *x,
             const double *y, const double *z, const double *H, const double *V,
             const double *rho, const double *vx, const double *vy, const double *vz,
             const double *P, const double *B, const double *grad, double dt, double *c,
             orc_counters *cnt);

/* The flux loop's faces: every unordered pair {i, j} with r_ij < max(H_i, H_j),
 * as (lower index, higher index).  orc_face_list allocates fa and fb (free
 * them); orc_face_list_copy copies at most cap faces into caller arrays and
 * returns the total in nf_out (call with fa = fb = NULL to size them). */
int orc_face_list(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, const double *H, int64_t *nf_out, int64_t **fa_out,
                  int64_t **fb_out);
int orc_face_list_copy(const orc_params *p, int64_t n, const double *x, const double *y,
                       const double *z, const double *H, int64_t cap, int64_t *fa,
                       int64_t *fb, int64_t *nf_out);

/* Flux loop (sec. 2.3.3, 2.3.4, 2.3.6): for every unordered pair with
 * r_ij < max(H_i, H_j), dQ_i -= dt c_ij and dQ_j += dt c_ij.
 * Out: dQ[5n]; scale[5n] = dt * sum_j |c_ij| per component (the size against
 * which accumulated sums are judged). */
int orc_fluxes(const orc_params *p, int64_t n, const double *x, const double *y,
               const double *z, const double *H, const double *V, const double *rho,
               const double *vx, const double *vy, const double *vz, const double *P,
               const double *B, const double *grad, double dt, double *dQ, double *scale,
               orc_counters *cnt);

/* Flux loop with the comoving factor and the gravity work of the exchanged
 * mass: dQ_i -= dt inv_a c_ij, and, when gwork (3n) is given, every face adds
 * dm_ij (x_j - x_i) to gwork of both particles, dm_ij = dt inv_a c_m,ij the
 * mass that goes from i to j (sec. 2.3.8, eq. gravity_source). */
int orc_fluxes_src(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *H, const double *V, const double *rho,
                   const double *vx, const double *vy, const double *vz, const double *P,
                   const double *B, const double *grad, double dt, double inv_a, double *dQ,
                   double *scale, double *gwork, orc_counters *cnt);

/* E_kin^max,i = max_j 1/2 m_i |v_j - v_i|^2 over the neighbours r_ij < H_i
 * (sec. 2.3.7). */
int orc_ekin_max(const orc_params *p, int64_t n, const double *x, const double *y,
                 const double *z, const double *H, const double *m, const double *vx,
                 const double *vy, const double *vz, double *ekin_max);

/* After the density pass: where emode is set, the pressure comes from the
 * entropy, U := P V / (gamma - 1) with P = (S / m) rho^gamma; elsewhere S is
 * reset from U, S := m P / rho^gamma with P = (gamma - 1) U / V. */
int orc_entropy_pressure(const orc_params *p, int64_t n, const double *m, const double *V,
                         double *U, double *S, const int32_t *emode);

/* Close of the step with source terms (sec. 2.3.4 eq. source_term_discr,
 * 2.3.7, 2.3.8, 2.3.9): hydro update, gravity source, Hubble terms, the
 * three-way pressure switch, drift (scaled by inv_a).  gwork and ekin_max
 * may be NULL; V and H are the step's volumes and support radii. */
/* Individual time steps (sec. 2.3.4, sec. 2.3.10).  A rung r gives the step
 * 2^-r dt0; ORC_RUNG_MAX bounds it. */
#define ORC_RUNG_MAX 30

/* The rung of each particle from its own step dt_i (the smallest r >= 0 with
 * dt_i > 2^-r dt0), then the limiter |r_i - r_j| <= 2 over the pairs of the
 * flux loop (the lower rung raised).  -3: a step below 2^-ORC_RUNG_MAX dt0. */
int orc_rungs(const orc_params *p, int64_t n, const double *x, const double *y,
              const double *z, const double *H, const double *dt_i, double dt0, int32_t *rung);

/* One base step dt0 on individual steps (the reading is at the definition):
 * the state is advanced in place like orc_step's; rung (n) receives the
 * rungs used, or, with rungs_given, holds them (0..ORC_RUNG_MAX, no
 * criterion or limiter applied: for tests of the sub-step scheme itself);
 * nsub_out receives the number of sub-steps. */
int orc_step_rungs(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
                   double *vx, double *vy, double *vz, double *E, double *U, double *H,
                   double dt0, int32_t *rung, int rungs_given, int64_t *nsub_out,
                   orc_counters *cnt);

int orc_update_src(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
                   double *vx, double *vy, double *vz, double *E, double *U, const double *dQ,
                   double dt, const orc_sources *src, const double *gwork,
                   const double *ekin_max, const double *V, const double *H,
                   orc_counters *cnt);

/* One full step with source terms. */
int orc_step_src(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
                 double *vx, double *vy, double *vz, double *E, double *U, double *H,
                 double dt_max, const orc_sources *src, double *dt_out, orc_counters *cnt);

/* Close of the step (eq. hydro_discr, internal-energy integration and the
 * pressure switch of sec. 2.3.7, drift).  Updates x,y,z,m,vx,vy,vz,E,U in place. */
int orc_update(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
               double *vx, double *vy, double *vz, double *E, double *U, const double *dQ,
               double dt, orc_counters *cnt);

/* One full step: density, gradients, dt = min(dt_max, min_i dt_i), fluxes,
 * update.  State arrays are updated in place; dt_out receives the step. */
int orc_step(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
             double *vx, double *vy, double *vz, double *E, double *U, double *H,
             double dt_max, double *dt_out, orc_counters *cnt);

#ifdef __cplusplus
}
#endif
#endif
