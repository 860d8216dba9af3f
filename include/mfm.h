/*
 * mfm.h -- C ABI of the MI355X library for the neighbour loops of the
 * mesh-less finite-volume (MFV) and mesh-less finite-mass (MFM) hydro scheme
 * of Alonso Asensio, Dalla Vecchia, Potter & Stadel, "Mesh-free hydrodynamics
 * in pkdgrav3 for galaxy formation simulations" (arXiv 2211.12243).
 *
 * The paper splits one hydro step into four loops over neighbouring particles
 * (sec. 2.2.3): (1) smoothing length and number density, (2) gradients and
 * limiter, (3) extrapolation, Riemann solver and fluxes, (4) time step.  The
 * entry points below are those loops, plus the neighbour-cell build that they
 * share and the close of the step (eq. hydro_discr and sec. 2.3.7).
 *
 * Memory.  Every array is DEVICE memory owned by the caller (for example torch
 * tensors), structure of arrays, FP64, length n unless stated.  The library
 * never allocates or frees device memory: mfm_create carves its scratch space
 * out of one caller-supplied device workspace of mfm_workspace_bytes() bytes,
 * which must stay alive until mfm_destroy.  The library never frees caller
 * memory.  Host structs passed by pointer are copied; they may be freed after
 * the call returns.
 *
 * Streams.  Every call enqueues work on the hipStream_t given to mfm_create
 * and returns without waiting, except where stated ("synchronises").
 *
 * Errors.  Every function returns MFM_OK (0) or a negative MFM_E_* code; no
 * exception or abort crosses the ABI.  mfm_strerror() gives the text, and
 * mfm_last_error() the message of the last failure on a context (for
 * MFM_E_HIP it holds the HIP runtime's error string).  Conditions found inside
 * kernels (an H solve that did not converge, an overflowing neighbour list)
 * are counted in device counters and surface at the next synchronising call.
 *
 * Threads.  A context may be used by one host thread at a time.
 */
#ifndef MFM_H
#define MFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MFM_OK 0
#define MFM_E_ARG (-1)        /* null pointer, n out of range, invalid parameter */
#define MFM_E_WORKSPACE (-2)  /* workspace missing or smaller than mfm_workspace_bytes() */
#define MFM_E_HIP (-3)        /* HIP runtime error (text in mfm_last_error) */
#define MFM_E_H_NOCONV (-4)   /* some smoothing-length solve hit its iteration cap */
#define MFM_E_CELLS (-5)      /* smoothing lengths outgrew their search radii: rebuild and repeat */
#define MFM_E_LIST (-6)       /* the neighbour lists do not fit the list pool (see max_list) */
#define MFM_E_NONFINITE (-7)  /* a non-finite time step or state was produced */
#define MFM_E_STATE (-8)      /* call order violated (e.g. mfm_fluxes before mfm_gradients) */

/* parameter values */
#define MFM_SCHEME_MFV 0 /* face moves with the mean particle velocity; mass flows */
#define MFM_SCHEME_MFM 1 /* face moves with the contact of the Riemann problem; no mass flux */
#define MFM_FP64 0       /* all pair arithmetic in FP64 */
#define MFM_MIXED 1      /* FP32 pair arithmetic, FP64 accumulators (see mfm_params.precision) */
#define MFM_GUESS_PLAIN 0
#define MFM_GUESS_LEARNED 1
#define MFM_LIMIT_BJ 1       /* conditioned Barth-Jespersen slope limiter (sec. 2.3.6) */
#define MFM_LIMIT_PAIRWISE 2 /* pairwise face limiter with psi1, psi2 (sec. 2.3.6) */

/* Hydro parameters (sec. 2.3).  mfm_default_params() fills the paper's
 * defaults: N_NGB = 32, N_cond threshold 100 with x1.2 boosts (sec. 2.3.5),
 * psi1 = 0.5, psi2 = 0.25 (sec. 2.3.6), alpha1 = 1/100 (sec. 2.3.7). */
typedef struct mfm_params {
  int32_t scheme;        /* MFM_SCHEME_MFV or MFM_SCHEME_MFM */
  int32_t precision;     /* MFM_FP64 or MFM_MIXED */
  int32_t limiter;       /* OR of MFM_LIMIT_* */
  int32_t max_boosts;    /* N_NGB boosts allowed per particle and step (default 5) */
  int32_t h_maxit;       /* smoothing-length iteration cap (default 64) */
  int32_t riemann_maxit; /* Riemann Newton cap (default 100) */
  int32_t guess;         /* MFM_GUESS_PLAIN or MFM_GUESS_LEARNED */
  int32_t max_list;      /* list pool, in entries per particle (default 160): the
                            lists of each chunk of 16 consecutive particles take
                            16 x (the chunk's longest candidate list + 1/8 + 4),
                            planned from the previous search, so a few long
                            lists cost little; the pool must hold the sum */
  double gamma;          /* adiabatic index (> 1) */
  double n_ngb;          /* neighbour number N_NGB (> 32/3, non-integer allowed) */
  double ncond_max;      /* condition-number threshold (default 100) */
  double ngb_boost;      /* N_NGB factor when a particle fails the check (default 1.2) */
  double h_tol;          /* relative tolerance of the smoothing-length solve (default 1e-13):
                            it ends on a Newton step below h_tol H, or below
                            1e-2 sqrt(h_tol) H, where its quadratic convergence
                            leaves H far closer than h_tol to the root */
  double c_cfl;          /* CFL factor (default 0.2) */
  double psi1, psi2;     /* pairwise limiter constants */
  double riemann_tol;    /* relative Newton step tolerance of the exact solver (default 1e-10) */
  double alpha1;         /* dual-energy switch: U > alpha1 E_kin -> U from E (default 0.01) */
  double box[3];         /* periodic box sides; all > 0 (the library needs a periodic box) */
  double cell_margin;    /* search margin (>= 1, default 1.10): a pair is a
                            candidate when r < cell_margin * max(H_i, H_j) at
                            the build, and an H may grow by at most this
                            factor in one density pass */
  int32_t reserved;      /* must be 0 */
  int32_t pad0;
  double alpha2, alpha3; /* entropy switch (sec. 2.3.7): the pressure comes from the entropy
                            when U < alpha2 (E_kin^max + U) or U < alpha3 E_grav (default
                            1/1000 each) */
  int32_t entropy_switch;/* 1: criterion (ii) of the pressure switch is on (needs S, emode) */
  int32_t pad1;
  double mixed_jump;     /* mixed path: a face whose two particles' pressures or densities
                            differ by more than this factor is computed in FP64 (in the flux
                            loop's second pass); default 8, 0 = none.  Across strong jumps the
                            FP32 face arithmetic loses accuracy (cancelling extrapolations,
                            strong shocks and rarefactions) */
} mfm_params;

/* The particle set: device pointers, each of n FP64 values (B: 6n, grad: 15n,
 * dQ: 5n, entry k of particle i at [k * n + i]).
 *   state (read and written): x, y, z  positions in [0, box)
 *                             vx, vy, vz velocities
 *                             m  mass, E total energy, U internal energy
 *                                (E and U extensive: per particle, not per mass)
 *                             H  support radius of the kernel (the start value
 *                                of the smoothing-length solve; overwritten)
 *   outputs of mfm_density:   V volume 1/omega^-1, rho = m/V, P = (gamma-1)U/V,
 *                             c sound speed, ncond (the unweighted check value)
 *   outputs of mfm_gradients: B = E^-1 (xx,xy,xz,yy,yz,zz), grad (for q in
 *                             rho, vx, vy, vz, P the d/dx, d/dy, d/dz, already
 *                             multiplied by the slope limiter), ncond (of the
 *                             volume-weighted E), dt_i
 *   output of mfm_fluxes:     dQ = -dt sum_j F_ij A_ij for (m, px, py, pz, E)
 *   id (optional int64):      moved with the state whenever the state is permuted
 */
typedef struct mfm_particles {
  int64_t n;
  double *x, *y, *z, *vx, *vy, *vz, *m, *E, *U, *H;
  double *V, *rho, *P, *c, *ncond;
  double *B, *grad, *dQ, *dt_i;
  int64_t *id; /* optional (may be NULL): caller's particle labels, permuted with the state */
  /* source terms (sec. 2.3.7, 2.3.8), optional, permuted with the state: */
  double *S;      /* extensive entropy S = m P / rho^gamma (needed by the entropy switch) */
  int32_t *emode; /* 1 where the next density pass takes the pressure from S (switch) */
  double *accel;  /* 3n: external gravitational acceleration, entry k of i at [k n + i] */
} mfm_particles;

/* Counters and conserved totals (filled by mfm_diagnostics). */
typedef struct mfm_diag {
  int64_t h_noconv;      /* smoothing-length solves that hit h_maxit */
  int64_t ncond_boosts;  /* N_NGB boosts applied */
  int64_t ncond_fail;    /* particles still above ncond_max after max_boosts */
  int64_t cell_rebuilds; /* cell grids rebuilt because H outgrew them */
  int64_t list_overflow; /* particles whose lists outgrew their planned block (pass redone) */
  int64_t grad_pairs;    /* sum_i #{j != i : r_ij < H_i} of the last mfm_gradients */
  int64_t faces;         /* #{unordered pairs : r_ij < max(H_i, H_j)} of the last mfm_fluxes */
  int64_t riemann_iters; /* Newton iterations of the last mfm_fluxes */
  int64_t riemann_maxit; /* faces that hit riemann_maxit */
  int64_t vacuum;        /* faces with vacuum generation (no flux) */
  int64_t positivity;    /* faces that fell back to first-order states */
  int64_t neg_mass;      /* particles whose MFV mass became non-positive (not clamped) */
  int64_t singular_e;    /* particles with a singular E matrix */
  int64_t guess_fallback;/* learned guesses rejected for the plain one */
  int64_t fp64_inverse;  /* mixed path: E matrices inverted in FP64 */
  int64_t u_guard;       /* particles whose updated internal energy was not positive; they
                            keep their start-of-step value (mfm_update) */
  int64_t hard_faces;    /* faces solved in the flux loop's FP64 second pass (mixed_jump,
                            learned guess) */
  int64_t hard_overflow; /* faces that found the second pass's queue full and were solved in
                            the first pass */
  double mass, px, py, pz, energy; /* sums over particles of m, m v, E */
} mfm_diag;

/* Fill p with the defaults listed above (MFV, FP64, both limiters, gamma 5/3,
 * unit periodic box). */
void mfm_default_params(mfm_params *p);

/* Bytes of device workspace a context for up to n_max particles needs. */
size_t mfm_workspace_bytes(const mfm_params *p, int64_t n_max);

/* Create a context.  workspace: device pointer of at least
 * mfm_workspace_bytes(p, n_max) bytes, 256-byte aligned, in ordinary
 * (coarse-grained) device memory such as hipMalloc returns: the flux loop
 * adds into it with the GPU's native FP64 atomics, which fine-grained or
 * host-coherent memory does not support.  The context owns its contents
 * until mfm_destroy.  stream: a hipStream_t (NULL = the default stream).
 * Returns MFM_E_ARG for invalid parameters, MFM_E_WORKSPACE when the
 * workspace is missing or too small. */
int mfm_create(const mfm_params *p, int64_t n_max, void *workspace, size_t workspace_bytes,
               void *stream, struct mfm_ctx **out);
int mfm_destroy(struct mfm_ctx *ctx);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: a context
 * like mfm_create's whose workspace is the library's own static device array
 * on the current GPU (mfm_static_workspace_bytes() = 64 MiB; each GPU the
 * library runs on holds one until the process ends).  The call allocates
 * nothing: no hipMalloc, no library allocator.  The caller still owns the
 * particle arrays.
 *   - Limit: mfm_workspace_bytes(p, n_max) must fit in the array (about
 *     12 000 particles at the default max_list); larger requests return
 *     MFM_E_WORKSPACE.
 *   - One such context per GPU at a time (MFM_E_STATE while one exists;
 *     mfm_destroy releases it).  All its calls share the GPU's array, which
 *     keeps the last call's contents: calls that overlap on one GPU race.
 *   - Counters start at zero; every other part of the array is written
 *     before it is read.
 * Returns MFM_E_ARG for invalid parameters, MFM_E_HIP if the device or the
 * array's address cannot be obtained. */
size_t mfm_static_workspace_bytes(void);
int mfm_create_static(const mfm_params *p, int64_t n_max, void *stream, struct mfm_ctx **out);

/* Sort the particles along a Morton (Z-order) curve of 10 bits per axis of
 * their place in the box (sec. 2.2.1: particles are reordered in memory so
 * that spatial neighbours are contiguous), permute the state arrays (x..H,
 * and S, emode, accel when given) IN PLACE into that order, and build the
 * neighbour-search tree over buckets of 64 consecutive particles (sec.
 * 2.2.3): per node the bounding box and cell_margin times the largest H.
 * The sort is stable: particles with the same key keep their order from
 * before the call, so a second call on unchanged particles is the identity.
 * perm (device int64, n, may be NULL) receives for each new slot k the slot
 * the particle had before the call.  The H values at this call bound the
 * next mfm_density (see cell_margin).  Does not synchronise. */
int mfm_build_cells(struct mfm_ctx *ctx, const mfm_particles *parts, int64_t *perm);

/* Loop (1), sec. 2.3.2 and 2.3.5: per particle, solve
 * (4 pi/3) H^3 omega^-1(H) = N_NGB for H, with omega^-1 = sum_j W(r_ij, H)
 * (self included); if the condition number of E~ = sum_j W d d^T exceeds
 * ncond_max, multiply N_NGB by ngb_boost and solve again.  Writes H, V, rho,
 * P, c, ncond and the neighbour lists used by the next two loops.  Requires
 * mfm_build_cells on the same positions.  If some H reaches its bound (half
 * the smallest box side, or cell_margin times its value at the build) the
 * pass is discarded: every H is replaced by its root, or by an estimate of it
 * where the bound was reached, the next mfm_build_cells searches with those
 * (and a larger margin after a second such pass in a row), and the call
 * returns MFM_E_CELLS; build and density are then repeated (mfm_step does
 * this, up to 6 attempts).  The neighbour lists go to blocks planned from the
 * previous search's list lengths; a list longer than its block leaves the
 * state untouched and the pass is planned again from the lengths it found
 * (inside this call; mfm_step takes another attempt).
 * Synchronises (it reads the pass counters). */
int mfm_density(struct mfm_ctx *ctx, const mfm_particles *parts);

/* Loops (2) and (4), sec. 2.3.3, 2.3.6, 2.3.10: E_i = sum_j V_j W_ij d d^T,
 * B_i = E_i^-1, grad q_i = B_i sum_j V_j W_ij (q_j - q_i) d for q in
 * (rho, v, P), conditioned slope limiter, signal velocity and
 * dt_i = c_cfl H_i / v_sig,i.  dt_dev (device double) receives
 * min(dt_max, min_i dt_i); it stays on the device. */
int mfm_gradients(struct mfm_ctx *ctx, const mfm_particles *parts, double dt_max,
                  double *dt_dev);

/* Loop (3), sec. 2.3.3, 2.3.4, 2.3.6: for every unordered pair with
 * r_ij < max(H_i, H_j), the face vector A_ij, half-step extrapolation of the
 * primitives to the face, pairwise limiter, exact Riemann solve, MFV or MFM
 * flux; dQ_i -= dt F_ij A_ij and dQ_j += dt F_ij A_ij with the same value
 * (bitwise antisymmetric).  dt_dev: device pointer to the step (from
 * mfm_gradients). */
int mfm_fluxes(struct mfm_ctx *ctx, const mfm_particles *parts, const double *dt_dev);

/* Comoving integration (sec. 2.3.9) for the following steps: inv_a = 1/a
 * multiplies every spatial derivative -- the fluxes, the gradients of the
 * half-step predictor -- and the drift; hubble_n, hubble_np1 are the Hubble
 * rate at the start and end of the step, used in the implicit update
 * X = (X~ - eta dt H^n X^n) / (1 + eta dt H^(n+1)) of momentum (eta 1/2),
 * total energy (1), internal energy and entropy (3 (gamma - 1) / 2).  The
 * total-energy form holds for gamma = 5/3 only: other gammas with a nonzero
 * Hubble rate return MFM_E_ARG.  Defaults 1, 0, 0 (physical coordinates). */
int mfm_set_cosmology(struct mfm_ctx *ctx, double inv_a, double hubble_n, double hubble_np1);

/* Close of the step, eq. hydro_discr and sec. 2.3.7: m += dQ_m, m v += dQ_p,
 * E += dQ_E, U += dQ_E - v.dQ_p + v^2/2 dQ_m; with accel, the gravity source
 * of sec. 2.3.8 by eq. source_term_discr (momentum m a, work P.a and
 * 1/2 a . sum_j dm_ij r_ij); the Hubble terms (mfm_set_cosmology); the
 * pressure switch: U := E - E_kin when E - E_kin > alpha1 (E_grav + E_kin),
 * else with the entropy switch emode := 1 when U < alpha2 (E_kin^max + U) or
 * U < alpha3 E_grav, else the integrated U; and the drift
 * x += dt inv_a (v_old + v_new)/2 (periodic wrap).  An internal energy that
 * would not be positive keeps its start-of-step value (counted in
 * mfm_diag.u_guard). */
int mfm_update(struct mfm_ctx *ctx, const mfm_particles *parts, const double *dt_dev);

/* One full step: cells, density, gradients, fluxes, update.  dt_host receives
 * the step taken.  Synchronises.  The cells stage sorts as mfm_build_cells
 * does, except while the order of the last sort still groups the particles
 * well: a step on the same arrays (same x pointer and count) after a step
 * whose cells, search and density stages took no longer than those of the
 * step of that sort (timed with events; at most 16 steps after it) builds
 * the tree over the particles in their present order instead.  Which pairs
 * interact does not depend on the order; mfm_build_cells and
 * mfm_step_rungs always sort, and so does every step on a context from
 * mfm_create_static.  A context from mfm_create makes two events for this
 * on its first step (freed by mfm_destroy). */
int mfm_step(struct mfm_ctx *ctx, const mfm_particles *parts, double dt_max, double *dt_host);

/* Individual time steps (sec. 2.3.4, last paragraphs; sec. 2.3.10): one base
 * step dt0 on a power-of-two hierarchy.
 *   - Rungs: each particle's step is 2^-r dt0 with r the smallest integer
 *     >= 0 such that its CFL step exceeds 2^-r dt0, raised until every pair
 *     of the flux loop (r < max(H_i, H_j)) differs by at most two rungs; set
 *     when the base step starts (every particle synchronised) and kept
 *     through it.  With rungs_given, rung (device int32, n, in the input
 *     order, permuted with the particles) holds them instead (0 ..
 *     MFM_RUNG_MAX; no criterion, no limiter); else rung, when not NULL,
 *     receives them (in the order of the particles after the call).
 *   - The base step is cut into 2^max(r) sub-steps.  At each, the particles
 *     whose step begins run the density and gradient loops, at the
 *     positions of that time (a particle in mid-step: its step-start
 *     position plus the elapsed time times its velocity, with its H, V, B,
 *     gradients and state from its step start).  Every face with such an
 *     end is solved with dt = min(dt_i, dt_j), each side predicted from its
 *     step start over the elapsed time plus dt/2, and dt A_ij F_ij goes to
 *     both particles; a particle whose step ends closes it (mfm_update's
 *     close with its own step and the contributions summed over it).
 *   - With every rung equal this is 2^r steps of mfm_step with 2^-r dt0.
 * No source terms (mfm_set_cosmology at its defaults, no accel) and no
 * entropy switch: MFM_E_ARG otherwise; a step that needs a rung deeper than
 * MFM_RUNG_MAX: MFM_E_NONFINITE.  nsub_out (host, may be NULL) receives the
 * number of sub-steps.  Synchronises once per sub-step.  The first call on a
 * context from mfm_create allocates a small pinned host buffer and an event
 * (freed by mfm_destroy) for the per-sub-step read of the pass counters; a
 * context from mfm_create_static allocates nothing and reads them with a
 * synchronising copy. */
#define MFM_RUNG_MAX 24
int mfm_step_rungs(struct mfm_ctx *ctx, const mfm_particles *parts, double dt0, int32_t *rung,
                   int rungs_given, int64_t *nsub_out);

/* Counters accumulated since the last mfm_reset_counters, and the conserved
 * totals of the current state.  Synchronises. */
int mfm_diagnostics(struct mfm_ctx *ctx, const mfm_particles *parts, mfm_diag *out);
int mfm_reset_counters(struct mfm_ctx *ctx);

/* Kernel timing on the context's stream with HIP events.  While enabled every
 * launch of the loops is bracketed by events; mfm_kernel_times (synchronises)
 * returns, per stage (0 cells, 1 neighbour search, 2 density, 3 gradients,
 * 4 fluxes: the whole flux loop, 5 update, 6 the flux loop's first-pass
 * kernel alone, 7 its FP64 second pass alone), the summed milliseconds and
 * launch counts since enabling. */
#define MFM_NSTAGES 8
int mfm_enable_timing(struct mfm_ctx *ctx, int on);
int mfm_kernel_times(struct mfm_ctx *ctx, double *ms_out, int64_t *count_out);

const char *mfm_strerror(int status);
const char *mfm_last_error(struct mfm_ctx *ctx);

/* ------------------------------------------------------------------------
 * Learned starting value of the exact Riemann iteration (sec. 2.3.3 uses the
 * exact solver; the guess only changes how many Newton steps it takes).
 *
 * The network maps six features of a face's Riemann problem (left and right
 * states in the face frame) -- ln(rho_L/rho_R), ln(P_L/P_R),
 * slog((u_R-u_L)/c_avg) with slog(v) = sign(v) ln(1+|v|), ln(p0/P_avg) with
 * P_avg = (P_L+P_R)/2, and 1/0 indicators of p0 being the two-rarefaction or
 * the two-shock estimate -- to y = ln(p* / p0), the error of the plain
 * starting value p0 (Toro's adaptive choice: the primitive-variable,
 * two-rarefaction or two-shock estimate, floored at 1e-10 P_avg).
 * Architecture: 6 -> 64 -> 64 -> 64 -> 1, SiLU hidden activations, BF16
 * operands with FP32 accumulation on the matrix cores.  The FP32 parameter
 * vector (mfm_mlp_param_count floats) is, in order: W1 [16][64] (row k is
 * input feature k; rows 6..15 are padding and must be zero), b1 [64],
 * W2 [64][64], b2 [64], W3 [64][64], b3 [64], w4 [64], b4 [1]; a layer
 * computes a_out[n] = silu(b[n] + sum_k a_in[k] W[k][n]).  Inputs are
 * standardised with norm[0..5] (means) and norm[6..11] (standard deviations,
 * > 0); the output is y = norm[12] + norm[13] * net(x) (norm[13] > 0);
 * norm[14..15] are unused.
 *
 * In the flux loop (params.guess = MFM_GUESS_LEARNED), the Newton iteration
 * starts from the prediction p0 e^y when that is finite and above the
 * pressure floor; if its second residual exceeds its first, or it needs more
 * than 8 steps, the face is solved again from the plain guess and
 * guess_fallback counts it (riemann_iters counts the steps of both tries).
 * Results therefore agree with the plain guess to the solver's tolerance
 * whatever the weights are.
 *
 * A state is caller-owned device memory of mfm_mlp_state_bytes bytes
 * (256-byte aligned) holding the FP32 parameters, Adam moments, gradient,
 * normalisation and BF16 weight copies.  Calls on one state are ordered by
 * the stream they are given; stream may be null (the default stream).
 * ------------------------------------------------------------------------ */
size_t mfm_mlp_state_bytes(void);
int mfm_mlp_param_count(void);

/* Load parameters and normalisation (host arrays of mfm_mlp_param_count and
 * 16 floats) and clear the Adam moments.  Synchronises. */
int mfm_mlp_init(void *state_dev, const float *params_host, const float *norm_host, void *stream);

/* Gradient of the mean squared error, in standardised units,
 * L = (1/n) sum_r (net(x_r) - (t_r - norm[12]) / norm[13])^2 over n rows of a
 * device array (row r: features at [r*stride + 0..5], target t_r at
 * [r*stride + 6]; the face dump's layout, stride 8).  Overwrites the stored
 * gradient; loss_host (optional) receives L (then synchronises). */
int mfm_mlp_backward(void *state_dev, const float *rows_dev, int64_t n, int64_t stride,
                     float *loss_host, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on the
 * stored gradient, then the BF16 weight copies are refreshed. */
int mfm_mlp_adam(void *state_dev, float lr, int step, void *stream);

/* mfm_mlp_backward then mfm_mlp_adam; loss_host (optional) receives the
 * loss before the step (then synchronises). */
int mfm_mlp_train_step(void *state_dev, const float *rows_dev, int64_t n, int64_t stride,
                       float lr, int step, float *loss_host, void *stream);

/* y_dev[r] = predicted ln(p* / p0) for n rows laid out as in
 * mfm_mlp_backward (the target column is not read). */
int mfm_mlp_predict(const void *state_dev, const float *rows_dev, int64_t n, int64_t stride,
                    float *y_dev, void *stream);

/* Copy the FP32 parameters and/or the last gradient to the host (either may
 * be null).  Synchronises. */
int mfm_mlp_get(const void *state_dev, float *params_host, float *grad_host, void *stream);

/* Use the network in state_dev (null detaches) for the context's learned
 * guess.  The state must stay valid while mfm_fluxes may run; mfm_fluxes
 * returns MFM_E_STATE when the learned guess is selected and none is
 * attached. */
int mfm_mlp_attach(struct mfm_ctx *ctx, const void *state_dev);

/* Training data: while armed, every face the flux loop solves appends one
 * record of 8 floats to records_dev -- the six features, the target
 * ln(p* / p0) of the converged solution (p0: the plain starting value), and
 * the number of Newton steps the face's solve took -- until capacity records are stored (further faces are
 * counted but not written).  Records are in no particular order.  Arming
 * (records_dev non-null) or disarming (null) resets the count.  Synchronises. */
int mfm_face_dump(struct mfm_ctx *ctx, float *records_dev, int64_t capacity);
/* Records stored since arming (at most the capacity).  Synchronises. */
int mfm_face_dump_count(struct mfm_ctx *ctx, int64_t *count_host);

#ifdef __cplusplus
}
#endif
#endif
