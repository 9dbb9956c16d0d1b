/*
 * gea.h -- C ABI of the MI355X (gfx950) library that advances the dry
 * compressible Euler equations by one segregated pressure-based time step
 * (GEA, arXiv:2303.10499, Sec. 3) on a uniform hexahedral mesh, and solves
 * its pressure equation.
 *
 * Problem statement (Sec. 3, the paragraph before Step 1): given rho^n, u^n,
 * T^n, p^n and p'^n, find the end-of-step (rho, u, T, p, p')^{n+1} through
 *   Step 1 (eqs. e1_d, step2_sd, step1_3sd)  mass flux, density and momentum
 *           predictors, kinetic energy;
 *   Step 2 (eqs. step3_sd, step3_2sd, step3_3sd) energy in total-energy form
 *           (eq. ent, e = c_v T + |u|^2/2 + g z) with its diffusion at the
 *           new level (one SPD solve for T per sweep), e -> T recovery and
 *           the EOS density rho^{n+2/3} = p^n/(R T^{n+1});
 *   Step 3 (eqs. step2_sd corrector, p_prime_sd, step4_4sd) PISO correctors:
 *           H operator, predicted face flux, pressure equation, flux and
 *           velocity correction, end-of-step p, K, rho.
 * The pressure equation is the SPD Helmholtz system
 *     c_i p'_i + sum_f w_f (p'_i - p'_nb) = b_i,
 *     c = V/(R T dt),  w_f = (D_P + D_N)/2 * S_f/d_f,  D = rho^{n+2/3} dt/rho^{n+1/3},
 * obtained from BDF1 continuity with rho^{n+1} = (p' - rho^{n+2/3} g z)/(R T)
 * (eqs. p_split, p, step4_4sd); the printed eq. p_prime_sd is garbled.
 *
 * Conventions
 *  - Units SI.  g > 0; Phi = g z; p = p' - rho Phi; the momentum force is
 *    -(grad p' - Phi grad rho) (eq. mom_split with gravity pointing down).
 *  - Layout: structure of arrays, FP64, cell index i + nx*(j + ny*k), x
 *    fastest, z vertical.  ny == 1 selects the 2D xz-plane (velocity
 *    components u, w); otherwise 3D (u, v, w).  A velocity argument holds
 *    ndim consecutive blocks of ncell values.
 *  - Memory: the caller owns every input and output array and the device
 *    workspace (size from gea_workspace_bytes, 256-byte aligned).  The
 *    library allocates no device memory; it owns only the opaque context
 *    and, inside it, a 4 KB pinned host buffer through which it reads the
 *    solver's convergence scalars.
 *  - Streams: all device work is enqueued on the stream given to
 *    gea_init_mesh.  gea_step, gea_pressure_solve and gea_init_bubble return
 *    after the work completed (convergence is decided from device values);
 *    device-to-device copies are ordered on the stream.
 *  - Errors: every call returns a gea_status; no C++ exception crosses the
 *    ABI; gea_last_error gives a message.  A step that fails (no
 *    convergence within max_iter, a non-finite value) leaves the state as it
 *    was before that step.
 */
#ifndef GEA_H
#define GEA_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gea_ctx gea_ctx;

typedef enum {
  GEA_OK = 0,
  GEA_ERR_ARG = -1,     /* bad dimension, null pointer, non-positive constant, small workspace */
  GEA_ERR_ALLOC = -2,   /* host allocation of the context failed                             */
  GEA_ERR_HIP = -3,     /* a HIP runtime call failed                                         */
  GEA_ERR_NOCONV = -4,  /* pressure solve did not reach tol within max_iter                  */
  GEA_ERR_NAN = -5,     /* a non-finite value appeared                                       */
  GEA_ERR_STATE = -6    /* call order violated (e.g. step before a state was set)            */
} gea_status;

typedef enum { GEA_HOST = 0, GEA_DEVICE = 1 } gea_ptr_kind;

/* pressure solver of Step 3 */
typedef enum {
  GEA_PCG_JACOBI_FP64 = 0, /* conjugate gradients, Jacobi preconditioner, FP64 throughout        */
  GEA_IR_FP32_FP64 = 1,    /* FP64 iterative refinement around an FP32 inner Jacobi-PCG           */
  GEA_LEARNED_MIXED = 2    /* learned initial guess and preconditioner (flexible CG) inside the
                              FP64 refinement, Jacobi-PCG fallback on stall                        */
} gea_solver;

typedef struct { int32_t nx, ny, nz; double lx, ly, lz; } gea_mesh;

typedef struct {
  double R, cp, cv, g, p0, theta0; /* gas constants; p0, theta0 only enter the initial state        */
  double mu, Pr, dt;               /* artificial viscosity (Remark 1), Prandtl number, time step     */
  int32_t n_corr;                  /* PISO correctors per step (>= 1)                                */
  int32_t n_energy_sweeps;         /* Picard sweeps of the energy equation (>= 1)                    */
  int32_t solver;                  /* gea_solver                                                     */
  double tol;                      /* stop when ||b - A x||_2 <= tol ||b||_2                         */
  int32_t max_iter;                /* iteration cap of one solve (FP64 CG iterations, or the sum of
                                      inner iterations in the refined forms)                         */
  int32_t check_every;             /* host reads the convergence flag every this many iterations     */
  double inner_tol;                /* relative tolerance of each inner solve (refined forms)         */
  int32_t learned_steps;           /* learned form: network-preconditioned flexible-CG iterations
                                      per solve before Jacobi-PCG continues (>= 1; 1 = the learned
                                      initial guess with an optimal step length).  At most: the
                                      iteration stops (a fallback) once ||r|| falls less than 10 %
                                      over 2 iterations or grows past twice its start, and
                                      (with more than one step) a correction leaving the true
                                      residual above its start is dropped                            */
  double inner_target;             /* refined forms: an inner solve aims at inner_target * tol ||b||
                                      for the outer residual (in (0, 1]; 0 selects 0.8)            */
  int32_t learned_always;          /* learned form: 0 = per corrector, run the network only while
                                      the inner iterations it saves (running averages with and
                                      without it, the other way re-tried after 16 solves, the
                                      period doubling up to 256 while the choice holds) take
                                      longer than one application (both timed on the device);
                                      1 = on every solve                                          */
  int32_t energy_form;             /* Step 2: 0 = total-energy form (flux phi I4(e + R T)); 1 = the
                                      enthalpy form of eq. step3_sd (h = c_p T, lagged p^{n-1} and
                                      K^{n-1} in b~_e, gravity work rho* g w*)                      */
  int32_t transport;               /* Steps 1-2: 0 = explicit transport (Picard sweeps, implicit
                                      diffusion of the energy); 1 = implicit transport as eqs.
                                      step2_sd (Step 1) and step3_sd write it: per velocity
                                      component and once for T a non-symmetric system, solved by
                                      Jacobi-preconditioned BiCGStab to 1e-13                      */
} gea_params;

/* initial perturbation of Sec. 4: kind 0 none; 1 cosine bubble
 * theta' = amp/2 (1 + cos(pi r/rc)) for r <= rc (eq. dcEqn1); 2 uniform
 * bubble theta' = amp for r <= rc (eq. dcEqn2).  yc is unused in 2D. */
typedef struct { int32_t kind; double xc, yc, zc, rc, amp; } gea_bubble;

typedef struct {
  int32_t iters;        /* CG iterations (FP64 form) or inner iterations summed (refined forms) */
  int32_t outer_iters;  /* refinement steps (0 for the FP64 form)                               */
  int32_t fallbacks;    /* learned form: times the Jacobi-PCG fallback took over                */
  int32_t status;       /* gea_status of this solve                                             */
  double rel_res0;      /* ||b - A x0|| / ||b||                                                 */
  double rel_res;       /* residual norm at exit / ||b||: recursive (FP64 form) or true (refined) */
} gea_solve_stats;

typedef struct {
  int32_t steps_done;
  int32_t n_solves;            /* solves of the last step (= n_corr)                   */
  gea_solve_stats solve[8];    /* per corrector, last step                             */
  int64_t total_iters;         /* all solves of this call                              */
  int64_t total_solves;
  double eos_mismatch;         /* max |rho^{n+1} - p^{n+1}/(R T^{n+1})| of the last step */
  double mass;                 /* sum of rho^{n+1} V after the last step               */
  double max_rel_res;          /* largest exit residual (rel_res) of all solves of this call */
  int64_t total_fallbacks;     /* learned form: fallbacks of all solves of this call   */
  int64_t energy_iters;        /* CG iterations of the Step-2 energy solves of this call */
  int64_t transport_iters;     /* implicit transport: BiCGStab iterations of this call   */
} gea_step_stats;

/* field selectors for gea_get_fields (bit mask; output packed in bit order) */
enum {
  GEA_FIELD_RHO = 1u << 0,
  GEA_FIELD_U = 1u << 1,       /* ndim blocks */
  GEA_FIELD_T = 1u << 2,
  GEA_FIELD_PPRIME = 1u << 3,
  GEA_FIELD_P = 1u << 4,
  GEA_FIELD_C = 1u << 5,       /* pressure system of the last assembly: c    */
  GEA_FIELD_D = 1u << 6,       /*                                          D  */
  GEA_FIELD_B = 1u << 7,       /*                                          b  */
  GEA_FIELD_PHI = 1u << 8,     /* face mass flux of the state: ndim blocks,
                                  block d, value P: the face between cell P
                                  and cell P + stride_d (0 where P is at the
                                  upper wall); strides 1, nx, nx*ny (3D) or
                                  1, nx (2D) */
  GEA_FIELD_HISTORY = 1u << 9  /* 2 blocks: p^{n-1} and K^{n-1} of the
                                  enthalpy form's lagged terms (a state
                                  without history reports its own p and K) */
};

/* Bytes of device workspace needed for this mesh and parameter set. */
gea_status gea_workspace_bytes(const gea_mesh* mesh, const gea_params* params, size_t* bytes);

/* Create a context for a uniform hexahedral mesh of nx x ny x nz cells over
 * lx x ly x lz metres, enclosed by impenetrable free-slip walls (the
 * finite-volume setting of Sec. 3 and the closed box of Sec. 4; ny == 1 is
 * the one-cell-thick xz-plane).  params holds the constants of Sec. 2 (R,
 * c_p, c_v, g), the viscosity of Remark 1 and the time step of Sec. 3.
 * hip_stream is a hipStream_t (NULL = default stream);
 * workspace is device memory of at least gea_workspace_bytes, owned by the
 * caller and kept alive until gea_destroy.  Returns GEA_ERR_ARG for
 * non-positive sizes or constants, more than 2^31 - 1 cells, or a short
 * workspace. */
gea_status gea_init_mesh(const gea_mesh* mesh, const gea_params* params, void* hip_stream,
                         void* workspace, size_t workspace_bytes, gea_ctx** out);

/* Change solver form and tolerances of an existing context. */
gea_status gea_set_solver(gea_ctx* ctx, int32_t solver, double tol, int32_t max_iter,
                          double inner_tol);

/* Build the initial state of Sec. 4 on the device (eqs. rho_wb, dcEqn1,
 * dcEqn2, e0): a neutral atmosphere with theta0, a discretely hydrostatic
 * background column (p'_{k+1} - p'_k = g z_{k+1/2} (rho_{k+1} - rho_k)), the
 * temperature perturbed by theta' at unchanged pressure, u = 0, and the
 * face mass flux of those cell fields (0, since u = 0). */
gea_status gea_init_bubble(gea_ctx* ctx, const gea_bubble* bubble);

/* Copy a state in: the given fields of the problem statement of Sec. 3
 * (rho^n, u^n, T^n, p^n) and the split pressure p'^n = p^n + rho^n g z of
 * eq. p_split.  rho, T, p_prime, p: ncell values; u: ndim*ncell;
 * T_bg: nz values (background temperature column that the energy diffusion
 * term subtracts).  All pointers of the given kind, none may be NULL.  The
 * state's face mass flux, which Steps 1-3 transport with, becomes the
 * fourth-order interpolation I4(rho u . n)_f S_f of these fields (eq. e1_d;
 * 0 on the walls); gea_set_face_flux replaces it. */
gea_status gea_set_state(gea_ctx* ctx, const double* rho, const double* u, const double* T,
                         const double* p_prime, const double* p, const double* T_bg,
                         gea_ptr_kind kind);

/* Replace the current state's face mass flux (layout of GEA_FIELD_PHI,
 * ndim*ncell values of the given kind; values on the upper walls are
 * ignored and stored as 0).  A step transports with the flux of the state it
 * starts from and leaves the last corrector's corrected flux for the next
 * one (Sec. 3, Steps 1-3 and eq. e1_d), so a state copied out with
 * gea_get_fields (all fields and GEA_FIELD_PHI) and copied back in with
 * gea_set_state and this call continues bitwise as the original would. */
gea_status gea_set_face_flux(gea_ctx* ctx, const double* phi, gea_ptr_kind kind);

/* Give the current state the lagged terms p^{n-1}, K^{n-1} (ncell values
 * each, of the given kind) that the enthalpy form of Step 2 (energy_form 1;
 * eq. step3_sd, b~_e) reads.  A step in that form hands p^n, K^n = |u^n|^2/2
 * to the next state; a state without history (after gea_init_bubble,
 * gea_set_state, or a step in the total-energy form) takes its own p and K,
 * so that its first step has no lagged terms. */
gea_status gea_set_history(gea_ctx* ctx, const double* p_prev, const double* K_prev,
                           gea_ptr_kind kind);

/* Advance nsteps time steps (Sec. 3, Steps 1-3).  stats may be NULL. */
gea_status gea_step(gea_ctx* ctx, int32_t nsteps, gea_step_stats* stats);

/* Assemble the pressure system the next step's first corrector would solve
 * (Steps 1-2 and Step 3a-b from the current state, without changing it) and
 * solve it with the context's solver.  b: NULL to use the assembled
 * right-hand side, else ncell values that replace it.  x: ncell values, in:
 * initial guess, out: solution. */
gea_status gea_pressure_solve(gea_ctx* ctx, const double* b, double* x, gea_ptr_kind kind,
                              gea_solve_stats* stats);

/* y = A x with the operator of the last assembly (gea_pressure_solve or the
 * last corrector of gea_step). */
gea_status gea_apply_pressure_operator(gea_ctx* ctx, const double* x, double* y,
                                       gea_ptr_kind kind);

/* Extrema of the current state, as the paper reports them for its validation
 * runs (Sec. 4, Tables 1 and 3): the velocity components and the potential
 * temperature perturbation theta' = T/pi - theta0, pi = (p/p0)^{R/c_p}
 * (Sec. 2, eqs. theta, theta_split; p0 and theta0 from the parameters).
 * v is 0 in 2D.  Computed on the device; returns after the copy. */
typedef struct {
  double u_min, u_max, v_min, v_max, w_min, w_max, theta_min, theta_max;
} gea_extrema;
gea_status gea_state_extrema(gea_ctx* ctx, gea_extrema* out);

/* Copy the selected fields out, packed in bit order (see GEA_FIELD_*): the
 * end-of-step state (rho, u, T, p', p)^{n+1} of the problem statement of
 * Sec. 3, and the coefficients c, D and right-hand side b of the pressure
 * system (eq. p_prime_sd, in the re-derived form stated at the top of this
 * file) of the last assembly.  out: the caller's array of (number of
 * selected fields, counting U as ndim) x ncell values, of the given kind;
 * with GEA_DEVICE the copy is ordered on the context's stream. */
gea_status gea_get_fields(gea_ctx* ctx, uint32_t field_mask, double* out, gea_ptr_kind kind);

/* Measurement support.  With timing on, every kernel launch is bracketed by
 * two events on the context's stream and its device time is summed per
 * kernel class:
 *   0 FP64 CG iteration kernel (the scalars of the iteration before it from
 *     that iteration's partials, except at the start of a batch of
 *     iterations; the previous update of r and x, the new direction p,
 *     q = A p, the iteration's partial dot products)
 *   1 FP64 CG scalar kernel (one workgroup, at the end of each batch:
 *     alpha, beta, stop test)
 *   2 FP32 inner CG iteration kernel  3 FP32 inner CG scalar kernel
 *   4 solver set-up kernels (initial residual and its scalars, refinement
 *     residual and correction, FP32 coefficient copy)
 *   5 explicit step kernels (Steps 1-3 outside the solve)
 *   6 learned network kernels
 *   7 Step-2 energy solves (CG set-up, iteration and scalar kernels), and
 *     with transport = 1 the BiCGStab solves of Steps 1 and 2
 * reset = 1 clears the sums.  Timing adds two event records per launch. */
gea_status gea_kernel_timing(gea_ctx* ctx, int32_t on, int32_t reset);

/* Summed device milliseconds and launch counts per class (8 entries each). */
gea_status gea_kernel_times(gea_ctx* ctx, double* ms, int64_t* launches);

/* Average device milliseconds of one launch of the CG kernels on the
 * pressure system of the last assembly, each launched reps times back to
 * back between two events on the context's stream: ms[0] FP64 iteration
 * kernel, ms[1] FP64 scalar kernel, ms[2] FP32 iteration kernel, ms[3] FP32
 * scalar kernel (iteration 1 of a fresh solve inside a batch: it forms
 * iteration 0's scalars and applies its update, as every later one does).  Uses scratch
 * vectors only; the state is not changed. */
gea_status gea_time_solver_kernels(gea_ctx* ctx, int32_t reps, double* ms);

/* Average device milliseconds of one launch of each of the six forward
 * convolutions of the learned form's network (ms[6], layers in the order of
 * include/gea_learned.h), each launched reps times back to back between two
 * events on the context's stream on the network's current activations, and
 * the algorithmic GFLOP of one launch (2 x cells x C_out x taps x C_in with
 * the logical channel counts; gflop[6]).  Needs loaded weights
 * (GEA_ERR_STATE otherwise); overwrites only the network's activations. */
gea_status gea_time_network(gea_ctx* ctx, int32_t reps, double* ms, double* gflop);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the FP64
 * Jacobi-PCG solve of gea_pressure_solve's FP64 form on a system the caller
 * passes, with every work vector, partial sum and solver scalar in one
 * static device array of the library (about 60 MB per GPU, held from the
 * first call on a device until the process ends).  It allocates nothing
 * and needs no context.
 *   mesh: at most 2^20 cells (GEA_ERR_ARG beyond, see gea_last_error(NULL));
 *   c, D, b: ncell device values of the system c_i x_i + sum_f w_f (x_i -
 *     x_nb) = b_i, w_f = (D_P + D_N)/2 S_f/d_f (as gea_get_fields returns
 *     them); x: ncell device values, in: initial guess, out: solution;
 *   stops at ||b - A x||_2 <= tol ||b||_2 (recursive residual) or after
 *   max_iter iterations (GEA_ERR_NOCONV); hip_stream: a stream of the
 *   current device (NULL = default stream); stats: host, filled.
 * Returns after the solve completed.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other threads, other streams) race
 * and give wrong results. */
gea_status gea_pressure_solve_static(const gea_mesh* mesh, const double* c, const double* D,
                                     const double* b, double* x, double tol, int32_t max_iter,
                                     void* hip_stream, gea_solve_stats* stats);

/* Release the context (the workspace stays with its owner). */
void gea_destroy(gea_ctx* ctx);

/* Last error message of this context (or of the last failed gea_init_mesh
 * when ctx is NULL). */
const char* gea_last_error(const gea_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
