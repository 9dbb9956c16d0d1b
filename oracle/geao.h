/*
 * geao.h -- plain, slow FP64 CPU oracle of one segregated pressure-based time
 * step of the dry compressible Euler equations (GEA, arXiv:2303.10499, Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * this library.  It shares no code, header or constant table with the GPU
 * library; both sides only see the same plain-number inputs.
 *
 * What it computes (each function cites the passage it follows):
 *   - initial state of the rising-bubble tests (Sec. 4, eqs. rho_wb, dcEqn1,
 *     dcEqn2, e0) with a discretely balanced hydrostatic background;
 *   - Step 1 (eqs. e1_d, step2_sd, step1_3sd): mass flux, density predictor,
 *     momentum predictor, kinetic energy;
 *   - Step 2 (eqs. step3_sd, step3_2sd, step3_3sd) in total-energy form
 *     (eq. ent with e = c_v T + K + g z): energy sweeps, e -> T, EOS density;
 *   - Step 3 (eqs. step2_sd [corrector], p_prime_sd, step4_4sd) with PISO
 *     correctors: H operator, predicted face flux, pressure equation, Jacobi
 *     preconditioned CG, flux and velocity correction, end-of-step update.
 * Discrete operators follow Sec. 3's last paragraph: 2nd-order gradient and
 * Laplacian, 4th-order interpolation in the convective (divergence) terms.
 *
 * Layout: every field is a structure-of-arrays FP64 vector over the cells,
 * index i + nx*(j + ny*k), x fastest, z vertical.  ny == 1 means the 2D
 * xz-plane (directions x, z; velocity components u, w).  Otherwise 3D
 * (directions x, y, z; components u, v, w).  Velocities and face arrays hold
 * ndim consecutive blocks of ncell doubles.  A face array for direction d
 * stores, at index P, the value on the face between cell P and its +d
 * neighbour; on the +d wall face it stores 0.
 *
 * Readings of passages that are garbled or silent are listed in the C file
 * next to the code they decide.
 */
#ifndef GEAO_H
#define GEAO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int32_t nx, ny, nz; double lx, ly, lz; } geao_mesh;

typedef struct {
  double R, cp, cv, g, p0, theta0, mu, Pr, dt;
  int32_t n_corr, n_energy_sweeps;
  double tol;
  int32_t max_iter;
  int32_t energy_form;   /* Step 2: 0 total-energy form (geao_energy), 1 the
                            enthalpy form of eq. step3_sd (geao_energy_enthalpy) */
  int32_t transport;     /* 0: explicit Picard sweeps of the transport terms;
                            1: Steps 1-2 implicit in the transported quantity,
                            BiCGStab solves (geao_momentum_predictor_implicit,
                            geao_energy_implicit) */
} geao_params;

/* kind 0: no perturbation; 1: cosine theta' = amp/2 (1 + cos(pi r / rc)) for
 * r <= rc (eq. dcEqn1, amp = theta_c); 2: uniform theta' = amp for r <= rc
 * (eq. dcEqn2).  yc is ignored in 2D. */
typedef struct { int32_t kind; double xc, yc, zc, rc, amp; } geao_bubble;

typedef struct {
  int32_t iters, converged;
  double rel_res0;       /* ||b - A x0|| / ||b||                       */
  double rel_res;        /* recursive residual norm at exit / ||b||    */
  double true_rel_res;   /* ||b - A x|| / ||b|| recomputed at exit     */
} geao_solve_stats;

typedef struct {
  int32_t n_solves;
  geao_solve_stats solve[16];
  double eos_mismatch;   /* max |rho^{n+1} - p^{n+1} / (R T^{n+1})|     */
} geao_step_stats;

enum { GEAO_OK = 0, GEAO_ERR_ARG = -1, GEAO_ERR_NOCONV = -4, GEAO_ERR_NAN = -5 };

/* relative residual to which each energy sweep's implicit-diffusion system
 * is solved (Step 2, see geao_energy) */
#define GEAO_ENERGY_TOL 1e-13
/* relative residual of the implicit-transport solves (transport = 1) */
#define GEAO_TRANSPORT_TOL 1e-13

int geao_ndim(const geao_mesh* m);

/* ---- initial state (Sec. 4) ------------------------------------------ */
/* Fills rho, u (ndim*ncell), T, pp (= p'), p, and Tbg (nz values, the
 * background temperature column used by the energy diffusion term). */
int geao_init_bubble(const geao_mesh* m, const geao_params* q, const geao_bubble* b,
                     double* rho, double* u, double* T, double* pp, double* p, double* Tbg);

/* ---- discrete operators (Sec. 3, last paragraph) ---------------------- */
void geao_face_interp4(const geao_mesh* m, const double* s, int dir, double* out);
void geao_face_sngrad(const geao_mesh* m, const double* s, int dir, double* out);
/* cell vector from face-normal values; faces is ndim face arrays */
void geao_reconstruct(const geao_mesh* m, const double* faces, double* out);
/* (1/V) sum over the faces of a cell of the outward face flux */
void geao_divergence(const geao_mesh* m, const double* faces, double* out);
/* sum_f mu snGrad(u_c)_f S_f for velocity component comp, with the wall
 * treatment of free-slip impenetrable walls (not divided by V) */
void geao_viscous(const geao_mesh* m, const double* uc, int comp, double mu, double* out);
/* sum_out phi_f I4(s)_f (not divided by V) */
void geao_convective(const geao_mesh* m, const double* phi, const double* s, double* out);
/* potential g z at cell centres */
void geao_potential(const geao_mesh* m, const geao_params* q, double* out);

/* ---- the sub-steps of one time step (Sec. 3) -------------------------- */
void geao_mass_predictor(const geao_mesh* m, const geao_params* q, const double* rho,
                         const double* u, double* phi, double* rho_star);
/* phi = I4(rho u . n) S on interior faces (ndim face arrays; 0 on walls):
 * the flux of a state given by its cell fields alone */
void geao_face_mass_flux(const geao_mesh* m, const double* rho, const double* u, double* phi);
/* rho* = rho^n - dt/V sum_out phi^n with the state's flux */
void geao_density_predictor(const geao_mesh* m, const geao_params* q, const double* rho,
                            const double* phi, double* rho_star);
void geao_momentum_predictor(const geao_mesh* m, const geao_params* q, const double* rho,
                             const double* u, const double* pp, const double* rho_star,
                             const double* phi, double* u_star);
void geao_energy(const geao_mesh* m, const geao_params* q, const double* rho, const double* u,
                 const double* T, const double* u_star, const double* rho_star,
                 const double* phi, const double* Tbg, double* T_new);
/* Implicit transport (transport = 1; see geao.c): operators, their
 * diagonals (comp >= 0: momentum component; comp = -1: energy with
 * coefficient cT), the BiCGStab solve of a momentum system, and the two
 * implicit predictors (u_star: in the initial guess, out the solution). */
void geao_momentum_operator(const geao_mesh* m, const geao_params* q, const double* rho_star,
                            const double* phi, int comp, const double* x, double* y);
void geao_energy_operator(const geao_mesh* m, const geao_params* q, const double* cT,
                          const double* phi, const double* x, double* y);
void geao_transport_diag(const geao_mesh* m, const geao_params* q, const double* rho_star,
                         const double* cT, const double* phi, int comp, double* diag);
int geao_bicgstab_momentum(const geao_mesh* m, const geao_params* q, const double* rho_star,
                           const double* phi, int comp, const double* b, double* x, double tol,
                           int max_iter, geao_solve_stats* st);
int geao_momentum_predictor_implicit(const geao_mesh* m, const geao_params* q, const double* rho,
                                     const double* u, const double* pp, const double* rho_star,
                                     const double* phi, double* u_star);
int geao_energy_implicit(const geao_mesh* m, const geao_params* q, const double* rho,
                         const double* u, const double* T, const double* p, const double* p_old,
                         const double* K_old, const double* u_star, const double* rho_star,
                         const double* phi, const double* Tbg, double* T_new);
/* Step 2 in the enthalpy form of eq. step3_sd (see geao.c); p_old, K_old:
 * p^{n-1} and K^{n-1} of the lagged terms of b~_e */
void geao_energy_enthalpy(const geao_mesh* m, const geao_params* q, const double* rho,
                          const double* T, const double* p, const double* p_old,
                          const double* K_old, const double* u_star, const double* rho_star,
                          const double* phi, const double* Tbg, double* T_new);
void geao_eos_coeffs(const geao_mesh* m, const geao_params* q, const double* p,
                     const double* T_new, const double* rho_star,
                     double* rho23, double* psi, double* c, double* D);
void geao_H(const geao_mesh* m, const geao_params* q, const double* rho, const double* u,
            const double* u_prev, const double* phi, double* H);
void geao_predicted_flux_rhs(const geao_mesh* m, const geao_params* q, const double* rho,
                             const double* rho23, const double* psi, const double* D,
                             const double* H, double* phi_tilde, double* b);
void geao_apply_A(const geao_mesh* m, const double* c, const double* D, const double* x,
                  double* y);
int geao_pcg(const geao_mesh* m, const double* c, const double* D, const double* b, double* x,
             double tol, int max_iter, geao_solve_stats* st);
void geao_correct(const geao_mesh* m, const geao_params* q, const double* pp,
                  const double* rho23, const double* H, const double* D,
                  const double* rho_star, const double* phi_tilde, double* phi, double* u);
void geao_finalize(const geao_mesh* m, const geao_params* q, const double* rho_old,
                   const double* phi, const double* pp, const double* rho23, const double* psi,
                   double* rho_new, double* p_new, double* eos_mismatch);

/* Steps 1-2 and the first corrector's Step 3a-b of the step that would start
 * from this state: returns the pressure system (c, D, b) it would solve.
 * p_old, K_old: the state's p^{n-1}, K^{n-1} (read by the enthalpy form). */
int geao_pressure_system(const geao_mesh* m, const geao_params* q, const double* rho,
                         const double* u, const double* T, const double* pp, const double* p,
                         const double* phi, const double* p_old, const double* K_old,
                         const double* Tbg, double* c, double* D, double* b);

/* One full step n -> n+1, in place; phi (ndim face arrays, the face flux of
 * the state) in: phi^n, out: phi^{n+1} (the last corrector's flux); p_old,
 * K_old in: p^{n-1}, K^{n-1}, out: p^n, K^n (the enthalpy form's lagged
 * terms; kept up to date in both forms). */
int geao_step(const geao_mesh* m, const geao_params* q, double* rho, double* u, double* T,
              double* pp, double* p, double* phi, double* p_old, double* K_old,
              const double* Tbg, geao_step_stats* st);

/* potential temperature fluctuation theta' = T/(p/p0)^{R/cp} - theta0 (eqs. theta, theta_split) */
void geao_theta_prime(const geao_mesh* m, const geao_params* q, const double* T, const double* p,
                      double* out);

/* threads the per-cell loops run on: 1, or the OpenMP team size of the
 * -fopenmp build (timing only; both builds give the same results) */
int geao_threads(void);

#ifdef __cplusplus
}
#endif
#endif
