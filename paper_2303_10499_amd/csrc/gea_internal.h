// gea_internal.h -- declarations shared by the library's translation units:
// mesh geometry passed to kernels by value, physical constants, device
// scalars of the solvers, and the host-side launchers of every kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gea {

constexpr int kBlock = 256;     // threads per workgroup (4 waves of 64)
constexpr int kMaxDim = 3;

// Uniform hexahedral mesh.  Direction d = 0..ndim-1 is x, (y,) z; z is the
// last direction.  Index P = i + nx*(j + ny*k).
struct Geo {
  int ndim;
  int nx, ny, nz;
  int nc;                  // number of cells (< 2^31)
  int n[kMaxDim];          // cells along direction d
  int st[kMaxDim];         // index stride of direction d
  double h[kMaxDim];       // spacing along d
  double S[kMaxDim];       // area of the faces normal to d
  double V;                // cell volume
  double dz;
  double inv_h[kMaxDim];   // 1/h (0 for an absent direction)
  double inv_V;            // 1/V
};

struct Phys {
  double R, cp, cv, g, mu, Pr, dt, p0, theta0;
  double inv_dt, inv_cv;   // 1/dt, 1/c_v
};

template <int NDIM, typename T = double>
struct Vec {
  T* p[NDIM];
};

// Device-resident solver scalars.  Written by the one-workgroup set-up and
// scalar kernels, read by later kernels on the stream and by the host.
struct CgScalars {
  double rz;        // <r, z> of the current iterate
  double rr;        // ||r||^2
  double bb;        // ||b||^2 (of the system being solved)
  double alpha;     // step length of the update the next iteration kernel applies
  double beta;      // its direction coefficient
  double tol2;      // tol^2
  double aux[6];    // reduction results of the step kernels
  double rr0;       // ||r||^2 where a resumed solve started
  int iter;         // completed iterations
  int max_iter;
  int done;         // 1 once converged or failed
  int status;       // 0 ok, -4 no convergence, -5 non-finite
  int fin;          // 1: the next iteration kernel applies the last x update only
  int done_iter;    // the launch that applied the last update (later launches of its
                    // batch return at once); -1 while the solve runs
  int corrected;    // 1: that last update also added the iterate to the outer one
                    // (an inner solve of the refinement, CgVectors::xo)
};

// Number of workgroups of the grid-stride kernels: a fixed multiple of the
// CU count, so the per-workgroup partial sums stay few.
int grid_for(int nc);

// Launch shape of the z-marching stencil kernels: kc planes per chunk and
// the number of workgroups (one per column tile and chunk).
constexpr int kMaxZBlocks = 4096;
struct ZPlan {
  int kc;
  int blocks;
};
ZPlan zplan(const Geo& G);
// 3D column tiles of 64 x ty cells (64 ty threads a workgroup) marching
// chunks of kc planes (fewer chunks where zplan would need them); never more
// workgroups than zplan's for ty >= 4 and kc >= its chunk
ZPlan zplan3(const Geo& G, int ty, int kc);

// ---- explicit step kernels (gea_step.hip) ----------------------------------
// The refinement's first residual r = b - A x formed in the pass that forms
// b (3D): the FP32 inner right-hand side, optionally the cleared inner
// iterate and direction, and the 2 + 2 per-workgroup partials the residual
// check reads (outer: ||r||^2, ||b||^2; inner: <r32, r32/diag>, ||r32||^2).
struct RhsResidual {
  const double* x;
  float* r32;
  float* x32;
  int zero_inner;
  double* o_part;
  double* i_part;
};

// the face mass flux I4(rho u . n)_f S_f of a state given by its cell fields
// (0 on walls): face d of cell P is the face between P and P + st[d]
void launch_face_mass_flux(hipStream_t s, const Geo& G, const double* rho, double* const* u,
                           double* const* phi);
// sets the flux of the upper wall faces to 0
void launch_clear_wall_faces(hipStream_t s, const Geo& G, double* const* phi);
// Step 1 (rho* from the state's face flux phi, e^n, momentum predictor): one
// pass in 3D, the two kernels in 2D; pp_copy (or null) also receives p' (the
// solve's initial guess), Ks (or null) K* = |u*|^2/2 for the energy sweeps
void launch_step1(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                  double* const* u, const double* T, const double* pp, double* const* phi,
                  double* rho_star, double* e0, double* const* u_star, double* pp_copy,
                  double* const* b_out = nullptr,  // b_out: implicit transport's V (rho u/dt - R(F))
                  double* Ks = nullptr);
// Step 2, one sweep: the right-hand side b, coefficient c and 1/diag of the
// implicit-diffusion system for T, the initial guess x = T_prev, and the
// solve's set-up (r = b - A x, partials <r, r/diag>, ||r||^2 in
// u_part and ||b||^2 in b_part, one per workgroup); returns the workgroup
// count (k_cg_start's nu).  The system's D is (mu/Pr) c_p everywhere.  The
// sweep stages a_prev and T_prev: with ks (and always in the enthalpy form)
// a_prev = Ks (K*, from Step 1) and the transported quantity is formed from
// T and K*; else (the first total-energy sweep) a_prev = e^n.
int launch_energy_rhs(hipStream_t s, const Geo& G, const Phys& ph, bool enth, bool ks,
                      const double* rho, const double* e0, const double* a_prev,
                      const double* T_prev, double* const* phi, const double* rho_star,
                      const double* Ks, const double* Tbg, double* b, double* c,
                      double* x, double* r, double* u_part, double* b_part);
// after the last sweep's solve: the EOS density and pressure-equation
// coefficients rho23, psi, c, D
void launch_energy_post(hipStream_t s, const Geo& G, const Phys& ph, const double* T,
                        const double* p, const double* rho_star, double* rho23, double* psi,
                        double* c, double* D);
// Step 2 in enthalpy form (enth = true above): p^{n-1} = p, K^{n-1} = |u|^2/2
// for a state without history; and the sweep-independent balance q and the
// next state's p^n, K^n
void launch_history_init(hipStream_t s, const Geo& G, const double* p, double* const* u,
                         double* pm, double* Km);
void launch_enthalpy_prep(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                          const double* T, const double* p, const double* pm, const double* Km,
                          double* const* u, double* const* u_star, const double* rho_star,
                          double* q, double* pm_next, double* Km_next);
// relative residual to which each energy sweep's system is solved
constexpr double kEnergyTol = 1e-13;
void launch_H(hipStream_t s, const Geo& G, const Phys& ph, const double* rho, double* const* u,
              double* const* u_prev, double* const* phi, double* const* H);
int launch_rhs(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                const double* rho23, const double* psi, const double* c, const double* D,
                double* const* H, double* b, double* dinv, float* c32, float* D32,
                float* dinv32,  // FP32 copies of c, D, 1/diag written unless c32 is null;
                                // 1/diag written unless dinv is null
                const RhsResidual* res = nullptr);  // returns the residual partials' count, 0: not formed
void launch_correct(hipStream_t s, const Geo& G, const Phys& ph, const double* pp,
                    const double* rho23, const double* psi, double* const* H, const double* D,
                    const double* rho_star, double* const* u_out, bool last,
                    const double* rho_old, double* rho_new, double* p_new,
                    double* const* phi_out,  // last: the corrected face fluxes
                    double* partials, CgScalars* sc);
// extrema (min, max) of u, v (0 in 2D), w and theta' into out[8]; part holds
// 8 values per workgroup of the grid-stride grid
int launch_extrema(hipStream_t s, const Geo& G, const Phys& ph, double* const* u, const double* T,
                   const double* p, double* part, double* out);
void launch_init_column(hipStream_t s, const Geo& G, const Phys& ph, double* rho_a,
                        double* pp_a, double* Tbg);
void launch_init_fields(hipStream_t s, const Geo& G, const Phys& ph, int kind, double xc,
                        double yc, double zc, double rc, double amp, const double* rho_a,
                        const double* pp_a, const double* Tbg, double* rho, double* const* u,
                        double* T, double* pp, double* p);

// ---- Jacobi-PCG kernels (gea_cg.hip) ----------------------------------------
// FP64 solve of A x = b; r, p, q are work vectors.  Iterations are enqueued
// in batches; a device flag turns the remaining launches of a batch into
// no-ops once the solve is done.
template <typename T>
struct CgVectors {
  T* x;
  T* r;    // residual and A p, double buffered by iteration parity (r, r1;
  T* r1;   // q, q1): the iteration kernel reads the old values with halo
  T* p0;   // while writing the new ones; so is the direction (p0, p1)
  T* p1;
  T* q;
  T* q1;
  const T* c;
  const T* D;     // null: D is Dc in every cell (the energy sweeps' system)
  const T* dinv;  // (with D null: unused, the iteration kernels form 1/diag from c;
                  // such a system starts with cg_start_from, not cg_init)
  const T* b;
  T Dc = T(0);
  // FP32 inner solve of the refinement: its outer FP64 iterate, to which the
  // last update adds the inner one (x + alpha p, not stored back to x); null
  // otherwise
  double* xo = nullptr;
};

// The vectors one iteration kernel reads (_in) and writes (_out).
template <typename T>
struct CgIter {
  T* x;
  const T* r_in;
  T* r_out;
  const T* q_in;
  T* q_out;
  const T* p_in;
  T* p_out;
  const T* c;
  const T* D;
  const T* dinv;
  T Dc;  // D in every cell when the kernel's CD flag is set (D unused)
  double* xo;  // (CgVectors::xo)
};

// Per-workgroup partial sums of one CG instance: s (iteration kernel, 7
// values per workgroup, in two sets by iteration parity: 14 ns doubles),
// u[1] (the set-up kernel's <r, z>, ||r||^2; u[0] is unused), b (||b||^2 at
// set-up).
struct CgWork {
  double* s;
  int ns;   // workgroups of the iteration kernel's grid (iter_grid of the precision)
  double* u[2];
  double* b;
  CgScalars* sc;
};

template <typename T>
int iter_grid(const Geo& G);  // workgroups of the CG iteration kernel in precision T
template <typename T>
void cg_init(hipStream_t s, const Geo& G, const CgVectors<T>& v, const CgWork& w, double tol,
             int max_iter);
// iteration `iter` of a solve set up by cg_init / launch_residual64.  The
// host enqueues batches of iterations and ends each with cg_scalars: the
// first iteration kernel of a batch takes the scalars the kernel before it
// left (fold = false); each later one (fold = true) forms the scalars of the
// iteration before it from that iteration's partials, in every workgroup.
// A grid above 512 workgroups does not fold (cg_folds false): the host then
// follows every iteration kernel with cg_scalars.
template <typename T>
void cg_iter_kernel(hipStream_t s, const Geo& G, const CgVectors<T>& v, int iter, const CgWork& w,
                    bool fold);
void cg_scalars(hipStream_t s, const Geo& G, int iter, const CgWork& w);
bool cg_folds(const CgWork& w);
// Jacobi-PCG resumed on the FP32 inner system from its current iterate and
// residual, keeping the set-up's ||b||^2 and tolerance: its scalars from
// 2 x n partials <r, r/diag>, <r, r> of that residual (fcg_handover forms
// them); then cg_iter_kernel / cg_scalars from iteration 0
void cg_resume_scalars(hipStream_t s, const double* part, int n, const CgWork& w, int max_iter);
void launch_apply_A(hipStream_t s, const Geo& G, const double* c, const double* D,
                    const double* x, double* y);

// Mixed precision: FP64 residual r = b - A x and its FP32 copy as the inner
// right-hand side, outer stop test and inner setup; x += dx.  With a gate
// (the scalars of an inner solve enqueued ahead of the host's read) these
// kernels do nothing unless that solve is done, so a solve cut short by its
// batch can be continued on the same vectors.
// the residual check alone, on n partials a fused pass formed
void launch_residual_check(hipStream_t s, int n, double tol, double inner_tol, double target,
                           int inner_max, const double* o_part, const CgWork& w32,
                           CgScalars* sc64, const CgScalars* gate = nullptr);
// (zero_inner: also clear the inner iterate and first direction, which a
// Jacobi-PCG started on this set-up reads; the flexible CG needs neither)
void launch_residual64(hipStream_t s, const Geo& G, const double* c, const double* D,
                       const double* b, const double* x, const CgVectors<float>& v32,
                       double tol, double inner_tol, double target, int inner_max, double* o_part,
                       const CgWork& w32, CgScalars* sc64, bool zero_inner = true,
                       const CgScalars* gate = nullptr);
void launch_cast_coeffs(hipStream_t s, const Geo& G, const double* c, const double* D,
                        const double* dinv, float* c32, float* D32, float* dinv32);
// x += dx unless the inner solve's last update added it already (own: that
// solve's scalars) or, with a gate, that solve is not done
void launch_add_correction(hipStream_t s, const Geo& G, double* x, const float* dx,
                           const CgScalars* own, const CgScalars* gate = nullptr);
// y = b - y
void launch_sub(hipStream_t s, const Geo& G, const double* b, double* y);
// a = v
void launch_fill(hipStream_t s, const Geo& G, double* a, double v);

// ---- implicit transport (gea_bicg.hip) --------------------------------------
// Operator (times V): (A x)_P = rho*_P tcoef x_P + gamma sum_out phi I4(x)
//   + sum_f k_d (x_P - x_nb) + 2 k_d x_P on the walls normal to d = wall_comp.
struct TrOp {
  const double* rho_star;
  double tcoef;
  const double* phi[3];
  double gamma;
  double k[3];
  int wall_comp;  // -1: no wall term
};
// BiCGStab work vectors (ncell each); r also holds s between the half steps
struct TrVecs {
  double *b, *dinv, *r, *rh, *p, *v, *y, *z, *t;
};
struct TrScalars {
  double bb, rr, rr0, rho, rho_old, alpha, omega, beta, tol2;
  int iter, max_iter, status, done;  // status 0 ok, -4 no convergence or breakdown, -5 non-finite
};
// set-up of a momentum component (x0: the initial guess; v.b the right-hand
// side V (rho^n u^n/dt - R(F^n)) from Step 1's pass) or of the energy solve
// (writes the known transported part into w and T^n into x); each stores 2
// partials a workgroup (zplan(G).blocks workgroups) for launch_tr_start
void launch_tr_setup_mom(hipStream_t s, const Geo& G, const TrOp& op, const double* x0,
                         const TrVecs& v, double* part);  // v.b: the component's right-hand side
void launch_tr_setup_energy(hipStream_t s, const Geo& G, const Phys& ph, bool enth, const TrOp& op,
                            const double* rho, const double* e0, double* const* u_star,
                            double* w, const double* Tn, const double* Tbg, double* x,
                            const TrVecs& v, double* part);
void launch_tr_start(hipStream_t s, const Geo& G, const double* part, double tol, int max_iter,
                     TrScalars* sc);
// one BiCGStab iteration (nine launches; all return at once once sc->done)
void launch_tr_iteration(hipStream_t s, const Geo& G, const TrOp& op, double* x, const TrVecs& v,
                         double* part, TrScalars* sc);
// relative residual of the implicit-transport solves
constexpr double kTransportTol = 1e-13;
// a solve's scalars from the set-up partials another kernel formed (nu
// workgroups: <r, r/diag>, ||r||^2 in u_part, ||b||^2 in b_part)
void cg_start_from(hipStream_t s, const double* u_part, int nu, const double* b_part, double tol,
                   int max_iter, CgScalars* sc);

// ---- learned form: flexible CG (gea_fcg.hip) ----------------------------------
struct FcgScalars {
  double rr, bb, tol2;
  double s, inv_s;      // max |r| and its inverse (scale of the network input)
  double rz_prev[2];    // <z, r> of iterations of even / odd index
  double hist[10];      // ||r||^2 of the last ten iterations (the stall test reads 2 back)
  int iter, max_iter;
  int done;
  int status;           // 0 ok, 1 stalled, diverging or non-finite (fall back), 2 iteration cap
  int restart;          // the hand-over dropped the correction (the resumed solve starts at 0)
};

struct FcgVectors {
  float *d, *r, *r_old, *z, *p0, *p1, *q;
  float* r0;          // the starting residual, kept for the hand-over (or null)
  const float *c, *D;
  const float* dinv;  // 1/diag, for the resumed Jacobi-PCG's set-up
  double *part_d, *part_s, *part_u;
};

// flexible-CG set-up on the inner system whose ||b||^2, tolerance and done
// flag the refinement's residual check left in sys
void fcg_start(hipStream_t s, const Geo& G, const FcgVectors& v, const CgScalars* sys,
               int max_iter, FcgScalars* sc);
// one iteration once z = M(r) is in v.z: dots, direction + operator, update,
// check (last: the last one enqueued, which keeps no r_old).  Without r0
// (a single flexible step) the last one also sets up the Jacobi-PCG that
// resumes the solve: 2 x n partials <r, r/diag>, <r, r> in v.part_d, n the
// returned count, else 0 (then cg_resume_scalars finishes the set-up).
int fcg_iteration_after_z(hipStream_t s, const Geo& G, const FcgVectors& v, int iter, bool last,
                          FcgScalars* sc);
// hand-over after several flexible steps (v.r0 kept): v.r = r0 - A d afresh
// from the flexible CG's iterate d (or, when that is not finite or larger
// than r0, d = 0 and r = r0: sc->restart), then the resumed Jacobi-PCG's
// scalars in w.sc (max_iter iterations remain)
void fcg_handover(hipStream_t s, const Geo& G, const FcgVectors& v, const CgWork& w, int max_iter,
                  FcgScalars* sc);
// training pair: s = max |r0| (s_out[0], 1/s in s_out[1]); in_r = r0/s,
// in_a = c/diag, out_d = (x - x0)/s
void pair_outputs(hipStream_t s, const Geo& G, const double* r0, const double* c,
                  const double* dinv, const double* x, const double* x0, double* part,
                  double* s_out, float* in_r, float* in_a, float* out_d);

}  // namespace gea
