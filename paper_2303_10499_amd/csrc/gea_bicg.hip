// gea_bicg.hip -- implicit transport of Steps 1 and 2 (Sec. 3, eqs. step2_sd
// of Step 1 and step3_sd with their convective and diffusive terms at the
// new level): the matrix-free non-symmetric operators and BiCGStab with the
// Jacobi preconditioner on the right (van der Vorst's algorithm).
//
// One operator serves both systems (times the cell volume):
//   (A x)_P = c_P x_P + gamma sum_out phi_f I4(x)_f + sum_f k_d (x_P - x_nb)
//             + sum_{wall faces along d = wall_comp} 2 k_d x_P,
// c_P = rho*_P tcoef.  Momentum component m: tcoef = V/dt, gamma = 1,
// k_d = mu S_d/h_d, wall_comp = m (the wall-normal component vanishes on the
// wall, half a spacing away).  Energy (unknown T): tcoef = c_v V/dt or
// c_p V/dt, gamma = c_p, k_d = (mu/Pr) c_p S_d/h_d, adiabatic walls.  I4 is
// the cubic face interpolation (-1, 9, 9, -1)/16 with two cells on each
// side, else the linear mean; there is no convective flux through a wall.
//
// Every kernel of an iteration is a grid-stride pass (8.4 M cells: about
// 2048 workgroups); each stores one partial a workgroup for every dot
// product it forms, and a one-workgroup kernel sums them in workgroup order
// (bitwise reproducible) and updates the solver scalars.  All kernels of an
// iteration return at once when the scalars say the solve is done, so the
// host enqueues iterations in batches and reads the scalars once a batch.
#include <hip/hip_runtime.h>

#include "gea_internal.h"
#include "gea_reduce.h"

namespace gea {
namespace {

template <int NDIM>
struct TrOpD {
  const double* rho_star;
  double tcoef;
  const double* phi[NDIM];
  double gamma;
  double k[NDIM];
  int wall_comp;
};

template <int NDIM>
TrOpD<NDIM> dev_op(const TrOp& o) {
  TrOpD<NDIM> d;
  d.rho_star = o.rho_star;
  d.tcoef = o.tcoef;
  d.gamma = o.gamma;
  d.wall_comp = o.wall_comp;
  for (int i = 0; i < NDIM; ++i) {
    d.phi[i] = o.phi[i];
    d.k[i] = o.k[i];
  }
  return d;
}

template <int NDIM>
Vec<NDIM> uvec(double* const* a) {
  Vec<NDIM> v;
  for (int d = 0; d < NDIM; ++d) v.p[d] = a[d];
  return v;
}

__device__ __forceinline__ bool tr_done(const TrScalars* sc) {
  return __hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// face value of x between cell P (coordinate q along d, n cells) and P + st
__device__ __forceinline__ double i4_face(const double* __restrict__ x, int P, int st, int q, int n) {
  if (q >= 1 && q + 2 <= n - 1)
    return (-x[P - st] + 9.0 * x[P] + 9.0 * x[P + st] - x[P + 2 * st]) / 16.0;
  return 0.5 * (x[P] + x[P + st]);
}

// weight of the face's lower cell (q) or upper cell in its I4 value
__device__ __forceinline__ double i4_weight(int q, int n) {
  return (q >= 1 && q + 2 <= n - 1) ? 9.0 / 16.0 : 0.5;
}

// (A x)_P and, when diag is given, the diagonal entry
template <int NDIM>
__device__ __forceinline__ double tr_apply(const Geo& G, const TrOpD<NDIM>& op,
                                           const double* __restrict__ x, int P,
                                           double* diag = nullptr) {
  const double xc = x[P];
  const double c = op.rho_star[P] * op.tcoef;
  double conv = 0.0, cdiag = 0.0, lap = 0.0, ldiag = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    const int st = G.st[d], n = G.n[d], q = (P / st) % n;
    const double* f = op.phi[d];
    if (q + 1 < n) {
      const double fh = f[P];
      conv += fh * i4_face(x, P, st, q, n);
      cdiag += fh * i4_weight(q, n);
      lap += op.k[d] * (xc - x[P + st]);
      ldiag += op.k[d];
    } else if (op.wall_comp == d) {
      lap += 2.0 * op.k[d] * xc;
      ldiag += 2.0 * op.k[d];
    }
    if (q > 0) {
      const double fl = f[P - st];
      conv -= fl * i4_face(x, P - st, st, q - 1, n);
      cdiag -= fl * i4_weight(q - 1, n);
      lap += op.k[d] * (xc - x[P - st]);
      ldiag += op.k[d];
    } else if (op.wall_comp == d) {
      lap += 2.0 * op.k[d] * xc;
      ldiag += 2.0 * op.k[d];
    }
  }
  if (diag) *diag = c + op.gamma * cdiag + ldiag;
  return c * xc + op.gamma * conv + lap;
}

template <int N>
__device__ __forceinline__ void store_partials(double (&v)[N], double* part) {
  __shared__ double sh[N][kBlock / 64];
  Reducer<0u, N>::block(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) part[k * gridDim.x + blockIdx.x] = v[k];
  }
}

// ---- set-up ------------------------------------------------------------------

// momentum component: b = A u^n + c (x0 - u^n) (= V (rho^n u^n/dt - R(F^n))
// when x0 is the explicit predictor's u*), r = b - A x0, rh = r, p = v = 0;
// partials ||b||^2, ||r||^2
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_tr_setup_mom(Geo G, TrOpD<NDIM> op,
                                                         const double* __restrict__ un,
                                                         const double* __restrict__ x0, TrVecs v,
                                                         double* part) {
  double red[2] = {0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    double diag;
    const double aun = tr_apply<NDIM>(G, op, un, P);
    const double ax0 = tr_apply<NDIM>(G, op, x0, P, &diag);
    const double c = op.rho_star[P] * op.tcoef;
    const double b = aun + c * (x0[P] - un[P]);
    const double r = b - ax0;
    v.b[P] = b;
    v.dinv[P] = 1.0 / diag;
    v.r[P] = r;
    v.rh[P] = r;
    v.p[P] = 0.0;
    v.v[P] = 0.0;
    red[0] += b * b;
    red[1] += r * r;
  }
  store_partials<2>(red, part);
}

// the known part of Step 2's transported quantity: K* (+ Phi in the
// total-energy form)
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_tr_known(Geo G, Phys ph, Vec<NDIM> u_star, int enth,
                                                     double* __restrict__ w) {
  GEA_FOR_CELLS(P, G) {
    double kin = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) kin += u_star.p[d][P] * u_star.p[d][P];
    const int kz = P / G.st[NDIM - 1];
    w[P] = 0.5 * kin + (enth ? 0.0 : ph.g * (kz + 0.5) * G.dz);
  }
}

// energy: b = local - sum_out phi I4(w) + bg, local = V/dt (rho^n e^n - rho* w)
// (total energy, e0 = e^n) or V/dt q (enthalpy form, e0 = q); x = T^n (the
// initial guess, written into the solution buffer), r = b - A x, rh = r,
// p = v = 0; partials ||b||^2, ||r||^2
template <int NDIM, bool ENTH>
__global__ __launch_bounds__(kBlock) void k_tr_setup_energy(
    Geo G, Phys ph, TrOpD<NDIM> op, const double* __restrict__ rho, const double* __restrict__ e0,
    const double* __restrict__ w, const double* __restrict__ Tn, const double* __restrict__ Tbg,
    double* __restrict__ x, TrVecs v, double* part) {
  constexpr int Z = NDIM - 1;
  double red[2] = {0.0, 0.0};
  const double kcoef = ph.mu / ph.Pr * ph.cp;
  const double kdz = kcoef * G.S[Z] / G.h[Z];
  GEA_FOR_CELLS(P, G) {
    const double rs = op.rho_star[P];
    const double local = ENTH ? G.V / ph.dt * e0[P] : G.V / ph.dt * (rho[P] * e0[P] - rs * w[P]);
    double convw = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int st = G.st[d], n = G.n[d], q = (P / st) % n;
      if (q + 1 < n) convw += op.phi[d][P] * i4_face(w, P, st, q, n);
      if (q > 0) convw -= op.phi[d][P - st] * i4_face(w, P - st, st, q - 1, n);
    }
    const int k = P / G.st[Z], nz = G.n[Z];
    double bg = 0.0;
    if (k + 1 < nz) bg += kdz * (Tbg[k] - Tbg[k + 1]);
    if (k > 0) bg += kdz * (Tbg[k] - Tbg[k - 1]);
    const double b = local - convw + bg;
    double diag;
    const double ax = tr_apply<NDIM>(G, op, Tn, P, &diag);
    const double r = b - ax;
    x[P] = Tn[P];
    v.b[P] = b;
    v.dinv[P] = 1.0 / diag;
    v.r[P] = r;
    v.rh[P] = r;
    v.p[P] = 0.0;
    v.v[P] = 0.0;
    red[0] += b * b;
    red[1] += r * r;
  }
  store_partials<2>(red, part);
}

// ---- one iteration -----------------------------------------------------------

// p = r + beta (p - omega v), y = dinv p
__global__ __launch_bounds__(kBlock) void k_tr_dir(int nc, TrVecs v, const TrScalars* sc) {
  if (tr_done(sc)) return;
  const double beta = sc->beta, omega = sc->omega;
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < nc; P += gridDim.x * blockDim.x) {
    const double pn = v.r[P] + beta * (v.p[P] - omega * v.v[P]);
    v.p[P] = pn;
    v.y[P] = v.dinv[P] * pn;
  }
}

// v = A y; partial <rh, v>
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_tr_matvec_v(Geo G, TrOpD<NDIM> op, TrVecs v,
                                                        const TrScalars* sc, double* part) {
  if (tr_done(sc)) return;
  double red[1] = {0.0};
  GEA_FOR_CELLS(P, G) {
    const double av = tr_apply<NDIM>(G, op, v.y, P);
    v.v[P] = av;
    red[0] += v.rh[P] * av;
  }
  store_partials<1>(red, part);
}

// x += alpha y, s = r - alpha v (into r), z = dinv s; partial ||s||^2
__global__ __launch_bounds__(kBlock) void k_tr_half(int nc, double* __restrict__ x, TrVecs v,
                                                    const TrScalars* sc, double* part) {
  if (tr_done(sc)) return;
  const double alpha = sc->alpha;
  double red[1] = {0.0};
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < nc; P += gridDim.x * blockDim.x) {
    x[P] += alpha * v.y[P];
    const double s = v.r[P] - alpha * v.v[P];
    v.r[P] = s;
    v.z[P] = v.dinv[P] * s;
    red[0] += s * s;
  }
  store_partials<1>(red, part);
}

// t = A z; partials <t, s>, <t, t>
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_tr_matvec_t(Geo G, TrOpD<NDIM> op, TrVecs v,
                                                        const TrScalars* sc, double* part) {
  if (tr_done(sc)) return;
  double red[2] = {0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    const double t = tr_apply<NDIM>(G, op, v.z, P);
    v.t[P] = t;
    red[0] += t * v.r[P];
    red[1] += t * t;
  }
  store_partials<2>(red, part);
}

// x += omega z, r = s - omega t; partials <rh, r>, ||r||^2
__global__ __launch_bounds__(kBlock) void k_tr_update(int nc, double* __restrict__ x, TrVecs v,
                                                      const TrScalars* sc, double* part) {
  if (tr_done(sc)) return;
  const double omega = sc->omega;
  double red[2] = {0.0, 0.0};
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < nc; P += gridDim.x * blockDim.x) {
    x[P] += omega * v.z[P];
    const double r = v.r[P] - omega * v.t[P];
    v.r[P] = r;
    red[0] += v.rh[P] * r;
    red[1] += r * r;
  }
  store_partials<2>(red, part);
}

// ---- scalar kernels (one workgroup) -----------------------------------------

template <int N>
__device__ __forceinline__ void sum_partials(const double* part, int nb, double (&a)[N]) {
  __shared__ double sh[N][kBlock / 64];
#pragma unroll
  for (int k = 0; k < N; ++k) a[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
#pragma unroll
    for (int k = 0; k < N; ++k) a[k] += part[k * nb + b];
  }
  Reducer<0u, N>::block(a, sh);
}

__device__ __forceinline__ void tr_finish(TrScalars* sc, int status) {
  sc->status = status;
  __hip_atomic_store(&sc->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// after the set-up: ||b||^2, rho = <rh, r> = ||r||^2, the first beta
__global__ __launch_bounds__(kBlock) void k_tr_start(const double* part, int nb, double tol,
                                                     int max_iter, TrScalars* sc) {
  double a[2];
  sum_partials<2>(part, nb, a);
  if (threadIdx.x != 0) return;
  sc->bb = a[0];
  sc->rr = a[1];
  sc->rr0 = a[1];
  sc->rho = a[1];
  sc->rho_old = 1.0;
  sc->alpha = 1.0;
  sc->omega = 1.0;
  sc->beta = a[1];  // (rho / rho_old) (alpha / omega) with rho_old = alpha = omega = 1
  sc->tol2 = tol * tol;
  sc->iter = 0;
  sc->max_iter = max_iter;
  sc->status = 0;
  sc->done = 0;
  if (!isfinite(a[0]) || !isfinite(a[1]))
    tr_finish(sc, -5);
  else if (a[0] == 0.0 || a[1] <= sc->tol2 * a[0])
    tr_finish(sc, 0);  // (b = 0: the caller sets x = 0)
  else if (max_iter < 1 || a[1] == 0.0)
    tr_finish(sc, -4);
}

// alpha = rho / <rh, v>
__global__ __launch_bounds__(kBlock) void k_tr_alpha(const double* part, int nb, TrScalars* sc) {
  if (tr_done(sc)) return;
  double a[1];
  sum_partials<1>(part, nb, a);
  if (threadIdx.x != 0) return;
  if (!(a[0] != 0.0) || !isfinite(a[0])) {
    tr_finish(sc, isfinite(a[0]) ? -4 : -5);
    return;
  }
  sc->alpha = sc->rho / a[0];
}

// ||s||^2: converged after the half step?
__global__ __launch_bounds__(kBlock) void k_tr_half_check(const double* part, int nb,
                                                          TrScalars* sc) {
  if (tr_done(sc)) return;
  double a[1];
  sum_partials<1>(part, nb, a);
  if (threadIdx.x != 0) return;
  sc->iter += 1;
  if (!isfinite(a[0])) {
    tr_finish(sc, -5);
  } else if (a[0] <= sc->tol2 * sc->bb) {
    sc->rr = a[0];
    tr_finish(sc, 0);
  }
}

// omega = <t, s> / <t, t>
__global__ __launch_bounds__(kBlock) void k_tr_omega(const double* part, int nb, TrScalars* sc) {
  if (tr_done(sc)) return;
  double a[2];
  sum_partials<2>(part, nb, a);
  if (threadIdx.x != 0) return;
  if (!(a[1] != 0.0) || !isfinite(a[0]) || !isfinite(a[1])) {
    tr_finish(sc, isfinite(a[1]) ? -4 : -5);
    return;
  }
  sc->omega = a[0] / a[1];
}

// rho_new = <rh, r>, ||r||^2: stop test, the next beta
__global__ __launch_bounds__(kBlock) void k_tr_end(const double* part, int nb, TrScalars* sc) {
  if (tr_done(sc)) return;
  double a[2];
  sum_partials<2>(part, nb, a);
  if (threadIdx.x != 0) return;
  sc->rr = a[1];
  if (!isfinite(a[0]) || !isfinite(a[1])) {
    tr_finish(sc, -5);
    return;
  }
  if (a[1] <= sc->tol2 * sc->bb) {
    tr_finish(sc, 0);
    return;
  }
  if (sc->iter >= sc->max_iter || sc->omega == 0.0 || a[0] == 0.0) {
    tr_finish(sc, -4);
    return;
  }
  sc->beta = (a[0] / sc->rho) * (sc->alpha / sc->omega);
  sc->rho_old = sc->rho;
  sc->rho = a[0];
}

}  // namespace

// ---- launchers ---------------------------------------------------------------

void launch_tr_setup_mom(hipStream_t s, const Geo& G, const TrOp& op, const double* un,
                         const double* x0, const TrVecs& v, double* part) {
  const int gb = grid_for(G.nc);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_tr_setup_mom<2>, dim3(gb), dim3(kBlock), 0, s, G, dev_op<2>(op), un, x0, v, part);
  else
    hipLaunchKernelGGL(k_tr_setup_mom<3>, dim3(gb), dim3(kBlock), 0, s, G, dev_op<3>(op), un, x0, v, part);
}

void launch_tr_setup_energy(hipStream_t s, const Geo& G, const Phys& ph, bool enth, const TrOp& op,
                            const double* rho, const double* e0, double* const* u_star,
                            double* w, const double* Tn, const double* Tbg, double* x,
                            const TrVecs& v, double* part) {
  const int gb = grid_for(G.nc);
  if (G.ndim == 2) {
    hipLaunchKernelGGL(k_tr_known<2>, dim3(gb), dim3(kBlock), 0, s, G, ph, uvec<2>(u_star), (int)enth, w);
    if (enth)
      hipLaunchKernelGGL((k_tr_setup_energy<2, true>), dim3(gb), dim3(kBlock), 0, s, G, ph, dev_op<2>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
    else
      hipLaunchKernelGGL((k_tr_setup_energy<2, false>), dim3(gb), dim3(kBlock), 0, s, G, ph, dev_op<2>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
  } else {
    hipLaunchKernelGGL(k_tr_known<3>, dim3(gb), dim3(kBlock), 0, s, G, ph, uvec<3>(u_star), (int)enth, w);
    if (enth)
      hipLaunchKernelGGL((k_tr_setup_energy<3, true>), dim3(gb), dim3(kBlock), 0, s, G, ph, dev_op<3>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
    else
      hipLaunchKernelGGL((k_tr_setup_energy<3, false>), dim3(gb), dim3(kBlock), 0, s, G, ph, dev_op<3>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
  }
}

void launch_tr_start(hipStream_t s, const Geo& G, const double* part, double tol, int max_iter,
                     TrScalars* sc) {
  hipLaunchKernelGGL(k_tr_start, dim3(1), dim3(kBlock), 0, s, part, grid_for(G.nc), tol, max_iter, sc);
}

void launch_tr_iteration(hipStream_t s, const Geo& G, const TrOp& op, double* x, const TrVecs& v,
                         double* part, TrScalars* sc) {
  const int gb = grid_for(G.nc);
  const dim3 grid(gb), block(kBlock);
  hipLaunchKernelGGL(k_tr_dir, grid, block, 0, s, G.nc, v, (const TrScalars*)sc);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_tr_matvec_v<2>, grid, block, 0, s, G, dev_op<2>(op), v, (const TrScalars*)sc, part);
  else
    hipLaunchKernelGGL(k_tr_matvec_v<3>, grid, block, 0, s, G, dev_op<3>(op), v, (const TrScalars*)sc, part);
  hipLaunchKernelGGL(k_tr_alpha, dim3(1), block, 0, s, (const double*)part, gb, sc);
  hipLaunchKernelGGL(k_tr_half, grid, block, 0, s, G.nc, x, v, (const TrScalars*)sc, part);
  hipLaunchKernelGGL(k_tr_half_check, dim3(1), block, 0, s, (const double*)part, gb, sc);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_tr_matvec_t<2>, grid, block, 0, s, G, dev_op<2>(op), v, (const TrScalars*)sc, part);
  else
    hipLaunchKernelGGL(k_tr_matvec_t<3>, grid, block, 0, s, G, dev_op<3>(op), v, (const TrScalars*)sc, part);
  hipLaunchKernelGGL(k_tr_omega, dim3(1), block, 0, s, (const double*)part, gb, sc);
  hipLaunchKernelGGL(k_tr_update, grid, block, 0, s, G.nc, x, v, (const TrScalars*)sc, part);
  hipLaunchKernelGGL(k_tr_end, dim3(1), block, 0, s, (const double*)part, gb, sc);
}

}  // namespace gea
