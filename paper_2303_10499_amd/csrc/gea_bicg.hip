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
// The operator kernels march column tiles through z like the explicit step
// kernels (the line along z in registers, the x/y neighbours from the
// caches, the flux of the face below carried from the plane below); the
// vector updates are grid-stride passes.  Each kernel stores one partial a
// workgroup for every dot product it forms, and a one-workgroup kernel sums
// them in workgroup order (bitwise reproducible) and updates the solver
// scalars.  All kernels of an iteration return at once when the scalars say
// the solve is done, so the host enqueues iterations in batches and reads
// the scalars once a batch.
#include <hip/hip_runtime.h>

#include "gea_internal.h"
#include "gea_reduce.h"
#include "gea_stencil.h"

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

// weight of the face's lower cell (q) or upper cell in its I4 value
__device__ __forceinline__ double i4_weight(int q, int n) {
  return (q >= 1 && q + 2 <= n - 1) ? 9.0 / 16.0 : 0.5;
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

// The operator at cell P of a column (plane k): (A x)_P and its diagonal.
// zx holds x along the column (k-2..k+2); the x/y lines are loaded here;
// fz_lo, fz_hi are the fluxes of the faces below and above (0 on a wall).
template <int NDIM>
__device__ __forceinline__ double tr_plane(const Geo& G, const TrOpD<NDIM>& op, const Col& c,
                                           int P, int k, const double* __restrict__ x,
                                           const Line& zx, double fz_lo, double fz_hi,
                                           double* diag) {
  constexpr int Z = NDIM - 1;
  const int nz = G.n[Z];
  const double xc = zx.c;
  const double cP = op.rho_star[P] * op.tcoef;
  double conv = 0.0, cdiag = 0.0, lap = 0.0, ldiag = 0.0;
  auto faces = [&](const Line& l, int q, int n, double fh, double fl, double kd, bool wall) {
    const double wallk = wall ? 2.0 * kd : 0.0;
    if (q + 1 < n) {
      conv += fh * i4_hi(l, q, n);
      cdiag += fh * i4_weight(q, n);
      lap += kd * (xc - l.p1);
      ldiag += kd;
    } else {
      lap += wallk * xc;
      ldiag += wallk;
    }
    if (q > 0) {
      conv -= fl * i4_lo(l, q, n);
      cdiag -= fl * i4_weight(q - 1, n);
      lap += kd * (xc - l.m1);
      ldiag += kd;
    } else {
      lap += wallk * xc;
      ldiag += wallk;
    }
  };
#pragma unroll
  for (int d = 0; d < Z; ++d) {
    const int st = G.st[d], n = G.n[d], q = coord(c, d);
    const Line l = line_at([&](int Q) { return x[Q]; }, P, st, q, n);
    const double fh = op.phi[d][P], fl = op.phi[d][nb(q > 0, P - st, P)];
    faces(l, q, n, fh, fl, op.k[d], op.wall_comp == d);
  }
  faces(zx, k, nz, fz_hi, fz_lo, op.k[Z], op.wall_comp == Z);
  *diag = cP + op.gamma * cdiag + ldiag;
  return cP * xc + op.gamma * conv + lap;
}

// sum_out phi I4(w) at cell P (the explicit part of Step 2's transport)
template <int NDIM>
__device__ __forceinline__ double tr_conv(const Geo& G, const TrOpD<NDIM>& op, const Col& c, int P,
                                          int k, const double* __restrict__ w, const Line& zw,
                                          double fz_lo, double fz_hi) {
  constexpr int Z = NDIM - 1;
  double conv = 0.0;
#pragma unroll
  for (int d = 0; d < Z; ++d) {
    const int st = G.st[d], n = G.n[d], q = coord(c, d);
    const Line l = line_at([&](int Q) { return w[Q]; }, P, st, q, n);
    if (q + 1 < n) conv += op.phi[d][P] * i4_hi(l, q, n);
    if (q > 0) conv -= op.phi[d][P - st] * i4_lo(l, q, n);
  }
  const int nz = G.n[Z];
  if (k + 1 < nz) conv += fz_hi * i4_hi(zw, k, nz);
  if (k > 0) conv -= fz_lo * i4_lo(zw, k, nz);
  return conv;
}

// ---- set-up ------------------------------------------------------------------

// momentum component: b = V (rho^n u^n/dt - R(F^n)) from the explicit
// predictor's pass, r = b - A x0, rh = r, p = v = 0, 1/diag; partials
// ||b||^2, ||r||^2
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_tr_setup_mom(Geo G, int kc, TrOpD<NDIM> op,
                                                         const double* __restrict__ x0, TrVecs v,
                                                         double* part) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  double red[2] = {0.0, 0.0};
  if (c.act) {
    const int nz = G.n[Z], pl = c.pl;
    int P = c.base + pl * c.k0;
    Line zx = line_at([&](int Q) { return x0[Q]; }, P, pl, c.k0, nz);
    double flo = c.k0 > 0 ? op.phi[Z][P - pl] : 0.0;
    for (int k = c.k0; k < c.k1; ++k, P += pl) {
      const double fhi = op.phi[Z][P];
      const double xn = x0[nb(k + 3 < nz, P + 3 * pl, P)];
      double diag;
      const double ax = tr_plane<NDIM>(G, op, c, P, k, x0, zx, flo, fhi, &diag);
      const double b = v.b[P], r = b - ax;
      v.dinv[P] = 1.0 / diag;
      v.r[P] = r;
      v.rh[P] = r;
      v.p[P] = 0.0;
      v.v[P] = 0.0;
      red[0] += b * b;
      red[1] += r * r;
      flo = fhi;
      zx = shift(zx, k + 3 < nz ? xn : 0.0);
    }
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
    Geo G, Phys ph, int kc, TrOpD<NDIM> op, const double* __restrict__ rho,
    const double* __restrict__ e0, const double* __restrict__ w, const double* __restrict__ Tn,
    const double* __restrict__ Tbg, double* __restrict__ x, TrVecs v, double* part) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  double red[2] = {0.0, 0.0};
  if (c.act) {
    const int nz = G.n[Z], pl = c.pl;
    const double kdz = op.k[Z];   // (mu/Pr) c_p S_z/h_z
    int P = c.base + pl * c.k0;
    Line zT = line_at([&](int Q) { return Tn[Q]; }, P, pl, c.k0, nz);
    Line zw = line_at([&](int Q) { return w[Q]; }, P, pl, c.k0, nz);
    double flo = c.k0 > 0 ? op.phi[Z][P - pl] : 0.0;
    for (int k = c.k0; k < c.k1; ++k, P += pl) {
      const double fhi = op.phi[Z][P];
      const int Pn = nb(k + 3 < nz, P + 3 * pl, P);
      const double Tnext = Tn[Pn], wnext = w[Pn];
      const double rs = op.rho_star[P];
      const double local = ENTH ? G.V / ph.dt * e0[P] : G.V / ph.dt * (rho[P] * e0[P] - rs * zw.c);
      const double convw = tr_conv<NDIM>(G, op, c, P, k, w, zw, flo, fhi);
      double bg = 0.0;
      if (k + 1 < nz) bg += kdz * (Tbg[k] - Tbg[k + 1]);
      if (k > 0) bg += kdz * (Tbg[k] - Tbg[k - 1]);
      const double b = local - convw + bg;
      double diag;
      const double ax = tr_plane<NDIM>(G, op, c, P, k, Tn, zT, flo, fhi, &diag);
      const double r = b - ax;
      x[P] = zT.c;
      v.b[P] = b;
      v.dinv[P] = 1.0 / diag;
      v.r[P] = r;
      v.rh[P] = r;
      v.p[P] = 0.0;
      v.v[P] = 0.0;
      red[0] += b * b;
      red[1] += r * r;
      flo = fhi;
      const bool more = k + 3 < nz;
      zT = shift(zT, more ? Tnext : 0.0);
      zw = shift(zw, more ? wnext : 0.0);
    }
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

// out = A in (TWO = 0: v = A y, partial <rh, v>; TWO = 1: t = A z, partials
// <t, s>, <t, t> with s in r)
template <int NDIM, int TWO>
__global__ __launch_bounds__(kBlock) void k_tr_matvec(Geo G, int kc, TrOpD<NDIM> op,
                                                      const double* __restrict__ in,
                                                      double* __restrict__ out,
                                                      const double* __restrict__ dv,
                                                      const TrScalars* sc, double* part) {
  if (tr_done(sc)) return;
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  double red[2] = {0.0, 0.0};
  if (c.act) {
    const int nz = G.n[Z], pl = c.pl;
    int P = c.base + pl * c.k0;
    Line zx = line_at([&](int Q) { return in[Q]; }, P, pl, c.k0, nz);
    double flo = c.k0 > 0 ? op.phi[Z][P - pl] : 0.0;
    for (int k = c.k0; k < c.k1; ++k, P += pl) {
      const double fhi = op.phi[Z][P];
      const double xn = in[nb(k + 3 < nz, P + 3 * pl, P)];
      const double d = dv[P];
      double diag;
      const double a = tr_plane<NDIM>(G, op, c, P, k, in, zx, flo, fhi, &diag);
      out[P] = a;
      if (TWO) {
        red[0] += a * d;
        red[1] += a * a;
      } else {
        red[0] += d * a;
      }
      flo = fhi;
      zx = shift(zx, k + 3 < nz ? xn : 0.0);
    }
  }
  if (TWO) {
    store_partials<2>(red, part);
  } else {
    double one[1] = {red[0]};
    store_partials<1>(one, part);
  }
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

void launch_tr_setup_mom(hipStream_t s, const Geo& G, const TrOp& op, const double* x0,
                         const TrVecs& v, double* part) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_tr_setup_mom<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, zp.kc, dev_op<2>(op), x0, v, part);
  else
    hipLaunchKernelGGL(k_tr_setup_mom<3>, dim3(zp.blocks), dim3(kBlock), 0, s, G, zp.kc, dev_op<3>(op), x0, v, part);
}

void launch_tr_setup_energy(hipStream_t s, const Geo& G, const Phys& ph, bool enth, const TrOp& op,
                            const double* rho, const double* e0, double* const* u_star,
                            double* w, const double* Tn, const double* Tbg, double* x,
                            const TrVecs& v, double* part) {
  const int gb = grid_for(G.nc);
  const ZPlan zp = zplan(G);
  if (G.ndim == 2) {
    hipLaunchKernelGGL(k_tr_known<2>, dim3(gb), dim3(kBlock), 0, s, G, ph, uvec<2>(u_star), (int)enth, w);
    if (enth)
      hipLaunchKernelGGL((k_tr_setup_energy<2, true>), dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, dev_op<2>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
    else
      hipLaunchKernelGGL((k_tr_setup_energy<2, false>), dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, dev_op<2>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
  } else {
    hipLaunchKernelGGL(k_tr_known<3>, dim3(gb), dim3(kBlock), 0, s, G, ph, uvec<3>(u_star), (int)enth, w);
    if (enth)
      hipLaunchKernelGGL((k_tr_setup_energy<3, true>), dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, dev_op<3>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
    else
      hipLaunchKernelGGL((k_tr_setup_energy<3, false>), dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, dev_op<3>(op), rho, e0, (const double*)w, Tn, Tbg, x, v, part);
  }
}

void launch_tr_start(hipStream_t s, const Geo& G, const double* part, double tol, int max_iter,
                     TrScalars* sc) {
  hipLaunchKernelGGL(k_tr_start, dim3(1), dim3(kBlock), 0, s, part, zplan(G).blocks, tol, max_iter, sc);
}

void launch_tr_iteration(hipStream_t s, const Geo& G, const TrOp& op, double* x, const TrVecs& v,
                         double* part, TrScalars* sc) {
  const int gb = grid_for(G.nc);
  const ZPlan zp = zplan(G);
  const dim3 grid(gb), block(kBlock), zgrid(zp.blocks);
  const TrScalars* csc = sc;
  hipLaunchKernelGGL(k_tr_dir, grid, block, 0, s, G.nc, v, csc);
  if (G.ndim == 2)
    hipLaunchKernelGGL((k_tr_matvec<2, 0>), zgrid, block, 0, s, G, zp.kc, dev_op<2>(op), (const double*)v.y, v.v, (const double*)v.rh, csc, part);
  else
    hipLaunchKernelGGL((k_tr_matvec<3, 0>), zgrid, block, 0, s, G, zp.kc, dev_op<3>(op), (const double*)v.y, v.v, (const double*)v.rh, csc, part);
  hipLaunchKernelGGL(k_tr_alpha, dim3(1), block, 0, s, (const double*)part, zp.blocks, sc);
  hipLaunchKernelGGL(k_tr_half, grid, block, 0, s, G.nc, x, v, csc, part);
  hipLaunchKernelGGL(k_tr_half_check, dim3(1), block, 0, s, (const double*)part, gb, sc);
  if (G.ndim == 2)
    hipLaunchKernelGGL((k_tr_matvec<2, 1>), zgrid, block, 0, s, G, zp.kc, dev_op<2>(op), (const double*)v.z, v.t, (const double*)v.r, csc, part);
  else
    hipLaunchKernelGGL((k_tr_matvec<3, 1>), zgrid, block, 0, s, G, zp.kc, dev_op<3>(op), (const double*)v.z, v.t, (const double*)v.r, csc, part);
  hipLaunchKernelGGL(k_tr_omega, dim3(1), block, 0, s, (const double*)part, zp.blocks, sc);
  hipLaunchKernelGGL(k_tr_update, grid, block, 0, s, G.nc, x, v, csc, part);
  hipLaunchKernelGGL(k_tr_end, dim3(1), block, 0, s, (const double*)part, gb, sc);
}

}  // namespace gea
