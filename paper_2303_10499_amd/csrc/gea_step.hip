// gea_step.hip -- explicit kernels of one segregated pressure-based step
// (GEA, Sec. 3): Step 1 mass flux and predictors, Step 2 energy sweeps with
// e -> T recovery and EOS coefficients, Step 3 H operator, predicted flux and
// pressure right-hand side, flux/velocity correction and end-of-step update;
// plus the initial bubble state of Sec. 4.
//
// One thread per cell in grid-stride loops over the SoA FP64 fields; x is
// the fastest index, so the x-neighbours of a wave are contiguous and the
// (y,) z-neighbours are whole rows that the neighbouring waves also read
// (L2/MALL hits).  A face value is computed by one formula whichever of its
// two cells evaluates it, so the flux leaving one cell is bitwise the flux
// entering the other and the divergence telescopes.
#include "gea_reduce.h"

namespace gea {

namespace {

__device__ __forceinline__ double phi_cell(const Geo& G, const Phys& ph, int kz) {
  return ph.g * (kz + 0.5) * G.dz;
}

// Phi on the face between a cell with coordinate cq along d (and height
// index kz) and its +d neighbour
template <int NDIM>
__device__ __forceinline__ double phi_face(const Geo& G, const Phys& ph, int d, int cq, int kz) {
  return d == NDIM - 1 ? ph.g * (cq + 1.0) * G.dz : phi_cell(G, ph, kz);
}

// Fourth-order point-value interpolation at the face between Q and Q+st
// (coordinate cq of Q along a direction with n cells): cubic with two cells
// on each side, linear next to a wall.
template <typename F>
__device__ __forceinline__ double interp4(F s, int Q, int st, int cq, int n) {
  if (cq >= 1 && cq + 2 <= n - 1)
    return (-s(Q - st) + 9.0 * s(Q) + 9.0 * s(Q + st) - s(Q + 2 * st)) / 16.0;
  return 0.5 * (s(Q) + s(Q + st));
}

// sum_out phi_f I4(s)_f
template <int NDIM>
__device__ __forceinline__ double convective(const Geo& G, const Vec<NDIM>& phi, const double* s,
                                             int P, const int* c) {
  double acc = 0.0;
  auto f = [&](int Q) { return s[Q]; };
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    const int st = G.st[d], n = G.n[d];
    if (c[d] + 1 < n) acc += phi.p[d][P] * interp4(f, P, st, c[d], n);
    if (c[d] > 0) acc -= phi.p[d][P - st] * interp4(f, P - st, st, c[d] - 1, n);
  }
  return acc;
}

// sum_f mu snGrad(u_comp) S with free-slip impenetrable walls
template <int NDIM>
__device__ __forceinline__ double viscous(const Geo& G, const double* uc, int comp, double mu,
                                          int P, const int* c) {
  double acc = 0.0;
  const double up = uc[P];
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    const int st = G.st[d];
    const double k = mu * G.S[d] / G.h[d];
    if (c[d] + 1 < G.n[d]) acc += k * (uc[P + st] - up);
    else if (comp == d) acc += 2.0 * k * (0.0 - up);
    if (c[d] > 0) acc += k * (uc[P - st] - up);
    else if (comp == d) acc += 2.0 * k * (0.0 - up);
  }
  return acc;
}

// F on the face between Q and Q+st along d: grad p' - Phi grad rho
template <int NDIM>
__device__ __forceinline__ double force_face(const Geo& G, const Phys& ph, const double* pp,
                                             const double* rho, int Q, int d, int cq, int kz) {
  const int st = G.st[d];
  return ((pp[Q + st] - pp[Q]) - phi_face<NDIM>(G, ph, d, cq, kz) * (rho[Q + st] - rho[Q])) /
         G.h[d];
}

// cell value of component d of R(F): mean of the two faces, 0 on walls
template <int NDIM>
__device__ __forceinline__ double reconstruct(const Geo& G, const Phys& ph, const double* pp,
                                              const double* rho, int P, const int* c, int d) {
  const double hi = (c[d] + 1 < G.n[d]) ? force_face<NDIM>(G, ph, pp, rho, P, d, c[d], c[NDIM - 1]) : 0.0;
  const int kz_lo = (d == NDIM - 1) ? c[d] - 1 : c[NDIM - 1];
  const double lo =
      (c[d] > 0) ? force_face<NDIM>(G, ph, pp, rho, P - G.st[d], d, c[d] - 1, kz_lo) : 0.0;
  return 0.5 * (lo + hi);
}

template <int NDIM>
__device__ __forceinline__ double kinetic(const Vec<NDIM>& u, int P) {
  double k = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) k += u.p[d][P] * u.p[d][P];
  return 0.5 * k;
}

// ---- Step 1 ----------------------------------------------------------------

// phi_f = I4(rho u . n) S on interior faces, rho* = rho - dt/V sum_out phi
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_mass_flux(Geo G, Phys ph, const double* __restrict__ rho,
                                                      Vec<NDIM> u, Vec<NDIM> phi,
                                                      double* __restrict__ rho_star) {
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    double sum = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const double* ud = u.p[d];
      const int st = G.st[d], n = G.n[d];
      auto mom = [&](int Q) { return rho[Q] * ud[Q]; };
      double hi = 0.0, lo = 0.0;
      if (c[d] + 1 < n) hi = interp4(mom, P, st, c[d], n) * G.S[d];
      if (c[d] > 0) lo = interp4(mom, P - st, st, c[d] - 1, n) * G.S[d];
      phi.p[d][P] = hi;
      sum += hi;
      sum -= lo;
    }
    rho_star[P] = rho[P] - ph.dt / G.V * sum;
  }
}

// rho* u* = rho u - dt/V [sum_out phi I4(u) - sum mu snGrad(u) S] - dt R(F)
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_mom_predict(Geo G, Phys ph,
                                                        const double* __restrict__ rho, Vec<NDIM> u,
                                                        const double* __restrict__ pp,
                                                        const double* __restrict__ rho_star,
                                                        Vec<NDIM> phi, Vec<NDIM> u_star) {
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      const double* uc = u.p[cc];
      const double conv = convective<NDIM>(G, phi, uc, P, c);
      const double visc = viscous<NDIM>(G, uc, cc, ph.mu, P, c);
      const double RF = reconstruct<NDIM>(G, ph, pp, rho, P, c, cc);
      const double mom = rho[P] * uc[P] - ph.dt / G.V * (conv - visc) - ph.dt * RF;
      u_star.p[cc][P] = mom / rho_star[P];
    }
  }
}

// ---- Step 2 ----------------------------------------------------------------

// e^n = c_v T + K + Phi
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_energy_init(Geo G, Phys ph, const double* __restrict__ T,
                                                        Vec<NDIM> u, double* __restrict__ e0) {
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    e0[P] = ph.cv * T[P] + kinetic<NDIM>(u, P) + phi_cell(G, ph, c[NDIM - 1]);
  }
}

// One Picard sweep of the total-energy equation with frozen flux phi:
//   rho* e = rho^n e^n - dt/V sum_out phi I4(e + R T) + dt/V sum (mu/Pr) c_p snGrad(T - T_bg) S
//   T = (e - K* - Phi)/c_v
// The last sweep also forms the EOS density and pressure-equation coefficients.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_energy_sweep(
    Geo G, Phys ph, const double* __restrict__ rho, const double* __restrict__ e0,
    const double* __restrict__ e_prev, const double* __restrict__ T_prev, Vec<NDIM> phi,
    const double* __restrict__ rho_star, Vec<NDIM> u_star, const double* __restrict__ Tbg,
    double* __restrict__ e_next, double* __restrict__ T_next, int last,
    const double* __restrict__ p, double* __restrict__ rho23, double* __restrict__ psi,
    double* __restrict__ cc, double* __restrict__ D) {
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    const int kz = c[NDIM - 1];
    auto hhat = [&](int Q) { return e_prev[Q] + ph.R * T_prev[Q]; };
    double conv = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int st = G.st[d], n = G.n[d];
      if (c[d] + 1 < n) conv += phi.p[d][P] * interp4(hhat, P, st, c[d], n);
      if (c[d] > 0) conv -= phi.p[d][P - st] * interp4(hhat, P - st, st, c[d] - 1, n);
    }
    const double Tp = T_prev[P] - Tbg[kz];
    double diff = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int st = G.st[d];
      const double k = ph.mu / ph.Pr * ph.cp * G.S[d] / G.h[d];
      const int up = (d == NDIM - 1) ? 1 : 0;
      if (c[d] + 1 < G.n[d]) diff += k * ((T_prev[P + st] - Tbg[kz + up]) - Tp);
      if (c[d] > 0) diff += k * ((T_prev[P - st] - Tbg[kz - up]) - Tp);
    }
    const double rhoe = rho[P] * e0[P] - ph.dt / G.V * conv + ph.dt / G.V * diff;
    const double e = rhoe / rho_star[P];
    const double T = (e - kinetic<NDIM>(u_star, P) - phi_cell(G, ph, kz)) / ph.cv;
    e_next[P] = e;
    T_next[P] = T;
    if (last) {
      rho23[P] = p[P] / (ph.R * T);
      psi[P] = 1.0 / (ph.R * T);
      cc[P] = psi[P] * G.V / ph.dt;
      D[P] = rho23[P] / (rho_star[P] / ph.dt);
    }
  }
}

// ---- Step 3 ----------------------------------------------------------------

// H(u) = rho^n u^n/dt - (1/V) sum_out phi I4(u) + (1/V) sum mu snGrad(u) S
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_H(Geo G, Phys ph, const double* __restrict__ rho,
                                              Vec<NDIM> u, Vec<NDIM> u_prev, Vec<NDIM> phi,
                                              Vec<NDIM> H) {
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      const double* uc = u_prev.p[cc];
      const double conv = convective<NDIM>(G, phi, uc, P, c);
      const double visc = viscous<NDIM>(G, uc, cc, ph.mu, P, c);
      H.p[cc][P] = rho[P] * u.p[cc][P] / ph.dt - conv / G.V + visc / G.V;
    }
  }
}

// predicted flux on the face between Q and Q+st along d:
// D_f S [H_f . n + Phi_f (rho23_N - rho23_P)/d]
template <int NDIM>
__device__ __forceinline__ double phi_tilde(const Geo& G, const Phys& ph, const double* D,
                                            const double* Hd, const double* rho23, int Q, int d,
                                            int cq, int kz) {
  const int st = G.st[d];
  const double Df = 0.5 * (D[Q] + D[Q + st]);
  const double Hf = 0.5 * (Hd[Q] + Hd[Q + st]);
  return Df * G.S[d] * (Hf + phi_face<NDIM>(G, ph, d, cq, kz) * (rho23[Q + st] - rho23[Q]) / G.h[d]);
}

// b = (V/dt)(rho^n + psi rho23 Phi) - sum_out phitilde; 1/diag of the operator
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_rhs(Geo G, Phys ph, const double* __restrict__ rho,
                                                const double* __restrict__ rho23,
                                                const double* __restrict__ psi,
                                                const double* __restrict__ cc,
                                                const double* __restrict__ D, Vec<NDIM> H,
                                                double* __restrict__ b, double* __restrict__ dinv) {
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    const int kz = c[NDIM - 1];
    double sum = 0.0;
    double diag = cc[P];
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int st = G.st[d];
      const double k = G.S[d] / G.h[d];
      if (c[d] + 1 < G.n[d]) {
        sum += phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P, d, c[d], kz);
        diag += 0.5 * (D[P] + D[P + st]) * k;
      }
      if (c[d] > 0) {
        const int kzl = (d == NDIM - 1) ? kz - 1 : kz;
        sum -= phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P - st, d, c[d] - 1, kzl);
        diag += 0.5 * (D[P - st] + D[P]) * k;
      }
    }
    const double Phi = phi_cell(G, ph, kz);
    b[P] = G.V / ph.dt * (rho[P] + psi[P] * rho23[P] * Phi) - sum;
    dinv[P] = 1.0 / diag;
  }
}

// u = (H - R(F))/A with F from p' and rho23, A = rho*/dt.  The last corrector
// also takes rho^{n+1} = rho^n - dt/V sum_out (phitilde - w (p'_N - p'_P)),
// p^{n+1} = p' - rho23 Phi, and reduces [mass, max |rho - psi p|, non-finite count].
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_correct(
    Geo G, Phys ph, const double* __restrict__ pp, const double* __restrict__ rho23,
    const double* __restrict__ psi, Vec<NDIM> H, const double* __restrict__ D,
    const double* __restrict__ rho_star, Vec<NDIM> u_out, int last,
    const double* __restrict__ rho_old, double* __restrict__ rho_new, double* __restrict__ p_new,
    double* partials, CgScalars* sc) {
  double red[3] = {0.0, 0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    const int kz = c[NDIM - 1];
    const double A = rho_star[P] / ph.dt;
    bool finite = true;
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      const double RF = reconstruct<NDIM>(G, ph, pp, rho23, P, c, cc);
      const double un = (H.p[cc][P] - RF) / A;
      u_out.p[cc][P] = un;
      finite = finite && isfinite(un);
    }
    if (last) {
      double sum = 0.0;
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        const int st = G.st[d];
        const double k = G.S[d] / G.h[d];
        if (c[d] + 1 < G.n[d]) {
          const double w = 0.5 * (D[P] + D[P + st]) * k;
          sum += phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P, d, c[d], kz) - w * (pp[P + st] - pp[P]);
        }
        if (c[d] > 0) {
          const int kzl = (d == NDIM - 1) ? kz - 1 : kz;
          const double w = 0.5 * (D[P - st] + D[P]) * k;
          sum -= phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P - st, d, c[d] - 1, kzl) -
                 w * (pp[P] - pp[P - st]);
        }
      }
      const double rn = rho_old[P] - ph.dt / G.V * sum;
      const double pn = pp[P] - rho23[P] * phi_cell(G, ph, kz);
      rho_new[P] = rn;
      p_new[P] = pn;
      red[0] += rn * G.V;
      red[1] = fmax(red[1], fabs(rn - psi[P] * pn));
      finite = finite && isfinite(rn) && isfinite(pn);
    }
    red[2] += finite ? 0.0 : 1.0;
  }
  if (!last) return;
  __shared__ double sh[3][kBlock / 64];
  Reducer<0x2u, 3>::block(red, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) partials[k * gridDim.x + blockIdx.x] = red[k];
}

// one workgroup: [sum of mass, max |rho - psi p|, non-finite count] over the
// correction kernel's per-workgroup partials, in workgroup order
__global__ __launch_bounds__(kBlock) void k_finalize_reduce(const double* partials, int n,
                                                            CgScalars* sc) {
  __shared__ double sh[3][kBlock / 64];
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += kBlock) {
    a[0] += partials[b];
    a[1] = fmax(a[1], partials[n + b]);
    a[2] += partials[2 * n + b];
  }
  Reducer<0x2u, 3>::block(a, sh);
  if (threadIdx.x == 0) {
    sc->aux[0] = a[0];
    sc->aux[1] = a[1];
    sc->aux[2] = a[2];
  }
}

// ---- initial state (Sec. 4) --------------------------------------------------

// Background column of a neutral atmosphere with a discretely hydrostatic p'
// (one thread: a short sequential recurrence over the nz levels).
__global__ void k_init_column(Geo G, Phys ph, double* rho_a, double* pp_a, double* Tbg) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int nz = G.nz;
  for (int k = 0; k < nz; ++k) {
    const double z = (k + 0.5) * G.dz;
    const double pib = 1.0 - ph.g * z / (ph.cp * ph.theta0);
    rho_a[k] = ph.p0 * pow(pib, ph.cv / ph.R) / (ph.R * ph.theta0);
  }
  const double z0 = 0.5 * G.dz;
  const double pib0 = 1.0 - ph.g * z0 / (ph.cp * ph.theta0);
  pp_a[0] = ph.p0 * pow(pib0, ph.cp / ph.R) + rho_a[0] * ph.g * z0;
  for (int k = 0; k + 1 < nz; ++k)
    pp_a[k + 1] = pp_a[k] + ph.g * (k + 1.0) * G.dz * (rho_a[k + 1] - rho_a[k]);
  for (int k = 0; k < nz; ++k) {
    const double Phi = ph.g * (k + 0.5) * G.dz;
    const double pb = pp_a[k] - rho_a[k] * Phi;
    Tbg[k] = pb / (ph.R * rho_a[k]);
  }
}

template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_init_fields(Geo G, Phys ph, int kind, double xc,
                                                        double yc, double zc, double rc, double amp,
                                                        const double* rho_a, const double* pp_a,
                                                        const double* Tbg, double* rho, Vec<NDIM> u,
                                                        double* T, double* pp, double* p) {
  constexpr double kPi = 3.141592653589793;
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    const int k = c[NDIM - 1];
    const double x = (c[0] + 0.5) * G.h[0];
    const double z = (k + 0.5) * G.dz;
    double r2 = (x - xc) * (x - xc) + (z - zc) * (z - zc);
    if constexpr (NDIM == 3) {
      const double y = (c[1] + 0.5) * G.h[1];
      r2 += (y - yc) * (y - yc);
    }
    const double r = sqrt(r2);
    double th = 0.0;
    if (kind == 1 && r <= rc) th = 0.5 * amp * (1.0 + cos(kPi * r / rc));
    if (kind == 2 && r <= rc) th = amp;
    const double Phi = ph.g * z;
    const double pb = pp_a[k] - rho_a[k] * Phi;
    const double Tv = Tbg[k] * (1.0 + th / ph.theta0);
    T[P] = Tv;
    p[P] = pb;
    const double rv = pb / (ph.R * Tv);
    rho[P] = rv;
    pp[P] = pb + rv * Phi;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) u.p[d][P] = 0.0;
  }
}

template <int NDIM>
Vec<NDIM> vec(double* const* a) {
  Vec<NDIM> v;
  for (int d = 0; d < NDIM; ++d) v.p[d] = a[d];
  return v;
}

}  // namespace

int grid_for(int nc) {
  const int need = (nc + kBlock - 1) / kBlock;
  const int cap = 2048;  // 8 workgroups per CU on 256 CUs
  return need < 1 ? 1 : (need < cap ? need : cap);
}

#define V2(a) vec<2>(a)
#define V3(a) vec<3>(a)

void launch_mass_flux(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                      double* const* u, double* const* phi, double* rho_star) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_mass_flux<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, V2(u), V2(phi), rho_star);
  else
    hipLaunchKernelGGL(k_mass_flux<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, V3(u), V3(phi), rho_star);
}

void launch_mom_predict(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                        double* const* u, const double* pp, const double* rho_star,
                        double* const* phi, double* const* u_star) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_mom_predict<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, V2(u), pp, rho_star, V2(phi), V2(u_star));
  else
    hipLaunchKernelGGL(k_mom_predict<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, V3(u), pp, rho_star, V3(phi), V3(u_star));
}

void launch_energy_init(hipStream_t s, const Geo& G, const Phys& ph, const double* T,
                        double* const* u, double* e0) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_energy_init<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, T, V2(u), e0);
  else
    hipLaunchKernelGGL(k_energy_init<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, T, V3(u), e0);
}

void launch_energy_sweep(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                         const double* e0, const double* e_prev, const double* T_prev,
                         double* const* phi, const double* rho_star, double* const* u_star,
                         const double* Tbg, double* e_next, double* T_next, bool last,
                         const double* p, double* rho23, double* psi, double* c, double* D) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_energy_sweep<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, e0, e_prev, T_prev, V2(phi), rho_star, V2(u_star), Tbg, e_next, T_next, (int)last, p, rho23, psi, c, D);
  else
    hipLaunchKernelGGL(k_energy_sweep<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, e0, e_prev, T_prev, V3(phi), rho_star, V3(u_star), Tbg, e_next, T_next, (int)last, p, rho23, psi, c, D);
}

void launch_H(hipStream_t s, const Geo& G, const Phys& ph, const double* rho, double* const* u,
              double* const* u_prev, double* const* phi, double* const* H) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_H<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, V2(u), V2(u_prev), V2(phi), V2(H));
  else
    hipLaunchKernelGGL(k_H<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, V3(u), V3(u_prev), V3(phi), V3(H));
}

void launch_rhs(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                const double* rho23, const double* psi, const double* c, const double* D,
                double* const* H, double* b, double* dinv) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_rhs<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, rho23, psi, c, D, V2(H), b, dinv);
  else
    hipLaunchKernelGGL(k_rhs<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, rho, rho23, psi, c, D, V3(H), b, dinv);
}

void launch_correct(hipStream_t s, const Geo& G, const Phys& ph, const double* pp,
                    const double* rho23, const double* psi, double* const* H, const double* D,
                    const double* rho_star, double* const* u_out, bool last,
                    const double* rho_old, double* rho_new, double* p_new, double* partials,
                    CgScalars* sc) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_correct<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, pp, rho23, psi, V2(H), D, rho_star, V2(u_out), (int)last, rho_old, rho_new, p_new, partials, sc);
  else
    hipLaunchKernelGGL(k_correct<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, pp, rho23, psi, V3(H), D, rho_star, V3(u_out), (int)last, rho_old, rho_new, p_new, partials, sc);
  if (last)
    hipLaunchKernelGGL(k_finalize_reduce, dim3(1), dim3(kBlock), 0, s, (const double*)partials, grid_for(G.nc), sc);
}

void launch_init_column(hipStream_t s, const Geo& G, const Phys& ph, double* rho_a,
                        double* pp_a, double* Tbg) {
  hipLaunchKernelGGL(k_init_column, dim3(1), dim3(64), 0, s, G, ph, rho_a, pp_a, Tbg);
}

void launch_init_fields(hipStream_t s, const Geo& G, const Phys& ph, int kind, double xc,
                        double yc, double zc, double rc, double amp, const double* rho_a,
                        const double* pp_a, const double* Tbg, double* rho, double* const* u,
                        double* T, double* pp, double* p) {
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_init_fields<2>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, kind, xc, yc, zc, rc, amp, rho_a, pp_a, Tbg, rho, V2(u), T, pp, p);
  else
    hipLaunchKernelGGL(k_init_fields<3>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, kind, xc, yc, zc, rc, amp, rho_a, pp_a, Tbg, rho, V3(u), T, pp, p);
}

}  // namespace gea
