// gea_step.hip -- explicit kernels of one segregated pressure-based step
// (GEA, Sec. 3): Step 1 mass flux and predictors, Step 2 energy sweeps with
// e -> T recovery and EOS coefficients, Step 3 H operator, predicted flux and
// pressure right-hand side, flux/velocity correction and end-of-step update;
// plus the initial bubble state of Sec. 4.
//
// The stencil kernels march column tiles through z (one thread per vertical
// column of cells, SoA FP64 fields, x fastest).  A face value is computed by
// one formula whichever of its two cells evaluates it, and a z-face value is
// computed once and carried to the cell above, so the flux leaving one cell
// is bitwise the flux entering the other and the divergence telescopes.
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

// F on the face between Q and Q+st along d: grad p' - Phi grad rho
template <int NDIM>
__device__ __forceinline__ double force_face(const Geo& G, const Phys& ph, const double* pp,
                                             const double* rho, int Q, int d, int cq, int kz) {
  const int st = G.st[d];
  return ((pp[Q + st] - pp[Q]) - phi_face<NDIM>(G, ph, d, cq, kz) * (rho[Q + st] - rho[Q])) *
         G.inv_h[d];
}

template <int NDIM>
__device__ __forceinline__ double kinetic(const Vec<NDIM>& u, int P) {
  double k = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) k += u.p[d][P] * u.p[d][P];
  return 0.5 * k;
}

// Five consecutive values of a cell field along one direction, centred on
// the cell; entries outside the mesh are never used and left 0.
struct Line {
  double m2, m1, c, p1, p2;
};

template <typename F>
__device__ __forceinline__ Line line_at(F s, int P, int st, int q, int n) {
  Line L;
  L.c = s(P);
  L.m1 = q >= 1 ? s(P - st) : 0.0;
  L.m2 = q >= 2 ? s(P - 2 * st) : 0.0;
  L.p1 = q + 1 < n ? s(P + st) : 0.0;
  L.p2 = q + 2 < n ? s(P + 2 * st) : 0.0;
  return L;
}

// next plane: drop the lowest value, append the one two planes above
__device__ __forceinline__ Line shift(const Line& L, double next) {
  return Line{L.m1, L.c, L.p1, L.p2, next};
}

// interp4 on the face above (q + 1/2) and below (q - 1/2) the centre of a line
__device__ __forceinline__ double i4_hi(const Line& s, int q, int n) {
  if (q >= 1 && q + 2 <= n - 1) return (-s.m1 + 9.0 * s.c + 9.0 * s.p1 - s.p2) / 16.0;
  return 0.5 * (s.c + s.p1);
}
__device__ __forceinline__ double i4_lo(const Line& s, int q, int n) {
  if (q >= 2 && q + 1 <= n - 1) return (-s.m2 + 9.0 * s.m1 + 9.0 * s.c - s.p1) / 16.0;
  return 0.5 * (s.m1 + s.c);
}

// mu snGrad(u_comp) S on the two faces of a line; walls normal to the line
// hold the normal component at 0 and leave the tangential ones free
__device__ __forceinline__ void visc_add(double& acc, const Line& s, int q, int n, double k,
                                         bool normal) {
  if (q + 1 < n) acc += k * (s.p1 - s.c);
  else if (normal) acc += 2.0 * k * (0.0 - s.c);
  if (q > 0) acc += k * (s.m1 - s.c);
  else if (normal) acc += 2.0 * k * (0.0 - s.c);
}


// ---- Step 1 ----------------------------------------------------------------

// phi_f = I4(rho u . n) S on interior faces, rho* = rho - dt/V sum_out phi
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_mass_flux(Geo G, Phys ph, int kc,
                                                      const double* __restrict__ rho,
                                                      Vec<NDIM> u, Vec<NDIM> phi,
                                                      double* __restrict__ rho_star) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  if (!c.act) return;
  const int nz = G.n[Z], pl = c.pl;
  const double* uz = u.p[Z];
  auto mz = [&](int Q) { return rho[Q] * uz[Q]; };
  int P = c.base + pl * c.k0;
  Line z = line_at(mz, P, pl, c.k0, nz);
  double flo = c.k0 > 0 ? i4_lo(z, c.k0, nz) * G.S[Z] : 0.0;
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    double sum = 0.0;
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const double* ud = u.p[d];
      const int st = G.st[d], n = G.n[d], q = coord(c, d);
      auto m = [&](int Q) { return rho[Q] * ud[Q]; };
      const Line s = line_at(m, P, st, q, n);
      const double hi = q + 1 < n ? i4_hi(s, q, n) * G.S[d] : 0.0;
      const double lo = q > 0 ? i4_lo(s, q, n) * G.S[d] : 0.0;
      phi.p[d][P] = hi;
      sum += hi;
      sum -= lo;
    }
    const double hi = k + 1 < nz ? i4_hi(z, k, nz) * G.S[Z] : 0.0;
    phi.p[Z][P] = hi;
    sum += hi;
    sum -= flo;
    flo = hi;
    rho_star[P] = rho[P] - ph.dt / G.V * sum;
    z = shift(z, k + 3 < nz ? mz(P + 3 * pl) : 0.0);
  }
}

// rho* u* = rho u - dt/V [sum_out phi I4(u) - sum mu snGrad(u) S] - dt R(F)
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_mom_predict(Geo G, Phys ph, int kc,
                                                        const double* __restrict__ rho, Vec<NDIM> u,
                                                        const double* __restrict__ pp,
                                                        const double* __restrict__ rho_star,
                                                        Vec<NDIM> phi, Vec<NDIM> u_star) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  if (!c.act) return;
  const int nz = G.n[Z], pl = c.pl;
  int P = c.base + pl * c.k0;
  Line z[NDIM];
  double flo[NDIM];
  const double phz_lo = c.k0 > 0 ? phi.p[Z][P - pl] : 0.0;
#pragma unroll
  for (int cc = 0; cc < NDIM; ++cc) {
    const double* uc = u.p[cc];
    z[cc] = line_at([&](int Q) { return uc[Q]; }, P, pl, c.k0, nz);
    flo[cc] = c.k0 > 0 ? phz_lo * i4_lo(z[cc], c.k0, nz) : 0.0;
  }
  double Flo = c.k0 > 0 ? force_face<NDIM>(G, ph, pp, rho, P - pl, Z, c.k0 - 1, c.k0 - 1) : 0.0;
  const double kvz = ph.mu * G.S[Z] / G.h[Z];
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    const double Fhi = k + 1 < nz ? force_face<NDIM>(G, ph, pp, rho, P, Z, k, k) : 0.0;
    const double r = rho[P], inv_rs = 1.0 / rho_star[P], phz = phi.p[Z][P];
    double fhi_d[NDIM - 1], flo_d[NDIM - 1];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int q = coord(c, d);
      fhi_d[d] = q + 1 < G.n[d] ? phi.p[d][P] : 0.0;
      flo_d[d] = q > 0 ? phi.p[d][P - G.st[d]] : 0.0;
    }
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      const double* uc = u.p[cc];
      double conv = 0.0, visc = 0.0;
      Line s[NDIM - 1];
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int st = G.st[d], n = G.n[d], q = coord(c, d);
        s[d] = line_at([&](int Q) { return uc[Q]; }, P, st, q, n);
        if (q + 1 < n) conv += fhi_d[d] * i4_hi(s[d], q, n);
        if (q > 0) conv -= flo_d[d] * i4_lo(s[d], q, n);
      }
      double fh = 0.0;
      if (k + 1 < nz) {
        fh = phz * i4_hi(z[cc], k, nz);
        conv += fh;
      }
      if (k > 0) conv -= flo[cc];
      flo[cc] = fh;
#pragma unroll
      for (int d = 0; d < Z; ++d)
        visc_add(visc, s[d], coord(c, d), G.n[d], ph.mu * G.S[d] / G.h[d], cc == d);
      visc_add(visc, z[cc], k, nz, kvz, cc == Z);
      double RF;
      if (cc == Z) {
        RF = 0.5 * (Flo + Fhi);
      } else {
        const int st = G.st[cc], n = G.n[cc], q = coord(c, cc);
        const double hi = q + 1 < n ? force_face<NDIM>(G, ph, pp, rho, P, cc, q, k) : 0.0;
        const double lo = q > 0 ? force_face<NDIM>(G, ph, pp, rho, P - st, cc, q - 1, k) : 0.0;
        RF = 0.5 * (lo + hi);
      }
      const double mom = r * z[cc].c - ph.dt / G.V * (conv - visc) - ph.dt * RF;
      u_star.p[cc][P] = mom * inv_rs;
      z[cc] = shift(z[cc], k + 3 < nz ? uc[P + 3 * pl] : 0.0);
    }
    Flo = Fhi;
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
    Geo G, Phys ph, int kc, const double* __restrict__ rho, const double* __restrict__ e0,
    const double* __restrict__ e_prev, const double* __restrict__ T_prev, Vec<NDIM> phi,
    const double* __restrict__ rho_star, Vec<NDIM> u_star, const double* __restrict__ Tbg,
    double* __restrict__ e_next, double* __restrict__ T_next, int last,
    const double* __restrict__ p, double* __restrict__ rho23, double* __restrict__ psi,
    double* __restrict__ cc, double* __restrict__ D) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  if (!c.act) return;
  const int nz = G.n[Z], pl = c.pl;
  auto hhat = [&](int Q) { return e_prev[Q] + ph.R * T_prev[Q]; };
  int P = c.base + pl * c.k0;
  Line ze = line_at([&](int Q) { return e_prev[Q]; }, P, pl, c.k0, nz);
  Line zT = line_at([&](int Q) { return T_prev[Q]; }, P, pl, c.k0, nz);
  auto hz_of = [&]() {
    return Line{ze.m2 + ph.R * zT.m2, ze.m1 + ph.R * zT.m1, ze.c + ph.R * zT.c,
                ze.p1 + ph.R * zT.p1, ze.p2 + ph.R * zT.p2};
  };
  double flo = c.k0 > 0 ? phi.p[Z][P - pl] * i4_lo(hz_of(), c.k0, nz) : 0.0;
  const double kdz = ph.mu / ph.Pr * ph.cp * G.S[Z] / G.h[Z];
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    double conv = 0.0;
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int st = G.st[d], n = G.n[d], q = coord(c, d);
      const Line s = line_at(hhat, P, st, q, n);
      if (q + 1 < n) conv += phi.p[d][P] * i4_hi(s, q, n);
      if (q > 0) conv -= phi.p[d][P - st] * i4_lo(s, q, n);
    }
    double fh = 0.0;
    if (k + 1 < nz) {
      fh = phi.p[Z][P] * i4_hi(hz_of(), k, nz);
      conv += fh;
    }
    if (k > 0) conv -= flo;
    flo = fh;
    const double Tp = zT.c - Tbg[k];
    double diff = 0.0;
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int st = G.st[d], n = G.n[d], q = coord(c, d);
      const double kd = ph.mu / ph.Pr * ph.cp * G.S[d] / G.h[d];
      if (q + 1 < n) diff += kd * ((T_prev[P + st] - Tbg[k]) - Tp);
      if (q > 0) diff += kd * ((T_prev[P - st] - Tbg[k]) - Tp);
    }
    if (k + 1 < nz) diff += kdz * ((zT.p1 - Tbg[k + 1]) - Tp);
    if (k > 0) diff += kdz * ((zT.m1 - Tbg[k - 1]) - Tp);
    const double inv_rs = 1.0 / rho_star[P];
    const double rhoe = rho[P] * e0[P] - ph.dt * G.inv_V * conv + ph.dt * G.inv_V * diff;
    const double e = rhoe * inv_rs;
    const double T = (e - kinetic<NDIM>(u_star, P) - phi_cell(G, ph, k)) * ph.inv_cv;
    e_next[P] = e;
    T_next[P] = T;
    if (last) {
      const double ps = 1.0 / (ph.R * T);
      const double r23 = p[P] * ps;
      rho23[P] = r23;
      psi[P] = ps;
      cc[P] = ps * G.V * ph.inv_dt;
      D[P] = r23 * ph.dt * inv_rs;
    }
    const bool more = k + 3 < nz;
    ze = shift(ze, more ? e_prev[P + 3 * pl] : 0.0);
    zT = shift(zT, more ? T_prev[P + 3 * pl] : 0.0);
  }
}

// ---- Step 3 ----------------------------------------------------------------

// H(u) = rho^n u^n/dt - (1/V) sum_out phi I4(u) + (1/V) sum mu snGrad(u) S
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_H(Geo G, Phys ph, int kc,
                                              const double* __restrict__ rho, Vec<NDIM> u,
                                              Vec<NDIM> u_prev, Vec<NDIM> phi, Vec<NDIM> H) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  if (!c.act) return;
  const int nz = G.n[Z], pl = c.pl;
  int P = c.base + pl * c.k0;
  Line z[NDIM];
  double flo[NDIM];
  const double phz_lo = c.k0 > 0 ? phi.p[Z][P - pl] : 0.0;
#pragma unroll
  for (int cc = 0; cc < NDIM; ++cc) {
    const double* uc = u_prev.p[cc];
    z[cc] = line_at([&](int Q) { return uc[Q]; }, P, pl, c.k0, nz);
    flo[cc] = c.k0 > 0 ? phz_lo * i4_lo(z[cc], c.k0, nz) : 0.0;
  }
  const double kvz = ph.mu * G.S[Z] / G.h[Z];
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    const double r = rho[P], phz = phi.p[Z][P];
    double fhi_d[NDIM - 1], flo_d[NDIM - 1];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int q = coord(c, d);
      fhi_d[d] = q + 1 < G.n[d] ? phi.p[d][P] : 0.0;
      flo_d[d] = q > 0 ? phi.p[d][P - G.st[d]] : 0.0;
    }
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      const double* uc = u_prev.p[cc];
      double conv = 0.0, visc = 0.0;
      Line s[NDIM - 1];
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int st = G.st[d], n = G.n[d], q = coord(c, d);
        s[d] = line_at([&](int Q) { return uc[Q]; }, P, st, q, n);
        if (q + 1 < n) conv += fhi_d[d] * i4_hi(s[d], q, n);
        if (q > 0) conv -= flo_d[d] * i4_lo(s[d], q, n);
      }
      double fh = 0.0;
      if (k + 1 < nz) {
        fh = phz * i4_hi(z[cc], k, nz);
        conv += fh;
      }
      if (k > 0) conv -= flo[cc];
      flo[cc] = fh;
#pragma unroll
      for (int d = 0; d < Z; ++d)
        visc_add(visc, s[d], coord(c, d), G.n[d], ph.mu * G.S[d] / G.h[d], cc == d);
      visc_add(visc, z[cc], k, nz, kvz, cc == Z);
      H.p[cc][P] = r * u.p[cc][P] * ph.inv_dt - conv * G.inv_V + visc * G.inv_V;
      z[cc] = shift(z[cc], k + 3 < nz ? uc[P + 3 * pl] : 0.0);
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
  return Df * G.S[d] * (Hf + phi_face<NDIM>(G, ph, d, cq, kz) * (rho23[Q + st] - rho23[Q]) * G.inv_h[d]);
}

// b = (V/dt)(rho^n + psi rho23 Phi) - sum_out phitilde; 1/diag of the operator
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_rhs(Geo G, Phys ph, int kc,
                                                const double* __restrict__ rho,
                                                const double* __restrict__ rho23,
                                                const double* __restrict__ psi,
                                                const double* __restrict__ cc,
                                                const double* __restrict__ D, Vec<NDIM> H,
                                                double* __restrict__ b, double* __restrict__ dinv) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  if (!c.act) return;
  const int nz = G.n[Z], pl = c.pl;
  const double kz_ = G.S[Z] / G.h[Z];
  int P = c.base + pl * c.k0;
  double flux_lo = 0.0, diag_lo = 0.0;
  if (c.k0 > 0) {
    flux_lo = phi_tilde<NDIM>(G, ph, D, H.p[Z], rho23, P - pl, Z, c.k0 - 1, c.k0 - 1);
    diag_lo = 0.5 * (D[P - pl] + D[P]) * kz_;
  }
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    double sum = 0.0;
    double diag = cc[P];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int st = G.st[d], q = coord(c, d);
      const double kd = G.S[d] / G.h[d];
      if (q + 1 < G.n[d]) {
        sum += phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P, d, q, k);
        diag += 0.5 * (D[P] + D[P + st]) * kd;
      }
      if (q > 0) {
        sum -= phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P - st, d, q - 1, k);
        diag += 0.5 * (D[P - st] + D[P]) * kd;
      }
    }
    double flux_hi = 0.0, diag_hi = 0.0;
    if (k + 1 < nz) {
      flux_hi = phi_tilde<NDIM>(G, ph, D, H.p[Z], rho23, P, Z, k, k);
      diag_hi = 0.5 * (D[P] + D[P + pl]) * kz_;
      sum += flux_hi;
      diag += diag_hi;
    }
    if (k > 0) {
      sum -= flux_lo;
      diag += diag_lo;
    }
    flux_lo = flux_hi;
    diag_lo = diag_hi;
    const double Phi = phi_cell(G, ph, k);
    b[P] = G.V / ph.dt * (rho[P] + psi[P] * rho23[P] * Phi) - sum;
    dinv[P] = 1.0 / diag;
  }
}

// u = (H - R(F))/A with F from p' and rho23, A = rho*/dt.  The last corrector
// also takes rho^{n+1} = rho^n - dt/V sum_out (phitilde - w (p'_N - p'_P)),
// p^{n+1} = p' - rho23 Phi, and reduces [mass, max |rho - psi p|, non-finite count].
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_correct(
    Geo G, Phys ph, int kc, const double* __restrict__ pp, const double* __restrict__ rho23,
    const double* __restrict__ psi, Vec<NDIM> H, const double* __restrict__ D,
    const double* __restrict__ rho_star, Vec<NDIM> u_out, int last,
    const double* __restrict__ rho_old, double* __restrict__ rho_new, double* __restrict__ p_new,
    double* partials) {
  constexpr int Z = NDIM - 1;
  double red[3] = {0.0, 0.0, 0.0};
  const Col c = col_of<NDIM>(G, kc);
  if (c.act) {
    const int nz = G.n[Z], pl = c.pl;
    const double kz_ = G.S[Z] / G.h[Z];
    int P = c.base + pl * c.k0;
    double Flo = 0.0, flux_lo = 0.0;
    if (c.k0 > 0) {
      Flo = force_face<NDIM>(G, ph, pp, rho23, P - pl, Z, c.k0 - 1, c.k0 - 1);
      if (last) {
        const double w = 0.5 * (D[P - pl] + D[P]) * kz_;
        flux_lo = phi_tilde<NDIM>(G, ph, D, H.p[Z], rho23, P - pl, Z, c.k0 - 1, c.k0 - 1) -
                  w * (pp[P] - pp[P - pl]);
      }
    }
    for (int k = c.k0; k < c.k1; ++k, P += pl) {
      const double inv_A = ph.dt / rho_star[P];
      const double Fhi = k + 1 < nz ? force_face<NDIM>(G, ph, pp, rho23, P, Z, k, k) : 0.0;
      bool finite = true;
#pragma unroll
      for (int cmp = 0; cmp < NDIM; ++cmp) {
        double RF;
        if (cmp == Z) {
          RF = 0.5 * (Flo + Fhi);
        } else {
          const int st = G.st[cmp], n = G.n[cmp], q = coord(c, cmp);
          const double hi = q + 1 < n ? force_face<NDIM>(G, ph, pp, rho23, P, cmp, q, k) : 0.0;
          const double lo = q > 0 ? force_face<NDIM>(G, ph, pp, rho23, P - st, cmp, q - 1, k) : 0.0;
          RF = 0.5 * (lo + hi);
        }
        const double un = (H.p[cmp][P] - RF) * inv_A;
        u_out.p[cmp][P] = un;
        finite = finite && isfinite(un);
      }
      Flo = Fhi;
      if (last) {
        double sum = 0.0;
#pragma unroll
        for (int d = 0; d < Z; ++d) {
          const int st = G.st[d], q = coord(c, d);
          const double kd = G.S[d] / G.h[d];
          if (q + 1 < G.n[d]) {
            const double w = 0.5 * (D[P] + D[P + st]) * kd;
            sum += phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P, d, q, k) - w * (pp[P + st] - pp[P]);
          }
          if (q > 0) {
            const double w = 0.5 * (D[P - st] + D[P]) * kd;
            sum -= phi_tilde<NDIM>(G, ph, D, H.p[d], rho23, P - st, d, q - 1, k) -
                   w * (pp[P] - pp[P - st]);
          }
        }
        double flux_hi = 0.0;
        if (k + 1 < nz) {
          const double w = 0.5 * (D[P] + D[P + pl]) * kz_;
          flux_hi = phi_tilde<NDIM>(G, ph, D, H.p[Z], rho23, P, Z, k, k) - w * (pp[P + pl] - pp[P]);
          sum += flux_hi;
        }
        if (k > 0) sum -= flux_lo;
        flux_lo = flux_hi;
        const double rn = rho_old[P] - ph.dt / G.V * sum;
        const double pn = pp[P] - rho23[P] * phi_cell(G, ph, k);
        rho_new[P] = rn;
        p_new[P] = pn;
        red[0] += rn * G.V;
        red[1] = fmax(red[1], fabs(rn - psi[P] * pn));
        finite = finite && isfinite(rn) && isfinite(pn);
      }
      red[2] += finite ? 0.0 : 1.0;
    }
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

// Column tiles of the z-marching kernels: the default chunk of planes, made
// longer on large meshes so that there are at most kMaxZBlocks workgroups
// (each leaves per-workgroup partials) unless the columns alone need more.
template <int NDIM>
ZPlan zplan_t(const Geo& G) {
  using T = ZTile<NDIM>;
  const int ntx = (G.nx + T::TX - 1) / T::TX;
  const int nty = NDIM == 3 ? (G.ny + T::TY - 1) / T::TY : 1;
  const int cols = ntx * nty, nz = G.n[NDIM - 1];
  int kc = T::KC < nz ? T::KC : nz;
  int nk = (nz + kc - 1) / kc;
  const int maxk = kMaxZBlocks / cols > 1 ? kMaxZBlocks / cols : 1;
  if (nk > maxk) {
    kc = (nz + maxk - 1) / maxk;
    nk = (nz + kc - 1) / kc;
  }
  return ZPlan{kc, cols * nk};
}

ZPlan zplan(const Geo& G) { return G.ndim == 2 ? zplan_t<2>(G) : zplan_t<3>(G); }

#define V2(a) vec<2>(a)
#define V3(a) vec<3>(a)

void launch_mass_flux(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                      double* const* u, double* const* phi, double* rho_star) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_mass_flux<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V2(u), V2(phi), rho_star);
  else
    hipLaunchKernelGGL(k_mass_flux<3>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V3(u), V3(phi), rho_star);
}

void launch_mom_predict(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                        double* const* u, const double* pp, const double* rho_star,
                        double* const* phi, double* const* u_star) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_mom_predict<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V2(u), pp, rho_star, V2(phi), V2(u_star));
  else
    hipLaunchKernelGGL(k_mom_predict<3>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V3(u), pp, rho_star, V3(phi), V3(u_star));
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
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_energy_sweep<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, e0, e_prev, T_prev, V2(phi), rho_star, V2(u_star), Tbg, e_next, T_next, (int)last, p, rho23, psi, c, D);
  else
    hipLaunchKernelGGL(k_energy_sweep<3>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, e0, e_prev, T_prev, V3(phi), rho_star, V3(u_star), Tbg, e_next, T_next, (int)last, p, rho23, psi, c, D);
}

void launch_H(hipStream_t s, const Geo& G, const Phys& ph, const double* rho, double* const* u,
              double* const* u_prev, double* const* phi, double* const* H) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_H<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V2(u), V2(u_prev), V2(phi), V2(H));
  else
    hipLaunchKernelGGL(k_H<3>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V3(u), V3(u_prev), V3(phi), V3(H));
}

void launch_rhs(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                const double* rho23, const double* psi, const double* c, const double* D,
                double* const* H, double* b, double* dinv) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_rhs<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, rho23, psi, c, D, V2(H), b, dinv);
  else
    hipLaunchKernelGGL(k_rhs<3>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, rho23, psi, c, D, V3(H), b, dinv);
}

void launch_correct(hipStream_t s, const Geo& G, const Phys& ph, const double* pp,
                    const double* rho23, const double* psi, double* const* H, const double* D,
                    const double* rho_star, double* const* u_out, bool last,
                    const double* rho_old, double* rho_new, double* p_new, double* partials,
                    CgScalars* sc) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_correct<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, pp, rho23, psi, V2(H), D, rho_star, V2(u_out), (int)last, rho_old, rho_new, p_new, partials);
  else
    hipLaunchKernelGGL(k_correct<3>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, pp, rho23, psi, V3(H), D, rho_star, V3(u_out), (int)last, rho_old, rho_new, p_new, partials);
  if (last)
    hipLaunchKernelGGL(k_finalize_reduce, dim3(1), dim3(kBlock), 0, s, (const double*)partials, zp.blocks, sc);
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
