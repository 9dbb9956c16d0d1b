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
#include "gea_stencil.h"

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


// mu snGrad(u_comp) S on the two faces of a line; walls normal to the line
// hold the normal component at 0 and leave the tangential ones free
__device__ __forceinline__ void visc_add(double& acc, const Line& s, int q, int n, double k,
                                         bool normal) {
  const double wall = normal ? 2.0 * k * (0.0 - s.c) : 0.0;
  acc += q + 1 < n ? k * (s.p1 - s.c) : wall;
  acc += q > 0 ? k * (s.m1 - s.c) : wall;
}

// F = grad p' - Phi grad rho on a face, from the values on its two sides
// (low, high along the face normal)
__device__ __forceinline__ double force_val(double p_lo, double p_hi, double r_lo, double r_hi,
                                            double phif, double inv_h) {
  return ((p_hi - p_lo) - phif * (r_hi - r_lo)) * inv_h;
}

// predicted flux on a face from its two sides' D, H.n and rho23:
// D_f S [H_f . n + Phi_f (rho23_N - rho23_P)/h]
__device__ __forceinline__ double phit_val(double D_lo, double D_hi, double H_lo, double H_hi,
                                           double r_lo, double r_hi, double S, double phif,
                                           double inv_h) {
  const double Df = 0.5 * (D_lo + D_hi);
  const double Hf = 0.5 * (H_lo + H_hi);
  return Df * S * (Hf + phif * (r_hi - r_lo) * inv_h);
}

// the five staged values of a line through the own cell, stride 1 (x) or HX (y)
__device__ __forceinline__ Line line_lds(const double* s, int h, int str) {
  return Line{s[h - 2 * str], s[h - str], s[h], s[h + str], s[h + 2 * str]};
}


// ---- Step 1 ----------------------------------------------------------------

// rho* = rho - dt/V sum_out phi with the state's face flux phi (eq. e1_d);
// also e^n = c_v T + K + Phi, the total energy the Step 2 sweeps start from
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_density_predictor(Geo G, Phys ph, int kc,
                                                              const double* __restrict__ rho,
                                                              Vec<NDIM> u, const double* __restrict__ T,
                                                              Vec<NDIM> phi, double* __restrict__ rho_star,
                                                              double* __restrict__ e0) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  if (!c.act) return;
  const int nz = G.n[Z], pl = c.pl;
  int P = c.base + pl * c.k0;
  double flo = c.k0 > 0 ? phi.p[Z][P - pl] : 0.0;
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    // loads of the plane
    double fh[NDIM - 1], fl[NDIM - 1];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      fh[d] = phi.p[d][P];
      fl[d] = phi.p[d][nb(coord(c, d) > 0, P - G.st[d], P)];
    }
    const double fz = phi.p[Z][P], r = rho[P], Tc = T[P];
    double uc[NDIM];
#pragma unroll
    for (int d = 0; d < NDIM; ++d) uc[d] = u.p[d][P];
    // net outward flux
    double sum = 0.0;
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int n = G.n[d], q = coord(c, d);
      sum += q + 1 < n ? fh[d] : 0.0;
      sum -= q > 0 ? fl[d] : 0.0;
    }
    const double hi = k + 1 < nz ? fz : 0.0;
    sum += hi;
    sum -= flo;
    flo = hi;
    rho_star[P] = r - ph.dt / G.V * sum;
    double kin = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) kin += uc[d] * uc[d];
    e0[P] = ph.cv * Tc + 0.5 * kin + phi_cell(G, ph, k);
  }
}

// a given face flux: the upper wall faces hold 0
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_clear_wall_faces(Geo G, Vec<NDIM> phi) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < G.nc; P += gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
      if ((P / G.st[d]) % G.n[d] + 1 == G.n[d]) phi.p[d][P] = 0.0;
  }
}

// phi_f = I4(rho u . n)_f S_f on interior faces, 0 on walls (eq. e1_d from
// the cell fields): the flux of a state given by its cell fields alone
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_face_mass_flux(Geo G, const double* __restrict__ rho,
                                                           Vec<NDIM> u, Vec<NDIM> phi) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < G.nc; P += gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int st = G.st[d], n = G.n[d], i = (P / st) % n;
      const double* ud = u.p[d];
      double v = 0.0;
      if (i + 1 < n) {
        const double mc = rho[P] * ud[P], mp = rho[P + st] * ud[P + st];
        if (i >= 1 && i + 2 <= n - 1)
          v = (-(rho[P - st] * ud[P - st]) + 9.0 * mc + 9.0 * mp - rho[P + 2 * st] * ud[P + 2 * st]) / 16.0;
        else
          v = 0.5 * (mc + mp);
        v *= G.S[d];
      }
      phi.p[d][P] = v;
    }
  }
}

// rho* u* = rho u - dt/V [sum_out phi I4(u) - sum mu snGrad(u) S] - dt R(F)
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_mom_predict(Geo G, Phys ph, int kc,
                                                        const double* __restrict__ rho, Vec<NDIM> u,
                                                        const double* __restrict__ pp,
                                                        const double* __restrict__ rho_star,
                                                        Vec<NDIM> phi, Vec<NDIM> u_star,
                                                        double* __restrict__ pp_copy,
                                                        Vec<NDIM> b_out, double* __restrict__ Ks) {
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
  double Flo = 0.0;
  if (c.k0 > 0)
    Flo = force_val(pp[P - pl], pp[P], rho[P - pl], rho[P], phi_face<NDIM>(G, ph, Z, c.k0 - 1, c.k0 - 1),
                    G.inv_h[Z]);
  const double kvz = ph.mu * G.S[Z] / G.h[Z];
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    // loads of the plane
    const bool up = k + 1 < nz;
    const int Pu = nb(up, P + pl, P), Pn = nb(k + 3 < nz, P + 3 * pl, P);
    const double r = rho[P], pc = pp[P], rs = rho_star[P], phz = phi.p[Z][P];
    const double p_up = pp[Pu], r_up = rho[Pu];
    double fhi[NDIM - 1], flod[NDIM - 1], p_hi[NDIM - 1], p_lo[NDIM - 1], r_hi[NDIM - 1],
        r_lo[NDIM - 1];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int st = G.st[d], q = coord(c, d);
      const int Ph = nb(q + 1 < G.n[d], P + st, P), Pl = nb(q > 0, P - st, P);
      fhi[d] = phi.p[d][P];
      flod[d] = phi.p[d][Pl];
      p_hi[d] = pp[Ph];
      p_lo[d] = pp[Pl];
      r_hi[d] = rho[Ph];
      r_lo[d] = rho[Pl];
    }
    Line s[NDIM][NDIM - 1];
    double zn[NDIM];
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      const double* uc = u.p[cc];
#pragma unroll
      for (int d = 0; d < Z; ++d)
        s[cc][d] = line_at([&](int Q) { return uc[Q]; }, P, G.st[d], coord(c, d), G.n[d]);
      zn[cc] = uc[Pn];
    }
    // update
    const double Fhi = up ? force_val(pc, p_up, r, r_up, phi_face<NDIM>(G, ph, Z, k, k), G.inv_h[Z]) : 0.0;
    const double inv_rs = 1.0 / rs;
    double us[NDIM];
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      double conv = 0.0, visc = 0.0;
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int n = G.n[d], q = coord(c, d);
        conv = q + 1 < n ? conv + fhi[d] * i4_hi(s[cc][d], q, n) : conv;
        conv = q > 0 ? conv - flod[d] * i4_lo(s[cc][d], q, n) : conv;
      }
      double fh = 0.0;
      if (up) {
        fh = phz * i4_hi(z[cc], k, nz);
        conv += fh;
      }
      if (k > 0) conv -= flo[cc];
      flo[cc] = fh;
#pragma unroll
      for (int d = 0; d < Z; ++d)
        visc_add(visc, s[cc][d], coord(c, d), G.n[d], ph.mu * G.S[d] / G.h[d], cc == d);
      visc_add(visc, z[cc], k, nz, kvz, cc == Z);
      double RF;
      if (cc == Z) {
        RF = 0.5 * (Flo + Fhi);
      } else {
        const int n = G.n[cc], q = coord(c, cc);
        const double phf = phi_cell(G, ph, k);
        const double hi = q + 1 < n ? force_val(pc, p_hi[cc], r, r_hi[cc], phf, G.inv_h[cc]) : 0.0;
        const double lo = q > 0 ? force_val(p_lo[cc], pc, r_lo[cc], r, phf, G.inv_h[cc]) : 0.0;
        RF = 0.5 * (lo + hi);
      }
      const double mom = r * z[cc].c - ph.dt / G.V * (conv - visc) - ph.dt * RF;
      us[cc] = mom * inv_rs;
      // implicit transport: the predictor system's right-hand side V (rho u/dt - R(F))
      if (b_out.p[0]) b_out.p[cc][P] = G.V * (r * z[cc].c / ph.dt - RF);
    }
    double ks = 0.0;
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      u_star.p[cc][P] = us[cc];
      ks += us[cc] * us[cc];
      z[cc] = shift(z[cc], k + 3 < nz ? zn[cc] : 0.0);
    }
    if (Ks) Ks[P] = 0.5 * ks;  // K* for the energy sweeps
    if (pp_copy) pp_copy[P] = pc;
    Flo = Fhi;
  }
}

// Step 1 on a 3D mesh in one pass: k_density_predictor's rho* and e^n from
// the state's face flux, then k_mom_predict's momentum predictor, which
// takes the own cell's six face fluxes and rho*.  Same formulas and order as
// the two kernels.  The x/y neighbourhoods of u (two cells, for I4) and of p'
// and rho (one cell, for the force) are staged in rings of three LDS planes
// filled three planes ahead of the plane computed; the staged own values of
// plane k + 2 feed the register lines of u along z, and those of plane k + 1
// the force on the face above, so each value is loaded from HBM once a chunk
// (as in k_H3).
template <int TY>
__global__ __launch_bounds__(64 * TY) void k_step1_3(Geo G, Phys ph, int kc,
                                                    const double* __restrict__ rho, Vec<3> u,
                                                    const double* __restrict__ T,
                                                    const double* __restrict__ pp, Vec<3> phi,
                                                    double* __restrict__ rho_star,
                                                    double* __restrict__ e0, Vec<3> u_star,
                                                    double* __restrict__ pp_copy, Vec<3> b_out,
                                                    double* __restrict__ Ks) {
  using St = Stage3<2, TY>;
  using St1 = Stage3<1, TY>;
  constexpr int Z = 2, HP = St::HP, HX = St::HX, NU = St::NU;
  constexpr int HP1 = St1::HP, HX1 = St1::HX, NU1 = St1::NU;
  __shared__ double su[3][3][HP];   // u (3 components): two-cell halo (I4)
  __shared__ double sq[3][2][HP1];  // p', rho: one-cell halo (the force)
  const Col c = col_of3<TY>(G, kc);
  const St st = stage3<2, TY>(G, c);
  const St1 st1 = stage3<1, TY>(G, c);
  const int nz = G.n[Z], pl = c.pl, qo = st.qo, ho = st.ho, ho1 = st1.ho;
  const int Pxl = nb(clampi(c.i, G.nx) > 0, qo - 1, qo);
  const int Pyl = nb(clampi(c.j, G.ny) > 0, qo - G.nx, qo);
  // highest plane the chunk reads; planes above the chunk are loaded for the
  // own column only (the halo slots load it again)
  const int ktop = min(c.k1 + 1, nz - 1);
  struct Planes {
    double u[3][NU], q[2][NU1];  // u; p' and rho
  };
  Planes fs;                     // staged plane in flight
  double fT, fph[3], fpl[2];     // own cell's values of the next plane
  auto fetch = [&](int kk, Planes& dst) {
    const int kq = min(kk, ktop), o = pl * kq;
    const bool halo = kq < c.k1;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int Q = (halo ? st.q[m] : qo) + o;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) dst.u[cc][m] = u.p[cc][Q];
    }
#pragma unroll
    for (int m = 0; m < NU1; ++m) {
      const int Q = (halo ? st1.q[m] : qo) + o;
      dst.q[0][m] = pp[Q];
      dst.q[1][m] = rho[Q];
    }
  };
  auto own = [&](int kk) {
    const int o = pl * min(kk, c.k1 - 1), P = qo + o;
    fT = T[P];
    fph[0] = phi.p[0][P];
    fph[1] = phi.p[1][P];
    fph[2] = phi.p[Z][P];
    fpl[0] = phi.p[0][Pxl + o];
    fpl[1] = phi.p[1][Pyl + o];
  };
  auto stage = [&](int sl, const Planes& src) {
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int m = 0; m < NU; ++m)
        su[sl][f][st.h[m]] = src.u[f][m];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int m = 0; m < NU1; ++m)
        sq[sl][f][st1.h[m]] = src.q[f][m];
  };
  Line z[3];       // u along z (momentum); planes k0-3 .. k0+1 before the loop
  double flo[3];   // momentum flux through the face below
  double fmlo;     // mass flux through the face below
  double Flo = 0.0;
  {
    const int P = qo + pl * c.k0;
    fmlo = c.k0 > 0 ? phi.p[Z][P - pl] : 0.0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double* uc = u.p[cc];
      z[cc].m2 = 0.0;
      z[cc].m1 = uc[nb(c.k0 >= 2, P - 2 * pl, P)];
      z[cc].c = uc[nb(c.k0 >= 1, P - pl, P)];
    }
    if (c.k0 > 0)
      Flo = force_val(pp[P - pl], pp[P], rho[P - pl], rho[P],
                      phi_face<3>(G, ph, Z, c.k0 - 1, c.k0 - 1), G.inv_h[Z]);
    Planes f1;  // the chunk's first two planes are loaded together
    fetch(c.k0, fs);
    fetch(c.k0 + 1, f1);
    stage(0, fs);
    stage(1, f1);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      z[cc].p1 = fs.u[cc][0];
      z[cc].p2 = f1.u[cc][0];
      const Line L{z[cc].m1, z[cc].c, z[cc].p1, z[cc].p2, 0.0};  // centred on k0
      flo[cc] = c.k0 > 0 ? fmlo * i4_lo(L, c.k0, nz) : 0.0;
    }
  }
  own(c.k0);
  fetch(c.k0 + 2, fs);
  const double kvz = ph.mu * G.S[Z] / G.h[Z];
  int sl = 0;  // slot of plane k
  for (int k = c.k0; k < c.k1; ++k) {
    // every thread is done with plane k-1, whose slot takes plane k+2
    lds_barrier();
    stage(sl == 0 ? 2 : sl - 1, fs);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) z[cc] = shift(z[cc], fs.u[cc][0]);
    const double Tc = fT;
    const double fh3[3] = {fph[0], fph[1], fph[2]}, fl2[2] = {fpl[0], fpl[1]};
    own(k + 1);
    fetch(k + 3, fs);
    const bool up = k + 1 < nz;
    const double* Sp = sq[sl][0];
    const double* Sr = sq[sl][1];
    const int su1 = sl == 2 ? 0 : sl + 1;  // slot of plane k+1
    const double r = Sr[ho1], pc = Sp[ho1];
    const double p_up = sq[su1][0][ho1], r_up = sq[su1][1][ho1];
    // the state's flux through the faces of the cell, rho*, e^n
    double sum = 0.0, fhi[2], flod[2];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int n = G.n[d], q = coord(c, d);
      fhi[d] = q + 1 < n ? fh3[d] : 0.0;
      flod[d] = q > 0 ? fl2[d] : 0.0;
      sum += fhi[d];
      sum -= flod[d];
    }
    const double phz = up ? fh3[Z] : 0.0;
    sum += phz;
    sum -= fmlo;
    fmlo = phz;
    const double rs = r - ph.dt / G.V * sum;
    double kin = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) kin += z[d].c * z[d].c;
    const double e0c = ph.cv * Tc + 0.5 * kin + phi_cell(G, ph, k);
    // momentum predictor
    const double Fhi = up ? force_val(pc, p_up, r, r_up, phi_face<3>(G, ph, Z, k, k), G.inv_h[Z]) : 0.0;
    const double inv_rs = 1.0 / rs;
    double us[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const Line s[2] = {line_lds(su[sl][cc], ho, 1), line_lds(su[sl][cc], ho, HX)};
      double conv = 0.0, visc = 0.0;
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int n = G.n[d], q = coord(c, d);
        conv = q + 1 < n ? conv + fhi[d] * i4_hi(s[d], q, n) : conv;
        conv = q > 0 ? conv - flod[d] * i4_lo(s[d], q, n) : conv;
      }
      double fhz = 0.0;
      if (up) {
        fhz = phz * i4_hi(z[cc], k, nz);
        conv += fhz;
      }
      if (k > 0) conv -= flo[cc];
      flo[cc] = fhz;
#pragma unroll
      for (int d = 0; d < Z; ++d)
        visc_add(visc, s[d], coord(c, d), G.n[d], ph.mu * G.S[d] / G.h[d], cc == d);
      visc_add(visc, z[cc], k, nz, kvz, cc == Z);
      double RF;
      if (cc == Z) {
        RF = 0.5 * (Flo + Fhi);
      } else {
        const int n = G.n[cc], q = coord(c, cc), sd = cc == 0 ? 1 : HX1;
        const double phf = phi_cell(G, ph, k);
        const double hi = q + 1 < n ? force_val(pc, Sp[ho1 + sd], r, Sr[ho1 + sd], phf, G.inv_h[cc]) : 0.0;
        const double lo = q > 0 ? force_val(Sp[ho1 - sd], pc, Sr[ho1 - sd], r, phf, G.inv_h[cc]) : 0.0;
        RF = 0.5 * (lo + hi);
      }
      const double mom = r * z[cc].c - ph.dt / G.V * (conv - visc) - ph.dt * RF;
      us[cc] = mom * inv_rs;
      // implicit transport: the predictor system's right-hand side V (rho u/dt - R(F))
      if (b_out.p[0] && c.act) b_out.p[cc][qo + pl * k] = G.V * (r * z[cc].c / ph.dt - RF);
    }
    if (c.act) {
      const int P = qo + pl * k;
      rho_star[P] = rs;
      e0[P] = e0c;
      double ks = 0.0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        u_star.p[cc][P] = us[cc];
        ks += us[cc] * us[cc];
      }
      if (Ks) Ks[P] = 0.5 * ks;  // K* for the energy sweeps
      if (pp_copy) pp_copy[P] = pc;
    }
    Flo = Fhi;
    sl = su1;
  }
}

// ---- Step 2 ----------------------------------------------------------------

// Step 2, sweep s: the right-hand side of the implicit-diffusion system
//   c T + sum_f k_f (T_P - T_nb) = b,   c = rho* c_v V/dt,  k_f = (mu/Pr) c_p S_f/h_f,
//   b = V/dt (rho^n e^n - rho* (K* + Phi)) - sum_out phi I4(e + R T)^(s-1)
//       + sum_f k_f (T_bg,P - T_bg,nb)
// (the total-energy balance times V/dt with e = c_v T + K* + Phi, the
// diffusion of h' = c_p (T - T_bg) at the new level, the convective flux
// from the previous sweep with the frozen Step-1 flux), its 1/diag, the
// initial guess T^(s-1) and the solve's set-up as the CG set-up kernel forms
// it: r = b - A T^(s-1) and the partials <r, r/diag>,
// ||r||^2 (u_part) and ||b||^2 (b_part) of each workgroup.
struct EnergySys {
  double* b;
  double* c;      // (the iteration kernels form 1/diag from c: D is a constant)
  double* x;      // the solve's initial guess (and later solution); null: T_prev itself
  double* r;
  double* u_part;
  double* b_part;
};

// The quantity a sweep transports, on a line of cells, from the two fields
// the sweep stages (a, T): KS false (the first sweep of the total-energy
// form): a = e^n and the quantity is e + R T; KS true: a = K* (written by
// Step 1) and the quantity is (c_v + R) T + K* + Phi (total energy: e + R T
// with e = c_v T + K* + Phi, so no pass forms e between sweeps) or c_p T + K*
// (enthalpy form).  kz: the line's centre plane; along z (zl) Phi changes
// from cell to cell, across a plane it does not.
template <bool ENTH, bool KS>
__device__ __forceinline__ Line transported(const Geo& G, const Phys& ph, const Line& a,
                                            const Line& T, int kz, bool zl) {
  auto one = [&](double av, double Tv, int kk) {
    if (!KS) return ENTH ? av : av + ph.R * Tv;
    return ENTH ? ph.cp * Tv + av : (ph.cv + ph.R) * Tv + av + phi_cell(G, ph, kk);
  };
  const int d = zl ? 1 : 0;
  return Line{one(a.m2, T.m2, kz - 2 * d), one(a.m1, T.m1, kz - d), one(a.c, T.c, kz),
              one(a.p1, T.p1, kz + d), one(a.p2, T.p2, kz + 2 * d)};
}

// ENTH: the enthalpy form (eq. step3_sd): e0 holds the sweep-independent
// balance q = rho^n c_p T^n + rho^n K^{n-1} - p^{n-1} - rho* K* + p^n
// - dt rho* g w*, the transported quantity is c_p T^(s-1) + K*, and the
// unknown's coefficient is rho* c_p V/dt.  Otherwise (total energy) e0 = e^n
// and the transported quantity is e + R T of the previous sweep.  KS: the
// sweep stages T^(s-1) and K* (a_prev = K*), else e^n and T^n (a_prev = e^n,
// the first sweep of the total-energy form); see transported().
template <int NDIM, bool ENTH, bool KS>
__global__ __launch_bounds__(kBlock) void k_energy_rhs(
    Geo G, Phys ph, int kc, const double* __restrict__ rho, const double* __restrict__ e0,
    const double* __restrict__ a_prev, const double* __restrict__ T_prev, Vec<NDIM> phi,
    const double* __restrict__ rho_star, const double* __restrict__ Ks,
    const double* __restrict__ Tbg, EnergySys sy) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  double red[3] = {0.0, 0.0, 0.0};
  if (c.act) {
    const int nz = G.n[Z], pl = c.pl;
    int P = c.base + pl * c.k0;
    Line ze = line_at([&](int Q) { return a_prev[Q]; }, P, pl, c.k0, nz);
    Line zT = line_at([&](int Q) { return T_prev[Q]; }, P, pl, c.k0, nz);
    auto hhat = [&](const Line& a, const Line& T, int kz, bool zl) {
      return transported<ENTH, KS>(G, ph, a, T, kz, zl);
    };
    double flo = c.k0 > 0 ? phi.p[Z][P - pl] * i4_lo(hhat(ze, zT, c.k0, true), c.k0, nz) : 0.0;
    const double kcoef = ph.mu / ph.Pr * ph.cp;
    const double kdz = kcoef * G.S[Z] / G.h[Z];      // background part of the flux
    const double wz = kcoef * (G.S[Z] / G.h[Z]);    // operator weight (D = kcoef on both sides)
    for (int k = c.k0; k < c.k1; ++k, P += pl) {
      // loads of the plane
      const int Pn = nb(k + 3 < nz, P + 3 * pl, P);
      Line le[NDIM - 1], lT[NDIM - 1];
      double fhi[NDIM - 1], flod[NDIM - 1];
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int st = G.st[d], n = G.n[d], q = coord(c, d);
        le[d] = line_at([&](int Q) { return a_prev[Q]; }, P, st, q, n);
        lT[d] = line_at([&](int Q) { return T_prev[Q]; }, P, st, q, n);
        fhi[d] = phi.p[d][P];
        flod[d] = phi.p[d][nb(q > 0, P - st, P)];
      }
      // e^n and K* of the cell: one of them is the staged a_prev's own value
      const double phz = phi.p[Z][P], rs = rho_star[P], r = rho[P], e0c = KS ? e0[P] : ze.c;
      const double ks = KS ? ze.c : Ks[P];
      const double e_n = a_prev[Pn], T_n = T_prev[Pn];
      const double tb = Tbg[k], tb_up = Tbg[k + 1 < nz ? k + 1 : k], tb_dn = Tbg[k > 0 ? k - 1 : k];
      // convective flux of e + R T
      double conv = 0.0;
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int n = G.n[d], q = coord(c, d);
        const Line h = hhat(le[d], lT[d], k, false);
        conv = q + 1 < n ? conv + fhi[d] * i4_hi(h, q, n) : conv;
        conv = q > 0 ? conv - flod[d] * i4_lo(h, q, n) : conv;
      }
      double fh = 0.0;
      if (k + 1 < nz) {
        fh = phz * i4_hi(hhat(ze, zT, k, true), k, nz);
        conv += fh;
      }
      if (k > 0) conv -= flo;
      flo = fh;
      // the background temperature's diffusion (z faces only: T_bg is a column)
      double bg = 0.0;
      if (k + 1 < nz) bg += kdz * (tb - tb_up);
      if (k > 0) bg += kdz * (tb - tb_dn);
      const double rest = ks + phi_cell(G, ph, k);
      const double bP = ENTH ? G.V / ph.dt * e0c - conv + bg : G.V / ph.dt * (r * e0c - rs * rest) - conv + bg;
      const double cP = rs * (ENTH ? ph.cp : ph.cv) * G.V / ph.dt;
      // operator on the initial guess and the diagonal
      const double xc = zT.c;
      double ax = cP * xc, diag = cP;
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int n = G.n[d], q = coord(c, d);
        const double w = kcoef * (G.S[d] / G.h[d]);
        if (q + 1 < n) {
          ax += w * (xc - lT[d].p1);
          diag += w;
        }
        if (q > 0) {
          ax += w * (xc - lT[d].m1);
          diag += w;
        }
      }
      if (k + 1 < nz) {
        ax += wz * (xc - zT.p1);
        diag += wz;
      }
      if (k > 0) {
        ax += wz * (xc - zT.m1);
        diag += wz;
      }
      // (1/diag is not stored: the iteration kernels form it from c)
      const double di = 1.0 / diag, rr = bP - ax;
      sy.b[P] = bP;
      sy.c[P] = cP;
      if (sy.x) sy.x[P] = xc;  // (null: the solve runs in place on T_prev)
      sy.r[P] = rr;
      red[0] += rr * (rr * di);
      red[1] += rr * rr;
      red[2] += bP * bP;
      const bool more = k + 3 < nz;
      ze = shift(ze, more ? e_n : 0.0);
      zT = shift(zT, more ? T_n : 0.0);
    }
  }
  __shared__ double sh[3][kBlock / 64];
  Reducer<0u, 3>::block(red, sh);
  if (threadIdx.x == 0) {
    sy.u_part[blockIdx.x] = red[0];
    sy.u_part[gridDim.x + blockIdx.x] = red[1];
    sy.b_part[blockIdx.x] = red[2];
  }
}

// The lagged terms of a state without history: p^{n-1} = p^n, K^{n-1} = K^n.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_history_init(Geo G, const double* __restrict__ p,
                                                         Vec<NDIM> u, double* __restrict__ pm,
                                                         double* __restrict__ Km) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < G.nc; P += gridDim.x * blockDim.x) {
    double kin = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) kin += u.p[d][P] * u.p[d][P];
    Km[P] = 0.5 * kin;
    pm[P] = p[P];
  }
}

// Step 2 in enthalpy form (eq. step3_sd), the sweep-independent part: the
// balance q = rho^n c_p T^n + rho^n K^{n-1} - p^{n-1} - rho* K* + p^n
// - dt rho* g w* (times V/dt it is the right-hand side without the fluxes),
// the first sweep's transported quantity c_p T^n + K*, and the next state's
// lagged terms p^n, K^n.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_enthalpy_prep(
    Geo G, Phys ph, const double* __restrict__ rho, const double* __restrict__ T,
    const double* __restrict__ p, const double* __restrict__ pm, const double* __restrict__ Km,
    Vec<NDIM> u, Vec<NDIM> u_star, const double* __restrict__ rho_star, double* __restrict__ q,
    double* __restrict__ pm_next, double* __restrict__ Km_next) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < G.nc; P += gridDim.x * blockDim.x) {
    const double r = rho[P], Tc = T[P], pc = p[P], rs = rho_star[P];
    double ks = 0.0, kn = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      ks += u_star.p[d][P] * u_star.p[d][P];
      kn += u.p[d][P] * u.p[d][P];
    }
    ks *= 0.5;
    const double hn = ph.cp * Tc;
    q[P] = r * hn + r * Km[P] - pm[P] - rs * ks + pc - ph.dt * rs * ph.g * u_star.p[NDIM - 1][P];
    pm_next[P] = pc;
    Km_next[P] = 0.5 * kn;
  }
}

// After the last sweep's solve: the EOS density of eq. step3_3sd and the
// pressure-equation coefficients: rho^{n+2/3} = p^n/(R T^{n+1}),
// psi = 1/(R T), c = psi V/dt, D = rho^{n+2/3} dt/rho*.  (Between sweeps no
// pass is needed: the next sweep forms its transported quantity from T and
// K*, see transported().)
__global__ __launch_bounds__(kBlock) void k_energy_post(
    Geo G, Phys ph, const double* __restrict__ T, const double* __restrict__ p,
    const double* __restrict__ rho_star, double* __restrict__ rho23, double* __restrict__ psi,
    double* __restrict__ cc, double* __restrict__ D) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < G.nc; P += gridDim.x * blockDim.x) {
    const double Tc = T[P];
    const double r23 = p[P] / (ph.R * Tc), ps = 1.0 / (ph.R * Tc);
    rho23[P] = r23;
    psi[P] = ps;
    cc[P] = ps * G.V / ph.dt;
    D[P] = r23 / (rho_star[P] / ph.dt);
  }
}

// k_energy_rhs on a 3D mesh with the x/y neighbourhoods of e and T staged in
// a ring of three LDS planes filled three planes ahead of the plane computed
// (the staged own values of plane k + 2 feed the register lines along z, as
// in k_H3) and the next plane's own-cell loads in flight.  Same formulas and
// order as k_energy_rhs.  On the 3D benchmark mesh: 213 us and 1162 MB of
// HBM traffic a launch, against 212 us and 1259 MB with a two-plane ring and
// separate loads of the column three planes up; held to 128 VGPRs (two
// workgroups a CU, 9 registers spilled) 223 us; 64x4 tiles in 43-plane
// chunks 222 us; 32-plane chunks 225 us.
template <int TY, bool ENTH, bool KS>
__global__ __launch_bounds__(64 * TY) void k_energy_rhs3(
    Geo G, Phys ph, int kc, const double* __restrict__ rho, const double* __restrict__ e0,
    const double* __restrict__ a_prev, const double* __restrict__ T_prev, Vec<3> phi,
    const double* __restrict__ rho_star, const double* __restrict__ Ks,
    const double* __restrict__ Tbg, EnergySys sy) {
  using St = Stage3<2, TY>;
  constexpr int Z = 2, HP = St::HP, HX = St::HX, NU = St::NU;
  __shared__ double su[3][2][HP];  // a (e^n or K*), T; plane k in slot (k - k0) % 3
  const Col c = col_of3<TY>(G, kc);
  const St st = stage3<2, TY>(G, c);
  const int nz = G.n[Z], pl = c.pl, qo = st.qo, ho = st.ho;
  const int Pxl = nb(clampi(c.i, G.nx) > 0, qo - 1, qo);
  const int Pyl = nb(clampi(c.j, G.ny) > 0, qo - G.nx, qo);
  // highest plane the chunk's z lines read; planes above the chunk are
  // loaded for the own column only (the halo slots load it again)
  const int ktop = min(c.k1 + 1, nz - 1);
  double fs[2][NU];                             // staged plane in flight
  double fh[2], fl[2], fz, frs, fr, fe0, fks;   // own cell's values of the next plane
  auto fetch = [&](int kk, double (&dst)[2][NU]) {
    const int kq = min(kk, ktop), o = pl * kq;
    const bool halo = kq < c.k1;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int Q = (halo ? st.q[m] : qo) + o;
      dst[0][m] = a_prev[Q];
      dst[1][m] = T_prev[Q];
    }
  };
  auto own = [&](int kk) {
    const int o = pl * min(kk, c.k1 - 1), P = qo + o;
    fh[0] = phi.p[0][P];
    fh[1] = phi.p[1][P];
    fl[0] = phi.p[0][Pxl + o];
    fl[1] = phi.p[1][Pyl + o];
    fz = phi.p[Z][P];
    frs = rho_star[P];
    fr = rho[P];
    // (the staged a_prev's own value is e^n (KS false) or K* (KS true))
    if (KS)
      fe0 = e0[P];
    else
      fks = Ks[P];
  };
  auto stage = [&](int sl, const double (&src)[2][NU]) {
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int m = 0; m < NU; ++m)
        su[sl][f][st.h[m]] = src[f][m];
  };
  auto hhat = [&](const Line& a, const Line& T, int kz, bool zl) {
    return transported<ENTH, KS>(G, ph, a, T, kz, zl);
  };
  // the z lines hold planes k0-3 .. k0+1 before the loop (k0-3 is never read)
  Line ze, zT;
  double flo;
  {
    const int P = qo + pl * c.k0;
    const int Q2 = nb(c.k0 >= 2, P - 2 * pl, P), Q1 = nb(c.k0 >= 1, P - pl, P);
    ze.m2 = 0.0;
    zT.m2 = 0.0;
    ze.m1 = a_prev[Q2];
    zT.m1 = T_prev[Q2];
    ze.c = a_prev[Q1];
    zT.c = T_prev[Q1];
    const double phz_lo = c.k0 > 0 ? phi.p[Z][P - pl] : 0.0;
    double f1[2][NU];  // the chunk's first two planes are loaded together
    fetch(c.k0, fs);
    fetch(c.k0 + 1, f1);
    stage(0, fs);
    stage(1, f1);
    ze.p1 = fs[0][0];
    zT.p1 = fs[1][0];
    ze.p2 = f1[0][0];
    zT.p2 = f1[1][0];
    const Line Le{ze.m1, ze.c, ze.p1, ze.p2, 0.0}, LT{zT.m1, zT.c, zT.p1, zT.p2, 0.0};  // centred on k0
    flo = c.k0 > 0 ? phz_lo * i4_lo(hhat(Le, LT, c.k0, true), c.k0, nz) : 0.0;
  }
  own(c.k0);
  fetch(c.k0 + 2, fs);
  const double kcoef = ph.mu / ph.Pr * ph.cp;
  const double kdz = kcoef * G.S[Z] / G.h[Z];
  const double wz = kcoef * (G.S[Z] / G.h[Z]);
  double red[3] = {0.0, 0.0, 0.0};
  int sl = 0;  // slot of plane k
  for (int k = c.k0; k < c.k1; ++k) {
    // every thread is done with plane k-1, whose slot takes plane k+2
    lds_barrier();
    stage(sl == 0 ? 2 : sl - 1, fs);
    ze = shift(ze, fs[0][0]);
    zT = shift(zT, fs[1][0]);
    const double fhi[2] = {fh[0], fh[1]}, flod[2] = {fl[0], fl[1]};
    const double phz = fz, rs = frs, r = fr, e0c = KS ? fe0 : ze.c;
    const double ks = KS ? ze.c : fks;  // K* of the cell
    const double tb = Tbg[k], tb_up = Tbg[k + 1 < nz ? k + 1 : k], tb_dn = Tbg[k > 0 ? k - 1 : k];
    own(k + 1);
    fetch(k + 3, fs);
    Line le[2], lT[2];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      le[d] = line_lds(su[sl][0], ho, d == 0 ? 1 : HX);
      lT[d] = line_lds(su[sl][1], ho, d == 0 ? 1 : HX);
    }
    double conv = 0.0;
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int n = G.n[d], q = coord(c, d);
      const Line h = hhat(le[d], lT[d], k, false);
      conv = q + 1 < n ? conv + fhi[d] * i4_hi(h, q, n) : conv;
      conv = q > 0 ? conv - flod[d] * i4_lo(h, q, n) : conv;
    }
    double fhz = 0.0;
    if (k + 1 < nz) {
      fhz = phz * i4_hi(hhat(ze, zT, k, true), k, nz);
      conv += fhz;
    }
    if (k > 0) conv -= flo;
    flo = fhz;
    double bg = 0.0;
    if (k + 1 < nz) bg += kdz * (tb - tb_up);
    if (k > 0) bg += kdz * (tb - tb_dn);
    const double rest = ks + phi_cell(G, ph, k);
    const double bP = ENTH ? G.V / ph.dt * e0c - conv + bg : G.V / ph.dt * (r * e0c - rs * rest) - conv + bg;
    const double cP = rs * (ENTH ? ph.cp : ph.cv) * G.V / ph.dt;
    const double xc = zT.c;
    double ax = cP * xc, diag = cP;
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int n = G.n[d], q = coord(c, d);
      const double w = kcoef * (G.S[d] / G.h[d]);
      ax = q + 1 < n ? ax + w * (xc - lT[d].p1) : ax;
      diag = q + 1 < n ? diag + w : diag;
      ax = q > 0 ? ax + w * (xc - lT[d].m1) : ax;
      diag = q > 0 ? diag + w : diag;
    }
    if (k + 1 < nz) {
      ax += wz * (xc - zT.p1);
      diag += wz;
    }
    if (k > 0) {
      ax += wz * (xc - zT.m1);
      diag += wz;
    }
    if (c.act) {
      const int P = qo + pl * k;
      // (1/diag is not stored: the iteration kernel forms it from c)
      const double di = 1.0 / diag, rr = bP - ax;
      sy.b[P] = bP;
      sy.c[P] = cP;
      if (sy.x) sy.x[P] = xc;  // (null: the solve runs in place on T_prev)
      sy.r[P] = rr;
      red[0] += rr * (rr * di);
      red[1] += rr * rr;
      red[2] += bP * bP;
    }
    sl = sl == 2 ? 0 : sl + 1;
  }
  __shared__ double sh[3][TY];
  Reducer<0u, 3, 64 * TY>::block(red, sh);
  if (threadIdx.x == 0) {
    sy.u_part[blockIdx.x] = red[0];
    sy.u_part[gridDim.x + blockIdx.x] = red[1];
    sy.b_part[blockIdx.x] = red[2];
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
    // loads of the plane
    const int Pn = nb(k + 3 < nz, P + 3 * pl, P);
    const double r = rho[P], phz = phi.p[Z][P];
    double fhi[NDIM - 1], flod[NDIM - 1];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int q = coord(c, d);
      fhi[d] = phi.p[d][P];
      flod[d] = phi.p[d][nb(q > 0, P - G.st[d], P)];
    }
    Line s[NDIM][NDIM - 1];
    double zn[NDIM], un[NDIM];
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      const double* uc = u_prev.p[cc];
#pragma unroll
      for (int d = 0; d < Z; ++d)
        s[cc][d] = line_at([&](int Q) { return uc[Q]; }, P, G.st[d], coord(c, d), G.n[d]);
      zn[cc] = uc[Pn];
      un[cc] = u.p[cc][P];
    }
    // H
    double h[NDIM];
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      double conv = 0.0, visc = 0.0;
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int n = G.n[d], q = coord(c, d);
        conv = q + 1 < n ? conv + fhi[d] * i4_hi(s[cc][d], q, n) : conv;
        conv = q > 0 ? conv - flod[d] * i4_lo(s[cc][d], q, n) : conv;
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
        visc_add(visc, s[cc][d], coord(c, d), G.n[d], ph.mu * G.S[d] / G.h[d], cc == d);
      visc_add(visc, z[cc], k, nz, kvz, cc == Z);
      h[cc] = r * un[cc] * ph.inv_dt - conv * G.inv_V + visc * G.inv_V;
    }
#pragma unroll
    for (int cc = 0; cc < NDIM; ++cc) {
      H.p[cc][P] = h[cc];
      z[cc] = shift(z[cc], k + 3 < nz ? zn[cc] : 0.0);
    }
  }
}

// k_H on a 3D mesh.  The x/y neighbourhoods of u_prev (two cells, for I4)
// are staged in a ring of three LDS planes that is filled three planes ahead
// of the plane computed, and the staged own value of plane k + 2 is the one
// the register line along z takes in: each value of u_prev comes from HBM once
// a chunk.  (A separate load of the column three planes up, as the explicit
// kernels with a two-plane ring make, came back from HBM: between it and the
// plane's staging load, more data passes through an XCD's L2 than it holds.)
// Same formulas and order as k_H.
template <int TY>
__global__ __launch_bounds__(64 * TY) void k_H3(Geo G, Phys ph, int kc,
                                               const double* __restrict__ rho, Vec<3> u,
                                               Vec<3> u_prev, Vec<3> phi, Vec<3> H) {
  using St = Stage3<2, TY>;
  constexpr int Z = 2, HP = St::HP, HX = St::HX, NU = St::NU;
  __shared__ double su[3][3][HP];  // plane k in slot (k - k0) % 3
  const Col c = col_of3<TY>(G, kc);
  const St st = stage3<2, TY>(G, c);
  const int nz = G.n[Z], pl = c.pl, qo = st.qo;
  const int Pxl = nb(clampi(c.i, G.nx) > 0, qo - 1, qo);
  const int Pyl = nb(clampi(c.j, G.ny) > 0, qo - G.nx, qo);
  // highest plane the chunk's z lines read; planes above the chunk are
  // loaded for the own column only (the halo slots load it again)
  const int ktop = min(c.k1 + 1, nz - 1);
  double fu[3][NU];                       // staged plane in flight
  double fr, fz, fh[2], fl[2], fun[3];    // own cell's values of the next plane
  auto fetch = [&](int kk, double (&dst)[3][NU]) {
    const int kq = min(kk, ktop), o = pl * kq;
    const bool halo = kq < c.k1;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int Q = (halo ? st.q[m] : qo) + o;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) dst[cc][m] = u_prev.p[cc][Q];
    }
  };
  auto own = [&](int kk) {
    const int o = pl * min(kk, c.k1 - 1), P = qo + o;
    fr = rho[P];
    fz = phi.p[Z][P];
    fh[0] = phi.p[0][P];
    fh[1] = phi.p[1][P];
    fl[0] = phi.p[0][Pxl + o];
    fl[1] = phi.p[1][Pyl + o];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) fun[cc] = u.p[cc][P];
  };
  auto stage = [&](int sl, const double (&src)[3][NU]) {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int m = 0; m < NU; ++m)
        su[sl][cc][st.h[m]] = src[cc][m];
  };
  // the z lines hold planes k0-3 .. k0+1 before the loop (k0-3 is never
  // read); the chunk's first two planes are loaded together
  Line z[3];
  double flo[3];
  {
    const int P = qo + pl * c.k0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double* uc = u_prev.p[cc];
      z[cc].m2 = 0.0;
      z[cc].m1 = uc[nb(c.k0 >= 2, P - 2 * pl, P)];
      z[cc].c = uc[nb(c.k0 >= 1, P - pl, P)];
    }
    const double phz_lo = c.k0 > 0 ? phi.p[Z][P - pl] : 0.0;
    double f1[3][NU];
    fetch(c.k0, fu);
    fetch(c.k0 + 1, f1);
    stage(0, fu);
    stage(1, f1);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      z[cc].p1 = fu[cc][0];
      z[cc].p2 = f1[cc][0];
      const Line L{z[cc].m1, z[cc].c, z[cc].p1, z[cc].p2, 0.0};  // centred on k0
      flo[cc] = c.k0 > 0 ? phz_lo * i4_lo(L, c.k0, nz) : 0.0;
    }
  }
  own(c.k0);
  fetch(c.k0 + 2, fu);
  const double kvz = ph.mu * G.S[Z] / G.h[Z];
  int sl = 0;  // slot of plane k
  for (int k = c.k0; k < c.k1; ++k) {
    // every thread is done with plane k-1, whose slot takes plane k+2
    lds_barrier();
    stage(sl == 0 ? 2 : sl - 1, fu);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) z[cc] = shift(z[cc], fu[cc][0]);
    const double r = fr, phz = fz;
    const double fhi[2] = {fh[0], fh[1]}, flod[2] = {fl[0], fl[1]};
    double un[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) un[cc] = fun[cc];
    own(k + 1);
    fetch(k + 3, fu);
    double h[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const Line s[2] = {line_lds(su[sl][cc], st.ho, 1), line_lds(su[sl][cc], st.ho, HX)};
      double conv = 0.0, visc = 0.0;
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int n = G.n[d], q = coord(c, d);
        conv = q + 1 < n ? conv + fhi[d] * i4_hi(s[d], q, n) : conv;
        conv = q > 0 ? conv - flod[d] * i4_lo(s[d], q, n) : conv;
      }
      double fhz = 0.0;
      if (k + 1 < nz) {
        fhz = phz * i4_hi(z[cc], k, nz);
        conv += fhz;
      }
      if (k > 0) conv -= flo[cc];
      flo[cc] = fhz;
#pragma unroll
      for (int d = 0; d < Z; ++d)
        visc_add(visc, s[d], coord(c, d), G.n[d], ph.mu * G.S[d] / G.h[d], cc == d);
      visc_add(visc, z[cc], k, nz, kvz, cc == Z);
      h[cc] = r * un[cc] * ph.inv_dt - conv * G.inv_V + visc * G.inv_V;
    }
    if (c.act) {
      const int P = qo + pl * k;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) H.p[cc][P] = h[cc];
    }
    sl = sl == 2 ? 0 : sl + 1;
  }
}

// b = (V/dt)(rho^n + psi rho23 Phi) - sum_out phitilde; 1/diag of the operator
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_rhs(Geo G, Phys ph, int kc,
                                                const double* __restrict__ rho,
                                                const double* __restrict__ rho23,
                                                const double* __restrict__ psi,
                                                const double* __restrict__ cc,
                                                const double* __restrict__ D, Vec<NDIM> H,
                                                double* __restrict__ b, double* __restrict__ dinv,
                                                float* __restrict__ c32, float* __restrict__ D32,
                                                float* __restrict__ dinv32) {
  constexpr int Z = NDIM - 1;
  const Col c = col_of<NDIM>(G, kc);
  if (!c.act) return;
  const int nz = G.n[Z], pl = c.pl;
  const double kz_ = G.S[Z] / G.h[Z];
  int P = c.base + pl * c.k0;
  double flux_lo = 0.0, diag_lo = 0.0;
  if (c.k0 > 0) {
    const int Q = P - pl;
    flux_lo = phit_val(D[Q], D[P], H.p[Z][Q], H.p[Z][P], rho23[Q], rho23[P], G.S[Z],
                       phi_face<NDIM>(G, ph, Z, c.k0 - 1, c.k0 - 1), G.inv_h[Z]);
    diag_lo = 0.5 * (D[Q] + D[P]) * kz_;
  }
  for (int k = c.k0; k < c.k1; ++k, P += pl) {
    // loads of the plane
    const bool up = k + 1 < nz;
    const int Pu = nb(up, P + pl, P);
    const double Dc = D[P], r23 = rho23[P], cP = cc[P], rP = rho[P], psP = psi[P];
    const double D_up = D[Pu], Hz = H.p[Z][P], Hz_up = H.p[Z][Pu], r23_up = rho23[Pu];
    double D_hi[NDIM - 1], D_lo[NDIM - 1], Hc[NDIM - 1], H_hi[NDIM - 1], H_lo[NDIM - 1],
        r_hi[NDIM - 1], r_lo[NDIM - 1];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int st = G.st[d], q = coord(c, d);
      const int Ph = nb(q + 1 < G.n[d], P + st, P), Pl = nb(q > 0, P - st, P);
      D_hi[d] = D[Ph];
      D_lo[d] = D[Pl];
      Hc[d] = H.p[d][P];
      H_hi[d] = H.p[d][Ph];
      H_lo[d] = H.p[d][Pl];
      r_hi[d] = rho23[Ph];
      r_lo[d] = rho23[Pl];
    }
    // right-hand side and diagonal
    double sum = 0.0;
    double diag = cP;
    const double phc = phi_cell(G, ph, k);
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int q = coord(c, d);
      const double kd = G.S[d] / G.h[d];
      if (q + 1 < G.n[d]) {
        sum += phit_val(Dc, D_hi[d], Hc[d], H_hi[d], r23, r_hi[d], G.S[d], phc, G.inv_h[d]);
        diag += 0.5 * (Dc + D_hi[d]) * kd;
      }
      if (q > 0) {
        sum -= phit_val(D_lo[d], Dc, H_lo[d], Hc[d], r_lo[d], r23, G.S[d], phc, G.inv_h[d]);
        diag += 0.5 * (D_lo[d] + Dc) * kd;
      }
    }
    double flux_hi = 0.0, diag_hi = 0.0;
    if (up) {
      flux_hi = phit_val(Dc, D_up, Hz, Hz_up, r23, r23_up, G.S[Z], phi_face<NDIM>(G, ph, Z, k, k),
                         G.inv_h[Z]);
      diag_hi = 0.5 * (Dc + D_up) * kz_;
      sum += flux_hi;
      diag += diag_hi;
    }
    if (k > 0) {
      sum -= flux_lo;
      diag += diag_lo;
    }
    flux_lo = flux_hi;
    diag_lo = diag_hi;
    b[P] = G.V / ph.dt * (rP + psP * r23 * phc) - sum;
    const double di = 1.0 / diag;
    if (dinv) dinv[P] = di;  // (null: the coefficients of an earlier corrector stand)
    if (c32) {  // FP32 copies of the operator for the refined forms
      c32[P] = (float)cP;
      D32[P] = (float)Dc;
      dinv32[P] = (float)di;
    }
  }
}

// k_rhs on a 3D mesh with the x/y neighbours of D, rho23, H_x and H_y (and
// x) staged in a ring of three LDS planes filled three planes ahead, and the
// next plane's own-cell loads in flight while a plane is computed.  Same
// formulas and order as k_rhs.  (With two planes and separate loads of the
// column one plane up, which the next plane's staging loaded again, the
// counters showed 1.11x the algorithmic bytes.)
template <int TY, bool RES>
__global__ __launch_bounds__(64 * TY) void k_rhs3(Geo G, Phys ph, int kc,
                                                 const double* __restrict__ rho,
                                                 const double* __restrict__ rho23,
                                                 const double* __restrict__ psi,
                                                 const double* __restrict__ cc,
                                                 const double* __restrict__ D, Vec<3> H,
                                                 double* __restrict__ b, double* __restrict__ dinv,
                                                 float* __restrict__ c32, float* __restrict__ D32,
                                                 float* __restrict__ dinv32, RhsResidual res) {
  using St = Stage3<1, TY>;
  constexpr int Z = 2, HP = St::HP, HX = St::HX, NU = St::NU;
  constexpr int NF = RES ? 5 : 4;
  // D, rho23, H_x, H_y (, x of the residual); plane k in slot (k - k0) % 3,
  // filled three planes ahead (as in k_H3): plane k+1's own values are the
  // ones the face above needs
  __shared__ double ss[3][NF][HP];
  const Col c = col_of3<TY>(G, kc);
  const St st = stage3<1, TY>(G, c);
  const int nz = G.n[Z], pl = c.pl, qo = st.qo, ho = st.ho;
  const double kz_ = G.S[Z] / G.h[Z];
  const double* __restrict__ xv = res.x;
  // highest plane read: the plane above the chunk, for its own column only
  // (the halo slots load it again)
  const int ktop = min(c.k1, nz - 1);
  double fs[NF][NU];                  // staged plane in flight
  double fc, fr, fps, fHzn;           // own c, rho, psi of the next plane, H_z one above it
  auto fetch = [&](int kk, double (&dst)[NF][NU]) {
    const int kq = min(kk, ktop), o = pl * kq;
    const bool halo = kq < c.k1;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int Q = (halo ? st.q[m] : qo) + o;
      dst[0][m] = D[Q];
      dst[1][m] = rho23[Q];
      dst[2][m] = H.p[0][Q];
      dst[3][m] = H.p[1][Q];
      if (RES) dst[NF - 1][m] = xv[Q];
    }
  };
  auto own = [&](int kk) {
    const int P = qo + pl * min(kk, c.k1 - 1);
    fc = cc[P];
    fr = rho[P];
    fps = psi[P];
    fHzn = H.p[Z][qo + pl * min(kk + 1, nz - 1)];
  };
  auto stage = [&](int sl, const double (&src)[NF][NU]) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int m = 0; m < NU; ++m) ss[sl][f][st.h[m]] = src[f][m];
  };
  double flux_lo = 0.0, diag_lo = 0.0;
  double xm = 0.0, dm = 0.0;  // residual: x and D one plane down
  double hz = H.p[Z][qo + pl * c.k0];  // H_z of the plane computed
  if (c.k0 > 0) {
    const int P = qo + pl * c.k0, Q = P - pl;
    flux_lo = phit_val(D[Q], D[P], H.p[Z][Q], H.p[Z][P], rho23[Q], rho23[P], G.S[Z],
                       phi_face<3>(G, ph, Z, c.k0 - 1, c.k0 - 1), G.inv_h[Z]);
    diag_lo = 0.5 * (D[Q] + D[P]) * kz_;
    if (RES) {
      xm = xv[Q];
      dm = D[Q];
    }
  }
  double ro[2] = {0.0, 0.0}, ri[2] = {0.0, 0.0};
  {
    double f1[NF][NU];  // the chunk's first two planes, loaded together
    fetch(c.k0, fs);
    fetch(c.k0 + 1, f1);
    stage(0, fs);
    stage(1, f1);
  }
  own(c.k0);
  fetch(c.k0 + 2, fs);
  int sl = 0;  // slot of plane k
  for (int k = c.k0; k < c.k1; ++k) {
    // every thread is done with plane k-1, whose slot takes plane k+2
    lds_barrier();
    stage(sl == 0 ? 2 : sl - 1, fs);
    const double cP = fc, rP = fr, psP = fps, Hz = hz, Hz_up = fHzn;
    hz = fHzn;
    own(k + 1);
    fetch(k + 3, fs);
    const int su = sl == 2 ? 0 : sl + 1;  // slot of plane k+1
    const double D_up = ss[su][0][ho], r23_up = ss[su][1][ho];
    const double x_up = RES ? ss[su][NF - 1][ho] : 0.0;
    const bool up = k + 1 < nz;
    const double* SD = ss[sl][0];
    const double* Sr = ss[sl][1];
    const double Dc = SD[ho], r23 = Sr[ho];
    double sum = 0.0;
    double diag = cP;
    const double phc = phi_cell(G, ph, k);
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int q = coord(c, d), sd = d == 0 ? 1 : HX;
      const double* SH = ss[sl][2 + d];
      const double kd = G.S[d] / G.h[d];
      const double Hc = SH[ho];
      if (q + 1 < G.n[d]) {
        sum += phit_val(Dc, SD[ho + sd], Hc, SH[ho + sd], r23, Sr[ho + sd], G.S[d], phc, G.inv_h[d]);
        diag += 0.5 * (Dc + SD[ho + sd]) * kd;
      }
      if (q > 0) {
        sum -= phit_val(SD[ho - sd], Dc, SH[ho - sd], Hc, Sr[ho - sd], r23, G.S[d], phc, G.inv_h[d]);
        diag += 0.5 * (SD[ho - sd] + Dc) * kd;
      }
    }
    double flux_hi = 0.0, diag_hi = 0.0;
    if (up) {
      flux_hi = phit_val(Dc, D_up, Hz, Hz_up, r23, r23_up, G.S[Z], phi_face<3>(G, ph, Z, k, k),
                         G.inv_h[Z]);
      diag_hi = 0.5 * (Dc + D_up) * kz_;
      sum += flux_hi;
      diag += diag_hi;
    }
    if (k > 0) {
      sum -= flux_lo;
      diag += diag_lo;
    }
    flux_lo = flux_hi;
    diag_lo = diag_hi;
    // residual of the solve's initial guess: the operator as the refinement
    // residual kernel applies it, same order
    double ax = 0.0;
    if (RES) {
      const double* Sx = ss[sl][NF - 1];
      const double xc = Sx[ho];
      const double xp = up ? x_up : 0.0, dp = up ? D_up : 0.0;
      ax = cP * xc;
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int q = coord(c, d), sd = d == 0 ? 1 : HX;
        const double kd = G.S[d] / G.h[d];
        ax = q + 1 < G.n[d] ? ax + 0.5 * (Dc + SD[ho + sd]) * kd * (xc - Sx[ho + sd]) : ax;
        ax = q > 0 ? ax + 0.5 * (SD[ho - sd] + Dc) * kd * (xc - Sx[ho - sd]) : ax;
      }
      if (up) ax += 0.5 * (Dc + dp) * kz_ * (xc - xp);
      if (k > 0) ax += 0.5 * (dm + Dc) * kz_ * (xc - xm);
      xm = xc;
      dm = Dc;
    }
    if (c.act) {
      const int P = qo + pl * k;
      const double bp = G.V / ph.dt * (rP + psP * r23 * phc) - sum;
      b[P] = bp;
      const double di = 1.0 / diag;
      if (dinv) dinv[P] = di;  // (null: the coefficients of an earlier corrector stand)
      if (c32) {  // FP32 copies of the operator for the refined forms
        c32[P] = (float)cP;
        D32[P] = (float)Dc;
        dinv32[P] = (float)di;
      }
      if (RES) {
        const double r = bp - ax;
        const float rf = (float)r;
        res.r32[P] = rf;
        if (res.zero_inner) res.x32[P] = 0.0f;
        ro[0] += r * r;
        ro[1] += bp * bp;
        ri[0] += (double)rf * (double)(rf * (float)di);
        ri[1] += (double)rf * (double)rf;
      }
    }
    sl = su;
  }
  if (RES) {
    double v[4] = {ro[0], ro[1], ri[0], ri[1]};
    __shared__ double sh[4][TY];
    Reducer<0u, 4, 64 * TY>::block(v, sh);
    if (threadIdx.x == 0) {
      res.o_part[blockIdx.x] = v[0];
      res.o_part[gridDim.x + blockIdx.x] = v[1];
      res.i_part[blockIdx.x] = v[2];
      res.i_part[gridDim.x + blockIdx.x] = v[3];
    }
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
    Vec<NDIM> phi_out, double* partials) {
  constexpr int Z = NDIM - 1;
  double red[3] = {0.0, 0.0, 0.0};
  const Col c = col_of<NDIM>(G, kc);
  if (c.act) {
    const int nz = G.n[Z], pl = c.pl;
    const double kz_ = G.S[Z] / G.h[Z];
    int P = c.base + pl * c.k0;
    double Flo = 0.0, flux_lo = 0.0;
    if (c.k0 > 0) {
      const int Q = P - pl;
      const double phf = phi_face<NDIM>(G, ph, Z, c.k0 - 1, c.k0 - 1);
      Flo = force_val(pp[Q], pp[P], rho23[Q], rho23[P], phf, G.inv_h[Z]);
      if (last) {
        const double w = 0.5 * (D[Q] + D[P]) * kz_;
        flux_lo = phit_val(D[Q], D[P], H.p[Z][Q], H.p[Z][P], rho23[Q], rho23[P], G.S[Z], phf,
                           G.inv_h[Z]) -
                  w * (pp[P] - pp[Q]);
      }
    }
    for (int k = c.k0; k < c.k1; ++k, P += pl) {
      // loads of the plane
      const bool up = k + 1 < nz;
      const int Pu = nb(up, P + pl, P);
      const double pc = pp[P], r23 = rho23[P], rs = rho_star[P], p_up = pp[Pu], r_up = rho23[Pu];
      double Hc[NDIM], p_hi[NDIM - 1], p_lo[NDIM - 1], r_hi[NDIM - 1], r_lo[NDIM - 1];
#pragma unroll
      for (int d = 0; d < NDIM; ++d) Hc[d] = H.p[d][P];
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int st = G.st[d], q = coord(c, d);
        const int Ph = nb(q + 1 < G.n[d], P + st, P), Pl = nb(q > 0, P - st, P);
        p_hi[d] = pp[Ph];
        p_lo[d] = pp[Pl];
        r_hi[d] = rho23[Ph];
        r_lo[d] = rho23[Pl];
      }
      // velocity correction
      const double inv_A = ph.dt / rs;
      const double phc = phi_cell(G, ph, k);
      const double Fhi = up ? force_val(pc, p_up, r23, r_up, phi_face<NDIM>(G, ph, Z, k, k), G.inv_h[Z]) : 0.0;
      bool finite = true;
      double uo[NDIM];
#pragma unroll
      for (int cmp = 0; cmp < NDIM; ++cmp) {
        double RF;
        if (cmp == Z) {
          RF = 0.5 * (Flo + Fhi);
        } else {
          const int n = G.n[cmp], q = coord(c, cmp);
          const double hi = q + 1 < n ? force_val(pc, p_hi[cmp], r23, r_hi[cmp], phc, G.inv_h[cmp]) : 0.0;
          const double lo = q > 0 ? force_val(p_lo[cmp], pc, r_lo[cmp], r23, phc, G.inv_h[cmp]) : 0.0;
          RF = 0.5 * (lo + hi);
        }
        uo[cmp] = (Hc[cmp] - RF) * inv_A;
        finite = finite && isfinite(uo[cmp]);
      }
#pragma unroll
      for (int cmp = 0; cmp < NDIM; ++cmp) u_out.p[cmp][P] = uo[cmp];
      Flo = Fhi;
      if (last) {
        // loads for the new density
        const double Dc = D[P], D_up = D[Pu], Hz_up = H.p[Z][Pu], r_old = rho_old[P], psP = psi[P];
        double D_hi[NDIM - 1], D_lo[NDIM - 1], H_hi[NDIM - 1], H_lo[NDIM - 1];
#pragma unroll
        for (int d = 0; d < Z; ++d) {
          const int st = G.st[d], q = coord(c, d);
          const int Ph = nb(q + 1 < G.n[d], P + st, P), Pl = nb(q > 0, P - st, P);
          D_hi[d] = D[Ph];
          D_lo[d] = D[Pl];
          H_hi[d] = H.p[d][Ph];
          H_lo[d] = H.p[d][Pl];
        }
        double sum = 0.0;
#pragma unroll
        for (int d = 0; d < Z; ++d) {
          const int q = coord(c, d);
          const double kd = G.S[d] / G.h[d];
          double fx = 0.0;
          if (q + 1 < G.n[d]) {
            const double w = 0.5 * (Dc + D_hi[d]) * kd;
            fx = phit_val(Dc, D_hi[d], Hc[d], H_hi[d], r23, r_hi[d], G.S[d], phc, G.inv_h[d]) -
                 w * (p_hi[d] - pc);
            sum += fx;
          }
          phi_out.p[d][P] = fx;  // the next state's flux (0 on the wall)
          if (q > 0) {
            const double w = 0.5 * (D_lo[d] + Dc) * kd;
            sum -= phit_val(D_lo[d], Dc, H_lo[d], Hc[d], r_lo[d], r23, G.S[d], phc, G.inv_h[d]) -
                   w * (pc - p_lo[d]);
          }
        }
        double flux_hi = 0.0;
        if (up) {
          const double w = 0.5 * (Dc + D_up) * kz_;
          flux_hi = phit_val(Dc, D_up, Hc[Z], Hz_up, r23, r_up, G.S[Z], phi_face<NDIM>(G, ph, Z, k, k),
                             G.inv_h[Z]) -
                    w * (p_up - pc);
          sum += flux_hi;
        }
        if (k > 0) sum -= flux_lo;
        flux_lo = flux_hi;
        phi_out.p[Z][P] = flux_hi;
        const double rn = r_old - ph.dt / G.V * sum;
        const double pn = pc - r23 * phc;
        rho_new[P] = rn;
        p_new[P] = pn;
        red[0] += rn * G.V;
        red[1] = fmax(red[1], fabs(rn - psP * pn));
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

// k_correct on a 3D mesh with the x/y neighbours of p' and rho23 (and, on the
// last corrector, D, H_x and H_y) staged in LDS and the next plane's loads in
// flight while a plane is computed.  Same formulas and order as k_correct.
template <bool LAST, int TY>
__global__ __launch_bounds__(64 * TY) void k_correct3(
    Geo G, Phys ph, int kc, const double* __restrict__ pp, const double* __restrict__ rho23,
    const double* __restrict__ psi, Vec<3> H, const double* __restrict__ D,
    const double* __restrict__ rho_star, Vec<3> u_out, const double* __restrict__ rho_old,
    double* __restrict__ rho_new, double* __restrict__ p_new, Vec<3> phi_out, double* partials) {
  using St = Stage3<1, TY>;
  constexpr int Z = 2, HP = St::HP, HX = St::HX, NU = St::NU;
  constexpr int NF = LAST ? 5 : 2;
  __shared__ double ss[2][NF][HP];  // p', rho23 (, D, H_x, H_y)
  const Col c = col_of3<TY>(G, kc);
  const St st = stage3<1, TY>(G, c);
  const int nz = G.n[Z], pl = c.pl, qo = st.qo, ho = st.ho;
  const double kz_ = G.S[Z] / G.h[Z];
  // raw values of the plane in flight
  double fs[NF][NU], frs, fpu, fru, fH[3], fDu = 0.0, fHzu = 0.0, fro = 0.0, fps = 0.0;
  auto fetch = [&](int kk) {
    const int o = pl * kk, P = qo + o;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int Q = st.q[m] + o;
      fs[0][m] = pp[Q];
      fs[1][m] = rho23[Q];
      if (LAST) {
        fs[2 % NF][m] = D[Q];
        fs[3 % NF][m] = H.p[0][Q];
        fs[4 % NF][m] = H.p[1][Q];
      }
    }
    const int Pu = nb(kk + 1 < nz, P + pl, P);
    frs = rho_star[P];
    fpu = pp[Pu];
    fru = rho23[Pu];
#pragma unroll
    for (int d = 0; d < 3; ++d) fH[d] = H.p[d][P];
    if (LAST) {
      fDu = D[Pu];
      fHzu = H.p[Z][Pu];
      fro = rho_old[P];
      fps = psi[P];
    }
  };
  double red[3] = {0.0, 0.0, 0.0};
  double Flo = 0.0, flux_lo = 0.0;
  if (c.k0 > 0) {
    const int P = qo + pl * c.k0, Q = P - pl;
    const double phf = phi_face<3>(G, ph, Z, c.k0 - 1, c.k0 - 1);
    Flo = force_val(pp[Q], pp[P], rho23[Q], rho23[P], phf, G.inv_h[Z]);
    if (LAST) {
      const double w = 0.5 * (D[Q] + D[P]) * kz_;
      flux_lo = phit_val(D[Q], D[P], H.p[Z][Q], H.p[Z][P], rho23[Q], rho23[P], G.S[Z], phf,
                         G.inv_h[Z]) -
                w * (pp[P] - pp[Q]);
    }
  }
  fetch(c.k0);
  for (int k = c.k0; k < c.k1; ++k) {
    const int sl = k & 1;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int m = 0; m < NU; ++m)
        ss[sl][f][st.h[m]] = fs[f][m];
    const double rs = frs, p_up = fpu, r_up = fru, D_up = fDu, Hz_up = fHzu, r_old = fro, psP = fps;
    const double Hc[3] = {fH[0], fH[1], fH[2]};
    fetch(k + 1 < c.k1 ? k + 1 : k);
    lds_barrier();
    const bool up = k + 1 < nz;
    const double* Sp = ss[sl][0];
    const double* Sr = ss[sl][1];
    const double pc = Sp[ho], r23 = Sr[ho];
    // velocity correction
    const double inv_A = ph.dt / rs;
    const double phc = phi_cell(G, ph, k);
    const double Fhi = up ? force_val(pc, p_up, r23, r_up, phi_face<3>(G, ph, Z, k, k), G.inv_h[Z]) : 0.0;
    bool finite = true;
    double uo[3];
#pragma unroll
    for (int cmp = 0; cmp < 3; ++cmp) {
      double RF;
      if (cmp == Z) {
        RF = 0.5 * (Flo + Fhi);
      } else {
        const int n = G.n[cmp], q = coord(c, cmp), sd = cmp == 0 ? 1 : HX;
        const double hi = q + 1 < n ? force_val(pc, Sp[ho + sd], r23, Sr[ho + sd], phc, G.inv_h[cmp]) : 0.0;
        const double lo = q > 0 ? force_val(Sp[ho - sd], pc, Sr[ho - sd], r23, phc, G.inv_h[cmp]) : 0.0;
        RF = 0.5 * (lo + hi);
      }
      uo[cmp] = (Hc[cmp] - RF) * inv_A;
      finite = finite && isfinite(uo[cmp]);
    }
    Flo = Fhi;
    const int P = qo + pl * k;
    if (c.act) {
#pragma unroll
      for (int cmp = 0; cmp < 3; ++cmp) u_out.p[cmp][P] = uo[cmp];
    }
    if (LAST) {
      const double* SD = ss[sl][2 % NF];
      const double Dc = SD[ho];
      double sum = 0.0, fxy[2] = {0.0, 0.0};
#pragma unroll
      for (int d = 0; d < Z; ++d) {
        const int q = coord(c, d), sd = d == 0 ? 1 : HX;
        const double* SH = ss[sl][(3 + d) % NF];
        const double kd = G.S[d] / G.h[d];
        if (q + 1 < G.n[d]) {
          const double w = 0.5 * (Dc + SD[ho + sd]) * kd;
          fxy[d] = phit_val(Dc, SD[ho + sd], Hc[d], SH[ho + sd], r23, Sr[ho + sd], G.S[d], phc, G.inv_h[d]) -
                   w * (Sp[ho + sd] - pc);
          sum += fxy[d];
        }
        if (q > 0) {
          const double w = 0.5 * (SD[ho - sd] + Dc) * kd;
          sum -= phit_val(SD[ho - sd], Dc, SH[ho - sd], Hc[d], Sr[ho - sd], r23, G.S[d], phc, G.inv_h[d]) -
                 w * (pc - Sp[ho - sd]);
        }
      }
      double flux_hi = 0.0;
      if (up) {
        const double w = 0.5 * (Dc + D_up) * kz_;
        flux_hi = phit_val(Dc, D_up, Hc[Z], Hz_up, r23, r_up, G.S[Z], phi_face<3>(G, ph, Z, k, k),
                           G.inv_h[Z]) -
                  w * (p_up - pc);
        sum += flux_hi;
      }
      if (k > 0) sum -= flux_lo;
      flux_lo = flux_hi;
      const double rn = r_old - ph.dt / G.V * sum;
      const double pn = pc - r23 * phc;
      if (c.act) {
        rho_new[P] = rn;
        p_new[P] = pn;
        phi_out.p[0][P] = fxy[0];  // the next state's flux (0 on the walls)
        phi_out.p[1][P] = fxy[1];
        phi_out.p[Z][P] = flux_hi;
        red[0] += rn * G.V;
        red[1] = fmax(red[1], fabs(rn - psP * pn));
      }
      finite = finite && isfinite(rn) && isfinite(pn);
    }
    if (c.act) red[2] += finite ? 0.0 : 1.0;
  }
  if (!LAST) return;
  __shared__ double sh[3][TY];
  Reducer<0x2u, 3, 64 * TY>::block(red, sh);
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

// ---- diagnostics ----------------------------------------------------------------

// Extrema of the velocity components and of the potential temperature
// perturbation theta' = T/pi - theta0, pi = (p/p0)^{R/c_p} (Sec. 2,
// eqs. theta, theta_split), as maxima of (-min, max) pairs: per workgroup
// into part (8 values a workgroup, component-major), then one workgroup.
__global__ __launch_bounds__(kBlock) void k_extrema(Geo G, Phys ph, const double* __restrict__ ux,
                                                    const double* __restrict__ uy,
                                                    const double* __restrict__ uz,
                                                    const double* __restrict__ T,
                                                    const double* __restrict__ p, double* part) {
  __shared__ double sh[8][kBlock / 64];
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = -INFINITY;
  const double kappa = ph.R / ph.cp;
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < G.nc; P += gridDim.x * blockDim.x) {
    const double u = ux[P], v = uy ? uy[P] : 0.0, w = uz[P];
    const double th = T[P] / pow(p[P] / ph.p0, kappa) - ph.theta0;
    a[0] = fmax(a[0], -u);
    a[1] = fmax(a[1], u);
    a[2] = fmax(a[2], -v);
    a[3] = fmax(a[3], v);
    a[4] = fmax(a[4], -w);
    a[5] = fmax(a[5], w);
    a[6] = fmax(a[6], -th);
    a[7] = fmax(a[7], th);
  }
  Reducer<0xFFu, 8>::block(a, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) part[k * gridDim.x + blockIdx.x] = a[k];
}

__global__ __launch_bounds__(kBlock) void k_extrema_final(const double* part, int n, double* out) {
  __shared__ double sh[8][kBlock / 64];
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = -INFINITY;
  for (int b = threadIdx.x; b < n; b += kBlock)
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fmax(a[k], part[k * n + b]);
  Reducer<0xFFu, 8>::block(a, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = (k & 1) ? a[k] : -a[k];
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

ZPlan zplan3(const Geo& G, int ty, int kc0) {
  const int cols = ((G.nx + 63) / 64) * ((G.ny + ty - 1) / ty), nz = G.nz;
  int kc = kc0 < nz ? kc0 : nz;
  int nk = (nz + kc - 1) / kc;
  const int maxk = kMaxZBlocks / cols > 1 ? kMaxZBlocks / cols : 1;
  if (nk > maxk) {
    kc = (nz + maxk - 1) / maxk;
    nk = (nz + kc - 1) / kc;
  }
  return ZPlan{kc, cols * nk};
}

namespace {

// rows of the column tiles of the LDS-staged 3D step kernels (taller tiles
// re-read fewer halo rows) and planes of a chunk, measured per kernel on the
// 256 x 256 x 128 mesh.  The kernels with three-plane rings hold one
// 512-thread workgroup a CU (registers or LDS), and 64 x 8 tiles in 64-plane
// chunks give 256 workgroups, one for each CU, which all run at once: k_H3
// took 185 us so against 205 us in 64 x 4 tiles of 16 planes (2048
// workgroups, three a CU, the last of three rounds a third empty) and 207 us
// in 43-plane chunks (one round).
constexpr int kTyStep1 = 8, kTyEnergy = 8, kTyH = 8, kTyRhs = 8, kTyCorr = 8;
constexpr int kKcStep1 = 64, kKcEnergy = 64, kKcH = 64, kKcRhs = 32, kKcCorr = 32, kKcCorrLast = 64;

}  // namespace

#define V2(a) vec<2>(a)
#define V3(a) vec<3>(a)

void launch_face_mass_flux(hipStream_t s, const Geo& G, const double* rho, double* const* u,
                           double* const* phi) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_face_mass_flux<2>, grid, block, 0, s, G, rho, V2(u), V2(phi));
  else
    hipLaunchKernelGGL(k_face_mass_flux<3>, grid, block, 0, s, G, rho, V3(u), V3(phi));
}

void launch_clear_wall_faces(hipStream_t s, const Geo& G, double* const* phi) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_clear_wall_faces<2>, grid, block, 0, s, G, V2(phi));
  else
    hipLaunchKernelGGL(k_clear_wall_faces<3>, grid, block, 0, s, G, V3(phi));
}

void launch_step1(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                  double* const* u, const double* T, const double* pp, double* const* phi,
                  double* rho_star, double* e0, double* const* u_star, double* pp_copy,
                  double* const* b_out, double* Ks) {
  double* const nob[3] = {nullptr, nullptr, nullptr};
  double* const* bo = b_out ? b_out : nob;
  if (G.ndim == 2) {
    const ZPlan zp = zplan(G);
    hipLaunchKernelGGL(k_density_predictor<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V2(u), T, V2(phi), rho_star, e0);
    hipLaunchKernelGGL(k_mom_predict<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V2(u), pp, rho_star, V2(phi), V2(u_star), pp_copy, V2(bo), Ks);
    return;
  }
  const ZPlan zp3 = zplan3(G, kTyStep1, kKcStep1);
  hipLaunchKernelGGL(k_step1_3<kTyStep1>, dim3(zp3.blocks), dim3(64 * kTyStep1), 0, s, G, ph, zp3.kc, rho, V3(u), T, pp, V3(phi), rho_star, e0, V3(u_star), pp_copy, V3(bo), Ks);
}

int launch_energy_rhs(hipStream_t s, const Geo& G, const Phys& ph, bool enth, bool ks,
                      const double* rho, const double* e0, const double* a_prev,
                      const double* T_prev, double* const* phi, const double* rho_star,
                      const double* Ks, const double* Tbg, double* b, double* c,
                      double* x, double* r, double* u_part, double* b_part) {
  const ZPlan zp = zplan(G), zp3 = G.ndim == 3 ? zplan3(G, kTyEnergy, kKcEnergy) : zp;
  const EnergySys sy{b, c, x, r, u_part, b_part};
  // (the enthalpy form always stages T and K*)
  if (G.ndim == 2) {
    if (enth)
      hipLaunchKernelGGL((k_energy_rhs<2, true, true>), dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, e0, a_prev, T_prev, V2(phi), rho_star, Ks, Tbg, sy);
    else if (ks)
      hipLaunchKernelGGL((k_energy_rhs<2, false, true>), dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, e0, a_prev, T_prev, V2(phi), rho_star, Ks, Tbg, sy);
    else
      hipLaunchKernelGGL((k_energy_rhs<2, false, false>), dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, e0, a_prev, T_prev, V2(phi), rho_star, Ks, Tbg, sy);
    return zp.blocks;
  }
  if (enth)
    hipLaunchKernelGGL((k_energy_rhs3<kTyEnergy, true, true>), dim3(zp3.blocks), dim3(64 * kTyEnergy), 0, s, G, ph, zp3.kc, rho, e0, a_prev, T_prev, V3(phi), rho_star, Ks, Tbg, sy);
  else if (ks)
    hipLaunchKernelGGL((k_energy_rhs3<kTyEnergy, false, true>), dim3(zp3.blocks), dim3(64 * kTyEnergy), 0, s, G, ph, zp3.kc, rho, e0, a_prev, T_prev, V3(phi), rho_star, Ks, Tbg, sy);
  else
    hipLaunchKernelGGL((k_energy_rhs3<kTyEnergy, false, false>), dim3(zp3.blocks), dim3(64 * kTyEnergy), 0, s, G, ph, zp3.kc, rho, e0, a_prev, T_prev, V3(phi), rho_star, Ks, Tbg, sy);
  return zp3.blocks;
}

void launch_energy_post(hipStream_t s, const Geo& G, const Phys& ph, const double* T,
                        const double* p, const double* rho_star, double* rho23, double* psi,
                        double* c, double* D) {
  hipLaunchKernelGGL(k_energy_post, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, ph, T, p, rho_star,
                     rho23, psi, c, D);
}

void launch_history_init(hipStream_t s, const Geo& G, const double* p, double* const* u,
                         double* pm, double* Km) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_history_init<2>, grid, block, 0, s, G, p, V2(u), pm, Km);
  else
    hipLaunchKernelGGL(k_history_init<3>, grid, block, 0, s, G, p, V3(u), pm, Km);
}

void launch_enthalpy_prep(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
                          const double* T, const double* p, const double* pm, const double* Km,
                          double* const* u, double* const* u_star, const double* rho_star,
                          double* q, double* pm_next, double* Km_next) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_enthalpy_prep<2>, grid, block, 0, s, G, ph, rho, T, p, pm, Km, V2(u), V2(u_star), rho_star, q, pm_next, Km_next);
  else
    hipLaunchKernelGGL(k_enthalpy_prep<3>, grid, block, 0, s, G, ph, rho, T, p, pm, Km, V3(u), V3(u_star), rho_star, q, pm_next, Km_next);
}

void launch_H(hipStream_t s, const Geo& G, const Phys& ph, const double* rho, double* const* u,
              double* const* u_prev, double* const* phi, double* const* H) {
  const ZPlan zp = zplan(G), zp3 = G.ndim == 3 ? zplan3(G, kTyH, kKcH) : zp;
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_H<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, V2(u), V2(u_prev), V2(phi), V2(H));
  else
    hipLaunchKernelGGL(k_H3<kTyH>, dim3(zp3.blocks), dim3(64 * kTyH), 0, s, G, ph, zp3.kc, rho, V3(u), V3(u_prev), V3(phi), V3(H));
}

int launch_rhs(hipStream_t s, const Geo& G, const Phys& ph, const double* rho,
               const double* rho23, const double* psi, const double* c, const double* D,
               double* const* H, double* b, double* dinv, float* c32, float* D32,
               float* dinv32, const RhsResidual* res) {
  const ZPlan zp = zplan(G), zp3 = G.ndim == 3 ? zplan3(G, kTyRhs, kKcRhs) : zp;
  if (G.ndim == 2) {
    hipLaunchKernelGGL(k_rhs<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, rho, rho23, psi, c, D, V2(H), b, dinv, c32, D32, dinv32);
    return 0;
  }
  if (res) {
    hipLaunchKernelGGL((k_rhs3<kTyRhs, true>), dim3(zp3.blocks), dim3(64 * kTyRhs), 0, s, G, ph, zp3.kc, rho, rho23, psi, c, D, V3(H), b, dinv, c32, D32, dinv32, *res);
    return zp3.blocks;
  }
  hipLaunchKernelGGL((k_rhs3<kTyRhs, false>), dim3(zp3.blocks), dim3(64 * kTyRhs), 0, s, G, ph, zp3.kc, rho, rho23, psi, c, D, V3(H), b, dinv, c32, D32, dinv32, RhsResidual{});
  return 0;
}

void launch_correct(hipStream_t s, const Geo& G, const Phys& ph, const double* pp,
                    const double* rho23, const double* psi, double* const* H, const double* D,
                    const double* rho_star, double* const* u_out, bool last,
                    const double* rho_old, double* rho_new, double* p_new, double* const* phi_out,
                    double* partials, CgScalars* sc) {
  const ZPlan zp = zplan(G),
              zp3 = G.ndim == 3 ? zplan3(G, kTyCorr, last ? kKcCorrLast : kKcCorr) : zp;
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_correct<2>, dim3(zp.blocks), dim3(kBlock), 0, s, G, ph, zp.kc, pp, rho23, psi, V2(H), D, rho_star, V2(u_out), (int)last, rho_old, rho_new, p_new, V2(phi_out), partials);
  else if (last)
    hipLaunchKernelGGL((k_correct3<true, kTyCorr>), dim3(zp3.blocks), dim3(64 * kTyCorr), 0, s, G, ph, zp3.kc, pp, rho23, psi, V3(H), D, rho_star, V3(u_out), rho_old, rho_new, p_new, V3(phi_out), partials);
  else
    hipLaunchKernelGGL((k_correct3<false, kTyCorr>), dim3(zp3.blocks), dim3(64 * kTyCorr), 0, s, G, ph, zp3.kc, pp, rho23, psi, V3(H), D, rho_star, V3(u_out), rho_old, rho_new, p_new, V3(phi_out), partials);
  if (last)
    hipLaunchKernelGGL(k_finalize_reduce, dim3(1), dim3(kBlock), 0, s, (const double*)partials, zp3.blocks, sc);
}

int launch_extrema(hipStream_t s, const Geo& G, const Phys& ph, double* const* u, const double* T,
                   const double* p, double* part, double* out) {
  const int gb = grid_for(G.nc);
  hipLaunchKernelGGL(k_extrema, dim3(gb), dim3(kBlock), 0, s, G, ph, (const double*)u[0],
                     (const double*)(G.ndim == 3 ? u[1] : nullptr), (const double*)u[G.ndim - 1], T,
                     p, part);
  hipLaunchKernelGGL(k_extrema_final, dim3(1), dim3(kBlock), 0, s, (const double*)part, gb, out);
  return gb;
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
