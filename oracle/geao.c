/*
 * geao.c -- plain FP64 CPU oracle (test infrastructure only; see geao.h).
 *
 * Written for a reader who has the paper at hand: loops over cells and faces,
 * no blocking, no fusion.  Each function names the passage it follows.
 *
 * Readings taken where the paper is silent, garbled or inconsistent:
 *  [R1] Sign of gravity in the pressure split (eqs. p_split, mom_split,
 *       p_prime_sd, step4_4sd).  The energy definition and eq. mom use
 *       g > 0 with +rho g k.  The split is only consistent with eq. mom if
 *       "g z" there means g.x with g pointing down.  With Phi = g z (g > 0):
 *       p = p' - rho Phi, and the momentum force is -(grad p' - Phi grad rho).
 *  [R2] Pressure equation (eq. p_prime_sd) is garbled: its left-hand
 *       coefficient lacks dt/rho^{n+1/3} that its right-hand side carries.
 *       It is re-derived from BDF1 continuity with the end-of-step density
 *       rho^{n+1} = p^{n+1}/(R T^{n+1}) = psi (p' - rho^{n+2/3} Phi) and the
 *       corrected face flux phi = D_f S (H_f.n - F_f):
 *          c_i p'_i + sum_f w_f (p'_i - p'_nb) = b_i,
 *          c = psi V/dt, w_f = D_f S_f/d_f, D = rho^{n+2/3} dt / rho^{n+1/3},
 *          b = (V/dt)(rho^n + psi rho^{n+2/3} Phi) - sum_out phitilde_f.
 *  [R3] The predictor's pressure term (eq. step2_sd, Step 1) uses grad p^n
 *       without the weight; the split form grad p'^n - Phi grad rho^n
 *       (eq. mom_split) is used instead.
 *  [R4] Steps 1-3 are written implicitly in u and h, with no linear solver
 *       named.  Transport is taken by explicit Picard sweeps with the frozen
 *       mass flux phi^n: one for the momentum predictor, n_energy_sweeps for
 *       the energy, one per PISO corrector.
 *  [R5] Energy in total-energy form (eq. ent) with e = c_v T + K + Phi
 *       (Sec. 2): the flux of rho u e + p u is phi I4(e + R T).
 *  [R7] The diffusion term of Remark 1 acts on h' = c_p (T - T_bg), with
 *       adiabatic walls, so a resting stratified atmosphere stays at rest.
 *  [R9] n_corr PISO correctors (a parameter; 2 in every workload).
 *  [R10] Fourth-order divergence: point-value cubic interpolation
 *       (-1, 9, 9, -1)/16 on faces with two cells on each side, linear on
 *       faces next to a wall, zero convective flux through walls.
 *  [R11] rho^{n+1} is the conservative update rho^n - dt/V sum_out phi; the
 *       EOS form of eq. step4_4sd differs from it by dt/V times the pressure
 *       residual, reported as eos_mismatch.
 *  [R12] The flux phi^n of Steps 1-3 (eq. e1_d: the face value of rho^n u^n
 *       times the face area) is part of the state: the last corrector's
 *       corrected flux of the previous step, which satisfies that step's
 *       discrete continuity.  Only a state given by cell fields alone (the
 *       initial state) gets the cubic face interpolation of rho u.  (Forming
 *       it from the cell momentum every step grows a grid-scale mode at a
 *       rate ~|u|/h on the 5 m smooth bubble of Sec. 4.1.)
 *  [R13] The solve stops when ||b - A x||_2 <= tol ||b||_2 (recursive
 *       residual), starting from x0 = p' of the previous corrector.
 *  [R14] Initial state: eq. rho_wb read with the background theta0 in the
 *       pressure and the perturbed theta in the temperature; the discrete
 *       background column is made to satisfy F_f = 0 exactly.
 *  Walls (Sec. 4, impenetrable free-slip): no mass or convective flux; no
 *  p' flux (homogeneous Neumann) and F = 0 on walls; wall-normal velocity is
 *  0 at the wall (viscous flux mu (0 - u_n)/(d/2) S), tangential components
 *  feel no shear; energy diffusion adiabatic.
 */
#include "geao.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* With -fopenmp (the all-core timing build) the loops below that write one
 * cell per iteration are shared among threads; no reduction is: every sum
 * and maximum keeps its serial order, so both builds give the same bits. */
#ifdef _OPENMP
#include <omp.h>
#define PER_CELL _Pragma("omp parallel for schedule(static)")
#else
#define PER_CELL
#endif

int geao_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* mesh geometry                                                             */

typedef struct {
  int ndim;      /* 2 (xz-plane) or 3 */
  long nc;       /* number of cells */
  int n[3];      /* cells along direction d */
  long st[3];    /* index stride of direction d */
  double h[3];   /* spacing along d */
  double S[3];   /* area of a face normal to d */
  double V;      /* cell volume */
  int zdir;      /* index of the vertical direction */
  double dz;
} geom;

static geom make_geom(const geao_mesh* m) {
  geom G;
  double dx = m->lx / m->nx, dy = m->ly / m->ny, dz = m->lz / m->nz;
  G.nc = (long)m->nx * m->ny * m->nz;
  G.V = dx * dy * dz;
  G.dz = dz;
  if (m->ny == 1) {
    G.ndim = 2;
    G.n[0] = m->nx; G.st[0] = 1;      G.h[0] = dx; G.S[0] = dy * dz;
    G.n[1] = m->nz; G.st[1] = m->nx;  G.h[1] = dz; G.S[1] = dx * dy;
    G.n[2] = 1;     G.st[2] = 0;      G.h[2] = 0;  G.S[2] = 0;
    G.zdir = 1;
  } else {
    G.ndim = 3;
    G.n[0] = m->nx; G.st[0] = 1;                     G.h[0] = dx; G.S[0] = dy * dz;
    G.n[1] = m->ny; G.st[1] = m->nx;                 G.h[1] = dy; G.S[1] = dx * dz;
    G.n[2] = m->nz; G.st[2] = (long)m->nx * m->ny;   G.h[2] = dz; G.S[2] = dx * dy;
    G.zdir = 2;
  }
  return G;
}

int geao_ndim(const geao_mesh* m) { return m->ny == 1 ? 2 : 3; }

/* position of cell P along direction d */
static int coord(const geom* G, long P, int d) { return (int)((P / G->st[d]) % G->n[d]); }

static int has_hi(const geom* G, long P, int d) { return coord(G, P, d) + 1 < G->n[d]; }
static int has_lo(const geom* G, long P, int d) { return coord(G, P, d) > 0; }

/* Phi = g z at the centre of cell P */
static double phi_cell(const geom* G, const geao_params* q, long P) {
  return q->g * (coord(G, P, G->zdir) + 0.5) * G->dz;
}
/* Phi on the face between P and its +d neighbour */
static double phi_face(const geom* G, const geao_params* q, long P, int d) {
  if (d == G->zdir) return q->g * (coord(G, P, d) + 1.0) * G->dz;
  return phi_cell(G, q, P);
}

static double* zalloc(long n) { return (double*)calloc((size_t)n, sizeof(double)); }

/* ------------------------------------------------------------------------ */
/* discrete operators (Sec. 3, last paragraph; readings R10, walls)          */

/* Face value of s between P and P+st_d: cubic interpolation at the midpoint
 * when two cells lie on each side, else the linear mean. */
static double interp4(const geom* G, const double* s, long P, int d) {
  long st = G->st[d];
  int i = coord(G, P, d);
  if (i >= 1 && i + 2 <= G->n[d] - 1)
    return (-s[P - st] + 9.0 * s[P] + 9.0 * s[P + st] - s[P + 2 * st]) / 16.0;
  return 0.5 * (s[P] + s[P + st]);
}

void geao_face_interp4(const geao_mesh* m, const double* s, int dir, double* out) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P) out[P] = has_hi(&G, P, dir) ? interp4(&G, s, P, dir) : 0.0;
}

void geao_face_sngrad(const geao_mesh* m, const double* s, int dir, double* out) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P)
    out[P] = has_hi(&G, P, dir) ? (s[P + G.st[dir]] - s[P]) / G.h[dir] : 0.0;
}

/* cell value of component d: mean of the two face-normal values along d */
static double reconstruct1(const geom* G, const double* Fd, long P, int d) {
  double hi = has_hi(G, P, d) ? Fd[P] : 0.0;
  double lo = has_lo(G, P, d) ? Fd[P - G->st[d]] : 0.0;
  return 0.5 * (lo + hi);
}

void geao_reconstruct(const geao_mesh* m, const double* faces, double* out) {
  geom G = make_geom(m);
  for (int d = 0; d < G.ndim; ++d)
    PER_CELL
    for (long P = 0; P < G.nc; ++P) out[d * G.nc + P] = reconstruct1(&G, faces + d * G.nc, P, d);
}

/* sum over the faces of P of the outward flux */
static double sum_out(const geom* G, const double* faces, long P) {
  double s = 0.0;
  for (int d = 0; d < G->ndim; ++d) {
    const double* f = faces + d * G->nc;
    if (has_hi(G, P, d)) s += f[P];
    if (has_lo(G, P, d)) s -= f[P - G->st[d]];
  }
  return s;
}

void geao_divergence(const geao_mesh* m, const double* faces, double* out) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P) out[P] = sum_out(&G, faces, P) / G.V;
}

/* sum_out phi_f I4(s)_f */
static double convective1(const geom* G, const double* phi, const double* s, long P) {
  double acc = 0.0;
  for (int d = 0; d < G->ndim; ++d) {
    const double* f = phi + d * G->nc;
    long st = G->st[d];
    if (has_hi(G, P, d)) acc += f[P] * interp4(G, s, P, d);
    if (has_lo(G, P, d)) acc -= f[P - st] * interp4(G, s, P - st, d);
  }
  return acc;
}

void geao_convective(const geao_mesh* m, const double* phi, const double* s, double* out) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P) out[P] = convective1(&G, phi, s, P);
}

/* sum_f mu snGrad(u_comp)_f S_f: interior faces use (u_N - u_P)/d; on a wall
 * the wall-normal component (comp == d) is 0 at distance d/2, tangential
 * components see zero shear. */
static double viscous1(const geom* G, const double* uc, int comp, double mu, long P) {
  double acc = 0.0;
  for (int d = 0; d < G->ndim; ++d) {
    long st = G->st[d];
    double k = mu * G->S[d] / G->h[d];
    if (has_hi(G, P, d)) acc += k * (uc[P + st] - uc[P]);
    else if (comp == d) acc += 2.0 * k * (0.0 - uc[P]);
    if (has_lo(G, P, d)) acc += k * (uc[P - st] - uc[P]);
    else if (comp == d) acc += 2.0 * k * (0.0 - uc[P]);
  }
  return acc;
}

void geao_viscous(const geao_mesh* m, const double* uc, int comp, double mu, double* out) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P) out[P] = viscous1(&G, uc, comp, mu, P);
}

void geao_potential(const geao_mesh* m, const geao_params* q, double* out) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P) out[P] = phi_cell(&G, q, P);
}

/* F_f = [(p'_N - p'_P) - Phi_f (rho_N - rho_P)] / d on interior faces, 0 on
 * walls: the face-normal value of grad p' - Phi grad rho (eq. mom_split, R1). */
static void force_faces(const geom* G, const geao_params* q, const double* pp, const double* rho,
                        double* F) {
  for (int d = 0; d < G->ndim; ++d) {
    long st = G->st[d];
    PER_CELL
    for (long P = 0; P < G->nc; ++P) {
      double v = 0.0;
      if (has_hi(G, P, d))
        v = ((pp[P + st] - pp[P]) - phi_face(G, q, P, d) * (rho[P + st] - rho[P])) / G->h[d];
      F[d * G->nc + P] = v;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* initial state: Sec. 4, eqs. rho_wb, dcEqn1, dcEqn2, e0 (reading R14)      */

int geao_init_bubble(const geao_mesh* m, const geao_params* q, const geao_bubble* b,
                     double* rho, double* u, double* T, double* pp, double* p, double* Tbg) {
  if (m->nx < 1 || m->ny < 1 || m->nz < 1) return GEAO_ERR_ARG;
  geom G = make_geom(m);
  int nz = m->nz;
  double* rho_a = zalloc(nz);
  double* pp_a = zalloc(nz);
  double dx = m->lx / m->nx, dy = m->ly / m->ny;
  /* background: Exner function pi_b(z) = 1 - g z /(c_p theta0) of a neutral
   * atmosphere; density rho_a = p0 pi_b^{c_v/R} / (R theta0) (eq. rho_wb) */
  for (int k = 0; k < nz; ++k) {
    double z = (k + 0.5) * G.dz;
    double pib = 1.0 - q->g * z / (q->cp * q->theta0);
    rho_a[k] = q->p0 * pow(pib, q->cv / q->R) / (q->R * q->theta0);
  }
  /* discrete hydrostatic column: p'_{k+1} - p'_k = Phi_{k+1/2} (rho_{k+1} - rho_k)
   * makes F_f = 0 on every face of the unperturbed state */
  {
    double z0 = 0.5 * G.dz;
    double pib0 = 1.0 - q->g * z0 / (q->cp * q->theta0);
    pp_a[0] = q->p0 * pow(pib0, q->cp / q->R) + rho_a[0] * q->g * z0;
    for (int k = 0; k + 1 < nz; ++k)
      pp_a[k + 1] = pp_a[k] + q->g * (k + 1.0) * G.dz * (rho_a[k + 1] - rho_a[k]);
  }
  for (int k = 0; k < nz; ++k) {
    double Phi = q->g * (k + 0.5) * G.dz;
    double pb = pp_a[k] - rho_a[k] * Phi;
    Tbg[k] = pb / (q->R * rho_a[k]);
  }
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    int i = (int)(P % m->nx);
    int j = (int)((P / m->nx) % m->ny);
    int k = (int)(P / ((long)m->nx * m->ny));
    double x = (i + 0.5) * dx, y = (j + 0.5) * dy, z = (k + 0.5) * G.dz;
    double r2 = (x - b->xc) * (x - b->xc) + (z - b->zc) * (z - b->zc);
    if (G.ndim == 3) r2 += (y - b->yc) * (y - b->yc);
    double r = sqrt(r2);
    double th = 0.0;
    if (b->kind == 1 && r <= b->rc) th = 0.5 * b->amp * (1.0 + cos(M_PI * r / b->rc));
    if (b->kind == 2 && r <= b->rc) th = b->amp;
    double Phi = q->g * z;
    double pb = pp_a[k] - rho_a[k] * Phi;
    double Tb = Tbg[k];
    T[P] = Tb * (1.0 + th / q->theta0);
    p[P] = pb;
    rho[P] = p[P] / (q->R * T[P]);
    pp[P] = p[P] + rho[P] * Phi;
    for (int d = 0; d < G.ndim; ++d) u[d * G.nc + P] = 0.0;
  }
  free(rho_a);
  free(pp_a);
  return GEAO_OK;
}

/* ------------------------------------------------------------------------ */
/* Step 1 (eqs. e1_d, step2_sd, step1_3sd)                                   */

/* phi_f = I4(rho^n u^n . n)_f S_f on interior faces; rho* = rho^n - dt/V sum_out phi */
void geao_mass_predictor(const geao_mesh* m, const geao_params* q, const double* rho,
                         const double* u, double* phi, double* rho_star) {
  geom G = make_geom(m);
  double* mom = zalloc(G.nc);
  for (int d = 0; d < G.ndim; ++d) {
    PER_CELL
    for (long P = 0; P < G.nc; ++P) mom[P] = rho[P] * u[d * G.nc + P];
    PER_CELL
    for (long P = 0; P < G.nc; ++P)
      phi[d * G.nc + P] = has_hi(&G, P, d) ? interp4(&G, mom, P, d) * G.S[d] : 0.0;
  }
  PER_CELL
  for (long P = 0; P < G.nc; ++P) rho_star[P] = rho[P] - q->dt / G.V * sum_out(&G, phi, P);
  free(mom);
}

/* phi_f = I4(rho u . n)_f S_f on interior faces (eq. e1_d from cell values) */
void geao_face_mass_flux(const geao_mesh* m, const double* rho, const double* u, double* phi) {
  geom G = make_geom(m);
  double* mom = zalloc(G.nc);
  for (int d = 0; d < G.ndim; ++d) {
    PER_CELL
    for (long P = 0; P < G.nc; ++P) mom[P] = rho[P] * u[d * G.nc + P];
    PER_CELL
    for (long P = 0; P < G.nc; ++P)
      phi[d * G.nc + P] = has_hi(&G, P, d) ? interp4(&G, mom, P, d) * G.S[d] : 0.0;
  }
  free(mom);
}

/* rho* = rho^n - dt/V sum_out phi^n (eq. e1_d with the state's flux) */
void geao_density_predictor(const geao_mesh* m, const geao_params* q, const double* rho,
                            const double* phi, double* rho_star) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P) rho_star[P] = rho[P] - q->dt / G.V * sum_out(&G, phi, P);
}

/* rho* u* = rho^n u^n - dt/V [sum_out phi I4(u^n) - sum_f mu snGrad(u^n) S]
 *           - dt R(F^n),   F^n from p'^n and rho^n (R3, R4)                  */
void geao_momentum_predictor(const geao_mesh* m, const geao_params* q, const double* rho,
                             const double* u, const double* pp, const double* rho_star,
                             const double* phi, double* u_star) {
  geom G = make_geom(m);
  double* F = zalloc(G.ndim * G.nc);
  force_faces(&G, q, pp, rho, F);
  for (int c = 0; c < G.ndim; ++c) {
    const double* uc = u + c * G.nc;
    PER_CELL
    for (long P = 0; P < G.nc; ++P) {
      double conv = convective1(&G, phi, uc, P);
      double visc = viscous1(&G, uc, c, q->mu, P);
      double RF = reconstruct1(&G, F + c * G.nc, P, c);
      double mom = rho[P] * uc[P] - q->dt / G.V * (conv - visc) - q->dt * RF;
      u_star[c * G.nc + P] = mom / rho_star[P];
    }
  }
  free(F);
}

static double kinetic(const geom* G, const double* u, long P) {
  double k = 0.0;
  for (int d = 0; d < G->ndim; ++d) k += u[d * G->nc + P] * u[d * G->nc + P];
  return 0.5 * k;
}

/* ------------------------------------------------------------------------ */
/* Step 2 in total-energy form (eqs. ent, step3_sd, step3_2sd; R4, R5, R7)   */

/* The diffusion term of Step 2 is taken at the new level, as eq. step3_sd
 * writes it; the convective term by Picard sweeps with the frozen flux.
 * Sweep s solves, with e = c_v T + K* + Phi and T' = T - T_bg,
 *   rho* e^(s) = rho^n e^n - dt/V sum_out phi I4(e + R T)^(s-1)
 *                + dt/V sum_f (mu/Pr) c_p snGrad(T'^(s))_f S_f,
 * i.e. (times V/dt) the SPD system
 *   c_i T_i + sum_f k_f (T_i - T_nb) = b_i,   c = rho* c_v V/dt,
 *   k_f = (mu/Pr) c_p S_f/h_f (interior faces; adiabatic walls),
 *   b = V/dt (rho^n e^n - rho* (K* + Phi)) - sum_out phi I4(e + R T)^(s-1)
 *       + sum_f k_f (T_bg,i - T_bg,nb),
 * by Jacobi-PCG from T^(s-1) to a relative residual of GEAO_ENERGY_TOL.
 * (Explicit diffusion sweeps converge to this only while
 * dt (mu/Pr) c_p/(rho c_v) sum_d 4/h_d^2 < 1.) */
void geao_energy(const geao_mesh* m, const geao_params* q, const double* rho, const double* u,
                 const double* T, const double* u_star, const double* rho_star,
                 const double* phi, const double* Tbg, double* T_new) {
  geom G = make_geom(m);
  double* e_n = zalloc(G.nc);
  double* e = zalloc(G.nc);
  double* Tk = zalloc(G.nc);
  double* hhat = zalloc(G.nc);
  double* cT = zalloc(G.nc);
  double* DT = zalloc(G.nc);
  double* bT = zalloc(G.nc);
  const double kcoef = q->mu / q->Pr * q->cp;  /* w_f = (D_P + D_N)/2 S/h with D = kcoef */
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    e_n[P] = q->cv * T[P] + kinetic(&G, u, P) + phi_cell(&G, q, P);  /* e = c_v T + K + g z */
    e[P] = e_n[P];
    Tk[P] = T[P];
    cT[P] = rho_star[P] * q->cv * G.V / q->dt;
    DT[P] = kcoef;
  }
  for (int s = 0; s < q->n_energy_sweeps; ++s) {
    PER_CELL
    for (long P = 0; P < G.nc; ++P) hhat[P] = e[P] + q->R * Tk[P];  /* e + p/rho */
    PER_CELL
    for (long P = 0; P < G.nc; ++P) {
      double conv = convective1(&G, phi, hhat, P);
      /* the background part of the diffusion of h' = c_p (T - T_bg) */
      double bg = 0.0;
      int kz = coord(&G, P, G.zdir);
      for (int d = 0; d < G.ndim; ++d) {
        double k = kcoef * G.S[d] / G.h[d];
        long st = G.st[d];
        if (has_hi(&G, P, d)) bg += k * (Tbg[kz] - Tbg[coord(&G, P + st, G.zdir)]);
        if (has_lo(&G, P, d)) bg += k * (Tbg[kz] - Tbg[coord(&G, P - st, G.zdir)]);
      }
      double rest = kinetic(&G, u_star, P) + phi_cell(&G, q, P);
      bT[P] = G.V / q->dt * (rho[P] * e_n[P] - rho_star[P] * rest) - conv + bg;
    }
    geao_solve_stats st;
    geao_pcg(m, cT, DT, bT, Tk, GEAO_ENERGY_TOL, q->max_iter, &st);
    PER_CELL
    for (long P = 0; P < G.nc; ++P)
      e[P] = q->cv * Tk[P] + kinetic(&G, u_star, P) + phi_cell(&G, q, P);
  }
  memcpy(T_new, Tk, sizeof(double) * G.nc);
  free(e_n); free(e); free(Tk); free(hhat); free(cT); free(DT); free(bT);
}

/* ------------------------------------------------------------------------ */
/* Step 2 in enthalpy form (eqs. over_ent, ent_LES, step3_sd, step3_2sd; R16) */

/* The form the paper solves: with h = c_p T (eq. K_h) as the unknown,
 *   rho* h/dt + (1/V) sum_out phi I4(h) - (1/V) sum_f (mu/Pr) snGrad(h') S
 *     = b~_e - rho* K* / dt - (1/V) sum_out phi I4(K*) + p^n/dt - rho* g w*,
 *   b~_e = (rho^n h^n + rho^n K^{n-1} - p^{n-1})/dt,
 * where rho*, u* = (.., w*) and K* come from Step 1 and phi is the state's
 * face flux.  As in the total-energy form, the convective term of h takes
 * the previous sweep's h (sweep 1: h^n), the diffusion term the new one, and
 * the diffusion acts on h' = c_p (T - T_bg) with adiabatic walls.  Sweep s
 * solves (times V, for T) the SPD system
 *   c_i T_i + sum_f k_f (T_i - T_nb) = b_i,   c = rho* c_p V/dt,
 *   k_f = (mu/Pr) c_p S_f/h_f,
 *   b = V [b~_e - rho* K* / dt + p^n/dt - rho* g w*] - sum_out phi I4(K*)
 *       - sum_out phi I4(c_p T^(s-1)) + sum_f k_f (T_bg,i - T_bg,nb)
 * by Jacobi-PCG from T^(s-1) to GEAO_ENERGY_TOL.  eq. step3_2sd then holds
 * with h = c_p T at both levels. */
void geao_energy_enthalpy(const geao_mesh* m, const geao_params* q, const double* rho,
                          const double* T, const double* p, const double* p_old,
                          const double* K_old, const double* u_star, const double* rho_star,
                          const double* phi, const double* Tbg, double* T_new) {
  geom G = make_geom(m);
  double* Ks = zalloc(G.nc);
  double* h = zalloc(G.nc);
  double* Tk = zalloc(G.nc);
  double* src = zalloc(G.nc);
  double* cT = zalloc(G.nc);
  double* DT = zalloc(G.nc);
  double* bT = zalloc(G.nc);
  const double kcoef = q->mu / q->Pr * q->cp;
  const double* w_star = u_star + (long)G.zdir * G.nc;  /* vertical component of u* */
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    Ks[P] = kinetic(&G, u_star, P);
    Tk[P] = T[P];
    cT[P] = rho_star[P] * q->cp * G.V / q->dt;
    DT[P] = kcoef;
  }
  /* the terms no sweep changes */
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    double b_e = (rho[P] * q->cp * T[P] + rho[P] * K_old[P] - p_old[P]) / q->dt;
    double local = b_e - rho_star[P] * Ks[P] / q->dt + p[P] / q->dt - rho_star[P] * q->g * w_star[P];
    double conv_K = convective1(&G, phi, Ks, P);
    double bg = 0.0;
    int kz = coord(&G, P, G.zdir);
    for (int d = 0; d < G.ndim; ++d) {
      double k = kcoef * G.S[d] / G.h[d];
      long st = G.st[d];
      if (has_hi(&G, P, d)) bg += k * (Tbg[kz] - Tbg[coord(&G, P + st, G.zdir)]);
      if (has_lo(&G, P, d)) bg += k * (Tbg[kz] - Tbg[coord(&G, P - st, G.zdir)]);
    }
    src[P] = G.V * local - conv_K + bg;
  }
  for (int s = 0; s < q->n_energy_sweeps; ++s) {
    PER_CELL
    for (long P = 0; P < G.nc; ++P) h[P] = q->cp * Tk[P];
    PER_CELL
    for (long P = 0; P < G.nc; ++P) bT[P] = src[P] - convective1(&G, phi, h, P);
    geao_solve_stats st;
    geao_pcg(m, cT, DT, bT, Tk, GEAO_ENERGY_TOL, q->max_iter, &st);
  }
  memcpy(T_new, Tk, sizeof(double) * G.nc);
  free(Ks); free(h); free(Tk); free(src); free(cT); free(DT); free(bT);
}

/* eq. step3_3sd: rho^{n+2/3} R T^{n+1} = p^n; and the pressure-equation
 * coefficients of reading R2: psi = 1/(R T), c = psi V/dt, D = rho23 dt / rho* */
void geao_eos_coeffs(const geao_mesh* m, const geao_params* q, const double* p,
                     const double* T_new, const double* rho_star,
                     double* rho23, double* psi, double* c, double* D) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    rho23[P] = p[P] / (q->R * T_new[P]);
    psi[P] = 1.0 / (q->R * T_new[P]);
    c[P] = psi[P] * G.V / q->dt;
    D[P] = rho23[P] / (rho_star[P] / q->dt);
  }
}

/* ------------------------------------------------------------------------ */
/* Step 3 (eqs. step2_sd [corrector], p_prime_sd, step4_4sd; PISO)           */

/* H(u) = rho^n u^n/dt - (1/V) sum_out phi I4(u) + (1/V) sum_f mu snGrad(u) S */
void geao_H(const geao_mesh* m, const geao_params* q, const double* rho, const double* u,
            const double* u_prev, const double* phi, double* H) {
  geom G = make_geom(m);
  for (int c = 0; c < G.ndim; ++c) {
    const double* uc = u_prev + c * G.nc;
    PER_CELL
    for (long P = 0; P < G.nc; ++P) {
      double conv = convective1(&G, phi, uc, P);
      double visc = viscous1(&G, uc, c, q->mu, P);
      H[c * G.nc + P] = rho[P] * u[c * G.nc + P] / q->dt - conv / G.V + visc / G.V;
    }
  }
}

/* phitilde_f = D_f S_f [H_f . n + Phi_f (rho23_N - rho23_P)/d] with face means
 * of D and H; b = (V/dt)(rho^n + psi rho23 Phi) - sum_out phitilde (R2) */
void geao_predicted_flux_rhs(const geao_mesh* m, const geao_params* q, const double* rho,
                             const double* rho23, const double* psi, const double* D,
                             const double* H, double* phi_tilde, double* b) {
  geom G = make_geom(m);
  for (int d = 0; d < G.ndim; ++d) {
    long st = G.st[d];
    const double* Hd = H + d * G.nc;
    PER_CELL
    for (long P = 0; P < G.nc; ++P) {
      double v = 0.0;
      if (has_hi(&G, P, d)) {
        double Df = 0.5 * (D[P] + D[P + st]);
        double Hf = 0.5 * (Hd[P] + Hd[P + st]);
        v = Df * G.S[d] * (Hf + phi_face(&G, q, P, d) * (rho23[P + st] - rho23[P]) / G.h[d]);
      }
      phi_tilde[d * G.nc + P] = v;
    }
  }
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    double Phi = phi_cell(&G, q, P);
    b[P] = G.V / q->dt * (rho[P] + psi[P] * rho23[P] * Phi) - sum_out(&G, phi_tilde, P);
  }
}

/* y = A x, (A x)_i = c_i x_i + sum_f w_f (x_i - x_nb), w_f = (D_P + D_N)/2 S/d */
static void apply_A(const geom* G, const double* c, const double* D, const double* x, double* y) {
  PER_CELL
  for (long P = 0; P < G->nc; ++P) {
    double acc = c[P] * x[P];
    for (int d = 0; d < G->ndim; ++d) {
      long st = G->st[d];
      double k = G->S[d] / G->h[d];
      if (has_hi(G, P, d)) acc += 0.5 * (D[P] + D[P + st]) * k * (x[P] - x[P + st]);
      if (has_lo(G, P, d)) acc += 0.5 * (D[P - st] + D[P]) * k * (x[P] - x[P - st]);
    }
    y[P] = acc;
  }
}

void geao_apply_A(const geao_mesh* m, const double* c, const double* D, const double* x,
                  double* y) {
  geom G = make_geom(m);
  apply_A(&G, c, D, x, y);
}

static double dot(long n, const double* a, const double* b) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Conjugate gradients with the Jacobi (diagonal) preconditioner, textbook
 * form; stops when the recursive residual satisfies ||r|| <= tol ||b|| (R13). */
int geao_pcg(const geao_mesh* m, const double* c, const double* D, const double* b, double* x,
             double tol, int max_iter, geao_solve_stats* st) {
  geom G = make_geom(m);
  long n = G.nc;
  double* r = zalloc(n);
  double* z = zalloc(n);
  double* pdir = zalloc(n);
  double* q = zalloc(n);
  double* diag = zalloc(n);
  PER_CELL
  for (long P = 0; P < n; ++P) {
    double a = c[P];
    for (int d = 0; d < G.ndim; ++d) {
      double k = G.S[d] / G.h[d];
      if (has_hi(&G, P, d)) a += 0.5 * (D[P] + D[P + G.st[d]]) * k;
      if (has_lo(&G, P, d)) a += 0.5 * (D[P - G.st[d]] + D[P]) * k;
    }
    diag[P] = a;
  }
  double nb = sqrt(dot(n, b, b));
  int status = GEAO_OK;
  int it = 0;
  double nr;
  if (nb == 0.0) {
    PER_CELL
    for (long P = 0; P < n; ++P) x[P] = 0.0;
    nb = 1.0;
  }
  apply_A(&G, c, D, x, q);
  PER_CELL
  for (long P = 0; P < n; ++P) r[P] = b[P] - q[P];
  PER_CELL
  for (long P = 0; P < n; ++P) z[P] = r[P] / diag[P];
  PER_CELL
  for (long P = 0; P < n; ++P) pdir[P] = z[P];
  double rz = dot(n, r, z);
  nr = sqrt(dot(n, r, r));
  st->rel_res0 = nr / nb;
  if (!isfinite(nr)) status = GEAO_ERR_NAN;
  while (status == GEAO_OK && nr > tol * nb) {
    if (it >= max_iter) { status = GEAO_ERR_NOCONV; break; }
    apply_A(&G, c, D, pdir, q);
    double alpha = rz / dot(n, pdir, q);
    PER_CELL
    for (long P = 0; P < n; ++P) x[P] += alpha * pdir[P];
    PER_CELL
    for (long P = 0; P < n; ++P) r[P] -= alpha * q[P];
    PER_CELL
    for (long P = 0; P < n; ++P) z[P] = r[P] / diag[P];
    double rz_new = dot(n, r, z);
    double beta = rz_new / rz;
    PER_CELL
    for (long P = 0; P < n; ++P) pdir[P] = z[P] + beta * pdir[P];
    rz = rz_new;
    nr = sqrt(dot(n, r, r));
    ++it;
    if (!isfinite(nr)) { status = GEAO_ERR_NAN; break; }
  }
  st->iters = it;
  st->rel_res = nr / nb;
  st->converged = status == GEAO_OK;
  apply_A(&G, c, D, x, q);
  PER_CELL
  for (long P = 0; P < n; ++P) r[P] = b[P] - q[P];
  st->true_rel_res = sqrt(dot(n, r, r)) / nb;
  free(r); free(z); free(pdir); free(q); free(diag);
  return status;
}

/* ------------------------------------------------------------------------ */
/* implicit transport (eqs. step2_sd of Step 1 and step3_sd with the         */
/* convective and diffusive terms at the new level, as written; R19)        */

typedef void (*op_fn)(const geom* G, const void* ctx, const double* x, double* y);

/* weight of cell P in the I4 value of its upper (hi = 1) or lower face along d */
static double i4_self_weight(const geom* G, long P, int d, int hi) {
  int q = hi ? coord(G, P, d) : coord(G, P, d) - 1;  /* the face's lower cell */
  return (q >= 1 && q + 2 <= G->n[d] - 1) ? 9.0 / 16.0 : 0.5;
}

/* diagonal entry of x -> sum_out phi I4(x) */
static double convective_diag(const geom* G, const double* phi, long P) {
  double a = 0.0;
  for (int d = 0; d < G->ndim; ++d) {
    const double* f = phi + d * G->nc;
    if (has_hi(G, P, d)) a += f[P] * i4_self_weight(G, P, d, 1);
    if (has_lo(G, P, d)) a -= f[P - G->st[d]] * i4_self_weight(G, P, d, 0);
  }
  return a;
}

/* momentum component comp (times V):
 *   (A u)_P = rho*_P V/dt u_P + sum_out phi I4(u) - sum_f mu snGrad(u)_f S_f */
typedef struct {
  const geao_params* q;
  const double* rho_star;
  const double* phi;
  int comp;
} mom_ctx;

static void mom_op(const geom* G, const void* vc, const double* x, double* y) {
  const mom_ctx* c = (const mom_ctx*)vc;
  PER_CELL
  for (long P = 0; P < G->nc; ++P)
    y[P] = c->rho_star[P] * G->V / c->q->dt * x[P] + convective1(G, c->phi, x, P) -
           viscous1(G, x, c->comp, c->q->mu, P);
}

static double mom_diag(const geom* G, const mom_ctx* c, long P) {
  double a = c->rho_star[P] * G->V / c->q->dt + convective_diag(G, c->phi, P);
  for (int d = 0; d < G->ndim; ++d) {
    double k = c->q->mu * G->S[d] / G->h[d];
    a += has_hi(G, P, d) ? k : (c->comp == d ? 2.0 * k : 0.0);
    a += has_lo(G, P, d) ? k : (c->comp == d ? 2.0 * k : 0.0);
  }
  return a;
}

/* energy, unknown T (times V):
 *   (A T)_P = cT_P T_P + c_p sum_out phi I4(T) + sum_f k_f (T_P - T_nb),
 * k_f = (mu/Pr) c_p S_f/h_f on interior faces (adiabatic walls) */
typedef struct {
  const geao_params* q;
  const double* cT;
  const double* DT;
  const double* phi;
} energy_ctx;

static void energy_op(const geom* G, const void* vc, const double* x, double* y) {
  const energy_ctx* c = (const energy_ctx*)vc;
  apply_A(G, c->cT, c->DT, x, y);
  PER_CELL
  for (long P = 0; P < G->nc; ++P) y[P] += c->q->cp * convective1(G, c->phi, x, P);
}

/* BiCGStab (van der Vorst 1992) with the Jacobi preconditioner on the right:
 * each search direction is scaled by dinv = 1/diag(A) before the operator
 * is applied.  Stops when the recursive residual (of s after the first half
 * step, or of r) satisfies ||.|| <= tol ||b||; a zero denominator ends the
 * solve as not converged. */
static int bicgstab(const geom* G, op_fn A, const void* ctx, const double* b, double* x,
                    const double* dinv, double tol, int max_iter, geao_solve_stats* st) {
  long n = G->nc;
  double* r = zalloc(n);
  double* rh = zalloc(n);
  double* p = zalloc(n);
  double* v = zalloc(n);
  double* y = zalloc(n);
  double* sv = zalloc(n);
  double* z = zalloc(n);
  double* t = zalloc(n);
  A(G, ctx, x, t);
  PER_CELL
  for (long P = 0; P < n; ++P) {
    r[P] = b[P] - t[P];
    rh[P] = r[P];
  }
  double bb = dot(n, b, b), rr = dot(n, r, r);
  double tol2 = tol * tol;
  st->rel_res0 = bb > 0 ? sqrt(rr / bb) : 0.0;
  int status = GEAO_ERR_NOCONV, it = 0;
  if (bb == 0.0) {
    memset(x, 0, sizeof(double) * n);
    rr = 0.0;
    status = GEAO_OK;
  } else if (rr <= tol2 * bb) {
    status = GEAO_OK;
  }
  double rho_old = 1.0, alpha = 1.0, omega = 1.0;
  while (status == GEAO_ERR_NOCONV && it < max_iter) {
    double rho = dot(n, rh, r);
    if (rho == 0.0) break;
    double beta = (rho / rho_old) * (alpha / omega);
    PER_CELL
    for (long P = 0; P < n; ++P) {
      p[P] = r[P] + beta * (p[P] - omega * v[P]);
      y[P] = dinv[P] * p[P];
    }
    A(G, ctx, y, v);
    double rv = dot(n, rh, v);
    if (rv == 0.0) break;
    alpha = rho / rv;
    PER_CELL
    for (long P = 0; P < n; ++P) {
      x[P] += alpha * y[P];
      sv[P] = r[P] - alpha * v[P];
    }
    ++it;
    double ss = dot(n, sv, sv);
    if (!isfinite(ss)) { status = GEAO_ERR_NAN; break; }
    if (ss <= tol2 * bb) {
      memcpy(r, sv, sizeof(double) * n);
      rr = ss;
      status = GEAO_OK;
      break;
    }
    PER_CELL
    for (long P = 0; P < n; ++P) z[P] = dinv[P] * sv[P];
    A(G, ctx, z, t);
    double tt = dot(n, t, t);
    if (tt == 0.0) break;
    omega = dot(n, t, sv) / tt;
    PER_CELL
    for (long P = 0; P < n; ++P) {
      x[P] += omega * z[P];
      r[P] = sv[P] - omega * t[P];
    }
    rr = dot(n, r, r);
    rho_old = rho;
    if (!isfinite(rr)) { status = GEAO_ERR_NAN; break; }
    if (rr <= tol2 * bb) status = GEAO_OK;
    if (omega == 0.0) break;
  }
  st->iters = it;
  st->converged = status == GEAO_OK;
  st->rel_res = bb > 0 ? sqrt(rr / bb) : 0.0;
  A(G, ctx, x, t);
  PER_CELL
  for (long P = 0; P < n; ++P) r[P] = b[P] - t[P];
  st->true_rel_res = bb > 0 ? sqrt(dot(n, r, r) / bb) : 0.0;
  free(r); free(rh); free(p); free(v); free(y); free(sv); free(z); free(t);
  return status;
}

/* y = A x of the implicit predictor's operator for component comp */
void geao_momentum_operator(const geao_mesh* m, const geao_params* q, const double* rho_star,
                            const double* phi, int comp, const double* x, double* y) {
  geom G = make_geom(m);
  mom_ctx c = {q, rho_star, phi, comp};
  mom_op(&G, &c, x, y);
}

/* y = A x of the implicit energy operator (cT: the unknown's coefficient) */
void geao_energy_operator(const geao_mesh* m, const geao_params* q, const double* cT,
                          const double* phi, const double* x, double* y) {
  geom G = make_geom(m);
  double* DT = zalloc(G.nc);
  for (long P = 0; P < G.nc; ++P) DT[P] = q->mu / q->Pr * q->cp;
  energy_ctx c = {q, cT, DT, phi};
  energy_op(&G, &c, x, y);
  free(DT);
}

/* the diagonal of the momentum operator (comp >= 0) or, with comp = -1, of
 * the energy operator with coefficient cT (rho_star unused) */
void geao_transport_diag(const geao_mesh* m, const geao_params* q, const double* rho_star,
                         const double* cT, const double* phi, int comp, double* diag) {
  geom G = make_geom(m);
  const double kcoef = q->mu / q->Pr * q->cp;
  mom_ctx mc = {q, rho_star, phi, comp};
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    if (comp >= 0) {
      diag[P] = mom_diag(&G, &mc, P);
    } else {
      double a = cT[P] + q->cp * convective_diag(&G, phi, P);
      for (int d = 0; d < G.ndim; ++d) {
        double k = kcoef * G.S[d] / G.h[d];
        if (has_hi(&G, P, d)) a += k;
        if (has_lo(&G, P, d)) a += k;
      }
      diag[P] = a;
    }
  }
}

/* BiCGStab on the momentum operator of component comp (test access) */
int geao_bicgstab_momentum(const geao_mesh* m, const geao_params* q, const double* rho_star,
                           const double* phi, int comp, const double* b, double* x, double tol,
                           int max_iter, geao_solve_stats* st) {
  geom G = make_geom(m);
  mom_ctx c = {q, rho_star, phi, comp};
  double* dinv = zalloc(G.nc);
  for (long P = 0; P < G.nc; ++P) dinv[P] = 1.0 / mom_diag(&G, &c, P);
  int rc = bicgstab(&G, mom_op, &c, b, x, dinv, tol, max_iter, st);
  free(dinv);
  return rc;
}

/* eq. step2_sd of Step 1 implicit in u^{n+1/3}: for each component c
 *   (rho* V/dt) u + sum_out phi I4(u) - sum_f mu snGrad(u) S = V (rho^n u^n/dt - R(F^n)),
 * F^n from p'^n and rho^n as in the explicit predictor; solved by BiCGStab
 * to GEAO_TRANSPORT_TOL from the value u_star holds on entry (the explicit
 * predictor's).  Returns the first failing solve's status. */
int geao_momentum_predictor_implicit(const geao_mesh* m, const geao_params* q, const double* rho,
                                     const double* u, const double* pp, const double* rho_star,
                                     const double* phi, double* u_star) {
  geom G = make_geom(m);
  double* F = zalloc(G.ndim * G.nc);
  double* b = zalloc(G.nc);
  double* dinv = zalloc(G.nc);
  force_faces(&G, q, pp, rho, F);
  int status = GEAO_OK;
  for (int c = 0; c < G.ndim && status == GEAO_OK; ++c) {
    const double* uc = u + c * G.nc;
    mom_ctx ctx = {q, rho_star, phi, c};
    PER_CELL
    for (long P = 0; P < G.nc; ++P) {
      b[P] = G.V * (rho[P] * uc[P] / q->dt - reconstruct1(&G, F + c * G.nc, P, c));
      dinv[P] = 1.0 / mom_diag(&G, &ctx, P);
    }
    geao_solve_stats st;
    status = bicgstab(&G, mom_op, &ctx, b, u_star + c * G.nc, dinv, GEAO_TRANSPORT_TOL,
                      q->max_iter, &st);
  }
  free(F); free(b); free(dinv);
  return status;
}

/* Step 2 with the transport of the energy implicit (either energy form):
 * the unknown T, transported as c_p T, at the new level in both the
 * convective and the diffusive term; the known part of the transported
 * quantity (K* + Phi in the total-energy form, K* in the enthalpy form)
 * explicit.  One BiCGStab solve from T^n to GEAO_TRANSPORT_TOL of
 *   cT T + c_p sum_out phi I4(T) + sum_f k_f (T_P - T_nb) = b,
 * total energy: cT = rho* c_v V/dt,
 *   b = V/dt (rho^n e^n - rho* (K* + Phi)) - sum_out phi I4(K* + Phi) + bg;
 * enthalpy:     cT = rho* c_p V/dt,
 *   b = V [b~_e - rho* K* / dt + p^n/dt - rho* g w*] - sum_out phi I4(K*) + bg;
 * bg the background column's diffusion as in the sweeps. */
int geao_energy_implicit(const geao_mesh* m, const geao_params* q, const double* rho,
                         const double* u, const double* T, const double* p, const double* p_old,
                         const double* K_old, const double* u_star, const double* rho_star,
                         const double* phi, const double* Tbg, double* T_new) {
  geom G = make_geom(m);
  const int enth = q->energy_form == 1;
  double* w = zalloc(G.nc);
  double* cT = zalloc(G.nc);
  double* DT = zalloc(G.nc);
  double* b = zalloc(G.nc);
  double* dinv = zalloc(G.nc);
  const double kcoef = q->mu / q->Pr * q->cp;
  const double* w_star = u_star + (long)G.zdir * G.nc;
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    w[P] = kinetic(&G, u_star, P) + (enth ? 0.0 : phi_cell(&G, q, P));
    cT[P] = rho_star[P] * (enth ? q->cp : q->cv) * G.V / q->dt;
    DT[P] = kcoef;
  }
  PER_CELL
  for (long P = 0; P < G.nc; ++P) {
    double local;
    if (enth) {
      double b_e = (rho[P] * q->cp * T[P] + rho[P] * K_old[P] - p_old[P]) / q->dt;
      local = G.V * (b_e - rho_star[P] * w[P] / q->dt + p[P] / q->dt -
                     rho_star[P] * q->g * w_star[P]);
    } else {
      double e_n = q->cv * T[P] + kinetic(&G, u, P) + phi_cell(&G, q, P);
      local = G.V / q->dt * (rho[P] * e_n - rho_star[P] * w[P]);
    }
    double bg = 0.0;
    int kz = coord(&G, P, G.zdir);
    for (int d = 0; d < G.ndim; ++d) {
      double k = kcoef * G.S[d] / G.h[d];
      long st = G.st[d];
      if (has_hi(&G, P, d)) bg += k * (Tbg[kz] - Tbg[coord(&G, P + st, G.zdir)]);
      if (has_lo(&G, P, d)) bg += k * (Tbg[kz] - Tbg[coord(&G, P - st, G.zdir)]);
    }
    b[P] = local - convective1(&G, phi, w, P) + bg;
    double a = cT[P] + q->cp * convective_diag(&G, phi, P);
    for (int d = 0; d < G.ndim; ++d) {
      double k = kcoef * G.S[d] / G.h[d];
      if (has_hi(&G, P, d)) a += k;
      if (has_lo(&G, P, d)) a += k;
    }
    dinv[P] = 1.0 / a;
  }
  memcpy(T_new, T, sizeof(double) * G.nc);
  energy_ctx ctx = {q, cT, DT, phi};
  geao_solve_stats st;
  int status = bicgstab(&G, energy_op, &ctx, b, T_new, dinv, GEAO_TRANSPORT_TOL, q->max_iter, &st);
  free(w); free(cT); free(DT); free(b); free(dinv);
  return status;
}

/* phi^(k) = phitilde - w (p'_N - p'_P);  u^(k) = (H - R(F^(k))) / A, A = rho* / dt,
 * F^(k) from p'^(k) and rho^{n+2/3} (eq. step2_sd corrector, R1) */
void geao_correct(const geao_mesh* m, const geao_params* q, const double* pp,
                  const double* rho23, const double* H, const double* D,
                  const double* rho_star, const double* phi_tilde, double* phi, double* u) {
  geom G = make_geom(m);
  double* F = zalloc(G.ndim * G.nc);
  for (int d = 0; d < G.ndim; ++d) {
    long st = G.st[d];
    PER_CELL
    for (long P = 0; P < G.nc; ++P) {
      double v = 0.0;
      if (has_hi(&G, P, d)) {
        double w = 0.5 * (D[P] + D[P + st]) * G.S[d] / G.h[d];
        v = phi_tilde[d * G.nc + P] - w * (pp[P + st] - pp[P]);
      }
      phi[d * G.nc + P] = v;
    }
  }
  force_faces(&G, q, pp, rho23, F);
  for (int c = 0; c < G.ndim; ++c)
    PER_CELL
    for (long P = 0; P < G.nc; ++P) {
      double A = rho_star[P] / q->dt;
      u[c * G.nc + P] = (H[c * G.nc + P] - reconstruct1(&G, F + c * G.nc, P, c)) / A;
    }
  free(F);
}

/* eq. step4_4sd with R11: p = p' - rho23 Phi; rho^{n+1} = rho^n - dt/V sum_out phi */
void geao_finalize(const geao_mesh* m, const geao_params* q, const double* rho_old,
                   const double* phi, const double* pp, const double* rho23, const double* psi,
                   double* rho_new, double* p_new, double* eos_mismatch) {
  geom G = make_geom(m);
  double mm = 0.0;
  for (long P = 0; P < G.nc; ++P) {
    p_new[P] = pp[P] - rho23[P] * phi_cell(&G, q, P);
    rho_new[P] = rho_old[P] - q->dt / G.V * sum_out(&G, phi, P);
    double mis = fabs(rho_new[P] - psi[P] * p_new[P]);
    if (mis > mm) mm = mis;
  }
  *eos_mismatch = mm;
}

/* ------------------------------------------------------------------------ */
/* one step (Sec. 3: Step 1, Step 2, Step 3 with PISO)                       */

typedef struct {
  double *phi, *rho_star, *u_star, *T_new, *rho23, *psi, *c, *D, *H, *phi_tilde, *b;
  double *phi_corr;   /* corrected face flux of the latest corrector */
} work_t;

static work_t work_alloc(const geom* G) {
  work_t w;
  w.phi = zalloc(G->ndim * G->nc);
  w.rho_star = zalloc(G->nc);
  w.u_star = zalloc(G->ndim * G->nc);
  w.T_new = zalloc(G->nc);
  w.rho23 = zalloc(G->nc);
  w.psi = zalloc(G->nc);
  w.c = zalloc(G->nc);
  w.D = zalloc(G->nc);
  w.H = zalloc(G->ndim * G->nc);
  w.phi_tilde = zalloc(G->ndim * G->nc);
  w.b = zalloc(G->nc);
  w.phi_corr = zalloc(G->ndim * G->nc);
  return w;
}

static void work_free(work_t* w) {
  free(w->phi); free(w->rho_star); free(w->u_star); free(w->T_new); free(w->rho23);
  free(w->psi); free(w->c); free(w->D); free(w->H); free(w->phi_tilde); free(w->b);
  free(w->phi_corr);
}

static int check_args(const geao_mesh* m, const geao_params* q) {
  if (m->nx < 1 || m->ny < 1 || m->nz < 1) return 0;
  if (!(m->lx > 0 && m->ly > 0 && m->lz > 0)) return 0;
  if (!(q->R > 0 && q->cp > 0 && q->cv > 0 && q->dt > 0 && q->Pr > 0)) return 0;
  if (q->n_corr < 1 || q->n_energy_sweeps < 1 || q->max_iter < 0) return 0;
  if (q->energy_form != 0 && q->energy_form != 1) return 0;
  if (q->transport != 0 && q->transport != 1) return 0;
  return 1;
}

/* Steps 1 and 2 of the step starting from the given state (phi: its flux) */
static int steps_1_2(const geao_mesh* m, const geao_params* q, const double* rho,
                     const double* u, const double* T, const double* pp, const double* p,
                     const double* phi, const double* p_old, const double* K_old,
                     const double* Tbg, work_t* w) {
  geom G = make_geom(m);
  memcpy(w->phi, phi, sizeof(double) * G.ndim * G.nc);
  geao_density_predictor(m, q, rho, w->phi, w->rho_star);
  geao_momentum_predictor(m, q, rho, u, pp, w->rho_star, w->phi, w->u_star);
  if (q->transport == 1) {
    /* the explicit predictor's u* is the implicit solve's initial guess */
    int rc = geao_momentum_predictor_implicit(m, q, rho, u, pp, w->rho_star, w->phi, w->u_star);
    if (rc == GEAO_OK)
      rc = geao_energy_implicit(m, q, rho, u, T, p, p_old, K_old, w->u_star, w->rho_star, w->phi,
                                Tbg, w->T_new);
    if (rc != GEAO_OK) return rc;
  } else if (q->energy_form == 1)
    geao_energy_enthalpy(m, q, rho, T, p, p_old, K_old, w->u_star, w->rho_star, w->phi, Tbg,
                         w->T_new);
  else
    geao_energy(m, q, rho, u, T, w->u_star, w->rho_star, w->phi, Tbg, w->T_new);
  geao_eos_coeffs(m, q, p, w->T_new, w->rho_star, w->rho23, w->psi, w->c, w->D);
  return GEAO_OK;
}

int geao_pressure_system(const geao_mesh* m, const geao_params* q, const double* rho,
                         const double* u, const double* T, const double* pp, const double* p,
                         const double* phi, const double* p_old, const double* K_old,
                         const double* Tbg, double* c, double* D, double* b) {
  if (!check_args(m, q)) return GEAO_ERR_ARG;
  geom G = make_geom(m);
  work_t w = work_alloc(&G);
  int rc = steps_1_2(m, q, rho, u, T, pp, p, phi, p_old, K_old, Tbg, &w);
  if (rc != GEAO_OK) {
    work_free(&w);
    return rc;
  }
  geao_H(m, q, rho, u, w.u_star, w.phi, w.H);
  geao_predicted_flux_rhs(m, q, rho, w.rho23, w.psi, w.D, w.H, w.phi_tilde, w.b);
  memcpy(c, w.c, sizeof(double) * G.nc);
  memcpy(D, w.D, sizeof(double) * G.nc);
  memcpy(b, w.b, sizeof(double) * G.nc);
  work_free(&w);
  return GEAO_OK;
}

int geao_step(const geao_mesh* m, const geao_params* q, double* rho, double* u, double* T,
              double* pp, double* p, double* phi, double* p_old, double* K_old,
              const double* Tbg, geao_step_stats* st) {
  if (!check_args(m, q)) return GEAO_ERR_ARG;
  geom G = make_geom(m);
  work_t w = work_alloc(&G);
  double* u_k = zalloc(G.ndim * G.nc);
  double* pp_k = zalloc(G.nc);
  double* rho_new = zalloc(G.nc);
  double* p_new = zalloc(G.nc);
  int status = GEAO_OK;
  st->n_solves = 0;

  status = steps_1_2(m, q, rho, u, T, pp, p, phi, p_old, K_old, Tbg, &w);

  memcpy(u_k, w.u_star, sizeof(double) * G.ndim * G.nc);
  memcpy(pp_k, pp, sizeof(double) * G.nc);
  /* every corrector convects with the frozen Step-1 flux phi^n (eq. step2_sd
   * of Step 3 and the H operator); the corrected flux only feeds the
   * end-of-step density */
  for (int k = 0; k < q->n_corr && status == GEAO_OK; ++k) {
    geao_H(m, q, rho, u, u_k, w.phi, w.H);
    geao_predicted_flux_rhs(m, q, rho, w.rho23, w.psi, w.D, w.H, w.phi_tilde, w.b);
    geao_solve_stats ss;
    int rc = geao_pcg(m, w.c, w.D, w.b, pp_k, q->tol, q->max_iter, &ss);
    if (st->n_solves < 16) st->solve[st->n_solves++] = ss;
    if (rc != GEAO_OK) { status = rc; break; }
    geao_correct(m, q, pp_k, w.rho23, w.H, w.D, w.rho_star, w.phi_tilde, w.phi_corr, u_k);
  }
  if (status == GEAO_OK) {
    geao_finalize(m, q, rho, w.phi_corr, pp_k, w.rho23, w.psi, rho_new, p_new, &st->eos_mismatch);
    for (long P = 0; P < G.nc; ++P)
      if (!isfinite(rho_new[P]) || !isfinite(p_new[P]) || !isfinite(w.T_new[P])) status = GEAO_ERR_NAN;
  }
  if (status == GEAO_OK) {
    /* the lagged terms of the next step: p^n, K^n */
    for (long P = 0; P < G.nc; ++P) K_old[P] = kinetic(&G, u, P);
    memcpy(p_old, p, sizeof(double) * G.nc);
    memcpy(rho, rho_new, sizeof(double) * G.nc);
    memcpy(u, u_k, sizeof(double) * G.ndim * G.nc);
    memcpy(T, w.T_new, sizeof(double) * G.nc);
    memcpy(pp, pp_k, sizeof(double) * G.nc);
    memcpy(p, p_new, sizeof(double) * G.nc);
    memcpy(phi, w.phi_corr, sizeof(double) * G.ndim * G.nc);  /* phi^{n+1} */
  }
  work_free(&w);
  free(u_k); free(pp_k); free(rho_new); free(p_new);
  return status;
}

void geao_theta_prime(const geao_mesh* m, const geao_params* q, const double* T, const double* p,
                      double* out) {
  geom G = make_geom(m);
  PER_CELL
  for (long P = 0; P < G.nc; ++P)
    out[P] = T[P] / pow(p[P] / q->p0, q->R / q->cp) - q->theta0;
}
