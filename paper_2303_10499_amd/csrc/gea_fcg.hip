// gea_fcg.hip -- flexible conjugate gradients for the learned form of the
// pressure solve, and the kernels that cut training pairs from the solver.
//
// The inner FP32 solve of the refinement (A d = r, d0 = 0) with a nonlinear
// preconditioner z = M(r) = s * net(r/s, c/diag), s = max |r|:
//   p = z + beta p_old,  beta = (<z, r> - <z, r_old>) / <z_old, r_old>
//   q = A p, alpha = <z, r> / <p, q>, d += alpha p, r_old = r, r -= alpha q
// (Polak-Ribiere beta, which keeps CG convergent for a preconditioner that
// changes from one iteration to the next).  The first direction is the
// network's correction itself, so the first step is the learned initial
// guess with an optimal step length.  A one-workgroup kernel per iteration
// publishes ||r||, max |r| (the next scale) and the stop / stall decision:
// converged, non-finite, ||r|| grown past twice its start, or ||r|| not
// reduced by 10 % over the last 2 iterations (then the caller falls back to
// Jacobi-PCG, whose iterations cost a small fraction of a network
// application: the 3D network's first step cuts ||r||^2 about a hundredfold
// and the next ones leave it flat; one flat step is tolerated, as a
// Polak-Ribiere direction can recover on the next).  A network that does not fit the system
// (far outside what it was trained on) can make the flexible iteration
// diverge within a few steps, its residual growing by tens of orders of
// magnitude: hence the growth test, and the hand-over that drops a
// correction leaving the true residual above the start.
#include "gea_reduce.h"

namespace gea {

namespace {

template <int N>
__device__ __forceinline__ void store_part(double (&v)[N], double* part) {
  __shared__ double sh[N][kBlock / 64];
  Reducer<0u, N>::block(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < N; ++k) part[k * gridDim.x + blockIdx.x] = v[k];
}

// <z, r>, <z, r_old>
__global__ __launch_bounds__(kBlock) void k_fcg_dots(int n, const float* __restrict__ z,
                                                     const float* __restrict__ r,
                                                     const float* __restrict__ r_old,
                                                     double* part, const FcgScalars* sc) {
  if (sc->done) return;
  double v[2] = {0.0, 0.0};
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x) {
    const double zd = z[P];
    v[0] += zd * (double)r[P];
    v[1] += zd * (double)r_old[P];
  }
  store_part<2>(v, part);
}

// sum of the k-th value of n per-workgroup partials, fixed order, in every thread
__device__ __forceinline__ double sum_part(const double* part, int n, int k) {
  __shared__ double sh[1][kBlock / 64];
  double a[1] = {0.0};
  for (int b = threadIdx.x; b < n; b += kBlock) a[0] += part[k * n + b];
  Reducer<0u, 1>::block(a, sh);
  return a[0];
}

// beta from the dot partials; p = z + beta p_old; q = A p; partial <p, q>.
// Iteration 0 (ITER0): p = z (beta = 0, no previous direction), and the
// partials also carry <z, r> (no dot kernel before it); p is stored only for
// a later iteration (keep_p).  Cache-only stencil, used on 2D meshes.
template <int NDIM, bool ITER0>
__global__ __launch_bounds__(kBlock) void k_fcg_spmv(Geo G, int iter, const float* __restrict__ z,
                                                     const float* __restrict__ p_old,
                                                     float* __restrict__ p_new,
                                                     float* __restrict__ q,
                                                     const float* __restrict__ c,
                                                     const float* __restrict__ D,
                                                     const float* __restrict__ r, int keep_p,
                                                     const double* dots, int nd, double* part,
                                                     FcgScalars* sc) {
  if (sc->done) return;
  float beta = 0.f;
  if (!ITER0) {
    const double zr = sum_part(dots, nd, 0);
    const double zro = sum_part(dots, nd, 1);
    const double beta_d = (zr - zro) / sc->rz_prev[(iter + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->rz_prev[iter & 1] = zr;
    beta = (float)beta_d;
  }
  float kk[NDIM];
  for (int d = 0; d < NDIM; ++d) kk[d] = (float)(G.S[d] / G.h[d]);
  double acc[2] = {0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    int cc[NDIM];
    cell_coords<NDIM>(G, P, cc);
    auto pn = [&](int Q) { return ITER0 ? z[Q] : z[Q] + beta * p_old[Q]; };
    const float pp = pn(P), dp = D[P];
    float a = c[P] * pp;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int st = G.st[d];
      if (cc[d] + 1 < G.n[d]) a += 0.5f * (dp + D[P + st]) * kk[d] * (pp - pn(P + st));
      if (cc[d] > 0) a += 0.5f * (D[P - st] + dp) * kk[d] * (pp - pn(P - st));
    }
    if (keep_p) p_new[P] = pp;
    q[P] = a;
    acc[0] += (double)pp * (double)a;
    if (ITER0) acc[1] += (double)pp * (double)r[P];
  }
  if (ITER0) {
    store_part<2>(acc, part);
  } else {
    double pq[1] = {acc[0]};
    store_part<1>(pq, part);
  }
}

// k_fcg_spmv on a 3D mesh: 64x4 column tiles marching in z with the new
// direction formed on the tile and a one-cell halo in LDS, the next plane's
// loads in flight while a plane is computed.  Same formulas and order.
template <bool ITER0>
__global__ __launch_bounds__(kBlock) void k_fcg_spmv3(Geo G, int kc, int iter,
                                                      const float* __restrict__ z,
                                                      const float* __restrict__ p_old,
                                                      float* __restrict__ p_new,
                                                      float* __restrict__ q,
                                                      const float* __restrict__ c,
                                                      const float* __restrict__ D,
                                                      const float* __restrict__ r, int keep_p,
                                                      const double* dots, int nd, double* part,
                                                      FcgScalars* sc) {
  using St = Stage3<1, 4>;
  constexpr int HP = St::HP, HX = St::HX, NU = St::NU;
  __shared__ float sp[2][HP], sd[2][HP];
  if (sc->done) return;
  float beta = 0.f;
  if (!ITER0) {
    const double zr = sum_part(dots, nd, 0);
    const double zro = sum_part(dots, nd, 1);
    const double beta_d = (zr - zro) / sc->rz_prev[(iter + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->rz_prev[iter & 1] = zr;
    beta = (float)beta_d;
  }
  const float kx = (float)(G.S[0] / G.h[0]), ky = (float)(G.S[1] / G.h[1]),
              kz = (float)(G.S[2] / G.h[2]);
  const Col col = col_of3<4>(G, kc);
  const St st = stage3<1, 4>(G, col);
  const int nz = G.nz, pl = col.pl, qo = st.qo, ho = st.ho;
  // raw values of the plane in flight: staged z (and p_old), D; own c, r and
  // the own column's direction and D one plane up
  float fz[NU], fo[NU], fd[NU], fc, fr, fzu, fou, fdu;
  auto fetch = [&](int kk) {
    const int o = pl * kk, P = qo + o;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int Q = st.q[m] + o;
      fz[m] = z[Q];
      fo[m] = ITER0 ? 0.f : p_old[Q];
      fd[m] = D[Q];
    }
    const int Pu = kk + 1 < nz ? P + pl : P;
    fc = c[P];
    fr = ITER0 ? r[P] : 0.f;
    fzu = z[Pu];
    fou = ITER0 ? 0.f : p_old[Pu];
    fdu = D[Pu];
  };
  auto pn = [&](float zv, float ov) { return ITER0 ? zv : zv + beta * ov; };
  double acc[2] = {0.0, 0.0};
  float pm = 0.f, dm = 0.f;  // direction and D one plane down
  if (col.k0 > 0) {
    const int Q = qo + pl * (col.k0 - 1);
    pm = pn(z[Q], ITER0 ? 0.f : p_old[Q]);
    dm = D[Q];
  }
  fetch(col.k0);
  for (int k = col.k0; k < col.k1; ++k) {
    const int sl = k & 1;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      sp[sl][st.h[m]] = pn(fz[m], fo[m]);
      sd[sl][st.h[m]] = fd[m];
    }
    const float cP = fc, rP = fr, pu = pn(fzu, fou), du = fdu;
    fetch(k + 1 < col.k1 ? k + 1 : k);
    lds_barrier();
    const float pp = sp[sl][ho], dp = sd[sl][ho];
    float a = cP * pp;
    const int i = col.i, j = col.j;
    if (i + 1 < G.nx) a += 0.5f * (dp + sd[sl][ho + 1]) * kx * (pp - sp[sl][ho + 1]);
    if (i > 0) a += 0.5f * (sd[sl][ho - 1] + dp) * kx * (pp - sp[sl][ho - 1]);
    if (j + 1 < G.ny) a += 0.5f * (dp + sd[sl][ho + HX]) * ky * (pp - sp[sl][ho + HX]);
    if (j > 0) a += 0.5f * (sd[sl][ho - HX] + dp) * ky * (pp - sp[sl][ho - HX]);
    if (k + 1 < nz) a += 0.5f * (dp + du) * kz * (pp - pu);
    if (k > 0) a += 0.5f * (dm + dp) * kz * (pp - pm);
    pm = pp;
    dm = dp;
    if (col.act) {
      const int P = qo + pl * k;
      if (keep_p) p_new[P] = pp;
      q[P] = a;
      acc[0] += (double)pp * (double)a;
      if (ITER0) acc[1] += (double)pp * (double)rP;
    }
  }
  if (ITER0) {
    store_part<2>(acc, part);
  } else {
    double pq[1] = {acc[0]};
    store_part<1>(pq, part);
  }
}

// alpha = <z, r>/<p, q>; d += alpha p, r_old = r, r -= alpha q;
// partials ||r||^2 and max |r| (as a sum of per-workgroup maxima stored apart).
// Iteration 0 (ITER0): p = z, <z, r> from the direction kernel's partials,
// and d = alpha p (d needs no clearing; it is cleared here when the solve has
// already stopped).  The last iteration (LAST) keeps no r_old and, when
// res_part is set, also forms the partials <r, r/diag>, <r, r> of the
// residual the resumed Jacobi-PCG starts from (also when the solve had
// stopped before this iteration).
template <bool ITER0, bool LAST>
__global__ __launch_bounds__(kBlock) void k_fcg_update(int n, int iter, float* __restrict__ d,
                                                       const float* p,
                                                       float* __restrict__ r,
                                                       float* __restrict__ r_old,
                                                       const float* __restrict__ q,
                                                       const double* pq_part, int np,
                                                       double* part, FcgScalars* sc,
                                                       const float* __restrict__ dinv,
                                                       double* res_part) {
  bool step = !sc->done;
  float alpha = 0.f;
  if (step) {
    const double pq = sum_part(pq_part, np, 0);
    double zr = sc->rz_prev[iter & 1];
    if (ITER0) {
      zr = sum_part(pq_part, np, 1);
      if (blockIdx.x == 0 && threadIdx.x == 0) sc->rz_prev[0] = zr;
    }
    const double alpha_d = zr / pq;
    if (!isfinite(alpha_d) || alpha_d == 0.0) {
      // no usable step (e.g. a network that outputs nothing): stop as stalled,
      // leaving d and r untouched; every workgroup takes this same branch
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->status = 1;
        sc->done = 1;
      }
      step = false;
    }
    alpha = (float)alpha_d;
  }
  if (!step && !ITER0 && !(LAST && res_part)) return;
  __shared__ double sh[2][kBlock / 64];
  double v[2] = {0.0, 0.0};
  double w[2] = {0.0, 0.0};
  const bool res = LAST && res_part;
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x) {
    float rn = r[P];
    if (step) {
      if (ITER0)
        d[P] = alpha * p[P];
      else
        d[P] += alpha * p[P];
      const float ro = rn;
      if (!LAST) r_old[P] = ro;
      rn = ro - alpha * q[P];
      r[P] = rn;
      v[0] += (double)rn * (double)rn;
      v[1] = fmax(v[1], fabs((double)rn));
    } else if (ITER0) {
      d[P] = 0.f;
    }
    if (res) {
      const double rd = (double)rn;
      w[0] += rd * (double)(rn * dinv[P]);
      w[1] += rd * rd;
    }
  }
  if (step) {
    Reducer<0x2u, 2>::block(v, sh);
    if (threadIdx.x == 0) {
      part[blockIdx.x] = v[0];
      part[gridDim.x + blockIdx.x] = v[1];
    }
  }
  if (res) store_part<2>(w, res_part);
}

// Hand-over to Jacobi-PCG after several flexible steps: the residual of the
// flexible CG's correction taken afresh, r = r0 - A d with the inner
// system's FP32 operator, in place of the recurrence residual, and the
// resumed solve's set-up partials <r, r/diag>, <r, r>.  Flexible steps with
// poor directions (long steps that mostly cancel) leave a recurrence
// residual that has drifted far from the true one at FP32 rounding of d;
// resumed from it, the Jacobi-PCG would converge on the drift and leave it to
// the next refinement step.  (After a single step, r0 - alpha A z differs
// from r0 - A (alpha z) by rounding of terms no larger than r0 itself, and
// the last update's partials serve.)
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_fcg_handover(Geo G, Stencil<NDIM, float> K, int kc,
                                                         const float* __restrict__ d,
                                                         const float* __restrict__ r0,
                                                         const float* __restrict__ c,
                                                         const float* __restrict__ D,
                                                         const float* __restrict__ dinv,
                                                         float* __restrict__ r, double* part) {
  double w[4] = {0.0, 0.0, 0.0, 0.0};
  const Col col = col_of<NDIM>(G, kc);
  if (col.act) {  // a column walking up through z (A d as the refinement residual forms A x)
    ColumnA<NDIM, float> A{d, D};
    A.nz = G.n[NDIM - 1];
    A.pl = col.pl;
    int P = col.base + col.pl * col.k0;
    A.start(col, P);
    for (int k = col.k0; k < col.k1; ++k, P += col.pl) {
      const float r0p = r0[P], mp = dinv[P];
      const float rn = r0p - A.at(G, K, col, P, k, c);
      A.next();
      r[P] = rn;
      const double rd = (double)rn, r0d = (double)r0p;
      w[0] += rd * (double)(rn * mp);
      w[1] += rd * rd;
      w[2] += r0d * (double)(r0p * mp);
      w[3] += r0d * r0d;
    }
  }
  store_part<4>(w, part);
}

// One workgroup after the hand-over pass: keep the flexible CG's correction
// (<r, r/diag>, <r, r> of r = r0 - A d) or, when that residual is not finite
// or larger than r0, drop it (restart: d = 0, r = r0, and r0's sums); the
// chosen pair goes to pick[0], pick[1] for the resumed solve's set-up.
__global__ __launch_bounds__(kBlock) void k_fcg_pick(const double* part, int n, double* pick,
                                                     FcgScalars* sc) {
  __shared__ double sh[4][kBlock / 64];
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += kBlock)
    for (int k = 0; k < 4; ++k) a[k] += part[k * n + b];
  Reducer<0u, 4>::block(a, sh);
  if (threadIdx.x != 0) return;
  const bool keep = isfinite(a[0]) && isfinite(a[1]) && a[1] <= a[3];
  sc->restart = keep ? 0 : 1;
  pick[0] = keep ? a[0] : a[2];
  pick[1] = keep ? a[1] : a[3];
}

// d = 0, r = r0 where the pick dropped the flexible CG's correction
__global__ __launch_bounds__(kBlock) void k_fcg_restart(int n, float* __restrict__ d,
                                                        float* __restrict__ r,
                                                        const float* __restrict__ r0,
                                                        const FcgScalars* sc) {
  if (!sc->restart) return;
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x) {
    d[P] = 0.f;
    r[P] = r0[P];
  }
}

// One workgroup: ||r||^2 and max |r| from the update partials (or from the
// start kernel), stop / stall decision, next scale 1/s.
__global__ __launch_bounds__(kBlock) void k_fcg_check(const double* part, int n, int iter,
                                                      int init, const CgScalars* sys,
                                                      int max_iter, FcgScalars* sc) {
  __shared__ double sh[2][kBlock / 64];
  if (!init && sc->done) return;
  double a[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += kBlock) {
    a[0] += part[b];
    a[1] = fmax(a[1], part[n + b]);
  }
  Reducer<0x2u, 2>::block(a, sh);
  if (threadIdx.x != 0) return;
  if (init) {  // ||b||^2 and tolerance of the inner system as its set-up left them
    sc->bb = sys->bb;
    sc->tol2 = sys->tol2;
    sc->max_iter = max_iter;
    sc->status = 0;
    sc->rz_prev[0] = sc->rz_prev[1] = 1.0;
    for (int k = 0; k < 10; ++k) sc->hist[k] = a[0];
  }
  sc->rr = a[0];
  sc->iter = iter;
  sc->s = a[1];
  sc->inv_s = a[1] > 0 ? 1.0 / a[1] : 0.0;
  const double old = sc->hist[(iter + 8) % 10];  // ||r||^2 two iterations ago
  sc->hist[iter % 10] = a[0];
  int done = init && sys->done ? 1 : 0;  // nothing to solve (the refinement has converged)
  if (done) {
  } else if (!isfinite(a[0]) || !isfinite(a[1]) || a[0] > 4.0 * sc->bb) {
    sc->status = 1;  // stall (or divergence): fall back
    done = 1;
  } else if (a[0] <= sc->tol2 * sc->bb) {
    done = 1;
  } else if (iter >= 2 && a[0] > 0.81 * old) {
    sc->status = 1;
    done = 1;
  } else if (iter >= sc->max_iter) {
    sc->status = 2;
    done = 1;
  }
  sc->done = done;
}

// inner start: partials ||r||^2 and max |r| of r (= r32, set by the
// refinement residual), and (when r0 is set) its copy for the hand-over.
// d, the direction and r_old need no clearing: the first iteration writes d
// and reads neither of the others.
__global__ __launch_bounds__(kBlock) void k_fcg_start(int n, const float* __restrict__ r,
                                                      float* __restrict__ r0, double* part) {
  __shared__ double sh[2][kBlock / 64];
  double v[2] = {0.0, 0.0};
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x) {
    const float rf = r[P];
    if (r0) r0[P] = rf;
    const double rv = rf;
    v[0] += rv * rv;
    v[1] = fmax(v[1], fabs(rv));
  }
  Reducer<0x2u, 2>::block(v, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v[0];
    part[gridDim.x + blockIdx.x] = v[1];
  }
}

// ---- training pairs --------------------------------------------------------------

// partial max |r|
__global__ __launch_bounds__(kBlock) void k_maxabs(int n, const double* __restrict__ r, double* part) {
  __shared__ double sh[1][kBlock / 64];
  double v[1] = {0.0};
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x)
    v[0] = fmax(v[0], fabs(r[P]));
  Reducer<0x1u, 1>::block(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_maxabs_final(const double* part, int n, double* out) {
  __shared__ double sh[1][kBlock / 64];
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < n; b += kBlock) v[0] = fmax(v[0], part[b]);
  Reducer<0x1u, 1>::block(v, sh);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[0] > 0 ? 1.0 / v[0] : 0.0;
  }
}

// in_r = r0/s, in_a = c/diag, out_d = (x - x0)/s
__global__ __launch_bounds__(kBlock) void k_pair(int n, const double* __restrict__ r0,
                                                 const double* __restrict__ c,
                                                 const double* __restrict__ dinv,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ x0,
                                                 const double* __restrict__ s, float* in_r,
                                                 float* in_a, float* out_d) {
  const double is = s[1];
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x) {
    in_r[P] = (float)(r0[P] * is);
    in_a[P] = (float)(c[P] * dinv[P]);
    out_d[P] = (float)((x[P] - x0[P]) * is);
  }
}

}  // namespace

void fcg_start(hipStream_t s, const Geo& G, const FcgVectors& v, const CgScalars* sys,
               int max_iter, FcgScalars* sc) {
  const int gu = grid_for(G.nc);
  hipLaunchKernelGGL(k_fcg_start, dim3(gu), dim3(kBlock), 0, s, G.nc, (const float*)v.r, v.r0, v.part_u);
  hipLaunchKernelGGL(k_fcg_check, dim3(1), dim3(kBlock), 0, s, (const double*)v.part_u, gu, 0, 1,
                     sys, max_iter, sc);
}

int fcg_iteration_after_z(hipStream_t s, const Geo& G, const FcgVectors& v, int iter, bool last,
                          FcgScalars* sc) {
  const int gu = grid_for(G.nc);
  const dim3 gr(gu), bl(kBlock);
  const bool it0 = iter == 0;
  if (!it0)
    hipLaunchKernelGGL(k_fcg_dots, gr, bl, 0, s, G.nc, (const float*)v.z, (const float*)v.r,
                       (const float*)v.r_old, v.part_d, (const FcgScalars*)sc);
  const float* p_old = (iter & 1) ? v.p1 : v.p0;
  float* p_new = (iter & 1) ? v.p0 : v.p1;
  // iteration 0's direction is z itself: stored only for a later iteration
  const int keep_p = !(it0 && last);
  const float* p_upd = keep_p ? p_new : v.z;
  int ns = gu;  // partials of the direction kernel
  if (G.ndim == 2) {
    if (it0)
      hipLaunchKernelGGL((k_fcg_spmv<2, true>), gr, bl, 0, s, G, iter, (const float*)v.z, p_old, p_new, v.q,
                         v.c, v.D, (const float*)v.r, keep_p, (const double*)v.part_d, gu, v.part_s, sc);
    else
      hipLaunchKernelGGL((k_fcg_spmv<2, false>), gr, bl, 0, s, G, iter, (const float*)v.z, p_old, p_new, v.q,
                         v.c, v.D, (const float*)v.r, keep_p, (const double*)v.part_d, gu, v.part_s, sc);
  } else {
    const ZPlan zp = zplan3(G, 4, ZTile<3>::KC);
    ns = zp.blocks;
    if (it0)
      hipLaunchKernelGGL(k_fcg_spmv3<true>, dim3(zp.blocks), bl, 0, s, G, zp.kc, iter, (const float*)v.z, p_old,
                         p_new, v.q, v.c, v.D, (const float*)v.r, keep_p, (const double*)v.part_d, gu,
                         v.part_s, sc);
    else
      hipLaunchKernelGGL(k_fcg_spmv3<false>, dim3(zp.blocks), bl, 0, s, G, zp.kc, iter, (const float*)v.z, p_old,
                         p_new, v.q, v.c, v.D, (const float*)v.r, keep_p, (const double*)v.part_d, gu,
                         v.part_s, sc);
  }
#define GEA_UPD(I0, L)                                                                          \
  hipLaunchKernelGGL((k_fcg_update<I0, L>), gr, bl, 0, s, G.nc, iter, v.d, p_upd, v.r, v.r_old, \
                     (const float*)v.q, (const double*)v.part_s, ns, v.part_u, sc, v.dinv,       \
                     v.r0 ? nullptr : v.part_d)
  if (it0 && last) GEA_UPD(true, true);
  else if (it0) GEA_UPD(true, false);
  else if (last) GEA_UPD(false, true);
  else GEA_UPD(false, false);
#undef GEA_UPD
  hipLaunchKernelGGL(k_fcg_check, dim3(1), bl, 0, s, (const double*)v.part_u, gu, iter + 1, 0,
                     (const CgScalars*)nullptr, 0, sc);
  return last && !v.r0 ? gu : 0;
}

void fcg_handover(hipStream_t s, const Geo& G, const FcgVectors& v, const CgWork& w, int max_iter,
                  FcgScalars* sc) {
  const ZPlan zp = zplan(G);
  const int gu = zp.blocks, gc = grid_for(G.nc);
  if (G.ndim == 2) {
    const Stencil<2, float> K{{(float)(G.S[0] / G.h[0]), (float)(G.S[1] / G.h[1])}};
    hipLaunchKernelGGL(k_fcg_handover<2>, dim3(gu), dim3(kBlock), 0, s, G, K, zp.kc, (const float*)v.d,
                       (const float*)v.r0, v.c, v.D, v.dinv, v.r, v.part_d);
  } else {
    const Stencil<3, float> K{{(float)(G.S[0] / G.h[0]), (float)(G.S[1] / G.h[1]), (float)(G.S[2] / G.h[2])}};
    hipLaunchKernelGGL(k_fcg_handover<3>, dim3(gu), dim3(kBlock), 0, s, G, K, zp.kc, (const float*)v.d,
                       (const float*)v.r0, v.c, v.D, v.dinv, v.r, v.part_d);
  }
  // (part_u is free once the last check has run)
  hipLaunchKernelGGL(k_fcg_pick, dim3(1), dim3(kBlock), 0, s, (const double*)v.part_d, gu, v.part_u, sc);
  hipLaunchKernelGGL(k_fcg_restart, dim3(gc), dim3(kBlock), 0, s, G.nc, v.d, v.r, (const float*)v.r0,
                     (const FcgScalars*)sc);
  cg_resume_scalars(s, v.part_u, 1, w, max_iter);
}

void pair_outputs(hipStream_t s, const Geo& G, const double* r0, const double* c,
                  const double* dinv, const double* x, const double* x0, double* part,
                  double* s_out, float* in_r, float* in_a, float* out_d) {
  const int gu = grid_for(G.nc);
  hipLaunchKernelGGL(k_maxabs, dim3(gu), dim3(kBlock), 0, s, G.nc, r0, part);
  hipLaunchKernelGGL(k_maxabs_final, dim3(1), dim3(kBlock), 0, s, (const double*)part, gu, s_out);
  hipLaunchKernelGGL(k_pair, dim3(gu), dim3(kBlock), 0, s, G.nc, r0, c, dinv, x, x0,
                     (const double*)s_out, in_r, in_a, out_d);
}

}  // namespace gea
