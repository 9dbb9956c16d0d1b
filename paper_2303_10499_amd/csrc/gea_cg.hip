// gea_cg.hip -- Jacobi-preconditioned conjugate gradients on the matrix-free
// pressure operator of Step 3 (GEA, Sec. 3, eq. p_prime_sd re-derived):
//     (A x)_i = c_i x_i + sum_f w_f (x_i - x_nb),  w_f = (D_P + D_N)/2 S_f/d_f,
// homogeneous Neumann on walls.  Face weights are formed on the fly from
// the cell coefficient D (two FP64 coefficient arrays instead of ndim face
// arrays).  Two kernels per iteration, each ending in a single-pass grid
// reduction whose last workgroup writes the CG scalars to device memory:
//   spmv:   p = z + beta p_old  (z = r/diag, on the fly, own cell and
//           neighbours), q = A p, <p, q>            -> alpha
//   update: x += alpha p, r -= alpha q, <r, z>, <r, r> -> beta, convergence
// so the host never waits inside a solve; it polls the done flag every few
// iterations.  The same kernels, instantiated on float with FP64 dot
// accumulation, are the inner solver of the mixed-precision refinement.
#include "gea_reduce.h"

namespace gea {

namespace {

template <int NDIM, typename T>
struct Stencil {
  T k[NDIM];  // S_d / h_d in the working precision
};

template <int NDIM, typename T>
__device__ __forceinline__ T apply_A_at(const Geo& G, const Stencil<NDIM, T>& K, const int* c,
                                        int P, const T* __restrict__ cc, const T* __restrict__ D,
                                        const T* __restrict__ x) {
  const T xp = x[P];
  const T dp = D[P];
  T acc = cc[P] * xp;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    const int st = G.st[d];
    if (c[d] + 1 < G.n[d]) acc += T(0.5) * (dp + D[P + st]) * K.k[d] * (xp - x[P + st]);
    if (c[d] > 0) acc += T(0.5) * (D[P - st] + dp) * K.k[d] * (xp - x[P - st]);
  }
  return acc;
}

// r = b - A x, p_old = 0, beta = 0; scalars rz, rr, bb and the done flag
template <int NDIM, typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init(Geo G, Stencil<NDIM, T> K, CgVectors<T> v,
                                                    double tol2, int max_iter, double* partials,
                                                    CgScalars* sc) {
  double red[3] = {0.0, 0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    const T r = v.b[P] - apply_A_at<NDIM, T>(G, K, c, P, v.c, v.D, v.x);
    v.r[P] = r;
    v.p0[P] = T(0);
    const double rd = (double)r;
    red[0] += rd * (double)(r * v.dinv[P]);
    red[1] += rd * rd;
    red[2] += (double)v.b[P] * (double)v.b[P];
  }
  double out[3];
  if (Reducer<0u, 3>::grid(red, partials, &sc->ticket[0], out) && threadIdx.x == 0) {
    sc->rz = out[0];
    sc->rr = out[1];
    sc->bb = out[2];
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->tol2 = tol2;
    sc->iter = 0;
    sc->max_iter = max_iter;
    const bool finite = isfinite(out[0]) && isfinite(out[1]) && isfinite(out[2]);
    sc->status = finite ? 0 : -5;
    sc->done = (!finite || out[1] <= tol2 * out[2]) ? 1 : 0;
  }
}

// p = r/diag + beta p_old (own cell and neighbours), q = A p, alpha = rz/<p,q>
template <int NDIM, typename T>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(Geo G, Stencil<NDIM, T> K, CgVectors<T> v,
                                                    const T* __restrict__ p_old,
                                                    T* __restrict__ p_new, double* partials,
                                                    CgScalars* sc) {
  if (__hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const T beta = (T)sc->beta;
  const T* __restrict__ r = v.r;
  const T* __restrict__ dinv = v.dinv;
  const T* __restrict__ D = v.D;
  double red[1] = {0.0};
  GEA_FOR_CELLS(P, G) {
    int c[NDIM];
    cell_coords<NDIM>(G, P, c);
    auto pn = [&](int Q) { return r[Q] * dinv[Q] + beta * p_old[Q]; };
    const T pp = pn(P);
    const T dp = D[P];
    T acc = v.c[P] * pp;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int st = G.st[d];
      if (c[d] + 1 < G.n[d]) acc += T(0.5) * (dp + D[P + st]) * K.k[d] * (pp - pn(P + st));
      if (c[d] > 0) acc += T(0.5) * (D[P - st] + dp) * K.k[d] * (pp - pn(P - st));
    }
    p_new[P] = pp;
    v.q[P] = acc;
    red[0] += (double)pp * (double)acc;
  }
  double out[1];
  if (Reducer<0u, 1>::grid(red, partials, &sc->ticket[0], out) && threadIdx.x == 0) {
    sc->alpha = sc->rz / out[0];
    if (!isfinite(sc->alpha)) {
      sc->status = -5;
      __hip_atomic_store(&sc->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// x += alpha p, r -= alpha q, beta = <r,z>_new/<r,z>, stop test on ||r||
template <int NDIM, typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(Geo G, CgVectors<T> v,
                                                      const T* __restrict__ p_cur,
                                                      double* partials, CgScalars* sc) {
  if (__hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const T alpha = (T)sc->alpha;
  double red[2] = {0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    v.x[P] += alpha * p_cur[P];
    const T r = v.r[P] - alpha * v.q[P];
    v.r[P] = r;
    const double rd = (double)r;
    red[0] += rd * (double)(r * v.dinv[P]);
    red[1] += rd * rd;
  }
  double out[2];
  if (Reducer<0u, 2>::grid(red, partials, &sc->ticket[0], out) && threadIdx.x == 0) {
    sc->beta = out[0] / sc->rz;
    sc->rz = out[0];
    sc->rr = out[1];
    sc->iter += 1;
    int done = 0;
    if (!isfinite(out[0]) || !isfinite(out[1])) {
      sc->status = -5;
      done = 1;
    } else if (out[1] <= sc->tol2 * sc->bb) {
      done = 1;
    } else if (sc->iter >= sc->max_iter) {
      sc->status = -4;
      done = 1;
    }
    __hip_atomic_store(&sc->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_apply_A(Geo G, Stencil<NDIM, double> K,
                                                    const double* c, const double* D,
                                                    const double* x, double* y) {
  GEA_FOR_CELLS(P, G) {
    int cc[NDIM];
    cell_coords<NDIM>(G, P, cc);
    y[P] = apply_A_at<NDIM, double>(G, K, cc, P, c, D, x);
  }
}

// ---- mixed precision ----------------------------------------------------------

// FP64 outer residual r = b - A x; its FP32 copy becomes the inner right-hand
// side and initial inner residual (inner x = 0, inner p_old = 0).  Reduces
// ||r||^2, ||b||^2 in FP64 for the outer test and <r32, r32/diag>, ||r32||^2
// for the inner start.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_residual64(Geo G, Stencil<NDIM, double> K,
                                                       const double* __restrict__ c,
                                                       const double* __restrict__ D,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ r64,
                                                       CgVectors<float> v32, double tol2,
                                                       double inner_tol2, int inner_max,
                                                       double* partials, CgScalars* sc64,
                                                       CgScalars* sc32) {
  double red[4] = {0.0, 0.0, 0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    int cc[NDIM];
    cell_coords<NDIM>(G, P, cc);
    const double r = b[P] - apply_A_at<NDIM, double>(G, K, cc, P, c, D, x);
    r64[P] = r;
    const float rf = (float)r;
    v32.r[P] = rf;
    v32.x[P] = 0.0f;
    v32.p0[P] = 0.0f;
    red[0] += r * r;
    red[1] += b[P] * b[P];
    red[2] += (double)rf * (double)(rf * v32.dinv[P]);
    red[3] += (double)rf * (double)rf;
  }
  double out[4];
  if (Reducer<0u, 4>::grid(red, partials, &sc64->ticket[0], out) && threadIdx.x == 0) {
    sc64->rr = out[0];
    sc64->bb = out[1];
    sc64->tol2 = tol2;
    const bool finite = isfinite(out[0]) && isfinite(out[1]);
    sc64->status = finite ? 0 : -5;
    sc64->done = (!finite || out[0] <= tol2 * out[1]) ? 1 : 0;
    sc32->rz = out[2];
    sc32->rr = out[3];
    sc32->bb = out[3];
    sc32->alpha = 0.0;
    sc32->beta = 0.0;
    sc32->tol2 = inner_tol2;
    sc32->iter = 0;
    sc32->max_iter = inner_max;
    sc32->status = 0;
    __hip_atomic_store(&sc32->done, (sc64->done || out[3] == 0.0) ? 1 : 0, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(kBlock) void k_cast_coeffs(int n, const double* c, const double* D,
                                                        const double* dinv, float* c32, float* D32,
                                                        float* dinv32) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x) {
    c32[P] = (float)c[P];
    D32[P] = (float)D[P];
    dinv32[P] = (float)dinv[P];
  }
}

__global__ __launch_bounds__(kBlock) void k_add_correction(int n, double* x, const float* dx) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x)
    x[P] += (double)dx[P];
}

template <int NDIM, typename T>
Stencil<NDIM, T> stencil(const Geo& G) {
  Stencil<NDIM, T> K;
  for (int d = 0; d < NDIM; ++d) K.k[d] = (T)(G.S[d] / G.h[d]);
  return K;
}

template <typename T>
void cg_init_t(hipStream_t s, const Geo& G, const CgVectors<T>& v, double tol2, int max_iter,
               double* partials, CgScalars* sc) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL((k_cg_init<2, T>), grid, block, 0, s, G, stencil<2, T>(G), v, tol2, max_iter, partials, sc);
  else
    hipLaunchKernelGGL((k_cg_init<3, T>), grid, block, 0, s, G, stencil<3, T>(G), v, tol2, max_iter, partials, sc);
}

template <typename T>
void cg_spmv_t(hipStream_t s, const Geo& G, const CgVectors<T>& v, int parity, double* partials,
               CgScalars* sc) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  const T* p_old = parity ? v.p1 : v.p0;
  T* p_new = parity ? v.p0 : v.p1;
  if (G.ndim == 2)
    hipLaunchKernelGGL((k_cg_spmv<2, T>), grid, block, 0, s, G, stencil<2, T>(G), v, p_old, p_new, partials, sc);
  else
    hipLaunchKernelGGL((k_cg_spmv<3, T>), grid, block, 0, s, G, stencil<3, T>(G), v, p_old, p_new, partials, sc);
}

template <typename T>
void cg_update_t(hipStream_t s, const Geo& G, const CgVectors<T>& v, int parity,
                 double* partials, CgScalars* sc) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  const T* p_new = parity ? v.p0 : v.p1;
  if (G.ndim == 2)
    hipLaunchKernelGGL((k_cg_update<2, T>), grid, block, 0, s, G, v, p_new, partials, sc);
  else
    hipLaunchKernelGGL((k_cg_update<3, T>), grid, block, 0, s, G, v, p_new, partials, sc);
}

}  // namespace

void launch_cg_init(hipStream_t s, const Geo& G, const CgVectors<double>& v, double tol,
                        int max_iter, double* partials, CgScalars* sc) {
  cg_init_t<double>(s, G, v, tol * tol, max_iter, partials, sc);
}

void launch_cg_spmv(hipStream_t s, const Geo& G, const CgVectors<double>& v, int parity,
                    double* partials, CgScalars* sc) {
  cg_spmv_t<double>(s, G, v, parity, partials, sc);
}

void launch_cg_update(hipStream_t s, const Geo& G, const CgVectors<double>& v, int parity,
                      double* partials, CgScalars* sc) {
  cg_update_t<double>(s, G, v, parity, partials, sc);
}

void launch_cg32_spmv(hipStream_t s, const Geo& G, const CgVectors<float>& v, int parity,
                      double* partials, CgScalars* sc) {
  cg_spmv_t<float>(s, G, v, parity, partials, sc);
}

void launch_cg32_update(hipStream_t s, const Geo& G, const CgVectors<float>& v, int parity,
                        double* partials, CgScalars* sc) {
  cg_update_t<float>(s, G, v, parity, partials, sc);
}

void launch_apply_A(hipStream_t s, const Geo& G, const double* c, const double* D,
                    const double* x, double* y) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_apply_A<2>, grid, block, 0, s, G, stencil<2, double>(G), c, D, x, y);
  else
    hipLaunchKernelGGL(k_apply_A<3>, grid, block, 0, s, G, stencil<3, double>(G), c, D, x, y);
}

void launch_residual64(hipStream_t s, const Geo& G, const double* c, const double* D,
                           const double* b, const double* x, double* r64,
                           const CgVectors<float>& v32, double tol, double inner_tol,
                           int inner_max, double* partials, CgScalars* sc64, CgScalars* sc32) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_residual64<2>, grid, block, 0, s, G, stencil<2, double>(G), c, D, b, x, r64, v32, tol * tol, inner_tol * inner_tol, inner_max, partials, sc64, sc32);
  else
    hipLaunchKernelGGL(k_residual64<3>, grid, block, 0, s, G, stencil<3, double>(G), c, D, b, x, r64, v32, tol * tol, inner_tol * inner_tol, inner_max, partials, sc64, sc32);
}

void launch_cast_coeffs(hipStream_t s, const Geo& G, const double* c, const double* D,
                        const double* dinv, float* c32, float* D32, float* dinv32) {
  hipLaunchKernelGGL(k_cast_coeffs, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, c, D, dinv, c32, D32, dinv32);
}

void launch_add_correction(hipStream_t s, const Geo& G, double* x, const float* dx) {
  hipLaunchKernelGGL(k_add_correction, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, x, dx);
}

}  // namespace gea
