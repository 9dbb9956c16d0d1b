// gea_cg.hip -- Jacobi-preconditioned conjugate gradients on the matrix-free
// pressure operator of Step 3 (GEA, Sec. 3, eq. p_prime_sd re-derived):
//     (A x)_i = c_i x_i + sum_f w_f (x_i - x_nb),  w_f = (D_P + D_N)/2 S_f/d_f,
// homogeneous Neumann on walls; face weights are formed on the fly from the
// cell coefficient D.
//
// One iteration is two kernels:
//   spmv:   p = r/diag + beta p_old on the tile and its halo, q = A p, <p, q>
//   update: x += alpha p, r -= alpha q, <r, r/diag>, <r, r>
// Dot products: every workgroup reduces its values (wave xor-shuffles, then
// LDS) and stores one partial per workgroup.  The next kernel, which needs
// the scalar, sums all partials of the previous kernel at its start, every
// workgroup in the same fixed order, so all workgroups hold bitwise the same
// alpha/beta and no grid-wide fence or atomic is needed (an agent-scope
// release in every workgroup costs more than the stream kernel it ends).
// The stop test (||r|| <= tol ||b||, iteration cap, non-finite) is taken by
// the spmv kernel from the partials of the update before it; workgroup 0
// publishes scalars and the done flag, which later launches of a batch read
// to return at once.  A one-workgroup check kernel closes each batch so the
// host sees the latest residual.
//
// The spmv kernel stages, per workgroup, a 64 x 8 (3D) or 256 x 1 (2D)
// column tile of p and D with a one-cell halo in an LDS ring of three
// planes and marches along z, so every value is loaded once per workgroup;
// workgroups are mapped so that each XCD (own L2) works on a contiguous
// block of tiles.  The same kernels instantiated on float, with FP64 dot
// accumulation, are the inner solver of the mixed-precision refinement.
#include "gea_reduce.h"

namespace gea {

namespace {

constexpr int kTX3 = 64, kTY3 = 4, kKC3 = 16;  // 3D tile and z chunk
constexpr int kTX2 = 256, kKC2 = 16;           // 2D row segment and z chunk

template <int NDIM, typename T>
struct Stencil {
  T k[NDIM];  // S_d / h_d in the working precision
};

// sum of n partials, identical in every workgroup; result in all threads
template <int N>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int n,
                                             double (&out)[N]) {
  __shared__ double sh[N][kBlock / 64];
  double a[N];
#pragma unroll
  for (int k = 0; k < N; ++k) a[k] = 0.0;
#pragma unroll 8
  for (int b = threadIdx.x; b < n; b += kBlock) {
#pragma unroll
    for (int k = 0; k < N; ++k) a[k] += part[k * n + b];
  }
  Reducer<0u, N>::block(a, sh);
#pragma unroll
  for (int k = 0; k < N; ++k) out[k] = a[k];
}

// store this workgroup's N sums at part[k * gridDim.x + blockIdx.x]
template <int N>
__device__ __forceinline__ void store_partials(double (&v)[N], double* __restrict__ part) {
  __shared__ double sh[N][kBlock / 64];
  Reducer<0u, N>::block(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) part[k * gridDim.x + blockIdx.x] = v[k];
  }
}

__device__ __forceinline__ int load_done(CgScalars* sc) {
  return __hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

// Stop test from the update partials of the previous iteration.  Returns
// true (in every workgroup) when the solve ends here; workgroup 0 then
// publishes the result.  Otherwise beta is returned through *beta_out.
__device__ __forceinline__ bool spmv_prologue(const double* u_part, int nu, int iter,
                                              CgScalars* sc, double* beta_out) {
  double s[2];
  sum_partials<2>(u_part, nu, s);
  const double rz = s[0], rr = s[1];
  int stop = 0, status = 0;
  if (!isfinite(rz) || !isfinite(rr)) {
    stop = 1;
    status = -5;
  } else if (rr <= sc->tol2 * sc->bb) {
    stop = 1;
  } else if (iter >= sc->max_iter) {
    stop = 1;
    status = -4;
  }
  if (stop) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->rz = rz;
      sc->rr = rr;
      sc->iter = iter;
      sc->status = status;
      __hip_atomic_store(&sc->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
  }
  const double rz_old = sc->rzs[(iter + 1) & 1];
  *beta_out = iter == 0 ? 0.0 : rz / rz_old;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rzs[iter & 1] = rz;
    sc->rz = rz;
    sc->rr = rr;
    sc->iter = iter;
  }
  return false;
}

// A x at the cells of a column walking up through z: x and D of the planes
// below, at and above the current one stay in registers, x/y neighbours
// come from the caches.  The terms are summed in the order of apply_A_at.
template <int NDIM, typename T>
struct ColumnA {
  const T* x;
  const T* D;
  T xm, xc, xp, dm, dc, dp;
  int nz, pl;
  __device__ void start(const Col& c, int P) {
    xm = c.k0 > 0 ? x[P - pl] : T(0);
    dm = c.k0 > 0 ? D[P - pl] : T(0);
    xc = x[P];
    dc = D[P];
  }
  // A x at cell P of plane k (loads the plane above first).  Neighbour loads
  // are clamped to the cell itself where the neighbour does not exist, and
  // the wall tests are selects, so no branch separates the plane's loads.
  __device__ T at(const Geo& G, const Stencil<NDIM, T>& K, const Col& c, int P, int k,
                  const T* __restrict__ cc) {
    constexpr int Z = NDIM - 1;
    const bool up = k + 1 < nz;
    const int Pu = up ? P + pl : P;
    const T xu = x[Pu], du = D[Pu], cP = cc[P];
    T x_hi[Z > 0 ? Z : 1], x_lo[Z > 0 ? Z : 1], d_hi[Z > 0 ? Z : 1], d_lo[Z > 0 ? Z : 1];
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int st = G.st[d], q = coord(c, d);
      const int Ph = q + 1 < G.n[d] ? P + st : P, Pl = q > 0 ? P - st : P;
      x_hi[d] = x[Ph];
      d_hi[d] = D[Ph];
      x_lo[d] = x[Pl];
      d_lo[d] = D[Pl];
    }
    xp = up ? xu : T(0);
    dp = up ? du : T(0);
    T acc = cP * xc;
#pragma unroll
    for (int d = 0; d < Z; ++d) {
      const int q = coord(c, d);
      acc = q + 1 < G.n[d] ? acc + T(0.5) * (dc + d_hi[d]) * K.k[d] * (xc - x_hi[d]) : acc;
      acc = q > 0 ? acc + T(0.5) * (d_lo[d] + dc) * K.k[d] * (xc - x_lo[d]) : acc;
    }
    if (up) acc += T(0.5) * (dc + dp) * K.k[Z] * (xc - xp);
    if (k > 0) acc += T(0.5) * (dm + dc) * K.k[Z] * (xc - xm);
    return acc;
  }
  __device__ void next() {
    xm = xc;
    dm = dc;
    xc = xp;
    dc = dp;
  }
};

// r = b - A x, p_old = 0; partials (<r, r/diag>, <r, r>) -> u_part, <b, b> -> b_part
// (column tiles: one partial per workgroup of the z-marching grid)
template <int NDIM, typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init(Geo G, Stencil<NDIM, T> K, CgVectors<T> v,
                                                    int kc, double* u_part, double* b_part) {
  double red[2] = {0.0, 0.0};
  double bb[1] = {0.0};
  const Col c = col_of<NDIM>(G, kc);
  if (c.act) {
    ColumnA<NDIM, T> A{v.x, v.D};
    A.nz = G.n[NDIM - 1];
    A.pl = c.pl;
    int P = c.base + c.pl * c.k0;
    A.start(c, P);
    for (int k = c.k0; k < c.k1; ++k, P += c.pl) {
      const T bp = v.b[P], di = v.dinv[P];
      const T r = bp - A.at(G, K, c, P, k, v.c);
      A.next();
      v.r[P] = r;
      v.p0[P] = T(0);
      const double rd = (double)r;
      red[0] += rd * (double)(r * di);
      red[1] += rd * rd;
      bb[0] += (double)bp * (double)bp;
    }
  }
  store_partials<2>(red, u_part);
  store_partials<1>(bb, b_part);
}

// one workgroup: reduce the partials of the last update (or of init) and
// publish residual and stop test; with init != 0 also ||b||^2 and the setup
__global__ __launch_bounds__(kBlock) void k_cg_check(const double* u_part, int nu,
                                                     const double* b_part, int init, double tol2,
                                                     int max_iter, int iter, CgScalars* sc) {
  if (!init && load_done(sc)) return;
  double s[2];
  sum_partials<2>(u_part, nu, s);
  double bbv[1] = {0.0};
  if (init) sum_partials<1>(b_part, nu, bbv);
  if (threadIdx.x != 0) return;
  if (init) {
    sc->bb = bbv[0];
    sc->tol2 = tol2;
    sc->max_iter = max_iter;
    sc->status = 0;
    sc->alpha = 0.0;
    sc->rzs[0] = s[0];
    sc->rzs[1] = s[0];
  }
  const double bb = sc->bb;
  sc->rz = s[0];
  sc->rr = s[1];
  sc->iter = iter;
  int done = 0;
  if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(bb)) {
    sc->status = -5;
    done = 1;
  } else if (s[1] <= sc->tol2 * bb) {
    done = 1;
  } else if (iter >= sc->max_iter) {
    sc->status = -4;
    done = 1;
  }
  __hip_atomic_store(&sc->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 3D: p = r/diag + beta p_old, q = A p, partial <p, q>, on a 64 x 8 column
// tile marching over 16 planes.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_spmv3(Geo G, Stencil<3, T> K, CgVectors<T> v,
                                                     const T* __restrict__ p_old,
                                                     T* __restrict__ p_new, int iter,
                                                     const double* u_part, int nu,
                                                     double* s_part, CgScalars* sc) {
  constexpr int TX = kTX3, TY = kTY3, KC = kKC3;
  constexpr int HX = TX + 2, HY = TY + 2, HP = HX * HY;
  constexpr int RPT = TX * TY / kBlock;
  constexpr int HPT = (HP + kBlock - 1) / kBlock;  // staged cells per thread and plane
  // Plane kk+1 is loaded into registers while plane kk-1 is computed.  FP32:
  // a ring of 4 planes, where the slot a plane is written to was last read
  // two planes earlier, before the previous barrier, so one barrier per plane
  // suffices.  FP64: a ring of 3 (4 would not leave room for 4 workgroups per
  // CU) and a second barrier before the next write.
  constexpr int NS = sizeof(T) == 8 ? 3 : 4;
  __shared__ T sp[NS][HP];
  __shared__ T sd[NS][HP];
  if (load_done(sc)) return;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int b = xcd_block();
  const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
  const int i0 = tx * TX, j0 = ty * TY, k0 = tz * KC;
  const int k1 = min(k0 + KC, nz);
  const T kx = K.k[0], ky = K.k[1], kz = K.k[2];
  // global index of each staged cell of this thread in plane 0 (-1: outside)
  int qh[HPT];
#pragma unroll
  for (int u = 0; u < HPT; ++u) {
    const int h = threadIdx.x + kBlock * u;
    const int hx = h % HX, hy = h / HX;
    const int i = i0 + hx - 1, j = j0 + hy - 1;
    qh[u] = (h < HP && i >= 0 && i < nx && j >= 0 && j < ny) ? i + nx * j : -1;
  }
  const int plane = nx * ny;
  // staged values: z = r/diag, the old direction and D (p = z + beta p_old
  // is formed when a plane is written to LDS, once beta is known)
  T pz[HPT], po[HPT], pd[HPT];
  auto fetch = [&](int kk) {
#pragma unroll
    for (int u = 0; u < HPT; ++u) {
      pz[u] = T(0);
      po[u] = T(0);
      pd[u] = T(0);
      if (kk >= 0 && kk < nz && qh[u] >= 0) {
        const int Q = qh[u] + plane * kk;
        pz[u] = v.r[Q] * v.dinv[Q];
        po[u] = p_old[Q];
        pd[u] = v.D[Q];
      }
    }
  };
  fetch(k0 - 1);  // in flight while the previous kernel's partials are summed
  double beta_d = 0.0;
  if (spmv_prologue(u_part, nu, iter, sc, &beta_d)) return;
  const T beta = (T)beta_d;
  double acc = 0.0;
  for (int kk = k0 - 1; kk <= k1; ++kk) {
    const int sl = (kk + NS) % NS;
#pragma unroll
    for (int u = 0; u < HPT; ++u) {
      const int h = threadIdx.x + kBlock * u;
      if (h < HP) {
        sp[sl][h] = pz[u] + beta * po[u];
        sd[sl][h] = pd[u];
      }
    }
    if (kk + 1 <= k1) fetch(kk + 1);
    __syncthreads();
    const int k = kk - 1;
    if (k >= k0 && k < k1) {
      const int sm = (k - 1 + NS) % NS, s0 = (k + NS) % NS, sP = (k + 1) % NS;
#pragma unroll
      for (int m = 0; m < RPT; ++m) {
        const int t = threadIdx.x + kBlock * m;
        const int lx = t % TX, ly = t / TX;
        const int i = i0 + lx, j = j0 + ly;
        if (i < nx && j < ny) {
          const int h = (lx + 1) + HX * (ly + 1);
          const int P = i + nx * (j + ny * k);
          const T pp = sp[s0][h], dp = sd[s0][h];
          T a = v.c[P] * pp;
          if (i + 1 < nx) a += T(0.5) * (dp + sd[s0][h + 1]) * kx * (pp - sp[s0][h + 1]);
          if (i > 0) a += T(0.5) * (sd[s0][h - 1] + dp) * kx * (pp - sp[s0][h - 1]);
          if (j + 1 < ny) a += T(0.5) * (dp + sd[s0][h + HX]) * ky * (pp - sp[s0][h + HX]);
          if (j > 0) a += T(0.5) * (sd[s0][h - HX] + dp) * ky * (pp - sp[s0][h - HX]);
          if (k + 1 < nz) a += T(0.5) * (dp + sd[sP][h]) * kz * (pp - sp[sP][h]);
          if (k > 0) a += T(0.5) * (sd[sm][h] + dp) * kz * (pp - sp[sm][h]);
          p_new[P] = pp;
          v.q[P] = a;
          acc += (double)pp * (double)a;
        }
      }
    }
    if (NS == 3) __syncthreads();
  }
  double red[1] = {acc};
  store_partials<1>(red, s_part);
}

// 2D: p = r/diag + beta p_old, q = A p, partial <p, q>.  A workgroup owns a
// 256-cell row segment and marches it over 16 rows of z; each wave owns 64
// consecutive cells.  The rows below and above a cell stay in registers and
// x-neighbours come from the neighbouring lanes (the first and last lane of a
// wave also load the cell just beyond the wave), so the kernel needs neither
// LDS nor barriers.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_spmv2(Geo G, Stencil<2, T> K, CgVectors<T> v,
                                                     const T* __restrict__ p_old,
                                                     T* __restrict__ p_new, int iter,
                                                     const double* u_part, int nu,
                                                     double* s_part, CgScalars* sc) {
  constexpr int TX = kTX2, KC = kKC2;
  static_assert(TX == kBlock, "one cell of the row segment per thread");
  if (load_done(sc)) return;
  const int nx = G.nx, nz = G.nz;
  const int ntx = (nx + TX - 1) / TX;
  const int b = xcd_block();
  const int tx = b % ntx, tz = b / ntx;
  const int lane = threadIdx.x & 63;
  const int i = tx * TX + threadIdx.x;
  const int k0 = tz * KC, k1 = min(k0 + KC, nz);
  const T kx = K.k[0], kz = K.k[1];
  const bool in = i < nx;
  // the cell beyond the wave that an edge lane supplies (lane 0: left, lane 63: right)
  const int ie = lane == 0 ? i - 1 : (lane == 63 ? i + 1 : -1);
  const bool edge = ie >= 0 && ie < nx;
  // raw values of row kk (z = r/diag, old direction, D), own cell and edge cell
  struct Raw {
    T z, o, d, ze, oe, de;
  };
  auto fetch = [&](int kk) {
    Raw w{T(0), T(0), T(0), T(0), T(0), T(0)};
    if (kk >= 0 && kk < nz) {
      if (in) {
        const int Q = i + nx * kk;
        w.z = v.r[Q] * v.dinv[Q];
        w.o = p_old[Q];
        w.d = v.D[Q];
      }
      if (edge) {
        const int Q = ie + nx * kk;
        w.ze = v.r[Q] * v.dinv[Q];
        w.oe = p_old[Q];
        w.de = v.D[Q];
      }
    }
    return w;
  };
  // rows k0-1 .. k0+PD in flight while the previous kernel's partials are
  // summed; afterwards row k+PD+1 is requested while row k is computed
  constexpr int PD = 3;
  Raw ring[PD + 1];
  const Raw wm = fetch(k0 - 1);
#pragma unroll
  for (int w = 0; w <= PD; ++w) ring[w] = fetch(k0 + w);
  double beta_d = 0.0;
  if (spmv_prologue(u_part, nu, iter, sc, &beta_d)) return;
  const T beta = (T)beta_d;
  T pm = wm.z + beta * wm.o, dm = wm.d;
  T pc = ring[0].z + beta * ring[0].o, dc = ring[0].d;
  T pec = ring[0].ze + beta * ring[0].oe, dec = ring[0].de;
  double acc = 0.0;
#pragma unroll
  for (int it = 0; it < KC; ++it) {
    const int k = k0 + it;
    if (k >= k1) break;
    const Raw& wn = ring[(it + 1) % (PD + 1)];
    const T pn = wn.z + beta * wn.o, dn = wn.d;
    const T pen = wn.ze + beta * wn.oe, den = wn.de;
    // slot of row k is free now: request row k+PD+1 into it
    ring[it % (PD + 1)] = (k + PD + 1 <= k1) ? fetch(k + PD + 1) : Raw{T(0), T(0), T(0), T(0), T(0), T(0)};
    T pl = __shfl_up(pc, 1, 64), pr = __shfl_down(pc, 1, 64);
    T dl = __shfl_up(dc, 1, 64), dr = __shfl_down(dc, 1, 64);
    if (lane == 0) {
      pl = pec;
      dl = dec;
    }
    if (lane == 63) {
      pr = pec;
      dr = dec;
    }
    if (in) {
      const int P = i + nx * k;
      T a = v.c[P] * pc;
      if (i + 1 < nx) a += T(0.5) * (dc + dr) * kx * (pc - pr);
      if (i > 0) a += T(0.5) * (dl + dc) * kx * (pc - pl);
      if (k + 1 < nz) a += T(0.5) * (dc + dn) * kz * (pc - pn);
      if (k > 0) a += T(0.5) * (dm + dc) * kz * (pc - pm);
      p_new[P] = pc;
      v.q[P] = a;
      acc += (double)pc * (double)a;
    }
    pm = pc;
    dm = dc;
    pc = pn;
    dc = dn;
    pec = pen;
    dec = den;
  }
  double red[1] = {acc};
  store_partials<1>(red, s_part);
}

// alpha = <r,z>/<p,q> from the spmv partials; x += alpha p, r -= alpha q;
// partials (<r, r/diag>, <r, r>)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(Geo G, CgVectors<T> v,
                                                      const T* __restrict__ p_cur, int iter,
                                                      const double* s_part, int ns,
                                                      double* u_part, CgScalars* sc) {
  if (load_done(sc)) return;
  double pq[1];
  sum_partials<1>(s_part, ns, pq);
  const double alpha_d = sc->rzs[iter & 1] / pq[0];
  if (!isfinite(alpha_d)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->status = -5;
      sc->iter = iter;
      __hip_atomic_store(&sc->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->alpha = alpha_d;
  const T alpha = (T)alpha_d;
  double red[2] = {0.0, 0.0};
  GEA_FOR_CELLS(P, G) {
    v.x[P] += alpha * p_cur[P];
    const T r = v.r[P] - alpha * v.q[P];
    v.r[P] = r;
    const double rd = (double)r;
    red[0] += rd * (double)(r * v.dinv[P]);
    red[1] += rd * rd;
  }
  store_partials<2>(red, u_part);
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

// FP64 outer residual r = b - A x and its FP32 copy as the inner right-hand
// side / initial inner residual (inner x = 0, inner p_old = 0).  Partials:
// outer (||r||^2, ||b||^2) -> o_part; inner (<r32, r32/diag>, ||r32||^2) ->
// i_part (the slot the inner solver's first spmv reads).
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_residual64(Geo G, Stencil<NDIM, double> K,
                                                       const double* __restrict__ c,
                                                       const double* __restrict__ D,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ r64,
                                                       CgVectors<float> v32, int kc,
                                                       double* o_part, double* i_part) {
  double ro[2] = {0.0, 0.0};
  double ri[2] = {0.0, 0.0};
  const Col col = col_of<NDIM>(G, kc);
  if (col.act) {
    ColumnA<NDIM, double> A{x, D};
    A.nz = G.n[NDIM - 1];
    A.pl = col.pl;
    int P = col.base + col.pl * col.k0;
    A.start(col, P);
    for (int k = col.k0; k < col.k1; ++k, P += col.pl) {
      const double bp = b[P];
      const float di = v32.dinv[P];
      const double r = bp - A.at(G, K, col, P, k, c);
      A.next();
      r64[P] = r;
      const float rf = (float)r;
      v32.r[P] = rf;
      v32.x[P] = 0.0f;
      v32.p0[P] = 0.0f;
      ro[0] += r * r;
      ro[1] += bp * bp;
      ri[0] += (double)rf * (double)(rf * di);
      ri[1] += (double)rf * (double)rf;
    }
  }
  store_partials<2>(ro, o_part);
  store_partials<2>(ri, i_part);
}

// one workgroup: outer stop test and the inner solver's setup
__global__ __launch_bounds__(kBlock) void k_residual_check(const double* o_part,
                                                           const double* i_part, int n,
                                                           double tol2, double inner_tol2,
                                                           int inner_max, CgScalars* sc64,
                                                           CgScalars* sc32) {
  double o[2], in[2];
  sum_partials<2>(o_part, n, o);
  sum_partials<2>(i_part, n, in);
  if (threadIdx.x != 0) return;
  sc64->rr = o[0];
  sc64->bb = o[1];
  sc64->tol2 = tol2;
  const bool finite = isfinite(o[0]) && isfinite(o[1]);
  sc64->status = finite ? 0 : -5;
  const int outer_done = (!finite || o[0] <= tol2 * o[1]) ? 1 : 0;
  __hip_atomic_store(&sc64->done, outer_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  sc32->rz = in[0];
  sc32->rr = in[1];
  sc32->bb = in[1];
  sc32->rzs[0] = in[0];
  sc32->rzs[1] = in[0];
  sc32->alpha = 0.0;
  // inner tolerance: what the outer residual still needs (with a factor 0.1
  // for the FP32 solve's own error), never looser than 0.5 nor tighter than
  // the configured inner tolerance
  double it2 = inner_tol2;
  if (o[0] > 0.0 && finite) {
    const double need = 0.1 * sqrt(tol2 * o[1] / o[0]);
    const double it = fmax(sqrt(inner_tol2), fmin(0.5, need));
    it2 = it * it;
  }
  sc32->tol2 = it2;
  sc32->iter = 0;
  sc32->max_iter = inner_max;
  sc32->status = 0;
  __hip_atomic_store(&sc32->done, (outer_done || in[1] == 0.0) ? 1 : 0, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
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

__global__ __launch_bounds__(kBlock) void k_sub(int n, const double* b, double* y) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x)
    y[P] = b[P] - y[P];
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

}  // namespace

int spmv_grid(const Geo& G) {
  if (G.ndim == 3)
    return ((G.nx + kTX3 - 1) / kTX3) * ((G.ny + kTY3 - 1) / kTY3) * ((G.nz + kKC3 - 1) / kKC3);
  return ((G.nx + kTX2 - 1) / kTX2) * ((G.nz + kKC2 - 1) / kKC2);
}

// Partials in the slot iteration 0 reads were written by the set-up kernel
// (the initial residual, one per workgroup of the column-tile grid); later
// slots by the update kernel (one per workgroup of its grid-stride grid).
int partials_for(const Geo& G, int iter) { return iter == 0 ? zplan(G).blocks : grid_for(G.nc); }

template <typename T>
void cg_init(hipStream_t s, const Geo& G, const CgVectors<T>& v, const CgWork& w, double tol,
             int max_iter) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL((k_cg_init<2, T>), dim3(zp.blocks), dim3(kBlock), 0, s, G, stencil<2, T>(G), v, zp.kc, w.u[1], w.b);
  else
    hipLaunchKernelGGL((k_cg_init<3, T>), dim3(zp.blocks), dim3(kBlock), 0, s, G, stencil<3, T>(G), v, zp.kc, w.u[1], w.b);
  hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(kBlock), 0, s, (const double*)w.u[1], zp.blocks,
                     (const double*)w.b, 1, tol * tol, max_iter, 0, w.sc);
}

template <typename T>
void cg_spmv(hipStream_t s, const Geo& G, const CgVectors<T>& v, int iter, const CgWork& w) {
  const T* p_old = (iter & 1) ? v.p1 : v.p0;
  T* p_new = (iter & 1) ? v.p0 : v.p1;
  const int gu = partials_for(G, iter);
  const double* up = w.u[(iter + 1) & 1];
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_cg_spmv2<T>, dim3(spmv_grid(G)), dim3(kBlock), 0, s, G, stencil<2, T>(G), v, p_old, p_new, iter, up, gu, w.s, w.sc);
  else
    hipLaunchKernelGGL(k_cg_spmv3<T>, dim3(spmv_grid(G)), dim3(kBlock), 0, s, G, stencil<3, T>(G), v, p_old, p_new, iter, up, gu, w.s, w.sc);
}

template <typename T>
void cg_update(hipStream_t s, const Geo& G, const CgVectors<T>& v, int iter, const CgWork& w) {
  const T* p_cur = (iter & 1) ? v.p0 : v.p1;
  hipLaunchKernelGGL(k_cg_update<T>, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, v, p_cur, iter,
                     (const double*)w.s, spmv_grid(G), w.u[iter & 1], w.sc);
}

void cg_check(hipStream_t s, const Geo& G, int iter, const CgWork& w) {
  // the residual after `iter` completed iterations sits in the partials of
  // update iter-1, i.e. slot (iter + 1) & 1
  hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(kBlock), 0, s, (const double*)w.u[(iter + 1) & 1],
                     partials_for(G, iter), (const double*)nullptr, 0, 0.0, 0, iter, w.sc);
}

template void cg_init<double>(hipStream_t, const Geo&, const CgVectors<double>&, const CgWork&, double, int);
template void cg_init<float>(hipStream_t, const Geo&, const CgVectors<float>&, const CgWork&, double, int);
template void cg_spmv<double>(hipStream_t, const Geo&, const CgVectors<double>&, int, const CgWork&);
template void cg_spmv<float>(hipStream_t, const Geo&, const CgVectors<float>&, int, const CgWork&);
template void cg_update<double>(hipStream_t, const Geo&, const CgVectors<double>&, int, const CgWork&);
template void cg_update<float>(hipStream_t, const Geo&, const CgVectors<float>&, int, const CgWork&);

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
                       const CgVectors<float>& v32, double tol, double inner_tol, int inner_max,
                       double* o_part, const CgWork& w32, CgScalars* sc64) {
  const ZPlan zp = zplan(G);
  const int gu = zp.blocks;
  const dim3 grid(gu), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_residual64<2>, grid, block, 0, s, G, stencil<2, double>(G), c, D, b, x, r64, v32, zp.kc, o_part, w32.u[1]);
  else
    hipLaunchKernelGGL(k_residual64<3>, grid, block, 0, s, G, stencil<3, double>(G), c, D, b, x, r64, v32, zp.kc, o_part, w32.u[1]);
  hipLaunchKernelGGL(k_residual_check, dim3(1), block, 0, s, (const double*)o_part,
                     (const double*)w32.u[1], gu, tol * tol, inner_tol * inner_tol, inner_max,
                     sc64, w32.sc);
}

void launch_cast_coeffs(hipStream_t s, const Geo& G, const double* c, const double* D,
                        const double* dinv, float* c32, float* D32, float* dinv32) {
  hipLaunchKernelGGL(k_cast_coeffs, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, c, D, dinv, c32, D32, dinv32);
}

void launch_add_correction(hipStream_t s, const Geo& G, double* x, const float* dx) {
  hipLaunchKernelGGL(k_add_correction, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, x, dx);
}

void launch_sub(hipStream_t s, const Geo& G, const double* b, double* y) {
  hipLaunchKernelGGL(k_sub, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, b, y);
}

}  // namespace gea
