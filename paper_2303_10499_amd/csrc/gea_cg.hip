// gea_cg.hip -- Jacobi-preconditioned conjugate gradients on the matrix-free
// pressure operator of Step 3 (GEA, Sec. 3, eq. p_prime_sd re-derived):
//     (A x)_i = c_i x_i + sum_f w_f (x_i - x_nb),  w_f = (D_P + D_N)/2 S_f/d_f,
// homogeneous Neumann on walls; face weights are formed on the fly from the
// cell coefficient D.
//
// One iteration is one stencil kernel:
//   iteration j:  r_j = r_{j-1} - alpha q_{j-1} and p_j = r_j/diag + beta p_{j-1}
//                 on the tile and its halo, x += alpha p_{j-1} on the own cells,
//                 q_j = A p_j, and partials <p,q>, <q,z>, <q,q/diag>, <r,r>,
//                 <q,r>, <q,q>, <r,z> (z = r/diag) of iteration j
//   scalars j:    alpha_j = <r,z>/<p,q>; <r,z> and ||r||^2 after the update
//                 r - alpha_j q follow without another pass over the vectors,
//                 <r - a q, M (r - a q)> = <r,z> - 2a<q,z> + a^2<q,Mq> (and the
//                 same for ||r||^2), each from directly summed values of the
//                 iterate before, so rounding does not accumulate; beta_j, the
//                 stop test (||r|| <= tol ||b||, iteration cap, non-finite).
// This is Jacobi-PCG with the same iterates; it reads and writes 11 arrays
// per iteration instead of 14 (separate operator and update kernels) and
// needs no grid-wide reduction inside the stencil kernel.  The residual,
// direction, A p and the partials are double buffered by iteration parity
// (the stencil kernel reads the old values with halo while writing the new
// ones).  The scalars of iteration j are formed at the start of iteration
// j+1's kernel by every workgroup, each summing j's partials in workgroup
// order (so all take bitwise the same values; workgroup 0 publishes them);
// the host enqueues iterations in batches and ends each with a
// one-workgroup scalar kernel that forms the last iteration's scalars for it
// to read, and the batch's next iteration kernel takes them from there.
// When the scalars show the solve converged, that iteration kernel only
// applies the last x update and marks its launch as the last (later launches
// of the batch return at once); the scalar kernel at the batch's end then
// sets the done flag, on which later launches return at once.  (One scalar
// kernel an iteration cost 3.5 us on the 30 us FP32 iteration of the 2D
// benchmark mesh.)  Every workgroup reads all 7 ns partials, so the fold
// costs L2 traffic that grows as ns^2: it is used up to 512 workgroups (the
// 2D mesh's FP32 and both 3D grids: 14.7 MB a launch at 512, +2.7 us on the
// 79 us 3D FP32 iteration); larger grids (the 2D FP64 one, 1024) keep one
// scalar kernel an iteration (folded there the iteration took 73-77 us
// instead of 68).  Dot products: every workgroup reduces its values (wave
// xor-shuffles, then LDS) and stores one partial; the sums over partials
// run in workgroup order, so results are bitwise reproducible.
//
// The 3D stencil kernel stages, per workgroup, a 64 x 4 column tile of p, D,
// r and 1/diag with a one-cell halo in an LDS ring of planes and marches
// along z, so every value is loaded once per workgroup; workgroups are
// mapped so that each XCD (own L2) works on a contiguous block of tiles.  The
// same kernels instantiated on float, with FP64 dot accumulation, are the
// inner solver of the mixed-precision refinement.
#include "gea_reduce.h"

namespace gea {

namespace {

constexpr int kTX3 = 64, kTY3 = 8;  // 3D tile
constexpr int kFoldMaxParts = 512;   // largest iteration grid that folds its scalars
// z chunk of the 3D iteration kernel
template <typename T>
constexpr int kKC3 = sizeof(T) == 8 ? 64 : 32;
constexpr int kTX2 = 256;  // 2D row segment
// z chunk of the 2D iteration kernel
template <typename T>
constexpr int kKC2 = sizeof(T) == 8 ? 16 : 32;

// sum of n partials, identical in every workgroup; result in all threads.
// (Unrolling keeps each thread's order of additions: U only trades
// registers for loads in flight.  LDSB: barriers that order LDS only.)
template <int N, int U = 8, bool LDSB = false>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int n,
                                             double (&out)[N]) {
  __shared__ double sh[N][kBlock / 64];
  double a[N];
#pragma unroll
  for (int k = 0; k < N; ++k) a[k] = 0.0;
#pragma unroll U
  for (int b = threadIdx.x; b < n; b += kBlock) {
#pragma unroll
    for (int k = 0; k < N; ++k) a[k] += part[k * n + b];
  }
  if constexpr (LDSB)
    Reducer<0u, N>::block_lds(a, sh);
  else
    Reducer<0u, N>::block(a, sh);
#pragma unroll
  for (int k = 0; k < N; ++k) out[k] = a[k];
}

// store this workgroup's N sums at part[k * gridDim.x + blockIdx.x]
template <int N, int NT = kBlock>
__device__ __forceinline__ void store_partials(double (&v)[N], double* __restrict__ part) {
  __shared__ double sh[N][NT / 64];
  Reducer<0u, N, NT>::block(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) part[k * gridDim.x + blockIdx.x] = v[k];
  }
}

__device__ __forceinline__ int load_done(CgScalars* sc) {
  return __hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A kernel enqueued behind an inner solve whose outcome the host has not
// read yet acts only once that solve is done (gate->done); with the gate
// unset (null) it always acts.
__device__ __forceinline__ bool gate_closed(const CgScalars* gate) {
  return gate != nullptr &&
         __hip_atomic_load(&gate->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// the partials of iteration `iter` within the parity-buffered set
__device__ __forceinline__ double* iter_part(double* part, int ns, int iter) {
  return part + (iter & 1) * 7L * ns;
}

// alpha, the residual after the update, beta and the stop test of iteration
// `iter` from its ns partials (see the file header); every thread of every
// workgroup that forms them gets the same values
struct StepScalars {
  double alpha, beta, rz, rr;
  int fin, status;
  bool bad;
};
__device__ __forceinline__ StepScalars step_scalars(const double* part, int ns, int iter,
                                                    const CgScalars* sc) {
  double s[7];
  // (few registers, and the iteration kernels' first loads stay in flight)
  sum_partials<7, 2, true>(part, ns, s);
  const double pq = s[0], qz = s[1], qmq = s[2], rr0 = s[3], qr = s[4], qq = s[5], rz0 = s[6];
  StepScalars o;
  o.alpha = rz0 / pq;
  o.rz = rz0 - 2.0 * o.alpha * qz + o.alpha * o.alpha * qmq;
  o.rr = fmax(rr0 - 2.0 * o.alpha * qr + o.alpha * o.alpha * qq, 0.0);
  o.beta = o.rz / rz0;
  o.bad = !isfinite(o.alpha) || !isfinite(o.rz) || !isfinite(o.rr) || !isfinite(o.beta);
  o.fin = 0;
  o.status = 0;
  if (o.bad) {
    o.status = -5;
  } else if (o.rr <= sc->tol2 * sc->bb) {
    o.fin = 1;
  } else if (iter + 1 >= sc->max_iter) {
    o.fin = 1;
    o.status = -4;
  }
  return o;
}

// (one thread) the scalars of iteration `iter` for the host and the next
// kernels
__device__ __forceinline__ void publish(const StepScalars& o, int iter, CgScalars* sc) {
  sc->iter = iter + 1;
  sc->alpha = o.alpha;
  sc->beta = o.beta;
  sc->rz = o.rz;
  sc->rr = o.rr;
  sc->status = o.status;
  sc->fin = o.fin;
}

// Where an iteration kernel stands in its batch: the partial sets, this
// launch's iteration index and whether it forms the previous iteration's
// scalars itself
struct CgStep {
  double* part;
  int ns;
  int iter;
  int fold;
};

// Whether an iteration kernel has work: false once the solve is done or an
// earlier launch of its batch ended it.  Within a launch only done_iter
// changes (workgroup 0 sets it to this launch's index), so every workgroup
// takes the same branch here and in step_take; the done flag is set by the
// scalar kernel at the end of the batch.
__device__ __forceinline__ bool step_live(const CgStep& st, CgScalars* sc) {
  if (load_done(sc)) return false;
  const int di = __hip_atomic_load(&sc->done_iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return !(di >= 0 && di < st.iter);
}

// The update an iteration kernel applies (alpha, beta of the iteration
// before it) and whether it is the solve's last; false: return at once.
// The kernels call it after issuing their first loads.
template <typename T>
__device__ __forceinline__ bool step_take(const CgStep& st, CgScalars* sc, T& alpha, T& beta,
                                          int& fin) {
  if (st.fold) {
    const StepScalars o = step_scalars(iter_part(st.part, st.ns, st.iter - 1), st.ns, st.iter - 1, sc);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      publish(o, st.iter - 1, sc);
      if (o.bad)  // a non-finite value ends the solve without this update
        __hip_atomic_store(&sc->done_iter, st.iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (o.bad) return false;
    alpha = (T)o.alpha;
    beta = (T)o.beta;
    fin = o.fin;
  } else {
    alpha = (T)sc->alpha;
    beta = (T)sc->beta;
    fin = sc->fin;
  }
  return true;
}

// (after the last x update) later launches of the batch return at once;
// corrected: that update also corrected the outer iterate
__device__ __forceinline__ void step_last(const CgStep& st, CgScalars* sc, bool corrected) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (corrected) sc->corrected = 1;
    __hip_atomic_store(&sc->done_iter, st.iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The last x update at cell P: x += alpha p, or, for an inner solve of the
// refinement, the outer iterate takes the updated inner one (rounded to T as
// a stored x would be) and x is left as it was (the next refinement
// residual clears it).
template <typename T>
__device__ __forceinline__ void last_update(const CgIter<T>& v, int P, T alpha) {
  const T xn = v.x[P] + alpha * v.p_in[P];
  if (v.xo)
    v.xo[P] += (double)xn;
  else
    v.x[P] = xn;
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
      const double rd = (double)r;
      red[0] += rd * (double)(r * di);
      red[1] += rd * rd;
      bb[0] += (double)bp * (double)bp;
    }
  }
  store_partials<2>(red, u_part);
  store_partials<1>(bb, b_part);
}

// one workgroup: set-up of a solve from the set-up kernel's partials
// (<r, z>, ||r||^2 and ||b||^2 of the initial residual)
__global__ __launch_bounds__(kBlock) void k_cg_start(const double* u_part, int nu,
                                                     const double* b_part, double tol2,
                                                     int max_iter, CgScalars* sc) {
  double s[2], bbv[1];
  sum_partials<2>(u_part, nu, s);
  sum_partials<1>(b_part, nu, bbv);
  if (threadIdx.x != 0) return;
  const double bb = bbv[0];
  sc->bb = bb;
  sc->tol2 = tol2;
  sc->max_iter = max_iter;
  sc->alpha = 0.0;
  sc->beta = 0.0;
  sc->fin = 0;
  sc->done_iter = -1;
  sc->corrected = 0;
  sc->rz = s[0];
  sc->rr = s[1];
  sc->rr0 = s[1];
  sc->iter = 0;
  int done = 0, status = 0;
  if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(bb)) {
    done = 1;
    status = -5;
  } else if (s[1] <= tol2 * bb) {
    done = 1;
  } else if (max_iter <= 0) {
    done = 1;
    status = -4;
  }
  sc->status = status;
  __hip_atomic_store(&sc->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// one workgroup after iteration `iter`: alpha, the residual after the
// update, beta and the stop test (see the file header)
__global__ __launch_bounds__(kBlock) void k_cg_scalars(double* part, int ns, int iter,
                                                       CgScalars* sc) {
  if (load_done(sc)) return;
  if (sc->done_iter >= 0) {  // a launch of the batch ended the solve
    if (threadIdx.x == 0) __hip_atomic_store(&sc->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const StepScalars o = step_scalars(iter_part(part, ns, iter), ns, iter, sc);
  if (threadIdx.x != 0) return;
  publish(o, iter, sc);
  if (o.bad) __hip_atomic_store(&sc->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the seven partials of an iteration: <p,q>, <q,z>, <q,q/diag>, <r,r>, <q,r>,
// <q,q>, <r,z> of one cell
template <typename T>
__device__ __forceinline__ void iter_dots(double (&acc)[7], T p, T a, T r, T m) {
  const T z = r * m, mq = a * m;
  acc[0] += (double)p * (double)a;
  acc[1] += (double)a * (double)z;
  acc[2] += (double)a * (double)mq;
  acc[3] += (double)r * (double)r;
  acc[4] += (double)a * (double)r;
  acc[5] += (double)a * (double)a;
  acc[6] += (double)r * (double)z;
}

// Loads and stores of the iteration's streams that no other workgroup reads
// in the same pass (the own cells' x and c; the new r, p, A p, x) marked
// non-temporal, so that they do not push out of the L2 the halo rows that
// neighbouring workgroups re-read.  3D kernel: 151.8 -> 145.5 us (FP64) and
// 82.0 -> 79.2 us (FP32) on 8.4 M cells.  2D: the FP64 kernel gains (72.4 ->
// 68.1 us on 4.2 M cells); the FP32 one, whose 185 MB of vectors stay in
// the 256 MB last-level cache between iterations, loses (29.9 -> 35.9 us),
// so it keeps ordinary accesses.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// 3D iteration kernel: a workgroup owns a 64 x 8 column tile and marches it
// through a chunk of planes (32 in FP32, 64 in FP64, whose loads carry twice
// the bytes).  Thread t stages its two own cells (t % 64, t / 64) and
// (t % 64, t / 64 + 4) and, for t < 148, one halo cell of the tile; each
// staged plane is loaded into registers ahead (two planes in FP32, one in
// FP64: old residual, old A p, old direction, D, 1/diag), turned into the new residual
// and direction, and p and D are written to an LDS ring.  The own cells'
// new residual and x update are stored there, and their residual and 1/diag
// stay in the thread's registers for the dot products of the plane, which
// is computed one step later.
// CD: D is v.Dc in every cell (no D array is read), and 1/diag is formed
// from c (the diagonal is c plus Dc S/h for each face inside the mesh, summed
// in the order the energy system's set-up sums it), so c is staged in place
// of 1/diag and no 1/diag array is read
template <typename T, bool CD>
__global__ __launch_bounds__(kBlock) void k_cg_iter3(Geo G, Stencil<3, T> K, CgIter<T> v,
                                                     CgStep stp, CgScalars* sc) {
  constexpr int TX = kTX3, TY = kTY3, KC = kKC3<T>;
  constexpr int HX = TX + 2, HY = TY + 2, HP = HX * HY;
  constexpr int RPT = TX * TY / kBlock;  // own cells per thread
  constexpr int NH = HP - TX * TY;       // halo cells of a plane
  static_assert(TX == 64 && RPT * kBlock == TX * TY && NH <= kBlock, "tile layout");
  // Plane kk+1 is loaded into registers while plane kk-1 is computed.  FP32:
  // a ring of 4 planes, where the slot a plane is written to was last read
  // two planes earlier, before the previous barrier, so one barrier per plane
  // suffices.  FP64: a ring of 3 and a second barrier before the next write.
  constexpr int NS = sizeof(T) == 8 ? 3 : 4;
  __shared__ T sp[NS][HP];  // direction
  __shared__ T sd[NS][HP];  // D
  if (!step_live(stp, sc)) return;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int b = xcd_block();
  const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
  const int i0 = tx * TX, j0 = ty * TY, k0 = tz * KC;
  const int k1 = min(k0 + KC, nz);
  const int plane = nx * ny;
  const int lx = threadIdx.x % TX, ly0 = threadIdx.x / TX;
  const int i = i0 + lx;
  int jo[RPT];
  bool in[RPT];
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    jo[m] = j0 + ly0 + m * (kBlock / TX);
    in[m] = i < nx && jo[m] < ny;
  }
  const T kx = K.k[0], ky = K.k[1], kz = K.k[2];
  const T wx = v.Dc * kx, wy = v.Dc * ky, wz = v.Dc * kz;  // (CD) face weights
  // staged cells of this thread: [0, RPT) its own cells, [RPT] halo cell e = t
  // (row 0, row TY+1, then the two side columns); global index in plane 0,
  // clamped into the mesh (values staged for cells outside it are never read,
  // and unconditional loads are not waited for where branches would merge)
  constexpr int NU = RPT + 1;
  int qh[NU], hh[NU];
  // faces inside the mesh of each staged cell (CD): x+, x-, y+, y- in bits 0-3
  int fm[NU];
  auto faces = [&](int gi, int gj) {
    return (gi + 1 < nx ? 1 : 0) | (gi > 0 ? 2 : 0) | (gj + 1 < ny ? 4 : 0) | (gj > 0 ? 8 : 0);
  };
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    hh[m] = (lx + 1) + HX * (jo[m] - j0 + 1);
    qh[m] = (i < nx ? i : nx - 1) + nx * (jo[m] < ny ? jo[m] : ny - 1);
    fm[m] = faces(i, jo[m]);
  }
  {
    const int e = threadIdx.x;
    int hx = 0, hy = 0;
    if (e < HX) {
      hx = e;
    } else if (e < 2 * HX) {
      hx = e - HX;
      hy = TY + 1;
    } else {
      const int e2 = e - 2 * HX;
      hy = 1 + e2 / 2;
      hx = (e2 & 1) ? HX - 1 : 0;
    }
    const int gi = i0 + hx - 1, gj = j0 + hy - 1;
    hh[RPT] = hx + HX * hy;
    fm[RPT] = faces(gi, gj);
    // threads without a halo cell load their own cell again (a cache hit)
    qh[RPT] = e < NH ? (gi < 0 ? 0 : (gi >= nx ? nx - 1 : gi)) + nx * (gj < 0 ? 0 : (gj >= ny ? ny - 1 : gj))
                     : qh[0];
  }
  const bool halo = threadIdx.x < NH;
  // raw values of a plane in flight: old residual, old A p, old direction,
  // D, 1/diag of the staged cells, x and c of the own cells.  FP32 keeps two
  // planes in flight (FP64 one, whose registers would cost occupancy): the
  // set a plane is consumed from is refilled with the plane PF further on.
  struct Raw {
    T r[NU], q[NU], p[NU], d[NU], m[NU], x[RPT], c[RPT];
  };
  constexpr int PF = sizeof(T) == 8 ? 1 : 2;
  T alpha = T(0), beta = T(0);  // (from step_take, after the first loads)
  auto fetch = [&](Raw& f, int kk) {
    const int o = plane * (kk < 0 ? 0 : (kk >= nz ? nz - 1 : kk));
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int Q = qh[u] + o;
      f.r[u] = v.r_in[Q];
      f.q[u] = v.q_in[Q];
      f.p[u] = v.p_in[Q];
      f.d[u] = CD ? v.Dc : v.D[Q];
      f.m[u] = CD ? v.c[Q] : v.dinv[Q];  // (CD: c, turned into 1/diag when staged)
      if (u < RPT) {  // own cell: x for its update, c for the operator
        f.x[u] = ld_stream<true>(&v.x[Q]);
        if (!CD) f.c[u] = ld_stream<true>(&v.c[Q]);
      }
    }
  };
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // own cells' new residual, 1/diag and c of the last staged plane (the
  // compute step reads no global memory: a load issued after the next
  // planes' loads would wait for all of them)
  T r_own[RPT], m_own[RPT], c_own[RPT];
#pragma unroll
  for (int m = 0; m < RPT; ++m) r_own[m] = m_own[m] = c_own[m] = T(0);
  // stage plane kk from f, refill f with plane kk + PF, compute plane kk - 1
  auto plane_step = [&](Raw& f, int kk) {
    const int sl = (kk + NS) % NS;
    T r_prev[RPT], m_prev[RPT], c_prev[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      r_prev[m] = r_own[m];
      m_prev[m] = m_own[m];
      c_prev[m] = c_own[m];
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (u == RPT && !halo) break;
      const T rn = f.r[u] - alpha * f.q[u];
      T mv = f.m[u];
      if constexpr (CD) {
        T dg = f.m[u];
        dg += (fm[u] & 1) ? wx : T(0);
        dg += (fm[u] & 2) ? wx : T(0);
        dg += (fm[u] & 4) ? wy : T(0);
        dg += (fm[u] & 8) ? wy : T(0);
        dg += kk + 1 < nz ? wz : T(0);
        dg += kk > 0 ? wz : T(0);
        mv = T(1) / dg;
      }
      sp[sl][hh[u]] = rn * mv + beta * f.p[u];
      sd[sl][hh[u]] = f.d[u];
      if (u < RPT) {
        r_own[u] = rn;
        m_own[u] = mv;
        c_own[u] = CD ? f.m[u] : f.c[u];
        if (kk >= k0 && kk < k1 && in[u]) {
          const int Q = qh[u] + plane * kk;
          st_stream<true>(rn, &v.r_out[Q]);
          st_stream<true>(f.x[u] + alpha * f.p[u], &v.x[Q]);
        }
      }
    }
    // FP32: refilled at every plane (the last two refills reload plane k1,
    // an L2 hit), so that on every path the wait for one set leaves the
    // other in flight
    if (PF == 2 || kk + 1 <= k1) fetch(f, min(kk + PF, k1));
    lds_barrier();
    const int k = kk - 1;
    if (k >= k0 && k < k1) {
      const int sM = (k - 1 + NS) % NS, s0 = (k + NS) % NS, sP = (k + 1) % NS;
#pragma unroll
      for (int m = 0; m < RPT; ++m) {
        if (!in[m]) continue;
        const int j = jo[m];
        const int h = hh[m];
        const int P = i + nx * (j + ny * k);
        const T pp = sp[s0][h], dp = sd[s0][h];
        T a = c_prev[m] * pp;
        if (i + 1 < nx) a += T(0.5) * (dp + sd[s0][h + 1]) * kx * (pp - sp[s0][h + 1]);
        if (i > 0) a += T(0.5) * (sd[s0][h - 1] + dp) * kx * (pp - sp[s0][h - 1]);
        if (j + 1 < ny) a += T(0.5) * (dp + sd[s0][h + HX]) * ky * (pp - sp[s0][h + HX]);
        if (j > 0) a += T(0.5) * (sd[s0][h - HX] + dp) * ky * (pp - sp[s0][h - HX]);
        if (k + 1 < nz) a += T(0.5) * (dp + sd[sP][h]) * kz * (pp - sp[sP][h]);
        if (k > 0) a += T(0.5) * (sd[sM][h] + dp) * kz * (pp - sp[sM][h]);
        st_stream<true>(pp, &v.p_out[P]);
        st_stream<true>(a, &v.q_out[P]);
        iter_dots(acc, pp, a, r_prev[m], m_prev[m]);
      }
    }
    if (NS == 3) lds_barrier();
  };
  Raw f0, f1;
  fetch(f0, k0 - 1);
  if (PF == 2) {
    // all of the first set's loads ahead of the second's, as in the loop
    __builtin_amdgcn_sched_barrier(0);
    fetch(f1, k0);
  }
  // the scalars, while the first planes' loads are in flight
  int fin;
  if (!step_take(stp, sc, alpha, beta, fin)) return;
  if (fin) {  // the solve has converged: its last x update only
#pragma unroll
    for (int m = 0; m < RPT; ++m)
      if (in[m])
        for (int k = k0; k < k1; ++k) {
          const int P = i + nx * (jo[m] + ny * k);
          last_update(v, P, alpha);
        }
    step_last(stp, sc, v.xo != nullptr);
    return;
  }
  if (PF == 2) {
    int kk = k0 - 1;
    for (; kk + 1 <= k1; kk += 2) {
      plane_step(f0, kk);
      plane_step(f1, kk + 1);
    }
    if (kk <= k1) plane_step(f0, kk);
  } else {
    for (int kk = k0 - 1; kk <= k1; ++kk) plane_step(f0, kk);
  }
  store_partials<7>(acc, iter_part(stp.part, stp.ns, stp.iter));
}

// 2D iteration kernel: a workgroup owns a 256-cell row segment and marches it
// over a chunk of rows of z (32 in FP32, 16 in FP64); each wave owns 64
// consecutive cells.  The rows below and
// above a cell stay in registers and x-neighbours come from the neighbouring
// lanes (the first and last lane of a wave also load the cell just beyond the
// wave), so the kernel needs neither LDS nor barriers.
template <typename T, bool CD>
__global__ __launch_bounds__(kBlock) void k_cg_iter2(Geo G, Stencil<2, T> K, CgIter<T> v,
                                                     CgStep stp, CgScalars* sc) {
  constexpr int TX = kTX2, KC = kKC2<T>;
  constexpr bool NT2 = sizeof(T) == 8;  // (see ld_stream)
  static_assert(TX == kBlock, "one cell of the row segment per thread");
  if (!step_live(stp, sc)) return;
  const int nx = G.nx, nz = G.nz;
  const int ntx = (nx + TX - 1) / TX;
  const int b = xcd_block();
  const int tx = b % ntx, tz = b / ntx;
  const int lane = threadIdx.x & 63;
  const int i = tx * TX + threadIdx.x;
  const int k0 = tz * KC, k1 = min(k0 + KC, nz);
  const bool in = i < nx;
  const T kx = K.k[0], kz = K.k[1];
  // the cell beyond the wave that an edge lane supplies (lane 0: left, lane 63: right)
  const int ie = lane == 0 ? i - 1 : (lane == 63 ? i + 1 : -1);
  const bool edge = ie >= 0 && ie < nx;
  // raw values of row kk (old residual, old A p, old direction, D, 1/diag),
  // own cell and edge cell (CD: me holds the edge cell's c, and 1/diag is
  // formed from c where it is used, as in k_cg_iter3)
  struct Raw {
    T r, q, p, d, m, x, c, re, qe, pe, de, me;
  };
  const T wx = v.Dc * kx, wz = v.Dc * kz;  // (CD) face weights
  auto diag_inv = [&](T c, int ci, int kk) {
    T dg = c;
    dg += ci + 1 < nx ? wx : T(0);
    dg += ci > 0 ? wx : T(0);
    dg += kk + 1 < nz ? wz : T(0);
    dg += kk > 0 ? wz : T(0);
    return T(1) / dg;
  };
  auto m_own = [&](const Raw& w, int kk) { return CD ? diag_inv(w.c, i, kk) : w.m; };
  auto m_edge = [&](const Raw& w, int kk) { return CD ? diag_inv(w.me, ie, kk) : w.me; };
  // unconditional loads from indices clamped into the mesh (values of cells
  // or rows outside it are never used; a load under a branch would be
  // waited for where the branches merge)
  const int ic = in ? i : nx - 1, iec = edge ? ie : ic;
  auto fetch = [&](int kk) {
    const int kc = kk < 0 ? 0 : (kk >= nz ? nz - 1 : kk);
    const int Q = ic + nx * kc, Qe = iec + nx * kc;
    return Raw{v.r_in[Q], v.q_in[Q], v.p_in[Q], CD ? v.Dc : v.D[Q], CD ? T(0) : v.dinv[Q],
               ld_stream<NT2>(&v.x[Q]), ld_stream<NT2>(&v.c[Q]),
               v.r_in[Qe], v.q_in[Qe], v.p_in[Qe], CD ? v.Dc : v.D[Qe], CD ? v.c[Qe] : v.dinv[Qe]};
  };
  // rows k0-1 .. k0+PD in flight while the scalars are formed or read;
  // afterwards row k+PD+1 is requested while row k is computed
  constexpr int PD = sizeof(T) == 8 ? 2 : 3;
  Raw ring[PD + 1];
  const Raw wm = fetch(k0 - 1);
#pragma unroll
  for (int w = 0; w <= PD; ++w) ring[w] = fetch(k0 + w);
  T alpha, beta;
  int fin;
  if (!step_take(stp, sc, alpha, beta, fin)) return;
  if (fin) {  // the solve has converged: its last x update only
    if (in)
      for (int k = k0; k < k1; ++k) last_update(v, i + nx * k, alpha);
    step_last(stp, sc, v.xo != nullptr);
    return;
  }
  // new residual and direction from raw values
  auto rnew = [&](T r, T q) { return r - alpha * q; };
  auto pnew = [&](T rn, T m, T po) { return rn * m + beta * po; };
  T pm = pnew(rnew(wm.r, wm.q), m_own(wm, k0 - 1), wm.p), dm = wm.d;
  Raw cur = ring[0];
  T rc = rnew(cur.r, cur.q), mc = m_own(cur, k0);
  T pc = pnew(rc, mc, cur.p), dc = cur.d;
  T pec = pnew(rnew(cur.re, cur.qe), m_edge(cur, k0), cur.pe), dec = cur.de;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int it = 0; it < KC; ++it) {
    const int k = k0 + it;
    if (k >= k1) break;
    const Raw wn = ring[(it + 1) % (PD + 1)];
    const T rn = rnew(wn.r, wn.q), mn = m_own(wn, k + 1);
    const T pn = pnew(rn, mn, wn.p), dn = wn.d;
    const T pen = pnew(rnew(wn.re, wn.qe), m_edge(wn, k + 1), wn.pe), den = wn.de;
    // slot of row k is free now: request row k+PD+1 into it
    if (k + PD + 1 <= k1) ring[it % (PD + 1)] = fetch(k + PD + 1);
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
      T a = cur.c * pc;
      if (i + 1 < nx) a += T(0.5) * (dc + dr) * kx * (pc - pr);
      if (i > 0) a += T(0.5) * (dl + dc) * kx * (pc - pl);
      if (k + 1 < nz) a += T(0.5) * (dc + dn) * kz * (pc - pn);
      if (k > 0) a += T(0.5) * (dm + dc) * kz * (pc - pm);
      st_stream<NT2>(pc, &v.p_out[P]);
      st_stream<NT2>(a, &v.q_out[P]);
      st_stream<NT2>(rc, &v.r_out[P]);
      st_stream<NT2>(cur.x + alpha * cur.p, &v.x[P]);
      iter_dots(acc, pc, a, rc, mc);
    }
    pm = pc;
    dm = dc;
    pc = pn;
    dc = dn;
    pec = pen;
    dec = den;
    rc = rn;
    mc = mn;
    cur = wn;
  }
  store_partials<7>(acc, iter_part(stp.part, stp.ns, stp.iter));
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
// i_part (what the inner solve's set-up kernel reads).
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_residual64(Geo G, Stencil<NDIM, double> K,
                                                       const double* __restrict__ c,
                                                       const double* __restrict__ D,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       CgVectors<float> v32, int kc,
                                                       double* o_part, double* i_part,
                                                       int zero_inner, const CgScalars* gate) {
  if (gate_closed(gate)) return;
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
      const float rf = (float)r;
      v32.r[P] = rf;
      if (zero_inner) v32.x[P] = 0.0f;
      ro[0] += r * r;
      ro[1] += bp * bp;
      ri[0] += (double)rf * (double)(rf * di);
      ri[1] += (double)rf * (double)rf;
    }
  }
  store_partials<2>(ro, o_part);
  store_partials<2>(ri, i_part);
}

// k_residual64 on a 3D mesh with the x/y neighbours of x and D staged in LDS
// and the next plane's loads in flight while a plane is computed.  Same
// formulas and order as k_residual64.
template <int TY>
__global__ __launch_bounds__(64 * TY) void k_residual64_3(Geo G, Stencil<3, double> K,
                                                         const double* __restrict__ c,
                                                         const double* __restrict__ D,
                                                         const double* __restrict__ b,
                                                         const double* __restrict__ x,
                                                         CgVectors<float> v32, int kc,
                                                         double* o_part, double* i_part,
                                                         int zero_inner, const CgScalars* gate) {
  if (gate_closed(gate)) return;
  using St = Stage3<1, TY>;
  constexpr int HP = St::HP, HX = St::HX, NU = St::NU;
  __shared__ double sx[2][HP], sd[2][HP];
  const Col col = col_of3<TY>(G, kc);
  const St st = stage3<1, TY>(G, col);
  const int nz = G.nz, pl = col.pl, qo = st.qo, ho = st.ho;
  // raw values of the plane in flight
  double fx[NU], fd[NU], fb, fc, fxu, fdu;
  float fdi;
  auto fetch = [&](int kk) {
    const int o = pl * kk, P = qo + o;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      fx[m] = x[st.q[m] + o];
      fd[m] = D[st.q[m] + o];
    }
    const int Pu = kk + 1 < nz ? P + pl : P;
    fb = b[P];
    fc = c[P];
    fdi = v32.dinv[P];
    fxu = x[Pu];
    fdu = D[Pu];
  };
  double ro[2] = {0.0, 0.0};
  double ri[2] = {0.0, 0.0};
  double xm = 0.0, dm = 0.0;
  if (col.k0 > 0) {
    xm = x[qo + pl * (col.k0 - 1)];
    dm = D[qo + pl * (col.k0 - 1)];
  }
  fetch(col.k0);
  for (int k = col.k0; k < col.k1; ++k) {
    const int sl = k & 1;
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      sx[sl][st.h[m]] = fx[m];
      sd[sl][st.h[m]] = fd[m];
    }
    const double bp = fb, cP = fc, xu = fxu, du = fdu;
    const float di = fdi;
    fetch(k + 1 < col.k1 ? k + 1 : k);
    lds_barrier();
    const bool up = k + 1 < nz;
    const double xc = sx[sl][ho], dc = sd[sl][ho];
    const double xp = up ? xu : 0.0, dp = up ? du : 0.0;
    double acc = cP * xc;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int q = coord(col, d), sd_ = d == 0 ? 1 : HX;
      acc = q + 1 < G.n[d] ? acc + 0.5 * (dc + sd[sl][ho + sd_]) * K.k[d] * (xc - sx[sl][ho + sd_]) : acc;
      acc = q > 0 ? acc + 0.5 * (sd[sl][ho - sd_] + dc) * K.k[d] * (xc - sx[sl][ho - sd_]) : acc;
    }
    if (up) acc += 0.5 * (dc + dp) * K.k[2] * (xc - xp);
    if (k > 0) acc += 0.5 * (dm + dc) * K.k[2] * (xc - xm);
    xm = xc;
    dm = dc;
    if (col.act) {
      const int P = qo + pl * k;
      const double r = bp - acc;
      const float rf = (float)r;
      v32.r[P] = rf;
      if (zero_inner) v32.x[P] = 0.0f;
      ro[0] += r * r;
      ro[1] += bp * bp;
      ri[0] += (double)rf * (double)(rf * di);
      ri[1] += (double)rf * (double)rf;
    }
  }
  store_partials<2, 64 * TY>(ro, o_part);
  store_partials<2, 64 * TY>(ri, i_part);
}

// one workgroup: outer stop test and the inner solver's setup
__global__ __launch_bounds__(kBlock) void k_residual_check(const double* o_part,
                                                           const double* i_part, int n,
                                                           double tol2, double inner_tol2,
                                                           double target, int inner_max,
                                                           CgScalars* sc64,
                                                           CgScalars* sc32, const CgScalars* gate) {
  // (every thread reads the gate before sum_partials' barriers; thread 0
  // writes sc32, which may be the gate, only after them)
  if (gate_closed(gate)) return;
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
  sc32->alpha = 0.0;
  sc32->beta = 0.0;
  sc32->fin = 0;
  sc32->done_iter = -1;
  sc32->corrected = 0;
  // inner tolerance: what the outer residual still needs (times the target
  // fraction, a margin for the FP32 solve's own error), never looser than
  // 0.5 nor tighter than the configured inner tolerance
  double it2 = inner_tol2;
  if (o[0] > 0.0 && finite) {
    const double need = target * sqrt(tol2 * o[1] / o[0]);
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

// one workgroup: scalars of the resumed solve (its ||b||^2 and tolerance are
// those the set-up kernel gave the inner system; max_iter iterations remain)
__global__ __launch_bounds__(kBlock) void k_cg_resume_start(const double* part, int n, int max_iter,
                                                            CgScalars* sc) {
  double s[2];
  sum_partials<2>(part, n, s);
  if (threadIdx.x != 0) return;
  sc->rz = s[0];
  sc->rr = s[1];
  sc->rr0 = s[1];
  sc->alpha = 0.0;
  sc->beta = 0.0;
  sc->fin = 0;
  sc->done_iter = -1;
  sc->corrected = 0;
  sc->iter = 0;
  sc->max_iter = max_iter;
  const bool finite = isfinite(s[0]) && isfinite(s[1]);
  sc->status = finite ? 0 : -5;
  // (already done: the refinement's residual check found nothing left to solve)
  const int done = (sc->done || !finite || s[1] <= sc->tol2 * sc->bb || sc->max_iter <= 0) ? 1 : 0;
  __hip_atomic_store(&sc->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

__global__ __launch_bounds__(kBlock) void k_fill(int n, double* a, double v) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x) a[P] = v;
}

__global__ __launch_bounds__(kBlock) void k_sub(int n, const double* b, double* y) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < n; P += gridDim.x * blockDim.x)
    y[P] = b[P] - y[P];
}

__global__ __launch_bounds__(kBlock) void k_add_correction(int n, double* x, const float* dx,
                                                           const CgScalars* own,
                                                           const CgScalars* gate) {
  if (gate_closed(gate) || own->corrected) return;
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

template <typename T>
int iter_grid(const Geo& G) {
  if (G.ndim == 3)
    return ((G.nx + kTX3 - 1) / kTX3) * ((G.ny + kTY3 - 1) / kTY3) * ((G.nz + kKC3<T> - 1) / kKC3<T>);
  return ((G.nx + kTX2 - 1) / kTX2) * ((G.nz + kKC2<T> - 1) / kKC2<T>);
}
template int iter_grid<double>(const Geo&);
template int iter_grid<float>(const Geo&);

template <typename T>
void cg_init(hipStream_t s, const Geo& G, const CgVectors<T>& v, const CgWork& w, double tol,
             int max_iter) {
  const ZPlan zp = zplan(G);
  if (G.ndim == 2)
    hipLaunchKernelGGL((k_cg_init<2, T>), dim3(zp.blocks), dim3(kBlock), 0, s, G, stencil<2, T>(G), v, zp.kc, w.u[1], w.b);
  else
    hipLaunchKernelGGL((k_cg_init<3, T>), dim3(zp.blocks), dim3(kBlock), 0, s, G, stencil<3, T>(G), v, zp.kc, w.u[1], w.b);
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kBlock), 0, s, (const double*)w.u[1], zp.blocks,
                     (const double*)w.b, tol * tol, max_iter, w.sc);
}

// the vectors iteration `iter` reads and writes (by parity; the set-up
// kernels leave the residual in r).  Iteration 0 has no update to apply and
// no previous direction (alpha = 0, beta = 0): it reads r in place of the
// old A p and of the old direction, so that only finite values enter
// r - 0 q, x + 0 p and r/diag + 0 p, and no set-up pass clears a direction.
template <typename T>
CgIter<T> iter_vectors(const CgVectors<T>& v, int iter) {
  const bool odd = iter & 1;
  return CgIter<T>{v.x,
                   odd ? v.r1 : v.r, odd ? v.r : v.r1,
                   iter == 0 ? v.r : (odd ? v.q : v.q1), odd ? v.q1 : v.q,
                   iter == 0 ? v.r : (odd ? v.p1 : v.p0), odd ? v.p0 : v.p1,
                   v.c, v.D, v.dinv, v.Dc, v.xo};
}

bool cg_folds(const CgWork& w) { return w.ns <= kFoldMaxParts; }

template <typename T>
void cg_iter_kernel(hipStream_t s, const Geo& G, const CgVectors<T>& v, int iter, const CgWork& w,
                    bool fold) {
  const CgIter<T> it = iter_vectors(v, iter);
  const CgStep stp{w.s, w.ns, iter, fold && iter > 0 && cg_folds(w) ? 1 : 0};
  const bool cd = v.D == nullptr;
  if (G.ndim == 2) {
    if (cd)
      hipLaunchKernelGGL((k_cg_iter2<T, true>), dim3(iter_grid<T>(G)), dim3(kBlock), 0, s, G, stencil<2, T>(G), it, stp, w.sc);
    else
      hipLaunchKernelGGL((k_cg_iter2<T, false>), dim3(iter_grid<T>(G)), dim3(kBlock), 0, s, G, stencil<2, T>(G), it, stp, w.sc);
  } else {
    if (cd)
      hipLaunchKernelGGL((k_cg_iter3<T, true>), dim3(iter_grid<T>(G)), dim3(kBlock), 0, s, G, stencil<3, T>(G), it, stp, w.sc);
    else
      hipLaunchKernelGGL((k_cg_iter3<T, false>), dim3(iter_grid<T>(G)), dim3(kBlock), 0, s, G, stencil<3, T>(G), it, stp, w.sc);
  }
}

void cg_scalars(hipStream_t s, const Geo& G, int iter, const CgWork& w) {
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kBlock), 0, s, w.s, w.ns, iter, w.sc);
}

template void cg_init<double>(hipStream_t, const Geo&, const CgVectors<double>&, const CgWork&, double, int);
template void cg_init<float>(hipStream_t, const Geo&, const CgVectors<float>&, const CgWork&, double, int);
template void cg_iter_kernel<double>(hipStream_t, const Geo&, const CgVectors<double>&, int, const CgWork&, bool);
template void cg_iter_kernel<float>(hipStream_t, const Geo&, const CgVectors<float>&, int, const CgWork&, bool);


void launch_apply_A(hipStream_t s, const Geo& G, const double* c, const double* D,
                    const double* x, double* y) {
  const dim3 grid(grid_for(G.nc)), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_apply_A<2>, grid, block, 0, s, G, stencil<2, double>(G), c, D, x, y);
  else
    hipLaunchKernelGGL(k_apply_A<3>, grid, block, 0, s, G, stencil<3, double>(G), c, D, x, y);
}

void launch_residual64(hipStream_t s, const Geo& G, const double* c, const double* D,
                       const double* b, const double* x, const CgVectors<float>& v32,
                       double tol, double inner_tol, double target, int inner_max, double* o_part,
                       const CgWork& w32, CgScalars* sc64, bool zero_inner,
                       const CgScalars* gate) {
  constexpr int TY = 8;  // 64x8 column tiles in 3D
  const ZPlan zp = G.ndim == 2 ? zplan(G) : zplan3(G, TY, ZTile<3>::KC);
  const int gu = zp.blocks;
  const dim3 grid(gu), block(kBlock);
  if (G.ndim == 2)
    hipLaunchKernelGGL(k_residual64<2>, grid, block, 0, s, G, stencil<2, double>(G), c, D, b, x, v32, zp.kc, o_part, w32.u[1], (int)zero_inner, gate);
  else
    hipLaunchKernelGGL(k_residual64_3<TY>, grid, dim3(64 * TY), 0, s, G, stencil<3, double>(G), c, D, b, x, v32, zp.kc, o_part, w32.u[1], (int)zero_inner, gate);
  hipLaunchKernelGGL(k_residual_check, dim3(1), block, 0, s, (const double*)o_part,
                     (const double*)w32.u[1], gu, tol * tol, inner_tol * inner_tol, target,
                     inner_max, sc64, w32.sc, gate);
}

void launch_residual_check(hipStream_t s, int n, double tol, double inner_tol, double target,
                           int inner_max, const double* o_part, const CgWork& w32,
                           CgScalars* sc64, const CgScalars* gate) {
  hipLaunchKernelGGL(k_residual_check, dim3(1), dim3(kBlock), 0, s, o_part, (const double*)w32.u[1], n,
                     tol * tol, inner_tol * inner_tol, target, inner_max, sc64, w32.sc, gate);
}

void cg_resume_scalars(hipStream_t s, const double* part, int n, const CgWork& w, int max_iter) {
  hipLaunchKernelGGL(k_cg_resume_start, dim3(1), dim3(kBlock), 0, s, part, n, max_iter, w.sc);
}

void launch_cast_coeffs(hipStream_t s, const Geo& G, const double* c, const double* D,
                        const double* dinv, float* c32, float* D32, float* dinv32) {
  hipLaunchKernelGGL(k_cast_coeffs, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, c, D, dinv, c32, D32, dinv32);
}

void launch_add_correction(hipStream_t s, const Geo& G, double* x, const float* dx,
                           const CgScalars* own, const CgScalars* gate) {
  hipLaunchKernelGGL(k_add_correction, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, x, dx, own,
                     gate);
}

void cg_start_from(hipStream_t s, const double* u_part, int nu, const double* b_part, double tol,
                   int max_iter, CgScalars* sc) {
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kBlock), 0, s, u_part, nu, b_part, tol * tol,
                     max_iter, sc);
}

void launch_fill(hipStream_t s, const Geo& G, double* a, double v) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, a, v);
}

void launch_sub(hipStream_t s, const Geo& G, const double* b, double* y) {
  hipLaunchKernelGGL(k_sub, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G.nc, b, y);
}

}  // namespace gea
