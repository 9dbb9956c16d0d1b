// gea_reduce.h -- workgroup reductions for wave64 and cell coordinates.
//
// A value is reduced inside each wave with xor shuffles and across the
// waves of the workgroup through LDS.  Grid-wide sums are formed from one
// partial per workgroup by the kernel that consumes them, in workgroup
// order; the order of every addition is fixed by indices, not by timing, so
// results are bitwise reproducible run to run.
#pragma once
#include "gea_internal.h"

namespace gea {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <unsigned MAXMASK, int K>
__device__ __forceinline__ double combine(double a, double b) {
  return ((MAXMASK >> K) & 1u) ? fmax(a, b) : a + b;
}

template <unsigned MAXMASK, int N, int NT = kBlock>
struct Reducer {
  static constexpr int kWaves = NT / 64;

  // Result in v[] of thread 0 (and, after the call, of every thread via sh).
  __device__ static void block(double (&v)[N], double (*sh)[kWaves]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k)
      v[k] = ((MAXMASK >> k) & 1u) ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < N; ++k) sh[k][w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a = sh[k][0];
      for (int i = 1; i < kWaves; ++i) a = ((MAXMASK >> k) & 1u) ? fmax(a, sh[k][i]) : a + sh[k][i];
      v[k] = a;
    }
    __syncthreads();
  }

  // The same with barriers that order LDS only (sh is all they exchange), so
  // that global loads issued before the call stay in flight across them.
  __device__ static void block_lds(double (&v)[N], double (*sh)[kWaves]);
};

// Workgroup barrier that orders LDS accesses only.  __syncthreads() is also a
// release fence for global memory, which waits for every global load and
// store in flight -- including the next plane's loads issued just before it.
// For kernels in which no thread reads, across the barrier, what another
// thread of the workgroup wrote to global memory.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <unsigned MAXMASK, int N, int NT>
__device__ void Reducer<MAXMASK, N, NT>::block_lds(double (&v)[N], double (*sh)[kWaves]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k)
    v[k] = ((MAXMASK >> k) & 1u) ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k][w] = v[k];
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double a = sh[k][0];
    for (int i = 1; i < kWaves; ++i) a = ((MAXMASK >> k) & 1u) ? fmax(a, sh[k][i]) : a + sh[k][i];
    v[k] = a;
  }
  lds_barrier();
}

// 2D/3D cell coordinates: c[0] = i, then (j,) k.
template <int NDIM>
__device__ __forceinline__ void cell_coords(const Geo& G, int P, int* c) {
  c[0] = P % G.nx;
  const int r = P / G.nx;
  if constexpr (NDIM == 2) {
    c[1] = r;
  } else {
    c[1] = r % G.ny;
    c[2] = r / G.ny;
  }
}

// Workgroup index remapped so that the hardware's round-robin placement of
// consecutive workgroups over the 8 XCDs gives each XCD a contiguous range
// of the logical order (its own L2 then holds the neighbours it re-reads).
__device__ __forceinline__ int xcd_block() {
  const int G = gridDim.x, b = blockIdx.x;
  return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
}

// Cells of a workgroup: grid-stride over the mesh in x-fastest order.  (A
// contiguous chunk per workgroup in XCD-aware order was measured slower for
// the cache-only stencil kernels on MI355X.)
#define GEA_FOR_CELLS(P, G) \
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < (G).nc; P += gridDim.x * blockDim.x)

// ---- z-marching column tiles ----------------------------------------------------
//
// A workgroup owns a TX x TY column of cells (TX cells of one row in 2D) and
// marches it through kc consecutive planes along z; each thread walks one
// vertical column.  Values along z stay in registers (a short queue shifted
// once per plane), the flux through the face below a cell is the one the
// same thread formed one plane earlier, and x/y neighbours come from the
// caches: the workgroup's own rows and the halo rows of the neighbouring
// columns, which the XCD-aware block order keeps on the same XCD.

template <int NDIM>
struct ZTile;
template <>
struct ZTile<3> {
  static constexpr int TX = 64, TY = 4, KC = 32;
};
template <>
struct ZTile<2> {
  static constexpr int TX = 256, TY = 1, KC = 8;
};

struct Col {
  int i, j;      // x (and y) coordinates of the column
  int k0, k1;    // planes [k0, k1) of the chunk
  int base;      // cell index of the column at k = 0
  int pl;        // index stride between planes
  bool act;      // inside the mesh
};

template <int NDIM>
__device__ __forceinline__ Col col_of(const Geo& G, int kc) {
  using T = ZTile<NDIM>;
  const int ntx = (G.nx + T::TX - 1) / T::TX;
  const int nty = NDIM == 3 ? (G.ny + T::TY - 1) / T::TY : 1;
  const int b = xcd_block();
  const int bx = b % ntx, by = (b / ntx) % nty, bk = b / (ntx * nty);
  const int nz = G.n[NDIM - 1];
  Col c;
  c.i = bx * T::TX + (int)threadIdx.x % T::TX;
  c.j = NDIM == 3 ? by * T::TY + (int)threadIdx.x / T::TX : 0;
  c.k0 = bk * kc;
  c.k1 = min(c.k0 + kc, nz);
  c.pl = G.st[NDIM - 1];
  c.base = NDIM == 3 ? c.i + G.nx * c.j : c.i;
  c.act = c.i < G.nx && (NDIM == 2 || c.j < G.ny) && c.k0 < nz;
  return c;
}

// Column tiles of the LDS-staged 3D kernels: 64 x TY cells, one thread (of
// 64 TY) a column, the same block order as col_of.
template <int TY>
__device__ __forceinline__ Col col_of3(const Geo& G, int kc) {
  constexpr int TX = 64;
  const int ntx = (G.nx + TX - 1) / TX, nty = (G.ny + TY - 1) / TY;
  const int b = xcd_block();
  const int bx = b % ntx, by = (b / ntx) % nty, bk = b / (ntx * nty);
  Col c;
  c.i = bx * TX + (int)threadIdx.x % TX;
  c.j = by * TY + (int)threadIdx.x / TX;
  c.k0 = bk * kc;
  c.k1 = min(c.k0 + kc, G.nz);
  c.pl = G.st[2];
  c.base = c.i + G.nx * c.j;
  c.act = c.i < G.nx && c.j < G.ny && c.k0 < G.nz;
  return c;
}

// Plane staging of the 3D kernels: the workgroup's 64 x TY column tile with
// a halo of HW cells along x and y (64x4, HW = 2: 68x8 = 544 cells a plane,
// for the fourth-order interpolation; HW = 1: 66x6 = 396).  Thread t stages
// its own cell (slot 0) and halo cells t, NT + t, ... (slots 1, 2, ...): the
// HW rows below the tile, the HW rows above it, then the side columns.
// Indices are clamped into the mesh, so every staging load is unconditional
// and in bounds; a staged value of a cell outside the mesh is only ever read
// into a term that a wall test discards.
template <int HW_, int TY_>
struct Stage3 {
  static constexpr int TX = 64, TY = TY_, HW = HW_, NT = TX * TY;
  static constexpr int HX = TX + 2 * HW, HY = TY + 2 * HW, HP = HX * HY;
  static constexpr int NH = HP - TX * TY;            // halo cells
  static constexpr int NU = 1 + (NH + NT - 1) / NT;  // slots a thread
  int q[NU];     // cell index in plane 0 (clamped into the mesh)
  int h[NU];     // index in the staged plane
  bool has[NU];  // the thread stages a cell in this slot
  int qo;        // the thread's own column, clamped into the mesh
  int ho;        // its cell in the staged plane
};

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

template <int HW, int TY>
__device__ __forceinline__ Stage3<HW, TY> stage3(const Geo& G, const Col& c) {
  using S = Stage3<HW, TY>;
  S st;
  const int lx = (int)threadIdx.x % S::TX, ly = (int)threadIdx.x / S::TX;
  const int i0 = c.i - lx, j0 = c.j - ly;
  st.ho = (lx + HW) + S::HX * (ly + HW);
  st.qo = clampi(c.i, G.nx) + G.nx * clampi(c.j, G.ny);
  st.q[0] = st.qo;
  st.h[0] = st.ho;
  st.has[0] = true;
#pragma unroll
  for (int m = 1; m < S::NU; ++m) {
    int e = (int)threadIdx.x + (m - 1) * S::NT;
    st.has[m] = e < S::NH;
    if (!st.has[m]) {  // no cell in this slot: the own cell again (the step kernels store
                       // it unconditionally, to its own place: the same value as slot 0)
      st.q[m] = st.qo;
      st.h[m] = st.ho;
      continue;
    }
    int hx, hy;
    if (e < HW * S::HX) {
      hy = e / S::HX;
      hx = e % S::HX;
    } else if (e < 2 * HW * S::HX) {
      e -= HW * S::HX;
      hy = S::TY + HW + e / S::HX;
      hx = e % S::HX;
    } else {
      e -= 2 * HW * S::HX;
      hy = HW + e / (2 * HW);
      const int s = e % (2 * HW);
      hx = s < HW ? s : S::HX - 2 * HW + s;
    }
    st.h[m] = hx + S::HX * hy;
    st.q[m] = clampi(i0 + hx - HW, G.nx) + G.nx * clampi(j0 + hy - HW, G.ny);
  }
  return st;
}

// coordinate of the column along an x/y direction
__device__ __forceinline__ int coord(const Col& c, int d) { return d == 0 ? c.i : c.j; }

template <int NDIM, typename T>
struct Stencil {
  T k[NDIM];  // S_d / h_d in the working precision
};

// A x at the cells of a column walking up through z: x and D of the planes
// below, at and above the current one stay in registers, x/y neighbours
// come from the caches.  The terms are summed in the order x+, x-, y+, y-,
// z+, z- (the order of the CG kernels' operator).
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

}  // namespace gea
