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

template <unsigned MAXMASK, int N>
struct Reducer {
  static constexpr int kWaves = kBlock / 64;

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

// coordinate of the column along an x/y direction
__device__ __forceinline__ int coord(const Col& c, int d) { return d == 0 ? c.i : c.j; }

}  // namespace gea
