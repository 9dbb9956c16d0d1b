// gea_stencil.h -- the five-point lines along one direction that the
// fourth-order face interpolation of Sec. 3 (reading R10: cubic with two
// cells on each side of a face, linear next to a wall) reads, shared by the
// explicit step kernels and the implicit-transport operator.
#pragma once
#include "gea_internal.h"

namespace gea {
namespace {

// Five consecutive values of a cell field along one direction, centred on
// the cell.  Positions outside the mesh hold the centre value (their load is
// clamped to the cell itself) and are never used.
struct Line {
  double m2, m1, c, p1, p2;
};

// Index of a neighbour if it exists, else of the cell itself.  Every load of
// a plane is then made unconditionally from inside the mesh and each wall
// test is a select on loaded values: no branch separates a plane's loads, so
// they are all in flight together.
__device__ __forceinline__ int nb(bool ok, int Q, int P) { return ok ? Q : P; }

template <typename F>
__device__ __forceinline__ Line line_at(F s, int P, int st, int q, int n) {
  Line L;
  L.m2 = s(nb(q >= 2, P - 2 * st, P));
  L.m1 = s(nb(q >= 1, P - st, P));
  L.c = s(P);
  L.p1 = s(nb(q + 1 < n, P + st, P));
  L.p2 = s(nb(q + 2 < n, P + 2 * st, P));
  return L;
}

// next plane: drop the lowest value, append the one two planes above
__device__ __forceinline__ Line shift(const Line& L, double next) {
  return Line{L.m1, L.c, L.p1, L.p2, next};
}

// interp4 on the face above (q + 1/2) and below (q - 1/2) the centre of a
// line; linear next to a wall
__device__ __forceinline__ double i4_hi(const Line& s, int q, int n) {
  const double f4 = (-s.m1 + 9.0 * s.c + 9.0 * s.p1 - s.p2) / 16.0;
  const double f2 = 0.5 * (s.c + s.p1);
  return (q >= 1 && q + 2 <= n - 1) ? f4 : f2;
}
__device__ __forceinline__ double i4_lo(const Line& s, int q, int n) {
  const double f4 = (-s.m2 + 9.0 * s.m1 + 9.0 * s.c - s.p1) / 16.0;
  const double f2 = 0.5 * (s.m1 + s.c);
  return (q >= 2 && q + 1 <= n - 1) ? f4 : f2;
}

}  // namespace
}  // namespace gea
