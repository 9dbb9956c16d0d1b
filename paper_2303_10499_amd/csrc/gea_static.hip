// gea_static.hip -- gea_pressure_solve_static: the FP64 Jacobi-PCG solve of
// the pressure system (Sec. 3, Step 3, in the re-derived SPD form stated in
// gea.h) for callers that cannot allocate device memory.  It runs the same
// CG kernels as gea_pressure_solve's FP64 form; its work vectors, partial
// sums and solver scalars live in one file-scope device array instead of a
// caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/gea.h"
#include "gea_internal.h"

namespace gea {

// defined in gea_api.hip
Geo mesh_geo(const gea_mesh& m);
void set_call_error(const std::string& msg);

namespace {

// Capacity of the static work area: meshes of up to 2^20 cells.
constexpr long kStaticMaxCells = 1L << 20;
constexpr int kStaticVectors = 7;             // r, r1, p0, p1, q, q1, 1/diag
constexpr long kStaticIterParts = 7L * 65536;  // 7 partials per iteration-kernel workgroup, two parity sets
constexpr long kStaticSetupParts = 3L * kMaxZBlocks;  // set-up: 2 + 1 per workgroup
constexpr long kStaticScalarDoubles = 32;     // one CgScalars (256 bytes)
constexpr long kStaticDoubles =
    kStaticVectors * kStaticMaxCells + kStaticIterParts + kStaticSetupParts + kStaticScalarDoubles;
static_assert(sizeof(CgScalars) <= kStaticScalarDoubles * sizeof(double), "scalar slot");

}  // namespace
}  // namespace gea

// The work area.  In host code this name is only a stand-in for the symbol:
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[gea::kStaticDoubles];

namespace gea {
namespace {

std::mutex g_static_mu;
constexpr int kMaxDevices = 64;
double* g_static_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (looked up on the
// first call there)
hipError_t static_area(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_static_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_static_ptr[dev];
  return hipSuccess;
}

// 1/diag of the operator, diag = c + sum_f w_f, w_f = (D_P + D_N)/2 S_f/d_f,
// summed in the order the right-hand-side kernels use (x, y: upper then
// lower face; then z: upper, lower), so the result is theirs bitwise.
__global__ __launch_bounds__(kBlock) void k_static_diag_inv(Geo G, const double* __restrict__ c,
                                                            const double* __restrict__ D,
                                                            double* __restrict__ dinv) {
  const int Z = G.ndim - 1;
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < G.nc; P += gridDim.x * blockDim.x) {
    const double Dc = D[P];
    double diag = c[P];
    for (int d = 0; d < Z; ++d) {
      const int q = (P / G.st[d]) % G.n[d];
      const double kd = G.S[d] / G.h[d];
      if (q + 1 < G.n[d]) diag += 0.5 * (Dc + D[P + G.st[d]]) * kd;
      if (q > 0) diag += 0.5 * (D[P - G.st[d]] + Dc) * kd;
    }
    const int k = P / G.st[Z];
    const double kz = G.S[Z] / G.h[Z];
    double hi = 0.0, lo = 0.0;
    if (k + 1 < G.n[Z]) {
      hi = 0.5 * (Dc + D[P + G.st[Z]]) * kz;
      diag += hi;
    }
    if (k > 0) {
      lo = 0.5 * (D[P - G.st[Z]] + Dc) * kz;
      diag += lo;
    }
    dinv[P] = 1.0 / diag;
  }
}

__global__ __launch_bounds__(kBlock) void k_static_fill(long n, double* __restrict__ a, double v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = v;
}

}  // namespace
}  // namespace gea

using namespace gea;

extern "C" {

gea_status gea_pressure_solve_static(const gea_mesh* mesh, const double* c, const double* D,
                                     const double* b, double* x, double tol, int32_t max_iter,
                                     void* hip_stream, gea_solve_stats* stats) {
  auto fail = [](gea_status st, const std::string& msg) {
    set_call_error(msg);
    return st;
  };
  if (!mesh || !c || !D || !b || !x || !stats) return fail(GEA_ERR_ARG, "null argument");
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1 || !(mesh->lx > 0) || !(mesh->ly > 0) ||
      !(mesh->lz > 0))
    return fail(GEA_ERR_ARG, "non-positive mesh size");
  if (!(tol > 0) || max_iter < 0) return fail(GEA_ERR_ARG, "tol must be > 0 and max_iter >= 0");
  const long ncl = (long)mesh->nx * mesh->ny * mesh->nz;
  if (ncl > kStaticMaxCells) {
    char buf[160];
    std::snprintf(buf, sizeof buf,
                  "gea_pressure_solve_static: %ld cells exceed its static work area of %ld cells",
                  ncl, kStaticMaxCells);
    return fail(GEA_ERR_ARG, buf);
  }
  const Geo G = mesh_geo(*mesh);
  const int ns = iter_grid<double>(G);
  const int nzb = zplan(G).blocks;
  if ((long)14 * ns > kStaticIterParts || nzb > kMaxZBlocks)
    return fail(GEA_ERR_ARG, "gea_pressure_solve_static: mesh shape needs more partial sums "
                             "than its static work area holds");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  *stats = gea_solve_stats{};
  auto hip_fail = [&](hipError_t e, const char* what) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return fail(GEA_ERR_HIP, buf);
  };
  double* base = nullptr;
  hipError_t e = static_area(&base);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  // carve the work area (every piece 256-byte aligned: kStaticMaxCells and
  // the partial counts are multiples of 32 doubles)
  const long N = kStaticMaxCells;
  double* vec[kStaticVectors];
  for (int k = 0; k < kStaticVectors; ++k) vec[k] = base + k * N;
  double* iter_parts = base + kStaticVectors * N;
  double* setup_parts = iter_parts + kStaticIterParts;
  CgScalars* sc = reinterpret_cast<CgScalars*>(setup_parts + kStaticSetupParts);
  CgWork w;
  w.s = iter_parts;
  w.ns = ns;
  w.u[0] = nullptr;
  w.u[1] = setup_parts;
  w.b = setup_parts + 2L * kMaxZBlocks;
  w.sc = sc;
  CgVectors<double> v{x, vec[0], vec[1], vec[2], vec[3], vec[4], vec[5], c, D, vec[6], b};
  // the scalars keep the last call's values: clear them (a fill kernel, no
  // memset node), then 1/diag and the solve's set-up
  hipLaunchKernelGGL(k_static_fill, dim3(1), dim3(kBlock), 0, s,
                     (long)(sizeof(CgScalars) / sizeof(double)), reinterpret_cast<double*>(sc), 0.0);
  hipLaunchKernelGGL(k_static_diag_inv, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, G, c, D, vec[6]);
  cg_init<double>(s, G, v, w, tol, max_iter);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "solve set-up");
  CgScalars hs;
  auto read = [&]() -> hipError_t {
    hipError_t r = hipMemcpyAsync(&hs, sc, sizeof hs, hipMemcpyDeviceToHost, s);
    return r != hipSuccess ? r : hipStreamSynchronize(s);
  };
  if ((e = read()) != hipSuccess) return hip_fail(e, "reading the solver scalars");
  stats->rel_res0 = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
  if (hs.bb == 0.0) {  // b = 0: x = 0
    hipLaunchKernelGGL(k_static_fill, dim3(grid_for(G.nc)), dim3(kBlock), 0, s, (long)G.nc, x, 0.0);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "clearing x");
    stats->status = GEA_OK;
    return GEA_OK;
  }
  // batches of iterations: launches after convergence find the done flag
  // set and return at once; the next batch's length follows the residual's
  // observed decay
  long j = 0;
  int batch = 8, prev_iter = hs.iter;
  double prev_rr = hs.rr;
  const long cap = (long)max_iter + 64;
  while (!hs.done) {
    if (j > cap) return fail(GEA_ERR_HIP, "gea_pressure_solve_static: solver flag never set");
    for (int k = 0; k < batch; ++k, ++j) {
      cg_iter_kernel<double>(s, G, v, (int)j, w, k > 0);
      if (k == batch - 1 || !cg_folds(w)) cg_scalars(s, G, (int)j, w);
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "CG iteration launch");
    if ((e = read()) != hipSuccess) return hip_fail(e, "reading the solver scalars");
    const int di = hs.iter - prev_iter;
    batch = 8;
    if (!hs.done && di > 0 && hs.rr > 0 && prev_rr > 0) {
      const double rate = std::log(hs.rr / prev_rr) / di;
      const double need = std::log(hs.tol2 * hs.bb / hs.rr);
      if (rate < -1e-9) {
        const double est = 0.9 * need / rate;
        batch = est < 1.0 ? 1 : (est > 512.0 ? 512 : (int)est);
      }
    }
    prev_iter = hs.iter;
    prev_rr = hs.rr;
  }
  stats->iters = hs.iter;
  stats->rel_res = std::sqrt(hs.rr / hs.bb);
  stats->status = hs.status == 0 ? GEA_OK : (hs.status == -4 ? GEA_ERR_NOCONV : GEA_ERR_NAN);
  if (stats->status != GEA_OK)
    set_call_error(stats->status == GEA_ERR_NOCONV ? "gea_pressure_solve_static: no convergence"
                                                   : "gea_pressure_solve_static: non-finite value");
  return (gea_status)stats->status;
}

}  // extern "C"
