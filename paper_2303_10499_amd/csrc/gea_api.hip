// gea_api.hip -- the C ABI of include/gea.h: context, workspace carving,
// the time step's kernel sequence (Sec. 3: Step 1, Step 2, PISO Step 3) and
// the pressure solvers (FP64 Jacobi-PCG, FP32/FP64 iterative refinement).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "../../include/gea.h"
#include "../../include/gea_learned.h"
#include "gea_cnn_internal.h"
#include "gea_internal.h"

using namespace gea;

namespace {

thread_local std::string g_init_error;

// Carves 256-byte aligned buffers out of one workspace; with a null base it
// only measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct State {
  double* rho;
  double* u[3];
  double* T;
  double* pp;
  double* p;
  double* phi[3];  // face mass flux: face d of cell P lies between P and P + st[d]
  double* pm;      // p^{n-1} and K^{n-1} of the enthalpy form's lagged terms, valid
  double* Km;      //   while the context's hist[] flag of this state is set
};

constexpr int kMaxPartials = 2048 * 8;

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(call)                                 \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) throw HipError{e_, #call}; \
  } while (0)

// Optional per-kernel-class device timing: events recorded on the stream
// around each launch, summed after the next stream synchronisation.
struct KernelTimer {
  static constexpr int kClasses = 8;
  bool on = false;
  double ms[kClasses] = {};
  long long launches[kClasses] = {};
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Pending {
    int k;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;

  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  template <typename F>
  void run(int k, hipStream_t s, F&& launch) {
    if (!on) {
      launch();
      return;
    }
    hipEvent_t a = take(), b = take();
    HIPCHK(hipEventRecord(a, s));
    launch();
    HIPCHK(hipEventRecord(b, s));
    pending.push_back({k, a, b});
    if (used > 4096) {
      HIPCHK(hipStreamSynchronize(s));
      flush();
    }
  }
  // call only after the stream has been synchronised
  void flush() {
    for (const Pending& p : pending) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, p.a, p.b));
      ms[p.k] += t;
      launches[p.k] += 1;
    }
    pending.clear();
    used = 0;
  }
  void reset() {
    for (int k = 0; k < kClasses; ++k) {
      ms[k] = 0.0;
      launches[k] = 0;
    }
  }
  ~KernelTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

// Whether the learned form runs its network on a corrector's solve: it runs
// while the inner iterations it saves, in running averages of solves with
// and without it, take longer than one application (network, flexible-CG
// step and set-up).  The other choice is re-tried after a period of solves
// that starts at 16 and doubles, up to 256, each time a re-try leaves the
// choice as it was (a re-try that changes it sets the period back to 16):
// where the network keeps not paying, re-tries stop costing the solver.
struct NetGate {
  static constexpr int kFirst = 16, kMost = 256;
  double it_net = -1.0, it_plain = -1.0;  // inner iterations a solve that needed any
  int since = 0;       // solves since the last re-try
  int every = kFirst;  // re-try period
  // the choice the averages make, -1 while one of them or a time is missing
  static int choice(double it_net, double it_plain, double t_net, double t_iter) {
    if (it_net < 0 || it_plain < 0 || !(t_net > 0) || !(t_iter > 0)) return -1;
    return (it_plain - it_net) * t_iter > t_net ? 1 : 0;
  }
  bool use(double t_net, double t_iter) const {
    if (it_net < 0) return true;    // first with the network,
    if (it_plain < 0) return false;  // then once without
    if (!(t_net > 0)) return true;    // (times still to be taken: the network's
    if (!(t_iter > 0)) return false;  // in a solve with it, an iteration's without)
    const bool pays = choice(it_net, it_plain, t_net, t_iter) == 1;
    return since + 1 >= every ? !pays : pays;
  }
  void record(bool net, double its, double t_net, double t_iter) {
    const int before = choice(it_net, it_plain, t_net, t_iter);
    double& e = net ? it_net : it_plain;
    e = e < 0 ? its : 0.75 * e + 0.25 * its;
    if (before >= 0 && (net ? 1 : 0) != before) {  // a re-try
      const int after = choice(it_net, it_plain, t_net, t_iter);
      every = after == before ? (2 * every < kMost ? 2 * every : kMost) : kFirst;
      since = 0;
    } else {
      ++since;
    }
  }
};

struct gea_ctx {
  gea_mesh mesh;
  gea_params prm;
  Geo G;
  Phys ph;
  hipStream_t stream;
  State st[2];
  int cur = 0;
  double* Tbg;
  double* rho_a;
  double* pp_a;
  // step work arrays
  double* rho_star;
  double* ustar[3];
  double* e0;
  double* ea;  // K* (explicit transport) or the implicit energy system's known part
  double* rho23;
  double* psi;
  double* c;
  double* D;
  double* H[3];
  double* b;
  double* dinv;
  // FP64 CG (residual and A p double buffered)
  double* r;
  double* r1;
  double* p0;
  double* p1;
  double* q;
  double* q1;
  double* xs;  // scratch vector (solutions, operator application)
  // mixed precision
  double* r64;
  float* c32;
  float* D32;
  float* dinv32;
  float* r32;
  float* r132;
  float* p032;
  float* p132;
  float* q32;
  float* q132;
  float* d32;
  // reductions
  double* partials;  // per-workgroup partials of the step kernels
  double* ext;       // extrema of the state (8 values)
  double* o_part;    // partials of the refinement's outer residual
  CgScalars* sc;     // FP64 solver and step scalars
  CgScalars* sc32;   // inner FP32 solver scalars
  CgWork w64;
  CgWork w32;
  // learned form
  float* r_old32;
  float* z32;
  double* pair_part;
  double* pair_s;      // max |r0| and its inverse (training pairs)
  FcgScalars* fsc;
  FcgVectors fv;
  // implicit transport (transport = 1): BiCGStab vectors and scalars
  TrVecs trv{};
  double* trb[3] = {nullptr, nullptr, nullptr};  // the predictor systems' right-hand sides
  TrScalars* tsc = nullptr;
  Cnn net;             // network at the mesh resolution (learned form only)
  bool has_net_space = false;
  bool has_net = false;
  int fallbacks = 0;
  // learned form: the gate per corrector, its decision for the solve being
  // assembled, and the device times (ms) of one network application and
  // one FP32 inner iteration, each taken once from events around real work
  NetGate gate[8];
  bool net_now = false;
  double t_net_ms = -1.0, t_iter_ms = -1.0;
  hipEvent_t ev_net[2] = {}, ev_it[2] = {};
  int net_probe = 0;  // 1: ev_net recorded, not yet read
  int it_probe = 0;   // batch length recorded between ev_it, 0: none
  int it_probe_iter0 = 0;
  KernelTimer timer;
  // iterations of the previous step's solve of the same corrector (and
  // refinement step): the first batch's length
  int last_iters64[8] = {};
  int last_iters_energy[8] = {};  // of the previous step's energy solves, per sweep
  int last_iters32[8][4] = {};
  int last_iters_res = 0;  // iterations of the last Jacobi-PCG resumed after the network
  bool has_state = false;
  bool hist[2] = {false, false};  // st[i].pm, st[i].Km hold the state's history
  bool has_system = false;
  bool sys32 = false;  // c32, D32, dinv32 hold the current operator
  int res_parts = 0;   // partials of a first residual check the system build formed
  // Work that follows a converged solve (the corrector's correction),
  // enqueued by the refined forms right behind an outer residual check that
  // the previous step's same check found converged, before the host reads
  // it; when that read says otherwise the tail is enqueued again after the
  // solve (it reads nothing the solve writes).
  const std::function<void()>* tail = nullptr;
  bool tail_done = false;   // the tail ran behind the final residual check
  CgScalars last_h64{};     // the FP64 scalars as the last outer residual check read them
  int corr = 0;             // corrector of the solve in progress
  bool conv_hist[8][4] = {};  // [corrector][outer step]: that check converged last time
  bool predict_conv(int outer) const {
    return tail && corr < 8 && conv_hist[corr][outer < 3 ? outer : 3];
  }
  bool predict_unconv(int outer) const {
    return tail && corr < 8 && !conv_hist[corr][outer < 3 ? outer : 3];
  }
  void note_conv(int outer, bool c) {
    if (corr < 8) conv_hist[corr][outer < 3 ? outer : 3] = c;
  }
  std::string err;
  // pinned host buffer the solver scalars are read through (device-to-host
  // copies into it are asynchronous, so several go out with one wait)
  char* pin = nullptr;
  static constexpr size_t kPinBytes = 4096;
  // snapshots: device structs copied into the upper half of the pinned
  // buffer where the stream reaches them, delivered at the next read
  static constexpr size_t kSnapBase = 2048, kSnapSlot = 256;
  struct Snap {
    void* host;
    size_t bytes;
  };
  Snap snaps[8];
  int nsnap = 0;
  ~gea_ctx() {
    for (hipEvent_t e : {ev_net[0], ev_net[1], ev_it[0], ev_it[1]})
      if (e) (void)hipEventDestroy(e);
    if (pin) (void)hipHostFree(pin);
  }
};

namespace {

Geo make_geo(const gea_mesh& m) {
  Geo G;
  const double dx = m.lx / m.nx, dy = m.ly / m.ny, dz = m.lz / m.nz;
  G.nx = m.nx;
  G.ny = m.ny;
  G.nz = m.nz;
  G.nc = m.nx * m.ny * m.nz;
  G.V = dx * dy * dz;
  G.dz = dz;
  if (m.ny == 1) {
    G.ndim = 2;
    G.n[0] = m.nx; G.st[0] = 1;    G.h[0] = dx; G.S[0] = dy * dz;
    G.n[1] = m.nz; G.st[1] = m.nx; G.h[1] = dz; G.S[1] = dx * dy;
    G.n[2] = 1;    G.st[2] = 0;    G.h[2] = 0;  G.S[2] = 0;
  } else {
    G.ndim = 3;
    G.n[0] = m.nx; G.st[0] = 1;           G.h[0] = dx; G.S[0] = dy * dz;
    G.n[1] = m.ny; G.st[1] = m.nx;        G.h[1] = dy; G.S[1] = dx * dz;
    G.n[2] = m.nz; G.st[2] = m.nx * m.ny; G.h[2] = dz; G.S[2] = dx * dy;
  }
  for (int d = 0; d < kMaxDim; ++d) G.inv_h[d] = G.h[d] > 0 ? 1.0 / G.h[d] : 0.0;
  G.inv_V = 1.0 / G.V;
  return G;
}

}  // namespace

namespace gea {
Geo mesh_geo(const gea_mesh& m) { return make_geo(m); }
void set_call_error(const std::string& msg) { g_init_error = msg; }
}  // namespace gea

namespace {

size_t carve(Carver& cv, gea_ctx* x, const gea_mesh& m, bool learned, bool transport) {
  const size_t nc = (size_t)m.nx * m.ny * m.nz;
  const int nd = m.ny == 1 ? 2 : 3;
  for (int s = 0; s < 2; ++s) {
    State& S = x->st[s];
    S.rho = cv.take<double>(nc);
    for (int d = 0; d < 3; ++d) S.u[d] = d < nd ? cv.take<double>(nc) : nullptr;
    S.T = cv.take<double>(nc);
    S.pp = cv.take<double>(nc);
    S.p = cv.take<double>(nc);
    for (int d = 0; d < 3; ++d) S.phi[d] = d < nd ? cv.take<double>(nc) : nullptr;
    S.pm = cv.take<double>(nc);
    S.Km = cv.take<double>(nc);
  }
  x->Tbg = cv.take<double>(m.nz);
  x->rho_a = cv.take<double>(m.nz);
  x->pp_a = cv.take<double>(m.nz);
  x->rho_star = cv.take<double>(nc);
  for (int d = 0; d < 3; ++d) x->ustar[d] = d < nd ? cv.take<double>(nc) : nullptr;
  x->e0 = cv.take<double>(nc);
  x->ea = cv.take<double>(nc);
  x->rho23 = cv.take<double>(nc);
  x->psi = cv.take<double>(nc);
  x->c = cv.take<double>(nc);
  x->D = cv.take<double>(nc);
  for (int d = 0; d < 3; ++d) x->H[d] = d < nd ? cv.take<double>(nc) : nullptr;
  x->b = cv.take<double>(nc);
  x->dinv = cv.take<double>(nc);
  x->r = cv.take<double>(nc);
  x->r1 = cv.take<double>(nc);
  x->p0 = cv.take<double>(nc);
  x->p1 = cv.take<double>(nc);
  x->q = cv.take<double>(nc);
  x->q1 = cv.take<double>(nc);
  x->xs = cv.take<double>(nc);
  x->r64 = cv.take<double>(nc);
  x->c32 = cv.take<float>(nc);
  x->D32 = cv.take<float>(nc);
  x->dinv32 = cv.take<float>(nc);
  x->r32 = cv.take<float>(nc);
  x->r132 = cv.take<float>(nc);
  x->p032 = cv.take<float>(nc);
  x->p132 = cv.take<float>(nc);
  x->q32 = cv.take<float>(nc);
  x->q132 = cv.take<float>(nc);
  x->d32 = cv.take<float>(nc);
  {
    const int zb = 3 * zplan(make_geo(m)).blocks;  // partials of the correction kernel
    x->partials = cv.take<double>(zb > kMaxPartials ? zb : kMaxPartials);
  }
  x->o_part = cv.take<double>(kMaxPartials);
  x->ext = cv.take<double>(8);
  // the solver scalars side by side, 256 bytes apart: a poll copies them in one piece
  x->sc = cv.take<CgScalars>(1);
  x->sc32 = cv.take<CgScalars>(1);
  x->fsc = cv.take<FcgScalars>(1);
  x->tsc = cv.take<TrScalars>(1);
  if (transport)
    for (double** a : {&x->trv.b, &x->trv.dinv, &x->trv.r, &x->trv.rh, &x->trv.p, &x->trv.v,
                       &x->trv.y, &x->trv.z, &x->trv.t})
      *a = cv.take<double>(nc);
  if (transport)
    for (int d = 0; d < nd; ++d) x->trb[d] = cv.take<double>(nc);
  // partials: 7 per workgroup of the iteration kernel's grid, in two sets
  // (by iteration parity); 2 (and 1 for ||b||^2) per workgroup of the set-up
  // kernels' column-tile grid
  const int ns = std::max(iter_grid<double>(make_geo(m)), iter_grid<float>(make_geo(m)));
  const int nzb = zplan(make_geo(m)).blocks;
  for (CgWork* w : {&x->w64, &x->w32}) {
    w->s = cv.take<double>(14 * (size_t)ns);
    w->u[0] = nullptr;
    w->u[1] = cv.take<double>(2 * (size_t)nzb);
    w->b = cv.take<double>(nzb);
  }
  x->w64.sc = x->sc;
  x->w32.sc = x->sc32;
  x->w64.ns = iter_grid<double>(make_geo(m));
  x->w32.ns = iter_grid<float>(make_geo(m));
  x->r_old32 = cv.take<float>(nc);
  x->z32 = cv.take<float>(nc);
  x->pair_part = cv.take<double>(3 * 2048);
  x->pair_s = cv.take<double>(2);
  x->fv.part_d = cv.take<double>(4 * (size_t)std::max(2048, zplan(make_geo(m)).blocks));  // (4 sums a workgroup at the hand-over)
  x->fv.part_s = cv.take<double>(2 * (size_t)std::max(2048, zplan(make_geo(m)).blocks));
  x->fv.part_u = cv.take<double>(2 * 2048);
  // the network (inference buffers) only for the learned form on a mesh whose
  // dimensions are multiples of 4
  x->has_net_space = learned && cnn_dims_ok(nd, m.nx, m.ny, m.nz);
  if (x->has_net_space) cv.off = cnn_carve(x->net, nd, m.nx, m.ny, m.nz, false, cv.base, cv.off);
  return cv.off + 256;
}

gea_status check_params(const gea_mesh* m, const gea_params* q, std::string& err) {
  if (!m || !q) {
    err = "null mesh or params";
    return GEA_ERR_ARG;
  }
  if (m->nx < 1 || m->ny < 1 || m->nz < 1) {
    err = "mesh dimensions must be positive";
    return GEA_ERR_ARG;
  }
  if ((double)m->nx * m->ny * m->nz > 2147483647.0 / 1.0) {
    err = "more than 2^31-1 cells";
    return GEA_ERR_ARG;
  }
  if (!(m->lx > 0 && m->ly > 0 && m->lz > 0)) {
    err = "domain lengths must be positive";
    return GEA_ERR_ARG;
  }
  if (!(q->R > 0 && q->cp > 0 && q->cv > 0 && q->dt > 0 && q->Pr > 0 && q->g >= 0 &&
        q->mu >= 0 && q->p0 > 0 && q->theta0 > 0)) {
    err = "physical constants must be positive (g, mu non-negative)";
    return GEA_ERR_ARG;
  }
  if (q->n_corr < 1 || q->n_corr > 8 || q->n_energy_sweeps < 1) {
    err = "n_corr must be in 1..8 and n_energy_sweeps >= 1";
    return GEA_ERR_ARG;
  }
  if (q->solver < 0 || q->solver > 2 || !(q->tol > 0) || q->max_iter < 1) {
    err = "bad solver, tol or max_iter";
    return GEA_ERR_ARG;
  }
  if (q->solver != GEA_PCG_JACOBI_FP64 && !(q->inner_tol > 0 && q->inner_tol < 1)) {
    err = "inner_tol must be in (0, 1) for the refined solvers";
    return GEA_ERR_ARG;
  }
  if (!(q->inner_target >= 0 && q->inner_target <= 1)) {
    err = "inner_target must be in [0, 1] (0 selects 0.8)";
    return GEA_ERR_ARG;
  }
  if (q->solver == GEA_LEARNED_MIXED && q->learned_steps < 1) {
    err = "learned_steps must be >= 1";
    return GEA_ERR_ARG;
  }
  if (q->energy_form != 0 && q->energy_form != 1) {
    err = "energy_form must be 0 (total energy) or 1 (enthalpy)";
    return GEA_ERR_ARG;
  }
  if (q->transport != 0 && q->transport != 1) {
    err = "transport must be 0 (explicit sweeps) or 1 (implicit, BiCGStab)";
    return GEA_ERR_ARG;
  }
  return GEA_OK;
}

void setup_geometry(gea_ctx* x) {
  x->G = make_geo(x->mesh);
  const gea_params& q = x->prm;
  x->ph = Phys{q.R, q.cp, q.cv, q.g, q.mu, q.Pr, q.dt, q.p0, q.theta0, 1.0 / q.dt, 1.0 / q.cv};
}

// A device struct to read along with the solver scalars.
struct Extra {
  const void* dev = nullptr;
  void* host = nullptr;
  size_t bytes = 0;
};

// Wait for the stream by polling it: the host acts on the solver scalars
// as soon as the copy lands, without a blocking wait's wake-up latency.
void wait_stream(gea_ctx* x) {
  hipError_t e;
  while ((e = hipStreamQuery(x->stream)) == hipErrorNotReady) {
  }
  HIPCHK(e);
}

// Copy a device struct into the pinned buffer at this point of the stream;
// the host copy in *host is filled at the next read.
void snapshot(gea_ctx* x, const void* dev, void* host, size_t bytes) {
  if (x->nsnap >= 8 || bytes > gea_ctx::kSnapSlot)
    throw HipError{hipErrorInvalidValue, "snapshot slots exhausted"};
  char* slot = x->pin + gea_ctx::kSnapBase + gea_ctx::kSnapSlot * x->nsnap;
  HIPCHK(hipMemcpyAsync(slot, dev, bytes, hipMemcpyDeviceToHost, x->stream));
  x->snaps[x->nsnap++] = gea_ctx::Snap{host, bytes};
}

// Device structs to the host through the pinned buffer with one wait.  Part
// k lands at a 256-byte aligned offset; parts laid out the same way on the
// device (the solver scalars are) go in one copy.
void read_structs(gea_ctx* x, const Extra* parts, int n) {
  size_t off = 0;
  bool one = true;
  for (int k = 0; k < n; ++k) {
    if (off + parts[k].bytes > gea_ctx::kSnapBase) throw HipError{hipErrorInvalidValue, "pinned read buffer too small"};
    one = one && static_cast<const char*>(parts[k].dev) == static_cast<const char*>(parts[0].dev) + off;
    off += (parts[k].bytes + 255) & ~(size_t)255;
  }
  if (one) {
    const size_t span = off - ((parts[n - 1].bytes + 255) & ~(size_t)255) + parts[n - 1].bytes;
    HIPCHK(hipMemcpyAsync(x->pin, parts[0].dev, span, hipMemcpyDeviceToHost, x->stream));
  } else {
    off = 0;
    for (int k = 0; k < n; ++k) {
      HIPCHK(hipMemcpyAsync(x->pin + off, parts[k].dev, parts[k].bytes, hipMemcpyDeviceToHost, x->stream));
      off += (parts[k].bytes + 255) & ~(size_t)255;
    }
  }
  wait_stream(x);
  off = 0;
  for (int k = 0; k < n; ++k) {
    std::memcpy(parts[k].host, x->pin + off, parts[k].bytes);
    off += (parts[k].bytes + 255) & ~(size_t)255;
  }
  for (int k = 0; k < x->nsnap; ++k)
    std::memcpy(x->snaps[k].host, x->pin + gea_ctx::kSnapBase + gea_ctx::kSnapSlot * k,
                x->snaps[k].bytes);
  x->nsnap = 0;
  x->timer.flush();
}

// Device scalars (and an optional second struct) to the host with one wait.
void read_scalars(gea_ctx* x, CgScalars* dev, CgScalars* host, const Extra& extra = Extra{}) {
  const Extra parts[2] = {Extra{dev, host, sizeof(CgScalars)}, extra};
  read_structs(x, parts, extra.bytes ? 2 : 1);
}

// Host loop of one CG solve: enqueue batches of iterations, read the device
// scalars after each batch.  The batch length is predicted from the
// residual's observed decay rate so that few launches follow convergence
// (those find the done flag set and return at once).  A solve enqueued
// behind kernels whose outcome the host has not read (hs.rr = 0 on entry)
// takes its starting residual from the device scalars' rr0.  A solve whose
// first j0 iterations are already enqueued and read (hs) continues at
// iteration j0.
template <typename LaunchIter>
gea_status run_cg(gea_ctx* x, CgScalars* dsc, CgScalars& hs, int max_iter, int first_batch,
                  LaunchIter&& launch_iter, const Extra& extra = Extra{}, long j0 = 0,
                  bool time_iter = false) {
  const int every = x->prm.check_every > 0 ? x->prm.check_every : 8;
  const long cap = j0 + (long)max_iter + 4L * every + 64;
  int batch = first_batch > 0 ? first_batch : every;
  long j = j0;
  int prev_iter = hs.iter;
  double prev_rr = hs.rr;
  while (!hs.done) {
    if (j > cap) {
      x->err = "solver flag never set";
      return GEA_ERR_HIP;
    }
    // time_iter: events around a batch of at least two launches, kept as
    // the time of one iteration if every launch of it did one
    const bool timed = time_iter && x->t_iter_ms < 0 && batch >= 2 && hs.rr > 0;
    if (timed) HIPCHK(hipEventRecord(x->ev_it[0], x->stream));
    for (int k = 0; k < batch; ++k, ++j) launch_iter((int)j, k > 0, k == batch - 1);
    if (timed) HIPCHK(hipEventRecord(x->ev_it[1], x->stream));
    HIPCHK(hipGetLastError());
    const int iter_before = hs.iter;
    read_scalars(x, dsc, &hs, extra);
    if (timed && hs.iter - iter_before == batch) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, x->ev_it[0], x->ev_it[1]));
      x->t_iter_ms = (double)t / batch;
    }
    if (prev_rr <= 0.0) {
      prev_rr = hs.rr0;
      prev_iter = 0;
    }
    const int di = hs.iter - prev_iter;
    batch = every;
    if (!hs.done && di > 0 && hs.rr > 0 && prev_rr > 0 && hs.bb > 0) {
      const double rate = std::log(hs.rr / prev_rr) / di;    // per iteration, < 0 when converging
      const double need = std::log(hs.tol2 * hs.bb / hs.rr);  // < 0 while not converged
      if (rate < -1e-9) {
        const double est = 0.9 * need / rate;
        batch = est < 1.0 ? 1 : (est > 512.0 ? 512 : (int)est);
      }
    }
    prev_iter = hs.iter;
    prev_rr = hs.rr;
  }
  return GEA_OK;
}

// The gate of the corrector in progress, with the timings of earlier
// probes read in once their events have completed.
NetGate& net_gate(gea_ctx* x) {
  if (x->net_probe && hipEventQuery(x->ev_net[1]) == hipSuccess) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, x->ev_net[0], x->ev_net[1]) == hipSuccess) x->t_net_ms = t;
    x->net_probe = 0;
  }
  return x->gate[x->corr < 8 ? x->corr : 7];
}

// Pressure right-hand side and 1/diag from H; the refined forms also get the
// FP32 copies of the operator from the same pass.
// With xv given, a refined form's first residual check on xv (the solve's
// initial guess) is formed in the same pass (3D); the solve then starts
// from its one-workgroup check.  coeffs = false: 1/diag and the FP32 copies
// of c, D, 1/diag are those an earlier corrector of the step wrote (c and D
// change only in Step 2), and only b (and the residual) are formed.
void build_system(gea_ctx* x, const State& S, const double* xv = nullptr, bool coeffs = true) {
  const bool f32 = x->prm.solver != GEA_PCG_JACOBI_FP64;
  x->net_now = x->prm.solver == GEA_LEARNED_MIXED && x->has_net &&
               (x->prm.learned_always || net_gate(x).use(x->t_net_ms, x->t_iter_ms));
  // the learned form's first inner solve is the flexible CG, which needs no
  // cleared inner iterate or direction
  const bool zero_inner = !x->net_now;
  const RhsResidual res{xv, x->r32, x->d32, (int)zero_inner, x->o_part, x->w32.u[1]};
  const bool c32 = f32 && (coeffs || !x->sys32);
  x->res_parts = launch_rhs(x->stream, x->G, x->ph, S.rho, x->rho23, x->psi, x->c, x->D, x->H,
                            x->b, coeffs ? x->dinv : nullptr, c32 ? x->c32 : nullptr,
                            c32 ? x->D32 : nullptr, c32 ? x->dinv32 : nullptr,
                            f32 && xv ? &res : nullptr);
  x->sys32 = f32;
}

// The refinement's residual check of xv: from the partials the system build
// formed (first check of a solve), else a residual pass of its own.
// With a gate the check acts only if the inner solve behind those scalars
// is done.
// (0.8 measured best of 0.1 / 0.25 / 0.5 / 0.8 on both evaluation meshes: a
// smaller target overshoots the tolerance, and on the 2D mesh the second
// corrector's solve then needs ~150 inner iterations instead of ~10)
double inner_target(const gea_ctx* x) { return x->prm.inner_target > 0 ? x->prm.inner_target : 0.8; }

void residual_check(gea_ctx* x, const double* xv, const CgVectors<float>& v, int budget,
                    bool zero_inner, const CgScalars* gate = nullptr) {
  const int n = x->res_parts;
  x->res_parts = 0;
  x->timer.run(4, x->stream, [&] {
    if (n > 0)
      launch_residual_check(x->stream, n, x->prm.tol, x->prm.inner_tol, inner_target(x), budget > 0 ? budget : 1,
                            x->o_part, x->w32, x->sc, gate);
    else
      launch_residual64(x->stream, x->G, x->c, x->D, x->b, xv, v, x->prm.tol, x->prm.inner_tol, inner_target(x),
                        budget > 0 ? budget : 1, x->o_part, x->w32, x->sc, zero_inner, gate);
  });
}

// FP32 copies of the operator unless the system build wrote them.
void cast_system(gea_ctx* x) {
  if (x->sys32) return;
  x->timer.run(4, x->stream, [&] {
    launch_cast_coeffs(x->stream, x->G, x->c, x->D, x->dinv, x->c32, x->D32, x->dinv32);
  });
  x->sys32 = true;
}

// FP64 Jacobi-PCG on (c, D, dinv, b) from the initial guess in xv.
gea_status solve_pcg64(gea_ctx* x, double* xv, gea_solve_stats* out) {
  const Geo& G = x->G;
  const CgWork& w = x->w64;
  CgVectors<double> v{xv, x->r, x->r1, x->p0, x->p1, x->q, x->q1, x->c, x->D, x->dinv, x->b};
  x->timer.run(4, x->stream, [&] { cg_init<double>(x->stream, G, v, w, x->prm.tol, x->prm.max_iter); });
  HIPCHK(hipGetLastError());
  CgScalars hs;
  read_scalars(x, x->sc, &hs);
  out->rel_res0 = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
  if (hs.bb == 0.0) {
    HIPCHK(hipMemsetAsync(xv, 0, sizeof(double) * G.nc, x->stream));
    out->iters = 0;
    out->rel_res = 0.0;
    out->status = GEA_OK;
    return GEA_OK;
  }
  int& last64 = x->last_iters64[x->corr < 8 ? x->corr : 7];
  const int first = last64 > 0 ? (int)(0.9 * last64) : 0;
  gea_status rc = run_cg(
      x, x->sc, hs, x->prm.max_iter, first,
      [&](int j, bool fold, bool last) {
        x->timer.run(0, x->stream, [&] { cg_iter_kernel<double>(x->stream, G, v, j, w, fold); });
        if (last || !cg_folds(w)) x->timer.run(1, x->stream, [&] { cg_scalars(x->stream, G, j, w); });
      });
  if (rc != GEA_OK) return rc;
  last64 = hs.iter;
  out->iters = hs.iter;
  out->outer_iters = 0;
  out->rel_res = std::sqrt(hs.rr / hs.bb);
  out->status = hs.status == 0 ? GEA_OK : (hs.status == -4 ? GEA_ERR_NOCONV : GEA_ERR_NAN);
  return (gea_status)out->status;
}

// FP64 outer residual + FP32 inner Jacobi-PCG on the correction.
// An inner solve goes out unread behind its residual check when the same
// check did not converge last step and the solve's length is known: a batch
// of that length and a margin, then the correction and (next pass) the
// following check, both gated on the inner solve being done, so that one
// read covers all three (as the learned form's inner solves do).  When the
// batch fell short, the gated kernels did nothing and the same solve
// continues after the read.
gea_status solve_mixed(gea_ctx* x, double* xv, gea_solve_stats* out) {
  const Geo& G = x->G;
  const CgWork& w = x->w32;
  cast_system(x);
  CgVectors<float> v{x->d32, x->r32, x->r132, x->p032, x->p132, x->q32, x->q132, x->c32, x->D32, x->dinv32, x->r32};
  v.xo = xv;  // the last inner update corrects xv (launch_add_correction then does nothing)
  int total = 0;
  int outer = 0;
  CgScalars h64, h32;
  bool unread = false;
  int unread_n = 0;      // launches of the unread solve's batch
  int unread_outer = 0;  // the check it follows
  CgScalars s_res{}, s_cg{};
  auto iterate = [&](int j, bool fold, bool last) {
    x->timer.run(2, x->stream, [&] { cg_iter_kernel<float>(x->stream, G, v, j, w, fold); });
    if (last || !cg_folds(w)) x->timer.run(3, x->stream, [&] { cg_scalars(x->stream, G, j, w); });
  };
  auto last32_of = [&](int o) -> int& {
    return x->last_iters32[x->corr < 8 ? x->corr : 7][o < 3 ? o : 3];
  };
  out->rel_res0 = -1.0;
  out->status = GEA_OK;
  for (int guard = 0;; ++guard) {
    if (guard > x->prm.max_iter + 16) {
      out->status = GEA_ERR_NOCONV;
      break;
    }
    const int budget = x->prm.max_iter - total - (unread ? unread_n : 0);
    // behind an unread inner solve the check acts only if that solve is done
    residual_check(x, xv, v, budget, true, unread ? x->sc32 : nullptr);
    HIPCHK(hipGetLastError());
    if (!unread && last32_of(outer) > 0 && x->predict_unconv(outer)) {
      // (were this check converged after all, the inner system starts done,
      // its iterate zero, and the correction adds zero)
      snapshot(x, x->sc, &s_res, sizeof s_res);
      const int n = last32_of(outer);
      unread_n = n + 4 + n / 32;
      for (int j = 0; j < unread_n; ++j) iterate(j, j > 0, j == unread_n - 1);
      HIPCHK(hipGetLastError());
      snapshot(x, x->sc32, &s_cg, sizeof s_cg);
      x->timer.run(4, x->stream, [&] { launch_add_correction(x->stream, G, xv, x->d32, x->sc32, x->sc32); });
      unread = true;
      unread_outer = outer;
      ++outer;
      continue;
    }
    const bool spec = x->predict_conv(outer);
    if (spec) (*x->tail)();
    read_scalars(x, x->sc, &h64, Extra{x->sc32, &h32, sizeof h32});
    if (unread) {  // the inner solve enqueued unread, and the check before it
      unread = false;
      x->note_conv(unread_outer, s_res.done != 0);
      if (out->rel_res0 < 0) out->rel_res0 = s_res.bb > 0 ? std::sqrt(s_res.rr / s_res.bb) : 0.0;
      total += s_cg.iter;
      if (s_cg.status == -5) {
        out->status = GEA_ERR_NAN;
        break;
      }
      if (!s_cg.done) {
        // The batch ended before the solve did (h32 holds its scalars as the
        // batch left them): continue it at the next iteration, then correct.
        const int before = h32.iter;
        const int left = x->prm.max_iter - total;
        gea_status rc = run_cg(x, x->sc32, h32, left > 0 ? left : 1, 0, iterate, Extra{}, unread_n);
        if (rc != GEA_OK) return rc;
        total += h32.iter - before;
        last32_of(unread_outer) = h32.iter;
        if (h32.status == -5) {
          out->status = GEA_ERR_NAN;
          break;
        }
        x->timer.run(4, x->stream, [&] { launch_add_correction(x->stream, G, xv, x->d32, x->sc32); });
        continue;
      }
      last32_of(unread_outer) = s_cg.iter;
    }
    x->note_conv(outer, h64.done != 0);
    x->last_h64 = h64;
    const double rel = h64.bb > 0 ? std::sqrt(h64.rr / h64.bb) : 0.0;
    if (out->rel_res0 < 0) out->rel_res0 = rel;
    out->rel_res = rel;
    if (h64.status != 0) {
      out->status = GEA_ERR_NAN;
      break;
    }
    if (h64.bb == 0.0) {
      HIPCHK(hipMemsetAsync(xv, 0, sizeof(double) * G.nc, x->stream));
      out->rel_res = 0.0;
      break;
    }
    if (h64.done) {
      x->tail_done = spec;
      break;
    }
    if (total >= x->prm.max_iter) {
      out->status = GEA_ERR_NOCONV;
      break;
    }
    int& last32 = last32_of(outer);
    const int first = last32 > 0 ? (int)(0.9 * last32) : 0;
    gea_status rc = run_cg(
        x, x->sc32, h32, budget, first,
        [&](int j, bool fold, bool last) { iterate(j, fold, last); },
        Extra{}, 0, x->prm.solver == GEA_LEARNED_MIXED);
    if (rc != GEA_OK) return rc;
    last32 = h32.iter;
    total += h32.iter;
    ++outer;
    if (h32.status == -5) {
      out->status = GEA_ERR_NAN;
      break;
    }
    x->timer.run(4, x->stream, [&] { launch_add_correction(x->stream, G, xv, x->d32, x->sc32); });
  }
  out->iters = total;
  out->outer_iters = outer;
  return (gea_status)out->status;
}

// the flexible CG's vectors on the inner FP32 system (no copy of the
// starting residual: see learned_inner)
FcgVectors& fcg_vectors(gea_ctx* x) {
  FcgVectors& v = x->fv;
  v.d = x->d32;
  v.r = x->r32;
  v.r_old = x->r_old32;
  v.z = x->z32;
  v.p0 = x->p032;
  v.p1 = x->p132;
  v.q = x->q32;
  v.r0 = nullptr;
  v.c = x->c32;
  v.D = x->D32;
  v.dinv = x->dinv32;
  return v;
}

// Flexible CG with the network as preconditioner on the FP32 correction
// system set up by the refinement residual (r32, c32, D32): enqueues at most
// `steps` iterations and returns how many it enqueued.  The host reads the
// flexible-CG scalars only between iterations, never after the last one:
// the caller reads them with its next read of the solver scalars.  (After
// the stop decision the iteration kernels return at once.)  With several
// steps the set-up keeps the starting residual in q132 (the resumed
// Jacobi-PCG first writes it at its iteration 1) for fcg_handover; a single
// step forms the resume's partials itself: *res_parts is their count.
int learned_inner(gea_ctx* x, int budget, int steps, int* res_parts) {
  const Geo& G = x->G;
  FcgVectors& v = fcg_vectors(x);
  if (steps > 1) v.r0 = x->q132;
  *res_parts = 0;
  // the first application is timed (set-up, network and flexible-CG step)
  const bool timed = x->t_net_ms < 0 && !x->net_probe;
  if (timed) HIPCHK(hipEventRecord(x->ev_net[0], x->stream));
  x->timer.run(4, x->stream, [&] { fcg_start(x->stream, G, v, x->sc32, budget, x->fsc); });
  const int cap = steps < budget ? steps : budget;
  int it = 0;
  while (it < cap) {
    if (it > 0) {
      FcgScalars hf;
      const Extra part{x->fsc, &hf, sizeof hf};
      read_structs(x, &part, 1);
      if (hf.done) break;
    }
    x->timer.run(6, x->stream, [&] {
      cnn_input_from_residual(x->net, x->r32, &x->fsc->inv_s, x->c32, x->dinv32);
      cnn_forward_scaled(x->net, &x->fsc->s, x->z32);
    });
    const bool last = it + 1 == cap;
    x->timer.run(2, x->stream, [&] {
      const int n = fcg_iteration_after_z(x->stream, G, v, it, last, x->fsc);
      if (last) *res_parts = n;
    });
    HIPCHK(hipGetLastError());
    ++it;
    if (timed && it == 1) {
      HIPCHK(hipEventRecord(x->ev_net[1], x->stream));
      x->net_probe = 1;
    }
  }
  return it;
}

// FP64 refinement whose inner solves use the learned preconditioner; when
// an inner solve stalls the rest of this solve uses Jacobi-PCG (fallback).
gea_status solve_learned(gea_ctx* x, double* xv, gea_solve_stats* out) {
  if (!x->has_net) return solve_mixed(x, xv, out);
  if (!x->net_now) {  // the gate chose the refinement alone for this solve
    gea_status rc = solve_mixed(x, xv, out);
    if (rc == GEA_OK && out->outer_iters > 0) net_gate(x).record(false, out->iters, x->t_net_ms, x->t_iter_ms);
    return rc;
  }
  const Geo& G = x->G;
  const CgWork& w = x->w32;
  cast_system(x);
  CgVectors<float> v{x->d32, x->r32, x->r132, x->p032, x->p132, x->q32, x->q132, x->c32, x->D32, x->dinv32, x->r32};
  v.xo = xv;  // (as in solve_mixed)
  int total = 0, outer = 0, fallbacks = 0;
  bool use_net = true;
  CgScalars h64, h32;
  // An inner solve enqueued without a host read: the scalars of the residual
  // check before it (s_res) and of its flexible-CG and Jacobi-PCG parts
  // (s_fcg, s_cg) arrive as snapshots with the next read.
  bool unread = false;
  int unread_bound = 0;  // iterations it may have taken
  int unread_first = 0;  // Jacobi-PCG launches enqueued with it
  CgScalars s_res{}, s_cg{};
  FcgScalars s_fcg{};
  auto iterate = [&](int j, bool fold, bool last) {
    x->timer.run(2, x->stream, [&] { cg_iter_kernel<float>(x->stream, G, v, j, w, fold); });
    if (last || !cg_folds(w)) x->timer.run(3, x->stream, [&] { cg_scalars(x->stream, G, j, w); });
  };
  // network step(s), then Jacobi-PCG resumed from their iterate and residual
  // (when the flexible CG has converged the resumed solve starts done and its
  // iteration kernels return at once); returns the network steps enqueued
  auto learned_then_resume = [&](int budget) {
    int res_parts = 0;
    const int launched = learned_inner(x, budget, x->prm.learned_steps, &res_parts);
    const int left = budget - launched;
    // (one step: its one iteration was the last, so res_parts > 0; several:
    // the starting residual was kept)
    x->timer.run(4, x->stream, [&] {
      if (res_parts > 0)
        cg_resume_scalars(x->stream, x->fv.part_d, res_parts, w, left > 0 ? left : 0);
      else
        fcg_handover(x->stream, G, x->fv, w, left > 0 ? left : 0, x->fsc);
    });
    return launched;
  };
  out->rel_res0 = -1.0;
  out->status = GEA_OK;
  for (int guard = 0;; ++guard) {
    if (guard > x->prm.max_iter + 16) {
      out->status = GEA_ERR_NOCONV;
      break;
    }
    const int budget = x->prm.max_iter - total - unread_bound;
    // behind an unread inner solve the check acts only if that solve is done
    residual_check(x, xv, v, budget, !use_net, unread ? x->sc32 : nullptr);
    HIPCHK(hipGetLastError());
    // The learned inner solve goes out unread behind this check when the
    // same check did not converge last step and the resumed Jacobi-PCG's
    // length is known: a first batch of that length and a margin, then the
    // correction, then (next pass) the following check; one read then covers
    // all.  (Were this check converged, the inner system starts done and the
    // correction adds zero.)  The correction and the check are gated on the
    // inner solve being done: when the batch fell short they do nothing, and
    // after the read the same Jacobi-PCG continues where the batch ended.
    if (use_net && !unread && x->last_iters_res > 0 && x->predict_unconv(outer)) {
      snapshot(x, x->sc, &s_res, sizeof s_res);
      const int launched = learned_then_resume(budget > 0 ? budget : 1);
      use_net = false;
      unread_first = x->last_iters_res + 4 + x->last_iters_res / 32;
      for (int j = 0; j < unread_first; ++j) iterate(j, j > 0, j == unread_first - 1);
      HIPCHK(hipGetLastError());
      snapshot(x, x->sc32, &s_cg, sizeof s_cg);
      snapshot(x, x->fsc, &s_fcg, sizeof s_fcg);
      x->timer.run(4, x->stream, [&] { launch_add_correction(x->stream, G, xv, x->d32, x->sc32, x->sc32); });
      unread = true;
      unread_bound = launched + unread_first;
      ++outer;
      continue;
    }
    const bool spec = x->predict_conv(outer);
    if (spec) (*x->tail)();
    read_scalars(x, x->sc, &h64, Extra{x->sc32, &h32, sizeof h32});
    if (unread) {  // the inner solve enqueued unread, and the check before it
      unread = false;
      unread_bound = 0;
      x->note_conv(0, s_res.done != 0);
      if (out->rel_res0 < 0) out->rel_res0 = s_res.bb > 0 ? std::sqrt(s_res.rr / s_res.bb) : 0.0;
      total += s_cg.iter + s_fcg.iter;
      x->last_iters_res = s_cg.iter;
      if (s_fcg.status == 1) ++fallbacks;  // stalled: Jacobi-PCG took over
      if (s_cg.status == -5) {
        out->status = GEA_ERR_NAN;
        break;
      }
      if (!s_cg.done) {
        // The batch ended before the resumed Jacobi-PCG: the gated correction
        // and check did nothing (h32 holds the solve's scalars as the batch
        // left them).  Continue it at the next iteration, then correct.
        const int before = h32.iter;
        const int left = x->prm.max_iter - total;
        gea_status rc = run_cg(x, x->sc32, h32, left > 0 ? left : 1, 0, iterate, Extra{},
                               unread_first);
        if (rc != GEA_OK) return rc;
        total += h32.iter - before;
        x->last_iters_res = h32.iter;
        if (h32.status == -5) {
          out->status = GEA_ERR_NAN;
          break;
        }
        x->timer.run(4, x->stream, [&] { launch_add_correction(x->stream, G, xv, x->d32, x->sc32); });
        continue;
      }
    }
    x->note_conv(outer, h64.done != 0);
    x->last_h64 = h64;
    const double rel = h64.bb > 0 ? std::sqrt(h64.rr / h64.bb) : 0.0;
    if (out->rel_res0 < 0) out->rel_res0 = rel;
    out->rel_res = rel;
    if (h64.status != 0) {
      out->status = GEA_ERR_NAN;
      break;
    }
    if (h64.bb == 0.0) {
      HIPCHK(hipMemsetAsync(xv, 0, sizeof(double) * G.nc, x->stream));
      out->rel_res = 0.0;
      break;
    }
    if (h64.done) {
      x->tail_done = spec;
      break;
    }
    if (total >= x->prm.max_iter) {
      out->status = GEA_ERR_NOCONV;
      break;
    }
    int done_iters = 0;
    FcgScalars hf{};
    Extra fcg;  // the flexible-CG scalars, read along with the CG's
    const int last32 = x->last_iters32[x->corr < 8 ? x->corr : 7][outer < 3 ? outer : 3];
    int first = last32 > 0 ? (int)(0.9 * last32) : 0;
    if (use_net) {
      learned_then_resume(budget > 0 ? budget : 1);
      use_net = false;
      h32 = CgScalars{};
      fcg = Extra{x->fsc, &hf, sizeof hf};
      first = x->last_iters_res > 0 ? x->last_iters_res + 4 : 0;
    }
    gea_status rc = run_cg(x, x->sc32, h32, budget, first, iterate, fcg, 0, true);
    if (rc != GEA_OK) return rc;
    done_iters += h32.iter;
    if (fcg.bytes) {
      x->last_iters_res = h32.iter;
      done_iters += hf.iter;
      if (hf.status == 1) ++fallbacks;  // stalled: Jacobi-PCG took over
    }
    if (h32.status == -5) {
      out->status = GEA_ERR_NAN;
      break;
    }
    total += done_iters;
    ++outer;
    // a stalled learned correction is still a descent step: keep it
    x->timer.run(4, x->stream, [&] { launch_add_correction(x->stream, G, xv, x->d32, x->sc32); });
  }
  out->iters = total;
  out->outer_iters = outer;
  out->fallbacks = fallbacks;
  x->fallbacks += fallbacks;
  if (out->status == GEA_OK && outer > 0) net_gate(x).record(true, total, x->t_net_ms, x->t_iter_ms);
  return (gea_status)out->status;
}

gea_status solve(gea_ctx* x, double* xv, gea_solve_stats* out) {
  *out = gea_solve_stats{};
  if (x->prm.solver == GEA_PCG_JACOBI_FP64) return solve_pcg64(x, xv, out);
  if (x->prm.solver == GEA_LEARNED_MIXED) return solve_learned(x, xv, out);
  return solve_mixed(x, xv, out);
}

// One energy sweep's system (Step 2), set up by the RHS pass: Jacobi-PCG in
// FP64 on (c, D = (mu/Pr) c_p, 1/diag, b) from the initial guess in T, to kEnergyTol.
gea_status solve_energy(gea_ctx* x, double* T, int nparts, int sweep, int* iters) {
  const Geo& G = x->G;
  const CgWork& w = x->w64;
  // D = (mu/Pr) c_p in every cell: the iteration kernels take it as a value
  // and form 1/diag from c (no 1/diag array)
  CgVectors<double> v{T, x->r, x->r1, x->p0, x->p1, x->q, x->q1, x->c, nullptr, nullptr, x->b,
                      x->prm.mu / x->prm.Pr * x->prm.cp};
  x->timer.run(7, x->stream, [&] {
    cg_start_from(x->stream, w.u[1], nparts, w.b, kEnergyTol, x->prm.max_iter, w.sc);
  });
  CgScalars hs{};  // rr = 0: the first read supplies the starting residual
  int& last = x->last_iters_energy[sweep < 8 ? sweep : 7];
  gea_status rc = run_cg(
      x, x->sc, hs, x->prm.max_iter, last > 0 ? last + 1 : 0,
      [&](int j, bool fold, bool last) {
        x->timer.run(7, x->stream, [&] {
          cg_iter_kernel<double>(x->stream, G, v, j, w, fold);
          if (last || !cg_folds(w)) cg_scalars(x->stream, G, j, w);
        });
      });
  if (rc != GEA_OK) return rc;
  last = hs.iter;
  *iters = hs.iter;
  if (hs.status == -4) {
    x->err = "energy solve did not converge";
    return GEA_ERR_NOCONV;
  }
  if (hs.status != 0) return GEA_ERR_NAN;
  return GEA_OK;
}

// Steps 1 and 2 from state s; the last energy sweep writes T_out; p' is
// copied to pp_out when given (the pressure solve's initial guess).  Each
// energy sweep solves its implicit-diffusion system for T (pressure-solve
// work vectors, which are free until Step 3).
// Implicit transport (transport = 1): the momentum operator of component
// comp and the energy operator (unknown T) of Steps 1 and 2, with the
// state's face flux
TrOp momentum_op(const gea_ctx* x, const State& S, int comp) {
  const Geo& G = x->G;
  TrOp op{};
  op.rho_star = x->rho_star;
  op.tcoef = G.V / x->ph.dt;
  op.gamma = 1.0;
  op.wall_comp = comp;
  for (int d = 0; d < G.ndim; ++d) {
    op.phi[d] = S.phi[d];
    op.k[d] = x->ph.mu * G.S[d] / G.h[d];
  }
  return op;
}

TrOp energy_op(const gea_ctx* x, const State& S, bool enth) {
  const Geo& G = x->G;
  TrOp op{};
  op.rho_star = x->rho_star;
  op.tcoef = (enth ? x->ph.cp : x->ph.cv) * G.V / x->ph.dt;
  op.gamma = x->ph.cp;
  op.wall_comp = -1;
  for (int d = 0; d < G.ndim; ++d) {
    op.phi[d] = S.phi[d];
    op.k[d] = x->ph.mu / x->ph.Pr * x->ph.cp * G.S[d] / G.h[d];
  }
  return op;
}

// One BiCGStab solve behind its enqueued set-up: iterations in batches
// (doubling up to 16), the scalars read once a batch.
gea_status bicg_run(gea_ctx* x, const TrOp& op, double* xv, int* iters) {
  const Geo& G = x->G;
  x->timer.run(7, x->stream, [&] {
    launch_tr_start(x->stream, G, x->partials, kTransportTol, x->prm.max_iter, x->tsc);
  });
  TrScalars hs{};
  int batch = 2;
  long launched = 0;
  for (;;) {
    for (int k = 0; k < batch; ++k)
      x->timer.run(7, x->stream, [&] {
        launch_tr_iteration(x->stream, G, op, xv, x->trv, x->partials, x->tsc);
      });
    HIPCHK(hipGetLastError());
    launched += batch;
    const Extra part{x->tsc, &hs, sizeof hs};
    read_structs(x, &part, 1);
    if (hs.done) break;
    if (launched > (long)x->prm.max_iter + 32) {
      x->err = "implicit transport solve: the solver never finished";
      return GEA_ERR_NOCONV;
    }
    batch = batch < 16 ? 2 * batch : 16;
  }
  if (hs.bb == 0.0) launch_fill(x->stream, G, xv, 0.0);  // b = 0: x = 0
  *iters = hs.iter;
  if (hs.status == 0) return GEA_OK;
  x->err = hs.status == -5 ? "non-finite value in an implicit transport solve"
                           : "implicit transport solve did not converge";
  return hs.status == -5 ? GEA_ERR_NAN : GEA_ERR_NOCONV;
}

// the current state's p^{n-1}, K^{n-1}: its own p^n, K^n if it has none
void ensure_history(gea_ctx* x) {
  if (x->hist[x->cur]) return;
  const State& S = x->st[x->cur];
  launch_history_init(x->stream, x->G, S.p, S.u, S.pm, S.Km);
  HIPCHK(hipGetLastError());
  x->hist[x->cur] = true;
}

gea_status steps_1_2(gea_ctx* x, const State& S, double* T_out, double* pp_out = nullptr,
                     int64_t* energy_iters = nullptr, int64_t* transport_iters = nullptr) {
  const Geo& G = x->G;
  const Phys& ph = x->ph;
  hipStream_t s = x->stream;
  const bool enth = x->prm.energy_form == 1;
  const bool implicit = x->prm.transport == 1;
  x->timer.run(5, x->stream, [&] {
    // (explicit transport: K* into ea for the energy sweeps)
    launch_step1(s, G, ph, S.rho, S.u, S.T, S.pp, S.phi, x->rho_star, x->e0, x->ustar, pp_out,
                 implicit ? x->trb : nullptr, implicit ? nullptr : x->ea);
  });
  if (implicit) {
    // Step 1's momentum predictor implicit: per component from the explicit
    // predictor's u*, with the right-hand side Step 1's pass wrote
    for (int d = 0; d < G.ndim; ++d) {
      const TrOp op = momentum_op(x, S, d);
      TrVecs v = x->trv;
      v.b = x->trb[d];
      x->timer.run(7, x->stream, [&] { launch_tr_setup_mom(s, G, op, x->ustar[d], v, x->partials); });
      int its = 0;
      gea_status rc = bicg_run(x, op, x->ustar[d], &its);
      if (transport_iters) *transport_iters += its;
      if (rc != GEA_OK) return rc;
    }
    if (enth) {
      const State& N = x->st[1 - x->cur];
      ensure_history(x);
      x->timer.run(5, x->stream, [&] {
        launch_enthalpy_prep(s, G, ph, S.rho, S.T, S.p, S.pm, S.Km, S.u, x->ustar, x->rho_star,
                             x->e0, N.pm, N.Km);
      });
    }
    // Step 2 in one implicit solve for T
    const TrOp op = energy_op(x, S, enth);
    x->timer.run(7, x->stream, [&] {
      launch_tr_setup_energy(s, G, ph, enth, op, S.rho, x->e0, x->ustar, x->ea, S.T, x->Tbg, T_out,
                             x->trv, x->partials);
    });
    int its = 0;
    gea_status rc = bicg_run(x, op, T_out, &its);
    if (transport_iters) *transport_iters += its;
    if (rc != GEA_OK) return rc;
    x->timer.run(5, x->stream, [&] {
      launch_energy_post(s, G, ph, T_out, S.p, x->rho_star, x->rho23, x->psi, x->c, x->D);
    });
    x->sys32 = false;
    return GEA_OK;
  }
  const double* Ks = x->ea;  // K*, from Step 1
  if (enth) {
    // e0 becomes the sweep-independent balance; the next state's p^n, K^n go
    // to the other state's history arrays
    const State& N = x->st[1 - x->cur];
    ensure_history(x);
    x->timer.run(5, x->stream, [&] {
      launch_enthalpy_prep(s, G, ph, S.rho, S.T, S.p, S.pm, S.Km, S.u, x->ustar, x->rho_star,
                           x->e0, N.pm, N.Km);
    });
  }
  const double* T_prev = S.T;
  const int ns = x->prm.n_energy_sweeps;
  for (int sw = 0; sw < ns; ++sw) {
    const bool last = sw == ns - 1;
    // the first total-energy sweep transports e^n + R T^n; every other sweep
    // forms its transported quantity from T^(s-1) and K*.  Every sweep solves
    // into T_out: after the first, the initial guess is already there.
    const bool ks = enth || sw > 0;
    double* T_next = T_out;
    int nparts = 0;
    x->timer.run(5, x->stream, [&] {
      nparts = launch_energy_rhs(s, G, ph, enth, ks, S.rho, x->e0, ks ? Ks : x->e0, T_prev, S.phi,
                                 x->rho_star, Ks, x->Tbg, x->b, x->c,
                                 T_next == T_prev ? nullptr : T_next, x->r, x->w64.u[1], x->w64.b);
    });
    HIPCHK(hipGetLastError());
    int its = 0;
    gea_status rc = solve_energy(x, T_next, nparts, sw, &its);
    if (energy_iters) *energy_iters += its;
    if (rc != GEA_OK) return rc;
    if (last)
      x->timer.run(5, x->stream, [&] {
        launch_energy_post(s, G, ph, T_next, S.p, x->rho_star, x->rho23, x->psi, x->c, x->D);
      });
    T_prev = T_next;
  }
  x->sys32 = false;  // c and D changed
  return GEA_OK;
}

gea_status one_step(gea_ctx* x, gea_step_stats* stats) {
  const Geo& G = x->G;
  const Phys& ph = x->ph;
  hipStream_t s = x->stream;
  const State& S = x->st[x->cur];
  const State& N = x->st[1 - x->cur];
  {
    gea_status rc = steps_1_2(x, S, N.T, N.pp, &stats->energy_iters, &stats->transport_iters);
    if (rc != GEA_OK) return rc;
  }
  const int nc = x->prm.n_corr;
  stats->n_solves = 0;
  for (int k = 0; k < nc; ++k) {
    const bool last = k == nc - 1;
    x->corr = k;  // (the learned form's gate decides per corrector, before the assembly)
    x->timer.run(5, x->stream, [&] { launch_H(s, G, ph, S.rho, S.u, x->ustar, S.phi, x->H); });
    // (c, D and 1/diag change only in Step 2: later correctors form b only)
    x->timer.run(5, x->stream, [&] { build_system(x, S, N.pp, k == 0); });
    HIPCHK(hipGetLastError());
    x->has_system = true;
    double* uo[3] = {x->ustar[0], x->ustar[1], x->ustar[2]};
    if (last)
      for (int d = 0; d < 3; ++d) uo[d] = N.u[d];
    const std::function<void()> correct = [&] {
      x->timer.run(5, x->stream, [&] { launch_correct(s, G, ph, N.pp, x->rho23, x->psi, x->H, x->D, x->rho_star, uo, last, S.rho,
                     N.rho, N.p, N.phi, x->partials, x->sc); });
    };
    gea_solve_stats ss;
    x->tail = &correct;
    x->tail_done = false;
    x->corr = k;
    gea_status rc = solve(x, N.pp, &ss);
    x->tail = nullptr;
    stats->solve[stats->n_solves++] = ss;
    stats->total_iters += ss.iters;
    stats->total_solves += 1;
    stats->total_fallbacks += ss.fallbacks;
    if (ss.rel_res > stats->max_rel_res) stats->max_rel_res = ss.rel_res;
    if (rc != GEA_OK) return rc;
    if (!x->tail_done) correct();
    HIPCHK(hipGetLastError());
  }
  // the end-of-step reductions land in the FP64 scalars: already read when
  // the last correction ran ahead of the last residual check's read
  CgScalars hs;
  if (x->tail_done)
    hs = x->last_h64;
  else
    read_scalars(x, x->sc, &hs);
  stats->mass = hs.aux[0];
  stats->eos_mismatch = hs.aux[1];
  if (hs.aux[2] != 0.0) return GEA_ERR_NAN;
  // the enthalpy form's Step 2 wrote the new state's p^{n-1}, K^{n-1}
  x->hist[1 - x->cur] = x->prm.energy_form == 1;
  x->cur = 1 - x->cur;
  stats->steps_done += 1;
  return GEA_OK;
}

gea_status fail(gea_ctx* x, gea_status st, const std::string& msg) {
  if (x) x->err = msg;
  return st;
}

hipMemcpyKind kind_in(gea_ptr_kind k) {
  return k == GEA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_out(gea_ptr_kind k) {
  return k == GEA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

template <typename F>
gea_status guarded(gea_ctx* x, F&& f) {
  try {
    return f();
  } catch (const HipError& e) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e.e, hipGetErrorString(e.e),
                  e.what);
    return fail(x, GEA_ERR_HIP, buf);
  } catch (const std::bad_alloc&) {
    return fail(x, GEA_ERR_ALLOC, "host allocation failed");
  } catch (...) {
    return fail(x, GEA_ERR_HIP, "unexpected exception");
  }
}

}  // namespace

extern "C" {

gea_status gea_workspace_bytes(const gea_mesh* mesh, const gea_params* params, size_t* bytes) {
  std::string err;
  gea_status st = check_params(mesh, params, err);
  if (st != GEA_OK) {
    g_init_error = err;
    return st;
  }
  if (!bytes) return GEA_ERR_ARG;
  gea_ctx tmp;
  Carver cv(nullptr);
  *bytes = carve(cv, &tmp, *mesh, params->solver == GEA_LEARNED_MIXED, params->transport == 1);
  return GEA_OK;
}

gea_status gea_init_mesh(const gea_mesh* mesh, const gea_params* params, void* hip_stream,
                         void* workspace, size_t workspace_bytes, gea_ctx** out) {
  std::string err;
  if (!out) {
    g_init_error = "null output pointer";
    return GEA_ERR_ARG;
  }
  *out = nullptr;
  gea_status st = check_params(mesh, params, err);
  if (st != GEA_OK) {
    g_init_error = err;
    return st;
  }
  size_t need = 0;
  gea_workspace_bytes(mesh, params, &need);
  if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
    g_init_error = "workspace missing, smaller than gea_workspace_bytes, or not 256-byte aligned";
    return GEA_ERR_ARG;
  }
  gea_ctx* x = new (std::nothrow) gea_ctx();
  if (!x) {
    g_init_error = "context allocation failed";
    return GEA_ERR_ALLOC;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&x->pin), gea_ctx::kPinBytes, hipHostMallocDefault) !=
      hipSuccess) {
    x->pin = nullptr;
    delete x;
    g_init_error = "pinned host buffer allocation failed";
    return GEA_ERR_ALLOC;
  }
  x->mesh = *mesh;
  x->prm = *params;
  x->stream = static_cast<hipStream_t>(hip_stream);
  x->net.s = x->stream;
  setup_geometry(x);
  Carver cv(workspace);
  carve(cv, x, *mesh, params->solver == GEA_LEARNED_MIXED, params->transport == 1);
  gea_status rc = guarded(x, [&]() {
    // zero the solver scalars once
    HIPCHK(hipMemsetAsync(x->sc, 0, sizeof(CgScalars), x->stream));
    HIPCHK(hipMemsetAsync(x->sc32, 0, sizeof(CgScalars), x->stream));
    HIPCHK(hipGetLastError());
    for (hipEvent_t* e : {&x->ev_net[0], &x->ev_net[1], &x->ev_it[0], &x->ev_it[1]})
      HIPCHK(hipEventCreate(e));
    HIPCHK(hipStreamSynchronize(x->stream));
    return GEA_OK;
  });
  if (rc != GEA_OK) {
    g_init_error = x->err;
    delete x;
    return rc;
  }
  *out = x;
  return GEA_OK;
}

gea_status gea_set_solver(gea_ctx* x, int32_t solver, double tol, int32_t max_iter,
                          double inner_tol) {
  if (!x) return GEA_ERR_ARG;
  if (solver == GEA_LEARNED_MIXED && !x->has_net_space)
    return fail(x, GEA_ERR_STATE, "learned form needs a context created with it (network buffers)");
  gea_params q = x->prm;
  q.solver = solver;
  q.tol = tol;
  q.max_iter = max_iter;
  q.inner_tol = inner_tol;
  std::string err;
  gea_status st = check_params(&x->mesh, &q, err);
  if (st != GEA_OK) return fail(x, st, err);
  x->prm = q;
  return GEA_OK;
}

gea_status gea_init_bubble(gea_ctx* x, const gea_bubble* b) {
  if (!x) return GEA_ERR_ARG;
  if (!b || b->kind < 0 || b->kind > 2 || !(b->rc > 0) || !std::isfinite(b->amp))
    return fail(x, GEA_ERR_ARG, "bad bubble");
  return guarded(x, [&]() {
    const State& S = x->st[x->cur];
    launch_init_column(x->stream, x->G, x->ph, x->rho_a, x->pp_a, x->Tbg);
    launch_init_fields(x->stream, x->G, x->ph, b->kind, b->xc, b->yc, b->zc, b->rc, b->amp,
                       x->rho_a, x->pp_a, x->Tbg, S.rho, S.u, S.T, S.pp, S.p);
    launch_face_mass_flux(x->stream, x->G, S.rho, S.u, S.phi);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(x->stream));
    x->has_state = true;
    x->hist[x->cur] = false;
    x->has_system = false;
    return GEA_OK;
  });
}

gea_status gea_set_state(gea_ctx* x, const double* rho, const double* u, const double* T,
                         const double* p_prime, const double* p, const double* T_bg,
                         gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!rho || !u || !T || !p_prime || !p || !T_bg) return fail(x, GEA_ERR_ARG, "null field");
  return guarded(x, [&]() {
    const State& S = x->st[x->cur];
    const size_t n = sizeof(double) * x->G.nc;
    hipStream_t s = x->stream;
    HIPCHK(hipMemcpyAsync(S.rho, rho, n, kind_in(kind), s));
    for (int d = 0; d < x->G.ndim; ++d)
      HIPCHK(hipMemcpyAsync(S.u[d], u + (size_t)d * x->G.nc, n, kind_in(kind), s));
    HIPCHK(hipMemcpyAsync(S.T, T, n, kind_in(kind), s));
    HIPCHK(hipMemcpyAsync(S.pp, p_prime, n, kind_in(kind), s));
    HIPCHK(hipMemcpyAsync(S.p, p, n, kind_in(kind), s));
    HIPCHK(hipMemcpyAsync(x->Tbg, T_bg, sizeof(double) * x->G.nz, kind_in(kind), s));
    launch_face_mass_flux(s, x->G, S.rho, S.u, S.phi);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    x->has_state = true;
    x->hist[x->cur] = false;
    x->has_system = false;
    return GEA_OK;
  });
}

gea_status gea_set_face_flux(gea_ctx* x, const double* phi, gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!phi) return fail(x, GEA_ERR_ARG, "null flux");
  if (!x->has_state) return fail(x, GEA_ERR_STATE, "no state: call gea_init_bubble or gea_set_state");
  return guarded(x, [&]() {
    const State& S = x->st[x->cur];
    const size_t n = sizeof(double) * x->G.nc;
    for (int d = 0; d < x->G.ndim; ++d)
      HIPCHK(hipMemcpyAsync(S.phi[d], phi + (size_t)d * x->G.nc, n, kind_in(kind), x->stream));
    launch_clear_wall_faces(x->stream, x->G, S.phi);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(x->stream));
    return GEA_OK;
  });
}

gea_status gea_set_history(gea_ctx* x, const double* p_prev, const double* K_prev,
                           gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!p_prev || !K_prev) return fail(x, GEA_ERR_ARG, "null field");
  if (!x->has_state) return fail(x, GEA_ERR_STATE, "no state: call gea_init_bubble or gea_set_state");
  return guarded(x, [&]() {
    const State& S = x->st[x->cur];
    const size_t n = sizeof(double) * x->G.nc;
    HIPCHK(hipMemcpyAsync(S.pm, p_prev, n, kind_in(kind), x->stream));
    HIPCHK(hipMemcpyAsync(S.Km, K_prev, n, kind_in(kind), x->stream));
    HIPCHK(hipStreamSynchronize(x->stream));
    x->hist[x->cur] = true;
    return GEA_OK;
  });
}

gea_status gea_step(gea_ctx* x, int32_t nsteps, gea_step_stats* stats) {
  if (!x) return GEA_ERR_ARG;
  if (nsteps < 0) return fail(x, GEA_ERR_ARG, "nsteps < 0");
  if (!x->has_state) return fail(x, GEA_ERR_STATE, "no state: call gea_init_bubble or gea_set_state");
  gea_step_stats local{};
  gea_step_stats* st = stats ? stats : &local;
  *st = gea_step_stats{};
  return guarded(x, [&]() {
    for (int n = 0; n < nsteps; ++n) {
      gea_status rc = one_step(x, st);
      if (rc != GEA_OK) {
        HIPCHK(hipStreamSynchronize(x->stream));
        return fail(x, rc, rc == GEA_ERR_NOCONV ? "pressure solve did not converge; step rolled back"
                                                : "non-finite value; step rolled back");
      }
    }
    return GEA_OK;
  });
}

gea_status gea_pressure_solve(gea_ctx* x, const double* b, double* xv, gea_ptr_kind kind,
                              gea_solve_stats* stats) {
  if (!x) return GEA_ERR_ARG;
  if (!xv) return fail(x, GEA_ERR_ARG, "null x");
  if (!x->has_state) return fail(x, GEA_ERR_STATE, "no state");
  gea_solve_stats local{};
  gea_solve_stats* st = stats ? stats : &local;
  return guarded(x, [&]() {
    const Geo& G = x->G;
    hipStream_t s = x->stream;
    const State& S = x->st[x->cur];
    const State& N = x->st[1 - x->cur];
    {
      gea_status rc = steps_1_2(x, S, N.T);
      if (rc != GEA_OK) return fail(x, rc, "energy solve failed");
    }
    x->corr = 0;
    x->timer.run(5, x->stream, [&] { launch_H(s, G, x->ph, S.rho, S.u, x->ustar, S.phi, x->H); });
    x->timer.run(5, x->stream, [&] { build_system(x, S); });
    HIPCHK(hipGetLastError());
    const size_t n = sizeof(double) * G.nc;
    if (b) HIPCHK(hipMemcpyAsync(x->b, b, n, kind_in(kind), s));
    HIPCHK(hipMemcpyAsync(x->xs, xv, n, kind_in(kind), s));
    x->has_system = true;
    gea_status rc = solve(x, x->xs, st);
    HIPCHK(hipMemcpyAsync(xv, x->xs, n, kind_out(kind), s));
    HIPCHK(hipStreamSynchronize(s));
    if (rc != GEA_OK) return fail(x, rc, "pressure solve failed");
    return GEA_OK;
  });
}

gea_status gea_apply_pressure_operator(gea_ctx* x, const double* xin, double* y,
                                       gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!xin || !y) return fail(x, GEA_ERR_ARG, "null vector");
  if (!x->has_system) return fail(x, GEA_ERR_STATE, "no assembled pressure system");
  return guarded(x, [&]() {
    const size_t n = sizeof(double) * x->G.nc;
    HIPCHK(hipMemcpyAsync(x->xs, xin, n, kind_in(kind), x->stream));
    launch_apply_A(x->stream, x->G, x->c, x->D, x->xs, x->r64);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(y, x->r64, n, kind_out(kind), x->stream));
    HIPCHK(hipStreamSynchronize(x->stream));
    return GEA_OK;
  });
}

gea_status gea_state_extrema(gea_ctx* x, gea_extrema* out) {
  if (!x) return GEA_ERR_ARG;
  if (!out) return fail(x, GEA_ERR_ARG, "null output");
  if (!x->has_state) return fail(x, GEA_ERR_STATE, "no state");
  return guarded(x, [&]() {
    const State& S = x->st[x->cur];
    launch_extrema(x->stream, x->G, x->ph, S.u, S.T, S.p, x->o_part, x->ext);
    HIPCHK(hipGetLastError());
    double v[8];
    const Extra part{x->ext, v, sizeof v};
    read_structs(x, &part, 1);
    *out = gea_extrema{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
    return GEA_OK;
  });
}

gea_status gea_get_fields(gea_ctx* x, uint32_t mask, double* out, gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!out) return fail(x, GEA_ERR_ARG, "null output");
  if (!x->has_state) return fail(x, GEA_ERR_STATE, "no state");
  if ((mask & (GEA_FIELD_C | GEA_FIELD_D | GEA_FIELD_B)) && !x->has_system)
    return fail(x, GEA_ERR_STATE, "no assembled pressure system");
  return guarded(x, [&]() {
    const State& S = x->st[x->cur];
    const size_t n = (size_t)x->G.nc;
    size_t off = 0;
    auto put = [&](const double* src) {
      HIPCHK(hipMemcpyAsync(out + off, src, n * sizeof(double), kind_out(kind), x->stream));
      off += n;
    };
    if (mask & GEA_FIELD_RHO) put(S.rho);
    if (mask & GEA_FIELD_U)
      for (int d = 0; d < x->G.ndim; ++d) put(S.u[d]);
    if (mask & GEA_FIELD_T) put(S.T);
    if (mask & GEA_FIELD_PPRIME) put(S.pp);
    if (mask & GEA_FIELD_P) put(S.p);
    if (mask & GEA_FIELD_C) put(x->c);
    if (mask & GEA_FIELD_D) put(x->D);
    if (mask & GEA_FIELD_B) put(x->b);
    if (mask & GEA_FIELD_PHI)
      for (int d = 0; d < x->G.ndim; ++d) put(S.phi[d]);
    if (mask & GEA_FIELD_HISTORY) {
      ensure_history(x);
      put(S.pm);
      put(S.Km);
    }
    HIPCHK(hipStreamSynchronize(x->stream));
    return GEA_OK;
  });
}

gea_status gea_kernel_timing(gea_ctx* x, int32_t on, int32_t reset) {
  if (!x) return GEA_ERR_ARG;
  return guarded(x, [&]() {
    HIPCHK(hipStreamSynchronize(x->stream));
    x->timer.flush();
    if (reset) x->timer.reset();
    x->timer.on = on != 0;
    return GEA_OK;
  });
}

gea_status gea_time_solver_kernels(gea_ctx* x, int32_t reps, double* ms) {
  if (!x || !ms || reps < 1) return GEA_ERR_ARG;
  if (!x->has_system) return fail(x, GEA_ERR_STATE, "no assembled pressure system");
  return guarded(x, [&]() {
    const Geo& G = x->G;
    hipStream_t s = x->stream;
    const State& S = x->st[x->cur];
    hipEvent_t ev[3];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    auto elapsed = [&](hipEvent_t a, hipEvent_t b) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, a, b));
      return (double)t / reps;
    };
    // FP64: a fresh solve set-up that never reports done (tol 0), its first
    // iteration, then iteration 1's kernels (an update pending, as in every
    // later iteration) launched back to back
    HIPCHK(hipMemcpyAsync(x->xs, S.pp, sizeof(double) * G.nc, hipMemcpyDeviceToDevice, s));
    CgVectors<double> v{x->xs, x->r, x->r1, x->p0, x->p1, x->q, x->q1, x->c, x->D, x->dinv, x->b};
    cg_init<double>(s, G, v, x->w64, 0.0, 1 << 30);
    cg_iter_kernel<double>(s, G, v, 0, x->w64, false);
    cg_scalars(s, G, 0, x->w64);
    cg_iter_kernel<double>(s, G, v, 1, x->w64, true);  // warm-up
    HIPCHK(hipEventRecord(ev[0], s));
    for (int k = 0; k < reps; ++k) cg_iter_kernel<double>(s, G, v, 1, x->w64, true);
    HIPCHK(hipEventRecord(ev[1], s));
    for (int k = 0; k < reps; ++k) cg_scalars(s, G, 1, x->w64);
    HIPCHK(hipEventRecord(ev[2], s));
    HIPCHK(hipEventSynchronize(ev[2]));
    ms[0] = elapsed(ev[0], ev[1]);
    ms[1] = elapsed(ev[1], ev[2]);
    // FP32 inner kernels on the refinement's set-up (outer tol 0: not done)
    launch_cast_coeffs(s, G, x->c, x->D, x->dinv, x->c32, x->D32, x->dinv32);
    CgVectors<float> v32{x->d32, x->r32, x->r132, x->p032, x->p132, x->q32, x->q132, x->c32, x->D32, x->dinv32, x->r32};
    launch_residual64(s, G, x->c, x->D, x->b, x->xs, v32, 0.0, 1e-30, 0.1, 1 << 30, x->o_part,
                      x->w32, x->sc);
    cg_iter_kernel<float>(s, G, v32, 0, x->w32, false);
    cg_scalars(s, G, 0, x->w32);
    cg_iter_kernel<float>(s, G, v32, 1, x->w32, true);
    HIPCHK(hipEventRecord(ev[0], s));
    for (int k = 0; k < reps; ++k) cg_iter_kernel<float>(s, G, v32, 1, x->w32, true);
    HIPCHK(hipEventRecord(ev[1], s));
    for (int k = 0; k < reps; ++k) cg_scalars(s, G, 1, x->w32);
    HIPCHK(hipEventRecord(ev[2], s));
    HIPCHK(hipEventSynchronize(ev[2]));
    ms[2] = elapsed(ev[0], ev[1]);
    ms[3] = elapsed(ev[1], ev[2]);
    for (auto& e : ev) HIPCHK(hipEventDestroy(e));
    HIPCHK(hipGetLastError());
    return GEA_OK;
  });
}

gea_status gea_time_network(gea_ctx* x, int32_t reps, double* ms, double* gflop) {
  if (!x || !ms || !gflop || reps < 1) return GEA_ERR_ARG;
  if (!x->has_net) return fail(x, GEA_ERR_STATE, "no network weights loaded");
  return guarded(x, [&]() {
    hipStream_t s = x->stream;
    x->net.s = s;
    hipEvent_t ev[2];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    for (int l = 0; l < kCnnLayers; ++l) {
      cnn_conv_layer(x->net, l);  // warm-up
      HIPCHK(hipEventRecord(ev[0], s));
      for (int k = 0; k < reps; ++k) cnn_conv_layer(x->net, l);
      HIPCHK(hipEventRecord(ev[1], s));
      HIPCHK(hipEventSynchronize(ev[1]));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
      ms[l] = (double)t / reps;
      gflop[l] = cnn_layer_flops(x->net, l) * 1e-9;
    }
    for (auto& e : ev) HIPCHK(hipEventDestroy(e));
    HIPCHK(hipGetLastError());
    return GEA_OK;
  });
}

gea_status gea_kernel_times(gea_ctx* x, double* ms, int64_t* launches) {
  if (!x || !ms || !launches) return GEA_ERR_ARG;
  return guarded(x, [&]() {
    HIPCHK(hipStreamSynchronize(x->stream));
    x->timer.flush();
    for (int k = 0; k < 8; ++k) {
      ms[k] = x->timer.ms[k];
      launches[k] = x->timer.launches[k];
    }
    return GEA_OK;
  });
}

gea_status gea_load_weights(gea_ctx* x, const float* params, gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!params) return fail(x, GEA_ERR_ARG, "null params");
  if (!x->has_net_space)
    return fail(x, GEA_ERR_STATE,
                "no network buffers: create the context with the learned solver on a mesh whose "
                "dimensions are multiples of 4");
  return guarded(x, [&]() {
    x->net.s = x->stream;
    HIPCHK(hipMemcpyAsync(x->net.master, params, sizeof(float) * x->net.nparams, kind_in(kind),
                          x->stream));
    cnn_pack_weights(x->net);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(x->stream));
    x->has_net = true;
    return GEA_OK;
  });
}

gea_status gea_make_pair(gea_ctx* x, double rel_tol, float* in_r, float* in_a, float* out_d,
                         double* scale, gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!in_r || !in_a || !out_d || !(rel_tol > 0)) return fail(x, GEA_ERR_ARG, "bad pair arguments");
  if (!x->has_state) return fail(x, GEA_ERR_STATE, "no state");
  return guarded(x, [&]() {
    const Geo& G = x->G;
    hipStream_t s = x->stream;
    const State& S = x->st[x->cur];
    const State& N = x->st[1 - x->cur];
    {
      gea_status rc = steps_1_2(x, S, N.T);
      if (rc != GEA_OK) return fail(x, rc, "energy solve failed");
    }
    launch_H(s, G, x->ph, S.rho, S.u, x->ustar, S.phi, x->H);
    build_system(x, S);
    // r0 = b - A p'  (FP64), then the tight FP64 solve from x0 = p'
    launch_apply_A(s, G, x->c, x->D, S.pp, x->r64);
    const size_t n = sizeof(double) * G.nc;
    HIPCHK(hipMemcpyAsync(x->xs, S.pp, n, hipMemcpyDeviceToDevice, s));
    launch_sub(s, G, x->b, x->r64);
    gea_params keep = x->prm;
    x->prm.tol = rel_tol;
    x->prm.max_iter = 200000;
    gea_solve_stats st;
    gea_status rc = solve_pcg64(x, x->xs, &st);
    x->prm = keep;
    if (rc != GEA_OK) return fail(x, rc, "pair solve failed");
    float* tr = in_r;
    float* ta = in_a;
    float* td = out_d;
    if (kind == GEA_HOST) {  // stage through device scratch (the FP32 work vectors)
      tr = x->r_old32;
      ta = x->z32;
      td = x->q32;
    }
    pair_outputs(s, G, x->r64, x->c, x->dinv, x->xs, S.pp, x->pair_part, x->pair_s, tr, ta, td);
    HIPCHK(hipGetLastError());
    if (kind == GEA_HOST) {
      const size_t nf = sizeof(float) * G.nc;
      HIPCHK(hipMemcpyAsync(in_r, tr, nf, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(in_a, ta, nf, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(out_d, td, nf, hipMemcpyDeviceToHost, s));
    }
    double hs[2];
    HIPCHK(hipMemcpyAsync(hs, x->pair_s, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (scale) *scale = hs[0];
    x->has_system = true;
    return GEA_OK;
  });
}

gea_status gea_learned_apply(gea_ctx* x, const float* r, float* z, double* scale,
                             gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!r || !z || !scale) return fail(x, GEA_ERR_ARG, "null argument");
  if (!x->has_net) return fail(x, GEA_ERR_STATE, "no network weights loaded");
  if (!x->has_system) return fail(x, GEA_ERR_STATE, "no assembled pressure system");
  return guarded(x, [&]() {
    const Geo& G = x->G;
    hipStream_t s = x->stream;
    cast_system(x);
    HIPCHK(hipMemcpyAsync(x->r32, r, sizeof(float) * G.nc, kind_in(kind), s));
    // the flexible CG's set-up forms s = max |r| and 1/s on the device
    fcg_start(s, G, fcg_vectors(x), x->sc32, 1, x->fsc);
    cnn_input_from_residual(x->net, x->r32, &x->fsc->inv_s, x->c32, x->dinv32);
    cnn_forward_scaled(x->net, &x->fsc->s, x->z32);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(z, x->z32, sizeof(float) * G.nc, kind_out(kind), s));
    FcgScalars hf;
    const Extra part{x->fsc, &hf, sizeof hf};
    read_structs(x, &part, 1);
    *scale = hf.s;
    return GEA_OK;
  });
}

gea_status gea_learned_activation(gea_ctx* x, int32_t which, float* out, gea_ptr_kind kind) {
  if (!x) return GEA_ERR_ARG;
  if (!out || which < 0 || which > 9) return fail(x, GEA_ERR_ARG, "bad activation");
  if (!x->has_net) return fail(x, GEA_ERR_STATE, "no network weights loaded");
  return cnn_copy_activation(x->net, which, out, kind, x->err);
}

void gea_destroy(gea_ctx* x) { delete x; }

const char* gea_last_error(const gea_ctx* x) {
  return x ? x->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
