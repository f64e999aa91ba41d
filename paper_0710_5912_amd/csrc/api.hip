// api.hip -- the C ABI of include/le.h.
//
// One engine serves both entry families: a single run (le_ctx) is an engine
// with one run, a batch (le_batch) an engine with many.  Runs are grouped in
// classes of equal (nx, ny, precision, inertial); each stage of a step is one
// launch per class covering all of its runs (grid z = run), so a step of a
// 96-run batch is a handful of launches, and chunks of steps are captured
// once into a HIP graph and replayed.  The shear clock of every run is kept
// on the host; the per-step strain offsets reach the kernels through a
// device table [step][run] refreshed once per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/le.h"
#include "../../include/le_train.h"
#include "cnn.hpp"
#include "common.hpp"
#include "ops.hpp"

using namespace le;

namespace {

constexpr int64_t kChunkCap = 1024;  // steps per host chunk
constexpr int64_t kProfChunk = 256;  // steps per chunk while stage timing is on
constexpr int kRealBlocks = 1024;    // blocks of the real-space reduction
constexpr int64_t kGraphMin = 8;     // shortest chunk worth capturing
constexpr int64_t kGraphChunk = 128; // longest captured chunk (longer graphs replay slower)
constexpr size_t kGraphCacheMax = 16;  // holds every power-of-two piece of both step kinds

thread_local char g_last_error[256] = "";

int fail_hip(hipError_t e, const char* what, int line) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (line %d): %s", what, line,
                hipGetErrorString(e));
  return LE_EDEVICE;
}

#define LE_TRY(expr)                                                  \
  do {                                                                \
    const hipError_t le_e_ = (expr);                                  \
    if (le_e_ != hipSuccess) return fail_hip(le_e_, #expr, __LINE__); \
  } while (0)

#define LE_RC(expr)            \
  do {                         \
    const int le_rc_ = (expr); \
    if (le_rc_) return le_rc_; \
  } while (0)

// ---- shear clock (section "Numerical method": the sawtooth s(t)) --------
// Evaluated without contraction so it rounds exactly like a plain evaluation
// of gdot * (n * dt) and of the subtraction of c * k.
#pragma clang fp contract(off)
double strain_total(const le_params& p, int64_t n) { return p.gdot * ((double)n * p.dt); }
int64_t wrap_count(const le_params& p, int64_t n) {
  const double c = p.lx / p.ly;
  return (int64_t)std::floor((strain_total(p, n) + 0.5 * c) / c);
}
double strain_offset(const le_params& p, int64_t n) {
  const double c = p.lx / p.ly;
  return strain_total(p, n) - c * (double)wrap_count(p, n);
}
// The sawtooth at the midpoint of step n, t = (n + 1/2) dt, in the frame of
// step n (wrap count k_n): the LE_SCHEME_MIDPOINT_S variant.
double strain_offset_mid(const le_params& p, int64_t n) {
  const double c = p.lx / p.ly;
  return p.gdot * (((double)n + 0.5) * p.dt) - c * (double)wrap_count(p, n);
}
#pragma clang fp contract(on)

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const le_params* p) {
  if (!p) return LE_EINVAL;
  if (!pow2_in(p->nx, 8, 4096) || !pow2_in(p->ny, 8, 4096)) return LE_EINVAL;
  if (!finite_pos(p->lx) || !finite_pos(p->ly)) return LE_EINVAL;
  if (!std::isfinite(p->gdot)) return LE_EINVAL;
  if (!finite_pos(p->A) || !finite_pos(p->B) || !finite_pos(p->kappa) || !finite_pos(p->M))
    return LE_EINVAL;
  if (!finite_pos(p->eta) || !std::isfinite(p->rho) || p->rho < 0.0) return LE_EINVAL;
  if (!finite_pos(p->dt)) return LE_EINVAL;
  if (p->precision != LE_FP64 && p->precision != LE_FP32) return LE_EINVAL;
  if (p->gdot != 0.0 && (p->nx < p->ny || p->nx % p->ny != 0)) return LE_EINVAL;
  return LE_OK;
}

// Twiddle table exp(-2 pi i k / n), k < n, rounded from long double, into
// tw[0 .. 2n).
template <typename T>
void fill_twiddles(T* tw, int n) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < n; ++k) {
    const long double a = -2.0L * pi * (long double)k / (long double)n;
    tw[2 * k] = (T)std::cos(a);
    tw[2 * k + 1] = (T)std::sin(a);
  }
}
template <typename T>
std::vector<T> twiddles(int n) {
  std::vector<T> tw(2 * (size_t)n);
  fill_twiddles(tw.data(), n);
  return tw;
}

// The Geo of a validated parameter set.
Geo make_geo(const le_params& p) {
  Geo g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.r = p.nx >= p.ny ? p.nx / p.ny : 0;
  g.f_half = 0;
  g.upwind3 = 0;
  g.banded = 0;
  g.lx = p.lx;
  g.ly = p.ly;
  g.dx = p.lx / p.nx;
  g.dy = p.ly / p.ny;
  g.c = p.lx / p.ly;
  g.A = p.A;
  g.B = p.B;
  g.kappa = p.kappa;
  g.M = p.M;
  g.eta = p.eta;
  g.rho = p.rho;
  g.dt = p.dt;
  g.kx0 = 6.283185307179586476925286766559 / p.lx;
  g.ky0 = 6.283185307179586476925286766559 / p.ly;
  return g;
}

struct RunHost {
  le_params p;
  Geo g;
  bool inertial;
  size_t tsize, n_real, n_spec;
  void* buf[NBUF];
  void* twx = nullptr;
  void* twy = nullptr;
  int64_t wraps = 0;   // wrap count the stored fields are expressed in
  int cls = 0;         // class index
  int internal = 0;    // position in the class-grouped order
};

struct Class {
  int nx, ny, prec;
  bool inertial;
  Ops ops;
  // kernel variants, chosen by autotune() at creation
  int adv_variant = 0;       // Ops::advect
  int mu_variant = 0;        // Ops::mu_source
  int col_ch_variant = 0;    // Ops::column, Cahn-Hilliard pass
  int col_flow_variant = 0;  // Ops::column, flow (or Stokes) pass
  int row_variant = 0;       // Ops::row_c2r (inverse row transforms)
  int row_fwd_variant = 0;   // Ops::row_r2c (forward row transforms, also of the
                             // two-kernel stencil stages)
  bool upwind3 = false;      // LE_SCHEME_UPWIND3: the upwind advection kernel
  bool banded = false;       // LE_SCHEME_BANDED: the banded column kernels
  int advect() const { return upwind3 ? kAdvUpwind : adv_variant; }
  // Ops::column with the banded flag of the scheme
  void column(int mode, const Run* runs, int nruns, int nx, const StepArgs* sa, int bin0,
              int bin1, int bout0, int bout1, int variant, hipStream_t st) const {
    ops.column(mode | (banded ? COL_BANDED : 0), runs, nruns, nx, sa, bin0, bin1, bout0, bout1,
               variant, st);
  }
  std::vector<int> members;  // run ids
  int first = 0;             // internal index of members[0]
};

}  // namespace

struct le_ctx {
  std::vector<RunHost> runs;
  std::vector<Class> classes;
  int nruns = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t step = 0;
  Run* d_desc = nullptr;         // descriptors, internal order
  StepArgs* d_args = nullptr;    // [kChunkCap][nruns]
  StepArgs* h_args = nullptr;    // pinned
  // observables scratch (sized for the largest run)
  double* d_spart = nullptr;
  double* d_rpart = nullptr;
  double* d_bins = nullptr;
  double* d_counts = nullptr;
  double* d_gsum = nullptr;      // shell group sums, then group weights
  double* d_out = nullptr;
  double* h_out = nullptr;
  int nsblk_max = 0, nbins_max = 0;
  void* h_stage = nullptr;       // pinned staging, largest run
  size_t stage_bytes = 0;
  bool use_graphs = true;
  std::map<int64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  bool profiling = false;
  std::vector<hipEvent_t> events;  // kProfChunk * (LE_NSTAGES + 1)
  double stage_ms[LE_NSTAGES] = {0};
  int64_t stage_n[LE_NSTAGES] = {0};
  Net* net = nullptr;              // learned corrector (single inertial run)
  double* d_restrict = nullptr;    // restriction output
  // corrector audit: every `audit_every` corrected steps a window of
  // `audit_window` steps is run both corrected and plain from the same state
  // (two snapshots of phi, omega_h, psi_h); a failed audit keeps the plain
  // result and every later corrected step runs plain (until the next
  // le_corrector_load or le_corrector_audit)
  int64_t audit_every = 0, audit_window = 0, since_audit = 0, audits = 0;
  double audit_tol = 0.0, audit_dev = 0.0;
  bool corr_fallback = false;
  int corr_proj = 0;        // le_corrector_projection
  bool midpoint_s = false;  // LE_SCHEME_MIDPOINT_S
  bool recovery = false;    // le_set_recovery
  void* snap[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  // engines of several grid classes: one stream per class (default priority)
  // so that the classes' independent kernels overlap, forked from and joined
  // back into `stream` around every chunk of steps
  std::vector<hipStream_t> cls_streams;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
};

// Network with training state, driven through device pointers.
struct le_cnn {
  Net net;
};

// A batch handle owns an engine of many runs.
struct le_batch {
  le_ctx* e;
};

namespace {

using Engine = le_ctx;

const Run* desc(const Engine* e, const RunHost& r) { return e->d_desc + r.internal; }

// Drops the cached graphs whose key keep() rejects.  The stream is drained
// first, so no dropped graph is still executing.
template <typename Keep>
void drop_graphs(Engine* e, Keep&& keep) {
  bool any = false;
  for (const auto& kv : e->graphs) any = any || !keep(kv.first);
  if (!any) return;
  (void)hipStreamSynchronize(e->stream);
  for (auto it = e->graphs.begin(); it != e->graphs.end();) {
    if (!keep(it->first)) {
      (void)hipGraphExecDestroy(it->second.second);
      (void)hipGraphDestroy(it->second.first);
      it = e->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

void release(Engine* e) {
  for (auto& kv : e->graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  e->graphs.clear();
  for (hipEvent_t ev : e->events)
    if (ev) (void)hipEventDestroy(ev);
  e->events.clear();
  for (auto& r : e->runs) {
    for (void*& b : r.buf)
      if (b) (void)hipFree(b);
    if (r.twx) (void)hipFree(r.twx);
    if (r.twy) (void)hipFree(r.twy);
  }
  void* dev[] = {e->d_desc,   e->d_args,   e->d_spart, e->d_rpart,
                 e->d_bins,   e->d_counts, e->d_gsum,  e->d_out};
  for (void* d : dev)
    if (d) (void)hipFree(d);
  if (e->h_args) (void)hipHostFree(e->h_args);
  if (e->h_out) (void)hipHostFree(e->h_out);
  if (e->h_stage) (void)hipHostFree(e->h_stage);
  if (e->net) {
    net_destroy(e->net);
    delete e->net;
    e->net = nullptr;
  }
  if (e->d_restrict) (void)hipFree(e->d_restrict);
  for (auto& sn : e->snap)
    for (void*& b : sn)
      if (b) {
        (void)hipFree(b);
        b = nullptr;
      }
  for (hipStream_t cs : e->cls_streams)
    if (cs) (void)hipStreamDestroy(cs);
  e->cls_streams.clear();
  for (hipEvent_t ev : e->join_ev)
    if (ev) (void)hipEventDestroy(ev);
  e->join_ev.clear();
  if (e->fork_ev) (void)hipEventDestroy(e->fork_ev);
  if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
}

int alloc(void** p, size_t bytes) {
  return hipMalloc(p, bytes) == hipSuccess ? LE_OK : LE_ENOMEM;
}

int upload_real(Engine* e, const RunHost& r, const double* src, int b) {
  if (r.tsize == sizeof(double)) {
    std::memcpy(e->h_stage, src, r.n_real * sizeof(double));
  } else {
    float* s = static_cast<float*>(e->h_stage);
    for (size_t i = 0; i < r.n_real; ++i) s[i] = (float)src[i];
  }
  LE_TRY(hipMemcpyAsync(r.buf[b], e->h_stage, r.n_real * r.tsize, hipMemcpyHostToDevice,
                        e->stream));
  LE_TRY(hipStreamSynchronize(e->stream));
  return LE_OK;
}

int download_real(Engine* e, const RunHost& r, int b, double* dst) {
  LE_TRY(hipMemcpyAsync(e->h_stage, r.buf[b], r.n_real * r.tsize, hipMemcpyDeviceToHost,
                        e->stream));
  LE_TRY(hipStreamSynchronize(e->stream));
  if (r.tsize == sizeof(double)) {
    std::memcpy(dst, e->h_stage, r.n_real * sizeof(double));
  } else {
    const float* s = static_cast<const float*>(e->h_stage);
    for (size_t i = 0; i < r.n_real; ++i) dst[i] = (double)s[i];
  }
  return LE_OK;
}

// StepArgs of run r at step n into the table slot d_args[r.internal].
int set_args_one(Engine* e, const RunHost& r, int64_t n) {
  StepArgs* h = e->h_args + r.internal;
  h->s = strain_offset(r.p, n);
  h->pad = 0.0;
  LE_TRY(hipMemcpyAsync(e->d_args + r.internal, h, sizeof(StepArgs), hipMemcpyHostToDevice,
                        e->stream));
  return LE_OK;
}

// psi of run r from the flow constraint at the current step (Poisson from
// omega, or the Stokes solve from phi); omega's row spectrum must be current.
int solve_psi(Engine* e, const RunHost& r) {
  LE_RC(set_args_one(e, r, e->step));
  const Class& k = e->classes[r.cls];
  const StepArgs* sa = e->d_args + r.internal;
  if (r.inertial) {
    k.column(COL_POISSON, desc(e, r), 1, r.p.nx, sa, B_OM_S, B_OM_S, B_PS_S, B_PS_S, 0,
                 e->stream);
  } else {
    k.ops.mu_source(desc(e, r), 1, r.p.ny, sa, k.mu_variant, k.row_fwd_variant, e->stream);
    k.column(COL_STOKES, desc(e, r), 1, r.p.nx, sa, B_GH, B_GH, B_PS_S, B_PS_S,
                 k.col_flow_variant, e->stream);
  }
  LE_TRY(hipGetLastError());
  return LE_OK;
}

// The stages of one step for every run; sa: the step's row of the table.
// ev: LE_NSTAGES + 1 events recorded around the stages when timing.
void enqueue_step(Engine* e, const StepArgs* sa, hipEvent_t* ev) {
  auto mark = [&](int k) {
    if (ev) (void)hipEventRecord(ev[k], e->stream);
  };
  hipStream_t st = e->stream;
  mark(0);
  for (const Class& k : e->classes) {
    const Run* d = e->d_desc + k.first;
    const int n = (int)k.members.size();
    if (k.inertial)
      k.ops.row_c2r(d, n, k.ny, B_OM_S, B_OM_R, B_PS_S, B_PS_R, 2, k.row_variant, st);
    else
      k.ops.row_c2r(d, n, k.ny, B_PS_S, B_PS_R, B_PS_S, B_PS_R, 1, k.row_variant, st);
  }
  mark(1);
  for (const Class& k : e->classes)
    k.ops.advect(e->d_desc + k.first, (int)k.members.size(), k.ny, sa + k.first, k.inertial,
                 k.advect(), k.row_fwd_variant, st);
  mark(2);
  for (const Class& k : e->classes)
    k.column(COL_CH, e->d_desc + k.first, (int)k.members.size(), k.nx, sa + k.first,
                 B_PHIH, B_FH, B_PHIN, B_PHIN, k.col_ch_variant, st);
  mark(3);
  for (const Class& k : e->classes)
    k.ops.row_c2r(e->d_desc + k.first, (int)k.members.size(), k.ny, B_PHIN, B_PHI, B_PHIN,
                  B_PHI, 1, k.row_variant, st);
  mark(4);
  for (const Class& k : e->classes)
    k.ops.mu_source(e->d_desc + k.first, (int)k.members.size(), k.ny, sa + k.first,
                    k.mu_variant, k.row_fwd_variant, st);
  mark(5);
  for (const Class& k : e->classes) {
    if (k.inertial)
      k.column(COL_FLOW, e->d_desc + k.first, (int)k.members.size(), k.nx, sa + k.first,
                   B_OMH, B_GH, B_OM_S, B_PS_S, k.col_flow_variant, st);
    else
      k.column(COL_STOKES, e->d_desc + k.first, (int)k.members.size(), k.nx,
                   sa + k.first, B_GH, B_GH, B_PS_S, B_PS_S, k.col_flow_variant, st);
  }
  mark(6);
}

// Enqueue `count` steps whose StepArgs rows are d_args[0 .. count).  Chunks
// of at least kGraphMin steps are captured once per length into a HIP graph
// and replayed (the strain offsets stay in device memory, so one graph
// serves every chunk of that length).  Stage timing brackets direct launches
// with events, so timed chunks are never captured.
// Enqueue `count` steps through enqueue_one(k, events): replayed from the
// graph cached under `key` when there is one, else captured (chunks of at
// least kGraphMin steps, when not timing stages) or launched directly.
template <typename F>
int enqueue_chunk(Engine* e, int64_t key, int64_t count, F&& enqueue_one);

// Copy the chunk's StepArgs rows h_args[0 .. count) to the device and
// enqueue the chunk through launch(n) (n steps, rows at d_args[0 .. n)).
// With graphs on, the chunk runs as power-of-two pieces, largest first, each
// piece's rows copied to the start of d_args (stream order keeps a piece's
// copy behind the previous piece's kernels): chunks of any length then
// replay the same few captured graphs instead of capturing one per length.
template <typename F>
int enqueue_pieces(Engine* e, int64_t count, size_t row, F&& launch) {
  const bool split = e->use_graphs && !e->profiling;
  int64_t k0 = 0;
  while (k0 < count) {
    int64_t n = count - k0;
    if (split) {
      int64_t b = 1;
      while (2 * b <= n) b *= 2;
      n = b;
    }
    LE_TRY(hipMemcpyAsync(e->d_args, e->h_args + (size_t)k0 * row,
                          (size_t)n * row * sizeof(StepArgs), hipMemcpyHostToDevice, e->stream));
    LE_RC(launch(n));
    k0 += n;
  }
  return LE_OK;
}

template <typename F>
int enqueue_chunk(Engine* e, int64_t key, int64_t count, F&& enqueue_one) {
  const bool graph_ok = e->use_graphs && count >= kGraphMin && !e->profiling;
  auto it = graph_ok ? e->graphs.find(key) : e->graphs.end();
  if (graph_ok && it == e->graphs.end()) {
    if (e->graphs.size() >= kGraphCacheMax) {
      auto old = e->graphs.begin();
      (void)hipStreamSynchronize(e->stream);  // the evicted graph may still run
      (void)hipGraphExecDestroy(old->second.second);
      (void)hipGraphDestroy(old->second.first);
      e->graphs.erase(old);
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    int rc = LE_OK;
    hipError_t err = hipStreamBeginCapture(e->stream, hipStreamCaptureModeRelaxed);
    if (err == hipSuccess) {
      for (int64_t k = 0; k < count && rc == LE_OK; ++k) rc = enqueue_one(k, nullptr);
      err = hipStreamEndCapture(e->stream, &g);
      if (rc != LE_OK && err == hipSuccess) err = hipErrorUnknown;
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
      // leave capture mode, drop the partial graph and launch directly
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(e->stream, &cs) == hipSuccess &&
          cs != hipStreamCaptureStatusNone) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(e->stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
      }
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      fail_hip(err, "graph capture (falling back to direct launches)", __LINE__);
      e->use_graphs = false;
    } else {
      it = e->graphs.emplace(key, std::make_pair(g, ge)).first;
    }
  }
  if (it != e->graphs.end()) {
    LE_TRY(hipGraphLaunch(it->second.second, e->stream));
    return LE_OK;
  }
  for (int64_t k = 0; k < count; ++k)
    LE_RC(enqueue_one(k, e->profiling ? &e->events[(size_t)k * (LE_NSTAGES + 1)] : nullptr));
  return LE_OK;
}

// One step of one class on stream st (the stages of enqueue_step).
// The stages of one step of n runs of class k (descriptors d, StepArgs a);
// with inverse == false the real omega and psi are taken as they are (the
// inverse row transforms of stage 0 are skipped).
void enqueue_runs_step(const Class& k, const Run* d, int n, const StepArgs* a, hipStream_t st,
                       bool inverse = true) {
  if (inverse) {
    if (k.inertial)
      k.ops.row_c2r(d, n, k.ny, B_OM_S, B_OM_R, B_PS_S, B_PS_R, 2, k.row_variant, st);
    else
      k.ops.row_c2r(d, n, k.ny, B_PS_S, B_PS_R, B_PS_S, B_PS_R, 1, k.row_variant, st);
  }
  k.ops.advect(d, n, k.ny, a, k.inertial, k.advect(), k.row_fwd_variant, st);
  k.column(COL_CH, d, n, k.nx, a, B_PHIH, B_FH, B_PHIN, B_PHIN, k.col_ch_variant, st);
  k.ops.row_c2r(d, n, k.ny, B_PHIN, B_PHI, B_PHIN, B_PHI, 1, k.row_variant, st);
  k.ops.mu_source(d, n, k.ny, a, k.mu_variant, k.row_fwd_variant, st);
  if (k.inertial)
    k.column(COL_FLOW, d, n, k.nx, a, B_OMH, B_GH, B_OM_S, B_PS_S, k.col_flow_variant, st);
  else
    k.column(COL_STOKES, d, n, k.nx, a, B_GH, B_GH, B_PS_S, B_PS_S, k.col_flow_variant,
                 st);
}

void enqueue_class_step(const Engine* e, const Class& k, const StepArgs* sa, hipStream_t st) {
  enqueue_runs_step(k, e->d_desc + k.first, (int)k.members.size(), sa + k.first, st);
}

// Enqueue `count` plain steps whose StepArgs rows are d_args[0 .. count)
// (one graph per chunk length serves every chunk of that length: the strain
// offsets stay in device memory).  Stage timing brackets direct launches
// with events, so timed chunks are never captured.  With several classes
// (and no stage timing) each class runs the whole chunk on its own stream
// between a fork and a join on the engine's stream.
int enqueue_steps(Engine* e, int64_t count) {
  const size_t row = (size_t)e->nruns;
  if (!e->cls_streams.empty() && !e->profiling) {
    return enqueue_chunk(e, count, count, [&](int64_t k, hipEvent_t*) {
      const size_t nc = e->classes.size();
      if (k == 0) {
        if (hipEventRecord(e->fork_ev, e->stream) != hipSuccess) return (int)LE_EDEVICE;
        for (size_t c = 0; c < nc; ++c)
          if (hipStreamWaitEvent(e->cls_streams[c], e->fork_ev, 0) != hipSuccess)
            return (int)LE_EDEVICE;
      }
      for (size_t c = 0; c < nc; ++c)
        enqueue_class_step(e, e->classes[c], e->d_args + k * row, e->cls_streams[c]);
      if (k + 1 == count) {
        for (size_t c = 0; c < nc; ++c) {
          if (hipEventRecord(e->join_ev[c], e->cls_streams[c]) != hipSuccess ||
              hipStreamWaitEvent(e->stream, e->join_ev[c], 0) != hipSuccess)
            return (int)LE_EDEVICE;
        }
      }
      return (int)LE_OK;
    });
  }
  return enqueue_chunk(e, count, count, [&](int64_t k, hipEvent_t* ev) {
    enqueue_step(e, e->d_args + k * row, ev);
    return LE_OK;
  });
}

// Re-express run r's state after its strain offset jumped by -dk c.
void enqueue_remap(Engine* e, const RunHost& r, int64_t dk) {
  const int dkr = (int)((dk * (int64_t)r.g.r) % r.p.nx);
  const Ops& o = e->classes[r.cls].ops;
  o.remap_real(desc(e, r), B_PHI, B_TMP, dkr, e->stream);
  o.copy_real(desc(e, r), B_TMP, B_PHI, e->stream);
  o.remap_spec(desc(e, r), B_PS_S, dkr, e->stream);
  if (r.inertial) o.remap_spec(desc(e, r), B_OM_S, dkr, e->stream);
}

void harvest_times(Engine* e, int64_t count) {
  for (int64_t k = 0; k < count; ++k) {
    hipEvent_t* ev = &e->events[(size_t)k * (LE_NSTAGES + 1)];
    for (int s = 0; s < LE_NSTAGES; ++s) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[s], ev[s + 1]) == hipSuccess) {
        e->stage_ms[s] += ms;
        e->stage_n[s] += 1;
      }
    }
  }
}

// Sums of run r's observables into h_out (OBS_NTOTAL values + 2 nbins).
int reduce_observables(Engine* e, const RunHost& r, bool spectral) {
  const Ops& o = e->classes[r.cls].ops;
  const int nbins = r.p.ny / 2;
  int nsblk = 0;
  if (spectral) {
    LE_RC(set_args_one(e, r, e->step));
    o.row_r2c(desc(e, r), 1, r.p.ny, B_PHI, B_PHIH, e->classes[r.cls].row_fwd_variant,
              e->stream);
    o.obs_spectral(desc(e, r), r.p.nx, e->d_args + r.internal, B_PHIH,
                   r.inertial ? B_PS_S : -1, e->d_spart, e->d_bins, e->d_counts, e->stream);
    nsblk = o.obs_blocks(r.p.nx);
  }
  o.obs_real(desc(e, r), B_PHI, e->d_rpart, kRealBlocks, e->stream);
  launch_obs_final(e->d_spart, nsblk, e->d_rpart, kRealBlocks, e->d_bins, e->d_counts,
                   spectral ? nbins : 0, e->d_gsum, e->d_out, e->stream);
  LE_TRY(hipGetLastError());
  const size_t nout = OBS_NTOTAL + (spectral ? 2 * (size_t)nbins : 0);
  LE_TRY(hipMemcpyAsync(e->h_out, e->d_out, nout * sizeof(double), hipMemcpyDeviceToHost,
                        e->stream));
  LE_TRY(hipStreamSynchronize(e->stream));
  return LE_OK;
}

int observables_of(Engine* e, const RunHost& r, le_obs* o, double* Sk, int32_t sk_cap) {
  LE_RC(reduce_observables(e, r, true));
  const double* h = e->h_out;
  const double N = (double)r.n_real;
  const int nbins = r.p.ny / 2;
  le_obs v;
  std::memset(&v, 0, sizeof(v));
  v.step = e->step;
  v.wraps = r.wraps;
  v.t = (double)e->step * r.p.dt;
  v.strain = strain_total(r.p, e->step);
  v.s = strain_offset(r.p, e->step);
  v.mean_phi = h[OBS_SUM_PHI] / N;
  v.phi2 = h[OBS_SUM_PHI2] / N;
  v.Ls = h[OBS_SUM_S_NZ] > 0.0 ? h[OBS_SUM_S_OVER_Q] / h[OBS_SUM_S_NZ] : 0.0;
  const double l = std::sqrt(r.p.kappa / r.p.A);
  const double tot = h[OBS_SUM_S];
  v.Dxx = tot > 0.0 ? l * h[OBS_XX] / tot : 0.0;
  v.Dxy = tot > 0.0 ? l * h[OBS_XY] / tot : 0.0;
  v.Dyy = tot > 0.0 ? l * h[OBS_YY] / tot : 0.0;
  const double mid = 0.5 * (v.Dxx + v.Dyy);
  const double rad = std::sqrt(0.25 * (v.Dxx - v.Dyy) * (v.Dxx - v.Dyy) + v.Dxy * v.Dxy);
  const double hi = mid + rad, lo = mid - rad;
  v.L_perp = hi > 0.0 ? 1.0 / hi : INFINITY;
  v.L_par = lo > 0.0 ? 1.0 / lo : INFINITY;
  v.sigma_xy = -r.p.kappa * h[OBS_XY] / N;
  v.sigma_xy_re = r.inertial ? r.p.rho * h[OBS_RE] / (N * N) : 0.0;
  v.nbins = nbins;
  v.dk = 6.283185307179586476925286766559 / r.p.ly;
  v.finite = h[OBS_NONFINITE] == 0.0 ? 1 : 0;
  if (Sk) {
    const int nb = sk_cap < nbins ? sk_cap : nbins;
    for (int b = 0; b < nb; ++b) {
      const double w = h[OBS_NTOTAL + nbins + b];
      Sk[b] = w > 0.0 ? h[OBS_NTOTAL + b] / w : 0.0;
    }
  }
  *o = v;
  return LE_OK;
}

// Build an engine for n runs; on failure everything is released.
// ---------------------------------------------------------------- autotuner
//
// Each class (runs sharing nx, ny, precision, inertia) picks its kernel
// variants by timing every candidate on its own buffers at creation: the
// advect and mu/source variants (fused kernel vs strip stencil over 4 .. 32
// row strips) and the column block shapes of both column passes.  The timed
// launches read the state and write only step temporaries (the flow pass is
// timed into the spectral scratch buffers), so the state is untouched.
// LE_TUNE_<STAGE>=v (ADV, MU, COL_CH, COL_FLOW) fixes a variant instead, for
// tests that exercise every path.
namespace {

constexpr int kRowCand[] = {0, 1, 2, 3, 4, 5};
constexpr int kAdvCand[] = {0, kAdvBatch + 4, kAdvBatch + 8, kAdvBatch + 16,
                             2,  4,  8,  16, 32, kStripFft + 2, kStripFft + 4,
                             kStripFft + 8, kStripFft1 + 2, kStripFft1 + 4, kStripFft1 + 8,
                             kAdvBatch2 + 2, kAdvBatch2 + 4, kAdvBatch2 + 8,
                             kAdvBatch3 + 2, kAdvBatch3 + 4, kAdvBatch3 + 8};
constexpr int kMuCand[] = {0, kAdvBatch + 4, kAdvBatch + 8, kAdvBatch + 16,
                            2, 4, 8, 16, 32, kStripFft + 2, kStripFft + 4, kStripFft + 8,
                            kAdvBatch2 + 2, kAdvBatch2 + 4, kAdvBatch2 + 8,
                            kAdvBatch3 + 2, kAdvBatch3 + 4, kAdvBatch3 + 8};
constexpr int kColCand[] = {0, 1, 2, 3, 4};

int env_variant(const char* name) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : -1;
}

// Milliseconds of 3 launches of f.
template <typename F>
int time_launches(Engine* e, hipEvent_t a, hipEvent_t b, F&& f, float* ms) {
  LE_TRY(hipEventRecord(a, e->stream));
  for (int i = 0; i < 3; ++i) f();
  LE_TRY(hipEventRecord(b, e->stream));
  LE_TRY(hipEventSynchronize(b));
  LE_TRY(hipGetLastError());
  LE_TRY(hipEventElapsedTime(ms, a, b));
  return LE_OK;
}

// Every candidate is launched once untimed (code loading, clocks), then
// timed in three rounds (alternating orders), keeping each candidate's best.
// A later candidate replaces the current choice only when it is faster by
// more than kTuneMargin: near-ties keep the earlier candidate, so the choice
// does not follow the timing noise from one context to the next.  The lists
// put first the shapes that re-read the fewest halo rows (the four-row
// batches): back-to-back timing finds re-read rows in the last-level cache,
// which the step does not.
constexpr float kTuneMargin = 0.02f;
template <size_t N, typename F>
int pick(Engine* e, hipEvent_t a, hipEvent_t b, const int (&cand)[N], const char* env, int* out,
         F&& launch) {
  const int forced = env_variant(env);
  if (forced >= 0) {
    *out = forced;
    return LE_OK;
  }
  for (size_t i = 0; i < N; ++i) launch(cand[i]);
  float best[N];
  for (size_t i = 0; i < N; ++i) best[i] = 3.4e38f;
  for (int round = 0; round < 3; ++round) {
    for (size_t j = 0; j < N; ++j) {
      const size_t i = round % 2 == 0 ? j : N - 1 - j;
      float ms = 0.0f;
      LE_RC(time_launches(e, a, b, [&] { launch(cand[i]); }, &ms));
      if (ms < best[i]) best[i] = ms;
    }
  }
  size_t w = 0;
  for (size_t i = 1; i < N; ++i)
    if (best[i] < best[w] * (1.0f - kTuneMargin)) w = i;
  *out = cand[w];
  const char* log = std::getenv("LE_TUNE_LOG");
  if (log && log[0] == '1') {
    std::fprintf(stderr, "le tune %s:", env);
    for (size_t i = 0; i < N; ++i) std::fprintf(stderr, " %d=%.1fus", cand[i], best[i] * 1e3f / 3);
    std::fprintf(stderr, " -> %d\n", cand[w]);
  }
  return LE_OK;
}

// Tuning cache: the choices of every (device, nx, ny, precision, inertia,
// runs in the class) tuned so far in this process, so later contexts of the
// same shape take the same kernels (equal results, no re-timing); with
// LE_TUNE_CACHE=<file> also kept on disk across processes (one line per
// entry: the key's six integers, then the six variants).  LE_TUNE_CACHE=off
// re-times every context.  Variants fixed by LE_TUNE_* still apply.
struct TuneEntry {
  int key[6];
  int val[6];  // advect, mu_source, column_ch, column_flow, row, row_fwd
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
bool g_tune_loaded = false;

const char* tune_cache_path() {
  const char* p = std::getenv("LE_TUNE_CACHE");
  return (p && p[0] && std::strcmp(p, "off") != 0) ? p : nullptr;
}
bool tune_cache_off() {
  const char* p = std::getenv("LE_TUNE_CACHE");
  return p && std::strcmp(p, "off") == 0;
}

void tune_key(const Class& k, int dev, int* key) {
  const int v[6] = {dev, k.nx, k.ny, k.prec, k.inertial ? 1 : 0, (int)k.members.size()};
  std::memcpy(key, v, sizeof(v));
}

// Caller holds g_tune_mu.
void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  TuneEntry t;
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %d", &t.key[0], &t.key[1], &t.key[2],
                     &t.key[3], &t.key[4], &t.key[5], &t.val[0], &t.val[1], &t.val[2],
                     &t.val[3], &t.val[4], &t.val[5]) == 12)
    g_tune.push_back(t);
  std::fclose(f);
}

bool tune_cache_find(const int* key, int* val) {
  for (const TuneEntry& t : g_tune)
    if (std::memcmp(t.key, key, sizeof(t.key)) == 0) {
      std::memcpy(val, t.val, sizeof(t.val));
      return true;
    }
  return false;
}

void tune_cache_add(const int* key, const int* val) {
  TuneEntry t;
  std::memcpy(t.key, key, sizeof(t.key));
  std::memcpy(t.val, val, sizeof(t.val));
  g_tune.push_back(t);
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d\n", key[0], key[1], key[2], key[3], key[4],
               key[5], val[0], val[1], val[2], val[3], val[4], val[5]);
  std::fclose(f);
}

int autotune(Engine* e) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return LE_EDEVICE;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  const bool cache = !tune_cache_off();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (cache) tune_cache_load();
  int rc = LE_OK;
  for (Class& k : e->classes) {
    int key[6], val[6];
    tune_key(k, dev, key);
    if (cache && tune_cache_find(key, val)) {
      const char* envs[6] = {"LE_TUNE_ADV", "LE_TUNE_MU", "LE_TUNE_COL_CH",
                             "LE_TUNE_COL_FLOW", "LE_TUNE_ROW", "LE_TUNE_ROW_FWD"};
      int* dst[6] = {&k.adv_variant, &k.mu_variant, &k.col_ch_variant,
                     &k.col_flow_variant, &k.row_variant, &k.row_fwd_variant};
      for (int i = 0; i < 6; ++i) {
        const int forced = env_variant(envs[i]);
        *dst[i] = forced >= 0 ? forced : val[i];
      }
      continue;
    }
    const Run* d = e->d_desc + k.first;
    const int n = (int)k.members.size();
    const StepArgs* sa = e->d_args + k.first;
    hipStream_t st = e->stream;
    // row transforms first (the strip variants below use them); timed on the
    // inverse transforms of stages 0 and 3, into the real scratch
    rc = rc ? rc : pick(e, a, b, kRowCand, "LE_TUNE_ROW", &k.row_variant, [&](int v) {
      k.ops.row_c2r(d, n, k.ny, B_PS_S, B_TMP, B_PS_S, B_TMP, 2, v, st);
      k.ops.row_c2r(d, n, k.ny, B_PHIN, B_TMP, B_PHIN, B_TMP, 1, v, st);
    });
    // forward row transforms: timed as the two-kernel advection stage runs
    // them, three real scratch fields into three spectral ones (a working set
    // beyond the last-level cache on large grids, as in a step)
    rc = rc ? rc : pick(e, a, b, kRowCand, "LE_TUNE_ROW_FWD", &k.row_fwd_variant, [&](int v) {
      const int bins[3] = {B_TMP, B_R1, B_R2}, bouts[3] = {B_PHIH, B_FH, B_PHIN};
      k.ops.row_r2c_n(d, n, k.ny, bins, bouts, 3, v, st);
    });
    rc = rc ? rc : pick(e, a, b, kAdvCand, "LE_TUNE_ADV", &k.adv_variant, [&](int v) {
      k.ops.advect(d, n, k.ny, sa, k.inertial, v, k.row_fwd_variant, st);
    });
    rc = rc ? rc : pick(e, a, b, kMuCand, "LE_TUNE_MU", &k.mu_variant, [&](int v) {
      k.ops.mu_source(d, n, k.ny, sa, v, k.row_fwd_variant, st);
    });
    rc = rc ? rc : pick(e, a, b, kColCand, "LE_TUNE_COL_CH", &k.col_ch_variant, [&](int v) {
      k.column(COL_CH, d, n, k.nx, sa, B_PHIH, B_FH, B_PHIN, B_PHIN, v, st);
    });
    rc = rc ? rc : pick(e, a, b, kColCand, "LE_TUNE_COL_FLOW", &k.col_flow_variant, [&](int v) {
      if (k.inertial)
        k.column(COL_FLOW, d, n, k.nx, sa, B_OMH, B_GH, B_PHIH, B_FH, v, st);
      else
        k.column(COL_STOKES, d, n, k.nx, sa, B_GH, B_GH, B_PHIN, B_PHIN, v, st);
    });
    if (!rc && cache) {
      // only choices the timing made are shared (not ones fixed by LE_TUNE_*)
      const char* envs[6] = {"LE_TUNE_ADV", "LE_TUNE_MU", "LE_TUNE_COL_CH",
                             "LE_TUNE_COL_FLOW", "LE_TUNE_ROW", "LE_TUNE_ROW_FWD"};
      bool forced = false;
      for (const char* v : envs) forced = forced || env_variant(v) >= 0;
      const int got[6] = {k.adv_variant, k.mu_variant, k.col_ch_variant, k.col_flow_variant,
                          k.row_variant, k.row_fwd_variant};
      if (!forced) tune_cache_add(key, got);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // namespace

int create_engine(int32_t n, const le_params* ps, const double* const* phi0s,
                  const double* const* omega0s, Engine** out) {
  if (!out || n < 1 || !ps || !phi0s) return LE_EINVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    LE_RC(validate(&ps[i]));
    if (!phi0s[i]) return LE_EINVAL;
    if (ps[i].stream != ps[0].stream) return LE_EINVAL;
  }
  Engine* e = new (std::nothrow) Engine();
  if (!e) return LE_ENOMEM;
  e->nruns = n;
  e->runs.resize(n);
  {
    const char* env = std::getenv("LE_GRAPHS");
    e->use_graphs = !(env && env[0] == '0');
  }
  for (int i = 0; i < n; ++i) {
    RunHost& r = e->runs[i];
    const le_params& p = ps[i];
    r.p = p;
    r.p.stream = nullptr;
    for (void*& b : r.buf) b = nullptr;
    r.g = make_geo(p);
    r.inertial = p.rho > 0.0;
    r.tsize = p.precision == LE_FP64 ? sizeof(double) : sizeof(float);
    r.n_real = (size_t)p.nx * p.ny;
    r.n_spec = spec_elems(p.nx, p.ny);   // tiled, with the pad column
    r.wraps = wrap_count(r.p, 0);
    int cls = -1;
    for (size_t k = 0; k < e->classes.size(); ++k) {
      const Class& c = e->classes[k];
      if (c.nx == p.nx && c.ny == p.ny && c.prec == p.precision && c.inertial == r.inertial)
        cls = (int)k;
    }
    if (cls < 0) {
      Class c;
      c.nx = p.nx;
      c.ny = p.ny;
      c.prec = p.precision;
      c.inertial = r.inertial;
      if (!get_ops(p.precision, p.nx, p.ny, &c.ops)) {
        delete e;
        return LE_EINVAL;
      }
      e->classes.push_back(c);
      cls = (int)e->classes.size() - 1;
    }
    r.cls = cls;
    e->classes[cls].members.push_back(i);
  }
  int pos = 0;
  for (Class& c : e->classes) {
    c.first = pos;
    for (size_t k = 0; k < c.members.size(); ++k) e->runs[c.members[k]].internal = pos + (int)k;
    pos += (int)c.members.size();
  }

  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) {
    delete e;
    return LE_EDEVICE;
  }
  int rc = LE_OK;
  if (ps[0].stream) {
    e->stream = static_cast<hipStream_t>(ps[0].stream);
  } else if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) == hipSuccess) {
    e->own_stream = true;
  } else {
    rc = LE_EDEVICE;
  }
  size_t max_real = 0;
  for (RunHost& r : e->runs) {
    const size_t rb = r.n_real * r.tsize, sb = r.n_spec * 2 * r.tsize;
    max_real = std::max(max_real, r.n_real);
    const int specs[] = {B_PS_S, B_PHIH, B_FH, B_GH, B_PHIN};
    const int reals[] = {B_PHI, B_OM_R, B_PS_R, B_TMP, B_R1, B_R2};
    for (int b : specs) rc = rc ? rc : alloc(&r.buf[b], sb);
    for (int b : reals) rc = rc ? rc : alloc(&r.buf[b], rb);
    if (r.inertial) {
      rc = rc ? rc : alloc(&r.buf[B_OM_S], sb);
      rc = rc ? rc : alloc(&r.buf[B_OMH], sb);
    }
    // twiddle tables are FP64 for both precisions (FP32 runs round each
    // twiddle once, from FP64)
    rc = rc ? rc : alloc(&r.twx, (size_t)r.p.nx * 2 * sizeof(double));
    rc = rc ? rc : alloc(&r.twy, (size_t)r.p.ny * 4 * sizeof(double));
    if (!rc) {
      auto a = twiddles<double>(r.p.nx);
      auto b = twiddles<double>(2 * r.p.ny);
      if (hipMemcpy(r.twx, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice) ||
          hipMemcpy(r.twy, b.data(), b.size() * sizeof(double), hipMemcpyHostToDevice))
        rc = LE_EDEVICE;
    }
    const Ops& o = e->classes[r.cls].ops;
    e->nsblk_max = std::max(e->nsblk_max, o.obs_blocks(r.p.nx));
    e->nbins_max = std::max(e->nbins_max, r.p.ny / 2);
  }
  // descriptors in the class-grouped order
  if (!rc) {
    std::vector<Run> h(n);
    for (const RunHost& r : e->runs) {
      Run& d = h[r.internal];
      d.g = r.g;
      for (int b = 0; b < NBUF; ++b) d.buf[b] = r.buf[b];
      d.twx = r.twx;
      d.twy = r.twy;
    }
    rc = alloc((void**)&e->d_desc, sizeof(Run) * n);
    if (!rc && hipMemcpy(e->d_desc, h.data(), sizeof(Run) * n, hipMemcpyHostToDevice))
      rc = LE_EDEVICE;
  }
  const size_t nout = OBS_NTOTAL + 2 * (size_t)e->nbins_max;
  rc = rc ? rc : alloc((void**)&e->d_args, sizeof(StepArgs) * kChunkCap * n);
  rc = rc ? rc : alloc((void**)&e->d_spart, (size_t)e->nsblk_max * OBS_NSPEC * sizeof(double));
  rc = rc ? rc : alloc((void**)&e->d_rpart, (size_t)kRealBlocks * 3 * sizeof(double));
  rc = rc ? rc : alloc((void**)&e->d_bins, (size_t)e->nsblk_max * e->nbins_max * sizeof(double));
  rc = rc ? rc : alloc((void**)&e->d_counts,
                       (size_t)e->nsblk_max * e->nbins_max * sizeof(double));
  rc = rc ? rc : alloc((void**)&e->d_gsum, 2 * (size_t)obs_shell_groups(e->nsblk_max) *
                                               e->nbins_max * sizeof(double));
  rc = rc ? rc : alloc((void**)&e->d_out, nout * sizeof(double));
  if (!rc && hipHostMalloc((void**)&e->h_args, sizeof(StepArgs) * kChunkCap * n) != hipSuccess)
    rc = LE_ENOMEM;
  if (!rc && hipHostMalloc((void**)&e->h_out, nout * sizeof(double)) != hipSuccess)
    rc = LE_ENOMEM;
  e->stage_bytes = max_real * sizeof(double);
  if (!rc && hipHostMalloc(&e->h_stage, e->stage_bytes) != hipSuccess) rc = LE_ENOMEM;
  // initial state: phi0, omega0 and psi0 from the flow constraint at s = 0
  for (int i = 0; i < n && !rc; ++i) {
    RunHost& r = e->runs[i];
    rc = upload_real(e, r, phi0s[i], B_PHI);
    if (!rc && r.inertial) {
      const double* w0 = omega0s ? omega0s[i] : nullptr;
      if (w0) {
        rc = upload_real(e, r, w0, B_OM_R);
      } else if (hipMemsetAsync(r.buf[B_OM_R], 0, r.n_real * r.tsize, e->stream) !=
                 hipSuccess) {
        rc = LE_EDEVICE;
      }
      if (!rc)
        e->classes[r.cls].ops.row_r2c(desc(e, r), 1, r.p.ny, B_OM_R, B_OM_S,
                                      e->classes[r.cls].row_fwd_variant, e->stream);
    }
    if (!rc) rc = solve_psi(e, r);
  }
  if (!rc) rc = autotune(e);
  if (!rc && e->classes.size() > 1 && !(std::getenv("LE_CLASS_STREAMS") &&
                                        std::getenv("LE_CLASS_STREAMS")[0] == '0')) {
    if (hipEventCreateWithFlags(&e->fork_ev, hipEventDisableTiming) != hipSuccess)
      rc = LE_EDEVICE;
    for (size_t c = 0; c < e->classes.size() && !rc; ++c) {
      hipStream_t cs = nullptr;
      hipEvent_t ev = nullptr;
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        rc = LE_EDEVICE;
        break;
      }
      e->cls_streams.push_back(cs);
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        rc = LE_EDEVICE;
        break;
      }
      e->join_ev.push_back(ev);
    }
  }
  if (!rc && hipStreamSynchronize(e->stream) != hipSuccess) rc = LE_EDEVICE;
  if (rc) {
    release(e);
    delete e;
    return rc;
  }
  *out = e;
  return LE_OK;
}

int step_engine(Engine* e, int64_t nsteps) {
  if (!e || nsteps < 0) return LE_EINVAL;
  const size_t row = (size_t)e->nruns;
  int64_t remaining = nsteps;
  while (remaining > 0) {
    const int64_t n0 = e->step;
    const int64_t cap = e->profiling ? kProfChunk : (e->use_graphs ? kGraphChunk : kChunkCap);
    int64_t count = remaining < cap ? remaining : cap;
    // fill the table; end the chunk after the first step on which any run wraps
    for (int64_t k = 0; k < count; ++k) {
      bool wrap = false;
      for (const RunHost& r : e->runs) {
        StepArgs& a = e->h_args[(size_t)k * row + r.internal];
        a.s = e->midpoint_s ? strain_offset_mid(r.p, n0 + k) : strain_offset(r.p, n0 + k);
        a.pad = 0.0;
        wrap = wrap || wrap_count(r.p, n0 + k + 1) != wrap_count(r.p, n0 + k);
      }
      if (wrap) {
        count = k + 1;
        break;
      }
    }
    LE_RC(enqueue_pieces(e, count, row, [&](int64_t n) { return enqueue_steps(e, n); }));
    e->step = n0 + count;
    for (RunHost& r : e->runs) {
      const int64_t k_new = wrap_count(r.p, e->step);
      if (k_new != r.wraps) {
        enqueue_remap(e, r, k_new - r.wraps);
        r.wraps = k_new;
      }
    }
    LE_TRY(hipGetLastError());
    LE_TRY(hipStreamSynchronize(e->stream));  // h_args is reused by the next chunk
    if (e->profiling) harvest_times(e, count);
    remaining -= count;
  }
  if (nsteps > 0) {
    for (const RunHost& r : e->runs) {
      LE_RC(reduce_observables(e, r, false));
      if (e->h_out[OBS_NONFINITE] != 0.0) return LE_ENONFINITE;
    }
  }
  return LE_OK;
}

int get_state_of(Engine* e, int run, double* phi, double* omega, double* psi, int64_t* step,
                 int64_t* wraps) {
  if (!e || run < 0 || run >= e->nruns) return LE_EINVAL;
  const RunHost& r = e->runs[run];
  const Ops& o = e->classes[r.cls].ops;
  if (phi) LE_RC(download_real(e, r, B_PHI, phi));
  if (omega) {
    if (r.inertial) {
      o.row_c2r(desc(e, r), 1, r.p.ny, B_OM_S, B_OM_R, B_OM_S, B_OM_R, 1,
                e->classes[r.cls].row_variant, e->stream);
      LE_TRY(hipGetLastError());
      LE_RC(download_real(e, r, B_OM_R, omega));
    } else {
      std::memset(omega, 0, r.n_real * sizeof(double));
    }
  }
  if (psi) {
    o.row_c2r(desc(e, r), 1, r.p.ny, B_PS_S, B_PS_R, B_PS_S, B_PS_R, 1,
              e->classes[r.cls].row_variant, e->stream);
    LE_TRY(hipGetLastError());
    LE_RC(download_real(e, r, B_PS_R, psi));
  }
  if (step) *step = e->step;
  if (wraps) *wraps = r.wraps;
  return LE_OK;
}

int profile_engine(Engine* e, int enable) {
  if (!e) return LE_EINVAL;
  if (enable && e->events.empty()) {
    e->events.assign((size_t)kProfChunk * (LE_NSTAGES + 1), nullptr);
    for (auto& ev : e->events) LE_TRY(hipEventCreate(&ev));
  }
  e->profiling = enable != 0;
  for (int s = 0; s < LE_NSTAGES; ++s) {
    e->stage_ms[s] = 0.0;
    e->stage_n[s] = 0;
  }
  return LE_OK;
}

int stage_times_of(Engine* e, double* ms, int64_t* launches, int32_t cap) {
  if (!e || cap < 0) return LE_EINVAL;
  const int n = cap < LE_NSTAGES ? cap : LE_NSTAGES;
  for (int s = 0; s < n; ++s) {
    if (ms) ms[s] = e->stage_ms[s];
    if (launches) launches[s] = e->stage_n[s];
  }
  return LE_OK;
}

// Coarse steps each followed by the learned correction: omega to real
// space, phi += r_phi - mean(r_phi), omega += r_omega, then psi from the
// corrected omega by the Poisson solve at the step's strain offset.
int corrected_steps(Engine* e, int64_t ncoarse) {
  RunHost& r = e->runs[0];
  const Ops& o = e->classes[r.cls].ops;
  const Run* d = desc(e, r);
  int64_t remaining = ncoarse;
  while (remaining > 0) {
    const int64_t n0 = e->step;
    // while timing stages every step of a chunk records into the event pool,
    // which holds kProfChunk steps
    const int64_t cap = e->profiling ? kProfChunk : (e->use_graphs ? kGraphChunk : kChunkCap);
    int64_t count = remaining < cap ? remaining : cap;
    for (int64_t k = 0; k < count; ++k) {
      e->h_args[k].s =
          e->midpoint_s ? strain_offset_mid(r.p, n0 + k) : strain_offset(r.p, n0 + k);
      e->h_args[k].pad = 0.0;
      if (wrap_count(r.p, n0 + k + 1) != wrap_count(r.p, n0 + k)) {
        count = k + 1;
        break;
      }
    }
    // corrected chunks share the graph cache under negative keys
    LE_RC(enqueue_pieces(e, count, 1, [&](int64_t n) {
      return enqueue_chunk(e, -n, n, [&](int64_t k, hipEvent_t* ev) {
        const StepArgs* sa = e->d_args + k;
        enqueue_step(e, sa, ev);
        o.row_c2r(d, 1, r.p.ny, B_OM_S, B_OM_R, B_OM_S, B_OM_R, 1,
                  e->classes[r.cls].row_variant, e->stream);
        int rc = r.tsize == sizeof(double)
                     ? net_residual<double>(e->net, static_cast<const double*>(r.buf[B_PHI]),
                                            static_cast<const double*>(r.buf[B_OM_R]),
                                            e->stream)
                     : net_residual<float>(e->net, static_cast<const float*>(r.buf[B_PHI]),
                                           static_cast<const float*>(r.buf[B_OM_R]), e->stream);
        if (rc) return (int)LE_EDEVICE;
        const CorrArgs ca{net_z_out(e->net), net_partials(e->net), net_tiles(e->net),
                          e->net->scales[2], e->net->scales[3], e->corr_proj};
        o.row_r2c_corr(d, r.p.ny, ca, e->classes[r.cls].row_fwd_variant, e->stream);
        e->classes[r.cls].column(COL_POISSON, d, 1, r.p.nx, sa, B_OM_S, B_OM_S, B_PS_S, B_PS_S,
                                 0, e->stream);
        return (int)LE_OK;
      });
    }));
    e->step = n0 + count;
    const int64_t k_new = wrap_count(r.p, e->step);
    if (k_new != r.wraps) {
      enqueue_remap(e, r, k_new - r.wraps);
      r.wraps = k_new;
    }
    LE_TRY(hipGetLastError());
    LE_TRY(hipStreamSynchronize(e->stream));
    if (e->profiling) harvest_times(e, count);
    remaining -= count;
  }
  return LE_OK;
}

// Two state snapshots of run 0 (phi, omega_h, psi_h), allocated on first use.
int alloc_snapshots(Engine* e, const RunHost& r) {
  const size_t bytes[3] = {r.n_real * r.tsize, r.n_spec * 2 * r.tsize, r.n_spec * 2 * r.tsize};
  for (auto& sn : e->snap)
    for (int i = 0; i < 3; ++i)
      if (!sn[i] && (i != 1 || r.inertial)) LE_RC(alloc(&sn[i], bytes[i]));
  return LE_OK;
}

// The state between steps: real phi and the row spectra of omega and psi.
int copy_state(Engine* e, const RunHost& r, bool to_snap, int k) {
  const int bufs[3] = {B_PHI, B_OM_S, B_PS_S};
  const size_t bytes[3] = {r.n_real * r.tsize, r.n_spec * 2 * r.tsize, r.n_spec * 2 * r.tsize};
  for (int i = 0; i < 3; ++i) {
    void* live = r.buf[bufs[i]];
    void* snap = e->snap[k][i];
    if (!live) continue;  // omega's spectrum of a Stokes run
    LE_TRY(hipMemcpyAsync(to_snap ? snap : live, to_snap ? live : snap, bytes[i],
                          hipMemcpyDeviceToDevice, e->stream));
  }
  return LE_OK;
}

// Mean phi and L_s of the current state.
int audit_measure(Engine* e, const RunHost& r, double* mean, double* Ls, bool* finite) {
  LE_RC(reduce_observables(e, r, true));
  const double* h = e->h_out;
  *mean = h[OBS_SUM_PHI] / (double)r.n_real;
  *Ls = h[OBS_SUM_S_NZ] > 0.0 ? h[OBS_SUM_S_OVER_Q] / h[OBS_SUM_S_NZ] : 0.0;
  *finite = h[OBS_NONFINITE] == 0.0;
  return LE_OK;
}

// One audit window of n steps: corrected from the saved state, then plain
// from the same state.  Passed (finite, L_s within the tolerance of the
// plain run's, mean phi equal to 1e-9, FP32 runs 1e-5): the corrected state
// is restored.
// Failed: the plain state stays and the context falls back to plain steps.
int audit_window(Engine* e, int64_t n) {
  RunHost& r = e->runs[0];
  const int64_t step0 = e->step, wraps0 = r.wraps;
  LE_RC(copy_state(e, r, true, 0));
  LE_RC(corrected_steps(e, n));
  double mc, lc, mp, lp;
  bool fc, fp;
  LE_RC(audit_measure(e, r, &mc, &lc, &fc));
  LE_RC(copy_state(e, r, true, 1));
  const int64_t step1 = e->step, wraps1 = r.wraps;
  LE_RC(copy_state(e, r, false, 0));
  e->step = step0;
  r.wraps = wraps0;
  LE_RC(step_engine(e, n));
  LE_RC(audit_measure(e, r, &mp, &lp, &fp));
  if (!fp) return LE_ENONFINITE;
  const double dev = lp > 0.0 ? std::fabs(lc - lp) / lp : (lc == lp ? 0.0 : INFINITY);
  e->audits += 1;
  e->audit_dev = fc ? dev : INFINITY;
  const double mean_tol = r.tsize == sizeof(double) ? 1e-9 : 1e-5;
  if (fc && dev <= e->audit_tol && std::fabs(mc - mp) <= mean_tol) {
    LE_RC(copy_state(e, r, false, 1));
    e->step = step1;
    r.wraps = wraps1;
  } else {
    e->corr_fallback = true;
  }
  LE_TRY(hipStreamSynchronize(e->stream));
  return LE_OK;
}

int step_corrected(Engine* e, int64_t ncoarse) {
  if (!e || ncoarse < 0 || !e->net || e->nruns != 1) return LE_EINVAL;
  RunHost& r = e->runs[0];
  int64_t remaining = ncoarse;
  while (remaining > 0 && !e->corr_fallback) {
    int64_t n = remaining;
    if (e->audit_every > 0) {
      if (e->since_audit >= e->audit_every) {
        n = std::min(remaining, e->audit_window);
        LE_RC(audit_window(e, n));
        e->since_audit = 0;
        remaining -= n;
        continue;
      }
      n = std::min(remaining, e->audit_every - e->since_audit);
    }
    LE_RC(corrected_steps(e, n));
    e->since_audit += n;
    remaining -= n;
  }
  if (remaining > 0) return step_engine(e, remaining);
  if (ncoarse > 0) {
    LE_RC(reduce_observables(e, r, false));
    if (e->h_out[OBS_NONFINITE] != 0.0) return LE_ENONFINITE;
  }
  return LE_OK;
}

// le_step with recovery: the state at the call's start is kept; if the call
// ends non-finite, its steps are replayed one by one from that state (the
// step is deterministic) and the context stops at the last step whose phi is
// finite.
int step_recover(Engine* e, int64_t nsteps) {
  if (nsteps <= 0) return step_engine(e, nsteps);
  RunHost& r = e->runs[0];
  const int64_t step0 = e->step, wraps0 = r.wraps;
  LE_RC(copy_state(e, r, true, 0));
  int rc = step_engine(e, nsteps);
  if (rc != LE_ENONFINITE) return rc;
  LE_RC(copy_state(e, r, false, 0));
  e->step = step0;
  r.wraps = wraps0;
  for (int64_t k = 0; k < nsteps; ++k) {
    const int64_t sk = e->step, wk = r.wraps;
    LE_RC(copy_state(e, r, true, 1));
    rc = step_engine(e, 1);
    if (rc == LE_ENONFINITE) {
      LE_RC(copy_state(e, r, false, 1));
      e->step = sk;
      r.wraps = wk;
      LE_TRY(hipStreamSynchronize(e->stream));
      return LE_ENONFINITE;
    }
    LE_RC(rc);
  }
  return LE_OK;
}

int corrector_audit(Engine* e, int64_t every, int64_t window, double tol) {
  if (!e || !e->net || every < 0 || (every > 0 && (window < 1 || !(tol >= 0.0))))
    return LE_EINVAL;
  RunHost& r = e->runs[0];
  if (every > 0) LE_RC(alloc_snapshots(e, r));
  e->audit_every = every;
  e->audit_window = window;
  e->audit_tol = tol;
  e->since_audit = 0;
  e->audits = 0;
  e->audit_dev = 0.0;
  e->corr_fallback = false;
  return LE_OK;
}

void destroy_engine(Engine* e) {
  if (!e) return;
  if (e->stream) (void)hipStreamSynchronize(e->stream);
  release(e);
  delete e;
}

}  // namespace

// ---------------------------------------------------------------- no-allocation step
//
// le_step_noalloc takes every device buffer beyond the caller's three fields
// from one file-scope device array, `scratch`.  In host code the array's
// name is only a handle: its device address is looked up once per device
// with hipGetSymbolAddress (each device holds its own copy) and only that
// address reaches kernels and copies.
constexpr size_t kNoAllocBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kNoAllocDevices = 64;
std::atomic<void*> g_scratch_dev[kNoAllocDevices];

// Set-up of one call: the run descriptor (a kernel argument) into d, and the
// twiddle tables exp(-2 pi i k / nx), k < nx, and exp(-2 pi i k / (2 ny)),
// k < 2 ny (sincospi of the exact fraction -2k/n).
__global__ void k_noalloc_setup(Run h, Run* __restrict__ d, double* __restrict__ twx,
                                double* __restrict__ twy, int nx, int ny) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *d = h;
  if (i < nx) sincospi(-2.0 * (double)i / (double)nx, &twx[2 * i + 1], &twx[2 * i]);
  if (i < 2 * ny) sincospi(-2.0 * (double)i / (double)(2 * ny), &twy[2 * i + 1], &twy[2 * i]);
}

// StepArgs of steps n0 .. n0 + count - 1: the sawtooth s_n formed exactly as
// the host clock forms it (same operations, no contraction).
__global__ void k_step_args(StepArgs* __restrict__ out, int count, long long n0, double gdot,
                            double dt, double c) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const double X = gdot * ((double)(n0 + k) * dt);
  const double w = floor((X + 0.5 * c) / c);
  out[k].s = X - c * w;
  out[k].pad = 0.0;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Device address of this device's scratch array (looked up on first use).
int noalloc_scratch(void** out) {
  int dev = 0;
  LE_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "le_step_noalloc: device %d beyond the %d supported", dev, kNoAllocDevices);
    return LE_EDEVICE;
  }
  void* p = g_scratch_dev[dev].load();
  if (!p) {
    LE_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev].store(p);
  }
  *out = p;
  return LE_OK;
}

int step_noalloc(const le_params* pp, double* phi, double* omega, double* psi, int64_t step0,
                 int64_t nsteps) {
  LE_RC(validate(pp));
  const le_params& p = *pp;
  const bool inertial = p.rho > 0.0;
  if (!phi || !psi || (inertial && !omega) || step0 < 0 || nsteps < 0) return LE_EINVAL;
  if (p.precision != LE_FP64) {
    std::snprintf(g_last_error, sizeof(g_last_error), "le_step_noalloc: LE_FP64 only");
    return LE_EINVAL;
  }
  if (nsteps == 0) return LE_OK;
  // layout of the scratch array
  const size_t n_real = (size_t)p.nx * p.ny;
  const size_t spec_b = spec_elems(p.nx, p.ny) * 2 * sizeof(double);
  size_t off = 0;
  const size_t o_run = off;   off = align256(off + sizeof(Run));
  const size_t o_args = off;  off = align256(off + (size_t)kChunkCap * sizeof(StepArgs));
  const size_t o_twx = off;   off = align256(off + (size_t)p.nx * 2 * sizeof(double));
  const size_t o_twy = off;   off = align256(off + (size_t)p.ny * 4 * sizeof(double));
  const size_t o_rpart = off; off = align256(off + (size_t)kRealBlocks * 3 * sizeof(double));
  const size_t o_out = off;   off = align256(off + (size_t)OBS_NTOTAL * sizeof(double));
  const int specs[] = {B_OM_S, B_PS_S, B_PHIH, B_FH, B_OMH, B_GH, B_PHIN};
  const int reals[] = {B_TMP, B_R1, B_R2};
  size_t o_buf[NBUF] = {0};
  for (int b : specs) {
    if (!inertial && (b == B_OM_S || b == B_OMH)) continue;
    o_buf[b] = off;
    off = align256(off + spec_b);
  }
  for (int b : reals) {
    o_buf[b] = off;
    off = align256(off + n_real * sizeof(double));
  }
  if (off > kNoAllocBytes) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "le_step_noalloc: a %dx%d grid needs %zu bytes of scratch, the maximum is %zu",
                  p.nx, p.ny, off, kNoAllocBytes);
    return LE_EINVAL;
  }
  void* base = nullptr;
  LE_RC(noalloc_scratch(&base));
  unsigned char* sc = static_cast<unsigned char*>(base);
  hipStream_t st = static_cast<hipStream_t>(p.stream);
  Class k;
  k.nx = p.nx;
  k.ny = p.ny;
  k.prec = LE_FP64;
  k.inertial = inertial;
  if (!get_ops(LE_FP64, p.nx, p.ny, &k.ops)) return LE_EINVAL;
  Run h;
  h.g = make_geo(p);
  for (int b = 0; b < NBUF; ++b) h.buf[b] = o_buf[b] ? sc + o_buf[b] : nullptr;
  h.buf[B_PHI] = phi;
  h.buf[B_OM_R] = inertial ? omega : nullptr;
  h.buf[B_PS_R] = psi;
  h.twx = sc + o_twx;
  h.twy = sc + o_twy;
  Run* d = reinterpret_cast<Run*>(sc + o_run);
  StepArgs* args = reinterpret_cast<StepArgs*>(sc + o_args);
  double* rpart = reinterpret_cast<double*>(sc + o_rpart);
  double* out = reinterpret_cast<double*>(sc + o_out);
  {
    const int nt = p.nx > 2 * p.ny ? p.nx : 2 * p.ny;
    hipLaunchKernelGGL(k_noalloc_setup, dim3((nt + 255) / 256), dim3(256), 0, st, h, d,
                       reinterpret_cast<double*>(sc + o_twx),
                       reinterpret_cast<double*>(sc + o_twy), p.nx, p.ny);
  }
  // the caller's omega and psi are the real fields of step step0: the first
  // step takes them as they are
  bool inverse = false;
  int64_t n0 = step0, remaining = nsteps;
  int64_t wraps = wrap_count(p, n0);
  while (remaining > 0) {
    int64_t count = remaining < kChunkCap ? remaining : kChunkCap;
    for (int64_t q = 0; q < count; ++q)
      if (wrap_count(p, n0 + q + 1) != wrap_count(p, n0 + q)) {
        count = q + 1;
        break;
      }
    hipLaunchKernelGGL(k_step_args, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, args,
                       (int)count, (long long)n0, p.gdot, p.dt, p.lx / p.ly);
    for (int64_t q = 0; q < count; ++q) {
      enqueue_runs_step(k, d, 1, args + q, st, inverse);
      inverse = true;
    }
    n0 += count;
    const int64_t k_new = wrap_count(p, n0);
    if (k_new != wraps) {
      const int dkr = (int)(((k_new - wraps) * (int64_t)h.g.r) % p.nx);
      k.ops.remap_real(d, B_PHI, B_TMP, dkr, st);
      k.ops.copy_real(d, B_TMP, B_PHI, st);
      k.ops.remap_spec(d, B_PS_S, dkr, st);
      if (inertial) k.ops.remap_spec(d, B_OM_S, dkr, st);
      wraps = k_new;
    }
    LE_TRY(hipGetLastError());
    remaining -= count;
  }
  // the state's real omega and psi into the caller's fields
  if (inertial)
    k.ops.row_c2r(d, 1, p.ny, B_OM_S, B_OM_R, B_PS_S, B_PS_R, 2, k.row_variant, st);
  else
    k.ops.row_c2r(d, 1, p.ny, B_PS_S, B_PS_R, B_PS_S, B_PS_R, 1, k.row_variant, st);
  k.ops.obs_real(d, B_PHI, rpart, kRealBlocks, st);
  launch_obs_final(nullptr, 0, rpart, kRealBlocks, nullptr, nullptr, 0, nullptr, out, st);
  LE_TRY(hipGetLastError());
  double bad = 0.0;
  LE_TRY(hipMemcpyAsync(&bad, out + OBS_NONFINITE, sizeof(double), hipMemcpyDeviceToHost, st));
  LE_TRY(hipStreamSynchronize(st));
  return bad == 0.0 ? LE_OK : LE_ENONFINITE;
}

}  // namespace

extern "C" {

const char* le_last_error(void) { return g_last_error; }

const char* le_strerror(int code) {
  switch (code) {
    case LE_OK: return "ok";
    case LE_EINVAL: return "invalid argument";
    case LE_ENOMEM: return "out of memory";
    case LE_EDEVICE: return "HIP device error";
    case LE_ENONFINITE: return "state became non-finite";
    case LE_ESTATE: return "invalid context state";
    default: return "unknown error";
  }
}

int le_create(const le_params* p, const double* phi0, const double* omega0, le_ctx** out) {
  if (!out || !phi0 || !p) return LE_EINVAL;
  const double* const phis[1] = {phi0};
  const double* const oms[1] = {omega0};
  LE_RC(create_engine(1, p, phis, oms, out));
  // a step call that goes non-finite stops at the last finite step unless
  // the caller turns this off (le_set_recovery(c, 0))
  const int rc = alloc_snapshots(*out, (*out)->runs[0]);
  if (rc) {
    destroy_engine(*out);
    *out = nullptr;
    return rc;
  }
  (*out)->recovery = true;
  return LE_OK;
}

int le_step_noalloc(const le_params* p, double* phi_dev, double* omega_dev, double* psi_dev,
                    int64_t step0, int64_t nsteps) {
  return step_noalloc(p, phi_dev, omega_dev, psi_dev, step0, nsteps);
}

int le_step(le_ctx* c, int64_t nsteps) {
  if (c && c->recovery) return step_recover(c, nsteps);
  return step_engine(c, nsteps);
}

int le_set_recovery(le_ctx* c, int enable) {
  if (!c || c->nruns != 1) return LE_EINVAL;
  if (enable) LE_RC(alloc_snapshots(c, c->runs[0]));
  c->recovery = enable != 0;
  return LE_OK;
}

int le_set_scheme(le_ctx* c, int32_t flags) {
  if (!c ||
      (flags & ~(LE_SCHEME_F_HALF | LE_SCHEME_MIDPOINT_S | LE_SCHEME_UPWIND3 | LE_SCHEME_BANDED)) !=
          0)
    return LE_EINVAL;
  // every run of the engine (one for a context, all of a batch)
  c->midpoint_s = (flags & LE_SCHEME_MIDPOINT_S) != 0;
  const bool up = (flags & LE_SCHEME_UPWIND3) != 0;
  const bool band = (flags & LE_SCHEME_BANDED) != 0;
  bool relaunch = false;
  for (Class& k : c->classes) {
    relaunch = relaunch || k.upwind3 != up || k.banded != band;
    k.upwind3 = up;
    k.banded = band;
  }
  // captured graphs hold the other advection or column kernels
  if (relaunch) drop_graphs(c, [](int64_t) { return false; });
  std::vector<Run> h((size_t)c->nruns);
  LE_TRY(hipMemcpy(h.data(), c->d_desc, sizeof(Run) * h.size(), hipMemcpyDeviceToHost));
  for (RunHost& r : c->runs) {
    r.g.f_half = (flags & LE_SCHEME_F_HALF) ? 1 : 0;
    r.g.upwind3 = up ? 1 : 0;
    r.g.banded = (flags & LE_SCHEME_BANDED) ? 1 : 0;
    h[r.internal].g = r.g;
  }
  LE_TRY(hipStreamSynchronize(c->stream));
  LE_TRY(hipMemcpy(c->d_desc, h.data(), sizeof(Run) * h.size(), hipMemcpyHostToDevice));
  return LE_OK;
}

int le_observables(le_ctx* c, le_obs* o, double* Sk, int32_t sk_cap) {
  if (!c || !o) return LE_EINVAL;
  return observables_of(c, c->runs[0], o, Sk, sk_cap);
}

void le_destroy(le_ctx* c) { destroy_engine(c); }

int le_get_state(le_ctx* c, double* phi, double* omega, double* psi, int64_t* step,
                 int64_t* wraps) {
  return get_state_of(c, 0, phi, omega, psi, step, wraps);
}

int le_set_state(le_ctx* c, const double* phi, const double* omega, const double* psi,
                 int64_t step, int64_t wraps) {
  if (!c || !phi || !psi || step < 0) return LE_EINVAL;
  RunHost& r = c->runs[0];
  if (r.inertial && !omega) return LE_EINVAL;
  if (wraps != wrap_count(r.p, step)) return LE_EINVAL;
  const Ops& o = c->classes[r.cls].ops;
  LE_RC(upload_real(c, r, phi, B_PHI));
  if (r.inertial) {
    LE_RC(upload_real(c, r, omega, B_OM_R));
    o.row_r2c(desc(c, r), 1, r.p.ny, B_OM_R, B_OM_S, c->classes[r.cls].row_fwd_variant,
              c->stream);
  }
  LE_RC(upload_real(c, r, psi, B_PS_R));
  o.row_r2c(desc(c, r), 1, r.p.ny, B_PS_R, B_PS_S, c->classes[r.cls].row_fwd_variant,
            c->stream);
  LE_TRY(hipGetLastError());
  LE_TRY(hipStreamSynchronize(c->stream));
  c->step = step;
  r.wraps = wraps;
  return LE_OK;
}

int time_stage_of(Engine* e, int32_t stage, int32_t reps, double* ms_per_launch) {
  if (!e || stage < 0 || stage >= LE_NSTAGES || reps < 1 || !ms_per_launch) return LE_EINVAL;
  if (e->profiling) return LE_ESTATE;
  for (const RunHost& r : e->runs) LE_RC(set_args_one(e, r, e->step));
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return LE_EDEVICE;
  }
  // each launch covers every class, as one stage of a step does
  auto launch = [&]() {
    hipStream_t st = e->stream;
    for (const Class& k : e->classes) {
      const Run* d = e->d_desc + k.first;
      const int n = (int)k.members.size();
      const StepArgs* sa = e->d_args + k.first;
      switch (stage) {
        case 0:  // inverse row transforms of the state spectra, into the real scratch
          if (k.inertial)
            k.ops.row_c2r(d, n, k.ny, B_OM_S, B_TMP, B_PS_S, B_TMP, 2, k.row_variant, st);
          else
            k.ops.row_c2r(d, n, k.ny, B_PS_S, B_TMP, B_PS_S, B_TMP, 1, k.row_variant, st);
          break;
        case 1:
          k.ops.advect(d, n, k.ny, sa, k.inertial, k.advect(), k.row_fwd_variant, st);
          break;
        case 2:
          k.column(COL_CH, d, n, k.nx, sa, B_PHIH, B_FH, B_PHIN, B_PHIN, k.col_ch_variant,
                       st);
          break;
        case 3:  // into the real scratch
          k.ops.row_c2r(d, n, k.ny, B_PHIN, B_TMP, B_PHIN, B_TMP, 1, k.row_variant, st);
          break;
        case 4:
          k.ops.mu_source(d, n, k.ny, sa, k.mu_variant, k.row_fwd_variant, st);
          break;
        default:  // outputs into the spectral scratch, the state untouched
          if (k.inertial)
            k.column(COL_FLOW, d, n, k.nx, sa, B_OMH, B_GH, B_PHIH, B_FH,
                         k.col_flow_variant, st);
          else
            k.column(COL_STOKES, d, n, k.nx, sa, B_GH, B_GH, B_PHIN, B_PHIN,
                         k.col_flow_variant, st);
          break;
      }
    }
  };
  int rc = LE_OK;
  launch();
  float ms = 0.0f;
  if (hipEventRecord(a, e->stream) != hipSuccess) rc = LE_EDEVICE;
  for (int i = 0; i < reps && !rc; ++i) launch();
  if (!rc && (hipEventRecord(b, e->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
              hipGetLastError() != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
    rc = LE_EDEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!rc) *ms_per_launch = (double)ms / reps;
  return rc;
}

// Checkpoint blob: a header, then phi (real), the omega row spectrum
// (inertial runs) and the psi row spectrum, as stored (storage precision,
// the library's layout).
struct CkptHeader {
  uint64_t magic;
  int32_t version, nx, ny, precision, inertial;
  int32_t tile;  // modes per tile of the row-spectral layout (kTW)
  int64_t step, wraps;
  uint64_t bytes;
};
constexpr uint64_t kCkptMagic = 0x31504b43484d454cull;  // "LEMHCKP1"

int64_t ckpt_bytes(const RunHost& r) {
  const size_t spec = r.n_spec * 2 * r.tsize;
  return (int64_t)(sizeof(CkptHeader) + r.n_real * r.tsize + (r.inertial ? spec : 0) + spec);
}

int le_checkpoint_size(le_ctx* c, int64_t* bytes) {
  if (!c || !bytes || c->nruns != 1) return LE_EINVAL;
  *bytes = ckpt_bytes(c->runs[0]);
  return LE_OK;
}

int le_checkpoint_save(le_ctx* c, void* buf, int64_t cap) {
  if (!c || !buf || c->nruns != 1) return LE_EINVAL;
  const RunHost& r = c->runs[0];
  const int64_t need = ckpt_bytes(r);
  if (cap < need) return LE_EINVAL;
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kCkptMagic;
  h.version = 1;
  h.tile = kTW;
  h.nx = r.p.nx;
  h.ny = r.p.ny;
  h.precision = r.p.precision;
  h.inertial = r.inertial ? 1 : 0;
  h.step = c->step;
  h.wraps = r.wraps;
  h.bytes = (uint64_t)need;
  unsigned char* o = static_cast<unsigned char*>(buf);
  std::memcpy(o, &h, sizeof(h));
  size_t off = sizeof(h);
  const int bufs[3] = {B_PHI, B_OM_S, B_PS_S};
  const size_t sizes[3] = {r.n_real * r.tsize, r.n_spec * 2 * r.tsize, r.n_spec * 2 * r.tsize};
  for (int i = 0; i < 3; ++i) {
    if (i == 1 && !r.inertial) continue;
    LE_TRY(hipMemcpyAsync(o + off, r.buf[bufs[i]], sizes[i], hipMemcpyDeviceToHost, c->stream));
    off += sizes[i];
  }
  LE_TRY(hipStreamSynchronize(c->stream));
  return LE_OK;
}

int le_checkpoint_load(le_ctx* c, const void* buf, int64_t bytes) {
  if (!c || !buf || c->nruns != 1 || bytes < (int64_t)sizeof(CkptHeader)) return LE_EINVAL;
  RunHost& r = c->runs[0];
  CkptHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kCkptMagic || h.version != 1 || h.tile != kTW || h.nx != r.p.nx ||
      h.ny != r.p.ny || h.precision != r.p.precision || h.inertial != (r.inertial ? 1 : 0) ||
      (int64_t)h.bytes != ckpt_bytes(r) || bytes < ckpt_bytes(r) || h.step < 0 ||
      h.wraps != wrap_count(r.p, h.step))
    return LE_EINVAL;
  const unsigned char* in = static_cast<const unsigned char*>(buf);
  size_t off = sizeof(h);
  const int bufs[3] = {B_PHI, B_OM_S, B_PS_S};
  const size_t sizes[3] = {r.n_real * r.tsize, r.n_spec * 2 * r.tsize, r.n_spec * 2 * r.tsize};
  for (int i = 0; i < 3; ++i) {
    if (i == 1 && !r.inertial) continue;
    LE_TRY(hipMemcpyAsync(r.buf[bufs[i]], in + off, sizes[i], hipMemcpyHostToDevice, c->stream));
    off += sizes[i];
  }
  LE_TRY(hipStreamSynchronize(c->stream));
  c->step = h.step;
  r.wraps = h.wraps;
  return LE_OK;
}

int le_time_stage(le_ctx* c, int32_t stage, int32_t reps, double* ms_per_launch) {
  return time_stage_of(c, stage, reps, ms_per_launch);
}

int le_profile(le_ctx* c, int enable) { return profile_engine(c, enable); }

int tuning_of(le_ctx* c, int32_t* out, int32_t cap) {
  if (!c || cap < 0 || (cap > 0 && !out)) return LE_EINVAL;
  int32_t w = 0;
  for (const Class& k : c->classes) {
    const int32_t rec[LE_TUNING_FIELDS] = {k.nx, k.ny, k.prec, k.inertial ? 1 : 0,
                                           k.adv_variant, k.mu_variant, k.col_ch_variant,
                                           k.col_flow_variant, k.row_variant,
                                           k.row_fwd_variant};
    for (int i = 0; i < LE_TUNING_FIELDS && w < cap; ++i) out[w++] = rec[i];
  }
  return (int)c->classes.size();
}

int le_stage_times(le_ctx* c, double* ms, int64_t* launches, int32_t cap) {
  return stage_times_of(c, ms, launches, cap);
}

int le_batch_create(int32_t n, const le_params* ps, const double* const* phi0s,
                    const double* const* omega0s, le_batch** out) {
  if (!out) return LE_EINVAL;
  *out = nullptr;
  le_batch* b = new (std::nothrow) le_batch();
  if (!b) return LE_ENOMEM;
  const int rc = create_engine(n, ps, phi0s, omega0s, &b->e);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return LE_OK;
}

int le_batch_step(le_batch* b, int64_t nsteps) {
  return b ? step_engine(b->e, nsteps) : LE_EINVAL;
}

int le_batch_observables(le_batch* b, int32_t run, le_obs* o, double* Sk, int32_t sk_cap) {
  if (!b || !o || run < 0 || run >= b->e->nruns) return LE_EINVAL;
  return observables_of(b->e, b->e->runs[run], o, Sk, sk_cap);
}

int le_batch_get_state(le_batch* b, int32_t run, double* phi, double* omega, double* psi,
                       int64_t* step, int64_t* wraps) {
  return b ? get_state_of(b->e, run, phi, omega, psi, step, wraps) : LE_EINVAL;
}

int le_batch_profile(le_batch* b, int enable) {
  return b ? profile_engine(b->e, enable) : LE_EINVAL;
}

int le_tuning(le_ctx* c, int32_t* out, int32_t cap) { return tuning_of(c, out, cap); }

int le_batch_set_scheme(le_batch* b, int32_t flags) {
  return b ? le_set_scheme(b->e, flags) : LE_EINVAL;
}

int le_batch_tuning(le_batch* b, int32_t* out, int32_t cap) {
  return b ? tuning_of(b->e, out, cap) : LE_EINVAL;
}

int le_batch_stage_times(le_batch* b, double* ms, int64_t* launches, int32_t cap) {
  return b ? stage_times_of(b->e, ms, launches, cap) : LE_EINVAL;
}

int le_corrector_load(le_ctx* c, const float* params, int32_t nparams, const float* scales) {
  if (!c || !params || !scales || nparams != kCnnParams || c->nruns != 1) return LE_EINVAL;
  RunHost& r = c->runs[0];
  if (!r.inertial) return LE_EINVAL;
  if (!c->net) {
    Net* n = new (std::nothrow) Net();
    if (!n) return LE_ENOMEM;
    if (net_create(n, r.p.ny, r.p.nx, false)) {
      delete n;
      return LE_EINVAL;
    }
    c->net = n;
  }
  for (int k = 0; k < 4; ++k) c->net->scales[k] = scales[k];
  if (net_set_params(c->net, params, c->stream)) return LE_EDEVICE;
  c->corr_fallback = false;
  c->since_audit = 0;
  c->audits = 0;
  c->audit_dev = 0.0;
  // captured corrected chunks hold the old scales as launch arguments
  drop_graphs(c, [](int64_t key) { return key >= 0; });
  LE_TRY(hipStreamSynchronize(c->stream));
  return LE_OK;
}

int le_step_corrected(le_ctx* c, int64_t ncoarse) { return step_corrected(c, ncoarse); }

int le_corrector_projection(le_ctx* c, int32_t mode) {
  if (!c || (mode != 0 && mode != 1)) return LE_EINVAL;
  if (mode == 1 && (c->runs[0].p.nx % 16 || c->runs[0].p.ny % 16)) return LE_EINVAL;
  // captured corrected chunks hold the projection as a launch argument
  if (c->corr_proj != mode) drop_graphs(c, [](int64_t key) { return key >= 0; });
  c->corr_proj = mode;
  return LE_OK;
}

int le_corrector_audit(le_ctx* c, int64_t every, int64_t window, double tol) {
  return corrector_audit(c, every, window, tol);
}

int le_corrector_status(le_ctx* c, int32_t* fallback, int64_t* audits, double* last_dev) {
  if (!c) return LE_EINVAL;
  if (fallback) *fallback = c->corr_fallback ? 1 : 0;
  if (audits) *audits = c->audits;
  if (last_dev) *last_dev = c->audit_dev;
  return LE_OK;
}

int le_restrict(le_ctx* c, int32_t factor, double* phi_out, double* omega_out) {
  if (!c || factor < 1) return LE_EINVAL;
  RunHost& r = c->runs[0];
  if (r.p.nx % factor || r.p.ny % factor) return LE_EINVAL;
  const Ops& o = c->classes[r.cls].ops;
  const size_t nc = r.n_real / ((size_t)factor * factor);
  if (!c->d_restrict) LE_RC(alloc((void**)&c->d_restrict, r.n_real * sizeof(double)));
  if (phi_out) {
    o.restrict_real(desc(c, r), B_PHI, factor, c->d_restrict, c->stream);
    LE_TRY(hipMemcpyAsync(phi_out, c->d_restrict, nc * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    LE_TRY(hipStreamSynchronize(c->stream));
  }
  if (omega_out) {
    if (r.inertial) {
      o.row_c2r(desc(c, r), 1, r.p.ny, B_OM_S, B_OM_R, B_OM_S, B_OM_R, 1,
                c->classes[r.cls].row_variant, c->stream);
      o.restrict_real(desc(c, r), B_OM_R, factor, c->d_restrict, c->stream);
      LE_TRY(hipMemcpyAsync(omega_out, c->d_restrict, nc * sizeof(double),
                            hipMemcpyDeviceToHost, c->stream));
      LE_TRY(hipStreamSynchronize(c->stream));
    } else {
      std::memset(omega_out, 0, nc * sizeof(double));
    }
  }
  return LE_OK;
}

int le_set_fields(le_ctx* c, const double* phi, const double* omega, int64_t step) {
  if (!c || !phi || step < 0) return LE_EINVAL;
  RunHost& r = c->runs[0];
  const Ops& o = c->classes[r.cls].ops;
  LE_RC(upload_real(c, r, phi, B_PHI));
  c->step = step;
  r.wraps = wrap_count(r.p, step);
  if (r.inertial) {
    if (omega) {
      LE_RC(upload_real(c, r, omega, B_OM_R));
    } else {
      LE_TRY(hipMemsetAsync(r.buf[B_OM_R], 0, r.n_real * r.tsize, c->stream));
    }
    o.row_r2c(desc(c, r), 1, r.p.ny, B_OM_R, B_OM_S, c->classes[r.cls].row_fwd_variant,
              c->stream);
  }
  LE_RC(solve_psi(c, r));
  LE_TRY(hipStreamSynchronize(c->stream));
  return LE_OK;
}

int le_cnn_nparams(void) { return kCnnParams; }

int le_cnn_create(int32_t H, int32_t W, le_cnn** out) {
  if (!out) return LE_EINVAL;
  *out = nullptr;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return LE_EDEVICE;
  le_cnn* c = new (std::nothrow) le_cnn();
  if (!c) return LE_ENOMEM;
  const int rc = net_create(&c->net, H, W, true);
  if (rc) {
    delete c;
    return rc == -1 ? LE_EINVAL : (rc == -2 ? LE_ENOMEM : LE_EDEVICE);
  }
  *out = c;
  return LE_OK;
}

void le_cnn_destroy(le_cnn* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  net_destroy(&c->net);
  delete c;
}

int le_cnn_set_params(le_cnn* c, const float* params, int32_t n, const float* scales) {
  if (!c || !params || !scales || n != kCnnParams) return LE_EINVAL;
  for (int k = 0; k < 4; ++k) c->net.scales[k] = scales[k];
  if (net_set_params(&c->net, params, nullptr)) return LE_EDEVICE;
  LE_TRY(hipMemset(c->net.m, 0, kCnnParams * sizeof(float)));
  LE_TRY(hipMemset(c->net.v, 0, kCnnParams * sizeof(float)));
  LE_TRY(hipDeviceSynchronize());
  return LE_OK;
}

int le_cnn_get_params(le_cnn* c, float* params, int32_t n) {
  if (!c || !params || n != kCnnParams) return LE_EINVAL;
  LE_TRY(hipDeviceSynchronize());
  LE_TRY(hipMemcpy(params, c->net.params, kCnnParams * sizeof(float), hipMemcpyDeviceToHost));
  return LE_OK;
}

int le_cnn_forward(le_cnn* c, const float* x, float* r, void* stream) {
  if (!c || !x || !r) return LE_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net_forward_planes(&c->net, x, r, st)) return LE_EDEVICE;
  LE_TRY(hipStreamSynchronize(st));
  return LE_OK;
}

int le_cnn_grad(le_cnn* c, const float* xs, const float* ts, int32_t batch, double* loss,
                float* grad_host, void* stream) {
  if (!c || !xs || !ts || batch < 1) return LE_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  LE_TRY(hipMemsetAsync(c->net.grad, 0, kCnnParams * sizeof(float), st));
  if (net_grad(&c->net, xs, ts, batch, loss, st)) return LE_EDEVICE;
  if (grad_host) {
    LE_TRY(hipMemcpyAsync(grad_host, c->net.grad, kCnnParams * sizeof(float),
                          hipMemcpyDeviceToHost, st));
    LE_TRY(hipStreamSynchronize(st));
  }
  return LE_OK;
}

int le_cnn_adam(le_cnn* c, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!c || !(lr >= 0.f)) return LE_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net_adam(&c->net, lr, beta1, beta2, eps, st)) return LE_EDEVICE;
  LE_TRY(hipStreamSynchronize(st));
  return LE_OK;
}

int le_cnn_layer_fwd(le_cnn* c, int32_t layer, const uint16_t* a_in, float* z_out,
                     uint16_t* a_out, void* stream) {
  if (!c || !a_in || !z_out || layer < 0 || layer > 3 || (layer < 3 && !a_out))
    return LE_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net_layer_fwd(&c->net, layer, a_in, z_out, a_out, st)) return LE_EDEVICE;
  LE_TRY(hipStreamSynchronize(st));
  return LE_OK;
}

int le_cnn_layer_bwd(le_cnn* c, int32_t layer, const float* dz, const uint16_t* a_in,
                     const float* zprev, float* dzprev, float* dw, void* stream) {
  if (!c || !dz || !a_in || layer < 0 || layer > 3) return LE_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net_layer_bwd(&c->net, layer, dz, a_in, zprev, dzprev, dw, st)) return LE_EDEVICE;
  LE_TRY(hipStreamSynchronize(st));
  return LE_OK;
}

int le_cnn_mfma_probe(const uint16_t* a, const uint16_t* b, float* c) {
  if (!a || !b || !c) return LE_EINVAL;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return LE_EDEVICE;
  return mfma_probe(a, b, c, nullptr) ? LE_EDEVICE : LE_OK;
}

void le_batch_destroy(le_batch* b) {
  if (!b) return;
  destroy_engine(b->e);
  delete b;
}

}  // extern "C"

namespace le {
bool get_ops(int precision, int nx, int ny, Ops* ops) {
  return precision == LE_FP64 ? get_ops_f64(nx, ny, ops) : get_ops_f32(nx, ny, ops);
}
}  // namespace le
