// api.hip -- the C ABI of include/le.h: context, device buffers, shear clock,
// step schedule and observables.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/le.h"
#include "common.hpp"
#include "ops.hpp"

using namespace le;

namespace {

constexpr int kArgsCap = 4096;   // steps per host chunk (one StepArgs each)
constexpr int kRealBlocks = 256;  // blocks of the real-space reduction
constexpr int kProfChunk = 256;   // steps per chunk while stage timing is on

// Text of the last failing HIP call on this thread (le_last_error).
thread_local char g_last_error[256] = "";

int fail_hip(hipError_t e, const char* what, int line) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (line %d): %s", what, line,
                hipGetErrorString(e));
  return LE_EDEVICE;
}

#define LE_TRY(expr)                                             \
  do {                                                           \
    const hipError_t le_e_ = (expr);                             \
    if (le_e_ != hipSuccess) return fail_hip(le_e_, #expr, __LINE__); \
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
#pragma clang fp contract(on)

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

struct le_ctx {
  le_params p;
  Geo geo;
  Ops ops;
  size_t tsize;         // bytes per real value (4 or 8)
  size_t n_real;        // nx * ny
  size_t n_spec;        // ny * (nx/2 + 1) complex values
  bool inertial;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t step = 0, wraps = 0;
  // device buffers (storage type T)
  void* phi = nullptr;   // real, state
  void* om_s = nullptr;  // row spectrum of omega, state (inertial)
  void* ps_s = nullptr;  // row spectrum of psi, state
  void* om_r = nullptr;  // real scratch
  void* ps_r = nullptr;  // real scratch
  void* phih = nullptr;  // row spectra, scratch
  void* fh = nullptr;
  void* omh = nullptr;
  void* gh = nullptr;
  void* phin = nullptr;
  void* twx = nullptr;   // exp(-2 pi i k / nx), k < nx
  void* twy = nullptr;   // exp(-2 pi i k / (2 ny)), k < 2 ny
  StepArgs* d_args = nullptr;
  StepArgs* h_args = nullptr;  // pinned
  double* d_spart = nullptr;
  double* d_rpart = nullptr;
  double* d_bins = nullptr;
  double* d_counts = nullptr;
  double* d_out = nullptr;
  double* h_out = nullptr;     // pinned
  int nsblk = 0, nbins = 0;
  void* h_stage = nullptr;     // pinned host staging for up/downloads
  // captured step sequences, keyed by their length in steps
  bool use_graphs = true;
  std::map<int64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  // stage timing (le_profile)
  bool profiling = false;
  std::vector<hipEvent_t> events;   // kProfChunk * (LE_NSTAGES + 1)
  double stage_ms[LE_NSTAGES] = {0};
  int64_t stage_n[LE_NSTAGES] = {0};
};

namespace {

void release(le_ctx* c) {
  void* dev[] = {c->phi, c->om_s, c->ps_s, c->om_r, c->ps_r, c->phih, c->fh, c->omh,
                 c->gh, c->phin, c->twx, c->twy, c->d_args, c->d_spart, c->d_rpart,
                 c->d_bins, c->d_counts, c->d_out};
  for (void* d : dev)
    if (d) (void)hipFree(d);
  if (c->h_args) (void)hipHostFree(c->h_args);
  if (c->h_out) (void)hipHostFree(c->h_out);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  for (auto& kv : c->graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  c->graphs.clear();
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

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

// Twiddle table exp(-2 pi i k / n), k < n, rounded from long double.
template <typename T>
std::vector<T> twiddles(int n) {
  std::vector<T> tw(2 * (size_t)n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < n; ++k) {
    const long double a = -2.0L * pi * (long double)k / (long double)n;
    tw[2 * k] = (T)std::cos(a);
    tw[2 * k + 1] = (T)std::sin(a);
  }
  return tw;
}

int upload_twiddles(le_ctx* c) {
  const int nx = c->p.nx, ny = c->p.ny;
  if (c->p.precision == LE_FP64) {
    auto a = twiddles<double>(nx);
    auto b = twiddles<double>(2 * ny);
    LE_TRY(hipMemcpy(c->twx, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice));
    LE_TRY(hipMemcpy(c->twy, b.data(), b.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    auto a = twiddles<float>(nx);
    auto b = twiddles<float>(2 * ny);
    LE_TRY(hipMemcpy(c->twx, a.data(), a.size() * sizeof(float), hipMemcpyHostToDevice));
    LE_TRY(hipMemcpy(c->twy, b.data(), b.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  return LE_OK;
}

// host doubles -> device storage type, through the pinned staging buffer
int upload_real(le_ctx* c, const double* src, void* dst) {
  if (c->tsize == sizeof(double)) {
    std::memcpy(c->h_stage, src, c->n_real * sizeof(double));
  } else {
    float* s = static_cast<float*>(c->h_stage);
    for (size_t i = 0; i < c->n_real; ++i) s[i] = (float)src[i];
  }
  LE_TRY(hipMemcpyAsync(dst, c->h_stage, c->n_real * c->tsize, hipMemcpyHostToDevice, c->stream));
  LE_TRY(hipStreamSynchronize(c->stream));
  return LE_OK;
}

int download_real(le_ctx* c, const void* src, double* dst) {
  LE_TRY(hipMemcpyAsync(c->h_stage, src, c->n_real * c->tsize, hipMemcpyDeviceToHost, c->stream));
  LE_TRY(hipStreamSynchronize(c->stream));
  if (c->tsize == sizeof(double)) {
    std::memcpy(dst, c->h_stage, c->n_real * sizeof(double));
  } else {
    const float* s = static_cast<const float*>(c->h_stage);
    for (size_t i = 0; i < c->n_real; ++i) dst[i] = (double)s[i];
  }
  return LE_OK;
}

// One StepArgs (s at step n) into d_args[0], for set-up and observables.
int set_args0(le_ctx* c, int64_t n) {
  c->h_args[0].s = strain_offset(c->p, n);
  c->h_args[0].pad = 0.0;
  LE_TRY(hipMemcpyAsync(c->d_args, c->h_args, sizeof(StepArgs), hipMemcpyHostToDevice, c->stream));
  return LE_OK;
}

// psi from the flow constraint at the current step (Poisson from omega, or
// the Stokes solve from phi); omega's row spectrum must be current.
int solve_psi(le_ctx* c) {
  int rc = set_args0(c, c->step);
  if (rc) return rc;
  if (c->inertial) {
    c->ops.column(COL_POISSON, c->om_s, nullptr, c->ps_s, nullptr, c->d_args, c->geo, c->twy,
                  c->stream);
  } else {
    c->ops.mu_source(c->phi, c->gh, c->d_args, c->geo, 1.0 / c->p.eta, c->twx, c->stream);
    c->ops.column(COL_STOKES, c->gh, nullptr, c->ps_s, nullptr, c->d_args, c->geo, c->twy,
                  c->stream);
  }
  LE_TRY(hipGetLastError());
  return LE_OK;
}

// The stages of one step n -> n+1 at s = sa->s.  ev: LE_NSTAGES + 1 events
// recorded around the stages when timing, else nullptr.
void enqueue_step(le_ctx* c, const StepArgs* sa, hipEvent_t* ev) {
  const Ops& o = c->ops;
  auto mark = [&](int k) {
    if (ev) (void)hipEventRecord(ev[k], c->stream);
  };
  mark(0);
  if (c->inertial) {
    o.row_c2r(c->om_s, c->om_r, c->ps_s, c->ps_r, c->geo, c->twx, c->stream);
  } else {
    o.row_c2r(c->ps_s, c->ps_r, nullptr, nullptr, c->geo, c->twx, c->stream);
  }
  mark(1);
  o.advect(c->phi, c->om_r, c->ps_r, c->phih, c->fh, c->omh, sa, c->geo, c->twx, c->inertial,
           c->stream);
  mark(2);
  o.column(COL_CH, c->phih, c->fh, c->phin, nullptr, sa, c->geo, c->twy, c->stream);
  mark(3);
  o.row_c2r(c->phin, c->phi, nullptr, nullptr, c->geo, c->twx, c->stream);
  mark(4);
  if (c->inertial) {
    o.mu_source(c->phi, c->gh, sa, c->geo, 1.0 / c->p.rho, c->twx, c->stream);
    mark(5);
    o.column(COL_FLOW, c->omh, c->gh, c->om_s, c->ps_s, sa, c->geo, c->twy, c->stream);
  } else {
    o.mu_source(c->phi, c->gh, sa, c->geo, 1.0 / c->p.eta, c->twx, c->stream);
    mark(5);
    o.column(COL_STOKES, c->gh, nullptr, c->ps_s, nullptr, sa, c->geo, c->twy, c->stream);
  }
  mark(6);
}

// Accumulate the stage times of `count` profiled steps (stream drained).
void harvest_times(le_ctx* c, int64_t count) {
  for (int64_t k = 0; k < count; ++k) {
    hipEvent_t* ev = &c->events[(size_t)k * (LE_NSTAGES + 1)];
    for (int s = 0; s < LE_NSTAGES; ++s) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[s], ev[s + 1]) == hipSuccess) {
        c->stage_ms[s] += ms;
        c->stage_n[s] += 1;
      }
    }
  }
}

// Enqueue `count` steps reading their StepArgs from d_args[0 .. count).  Runs
// of at least kGraphMin steps are captured once into a HIP graph per length
// and replayed; the per-step strain offsets stay in device memory, so one
// graph serves every chunk of that length.
constexpr int64_t kGraphMin = 8;
constexpr size_t kGraphCacheMax = 4;
int enqueue_steps(le_ctx* c, int64_t count) {
  // Stage timing brackets direct launches with events (event-record nodes
  // are not taken under capture here), so timed chunks are never captured.
  const int64_t key = count;
  const bool graph_ok = c->use_graphs && count >= kGraphMin && !c->profiling;
  auto it = graph_ok ? c->graphs.find(key) : c->graphs.end();
  if (graph_ok && it == c->graphs.end()) {
    if (c->graphs.size() >= kGraphCacheMax) {
      auto old = c->graphs.begin();
      (void)hipGraphExecDestroy(old->second.second);
      (void)hipGraphDestroy(old->second.first);
      c->graphs.erase(old);
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      for (int64_t k = 0; k < count; ++k) enqueue_step(c, c->d_args + k, nullptr);
      e = hipStreamEndCapture(c->stream, &g);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      // leave capture mode, drop the partial graph and launch directly
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(c->stream, &cs) == hipSuccess &&
          cs != hipStreamCaptureStatusNone) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(c->stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
      }
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      fail_hip(e, "graph capture (falling back to direct launches)", __LINE__);
      c->use_graphs = false;
    } else {
      it = c->graphs.emplace(key, std::make_pair(g, ge)).first;
    }
  }
  if (it != c->graphs.end()) {
    LE_TRY(hipGraphLaunch(it->second.second, c->stream));
    return LE_OK;
  }
  for (int64_t k = 0; k < count; ++k)
    enqueue_step(c, c->d_args + k,
                 c->profiling ? &c->events[(size_t)k * (LE_NSTAGES + 1)] : nullptr);
  return LE_OK;
}

// Remap the state after the strain offset jumped by -dk * c.
void enqueue_remap(le_ctx* c, int64_t dk) {
  const int dkr = (int)((dk * (int64_t)c->geo.r) % c->p.nx);
  c->ops.remap_real(c->phi, c->om_r, c->geo, dkr, c->stream);
  std::swap(c->phi, c->om_r);
  c->ops.remap_spec(c->ps_s, c->geo, dkr, c->twx, c->stream);
  if (c->inertial) c->ops.remap_spec(c->om_s, c->geo, dkr, c->twx, c->stream);
}

// Sums of the observables into h_out (OBS_NTOTAL values + 2 nbins).
int reduce_observables(le_ctx* c) {
  int rc = set_args0(c, c->step);
  if (rc) return rc;
  c->ops.row_r2c(c->phi, c->phih, c->geo, c->twx, c->stream);
  c->ops.obs_spectral(c->phih, c->inertial ? c->ps_s : nullptr, c->d_spart, c->d_bins,
                      c->d_counts, c->d_args, c->geo, c->twy, c->stream);
  c->ops.obs_real(c->phi, c->n_real, c->d_rpart, kRealBlocks, c->stream);
  launch_obs_final(c->d_spart, c->nsblk, c->d_rpart, kRealBlocks, c->d_bins, c->d_counts,
                   c->nbins, c->d_out, c->stream);
  LE_TRY(hipGetLastError());
  const size_t nout = OBS_NTOTAL + 2 * (size_t)c->nbins;
  LE_TRY(hipMemcpyAsync(c->h_out, c->d_out, nout * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  LE_TRY(hipStreamSynchronize(c->stream));
  return LE_OK;
}

int alloc(void** p, size_t bytes) {
  return hipMalloc(p, bytes) == hipSuccess ? LE_OK : LE_ENOMEM;
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
  if (!out || !phi0) return LE_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  le_ctx* c = new (std::nothrow) le_ctx();
  if (!c) return LE_ENOMEM;
  c->p = *p;
  if (!get_ops(p->precision, p->nx, p->ny, &c->ops)) {
    delete c;
    return LE_EINVAL;
  }
  Geo& g = c->geo;
  g.nx = p->nx;
  g.ny = p->ny;
  g.r = p->nx >= p->ny ? p->nx / p->ny : 0;
  g.pad0 = 0;
  g.lx = p->lx;
  g.ly = p->ly;
  g.dx = p->lx / p->nx;
  g.dy = p->ly / p->ny;
  g.c = p->lx / p->ly;
  g.A = p->A;
  g.B = p->B;
  g.kappa = p->kappa;
  g.M = p->M;
  g.eta = p->eta;
  g.rho = p->rho;
  g.dt = p->dt;
  g.kx0 = 6.283185307179586476925286766559 / p->lx;
  g.ky0 = 6.283185307179586476925286766559 / p->ly;
  c->inertial = p->rho > 0.0;
  {
    const char* e = std::getenv("LE_GRAPHS");
    c->use_graphs = !(e && e[0] == '0');
  }
  c->tsize = p->precision == LE_FP64 ? sizeof(double) : sizeof(float);
  c->n_real = (size_t)p->nx * p->ny;
  c->n_spec = (size_t)p->ny * (p->nx / 2 + 1);
  c->nsblk = c->ops.obs_blocks(g);
  c->nbins = p->ny / 2;
  c->step = 0;
  c->wraps = wrap_count(c->p, 0);

  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) {
    delete c;
    return LE_EDEVICE;
  }
  if (p->stream) {
    c->stream = static_cast<hipStream_t>(p->stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return LE_EDEVICE;
    }
    c->own_stream = true;
  }
  const size_t rb = c->n_real * c->tsize, sb = c->n_spec * 2 * c->tsize;
  rc = LE_OK;
  rc = rc ? rc : alloc(&c->phi, rb);
  rc = rc ? rc : alloc(&c->ps_s, sb);
  rc = rc ? rc : alloc(&c->om_r, rb);
  rc = rc ? rc : alloc(&c->ps_r, rb);
  rc = rc ? rc : alloc(&c->phih, sb);
  rc = rc ? rc : alloc(&c->fh, sb);
  rc = rc ? rc : alloc(&c->gh, sb);
  rc = rc ? rc : alloc(&c->phin, sb);
  if (c->inertial) {
    rc = rc ? rc : alloc(&c->om_s, sb);
    rc = rc ? rc : alloc(&c->omh, sb);
  }
  rc = rc ? rc : alloc(&c->twx, (size_t)p->nx * 2 * c->tsize);
  rc = rc ? rc : alloc(&c->twy, (size_t)p->ny * 4 * c->tsize);
  rc = rc ? rc : alloc((void**)&c->d_args, kArgsCap * sizeof(StepArgs));
  rc = rc ? rc : alloc((void**)&c->d_spart, (size_t)c->nsblk * OBS_NSPEC * sizeof(double));
  rc = rc ? rc : alloc((void**)&c->d_rpart, (size_t)kRealBlocks * 3 * sizeof(double));
  rc = rc ? rc : alloc((void**)&c->d_bins, (size_t)c->nsblk * c->nbins * sizeof(double));
  rc = rc ? rc : alloc((void**)&c->d_counts, (size_t)c->nsblk * c->nbins * sizeof(double));
  rc = rc ? rc : alloc((void**)&c->d_out, (OBS_NTOTAL + 2 * (size_t)c->nbins) * sizeof(double));
  if (!rc && hipHostMalloc((void**)&c->h_args, kArgsCap * sizeof(StepArgs)) != hipSuccess)
    rc = LE_ENOMEM;
  if (!rc && hipHostMalloc((void**)&c->h_out, (OBS_NTOTAL + 2 * (size_t)c->nbins) *
                                                  sizeof(double)) != hipSuccess)
    rc = LE_ENOMEM;
  if (!rc && hipHostMalloc(&c->h_stage, c->n_real * sizeof(double)) != hipSuccess)
    rc = LE_ENOMEM;
  if (!rc) rc = upload_twiddles(c);
  if (!rc) rc = upload_real(c, phi0, c->phi);
  if (!rc && c->inertial) {
    if (omega0) {
      rc = upload_real(c, omega0, c->om_r);
    } else if (hipMemsetAsync(c->om_r, 0, rb, c->stream) != hipSuccess) {
      rc = LE_EDEVICE;
    }
    if (!rc) {
      c->ops.row_r2c(c->om_r, c->om_s, c->geo, c->twx, c->stream);
      if (hipGetLastError() != hipSuccess) rc = LE_EDEVICE;
    }
  }
  if (!rc) rc = solve_psi(c);
  if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = LE_EDEVICE;
  if (rc) {
    release(c);
    delete c;
    return rc;
  }
  *out = c;
  return LE_OK;
}

int le_step(le_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return LE_EINVAL;
  int64_t remaining = nsteps;
  while (remaining > 0) {
    const int64_t n0 = c->step;
    const int64_t cap = c->profiling ? kProfChunk : kArgsCap;
    int64_t count = remaining < cap ? remaining : cap;
    int64_t k_end = wrap_count(c->p, n0);
    for (int64_t k = 0; k < count; ++k) {
      c->h_args[k].s = strain_offset(c->p, n0 + k);
      c->h_args[k].pad = 0.0;
      const int64_t kn = wrap_count(c->p, n0 + k + 1);
      if (kn != k_end) {   // this step ends on a strain jump: remap after it
        count = k + 1;
        k_end = kn;
        break;
      }
    }
    LE_TRY(hipMemcpyAsync(c->d_args, c->h_args, (size_t)count * sizeof(StepArgs),
                          hipMemcpyHostToDevice, c->stream));
    int rc = enqueue_steps(c, count);
    if (rc) return rc;
    c->step = n0 + count;
    if (k_end != c->wraps) {
      enqueue_remap(c, k_end - c->wraps);
      c->wraps = k_end;
    }
    LE_TRY(hipGetLastError());
    LE_TRY(hipStreamSynchronize(c->stream));  // h_args is reused by the next chunk
    if (c->profiling) harvest_times(c, count);
    remaining -= count;
  }
  if (nsteps > 0) {
    c->ops.obs_real(c->phi, c->n_real, c->d_rpart, kRealBlocks, c->stream);
    launch_obs_final(c->d_spart, 0, c->d_rpart, kRealBlocks, c->d_bins, c->d_counts, 0,
                     c->d_out, c->stream);
    LE_TRY(hipGetLastError());
    LE_TRY(hipMemcpyAsync(c->h_out, c->d_out, OBS_NTOTAL * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
    LE_TRY(hipStreamSynchronize(c->stream));
    if (c->h_out[OBS_NONFINITE] != 0.0) return LE_ENONFINITE;
  }
  return LE_OK;
}

int le_observables(le_ctx* c, le_obs* o, double* Sk, int32_t sk_cap) {
  if (!c || !o) return LE_EINVAL;
  int rc = reduce_observables(c);
  if (rc) return rc;
  const double* h = c->h_out;
  const double N = (double)c->n_real;
  le_obs r;
  std::memset(&r, 0, sizeof(r));
  r.step = c->step;
  r.wraps = c->wraps;
  r.t = (double)c->step * c->p.dt;
  r.strain = strain_total(c->p, c->step);
  r.s = strain_offset(c->p, c->step);
  r.mean_phi = h[OBS_SUM_PHI] / N;
  r.phi2 = h[OBS_SUM_PHI2] / N;
  r.Ls = h[OBS_SUM_S_NZ] > 0.0 ? h[OBS_SUM_S_OVER_Q] / h[OBS_SUM_S_NZ] : 0.0;
  const double l = std::sqrt(c->p.kappa / c->p.A);
  const double tot = h[OBS_SUM_S];
  r.Dxx = tot > 0.0 ? l * h[OBS_XX] / tot : 0.0;
  r.Dxy = tot > 0.0 ? l * h[OBS_XY] / tot : 0.0;
  r.Dyy = tot > 0.0 ? l * h[OBS_YY] / tot : 0.0;
  const double mid = 0.5 * (r.Dxx + r.Dyy);
  const double rad = std::sqrt(0.25 * (r.Dxx - r.Dyy) * (r.Dxx - r.Dyy) + r.Dxy * r.Dxy);
  const double hi = mid + rad, lo = mid - rad;
  r.L_perp = hi > 0.0 ? 1.0 / hi : INFINITY;
  r.L_par = lo > 0.0 ? 1.0 / lo : INFINITY;
  r.sigma_xy = -c->p.kappa * h[OBS_XY] / N;
  r.sigma_xy_re = c->inertial ? c->p.rho * h[OBS_RE] / (N * N) : 0.0;
  r.nbins = c->nbins;
  r.dk = 6.283185307179586476925286766559 / c->p.ly;
  r.finite = h[OBS_NONFINITE] == 0.0 ? 1 : 0;
  if (Sk) {
    const int nb = sk_cap < c->nbins ? sk_cap : c->nbins;
    for (int b = 0; b < nb; ++b) {
      const double w = h[OBS_NTOTAL + c->nbins + b];
      Sk[b] = w > 0.0 ? h[OBS_NTOTAL + b] / w : 0.0;
    }
  }
  *o = r;
  return LE_OK;
}

void le_destroy(le_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  release(c);
  delete c;
}

int le_get_state(le_ctx* c, double* phi, double* omega, double* psi, int64_t* step,
                 int64_t* wraps) {
  if (!c) return LE_EINVAL;
  int rc;
  if (phi && (rc = download_real(c, c->phi, phi))) return rc;
  if (omega) {
    if (c->inertial) {
      c->ops.row_c2r(c->om_s, c->om_r, nullptr, nullptr, c->geo, c->twx, c->stream);
      LE_TRY(hipGetLastError());
      if ((rc = download_real(c, c->om_r, omega))) return rc;
    } else {
      std::memset(omega, 0, c->n_real * sizeof(double));
    }
  }
  if (psi) {
    c->ops.row_c2r(c->ps_s, c->ps_r, nullptr, nullptr, c->geo, c->twx, c->stream);
    LE_TRY(hipGetLastError());
    if ((rc = download_real(c, c->ps_r, psi))) return rc;
  }
  if (step) *step = c->step;
  if (wraps) *wraps = c->wraps;
  return LE_OK;
}

int le_profile(le_ctx* c, int enable) {
  if (!c) return LE_EINVAL;
  if (enable && c->events.empty()) {
    c->events.resize((size_t)kProfChunk * (LE_NSTAGES + 1));
    for (auto& e : c->events) {
      if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        return LE_EDEVICE;
      }
    }
  }
  c->profiling = enable != 0;
  for (int s = 0; s < LE_NSTAGES; ++s) {
    c->stage_ms[s] = 0.0;
    c->stage_n[s] = 0;
  }
  return LE_OK;
}

int le_stage_times(le_ctx* c, double* ms, int64_t* launches, int32_t cap) {
  if (!c || cap < 0) return LE_EINVAL;
  const int n = cap < LE_NSTAGES ? cap : LE_NSTAGES;
  for (int s = 0; s < n; ++s) {
    if (ms) ms[s] = c->stage_ms[s];
    if (launches) launches[s] = c->stage_n[s];
  }
  return LE_OK;
}

int le_set_state(le_ctx* c, const double* phi, const double* omega, const double* psi,
                 int64_t step, int64_t wraps) {
  if (!c || !phi || !psi || step < 0) return LE_EINVAL;
  if (c->inertial && !omega) return LE_EINVAL;
  if (wraps != wrap_count(c->p, step)) return LE_EINVAL;
  int rc;
  if ((rc = upload_real(c, phi, c->phi))) return rc;
  if (c->inertial) {
    if ((rc = upload_real(c, omega, c->om_r))) return rc;
    c->ops.row_r2c(c->om_r, c->om_s, c->geo, c->twx, c->stream);
  }
  if ((rc = upload_real(c, psi, c->ps_r))) return rc;
  c->ops.row_r2c(c->ps_r, c->ps_s, c->geo, c->twx, c->stream);
  LE_TRY(hipGetLastError());
  LE_TRY(hipStreamSynchronize(c->stream));
  c->step = step;
  c->wraps = wraps;
  return LE_OK;
}

}  // extern "C"

namespace le {
bool get_ops(int precision, int nx, int ny, Ops* ops) {
  return precision == LE_FP64 ? get_ops_f64(nx, ny, ops) : get_ops_f32(nx, ny, ops);
}
}  // namespace le
