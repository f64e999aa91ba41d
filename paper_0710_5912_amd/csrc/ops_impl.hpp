// ops_impl.hpp -- template launchers behind the Ops table (included once per
// precision by ops_f64.hip / ops_f32.hip).
#pragma once

#include "ops.hpp"
#include "stages.hpp"

namespace le {

template <typename T, int L>
struct RowLaunch {
  using C = RowCfg<L>;
  static dim3 grid(const Geo& g) { return dim3((g.ny + C::G - 1) / C::G); }
  static void r2c(const void* x, void* X, const Geo& g, const void* tw, hipStream_t st) {
    hipLaunchKernelGGL((k_row_r2c<T, L>), grid(g), dim3(C::THREADS), 0, st,
                       static_cast<const T*>(x), static_cast<c2<T>*>(X), g.ny,
                       static_cast<const c2<T>*>(tw));
  }
  static void c2r(const void* X0, void* x0, const void* X1, void* x1, const Geo& g,
                  const void* tw, hipStream_t st) {
    dim3 gr = grid(g);
    gr.y = X1 ? 2 : 1;
    hipLaunchKernelGGL((k_row_c2r<T, L>), gr, dim3(C::THREADS), 0, st,
                       static_cast<const c2<T>*>(X0), static_cast<T*>(x0),
                       static_cast<const c2<T>*>(X1), static_cast<T*>(x1), g.ny,
                       static_cast<const c2<T>*>(tw));
  }
  static void advect(const void* phi, const void* om, const void* psi, void* phih, void* fh,
                     void* omh, const StepArgs* sa, const Geo& g, const void* tw,
                     bool inertial, hipStream_t st) {
    dim3 gr = grid(g);
    gr.y = inertial ? 3 : 2;
    hipLaunchKernelGGL((k_advect<T, L>), gr, dim3(C::THREADS), 0, st,
                       static_cast<const T*>(phi), static_cast<const T*>(om),
                       static_cast<const T*>(psi), static_cast<c2<T>*>(phih),
                       static_cast<c2<T>*>(fh), static_cast<c2<T>*>(omh), sa, g,
                       static_cast<const c2<T>*>(tw));
  }
  static void mu_source(const void* phi, void* gh, const StepArgs* sa, const Geo& g,
                        double inv, const void* tw, hipStream_t st) {
    using M = MuCfg<L>;
    hipLaunchKernelGGL((k_mu_source<T, L>), dim3((g.ny + M::G - 1) / M::G), dim3(M::THREADS),
                       0, st, static_cast<const T*>(phi), static_cast<c2<T>*>(gh), sa, g, inv,
                       static_cast<const c2<T>*>(tw));
  }
};

template <typename T, int L>
struct ColLaunch {
  using C = ColCfg<L>;
  static dim3 grid(const Geo& g) { return dim3((g.nx / 2 + 1 + C::CW - 1) / C::CW); }
  static void column(int mode, const void* in0, const void* in1, void* out0, void* out1,
                     const StepArgs* sa, const Geo& g, const void* tw, hipStream_t st) {
    auto i0 = static_cast<const c2<T>*>(in0);
    auto i1 = static_cast<const c2<T>*>(in1);
    auto o0 = static_cast<c2<T>*>(out0);
    auto o1 = static_cast<c2<T>*>(out1);
    auto w = static_cast<const c2<T>*>(tw);
    switch (mode) {
      case COL_CH:
        hipLaunchKernelGGL((k_column<T, L, COL_CH>), grid(g), dim3(C::THREADS), 0, st, i0, i1,
                           o0, o1, sa, g, w);
        break;
      case COL_FLOW:
        hipLaunchKernelGGL((k_column<T, L, COL_FLOW>), grid(g), dim3(C::THREADS), 0, st, i0,
                           i1, o0, o1, sa, g, w);
        break;
      case COL_STOKES:
        hipLaunchKernelGGL((k_column<T, L, COL_STOKES>), grid(g), dim3(C::THREADS), 0, st, i0,
                           i1, o0, o1, sa, g, w);
        break;
      default:
        hipLaunchKernelGGL((k_column<T, L, COL_POISSON>), grid(g), dim3(C::THREADS), 0, st,
                           i0, i1, o0, o1, sa, g, w);
        break;
    }
  }
  static void obs(const void* phih, const void* psih, double* part, double* bins,
                  double* counts, const StepArgs* sa, const Geo& g, const void* tw,
                  hipStream_t st) {
    hipLaunchKernelGGL((k_obs_spectral<T, L>), grid(g), dim3(C::THREADS), 0, st,
                       static_cast<const c2<T>*>(phih), static_cast<const c2<T>*>(psih), part,
                       bins, counts, sa, g, static_cast<const c2<T>*>(tw));
  }
  static int blocks(const Geo& g) { return (int)grid(g).x; }
};

template <typename T>
struct Misc {
  static void obs_real(const void* phi, size_t n, double* part, int nblk, hipStream_t st) {
    hipLaunchKernelGGL((k_obs_real<T>), dim3(nblk), dim3(256), 0, st,
                       static_cast<const T*>(phi), n, part);
  }
  static void remap_spec(void* X, const Geo& g, int dkr, const void* tw, hipStream_t st) {
    hipLaunchKernelGGL((k_remap_spec<T>), dim3(1024), dim3(256), 0, st, static_cast<c2<T>*>(X),
                       g.nx, g.ny, dkr, static_cast<const c2<T>*>(tw));
  }
  static void remap_real(const void* in, void* out, const Geo& g, int dkr, hipStream_t st) {
    hipLaunchKernelGGL((k_remap_real<T>), dim3(1024), dim3(256), 0, st,
                       static_cast<const T*>(in), static_cast<T*>(out), g.nx, g.ny, dkr);
  }
};

template <typename T, int L>
void set_row(Ops* o) {
  o->row_r2c = &RowLaunch<T, L>::r2c;
  o->row_c2r = &RowLaunch<T, L>::c2r;
  o->advect = &RowLaunch<T, L>::advect;
  o->mu_source = &RowLaunch<T, L>::mu_source;
}

template <typename T, int L>
void set_col(Ops* o) {
  o->column = &ColLaunch<T, L>::column;
  o->obs_spectral = &ColLaunch<T, L>::obs;
  o->obs_blocks = &ColLaunch<T, L>::blocks;
}

template <typename T>
bool fill_ops(int nx, int ny, Ops* o) {
  switch (nx) {
    case 8: set_row<T, 4>(o); break;
    case 16: set_row<T, 8>(o); break;
    case 32: set_row<T, 16>(o); break;
    case 64: set_row<T, 32>(o); break;
    case 128: set_row<T, 64>(o); break;
    case 256: set_row<T, 128>(o); break;
    case 512: set_row<T, 256>(o); break;
    case 1024: set_row<T, 512>(o); break;
    case 2048: set_row<T, 1024>(o); break;
    case 4096: set_row<T, 2048>(o); break;
    default: return false;
  }
  switch (ny) {
    case 8: set_col<T, 8>(o); break;
    case 16: set_col<T, 16>(o); break;
    case 32: set_col<T, 32>(o); break;
    case 64: set_col<T, 64>(o); break;
    case 128: set_col<T, 128>(o); break;
    case 256: set_col<T, 256>(o); break;
    case 512: set_col<T, 512>(o); break;
    case 1024: set_col<T, 1024>(o); break;
    case 2048: set_col<T, 2048>(o); break;
    case 4096: set_col<T, 4096>(o); break;
    default: return false;
  }
  o->obs_real = &Misc<T>::obs_real;
  o->remap_spec = &Misc<T>::remap_spec;
  o->remap_real = &Misc<T>::remap_real;
  return true;
}

}  // namespace le
