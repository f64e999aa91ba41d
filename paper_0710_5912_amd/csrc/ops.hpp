// ops.hpp -- type-erased launchers of the stage kernels for one precision and
// one grid, so the runtime can pick the instantiation at context creation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.hpp"

namespace le {

struct Ops {
  // forward row transform of a real field into a row spectrum
  void (*row_r2c)(const void* x, void* X, const Geo& g, const void* twx, hipStream_t st);
  // inverse row transform of one (X1 == nullptr) or two fields
  void (*row_c2r)(const void* X0, void* x0, const void* X1, void* x1, const Geo& g,
                  const void* twx, hipStream_t st);
  // stage 1a + forward row transforms (omega parts only when inertial)
  void (*advect)(const void* phi, const void* om, const void* psi, void* phih, void* fh,
                 void* omh, const StepArgs* sa, const Geo& g, const void* twx, bool inertial,
                 hipStream_t st);
  // stage 2a + forward row transform of g
  void (*mu_source)(const void* phi, void* gh, const StepArgs* sa, const Geo& g,
                    double inv_coef, const void* twx, hipStream_t st);
  // column transform + per-mode update + inverse (mode: ColMode)
  void (*column)(int mode, const void* in0, const void* in1, void* out0, void* out1,
                 const StepArgs* sa, const Geo& g, const void* twy, hipStream_t st);
  // spectral observable partials; returns nothing, see obs_blocks
  void (*obs_spectral)(const void* phih, const void* psih, double* part, double* bins,
                       double* counts, const StepArgs* sa, const Geo& g, const void* twy,
                       hipStream_t st);
  int (*obs_blocks)(const Geo& g);
  void (*obs_real)(const void* phi, size_t n, double* part, int nblk, hipStream_t st);
  void (*remap_spec)(void* X, const Geo& g, int dkr, const void* twx, hipStream_t st);
  void (*remap_real)(const void* in, void* out, const Geo& g, int dkr, hipStream_t st);
};

// Fill *ops for precision (0 = double, 1 = float) and the grid; false if the
// grid is outside the instantiated range (8 .. 4096, powers of two).
bool get_ops(int precision, int nx, int ny, Ops* ops);
bool get_ops_f64(int nx, int ny, Ops* ops);
bool get_ops_f32(int nx, int ny, Ops* ops);

void launch_obs_final(const double* spart, int nsblk, const double* rpart, int nrblk,
                      const double* bins, const double* counts, int nbins, double* out,
                      hipStream_t st);

}  // namespace le
