// ops.hpp -- type-erased launchers of the stage kernels for one precision and
// one grid shape.  Every step launcher covers `nruns` runs of that shape at
// once (grid z = run); `runs` is a device array of descriptors and `sa` the
// matching per-run StepArgs of the step.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.hpp"

namespace le {

// The corrected step's update (row_r2c_corr): network output z ([pixel][2]
// FP32), nblk per-tile FP64 partial sums of z_phi, output scales.
struct CorrArgs {
  const float* z;
  const double* part;
  int nblk;
  float s2, s3;
  int proj;  // 0: subtract the mean of z_phi; 1: subtract its tile means,
             // interpolated bilinearly between the 16 x 16 tile centres
};

// Advect variants from kStripFft on: kStripFft + k = the strip stencil over
// k-row strips with the row transforms in the same kernel, two x pairs per
// thread; kStripFft1 + k the same with one pair per thread.
constexpr int kStripFft = 64, kStripFft1 = 96;
// Advect and mu_source variants kAdvBatch + k, kAdvBatch2 + k and
// kAdvBatch3 + k: the batched one-kernel form over k-row strips in batches of
// four rows (16 values per thread in the row transforms), two rows (8) or two
// rows (16) (nx 512 .. 4096 with at least one wavefront per transform group,
// mu_source on square cells; elsewhere the two-kernel strip over k rows).
constexpr int kAdvBatch = 128, kAdvBatch2 = 192, kAdvBatch3 = 256;
// Advect variant kAdvUpwind: the third-order upwind differences of the scheme
// switch LE_SCHEME_UPWIND3 (stencil kernel, then the forward row transforms).
constexpr int kAdvUpwind = 1024;

struct Ops {
  // row transforms; variant (a tuning choice): 0 = 8 values per thread, 1 = 4
  void (*row_r2c)(const Run* runs, int nruns, int ny, int bin, int bout, int variant,
                  hipStream_t st);
  // njobs (<= 3) forward row transforms in one launch: real bins[k] -> spectra bouts[k]
  void (*row_r2c_n)(const Run* runs, int nruns, int ny, const int* bins, const int* bouts,
                    int njobs, int variant, hipStream_t st);
  // one run: the corrected step's update of phi and omega from the network
  // output and the forward row transform of omega (B_OM_R -> B_OM_S)
  void (*row_r2c_corr)(const Run* runs, int ny, const CorrArgs& ca, int variant, hipStream_t st);
  // inverse row transforms: bin0 -> bout0 and, when nfields == 2, bin1 -> bout1
  void (*row_c2r)(const Run* runs, int nruns, int ny, int bin0, int bout0, int bin1, int bout1,
                  int nfields, int variant, hipStream_t st);
  // stage 1a + forward row transforms (omega parts only when inertial);
  // variant: 0 fused, 0 < k < kStripFft strip stencil over k-row strips +
  // in-place transforms, kStripFft + k the same strips with the transforms
  // in one kernel
  void (*advect)(const Run* runs, int nruns, int ny, const StepArgs* sa, bool inertial,
                 int variant, int row_variant, hipStream_t st);
  // stage 2a + forward row transform of g; variant: 0 two kernels through
  // the real scratch, 0 < k < kStripFft strip stencil over k-row strips
  // (square cells) + in-place transform, kStripFft + k the same strips with
  // the transform in one kernel
  void (*mu_source)(const Run* runs, int nruns, int ny, const StepArgs* sa, int variant,
                    int row_variant, hipStream_t st);
  // column transform + per-mode update (ColMode) + inverse column transform;
  // variant 0 .. kColVariants-1 picks the block shape
  void (*column)(int mode, const Run* runs, int nruns, int nx, const StepArgs* sa, int bin0,
                 int bin1, int bout0, int bout1, int variant, hipStream_t st);
  // one run: spectral observable partials (bpsi < 0: no psi)
  void (*obs_spectral)(const Run* run, int nx, const StepArgs* sa, int bphi, int bpsi,
                       double* part, double* bins, double* counts, hipStream_t st);
  int (*obs_blocks)(int nx);
  void (*obs_real)(const Run* run, int b, double* part, int nblk, hipStream_t st);
  void (*remap_spec)(const Run* run, int b, int dkr, hipStream_t st);
  void (*remap_real)(const Run* run, int bin, int bout, int dkr, hipStream_t st);
  void (*copy_real)(const Run* run, int bin, int bout, hipStream_t st);
  void (*restrict_real)(const Run* run, int bin, int f, double* out, hipStream_t st);
};

// Fill *ops for precision (0 = double, 1 = float) and the grid; false if the
// grid is outside the instantiated range (8 .. 4096, powers of two).
bool get_ops(int precision, int nx, int ny, Ops* ops);
bool get_ops_f64(int nx, int ny, Ops* ops);
bool get_ops_f32(int nx, int ny, Ops* ops);

// Final reductions of the observables' partials into out (OBS_NTOTAL sums,
// then nbins shell sums, then nbins shell weights); gsum: scratch of
// 2 obs_shell_groups(nsblk) nbins doubles (unused when nbins == 0).
void launch_obs_final(const double* spart, int nsblk, const double* rpart, int nrblk,
                      const double* bins, const double* counts, int nbins, double* gsum,
                      double* out, hipStream_t st);
int obs_shell_groups(int nsblk);

}  // namespace le
