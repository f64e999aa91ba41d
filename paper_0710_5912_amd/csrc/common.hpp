// common.hpp -- shared device/host definitions of the model-H library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace le {

// Geometry and physical constants of one run (see le_params in le.h).
struct Geo {
  int nx, ny;     // grid
  int r;          // nx / ny: x offset in cells of the sheared y stencil
  int f_half;     // 1: f = (phi_h)^3 from the advected phi instead of (phi^n)^3
  int upwind3;    // 1: third-order upwind differences of the advected fields
  int banded;     // 1: y part of the per-mode operators by central differences
  double lx, ly, dx, dy, c;   // c = lx / ly, the sawtooth jump
  double A, B, kappa, M, eta, rho, dt;
  double kx0, ky0;   // 2 pi / lx, 2 pi / ly (wavenumber quanta)
};

// Per-step values computed by the host shear clock.
struct StepArgs {
  double s;       // sawtooth strain offset s_n used by every operator of step n
  double pad;
};

// Device buffers of one run (storage type T, as void*).
enum Buf {
  B_PHI = 0,  // real phi (state)
  B_OM_S,     // row spectrum of omega (state, inertial runs)
  B_PS_S,     // row spectrum of psi (state)
  B_OM_R,     // real scratch: omega
  B_PS_R,     // real scratch: psi
  B_PHIH,     // row spectra, scratch
  B_FH,
  B_OMH,
  B_GH,
  B_PHIN,
  B_TMP,      // real scratch (remap, downloads, stencil outputs)
  B_R1,       // real scratch (stencil outputs of the two-kernel stage forms)
  B_R2,
  NBUF
};

// Row spectra (modes m = 0 .. nx/2 of every row) are stored column-tiled:
// tiles of kTW adjacent modes, each tile holding its ny rows one after the
// other, so element (row j, mode m) sits at
//   ((m / kTW) * ny + j) * kTW + m % kTW.
// A column pass then reads and writes each tile as one contiguous run, and a
// row pass writes kTW adjacent modes of a row per tile.  The last tile is
// padded (nx/2 + 1 is odd); the pad column is never read as data.
constexpr int kTW = 2;
__host__ __device__ constexpr int spec_tiles(int nx) { return (nx / 2 + 1 + kTW - 1) / kTW; }
// Complex elements of one row-spectrum buffer.
__host__ __device__ constexpr size_t spec_elems(int nx, int ny) {
  return (size_t)spec_tiles(nx) * (size_t)ny * kTW;
}
__host__ __device__ __forceinline__ size_t spec_index(int ny, int j, int m) {
  return ((size_t)(m / kTW) * (size_t)ny + (size_t)j) * kTW + (size_t)(m % kTW);
}

// Descriptor of one run, read by the kernels (blockIdx.z picks the run).
struct Run {
  Geo g;
  void* buf[NBUF];
  const void* twx;   // FP64 complex exp(-2 pi i k / nx), k < nx
  const void* twy;   // FP64 complex exp(-2 pi i k / (2 ny)), k < 2 ny
};

// Column-kernel variants (per-mode update applied between the transforms).
enum ColMode { COL_CH = 0, COL_FLOW = 1, COL_STOKES = 2, COL_POISSON = 3 };
// Flag on a column mode: the per-mode operators of the banded scheme switch
// (a kernel of its own, so the default kernels carry none of its code).
constexpr int COL_BANDED = 8;

// Observable partial sums (FP64), in this order.
enum {
  OBS_SUM_S = 0,       // sum over all modes of S
  OBS_SUM_S_NZ,        // sum over q != 0 of S
  OBS_SUM_S_OVER_Q,    // sum over q != 0 of S / |q_lab|
  OBS_XX,              // sum qx^2 S
  OBS_XY,              // sum qx q_lab_y S
  OBS_YY,              // sum q_lab_y^2 S
  OBS_RE,              // sum qx q_lab_y |Psi|^2
  OBS_NSPEC,
  OBS_SUM_PHI = OBS_NSPEC,   // real-space sum phi
  OBS_SUM_PHI2,              // real-space sum phi^2
  OBS_NONFINITE,             // count of non-finite phi values
  OBS_NTOTAL
};

}  // namespace le
