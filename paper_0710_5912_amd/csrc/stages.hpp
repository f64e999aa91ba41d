// stages.hpp -- the stage kernels of the split step (Appendix B), templated
// on the storage type T (float or double) and the transform lengths.
//
// Field layouts in HBM:
//   real field       T[ny][nx], x fastest
//   row spectrum     the unnormalised DFT of each real row along x, modes
//                    m = 0 .. nx/2 (DC and Nyquist real), column-tiled:
//                    (row j, mode m) at spec_index(ny, j, m) (common.hpp),
//                    so that each tile of kTW modes is one contiguous run
//                    down the column.
// A 2D transform is a row transform (fused into the row kernels) followed by
// a column transform over each of the nx/2+1 columns (fused into the column
// kernels, which also apply the per-mode update and the inverse column
// transform, scaled by 1/ny).  Row kernels own G whole rows per block, column
// kernels CW adjacent columns per block.
#pragma once

#include "common.hpp"
#include "fft.hpp"
#include "ops.hpp"

namespace le {

// Launch shapes.  E: values per thread of a transform (P = L/E threads per
// transform); G: rows per block; CW: adjacent columns per block.
constexpr int row_elems(int L) { return L >= 8 ? 8 : L; }
constexpr int col_elems(int L) { return L >= 8 ? 8 : L; }

// Occupancy hint for the stage kernels (waves per SIMD the register
// allocation must allow).
#ifndef LE_COL_DUAL
#define LE_COL_DUAL 1
#endif
#ifndef LE_WAVES
#define LE_WAVES 2
#endif
#ifndef LE_WAVES_COL
#define LE_WAVES_COL LE_WAVES
#endif
#define LE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(LE_WAVES)))
#define LE_OCCUPANCY_COL __attribute__((amdgpu_waves_per_eu(LE_WAVES_COL)))
// Keep the scheduler from interleaving consecutive unrolled iterations (which
// would hoist every iteration's loads and blow the register budget).
#define LE_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int L, int E_ = row_elems(L), int GDIV = 1>
struct RowCfg {
  static constexpr int E = E_;
  static constexpr int P = L / E;
  static constexpr int G0 = clampi(128 / P, 1, 16);
  static constexpr int G = G0 / GDIV > 1 ? G0 / GDIV : 1;  // rows per block
  static constexpr int THREADS = G * P;
};

// Column kernel shapes, VAR (a tuning choice, 0 .. 4): E values per thread
// (8, or 16 for VAR 3 and 4: two register passes fewer LDS exchanges) and
// CW adjacent columns per block: CW0 = 256/P (VAR 0, 3), twice that (VAR 1,
// 4) where threads <= 1024 and LDS <= 160 KB allow, or a quarter (VAR 2:
// more, smaller blocks for grids whose column pass has few blocks).
template <typename T, int L, int VAR>
struct ColCfg {
  static constexpr int E = (VAR >= 3 && L >= 16) ? 16 : col_elems(L);
  static constexpr int P = L / E;
  static constexpr int CW0 = clampi(256 / P, 1, 64);
  static constexpr int CWD = (VAR == 1 || VAR == 4) ? 2 * CW0
                             : (VAR == 2 ? (CW0 / 4 > 1 ? CW0 / 4 : 1) : CW0);
  static constexpr bool FITS =
      CWD <= 64 && CWD * P <= 1024 && (long)CWD * L * (long)sizeof(c2<T>) <= 160L * 1024;
  static constexpr int CW = FITS ? CWD : CW0;
  static constexpr int THREADS = CW * P;
};
constexpr int kColVariants = 5;

// Observables' column kernel (its LDS also holds the shell partials).
template <int L>
struct ObsCfg {
  static constexpr int E = col_elems(L);
  static constexpr int P = L / E;
  static constexpr int CW = clampi(256 / P, 1, 64);
  static constexpr int THREADS = CW * P;
};

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// Give each XCD a contiguous range of logical blocks so that neighbouring
// rows (stencil halos) and columns sharing cache lines meet in one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7;
  return x * q + (x < rem ? x : rem) + (b >> 3);
}

// Logical (x, y, z) of this block: the XCD-aware map applied to the linear
// block index, so consecutive x (rows or columns) of one field and run land
// in one L2.
struct BPos {
  int x, y, z;
};
__device__ __forceinline__ BPos block_pos() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int nb = gx * gy * gridDim.z;
  const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int l = xcd_block(lin, nb);
  const int rest = l / gx;
  return {l % gx, rest % gy, rest / gy};
}

template <typename T>
__device__ __forceinline__ gp<T> bufp(const Run& R, int b) {
  return to_global<T>(R.buf[b]);
}

// ---------------------------------------------------------------- helpers

// Row j of a (column-tiled) row spectrum X with ny rows: the packed half
// spectrum of row_r2c (v[q] = X[m], m = t + q P, with (X[0], X[L]) at m = 0)
// stored as modes 0 .. L.
template <typename T, int L, int E>
__device__ __forceinline__ void store_row_spec(gp<c2<T>> __restrict__ X, int ny, int j,
                                               const c2<T>* v, int t) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = t + q * P;
    if (m == 0) {
      stg<T>(X + spec_index(ny, j, 0), {v[q].x, T(0)});
      stg<T>(X + spec_index(ny, j, L), {v[q].y, T(0)});
    } else {
      stg<T>(X + spec_index(ny, j, m), v[q]);
    }
  }
}

template <typename T, int L, int E>
__device__ __forceinline__ void load_row_spec(gp<const c2<T>> __restrict__ X, int ny, int j,
                                              c2<T>* v, int t) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = t + q * P;
    const c2<T> xm = ldg<T>(X + spec_index(ny, j, m));
    v[q] = (m == 0) ? c2<T>{xm.x, X[spec_index(ny, j, L)].x} : xm;
  }
}

// Signed wavenumbers of column m (0 .. nx/2) and row n (0 .. ny-1) and the
// odd product qx qy (zero on the Nyquist row/column, so every multiplier is
// Hermitian and the transforms stay real).
struct Modes {
  double qx, qy, P;
};
// Step kernels: wavenumbers as multiples of the quanta 2 pi / l.
__device__ __forceinline__ Modes modes(const Geo& g, int m, int n) {
  const int ms = (m >= g.nx / 2) ? m - g.nx : m;
  const int ns = (n >= g.ny / 2) ? n - g.ny : n;
  Modes r;
  r.qx = g.kx0 * (double)ms;
  r.qy = g.ky0 * (double)ns;
  r.P = (m == g.nx / 2 || n == g.ny / 2) ? 0.0 : r.qx * r.qy;
  return r;
}

// Observables: wavenumbers formed as (2 pi m) / l, the exact rounding the
// shell decision is specified with.
__device__ __forceinline__ Modes modes_exact(const Geo& g, int m, int n) {
  const int ms = (m >= g.nx / 2) ? m - g.nx : m;
  const int ns = (n >= g.ny / 2) ? n - g.ny : n;
  const double twopi = 6.283185307179586476925286766559;
  Modes r;
  r.qx = twopi * (double)ms / g.lx;
  r.qy = twopi * (double)ns / g.ly;
  r.P = (m == g.nx / 2 || n == g.ny / 2) ? 0.0 : r.qx * r.qy;
  return r;
}

// 1/x to full double precision: hardware estimate plus two Newton steps
// (x != 0; the callers mask the q = 0 mode).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// lambda(q; s) = D + Delta, D = -((1 + s^2) qx^2 + qy^2), Delta = 2 s qx qy:
// the eigenvalue of the cosheared Laplacian block of Appendix B.
__device__ __forceinline__ double lambda_of(const Modes& q, double s) {
  const double D = -((1.0 + s * s) * q.qx * q.qx + q.qy * q.qy);
  return D + 2.0 * s * q.P;
}

// The banded scheme switch: the same operator with its y part by the central
// differences of the stencils, i.e. the eigenvalue of the cyclic banded
// operator of column m on the y wave n:
//   -(1 + s^2) qx^2 - 4 sin^2(pi n / ny) / dy^2 + 2 s qx sin(2 pi n / ny) / dy,
// the cross term dropped on the x Nyquist column (the y Nyquist row has
// sin = 0).  Solving the cyclic tri-/penta-diagonal systems of each column
// is the per-mode division by this value (the DFT along y diagonalizes
// them: their coefficients do not depend on y).
__device__ __forceinline__ double lambda_banded(const Geo& g, int m, int n, double s) {
  const int ms = (m >= g.nx / 2) ? m - g.nx : m;
  const double qx = g.kx0 * (double)ms;
  double sh, ch, s2, c2;
  sincospi((double)n / (double)g.ny, &sh, &ch);        // sin, cos(pi n / ny)
  sincospi(2.0 * (double)n / (double)g.ny, &s2, &c2);  // sin, cos(2 pi n / ny)
  const double cross = (m == g.nx / 2) ? 0.0 : 2.0 * s * qx * s2 / g.dy;
  return -((1.0 + s * s) * qx * qx) - 4.0 * sh * sh / (g.dy * g.dy) + cross;
}

// ---------------------------------------------------------------- row kernels

// Forward row transforms: blockIdx.y picks the job (real buffer bin, row
// stride rs elements -> row spectrum bout).  With rs = nx + 2 the real rows
// sit at the spectral rows' offsets and the transform may run in place
// (bin == bout): a block reads its whole row before it writes any of it.
struct R2cJob {
  int bin, bout, rs;
};
struct R2cJobs {
  R2cJob j[3];
};

template <typename T, int L, int E = row_elems(L), int GDIV = 1>
__global__ __launch_bounds__((RowCfg<L, E, GDIV>::THREADS)) LE_OCCUPANCY void k_row_r2c(
    const Run* __restrict__ runs, R2cJobs jobs) {
  using C = RowCfg<L, E, GDIV>;
  __shared__ c2<T> lds[C::G * L];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const R2cJob job = jobs.j[bp.y];
  const int ny = R.g.ny;
  auto x = bufp<T>(R, job.bin);
  auto X = bufp<c2<T>>(R, job.bout);
  auto tw = to_global<const c2<double>>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j = bp.x * C::G + g;
  const bool ok = j < ny;
  auto xr = reinterpret_cast<gp<const c2<T>>>(x + (size_t)(ok ? j : 0) * job.rs);
  c2<T> v[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) v[q] = ldg<T>(xr + t + q * C::P);
  row_r2c<T, L, C::E>(v, lds + g * L, tw, t);
  if (ok) store_row_spec<T, L, C::E>(X, ny, j, v, t);
}

// The corrected step's update and the vorticity's forward row transform in
// one pass (one run): phi += s2 (z_phi - mean), omega += s3 z_omega with z
// the network output ([pixel][2] FP32) and mean = (sum of the nblk per-tile
// partials of z_phi) / (nx ny), formed by every block in the same fixed
// order; the corrected real rows are stored and omega's row spectrum is
// written to B_OM_S.
template <typename T, int L, int E = row_elems(L), int GDIV = 1>
__global__ __launch_bounds__((RowCfg<L, E, GDIV>::THREADS)) LE_OCCUPANCY void k_row_r2c_corr(
    const Run* __restrict__ runs, CorrArgs ca) {
  using C = RowCfg<L, E, GDIV>;
  constexpr int NW = (C::THREADS + 63) / 64;
  __shared__ c2<T> lds[C::G * L];
  __shared__ double wred[NW];
  const Run& R = runs[0];
  const int ny = R.g.ny;
  auto phi = reinterpret_cast<gp<c2<T>>>(bufp<T>(R, B_PHI));
  auto om = reinterpret_cast<gp<c2<T>>>(bufp<T>(R, B_OM_R));
  auto X = bufp<c2<T>>(R, B_OM_S);
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  auto zz = to_global<const f32x4>(reinterpret_cast<const f32x4*>(ca.z));
  auto tw = to_global<const c2<double>>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j = blockIdx.x * C::G + g;
  const bool ok = j < ny;
  const size_t row = (size_t)(ok ? j : 0) * L;
  // the row's operands are requested before the mean is formed
  c2<T> f[C::E], w[C::E];
  f32x4 zq[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) {
    const size_t m = row + t + q * C::P;  // the pair (2m, 2m + 1) of the field
    zq[q] = zz[m];                        // z_phi, z_omega of both points
    f[q] = ldg<T>(phi + m);
    w[q] = ldg<T>(om + m);
  }
  // sum of the partials: per thread a strided sum, a butterfly within each
  // wavefront, then the wavefront sums in order (the same order in every
  // block)
  double acc = 0.0;
  for (int k = threadIdx.x; k < ca.nblk; k += C::THREADS) acc += ca.part[k];
  constexpr int WS = C::THREADS < 64 ? C::THREADS : 64;  // lanes of a (partial) wavefront
#pragma unroll
  for (int off = WS / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, WS);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = acc;
  __syncthreads();
  double total = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) total += wred[k];
  const double mean = total / ((double)ny * (double)(2 * L));
  // with ca.proj, the subtracted field is the tile means of z_phi
  // interpolated bilinearly between the tile centres (periodic): it sums to
  // the same total, and it removes the residual's content at scales beyond a
  // tile
  constexpr int FT = 16;
  const int tx = 2 * L / FT, ty = ny / FT;
  auto tile_mean = [&](int x) {
    const double u = (x + 0.5) / FT - 0.5, w = (ok ? j : 0) + 0.5;
    const double vv = w / FT - 0.5;
    const int i0 = (int)floor(u), j0 = (int)floor(vv);
    const double fx = u - i0, fy = vv - j0;
    const int ia = (i0 + tx) % tx, ib = (i0 + 1) % tx;
    const int ja = (j0 + ty) % ty, jb = (j0 + 1) % ty;
    const double inv = 1.0 / (FT * FT);
    return inv * ((1.0 - fy) * ((1.0 - fx) * ca.part[ja * tx + ia] + fx * ca.part[ja * tx + ib]) +
                  fy * ((1.0 - fx) * ca.part[jb * tx + ia] + fx * ca.part[jb * tx + ib]));
  };
  c2<T> v[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) {
    const size_t m = row + t + q * C::P;
    const int x0 = 2 * (t + q * C::P);
    const double m0 = ca.proj ? tile_mean(x0) : mean, m1 = ca.proj ? tile_mean(x0 + 1) : mean;
    const c2<T> fn = {(T)((double)f[q].x + (double)ca.s2 * ((double)zq[q].x - m0)),
                      (T)((double)f[q].y + (double)ca.s2 * ((double)zq[q].z - m1))};
    v[q] = {(T)((double)w[q].x + (double)ca.s3 * (double)zq[q].y),
            (T)((double)w[q].y + (double)ca.s3 * (double)zq[q].w)};
    if (ok) {
      stg<T>(phi + m, fn);
      stg<T>(om + m, v[q]);
    }
  }
  row_r2c<T, L, C::E>(v, lds + g * L, tw, t);
  if (ok) store_row_spec<T, L, C::E>(X, ny, j, v, t);
}

// Inverse row transform; the block's y picks the field (bin0 -> bout0, or
// bin1 -> bout1).
template <typename T, int L, int E = row_elems(L), int GDIV = 1>
__global__ __launch_bounds__((RowCfg<L, E, GDIV>::THREADS)) LE_OCCUPANCY void k_row_c2r(
    const Run* __restrict__ runs, int bin0, int bout0, int bin1, int bout1) {
  using C = RowCfg<L, E, GDIV>;
  __shared__ c2<T> lds[C::G * L];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const int ny = R.g.ny;
  auto X = bufp<const c2<T>>(R, bp.y == 0 ? bin0 : bin1);
  auto x = bufp<T>(R, bp.y == 0 ? bout0 : bout1);
  auto tw = to_global<const c2<double>>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j = bp.x * C::G + g;
  const bool ok = j < ny;
  const int jj = ok ? j : 0;
  c2<T> v[C::E];
  load_row_spec<T, L, C::E>(X, ny, jj, v, t);
  row_c2r<T, L, C::E>(v, lds + g * L, tw, t);
  if (ok) {
    auto xr = reinterpret_cast<gp<c2<T>>>(x + (size_t)j * 2 * L);
#pragma unroll
    for (int q = 0; q < C::E; ++q) stg<T>(xr + t + q * C::P, v[q]);
  }
}

// Row stride of an LDS area that stages NR row spectra for tile-run stores:
// at least L + 1 (the Nyquist slot), padded so that the NR kTW elements of
// the tile runs that one bank row's worth of lanes reads (16 lanes in FP64,
// 32 in FP32) fall on distinct banks.
template <typename T, int NR>
constexpr int staged_stride(int L) {
  constexpr int S = 256 / (int)sizeof(c2<T>);
  return L + (S / NR > 1 ? S / NR : 1);
}

// Visits the elements of the tile runs of nr staged rows, f(r, m) for row r
// and mode m <= L, thread t taking elements t, t + NT, ...: element e is
// entry w = e mod (kTW nr) of tile k = e / (kTW nr), i.e. row w / kTW, mode
// k kTW + w mod kTW.  RUN = kTW nr when known at compile time (the division
// then folds to shifts), else 0.
template <int L, int NT, int RUN, typename F>
__device__ __forceinline__ void for_tile_runs(int nr, F&& f) {
  const int run = RUN > 0 ? RUN : kTW * nr;
  const int total = (L / kTW + 1) * run;
  for (int e = threadIdx.x; e < total; e += NT) {
    const int k = e / run, w = e % run;
    const int r = w / kTW, m = k * kTW + w % kTW;
    if (m <= L) f(r, m);
  }
}
template <int L, int NT, int NR, typename F>
__device__ __forceinline__ void tile_runs(int nr, F&& f) {
  if (nr == NR)
    for_tile_runs<L, NT, kTW * NR>(nr, f);
  else
    for_tile_runs<L, NT, 0>(nr, f);
}

// Row transforms with the row spectra staged through LDS.  A block owns RB
// consecutive rows (RB >= RB0, a power of two): the forward transforms leave
// the RB rows' complex transforms in LDS (row_r2c_z), and the block stores
// the half spectra tile by tile (r2c_mode), consecutive
// threads writing consecutive elements of a tile (the RB rows' kTW modes),
// so every store instruction writes whole runs of RB kTW values instead of
// one row's kTW values per tile; the inverse loads the same runs into LDS
// and hands each row to its transform group.  Rows in LDS have the stride
// staged_stride (room for the packed DC/Nyquist slot plus the Nyquist mode).
template <int L, int E, int RB0>
struct RowT {
  static constexpr int P = L / E;
  static constexpr int G0 = clampi(128 / P, 1, 16);
  static constexpr int RB = G0 > RB0 ? G0 : RB0;  // rows per block
  static constexpr int THREADS = RB * P;
  static constexpr bool OK = THREADS <= 1024 && (long)RB * (L + 16) * 16 <= 160L * 1024;
};
// Blocks of the staged row kernels are taken in launch order (consecutive
// blocks go to different XCDs and run at the same time), so the blocks in
// flight cover consecutive rows: their tile runs lie next to each other.
__device__ __forceinline__ BPos block_pos_linear() {
  return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
}

template <typename T, int L, int E, int RB0>
__global__ __launch_bounds__((RowT<L, E, RB0>::THREADS)) LE_OCCUPANCY void k_row_r2c_t(
    const Run* __restrict__ runs, R2cJobs jobs) {
  using C = RowT<L, E, RB0>;
  constexpr int LS = staged_stride<T, C::RB>(L);
  __shared__ c2<T> lds[C::RB * LS];
  __shared__ c2<double> wtab[TwTab<L>::N];
  const BPos bp = block_pos_linear();
  const Run& R = runs[bp.z];
  const R2cJob job = jobs.j[bp.y];
  const int ny = R.g.ny;
  auto x = bufp<T>(R, job.bin);
  auto X = bufp<c2<T>>(R, job.bout);
  auto tw = to_global<const c2<double>>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j0 = bp.x * C::RB;  // ny is a power of two >= 8: whole blocks when RB <= ny
  const int rows = C::RB < ny ? C::RB : ny;
  const bool ok = g < rows;
  auto xr = reinterpret_cast<gp<const c2<T>>>(x + (size_t)(j0 + (ok ? g : 0)) * job.rs);
  c2<T> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) v[q] = ldg<T>(xr + t + q * C::P);
  tw_tab_fill<L, C::THREADS>(wtab, tw);
  row_r2c_z<T, L, E>(v, lds + g * LS, tw, t);
  __syncthreads();
  // tile k holds modes 2k, 2k + 1 (k = L/2: the Nyquist mode and the pad)
  tile_runs<L, C::THREADS, C::RB>(rows, [&](int r, int m) {
    stg<T>(X + spec_index(ny, j0 + r, m), r2c_mode<T, L>(lds + r * LS, wtab, m));
  });
}

template <typename T, int L, int E, int RB0>
__global__ __launch_bounds__((RowT<L, E, RB0>::THREADS)) LE_OCCUPANCY void k_row_c2r_t(
    const Run* __restrict__ runs, int bin0, int bout0, int bin1, int bout1) {
  using C = RowT<L, E, RB0>;
  constexpr int LS = staged_stride<T, C::RB>(L);
  __shared__ c2<T> lds[C::RB * LS];
  const BPos bp = block_pos_linear();
  const Run& R = runs[bp.z];
  const int ny = R.g.ny;
  auto X = bufp<const c2<T>>(R, bp.y == 0 ? bin0 : bin1);
  auto x = bufp<T>(R, bp.y == 0 ? bout0 : bout1);
  auto tw = to_global<const c2<double>>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j0 = bp.x * C::RB;
  const int rows = C::RB < ny ? C::RB : ny;
  tile_runs<L, C::THREADS, C::RB>(rows, [&](int r, int m) {
    lds[r * LS + m] = ldg<T>(X + spec_index(ny, j0 + r, m));
  });
  __syncthreads();
  const bool ok = g < rows;
  const int gr = ok ? g : 0;
  c2<T> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = t + q * C::P;
    v[q] = lds[gr * LS + m];
    if (m == 0) v[q].y = lds[gr * LS + L].x;
  }
  __syncthreads();
  row_c2r<T, L, E>(v, lds + g * L, tw, t);
  if (ok) {
    auto xr = reinterpret_cast<gp<c2<T>>>(x + (size_t)(j0 + g) * 2 * L);
#pragma unroll
    for (int q = 0; q < E; ++q) stg<T>(xr + t + q * C::P, v[q]);
  }
}

// Stencil coefficients of one step, in the storage precision.
template <typename T>
struct Stencil {
  T inv2dx, inv2dy, w, wm;  // 1/(2dx), 1/(2dy), |s|/c, 1 - |s|/c
  int off;                  // sign(s) * r: x offset of the diagonal y difference
};

template <typename T>
__device__ __forceinline__ Stencil<T> make_stencil(const Geo& g, double s) {
  Stencil<T> st;
  const double w = fabs(s) / g.c;
  st.inv2dx = T(1.0 / (2.0 * g.dx));
  st.inv2dy = T(1.0 / (2.0 * g.dy));
  st.w = T(w);
  st.wm = T(1.0 - w);
  st.off = s >= 0.0 ? g.r : -g.r;
  return st;
}

// ------------------------------------------------ x-pair access for row stencils
//
// The row kernels give thread t of a row the x pairs (x, x+1), x = 2(t + qP),
// q = 0 .. E-1: the layout the row transform consumes.  A stencil needs the
// values at x-1 and x+2 too; they are the neighbouring lanes' pairs, moved
// across the wavefront with DPP (wave_shr:1 / wave_shl:1), and only the
// lanes whose neighbour is not the adjacent lane (first/last of a row group
// or of the wavefront) read them from memory.

constexpr int kDppWaveShr1 = 0x138;  // lane i receives lane i-1 (lane 0 keeps its own)
constexpr int kDppWaveShl1 = 0x130;  // lane i receives lane i+1 (lane 63 keeps its own)

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  const int b = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  int lo = (int)b, hi = (int)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                                (unsigned)lo));
}

// f[x-1], f[x], f[x+1], f[x+2] of one row.
template <typename T>
struct Quad {
  T l, a0, a1, r;
};

// Row `row` (NX values), pair at even x.  Lanes with edge_l / edge_r take
// x-1 / x+2 from the halo values at xl / xr (the values left of the first and
// right of the last pair of the lane's run of adjacent lanes), which every
// lane reads: one address per run, so the reads cost no extra traffic and no
// branch.  Every lane of the wavefront must execute this (DPP reads the
// neighbours' registers).
template <typename T, int NX>
__device__ __forceinline__ Quad<T> load_quad(gp<const T> __restrict__ row, int x, int xl, int xr,
                                             bool edge_l, bool edge_r) {
  const c2<T> p = ldg<T>(reinterpret_cast<gp<const c2<T>>>(row + x));
  const T hl = row[xl & (NX - 1)];
  const T hr = row[xr & (NX - 1)];
  const T nl = dpp_mov<kDppWaveShr1>(p.y);
  const T nr = dpp_mov<kDppWaveShl1>(p.x);
  return {edge_l ? hl : nl, p.x, p.y, edge_r ? hr : nr};
}

// Lanes of a row group: thread t of P; runs of adjacent lanes are whole
// wavefronts when P >= 64, else the whole group.
template <int P>
struct LaneRun {
  int tl, tr;          // first and last t of the lane's run
  bool edge_l, edge_r;
  __device__ __forceinline__ LaneRun(int t) {
    tl = P >= 64 ? (t & ~63) : 0;
    tr = P >= 64 ? (t | 63) : P - 1;
    edge_l = t == tl;
    edge_r = t == tr;
  }
  // halo positions of pair slot q
  __device__ __forceinline__ int xl(int q) const { return 2 * (tl + q * P) - 1; }
  __device__ __forceinline__ int xr(int q) const { return 2 * (tr + q * P) + 2; }
};

// Aligned pair (f[x], f[x+1]) of a row, x even, taken periodically.
template <typename T, int NX>
__device__ __forceinline__ c2<T> load_pair(gp<const T> __restrict__ row, int x) {
  return ldg<T>(reinterpret_cast<gp<const c2<T>>>(row + (x & (NX - 1))));
}

// Central x difference at x and x+1.
template <typename T>
__device__ __forceinline__ void quad_dx(const Quad<T>& q, T inv2dx, T& d0, T& d1) {
  d0 = (q.a1 - q.l) * inv2dx;
  d1 = (q.r - q.a0) * inv2dx;
}

// Sheared y difference (Eq. p1y) at x and x+1 from rows j+1 (up) and j-1
// (dn): plain part up(x) - dn(x) weighted 1 - |s|/c, diagonal part
// up(x - off) - dn(x + off) weighted |s|/c, off = sign(s) r (unsheared:
// weights 1 and 0, the same value).  R1: r = 1, the diagonal values are the
// quads' own neighbours; otherwise r is even and they are aligned pairs read
// from the rows.  Branch-free.
template <typename T, int NX, bool R1>
__device__ __forceinline__ void quad_dys(const Quad<T>& up, const Quad<T>& dn,
                                         gp<const T> __restrict__ rowu, gp<const T> __restrict__ rowd,
                                         int x, const Stencil<T>& st, T& d0, T& d1) {
  T u0, u1, m0, m1;  // up(x - off), up(x + 1 - off), dn(x + off), dn(x + 1 + off)
  if constexpr (R1) {
    const bool pos = st.off > 0;
    u0 = pos ? up.l : up.a1;
    u1 = pos ? up.a0 : up.r;
    m0 = pos ? dn.a1 : dn.l;
    m1 = pos ? dn.r : dn.a0;
  } else {
    const c2<T> pu = load_pair<T, NX>(rowu, x - st.off);
    const c2<T> pd = load_pair<T, NX>(rowd, x + st.off);
    u0 = pu.x; u1 = pu.y; m0 = pd.x; m1 = pd.y;
  }
  d0 = (st.wm * (up.a0 - dn.a0) + st.w * (u0 - m0)) * st.inv2dy;
  d1 = (st.wm * (up.a1 - dn.a1) + st.w * (u1 - m1)) * st.inv2dy;
}

// One output field of a bracket row kernel.
//   JOB_ADVECT: out = a - dt [Dx a Dys b - Dys a Dx b]   (stage 1a, b = psi)
//   JOB_CUBE:   out = a^3                                  (stage 1a, f; with
//               geo.f_half the JOB_ADVECT value of a with b = psi, cubed)
//   JOB_SOURCE: out = -[Dx a Dys b - Dys a Dx b] / c       (stage 2a, a = phi,
//               b = mu, c = rho, or eta on the Stokes branch)
enum JobKind { JOB_ADVECT = 0, JOB_CUBE = 1, JOB_SOURCE = 2 };
struct Job {
  int kind, a, b, out;  // Buf indices
};
struct Jobs {
  Job j[3];
};

// Bracket jobs of a row: blockIdx.y picks the job, each computed on x pairs
// and passed through the forward row transform into a row spectrum.
template <typename T, int L, bool R1>
__global__ __launch_bounds__(RowCfg<L>::THREADS) LE_OCCUPANCY void k_bracket(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, Jobs jobs) {
  using C = RowCfg<L>;
  constexpr int NX = 2 * L;
  __shared__ c2<T> lds[C::G * L];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const Job job = jobs.j[bp.y];
  auto tw = to_global<const c2<double>>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const LaneRun<C::P> lr(t);
  const int j0 = bp.x * C::G + g;
  const bool ok = j0 < geo.ny;
  const int j = ok ? j0 : 0;
  const int jp = (j + 1 == geo.ny) ? 0 : j + 1;
  const int jm = (j == 0) ? geo.ny - 1 : j - 1;
  auto fa = bufp<const T>(R, job.a);
  auto a_c = fa + (size_t)j * NX;
  c2<T> v[C::E];
  // f of the advected phi (job.b = psi): the advection job's value, cubed
  const bool cube_half = job.kind == JOB_CUBE && geo.f_half;
  if (job.kind == JOB_CUBE && !cube_half) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) {
      const c2<T> p = load_pair<T, NX>(a_c, 2 * (t + q * C::P));
      v[q] = {p.x * p.x * p.x, p.y * p.y * p.y};
    }
  } else {
    const Stencil<T> st = make_stencil<T>(geo, sa[bp.z].s);
    auto fb = bufp<const T>(R, job.b);
    auto a_p = fa + (size_t)jp * NX;
    auto a_m = fa + (size_t)jm * NX;
    auto b_c = fb + (size_t)j * NX;
    auto b_p = fb + (size_t)jp * NX;
    auto b_m = fb + (size_t)jm * NX;
    const bool adv = job.kind != JOB_SOURCE;
    const T alpha = adv ? T(1) : T(0);
    const T beta = adv ? T(-geo.dt) : T(-1.0 / (geo.rho > 0.0 ? geo.rho : geo.eta));
#pragma unroll
    for (int q = 0; q < C::E; ++q) {
      const int x = 2 * (t + q * C::P);
      const Quad<T> A = load_quad<T, NX>(a_c, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
      const Quad<T> Ap = load_quad<T, NX>(a_p, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
      const Quad<T> Am = load_quad<T, NX>(a_m, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
      const Quad<T> B = load_quad<T, NX>(b_c, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
      const Quad<T> Bp = load_quad<T, NX>(b_p, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
      const Quad<T> Bm = load_quad<T, NX>(b_m, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
      T ax0, ax1, ay0, ay1, bx0, bx1, by0, by1;
      quad_dx(A, st.inv2dx, ax0, ax1);
      quad_dx(B, st.inv2dx, bx0, bx1);
      quad_dys<T, NX, R1>(Ap, Am, a_p, a_m, x, st, ay0, ay1);
      quad_dys<T, NX, R1>(Bp, Bm, b_p, b_m, x, st, by0, by1);
      v[q] = {alpha * A.a0 + beta * (by0 * ax0 - bx0 * ay0),
              alpha * A.a1 + beta * (by1 * ax1 - bx1 * ay1)};
      if (cube_half) v[q] = {v[q].x * v[q].x * v[q].x, v[q].y * v[q].y * v[q].y};
      LE_SCHED_FENCE();
    }
  }
  row_r2c<T, L, C::E>(v, lds + g * L, tw, t);
  auto out = bufp<c2<T>>(R, job.out);
  if (ok) store_row_spec<T, L, C::E>(out, geo.ny, j, v, t);
}

// Stage 1a (Eq. advective) as a stencil over row strips, no transform:
//   phi_h = phi - dt [Dx phi Dys psi - Dys phi Dx psi],  f = phi^3,
//   omega_h = omega - dt [Dx omega Dys psi - Dys omega Dx psi]  (inertial)
// into the real scratch fields B_TMP, B_R1, B_R2, for the forward row
// transforms that follow.
// Thread: one x pair of a row, walking `rows` consecutive rows; it keeps the
// quads of rows j-1, j, j+1 in registers and reads one new row per field and
// step (row j+2, requested a step ahead).
constexpr int strip_threads(int nx) { return nx / 2 < 256 ? nx / 2 : 256; }

template <typename T, int NX, int TPB_ = strip_threads(NX)>
struct StripLanes {
  static constexpr int TPB = TPB_;
  int x, xl, xr;  // pair position; halo positions of the lane's run
  bool edge_l, edge_r;
  __device__ __forceinline__ StripLanes(int bx) {
    const int p = bx * TPB + (int)threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int first = TPB >= 64 ? p - lane : bx * TPB;
    const int last = TPB >= 64 ? first + 63 : bx * TPB + TPB - 1;
    x = 2 * p;
    xl = 2 * first - 1;
    xr = 2 * last + 2;
    edge_l = p == first;
    edge_r = p == last;
  }
};

// Raw values of a row for a quad: the pair and the halo this lane may need.
template <typename T>
struct RawQuad {
  c2<T> p;
  T h;
};
template <typename T, int NX, int TPB>
__device__ __forceinline__ RawQuad<T> load_raw(gp<const T> __restrict__ row,
                                               const StripLanes<T, NX, TPB>& sl) {
  RawQuad<T> r;
  r.p = ldg<T>(reinterpret_cast<gp<const c2<T>>>(row + sl.x));
  r.h = row[(sl.edge_r ? sl.xr : sl.xl) & (NX - 1)];
  return r;
}
// Every lane of the wavefront must execute this (DPP).
template <typename T, int NX, int TPB>
__device__ __forceinline__ Quad<T> to_quad(const RawQuad<T>& r, const StripLanes<T, NX, TPB>& sl) {
  const T nl = dpp_mov<kDppWaveShr1>(r.p.y);
  const T nr = dpp_mov<kDppWaveShl1>(r.p.x);
  return {sl.edge_l ? r.h : nl, r.p.x, r.p.y, sl.edge_r ? r.h : nr};
}

template <typename T, int NX, bool R1>
__global__ __launch_bounds__(strip_threads(NX)) void k_adv_strip(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, int rows, int inertial) {
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const int ny = geo.ny;
  const StripLanes<T, NX> sl(bp.x);
  const int j0 = bp.y * rows;
  const int j1 = min(j0 + rows, ny);
  auto phi = bufp<const T>(R, B_PHI);
  auto psi = bufp<const T>(R, B_PS_R);
  auto om = bufp<const T>(R, B_OM_R);
  auto o_phi = bufp<T>(R, B_TMP);
  auto o_f = bufp<T>(R, B_R1);
  auto o_om = bufp<T>(R, B_R2);
  const Stencil<T> st = make_stencil<T>(geo, sa[bp.z].s);
  const T dt = T(geo.dt);
  const bool fh = geo.f_half != 0;
  const bool inr = inertial != 0;
  auto row = [&](gp<const T> f, int j) { return f + (size_t)(j < 0 ? j + ny : (j >= ny ? j - ny : j)) * NX; };
  Quad<T> Fm = to_quad(load_raw(row(phi, j0 - 1), sl), sl);
  Quad<T> Fc = to_quad(load_raw(row(phi, j0), sl), sl);
  Quad<T> Sm = to_quad(load_raw(row(psi, j0 - 1), sl), sl);
  Quad<T> Sc = to_quad(load_raw(row(psi, j0), sl), sl);
  Quad<T> Wm = Fm, Wc = Fc;
  if (inr) {
    Wm = to_quad(load_raw(row(om, j0 - 1), sl), sl);
    Wc = to_quad(load_raw(row(om, j0), sl), sl);
  }
  RawQuad<T> rF = load_raw(row(phi, j0 + 1), sl);
  RawQuad<T> rS = load_raw(row(psi, j0 + 1), sl);
  RawQuad<T> rW = inr ? load_raw(row(om, j0 + 1), sl) : rF;
  for (int j = j0; j < j1; ++j) {
    const Quad<T> Fp = to_quad(rF, sl);
    const Quad<T> Sp = to_quad(rS, sl);
    const Quad<T> Wp = inr ? to_quad(rW, sl) : Fp;
    if (j + 1 < j1) {  // row j+2, a step ahead
      rF = load_raw(row(phi, j + 2), sl);
      rS = load_raw(row(psi, j + 2), sl);
      if (inr) rW = load_raw(row(om, j + 2), sl);
    }
    T sx0, sx1, sy0, sy1, ax0, ax1, ay0, ay1;
    quad_dx(Sc, st.inv2dx, sx0, sx1);
    quad_dys<T, NX, R1>(Sp, Sm, row(psi, j + 1), row(psi, j - 1), sl.x, st, sy0, sy1);
    quad_dx(Fc, st.inv2dx, ax0, ax1);
    quad_dys<T, NX, R1>(Fp, Fm, row(phi, j + 1), row(phi, j - 1), sl.x, st, ay0, ay1);
    const size_t o = (size_t)j * NX + sl.x;
    const T h0 = Fc.a0 - dt * (ax0 * sy0 - ay0 * sx0), h1 = Fc.a1 - dt * (ax1 * sy1 - ay1 * sx1);
    const T c0 = fh ? h0 : Fc.a0, c1 = fh ? h1 : Fc.a1;
    stg<T>(reinterpret_cast<gp<c2<T>>>(o_phi + o), {h0, h1});
    stg<T>(reinterpret_cast<gp<c2<T>>>(o_f + o), {c0 * c0 * c0, c1 * c1 * c1});
    if (inr) {
      quad_dx(Wc, st.inv2dx, ax0, ax1);
      quad_dys<T, NX, R1>(Wp, Wm, row(om, j + 1), row(om, j - 1), sl.x, st, ay0, ay1);
      stg<T>(reinterpret_cast<gp<c2<T>>>(o_om + o),
             {Wc.a0 - dt * (ax0 * sy0 - ay0 * sx0), Wc.a1 - dt * (ax1 * sy1 - ay1 * sx1)});
    }
    Fm = Fc; Fc = Fp;
    Sm = Sc; Sc = Sp;
    Wm = Wc; Wc = Wp;
  }
}

// Stage 1a with third-order upwind differences of the advected fields (the
// alternative Appendix B keeps in a comment):
//   out = a - dt (vx Dx^up a + vy Dys^up a),  vx = Dys psi, vy = -Dx psi,
// with the central Eq. p1y differences of psi, and the upwind differences
// taken over offsets -2 .. 1 with weights (1, -6, 3, 2)/6 where the velocity
// component is positive, the mirror image where it is not.  The y samples of
// row j + k lie on the sheared line: (1 - |s|/c) a[j+k][i] + |s|/c
// a[j+k][i - sign(s) r k].  One thread per x pair of a row, every value read
// from memory (a switch for studies of the scheme, not a tuned path); real
// outputs phi_h, f, omega_h into B_TMP, B_R1, B_R2 for the forward row
// transforms that follow.
template <typename T, int NX>
__global__ __launch_bounds__(256) void k_adv_upwind(const Run* __restrict__ runs,
                                                    const StepArgs* __restrict__ sa,
                                                    int inertial) {
  const Run& R = runs[blockIdx.z];
  const Geo& geo = R.g;
  const int ny = geo.ny;
  const int j = blockIdx.y;
  const int x = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (x >= NX) return;
  auto phi = bufp<const T>(R, B_PHI);
  auto psi = bufp<const T>(R, B_PS_R);
  auto om = bufp<const T>(R, B_OM_R);
  const double s = sa[blockIdx.z].s;
  const T w = T(fabs(s) / geo.c), wm = T(1.0 - fabs(s) / geo.c);
  const int sg = s >= 0.0 ? 1 : -1;
  const int r = geo.r;
  const T i2dx = T(1.0 / (2.0 * geo.dx)), i2dy = T(1.0 / (2.0 * geo.dy));
  const T i6dx = T(1.0 / (6.0 * geo.dx)), i6dy = T(1.0 / (6.0 * geo.dy));
  const T dt = T(geo.dt);
  auto at = [&](gp<const T> f, int dj, int ii) {
    int jj = j + dj;
    jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
    return f[(size_t)jj * NX + (size_t)(ii & (NX - 1))];
  };
  // the sheared sample of row j + k at column i
  auto samp = [&](gp<const T> f, int k, int i) {
    return wm * at(f, k, i) + w * at(f, k, i - sg * r * k);
  };
  auto up = [&](T a_m2, T a_m1, T a_0, T a_p1, T a_p2, T v, T inv6) {
    return v > T(0) ? (a_m2 - T(6) * a_m1 + T(3) * a_0 + T(2) * a_p1) * inv6
                    : (-a_p2 + T(6) * a_p1 - T(3) * a_0 - T(2) * a_m1) * inv6;
  };
  const bool fh = geo.f_half != 0;
  T out_phi[2], out_f[2], out_om[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = x + e;
    const T vx = (wm * (at(psi, 1, i) - at(psi, -1, i)) +
                  w * (at(psi, 1, i - sg * r) - at(psi, -1, i + sg * r))) * i2dy;
    const T vy = -(at(psi, 0, i + 1) - at(psi, 0, i - 1)) * i2dx;
    auto adv = [&](gp<const T> f) {
      const T dx = up(at(f, 0, i - 2), at(f, 0, i - 1), at(f, 0, i), at(f, 0, i + 1),
                      at(f, 0, i + 2), vx, i6dx);
      const T dy = up(samp(f, -2, i), samp(f, -1, i), at(f, 0, i), samp(f, 1, i),
                      samp(f, 2, i), vy, i6dy);
      return at(f, 0, i) - dt * (vx * dx + vy * dy);
    };
    const T h = adv(phi);
    const T c = fh ? h : at(phi, 0, i);
    out_phi[e] = h;
    out_f[e] = c * c * c;
    out_om[e] = inertial ? adv(om) : T(0);
  }
  const size_t o = (size_t)j * NX + x;
  stg<T>(reinterpret_cast<gp<c2<T>>>(bufp<T>(R, B_TMP) + o), {out_phi[0], out_phi[1]});
  stg<T>(reinterpret_cast<gp<c2<T>>>(bufp<T>(R, B_R1) + o), {out_f[0], out_f[1]});
  if (inertial)
    stg<T>(reinterpret_cast<gp<c2<T>>>(bufp<T>(R, B_R2) + o), {out_om[0], out_om[1]});
}

// Stage 1a over row strips with the forward row transforms in the same
// kernel (no real rows written and read back).  The block owns whole rows:
// NX/(2 SEG) threads, thread t the SEG x pairs t + g NX/(2 SEG), each walked
// down the strip as in k_adv_strip.  The output rows go through LDS to four
// groups of threads (4 SEG values each) for the row transforms and are
// stored as row spectra: strips of four or more rows collect four rows and
// transform them in one round per field (phi_h, f and, with inertia,
// omega_h), group k taking row k; shorter strips transform every row in one
// round, group k taking field k (group 3 idles).  SEG = 2 halves the
// threads and doubles each one's registers.
constexpr bool strip_fft_ok(int nx) { return nx >= 256 && nx <= 2048; }
constexpr bool adv_strip_fft_ok(int nx) { return nx >= 256 && nx <= 1024; }

template <typename T, int NX, bool R1, int SEG>
__global__ __launch_bounds__(NX / 2 / SEG) void k_adv_strip_fft(const Run* __restrict__ runs,
                                                               const StepArgs* __restrict__ sa,
                                                               int rows, int inertial) {
  constexpr int L = NX / 2, TPB = L / SEG, EF = 4 * SEG, PF = L / EF;
  static_assert(TPB == 4 * PF && TPB >= 64, "four transform groups, whole wavefronts");
  __shared__ c2<T> buf[3 * 4 * L];  // [field][batch row][pair]
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const int ny = geo.ny;
  static_assert(SEG == 1 || SEG == 2, "one or two x pairs per thread");
  const StripLanes<T, NX, TPB> sl0(0), sl1(SEG - 1);
  const int j0 = bp.y * rows;
  const int j1 = min(j0 + rows, ny);
  auto phi = bufp<const T>(R, B_PHI);
  auto psi = bufp<const T>(R, B_PS_R);
  auto om = bufp<const T>(R, B_OM_R);
  auto tw = to_global<const c2<double>>(R.twx);
  const Stencil<T> st = make_stencil<T>(geo, sa[bp.z].s);
  const T dt = T(geo.dt);
  const bool fh = geo.f_half != 0;
  const bool inr = inertial != 0;
  const int grp = threadIdx.x / PF, tt = threadIdx.x % PF;
  const int nf = inr ? 3 : 2;
  // strips of four or more rows transform in batches of four rows, one
  // round per field; shorter strips transform every row in one round
  const bool batch = rows >= 4;
  auto row = [&](gp<const T> f, int j) {
    return f + (size_t)(j < 0 ? j + ny : (j >= ny ? j - ny : j)) * NX;
  };
  // rolling quads of rows j-1 (m), j (c) and the raw row j+1, per x segment
  Quad<T> Fm[SEG], Fc[SEG], Sm[SEG], Sc[SEG], Wm[SEG], Wc[SEG];
  RawQuad<T> rF[SEG], rS[SEG], rW[SEG];
#pragma unroll
  for (int g = 0; g < SEG; ++g) {
    const StripLanes<T, NX, TPB>& sl = g ? sl1 : sl0;
    Fm[g] = to_quad(load_raw(row(phi, j0 - 1), sl), sl);
    Fc[g] = to_quad(load_raw(row(phi, j0), sl), sl);
    Sm[g] = to_quad(load_raw(row(psi, j0 - 1), sl), sl);
    Sc[g] = to_quad(load_raw(row(psi, j0), sl), sl);
    Wm[g] = Fm[g];
    Wc[g] = Fc[g];
    if (inr) {
      Wm[g] = to_quad(load_raw(row(om, j0 - 1), sl), sl);
      Wc[g] = to_quad(load_raw(row(om, j0), sl), sl);
    }
    rF[g] = load_raw(row(phi, j0 + 1), sl);
    rS[g] = load_raw(row(psi, j0 + 1), sl);
    rW[g] = inr ? load_raw(row(om, j0 + 1), sl) : rF[g];
  }
  for (int j = j0; j < j1; ++j) {
    const int slot = batch ? (j - j0) & 3 : 0;
#pragma unroll
    for (int g = 0; g < SEG; ++g) {
      const StripLanes<T, NX, TPB>& sl = g ? sl1 : sl0;
      const Quad<T> Fp = to_quad(rF[g], sl);
      const Quad<T> Sp = to_quad(rS[g], sl);
      const Quad<T> Wp = inr ? to_quad(rW[g], sl) : Fp;
      if (j + 1 < j1) {  // row j+2, a step ahead
        rF[g] = load_raw(row(phi, j + 2), sl);
        rS[g] = load_raw(row(psi, j + 2), sl);
        if (inr) rW[g] = load_raw(row(om, j + 2), sl);
      }
      T sx0, sx1, sy0, sy1, ax0, ax1, ay0, ay1;
      quad_dx(Sc[g], st.inv2dx, sx0, sx1);
      quad_dys<T, NX, R1>(Sp, Sm[g], row(psi, j + 1), row(psi, j - 1), sl.x, st, sy0, sy1);
      quad_dx(Fc[g], st.inv2dx, ax0, ax1);
      quad_dys<T, NX, R1>(Fp, Fm[g], row(phi, j + 1), row(phi, j - 1), sl.x, st, ay0, ay1);
      const int pr = slot * L + sl.x / 2;
      const T h0 = Fc[g].a0 - dt * (ax0 * sy0 - ay0 * sx0);
      const T h1 = Fc[g].a1 - dt * (ax1 * sy1 - ay1 * sx1);
      const T c0 = fh ? h0 : Fc[g].a0, c1 = fh ? h1 : Fc[g].a1;
      buf[pr] = {h0, h1};
      buf[4 * L + pr] = {c0 * c0 * c0, c1 * c1 * c1};
      if (inr) {
        quad_dx(Wc[g], st.inv2dx, ax0, ax1);
        quad_dys<T, NX, R1>(Wp, Wm[g], row(om, j + 1), row(om, j - 1), sl.x, st, ay0, ay1);
        buf[8 * L + pr] = {Wc[g].a0 - dt * (ax0 * sy0 - ay0 * sx0),
                           Wc[g].a1 - dt * (ax1 * sy1 - ay1 * sx1)};
      }
      Fm[g] = Fc[g]; Fc[g] = Fp;
      Sm[g] = Sc[g]; Sc[g] = Sp;
      Wm[g] = Wc[g]; Wc[g] = Wp;
    }
    if (!batch) {  // one round per row: group k transforms field k (group 3 idles)
      c2<T>* area = buf + (grp < 3 ? grp * 4 : 1) * L;
      __syncthreads();
      c2<T> v[EF];
#pragma unroll
      for (int q = 0; q < EF; ++q) v[q] = area[tt + q * PF];
      __syncthreads();
      row_r2c<T, L, EF>(v, area, tw, tt);
      if (grp < nf) {
        auto out = bufp<c2<T>>(R, grp == 0 ? B_PHIH : (grp == 1 ? B_FH : B_OMH));
        store_row_spec<T, L, EF>(out, ny, j, v, tt);
      }
      __syncthreads();
    } else if (slot == 3 || j + 1 == j1) {  // a batch of up to four rows is complete
      for (int f = 0; f < nf; ++f) {
        c2<T>* area = buf + (f * 4 + grp) * L;
        __syncthreads();
        c2<T> v[EF];
#pragma unroll
        for (int q = 0; q < EF; ++q) v[q] = area[tt + q * PF];
        __syncthreads();
        row_r2c<T, L, EF>(v, area, tw, tt);
        if (grp <= slot) {
          auto out = bufp<c2<T>>(R, f == 0 ? B_PHIH : (f == 1 ? B_FH : B_OMH));
          store_row_spec<T, L, EF>(out, ny, j - slot + grp, v, tt);
        }
      }
      __syncthreads();
    }
  }
}

// Stage 1a for long rows in batches of NR rows (4 or 2).  The block owns
// whole rows (NR transform groups of L/EF threads, each thread L/(NR L/EF)
// x pairs) and walks its strip NR rows at a time.  For each batch and
// output field (phi_h, f and, with inertia, omega_h) it walks the NR rows,
// one x segment of pairs at a time, with a rolling window of input quads
// (rows j-1, j, j+1), writes the NR output rows to LDS, transforms them
// (group g row g; the complex transforms stay in LDS) and stores the half
// spectra tile by tile, formed as they are stored (r2c_mode), so that each
// store writes the NR rows' kTW modes of a tile as one run.
// FP64 (kAdvSplit): one output field per block, the grid's x; the fields of
// a batch are consecutive blocks (one XCD, the same time), so the input
// rows they share, and the halo rows of the neighbouring batch, come from
// the L2.  A wave's loads wait for its earlier stores too (one counter for
// both): a block that went on to the next field would wait for the last
// field's stores at its first load, whereas the next block on the CU
// starts while they drain (one block per CU: LDS).  FP32 (two blocks per
// CU) computes the fields one after another in one block, which measured
// faster there.
// LDS: NR rows of L + 1 complex values, so the form fits the 2048-point rows
// of nx = 4096 in FP64 (NR = 2: two blocks per CU).
constexpr bool adv_batch_ok(int nx) { return nx >= 512 && nx <= 4096; }

template <typename T, int NX, int NR, int EF_>
struct AdvBatch {
  static constexpr int L = NX / 2, EF = EF_, PF = L / EF, TPB = NR * PF, SEG = L / TPB;
  static_assert(TPB * SEG == L && TPB >= 64, "whole wavefronts");
};
template <typename T>
constexpr bool kAdvSplit = sizeof(T) == 8;

template <typename T, int NX, bool R1, int NR, int EF_>
__global__ __launch_bounds__((AdvBatch<T, NX, NR, EF_>::TPB)) void k_adv_batch(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, int rows, int inertial) {
  using C = AdvBatch<T, NX, NR, EF_>;
  constexpr int L = C::L, EF = C::EF, PF = C::PF, TPB = C::TPB;
  constexpr int LS = staged_stride<T, NR>(L);
  __shared__ c2<T> buf[NR * LS];
  __shared__ c2<double> wtab[TwTab<L>::N];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const int ny = geo.ny;
  const int jb0 = bp.y * rows;
  const int jb1 = min(jb0 + rows, ny);
  auto phi = bufp<const T>(R, B_PHI);
  auto psi = bufp<const T>(R, B_PS_R);
  auto om = bufp<const T>(R, B_OM_R);
  auto tw = to_global<const c2<double>>(R.twx);
  tw_tab_fill<L, TPB>(wtab, tw);  // read after the loop's first barrier
  const Stencil<T> st = make_stencil<T>(geo, sa[bp.z].s);
  const T dt = T(geo.dt);
  const bool fh = geo.f_half != 0;
  // fields [f0, f1): 0: phi_h from (phi, psi); 1: f from phi (phi_h when
  // f_half); 2: omega_h from (omega, psi)
  const int f0 = kAdvSplit<T> ? bp.x : 0;
  const int f1 = kAdvSplit<T> ? bp.x + 1 : (inertial ? 3 : 2);
  const int grp = threadIdx.x / PF, tt = threadIdx.x % PF;
  auto row = [&](gp<const T> a, int j) {
    return a + (size_t)(j < 0 ? j + ny : (j >= ny ? j - ny : j)) * NX;
  };
  for (int j0 = jb0; j0 < jb1; j0 += NR) {
    for (int f = f0; f < f1; ++f) {
      auto fa = (f == 2) ? om : phi;
      const bool cube_plain = f == 1 && !fh;
      auto out = bufp<c2<T>>(R, f == 0 ? B_PHIH : (f == 1 ? B_FH : B_OMH));
      __syncthreads();  // the previous round's LDS reads are done
      if (cube_plain) {
#pragma unroll 1
        for (int g = 0; g < C::SEG; ++g) {
          const StripLanes<T, NX, TPB> sl(g);
          for (int r = 0; r < NR; ++r) {
            const c2<T> pr = ldg<T>(reinterpret_cast<gp<const c2<T>>>(row(phi, j0 + r) + sl.x));
            buf[r * L + sl.x / 2] = {pr.x * pr.x * pr.x, pr.y * pr.y * pr.y};
          }
        }
      }
      // every input row of a segment requested at once (rows j0-1 .. j0+NR);
      // PREF: the next segment's before this segment's stencil, their latency
      // hidden behind it (FP64 square cells at nx = 4096, where the registers
      // allow it at the occupancy that LDS sets; elsewhere it spilled or
      // halved the occupancy)
      constexpr bool PREF = sizeof(T) == 8 && NX >= 4096 && R1;
      auto load_seg = [&](int g, RawQuad<T>* a, RawQuad<T>* b) {
        const StripLanes<T, NX, TPB> sl(g);
#pragma unroll
        for (int k = 0; k < NR + 2; ++k) {
          a[k] = load_raw(row(fa, j0 - 1 + k), sl);
          b[k] = load_raw(row(psi, j0 - 1 + k), sl);
        }
      };
      auto stencil_seg = [&](int g, const RawQuad<T>* a, const RawQuad<T>* b) {
        const StripLanes<T, NX, TPB> sl(g);
        Quad<T> Am = to_quad(a[0], sl), Ac = to_quad(a[1], sl);
        Quad<T> Bm = to_quad(b[0], sl), Bc = to_quad(b[1], sl);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int j = j0 + r;
          const Quad<T> Ap = to_quad(a[r + 2], sl);
          const Quad<T> Bp = to_quad(b[r + 2], sl);
          T bx0, bx1, by0, by1, ax0, ax1, ay0, ay1;
          quad_dx(Bc, st.inv2dx, bx0, bx1);
          quad_dys<T, NX, R1>(Bp, Bm, row(psi, j + 1), row(psi, j - 1), sl.x, st, by0, by1);
          quad_dx(Ac, st.inv2dx, ax0, ax1);
          quad_dys<T, NX, R1>(Ap, Am, row(fa, j + 1), row(fa, j - 1), sl.x, st, ay0, ay1);
          T h0 = Ac.a0 - dt * (ax0 * by0 - ay0 * bx0);
          T h1 = Ac.a1 - dt * (ax1 * by1 - ay1 * bx1);
          if (f == 1) {
            h0 = h0 * h0 * h0;
            h1 = h1 * h1 * h1;
          }
          buf[r * L + sl.x / 2] = {h0, h1};
          Am = Ac; Ac = Ap;
          Bm = Bc; Bc = Bp;
        }
      };
      if (!cube_plain) {
        if constexpr (PREF) {
          RawQuad<T> ra[NR + 2], rb[NR + 2];
          load_seg(0, ra, rb);
#pragma unroll
          for (int g = 0; g < C::SEG; ++g) {
            RawQuad<T> na[NR + 2], nb[NR + 2];
            if (g + 1 < C::SEG) load_seg(g + 1, na, nb);
            stencil_seg(g, ra, rb);
            if (g + 1 < C::SEG) {
#pragma unroll
              for (int k = 0; k < NR + 2; ++k) {
                ra[k] = na[k];
                rb[k] = nb[k];
              }
            }
          }
        } else {
#pragma unroll 1
          for (int g = 0; g < C::SEG; ++g) {
            RawQuad<T> ra[NR + 2], rb[NR + 2];
            load_seg(g, ra, rb);
            stencil_seg(g, ra, rb);
          }
        }
      }
      __syncthreads();
      c2<T> v[EF];
#pragma unroll
      for (int q = 0; q < EF; ++q) v[q] = buf[grp * L + tt + q * PF];
      __syncthreads();
      row_r2c_z<T, L, EF>(v, buf + grp * LS, tw, tt);
      __syncthreads();
      const int nr = min(NR, jb1 - j0);
      tile_runs<L, TPB, NR>(nr, [&](int r, int m) {
        stg<T>(out + spec_index(ny, j0 + r, m), r2c_mode<T, L>(buf + r * LS, wtab, m));
      });
    }
  }
}

// Stage 2a as a stencil over row strips (square cells, r = 1), no transform:
//   mu = B phi^3 - A phi - kappa [(1+s^2) Dxx + Dyy - 2 s Dxy] phi,
//   g = -[Dx phi Dys mu - Dys phi Dx mu] / c   (c = rho, or eta for Stokes)
// into the real scratch field B_TMP.
// mu never leaves the registers: a thread walks its strip keeping the phi
// quads of rows j-1 .. j+2 and the mu quads of rows j-1 .. j+1; mu at x-1 /
// x+2 for the first / last lane of a run is computed by that lane from one
// more phi value per row (x-2 / x+3).
template <typename T>
struct PhiRow {
  Quad<T> q;
  T e;  // phi at x-2 (first lane of a run) or x+3 (last lane)
};
template <typename T>
struct RawPhi {
  RawQuad<T> r;
  T e;
};
template <typename T, int NX, int TPB>
__device__ __forceinline__ RawPhi<T> load_phi(gp<const T> __restrict__ row,
                                              const StripLanes<T, NX, TPB>& sl) {
  RawPhi<T> o;
  o.r = load_raw<T, NX>(row, sl);
  o.e = row[(sl.edge_r ? sl.xr + 1 : sl.xl - 1) & (NX - 1)];
  return o;
}
template <typename T, int NX, int TPB>
__device__ __forceinline__ PhiRow<T> to_phirow(const RawPhi<T>& r, const StripLanes<T, NX, TPB>& sl) {
  return {to_quad<T, NX>(r.r, sl), r.e};
}

template <typename T>
struct MuCoef {
  T cxx, cyy, cxy, A, B, kap;
};
// mu at one point from the 3x3 phi neighbourhood (rows d, c, u = j-1, j, j+1;
// columns w, m, e = x-1, x, x+1).
template <typename T>
__device__ __forceinline__ T mu_at(const MuCoef<T>& k, T dw, T dm, T de, T cw, T cm, T ce, T uw,
                                   T um, T ue) {
  const T two = T(2);
  const T dxx = ce - two * cm + cw;
  const T dyy = um - two * cm + dm;
  const T dxy = ue - de - uw + dw;
  return k.B * cm * cm * cm - k.A * cm - k.kap * (k.cxx * dxx + k.cyy * dyy + k.cxy * dxy);
}
// mu quad of row j from the phi rows j-1 (d), j (c), j+1 (u).  Every lane of
// the wavefront must execute this (DPP).
template <typename T, int NX, int TPB>
__device__ __forceinline__ Quad<T> mu_quad(const MuCoef<T>& k, const PhiRow<T>& d,
                                           const PhiRow<T>& c, const PhiRow<T>& u,
                                           const StripLanes<T, NX, TPB>& sl) {
  const T m0 = mu_at(k, d.q.l, d.q.a0, d.q.a1, c.q.l, c.q.a0, c.q.a1, u.q.l, u.q.a0, u.q.a1);
  const T m1 = mu_at(k, d.q.a0, d.q.a1, d.q.r, c.q.a0, c.q.a1, c.q.r, u.q.a0, u.q.a1, u.q.r);
  // halo mu: at x-1 (neighbourhood x-2 .. x) or at x+2 (x+1 .. x+3)
  const T mh = sl.edge_r
                   ? mu_at(k, d.q.a1, d.q.r, d.e, c.q.a1, c.q.r, c.e, u.q.a1, u.q.r, u.e)
                   : mu_at(k, d.e, d.q.l, d.q.a0, c.e, c.q.l, c.q.a0, u.e, u.q.l, u.q.a0);
  const T nl = dpp_mov<kDppWaveShr1>(m1);
  const T nr = dpp_mov<kDppWaveShl1>(m0);
  return {sl.edge_l ? mh : nl, m0, m1, sl.edge_r ? mh : nr};
}

template <typename T, int NX>
__global__ __launch_bounds__(strip_threads(NX)) void k_mug_strip(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, int rows) {
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const int ny = geo.ny;
  const StripLanes<T, NX> sl(bp.x);
  const int j0 = bp.y * rows;
  const int j1 = min(j0 + rows, ny);
  auto phi = bufp<const T>(R, B_PHI);
  auto o_g = bufp<T>(R, B_TMP);
  const double s = sa[bp.z].s;
  const MuCoef<T> k = {T((1.0 + s * s) / (geo.dx * geo.dx)), T(1.0 / (geo.dy * geo.dy)),
                       T(-2.0 * s / (4.0 * geo.dx * geo.dy)), T(geo.A), T(geo.B), T(geo.kappa)};
  const Stencil<T> st = make_stencil<T>(geo, s);
  const T neg_inv = T(-1.0 / (geo.rho > 0.0 ? geo.rho : geo.eta));
  auto row = [&](int j) {  // j in [-2, ny + 4]: one wrap at most, no division
    return phi + (size_t)(j < 0 ? j + ny : (j >= ny ? j - ny : j)) * NX;
  };
  PhiRow<T> F0 = to_phirow(load_phi(row(j0 - 2), sl), sl);  // rows j-2 .. j+1 at j = j0
  PhiRow<T> F1 = to_phirow(load_phi(row(j0 - 1), sl), sl);
  PhiRow<T> F2 = to_phirow(load_phi(row(j0), sl), sl);
  PhiRow<T> F3 = to_phirow(load_phi(row(j0 + 1), sl), sl);
  Quad<T> Mm = mu_quad(k, F0, F1, F2, sl);  // mu rows j-1, j
  Quad<T> Mc = mu_quad(k, F1, F2, F3, sl);
  RawPhi<T> rn = load_phi(row(j0 + 2), sl);
  for (int j = j0; j < j1; ++j) {
    // window: F1 = phi(j-1), F2 = phi(j), F3 = phi(j+1); rn = phi(j+2)
    const PhiRow<T> F4 = to_phirow(rn, sl);
    if (j + 1 < j1) rn = load_phi(row(j + 3), sl);
    const Quad<T> Mp = mu_quad(k, F2, F3, F4, sl);  // mu(j+1)
    T px0, px1, py0, py1, mx0, mx1, my0, my1;
    quad_dx(F2.q, st.inv2dx, px0, px1);
    quad_dys<T, NX, true>(F3.q, F1.q, row(j + 1), row(j - 1), sl.x, st, py0, py1);
    quad_dx(Mc, st.inv2dx, mx0, mx1);
    quad_dys<T, NX, true>(Mp, Mm, row(j + 1), row(j - 1), sl.x, st, my0, my1);
    const size_t o = (size_t)j * NX + sl.x;
    stg<T>(reinterpret_cast<gp<c2<T>>>(o_g + o),
           {neg_inv * (px0 * my0 - py0 * mx0), neg_inv * (px1 * my1 - py1 * mx1)});
    F1 = F2; F2 = F3; F3 = F4;
    Mm = Mc; Mc = Mp;
  }
}

// Stage 2a over row strips with the forward row transform of g in the same
// kernel (square cells, as k_mug_strip).  The block owns whole rows: NX/2
// threads, one x pair each, walking the strip as k_mug_strip does.  The g
// rows collect in LDS four at a time; each batch goes through the row
// transform by four groups of NX/8 threads (4 values each), group k taking
// row k of the batch, and is stored as row spectra of B_GH.
template <typename T, int NX>
__global__ __launch_bounds__(NX / 2) void k_mug_strip_fft(const Run* __restrict__ runs,
                                                         const StepArgs* __restrict__ sa,
                                                         int rows) {
  constexpr int L = NX / 2, TPB = L, EF = 4, PF = L / EF;
  static_assert(TPB == 4 * PF && TPB >= 64, "four transform groups, whole wavefronts");
  __shared__ c2<T> buf[4 * L];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const int ny = geo.ny;
  const StripLanes<T, NX, TPB> sl(0);
  const int j0 = bp.y * rows;
  const int j1 = min(j0 + rows, ny);
  auto phi = bufp<const T>(R, B_PHI);
  auto out = bufp<c2<T>>(R, B_GH);
  auto tw = to_global<const c2<double>>(R.twx);
  const double s = sa[bp.z].s;
  const MuCoef<T> k = {T((1.0 + s * s) / (geo.dx * geo.dx)), T(1.0 / (geo.dy * geo.dy)),
                       T(-2.0 * s / (4.0 * geo.dx * geo.dy)), T(geo.A), T(geo.B), T(geo.kappa)};
  const Stencil<T> st = make_stencil<T>(geo, s);
  const T neg_inv = T(-1.0 / (geo.rho > 0.0 ? geo.rho : geo.eta));
  const int grp = threadIdx.x / PF, tt = threadIdx.x % PF;
  auto row = [&](int j) {  // j in [-2, ny + 4]: one wrap at most, no division
    return phi + (size_t)(j < 0 ? j + ny : (j >= ny ? j - ny : j)) * NX;
  };
  PhiRow<T> F0 = to_phirow(load_phi(row(j0 - 2), sl), sl);  // rows j-2 .. j+1 at j = j0
  PhiRow<T> F1 = to_phirow(load_phi(row(j0 - 1), sl), sl);
  PhiRow<T> F2 = to_phirow(load_phi(row(j0), sl), sl);
  PhiRow<T> F3 = to_phirow(load_phi(row(j0 + 1), sl), sl);
  Quad<T> Mm = mu_quad(k, F0, F1, F2, sl);  // mu rows j-1, j
  Quad<T> Mc = mu_quad(k, F1, F2, F3, sl);
  RawPhi<T> rn = load_phi(row(j0 + 2), sl);
  for (int j = j0; j < j1; ++j) {
    const PhiRow<T> F4 = to_phirow(rn, sl);
    if (j + 1 < j1) rn = load_phi(row(j + 3), sl);
    const Quad<T> Mp = mu_quad(k, F2, F3, F4, sl);  // mu(j+1)
    T px0, px1, py0, py1, mx0, mx1, my0, my1;
    quad_dx(F2.q, st.inv2dx, px0, px1);
    quad_dys<T, NX, true>(F3.q, F1.q, row(j + 1), row(j - 1), sl.x, st, py0, py1);
    quad_dx(Mc, st.inv2dx, mx0, mx1);
    quad_dys<T, NX, true>(Mp, Mm, row(j + 1), row(j - 1), sl.x, st, my0, my1);
    const int slot = (j - j0) & 3;
    buf[slot * L + sl.x / 2] = {neg_inv * (px0 * my0 - py0 * mx0),
                                neg_inv * (px1 * my1 - py1 * mx1)};
    F1 = F2; F2 = F3; F3 = F4;
    Mm = Mc; Mc = Mp;
    if (slot == 3 || j + 1 == j1) {  // a batch of up to four rows is complete
      __syncthreads();
      c2<T> v[EF];
#pragma unroll
      for (int q = 0; q < EF; ++q) v[q] = buf[grp * L + tt + q * PF];
      __syncthreads();
      row_r2c<T, L, EF>(v, buf + grp * L, tw, tt);
      if (grp <= slot) store_row_spec<T, L, EF>(out, ny, j - slot + grp, v, tt);
      __syncthreads();
    }
  }
}

// Stage 2a for long rows (square cells) in batches of NR rows, with the
// forward row transform of g in the same kernel: the batched layout of
// k_adv_batch (NR transform groups of L/EF threads; the block walks its strip
// NR rows at a time, each batch one x segment of pairs after another).  For
// a segment a thread requests its x pair of the phi rows j0-2 .. j0+NR+1 at
// once, forms mu on rows j0-1 .. j0+NR in registers (the k_mug_strip
// neighbourhoods) and g on the NR rows into LDS; the NR rows are then
// transformed (group g row g) and stored tile by tile as k_adv_batch stores
// them (B_GH).  The phi halo rows are read again by the neighbouring batch
// (from the L2); nothing goes through the real scratch.
template <typename T, int NX, int NR, int EF_>
__global__ __launch_bounds__((AdvBatch<T, NX, NR, EF_>::TPB)) void k_mug_batch(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, int rows) {
  using C = AdvBatch<T, NX, NR, EF_>;
  constexpr int L = C::L, EF = C::EF, PF = C::PF, TPB = C::TPB;
  constexpr int LS = staged_stride<T, NR>(L);
  __shared__ c2<T> buf[NR * LS];
  __shared__ c2<double> wtab[TwTab<L>::N];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const int ny = geo.ny;
  const int jb0 = bp.y * rows;
  const int jb1 = min(jb0 + rows, ny);
  auto phi = bufp<const T>(R, B_PHI);
  auto out = bufp<c2<T>>(R, B_GH);
  auto tw = to_global<const c2<double>>(R.twx);
  tw_tab_fill<L, TPB>(wtab, tw);  // read after the loop's first barrier
  const double s = sa[bp.z].s;
  const MuCoef<T> k = {T((1.0 + s * s) / (geo.dx * geo.dx)), T(1.0 / (geo.dy * geo.dy)),
                       T(-2.0 * s / (4.0 * geo.dx * geo.dy)), T(geo.A), T(geo.B), T(geo.kappa)};
  const Stencil<T> st = make_stencil<T>(geo, s);
  const T neg_inv = T(-1.0 / (geo.rho > 0.0 ? geo.rho : geo.eta));
  const int grp = threadIdx.x / PF, tt = threadIdx.x % PF;
  auto row = [&](int j) {  // j in [-2, ny + 4]: one wrap at most, no division
    return phi + (size_t)(j < 0 ? j + ny : (j >= ny ? j - ny : j)) * NX;
  };
  for (int j0 = jb0; j0 < jb1; j0 += NR) {
    __syncthreads();  // the previous batch's LDS reads are done
#pragma unroll 1
    for (int g = 0; g < C::SEG; ++g) {
      const StripLanes<T, NX, TPB> sl(g);
      RawPhi<T> rp[NR + 4];  // rows j0-2 .. j0+NR+1, requested at once
#pragma unroll
      for (int kk = 0; kk < NR + 4; ++kk) rp[kk] = load_phi(row(j0 - 2 + kk), sl);
      PhiRow<T> F1 = to_phirow(rp[1], sl), F2 = to_phirow(rp[2], sl), F3 = to_phirow(rp[3], sl);
      Quad<T> Mm = mu_quad(k, to_phirow(rp[0], sl), F1, F2, sl);  // mu rows j0-1, j0
      Quad<T> Mc = mu_quad(k, F1, F2, F3, sl);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        // window: F1 = phi(j-1), F2 = phi(j), F3 = phi(j+1), j = j0 + r
        const int j = j0 + r;
        const PhiRow<T> F4 = to_phirow(rp[r + 4], sl);
        const Quad<T> Mp = mu_quad(k, F2, F3, F4, sl);  // mu(j+1)
        T px0, px1, py0, py1, mx0, mx1, my0, my1;
        quad_dx(F2.q, st.inv2dx, px0, px1);
        quad_dys<T, NX, true>(F3.q, F1.q, row(j + 1), row(j - 1), sl.x, st, py0, py1);
        quad_dx(Mc, st.inv2dx, mx0, mx1);
        quad_dys<T, NX, true>(Mp, Mm, row(j + 1), row(j - 1), sl.x, st, my0, my1);
        buf[r * L + sl.x / 2] = {neg_inv * (px0 * my0 - py0 * mx0),
                                 neg_inv * (px1 * my1 - py1 * mx1)};
        F1 = F2; F2 = F3; F3 = F4;
        Mm = Mc; Mc = Mp;
      }
    }
    __syncthreads();
    c2<T> v[EF];
#pragma unroll
    for (int q = 0; q < EF; ++q) v[q] = buf[grp * L + tt + q * PF];
    __syncthreads();
    row_r2c_z<T, L, EF>(v, buf + grp * LS, tw, tt);
    __syncthreads();
    const int nr = min(NR, jb1 - j0);
    tile_runs<L, TPB, NR>(nr, [&](int r, int m) {
      stg<T>(out + spec_index(ny, j0 + r, m), r2c_mode<T, L>(buf + r * LS, wtab, m));
    });
  }
}

// Chemical potential (Eq. mu, stage 2a) on x pairs into a real field:
//   mu = B phi^3 - A phi - kappa [(1+s^2) Dxx + Dyy - 2 s Dxy] phi.
template <typename T, int L>
__global__ __launch_bounds__(RowCfg<L>::THREADS) LE_OCCUPANCY void k_mu(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, int bin, int bout) {
  using C = RowCfg<L>;
  constexpr int NX = 2 * L;
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const LaneRun<C::P> lr(t);
  const int j0 = bp.x * C::G + g;
  const bool ok = j0 < geo.ny;
  const int j = ok ? j0 : 0;
  const int jp = (j + 1 == geo.ny) ? 0 : j + 1;
  const int jm = (j == 0) ? geo.ny - 1 : j - 1;
  auto phi = bufp<const T>(R, bin);
  auto mu = bufp<T>(R, bout) + (size_t)j * NX;
  const double s = sa[bp.z].s;
  const T cxx = T((1.0 + s * s) / (geo.dx * geo.dx));
  const T cyy = T(1.0 / (geo.dy * geo.dy));
  const T cxy = T(-2.0 * s / (4.0 * geo.dx * geo.dy));
  const T A = T(geo.A), B = T(geo.B), kap = T(geo.kappa);
  const T two = T(2);
  auto p_c = phi + (size_t)j * NX;
  auto p_p = phi + (size_t)jp * NX;
  auto p_m = phi + (size_t)jm * NX;
#pragma unroll
  for (int q = 0; q < C::E; ++q) {
    const int x = 2 * (t + q * C::P);
    const Quad<T> c = load_quad<T, NX>(p_c, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
    const Quad<T> u = load_quad<T, NX>(p_p, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
    const Quad<T> d = load_quad<T, NX>(p_m, x, lr.xl(q), lr.xr(q), lr.edge_l, lr.edge_r);
    const T dxx0 = c.a1 - two * c.a0 + c.l, dxx1 = c.r - two * c.a1 + c.a0;
    const T dyy0 = u.a0 - two * c.a0 + d.a0, dyy1 = u.a1 - two * c.a1 + d.a1;
    const T dxy0 = u.a1 - d.a1 - u.l + d.l, dxy1 = u.r - d.r - u.a0 + d.a0;
    const T m0 = B * c.a0 * c.a0 * c.a0 - A * c.a0 - kap * (cxx * dxx0 + cyy * dyy0 + cxy * dxy0);
    const T m1 = B * c.a1 * c.a1 * c.a1 - A * c.a1 - kap * (cxx * dxx1 + cyy * dyy1 + cxy * dxy1);
    if (ok) stg<T>(reinterpret_cast<gp<c2<T>>>(mu + x), {m0, m1});
  }
}

// Strain-wrap remap of a row spectrum: row j shifted by sh_j = (dkr * j) mod nx,
// X[j][m] *= exp(-2 pi i m sh_j / nx).  e runs over the tiled storage.
template <typename T>
__global__ void k_remap_spec(const Run* __restrict__ run, int b, int dkr) {
  const int nx = run->g.nx, ny = run->g.ny;
  auto X = bufp<c2<T>>(*run, b);
  auto twx = to_global<const c2<double>>(run->twx);
  const int S = nx / 2 + 1;
  const size_t total = spec_elems(nx, ny);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t tile = e / ((size_t)ny * kTW), rem = e % ((size_t)ny * kTW);
    const int j = (int)(rem / kTW), m = (int)(tile * kTW + rem % kTW);
    if (m >= S) continue;  // pad column
    const long long sh = (((long long)dkr * j) % nx + nx) % nx;
    const int idx = (int)(((long long)m * sh) % nx);
    const c2<double> w = ldg<double>(twx + idx);
    stg<T>(X + e, cmul(ldg<T>(X + e), c2<T>{static_cast<T>(w.x), static_cast<T>(w.y)}));
  }
}

// Strain-wrap remap of a real field: out[j][i] = in[j][(i - dkr j) mod nx].
template <typename T>
__global__ void k_remap_real(const Run* __restrict__ run, int bin, int bout, int dkr) {
  const int nx = run->g.nx, ny = run->g.ny;
  auto in = bufp<const T>(*run, bin);
  auto out = bufp<T>(*run, bout);
  const size_t total = (size_t)ny * nx;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / nx), i = (int)(e % nx);
    const long long sh = (((long long)dkr * j) % nx + nx) % nx;
    out[e] = in[(size_t)j * nx + (size_t)((i - sh + nx) % nx)];
  }
}

// f x f block means of a real field into out[(ny/f)][(nx/f)] (FP64).
template <typename T>
__global__ void k_restrict(const Run* __restrict__ run, int bin, int f, double* __restrict__ out) {
  const int nx = run->g.nx, ny = run->g.ny, cx = nx / f, cy = ny / f;
  auto in = bufp<const T>(*run, bin);
  const double inv = 1.0 / ((double)f * f);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < cx * cy; e += gridDim.x * blockDim.x) {
    const int J = e / cx, I = e % cx;
    double acc = 0.0;
    for (int a = 0; a < f; ++a)
      for (int b = 0; b < f; ++b) acc += (double)in[(size_t)(J * f + a) * nx + I * f + b];
    out[e] = acc * inv;
  }
}

// Plain copy of a real field (bin -> bout).
template <typename T>
__global__ void k_copy_real(const Run* __restrict__ run, int bin, int bout) {
  const size_t total = (size_t)run->g.ny * run->g.nx;
  auto in = bufp<const T>(*run, bin);
  auto out = bufp<T>(*run, bout);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    out[e] = in[e];
}

// ---------------------------------------------------------------- column kernels

// Column transform, per-mode update, inverse column transform.
//  COL_CH      (phi_h, f) -> phi'         stage 1b (Cahn-Hilliard)
//  COL_FLOW    (omega_h, g) -> (omega', psi')   stages 2b and 3
//  COL_STOKES  g -> psi'                  zero-Reynolds solve
//  COL_POISSON omega -> psi               set-up: psi from omega
template <typename T, int L, int MODE, int VAR, bool BANDED = false>
__global__ __launch_bounds__((ColCfg<T, L, VAR>::THREADS)) LE_OCCUPANCY_COL void k_column(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, int bin0, int bin1,
    int bout0, int bout1) {
  using C = ColCfg<T, L, VAR>;
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  auto in0 = bufp<const c2<T>>(R, bin0);
  auto in1 = bufp<const c2<T>>(R, bin1);
  auto out0 = bufp<c2<T>>(R, bout0);
  auto out1 = bufp<c2<T>>(R, bout1);
  auto tw = to_global<const c2<double>>(R.twy);
  constexpr int NIN = (MODE == COL_CH || MODE == COL_FLOW) ? 2 : 1;
  constexpr int NOUT = (MODE == COL_FLOW) ? 2 : 1;
  // Both fields' transforms side by side (one barrier per pass for the two)
  // where LDS holds two areas: in FP32 and for columns up to 512 values (in
  // FP64 at 2048 and 4096 the doubled LDS halves the blocks per CU and the
  // pass runs slower).
  constexpr bool DUAL = LE_COL_DUAL && NIN == 2 && (sizeof(T) == 4 || L <= 512) &&
                        2L * C::CW * L * (long)sizeof(c2<T>) <= 160L * 1024;
  __shared__ c2<T> lds[(DUAL ? 2 : 1) * C::CW * L];
  c2<T>* const lds1 = lds + (DUAL ? C::CW * L : 0);
  // the flow pass's second inverse transform follows the first output's
  // stores: its twiddles come from an LDS copy (fft_group TWL)
  constexpr bool LTW = MODE == COL_FLOW && !DUAL && L > C::E;
  __shared__ c2<double> ltw[LTW ? L / C::E : 1];
  const int S = geo.nx / 2 + 1;
  const int c = threadIdx.x % C::CW, t = threadIdx.x / C::CW;
  const int m0 = bp.x * C::CW + c;
  const bool ok = m0 < S;
  const int m = ok ? m0 : 0;
  // column m of the tiled spectra: element n at col + n kTW
  const size_t col = spec_index(L, 0, m);
  if constexpr (LTW) fft_ltw_fill<L, C::E, C::THREADS>(ltw, tw);  // read after later barriers
  c2<T> v0[C::E], v1[C::E];
  // PRE: the second field's loads are issued before the first field's
  // transform, so their latency hides behind it.  Only where the registers
  // already limit the shape to two waves per SIMD (FP64, 16 values per
  // thread) and the CH pass (the flow pass would spill): elsewhere the
  // extra registers cost occupancy (measured slower at 1024^2 and 2048^2).
  constexpr bool PRE = NIN == 2 && !DUAL && MODE == COL_CH && C::E == 16 && sizeof(T) == 8;
#pragma unroll
  for (int q = 0; q < C::E; ++q) v0[q] = ldg<T>(in0 + col + (size_t)(t + q * C::P) * kTW);
  if constexpr (DUAL || PRE) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) v1[q] = ldg<T>(in1 + col + (size_t)(t + q * C::P) * kTW);
  }
  if constexpr (DUAL) {
    fft_group2<T, L, C::E, -1>(v0, v1, lds + c, lds1 + c, C::CW, tw, t);
  } else {
    fft_group<T, L, C::E, -1>(v0, lds + c, C::CW, tw, t);
  }
  if constexpr (NIN == 2 && !DUAL) {
    if constexpr (!PRE) {
#pragma unroll
      for (int q = 0; q < C::E; ++q) v1[q] = ldg<T>(in1 + col + (size_t)(t + q * C::P) * kTW);
    }
    __syncthreads();
    fft_group<T, L, C::E, -1>(v1, lds + c, C::CW, tw, t);
  }
  const double s = sa[bp.z].s;
  const double inv_ny = 1.0 / (double)geo.ny;
  const double dtnu = geo.rho > 0.0 ? geo.dt * (geo.eta / geo.rho) : 0.0;
#pragma unroll
  for (int q = 0; q < C::E; ++q) {
    const int n = t + q * C::P;
    const Modes md = modes(geo, m, n);
    const double lam = BANDED ? lambda_banded(geo, m, n, s) : lambda_of(md, s);
    const bool zero = (m == 0 && n == 0);
    const double a0x = (double)v0[q].x, a0y = (double)v0[q].y;
    if constexpr (MODE == COL_CH) {
      // phi' = phi_h + (1 + D4/2)^-1 (-A D2 phi_h - D4 phi_h + B D2 f)
      const double d2 = geo.dt * geo.M * lam;
      const double d4 = geo.dt * geo.kappa * geo.M * lam * lam;
      const double den = rcp64(1.0 + 0.5 * d4);
      const double h1 = (1.0 + (-geo.A * d2 - d4) * den) * inv_ny;
      const double h2 = (geo.B * d2 * den) * inv_ny;
      const double a1x = (double)v1[q].x, a1y = (double)v1[q].y;
      v0[q] = {T(h1 * a0x + h2 * a1x), T(h1 * a0y + h2 * a1y)};
    } else if constexpr (MODE == COL_FLOW) {
      // omega' = omega_h + (1 - C/2)^-1 (C omega_h + dt g), C = dt nu lambda;
      // psi' = -omega' / lambda; the q = 0 mode of both is zero.
      const double ct = dtnu * lam;
      const double den = rcp64(1.0 - 0.5 * ct);
      double b1 = (1.0 + ct * den) * inv_ny;
      double b2 = (geo.dt * den) * inv_ny;
      double il = zero ? 0.0 : -rcp64(lam);
      if (zero) { b1 = 0.0; b2 = 0.0; }
      const double a1x = (double)v1[q].x, a1y = (double)v1[q].y;
      const double ox = b1 * a0x + b2 * a1x, oy = b1 * a0y + b2 * a1y;
      v0[q] = {T(ox), T(oy)};
      v1[q] = {T(il * ox), T(il * oy)};
    } else if constexpr (MODE == COL_STOKES) {
      // psi' = g / lambda^2
      const double p = zero ? 0.0 : inv_ny * rcp64(lam * lam);
      v0[q] = {T(p * a0x), T(p * a0y)};
    } else {
      // psi = -omega / lambda
      const double p = zero ? 0.0 : -inv_ny * rcp64(lam);
      v0[q] = {T(p * a0x), T(p * a0y)};
    }
    LE_SCHED_FENCE();
  }
  __syncthreads();
  if constexpr (DUAL && NOUT == 2) {
    fft_group2<T, L, C::E, +1>(v0, v1, lds + c, lds1 + c, C::CW, tw, t);
    if (ok) {
#pragma unroll
      for (int q = 0; q < C::E; ++q) {
        stg<T>(out0 + col + (size_t)(t + q * C::P) * kTW, v0[q]);
        stg<T>(out1 + col + (size_t)(t + q * C::P) * kTW, v1[q]);
      }
    }
    return;
  }
  fft_group<T, L, C::E, +1>(v0, lds + c, C::CW, tw, t);
  if (ok) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) stg<T>(out0 + col + (size_t)(t + q * C::P) * kTW, v0[q]);
  }
  if constexpr (NOUT == 2) {
    __syncthreads();
    fft_group<T, L, C::E, +1, LTW>(v1, lds + c, C::CW, tw, t, ltw);
    if (ok) {
#pragma unroll
      for (int q = 0; q < C::E; ++q) stg<T>(out1 + col + (size_t)(t + q * C::P) * kTW, v1[q]);
    }
  }
}

// ---------------------------------------------------------------- observables

// Lab-frame products and shell index of mode (m, n), evaluated without
// contraction so the integer shell decision is reproducible.
__device__ __forceinline__ void obs_mode(const Geo& g, int m, int n, double s, double dk,
                                         double& xx, double& xy, double& yy, double& qmod,
                                         int& bin) {
#pragma clang fp contract(off)
  const Modes md = modes_exact(g, m, n);
  xx = md.qx * md.qx;
  xy = md.P - s * xx;
  yy = md.qy * md.qy - 2.0 * s * md.P + s * s * xx;
  const double q2 = xx + yy;
  qmod = sqrt(q2);
  bin = (int)floor(qmod / dk + 0.5);
}

// Spectral observables: column transforms of phi (and psi), per-block fixed
// order partial sums of OBS_* and of the S(k) shells.
template <typename T, int L>
__global__ __launch_bounds__(ObsCfg<L>::THREADS) LE_OCCUPANCY void k_obs_spectral(
    const Run* __restrict__ run, const StepArgs* __restrict__ sa, int bphi, int bpsi,
    double* __restrict__ part, double* __restrict__ bins, double* __restrict__ counts) {
  using C = ObsCfg<L>;
  const Geo& geo = run->g;
  auto phih = bufp<const c2<T>>(*run, bphi);
  gp<const c2<T>> psih = bpsi >= 0 ? bufp<const c2<T>>(*run, bpsi) : nullptr;
  auto tw = to_global<const c2<double>>(run->twy);
  constexpr int NB = L / 2;  // shells 1 .. ny/2
  constexpr int NBT = (NB + C::THREADS - 1) / C::THREADS;
  constexpr int NE = C::CW * L;
  constexpr size_t LDS_BYTES = (size_t)NE * sizeof(c2<T>);
  constexpr size_t BIN_BYTES = (size_t)NE * (sizeof(double) + sizeof(int));
  __shared__ __attribute__((aligned(16))) unsigned char raw[LDS_BYTES > BIN_BYTES ? LDS_BYTES : BIN_BYTES];
  c2<T>* lds = reinterpret_cast<c2<T>*>(raw);
  double* bval = reinterpret_cast<double*>(raw);
  int* bidx = reinterpret_cast<int*>(bval + NE);
  __shared__ double red[OBS_NSPEC * ((C::THREADS + 63) / 64)];

  const int S = geo.nx / 2 + 1;
  const int c = threadIdx.x % C::CW, t = threadIdx.x / C::CW;
  const int m0 = xcd_block(blockIdx.x, gridDim.x) * C::CW + c;
  const bool ok = m0 < S;
  const int m = ok ? m0 : 0;
  const size_t col = spec_index(L, 0, m);
  c2<T> v0[C::E], v1[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) v0[q] = ldg<T>(phih + col + (size_t)(t + q * C::P) * kTW);
  fft_group<T, L, C::E, -1>(v0, lds + c, C::CW, tw, t);
  const bool has_psi = psih != nullptr;
  if (has_psi) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) v1[q] = ldg<T>(psih + col + (size_t)(t + q * C::P) * kTW);
    __syncthreads();
    fft_group<T, L, C::E, -1>(v1, lds + c, C::CW, tw, t);
  }
  const double s = sa->s;
  const double N = (double)geo.nx * (double)geo.ny;
  const double dk = 6.283185307179586476925286766559 / geo.ly;
  const double wgt = (!ok) ? 0.0 : ((m == 0 || m == geo.nx / 2) ? 1.0 : 2.0);
  double acc[OBS_NSPEC];
#pragma unroll
  for (int k = 0; k < OBS_NSPEC; ++k) acc[k] = 0.0;
  __syncthreads();  // transforms done: LDS becomes the shell scratch
#pragma unroll
  for (int q = 0; q < C::E; ++q) {
    const int n = t + q * C::P;
    double xx, xy, yy, qmod;
    int bin;
    obs_mode(geo, m, n, s, dk, xx, xy, yy, qmod, bin);
    const double px = (double)v0[q].x, py = (double)v0[q].y;
    const double S2 = (px * px + py * py) / N;
    const double wS = wgt * S2;
    acc[OBS_SUM_S] += wS;
    if (!(m == 0 && n == 0)) {
      acc[OBS_SUM_S_NZ] += wS;
      acc[OBS_SUM_S_OVER_Q] += wS / qmod;
    }
    acc[OBS_XX] += xx * wS;
    acc[OBS_XY] += xy * wS;
    acc[OBS_YY] += yy * wS;
    if (has_psi) {
      const double sx = (double)v1[q].x, sy = (double)v1[q].y;
      acc[OBS_RE] += wgt * xy * (sx * sx + sy * sy);
    }
    const int e = n * C::CW + c;
    const bool inb = (bin >= 1 && bin <= NB && wgt > 0.0);
    bidx[e] = inb ? bin : 0;
    bval[e] = inb ? wS : 0.0;
    LE_SCHED_FENCE();
  }
  // fixed-order block reduction of each sum: a butterfly across each
  // wavefront (DPP/permute shuffles, no barrier), then the wavefront sums in
  // wavefront order
  constexpr int NW = (C::THREADS + 63) / 64;
  constexpr int WS = C::THREADS < 64 ? C::THREADS : 64;
#pragma unroll
  for (int k = 0; k < OBS_NSPEC; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = WS / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, WS);
    if ((threadIdx.x & 63) == 0) red[k * NW + (threadIdx.x >> 6)] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < OBS_NSPEC) {
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += red[threadIdx.x * NW + w];
    part[(size_t)blockIdx.x * OBS_NSPEC + threadIdx.x] = v;
  }
  // Shells: thread owns shells b = 1 + tid + k * THREADS.  For each column
  // the modes of shell b lie in at most two runs of n (|q_lab| is a parabola
  // in qy); each run is bracketed from the shell radii, widened by two rows,
  // and the stored per-mode decisions pick the members, in increasing n.
  __syncthreads();
  const int ny = geo.ny;
  const double rad = geo.ly / 6.283185307179586476925286766559;  // n' per unit qy
  for (int k = 0; k < NBT; ++k) {
    const int b = 1 + (int)threadIdx.x + k * C::THREADS;
    double sb = 0.0, cb = 0.0;
    if (b <= NB) {
      const double qlo = (b - 0.5) * dk, qhi = (b + 0.5) * dk;
      for (int cc = 0; cc < C::CW; ++cc) {
        const int mc = xcd_block(blockIdx.x, gridDim.x) * C::CW + cc;
        if (mc >= S) break;
        // the Nyquist row drops the cross term: it is checked outright; the
        // Nyquist column (no cross term either) has |q_lab|^2 =
        // (1 + s^2) qx^2 + qy^2, bracketed about qy = 0
        // a mode's weight is its column's (1 on the DC and Nyquist columns, 2
        // on the others: each stands for its conjugate too)
        const double wcol = (mc == 0 || mc == geo.nx / 2) ? 1.0 : 2.0;
        auto take = [&](int n) {
          const int e = n * C::CW + cc;
          if (bidx[e] == b) { sb += bval[e]; cb += wcol; }
        };
        take(ny / 2);
        const bool nyq = mc == geo.nx / 2;
        const Modes md = modes(geo, mc, 0);
        const double qx2 = md.qx * md.qx * (nyq ? 1.0 + s * s : 1.0);
        if (qhi * qhi <= qx2 * (1.0 - 1e-12)) continue;
        const double a = sqrt(fmax(0.0, qlo * qlo - qx2));
        const double c2v = sqrt(fmax(0.0, qhi * qhi - qx2));
        const double sh = nyq ? 0.0 : s * md.qx;
        int lo1 = (int)floor((-c2v + sh) * rad) - 2, hi1 = (int)ceil((-a + sh) * rad) + 2;
        int lo2 = (int)floor((a + sh) * rad) - 2, hi2 = (int)ceil((c2v + sh) * rad) + 2;
        if (lo2 <= hi1 + 1) { hi1 = hi2; lo2 = 1; hi2 = 0; }   // the runs touch: merge
        const int nlo = -ny / 2 + 1, nhi = ny / 2 - 1;          // Nyquist row done above
        for (int run = 0; run < 2; ++run) {
          int lo = run == 0 ? lo1 : lo2, hi = run == 0 ? hi1 : hi2;
          lo = lo < nlo ? nlo : lo;
          hi = hi > nhi ? nhi : hi;
          for (int np = lo; np <= hi; ++np) take(np < 0 ? np + ny : np);
        }
      }
      bins[(size_t)blockIdx.x * NB + (b - 1)] = sb;
      counts[(size_t)blockIdx.x * NB + (b - 1)] = cb;
    }
  }
}

// Real-space partial sums: sum phi, sum phi^2 (FP64) and the non-finite
// count.  Block b sums its contiguous slice (pairs of values per load), each
// thread in a fixed order, then a butterfly within each wavefront and the four
// wavefront sums in order: deterministic.
template <typename T>
__global__ __launch_bounds__(256) void k_obs_real(const Run* __restrict__ run, int bphi,
                                                  double* __restrict__ part) {
  __shared__ double red[3][4];
  auto phi = reinterpret_cast<gp<const c2<T>>>(bufp<const T>(*run, bphi));
  const size_t n = (size_t)run->g.nx * run->g.ny / 2;  // pairs (nx is even)
  const size_t per = (n + gridDim.x - 1) / gridDim.x;
  const size_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  double a = 0.0, b = 0.0, bad = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += 256) {
    const c2<T> v = ldg<T>(phi + e);
    const double x0 = (double)v.x, x1 = (double)v.y;
    if (isfinite(x0)) { a += x0; b += x0 * x0; } else { bad += 1.0; }
    if (isfinite(x1)) { a += x1; b += x1 * x1; } else { bad += 1.0; }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
    bad += __shfl_xor(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
    red[2][threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 3)
    part[(size_t)blockIdx.x * 3 + threadIdx.x] =
        ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) + red[threadIdx.x][3];
}

}  // namespace le
