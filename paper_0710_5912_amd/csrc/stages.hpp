// stages.hpp -- the stage kernels of the split step (Appendix B), templated
// on the storage type T (float or double) and the transform lengths.
//
// Field layouts in HBM (all row-major, x fastest):
//   real field       T[ny][nx]
//   row spectrum     c2<T>[ny][nx/2 + 1]: the unnormalised DFT of each real
//                    row along x, modes m = 0 .. nx/2 (DC and Nyquist real).
// A 2D transform is a row transform (fused into the row kernels) followed by
// a column transform over each of the nx/2+1 columns (fused into the column
// kernels, which also apply the per-mode update and the inverse column
// transform, scaled by 1/ny).  Row kernels own G whole rows per block, column
// kernels CW adjacent columns per block.
#pragma once

#include "common.hpp"
#include "fft.hpp"

namespace le {

// Launch shapes.  E: values per thread of a transform (P = L/E threads per
// transform); G: rows per block; CW: adjacent columns per block.
constexpr int row_elems(int L) { return L >= 8 ? 8 : L; }
constexpr int col_elems(int L) { return L >= 8 ? 8 : L; }

// Occupancy hint for the stage kernels (waves per SIMD the register
// allocation must allow).
#define LE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(2)))
// Keep the scheduler from interleaving consecutive unrolled iterations (which
// would hoist every iteration's loads and blow the register budget).
#define LE_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int L>
struct RowCfg {
  static constexpr int E = row_elems(L);
  static constexpr int P = L / E;
  static constexpr int G = clampi(128 / P, 1, 16);
  static constexpr int THREADS = G * P;
};

template <int L>
struct MuCfg {
  static constexpr int E = row_elems(L);
  static constexpr int P = L / E;
  static constexpr int G = clampi(256 / P, 1, 16);
  static constexpr int THREADS = G * P;
};

template <int L>
struct ColCfg {
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
__device__ __forceinline__ T* bufp(const Run& R, int b) {
  return static_cast<T*>(R.buf[b]);
}

// ---------------------------------------------------------------- helpers

template <typename T, int L, int E>
__device__ __forceinline__ void store_row_spec(c2<T>* __restrict__ X, const c2<T>* v, int t) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = t + q * P;
    if (m == 0) {
      X[0] = {v[q].x, T(0)};
      X[L] = {v[q].y, T(0)};
    } else {
      X[m] = v[q];
    }
  }
}

template <typename T, int L, int E>
__device__ __forceinline__ void load_row_spec(const c2<T>* __restrict__ X, c2<T>* v, int t) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = t + q * P;
    v[q] = (m == 0) ? c2<T>{X[0].x, X[L].x} : X[m];
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

// ---------------------------------------------------------------- row kernels

// Forward row transform of one real field (buffer bin -> row spectrum bout).
template <typename T, int L>
__global__ __launch_bounds__(RowCfg<L>::THREADS) LE_OCCUPANCY void k_row_r2c(
    const Run* __restrict__ runs, int bin, int bout) {
  using C = RowCfg<L>;
  __shared__ c2<T> lds[C::G * L];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const int ny = R.g.ny;
  const T* x = bufp<T>(R, bin);
  c2<T>* X = bufp<c2<T>>(R, bout);
  const c2<T>* tw = static_cast<const c2<T>*>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j = bp.x * C::G + g;
  const bool ok = j < ny;
  const c2<T>* xr = reinterpret_cast<const c2<T>*>(x + (size_t)(ok ? j : 0) * 2 * L);
  c2<T> v[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) v[q] = xr[t + q * C::P];
  row_r2c<T, L, C::E>(v, lds + g * L, tw, t);
  if (ok) store_row_spec<T, L, C::E>(X + (size_t)j * (L + 1), v, t);
}

// Inverse row transform; the block's y picks the field (bin0 -> bout0, or
// bin1 -> bout1).
template <typename T, int L>
__global__ __launch_bounds__(RowCfg<L>::THREADS) LE_OCCUPANCY void k_row_c2r(
    const Run* __restrict__ runs, int bin0, int bout0, int bin1, int bout1) {
  using C = RowCfg<L>;
  __shared__ c2<T> lds[C::G * L];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const int ny = R.g.ny;
  const c2<T>* X = bufp<const c2<T>>(R, bp.y == 0 ? bin0 : bin1);
  T* x = bufp<T>(R, bp.y == 0 ? bout0 : bout1);
  const c2<T>* tw = static_cast<const c2<T>*>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j = bp.x * C::G + g;
  const bool ok = j < ny;
  const int jj = ok ? j : 0;
  c2<T> v[C::E];
  load_row_spec<T, L, C::E>(X + (size_t)jj * (L + 1), v, t);
  row_c2r<T, L, C::E>(v, lds + g * L, tw, t);
  if (ok) {
    c2<T>* xr = reinterpret_cast<c2<T>*>(x + (size_t)j * 2 * L);
#pragma unroll
    for (int q = 0; q < C::E; ++q) xr[t + q * C::P] = v[q];
  }
}

// Periodic read of a real field at (row jj, column i), nx a power of two.
template <typename T>
__device__ __forceinline__ T at(const T* __restrict__ f, int jj, int i, int nx) {
  return f[(size_t)jj * nx + (i & (nx - 1))];
}

// Stencil coefficients of one step, in the storage precision.
template <typename T>
struct Stencil {
  T inv2dx, inv2dy, w, wm;  // 1/(2dx), 1/(2dy), |s|/c, 1 - |s|/c
  int off;                  // sign(s) * r: x offset of the diagonal y difference
  bool sheared;             // w != 0
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
  st.sheared = w != 0.0;
  return st;
}

// Central x difference at (j, i) and (j, i+1) from a field in global memory.
template <typename T>
__device__ __forceinline__ void dx_pair(const T* f, int j, int i, int nx, T inv2dx, T& d0, T& d1) {
  const T a = at(f, j, i - 1, nx), b = at(f, j, i, nx), c = at(f, j, i + 1, nx),
          d = at(f, j, i + 2, nx);
  d0 = (c - a) * inv2dx;
  d1 = (d - b) * inv2dx;
}

// Shear-interpolated y difference (Eq. p1y, offsets +-r, weight |s|/c) at
// (j, i) and (j, i+1); jp = j+1, jm = j-1 (periodic).
template <typename T>
__device__ __forceinline__ void dys_pair(const T* f, int jp, int jm, int i, int nx,
                                         const Stencil<T>& st, T& d0, T& d1) {
  const T p0 = at(f, jp, i, nx), p1 = at(f, jp, i + 1, nx);
  const T m0 = at(f, jm, i, nx), m1 = at(f, jm, i + 1, nx);
  if (st.sheared) {
    const T pd0 = at(f, jp, i - st.off, nx), pd1 = at(f, jp, i + 1 - st.off, nx);
    const T md0 = at(f, jm, i + st.off, nx), md1 = at(f, jm, i + 1 + st.off, nx);
    d0 = (st.wm * (p0 - m0) + st.w * (pd0 - md0)) * st.inv2dy;
    d1 = (st.wm * (p1 - m1) + st.w * (pd1 - md1)) * st.inv2dy;
  } else {
    d0 = (p0 - m0) * st.inv2dy;
    d1 = (p1 - m1) * st.inv2dy;
  }
}

// Stage 1a (Eq. advective), one output field per blockIdx.y:
//   0: phi_h = phi - dt [Dys psi Dx phi - Dx psi Dys phi]
//   1: f = phi^3
//   2: omega_h = omega - dt [Dys psi Dx omega - Dx psi Dys omega]  (inertial)
// followed by the forward row transform of that field.
template <typename T, int L>
__global__ __launch_bounds__(RowCfg<L>::THREADS) LE_OCCUPANCY void k_advect(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa) {
  using C = RowCfg<L>;
  constexpr int NX = 2 * L;
  __shared__ c2<T> lds[C::G * L];
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const T* phi = bufp<const T>(R, B_PHI);
  const T* om = bufp<const T>(R, B_OM_R);
  const T* psi = bufp<const T>(R, B_PS_R);
  const c2<T>* tw = static_cast<const c2<T>*>(R.twx);
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j0 = bp.x * C::G + g;
  const bool ok = j0 < geo.ny;
  const int j = ok ? j0 : 0;
  const int jp = (j + 1 == geo.ny) ? 0 : j + 1;
  const int jm = (j == 0) ? geo.ny - 1 : j - 1;
  const int field = bp.y;
  const Stencil<T> st = make_stencil<T>(geo, sa[bp.z].s);
  const T dt = T(geo.dt);
  c2<T> v[C::E];
  if (field == 1) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) {
      const int i = 2 * (t + q * C::P);
      const T p0 = phi[(size_t)j * NX + i], p1 = phi[(size_t)j * NX + i + 1];
      v[q] = {p0 * p0 * p0, p1 * p1 * p1};
    }
  } else {
    const T* a = field == 0 ? phi : om;
#pragma unroll
    for (int q = 0; q < C::E; ++q) {
      const int i = 2 * (t + q * C::P);
      T sx0, sx1, sy0, sy1, ax0, ax1, ay0, ay1;
      dx_pair(psi, j, i, NX, st.inv2dx, sx0, sx1);
      dys_pair(psi, jp, jm, i, NX, st, sy0, sy1);
      dx_pair(a, j, i, NX, st.inv2dx, ax0, ax1);
      dys_pair(a, jp, jm, i, NX, st, ay0, ay1);
      const T a0 = a[(size_t)j * NX + i], a1 = a[(size_t)j * NX + i + 1];
      v[q] = {a0 - dt * (sy0 * ax0 - sx0 * ay0), a1 - dt * (sy1 * ax1 - sx1 * ay1)};
      LE_SCHED_FENCE();
    }
  }
  row_r2c<T, L, C::E>(v, lds + g * L, tw, t);
  c2<T>* out = bufp<c2<T>>(R, field == 0 ? B_PHIH : (field == 1 ? B_FH : B_OMH));
  if (ok) store_row_spec<T, L, C::E>(out + (size_t)j * (L + 1), v, t);
}

// Stage 2a: mu = B phi^3 - A phi - kappa [(1+s^2) Dxx + Dyy - 2 s Dxy] phi on
// rows j0-1 .. j0+G (into LDS), then g = -[Dx phi Dys mu - Dys phi Dx mu] * inv
// (inv = 1/rho, or 1/eta on the Stokes branch) and its forward row transform.
template <typename T, int L>
__global__ __launch_bounds__(MuCfg<L>::THREADS) LE_OCCUPANCY void k_mu_source(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa) {
  using C = MuCfg<L>;
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const T* phi = bufp<const T>(R, B_PHI);
  c2<T>* gh = bufp<c2<T>>(R, B_GH);
  const c2<T>* tw = static_cast<const c2<T>*>(R.twx);
  const double inv_coef = 1.0 / (geo.rho > 0.0 ? geo.rho : geo.eta);
  constexpr int NX = 2 * L;
  constexpr int MU_ROWS = C::G + 2;
  constexpr int LDS_T = MU_ROWS * NX;  // >= C::G * L complex
  __shared__ __attribute__((aligned(16))) T smu[LDS_T];
  c2<T>* lds = reinterpret_cast<c2<T>*>(smu);
  const int ny = geo.ny;
  const int jbase = bp.x * C::G;
  const double s = sa[bp.z].s;
  const T cxx = T((1.0 + s * s) / (geo.dx * geo.dx));
  const T cyy = T(1.0 / (geo.dy * geo.dy));
  const T cxy = T(-2.0 * s / (4.0 * geo.dx * geo.dy));
  const T A = T(geo.A), B = T(geo.B), kap = T(geo.kappa);
  const T two = T(2);
  for (int e = threadIdx.x; e < MU_ROWS * NX; e += C::THREADS) {
    const int k = e / NX, i = e % NX;
    int jj = jbase - 1 + k;
    jj = (jj % ny + ny) % ny;
    const int jp = (jj + 1 == ny) ? 0 : jj + 1;
    const int jm = (jj == 0) ? ny - 1 : jj - 1;
    const T c = at(phi, jj, i, NX);
    const T dxx = at(phi, jj, i + 1, NX) - two * c + at(phi, jj, i - 1, NX);
    const T dyy = at(phi, jp, i, NX) - two * c + at(phi, jm, i, NX);
    const T dxy = at(phi, jp, i + 1, NX) - at(phi, jm, i + 1, NX) - at(phi, jp, i - 1, NX) +
                  at(phi, jm, i - 1, NX);
    smu[e] = B * c * c * c - A * c - kap * (cxx * dxx + cyy * dyy + cxy * dxy);
  }
  __syncthreads();
  const int g = threadIdx.x / C::P, t = threadIdx.x % C::P;
  const int j0 = jbase + g;
  const bool ok = j0 < ny;
  const int j = ok ? j0 : 0;
  const int jp = (j + 1 == ny) ? 0 : j + 1;
  const int jm = (j == 0) ? ny - 1 : j - 1;
  const Stencil<T> st = make_stencil<T>(geo, s);
  const T* mu_c = smu + (g + 1) * NX;   // row j
  const T* mu_p = smu + (g + 2) * NX;   // row j + 1
  const T* mu_m = smu + g * NX;         // row j - 1
  const T neg_inv = T(-inv_coef);
  c2<T> v[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) {
    const int i = 2 * (t + q * C::P);
    T px0, px1, py0, py1;
    dx_pair(phi, j, i, NX, st.inv2dx, px0, px1);
    dys_pair(phi, jp, jm, i, NX, st, py0, py1);
    const T mx0 = (mu_c[(i + 1) & (NX - 1)] - mu_c[(i - 1) & (NX - 1)]) * st.inv2dx;
    const T mx1 = (mu_c[(i + 2) & (NX - 1)] - mu_c[i]) * st.inv2dx;
    T my0, my1;
    {
      const T p0 = mu_p[i], p1 = mu_p[i + 1];
      const T m0 = mu_m[i], m1 = mu_m[i + 1];
      if (st.sheared) {
        const T pd0 = mu_p[(i - st.off) & (NX - 1)], pd1 = mu_p[(i + 1 - st.off) & (NX - 1)];
        const T md0 = mu_m[(i + st.off) & (NX - 1)], md1 = mu_m[(i + 1 + st.off) & (NX - 1)];
        my0 = (st.wm * (p0 - m0) + st.w * (pd0 - md0)) * st.inv2dy;
        my1 = (st.wm * (p1 - m1) + st.w * (pd1 - md1)) * st.inv2dy;
      } else {
        my0 = (p0 - m0) * st.inv2dy;
        my1 = (p1 - m1) * st.inv2dy;
      }
    }
    v[q] = {neg_inv * (px0 * my0 - py0 * mx0), neg_inv * (px1 * my1 - py1 * mx1)};
    LE_SCHED_FENCE();
  }
  __syncthreads();  // mu is dead; its LDS becomes the transform's
  row_r2c<T, L, C::E>(v, lds + g * L, tw, t);
  if (ok) store_row_spec<T, L, C::E>(gh + (size_t)j * (L + 1), v, t);
}

// Strain-wrap remap of a row spectrum: row j shifted by sh_j = (dkr * j) mod nx,
// X[j][m] *= exp(-2 pi i m sh_j / nx).
template <typename T>
__global__ void k_remap_spec(const Run* __restrict__ run, int b, int dkr) {
  const int nx = run->g.nx, ny = run->g.ny;
  c2<T>* X = bufp<c2<T>>(*run, b);
  const c2<T>* twx = static_cast<const c2<T>*>(run->twx);
  const int S = nx / 2 + 1;
  const size_t total = (size_t)ny * S;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / S), m = (int)(e % S);
    const long long sh = (((long long)dkr * j) % nx + nx) % nx;
    const int idx = (int)(((long long)m * sh) % nx);
    X[e] = cmul(X[e], twx[idx]);
  }
}

// Strain-wrap remap of a real field: out[j][i] = in[j][(i - dkr j) mod nx].
template <typename T>
__global__ void k_remap_real(const Run* __restrict__ run, int bin, int bout, int dkr) {
  const int nx = run->g.nx, ny = run->g.ny;
  const T* in = bufp<const T>(*run, bin);
  T* out = bufp<T>(*run, bout);
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
  const T* in = bufp<const T>(*run, bin);
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
  const T* in = bufp<const T>(*run, bin);
  T* out = bufp<T>(*run, bout);
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
template <typename T, int L, int MODE>
__global__ __launch_bounds__(ColCfg<L>::THREADS) LE_OCCUPANCY void k_column(
    const Run* __restrict__ runs, const StepArgs* __restrict__ sa, int bin0, int bin1,
    int bout0, int bout1) {
  using C = ColCfg<L>;
  const BPos bp = block_pos();
  const Run& R = runs[bp.z];
  const Geo& geo = R.g;
  const c2<T>* in0 = bufp<const c2<T>>(R, bin0);
  const c2<T>* in1 = bufp<const c2<T>>(R, bin1);
  c2<T>* out0 = bufp<c2<T>>(R, bout0);
  c2<T>* out1 = bufp<c2<T>>(R, bout1);
  const c2<T>* tw = static_cast<const c2<T>*>(R.twy);
  constexpr int NIN = (MODE == COL_CH || MODE == COL_FLOW) ? 2 : 1;
  constexpr int NOUT = (MODE == COL_FLOW) ? 2 : 1;
  __shared__ c2<T> lds[C::CW * L];
  const int S = geo.nx / 2 + 1;
  const int c = threadIdx.x % C::CW, t = threadIdx.x / C::CW;
  const int m0 = bp.x * C::CW + c;
  const bool ok = m0 < S;
  const int m = ok ? m0 : 0;
  c2<T> v0[C::E], v1[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) v0[q] = in0[(size_t)(t + q * C::P) * S + m];
  fft_group<T, L, C::E, -1>(v0, lds + c, C::CW, tw, t);
  if constexpr (NIN == 2) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) v1[q] = in1[(size_t)(t + q * C::P) * S + m];
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
    const double lam = lambda_of(md, s);
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
  fft_group<T, L, C::E, +1>(v0, lds + c, C::CW, tw, t);
  if (ok) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) out0[(size_t)(t + q * C::P) * S + m] = v0[q];
  }
  if constexpr (NOUT == 2) {
    __syncthreads();
    fft_group<T, L, C::E, +1>(v1, lds + c, C::CW, tw, t);
    if (ok) {
#pragma unroll
      for (int q = 0; q < C::E; ++q) out1[(size_t)(t + q * C::P) * S + m] = v1[q];
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
__global__ __launch_bounds__(ColCfg<L>::THREADS) LE_OCCUPANCY void k_obs_spectral(
    const Run* __restrict__ run, const StepArgs* __restrict__ sa, int bphi, int bpsi,
    double* __restrict__ part, double* __restrict__ bins, double* __restrict__ counts) {
  using C = ColCfg<L>;
  const Geo& geo = run->g;
  const c2<T>* phih = bufp<const c2<T>>(*run, bphi);
  const c2<T>* psih = bpsi >= 0 ? bufp<const c2<T>>(*run, bpsi) : nullptr;
  const c2<T>* tw = static_cast<const c2<T>*>(run->twy);
  constexpr int NB = L / 2;  // shells 1 .. ny/2
  constexpr int NBT = (NB + C::THREADS - 1) / C::THREADS;
  constexpr int NE = C::CW * L;
  constexpr size_t LDS_BYTES = (size_t)NE * sizeof(c2<T>);
  constexpr size_t BIN_BYTES = (size_t)NE * (2 * sizeof(double) + sizeof(int));
  __shared__ __attribute__((aligned(16))) unsigned char raw[LDS_BYTES > BIN_BYTES ? LDS_BYTES : BIN_BYTES];
  c2<T>* lds = reinterpret_cast<c2<T>*>(raw);
  double* bval = reinterpret_cast<double*>(raw);
  double* bwgt = bval + NE;
  int* bidx = reinterpret_cast<int*>(bwgt + NE);
  __shared__ double red[C::THREADS];

  const int S = geo.nx / 2 + 1;
  const int c = threadIdx.x % C::CW, t = threadIdx.x / C::CW;
  const int m0 = xcd_block(blockIdx.x, gridDim.x) * C::CW + c;
  const bool ok = m0 < S;
  const int m = ok ? m0 : 0;
  c2<T> v0[C::E], v1[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) v0[q] = phih[(size_t)(t + q * C::P) * S + m];
  fft_group<T, L, C::E, -1>(v0, lds + c, C::CW, tw, t);
  const bool has_psi = psih != nullptr;
  if (has_psi) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) v1[q] = psih[(size_t)(t + q * C::P) * S + m];
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
    bwgt[e] = inb ? wgt : 0.0;
    LE_SCHED_FENCE();
  }
  // fixed-order block reduction of each sum
  for (int k = 0; k < OBS_NSPEC; ++k) {
    red[threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = C::THREADS / 2; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * OBS_NSPEC + k] = red[0];
    __syncthreads();
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
        // the Nyquist row (and the whole Nyquist column) drop the cross
        // term: they are checked outright
        auto take = [&](int n) {
          const int e = n * C::CW + cc;
          if (bidx[e] == b) { sb += bval[e]; cb += bwgt[e]; }
        };
        if (mc == geo.nx / 2) {
          for (int n = 0; n < ny; ++n) take(n);
          continue;
        }
        take(ny / 2);
        const Modes md = modes(geo, mc, 0);
        const double qx2 = md.qx * md.qx;
        if (qhi * qhi <= qx2 * (1.0 - 1e-12)) continue;
        const double a = sqrt(fmax(0.0, qlo * qlo - qx2));
        const double c2v = sqrt(fmax(0.0, qhi * qhi - qx2));
        const double sh = s * md.qx;
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

// Real-space partial sums: sum phi, sum phi^2 (FP64) and the non-finite count.
template <typename T>
__global__ __launch_bounds__(256) void k_obs_real(const Run* __restrict__ run, int bphi,
                                                  double* __restrict__ part) {
  __shared__ double red[3][256];
  const T* phi = bufp<const T>(*run, bphi);
  const size_t n = (size_t)run->g.nx * run->g.ny;
  const size_t per = (n + gridDim.x - 1) / gridDim.x;
  const size_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  double a = 0.0, b = 0.0, bad = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += 256) {
    const double x = (double)phi[e];
    if (isfinite(x)) { a += x; b += x * x; } else { bad += 1.0; }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = bad;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) part[(size_t)blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace le
