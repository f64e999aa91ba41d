// fft.hpp -- LDS-staged Stockham FFTs for gfx950 (wave64).
//
// The paper moves every field between real and reciprocal space twice per
// step with a library 2D FFT (Appendix B, stage 1b); here the 2D transform is
// split into a real-to-complex transform along each row (x) and a complex
// transform along each column (y), and both halves are fused into the stage
// kernels.  This header holds the building blocks:
//
//   * c2<T>          complex value (T = float or double);
//   * dft_reg        radix-R DFT on R values held in registers (R <= 16);
//   * fft_group      length-L complex FFT done by a group of L/E threads that
//                    each hold E values, exchanging through LDS between the
//                    passes (Stockham autosort: natural order in and out);
//   * row_r2c/c2r    real row of 2L values <-> L packed complex values.
//
// Forward transforms are unnormalised, F[a](m) = sum_i a_i exp(-2 pi i m i/n).
#pragma once

#include <hip/hip_runtime.h>

namespace le {

template <typename T>
struct alignas(2 * sizeof(T)) c2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ c2<T> cmulc(c2<T> a, c2<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// cos and sin of 2 pi k / 16, k = 0..15, to double precision.
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// d * exp(DIR * 2 pi i * k / R), DIR = -1 forward, +1 inverse.  k is a
// compile-time constant after unrolling, so the trivial cases fold away.
template <typename T, int DIR, int R>
__device__ __forceinline__ c2<T> rot(c2<T> d, int k) {
  k &= (R - 1);
  if (k == 0) return d;
  if (4 * k == R) return DIR < 0 ? c2<T>{d.y, -d.x} : c2<T>{-d.y, d.x};
  if (2 * k == R) return {-d.x, -d.y};
  if (4 * k == 3 * R) return DIR < 0 ? c2<T>{-d.y, d.x} : c2<T>{d.y, -d.x};
  const int i16 = k * (16 / R);
  const T cr = static_cast<T>(kCos16[i16]);
  const T sr = static_cast<T>(DIR * kSin16[i16]);
  return {d.x * cr - d.y * sr, d.x * sr + d.y * cr};
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

// In-register radix-R DFT (R = 1, 2, 4, 8, 16): radix-2 decimation in
// frequency, then a compile-time bit-reversal rename.
template <typename T, int DIR, int R>
__device__ __forceinline__ void dft_reg(c2<T>* v) {
  if constexpr (R >= 2) {
#pragma unroll
    for (int span = R / 2; span >= 1; span >>= 1) {
#pragma unroll
      for (int start = 0; start < R; start += 2 * span) {
#pragma unroll
        for (int k = 0; k < span; ++k) {
          const c2<T> a = v[start + k];
          const c2<T> b = v[start + k + span];
          v[start + k] = cadd(a, b);
          v[start + k + span] = rot<T, DIR, R>(csub(a, b), k * (R / (2 * span)));
        }
      }
    }
    constexpr int bits = ilog2(R);
    c2<T> tmp[R];
#pragma unroll
    for (int i = 0; i < R; ++i) tmp[i] = v[bitrev(i, bits)];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = tmp[i];
  }
}

// Radix of the first Stockham pass: L / E^n with 1 < R0 <= E.
constexpr int first_radix(int L, int E) {
  int r = L;
  while (r > E) r /= E;
  return r;
}

// Elements per thread used for a transform of length L.
constexpr int elems_for(int L) { return L >= 1024 ? 16 : (L >= 8 ? 8 : L); }

// Length-L complex FFT by a group of P = L/E threads; thread t in [0, P).
// On entry v[q] = x[t + q P]; on exit v[q] = X[t + q P].
// lds: the group's LDS area, element i at lds[i * LS].  tw: table of
// exp(-2 pi i k / (2L)), k < 2L.  Every thread of the block must call this
// with the same L (the passes contain __syncthreads()).  On return other
// threads may still read lds: barrier before reusing it.
template <typename T, int L, int E, int DIR>
__device__ __forceinline__ void fft_group(c2<T>* v, c2<T>* lds, int LS,
                                          const c2<T>* __restrict__ tw, int t) {
  constexpr int P = L / E;
  constexpr int R0 = first_radix(L, E);
  constexpr int Q = E / R0;
  static_assert(L % E == 0 && E % R0 == 0, "bad FFT factorisation");
  // pass 0: radix R0, Q butterflies per thread, operands already in registers
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    c2<T> b[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) b[r] = v[q + r * Q];
    dft_reg<T, DIR, R0>(b);
    if constexpr (L == R0) {
#pragma unroll
      for (int r = 0; r < R0; ++r) v[r] = b[r];
    } else {
      const int j = t + q * P;
#pragma unroll
      for (int r = 0; r < R0; ++r) lds[(j * R0 + r) * LS] = b[r];
    }
  }
  if constexpr (L > R0) {
    int Ns = R0;
#pragma unroll
    for (int pass = 1; pass < 8; ++pass) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < E; ++r) v[r] = lds[(t + r * P) * LS];
      const int k = t & (Ns - 1);
      // twiddle exp(DIR 2 pi i r k / (Ns E)) = tw[r k (2L / (Ns E))]
      const int step = (2 * L / E) / Ns * k;
#pragma unroll
      for (int r = 1; r < E; ++r) {
        const c2<T> w = tw[r * step];
        v[r] = DIR < 0 ? cmul(v[r], w) : cmulc(v[r], w);
      }
      dft_reg<T, DIR, E>(v);
      if (Ns * E == L) break;
      __syncthreads();
      const int idxD = (t / Ns) * Ns * E + k;
#pragma unroll
      for (int r = 0; r < E; ++r) lds[(idxD + r * Ns) * LS] = v[r];
      Ns *= E;
    }
  }
}

// Real row x[0 .. 2L) to its packed half spectrum.
// On entry v[q] = (x[2m], x[2m+1]) for m = t + q P.  On exit v[q] = X[m]
// for m >= 1 and v[q] = (X[0], X[L]) for m = 0 (DC and Nyquist are real).
// lds must hold L values (stride 1); tw: exp(-2 pi i k / (2L)), k < 2L.
template <typename T, int L, int E>
__device__ __forceinline__ void row_r2c(c2<T>* v, c2<T>* lds,
                                        const c2<T>* __restrict__ tw, int t) {
  constexpr int P = L / E;
  fft_group<T, L, E, -1>(v, lds, 1, tw, t);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) lds[t + q * P] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = t + q * P;
    const c2<T> z = v[q];
    if (m == 0) {
      v[q] = {z.x + z.y, z.x - z.y};
    } else {
      const c2<T> zc = lds[L - m];
      const T h = static_cast<T>(0.5);
      const c2<T> e = {h * (z.x + zc.x), h * (z.y - zc.y)};
      const c2<T> o = {h * (z.y + zc.y), -h * (z.x - zc.x)};
      v[q] = cadd(e, cmul(o, tw[m]));
    }
  }
}

// Packed half spectrum to the real row, scaled by 1/(2L) so that
// row_c2r(row_r2c(x)) = x.  On entry v[q] = packed X[m], m = t + q P; on exit
// v[q] = (x[2m], x[2m+1]).
template <typename T, int L, int E>
__device__ __forceinline__ void row_c2r(c2<T>* v, c2<T>* lds,
                                        const c2<T>* __restrict__ tw, int t) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) lds[t + q * P] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int m = t + q * P;
    const c2<T> X = v[q];
    if (m == 0) {
      v[q] = {X.x + X.y, X.x - X.y};
    } else {
      const c2<T> Xc = lds[L - m];
      const c2<T> a = {X.x + Xc.x, X.y - Xc.y};          // X + conj(Xc)
      const c2<T> d = {X.x - Xc.x, X.y + Xc.y};          // X - conj(Xc)
      const c2<T> b = cmulc(d, tw[m]);                    // times exp(+2 pi i m / 2L)
      v[q] = {a.x - b.y, a.y + b.x};                      // a + i b
    }
  }
  __syncthreads();
  fft_group<T, L, E, +1>(v, lds, 1, tw, t);
  const T sc = static_cast<T>(1.0 / (2.0 * L));
#pragma unroll
  for (int q = 0; q < E; ++q) v[q] = {v[q].x * sc, v[q].y * sc};
}

}  // namespace le
