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

// Pointer into device global memory.  The run descriptors hold plain
// pointers; giving them the global address space lets every access compile
// to global_load/store, which (unlike flat accesses) do not share the LDS
// wait counter, so LDS passes do not wait on outstanding memory traffic.
template <typename T>
using gp = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gp<T> to_global(const void* p) {
  return (gp<T>)(p);
}

// Whole-value load and store of a complex through a global pointer (one
// 8- or 16-byte access).
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ c2<T> ldg(gp<const c2<T>> p) {
  const vec2<T> v = *reinterpret_cast<gp<const vec2<T>>>(p);
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ c2<T> ldg(gp<c2<T>> p) {
  return ldg<T>(static_cast<gp<const c2<T>>>(p));
}
template <typename T>
__device__ __forceinline__ void stg(gp<c2<T>> p, c2<T> a) {
  *reinterpret_cast<gp<vec2<T>>>(p) = vec2<T>{a.x, a.y};
}

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

// Number of LDS passes (twiddled radix-E passes) of a length-L transform.
constexpr int fft_passes(int L, int E) {
  int n = 0;
  for (int Ns = first_radix(L, E); Ns < L; Ns *= E) ++n;
  return n;
}

// v[r] *= w^r (r = 1 .. E-1; conj(w)^r for DIR > 0).  The powers come from
// a product tree of depth <= 3 in FP64 (error ~1e-15), each rounded once to T.
// With v1 != nullptr (TWO) the same powers also multiply v1.
template <typename T, int DIR, int E, bool TWO = false>
__device__ __forceinline__ void twiddle_powers(c2<T>* v, c2<double> w1, c2<T>* v1 = nullptr) {
  auto app = [&](int r, c2<double> wd) {
    const c2<T> w = {static_cast<T>(wd.x), static_cast<T>(wd.y)};
    v[r] = DIR < 0 ? cmul(v[r], w) : cmulc(v[r], w);
    if constexpr (TWO) v1[r] = DIR < 0 ? cmul(v1[r], w) : cmulc(v1[r], w);
  };
  if constexpr (E >= 2) app(1, w1);
  if constexpr (E >= 4) {
    const c2<double> w2 = cmul(w1, w1);
    app(2, w2);
    app(3, cmul(w2, w1));
    if constexpr (E >= 8) {
      const c2<double> w4 = cmul(w2, w2);
      app(4, w4);
      app(5, cmul(w4, w1));
      app(6, cmul(w4, w2));
      app(7, cmul(w4, cmul(w2, w1)));
      if constexpr (E >= 16) {
        const c2<double> w8 = cmul(w4, w4);
        app(8, w8);
#pragma unroll
        for (int r = 9; r < 16; ++r) {
          // w^r = w^8 w^(r-8), r - 8 in 1 .. 7
          const int a = r - 8;
          c2<double> wa = (a & 4) ? w4 : c2<double>{1.0, 0.0};
          if (a & 2) wa = (a & 4) ? cmul(wa, w2) : w2;
          if (a & 1) wa = (a & 6) ? cmul(wa, w1) : w1;
          app(r, cmul(w8, wa));
        }
      }
    }
  }
}

// LDS slot of element i of a transform's exchange area, a permutation within
// aligned runs of elements (the area keeps its size) that spreads the strided
// accesses of the Stockham passes over the banks.  LDS serves 128 bytes per
// clock: 8 lanes of 16-byte (FP64) complex values or 16 lanes of 8-byte
// (FP32) ones.  FP64: the low three bits XORed by bits 3..5 and 4..6, which
// puts any 8 consecutive lanes of the passes' accesses (first-pass strides of
// 2 to 16 elements, later passes' groups of 2 to 256) and any 8 consecutive
// elements on distinct bank groups.  FP32: the low four bits XORed by the
// next four (lanes 16 or more elements apart).
template <typename T>
__device__ __forceinline__ int lds_slot(int i) {
  if constexpr (sizeof(T) == 8) return i ^ (((i >> 3) ^ (i >> 4)) & 7);
  return i ^ ((i >> 4) & 15);
}

// Length-L complex FFT by a group of P = L/E threads; thread t in [0, P).
// On entry v[q] = x[t + q P]; on exit v[q] = X[t + q P].
// lds: the group's LDS area, element i at lds[lds_slot<T>(i) * LS].  tw: the FP64 table
// exp(-2 pi i k / (2L)), k < 2L.  Pass p (stride Ns = R0 E^p) needs w^r,
// w = exp(-2 pi i k / (Ns E)), k = t mod Ns, r = 1 .. E-1: w is read from
// the table one pass ahead (its latency hides behind the pass before), the
// powers are formed in FP64 and rounded once to T.  Every thread of the
// block must call this with the same L (the passes contain
// __syncthreads()).  On return other threads may still read lds: barrier
// before reusing it.
// TWL: w from ltw, an LDS copy of the table's even entries ltw[i] =
// tw[2 i], i < L/E (fft_ltw_fill), instead of global memory, for transforms
// that follow stores of the same thread (a global read would wait for
// them: a wave's loads and stores share one counter).
template <int L, int E, int NT>
__device__ __forceinline__ void fft_ltw_fill(c2<double>* ltw, gp<const c2<double>> __restrict__ tw) {
  for (int i = threadIdx.x; i < L / E; i += NT) ltw[i] = ldg<double>(tw + 2 * i);
}
template <typename T, int L, int E, int DIR, bool TWL = false>
__device__ __forceinline__ void fft_group(c2<T>* v, c2<T>* lds, int LS,
                                          gp<const c2<double>> __restrict__ tw, int t,
                                          const c2<double>* ltw = nullptr) {
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
      for (int r = 0; r < R0; ++r) lds[lds_slot<T>(j * R0 + r) * LS] = b[r];
    }
  }
  if constexpr (L > R0) {
    constexpr int NP = fft_passes(L, E);
    // entry (2L/E)/Ns (t mod Ns): even, below 2L/E, as Ns <= L/E
    auto tw_of = [&](int Ns) {
      const int k = (2 * L / E) / Ns * (t & (Ns - 1));
      if constexpr (TWL)
        return ltw[k >> 1];
      else
        return ldg<double>(tw + k);
    };
    c2<double> wn = tw_of(R0);
    int Ns = R0;
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const c2<double> w = wn;
      if (pass + 1 < NP) wn = tw_of(Ns * E);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < E; ++r) v[r] = lds[lds_slot<T>(t + r * P) * LS];
      twiddle_powers<T, DIR, E>(v, w);
      dft_reg<T, DIR, E>(v);
      if (pass + 1 == NP) break;
      __syncthreads();
      const int k = t & (Ns - 1);
      const int idxD = (t / Ns) * Ns * E + k;
#pragma unroll
      for (int r = 0; r < E; ++r) lds[lds_slot<T>(idxD + r * Ns) * LS] = v[r];
      Ns *= E;
    }
  }
}

// Two independent length-L transforms (v0 in lds0, v1 in lds1) by the same
// group, pass by pass: each pass of both shares one pair of barriers, and
// each result equals fft_group's for that array alone (same operations).
template <typename T, int L, int E, int DIR>
__device__ __forceinline__ void fft_group2(c2<T>* v0, c2<T>* v1, c2<T>* lds0, c2<T>* lds1,
                                           int LS, gp<const c2<double>> __restrict__ tw,
                                           int t) {
  constexpr int P = L / E;
  constexpr int R0 = first_radix(L, E);
  constexpr int Q = E / R0;
  static_assert(L % E == 0 && E % R0 == 0, "bad FFT factorisation");
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    c2<T> b0[R0], b1[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      b0[r] = v0[q + r * Q];
      b1[r] = v1[q + r * Q];
    }
    dft_reg<T, DIR, R0>(b0);
    dft_reg<T, DIR, R0>(b1);
    if constexpr (L == R0) {
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        v0[r] = b0[r];
        v1[r] = b1[r];
      }
    } else {
      const int j = t + q * P;
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        lds0[lds_slot<T>(j * R0 + r) * LS] = b0[r];
        lds1[lds_slot<T>(j * R0 + r) * LS] = b1[r];
      }
    }
  }
  if constexpr (L > R0) {
    constexpr int NP = fft_passes(L, E);
    auto tw_of = [&](int Ns) { return ldg<double>(tw + (2 * L / E) / Ns * (t & (Ns - 1))); };
    c2<double> wn = tw_of(R0);
    int Ns = R0;
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const c2<double> w = wn;
      if (pass + 1 < NP) wn = tw_of(Ns * E);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < E; ++r) {
        v0[r] = lds0[lds_slot<T>(t + r * P) * LS];
        v1[r] = lds1[lds_slot<T>(t + r * P) * LS];
      }
      twiddle_powers<T, DIR, E, true>(v0, w, v1);
      dft_reg<T, DIR, E>(v0);
      dft_reg<T, DIR, E>(v1);
      if (pass + 1 == NP) break;
      __syncthreads();
      const int k = t & (Ns - 1);
      const int idxD = (t / Ns) * Ns * E + k;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        lds0[lds_slot<T>(idxD + r * Ns) * LS] = v0[r];
        lds1[lds_slot<T>(idxD + r * Ns) * LS] = v1[r];
      }
      Ns *= E;
    }
  }
}

// exp(-i pi q / E) for q < E, E a power of two up to 16 (cos and sin of
// multiples of pi/16, correctly rounded).  The table entry m = t + q L/E of
// exp(-2 pi i m / (2L)) is tw[t] times this, so a transform thread that
// needs the E entries t + q L/E reads one and forms the others in FP64.
template <int E>
__device__ __forceinline__ c2<double> root_step(int q) {
  static_assert(E >= 1 && E <= 16 && (E & (E - 1)) == 0, "E: power of two up to 16");
  constexpr double c[9] = {1.0,
                           0.98078528040323044913,
                           0.92387953251128675613,
                           0.83146961230254523708,
                           0.70710678118654752440,
                           0.55557023301960222474,
                           0.38268343236508977173,
                           0.19509032201612826785,
                           0.0};
  const int k = q * (16 / E);  // angle k pi / 16, k < 16
  // cos(k pi/16) = c[k] (k <= 8) or -c[16 - k]; sin(k pi/16) = c[8 - k] or c[k - 8]
  const double cs = k <= 8 ? c[k] : -c[16 - k];
  const double sn = k <= 8 ? c[8 - k] : c[k - 8];
  return {cs, -sn};
}

// Real row x[0 .. 2L) to its packed half spectrum.
// On entry v[q] = (x[2m], x[2m+1]) for m = t + q P.  On exit v[q] = X[m]
// for m >= 1 and v[q] = (X[0], X[L]) for m = 0 (DC and Nyquist are real).
// lds must hold L values (stride 1); tw: the FP64 table exp(-2 pi i k / (2L)),
// k < 2L.
template <typename T, int L, int E>
__device__ __forceinline__ void row_r2c(c2<T>* v, c2<T>* lds, gp<const c2<double>> __restrict__ tw,
                                        int t) {
  constexpr int P = L / E;
  fft_group<T, L, E, -1>(v, lds, 1, tw, t);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) lds[t + q * P] = v[q];
  __syncthreads();
  const c2<double> w0 = ldg<double>(tw + t);  // tw[t + q P] = w0 root_step<E>(q)
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
      const c2<double> wd = q == 0 ? w0 : cmul(w0, root_step<E>(q));
      v[q] = cadd(e, cmul(o, c2<T>{static_cast<T>(wd.x), static_cast<T>(wd.y)}));
    }
  }
}

// The table entries tw[m], m <= L, as products of two small LDS tables (the
// low entries tw[0 .. LO) and every LO-th entry), for loops that store to
// global memory: a table read from global memory there would wait for the
// loop's earlier stores (a wave's loads and stores share one counter), an
// LDS read does not.  tw_tab_fill (every thread of the block) before a
// barrier, then tw_tab.
template <int L>
struct TwTab {
  static constexpr int LO = L < 64 ? L : 64, NH = L / LO + 1, N = LO + NH;
};
template <int L, int NT>
__device__ __forceinline__ void tw_tab_fill(c2<double>* tab, gp<const c2<double>> __restrict__ tw) {
  using W = TwTab<L>;
  for (int i = threadIdx.x; i < W::N; i += NT)
    tab[i] = ldg<double>(tw + (i < W::LO ? i : (i - W::LO) * W::LO));
}
template <int L>
__device__ __forceinline__ c2<double> tw_tab(const c2<double>* tab, int m) {
  using W = TwTab<L>;
  return cmul(tab[m % W::LO], tab[W::LO + m / W::LO]);
}

// row_r2c split for callers that store the spectrum from LDS: row_r2c_z
// leaves the complex DFT z of the packed row in lds[0 .. L) (stride 1;
// visible to the block after its next barrier), and r2c_mode forms mode m
// (0 .. L) of the half spectrum from it with row_r2c's arithmetic, m = 0 and
// m = L being the real DC and Nyquist values, the twiddle from the LDS
// tables of tw_tab.  This saves the LDS pass that stages row_r2c's result
// for the stores.
template <typename T, int L, int E>
__device__ __forceinline__ void row_r2c_z(c2<T>* v, c2<T>* lds,
                                          gp<const c2<double>> __restrict__ tw, int t) {
  constexpr int P = L / E;
  fft_group<T, L, E, -1>(v, lds, 1, tw, t);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) lds[t + q * P] = v[q];
}
template <typename T, int L>
__device__ __forceinline__ c2<T> r2c_mode(const c2<T>* lds, const c2<double>* wtab, int m) {
  if (m == 0 || m == L) {
    const c2<T> z = lds[0];
    return m == 0 ? c2<T>{z.x + z.y, T(0)} : c2<T>{z.x - z.y, T(0)};
  }
  const c2<T> z = lds[m], zc = lds[L - m];
  const T h = static_cast<T>(0.5);
  const c2<T> e = {h * (z.x + zc.x), h * (z.y - zc.y)};
  const c2<T> o = {h * (z.y + zc.y), -h * (z.x - zc.x)};
  const c2<double> wd = tw_tab<L>(wtab, m);
  return cadd(e, cmul(o, c2<T>{static_cast<T>(wd.x), static_cast<T>(wd.y)}));
}

// Packed half spectrum to the real row, scaled by 1/(2L) so that
// row_c2r(row_r2c(x)) = x.  On entry v[q] = packed X[m], m = t + q P; on exit
// v[q] = (x[2m], x[2m+1]).
template <typename T, int L, int E>
__device__ __forceinline__ void row_c2r(c2<T>* v, c2<T>* lds, gp<const c2<double>> __restrict__ tw,
                                        int t) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) lds[t + q * P] = v[q];
  __syncthreads();
  const c2<double> w0 = ldg<double>(tw + t);  // tw[t + q P] = w0 root_step<E>(q)
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
      const c2<double> wd = q == 0 ? w0 : cmul(w0, root_step<E>(q));
      const c2<T> b = cmulc(d, c2<T>{static_cast<T>(wd.x), static_cast<T>(wd.y)});                   // times exp(+2 pi i m / 2L)
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
