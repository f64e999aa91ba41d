// cnn.hip -- BF16 MFMA kernels of the corrector network (see cnn.hpp).
#include "cnn.hpp"

#include <cstring>

#include "common.hpp"

namespace le {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kOffW[kCnnLayers] = {0, 608, 9856, 19104};
constexpr int kOffB[kCnnLayers] = {576, 9824, 19072, 19680};

constexpr int pad16(int k) { return (k + 15) / 16 * 16; }

// FP32 -> BF16, round to nearest even (the hardware conversion).
__device__ __forceinline__ uint16_t f2bf(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((unsigned)h) << 16); }

// c += a b for one 32x32x16 tile.  Lane l holds A[l % 32][8 (l / 32) + e],
// B[8 (l / 32) + e][l % 32] (e < 8) and C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
// in register r < 16.
__device__ __forceinline__ f32x16 mfma(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ int c_row(int r, int half) { return 8 * (r >> 2) + 4 * half + (r & 3); }

// Logistic function from the hardware base-2 exponential and reciprocal
// (about 1 ulp each: far below the BF16 rounding of the activations).
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

// Pixel p shifted by (dy, dx) on the periodic H x W grid (powers of two).
__device__ __forceinline__ int nb(int p, int dy, int dx, int H, int W, int lgW) {
  const int py = p >> lgW, px = p & (W - 1);
  return (((py + dy) & (H - 1)) << lgW) | ((px + dx) & (W - 1));
}

// ---------------------------------------------------------------- forward

// z[p][co] = b[co] + sum_{tap, ci} W[co][ci][tap] a[p + tap - (1,1)][ci];
// a_out = bf16(silu(z)) when ACT.  Block: 4 waves, each a 32-pixel tile.
template <int CIN, int COUT, bool ACT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ a_in,
                                                  const uint16_t* __restrict__ wt,
                                                  const float* __restrict__ bias,
                                                  float* __restrict__ z_out,
                                                  uint16_t* __restrict__ a_out, int H, int W,
                                                  int lgW) {
  constexpr int K = 9 * CIN, KP = pad16(K);
  const int lane = threadIdx.x & 63, half = lane >> 5, i = lane & 31;
  const int p0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
  const int p = p0 + i;
  f32x16 acc = {};
  // every operand of the tile is requested before the first product: at
  // 32 pixels per wavefront a 256^2 grid gives only ~2 wavefronts per SIMD,
  // too few to hide a load per k step
  constexpr int NKS = KP / 16;
  u16x8 av[NKS], bv[NKS];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    const int k0 = ks * 16 + half * 8;
    if constexpr (CIN % 8 == 0) {
      const int tap = k0 / CIN, ci0 = k0 % CIN;
      const int q = nb(p, tap / 3 - 1, tap % 3 - 1, H, W, lgW);
      av[ks] = *reinterpret_cast<const u16x8*>(a_in + (size_t)q * CIN + ci0);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        uint16_t v = 0;
        if (k < K) {
          const int tap = k / CIN, ci = k % CIN;
          v = a_in[(size_t)nb(p, tap / 3 - 1, tap % 3 - 1, H, W, lgW) * CIN + ci];
        }
        av[ks][e] = v;
      }
    }
    bv[ks] = *reinterpret_cast<const u16x8*>(wt + (size_t)i * KP + k0);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) acc = mfma(av[ks], bv[ks], acc);
  const int co = i;
  if (co < COUT) {
    const float bc = bias[co];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int pp = p0 + c_row(r, half);
      const float z = acc[r] + bc;
      z_out[(size_t)pp * COUT + co] = z;
      if constexpr (ACT) a_out[(size_t)pp * COUT + co] = f2bf(silu(z));
    }
  }
}

// ---------------------------------------------------------------- fused inference

// The corrected step runs the whole network over one 16 x 16 output tile per
// block.  The state planes of the tile and a 4-pixel halo (one pixel per 3x3
// layer) are read once; every intermediate activation stays in LDS as
// [pixel][kFS] BF16 (32 channels and 8 of padding: an 80-byte pixel stride
// puts the 16-byte reads of consecutive pixels on distinct banks).  Layer l
// computes the (22 - 2l)^2 pixels the next layer needs.  Each value is formed
// with the k order, products and roundings of the per-layer kernel above, so
// it equals the per-layer result bit for bit.
constexpr int kFT = 16, kFH = 4, kFR = kFT + 2 * kFH, kFS = 40, kFWaves = 8;

// One layer on the tile: input region SIN x SIN (LDS), output region
// (SIN - 2)^2, weights wt in LDS as [COUT][KP + 8] (the 8 of padding spread
// the rows over the banks).  Hidden layers write bf16(silu(z)) to LDS; the last writes z
// of both channels to z_out at the global pixels (tile origin gy0, gx0) and
// adds channel 0 into zs (FP64, lanes 0 and 32 of each wavefront).
template <int CIN, int SIN, bool LAST>
__device__ __forceinline__ void fused_layer(const uint16_t* __restrict__ in,
                                            uint16_t* __restrict__ out,
                                            const uint16_t* __restrict__ wt,
                                            const float* __restrict__ bias,
                                            float* __restrict__ z_out, int gy0, int gx0, int H,
                                            int W, int lgW, double& zs) {
  constexpr int COUT = LAST ? 2 : 32;
  constexpr int SOUT = SIN - 2, NP = SOUT * SOUT, NT = (NP + 31) / 32;
  constexpr int K = 9 * CIN, KP = pad16(K), NKS = KP / 16;
  const int lane = threadIdx.x & 63, half = lane >> 5, i = lane & 31;
  u16x8 bv[NKS];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks)
    bv[ks] = i < COUT ? *reinterpret_cast<const u16x8*>(wt + i * (KP + 8) + ks * 16 + half * 8)
                      : u16x8{};
  const float bc = i < COUT ? bias[i] : 0.f;
  for (int tile = (int)(threadIdx.x >> 6); tile < NT; tile += kFWaves) {
    // rows past the region repeat its last pixel; their results are dropped
    const int t = min(tile * 32 + i, NP - 1);
    const int oy = t / SOUT, ox = t - oy * SOUT;
    u16x8 av[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int k0 = ks * 16 + half * 8;
      if constexpr (CIN == 2) {
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const int k = k0 + e, tap = k / 2;
          unsigned v = 0;
          if (k < K) {
            const int q = (oy + tap / 3) * SIN + ox + tap % 3;
            v = *reinterpret_cast<const unsigned*>(in + 2 * q);
          }
          av[ks][e] = (uint16_t)(v & 0xffffu);
          av[ks][e + 1] = (uint16_t)(v >> 16);
        }
      } else {
        const int tap = k0 / CIN, ci0 = k0 % CIN;
        const int q = (oy + tap / 3) * SIN + ox + tap % 3;
        av[ks] = *reinterpret_cast<const u16x8*>(in + q * kFS + ci0);
      }
    }
    f32x16 acc = {};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) acc = mfma(av[ks], bv[ks], acc);
    if (i < COUT) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int tt = tile * 32 + c_row(r, half);
        if (tt < NP) {
          const float z = acc[r] + bc;
          if constexpr (!LAST) {
            out[tt * kFS + i] = f2bf(silu(z));
          } else {
            const int y = tt / SOUT, x = tt - y * SOUT;
            const int gp = (((gy0 + y) & (H - 1)) << lgW) | ((gx0 + x) & (W - 1));
            z_out[(size_t)gp * 2 + i] = z;
            if (i == 0) zs += (double)z;
          }
        }
      }
    }
  }
}

// Grid: (H / 16) (W / 16) blocks of 512 threads, tile b at rows
// 16 (b / (W / 16)), columns 16 (b % (W / 16)).  part[b] = the tile's FP64 sum
// of z[.][0] (fixed order).
template <typename T>
__global__ __launch_bounds__(kFWaves * 64) void k_net_fused(
    const T* __restrict__ phi, const T* __restrict__ om, float s0, float s1,
    const uint16_t* __restrict__ w0, const uint16_t* __restrict__ w1,
    const uint16_t* __restrict__ w2, const uint16_t* __restrict__ w3,
    const float* __restrict__ params, float* __restrict__ z3, double* __restrict__ part, int H,
    int W, int lgW) {
  __shared__ __align__(16) uint16_t in0[kFR * kFR * 2];
  __shared__ __align__(16) uint16_t buf_a[(kFR - 2) * (kFR - 2) * kFS];
  __shared__ __align__(16) uint16_t buf_b[(kFR - 4) * (kFR - 4) * kFS];
  constexpr int KP0 = pad16(18), KP = pad16(288);
  __shared__ __align__(16) uint16_t wl0[32 * (KP0 + 8)];
  __shared__ __align__(16) uint16_t wl1[32 * (KP + 8)];
  __shared__ __align__(16) uint16_t wl2[32 * (KP + 8)];
  __shared__ __align__(16) uint16_t wl3[2 * (KP + 8)];
  __shared__ double wsum[2 * kFWaves];
  const int tiles_x = W / kFT;
  const int ty0 = (int)(blockIdx.x / tiles_x) * kFT, tx0 = (int)(blockIdx.x % tiles_x) * kFT;
  // every global read of the block is issued before the first is used: the
  // 16-byte chunks of the four weight matrices (rows past the last layer's
  // two outputs are not needed) and the state planes of the region
  constexpr int C0 = 32 * KP0 / 8, C1 = 32 * KP / 8, C3 = 2 * KP / 8;
  constexpr int NCH = C0 + 2 * C1 + C3, NCH_T = (NCH + kFWaves * 64 - 1) / (kFWaves * 64);
  u16x8 wv[NCH_T];
#pragma unroll
  for (int u = 0; u < NCH_T; ++u) {
    int c = (int)threadIdx.x + u * kFWaves * 64;
    const uint16_t* src = nullptr;
    if (c < C0) {
      src = w0 + c * 8;
    } else if ((c -= C0) < C1) {
      src = w1 + c * 8;
    } else if ((c -= C1) < C1) {
      src = w2 + c * 8;
    } else if ((c -= C1) < C3) {
      src = w3 + c * 8;
    }
    wv[u] = src ? *reinterpret_cast<const u16x8*>(src) : u16x8{};
  }
  constexpr int NPX = kFR * kFR, NPX_T = (NPX + kFWaves * 64 - 1) / (kFWaves * 64);
  T xv[NPX_T][2];
#pragma unroll
  for (int u = 0; u < NPX_T; ++u) {
    const int q = (int)threadIdx.x + u * kFWaves * 64;
    const int ry = q / kFR, rx = q - ry * kFR;
    const int gp = (((ty0 - kFH + ry) & (H - 1)) << lgW) | ((tx0 - kFH + rx) & (W - 1));
    xv[u][0] = q < NPX ? phi[gp] : T(0);
    xv[u][1] = q < NPX ? om[gp] : T(0);
  }
#pragma unroll
  for (int u = 0; u < NCH_T; ++u) {
    int c = (int)threadIdx.x + u * kFWaves * 64;
    uint16_t* dst = nullptr;
    if (c < C0) {
      dst = wl0 + (c / (KP0 / 8)) * (KP0 + 8) + (c % (KP0 / 8)) * 8;
    } else if ((c -= C0) < C1) {
      dst = wl1 + (c / (KP / 8)) * (KP + 8) + (c % (KP / 8)) * 8;
    } else if ((c -= C1) < C1) {
      dst = wl2 + (c / (KP / 8)) * (KP + 8) + (c % (KP / 8)) * 8;
    } else if ((c -= C1) < C3) {
      dst = wl3 + (c / (KP / 8)) * (KP + 8) + (c % (KP / 8)) * 8;
    }
    if (dst) *reinterpret_cast<u16x8*>(dst) = wv[u];
  }
#pragma unroll
  for (int u = 0; u < NPX_T; ++u) {
    const int q = (int)threadIdx.x + u * kFWaves * 64;
    if (q < NPX) {
      in0[2 * q] = f2bf((float)xv[u][0] * s0);
      in0[2 * q + 1] = f2bf((float)xv[u][1] * s1);
    }
  }
  __syncthreads();
  double zs = 0.0;
  fused_layer<2, kFR, false>(in0, buf_a, wl0, params + kOffB[0], nullptr, 0, 0, H, W, lgW, zs);
  __syncthreads();
  fused_layer<32, kFR - 2, false>(buf_a, buf_b, wl1, params + kOffB[1], nullptr, 0, 0, H, W,
                                  lgW, zs);
  __syncthreads();
  fused_layer<32, kFR - 4, false>(buf_b, buf_a, wl2, params + kOffB[2], nullptr, 0, 0, H, W,
                                  lgW, zs);
  __syncthreads();
  fused_layer<32, kFR - 6, true>(buf_a, nullptr, wl3, params + kOffB[3], z3, ty0, tx0, H, W,
                                 lgW, zs);
  const int lane = threadIdx.x & 63;
  if ((lane & 31) == 0) wsum[(threadIdx.x >> 6) * 2 + (lane >> 5)] = zs;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 2 * kFWaves; ++k) t += wsum[k];
    part[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- input grad

// da[p][ci] = sum_{tap, co} W[co][ci][tap] dz[p + (1,1) - tap][co], then
// dzprev = da * silu'(zprev).  CIN = 32 (every layer with an input grad).
template <int COUT>
__global__ __launch_bounds__(256) void k_conv_dx(const float* __restrict__ dz,
                                                 const uint16_t* __restrict__ wx,
                                                 const float* __restrict__ zprev,
                                                 float* __restrict__ dzprev, int H, int W,
                                                 int lgW) {
  constexpr int CIN = 32, K = 9 * COUT, KP = pad16(K);
  const int lane = threadIdx.x & 63, half = lane >> 5, i = lane & 31;
  const int p0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
  const int p = p0 + i;
  f32x16 acc = {};
#pragma unroll 2
  for (int ks = 0; ks < KP / 16; ++ks) {
    const int k0 = ks * 16 + half * 8;
    u16x8 av;
    if constexpr (COUT % 8 == 0) {
      const int tap = k0 / COUT, co0 = k0 % COUT;
      const int q = nb(p, 1 - tap / 3, 1 - tap % 3, H, W, lgW);
      const float4 x0 = *reinterpret_cast<const float4*>(dz + (size_t)q * COUT + co0);
      const float4 x1 = *reinterpret_cast<const float4*>(dz + (size_t)q * COUT + co0 + 4);
      av[0] = f2bf(x0.x); av[1] = f2bf(x0.y); av[2] = f2bf(x0.z); av[3] = f2bf(x0.w);
      av[4] = f2bf(x1.x); av[5] = f2bf(x1.y); av[6] = f2bf(x1.z); av[7] = f2bf(x1.w);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        uint16_t v = 0;
        if (k < K) {
          const int tap = k / COUT, co = k % COUT;
          v = f2bf(dz[(size_t)nb(p, 1 - tap / 3, 1 - tap % 3, H, W, lgW) * COUT + co]);
        }
        av[e] = v;
      }
    }
    const u16x8 bv = *reinterpret_cast<const u16x8*>(wx + (size_t)i * KP + k0);
    acc = mfma(av, bv, acc);
  }
  const int ci = i;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const size_t e = (size_t)(p0 + c_row(r, half)) * CIN + ci;
    dzprev[e] = zprev ? acc[r] * silu_grad(zprev[e]) : acc[r];
  }
}

// ---------------------------------------------------------------- weight grad

// part[chunk][co][kcol] = sum_{p in chunk} dz[p][co] a[p + tap - (1,1)][ci],
// kcol = tap CIN + ci.  Block x: a chunk of kDwChunk pixels; each wave one
// 32-column tile (blockIdx.y * 4 + wave).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_dw(const float* __restrict__ dz,
                                                 const uint16_t* __restrict__ a,
                                                 float* __restrict__ part, int H, int W,
                                                 int lgW) {
  constexpr int NK = 9 * CIN, NKT = (NK + 31) / 32, NKP = NKT * 32;
  const int lane = threadIdx.x & 63, half = lane >> 5, i = lane & 31;
  const int ct = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (ct >= NKT) return;
  const int chunk = blockIdx.x;
  const int kcol = ct * 32 + i;
  const bool colok = kcol < NK;
  const int tap = colok ? kcol / CIN : 0, ci = colok ? kcol % CIN : 0;
  const int co = i;
  f32x16 acc = {};
  for (int ks = 0; ks < kDwChunk / 16; ++ks) {
    const int pc = chunk * kDwChunk + ks * 16 + half * 8;
    u16x8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      av[e] = co < COUT ? f2bf(dz[(size_t)(pc + e) * COUT + co]) : (uint16_t)0;
      bv[e] = colok ? a[(size_t)nb(pc + e, tap / 3 - 1, tap % 3 - 1, H, W, lgW) * CIN + ci]
                    : (uint16_t)0;
    }
    acc = mfma(av, bv, acc);
  }
  if (colok) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(r, half);
      if (row < COUT) part[((size_t)chunk * 32 + row) * NKP + kcol] = acc[r];
    }
  }
}

// grad[W(co, ci, tap)] += sum over chunks (in order) of part[chunk][co][kcol].
template <int CIN, int COUT>
__global__ void k_dw_reduce(const float* __restrict__ part, int nchunk, float* __restrict__ gw) {
  constexpr int NK = 9 * CIN, NKP = (NK + 31) / 32 * 32;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= COUT * NK) return;
  const int co = e / NK, kcol = e % NK;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[((size_t)c * 32 + co) * NKP + kcol];
  const int tap = kcol / CIN, ci = kcol % CIN;
  gw[(co * CIN + ci) * 9 + tap] += s;
}

// gb[co] += sum_p dz[p][co] (one block per channel, fixed-order tree).
__global__ __launch_bounds__(256) void k_db(const float* __restrict__ dz, int P, int cout,
                                            float* __restrict__ gb) {
  __shared__ float red[256];
  const int co = blockIdx.x;
  float s = 0.f;
  for (int p = threadIdx.x; p < P; p += 256) s += dz[(size_t)p * cout + co];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) gb[co] += red[0];
}

// ---------------------------------------------------------------- loss, I/O

// r = z4 * s_out; e = r - t; dz4 = scale * e * s_out; per-block sum of e^2.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ z4,
                                              const float* __restrict__ t, int P, float s2,
                                              float s3, float scale, float* __restrict__ dz4,
                                              double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int p = blockIdx.x * 256 + threadIdx.x; p < P; p += gridDim.x * 256) {
    const float e0 = z4[2 * (size_t)p] * s2 - t[p];
    const float e1 = z4[2 * (size_t)p + 1] * s3 - t[(size_t)P + p];
    dz4[2 * (size_t)p] = scale * e0 * s2;
    dz4[2 * (size_t)p + 1] = scale * e1 * s3;
    acc += (double)e0 * e0 + (double)e1 * e1;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[slot] += sum of n partials (one thread, fixed order).
// out[0] (+)= sum of part[0 .. n), n <= 1024, as one block's fixed-order
// tree; acc = 0 overwrites (no clearing launch needed, so the call may sit
// in a captured graph).  Launch with 256 threads.
__global__ __launch_bounds__(256) void k_sum_into(const double* __restrict__ part, int n,
                                                  double* __restrict__ out, int acc) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (acc ? out[0] : 0.0) + red[0];
}

template <typename T>
__global__ void k_pack_input(const T* __restrict__ x0, const T* __restrict__ x1, int P,
                             float s0, float s1, uint16_t* __restrict__ a0) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
    a0[2 * (size_t)p] = f2bf((float)x0[p] * s0);
    a0[2 * (size_t)p + 1] = f2bf((float)x1[p] * s1);
  }
}

__global__ void k_unpack_out(const float* __restrict__ z4, int P, float s2, float s3,
                             float* __restrict__ r) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
    r[p] = z4[2 * (size_t)p] * s2;
    r[(size_t)P + p] = z4[2 * (size_t)p + 1] * s3;
  }
}

// BF16 GEMM operands of every layer from the FP32 master weights.
__global__ void k_pack_weights(const float* __restrict__ params, uint16_t* wt0, uint16_t* wt1,
                               uint16_t* wt2, uint16_t* wt3, uint16_t* wx1, uint16_t* wx2,
                               uint16_t* wx3) {
  uint16_t* wt[4] = {wt0, wt1, wt2, wt3};
  uint16_t* wx[4] = {nullptr, wx1, wx2, wx3};
  const int l = blockIdx.y;
  const int cin = kCnnCin[l], cout = kCnnCout[l];
  const int kp = pad16(9 * cin), kpx = pad16(9 * cout);
  const float* Wl = params + kOffW[l];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 32 * kp; e += gridDim.x * blockDim.x) {
    const int j = e / kp, k = e % kp;
    float v = 0.f;
    if (j < cout && k < 9 * cin) v = Wl[(j * cin + k % cin) * 9 + k / cin];
    wt[l][e] = f2bf(v);
  }
  if (l == 0) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 32 * kpx;
       e += gridDim.x * blockDim.x) {
    const int ci = e / kpx, k = e % kpx;
    float v = 0.f;
    if (ci < cin && k < 9 * cout) v = Wl[((k % cout) * cin + ci) * 9 + k / cout];
    wx[l][e] = f2bf(v);
  }
}

// Adam with bias correction; the gradient is cleared for the next batch.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    g[e] = 0.f;
  }
}

__global__ void k_mfma_probe(const uint16_t* __restrict__ a, const uint16_t* __restrict__ b,
                             float* __restrict__ c) {
  const int lane = threadIdx.x, half = lane >> 5, i = lane & 31;
  u16x8 av, bv;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    av[e] = a[i * 16 + 8 * half + e];
    bv[e] = b[(8 * half + e) * 32 + i];
  }
  f32x16 acc = {};
  acc = mfma(av, bv, acc);
#pragma unroll
  for (int r = 0; r < 16; ++r) c[c_row(r, half) * 32 + i] = acc[r];
}

#define CNN_TRY(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return -3;       \
  } while (0)

int alloc_dev(void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess ? 0 : -2; }

void launch_fwd(const Net* n, int li, const uint16_t* a_in, float* z, uint16_t* a_out,
                hipStream_t st) {
  const dim3 g(n->P / 128), b(256);
  switch (li) {
    case 0:
      hipLaunchKernelGGL((k_conv_fwd<2, 32, true>), g, b, 0, st, a_in, n->wt[0],
                         n->params + kOffB[0], z, a_out, n->H, n->W, n->lgW);
      break;
    case 1:
      hipLaunchKernelGGL((k_conv_fwd<32, 32, true>), g, b, 0, st, a_in, n->wt[1],
                         n->params + kOffB[1], z, a_out, n->H, n->W, n->lgW);
      break;
    case 2:
      hipLaunchKernelGGL((k_conv_fwd<32, 32, true>), g, b, 0, st, a_in, n->wt[2],
                         n->params + kOffB[2], z, a_out, n->H, n->W, n->lgW);
      break;
    default:
      hipLaunchKernelGGL((k_conv_fwd<32, 2, false>), g, b, 0, st, a_in, n->wt[3],
                         n->params + kOffB[3], z, a_out, n->H, n->W, n->lgW);
      break;
  }
}

// Weight and bias gradients of layer li accumulated into n->grad; the input
// gradient (times silu' of zprev, when given) into dzprev for li > 0.
void launch_bwd(const Net* n, int li, const float* dz, const uint16_t* a_in, const float* zprev,
                float* dzprev, hipStream_t st) {
  const int nchunk = n->P / kDwChunk;
  const dim3 b(256);
  float* gw = n->grad + kOffW[li];
  float* gb = n->grad + kOffB[li];
  if (li == 0) {
    hipLaunchKernelGGL((k_conv_dw<2, 32>), dim3(nchunk, 1), b, 0, st, dz, a_in, n->part, n->H,
                       n->W, n->lgW);
    hipLaunchKernelGGL((k_dw_reduce<2, 32>), dim3((32 * 18 + 255) / 256), b, 0, st, n->part,
                       nchunk, gw);
  } else if (li < 3) {
    hipLaunchKernelGGL((k_conv_dw<32, 32>), dim3(nchunk, 3), b, 0, st, dz, a_in, n->part, n->H,
                       n->W, n->lgW);
    hipLaunchKernelGGL((k_dw_reduce<32, 32>), dim3((32 * 288 + 255) / 256), b, 0, st, n->part,
                       nchunk, gw);
  } else {
    hipLaunchKernelGGL((k_conv_dw<32, 2>), dim3(nchunk, 3), b, 0, st, dz, a_in, n->part, n->H,
                       n->W, n->lgW);
    hipLaunchKernelGGL((k_dw_reduce<32, 2>), dim3((2 * 288 + 255) / 256), b, 0, st, n->part,
                       nchunk, gw);
  }
  hipLaunchKernelGGL(k_db, dim3(kCnnCout[li]), b, 0, st, dz, n->P, kCnnCout[li], gb);
  if (li > 0 && dzprev) {
    const dim3 g(n->P / 128);
    if (li < 3)
      hipLaunchKernelGGL((k_conv_dx<32>), g, b, 0, st, dz, n->wx[li], zprev, dzprev, n->H, n->W,
                         n->lgW);
    else
      hipLaunchKernelGGL((k_conv_dx<2>), g, b, 0, st, dz, n->wx[li], zprev, dzprev, n->H, n->W,
                         n->lgW);
  }
}

void launch_pack_weights(Net* n, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_weights, dim3(16, 4), dim3(256), 0, st, n->params, n->wt[0],
                     n->wt[1], n->wt[2], n->wt[3], n->wx[1], n->wx[2], n->wx[3]);
}

}  // namespace

int net_create(Net* n, int H, int W, bool training) {
  if (H < 16 || W < 16 || (H & (H - 1)) || (W & (W - 1)) || (size_t)H * W % kDwChunk) return -1;
  n->H = H;
  n->W = W;
  n->lgW = 0;
  while ((1 << n->lgW) < W) ++n->lgW;
  n->P = H * W;
  const size_t P = (size_t)n->P;
  int rc = 0;
  rc = rc ? rc : alloc_dev((void**)&n->params, kCnnParams * sizeof(float));
  for (int l = 0; l < kCnnLayers; ++l) {
    rc = rc ? rc : alloc_dev((void**)&n->wt[l], 32 * (size_t)pad16(9 * kCnnCin[l]) * 2);
    if (l > 0) rc = rc ? rc : alloc_dev((void**)&n->wx[l], 32 * (size_t)pad16(9 * kCnnCout[l]) * 2);
    rc = rc ? rc : alloc_dev((void**)&n->act[l], P * kCnnCin[l] * 2);
    rc = rc ? rc : alloc_dev((void**)&n->z[l], P * kCnnCout[l] * sizeof(float));
  }
  // reduction scratch: the corrected step's P/256 per-tile partials; the
  // loss's 256 partials and its running sum at [1024]
  const size_t nred = (P / 256 > 2048 ? P / 256 : 2048);
  rc = rc ? rc : alloc_dev((void**)&n->red, nred * sizeof(double));
  if (training) {
    rc = rc ? rc : alloc_dev((void**)&n->grad, kCnnParams * sizeof(float));
    rc = rc ? rc : alloc_dev((void**)&n->m, kCnnParams * sizeof(float));
    rc = rc ? rc : alloc_dev((void**)&n->v, kCnnParams * sizeof(float));
    rc = rc ? rc : alloc_dev((void**)&n->dz[0], P * 32 * sizeof(float));
    rc = rc ? rc : alloc_dev((void**)&n->dz[1], P * 32 * sizeof(float));
    rc = rc ? rc : alloc_dev((void**)&n->part, (P / kDwChunk) * 32 * 288 * sizeof(float));
    if (!rc && (hipMemset(n->grad, 0, kCnnParams * 4) || hipMemset(n->m, 0, kCnnParams * 4) ||
                hipMemset(n->v, 0, kCnnParams * 4)))
      rc = -3;
  }
  if (rc) net_destroy(n);
  return rc;
}

void net_destroy(Net* n) {
  void* ps[] = {n->params, n->grad, n->m, n->v, n->dz[0], n->dz[1], n->part, n->red};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  for (int l = 0; l < kCnnLayers; ++l) {
    if (n->wt[l]) (void)hipFree(n->wt[l]);
    if (n->wx[l]) (void)hipFree(n->wx[l]);
    if (n->act[l]) (void)hipFree(n->act[l]);
    if (n->z[l]) (void)hipFree(n->z[l]);
  }
  *n = Net();
}

int net_set_params(Net* n, const float* host, hipStream_t st) {
  CNN_TRY(hipMemcpyAsync(n->params, host, kCnnParams * sizeof(float), hipMemcpyHostToDevice, st));
  launch_pack_weights(n, st);
  CNN_TRY(hipGetLastError());
  n->adam_t = 0;
  return 0;
}

int net_forward_planes(Net* n, const float* x, float* r, hipStream_t st) {
  const int P = n->P;
  hipLaunchKernelGGL((k_pack_input<float>), dim3(256), dim3(256), 0, st, x, x + P, P,
                     n->scales[0], n->scales[1], n->act[0]);
  for (int l = 0; l < kCnnLayers; ++l)
    launch_fwd(n, l, n->act[l], n->z[l], l < 3 ? n->act[l + 1] : nullptr, st);
  hipLaunchKernelGGL(k_unpack_out, dim3(256), dim3(256), 0, st, n->z[3], P, n->scales[2],
                     n->scales[3], r);
  CNN_TRY(hipGetLastError());
  return 0;
}

int net_grad(Net* n, const float* xs, const float* ts, int B, double* loss, hipStream_t st) {
  if (!n->grad || B < 1) return -1;
  const int P = n->P;
  const float scale = 2.0f / ((float)B * 2.0f * (float)P);
  CNN_TRY(hipMemsetAsync(n->red + 1024, 0, sizeof(double), st));
  for (int s = 0; s < B; ++s) {
    const float* x = xs + (size_t)s * 2 * P;
    const float* t = ts + (size_t)s * 2 * P;
    hipLaunchKernelGGL((k_pack_input<float>), dim3(256), dim3(256), 0, st, x, x + P, P,
                       n->scales[0], n->scales[1], n->act[0]);
    for (int l = 0; l < kCnnLayers; ++l)
      launch_fwd(n, l, n->act[l], n->z[l], l < 3 ? n->act[l + 1] : nullptr, st);
    hipLaunchKernelGGL(k_loss, dim3(256), dim3(256), 0, st, n->z[3], t, P, n->scales[2],
                       n->scales[3], scale, n->dz[0], n->red);
    hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, st, n->red, 256, n->red + 1024, 1);
    int cur = 0;
    for (int l = kCnnLayers - 1; l >= 0; --l) {
      launch_bwd(n, l, n->dz[cur], n->act[l], l > 0 ? n->z[l - 1] : nullptr,
                 l > 0 ? n->dz[cur ^ 1] : nullptr, st);
      cur ^= 1;
    }
  }
  CNN_TRY(hipGetLastError());
  double h = 0.0;
  CNN_TRY(hipMemcpyAsync(&h, n->red + 1024, sizeof(double), hipMemcpyDeviceToHost, st));
  CNN_TRY(hipStreamSynchronize(st));
  if (loss) *loss = h / ((double)B * 2.0 * P);
  return 0;
}

int net_adam(Net* n, float lr, float b1, float b2, float eps, hipStream_t st) {
  if (!n->grad) return -1;
  n->adam_t += 1;
  const float c1 = 1.f - powf(b1, (float)n->adam_t);
  const float c2 = 1.f - powf(b2, (float)n->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(80), dim3(256), 0, st, n->params, n->grad, n->m, n->v,
                     kCnnParams, lr, b1, b2, eps, c1, c2);
  launch_pack_weights(n, st);
  CNN_TRY(hipGetLastError());
  return 0;
}

int net_layer_fwd(Net* n, int li, const uint16_t* a_in, float* z_out, uint16_t* a_out,
                  hipStream_t st) {
  if (li < 0 || li >= kCnnLayers) return -1;
  launch_fwd(n, li, a_in, z_out, li < 3 ? a_out : nullptr, st);
  CNN_TRY(hipGetLastError());
  return 0;
}

int net_layer_bwd(Net* n, int li, const float* dz, const uint16_t* a_in, const float* zprev,
                  float* dzprev, float* dw, hipStream_t st) {
  if (li < 0 || li >= kCnnLayers || !n->grad) return -1;
  CNN_TRY(hipMemsetAsync(n->grad, 0, kCnnParams * sizeof(float), st));
  launch_bwd(n, li, dz, a_in, zprev, dzprev, st);
  CNN_TRY(hipGetLastError());
  if (dw) {
    const int len = kOffB[li] + kCnnCout[li] - kOffW[li];
    CNN_TRY(hipMemcpyAsync(dw, n->grad + kOffW[li], len * sizeof(float), hipMemcpyDeviceToDevice,
                           st));
  }
  return 0;
}

int net_tiles(const Net* n) { return (n->H / kFT) * (n->W / kFT); }

template <typename T>
int net_residual(Net* n, const T* phi, const T* omega, hipStream_t st) {
  hipLaunchKernelGGL((k_net_fused<T>), dim3(net_tiles(n)), dim3(kFWaves * 64), 0, st, phi, omega,
                     n->scales[0], n->scales[1], n->wt[0], n->wt[1], n->wt[2], n->wt[3],
                     n->params, n->z[3], n->red, n->H, n->W, n->lgW);
  CNN_TRY(hipGetLastError());
  return 0;
}
template int net_residual<double>(Net*, const double*, const double*, hipStream_t);
template int net_residual<float>(Net*, const float*, const float*, hipStream_t);

int mfma_probe(const uint16_t* a, const uint16_t* b, float* c, hipStream_t st) {
  uint16_t *da = nullptr, *db = nullptr;
  float* dc = nullptr;
  int rc = 0;
  rc = rc ? rc : alloc_dev((void**)&da, 32 * 16 * 2);
  rc = rc ? rc : alloc_dev((void**)&db, 16 * 32 * 2);
  rc = rc ? rc : alloc_dev((void**)&dc, 32 * 32 * 4);
  if (!rc && (hipMemcpyAsync(da, a, 32 * 16 * 2, hipMemcpyHostToDevice, st) ||
              hipMemcpyAsync(db, b, 16 * 32 * 2, hipMemcpyHostToDevice, st)))
    rc = -3;
  if (!rc) {
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, st, da, db, dc);
    if (hipGetLastError() || hipMemcpyAsync(c, dc, 32 * 32 * 4, hipMemcpyDeviceToHost, st) ||
        hipStreamSynchronize(st))
      rc = -3;
  }
  if (da) (void)hipFree(da);
  if (db) (void)hipFree(db);
  if (dc) (void)hipFree(dc);
  return rc;
}

}  // namespace le
