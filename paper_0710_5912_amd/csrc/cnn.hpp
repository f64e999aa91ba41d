// cnn.hpp -- the learned coarse-step corrector's network on gfx950.
//
// Four 3x3 convolutions 2 -> 32 -> 32 -> 32 -> 2, SiLU between them,
// circular padding (the cosheared frame is periodic).  Activations are BF16
// in pixel-major (NHWC) layout, pre-activations and gradients FP32.  Every
// convolution is an implicit GEMM on the BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation):
//   forward       M = pixels, N = Cout, K = 9 Cin
//   input grad    M = pixels, N = Cin,  K = 9 Cout
//   weight grad   M = Cout,   N = 9 Cin, K = pixels (split over pixel chunks,
//                 chunks summed in a fixed order)
// Master weights are FP32; the MFMA operands are BF16 copies repacked after
// every optimiser step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace le {

constexpr int kCnnLayers = 4;
constexpr int kCnnCin[kCnnLayers] = {2, 32, 32, 32};
constexpr int kCnnCout[kCnnLayers] = {32, 32, 32, 2};
constexpr int kCnnParams = 2 * 32 * 9 + 32 + 32 * 32 * 9 + 32 + 32 * 32 * 9 + 32 + 32 * 2 * 9 + 2;
constexpr int kDwChunk = 256;   // pixels per weight-gradient partial

// Network state on one device (weights and, when training, optimiser state
// and per-sample buffers for a grid of H x W pixels).
struct Net {
  int H = 0, W = 0, lgW = 0, P = 0;
  float* params = nullptr;      // FP32 master, kCnnParams
  float* grad = nullptr;        // FP32, kCnnParams
  float* m = nullptr;           // Adam moments
  float* v = nullptr;
  uint16_t* wt[kCnnLayers] = {};   // forward operands  [32][KP]
  uint16_t* wx[kCnnLayers] = {};   // input-grad operands [32][KPX] (layers 1..3)
  float scales[4] = {1.f, 1.f, 1.f, 1.f};   // in_phi, in_omega, out_phi, out_omega
  uint16_t* act[kCnnLayers] = {};  // inputs of each layer, BF16 [P][Cin]
  float* z[kCnnLayers] = {};       // pre-activations FP32 [P][Cout]
  float* dz[2] = {};               // gradient ping-pong FP32 [P][32]
  float* part = nullptr;           // weight-gradient partials
  double* red = nullptr;           // reduction scratch (FP64)
  int64_t adam_t = 0;
};

int net_create(Net* n, int H, int W, bool training);
void net_destroy(Net* n);
int net_set_params(Net* n, const float* host, hipStream_t st);
// Forward on FP32 planes x[2][P] (phi, omega) -> residual planes r[2][P].
int net_forward_planes(Net* n, const float* x, float* r, hipStream_t st);
// Gradient of the mean squared residual error, accumulated over a batch.
int net_grad(Net* n, const float* xs, const float* ts, int B, double* loss, hipStream_t st);
int net_adam(Net* n, float lr, float b1, float b2, float eps, hipStream_t st);

// Per-layer entry points (parity tests): layer li in 0..3.
int net_layer_fwd(Net* n, int li, const uint16_t* a_in, float* z_out, uint16_t* a_out,
                  hipStream_t st);
int net_layer_bwd(Net* n, int li, const float* dz, const uint16_t* a_in, const float* zprev,
                  float* dzprev, float* dw, hipStream_t st);

// Inference on the engine's fields (storage T, real planes): the network's
// output z ([P][2] FP32) into z_out() and the per-tile FP64 sums of z_phi
// (net_tiles() of them) into partials(); the update itself,
// phi += s2 (z_phi - mean) and omega += s3 z_omega, is left to the caller.
template <typename T>
int net_residual(Net* n, const T* phi, const T* omega, hipStream_t st);
int net_tiles(const Net* n);
inline const float* net_z_out(const Net* n) { return n->z[3]; }
inline const double* net_partials(const Net* n) { return n->red; }

// One 32x32x16 MFMA on a single wave: c = a (32x16) b (16x32), all row-major,
// BF16 bit patterns in, FP32 out (lane-layout check).
int mfma_probe(const uint16_t* a, const uint16_t* b, float* c, hipStream_t st);

}  // namespace le
