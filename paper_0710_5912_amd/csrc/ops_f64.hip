// Stage-kernel instantiations in FP64.
#include "ops_impl.hpp"

namespace le {

// Final fixed-order reductions over blocks.
// k_obs_final_sums: block i < OBS_NTOTAL produces sum i (a strided sum per
// thread, a butterfly within each wavefront, the wavefront sums in order).
__global__ __launch_bounds__(256) void k_obs_final_sums(const double* __restrict__ spart,
                                                        int nsblk,
                                                        const double* __restrict__ rpart,
                                                        int nrblk, double* __restrict__ out) {
  __shared__ double red[4];
  const int i = blockIdx.x, tid = threadIdx.x;
  double a = 0.0;
  if (i < OBS_NSPEC) {
    for (int b = tid; b < nsblk; b += 256) a += spart[(size_t)b * OBS_NSPEC + i];
  } else {
    for (int b = tid; b < nrblk; b += 256) a += rpart[(size_t)b * 3 + (i - OBS_NSPEC)];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = a;
  __syncthreads();
  if (tid == 0) out[i] = ((red[0] + red[1]) + red[2]) + red[3];
}

// k_obs_shells_group: thread (k, g) sums shell k's partials over the spectral
// blocks g G .. g G + G - 1 in block order (consecutive threads read
// consecutive shells of a block's row: coalesced); k_obs_final_shells then
// sums the groups in order.  Fixed order throughout: deterministic.
constexpr int kShellGroup = 32;
__global__ __launch_bounds__(256) void k_obs_shells_group(const double* __restrict__ bins,
                                                          const double* __restrict__ counts,
                                                          int nsblk, int nbins,
                                                          double* __restrict__ gsum,
                                                          double* __restrict__ gcnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (k >= nbins) return;
  const int b0 = g * kShellGroup, b1 = min(b0 + kShellGroup, nsblk);
  double a = 0.0, w = 0.0;
  for (int b = b0; b < b1; ++b) {
    a += bins[(size_t)b * nbins + k];
    w += counts[(size_t)b * nbins + k];
  }
  gsum[(size_t)g * nbins + k] = a;
  gcnt[(size_t)g * nbins + k] = w;
}

__global__ __launch_bounds__(256) void k_obs_final_shells(const double* __restrict__ gsum,
                                                          const double* __restrict__ gcnt,
                                                          int ngroups, int nbins,
                                                          double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nbins) return;
  double a = 0.0, w = 0.0;
  for (int g = 0; g < ngroups; ++g) {
    a += gsum[(size_t)g * nbins + k];
    w += gcnt[(size_t)g * nbins + k];
  }
  out[OBS_NTOTAL + k] = a;
  out[OBS_NTOTAL + nbins + k] = w;
}

int obs_shell_groups(int nsblk) { return (nsblk + kShellGroup - 1) / kShellGroup; }

bool get_ops_f64(int nx, int ny, Ops* ops) { return fill_ops<double>(nx, ny, ops); }

void launch_obs_final(const double* spart, int nsblk, const double* rpart, int nrblk,
                      const double* bins, const double* counts, int nbins, double* gsum,
                      double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_obs_final_sums, dim3(OBS_NTOTAL), dim3(256), 0, st, spart, nsblk, rpart,
                     nrblk, out);
  if (nbins > 0) {
    const int ng = obs_shell_groups(nsblk);
    double* gcnt = gsum + (size_t)ng * nbins;
    hipLaunchKernelGGL(k_obs_shells_group, dim3((nbins + 255) / 256, ng), dim3(256), 0, st,
                       bins, counts, nsblk, nbins, gsum, gcnt);
    hipLaunchKernelGGL(k_obs_final_shells, dim3((nbins + 255) / 256), dim3(256), 0, st, gsum,
                       gcnt, ng, nbins, out);
  }
}

}  // namespace le
