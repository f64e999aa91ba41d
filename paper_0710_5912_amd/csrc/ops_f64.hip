// Stage-kernel instantiations in FP64.
#include "ops_impl.hpp"

namespace le {

// Final fixed-order reduction over blocks; block i produces output i.
// out: OBS_NTOTAL sums, then nbins shell sums, then nbins shell weights.
__global__ __launch_bounds__(256) void k_obs_final(const double* __restrict__ spart, int nsblk,
                                                   const double* __restrict__ rpart, int nrblk,
                                                   const double* __restrict__ bins,
                                                   const double* __restrict__ counts, int nbins,
                                                   double* __restrict__ out) {
  __shared__ double red[2][256];
  const int i = blockIdx.x, tid = threadIdx.x;
  double a = 0.0, w = 0.0;
  if (i < OBS_NSPEC) {
    for (int b = tid; b < nsblk; b += 256) a += spart[(size_t)b * OBS_NSPEC + i];
  } else if (i < OBS_NTOTAL) {
    for (int b = tid; b < nrblk; b += 256) a += rpart[(size_t)b * 3 + (i - OBS_NSPEC)];
  } else {
    const int k = i - OBS_NTOTAL;
    for (int b = tid; b < nsblk; b += 256) {
      a += bins[(size_t)b * nbins + k];
      w += counts[(size_t)b * nbins + k];
    }
  }
  red[0][tid] = a;
  red[1][tid] = w;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] += red[1][tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (i < OBS_NTOTAL) {
      out[i] = red[0][0];
    } else {
      out[i] = red[0][0];
      out[i + nbins] = red[1][0];
    }
  }
}

bool get_ops_f64(int nx, int ny, Ops* ops) { return fill_ops<double>(nx, ny, ops); }

void launch_obs_final(const double* spart, int nsblk, const double* rpart, int nrblk,
                      const double* bins, const double* counts, int nbins, double* out,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_obs_final, dim3(OBS_NTOTAL + nbins), dim3(256), 0, st, spart, nsblk,
                     rpart, nrblk, bins, counts, nbins, out);
}

}  // namespace le
