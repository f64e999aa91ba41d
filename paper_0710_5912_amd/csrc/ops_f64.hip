// Stage-kernel instantiations in FP64.
#include "ops_impl.hpp"

namespace le {

// Final fixed-order reduction over blocks.  out: OBS_NTOTAL sums, then nbins
// shell sums, then nbins shell weights.
__global__ void k_obs_final(const double* __restrict__ spart, int nsblk,
                            const double* __restrict__ rpart, int nrblk,
                            const double* __restrict__ bins, const double* __restrict__ counts,
                            int nbins, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < OBS_NSPEC) {
    double a = 0.0;
    for (int b = 0; b < nsblk; ++b) a += spart[(size_t)b * OBS_NSPEC + i];
    out[i] = a;
  } else if (i < OBS_NTOTAL) {
    const int k = i - OBS_NSPEC;
    double a = 0.0;
    for (int b = 0; b < nrblk; ++b) a += rpart[(size_t)b * 3 + k];
    out[i] = a;
  } else if (i < OBS_NTOTAL + nbins) {
    const int k = i - OBS_NTOTAL;
    double a = 0.0, w = 0.0;
    for (int b = 0; b < nsblk; ++b) {
      a += bins[(size_t)b * nbins + k];
      w += counts[(size_t)b * nbins + k];
    }
    out[OBS_NTOTAL + k] = a;
    out[OBS_NTOTAL + nbins + k] = w;
  }
}

bool get_ops_f64(int nx, int ny, Ops* ops) { return fill_ops<double>(nx, ny, ops); }

void launch_obs_final(const double* spart, int nsblk, const double* rpart, int nrblk,
                      const double* bins, const double* counts, int nbins, double* out,
                      hipStream_t st) {
  const int n = OBS_NTOTAL + nbins;
  hipLaunchKernelGGL(k_obs_final, dim3((n + 255) / 256), dim3(256), 0, st, spart, nsblk, rpart,
                     nrblk, bins, counts, nbins, out);
}

}  // namespace le
