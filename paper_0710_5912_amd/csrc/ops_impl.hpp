// ops_impl.hpp -- template launchers behind the Ops table (included once per
// precision by ops_f64.hip / ops_f32.hip).
#pragma once

#include "ops.hpp"
#include "stages.hpp"


namespace le {

// Row transform shapes (variant, a tuning choice): 0 = 8 values per thread,
// 1 = 4 (twice the threads per row: shorter chains for latency-bound grids),
// 2 and 3 = the same with a quarter of the rows per block (more blocks for
// small grids), 4 and 5 = 8 values per thread, at least four or two rows
// per block, the spectra staged through LDS and stored (loaded) tile by
// tile.
template <typename T, int L>
struct RowLaunch {
  using C = RowCfg<L>;
  static dim3 grid(int ny, int fields, int nruns) {
    return dim3((ny + C::G - 1) / C::G, fields, nruns);
  }
  template <int E, int GD>
  static void r2c_shape(const Run* runs, int nruns, int ny, const R2cJobs& jobs, int njobs,
                        hipStream_t st) {
    using CE = RowCfg<L, E, GD>;
    hipLaunchKernelGGL((k_row_r2c<T, L, E, GD>), dim3((ny + CE::G - 1) / CE::G, njobs, nruns),
                       dim3(CE::THREADS), 0, st, runs, jobs);
  }
  template <int E, int GD>
  static void c2r_shape(const Run* runs, int nruns, int ny, int bin0, int bout0, int bin1,
                        int bout1, int nfields, hipStream_t st) {
    using CE = RowCfg<L, E, GD>;
    hipLaunchKernelGGL((k_row_c2r<T, L, E, GD>),
                       dim3((ny + CE::G - 1) / CE::G, nfields, nruns), dim3(CE::THREADS), 0, st,
                       runs, bin0, bout0, bin1, bout1);
  }
  static constexpr int E4 = L >= 16 ? 4 : row_elems(L);
  // the LDS-staged shapes: 8 values per thread, at least RB0 rows per block
  template <int RB0>
  static void r2c_t(const Run* runs, int nruns, int ny, const R2cJobs& jobs, int njobs,
                    hipStream_t st) {
    constexpr int E = row_elems(L);
    using CE = RowT<L, E, RB0>;
    static_assert(CE::OK, "staged row shape does not fit");
    hipLaunchKernelGGL((k_row_r2c_t<T, L, E, RB0>),
                       dim3((ny + CE::RB - 1) / CE::RB, njobs, nruns), dim3(CE::THREADS), 0, st,
                       runs, jobs);
  }
  template <int RB0>
  static void c2r_t(const Run* runs, int nruns, int ny, int bin0, int bout0, int bin1,
                    int bout1, int nfields, hipStream_t st) {
    constexpr int E = row_elems(L);
    using CE = RowT<L, E, RB0>;
    static_assert(CE::OK, "staged row shape does not fit");
    hipLaunchKernelGGL((k_row_c2r_t<T, L, E, RB0>),
                       dim3((ny + CE::RB - 1) / CE::RB, nfields, nruns), dim3(CE::THREADS), 0,
                       st, runs, bin0, bout0, bin1, bout1);
  }
  static void r2c_jobs(const Run* runs, int nruns, int ny, const R2cJobs& jobs, int njobs,
                       int variant, hipStream_t st) {
    switch (variant) {
      case 1: r2c_shape<E4, 1>(runs, nruns, ny, jobs, njobs, st); break;
      case 2: r2c_shape<row_elems(L), 4>(runs, nruns, ny, jobs, njobs, st); break;
      case 3: r2c_shape<E4, 4>(runs, nruns, ny, jobs, njobs, st); break;
      case 4: r2c_t<4>(runs, nruns, ny, jobs, njobs, st); break;
      case 5: r2c_t<2>(runs, nruns, ny, jobs, njobs, st); break;
      default: r2c_shape<row_elems(L), 1>(runs, nruns, ny, jobs, njobs, st); break;
    }
  }
  static void r2c(const Run* runs, int nruns, int ny, int bin, int bout, int variant,
                  hipStream_t st) {
    R2cJobs jobs{{{bin, bout, 2 * L}, {}, {}}};
    r2c_jobs(runs, nruns, ny, jobs, 1, variant, st);
  }
  static void r2c_n(const Run* runs, int nruns, int ny, const int* bins, const int* bouts,
                    int njobs, int variant, hipStream_t st) {
    R2cJobs jobs{};
    for (int k = 0; k < njobs && k < 3; ++k) jobs.j[k] = {bins[k], bouts[k], 2 * L};
    r2c_jobs(runs, nruns, ny, jobs, njobs < 3 ? njobs : 3, variant, st);
  }
  template <int E, int GD>
  static void r2c_corr_shape(const Run* runs, int ny, const CorrArgs& ca, hipStream_t st) {
    using CE = RowCfg<L, E, GD>;
    hipLaunchKernelGGL((k_row_r2c_corr<T, L, E, GD>), dim3((ny + CE::G - 1) / CE::G),
                       dim3(CE::THREADS), 0, st, runs, ca);
  }
  static void r2c_corr(const Run* runs, int ny, const CorrArgs& ca, int variant, hipStream_t st) {
    switch (variant) {
      case 1: r2c_corr_shape<E4, 1>(runs, ny, ca, st); break;
      case 2: r2c_corr_shape<row_elems(L), 4>(runs, ny, ca, st); break;
      case 3: r2c_corr_shape<E4, 4>(runs, ny, ca, st); break;
      default: r2c_corr_shape<row_elems(L), 1>(runs, ny, ca, st); break;
    }
  }
  static void c2r(const Run* runs, int nruns, int ny, int bin0, int bout0, int bin1, int bout1,
                  int nfields, int variant, hipStream_t st) {
    switch (variant) {
      case 1: c2r_shape<E4, 1>(runs, nruns, ny, bin0, bout0, bin1, bout1, nfields, st); break;
      case 2:
        c2r_shape<row_elems(L), 4>(runs, nruns, ny, bin0, bout0, bin1, bout1, nfields, st);
        break;
      case 3: c2r_shape<E4, 4>(runs, nruns, ny, bin0, bout0, bin1, bout1, nfields, st); break;
      case 4: c2r_t<4>(runs, nruns, ny, bin0, bout0, bin1, bout1, nfields, st); break;
      case 5: c2r_t<2>(runs, nruns, ny, bin0, bout0, bin1, bout1, nfields, st); break;
      default:
        c2r_shape<row_elems(L), 1>(runs, nruns, ny, bin0, bout0, bin1, bout1, nfields, st);
        break;
    }
  }
  // the r = 1 (square cell grid, nx = ny) form when it applies
  static void bracket(const Run* runs, int nruns, int ny, const StepArgs* sa, const Jobs& jobs,
                      int njobs, hipStream_t st) {
    if (ny == 2 * L)
      hipLaunchKernelGGL((k_bracket<T, L, true>), grid(ny, njobs, nruns), dim3(C::THREADS), 0,
                         st, runs, sa, jobs);
    else
      hipLaunchKernelGGL((k_bracket<T, L, false>), grid(ny, njobs, nruns), dim3(C::THREADS), 0,
                         st, runs, sa, jobs);
  }
  template <int SEG>
  static void strip_fft(const Run* runs, const StepArgs* sa, int ny, dim3 gf, int rows,
                        bool inertial, hipStream_t st) {
    constexpr int NX = 2 * L;
    if (ny == NX)
      hipLaunchKernelGGL((k_adv_strip_fft<T, NX, true, SEG>), gf, dim3(L / SEG), 0, st, runs,
                         sa, rows, inertial ? 1 : 0);
    else
      hipLaunchKernelGGL((k_adv_strip_fft<T, NX, false, SEG>), gf, dim3(L / SEG), 0, st, runs,
                         sa, rows, inertial ? 1 : 0);
  }
  // The batched one-kernel forms (advect, and mu_source on square cells):
  // NR rows per batch, EF values per thread in the row transforms.  Returns
  // false where the shape does not apply to this row length (fewer than one
  // wavefront per transform group, or a row outside nx 512 .. 4096).
  template <int NR, int EF>
  static bool batch_shape(bool mu, const Run* runs, const StepArgs* sa, int ny, dim3 gb,
                          int rows, bool inertial, hipStream_t st) {
    constexpr int NX = 2 * L;
    if constexpr (adv_batch_ok(NX) && NR * (NX / 2 / EF) >= 64) {
      using CB = AdvBatch<T, NX, NR, EF>;
      // FP64 advection: one block per output field (kAdvSplit)
      const dim3 ga(kAdvSplit<T> ? (inertial ? 3 : 2) : 1, gb.y, gb.z);
      if (mu)
        hipLaunchKernelGGL((k_mug_batch<T, NX, NR, EF>), gb, dim3(CB::TPB), 0, st, runs, sa,
                           rows);
      else if (ny == NX)
        hipLaunchKernelGGL((k_adv_batch<T, NX, true, NR, EF>), ga, dim3(CB::TPB), 0, st, runs,
                           sa, rows, inertial ? 1 : 0);
      else
        hipLaunchKernelGGL((k_adv_batch<T, NX, false, NR, EF>), ga, dim3(CB::TPB), 0, st,
                           runs, sa, rows, inertial ? 1 : 0);
      return true;
    }
    return false;
  }
  // variant kAdvBatch + k (four rows per batch, 16 values per thread),
  // kAdvBatch2 + k (two, 8), kAdvBatch3 + k (two, 16); k rows per block.
  // False (and *rows set) where the shape does not apply: the caller falls
  // back to the two-kernel strip over k rows.
  static bool batch(bool mu, const Run* runs, int nruns, const StepArgs* sa, int ny,
                    int variant, bool inertial, hipStream_t st, int* rows) {
    const int base = variant >= kAdvBatch3   ? kAdvBatch3
                     : variant >= kAdvBatch2 ? kAdvBatch2
                                             : kAdvBatch;
    *rows = variant - base > 0 ? variant - base : 1;
    const dim3 gb(1, (ny + *rows - 1) / *rows, nruns);
    switch (base) {
      case kAdvBatch3: return batch_shape<2, 16>(mu, runs, sa, ny, gb, *rows, inertial, st);
      case kAdvBatch2: return batch_shape<2, 8>(mu, runs, sa, ny, gb, *rows, inertial, st);
      default: return batch_shape<4, 16>(mu, runs, sa, ny, gb, *rows, inertial, st);
    }
  }
  // variant 0: the fused bracket kernel (stencil and row transform per
  // block); variant 0 < k < kStripFft: the strip stencil over k-row strips
  // into the spectral buffers, then in-place row transforms; variant
  // kStripFft + k (two x pairs per thread) and kStripFft1 + k (one): strip
  // stencil and row transforms in one kernel over k-row strips (nx 256 ..
  // 1024; elsewhere the two-kernel form)
  static void advect(const Run* runs, int nruns, int ny, const StepArgs* sa, bool inertial,
                     int variant, int row_variant, hipStream_t st) {
    if (variant <= 0) {
      Jobs jobs{{{JOB_ADVECT, B_PHI, B_PS_R, B_PHIH},
                 {JOB_CUBE, B_PHI, B_PS_R, B_FH},
                 {JOB_ADVECT, B_OM_R, B_PS_R, B_OMH}}};
      bracket(runs, nruns, ny, sa, jobs, inertial ? 3 : 2, st);
      return;
    }
    constexpr int NX = 2 * L, TPB = strip_threads(NX);
    if (variant == kAdvUpwind) {
      const dim3 gu((NX / 2 + 255) / 256, ny, nruns);
      hipLaunchKernelGGL((k_adv_upwind<T, NX>), gu, dim3(NX / 2 < 256 ? NX / 2 : 256), 0, st,
                         runs, sa, inertial ? 1 : 0);
      R2cJobs jobs{{{B_TMP, B_PHIH, NX}, {B_R1, B_FH, NX}, {B_R2, B_OMH, NX}}};
      r2c_jobs(runs, nruns, ny, jobs, inertial ? 3 : 2, row_variant, st);
      return;
    }
    if (variant >= kAdvBatch) {
      int rows = 0;
      if (batch(false, runs, nruns, sa, ny, variant, inertial, st, &rows)) return;
      variant = rows;  // shapes outside the batched kernel's range: the two-kernel form
    }
    if (variant >= kStripFft) {
      const bool two = variant < kStripFft1;
      const int rows = variant - (two ? kStripFft : kStripFft1);
      if constexpr (adv_strip_fft_ok(NX)) {
        const dim3 gf(1, (ny + rows - 1) / rows, nruns);
        if (two)
          strip_fft<2>(runs, sa, ny, gf, rows, inertial, st);
        else
          strip_fft<1>(runs, sa, ny, gf, rows, inertial, st);
        return;
      }
      variant = rows;  // grids outside the fused kernel's range: the two-kernel form
    }
    const dim3 gs(NX / 2 / TPB, (ny + variant - 1) / variant, nruns);
    if (ny == NX)
      hipLaunchKernelGGL((k_adv_strip<T, NX, true>), gs, dim3(TPB), 0, st, runs, sa, variant,
                         inertial ? 1 : 0);
    else
      hipLaunchKernelGGL((k_adv_strip<T, NX, false>), gs, dim3(TPB), 0, st, runs, sa, variant,
                         inertial ? 1 : 0);
    R2cJobs jobs{{{B_TMP, B_PHIH, NX}, {B_R1, B_FH, NX}, {B_R2, B_OMH, NX}}};
    r2c_jobs(runs, nruns, ny, jobs, inertial ? 3 : 2, row_variant, st);
  }
  // variant 0: mu into the real scratch field, then the source bracket and
  // its row transform; variant 0 < k < kStripFft (square cells only): the
  // strip stencil (mu in registers) over k-row strips into B_GH, then its
  // in-place row transform; kStripFft + k: the same strips with the row
  // transforms in one kernel (nx 256 .. 2048; elsewhere the two-kernel form);
  // kAdvBatch + k .. kAdvBatch1 + k: the batched one-kernel forms over k-row
  // strips (as for advect; elsewhere the two-kernel form)
  static void mu_source(const Run* runs, int nruns, int ny, const StepArgs* sa, int variant,
                        int row_variant, hipStream_t st) {
    constexpr int NX = 2 * L, TPB = strip_threads(NX);
    if (variant <= 0 || ny != NX) {
      hipLaunchKernelGGL((k_mu<T, L>), grid(ny, 1, nruns), dim3(C::THREADS), 0, st, runs, sa,
                         (int)B_PHI, (int)B_TMP);
      Jobs jobs{{{JOB_SOURCE, B_PHI, B_TMP, B_GH}, {}, {}}};
      bracket(runs, nruns, ny, sa, jobs, 1, st);
      return;
    }
    if (variant >= kAdvBatch) {
      int rows = 0;
      if (batch(true, runs, nruns, sa, ny, variant, false, st, &rows)) return;
      variant = rows;  // shapes outside the batched kernel's range: the two-kernel form
    }
    if (variant >= kStripFft) {
      const int rows = variant - kStripFft;
      if constexpr (strip_fft_ok(NX)) {
        hipLaunchKernelGGL((k_mug_strip_fft<T, NX>), dim3(1, (ny + rows - 1) / rows, nruns),
                           dim3(NX / 2), 0, st, runs, sa, rows);
        return;
      }
      variant = rows;  // grids outside the fused kernel's range: the two-kernel form
    }
    const dim3 gs(NX / 2 / TPB, (ny + variant - 1) / variant, nruns);
    hipLaunchKernelGGL((k_mug_strip<T, NX>), gs, dim3(TPB), 0, st, runs, sa, variant);
    R2cJobs jobs{{{B_TMP, B_GH, NX}, {}, {}}};
    r2c_jobs(runs, nruns, ny, jobs, 1, row_variant, st);
  }
};

template <typename T, int L>
struct ColLaunch {
  template <int MODE, int VAR, bool BANDED = false>
  static void launch(const Run* runs, int nruns, int nx, const StepArgs* sa, int bin0, int bin1,
                     int bout0, int bout1, hipStream_t st) {
    using C = ColCfg<T, L, VAR>;
    const dim3 gr((nx / 2 + 1 + C::CW - 1) / C::CW, 1, nruns), bl(C::THREADS);
    hipLaunchKernelGGL((k_column<T, L, MODE, VAR, BANDED>), gr, bl, 0, st, runs, sa, bin0, bin1,
                       bout0, bout1);
  }
  template <int MODE>
  static void by_variant(int variant, const Run* runs, int nruns, int nx, const StepArgs* sa,
                         int bin0, int bin1, int bout0, int bout1, hipStream_t st) {
    switch (variant) {
      case 1: launch<MODE, 1>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st); break;
      case 2: launch<MODE, 2>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st); break;
      case 3: launch<MODE, 3>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st); break;
      case 4: launch<MODE, 4>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st); break;
      default: launch<MODE, 0>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st); break;
    }
  }
  // mode: a ColMode, with COL_BANDED for the banded scheme (shape 0 whatever
  // the variant: a switch for checks of the scheme, not a tuned path)
  static void column(int mode, const Run* runs, int nruns, int nx, const StepArgs* sa,
                     int bin0, int bin1, int bout0, int bout1, int variant, hipStream_t st) {
    if (mode & COL_BANDED) {
      switch (mode & ~COL_BANDED) {
        case COL_CH:
          launch<COL_CH, 0, true>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
          break;
        case COL_FLOW:
          launch<COL_FLOW, 0, true>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
          break;
        case COL_STOKES:
          launch<COL_STOKES, 0, true>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
          break;
        default:
          launch<COL_POISSON, 0, true>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
          break;
      }
      return;
    }
    switch (mode) {
      case COL_CH:
        by_variant<COL_CH>(variant, runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
        break;
      case COL_FLOW:
        by_variant<COL_FLOW>(variant, runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
        break;
      case COL_STOKES:
        by_variant<COL_STOKES>(variant, runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
        break;
      default:
        launch<COL_POISSON, 0>(runs, nruns, nx, sa, bin0, bin1, bout0, bout1, st);
        break;
    }
  }
  using O = ObsCfg<L>;
  static int obs_nblk(int nx) { return (nx / 2 + 1 + O::CW - 1) / O::CW; }
  static void obs(const Run* run, int nx, const StepArgs* sa, int bphi, int bpsi, double* part,
                  double* bins, double* counts, hipStream_t st) {
    hipLaunchKernelGGL((k_obs_spectral<T, L>), dim3(obs_nblk(nx)), dim3(O::THREADS), 0, st, run,
                       sa, bphi, bpsi, part, bins, counts);
  }
  static int blocks(int nx) { return obs_nblk(nx); }
};

template <typename T>
struct Misc {
  static void obs_real(const Run* run, int b, double* part, int nblk, hipStream_t st) {
    hipLaunchKernelGGL((k_obs_real<T>), dim3(nblk), dim3(256), 0, st, run, b, part);
  }
  static void remap_spec(const Run* run, int b, int dkr, hipStream_t st) {
    hipLaunchKernelGGL((k_remap_spec<T>), dim3(1024), dim3(256), 0, st, run, b, dkr);
  }
  static void remap_real(const Run* run, int bin, int bout, int dkr, hipStream_t st) {
    hipLaunchKernelGGL((k_remap_real<T>), dim3(1024), dim3(256), 0, st, run, bin, bout, dkr);
  }
  static void copy_real(const Run* run, int bin, int bout, hipStream_t st) {
    hipLaunchKernelGGL((k_copy_real<T>), dim3(1024), dim3(256), 0, st, run, bin, bout);
  }
  static void restrict_real(const Run* run, int bin, int f, double* out, hipStream_t st) {
    hipLaunchKernelGGL((k_restrict<T>), dim3(256), dim3(256), 0, st, run, bin, f, out);
  }
};

template <typename T, int L>
void set_row(Ops* o) {
  o->row_r2c = &RowLaunch<T, L>::r2c;
  o->row_r2c_n = &RowLaunch<T, L>::r2c_n;
  o->row_r2c_corr = &RowLaunch<T, L>::r2c_corr;
  o->row_c2r = &RowLaunch<T, L>::c2r;
  o->advect = &RowLaunch<T, L>::advect;
  o->mu_source = &RowLaunch<T, L>::mu_source;
}

template <typename T, int L>
void set_col(Ops* o) {
  o->column = &ColLaunch<T, L>::column;
  o->obs_spectral = &ColLaunch<T, L>::obs;
  o->obs_blocks = &ColLaunch<T, L>::blocks;
}

template <typename T>
bool fill_ops(int nx, int ny, Ops* o) {
  switch (nx) {
    case 8: set_row<T, 4>(o); break;
    case 16: set_row<T, 8>(o); break;
    case 32: set_row<T, 16>(o); break;
    case 64: set_row<T, 32>(o); break;
    case 128: set_row<T, 64>(o); break;
    case 256: set_row<T, 128>(o); break;
    case 512: set_row<T, 256>(o); break;
    case 1024: set_row<T, 512>(o); break;
    case 2048: set_row<T, 1024>(o); break;
    case 4096: set_row<T, 2048>(o); break;
    default: return false;
  }
  switch (ny) {
    case 8: set_col<T, 8>(o); break;
    case 16: set_col<T, 16>(o); break;
    case 32: set_col<T, 32>(o); break;
    case 64: set_col<T, 64>(o); break;
    case 128: set_col<T, 128>(o); break;
    case 256: set_col<T, 256>(o); break;
    case 512: set_col<T, 512>(o); break;
    case 1024: set_col<T, 1024>(o); break;
    case 2048: set_col<T, 2048>(o); break;
    case 4096: set_col<T, 4096>(o); break;
    default: return false;
  }
  o->obs_real = &Misc<T>::obs_real;
  o->remap_spec = &Misc<T>::remap_spec;
  o->remap_real = &Misc<T>::remap_real;
  o->copy_real = &Misc<T>::copy_real;
  o->restrict_real = &Misc<T>::restrict_real;
  return true;
}

}  // namespace le
