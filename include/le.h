/*
 * le.h -- C ABI of the MI355X sheared model-H time step.
 *
 * The library advances 2D model H (Cahn-Hilliard for the composition phi
 * coupled to the Navier-Stokes streamfunction/vorticity equations) under an
 * applied shear flow, in the cosheared frame of Fielding's paper ("Numerical
 * method"; Appendix A), by the split step of Appendix B:
 *
 *   1a  phi, omega advected by psi^n (explicit Euler, Eq. advective, with the
 *       shear-interpolated y stencil of Eq. p1y); f = phi^3;
 *   1b  Cahn-Hilliard diffusive update per Fourier mode (explicit in
 *       nabla_c^2 and f, Crank-Nicolson in nabla_c^4);
 *   2a  mu and the vorticity source g = -[d_x phi d_y mu - d_y phi d_x mu]/rho
 *       by finite differences (Eqs. vortNum, G);
 *   2b  omega by Crank-Nicolson per mode (Eq. forOmega);
 *   3   psi = -omega / lambda per mode, or at rho = 0 the biharmonic solve
 *       psi = g / lambda^2 ("Algorithm at zero Reynolds number").
 *
 * The sawtooth strain s(t) of Eq. coshearedNabluFinal is kept in
 * [-Lx/2Ly, Lx/2Ly); at each jump the fields are remapped so the lab-frame
 * field is continuous.
 *
 * Conventions for every function below:
 *   - Host arrays are nx*ny doubles, row-major [j][i], x (flow direction)
 *     fastest, in the cosheared frame.  They are read or written during the
 *     call only; the library never keeps a caller pointer.  In LE_FP32 mode
 *     they are converted on upload and download.
 *   - The context owns all device memory it allocates.  Caller-provided
 *     outputs are written only when the call returns LE_OK.
 *   - All functions return LE_OK (0) or a negative LE_E* code; no C++
 *     exception crosses this boundary.  le_strerror() names a code.
 *   - A context is used by one host thread at a time; separate contexts are
 *     independent.  Work is enqueued on the context's HIP stream and every
 *     function returns after that stream has drained.
 */
#ifndef LE_H
#define LE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LE_OK = 0,
  LE_EINVAL = -1,     /* invalid parameters or arguments; nothing allocated */
  LE_ENOMEM = -2,     /* device or host allocation failed */
  LE_EDEVICE = -3,    /* a HIP call failed (no device, launch error, ...) */
  LE_ENONFINITE = -4, /* the state became non-finite; stepping stopped */
  LE_ESTATE = -5      /* call not valid in the context's current state */
};

enum { LE_FP64 = 0, LE_FP32 = 1 };

typedef struct le_ctx le_ctx;

/*
 * Problem statement of the paper's "Governing equations", "Flow geometry" and
 * "Choice of units" sections, with the free energy written generally:
 *   mu = B phi^3 - A phi - kappa nabla^2 phi,  d_t phi + v.grad phi = M nabla^2 mu,
 *   rho (d_t omega + v.grad omega) = eta nabla^2 omega - [curl(phi grad mu)].z.
 * The paper's units are A = B = 1, kappa = M = l^2, ly = 1.
 */
typedef struct le_params {
  int32_t nx, ny;      /* powers of two, 8 <= nx, ny <= 4096; if gdot != 0
                          then nx must be a multiple of ny (strain-wrap remap) */
  double lx, ly;       /* box; dx = lx/nx, dy = ly/ny */
  double gdot;         /* applied shear rate, any sign; 0 = unsheared */
  double A, B, kappa;  /* free-energy constants, all > 0 */
  double M;            /* mobility > 0 */
  double eta, rho;     /* viscosity > 0; density >= 0 (0 = Stokes branch) */
  double dt;           /* time step > 0 */
  int32_t precision;   /* LE_FP64, or LE_FP32: FP32 storage, stencils and
                          FFTs with the per-mode solves and all reductions in
                          FP64 */
  void* stream;        /* hipStream_t to enqueue on (e.g. torch's current
                          stream); NULL = the library creates its own */
} le_params;

/*
 * Observables of the paper's "Lengthscales and timescales" section at the
 * context's current step.  Wave vectors are lab-frame, q_lab = (qx, qy - s qx).
 */
typedef struct le_obs {
  int64_t step, wraps;   /* steps taken; strain jumps taken */
  double t, strain, s;   /* t = step*dt; strain = gdot*t; s = sawtooth offset */
  double mean_phi;       /* (1/N) sum phi -- conserved by the method */
  double phi2;           /* (1/N) sum phi^2 */
  double Ls;             /* Eq. L_structure: sum_{q!=0} S/|q| / sum_{q!=0} S */
  double Dxx, Dxy, Dyy;  /* Eq. L_matrix: l sum q_a q_b S / sum S, l = sqrt(kappa/A) */
  double L_par, L_perp;  /* 1/lambda_min(D) (inf if <= 0), 1/lambda_max(D) */
  double sigma_xy;       /* interfacial excess shear stress -kappa <d_x phi d_y phi> */
  double sigma_xy_re;    /* Reynolds stress -rho <v_x v_y> of the flow (0 if rho = 0) */
  int32_t nbins;         /* number of S(k) shells reported (ny/2) */
  double dk;             /* shell width 2 pi / ly; shell b covers |q| in [(b-1/2)dk, (b+1/2)dk) */
  int32_t finite;        /* 1 if every phi value is finite */
} le_obs;

/*
 * Create a context: validate p, allocate the device state, upload phi0 and
 * omega0 (omega0 may be NULL: zero vorticity; ignored when rho == 0) and set
 * psi0 from the flow constraint at s = 0 (a Poisson solve from omega0, or the
 * Stokes solve from phi0 at rho = 0).  On success *out owns the context.
 * Errors: LE_EINVAL (bad p or NULL phi0/out), LE_ENOMEM, LE_EDEVICE.
 */
int le_create(const le_params* p, const double* phi0, const double* omega0,
              le_ctx** out);

/* Advance nsteps >= 0 full time steps (the sawtooth clock advances with
 * them).  Returns LE_ENONFINITE if phi became non-finite, checked at the end
 * of the call; the context is then left at the last step whose phi is finite
 * (step counter and wrap count included; see le_set_recovery, on by
 * default).  nsteps < 0: LE_EINVAL. */
int le_step(le_ctx* c, int64_t nsteps);

/*
 * le_step without a context, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  phi_dev, omega_dev, psi_dev: the caller's device arrays of
 * nx*ny doubles, row-major [j][i] (x fastest), the real fields phi, omega,
 * psi of step step0 >= 0 (the state le_get_state returns; omega_dev is
 * ignored and may be NULL when rho == 0); on return they hold the state of
 * step step0 + nsteps, remapped at every strain wrap as le_step does.  Every
 * other buffer (row spectra, stencil outputs, twiddles, the descriptor, the
 * strain offsets and the reduction) lives in one static device array of
 * 8 MiB that the library holds on each device it runs on until the process
 * ends; the call allocates nothing.  Limits: p->precision == LE_FP64 and a
 * grid whose buffers fit that array (up to 256 x 256, or equivalently small
 * non-square grids), else LE_EINVAL (le_last_error names the size).  The
 * kernel shapes are the defaults (no autotuning), so results equal a
 * context's to rounding, not bit for bit.  Runs on p->stream (NULL: the null
 * stream) and returns after draining it.  No recovery: LE_ENONFINITE leaves
 * the non-finite state in the caller's arrays.  Calls on one device share
 * the static array: calls that overlap in time on one device race (run them
 * on one stream, one after another); the array keeps the last call's
 * contents, none of which a later call reads before writing it.
 */
int le_step_noalloc(const le_params* p, double* phi_dev, double* omega_dev, double* psi_dev,
                    int64_t step0, int64_t nsteps);

/*
 * Recovery from a non-finite state (failure handling; not part of the
 * method).  On (the default of every context from le_create): le_step keeps
 * a copy of the state at the start of each call (two state snapshots, taken
 * from the context's memory at creation); when the call ends with a
 * non-finite phi it replays the call's steps one at a time from that copy
 * and leaves the context at the last step whose phi is finite, returning
 * LE_ENONFINITE.  A call that starts from a non-finite state is left at its
 * start.  enable = 0: le_step skips the copy and returns LE_ENONFINITE with
 * the non-finite state in place.  Single contexts only (LE_EINVAL for NULL);
 * LE_ENOMEM if the snapshots cannot be allocated when re-enabled.
 */
int le_set_recovery(le_ctx* c, int enable);

/*
 * Scheme variants either side of the default reading of Appendix B (for
 * convergence studies; the default, flags = 0, is the scheme as read):
 *   LE_SCHEME_F_HALF      f = (phi^{n+1/2})^3, the cube of the advected phi
 *                         (the stage 1b update formula writes f^n, the
 *                         default takes that as (phi^n)^3);
 *   LE_SCHEME_MIDPOINT_S  every operator of step n at the sawtooth of the
 *                         step's midpoint, s(t_n + dt/2) in the frame of step
 *                         n, instead of s(t_n) (observables stay at s(t_n));
 *   LE_SCHEME_UPWIND3     the derivatives of the advected fields (phi and
 *                         omega in stage 1a) by the third-order upwind
 *                         differences that Appendix B keeps as a commented-out
 *                         alternative to Eq. p1y, upwind with respect to the
 *                         local velocity (d_y psi, -d_x psi); the y samples
 *                         are sheared as in Eq. p1y (weight |s|/c on the
 *                         column r k cells along the grid diagonal for row
 *                         j + k).  The derivatives of psi stay central;
 *   LE_SCHEME_BANDED      the per-mode operators of stages 1b, 2b and 3 with
 *                         their y part by the stencils' central differences
 *                         (Fourier in x only): per x wavenumber a cyclic
 *                         tridiagonal system (omega, Poisson) or
 *                         pentadiagonal one (Cahn-Hilliard, Stokes) in y.
 *                         Their coefficients do not depend on y, so the
 *                         column transform diagonalizes them: the solves are
 *                         per-mode divisions by the banded operators'
 *                         eigenvalues (the observables stay spectral).
 * Takes effect from the next step; flags outside these bits: LE_EINVAL.
 */
enum {
  LE_SCHEME_F_HALF = 1,
  LE_SCHEME_MIDPOINT_S = 2,
  LE_SCHEME_UPWIND3 = 4,
  LE_SCHEME_BANDED = 8
};
int le_set_scheme(le_ctx* c, int32_t flags);

/*
 * Compute the observables of the current state into *o.  If Sk is non-NULL,
 * the shell-averaged structure factor S(k_b) = mean over the modes of shell
 * b of |F[phi](q)|^2 / N is written for b = 1 .. min(sk_cap, ny/2) into
 * Sk[0 ..]; shells with no modes read 0.
 */
int le_observables(le_ctx* c, le_obs* o, double* Sk, int32_t sk_cap);

/* Release the context and everything it owns.  NULL is accepted. */
void le_destroy(le_ctx* c);

/* Copy the current state to the host (any pointer may be NULL to skip that
 * field; psi and omega are real-space fields).  step/wraps may be NULL. */
int le_get_state(le_ctx* c, double* phi, double* omega, double* psi,
                 int64_t* step, int64_t* wraps);

/* Replace the state (phi and psi required; omega required when rho > 0) and
 * the clock (step >= 0; wraps must equal the wrap count implied by step). */
int le_set_state(le_ctx* c, const double* phi, const double* omega,
                 const double* psi, int64_t step, int64_t wraps);

/*
 * Checkpoint of the exact stored state, for a bitwise resume (le_get_state /
 * le_set_state pass omega and psi through real space, which rounds).
 * le_checkpoint_size: the blob's byte count.  le_checkpoint_save writes into
 * buf (cap >= that size, else LE_EINVAL) a header (format tag, nx, ny,
 * precision, inertia, the spectral layout's tile width, step, wraps) and the
 * stored fields as they are on the device: phi (real), the row spectra of
 * omega (rho > 0) and psi, in storage precision and the library's layout.
 * le_checkpoint_load restores such a blob into a context of the same nx, ny,
 * precision and inertia and a library of the same layout (LE_EINVAL
 * otherwise, or for a damaged or short blob); the continued run equals the
 * saved one bit for bit when both contexts use the same kernel variants
 * (le_tuning).  Single contexts only.
 */
int le_checkpoint_size(le_ctx* c, int64_t* bytes);
int le_checkpoint_save(le_ctx* c, void* buf, int64_t cap);
int le_checkpoint_load(le_ctx* c, const void* buf, int64_t bytes);

/* Static description of an error code. */
const char* le_strerror(int code);

/* Text naming the last HIP call that failed on the calling thread and the
 * HIP error it returned ("" if none); valid until the next failure. */
const char* le_last_error(void);

/*
 * Per-stage GPU timing.  With profiling enabled, le_step brackets every stage
 * launch with HIP events on the context's stream and accumulates the elapsed
 * time per stage.  Stage indices:
 *   0 inverse row transform of omega and psi    3 inverse row transform of phi
 *   1 advection + forward row transforms (1a)    4 mu and g + forward row transform (2a)
 *   2 column pass, Cahn-Hilliard update (1b)     5 column pass, omega and psi (2b, 3)
 * le_profile(c, 1) enables and clears the counters, le_profile(c, 0) disables.
 * le_stage_times writes min(cap, LE_NSTAGES) accumulated milliseconds and
 * launch counts (either pointer may be NULL).
 */
enum { LE_NSTAGES = 6 };
int le_profile(le_ctx* c, int enable);
int le_stage_times(le_ctx* c, double* ms, int64_t* launches, int32_t cap);

/*
 * le_time_stage: the average duration (milliseconds) of one launch of stage
 * `stage` (numbered as above, with the autotuned variant) over `reps`
 * back-to-back launches on the context's stream, after one untimed launch.
 * The launches read the current state and write only scratch buffers, so
 * the state is neither advanced nor changed.
 * LE_EINVAL for a bad stage, reps < 1 or NULL; LE_ESTATE while le_profile
 * timing is enabled.
 */
int le_time_stage(le_ctx* c, int32_t stage, int32_t reps, double* ms_per_launch);

/*
 * Kernel variants (not part of the method: how its stages are laid out on
 * the GPU).  At creation every group of runs sharing (nx, ny, precision,
 * rho > 0) times the candidate kernel variants of its stages on its own
 * buffers and keeps the fastest; every variant computes the same stage (to
 * rounding; runs are bit-identical only between equal variants).  le_tuning
 * writes, per group, LE_TUNING_FIELDS int32 values
 *   nx, ny, precision, inertial, advect, mu_source, column_ch, column_flow,
 *   row, row_fwd
 * (advect / mu_source: 0 = one fused stencil-and-row-transform kernel,
 * 0 < k < 64 = a stencil kernel over k-row strips then in-place row
 * transforms; advect 64 + k and 96 + k (two or one x pairs per thread, nx
 * 256 .. 1024) and mu_source 64 + k (nx 256 .. 2048) = the k-row strip
 * stencil and the row transforms in one kernel (other nx: as k);
 * column_*: block shape 0 .. 4 (8 or 16 values per thread, columns per
 * block); row / row_fwd: shape 0 .. 5 of the inverse / forward row
 * transforms (8 or 4 values per thread; all or a quarter of the rows per
 * block, or 4 and 5: groups of four consecutive rows stored or loaded
 * together)), at most cap
 * values in all, and returns the number of
 * groups (LE_EINVAL for NULL c, cap < 0 or out NULL with cap > 0).  The
 * environment variables LE_TUNE_ADV, LE_TUNE_MU, LE_TUNE_COL_CH,
 * LE_TUNE_COL_FLOW, LE_TUNE_ROW and LE_TUNE_ROW_FWD, when set, fix the
 * corresponding variant at creation (LE_TUNE_LOG=1 prints every candidate's
 * time to stderr).  The choices are cached per (device, nx, ny, precision,
 * inertia, runs in the group) for the life of the process, so later
 * contexts and batches of the same shape take the same kernels (and give the
 * same results) without re-timing; LE_TUNE_CACHE=<file> also keeps them in
 * that text file across processes, LE_TUNE_CACHE=off times every creation
 * afresh.  Choices fixed through LE_TUNE_* are not cached.
 */
enum { LE_TUNING_FIELDS = 10 };
int le_tuning(le_ctx* c, int32_t* out, int32_t cap);

/*
 * Batched runs.  Many independent runs (each with its own grid, shear rate,
 * density, precision and initial state) advance together: every stage of a
 * step is one launch per group of runs sharing (nx, ny, precision, rho > 0),
 * each group runs a chunk of steps on a stream of its own (forked from and
 * joined back into the batch's stream, so the groups' kernels overlap;
 * LE_CLASS_STREAMS=0 at creation keeps every group on the batch's stream),
 * and chunks of steps are replayed from captured HIP graphs.  Each run's
 * result is the one le_create/le_step would give for it alone.
 *
 * le_batch_create: n >= 1 runs; ps[i], phi0s[i] as for le_create; omega0s may
 *   be NULL (all zero) or hold NULL entries.  Every ps[i].stream must be equal
 *   (the batch runs on one stream).  Errors as le_create.
 * le_batch_step: advance every run by nsteps (one common step counter).
 * le_batch_observables / le_batch_get_state: as le_observables /
 *   le_get_state for run index 0 <= run < n (LE_EINVAL otherwise).
 * le_batch_profile / le_batch_stage_times: as le_profile / le_stage_times,
 *   each stage timed across all runs.
 * le_batch_tuning: as le_tuning, one record per group of runs.
 */
typedef struct le_batch le_batch;
int le_batch_create(int32_t n, const le_params* ps, const double* const* phi0s,
                    const double* const* omega0s, le_batch** out);
int le_batch_step(le_batch* b, int64_t nsteps);
int le_batch_observables(le_batch* b, int32_t run, le_obs* o, double* Sk, int32_t sk_cap);
int le_batch_get_state(le_batch* b, int32_t run, double* phi, double* omega, double* psi,
                       int64_t* step, int64_t* wraps);
int le_batch_profile(le_batch* b, int enable);
int le_batch_stage_times(le_batch* b, double* ms, int64_t* launches, int32_t cap);
int le_batch_tuning(le_batch* b, int32_t* out, int32_t cap);
int le_batch_set_scheme(le_batch* b, int32_t flags);  /* le_set_scheme for every run */
void le_batch_destroy(le_batch* b);  /* NULL-safe */

/*
 * Learned coarse-step corrector (single inertial run).  After every plain
 * step the network maps the state (phi, omega) to a residual r, applied as
 *   phi += r_phi - mean(r_phi),  omega += r_omega,
 * and psi is re-solved from the corrected omega (Poisson solve at the step's
 * strain offset).  The mean-phi projection keeps the conserved mean exact.
 *
 * le_corrector_load: params = the network's FP32 weight vector (length
 *   le_cnn_nparams(); per layer W[co][ci][ky][kx] then b[co], layers
 *   2->32->32->32->2); scales = {in_phi, in_omega, out_phi, out_omega}.
 *   Needs rho > 0, nx, ny >= 16 and nx*ny a multiple of 256 (LE_EINVAL).
 * le_step_corrected: ncoarse corrected steps (LE_EINVAL before a load).
 * le_restrict: factor x factor block means of phi and omega (real space) into
 *   host arrays of (ny/factor)*(nx/factor) doubles (either may be NULL).
 * le_set_fields: replace phi and omega (NULL: zero) and the step counter;
 *   psi is re-solved from the flow constraint at that step.
 */
int le_corrector_load(le_ctx* c, const float* params, int32_t nparams, const float* scales);
int le_step_corrected(le_ctx* c, int64_t ncoarse);
/* le_corrector_projection: mode 0 (the default) subtracts the mean of the
 * phi residual (above); mode 1 subtracts its 16 x 16 tile means, interpolated
 * bilinearly between the tile centres (periodic), which keeps the mean exact
 * and takes out the residual's content at scales beyond a tile.  LE_EINVAL
 * for other modes, or mode 1 when nx or ny is not a multiple of 16. */
int le_corrector_projection(le_ctx* c, int32_t mode);

int le_restrict(le_ctx* c, int32_t factor, double* phi_out, double* omega_out);
int le_set_fields(le_ctx* c, const double* phi, const double* omega, int64_t step);

/*
 * Corrector audit (failure detection; the paper has no corrector, so this
 * is a safeguard of the learned step, not part of the method).  With
 * every > 0, le_step_corrected runs, after each `every` corrected steps, an
 * audit window of `window` steps (fewer if the call ends first) twice from
 * the same state: corrected, then plain.  The audit passes when the
 * corrected state is finite, its L_s is within relative `tol` of the plain
 * run's and its mean phi equals the plain run's (to 1e-9; FP32 runs 1e-5);
 * then the corrected state continues.  On a failed audit the plain state is
 * kept and every later corrected step of the context runs as a plain step
 * (the fallback), until the next le_corrector_load or le_corrector_audit.
 * every = 0 switches audits off (the default).  The context allocates two
 * state snapshots (phi and the omega, psi row spectra) on the first call
 * with every > 0.
 * Errors: LE_EINVAL (no corrector loaded, every < 0, or every > 0 with
 * window < 1 or tol < 0 or NaN), LE_ENOMEM.
 * le_corrector_status: fallback (1 once an audit failed), the number of
 * audits run and the last audit's relative L_s deviation (INFINITY when the
 * corrected state was not finite); NULL outputs are skipped.
 */
int le_corrector_audit(le_ctx* c, int64_t every, int64_t window, double tol);
int le_corrector_status(le_ctx* c, int32_t* fallback, int64_t* audits, double* last_dev);

/* The corrector network's training entry points (device pointers, not part
 * of the time-step contract) are declared in le_train.h. */

#ifdef __cplusplus
}
#endif

#endif /* LE_H */
