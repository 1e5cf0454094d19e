/*
 * letkf.h -- C-ABI of an MI355X (gfx950) library for the LETKF local analysis
 * applied at every grid point of a D2Q9 lattice-Boltzmann ensemble.
 *
 * What is computed (arXiv 2308.03310, Sec. II-B and Algorithm 1): for every
 * grid point, the R-localized local problem
 *
 *     Q    = ((k-1)/rho) I + dY^T R_loc^-1 dY          eq. (letkf_q), inflated
 *     Pa   = Q^-1,  wbar = Pa dY^T R_loc^-1 (yo - ybar) eq. (letkf_wa)
 *     dW   = sqrt(k-1) Pa^(1/2)                         eq. (letkf_dwa)
 *     x^a_m = xbar + dX (wbar + dw_m)                    eq. (letkf_xa)
 *
 * where dY are the forecast-observation perturbations H(x_m) - ybar (eqs.
 * enkf_ybar, enkf_deltay; H takes density or velocity moments, Sec. II-A),
 * R_loc^-1 = G o R^-1 with a diagonal localization G (Sec. II-B), and the
 * nine distribution functions of a point share one transform (Sec. II-B).
 * Pa and Pa^(1/2) come from a symmetric eigendecomposition of Q (Sec. III).
 *
 * Layout conventions
 *   - ensembles are member-major FP64:  f[k][9][ny][nx], flat index
 *     ((m*9 + i)*ny + y)*nx + x, on the device;
 *   - D2Q9 direction order i = 0..8:
 *       c = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1);
 *   - the lattice is periodic in x and y; distances are minimum-image
 *     Euclidean lattice distances.
 *
 * Ownership: the caller owns every array passed in (device memory) and the
 * HIP stream; a plan owns its device workspace, which is allocated in
 * letkf_plan() only (analyze/cycle never allocate).  A plan is bound to the
 * device that was current when it was made and is used by one stream at a
 * time.
 *
 * Errors: every call returns an int status (no exceptions cross the ABI).
 * Argument errors found on the host return before anything is enqueued.
 * Errors found on the device (invalid observation record, non-finite result,
 * eigensolver not converged) are recorded in the plan and reported by
 * letkf_status(); when an invalid observation is found the analysis output
 * is left unwritten.
 */
#ifndef LETKF_H
#define LETKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define LETKF_OK          0
#define LETKF_EINVAL      1  /* invalid argument (host check) or invalid observation (device check) */
#define LETKF_ENOMEM      2  /* workspace exceeds the HBM budget or device allocation failed */
#define LETKF_EDEVICE     3  /* no usable gfx950 device, or a HIP runtime error */
#define LETKF_EBUSY       4  /* plan in use by another call */
#define LETKF_ENONFINITE  5  /* a non-finite analysis value was produced */
#define LETKF_ENOTCONV    6  /* eigensolver hit its sweep limit before converging */
#define LETKF_EIO         7  /* the tuning cache file could not be written */

/* ---- enums ---- */
/* Localization function G (Sec. II-B, R-localization). */
#define LETKF_LOC_GAUSS   0  /* exp(-r^2/(2L^2)) for r <= 2L (inclusive), else 0 */
#define LETKF_LOC_GC      1  /* Gaspari-Cohn 5th-order, half-width L, zero for r >= 2L */
#define LETKF_LOC_NONE    2  /* G = 1: every observation is local (global ETKF) */

/* Arithmetic of the Gram and update contractions.  Forecast observations,
 * the eigensolve and the eigenvalue scaling are FP64 in every form. */
#define LETKF_PREC_FP64   0
#define LETKF_PREC_FP32   1
#define LETKF_PREC_BF16   2

/* Observed variable at a lattice point (moments, Sec. II-A). */
#define LETKF_OBS_RHO     0  /* density  sum_i f_i */
#define LETKF_OBS_U       1  /* x-velocity (sum_i c_x,i f_i) / rho */
#define LETKF_OBS_V       2  /* y-velocity (sum_i c_y,i f_i) / rho */

#define LETKF_MAX_K       64 /* largest ensemble size (one wavefront row per member) */

/* One analysis problem's shape and parameters. */
typedef struct letkf_problem {
  int32_t nx, ny;       /* periodic lattice size, >= 1 each */
  int32_t k;            /* ensemble size M, 2 <= k <= LETKF_MAX_K */
  int32_t n_obs_max;    /* largest observation count a call may pass, >= 0 */
  double  loc_len;      /* localization length L (lattice units), finite, > 0 */
  double  infl;         /* multiplicative inflation rho, finite, > 0 */
  int32_t loc;          /* LETKF_LOC_* */
  int32_t precision;    /* LETKF_PREC_* */
} letkf_problem;

/* Plan flags. */
#define LETKF_FLAG_PHASE_TIMING 1  /* record HIP events around every kernel phase */
#define LETKF_FLAG_CYCLE        2  /* also allocate the lattice-BGK ping-pong buffer that
                                      letkf_cycle needs (one ensemble per problem) */
#define LETKF_FLAG_OBS_ON_HOST  4  /* the observation arrays of letkf_io (Algorithm 1's Y^o)
                                      are host memory: each call checks them on the host
                                      (LETKF_EINVAL before anything is enqueued) and copies
                                      them with hipMemcpyAsync on the call's stream into
                                      buffers the plan allocated for n_obs_max observations.
                                      The host arrays must stay unchanged until the stream
                                      has executed the copy (pinned memory makes the copy
                                      asynchronous; pageable memory is staged before the
                                      call returns) */
#define LETKF_FLAG_DETERMINISTIC 8 /* results may depend on nothing but the inputs: the
                                      observation-cell edge (which sets the summation order
                                      of the Gram matrix) stays at its default whatever
                                      letkf_tune measures or the tuning cache holds; only
                                      settings that leave every bit unchanged (the Gram
                                      kernel form) are tuned.  Without the flag the results
                                      are still bitwise reproducible for a fixed setting,
                                      alone or batched, on any stream */
#define LETKF_FLAG_GRAPH_CAPTURE 16 /* the plan's analyze / cycle calls will be captured into
                                      HIP graphs: refused together with PHASE_TIMING (its
                                      event records cannot be read back from replays).  Every
                                      call enqueues only kernels and, with OBS_ON_HOST and
                                      odd n_steps cycles, asynchronous copies: no allocation,
                                      memset or host synchronization */
#define LETKF_FLAG_NSQRT        32 /* form the transform of eqs. letkf_wa / letkf_dwa without
                                      the eigendecomposition: Q^-1/2 by the coupled
                                      Newton-Schulz iteration on MFMA (as in
                                      letkf_invsqrt_batched), wbar = Q^-1/2 (Q^-1/2 b), in
                                      FP64 whatever the problem's precision form (which
                                      still sets the Gram's).  Its cost grows with
                                      log cond(Q), the EVD's does not; accuracy about
                                      1e-17 cond(Q) relative */

/* Plan options (pass NULL for the defaults: no budget, no flags, no cache). */
typedef struct letkf_options {
  uint64_t hbm_budget_bytes;    /* workspace limit; 0 = no limit */
  int32_t  flags;               /* LETKF_FLAG_* */
  int32_t  reserved;            /* must be 0 */
  const char* tune_cache_path;  /* NULL, or a text file of letkf_tune results: letkf_plan
                                   applies the entry recorded for the same problem list and
                                   device (if any), letkf_tune records its choice there */
} letkf_options;

typedef struct letkf_plan_s* letkf_plan_t;

/*
 * letkf_plan -- validate the problems and allocate all device workspace.
 *   probs[n_probs]: problem descriptors (host memory, copied).
 *   opt:            may be NULL.
 *   out:            receives the plan handle (set to NULL on error).
 * Returns LETKF_EINVAL (any descriptor out of range, n_probs < 1, out NULL,
 * unknown flag, reserved != 0, GRAPH_CAPTURE with PHASE_TIMING), LETKF_ENOMEM
 * (workspace above hbm_budget_bytes or hipMalloc failure) or LETKF_EDEVICE
 * (no gfx950 device).  Host checks run before any device call.  A tuning
 * cache that is missing or unreadable is not an error (defaults apply).
 */
int letkf_plan(const letkf_problem* probs, int32_t n_probs, const letkf_options* opt,
               letkf_plan_t* out);

/* One analysis call: background in, analysis out (Algorithm 1 REQUIRE/ENSURE). */
typedef struct letkf_io {
  int32_t problem;          /* index into the plan's problems */
  int32_t n_obs;            /* 0 <= n_obs <= n_obs_max */
  const double*  xb;        /* device, [k][9][ny][nx] forecast ensemble */
  double*        xa;        /* device, [k][9][ny][nx] analysis; may equal xb */
  const int32_t* obs_ix;    /* [n_obs] lattice x in [0, nx)  (device; host with OBS_ON_HOST) */
  const int32_t* obs_iy;    /* [n_obs] lattice y in [0, ny) */
  const int32_t* obs_kind;  /* [n_obs] LETKF_OBS_* */
  const double*  obs_val;   /* [n_obs] observed values y^o, finite */
  const double*  obs_var;   /* [n_obs] error variances sigma^2 (R diagonal);
                               > 0, +inf means "ignore this observation" */
} letkf_io;

/*
 * letkf_analyze -- enqueue n_io analyses on hip_stream (a hipStream_t, or
 * NULL for the null stream).  Asynchronous and stream-ordered; returns after
 * host checks (LETKF_EINVAL: bad problem index, n_obs out of range, NULL
 * pointer with n_obs > 0 or NULL xb/xa; with OBS_ON_HOST also any invalid
 * observation record).  Device-side observation checks (index range, kind,
 * variance > 0 or +inf, finite value) set the plan status to LETKF_EINVAL and
 * skip the analysis of that problem.  In-place (xa == xb) is legal: the
 * background is fully consumed before any analysis value is written.
 * The eigensolve of each point's ((k-1)/rho) I + C uses refined hardware
 * reciprocal and square-root estimates: the entries of C (observation-space
 * spread products over variances) are expected to be exactly zero or
 * between about 1e-150 and 1e150 in magnitude.
 */
int letkf_analyze(letkf_plan_t plan, const letkf_io* io, int32_t n_io, void* hip_stream);

/* One data-assimilation cycle (Sec. II-B, DA cycle steps 2-3): n_steps
 * lattice-BGK steps (the lattice Boltzmann equation of Sec. II-A, collide
 * then stream, single relaxation time tau) with a Kolmogorov body force
 * F_x(y) = force_amp * sin(2 pi force_kx y / ny), F_y = 0, added as the
 * source 3 w_i (c_i . F) after relaxation; then one analysis.  The ensemble
 * is advanced and analysed in place: io.xa must equal io.xb.  The plan must
 * have been made with LETKF_FLAG_CYCLE (else LETKF_EINVAL, unless n_steps is
 * 0).  If the device finds an invalid observation (status LETKF_EINVAL), the
 * ensemble is left holding the advanced state of all n_steps steps, not
 * analysed. */
typedef struct letkf_cycle_io {
  letkf_io io;
  int32_t  n_steps;    /* >= 0 */
  int32_t  force_kx;   /* forcing wavenumber */
  double   tau;        /* BGK relaxation time, > 0.5 */
  double   force_amp;  /* body-force amplitude */
} letkf_cycle_io;

int letkf_cycle(letkf_plan_t plan, const letkf_cycle_io* io, int32_t n_io, void* hip_stream);

/*
 * letkf_advance -- the forecast step of the DA cycle (Sec. II-B, step 2)
 * alone: each io's ensemble (io.xb == io.xa, device) is advanced n_steps
 * lattice-BGK steps in place, as letkf_cycle does before its analysis; the
 * observation fields of io are ignored.  Needs a plan made with
 * LETKF_FLAG_CYCLE (for n_steps > 0).  Asynchronous on hip_stream.  Returns
 * LETKF_EINVAL for a bad problem index, xa != xb, n_steps < 0 or tau <= 0.5,
 * LETKF_EBUSY, LETKF_EDEVICE.
 */
int letkf_advance(letkf_plan_t plan, const letkf_cycle_io* io, int32_t n_io, void* hip_stream);

/*
 * letkf_tune -- project autotuner for the plan's launch settings.  Runs the
 * analyses io[0..n_io) (every problem once gives the batched form) with each
 * candidate setting -- observation-cell edge 4, 8 or 16 lattice points (the
 * tile of the local-observation search) x the kernel form (LETKF_FORM_*) --
 * times each on hip_stream with HIP events, and
 * keeps the fastest in the plan for later letkf_analyze / letkf_cycle calls.
 * Synchronizes the stream (not usable under graph capture).  On return the
 * outputs hold one analysis made with the chosen setting; out (may be NULL)
 * receives it.  With LETKF_FLAG_DETERMINISTIC only the kernel form is timed
 * and the cell edge keeps its default.  With a tune_cache_path the choice is
 * recorded in that file under a key of the problem list and device (the
 * setting still applies if that fails, and LETKF_EIO is returned).  Errors as
 * letkf_analyze, plus LETKF_EDEVICE.
 */
/* Kernel forms of the Gram -> eigensolve -> update steps (letkf_tuning.form);
 * a plan starts in LETKF_FORM_AUTO (or the form its tuning cache names). */
#define LETKF_FORM_GRID       0  /* a Gram launch and an eigensolve launch per slab of points */
#define LETKF_FORM_PERSISTENT 1  /* the same, the Gram launches as persistent work queues */
#define LETKF_FORM_FUSED      2  /* one persistent launch per width class doing the Gram,
                                    eigensolve, transform and update of every point of the
                                    call's problems on the caller's member-major arrays (no
                                    point-major copy, C kept in LDS); problems ordered by
                                    estimated cost, dearest first (plans with
                                    LETKF_FLAG_NSQRT run it as GRID) */
#define LETKF_FORM_AUTO       3  /* FUSED for the problems with 33 <= k <= 64, GRID for the
                                    narrower ones (where the Gram's own occupancy matters
                                    more than C's round trip through HBM) */

typedef struct letkf_tuning {
  int32_t cell;             /* observation-cell edge chosen */
  int32_t form;             /* LETKF_FORM_* */
  double  ms_per_call;      /* measured time of one call with that setting */
} letkf_tuning;

int letkf_tune(letkf_plan_t plan, const letkf_io* io, int32_t n_io, void* hip_stream,
               letkf_tuning* out);

/*
 * letkf_set_tuning -- apply a setting (from letkf_tune, e.g. kept from an
 * earlier run) without timing anything: cell in {4, 8, 16}, form one of
 * LETKF_FORM_* (letkf_tune reports GRID, PERSISTENT or FUSED); ms_per_call
 * is ignored.  Waits for the plan's last stream.
 * Returns LETKF_EINVAL for other values.  Results depend on the cell edge
 * only through the summation order of the Gram matrix (rounding level); the
 * three forms give bitwise-identical results.
 */
int letkf_set_tuning(letkf_plan_t plan, const letkf_tuning* t);

/*
 * letkf_status -- device-detected status of the plan's calls since the last
 * letkf_status.  sync != 0 waits for the plan's last stream first; sync == 0
 * does not wait for it (the word is read on a stream of the plan's own, so
 * the value reflects the work completed so far).  Returns LETKF_OK or the
 * most severe code found (EINVAL, then ENONFINITE, then ENOTCONV); the bits
 * that were read are cleared (an error raised after the read stays for the
 * next call).
 */
int letkf_status(letkf_plan_t plan, int32_t sync);

/* Release the plan's workspace.  NULL is accepted. */
int letkf_plan_destroy(letkf_plan_t plan);

/* Static string for a status code. */
const char* letkf_strerror(int code);

/* Device bytes held by the plan's workspace. */
uint64_t letkf_plan_workspace_bytes(letkf_plan_t plan);

/* Phases of one analysis, in launch order. */
#define LETKF_PHASE_BIN        0  /* observation checks + cell binning */
#define LETKF_PHASE_TRANSPOSE  1  /* member-major -> point-major ensemble */
#define LETKF_PHASE_OBSOP      2  /* forecast observations, mean, perturbations */
#define LETKF_PHASE_GRAM       3  /* localized Gram matrix and right-hand side */
#define LETKF_PHASE_EVD        4  /* eigensolve, transform, update */
#define LETKF_PHASE_UNTRANS    5  /* point-major -> member-major analysis */
#define LETKF_PHASE_FUSED      6  /* Gram + eigensolve + update in one launch (the fused form) */
#define LETKF_N_PHASES         7

/*
 * letkf_phase_times -- for a plan made with LETKF_FLAG_PHASE_TIMING: waits for
 * the plan's last stream, then writes the summed GPU time (ms, from HIP
 * events recorded on the analysis stream) of each phase over the analyze
 * calls since the previous letkf_phase_times (at most the last 256 calls;
 * with n_io > 1 the first analysis of each call is timed) to ms[0..n-1], the
 * number of kernel launches of each phase per timed call to launches[0..n-1]
 * (may be NULL) and returns the number of calls summed (>= 0), or -LETKF_*
 * on error.  Resets the accumulation.
 */
int letkf_phase_times(letkf_plan_t plan, double* ms, int32_t* launches, int32_t n);

/*
 * letkf_eigh_batched -- batched symmetric eigendecomposition (the role of the
 * batched EVD of Sec. III), FP64, one k x k matrix per problem.
 *   a:   device, [batch][k][k] symmetric matrices (row-major; the upper
 *        triangle is read), 1 <= k <= LETKF_MAX_K;
 *   lam: device, [batch][k] eigenvalues (ascending order is NOT guaranteed);
 *   vec: device, [batch][k][k], column j is the eigenvector of lam[j].
 *   status: device int32 (may be NULL); bit (1 << LETKF_ENOTCONV) is OR-ed
 *        in if a matrix did not converge.
 * Each matrix is scaled by a power of two (exact) so that its largest entry
 * lies in [0.5, 1) before the solve, and its eigenvalues are scaled back, so
 * the result does not depend on the matrix's magnitude; entries smaller than
 * about 2^-1022 times the largest are flushed in that scaling.  Entries must
 * be finite (a NaN or infinite entry leaves the results undefined).
 * Asynchronous on hip_stream.  Returns LETKF_EINVAL for bad sizes or NULL
 * pointers.
 */
int letkf_eigh_batched(const double* a, int32_t batch, int32_t k, double* lam, double* vec,
                       int32_t* status, void* hip_stream);

/*
 * letkf_invsqrt_batched -- batched inverse square root of symmetric positive
 * definite matrices, FP64, by the coupled Newton-Schulz iteration on MFMA:
 * the direct route to the symmetric square root of eq. letkf_dwa
 * (W = sqrt(k-1) Q^-1/2) that avoids the eigendecomposition, kept beside
 * letkf_eigh_batched for the comparison of the two.
 *   a:   device, [batch][k][k] symmetric positive definite (the full matrices
 *        are read), 1 <= k <= LETKF_MAX_K;
 *   x:   device, [batch][k][k] receives A^-1/2;
 *   status: device int32 (may be NULL); bit (1 << LETKF_ENOTCONV) is OR-ed in
 *        if a matrix's iteration did not converge (A not positive definite,
 *        non-finite, or so ill-conditioned that 64 steps do not suffice: the
 *        iteration takes about log_2.25(cond A) + 5 steps);
 *   steps: device, [batch] int32 (may be NULL): the steps each matrix took
 *        (each step is three k x k products, 6 k^3 flops).
 * Accuracy: about 1e-17 cond(A) relative to ||A^-1/2||, which the status does
 * not reflect; for the LETKF matrix cond(Q) <= 1 + rho lambda_max(C) / (k-1).
 * Asynchronous on hip_stream.  Returns LETKF_EINVAL for bad sizes or NULL
 * pointers.
 */
int letkf_invsqrt_batched(const double* a, int32_t batch, int32_t k, double* x,
                          int32_t* status, int32_t* steps, void* hip_stream);

/*
 * letkf_analyze_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one analysis of one problem, as letkf_analyze on a plan made
 * for *prob alone with no flags, without a plan.  Its workspace (the
 * point-major ensemble, the sorted observations and their perturbations, the
 * cell table, the Gram output slab) is a static device array of
 * LETKF_NOALLOC_BYTES per GPU, held from the library's first use of the GPU
 * until the process ends; the call allocates nothing.
 *   prob: the problem (as for letkf_plan; precision any form);
 *   io:   its arrays, device memory (io->problem is ignored; xa may equal xb);
 *   status: device int32, caller-owned: set to 0 on the stream, then the
 *        device status bits of the analysis are OR-ed in (bit n <-> code n:
 *        LETKF_EINVAL for an invalid observation, LETKF_ENONFINITE,
 *        LETKF_ENOTCONV); read it after the stream has executed the call.
 * Asynchronous on hip_stream.  Returns LETKF_EINVAL as letkf_plan and
 * letkf_analyze's host checks do, LETKF_ENOMEM when the problem's workspace
 * (about 9 k nx ny doubles for the ensemble plus n_obs_max (KP + 6) doubles,
 * with KP = max(16, the power of two >= k), plus a Gram slab of at least 256
 * points) does not fit in LETKF_NOALLOC_BYTES, LETKF_EDEVICE without a gfx950
 * device.  All calls on one GPU share its array: calls whose executions
 * overlap on one GPU (different streams, or host threads) race and give
 * undefined results; calls ordered on one stream are safe.
 */
#define LETKF_NOALLOC_BYTES (64ull << 20)
int letkf_analyze_noalloc(const letkf_problem* prob, const letkf_io* io, int32_t* status,
                          void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LETKF_H */
