/*
 * cf.h — C ABI of libcf, the MI355X (gfx950) hot path of QML power-spectrum
 * estimation and the pixel-space Gaussian likelihood of
 * "CosmoForge I" (Galloni & Pagano), Sects. 2.1-2.6 and Apps. A-C.
 *
 * Every entry point runs its whole computation in HIP kernels on the current
 * HIP device and returns only when the results are written.  Two calls on one
 * device from different host threads run at the same time, each on a call
 * lane of its own (streams, events, workspace); a third waits for the first
 * lane.  Once two calls have overlapped on a device, single factorisations
 * there stop reserving CUs for their chain of diagonal blocks.  The entry
 * points that allocate nothing share one scratch array per device and are
 * serialised among themselves.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  - Data vector order [T | Q | U] over the same retained pixels, in ascending
 *    HEALPix RING index (or explicit-direction order), paper Sect. A.2
 *    "multi-field structure".
 *  - Spectra arrays are [6][lmax+1] in TT, EE, BB, TE, TB, EB order, in uK^2;
 *    rows of spectra whose fields are absent are ignored.
 *  - W_l = B_l^2 p_l^2 (beam and pixel window), Eq. signal_cov.  The signal
 *    band equals the analysis window [lmin, lmax].
 *  - Matrices are row-major doubles; symmetric outputs are written in full.
 *  - Fisher / spectra index = s * nbins + b, s running over the set bits of
 *    cf_bins.spectra in TT, EE, BB, TE, TB, EB order.
 *  - Ownership: the caller owns every input and output.  The library keeps
 *    no pointer after returning.
 *  - Memory space: large arrays (noise, maps, scan spectra, outputs) live in
 *    host or device memory according to cf_problem.mem; small descriptors
 *    (mask, directions, spectra of cf_problem, beams, bins) are host memory.
 *  - Errors: a non-zero cf_status is returned and cf_last_error() describes
 *    it; outputs are left untouched unless the status is CF_OK.
 */
#ifndef CF_H
#define CF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CF_OK = 0,
  CF_EINVAL = 1,   /* bad argument: NaN/Inf, broken l-range chain, bins outside [lmin,lmax], ... */
  CF_ENOTPD = 2,   /* C (or F) not positive definite; cf_report.fail_index = failing pivot */
  CF_ENOMEM = 3,   /* device allocation failed */
  CF_EDEVICE = 4,  /* HIP runtime error */
  CF_ENOCONV = 5   /* mixed-precision refinement did not converge */
} cf_status;

typedef enum { CF_FP64 = 0, CF_MIXED_FP32 = 1, CF_MIXED_BF16X3 = 2 } cf_precision;
typedef enum { CF_T = 1, CF_QU = 2, CF_TQU = 3 } cf_fields;
typedef enum { CF_TT = 1, CF_EE = 2, CF_BB = 4, CF_TE = 8, CF_TB = 16, CF_EB = 32 } cf_spectrum;
typedef enum { CF_NOISE_DIAG = 0, CF_NOISE_DENSE = 1 } cf_noise_kind;
typedef enum { CF_MEM_HOST = 0, CF_MEM_DEVICE = 1 } cf_mem;

/* One masked-map problem (paper Sect. 2.1: data d, mask, C_l, beam, pixel
 * window, noise covariance N; l-range chain of the configuration appendix). */
typedef struct {
  int32_t nside;          /* > 0: HEALPix RING pixel centres; 0: explicit directions */
  const uint8_t* mask;    /* [12 nside^2] keep-flags (1 = keep), NULL = full sky     */
  int64_t ndir;           /* number of explicit directions (nside == 0)             */
  const double* theta;    /* [ndir] colatitudes (rad)                               */
  const double* phi;      /* [ndir] longitudes (rad)                                */
  int32_t fields;         /* cf_fields                                              */
  int32_t lmin, lmax;     /* 0 <= lmin <= lmax <= 1023; lmin >= 2 when Q,U present  */
  const double* cl;       /* [6][lmax+1] fiducial / model spectra, uK^2             */
  const double* bl;       /* [lmax+1] beam B_l, NULL = 1                            */
  const double* pl;       /* [lmax+1] pixel window p_l, NULL = 1                    */
  int32_t noise_kind;     /* cf_noise_kind                                          */
  const double* noise;    /* DIAG: [n]; DENSE: [n][n] symmetric positive definite   */
  int32_t noise_rank;     /* >= 0: N += U U^T                                        */
  const double* noise_U;  /* [n][noise_rank]                                        */
  int32_t mem;            /* cf_mem of noise, noise_U, maps, scan spectra, outputs  */
} cf_problem;

/* Native multipole bins (Sect. 2.4); delta_l = 1 is nbins = lmax-lmin+1 bins of one l. */
typedef struct {
  int32_t nbins;
  const int32_t* lo;      /* [nbins] first multipole of each bin */
  const int32_t* hi;      /* [nbins] last multipole of each bin  */
  uint32_t spectra;       /* OR of cf_spectrum                    */
} cf_bins;

/* Optional execution controls (NULL = defaults). */
typedef struct {
  void* stream;           /* hipStream_t the call is ordered on (NULL: none): the call starts
                             after the work queued on it and the work queued on it after the call
                             waits for the call; the kernels run on the library's own streams */
  int32_t stage_timing;   /* 1: record per-stage device time in the report      */
  int32_t refine_max;     /* mixed precision: max refinement steps (-1 default)  */
  int32_t allow_fallback; /* mixed precision: fall back to FP64 instead of ENOCONV */
  int32_t no_graph;       /* 1: launch every kernel eagerly instead of replaying captured hipGraphs */
  int32_t autotune;       /* 1: time the candidate batch sizes of a new scan shape and keep the best */
} cf_exec;

/* Optional report (NULL = none). */
typedef struct {
  double ms_total;        /* device time of the call                                  */
  double ms_stage[8];     /* build, potrf, ybuild, trsm, syrk, reduce, qml, other     */
  double flops;           /* algorithmic flop count of the call                        */
  double logdet;          /* ln|C| of the (last) factorised covariance                 */
  int64_t n;              /* data dimension                                            */
  int64_t nmodes;         /* harmonic modes (columns of Y)                             */
  int32_t fail_index;     /* CF_ENOTPD: first non-positive pivot, else -1              */
  int32_t ir_iters;       /* refinement steps taken                                    */
  double est_err[4];      /* mixed precision error estimates                           */
  int64_t n_fallback;     /* fallbacks taken                                           */
  /* With cf_exec.stage_timing: every launch of the FP64 matrix-core GEMM is bracketed by events
   * on its stream and summed per kernel instance.  id 0-7: (128 x 128 tile) + 2 (A stored
   * transposed) + 4 (B stored transposed); 8 + (128 tile): the separately named Z = G^T G
   * instance; 10 + (128 tile): the Cholesky updates C -= L L^T, also named apart:               */
  double gemm_ms[16];        /* summed device time of the instance's launches                  */
  double gemm_flops[16];     /* their algorithmic flops, 2 M N K, outputs of a lower-triangular
                                product counted on the triangle only                          */
  int64_t gemm_launches[16]; /* their number                                                  */
  double gemm_bytes[16];     /* their algorithmic HBM bytes: A and B read once, C written once
                                (read as well when beta != 0), lower outputs on the triangle only */
} cf_report;

/* Data dimension n = nmaps * npix of a problem, or -1 (see cf_last_error). */
int64_t cf_problem_dim(const cf_problem* prob);

/* Number of harmonic modes (columns of Y = V^T) of a problem: nfields_modes * ((lmax+1)^2 - lmin^2). */
int64_t cf_problem_nmodes(const cf_problem* prob);

/* Pixel covariance C = S + N (Eqs. total_cov, signal_cov and its spin-2 extension, App. A).
 * C_out: [n][n], full symmetric matrix, in prob->mem space.  n_out (host) receives n. */
int cf_cov_build(const cf_problem* prob, double* C_out, int64_t* n_out,
                 const cf_exec* ex, cf_report* rep);

/* Fisher matrix F_bb' = 1/2 tr[C^-1 P_b C^-1 P_b'] (Eq. fisher) with native bins (Sect. 2.4),
 * evaluated as block Frobenius products of Z = Y^T C^-1 Y (Eqs. projected_inv,
 * fisher_harmonic, sparse_trace).  F_out: [(ns*nb)^2] in prob->mem space.  Mixed precisions
 * factor C with FP32 or split-BF16x3 updates and refine C^-1 Y once with an FP64 residual
 * (Z = G^T G + G^T L^-1 (Y - C L^-T G), G = L^-1 Y, products in FP64). */
int cf_fisher(const cf_problem* prob, const cf_bins* bins, int32_t precision, double* F_out,
              const cf_exec* ex, cf_report* rep);

/* QML estimates for nmaps maps (Eqs. q_ell, noise_bias, qml_estimate, q_harmonic):
 *   y_out    [nmaps][ns*nb]  raw quadratic forms 1/2 d^T C^-1 P_b C^-1 d
 *   bias_out [ns*nb]         noise bias 1/2 tr[C^-1 P_b C^-1 N]
 *   chat_out [nmaps][ns*nb]  deconvolved estimates F^-1 (y - b)
 *   F_out    [(ns*nb)^2]     Fisher matrix (nullable)
 * maps: [nmaps][n].  All in prob->mem space. */
int cf_qml(const cf_problem* prob, const cf_bins* bins, const double* maps, int32_t nmaps,
           int32_t precision, double* y_out, double* bias_out, double* chat_out, double* F_out,
           const cf_exec* ex, cf_report* rep);

/* Cross-QML of two data sets filtered independently (Eq. q_cross, Sect. 2.2 "Cross-correlation"):
 *   q_out    [nmaps][ns*nb]  q^x_b = 1/2 d1^T C1^-1 P_b C2^-1 d2 for the map pairs (maps1[j], maps2[j])
 *   chat_out [nmaps][ns*nb]  W^-1 q^x (no noise-bias term: the two noises are independent)
 *   W_out    [(ns*nb)^2]     mode-mixing matrix W_bb' = 1/2 tr[C1^-1 P_b C2^-1 P_b'] (nullable)
 * prob1 and prob2 describe the two data sets: C_a = S + N_a with the same geometry, fields,
 * l-range, spectra, beam, pixel window and memory space (else CF_EINVAL); they differ in their
 * noise.  maps1, maps2: [nmaps][n].  FP64. */
int cf_qml_cross(const cf_problem* prob1, const cf_problem* prob2, const cf_bins* bins, const double* maps1,
                 const double* maps2, int32_t nmaps, double* q_out, double* chat_out, double* W_out,
                 const cf_exec* ex, cf_report* rep);

/* Pixel likelihood over a parameter scan (Eq. pixel_likelihood, Sect. 2.6):
 *   -2 ln L_{i,p,j} = d_{p,j}^T C_{i,p}^-1 d_{p,j} + ln|C_{i,p}|  (n ln 2 pi excluded)
 * for points i < npoints, problems p < nprob and maps j < nmaps.
 *   cl_points [npoints][nprob][6][lstride]: spectra of each point and problem, lstride >= lmax_p+1
 *   maps[p]   [nmaps][n_p]
 *   m2lnL     [npoints][nprob][nmaps];  chi2 same shape (nullable);  logdet [npoints][nprob] (nullable)
 * Geometry, beam, window and noise come from probs[p]; its cl is not used.  Memory space
 * of cl_points, maps and outputs: probs[0].mem.  Mixed precisions: chi^2 from FP64-refined solves;
 * ln|C| = ln|L L^T| of the mixed factor L plus a stochastic estimate of tr X - |X|_F^2 / 2,
 * X = L^-1 (C - L L^T) L^-T, from 384 fixed +-1 probe vectors with FP64 solves (deterministic;
 * standard deviation about 0.07 |X|_F). */
int cf_loglike_batch(const cf_problem* probs, int32_t nprob, int32_t npoints,
                     const double* cl_points, int32_t lstride, const double* const* maps,
                     int32_t nmaps, int32_t precision, double* m2lnL, double* chi2,
                     double* logdet, const cf_exec* ex, cf_report* rep);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): cf_loglike_batch with the same arguments, results and errors, that
 * allocates nothing.  Its workspace is a static device array of 64 MiB per GPU (held from the
 * library's first use on that GPU until the process ends); it creates no streams, events, graphs or
 * pinned buffers and runs every launch eagerly, in order, on cf_exec.stream (NULL: the null
 * stream), returning when the results are written.  It does not autotune (cf_exec.autotune,
 * no_graph and stage_timing are ignored): the batch of points factorised together is the largest
 * (at most 128) whose workspace fits the array.  CF_EINVAL when even one point does not fit (for
 * FP64 with 64 maps, up to about n = 2600; host-memory problems also stage their inputs in it).
 * Calls on one GPU share the array, which keeps the last call's contents; the library serialises
 * these calls per device (other entry points run beside them on call lanes of their own, never on
 * the array) and each returns after its work is done, so calls never overlap on it. */
int cf_loglike_batch_noalloc(const cf_problem* probs, int32_t nprob, int32_t npoints,
                             const double* cl_points, int32_t lstride, const double* const* maps,
                             int32_t nmaps, int32_t precision, double* m2lnL, double* chi2,
                             double* logdet, const cf_exec* ex, cf_report* rep);

/* Iterative QML for one map (Sects. 2.2 and 2.6: the single-step estimate is one Newton step towards
 * the maximum of the pixel likelihood; the paper describes the iteration as re-entering the QML with
 * the previous estimates in place of the fiducial).  Iteration i runs the FP64 QML of cf_qml with
 * fiducial C^(i) (C^(0) = prob->cl); C^(i+1) takes every estimated band as a flat band over its
 * multipoles, and at every multipole the spectrum matrix over the problem's harmonic fields is
 * replaced by its nearest positive semi-definite matrix (negative eigenvalues set to zero).  Stops
 * at the first iteration whose estimates moved by less than tol Fisher errors sqrt((F^-1)_bb) from
 * the previous ones.
 *   map: [n] in prob->mem;  chat_out [ns*nb] and F_out [(ns*nb)^2] (nullable, F at the last
 *   fiducial) in prob->mem;  cl_out [6][lmax+1] host (nullable): the last fiducial;  iters_out
 *   host (nullable).
 * CF_ENOCONV (outputs untouched) if max_iter iterations do not settle; the errors of cf_qml. */
int cf_qml_iterate(const cf_problem* prob, const cf_bins* bins, const double* map, int32_t max_iter,
                   double tol, double* chat_out, double* F_out, double* cl_out, int32_t* iters_out,
                   const cf_exec* ex, cf_report* rep);

/* Decorrelated normalisation (Sect. 2.5, Eq. decorrelated): out[v] = F^-1/2 q[v] with
 * F^-1/2 = U Xi^-1/2 U^T from the eigendecomposition F = U Xi U^T (cyclic Jacobi in FP64), the
 * eigenvalues below 1e-12 of the largest set to zero.  F: [K][K], only its lower triangle is read;
 * q, out: [nvec][K] (nvec = 0 with q = out = NULL computes only Fmhalf_out); Fmhalf_out: [K][K]
 * F^-1/2 (nullable; with it the caller can carry theory spectra through the same window F^1/2).
 * 1 <= K <= 1024.  All arrays in memory space mem.  A rotation is skipped when |a_pq| is at most
 * max(1e-15 sqrt(|a_pp a_qq|), 2e-17 |F|_F); CF_ENOCONV if a sweep still rotates after 60 sweeps;
 * cf_report.ir_iters = sweeps run.  Host arrays are checked for NaN/Inf (CF_EINVAL); device
 * arrays are not. */
int cf_decorrelate(const double* F, int32_t K, const double* q, int32_t nvec, int32_t mem, double* out,
                   double* Fmhalf_out, const cf_exec* ex, cf_report* rep);

/* ---------------------------------------------------------------------------------------------
 * Pixel likelihood through the harmonic basis with multipole switching (Sects. 2.3.2, 2.3.4, 2.6;
 * Eqs. C_switched, N_eff, K_kernel, smw, logdet).  The inference window is the multipole range
 * [win_lmin, win_lmax] on the harmonic fields win_fields (OR of CF_FIELD_T, CF_FIELD_E,
 * CF_FIELD_B, a subset of the problem's fields).  Everything outside it stays at the problem's
 * spectra prob->cl and is absorbed into N_eff = N + fixed signal (Eq. N_eff), factored once by
 * cf_smw_create together with the maps' solves.  Each point of cf_smw_loglike then costs one
 * Cholesky factorisation of a k_win x k_win matrix, k_win = nfields_win * ((win_lmax+1)^2 -
 * win_lmin^2), instead of one of the n x n pixel covariance:
 *   C = N_eff + V_win^T Lambda_win V_win,  Lambda_win = R R^T per multipole,
 *   -2 ln L = d^T N_eff^-1 d - |L^-1 R^T V_win N_eff^-1 d|^2 + ln|N_eff| + ln|I + R^T M R|,
 *   L L^T = I + R^T M R,  M = V_win N_eff^-1 V_win^T,
 * equal to the -2 ln L of cf_loglike_batch at the same spectra (n ln 2 pi excluded).
 * Requirements: every spectrum coupling a window field to a field outside the window vanishes in
 * prob->cl on [win_lmin, win_lmax] (else N_eff need not be positive definite: CF_EINVAL); each
 * point's spectra restricted to the window fields are positive semi-definite at every window
 * multipole (else CF_EINVAL).  Only those entries of a point's spectra are read.
 * ------------------------------------------------------------------------------------------- */
enum { CF_FIELD_T = 1, CF_FIELD_E = 2, CF_FIELD_B = 4 };
typedef struct cf_smw cf_smw;

/* Factor N_eff and solve the window's harmonic rows and the maps against it.  maps: [nmaps][n] in
 * prob->mem space.  The handle keeps device buffers of about 8 (k_win^2 + k_win nmaps) bytes on the
 * current device and copies of the geometry-independent data it needs; the problem and the maps
 * may be released after the call.  On error *out is left NULL.
 * Field groups (App. field_blocks): when the window holds T and E and/or B and N_eff couples no T
 * pixel with a Q, U pixel (no TE, TB in the fixed spectra, no T-P block in N), M has no T x (E,B)
 * block; the handle then records two groups (cf_report.ir_iters = 2, else 1). */
int cf_smw_create(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, uint32_t win_fields,
                  const double* maps, int32_t nmaps, const cf_exec* ex, cf_smw** out, cf_report* rep);

/* -2 ln L, chi^2 and ln|C| at npoints spectra, on the device the handle was created on.
 *   cl_points [npoints][6][lstride] (lstride >= lmax+1 of the problem)
 *   m2lnL [npoints][nmaps];  chi2 same shape (nullable);  logdet [npoints] (nullable)
 * Memory space of cl_points and the outputs: the problem's mem at creation.  Calls on one handle
 * must not overlap.  On a handle with two field groups, a call whose points all have TE and TB
 * equal to zero inside the window factorises K' as its T block and its E,B block separately
 * (k_T^3/3 + k_EB^3/3 instead of k_win^3/3 per point; cf_report.ir_iters = 2); any other call
 * factorises the dense K' (ir_iters = 1). */
int cf_smw_loglike(cf_smw* h, int32_t npoints, const double* cl_points, int32_t lstride, double* m2lnL,
                   double* chi2, double* logdet, const cf_exec* ex, cf_report* rep);

/* k_win of a handle (or -1), and its release (NULL is a no-op). */
int64_t cf_smw_dim(const cf_smw* h);
void cf_smw_destroy(cf_smw* h);

/* Fisher matrix and QML estimates in the harmonic basis with multipole switching (Sects. 2.3.3 and
 * 2.3.4; Eqs. projected_inv_smw, weighted_data_smw, q_harmonic, N_eff; App. smw_stable).  The
 * estimation window [win_lmin, win_lmax] holds every harmonic field of the problem; multipoles of
 * [lmin, lmax] outside it stay at the fiducial prob->cl and enter N_eff.  With M = V N_eff^-1 V^T,
 * b = V N_eff^-1 d, Lambda = R R^T at the fiducial and K' = I + R^T M R:
 *   Z = V C^-1 V^T = M R K'^-1 R^-1 (= M (I + Lambda M)^-1),  w = V C^-1 d = R^-T K'^-1 R^T b,
 *   noise bias b_b = 1/2 tr[E_b A T A^T], A = R^-T K'^-1 R^T, T = V N_eff^-1 N N_eff^-1 V^T,
 * then F, y, C_hat as in cf_qml; the results equal cf_qml's with the same bins (all inside the
 * window).  Needs Lambda positive definite at every window multipole (CF_EINVAL otherwise).
 * Outputs as cf_qml: y_out [nmaps][ns*nb], bias_out [ns*nb], chat_out [nmaps][ns*nb], F_out
 * [(ns*nb)^2] (nullable), all in prob->mem space; maps [nmaps][n].  FP64. */
int cf_smw_qml(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, const cf_bins* bins,
               const double* maps, int32_t nmaps, double* y_out, double* bias_out, double* chat_out,
               double* F_out, const cf_exec* ex, cf_report* rep);

/* Joint QML of two data sets of one sky (Sect. 2.2, cross-correlation; Eq. C_joint): the data
 * vector (d1, d2) has covariance [[S + N1, S + N12], [S + N12^T, S + N2]] and derivatives
 * [[P_b, P_b], [P_b, P_b]]; F, y, the noise bias (of the joint noise, N12 included) and C_hat are
 * those of the standard estimator (Eqs. fisher, q_ell, noise_bias, qml_estimate) on that
 * 2n-dimensional system.  Geometry, spectra, beam and pixel window are taken from p1; p2 supplies
 * the noise N2 and must match p1 in n, fields, l-range and memory space.  N12: dense n x n,
 * row-major, N12[i][j] = Cov(noise1_i, noise2_j), or NULL for independent noise.  maps1, maps2:
 * [nmaps][n] (map j of data set 1 pairs with map j of data set 2).  Outputs as cf_qml, all in
 * p1->mem space.  FP64.  CF_ENOTPD if the joint covariance is not positive definite. */
int cf_qml_joint(const cf_problem* p1, const cf_problem* p2, const double* N12, const cf_bins* bins,
                 const double* maps1, const double* maps2, int32_t nmaps, double* y_out, double* bias_out,
                 double* chat_out, double* F_out, const cf_exec* ex, cf_report* rep);

/* ---------------------------------------------------------------------------------------------
 * Cost-based choice of the computation basis for a likelihood scan (Sect. 3, the "auto" selector
 * of the ComputationBasis interface; per-point costs as in the complexity table of App. C).
 *   pixel:    npoints * (n^3/3 + n^2 nmaps)            (C = S + N factorised at every point)
 *   harmonic: n^3/3 + n^2 (k + nmaps) + n k (k + nmaps) (N_eff factorised once with the window's
 *             rows and the maps) + npoints * (k^3/3 + k^2 nmaps), with k = k_win, or with the
 *             T and E,B field groups factorised apart (k_T^3/3 + k_EB^3/3 + ...) when the fixed
 *             spectra carry no TE, TB and the noise has no T-P block (diagonal noise without a
 *             low-rank part, or a dense noise in host memory found block-diagonal).
 * The harmonic basis is chosen when it is cheaper and the window couples no varied field to a fixed
 * one (harmonic_ok); the caller states the window in which its points' spectra vary.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
  int32_t basis;          /* 0 pixel basis (cf_loglike_batch), 1 harmonic basis (cf_smw_*)        */
  int32_t harmonic_ok;    /* 0: the window couples a varied and a fixed field (pixel basis only) */
  int32_t groups;         /* field groups of the harmonic kernel (1, or 2: T | E,B)              */
  int64_t n, k_win;       /* data dimension and window modes                                   */
  double cost_pixel;      /* flops of the whole scan in the pixel basis                         */
  double cost_harmonic;   /* flops of the whole scan in the harmonic basis, setup included       */
} cf_basis_choice;

/* Fills *out for a scan of npoints points with nmaps maps over the window [win_lmin, win_lmax] on
 * win_fields (OR of CF_FIELD_T, CF_FIELD_E, CF_FIELD_B).  Host-only (no device work). */
int cf_select_basis(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, uint32_t win_fields,
                    int32_t npoints, int32_t nmaps, cf_basis_choice* out);

/* -2 ln L of one problem over npoints points in the basis cf_select_basis picks: the pixel basis
 * runs cf_loglike_batch (FP64), the harmonic basis creates a cf_smw handle for the window, runs
 * cf_smw_loglike and releases it.  The points' spectra must differ from prob->cl only inside the
 * window (the harmonic basis reads nothing else).  cl_points [npoints][6][lstride], maps [nmaps][n],
 * outputs m2lnL, chi2 [npoints][nmaps] and logdet [npoints] in prob->mem space; choice (host,
 * nullable) receives the selector's record. */
int cf_loglike_auto(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, uint32_t win_fields,
                    int32_t npoints, const double* cl_points, int32_t lstride, const double* maps,
                    int32_t nmaps, double* m2lnL, double* chi2, double* logdet, cf_basis_choice* choice,
                    const cf_exec* ex, cf_report* rep);

/* ---------------------------------------------------------------------------------------------
 * Likelihood emulator.  Not part of the paper's method: a surrogate of the -2 ln L of
 * cf_loglike_batch over a box of model parameters, whose uncertain or out-of-box queries are
 * sent back to the exact likelihood.
 *
 * Network: in_dim -> width -> ... -> width -> 1 (depth hidden layers, SiLU after each hidden
 * layer, linear output).  Hidden-to-hidden products run on bfloat16 operands with FP32
 * accumulation; the input and output layers, biases, master weights and Adam moments are FP32.
 * Parameters of one member, flat (cf_emu_param_count floats): for each layer l in order,
 * W_l [out][in] row-major then b_l [out].
 * Inputs are normalised to [-1, 1] on the per-parameter [min, max] box of the training inputs
 * (the hull).  The networks learn the residual of the targets about a least-squares polynomial
 * baseline in the normalised inputs (degree cf_emu_opts.baseline), standardised with the
 * residual's training mean and standard deviation; predictions add the baseline back.
 * The ensemble's prediction is the mean of its members; its spread is their sample standard
 * deviation (both in units of -2 ln L).
 * ------------------------------------------------------------------------------------------- */
typedef struct cf_emu cf_emu;

/* Spectra linear in the parameters: cl(x) = base + sum_k x_k basis_k, each [6][lstride]
 * (host memory).  The exact -2 ln L of a query x is cf_loglike_batch at cl(x). */
typedef struct {
  int32_t nparam;          /* = emulator in_dim                   */
  int32_t lstride;         /* >= lmax+1 of the exact problem      */
  const double* base;      /* [6][lstride]                        */
  const double* basis;     /* [nparam][6][lstride]                */
} cf_linear_spectra;

/* Training controls (NULL = defaults in brackets). */
typedef struct {
  int32_t epochs;          /* passes over the training split [200]                          */
  int32_t batch;           /* minibatch rows, 1..65536 [1024]                               */
  double lr;               /* Adam step size at the first step, cosine-decayed to 0 [1e-3]  */
  double beta1, beta2;     /* Adam moment decay [0.9, 0.999]                                */
  double eps;              /* Adam denominator guard [1e-8]                                 */
  double val_frac;         /* held-out fraction, 0 <= val_frac < 1 [0.1]                    */
  int32_t baseline;        /* degree 0, 1 or 2 of the polynomial fitted to the targets by    */
                           /* least squares before the networks learn the residual [2]       */
} cf_emu_opts;

/* Create an ensemble of `ensemble` (1..16) networks with in_dim 1..8 inputs, width 64, 128 or
 * 256 and depth 1..8 hidden layers on the current device.  Weights are drawn uniformly in
 * +-1/sqrt(fan_in) from a splitmix64 stream seeded with seed + member; Adam moments are zero. */
int cf_emu_create(int32_t in_dim, int32_t width, int32_t depth, int32_t ensemble, uint64_t seed,
                  cf_emu** out);
void cf_emu_destroy(cf_emu* emu);
int64_t cf_emu_param_count(const cf_emu* emu);   /* floats per member, or -1 */
/* Shape of an ensemble (any output pointer may be NULL). */
int cf_emu_shape(const cf_emu* emu, int32_t* in_dim, int32_t* width, int32_t* depth, int32_t* ensemble);

/* Train every member on (x [N][in_dim], y [N]) in memory space `mem` with MSE loss and Adam.
 * A seeded random split keeps val_frac of the rows out of training.  The first call fixes the
 * hull, the baseline and the target scaling; later calls continue from the current weights and
 * moments.
 * Report: ms_total device time, flops algorithmic, est_err = {final training loss (standardised
 * MSE, member mean), held-out RMS error, held-out max |error|, held-out mean spread} (-2 ln L units;
 * zero when nothing is held out), ir_iters = optimiser steps of this call. */
int cf_emu_train(cf_emu* emu, const double* x, const double* y, int64_t N, int32_t mem,
                 const cf_emu_opts* opts, const cf_exec* ex, cf_report* rep);

/* Predict -2 ln L for N queries x [N][in_dim] (memory space `mem`, as are y_out, spread_out and
 * used_fallback).  A query needs the exact likelihood when it lies outside the hull or its spread
 * exceeds spread_max.  With exact_prob, exact_map ([n] in exact_prob->mem space) and model given,
 * those queries are evaluated by cf_loglike_batch (FP64) at cl(x) and flagged in used_fallback;
 * with exact_prob NULL the ensemble mean is returned for every query and used_fallback marks the
 * queries that would need the exact likelihood.  spread_out, used_fallback nullable.
 * Report: ms_total wall time of the call, n_fallback, est_err[0] ms of the ensemble inference,
 * est_err[1] ms of the exact evaluations. */
int cf_emu_predict(cf_emu* emu, const double* x, int64_t N, int32_t mem, double spread_max,
                   const cf_problem* exact_prob, const cf_linear_spectra* model,
                   const double* exact_map, double* y_out, double* spread_out,
                   uint8_t* used_fallback, const cf_exec* ex, cf_report* rep);

/* cf_emu_predict with the exact fallback through a harmonic-basis likelihood handle (cf_smw_create
 * with one map): queries outside the hull or with spread above spread_max get cf_smw_loglike at
 * cl(x) (FP64).  The handle evaluates the model's spectra inside its window (its fields and
 * multipoles) and holds everything else at the fiducial it was made with, so its values equal the
 * exact pixel likelihood when the model varies the spectra only inside that window.  The memory
 * space of the handle (its problem's mem) need not match `mem`. */
int cf_emu_predict_smw(cf_emu* emu, const double* x, int64_t N, int32_t mem, double spread_max,
                       const cf_smw* exact_smw, const cf_linear_spectra* model, double* y_out,
                       double* spread_out, uint8_t* used_fallback, const cf_exec* ex, cf_report* rep);

/* Inspection and checking of the networks (host memory, raw network units: inputs already
 * normalised, outputs and targets standardised).
 *   cf_emu_get_params / set_params: FP32 master parameters of one member (set refreshes the
 *     bfloat16 copies; moments are kept).
 *   cf_emu_forward: out [ensemble][N] member outputs.
 *   cf_emu_gradient: grad [ensemble][P] gradient of mean((f(x) - y)^2) over the N rows, loss
 *     [ensemble] (nullable) its value; the weights are not changed.
 *   cf_emu_adam: one Adam step of every member with the given gradient [ensemble][P] and step
 *     size lr (moment decays of the last cf_emu_train options, else the defaults). */
int cf_emu_get_params(const cf_emu* emu, int32_t member, float* out);
int cf_emu_set_params(cf_emu* emu, int32_t member, const float* in);
int cf_emu_forward(cf_emu* emu, const double* x, int64_t N, float* out);
int cf_emu_gradient(cf_emu* emu, const double* x, const double* y, int64_t N, float* grad,
                    double* loss);
int cf_emu_adam(cf_emu* emu, const float* grad, double lr);

/* Write / read the whole emulator state (shape, weights, moments, step count, hull, scaling,
 * optimiser constants) as a little-endian binary file. cf_emu_load creates on the current device. */
int cf_emu_save(const cf_emu* emu, const char* path);
int cf_emu_load(const char* path, cf_emu** out);

/* Thread-local description of the last error on this thread. */
const char* cf_last_error(void);

/* Library version string. */
const char* cf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CF_H */
