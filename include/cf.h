/*
 * cf.h — C ABI of libcf, the MI355X (gfx950) hot path of QML power-spectrum
 * estimation and the pixel-space Gaussian likelihood of
 * "CosmoForge I" (Galloni & Pagano), Sects. 2.1-2.6 and Apps. A-C.
 *
 * Every entry point runs its whole computation in HIP kernels on the current
 * HIP device and returns only when the results are written.  Calls that use
 * the same device are serialised by the library (one workspace per device).
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
  void* stream;           /* hipStream_t to run on; NULL = the library's stream */
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
 * fisher_harmonic, sparse_trace).  F_out: [(ns*nb)^2] in prob->mem space. */
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

/* Pixel likelihood over a parameter scan (Eq. pixel_likelihood, Sect. 2.6):
 *   -2 ln L_{i,p,j} = d_{p,j}^T C_{i,p}^-1 d_{p,j} + ln|C_{i,p}|  (n ln 2 pi excluded)
 * for points i < npoints, problems p < nprob and maps j < nmaps.
 *   cl_points [npoints][nprob][6][lstride]: spectra of each point and problem, lstride >= lmax_p+1
 *   maps[p]   [nmaps][n_p]
 *   m2lnL     [npoints][nprob][nmaps];  chi2 same shape (nullable);  logdet [npoints][nprob] (nullable)
 * Geometry, beam, window and noise come from probs[p]; its cl is not used.  Memory space
 * of cl_points, maps and outputs: probs[0].mem. */
int cf_loglike_batch(const cf_problem* probs, int32_t nprob, int32_t npoints,
                     const double* cl_points, int32_t lstride, const double* const* maps,
                     int32_t nmaps, int32_t precision, double* m2lnL, double* chi2,
                     double* logdet, const cf_exec* ex, cf_report* rep);

/* Thread-local description of the last error on this thread. */
const char* cf_last_error(void);

/* Library version string. */
const char* cf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CF_H */
