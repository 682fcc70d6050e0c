// Internal declarations of libcf (host launchers and shared device helpers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <vector>

struct cf_smw;   // the harmonic-basis likelihood handle of the C ABI

namespace cf {

// Memory space and number of maps of a harmonic-basis handle (false for NULL).
bool smw_describe(const ::cf_smw* h, int* mem, int* nmaps);

// -------------------------------------------------------------------------------------------
// Launch-time error plumbing: launchers return hipError_t; the API layer converts to cf_status.
// -------------------------------------------------------------------------------------------
#define CF_HIP_TRY(expr)                                  \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return _e;                      \
  } while (0)

constexpr int kMaxL = 1024;          // lmax bound of the ABI
constexpr int kNB = 64;              // diagonal block of the blocked Cholesky / triangular solves
constexpr int kPixRec = 10;          // doubles per pixel record: n(3), e_theta(3), e_phi(2), z, phi
constexpr int kCoef = 8;             // doubles per multipole of the recurrence table
constexpr int kCovIB = 8;            // scan points sharing one pixel-pair recurrence in k_cov_build

// Per-multipole recurrence coefficients (table [lmax+1][kCoef]):
//   0: aP, 1: gP            P_{l+1}   = aP mu P_l - gP P_{l-1}
//   2: a2, 3: b2, 4: g2     d_{2,+-2}^{l+1} = (a2 mu -+ b2) d^l - g2 d^{l-1}
//   5: a0, 6: g0            d_{20}^{l+1}  = a0 mu d^l - g0 d^{l-1}
//   7: sqrt((2l+1)/(4 pi))

// Device-side problem geometry / weights.
struct DevProblem {
  int npx;            // retained pixels
  int nmaps;          // 1 (T), 2 (QU) or 3 (TQU)
  int has_t, has_p;   // T present, Q/U present
  int n;              // nmaps * npx
  int lmin, lmax;
  int kf;             // modes per harmonic field: (lmax+1)^2 - lmin^2
  int nfm;            // harmonic fields: 1 (T), 2 (E,B), 3 (T,E,B)
  int64_t k;          // total modes nfm * kf
  const double* pix;  // [npx][kPixRec]
  const double* coef; // [lmax+1][kCoef]
  const double* cw;   // [6][lmax+1] c^XY_l = (2l+1)/(4pi) C^XY_l W_l (zero below lmin) for XY = TT,
                      // EE + BB, EE - BB, TE, TB, EB
  const double* wl;   // [lmax+1] W_l
  const double* lam;  // [6][lmax+1] C^XY_l W_l (mode covariance)
};

// ---------------------------------------------------------------- geometry / tables
hipError_t launch_geometry(const int* ring_idx, int nside, const double* theta, const double* phi,
                           int npx, double* pix, hipStream_t s);
// Items (scan points) i < nitems: spectra at cl + i*cl_stride, row x at + x*cl_ld.
// Outputs cw, lam: [nitems][6][lmax+1]; wl, coef: item 0 only (nullable).
// i0p (nullable): device-side item offset added to every item index (captured scan batches).
// interleave > 1: cw instead laid out [chunk][lmax+1][6][interleave] (item i in chunk
// i / interleave, slot i % interleave), zero-filled up to a whole number of chunks.
hipError_t launch_tables(const double* cl, const double* bl, const double* pl, int lmin, int lmax,
                         int nitems, int64_t cl_stride, int64_t cl_ld, double* cw, double* wl,
                         double* lam, double* coef, hipStream_t s, const int64_t* i0p = nullptr,
                         int interleave = 1);

// ---------------------------------------------------------------- covariance assembly
// C (n x n, ld) = S + N for a batch: C advances by c_stride per batch item.  interleave 1: cw
// [item][6][lmax+1], advancing by cw_stride per item; interleave kCovIB: cw in the interleaved
// layout of launch_tables, advancing by cw_stride per chunk of kCovIB items.
// lower_only: write only entries on or below the diagonal.  noise_kind 0 diag [n], 1 dense [n][n].
hipError_t launch_cov_build(const DevProblem& P, const double* cw, int64_t cw_stride, int nbatch,
                            int noise_kind, const double* noise, int noise_rank,
                            const double* noise_U, double* C, int64_t ldc, int64_t c_stride,
                            int lower_only, int* flag, hipStream_t s, int interleave = 1);

// ---------------------------------------------------------------- dense FP64 kernels
struct GemmDesc {
  int64_t M, N, K;
  const double* A; int64_t lda; int at;   // at: A(i,k) = A[k*lda+i] else A[i*lda+k]
  const double* B; int64_t ldb; int bt;   // bt: B(k,j) = B[j*ldb+k] else B[k*ldb+j]
  double* C; int64_t ldc;
  double alpha, beta;
  int lower;                              // skip output tiles strictly above the diagonal
  int64_t diag_off;                       // with lower: the diagonal is col = row + diag_off
  int batch; int64_t sA, sB, sC;          // batch count and element strides
  int mode;                               // 0 FP64 MFMA, 1 FP32 MFMA, 2 split-BF16 x3 MFMA
  int tag;                                // 1: Z = G^T G (a separately named kernel instance)
  int tile;                               // 0: by size; 64 or 128: that workgroup tile
  int prio;                               // wave priority (0-3) of the launch's waves (s_setprio):
                                          // critical-path work wins SIMD issue over bulk updates
};
hipError_t gemm_f64(const GemmDesc& g, hipStream_t s);

// Events around every FP64 GEMM launch of the calling thread while a call with stage timing is
// running (g_ktimer set by the API layer); resolved into cf_report.gemm_* when the call finishes.
constexpr int kGemmIds = 16;
struct KernTimer {
  struct Rec { int id; hipEvent_t a, b; double flops, bytes; };
  std::vector<Rec> rec;
};
extern thread_local KernTimer* g_ktimer;

// A (batched) Cholesky factor with the inverses of its diagonal blocks.  Users of a factor read
// the blocks below the diagonal and the inverted 64 x 64 diagonal blocks.
struct Factor {
  double* L = nullptr; int64_t n = 0, ld = 0, sL = 0;   // row-major, lower; batch stride sL
  // Extra rows below the n x n matrix (rows n .. rows-1, same ld) are carried through the
  // factorisation like rows of a larger matrix: on return they hold B L^-T for their input B,
  // i.e. the transposed forward solve (L^-1 B^T)^T.  Panels ending at or before column p_early
  // only touch rows below rows_early (callers put rows that vanish on those columns last).
  int64_t rows = 0;                                    // 0: n
  int64_t rows_early = 0, p_early = 0;
  double* Li64 = nullptr; int64_t sLi64 = 0;           // [ceil(n/64)][64][64] inverted 64-blocks
  double* Li256 = nullptr; int64_t sLi256 = 0;         // [n/256][256][256] inverted full 256-blocks (nullable)
  double* ldpart = nullptr; int64_t sPart = 0;         // [ceil(n/64)] per-block sums of ln L_ii
  int* fail = nullptr;                                 // first non-positive pivot (atomicMin)
  int batch = 1;
  int mode = 0;                                        // GEMM mode of the bulk updates and solves
  int panel = 0;                                       // outer panel width (0: 256 single, 512 batched)
  int tile = 0;                                        // GEMM tile of the updates (0: by size)
};
// Streams for the factorisation: s carries the critical path (diagonal blocks, panels and the
// lookahead column update), s1 the bulk trailing updates, s2 the 256-block inverses.
struct Streams {
  hipStream_t s, s1, s2;
  hipEvent_t eL, eB, eI;
  hipEvent_t* ring = nullptr;   // 4 events: host-side pacing of the panel loop (nullable)
  // Lookahead update issued on s1 ahead of the trailing update (eA: its completion), for streams
  // whose s owns only a few CUs; nullptr: the lookahead runs on s.
  hipEvent_t eA = nullptr;
  // Set (and eA unset): the trailing update is split in two, the panel after next first (eT: its
  // completion), so that the next lookahead waits only for those columns (lookahead of depth two).
  // Measured: batch of 8 at n = 5952 16.45 -> 16.21 ms; the single factorisation, whose lookahead
  // runs on the bulk CUs, was slower with the second part on its solve-row stream (9.3 -> 10.2 ms).
  hipEvent_t eT = nullptr;
};
// Scratch for the 256-block inverses: batch * (2*64*64 + 128*128) doubles.
inline int64_t potrf_scratch(int batch) { return (int64_t)batch * (2 * 64 * 64 + 128 * 128); }
// Factor F.L in place (right-looking, lookahead of one 256-column panel); on return every stream
// of st has been joined into st.s.
hipError_t potrf_f64(Factor& F, double* scratch, const Streams& st);

// Forward substitution G = L^-1 Y for rows [r0, n) (rows of Y below r0 are taken as zero;
// the solve starts at the 64-row block holding r0).  Y (n x ncol, ldy) is consumed as workspace.
hipError_t trsm_lower_f64(const Factor& F, double* Y, int64_t ldy, int64_t sY, double* G, int64_t ldg,
                          int64_t sG, int64_t ncol, int64_t r0, hipStream_t s);

// Backward substitution X = L^-T B (B, n x ncol, consumed as workspace; result in X).
hipError_t trsm_lower_t_f64(const Factor& F, double* B, int64_t ldb, int64_t sB, double* X, int64_t ldx,
                            int64_t sX, int64_t ncol, hipStream_t s);

// W[j][m] = sum_{i < K} A[i][j] U[i][m] for skinny U (nmaps <= 8): partial sums over 32 row chunks
// in `part` ([32][M][nmaps]) reduced in a fixed order.
// W[r][m] = A[r][:] . U[m][:] (rows of A, row-major ld lda, K columns; nmaps <= 8 rows of U, ld
// ldu; W ld ldw).  Rows r >= rskip read only columns >= c0 (the caller guarantees zeros before).
hipError_t launch_rowdot(const double* A, int64_t lda, int64_t M, int64_t K, const double* U, int64_t ldu,
                         int nmaps, double* W, int64_t ldw, int64_t rskip, int64_t c0, hipStream_t s);
hipError_t gemv_tn(const double* A, int64_t lda, int64_t M, int64_t K, const double* U, int nmaps,
                   double* W, int64_t ldw, double* part, hipStream_t s);

// ---------------------------------------------------------------- harmonic basis
// Y (npix x k, ld ldy); the E,B columns start pgap columns after the T columns (room for
// other columns solved together with Y).
hipError_t launch_ybuild(const DevProblem& P, double* Y, int64_t ldy, hipStream_t s, int64_t pgap = 0);

// ---------------------------------------------------------------- Fisher / QML reductions
hipError_t launch_symmetrize(double* Z, int64_t k, int64_t ldz, hipStream_t s);
// Gram[l][l'][p][q] for l >= l' (p, q over the nfm^2 field pairs, upper-triangular q >= p).
hipError_t launch_gram(const DevProblem& P, const double* Z, int64_t ldz, double* gram,
                       double* ztr, hipStream_t s);
// Cross Gram of Z1 and Z2 (cross-QML): per l >= l', the nfm^4 values <Z2^{p1}, Z1^{p2}>.
hipError_t launch_gram_cross(const DevProblem& P, const double* Z1, const double* Z2, int64_t ldz, double* gx,
                             hipStream_t s);
struct SpecSel {
  int ns;            // selected spectra
  int spec[6];       // spectrum ids (0..5 TT,EE,BB,TE,TB,EB)
  int nb;            // bins
  const int* lo;     // device [nb]
  const int* hi;     // device [nb]
};
hipError_t launch_fisher_assemble(const DevProblem& P, const SpecSel& S, const double* gram,
                                  double* F, hipStream_t s,
                                  bool cross = false);
hipError_t launch_bias_assemble(const DevProblem& P, const SpecSel& S, const double* gram,
                                const double* ztr, double* bias, hipStream_t s);
hipError_t launch_quad_assemble(const DevProblem& P, const SpecSel& S, const double* w, int64_t ldw,
                                int nmaps, double* y, hipStream_t s,
                                const double* w2 = nullptr);
// Cholesky solve of the small SPD system F X = R (k x k, nrhs columns given as rows [nrhs][k]).
hipError_t launch_small_spd_solve(double* F, int k, const double* R, double* X, int nrhs, int* fail,
                                  hipStream_t s);
hipError_t launch_transpose(const double* A, int64_t rows, int64_t cols, int64_t lda, double* B,
                            int64_t ldb, hipStream_t s);
hipError_t launch_colsumsq(const double* U, int64_t rows, int64_t cols, int64_t ldu, int64_t sU,
                           int batch, double* out, int64_t sOut, hipStream_t s);
// out[b][r] = sum_c X[b][r][c]^2 for a batch of row-major (rows x cols, ld ldx) matrices.
hipError_t launch_rowsumsq(const double* X, int64_t rows, int64_t cols, int64_t ldx, int64_t sX, int batch,
                           double* out, int64_t sOut, hipStream_t s);
// Stochastic log-det correction of a mixed-precision factor: probe blocks (+-1 by a counter hash)
// written (sub = 0) or subtracted (sub = 1) for B blocks of n x m, and ld[b] += mean over the m
// probes of t1 - n - t2 / 2.
hipError_t launch_probes(double* P, int64_t n, int64_t m, int B, int sub, hipStream_t s);
hipError_t launch_ld_correct(double* ld, const double* t1, const double* t2, int B, int64_t m, int64_t n,
                             hipStream_t s);
// A[r][c] = v over a rows x cols block (leading dimension ld).
hipError_t launch_fill_block(double* A, int64_t ld, int64_t rows, int64_t cols, double v, hipStream_t s);
hipError_t launch_coldot(const double* U, const double* V, int64_t rows, int64_t cols, int64_t ld,
                         int64_t sU, int64_t sV, int batch, double* out, int64_t sOut, hipStream_t s);
hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s);
// out[i][j] += d[i] X[i][j] (rows x cols, row-major)
hipError_t launch_rowscale_add(const double* d, const double* X, double* out, int64_t rows, int64_t cols,
                              hipStream_t s);
hipError_t launch_sum_parts(const double* parts, int nparts, int64_t sP, int batch, double* out,
                            int64_t sOut, hipStream_t s);
hipError_t launch_add_scalar(const double* vec, int64_t nper, int batch, const double* scal,
                             double* out, hipStream_t s);
hipError_t launch_sub_bias(double* q, const double* bias, int K, int nmaps, hipStream_t s);
hipError_t launch_scan_finish(const double* chi2b, const double* ldb, int B, int nmaps, int64_t i0,
                              int prob, int nprob, double* m2, double* chi2, double* logdet,
                              hipStream_t s, const int64_t* i0p = nullptr);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s);

// ---------------------------------------------------------------- decorrelated normalisation
// R = F^-1/2 (lower triangle of F [K][K] read, K <= 1024) by one-workgroup cyclic Jacobi: A, U, R
// [K][K] and w [K] scratch/outputs (U eigenvectors, w the cut Xi^-1/2); info[2]: sweeps, not
// converged.  out[v] = R q[v] for nvec rows q [nvec][K].
hipError_t launch_inverse_sqrt(const double* F, int K, double* A, double* U, double* w, double* R,
                               int max_sweeps, double cutoff, int* info, hipStream_t s);
hipError_t launch_apply_rows(const double* R, const double* q, int K, int nvec, double* out, hipStream_t s);

// ---------------------------------------------------------------- harmonic-basis likelihood
// Per-point pieces of the SMW likelihood with multipole switching (smw.hip).  Window modes are
// [field slot][l][m] over nf varied fields (fld: harmonic fields T 0, E 1, B 2), kwf per field.
// R: [batch][nl][3][3] lower factors of Lambda_l; K: per point a slot of [kw + nmaps][kw].
hipError_t launch_smw_lambda(const double* cl, int64_t cl_stride, int64_t cl_ld, const double* wl, int wlo,
                             int nl, int nf, const int* fld, int batch, double* R, int* bad, hipStream_t s);
hipError_t launch_smw_kernel(const double* M, int64_t ldm, int64_t kw, int64_t kwf, int nf, int wlo, int nl,
                             const double* R, int batch, double* K, int64_t slot, hipStream_t s);
// out = B A (right = 0; A is k x other) or A B (right = 1; A is other x k) with B the per-mode block
// operator of one point's R (kind 0 R, 1 R^T, 2 R^-1, 3 R^-T) over nf window fields of kwf modes;
// out must not alias A.
hipError_t launch_apply_rblock(const double* A, int64_t lda, double* out, int64_t ldo, int64_t other, int64_t kwf,
                              int nf, int wlo, const double* R, int kind, int right, hipStream_t s);
// flag |= 1 if any entry of nb blocks rows x cols (leading dimension ld, stride sb) is non-zero.
hipError_t launch_any_nonzero(const double* A, int64_t ld, int64_t rows, int64_t cols, int64_t sb, int nb,
                              int* flag, hipStream_t s);
hipError_t launch_smw_rhs(const double* b, int nmaps, int64_t kw, int64_t kwf, int nf, int wlo, int nl,
                          const double* R, int batch, double* K, int64_t slot, hipStream_t s);
hipError_t launch_smw_finish(const double* chi2N, const double* ldN, const double* x2b, const double* ldK,
                             int B, int nmaps, int64_t i0, double* m2, double* chi2, double* logdet,
                             hipStream_t s);

// ---------------------------------------------------------------- likelihood emulator
// Error text for cf_last_error() from code outside the API translation unit.
int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

struct EmuNet {                 // device state of an ensemble
  int in, W, D, E;              // inputs (<= 8), width (64/128/256), hidden layers, members
  int64_t P;                    // FP32 parameters per member
  float* master;                // [E][P]
  float* m;                     // [E][P] Adam first moments
  float* v;                     // [E][P] Adam second moments
  __bf16* wq;                   // [E][D-1][2][W][W]: W_l and W_l^T (l = 1..D-1) in bfloat16
};
struct EmuTrain {               // one minibatch
  int64_t n;                    // valid rows
  int64_t rows;                 // rows rounded up to a multiple of 64
  const float* xn;              // [*][8] normalised inputs
  const float* yn;              // [*] standardised targets
  const int* idx;               // [E][idx_stride] source rows of this batch, NULL = identity
  int64_t idx_stride;
  float scale;                  // 2 / n
  __bf16* hq;                   // [E][D-1][rows][W] hidden activations h_0..h_{D-2}
  float* z;                     // [E][D-1][rows][W] pre-activations z_1..z_{D-2}
  float* hD;                    // [E][rows][W] h_{D-1}
  float* d;                     // [E][D][rows][W] deltas of the hidden layers
  float* dout;                  // [E][rows] output deltas
  float* sq;                    // [E][rows] squared residuals
  float* xb;                    // [E][rows][8] gathered inputs
};
struct EmuAdam {
  float lr, b1, b2, eps, c1, c2;   // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
  int do_adam;                     // apply the update (else only write grad)
  float* grad;                     // [E][P] gradient output, nullable
  float* loss;                     // [E] mean squared residual, nullable
  float inv_n;
};
// Input box and target model: u = (2x - lo - hi) / (hi - lo); the networks learn
// (y - q(u) - ymu) / ysig with q a polynomial baseline of degree qdeg (0, 1 or 2) whose
// coefficients qc are ordered 1, u_k (k < in), u_i u_j (i <= j, row by row).
constexpr int kEmuQ = 45;
struct EmuScale {
  double lo[8], hi[8], ymu, ysig;
  int qdeg;
  double qc[kEmuQ];
};
__host__ __device__ inline int emu_nfeat(int in, int qdeg) {
  return qdeg <= 0 ? 0 : (qdeg == 1 ? 1 + in : 1 + in + in * (in + 1) / 2);
}
__host__ __device__ inline double emu_baseline(const EmuScale& sc, const double* u, int in) {
  if (sc.qdeg <= 0) return 0.0;
  double s = sc.qc[0];
  int o = 1;
  for (int k = 0; k < in; ++k) s += sc.qc[o++] * u[k];
  if (sc.qdeg >= 2)
    for (int i = 0; i < in; ++i)
      for (int j = i; j < in; ++j) s += sc.qc[o++] * u[i] * u[j];
  return s;
}
struct EmuInfer {
  const double* x;              // [n][in]
  int64_t n;
  int raw;                      // 1: x already normalised, no routing outputs
  EmuScale sc;
  double spread_max;
  double* y;                    // [n] ensemble mean (-2 ln L units)
  double* spread;               // [n] ensemble sample standard deviation, nullable
  uint8_t* flag;                // [n] 1 = outside the hull or spread > spread_max
  float* raw_out;               // [E][n] member outputs, nullable
};

int64_t emu_param_count(int in, int W, int D);
int64_t emu_off_w(int l, int in, int W, int D);
hipError_t launch_emu_train_step(const EmuNet& net, const EmuTrain& tr, const EmuAdam& A, hipStream_t s);
hipError_t launch_emu_infer(const EmuNet& net, const EmuInfer& q, hipStream_t s);
hipError_t launch_emu_adam(const EmuNet& net, const float* grad, const EmuAdam& A, hipStream_t s);
hipError_t launch_emu_refresh(const EmuNet& net, hipStream_t s);
hipError_t launch_emu_prep(const double* x, const double* y, const int* rows, int64_t n, int in,
                           const EmuScale& sc, float* xn, float* yn, hipStream_t s);
hipError_t launch_emu_scatter(const double* val, const int* idx, int64_t n, double* y, hipStream_t s);

}  // namespace cf
