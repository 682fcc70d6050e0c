// Fisher matrix, noise bias and QML quadratic forms from Z = Y^T C^-1 Y (paper Eqs. fisher_harmonic,
// sparse_trace, q_harmonic; App. C.1), plus the small dense helpers of the path.
//
// Z is ordered [field][l][m].  For every multipole pair (l >= l') one workgroup forms the Gram
// matrix of the field blocks Z^{ad}_{ll'} (rows: field a at l, columns: field d at l'):
//   gram[(a,d),(b,c)] = <Z^{ad}_{ll'}, Z^{bc}_{ll'}>_F ,
// which is all the sparse trace of Eq. sparse_trace needs: for spectra XY, X'Y' with field-pair
// sets sigma(XX) = {(X,X)}, sigma(XY) = {(X,Y),(Y,X)},
//   F = 1/2 sum_{l in b, l' in b'} W_l W_l' sum_{(a,c) in sigma} sum_{(a',c') in sigma'} gram_{ll'}[(c,a'),(a,c')].
// The same Gram entries give the noise bias through 1/2 tr[E_b (Z - Z Lambda Z)]:
//   b = 1/2 sum_{l in b} W_l sum_{(a,c)} ( tr Z^{ca}_{ll} - sum_{l'} sum_{f,g} Lambda_l'[f,g] gram_{ll'}[(c,f),(a,g)] ).
#include "cf_internal.h"
#include <climits>

namespace cf {
namespace {

__device__ __forceinline__ int qidx(int p1, int p2, int np) {   // p1 <= p2
  return p1 * (2 * np - p1 + 1) / 2 + (p2 - p1);
}

// Z lower triangle -> full symmetric, through 32 x 32 LDS tiles.
__global__ __launch_bounds__(256) void k_symmetrize(double* Z, int64_t k, int64_t ldz) {
  __shared__ double t[32][33];
  const int64_t bi = blockIdx.y, bj = blockIdx.x;   // source tile (bi, bj) with bi > bj, lower
  if (bj >= bi) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    int64_t gr = bi * 32 + r, gc = bj * 32 + tx;
    t[r][tx] = (gr < k && gc < k) ? Z[gr * ldz + gc] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int64_t gr = bj * 32 + r, gc = bi * 32 + tx;     // transposed destination (upper)
    if (gr < k && gc < k) Z[gr * ldz + gc] = t[tx][r];
  }
}
// diagonal 32 x 32 tiles: copy lower to upper in place
__global__ __launch_bounds__(256) void k_symmetrize_diag(double* Z, int64_t k, int64_t ldz) {
  const int64_t b = blockIdx.x;
  for (int idx = threadIdx.x; idx < 32 * 32; idx += 256) {
    int r = idx / 32, c = idx % 32;
    int64_t gr = b * 32 + r, gc = b * 32 + c;
    if (c > r && gr < k && gc < k) Z[gr * ldz + gc] = Z[gc * ldz + gr];
  }
}

template <int NF>
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ Z, int64_t ldz, int lmin,
                                              int lmax, int kf, double* __restrict__ gram,
                                              double* __restrict__ ztr) {
  constexpr int NP = NF * NF, NQ = NP * (NP + 1) / 2;
  __shared__ double red[NQ > NP ? NQ : NP][257];
  const int pid = blockIdx.x;
  // pid -> (li >= lj)
  int li = (int)((sqrt(8.0 * pid + 1.0) - 1.0) * 0.5);
  while (li * (li + 1) / 2 > pid) --li;
  while ((li + 1) * (li + 2) / 2 <= pid) ++li;
  const int lj = pid - li * (li + 1) / 2;
  const int l = lmin + li, lp = lmin + lj;
  const int nm = 2 * l + 1, nmp = 2 * lp + 1;
  const int64_t rb = (int64_t)l * l - (int64_t)lmin * lmin;
  const int64_t cb = (int64_t)lp * lp - (int64_t)lmin * lmin;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  const int tot = nm * nmp;
  for (int e = threadIdx.x; e < tot; e += 256) {
    const int m = e / nmp, mp = e % nmp;
    double z[NP];
#pragma unroll
    for (int a = 0; a < NF; ++a)
#pragma unroll
      for (int d = 0; d < NF; ++d)
        z[a * NF + d] = Z[((int64_t)a * kf + rb + m) * ldz + (int64_t)d * kf + cb + mp];
    int q = 0;
#pragma unroll
    for (int p1 = 0; p1 < NP; ++p1)
#pragma unroll
      for (int p2 = p1; p2 < NP; ++p2) { acc[q] = fma(z[p1], z[p2], acc[q]); ++q; }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int q = threadIdx.x; q < NQ; q += 256) {
    double s = 0.0;
    for (int t = 0; t < 256; ++t) s += red[q][t];
    gram[(int64_t)pid * NQ + q] = s;
  }
  if (li == lj) {
    __syncthreads();
    double tr[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) tr[p] = 0.0;
    for (int m = threadIdx.x; m < nm; m += 256) {
#pragma unroll
      for (int a = 0; a < NF; ++a)
#pragma unroll
        for (int d = 0; d < NF; ++d)
          tr[a * NF + d] += Z[((int64_t)a * kf + rb + m) * ldz + (int64_t)d * kf + rb + m];
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) red[p][threadIdx.x] = tr[p];
    __syncthreads();
    for (int p = threadIdx.x; p < NP; p += 256) {
      double s = 0.0;
      for (int t = 0; t < 256; ++t) s += red[p][t];
      ztr[(int64_t)li * NP + p] = s;
    }
  }
}

// Cross Gram of two projected inverses (cross-QML): for every l >= l' and every pair of field
// pairs, gx[(p1, p2)] = <Z2^{p1}_{l l'}, Z1^{p2}_{l l'}>_F with p = a * NF + d (no symmetry in
// (p1, p2), so all NP^2 are kept).  Per-thread partial sums, then a fixed-order wave and
// workgroup reduction.
template <int NF>
__global__ __launch_bounds__(256) void k_gram_cross(const double* __restrict__ Z1, const double* __restrict__ Z2,
                                                    int64_t ldz, int lmin, int kf, double* __restrict__ gx) {
  constexpr int NP = NF * NF, NQ = NP * NP;
  __shared__ double red[4][NQ];
  const int pid = blockIdx.x;
  int li = (int)((sqrt(8.0 * pid + 1.0) - 1.0) * 0.5);
  while (li * (li + 1) / 2 > pid) --li;
  while ((li + 1) * (li + 2) / 2 <= pid) ++li;
  const int lj = pid - li * (li + 1) / 2;
  const int l = lmin + li, lp = lmin + lj;
  const int nm = 2 * l + 1, nmp = 2 * lp + 1;
  const int64_t rb = (int64_t)l * l - (int64_t)lmin * lmin;
  const int64_t cb = (int64_t)lp * lp - (int64_t)lmin * lmin;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int e = threadIdx.x; e < nm * nmp; e += 256) {
    const int m = e / nmp, mp = e % nmp;
    double z1[NP], z2[NP];
#pragma unroll
    for (int a = 0; a < NF; ++a)
#pragma unroll
      for (int d = 0; d < NF; ++d) {
        const int64_t at = ((int64_t)a * kf + rb + m) * ldz + (int64_t)d * kf + cb + mp;
        z1[a * NF + d] = Z1[at];
        z2[a * NF + d] = Z2[at];
      }
#pragma unroll
    for (int p1 = 0; p1 < NP; ++p1)
#pragma unroll
      for (int p2 = 0; p2 < NP; ++p2) acc[p1 * NP + p2] = fma(z2[p1], z1[p2], acc[p1 * NP + p2]);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NQ; q += 256)
    gx[(int64_t)pid * NQ + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
}

// spectrum id (0..5 = TT,EE,BB,TE,TB,EB) -> its absolute field letters (0 T, 1 E, 2 B)
__device__ __forceinline__ void spec_fields(int s, int& x, int& y) {
  const int X[6] = {0, 1, 2, 0, 0, 1}, Yv[6] = {0, 1, 2, 1, 2, 2};
  x = X[s]; y = Yv[s];
}
__device__ __forceinline__ int field_pair_spec(int f, int g) {   // absolute letters -> spectrum id
  const int tab[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  return tab[f][g];
}

struct GramView {
  const double* gram;
  int lmin, nf, np, nq;
  int cross;      // 1: gram holds the full cross Gram <Z2^{p1}, Z1^{p2}> (np^2 per l >= l')
  int off;        // absolute letter -> harmonic field index: idx = letter - off (QU: E->0, B->1)
  __device__ double get(int l, int lp, int x, int y, int u, int v) const {
    // <Z^{xy}_{l l'}, Z^{uv}_{l l'}> with fields as harmonic indices
    int li = l - lmin, lj = lp - lmin;
    int p1, p2;
    if (li >= lj) { p1 = x * nf + y; p2 = u * nf + v; }
    else { int t = li; li = lj; lj = t; p1 = y * nf + x; p2 = v * nf + u; }
    int64_t pid = (int64_t)li * (li + 1) / 2 + lj;
    if (cross) return gram[(pid * np + p1) * np + p2];   // <Z2^{xy}, Z1^{uv}>: order kept
    if (p1 > p2) { int t = p1; p1 = p2; p2 = t; }
    return gram[pid * nq + qidx(p1, p2, np)];
  }
};

__global__ void k_fisher_assemble(GramView G, int ns, int s0, int s1, int s2, int s3, int s4, int s5,
                                  int nb, const int* lo, const int* hi, const double* wl, double* F) {
  const int K = ns * nb;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * K) return;
  const int A = idx / K, B = idx % K;
  if (A < B) return;                   // one evaluation per symmetric pair, mirrored below
  const int specs[6] = {s0, s1, s2, s3, s4, s5};
  const int sa = specs[A / nb], ba = A % nb, sb = specs[B / nb], bb = B % nb;
  int xa, ya, xb, yb;
  spec_fields(sa, xa, ya);
  spec_fields(sb, xb, yb);
  xa -= G.off; ya -= G.off; xb -= G.off; yb -= G.off;
  const int npa = (xa == ya) ? 1 : 2, npb = (xb == yb) ? 1 : 2;
  double sum = 0.0;
  for (int l = lo[ba]; l <= hi[ba]; ++l) {
    for (int lp = lo[bb]; lp <= hi[bb]; ++lp) {
      double t = 0.0;
      for (int u = 0; u < npa; ++u) {
        const int a = u ? ya : xa, c = u ? xa : ya;
        for (int v = 0; v < npb; ++v) {
          const int a2 = v ? yb : xb, c2 = v ? xb : yb;
          t += G.get(l, lp, c, a2, a, c2);
        }
      }
      sum = fma(wl[l] * wl[lp], t, sum);
    }
  }
  F[idx] = 0.5 * sum;
  F[(int64_t)B * K + A] = 0.5 * sum;
}

// One workgroup per parameter A: the (l, sigma, l', f, g) terms are spread over the threads and
// reduced in a fixed order.
__global__ __launch_bounds__(256) void k_bias_assemble(GramView G, const double* ztr, int lmin, int lmax,
                                                       int ns, int s0, int s1, int s2, int s3, int s4,
                                                       int s5, int nb, const int* lo, const int* hi,
                                                       const double* wl, const double* lam,
                                                       double* bias) {
  __shared__ double red[256];
  const int A = blockIdx.x;
  const int specs[6] = {s0, s1, s2, s3, s4, s5};
  const int sa = specs[A / nb], ba = A % nb;
  int xa, ya;
  spec_fields(sa, xa, ya);
  const int L = lmax + 1, nl = lmax - lmin + 1;
  const int nf = G.nf, nff = nf * nf;
  const int npa = (xa == ya) ? 1 : 2;
  const int l0 = lo[ba], nlb = hi[ba] - lo[ba] + 1;
  // term index t = ((lb * npa + u) * nl + lpi) * nff + fg ; plus the trace terms
  const int nterm = nlb * npa * nl * nff;
  double acc = 0.0;
  for (int t = threadIdx.x; t < nterm; t += 256) {
    const int fg = t % nff, r1 = t / nff;
    const int lpi = r1 % nl, r2 = r1 / nl;
    const int u = r2 % npa, lb = r2 / npa;
    const int l = l0 + lb, lp = lmin + lpi;
    const int f = fg / nf, g = fg % nf;
    const double lv = lam[field_pair_spec(f + G.off, g + G.off) * L + lp];
    if (lv == 0.0) continue;
    const int a = (u ? ya : xa) - G.off, c = (u ? xa : ya) - G.off;
    acc -= wl[l] * lv * G.get(l, lp, c, f, a, g);
  }
  for (int t = threadIdx.x; t < nlb * npa; t += 256) {
    const int u = t % npa, lb = t / npa, l = l0 + lb;
    const int a = (u ? ya : xa) - G.off, c = (u ? xa : ya) - G.off;
    acc += wl[l] * ztr[(l - lmin) * nff + c * nf + a];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bias[A] = 0.5 * red[0];
}

// y[map][A] = 1/2 sum_{l in b} W_l sum_{(a,c) in sigma} sum_m w[a,l,m] w[c,l,m];  w is [k][ldw].
// With w2 (cross-QML, Eq. q_cross): the bilinear form 1/2 sum w1[a] w2[c] over sigma instead.
__global__ void k_quad_assemble(const double* w, const double* w2, int64_t ldw, int nmaps, int lmin, int kf,
                                int off, int ns, int s0, int s1, int s2, int s3, int s4, int s5, int nb,
                                const int* lo, const int* hi, const double* wl, double* y) {
  const int K = ns * nb;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * nmaps) return;
  const int map = idx / K, A = idx % K;
  const int specs[6] = {s0, s1, s2, s3, s4, s5};
  const int sa = specs[A / nb], ba = A % nb;
  int xa, ya;
  spec_fields(sa, xa, ya);
  xa -= off; ya -= off;
  double sum = 0.0;
  for (int l = lo[ba]; l <= hi[ba]; ++l) {
    const int64_t base = (int64_t)l * l - (int64_t)lmin * lmin;
    double t = 0.0;
    if (w2) {
      for (int m = 0; m < 2 * l + 1; ++m) {
        const int64_t ia = ((int64_t)xa * kf + base + m) * ldw + map, ic = ((int64_t)ya * kf + base + m) * ldw + map;
        t = fma(w[ia], w2[ic], t);
        if (xa != ya) t = fma(w[ic], w2[ia], t);
      }
    } else {
      for (int m = 0; m < 2 * l + 1; ++m) {
        const double wa = w[((int64_t)xa * kf + base + m) * ldw + map];
        const double wc = w[((int64_t)ya * kf + base + m) * ldw + map];
        t = fma(wa, wc, t);
      }
      if (xa != ya) t *= 2.0;
    }
    sum = fma(wl[l], t, sum);
  }
  y[(int64_t)map * K + A] = 0.5 * sum;
}

// Single-workgroup Cholesky solve of a small SPD system: F (k x k, overwritten with its factor),
// right-hand sides R [nrhs][k] -> X [nrhs][k].  The factorisation is right-looking with one
// barrier per column (threads on a 32 x 32 grid of row/column strides); the substitutions run one
// right-hand side per wave with the dot products reduced across the wave.  KS > 0: the matrix is
// worked on in LDS (k <= KS; copied in and the factor copied back), the same operations in the same
// order as on F in place (KS = 0), so both give the same bits; in place, every column step reads
// and writes device memory (a k = 72 solve: 154 us).
template <int KS>
__global__ __launch_bounds__(1024) void k_small_spd_solve(double* F, int k, const double* R, double* X,
                                                          int nrhs, int* fail) {
  constexpr int XS = KS > 0 ? KS : 1024;
  __shared__ double xs[16][XS];
  __shared__ double Ls[KS > 0 ? KS * (KS + 1) : 1];
  const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
  double* M = KS > 0 ? Ls : F;
  const int ld = KS > 0 ? KS + 1 : k;
  if constexpr (KS > 0) {
    for (int idx = tid; idx < k * k; idx += blockDim.x) Ls[(idx / k) * ld + idx % k] = F[idx];
    __syncthreads();
  }
  for (int j = 0; j < k; ++j) {
    const double d = M[j * ld + j];
    const double inv = 1.0 / d;
    for (int r = j + 1 + ty; r < k; r += 32) {
      const double fr = M[r * ld + j] * inv;
      for (int q = j + 1 + tx; q <= r; q += 32) M[r * ld + q] -= fr * M[q * ld + j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < k * k; idx += blockDim.x) {
    const int r = idx / k, q = idx % k;
    if (q < r) M[r * ld + q] /= sqrt(M[q * ld + q]);
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < k; ++j) {
      const double d = M[j * ld + j];
      if (!(d > 0.0) || !isfinite(d)) { atomicMin(fail, j); break; }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < k; idx += blockDim.x) M[idx * ld + idx] = sqrt(M[idx * ld + idx]);
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  double* x = xs[wave];
  for (int rr = wave; rr < nrhs; rr += 16) {
    const double* b = R + (int64_t)rr * k;
    for (int i = 0; i < k; ++i) {            // L y = b
      double p = 0.0;
      for (int q = lane; q < i; q += 64) p = fma(M[i * ld + q], x[q], p);
      for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o);
      if (lane == 0) x[i] = (b[i] - p) / M[i * ld + i];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
    for (int i = k - 1; i >= 0; --i) {       // L^T x = y
      double p = 0.0;
      for (int q = i + 1 + lane; q < k; q += 64) p = fma(M[q * ld + i], x[q], p);
      for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o);
      if (lane == 0) x[i] = (x[i] - p) / M[i * ld + i];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
    for (int i = lane; i < k; i += 64) X[(int64_t)rr * k + i] = x[i];
    __builtin_amdgcn_wave_barrier();
  }
  if constexpr (KS > 0) {
    __syncthreads();
    for (int idx = tid; idx < k * k; idx += blockDim.x) F[idx] = Ls[(idx / k) * ld + idx % k];
  }
}

__global__ void k_transpose(const double* A, int64_t rows, int64_t cols, int64_t lda, double* B,
                            int64_t ldb) {
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  for (int r = ty; r < 32; r += 8)
    t[r][tx] = (r0 + r < rows && c0 + tx < cols) ? A[(r0 + r) * lda + c0 + tx] : 0.0;
  __syncthreads();
  for (int r = ty; r < 32; r += 8)
    if (c0 + r < cols && r0 + tx < rows) B[(c0 + r) * ldb + r0 + tx] = t[tx][r];
}

// out[b][j] = sum_i U[b][i*ldu + j*cs]^2: one workgroup per (column, batch item), fixed-order tree sum.
__global__ __launch_bounds__(256) void k_colsumsq(const double* U, int64_t rows, int64_t cols, int64_t ldu,
                                                  int64_t cs, int64_t sU, double* out, int64_t sOut) {
  __shared__ double red[256];
  const int64_t j = blockIdx.x;
  const double* u = U + blockIdx.z * sU + j * cs;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) { const double v = u[i * ldu]; s = fma(v, v, s); }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.z * sOut + j] = red[0];
}

// out[b][j] = sum_i U[b][i][j] V[b][i][j]: one workgroup per (column, batch item), fixed order.
__global__ __launch_bounds__(256) void k_coldot(const double* U, const double* V, int64_t rows, int64_t ld,
                                                int64_t sU, int64_t sV, double* out, int64_t sOut) {
  __shared__ double red[256];
  const int64_t j = blockIdx.x;
  const double* u = U + blockIdx.z * sU + j;
  const double* v = V + blockIdx.z * sV + j;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) s = fma(u[i * ld], v[i * ld], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.z * sOut + j] = red[0];
}

// out[i][j] += d[i] X[i][j] for a rows x cols row-major X (a diagonal matrix applied from the left)
__global__ void k_rowscale_add(const double* d, const double* X, double* out, int64_t rows, int64_t cols) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  out[t] += d[t / cols] * X[t];
}

__global__ void k_axpy(double* y, const double* x, double a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], y[i]);
}

__global__ void k_sum_parts(const double* parts, int nparts, int64_t sP, double* out, int64_t sOut) {
  if (threadIdx.x != 0) return;
  const double* p = parts + blockIdx.x * sP;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += p[i];
  out[blockIdx.x * sOut] = 2.0 * s;
}

__global__ void k_add_scalar(const double* vec, int64_t nper, const double* scal, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nper) return;
  out[blockIdx.y * nper + i] = vec[blockIdx.y * nper + i] + scal[blockIdx.y];
}

__global__ void k_sub_bias(double* q, const double* bias, int K, int nmaps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K * nmaps) q[i] -= bias[i % K];
}

// Scatter a batch of per-point chi^2 [B][nmaps] and ln|C| [B] into the scan outputs
// [npoints][nprob][nmaps] (m2lnL, chi2) and [npoints][nprob] (logdet).
__global__ void k_scan_finish(const double* chi2b, const double* ldb, int B, int nmaps, int64_t i0h,
                              int prob, int nprob, double* m2, double* chi2, double* logdet,
                              const int64_t* i0p) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * nmaps) return;
  const int64_t i0 = i0p ? *i0p : i0h;
  const int b = idx / nmaps, j = idx % nmaps;
  const int64_t row = (i0 + b) * nprob + prob;
  const double x = chi2b[idx], l = ldb[b];
  m2[row * nmaps + j] = x + l;
  if (chi2) chi2[row * nmaps + j] = x;
  if (logdet && j == 0) logdet[row] = l;
}

// Skinny A^T U: part[chunk][j][m] = sum over the chunk's rows i of A[i][j] U[i][m].
template <int NM>
__global__ __launch_bounds__(256) void k_gemv_tn_part(const double* __restrict__ A, int64_t lda, int64_t M,
                                                      int64_t K, const double* __restrict__ U,
                                                      double* __restrict__ part, int64_t rows_per) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * rows_per;
  const int64_t i1 = (i0 + rows_per < K) ? i0 + rows_per : K;
  double acc[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) acc[m] = 0.0;
  if (j < M) {
    for (int64_t i = i0; i < i1; ++i) {
      const double a = A[i * lda + j];
#pragma unroll
      for (int m = 0; m < NM; ++m) acc[m] = fma(a, U[i * NM + m], acc[m]);
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) part[((int64_t)blockIdx.y * M + j) * NM + m] = acc[m];
  }
}
// W[r][m] = sum_c A[r][c] U[m][c] for rows r of A (row-major, ld lda) and NM rows of U (ld ldu):
// one wave per row, lanes stride over the columns two at a time, a fixed-order shuffle reduction.
// Rows r >= rskip start at column c0 (their entries before it are zero).
template <int NM>
__global__ __launch_bounds__(256) void k_rowdot(const double* __restrict__ A, int64_t lda, int64_t M,
                                                int64_t K, const double* __restrict__ U, int64_t ldu,
                                                double* __restrict__ W, int64_t ldw, int64_t rskip,
                                                int64_t c0) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= M) return;
  const double* a = A + r * lda;
  double acc[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) acc[m] = 0.0;
  int64_t c = (r >= rskip ? c0 : 0) & ~int64_t(1);
  for (c += 2 * lane; c + 1 < K; c += 128) {
    const double a0 = a[c], a1 = a[c + 1];
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[m] = fma(a1, U[m * ldu + c + 1], fma(a0, U[m * ldu + c], acc[m]));
  }
  if (c < K) {
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[m] = fma(a[c], U[m * ldu + c], acc[m]);
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    double v = acc[m];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) W[r * ldw + m] = v;
  }
}

__global__ void k_gemv_tn_reduce(const double* part, int64_t M, int nm, int nchunk, double* W, int64_t ldw) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * nm) return;
  const int64_t j = idx / nm;
  const int m = (int)(idx % nm);
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[((int64_t)c * M + j) * nm + m];
  W[j * ldw + m] = s;
}

__global__ void k_fill(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_int(int* p, int64_t n, int v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

GramView make_view(const DevProblem& P, const double* gram) {
  GramView G;
  G.gram = gram; G.lmin = P.lmin; G.nf = P.nfm; G.np = P.nfm * P.nfm;
  G.nq = G.np * (G.np + 1) / 2;
  G.off = P.has_t ? 0 : 1;   // QU only: E is harmonic field 0
  G.cross = 0;
  return G;
}

}  // namespace

hipError_t launch_symmetrize(double* Z, int64_t k, int64_t ldz, hipStream_t s) {
  const int64_t nt = (k + 31) / 32;
  hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)nt, (unsigned)nt), dim3(256), 0, s, Z, k, ldz);
  CF_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_symmetrize_diag, dim3((unsigned)nt), dim3(256), 0, s, Z, k, ldz);
  return hipGetLastError();
}

hipError_t launch_gram(const DevProblem& P, const double* Z, int64_t ldz, double* gram, double* ztr,
                       hipStream_t s) {
  const int nl = P.lmax - P.lmin + 1;
  const unsigned npairs = (unsigned)(nl * (nl + 1) / 2);
  switch (P.nfm) {
    case 1: hipLaunchKernelGGL(k_gram<1>, dim3(npairs), dim3(256), 0, s, Z, ldz, P.lmin, P.lmax, P.kf, gram, ztr); break;
    case 2: hipLaunchKernelGGL(k_gram<2>, dim3(npairs), dim3(256), 0, s, Z, ldz, P.lmin, P.lmax, P.kf, gram, ztr); break;
    case 3: hipLaunchKernelGGL(k_gram<3>, dim3(npairs), dim3(256), 0, s, Z, ldz, P.lmin, P.lmax, P.kf, gram, ztr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram_cross(const DevProblem& P, const double* Z1, const double* Z2, int64_t ldz, double* gx,
                             hipStream_t s) {
  const int nl = P.lmax - P.lmin + 1;
  const unsigned npairs = (unsigned)(nl * (nl + 1) / 2);
  switch (P.nfm) {
    case 1: hipLaunchKernelGGL(k_gram_cross<1>, dim3(npairs), dim3(256), 0, s, Z1, Z2, ldz, P.lmin, P.kf, gx); break;
    case 2: hipLaunchKernelGGL(k_gram_cross<2>, dim3(npairs), dim3(256), 0, s, Z1, Z2, ldz, P.lmin, P.kf, gx); break;
    case 3: hipLaunchKernelGGL(k_gram_cross<3>, dim3(npairs), dim3(256), 0, s, Z1, Z2, ldz, P.lmin, P.kf, gx); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fisher_assemble(const DevProblem& P, const SpecSel& S, const double* gram,
                                  double* F, hipStream_t s, bool cross) {
  const int K = S.ns * S.nb;
  GramView G = make_view(P, gram);
  G.cross = cross ? 1 : 0;
  hipLaunchKernelGGL(k_fisher_assemble, dim3(blocks((int64_t)K * K, 128)), dim3(128), 0, s,
                     G, S.ns, S.spec[0], S.spec[1], S.spec[2], S.spec[3], S.spec[4],
                     S.spec[5], S.nb, S.lo, S.hi, P.wl, F);
  return hipGetLastError();
}

hipError_t launch_bias_assemble(const DevProblem& P, const SpecSel& S, const double* gram,
                                const double* ztr, double* bias, hipStream_t s) {
  const int K = S.ns * S.nb;
  hipLaunchKernelGGL(k_bias_assemble, dim3(K), dim3(256), 0, s, make_view(P, gram), ztr,
                     P.lmin, P.lmax, S.ns, S.spec[0], S.spec[1], S.spec[2], S.spec[3], S.spec[4],
                     S.spec[5], S.nb, S.lo, S.hi, P.wl, P.lam, bias);
  return hipGetLastError();
}

hipError_t launch_quad_assemble(const DevProblem& P, const SpecSel& S, const double* w, int64_t ldw,
                                int nmaps, double* y, hipStream_t s, const double* w2) {
  const int K = S.ns * S.nb;
  hipLaunchKernelGGL(k_quad_assemble, dim3(blocks((int64_t)K * nmaps, 128)), dim3(128), 0, s, w, w2, ldw,
                     nmaps, P.lmin, P.kf, P.has_t ? 0 : 1, S.ns, S.spec[0], S.spec[1], S.spec[2],
                     S.spec[3], S.spec[4], S.spec[5], S.nb, S.lo, S.hi, P.wl, y);
  return hipGetLastError();
}

hipError_t launch_small_spd_solve(double* F, int k, const double* R, double* X, int nrhs, int* fail,
                                  hipStream_t s) {
  if (k <= 96)
    hipLaunchKernelGGL(k_small_spd_solve<96>, dim3(1), dim3(1024), 0, s, F, k, R, X, nrhs, fail);
  else
    hipLaunchKernelGGL(k_small_spd_solve<0>, dim3(1), dim3(1024), 0, s, F, k, R, X, nrhs, fail);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* A, int64_t rows, int64_t cols, int64_t lda, double* B,
                            int64_t ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3(blocks(cols, 32), blocks(rows, 32)), dim3(256), 0, s, A, rows,
                     cols, lda, B, ldb);
  return hipGetLastError();
}

hipError_t launch_colsumsq(const double* U, int64_t rows, int64_t cols, int64_t ldu, int64_t sU,
                           int batch, double* out, int64_t sOut, hipStream_t s) {
  hipLaunchKernelGGL(k_colsumsq, dim3((unsigned)cols, 1, batch), dim3(256), 0, s, U, rows, cols, ldu,
                     (int64_t)1, sU, out, sOut);
  return hipGetLastError();
}

hipError_t launch_rowsumsq(const double* X, int64_t rows, int64_t cols, int64_t ldx, int64_t sX, int batch,
                           double* out, int64_t sOut, hipStream_t s) {
  hipLaunchKernelGGL(k_colsumsq, dim3((unsigned)rows, 1, batch), dim3(256), 0, s, X, cols, rows, (int64_t)1,
                     ldx, sX, out, sOut);
  return hipGetLastError();
}

hipError_t launch_coldot(const double* U, const double* V, int64_t rows, int64_t cols, int64_t ld,
                         int64_t sU, int64_t sV, int batch, double* out, int64_t sOut, hipStream_t s) {
  hipLaunchKernelGGL(k_coldot, dim3((unsigned)cols, 1, batch), dim3(256), 0, s, U, V, rows, ld, sU, sV, out, sOut);
  return hipGetLastError();
}

hipError_t launch_rowscale_add(const double* d, const double* X, double* out, int64_t rows, int64_t cols,
                              hipStream_t s) {
  const int64_t nt = rows * cols;
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rowscale_add, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, d, X, out, rows, cols);
  return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(blocks(n, 256)), dim3(256), 0, s, y, x, a, n);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const double* parts, int nparts, int64_t sP, int batch, double* out,
                            int64_t sOut, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3(batch), dim3(64), 0, s, parts, nparts, sP, out, sOut);
  return hipGetLastError();
}

hipError_t launch_add_scalar(const double* vec, int64_t nper, int batch, const double* scal,
                             double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_add_scalar, dim3(blocks(nper, 64), batch), dim3(64), 0, s, vec, nper, scal, out);
  return hipGetLastError();
}

hipError_t launch_sub_bias(double* q, const double* bias, int K, int nmaps, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_bias, dim3(blocks((int64_t)K * nmaps, 256)), dim3(256), 0, s, q, bias, K, nmaps);
  return hipGetLastError();
}

hipError_t launch_scan_finish(const double* chi2b, const double* ldb, int B, int nmaps, int64_t i0,
                              int prob, int nprob, double* m2, double* chi2, double* logdet,
                              hipStream_t s, const int64_t* i0p) {
  hipLaunchKernelGGL(k_scan_finish, dim3(blocks((int64_t)B * nmaps, 256)), dim3(256), 0, s, chi2b, ldb,
                     B, nmaps, i0, prob, nprob, m2, chi2, logdet, i0p);
  return hipGetLastError();
}

// Probe vectors of the stochastic log-det correction: entry (i, j) of the n x m probe block is
// +1 or -1 by the low bit of splitmix64 (Steele, Lea and Flood 2014) of the counter i * m + j,
// the same for every point of a batch.
__device__ __forceinline__ double probe_sign(int64_t i, int64_t j, int64_t m) {
  uint64_t z = 0x3c6ef372fe94f82aull + (uint64_t)(i * m + j) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (z & 1) ? 1.0 : -1.0;
}

// P[b][i][j] = z(i, j) (sub = 0) or P[b][i][j] -= z(i, j) (sub = 1), P: B blocks of n x m.
__global__ void k_probes(double* P, int64_t n, int64_t m, int B, int sub) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * n * m) return;
  const int64_t r = idx % (n * m), i = r / m, j = r % m;
  const double z = probe_sign(i, j, m);
  P[idx] = sub ? P[idx] - z : z;
}

// ld[b] += (1/m) sum_j (t1[b][j] - n - t2[b][j] / 2): the estimate of tr X - |X|_F^2 / 2 with
// t1 = z^T X z + z^T z and t2 = |X z|^2 per probe.
__global__ void k_ld_correct(double* ld, const double* t1, const double* t2, int B, int64_t m, int64_t n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int64_t j = 0; j < m; ++j) s += (t1[b * m + j] - (double)n) - 0.5 * t2[b * m + j];
  ld[b] += s / (double)m;
}

// A[r][c] = v for r < rows, c < cols (leading dimension ld).
__global__ void k_fill_block(double* A, int64_t ld, int64_t rows, int64_t cols, double v) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  A[(idx / cols) * ld + idx % cols] = v;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { if (threadIdx.x == 0) *p = v; }
__global__ void k_add_i64(int64_t* p, int64_t v) { if (threadIdx.x == 0) *p += v; }

hipError_t launch_probes(double* P, int64_t n, int64_t m, int B, int sub, hipStream_t s) {
  const int64_t tot = (int64_t)B * n * m;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_probes, dim3(blocks(tot, 256)), dim3(256), 0, s, P, n, m, B, sub);
  return hipGetLastError();
}

hipError_t launch_ld_correct(double* ld, const double* t1, const double* t2, int B, int64_t m, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_ld_correct, dim3((B + 63) / 64), dim3(64), 0, s, ld, t1, t2, B, m, n);
  return hipGetLastError();
}

hipError_t launch_fill_block(double* A, int64_t ld, int64_t rows, int64_t cols, double v, hipStream_t s) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_block, dim3(blocks(tot, 256)), dim3(256), 0, s, A, ld, rows, cols, v);
  return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t gemv_tn(const double* A, int64_t lda, int64_t M, int64_t K, const double* U, int nmaps,
                   double* W, int64_t ldw, double* part, hipStream_t s) {
  constexpr int NCH = 32;
  const int64_t rows_per = (K + NCH - 1) / NCH;
  dim3 grid(blocks(M, 256), NCH);
  switch (nmaps) {
#define CF_GV(NMv) case NMv: hipLaunchKernelGGL(k_gemv_tn_part<NMv>, grid, dim3(256), 0, s, A, lda, M, K, U, part, rows_per); break;
    CF_GV(1) CF_GV(2) CF_GV(3) CF_GV(4) CF_GV(5) CF_GV(6) CF_GV(7) CF_GV(8)
#undef CF_GV
    default: return hipErrorInvalidValue;
  }
  CF_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_gemv_tn_reduce, dim3(blocks(M * nmaps, 256)), dim3(256), 0, s, part, M, nmaps, NCH, W, ldw);
  return hipGetLastError();
}

hipError_t launch_rowdot(const double* A, int64_t lda, int64_t M, int64_t K, const double* U, int64_t ldu,
                         int nmaps, double* W, int64_t ldw, int64_t rskip, int64_t c0, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  dim3 grid((unsigned)((M + 3) / 4));
  switch (nmaps) {
#define CF_RD(NMv) case NMv: hipLaunchKernelGGL(k_rowdot<NMv>, grid, dim3(256), 0, s, A, lda, M, K, U, ldu, W, ldw, rskip, c0); break;
    CF_RD(1) CF_RD(2) CF_RD(3) CF_RD(4) CF_RD(5) CF_RD(6) CF_RD(7) CF_RD(8)
#undef CF_RD
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace cf
