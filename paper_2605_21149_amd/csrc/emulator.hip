// Likelihood emulator networks: fused row-tile forward / backward kernels on bfloat16 MFMA,
// weight-gradient tiles with the Adam update fused into their epilogue, and ensemble inference
// with hull and spread routing.
//
// Network of one member: h_0 = silu(W_0 x + b_0) (FP32 VALU, in_dim <= 8 inputs),
// h_l = silu(W_l h_{l-1} + b_l) for l = 1..D-1 (width x width, bfloat16 operands into
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation), f = W_D h_{D-1} + b_D (FP32 VALU).
// Flat FP32 parameters per member: for l = 0..D, W_l [out][in] row-major then b_l [out].
//
// A row tile is 64 rows on 256 threads (4 waves).  Wave w owns output columns
// [w*width/4, (w+1)*width/4) of every hidden layer; with the MFMA lane layout (output register i
// of lane l is row 4*(l/16) + i, column l%16 of a 16x16 tile) every lane owns the same
// (row, column) set in all layers, so pre-activations saved in the forward pass are read back by
// the lane that wrote them.  The backward data pass (the deltas of every layer) is row-local and
// runs in the same kernel; the weight gradients, which reduce over the batch, run in a second
// kernel whose tiles apply Adam to the entries they own.
#include "cf_internal.h"

namespace cf {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kTM = 64;      // rows per tile
constexpr int kXin = 8;      // padded input width

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ float adam_update(float* p, float* m, float* v, float g, const EmuAdam& A) {
  const float mm = A.b1 * *m + (1.0f - A.b1) * g;
  const float vv = A.b2 * *v + (1.0f - A.b2) * g * g;
  *m = mm;
  *v = vv;
  const float np = *p - A.lr * (mm * A.c1) / (sqrtf(vv * A.c2) + A.eps);
  *p = np;
  return np;
}

// acc[a][b]: rows 16a + (0..15), columns cw + 16b + (0..15) of  H (LDS, [64][W+8]) x B, with
// B(k, c) = Wg[c*W + k] (bfloat16, global).
template <int W>
__device__ __forceinline__ void mma_layer(const __bf16* __restrict__ H, const __bf16* __restrict__ Wg,
                                          int cw, int lane, flt4 (&acc)[4][W / 64]) {
  constexpr int NB = W / 64, LDH = W + 8;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < W; k0 += 32) {
    bf16x8 A[4], B[NB];
#pragma unroll
    for (int a = 0; a < 4; ++a) A[a] = *reinterpret_cast<const bf16x8*>(H + (16 * a + lr) * LDH + k0 + lk);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      B[b] = *reinterpret_cast<const bf16x8*>(Wg + (int64_t)(cw + 16 * b + lr) * W + k0 + lk);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], B[b], acc[a][b], 0, 0, 0);
  }
}

// z_0 for the lane's elements: acc[a][b][i] = b_0[c] + sum_k x[r][k] W_0[c][k].
template <int W>
__device__ __forceinline__ void input_layer(const float* __restrict__ P, int in, const float* xs, int cw,
                                            int lane, flt4 (&acc)[4][W / 64]) {
  constexpr int NB = W / 64;
  const int lr = lane & 15, rg = (lane >> 4) * 4;
  const float* W0 = P;
  const float* b0 = P + (int64_t)W * in;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c = cw + 16 * b + lr;
    float w[kXin];
#pragma unroll
    for (int k = 0; k < kXin; ++k) w[k] = k < in ? W0[c * in + k] : 0.0f;
    const float bias = b0[c];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float* xr = xs + (16 * a + rg + i) * kXin;
        float z = bias;
#pragma unroll
        for (int k = 0; k < kXin; ++k) z = fmaf(xr[k], w[k], z);
        acc[a][b][i] = z;
      }
  }
}

// Write silu(acc) as bfloat16 into the LDS tile H ([64][W+8]).
template <int W>
__device__ __forceinline__ void store_act(__bf16* H, int cw, int lane, const flt4 (&acc)[4][W / 64]) {
  constexpr int NB = W / 64, LDH = W + 8;
  const int lr = lane & 15, rg = (lane >> 4) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) H[(16 * a + rg + i) * LDH + cw + 16 * b + lr] = (__bf16)silu(acc[a][b][i]);
}

// Store / load the lane's elements of a [rows][W] FP32 array (rows from row0).
template <int W>
__device__ __forceinline__ void store_lane(float* G, int64_t row0, int cw, int lane, const flt4 (&v)[4][W / 64]) {
  constexpr int NB = W / 64;
  const int lr = lane & 15, rg = (lane >> 4) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) G[(row0 + 16 * a + rg + i) * W + cw + 16 * b + lr] = v[a][b][i];
}

// Copy the bfloat16 tile H ([64][W+8] LDS) to rows row0.. of G ([rows][W]).
template <int W>
__device__ __forceinline__ void copy_tile_out(const __bf16* H, __bf16* G, int64_t row0, int tid) {
  constexpr int LDH = W + 8, C8 = W / 8;
  for (int q = tid; q < kTM * C8; q += 256) {
    const int r = q / C8, c = (q % C8) * 8;
    *reinterpret_cast<bf16x8*>(G + (row0 + r) * W + c) = *reinterpret_cast<const bf16x8*>(H + r * LDH + c);
  }
}

__host__ __device__ __forceinline__ int64_t off_w(int l, int in, int W, int D) {
  return l == 0 ? 0 : (int64_t)W * in + W + (int64_t)(l - 1) * ((int64_t)W * W + W);
}
__host__ __device__ __forceinline__ int64_t off_b(int l, int in, int W, int D) {
  return off_w(l, in, W, D) + (l == 0 ? (int64_t)W * in : (l < D ? (int64_t)W * W : (int64_t)W));
}

// Forward pass of member e over the tile; on return acc holds z_{D-1} and red[0..255] the
// per-wave partial output sums (valid after a barrier).  TRAIN: saves h_l (l < D-1, bfloat16),
// z_l (1 <= l < D-1) and h_{D-1} (FP32) for the backward passes.
template <int W, bool TRAIN>
__device__ __forceinline__ void forward(const EmuNet& net, int e, const float* xs, __bf16* Hb, float* red,
                                        flt4 (&acc)[4][W / 64], const EmuTrain* tr, int64_t row0,
                                        int wave, int lane, int tid, int* cur_out) {
  constexpr int NB = W / 64, LDH = W + 8;
  const int in = net.in, D = net.D;
  const float* P = net.master + (int64_t)e * net.P;
  const int cw = wave * (W / 4);
  const int lr = lane & 15, rg = (lane >> 4) * 4;
  input_layer<W>(P, in, xs, cw, lane, acc);
  int cur = 0;
  for (int l = 1; l < D; ++l) {
    store_act<W>(Hb + cur * kTM * LDH, cw, lane, acc);
    __syncthreads();
    if (TRAIN) copy_tile_out<W>(Hb + cur * kTM * LDH, tr->hq + ((int64_t)e * (D - 1) + (l - 1)) * tr->rows * W, row0, tid);
    const __bf16* Wq = net.wq + ((int64_t)e * (D - 1) + (l - 1)) * 2 * W * W;
    mma_layer<W>(Hb + cur * kTM * LDH, Wq, cw, lane, acc);
    const float* bl = P + off_b(l, in, W, D);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float bias = bl[cw + 16 * b + lr];
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] += bias;
    }
    if (TRAIN && l < D - 1) store_lane<W>(tr->z + ((int64_t)e * (D - 1) + (l - 1)) * tr->rows * W, row0, cw, lane, acc);
    cur ^= 1;
  }
  // output layer: per-wave partial sums of silu(z_{D-1}) . W_D
  const float* wD = P + off_w(D, in, W, D);
  float wo[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) wo[b] = wD[cw + 16 * b + lr];
  if (TRAIN) {
    flt4 h[4][NB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) h[a][b][i] = silu(acc[a][b][i]);
    store_lane<W>(tr->hD + (int64_t)e * tr->rows * W, row0, cw, lane, h);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float s = 0.0f;
#pragma unroll
      for (int b = 0; b < NB; ++b) s = fmaf(silu(acc[a][b][i]), wo[b], s);
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      s += __shfl_xor(s, 8);
      if (lr == 0) red[wave * kTM + 16 * a + rg + i] = s;
    }
  *cur_out = cur;
}

// ------------------------------------------------------------------------------ training rows
// One tile of one member: gather rows, forward, loss, output delta, deltas of every hidden layer.
template <int W>
__global__ __launch_bounds__(256) void k_emu_train_rows(EmuNet net, EmuTrain tr) {
  constexpr int NB = W / 64, LDH = W + 8;
  __shared__ __align__(16) __bf16 Hb[2 * kTM * LDH];
  __shared__ float xs[kTM * kXin];
  __shared__ float red[4 * kTM];
  __shared__ float dsh[kTM];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int e = blockIdx.y;
  const int D = net.D, in = net.in;
  const int64_t row0 = (int64_t)blockIdx.x * kTM;
  const int* idx = tr.idx ? tr.idx + (int64_t)e * tr.idx_stride : nullptr;
  for (int q = tid; q < kTM * kXin; q += 256) {
    const int r = q / kXin, k = q % kXin;
    const int64_t row = row0 + r;
    float v = 0.0f;
    if (row < tr.n && k < in) {
      const int64_t src = idx ? idx[row] : row;
      v = tr.xn[src * kXin + k];
    }
    xs[q] = v;
    tr.xb[((int64_t)e * tr.rows + row) * kXin + k] = v;
  }
  __syncthreads();
  flt4 acc[4][NB];
  int cur = 0;
  forward<W, true>(net, e, xs, Hb, red, acc, &tr, row0, wave, lane, tid, &cur);
  __syncthreads();
  const float* P = net.master + (int64_t)e * net.P;
  if (tid < kTM) {
    const int64_t row = row0 + tid;
    float dout = 0.0f, sq = 0.0f;
    if (row < tr.n) {
      const int64_t src = idx ? idx[row] : row;
      const float out = red[tid] + red[kTM + tid] + red[2 * kTM + tid] + red[3 * kTM + tid] + P[off_b(D, in, W, D)];
      const float diff = out - tr.yn[src];
      dout = tr.scale * diff;
      sq = diff * diff;
    }
    dsh[tid] = dout;
    tr.dout[(int64_t)e * tr.rows + row] = dout;
    tr.sq[(int64_t)e * tr.rows + row] = sq;
  }
  __syncthreads();
  const int cw = wave * (W / 4);
  const int lr = lane & 15, rg = (lane >> 4) * 4;
  // delta of the last hidden layer
  {
    const float* wD = P + off_w(D, in, W, D);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float wo = wD[cw + 16 * b + lr];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[a][b][i] = dsh[16 * a + rg + i] * wo * silu_grad(acc[a][b][i]);
    }
  }
  float* dbase = tr.d + (int64_t)e * D * tr.rows * W;
  store_lane<W>(dbase + (int64_t)(D - 1) * tr.rows * W, row0, cw, lane, acc);
  int p = 0;
  for (int l = D - 1; l >= 1; --l) {
    // acc holds delta_l; write it as the A operand of dh_{l-1} = delta_l W_l
    __bf16* Hp = Hb + p * kTM * LDH;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) Hp[(16 * a + rg + i) * LDH + cw + 16 * b + lr] = (__bf16)acc[a][b][i];
    __syncthreads();
    const __bf16* WqT = net.wq + ((int64_t)e * (D - 1) + (l - 1)) * 2 * W * W + (int64_t)W * W;
    mma_layer<W>(Hp, WqT, cw, lane, acc);
    flt4 z[4][NB];
    if (l - 1 >= 1) {
      const float* zg = tr.z + ((int64_t)e * (D - 1) + (l - 2)) * tr.rows * W;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) z[a][b][i] = zg[(row0 + 16 * a + rg + i) * W + cw + 16 * b + lr];
    } else {
      input_layer<W>(P, in, xs, cw, lane, z);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[a][b][i] *= silu_grad(z[a][b][i]);
    store_lane<W>(dbase + (int64_t)(l - 1) * tr.rows * W, row0, cw, lane, acc);
    p ^= 1;
  }
}

// ------------------------------------------------------------------------------ weight gradients
// blockIdx.x < (D-1)*(W/64)^2: 64x64 tile (tj, tk) of the gradient of W_l, l = 1..D-1,
//   g[j][k] = sum_r delta_l[r][j] h_{l-1}[r][k]   (bfloat16 operands, FP32 accumulation);
// otherwise column group vj of 64: gradients of W_0, of every bias and of W_D in FP32
//   (group 0 also b_D and the loss).
template <int W>
__global__ __launch_bounds__(256) void k_emu_wgrad(EmuNet net, EmuTrain tr, EmuAdam A) {
  constexpr int TB = W / 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int e = blockIdx.y;
  const int D = net.D, in = net.in;
  const int64_t rows = tr.rows;
  float* P = net.master + (int64_t)e * net.P;
  float* M = net.m + (int64_t)e * net.P;
  float* V = net.v + (int64_t)e * net.P;
  float* G = A.grad ? A.grad + (int64_t)e * net.P : nullptr;
  const int ntm = (D - 1) * TB * TB;
  if ((int)blockIdx.x < ntm) {
    __shared__ __align__(16) __bf16 As[64 * 40];
    __shared__ __align__(16) __bf16 Bs[64 * 40];
    const int l = 1 + blockIdx.x / (TB * TB);
    const int rem = blockIdx.x % (TB * TB);
    const int j0 = (rem / TB) * 64, k0 = (rem % TB) * 64;
    const float* dl = tr.d + ((int64_t)e * D + l) * rows * W;
    const __bf16* hl = tr.hq + ((int64_t)e * (D - 1) + (l - 1)) * rows * W;
    const int jw = (wave >> 1) * 32, kw = (wave & 1) * 32;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    flt4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
    const int sr = tid >> 3, sq8 = (tid & 7) * 8;
    for (int64_t r0 = 0; r0 < rows; r0 += 32) {
      const float* src = dl + (r0 + sr) * W + j0 + sq8;
      const float4 v0 = *reinterpret_cast<const float4*>(src);
      const float4 v1 = *reinterpret_cast<const float4*>(src + 4);
      const bf16x8 hv = *reinterpret_cast<const bf16x8*>(hl + (r0 + sr) * W + k0 + sq8);
      __syncthreads();
      As[(sq8 + 0) * 40 + sr] = (__bf16)v0.x;
      As[(sq8 + 1) * 40 + sr] = (__bf16)v0.y;
      As[(sq8 + 2) * 40 + sr] = (__bf16)v0.z;
      As[(sq8 + 3) * 40 + sr] = (__bf16)v0.w;
      As[(sq8 + 4) * 40 + sr] = (__bf16)v1.x;
      As[(sq8 + 5) * 40 + sr] = (__bf16)v1.y;
      As[(sq8 + 6) * 40 + sr] = (__bf16)v1.z;
      As[(sq8 + 7) * 40 + sr] = (__bf16)v1.w;
#pragma unroll
      for (int q = 0; q < 8; ++q) Bs[(sq8 + q) * 40 + sr] = hv[q];
      __syncthreads();
      bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&As[(jw + lr) * 40 + lk]);
      bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&As[(jw + 16 + lr) * 40 + lk]);
      bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&Bs[(kw + lr) * 40 + lk]);
      bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&Bs[(kw + 16 + lr) * 40 + lk]);
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    const int64_t ow = off_w(l, in, W, D);
    __bf16* Wq = net.wq + ((int64_t)e * (D - 1) + (l - 1)) * 2 * W * W;
    __bf16* WqT = Wq + (int64_t)W * W;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = j0 + jw + 16 * a + (lane >> 4) * 4 + i;
          const int k = k0 + kw + 16 * b + lr;
          const int64_t f = ow + (int64_t)j * W + k;
          const float g = acc[a][b][i];
          if (G) G[f] = g;
          if (A.do_adam) {
            const float np = adam_update(P + f, M + f, V + f, g, A);
            Wq[(int64_t)j * W + k] = (__bf16)np;
            WqT[(int64_t)k * W + j] = (__bf16)np;
          }
        }
    return;
  }
  // vector group
  constexpr int NV = 2 * kXin + 1;   // W_0 row (<= 8), biases b_0..b_{D-1} (<= 8), W_D entry
  __shared__ float vred[4][64][NV];
  __shared__ float sred[2][256];
  const int vj = blockIdx.x - ntm;
  const int jl = tid & 63, ph = tid >> 6;
  const int j = vj * 64 + jl;
  float s[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) s[q] = 0.0f;
  const float* d0 = tr.d + (int64_t)e * D * rows * W;
  const float* xb = tr.xb + (int64_t)e * rows * kXin;
  const float* dout = tr.dout + (int64_t)e * rows;
  const float* hD = tr.hD + (int64_t)e * rows * W;
  for (int64_t r = ph; r < rows; r += 4) {
    const float dv = d0[r * W + j];
#pragma unroll
    for (int k = 0; k < kXin; ++k) s[k] = fmaf(dv, xb[r * kXin + k], s[k]);
#pragma unroll
    for (int l = 0; l < kXin; ++l)
      if (l < D) s[kXin + l] += d0[((int64_t)l * rows + r) * W + j];
    s[2 * kXin] = fmaf(dout[r], hD[r * W + j], s[2 * kXin]);
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) vred[ph][jl][q] = s[q];
  // b_D and the loss (group 0)
  float sd = 0.0f, ss = 0.0f;
  if (vj == 0) {
    const float* sqv = tr.sq + (int64_t)e * rows;
    for (int64_t r = tid; r < rows; r += 256) {
      sd += dout[r];
      ss += sqv[r];
    }
    sred[0][tid] = sd;
    sred[1][tid] = ss;
  }
  __syncthreads();
  if (ph == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q] = vred[0][jl][q] + vred[1][jl][q] + vred[2][jl][q] + vred[3][jl][q];
    for (int k = 0; k < in; ++k) {
      const int64_t f = off_w(0, in, W, D) + (int64_t)j * in + k;
      if (G) G[f] = s[k];
      if (A.do_adam) adam_update(P + f, M + f, V + f, s[k], A);
    }
    for (int l = 0; l < D; ++l) {
      const int64_t f = off_b(l, in, W, D) + j;
      if (G) G[f] = s[kXin + l];
      if (A.do_adam) adam_update(P + f, M + f, V + f, s[kXin + l], A);
    }
    const int64_t f = off_w(D, in, W, D) + j;
    if (G) G[f] = s[2 * kXin];
    if (A.do_adam) adam_update(P + f, M + f, V + f, s[2 * kXin], A);
  }
  if (vj == 0) {
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        sred[0][tid] += sred[0][tid + w];
        sred[1][tid] += sred[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int64_t f = off_b(D, in, W, D);
      if (G) G[f] = sred[0][0];
      if (A.do_adam) adam_update(P + f, M + f, V + f, sred[0][0], A);
      if (A.loss) A.loss[e] = sred[1][0] * A.inv_n;
    }
  }
}

// ------------------------------------------------------------------------------ inference
// Rows of one tile through every member; mean, spread and routing flag per row.
template <int W>
__global__ __launch_bounds__(256) void k_emu_infer(EmuNet net, EmuInfer q) {
  constexpr int LDH = W + 8;
  __shared__ __align__(16) __bf16 Hb[2 * kTM * LDH];
  __shared__ float xs[kTM * kXin];
  __shared__ float red[4 * kTM];
  __shared__ float outs[16 * kTM];
  __shared__ int inside[kTM];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int in = net.in, D = net.D;
  const int64_t row0 = (int64_t)blockIdx.x * kTM;
  if (tid < kTM) inside[tid] = 1;
  __syncthreads();
  for (int t = tid; t < kTM * kXin; t += 256) {
    const int r = t / kXin, k = t % kXin;
    const int64_t row = row0 + r;
    float v = 0.0f;
    if (row < q.n && k < in) {
      const double x = q.x[row * in + k];
      if (q.raw) {
        v = (float)x;
      } else {
        v = (float)((2.0 * x - q.sc.lo[k] - q.sc.hi[k]) / (q.sc.hi[k] - q.sc.lo[k]));
        if (!(x >= q.sc.lo[k] && x <= q.sc.hi[k])) inside[r] = 0;
      }
    }
    xs[t] = v;
  }
  flt4 acc[4][W / 64];
  for (int e = 0; e < net.E; ++e) {
    __syncthreads();
    int cur = 0;
    forward<W, false>(net, e, xs, Hb, red, acc, nullptr, row0, wave, lane, tid, &cur);
    __syncthreads();
    if (tid < kTM) {
      const float* P = net.master + (int64_t)e * net.P;
      const float out = red[tid] + red[kTM + tid] + red[2 * kTM + tid] + red[3 * kTM + tid] + P[off_b(D, in, W, D)];
      outs[e * kTM + tid] = out;
      const int64_t row = row0 + tid;
      if (q.raw_out && row < q.n) q.raw_out[(int64_t)e * q.n + row] = out;
    }
  }
  __syncthreads();
  if (tid < kTM && row0 + tid < q.n && !q.raw) {
    const int64_t row = row0 + tid;
    double mean = 0.0;
    for (int e = 0; e < net.E; ++e) mean += outs[e * kTM + tid];
    mean /= net.E;
    double var = 0.0;
    for (int e = 0; e < net.E; ++e) {
      const double dv = outs[e * kTM + tid] - mean;
      var += dv * dv;
    }
    const double spread = net.E > 1 ? q.sc.ysig * sqrt(var / (net.E - 1)) : 0.0;
    double u[kXin];
    for (int k = 0; k < in; ++k) u[k] = (2.0 * q.x[row * in + k] - q.sc.lo[k] - q.sc.hi[k]) / (q.sc.hi[k] - q.sc.lo[k]);
    q.y[row] = emu_baseline(q.sc, u, in) + q.sc.ymu + q.sc.ysig * mean;
    if (q.spread) q.spread[row] = spread;
    q.flag[row] = (!inside[tid] || !(spread <= q.spread_max)) ? 1 : 0;
  }
}

// ------------------------------------------------------------------------------ helpers
__global__ void k_emu_adam(EmuNet net, const float* grad, EmuAdam A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)net.E * net.P) return;
  adam_update(net.master + t, net.m + t, net.v + t, grad[t], A);
}

__global__ void k_emu_refresh(EmuNet net) {
  const int W = net.W, D = net.D;
  const int64_t per = (int64_t)W * W;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)net.E * (D - 1) * per) return;
  const int64_t el = t / per;                 // e * (D-1) + (l-1)
  const int e = (int)(el / (D - 1)), l = (int)(el % (D - 1)) + 1;
  const int64_t jk = t % per;
  const int j = (int)(jk / W), k = (int)(jk % W);
  const float p = net.master[(int64_t)e * net.P + off_w(l, net.in, W, D) + jk];
  __bf16* Wq = net.wq + el * 2 * per;
  Wq[jk] = (__bf16)p;
  Wq[per + (int64_t)k * W + j] = (__bf16)p;
}

__global__ void k_emu_prep(const double* x, const double* y, const int* rows, int64_t n, int in,
                           EmuScale sc, float* xn, float* yn) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t r = rows ? rows[t] : t;
  double u[kXin];
  for (int k = 0; k < kXin; ++k) {
    u[k] = k < in ? (2.0 * x[r * in + k] - sc.lo[k] - sc.hi[k]) / (sc.hi[k] - sc.lo[k]) : 0.0;
    xn[t * kXin + k] = (float)u[k];
  }
  yn[t] = (float)((y[r] - emu_baseline(sc, u, in) - sc.ymu) / sc.ysig);
}

__global__ void k_emu_scatter(const double* val, const int* idx, int64_t n, double* y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[idx[t]] = val[t];
}

}  // namespace

int64_t emu_param_count(int in, int W, int D) { return off_b(D, in, W, D) + 1; }
int64_t emu_off_w(int l, int in, int W, int D) { return off_w(l, in, W, D); }

hipError_t launch_emu_train_step(const EmuNet& net, const EmuTrain& tr, const EmuAdam& A, hipStream_t s) {
  const dim3 g1((unsigned)(tr.rows / kTM), (unsigned)net.E);
  const dim3 g2((unsigned)((net.D - 1) * (net.W / 64) * (net.W / 64) + net.W / 64), (unsigned)net.E);
  switch (net.W) {
    case 64:
      hipLaunchKernelGGL(k_emu_train_rows<64>, g1, dim3(256), 0, s, net, tr);
      hipLaunchKernelGGL(k_emu_wgrad<64>, g2, dim3(256), 0, s, net, tr, A);
      break;
    case 128:
      hipLaunchKernelGGL(k_emu_train_rows<128>, g1, dim3(256), 0, s, net, tr);
      hipLaunchKernelGGL(k_emu_wgrad<128>, g2, dim3(256), 0, s, net, tr, A);
      break;
    case 256:
      hipLaunchKernelGGL(k_emu_train_rows<256>, g1, dim3(256), 0, s, net, tr);
      hipLaunchKernelGGL(k_emu_wgrad<256>, g2, dim3(256), 0, s, net, tr, A);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_emu_infer(const EmuNet& net, const EmuInfer& q, hipStream_t s) {
  if (q.n <= 0) return hipSuccess;
  const dim3 g((unsigned)((q.n + kTM - 1) / kTM));
  switch (net.W) {
    case 64: hipLaunchKernelGGL(k_emu_infer<64>, g, dim3(256), 0, s, net, q); break;
    case 128: hipLaunchKernelGGL(k_emu_infer<128>, g, dim3(256), 0, s, net, q); break;
    case 256: hipLaunchKernelGGL(k_emu_infer<256>, g, dim3(256), 0, s, net, q); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_emu_adam(const EmuNet& net, const float* grad, const EmuAdam& A, hipStream_t s) {
  const int64_t n = (int64_t)net.E * net.P;
  hipLaunchKernelGGL(k_emu_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, net, grad, A);
  return hipGetLastError();
}

hipError_t launch_emu_refresh(const EmuNet& net, hipStream_t s) {
  const int64_t n = (int64_t)net.E * (net.D - 1) * net.W * net.W;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_emu_refresh, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, net);
  return hipGetLastError();
}

hipError_t launch_emu_prep(const double* x, const double* y, const int* rows, int64_t n, int in,
                           const EmuScale& sc, float* xn, float* yn, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_emu_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, rows, n, in, sc, xn, yn);
  return hipGetLastError();
}

hipError_t launch_emu_scatter(const double* val, const int* idx, int64_t n, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_emu_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, val, idx, n, y);
  return hipGetLastError();
}

}  // namespace cf
