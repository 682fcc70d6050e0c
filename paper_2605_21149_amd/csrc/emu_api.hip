// C ABI of the likelihood emulator: creation, training loop, ensemble prediction with exact
// fallback, inspection entry points and the state file.
#include "../../include/cf.h"
#include "cf_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

using namespace cf;

struct cf_emu {
  EmuNet net{};
  int dev = 0;
  uint64_t seed = 0;
  int64_t step = 0;             // Adam steps taken so far
  int64_t calls = 0;            // training calls so far (decorrelates their shuffles)
  int scaled = 0;               // hull and target scaling fixed
  EmuScale sc{};
  double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  hipStream_t s = nullptr;
  float* grad = nullptr;        // [E][P]
  float* loss = nullptr;        // [E]
  void* buf[6] = {};            // growable prediction buffers
  size_t cap[6] = {};
  std::mutex mu;
};

namespace {

#define EMU_DEV(expr)                                                                         \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess)                                                                     \
      return set_error(_e == hipErrorOutOfMemory ? CF_ENOMEM : CF_EDEVICE, "%s: %s (%s:%d)", #expr, \
                       hipGetErrorString(_e), __FILE__, __LINE__);                            \
  } while (0)

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014)
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  uint64_t below(uint64_t n) { return n ? next() % n : 0; }   // bias < n / 2^64: immaterial here
};

void shuffle(int* a, int64_t n, SplitMix& r) {
  for (int64_t i = n - 1; i > 0; --i) std::swap(a[i], a[r.below((uint64_t)i + 1)]);
}

// Device buffers released (after the stream drains) when the holder goes out of scope.
struct Scratch {
  hipStream_t s = nullptr;
  std::vector<void*> dev, host;
  ~Scratch() {
    if (s) (void)hipStreamSynchronize(s);
    for (void* p : dev) (void)hipFree(p);
    for (void* p : host) (void)hipHostFree(p);
  }
  template <typename T>
  int alloc(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return set_error(CF_ENOMEM, "emulator scratch of %zu bytes: %s", count * sizeof(T), hipGetErrorString(e));
    dev.push_back(p);
    *out = static_cast<T*>(p);
    return CF_OK;
  }
  template <typename T>
  int pinned(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) return set_error(CF_ENOMEM, "pinned buffer of %zu bytes: %s", count * sizeof(T), hipGetErrorString(e));
    host.push_back(p);
    *out = static_cast<T*>(p);
    return CF_OK;
  }
};

int grow(cf_emu* m, int slot, size_t bytes, void** out) {
  if (bytes > m->cap[slot]) {
    if (m->buf[slot]) EMU_DEV(hipFree(m->buf[slot]));
    m->buf[slot] = nullptr;
    m->cap[slot] = 0;
    const size_t want = std::max<size_t>(bytes + (bytes >> 3), 256);
    hipError_t e = hipMalloc(&m->buf[slot], want);
    if (e != hipSuccess) {
      m->buf[slot] = nullptr;
      return set_error(CF_ENOMEM, "emulator buffer of %zu bytes: %s", want, hipGetErrorString(e));
    }
    m->cap[slot] = want;
  }
  *out = m->buf[slot];
  return CF_OK;
}

int check_device(const cf_emu* m) {
  int id = -1;
  EMU_DEV(hipGetDevice(&id));
  if (id != m->dev) return set_error(CF_EINVAL, "emulator lives on device %d, current device is %d", m->dev, id);
  return CF_OK;
}

hipStream_t stream_of(cf_emu* m, const cf_exec* ex) { return (ex && ex->stream) ? (hipStream_t)ex->stream : m->s; }

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

EmuAdam adam_consts(const cf_emu* m, double lr) {
  const double t = (double)(m->step + 1);
  EmuAdam A{};
  A.lr = (float)lr;
  A.b1 = (float)m->b1;
  A.b2 = (float)m->b2;
  A.eps = (float)m->eps;
  A.c1 = (float)(1.0 / (1.0 - std::pow(m->b1, t)));
  A.c2 = (float)(1.0 / (1.0 - std::pow(m->b2, t)));
  A.do_adam = 1;
  return A;
}

// Training-pass scratch for minibatches of up to `rows` (multiple of 64) rows.
int train_scratch(Scratch& S, const EmuNet& net, int64_t rows, EmuTrain& tr) {
  const size_t E = net.E, D = net.D, W = net.W;
  tr.rows = rows;
  if (int st = S.alloc(&tr.hq, E * (D - 1) * rows * W)) return st;
  if (int st = S.alloc(&tr.z, E * (D - 1) * rows * W)) return st;
  if (int st = S.alloc(&tr.hD, E * rows * W)) return st;
  if (int st = S.alloc(&tr.d, E * D * rows * W)) return st;
  if (int st = S.alloc(&tr.dout, E * rows)) return st;
  if (int st = S.alloc(&tr.sq, E * rows)) return st;
  if (int st = S.alloc(&tr.xb, E * rows * 8)) return st;
  return CF_OK;
}

// Algorithmic flops of one row through one member: forward, backward data, weight gradients.
double train_flops_per_row(const EmuNet& n) {
  const double in = n.in, W = n.W, H = (double)(n.D - 1) * W * W;
  const double fwd = 2.0 * (in * W + H + W);
  return fwd + 2.0 * H + fwd;
}

// Least-squares polynomial baseline of degree sc.qdeg through (u(x_r), y_r) over the training
// rows: normal equations (features 1, u_k, u_i u_j on [-1, 1]) solved by Cholesky in FP64.
int fit_baseline(const double* x, const double* y, const int* rows, int64_t nt, int in, EmuScale& sc) {
  for (double& c : sc.qc) c = 0.0;
  const int nf = emu_nfeat(in, sc.qdeg);
  if (nf == 0) return CF_OK;
  if (nt < 4 * nf) return set_error(CF_EINVAL, "%lld training rows are too few for a degree-%d baseline", (long long)nt, sc.qdeg);
  std::vector<double> A((size_t)nf * nf, 0.0), b((size_t)nf, 0.0), f((size_t)nf), u(8);
  for (int64_t i = 0; i < nt; ++i) {
    const int64_t r = rows[i];
    for (int k = 0; k < in; ++k) u[k] = (2.0 * x[r * in + k] - sc.lo[k] - sc.hi[k]) / (sc.hi[k] - sc.lo[k]);
    int o = 0;
    f[o++] = 1.0;
    for (int k = 0; k < in; ++k) f[o++] = u[k];
    if (sc.qdeg >= 2)
      for (int p = 0; p < in; ++p)
        for (int q = p; q < in; ++q) f[o++] = u[p] * u[q];
    for (int p = 0; p < nf; ++p) {
      b[p] += f[p] * y[r];
      for (int q = 0; q <= p; ++q) A[(size_t)p * nf + q] += f[p] * f[q];
    }
  }
  for (int p = 0; p < nf; ++p) {                 // Cholesky A = L L^T (lower, in place)
    for (int q = 0; q <= p; ++q) {
      double s = A[(size_t)p * nf + q];
      for (int k = 0; k < q; ++k) s -= A[(size_t)p * nf + k] * A[(size_t)q * nf + k];
      if (p == q) {
        if (!(s > 0.0)) return set_error(CF_EINVAL, "training inputs do not determine the baseline");
        A[(size_t)p * nf + p] = std::sqrt(s);
      } else {
        A[(size_t)p * nf + q] = s / A[(size_t)q * nf + q];
      }
    }
  }
  for (int p = 0; p < nf; ++p) {                 // L z = b, then L^T c = z
    double s = b[p];
    for (int k = 0; k < p; ++k) s -= A[(size_t)p * nf + k] * b[k];
    b[p] = s / A[(size_t)p * nf + p];
  }
  for (int p = nf - 1; p >= 0; --p) {
    double s = b[p];
    for (int k = p + 1; k < nf; ++k) s -= A[(size_t)k * nf + p] * b[k];
    b[p] = s / A[(size_t)p * nf + p];
  }
  for (int p = 0; p < nf; ++p) sc.qc[p] = b[p];
  return CF_OK;
}

}  // namespace

extern "C" {

int cf_emu_create(int32_t in_dim, int32_t width, int32_t depth, int32_t ensemble, uint64_t seed,
                  cf_emu** out) {
  if (!out) return set_error(CF_EINVAL, "out is NULL");
  *out = nullptr;
  if (in_dim < 1 || in_dim > 8) return set_error(CF_EINVAL, "in_dim %d outside 1..8", in_dim);
  if (width != 64 && width != 128 && width != 256) return set_error(CF_EINVAL, "width %d is not 64, 128 or 256", width);
  if (depth < 1 || depth > 8) return set_error(CF_EINVAL, "depth %d outside 1..8", depth);
  if (ensemble < 1 || ensemble > 16) return set_error(CF_EINVAL, "ensemble %d outside 1..16", ensemble);
  cf_emu* m = new cf_emu();
  EmuNet& n = m->net;
  n.in = in_dim; n.W = width; n.D = depth; n.E = ensemble;
  n.P = emu_param_count(in_dim, width, depth);
  m->seed = seed;
  auto bail = [&](int st) { cf_emu_destroy(m); return st; };
  hipError_t e = hipGetDevice(&m->dev);
  if (e != hipSuccess) return bail(set_error(CF_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
  const size_t np = (size_t)n.E * n.P;
  const size_t nq = (size_t)n.E * (n.D - 1) * 2 * n.W * n.W;
  if (hipMalloc(&n.master, np * 4) != hipSuccess || hipMalloc(&n.m, np * 4) != hipSuccess ||
      hipMalloc(&n.v, np * 4) != hipSuccess || hipMalloc(&n.wq, std::max<size_t>(nq, 1) * 2) != hipSuccess ||
      hipMalloc(&m->grad, np * 4) != hipSuccess || hipMalloc(&m->loss, (size_t)n.E * 4) != hipSuccess)
    return bail(set_error(CF_ENOMEM, "emulator parameters (%zu floats)", np));
  if (hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking) != hipSuccess)
    return bail(set_error(CF_EDEVICE, "stream creation failed"));
  std::vector<float> h(np);
  for (int me = 0; me < n.E; ++me) {
    SplitMix r{seed + (uint64_t)me};
    float* p = h.data() + (size_t)me * n.P;
    size_t o = 0;
    for (int l = 0; l <= n.D; ++l) {
      const int fin = l == 0 ? n.in : n.W;
      const int fout = l == n.D ? 1 : n.W;
      const double a = 1.0 / std::sqrt((double)fin);
      for (int64_t q = 0; q < (int64_t)fin * fout + fout; ++q) p[o++] = (float)(a * (2.0 * r.uniform() - 1.0));
    }
  }
  if (hipMemcpy(n.master, h.data(), np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n.m, 0, np * 4) != hipSuccess || hipMemset(n.v, 0, np * 4) != hipSuccess)
    return bail(set_error(CF_EDEVICE, "emulator initialisation copy failed"));
  if (launch_emu_refresh(n, m->s) != hipSuccess || hipStreamSynchronize(m->s) != hipSuccess)
    return bail(set_error(CF_EDEVICE, "emulator weight refresh failed"));
  *out = m;
  return CF_OK;
}

void cf_emu_destroy(cf_emu* m) {
  if (!m) return;
  if (m->s) (void)hipStreamSynchronize(m->s);
  for (void* p : {(void*)m->net.master, (void*)m->net.m, (void*)m->net.v, (void*)m->net.wq,
                  (void*)m->grad, (void*)m->loss})
    if (p) (void)hipFree(p);
  for (void* p : m->buf)
    if (p) (void)hipFree(p);
  if (m->s) (void)hipStreamDestroy(m->s);
  delete m;
}

int64_t cf_emu_param_count(const cf_emu* m) {
  if (!m) { set_error(CF_EINVAL, "emulator is NULL"); return -1; }
  return m->net.P;
}

int cf_emu_shape(const cf_emu* m, int32_t* in_dim, int32_t* width, int32_t* depth, int32_t* ensemble) {
  if (!m) return set_error(CF_EINVAL, "emulator is NULL");
  if (in_dim) *in_dim = m->net.in;
  if (width) *width = m->net.W;
  if (depth) *depth = m->net.D;
  if (ensemble) *ensemble = m->net.E;
  return CF_OK;
}

int cf_emu_train(cf_emu* m, const double* x, const double* y, int64_t N, int32_t mem,
                 const cf_emu_opts* opts, const cf_exec* ex, cf_report* rep) {
  if (rep) { std::memset(rep, 0, sizeof *rep); rep->fail_index = -1; }
  if (!m) return set_error(CF_EINVAL, "emulator is NULL");
  if (!x || !y) return set_error(CF_EINVAL, "x or y is NULL");
  if (N < 2 || N > (int64_t)1 << 30) return set_error(CF_EINVAL, "N = %lld outside 2..2^30", (long long)N);
  if (mem != CF_MEM_HOST && mem != CF_MEM_DEVICE) return set_error(CF_EINVAL, "unknown mem %d", mem);
  cf_emu_opts o{200, 1024, 1e-3, 0.9, 0.999, 1e-8, 0.1, 2};
  if (opts) o = *opts;
  if (o.epochs < 1) return set_error(CF_EINVAL, "epochs %d < 1", o.epochs);
  if (o.batch < 1 || o.batch > 65536) return set_error(CF_EINVAL, "batch %d outside 1..65536", o.batch);
  if (!(o.lr > 0.0) || !std::isfinite(o.lr)) return set_error(CF_EINVAL, "lr must be positive");
  if (!(o.beta1 >= 0.0 && o.beta1 < 1.0) || !(o.beta2 >= 0.0 && o.beta2 < 1.0))
    return set_error(CF_EINVAL, "Adam betas must lie in [0, 1)");
  if (!(o.eps > 0.0)) return set_error(CF_EINVAL, "eps must be positive");
  if (!(o.val_frac >= 0.0 && o.val_frac < 1.0)) return set_error(CF_EINVAL, "val_frac outside [0, 1)");
  if (o.baseline < 0 || o.baseline > 2) return set_error(CF_EINVAL, "baseline degree %d outside 0..2", o.baseline);
  std::lock_guard<std::mutex> lk(m->mu);
  if (int st = check_device(m)) return st;
  const EmuNet& n = m->net;
  const int in = n.in, E = n.E;
  hipStream_t s = stream_of(m, ex);
  // host view of the data (validation and statistics)
  std::vector<double> hx, hy;
  const double *xh = x, *yh = y;
  if (mem == CF_MEM_DEVICE) {
    hx.resize((size_t)N * in);
    hy.resize((size_t)N);
    EMU_DEV(hipMemcpyAsync(hx.data(), x, hx.size() * 8, hipMemcpyDeviceToHost, s));
    EMU_DEV(hipMemcpyAsync(hy.data(), y, hy.size() * 8, hipMemcpyDeviceToHost, s));
    EMU_DEV(hipStreamSynchronize(s));
    xh = hx.data();
    yh = hy.data();
  }
  if (!finite_all(xh, N * in) || !finite_all(yh, N)) return set_error(CF_EINVAL, "non-finite training value");
  // seeded split
  std::vector<int> perm((size_t)N);
  for (int64_t i = 0; i < N; ++i) perm[i] = (int)i;
  SplitMix rs{m->seed ^ 0xA5A5A5A5DEADBEEFull};
  shuffle(perm.data(), N, rs);
  const int64_t nval = (int64_t)std::floor(o.val_frac * (double)N + 0.5);
  const int64_t nt = N - nval;
  if (nt < 1) return set_error(CF_EINVAL, "no training rows left after the held-out split");
  if (!m->scaled) {
    EmuScale sc{};
    for (int k = 0; k < 8; ++k) { sc.lo[k] = -1.0; sc.hi[k] = 1.0; }
    for (int k = 0; k < in; ++k) {
      double lo = INFINITY, hi = -INFINITY;
      for (int64_t i = nval; i < N; ++i) {
        const double v = xh[(size_t)perm[i] * in + k];
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      if (!(hi > lo)) return set_error(CF_EINVAL, "training inputs are constant in parameter %d", k);
      sc.lo[k] = lo;
      sc.hi[k] = hi;
    }
    sc.qdeg = o.baseline;
    if (int st = fit_baseline(xh, yh, perm.data() + nval, nt, in, sc)) return st;
    double mu = 0.0;
    std::vector<double> res((size_t)nt);
    std::vector<double> u(8);
    for (int64_t i = 0; i < nt; ++i) {
      const int64_t r = perm[nval + i];
      for (int k = 0; k < in; ++k) u[k] = (2.0 * xh[r * in + k] - sc.lo[k] - sc.hi[k]) / (sc.hi[k] - sc.lo[k]);
      res[i] = yh[r] - emu_baseline(sc, u.data(), in);
      mu += res[i];
    }
    mu /= (double)nt;
    double var = 0.0;
    for (double r : res) var += (r - mu) * (r - mu);
    const double sig = std::sqrt(var / (double)nt);
    if (!(sig > 0.0)) return set_error(CF_EINVAL, "training targets are exactly fitted by the baseline");
    sc.ymu = mu;
    sc.ysig = sig;
    m->sc = sc;
    m->scaled = 1;
  }
  m->b1 = o.beta1;
  m->b2 = o.beta2;
  m->eps = o.eps;
  Scratch S;
  S.s = s;
  const double* xd = x;
  const double* yd = y;
  if (mem == CF_MEM_HOST) {
    double *tx, *ty;
    if (int st = S.alloc(&tx, (size_t)N * in)) return st;
    if (int st = S.alloc(&ty, (size_t)N)) return st;
    EMU_DEV(hipMemcpyAsync(tx, x, (size_t)N * in * 8, hipMemcpyHostToDevice, s));
    EMU_DEV(hipMemcpyAsync(ty, y, (size_t)N * 8, hipMemcpyHostToDevice, s));
    xd = tx;
    yd = ty;
  }
  int* trows;
  float *xn, *yn;
  if (int st = S.alloc(&trows, (size_t)nt)) return st;
  if (int st = S.alloc(&xn, (size_t)nt * 8)) return st;
  if (int st = S.alloc(&yn, (size_t)nt)) return st;
  EMU_DEV(hipMemcpyAsync(trows, perm.data() + nval, (size_t)nt * 4, hipMemcpyHostToDevice, s));
  EMU_DEV(launch_emu_prep(xd, yd, trows, nt, in, m->sc, xn, yn, s));
  EMU_DEV(hipStreamSynchronize(s));   // perm is rewritten below
  const int64_t B = std::min<int64_t>(o.batch, nt);
  const int64_t spe = nt / B;
  const int64_t T = (int64_t)o.epochs * spe;
  EmuTrain tr{};
  if (int st = train_scratch(S, n, (B + 63) / 64 * 64, tr)) return st;
  tr.n = B;
  tr.xn = xn;
  tr.yn = yn;
  tr.idx_stride = nt;
  tr.scale = (float)(2.0 / (double)B);
  int* idx_dev[2];
  int* idx_host[2];
  float* hist;
  for (int b = 0; b < 2; ++b) {
    if (int st = S.alloc(&idx_dev[b], (size_t)E * nt)) return st;
    if (int st = S.pinned(&idx_host[b], (size_t)E * nt)) return st;
  }
  if (int st = S.alloc(&hist, (size_t)T * E)) return st;
  hipEvent_t ev[2] = {nullptr, nullptr}, t0 = nullptr, t1 = nullptr;
  struct EvGuard {
    hipEvent_t* e[4];
    ~EvGuard() { for (auto p : e) if (*p) (void)hipEventDestroy(*p); }
  } eg{{&ev[0], &ev[1], &t0, &t1}};
  EMU_DEV(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  EMU_DEV(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  EMU_DEV(hipEventCreate(&t0));
  EMU_DEV(hipEventCreate(&t1));
  EMU_DEV(hipEventRecord(t0, s));
  const double pi = 3.14159265358979323846;
  int64_t u = 0;
  for (int ep = 0; ep < o.epochs; ++ep) {
    const int b = ep & 1;
    if (ep >= 2) EMU_DEV(hipEventSynchronize(ev[b]));
    for (int me = 0; me < E; ++me) {
      int* p = idx_host[b] + (size_t)me * nt;
      for (int64_t i = 0; i < nt; ++i) p[i] = (int)i;
      SplitMix r{m->seed * 0x9E3779B97F4A7C15ull + ((uint64_t)m->calls << 40) + ((uint64_t)ep << 8) + (uint64_t)me};
      shuffle(p, nt, r);
    }
    EMU_DEV(hipMemcpyAsync(idx_dev[b], idx_host[b], (size_t)E * nt * 4, hipMemcpyHostToDevice, s));
    EMU_DEV(hipEventRecord(ev[b], s));
    for (int64_t st = 0; st < spe; ++st, ++u) {
      tr.idx = idx_dev[b] + st * B;
      EmuAdam A = adam_consts(m, o.lr * 0.5 * (1.0 + std::cos(pi * (double)u / (double)T)));
      A.loss = hist + u * E;
      A.inv_n = (float)(1.0 / (double)B);
      EMU_DEV(launch_emu_train_step(n, tr, A, s));
      ++m->step;
    }
  }
  EMU_DEV(hipEventRecord(t1, s));
  EMU_DEV(hipEventSynchronize(t1));
  ++m->calls;
  float ms = 0.f;
  EMU_DEV(hipEventElapsedTime(&ms, t0, t1));
  std::vector<float> hh((size_t)spe * E);
  EMU_DEV(hipMemcpy(hh.data(), hist + (T - spe) * E, hh.size() * 4, hipMemcpyDeviceToHost));
  double last = 0.0;
  for (float v : hh) last += v;
  last /= (double)hh.size();
  double vrms = 0.0, vmax = 0.0, vspread = 0.0;
  if (nval > 0) {
    std::vector<double> xv((size_t)nval * in);
    for (int64_t i = 0; i < nval; ++i)
      for (int k = 0; k < in; ++k) xv[i * in + k] = xh[(size_t)perm[i] * in + k];
    double *xvd, *yv, *sv;
    uint8_t* fv;
    if (int st = S.alloc(&xvd, xv.size())) return st;
    if (int st = S.alloc(&yv, (size_t)nval)) return st;
    if (int st = S.alloc(&sv, (size_t)nval)) return st;
    if (int st = S.alloc(&fv, (size_t)nval)) return st;
    EMU_DEV(hipMemcpyAsync(xvd, xv.data(), xv.size() * 8, hipMemcpyHostToDevice, s));
    EmuInfer q{};
    q.x = xvd; q.n = nval; q.raw = 0;
    q.sc = m->sc;
    q.spread_max = INFINITY;
    q.y = yv; q.spread = sv; q.flag = fv;
    EMU_DEV(launch_emu_infer(n, q, s));
    std::vector<double> hyv((size_t)nval), hsv((size_t)nval);
    EMU_DEV(hipMemcpyAsync(hyv.data(), yv, (size_t)nval * 8, hipMemcpyDeviceToHost, s));
    EMU_DEV(hipMemcpyAsync(hsv.data(), sv, (size_t)nval * 8, hipMemcpyDeviceToHost, s));
    EMU_DEV(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nval; ++i) {
      const double err = hyv[i] - yh[perm[i]];
      vrms += err * err;
      vmax = std::max(vmax, std::fabs(err));
      vspread += hsv[i];
    }
    vrms = std::sqrt(vrms / (double)nval);
    vspread /= (double)nval;
  }
  if (rep) {
    rep->ms_total = ms;
    rep->flops = (double)T * E * B * train_flops_per_row(n);
    rep->est_err[0] = last;
    rep->est_err[1] = vrms;
    rep->est_err[2] = vmax;
    rep->est_err[3] = vspread;
    rep->ir_iters = (int32_t)std::min<int64_t>(T, INT32_MAX);
    rep->n = N;
  }
  return CF_OK;
}

}  // extern "C"

namespace {
// Prediction with the exact fallback through either the pixel likelihood (exact_prob, exact_map)
// or a harmonic-basis handle (smw, one map); both NULL: routing flags only.
int emu_predict(cf_emu* m, const double* x, int64_t N, int32_t mem, double spread_max,
                const cf_problem* exact_prob, const cf_smw* smw, const cf_linear_spectra* model,
                const double* exact_map, double* y_out, double* spread_out,
                uint8_t* used_fallback, const cf_exec* ex, cf_report* rep) {
  const auto w0 = std::chrono::steady_clock::now();
  if (rep) { std::memset(rep, 0, sizeof *rep); rep->fail_index = -1; }
  if (!m) return set_error(CF_EINVAL, "emulator is NULL");
  if (!x || !y_out) return set_error(CF_EINVAL, "x or y_out is NULL");
  if (N < 1 || N > (int64_t)1 << 30) return set_error(CF_EINVAL, "N = %lld outside 1..2^30", (long long)N);
  if (mem != CF_MEM_HOST && mem != CF_MEM_DEVICE) return set_error(CF_EINVAL, "unknown mem %d", mem);
  if (!(spread_max >= 0.0)) return set_error(CF_EINVAL, "spread_max must be >= 0");
  if (exact_prob || smw) {
    if (!model || (exact_prob && !exact_map)) return set_error(CF_EINVAL, "exact fallback needs the spectra model and the map");
    if (model->nparam != m->net.in) return set_error(CF_EINVAL, "model has %d parameters, emulator %d", model->nparam, m->net.in);
    if (!model->base || !model->basis || model->lstride < 1) return set_error(CF_EINVAL, "incomplete spectra model");
  }
  int smw_mem = CF_MEM_DEVICE, smw_maps = 0;
  if (smw) {
    if (!cf::smw_describe(smw, &smw_mem, &smw_maps)) return set_error(CF_EINVAL, "invalid harmonic-basis handle");
    if (smw_maps != 1) return set_error(CF_EINVAL, "the harmonic-basis handle holds %d maps; the fallback needs one", smw_maps);
  }
  std::lock_guard<std::mutex> lk(m->mu);
  if (!m->scaled) return set_error(CF_EINVAL, "emulator has not been trained");
  if (int st = check_device(m)) return st;
  const EmuNet& n = m->net;
  const int in = n.in;
  hipStream_t s = stream_of(m, ex);
  void *bx, *by, *bs, *bf;
  if (int st = grow(m, 0, (size_t)N * in * 8, &bx)) return st;
  if (int st = grow(m, 1, (size_t)N * 8, &by)) return st;
  if (int st = grow(m, 2, (size_t)N * 8, &bs)) return st;
  if (int st = grow(m, 3, (size_t)N, &bf)) return st;
  const double* xd = x;
  if (mem == CF_MEM_HOST) {
    EMU_DEV(hipMemcpyAsync(bx, x, (size_t)N * in * 8, hipMemcpyHostToDevice, s));
    xd = static_cast<const double*>(bx);
  }
  double* yd = mem == CF_MEM_DEVICE ? y_out : static_cast<double*>(by);
  double* sd = (mem == CF_MEM_DEVICE && spread_out) ? spread_out : static_cast<double*>(bs);
  uint8_t* fd = (mem == CF_MEM_DEVICE && used_fallback) ? used_fallback : static_cast<uint8_t*>(bf);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct EvGuard {
    hipEvent_t* e[2];
    ~EvGuard() { for (auto p : e) if (*p) (void)hipEventDestroy(*p); }
  } eg{{&e0, &e1}};
  EMU_DEV(hipEventCreate(&e0));
  EMU_DEV(hipEventCreate(&e1));
  EmuInfer q{};
  q.x = xd; q.n = N; q.raw = 0;
  q.sc = m->sc;
  q.spread_max = spread_max;
  q.y = yd; q.spread = sd; q.flag = fd;
  EMU_DEV(hipEventRecord(e0, s));
  EMU_DEV(launch_emu_infer(n, q, s));
  EMU_DEV(hipEventRecord(e1, s));
  std::vector<uint8_t> hf((size_t)N);
  EMU_DEV(hipMemcpyAsync(hf.data(), fd, (size_t)N, hipMemcpyDeviceToHost, s));
  EMU_DEV(hipStreamSynchronize(s));
  float ms_inf = 0.f;
  EMU_DEV(hipEventElapsedTime(&ms_inf, e0, e1));
  std::vector<int> fb;
  for (int64_t i = 0; i < N; ++i)
    if (hf[i]) fb.push_back((int)i);
  double ms_exact = 0.0;
  if ((exact_prob || smw) && !fb.empty()) {
    const auto x0 = std::chrono::steady_clock::now();
    const int64_t nf = (int64_t)fb.size();
    const int L = model->lstride;
    std::vector<double> hx;
    const double* xh = x;
    if (mem == CF_MEM_DEVICE) {
      hx.resize((size_t)N * in);
      EMU_DEV(hipMemcpy(hx.data(), x, hx.size() * 8, hipMemcpyDeviceToHost));
      xh = hx.data();
    }
    std::vector<double> cl((size_t)nf * 6 * L);
    for (int64_t i = 0; i < nf; ++i) {
      double* c = cl.data() + (size_t)i * 6 * L;
      std::memcpy(c, model->base, sizeof(double) * 6 * L);
      for (int k = 0; k < in; ++k) {
        const double t = xh[(size_t)fb[i] * in + k];
        const double* bk = model->basis + (size_t)k * 6 * L;
        for (int j = 0; j < 6 * L; ++j) c[j] += t * bk[j];
      }
    }
    Scratch S;
    S.s = s;
    double* vals;
    int* idx;
    if (int st = S.alloc(&vals, (size_t)nf)) return st;
    if (int st = S.alloc(&idx, (size_t)nf)) return st;
    EMU_DEV(hipMemcpyAsync(idx, fb.data(), (size_t)nf * 4, hipMemcpyHostToDevice, s));
    cf_exec ex2{};
    ex2.stream = s;
    ex2.refine_max = -1;
    const double* maps[1] = {exact_map};
    if (smw) {
      // the handle's memory space holds its spectra and outputs
      if (smw_mem == CF_MEM_DEVICE) {
        double* cld;
        if (int st = S.alloc(&cld, cl.size())) return st;
        EMU_DEV(hipMemcpyAsync(cld, cl.data(), cl.size() * 8, hipMemcpyHostToDevice, s));
        if (int st = cf_smw_loglike(const_cast<cf_smw*>(smw), (int32_t)nf, cld, L, vals, nullptr, nullptr, &ex2, nullptr))
          return st;
      } else {
        std::vector<double> hv((size_t)nf);
        if (int st = cf_smw_loglike(const_cast<cf_smw*>(smw), (int32_t)nf, cl.data(), L, hv.data(), nullptr, nullptr,
                                    &ex2, nullptr))
          return st;
        EMU_DEV(hipMemcpyAsync(vals, hv.data(), (size_t)nf * 8, hipMemcpyHostToDevice, s));
        EMU_DEV(hipStreamSynchronize(s));
      }
    } else if (exact_prob->mem == CF_MEM_DEVICE) {
      double* cld;
      if (int st = S.alloc(&cld, cl.size())) return st;
      EMU_DEV(hipMemcpyAsync(cld, cl.data(), cl.size() * 8, hipMemcpyHostToDevice, s));
      if (int st = cf_loglike_batch(exact_prob, 1, (int32_t)nf, cld, L, maps, 1, CF_FP64, vals, nullptr, nullptr, &ex2, nullptr))
        return st;
    } else {
      std::vector<double> hv((size_t)nf);
      if (int st = cf_loglike_batch(exact_prob, 1, (int32_t)nf, cl.data(), L, maps, 1, CF_FP64, hv.data(), nullptr, nullptr, &ex2, nullptr))
        return st;
      EMU_DEV(hipMemcpyAsync(vals, hv.data(), (size_t)nf * 8, hipMemcpyHostToDevice, s));
      EMU_DEV(hipStreamSynchronize(s));
    }
    EMU_DEV(launch_emu_scatter(vals, idx, nf, yd, s));
    EMU_DEV(hipStreamSynchronize(s));
    ms_exact = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - x0).count();
  }
  if (mem == CF_MEM_HOST) {
    EMU_DEV(hipMemcpyAsync(y_out, yd, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    if (spread_out) EMU_DEV(hipMemcpyAsync(spread_out, sd, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    if (used_fallback) std::memcpy(used_fallback, hf.data(), (size_t)N);
  }
  EMU_DEV(hipStreamSynchronize(s));
  if (rep) {
    rep->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
    rep->n_fallback = (int64_t)fb.size();
    rep->est_err[0] = ms_inf;
    rep->est_err[1] = ms_exact;
    rep->flops = (double)N * n.E * (2.0 * ((double)n.in * n.W + (double)(n.D - 1) * n.W * n.W + n.W));
    rep->n = N;
  }
  return CF_OK;
}
}  // namespace

extern "C" {

int cf_emu_predict(cf_emu* m, const double* x, int64_t N, int32_t mem, double spread_max,
                   const cf_problem* exact_prob, const cf_linear_spectra* model,
                   const double* exact_map, double* y_out, double* spread_out,
                   uint8_t* used_fallback, const cf_exec* ex, cf_report* rep) {
  return emu_predict(m, x, N, mem, spread_max, exact_prob, nullptr, model, exact_map, y_out, spread_out,
                     used_fallback, ex, rep);
}

int cf_emu_predict_smw(cf_emu* m, const double* x, int64_t N, int32_t mem, double spread_max,
                       const cf_smw* exact_smw, const cf_linear_spectra* model, double* y_out,
                       double* spread_out, uint8_t* used_fallback, const cf_exec* ex, cf_report* rep) {
  if (!exact_smw) return set_error(CF_EINVAL, "harmonic-basis handle is NULL");
  return emu_predict(m, x, N, mem, spread_max, nullptr, exact_smw, model, nullptr, y_out, spread_out,
                     used_fallback, ex, rep);
}

int cf_emu_get_params(const cf_emu* m, int32_t member, float* out) {
  if (!m || !out) return set_error(CF_EINVAL, "NULL argument");
  if (member < 0 || member >= m->net.E) return set_error(CF_EINVAL, "member %d outside 0..%d", member, m->net.E - 1);
  if (int st = check_device(m)) return st;
  EMU_DEV(hipStreamSynchronize(m->s));
  EMU_DEV(hipMemcpy(out, m->net.master + (size_t)member * m->net.P, (size_t)m->net.P * 4, hipMemcpyDeviceToHost));
  return CF_OK;
}

int cf_emu_set_params(cf_emu* m, int32_t member, const float* in) {
  if (!m || !in) return set_error(CF_EINVAL, "NULL argument");
  if (member < 0 || member >= m->net.E) return set_error(CF_EINVAL, "member %d outside 0..%d", member, m->net.E - 1);
  for (int64_t i = 0; i < m->net.P; ++i)
    if (!std::isfinite(in[i])) return set_error(CF_EINVAL, "non-finite parameter %lld", (long long)i);
  std::lock_guard<std::mutex> lk(m->mu);
  if (int st = check_device(m)) return st;
  EMU_DEV(hipStreamSynchronize(m->s));
  EMU_DEV(hipMemcpy(m->net.master + (size_t)member * m->net.P, in, (size_t)m->net.P * 4, hipMemcpyHostToDevice));
  EMU_DEV(launch_emu_refresh(m->net, m->s));
  EMU_DEV(hipStreamSynchronize(m->s));
  return CF_OK;
}

int cf_emu_forward(cf_emu* m, const double* x, int64_t N, float* out) {
  if (!m || !x || !out) return set_error(CF_EINVAL, "NULL argument");
  if (N < 1 || N > (int64_t)1 << 26) return set_error(CF_EINVAL, "N = %lld outside 1..2^26", (long long)N);
  std::lock_guard<std::mutex> lk(m->mu);
  if (int st = check_device(m)) return st;
  const EmuNet& n = m->net;
  Scratch S;
  S.s = m->s;
  double* xd;
  float* od;
  if (int st = S.alloc(&xd, (size_t)N * n.in)) return st;
  if (int st = S.alloc(&od, (size_t)N * n.E)) return st;
  EMU_DEV(hipMemcpyAsync(xd, x, (size_t)N * n.in * 8, hipMemcpyHostToDevice, m->s));
  EmuInfer q{};
  q.x = xd; q.n = N; q.raw = 1; q.raw_out = od;
  q.sc.ysig = 1.0;
  q.spread_max = INFINITY;
  EMU_DEV(launch_emu_infer(n, q, m->s));
  EMU_DEV(hipMemcpyAsync(out, od, (size_t)N * n.E * 4, hipMemcpyDeviceToHost, m->s));
  EMU_DEV(hipStreamSynchronize(m->s));
  return CF_OK;
}

int cf_emu_gradient(cf_emu* m, const double* x, const double* y, int64_t N, float* grad, double* loss) {
  if (!m || !x || !y || !grad) return set_error(CF_EINVAL, "NULL argument");
  if (N < 1 || N > 65536) return set_error(CF_EINVAL, "N = %lld outside 1..65536", (long long)N);
  std::lock_guard<std::mutex> lk(m->mu);
  if (int st = check_device(m)) return st;
  const EmuNet& n = m->net;
  hipStream_t s = m->s;
  Scratch S;
  S.s = s;
  double *xd, *yd;
  float *xn, *yn;
  if (int st = S.alloc(&xd, (size_t)N * n.in)) return st;
  if (int st = S.alloc(&yd, (size_t)N)) return st;
  if (int st = S.alloc(&xn, (size_t)N * 8)) return st;
  if (int st = S.alloc(&yn, (size_t)N)) return st;
  EMU_DEV(hipMemcpyAsync(xd, x, (size_t)N * n.in * 8, hipMemcpyHostToDevice, s));
  EMU_DEV(hipMemcpyAsync(yd, y, (size_t)N * 8, hipMemcpyHostToDevice, s));
  EmuScale id{};
  for (int k = 0; k < 8; ++k) { id.lo[k] = -1.0; id.hi[k] = 1.0; }
  id.ymu = 0.0;
  id.ysig = 1.0;
  EMU_DEV(launch_emu_prep(xd, yd, nullptr, N, n.in, id, xn, yn, s));
  EmuTrain tr{};
  if (int st = train_scratch(S, n, (N + 63) / 64 * 64, tr)) return st;
  tr.n = N;
  tr.xn = xn;
  tr.yn = yn;
  tr.idx = nullptr;
  tr.scale = (float)(2.0 / (double)N);
  EmuAdam A{};
  A.do_adam = 0;
  A.grad = m->grad;
  A.loss = m->loss;
  A.inv_n = (float)(1.0 / (double)N);
  EMU_DEV(launch_emu_train_step(n, tr, A, s));
  EMU_DEV(hipMemcpyAsync(grad, m->grad, (size_t)n.E * n.P * 4, hipMemcpyDeviceToHost, s));
  std::vector<float> hl((size_t)n.E);
  EMU_DEV(hipMemcpyAsync(hl.data(), m->loss, (size_t)n.E * 4, hipMemcpyDeviceToHost, s));
  EMU_DEV(hipStreamSynchronize(s));
  if (loss)
    for (int e = 0; e < n.E; ++e) loss[e] = hl[e];
  return CF_OK;
}

int cf_emu_adam(cf_emu* m, const float* grad, double lr) {
  if (!m || !grad) return set_error(CF_EINVAL, "NULL argument");
  if (!(lr > 0.0) || !std::isfinite(lr)) return set_error(CF_EINVAL, "lr must be positive");
  std::lock_guard<std::mutex> lk(m->mu);
  if (int st = check_device(m)) return st;
  const EmuNet& n = m->net;
  EMU_DEV(hipMemcpyAsync(m->grad, grad, (size_t)n.E * n.P * 4, hipMemcpyHostToDevice, m->s));
  const EmuAdam A = adam_consts(m, lr);
  EMU_DEV(launch_emu_adam(n, m->grad, A, m->s));
  EMU_DEV(launch_emu_refresh(n, m->s));
  EMU_DEV(hipStreamSynchronize(m->s));
  ++m->step;
  return CF_OK;
}

// State file: "CFEMU002", int32 in, W, D, E, scaled, qdeg; int64 P, step, calls; uint64 seed;
// double lo[8], hi[8], ymu, ysig, b1, b2, eps, qc[45]; float master[E][P], m[E][P], v[E][P].
int cf_emu_save(const cf_emu* m, const char* path) {
  if (!m || !path) return set_error(CF_EINVAL, "NULL argument");
  if (int st = check_device(m)) return st;
  const EmuNet& n = m->net;
  const size_t np = (size_t)n.E * n.P;
  std::vector<float> a(np), b(np), c(np);
  EMU_DEV(hipStreamSynchronize(m->s));
  EMU_DEV(hipMemcpy(a.data(), n.master, np * 4, hipMemcpyDeviceToHost));
  EMU_DEV(hipMemcpy(b.data(), n.m, np * 4, hipMemcpyDeviceToHost));
  EMU_DEV(hipMemcpy(c.data(), n.v, np * 4, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) return set_error(CF_EINVAL, "cannot open %s for writing", path);
  const int32_t hi[6] = {n.in, n.W, n.D, n.E, m->scaled, m->sc.qdeg};
  const int64_t hl[3] = {n.P, m->step, m->calls};
  const double hd[21] = {m->sc.lo[0], m->sc.lo[1], m->sc.lo[2], m->sc.lo[3], m->sc.lo[4], m->sc.lo[5],
                         m->sc.lo[6], m->sc.lo[7], m->sc.hi[0], m->sc.hi[1], m->sc.hi[2], m->sc.hi[3],
                         m->sc.hi[4], m->sc.hi[5], m->sc.hi[6], m->sc.hi[7], m->sc.ymu, m->sc.ysig,
                         m->b1, m->b2, m->eps};
  bool ok = std::fwrite("CFEMU002", 1, 8, f) == 8 && std::fwrite(hi, 4, 6, f) == 6 &&
            std::fwrite(hl, 8, 3, f) == 3 && std::fwrite(&m->seed, 8, 1, f) == 1 &&
            std::fwrite(hd, 8, 21, f) == 21 && std::fwrite(m->sc.qc, 8, kEmuQ, f) == (size_t)kEmuQ &&
            std::fwrite(a.data(), 4, np, f) == np &&
            std::fwrite(b.data(), 4, np, f) == np && std::fwrite(c.data(), 4, np, f) == np;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return set_error(CF_EINVAL, "write to %s failed", path);
  return CF_OK;
}

int cf_emu_load(const char* path, cf_emu** out) {
  if (!path || !out) return set_error(CF_EINVAL, "NULL argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return set_error(CF_EINVAL, "cannot open %s", path);
  char magic[8];
  int32_t hi[6];
  int64_t hl[3];
  uint64_t seed;
  double hd[21], qc[kEmuQ];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "CFEMU002", 8) == 0 &&
            std::fread(hi, 4, 6, f) == 6 && std::fread(hl, 8, 3, f) == 3 &&
            std::fread(&seed, 8, 1, f) == 1 && std::fread(hd, 8, 21, f) == 21 &&
            std::fread(qc, 8, kEmuQ, f) == (size_t)kEmuQ;
  if (!ok) { std::fclose(f); return set_error(CF_EINVAL, "%s is not an emulator state file", path); }
  cf_emu* m = nullptr;
  if (int st = cf_emu_create(hi[0], hi[1], hi[2], hi[3], seed, &m)) { std::fclose(f); return st; }
  if (m->net.P != hl[0]) {
    std::fclose(f);
    cf_emu_destroy(m);
    return set_error(CF_EINVAL, "%s: parameter count mismatch", path);
  }
  const size_t np = (size_t)m->net.E * m->net.P;
  std::vector<float> a(np), b(np), c(np);
  ok = std::fread(a.data(), 4, np, f) == np && std::fread(b.data(), 4, np, f) == np &&
       std::fread(c.data(), 4, np, f) == np;
  std::fclose(f);
  if (!ok) { cf_emu_destroy(m); return set_error(CF_EINVAL, "%s is truncated", path); }
  m->scaled = hi[4];
  m->step = hl[1];
  m->calls = hl[2];
  for (int k = 0; k < 8; ++k) { m->sc.lo[k] = hd[k]; m->sc.hi[k] = hd[8 + k]; }
  m->sc.ymu = hd[16]; m->sc.ysig = hd[17];
  m->sc.qdeg = hi[5];
  std::memcpy(m->sc.qc, qc, sizeof qc);
  m->b1 = hd[18]; m->b2 = hd[19]; m->eps = hd[20];
  if (hipMemcpy(m->net.master, a.data(), np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->net.m, b.data(), np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->net.v, c.data(), np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      launch_emu_refresh(m->net, m->s) != hipSuccess || hipStreamSynchronize(m->s) != hipSuccess) {
    cf_emu_destroy(m);
    return set_error(CF_EDEVICE, "upload of %s failed", path);
  }
  *out = m;
  return CF_OK;
}

}  // extern "C"
