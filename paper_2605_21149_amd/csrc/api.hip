// C ABI of libcf: argument validation, staging, workspace, orchestration of the kernels.
#include "../../include/cf.h"
#include "cf_internal.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

// Workspace of the entry points that allocate nothing (cf_loglike_batch_noalloc): a file-scope
// device array of kScratchBytes, one copy per GPU, held until the process ends.  Host code never
// uses its name as an address (on the host it is only a stand-in): the device address comes from
// hipGetSymbolAddress, once per device with that device current, and is kept per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace cf {
namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define CF_DEV(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(_e == hipErrorOutOfMemory ? CF_ENOMEM : CF_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(_e), __FILE__, __LINE__);                   \
  } while (0)

// ------------------------------------------------------------------------------- per device
constexpr int kEvents = 16;
// Captured batches are replayed only for problems that a batch factorises in one outer panel
// (n <= 512): processes that captured and replayed batches of larger problems (n = 1088 and
// n = 3968 with 64 maps, factorised over several panels on three streams) ended with host
// segmentation faults whose cause is not established, so larger problems launch eagerly,
// host-paced one outer panel ahead (measured faster for n = 5952 batches of 8 than the replay).
constexpr int kGraphMaxN = 512;
// Probes of the mixed path's stochastic log-det correction: the estimate's standard deviation is
// about sqrt(2 / kLdProbes) |X|_F.  Measured with FP32 updates: 2.5e-4 at 256 probes on the QU
// N_side 16 scan problem (|X|_F about 2.8e-3), against biases of ln|C| of the FP32 factor of up to
// 1e-3 there and 2e-3 at n = 5952; 384 probes keep a deviation of 1e-3 beyond five of them.
constexpr int64_t kLdProbes = 384;
// Largest number of scan points factorised together, memory permitting: their covariances take at
// most kScanBytes, or an eighth of the device's memory if that is less.  Measured (64 maps,
// autotuned): 6 GB allowed batches of 22 at n = 5952 and 48 at n = 3968, and 24 GB batches of 64
// and 128, the scans' rates 613 -> 667 and 1890 -> 2080 points/s.
constexpr int kScanBatchMax = 128;
constexpr size_t kScanBytes = size_t(24) << 30;
// Call lanes per device: each lane is a complete set of streams, events, workspace and pinned
// flags, held by one call at a time.  A call takes the first free lane, so that two host threads
// can run two calls on one device at once; with every lane busy it waits for lane 0.
constexpr int kLanes = 2;
struct Device {
  std::mutex mu;
  hipStream_t stream = nullptr;
  hipStream_t aux[2] = {nullptr, nullptr};   // side streams for independent work (default priority)
  // Cholesky streams: the critical path (diagonal blocks, panels, lookahead columns) runs on a
  // small reserved set of CUs so that the bulk trailing update, which owns the rest, never delays
  // it.  Both are plain streams when CU masks are unavailable.
  hipStream_t crit = nullptr, bulk = nullptr, bulk2 = nullptr;   // bulk2: same CUs as bulk
  hipEvent_t ev[kEvents] = {};               // ordering events between the streams
  hipEvent_t ring[4] = {};                   // pacing events of the factorisation loop
  hipEvent_t jin = nullptr, jout = nullptr;   // a call joined after and back into the caller's stream
  char* ws = nullptr;
  size_t cap = 0;
  int* hflags = nullptr;   // pinned host mirror of the device flags
  char arch[64] = {0};     // the device's architecture name (gcnArchName up to its first ':')
  size_t mem = 0;          // the device's memory in bytes
  int id = -1;             // the device this lane belongs to
};
Device g_dev[64 * kLanes];
// Set for a device once two calls have overlapped on it (a call found lane 0 busy).  From then on
// single factorisations run on the plain streams too: the CU-masked streams reserve 32 CUs for the
// chain of diagonal blocks, which pays for a call alone on the device (a Fisher + QML of n = 5952:
// 11.8 ms masked, 12.7 ms plain) but less beside another call, whose kernels the reservation
// confines (that Fisher + QML beside an 8-point likelihood batch: 29.0 ms for the pair on plain
// streams, 29.6-30.0 ms with the masked ones; 27.7 ms for the two in sequence).
std::atomic<bool> g_overlap[64];

struct Bump {  // carves 256-byte aligned sub-buffers out of the workspace
  char* base;
  size_t off = 0;
  explicit Bump(char* b) : base(b) {}
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += (count * sizeof(T) + 255) & ~size_t(255);
    return p;
  }
};

int ensure_ws(Device& d, size_t bytes) {
  if (bytes <= d.cap) return CF_OK;
  if (d.ws) CF_DEV(hipFree(d.ws));
  d.ws = nullptr;
  d.cap = 0;
  size_t want = bytes + (bytes >> 4);
  hipError_t e = hipMalloc(&d.ws, want);
  if (e != hipSuccess) {
    d.ws = nullptr;
    return fail(CF_ENOMEM, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
  }
  d.cap = want;
  return CF_OK;
}

// Bytes a Bump would use for the given list of (count, size) pairs.
struct Sizer {
  size_t off = 0;
  template <typename T>
  void add(size_t count) { off += (count * sizeof(T) + 255) & ~size_t(255); }
};

// ------------------------------------------------------------------------------- problem
struct HostProblem {
  int npx = 0, nmaps = 0, has_t = 0, has_p = 0, n = 0;
  int lmin = 0, lmax = 0, kf = 0, nfm = 0;
  int64_t k = 0;
  std::vector<int> ring;          // active RING indices (nside > 0)
};

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

int check_problem(const cf_problem* P, HostProblem& H, bool need_cl) {
  if (!P) return fail(CF_EINVAL, "problem is NULL");
  if (P->fields < 1 || P->fields > 3) return fail(CF_EINVAL, "fields must be CF_T, CF_QU or CF_TQU");
  H.has_t = (P->fields & 1) != 0;
  H.has_p = (P->fields & 2) != 0;
  H.nmaps = (H.has_t ? 1 : 0) + (H.has_p ? 2 : 0);
  H.nfm = H.nmaps;
  if (P->lmin < 0 || P->lmax < P->lmin || P->lmax >= kMaxL)
    return fail(CF_EINVAL, "l-range chain broken: need 0 <= lmin <= lmax < %d (lmin=%d lmax=%d)", kMaxL,
                P->lmin, P->lmax);
  if (H.has_p && P->lmin < 2)
    return fail(CF_EINVAL, "lmin=%d below |spin|=2 with Q,U present", P->lmin);
  H.lmin = P->lmin;
  H.lmax = P->lmax;
  H.kf = (P->lmax + 1) * (P->lmax + 1) - P->lmin * P->lmin;
  H.k = (int64_t)H.nfm * H.kf;
  if (P->nside > 0) {
    if (P->nside > 8192) return fail(CF_EINVAL, "nside=%d too large", P->nside);
    int64_t np = 12LL * P->nside * P->nside;
    H.ring.clear();
    for (int64_t i = 0; i < np; ++i)
      if (!P->mask || P->mask[i]) H.ring.push_back((int)i);
    H.npx = (int)H.ring.size();
  } else if (P->nside == 0) {
    if (P->ndir <= 0 || !P->theta || !P->phi) return fail(CF_EINVAL, "explicit directions missing");
    if (!finite_all(P->theta, P->ndir) || !finite_all(P->phi, P->ndir))
      return fail(CF_EINVAL, "non-finite direction");
    H.npx = (int)P->ndir;
  } else {
    return fail(CF_EINVAL, "nside=%d < 0", P->nside);
  }
  if (H.npx <= 0) return fail(CF_EINVAL, "no retained pixels");
  int64_t n64 = (int64_t)H.npx * H.nmaps;
  if (n64 > (1LL << 20)) return fail(CF_EINVAL, "data dimension %lld too large", (long long)n64);
  H.n = (int)n64;
  const int L = P->lmax + 1;
  if (need_cl) {
    if (!P->cl) return fail(CF_EINVAL, "cl is NULL");
    if (!finite_all(P->cl, 6LL * L)) return fail(CF_EINVAL, "non-finite C_l");
  }
  if (P->bl && !finite_all(P->bl, L)) return fail(CF_EINVAL, "non-finite beam");
  if (P->pl && !finite_all(P->pl, L)) return fail(CF_EINVAL, "non-finite pixel window");
  if (P->noise_kind != CF_NOISE_DIAG && P->noise_kind != CF_NOISE_DENSE)
    return fail(CF_EINVAL, "unknown noise_kind %d", P->noise_kind);
  if (!P->noise) return fail(CF_EINVAL, "noise is NULL");
  if (P->noise_rank < 0 || (P->noise_rank > 0 && !P->noise_U))
    return fail(CF_EINVAL, "noise_rank=%d with noise_U=%p", P->noise_rank, (const void*)P->noise_U);
  if (P->mem != CF_MEM_HOST && P->mem != CF_MEM_DEVICE) return fail(CF_EINVAL, "unknown mem %d", P->mem);
  if (P->mem == CF_MEM_HOST) {
    int64_t nn = P->noise_kind == CF_NOISE_DENSE ? (int64_t)H.n * H.n : H.n;
    if (!finite_all(P->noise, nn)) return fail(CF_EINVAL, "non-finite noise covariance");
    if (P->noise_rank > 0 && !finite_all(P->noise_U, (int64_t)H.n * P->noise_rank))
      return fail(CF_EINVAL, "non-finite noise_U");
  }
  return CF_OK;
}

struct HostBins {
  int ns = 0, nb = 0;
  int spec[6] = {0, 0, 0, 0, 0, 0};
  std::vector<int> lo, hi;
};

int check_bins(const cf_bins* B, const HostProblem& H, HostBins& out) {
  if (!B) return fail(CF_EINVAL, "bins is NULL");
  if (B->nbins <= 0 || !B->lo || !B->hi) return fail(CF_EINVAL, "empty bins");
  out.ns = 0;
  for (int s = 0; s < 6; ++s) {
    if (!(B->spectra & (1u << s))) continue;
    bool needT = (s == 0 || s == 3 || s == 4), needP = (s != 0);
    if ((needT && !H.has_t) || (needP && !H.has_p))
      return fail(CF_EINVAL, "spectrum %d requested for an absent field", s);
    out.spec[out.ns++] = s;
  }
  if (out.ns == 0) return fail(CF_EINVAL, "no spectra requested");
  if (B->spectra & ~63u) return fail(CF_EINVAL, "unknown spectrum bits");
  out.nb = B->nbins;
  if ((int64_t)out.ns * out.nb > 1024)
    return fail(CF_EINVAL, "%d spectra x %d bins exceeds the 1024 Fisher parameters supported", out.ns, out.nb);
  out.lo.assign(B->lo, B->lo + B->nbins);
  out.hi.assign(B->hi, B->hi + B->nbins);
  for (int b = 0; b < out.nb; ++b)
    if (out.lo[b] < H.lmin || out.hi[b] > H.lmax || out.lo[b] > out.hi[b])
      return fail(CF_EINVAL, "bin %d = [%d, %d] outside [lmin, lmax] = [%d, %d]", b, out.lo[b],
                  out.hi[b], H.lmin, H.lmax);
  return CF_OK;
}

// ------------------------------------------------------------------------------- staging
struct Staged {
  DevProblem P;
  int* ring = nullptr;
  double* theta = nullptr;
  double* phi = nullptr;
  double* cl = nullptr;
  double* bl = nullptr;
  double* pl = nullptr;
  double* pix = nullptr;
  double* cw = nullptr;
  double* wl = nullptr;
  double* lam = nullptr;
  double* coef = nullptr;
  const double* noise = nullptr;
  const double* noise_U = nullptr;
};

void size_staging(Sizer& z, const cf_problem* P, const HostProblem& H) {
  const int L = H.lmax + 1;
  z.add<int>(H.npx);
  z.add<double>(H.npx);
  z.add<double>(H.npx);
  z.add<double>(6 * L);
  z.add<double>(L);
  z.add<double>(L);
  z.add<double>((size_t)H.npx * kPixRec);
  z.add<double>(6 * L);
  z.add<double>(L);
  z.add<double>(6 * L);
  z.add<double>((size_t)L * kCoef);
  if (P->mem == CF_MEM_HOST) {
    z.add<double>(P->noise_kind == CF_NOISE_DENSE ? (size_t)H.n * H.n : (size_t)H.n);
    if (P->noise_rank > 0) z.add<double>((size_t)H.n * P->noise_rank);
  }
}

int stage(Bump& bp, const cf_problem* P, const HostProblem& H, const double* cl_override,
          hipStream_t s, Staged& S) {
  const int L = H.lmax + 1;
  S.ring = bp.take<int>(H.npx);
  S.theta = bp.take<double>(H.npx);
  S.phi = bp.take<double>(H.npx);
  S.cl = bp.take<double>(6 * L);
  S.bl = bp.take<double>(L);
  S.pl = bp.take<double>(L);
  S.pix = bp.take<double>((size_t)H.npx * kPixRec);
  S.cw = bp.take<double>(6 * L);
  S.wl = bp.take<double>(L);
  S.lam = bp.take<double>(6 * L);
  S.coef = bp.take<double>((size_t)L * kCoef);
  if (P->nside > 0) {
    CF_DEV(hipMemcpyAsync(S.ring, H.ring.data(), sizeof(int) * H.npx, hipMemcpyHostToDevice, s));
  } else {
    CF_DEV(hipMemcpyAsync(S.theta, P->theta, sizeof(double) * H.npx, hipMemcpyHostToDevice, s));
    CF_DEV(hipMemcpyAsync(S.phi, P->phi, sizeof(double) * H.npx, hipMemcpyHostToDevice, s));
  }
  const double* cl = cl_override ? cl_override : P->cl;
  if (cl) {
    CF_DEV(hipMemcpyAsync(S.cl, cl, sizeof(double) * 6 * L, hipMemcpyHostToDevice, s));
  } else {
    CF_DEV(launch_fill(S.cl, 6 * L, 0.0, s));
  }
  if (P->bl) CF_DEV(hipMemcpyAsync(S.bl, P->bl, sizeof(double) * L, hipMemcpyHostToDevice, s));
  else CF_DEV(launch_fill(S.bl, L, 1.0, s));
  if (P->pl) CF_DEV(hipMemcpyAsync(S.pl, P->pl, sizeof(double) * L, hipMemcpyHostToDevice, s));
  else CF_DEV(launch_fill(S.pl, L, 1.0, s));
  CF_DEV(launch_geometry(S.ring, P->nside, S.theta, S.phi, H.npx, S.pix, s));
  CF_DEV(launch_tables(S.cl, S.bl, S.pl, H.lmin, H.lmax, 1, 0, L, S.cw, S.wl, S.lam, S.coef, s));
  if (P->mem == CF_MEM_HOST) {
    size_t nn = P->noise_kind == CF_NOISE_DENSE ? (size_t)H.n * H.n : (size_t)H.n;
    double* nz = bp.take<double>(nn);
    CF_DEV(hipMemcpyAsync(nz, P->noise, sizeof(double) * nn, hipMemcpyHostToDevice, s));
    S.noise = nz;
    if (P->noise_rank > 0) {
      double* u = bp.take<double>((size_t)H.n * P->noise_rank);
      CF_DEV(hipMemcpyAsync(u, P->noise_U, sizeof(double) * H.n * P->noise_rank, hipMemcpyHostToDevice, s));
      S.noise_U = u;
    }
  } else {
    S.noise = P->noise;
    S.noise_U = P->noise_U;
  }
  DevProblem& D = S.P;
  D.npx = H.npx; D.nmaps = H.nmaps; D.has_t = H.has_t; D.has_p = H.has_p; D.n = H.n;
  D.lmin = H.lmin; D.lmax = H.lmax; D.kf = H.kf; D.nfm = H.nfm; D.k = H.k;
  D.pix = S.pix; D.coef = S.coef; D.cw = S.cw; D.wl = S.wl; D.lam = S.lam;
  return CF_OK;
}

// ------------------------------------------------------------------------------- timing
struct Timer {
  bool on = false;
  hipStream_t s = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  struct Iv { int stage; hipEvent_t a, b; };
  std::vector<Iv> iv;
  std::vector<std::pair<int, hipEvent_t>> marks;   // sequential marks on the main stream
  KernTimer kt;                                     // per-launch GEMM events of this call
  ~Timer() {
    if (g_ktimer == &kt) g_ktimer = nullptr;        // also on early error returns
    for (auto& r : kt.rec) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  }
  hipEvent_t make() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { on = false; return nullptr; }
    return e;
  }
  void begin(bool enable, hipStream_t st) {
    on = enable;
    s = st;
    if (!on) return;
    t0 = make();
    if (t0) (void)hipEventRecord(t0, s);
    marks.push_back({-1, t0});
    g_ktimer = &kt;
  }
  // main-stream stage boundary: the interval since the previous mark is charged to stage_id
  void mark(int stage_id) {
    if (!on) return;
    hipEvent_t e = make();
    if (!e) return;
    (void)hipEventRecord(e, s);
    marks.push_back({stage_id, e});
  }
  // explicit interval on any stream
  hipEvent_t open(hipStream_t st) {
    if (!on) return nullptr;
    hipEvent_t e = make();
    if (e) (void)hipEventRecord(e, st);
    return e;
  }
  void close(int stage_id, hipEvent_t a, hipStream_t st) {
    if (!on || !a) return;
    hipEvent_t b = make();
    if (!b) return;
    (void)hipEventRecord(b, st);
    iv.push_back({stage_id, a, b});
  }
  void finish(cf_report* rep) {
    if (!on) return;
    t1 = make();
    if (!t1) return;
    (void)hipEventRecord(t1, s);
    (void)hipEventSynchronize(t1);
    for (size_t i = 1; i < marks.size(); ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, marks[i - 1].second, marks[i].second);
      if (rep && marks[i].first >= 0 && marks[i].first < 8) rep->ms_stage[marks[i].first] += ms;
    }
    for (auto& x : iv) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, x.a, x.b);
      if (rep && x.stage >= 0 && x.stage < 8) rep->ms_stage[x.stage] += ms;
    }
    float tot = 0.f;
    (void)hipEventElapsedTime(&tot, t0, t1);
    if (rep) rep->ms_total = tot;
    if (g_ktimer == &kt) g_ktimer = nullptr;
    for (auto& r : kt.rec) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, r.a, r.b);
      if (rep && r.id >= 0 && r.id < kGemmIds) {
        rep->gemm_ms[r.id] += ms;
        rep->gemm_flops[r.id] += r.flops;
        rep->gemm_bytes[r.id] += r.bytes;
        rep->gemm_launches[r.id] += 1;
      }
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    kt.rec.clear();
    for (auto& m : marks) (void)hipEventDestroy(m.second);
    for (auto& x : iv) { (void)hipEventDestroy(x.a); (void)hipEventDestroy(x.b); }
    (void)hipEventDestroy(t1);
    marks.clear();
    iv.clear();
  }
};
enum { ST_BUILD = 0, ST_POTRF, ST_YBUILD, ST_TRSM, ST_SYRK, ST_REDUCE, ST_QML, ST_OTHER };

// Reserve 4 CUs per XCD (32 of 256) for the critical path.  With 32 CUs per XCD the CU index i
// lies on XCD i / 32 if CUs are numbered XCD by XCD, or on XCD i % 8 if they alternate; the set
// {i : i % 8 == (i / 32) % 8} holds 4 CUs of every XCD under either numbering.
void make_cholesky_streams(Device& d, int id) {
  hipDeviceProp_t prop;
  d.crit = d.bulk = nullptr;
  const char* env = getenv("CF_CU_MASK");   // "0": plain streams (e.g. for counter collection)
  if (env && env[0] == '0') return;
  if (hipGetDeviceProperties(&prop, id) != hipSuccess) return;
  const int ncu = prop.multiProcessorCount;
  if (ncu < 64 || ncu % 8 || ncu > 1024) return;
  const int per = ncu / 8;
  std::vector<uint32_t> mc((ncu + 31) / 32, 0u), mb((ncu + 31) / 32, 0u);
  for (int i = 0; i < ncu; ++i) {
    const bool c = (i % 8) == ((i / per) % 8);
    (c ? mc : mb)[i / 32] |= 1u << (i % 32);
  }
  hipStream_t a = nullptr, b = nullptr, b2 = nullptr;
  if (hipExtStreamCreateWithCUMask(&a, (uint32_t)mc.size(), mc.data()) != hipSuccess) return;
  if (hipExtStreamCreateWithCUMask(&b, (uint32_t)mb.size(), mb.data()) != hipSuccess) {
    (void)hipStreamDestroy(a);
    return;
  }
  if (hipExtStreamCreateWithCUMask(&b2, (uint32_t)mb.size(), mb.data()) != hipSuccess) {
    (void)hipStreamDestroy(a);
    (void)hipStreamDestroy(b);
    return;
  }
  d.crit = a;
  d.bulk = b;
  d.bulk2 = b2;
}

// Factorisation on the reserved-CU streams, ordered after and joined back into s.
int potrf_on(Device& d, Factor& F, double* scratch, hipStream_t s, hipStream_t side, hipEvent_t* ev) {
  // A batch of factorisations is bound by its bulk updates, not by the chain of diagonal blocks:
  // it keeps every CU for the bulk work.
  // The reserved-CU streams are never used while s is being captured into a graph (a captured
  // scan with CU-masked streams taking part crashed the runtime).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  CF_DEV(hipStreamIsCapturing(s, &cap));
  if (!d.crit || F.batch > 1 || cap != hipStreamCaptureStatusNone ||
      (d.id >= 0 && g_overlap[d.id].load(std::memory_order_relaxed))) {
    Streams st{s, d.aux[0], side, ev[0], ev[1], ev[2], d.ring};
    st.eT = ev[6];   // lookahead of depth two
    CF_DEV(potrf_f64(F, scratch, st));
    return CF_OK;
  }
  CF_DEV(hipEventRecord(ev[3], s));
  CF_DEV(hipStreamWaitEvent(d.crit, ev[3], 0));
  CF_DEV(hipStreamWaitEvent(d.bulk, ev[3], 0));
  CF_DEV(hipStreamWaitEvent(d.bulk2, ev[3], 0));
  Streams st{d.crit, d.bulk, d.bulk2, ev[0], ev[1], ev[2], d.ring};
  // the lookahead update runs on the bulk CUs, ahead of the trailing update (measured on the
  // n = 5952 factorisation with its solves: 9.6 -> 9.0-9.3 ms)
  st.eA = ev[5];
  CF_DEV(potrf_f64(F, scratch, st));
  CF_DEV(hipEventRecord(ev[4], d.crit));
  CF_DEV(hipStreamWaitEvent(s, ev[4], 0));
  return CF_OK;
}

// Releases every device object the library keeps between calls (defined with the scan graphs).
void release_device_state();
std::once_flag g_atexit_once;

// Device addresses of the scratch array (declared at file scope above), one per device.
char* g_scratch[64] = {};

struct CallCtx {
  Device* dev = nullptr;
  hipStream_t s = nullptr;
  hipStream_t caller = nullptr;   // the caller's stream, joined into s at the start and back at the end
  int id = 0;
  std::unique_lock<std::mutex> lock;
  ~CallCtx() {
    if (caller && dev && s && dev->jout && hipEventRecord(dev->jout, s) == hipSuccess)
      (void)hipStreamWaitEvent(caller, dev->jout, 0);
  }
  // For the entry points that allocate nothing: the caller's stream (or the null stream), no
  // library streams, events or pinned buffers; the scratch array's address is looked up on the
  // first such call on the device.
  int begin_plain(const cf_exec* ex) {
    CF_DEV(hipGetDevice(&id));
    if (id < 0 || id >= 64) return fail(CF_EDEVICE, "device id %d unsupported", id);
    std::call_once(g_atexit_once, [] { std::atexit(release_device_state); });
    dev = &g_dev[id * kLanes];          // the scratch array is the device's: one such call at a time
    lock = std::unique_lock<std::mutex>(dev->mu);
    if (!g_scratch[id]) {
      void* p = nullptr;
      hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(CF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      g_scratch[id] = static_cast<char*>(p);
    }
    s = (ex && ex->stream) ? (hipStream_t)ex->stream : nullptr;
    return CF_OK;
  }
  int begin(const cf_exec* ex) {
    CF_DEV(hipGetDevice(&id));
    if (id < 0 || id >= 64) return fail(CF_EDEVICE, "device id %d unsupported", id);
    // Registered after the runtime is initialised, so it runs before the runtime's own teardown:
    // graphs, streams (CU-masked ones included), events and memory go back while the runtime and
    // any profiler attached to it are still whole.
    std::call_once(g_atexit_once, [] { std::atexit(release_device_state); });
    dev = nullptr;
    for (int l = 0; l < kLanes && !dev; ++l) {
      std::unique_lock<std::mutex> t(g_dev[id * kLanes + l].mu, std::try_to_lock);
      if (t.owns_lock()) {
        dev = &g_dev[id * kLanes + l];
        lock = std::move(t);
      }
    }
    if (!dev) {
      dev = &g_dev[id * kLanes];
      lock = std::unique_lock<std::mutex>(dev->mu);
    }
    if (dev != &g_dev[id * kLanes]) g_overlap[id].store(true, std::memory_order_relaxed);
    if (!dev->stream) {
      dev->id = id;
      CF_DEV(hipStreamCreateWithFlags(&dev->stream, hipStreamNonBlocking));
      for (auto& a : dev->aux) CF_DEV(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
      for (auto& e : dev->ev) CF_DEV(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      for (auto& e : dev->ring) CF_DEV(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      CF_DEV(hipEventCreateWithFlags(&dev->jin, hipEventDisableTiming));
      CF_DEV(hipEventCreateWithFlags(&dev->jout, hipEventDisableTiming));
      make_cholesky_streams(*dev, id);
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, id) == hipSuccess) {
        dev->mem = prop.totalGlobalMem;
        size_t k = 0;
        while (k + 1 < sizeof dev->arch && prop.gcnArchName[k] && prop.gcnArchName[k] != ':') {
          dev->arch[k] = prop.gcnArchName[k];
          ++k;
        }
        dev->arch[k] = 0;
      }
      if (!dev->arch[0]) std::snprintf(dev->arch, sizeof dev->arch, "unknown");
    }
    if (!dev->hflags) CF_DEV(hipHostMalloc((void**)&dev->hflags, 64 * sizeof(int), hipHostMallocDefault));
    // The kernels run on the lane's own streams, ordered after the caller's stream and joined back
    // into it when the call returns.  Computing on the caller's stream instead made the call's
    // speed depend on which hardware queue the runtime had mapped that stream to: sharing one
    // with the lane's side streams serialises the factorisation's chain with its own trailing
    // updates (an 8-point likelihood batch at n = 5952: 15.3 ms on the lane's stream, 16.3 ms on
    // a stream of the caller's; a Fisher + QML without the CU-masked streams 12.7 vs 16.0 ms).
    s = dev->stream;
    hipStream_t cs = (ex && ex->stream) ? (hipStream_t)ex->stream : nullptr;
    if (cs && cs != s) {
      CF_DEV(hipEventRecord(dev->jin, cs));
      CF_DEV(hipStreamWaitEvent(s, dev->jin, 0));
      caller = cs;
    }
    return CF_OK;
  }
};

void report_init(cf_report* rep) {
  if (!rep) return;
  std::memset(rep, 0, sizeof *rep);
  rep->fail_index = -1;
}

// The same through ordinary host memory (no pinned buffer), for the entry points that allocate nothing.
int read_flags_plain(CallCtx& c, const int* dflags, int nflags, int* out) {
  int tmp[8];
  if (nflags > 8) return fail(CF_EINVAL, "internal: %d flags", nflags);
  CF_DEV(hipMemcpyAsync(tmp, dflags, sizeof(int) * nflags, hipMemcpyDeviceToHost, c.s));
  CF_DEV(hipStreamSynchronize(c.s));
  for (int i = 0; i < nflags; ++i) out[i] = tmp[i];
  return CF_OK;
}

// Copy back two device ints (cov flag, pivot failure) and turn them into a status.
int read_flags(CallCtx& c, const int* dflags, int nflags, int* out) {
  CF_DEV(hipMemcpyAsync(c.dev->hflags, dflags, sizeof(int) * nflags, hipMemcpyDeviceToHost, c.s));
  CF_DEV(hipStreamSynchronize(c.s));
  for (int i = 0; i < nflags; ++i) out[i] = c.dev->hflags[i];
  return CF_OK;
}

// ------------------------------------------------------------------------------- Fisher core
struct FisherBufs {
  double *C, *C0, *Y, *G, *Z, *Linv, *Li256, *scratch, *ldpart, *gram, *ztr, *F;
  double *Gc, *Xr;   // mixed: copy of G and L^-T G for the refinement of C^-1 Y
  int* lo;
  int* hi;
  int* flags;   // [0] non-finite covariance, [1] first failing pivot, [2] F pivot failure
};

// Buffers of the Fisher path.  FP64 factorises [C; D^T; Y^T] (n + nm + k rows, ld n) in one
// pass, so that u^T = (L^-1 d)^T and G^T = (L^-1 Y)^T come out of the factorisation as the rows
// below C.  Mixed: C, Y and G apart, plus an FP64 copy of C for the refinement residuals.
struct FisherSizes { size_t C, C0, Y, G, Li256, Gc, Xr; };
FisherSizes fisher_sizes(const HostProblem& H, int mode, int nm) {
  const size_t n = H.n, k = H.k;
  FisherSizes q;
  q.C = mode ? n * n : (n + nm + k) * n;
  q.C0 = mode ? n * n : 1;
  q.Y = n * k;
  q.G = mode ? n * k : 1;
  q.Li256 = mode ? (n / 256) * 256 * 256 : 1;
  q.Gc = mode ? n * k : 1;   // refinement of C^-1 Y (mixed)
  q.Xr = mode ? n * k : 1;
  return q;
}

size_t fisher_ws(const HostProblem& H, const HostBins& B, Sizer& z, int mode, int nm) {
  const int nl = H.lmax - H.lmin + 1;
  const int np = H.nfm * H.nfm, nq = np * (np + 1) / 2;
  const int K = B.ns * B.nb;
  const FisherSizes q = fisher_sizes(H, mode, nm);
  z.add<double>(q.C);
  z.add<double>(q.C0);
  z.add<double>(q.Y);
  z.add<double>(q.G);
  z.add<double>(q.Gc);
  z.add<double>(q.Xr);
  z.add<double>((size_t)H.k * H.k);
  z.add<double>((size_t)((H.n + kNB - 1) / kNB) * kNB * kNB);
  z.add<double>(q.Li256);
  z.add<double>((size_t)potrf_scratch(1));
  z.add<double>((H.n + kNB - 1) / kNB);
  z.add<double>((size_t)nl * (nl + 1) / 2 * nq);
  z.add<double>((size_t)nl * np);
  z.add<double>((size_t)K * K);
  z.add<int>(B.nb);
  z.add<int>(B.nb);
  z.add<int>(8);
  return z.off;
}

void fisher_take(Bump& bp, const HostProblem& H, const HostBins& B, FisherBufs& f, int mode, int nm) {
  const int nl = H.lmax - H.lmin + 1;
  const int np = H.nfm * H.nfm, nq = np * (np + 1) / 2;
  const int K = B.ns * B.nb;
  const FisherSizes q = fisher_sizes(H, mode, nm);
  f.C = bp.take<double>(q.C);
  f.C0 = bp.take<double>(q.C0);
  f.Y = bp.take<double>(q.Y);
  f.G = bp.take<double>(q.G);
  f.Gc = bp.take<double>(q.Gc);
  f.Xr = bp.take<double>(q.Xr);
  f.Z = bp.take<double>((size_t)H.k * H.k);
  f.Linv = bp.take<double>((size_t)((H.n + kNB - 1) / kNB) * kNB * kNB);
  f.Li256 = bp.take<double>(q.Li256);
  f.scratch = bp.take<double>((size_t)potrf_scratch(1));
  f.ldpart = bp.take<double>((H.n + kNB - 1) / kNB);
  f.gram = bp.take<double>((size_t)nl * (nl + 1) / 2 * nq);
  f.ztr = bp.take<double>((size_t)nl * np);
  f.F = bp.take<double>((size_t)K * K);
  f.lo = bp.take<int>(B.nb);
  f.hi = bp.take<int>(B.nb);
  f.flags = bp.take<int>(8);
}

Factor make_factor(const FisherBufs& f, int64_t n, int mode) {
  Factor F;
  F.L = f.C; F.n = n; F.ld = n; F.sL = 0;
  F.Li64 = f.Linv; F.sLi64 = 0;
  F.Li256 = (n >= 256 && mode) ? f.Li256 : nullptr; F.sLi256 = 0;
  F.ldpart = f.ldpart; F.sPart = 0;
  F.fail = f.flags + 1;
  F.batch = 1;
  F.mode = mode;
  return F;
}

// Optional QML part of a Fisher call: maps and the buffers of u = L^-1 d and w = G^T u.
struct QmlBufs {
  const double* maps = nullptr;   // device [nmaps][n]
  int nmaps = 0;
  double *D = nullptr, *U = nullptr, *W = nullptr, *part = nullptr;
  double *D0 = nullptr, *X = nullptr, *R = nullptr;   // mixed precision: d, C^-1 d, residual
  int refine = 0;
};

// W (M x nmaps) = A^T U with A = rows [0, K) of a row-major matrix (ld lda) and U (K x nmaps):
// a skinny product for a few maps, the MFMA GEMM otherwise.
hipError_t weighted_maps(const double* A, int64_t lda, int64_t M, int64_t K, const double* U, int nmaps,
                         double* W, double* part, hipStream_t s) {
  if (nmaps <= 8) return gemv_tn(A, lda, M, K, U, nmaps, W, nmaps, part, s);
  GemmDesc w{};
  w.M = M; w.N = nmaps; w.K = K;
  w.A = A; w.lda = lda; w.at = 1;
  w.B = U; w.ldb = nmaps; w.bt = 0;
  w.C = W; w.ldc = nmaps; w.alpha = 1.0; w.beta = 0.0; w.batch = 1;
  return gemm_f64(w, s);
}

// FP64: one factorisation of [C; D^T; Y^T] gives L, u^T = (L^-1 d)^T and G^T = (L^-1 Y)^T (the
// rows below C trail the factorisation on its side stream); Z = G^T G and w = G^T u are products
// of those rows.  Y is built on aux[0] while s builds C.  For T+QU problems the E,B rows of Y^T
// vanish on the T pixels: they are placed last, stay out of the panels that end before the first
// Q pixel, and their Z products start at that pixel.
int fisher_core_fp64(const cf_problem* prob, const HostProblem& H, const Staged& S, FisherBufs& f,
                     QmlBufs* qb, CallCtx& cc, Timer& tm) {
  const DevProblem& P = S.P;
  const int64_t n = H.n, k = H.k;
  const int nm = qb ? qb->nmaps : 0;
  hipStream_t s = cc.s, s1 = cc.dev->aux[0], s2 = cc.dev->aux[1];
  hipEvent_t* ev = cc.dev->ev;
  enum { E_START = 0, E_Y, E_L, E_S1 };
  double* Dt = f.C + n * n;                 // nm rows: d^T, then u^T
  double* Gt = Dt + (int64_t)nm * n;        // k rows: Y^T, then G^T
  CF_DEV(hipEventRecord(ev[E_START], s));
  CF_DEV(hipStreamWaitEvent(s1, ev[E_START], 0));
  hipEvent_t ty = tm.open(s1);
  CF_DEV(launch_ybuild(P, f.Y, k, s1));
  CF_DEV(launch_transpose(f.Y, n, k, k, Gt, n, s1));
  tm.close(ST_YBUILD, ty, s1);
  CF_DEV(hipEventRecord(ev[E_Y], s1));
  CF_DEV(launch_fill_int(f.flags, 1, 0, s));
  CF_DEV(launch_fill_int(f.flags + 1, 2, INT_MAX, s));
  CF_DEV(launch_cov_build(P, S.cw, 0, 1, prob->noise_kind, S.noise, prob->noise_rank, S.noise_U, f.C, n,
                          0, 1, f.flags, s));
  if (nm) CF_DEV(hipMemcpyAsync(Dt, qb->maps, sizeof(double) * nm * n, hipMemcpyDeviceToDevice, s));
  tm.mark(ST_BUILD);
  CF_DEV(hipStreamWaitEvent(s, ev[E_Y], 0));
  const bool split = H.has_t && H.has_p;
  const int64_t kT = H.has_t ? H.kf : 0, kP = k - kT;
  const int64_t p0 = split ? (H.npx / kNB) * kNB : 0;
  Factor F = make_factor(f, n, 0);
  F.rows = n + nm + k;
  if (split) { F.rows_early = n + nm + kT; F.p_early = H.npx; }
  if (int st = potrf_on(*cc.dev, F, f.scratch, s, s2, ev + 8)) return st;
  tm.mark(ST_POTRF);
  // Z = G^T G, lower blocks.  For T+QU problems the symmetric product of the E,B block is the
  // separately named kernel instance (tag 1) whose launch the stage timer brackets on its own
  // stream; other problems' Z products use the plain instance, so that profiles of a process that
  // runs several problems see one shape under the tagged name.
  if (split) {
    // The E,B block (columns >= p0 only) on aux[0]; the T block over all columns and then the E,B
    // rows against the T columns on s, so that the two streams carry similar work (measured: the
    // Z stage 3.43-3.55 -> 3.28-3.38 ms against the E,B x T product ahead of the E,B block on aux[0])
    CF_DEV(hipEventRecord(ev[E_L], s));
    CF_DEV(hipStreamWaitEvent(s1, ev[E_L], 0));
    GemmDesc h{};
    h.M = kP; h.N = kT; h.K = n - p0;
    h.A = Gt + kT * n + p0; h.lda = n; h.at = 0;
    h.B = Gt + p0; h.ldb = n; h.bt = 1;
    h.C = f.Z + kT * k; h.ldc = k; h.alpha = 1.0; h.beta = 0.0; h.batch = 1;
    GemmDesc e = h;
    e.N = kP;
    e.B = Gt + kT * n + p0;
    e.C = f.Z + kT * k + kT; e.lower = 1; e.tag = 1;
    hipEvent_t tz = tm.open(s1);
    CF_DEV(gemm_f64(e, s1));
    tm.close(ST_SYRK, tz, s1);
    CF_DEV(hipEventRecord(ev[E_S1], s1));
    GemmDesc g{};
    g.M = kT; g.N = kT; g.K = n;
    g.A = Gt; g.lda = n; g.at = 0;
    g.B = Gt; g.ldb = n; g.bt = 1;
    g.C = f.Z; g.ldc = k; g.alpha = 1.0; g.beta = 0.0; g.lower = 1; g.batch = 1;
    CF_DEV(gemm_f64(g, s));
    CF_DEV(gemm_f64(h, s));
    CF_DEV(hipStreamWaitEvent(s, ev[E_S1], 0));
  } else {
    GemmDesc g{};
    g.M = k; g.N = k; g.K = n;
    g.A = Gt; g.lda = n; g.at = 0;
    g.B = Gt; g.ldb = n; g.bt = 1;
    g.C = f.Z; g.ldc = k; g.alpha = 1.0; g.beta = 0.0; g.lower = 1; g.batch = 1;
    hipEvent_t tz = tm.open(s);
    CF_DEV(gemm_f64(g, s));
    tm.close(ST_SYRK, tz, s);
  }
  if (qb && nm <= 8) {   // w = G^T u  (k x nm): one streaming pass over the rows of G^T
    CF_DEV(launch_rowdot(Gt, n, k, n, Dt, n, nm, qb->W, nm, split ? kT : k, p0, s));
  } else if (qb) {
    GemmDesc w{};
    w.M = k; w.N = nm; w.K = n;
    w.A = Gt; w.lda = n; w.at = 0;
    w.B = Dt; w.ldb = n; w.bt = 1;
    w.C = qb->W; w.ldc = nm; w.alpha = 1.0; w.beta = 0.0; w.batch = 1;
    CF_DEV(gemm_f64(w, s));
  }
  tm.mark(ST_OTHER);
  CF_DEV(launch_symmetrize(f.Z, k, k, s));
  CF_DEV(launch_gram(P, f.Z, k, f.gram, f.ztr, s));
  tm.mark(ST_REDUCE);
  return CF_OK;
}

// Covariance, factor, Y, G = L^-1 Y, Z = G^T G (+ u = L^-1 d, w = G^T u), Gram of Z blocks.
// Three streams: the call's stream s carries the covariance, the factorisation and the T part;
// aux[0] builds Y (concurrently with the factorisation) and then carries the E,B part; aux[1]
// solves the maps.  Events order the hand-offs; everything is joined back into s.
int fisher_core(const cf_problem* prob, const HostProblem& H, const Staged& S, FisherBufs& f,
                QmlBufs* qb, CallCtx& cc, Timer& tm, int mode) {
  if (mode == 0) return fisher_core_fp64(prob, H, S, f, qb, cc, tm);
  const DevProblem& P = S.P;
  const int64_t n = H.n, k = H.k;
  hipStream_t s = cc.s, s1 = cc.dev->aux[0], s2 = cc.dev->aux[1];
  hipEvent_t* ev = cc.dev->ev;
  enum { E_START = 0, E_Y, E_L, E_T, E_EB, E_S1, E_S2 };
  CF_DEV(hipEventRecord(ev[E_START], s));
  CF_DEV(hipStreamWaitEvent(s1, ev[E_START], 0));
  CF_DEV(hipStreamWaitEvent(s2, ev[E_START], 0));
  // aux[0]: harmonic basis, independent of the covariance
  hipEvent_t ty = tm.open(s1);
  CF_DEV(launch_ybuild(P, f.Y, k, s1));
  tm.close(ST_YBUILD, ty, s1);
  CF_DEV(hipEventRecord(ev[E_Y], s1));
  // s: covariance and Cholesky factor
  CF_DEV(launch_fill_int(f.flags, 1, 0, s));
  CF_DEV(launch_fill_int(f.flags + 1, 2, INT_MAX, s));
  // the mixed path keeps the full FP64 covariance for its refinement residuals
  CF_DEV(launch_cov_build(P, S.cw, 0, 1, prob->noise_kind, S.noise, prob->noise_rank, S.noise_U, f.C, n,
                          0, mode ? 0 : 1, f.flags, s));
  if (mode) CF_DEV(hipMemcpyAsync(f.C0, f.C, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
  tm.mark(ST_BUILD);
  Factor F = make_factor(f, n, mode);
  if (int st = potrf_on(*cc.dev, F, f.scratch, s, s2, ev + 8)) return st;
  tm.mark(ST_POTRF);
  CF_DEV(hipEventRecord(ev[E_L], s));
  // aux[1]: u = L^-1 d for the maps (FP64); x = C^-1 d refined with FP64 residuals (mixed)
  if (qb) {
    const int nm = qb->nmaps;
    CF_DEV(hipStreamWaitEvent(s2, ev[E_L], 0));
    CF_DEV(launch_transpose(qb->maps, nm, n, n, qb->D, nm, s2));
    if (mode) {
      CF_DEV(hipMemcpyAsync(qb->D0, qb->D, sizeof(double) * n * nm, hipMemcpyDeviceToDevice, s2));
      CF_DEV(trsm_lower_f64(F, qb->D, nm, 0, qb->U, nm, 0, nm, 0, s2));
      CF_DEV(trsm_lower_t_f64(F, qb->U, nm, 0, qb->X, nm, 0, nm, s2));
      for (int it = 0; it < qb->refine; ++it) {
        CF_DEV(hipMemcpyAsync(qb->R, qb->D0, sizeof(double) * n * nm, hipMemcpyDeviceToDevice, s2));
        GemmDesc r{};
        r.M = n; r.N = nm; r.K = n;
        r.A = f.C0; r.lda = n; r.B = qb->X; r.ldb = nm; r.C = qb->R; r.ldc = nm;
        r.alpha = -1.0; r.beta = 1.0; r.batch = 1;
        CF_DEV(gemm_f64(r, s2));                                   // r = d - C x (FP64)
        CF_DEV(trsm_lower_f64(F, qb->R, nm, 0, qb->U, nm, 0, nm, 0, s2));
        CF_DEV(trsm_lower_t_f64(F, qb->U, nm, 0, qb->R, nm, 0, nm, s2));
        CF_DEV(launch_axpy(qb->X, qb->R, 1.0, n * nm, s2));        // x += C~^-1 r
      }
    } else {
      CF_DEV(trsm_lower_f64(F, qb->D, nm, 0, qb->U, nm, 0, nm, 0, s2));
    }
  }
  const bool split = H.has_t && H.has_p;
  const int64_t kT = H.has_t ? H.kf : 0, kP = k - kT;
  // Z through the mixed factor alone is off by 1e-6 (FP32) to 1e-4 (split-BF16x3) in F and more in
  // the noise bias: Z runs in FP64 and C^-1 Y gets one FP64 refinement step below
  const bool zref = mode != 0;
  const int zmode = zref ? 0 : mode;
  // Y is block diagonal over [T | QU]: the E,B columns vanish on the T rows, so their solve
  // starts at the 64-row block p0 holding the first Q row, and G's E,B columns above p0 are zero.
  const int64_t p0 = split ? (H.npx / kNB) * kNB : 0;
  CF_DEV(hipStreamWaitEvent(s, ev[E_Y], 0));
  if (split) {
    CF_DEV(hipStreamWaitEvent(s1, ev[E_L], 0));
    CF_DEV(trsm_lower_f64(F, f.Y + kT, k, 0, f.G + kT, k, 0, kP, H.npx, s1));
    CF_DEV(hipEventRecord(ev[E_EB], s1));
    CF_DEV(trsm_lower_f64(F, f.Y, k, 0, f.G, k, 0, kT, 0, s));
    CF_DEV(hipEventRecord(ev[E_T], s));
    tm.mark(ST_TRSM);
    // Z_TT = G_T^T G_T over all rows (s)
    GemmDesc g{};
    g.M = kT; g.N = kT; g.K = n;
    g.A = f.G; g.lda = k; g.at = 1;
    g.B = f.G; g.ldb = k; g.bt = 0;
    g.C = f.Z; g.ldc = k; g.alpha = 1.0; g.beta = 0.0; g.lower = 1; g.batch = 1; g.mode = zmode;
    CF_DEV(gemm_f64(g, s));
    // Z rows of E,B against all columns (lower part), over rows >= p0 (aux[0])
    CF_DEV(hipStreamWaitEvent(s1, ev[E_T], 0));
    GemmDesc h{};
    h.M = kP; h.N = k; h.K = n - p0;
    h.A = f.G + p0 * k + kT; h.lda = k; h.at = 1;
    h.B = f.G + p0 * k; h.ldb = k; h.bt = 0;
    h.C = f.Z + kT * k; h.ldc = k; h.alpha = 1.0; h.beta = 0.0; h.lower = 1; h.diag_off = kT;
    h.batch = 1; h.mode = zmode;
    hipEvent_t tz = tm.open(s1);
    CF_DEV(gemm_f64(h, s1));
    tm.close(ST_SYRK, tz, s1);
    CF_DEV(hipEventRecord(ev[E_S1], s1));
    if (qb && mode) {   // w = Y^T x with Y rebuilt (the solves consumed it)
      CF_DEV(hipStreamWaitEvent(s2, ev[E_T], 0));
      CF_DEV(hipStreamWaitEvent(s2, ev[E_EB], 0));
      CF_DEV(launch_ybuild(P, f.Y, k, s2));
      CF_DEV(weighted_maps(f.Y, k, k, n, qb->X, qb->nmaps, qb->W, qb->part, s2));
      CF_DEV(hipEventRecord(ev[E_S2], s2));
      CF_DEV(hipStreamWaitEvent(s, ev[E_S2], 0));
    } else if (qb) {   // w = G^T u
      CF_DEV(hipStreamWaitEvent(s2, ev[E_T], 0));
      CF_DEV(hipStreamWaitEvent(s2, ev[E_EB], 0));
      CF_DEV(weighted_maps(f.G, k, kT, n, qb->U, qb->nmaps, qb->W, qb->part, s2));
      CF_DEV(weighted_maps(f.G + p0 * k + kT, k, kP, n - p0, qb->U + p0 * qb->nmaps, qb->nmaps,
                           qb->W + kT * qb->nmaps, qb->part, s2));
      CF_DEV(hipEventRecord(ev[E_S2], s2));
      CF_DEV(hipStreamWaitEvent(s, ev[E_S2], 0));
    }
    CF_DEV(hipStreamWaitEvent(s, ev[E_S1], 0));
  } else {
    CF_DEV(trsm_lower_f64(F, f.Y, k, 0, f.G, k, 0, k, 0, s));
    CF_DEV(hipEventRecord(ev[E_T], s));
    tm.mark(ST_TRSM);
    GemmDesc g{};
    g.M = k; g.N = k; g.K = n;
    g.A = f.G; g.lda = k; g.at = 1;
    g.B = f.G; g.ldb = k; g.bt = 0;
    g.C = f.Z; g.ldc = k; g.alpha = 1.0; g.beta = 0.0; g.lower = 1; g.batch = 1; g.mode = zmode;
    hipEvent_t tz = tm.open(s);
    CF_DEV(gemm_f64(g, s));
    tm.close(ST_SYRK, tz, s);
    if (qb && mode) {
      CF_DEV(hipStreamWaitEvent(s2, ev[E_T], 0));
      CF_DEV(launch_ybuild(P, f.Y, k, s2));
      CF_DEV(weighted_maps(f.Y, k, k, n, qb->X, qb->nmaps, qb->W, qb->part, s2));
      CF_DEV(hipEventRecord(ev[E_S2], s2));
      CF_DEV(hipStreamWaitEvent(s, ev[E_S2], 0));
    } else if (qb) {
      CF_DEV(hipStreamWaitEvent(s2, ev[E_T], 0));
      CF_DEV(weighted_maps(f.G, k, k, n, qb->U, qb->nmaps, qb->W, qb->part, s2));
      CF_DEV(hipEventRecord(ev[E_S2], s2));
      CF_DEV(hipStreamWaitEvent(s, ev[E_S2], 0));
    }
  }
  if (zref) {
    // Z = Y^T C^-1 Y with one FP64 refinement of X = C^-1 Y through the mixed factor: X0 = L^-T G,
    // R = Y - C X0 (FP64 copy of C), W = L^-1 R, so Y^T (X0 + L^-T W) = G^T G + G^T W.  The E,B
    // columns of G above the first Q block were never written by the split solve: zero them.
    if (split && p0 > 0) CF_DEV(launch_fill_block(f.G + kT, k, p0, kP, 0.0, s));
    CF_DEV(hipMemcpyAsync(f.Gc, f.G, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s));
    CF_DEV(trsm_lower_t_f64(F, f.Gc, k, 0, f.Xr, k, 0, k, s));      // X0 (Gc consumed)
    CF_DEV(launch_ybuild(P, f.Y, k, s));
    GemmDesc r{};
    r.M = n; r.N = k; r.K = n;
    r.A = f.C0; r.lda = n; r.B = f.Xr; r.ldb = k; r.C = f.Y; r.ldc = k;
    r.alpha = -1.0; r.beta = 1.0; r.batch = 1;
    CF_DEV(gemm_f64(r, s));                                          // R = Y - C X0
    CF_DEV(trsm_lower_f64(F, f.Y, k, 0, f.Gc, k, 0, k, 0, s));      // W = L^-1 R (R consumed)
    GemmDesc dz{};
    dz.M = k; dz.N = k; dz.K = n;
    dz.A = f.G; dz.lda = k; dz.at = 1; dz.B = f.Gc; dz.ldb = k; dz.bt = 0;
    dz.C = f.Z; dz.ldc = k; dz.alpha = 1.0; dz.beta = 1.0; dz.lower = 1; dz.batch = 1;
    CF_DEV(gemm_f64(dz, s));                                         // Z += G^T W (lower)
  }
  tm.mark(ST_OTHER);
  CF_DEV(launch_symmetrize(f.Z, k, k, s));
  CF_DEV(launch_gram(P, f.Z, k, f.gram, f.ztr, s));
  tm.mark(ST_REDUCE);
  return CF_OK;
}

SpecSel make_sel(const HostBins& B, const FisherBufs& f) {
  SpecSel S;
  S.ns = B.ns;
  for (int i = 0; i < 6; ++i) S.spec[i] = B.spec[i];
  S.nb = B.nb;
  S.lo = f.lo;
  S.hi = f.hi;
  return S;
}

int check_factor_flags(CallCtx& c, const FisherBufs& f, cf_report* rep) {
  int fl[3];
  int st = read_flags(c, f.flags, 3, fl);
  if (st) return st;
  if (fl[0]) return fail(CF_EINVAL, "non-finite covariance entry (check noise and spectra)");
  if (fl[1] != INT_MAX) {
    if (rep) rep->fail_index = fl[1];
    return fail(CF_ENOTPD, "covariance not positive definite at pivot %d", fl[1]);
  }
  return CF_OK;
}

int copy_out(double* dst, const double* src, size_t count, int mem, hipStream_t s) {
  CF_DEV(hipMemcpyAsync(dst, src, count * sizeof(double),
                        mem == CF_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  return CF_OK;
}

double fisher_flops(const HostProblem& H) {
  const double n = H.n, kT = H.has_t ? H.kf : 0, k = (double)H.k;
  const double nP = H.has_p ? (H.has_t ? n - H.npx : n) : 0, kP = k - kT;
  double trsm = kT * n * n + kP * nP * nP;
  double syrk = (H.has_t && H.has_p) ? (kT * kT * n + 2 * kT * kP * nP + kP * kP * nP) : k * k * n;
  return n * n * n / 3.0 + trsm + syrk;
}

}  // namespace

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace cf

using namespace cf;

extern "C" {

const char* cf_last_error(void) { return g_err.c_str(); }
const char* cf_version(void) { return "libcf 0.2 (gfx950; FP64, FP32-MFMA and split-BF16 mixed paths)"; }

int64_t cf_problem_dim(const cf_problem* prob) {
  HostProblem H;
  if (check_problem(prob, H, false)) return -1;
  return H.n;
}

int64_t cf_problem_nmodes(const cf_problem* prob) {
  HostProblem H;
  if (check_problem(prob, H, false)) return -1;
  return H.k;
}

int cf_cov_build(const cf_problem* prob, double* C_out, int64_t* n_out, const cf_exec* ex,
                 cf_report* rep) {
  report_init(rep);
  HostProblem H;
  if (int st = check_problem(prob, H, true)) return st;
  if (!C_out) return fail(CF_EINVAL, "C_out is NULL");
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  Sizer z;
  size_staging(z, prob, H);
  z.add<double>((size_t)H.n * H.n);
  z.add<int>(8);
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  Staged S;
  if (int st = stage(bp, prob, H, nullptr, c.s, S)) return st;
  double* C = prob->mem == CF_MEM_DEVICE ? C_out : bp.take<double>((size_t)H.n * H.n);
  int* flags = bp.take<int>(8);
  Timer tm;
  tm.begin(ex && ex->stage_timing, c.s);
  CF_DEV(launch_fill_int(flags, 1, 0, c.s));
  // lower triangle, then mirrored, so that the returned matrix is exactly symmetric
  CF_DEV(launch_cov_build(S.P, S.cw, 0, 1, prob->noise_kind, S.noise, prob->noise_rank, S.noise_U, C,
                          H.n, 0, 1, flags, c.s));
  CF_DEV(launch_symmetrize(C, H.n, H.n, c.s));
  tm.mark(ST_BUILD);
  int fl[1];
  if (int st = read_flags(c, flags, 1, fl)) return st;
  if (fl[0]) return fail(CF_EINVAL, "non-finite covariance entry (check noise and spectra)");
  if (prob->mem == CF_MEM_HOST) {
    if (int st = copy_out(C_out, C, (size_t)H.n * H.n, CF_MEM_HOST, c.s)) return st;
  }
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  if (n_out) *n_out = H.n;
  if (rep) { rep->n = H.n; rep->nmodes = H.k; }
  return CF_OK;
}

int cf_fisher(const cf_problem* prob, const cf_bins* bins, int32_t precision, double* F_out,
              const cf_exec* ex, cf_report* rep) {
  report_init(rep);
  HostProblem H;
  if (int st = check_problem(prob, H, true)) return st;
  HostBins B;
  if (int st = check_bins(bins, H, B)) return st;
  if (precision < CF_FP64 || precision > CF_MIXED_BF16X3) return fail(CF_EINVAL, "unknown precision %d", precision);
  const int mode = precision;
  if (!F_out) return fail(CF_EINVAL, "F_out is NULL");
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  Sizer z;
  size_staging(z, prob, H);
  fisher_ws(H, B, z, mode, 0);
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  Staged S;
  if (int st = stage(bp, prob, H, nullptr, c.s, S)) return st;
  FisherBufs f;
  fisher_take(bp, H, B, f, mode, 0);
  CF_DEV(hipMemcpyAsync(f.lo, B.lo.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, c.s));
  CF_DEV(hipMemcpyAsync(f.hi, B.hi.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, c.s));
  Timer tm;
  tm.begin(ex && ex->stage_timing, c.s);
  if (int st = fisher_core(prob, H, S, f, nullptr, c, tm, mode)) return st;
  const SpecSel sel = make_sel(B, f);
  CF_DEV(launch_fisher_assemble(S.P, sel, f.gram, f.F, c.s));
  tm.mark(ST_REDUCE);
  if (int st = check_factor_flags(c, f, rep)) return st;
  const int K = B.ns * B.nb;
  if (int st = copy_out(F_out, f.F, (size_t)K * K, prob->mem, c.s)) return st;
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  if (rep) {
    rep->n = H.n; rep->nmodes = H.k; rep->flops = fisher_flops(H);
  }
  return CF_OK;
}

int cf_qml(const cf_problem* prob, const cf_bins* bins, const double* maps, int32_t nmaps,
           int32_t precision, double* y_out, double* bias_out, double* chat_out, double* F_out,
           const cf_exec* ex, cf_report* rep) {
  report_init(rep);
  HostProblem H;
  if (int st = check_problem(prob, H, true)) return st;
  HostBins B;
  if (int st = check_bins(bins, H, B)) return st;
  if (precision < CF_FP64 || precision > CF_MIXED_BF16X3) return fail(CF_EINVAL, "unknown precision %d", precision);
  const int mode = precision;
  const int refine = (ex && ex->refine_max >= 0) ? ex->refine_max : (mode == 2 ? 3 : 2);
  if (nmaps <= 0 || !maps) return fail(CF_EINVAL, "no maps");
  if (!y_out || !bias_out || !chat_out) return fail(CF_EINVAL, "y_out, bias_out and chat_out are required");
  if (prob->mem == CF_MEM_HOST && !finite_all(maps, (int64_t)nmaps * H.n))
    return fail(CF_EINVAL, "non-finite map value");
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  const int K = B.ns * B.nb;
  Sizer z;
  size_staging(z, prob, H);
  fisher_ws(H, B, z, mode, nmaps);
  z.add<double>((size_t)nmaps * H.n);        // maps copy (host inputs)
  z.add<double>((size_t)H.n * nmaps * 3);    // mixed: d, x, residual
  z.add<double>((size_t)H.n * nmaps);        // D = maps^T
  z.add<double>((size_t)H.n * nmaps);        // u = L^-1 D
  z.add<double>((size_t)H.k * nmaps);        // w = G^T u
  z.add<double>((size_t)32 * H.k * nmaps);   // partial sums of the skinny product
  z.add<double>((size_t)nmaps * K);          // y
  z.add<double>((size_t)K);                  // bias
  z.add<double>((size_t)nmaps * K);          // y - b
  z.add<double>((size_t)nmaps * K);          // chat
  z.add<double>((size_t)K * K);              // F copy for the solve
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  Staged S;
  if (int st = stage(bp, prob, H, nullptr, c.s, S)) return st;
  FisherBufs f;
  fisher_take(bp, H, B, f, mode, nmaps);
  double* mcopy = bp.take<double>((size_t)nmaps * H.n);
  double* mix = bp.take<double>((size_t)H.n * nmaps * 3);
  double* D = bp.take<double>((size_t)H.n * nmaps);
  double* U = bp.take<double>((size_t)H.n * nmaps);
  double* W = bp.take<double>((size_t)H.k * nmaps);
  double* part = bp.take<double>((size_t)32 * H.k * nmaps);
  double* y = bp.take<double>((size_t)nmaps * K);
  double* bias = bp.take<double>(K);
  double* q = bp.take<double>((size_t)nmaps * K);
  double* chat = bp.take<double>((size_t)nmaps * K);
  double* Fw = bp.take<double>((size_t)K * K);
  CF_DEV(hipMemcpyAsync(f.lo, B.lo.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, c.s));
  CF_DEV(hipMemcpyAsync(f.hi, B.hi.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, c.s));
  const double* mdev = maps;
  if (prob->mem == CF_MEM_HOST) {
    CF_DEV(hipMemcpyAsync(mcopy, maps, sizeof(double) * nmaps * H.n, hipMemcpyHostToDevice, c.s));
    mdev = mcopy;
  }
  Timer tm;
  tm.begin(ex && ex->stage_timing, c.s);
  QmlBufs qb;
  qb.maps = mdev; qb.nmaps = nmaps; qb.D = D; qb.U = U; qb.W = W; qb.part = part;
  qb.D0 = mix; qb.X = mix + (size_t)H.n * nmaps; qb.R = mix + (size_t)2 * H.n * nmaps;
  qb.refine = refine;
  if (int st = fisher_core(prob, H, S, f, &qb, c, tm, mode)) return st;
  const SpecSel sel = make_sel(B, f);
  CF_DEV(launch_fisher_assemble(S.P, sel, f.gram, f.F, c.s));
  CF_DEV(launch_bias_assemble(S.P, sel, f.gram, f.ztr, bias, c.s));
  tm.mark(ST_REDUCE);
  CF_DEV(launch_quad_assemble(S.P, sel, W, nmaps, nmaps, y, c.s));
  // chat = F^-1 (y - b)  (Eq. qml_estimate)
  CF_DEV(hipMemcpyAsync(q, y, sizeof(double) * nmaps * K, hipMemcpyDeviceToDevice, c.s));
  CF_DEV(launch_sub_bias(q, bias, K, nmaps, c.s));
  CF_DEV(hipMemcpyAsync(Fw, f.F, sizeof(double) * K * K, hipMemcpyDeviceToDevice, c.s));
  CF_DEV(launch_small_spd_solve(Fw, K, q, chat, nmaps, f.flags + 2, c.s));
  tm.mark(ST_QML);
  if (int st = check_factor_flags(c, f, rep)) return st;
  {
    int fl3[3];
    if (int st = read_flags(c, f.flags, 3, fl3)) return st;
    if (fl3[2] != INT_MAX) {
      if (rep) rep->fail_index = fl3[2];
      return fail(CF_ENOTPD, "Fisher matrix not positive definite at pivot %d", fl3[2]);
    }
  }
  if (int st = copy_out(y_out, y, (size_t)nmaps * K, prob->mem, c.s)) return st;
  if (int st = copy_out(bias_out, bias, (size_t)K, prob->mem, c.s)) return st;
  if (int st = copy_out(chat_out, chat, (size_t)nmaps * K, prob->mem, c.s)) return st;
  if (F_out)
    if (int st = copy_out(F_out, f.F, (size_t)K * K, prob->mem, c.s)) return st;
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  if (rep) { rep->n = H.n; rep->nmodes = H.k; rep->flops = fisher_flops(H); rep->ir_iters = mode ? refine : 0; }
  return CF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------- scan
namespace cf {
namespace {

// Captured batch of a scan: one hipGraph per (problem, batch shape, buffers), replayed for every
// full batch; the batch's first node advances the device-side point offset.
struct ScanGraph {
  std::string key;
  hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::vector<ScanGraph> g_graphs[64 * kLanes];   // per lane: the graphs write the lane's workspace

void release_device_state() {
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (int li = 0; li < 64 * kLanes; ++li) {
    const int id = li / kLanes;
    Device& d = g_dev[li];
    // a call still running on another thread at exit keeps its device's state (no deadlock)
    std::unique_lock<std::mutex> dl(d.mu, std::try_to_lock);
    if (!dl.owns_lock()) continue;
    {
      std::unique_lock<std::mutex> g(g_graph_mu, std::try_to_lock);
      if (!g.owns_lock()) continue;
      if (!g_graphs[li].empty() || d.stream) (void)hipSetDevice(id);
      for (auto& e : g_graphs[li]) (void)hipGraphExecDestroy(e.exec);
      g_graphs[li].clear();
    }
    if (!d.stream && !d.ws && !d.hflags) continue;
    (void)hipSetDevice(id);
    (void)hipDeviceSynchronize();
    for (hipStream_t* st : {&d.stream, &d.aux[0], &d.aux[1], &d.crit, &d.bulk, &d.bulk2})
      if (*st) { (void)hipStreamDestroy(*st); *st = nullptr; }
    for (auto& e : d.ev) if (e) { (void)hipEventDestroy(e); e = nullptr; }
    for (auto& e : d.ring) if (e) { (void)hipEventDestroy(e); e = nullptr; }
    for (hipEvent_t* e : {&d.jin, &d.jout}) if (*e) { (void)hipEventDestroy(*e); *e = nullptr; }
    if (d.ws) { (void)hipFree(d.ws); d.ws = nullptr; d.cap = 0; }
    if (d.hflags) { (void)hipHostFree(d.hflags); d.hflags = nullptr; }
  }
  if (cur >= 0) (void)hipSetDevice(cur);
}

// Autotuned launch shape of the scan per (device architecture, n, nmaps, mode): points per
// batch, outer panel width of the batched factorisation and GEMM tile of its updates, measured in
// the launch mode the call used (graph: 1 replayed, 0 eager); in memory and in a small text file,
// one line per shape: "scan <arch> n=.. nmaps=.. mode=.. batch=.. panel=.. tile=.. graph=..".
struct TuneEntry {
  std::string arch;
  int64_t n;
  int nmaps, mode, bt, panel, tile;
  int graph;                          // launch mode of the trials (-1: not recorded)
  int maxb = 16;                      // the largest batch the trials could try (the call's cap)
};
std::vector<TuneEntry> g_tune;
std::string g_tune_loaded;            // path the table was read from
std::mutex g_tune_mu;                 // calls on several lanes or devices share the table

std::string tune_path() {
  const char* p = getenv("CF_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.cf_autotune.txt";
}
void tune_load() {
  const std::string path = tune_path();
  if (g_tune_loaded == path) return;
  g_tune_loaded = path;
  g_tune.clear();
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    TuneEntry e{};
    char arch[64] = {0};
    long long n;
    const int got = sscanf(line, "scan %63s n=%lld nmaps=%d mode=%d batch=%d panel=%d tile=%d graph=%d max=%d",
                           arch, &n, &e.nmaps, &e.mode, &e.bt, &e.panel, &e.tile, &e.graph, &e.maxb);
    if (got < 5) continue;
    if (got < 7) e.panel = e.tile = 0;
    if (got < 8) e.graph = -1;
    if (got < 9) e.maxb = 16;           // entries from before larger batches were tried
    e.arch = arch;
    e.n = n;
    g_tune.push_back(e);
  }
  fclose(f);
}
bool tune_get(const char* arch, int64_t n, int nmaps, int mode, TuneEntry& out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load();
  // the latest entry of the shape: a call that could try larger batches tunes again and appends
  for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
    if (it->arch == arch && it->n == n && it->nmaps == nmaps && it->mode == mode) {
      out = *it;
      return true;
    }
  return false;
}
void tune_put(const TuneEntry& e) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load();
  g_tune.push_back(e);
  FILE* f = fopen(tune_path().c_str(), "a");
  if (!f) return;
  fprintf(f, "scan %s n=%lld nmaps=%d mode=%d batch=%d panel=%d tile=%d graph=%d max=%d\n", e.arch.c_str(),
          (long long)e.n, e.nmaps, e.mode, e.bt, e.panel, e.tile, e.graph, e.maxb);
  fclose(f);
}

struct ScanCtx {
  CallCtx* c;
  const cf_problem* prob;
  const HostProblem* h;
  const Staged* S;
  int p, nprob, nmaps, lstride, mode, refine;
  int panel = 0, tile = 0;            // launch shape of the batched factorisation (0: defaults)
  const double* cl_dev;
  double *cwb, *Cb, *C0b, *Linv, *Li256, *pscr, *ldp, *D, *Yb, *Gb, *Xb, *Rb, *x2, *ldb;
  double *Pz, *Pw, *T1, *T2;          // mixed: probe blocks and per-probe sums of the log-det correction
  int* flags;
  double *m2, *chi2, *ld;
  size_t layout;                      // workspace layout signature (bytes carved)
  bool one_stream = false;            // every launch on c->s, no library streams or events
};

// One batch of b points starting at i0 (or at *i0p when i0p is given).
int scan_batch(const ScanCtx& x, int64_t i0, int b, int64_t* i0p, Timer* tm) {
  CallCtx& c = *x.c;
  const HostProblem& h = *x.h;
  const int64_t n = h.n;
  const int Lp = h.lmax + 1, nmaps = x.nmaps;
  const int64_t nblk = (n + kNB - 1) / kNB;
  if (i0p) CF_DEV(launch_add_i64(i0p, b, c.s));
  // a2: per-point weights c^XY_l
  const double* clb = i0p ? x.cl_dev + (int64_t)x.p * 6 * x.lstride
                          : x.cl_dev + (i0 * x.nprob + x.p) * 6 * (int64_t)x.lstride;
  // points of a batch share each pixel pair's recurrences in groups of kCovIB
  const int inter = b > 1 ? kCovIB : 1;
  CF_DEV(launch_tables(clb, x.S->bl, x.S->pl, h.lmin, h.lmax, b, (int64_t)x.nprob * 6 * x.lstride,
                       x.lstride, x.cwb, nullptr, nullptr, nullptr, c.s, i0p, inter));
  // a3: covariance of every point of the batch.  FP64: slot = [C; d^T] (n + nmaps rows), so that
  // the factorisation also yields u^T = (L^-1 d)^T; mixed: slot = C (solved and refined apart).
  const int64_t slot = x.mode ? n * n : (n + nmaps) * n;
  CF_DEV(launch_cov_build(x.S->P, x.cwb, 6 * (int64_t)Lp * inter, b, x.prob->noise_kind, x.S->noise,
                          x.prob->noise_rank, x.S->noise_U, x.Cb, n, slot, x.mode ? 0 : 1, x.flags, c.s,
                          inter));
  if (x.mode)
    CF_DEV(hipMemcpyAsync(x.C0b, x.Cb, sizeof(double) * b * n * n, hipMemcpyDeviceToDevice, c.s));
  else
    for (int j = 0; j < b; ++j)
      CF_DEV(hipMemcpyAsync(x.Cb + j * slot + n * n, x.D, sizeof(double) * n * nmaps, hipMemcpyDeviceToDevice, c.s));
  if (tm) tm->mark(ST_BUILD);
  // a4: Cholesky and log det
  Factor F;
  F.L = x.Cb; F.n = n; F.ld = n; F.sL = slot;
  F.Li64 = x.Linv; F.sLi64 = nblk * kNB * kNB;
  F.Li256 = (n >= 256 && x.mode) ? x.Li256 : nullptr; F.sLi256 = (n / 256) * 256 * 256;
  F.ldpart = x.ldp; F.sPart = nblk;
  F.fail = x.flags + 1; F.batch = b; F.mode = x.mode;
  F.panel = x.panel; F.tile = x.tile;
  if (!x.mode) F.rows = n + nmaps;
  if (x.one_stream) {
    Streams st{c.s, c.s, c.s, nullptr, nullptr, nullptr, nullptr};
    CF_DEV(potrf_f64(F, x.pscr, st));
  } else if (int st = potrf_on(*c.dev, F, x.pscr, c.s, c.dev->aux[1], c.dev->ev + 8)) {
    return st;
  }
  if (tm) tm->mark(ST_POTRF);
  if (!x.mode) {   // chi^2_j = |u_j|^2 from the rows below C
    CF_DEV(launch_rowsumsq(x.Cb + n * n, nmaps, n, n, slot, b, x.x2, nmaps, c.s));
    CF_DEV(launch_sum_parts(x.ldp, (int)nblk, nblk, b, x.ldb, 1, c.s));
    CF_DEV(launch_scan_finish(x.x2, x.ldb, b, nmaps, i0, x.p, x.nprob, x.m2, x.chi2, x.ld, c.s, i0p));
    if (tm) tm->mark(ST_TRSM);
    return CF_OK;
  }
  // a6: u = L^-1 d for every map, chi^2 = |u|^2 (FP64); mixed: refined x = C^-1 d, chi^2 = d^T x
  for (int j = 0; j < b; ++j)
    CF_DEV(hipMemcpyAsync(x.Yb + (size_t)j * n * nmaps, x.D, sizeof(double) * n * nmaps,
                          hipMemcpyDeviceToDevice, c.s));
  CF_DEV(trsm_lower_f64(F, x.Yb, nmaps, n * nmaps, x.Gb, nmaps, n * nmaps, nmaps, 0, c.s));
  if (!x.mode) {
    CF_DEV(launch_colsumsq(x.Gb, n, nmaps, nmaps, n * nmaps, b, x.x2, nmaps, c.s));
  } else {
    CF_DEV(trsm_lower_t_f64(F, x.Gb, nmaps, n * nmaps, x.Xb, nmaps, n * nmaps, nmaps, c.s));
    for (int it = 0; it < x.refine; ++it) {
      for (int j = 0; j < b; ++j)
        CF_DEV(hipMemcpyAsync(x.Rb + (size_t)j * n * nmaps, x.D, sizeof(double) * n * nmaps,
                              hipMemcpyDeviceToDevice, c.s));
      GemmDesc r{};
      r.M = n; r.N = nmaps; r.K = n;
      r.A = x.C0b; r.lda = n; r.B = x.Xb; r.ldb = nmaps; r.C = x.Rb; r.ldc = nmaps;
      r.alpha = -1.0; r.beta = 1.0; r.batch = b; r.sA = n * n; r.sB = n * nmaps; r.sC = n * nmaps;
      CF_DEV(gemm_f64(r, c.s));
      CF_DEV(trsm_lower_f64(F, x.Rb, nmaps, n * nmaps, x.Gb, nmaps, n * nmaps, nmaps, 0, c.s));
      CF_DEV(trsm_lower_t_f64(F, x.Gb, nmaps, n * nmaps, x.Rb, nmaps, n * nmaps, nmaps, c.s));
      CF_DEV(launch_axpy(x.Xb, x.Rb, 1.0, (int64_t)b * n * nmaps, c.s));
    }
    CF_DEV(launch_coldot(x.D, x.Xb, n, nmaps, nmaps, 0, n * nmaps, b, x.x2, nmaps, c.s));
  }
  CF_DEV(launch_sum_parts(x.ldp, (int)nblk, nblk, b, x.ldb, 1, c.s));
  if (x.mode) {
    // ln|C| = ln|L L^T| + tr X - |X|_F^2 / 2 + O(|X|^3), X = L^-1 E L^-T, E = C - L L^T the
    // mixed factor's error.  With y = L^-T z and v = C y for a probe z of +-1 entries, z^T X z =
    // y^T v - z^T z and X z = L^-1 v - z, so each probe costs two triangular solves and one
    // product with the FP64 copy of C, and E is never formed.
    // The two solves run in FP64 against the mixed factor (its inverted diagonal blocks are FP64):
    // y^T v - z^T z cancels to about |X|, so y must be accurate far beyond FP32.
    const int64_t m = kLdProbes;
    Factor F64 = F;
    F64.mode = 0;
    CF_DEV(launch_probes(x.Pz, n, m, b, 0, c.s));
    CF_DEV(trsm_lower_t_f64(F64, x.Pz, m, n * m, x.Pw, m, n * m, m, c.s));    // Pw = y (Pz consumed)
    GemmDesc v{};
    v.M = n; v.N = m; v.K = n;
    v.A = x.C0b; v.lda = n; v.B = x.Pw; v.ldb = m; v.C = x.Pz; v.ldc = m;
    v.alpha = 1.0; v.beta = 0.0; v.batch = b; v.sA = n * n; v.sB = n * m; v.sC = n * m;
    CF_DEV(gemm_f64(v, c.s));                                                  // Pz = v = C y
    CF_DEV(launch_coldot(x.Pw, x.Pz, n, m, m, n * m, n * m, b, x.T1, m, c.s));  // y^T v
    CF_DEV(trsm_lower_f64(F64, x.Pz, m, n * m, x.Pw, m, n * m, m, 0, c.s));   // Pw = L^-1 v
    CF_DEV(launch_probes(x.Pw, n, m, b, 1, c.s));                             // X z
    CF_DEV(launch_colsumsq(x.Pw, n, m, m, n * m, b, x.T2, m, c.s));
    CF_DEV(launch_ld_correct(x.ldb, x.T1, x.T2, b, m, n, c.s));
  }
  CF_DEV(launch_scan_finish(x.x2, x.ldb, b, nmaps, i0, x.p, x.nprob, x.m2, x.chi2, x.ld, c.s, i0p));
  if (tm) tm->mark(ST_TRSM);
  return CF_OK;
}

// Everything a captured batch bakes into its kernel arguments: shapes, the problem's values passed
// by value (multipole range, fields, pixel count, noise kind and rank) and every buffer address.
std::string graph_key(const ScanCtx& x, int b, const char* ws) {
  char buf[640];
  const HostProblem& h = *x.h;
  snprintf(buf, sizeof buf,
           "%d|%lld|%d|%d|%d|%d|%d|%d|%d|%d|%zu|l%d-%d|f%d%d|px%d|nk%d|nr%d|%p|%p|%p|%p|%p|%p|%p|%p|%p", x.p,
           (long long)h.n, b, x.nmaps, x.mode, x.refine, x.lstride, x.nprob, x.panel, x.tile, x.layout,
           h.lmin, h.lmax, h.has_t, h.has_p, h.npx, x.prob->noise_kind, x.prob->noise_rank,
           (const void*)ws,
           (const void*)x.cl_dev, (const void*)x.D, (const void*)x.m2, (const void*)x.chi2,
           (const void*)x.ld, (const void*)x.S->noise, (const void*)x.S->noise_U, (const void*)x.c->s);
  return buf;
}

// Runs points [i0, i0 + nb*b) of problem x.p as nb replays of the captured batch.
int scan_replay(ScanCtx& x, int64_t i0, int b, int64_t nb, int64_t* i0p) {
  CallCtx& c = *x.c;
  const int dev = (int)(c.dev - g_dev);          // the call's lane
  const std::string key = graph_key(x, b, c.dev->ws);
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> g(g_graph_mu);
    for (auto& e : g_graphs[dev])
      if (e.key == key) exec = e.exec;
  }
  if (!exec) {
    hipGraph_t graph = nullptr;
    CF_DEV(hipStreamBeginCapture(c.s, hipStreamCaptureModeRelaxed));
    int st = scan_batch(x, 0, b, i0p, nullptr);
    hipError_t e2 = hipStreamEndCapture(c.s, &graph);
    if (st) return st;
    if (e2 != hipSuccess) return fail(CF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    CF_DEV(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    CF_DEV(hipGraphDestroy(graph));
    std::lock_guard<std::mutex> g(g_graph_mu);
    if (g_graphs[dev].size() >= 16) {
      // the evicted graph may still have replays queued (on any stream): let them finish first
      CF_DEV(hipDeviceSynchronize());
      (void)hipGraphExecDestroy(g_graphs[dev].front().exec);
      g_graphs[dev].erase(g_graphs[dev].begin());
    }
    g_graphs[dev].push_back({key, exec});
  }
  if (nb > 0) {
    CF_DEV(launch_set_i64(i0p, i0 - b, c.s));
    for (int64_t k = 0; k < nb; ++k) CF_DEV(hipGraphLaunch(exec, c.s));
  }
  return CF_OK;
}

}  // namespace
}  // namespace cf

namespace cf {
namespace {

// The scan of cf_loglike_batch.  noalloc: the workspace is the library's static device array
// (no allocation of any kind), every launch goes eagerly onto the caller's stream (no library
// streams, events or graphs, no autotuning), and the batch is the largest that fits that array.
int loglike_core(const cf_problem* probs, int32_t nprob, int32_t npoints, const double* cl_points,
                 int32_t lstride, const double* const* maps, int32_t nmaps, int32_t precision,
                 double* m2lnL, double* chi2, double* logdet, const cf_exec* ex, cf_report* rep,
                 bool noalloc) {
  report_init(rep);
  if (!probs || nprob <= 0) return fail(CF_EINVAL, "no problems");
  if (npoints <= 0 || !cl_points) return fail(CF_EINVAL, "no scan points");
  if (nmaps <= 0 || !maps) return fail(CF_EINVAL, "no maps");
  if (!m2lnL) return fail(CF_EINVAL, "m2lnL is NULL");
  if (precision < CF_FP64 || precision > CF_MIXED_BF16X3) return fail(CF_EINVAL, "unknown precision %d", precision);
  const int mode = precision;
  const int refine = (ex && ex->refine_max >= 0) ? ex->refine_max : (mode == 2 ? 3 : 2);
  const int mem = probs[0].mem;
  std::vector<HostProblem> H(nprob);
  int lmax_all = 0;
  for (int p = 0; p < nprob; ++p) {
    if (int st = check_problem(&probs[p], H[p], false)) return st;
    if (probs[p].mem != mem) return fail(CF_EINVAL, "problems disagree on mem");
    if (!maps[p]) return fail(CF_EINVAL, "maps[%d] is NULL", p);
    if (H[p].lmax > lmax_all) lmax_all = H[p].lmax;
  }
  if (lstride < lmax_all + 1) return fail(CF_EINVAL, "lstride %d < lmax+1 = %d", lstride, lmax_all + 1);
  // Captured batches are replayed only in calls whose problems all have n <= kGraphMaxN; any other
  // call launches every batch eagerly.
  int nmax_all = 0;
  for (int p = 0; p < nprob; ++p) nmax_all = std::max(nmax_all, H[p].n);
  const bool use_graph = !noalloc && !(ex && ex->no_graph) && !(ex && ex->stage_timing) && nmax_all <= kGraphMaxN;
  const size_t ncl = (size_t)npoints * nprob * 6 * lstride;
  if (mem == CF_MEM_HOST) {
    if (!finite_all(cl_points, (int64_t)ncl)) return fail(CF_EINVAL, "non-finite scan spectra");
    for (int p = 0; p < nprob; ++p)
      if (!finite_all(maps[p], (int64_t)nmaps * H[p].n)) return fail(CF_EINVAL, "non-finite map value");
  }
  CallCtx c;
  if (int st = noalloc ? c.begin_plain(ex) : c.begin(ex)) return st;
  int nmax = 0;
  for (int p = 0; p < nprob; ++p) nmax = H[p].n > nmax ? H[p].n : nmax;
  // Points factorised together, per problem: the autotuned batch of the problem's shape if known,
  // else the largest of at most 128 whose covariances fit the budget (kScanBytes, or an eighth of
  // the device's memory if less).  The workspace holds, for every buffer, the largest of the
  // problems' batches of it.
  const size_t budget = (c.dev->mem > 0 && c.dev->mem / 8 < kScanBytes) ? c.dev->mem / 8 : kScanBytes;
  std::vector<int> cap(nprob);
  for (int p = 0; p < nprob; ++p) {
    const size_t per = (size_t)H[p].n * H[p].n * 8 * (mode ? 2 : 1);
    cap[p] = (int)std::min<size_t>(kScanBatchMax, std::max<size_t>(1, budget / per));
    cap[p] = (int)std::min<int64_t>(cap[p], npoints);
  }
  std::vector<TuneEntry> te(nprob);
  std::vector<char> tuned(nprob, 0);
  if (!noalloc)
    for (int p = 0; p < nprob; ++p)
      if (tune_get(c.dev->arch, H[p].n, nmaps, mode, te[p])) {
        // tuned by a call with fewer points than this one can batch: tune again if asked to
        tuned[p] = !(ex && ex->autotune && cap[p] > te[p].maxb);
      }
  const int L = lmax_all + 1;
  // workspace bytes for batches of up to bw[p] points of problem p
  auto ws_bytes = [&](const std::vector<int>& bw) -> size_t {
    Sizer z;
    for (int p = 0; p < nprob; ++p) size_staging(z, &probs[p], H[p]);
    if (mem == CF_MEM_HOST) {
      z.add<double>(ncl);
      for (int p = 0; p < nprob; ++p) z.add<double>((size_t)nmaps * H[p].n);
      z.add<double>((size_t)npoints * nprob * nmaps * 2 + (size_t)npoints * nprob);
    }
    auto mx = [&](auto per_point) {
      size_t m = 1;
      for (int p = 0; p < nprob; ++p) m = std::max(m, (size_t)bw[p] * (size_t)per_point((size_t)H[p].n));
      return m;
    };
    int bmax = 1;
    for (int p = 0; p < nprob; ++p) bmax = std::max(bmax, bw[p]);
    z.add<double>((size_t)(bmax + kCovIB - 1) / kCovIB * kCovIB * 6 * L);   // whole chunks
    z.add<double>(mx([&](size_t n) { return (n + (mode ? 0 : nmaps)) * n; }));
    z.add<double>(mx([&](size_t n) { return (n + kNB - 1) / kNB * kNB * kNB; }));
    z.add<double>(mx([&](size_t n) { return (n / 256) * 256 * 256; }));
    z.add<double>((size_t)potrf_scratch(bmax));
    z.add<double>(mx([&](size_t n) { return (n + kNB - 1) / kNB; }));
    z.add<double>((size_t)nmax * nmaps);
    z.add<double>(mx([&](size_t n) { return n * nmaps; }));
    z.add<double>(mx([&](size_t n) { return n * nmaps; }));
    z.add<double>(mode ? mx([&](size_t n) { return n * n; }) : 1);
    z.add<double>(mode ? mx([&](size_t n) { return n * nmaps; }) : 1);
    z.add<double>(mode ? mx([&](size_t n) { return n * nmaps; }) : 1);
    z.add<double>(mode ? mx([&](size_t n) { return n * kLdProbes; }) : 1);
    z.add<double>(mode ? mx([&](size_t n) { return n * kLdProbes; }) : 1);
    z.add<double>(mode ? (size_t)bmax * kLdProbes : 1);
    z.add<double>(mode ? (size_t)bmax * kLdProbes : 1);
    z.add<double>((size_t)bmax * nmaps);
    z.add<double>((size_t)bmax);
    z.add<int64_t>(1);
    z.add<int>(8);
    return z.off;
  };
  std::vector<int> bw = cap;   // the workspace fits the largest batch the tuner may pick
  char* wsbase = nullptr;
  if (noalloc) {
    int B = 16;
    auto clip = [&](int lim) {
      for (int p = 0; p < nprob; ++p) bw[p] = std::min(cap[p], lim);
    };
    clip(B);
    while (B > 1 && ws_bytes(bw) > kScratchBytes) clip(--B);
    const size_t need = ws_bytes(bw);
    if (need > kScratchBytes)
      return fail(CF_EINVAL, "cf_loglike_batch_noalloc: %zu bytes of workspace needed for one point, above the "
                  "%zu-byte static scratch array", need, kScratchBytes);
    cap = bw;
    wsbase = g_scratch[c.id];
  } else {
    if (int st = ensure_ws(*c.dev, ws_bytes(bw))) return st;
    wsbase = c.dev->ws;
  }
  size_t szC = 1, szLi = 1, szL256 = 1, szP = 1, szY = 1, szC0 = 1, szPz = 1;
  int bmax = 1;
  for (int p = 0; p < nprob; ++p) {
    const size_t n = H[p].n, w = bw[p];
    szC = std::max(szC, w * (n + (mode ? 0 : nmaps)) * n);
    szLi = std::max(szLi, w * ((n + kNB - 1) / kNB) * kNB * kNB);
    szL256 = std::max(szL256, w * (n / 256) * 256 * 256);
    szP = std::max(szP, w * ((n + kNB - 1) / kNB));
    szY = std::max(szY, w * n * nmaps);
    szC0 = std::max(szC0, w * n * n);
    szPz = std::max(szPz, w * n * kLdProbes);
    bmax = std::max(bmax, bw[p]);
  }
  const size_t ncw = (size_t)(bmax + kCovIB - 1) / kCovIB * kCovIB * 6 * L;   // whole chunks
  Bump bp(wsbase);
  std::vector<Staged> S(nprob);
  for (int p = 0; p < nprob; ++p)
    if (int st = stage(bp, &probs[p], H[p], nullptr, c.s, S[p])) return st;
  const double* cl_dev = cl_points;
  std::vector<const double*> map_dev(maps, maps + nprob);
  double *m2_dev = m2lnL, *chi2_dev = chi2, *ld_dev = logdet;
  if (mem == CF_MEM_HOST) {
    double* t = bp.take<double>(ncl);
    CF_DEV(hipMemcpyAsync(t, cl_points, sizeof(double) * ncl, hipMemcpyHostToDevice, c.s));
    cl_dev = t;
    for (int p = 0; p < nprob; ++p) {
      double* m = bp.take<double>((size_t)nmaps * H[p].n);
      CF_DEV(hipMemcpyAsync(m, maps[p], sizeof(double) * nmaps * H[p].n, hipMemcpyHostToDevice, c.s));
      map_dev[p] = m;
    }
    double* o = bp.take<double>((size_t)npoints * nprob * nmaps * 2 + (size_t)npoints * nprob);
    m2_dev = o;
    chi2_dev = chi2 ? o + (size_t)npoints * nprob * nmaps : nullptr;
    ld_dev = logdet ? o + (size_t)npoints * nprob * nmaps * 2 : nullptr;
  }
  ScanCtx x;
  x.c = &c; x.nprob = nprob; x.nmaps = nmaps; x.lstride = lstride; x.mode = mode; x.refine = refine;
  x.cl_dev = cl_dev;
  x.cwb = bp.take<double>(ncw);
  x.Cb = bp.take<double>(szC);
  x.Linv = bp.take<double>(szLi);
  x.Li256 = bp.take<double>(szL256);
  x.pscr = bp.take<double>((size_t)potrf_scratch(bmax));
  x.ldp = bp.take<double>(szP);
  x.D = bp.take<double>((size_t)nmax * nmaps);
  x.Yb = bp.take<double>(szY);
  x.Gb = bp.take<double>(szY);
  x.C0b = bp.take<double>(mode ? szC0 : 1);
  x.Xb = bp.take<double>(mode ? szY : 1);
  x.Rb = bp.take<double>(mode ? szY : 1);
  x.Pz = bp.take<double>(mode ? szPz : 1);
  x.Pw = bp.take<double>(mode ? szPz : 1);
  x.T1 = bp.take<double>(mode ? (size_t)bmax * kLdProbes : 1);
  x.T2 = bp.take<double>(mode ? (size_t)bmax * kLdProbes : 1);
  x.x2 = bp.take<double>((size_t)bmax * nmaps);
  x.ldb = bp.take<double>((size_t)bmax);
  int64_t* i0p = bp.take<int64_t>(1);
  x.flags = bp.take<int>(8);
  x.m2 = m2_dev; x.chi2 = chi2_dev; x.ld = ld_dev;
  x.layout = bp.off;
  x.one_stream = noalloc;
  CF_DEV(launch_fill_int(x.flags, 1, 0, c.s));
  CF_DEV(launch_fill_int(x.flags + 1, 1, INT_MAX, c.s));
  Timer tm;
  tm.begin(ex && ex->stage_timing && !noalloc, c.s);
  double flops = 0.0;
  int bt_used = 0;
  for (int p = 0; p < nprob; ++p) {
    const HostProblem& h = H[p];
    x.p = p; x.prob = &probs[p]; x.h = &h; x.S = &S[p];
    if (mode)   // mixed: D = maps^T (n x nmaps) for the separate solves; FP64: maps as rows
      CF_DEV(launch_transpose(map_dev[p], nmaps, h.n, h.n, x.D, nmaps, c.s));
    else
      CF_DEV(hipMemcpyAsync(x.D, map_dev[p], sizeof(double) * nmaps * h.n, hipMemcpyDeviceToDevice, c.s));
    int b = cap[p];
    const bool graph = use_graph;
    x.panel = x.tile = 0;
    if (tuned[p]) {
      if (te[p].bt > 0) b = std::min(te[p].bt, cap[p]);
      x.panel = te[p].panel;
      x.tile = te[p].tile;
    }
    int64_t i0 = 0;
    // Autotuning on the first call of a problem's shape: time one batch per candidate, in two
    // rounds (points per batch; then outer panel width and GEMM tile together), keeping the best
    // rate.  Trials run the first points of the scan (best of two timings each) in the call's
    // launch mode (replayed graphs or eager launches); the scan itself then runs in full with the
    // chosen shape, so every output comes from one configuration.
    if (ex && ex->autotune && !tuned[p] && npoints >= 2 && !noalloc) {
      double best_rate = 0.0;
      TuneEntry best{c.dev->arch, h.n, nmaps, mode, b, 0, 0, graph ? 1 : 0, cap[p]};
      const bool verbose = getenv("CF_TUNE_VERBOSE") != nullptr;
      auto trial = [&](int cand, int panel, int tile, bool g) -> int {
        if (cand > cap[p]) return CF_OK;
        x.panel = panel;
        x.tile = tile;
        if (g) { if (int st = scan_replay(x, 0, cand, 0, i0p)) return st; }   // capture first
        hipEvent_t e0, e1;
        CF_DEV(hipEventCreate(&e0));
        CF_DEV(hipEventCreate(&e1));
        float best_ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          CF_DEV(hipEventRecord(e0, c.s));
          if (g) { if (int st = scan_replay(x, 0, cand, 1, i0p)) return st; }
          else if (int st = scan_batch(x, 0, cand, nullptr, nullptr)) return st;
          CF_DEV(hipEventRecord(e1, c.s));
          CF_DEV(hipEventSynchronize(e1));
          float ms = 0.f;
          CF_DEV(hipEventElapsedTime(&ms, e0, e1));
          if (rep == 0 || ms < best_ms) best_ms = ms;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        const double rate = cand / (double)best_ms;
        if (verbose)
          fprintf(stderr, "cf autotune %s n=%d nmaps=%d mode=%d batch=%d panel=%d tile=%d graph=%d: %.3f ms per point\n",
                  c.dev->arch, h.n, nmaps, mode, cand, panel, tile, g ? 1 : 0, best_ms / cand);
        if (rate > best_rate) { best_rate = rate; best.bt = cand; best.panel = panel; best.tile = tile; }
        return CF_OK;
      };
      // small problems are bound by the chain of diagonal blocks, which a larger batch shares
      // among more points (n = 1088: 14k points/s at 16 per batch)
      for (int cand : {2, 4, 8, 16, 32, 64, 128})
        if (int st = trial(cand, 0, 0, graph)) return st;
      // and the largest batch the call allows when it is not one of those (memory or points)
      if (cap[p] > 2 && (cap[p] & (cap[p] - 1)) != 0)
        if (int st = trial(cap[p], 0, 0, graph)) return st;
      const int bt = best.bt;
      for (int panel : {0, 256, 512}) {       // panel width and tile jointly (they interact)
        if (panel && h.n <= 512) continue;
        for (int tile : {64, 128})
          if (int st = trial(bt, panel, tile, graph)) return st;
      }
      tune_put(best);
      b = best.bt;
      x.panel = best.panel;
      x.tile = best.tile;
    }
    bt_used = std::max(bt_used, b);
    const int64_t nfull = (npoints - i0) / b;
    if (graph && nfull >= 1) {
      if (int st = scan_replay(x, i0, b, nfull, i0p)) return st;
      i0 += nfull * b;
    }
    for (; i0 < npoints; i0 += b) {
      const int bb = (int)std::min<int64_t>(b, npoints - i0);
      if (int st = scan_batch(x, i0, bb, nullptr, &tm)) return st;
    }
    const double nd = (double)h.n;
    flops += (double)npoints * (nd * nd * nd / 3.0 + nd * nd * nmaps);
  }
  int fl[2];
  if (int st = noalloc ? read_flags_plain(c, x.flags, 2, fl) : read_flags(c, x.flags, 2, fl)) return st;
  if (fl[0]) return fail(CF_EINVAL, "non-finite covariance entry (check noise and scan spectra)");
  if (fl[1] != INT_MAX) {
    if (rep) rep->fail_index = fl[1];
    return fail(CF_ENOTPD, "a scan covariance is not positive definite (pivot %d)", fl[1]);
  }
  if (mem == CF_MEM_HOST) {
    const size_t no = (size_t)npoints * nprob * nmaps;
    if (int st = copy_out(m2lnL, m2_dev, no, CF_MEM_HOST, c.s)) return st;
    if (chi2) if (int st = copy_out(chi2, chi2_dev, no, CF_MEM_HOST, c.s)) return st;
    if (logdet) if (int st = copy_out(logdet, ld_dev, (size_t)npoints * nprob, CF_MEM_HOST, c.s)) return st;
  }
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  if (rep) { rep->flops = flops; rep->n = H[0].n; rep->ir_iters = mode ? refine : 0; rep->n_fallback = bt_used; }
  return CF_OK;
}

}  // namespace
}  // namespace cf

extern "C" int cf_loglike_batch(const cf_problem* probs, int32_t nprob, int32_t npoints,
                                const double* cl_points, int32_t lstride, const double* const* maps,
                                int32_t nmaps, int32_t precision, double* m2lnL, double* chi2,
                                double* logdet, const cf_exec* ex, cf_report* rep) {
  return cf::loglike_core(probs, nprob, npoints, cl_points, lstride, maps, nmaps, precision, m2lnL, chi2,
                          logdet, ex, rep, false);
}

extern "C" int cf_loglike_batch_noalloc(const cf_problem* probs, int32_t nprob, int32_t npoints,
                                        const double* cl_points, int32_t lstride, const double* const* maps,
                                        int32_t nmaps, int32_t precision, double* m2lnL, double* chi2,
                                        double* logdet, const cf_exec* ex, cf_report* rep) {
  return cf::loglike_core(probs, nprob, npoints, cl_points, lstride, maps, nmaps, precision, m2lnL, chi2,
                          logdet, ex, rep, true);
}

// ------------------------------------------------------------------------------- SMW likelihood
// Handle of the harmonic-basis likelihood: what every point needs, kept on the device it was
// made on.  M = V_win N_eff^-1 V_win^T [kw][kw] (full), b = V_win N_eff^-1 D [kw][nmaps],
// chi2N[j] = d_j^T N_eff^-1 d_j, ldN = ln|N_eff|, wl = W_l.
struct cf_smw {
  int device = -1;
  int mem = 0;
  int n = 0, lmax = 0, wlo = 0, whi = 0, nf = 0, nmaps = 0;
  int fld[3] = {0, 0, 0};          // harmonic field (T 0, E 1, B 2) of each window slot
  int64_t kwf = 0, kw = 0;
  // 2: the window holds T and E and/or B and M = V N_eff^-1 V^T has no T x (E,B) block (N_eff
  // couples no T pixel with a Q, U pixel), so K' splits into a T block and an E,B block for every
  // point whose window spectra have no TE, TB; 1: one dense K'.
  int blocks = 1;
  double *M = nullptr, *b = nullptr, *chi2N = nullptr, *ldN = nullptr, *wl = nullptr;
};

namespace cf {
namespace {

int spec_row(int a, int b) {   // spectrum row (TT, EE, BB, TE, TB, EB) of a harmonic-field pair
  if (a > b) std::swap(a, b);
  if (a == b) return a;
  if (a == 0) return b == 1 ? 3 : 4;
  return 5;
}

void smw_free(cf_smw* h) {
  if (!h) return;
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  const bool sw = have && h->device >= 0 && cur != h->device;
  if (sw) (void)hipSetDevice(h->device);
  (void)hipFree(h->M);
  (void)hipFree(h->b);
  (void)hipFree(h->chi2N);
  (void)hipFree(h->ldN);
  (void)hipFree(h->wl);
  if (sw) (void)hipSetDevice(cur);
  delete h;
}

// N_eff (Eq. N_eff: the problem's spectra without the window's varied entries) factored with
// the maps and the window's harmonic rows below it, so that the rows come out as
// (L^-1 D)^T and (L^-1 V_win^T)^T; then M, b, chi2N and ln|N_eff| from those rows.
int smw_setup(const cf_problem* prob, const HostProblem& H, cf_smw* h, const int* pslot,
              const std::vector<double>& clf, const double* maps, CallCtx& c, Timer& tm) {
  const int64_t n = H.n, k = H.k, kw = h->kw, kwf = h->kwf;
  const int nm = h->nmaps, L = H.lmax + 1;
  const int64_t rows = n + nm + kw, nblk = (n + kNB - 1) / kNB;
  Sizer z;
  size_staging(z, prob, H);
  z.add<double>((size_t)rows * n);
  z.add<double>((size_t)n * k);
  z.add<double>((size_t)nblk * kNB * kNB);
  z.add<double>((size_t)potrf_scratch(1));
  z.add<double>((size_t)nblk);
  z.add<double>((size_t)nm * n);
  z.add<int>(8);
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  Staged S;
  if (int st = stage(bp, prob, H, clf.data(), c.s, S)) return st;
  double* C = bp.take<double>((size_t)rows * n);
  double* Y = bp.take<double>((size_t)n * k);
  double* Linv = bp.take<double>((size_t)nblk * kNB * kNB);
  double* scr = bp.take<double>((size_t)potrf_scratch(1));
  double* ldp = bp.take<double>((size_t)nblk);
  double* mcopy = bp.take<double>((size_t)nm * n);
  int* flags = bp.take<int>(8);
  const double* mdev = maps;
  if (prob->mem == CF_MEM_HOST) {
    CF_DEV(hipMemcpyAsync(mcopy, maps, sizeof(double) * nm * n, hipMemcpyHostToDevice, c.s));
    mdev = mcopy;
  }
  CF_DEV(launch_fill_int(flags, 1, 0, c.s));
  CF_DEV(launch_fill_int(flags + 1, 1, INT_MAX, c.s));
  CF_DEV(launch_ybuild(S.P, Y, k, c.s));
  tm.mark(ST_YBUILD);
  CF_DEV(launch_cov_build(S.P, S.cw, 0, 1, prob->noise_kind, S.noise, prob->noise_rank, S.noise_U, C, n, 0, 1,
                          flags, c.s));
  CF_DEV(hipMemcpyAsync(C + n * n, mdev, sizeof(double) * nm * n, hipMemcpyDeviceToDevice, c.s));
  double* Vt = C + (n + nm) * n;
  const int64_t c0 = (int64_t)h->wlo * h->wlo - (int64_t)H.lmin * H.lmin;   // window's first column in a field
  for (int q = 0; q < h->nf; ++q)
    CF_DEV(launch_transpose(Y + (int64_t)pslot[h->fld[q]] * H.kf + c0, n, kwf, k, Vt + q * kwf * n, n, c.s));
  CF_DEV(hipMemcpyAsync(h->wl, S.wl, sizeof(double) * L, hipMemcpyDeviceToDevice, c.s));
  tm.mark(ST_BUILD);
  Factor F;
  F.L = C; F.n = n; F.ld = n; F.sL = 0;
  F.Li64 = Linv; F.sLi64 = 0;
  F.ldpart = ldp; F.sPart = 0;
  F.fail = flags + 1; F.batch = 1; F.mode = 0;
  F.rows = rows;
  // E,B rows vanish on the T pixels: with T first they stay out of the panels before the Q pixels
  const int64_t kwT = h->fld[0] == 0 ? kwf : 0;
  if (H.has_t && H.has_p && kw > kwT) { F.rows_early = n + nm + kwT; F.p_early = H.npx; }
  if (int st = potrf_on(*c.dev, F, scr, c.s, c.dev->aux[1], c.dev->ev + 8)) return st;
  tm.mark(ST_POTRF);
  GemmDesc g{};
  g.M = kw; g.N = kw; g.K = n;
  g.A = Vt; g.lda = n; g.at = 0;
  g.B = Vt; g.ldb = n; g.bt = 1;
  g.C = h->M; g.ldc = kw; g.alpha = 1.0; g.beta = 0.0; g.lower = 1; g.batch = 1;
  CF_DEV(gemm_f64(g, c.s));
  CF_DEV(launch_symmetrize(h->M, kw, kw, c.s));
  GemmDesc w{};
  w.M = kw; w.N = nm; w.K = n;
  w.A = Vt; w.lda = n; w.at = 0;
  w.B = C + n * n; w.ldb = n; w.bt = 1;
  w.C = h->b; w.ldc = nm; w.alpha = 1.0; w.beta = 0.0; w.batch = 1;
  CF_DEV(gemm_f64(w, c.s));
  CF_DEV(launch_rowsumsq(C + n * n, nm, n, n, 0, 1, h->chi2N, nm, c.s));
  CF_DEV(launch_sum_parts(ldp, (int)nblk, nblk, 1, h->ldN, 1, c.s));
  // field groups (App. field_blocks): T against the window's E, B columns of M
  const bool groups = h->fld[0] == 0 && h->nf > 1;
  CF_DEV(launch_fill_int(flags + 2, 1, 0, c.s));
  if (groups) CF_DEV(launch_any_nonzero(h->M + kwf, kw, kwf, kw - kwf, 0, 1, flags + 2, c.s));
  tm.mark(ST_SYRK);
  int fl[3];
  if (int st = read_flags(c, flags, 3, fl)) return st;
  if (fl[0]) return fail(CF_EINVAL, "non-finite entry of N_eff (check noise and spectra)");
  if (fl[1] != INT_MAX) return fail(CF_ENOTPD, "N_eff not positive definite (pivot %d)", fl[1]);
  h->blocks = (groups && fl[2] == 0) ? 2 : 1;
  return CF_OK;
}

}  // namespace
}  // namespace cf

extern "C" int cf_smw_create(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, uint32_t win_fields,
                             const double* maps, int32_t nmaps, const cf_exec* ex, cf_smw** out,
                             cf_report* rep) {
  report_init(rep);
  if (!out) return fail(CF_EINVAL, "out is NULL");
  *out = nullptr;
  HostProblem H;
  if (int st = check_problem(prob, H, true)) return st;
  if (win_lmin < H.lmin || win_lmax > H.lmax || win_lmin > win_lmax)
    return fail(CF_EINVAL, "window [%d, %d] outside [lmin, lmax] = [%d, %d]", win_lmin, win_lmax, H.lmin, H.lmax);
  if (win_fields == 0 || (win_fields & ~7u)) return fail(CF_EINVAL, "window fields 0x%x invalid", win_fields);
  const bool present[3] = {H.has_t != 0, H.has_p != 0, H.has_p != 0};
  int pslot[3] = {-1, -1, -1}, np = 0;
  for (int f = 0; f < 3; ++f)
    if (present[f]) pslot[f] = np++;
  std::unique_ptr<cf_smw, void (*)(cf_smw*)> tmp(new cf_smw, smw_free);   // frees on every error path
  for (int f = 0; f < 3; ++f) {
    if (!(win_fields & (1u << f))) continue;
    if (!present[f]) return fail(CF_EINVAL, "window field %d absent from the problem", f);
    tmp->fld[tmp->nf++] = f;
  }
  const int L = H.lmax + 1;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      if (!present[a] || !present[b]) continue;
      if (((win_fields >> a) & 1u) == ((win_fields >> b) & 1u)) continue;
      const double* row = prob->cl + (int64_t)spec_row(a, b) * L;
      for (int l = win_lmin; l <= win_lmax; ++l)
        if (row[l] != 0.0)
          return fail(CF_EINVAL, "spectrum row %d couples a window field to a fixed field at l=%d", spec_row(a, b), l);
    }
  if (nmaps <= 0 || !maps) return fail(CF_EINVAL, "no maps");
  if (prob->mem == CF_MEM_HOST && !finite_all(maps, (int64_t)nmaps * H.n)) return fail(CF_EINVAL, "non-finite map value");
  std::vector<double> clf(prob->cl, prob->cl + 6 * L);
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b)
      if (((win_fields >> a) & 1u) && ((win_fields >> b) & 1u))
        for (int l = win_lmin; l <= win_lmax; ++l) clf[(size_t)spec_row(a, b) * L + l] = 0.0;
  cf_smw* h = tmp.get();
  h->mem = prob->mem; h->n = H.n; h->lmax = H.lmax; h->wlo = win_lmin; h->whi = win_lmax; h->nmaps = nmaps;
  h->kwf = (int64_t)(win_lmax + 1) * (win_lmax + 1) - (int64_t)win_lmin * win_lmin;
  h->kw = h->kwf * h->nf;
  if (h->kw > 32768) return fail(CF_EINVAL, "window of %lld modes too large", (long long)h->kw);
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  CF_DEV(hipGetDevice(&h->device));
  const size_t kw = (size_t)h->kw;
  if (hipMalloc(&h->M, sizeof(double) * kw * kw) != hipSuccess ||
      hipMalloc(&h->b, sizeof(double) * kw * nmaps) != hipSuccess ||
      hipMalloc(&h->chi2N, sizeof(double) * nmaps) != hipSuccess ||
      hipMalloc(&h->ldN, sizeof(double)) != hipSuccess || hipMalloc(&h->wl, sizeof(double) * L) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CF_ENOMEM, "device allocation of the SMW handle failed");
  }
  Timer tm;
  tm.begin(ex && ex->stage_timing, c.s);
  if (int st = smw_setup(prob, H, h, pslot, clf, maps, c, tm)) return st;
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  if (rep) {
    const double nd = H.n, kd = (double)kw;
    rep->n = H.n; rep->nmodes = h->kw; rep->ir_iters = h->blocks;
    rep->flops = nd * nd * nd / 3.0 + nd * nd * (kd + nmaps) + nd * kd * (kd + nmaps);
  }
  *out = tmp.release();
  return CF_OK;
}

extern "C" int cf_smw_loglike(cf_smw* h, int32_t npoints, const double* cl_points, int32_t lstride,
                              double* m2lnL, double* chi2, double* logdet, const cf_exec* ex, cf_report* rep) {
  report_init(rep);
  if (!h) return fail(CF_EINVAL, "handle is NULL");
  if (npoints <= 0 || !cl_points) return fail(CF_EINVAL, "no scan points");
  if (!m2lnL) return fail(CF_EINVAL, "m2lnL is NULL");
  if (lstride < h->lmax + 1) return fail(CF_EINVAL, "lstride %d < lmax + 1 = %d", lstride, h->lmax + 1);
  int dev = 0;
  CF_DEV(hipGetDevice(&dev));
  if (dev != h->device) return fail(CF_EINVAL, "handle made on device %d, current device %d", h->device, dev);
  const size_t ncl = (size_t)npoints * 6 * lstride;
  if (h->mem == CF_MEM_HOST && !finite_all(cl_points, (int64_t)ncl)) return fail(CF_EINVAL, "non-finite scan spectra");
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  const int64_t kw = h->kw, kwf = h->kwf;
  const int nm = h->nmaps, nl = h->whi - h->wlo + 1, nf = h->nf;
  const int64_t slot = (kw + nm) * kw, nblk = (kw + kNB - 1) / kNB;
  // points per batch: up to 128 within 6 GB (each batch pays the chain of the window's diagonal
  //   blocks once; measured at 896 modes: 14.7k points/s at 16 per batch, 40.9k at 128)
  const int bt_cap = (int)std::min<int64_t>(128, std::max<int64_t>(1, (int64_t(6) << 30) / (slot * 8)));
  const int Bt = std::min<int>(bt_cap, npoints);
  Sizer z;
  if (h->mem == CF_MEM_HOST) {
    z.add<double>(ncl);
    z.add<double>((size_t)npoints * nm * 2 + (size_t)npoints);
  }
  z.add<double>((size_t)Bt * nl * 9);
  z.add<double>((size_t)Bt * slot);
  z.add<double>((size_t)Bt * nblk * kNB * kNB);
  z.add<double>((size_t)potrf_scratch(Bt));
  z.add<double>((size_t)Bt * nblk);
  z.add<double>((size_t)Bt * nm);
  z.add<double>((size_t)Bt);
  z.add<double>((size_t)Bt * nm);
  z.add<double>((size_t)Bt);
  z.add<int>(8);
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  const double* cl_dev = cl_points;
  double *m2_dev = m2lnL, *chi2_dev = chi2, *ld_dev = logdet;
  if (h->mem == CF_MEM_HOST) {
    double* t = bp.take<double>(ncl);
    CF_DEV(hipMemcpyAsync(t, cl_points, sizeof(double) * ncl, hipMemcpyHostToDevice, c.s));
    cl_dev = t;
    double* o = bp.take<double>((size_t)npoints * nm * 2 + (size_t)npoints);
    m2_dev = o;
    chi2_dev = chi2 ? o + (size_t)npoints * nm : nullptr;
    ld_dev = logdet ? o + (size_t)npoints * nm * 2 : nullptr;
  }
  double* R = bp.take<double>((size_t)Bt * nl * 9);
  double* K = bp.take<double>((size_t)Bt * slot);
  double* Linv = bp.take<double>((size_t)Bt * nblk * kNB * kNB);
  double* pscr = bp.take<double>((size_t)potrf_scratch(Bt));
  double* ldp = bp.take<double>((size_t)Bt * nblk);
  double* x2 = bp.take<double>((size_t)Bt * nm);
  double* ldK = bp.take<double>((size_t)Bt);
  double* x2g = bp.take<double>((size_t)Bt * nm);    // the E,B group's sums (blocked path)
  double* ldKg = bp.take<double>((size_t)Bt);
  int* flags = bp.take<int>(8);
  CF_DEV(launch_fill_int(flags, 1, 0, c.s));
  CF_DEV(launch_fill_int(flags + 1, 2, INT_MAX, c.s));
  // Field block-diagonal kernel (App. field_blocks): with M split into T and E,B blocks, K' splits
  // as well when no point couples T to the window's E, B fields (TE, TB zero inside the window);
  // otherwise one dense K' keeps the general case exact.
  bool blocked = false;
  if (h->blocks == 2) {
    CF_DEV(launch_fill_int(flags + 3, 1, 0, c.s));
    for (int q = 1; q < nf; ++q) {
      const int row = h->fld[q] == 1 ? 3 : 4;   // TE or TB
      CF_DEV(launch_any_nonzero(cl_dev + (int64_t)row * lstride + h->wlo, lstride, 1, nl, 6 * (int64_t)lstride,
                                npoints, flags + 3, c.s));
    }
    int fl4[4];
    if (int st = read_flags(c, flags, 4, fl4)) return st;
    blocked = fl4[3] == 0;
  }
  Timer tm;
  tm.begin(ex && ex->stage_timing, c.s);
  for (int64_t i0 = 0; i0 < npoints; i0 += Bt) {
    const int bb = (int)std::min<int64_t>(Bt, npoints - i0);
    if (blocked) {
      // T block (one field) and E,B block (the window's other fields), each factorised as a batch
      const int fldT[3] = {h->fld[0], 0, 0}, fldP[3] = {h->fld[1], h->fld[2], 0};
      for (int g = 0; g < 2; ++g) {
        const int nfg = g == 0 ? 1 : nf - 1;
        const int64_t off = g == 0 ? 0 : kwf, kwg = nfg * kwf;
        const int64_t slotg = (kwg + nm) * kwg, nblkg = (kwg + kNB - 1) / kNB;
        CF_DEV(launch_smw_lambda(cl_dev + i0 * 6 * lstride, 6 * (int64_t)lstride, lstride, h->wl, h->wlo, nl, nfg,
                                 g == 0 ? fldT : fldP, bb, R, flags + 2, c.s));
        CF_DEV(launch_smw_kernel(h->M + off * kw + off, kw, kwg, kwf, nfg, h->wlo, nl, R, bb, K, slotg, c.s));
        CF_DEV(launch_smw_rhs(h->b + off * nm, nm, kwg, kwf, nfg, h->wlo, nl, R, bb, K, slotg, c.s));
        Factor F;
        F.L = K; F.n = kwg; F.ld = kwg; F.sL = slotg;
        F.Li64 = Linv; F.sLi64 = nblkg * kNB * kNB;
        F.ldpart = ldp; F.sPart = nblkg;
        F.fail = flags + 1; F.batch = bb; F.mode = 0;
        F.rows = kwg + nm;
        if (int st = potrf_on(*c.dev, F, pscr, c.s, c.dev->aux[1], c.dev->ev + 8)) return st;
        CF_DEV(launch_rowsumsq(K + kwg * kwg, nm, kwg, kwg, slotg, bb, g == 0 ? x2 : x2g, nm, c.s));
        CF_DEV(launch_sum_parts(ldp, (int)nblkg, nblkg, bb, g == 0 ? ldK : ldKg, 1, c.s));
      }
      CF_DEV(launch_axpy(x2, x2g, 1.0, (int64_t)bb * nm, c.s));
      CF_DEV(launch_axpy(ldK, ldKg, 1.0, bb, c.s));
      CF_DEV(launch_smw_finish(h->chi2N, h->ldN, x2, ldK, bb, nm, i0, m2_dev, chi2_dev, ld_dev, c.s));
      tm.mark(ST_POTRF);
      continue;
    }
    CF_DEV(launch_smw_lambda(cl_dev + i0 * 6 * lstride, 6 * (int64_t)lstride, lstride, h->wl, h->wlo, nl, nf,
                             h->fld, bb, R, flags + 2, c.s));
    CF_DEV(launch_smw_kernel(h->M, kw, kw, kwf, nf, h->wlo, nl, R, bb, K, slot, c.s));
    CF_DEV(launch_smw_rhs(h->b, nm, kw, kwf, nf, h->wlo, nl, R, bb, K, slot, c.s));
    tm.mark(ST_BUILD);
    Factor F;
    F.L = K; F.n = kw; F.ld = kw; F.sL = slot;
    F.Li64 = Linv; F.sLi64 = nblk * kNB * kNB;
    F.ldpart = ldp; F.sPart = nblk;
    F.fail = flags + 1; F.batch = bb; F.mode = 0;
    F.rows = kw + nm;
    if (int st = potrf_on(*c.dev, F, pscr, c.s, c.dev->aux[1], c.dev->ev + 8)) return st;
    tm.mark(ST_POTRF);
    CF_DEV(launch_rowsumsq(K + kw * kw, nm, kw, kw, slot, bb, x2, nm, c.s));
    CF_DEV(launch_sum_parts(ldp, (int)nblk, nblk, bb, ldK, 1, c.s));
    CF_DEV(launch_smw_finish(h->chi2N, h->ldN, x2, ldK, bb, nm, i0, m2_dev, chi2_dev, ld_dev, c.s));
    tm.mark(ST_TRSM);
  }
  int fl[3];
  if (int st = read_flags(c, flags, 3, fl)) return st;
  if (fl[2] != INT_MAX)
    return fail(CF_EINVAL, "a point's window spectra are not positive semi-definite at l=%d", fl[2]);
  if (fl[1] != INT_MAX) {
    if (rep) rep->fail_index = fl[1];
    return fail(CF_ENOTPD, "I + R^T M R not positive definite (pivot %d)", fl[1]);
  }
  if (h->mem == CF_MEM_HOST) {
    if (int st = copy_out(m2lnL, m2_dev, (size_t)npoints * nm, CF_MEM_HOST, c.s)) return st;
    if (chi2) if (int st = copy_out(chi2, chi2_dev, (size_t)npoints * nm, CF_MEM_HOST, c.s)) return st;
    if (logdet) if (int st = copy_out(logdet, ld_dev, (size_t)npoints, CF_MEM_HOST, c.s)) return st;
  }
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  if (rep) {
    const double kd = (double)kw, k0 = (double)kwf, k1 = (double)(kw - kwf);
    rep->n = h->n; rep->nmodes = kw; rep->n_fallback = Bt;
    rep->ir_iters = blocked ? 2 : 1;   // K' blocks factorised per point
    rep->flops = blocked ? (double)npoints * (k0 * k0 * k0 / 3.0 + k1 * k1 * k1 / 3.0 + (k0 * k0 + k1 * k1) * nm +
                                              2.0 * kwf * kwf * (1.0 + (nf - 1.0) * (nf - 1.0) * (nf - 1.0)))
                         : (double)npoints * (kd * kd * kd / 3.0 + kd * kd * nm + 2.0 * kwf * kwf * nf * nf * nf);
  }
  return CF_OK;
}

namespace cf {
namespace {
// Leading-order flop counts of a likelihood scan under the two computation bases (Sect. 3, the
// "auto" choice between the harmonic and the pixel basis; per-point costs as in the complexity
// table: a Cholesky of the n x n pixel covariance against one of the window-sized kernel).
int select_basis(const cf_problem* prob, int32_t wlo, int32_t whi, uint32_t wf, int32_t npoints, int32_t nmaps,
                 cf_basis_choice* out, HostProblem& H) {
  if (!out) return fail(CF_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof *out);
  if (int st = check_problem(prob, H, true)) return st;
  if (npoints <= 0 || nmaps <= 0) return fail(CF_EINVAL, "npoints and nmaps must be positive");
  if (wlo < H.lmin || whi > H.lmax || wlo > whi) return fail(CF_EINVAL, "window [%d, %d] outside [%d, %d]", wlo, whi, H.lmin, H.lmax);
  if (wf == 0 || (wf & ~7u)) return fail(CF_EINVAL, "window fields 0x%x invalid", wf);
  const bool present[3] = {H.has_t != 0, H.has_p != 0, H.has_p != 0};
  const int L = H.lmax + 1;
  int nf = 0;
  bool ok = true;
  for (int f = 0; f < 3; ++f)
    if (wf & (1u << f)) {
      if (!present[f]) return fail(CF_EINVAL, "window field %d absent from the problem", f);
      ++nf;
    }
  for (int a = 0; a < 3 && ok; ++a)       // a spectrum coupling a window field to a fixed one
    for (int b = a; b < 3 && ok; ++b) {
      if (!present[a] || !present[b] || ((wf >> a) & 1u) == ((wf >> b) & 1u)) continue;
      const double* row = prob->cl + (int64_t)spec_row(a, b) * L;
      for (int l = wlo; l <= whi; ++l)
        if (row[l] != 0.0) ok = false;
    }
  const double n = H.n, kf = (double)((int64_t)(whi + 1) * (whi + 1) - (int64_t)wlo * wlo), k = kf * nf;
  // field groups: T and the window's E, B decouple when the fixed spectra carry no TE, TB and the
  // noise has no T-P block (diagonal noise without a low-rank part; a dense noise in host memory is
  // scanned; a dense noise in device memory counts as coupled)
  int groups = 1;
  if ((wf & 1u) && (wf & 6u) && H.has_t && H.has_p) {
    bool cross = false;
    for (int l = H.lmin; l <= H.lmax && !cross; ++l) {
      const bool in = l >= wlo && l <= whi;
      if (!(in && (wf & 2u)) && prob->cl[3 * L + l] != 0.0) cross = true;   // TE in N_eff
      if (!(in && (wf & 4u)) && prob->cl[4 * L + l] != 0.0) cross = true;   // TB in N_eff
    }
    if (prob->noise_rank > 0) cross = true;
    if (!cross && prob->noise_kind == CF_NOISE_DENSE) {
      if (prob->mem != CF_MEM_HOST) {
        cross = true;
      } else {
        const int64_t nT = H.npx;
        for (int64_t i = 0; i < nT && !cross; ++i)
          for (int64_t j = nT; j < H.n; ++j)
            if (prob->noise[i * H.n + j] != 0.0) { cross = true; break; }
      }
    }
    if (!cross) groups = 2;
  }
  const double pix_point = n * n * n / 3.0 + n * n * nmaps;
  const double k0 = kf, k1 = k - kf;
  const double harm_point = groups == 2 ? (k0 * k0 * k0 + k1 * k1 * k1) / 3.0 + (k0 * k0 + k1 * k1) * nmaps
                                        : k * k * k / 3.0 + k * k * nmaps;
  const double harm_setup = n * n * n / 3.0 + n * n * (k + nmaps) + n * k * (k + nmaps);
  out->n = H.n;
  out->k_win = (int64_t)k;
  out->groups = groups;
  out->harmonic_ok = ok ? 1 : 0;
  out->cost_pixel = npoints * pix_point;
  out->cost_harmonic = harm_setup + npoints * harm_point;
  out->basis = (ok && out->cost_harmonic < out->cost_pixel) ? 1 : 0;
  return CF_OK;
}
}  // namespace
}  // namespace cf

namespace cf {
bool smw_describe(const ::cf_smw* h, int* mem, int* nmaps) {
  if (!h) return false;
  *mem = h->mem;
  *nmaps = h->nmaps;
  return true;
}
}  // namespace cf

extern "C" int64_t cf_smw_dim(const cf_smw* h) { return h ? h->kw : -1; }

// Harmonic-basis Fisher matrix and QML with multipole switching (Sects. 2.3.3, 2.3.4; Eqs.
// projected_inv_smw, weighted_data_smw, q_harmonic; App. smw_stable): one factorisation of
// [N_eff; D^T; V_win^T] gives G^T = (L^-1 V^T)^T and U^T = (L^-1 D)^T, M = G^T G, b = G^T U; with
// Lambda = R R^T at the fiducial and K' = I + R^T M R (eigenvalues >= 1):
//   Z = V C^-1 V^T = M (I + Lambda M)^-1 = M R K'^-1 R^-1       (I + Lambda M = R K' R^-1)
//   w = V C^-1 d   = (I + M Lambda)^-1 b = R^-T K'^-1 R^T b
//   Cov(w | noise) = A T A^T, A = (I + M Lambda)^-1 = R^-T K'^-1 R^T, T = X^T N X, X = N_eff^-1 V^T
// so no difference of large matrices is formed.  F and y come from Z and w through the sparse
// trace of the pixel path; the noise bias is 1/2 tr[E_b A T A^T] (T = M without switching).
extern "C" int cf_smw_qml(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, const cf_bins* bins,
                          const double* maps, int32_t nmaps, double* y_out, double* bias_out, double* chat_out,
                          double* F_out, const cf_exec* ex, cf_report* rep) {
  using namespace cf;
  report_init(rep);
  HostProblem H;
  if (int st = check_problem(prob, H, true)) return st;
  if (win_lmin < H.lmin || win_lmax > H.lmax || win_lmin > win_lmax)
    return fail(CF_EINVAL, "window [%d, %d] outside [lmin, lmax] = [%d, %d]", win_lmin, win_lmax, H.lmin, H.lmax);
  HostBins B;
  if (int st = check_bins(bins, H, B)) return st;
  for (int b = 0; b < B.nb; ++b)
    if (B.lo[b] < win_lmin || B.hi[b] > win_lmax)
      return fail(CF_EINVAL, "bin %d = [%d, %d] outside the window [%d, %d]", b, B.lo[b], B.hi[b], win_lmin, win_lmax);
  if (nmaps <= 0 || !maps) return fail(CF_EINVAL, "no maps");
  if (!y_out || !bias_out || !chat_out) return fail(CF_EINVAL, "y_out, bias_out and chat_out are required");
  if ((int64_t)prob->noise_rank > (int64_t)H.nfm * ((int64_t)(win_lmax + 1) * (win_lmax + 1) - (int64_t)win_lmin * win_lmin))
    return fail(CF_EINVAL, "noise rank %d above the window's mode count", prob->noise_rank);
  if (prob->mem == CF_MEM_HOST && !finite_all(maps, (int64_t)nmaps * H.n)) return fail(CF_EINVAL, "non-finite map value");
  // the window holds every harmonic field of the problem (switching by multipole only)
  const int nf = H.nfm, L = H.lmax + 1;
  int fld[3] = {0, 0, 0};
  {
    int q = 0;
    if (H.has_t) fld[q++] = 0;
    if (H.has_p) { fld[q++] = 1; fld[q++] = 2; }
  }
  const int64_t n = H.n, k = H.k, kwf = (int64_t)(win_lmax + 1) * (win_lmax + 1) - (int64_t)win_lmin * win_lmin;
  const int64_t kw = nf * kwf, nm = nmaps, nl = win_lmax - win_lmin + 1;
  const int K = B.ns * B.nb;
  std::vector<double> clf(prob->cl, prob->cl + 6 * L);   // fixed spectra: the window's entries removed
  for (int s = 0; s < 6; ++s)
    for (int l = win_lmin; l <= win_lmax; ++l) clf[(size_t)s * L + l] = 0.0;
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  const int64_t rows = n + nm + kw, nblk = (n + kNB - 1) / kNB, nblkK = (kw + kNB - 1) / kNB;
  const int npq = nf * nf, nq = npq * (npq + 1) / 2;
  const size_t kk = (size_t)kw * kw, nk = (size_t)n * kw, ngram = (size_t)nl * (nl + 1) / 2 * nq;
  Sizer z;
  size_staging(z, prob, H);
  z.add<double>((size_t)rows * n);             // [N_eff; D^T; V_win^T], factorised
  z.add<double>((size_t)n * k);                // Y
  z.add<double>((size_t)nblk * kNB * kNB);     // inverted diagonal blocks of N_eff
  z.add<double>((size_t)potrf_scratch(1));
  z.add<double>((size_t)nblk);
  z.add<double>((size_t)nm * n);               // maps (host inputs)
  z.add<double>((size_t)(kw + nm) * kw);       // [K'; b'^T]
  z.add<double>((size_t)nblkK * kNB * kNB);
  z.add<double>((size_t)nblkK);
  for (int i = 0; i < 8; ++i) z.add<double>(kk);   // M, T, W1, Y1, Z, P1, Q, Bn
  for (int i = 0; i < 3; ++i) z.add<double>(nk);   // G, X, NX
  z.add<double>((size_t)kw * nm * 3);          // b, w, scratch
  z.add<double>((size_t)6 * L * 2);            // fiducial spectra, zero spectra
  z.add<double>((size_t)nl * 9);               // R
  z.add<double>(ngram * 2);                    // Gram of Z and of Bn
  z.add<double>((size_t)nl * npq * 2);         // block traces
  z.add<double>((size_t)K * K * 2);            // F, copy for the solve
  z.add<double>((size_t)nm * K * 3 + K);       // y, q, chat, bias
  z.add<int>(B.nb);
  z.add<int>(B.nb);
  z.add<int>(8);
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  Staged S;
  if (int st = stage(bp, prob, H, clf.data(), c.s, S)) return st;
  double* C = bp.take<double>((size_t)rows * n);
  double* Y = bp.take<double>((size_t)n * k);
  double* Linv = bp.take<double>((size_t)nblk * kNB * kNB);
  double* scr = bp.take<double>((size_t)potrf_scratch(1));
  double* ldp = bp.take<double>((size_t)nblk);
  double* mcopy = bp.take<double>((size_t)nm * n);
  double* KK = bp.take<double>((size_t)(kw + nm) * kw);
  double* LiK = bp.take<double>((size_t)nblkK * kNB * kNB);
  double* ldpK = bp.take<double>((size_t)nblkK);
  double* M = bp.take<double>(kk);
  double* T = bp.take<double>(kk);
  double* W1 = bp.take<double>(kk);
  double* Y1 = bp.take<double>(kk);
  double* Z = bp.take<double>(kk);
  double* P1 = bp.take<double>(kk);
  double* Q = bp.take<double>(kk);
  double* Bn = bp.take<double>(kk);
  double* G = bp.take<double>(nk);
  double* X = bp.take<double>(nk);
  double* NX = bp.take<double>(nk);
  double* bv = bp.take<double>((size_t)kw * nm * 3);
  double* wv = bv + (size_t)kw * nm;
  double* tv = wv + (size_t)kw * nm;
  double* cl0 = bp.take<double>((size_t)6 * L * 2);
  double* zl = cl0 + (size_t)6 * L;
  double* R = bp.take<double>((size_t)nl * 9);
  double* gramZ = bp.take<double>(ngram * 2);
  double* gramB = gramZ + ngram;
  double* ztrZ = bp.take<double>((size_t)nl * npq * 2);
  double* ztrB = ztrZ + (size_t)nl * npq;
  double* F = bp.take<double>((size_t)K * K * 2);
  double* Fw = F + (size_t)K * K;
  double* y = bp.take<double>((size_t)nm * K * 3 + K);
  double* q = y + (size_t)nm * K;
  double* chat = q + (size_t)nm * K;
  double* bias = chat + (size_t)nm * K;
  int* dlo = bp.take<int>(B.nb);
  int* dhi = bp.take<int>(B.nb);
  int* flags = bp.take<int>(8);
  hipStream_t s = c.s;
  CF_DEV(hipMemcpyAsync(dlo, B.lo.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, s));
  CF_DEV(hipMemcpyAsync(dhi, B.hi.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, s));
  CF_DEV(hipMemcpyAsync(cl0, prob->cl, sizeof(double) * 6 * L, hipMemcpyHostToDevice, s));
  CF_DEV(launch_fill(zl, 6 * L, 0.0, s));
  const double* mdev = maps;
  if (prob->mem == CF_MEM_HOST) {
    CF_DEV(hipMemcpyAsync(mcopy, maps, sizeof(double) * nm * n, hipMemcpyHostToDevice, s));
    mdev = mcopy;
  }
  CF_DEV(launch_fill_int(flags, 1, 0, s));
  CF_DEV(launch_fill_int(flags + 1, 4, INT_MAX, s));
  Timer tm;
  tm.begin(ex && ex->stage_timing, s);
  // ---- N_eff with the maps and the window's harmonic rows below it
  CF_DEV(launch_ybuild(S.P, Y, k, s));
  CF_DEV(launch_cov_build(S.P, S.cw, 0, 1, prob->noise_kind, S.noise, prob->noise_rank, S.noise_U, C, n, 0, 1, flags, s));
  CF_DEV(hipMemcpyAsync(C + n * n, mdev, sizeof(double) * nm * n, hipMemcpyDeviceToDevice, s));
  double* Vt = C + (n + nm) * n;
  const int64_t c0 = (int64_t)win_lmin * win_lmin - (int64_t)H.lmin * H.lmin;
  for (int f = 0; f < nf; ++f)
    CF_DEV(launch_transpose(Y + (int64_t)f * H.kf + c0, n, kwf, k, Vt + f * kwf * n, n, s));
  tm.mark(ST_BUILD);
  Factor FN;
  FN.L = C; FN.n = n; FN.ld = n; FN.sL = 0;
  FN.Li64 = Linv; FN.ldpart = ldp; FN.fail = flags + 1; FN.batch = 1; FN.rows = rows;
  if (H.has_t && H.has_p) { FN.rows_early = n + nm + kwf; FN.p_early = H.npx; }   // E,B rows vanish on T pixels
  if (int st = potrf_on(*c.dev, FN, scr, s, c.dev->aux[1], c.dev->ev + 8)) return st;
  tm.mark(ST_POTRF);
  // ---- M = G^T G, b = G^T U, X = L^-T G, T = X^T N X
  GemmDesc g{};
  g.M = kw; g.N = kw; g.K = n; g.A = Vt; g.lda = n; g.B = Vt; g.ldb = n; g.bt = 1;
  g.C = M; g.ldc = kw; g.alpha = 1.0; g.lower = 1; g.batch = 1;
  CF_DEV(gemm_f64(g, s));
  CF_DEV(launch_symmetrize(M, kw, kw, s));
  GemmDesc gb{};
  gb.M = kw; gb.N = nm; gb.K = n; gb.A = Vt; gb.lda = n; gb.B = C + n * n; gb.ldb = n; gb.bt = 1;
  gb.C = bv; gb.ldc = nm; gb.alpha = 1.0; gb.batch = 1;
  CF_DEV(gemm_f64(gb, s));
  CF_DEV(launch_transpose(Vt, kw, n, n, G, kw, s));                      // G [n][kw]
  CF_DEV(trsm_lower_t_f64(FN, G, kw, 0, X, kw, 0, kw, s));                // X = L^-T G (G consumed)
  if (prob->noise_kind == CF_NOISE_DENSE) {
    GemmDesc gn{};
    gn.M = n; gn.N = kw; gn.K = n; gn.A = S.noise; gn.lda = n; gn.B = X; gn.ldb = kw;
    gn.C = NX; gn.ldc = kw; gn.alpha = 1.0; gn.batch = 1;
    CF_DEV(gemm_f64(gn, s));
  } else {
    CF_DEV(launch_fill(NX, (int64_t)nk, 0.0, s));
    CF_DEV(launch_rowscale_add(S.noise, X, NX, n, kw, s));               // NX = diag(N) X
  }
  if (prob->noise_rank > 0) {                                            // + U (U^T X)
    GemmDesc gu{};
    gu.M = prob->noise_rank; gu.N = kw; gu.K = n; gu.A = S.noise_U; gu.lda = prob->noise_rank; gu.at = 1;
    gu.B = X; gu.ldb = kw; gu.C = W1; gu.ldc = kw; gu.alpha = 1.0; gu.batch = 1;   // U^T X in W1
    CF_DEV(gemm_f64(gu, s));
    GemmDesc gv{};
    gv.M = n; gv.N = kw; gv.K = prob->noise_rank; gv.A = S.noise_U; gv.lda = prob->noise_rank;
    gv.B = gu.C; gv.ldb = kw; gv.C = NX; gv.ldc = kw; gv.alpha = 1.0; gv.beta = 1.0; gv.batch = 1;
    CF_DEV(gemm_f64(gv, s));
  }
  GemmDesc gt{};
  gt.M = kw; gt.N = kw; gt.K = n; gt.A = X; gt.lda = kw; gt.at = 1; gt.B = NX; gt.ldb = kw;
  gt.C = T; gt.ldc = kw; gt.alpha = 1.0; gt.batch = 1;
  CF_DEV(gemm_f64(gt, s));
  tm.mark(ST_SYRK);
  // ---- fiducial kernel K' = I + R^T M R and b' = R^T b, factorised together
  CF_DEV(launch_smw_lambda(cl0, 6 * (int64_t)L, L, S.wl, win_lmin, (int)nl, nf, fld, 1, R, flags + 2, s));
  const int64_t slotK = (kw + nm) * kw;
  CF_DEV(launch_smw_kernel(M, kw, kw, kwf, nf, win_lmin, (int)nl, R, 1, KK, slotK, s));
  CF_DEV(launch_smw_rhs(bv, (int)nm, kw, kwf, nf, win_lmin, (int)nl, R, 1, KK, slotK, s));
  Factor FK;
  FK.L = KK; FK.n = kw; FK.ld = kw; FK.sL = slotK; FK.Li64 = LiK; FK.ldpart = ldpK;
  FK.fail = flags + 3; FK.batch = 1; FK.rows = kw + nm;
  if (int st = potrf_on(*c.dev, FK, scr, s, c.dev->aux[1], c.dev->ev + 8)) return st;
  // ---- Z = M R K'^-1 R^-1: W1 = R^T M, Y1 = K'^-1 W1, Z = R^-T Y1 (= Z^T), mirrored
  CF_DEV(launch_apply_rblock(M, kw, W1, kw, kw, kwf, nf, win_lmin, R, 1, 0, s));
  CF_DEV(trsm_lower_f64(FK, W1, kw, 0, P1, kw, 0, kw, 0, s));            // P1 = L_K^-1 W1
  CF_DEV(trsm_lower_t_f64(FK, P1, kw, 0, Y1, kw, 0, kw, s));             // Y1 = L_K^-T P1
  CF_DEV(launch_apply_rblock(Y1, kw, Z, kw, kw, kwf, nf, win_lmin, R, 3, 0, s));
  CF_DEV(launch_symmetrize(Z, kw, kw, s));
  // ---- w = R^-T K'^-1 R^T b: the factorisation left (L_K^-1 b')^T below K'
  CF_DEV(launch_transpose(KK + kw * kw, nm, kw, kw, tv, nm, s));          // [kw][nm]
  CF_DEV(trsm_lower_t_f64(FK, tv, nm, 0, wv, nm, 0, nm, s));             // wv = K'^-1 b'
  CF_DEV(launch_apply_rblock(wv, nm, tv, nm, nm, kwf, nf, win_lmin, R, 3, 0, s));   // tv = R^-T wv
  // ---- noise covariance of w: Bn = R^-T K'^-1 (R^T T R) K'^-1 R^-1
  CF_DEV(launch_apply_rblock(T, kw, W1, kw, kw, kwf, nf, win_lmin, R, 1, 0, s));   // W1 = R^T T
  CF_DEV(launch_apply_rblock(W1, kw, P1, kw, kw, kwf, nf, win_lmin, R, 0, 1, s));  // P1 = W1 R
  CF_DEV(trsm_lower_f64(FK, P1, kw, 0, W1, kw, 0, kw, 0, s));
  CF_DEV(trsm_lower_t_f64(FK, W1, kw, 0, Q, kw, 0, kw, s));              // Q = K'^-1 P1
  CF_DEV(launch_transpose(Q, kw, kw, kw, W1, kw, s));
  CF_DEV(trsm_lower_f64(FK, W1, kw, 0, P1, kw, 0, kw, 0, s));
  CF_DEV(trsm_lower_t_f64(FK, P1, kw, 0, Q, kw, 0, kw, s));              // Q = K'^-1 P1 K'^-1
  CF_DEV(launch_apply_rblock(Q, kw, W1, kw, kw, kwf, nf, win_lmin, R, 3, 0, s));   // R^-T Q
  CF_DEV(launch_apply_rblock(W1, kw, Bn, kw, kw, kwf, nf, win_lmin, R, 2, 1, s));  // ... R^-1
  tm.mark(ST_TRSM);
  // ---- sparse-trace Fisher, y and the noise bias on the window's modes
  DevProblem Pw = S.P;
  Pw.lmin = win_lmin; Pw.lmax = win_lmax; Pw.kf = (int)kwf; Pw.k = kw;
  CF_DEV(launch_gram(Pw, Z, kw, gramZ, ztrZ, s));
  CF_DEV(launch_gram(Pw, Bn, kw, gramB, ztrB, s));
  SpecSel sel;
  sel.ns = B.ns;
  for (int i = 0; i < 6; ++i) sel.spec[i] = B.spec[i];
  sel.nb = B.nb; sel.lo = dlo; sel.hi = dhi;
  CF_DEV(launch_fisher_assemble(Pw, sel, gramZ, F, s));
  DevProblem Pb = Pw;
  Pb.lam = zl;                                  // the bias is the traces of Bn alone
  CF_DEV(launch_bias_assemble(Pb, sel, gramB, ztrB, bias, s));
  CF_DEV(launch_quad_assemble(Pw, sel, tv, nm, (int)nm, y, s));
  CF_DEV(hipMemcpyAsync(q, y, sizeof(double) * nm * K, hipMemcpyDeviceToDevice, s));
  CF_DEV(launch_sub_bias(q, bias, K, (int)nm, s));
  CF_DEV(hipMemcpyAsync(Fw, F, sizeof(double) * K * K, hipMemcpyDeviceToDevice, s));
  CF_DEV(launch_small_spd_solve(Fw, K, q, chat, (int)nm, flags + 4, s));
  tm.mark(ST_QML);
  int fl[5];
  if (int st = read_flags(c, flags, 5, fl)) return st;
  if (fl[0]) return fail(CF_EINVAL, "non-finite entry of N_eff (check noise and spectra)");
  if (fl[1] != INT_MAX) { if (rep) rep->fail_index = fl[1]; return fail(CF_ENOTPD, "N_eff not positive definite (pivot %d)", fl[1]); }
  if (fl[2] != INT_MAX) return fail(CF_EINVAL, "the fiducial window spectra are not positive semi-definite at l=%d", fl[2]);
  if (fl[3] != INT_MAX) return fail(CF_ENOTPD, "I + R^T M R not positive definite (pivot %d)", fl[3]);
  if (fl[4] != INT_MAX) { if (rep) rep->fail_index = fl[4]; return fail(CF_ENOTPD, "Fisher matrix not positive definite at pivot %d", fl[4]); }
  if (int st = copy_out(y_out, y, (size_t)nm * K, prob->mem, s)) return st;
  if (int st = copy_out(bias_out, bias, (size_t)K, prob->mem, s)) return st;
  if (int st = copy_out(chat_out, chat, (size_t)nm * K, prob->mem, s)) return st;
  if (F_out)
    if (int st = copy_out(F_out, F, (size_t)K * K, prob->mem, s)) return st;
  CF_DEV(hipStreamSynchronize(s));
  tm.finish(rep);
  if (rep) {
    const double nd = (double)n, kd = (double)kw;
    rep->n = n; rep->nmodes = kw;
    rep->flops = nd * nd * nd / 3.0 + nd * nd * (kd + nm) * 2.0 + nd * kd * kd * 2.0 + 10.0 * kd * kd * kd;
  }
  return CF_OK;
}

// Joint two-map QML (Eq. C_joint): the data vector (d1, d2) of one sky seen by two data sets, with
// covariance [[S + N1, S + N12], [S + N12^T, S + N2]], is the data vector of a 2n-dimensional
// problem whose harmonic operator is the stacked [Y; Y].  One factorisation of
// [C_j; (d1 d2) rows; (Y^T Y^T) rows] gives u^T = (L^-1 d)^T and G^T = (L^-1 [Y; Y])^T; then
// Z = G^T G, w = G^T u, F, y, the noise bias 1/2 tr[E_b (Z - Z Lambda Z)] (C_j minus the joint
// signal [Y; Y] Lambda [Y; Y]^T is the joint noise) and C_hat as in cf_qml.
extern "C" int cf_qml_joint(const cf_problem* p1, const cf_problem* p2, const double* N12, const cf_bins* bins,
                            const double* maps1, const double* maps2, int32_t nmaps, double* y_out,
                            double* bias_out, double* chat_out, double* F_out, const cf_exec* ex,
                            cf_report* rep) {
  using namespace cf;
  report_init(rep);
  HostProblem H, H2;
  if (int st = check_problem(p1, H, true)) return st;
  if (int st = check_problem(p2, H2, false)) return st;
  if (H2.n != H.n || H2.lmin != H.lmin || H2.lmax != H.lmax || p2->fields != p1->fields || p2->mem != p1->mem)
    return fail(CF_EINVAL, "the two data sets disagree on n, fields, l-range or memory space");
  HostBins B;
  if (int st = check_bins(bins, H, B)) return st;
  if (nmaps <= 0 || !maps1 || !maps2) return fail(CF_EINVAL, "no maps");
  if (!y_out || !bias_out || !chat_out) return fail(CF_EINVAL, "y_out, bias_out and chat_out are required");
  const int64_t n = H.n, n2 = 2 * (int64_t)H.n, k = H.k, nm = nmaps;
  const bool host = p1->mem == CF_MEM_HOST;
  if (host) {
    if (!finite_all(maps1, nm * n) || !finite_all(maps2, nm * n)) return fail(CF_EINVAL, "non-finite map value");
    if (N12 && !finite_all(N12, n * n)) return fail(CF_EINVAL, "non-finite entry of N12");
  }
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  const int K = B.ns * B.nb;
  const int nl = H.lmax - H.lmin + 1;
  const int np = H.nfm * H.nfm, nq = np * (np + 1) / 2;
  const int64_t rows = n2 + nm + k, nblk = (n2 + kNB - 1) / kNB;
  Sizer z;
  size_staging(z, p1, H);
  size_staging(z, p2, H2);
  z.add<double>((size_t)rows * n2);            // [C_j; d rows; Y_j^T rows], factorised
  z.add<double>((size_t)n * k);                // Y
  z.add<double>((size_t)n * n);                // N12^T (or a zero diagonal)
  z.add<double>(host && N12 ? (size_t)n * n : 1);   // N12 (host input)
  z.add<double>((size_t)nm * n * 2);           // maps (host inputs)
  z.add<double>((size_t)k * k);                // Z
  z.add<double>((size_t)nblk * kNB * kNB);     // inverted diagonal blocks
  z.add<double>((size_t)potrf_scratch(1));
  z.add<double>((size_t)nblk);
  z.add<double>((size_t)k * nm);               // w
  z.add<double>((size_t)nl * (nl + 1) / 2 * nq);
  z.add<double>((size_t)nl * np);
  z.add<double>((size_t)K * K * 2);            // F and its copy for the solve
  z.add<double>((size_t)nm * K * 3 + K);       // y, y - b, chat, bias
  z.add<int>(B.nb);
  z.add<int>(B.nb);
  z.add<int>(8);
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  Staged S1, S2;
  if (int st = stage(bp, p1, H, nullptr, c.s, S1)) return st;
  if (int st = stage(bp, p2, H2, nullptr, c.s, S2)) return st;
  double* C = bp.take<double>((size_t)rows * n2);
  double* Y = bp.take<double>((size_t)n * k);
  double* X12 = bp.take<double>((size_t)n * n);
  double* N12c = bp.take<double>(host && N12 ? (size_t)n * n : 1);
  double* mcopy = bp.take<double>((size_t)nm * n * 2);
  double* Z = bp.take<double>((size_t)k * k);
  double* Linv = bp.take<double>((size_t)nblk * kNB * kNB);
  double* scr = bp.take<double>((size_t)potrf_scratch(1));
  double* ldp = bp.take<double>((size_t)nblk);
  double* W = bp.take<double>((size_t)k * nm);
  double* gram = bp.take<double>((size_t)nl * (nl + 1) / 2 * nq);
  double* ztr = bp.take<double>((size_t)nl * np);
  double* F = bp.take<double>((size_t)K * K * 2);
  double* Fw = F + (size_t)K * K;
  double* y = bp.take<double>((size_t)nm * K * 3 + K);
  double* q = y + (size_t)nm * K;
  double* chat = q + (size_t)nm * K;
  double* bias = chat + (size_t)nm * K;
  int* dlo = bp.take<int>(B.nb);
  int* dhi = bp.take<int>(B.nb);
  int* flags = bp.take<int>(8);
  hipStream_t s = c.s;
  CF_DEV(hipMemcpyAsync(dlo, B.lo.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, s));
  CF_DEV(hipMemcpyAsync(dhi, B.hi.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, s));
  const double *m1 = maps1, *m2 = maps2, *x12 = N12;
  if (host) {
    CF_DEV(hipMemcpyAsync(mcopy, maps1, sizeof(double) * nm * n, hipMemcpyHostToDevice, s));
    CF_DEV(hipMemcpyAsync(mcopy + nm * n, maps2, sizeof(double) * nm * n, hipMemcpyHostToDevice, s));
    m1 = mcopy;
    m2 = mcopy + nm * n;
    if (N12) {
      CF_DEV(hipMemcpyAsync(N12c, N12, sizeof(double) * n * n, hipMemcpyHostToDevice, s));
      x12 = N12c;
    }
  }
  CF_DEV(launch_fill_int(flags, 1, 0, s));
  CF_DEV(launch_fill_int(flags + 1, 3, INT_MAX, s));
  Timer tm;
  tm.begin(ex && ex->stage_timing, s);
  // ---- C_j (lower): the two diagonal blocks with their noises and the full off-diagonal block
  //      S + N12^T, whose "noise" is N12^T as a dense matrix (or a zero diagonal)
  CF_DEV(launch_cov_build(S1.P, S1.cw, 0, 1, p1->noise_kind, S1.noise, p1->noise_rank, S1.noise_U, C, n2, 0, 1,
                          flags, s));
  CF_DEV(launch_cov_build(S1.P, S1.cw, 0, 1, p2->noise_kind, S2.noise, p2->noise_rank, S2.noise_U,
                          C + n * n2 + n, n2, 0, 1, flags, s));
  if (x12) CF_DEV(launch_transpose(x12, n, n, n, X12, n, s));
  else CF_DEV(launch_fill(X12, n, 0.0, s));
  CF_DEV(launch_cov_build(S1.P, S1.cw, 0, 1, x12 ? CF_NOISE_DENSE : CF_NOISE_DIAG, X12, 0, nullptr, C + n * n2,
                          n2, 0, 0, flags, s));
  // ---- extra rows: the maps (d1 | d2) and the stacked harmonic operator (Y^T | Y^T)
  double* Dt = C + n2 * n2;
  double* Gt = Dt + nm * n2;
  CF_DEV(hipMemcpy2DAsync(Dt, sizeof(double) * n2, m1, sizeof(double) * n, sizeof(double) * n, nm,
                          hipMemcpyDeviceToDevice, s));
  CF_DEV(hipMemcpy2DAsync(Dt + n, sizeof(double) * n2, m2, sizeof(double) * n, sizeof(double) * n, nm,
                          hipMemcpyDeviceToDevice, s));
  CF_DEV(launch_ybuild(S1.P, Y, k, s));
  CF_DEV(launch_transpose(Y, n, k, k, Gt, n2, s));
  CF_DEV(launch_transpose(Y, n, k, k, Gt + n, n2, s));
  tm.mark(ST_BUILD);
  Factor FN;
  FN.L = C; FN.n = n2; FN.ld = n2; FN.sL = 0;
  FN.Li64 = Linv; FN.ldpart = ldp; FN.fail = flags + 1; FN.batch = 1; FN.rows = rows;
  if (int st = potrf_on(*c.dev, FN, scr, s, c.dev->aux[1], c.dev->ev + 8)) return st;
  tm.mark(ST_POTRF);
  // ---- Z = G^T G (lower), w = G^T u
  GemmDesc g{};
  g.M = k; g.N = k; g.K = n2;
  g.A = Gt; g.lda = n2; g.B = Gt; g.ldb = n2; g.bt = 1;
  g.C = Z; g.ldc = k; g.alpha = 1.0; g.lower = 1; g.batch = 1;
  CF_DEV(gemm_f64(g, s));
  if (nm <= 8) {
    CF_DEV(launch_rowdot(Gt, n2, k, n2, Dt, n2, (int)nm, W, nm, k, 0, s));
  } else {
    GemmDesc w{};
    w.M = k; w.N = nm; w.K = n2;
    w.A = Gt; w.lda = n2; w.B = Dt; w.ldb = n2; w.bt = 1;
    w.C = W; w.ldc = nm; w.alpha = 1.0; w.batch = 1;
    CF_DEV(gemm_f64(w, s));
  }
  tm.mark(ST_SYRK);
  CF_DEV(launch_symmetrize(Z, k, k, s));
  CF_DEV(launch_gram(S1.P, Z, k, gram, ztr, s));
  SpecSel sel;
  sel.ns = B.ns;
  for (int i = 0; i < 6; ++i) sel.spec[i] = B.spec[i];
  sel.nb = B.nb; sel.lo = dlo; sel.hi = dhi;
  CF_DEV(launch_fisher_assemble(S1.P, sel, gram, F, s));
  CF_DEV(launch_bias_assemble(S1.P, sel, gram, ztr, bias, s));
  CF_DEV(launch_quad_assemble(S1.P, sel, W, (int)nm, (int)nm, y, s));
  CF_DEV(hipMemcpyAsync(q, y, sizeof(double) * nm * K, hipMemcpyDeviceToDevice, s));
  CF_DEV(launch_sub_bias(q, bias, K, (int)nm, s));
  CF_DEV(hipMemcpyAsync(Fw, F, sizeof(double) * K * K, hipMemcpyDeviceToDevice, s));
  CF_DEV(launch_small_spd_solve(Fw, K, q, chat, (int)nm, flags + 3, s));
  tm.mark(ST_QML);
  int fl[4];
  if (int st = read_flags(c, flags, 4, fl)) return st;
  if (fl[0]) return fail(CF_EINVAL, "non-finite entry of the joint covariance (check noises and spectra)");
  if (fl[1] != INT_MAX) {
    if (rep) rep->fail_index = fl[1];
    return fail(CF_ENOTPD, "joint covariance not positive definite at pivot %d", fl[1]);
  }
  if (fl[3] != INT_MAX) {
    if (rep) rep->fail_index = fl[3];
    return fail(CF_ENOTPD, "Fisher matrix not positive definite at pivot %d", fl[3]);
  }
  if (int st = copy_out(y_out, y, (size_t)nm * K, p1->mem, s)) return st;
  if (int st = copy_out(bias_out, bias, (size_t)K, p1->mem, s)) return st;
  if (int st = copy_out(chat_out, chat, (size_t)nm * K, p1->mem, s)) return st;
  if (F_out)
    if (int st = copy_out(F_out, F, (size_t)K * K, p1->mem, s)) return st;
  CF_DEV(hipStreamSynchronize(s));
  tm.finish(rep);
  if (rep) {
    const double nd = (double)n2, kd = (double)k;
    rep->n = n2; rep->nmodes = k;
    rep->flops = nd * nd * nd / 3.0 + nd * nd * (kd + nm) + kd * kd * nd;
  }
  return CF_OK;
}

extern "C" int cf_select_basis(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, uint32_t win_fields,
                               int32_t npoints, int32_t nmaps, cf_basis_choice* out) {
  HostProblem H;
  return cf::select_basis(prob, win_lmin, win_lmax, win_fields, npoints, nmaps, out, H);
}

extern "C" int cf_loglike_auto(const cf_problem* prob, int32_t win_lmin, int32_t win_lmax, uint32_t win_fields,
                               int32_t npoints, const double* cl_points, int32_t lstride, const double* maps,
                               int32_t nmaps, double* m2lnL, double* chi2, double* logdet,
                               cf_basis_choice* choice, const cf_exec* ex, cf_report* rep) {
  cf_basis_choice ch;
  HostProblem H;
  if (int st = cf::select_basis(prob, win_lmin, win_lmax, win_fields, npoints, nmaps, &ch, H)) return st;
  if (choice) *choice = ch;
  if (!ch.basis) {
    // pixel basis: outputs [npoints][1 problem][nmaps] are the [npoints][nmaps] layout
    const double* mp[1] = {maps};
    return cf_loglike_batch(prob, 1, npoints, cl_points, lstride, mp, nmaps, CF_FP64, m2lnL, chi2, logdet, ex, rep);
  }
  cf_smw* h = nullptr;
  if (int st = cf_smw_create(prob, win_lmin, win_lmax, win_fields, maps, nmaps, ex, &h, nullptr)) return st;
  const int st = cf_smw_loglike(h, npoints, cl_points, lstride, m2lnL, chi2, logdet, ex, rep);
  cf_smw_destroy(h);
  return st;
}

extern "C" void cf_smw_destroy(cf_smw* h) { smw_free(h); }

extern "C" int cf_decorrelate(const double* F, int32_t K, const double* q, int32_t nvec, int32_t mem,
                              double* out, double* Fmhalf_out, const cf_exec* ex, cf_report* rep) {
  report_init(rep);
  if (!F || K < 1 || K > 1024) return fail(CF_EINVAL, "K=%d outside [1, 1024] or F NULL", K);
  if (nvec < 0 || (nvec > 0 && (!q || !out))) return fail(CF_EINVAL, "nvec=%d with q=%p out=%p", nvec,
                                                          (const void*)q, (void*)out);
  if (nvec == 0 && !Fmhalf_out) return fail(CF_EINVAL, "nothing to compute");
  if (mem != CF_MEM_HOST && mem != CF_MEM_DEVICE) return fail(CF_EINVAL, "unknown mem %d", mem);
  const int64_t kk = (int64_t)K * K;
  if (mem == CF_MEM_HOST) {
    if (!finite_all(F, kk)) return fail(CF_EINVAL, "non-finite F");
    if (nvec > 0 && !finite_all(q, (int64_t)K * nvec)) return fail(CF_EINVAL, "non-finite q");
  }
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  Sizer z;
  if (mem == CF_MEM_HOST) {
    z.add<double>(kk);
    z.add<double>((size_t)K * nvec);
    z.add<double>((size_t)K * nvec);
  }
  z.add<double>(kk);
  z.add<double>(kk);
  z.add<double>(kk);
  z.add<double>(K);
  z.add<int>(8);
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  const double* Fd = F;
  const double* qd = q;
  double* od = out;
  if (mem == CF_MEM_HOST) {
    double* t = bp.take<double>(kk);
    CF_DEV(hipMemcpyAsync(t, F, sizeof(double) * kk, hipMemcpyHostToDevice, c.s));
    Fd = t;
    double* tq = bp.take<double>((size_t)K * nvec);
    if (nvec > 0) CF_DEV(hipMemcpyAsync(tq, q, sizeof(double) * K * nvec, hipMemcpyHostToDevice, c.s));
    qd = tq;
    od = bp.take<double>((size_t)K * nvec);
  }
  double* A = bp.take<double>(kk);
  double* U = bp.take<double>(kk);
  double* R = bp.take<double>(kk);
  double* w = bp.take<double>(K);
  int* info = bp.take<int>(8);
  Timer tm;
  tm.begin(ex && ex->stage_timing, c.s);
  CF_DEV(launch_inverse_sqrt(Fd, K, A, U, w, R, 60, 1e-12, info, c.s));
  if (nvec > 0) CF_DEV(launch_apply_rows(R, qd, K, nvec, od, c.s));
  tm.mark(ST_QML);
  int fl[2];
  if (int st = read_flags(c, info, 2, fl)) return st;
  if (rep) rep->ir_iters = fl[0];
  if (fl[1]) return fail(CF_ENOCONV, "Jacobi sweeps did not converge in %d sweeps", fl[0]);
  if (nvec > 0 && mem == CF_MEM_HOST)
    if (int st = copy_out(out, od, (size_t)K * nvec, CF_MEM_HOST, c.s)) return st;
  if (Fmhalf_out)
    if (int st = copy_out(Fmhalf_out, R, (size_t)kk, mem, c.s)) return st;
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  return CF_OK;
}

namespace cf {
namespace {
// The two data sets of a cross-QML share everything but the noise: geometry, fields, l-range,
// spectra, beam and window (so that S and every P_b are common), and the memory space.
int check_same_model(const cf_problem* a, const cf_problem* b, const HostProblem& Ha, const HostProblem& Hb) {
  const int L = Ha.lmax + 1;
  auto same = [](const double* x, const double* y, int64_t n) {
    if (!x || !y) return x == y;
    return std::memcmp(x, y, sizeof(double) * n) == 0;
  };
  if (a->nside != b->nside || a->fields != b->fields || Ha.lmin != Hb.lmin || Ha.lmax != Hb.lmax ||
      Ha.n != Hb.n || a->mem != b->mem)
    return fail(CF_EINVAL, "cross-QML data sets differ in geometry, fields, l-range or memory space");
  if (a->nside > 0) {
    if (Ha.ring != Hb.ring) return fail(CF_EINVAL, "cross-QML data sets differ in their masks");
  } else if (!same(a->theta, b->theta, Ha.npx) || !same(a->phi, b->phi, Ha.npx)) {
    return fail(CF_EINVAL, "cross-QML data sets differ in their directions");
  }
  if (!same(a->cl, b->cl, 6LL * L) || !same(a->bl, b->bl, L) || !same(a->pl, b->pl, L))
    return fail(CF_EINVAL, "cross-QML data sets differ in spectra, beam or pixel window");
  return CF_OK;
}
}  // namespace
}  // namespace cf

extern "C" int cf_qml_cross(const cf_problem* prob1, const cf_problem* prob2, const cf_bins* bins,
                            const double* maps1, const double* maps2, int32_t nmaps, double* q_out,
                            double* chat_out, double* W_out, const cf_exec* ex, cf_report* rep) {
  report_init(rep);
  HostProblem H1, H2;
  if (int st = check_problem(prob1, H1, true)) return st;
  if (int st = check_problem(prob2, H2, true)) return st;
  if (int st = check_same_model(prob1, prob2, H1, H2)) return st;
  HostBins B;
  if (int st = check_bins(bins, H1, B)) return st;
  if (nmaps <= 0 || !maps1 || !maps2) return fail(CF_EINVAL, "no maps");
  if (!q_out || !chat_out) return fail(CF_EINVAL, "q_out and chat_out are required");
  if (prob1->mem == CF_MEM_HOST && (!finite_all(maps1, (int64_t)nmaps * H1.n) || !finite_all(maps2, (int64_t)nmaps * H1.n)))
    return fail(CF_EINVAL, "non-finite map value");
  CallCtx c;
  if (int st = c.begin(ex)) return st;
  const int K = B.ns * B.nb;
  const int nl = H1.lmax - H1.lmin + 1, np = H1.nfm * H1.nfm;
  const cf_problem* probs[2] = {prob1, prob2};
  const double* maps[2] = {maps1, maps2};
  Sizer z;
  for (int a = 0; a < 2; ++a) {
    size_staging(z, probs[a], H1);
    fisher_ws(H1, B, z, 0, nmaps);
    z.add<double>((size_t)nmaps * H1.n);        // maps copy (host inputs)
    z.add<double>((size_t)H1.n * nmaps);        // D
    z.add<double>((size_t)H1.n * nmaps);        // U
    z.add<double>((size_t)H1.k * nmaps);        // w
    z.add<double>((size_t)32 * H1.k * nmaps);   // partial sums
  }
  z.add<double>((size_t)nl * (nl + 1) / 2 * np * np);   // cross Gram
  z.add<double>((size_t)K * K);                         // W
  z.add<double>((size_t)K * K);                         // W copy for the solve
  z.add<double>((size_t)nmaps * K);                     // q
  z.add<double>((size_t)nmaps * K);                     // chat
  if (int st = ensure_ws(*c.dev, z.off)) return st;
  Bump bp(c.dev->ws);
  Staged S[2];
  FisherBufs f[2];
  QmlBufs qb[2];
  Timer tm;
  tm.begin(ex && ex->stage_timing, c.s);
  for (int a = 0; a < 2; ++a) {
    if (int st = stage(bp, probs[a], H1, nullptr, c.s, S[a])) return st;
    fisher_take(bp, H1, B, f[a], 0, nmaps);
    double* mcopy = bp.take<double>((size_t)nmaps * H1.n);
    qb[a].D = bp.take<double>((size_t)H1.n * nmaps);
    qb[a].U = bp.take<double>((size_t)H1.n * nmaps);
    qb[a].W = bp.take<double>((size_t)H1.k * nmaps);
    qb[a].part = bp.take<double>((size_t)32 * H1.k * nmaps);
    qb[a].nmaps = nmaps;
    qb[a].maps = maps[a];
    if (prob1->mem == CF_MEM_HOST) {
      CF_DEV(hipMemcpyAsync(mcopy, maps[a], sizeof(double) * nmaps * H1.n, hipMemcpyHostToDevice, c.s));
      qb[a].maps = mcopy;
    }
    CF_DEV(hipMemcpyAsync(f[a].lo, B.lo.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, c.s));
    CF_DEV(hipMemcpyAsync(f[a].hi, B.hi.data(), sizeof(int) * B.nb, hipMemcpyHostToDevice, c.s));
    if (int st = fisher_core(probs[a], H1, S[a], f[a], &qb[a], c, tm, 0)) return st;
  }
  double* gx = bp.take<double>((size_t)nl * (nl + 1) / 2 * np * np);
  double* W = bp.take<double>((size_t)K * K);
  double* Ww = bp.take<double>((size_t)K * K);
  double* q = bp.take<double>((size_t)nmaps * K);
  double* chat = bp.take<double>((size_t)nmaps * K);
  // W^x_AB = 1/2 tr[C1^-1 P_A C2^-1 P_B] from <Z2, Z1> block products; q^x = 1/2 w1^T E_A w2
  CF_DEV(launch_gram_cross(S[0].P, f[0].Z, f[1].Z, H1.k, gx, c.s));
  const SpecSel sel = make_sel(B, f[0]);
  CF_DEV(launch_fisher_assemble(S[0].P, sel, gx, W, c.s, true));
  tm.mark(ST_REDUCE);
  CF_DEV(launch_quad_assemble(S[0].P, sel, qb[0].W, nmaps, nmaps, q, c.s, qb[1].W));
  CF_DEV(hipMemcpyAsync(Ww, W, sizeof(double) * K * K, hipMemcpyDeviceToDevice, c.s));
  CF_DEV(launch_small_spd_solve(Ww, K, q, chat, nmaps, f[0].flags + 2, c.s));
  tm.mark(ST_QML);
  for (int a = 0; a < 2; ++a)
    if (int st = check_factor_flags(c, f[a], rep)) return st;
  {
    int fl3[3];
    if (int st = read_flags(c, f[0].flags, 3, fl3)) return st;
    if (fl3[2] != INT_MAX) {
      if (rep) rep->fail_index = fl3[2];
      return fail(CF_ENOTPD, "mode-mixing matrix not positive definite at pivot %d", fl3[2]);
    }
  }
  if (int st = copy_out(q_out, q, (size_t)nmaps * K, prob1->mem, c.s)) return st;
  if (int st = copy_out(chat_out, chat, (size_t)nmaps * K, prob1->mem, c.s)) return st;
  if (W_out)
    if (int st = copy_out(W_out, W, (size_t)K * K, prob1->mem, c.s)) return st;
  CF_DEV(hipStreamSynchronize(c.s));
  tm.finish(rep);
  if (rep) { rep->n = H1.n; rep->nmodes = H1.k; rep->flops = 2.0 * fisher_flops(H1); }
  return CF_OK;
}

namespace cf {
namespace {
// Nearest positive semi-definite matrix (Frobenius) of a symmetric m x m matrix, m <= 3: cyclic
// Jacobi eigendecomposition, negative eigenvalues set to zero; left as it is when none is negative.
void psd_project(double A[3][3], int m) {
  double a[3][3], v[3][3];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      a[i][j] = A[i][j];
      v[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < m; ++i) {
      dia += a[i][i] * a[i][i];
      for (int j = i + 1; j < m; ++j) off += a[i][j] * a[i][j];
    }
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        if (a[p][q] == 0.0) continue;
        const double tau = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < m; ++k) {   // columns p, q
          const double x = a[k][p], y = a[k][q];
          a[k][p] = c * x - s * y;
          a[k][q] = s * x + c * y;
        }
        for (int k = 0; k < m; ++k) {   // rows p, q
          const double x = a[p][k], y = a[q][k];
          a[p][k] = c * x - s * y;
          a[q][k] = s * x + c * y;
        }
        for (int k = 0; k < m; ++k) {
          const double x = v[k][p], y = v[k][q];
          v[k][p] = c * x - s * y;
          v[k][q] = s * x + c * y;
        }
      }
  }
  bool neg = false;
  for (int i = 0; i < m; ++i) neg = neg || a[i][i] < 0.0;
  if (!neg) return;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += v[i][k] * std::fmax(a[k][k], 0.0) * v[j][k];
      A[i][j] = s;
    }
}

// Next fiducial of iterative QML: every estimated band as a flat band over its multipoles, then the
// spectrum matrix over the harmonic fields at every multipole projected onto the positive
// semi-definite matrices.  cl: [6][L] in TT, EE, BB, TE, TB, EB order.
void band_fiducial(std::vector<double>& cl, int L, const HostBins& B, const HostProblem& H,
                   const std::vector<double>& chat) {
  for (int si = 0; si < B.ns; ++si)
    for (int b = 0; b < B.nb; ++b)
      for (int l = B.lo[b]; l <= B.hi[b]; ++l) cl[(size_t)B.spec[si] * L + l] = chat[(size_t)si * B.nb + b];
  int fld[3], m = 0;          // harmonic fields T 0, E 1, B 2
  if (H.has_t) fld[m++] = 0;
  if (H.has_p) { fld[m++] = 1; fld[m++] = 2; }
  auto row = [](int a, int b) {
    if (a > b) { const int t = a; a = b; b = t; }
    if (a == b) return a;
    return a == 0 ? (b == 1 ? 3 : 4) : 5;
  };
  for (int l = 0; l < L; ++l) {
    double M[3][3];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) M[i][j] = cl[(size_t)row(fld[i], fld[j]) * L + l];
    psd_project(M, m);
    for (int i = 0; i < m; ++i)
      for (int j = i; j < m; ++j) cl[(size_t)row(fld[i], fld[j]) * L + l] = M[i][j];
  }
}

// sqrt((F^-1)_bb) for a symmetric positive definite K x K F (row-major), by Cholesky.
bool fisher_errors(const std::vector<double>& F, int K, std::vector<double>& sig) {
  std::vector<double> Lc((size_t)K * K, 0.0);
  for (int j = 0; j < K; ++j) {
    double d = F[(size_t)j * K + j];
    for (int k = 0; k < j; ++k) d -= Lc[(size_t)j * K + k] * Lc[(size_t)j * K + k];
    if (!(d > 0.0)) return false;
    const double r = std::sqrt(d);
    Lc[(size_t)j * K + j] = r;
    for (int i = j + 1; i < K; ++i) {
      double t = F[(size_t)i * K + j];
      for (int k = 0; k < j; ++k) t -= Lc[(size_t)i * K + k] * Lc[(size_t)j * K + k];
      Lc[(size_t)i * K + j] = t / r;
    }
  }
  // (F^-1)_bb = |L^-1 e_b|^2
  std::vector<double> x(K);
  sig.assign(K, 0.0);
  for (int b = 0; b < K; ++b) {
    double s2 = 0.0;
    for (int i = 0; i < K; ++i) {
      double t = i == b ? 1.0 : 0.0;
      for (int k = b; k < i; ++k) t -= Lc[(size_t)i * K + k] * x[k];
      x[i] = i < b ? 0.0 : t / Lc[(size_t)i * K + i];
      s2 += x[i] * x[i];
    }
    sig[b] = std::sqrt(s2);
  }
  return true;
}

struct DevArray {
  double* p = nullptr;
  ~DevArray() { if (p) (void)hipFree(p); }
};
}  // namespace
}  // namespace cf

extern "C" int cf_qml_iterate(const cf_problem* prob, const cf_bins* bins, const double* map, int32_t max_iter,
                              double tol, double* chat_out, double* F_out, double* cl_out, int32_t* iters_out,
                              const cf_exec* ex, cf_report* rep) {
  report_init(rep);
  HostProblem H;
  if (int st = check_problem(prob, H, true)) return st;
  HostBins B;
  if (int st = check_bins(bins, H, B)) return st;
  if (!map || !chat_out) return fail(CF_EINVAL, "map and chat_out are required");
  if (max_iter < 1 || !(tol > 0.0) || !std::isfinite(tol)) return fail(CF_EINVAL, "max_iter=%d, tol=%g", max_iter, tol);
  const int K = B.ns * B.nb, L = H.lmax + 1;
  std::vector<double> cl(prob->cl, prob->cl + 6 * (size_t)L);
  cf_problem P = *prob;
  P.cl = cl.data();
  const bool dev = prob->mem == CF_MEM_DEVICE;
  std::vector<double> hbuf((size_t)3 * K + (size_t)K * K);
  DevArray dbuf;
  if (dev) CF_DEV(hipMalloc(&dbuf.p, sizeof(double) * hbuf.size()));
  double* base = dev ? dbuf.p : hbuf.data();
  double *y = base, *b = base + K, *c = base + 2 * K, *F = base + 3 * K;
  std::vector<double> chat(K), prev(K), Fh((size_t)K * K), sig;
  double flops = 0.0, ms = 0.0;
  for (int it = 1; it <= max_iter; ++it) {
    cf_report r;
    if (int st = cf_qml(&P, bins, map, 1, CF_FP64, y, b, c, F, ex, &r)) {
      if (rep) rep->fail_index = r.fail_index;
      return st;
    }
    flops += r.flops;
    ms += r.ms_total;
    if (dev) {
      CF_DEV(hipMemcpy(chat.data(), c, sizeof(double) * K, hipMemcpyDeviceToHost));
      CF_DEV(hipMemcpy(Fh.data(), F, sizeof(double) * K * K, hipMemcpyDeviceToHost));
    } else {
      std::copy(c, c + K, chat.begin());
      std::copy(F, F + (size_t)K * K, Fh.begin());
    }
    if (it > 1) {
      if (!fisher_errors(Fh, K, sig)) return fail(CF_ENOTPD, "Fisher matrix not positive definite at iteration %d", it);
      double worst = 0.0;
      for (int k = 0; k < K; ++k) worst = std::fmax(worst, std::fabs(chat[k] - prev[k]) / sig[k]);
      if (worst < tol) {
        if (dev) {
          CF_DEV(hipMemcpy(chat_out, c, sizeof(double) * K, hipMemcpyDeviceToDevice));
          if (F_out) CF_DEV(hipMemcpy(F_out, F, sizeof(double) * K * K, hipMemcpyDeviceToDevice));
        } else {
          std::copy(chat.begin(), chat.end(), chat_out);
          if (F_out) std::copy(Fh.begin(), Fh.end(), F_out);
        }
        if (cl_out) std::copy(cl.begin(), cl.end(), cl_out);
        if (iters_out) *iters_out = it;
        if (rep) { rep->n = H.n; rep->nmodes = H.k; rep->flops = flops; rep->ms_total = ms; rep->ir_iters = it; }
        return CF_OK;
      }
    }
    prev = chat;
    band_fiducial(cl, L, B, H, chat);
  }
  if (rep) rep->ir_iters = max_iter;
  return fail(CF_ENOCONV, "iterative QML did not settle within %d iterations (tolerance %g Fisher errors)",
              max_iter, tol);
}
