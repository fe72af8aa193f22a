// C ABI of the multiple-shooting objective/gradient library: validation,
// system build (host, FP64, once per context), device buffers, and the kernel
// sequences of qoc_kernels.hip.
#include "../../include/qoc.h"
#include "qoc_internal.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_last_error = "no error";

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(QOC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_RETURN(expr)                          \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Largest eigenvalue of the symmetric tridiagonal matrix with zero diagonal and
// squared off-diagonal entries e2[0..n-2], by Sturm-sequence bisection (an upper
// bound to bisection accuracy).
double tridiag_max_eig(const std::vector<double> &e2) {
  const int n = (int)e2.size() + 1;
  auto count_below = [&](double x) {
    int cnt = 0;
    double d = -x;
    for (int i = 0; i < n; ++i) {
      if (i > 0) d = -x - e2[i - 1] / (d == 0.0 ? 1e-300 : d);
      if (d < 0) ++cnt;
    }
    return cnt;
  };
  double hi = 1.0;
  for (double v : e2) hi += 2.0 * std::sqrt(v);
  double lo = 0.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) == n) hi = mid; else lo = mid;
  }
  return hi;
}

// ||a + a^+||_2 on L levels: off-diagonal entries sqrt(1..L-1).
double ladder_norm(int L) {
  std::vector<double> e2;
  for (int i = 1; i < L; ++i) e2.push_back((double)i);
  return tridiag_max_eig(e2);
}

// ||b^+ a + b a^+||_2 on two L-level systems.  The operator keeps n = l_a + l_b; on
// each sector it is tridiagonal in l_a with entries sqrt(l_a) sqrt(n - l_a + 1).
double exchange_norm(int L) {
  double best = 0.0;
  for (int n = 1; n <= 2 * (L - 1); ++n) {
    const int k0 = std::max(0, n - (L - 1)), k1 = std::min(n, L - 1);
    if (k1 <= k0) continue;
    std::vector<double> e2;
    for (int k = k0 + 1; k <= k1; ++k) e2.push_back((double)k * (double)(n - k + 1));
    best = std::max(best, tridiag_max_eig(e2));
  }
  return best;
}

}  // namespace

struct qoc_ctx {
  int q = 0, L = 0, N = 0, E = 0, nf = 0, d1 = 0, M = 0, d = 0;
  long long NT = 0;
  int device = 0;
  int fp64 = 0;
  int shape = 0;                                   // kernel-instance index of (q, L)
  hipStream_t stream = nullptr;
  bool have_alpha = false, have_W = false;
  bool forward_valid = false;                      // forward sweep matches the current inputs
  bool grad_valid = false;                         // internal gradient buffers hold the last gradient
  size_t bytes = 0;
  std::vector<void *> allocs;
  double *roll_W = nullptr, *roll_U = nullptr;   // staging for host roll-out outputs
  qoc::DevSys dev{};
  // timing: per recorded evaluation, events at the phase boundaries
  static constexpr int kTimedCalls = 4096;
  bool timing = false;
  std::vector<hipEvent_t> events;                  // kTimedCalls * (N_PHASES + 1)
  std::vector<char> call_ph0, call_ph1;           // phases [ph0, ph1) run by each recorded call
  int n_timed = 0;

  template <typename P>
  int alloc(P **p, size_t bytes_) {
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, std::max<size_t>(bytes_, 16));
    if (e != hipSuccess) return fail(QOC_ENOMEM, std::string("hipMalloc of ") + std::to_string(bytes_) + " bytes failed");
    allocs.push_back(v);
    bytes += bytes_;
    *p = reinterpret_cast<P *>(v);
    return QOC_OK;
  }
  ~qoc_ctx() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (void *p : allocs) (void)hipFree(p);
  }
  hipEvent_t ev(int call, int k) { return events[(size_t)call * (qoc::N_PHASES + 1) + k]; }
};

namespace qoc {
const DevSys &ctx_dev(const qoc_ctx *ctx) { return ctx->dev; }
hipStream_t ctx_stream(const qoc_ctx *ctx) { return ctx->stream; }
int ctx_device(const qoc_ctx *ctx) { return ctx->device; }
int set_error(int code, const char *msg) { return fail(code, msg); }
}  // namespace qoc

extern "C" {

const char *qoc_last_error(void) { return g_last_error.c_str(); }

const char *qoc_strerror(int code) {
  switch (code) {
    case QOC_OK: return "ok";
    case QOC_EINVAL: return "invalid argument";
    case QOC_ENOMEM: return "out of device memory";
    case QOC_EDEVICE: return "HIP device error";
    case QOC_ENOTCONV: return "fixed-point solve bound not met";
    case QOC_EUNSUPPORTED: return "unsupported (qubits, levels) pair";
    case QOC_ESTATE: return "call out of order";
    default: return "unknown error";
  }
}

int qoc_create(const qoc_system_desc *desc, qoc_ctx **out) {
  if (!desc || !out) return fail(QOC_EINVAL, "qoc_create: NULL argument");
  *out = nullptr;
  const qoc_system_desc &D = *desc;
  if (D.n_qubits < 1 || D.n_qubits > 6) return fail(QOC_EINVAL, "n_qubits must be in 1..6");
  if (D.n_levels < 2 || D.n_levels > 8) return fail(QOC_EINVAL, "n_levels must be in 2..8");
  if (D.n_carriers < 1 || D.n_splines < 3) return fail(QOC_EINVAL, "need n_carriers >= 1 and n_splines >= 3");
  if (!(D.T > 0.0) || !std::isfinite(D.T)) return fail(QOC_EINVAL, "T must be finite and > 0");
  if (D.n_windows < 1 || D.n_steps < D.n_windows) return fail(QOC_EINVAL, "need 1 <= n_windows <= n_steps");
  if (!(D.mu >= 0.0) || !std::isfinite(D.mu)) return fail(QOC_EINVAL, "mu must be finite and >= 0");
  if (D.precision != QOC_FP64 && D.precision != QOC_FP32) return fail(QOC_EINVAL, "precision must be QOC_FP64 or QOC_FP32");
  if (D.fixed_point_iters < 0 || D.fixed_point_iters > 64) return fail(QOC_EINVAL, "fixed_point_iters must be in 0..64");
  if (D.checkpoint_every < 0) return fail(QOC_EINVAL, "checkpoint_every must be >= 0");
  if (!(D.solve_tol >= 0.0) || !std::isfinite(D.solve_tol)) return fail(QOC_EINVAL, "solve_tol must be finite and >= 0");
  if (!D.detuning || !D.anharmonicity || !D.carrier_freq || !D.target) return fail(QOC_EINVAL, "NULL system array");

  const int q = D.n_qubits, L = D.n_levels;
  long long N = 1;
  for (int j = 0; j < q; ++j) N *= L;
  const int E = 1 << q;
  const int nf = D.n_carriers, d1 = D.n_splines, M = D.n_windows;
  const long long NT = D.n_steps;
  if (!finite_all(D.detuning, q) || !finite_all(D.anharmonicity, q) || (D.cross_kerr && !finite_all(D.cross_kerr, q - 1)) ||
      (D.dipole && !finite_all(D.dipole, q - 1)) ||
      !finite_all(D.carrier_freq, (size_t)q * nf) || !finite_all(D.target, 2 * (size_t)E * E))
    return fail(QOC_EINVAL, "non-finite system parameter");
  // the target must be unitary (eq. mod-infid assumes V^+ V = I)
  {
    double worst = 0.0;
    for (int a = 0; a < E; ++a)
      for (int b = 0; b < E; ++b) {
        std::complex<double> acc = 0.0;
        for (int r = 0; r < E; ++r)
          acc += std::conj(std::complex<double>(D.target[2 * (a * E + r)], D.target[2 * (a * E + r) + 1])) *
                 std::complex<double>(D.target[2 * (b * E + r)], D.target[2 * (b * E + r) + 1]);
        worst = std::max(worst, std::abs(acc - (a == b ? 1.0 : 0.0)));
      }
    if (worst > 1e-10) return fail(QOC_EINVAL, "target is not unitary");
  }
  const int fp64 = D.precision == QOC_FP64;
  int hop = 0;
  if (D.dipole)
    for (int j = 0; j + 1 < q; ++j) hop |= D.dipole[j] != 0.0;
  int ld = 0, cpw = 1;
  int shape = 0;
  if (!qoc::layout_for(q, L, fp64, hop, &ld, &cpw, &shape))
    return fail(QOC_EUNSUPPORTED, "no kernel instance for q=" + std::to_string(q) + " L=" + std::to_string(L));

  HIP_OR_RETURN(hipSetDevice(D.device));
  qoc_ctx *c = new qoc_ctx();
  c->q = q; c->L = L; c->N = (int)N; c->E = E; c->nf = nf; c->d1 = d1; c->M = M;
  c->d = 2 * d1 * q * nf; c->NT = NT; c->device = D.device; c->fp64 = fp64; c->shape = shape;

  // ---- host system build (FP64)
  const double dt = D.T / (double)NT;
  std::vector<long long> kstart(M + 1);
  for (int m = 0; m <= M; ++m) kstart[m] = (long long)(((__int128)m * NT) / M);
  long long maxlen = 0;
  for (int m = 0; m < M; ++m) maxlen = std::max(maxlen, kstart[m + 1] - kstart[m]);
  std::vector<double> dinv(2 * N);
  std::vector<long long> stride(q);
  for (int j = 0; j < q; ++j) { stride[j] = 1; for (int k = j + 1; k < q; ++k) stride[j] *= L; }
  for (long long r = 0; r < N; ++r) {
    double h = 0.0;
    std::vector<int> l(q);
    for (int j = 0; j < q; ++j) l[j] = (int)((r / stride[j]) % L);
    for (int j = 0; j < q; ++j) h += D.detuning[j] * l[j] + 0.5 * D.anharmonicity[j] * l[j] * (l[j] - 1);
    if (D.cross_kerr)
      for (int j = 0; j + 1 < q; ++j) h += D.cross_kerr[j] * l[j] * l[j + 1];
    const std::complex<double> di = 1.0 / std::complex<double>(1.0, 0.5 * dt * h);
    dinv[2 * r] = di.real();
    dinv[2 * r + 1] = di.imag();
  }
  std::vector<int> ess(E);
  for (int e = 0; e < E; ++e) {
    long long r = 0;
    for (int j = 0; j < q; ++j) r += (long long)((e >> (q - 1 - j)) & 1) * stride[j];
    ess[e] = (int)r;
  }
  std::vector<double> Vemb(2 * (size_t)N * E, 0.0);
  for (int col = 0; col < E; ++col)
    for (int e = 0; e < E; ++e) {
      Vemb[2 * ((size_t)col * N + ess[e])] = D.target[2 * (col * E + e)];
      Vemb[2 * ((size_t)col * N + ess[e]) + 1] = D.target[2 * (col * E + e) + 1];
    }

  qoc::DevSys &s = c->dev;
  s.q = q; s.L = L; s.N = (int)N; s.E = E; s.nf = nf; s.d1 = d1; s.M = M; s.NT = NT;
  s.T = D.T; s.dt = dt; s.dtau = D.T / (double)(d1 - 2); s.mu = D.mu;
  s.nu_L = ladder_norm(L);
  s.hop = hop;
  s.beta = 0.0;
  for (int j = 0; j < 8; ++j) s.hop_c[j] = 0.0;
  if (hop) {
    const double nx = exchange_norm(L);
    for (int j = 0; j + 1 < q; ++j) {
      s.hop_c[j] = 0.5 * dt * D.dipole[j];
      s.beta += std::fabs(s.hop_c[j]) * nx;
    }
  }
  s.fp64 = fp64; s.ld = ld; s.cpw = cpw; s.ncg = (E + cpw - 1) / cpw; s.maxlen = maxlen;
  // layouts with at least two columns per wavefront split the backward sweep's state and
  // adjoint over the two halves of a wavefront: cpw/2 columns per backward wavefront
  s.ncg_b = cpw >= 2 ? (E + cpw / 2 - 1) / (cpw / 2) : s.ncg;
  s.ckpt_every = (D.checkpoint_every > 0 && D.checkpoint_every < maxlen) ? D.checkpoint_every : 0;
  s.ncp = s.ckpt_every ? (int)((maxlen - 1) / s.ckpt_every) : 0;
  s.kit_fixed = D.fixed_point_iters;
  s.solve_tol = D.solve_tol > 0.0 ? D.solve_tol : (fp64 ? std::ldexp(1.0, -54) : std::ldexp(1.0, -26));

  const size_t tsz = fp64 ? sizeof(double) : sizeof(float);
  const size_t nst = (size_t)M * E * N;           // complex entries of all window states
  int rc = QOC_OK;
  long long *kst = nullptr;
  double *car = nullptr, *dv = nullptr, *Vd = nullptr;
  int *essd = nullptr;
#define ALLOC(ptr, bytes_) if (rc == QOC_OK) rc = c->alloc(&(ptr), (bytes_))
  ALLOC(kst, sizeof(long long) * (M + 1));
  ALLOC(car, sizeof(double) * q * nf);
  ALLOC(dv, sizeof(double) * 2 * N);
  ALLOC(essd, sizeof(int) * E);
  ALLOC(Vd, sizeof(double) * 2 * N * E);
  double *alpha = nullptr, *W = nullptr;
  ALLOC(alpha, sizeof(double) * c->d);
  ALLOC(W, sizeof(double) * 2 * (size_t)(M - 1) * E * N);
  ALLOC(s.ctrl, tsz * 2 * (size_t)NT * q);
  ALLOC(s.Ufin, sizeof(double) * 2 * nst);
  ALLOC(s.lam0, sizeof(double) * 2 * nst);
  ALLOC(s.ckpt, sizeof(double) * 2 * nst * s.ncp);
  ALLOC(s.partials, sizeof(double) * 4 * M);
  ALLOC(s.scal, sizeof(double) * (5 + M));
  ALLOC(s.series, tsz * (size_t)M * s.ncg_b * maxlen * 2 * q);
  ALLOC(s.xy, sizeof(double) * (size_t)NT * 2 * q);
  ALLOC(s.grad_alpha, sizeof(double) * c->d);
  ALLOC(s.grad_W, sizeof(double) * 2 * (size_t)(M - 1) * E * N);
  ALLOC(s.kit, sizeof(int) * 2);
  ALLOC(s.rho_bits, sizeof(unsigned int) * 2);
  ALLOC(s.status, sizeof(int) * 2);
#undef ALLOC
  if (rc != QOC_OK) { delete c; return rc; }
  s.kstart = kst; s.carrier = car; s.dinv = dv; s.ess_row = essd; s.V = Vd; s.alpha = alpha; s.W = W;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(kst, kstart.data(), sizeof(long long) * (M + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(car, D.carrier_freq, sizeof(double) * q * nf, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dv, dinv.data(), sizeof(double) * 2 * N, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(essd, ess.data(), sizeof(int) * E, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(Vd, Vemb.data(), sizeof(double) * Vemb.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(s.status, 0, sizeof(int) * 2);
  if (e == hipSuccess) e = hipMemset(s.kit, 0, sizeof(int) * 2);
  if (e == hipSuccess) e = hipMemset(s.rho_bits, 0, sizeof(unsigned int) * 2);
  if (e != hipSuccess) { delete c; return hip_fail(e, "qoc_create upload"); }
  *out = c;
  return QOC_OK;
}

int qoc_destroy(qoc_ctx *ctx) {
  if (!ctx) return QOC_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return QOC_OK;
}

int qoc_get_info(const qoc_ctx *ctx, qoc_info *out) {
  if (!ctx || !out) return fail(QOC_EINVAL, "qoc_get_info: NULL argument");
  out->N = ctx->N; out->E = ctx->E; out->d = ctx->d; out->n_windows = ctx->M;
  out->n_window_doubles = 2LL * (ctx->M - 1) * ctx->N * ctx->E;
  out->n_terms = 4 + ctx->M;
  out->lane_digits = ctx->dev.ld;
  out->columns_per_wave = ctx->dev.cpw;
  out->device_bytes = (int64_t)ctx->bytes;
  return QOC_OK;
}

int qoc_set_stream(qoc_ctx *ctx, void *hip_stream) {
  if (!ctx) return fail(QOC_EINVAL, "qoc_set_stream: NULL context");
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return QOC_OK;
}

int qoc_set_schedule(qoc_ctx *ctx, int32_t backward) {
  if (!ctx) return fail(QOC_EINVAL, "qoc_set_schedule: NULL context");
  if (backward != QOC_BWD_AUTO && backward != QOC_BWD_ONE_WAVE && backward != QOC_BWD_TWO_WAVES &&
      backward != QOC_BWD_THREE_WAVES)
    return fail(QOC_EINVAL, "qoc_set_schedule: unknown backward schedule " + std::to_string(backward));
  if (backward == QOC_BWD_THREE_WAVES && ctx->dev.cpw != 1)
    return fail(QOC_EUNSUPPORTED, "qoc_set_schedule: a backward of three wavefronts needs a "
                                  "one-column-per-wavefront layout");
  ctx->dev.bwd_sched = backward;
  return QOC_OK;
}

int qoc_get_schedule(const qoc_ctx *ctx, int32_t *backward) {
  if (!ctx || !backward) return fail(QOC_EINVAL, "qoc_get_schedule: NULL argument");
  const int waves = qoc::bwd_waves(ctx->dev);
  *backward = waves == 3 ? QOC_BWD_THREE_WAVES : waves == 2 ? QOC_BWD_TWO_WAVES : QOC_BWD_ONE_WAVE;
  return QOC_OK;
}

static hipMemcpyKind kind_in(int32_t where) { return where == QOC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
static hipMemcpyKind kind_out(int32_t where) { return where == QOC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

int qoc_set_controls(qoc_ctx *ctx, const double *alpha, int64_t d, int32_t where) {
  if (!ctx || !alpha) return fail(QOC_EINVAL, "qoc_set_controls: NULL argument");
  if (d != ctx->d) return fail(QOC_EINVAL, "qoc_set_controls: expected d = " + std::to_string(ctx->d));
  if (where != QOC_HOST && where != QOC_DEVICE) return fail(QOC_EINVAL, "qoc_set_controls: bad memory kind");
  if (where == QOC_HOST && !finite_all(alpha, (size_t)d)) return fail(QOC_EINVAL, "qoc_set_controls: non-finite alpha");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  HIP_OR_RETURN(hipMemcpyAsync(const_cast<double *>(ctx->dev.alpha), alpha, sizeof(double) * d, kind_in(where), ctx->stream));
  ctx->have_alpha = true;
  ctx->forward_valid = false;
  ctx->grad_valid = false;
  return QOC_OK;
}

int qoc_set_window_states(qoc_ctx *ctx, const double *W, int64_t n_doubles, int32_t where) {
  if (!ctx) return fail(QOC_EINVAL, "qoc_set_window_states: NULL context");
  const int64_t need = 2LL * (ctx->M - 1) * ctx->N * ctx->E;
  if (n_doubles != need) return fail(QOC_EINVAL, "qoc_set_window_states: expected " + std::to_string(need) + " doubles");
  if (where != QOC_HOST && where != QOC_DEVICE) return fail(QOC_EINVAL, "qoc_set_window_states: bad memory kind");
  if (need == 0) { ctx->have_W = true; return QOC_OK; }
  if (!W) return fail(QOC_EINVAL, "qoc_set_window_states: NULL W");
  if (where == QOC_HOST && !finite_all(W, (size_t)need)) return fail(QOC_EINVAL, "qoc_set_window_states: non-finite W");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  HIP_OR_RETURN(hipMemcpyAsync(const_cast<double *>(ctx->dev.W), W, sizeof(double) * need, kind_in(where), ctx->stream));
  ctx->have_W = true;
  ctx->forward_valid = false;
  ctx->grad_valid = false;
  return QOC_OK;
}

static int check_status(qoc_ctx *ctx) {
  int st[2] = {0, 0};
  HIP_OR_RETURN(hipMemcpyAsync(st, ctx->dev.status, sizeof(int) * 2, hipMemcpyDeviceToHost, ctx->stream));
  HIP_OR_RETURN(hipStreamSynchronize(ctx->stream));
  if (st[0] & qoc::STATUS_NOTCONV) {
    HIP_OR_RETURN(hipMemsetAsync(ctx->dev.status, 0, sizeof(int) * 2, ctx->stream));
    HIP_OR_RETURN(hipStreamSynchronize(ctx->stream));
    return fail(QOC_ENOTCONV, "fixed-point contraction bound exceeded the solve tolerance (controls too large for dt)");
  }
  return QOC_OK;
}

// Phases [ph0, ph1) of one evaluation (objective: 0..3, gradient: 0..6, backward only: 3..6).
static int run(qoc_ctx *ctx, int ph0, int ph1, double *P, double *terms, double *ga, double *gW, int32_t where) {
  const bool grad = ph1 > qoc::PHASE_BOUNDARY + 1;
  if (!ctx) return fail(QOC_EINVAL, "NULL context");
  if (where != QOC_HOST && where != QOC_DEVICE) return fail(QOC_EINVAL, "bad memory kind");
  if (!ctx->have_alpha) return fail(QOC_ESTATE, "controls not set");
  if (ctx->M > 1 && !ctx->have_W) return fail(QOC_ESTATE, "window states not set");
  if (ph0 > 0 && !ctx->forward_valid) return fail(QOC_ESTATE, "no objective evaluated for the current inputs");
  if (grad && !ga) return fail(QOC_EINVAL, "grad_alpha is NULL");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  qoc::DevSys s = ctx->dev;
  if (grad && where == QOC_DEVICE) {
    s.grad_alpha = ga;
    if (gW) s.grad_W = gW;
  }
  const bool timed = ctx->timing && ctx->n_timed < qoc_ctx::kTimedCalls;
  const int call = ctx->n_timed;
  if (timed) HIP_OR_RETURN(hipEventRecord(ctx->ev(call, ph0), ctx->stream));
  for (int ph = ph0; ph < ph1; ++ph) {
    int e = qoc::launch_phase(s, ph, ctx->stream);
    if (e) { ctx->forward_valid = false; return hip_fail((hipError_t)e, "kernel launch"); }
    if (timed) HIP_OR_RETURN(hipEventRecord(ctx->ev(call, ph + 1), ctx->stream));
  }
  if (ph0 == 0) ctx->forward_valid = true;
  ctx->grad_valid = grad && !(where == QOC_DEVICE);
  if (timed) {
    ctx->call_ph0[call] = (char)ph0;
    ctx->call_ph1[call] = (char)ph1;
    ctx->n_timed++;
  }
  const hipMemcpyKind k = kind_out(where);
  if (P) HIP_OR_RETURN(hipMemcpyAsync(P, s.scal, sizeof(double), k, ctx->stream));
  if (terms) HIP_OR_RETURN(hipMemcpyAsync(terms, s.scal + 1, sizeof(double) * (4 + ctx->M), k, ctx->stream));
  if (grad && where == QOC_HOST) {
    HIP_OR_RETURN(hipMemcpyAsync(ga, s.grad_alpha, sizeof(double) * ctx->d, k, ctx->stream));
    if (gW && ctx->M > 1)
      HIP_OR_RETURN(hipMemcpyAsync(gW, s.grad_W, sizeof(double) * 2 * (size_t)(ctx->M - 1) * ctx->E * ctx->N, k, ctx->stream));
  }
  if (where == QOC_HOST) return check_status(ctx);
  return QOC_OK;
}

int qoc_enable_timing(qoc_ctx *ctx, int32_t on) {
  if (!ctx) return fail(QOC_EINVAL, "qoc_enable_timing: NULL context");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  HIP_OR_RETURN(hipStreamSynchronize(ctx->stream));
  if (on && ctx->events.empty()) {
    ctx->events.resize((size_t)qoc_ctx::kTimedCalls * (qoc::N_PHASES + 1));
    for (auto &e : ctx->events) HIP_OR_RETURN(hipEventCreate(&e));
    ctx->call_ph0.assign(qoc_ctx::kTimedCalls, 0);
    ctx->call_ph1.assign(qoc_ctx::kTimedCalls, 0);
  }
  ctx->timing = on != 0;
  ctx->n_timed = 0;
  return QOC_OK;
}

int qoc_get_timings(qoc_ctx *ctx, qoc_timings *out) {
  if (!ctx || !out) return fail(QOC_EINVAL, "qoc_get_timings: NULL argument");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  HIP_OR_RETURN(hipStreamSynchronize(ctx->stream));
  std::memset(out, 0, sizeof *out);
  double sum[8] = {0};
  int cnt[8] = {0};
  int ngrad = 0;
  for (int c = 0; c < ctx->n_timed; ++c) {
    const int p0 = ctx->call_ph0[c], p1 = ctx->call_ph1[c];
    ngrad += p1 > qoc::PHASE_BOUNDARY + 1 ? 1 : 0;
    for (int ph = p0; ph < p1; ++ph) {
      float ms = 0.f;
      HIP_OR_RETURN(hipEventElapsedTime(&ms, ctx->ev(c, ph), ctx->ev(c, ph + 1)));
      sum[ph] += ms;
      cnt[ph]++;
    }
    float tot = 0.f;
    HIP_OR_RETURN(hipEventElapsedTime(&tot, ctx->ev(c, p0), ctx->ev(c, p1)));
    sum[6] += tot;
    cnt[6]++;
  }
  out->n_calls = ctx->n_timed;
  out->n_grad_calls = ngrad;
  for (int ph = 0; ph < 7; ++ph) out->mean_ms[ph] = cnt[ph] ? sum[ph] / cnt[ph] : 0.0;
  int kit = 0;
  if (ctx->dev.kit_fixed > 0) kit = ctx->dev.kit_fixed;
  else HIP_OR_RETURN(hipMemcpy(&kit, ctx->dev.kit, sizeof(int), hipMemcpyDeviceToHost));
  out->fixed_point_iters = kit;
  return QOC_OK;
}

int qoc_objective(qoc_ctx *ctx, double *P, double *terms, int32_t where) {
  if (!P) return fail(QOC_EINVAL, "qoc_objective: NULL P");
  return run(ctx, 0, qoc::PHASE_BOUNDARY + 1, P, terms, nullptr, nullptr, where);
}

int qoc_gradient(qoc_ctx *ctx, double *P, double *terms, double *grad_alpha, double *grad_W, int32_t where) {
  return run(ctx, 0, qoc::PHASE_GRAD_W + 1, P, terms, grad_alpha, grad_W, where);
}

int qoc_backward(qoc_ctx *ctx, double *grad_alpha, double *grad_W, int32_t where) {
  return run(ctx, qoc::PHASE_BACKWARD, qoc::PHASE_GRAD_W + 1, nullptr, nullptr, grad_alpha, grad_W, where);
}

int qoc_rollout(qoc_ctx *ctx, double *W_out, double *U_out, int32_t where) {
  if (!ctx) return fail(QOC_EINVAL, "qoc_rollout: NULL context");
  if (where != QOC_HOST && where != QOC_DEVICE) return fail(QOC_EINVAL, "qoc_rollout: bad memory kind");
  if (!ctx->have_alpha) return fail(QOC_ESTATE, "controls not set");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  const size_t nW = 2 * (size_t)(ctx->M - 1) * ctx->E * ctx->N, nU = 2 * (size_t)ctx->E * ctx->N;
  double *wd = W_out, *ud = U_out;
  if (where == QOC_HOST) {
    if (!ctx->roll_W) {
      int rc = ctx->alloc(&ctx->roll_W, sizeof(double) * std::max<size_t>(nW, 2));
      if (rc == QOC_OK) rc = ctx->alloc(&ctx->roll_U, sizeof(double) * nU);
      if (rc != QOC_OK) return rc;
    }
    wd = ctx->roll_W;
    ud = ctx->roll_U;
  }
  if (!wd) {
    if (!ctx->roll_W) {
      int rc = ctx->alloc(&ctx->roll_W, sizeof(double) * std::max<size_t>(nW, 2));
      if (rc == QOC_OK) rc = ctx->alloc(&ctx->roll_U, sizeof(double) * nU);
      if (rc != QOC_OK) return rc;
    }
    wd = ctx->roll_W;
  }
  int e = qoc::launch_phase(ctx->dev, qoc::PHASE_CONTROLS, ctx->stream);
  if (!e) e = qoc::launch_phase(ctx->dev, qoc::PHASE_ROLLOUT, ctx->stream, wd, ud);
  if (e) return hip_fail((hipError_t)e, "roll-out kernels");
  if (where == QOC_HOST) {
    if (W_out && nW) HIP_OR_RETURN(hipMemcpyAsync(W_out, wd, sizeof(double) * nW, hipMemcpyDeviceToHost, ctx->stream));
    if (U_out) HIP_OR_RETURN(hipMemcpyAsync(U_out, ud, sizeof(double) * nU, hipMemcpyDeviceToHost, ctx->stream));
    return check_status(ctx);
  }
  return QOC_OK;
}


// ---------------------------------------------------------------------------- batches

// Sections of the pinned staging buffer of a batch: the systems, then the propagation items
// (16-byte int4 records), then the small-kernel block table.  Each section starts on a 256-byte
// boundary: the item records must be 16-byte aligned (their stores are 16-byte vector stores),
// and sizeof(DevSys) times an odd context count is not a multiple of 16.
struct StageLayout {
  size_t items, blocks, total;
};
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static StageLayout stage_layout_records(int n_sys, long long n_records, long long n_blocks) {
  StageLayout l;
  l.items = align256(sizeof(qoc::DevSys) * (size_t)n_sys);
  l.blocks = l.items + align256(sizeof(int4) * (size_t)n_records);
  l.total = l.blocks + sizeof(int2) * (size_t)n_blocks;
  return l;
}
// a batch object's capacity: forward and backward items up to max_items each
static StageLayout stage_layout(int max_ctx, long long max_items, long long max_blocks) {
  return stage_layout_records(max_ctx, 2 * max_items, max_blocks);
}

struct qoc_batch {
  int device = 0;
  int max_ctx = 0;
  long long max_items = 0;
  long long max_blocks = 0;
  qoc::DevSys *d_sys = nullptr;
  int4 *d_items = nullptr;       // forward items then backward items
  int2 *d_blocks = nullptr;      // all small-kernel tables
  char *h_stage = nullptr;       // pinned staging for the uploads
  size_t stage_bytes = 0;
  hipEvent_t uploaded = nullptr; // staging may be rewritten once this has passed
  bool pending = false;
  hipStream_t aux = nullptr;      // backward items of two wavefronts run here (default priority)
  hipStream_t aux2 = nullptr;     // backward items of three wavefronts run here (default priority)
  hipEvent_t fork = nullptr, join = nullptr, join2 = nullptr;
  int *d_status = nullptr;        // [max_ctx] status words gathered at the end of a run
  int *h_status = nullptr;        // pinned host copy of d_status
  hipEvent_t done = nullptr;      // recorded after the status copy of the last run
  int last_n = 0;                 // contexts of the last run (0: none yet)
  ~qoc_batch() {
    if (done) { (void)hipEventSynchronize(done); (void)hipEventDestroy(done); }
    if (uploaded) { (void)hipEventSynchronize(uploaded); (void)hipEventDestroy(uploaded); }
    if (aux) { (void)hipStreamSynchronize(aux); (void)hipStreamDestroy(aux); }
    if (aux2) { (void)hipStreamSynchronize(aux2); (void)hipStreamDestroy(aux2); }
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (join2) (void)hipEventDestroy(join2);
    (void)hipFree(d_sys); (void)hipFree(d_items); (void)hipFree(d_blocks); (void)hipFree(d_status);
    (void)hipHostFree(h_stage); (void)hipHostFree(h_status);
  }
};

int qoc_batch_create(int32_t device, int32_t max_contexts, int64_t max_items, qoc_batch **out) {
  if (!out || max_contexts < 1 || max_items < 1) return fail(QOC_EINVAL, "qoc_batch_create: bad arguments");
  *out = nullptr;
  HIP_OR_RETURN(hipSetDevice(device));
  qoc_batch *b = new qoc_batch();
  b->device = device;
  b->max_ctx = max_contexts;
  b->max_items = max_items;
  b->max_blocks = 4 * max_items + 1024LL * max_contexts;   // generous: small kernels need few blocks per system
  b->stage_bytes = stage_layout(max_contexts, max_items, b->max_blocks).total;
  hipError_t e = hipMalloc(&b->d_sys, sizeof(qoc::DevSys) * max_contexts);
  if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(int4) * 2 * max_items);
  if (e == hipSuccess) e = hipMalloc(&b->d_blocks, sizeof(int2) * b->max_blocks);
  if (e == hipSuccess) e = hipHostMalloc(&b->h_stage, b->stage_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->aux2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join2, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&b->d_status, sizeof(int) * max_contexts);
  if (e == hipSuccess) e = hipHostMalloc(&b->h_status, sizeof(int) * max_contexts, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e != hipSuccess) { delete b; return fail(QOC_ENOMEM, std::string("qoc_batch_create: ") + hipGetErrorString(e)); }
  *out = b;
  return QOC_OK;
}

int qoc_batch_destroy(qoc_batch *b) {
  if (!b) return QOC_OK;
  (void)hipSetDevice(b->device);
  delete b;
  return QOC_OK;
}

// ---- pieces shared by the batched entry points

// The contexts of one batched call: non-NULL, on `device`, of one precision, with inputs,
// each listed once.  `who` names the entry point in messages.
static int batch_check(qoc_ctx *const *ctxs, int32_t n, int device, const char *who) {
  const int fp64 = ctxs[0] ? ctxs[0]->fp64 : 0;
  for (int i = 0; i < n; ++i) {
    qoc_ctx *c = ctxs[i];
    if (!c) return fail(QOC_EINVAL, std::string(who) + ": NULL context");
    if (c->device != device) return fail(QOC_EINVAL, std::string(who) + ": context on another device");
    if (c->fp64 != fp64) return fail(QOC_EINVAL, std::string(who) + ": mixed precisions");
    if (!c->have_alpha || (c->M > 1 && !c->have_W)) return fail(QOC_ESTATE, std::string(who) + ": context without inputs");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(QOC_EINVAL, std::string(who) + ": context listed twice");
  }
  return QOC_OK;
}

// Propagation items of all contexts, longest first (cost ~ steps x entries per lane x qubits),
// in four sections by backward schedule, and the number of small-kernel blocks.  The records
// live in caller memory (the allocation-free call uses a static array): batch_counts sizes
// them, batch_fill writes and sorts them in place.  Equal costs keep their enumeration order,
// so both batched entry points launch the same item order.
struct ItemRec {
  long long cost, seq;
  int4 v;
};
struct BatchCounts {
  long long fwd = 0, bwd = 0, xw = 0, x3 = 0, nblocks = 0;
  bool any_grad = false;
  long long records() const { return fwd + bwd + xw + x3; }
};

static BatchCounts batch_counts(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad) {
  BatchCounts c;
  for (int i = 0; i < n; ++i) {
    const qoc_ctx *x = ctxs[i];
    const bool g = !want_grad || want_grad[i];
    c.any_grad |= g;
    c.fwd += (long long)x->M * x->dev.ncg;
    if (g) {
      const int waves = qoc::bwd_waves(x->dev);
      (waves == 3 ? c.x3 : waves == 2 ? c.xw : c.bwd) += (long long)x->M * x->dev.ncg_b;
    }
    for (int k = 0; k < qoc::SK_COUNT; ++k) {
      const bool gk = k == qoc::SK_SERIES || k == qoc::SK_PROJECT || k == qoc::SK_GRADW;
      if (!gk || g) c.nblocks += qoc::small_blocks(x->dev, k);
    }
  }
  return c;
}

// rec: c.records() slots, sections forward | one wavefront | two | three.
static void batch_fill(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad, const BatchCounts &c,
                       ItemRec *rec) {
  long long pos[4] = {0, c.fwd, c.fwd + c.bwd, c.fwd + c.bwd + c.xw};
  const long long start[4] = {pos[0], pos[1], pos[2], pos[3]};
  long long seq = 0;
  for (int i = 0; i < n; ++i) {
    const qoc_ctx *x = ctxs[i];
    const bool g = !want_grad || want_grad[i];
    const long long per_lane = (long long)x->N / std::max(1, (64 / x->dev.cpw)) + 1;
    const int waves = qoc::bwd_waves(x->dev);                                        // wavefronts per item
    const int sec = waves == 3 ? 3 : waves == 2 ? 2 : 1;
    for (int m = 0; m < x->M; ++m) {
      // window length from the floor split
      const long long len =
          (long long)(((__int128)(m + 1) * x->NT) / x->M) - (long long)(((__int128)m * x->NT) / x->M);
      for (int cg = 0; cg < x->dev.ncg; ++cg)
        rec[pos[0]++] = ItemRec{len * per_lane * x->q, seq++, make_int4(i, m, cg, x->shape)};
      if (g) {
        const long long bcost = (x->dev.cpw >= 2 || waves > 1 ? 1 : 2) * len * per_lane * x->q;  // one system per lane
        for (int cg = 0; cg < x->dev.ncg_b; ++cg)
          rec[pos[sec]++] = ItemRec{bcost, seq++, make_int4(i, m, cg, x->shape)};
      }
    }
  }
  auto longest_first = [](const ItemRec &p, const ItemRec &q) { return p.cost != q.cost ? p.cost > q.cost : p.seq < q.seq; };
  for (int k = 0; k < 4; ++k) std::sort(rec + start[k], rec + pos[k], longest_first);
}

// Device addresses of a batch's three tables.
struct DevTables {
  qoc::DevSys *sys;
  int4 *items;
  int2 *blocks;
};

// Writes the host image of a batch's tables (systems at 0, item records at lay.items, block
// table at lay.blocks) and fills `plan` with the matching addresses of the device tables.
static void batch_image(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad, const BatchCounts &c,
                        const ItemRec *rec, char *host, const DevTables &dev, const StageLayout &lay,
                        qoc::BatchPlan &plan) {
  qoc::DevSys *hs = reinterpret_cast<qoc::DevSys *>(host);
  int4 *hi = reinterpret_cast<int4 *>(host + lay.items);
  int2 *hb = reinterpret_cast<int2 *>(host + lay.blocks);
  for (int i = 0; i < n; ++i) hs[i] = ctxs[i]->dev;
  for (long long k = 0; k < c.records(); ++k) hi[k] = rec[k].v;
  plan.sys = dev.sys;
  plan.fwd_items = dev.items;
  plan.bwd_items = dev.items + c.fwd;
  plan.xw_items = dev.items + c.fwd + c.bwd;
  plan.x3_items = dev.items + c.fwd + c.bwd + c.xw;
  plan.n_fwd = (int)c.fwd;
  plan.n_bwd = (int)c.bwd;
  plan.n_xw = (int)c.xw;
  plan.n_x3 = (int)c.x3;
  plan.fp64 = ctxs[0]->fp64;
  long long off = 0;
  for (int kind = 0; kind < qoc::SK_COUNT; ++kind) {
    const bool gk = kind == qoc::SK_SERIES || kind == qoc::SK_PROJECT || kind == qoc::SK_GRADW;
    plan.blocks[kind] = dev.blocks + off;
    long long cnt = 0;
    for (int i = 0; i < n; ++i) {
      if (gk && want_grad && !want_grad[i]) continue;
      const int nb = qoc::small_blocks(ctxs[i]->dev, kind);
      for (int j = 0; j < nb; ++j) hb[off + cnt++] = make_int2(i, j);
    }
    plan.n_blocks[kind] = (int)cnt;
    off += cnt;
  }
}

// Launches the phases of a batched evaluation on st and marks the contexts evaluated.
static int batch_launch(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad, const BatchCounts &c,
                        const qoc::BatchPlan &plan, hipStream_t st) {
  const int nph = c.any_grad ? qoc::PHASE_GRAD_W + 1 : qoc::PHASE_BOUNDARY + 1;
  for (int ph = 0; ph < nph; ++ph) {
    int e = qoc::launch_batch_phase(plan, ph, st);
    if (e) {
      for (int i = 0; i < n; ++i) ctxs[i]->forward_valid = false;
      return hip_fail((hipError_t)e, "batched kernel launch");
    }
  }
  for (int i = 0; i < n; ++i) {
    qoc_ctx *c = ctxs[i];
    c->stream = st;
    c->forward_valid = true;
    c->grad_valid = !want_grad || want_grad[i];
  }
  return QOC_OK;
}

int qoc_batch_run(qoc_batch *b, qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad, void *hip_stream) {
  if (!b || !ctxs || n < 1) return fail(QOC_EINVAL, "qoc_batch_run: bad arguments");
  if (n > b->max_ctx) return fail(QOC_EINVAL, "qoc_batch_run: more contexts than the batch was created for");
  int rc = batch_check(ctxs, n, b->device, "qoc_batch_run");
  if (rc != QOC_OK) return rc;
  HIP_OR_RETURN(hipSetDevice(b->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const BatchCounts cnt = batch_counts(ctxs, n, want_grad);
  if (cnt.fwd > b->max_items || cnt.bwd + cnt.xw + cnt.x3 > b->max_items)
    return fail(QOC_EINVAL, "qoc_batch_run: more propagation items than the batch was created for");
  if (cnt.nblocks > b->max_blocks) return fail(QOC_EINVAL, "qoc_batch_run: small-kernel table exceeds the batch capacity");
  std::vector<ItemRec> rec((size_t)cnt.records());
  batch_fill(ctxs, n, want_grad, cnt, rec.data());

  // the previous run's uploads must have left the staging buffer
  if (b->pending) HIP_OR_RETURN(hipEventSynchronize(b->uploaded));
  const StageLayout lay = stage_layout(b->max_ctx, b->max_items, b->max_blocks);
  qoc::BatchPlan plan{};
  char *h = b->h_stage;
  batch_image(ctxs, n, want_grad, cnt, rec.data(), h, DevTables{b->d_sys, b->d_items, b->d_blocks}, lay, plan);
  plan.aux = b->aux;
  plan.aux2 = b->aux2;
  plan.fork = b->fork;
  plan.join = b->join;
  plan.join2 = b->join2;
  HIP_OR_RETURN(hipMemcpyAsync(b->d_sys, h, sizeof(qoc::DevSys) * n, hipMemcpyHostToDevice, st));
  HIP_OR_RETURN(hipMemcpyAsync(b->d_items, h + lay.items, sizeof(int4) * std::max<long long>(cnt.records(), 1),
                               hipMemcpyHostToDevice, st));
  HIP_OR_RETURN(hipMemcpyAsync(b->d_blocks, h + lay.blocks, sizeof(int2) * std::max<long long>(cnt.nblocks, 1),
                               hipMemcpyHostToDevice, st));
  HIP_OR_RETURN(hipEventRecord(b->uploaded, st));
  b->pending = true;
  rc = batch_launch(ctxs, n, want_grad, cnt, plan, st);
  if (rc != QOC_OK) return rc;
  // each context's status word moves into the batch's list (read by qoc_batch_status)
  {
    const int e = qoc::launch_gather_status(b->d_sys, n, b->d_status, st);
    if (e) return hip_fail((hipError_t)e, "qoc_batch_run: status gather");
  }
  HIP_OR_RETURN(hipMemcpyAsync(b->h_status, b->d_status, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  HIP_OR_RETURN(hipEventRecord(b->done, st));
  b->last_n = n;
  return QOC_OK;
}

// Host image of the allocation-free run's tables (the device copy is the static array of the
// kernel file) and its item records; one call at a time uses them.
static unsigned char g_noalloc_image[qoc::kNoAllocScratchBytes];
static ItemRec g_noalloc_records[qoc::kNoAllocScratchBytes / sizeof(int4)];
static std::mutex g_noalloc_lock;

int qoc_batch_run_noalloc(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad, void *hip_stream) {
  if (!ctxs || n < 1 || !ctxs[0]) return fail(QOC_EINVAL, "qoc_batch_run_noalloc: bad arguments");
  const int device = ctxs[0]->device;
  int rc = batch_check(ctxs, n, device, "qoc_batch_run_noalloc");
  if (rc != QOC_OK) return rc;
  const BatchCounts cnt = batch_counts(ctxs, n, want_grad);
  const StageLayout lay = stage_layout_records(n, cnt.records(), cnt.nblocks);
  if (lay.total > qoc::kNoAllocScratchBytes)
    return fail(QOC_EINVAL, "qoc_batch_run_noalloc: the batch needs " + std::to_string(lay.total) +
                                " bytes of tables, over the static capacity of " +
                                std::to_string(qoc::kNoAllocScratchBytes));
  HIP_OR_RETURN(hipSetDevice(device));
  void *dev = nullptr;
  {
    const int e = qoc::noalloc_scratch(device, &dev);
    if (e) return hip_fail((hipError_t)e, "qoc_batch_run_noalloc: address of the static tables");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char *d = static_cast<char *>(dev);
  qoc::BatchPlan plan{};
  std::lock_guard<std::mutex> guard(g_noalloc_lock);
  char *h = reinterpret_cast<char *>(g_noalloc_image);
  batch_fill(ctxs, n, want_grad, cnt, g_noalloc_records);
  batch_image(ctxs, n, want_grad, cnt, g_noalloc_records, h,
              DevTables{reinterpret_cast<qoc::DevSys *>(d), reinterpret_cast<int4 *>(d + lay.items),
                        reinterpret_cast<int2 *>(d + lay.blocks)},
              lay, plan);
  // no streams of a batch here: every kind of backward item runs on st (plan.aux stays NULL)
  HIP_OR_RETURN(hipMemcpyAsync(dev, h, lay.total, hipMemcpyHostToDevice, st));
  // the host image is reused by the next call: wait until this copy has read it
  HIP_OR_RETURN(hipStreamSynchronize(st));
  return batch_launch(ctxs, n, want_grad, cnt, plan, st);
}

int qoc_batch_status(qoc_batch *b, int32_t *status, int32_t n) {
  if (!b || !status) return fail(QOC_EINVAL, "qoc_batch_status: NULL argument");
  if (b->last_n == 0) return fail(QOC_ESTATE, "qoc_batch_status: the batch has not run");
  if (n != b->last_n)
    return fail(QOC_EINVAL, "qoc_batch_status: the last run had " + std::to_string(b->last_n) + " contexts");
  HIP_OR_RETURN(hipSetDevice(b->device));
  HIP_OR_RETURN(hipEventSynchronize(b->done));
  int bad = 0;
  for (int i = 0; i < n; ++i) {
    status[i] = (b->h_status[i] & qoc::STATUS_NOTCONV) ? QOC_ENOTCONV : QOC_OK;
    bad += status[i] != QOC_OK;
  }
  if (bad) g_last_error = std::to_string(bad) + " of " + std::to_string(n) +
                          " contexts exceeded the fixed-point contraction bound";
  return QOC_OK;
}

int qoc_batch_gradient(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad) {
  if (!ctxs || n < 1) return fail(QOC_EINVAL, "qoc_batch_gradient: bad arguments");
  long long nf = 0, nb = 0;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(QOC_EINVAL, "qoc_batch_gradient: NULL context");
    nf += (long long)ctxs[i]->M * ctxs[i]->dev.ncg;
    nb += (long long)ctxs[i]->M * ctxs[i]->dev.ncg_b;
  }
  qoc_batch *b = nullptr;
  int rc = qoc_batch_create(ctxs[0]->device, n, std::max(nf, nb), &b);
  if (rc != QOC_OK) return rc;
  hipStream_t st = ctxs[0]->stream;
  rc = qoc_batch_run(b, ctxs, n, want_grad, st);
  if (rc != QOC_OK) { qoc_batch_destroy(b); return rc; }
  std::vector<int32_t> status(n);
  rc = qoc_batch_status(b, status.data(), n);
  qoc_batch_destroy(b);
  if (rc != QOC_OK) return rc;
  std::string bad;
  for (int i = 0; i < n; ++i)
    if (status[i] != QOC_OK) bad += (bad.empty() ? "" : ", ") + std::to_string(i);
  if (!bad.empty())
    return fail(QOC_ENOTCONV, "qoc_batch_gradient: contexts " + bad + " exceeded the fixed-point contraction bound");
  return QOC_OK;
}

int qoc_read_results(qoc_ctx *ctx, double *P, double *terms, double *grad_alpha, double *grad_W, int32_t where) {
  if (!ctx) return fail(QOC_EINVAL, "qoc_read_results: NULL context");
  if (where != QOC_HOST && where != QOC_DEVICE) return fail(QOC_EINVAL, "qoc_read_results: bad memory kind");
  if (!ctx->forward_valid) return fail(QOC_ESTATE, "qoc_read_results: no evaluation for the current inputs");
  if ((grad_alpha || grad_W) && !ctx->grad_valid) return fail(QOC_ESTATE, "qoc_read_results: no gradient evaluated");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  const hipMemcpyKind k = kind_out(where);
  const qoc::DevSys &s = ctx->dev;
  if (P) HIP_OR_RETURN(hipMemcpyAsync(P, s.scal, sizeof(double), k, ctx->stream));
  if (terms) HIP_OR_RETURN(hipMemcpyAsync(terms, s.scal + 1, sizeof(double) * (4 + ctx->M), k, ctx->stream));
  if (grad_alpha) HIP_OR_RETURN(hipMemcpyAsync(grad_alpha, s.grad_alpha, sizeof(double) * ctx->d, k, ctx->stream));
  if (grad_W && ctx->M > 1)
    HIP_OR_RETURN(hipMemcpyAsync(grad_W, s.grad_W, sizeof(double) * 2 * (size_t)(ctx->M - 1) * ctx->E * ctx->N, k, ctx->stream));
  if (where == QOC_HOST) return check_status(ctx);
  return QOC_OK;
}

int qoc_synchronize(qoc_ctx *ctx) {
  if (!ctx) return fail(QOC_EINVAL, "qoc_synchronize: NULL context");
  HIP_OR_RETURN(hipSetDevice(ctx->device));
  return check_status(ctx);
}

}  // extern "C"
