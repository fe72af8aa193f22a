// Optimisation driver: the quadratic-penalty method of Sec. 3 (L-BFGS on P) with
// the settings of Sec. 5 (box constraints on the pulse amplitude, Tikhonov and
// control-energy terms, window states scaled by sigma, roll-out-estimate stopping
// rule of eq. rollout-infid-est).  It calls the objective/gradient ABI of the
// context it owns; the optimisation vectors (about 1e6 doubles at 4 qubits) and
// the L-BFGS history stay in device memory, and only scalars reach the host.  The
// two-loop recursion keeps its coefficients on the device, so an iteration waits
// for the device three times: for (|gr|_inf, g.p), once per trial point, and for
// the curvature pair.  The iteration is specified in include/qoc.h.
#include "../../include/qoc.h"
#include "qoc_internal.h"

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

namespace {

constexpr double kArmijo = 1e-4;       // sufficient-decrease constant
constexpr int kMaxHalvings = 30;        // backtracking steps before giving up
constexpr double kCurvature = 1e-12;    // keep (s, y) when s.y > kCurvature |s| |y|

int err(int code, const std::string &m) { return qoc::set_error(code, m.c_str()); }

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    const int e_ = (int)(expr);                                                               \
    if (e_ != 0) return err(QOC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString((hipError_t)e_)); \
  } while (0)

#define QOCCHK(expr)              \
  do {                            \
    const int rc_ = (expr);       \
    if (rc_ != QOC_OK) return rc_; \
  } while (0)

}  // namespace

struct qoc_opt {
  qoc_ctx *ctx = nullptr;
  qoc_opt_desc D{};
  int d = 0, M = 0, E = 0;
  long long nW = 0, n = 0;
  double amax = 0.0, dt = 0.0;
  hipStream_t st = nullptr;
  std::vector<void *> allocs;
  // device vectors
  double *x = nullptr, *g = nullptr, *xt = nullptr, *gt = nullptr, *p = nullptr, *q = nullptr, *gr = nullptr,
         *ytmp = nullptr, *Wbuf = nullptr, *ga = nullptr, *gW = nullptr, *gE = nullptr, *dtab = nullptr,
         *partials = nullptr, *res = nullptr, *acoef = nullptr, *bcoef = nullptr;
  // device scalars in res: [0..kObj) single values, then P and the 4 + M terms
  enum { R_GINF = 0, R_GP, R_GG, R_GS, R_EN, R_AA, R_SY, R_YY, R_SS, kObj = 12 };
  std::vector<double> hres;             // host copy of res
  std::vector<double *> S, Y;
  std::vector<double> rho, sy, yy;      // per history slot
  int hist = 0, newest = -1;            // pairs kept; slot of the newest (ring of D.memory slots)
  // current iterate and the last trial point (host scalars)
  struct Point {
    double F = 0, P = 0, energy = 0, tik = 0;
    std::vector<double> terms;
  } cur, trial;
  double grad_inf = 0.0, last_t = 0.0;
  int iters = 0, evals = 0, bwd = 0, stop = 0;

  ~qoc_opt() {
    for (void *v : allocs) (void)hipFree(v);
  }
  int alloc(double **ptr, size_t count) {
    void *v = nullptr;
    const size_t bytes = std::max<size_t>(count, 2) * sizeof(double);
    if (hipMalloc(&v, bytes) != hipSuccess) return err(QOC_ENOMEM, "qoc_opt: device allocation failed");
    allocs.push_back(v);
    if (hipMemset(v, 0, bytes) != hipSuccess) return err(QOC_EDEVICE, "qoc_opt: hipMemset failed");
    *ptr = static_cast<double *>(v);
    return QOC_OK;
  }
  // res[0..count) -> hres (waits for the stream); also reports a fixed-point bound
  // violation flagged by the evaluations queued since the last wait
  int fetch(int count) {
    int status[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(hres.data(), res, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(status, qoc::ctx_dev(ctx).status, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (status[0] & qoc::STATUS_NOTCONV) return qoc_synchronize(ctx);   // clears the flag, returns QOC_ENOTCONV
    return QOC_OK;
  }
  int dot(const double *a, const double *b, long long len, int slot) {
    HIPCHK(qoc::opt_dot(a, b, len, partials, res + slot, st));
    return QOC_OK;
  }
  double estimate(const Point &pt) const {
    const double J = pt.terms[0];
    double csum = 0.0;
    for (int m = 0; m + 1 < M; ++m) csum += std::sqrt(std::max(pt.terms[5 + m], 0.0));
    return J + 2.0 / std::sqrt((double)E) * std::sqrt(std::max(J, 0.0)) * csum + csum * csum / E;
  }
  // F at v (device vector): sets the context's inputs from v, objective, energy,
  // Tikhonov; one wait, which also returns the scalars the caller queued before
  int eval_objective(const double *v, Point &pt) {
    QOCCHK(qoc_set_controls(ctx, v, d, QOC_DEVICE));
    if (M > 1) {
      HIPCHK(qoc::opt_axpby(Wbuf, 1.0 / D.sigma, v + d, 0.0, nW, st));
      QOCCHK(qoc_set_window_states(ctx, Wbuf, nW, QOC_DEVICE));
    }
    HIPCHK(qoc::opt_energy(qoc::ctx_dev(ctx), v, dtab, partials, res + R_EN, st));
    QOCCHK(dot(v, v, d, R_AA));
    QOCCHK(qoc_objective(ctx, res + kObj, res + kObj + 1, QOC_DEVICE));
    QOCCHK(fetch(kObj + 5 + M));
    pt.P = hres[kObj];
    std::copy(hres.begin() + kObj + 1, hres.begin() + kObj + 5 + M, pt.terms.begin());
    pt.energy = dt * hres[R_EN];
    pt.tik = 0.5 * D.gamma_tik * hres[R_AA];
    pt.F = pt.P + pt.tik + D.gamma_energy * pt.energy;
    ++evals;
    return QOC_OK;
  }
  // gradient at the point of the last eval_objective (v), into out
  int eval_gradient(const double *v, double *out) {
    QOCCHK(qoc_backward(ctx, ga, gW, QOC_DEVICE));
    HIPCHK(qoc::opt_energy_grad(qoc::ctx_dev(ctx), dtab, gE, st));
    HIPCHK(qoc::opt_assemble(out, ga, v, gE, gW, d, nW, D.gamma_tik, D.gamma_energy, 1.0 / D.sigma, st));
    ++bwd;
    return QOC_OK;
  }
  int reduced(double *out, const double *v) {
    HIPCHK(qoc::opt_reduced(out, v, x, g, n, d, -amax, amax, st));
    return QOC_OK;
  }
  int iterate();
};

int qoc_opt::iterate() {
  QOCCHK(reduced(gr, g));
  HIPCHK(qoc::opt_maxabs(gr, n, partials, res + R_GINF, st));

  // p = -H gr (two-loop recursion, coefficients on the device), restricted to the free entries
  bool used_hist = hist > 0;
  HIPCHK(qoc::opt_axpby(q, 1.0, gr, 0.0, n, st));
  if (used_hist) {
    const int m = D.memory;
    for (int i = 0; i < hist; ++i) {                      // newest to oldest: a = rho s.q, q -= a y
      const int sl = (newest - i + m) % m;
      HIPCHK(qoc::opt_dot_to(S[sl], q, n, partials, acoef + sl, rho[sl], nullptr, 0.0, st));
      HIPCHK(qoc::opt_axpy_dev(q, acoef + sl, -1.0, Y[sl], n, st));
    }
    HIPCHK(qoc::opt_axpby(q, 0.0, q, sy[newest] / yy[newest], n, st));
    for (int i = hist - 1; i >= 0; --i) {                 // oldest to newest: q += (a - rho y.q) s
      const int sl = (newest - i + m) % m;
      HIPCHK(qoc::opt_dot_to(Y[sl], q, n, partials, bcoef + sl, -rho[sl], acoef + sl, 1.0, st));
      HIPCHK(qoc::opt_axpy_dev(q, bcoef + sl, 1.0, S[sl], n, st));
    }
  }
  HIPCHK(qoc::opt_axpby(p, -1.0, q, 0.0, n, st));
  QOCCHK(reduced(p, p));
  QOCCHK(dot(g, p, n, R_GP));
  QOCCHK(dot(gr, gr, n, R_GG));
  QOCCHK(fetch(R_GG + 1));
  grad_inf = hres[R_GINF];
  if (estimate(cur) < D.tol_estimate) { stop = 1; return QOC_OK; }
  if (D.tol_grad > 0.0 && grad_inf < D.tol_grad) { stop = 2; return QOC_OK; }
  if (!(hres[R_GP] < 0.0)) {                               // not a descent direction: restart
    hist = 0;
    newest = -1;
    used_hist = false;
    HIPCHK(qoc::opt_axpby(p, -1.0, gr, 0.0, n, st));
  }
  double t = 1.0;
  if (!used_hist) t = 1.0 / std::max(1.0, std::sqrt(hres[R_GG]));

  // backtracking on the projected step
  bool accepted = false;
  for (int h = 0; h < kMaxHalvings; ++h) {
    HIPCHK(qoc::opt_trial(xt, x, p, t, n, d, -amax, amax, st));
    HIPCHK(qoc::opt_axpby(q, 1.0, xt, 0.0, n, st));       // s = xt - x
    HIPCHK(qoc::opt_axpby(q, -1.0, x, 1.0, n, st));
    QOCCHK(dot(g, q, n, R_GS));
    QOCCHK(eval_objective(xt, trial));                     // (returns g.s with the objective)
    if (trial.F <= cur.F + kArmijo * hres[R_GS]) {
      accepted = true;
      break;
    }
    t *= 0.5;
  }
  if (!accepted) {                                         // the context holds the last trial: restore x
    QOCCHK(eval_objective(x, trial));
    stop = 3;
    return QOC_OK;
  }
  QOCCHK(eval_gradient(xt, gt));

  // curvature pair (s, y) = (xt - x, gt - g)
  HIPCHK(qoc::opt_axpby(ytmp, 1.0, gt, 0.0, n, st));
  HIPCHK(qoc::opt_axpby(ytmp, -1.0, g, 1.0, n, st));
  QOCCHK(dot(q, ytmp, n, R_SY));
  QOCCHK(dot(ytmp, ytmp, n, R_YY));
  QOCCHK(dot(q, q, n, R_SS));
  QOCCHK(fetch(R_SS + 1));
  const double s_y = hres[R_SY], y_y = hres[R_YY], s_s = hres[R_SS];
  if (s_y > kCurvature * std::sqrt(s_s * y_y)) {
    const int m = D.memory;
    const int sl = (newest + 1) % m;
    HIPCHK(hipMemcpyAsync(S[sl], q, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(Y[sl], ytmp, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    rho[sl] = 1.0 / s_y;
    sy[sl] = s_y;
    yy[sl] = y_y;
    newest = sl;
    hist = std::min(hist + 1, m);
  }
  std::swap(x, xt);
  std::swap(g, gt);
  std::swap(cur, trial);
  last_t = t;
  ++iters;
  return QOC_OK;
}

extern "C" {

int qoc_opt_create(qoc_ctx *ctx, const qoc_opt_desc *desc, const double *alpha0, const double *W0, int32_t where,
                   qoc_opt **out) {
  if (!ctx || !desc || !alpha0 || !out) return err(QOC_EINVAL, "qoc_opt_create: NULL argument");
  if (where != QOC_HOST && where != QOC_DEVICE) return err(QOC_EINVAL, "qoc_opt_create: bad memory kind");
  const qoc_opt_desc &Dd = *desc;
  if (!(Dd.sigma > 0.0) || !std::isfinite(Dd.sigma) || !(Dd.gamma_tik >= 0.0) || !std::isfinite(Dd.gamma_tik) ||
      !(Dd.gamma_energy >= 0.0) || !std::isfinite(Dd.gamma_energy) || !(Dd.amp_bound > 0.0) ||
      !std::isfinite(Dd.amp_bound) || Dd.memory < 1 || Dd.memory > 64 || !(Dd.tol_estimate >= 0.0) ||
      !(Dd.tol_grad >= 0.0))
    return err(QOC_EINVAL, "qoc_opt_create: invalid description");
  qoc_info info;
  QOCCHK(qoc_get_info(ctx, &info));
  std::unique_ptr<qoc_opt> o(new qoc_opt());
  o->ctx = ctx;
  o->D = Dd;
  o->d = info.d;
  o->M = info.n_windows;
  o->E = info.E;
  o->nW = info.n_window_doubles;
  o->n = o->d + o->nW;
  const qoc::DevSys &sys = qoc::ctx_dev(ctx);
  o->amax = Dd.amp_bound / (std::sqrt(2.0) * sys.nf);
  o->dt = sys.dt;
  o->st = qoc::ctx_stream(ctx);
  HIPCHK(hipSetDevice(qoc::ctx_device(ctx)));
  const long long n = o->n;
  QOCCHK(o->alloc(&o->x, n));
  QOCCHK(o->alloc(&o->g, n));
  QOCCHK(o->alloc(&o->xt, n));
  QOCCHK(o->alloc(&o->gt, n));
  QOCCHK(o->alloc(&o->p, n));
  QOCCHK(o->alloc(&o->q, n));
  QOCCHK(o->alloc(&o->gr, n));
  QOCCHK(o->alloc(&o->ytmp, n));
  QOCCHK(o->alloc(&o->Wbuf, o->nW));
  QOCCHK(o->alloc(&o->ga, o->d));
  QOCCHK(o->alloc(&o->gW, o->nW));
  QOCCHK(o->alloc(&o->gE, o->d));
  QOCCHK(o->alloc(&o->dtab, (size_t)2 * sys.NT * sys.q));
  QOCCHK(o->alloc(&o->partials, std::max(qoc::kOptGrid, qoc::opt_energy_blocks(sys))));
  QOCCHK(o->alloc(&o->res, qoc_opt::kObj + 5 + o->M));
  QOCCHK(o->alloc(&o->acoef, Dd.memory));
  QOCCHK(o->alloc(&o->bcoef, Dd.memory));
  o->hres.assign(qoc_opt::kObj + 5 + o->M, 0.0);
  o->S.resize(Dd.memory);
  o->Y.resize(Dd.memory);
  for (int i = 0; i < Dd.memory; ++i) {
    QOCCHK(o->alloc(&o->S[i], n));
    QOCCHK(o->alloc(&o->Y[i], n));
  }
  o->rho.assign(Dd.memory, 0.0);
  o->sy.assign(Dd.memory, 0.0);
  o->yy.assign(Dd.memory, 1.0);
  o->cur.terms.assign(4 + o->M, 0.0);
  o->trial.terms.assign(4 + o->M, 0.0);

  // start point: alpha0 clipped to the box; W0 or the roll-out of alpha0; x = [alpha, sigma W]
  const hipMemcpyKind kin = where == QOC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(hipMemcpyAsync(o->xt, alpha0, sizeof(double) * o->d, kin, o->st));
  HIPCHK(qoc::opt_trial(o->x, o->xt, o->p, 0.0, o->d, o->d, -o->amax, o->amax, o->st));
  if (o->M > 1) {
    if (W0) {
      HIPCHK(hipMemcpyAsync(o->Wbuf, W0, sizeof(double) * o->nW, kin, o->st));
    } else {
      QOCCHK(qoc_set_controls(ctx, o->x, o->d, QOC_DEVICE));
      QOCCHK(qoc_rollout(ctx, o->Wbuf, nullptr, QOC_DEVICE));
    }
    HIPCHK(qoc::opt_axpby(o->x + o->d, Dd.sigma, o->Wbuf, 0.0, o->nW, o->st));
  }
  QOCCHK(o->eval_objective(o->x, o->cur));
  QOCCHK(o->eval_gradient(o->x, o->g));
  HIPCHK(hipStreamSynchronize(o->st));
  *out = o.release();
  return QOC_OK;
}

int qoc_opt_destroy(qoc_opt *opt) {
  if (!opt) return err(QOC_EINVAL, "qoc_opt_destroy: NULL");
  (void)hipSetDevice(qoc::ctx_device(opt->ctx));
  (void)hipStreamSynchronize(opt->st);
  delete opt;
  return QOC_OK;
}

int qoc_opt_run(qoc_opt *opt, int32_t n_iters, qoc_opt_status *status) {
  if (!opt || n_iters < 0) return err(QOC_EINVAL, "qoc_opt_run: bad arguments");
  HIPCHK(hipSetDevice(qoc::ctx_device(opt->ctx)));
  for (int i = 0; i < n_iters && opt->stop == 0; ++i) QOCCHK(opt->iterate());
  if (opt->stop == 0) {                                    // refresh |gr| and the stop test at the iterate
    QOCCHK(opt->reduced(opt->gr, opt->g));
    HIPCHK(qoc::opt_maxabs(opt->gr, opt->n, opt->partials, opt->res + qoc_opt::R_GINF, opt->st));
    QOCCHK(opt->fetch(qoc_opt::R_GINF + 1));
    opt->grad_inf = opt->hres[qoc_opt::R_GINF];
  }
  if (status) {
    qoc_opt_status &s = *status;
    s.iterations = opt->iters;
    s.evaluations = opt->evals;
    s.backward_sweeps = opt->bwd;
    s.stop = opt->stop;
    s.F = opt->cur.F;
    s.P = opt->cur.P;
    s.J = opt->cur.terms[0];
    s.penalty = opt->cur.terms[1];
    s.energy = opt->cur.energy;
    s.tikhonov = opt->cur.tik;
    s.estimate = opt->estimate(opt->cur);
    s.grad_inf = opt->grad_inf;
    s.last_step = opt->last_t;
  }
  return QOC_OK;
}

int qoc_opt_get(qoc_opt *opt, double *alpha, double *W, int32_t where) {
  if (!opt) return err(QOC_EINVAL, "qoc_opt_get: NULL");
  if (where != QOC_HOST && where != QOC_DEVICE) return err(QOC_EINVAL, "qoc_opt_get: bad memory kind");
  HIPCHK(hipSetDevice(qoc::ctx_device(opt->ctx)));
  const hipMemcpyKind kout = where == QOC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (alpha) HIPCHK(hipMemcpyAsync(alpha, opt->x, sizeof(double) * opt->d, kout, opt->st));
  if (W && opt->M > 1) {
    HIPCHK(qoc::opt_axpby(opt->Wbuf, 1.0 / opt->D.sigma, opt->x + opt->d, 0.0, opt->nW, opt->st));
    HIPCHK(hipMemcpyAsync(W, opt->Wbuf, sizeof(double) * opt->nW, kout, opt->st));
  }
  HIPCHK(hipStreamSynchronize(opt->st));
  return QOC_OK;
}

}  // extern "C"
