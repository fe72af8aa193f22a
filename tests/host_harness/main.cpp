// Drives the library's host code through the C ABI on the HIP stand-in (no GPU): system
// builds, single-context calls, batches of odd and even sizes with mixed backward schedules,
// per-context status, the one-call batched gradient, and teardown without leaked device
// blocks.  Built with AddressSanitizer and UBSan by tests/test_host_harness.py; prints
// "HARNESS OK" at the end.  Test infrastructure only.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/qoc.h"

long standin_launches();
size_t standin_live_device_blocks();
size_t standin_live_pinned_blocks();

#define CHECK(x)                                                                           \
  do {                                                                                     \
    if (!(x)) {                                                                            \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #x, qoc_last_error()); \
      std::exit(1);                                                                        \
    }                                                                                      \
  } while (0)

struct Sys {
  int q, L, M;
  long long NT;
  std::vector<double> det, anh, ck, car, target, alpha, W;
  qoc_ctx *ctx = nullptr;
  int d = 0, N = 0, E = 0;
};

static void make(Sys &s, int q, int L, long long NT, int M, int schedule, unsigned seed) {
  s.q = q; s.L = L; s.NT = NT; s.M = M;
  s.E = 1 << q;
  s.N = 1;
  for (int j = 0; j < q; ++j) s.N *= L;
  const int nf = 2, d1 = 6;
  s.det.assign(q, 0.1); s.anh.assign(q, -1.2); s.ck.assign(q > 1 ? q - 1 : 1, 0.03);
  s.car.assign(q * nf, 0.2);
  s.target.assign(2 * s.E * s.E, 0.0);
  for (int a = 0; a < s.E; ++a)          // E x E discrete Fourier matrix, unitary
    for (int b = 0; b < s.E; ++b) {
      const std::complex<double> v = std::polar(1.0 / std::sqrt((double)s.E), 2 * M_PI * a * b / s.E);
      s.target[2 * (a * s.E + b)] = v.real();
      s.target[2 * (a * s.E + b) + 1] = v.imag();
    }
  qoc_system_desc D{};
  D.n_qubits = q; D.n_levels = L; D.detuning = s.det.data(); D.anharmonicity = s.anh.data();
  D.cross_kerr = s.ck.data(); D.n_carriers = nf; D.carrier_freq = s.car.data(); D.n_splines = d1;
  D.T = 10.0; D.n_steps = NT; D.n_windows = M; D.mu = 0.5; D.target = s.target.data();
  D.precision = QOC_FP32; D.checkpoint_every = 7; D.device = 0;
  CHECK(qoc_create(&D, &s.ctx) == QOC_OK);
  qoc_info inf;
  CHECK(qoc_get_info(s.ctx, &inf) == QOC_OK);
  s.d = inf.d;
  CHECK(qoc_set_schedule(s.ctx, schedule) == QOC_OK);
  srand(seed);
  s.alpha.resize(s.d);
  for (double &a : s.alpha) a = 0.01 * (rand() / (double)RAND_MAX - 0.5);
  s.W.resize(2 * (size_t)(M - 1) * s.N * s.E);
  for (double &w : s.W) w = rand() / (double)RAND_MAX - 0.5;
  CHECK(qoc_set_controls(s.ctx, s.alpha.data(), s.d, QOC_HOST) == QOC_OK);
  CHECK(qoc_set_window_states(s.ctx, M > 1 ? s.W.data() : nullptr, (int64_t)s.W.size(), QOC_HOST) == QOC_OK);
}

static void read_all(Sys &s, bool grad) {
  double P;
  std::vector<double> terms(4 + s.M), ga(s.d), gW(s.W.size() + 2);
  CHECK(qoc_read_results(s.ctx, &P, terms.data(), grad ? ga.data() : nullptr, grad ? gW.data() : nullptr,
                         QOC_HOST) == QOC_OK);
  CHECK(P == 0.5);
}

int main() {
  std::vector<Sys> sys(5);
  make(sys[0], 2, 3, 40, 4, QOC_BWD_AUTO, 1);
  make(sys[1], 3, 4, 45, 7, QOC_BWD_AUTO, 2);
  make(sys[2], 4, 4, 33, 5, QOC_BWD_AUTO, 3);
  make(sys[3], 4, 4, 30, 3, QOC_BWD_ONE_WAVE, 4);
  make(sys[4], 2, 2, 20, 1, QOC_BWD_TWO_WAVES, 5);

  // single-context calls, host outputs
  for (Sys &s : sys) {
    double P;
    std::vector<double> terms(4 + s.M), ga(s.d), gW(s.W.size() + 2);
    CHECK(qoc_objective(s.ctx, &P, terms.data(), QOC_HOST) == QOC_OK);
    CHECK(qoc_backward(s.ctx, ga.data(), s.M > 1 ? gW.data() : nullptr, QOC_HOST) == QOC_OK);
    CHECK(qoc_gradient(s.ctx, &P, terms.data(), ga.data(), s.M > 1 ? gW.data() : nullptr, QOC_HOST) == QOC_OK);
    CHECK(P == 0.5 && ga[0] == 1.0);
    std::vector<double> Wr(s.W.size() + 2), Ur(2 * (size_t)s.N * s.E);
    CHECK(qoc_rollout(s.ctx, s.M > 1 ? Wr.data() : nullptr, Ur.data(), QOC_HOST) == QOC_OK);
    CHECK(qoc_enable_timing(s.ctx, 1) == QOC_OK);
    CHECK(qoc_gradient(s.ctx, &P, nullptr, ga.data(), nullptr, QOC_HOST) == QOC_OK);
    qoc_timings tm;
    CHECK(qoc_get_timings(s.ctx, &tm) == QOC_OK && tm.n_calls == 1 && tm.n_grad_calls == 1);
  }

  // batches of every size from one to all, with capacities that are exactly sufficient
  std::vector<qoc_ctx *> ctxs;
  for (Sys &s : sys) ctxs.push_back(s.ctx);
  for (int n = 1; n <= (int)sys.size(); ++n) {
    long long items = 0;
    for (int i = 0; i < n; ++i) {
      qoc_info inf;
      CHECK(qoc_get_info(ctxs[i], &inf) == QOC_OK);
      items += (long long)inf.n_windows * 16;    // >= windows x column groups of every layout here
    }
    qoc_batch *b = nullptr;
    CHECK(qoc_batch_create(0, n, items, &b) == QOC_OK);
    std::vector<int32_t> want(n);
    for (int i = 0; i < n; ++i) want[i] = (i % 3) != 2;
    for (int rep = 0; rep < 2; ++rep) {
      CHECK(qoc_batch_run(b, ctxs.data(), n, want.data(), nullptr) == QOC_OK);
      std::vector<int32_t> st(n, 7);
      CHECK(qoc_batch_status(b, st.data(), n) == QOC_OK);
      for (int i = 0; i < n; ++i) CHECK(st[i] == QOC_OK);
      for (int i = 0; i < n; ++i) read_all(sys[i], want[i] != 0);
    }
    std::vector<int32_t> st(n + 1);
    CHECK(qoc_batch_status(b, st.data(), n + 1) == QOC_EINVAL);
    CHECK(qoc_batch_destroy(b) == QOC_OK);
    CHECK(qoc_batch_gradient(ctxs.data(), n, nullptr) == QOC_OK);
    for (int i = 0; i < n; ++i) read_all(sys[i], true);
  }

  // the allocation-free batched run: every size, twice, and results read back
  for (int n = (int)sys.size(); n >= 1; --n) {
    std::vector<int32_t> want(n);
    for (int i = 0; i < n; ++i) want[i] = (i % 2) == 0;
    for (int rep = 0; rep < 2; ++rep) {
      CHECK(qoc_batch_run_noalloc(ctxs.data(), n, want.data(), nullptr) == QOC_OK);
      for (int i = 0; i < n; ++i) read_all(sys[i], want[i] != 0);
    }
  }
  CHECK(qoc_batch_run_noalloc(nullptr, 1, nullptr, nullptr) == QOC_EINVAL);
  CHECK(qoc_batch_run_noalloc(ctxs.data(), 0, nullptr, nullptr) == QOC_EINVAL);
  {
    std::vector<qoc_ctx *> twice = {ctxs[0], ctxs[0]};
    CHECK(qoc_batch_run_noalloc(twice.data(), 2, nullptr, nullptr) == QOC_EINVAL);
  }
  {   // tables over the static capacity (the harness builds with a 256 KiB capacity): four
      // contexts of 4 qubits x 128 windows need ~330 KB, two ~165 KB
    std::vector<Sys> big(4);
    std::vector<qoc_ctx *> bc;
    for (int i = 0; i < 4; ++i) {
      make(big[i], 4, 4, 128, 128, QOC_BWD_ONE_WAVE, 100 + i);
      bc.push_back(big[i].ctx);
    }
    CHECK(qoc_batch_run_noalloc(bc.data(), 4, nullptr, nullptr) == QOC_EINVAL);
    CHECK(qoc_batch_run_noalloc(bc.data(), 2, nullptr, nullptr) == QOC_OK);
    read_all(big[1], true);
    for (Sys &s : big) CHECK(qoc_destroy(s.ctx) == QOC_OK);
  }

  // a context flagged by the bound check fails alone (the stand-in flags alpha[0] > 100)
  std::vector<double> big = sys[1].alpha;
  big[0] = 1000.0;
  CHECK(qoc_set_controls(sys[1].ctx, big.data(), sys[1].d, QOC_HOST) == QOC_OK);
  qoc_batch *b = nullptr;
  CHECK(qoc_batch_create(0, 3, 1000, &b) == QOC_OK);
  CHECK(qoc_batch_run(b, ctxs.data(), 3, nullptr, nullptr) == QOC_OK);
  int32_t st3[3];
  CHECK(qoc_batch_status(b, st3, 3) == QOC_OK);
  CHECK(st3[0] == QOC_OK && st3[1] == QOC_ENOTCONV && st3[2] == QOC_OK);
  CHECK(qoc_synchronize(sys[1].ctx) == QOC_OK);           // the flag moved into the batch
  CHECK(qoc_batch_destroy(b) == QOC_OK);
  CHECK(qoc_batch_gradient(ctxs.data(), 3, nullptr) == QOC_ENOTCONV);
  CHECK(qoc_batch_gradient(ctxs.data() + 2, 2, nullptr) == QOC_OK);

  // argument errors
  CHECK(qoc_batch_gradient(nullptr, 1, nullptr) == QOC_EINVAL);
  CHECK(qoc_batch_gradient(ctxs.data(), 0, nullptr) == QOC_EINVAL);
  qoc_batch *b1 = nullptr;
  CHECK(qoc_batch_create(0, 1, 2, &b1) == QOC_OK);
  int32_t s1;
  CHECK(qoc_batch_status(b1, &s1, 1) == QOC_ESTATE);
  CHECK(qoc_batch_run(b1, ctxs.data(), 1, nullptr, nullptr) == QOC_EINVAL);   // more items than capacity
  CHECK(qoc_batch_destroy(b1) == QOC_OK);

  for (Sys &s : sys) CHECK(qoc_destroy(s.ctx) == QOC_OK);
  CHECK(standin_live_device_blocks() == 1 && standin_live_pinned_blocks() == 0);   // the static tables remain
  std::printf("HARNESS OK (%ld launches)\n", standin_launches());
  return 0;
}
