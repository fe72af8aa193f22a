// A host-memory stand-in for the HIP runtime and for the kernel launchers of the library,
// so that the library's host code (qoc_api.cpp: validation, buffers, batch tables, status
// handling) runs on a machine without a GPU under AddressSanitizer and UBSan.
//
// "Device" allocations are ordinary heap blocks; copies and fills are synchronous; streams
// and events are heap objects (a use after destroy is a heap use-after-free).  The launch
// functions do not compute the method: they check every table entry a kernel would read
// against the sizes the host code declared (item and block indices in range, pointers
// non-null), touch the output buffers a kernel would write, and perform the status gather
// exactly.  Test infrastructure only.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

#include "../../paper_2407_13950_amd/csrc/qoc_internal.h"

struct ihipStream_t { int magic = 0x5157; };
struct ihipEvent_t { int magic = 0x4556; int recorded = 0; };

namespace {
std::map<const void *, size_t> g_device;     // live "device" blocks and their sizes
std::map<const void *, size_t> g_pinned;
long g_launches = 0;

[[noreturn]] void die(const char *what) {
  std::fprintf(stderr, "hip stand-in: %s\n", what);
  std::abort();
}
void check_stream(hipStream_t s) {
  if (s && s->magic != 0x5157) die("bad stream");
}
// [p, p + n) must lie inside one live device block
void check_range(const void *p, size_t n, const char *what) {
  if (!p) die(what);
  auto it = g_device.upper_bound(p);
  if (it == g_device.begin()) die(what);
  --it;
  const char *b = static_cast<const char *>(it->first), *q = static_cast<const char *>(p);
  if (q < b || q + n > b + it->second) die(what);
}
}  // namespace

extern "C" {
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipMalloc(void **p, size_t n) {
  *p = std::malloc(n ? n : 1);
  std::memset(*p, 0xA5, n);
  g_device[*p] = n;
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  if (!p) return hipSuccess;
  if (!g_device.erase(p)) die("hipFree of an unknown pointer");
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) {
  *p = std::malloc(n ? n : 1);
  g_pinned[*p] = n;
  return hipSuccess;
}
hipError_t hipHostFree(void *p) {
  if (!p) return hipSuccess;
  if (!g_pinned.erase(p)) die("hipHostFree of an unknown pointer");
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t st) {
  check_stream(st);
  std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemset(void *d, int v, size_t n) {
  std::memset(d, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st) {
  check_stream(st);
  std::memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t st) { check_stream(st); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *st, unsigned int) { *st = new ihipStream_t(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t st) { check_stream(st); delete st; return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t e, unsigned int) {
  check_stream(st);
  if (!e || e->magic != 0x4556) die("bad event");
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st) {
  check_stream(st);
  if (!e || e->magic != 0x4556) die("bad event");
  e->recorded = 1;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (!e || e->magic != 0x4556) die("bad event");
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  if (!e || e->magic != 0x4556) die("bad event");
  delete e;
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  if (a->magic != 0x4556 || b->magic != 0x4556) die("bad event");
  *ms = 1.0f;
  return hipSuccess;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hip stand-in error"; }
}  // extern "C"

long standin_launches() { return g_launches; }
size_t standin_live_device_blocks() { return g_device.size(); }
size_t standin_live_pinned_blocks() { return g_pinned.size(); }

namespace qoc {

// The layouts of the kernel file: lane digits per (q, L) and the dipole variant's index.
bool layout_for(int q, int L, int fp64, int hop, int *ld, int *cpw, int *shape) {
  (void)fp64;
  static const int table[][3] = {{1, 2, 0}, {1, 3, 0}, {1, 4, 0}, {2, 2, 1}, {2, 3, 2}, {2, 4, 1}, {3, 2, 2},
                                 {3, 3, 2}, {3, 4, 3}, {4, 2, 3}, {4, 3, 3}, {4, 4, 3}, {5, 2, 4}, {6, 2, 5}};
  const int n = (int)(sizeof table / sizeof table[0]);
  for (int i = 0; i < n; ++i)
    if (table[i][0] == q && table[i][1] == L) {
      int lpc = 1;
      for (int k = 0; k < table[i][2]; ++k) lpc *= L;
      int p2 = 1;
      while (p2 < lpc) p2 *= 2;
      *ld = table[i][2];
      *cpw = 64 / p2;
      if (shape) *shape = i + (hop ? n : 0);
      return true;
    }
  return false;
}

int small_blocks(const DevSys &s, int kind) {
  switch (kind) {
    case SK_CONTROLS: return (int)((s.NT + 255) / 256);
    case SK_KIT: return 1;
    case SK_BPARTIAL: return s.M;
    case SK_BFINAL: return 1;
    case SK_SERIES: return (int)((s.NT + 255) / 256);
    case SK_PROJECT: return s.q * s.nf * s.d1;
    case SK_GRADW: return s.M > 1 ? (int)(((size_t)(s.M - 1) * s.E * s.N + 255) / 256) : 0;
    default: return 0;
  }
}

static void check_sys(const DevSys &s) {
  const size_t nst = (size_t)s.M * s.E * s.N;
  check_range(s.kstart, sizeof(long long) * (s.M + 1), "kstart");
  check_range(s.alpha, sizeof(double) * 2 * s.d1 * s.q * s.nf, "alpha");
  check_range(s.Ufin, sizeof(double) * 2 * nst, "Ufin");
  check_range(s.lam0, sizeof(double) * 2 * nst, "lam0");
  check_range(s.scal, sizeof(double) * (5 + s.M), "scal");
  check_range(s.series, (s.fp64 ? sizeof(double) : sizeof(float)) * (size_t)s.M * s.ncg_b * s.maxlen * 2 * s.q, "series");
  check_range(s.status, sizeof(int), "status");
  check_range(s.kit, sizeof(int), "kit");
}

// What the phases write that the host reads back: P/terms, the gradients, the count.
static void touch_outputs(const DevSys &s, int phase) {
  if (phase == PHASE_CONTROLS) {
    *s.kit = 4;
    if (s.alpha[0] > 100.0) *s.status |= STATUS_NOTCONV;   // stands in for a failed bound check
  }
  if (phase == PHASE_BOUNDARY)
    for (int i = 0; i < 5 + s.M; ++i) s.scal[i] = 0.5 + i;
  if (phase == PHASE_PROJECT) {
    check_range(s.grad_alpha, sizeof(double) * 2 * s.d1 * s.q * s.nf, "grad_alpha");
    for (int i = 0; i < 2 * s.d1 * s.q * s.nf; ++i) s.grad_alpha[i] = 1.0;
  }
  if (phase == PHASE_GRAD_W && s.M > 1) {
    const size_t n = 2 * (size_t)(s.M - 1) * s.E * s.N;
    check_range(s.grad_W, sizeof(double) * n, "grad_W");
    for (size_t i = 0; i < n; ++i) s.grad_W[i] = 2.0;
  }
}

int launch_phase(const DevSys &s, int phase, hipStream_t st, double *Wout, double *Ufinal) {
  check_stream(st);
  check_sys(s);
  if (phase == PHASE_ROLLOUT) {
    if (Wout && s.M > 1) check_range(Wout, sizeof(double) * 2 * (size_t)(s.M - 1) * s.E * s.N, "roll-out W");
    if (Ufinal) check_range(Ufinal, sizeof(double) * 2 * (size_t)s.E * s.N, "roll-out U");
  }
  touch_outputs(s, phase);
  ++g_launches;
  return 0;
}

static void check_items(const BatchPlan &p, const int4 *items, int n, bool backward) {
  if (n == 0) return;
  check_range(items, sizeof(int4) * n, "item table");
  for (int i = 0; i < n; ++i) {
    const int4 it = items[i];
    check_range(p.sys + it.x, sizeof(DevSys), "item system");
    const DevSys &s = p.sys[it.x];
    if (it.y < 0 || it.y >= s.M) die("item window out of range");
    if (it.z < 0 || it.z >= (backward ? s.ncg_b : s.ncg)) die("item column group out of range");
    int ld, cpw, shape;
    if (!layout_for(s.q, s.L, s.fp64, s.hop, &ld, &cpw, &shape) || shape != it.w) die("item shape");
  }
}

int launch_batch_phase(const BatchPlan &p, int phase, hipStream_t st) {
  check_stream(st);
  static const int kinds[N_PHASES][2] = {{SK_CONTROLS, SK_KIT}, {-1, -1}, {SK_BPARTIAL, SK_BFINAL}, {-1, -1},
                                         {SK_SERIES, SK_PROJECT}, {SK_GRADW, -1}, {-1, -1}};
  if (phase == PHASE_FORWARD) check_items(p, p.fwd_items, p.n_fwd, false);
  if (phase == PHASE_BACKWARD) {
    check_items(p, p.bwd_items, p.n_bwd, true);
    check_items(p, p.xw_items, p.n_xw, true);
    check_items(p, p.x3_items, p.n_x3, true);
    if ((p.n_xw > 0) + (p.n_x3 > 0) + (p.n_bwd > 0) > 1) {
      check_stream(p.aux);
      check_stream(p.aux2);
    }
  }
  for (int k : kinds[phase]) {
    if (k < 0 || p.n_blocks[k] == 0) continue;
    check_range(p.blocks[k], sizeof(int2) * p.n_blocks[k], "block table");
    for (int i = 0; i < p.n_blocks[k]; ++i) {
      const int2 b = p.blocks[k][i];
      check_range(p.sys + b.x, sizeof(DevSys), "block system");
      if (b.y < 0 || b.y >= small_blocks(p.sys[b.x], k)) die("block index out of range");
      check_sys(p.sys[b.x]);
      if (b.y == 0) touch_outputs(p.sys[b.x], phase);
    }
  }
  ++g_launches;
  return 0;
}

// The static tables of the allocation-free run: a "device" block of the declared size.
int noalloc_scratch(int device, void **out) {
  static void *block = nullptr;
  if (device != 0) return (int)hipErrorInvalidDevice;
  if (!block) {
    block = std::malloc(kNoAllocScratchBytes);
    g_device[block] = kNoAllocScratchBytes;
  }
  *out = block;
  return 0;
}

int launch_gather_status(const DevSys *sys, int n, int *out, hipStream_t st) {
  check_stream(st);
  check_range(sys, sizeof(DevSys) * n, "gather systems");
  check_range(out, sizeof(int) * n, "gather output");
  for (int i = 0; i < n; ++i) {
    check_range(sys[i].status, sizeof(int), "gather status");
    out[i] = sys[i].status[0];
    sys[i].status[0] = 0;
  }
  ++g_launches;
  return 0;
}

}  // namespace qoc
