// Internal interface between the C-ABI host code (qoc_api.cpp) and the HIP
// kernels (qoc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/qoc.h"

namespace qoc {

// Everything one evaluation needs on the device, as plain pointers and sizes.
// Complex arrays are interleaved (re, im).  The control table holds the
// propagation precision (float for the FP32 path, double for the FP64 path);
// states, adjoints, reductions and gradients are double in both paths.
struct DevSys {
  int q, L, N, E, nf, d1, M;
  long long NT;
  double T, dt, dtau, mu;
  double nu_L;              // ||a + a^+||_2 for L levels (fixed-point contraction bound)
  int hop;                  // 1: dipole exchange terms of the chain present (kernel variant)
  double hop_c[8];          // (dt/2) J_j for the pairs (j, j+1), j < q-1
  double beta;              // ||D^{-1} (dt/2) H_J||_2 bound: (dt/2) sum_j |J_j| ||a^+ b + a b^+||_2
  int fp64;                 // 1: propagation in double, 0: float
  int ld;                   // lane digits of the register layout
  int cpw;                  // state columns per wavefront
  int ncg;                  // column groups (wavefronts) per window, forward sweep
  int ncg_b;                // column groups per window of the backward sweep (twice as many where it
                            // splits state and adjoint over the halves of a wavefront)
  long long maxlen;         // longest window, steps
  int ckpt_every;           // checkpoint spacing in steps (0 = none)
  int ncp;                  // checkpoints stored per window
  int kit_fixed;            // > 0: fixed-point iterations forced by the caller
  int bwd_sched;            // backward-sweep schedule: QOC_BWD_AUTO, _ONE_WAVE or _TWO_WAVES
  double solve_tol;         // per-step truncation target of the fixed point

  const long long *kstart;  // [M+1] first step of each window (floor split)
  const double *carrier;    // [q*nf] rad/ns
  const double *dinv;       // [2N] complex: 1/(1 + i dt/2 h_r)
  const int *ess_row;       // [E]
  const double *V;          // [2*N*E] target embedded in the essential rows, column-major
  const double *alpha;      // [d]
  const double *W;          // [2*(M-1)*E*N]: W^1..W^{M-1}, column-major N x E each

  void *ctrl;               // [NT*q] complex T: (dt/2) * 2 pi d_j(t_{k+1/2})
  double *Ufin;             // [2*M*E*N] complex: U^m(t_m)
  double *lam0;             // [2*M*E*N] complex: propagated adjoint at t_{m-1}
  double *ckpt;             // [2*M*ncp*E*N] complex checkpoints
  double *partials;         // [4*M]
  double *scal;             // [5+M]: P, J, penalty, |U^M|^2, Re gamma, Im gamma, |C^1|^2..|C^{M-1}|^2
  double *series;           // [M*ncg*maxlen*2q] in the propagation precision: per wavefront and step,
                            // Im<y,(a+a^+)z>, Re<y,(a-a^+)z>
  double *xy;               // [NT*2q]: the same summed over the window's columns
  double *grad_alpha;       // [d]
  double *grad_W;           // [2*(M-1)*E*N]
  int *kit;                 // [1] fixed-point iterations in use
  unsigned int *rho_bits;   // [1] max per-step contraction bound (float bits), reset by k_kit
  int *status;              // [1] device-side status bits (QOC_STATUS_*)
};

enum { STATUS_NOTCONV = 1 };

// Layout chosen for a (q, L) pair: lane digits, columns per wavefront and the
// kernel-instance index (the dipole variant when hop is set).  Returns false when
// no kernel instance exists for the pair.
bool layout_for(int q, int L, int fp64, int hop, int *ld, int *cpw, int *shape);

// Phases of one evaluation, launched in this order on one stream:
// objective = CONTROLS, FORWARD, BOUNDARY; gradient adds BACKWARD, PROJECT, GRAD_W.
// ROLLOUT (after CONTROLS) is the single-window propagation over [0, T].
enum Phase { PHASE_CONTROLS = 0, PHASE_FORWARD, PHASE_BOUNDARY, PHASE_BACKWARD, PHASE_PROJECT, PHASE_GRAD_W,
             PHASE_ROLLOUT, N_PHASES };

// The small FP64 kernels; small_blocks() gives each one's block count for a system.
enum SmallKind { SK_CONTROLS = 0, SK_KIT, SK_BPARTIAL, SK_BFINAL, SK_SERIES, SK_PROJECT, SK_GRADW, SK_COUNT };
int small_blocks(const DevSys &s, int kind);

// Returns 0 or a hipError_t value.
int launch_phase(const DevSys &s, int phase, hipStream_t st, double *Wout = nullptr, double *Ufinal = nullptr);

// Several systems evaluated together: the propagation phases run as one launch
// over all (system, window, column group) items, each small kernel as one launch
// over a (system, block) table.  All systems share the precision `fp64`.
// Wavefronts per backward item: the caller's schedule or, by default, several when the
// launch would otherwise leave SIMDs idle -- at most 1024 items (one wavefront per SIMD)
// in FP32, 256 in FP64, whose solving wavefronts need more registers -- and one
// otherwise.  "Several" is three for layouts with one column per wavefront (state,
// adjoint, inner products) and two for the others (the solves of both halves, and the
// inner products).  Two wavefronts on a one-column layout (state and adjoint, the inner
// products on the adjoint's chain) only on request.  A function of the system and its
// schedule setting alone, so a batched evaluation makes the same choice as a solo one.
#ifndef QOC_MULTI_WAVE_MAX_ITEMS_FP32
#define QOC_MULTI_WAVE_MAX_ITEMS_FP32 1024
#endif
#ifndef QOC_MULTI_WAVE_MAX_ITEMS_FP64
#define QOC_MULTI_WAVE_MAX_ITEMS_FP64 256
#endif
inline int bwd_waves(const DevSys &s) {
  if (s.bwd_sched == QOC_BWD_ONE_WAVE) return 1;
  if (s.bwd_sched == QOC_BWD_TWO_WAVES) return 2;
  if (s.bwd_sched == QOC_BWD_THREE_WAVES) return s.cpw == 1 ? 3 : 1;
  const long long items = (long long)s.M * s.ncg_b;
  if (items > (s.fp64 ? QOC_MULTI_WAVE_MAX_ITEMS_FP64 : QOC_MULTI_WAVE_MAX_ITEMS_FP32)) return 1;
  return s.cpw == 1 ? 3 : 2;
}

struct BatchPlan {
  const DevSys *sys;              // [n] device copy of the systems
  const int4 *fwd_items;          // [n_fwd] (system, window, column group, shape), longest first
  const int4 *bwd_items;          // [n_bwd]
  const int4 *xw_items;           // [n_xw] backward items of two wavefronts each (bwd_waves == 2)
  const int4 *x3_items;           // [n_x3] backward items of three wavefronts each (bwd_waves == 3)
  int n_fwd, n_bwd, n_xw, n_x3;
  hipStream_t aux, aux2;          // the xw and x3 items run there, forked from and joined to the caller's stream
  hipEvent_t fork, join, join2;
  const int2 *blocks[SK_COUNT];   // per small kernel: (system, block within the system)
  int n_blocks[SK_COUNT];
  int fp64;
};
int launch_batch_phase(const BatchPlan &p, int phase, hipStream_t st);
// out[i] = status word of sys[i] (device copies), which is cleared; i < n.
int launch_gather_status(const DevSys *sys, int n, int *out, hipStream_t st);

// Tables of the allocation-free batched run: a static device array of this many bytes per
// GPU.  noalloc_scratch() returns its address on `device` (which must be current), looked
// up once per device; 0 or a hipError_t value.
#ifndef QOC_NOALLOC_SCRATCH_BYTES
#define QOC_NOALLOC_SCRATCH_BYTES ((size_t)4 << 20)
#endif
constexpr size_t kNoAllocScratchBytes = QOC_NOALLOC_SCRATCH_BYTES;
int noalloc_scratch(int device, void **out);

// ---- optimisation driver (qoc_opt.cpp) and its FP64 kernels (qoc_opt_kernels.hip).
// Reductions use kOptGrid partial sums (partials: >= kOptGrid doubles) finished by one
// block in a fixed order; results land in device memory.  All return 0 or a hipError_t.
constexpr int kOptGrid = 512;
int opt_dot(const double *a, const double *b, long long n, double *partials, double *out, hipStream_t st);
// out[0] = cb * base[0] + cs * (a . b) (base may be NULL: out[0] = cs * (a . b)), all on the device
int opt_dot_to(const double *a, const double *b, long long n, double *partials, double *out, double cs,
               const double *base, double cb, hipStream_t st);
int opt_axpy_dev(double *y, const double *c, double s, const double *x, long long n, hipStream_t st);  // y += s c[0] x
int opt_maxabs(const double *v, long long n, double *partials, double *out, hipStream_t st);
int opt_axpby(double *y, double a, const double *x, double b, long long n, hipStream_t st);       // y = a x + b y
int opt_trial(double *xt, const double *x, const double *p, double t, long long n, long long d, double lo, double hi,
              hipStream_t st);                                                                       // clip(x + t p)
int opt_reduced(double *out, const double *v, const double *x, const double *g, long long n, long long d, double lo,
                double hi, hipStream_t st);                                                          // v off the active set
int opt_assemble(double *g, const double *ga, const double *alpha, const double *gE, const double *gW, long long d,
                 long long nW, double gtik, double gen, double s, hipStream_t st);
int opt_energy_blocks(const DevSys &s);                 // partials needed by opt_energy
// sum_k sum_j |d_j(t_{k+1/2})|^2 -> out; d_j per step -> dtab [2*NT*q]
int opt_energy(const DevSys &s, const double *alpha, double *dtab, double *partials, double *out, hipStream_t st);
int opt_energy_grad(const DevSys &s, const double *dtab, double *gE, hipStream_t st);

}  // namespace qoc

// Host-side views of a context for the optimisation driver (defined in qoc_api.cpp).
struct qoc_ctx;
namespace qoc {
const DevSys &ctx_dev(const qoc_ctx *ctx);
hipStream_t ctx_stream(const qoc_ctx *ctx);
int ctx_device(const qoc_ctx *ctx);
int set_error(int code, const char *msg);      // records the message for qoc_last_error, returns code
}  // namespace qoc
