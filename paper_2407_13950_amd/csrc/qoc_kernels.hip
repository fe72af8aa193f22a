// CDNA4 (gfx950) kernels for the multiple-shooting penalty objective and its
// discrete-adjoint gradient (arxiv 2407.13950).
//
// Data path of one objective+gradient evaluation:
//   k_kit            fixed-point iteration count from a 2-norm contraction bound
//   k_controls       per time step: (dt/2) * 2 pi d_j(t_{k+1/2})                        (Sec. 2, eq. dj-ctrl)
//   k_forward        per (window, column group): implicit-midpoint propagation from W^{m-1}
//                    with the state held in registers for the whole window               (Sec. 3, eqs. sch-op/sch-ic; Sec. 5)
//   k_boundary_*     FP64 penalty |U^m - W^m|^2, |U^M|^2, gamma = <V, U^M>, P            (eqs. mod-infid, penalty-fcn)
//   k_backward       per (window, column group): terminal condition (eq. terminal), reverse
//                    reconstruction of U and the discrete adjoint in one fused sweep, per-step
//                    inner products for the control gradient                            (eq. grad-int, discrete form)
//   k_series_reduce  sum of the per-step inner products over a window's column groups
//   k_project        B-spline x carrier projection onto dP/dalpha (FP64)
//   k_grad_W         dP/dW^m = mu (W^m - U^m) - 2 Lambda^{m+1}(t_m)                      (App. B, eq. dT-dW-j)
//
// Register layout of the propagation kernels.  A state column of N = L^q
// entries is spread over LPC = L^LD lanes of one wavefront; each lane holds
// EPL = L^(q-LD) entries in registers.  Row r = e*LPC + sub, where e is the
// register slot and sub the lane's position in its column.  The q digits of r
// (qubit 0 most significant) split into "register digits" (the leading q-LD,
// encoded in e) and "lane digits" (the trailing LD, encoded in sub).  A ladder
// operator on a register digit reads another register of the same lane (no data
// movement); on a lane digit it reads the lane +-L^k away, through a per-wavefront
// LDS exchange (see lane exchange).  A wavefront holds CPW = 64/pow2ceil(LPC)
// columns of one window, so all its lanes see the same control values at every step.
//
// One fixed-point (Jacobi) iteration for (I + i dt/2 H) z = u with the diagonal
// drift D = I + i dt/2 diag(h) split off:  z <- D^{-1} (u - i S), S = (dt/2) H_c z.
// For even L the registers are instead arranged by colour (red-black slot layout,
// see Geo): H_c only couples rows of opposite digit-sum parity, so the solve
// refreshes one colour at a time from the other's newest values, which reaches the
// Jacobi error bound of K iterations in K+1 half sweeps of half the work each.
// The optional dipole exchange of the chain (eq. sys-ham) joins the iteration in
// a second instance of every sweep kernel (HOP): it keeps the digit-sum parity, so
// a colour takes it from its own current values.
#include "qoc_internal.h"

#include <cmath>
#include <cstdio>
#include <mutex>

namespace qoc {
namespace {

constexpr int cipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}
constexpr int cpow2(int x) { return x <= 1 ? 1 : 2 * cpow2((x + 1) / 2); }

template <typename T> struct C2 { using type = float2; };
template <> struct C2<double> { using type = double2; };

// a*b + c as one fused instruction (the compiler would otherwise pair some products
// with separate adds when expressions combine several products).
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// s += a*v and s += conj(a)*v on split complex values, four fused operations each.
template <typename T>
__device__ __forceinline__ void cmac(T &sr, T &si, T ar, T ai, T vr, T vi) {
  sr = fma_(ar, vr, sr); sr = fma_(-ai, vi, sr);
  si = fma_(ar, vi, si); si = fma_(ai, vr, si);
}
template <typename T>
__device__ __forceinline__ void cmac_conj(T &sr, T &si, T ar, T ai, T vr, T vi) {
  sr = fma_(ar, vr, sr); sr = fma_(ai, vi, sr);
  si = fma_(ar, vi, si); si = fma_(-ai, vr, si);
}

template <typename T, int Q, int L, int LD>
struct Geo {
  static constexpr int N = cipow(L, Q);
  static constexpr int R = Q - LD;               // register digits
  static constexpr int EPL = cipow(L, R);        // entries per lane
  static constexpr int LPC = cipow(L, LD);       // lanes per column
  static constexpr int LPCP = cpow2(LPC);        // padded to a power of two
  static constexpr int CPW = 64 / LPCP;          // columns per wavefront
  static_assert(LPCP <= 64, "a column must fit in one wavefront");
  static constexpr int rstride(int j) { return cipow(L, R - 1 - j); }   // register digit j < R
  static constexpr int rdigit(int e, int j) { return (e / rstride(j)) % L; }
  static constexpr int lstride(int jj) { return cipow(L, LD - 1 - jj); } // lane digit jj (qubit R+jj)
  // Red-black slot layout (even L, at least one register digit).  An entry is red or black
  // by the parity of its digit sum; every ladder term couples the two colours.  Slot
  // i = c*H + s0*RT + t holds the entry of colour c whose leading register digit is
  // l0 = 2*s0 + b and whose remaining register digits form t, with b = (lane parity) ^
  // par(t) ^ c.  Layouts with every digit on lanes (one entry per lane) iterate Jacobi-style.
  static constexpr bool RB = (L % 2) == 0 && R >= 1;
  static constexpr int H = EPL / 2;              // slots per colour
  static constexpr int HALF = L / 2;             // values of s0
  static constexpr int RT = EPL / L;             // tuples of register digits 1..R-1
  static constexpr int tpar(int t) { return t == 0 ? 0 : (tpar(t / L) ^ ((t % L) & 1)); }
  static_assert(!RB || R >= 1, "red-black layout needs a register digit");
};

// Blocks are dealt to the 8 XCDs round-robin; map consecutive work items
// (column groups of one window, which read the same control-table slice) to
// one XCD's L2.  The grid is padded to a multiple of 8; items past the end exit.
__device__ __forceinline__ int xcd_item(int b, int nblk) {
  const int per = nblk / 8;
  return (b % 8) * per + b / 8;
}

__device__ __forceinline__ double bspline2(double x) {
  const double a = fabs(x);
  if (a < 0.5) return 0.75 - a * a;
  if (a < 1.5) return 0.5 * (a - 1.5) * (a - 1.5);
  return 0.0;
}

// ---------------------------------------------------------------------------- lane exchange

// Lane-digit ladder terms read values held by other lanes of the wavefront.  Each
// lane writes a record of NV values to a per-wavefront LDS buffer and reads the
// records of the lanes +-ST away (one 16-byte access per four floats).  kGuard
// records on both sides of the 64 lane records cover reads past the wavefront's
// ends; the buffer is zeroed once per launch and afterwards only ever holds state
// values, and every read outside a lane's own digit block meets a zero ladder
// weight.  LDS operations of one wavefront complete in issue order, so the
// exchange needs no wait, only compiler ordering (wave_sync).
constexpr int kGuard = 16;                      // >= every lane-digit stride
// Values per record: 2*EPL with EPL <= 4; twice that with the dipole exchange, whose
// records also carry the refreshed colour's own values.
constexpr int kXchgMaxNV = 16;
template <typename T, bool HOP>
constexpr int xchg_bytes() { return (64 + 2 * kGuard) * (HOP ? 16 : 8) * (int)sizeof(T); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Zero the whole exchange buffer (64 lanes, 16 bytes per store).
template <typename T, bool HOP>
__device__ __forceinline__ void xchg_clear(T *buf) {
  float4 *p = reinterpret_cast<float4 *>(buf);
  for (int i = threadIdx.x & 63; i < xchg_bytes<T, HOP>() / 16; i += 64) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  wave_sync();
}

// v[0..NV) -> record of lane `lane`;  record of lane `lane + D` -> v[0..NV).
// A record is split into planes of PW bytes (16 when the record size allows it,
// else 8); plane p of all 64 + 2 kGuard lanes is contiguous, so the 64 lanes of
// one access touch consecutive PW-byte words (no bank conflicts) and every access
// stays PW-aligned.
template <typename T, int NV>
struct XRec {
  static_assert(NV <= kXchgMaxNV && (NV * sizeof(T)) % 8 == 0, "exchange record");
  static constexpr int BYTES = NV * (int)sizeof(T);
  static constexpr int PW = BYTES % 16 == 0 ? 16 : 8;          // plane width in bytes
  static constexpr int PE = PW / (int)sizeof(T);               // values per plane
  static constexpr int NP = BYTES / PW;                        // planes
  static constexpr int PSTRIDE = (64 + 2 * kGuard) * PE;       // values between planes
};

template <typename T, int NV>
__device__ __forceinline__ void xput(T *buf, int lane, const T *v) {
  using X = XRec<T, NV>;
  T *p = buf + (kGuard + lane) * X::PE;
#pragma unroll
  for (int q = 0; q < X::NP; ++q) {
    const T *s = v + q * X::PE;
    T *d = p + q * X::PSTRIDE;
    if constexpr (X::PW == 16 && sizeof(T) == 4) *reinterpret_cast<float4 *>(d) = make_float4(s[0], s[1], s[2], s[3]);
    else if constexpr (X::PW == 16) *reinterpret_cast<double2 *>(d) = make_double2(s[0], s[1]);
    else if constexpr (sizeof(T) == 4) *reinterpret_cast<float2 *>(d) = make_float2(s[0], s[1]);
    else d[0] = s[0];
  }
}
template <typename T, int NV, int D>
__device__ __forceinline__ void xget(const T *buf, int lane, T *v) {
  static_assert(D >= -kGuard && D <= kGuard, "lane shift beyond the guard records");
  using X = XRec<T, NV>;
  const T *p = buf + (kGuard + lane + D) * X::PE;
#pragma unroll
  for (int q = 0; q < X::NP; ++q) {
    T *d = v + q * X::PE;
    const T *s = p + q * X::PSTRIDE;
    if constexpr (X::PW == 16 && sizeof(T) == 4) {
      const float4 c = *reinterpret_cast<const float4 *>(s);
      d[0] = c.x; d[1] = c.y; d[2] = c.z; d[3] = c.w;
    } else if constexpr (X::PW == 16) {
      const double2 c = *reinterpret_cast<const double2 *>(s);
      d[0] = c.x; d[1] = c.y;
    } else if constexpr (sizeof(T) == 4) {
      const float2 c = *reinterpret_cast<const float2 *>(s);
      d[0] = c.x; d[1] = c.y;
    } else {
      d[0] = s[0];
    }
  }
}

// record of lane `src` (0..63) -> v[0..NV)
template <typename T, int NV>
__device__ __forceinline__ void xget_from(const T *buf, int src, T *v) {
  using X = XRec<T, NV>;
  const T *p = buf + (kGuard + src) * X::PE;
#pragma unroll
  for (int q = 0; q < X::NP; ++q) {
    const T *sp = p + q * X::PSTRIDE;
#pragma unroll
    for (int i = 0; i < X::PE; ++i) v[q * X::PE + i] = sp[i];
  }
}

// ---------------------------------------------------------------------------- per-lane state

template <typename T, int Q, int L, int LD>
struct Lane {
  using G = Geo<T, Q, L, LD>;
  static constexpr int NH = G::RB ? G::HALF : 1;
  int lane, sub, col, par;
  bool valid;
  T *xb;                                            // this wavefront's exchange buffer (LDS)
  T wlo[LD > 0 ? LD : 1], whi[LD > 0 ? LD : 1];     // sqrt(l+1) (0 at the top level), sqrt(l) (0 at l = 0)
  // red-black layout: ladder weights on the leading register digit for an output
  // slot (s0, class beta), l0 = 2*s0 + (par ^ beta): sqrt(l0+1) and sqrt(l0), 0 off the ends
  T wup[2][NH], wdn[2][NH];
  T dr[G::EPL], di[G::EPL];                         // D^{-1} per entry
  // D^{-1} - 1 split into a rounded part and its remainder.  The same factor
  // multiplies every step, so in FP32 its rounding error would accumulate
  // linearly over a window; the remainder removes that drift.
  T mr[G::EPL], mi[G::EPL], mrl[G::EPL], mil[G::EPL];
  // Dipole exchange weights, (dt/2) J_j included (set by init_hop, dead otherwise).
  // Term A of the pair (j, j+1) reads the row with l_j + 1, l_{j+1} - 1 (weight
  // sqrt(l_j + 1) sqrt(l_{j+1})), term B the row with l_j - 1, l_{j+1} + 1 (weight
  // sqrt(l_j) sqrt(l_{j+1} + 1)), both zero off the ends of the digits.
  static constexpr int NPL = LD > 1 ? LD - 1 : 1;
  T hla[NPL], hlb[NPL];         // lane-digit pairs (R+jj, R+jj+1): full A and B weights
  T hsa, hsb;                   // pair (R-1, R): (dt/2) J_{R-1} sqrt(l_R), (dt/2) J_{R-1} sqrt(l_R + 1)

  // half: the two halves of the wavefront hold the same CPW/2 columns (split backward sweep)
  __device__ void init(const DevSys &s, int cg, T *xbuf, bool half = false) {
    xb = xbuf;
    lane = threadIdx.x & 63;                        // lane within this wavefront
    const int hl = half ? (lane & 31) : lane;
    const int slot = hl / G::LPCP;
    sub = hl % G::LPCP;
    col = cg * (half ? G::CPW / 2 : G::CPW) + slot;
    valid = (sub < G::LPC) && (col < s.E);
    par = 0;
#pragma unroll
    for (int jj = 0; jj < LD; ++jj) {
      const int st = G::lstride(jj);
      const int l = valid ? (sub / st) % L : 0;
      par ^= l & 1;
      wlo[jj] = (valid && l < L - 1) ? (T)sqrt((double)(l + 1)) : (T)0;
      whi[jj] = (valid && l > 0) ? (T)sqrt((double)l) : (T)0;
    }
#pragma unroll
    for (int beta = 0; beta < 2; ++beta)
#pragma unroll
      for (int s0 = 0; s0 < NH; ++s0) {
        const int l0 = 2 * s0 + (par ^ beta);
        wup[beta][s0] = (valid && l0 < L - 1) ? (T)sqrt((double)(l0 + 1)) : (T)0;
        wdn[beta][s0] = (valid && l0 > 0) ? (T)sqrt((double)l0) : (T)0;
      }
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      const int r = row(e);
      const double a = valid ? s.dinv[2 * r] : 1.0, b = valid ? s.dinv[2 * r + 1] : 0.0;
      dr[e] = (T)a;
      di[e] = (T)b;
      mr[e] = (T)(a - 1.0);
      mi[e] = (T)b;
      mrl[e] = (T)((a - 1.0) - (double)mr[e]);
      mil[e] = (T)(b - (double)mi[e]);
    }
  }
  __device__ void init_hop(const DevSys &s) {
    int l[LD > 0 ? LD : 1];
#pragma unroll
    for (int jj = 0; jj < LD; ++jj) l[jj] = valid ? (sub / G::lstride(jj)) % L : 0;
#pragma unroll
    for (int jj = 0; jj < NPL; ++jj) {
      hla[jj] = hlb[jj] = (T)0;
      if (jj + 1 < LD && valid) {
        const double J = s.hop_c[G::R + jj];
        const int a = l[jj], b = l[jj + 1];
        hla[jj] = (T)((a < L - 1 && b > 0) ? J * sqrt((double)(a + 1)) * sqrt((double)b) : 0.0);
        hlb[jj] = (T)((a > 0 && b < L - 1) ? J * sqrt((double)a) * sqrt((double)(b + 1)) : 0.0);
      }
    }
    hsa = hsb = (T)0;
    if (LD > 0 && G::R >= 1 && valid) {
      const double J = s.hop_c[G::R - 1];
      hsa = (T)(J * sqrt((double)l[0]));
      hsb = (T)(l[0] < L - 1 ? J * sqrt((double)(l[0] + 1)) : 0.0);
    }
  }
  // row of the state column held in register slot e
  __device__ __forceinline__ int row(int e) const {
    if constexpr (G::RB) {
      const int c = e / G::H, s0 = (e % G::H) / G::RT, t = e % G::RT;
      const int l0 = 2 * s0 + (par ^ G::tpar(t) ^ c);
      return (l0 * G::RT + t) * G::LPC + sub;
    } else {
      return e * G::LPC + sub;
    }
  }
  // x = (D^{-1} - 1) u  (CONJ: (conj(D)^{-1} - 1) u), remainder first.
  template <bool CONJ>
  __device__ __forceinline__ void scale_m1(int e, T ur, T ui, T &xr, T &xi) const {
    const T sg = CONJ ? (T)-1 : (T)1;
    if constexpr (sizeof(T) == 4) {
      xr = fma_(-sg * mi[e], ui, fma_(mr[e], ur, fma_(-sg * mil[e], ui, mrl[e] * ur)));
      xi = fma_(sg * mi[e], ur, fma_(mr[e], ui, fma_(sg * mil[e], ur, mrl[e] * ui)));
    } else {
      xr = mr[e] * ur - sg * mi[e] * ui;
      xi = mr[e] * ui + sg * mi[e] * ur;
    }
  }
};

// Lane-digit ladder terms for K complex values per lane: for every lane digit,
// S[o] += lo * v'[o] + hi * v''[o] with v', v'' the values o of the lanes one digit
// step up and down (lo = c'_j sqrt(l+1), hi = conj(c'_j) sqrt(l), zero off the ends).
// All neighbour records are requested before the first is used, so their LDS
// latencies overlap.
template <typename T, int LD, int K, int JJ>
struct LaneGets {
  template <typename LaneT>
  __device__ __forceinline__ static void load(const LaneT &ln, T (*n)[2 * K]) {
    if constexpr (JJ < LD) {
      constexpr int ST = LaneT::G::lstride(JJ);
      xget<T, 2 * K, ST>(ln.xb, ln.lane, n[2 * JJ]);
      xget<T, 2 * K, -ST>(ln.xb, ln.lane, n[2 * JJ + 1]);
      LaneGets<T, LD, K, JJ + 1>::load(ln, n);
    }
  }
};

// Two-level layouts: the neighbour of a lane along a lane digit of stride ST (1, 2, 4
// or 8, within a row of 16 lanes) is lane ^ ST, whichever way the digit steps (the
// other direction meets a zero weight).  DPP moves read it straight from that lane's
// register: xor 1 and 2 are quad permutations, xor 4 mirrors each half row and then
// reverses each quad ((i ^ 7) ^ 3 = i ^ 4), xor 8 rotates the row by 8.  No LDS round
// trip.
// The dipole pairs of adjacent digits read lane ^ (st_j | st_j+1): xor 3 reverses each
// quad, xor 6 mirrors each half row and swaps neighbours ((i ^ 7) ^ 1), xor 12 mirrors
// the row and reverses each quad ((i ^ 15) ^ 3).
template <int M>
__device__ __forceinline__ float lane_xor(float v) {
  constexpr int QP1 = 0xB1, QP2 = 0x4E, QP3 = 0x1B;     // quad_perm [1,0,3,2], [2,3,0,1], [3,2,1,0]
  constexpr int HMIR = 0x141, MIR = 0x140, ROR8 = 0x128; // row_half_mirror, row_mirror, row_ror:8
  int x = __float_as_int(v);
  if constexpr (M == 1) {
    x = __builtin_amdgcn_update_dpp(0, x, QP1, 0xF, 0xF, true);
  } else if constexpr (M == 2) {
    x = __builtin_amdgcn_update_dpp(0, x, QP2, 0xF, 0xF, true);
  } else if constexpr (M == 3) {
    x = __builtin_amdgcn_update_dpp(0, x, QP3, 0xF, 0xF, true);
  } else if constexpr (M == 4) {
    x = __builtin_amdgcn_update_dpp(0, x, HMIR, 0xF, 0xF, true);
    x = __builtin_amdgcn_update_dpp(0, x, QP3, 0xF, 0xF, true);
  } else if constexpr (M == 6) {
    x = __builtin_amdgcn_update_dpp(0, x, HMIR, 0xF, 0xF, true);
    x = __builtin_amdgcn_update_dpp(0, x, QP1, 0xF, 0xF, true);
  } else if constexpr (M == 8) {
    x = __builtin_amdgcn_update_dpp(0, x, ROR8, 0xF, 0xF, true);
  } else {
    static_assert(M == 12, "lane xor beyond a row of 16 lanes");
    x = __builtin_amdgcn_update_dpp(0, x, MIR, 0xF, 0xF, true);
    x = __builtin_amdgcn_update_dpp(0, x, QP3, 0xF, 0xF, true);
  }
  return __int_as_float(x);
}

// The lane exchange (and the dipole terms' reads) run through DPP for FP32 two-level
// layouts with at most four lane digits, with no LDS records at all.
template <typename T, int L, int LD>
__device__ __forceinline__ constexpr bool dpp_layout() {
  return sizeof(T) == 4 && L == 2 && LD >= 1 && LD <= 4;
}

template <int M, typename T, int NV>
__device__ __forceinline__ void xor_record(const T *own, T *out) {
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = lane_xor<M>(own[i]);
}

template <typename T, int LD, int K, int JJ>
struct DppGets {
  template <typename G>
  __device__ __forceinline__ static void load(const T *rec, T (*n)[2 * K]) {
    if constexpr (JJ < LD) {
      constexpr int ST = G::lstride(JJ);
#pragma unroll
      for (int i = 0; i < 2 * K; ++i) {
        n[2 * JJ][i] = lane_xor<ST>(rec[i]);
        n[2 * JJ + 1][i] = n[2 * JJ][i];
      }
      DppGets<T, LD, K, JJ + 1>::template load<G>(rec, n);
    }
  }
};

// Writes this lane's K complex values to the exchange.  FP32, and FP64 records of at most
// three complex values (one right-hand side), also request all neighbours' records at once
// (n[2jj]: lane digit jj one step up, n[2jj+1]: one step down), so their latencies overlap
// with the lane-independent work the caller does before lane_digit_terms; larger FP64
// records (both right-hand sides of the backward sweep: twice the registers) are read only
// where they are used.
template <typename T, int K> struct XPre { static constexpr bool value = sizeof(T) == 4 || K <= 3; };

// Planes after the first record's: a second record of KO complex values (the
// dipole exchange's own-colour values) rides in the same exchange.
template <typename T, int K>
__device__ __forceinline__ constexpr int xtail() { return XRec<T, 2 * K>::NP * XRec<T, 2 * K>::PSTRIDE; }

template <typename T, int Q, int L, int LD, int K, int KO = 0>
__device__ __forceinline__ void lane_exchange(const Lane<T, Q, L, LD> &ln, const T *vr, const T *vi,
                                              T (*n)[2 * K], const T *wr = nullptr, const T *wi = nullptr) {
  if constexpr (LD > 0) {
    T rec[2 * K];
#pragma unroll
    for (int o = 0; o < K; ++o) {
      rec[2 * o] = vr[o];
      rec[2 * o + 1] = vi[o];
    }
    if constexpr (dpp_layout<T, L, LD>()) {
      DppGets<T, LD, K, 0>::template load<Geo<T, Q, L, LD>>(rec, n);
      return;
    }
    xput<T, 2 * K>(ln.xb, ln.lane, rec);
    if constexpr (KO > 0) {
      static_assert(XRec<T, 2 * KO>::PE == XRec<T, 2 * K>::PE, "records of one exchange share the plane width");
      T rec2[2 * KO];
#pragma unroll
      for (int o = 0; o < KO; ++o) {
        rec2[2 * o] = wr[o];
        rec2[2 * o + 1] = wi[o];
      }
      xput<T, 2 * KO>(ln.xb + xtail<T, K>(), ln.lane, rec2);
    }
    wave_sync();
    if constexpr (XPre<T, K>::value) {
      LaneGets<T, LD, K, 0>::load(ln, n);
      // keep the caller's register-digit arithmetic after the reads' issue, where it covers
      // their latency (left alone, the scheduler places it between the write and the reads)
      __builtin_amdgcn_sched_barrier(0);
      wave_sync();
    }
  }
}

template <typename T, int Q, int L, int LD, int K, int JJ = 0>
__device__ __forceinline__ void lane_digit_terms(const Lane<T, Q, L, LD> &ln, const T *lor, const T *loi,
                                                 const T *hir, const T *hii, T (*n)[2 * K], T *Sr, T *Si) {
  if constexpr (JJ < LD) {
    constexpr int ST = Geo<T, Q, L, LD>::lstride(JJ);
    if constexpr (!XPre<T, K>::value) {
      xget<T, 2 * K, ST>(ln.xb, ln.lane, n[0]);
      xget<T, 2 * K, -ST>(ln.xb, ln.lane, n[1]);
    }
    const T *up = XPre<T, K>::value ? n[2 * JJ] : n[0];
    const T *dn = XPre<T, K>::value ? n[2 * JJ + 1] : n[1];
    if constexpr (dpp_layout<T, L, LD>()) {
      // two levels: up and dn are the same lane and one of the two weights is zero, so
      // one product with their sum gives the same value (half the multiply-adds)
      const T cr = lor[JJ] + hir[JJ], ci = loi[JJ] + hii[JJ];
#pragma unroll
      for (int o = 0; o < K; ++o) cmac(Sr[o], Si[o], cr, ci, up[2 * o], up[2 * o + 1]);
    } else {
#pragma unroll
      for (int o = 0; o < K; ++o) {
        cmac(Sr[o], Si[o], lor[JJ], loi[JJ], up[2 * o], up[2 * o + 1]);
        cmac(Sr[o], Si[o], hir[JJ], hii[JJ], dn[2 * o], dn[2 * o + 1]);
      }
    }
    lane_digit_terms<T, Q, L, LD, K, JJ + 1>(ln, lor, loi, hir, hii, n, Sr, Si);
  } else if constexpr (LD > 0 && !XPre<T, K>::value) {
    wave_sync();
  }
}

// ---------------------------------------------------------------------------- dipole exchange terms

// S += (dt/2) H_J v, H_J = sum_j J_j (a_{j+1}^+ a_j + a_{j+1} a_j^+) (eq. sys-ham, chain),
// on NO output slots for NRHS right-hand sides.  The exchange keeps the digit sum,
// so in the red-black layout (C >= 0) an output slot of colour C reads the current
// values of colour C (C < 0: plain layout, all EPL slots).  The layouts keep one
// register digit (R = 1), so every pair involves a lane digit and every source value
// comes from another lane: from the records at `base`, written by the caller's lane
// exchange (red-black: the own-colour values, record[b*NO + o], o the slot within the
// colour, sent behind the ladder's record; plain layout: the ladder's record itself).
// Every read of a value that lies outside the digit range meets a zero weight.

// Red-black output slot s0 of colour C, pair (register digit, first lane digit): the
// source row (l0 +- 1, lane digit -+ 1) sits in the neighbouring lane, whose lead
// parity is the other one, so A (l0 + 1) is its slot s0 + b and B (l0 - 1) its slot
// s0 - 1 + b, b the output's lead parity.
template <int HALF>
__device__ __forceinline__ constexpr int lead_up(int s0, int b) { return s0 + b < HALF ? s0 + b : s0; }
template <int HALF>
__device__ __forceinline__ constexpr int lead_dn(int s0, int b) { return s0 - 1 + b >= 0 ? s0 - 1 + b : s0; }

template <typename T, int Q, int L, int LD, int C, int NRHS, int JJ>
__device__ __forceinline__ void hop_lane_pairs(const Lane<T, Q, L, LD> &ln, const T *base, const T *own, T *Sr,
                                               T *Si) {
  using G = Geo<T, Q, L, LD>;
  if constexpr (JJ + 1 < LD) {
    constexpr int NO = C >= 0 ? G::H : G::EPL;
    constexpr int NV = 2 * NO * NRHS;
    constexpr int OFF = G::lstride(JJ) - G::lstride(JJ + 1);   // A: l_jj + 1, l_jj+1 - 1
    T a[NV], b[NV];
    if constexpr (dpp_layout<T, L, LD>()) {     // two levels: A and B both read lane ^ (st_jj | st_jj+1)
      xor_record<G::lstride(JJ) + G::lstride(JJ + 1), T, NV>(own, a);
#pragma unroll
      for (int i = 0; i < NV; ++i) b[i] = a[i];
    } else {
      xget<T, NV, OFF>(base, ln.lane, a);
      xget<T, NV, -OFF>(base, ln.lane, b);
    }
    if constexpr (dpp_layout<T, L, LD>()) {     // same operand, one of the weights zero: one product
      const T w = ln.hla[JJ] + ln.hlb[JJ];
#pragma unroll
      for (int i = 0; i < NO * NRHS; ++i) {
        Sr[i] = fma_(w, a[2 * i], Sr[i]);
        Si[i] = fma_(w, a[2 * i + 1], Si[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NO * NRHS; ++i) {
        Sr[i] = fma_(ln.hla[JJ], a[2 * i], Sr[i]);
        Si[i] = fma_(ln.hla[JJ], a[2 * i + 1], Si[i]);
        Sr[i] = fma_(ln.hlb[JJ], b[2 * i], Sr[i]);
        Si[i] = fma_(ln.hlb[JJ], b[2 * i + 1], Si[i]);
      }
    }
    hop_lane_pairs<T, Q, L, LD, C, NRHS, JJ + 1>(ln, base, own, Sr, Si);
  }
}

// base: the LDS records of the lane exchange; own: this lane's record values (the same
// layout), from which the two-level layouts shuffle the partner lanes' through DPP.
template <typename T, int Q, int L, int LD, int C, int NRHS>
__device__ __forceinline__ void hop_terms(const Lane<T, Q, L, LD> &ln, const T *base, const T *own, T *Sr,
                                          T *Si) {
  using G = Geo<T, Q, L, LD>;
  constexpr bool RBL = C >= 0;
  constexpr int NO = RBL ? G::H : G::EPL;
  constexpr int NV = 2 * NO * NRHS;
  constexpr int R = G::R;
  static_assert(!RBL || G::RB, "a colour needs the red-black layout");
  static_assert(R <= 1 || Q < 2, "layouts keep at most one register digit: no pair of two register digits");
  if constexpr (LD > 0) {
    // pair (0, 1): the register digit and lane digit 0.  A reads the lane one step
    // down in lane digit 0 (l_1 - 1), B the lane one step up.  (No register digit: every
    // pair is one of lane digits, below.)
    if constexpr (R == 1) {
      constexpr int ST = G::lstride(0);
      T dn[NV], up[NV];
      if constexpr (dpp_layout<T, L, LD>()) {   // two levels: both read lane ^ ST
        xor_record<ST, T, NV>(own, dn);
#pragma unroll
        for (int i = 0; i < NV; ++i) up[i] = dn[i];
      } else {
        xget<T, NV, -ST>(base, ln.lane, dn);
        xget<T, NV, ST>(base, ln.lane, up);
      }
#pragma unroll
      for (int o = 0; o < NO; ++o) {
#pragma unroll
        for (int b = 0; b < NRHS; ++b) {
          const int so = b * NO + o;
          if constexpr (RBL) {                  // l0 = 2 s0 + (lead parity)
            const int s0 = o;                   // RT = 1
            const int beta = C;
            const int bl = ln.par ^ beta;
            const int ia0 = b * NO + s0, ia1 = b * NO + lead_up<G::HALF>(s0, 1);
            const int ib0 = b * NO + lead_dn<G::HALF>(s0, 0), ib1 = b * NO + s0;
            const T ar = bl ? dn[2 * ia1] : dn[2 * ia0], ai = bl ? dn[2 * ia1 + 1] : dn[2 * ia0 + 1];
            const T br = bl ? up[2 * ib1] : up[2 * ib0], bi = bl ? up[2 * ib1 + 1] : up[2 * ib0 + 1];
            const T wa = ln.hsa * ln.wup[beta][s0], wb = ln.hsb * ln.wdn[beta][s0];
            if constexpr (dpp_layout<T, L, LD>()) {   // two levels: one slot, one partner lane, one weight
              Sr[so] = fma_(wa + wb, ar, Sr[so]);
              Si[so] = fma_(wa + wb, ai, Si[so]);
            } else {
              Sr[so] = fma_(wa, ar, Sr[so]);
              Si[so] = fma_(wa, ai, Si[so]);
              Sr[so] = fma_(wb, br, Sr[so]);
              Si[so] = fma_(wb, bi, Si[so]);
            }
          } else {                              // plain layout: slot o holds register digit o
            const int la = o;
            if (la < L - 1) {
              const int src = b * NO + o + 1;
              const T w = ln.hsa * (T)sqrt((double)(la + 1));
              Sr[so] = fma_(w, dn[2 * src], Sr[so]);
              Si[so] = fma_(w, dn[2 * src + 1], Si[so]);
            }
            if (la > 0) {
              const int src = b * NO + o - 1;
              const T w = ln.hsb * (T)sqrt((double)la);
              Sr[so] = fma_(w, up[2 * src], Sr[so]);
              Si[so] = fma_(w, up[2 * src + 1], Si[so]);
            }
          }
        }
      }
    }
    hop_lane_pairs<T, Q, L, LD, C, NRHS, 0>(ln, base, own, Sr, Si);
    if constexpr (!dpp_layout<T, L, LD>()) wave_sync();
  }
}

// S = (dt/2) H_c v for this lane's entries.  cr/ci: per-qubit scaled control
// c'_j = (dt/2) 2 pi d_j; the coefficient of a_j is c'_j, of a_j^+ conj(c'_j).
template <typename T, int Q, int L, int LD, bool HOP>
__device__ __forceinline__ void apply_Hc(const Lane<T, Q, L, LD> &ln, const T *cr, const T *ci,
                                         const T *lor, const T *loi, const T *hir, const T *hii,
                                         const T *vr, const T *vi, T *Sr, T *Si) {
  using G = Geo<T, Q, L, LD>;
  T n[2 * (LD > 0 ? LD : 1)][2 * G::EPL];
  lane_exchange<T, Q, L, LD, G::EPL>(ln, vr, vi, n);
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) { Sr[e] = 0; Si[e] = 0; }
#pragma unroll
  for (int j = 0; j < G::R; ++j) {
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      const int l = G::rdigit(e, j);
      const int st = G::rstride(j);
      if (l < L - 1) {  // c'_j sqrt(l+1) v[e+st]
        const T ar = cr[j] * (T)sqrt((double)(l + 1)), ai = ci[j] * (T)sqrt((double)(l + 1));
        cmac(Sr[e], Si[e], ar, ai, vr[e + st], vi[e + st]);
      }
      if (l > 0) {      // conj(c'_j) sqrt(l) v[e-st]
        const T ar = cr[j] * (T)sqrt((double)l), ai = ci[j] * (T)sqrt((double)l);
        cmac_conj(Sr[e], Si[e], ar, ai, vr[e - st], vi[e - st]);
      }
    }
  }
  lane_digit_terms<T, Q, L, LD, G::EPL>(ln, lor, loi, hir, hii, n, Sr, Si);
  if constexpr (HOP) {                    // reads the record above
    T own[2 * G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      own[2 * e] = vr[e];
      own[2 * e + 1] = vi[e];
    }
    hop_terms<T, Q, L, LD, -1, 1>(ln, ln.xb, own, Sr, Si);
  }
}

// Per-step control coefficients: c'_j for register digits, per-lane lowering
// (c'_j sqrt(l+1)) and raising (conj(c'_j) sqrt(l)) coefficients for lane digits,
// and in the red-black layout the lane's coefficients on the leading register digit.
template <typename T, int Q, int L, int LD>
struct Coef {
  static constexpr int NL = LD > 0 ? LD : 1, NH = Lane<T, Q, L, LD>::NH;
  T cr[Q], ci[Q], lor[NL], loi[NL], hir[NL], hii[NL];
  T ur[2][NH], ui[2][NH], dr[2][NH], di[2][NH];
};

// The control values of step k (uniform across the wavefront).  Layouts with several
// columns per wavefront (small systems, few wavefronts per SIMD, so a window's chain
// of steps is latency-bound) load them one step ahead; the large layouts keep the
// registers for occupancy.
template <typename G>
constexpr bool ctrl_ahead() { return G::CPW > 1; }

template <typename T, int Q>
__device__ __forceinline__ void load_ctrl(const T *ctrl, long long k, typename C2<T>::type *v) {
  using V2 = typename C2<T>::type;
  const V2 *cp = reinterpret_cast<const V2 *>(ctrl) + k * Q;
#pragma unroll
  for (int j = 0; j < Q; ++j) v[j] = cp[j];
}

template <typename T, int Q, int L, int LD>
__device__ __forceinline__ void step_coeffs(const Lane<T, Q, L, LD> &ln, const typename C2<T>::type *v,
                                            Coef<T, Q, L, LD> &c) {
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    c.cr[j] = v[j].x;
    c.ci[j] = v[j].y;
  }
#pragma unroll
  for (int jj = 0; jj < LD; ++jj) {
    const int j = Geo<T, Q, L, LD>::R + jj;
    c.lor[jj] = c.cr[j] * ln.wlo[jj];
    c.loi[jj] = c.ci[j] * ln.wlo[jj];
    c.hir[jj] = c.cr[j] * ln.whi[jj];
    c.hii[jj] = -c.ci[j] * ln.whi[jj];
  }
  if constexpr (Geo<T, Q, L, LD>::RB) {
#pragma unroll
    for (int beta = 0; beta < 2; ++beta)
#pragma unroll
      for (int s0 = 0; s0 < Coef<T, Q, L, LD>::NH; ++s0) {
        c.ur[beta][s0] = c.cr[0] * ln.wup[beta][s0];
        c.ui[beta][s0] = c.ci[0] * ln.wup[beta][s0];
        c.dr[beta][s0] = c.cr[0] * ln.wdn[beta][s0];
        c.di[beta][s0] = c.ci[0] * ln.wdn[beta][s0];
      }
  }
}

// Pair terms of the per-step inner products for rows e (digit l) and f (digit l+1):
// a1 = Im(conj(y_e) z_f + conj(y_f) z_e), a2 = Re(conj(y_e) z_f - conj(y_f) z_e).
template <typename T>
__device__ __forceinline__ void pair_terms(T yer, T yei, T zer, T zei, T yfr, T yfi, T zfr, T zfi, T &a1, T &a2) {
  a1 = yer * zfi;
  a2 = yer * zfr;
  a1 = fma_(-yei, zfr, a1); a1 = fma_(yfr, zei, a1); a1 = fma_(-yfi, zer, a1);
  a2 = fma_(yei, zfi, a2); a2 = fma_(-yfr, zer, a2); a2 = fma_(-yfi, zei, a2);
}
// The same terms added onto running sums a1, a2 (one chain each, no separate add).
template <typename T>
__device__ __forceinline__ void pair_terms_acc(T yer, T yei, T zer, T zei, T yfr, T yfi, T zfr, T zfi, T &a1,
                                               T &a2) {
  a1 = fma_(yer, zfi, a1); a1 = fma_(-yei, zfr, a1); a1 = fma_(yfr, zei, a1); a1 = fma_(-yfi, zer, a1);
  a2 = fma_(yer, zfr, a2); a2 = fma_(yei, zfi, a2); a2 = fma_(-yfr, zer, a2); a2 = fma_(-yfi, zei, a2);
}

// ---------------------------------------------------------------------------- red-black half sweep

// Operands of the leading register digit for the output slots (s0, t) of one colour:
// with X[u] the input-colour slot (u, t) and b the output's l0 parity, the upper
// neighbour l0+1 sits in X[s0+b] and the lower one l0-1 in X[s0-1+b].  P[u+1] =
// X[u+b] for u = -1..HALF-1 (one lane-masked select per interior u; the two end
// values only meet zero weights when they would fall outside the digit).
template <typename T, int HALF>
__device__ __forceinline__ void lead_operands(bool b, const T *xr, const T *xi, int stride, T *pr, T *pi) {
  pr[0] = xr[0];
  pi[0] = xi[0];
#pragma unroll
  for (int u = 0; u + 1 < HALF; ++u) {
    pr[u + 1] = b ? xr[(u + 1) * stride] : xr[u * stride];
    pi[u + 1] = b ? xi[(u + 1) * stride] : xi[u * stride];
  }
  pr[HALF] = xr[(HALF - 1) * stride];
  pi[HALF] = xi[(HALF - 1) * stride];
}

// Register-digit terms of S = (dt/2) H_c v on the H slots of colour C (S is
// initialised here), reading only the slots of colour 1-C of v.
template <typename T, int Q, int L, int LD, int C>
__device__ __forceinline__ void apply_half_regs(const Lane<T, Q, L, LD> &ln, const Coef<T, Q, L, LD> &cf,
                                                const T *vr, const T *vi, T *Sr, T *Si) {
  using G = Geo<T, Q, L, LD>;
  constexpr int IN = (1 - C) * G::H;
#pragma unroll
  for (int t = 0; t < G::RT; ++t) {            // leading register digit
    const int beta = G::tpar(t) ^ C;
    T pr[G::HALF + 1], pi[G::HALF + 1];
    lead_operands<T, G::HALF>(ln.par ^ beta, vr + IN + t, vi + IN + t, G::RT, pr, pi);
#pragma unroll
    for (int s0 = 0; s0 < G::HALF; ++s0) {
      const int o = s0 * G::RT + t;
      Sr[o] = 0;
      Si[o] = 0;
      if constexpr (L == 2) {
        // two levels: both operands are the one input slot and one weight is zero, so
        // one product with c_up + conj(c_dn) gives the same value
        cmac(Sr[o], Si[o], cf.ur[beta][s0] + cf.dr[beta][s0], cf.ui[beta][s0] - cf.di[beta][s0], pr[s0], pi[s0]);
      } else {
        cmac(Sr[o], Si[o], cf.ur[beta][s0], cf.ui[beta][s0], pr[s0 + 1], pi[s0 + 1]);
        cmac_conj(Sr[o], Si[o], cf.dr[beta][s0], cf.di[beta][s0], pr[s0], pi[s0]);
      }
    }
  }
#pragma unroll
  for (int j = 1; j < G::R; ++j) {             // other register digits: same s0, tuple t +- stride
    const int st = G::rstride(j);
#pragma unroll
    for (int o = 0; o < G::H; ++o) {
      const int l = (o % G::RT / st) % L;
      if (l < L - 1) {
        const T ar = cf.cr[j] * (T)sqrt((double)(l + 1)), ai = cf.ci[j] * (T)sqrt((double)(l + 1));
        cmac(Sr[o], Si[o], ar, ai, vr[IN + o + st], vi[IN + o + st]);
      }
      if (l > 0) {
        const T ar = cf.cr[j] * (T)sqrt((double)l), ai = cf.ci[j] * (T)sqrt((double)l);
        cmac_conj(Sr[o], Si[o], ar, ai, vr[IN + o - st], vi[IN + o - st]);
      }
    }
  }
}

// S = (dt/2) H_c v on the H slots of colour C, reading only the slots of colour 1-C.
// HOP: plus (dt/2) H_J from colour C's current values own (sent in the same exchange).
template <typename T, int Q, int L, int LD, int C, bool HOP = false>
__device__ __forceinline__ void apply_half(const Lane<T, Q, L, LD> &ln, const Coef<T, Q, L, LD> &cf,
                                           const T *vr, const T *vi, T *Sr, T *Si, const T *owr = nullptr,
                                           const T *owi = nullptr) {
  using G = Geo<T, Q, L, LD>;
  constexpr int IN = (1 - C) * G::H;
  // lane digits: output slot o reads slot IN + o of the neighbouring lanes (the
  // colour flips with the lane parity); requested first, used last
  T n[2 * (LD > 0 ? LD : 1)][2 * G::H];
  lane_exchange<T, Q, L, LD, G::H, HOP ? G::H : 0>(ln, vr + IN, vi + IN, n, owr, owi);
  apply_half_regs<T, Q, L, LD, C>(ln, cf, vr, vi, Sr, Si);
  lane_digit_terms<T, Q, L, LD, G::H>(ln, cf.lor, cf.loi, cf.hir, cf.hii, n, Sr, Si);
  if constexpr (HOP) {
    T own[2 * G::H];
#pragma unroll
    for (int o = 0; o < G::H; ++o) {
      own[2 * o] = owr[o];
      own[2 * o + 1] = owi[o];
    }
    hop_terms<T, Q, L, LD, C, 1>(ln, ln.xb + xtail<T, G::H>(), own, Sr, Si);
  }
}

__device__ __forceinline__ int kit_of(const DevSys &s) { return s.kit_fixed > 0 ? s.kit_fixed : *s.kit; }

// w = x - sg i D^{-1} S on the given slots (sg = +1 forward, -1 reverse/adjoint, with conj(D)).
template <typename T, int Q, int L, int LD, bool REV>
__device__ __forceinline__ void jacobi_update(const Lane<T, Q, L, LD> &ln, int e, T Sr, T Si, T xr, T xi, T &wr,
                                              T &wi) {
  if (!REV) {   // w = x - i D^{-1} S
    wr = fma_(ln.dr[e], Si, fma_(ln.di[e], Sr, xr));
    wi = fma_(-ln.dr[e], Sr, fma_(ln.di[e], Si, xi));
  } else {      // w = x + i conj(D)^{-1} S
    wr = fma_(-ln.dr[e], Si, fma_(ln.di[e], Sr, xr));
    wi = fma_(ln.dr[e], Sr, fma_(ln.di[e], Si, xi));
  }
}

// Red-black half sweep: refresh the increment on the slots of colour C from the
// current values of colour 1-C (HOP: and the exchange terms from colour C's own
// current values).
template <typename T, int Q, int L, int LD, bool REV, int C, bool HOP>
__device__ __forceinline__ void half_sweep(const Lane<T, Q, L, LD> &ln, const Coef<T, Q, L, LD> &cf, const T *ur,
                                           const T *ui, const T *xr, const T *xi, T *wr, T *wi) {
  using G = Geo<T, Q, L, LD>;
  constexpr int IN = (1 - C) * G::H, OUT = C * G::H;
  T vr[G::EPL], vi[G::EPL], Sr[G::H], Si[G::H];
#pragma unroll
  for (int o = 0; o < G::H; ++o) {
    vr[IN + o] = ur[IN + o] + wr[IN + o];
    vi[IN + o] = ui[IN + o] + wi[IN + o];
  }
  T orr[G::H], ori[G::H];
  if constexpr (HOP) {
#pragma unroll
    for (int o = 0; o < G::H; ++o) {
      orr[o] = ur[OUT + o] + wr[OUT + o];
      ori[o] = ui[OUT + o] + wi[OUT + o];
    }
  }
  apply_half<T, Q, L, LD, C, HOP>(ln, cf, vr, vi, Sr, Si, orr, ori);
#pragma unroll
  for (int o = 0; o < G::H; ++o)
    jacobi_update<T, Q, L, LD, REV>(ln, OUT + o, Sr[o], Si[o], xr[OUT + o], xi[OUT + o], wr[OUT + o], wi[OUT + o]);
}

// One implicit-midpoint solve for the increment w = z - u, with z the solution of
// (I + sg i dt/2 H) z = u (sg = +1 forward, -1 reverse/adjoint).  With
// D = I + sg i dt/2 diag(h):  w = (D^{-1} - 1) u - sg i D^{-1} (dt/2) H_c (u + w),
// started from w = (D^{-1} - 1) u.  Odd L: nit Jacobi iterations (every entry from
// the previous iterate).  Even L: H_c only couples entries of opposite digit-sum
// parity, so the two colours are refreshed alternately, each from the other's
// newest values; nit counts these half sweeps, each costing half an iteration.
// The increment is O(dt |H|) |u| small, so its FP32 rounding enters the FP64
// state only at that scale.  HOP: the dipole exchange H_J joins H_c in the
// iteration; it keeps the digit-sum parity, so a half sweep takes it from its own
// colour's current values (Jacobi-style within the colour).
template <typename T, int Q, int L, int LD, bool REV, bool HOP>
__device__ __forceinline__ void solve_increment(const Lane<T, Q, L, LD> &ln, int nit, const Coef<T, Q, L, LD> &cf,
                                                const T *ur, const T *ui, T *wr, T *wi) {
  using G = Geo<T, Q, L, LD>;
  T xr[G::EPL], xi[G::EPL];
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) {
    ln.template scale_m1<REV>(e, ur[e], ui[e], xr[e], xi[e]);
    wr[e] = xr[e];
    wi[e] = xi[e];
  }
  if constexpr (G::RB) {
    int h = 0;
    for (; h + 1 < nit; h += 2) {
      half_sweep<T, Q, L, LD, REV, 0, HOP>(ln, cf, ur, ui, xr, xi, wr, wi);
      half_sweep<T, Q, L, LD, REV, 1, HOP>(ln, cf, ur, ui, xr, xi, wr, wi);
    }
    if (h < nit) half_sweep<T, Q, L, LD, REV, 0, HOP>(ln, cf, ur, ui, xr, xi, wr, wi);
  } else {
    T vr[G::EPL], vi[G::EPL], Sr[G::EPL], Si[G::EPL];
    for (int it = 0; it < nit; ++it) {
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        vr[e] = ur[e] + wr[e];
        vi[e] = ui[e] + wi[e];
      }
      apply_Hc<T, Q, L, LD, HOP>(ln, cf.cr, cf.ci, cf.lor, cf.loi, cf.hir, cf.hii, vr, vi, Sr, Si);
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) jacobi_update<T, Q, L, LD, REV>(ln, e, Sr[e], Si[e], xr[e], xi[e], wr[e], wi[e]);
    }
  }
}

// Lane-digit inner-product terms of the last half sweep.  After it, the slots of
// colour C (updated last) and the neighbours' slots of colour 1-C (records n) are
// final; every pair of rows one lane digit apart has exactly one row of colour C,
// so pairing each own slot with its upper neighbour (weight sqrt(l+1)) and its
// lower neighbour (weight sqrt(l)) visits every pair once.  a1 = Im(conj(y) z' +
// conj(y') z) is symmetric in the pair and a2 = Re(conj(y_lo) z_hi - conj(y_hi) z_lo)
// changes sign with it.
template <typename T, int Q, int L, int LD, int K, int JJ = 0>
__device__ __forceinline__ void last_inner_lane(const Lane<T, Q, L, LD> &ln, T (*n)[4 * K], const T *zr, const T *zi,
                                                const T *yr, const T *yi, T *s1, T *s2) {
  using G = Geo<T, Q, L, LD>;
  if constexpr (JJ < LD) {
    constexpr int ST = G::lstride(JJ);
    T up[4 * K], dn[4 * K];
    if constexpr (XPre<T, 2 * K>::value) {
#pragma unroll
      for (int i = 0; i < 4 * K; ++i) {
        up[i] = n[2 * JJ][i];
        dn[i] = n[2 * JJ + 1][i];
      }
    } else {
      xget<T, 4 * K, ST>(ln.xb, ln.lane, up);
      xget<T, 4 * K, -ST>(ln.xb, ln.lane, dn);
    }
    T u1 = 0, u2 = 0, d1 = 0, d2 = 0;
#pragma unroll
    for (int o = 0; o < K; ++o) {      // record: K complex z values, then K complex y values
      pair_terms_acc(yr[o], yi[o], zr[o], zi[o], up[2 * K + 2 * o], up[2 * K + 2 * o + 1], up[2 * o], up[2 * o + 1], u1,
                     u2);
      pair_terms_acc(yr[o], yi[o], zr[o], zi[o], dn[2 * K + 2 * o], dn[2 * K + 2 * o + 1], dn[2 * o], dn[2 * o + 1], d1,
                     d2);
    }
    s1[G::R + JJ] = fma_(ln.whi[JJ], d1, ln.wlo[JJ] * u1);
    s2[G::R + JJ] = fma_(-ln.whi[JJ], d2, ln.wlo[JJ] * u2);
    last_inner_lane<T, Q, L, LD, K, JJ + 1>(ln, n, zr, zi, yr, yi, s1, s2);
  } else if constexpr (LD > 0 && !XPre<T, 2 * K>::value) {
    wave_sync();
  }
}

// Half sweep of two right-hand sides with the same matrix (the backward sweep's
// state and adjoint): their records travel in one exchange, so a step has half as
// many LDS round trips.  Each result equals half_sweep on its own bit for bit.
// LAST: also the lane-digit inner products of the final z and y (last_inner_lane).
// FIRST: the increments still equal their start values x (read in place of w).
template <typename T, int Q, int L, int LD, bool REV, int C, bool HOP, bool LAST = false, bool FIRST = false>
__device__ __forceinline__ void half_sweep2(const Lane<T, Q, L, LD> &ln, const Coef<T, Q, L, LD> &cf,
                                            const T *uar, const T *uai, const T *xar, const T *xai, T *war, T *wai,
                                            const T *ubr, const T *ubi, const T *xbr, const T *xbi, T *wbr,
                                            T *wbi, T *s1 = nullptr, T *s2 = nullptr) {
  using G = Geo<T, Q, L, LD>;
  constexpr int IN = (1 - C) * G::H, OUT = C * G::H;
  const T *car = FIRST ? xar : war, *cai = FIRST ? xai : wai, *cbr = FIRST ? xbr : wbr, *cbi = FIRST ? xbi : wbi;
  T var[G::EPL], vai[G::EPL], vbr[G::EPL], vbi[G::EPL], rr[2 * G::H], ri[2 * G::H];
#pragma unroll
  for (int o = 0; o < G::H; ++o) {
    var[IN + o] = uar[IN + o] + car[IN + o];
    vai[IN + o] = uai[IN + o] + cai[IN + o];
    vbr[IN + o] = ubr[IN + o] + cbr[IN + o];
    vbi[IN + o] = ubi[IN + o] + cbi[IN + o];
    rr[o] = var[IN + o];
    ri[o] = vai[IN + o];
    rr[G::H + o] = vbr[IN + o];
    ri[G::H + o] = vbi[IN + o];
  }
  T orr[2 * G::H], ori[2 * G::H];         // HOP: own-colour values, sent in the same exchange
  if constexpr (HOP) {
#pragma unroll
    for (int o = 0; o < G::H; ++o) {
      orr[o] = uar[OUT + o] + car[OUT + o];
      ori[o] = uai[OUT + o] + cai[OUT + o];
      orr[G::H + o] = ubr[OUT + o] + cbr[OUT + o];
      ori[G::H + o] = ubi[OUT + o] + cbi[OUT + o];
    }
  }
  T n[2 * (LD > 0 ? LD : 1)][4 * G::H];
  lane_exchange<T, Q, L, LD, 2 * G::H, HOP ? 2 * G::H : 0>(ln, rr, ri, n, orr, ori);
  T Sr[2 * G::H], Si[2 * G::H];
  apply_half_regs<T, Q, L, LD, C>(ln, cf, var, vai, Sr, Si);
  apply_half_regs<T, Q, L, LD, C>(ln, cf, vbr, vbi, Sr + G::H, Si + G::H);
  lane_digit_terms<T, Q, L, LD, 2 * G::H>(ln, cf.lor, cf.loi, cf.hir, cf.hii, n, Sr, Si);
  if constexpr (HOP) {
    T own[4 * G::H];
#pragma unroll
    for (int o = 0; o < 2 * G::H; ++o) {
      own[2 * o] = orr[o];
      own[2 * o + 1] = ori[o];
    }
    hop_terms<T, Q, L, LD, C, 2>(ln, ln.xb + xtail<T, 2 * G::H>(), own, Sr, Si);
  }
#pragma unroll
  for (int o = 0; o < G::H; ++o) {
    jacobi_update<T, Q, L, LD, REV>(ln, OUT + o, Sr[o], Si[o], xar[OUT + o], xai[OUT + o], war[OUT + o], wai[OUT + o]);
    jacobi_update<T, Q, L, LD, REV>(ln, OUT + o, Sr[G::H + o], Si[G::H + o], xbr[OUT + o], xbi[OUT + o], wbr[OUT + o],
                                    wbi[OUT + o]);
  }
  if constexpr (LAST) {
    T zr[G::H], zi[G::H], yr[G::H], yi[G::H];
#pragma unroll
    for (int o = 0; o < G::H; ++o) {
      zr[o] = uar[OUT + o] + war[OUT + o];
      zi[o] = uai[OUT + o] + wai[OUT + o];
      yr[o] = ubr[OUT + o] + wbr[OUT + o];
      yi[o] = ubi[OUT + o] + wbi[OUT + o];
    }
    last_inner_lane<T, Q, L, LD, G::H>(ln, n, zr, zi, yr, yi, s1, s2);
  }
}

// Lane-digit inner products taken inside the last half sweep: red-black layout in
// FP32 (FP64 lacks the registers to keep the records, it exchanges z and y again).
template <typename T, int Q, int L, int LD>
constexpr bool fused_inner() { return Geo<T, Q, L, LD>::RB && sizeof(T) == 4; }

// Two right-hand sides with the same matrix (a: state, b: adjoint); each result is
// bit-identical to solve_increment on its own.  When fused_inner, the lane-digit
// inner products of the solutions are left in s1, s2 (entries R..q-1), taken in
// the last half sweep; nit >= 1.
template <typename T, int Q, int L, int LD, bool REV, bool HOP>
__device__ __forceinline__ void solve_increment2(const Lane<T, Q, L, LD> &ln, int nit, const Coef<T, Q, L, LD> &cf,
                                                 const T *ar, const T *ai, T *war, T *wai,
                                                 const T *br, const T *bi, T *wbr, T *wbi, T *s1, T *s2) {
  using G = Geo<T, Q, L, LD>;
  if constexpr (G::RB) {
    T xar[G::EPL], xai[G::EPL], xbr[G::EPL], xbi[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      ln.template scale_m1<REV>(e, ar[e], ai[e], xar[e], xai[e]);
      ln.template scale_m1<REV>(e, br[e], bi[e], xbr[e], xbi[e]);
    }
    // Half sweeps alternate colour 0, 1, 0, ...; when fused_inner, the last one also takes
    // the lane-digit inner products.
    constexpr bool FI = fused_inner<T, Q, L, LD>();
    if constexpr (HOP) {
      // the dipole terms read the refreshed colour's own current values: w starts as x
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        war[e] = xar[e];
        wai[e] = xai[e];
        wbr[e] = xbr[e];
        wbi[e] = xbi[e];
      }
      int h = 0;
      for (; h + 2 < nit; h += 2) {
        half_sweep2<T, Q, L, LD, REV, 0, HOP>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi);
        half_sweep2<T, Q, L, LD, REV, 1, HOP>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi);
      }
      if (nit - h == 2) {
        half_sweep2<T, Q, L, LD, REV, 0, HOP>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi);
        half_sweep2<T, Q, L, LD, REV, 1, HOP, FI>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi, s1, s2);
      } else {
        half_sweep2<T, Q, L, LD, REV, 0, HOP, FI>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi, s1, s2);
      }
      return;
    }
    // The first half sweep reads x in place of w; w's colour 1 keeps x until the second
    // writes it (copied only when there is a single half sweep).
    if (nit < 2) {
#pragma unroll
      for (int o = G::H; o < G::EPL; ++o) {
        war[o] = xar[o];
        wai[o] = xai[o];
        wbr[o] = xbr[o];
        wbi[o] = xbi[o];
      }
      half_sweep2<T, Q, L, LD, REV, 0, HOP, FI, true>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi,
                                                      s1, s2);
      return;
    }
    half_sweep2<T, Q, L, LD, REV, 0, HOP, false, true>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi);
    int h = 1;
    for (; h + 2 < nit; h += 2) {
      half_sweep2<T, Q, L, LD, REV, 1, HOP>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi);
      half_sweep2<T, Q, L, LD, REV, 0, HOP>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi);
    }
    if (nit - h == 2) {
      half_sweep2<T, Q, L, LD, REV, 1, HOP>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi);
      half_sweep2<T, Q, L, LD, REV, 0, HOP, FI>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi, s1, s2);
    } else {
      half_sweep2<T, Q, L, LD, REV, 1, HOP, FI>(ln, cf, ar, ai, xar, xai, war, wai, br, bi, xbr, xbi, wbr, wbi, s1, s2);
    }
  } else {
    solve_increment<T, Q, L, LD, REV, HOP>(ln, nit, cf, ar, ai, war, wai);
    solve_increment<T, Q, L, LD, REV, HOP>(ln, nit, cf, br, bi, wbr, wbi);
  }
}

// ---------------------------------------------------------------------------- forward sweep

// One wavefront per (window, column group).  The state U (FP64 accumulator)
// starts from W^{m-1} (W^0 = I), advances over the window's steps entirely in
// registers, u_{k+1} = u_k + 2 w_k, and is written as U^m(t_m); optional
// checkpoints U_{k0 + i*C} are written on the way.  ROLLOUT: a single window over
// all steps from W^0, writing the states at the window boundaries instead.
template <typename T, int Q, int L, int LD, bool ROLLOUT, bool HOP>
__device__ __forceinline__ void forward_item(const DevSys &s, int m, int cg, double *Wout, double *Uout, T *xb) {
  using G = Geo<T, Q, L, LD>;
  Lane<T, Q, L, LD> ln;
  ln.init(s, cg, xb);
  if constexpr (HOP) ln.init_hop(s);

  double udr[G::EPL], udi[G::EPL];
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) {
    udr[e] = 0.0;
    udi[e] = 0.0;
    if (ln.valid) {
      const int r = ln.row(e);
      if (m == 0) {
        udr[e] = (r == s.ess_row[ln.col]) ? 1.0 : 0.0;
      } else {
        const double2 w = reinterpret_cast<const double2 *>(s.W)[((size_t)(m - 1) * s.E + ln.col) * s.N + r];
        udr[e] = w.x;
        udi[e] = w.y;
      }
    }
  }
  const long long k0 = ROLLOUT ? 0 : s.kstart[m];
  const long long k1 = ROLLOUT ? s.NT : s.kstart[m + 1];
  const int kit = kit_of(s);
  const T *ctrl = reinterpret_cast<const T *>(s.ctrl);
  int next_boundary = 1;
  int since = 0, icp = 0;              // steps since the last checkpoint, checkpoints written

  typename C2<T>::type cnext[Q];
  if constexpr (ctrl_ahead<G>()) load_ctrl<T, Q>(ctrl, k0, cnext);
  for (long long k = k0; k < k1; ++k) {
    typename C2<T>::type ccur[Q];
    if constexpr (ctrl_ahead<G>()) {
#pragma unroll
      for (int j = 0; j < Q; ++j) ccur[j] = cnext[j];
      load_ctrl<T, Q>(ctrl, k + 1 < k1 ? k + 1 : k, cnext);
    } else {
      load_ctrl<T, Q>(ctrl, k, ccur);
    }
    if (!ROLLOUT && s.ckpt_every > 0 && since == s.ckpt_every) {   // U_{k0 + (icp+1) C}
      double2 *cp = reinterpret_cast<double2 *>(s.ckpt) + (((size_t)m * s.ncp + icp) * s.E + ln.col) * s.N;
      if (ln.valid)
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) cp[ln.row(e)] = double2{udr[e], udi[e]};
      ++icp;
      since = 0;
    }
    ++since;
    Coef<T, Q, L, LD> cf;
    step_coeffs<T, Q, L, LD>(ln, ccur, cf);
    T ur[G::EPL], ui[G::EPL], wr[G::EPL], wi[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      ur[e] = (T)udr[e];
      ui[e] = (T)udi[e];
    }
    solve_increment<T, Q, L, LD, false, HOP>(ln, kit, cf, ur, ui, wr, wi);
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {   // u_{k+1} = 2 z - u_k = u_k + 2 w
      udr[e] += 2.0 * (double)wr[e];
      udi[e] += 2.0 * (double)wi[e];
    }
    if (ROLLOUT && next_boundary < s.M && k + 1 == s.kstart[next_boundary]) {
      if (ln.valid) {
        double2 *w = reinterpret_cast<double2 *>(Wout) + ((size_t)(next_boundary - 1) * s.E + ln.col) * s.N;
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) w[ln.row(e)] = double2{udr[e], udi[e]};
      }
      ++next_boundary;
    }
  }
  if (!ln.valid) return;
  double2 *dst = ROLLOUT ? reinterpret_cast<double2 *>(Uout) + (size_t)ln.col * s.N
                         : reinterpret_cast<double2 *>(s.Ufin) + ((size_t)m * s.E + ln.col) * s.N;
  if (ROLLOUT && !Uout) return;
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) dst[ln.row(e)] = double2{udr[e], udi[e]};
}

template <typename T, int Q, int L, int LD, bool ROLLOUT, bool HOP>
__global__ __launch_bounds__(64) void k_forward(DevSys s, double *Wout, double *Uout, int nitems) {
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nitems) return;
  __shared__ __align__(16) T xb[xchg_bytes<T, HOP>() / sizeof(T)];
  xchg_clear<T, HOP>(xb);
  if (ROLLOUT) forward_item<T, Q, L, LD, true, HOP>(s, 0, item, Wout, Uout, xb);
  else forward_item<T, Q, L, LD, false, HOP>(s, item / s.ncg, item % s.ncg, nullptr, nullptr, xb);
}

// Slot holding, in the lane one lane-digit step away, the row with the same
// register digits: the other colour's slot in the red-black layout.
template <typename G>
__device__ __forceinline__ constexpr int partner(int e) {
  if constexpr (G::RB) return e < G::H ? e + G::H : e - G::H;
  else return e;
}

// Register-digit part of the per-step inner products (see backward_item).
template <typename T, int Q, int L, int LD>
__device__ __forceinline__ void inner_register_digits(const Lane<T, Q, L, LD> &ln, const T *zr, const T *zi,
                                                      const T *yr, const T *yi, T *s1, T *s2) {
  using G = Geo<T, Q, L, LD>;
#pragma unroll
  for (int j = 0; j < G::R; ++j) {
    s1[j] = 0;
    s2[j] = 0;
  }
  if constexpr (G::RB) {
    // leading digit, pairs enumerated from the red slots: (red, upper black) with
    // weight sqrt(l0+1) and (lower black, red) with weight sqrt(l0)
#pragma unroll
    for (int t = 0; t < G::RT; ++t) {
      const int beta = G::tpar(t);
      T pzr[G::HALF + 1], pzi[G::HALF + 1], pyr[G::HALF + 1], pyi[G::HALF + 1];
      lead_operands<T, G::HALF>(ln.par ^ beta, zr + G::H + t, zi + G::H + t, G::RT, pzr, pzi);
      lead_operands<T, G::HALF>(ln.par ^ beta, yr + G::H + t, yi + G::H + t, G::RT, pyr, pyi);
#pragma unroll
      for (int s0 = 0; s0 < G::HALF; ++s0) {
        const int e = s0 * G::RT + t;
        T u1, u2, d1, d2;
        pair_terms(yr[e], yi[e], zr[e], zi[e], pyr[s0 + 1], pyi[s0 + 1], pzr[s0 + 1], pzi[s0 + 1], u1, u2);
        pair_terms(yr[e], yi[e], zr[e], zi[e], pyr[s0], pyi[s0], pzr[s0], pzi[s0], d1, d2);
        s1[0] = fma_(ln.wup[beta][s0], u1, s1[0]);
        s1[0] = fma_(ln.wdn[beta][s0], d1, s1[0]);
        s2[0] = fma_(ln.wup[beta][s0], u2, s2[0]);
        s2[0] = fma_(-ln.wdn[beta][s0], d2, s2[0]);
      }
    }
    // other register digits: slot e (digit l < L-1) pairs with the other colour's
    // slot at tuple t + stride
#pragma unroll
    for (int j = 1; j < G::R; ++j) {
      const int st = G::rstride(j);
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        const int l = (e % G::RT / st) % L;
        if (l < L - 1) {
          const int f = partner<G>(e) + st;
          T a1, a2;
          pair_terms(yr[e], yi[e], zr[e], zi[e], yr[f], yi[f], zr[f], zi[f], a1, a2);
          const T w = (T)sqrt((double)(l + 1));
          s1[j] = fma_(w, a1, s1[j]);
          s2[j] = fma_(w, a2, s2[j]);
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        const int l = G::rdigit(e, j);
        if (l < L - 1) {
          const int f = e + G::rstride(j);
          T a1, a2;
          pair_terms(yr[e], yi[e], zr[e], zi[e], yr[f], yi[f], zr[f], zi[f], a1, a2);
          const T w = (T)sqrt((double)(l + 1));
          s1[j] = fma_(w, a1, s1[j]);
          s2[j] = fma_(w, a2, s2[j]);
        }
      }
    }
  }
}

// Lane-digit part of the per-step inner products: pairs (row in this lane, the
// same register digits in the lane one digit step up); a1 = Im(conj(y) z' + conj(y') z),
// a2 = Re(conj(y) z' - conj(y') z) with ' the upper lane.  z' and y' pass through
// the exchange one after the other.
template <typename T, int Q, int L, int LD, bool ZROUND, int JJ = 0>
__device__ __forceinline__ void inner_lane_gets(const Lane<T, Q, L, LD> &ln, const T *zr, const T *zi,
                                                const T *yr, const T *yi, T *a1, T *a2) {
  using G = Geo<T, Q, L, LD>;
  if constexpr (JJ < LD) {
    constexpr int ST = G::lstride(JJ);
    T n[2 * G::EPL];
    xget<T, 2 * G::EPL, ST>(ln.xb, ln.lane, n);
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      const int f = partner<G>(e);   // the same row of the lane one digit step up
      const T ur = n[2 * f], ui = n[2 * f + 1];
      if constexpr (ZROUND) {        // z' terms: conj(y) z'
        a1[JJ] = fma_(yr[e], ui, a1[JJ]); a1[JJ] = fma_(-yi[e], ur, a1[JJ]);
        a2[JJ] = fma_(yr[e], ur, a2[JJ]); a2[JJ] = fma_(yi[e], ui, a2[JJ]);
      } else {                       // y' terms: conj(y') z
        a1[JJ] = fma_(ur, zi[e], a1[JJ]); a1[JJ] = fma_(-ui, zr[e], a1[JJ]);
        a2[JJ] = fma_(-ur, zr[e], a2[JJ]); a2[JJ] = fma_(-ui, zi[e], a2[JJ]);
      }
    }
    inner_lane_gets<T, Q, L, LD, ZROUND, JJ + 1>(ln, zr, zi, yr, yi, a1, a2);
  }
}

template <typename T, int Q, int L, int LD>
__device__ __forceinline__ void inner_lane_digits(const Lane<T, Q, L, LD> &ln, const T *zr, const T *zi, const T *yr,
                                                  const T *yi, T *s1, T *s2) {
  using G = Geo<T, Q, L, LD>;
  if constexpr (LD > 0) {
    T a1[LD], a2[LD], rec[2 * G::EPL];
#pragma unroll
    for (int jj = 0; jj < LD; ++jj) a1[jj] = a2[jj] = 0;
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      rec[2 * e] = zr[e];
      rec[2 * e + 1] = zi[e];
    }
    xput<T, 2 * G::EPL>(ln.xb, ln.lane, rec);
    wave_sync();
    inner_lane_gets<T, Q, L, LD, true>(ln, zr, zi, yr, yi, a1, a2);
    wave_sync();
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      rec[2 * e] = yr[e];
      rec[2 * e + 1] = yi[e];
    }
    xput<T, 2 * G::EPL>(ln.xb, ln.lane, rec);
    wave_sync();
    inner_lane_gets<T, Q, L, LD, false>(ln, zr, zi, yr, yi, a1, a2);
    wave_sync();
#pragma unroll
    for (int jj = 0; jj < LD; ++jj) {
      s1[G::R + jj] = ln.wlo[jj] * a1[jj];
      s2[G::R + jj] = ln.wlo[jj] * a2[jj];
    }
  }
}

// ---------------------------------------------------------------------------- backward sweep

// Steps per block barrier of the backward schedules that hand step records between
// wavefronts (a power of two).
constexpr int kX3Steps = 2;

// Per-step inner products are reduced over the wavefront's 64 lanes through LDS:
// every step each lane stores its 2q partial sums (propagation precision); every RB steps
// lane i sums, in FP64 and in lane order, the 64 partials of one (step, value)
// pair and writes it to the series (one coalesced store per flush).
template <typename T>
constexpr int red_elems() { return sizeof(T) == 4 ? 36 * 64 : 24 * 64; }   // 9 KB (FP32), 12 KB (FP64) per wavefront
// The one-wavefront FP32 sweep without the dipole terms (k_backward) buffers 64/(2q) steps, so
// every lane takes part in a flush (16.3 KB; eight such wavefronts with their exchange buffers
// fit one CU's LDS).
template <typename T, bool HOP>
constexpr int red_one_elems() { return sizeof(T) == 4 && !HOP ? 65 * 64 : red_elems<T>(); }

template <typename T, int Q, int RE = red_elems<T>()>
struct SeriesBuf {
  static constexpr int NV = 2 * Q;               // values per step
  static constexpr int VS = 65;                  // elements per (step, value) row: 64 lanes + 1 (bank offset)
  static constexpr int RS = NV * VS;             // elements per buffered step
  static constexpr int RB = (RE / RS < 64 / NV) ? RE / RS : 64 / NV;   // steps per flush
  static_assert(RB >= 1, "reduction buffer too small");
};

// ---- pieces shared by the backward sweep variants

// Start values of window m for one lane: U^m(t_m) (state) or the terminal adjoint of
// eq. terminal, mu/2 (W^m - U^m), or gamma V/E^2 for the last window (the split
// form: the part -U^M/E obeys the state's recursion, adds nothing to the control
// gradient, and returns in the W-gradient; App. B, eq. back-prop-2).
template <typename T, int Q, int L, int LD>
__device__ __forceinline__ void backward_start(const DevSys &s, int m, const Lane<T, Q, L, LD> &ln, bool adjoint,
                                               double *ar, double *ai) {
  using G = Geo<T, Q, L, LD>;
  const double2 *uf = reinterpret_cast<const double2 *>(s.Ufin) + ((size_t)m * s.E + ln.col) * s.N;
  const double E2 = (double)s.E * (double)s.E;
  const double gr = s.scal[4] / E2, gi = s.scal[5] / E2;
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) {
    ar[e] = ai[e] = 0.0;
    if (!ln.valid) continue;
    const int r = ln.row(e);
    const double2 u = uf[r];
    if (!adjoint) {
      ar[e] = u.x;
      ai[e] = u.y;
    } else if (m < s.M - 1) {
      const double2 w = reinterpret_cast<const double2 *>(s.W)[((size_t)m * s.E + ln.col) * s.N + r];
      ar[e] = 0.5 * s.mu * (w.x - u.x);
      ai[e] = 0.5 * s.mu * (w.y - u.y);
    } else {
      const double2 v = reinterpret_cast<const double2 *>(s.V)[(size_t)ln.col * s.N + r];
      ar[e] = gr * v.x - gi * v.y;
      ai[e] = gr * v.y + gi * v.x;
    }
  }
}

// Position of the current step k in its checkpoint interval, k - k0 = ic * C + jr,
// counted down from the window's last step.
struct CkptPos {
  int jr = 0, ic = 0;
  __device__ CkptPos(const DevSys &s, long long k0, long long k1) {
    if (s.ckpt_every > 0) {
      jr = (int)(k1 - 1 - k0) % s.ckpt_every;
      ic = (int)(k1 - 1 - k0) / s.ckpt_every;
    }
  }
};

// After step k: re-sync the state (U_k, stored at k - k0 = ic * C) and count down.
template <typename T, int Q, int L, int LD>
__device__ __forceinline__ void ckpt_step(const DevSys &s, int m, const Lane<T, Q, L, LD> &ln, bool state, CkptPos &c,
                                          double *ur, double *ui) {
  using G = Geo<T, Q, L, LD>;
  if (s.ckpt_every <= 0) return;
  if (c.jr == 0 && c.ic > 0 && state && ln.valid) {
    const double2 *cp =
        reinterpret_cast<const double2 *>(s.ckpt) + (((size_t)m * s.ncp + (c.ic - 1)) * s.E + ln.col) * s.N;
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      const double2 v = cp[ln.row(e)];
      ur[e] = v.x;
      ui[e] = v.y;
    }
  }
  if (c.jr == 0) {
    c.jr = s.ckpt_every - 1;
    --c.ic;
  } else {
    --c.jr;
  }
}

// The step's 2q inner products of this lane into the wavefront's series buffer; every
// RB steps, lane i sums one buffered (step, value) row over the 64 lanes in FP64, in
// lane order, and stores it in the propagation precision (idx = k - k0, len = window
// length): the lane values are products of that precision, so the stored sum keeps their
// accuracy, and the sums over column groups and steps that follow run in FP64.  Only
// this wavefront touches `red`, and its LDS operations complete in order.
template <typename T, int Q, int RE = red_elems<T>()>
__device__ __forceinline__ void series_put(T *red, T *ser, int lane, int idx, int len, const T *s1, const T *s2) {
  using SB = SeriesBuf<T, Q, RE>;
  T *slot = red + (idx % SB::RB) * SB::RS + lane;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    slot[(2 * j) * SB::VS] = s1[j];
    slot[(2 * j + 1) * SB::VS] = s2[j];
  }
  if (idx % SB::RB == 0) {             // steps idx .. idx+RB-1 are buffered: flush
    wave_sync();
    const int r = lane / SB::NV, vv = lane % SB::NV;
    if (r < SB::RB && idx + r < len) {
      const T *col = red + r * SB::RS + vv * SB::VS;
      double acc = 0.0;
#pragma unroll 8
      for (int l = 0; l < 64; ++l) acc += (double)col[l];
      ser[(size_t)(idx + r) * SB::NV + vv] = (T)acc;
    }
    wave_sync();
  }
}

// Layouts with two or more columns per wavefront (a column spans at most 32 lanes)
// split the backward sweep's two right-hand sides over the two halves of a
// wavefront: lanes 0..31 reconstruct the state and lanes 32..63 propagate the
// adjoint of the same CPW/2 columns, with the same instructions (DevSys.ncg_b
// backward wavefronts per window).  A lane then solves one system per step instead
// of two: these windows are latency-bound serial chains (few wavefronts), and the
// step gets shorter.
template <typename G, int Q>
constexpr bool split_rhs() { return G::CPW >= 2; }

template <typename T, int Q, int L, int LD, bool HOP, int RE = red_elems<T>()>
__device__ __forceinline__ void backward_item_split(const DevSys &s, int m, int cg, T *red, T *xb) {
  using G = Geo<T, Q, L, LD>;
  const int item = m * s.ncg_b + cg;
  Lane<T, Q, L, LD> ln;
  ln.init(s, cg, xb, true);
  if constexpr (HOP) ln.init_hop(s);
  const bool adj = ln.lane >= 32;                   // this lane's system: state (false) or adjoint (true)

  double ar[G::EPL], ai[G::EPL];                    // U (state lanes) or Lambda (adjoint lanes), FP64
  backward_start<T, Q, L, LD>(s, m, ln, adj, ar, ai);
  const long long k0 = s.kstart[m], k1 = s.kstart[m + 1];
  const int kit = kit_of(s);
  const T *ctrl = reinterpret_cast<const T *>(s.ctrl);
  T *ser = reinterpret_cast<T *>(s.series) + (size_t)item * s.maxlen * 2 * Q;
  CkptPos cp(s, k0, k1);
  typename C2<T>::type cnext[Q];
  load_ctrl<T, Q>(ctrl, k1 - 1, cnext);
  for (long long k = k1 - 1; k >= k0; --k) {
    typename C2<T>::type ccur[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) ccur[j] = cnext[j];
    load_ctrl<T, Q>(ctrl, k > k0 ? k - 1 : k, cnext);
    Coef<T, Q, L, LD> cf;
    step_coeffs<T, Q, L, LD>(ln, ccur, cf);
    T ur[G::EPL], ui[G::EPL], wr[G::EPL], wi[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      ur[e] = (T)ar[e];
      ui[e] = (T)ai[e];
    }
    solve_increment<T, Q, L, LD, true, HOP>(ln, kit, cf, ur, ui, wr, wi);
    // own solution (z or y) and the other half's (lane ^ 32)
    T vr[G::EPL], vi[G::EPL], pr[G::EPL], pi[G::EPL];
    {
      T rec[2 * G::EPL], oth[2 * G::EPL];
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        vr[e] = ur[e] + wr[e];
        vi[e] = ui[e] + wi[e];
        rec[2 * e] = vr[e];
        rec[2 * e + 1] = vi[e];
      }
      wave_sync();
      xput<T, 2 * G::EPL>(ln.xb, ln.lane, rec);
      wave_sync();
      xget_from<T, 2 * G::EPL>(ln.xb, ln.lane ^ 32, oth);
      wave_sync();
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        pr[e] = oth[2 * e];
        pi[e] = oth[2 * e + 1];
      }
    }
    T zr[G::EPL], zi[G::EPL], yr[G::EPL], yi[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      zr[e] = adj ? pr[e] : vr[e];
      zi[e] = adj ? pi[e] : vi[e];
      yr[e] = adj ? vr[e] : pr[e];
      yi[e] = adj ? vi[e] : pi[e];
    }
    // inner products (both halves compute them; the adjoint half contributes zeros)
    T s1[Q], s2[Q];
    inner_register_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
    inner_lane_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      s1[j] = adj ? (T)0 : s1[j];
      s2[j] = adj ? (T)0 : s2[j];
    }
    series_put<T, Q, RE>(red, ser, ln.lane, (int)(k - k0), (int)(k1 - k0), s1, s2);
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      ar[e] += 2.0 * (double)wr[e];
      ai[e] += 2.0 * (double)wi[e];
    }
    ckpt_step<T, Q, L, LD>(s, m, ln, !adj, cp, ar, ai);
  }
  if (!ln.valid || !adj) return;
  double2 *l0 = reinterpret_cast<double2 *>(s.lam0) + ((size_t)m * s.E + ln.col) * s.N;
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) l0[ln.row(e)] = double2{ar[e], ai[e]};
}

// One wavefront per (window, column group).  Starting from U^m(t_m) and the
// terminal condition of eq. terminal, each step k (descending) solves
//   (I - i dt/2 H_k) [z, y] = [U_{k+1}, Lambda_{k+1}]
// with one shared fixed point: z = (U_k + U_{k+1})/2 reconstructs the forward
// state (the rule is time-reversible), y is the adjoint midpoint.  Then
//   U_k = 2z - U_{k+1},  Lambda_k = 2y - Lambda_{k+1},
// and the per-step inner products Im<y, (a_j + a_j^+) z>, Re<y, (a_j - a_j^+) z>
// (summed over the wavefront's columns, in FP64 across lanes) go to the series.
//
// Last window: Lambda^M(t_M) = gamma V/E^2 - U^M/E.  The part -U^M/E obeys the
// same backward recursion as U itself, so at every step it equals -z/E and adds
// Re<z, i dH z>/E = 0 to the control gradient (dH Hermitian); only gamma V/E^2 is
// propagated, and the W-gradient adds the dropped part back exactly:
// Lambda^M(t_{M-1}) = -W^{M-1}/E + (propagated part)  (App. B, eq. back-prop-2).
// red: RE elements of series buffer (LDS).
template <typename T, int Q, int L, int LD, bool HOP, int RE = red_elems<T>()>
__device__ __forceinline__ void backward_item(const DevSys &s, int m, int cg, T *red, T *xb) {
  using G = Geo<T, Q, L, LD>;
  if constexpr (split_rhs<G, Q>()) {
    backward_item_split<T, Q, L, LD, HOP, RE>(s, m, cg, red, xb);
    return;
  }
  const int item = m * s.ncg_b + cg;
  Lane<T, Q, L, LD> ln;
  ln.init(s, cg, xb);
  if constexpr (HOP) ln.init_hop(s);

  double udr[G::EPL], udi[G::EPL], ldr[G::EPL], ldi[G::EPL];
  backward_start<T, Q, L, LD>(s, m, ln, false, udr, udi);
  backward_start<T, Q, L, LD>(s, m, ln, true, ldr, ldi);
  const long long k0 = s.kstart[m], k1 = s.kstart[m + 1];
  const int kit = kit_of(s);
  const T *ctrl = reinterpret_cast<const T *>(s.ctrl);
  T *ser = reinterpret_cast<T *>(s.series) + (size_t)item * s.maxlen * 2 * Q;
  CkptPos cp(s, k0, k1);

  for (long long k = k1 - 1; k >= k0; --k) {      // (one column per wavefront: the controls are not loaded ahead)
    typename C2<T>::type ccur[Q];
    load_ctrl<T, Q>(ctrl, k, ccur);
    Coef<T, Q, L, LD> cf;
    step_coeffs<T, Q, L, LD>(ln, ccur, cf);
    T ur[G::EPL], ui[G::EPL], lr[G::EPL], li[G::EPL];
    T wur[G::EPL], wui[G::EPL], wlr[G::EPL], wli[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      ur[e] = (T)udr[e];
      ui[e] = (T)udi[e];
      lr[e] = (T)ldr[e];
      li[e] = (T)ldi[e];
    }
    T s1[Q], s2[Q];
    solve_increment2<T, Q, L, LD, true, HOP>(ln, kit, cf, ur, ui, wur, wui, lr, li, wlr, wli, s1, s2);
    T zr[G::EPL], zi[G::EPL], yr[G::EPL], yi[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      zr[e] = ur[e] + wur[e];
      zi[e] = ui[e] + wui[e];
      yr[e] = lr[e] + wlr[e];
      yi[e] = li[e] + wli[e];
    }
    // inner products per qubit: s1 = Im(A + B), s2 = Re(A - B) with
    // A = <y, a_j z> = sum conj(y_r) sqrt(l+1) z_{r+st},  B = <y, a_j^+ z> = sum sqrt(l+1) conj(y_{r+st}) z_r
    inner_register_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
    if constexpr (!fused_inner<T, Q, L, LD>()) inner_lane_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
    series_put<T, Q, RE>(red, ser, ln.lane, (int)(k - k0), (int)(k1 - k0), s1, s2);
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      udr[e] += 2.0 * (double)wur[e];
      udi[e] += 2.0 * (double)wui[e];
      ldr[e] += 2.0 * (double)wlr[e];
      ldi[e] += 2.0 * (double)wli[e];
    }
    ckpt_step<T, Q, L, LD>(s, m, ln, true, cp, udr, udi);
  }
  if (!ln.valid) return;
  double2 *l0 = reinterpret_cast<double2 *>(s.lam0) + ((size_t)m * s.E + ln.col) * s.N;
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) l0[ln.row(e)] = double2{ldr[e], ldi[e]};
}

// Held to two waves per SIMD (a 256-register budget): the FP32 dipole variant, which would
// otherwise exceed it by a few registers, and the FP64 variant without dipole terms, which
// would otherwise take 289 and run one wave per SIMD; at two it keeps 25 values in scratch,
// reloaded a few times per step, and a 2048-item launch runs in one round instead of two.
template <typename T, int Q, int L, int LD, bool HOP>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu((HOP && sizeof(T) == 4) || (!HOP && sizeof(T) == 8) ? 2 : 1)))
void k_backward(DevSys s, int nitems) {
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nitems) return;
  __shared__ T red[red_one_elems<T, HOP>()];
  __shared__ __align__(16) T xb[xchg_bytes<T, HOP>() / sizeof(T)];
  xchg_clear<T, HOP>(xb);
  backward_item<T, Q, L, LD, HOP, red_one_elems<T, HOP>()>(s, item / s.ncg_b, item % s.ncg_b, red, xb);
}

// Two wavefronts per (window, column group) for the one-column-per-wavefront layout
// when a launch has few wavefronts (at most one per SIMD): wavefront 0 reconstructs
// the state and wavefront 1 propagates the adjoint, with the same instructions, so
// each solves one system per step.  Every step wavefront 0 passes z to wavefront 1
// through a double-buffered LDS record (one block barrier per step, taken by both
// wavefronts on every iteration), and wavefront 1 takes the inner products.
template <typename T, int Q, int L, int LD, bool HOP>
__device__ __forceinline__ void backward_item_xw(const DevSys &s, int m, int cg, T *red, T *xb, T *zb) {
  using G = Geo<T, Q, L, LD>;
  const int wv = threadIdx.x >> 6;                  // 0: state, 1: adjoint (uniform per wavefront)
  const int item = m * s.ncg_b + cg;
  Lane<T, Q, L, LD> ln;
  ln.init(s, cg, xb);
  if constexpr (HOP) ln.init_hop(s);

  double ar[G::EPL], ai[G::EPL];                    // U (wavefront 0) or Lambda (wavefront 1), FP64
  backward_start<T, Q, L, LD>(s, m, ln, wv == 1, ar, ai);
  const long long k0 = s.kstart[m], k1 = s.kstart[m + 1];
  const int kit = kit_of(s);
  const T *ctrl = reinterpret_cast<const T *>(s.ctrl);
  T *ser = reinterpret_cast<T *>(s.series) + (size_t)item * s.maxlen * 2 * Q;
  CkptPos cp(s, k0, k1);
  for (long long k = k1 - 1; k >= k0; --k) {
    typename C2<T>::type ccur[Q];
    load_ctrl<T, Q>(ctrl, k, ccur);
    Coef<T, Q, L, LD> cf;
    step_coeffs<T, Q, L, LD>(ln, ccur, cf);
    T ur[G::EPL], ui[G::EPL], wr[G::EPL], wi[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      ur[e] = (T)ar[e];
      ui[e] = (T)ai[e];
    }
    solve_increment<T, Q, L, LD, true, HOP>(ln, kit, cf, ur, ui, wr, wi);
    T *zrec = zb + (size_t)(k & 1) * 64 * 2 * G::EPL + (size_t)ln.lane * 2 * G::EPL;
    if (wv == 0) {
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        zrec[2 * e] = ur[e] + wr[e];
        zrec[2 * e + 1] = ui[e] + wi[e];
      }
    }
    __syncthreads();                                // both wavefronts, every step
    if (wv == 1) {
      T zr[G::EPL], zi[G::EPL], yr[G::EPL], yi[G::EPL];
#pragma unroll
      for (int e = 0; e < G::EPL; ++e) {
        zr[e] = zrec[2 * e];
        zi[e] = zrec[2 * e + 1];
        yr[e] = ur[e] + wr[e];
        yi[e] = ui[e] + wi[e];
      }
      T s1[Q], s2[Q];
      inner_register_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
      inner_lane_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
      series_put<T, Q>(red, ser, ln.lane, (int)(k - k0), (int)(k1 - k0), s1, s2);
    }
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
      ar[e] += 2.0 * (double)wr[e];
      ai[e] += 2.0 * (double)wi[e];
    }
    ckpt_step<T, Q, L, LD>(s, m, ln, wv == 0, cp, ar, ai);
  }
  if (wv == 0 || !ln.valid) return;
  double2 *l0 = reinterpret_cast<double2 *>(s.lam0) + ((size_t)m * s.E + ln.col) * s.N;
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) l0[ln.row(e)] = double2{ar[e], ai[e]};
}

// Layouts with two or more columns per wavefront, two wavefronts per item: wavefront 0
// solves the state (lanes 0..31) and the adjoint (lanes 32..63) as the split sweep does and
// leaves each lane's step solution in a double-buffered LDS record; in the next iteration
// wavefront 1 reads z (the state lane's record) and y (the adjoint lane's, 32 lanes on) and
// takes that step's inner products and the series flush, so they leave the solving
// wavefront's chain.  Loop and record reuse as in backward_item_x3: one iteration more
// than the window has steps, each ending with the block barrier outside the role branches.
template <typename T, int Q, int L, int LD, bool HOP>
__device__ __forceinline__ void backward_item_sx(const DevSys &s, int m, int cg, T *red, T *xb, T *rb) {
  using G = Geo<T, Q, L, LD>;
  constexpr int RS = 64 * 2 * G::EPL;               // elements of one step's record
  static_assert(2 * G::EPL <= 8, "a step record exceeds its LDS slot (64 lanes x 8 elements)");
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // 0: solves, 1: inner products
  const int item = m * s.ncg_b + cg;
  Lane<T, Q, L, LD> ln;
  ln.init(s, cg, xb, true);
  if constexpr (HOP) {
    if (wv == 0) ln.init_hop(s);
  }
  const bool adj = ln.lane >= 32;                   // state (false) or adjoint (true) half
  const long long k0 = s.kstart[m], k1 = s.kstart[m + 1];
  double ar[G::EPL], ai[G::EPL];                    // U (state lanes) or Lambda (adjoint lanes), FP64
  if (wv == 0) backward_start<T, Q, L, LD>(s, m, ln, adj, ar, ai);
  const int kit = kit_of(s);
  const T *ctrl = reinterpret_cast<const T *>(s.ctrl);
  T *ser = reinterpret_cast<T *>(s.series) + (size_t)item * s.maxlen * 2 * Q;
  CkptPos cp(s, k0, k1);
  typename C2<T>::type cnext[Q];
  if (wv == 0) load_ctrl<T, Q>(ctrl, k1 - 1, cnext);
  // Iteration b: wavefront 0 solves the B steps of block b, leaving each step's record in
  // slot k mod 2B; wavefront 1 takes the inner products of block b-1 (slot reuse as in
  // backward_item_x3).
  constexpr int B = kX3Steps;
  const long long nblk = (k1 - k0 + B - 1) / B;
  for (long long b = 0; b <= nblk; ++b) {
    if (wv == 0 && b < nblk) {
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const long long k = k1 - 1 - b * B - i;
        if (k < k0) break;                          // uniform: the window's first block may be short
        typename C2<T>::type ccur[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) ccur[j] = cnext[j];
        load_ctrl<T, Q>(ctrl, k > k0 ? k - 1 : k, cnext);
        Coef<T, Q, L, LD> cf;
        step_coeffs<T, Q, L, LD>(ln, ccur, cf);
        T ur[G::EPL], ui[G::EPL], wr[G::EPL], wi[G::EPL];
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) {
          ur[e] = (T)ar[e];
          ui[e] = (T)ai[e];
        }
        solve_increment<T, Q, L, LD, true, HOP>(ln, kit, cf, ur, ui, wr, wi);
        T *rec = rb + (size_t)(k & (2 * B - 1)) * RS + ln.lane * 2 * G::EPL;
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) {
          rec[2 * e] = ur[e] + wr[e];
          rec[2 * e + 1] = ui[e] + wi[e];
          ar[e] += 2.0 * (double)wr[e];
          ai[e] += 2.0 * (double)wi[e];
        }
        ckpt_step<T, Q, L, LD>(s, m, ln, !adj, cp, ar, ai);
      }
    }
    if (wv == 1 && b > 0) {                         // inner products of block b - 1
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const long long kp = k1 - 1 - (b - 1) * B - i;
        if (kp < k0) break;
        const T *base = rb + (size_t)(kp & (2 * B - 1)) * RS;
        const T *zrec = base + (ln.lane & 31) * 2 * G::EPL;
        const T *yrec = base + ((ln.lane & 31) + 32) * 2 * G::EPL;
        T zr[G::EPL], zi[G::EPL], yr[G::EPL], yi[G::EPL];
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) {
          zr[e] = zrec[2 * e];
          zi[e] = zrec[2 * e + 1];
          yr[e] = yrec[2 * e];
          yi[e] = yrec[2 * e + 1];
        }
        T s1[Q], s2[Q];
        inner_register_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
        inner_lane_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
#pragma unroll
        for (int j = 0; j < Q; ++j) {               // lanes 32..63 repeat lanes 0..31: count them once
          s1[j] = adj ? (T)0 : s1[j];
          s2[j] = adj ? (T)0 : s2[j];
        }
        series_put<T, Q>(red, ser, ln.lane, (int)(kp - k0), (int)(k1 - k0), s1, s2);
      }
    }
    __syncthreads();                                // every wavefront, every iteration
  }
  if (wv != 0 || !ln.valid || !adj) return;
  double2 *l0 = reinterpret_cast<double2 *>(s.lam0) + ((size_t)m * s.E + ln.col) * s.N;
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) l0[ln.row(e)] = double2{ar[e], ai[e]};
}

// Per block: wavefront 0's and wavefront 1's exchange buffers, the step records (2 kX3Steps
// slots: the split layouts' blocks of steps; the one-column form uses two), and wavefront 1's
// series buffer.
template <typename T, bool HOP>
constexpr int xw_lds_elems() {
  return 2 * (xchg_bytes<T, HOP>() / (int)sizeof(T)) + 2 * kX3Steps * 64 * 8 + red_elems<T>();
}

// Two wavefronts per item: state and adjoint for one-column layouts, solves and inner
// products for layouts with two or more columns per wavefront.
template <typename T, int Q, int L, int LD, bool HOP>
__device__ __forceinline__ void xw_item(const DevSys &s, int m, int cg, T *red, T *xb, T *zb) {
  if constexpr (Geo<T, Q, L, LD>::CPW == 1)
    backward_item_xw<T, Q, L, LD, HOP>(s, m, cg, red, xb, zb);
  else
    backward_item_sx<T, Q, L, LD, HOP>(s, m, cg, red, xb, zb);
}

template <typename T, int Q, int L, int LD, bool HOP>
__global__ __launch_bounds__(128) void k_backward_xw(DevSys s, int nitems) {
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nitems) return;                       // uniform over the block
  __shared__ __align__(16) T lds[xw_lds_elems<T, HOP>()];
  constexpr int XE = xchg_bytes<T, HOP>() / (int)sizeof(T);
  T *xb = lds + (threadIdx.x >> 6) * XE;
  T *zb = lds + 2 * XE;
  T *red = zb + 2 * kX3Steps * 64 * 8;
  xchg_clear<T, HOP>(xb);
  xw_item<T, Q, L, LD, HOP>(s, item / s.ncg_b, item % s.ncg_b, red, xb, zb);
}

// Three wavefronts per (window, column group) for the one-column-per-wavefront layout,
// for launches whose windows are long chains on an otherwise idle GPU: wavefront 0
// reconstructs the state, wavefront 1 propagates the adjoint, and each leaves its step
// solution (z or y) in a double-buffered LDS record; in the next iteration wavefront 2
// reads both records and takes that step's inner products while 0 and 1 solve the
// following step.  The inner products thus leave the solving wavefronts' chain: a step
// costs one solve and one barrier.  The loop runs one iteration more than the window
// has steps and ends every iteration with the block barrier, outside the role branches.
// A record of step k is rewritten (for step k-2) only in the iteration after the one in
// which wavefront 2 read it, i.e. after a barrier.
template <typename T, int Q, int L, int LD, bool HOP>
__device__ __forceinline__ void backward_item_x3(const DevSys &s, int m, int cg, T *red, T *xb, T *zb, T *yb) {
  using G = Geo<T, Q, L, LD>;
  constexpr int RS = 64 * 2 * G::EPL;               // elements of one step's record
  constexpr int B = kX3Steps;                       // steps per barrier
  static_assert(2 * G::EPL <= 8, "a step record exceeds its LDS slot (64 lanes x 8 elements)");
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // 0: state, 1: adjoint, 2: inner products
  const int item = m * s.ncg_b + cg;
  Lane<T, Q, L, LD> ln;
  ln.init(s, cg, xb);
  if constexpr (HOP) {
    if (wv < 2) ln.init_hop(s);
  }
  const long long k0 = s.kstart[m], k1 = s.kstart[m + 1];
  const int roff = ln.lane * 2 * G::EPL;
  double ar[G::EPL], ai[G::EPL];                    // U (wavefront 0) or Lambda (wavefront 1), FP64
  if (wv < 2) backward_start<T, Q, L, LD>(s, m, ln, wv == 1, ar, ai);
  const int kit = kit_of(s);
  const T *ctrl = reinterpret_cast<const T *>(s.ctrl);
  T *ser = reinterpret_cast<T *>(s.series) + (size_t)item * s.maxlen * 2 * Q;
  T *own = (wv == 0 ? zb : yb) + roff;
  CkptPos cp(s, k0, k1);
  // Iteration b: wavefronts 0 and 1 solve the B steps of block b (steps k1-1-bB .. k1-bB-B),
  // leaving z or y in record k mod 2B; wavefront 2 takes the inner products of block b-1.
  // Blocks b and b-1 cover 2B consecutive steps, so their records are distinct; a record of
  // block b-2 is rewritten only after the barrier that ended wavefront 2's reads of it.
  const long long nblk = (k1 - k0 + B - 1) / B;
  for (long long b = 0; b <= nblk; ++b) {
    if (wv < 2 && b < nblk) {
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const long long k = k1 - 1 - b * B - i;
        if (k < k0) break;                          // uniform: the window's first block may be short
        typename C2<T>::type ccur[Q];
        load_ctrl<T, Q>(ctrl, k, ccur);
        Coef<T, Q, L, LD> cf;
        step_coeffs<T, Q, L, LD>(ln, ccur, cf);
        T ur[G::EPL], ui[G::EPL], wr[G::EPL], wi[G::EPL];
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) {
          ur[e] = (T)ar[e];
          ui[e] = (T)ai[e];
        }
        solve_increment<T, Q, L, LD, true, HOP>(ln, kit, cf, ur, ui, wr, wi);
        T *rec = own + (size_t)(k & (2 * B - 1)) * RS;
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) {
          rec[2 * e] = ur[e] + wr[e];
          rec[2 * e + 1] = ui[e] + wi[e];
          ar[e] += 2.0 * (double)wr[e];
          ai[e] += 2.0 * (double)wi[e];
        }
        ckpt_step<T, Q, L, LD>(s, m, ln, wv == 0, cp, ar, ai);
      }
    }
    if (wv == 2 && b > 0) {                         // inner products of block b - 1
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const long long kp = k1 - 1 - (b - 1) * B - i;
        if (kp < k0) break;
        const T *zrec = zb + (size_t)(kp & (2 * B - 1)) * RS + roff;
        const T *yrec = yb + (size_t)(kp & (2 * B - 1)) * RS + roff;
        T zr[G::EPL], zi[G::EPL], yr[G::EPL], yi[G::EPL];
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) {
          zr[e] = zrec[2 * e];
          zi[e] = zrec[2 * e + 1];
          yr[e] = yrec[2 * e];
          yi[e] = yrec[2 * e + 1];
        }
        T s1[Q], s2[Q];
        inner_register_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
        inner_lane_digits<T, Q, L, LD>(ln, zr, zi, yr, yi, s1, s2);
        series_put<T, Q>(red, ser, ln.lane, (int)(kp - k0), (int)(k1 - k0), s1, s2);
      }
    }
    __syncthreads();                                // every wavefront, every iteration
  }
  if (wv != 1 || !ln.valid) return;
  double2 *l0 = reinterpret_cast<double2 *>(s.lam0) + ((size_t)m * s.E + ln.col) * s.N;
#pragma unroll
  for (int e = 0; e < G::EPL; ++e) l0[ln.row(e)] = double2{ar[e], ai[e]};
}

// Per block: three exchange buffers, the z and y records of 2 kX3Steps steps each, and
// wavefront 2's series buffer.
template <typename T, bool HOP>
constexpr int x3_lds_elems() {
  return 3 * (xchg_bytes<T, HOP>() / (int)sizeof(T)) + 2 * (2 * kX3Steps) * 64 * 8 + red_elems<T>();
}

template <typename T, int Q, int L, int LD, bool HOP>
__global__ __launch_bounds__(192) void k_backward_x3(DevSys s, int nitems) {
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= nitems) return;                       // uniform over the block
  __shared__ __align__(16) T lds[x3_lds_elems<T, HOP>()];
  constexpr int XE = xchg_bytes<T, HOP>() / (int)sizeof(T);
  T *xb = lds + (threadIdx.x >> 6) * XE;
  T *zb = lds + 3 * XE;
  T *yb = zb + 2 * kX3Steps * 64 * 8;
  T *red = yb + 2 * kX3Steps * 64 * 8;
  xchg_clear<T, HOP>(xb);
  backward_item_x3<T, Q, L, LD, HOP>(s, item / s.ncg_b, item % s.ncg_b, red, xb, zb, yb);
}

template <typename T, int Q, int L, int LD, bool HOP>
__device__ __forceinline__ void x3_item(const DevSys &s, int m, int cg, T *red, T *xb, T *zb, T *yb) {
  if constexpr (Geo<T, Q, L, LD>::CPW == 1) backward_item_x3<T, Q, L, LD, HOP>(s, m, cg, red, xb, zb, yb);
}

// ---------------------------------------------------------------------------- small FP64 kernels

// Fixed-point iteration count.  The Jacobi map w -> (D^{-1} - 1)u - i D^{-1} (dt/2) H_c (u + w)
// contracts in the 2-norm by rho_k <= |D^{-1}| nu_L sum_j |c'_j(t_k)| with |D^{-1}| <= 1,
// c'_j = (dt/2) 2 pi d_j and nu_L = ||a + a^+||_2; k_controls leaves max_k of that bound
// in rho_bits.  Starting from w = (D^{-1} - 1)u (error <= rho |z|):
//  Jacobi (odd L): K iterations leave <= rho^(K+1) |z|; K is the smallest count with
//    rho^(K+1) <= solve_tol.
//  red-black (even L): each half sweep multiplies the refreshed colour's error by a
//    block of the iteration matrix (2-norm <= rho), so after h half sweeps the colours
//    carry <= rho^(h+1) |z| and <= rho^h |z|, together <= rho^h sqrt(1 + rho^2) |z|;
//    h is the smallest count with that <= solve_tol.
//  with the dipole exchange H_J (beta >= |D^{-1}| ||(dt/2) H_J||_2 > 0), the start error is
//    <= (rho + beta)|z|; a Jacobi iteration contracts by rho + beta, and a half sweep of
//    colour C bounds that colour's error by rho (other colour) + beta (its own).
__device__ void kit_block(const DevSys &s) {
  if (threadIdx.x != 0) return;
  const double rho = (double)__uint_as_float(*s.rho_bits) * (1.0 + 1e-6);
  *s.rho_bits = 0u;                  // reset for the next evaluation
  const bool rb = (s.L % 2) == 0 && s.q - s.ld >= 1;   // the layout's red-black ordering (Geo::RB)
  const double beta = s.beta, tau = rho + beta;
  int K = 1;
  double err;
  if (beta == 0.0) {
    err = rb ? rho * sqrt(1.0 + rho * rho) : rho * rho;
    while (err > s.solve_tol && K < 64) { err *= rho; ++K; }
  } else if (!rb) {                  // Jacobi on H_c + H_J: tau^(K+1)
    err = tau * tau;
    while (err > s.solve_tol && K < 64) { err *= tau; ++K; }
  } else {
    // Red-black with the exchange term: a half sweep of colour C bounds that colour's
    // error by rho * (other colour) + beta * (its own previous error); both start at tau.
    double x0 = tau, x1 = tau;
    x0 = rho * x1 + beta * x0;
    err = sqrt(x0 * x0 + x1 * x1);
    while (err > s.solve_tol && K < 64) {
      ++K;
      if (K & 1) x0 = rho * x1 + beta * x0;
      else x1 = rho * x0 + beta * x1;
      err = sqrt(x0 * x0 + x1 * x1);
    }
  }
  if (s.kit_fixed <= 0) *s.kit = K;
  if (s.kit_fixed <= 0 && (err > s.solve_tol || tau >= 0.5)) atomicOr(s.status, (int)STATUS_NOTCONV);
}

// (dt/2) * 2 pi d_j(t_{k+1/2}) for every step; B_s(t) = B(t/dtau + 1/2 - s); and the
// per-step contraction bound nu_L sum_j |c'_j| maximised into rho_bits.
template <typename T>
__device__ void controls_block(const DevSys &s, int blk) {
  using V2 = typename C2<T>::type;
  __shared__ float smax[256];
  const long long k = (long long)blk * 256 + threadIdx.x;
  float rho = 0.f;
  if (k < s.NT) {
    const double t = (k + 0.5) * s.dt;
    const double x = t / s.dtau + 0.5;
    const int slo = max(0, (int)ceil(x - 1.5)), shi = min(s.d1 - 1, (int)floor(x + 1.5));
    const double scale = M_PI * s.dt;   // (dt/2) * 2 pi
    V2 *out = reinterpret_cast<V2 *>(s.ctrl) + k * s.q;
    double bound = 0.0;
    for (int j = 0; j < s.q; ++j) {
      double dre = 0.0, dim = 0.0;
      for (int f = 0; f < s.nf; ++f) {
        double er = 0.0, ei = 0.0;
        const double *a = s.alpha + (size_t)(j * s.nf + f) * 2 * s.d1;
        for (int sp = slo; sp <= shi; ++sp) {
          const double b = bspline2(x - sp);
          er += a[sp] * b;
          ei += a[s.d1 + sp] * b;
        }
        double sn, cs;
        sincos(s.carrier[j * s.nf + f] * t, &sn, &cs);
        dre += er * cs - ei * sn;
        dim += er * sn + ei * cs;
      }
      out[j] = V2{(T)(scale * dre), (T)(scale * dim)};
      bound += scale * sqrt(dre * dre + dim * dim);
    }
    rho = (float)(bound * s.nu_L);
  }
  smax[threadIdx.x] = rho;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(s.rho_bits, __float_as_uint(smax[0]));   // nonnegative floats order as integers
}

template <int NT_>
__device__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int w = NT_ / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per window: |U^m - W^m|_F^2 (m < M) or |U^M|_F^2 and gamma = <V, U^M>_F (m = M), in FP64.
__device__ void boundary_partial_block(const DevSys &s, int m) {
  __shared__ double sh[256];
  const size_t n = (size_t)s.E * s.N;
  const double2 *u = reinterpret_cast<const double2 *>(s.Ufin) + (size_t)m * n;
  double a = 0.0, b = 0.0, c = 0.0;
  if (m < s.M - 1) {
    const double2 *w = reinterpret_cast<const double2 *>(s.W) + (size_t)m * n;
    for (size_t i = threadIdx.x; i < n; i += 256) {
      const double dr = u[i].x - w[i].x, di = u[i].y - w[i].y;
      a += dr * dr + di * di;
    }
  } else {
    const double2 *V = reinterpret_cast<const double2 *>(s.V);
    for (size_t i = threadIdx.x; i < n; i += 256) {
      const double ur = u[i].x, ui = u[i].y, vr = V[i].x, vi = V[i].y;
      a += ur * ur + ui * ui;
      b += vr * ur + vi * ui;   // conj(v) u
      c += vr * ui - vi * ur;
    }
  }
  a = block_sum<256>(a, sh);
  b = block_sum<256>(b, sh);
  c = block_sum<256>(c, sh);
  if (threadIdx.x == 0) {
    s.partials[4 * m + 0] = a;
    s.partials[4 * m + 1] = b;
    s.partials[4 * m + 2] = c;
  }
}

__device__ void boundary_final_block(const DevSys &s) {
  // the per-window penalties are copied by all threads and summed by one, in window order,
  // from LDS (a serial loop over device memory would wait on every load in turn)
  __shared__ double pw[256];
  double pen = 0.0;
  for (int m0 = 0; m0 < s.M - 1; m0 += 256) {
    const int m = m0 + (int)threadIdx.x;
    if (m < s.M - 1) {
      pw[threadIdx.x] = s.partials[4 * m];
      s.scal[6 + m] = pw[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = min(256, s.M - 1 - m0);
      for (int i = 0; i < n; ++i) pen += pw[i];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double E = (double)s.E;
  const double nrm = s.partials[4 * (s.M - 1)], gr = s.partials[4 * (s.M - 1) + 1], gi = s.partials[4 * (s.M - 1) + 2];
  const double J = nrm / E - (gr * gr + gi * gi) / (E * E);
  pen *= 0.5 * s.mu;
  s.scal[0] = J + pen;
  s.scal[1] = J;
  s.scal[2] = pen;
  s.scal[3] = nrm;
  s.scal[4] = gr;
  s.scal[5] = gi;
}

// xy[k] = sum over the window's column groups of the per-wavefront series (stored in the
// propagation precision T), in FP64 and group order; one thread per step, reading each
// group's record of 2q values in pairs.
template <typename T>
__device__ void series_reduce_block(const DevSys &s, int blk) {
  using V2 = typename C2<T>::type;
  const long long k = (long long)blk * 256 + threadIdx.x;
  if (k >= s.NT) return;
  const int m = (int)(((k + 1) * s.M - 1) / s.NT);   // window of step k under the floor split
  const long long kk = k - s.kstart[m];
  const int w = 2 * s.q;
  double acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = 0.0;
  for (int cg = 0; cg < s.ncg_b; ++cg) {     // one contiguous record of 2q values per column group
    const V2 *src = reinterpret_cast<const V2 *>(reinterpret_cast<const T *>(s.series) +
                                                 (((size_t)m * s.ncg_b + cg) * s.maxlen + kk) * w);
#pragma unroll
    for (int i = 0; i < 6; ++i)
      if (2 * i < w) {
        const V2 v = src[i];
        acc[2 * i] += (double)v.x;
        acc[2 * i + 1] += (double)v.y;
      }
  }
#pragma unroll
  for (int i = 0; i < 12; ++i)
    if (i < w) s.xy[(size_t)k * w + i] = acc[i];
}

// dP/dalpha for one (qubit j, carrier f, spline s): with X = -2 dt 2 pi Im<y,(a+a^+)z>,
// Y = -2 dt 2 pi Re<y,(a-a^+)z> per step,
//   dP/dalpha1 = sum_k B_s(t_k) (cos(W t_k) X_k + sin(W t_k) Y_k),
//   dP/dalpha2 = sum_k B_s(t_k) (-sin(W t_k) X_k + cos(W t_k) Y_k).
__device__ void project_block(const DevSys &s, int b) {
  __shared__ double sh[256];
  const int sp = b % s.d1, jf = b / s.d1, j = jf / s.nf;
  const double om = s.carrier[jf];
  const double r = s.dtau / s.dt;
  const long long klo = max(0LL, (long long)floor((sp - 2.0) * r - 0.5));
  const long long khi = min(s.NT - 1, (long long)ceil((sp + 1.0) * r - 0.5));
  double a1 = 0.0, a2 = 0.0;
  // the carrier phase advances by om * 256 dt between a thread's steps: one sincos per
  // thread, then a rotation per step (about 20 per thread at 4 qubits; error ~1e-15)
  const long long k0 = klo + threadIdx.x;
  double sn, cs, sd, cd;
  sincos(om * ((k0 + 0.5) * s.dt), &sn, &cs);
  sincos(om * (256.0 * s.dt), &sd, &cd);
  for (long long k = k0; k <= khi; k += 256) {
    const double t = (k + 0.5) * s.dt;
    const double bs = bspline2(t / s.dtau + 0.5 - sp);
    if (bs != 0.0) {
      const double s1 = s.xy[(size_t)k * 2 * s.q + 2 * j], s2 = s.xy[(size_t)k * 2 * s.q + 2 * j + 1];
      a1 += bs * (cs * s1 + sn * s2);
      a2 += bs * (-sn * s1 + cs * s2);
    }
    const double sn2 = sn * cd + cs * sd;
    cs = cs * cd - sn * sd;
    sn = sn2;
  }
  a1 = block_sum<256>(a1, sh);
  a2 = block_sum<256>(a2, sh);
  if (threadIdx.x == 0) {
    const double fac = -4.0 * M_PI * s.dt;
    s.grad_alpha[((size_t)jf * 2 + 0) * s.d1 + sp] = fac * a1;
    s.grad_alpha[((size_t)jf * 2 + 1) * s.d1 + sp] = fac * a2;
  }
}

// dP/dW^m = mu (W^m - U^m(t_m)) - 2 Lambda^{m+1}(t_m).  For m = M-1 the backward sweep
// propagated only gamma V/E^2 of the last window's terminal condition; the dropped part
// -U^M/E equals -W^{M-1}/E at t_{M-1}, which adds (2/E) W^{M-1} here.
__device__ void grad_W_block(const DevSys &s, int blk) {
  const size_t n = (size_t)s.E * s.N;
  const size_t idx = (size_t)blk * 256 + threadIdx.x;
  if (idx >= (size_t)(s.M - 1) * n) return;
  const size_t m = idx / n, rest = idx % n;       // window m+1 (1-based) ends at t_{m+1}
  const double2 u = reinterpret_cast<const double2 *>(s.Ufin)[m * n + rest];
  const double2 l = reinterpret_cast<const double2 *>(s.lam0)[(m + 1) * n + rest];
  const double2 w = reinterpret_cast<const double2 *>(s.W)[idx];
  const double extra = (m + 2 == (size_t)s.M) ? 2.0 / (double)s.E : 0.0;
  s.grad_W[2 * idx] = s.mu * (w.x - u.x) - 2.0 * l.x + extra * w.x;
  s.grad_W[2 * idx + 1] = s.mu * (w.y - u.y) - 2.0 * l.y + extra * w.y;
}

// Single-system kernels and their batched forms.  A batched launch reads, per
// block, (system index, block index within that system) from a table.
template <typename T, int K>
__device__ __forceinline__ void small_block(const DevSys &s, int blk) {
  if constexpr (K == SK_CONTROLS) controls_block<T>(s, blk);
  else if constexpr (K == SK_KIT) kit_block(s);
  else if constexpr (K == SK_BPARTIAL) boundary_partial_block(s, blk);
  else if constexpr (K == SK_BFINAL) boundary_final_block(s);
  else if constexpr (K == SK_SERIES) series_reduce_block<T>(s, blk);
  else if constexpr (K == SK_PROJECT) project_block(s, blk);
  else grad_W_block(s, blk);
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_small(DevSys s) { small_block<T, K>(s, blockIdx.x); }

template <typename T, int K>
__global__ __launch_bounds__(256) void k_small_batch(const DevSys *sys, const int2 *blocks) {
  const int2 b = blocks[blockIdx.x];
  const DevSys s = sys[b.x];
  small_block<T, K>(s, b.y);
}

// ---------------------------------------------------------------------------- dispatch

// (q, L) -> lane digits, chosen so that each lane holds at most four entries
// per state (the backward sweep keeps about 16 such arrays live).  Two-level
// systems use two entries per lane: their windows are latency-bound chains (few
// wavefronts, several columns each), and halving a lane's entries halves its
// instructions per step.  For the same reason the 2-qubit 3-level and 3-qubit
// 4-level systems put every digit on lanes (one entry per lane, Jacobi iteration).
#define QOC_SHAPES(X)   \
  X(1, 2, 0) X(1, 3, 0) X(1, 4, 0) \
  X(2, 2, 1) X(2, 3, 2) X(2, 4, 1) \
  X(3, 2, 2) X(3, 3, 2) X(3, 4, 3) \
  X(4, 2, 3) X(4, 3, 3) X(4, 4, 3) \
  X(5, 2, 4) X(6, 2, 5)

enum KernelKind { KK_FWD, KK_BWD, KK_XW, KK_X3 };

// Kernel instances built in a compilation unit of their own (qoc_ilp_unit.hip, which
// includes this file with QOC_ILP_UNIT defined) that the build gives the instruction
// scheduler's ILP strategy.  It shortens these (the headline 4-qubit FP32 backward, the FP32
// forward of the 4-qubit system with dipole terms, and the latency-bound sweeps of the 2-qubit
// 3-level FP64 and 3-qubit 4-level FP32 systems as their default schedules run them) without
// costing occupancy their launches use; for other kernels it lowers occupancy a launch needs or
// spills (the 4-qubit FP32 backward with dipole terms among them).
template <typename T, int Q, int L, bool HOP, int KK>
constexpr bool ilp_held() {
  if constexpr (HOP) return sizeof(T) == 4 && Q == 4 && L == 4 && KK == KK_FWD;
  else if constexpr (sizeof(T) == 4 && Q == 4 && L == 4) return KK == KK_BWD;
  else if constexpr (sizeof(T) == 8 && Q == 2 && L == 3) return KK == KK_FWD || KK == KK_XW;
  else if constexpr (sizeof(T) == 4 && Q == 3 && L == 4) return KK == KK_FWD || KK == KK_X3;
  else return false;
}

}  // namespace

struct Kernels {
  void (*fwd)(DevSys, double *, double *, int);
  void (*roll)(DevSys, double *, double *, int);
  void (*bwd)(DevSys, int);
  void (*bwd_xw)(DevSys, int);     // two wavefronts per item
  void (*bwd_x3)(DevSys, int);     // three wavefronts per item (one-column layouts only)
};

// Fills the fields of *k that the ILP unit holds for (precision, q, L, dipole terms).
void ilp_kernels(int fp64, int q, int L, int hop, Kernels *k);

namespace {

#ifndef QOC_ILP_UNIT
// This unit's instances; those the ILP unit holds are left null for ilp_kernels().
template <typename T, int Q, int L, int LD, bool HOP>
Kernels make() {
  Kernels k{nullptr, k_forward<T, Q, L, LD, true, HOP>, nullptr, nullptr, nullptr};
  if constexpr (!ilp_held<T, Q, L, HOP, KK_FWD>()) k.fwd = k_forward<T, Q, L, LD, false, HOP>;
  if constexpr (!ilp_held<T, Q, L, HOP, KK_BWD>()) k.bwd = k_backward<T, Q, L, LD, HOP>;
  if constexpr (!ilp_held<T, Q, L, HOP, KK_XW>()) k.bwd_xw = k_backward_xw<T, Q, L, LD, HOP>;
  if constexpr (Geo<T, Q, L, LD>::CPW == 1 && !ilp_held<T, Q, L, HOP, KK_X3>()) k.bwd_x3 = k_backward_x3<T, Q, L, LD, HOP>;
  return k;
}

// Kernel-instance index: the shape, plus N_SHAPES for the dipole variant.
#define X(Q_, L_, LD_) SHAPE_##Q_##_##L_,
enum ShapeId { QOC_SHAPES(X) N_SHAPES };
#undef X

template <typename T>
bool lookup(int q, int L, bool hop, Kernels *k, int *ld, int *cpw, int *shape) {
#define X(Q_, L_, LD_)                                                             \
  if (q == Q_ && L == L_) {                                                        \
    if (k) {                                                                       \
      *k = hop ? make<T, Q_, L_, LD_, true>() : make<T, Q_, L_, LD_, false>();     \
      ilp_kernels(sizeof(T) == 8, q, L, hop, k);                                   \
    }                                                                              \
    *ld = LD_;                                                                     \
    *cpw = Geo<T, Q_, L_, LD_>::CPW;                                               \
    if (shape) *shape = SHAPE_##Q_##_##L_ + (hop ? N_SHAPES : 0);                  \
    return true;                                                                   \
  }
  QOC_SHAPES(X)
#undef X
  return false;
}

// Batched propagation: one wavefront per item (system, window, column group, shape),
// items ordered by the host (longest first).
template <typename T>
__global__ __launch_bounds__(64) void k_forward_batch(const DevSys *sys, const int4 *items) {
  __shared__ __align__(16) T xb[xchg_bytes<T, true>() / sizeof(T)];   // either variant
  xchg_clear<T, true>(xb);
  const int4 it = items[blockIdx.x];
  const DevSys s = sys[it.x];
  switch (it.w) {
#define X(Q_, L_, LD_)                                                                                     \
    case SHAPE_##Q_##_##L_: forward_item<T, Q_, L_, LD_, false, false>(s, it.y, it.z, nullptr, nullptr, xb); break; \
    case N_SHAPES + SHAPE_##Q_##_##L_:                                                                     \
      forward_item<T, Q_, L_, LD_, false, true>(s, it.y, it.z, nullptr, nullptr, xb);                     \
      break;
    QOC_SHAPES(X)
#undef X
    default: break;
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_backward_batch(const DevSys *sys, const int4 *items) {
  __shared__ T red[red_elems<T>()];
  __shared__ __align__(16) T xb[xchg_bytes<T, true>() / sizeof(T)];   // either variant
  xchg_clear<T, true>(xb);
  const int4 it = items[blockIdx.x];
  const DevSys s = sys[it.x];
  switch (it.w) {
#define X(Q_, L_, LD_)                                                                      \
    case SHAPE_##Q_##_##L_: backward_item<T, Q_, L_, LD_, false>(s, it.y, it.z, red, xb); break; \
    case N_SHAPES + SHAPE_##Q_##_##L_: backward_item<T, Q_, L_, LD_, true>(s, it.y, it.z, red, xb); break;
    QOC_SHAPES(X)
#undef X
    default: break;
  }
}

template <typename T>
__global__ __launch_bounds__(128) void k_backward_xw_batch(const DevSys *sys, const int4 *items) {
  __shared__ __align__(16) T lds[xw_lds_elems<T, true>()];   // either variant
  constexpr int XE = xchg_bytes<T, true>() / (int)sizeof(T);
  T *xb = lds + (threadIdx.x >> 6) * XE;
  T *zb = lds + 2 * XE;
  T *red = zb + 2 * kX3Steps * 64 * 8;
  xchg_clear<T, true>(xb);
  const int4 it = items[blockIdx.x];
  const DevSys s = sys[it.x];
  switch (it.w) {
#define X(Q_, L_, LD_)                                                                         \
    case SHAPE_##Q_##_##L_: xw_item<T, Q_, L_, LD_, false>(s, it.y, it.z, red, xb, zb); break; \
    case N_SHAPES + SHAPE_##Q_##_##L_: xw_item<T, Q_, L_, LD_, true>(s, it.y, it.z, red, xb, zb); break;
    QOC_SHAPES(X)
#undef X
    default: break;
  }
}

template <typename T>
__global__ __launch_bounds__(192) void k_backward_x3_batch(const DevSys *sys, const int4 *items) {
  __shared__ __align__(16) T lds[x3_lds_elems<T, true>()];   // either variant
  constexpr int XE = xchg_bytes<T, true>() / (int)sizeof(T);
  T *xb = lds + (threadIdx.x >> 6) * XE;
  T *zb = lds + 3 * XE;
  T *yb = zb + 2 * kX3Steps * 64 * 8;
  T *red = yb + 2 * kX3Steps * 64 * 8;
  xchg_clear<T, true>(xb);
  const int4 it = items[blockIdx.x];
  const DevSys s = sys[it.x];
  switch (it.w) {
#define X(Q_, L_, LD_)                                                                             \
    case SHAPE_##Q_##_##L_: x3_item<T, Q_, L_, LD_, false>(s, it.y, it.z, red, xb, zb, yb); break; \
    case N_SHAPES + SHAPE_##Q_##_##L_: x3_item<T, Q_, L_, LD_, true>(s, it.y, it.z, red, xb, zb, yb); break;
    QOC_SHAPES(X)
#undef X
    default: break;
  }
}

int grid8(int n) { return (n + 7) / 8 * 8; }

template <typename T, int K>
void small(const DevSys &s, hipStream_t st) {
  const int nb = small_blocks(s, K);
  if (nb > 0) hipLaunchKernelGGL((k_small<T, K>), dim3(nb), dim3(256), 0, st, s);
}

template <typename T>
int phase_T(const DevSys &s, int phase, hipStream_t st, double *Wout, double *Ufinal) {
  Kernels K;
  int ld, cpw;
  if (!lookup<T>(s.q, s.L, s.hop != 0, &K, &ld, &cpw, nullptr)) return (int)hipErrorInvalidValue;
  const int nitems = s.M * s.ncg;
  switch (phase) {
    case PHASE_CONTROLS:
      small<T, SK_CONTROLS>(s, st);
      small<T, SK_KIT>(s, st);
      break;
    case PHASE_FORWARD:
      hipLaunchKernelGGL(K.fwd, dim3(grid8(nitems)), dim3(64), 0, st, s, (double *)nullptr, (double *)nullptr, nitems);
      break;
    case PHASE_BOUNDARY:
      small<T, SK_BPARTIAL>(s, st);
      small<T, SK_BFINAL>(s, st);
      break;
    case PHASE_BACKWARD: {
      const int waves = bwd_waves(s);
      if (waves == 3 && K.bwd_x3)
        hipLaunchKernelGGL(K.bwd_x3, dim3(grid8(s.M * s.ncg_b)), dim3(192), 0, st, s, s.M * s.ncg_b);
      else if (waves == 2 && K.bwd_xw)
        hipLaunchKernelGGL(K.bwd_xw, dim3(grid8(s.M * s.ncg_b)), dim3(128), 0, st, s, s.M * s.ncg_b);
      else
        hipLaunchKernelGGL(K.bwd, dim3(grid8(s.M * s.ncg_b)), dim3(64), 0, st, s, s.M * s.ncg_b);
      break;
    }
    case PHASE_PROJECT:
      small<T, SK_SERIES>(s, st);
      small<T, SK_PROJECT>(s, st);
      break;
    case PHASE_GRAD_W:
      small<T, SK_GRADW>(s, st);
      break;
    case PHASE_ROLLOUT:
      hipLaunchKernelGGL(K.roll, dim3(grid8(s.ncg)), dim3(64), 0, st, s, Wout, Ufinal, s.ncg);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <typename T, int K>
void small_batched(const BatchPlan &p, hipStream_t st) {
  if (p.n_blocks[K] > 0)
    hipLaunchKernelGGL((k_small_batch<T, K>), dim3(p.n_blocks[K]), dim3(256), 0, st, p.sys, p.blocks[K]);
}

template <typename T>
int batch_phase_T(const BatchPlan &p, int phase, hipStream_t st) {
  switch (phase) {
    case PHASE_CONTROLS:
      small_batched<T, SK_CONTROLS>(p, st);
      small_batched<T, SK_KIT>(p, st);
      break;
    case PHASE_FORWARD:
      if (p.n_fwd > 0) hipLaunchKernelGGL(k_forward_batch<T>, dim3(p.n_fwd), dim3(64), 0, st, p.sys, p.fwd_items);
      break;
    case PHASE_BOUNDARY:
      small_batched<T, SK_BPARTIAL>(p, st);
      small_batched<T, SK_BFINAL>(p, st);
      break;
    case PHASE_BACKWARD: {
      // a single kind of backward items runs on st; with several kinds, the items of two and
      // of three wavefronts run beside the others, each kind on a stream of the batch forked
      // from st and joined back to it
      const int kinds = (p.n_bwd > 0) + (p.n_xw > 0) + (p.n_x3 > 0);
      if (kinds <= 1 || !p.aux || !p.aux2) {      // one kind, or no streams of the batch: all on st
        if (p.n_x3 > 0) hipLaunchKernelGGL(k_backward_x3_batch<T>, dim3(p.n_x3), dim3(192), 0, st, p.sys, p.x3_items);
        if (p.n_xw > 0) hipLaunchKernelGGL(k_backward_xw_batch<T>, dim3(p.n_xw), dim3(128), 0, st, p.sys, p.xw_items);
        if (p.n_bwd > 0) hipLaunchKernelGGL(k_backward_batch<T>, dim3(p.n_bwd), dim3(64), 0, st, p.sys, p.bwd_items);
        break;
      }
      hipError_t e = hipSuccess;
      if (p.n_xw > 0 || p.n_x3 > 0) e = hipEventRecord(p.fork, st);
      if (e == hipSuccess && p.n_xw > 0) e = hipStreamWaitEvent(p.aux, p.fork, 0);
      if (e == hipSuccess && p.n_x3 > 0) e = hipStreamWaitEvent(p.aux2, p.fork, 0);
      if (e != hipSuccess) return (int)e;
      if (p.n_x3 > 0)
        hipLaunchKernelGGL(k_backward_x3_batch<T>, dim3(p.n_x3), dim3(192), 0, p.aux2, p.sys, p.x3_items);
      if (p.n_xw > 0)
        hipLaunchKernelGGL(k_backward_xw_batch<T>, dim3(p.n_xw), dim3(128), 0, p.aux, p.sys, p.xw_items);
      if (p.n_bwd > 0) hipLaunchKernelGGL(k_backward_batch<T>, dim3(p.n_bwd), dim3(64), 0, st, p.sys, p.bwd_items);
      if (p.n_xw > 0) {
        e = hipEventRecord(p.join, p.aux);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, p.join, 0);
        if (e != hipSuccess) return (int)e;
      }
      if (p.n_x3 > 0) {
        e = hipEventRecord(p.join2, p.aux2);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, p.join2, 0);
        if (e != hipSuccess) return (int)e;
      }
      break;
    }
    case PHASE_PROJECT:
      small_batched<T, SK_SERIES>(p, st);
      small_batched<T, SK_PROJECT>(p, st);
      break;
    case PHASE_GRAD_W:
      small_batched<T, SK_GRADW>(p, st);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// Status words of the systems of a batch, in batch order: out[i] = system i's flags,
// which are then cleared (the batch reports them from here on).
__global__ __launch_bounds__(256) void k_gather_status(const DevSys *sys, int n, int *out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int *st = sys[i].status;
  out[i] = st[0];
  st[0] = 0;
}

// Tables of the allocation-free batched run (systems, item records, block table).  In host
// code this name is only a handle for hipGetSymbolAddress; the device address is looked up
// per GPU by noalloc_scratch() and used everywhere else.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

}  // namespace

int noalloc_scratch(int device, void **out) {
  constexpr int kMaxDevices = 64;
  static void *addr[kMaxDevices] = {};
  static std::mutex lock;
  if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    addr[device] = p;
  }
  *out = addr[device];
  return 0;
}

int launch_gather_status(const DevSys *sys, int n, int *out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_status, dim3((n + 255) / 256), dim3(256), 0, st, sys, n, out);
  return (int)hipGetLastError();
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

bool layout_for(int q, int L, int fp64, int hop, int *ld, int *cpw, int *shape) {
  return fp64 ? lookup<double>(q, L, hop != 0, nullptr, ld, cpw, shape)
              : lookup<float>(q, L, hop != 0, nullptr, ld, cpw, shape);
}

int launch_phase(const DevSys &s, int phase, hipStream_t st, double *Wout, double *Ufinal) {
  return s.fp64 ? phase_T<double>(s, phase, st, Wout, Ufinal) : phase_T<float>(s, phase, st, Wout, Ufinal);
}

int launch_batch_phase(const BatchPlan &p, int phase, hipStream_t st) {
  return p.fp64 ? batch_phase_T<double>(p, phase, st) : batch_phase_T<float>(p, phase, st);
}

#else   // QOC_ILP_UNIT

template <typename T, int Q, int L, int LD, bool HOP>
void ilp_fill(Kernels *k) {
  if constexpr (ilp_held<T, Q, L, HOP, KK_FWD>()) k->fwd = k_forward<T, Q, L, LD, false, HOP>;
  if constexpr (ilp_held<T, Q, L, HOP, KK_BWD>()) k->bwd = k_backward<T, Q, L, LD, HOP>;
  if constexpr (ilp_held<T, Q, L, HOP, KK_XW>()) k->bwd_xw = k_backward_xw<T, Q, L, LD, HOP>;
  if constexpr (Geo<T, Q, L, LD>::CPW == 1 && ilp_held<T, Q, L, HOP, KK_X3>()) k->bwd_x3 = k_backward_x3<T, Q, L, LD, HOP>;
}

}  // namespace

void ilp_kernels(int fp64, int q, int L, int hop, Kernels *k) {
#define X(Q_, L_, LD_)                                                                   \
  if (q == Q_ && L == L_) {                                                              \
    if (fp64) hop ? ilp_fill<double, Q_, L_, LD_, true>(k) : ilp_fill<double, Q_, L_, LD_, false>(k); \
    else hop ? ilp_fill<float, Q_, L_, LD_, true>(k) : ilp_fill<float, Q_, L_, LD_, false>(k);       \
  }
  QOC_SHAPES(X)
#undef X
}

#endif  // QOC_ILP_UNIT

}  // namespace qoc
