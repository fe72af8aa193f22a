// FP64 device kernels of the optimisation driver (qoc_opt.cpp): deterministic
// reductions and vector updates over the optimisation variables x = [alpha, sigma W],
// and the control-energy term of Sec. 5 with its gradient.  Every reduction runs
// over a fixed grid in a fixed order, so results do not depend on timing.
#include "qoc_internal.h"

#include <cmath>

namespace qoc {
namespace {

constexpr int kThreads = 256;

__device__ double block_reduce_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  return sh[0];
}

__device__ double block_reduce_max(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] = fmax(sh[t], sh[t + w]);
    __syncthreads();
  }
  return sh[0];
}

// partials[b] = sum over i = b*256 + t + k*(grid*256) of a_i b_i (each thread in index order)
__global__ __launch_bounds__(kThreads) void k_dot_partial(const double *a, const double *b, long long n,
                                                          double *partials) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    acc = fma(a[i], b[i], acc);
  const double s = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// partials[b] = max |v_i| over the block's indices, v_i zeroed on the active set (see k_reduced)
__global__ __launch_bounds__(kThreads) void k_maxabs_partial(const double *v, long long n, double *partials) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    acc = fmax(acc, fabs(v[i]));
  const double s = block_reduce_max(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[0] = sum (or max) of partials[0..m) in a fixed tree order; for sums, optionally
// combined with a device scalar: out[0] = cb * base[0] + cs * sum (base non-null).
template <bool MAX>
__global__ __launch_bounds__(kThreads) void k_finish(const double *partials, int m, double *out, const double *base,
                                                     double cb, double cs) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += kThreads) acc = MAX ? fmax(acc, partials[i]) : acc + partials[i];
  const double s = MAX ? block_reduce_max(acc, sh) : block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (MAX || !base) out[0] = MAX ? s : cs * s;
    else out[0] = cb * base[0] + cs * s;
  }
}

// y = a x + b y
__global__ __launch_bounds__(kThreads) void k_axpby(double *y, double a, const double *x, double b, long long n) {
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    y[i] = fma(a, x[i], b * y[i]);
}

// y = (s c[0]) x + y with the coefficient c[0] in device memory
__global__ __launch_bounds__(kThreads) void k_axpy_dev(double *y, const double *c, double s, const double *x,
                                                       long long n) {
  const double a = s * c[0];
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    y[i] = fma(a, x[i], y[i]);
}

// xt = x + t p, the first d entries clipped to [lo, hi]
__global__ __launch_bounds__(kThreads) void k_trial(double *xt, const double *x, const double *p, double t, long long n,
                                                    long long d, double lo, double hi) {
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    double v = fma(t, p[i], x[i]);
    if (i < d) v = fmin(fmax(v, lo), hi);
    xt[i] = v;
  }
}

// out = v with the active set zeroed: entry i < d of x at a bound with g pointing outwards
__global__ __launch_bounds__(kThreads) void k_reduced(double *out, const double *v, const double *x, const double *g,
                                                      long long n, long long d, double lo, double hi) {
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    bool active = false;
    if (i < d) active = (x[i] <= lo && g[i] > 0.0) || (x[i] >= hi && g[i] < 0.0);
    out[i] = active ? 0.0 : v[i];
  }
}

// g = [ga + gtik alpha + gen gE ; s gW]
__global__ __launch_bounds__(kThreads) void k_assemble(double *g, const double *ga, const double *alpha,
                                                       const double *gE, const double *gW, long long d, long long nW,
                                                       double gtik, double gen, double s) {
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < d + nW; i += (long long)gridDim.x * kThreads)
    g[i] = i < d ? fma(gen, gE[i], fma(gtik, alpha[i], ga[i])) : s * gW[i - d];
}

__device__ __forceinline__ double bspline(double x) {
  const double a = fabs(x);
  if (a < 0.5) return 0.75 - a * a;
  if (a < 1.5) return 0.5 * (a - 1.5) * (a - 1.5);
  return 0.0;
}

// d_j(t_{k+1/2}) in GHz for every step (eq. dj-ctrl, without the 2 pi of H_c), written to
// dtab[k*q + j] (complex), and per block the partial sum of sum_j |d_j|^2.
__global__ __launch_bounds__(kThreads) void k_energy_table(DevSys s, const double *alpha, double *dtab,
                                                           double *partials) {
  __shared__ double sh[kThreads];
  const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
  double e = 0.0;
  if (k < s.NT) {
    const double t = (k + 0.5) * s.dt;
    const double x = t / s.dtau + 0.5;
    const int slo = max(0, (int)ceil(x - 1.5)), shi = min(s.d1 - 1, (int)floor(x + 1.5));
    for (int j = 0; j < s.q; ++j) {
      double dre = 0.0, dim = 0.0;
      for (int f = 0; f < s.nf; ++f) {
        double er = 0.0, ei = 0.0;
        const double *a = alpha + (size_t)(j * s.nf + f) * 2 * s.d1;
        for (int sp = slo; sp <= shi; ++sp) {
          const double b = bspline(x - sp);
          er += a[sp] * b;
          ei += a[s.d1 + sp] * b;
        }
        double sn, cs;
        sincos(s.carrier[j * s.nf + f] * t, &sn, &cs);
        dre += er * cs - ei * sn;
        dim += er * sn + ei * cs;
      }
      dtab[2 * (k * s.q + j)] = dre;
      dtab[2 * (k * s.q + j) + 1] = dim;
      e += dre * dre + dim * dim;
    }
  }
  const double b = block_reduce_sum(e, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// d Ee / d alpha for one coefficient (j, f, part, s) per block:
//   part 0: 2 dt sum_k B_s(t_k) Re(conj(d_j) e^{i W t_k}),  part 1: the same with i e^{i W t_k},
// over the steps in the support of B_s.
__global__ __launch_bounds__(kThreads) void k_energy_grad(DevSys s, const double *dtab, double *gE) {
  __shared__ double sh[kThreads];
  const int idx = blockIdx.x;                 // ((j*nf + f)*2 + part)*d1 + sp
  const int sp = idx % s.d1, part = (idx / s.d1) % 2, jf = idx / (2 * s.d1);
  const int j = jf / s.nf;
  const double om = s.carrier[jf];
  // B_s(t) > 0 for |t/dtau + 1/2 - sp| < 3/2
  const double tlo = (sp - 2.0) * s.dtau, thi = (sp + 1.0) * s.dtau;
  long long k0 = (long long)floor(tlo / s.dt - 0.5) - 1, k1 = (long long)ceil(thi / s.dt - 0.5) + 1;
  k0 = k0 < 0 ? 0 : k0;
  k1 = k1 > s.NT ? s.NT : k1;
  double acc = 0.0;
  for (long long k = k0 + threadIdx.x; k < k1; k += kThreads) {
    const double t = (k + 0.5) * s.dt;
    const double b = bspline(t / s.dtau + 0.5 - sp);
    if (b == 0.0) continue;
    double sn, cs;
    sincos(om * t, &sn, &cs);
    const double dre = dtab[2 * (k * s.q + j)], dim = dtab[2 * (k * s.q + j) + 1];
    acc += b * (part == 0 ? (dre * cs + dim * sn) : (dim * cs - dre * sn));
  }
  const double r = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) gE[idx] = 2.0 * s.dt * r;
}

int grid_for(long long n) {
  const long long g = (n + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > kOptGrid ? kOptGrid : g));
}

}  // namespace

int opt_dot(const double *a, const double *b, long long n, double *partials, double *out, hipStream_t st) {
  return opt_dot_to(a, b, n, partials, out, 1.0, nullptr, 0.0, st);
}

int opt_dot_to(const double *a, const double *b, long long n, double *partials, double *out, double cs,
               const double *base, double cb, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kOptGrid), dim3(kThreads), 0, st, a, b, n, partials);
  hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kThreads), 0, st, partials, kOptGrid, out, base, cb, cs);
  return (int)hipGetLastError();
}

int opt_maxabs(const double *v, long long n, double *partials, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_maxabs_partial, dim3(kOptGrid), dim3(kThreads), 0, st, v, n, partials);
  hipLaunchKernelGGL(k_finish<true>, dim3(1), dim3(kThreads), 0, st, partials, kOptGrid, out, (const double *)nullptr,
                     0.0, 1.0);
  return (int)hipGetLastError();
}

int opt_axpy_dev(double *y, const double *c, double s, const double *x, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_dev, dim3(grid_for(n)), dim3(kThreads), 0, st, y, c, s, x, n);
  return (int)hipGetLastError();
}

int opt_axpby(double *y, double a, const double *x, double b, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kThreads), 0, st, y, a, x, b, n);
  return (int)hipGetLastError();
}

int opt_trial(double *xt, const double *x, const double *p, double t, long long n, long long d, double lo, double hi,
              hipStream_t st) {
  hipLaunchKernelGGL(k_trial, dim3(grid_for(n)), dim3(kThreads), 0, st, xt, x, p, t, n, d, lo, hi);
  return (int)hipGetLastError();
}

int opt_reduced(double *out, const double *v, const double *x, const double *g, long long n, long long d, double lo,
                double hi, hipStream_t st) {
  hipLaunchKernelGGL(k_reduced, dim3(grid_for(n)), dim3(kThreads), 0, st, out, v, x, g, n, d, lo, hi);
  return (int)hipGetLastError();
}

int opt_assemble(double *g, const double *ga, const double *alpha, const double *gE, const double *gW, long long d,
                 long long nW, double gtik, double gen, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(d + nW)), dim3(kThreads), 0, st, g, ga, alpha, gE, gW, d, nW, gtik,
                     gen, s);
  return (int)hipGetLastError();
}

int opt_energy_blocks(const DevSys &s) { return (int)((s.NT + kThreads - 1) / kThreads); }

int opt_energy(const DevSys &s, const double *alpha, double *dtab, double *partials, double *out, hipStream_t st) {
  const int nb = opt_energy_blocks(s);
  hipLaunchKernelGGL(k_energy_table, dim3(nb), dim3(kThreads), 0, st, s, alpha, dtab, partials);
  hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kThreads), 0, st, partials, nb, out, (const double *)nullptr, 0.0,
                     1.0);
  return (int)hipGetLastError();
}

int opt_energy_grad(const DevSys &s, const double *dtab, double *gE, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_grad, dim3(s.q * s.nf * 2 * s.d1), dim3(kThreads), 0, st, s, dtab, gE);
  return (int)hipGetLastError();
}

}  // namespace qoc
