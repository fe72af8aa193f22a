/*
 * qoc_oracle.c -- plain, slow FP64 CPU oracle of the multiple-shooting
 * quadratic-penalty objective and its exact discrete-adjoint gradient
 * (arxiv 2407.13950).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this file.  It shares no
 * code, header, table or helper with the HIP library; the two meet only on the
 * seeded inputs.
 *
 * What is computed, in the paper's notation (n replaced by the number of
 * essential states E when guard levels are present: the target acts on the
 * E essential rows and the guard rows of V are zero):
 *   model      H(t) = H_d + H_J + H_c(t), H_c = sum_j d_j a_j + conj(d_j) a_j^+  (Sec. 2, eqs. sys-ham, ctrl-ham)
 *              with the diagonal drift H_d of the synthetic systems (detuning, anharmonicity, cross-Kerr)
 *              and the dipole coupling of the chain H_J = sum_j J_j (a_{j+1}^+ a_j + a_{j+1} a_j^+)
 *              (eq. sys-ham, nearest neighbours; zero for the synthetic systems).
 *   controls   d_j(t) = 2 pi sum_f exp(i Omega_jf t) sum_s (a1_jfs + i a2_jfs) B_s(t)   (Sec. 2, eq. dj-ctrl
 *              and the B-spline expansion below it); quadratic cardinal B-splines.
 *   windows    M windows, window m starts from W^{m-1} (W^0 = I)                     (Sec. 3, eqs. sch-op, sch-ic)
 *   stepping   implicit midpoint rule, H evaluated at the step midpoint              (Sec. 5, time integrator)
 *   objective  P = J_V(U^M) + mu/2 sum_{m<M} |U^m - W^m|_F^2                          (Sec. 3, eqs. mod-infid, penalty-fcn)
 *   gradient   discrete adjoint of the stepping ("discretize-then-optimize", Sec. 5), terminal
 *              conditions of eq. terminal, the alpha-gradient of eq. grad-int in its exact
 *              time-discrete form, and the W-gradient mu(W^m - U^m) - 2 Lambda^{m+1}(t_m)
 *              (App. B, eq. dT-dW-j combined with eq. dT-dW-j-1).
 *   roll-out   single-window propagation over [0, T] recording the window-boundary states
 *              (Sec. 3.2, roll-out state; Sec. 5, W initialisation).
 *
 * Every linear solve of the implicit midpoint rule is carried out to rounding
 * level by a fixed-point iteration with a convergence test (not a fixed count).
 *
 * Layouts (shared with the inputs module): complex arrays are interleaved
 * (re, im) doubles; a window state is a column-major N x E matrix; W holds
 * W^1..W^{M-1}; alpha index ((j*nf + f)*2 + part)*d1 + s.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ----------------------------------------------------------------------------- problem */

typedef struct {
    int q;                    /* qubits                                        */
    int L;                    /* levels per qubit                              */
    const double *detuning;   /* [q] rad/ns, coefficient of l_j                */
    const double *anharm;     /* [q] rad/ns, coefficient of l_j(l_j-1)/2       */
    const double *cross_kerr; /* [q-1] rad/ns, coefficient of l_j l_{j+1}      */
    int nf;                   /* carriers per qubit                            */
    const double *carrier;    /* [q*nf] rad/ns                                 */
    int d1;                   /* B-spline coefficients per carrier             */
    double T;                 /* gate duration, ns                             */
    long n_steps;             /* N_T                                           */
    int M;                    /* windows                                       */
    double mu;                /* penalty coefficient                           */
    const double *target;     /* [2*E*E] E x E target, column-major            */
    const double *dipole;     /* [q-1] rad/ns, J_j of qubits j, j+1; NULL = 0  */
} orc_problem;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENOTCONV = -4 };

typedef struct {
    const orc_problem *p;
    int N, E;
    double dt;
    int *digit;     /* [N*q]: level of qubit j (j = 0 is the most significant) in row r */
    long *stride;   /* [q]: L^(q-1-j)                                                  */
    double *h;      /* [N]: drift diagonal                                              */
    int *ess_row;   /* [E]: row of essential state e (all levels 0/1)                  */
    cplx *V;        /* [N*E]: target embedded in the essential rows, column-major      */
    int status;
} orc_sys;

static long ipow(long b, int e) { long r = 1; while (e-- > 0) r *= b; return r; }

static void sys_free(orc_sys *s)
{
    free(s->digit); free(s->stride); free(s->h); free(s->ess_row); free(s->V);
}

/* Tensor-product basis: row r = sum_j l_j L^(q-1-j), qubit 0 most significant.
 * Essential state e (binary digits b_j, qubit 0 most significant) sits at the row
 * with l_j = b_j. */
static int sys_init(orc_sys *s, const orc_problem *p)
{
    memset(s, 0, sizeof *s);
    if (p->q < 1 || p->L < 2 || p->nf < 1 || p->d1 < 3 || p->n_steps < 1 || p->M < 1 ||
        p->M > p->n_steps || !(p->T > 0.0))
        return ORC_EINVAL;
    s->p = p;
    s->N = (int)ipow(p->L, p->q);
    s->E = (int)ipow(2, p->q);
    s->dt = p->T / (double)p->n_steps;
    s->digit = malloc(sizeof(int) * (size_t)s->N * p->q);
    s->stride = malloc(sizeof(long) * p->q);
    s->h = malloc(sizeof(double) * s->N);
    s->ess_row = malloc(sizeof(int) * s->E);
    s->V = calloc((size_t)s->N * s->E, sizeof(cplx));
    if (!s->digit || !s->stride || !s->h || !s->ess_row || !s->V) { sys_free(s); return ORC_ENOMEM; }
    for (int j = 0; j < p->q; ++j) s->stride[j] = ipow(p->L, p->q - 1 - j);
    for (int r = 0; r < s->N; ++r)
        for (int j = 0; j < p->q; ++j) s->digit[r * p->q + j] = (int)((r / s->stride[j]) % p->L);
    /* drift: sum_j [delta_j l_j + xi_j/2 l_j (l_j - 1)] + sum_j chi_j l_j l_{j+1} */
    for (int r = 0; r < s->N; ++r) {
        const int *l = s->digit + r * p->q;
        double v = 0.0;
        for (int j = 0; j < p->q; ++j)
            v += p->detuning[j] * l[j] + 0.5 * p->anharm[j] * l[j] * (l[j] - 1);
        for (int j = 0; j + 1 < p->q; ++j)
            v += (p->cross_kerr ? p->cross_kerr[j] : 0.0) * l[j] * l[j + 1];
        s->h[r] = v;
    }
    for (int e = 0; e < s->E; ++e) {
        long r = 0;
        for (int j = 0; j < p->q; ++j) r += (long)((e >> (p->q - 1 - j)) & 1) * s->stride[j];
        s->ess_row[e] = (int)r;
    }
    for (int c = 0; c < s->E; ++c)
        for (int e = 0; e < s->E; ++e)
            s->V[(size_t)c * s->N + s->ess_row[e]] =
                p->target[2 * (c * s->E + e)] + I * p->target[2 * (c * s->E + e) + 1];
    return ORC_OK;
}

/* ----------------------------------------------------------------------------- controls */

/* Quadratic cardinal B-spline with unit knot spacing, centred at 0, support (-3/2, 3/2). */
static double bspline2(double x)
{
    double a = fabs(x);
    if (a < 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (a - 1.5) * (a - 1.5);
    return 0.0;
}

/* B_s(t) = B((t - c_s)/dtau), centres c_s = (s - 1/2) dtau, dtau = T/(d1 - 2). */
static double spline_value(const orc_problem *p, int s, double t)
{
    double dtau = p->T / (double)(p->d1 - 2);
    return bspline2((t - (s - 0.5) * dtau) / dtau);
}

static int alpha_index(const orc_problem *p, int j, int f, int part, int s)
{
    return ((j * p->nf + f) * 2 + part) * p->d1 + s;
}

/* c_j(t) = 2 pi d_j(t): the coefficient of a_j in H_c; conj(c_j) multiplies a_j^+. */
static void controls(const orc_problem *p, const double *alpha, double t, cplx *c)
{
    for (int j = 0; j < p->q; ++j) {
        cplx d = 0.0;
        for (int f = 0; f < p->nf; ++f) {
            cplx env = 0.0;
            for (int s = 0; s < p->d1; ++s) {
                double b = spline_value(p, s, t);
                if (b == 0.0) continue;
                env += (alpha[alpha_index(p, j, f, 0, s)] + I * alpha[alpha_index(p, j, f, 1, s)]) * b;
            }
            d += env * cexp(I * p->carrier[j * p->nf + f] * t);
        }
        c[j] = 2.0 * M_PI * d;
    }
}

/* ----------------------------------------------------------------------------- operators */

/* out = (H_c + H_J) x, the off-diagonal part of H, with
 *   (a_j x)_r = sqrt(l_j+1) x_{r+stride_j},  (a_j^+ x)_r = sqrt(l_j) x_{r-stride_j},
 *   (a_{j+1}^+ a_j x)_r = sqrt(l_{j+1}) sqrt(l_j+1) x_{r+stride_j-stride_{j+1}},
 *   (a_{j+1} a_j^+ x)_r = sqrt(l_{j+1}+1) sqrt(l_j) x_{r-stride_j+stride_{j+1}}. */
static void apply_Hc(const orc_sys *s, const cplx *c, const cplx *x, cplx *out)
{
    const int q = s->p->q, L = s->p->L;
    for (int r = 0; r < s->N; ++r) {
        cplx acc = 0.0;
        for (int j = 0; j < q; ++j) {
            int l = s->digit[r * q + j];
            if (l < L - 1) acc += c[j] * sqrt((double)(l + 1)) * x[r + s->stride[j]];
            if (l > 0) acc += conj(c[j]) * sqrt((double)l) * x[r - s->stride[j]];
        }
        if (s->p->dipole)
            for (int j = 0; j + 1 < q; ++j) {
                const int la = s->digit[r * q + j], lb = s->digit[r * q + j + 1];
                const double J = s->p->dipole[j];
                if (la < L - 1 && lb > 0)
                    acc += J * sqrt((double)(la + 1)) * sqrt((double)lb) * x[r + s->stride[j] - s->stride[j + 1]];
                if (la > 0 && lb < L - 1)
                    acc += J * sqrt((double)la) * sqrt((double)(lb + 1)) * x[r - s->stride[j] + s->stride[j + 1]];
            }
        out[r] = acc;
    }
}

/* Solve (I + sgn i dt/2 H) z = rhs for one column, H = diag(h) + H_c + H_J, by the
 * fixed point z <- D^{-1}(rhs - sgn i dt/2 (H_c + H_J) z), D = I + sgn i dt/2 diag(h),
 * iterated until the update is at rounding level.  work: N scratch entries. */
static int imr_solve(const orc_sys *s, const cplx *c, int sgn, const cplx *rhs, cplx *z, cplx *work)
{
    const double hdt = 0.5 * s->dt;
    for (int r = 0; r < s->N; ++r) z[r] = rhs[r] / (1.0 + sgn * I * hdt * s->h[r]);
    for (int it = 0; it < 200; ++it) {
        apply_Hc(s, c, z, work);
        double dmax = 0.0, zmax = 0.0;
        for (int r = 0; r < s->N; ++r) {
            cplx zn = (rhs[r] - sgn * I * hdt * work[r]) / (1.0 + sgn * I * hdt * s->h[r]);
            double dz = cabs(zn - z[r]), az = cabs(zn);
            if (dz > dmax) dmax = dz;
            if (az > zmax) zmax = az;
            z[r] = zn;
        }
        if (dmax <= 1e-15 * zmax) return ORC_OK;
    }
    return ORC_ENOTCONV;
}

/* One implicit-midpoint step of one column from step k (time k dt) to k+1:
 * (I + i dt/2 H_k) u_{k+1} = (I - i dt/2 H_k) u_k, written as z = (I + i dt/2 H_k)^{-1} u_k,
 * u_{k+1} = 2 z - u_k.  sgn = -1 gives the reverse step u_{k+1} -> u_k. */
static int imr_step(const orc_sys *s, const double *alpha, long k, int sgn, cplx *u, cplx *z, cplx *work)
{
    cplx c[64];
    controls(s->p, alpha, (k + 0.5) * s->dt, c);
    int rc = imr_solve(s, c, sgn, u, z, work);
    for (int r = 0; r < s->N; ++r) u[r] = 2.0 * z[r] - u[r];
    return rc;
}

/* First step of window m (1-based): floor((m-1) N_T / M). */
static long window_start(const orc_problem *p, int m) { return (long)(((long long)(m - 1) * p->n_steps) / p->M); }

/* Column c of the initial state of window m: W^0 = I (embedded), else W^{m-1}. */
static void initial_column(const orc_sys *s, const double *W, int m, int c, cplx *u)
{
    if (m == 1) {
        for (int r = 0; r < s->N; ++r) u[r] = 0.0;
        u[s->ess_row[c]] = 1.0;
    } else {
        const double *w = W + 2 * ((size_t)(m - 2) * s->E + c) * s->N;
        for (int r = 0; r < s->N; ++r) u[r] = w[2 * r] + I * w[2 * r + 1];
    }
}

static cplx w_entry(const orc_sys *s, const double *W, int m, int c, int r)
{
    const double *w = W + 2 * (((size_t)(m - 1) * s->E + c) * s->N + r);
    return w[0] + I * w[1];
}

/* ----------------------------------------------------------------------------- evaluation */

typedef struct {
    /* outputs of the forward phase */
    cplx *Ufin;          /* [M][E][N]: U^m(t_m), column-major per window              */
    double *pen;         /* [M]: |U^m - W^m|_F^2 for m < M                            */
    double normU2;       /* |U^M|_F^2                                                 */
    cplx gamma;          /* <V, U^M>_F                                                */
} fwd_out;

/* Forward phase over windows m0..m1 (1-based, inclusive): every (window, column) pair
 * is independent once W is given, as in the paper's 2-D process grid (Sec. 4). */
static int forward_phase(const orc_sys *s, const double *alpha, const double *W, int m0, int m1, fwd_out *o)
{
    const orc_problem *p = s->p;
    const int N = s->N, E = s->E;
    int status = ORC_OK;
    int ntask = (m1 - m0 + 1) * E;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
    for (int t = 0; t < ntask; ++t) {
        int m = m0 + t / E, c = t % E;
        cplx *u = malloc(sizeof(cplx) * 3 * N);
        if (!u) { status = ORC_ENOMEM; continue; }
        cplx *z = u + N, *work = u + 2 * N;
        initial_column(s, W, m, c, u);
        for (long k = window_start(p, m); k < window_start(p, m + 1); ++k)
            if (imr_step(s, alpha, k, +1, u, z, work) != ORC_OK) status = ORC_ENOTCONV;
        memcpy(o->Ufin + ((size_t)(m - 1) * E + c) * N, u, sizeof(cplx) * N);
        free(u);
    }
    if (status != ORC_OK) return status;
    /* reductions in a fixed order */
    for (int m = m0; m <= m1 && m < p->M; ++m) {
        double acc = 0.0;
        for (int c = 0; c < E; ++c)
            for (int r = 0; r < N; ++r) {
                cplx dlt = o->Ufin[((size_t)(m - 1) * E + c) * N + r] - w_entry(s, W, m, c, r);
                acc += creal(dlt) * creal(dlt) + cimag(dlt) * cimag(dlt);
            }
        o->pen[m - 1] = acc;
    }
    if (m1 == p->M) {
        double nrm = 0.0;
        cplx g = 0.0;
        const cplx *UM = o->Ufin + (size_t)(p->M - 1) * E * N;
        for (int c = 0; c < E; ++c)
            for (int r = 0; r < N; ++r) {
                cplx u = UM[(size_t)c * N + r];
                nrm += creal(u) * creal(u) + cimag(u) * cimag(u);
                g += conj(s->V[(size_t)c * N + r]) * u;
            }
        o->normU2 = nrm;
        o->gamma = g;
    }
    return ORC_OK;
}

/* terms: [J, penalty, |U^M|^2, Re gamma, Im gamma, |C^1|^2 .. |C^{M-1}|^2] */
static double assemble_objective(const orc_sys *s, const fwd_out *o, double *terms)
{
    const orc_problem *p = s->p;
    const double E = (double)s->E;
    double J = o->normU2 / E - (creal(o->gamma) * creal(o->gamma) + cimag(o->gamma) * cimag(o->gamma)) / (E * E);
    double pen = 0.0;
    for (int m = 1; m < p->M; ++m) pen += o->pen[m - 1];
    pen *= 0.5 * p->mu;
    if (terms) {
        terms[0] = J; terms[1] = pen; terms[2] = o->normU2;
        terms[3] = creal(o->gamma); terms[4] = cimag(o->gamma);
        for (int m = 1; m < p->M; ++m) terms[4 + m] = o->pen[m - 1];
    }
    return J + pen;
}

/* Terminal condition of window m (eq. terminal): mu/2 (W^m - U^m) for m < M,
 * (gamma V - E U^M)/E^2 for m = M. */
static void terminal_column(const orc_sys *s, const double *W, const fwd_out *o, int m, int c, cplx *lam)
{
    const orc_problem *p = s->p;
    const int N = s->N;
    const cplx *U = o->Ufin + ((size_t)(m - 1) * s->E + c) * N;
    const double E = (double)s->E;
    for (int r = 0; r < N; ++r) {
        if (m < p->M) lam[r] = 0.5 * p->mu * (w_entry(s, W, m, c, r) - U[r]);
        else lam[r] = (o->gamma * s->V[(size_t)c * N + r] - E * U[r]) / (E * E);
    }
}

/* Adjoint phase for windows m0..m1.  Per (window, column): recompute and store the
 * forward trajectory, then step the adjoint backwards,
 *   y_k = (I - i dt/2 H_k)^{-1} Lambda_{k+1},  Lambda_k = 2 y_k - Lambda_{k+1},
 * and accumulate dP/dalpha = sum_k 2 dt Re <y_k, i dH_k/dalpha z_k>, z_k = (u_k + u_{k+1})/2,
 * with dH/d(Re d_j) = 2 pi (a_j + a_j^+), dH/d(Im d_j) = 2 pi i (a_j - a_j^+).
 * lam0: [M][E][N] receives Lambda^m(t_{m-1}); ga_task: [ntask][d] per-task alpha gradients. */
static int adjoint_phase(const orc_sys *s, const double *alpha, const double *W, int m0, int m1,
                         const fwd_out *o, cplx *lam0, double *ga_task)
{
    const orc_problem *p = s->p;
    const int N = s->N, E = s->E, q = p->q, L = p->L;
    const int d = 2 * p->d1 * p->q * p->nf;
    int status = ORC_OK;
    int ntask = (m1 - m0 + 1) * E;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
    for (int t = 0; t < ntask; ++t) {
        int m = m0 + t / E, c = t % E;
        long k0 = window_start(p, m), k1 = window_start(p, m + 1), nk = k1 - k0;
        double *ga = ga_task + (size_t)t * d;
        cplx *traj = malloc(sizeof(cplx) * (size_t)(nk + 1) * N);
        cplx *buf = malloc(sizeof(cplx) * 6 * N);
        if (!traj || !buf) { free(traj); free(buf); status = ORC_ENOMEM; continue; }
        cplx *lam = buf, *y = buf + N, *work = buf + 2 * N, *z = buf + 3 * N, *v1 = buf + 4 * N, *v2 = buf + 5 * N;
        memset(ga, 0, sizeof(double) * d);
        initial_column(s, W, m, c, traj);
        for (long k = k0; k < k1; ++k) {
            cplx *un = traj + (size_t)(k - k0 + 1) * N;
            memcpy(un, traj + (size_t)(k - k0) * N, sizeof(cplx) * N);
            if (imr_step(s, alpha, k, +1, un, z, work) != ORC_OK) status = ORC_ENOTCONV;
        }
        terminal_column(s, W, o, m, c, lam);
        for (long k = k1 - 1; k >= k0; --k) {
            double tk = (k + 0.5) * s->dt;
            cplx cc[64];
            controls(p, alpha, tk, cc);
            if (imr_solve(s, cc, -1, lam, y, work) != ORC_OK) status = ORC_ENOTCONV;
            const cplx *ua = traj + (size_t)(k - k0) * N, *ub = ua + N;
            for (int r = 0; r < N; ++r) z[r] = 0.5 * (ua[r] + ub[r]);
            for (int j = 0; j < q; ++j) {
                /* v1 = (a_j + a_j^+) z,  v2 = i (a_j - a_j^+) z */
                for (int r = 0; r < N; ++r) {
                    int l = s->digit[r * q + j];
                    cplx lo = (l < L - 1) ? sqrt((double)(l + 1)) * z[r + s->stride[j]] : 0.0;
                    cplx hi = (l > 0) ? sqrt((double)l) * z[r - s->stride[j]] : 0.0;
                    v1[r] = lo + hi;
                    v2[r] = I * (lo - hi);
                }
                cplx ip1 = 0.0, ip2 = 0.0;
                for (int r = 0; r < N; ++r) { ip1 += conj(y[r]) * I * v1[r]; ip2 += conj(y[r]) * I * v2[r]; }
                double X = 2.0 * s->dt * 2.0 * M_PI * creal(ip1);   /* d/d(Re d_j) */
                double Y = 2.0 * s->dt * 2.0 * M_PI * creal(ip2);   /* d/d(Im d_j) */
                for (int f = 0; f < p->nf; ++f) {
                    double om = p->carrier[j * p->nf + f];
                    double cs = cos(om * tk), sn = sin(om * tk);
                    for (int sidx = 0; sidx < p->d1; ++sidx) {
                        double b = spline_value(p, sidx, tk);
                        if (b == 0.0) continue;
                        /* Re d = sum b (a1 cos - a2 sin), Im d = sum b (a1 sin + a2 cos) */
                        ga[alpha_index(p, j, f, 0, sidx)] += b * (cs * X + sn * Y);
                        ga[alpha_index(p, j, f, 1, sidx)] += b * (-sn * X + cs * Y);
                    }
                }
            }
            for (int r = 0; r < N; ++r) lam[r] = 2.0 * y[r] - lam[r];
        }
        memcpy(lam0 + ((size_t)(m - 1) * E + c) * N, lam, sizeof(cplx) * N);
        free(traj); free(buf);
    }
    return status;
}

/* ----------------------------------------------------------------------------- C entry points */

static int alloc_fwd(const orc_sys *s, fwd_out *o)
{
    memset(o, 0, sizeof *o);
    o->Ufin = calloc((size_t)s->p->M * s->E * s->N, sizeof(cplx));
    o->pen = calloc((size_t)s->p->M, sizeof(double));
    return (o->Ufin && o->pen) ? ORC_OK : ORC_ENOMEM;
}

static void free_fwd(fwd_out *o) { free(o->Ufin); free(o->pen); }

int orc_objective(const orc_problem *p, const double *alpha, const double *W, double *P, double *terms)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    fwd_out o;
    rc = alloc_fwd(&s, &o);
    if (!rc) rc = forward_phase(&s, alpha, W, 1, p->M, &o);
    if (!rc) *P = assemble_objective(&s, &o, terms);
    free_fwd(&o);
    sys_free(&s);
    return rc;
}

/* grad_W has the layout of W: slot re = dP/dRe W, slot im = dP/dIm W. */
int orc_gradient(const orc_problem *p, const double *alpha, const double *W, double *P, double *terms,
                 double *grad_alpha, double *grad_W)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    const int N = s.N, E = s.E, M = p->M;
    const int d = 2 * p->d1 * p->q * p->nf;
    fwd_out o;
    cplx *lam0 = calloc((size_t)M * E * N, sizeof(cplx));
    double *ga_task = calloc((size_t)M * E * d, sizeof(double));
    rc = alloc_fwd(&s, &o);
    if (!rc && (!lam0 || !ga_task)) rc = ORC_ENOMEM;
    if (!rc) rc = forward_phase(&s, alpha, W, 1, M, &o);
    if (!rc) *P = assemble_objective(&s, &o, terms);
    if (!rc) rc = adjoint_phase(&s, alpha, W, 1, M, &o, lam0, ga_task);
    if (!rc) {
        for (int i = 0; i < d; ++i) {
            double acc = 0.0;
            for (int t = 0; t < M * E; ++t) acc += ga_task[(size_t)t * d + i];
            grad_alpha[i] = acc;
        }
        for (int m = 1; m < M; ++m)
            for (int c = 0; c < E; ++c)
                for (int r = 0; r < N; ++r) {
                    cplx g = p->mu * (w_entry(&s, W, m, c, r) - o.Ufin[((size_t)(m - 1) * E + c) * N + r])
                           - 2.0 * lam0[((size_t)m * E + c) * N + r];
                    double *dst = grad_W + 2 * (((size_t)(m - 1) * E + c) * N + r);
                    dst[0] = creal(g);
                    dst[1] = cimag(g);
                }
    }
    free_fwd(&o); free(lam0); free(ga_task);
    sys_free(&s);
    return rc;
}

/* Per-window pieces for windows m0..m1 (bounded samples and sampled checks):
 * Ufin_out [(m1-m0+1)][E][N] complex: U^m(t_m); pen_out [m1-m0+1]: |U^m - W^m|^2 (0 for m = M);
 * lam0_out [(m1-m0+1)][E][N]: Lambda^m(t_{m-1}) (NULL: skip the adjoint);
 * ga_out [d]: the windows' contribution to dP/dalpha.  Window M's terminal condition needs
 * gamma, so a sample that contains m = M computes it from U^M. */
int orc_windows(const orc_problem *p, const double *alpha, const double *W, int m0, int m1,
                double *Ufin_out, double *pen_out, double *lam0_out, double *ga_out)
{
    orc_sys s;
    if (m0 < 1 || m1 > p->M || m0 > m1) return ORC_EINVAL;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    const int N = s.N, E = s.E, M = p->M;
    const int d = 2 * p->d1 * p->q * p->nf;
    int nw = m1 - m0 + 1;
    fwd_out o;
    cplx *lam0 = calloc((size_t)M * E * N, sizeof(cplx));
    double *ga_task = lam0_out ? calloc((size_t)nw * E * d, sizeof(double)) : NULL;
    rc = alloc_fwd(&s, &o);
    if (!rc && (!lam0 || (lam0_out && !ga_task))) rc = ORC_ENOMEM;
    if (!rc) rc = forward_phase(&s, alpha, W, m0, m1, &o);
    if (!rc && lam0_out) rc = adjoint_phase(&s, alpha, W, m0, m1, &o, lam0, ga_task);
    if (!rc) {
        for (int i = 0; i < nw; ++i) {
            int m = m0 + i;
            memcpy(Ufin_out + 2 * (size_t)i * E * N, o.Ufin + (size_t)(m - 1) * E * N, sizeof(cplx) * E * N);
            pen_out[i] = (m < M) ? o.pen[m - 1] : 0.0;
            if (lam0_out)
                memcpy(lam0_out + 2 * (size_t)i * E * N, lam0 + (size_t)(m - 1) * E * N, sizeof(cplx) * E * N);
        }
        if (lam0_out)
            for (int k = 0; k < d; ++k) {
                double acc = 0.0;
                for (int t = 0; t < nw * E; ++t) acc += ga_task[(size_t)t * d + k];
                ga_out[k] = acc;
            }
    }
    free_fwd(&o); free(lam0); free(ga_task);
    sys_free(&s);
    return rc;
}

/* Roll-out: one window over [0, T] from W^0 = I; W_out [(M-1)][E][N] receives the states at
 * the window boundaries t_1..t_{M-1}; U_out [E][N] the final state. */
int orc_rollout(const orc_problem *p, const double *alpha, double *W_out, double *U_out)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    const int N = s.N, E = s.E, M = p->M;
    int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
    for (int c = 0; c < E; ++c) {
        cplx *u = malloc(sizeof(cplx) * 3 * N);
        if (!u) { status = ORC_ENOMEM; continue; }
        cplx *z = u + N, *work = u + 2 * N;
        initial_column(&s, NULL, 1, c, u);
        int m = 1;
        for (long k = 0; k < p->n_steps; ++k) {
            if (imr_step(&s, alpha, k, +1, u, z, work) != ORC_OK) status = ORC_ENOTCONV;
            if (m < M && k + 1 == window_start(p, m + 1)) {
                memcpy(W_out + 2 * (((size_t)(m - 1) * E + c) * N), u, sizeof(cplx) * N);
                ++m;
            }
        }
        if (U_out) memcpy(U_out + 2 * (size_t)c * N, u, sizeof(cplx) * N);
        free(u);
    }
    sys_free(&s);
    return status;
}

/* ----------------------------------------------------------------------------- pieces for the pins */

int orc_drift(const orc_problem *p, double *h_out)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    memcpy(h_out, s.h, sizeof(double) * s.N);
    sys_free(&s);
    return ORC_OK;
}

int orc_essential_rows(const orc_problem *p, int *rows)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    memcpy(rows, s.ess_row, sizeof(int) * s.E);
    sys_free(&s);
    return ORC_OK;
}

/* c_out [2q]: c_j(t) = 2 pi d_j(t), interleaved. */
int orc_controls(const orc_problem *p, const double *alpha, double t, double *c_out)
{
    cplx c[64];
    if (p->q > 64) return ORC_EINVAL;
    controls(p, alpha, t, c);
    memcpy(c_out, c, sizeof(cplx) * p->q);
    return ORC_OK;
}

int orc_spline_values(const orc_problem *p, double t, double *out)
{
    for (int s = 0; s < p->d1; ++s) out[s] = spline_value(p, s, t);
    return ORC_OK;
}

/* out = H(t) x for ncol columns of length N (interleaved complex). */
int orc_apply_H(const orc_problem *p, const double *alpha, double t, int ncol, const double *x, double *out)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    cplx c[64];
    controls(p, alpha, t, c);
    for (int k = 0; k < ncol; ++k) {
        const cplx *xc = (const cplx *)(x + 2 * (size_t)k * s.N);
        cplx *oc = (cplx *)(out + 2 * (size_t)k * s.N);
        apply_Hc(&s, c, xc, oc);
        for (int r = 0; r < s.N; ++r) oc[r] += s.h[r] * xc[r];
    }
    sys_free(&s);
    return ORC_OK;
}

/* Propagate ncol columns u (interleaved, N each) over steps k0..k1-1 (sgn = +1), or backwards
 * from k1 to k0 (sgn = -1, reverse steps k1-1 .. k0). */
int orc_propagate(const orc_problem *p, const double *alpha, long k0, long k1, int sgn, int ncol, double *u)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    cplx *z = malloc(sizeof(cplx) * 2 * s.N);
    if (!z) { sys_free(&s); return ORC_ENOMEM; }
    for (int k = 0; k < ncol && rc == ORC_OK; ++k) {
        cplx *uc = (cplx *)(u + 2 * (size_t)k * s.N);
        if (sgn > 0) {
            for (long st = k0; st < k1 && rc == ORC_OK; ++st) rc = imr_step(&s, alpha, st, +1, uc, z, z + s.N);
        } else {
            for (long st = k1 - 1; st >= k0 && rc == ORC_OK; --st) rc = imr_step(&s, alpha, st, -1, uc, z, z + s.N);
        }
    }
    free(z);
    sys_free(&s);
    return rc;
}

/* Generalised infidelity J_V(U) = |U|_F^2/E - |<V,U>_F|^2/E^2 of an N x E matrix (eq. mod-infid). */
int orc_infidelity(const orc_problem *p, const double *U, double *J)
{
    orc_sys s;
    int rc = sys_init(&s, p);
    if (rc) return rc;
    double nrm = 0.0;
    cplx g = 0.0;
    for (int c = 0; c < s.E; ++c)
        for (int r = 0; r < s.N; ++r) {
            cplx u = U[2 * ((size_t)c * s.N + r)] + I * U[2 * ((size_t)c * s.N + r) + 1];
            nrm += creal(u) * creal(u) + cimag(u) * cimag(u);
            g += conj(s.V[(size_t)c * s.N + r]) * u;
        }
    *J = nrm / s.E - (creal(g) * creal(g) + cimag(g) * cimag(g)) / ((double)s.E * s.E);
    sys_free(&s);
    return ORC_OK;
}

int orc_window_starts(const orc_problem *p, long *starts)
{
    for (int m = 1; m <= p->M + 1; ++m) starts[m - 1] = window_start(p, m);
    return ORC_OK;
}

/* Control energy of the optimisation settings (Sec. 5, energy penalty integral):
 *   Ee(alpha) = dt sum_{k=0}^{N_T-1} sum_j |d_j(t_{k+1/2})|^2,   d_j = c_j / (2 pi) in GHz,
 * the midpoint rule on the propagation grid, and its exact gradient
 *   dEe/dalpha_l = 2 dt sum_k sum_j Re(conj(d_j) dd_j/dalpha_l),
 * dd_j/da1_jfs = B_s(t) e^{i W_jf t}, dd_j/da2_jfs = i B_s(t) e^{i W_jf t}.  grad may be NULL. */
int orc_energy(const orc_problem *p, const double *alpha, double *E_out, double *grad)
{
    const double dt = p->T / (double)p->n_steps;
    const int d = p->q * p->nf * 2 * p->d1;
    cplx c[64];
    if (p->q > 64) return ORC_EINVAL;
    if (grad) memset(grad, 0, sizeof(double) * d);
    double E = 0.0;
    for (long k = 0; k < p->n_steps; ++k) {
        const double t = (k + 0.5) * dt;
        controls(p, alpha, t, c);
        for (int j = 0; j < p->q; ++j) {
            const cplx dj = c[j] / (2.0 * M_PI);
            E += creal(dj) * creal(dj) + cimag(dj) * cimag(dj);
            if (!grad) continue;
            for (int f = 0; f < p->nf; ++f) {
                const double om = p->carrier[j * p->nf + f];
                const cplx ph = cexp(I * om * t);
                for (int s = 0; s < p->d1; ++s) {
                    const double b = spline_value(p, s, t);
                    if (b == 0.0) continue;
                    grad[alpha_index(p, j, f, 0, s)] += 2.0 * dt * creal(conj(dj) * b * ph);
                    grad[alpha_index(p, j, f, 1, s)] += 2.0 * dt * creal(conj(dj) * I * b * ph);
                }
            }
        }
    }
    *E_out = dt * E;
    return ORC_OK;
}

/* Threads the parallel loops over (window, column) tasks use (1 without OpenMP). */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
