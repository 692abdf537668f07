/*
 * loc_oracle.c -- FP64 CPU oracle of the LOC ray march (TEST INFRASTRUCTURE ONLY).
 *
 * This is the plain, slow reference that the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark compare the HIP library against.  The product
 * path never calls it.  It shares no code, header, table or constant with the HIP
 * implementation; its only common ground with it is the seeded input generator.
 *
 * What it computes (Juvela 2020, "LOC program for line radiative transfer"):
 *
 *   Sect. 2, Eq. (3): over a ray step of length s through a cell of constant
 *   properties the photons in channel c are attenuated by exp(-tau_c) and the
 *   cell adds its own emission.  In intensity form
 *        I_out = I_in e^{-tau} + S (1 - e^{-tau}),   S = eta / kappa,
 *   written here as I_out = I_in e^{-tau} + eta p s beta with
 *   beta = (1 - e^{-tau})/tau, which stays finite where kappa -> 0.
 *
 *   Sect. 2, Eq. (2): the absorptions counted along the step are the path
 *   average of the intensity, I_in beta + S (1 - beta).  The ALI variant of
 *   Sect. 2 drops the locally emitted part and instead scales A_ul by the
 *   escape probability; what the march must deliver for that is
 *        J_k   += (a s / W_k) sum_c f_c I_in,c beta_c        (external field)
 *        Lam_k += (a s / W_k) sum_c f_c (1 - beta_c)         (diagonal operator)
 *   with f_c the fraction of the line emitted into channel c (Sect. 2: phi is
 *   replaced by the per-channel fraction) and each ray's share proportional to
 *   a s (Sect. 2: emission shared in proportion to path length, total known).
 *   This file returns the raw sums (before the 1/W_k); the Python side divides.
 *
 *   Sect. 2.1: 1D models are nested shells crossed by rays of given impact
 *   parameter; the Doppler shift is evaluated at the start of each step
 *   (Sect. 3.1).
 *
 *   Sect. 2.2: 3D rays follow the HEALPix directions; the main axis is the
 *   largest |component|; one ray starts per upstream surface element; a ray
 *   leaving through a side re-enters on the opposite side at the same
 *   main-axis coordinate and the work ends at the downstream border.
 *
 * Conventions shared with the inputs (not with the HIP code):
 *   channel centres v_c = vmin + (c + 1/2) dv;
 *   line profile p_c = exp(-((v_c + w)/b)^2) / (b sqrt(pi))  [s/cm], w = u.d
 *   (the gas velocity projected on the propagation direction; the line of gas
 *   moving towards the observer appears at negative channel velocity);
 *   f_c = p_c dv;  tau_c = kappa p_c s.
 *   3D cell (x,y,z) of an N^3 grid is stored at index (z N + y) N + x.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* beta = (1 - e^{-tau})/tau and 1 - beta, both accurate also for tiny |tau|. */
static void escape_terms(double tau, double* e, double* beta, double* omb)
{
    *e = exp(-tau);
    if (fabs(tau) < 1.0e-4) {
        /* Taylor series of (1 - e^{-tau})/tau: 1 - tau/2 + tau^2/6 - tau^3/24 + ... */
        *omb = tau * (0.5 - tau * (1.0 / 6.0 - tau * (1.0 / 24.0 - tau / 120.0)));
        *beta = 1.0 - *omb;
    } else {
        *beta = -expm1(-tau) / tau;
        *omb = 1.0 - *beta;
    }
}

/* One ray step through one cell for all channels.  Returns the raw per-step
 * sums sum_c f_c I_c beta_c, sum_c f_c (1-beta_c) and sum_c f_c through the
 * pointers (not multiplied by a s). */
static void cell_step(int nch, double vmin, double dv, double* I,
                      double kappa, double eta, double b, double w, double s,
                      double* sj, double* sl, double* se)
{
    double js = 0.0, ls = 0.0, es = 0.0;
    const double norm = 1.0 / (b * sqrt(M_PI));
    for (int c = 0; c < nch; ++c) {
        double v = vmin + (c + 0.5) * dv;
        double x = (v + w) / b;
        double p = exp(-x * x) * norm;
        double f = p * dv;
        double tau = kappa * p * s;
        double e, beta, omb;
        escape_terms(tau, &e, &beta, &omb);
        js += f * I[c] * beta;
        ls += f * omb;
        es += f;
        I[c] = I[c] * e + eta * p * s * beta;
    }
    *sj = js;
    *sl = ls;
    *se = es;
}

/* Per-thread accumulators, reduced in thread order at the end (deterministic
 * for a given thread count). */
typedef struct {
    double *J, *L, *W, *E;
    double cons;
} accum_t;

/* Number of threads the marches use when asked for 0 (all available). */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int nthreads_of(int req)
{
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

static accum_t* accum_alloc(int nt, long ncell)
{
    accum_t* a = (accum_t*)calloc((size_t)nt, sizeof(accum_t));
    for (int t = 0; t < nt; ++t) {
        a[t].J = (double*)calloc((size_t)ncell, sizeof(double));
        a[t].L = (double*)calloc((size_t)ncell, sizeof(double));
        a[t].W = (double*)calloc((size_t)ncell, sizeof(double));
        a[t].E = (double*)calloc((size_t)ncell, sizeof(double));
    }
    return a;
}

static void accum_reduce_free(accum_t* a, int nt, long ncell, double* J, double* L,
                              double* W, double* E, double* cons)
{
    for (long k = 0; k < ncell; ++k) {
        double j = 0, l = 0, w = 0, e = 0;
        for (int t = 0; t < nt; ++t) {
            j += a[t].J[k];
            l += a[t].L[k];
            w += a[t].W[k];
            e += a[t].E[k];
        }
        if (J) J[k] = j;
        if (L) L[k] = l;
        if (W) W[k] = w;
        if (E) E[k] = e;
    }
    double cs = 0;
    for (int t = 0; t < nt; ++t) cs += a[t].cons;
    if (cons) *cons = cs;
    for (int t = 0; t < nt; ++t) {
        free(a[t].J);
        free(a[t].L);
        free(a[t].W);
        free(a[t].E);
    }
    free(a);
}

/* ========================================================================= */
/* 1D shells (Sect. 2.1)                                                      */
/* ========================================================================= */

/* Steps of a ray with impact parameter b through shells with outer radii
 * R[0] < ... < R[n-1] (shell k spans (R[k-1], R[k]], R[-1] = 0).  The ray
 * enters at R[n-1], goes inwards to the innermost shell it reaches (the first
 * k with R[k] > b), whose chord is split at the tangent point into two halves,
 * and goes back out.  mu is the cosine between the propagation direction and
 * the outward radial direction at the start of each step.  Returns the number
 * of steps (at most 2n). */
int orc1d_ray_steps(int n, const double* R, double b, int* shell, double* s, double* mu)
{
    int kmin = 0;
    while (kmin < n && !(R[kmin] > b)) ++kmin;
    if (kmin >= n) return 0;
    int ns = 0;
    for (int k = n - 1; k > kmin; --k) {
        double zo = sqrt(R[k] * R[k] - b * b);
        double zi = sqrt(R[k - 1] * R[k - 1] - b * b);
        shell[ns] = k;
        s[ns] = zo - zi;
        mu[ns] = -zo / R[k];
        ++ns;
    }
    double zt = sqrt(R[kmin] * R[kmin] - b * b);
    shell[ns] = kmin; s[ns] = zt; mu[ns] = -zt / R[kmin]; ++ns;
    shell[ns] = kmin; s[ns] = zt; mu[ns] = 0.0; ++ns;
    for (int k = kmin + 1; k < n; ++k) {
        double zi = sqrt(R[k - 1] * R[k - 1] - b * b);
        double zo = sqrt(R[k] * R[k] - b * b);
        shell[ns] = k;
        s[ns] = zo - zi;
        mu[ns] = zi / R[k - 1];
        ++ns;
    }
    return ns;
}

/* March one transition through a 1D model with all rays.
 *   vr: radial velocity (outward positive), bD: Doppler width b, kappa, eta per shell.
 *   impact[j], area[j]: ray impact parameter and weight (annulus area).
 * Outputs (any may be NULL): raw per-shell sums Jraw, Lraw (see file header),
 * Wraw = sum a s, Eraw = sum a s sum_c f_c; I_out[j*nch + c] emergent intensity;
 * cons = sum_j a_j dv sum_c (I_bg - I_out). */
void orc1d_march(int n, const double* R, const double* vr, const double* bD,
                 const double* kappa, const double* eta,
                 int n_rays, const double* impact, const double* area,
                 int nch, double vmin, double dv, double I_bg, int n_threads,
                 double* Jraw, double* Lraw, double* Wraw, double* Eraw,
                 double* I_out, double* cons)
{
    int nt = nthreads_of(n_threads);
    accum_t* acc = accum_alloc(nt, n);
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        accum_t* A = &acc[tid];
        int* shell = (int*)malloc(sizeof(int) * 2 * (size_t)n);
        double* s = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* mu = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* I = (double*)malloc(sizeof(double) * (size_t)nch);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int j = 0; j < n_rays; ++j) {
            int ns = orc1d_ray_steps(n, R, impact[j], shell, s, mu);
            for (int c = 0; c < nch; ++c) I[c] = I_bg;
            double a = area[j];
            for (int i = 0; i < ns; ++i) {
                int k = shell[i];
                double w = vr[k] * mu[i];
                double sj, sl, se;
                cell_step(nch, vmin, dv, I, kappa[k], eta[k], bD[k], w, s[i], &sj, &sl, &se);
                A->J[k] += a * s[i] * sj;
                A->L[k] += a * s[i] * sl;
                A->W[k] += a * s[i];
                A->E[k] += a * s[i] * se;
            }
            double d = 0.0;
            for (int c = 0; c < nch; ++c) d += I_bg - I[c];
            A->cons += a * dv * d;
            if (I_out)
                for (int c = 0; c < nch; ++c) I_out[(size_t)j * nch + c] = I[c];
        }
        free(shell);
        free(s);
        free(mu);
        free(I);
    }
    accum_reduce_free(acc, nt, n, Jraw, Lraw, Wraw, Eraw, cons);
}

/* ========================================================================= */
/* 3D regular grid (Sect. 2.2)                                                */
/* ========================================================================= */

/* Main direction: the axis of the largest |component|; components equal to
 * within 1e-12 (relative) are resolved towards the lowest axis index. */
int orc3d_main_axis(const double* d)
{
    double mx = fabs(d[0]);
    if (fabs(d[1]) > mx) mx = fabs(d[1]);
    if (fabs(d[2]) > mx) mx = fabs(d[2]);
    for (int i = 0; i < 3; ++i)
        if (fabs(d[i]) >= mx * (1.0 - 1.0e-12)) return i;
    return 2;
}

/* Walk one ray of direction d across an N^3 grid of unit cells.  The ray
 * starts on the upstream face of the main axis m at transverse lattice point
 * (i + off, j + off) of the two other axes (in increasing axis order) and ends
 * when it leaves through the downstream face.  A ray leaving through a side
 * re-enters at the opposite side at the same main-axis coordinate; such a step
 * is flagged in restart[] (the ray carries background intensity again).
 * Crossings of several planes within 1e-12 cell of each other are taken as
 * one (edge and corner hits).  len[] is in cell units.  Returns the number of
 * steps, or -1 if cap is exceeded. */
int orc3d_walk(int N, const double* d, int i, int j, double off,
               int* cell, double* len, unsigned char* restart, int cap)
{
    int m = orc3d_main_axis(d);
    int ax_a = (m == 0) ? 1 : 0;
    int ax_b = (m == 2) ? 1 : 2;
    double p[3];
    int c[3];
    p[m] = (d[m] > 0) ? 0.0 : (double)N;
    c[m] = (d[m] > 0) ? 0 : N - 1;
    p[ax_a] = i + off; c[ax_a] = i;
    p[ax_b] = j + off; c[ax_b] = j;
    int ns = 0;
    int fresh = 1;
    for (;;) {
        double t[3];
        for (int ax = 0; ax < 3; ++ax) {
            if (d[ax] > 0) t[ax] = ((c[ax] + 1) - p[ax]) / d[ax];
            else if (d[ax] < 0) t[ax] = (c[ax] - p[ax]) / d[ax];
            else t[ax] = INFINITY;
        }
        double tmin = t[0];
        if (t[1] < tmin) tmin = t[1];
        if (t[2] < tmin) tmin = t[2];
        if (ns >= cap) return -1;
        cell[ns] = (c[2] * N + c[1]) * N + c[0];
        len[ns] = tmin;
        restart[ns] = (unsigned char)fresh;
        fresh = 0;
        ++ns;
        for (int ax = 0; ax < 3; ++ax) {
            if (t[ax] <= tmin + 1.0e-12) {
                if (d[ax] > 0) { p[ax] = c[ax] + 1; c[ax] += 1; }
                else { p[ax] = c[ax]; c[ax] -= 1; }
            } else {
                p[ax] += tmin * d[ax];
            }
        }
        if (c[m] < 0 || c[m] >= N) break;
        int axes[2] = {ax_a, ax_b};
        for (int q = 0; q < 2; ++q) {
            int ax = axes[q];
            if (c[ax] >= N) { c[ax] -= N; p[ax] -= N; fresh = 1; }
            else if (c[ax] < 0) { c[ax] += N; p[ax] += N; fresh = 1; }
        }
    }
    return ns;
}

/* Per-direction path length (cell units) summed over all N^2 rays, per cell:
 * out[dir*N^3 + cell]. */
void orc3d_path_sums(int N, int n_dir, const double* dirs, double* out)
{
    long nc = (long)N * N * N;
    int cap = 8 * N + 16;
    int* cell = (int*)malloc(sizeof(int) * (size_t)cap);
    double* len = (double*)malloc(sizeof(double) * (size_t)cap);
    unsigned char* rs = (unsigned char*)malloc((size_t)cap);
    for (int q = 0; q < n_dir; ++q) {
        double* o = out + (size_t)q * nc;
        memset(o, 0, sizeof(double) * (size_t)nc);
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                int ns = orc3d_walk(N, dirs + 3 * q, i, j, 0.5, cell, len, rs, cap);
                for (int k = 0; k < ns; ++k) o[cell[k]] += len[k];
            }
    }
    free(cell);
    free(len);
    free(rs);
}

/* March one transition through an N^3 grid of cells of size delta (cm) for
 * all directions; ray weight a = delta^2 |d_m|.  Per-cell inputs are FP64:
 * velocity components, Doppler width, kappa, eta.  Outputs as orc1d_march;
 * I_out[(dir*N*N + j*N + i)*nch + c] is the intensity leaving the downstream
 * face for ray (i, j) of each direction (may be NULL). */
void orc3d_march(int N, double delta, const double* vx, const double* vy, const double* vz,
                 const double* bD, const double* kappa, const double* eta,
                 int n_dir, const double* dirs,
                 int nch, double vmin, double dv, double I_bg, int n_threads,
                 double* Jraw, double* Lraw, double* Wraw, double* Eraw,
                 double* I_out, double* cons)
{
    long nc = (long)N * N * N;
    int nt = nthreads_of(n_threads);
    accum_t* acc = accum_alloc(nt, nc);
    long n_rays_total = (long)n_dir * N * N;
    int cap = 8 * N + 16;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        accum_t* A = &acc[tid];
        int* cell = (int*)malloc(sizeof(int) * (size_t)cap);
        double* len = (double*)malloc(sizeof(double) * (size_t)cap);
        unsigned char* rs = (unsigned char*)malloc((size_t)cap);
        double* I = (double*)malloc(sizeof(double) * (size_t)nch);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long r = 0; r < n_rays_total; ++r) {
            int q = (int)(r / ((long)N * N));
            int rem = (int)(r % ((long)N * N));
            int jj = rem / N, ii = rem % N;
            const double* d = dirs + 3 * q;
            int m = orc3d_main_axis(d);
            double a = delta * delta * fabs(d[m]);
            int ns = orc3d_walk(N, d, ii, jj, 0.5, cell, len, rs, cap);
            for (int k = 0; k < ns; ++k) {
                if (rs[k]) {
                    if (k > 0) {
                        double dsum = 0.0;
                        for (int c = 0; c < nch; ++c) dsum += I_bg - I[c];
                        A->cons += a * dv * dsum;
                    }
                    for (int c = 0; c < nch; ++c) I[c] = I_bg;
                }
                int cc = cell[k];
                double s = len[k] * delta;
                double w = vx[cc] * d[0] + vy[cc] * d[1] + vz[cc] * d[2];
                double sj, sl, se;
                cell_step(nch, vmin, dv, I, kappa[cc], eta[cc], bD[cc], w, s, &sj, &sl, &se);
                A->J[cc] += a * s * sj;
                A->L[cc] += a * s * sl;
                A->W[cc] += a * s;
                A->E[cc] += a * s * se;
            }
            double dsum = 0.0;
            for (int c = 0; c < nch; ++c) dsum += I_bg - I[c];
            A->cons += a * dv * dsum;
            if (I_out)
                for (int c = 0; c < nch; ++c) I_out[(size_t)r * nch + c] = I[c];
        }
        free(cell);
        free(len);
        free(rs);
        free(I);
    }
    accum_reduce_free(acc, nt, nc, Jraw, Lraw, Wraw, Eraw, cons);
}
