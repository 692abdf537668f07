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
 *   Hyperfine structure (Sect. 1; LTE between the components): the profile is
 *   the weighted sum of K such Gaussians, component k centred at the channel
 *   velocity v_k - w, p_c = sum_k w_k exp(-((v_c + w - v_k)/b)^2) / (b sqrt(pi))
 *   with the relative strengths w_k divided by their sum.
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

/* Line shape of one transition: n == 0 is the single Gaussian; otherwise n
 * hyperfine components at velocity offsets v[k] (cm/s) with relative
 * strengths w[k] (normalised here by their sum). */
typedef struct {
    int n;
    const double* v;
    const double* w;
    double wsum;
} shape_t;

static shape_t shape_of(int n, const double* v, const double* w)
{
    shape_t L = {n > 0 ? n : 0, v, w, 0.0};
    for (int k = 0; k < L.n; ++k) L.wsum += w[k];
    return L;
}

/* Profile density at u = v_c + w for Doppler width b (see file header). */
static double profile(const shape_t* L, double u, double b)
{
    const double norm = 1.0 / (b * sqrt(M_PI));
    if (L->n == 0) {
        double x = u / b;
        return exp(-x * x) * norm;
    }
    double p = 0.0;
    for (int k = 0; k < L->n; ++k) {
        double x = (u - L->v[k]) / b;
        p += L->w[k] * exp(-x * x);
    }
    return p / L->wsum * norm;
}

/* One ray step through one cell for all channels.  Returns the raw per-step
 * sums sum_c f_c I_c beta_c, sum_c f_c (1-beta_c) and sum_c f_c through the
 * pointers (not multiplied by a s). */
static void cell_step(const shape_t* L, int nch, double vmin, double dv, double* I,
                      double kappa, double eta, double b, double w, double s,
                      double* sj, double* sl, double* se)
{
    double js = 0.0, ls = 0.0, es = 0.0;
    for (int c = 0; c < nch; ++c) {
        double v = vmin + (c + 0.5) * dv;
        double p = profile(L, v + w, b);
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
 * cons = sum_j a_j dv sum_c (I_bg - I_out).  n_hf, hf_v, hf_w: line shape
 * (n_hf = 0: single Gaussian). */
void orc1d_march(int n, const double* R, const double* vr, const double* bD,
                 const double* kappa, const double* eta,
                 int n_rays, const double* impact, const double* area,
                 int nch, double vmin, double dv, double I_bg, int n_threads,
                 double* Jraw, double* Lraw, double* Wraw, double* Eraw,
                 double* I_out, double* cons, int n_hf, const double* hf_v, const double* hf_w)
{
    const shape_t shape = shape_of(n_hf, hf_v, hf_w);
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
                cell_step(&shape, nch, vmin, dv, I, kappa[k], eta[k], bD[k], w, s[i], &sj, &sl, &se);
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

/* Sub-iterations in an optically thick core (the paper's Sect. 4 suggests
 * updating the populations more often where the lines are thick).  The core
 * is the inner ball of shells 0..K.  A ray reaches it when its innermost
 * shell is inside it (R[K] > b); its path inside the core is one contiguous
 * piece of its step list: inwards from R[K], the two tangent halves, outwards
 * back to R[K].
 *
 * orc1d_core_entry: the intensity each ray carries when it reaches R[K] on
 * its way in (the march of its envelope steps only, from I_bg), into
 * I_enter[j*nch + c] for the rays that reach the core (others untouched).
 *
 * orc1d_march_core: the core piece of every ray that reaches the core, with
 * the same steps and weights as orc1d_march, starting from I_enter; raw
 * per-shell sums into Jraw, Lraw (all n entries written; zero outside the
 * core). */
void orc1d_core_entry(int n, const double* R, const double* vr, const double* bD,
                      const double* kappa, const double* eta, int n_rays, const double* impact,
                      int K, int nch, double vmin, double dv, double I_bg, double* I_enter)
{
    const shape_t shape = shape_of(0, NULL, NULL);
    int* shell = (int*)malloc(sizeof(int) * 2 * (size_t)n);
    double* s = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* mu = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    for (int j = 0; j < n_rays; ++j) {
        if (!(R[K] > impact[j])) continue;
        int ns = orc1d_ray_steps(n, R, impact[j], shell, s, mu);
        double* I = I_enter + (size_t)j * nch;
        for (int c = 0; c < nch; ++c) I[c] = I_bg;
        for (int i = 0; i < ns && shell[i] > K; ++i) {
            int k = shell[i];
            double sj, sl, se;
            cell_step(&shape, nch, vmin, dv, I, kappa[k], eta[k], bD[k], vr[k] * mu[i], s[i], &sj, &sl, &se);
        }
    }
    free(shell);
    free(s);
    free(mu);
}

void orc1d_march_core(int n, const double* R, const double* vr, const double* bD,
                      const double* kappa, const double* eta, int n_rays, const double* impact,
                      const double* area, int K, int nch, double vmin, double dv, const double* I_enter,
                      double* Jraw, double* Lraw)
{
    const shape_t shape = shape_of(0, NULL, NULL);
    int* shell = (int*)malloc(sizeof(int) * 2 * (size_t)n);
    double* s = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* mu = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* I = (double*)malloc(sizeof(double) * (size_t)nch);
    for (int k = 0; k < n; ++k) Jraw[k] = Lraw[k] = 0.0;
    for (int j = 0; j < n_rays; ++j) {
        if (!(R[K] > impact[j])) continue;
        int ns = orc1d_ray_steps(n, R, impact[j], shell, s, mu);
        for (int c = 0; c < nch; ++c) I[c] = I_enter[(size_t)j * nch + c];
        for (int i = 0; i < ns; ++i) {
            int k = shell[i];
            if (k > K) continue;             /* envelope steps: before and after the core piece */
            double sj, sl, se;
            cell_step(&shape, nch, vmin, dv, I, kappa[k], eta[k], bD[k], vr[k] * mu[i], s[i], &sj, &sl, &se);
            Jraw[k] += area[j] * s[i] * sj;
            Lraw[k] += area[j] * s[i] * sl;
        }
    }
    free(shell);
    free(s);
    free(mu);
    free(I);
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
 * face for ray (i, j) of each direction (may be NULL).  Line shape as in
 * orc1d_march. */
void orc3d_march(int N, double delta, const double* vx, const double* vy, const double* vz,
                 const double* bD, const double* kappa, const double* eta,
                 int n_dir, const double* dirs,
                 int nch, double vmin, double dv, double I_bg, int n_threads,
                 double* Jraw, double* Lraw, double* Wraw, double* Eraw,
                 double* I_out, double* cons, int n_hf, const double* hf_v, const double* hf_w)
{
    const shape_t shape = shape_of(n_hf, hf_v, hf_w);
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
                cell_step(&shape, nch, vmin, dv, I, kappa[cc], eta[cc], bD[cc], w, s, &sj, &sl, &se);
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

/* ========================================================================= */
/* 3D octree (Sect. 2.2)                                                      */
/* ========================================================================= */
/*
 * Tree: an N^3 root grid (level 0, cell (x,y,z) at (z N + y) N + x) whose cells
 * may be split into 8 children, recursively, down to level Lmax.  Cells are
 * numbered globally; child[g] is the global index of the first of the 8
 * children of cell g (child offset cx + 2 cy + 4 cz), or -1 if g is a leaf.
 * Lengths are in root-cell units inside the tracer.
 *
 * Rays of one direction live on nested lattices of lines parallel to the
 * direction (Sect. 2.2: the ray grid follows the spatial discretisation).  In
 * coordinates u that increase along the direction of travel on every axis
 * (u = x for d_x >= 0, u = N - x otherwise), a level-l line pierces the
 * upstream face u_m = 0 at transverse positions o + i h_l, with h_l = 2^-l root
 * cells and o = h_Lmax / 2.  A line is labelled by its finest-lattice indices
 * (la, lb): u_a = (la + 1/2) h_Lmax + t d_a (t = path length); its level is the
 * coarsest lattice that holds it.  The rules, all from Sect. 2.2:
 *   - a root line starts on every upstream surface element with the
 *     background intensity;
 *   - a ray that enters a leaf finer than its current level through the
 *     leaf's upstream face splits: for every level between, the three other
 *     lines of the next level that cross the same upstream face of the
 *     refined cell start there with a copy of the ray's intensity;
 *   - the ray entering a leaf C through its upstream face (the only line of
 *     C's level that does so) checks C's illuminated side faces: where the line
 *     of C's level that enters through a side face is not already present in
 *     the neighbouring leaf (the neighbour is coarser than that line's level),
 *     it is created at that face with the intensity the first ray carried at
 *     C's upstream face (with the background intensity at the model boundary);
 *   - each created ray is tagged with its line's level; a ray entering a leaf
 *     coarser than its tag ends there; otherwise its level becomes the leaf's
 *     (the photon-count rescaling of the paper is the change of the weight
 *     a = h_L^2 |d_m| in intensity form);
 *   - a ray leaving through a side of the model re-enters at the opposite side
 *     at the same main-axis coordinate with the background intensity; a ray
 *     leaving through the downstream face ends.
 * Crossings that coincide (to 1e-10 root cells) are taken one after the other
 * in the order a-face, b-face, main-axis face, as for lines shifted by an
 * infinitesimal amount towards +a (and a far smaller one towards +b); cells
 * are half-open [lo, hi) in u, and a point that a crossing leaves exactly on
 * a face of another axis is on the side that order gives (below the face if
 * that axis comes later).  Every leaf of level L is then crossed, per
 * direction, by the level-L lines that meet it, with a total path of
 * h_L / |d_m|.
 */

#define OCT_TOL 1.0e-10

typedef struct {
    int N, Lmax;
    long long P;             /* finest cells per axis: N << Lmax */
    double h;                /* finest cell size (root units) */
    const int* child;
    int ax[3];               /* storage axis of u-axis 0 (a), 1 (b), 2 (m) */
    int flip[3];             /* per storage axis: direction component < 0 */
    double du[3];            /* |d| along u-axes a, b, m */
} oct_geom_t;

static int oct_geom_init(oct_geom_t* G, int N, int Lmax, const int* child, const double* d)
{
    G->N = N;
    G->Lmax = Lmax;
    G->P = (long long)N << Lmax;
    G->h = 1.0 / (double)(1 << Lmax);
    G->child = child;
    int m = orc3d_main_axis(d);
    G->ax[2] = m;
    G->ax[0] = (m == 0) ? 1 : 0;
    G->ax[1] = (m == 2) ? 1 : 2;
    for (int s = 0; s < 3; ++s) G->flip[s] = d[s] < 0.0;
    for (int u = 0; u < 3; ++u) G->du[u] = fabs(d[G->ax[u]]);
    return m;
}

/* Leaf containing the finest cell with u-indices f[0..2] (a, b, m); returns
 * its global index and level. */
static long oct_leaf(const oct_geom_t* G, const long long* f, int* level)
{
    long long s[3];
    for (int u = 0; u < 3; ++u) {
        int sa = G->ax[u];
        s[sa] = G->flip[sa] ? (G->P - 1 - f[u]) : f[u];
    }
    const int L = G->Lmax;
    long g = ((long)(s[2] >> L) * G->N + (long)(s[1] >> L)) * G->N + (long)(s[0] >> L);
    int l = 0;
    while (G->child[g] >= 0) {
        ++l;
        const int sh = L - l;
        const int c = (int)((s[0] >> sh) & 1) + 2 * (int)((s[1] >> sh) & 1) + 4 * (int)((s[2] >> sh) & 1);
        g = G->child[g] + c;
    }
    *level = l;
    return g;
}

/* Event order: earlier time first, coinciding times in axis order a, b, m. */
static int oct_before(double t1, int r1, double t2, int r2)
{
    if (t1 < t2 - OCT_TOL) return 1;
    if (t1 > t2 + OCT_TOL) return 0;
    return r1 < r2;
}

static int oct_tz(long long v, int cap)
{
    int z = 0;
    while (z < cap && (v & 1) == 0) { v >>= 1; ++z; }
    return z;
}

/* Level of the line with finest-lattice indices (la, lb). */
static int oct_line_level(const oct_geom_t* G, long long la, long long lb)
{
    long long ma = ((la % G->P) + G->P) % G->P, mb = ((lb % G->P) + G->P) % G->P;
    int za = ma == 0 ? G->Lmax : oct_tz(ma, G->Lmax);
    int zb = mb == 0 ? G->Lmax : oct_tz(mb, G->Lmax);
    return G->Lmax - (za < zb ? za : zb);
}

static long long oct_clampll(long long v, long long lo, long long hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Finest-cell index along u-axis u of a point at coordinate pos reached by a
 * crossing of axis ex.  A point on a face of axis u is below it if that
 * crossing comes later in the order a, b, m, else above it. */
static long long oct_index_after(const oct_geom_t* G, double pos, int u, int ex)
{
    const double x = pos / G->h;
    const double k = nearbyint(x);
    if (fabs(x - k) <= OCT_TOL / G->h) return (long long)k - (u > ex ? 1 : 0);
    return (long long)floor(x);
}

typedef struct {
    long long l[2];          /* line indices (a, b) */
    long long f[3];          /* finest u-indices of the first cell */
    double t;                /* start time */
    int entry;               /* axis crossed to enter: 0 a, 1 b, 2 m */
    int tag, lcur;
    int vec;                 /* saved intensity vector, -1 = background */
} oct_ray_t;

typedef struct {
    oct_ray_t* r;
    int n, cap;
    double* vec;             /* saved vectors, nch each */
    int nv, capv;
} oct_stack_t;

static void oct_push(oct_stack_t* S, const oct_ray_t* r)
{
    if (S->n == S->cap) {
        S->cap = S->cap ? 2 * S->cap : 64;
        S->r = (oct_ray_t*)realloc(S->r, sizeof(oct_ray_t) * (size_t)S->cap);
    }
    S->r[S->n++] = *r;
}

static int oct_save(oct_stack_t* S, const double* I, int nch)
{
    if (S->nv == S->capv) {
        S->capv = S->capv ? 2 * S->capv : 16;
        S->vec = (double*)realloc(S->vec, sizeof(double) * (size_t)S->capv * (size_t)(nch > 0 ? nch : 1));
    }
    if (nch > 0) memcpy(S->vec + (size_t)S->nv * nch, I, sizeof(double) * (size_t)nch);
    return S->nv++;
}

/* Statistics of a march: rays started (root, split, side), rays ended by a
 * coarser leaf, model-side re-entries, steps. */
enum { OCT_ROOT, OCT_SPLIT, OCT_SIDE, OCT_TERM, OCT_WRAP, OCT_STEPS, OCT_NSTAT };

/* Trace every ray that the line (la, lb) of the finest lattice (a root line
 * has la, lb multiples of 2^Lmax) gives rise to.  With nch == 0 only the path
 * bookkeeping (W) is done.  'plain' traces the single line without splitting,
 * side rays or termination (lines of sight for maps); I_end then receives its
 * final intensity.  'brute' (the brute-force alternative of Sect. 2.2: a
 * regular lattice of 4^Lmax lines per root surface element) traces the single
 * line as 'plain' and weights every step with the finest lattice's h^2 |d_m|
 * instead of the crossed leaf's. */
static void oct_trace_root(const oct_geom_t* G, const shape_t* shape, long long la, long long lb, double root_cm,
                           const double* dvec, const double* vx, const double* vy, const double* vz,
                           const double* bD, const double* kappa, const double* eta,
                           int nch, double vmin, double dv, double I_bg, int plain, int brute,
                           accum_t* A, long long* stats, oct_stack_t* S, double* I, double* I_end)
{
    const int Lmax = G->Lmax;
    const double h = G->h;
    const double dm = G->du[2];
    if (brute) plain = 1;
    S->n = 0;
    S->nv = 0;
    oct_ray_t r0;
    r0.l[0] = la;
    r0.l[1] = lb;
    r0.f[0] = r0.l[0];
    r0.f[1] = r0.l[1];
    r0.f[2] = 0;
    r0.t = 0.0;
    r0.entry = 2;
    r0.tag = 0;
    r0.lcur = 0;
    r0.vec = -1;
    oct_push(S, &r0);
    stats[OCT_ROOT]++;
    while (S->n > 0) {
        oct_ray_t R = S->r[--S->n];
        if (nch > 0) {
            if (R.vec < 0) for (int c = 0; c < nch; ++c) I[c] = I_bg;
            else memcpy(I, S->vec + (size_t)R.vec * nch, sizeof(double) * (size_t)nch);
        }
        for (;;) {
            int L;
            const long g = oct_leaf(G, R.f, &L);
            if (!plain && L < R.tag) { stats[OCT_TERM]++; break; }
            const long long size = 1LL << (Lmax - L);
            const double Dc = (double)size * h;
            long long lo[3];
            for (int u = 0; u < 3; ++u) lo[u] = (R.f[u] / size) * size;
            if (!plain && R.entry == 2) {
                int saved = -1;
                /* upstream split, one level at a time */
                for (int l = R.lcur + 1; l <= L; ++l) {
                    const int sh = Lmax - l;
                    const long long st = 1LL << sh;
                    const long long sa = (R.f[0] >> sh) & 1, sb = (R.f[1] >> sh) & 1;
                    if (saved < 0) saved = oct_save(S, I, nch);
                    for (long long na = 0; na < 2; ++na)
                        for (long long nb = 0; nb < 2; ++nb) {
                            if (na == sa && nb == sb) continue;
                            oct_ray_t c = R;
                            c.l[0] = R.l[0] + (na - sa) * st;
                            c.l[1] = R.l[1] + (nb - sb) * st;
                            c.f[0] = R.f[0] + (na - sa) * st;
                            c.f[1] = R.f[1] + (nb - sb) * st;
                            c.entry = 2;
                            c.tag = l;
                            c.lcur = l;
                            c.vec = saved;
                            oct_push(S, &c);
                            stats[OCT_SPLIT]++;
                        }
                }
                /* side rays through the illuminated side faces of C */
                const double t_mexit = (double)(lo[2] + size) * h / dm;
                double tx[2] = {INFINITY, INFINITY};
                for (int x = 0; x < 2; ++x) {
                    if (!(G->du[x] > 0.0)) continue;
                    const double rel = ((double)R.l[x] + 0.5) * h + R.t * G->du[x] - (double)lo[x] * h;
                    tx[x] = R.t + (Dc - rel) / G->du[x];
                }
                for (int x = 0; x < 2; ++x) {
                    const int y = 1 - x;
                    if (!(G->du[x] > 0.0) || !oct_before(tx[x], x, t_mexit, 2)) continue;
                    const int shift_y = (G->du[y] > 0.0) && oct_before(tx[y], y, tx[x], x);
                    long long nl[2];
                    nl[x] = R.l[x] - size;
                    nl[y] = R.l[y] - (shift_y ? size : 0);
                    const int lev = oct_line_level(G, nl[0], nl[1]);
                    const int boundary = lo[x] == 0;
                    long long nf[3];
                    nf[x] = boundary ? G->P - 1 : lo[x] - 1;
                    nf[y] = lo[y];
                    nf[2] = lo[2];
                    int LN;
                    (void)oct_leaf(G, nf, &LN);
                    if (!(LN < L && LN < lev)) continue;
                    oct_ray_t c;
                    c.l[0] = nl[0];
                    c.l[1] = nl[1];
                    c.t = tx[x];
                    c.f[x] = lo[x];
                    const double py = ((double)nl[y] + 0.5) * h + tx[x] * G->du[y];
                    c.f[y] = oct_clampll(oct_index_after(G, py, y, x), lo[y], lo[y] + size - 1);
                    c.f[2] = oct_clampll(oct_index_after(G, tx[x] * dm, 2, x), lo[2], lo[2] + size - 1);
                    c.entry = x;
                    c.tag = lev;
                    c.lcur = L;
                    if (boundary) c.vec = -1;
                    else {
                        if (saved < 0) saved = oct_save(S, I, nch);
                        c.vec = saved;
                    }
                    oct_push(S, &c);
                    stats[OCT_SIDE]++;
                }
            }
            R.lcur = L;
            /* step through C */
            double te[3];
            for (int x = 0; x < 2; ++x)
                te[x] = G->du[x] > 0.0
                            ? ((double)(lo[x] + size) * h - ((double)R.l[x] + 0.5) * h) / G->du[x]
                            : INFINITY;
            te[2] = (double)(lo[2] + size) * h / dm;
            int ex = 0;
            for (int u = 1; u < 3; ++u)
                if (oct_before(te[u], u, te[ex], ex)) ex = u;
            double s = te[ex] - R.t;
            if (s < 0.0) s = 0.0;
            const double side = brute ? h : Dc;
            const double a_w = (side * root_cm) * (side * root_cm) * dm;
            const double s_cm = s * root_cm;
            if (nch > 0) {
                const double w = vx[g] * dvec[0] + vy[g] * dvec[1] + vz[g] * dvec[2];
                double in = 0.0, out = 0.0;
                for (int c = 0; c < nch; ++c) in += I[c];
                double sj, sl, se;
                cell_step(shape, nch, vmin, dv, I, kappa[g], eta[g], bD[g], w, s_cm, &sj, &sl, &se);
                for (int c = 0; c < nch; ++c) out += I[c];
                if (A) {
                    A->J[g] += a_w * s_cm * sj;
                    A->L[g] += a_w * s_cm * sl;
                    A->E[g] += a_w * s_cm * se;
                    A->cons += a_w * dv * (in - out);
                }
            }
            if (A) A->W[g] += a_w * s_cm;
            stats[OCT_STEPS]++;
            /* cross the exit face */
            R.t = te[ex];
            for (int u = 0; u < 3; ++u) {
                if (u == ex) continue;
                const double pu = u == 2 ? R.t * dm : ((double)R.l[u] + 0.5) * h + R.t * G->du[u];
                R.f[u] = oct_clampll(oct_index_after(G, pu, u, ex), lo[u], lo[u] + size - 1);
            }
            R.f[ex] = lo[ex] + size;
            R.entry = ex;
            if (ex == 2) {
                if (R.f[2] >= G->P) break;           /* downstream face: the ray escapes */
            } else if (R.f[ex] >= G->P) {             /* model side: re-enter opposite */
                R.f[ex] -= G->P;
                R.l[ex] -= G->P;
                if (nch > 0) for (int c = 0; c < nch; ++c) I[c] = I_bg;
                stats[OCT_WRAP]++;
            }
        }
        if (plain && I_end && nch > 0) memcpy(I_end, I, sizeof(double) * (size_t)nch);
    }
}

/* One transition through an octree for all directions (see above).
 * Per-cell FP64 inputs over all cells (only leaves are used).  Raw sums as
 * orc3d_march; 'stats' receives OCT_NSTAT counters (may be NULL).  With
 * nch == 0 only W is produced (kappa, eta, velocities may be NULL).  Line
 * shape as in orc1d_march. */
static void oct_march(int N, int Lmax, long n_cells, const int* child, double root_cm,
                      const double* vx, const double* vy, const double* vz,
                      const double* bD, const double* kappa, const double* eta,
                      int n_dir, const double* dirs,
                      int nch, double vmin, double dv, double I_bg, int n_threads,
                      double* Jraw, double* Lraw, double* Wraw, double* Eraw, double* cons,
                      long long* stats, int n_hf, const double* hf_v, const double* hf_w, int brute)
{
    const shape_t shape = shape_of(n_hf, hf_v, hf_w);
    int nt = nthreads_of(n_threads);
    accum_t* acc = accum_alloc(nt, n_cells);
    long long* st = (long long*)calloc((size_t)nt * OCT_NSTAT, sizeof(long long));
    /* tasks: root elements, or with 'brute' every line of the finest lattice */
    const long side = brute ? ((long)N << Lmax) : (long)N;
    long n_task = (long)n_dir * side * side;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        oct_stack_t S = {0};
        double* I = (double*)malloc(sizeof(double) * (size_t)(nch > 0 ? nch : 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (long r = 0; r < n_task; ++r) {
            const int q = (int)(r / (side * side));
            const long rem = r % (side * side);
            const int sh = brute ? 0 : Lmax;
            oct_geom_t G;
            oct_geom_init(&G, N, Lmax, child, dirs + 3 * q);
            oct_trace_root(&G, &shape, (long long)(rem % side) << sh, (long long)(rem / side) << sh, root_cm,
                           dirs + 3 * q, vx, vy, vz, bD, kappa, eta, nch, vmin, dv, I_bg, 0, brute, &acc[tid],
                           st + (size_t)tid * OCT_NSTAT, &S, I, NULL);
        }
        free(S.r);
        free(S.vec);
        free(I);
    }
    accum_reduce_free(acc, nt, n_cells, Jraw, Lraw, Wraw, Eraw, cons);
    if (stats)
        for (int k = 0; k < OCT_NSTAT; ++k) {
            long long v = 0;
            for (int t = 0; t < nt; ++t) v += st[(size_t)t * OCT_NSTAT + k];
            stats[k] = v;
        }
    free(st);
}

/* March one transition through an octree for all directions with the rays
 * the octree scheme creates and terminates (see above). */
void orcoct_march(int N, int Lmax, long n_cells, const int* child, double root_cm,
                  const double* vx, const double* vy, const double* vz,
                  const double* bD, const double* kappa, const double* eta,
                  int n_dir, const double* dirs,
                  int nch, double vmin, double dv, double I_bg, int n_threads,
                  double* Jraw, double* Lraw, double* Wraw, double* Eraw, double* cons,
                  long long* stats, int n_hf, const double* hf_v, const double* hf_w)
{
    oct_march(N, Lmax, n_cells, child, root_cm, vx, vy, vz, bD, kappa, eta, n_dir, dirs, nch, vmin, dv, I_bg,
              n_threads, Jraw, Lraw, Wraw, Eraw, cons, stats, n_hf, hf_v, hf_w, 0);
}

/* The brute-force alternative (Sect. 2.2): every line of the finest lattice
 * (4^Lmax per root surface element) traced straight through the leaves with
 * weight h_Lmax^2 |d_m|, re-entering with the background at model sides;
 * arguments and outputs as orcoct_march. */
void orcoct_march_brute(int N, int Lmax, long n_cells, const int* child, double root_cm,
                        const double* vx, const double* vy, const double* vz,
                        const double* bD, const double* kappa, const double* eta,
                        int n_dir, const double* dirs,
                        int nch, double vmin, double dv, double I_bg, int n_threads,
                        double* Jraw, double* Lraw, double* Wraw, double* Eraw, double* cons,
                        long long* stats, int n_hf, const double* hf_v, const double* hf_w)
{
    oct_march(N, Lmax, n_cells, child, root_cm, vx, vy, vz, bD, kappa, eta, n_dir, dirs, nch, vmin, dv, I_bg,
              n_threads, Jraw, Lraw, Wraw, Eraw, cons, stats, n_hf, hf_v, hf_w, 1);
}

/* +z map of an octree: one straight line of sight per root surface element
 * (x, y) on the level-0 ray lattice of the +z direction (transverse offset
 * h_Lmax / 2 from the element's corner), marched without accumulation.
 * I_out[(y N + x) * nch + c] is the intensity leaving the top face.  Line
 * shape as in orc1d_march. */
void orcoct_map_z(int N, int Lmax, const int* child, double root_cm,
                  const double* vx, const double* vy, const double* vz,
                  const double* bD, const double* kappa, const double* eta,
                  int nch, double vmin, double dv, double I_bg, int n_threads, double* I_out,
                  int n_hf, const double* hf_v, const double* hf_w)
{
    const shape_t shape = shape_of(n_hf, hf_v, hf_w);
    int nt = nthreads_of(n_threads);
    const double dz[3] = {0.0, 0.0, 1.0};
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        oct_stack_t S = {0};
        double* I = (double*)malloc(sizeof(double) * (size_t)nch);
        long long st[OCT_NSTAT];
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long r = 0; r < (long)N * N; ++r) {
            oct_geom_t G;
            oct_geom_init(&G, N, Lmax, child, dz);
            oct_trace_root(&G, &shape, (long long)(r % N) << Lmax, (long long)(r / N) << Lmax, root_cm, dz, vx, vy,
                           vz, bD, kappa, eta, nch, vmin, dv, I_bg, 1, 0, NULL, st, &S, I, I_out + (size_t)r * nch);
        }
        free(S.r);
        free(S.vec);
        free(I);
    }
}
