// kernels.hip -- gfx950 kernels of the ALI line ray march.
//
//   prepare      populations -> per (cell, transition) opacity/emissivity (khat, ehat)
//   lte          Boltzmann populations at T_kin
//   window table per (direction, cell) channel window of a regular grid or octree
//   march3d      3D regular grid: HEALPix directions, one ray per upstream surface
//                cell, side re-entry with background; per step and channel the
//                radiative update; per-step partial sums of the absorbed counts
//                and of the diagonal operator stored for the gather
//   gather3d     per (cell, transition) FP64 sums of march3d's per-step sums
//   march_oct    octree: replay of the host-built ray schedule (splits, side
//                rays, ends) with saved intensity vectors on a per-group stack
//   gather_oct   per-cell FP64 sums of the octree march's per-step sums
//   march1d      1D shells: impact-parameter rays whose steps were computed once
//                per model in FP64 (ray_steps); per-shell FP64 LDS accumulators
//   se           per-cell statistical equilibrium (FP64 partial-pivot elimination)
//                and the maximum relative population change
//   serve_*      the request loop's persistent, model-indexed kernels
//
// Lane mapping of the marches: a ray owns a group of LANES (8 or 16; up to 64
// for lines of sight) consecutive lanes of one wavefront, several rays per
// wavefront; the lanes cover the channel window of the current step,
// |v_c + w| <= K b, so only channels where the local profile is significantly
// non-zero are touched (App. A.2).  The ray's full channel vector lives in LDS.
// Per step the group reduces its two partial sums with DPP row operations.
#include <hip/hip_runtime.h>
#include <climits>
#include <cstdlib>
#include <math.h>

#include <type_traits>

#include "miloc_internal.h"

namespace miloc {

namespace {

constexpr float kLog2eF = 1.4426950408889634f;

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double fast_exp2(double x) { return exp2(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// 1 - beta and e^{-tau}, beta = (1 - e^{-tau})/tau (Sect. 2, Eqs. (2)-(3)).
// Small |tau|: Taylor series of 1 - beta (no cancellation); else direct.
__device__ __forceinline__ void escape_terms(float tau, float& omb, float& e)
{
    if (fabsf(tau) < 0.2f) {
        float h = (1.0f / 720.0f) - tau * (1.0f / 5040.0f);
        h = (1.0f / 120.0f) - tau * h;
        h = (1.0f / 24.0f) - tau * h;
        h = (1.0f / 6.0f) - tau * h;
        h = 0.5f - tau * h;
        omb = tau * h;
        e = (1.0f - tau) + tau * omb;
    } else {
        e = fast_exp2(-tau * kLog2eF);
        const float beta = (1.0f - e) * __builtin_amdgcn_rcpf(tau);
        omb = 1.0f - beta;
    }
}

__device__ __forceinline__ void escape_terms(double tau, double& omb, double& e)
{
    if (fabs(tau) < 1.0e-3) {
        double h = (1.0 / 120.0) - tau * (1.0 / 720.0);
        h = (1.0 / 24.0) - tau * h;
        h = (1.0 / 6.0) - tau * h;
        h = 0.5 - tau * h;
        omb = tau * h;
        e = (1.0 - tau) + tau * omb;
    } else {
        e = exp(-tau);
        omb = 1.0 + expm1(-tau) / tau;
    }
}

// Sum over a group of LANES (8, 16, 32 or 64) consecutive lanes; the total is
// valid in the group's last lane.  FP32 uses DPP row operations (no LDS
// traffic): quad swaps and the half-row mirror give the last lane of every 8
// its 8-lane sum, the row mirror its 16-lane row sum, row_bcast15 /
// row_bcast31 then fold rows 0->1, 2->3 and (64) 1->3.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v)
{
    const int src = __builtin_bit_cast(int, v);
    const int got = __builtin_amdgcn_update_dpp(0, src, CTRL, ROW_MASK, 0xF, false);
    return v + __builtin_bit_cast(float, got);
}

// The value of v in the lane that DPP control CTRL selects (all rows and banks).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF,
                                                                  false));
}

// Reduce-scatter over a group of 8 lanes: lane l of the group receives the
// sum over the group's lanes of p[l].  Three butterfly stages (pairs l and
// 7 - l by the half-row mirror, then l ^ 2 and l ^ 1 by quad permutations),
// each lane sending the half of its values that its partner keeps.
__device__ __forceinline__ float reduce_scatter8(const float (&p)[8], int lane)
{
    const bool hi = lane & 4, b1 = lane & 2, b0 = lane & 1;
    float q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = (hi ? p[4 + j] : p[j]) + dpp_mov<0x141>(hi ? p[j] : p[4 + j]);
    float r[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) r[m] = (b1 ? q[2 + m] : q[m]) + dpp_mov<0x4E>(b1 ? q[m] : q[2 + m]);
    return (b0 ? r[1] : r[0]) + dpp_mov<0xB1>(b0 ? r[0] : r[1]);
}

// Keeps v computed where it stands rather than sunk into a following branch
// that is its only use (an empty asm statement: no instruction).  Used on the
// group sums: sunk, their last DPP stage cannot be fused into its add.
template <typename T>
__device__ __forceinline__ void keep_here(T& v)
{
    asm volatile("" : "+v"(v));
}

template <int LANES>
__device__ __forceinline__ float group_sum(float v)
{
    v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    if (LANES >= 8) v = dpp_add<0x141, 0xF>(v);    // row_half_mirror
    if (LANES >= 16) v = dpp_add<0x140, 0xF>(v);   // row_mirror
    if (LANES >= 32) v = dpp_add<0x142, 0xA>(v);   // row_bcast15 into rows 1 and 3
    if (LANES == 64) v = dpp_add<0x143, 0xC>(v);   // row_bcast31 into rows 2 and 3
    return v;
}

template <int LANES>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LANES);
    return v;
}

// Radiative update of one step over the channel window.  Lanes take channels
// clo + lane, clo + lane + LANES, ...  Returns the partial sums
// sum e_c I_c beta_c and sum e_c (1 - beta_c) of this lane.
// Channel window [clo, chi] of a step: channels with |c - c*| <= Kw/ibs,
// c* = -(chalf + w), clipped to the band.  frac = clo - c*.
template <typename T>
__device__ __forceinline__ void window(double w, double chalf, T Kw, T ibs, int nch,
                                       int& clo, int& chi, T& frac, double dlo = 0.0, double dhi = 0.0)
{
    const double cstar = -(chalf + w);
    const double hw = (double)(Kw * fast_rcp(ibs));
    int lo = (int)ceil(cstar + dlo - hw);
    int hi = (int)floor(cstar + dhi + hw);
    lo = lo < 0 ? 0 : lo;
    hi = hi > nch - 1 ? nch - 1 : hi;
    clo = lo;
    chi = hi;
    frac = (T)((double)lo - cstar);
}

}  // namespace

// ---------------------------------------------------------------- prepare
// With ibg_sub (spectra) the emission term becomes ehat - I_bg khat, so that the
// march carries I - I_bg directly: I_out - I_bg = (I_in - I_bg) e^-tau
// + (ehat - I_bg khat) len e_c beta, without cancellation where I ~ I_bg.
template <typename T>
__device__ __forceinline__ void prepare_cell(int k, const MolDev* __restrict__ mol, int ntr,
                                             const double* __restrict__ x, const double* __restrict__ nmolLb,
                                             const double* __restrict__ ibg_sub,
                                             typename V2<T>::type* __restrict__ ke)
{
    const int L = mol->L;
    const double* xk = x + (size_t)k * L;
    const double base = nmolLb[k];
    for (int t = 0; t < ntr; ++t) {
        const double xu = xk[mol->up[t]];
        const double xl = xk[mol->lo[t]];
        const double f = base * mol->Ct[t];
        const double kap = f * (xl * mol->gratio[t] - xu);   // kappa term
        double eta = f * xu;                                   // eta term (occupation units)
        if (ibg_sub) eta -= ibg_sub[t] * kap;
        typename V2<T>::type v;
        v.x = (T)kap;
        v.y = (T)eta;
        ke[(size_t)k * ntr + t] = v;
    }
}

template <typename T>
__global__ void prepare_kernel(int nc, const MolDev* __restrict__ mol, int ntr,
                               const double* __restrict__ x, const double* __restrict__ nmolLb,
                               const double* __restrict__ ibg_sub,
                               typename V2<T>::type* __restrict__ ke)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    prepare_cell<T>(k, mol, ntr, x, nmolLb, ibg_sub, ke);
}

__global__ void lte_kernel(int nc, const MolDev* __restrict__ mol, const double* __restrict__ Tkin,
                           double* __restrict__ x)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    const int L = mol->L;
    const double T = Tkin[k];
    double s = 0.0;
    for (int i = 0; i < L; ++i) s += mol->g[i] * exp(-mol->E[i] / T);
    const double inv = 1.0 / s;
    for (int i = 0; i < L; ++i) x[(size_t)k * L + i] = mol->g[i] * exp(-mol->E[i] / T) * inv;
}

// ---------------------------------------------------------------- 3D march
// Per workgroup: rays of one direction (a block never straddles directions).
// The direction's step list is staged in LDS once and read as a broadcast.
// Several rays share a wavefront (8 lanes each for narrow lines), so each
// step issues the cell loads of several independent rays at once.
namespace {

// One move of the ray along a transverse axis with periodic re-entry.
__device__ __forceinline__ void move_transverse(int& c, int& idx, int s, int st, int N, bool& restart)
{
    c += s;
    const bool wrap = (unsigned)c >= (unsigned)N;
    c = wrap ? c - s * N : c;
    idx += wrap ? -s * (N - 1) * st : s * st;
    restart |= wrap;
}

}  // namespace

// Window table of one direction: for every cell the first channel of its
// window, the number of window channels and the profile argument of the first
// channel, all from the FP64 line-of-sight velocity (Sect. 3.1: Doppler shift
// per step; App. A.2: only channels where the profile is significant).  With
// hyperfine components the window runs from the lowest to the highest
// component centre (offsets dlo <= 0 <= dhi channels from the line centre)
// plus the cut on either side; the profile argument stays that of the
// reference centre.
template <typename T>
__global__ void window_table_kernel(int nc, int n_dir, const DirDev* __restrict__ dirs,
                                    const float4* __restrict__ vel, const double* __restrict__ bD,
                                    double dv, double chalf, double K, int nch, double dlo, double dhi,
                                    typename V4<T>::type* __restrict__ win)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (k >= nc || q >= n_dir) return;
    const DirDev& D = dirs[q];
    const float4 u = vel[k];
    const double w = ((double)u.x * D.d[0] + (double)u.y * D.d[1] + (double)u.z * D.d[2]) / dv;
    const double cstar = -(chalf + w);
    const double bc = bD[k] / dv;                 // Doppler width in channels
    const double hw = K * bc;
    int lo = (int)ceil(cstar + dlo - hw);
    int hi = (int)floor(cstar + dhi + hw);
    lo = lo < 0 ? 0 : lo;
    hi = hi > nch - 1 ? nch - 1 : hi;
    const int n = hi >= lo ? hi - lo + 1 : 0;
    const double ibs = 1.2011224087864498 / bc;   // sqrt(log2 e) / (b/dv)
    typename V4<T>::type r;
    r.x = (T)(((double)lo - cstar) * ibs);
    r.y = (T)ibs;
    r.z = __builtin_bit_cast(T, (typename std::conditional<sizeof(T) == 4, int, long long>::type)lo);
    r.w = __builtin_bit_cast(T, (typename std::conditional<sizeof(T) == 4, int, long long>::type)n);
    win[(size_t)q * nc + k] = r;
}

namespace {

template <typename T>
__device__ __forceinline__ int as_int(T v)
{
    return (int)__builtin_bit_cast(typename std::conditional<sizeof(T) == 4, int, long long>::type, v);
}

// 1 - beta for |tau| < 0.01 (3 terms; relative truncation error < 2e-8).
__device__ __forceinline__ float omb_thin(float tau)
{
    const float h = 0.5f - tau * ((1.0f / 6.0f) - tau * (1.0f / 24.0f));
    return tau * h;
}
__device__ __forceinline__ double omb_thin(double tau)
{
    double omb, e;
    escape_terms(tau, omb, e);
    return omb;
}
// 1 - beta for any tau.  FP32: both forms evaluated and one selected, so
// that a wavefront with mixed optical depths does not diverge.
__device__ __forceinline__ float omb_any(float tau)
{
    const float d = 1.0f - (1.0f - fast_exp2(-tau * kLog2eF)) * __builtin_amdgcn_rcpf(tau);
    float h = (1.0f / 720.0f) - tau * (1.0f / 5040.0f);
    h = (1.0f / 120.0f) - tau * h;
    h = (1.0f / 24.0f) - tau * h;
    h = (1.0f / 6.0f) - tau * h;
    h = 0.5f - tau * h;
    return fabsf(tau) < 0.2f ? tau * h : d;
}
__device__ __forceinline__ double omb_any(double tau)
{
    double omb, e;
    escape_terms(tau, omb, e);
    return omb;
}

// Hyperfine components of one transition {d_k = offset in channels, w_k =
// strength, sum 1}: the first kReg in registers, loaded together once per ray
// (a load inside the channel loop would wait on memory per component and
// channel); any further ones are read from memory where they are used.
template <typename T>
struct HfRegs {
    static constexpr int kReg = sizeof(T) == 4 ? 16 : 8;
    T d[kReg], w[kReg];
    const typename V2<T>::type* row;
    int n;
    __device__ __forceinline__ void load(const typename V2<T>::type* __restrict__ r, int count)
    {
        row = r;
        n = count;
#pragma unroll
        for (int k = 0; k < kReg; ++k) {
            const typename V2<T>::type c = r[k < count ? k : 0];
            d[k] = c.x;
            w[k] = k < count ? c.y : (T)0;
        }
    }
};

// Line shape at scaled profile argument xs (the reference centre at 0):
// KC = 0: exp2(-xs^2); otherwise the hyperfine multiplet (Sect. 1, LTE
// between the components) sum_k w_k exp2(-(xs - d_k ibs)^2) over KC register
// components (zero-strength padding beyond the transition's count), and, when
// KC is the whole register set, over the components past it in memory.
template <int KC, typename T>
__device__ __forceinline__ T line_shape(T xs, T ibs, const HfRegs<T>* __restrict__ hf)
{
    if constexpr (KC == 0) {
        return fast_exp2(-xs * xs);
    } else {
        T e = 0;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const T y = xs - hf->d[k] * ibs;
            e += hf->w[k] * fast_exp2(-y * y);
        }
        if constexpr (KC == HfRegs<T>::kReg) {
            for (int k = KC; k < hf->n; ++k) {
                const typename V2<T>::type c = hf->row[k];
                const T y = xs - c.x * ibs;
                e += c.y * fast_exp2(-y * y);
            }
        }
        return e;
    }
}

// The channel window of one step for one ray (Sect. 2: I e^-tau + S(1 -
// e^-tau) per channel, absorbed counts and the diagonal operator summed):
// channels clo .. clo + nwin - 1, profile argument x_j = x0 + j ibs (scaled
// so that the profile is exp2(-x^2)), tau_j = kl e_j, emission el e_j beta_j.
// Partial sums of this lane in sj, sl.  The series/exact choice for 1 - beta
// is made once per step for the whole wavefront (with HF the multiplet's
// profile peaks at most at 1, so |kl| still bounds every |tau_j|).
template <int LANES, typename T, int KC>
__device__ __forceinline__ void window_loop(T* __restrict__ I, int lane, int clo, int nwin, T x0, T ibs,
                                            T kl, T el, T& sj, T& sl, const HfRegs<T>* hf,
                                            unsigned* __restrict__ maser)
{
    const bool thin = __all(kl < (T)0.01 && kl > (T)-0.01);
    // A population inversion strong enough for a line-centre optical depth
    // below kMaserTauMin over one step is reported, not marched on (its
    // exponential gain leaves the FP32 range soon after); only steps off the
    // thin path can qualify.
    if (!thin && kl < (T)kMaserTauMin) *maser = 1u;
    T* __restrict__ row = I + clo;
    if (thin) {
        for (int j = lane; j < nwin; j += LANES) {
            const T xs = (T)j * ibs + x0;
            const T ec = line_shape<KC, T>(xs, ibs, hf);
            const T omb = omb_thin(kl * ec);
            const T Iin = row[j];
            const T u = ec - ec * omb;                 // e_c beta_c
            sj += Iin * u;
            sl += ec * omb;
            row[j] = Iin + u * (el - kl * Iin);        // e^-tau = 1 - tau beta
        }
    } else {
        for (int j = lane; j < nwin; j += LANES) {
            const T xs = (T)j * ibs + x0;
            const T ec = line_shape<KC, T>(xs, ibs, hf);
            const T omb = omb_any(kl * ec);
            const T Iin = row[j];
            const T u = ec - ec * omb;
            sj += Iin * u;
            sl += ec * omb;
            row[j] = Iin + u * (el - kl * Iin);
        }
    }
}

// One channel's radiative update (Sect. 2, Eq. (3) in intensity form) from
// its profile value ec and 1 - beta: the two partial sums of the step and
// I <- I + ec beta (el - kl I), i.e. I e^-tau + S (1 - e^-tau).
__device__ __forceinline__ void channel_update(float* __restrict__ p, float ec, float omb, float kl, float el,
                                               float& sj, float& sl)
{
    const float Iin = *p;
    const float u = fmaf(-ec, omb, ec);            // ec beta
    sj = fmaf(Iin, u, sj);
    sl = fmaf(ec, omb, sl);
    *p = fmaf(u, fmaf(-kl, Iin, el), Iin);
}

// 1 - beta for the optical-depth class of a step: CLS 0 when every |tau| is
// below 1e-3 (two series terms, relative truncation error < tau^2/12 < 1e-7),
// CLS 1 below 1e-2 (three terms), CLS 2 any tau.
template <int CLS>
__device__ __forceinline__ float omb_class(float tau)
{
    if constexpr (CLS == 0) return tau * fmaf(tau, -1.0f / 6.0f, 0.5f);
    else if constexpr (CLS == 1) return omb_thin(tau);
    else return omb_any(tau);
}

// The lane group's passes over the window of one step, FP32 single Gaussian:
// the first NU passes unrolled (channel lane + i LANES, constant LDS offsets
// from rl = I + clo + lane, profile argument xl + i LANES ibs), any further ones
// in a loop.  The NU intensities are read before any is used, whether their
// channel is in the window or not (one wait for all of them; a value outside
// the window is never used): every march keeps at least kVecTailPadWords
// words of its LDS allocation after each channel vector.
template <int LANES, int CLS>
__device__ __forceinline__ void window_passes_f32(float* __restrict__ rl, int lane, int nwin, float xl, float x0,
                                                  float ibs, float kl, float el, float& sj, float& sl)
{
    constexpr int NU = LANES >= 64 ? 1 : (LANES >= 32 ? 2 : 4);
    static_assert(NU * LANES <= kVecTailPadWords, "unconditional reads must stay in the LDS allocation");
    float Iv[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) Iv[i] = rl[i * LANES];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        if (lane + i * LANES < nwin) {
            // i LANES ibs is exact (LANES a power of two): no separate pass
            // stride to form
            const float xs = fmaf((float)(i * LANES), ibs, xl);
            const float ec = fast_exp2(-xs * xs);
            const float omb = omb_class<CLS>(kl * ec);
            const float u = fmaf(-ec, omb, ec);
            sj = fmaf(Iv[i], u, sj);
            sl = fmaf(ec, omb, sl);
            rl[i * LANES] = fmaf(u, fmaf(-kl, Iv[i], el), Iv[i]);
        }
    }
    for (int j = lane + NU * LANES; j < nwin; j += LANES) {
        const float xs = fmaf((float)j, ibs, x0);
        const float ec = fast_exp2(-xs * xs);
        channel_update(rl + (j - lane), ec, omb_class<CLS>(kl * ec), kl, el, sj, sl);
    }
}

template <int LANES, int CLS, bool MASK>
__device__ __forceinline__ void window_passes_pred(float* __restrict__ rl, int lane, int nwin, float xl,
                                                   float x0, float ibs, float l2len, float kh, float eh, float& sj,
                                                   float& sl);

// Channels the unrolled passes of a lane group reach from a window's start.
template <int LANES>
constexpr int pass_reach() { return (LANES >= 64 ? 1 : (LANES >= 32 ? 2 : 4)) * LANES; }

// FP32 single-Gaussian form of window_loop: the optical-depth class is voted
// once per step for the wavefront (no per-channel branch), the maser check
// as in window_loop.  Thin steps whose window start is at most nch_reach
// (the band's channel count minus pass_reach) in every lane take the
// unmasked predicated passes: the channels from the window start to the
// reach are all updated, those past the cut with their true (negligible)
// profile values, and all stay inside the vector.
template <int LANES>
__device__ __forceinline__ void window_f32(float* __restrict__ I, int lane, int clo, int nwin, float x0, float ibs,
                                           float kl, float el, float& sj, float& sl, unsigned* __restrict__ maser,
                                           int nch_reach)
{
    float* __restrict__ rl = I + clo + lane;
    const float xl = fmaf((float)lane, ibs, x0);
    const float akl = fabsf(kl);
    const unsigned long long all_lanes = __builtin_amdgcn_read_exec();
    const unsigned long long thin = __builtin_amdgcn_ballot_w64(akl < 1e-3f);
    if ((thin & __builtin_amdgcn_ballot_w64(clo <= nch_reach)) == all_lanes) {
        window_passes_pred<LANES, 0, false>(rl, lane, nwin, xl, x0, ibs, 0.0f, kl, el, sj, sl);
    } else if (thin == all_lanes) {
        window_passes_f32<LANES, 0>(rl, lane, nwin, xl, x0, ibs, kl, el, sj, sl);
    } else if (__all(akl < 1e-2f)) {
        window_passes_f32<LANES, 1>(rl, lane, nwin, xl, x0, ibs, kl, el, sj, sl);
    } else {
        if (kl < (float)kMaserTauMin) *maser = 1u;
        window_passes_f32<LANES, 2>(rl, lane, nwin, xl, x0, ibs, kl, el, sj, sl);
    }
}

// With HF the component count picks, once per step (it is uniform), a loop
// whose profile sum is unrolled over exactly 1..4 components, or over 8 or
// all register components with zero-strength padding.
// nch_reach: see window_f32 (INT_MIN: never the unmasked passes).
template <int LANES, typename T, bool HF = false>
__device__ __forceinline__ void window_channels(T* __restrict__ I, int lane, int clo, int nwin, T x0, T ibs,
                                                T kl, T el, T& sj, T& sl, const HfRegs<T>* hf,
                                                unsigned* __restrict__ maser, int nch_reach = INT_MIN)
{
    if constexpr (!HF) {
        if constexpr (std::is_same<T, float>::value)
            window_f32<LANES>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, maser, nch_reach);
        else
            window_loop<LANES, T, 0>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, hf, maser);
    } else {
        constexpr int R = HfRegs<T>::kReg;
        const int n = hf->n;
        if (n == 1) window_loop<LANES, T, 1>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, hf, maser);
        else if (n == 2) window_loop<LANES, T, 2>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, hf, maser);
        else if (n == 3) window_loop<LANES, T, 3>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, hf, maser);
        else if (n == 4) window_loop<LANES, T, 4>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, hf, maser);
        else if (n <= 8 || R == 8) window_loop<LANES, T, 8>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, hf, maser);
        else window_loop<LANES, T, R>(I, lane, clo, nwin, x0, ibs, kl, el, sj, sl, hf, maser);
    }
}

}  // namespace

// The step length of a crossing-pattern record (see StepRec).
__device__ __forceinline__ float step_length(float log2_len) { return fast_exp2(log2_len); }
__device__ __forceinline__ double step_length(double len) { return len; }

template <typename T, int LANES, bool ACCUM, bool HF>
__global__ __launch_bounds__(256) void march3d_kernel(March3DArgs<T> p)
{
    using T2 = typename V2<T>::type;
    using T4 = typename V4<T>::type;
    const int rpb = blockDim.x / LANES;
    const int lane = threadIdx.x % LANES;
    const int rib = threadIdx.x / LANES;
    // Consecutive workgroups are dealt round-robin to the 8 XCDs; remap so that
    // each XCD walks a contiguous range of rays (neighbouring rays of one
    // direction share cells and hence L2 lines).
    int bid = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    // transitions vary fastest: the blocks of all transitions of one ray tile
    // run back to back on one XCD and share the tile's window and cell lines
    const int t = p.trans_offset + bid % p.ntr;
    bid /= p.ntr;
    const int q = bid / p.blocks_per_dir;
    const int r = (bid - q * p.blocks_per_dir) * rpb + rib;
    extern __shared__ unsigned char smem_raw[];
    StepRec<T>* __restrict__ sst = reinterpret_cast<StepRec<T>*>(smem_raw);
    T* __restrict__ I = reinterpret_cast<T*>(smem_raw + p.step_lds_bytes) + (size_t)rib * p.ich;

    const DirDev D = p.dirs[q];
    for (int i = threadIdx.x; i < D.nsteps; i += blockDim.x) sst[i] = p.steps[D.step0 + i];
    __syncthreads();
    // Rays past the end of the last tile run a copy of the last ray so that
    // every lane of the wavefront takes part in the queue flushes; their own
    // results are never written.
    const int rpw = 64 / LANES;                 // rays per wavefront
    const int r_first = r - (rib % rpw);        // first ray of this wavefront
    if (r_first >= p.rays_per_dir) return;      // the whole wavefront is past the end
    const bool ray_ok = r < p.rays_per_dir;
    const int rr = ray_ok ? r : p.rays_per_dir - 1;

    const int N = p.N;
    const int i0 = rr % N, j0 = rr / N;
    int ca = i0, cb = j0;
    int idx = D.start_off + i0 * D.sta + j0 * D.stb;
    const T Ibg = p.Ibg[t];
    // {khat, ehat} and {J, Lambda} are stored cell-major: [cell][transition]
    const int ts = p.ntr_total;
    const T4* __restrict__ win = p.win + (size_t)q * p.nc;
    const T2* __restrict__ ke = p.ke + t;
    T2* __restrict__ E = p.E ? p.E + (size_t)(t - p.trans_offset) * p.e_tstride + (size_t)D.step0 * p.rays_per_dir
                             : nullptr;
    const T aw = (T)D.aw;
    const int ns = D.nsteps;
    HfRegs<T> hfr;
    if constexpr (HF) hfr.load(p.hf + (size_t)t * p.hfk, p.hfk);
    for (int c = lane; c < p.nch; c += LANES) I[c] = Ibg;

    // Per-step partial sums {a len sum_c e_c I_c beta_c, a len sum_c e_c (1 - beta_c)}
    // are queued in LDS and written every LANES steps to E[step][ray] with
    // plain stores, one entry per lane of the wavefront (lanes with the same
    // step write neighbouring rays: contiguous bytes).  Stores and loads share
    // the memory counter, so writing every step would make each step wait for
    // the previous step's store; device-scope atomics would in addition be
    // executed in the memory fabric.  The per-cell sums are formed afterwards
    // by gather3d_kernel.
    T2* __restrict__ qw = reinterpret_cast<T2*>(smem_raw + p.queue_lds_offset) + (size_t)(rib - rib % rpw) * LANES;
    const int wl = threadIdx.x & 63;            // lane in the wavefront
    const int q_ray = wl % rpw, q_step = wl / rpw;
    int qn = 0, qs0 = 0;

    // The cell of step s + 1 follows from the step list alone, so its window
    // and {khat, ehat} loads are issued before step s is computed.
    StepRec<T> rec_n = sst[0];
    bool restart_n = false;
    if (rec_n.flags & 1) idx += D.stride_m;
    if (rec_n.flags & 2) move_transverse(ca, idx, D.sa, D.sta, N, restart_n);
    if (rec_n.flags & 4) move_transverse(cb, idx, D.sb, D.stb, N, restart_n);
    T4 wv_n = win[idx];
    T2 kv_n = ke[(size_t)idx * ts];
    for (int s = 0; s < ns; ++s) {
        const StepRec<T> rec = rec_n;
        const bool restart = restart_n;
        const T4 wv = wv_n;
        const T2 kv = kv_n;
        if (s + 1 < ns) {
            rec_n = sst[s + 1];
            restart_n = false;
            if (rec_n.flags & 1) idx += D.stride_m;
            if (rec_n.flags & 2) move_transverse(ca, idx, D.sa, D.sta, N, restart_n);
            if (rec_n.flags & 4) move_transverse(cb, idx, D.sb, D.stb, N, restart_n);
            wv_n = win[idx];
            kv_n = ke[(size_t)idx * ts];
        }
        if (restart) {
            // Side exit: the ray re-enters on the opposite face carrying the
            // background again (Sect. 2.2).
            for (int c = lane; c < p.nch; c += LANES) I[c] = Ibg;
        }
        const int clo = as_int(wv.z);
        const int nwin = as_int(wv.w);
        const T len = step_length(rec.len);
        const T kl = kv.x * len;          // tau at the line centre
        const T el = kv.y * len;
        T sj = 0, sl = 0;
        window_channels<LANES, T, HF>(I, lane, clo, nwin, wv.x, wv.y, kl, el, sj, sl, &hfr, p.maser);
        if (ACCUM) {
            // every lane forms the weighted sums (the wavefront issues them
            // either way); only the group's last lane, which holds the
            // total, stores them
            const T wgt = aw * len;
            T2 v;
            v.x = wgt * group_sum<LANES>(sj);
            v.y = wgt * group_sum<LANES>(sl);
            keep_here(v.x);
            keep_here(v.y);
            if (lane == LANES - 1) qw[qn * rpw + (rib % rpw)] = v;
            ++qn;
            if (qn == LANES || s == ns - 1) {
                const int rq = r_first + q_ray;
                if (q_step < qn && rq < p.rays_per_dir)
                    E[(size_t)(qs0 + q_step) * p.rays_per_dir + rq] = qw[q_step * rpw + q_ray];
                qs0 += qn;
                qn = 0;
            }
        }
    }
    if (!ACCUM && p.Iout && ray_ok) {
        T* out = p.Iout + ((size_t)q * p.rays_per_dir + r) * p.nch;
        for (int c = lane; c < p.nch; c += LANES) out[c] = I[c];
    }
}

namespace {

// The lane group's passes over one step's window, FP32 single Gaussian,
// with the step length folded into the profile, e_c' = e_c len =
// exp2(log2 len - x^2): then tau = khat e_c', and the emission ehat e_c' beta
// and both sums come out multiplied by the length.  No branch per channel:
// the first NU channels of every lane are computed whether they lie in the
// window or not.  With MASK the profile of a channel outside the window is
// set to 0, which leaves its intensity as it was (I + 0 (ehat - khat I) = I)
// and adds nothing to the sums; the channel vector must then be followed by
// at least NU LANES words of its own (finite) padding, so that these writes
// never reach another ray's vector.  Without MASK (allowed when the window
// start plus NU LANES stays inside the band) the extra channels are updated
// with their true profile values, below e^-25 of the peak past the cut.
template <int LANES, int CLS, bool MASK>
__device__ __forceinline__ void window_passes_pred(float* __restrict__ rl, int lane, int nwin, float xl,
                                                   float x0, float ibs, float l2len, float kh, float eh, float& sj,
                                                   float& sl)
{
    constexpr int NU = LANES >= 64 ? 1 : (LANES >= 32 ? 2 : 4);
    float Iv[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) Iv[i] = rl[i * LANES];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const float xs = i == 0 ? xl : fmaf((float)(i * LANES), ibs, xl);
        const float e = fast_exp2(fmaf(-xs, xs, l2len));
        // MASK = false: every one of the NU LANES channels lies in the band,
        // and those past the window's cut take their (negligible) profile
        // values, as the channels of a march without a cut would
        const float ec = !MASK || lane + i * LANES < nwin ? e : 0.0f;
        const float omb = omb_class<CLS>(kh * ec);
        const float u = fmaf(-ec, omb, ec);
        sj = fmaf(Iv[i], u, sj);
        sl = fmaf(ec, omb, sl);
        rl[i * LANES] = fmaf(u, fmaf(-kh, Iv[i], eh), Iv[i]);
    }
    for (int j = lane + NU * LANES; j < nwin; j += LANES) {
        const float xs = fmaf((float)j, ibs, x0);
        const float ec = fast_exp2(fmaf(-xs, xs, l2len));
        channel_update(rl + (j - lane), ec, omb_class<CLS>(kh * ec), kh, eh, sj, sl);
    }
}

// Words of padding after each channel vector of march3d_f32_kernel: the
// predicated passes' reach (NU LANES), rounded so that the vectors of
// consecutive rays start 8 banks apart.
__host__ __device__ constexpr int f32_vec_gap(int lanes)
{
    return (lanes >= 64 ? 1 : (lanes >= 32 ? 2 : 4)) * lanes + 8;
}

// One transverse move with periodic re-entry (as move_transverse), the
// wrap-around corrections held in vector registers.
__device__ __forceinline__ void move_wrap(int& c, int& idx, int s, int wrap_c, int d_step, int d_wrap, int N,
                                          bool& restart)
{
    c += s;
    const bool wrap = (unsigned)c >= (unsigned)N;
    c -= wrap ? wrap_c : 0;
    idx += wrap ? d_wrap : d_step;
    restart |= wrap;
}

// A value the compiler keeps in a vector register (so that selects against
// it need no per-use copy from a scalar register).
__device__ __forceinline__ int in_vgpr(int v)
{
    int r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
    return r;
}

}  // namespace

// The FP32 single-Gaussian regular-grid march (the same rays, steps, sums and
// outputs as march3d_kernel<float, LANES, ACCUM, false>), arranged for
// instruction count:
//  * step records carry log2 of the length, absorbed by the profile exponent
//    (window_passes_pred); the optical-depth class of a step is voted on
//    |khat| times the direction's longest step, a bound on |tau|;
//  * the channel passes are predicated rather than branched per channel;
//  * the ray weight |d_m| multiplies the queued sums when they are written,
//    and 8- and 16-lane groups queue them in registers;
//  * the cell data of the coming steps are loaded into a ring of register
//    sets, several steps ahead, so no prefetched value is copied, and every
//    turn of the ring issues the same loads, so each step waits for its own
//    data only;
//  * the transverse wrap-around corrections sit in vector registers.
template <int LANES, bool ACCUM, bool OFF32>
__global__ __launch_bounds__(256) void march3d_f32_kernel(March3DArgs<float> p)
{
    const int rpb = blockDim.x / LANES;
    const int lane = threadIdx.x % LANES;
    const int rib = threadIdx.x / LANES;
    int bid = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    const int t = p.trans_offset + bid % p.ntr;
    bid /= p.ntr;
    const int q = bid / p.blocks_per_dir;
    const int r = (bid - q * p.blocks_per_dir) * rpb + rib;
    extern __shared__ unsigned char smem_raw[];
    StepRec<float>* __restrict__ sst = reinterpret_cast<StepRec<float>*>(smem_raw);
    float* __restrict__ I = reinterpret_cast<float*>(smem_raw + p.step_lds_bytes) + (size_t)rib * p.ich;

    const DirDev D = p.dirs[q];
    for (int i = threadIdx.x; i < D.nsteps; i += blockDim.x) sst[i] = p.steps[D.step0 + i];
    __syncthreads();
    const int rpw = 64 / LANES;
    const int r_first = r - (rib % rpw);
    if (r_first >= p.rays_per_dir) return;
    const bool ray_ok = r < p.rays_per_dir;
    const int rr = ray_ok ? r : p.rays_per_dir - 1;

    const int N = p.N;
    const int i0 = rr % N, j0 = rr / N;
    int ca = i0, cb = j0;
    int idx = D.start_off + i0 * D.sta + j0 * D.stb;
    const int wrap_a = in_vgpr(D.sa * N), wrap_b = in_vgpr(D.sb * N);
    const int da = in_vgpr(D.sa * D.sta), db = in_vgpr(D.sb * D.stb);
    const int dwa = in_vgpr(-D.sa * (N - 1) * D.sta), dwb = in_vgpr(-D.sb * (N - 1) * D.stb);
    const float Ibg = p.Ibg[t];
    // channel c of the ray lives at I[c - base] (base 0 without a span table)
    const int base = p.rbase ? p.rbase[(size_t)q * p.rays_per_dir + rr] : 0;
    const int ts = p.ntr_total;
    const unsigned kv_bytes = (unsigned)ts * (unsigned)sizeof(float2);
    const float4* __restrict__ win = p.win + (size_t)q * p.nc;
    const float2* __restrict__ ke = p.ke + t;
    float2* __restrict__ E = p.E ? p.E + (size_t)(t - p.trans_offset) * p.e_tstride + (size_t)D.step0 * p.rays_per_dir
                                 : nullptr;
    const float aw = (float)D.aw;
    const float kthin0 = (float)(1.0e-3 / D.maxlen);     // |khat| below: every |tau| < 1e-3
    const float kthin1 = (float)(1.0e-2 / D.maxlen);
    // channels one lane group's unrolled passes reach from the window start
    constexpr int kReach = (LANES >= 64 ? 1 : (LANES >= 32 ? 2 : 4)) * LANES;
    const int nch_reach = p.nch - kReach;
    const int ns = D.nsteps;
    // the padding after the vector is written too: the predicated passes
    // read it and must find finite values there
    for (int c = lane; c < p.ich; c += LANES) I[c] = Ibg;

    // Per-step sums {len sum_c e_c I_c beta_c, len sum_c e_c (1 - beta_c)}
    // wait in registers (lane k of a group holds the k-th step since the
    // last write; 8- and 16-lane group sums end in every lane of the group)
    // or, for wider groups, in an LDS queue; every LANES steps they are
    // written to E[step][ray] with the ray weight, rays of one step side by
    // side.
    constexpr bool kRegQueue = LANES <= 16;
    // 8-lane groups that accumulate keep instead each lane's own partial sums
    // of 8 consecutive steps and reduce-scatter them once per 8 steps (lane k
    // of a group then holds step k's totals): no per-step reduction or queue.
    constexpr bool kT8 = ACCUM && LANES == 8;
    float2* __restrict__ qw = reinterpret_cast<float2*>(smem_raw + p.queue_lds_offset) + (size_t)(rib - rib % rpw) * LANES;
    const int wl = threadIdx.x & 63;
    const int q_ray = wl % rpw, q_step = wl / rpw;
    int qn = 0, qs0 = 0;
    float qx = 0.0f, qy = 0.0f;

    // The cell data of step s are loaded while earlier steps are computed.
    // Past the last step the ray stays in its last cell and that cell's data
    // are loaded again (never used): every fetch issues the same two loads,
    // so the waits before a step can count the loads issued after its own
    // instead of waiting for all of them.
    // The step records are read from LDS 64 at a time, one per lane of the
    // wavefront, and each step takes its own with a lane read (no LDS access
    // and no wait per step).
    // (The empty asm uses make the read complete where it is issued rather
    // than before every later lane read.)
    int rb = 0;
    StepRec<float> vrec = sst[wl < ns ? wl : ns - 1];
    keep_here(vrec.len);
    keep_here(vrec.flags);
    auto fetch = [&](int s, float& l2len, bool& restart, float4& wv, float2& kv) {
        const bool live = s < ns;
        const int si = live ? s : ns - 1;
        if (si - rb >= 64) {
            rb += 64;
            vrec = sst[rb + wl < ns ? rb + wl : ns - 1];
            keep_here(vrec.len);
            keep_here(vrec.flags);
        }
        const int flags = __builtin_amdgcn_readlane(vrec.flags, si - rb);
        restart = false;
        if (live) {
            if (flags & 1) idx += D.stride_m;
            if (flags & 2) move_wrap(ca, idx, D.sa, wrap_a, da, dwa, N, restart);
            if (flags & 4) move_wrap(cb, idx, D.sb, wrap_b, db, dwb, N, restart);
        }
        l2len = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vrec.len), si - rb));
        if constexpr (OFF32) {
            // byte offsets below 2^32 from the uniform bases of the two tables
            // (the launch checks the sizes), the cell index below 2^24
            wv = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(win) + ((unsigned)idx << 4));
            // (the masks are no-ops that let the multiply be a 24-bit one)
            kv = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(ke) +
                                                  (((unsigned)idx & 0xFFFFFFu) * (kv_bytes & 0xFFFFFFu)));
        } else {
            wv = win[(unsigned)idx];
            kv = ke[(size_t)(unsigned)idx * (unsigned)ts];
        }
    };
    auto step = [&](int s, float l2len, bool restart, const float4& wv, const float2& kv, float& pj, float& pl) {
        if (restart) {
            // side exit: re-entry on the opposite face with the background (Sect. 2.2)
            for (int c = lane; c < p.ich; c += LANES) I[c] = Ibg;
        }
        const int clo = as_int(wv.z);
        const int nwin = as_int(wv.w);
        float* __restrict__ rl = I + (clo - base) + lane;
        const float xl = fmaf((float)lane, wv.y, wv.x);
        const float akh = fabsf(kv.x);
        // lane masks of the class tests, combined as masks (the ballot of a
        // combined condition would be rebuilt from a lane value)
        const unsigned long long all_lanes = __builtin_amdgcn_read_exec();
        const unsigned long long in_band = __builtin_amdgcn_ballot_w64(clo <= nch_reach);
        float sj = 0.0f, sl = 0.0f;
        if ((__builtin_amdgcn_ballot_w64(akh < kthin0) & in_band) == all_lanes) {
            window_passes_pred<LANES, 0, false>(rl, lane, nwin, xl, wv.x, wv.y, l2len, kv.x, kv.y, sj, sl);
        } else if (__builtin_amdgcn_ballot_w64(akh < kthin0) == all_lanes) {
            window_passes_pred<LANES, 0, true>(rl, lane, nwin, xl, wv.x, wv.y, l2len, kv.x, kv.y, sj, sl);
        } else if (__builtin_amdgcn_ballot_w64(akh < kthin1) == all_lanes) {
            window_passes_pred<LANES, 1, true>(rl, lane, nwin, xl, wv.x, wv.y, l2len, kv.x, kv.y, sj, sl);
        } else {
            if (kv.x * fast_exp2(l2len) < (float)kMaserTauMin) *p.maser = 1u;
            window_passes_pred<LANES, 2, true>(rl, lane, nwin, xl, wv.x, wv.y, l2len, kv.x, kv.y, sj, sl);
        }
        if constexpr (kT8) {
            pj = sj;
            pl = sl;
        } else if (ACCUM) {
            const float tx = group_sum<LANES>(sj);
            const float ty = group_sum<LANES>(sl);
            if constexpr (kRegQueue) {
                const bool mine = lane == qn;
                qx = mine ? tx : qx;
                qy = mine ? ty : qy;
                ++qn;
                if (qn == LANES || s == ns - 1) {
                    if (lane < qn && ray_ok)
                        E[(size_t)(qs0 + lane) * p.rays_per_dir + r] = make_float2(qx * aw, qy * aw);
                    qs0 += qn;
                    qn = 0;
                }
            } else {
                float2 v;
                v.x = tx;
                v.y = ty;
                keep_here(v.x);
                keep_here(v.y);
                if (lane == LANES - 1) qw[qn * rpw + (rib % rpw)] = v;
                ++qn;
                if (qn == LANES || s == ns - 1) {
                    const int rq = r_first + q_ray;
                    if (q_step < qn && rq < p.rays_per_dir) {
                        float2 o = qw[q_step * rpw + q_ray];
                        o.x *= aw;
                        o.y *= aw;
                        E[(size_t)(qs0 + q_step) * p.rays_per_dir + rq] = o;
                    }
                    qs0 += qn;
                    qn = 0;
                }
            }
        }
    };

    // a ring of kPrefetch register sets: set i holds step s0 + i; once that
    // step is done the set takes step s0 + i + kPrefetch, so each step's cell
    // loads are issued kPrefetch - 1 steps of work before they are used.
    // Whole turns of the ring run without conditions; the last ns mod
    // kPrefetch steps take the sets in order, shifting the ring.
    constexpr int kPrefetch = 4;
    float l2r[kPrefetch];
    bool rsr[kPrefetch];
    float4 wvr[kPrefetch];
    float2 kvr[kPrefetch];
    auto shift_ring = [&]() {
#pragma unroll
        for (int i = 0; i + 1 < kPrefetch; ++i) {
            l2r[i] = l2r[i + 1];
            rsr[i] = rsr[i + 1];
            wvr[i] = wvr[i + 1];
            kvr[i] = kvr[i + 1];
        }
    };
    if (ns > 0) {
#pragma unroll
        for (int i = 0; i < kPrefetch; ++i) fetch(i, l2r[i], rsr[i], wvr[i], kvr[i]);
        int s0 = 0;
        float pj[8], pl[8];
        if constexpr (kT8) {
            // two turns of the ring per 8 steps, then the sums of the 8 steps
            for (; s0 + 8 <= ns; s0 += 8) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    constexpr int M = kPrefetch - 1;
                    step(s0 + i, l2r[i & M], rsr[i & M], wvr[i & M], kvr[i & M], pj[i], pl[i]);
                    fetch(s0 + i + kPrefetch, l2r[i & M], rsr[i & M], wvr[i & M], kvr[i & M]);
                }
                const float tj = reduce_scatter8(pj, lane);
                const float tl = reduce_scatter8(pl, lane);
                if (ray_ok) E[(size_t)(s0 + lane) * p.rays_per_dir + r] = make_float2(tj * aw, tl * aw);
            }
            // the last ns mod 8 steps one at a time, each stored at once
            for (; s0 < ns; ++s0) {
                step(s0, l2r[0], rsr[0], wvr[0], kvr[0], pj[0], pl[0]);
                const float tj = group_sum<LANES>(pj[0]);
                const float tl = group_sum<LANES>(pl[0]);
                if (lane == 0 && ray_ok) E[(size_t)s0 * p.rays_per_dir + r] = make_float2(tj * aw, tl * aw);
                shift_ring();
                fetch(s0 + kPrefetch, l2r[kPrefetch - 1], rsr[kPrefetch - 1], wvr[kPrefetch - 1],
                      kvr[kPrefetch - 1]);
            }
        } else {
            for (; s0 + kPrefetch <= ns; s0 += kPrefetch) {
#pragma unroll
                for (int i = 0; i < kPrefetch; ++i) {
                    step(s0 + i, l2r[i], rsr[i], wvr[i], kvr[i], pj[i], pl[i]);
                    fetch(s0 + i + kPrefetch, l2r[i], rsr[i], wvr[i], kvr[i]);
                }
            }
            for (; s0 < ns; ++s0) {
                step(s0, l2r[0], rsr[0], wvr[0], kvr[0], pj[0], pl[0]);
                shift_ring();
            }
        }
    }
    if (!ACCUM && p.Iout && ray_ok) {
        float* out = p.Iout + ((size_t)q * p.rays_per_dir + r) * p.nch;
        for (int c = lane; c < p.nch; c += LANES) out[c] = I[c];
    }
}

// The channel span of every ray of a direction (grid y = direction, one
// thread per ray): the ray's cells as march3d steps through them, the lowest
// first window channel and the highest window start plus max(window, reach).
__global__ __launch_bounds__(256) void ray_span_kernel(March3DArgs<float> p, int reach, int* __restrict__ rbase,
                                                       int* __restrict__ wmax)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (r >= p.rays_per_dir) return;
    const DirDev D = p.dirs[q];
    const int N = p.N;
    int ca = r % N, cb = r / N;
    int idx = D.start_off + ca * D.sta + cb * D.stb;
    const float4* __restrict__ win = p.win + (size_t)q * p.nc;
    int lo = INT_MAX, hi = INT_MIN;
    bool restart = false;
    for (int s = 0; s < D.nsteps; ++s) {
        const StepRec<float> rec = p.steps[D.step0 + s];
        if (rec.flags & 1) idx += D.stride_m;
        if (rec.flags & 2) move_transverse(ca, idx, D.sa, D.sta, N, restart);
        if (rec.flags & 4) move_transverse(cb, idx, D.sb, D.stb, N, restart);
        const float4 wv = win[idx];
        const int clo = as_int(wv.z), nwin = as_int(wv.w);
        lo = clo < lo ? clo : lo;
        const int top = clo + (nwin > reach ? nwin : reach);
        hi = top > hi ? top : hi;
    }
    if (lo > hi) lo = hi = 0;
    rbase[(size_t)q * p.rays_per_dir + r] = lo;
    atomicMax(wmax, hi - lo);
}

// Sum, for every cell and transition, the per-step partial sums of all rays
// of the directions of one main axis that crossed the cell.  Thread = cell;
// the cell's transverse coordinates (ia, ib) vary fastest so that neighbouring
// threads read neighbouring rays.  For a step s of direction q the ray that was
// in the cell started at ((ia - sa na_s) mod N, (ib - sb nb_s) mod N).
template <typename T, int TILE>
__global__ __launch_bounds__(256) void gather3d_kernel(Gather3DArgs<T> p)
{
    using T2 = typename V2<T>::type;
    const int N = p.N;
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= N * N) return;
    const int ia = pos % N, ib = pos / N;
    const int cm = blockIdx.y;
    // up to TILE transitions per thread: their loads of one step are
    // independent, and the cell's accumulator row is updated in one piece
    const int t0 = blockIdx.z * TILE;
    const int nt = p.ntr - t0 < TILE ? p.ntr - t0 : TILE;
    const int NN = N * N;
    const T2* __restrict__ E = p.E + (size_t)t0 * p.e_tstride;
    double sj[TILE], sl[TILE];
#pragma unroll
    for (int q = 0; q < TILE; ++q) sj[q] = sl[q] = 0.0;
    for (int k = 0; k < p.nq; ++k) {
        const DirDev& D = p.dirs[p.qlist[k]];
        const int l = D.fwd ? cm : N - 1 - cm;
        const int s0 = p.lstart[D.lstart0 + l], s1 = p.lstart[D.lstart0 + l + 1];
        for (int s = s0; s < s1; ++s) {
            const int2 mv = p.moves[D.step0 + s];
            int i0 = ia - D.sa * mv.x;
            int j0 = ib - D.sb * mv.y;
            i0 += i0 < 0 ? N : 0;
            i0 -= i0 >= N ? N : 0;
            j0 += j0 < 0 ? N : 0;
            j0 -= j0 >= N ? N : 0;
            const size_t off = (size_t)(D.step0 + s) * NN + j0 * N + i0;
            // all loads of the step issued before any is used; columns past
            // the launch's transitions re-read the last one and are not stored
            T2 e[TILE];
#pragma unroll
            for (int q = 0; q < TILE; ++q) e[q] = E[(size_t)(q < nt ? q : nt - 1) * p.e_tstride + off];
#pragma unroll
            for (int q = 0; q < TILE; ++q) {
                sj[q] += (double)e[q].x;
                sl[q] += (double)e[q].y;
            }
        }
    }
    const size_t idx = (size_t)ia * p.st_a + (size_t)ib * p.st_b + (size_t)cm * p.st_m;
    double2* a = p.acc + idx * p.ntr_total + p.trans_offset + t0;
    // the first axis group's gather writes the sums (adding to the zeros it
    // replaces would give the same bits), the others add theirs
#pragma unroll
    for (int q = 0; q < TILE; ++q) {
        if (q < nt) {
            double2 v = p.overwrite ? make_double2(0.0, 0.0) : a[q];
            v.x += sj[q];
            v.y += sl[q];
            a[q] = v;
        }
    }
}

// Per-cell sums of the octree march's per-step partial sums, one thread per
// cell and all transitions of the launch: FP64 sums over the cell's steps
// (listed by the host), written to the accumulators.  TILE transitions of a
// step's row are read with unconditional wide loads (FP32 rows are 16-byte
// aligned), all issued before any is used; columns past the launch's
// transitions are read but never stored (E carries slack past its last row).
template <typename T, int TILE>
__global__ __launch_bounds__(256) void gather_oct_kernel(GatherOctArgs<T> p)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.nc) return;
    const long long a = p.cell_off[k], b = p.cell_off[k + 1];
    double2* acc = p.acc + (size_t)k * p.ntr_total + p.trans_offset;
    for (int t0 = 0; t0 < p.ntr; t0 += TILE) {
        double sj[TILE], sl[TILE];
#pragma unroll
        for (int q = 0; q < TILE; ++q) sj[q] = sl[q] = 0.0;
        // A cell's steps are listed in step order, which is direction-major:
        // the threads of a wavefront take the steps of one direction at a
        // time, so that neighbouring cells read the rows of a ray's
        // consecutive steps (neighbouring rows) together.  The next step's
        // index is loaded with the current step's row.
        long long i = a;
        unsigned idx_n = i < b ? p.cell_steps[i] : 0xFFFFFFFFu;
        for (int d = 0; d < p.n_dir; ++d) {
            const unsigned end = p.dir_off[d + 1];
            while (idx_n < end) {
                const unsigned idx = idx_n;
                ++i;
                idx_n = i < b ? p.cell_steps[i] : 0xFFFFFFFFu;
                const typename V2<T>::type* e = p.E + (size_t)idx * p.estride + t0;
                if constexpr (sizeof(T) == 4) {
                    const float4* __restrict__ e4 = reinterpret_cast<const float4*>(e);
                    float4 v[TILE / 2];
#pragma unroll
                    for (int q = 0; q < TILE / 2; ++q) v[q] = e4[q];
#pragma unroll
                    for (int q = 0; q < TILE / 2; ++q) {
                        sj[2 * q] += (double)v[q].x;
                        sl[2 * q] += (double)v[q].y;
                        sj[2 * q + 1] += (double)v[q].z;
                        sl[2 * q + 1] += (double)v[q].w;
                    }
                } else {
                    typename V2<T>::type v[TILE];
#pragma unroll
                    for (int q = 0; q < TILE; ++q) v[q] = e[q];
#pragma unroll
                    for (int q = 0; q < TILE; ++q) {
                        sj[q] += (double)v[q].x;
                        sl[q] += (double)v[q].y;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < TILE; ++q)
            if (t0 + q < p.ntr) acc[t0 + q] = make_double2(sj[q], sl[q]);
    }
}

// ---------------------------------------------------------------- octree march
namespace {

// Copies 16-byte pieces qa .. qb - 1 of a channel vector between LDS and
// device memory (both vectors 16-byte aligned and padded to whole pieces):
// each lane issues all of its loads of a round before its first store, so a
// copy costs one memory round trip per 4 LANES pieces rather than one per
// element.
template <int LANES, typename T>
__device__ __forceinline__ void copy_pieces(T* __restrict__ dst, const T* __restrict__ src, int qa, int qb, int lane)
{
    const int4* __restrict__ s4 = reinterpret_cast<const int4*>(src);
    int4* __restrict__ d4 = reinterpret_cast<int4*>(dst);
    for (int q0 = qa + lane; q0 < qb; q0 += 4 * LANES) {
        // lanes past the end load the last piece again (always in range) and
        // store nothing
        const int q1 = q0 + LANES, q2 = q0 + 2 * LANES, q3 = q0 + 3 * LANES;
        const int4 v0 = s4[q0];
        const int4 v1 = s4[q1 < qb ? q1 : qb - 1];
        const int4 v2 = s4[q2 < qb ? q2 : qb - 1];
        const int4 v3 = s4[q3 < qb ? q3 : qb - 1];
        d4[q0] = v0;
        if (q1 < qb) d4[q1] = v1;
        if (q2 < qb) d4[q2] = v2;
        if (q3 < qb) d4[q3] = v3;
    }
}

// Per-group stack of channel spans [lo, hi) in registers: entry e lives in
// lane e % LANES, slot e / LANES, as lo | hi << 16 (channel counts are at
// most 4096), so that a push or a read selects among SLOTS words once.
template <int LANES, int SLOTS>
struct SpanStack {
    int v[SLOTS];
    __device__ __forceinline__ void set(int e, int lane, int l, int h)
    {
        const int sel = lane == e % LANES ? e / LANES : -1;
        const int w = l | (h << 16);
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) v[s] = s == sel ? w : v[s];
    }
    // e < SLOTS * LANES: the slot is picked by a binary tree of selects on
    // the bits of e / LANES
    __device__ __forceinline__ void get(int e, int& l, int& h) const
    {
        static_assert((SLOTS & (SLOTS - 1)) == 0, "SLOTS is a power of two");
        const int sl = e / LANES;
        int a[SLOTS];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) a[s] = v[s];
#pragma unroll
        for (int k = 0, n = SLOTS; n > 1; ++k, n /= 2) {
            const bool b = (sl >> k) & 1;
#pragma unroll
            for (int j = 0; j < n / 2; ++j) a[j] = b ? a[2 * j + 1] : a[2 * j];
        }
        const int r = __shfl(a[0], e % LANES, LANES);
        l = r & 0xFFFF;
        h = r >> 16;
    }
};

}  // namespace

// Persistent lane groups (8 or 16 lanes) take work units (one root line's rays for one
// transition) from a global counter, largest units first.  Each unit replays
// its host-built step list: a record names the leaf and the step length and
// says how the ray's intensity starts (continue, background, or the top saved
// vector, Sect. 2.2: new rays copy the intensity of the ray that creates
// them) and whether to save the incoming intensity first.  Saved vectors live
// in a per-group stack in device memory.  The step itself is the regular
// grid's: channel window of the (direction, leaf) pair, I e^-tau + S(1 -
// e^-tau); with accumulation, the step's absorbed-count and Lambda sums go to
// the per-step buffer E (required then), summed per cell by gather_oct_kernel.
template <typename T, int LANES, bool ACCUM, bool HF>
__global__ __launch_bounds__(256) void march_oct_kernel(OctMarchArgs<T> p)
{
    using T2 = typename V2<T>::type;
    using T4 = typename V4<T>::type;
    const int lane = threadIdx.x % LANES;
    const int grp = threadIdx.x / LANES;
    const size_t gid = (size_t)blockIdx.x * (blockDim.x / LANES) + grp;
    extern __shared__ unsigned char smem_raw[];
    using T2q = typename V2<T>::type;
    T* __restrict__ I = reinterpret_cast<T*>(smem_raw) + (size_t)grp * p.ich;
    // per-step sums queued in LDS and written LANES at a time (plain stores,
    // gathered per cell afterwards): no device atomics in the march
    // FP32 with 8 lanes queues the two quad sums of each step of a chunk
    // (the group sum and the step weight are finished once per chunk), other
    // instances the weighted group sum
    constexpr bool kQuad = sizeof(T) == 4 && LANES == 8;
    constexpr int kQueue = kQuad ? 2 * LANES : LANES;
    T2q* __restrict__ queue = reinterpret_cast<T2q*>(smem_raw + (size_t)(blockDim.x / LANES) * p.ich * sizeof(T)) +
                              (size_t)grp * kQueue;
    T* __restrict__ stk = p.stack + gid * (size_t)p.depth * p.ich;
    constexpr int kPer = 16 / (int)sizeof(T);   // channels per 16-byte piece
    constexpr int kSpanSlots = 8;
    SpanStack<LANES, kSpanSlots> spans;
    // deeper stacks than the span registers hold copy whole vectors
    const bool use_spans = p.depth <= kSpanSlots * LANES;
    const int nch_reach = p.nch - pass_reach<LANES>();
    int lo = 0, hi = p.nch;                       // LDS contents unknown: a full reset first
    // Work units start only at chunk boundaries, which all groups of the
    // wavefront reach together: the records of a chunk are loaded (and the
    // per-step sums flushed) once per LANES steps for the whole wavefront
    // instead of whenever any of its groups crosses a boundary.  A group whose
    // unit ends inside a chunk idles to the boundary (units are thousands of
    // steps long).
    bool have = false, done = false;
    OctTreeRec tr{};
    int t = 0, s = 0, qn = 0, qs0 = 0, sp = -1;
    const T4* __restrict__ win = p.win;
    const T2* __restrict__ ke = p.ke;
    const uint2* __restrict__ rec = p.steps;
    const double* __restrict__ rec64 = nullptr;
    T2q* __restrict__ Et = nullptr;
    T aw = 0, Ibg = 0;
    HfRegs<T> hfr;
    // Records arrive LANES at a time, one per lane, and each lane also loads
    // the window and {khat, ehat} of its record's cell: the cell data of a
    // whole chunk are fetched in parallel instead of one dependent load per
    // step (the cells of a ray's steps are scattered over the tree), then
    // broadcast step by step with shuffles.  The next chunk's cell data are
    // loaded while the current one is processed, and the records of the chunk
    // after it one chunk earlier still, so that the cell loads never wait on
    // their record.
    uint2 mine{}, nx{}, nr{};
    double mine64 = 0.0, nx64 = 0.0, nr64 = 0.0;
    T4 mywv{}, nxwv{};
    T2 mykv{}, nxkv{};
    // FP32: {khat, ehat} times the step length of the lane's record, formed
    // once per chunk in the lane that loaded it and broadcast per step
    T2 mytau{};
    auto load_rec = [&](int s0, uint2& r, double& r64) {
        const int si = s0 + lane < tr.n ? s0 + lane : s0;
        r = rec[si];
        if (sizeof(T) == 8 && rec64) r64 = rec64[si];
    };
    auto load_cells = [&](const uint2& r, T4& wvv, T2& kvv) {
        const unsigned c = r.x & kOctCellMask;
        wvv = win[c];
        kvv = ke[(size_t)c * p.ntr_total];
    };
    // byte address of the group's first lane for the record broadcasts
    const int bp_base = (int)(threadIdx.x & ~(unsigned)(LANES - 1)) << 2;
    auto bcast = [&](auto v, int k) {
        using V = decltype(v);
        return __builtin_bit_cast(V, __builtin_amdgcn_ds_bpermute(bp_base + (k << 2), __builtin_bit_cast(int, v)));
    };
    for (;;) {
        if (have) {
            // a chunk boundary inside the unit (s is a positive multiple of LANES)
            mine = nx;
            mine64 = nx64;
            mywv = nxwv;
            mykv = nxkv;
            if (s + LANES < tr.n) {
                nx = nr;
                nx64 = nr64;
                load_cells(nx, nxwv, nxkv);
            }
            if (s + 2 * LANES < tr.n) load_rec(s + 2 * LANES, nr, nr64);
        } else if (!done) {
            unsigned long long item = 0;
            if (lane == 0) item = atomicAdd(p.counter, 1ull);
            item = __shfl(item, 0, LANES);
            if (item >= (unsigned long long)p.n_items) {
                done = true;
            } else {
                have = true;
                lo = 0;                           // a new transition's background everywhere
                hi = p.nch;
                const long long tree = (long long)(item / (unsigned long long)p.ntr);
                t = p.trans_offset + (int)(item % (unsigned long long)p.ntr);
                tr = p.trees[tree];
                win = p.win + (size_t)tr.q * p.nc;
                ke = p.ke + t;
                rec = p.steps + tr.off;
                aw = (T)p.aw[tr.q];
                Ibg = p.Ibg[t];
                if constexpr (HF) hfr.load(p.hf + (size_t)t * p.hfk, p.hfk);
                rec64 = p.len64 ? p.len64 + tr.off : nullptr;
                Et = p.E ? p.E + (size_t)tr.off * p.estride + (t - p.trans_offset) : nullptr;
                s = 0;
                qn = 0;
                qs0 = 0;
                sp = -1;
                load_rec(0, mine, mine64);
                load_cells(mine, mywv, mykv);
                if (LANES < tr.n) {
                    load_rec(LANES, nx, nx64);
                    load_cells(nx, nxwv, nxkv);
                }
                if (2 * LANES < tr.n) load_rec(2 * LANES, nr, nr64);
            }
        }
        // every group without a unit has found the counter exhausted
        if (__all(!have)) break;
        if constexpr (sizeof(T) == 4) {
            const T ln = __uint_as_float(mine.y);
            mytau = T2{mykv.x * ln, mykv.y * ln};
            // formed here, not recomputed before each broadcast
            keep_here(mytau.x);
            keep_here(mytau.y);
        }
        const int s_chunk = s;
        for (int k = 0; k < LANES; ++k) {
            if (!have || s >= tr.n) continue;
            const unsigned w0 = bcast(mine.x, k);
            // the step length enters the optical depths (formed per chunk for
            // FP32) and, without the per-chunk weights, the step weight
            T len = 0;
            if (sizeof(T) == 8 || !kQuad) len = (T)__uint_as_float(bcast(mine.y, k));
            if (sizeof(T) == 8 && rec64) len = (T)__shfl(mine64, k, LANES);
            T4 wv;
            if constexpr (sizeof(T) == 4) {
                wv.x = bcast(mywv.x, k);
                wv.y = bcast(mywv.y, k);
                wv.z = bcast(mywv.z, k);
                wv.w = bcast(mywv.w, k);
            } else {
                wv.x = __shfl(mywv.x, k, LANES);
                wv.y = __shfl(mywv.y, k, LANES);
                wv.z = __shfl(mywv.z, k, LANES);
                wv.w = __shfl(mywv.w, k, LANES);
            }
            T kl, el;
            if constexpr (sizeof(T) == 4) {
                kl = bcast(mytau.x, k);
                el = bcast(mytau.y, k);
            } else {
                kl = __shfl(mykv.x, k, LANES) * len;
                el = __shfl(mykv.y, k, LANES) * len;
            }
            // Most steps continue their ray and save nothing (a record's word
            // is then below kOctSave): one vote over the wavefront skips the
            // start and save handling.
            if (__builtin_amdgcn_ballot_w64(w0 >= kOctSave) != 0ull) {
                const unsigned mode = w0 >> kOctModeShift;
                // Channels outside the span [lo, hi) hold the background: the
                // span grows with each step's window, a new ray takes the span of
                // its saved vector, and only the span is reset or copied.
                if (mode == kOctModeBg) {
                    for (int c = lo + lane; c < hi; c += LANES) I[c] = Ibg;
                    lo = p.nch;
                    hi = 0;
                } else if (mode != kOctModeKeep && sp >= 0) {
                    int slo = 0, shi = p.nch;
                    if (use_spans) spans.get(sp, slo, shi);
                    // reset what the saved vector does not cover, then copy it
                    const int r0 = hi < slo ? hi : slo, r1 = lo > shi ? lo : shi;
                    for (int c = lo + lane; c < r0; c += LANES) I[c] = Ibg;
                    for (int c = r1 + lane; c < hi; c += LANES) I[c] = Ibg;
                    if (shi > slo)
                        copy_pieces<LANES, T>(I, stk + (size_t)sp * p.ich, slo / kPer, (shi + kPer - 1) / kPer, lane);
                    lo = slo;
                    hi = shi;
                    if (mode == kOctModePop) --sp;
                }
                if ((w0 & kOctSave) && sp + 1 < p.depth) {
                    ++sp;
                    if (!use_spans) {
                        lo = 0;
                        hi = p.nch;
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (hi > lo)
                        copy_pieces<LANES, T>(stk + (size_t)sp * p.ich, I, lo / kPer, (hi + kPer - 1) / kPer, lane);
                    if (use_spans) spans.set(sp, lane, lo, hi);
                }
            }
            __builtin_amdgcn_wave_barrier();
            const int clo = as_int(wv.z);
            const int nwin = as_int(wv.w);
            if (nwin > 0) {
                // the unmasked FP32 passes may change every channel up to the
                // reach, and a longer window is finished in a loop: the span
                // covers both whichever passes run
                constexpr int kR = pass_reach<LANES>();
                const int top = sizeof(T) == 4 && clo <= nch_reach ? clo + (nwin > kR ? nwin : kR) : clo + nwin;
                lo = clo < lo ? clo : lo;
                hi = top > hi ? top : hi;
            }
            T sj = 0, sl = 0;
            window_channels<LANES, T, HF>(I, lane, clo, nwin, wv.x, wv.y, kl, el, sj, sl, &hfr, p.maser, nch_reach);
            if (ACCUM) {
                if constexpr (kQuad) {
                    // every lane of a quad holds the quad's sum; lanes 0 and 4
                    // queue them for step k
                    float hj = dpp_add<0xB1, 0xF>((float)sj);
                    float hl = dpp_add<0xB1, 0xF>((float)sl);
                    hj = dpp_add<0x4E, 0xF>(hj);
                    hl = dpp_add<0x4E, 0xF>(hl);
                    keep_here(hj);
                    keep_here(hl);
                    if ((lane & 3) == 0) queue[2 * k + (lane >> 2)] = T2q{(T)hj, (T)hl};
                } else {
                    const T wgt = aw * len;
                    T2q v;
                    v.x = wgt * group_sum<LANES>(sj);
                    v.y = wgt * group_sum<LANES>(sl);
                    keep_here(v.x);
                    keep_here(v.y);
                    if (lane == LANES - 1) queue[qn] = v;
                    ++qn;
                    __builtin_amdgcn_wave_barrier();
                    if (qn == LANES || s == tr.n - 1) {
                        if (lane < qn) Et[(size_t)(qs0 + lane) * p.estride] = queue[lane];
                        qs0 += qn;
                        qn = 0;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            ++s;
        }
        if constexpr (ACCUM && kQuad) {
            // steps s_chunk .. s - 1 of the unit ran in this chunk: lane k
            // finishes step k's group sum (the two quad sums, the same
            // additions as a butterfly) and weight, aw times its own record's
            // length, and writes its row
            __builtin_amdgcn_wave_barrier();
            if (have && lane < s - s_chunk) {
                const T2q a = queue[2 * lane], b = queue[2 * lane + 1];
                const T wgt = aw * (T)__uint_as_float(mine.y);
                Et[(size_t)(s_chunk + lane) * p.estride] = T2q{wgt * (a.x + b.x), wgt * (a.y + b.y)};
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (have && s >= tr.n) {
            if (!ACCUM && p.Iout) {
                T* out = p.Iout + (size_t)tr.r * p.nch;
                for (int c = lane; c < p.nch; c += LANES) out[c] = I[c];
            }
            have = false;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- 1D march
namespace {

__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }

}  // namespace

// One workgroup marches rays ray0 .. ray0 + rays_per_block - 1 of one
// transition through a 1D shell model.  Each ray's steps {length, Doppler
// shift in channels} were computed once per model in FP64 by ray_steps_kernel
// (Sect. 2.1: the paths are fixed, so they are precomputed); the shell of step
// s follows from s and the ray's innermost shell.  Records arrive LANES at a
// time, one per lane (loading the next chunk a chunk ahead measured 11%
// slower in the request loop), and the next step's shell data are loaded
// before the current step runs.  With p.lds_acc the per-step sums go to
// per-shell FP64 LDS accumulators (LDS atomics do not stall the next step's
// loads; in FP64 the sum of a shell's visits by the workgroup's rays does not
// depend on their order beyond FP64 rounding), flushed to the FP64 global
// sums once per workgroup; otherwise each step issues two FP64 atomics.
template <typename T, int LANES, bool ACCUM, bool TRANS_GROUPS = false, bool HF = false>
__device__ __forceinline__ void march1d_block(const March1DArgs<T>& p, int ray0, int t_in, unsigned char* smem_raw)
{
    using T2 = typename V2<T>::type;
    const int lane = threadIdx.x % LANES;
    const int rib = threadIdx.x / LANES;
    // TRANS_GROUPS (lines of sight, no accumulation): the lane groups take
    // transitions t_in, t_in + 1, ... of ray ray0 instead of consecutive rays
    const int j = TRANS_GROUPS ? (t_in + rib < p.ntr_total ? ray0 : p.nrays) : ray0 + rib;
    const int t = TRANS_GROUPS ? (t_in + rib < p.ntr_total ? t_in + rib : t_in) : t_in;
    const int n = p.n;
    const bool lds_acc = ACCUM && p.lds_acc;
    double* __restrict__ sacc = reinterpret_cast<double*>(smem_raw);       // [n][2] when lds_acc
    T* __restrict__ I = reinterpret_cast<T*>(smem_raw + (lds_acc ? p.acc_lds_bytes : 0)) + (size_t)rib * p.nch;
    const int ts = p.ntr_total;      // cell-major [shell][transition]
    const int kmin0 = p.kmin[ray0];  // the block's rays are sorted by impact parameter
    if (lds_acc) {
        for (int k = kmin0 + (int)threadIdx.x; k < n; k += blockDim.x) {
            sacc[2 * k] = 0.0;
            sacc[2 * k + 1] = 0.0;
        }
        __syncthreads();
    }
    if (j < p.nrays) {
        const double a = p.area[j];
        const int kmin = p.kmin[j];
        const int nin = n - 1 - kmin;
        // the ray's steps s0 .. s0 + nsteps - 1: all of them, or (core
        // sub-iterations) its inward steps outside the core or its steps
        // inside the core (inwards from R[core_k], the tangent halves,
        // outwards back to R[core_k]); a ray of such a launch reaches the core
        int s0 = 0, nsteps = 2 * nin + 2;
        if (p.seg == kSegEnvelopeIn) {
            nsteps = n - 1 - p.core_k;
        } else if (p.seg == kSegCore) {
            s0 = n - 1 - p.core_k;
            nsteps = 2 * (p.core_k - kmin) + 2;
        }
        const T2* __restrict__ rec = p.steps + p.ray_off[j] + s0;
        const T Ibg = p.Ibg[t];
        HfRegs<T> hfr;
        if constexpr (HF) hfr.load(p.hf + (size_t)t * p.hfk, p.hfk);
        if (p.seg == kSegCore) {
            const T* __restrict__ src = p.Ient + ((size_t)(t - p.trans_offset) * p.nrays + j) * p.nch;
            for (int c = lane; c < p.nch; c += LANES) I[c] = src[c];
        } else {
            for (int c = lane; c < p.nch; c += LANES) I[c] = Ibg;
        }
        auto shell_of = [&](int sl) {
            const int s = sl + s0;
            return s < nin ? n - 1 - s : (s <= nin + 1 ? kmin : kmin + (s - nin - 1));
        };
        T2 mine = rec[lane < nsteps ? lane : 0];
        T2 r_n;
        r_n.x = __shfl(mine.x, 0, LANES);
        r_n.y = __shfl(mine.y, 0, LANES);
        int k_n = shell_of(0);
        T2 sv_n = p.shellv[k_n];
        T2 kev_n = p.ke[(size_t)k_n * ts + t];
        for (int s = 0; s < nsteps; ++s) {
            const T2 r = r_n;
            const int k = k_n;
            const T2 sv = sv_n;
            const T2 kev = kev_n;
            if (s + 1 < nsteps) {
                const int q = (s + 1) & (LANES - 1);
                if (q == 0) mine = rec[s + 1 + lane < nsteps ? s + 1 + lane : s + 1];
                r_n.x = __shfl(mine.x, q, LANES);
                r_n.y = __shfl(mine.y, q, LANES);
                k_n = shell_of(s + 1);
                sv_n = p.shellv[k_n];
                kev_n = p.ke[(size_t)k_n * ts + t];
            }
            int clo, chi;
            T frac;
            if (HF)
                window<T>((double)r.y, p.chalf, p.Kw, sv.y, p.nch, clo, chi, frac, p.hf_lo, p.hf_hi);
            else
                window<T>((double)r.y, p.chalf, p.Kw, sv.y, p.nch, clo, chi, frac);
            const T tl = r.x;
            T sj = 0, sl = 0;
            window_channels<LANES, T, HF>(I, lane, clo, chi - clo + 1, frac * sv.y, sv.y, kev.x * tl, kev.y * tl,
                                          sj, sl, &hfr, p.maser, p.nch - pass_reach<LANES>());
            if (ACCUM) {
                sj = group_sum<LANES>(sj);
                sl = group_sum<LANES>(sl);
                keep_here(sj);
                keep_here(sl);
                if (lane == LANES - 1) {
                    const double wgt = a * (double)tl;
                    if (lds_acc) {
                        lds_add(&sacc[2 * k], wgt * (double)sj);
                        lds_add(&sacc[2 * k + 1], wgt * (double)sl);
                    } else {
                        unsafeAtomicAdd(&p.acc[(size_t)k * ts + t].x, wgt * (double)sj);
                        unsafeAtomicAdd(&p.acc[(size_t)k * ts + t].y, wgt * (double)sl);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (!ACCUM && p.Iout) {
            T* out = p.Iout + ((size_t)(t - p.trans_offset) * p.nrays + j) * p.nch;
            for (int c = lane; c < p.nch; c += LANES) out[c] = I[c];
        }
    }
    if (lds_acc) {
        __syncthreads();
        for (int k = kmin0 + (int)threadIdx.x; k < n; k += blockDim.x) {
            const double vj = sacc[2 * k], vl = sacc[2 * k + 1];
            if (vj != 0.0 || vl != 0.0) {
                unsafeAtomicAdd(&p.acc[(size_t)k * ts + t].x, vj);
                unsafeAtomicAdd(&p.acc[(size_t)k * ts + t].y, vl);
            }
        }
    }
}

// Steps of 1D rays (Sect. 2.1), one workgroup per ray: ray j of impact
// parameter b_j enters at the outer radius (R[n-1] = 1), goes inwards to its
// innermost shell kmin_j, whose chord is split at the tangent point into two
// halves, and back out.  Record s: {path length, Doppler shift in channels
// v_r mu / dv}, mu = cosine between the direction and the outward radius at
// the start of the step.  FP64 geometry, rounded once to T.
template <typename T>
__global__ __launch_bounds__(256) void ray_steps_kernel(int n, const double* __restrict__ R,
                                                        const double* __restrict__ b,
                                                        const int* __restrict__ kmin,
                                                        const long long* __restrict__ off,
                                                        const double* __restrict__ vr_dv,
                                                        typename V2<T>::type* __restrict__ out)
{
    const int j = blockIdx.x;
    const double bj = b[j];
    const int km = kmin[j];
    const int nin = n - 1 - km;
    const int ns = 2 * nin + 2;
    typename V2<T>::type* __restrict__ o = out + off[j];
    auto z = [&](int k) { return sqrt(fmax(0.0, (R[k] - bj) * (R[k] + bj))); };
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        int k;
        double len, mu;
        if (s < nin) {
            k = n - 1 - s;
            const double zo = z(k);
            len = zo - z(k - 1);
            mu = -zo / R[k];
        } else if (s == nin) {
            k = km;
            len = z(k);
            mu = -len / R[k];
        } else if (s == nin + 1) {
            k = km;
            len = z(k);
            mu = 0.0;
        } else {
            k = km + (s - nin - 1);
            const double zi = z(k - 1);
            len = z(k) - zi;
            mu = zi / R[k - 1];
        }
        o[s].x = (T)len;
        o[s].y = (T)(vr_dv[k] * mu);
    }
}

// Ray-sampled shell volumes W_k = sum_j a_j (path of ray j in shell k): a ray
// with b_j < R_{k-1} crosses shell k twice, one with R_{k-1} <= b_j < R_k has
// it as its tangent shell (full chord).  With bsq given, the output is
// q_k = dv / (bsq_k W_k) instead (0 where W_k = 0).
__global__ __launch_bounds__(256) void shell_weights_kernel(int n, const double* __restrict__ R, int nrays,
                                                            const double* __restrict__ b,
                                                            const double* __restrict__ area,
                                                            const double* __restrict__ bsq, double dv,
                                                            double* __restrict__ out)
{
    // one wavefront per shell, its lanes over the rays; the lane sums are
    // combined in a fixed order, so W does not depend on the launch
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= n) return;
    const double ro = R[k], ri = k > 0 ? R[k - 1] : 0.0;
    double w = 0.0;
    for (int j = lane; j < nrays; j += 64) {
        const double bj = b[j];
        if (!(ro > bj)) continue;
        const double zo = sqrt((ro - bj) * (ro + bj));
        const double zi = ri > bj ? sqrt((ri - bj) * (ri + bj)) : 0.0;
        w += area[j] * 2.0 * (zo - zi);
    }
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
    if (lane == 0) out[k] = bsq ? (w > 0 ? dv / (bsq[k] * w) : 0.0) : w;
}

template <typename T, int LANES, bool ACCUM, bool HF>
__global__ __launch_bounds__(256) void march1d_kernel(March1DArgs<T> p)
{
    extern __shared__ unsigned char smem_raw[];
    const int rpb = blockDim.x / LANES;
    march1d_block<T, LANES, ACCUM, false, HF>(p, blockIdx.x * rpb, p.trans_offset + blockIdx.y, smem_raw);
}

// All transitions of a ray in one pass (the paper's Sect. 4 names this
// alternative to repeating the ray tracing per transition): one wavefront
// marches one 1D ray for kTbGroups transitions at once, a group of 16 lanes
// per transition.  The step records, the shell's data and the channel window
// are the wavefront's, and the line profile of each step (the same for every
// transition in velocity units) is evaluated once by the whole wavefront into
// LDS and read by every group.  The per-step sums of each transition go to
// the FP64 sums with device atomics.
namespace {
constexpr int kTbGroups = 4;
constexpr int kTbLanes = 16;
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void march1d_tb_kernel(March1DArgs<T> p)
{
    using T2 = typename V2<T>::type;
    extern __shared__ unsigned char smem_raw[];
    const int wid = threadIdx.x >> 6;                 // wavefront of the block
    const int wl = threadIdx.x & 63;                  // lane in the wavefront
    const int g = wl / kTbLanes;                      // group = transition slot
    const int lane = wl % kTbLanes;
    const int j = blockIdx.x * (blockDim.x >> 6) + wid;
    const int t = p.trans_offset + blockIdx.y * kTbGroups + g;
    const bool t_ok = t < p.trans_offset + p.ntr;
    const int tt = t_ok ? t : p.trans_offset;
    const int stride = p.nch + kVecTailPadWords;
    T* __restrict__ base = reinterpret_cast<T*>(smem_raw) + (size_t)wid * (kTbGroups + 1) * stride;
    T* __restrict__ I = base + (size_t)g * stride;
    T* __restrict__ prof = base + (size_t)kTbGroups * stride;
    if (j >= p.nrays) return;                         // the whole wavefront
    const int n = p.n;
    const int ts = p.ntr_total;
    const double a = p.area[j];
    const int kmin = p.kmin[j];
    const int nin = n - 1 - kmin;
    const int nsteps = 2 * nin + 2;
    const T2* __restrict__ rec = p.steps + p.ray_off[j];
    const T Ibg = p.Ibg[tt];
    for (int c = lane; c < p.nch; c += kTbLanes) I[c] = Ibg;
    auto shell_of = [&](int s) {
        return s < nin ? n - 1 - s : (s <= nin + 1 ? kmin : kmin + (s - nin - 1));
    };
    // records arrive 64 at a time, one per lane of the wavefront
    T2 mine = rec[wl < nsteps ? wl : 0];
    T2 r_n;
    r_n.x = __shfl(mine.x, 0, 64);
    r_n.y = __shfl(mine.y, 0, 64);
    int k_n = shell_of(0);
    T2 sv_n = p.shellv[k_n];
    T2 kev_n = p.ke[(size_t)k_n * ts + tt];
    for (int s = 0; s < nsteps; ++s) {
        const T2 r = r_n;
        const int k = k_n;
        const T2 sv = sv_n;
        const T2 kev = kev_n;
        if (s + 1 < nsteps) {
            const int q = (s + 1) & 63;
            if (q == 0) mine = rec[s + 1 + wl < nsteps ? s + 1 + wl : s + 1];
            r_n.x = __shfl(mine.x, q, 64);
            r_n.y = __shfl(mine.y, q, 64);
            k_n = shell_of(s + 1);
            sv_n = p.shellv[k_n];
            kev_n = p.ke[(size_t)k_n * ts + tt];
        }
        int clo, chi;
        T frac;
        window<T>((double)r.y, p.chalf, p.Kw, sv.y, p.nch, clo, chi, frac);
        const int nwin = chi - clo + 1;
        const T ibs = sv.y;
        const T x0 = frac * ibs;
        // the profile of the step, once for all transitions
        for (int jj = wl; jj < nwin; jj += 64) {
            const T xs = (T)jj * ibs + x0;
            prof[jj] = fast_exp2(-xs * xs);
        }
        __builtin_amdgcn_wave_barrier();
        const T tl = r.x;
        const T kl = t_ok ? kev.x * tl : (T)0;
        const T el = t_ok ? kev.y * tl : (T)0;
        T sj = 0, sl = 0;
        T* __restrict__ row = I + clo;
        const bool thin = __all(kl < (T)1e-3 && kl > (T)-1e-3);
        if (!thin && kl < (T)kMaserTauMin) *p.maser = 1u;
        if (thin) {
            for (int jj = lane; jj < nwin; jj += kTbLanes) {
                const T ec = prof[jj];
                const T tau = kl * ec;
                const T omb = std::is_same<T, float>::value ? tau * ((T)0.5 - tau * (T)(1.0 / 6.0)) : omb_any(tau);
                const T Iin = row[jj];
                const T u = ec - ec * omb;
                sj += Iin * u;
                sl += ec * omb;
                row[jj] = Iin + u * (el - kl * Iin);
            }
        } else {
            for (int jj = lane; jj < nwin; jj += kTbLanes) {
                const T ec = prof[jj];
                const T omb = omb_any(kl * ec);
                const T Iin = row[jj];
                const T u = ec - ec * omb;
                sj += Iin * u;
                sl += ec * omb;
                row[jj] = Iin + u * (el - kl * Iin);
            }
        }
        sj = group_sum<kTbLanes>(sj);
        sl = group_sum<kTbLanes>(sl);
        keep_here(sj);
        keep_here(sl);
        if (lane == kTbLanes - 1 && t_ok) {
            const double wgt = a * (double)tl;
            unsafeAtomicAdd(&p.acc[(size_t)k * ts + t].x, wgt * (double)sj);
            unsafeAtomicAdd(&p.acc[(size_t)k * ts + t].y, wgt * (double)sl);
        }
        __builtin_amdgcn_wave_barrier();              // prof and the vectors are rewritten next step
    }
}

// ---------------------------------------------------------------- SE solve
// One thread per cell.  The (L+1) x L augmented matrix lives in LDS with the
// thread index fastest, M[(row*(L+1) + col)*bs + tid].
// Statistical equilibrium of cell k (Sect. 2): rates with the absorbed counts
// in place of B I, ALI form with A scaled by the escape probability.  The
// augmented matrix lives in LDS, sm[(row*(L+1) + col)*bs + tid].  Returns the
// cell's maximum relative population change (0 if k is out of range).
__device__ double se_cell(const SEArgs& p, int k, int tid, int bs, double* __restrict__ sm)
{
    const MolDev* __restrict__ mol = p.mol;
    const int L = p.L;
    const int W = L + 1;
    double* M = sm;                                    // L*W*bs
    double* bz = sm + (size_t)L * W * bs;              // L*bs Boltzmann factors
#define MM(i, j) M[((i) * W + (j)) * bs + tid]
#define BZ(i) bz[(i) * bs + tid]
    double dmax = 0.0;
    if (k < p.nc) {
        const double* xo = p.x_old + (size_t)k * L;
        const double nH2 = p.nH2[k];
        const double T = p.Tkin[k];
        const double q = p.q[k];
        if (q < 0.0) {
            // a refined octree cell: no rays cross it, its populations are kept
            for (int i = 0; i < L; ++i) p.x_new[(size_t)k * L + i] = xo[i];
            return 0.0;
        }

        for (int i = 0; i < L; ++i) {
            for (int j = 0; j < W; ++j) MM(i, j) = 0.0;
            BZ(i) = mol->g[i] * exp(-mol->E[i] / T);
        }
        // collisions, every pair u > l; upward rate by detailed balance
        for (int u = 1; u < L; ++u) {
            for (int l = 0; l < u; ++l) {
                const double gam = mol->gamma[u * L + l];
                if (gam == 0.0) continue;
                const double Cul = nH2 * gam;
                const double Clu = Cul * BZ(u) / BZ(l);
                MM(l, u) += Cul;  MM(u, u) -= Cul;
                MM(u, l) += Clu;  MM(l, l) -= Clu;
            }
        }
        // radiative rates; ALI: A scaled by the escape probability 1 - Lambda
        for (int t = 0; t < p.ntr; ++t) {
            const int u = mol->up[t], l = mol->lo[t];
            const double A = mol->A[t];
            const double2 a = p.acc[(size_t)k * p.ntr + t];
            double J = a.x * q;
            const double Lam = a.y * q;
            double Rul;
            if (p.use_ali) {
                Rul = A * (1.0 - Lam) + A * J;
            } else {
                const double den = xo[l] * mol->gratio[t] - xo[u];
                const double S = den != 0.0 ? xo[u] / den : 0.0;
                J += S * Lam;
                Rul = A + A * J;
            }
            const double Rlu = mol->gratio[t] * A * J;
            MM(l, u) += Rul;  MM(u, u) -= Rul;
            MM(u, l) += Rlu;  MM(l, l) -= Rlu;
        }
        // replace the equation of the most populated level by sum x = 1
        int r = 0;
        for (int i = 1; i < L; ++i) if (xo[i] > xo[r]) r = i;
        for (int j = 0; j < L; ++j) MM(r, j) = 1.0;
        MM(r, L) = 1.0;
        // Gaussian elimination with partial pivoting
        for (int c = 0; c < L; ++c) {
            int piv = c;
            double best = fabs(MM(c, c));
            for (int i = c + 1; i < L; ++i) {
                const double v = fabs(MM(i, c));
                if (v > best) { best = v; piv = i; }
            }
            if (piv != c)
                for (int j = c; j < W; ++j) {
                    const double tmp = MM(c, j); MM(c, j) = MM(piv, j); MM(piv, j) = tmp;
                }
            const double inv = 1.0 / MM(c, c);
            for (int i = c + 1; i < L; ++i) {
                const double f = MM(i, c) * inv;
                if (f == 0.0) continue;
                for (int j = c + 1; j < W; ++j) MM(i, j) -= f * MM(c, j);
            }
        }
        for (int i = L - 1; i >= 0; --i) {
            double s = MM(i, L);
            for (int j = i + 1; j < L; ++j) s -= MM(i, j) * MM(j, L);
            MM(i, L) = s / MM(i, i);
        }
        bool bad = false;
        for (int i = 0; i < L; ++i) {
            const double xi = MM(i, L);
            p.x_new[(size_t)k * L + i] = xi;
            if (!(xi == xi) || xi < -1.0e-12 || fabs(xi) > 2.0) bad = true;
            if (xi >= 1.0e-10) {
                const double d = fabs(xi - xo[i]) / xi;
                dmax = d > dmax ? d : dmax;
            }
        }
        if (bad) atomicAdd(p.bad, 1u);
    }
#undef MM
#undef BZ
    return dmax;
}

// The same solve with the matrix in registers, for L known at compile time
// (every index below is a constant after unrolling).  Rates are entered per
// level pair u > l: all collisions, then the radiative transition of each
// pair (MolDev::pair_t); the pivot row exchange of partial pivoting is done
// with selects.  Same equations and pivot choice as se_cell; the radiative
// terms of a diagonal entry are summed in pair rather than transition order.
template <int L>
__device__ double se_cell_reg(const SEArgs& p, int k)
{
    constexpr int W = L + 1;
    const MolDev* __restrict__ mol = p.mol;
    const double* xo = p.x_old + (size_t)k * L;
    double* xn = p.x_new + (size_t)k * L;
    double x[L];
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = xo[i];
    const double q = p.q[k];
    if (q < 0.0) {
        // a refined octree cell: no rays cross it, its populations are kept
#pragma unroll
        for (int i = 0; i < L; ++i) xn[i] = x[i];
        return 0.0;
    }
    const double nH2 = p.nH2[k];
    const double T = p.Tkin[k];
    double bz[L];
#pragma unroll
    for (int i = 0; i < L; ++i) bz[i] = mol->g[i] * exp(-mol->E[i] / T);
    double M[L][W];
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) M[i][j] = 0.0;
    // collisions, every pair u > l; upward rate by detailed balance
#pragma unroll
    for (int u = 1; u < L; ++u) {
#pragma unroll
        for (int l = 0; l < u; ++l) {
            const double gam = mol->gamma[u * L + l];
            if (gam != 0.0) {
                const double Cul = nH2 * gam;
                const double Clu = Cul * bz[u] / bz[l];
                M[l][u] += Cul;  M[u][u] -= Cul;
                M[u][l] += Clu;  M[l][l] -= Clu;
            }
        }
    }
    // radiative rates, by level pair; ALI: A scaled by 1 - Lambda
#pragma unroll
    for (int u = 1; u < L; ++u) {
#pragma unroll
        for (int l = 0; l < u; ++l) {
            const int t = mol->pair_t[u * kMaxLevels + l];
            if (t >= 0) {
                const double A = mol->A[t];
                const double2 a = p.acc[(size_t)k * p.ntr + t];
                double J = a.x * q;
                const double Lam = a.y * q;
                double Rul;
                if (p.use_ali) {
                    Rul = A * (1.0 - Lam) + A * J;
                } else {
                    const double den = x[l] * mol->gratio[t] - x[u];
                    const double S = den != 0.0 ? x[u] / den : 0.0;
                    J += S * Lam;
                    Rul = A + A * J;
                }
                const double Rlu = mol->gratio[t] * A * J;
                M[l][u] += Rul;  M[u][u] -= Rul;
                M[u][l] += Rlu;  M[l][l] -= Rlu;
            }
        }
    }
    // replace the equation of the most populated level by sum x = 1
    int r = 0;
    double xr = x[0];
#pragma unroll
    for (int i = 1; i < L; ++i) {
        r = x[i] > xr ? i : r;
        xr = x[i] > xr ? x[i] : xr;
    }
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) M[i][j] = i == r ? 1.0 : M[i][j];
    // Gaussian elimination with partial pivoting
#pragma unroll
    for (int c = 0; c < L; ++c) {
        int piv = c;
        double best = fabs(M[c][c]);
#pragma unroll
        for (int i = c + 1; i < L; ++i) {
            const double v = fabs(M[i][c]);
            piv = v > best ? i : piv;
            best = v > best ? v : best;
        }
#pragma unroll
        for (int j = c; j < W; ++j) {
            const double rc = M[c][j];
            double rp = rc;
#pragma unroll
            for (int i = c + 1; i < L; ++i) rp = piv == i ? M[i][j] : rp;
#pragma unroll
            for (int i = c + 1; i < L; ++i) M[i][j] = piv == i ? rc : M[i][j];
            M[c][j] = rp;
        }
        const double inv = 1.0 / M[c][c];
#pragma unroll
        for (int i = c + 1; i < L; ++i) {
            const double f = M[i][c] * inv;
            if (f != 0.0) {
#pragma unroll
                for (int j = c + 1; j < W; ++j) M[i][j] -= f * M[c][j];
            }
        }
    }
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
        double sacc = M[i][L];
#pragma unroll
        for (int j = i + 1; j < L; ++j) sacc -= M[i][j] * M[j][L];
        M[i][L] = sacc / M[i][i];
    }
    bool bad = false;
    double dmax = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const double xi = M[i][L];
        xn[i] = xi;
        if (!(xi == xi) || xi < -1.0e-12 || fabs(xi) > 2.0) bad = true;
        if (xi >= 1.0e-10) {
            const double d = fabs(xi - x[i]) / xi;
            dmax = d > dmax ? d : dmax;
        }
    }
    if (bad) atomicAdd(p.bad, 1u);
    return dmax;
}

// Maximum over the block of a non-negative double (bit-pattern order), folded
// into *dst with one atomic per wavefront (or partial wavefront).
__device__ __forceinline__ void block_max_to(double v, int bs, unsigned long long* dst)
{
    const int width = bs < 64 ? bs : 64;
    unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    for (int o = width >> 1; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(bits, o, width);
        bits = other > bits ? other : bits;
    }
    if (((int)threadIdx.x % width) == 0 && bits != 0ull) atomicMax(dst, bits);
}

// Up to 10 levels two wavefronts per SIMD (at 10 levels the matrix and its
// pivoting take ~270 registers: 256 and a few spills, 17% faster than one
// wavefront); 11 and 12 levels keep the registers of one.
template <int L>
__global__ __launch_bounds__(256, (L <= 10 ? 2 : 1)) void se_reg_kernel(SEArgs p)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double dmax = k < p.nc ? se_cell_reg<L>(p, k) : 0.0;
    block_max_to(dmax, (int)blockDim.x, p.delta_bits);
}

__global__ void se_kernel(SEArgs p)
{
    extern __shared__ double sm[];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double dmax = se_cell(p, k, threadIdx.x, p.bs, sm);
    block_max_to(dmax, p.bs, p.delta_bits);
}

// ---------------------------------------------------------------- serving
// Model-indexed kernels for the 1D request loop.  Each runs a fixed grid that
// walks a device work list, so one captured graph serves every tick whatever
// set of models is resident; the lists are rewritten between ticks.

__global__ __launch_bounds__(256) void serve_prepare_kernel(const ServeModel* __restrict__ models,
                                                            const int2* __restrict__ items,
                                                            const int* __restrict__ n_items)
{
    const int n = *n_items;
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int2 it = items[w];
        const ServeModel& M = models[it.x];
        const int k = it.y + threadIdx.x;
        if (k < M.nc) {
            prepare_cell<float>(k, M.mol, M.T, M.x, M.nmolLb, M.mode ? M.ibg64 : nullptr, M.ke_w);
            for (int t = 0; t < M.T; ++t) M.acc_w[(size_t)k * M.T + t] = make_double2(0.0, 0.0);
        }
        if (it.y == 0 && threadIdx.x == 0) {
            *M.delta_bits = 0ull;
            *M.bad = 0u;
        }
    }
}

__global__ __launch_bounds__(256) void serve_march_kernel(const ServeModel* __restrict__ models,
                                                          const int4* __restrict__ items,
                                                          const int* __restrict__ n_items)
{
    extern __shared__ unsigned char smem_raw[];
    const int n = *n_items;
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int4 it = items[w];                  // model, transition, first ray, spectrum
        const ServeModel& M = models[it.x];
        if (it.w) {
            // the centre line of sight (stored after the model's rays), I - I_bg
            March1DArgs<float> a = M.m;
            a.ray_off += a.nrays;
            a.kmin += a.nrays;
            a.nrays = 1;
            a.Ibg = M.zero;
            a.Iout = M.spec;
            march1d_block<float, 64, false, true>(a, 0, it.y, smem_raw);
        } else {
            const March1DArgs<float> a = M.m;
            march1d_block<float, 16, true>(a, it.z, it.y, smem_raw);
        }
        __syncthreads();
    }
}

__global__ void serve_se_kernel(const ServeModel* __restrict__ models, const int2* __restrict__ items,
                                const int* __restrict__ n_items)
{
    extern __shared__ double sm[];
    const int n = *n_items;
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int2 it = items[w];
        const ServeModel& M = models[it.x];
        SEArgs a{};
        a.nc = M.nc;
        a.L = M.L;
        a.ntr = M.T;
        a.use_ali = 1;
        a.bs = blockDim.x;
        a.mol = M.mol;
        a.x_old = M.x;
        a.x_new = M.xn;
        a.nH2 = M.nH2;
        a.Tkin = M.Tk;
        a.q = M.q;
        a.acc = M.acc_w;
        a.delta_bits = M.delta_bits;
        a.bad = M.bad;
        const double dmax = se_cell(a, it.y + threadIdx.x, threadIdx.x, blockDim.x, sm);
        block_max_to(dmax, blockDim.x, M.delta_bits);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void serve_copy_kernel(const ServeModel* __restrict__ models,
                                                         const int2* __restrict__ items,
                                                         const int* __restrict__ n_items)
{
    const int n = *n_items;
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int2 it = items[w];
        const ServeModel& M = models[it.x];
        const int k = it.y + threadIdx.x;
        if (k < M.nc)
            for (int i = 0; i < M.L; ++i) M.x[(size_t)k * M.L + i] = M.xn[(size_t)k * M.L + i];
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_prepare(hipStream_t s, int nc, const MolDev* mol, int ntr, const double* x,
                          const double* nmolLb, const double* ibg_sub, void* ke, bool fp64)
{
    const int bs = 256;
    const int nb = (nc + bs - 1) / bs;
    if (fp64)
        hipLaunchKernelGGL(prepare_kernel<double>, dim3(nb), dim3(bs), 0, s, nc, mol, ntr, x, nmolLb,
                           ibg_sub, reinterpret_cast<double2*>(ke));
    else
        hipLaunchKernelGGL(prepare_kernel<float>, dim3(nb), dim3(bs), 0, s, nc, mol, ntr, x, nmolLb,
                           ibg_sub, reinterpret_cast<float2*>(ke));
    return hipGetLastError();
}

hipError_t launch_window_table(hipStream_t s, int nc, int n_dir, const DirDev* dirs, const float4* vel,
                               const double* bD, double dv, double chalf, double K, int nch, double dlo,
                               double dhi, void* win, bool fp64)
{
    const int bs = 256;
    const dim3 grid((nc + bs - 1) / bs, n_dir);
    if (fp64)
        hipLaunchKernelGGL(window_table_kernel<double>, grid, dim3(bs), 0, s, nc, n_dir, dirs, vel, bD, dv,
                           chalf, K, nch, dlo, dhi, reinterpret_cast<double4*>(win));
    else
        hipLaunchKernelGGL(window_table_kernel<float>, grid, dim3(bs), 0, s, nc, n_dir, dirs, vel, bD, dv,
                           chalf, K, nch, dlo, dhi, reinterpret_cast<float4*>(win));
    return hipGetLastError();
}

hipError_t launch_lte(hipStream_t s, int nc, const MolDev* mol, const double* Tkin, double* x)
{
    const int bs = 256;
    hipLaunchKernelGGL(lte_kernel, dim3((nc + bs - 1) / bs), dim3(bs), 0, s, nc, mol, Tkin, x);
    return hipGetLastError();
}

namespace {
template <typename T>
int rays_per_block(int lanes, int nch)
{
    int rpb = 256 / lanes;
    while (rpb > 1 && (size_t)rpb * nch * sizeof(T) + kVecTailPadWords * sizeof(float) > 65536) rpb >>= 1;
    return rpb;
}

template <typename T, int LANES, bool ACCUM, bool HF>
hipError_t do_march3d(hipStream_t s, March3DArgs<T> a, int max_steps)
{
    constexpr bool kF32 = std::is_same<T, float>::value && !HF;
    // Channel vectors are padded by 16 words so that the rays of one
    // wavefront start in different LDS banks; the FP32 single-Gaussian
    // kernel's predicated passes need their reach after each vector.
    a.ich = a.nch + (kF32 ? f32_vec_gap(LANES) : 16);
    // with a span table the vector holds the ray's span only (rounded to 32
    // words plus 8, so that the rays of a wavefront start 8 banks apart)
    if (kF32 && ACCUM && a.rbase) a.ich = (a.span_w + 31) / 32 * 32 + 8;
    // whole wavefronts only (the queue flush uses every lane of a wavefront)
    const int rpw = 64 / LANES;
    int rpb = 256 / LANES;
    while (rpb > rpw && (size_t)rpb * a.ich * sizeof(T) > 65536) rpb >>= 1;
    a.blocks_per_dir = (a.rays_per_dir + rpb - 1) / rpb;
    a.step_lds_bytes = (int)(((size_t)max_steps * sizeof(StepRec<T>) + 15) & ~(size_t)15);
    a.queue_lds_offset = a.step_lds_bytes + (int)((size_t)rpb * a.ich * sizeof(T));
    const dim3 grid(a.blocks_per_dir * a.n_dir * a.ntr);
    // the FP32 kernel with 8 or 16 lanes queues its sums in registers
    const bool lds_queue = !(kF32 && LANES <= 16);
    const size_t shm = (size_t)a.queue_lds_offset + (lds_queue ? (size_t)rpb * LANES * 2 * sizeof(T) : 0);
    if (shm > 163840) return hipErrorInvalidValue;
    if constexpr (kF32) {
        if (shm > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)march3d_f32_kernel<LANES, ACCUM, true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void*)march3d_f32_kernel<LANES, ACCUM, false>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            if (e != hipSuccess) return e;
        }
        // 32-bit table offsets while a direction's window table and the
        // {khat, ehat} table stay below 4 GB and the cells below 2^24
        const uint64_t nc = (uint64_t)a.nc;
        const bool off32 = nc < (1u << 24) && nc * sizeof(float4) < (1ull << 32) &&
                           nc * (uint64_t)a.ntr_total * sizeof(float2) < (1ull << 32) &&
                           !std::getenv("MILOC_WIDE_OFFSETS");
        if (off32)
            hipLaunchKernelGGL((march3d_f32_kernel<LANES, ACCUM, true>), grid, dim3(rpb * LANES), shm, s, a);
        else
            hipLaunchKernelGGL((march3d_f32_kernel<LANES, ACCUM, false>), grid, dim3(rpb * LANES), shm, s, a);
    } else {
        if (shm > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)march3d_kernel<T, LANES, ACCUM, HF>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((march3d_kernel<T, LANES, ACCUM, HF>), grid, dim3(rpb * LANES), shm, s, a);
    }
    return hipGetLastError();
}

template <typename T, int LANES, bool ACCUM, bool HF>
hipError_t do_march1d(hipStream_t s, March1DArgs<T> a)
{
    const int rpb = rays_per_block<T>(LANES, a.nch);
    const dim3 grid((a.nrays + rpb - 1) / rpb, a.ntr);
    a.acc_lds_bytes = (int)((((size_t)a.n * 2 * sizeof(double)) + 15) & ~(size_t)15);
    const size_t vec_bytes = (size_t)rpb * a.nch * sizeof(T) + kVecTailPadWords * sizeof(float);
    a.lds_acc = ACCUM && ((size_t)a.acc_lds_bytes + vec_bytes <= 65536) ? 1 : 0;
    const size_t shm = (a.lds_acc ? (size_t)a.acc_lds_bytes : 0) + vec_bytes;
    hipLaunchKernelGGL((march1d_kernel<T, LANES, ACCUM, HF>), grid, dim3(rpb * LANES), shm, s, a);
    return hipGetLastError();
}

template <typename T, bool HF>
hipError_t dispatch3d_hf(hipStream_t s, const March3DArgs<T>& a, int lanes, bool accum, int max_steps)
{
    if (lanes == 8)
        return accum ? do_march3d<T, 8, true, HF>(s, a, max_steps) : do_march3d<T, 8, false, HF>(s, a, max_steps);
    if (lanes == 16)
        return accum ? do_march3d<T, 16, true, HF>(s, a, max_steps) : do_march3d<T, 16, false, HF>(s, a, max_steps);
    if (lanes == 32)
        return accum ? do_march3d<T, 32, true, HF>(s, a, max_steps) : do_march3d<T, 32, false, HF>(s, a, max_steps);
    return accum ? do_march3d<T, 64, true, HF>(s, a, max_steps) : do_march3d<T, 64, false, HF>(s, a, max_steps);
}

template <typename T>
hipError_t dispatch3d(hipStream_t s, const March3DArgs<T>& a, int lanes, bool accum, int max_steps)
{
    return a.hf ? dispatch3d_hf<T, true>(s, a, lanes, accum, max_steps)
                : dispatch3d_hf<T, false>(s, a, lanes, accum, max_steps);
}

template <typename T, bool HF>
hipError_t dispatch1d_hf(hipStream_t s, const March1DArgs<T>& a, int lanes, bool accum)
{
    if (lanes == 8) return accum ? do_march1d<T, 8, true, HF>(s, a) : do_march1d<T, 8, false, HF>(s, a);
    if (lanes == 16) return accum ? do_march1d<T, 16, true, HF>(s, a) : do_march1d<T, 16, false, HF>(s, a);
    if (lanes == 32) return accum ? do_march1d<T, 32, true, HF>(s, a) : do_march1d<T, 32, false, HF>(s, a);
    return accum ? do_march1d<T, 64, true, HF>(s, a) : do_march1d<T, 64, false, HF>(s, a);
}

template <typename T>
hipError_t dispatch1d(hipStream_t s, const March1DArgs<T>& a, int lanes, bool accum)
{
    return a.hf ? dispatch1d_hf<T, true>(s, a, lanes, accum) : dispatch1d_hf<T, false>(s, a, lanes, accum);
}
}  // namespace

hipError_t launch_ray_spans(hipStream_t s, const March3DArgs<float>& a, int reach, int* rbase, int* wmax)
{
    if (a.rays_per_dir <= 0 || a.n_dir <= 0) return hipSuccess;
    const dim3 grid((a.rays_per_dir + 255) / 256, a.n_dir);
    hipLaunchKernelGGL(ray_span_kernel, grid, dim3(256), 0, s, a, reach, rbase, wmax);
    return hipGetLastError();
}
hipError_t launch_march3d(hipStream_t s, const March3DArgs<float>& a, int lanes, bool accum,
                          int max_steps)
{
    return dispatch3d<float>(s, a, lanes, accum, max_steps);
}
hipError_t launch_march3d(hipStream_t s, const March3DArgs<double>& a, int lanes, bool accum,
                          int max_steps)
{
    return dispatch3d<double>(s, a, lanes, accum, max_steps);
}
hipError_t launch_shell_weights(hipStream_t s, int n, const double* R, int nrays, const double* b,
                                const double* area, double* W, const double* bsq, double dv)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(shell_weights_kernel, dim3((n + 3) / 4), dim3(256), 0, s, n, R, nrays, b, area, bsq, dv, W);
    return hipGetLastError();
}

hipError_t launch_ray_steps(hipStream_t s, int n, const double* R, int nrays, const double* b, const int* kmin,
                            const long long* off, const double* vr_dv, void* out, bool fp64)
{
    if (nrays <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(ray_steps_kernel<double>, dim3(nrays), dim3(256), 0, s, n, R, b, kmin, off, vr_dv,
                           reinterpret_cast<double2*>(out));
    else
        hipLaunchKernelGGL(ray_steps_kernel<float>, dim3(nrays), dim3(256), 0, s, n, R, b, kmin, off, vr_dv,
                           reinterpret_cast<float2*>(out));
    return hipGetLastError();
}
hipError_t launch_march1d(hipStream_t s, const March1DArgs<float>& a, int lanes, bool accum)
{
    return dispatch1d<float>(s, a, lanes, accum);
}
hipError_t launch_march1d(hipStream_t s, const March1DArgs<double>& a, int lanes, bool accum)
{
    return dispatch1d<double>(s, a, lanes, accum);
}

template <typename T>
hipError_t do_march1d_tb(hipStream_t s, const March1DArgs<T>& a)
{
    constexpr int kWaves = 4;                          // rays per block
    const size_t shm = (size_t)kWaves * (kTbGroups + 1) * (a.nch + kVecTailPadWords) * sizeof(T);
    if (shm > 163840) return hipErrorInvalidValue;
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)march1d_tb_kernel<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((a.nrays + kWaves - 1) / kWaves, (a.ntr + kTbGroups - 1) / kTbGroups);
    hipLaunchKernelGGL(march1d_tb_kernel<T>, grid, dim3(64 * kWaves), shm, s, a);
    return hipGetLastError();
}
hipError_t launch_march1d_all_transitions(hipStream_t s, const March1DArgs<float>& a)
{
    return do_march1d_tb<float>(s, a);
}
hipError_t launch_march1d_all_transitions(hipStream_t s, const March1DArgs<double>& a)
{
    return do_march1d_tb<double>(s, a);
}

template <typename T>
hipError_t do_gather3d(hipStream_t s, const Gather3DArgs<T>& a)
{
    // a tile of all the launch's transitions up to 12
    const int tile = a.ntr < 12 ? a.ntr : 12;
    const int bs = 256;
    const dim3 grid((a.N * a.N + bs - 1) / bs, a.N, (a.ntr + tile - 1) / tile);
    const dim3 block(bs);
    switch (tile) {
    case 1: hipLaunchKernelGGL((gather3d_kernel<T, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((gather3d_kernel<T, 2>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((gather3d_kernel<T, 3>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((gather3d_kernel<T, 4>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((gather3d_kernel<T, 5>), grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL((gather3d_kernel<T, 6>), grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL((gather3d_kernel<T, 7>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((gather3d_kernel<T, 8>), grid, block, 0, s, a); break;
    case 9: hipLaunchKernelGGL((gather3d_kernel<T, 9>), grid, block, 0, s, a); break;
    case 10: hipLaunchKernelGGL((gather3d_kernel<T, 10>), grid, block, 0, s, a); break;
    case 11: hipLaunchKernelGGL((gather3d_kernel<T, 11>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((gather3d_kernel<T, 12>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}
hipError_t launch_gather3d(hipStream_t s, const Gather3DArgs<float>& a) { return do_gather3d(s, a); }
hipError_t launch_gather3d(hipStream_t s, const Gather3DArgs<double>& a) { return do_gather3d(s, a); }

template <typename T, int LANES, bool HF>
hipError_t do_march_oct(hipStream_t s, const OctMarchArgs<T>& a, int groups, bool accum)
{
    constexpr int kGroupsPerBlock = 256 / LANES;
    const int blocks = (groups + kGroupsPerBlock - 1) / kGroupsPerBlock;
    // channel vectors, then the per-step queues (two quad sums per step for
    // FP32 with 8 lanes)
    const size_t shm = (size_t)kGroupsPerBlock * a.ich * sizeof(T) +
                       (size_t)kGroupsPerBlock * LANES * (sizeof(T) == 4 && LANES == 8 ? 2 : 1) *
                           sizeof(typename V2<T>::type);
    // up to the 160 KB of LDS a workgroup may have (wide channel grids and
    // FP64 vectors: fewer workgroups per CU)
    if (shm > 163840) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    if (shm > 65536) {
        e = accum ? hipFuncSetAttribute((const void*)march_oct_kernel<T, LANES, true, HF>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)
                  : hipFuncSetAttribute((const void*)march_oct_kernel<T, LANES, false, HF>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    e = hipMemsetAsync(a.counter, 0, sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    if (accum)
        hipLaunchKernelGGL((march_oct_kernel<T, LANES, true, HF>), dim3(blocks), dim3(256), shm, s, a);
    else
        hipLaunchKernelGGL((march_oct_kernel<T, LANES, false, HF>), dim3(blocks), dim3(256), shm, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_oct(hipStream_t s, const OctMarchArgs<T>& a, int groups, bool accum, int lanes)
{
    if (a.hf)
        return lanes == 8 ? do_march_oct<T, 8, true>(s, a, groups, accum) : do_march_oct<T, 16, true>(s, a, groups, accum);
    return lanes == 8 ? do_march_oct<T, 8, false>(s, a, groups, accum) : do_march_oct<T, 16, false>(s, a, groups, accum);
}

template <typename T>
hipError_t do_gather_oct(hipStream_t s, const GatherOctArgs<T>& a)
{
    const dim3 grid((unsigned)((a.nc + 255) / 256));
    // the smallest even tile that holds the launch's transitions, at most 12
    switch (a.ntr <= 2 ? 2 : a.ntr <= 4 ? 4 : a.ntr <= 6 ? 6 : a.ntr <= 8 ? 8 : a.ntr <= 10 ? 10 : 12) {
    case 2: hipLaunchKernelGGL((gather_oct_kernel<T, 2>), grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((gather_oct_kernel<T, 4>), grid, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((gather_oct_kernel<T, 6>), grid, dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL((gather_oct_kernel<T, 8>), grid, dim3(256), 0, s, a); break;
    case 10: hipLaunchKernelGGL((gather_oct_kernel<T, 10>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((gather_oct_kernel<T, 12>), grid, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}
hipError_t launch_gather_oct(hipStream_t s, const GatherOctArgs<float>& a) { return do_gather_oct(s, a); }
hipError_t launch_gather_oct(hipStream_t s, const GatherOctArgs<double>& a) { return do_gather_oct(s, a); }

hipError_t launch_march_oct(hipStream_t s, const OctMarchArgs<float>& a, int groups, bool accum, int lanes)
{
    return dispatch_oct(s, a, groups, accum, lanes);
}
hipError_t launch_march_oct(hipStream_t s, const OctMarchArgs<double>& a, int groups, bool accum, int lanes)
{
    return dispatch_oct(s, a, groups, accum, lanes);
}

hipError_t launch_serve_tick(hipStream_t s, const ServeTables& tb, const ServeGrid& g)
{
    hipLaunchKernelGGL(serve_prepare_kernel, dim3(g.cell_blocks), dim3(256), 0, s, tb.models, tb.cell_items,
                       tb.n_cell);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(serve_march_kernel, dim3(g.march_blocks), dim3(256), g.march_lds, s, tb.models,
                       tb.march_items, tb.n_march);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(serve_se_kernel, dim3(g.se_blocks), dim3(g.se_bs), g.se_lds, s, tb.models, tb.se_items,
                       tb.n_se);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(serve_copy_kernel, dim3(g.cell_blocks), dim3(256), 0, s, tb.models, tb.cell_items,
                       tb.n_cell);
    return hipGetLastError();
}

hipError_t serve_set_attributes(const ServeGrid& g)
{
    hipError_t e = hipSuccess;
    if (g.march_lds > 65536)
        e = hipFuncSetAttribute((const void*)serve_march_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                g.march_lds);
    if (e == hipSuccess && g.se_lds > 65536)
        e = hipFuncSetAttribute((const void*)serve_se_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                g.se_lds);
    return e;
}

hipError_t launch_se(hipStream_t s, const SEArgs& a0)
{
    SEArgs a = a0;
    // up to 12 levels: the matrix in registers, 256 threads per workgroup
    const dim3 rg((a.nc + 255) / 256), rb(256);
    switch (a.L) {
    case 2: hipLaunchKernelGGL(se_reg_kernel<2>, rg, rb, 0, s, a); return hipGetLastError();
    case 3: hipLaunchKernelGGL(se_reg_kernel<3>, rg, rb, 0, s, a); return hipGetLastError();
    case 4: hipLaunchKernelGGL(se_reg_kernel<4>, rg, rb, 0, s, a); return hipGetLastError();
    case 5: hipLaunchKernelGGL(se_reg_kernel<5>, rg, rb, 0, s, a); return hipGetLastError();
    case 6: hipLaunchKernelGGL(se_reg_kernel<6>, rg, rb, 0, s, a); return hipGetLastError();
    case 7: hipLaunchKernelGGL(se_reg_kernel<7>, rg, rb, 0, s, a); return hipGetLastError();
    case 8: hipLaunchKernelGGL(se_reg_kernel<8>, rg, rb, 0, s, a); return hipGetLastError();
    case 9: hipLaunchKernelGGL(se_reg_kernel<9>, rg, rb, 0, s, a); return hipGetLastError();
    case 10: hipLaunchKernelGGL(se_reg_kernel<10>, rg, rb, 0, s, a); return hipGetLastError();
    case 11: hipLaunchKernelGGL(se_reg_kernel<11>, rg, rb, 0, s, a); return hipGetLastError();
    case 12: hipLaunchKernelGGL(se_reg_kernel<12>, rg, rb, 0, s, a); return hipGetLastError();
    default: break;
    }
    // LDS per thread: (L*(L+1) + L) doubles; block size = the largest power
    // of two (<= 256) that keeps the block within 64 KB.
    const size_t per = (size_t)(a.L * (a.L + 1) + a.L) * sizeof(double);
    int bs = 256;
    while (bs > 1 && per * bs > 65536) bs >>= 1;
    a.bs = bs;
    const size_t shm = per * bs;
    hipLaunchKernelGGL(se_kernel, dim3((a.nc + bs - 1) / bs), dim3(bs), shm, s, a);
    return hipGetLastError();
}

}  // namespace miloc
