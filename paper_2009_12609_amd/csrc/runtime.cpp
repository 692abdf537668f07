// runtime.cpp -- the C ABI of libmiloc (include/miloc.h): context state, input
// validation, device buffers and the iteration driver (Sect. 2: alternate the
// ray march and the equilibrium solve until the populations converge).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "geometry.h"
#include "octree.h"
#include "miloc.h"
#include "miloc_internal.h"

using namespace miloc;

namespace {

// CODATA-2018 exact h, k_B, c (CGS); atomic mass unit.
constexpr double kH = 6.62607015e-27;
constexpr double kK = 1.380649e-16;
constexpr double kC = 2.99792458e10;
constexpr double kAmu = 1.66053906660e-24;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtLog2e = 1.2011224087864498;   // sqrt(log2(e))
// Channel window half-widths in Doppler widths: the profile beyond is below
// e^-25 (FP32) / e^-42 (FP64) of its peak, i.e. far below the arithmetic's
// rounding level.
constexpr double kWindowK32 = 5.0;
constexpr double kWindowK64 = 6.5;

// A device region that DevBufs carve their storage from instead of calling
// hipMalloc, while it is installed on the calling thread (the allocation-free
// entry point installs the library's static scratch for the duration of one
// call).  Bump allocation in 256-byte units; nothing is returned before the
// region is uninstalled.
struct ScratchCarve {
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    bool overflow = false;
};
thread_local ScratchCarve* tls_carve = nullptr;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool carved = false;                 // storage from a ScratchCarve (not freed)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p && !carved) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        carved = false;
    }
    hipError_t ensure(size_t n)
    {
        if (n == 0) n = 8;
        if (p && bytes == n) return hipSuccess;
        release();
        if (ScratchCarve* sc = tls_carve) {
            const size_t off = (sc->used + 255) & ~(size_t)255;
            if (off > sc->size || n > sc->size - off) {
                sc->overflow = true;
                return hipErrorOutOfMemory;
            }
            p = sc->base + off;
            sc->used = off + n;
            bytes = n;
            carved = true;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) { p = nullptr; return e; }
        bytes = n;
        return hipSuccess;
    }
    template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

struct Status {
    miloc_status code;
};

}  // namespace

struct miloc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    hipEvent_t ev[6] = {};

    // molecule
    bool has_mol = false;
    int L = 0, T = 0;
    std::vector<double> E, g, A, nu, gamma;
    std::vector<int> up, lo;
    double mass_amu = 0;

    // model
    int kind = 0;   // 1: 1D shells, 3: 3D regular grid, 4: octree
    int64_t nc = 0;
    std::vector<double> R, nH2, Tk, bt, vr, X, impact;   // 1D (FP64)
    int nrays = 0;
    int N = 0;
    double delta = 0;
    std::vector<float> f_nH2, f_T, f_bt, f_vx, f_vy, f_vz, f_X;   // 3D
    OctModel oct;                                                 // octree structure

    // settings
    bool has_spec = false;
    int nch = 0;
    double vmin = 0, dv = 0;
    double Tbg = 2.73;
    std::vector<double> dirs;
    int precision = MILOC_MARCH_FP32;

    // device state
    bool dirty = true;        // static buffers need a rebuild
    bool base_ready = false;  // molecule + per-cell base arrays uploaded
    bool has_pops = false;
    bool has_rad = false;
    DevBuf d_mol, d_x, d_xnew, d_nH2, d_T, d_q, d_nmolLb, d_cellv, d_ke, d_acc, d_Ibg, d_Ibg64,
        d_zero, d_dirs, d_steps, d_flags, d_R, d_vrdv, d_area, d_vel, d_bD, d_win, d_lstart, d_moves, d_rbase, d_spanw,
        d_qlist, d_E, d_osteps, d_olen64, d_otrees, d_oaw, d_ostack, d_ocounter, d_ocell_off, d_ocell_steps, d_odir_off, d_oE, d_1steps, d_1off, d_1kmin;
    int64_t oct_trees = 0;
    int oct_depth = 0, oct_groups = 0;
    int64_t total_steps = 0;
    int trans_chunk = 1;
    int oct_estride = 1;                 // row stride (transitions) of the octree per-step sums
    int qcount[3] = {0, 0, 0}, qoff[3] = {0, 0, 0};
    std::vector<double> Iscale, Ibg;   // per transition: 2 h nu^3 / c^2, background (occupation)
    std::vector<double> Rn;            // 1D: outer radii / R_out
    // 1D spectra: step tables of the last requested lines of sight (reused
    // while the model, precision and impact parameters stay the same)
    std::vector<double> los_b;
    bool los_fp64 = false, los_valid = false;
    DevBuf d_los_b, d_los_steps, d_los_off, d_los_kmin, d_los_out;
    std::vector<double> q_host;
    int lanes = 32;
    double steps_per_trans = 0;
    double chalf = 0;
    double Kw = 0;
    int n_dir_dev = 0;
    // sub-iterations in the optically thick core of a 1D model
    int n_sub = 0;
    double sub_tau_min = 0.0;
    double sums_budget = 0.0;            // device bytes left for the 3D per-step sums (check_fits)
    int tbatch = 0;                      // 1D: all transitions of a ray in one pass
    // regular grids, FP32 single line: channel base of every (direction, ray)
    // (d_rbase) and the largest ray span, for the lane count span_lanes (0:
    // not built)
    int span_lanes = 0, span_w = 0;
    int sub_last_k = -1;                 // core extent of the last iteration (-1: none)
    std::vector<int> kmin_host;          // innermost shell of each ray (1D)
    DevBuf d_ient, d_sflags;             // core entry intensities; flags of the core solves
    std::vector<DirDev> dir_host;
    // hyperfine multiplets per transition: offsets (cm/s) and strengths
    // normalised to sum 1; empty = single Gaussian
    std::vector<std::vector<double>> hf_v, hf_w;
    int hfk = 0;                 // components per transition in d_hf (0: no multiplets)
    bool oct_lattice = false;    // octree rays: brute-force lattice instead of the created rays
    double hf_lo = 0, hf_hi = 0; // lowest / highest offset over all transitions, channels
    DevBuf d_hf;                 // [T][hfk] {offset / dv, strength}, zero-strength padding

    miloc_counters ctr{};

    // device bytes held in the context's buffers
    size_t device_bytes() const
    {
        const DevBuf* all[] = {&d_mol, &d_x, &d_xnew, &d_nH2, &d_T, &d_q, &d_nmolLb, &d_cellv, &d_ke, &d_acc,
                               &d_Ibg, &d_Ibg64, &d_zero, &d_dirs, &d_steps, &d_flags, &d_R, &d_vrdv, &d_area,
                               &d_vel, &d_bD, &d_win, &d_lstart, &d_moves, &d_qlist, &d_E, &d_osteps, &d_olen64,
                               &d_otrees, &d_oaw, &d_ostack, &d_ocounter, &d_ocell_off, &d_ocell_steps, &d_odir_off, &d_oE,
                               &d_1steps, &d_1off, &d_1kmin, &d_los_b, &d_los_steps, &d_los_off, &d_los_kmin,
                               &d_los_out, &d_hf, &d_ient, &d_sflags, &d_rbase, &d_spanw};
        size_t n = 0;
        for (const DevBuf* b : all) n += b->carved ? 0 : b->bytes;
        return n;
    }
};

namespace {

miloc_status fail(miloc_ctx* c, miloc_status code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail((ctx), _e == hipErrorOutOfMemory ? MILOC_ENOMEM : MILOC_EDEVICE,     \
                        std::string(#expr) + ": " + hipGetErrorString(_e));                 \
    } while (0)

// Timing events of a context; the allocation-free call runs on a context
// without events (and keeps no timings): there a record is skipped, a wait
// on an event waits for the stream and an elapsed time reads 0.
hipError_t ev_record(miloc_ctx* c, int i)
{
    return c->ev[i] ? hipEventRecord(c->ev[i], c->stream) : hipSuccess;
}
hipError_t ev_sync(miloc_ctx* c, int i)
{
    return c->ev[i] ? hipEventSynchronize(c->ev[i]) : hipStreamSynchronize(c->stream);
}
hipError_t ev_elapsed(miloc_ctx* c, float* ms, int a, int b)
{
    *ms = 0.0f;
    return c->ev[a] && c->ev[b] ? hipEventElapsedTime(ms, c->ev[a], c->ev[b]) : hipSuccess;
}

bool finite_all(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}
bool finite_all(const float* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}
template <typename T>
bool nonneg_all(const T* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!(a[i] >= 0)) return false;
    return true;
}
template <typename T>
bool positive_all(const T* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!(a[i] > 0)) return false;
    return true;
}

double doppler_b(double T, double bturb, double mass_amu)
{
    return std::sqrt(2.0 * kK * T / (mass_amu * kAmu) + bturb * bturb);
}

// Per-cell fields as FP64 regardless of model type.
struct CellView {
    const miloc_ctx* c;
    double nH2(int64_t k) const { return c->kind == 1 ? c->nH2[k] : (double)c->f_nH2[k]; }
    double T(int64_t k) const { return c->kind == 1 ? c->Tk[k] : (double)c->f_T[k]; }
    double bt(int64_t k) const { return c->kind == 1 ? c->bt[k] : (double)c->f_bt[k]; }
    double X(int64_t k) const { return c->kind == 1 ? c->X[k] : (double)c->f_X[k]; }
};

// Device bytes a context holds for a model (kind 1: shells, 3: regular
// grid, 4: octree): `fixed` for the populations, opacities, sums, per-cell
// data, the channel-window table and the ray tables, `sums` for the 3D
// march's per-step partial sums per transition of a launch.  steps: ray-cell
// steps of one transition (1D rays, the regular grid's crossing patterns per
// representative ray, or the octree schedule); rays: 1D rays, or rays per
// direction of a regular grid; trees: octree work units.
struct Footprint {
    size_t fixed = 0;
    size_t sums = 0;
};

Footprint footprint_of(int kind, int64_t nc, int L, int T, int nch, int n_dir, bool fp64, int64_t steps,
                       int64_t rays, int64_t trees)
{
    const size_t tsz = fp64 ? sizeof(double) : sizeof(float);
    const size_t c = (size_t)nc;
    Footprint f;
    f.fixed = sizeof(MolDev) + 16 + 2 * c * L * sizeof(double) + 4 * c * sizeof(double) +
              (size_t)T * c * (2 * tsz + sizeof(double2)) + (size_t)3 * T * sizeof(double);
    if (kind == 1) {
        f.fixed += c * (2 * sizeof(double) + 2 * tsz) + (size_t)rays * (2 * sizeof(double) + sizeof(int64_t) + sizeof(int)) +
                   (size_t)steps * 2 * tsz;
        return f;
    }
    f.fixed += c * (sizeof(float4) + sizeof(double)) + (size_t)n_dir * c * 4 * tsz + (size_t)n_dir * sizeof(DirDev);
    if (kind == 3) {
        const int64_t N = (int64_t)std::llround(std::cbrt((double)nc));
        // step records and moves, layer starts, the rays' channel bases
        f.fixed += (size_t)steps * (sizeof(StepRec<double>) + sizeof(int2)) + (size_t)n_dir * (N + 1) * sizeof(int) +
                   (size_t)n_dir * (size_t)rays * sizeof(int);
        f.sums = (size_t)steps * (size_t)rays * 2 * tsz;
    } else {
        // cell step lists, step records (+ FP64 lengths), work units, and at
        // most 2 GiB of saved-vector stacks
        f.fixed += (c + 1) * sizeof(int64_t) + (size_t)steps * (sizeof(uint32_t) + sizeof(uint2)) +
                   (fp64 ? (size_t)steps * sizeof(double) : 0) + (size_t)trees * sizeof(OctTreeRec) +
                   ((size_t)2 << 30);
        // FP32 rows hold an even number of transitions (16-byte rows)
        f.sums = (size_t)steps * 2 * tsz * (fp64 ? 1 : 2);
    }
    return f;
}

// Refuses (MILOC_ENOMEM, before the model's static arrays are allocated) a
// model whose arrays and tables plus one transition's per-step sums exceed
// the device memory this context can use: the free memory plus what it holds
// already, capped by MILOC_DEVICE_BUDGET_GB when set.  *sums_budget receives
// the bytes left for the per-step sums.
miloc_status check_fits(miloc_ctx* c, const Footprint& f, double* sums_budget)
{
    size_t free_b = 0, total_b = 0;
    HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
    double avail = (double)free_b + (double)c->device_bytes();
    if (const char* ev = std::getenv("MILOC_DEVICE_BUDGET_GB")) avail = std::min(avail, std::atof(ev) * 1e9);
    const double need = (double)f.fixed + (double)f.sums;
    if (need > avail) {
        char buf[320];
        std::snprintf(buf, sizeof buf,
                      "the model needs %.3f GB of device memory (%.3f GB of arrays and ray tables, %.3f GB of "
                      "per-step sums for one transition); %.3f GB are available",
                      need * 1e-9, (double)f.fixed * 1e-9, (double)f.sums * 1e-9, avail * 1e-9);
        return fail(c, MILOC_ENOMEM, buf);
    }
    *sums_budget = avail - (double)f.fixed;
    return MILOC_OK;
}

// Molecule and per-cell base arrays (needs molecule + model).
miloc_status ensure_base(miloc_ctx* c)
{
    if (!c->has_mol || c->kind == 0) return fail(c, MILOC_ESTATE, "molecule and model must be loaded first");
    if (c->base_ready) return MILOC_OK;
    MolDev m;
    std::memset(&m, 0, sizeof(m));
    m.L = c->L;
    m.T = c->T;
    const double Emin = *std::min_element(c->E.begin(), c->E.end());
    for (int i = 0; i < c->L; ++i) {
        m.E[i] = c->E[i] - Emin;
        m.g[i] = c->g[i];
    }
    for (int u = 0; u < c->L; ++u)
        for (int l = 0; l < u; ++l) m.gamma[u * c->L + l] = c->gamma[(size_t)u * c->L + l];
    for (int t = 0; t < c->T; ++t) {
        m.up[t] = c->up[t];
        m.lo[t] = c->lo[t];
        m.A[t] = c->A[t];
        m.gratio[t] = c->g[c->up[t]] / c->g[c->lo[t]];
        m.Ct[t] = kC * kC * kC * c->A[t] / (8.0 * kPi * c->nu[t] * c->nu[t] * c->nu[t]);
    }
    mol_pair_table(m);
    HIPCHK(c, c->d_mol.ensure(sizeof(MolDev)));
    HIPCHK(c, hipMemcpy(c->d_mol.p, &m, sizeof(MolDev), hipMemcpyHostToDevice));
    const int64_t nc = c->nc;
    std::vector<double> a(nc), b(nc);
    CellView cv{c};
    for (int64_t k = 0; k < nc; ++k) { a[k] = cv.nH2(k); b[k] = cv.T(k); }
    HIPCHK(c, c->d_nH2.ensure(nc * sizeof(double)));
    HIPCHK(c, c->d_T.ensure(nc * sizeof(double)));
    HIPCHK(c, hipMemcpy(c->d_nH2.p, a.data(), nc * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_T.p, b.data(), nc * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, c->d_x.ensure((size_t)nc * c->L * sizeof(double)));
    HIPCHK(c, c->d_xnew.ensure((size_t)nc * c->L * sizeof(double)));
    HIPCHK(c, c->d_flags.ensure(16));
    c->Iscale.resize(c->T);
    for (int t = 0; t < c->T; ++t) c->Iscale[t] = 2.0 * kH * std::pow(c->nu[t], 3) / (kC * kC);
    c->base_ready = true;
    return MILOC_OK;
}

// The marches' maser flag: the fourth 32-bit word of d_flags (after the
// convergence maximum and the failure counter of the equilibrium solve).
unsigned* maser_flag(miloc_ctx* c)
{
    return reinterpret_cast<unsigned*>(c->d_flags.as<char>() + 12);
}

template <typename TT>
void pack_cell_static(miloc_ctx* c, const std::vector<double>& b, std::vector<char>& out)
{
    // 1D shells: {v_r / dv, sqrt(log2 e) dv / b}
    const int64_t nc = c->nc;
    const double ibs_f = c->dv * kSqrtLog2e;
    using T2 = typename V2<TT>::type;
    out.resize(nc * sizeof(T2));
    T2* v = reinterpret_cast<T2*>(out.data());
    for (int64_t k = 0; k < nc; ++k) {
        v[k].x = (TT)(c->vr[k] / c->dv);
        v[k].y = (TT)(ibs_f / b[k]);
    }
}

// The length field of a regular-grid step record (see StepRec).
template <typename TT>
TT step_len_rec(double len)
{
    if (sizeof(TT) == sizeof(double)) return (TT)len;
    return (TT)std::log2(len);
}

template <typename TT>
miloc_status upload_steps(miloc_ctx* c, const std::vector<double>& len, const std::vector<int>& fl)
{
    std::vector<StepRec<TT>> st(len.size());
    for (size_t i = 0; i < len.size(); ++i) {
        st[i].len = step_len_rec<TT>(len[i]);
        st[i].flags = fl[i];
    }
    HIPCHK(c, c->d_steps.ensure(std::max<size_t>(1, st.size()) * sizeof(StepRec<TT>)));
    HIPCHK(c, hipMemcpy(c->d_steps.p, st.data(), st.size() * sizeof(StepRec<TT>),
                        hipMemcpyHostToDevice));
    return MILOC_OK;
}

// 1D: step records {len / R_out, Doppler shift in channels} of rays with the
// given impact parameters (/ R_out), built on the device; first step and
// innermost shell of each ray.
miloc_status upload_ray_steps(miloc_ctx* c, const std::vector<double>& bn, bool fp64, DevBuf& steps, DevBuf& off,
                              DevBuf& kmin)
{
    const int n = (int)c->nc;
    std::vector<int64_t> o;
    std::vector<int> km;
    const int64_t total = shell_ray_layout(n, c->Rn.data(), (int)bn.size(), bn.data(), o, km);
    DevBuf db;
    HIPCHK(c, db.ensure(std::max<size_t>(1, bn.size()) * sizeof(double)));
    HIPCHK(c, hipMemcpy(db.p, bn.data(), bn.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, off.ensure(std::max<size_t>(1, o.size()) * sizeof(int64_t)));
    HIPCHK(c, hipMemcpy(off.p, o.data(), o.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(c, kmin.ensure(std::max<size_t>(1, km.size()) * sizeof(int)));
    HIPCHK(c, hipMemcpy(kmin.p, km.data(), km.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, steps.ensure(std::max<int64_t>(1, total) * (fp64 ? sizeof(double2) : sizeof(float2))));
    HIPCHK(c, launch_ray_steps(c->stream, n, c->d_R.as<double>(), (int)bn.size(), db.as<double>(), kmin.as<int>(),
                               off.as<long long>(), c->d_vrdv.as<double>(), steps.p, fp64));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MILOC_OK;
}

// Build the direction table and step patterns for a list of directions, with
// the per-direction layer starts and cumulative transverse moves.
void build_patterns(int N, const std::vector<double>& dirs, std::vector<DirDev>& dd,
                    std::vector<double>& len, std::vector<int>& fl, std::vector<DirPattern>* keep,
                    std::vector<int>* lstart = nullptr, std::vector<int2>* moves = nullptr)
{
    const int nd = (int)dirs.size() / 3;
    const int64_t stride[3] = {1, N, (int64_t)N * N};
    dd.assign(nd, DirDev{});
    len.clear();
    fl.clear();
    if (lstart) lstart->clear();
    if (moves) moves->clear();
    for (int q = 0; q < nd; ++q) {
        const double* d = &dirs[3 * q];
        DirPattern P = regular_pattern(d, N);
        DirDev& D = dd[q];
        D.d[0] = d[0]; D.d[1] = d[1]; D.d[2] = d[2];
        D.aw = P.aw;
        D.sa = d[P.a] >= 0 ? 1 : -1;
        D.sb = d[P.b] >= 0 ? 1 : -1;
        D.sta = (int)stride[P.a];
        D.stb = (int)stride[P.b];
        const bool fwd = d[P.m] > 0;
        D.stride_m = fwd ? (int)stride[P.m] : -(int)stride[P.m];
        D.start_off = fwd ? 0 : (int)((N - 1) * stride[P.m]);
        D.step0 = (int)len.size();
        D.nsteps = (int)P.len.size();
        D.m = P.m;
        D.fwd = fwd ? 1 : 0;
        D.lstart0 = lstart ? (int)lstart->size() : 0;
        D.maxlen = P.len.empty() ? 0.0 : *std::max_element(P.len.begin(), P.len.end());
        len.insert(len.end(), P.len.begin(), P.len.end());
        fl.insert(fl.end(), P.flags.begin(), P.flags.end());
        if (lstart) lstart->insert(lstart->end(), P.layer_start.begin(), P.layer_start.end());
        if (moves)
            for (size_t i = 0; i < P.na.size(); ++i) moves->push_back(make_int2(P.na[i], P.nb[i]));
        if (keep) keep->push_back(std::move(P));
    }
}

int host_threads()
{
    const unsigned n = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, n));
}

// Upload an octree schedule; returns the device buffers through the arguments.
miloc_status upload_oct_schedule(miloc_ctx* c, const OctSchedule& S, DevBuf& steps, DevBuf& trees)
{
    HIPCHK(c, steps.ensure(std::max<size_t>(1, S.rec.size()) * sizeof(uint32_t)));
    HIPCHK(c, hipMemcpy(steps.p, S.rec.data(), S.rec.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPCHK(c, trees.ensure(std::max<size_t>(1, S.trees.size()) * sizeof(OctTreeRec)));
    HIPCHK(c, hipMemcpy(trees.p, S.trees.data(), S.trees.size() * sizeof(OctTreeRec), hipMemcpyHostToDevice));
    return MILOC_OK;
}

// Octree: ray schedules of every direction, direction table, weights W
// (root-cell units) and the persistent-group stack.
miloc_status build_octree_march(miloc_ctx* c, std::vector<double>& W)
{
    const int nd = (int)c->dirs.size() / 3;
    OctSchedule S;
    const bool fp64 = c->precision == MILOC_MARCH_FP64;
    const std::string e = octree_schedule(c->oct, c->dirs, c->oct_lattice ? OctRays::Lattice : OctRays::Scheme,
                                          host_threads(), S, fp64, c->nc);
    if (!e.empty()) return fail(c, MILOC_EINVAL, e);
    miloc_status fit = check_fits(c, footprint_of(4, c->nc, c->L, c->T, c->nch, nd, fp64, S.n_steps, 0,
                                                  (int64_t)S.trees.size()),
                                  &c->sums_budget);
    if (fit != MILOC_OK) return fit;
    HIPCHK(c, c->d_ocell_off.ensure(S.cell_off.size() * sizeof(int64_t)));
    HIPCHK(c, hipMemcpy(c->d_ocell_off.p, S.cell_off.data(), S.cell_off.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice));
    HIPCHK(c, c->d_ocell_steps.ensure(std::max<size_t>(1, S.cell_steps.size()) * sizeof(uint32_t)));
    HIPCHK(c, hipMemcpy(c->d_ocell_steps.p, S.cell_steps.data(), S.cell_steps.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice));
    std::vector<uint32_t>().swap(S.cell_steps);
    {
        std::vector<uint32_t> doff(S.dir_off.begin(), S.dir_off.end());
        HIPCHK(c, c->d_odir_off.ensure(doff.size() * sizeof(uint32_t)));
        HIPCHK(c, hipMemcpy(c->d_odir_off.p, doff.data(), doff.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    }
    // per-step sums: as many transitions per launch as fit the budget
    {
        // a launch lasts at least as long as its longest tree, so all
        // transitions go in one launch when they fit
        double budget_gb = 160.0;
        if (const char* ev = std::getenv("MILOC_STEP_BUFFER_GB")) budget_gb = std::atof(ev);
        budget_gb = std::min(budget_gb, c->sums_budget * 1e-9);
        const size_t per_t = (size_t)std::max<int64_t>(1, S.n_steps) * 2 * (fp64 ? sizeof(double) : sizeof(float));
        // FP32 rows padded to an even number of transitions (16-byte rows)
        auto stride_of = [&](int tc) { return fp64 ? tc : (tc + 1) / 2 * 2; };
        int tc = (int)std::min<double>((double)c->T, std::floor(budget_gb * 1e9 / (double)per_t));
        while (tc > 1 && (double)stride_of(tc) * per_t > budget_gb * 1e9) --tc;
        c->trans_chunk = tc < 1 ? 1 : tc;
        c->oct_estride = stride_of(c->trans_chunk);
        // slack: the gather reads whole tiles of up to 12 transitions past the last row
        HIPCHK(c, c->d_oE.ensure(per_t * c->oct_estride + 12 * 2 * sizeof(double)));
    }
    if (fp64) {
        HIPCHK(c, c->d_olen64.ensure(std::max<size_t>(1, S.len64.size()) * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->d_olen64.p, S.len64.data(), S.len64.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        c->d_olen64.release();
    }
    std::vector<DirDev> dd(nd);
    std::vector<double> aw(nd);
    for (int q = 0; q < nd; ++q) {
        const double* d = &c->dirs[3 * (size_t)q];
        DirDev& D = dd[q];
        D.d[0] = d[0]; D.d[1] = d[1]; D.d[2] = d[2];
        D.m = main_axis(d);
        D.aw = std::fabs(d[D.m]);
        aw[q] = D.aw;
    }
    // per direction every leaf of level L carries h_L^3 of sum a s (Sect. 2.2:
    // equal path length per cell for each direction)
    for (int64_t k = 0; k < c->nc; ++k) {
        const double hl = std::ldexp(1.0, -(int)c->oct.level[k]);
        W[k] = c->oct.child[k] >= 0 ? 0.0 : nd * hl * hl * hl;
    }
    c->dir_host = dd;
    c->n_dir_dev = nd;
    c->steps_per_trans = (double)S.n_steps;
    c->total_steps = S.n_steps;
    c->oct_trees = (int64_t)S.trees.size();
    c->oct_depth = S.max_depth;
    HIPCHK(c, c->d_dirs.ensure(dd.size() * sizeof(DirDev)));
    HIPCHK(c, hipMemcpy(c->d_dirs.p, dd.data(), dd.size() * sizeof(DirDev), hipMemcpyHostToDevice));
    HIPCHK(c, c->d_oaw.ensure(aw.size() * sizeof(double)));
    HIPCHK(c, hipMemcpy(c->d_oaw.p, aw.data(), aw.size() * sizeof(double), hipMemcpyHostToDevice));
    miloc_status st = upload_oct_schedule(c, S, c->d_osteps, c->d_otrees);
    if (st != MILOC_OK) return st;
    // persistent groups: 8 blocks of 16 groups per compute unit, fewer if the
    // saved-vector stacks would pass 2 GB
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDeviceProperties(&prop, c->device));
    const size_t tsz = c->precision == MILOC_MARCH_FP64 ? sizeof(double) : sizeof(float);
    const size_t per_group = (size_t)std::max(1, c->oct_depth) * oct_stride(c->nch, (int)tsz) * tsz;
    const int gpb = 256 / c->lanes;       // lane groups per 256-thread block
    int64_t groups = (int64_t)prop.multiProcessorCount * 8 * gpb;
    groups = std::min<int64_t>(groups, std::max<int64_t>(gpb, (int64_t)((2ull << 30) / per_group)));
    groups = std::min<int64_t>(groups, std::max<int64_t>(gpb, c->oct_trees * c->T));
    groups = (groups + gpb - 1) / gpb * gpb;
    c->oct_groups = (int)groups;
    HIPCHK(c, c->d_ostack.ensure((size_t)groups * per_group));
    HIPCHK(c, c->d_ocounter.ensure(sizeof(unsigned long long)));
    return MILOC_OK;
}

template <typename TT>
miloc_status launch_oct(miloc_ctx* c, int ntr, int toff, bool accum, TT* Iout, const DevBuf& steps,
                        const DevBuf& trees, int64_t n_trees, const double* aw, const void* win, int groups,
                        const double* len64)
{
    OctMarchArgs<TT> a{};
    a.nc = (int)c->nc;
    a.nch = c->nch;
    a.ich = oct_stride(c->nch, (int)sizeof(TT));
    a.ntr = ntr;
    a.trans_offset = toff;
    a.ntr_total = c->T;
    a.n_items = (long long)n_trees * ntr;
    a.trees = trees.as<OctTreeRec>();
    a.steps = steps.as<uint2>();
    a.len64 = len64;
    a.aw = aw;
    a.win = reinterpret_cast<const typename V4<TT>::type*>(win);
    a.ke = c->d_ke.as<typename V2<TT>::type>();
    a.Ibg = accum ? c->d_Ibg.as<TT>() : c->d_zero.as<TT>();
    a.E = accum ? c->d_oE.as<typename V2<TT>::type>() : nullptr;
    a.estride = c->oct_estride;
    a.Iout = Iout;
    a.counter = c->d_ocounter.as<unsigned long long>();
    a.stack = c->d_ostack.as<TT>();
    a.depth = accum ? c->oct_depth : 0;
    a.hf = c->hfk ? c->d_hf.as<typename V2<TT>::type>() : nullptr;
    a.hfk = c->hfk;
    a.maser = maser_flag(c);
    HIPCHK(c, launch_march_oct(c->stream, a, groups, accum, c->lanes));
    return MILOC_OK;
}

// Everything the march needs beyond the base arrays (needs the spectral grid).
miloc_status ensure_static(miloc_ctx* c)
{
    miloc_status st = ensure_base(c);
    if (st != MILOC_OK) return st;
    if (!c->has_spec) return fail(c, MILOC_ESTATE, "spectral grid not set");
    if (!c->dirty) return MILOC_OK;
    c->los_valid = false;
    const bool fp64 = c->precision == MILOC_MARCH_FP64;
    const int64_t nc = c->nc;
    CellView cv{c};
    std::vector<double> b(nc);
    double maxu = 0, maxb = 0;
    for (int64_t k = 0; k < nc; ++k) {
        b[k] = doppler_b(cv.T(k), cv.bt(k), c->mass_amu);
        maxb = std::max(maxb, b[k]);
        double u;
        if (c->kind >= 3) {
            const double ux = c->f_vx[k], uy = c->f_vy[k], uz = c->f_vz[k];
            u = std::sqrt(ux * ux + uy * uy + uz * uz);
        } else {
            u = std::fabs(c->vr[k]);
        }
        maxu = std::max(maxu, u + 5.0 * b[k]);
    }
    // hyperfine components widen the line by their offset range
    double vlo = 0.0, vhi = 0.0;
    int hfk = 0;
    for (int t = 0; t < c->T; ++t) {
        hfk = std::max(hfk, (int)c->hf_v[t].size());
        for (double v : c->hf_v[t]) {
            vlo = std::min(vlo, v);
            vhi = std::max(vhi, v);
        }
    }
    const double vmax = c->vmin + c->nch * c->dv;
    if (-maxu + vlo < c->vmin || maxu + vhi > vmax) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "velocity band [%g, %g] cm/s does not contain the line: |v| + 5 b = %g cm/s "
                      "beyond the component offsets [%g, %g] cm/s",
                      c->vmin, vmax, maxu, vlo, vhi);
        return fail(c, MILOC_EINVAL, buf);
    }
    c->hfk = hfk;
    c->hf_lo = vlo / c->dv;
    c->hf_hi = vhi / c->dv;
    const double Kd = fp64 ? kWindowK64 : kWindowK32;
    c->Kw = Kd * kSqrtLog2e;
    c->chalf = 0.5 + c->vmin / c->dv;
    // lanes per ray: the widest channel window over the cells (at most wmax
    // channels) is covered in one to three passes of the ray's lane group
    const double wmax = 2.0 * Kd * maxb / c->dv + 2.0 + (vhi - vlo) / c->dv;
    if (c->kind == 3)
        c->lanes = wmax <= 64.0 ? 8 : (wmax <= 128.0 ? 16 : 32);   // 8: measured faster up to ~64
    else if (c->kind == 4)
        c->lanes = 8;                     // octree: groups of 8 (measured faster than 16), any window width
    else
        c->lanes = 16;                    // 1D: groups of 16, any window width
    if (const char* ev = std::getenv("MILOC_LANES")) {
        const int l = std::atoi(ev);
        if ((c->kind == 1 && (l == 8 || l == 16 || l == 32 || l == 64)) || (c->kind == 4 && (l == 8 || l == 16)) ||
            (c->kind == 3 && (l == 8 || l == 16 || l == 32 || l == 64)))
            c->lanes = l;
    }

    // geometry, weights W (in march length units) and q = dv/(b sqrt(pi) W)
    std::vector<double> W(nc, 0.0);
    double Lunit;
    if (c->kind == 3) {
        const int N = c->N;
        Lunit = c->delta;
        std::vector<DirDev> dd;
        std::vector<double> len;
        std::vector<int> fl;
        std::vector<DirPattern> pats;
        std::vector<int> lst;
        std::vector<int2> mvs;
        build_patterns(N, c->dirs, dd, len, fl, &pats, &lst, &mvs);
        // W(cell) = sum over directions of aw * (path per ray in the cell's layer)
        std::vector<double> Wax[3];
        for (int a = 0; a < 3; ++a) Wax[a].assign(N, 0.0);
        double steps = 0;
        for (size_t q = 0; q < pats.size(); ++q) {
            const DirPattern& P = pats[q];
            const bool fwd = c->dirs[3 * q + P.m] > 0;
            for (int l = 0; l < N; ++l) Wax[P.m][fwd ? l : N - 1 - l] += P.aw * P.layer_len[l];
            steps += (double)P.len.size() * N * N;
        }
        for (int z = 0; z < N; ++z)
            for (int y = 0; y < N; ++y)
                for (int x = 0; x < N; ++x)
                    W[((int64_t)z * N + y) * N + x] = Wax[0][x] + Wax[1][y] + Wax[2][z];
        c->steps_per_trans = steps;
        c->dir_host = dd;
        c->n_dir_dev = (int)dd.size();
        c->total_steps = (int64_t)len.size();
        st = check_fits(c, footprint_of(3, nc, c->L, c->T, c->nch, (int)dd.size(), fp64, c->total_steps,
                                        (int64_t)N * N, 0),
                        &c->sums_budget);
        if (st != MILOC_OK) return st;
        HIPCHK(c, c->d_lstart.ensure(lst.size() * sizeof(int)));
        HIPCHK(c, hipMemcpy(c->d_lstart.p, lst.data(), lst.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(c, c->d_moves.ensure(mvs.size() * sizeof(int2)));
        HIPCHK(c, hipMemcpy(c->d_moves.p, mvs.data(), mvs.size() * sizeof(int2), hipMemcpyHostToDevice));
        std::vector<int> ql;
        for (int g = 0; g < 3; ++g) {
            c->qcount[g] = 0;
            c->qoff[g] = (int)ql.size();
            for (int q = 0; q < (int)dd.size(); ++q)
                if (dd[q].m == g) { ql.push_back(q); ++c->qcount[g]; }
        }
        HIPCHK(c, c->d_qlist.ensure(std::max<size_t>(1, ql.size()) * sizeof(int)));
        HIPCHK(c, hipMemcpy(c->d_qlist.p, ql.data(), ql.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(c, c->d_dirs.ensure(dd.size() * sizeof(DirDev)));
        HIPCHK(c, hipMemcpy(c->d_dirs.p, dd.data(), dd.size() * sizeof(DirDev), hipMemcpyHostToDevice));
        st = fp64 ? upload_steps<double>(c, len, fl) : upload_steps<float>(c, len, fl);
        if (st != MILOC_OK) return st;
    } else if (c->kind == 4) {
        Lunit = c->delta;
        st = build_octree_march(c, W);
        if (st != MILOC_OK) return st;
    } else {
        const int n = (int)c->nc;
        Lunit = c->R[n - 1];
        std::vector<double> Rn(n), bn(c->nrays), an(c->nrays);
        for (int k = 0; k < n; ++k) Rn[k] = c->R[k] / Lunit;
        Rn[n - 1] = 1.0;
        c->Rn = Rn;
        for (int j = 0; j < c->nrays; ++j) bn[j] = c->impact[j] / Lunit;
        // ray weights: annulus between the mid-points of neighbouring impact parameters
        for (int j = 0; j < c->nrays; ++j) {
            const double e0 = j == 0 ? 0.0 : 0.5 * (bn[j] + bn[j - 1]);
            const double e1 = j == c->nrays - 1 ? 1.0 : 0.5 * (bn[j] + bn[j + 1]);
            an[j] = kPi * (e1 * e1 - e0 * e0);
        }
        HIPCHK(c, c->d_area.ensure(c->nrays * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->d_area.p, an.data(), c->nrays * sizeof(double), hipMemcpyHostToDevice));
        std::vector<double> vrdv(n);
        for (int k = 0; k < n; ++k) vrdv[k] = c->vr[k] / c->dv;
        HIPCHK(c, c->d_R.ensure(n * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->d_R.p, Rn.data(), n * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, c->d_vrdv.ensure(n * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->d_vrdv.p, vrdv.data(), n * sizeof(double), hipMemcpyHostToDevice));
        st = upload_ray_steps(c, bn, fp64, c->d_1steps, c->d_1off, c->d_1kmin);
        if (st != MILOC_OK) return st;
        // ray-sampled volumes on the device (the rays' paths, FP64)
        {
            DevBuf db, dW;
            HIPCHK(c, db.ensure(c->nrays * sizeof(double)));
            HIPCHK(c, hipMemcpy(db.p, bn.data(), c->nrays * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(c, dW.ensure(n * sizeof(double)));
            HIPCHK(c, launch_shell_weights(c->stream, n, c->d_R.as<double>(), c->nrays, db.as<double>(),
                                           c->d_area.as<double>(), dW.as<double>()));
            HIPCHK(c, hipMemcpyAsync(W.data(), dW.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        std::vector<int64_t> o;
        c->steps_per_trans = (double)shell_ray_layout(n, Rn.data(), c->nrays, bn.data(), o, c->kmin_host);
    }
    std::vector<double> q(nc), nmolLb(nc);
    for (int64_t k = 0; k < nc; ++k) {
        const double bs = b[k] * std::sqrt(kPi);
        q[k] = W[k] > 0 ? c->dv / (bs * W[k]) : 0.0;
        if (c->kind == 4) {
            // the octree march leaves out the ray weight's h^2 (the leaf's
            // h_L with created rays, the finest h with the lattice); refined
            // cells are not solved
            const double hl = std::ldexp(1.0, -(c->oct_lattice ? c->oct.Lmax : (int)c->oct.level[k]));
            q[k] = c->oct.child[k] >= 0 ? -1.0 : q[k] * hl * hl;
        }
        nmolLb[k] = cv.nH2(k) * cv.X(k) * Lunit / bs;
    }
    c->q_host = q;
    HIPCHK(c, c->d_q.ensure(nc * sizeof(double)));
    HIPCHK(c, c->d_nmolLb.ensure(nc * sizeof(double)));
    HIPCHK(c, hipMemcpy(c->d_q.p, q.data(), nc * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_nmolLb.p, nmolLb.data(), nc * sizeof(double), hipMemcpyHostToDevice));
    const size_t tsz = fp64 ? sizeof(double) : sizeof(float);
    if (c->kind >= 3) {
        std::vector<float4> vel(nc);
        for (int64_t k = 0; k < nc; ++k) vel[k] = make_float4(c->f_vx[k], c->f_vy[k], c->f_vz[k], 0.0f);
        HIPCHK(c, c->d_vel.ensure(nc * sizeof(float4)));
        HIPCHK(c, c->d_bD.ensure(nc * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->d_vel.p, vel.data(), nc * sizeof(float4), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->d_bD.p, b.data(), nc * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, c->d_win.ensure((size_t)c->n_dir_dev * nc * 4 * tsz));
        HIPCHK(c, launch_window_table(c->stream, (int)nc, c->n_dir_dev, c->d_dirs.as<DirDev>(),
                                      c->d_vel.as<float4>(), c->d_bD.as<double>(), c->dv, c->chalf,
                                      Kd, c->nch, c->hf_lo, c->hf_hi, c->d_win.p, fp64));
        c->span_lanes = 0;                // the rays' channel spans follow the windows
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->d_cellv.release();
    } else {
        std::vector<char> cvb;
        if (fp64) pack_cell_static<double>(c, b, cvb); else pack_cell_static<float>(c, b, cvb);
        HIPCHK(c, c->d_cellv.ensure(cvb.size()));
        HIPCHK(c, hipMemcpy(c->d_cellv.p, cvb.data(), cvb.size(), hipMemcpyHostToDevice));
    }
    if (hfk > 0) {
        // transitions without a multiplet: one component at offset 0
        std::vector<double> tab((size_t)c->T * hfk * 2, 0.0);
        for (int t = 0; t < c->T; ++t) {
            double* row = tab.data() + (size_t)t * hfk * 2;
            if (c->hf_v[t].empty()) {
                row[1] = 1.0;
                continue;
            }
            for (size_t k = 0; k < c->hf_v[t].size(); ++k) {
                row[2 * k] = c->hf_v[t][k] / c->dv;
                row[2 * k + 1] = c->hf_w[t][k];
            }
        }
        HIPCHK(c, c->d_hf.ensure(tab.size() * tsz));
        if (fp64) {
            HIPCHK(c, hipMemcpy(c->d_hf.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        } else {
            std::vector<float> tf(tab.begin(), tab.end());
            HIPCHK(c, hipMemcpy(c->d_hf.p, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    } else {
        c->d_hf.release();
    }
    HIPCHK(c, c->d_ke.ensure((size_t)c->T * nc * 2 * tsz));
    HIPCHK(c, c->d_acc.ensure((size_t)c->T * nc * sizeof(double2)));
    if (c->kind == 3) {
        // per-step partial sums: as many transitions per march launch as fit the budget
        double budget_gb = 16.0;
        if (const char* ev = std::getenv("MILOC_STEP_BUFFER_GB")) budget_gb = std::atof(ev);
        budget_gb = std::min(budget_gb, c->sums_budget * 1e-9);
        const size_t per_t = (size_t)c->total_steps * c->N * c->N * 2 * tsz;
        int tc = (int)std::min<double>((double)c->T, std::floor(budget_gb * 1e9 / (double)per_t));
        c->trans_chunk = tc < 1 ? 1 : tc;
        HIPCHK(c, c->d_E.ensure(per_t * c->trans_chunk));
    }
    c->Ibg.resize(c->T);
    std::vector<char> ib(c->T * tsz);
    for (int t = 0; t < c->T; ++t) {
        const double xx = c->Tbg > 0 ? kH * c->nu[t] / (kK * c->Tbg) : INFINITY;
        c->Ibg[t] = std::isfinite(xx) ? 1.0 / std::expm1(xx) : 0.0;
        if (fp64) reinterpret_cast<double*>(ib.data())[t] = c->Ibg[t];
        else reinterpret_cast<float*>(ib.data())[t] = (float)c->Ibg[t];
    }
    HIPCHK(c, c->d_Ibg.ensure(ib.size()));
    HIPCHK(c, hipMemcpy(c->d_Ibg.p, ib.data(), ib.size(), hipMemcpyHostToDevice));
    HIPCHK(c, c->d_Ibg64.ensure(c->T * sizeof(double)));
    HIPCHK(c, hipMemcpy(c->d_Ibg64.p, c->Ibg.data(), c->T * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, c->d_zero.ensure(c->T * sizeof(double)));
    HIPCHK(c, hipMemset(c->d_zero.p, 0, c->T * sizeof(double)));
    c->dirty = false;
    return MILOC_OK;
}

void invalidate_model(miloc_ctx* c)
{
    c->los_valid = false;
    c->base_ready = false;
    c->dirty = true;
    c->has_pops = false;
    c->has_rad = false;
}

// March arguments of a 1D model's own ray set (every ray from I_bg, all of
// its steps, accumulation into acc).
template <typename TT>
void fill_march1d(miloc_ctx* c, int ntr, int toff, March1DArgs<TT>& a)
{
    a.n = (int)c->nc;
    a.nrays = c->nrays;
    a.nch = c->nch;
    a.ntr = ntr;
    a.trans_offset = toff;
    a.steps = c->d_1steps.as<typename V2<TT>::type>();
    a.ray_off = c->d_1off.as<long long>();
    a.kmin = c->d_1kmin.as<int>();
    a.area = c->d_area.as<double>();
    a.shellv = c->d_cellv.as<typename V2<TT>::type>();
    a.ke = c->d_ke.as<typename V2<TT>::type>();
    a.Ibg = c->d_Ibg.as<TT>();
    a.acc = c->d_acc.as<double2>();
    a.chalf = c->chalf;
    a.Kw = (TT)c->Kw;
    a.Iout = nullptr;
    a.ntr_total = c->T;
    a.hf = c->hfk ? c->d_hf.as<typename V2<TT>::type>() : nullptr;
    a.hfk = c->hfk;
    a.hf_lo = c->hf_lo;
    a.hf_hi = c->hf_hi;
    a.maser = maser_flag(c);
    a.seg = kSegWhole;
    a.core_k = 0;
    a.Ient = nullptr;
}

// Sub-iterations in the optically thick core of a 1D model (the paper's
// Sect. 4: populations updated more often where the lines are thick), after
// an iteration's global solve has left the new populations in d_x: the core
// is the shells 0..K, K the outermost shell whose radial line-centre optical
// depth to the surface (static gas, these populations, any transition)
// reaches sub_tau_min.  The rays that reach the core march their inward
// envelope steps once (the intensity they enter the core with; the envelope's
// populations stay as solved), then n_sub times: the core's opacities and
// emissivities, the core pieces of those rays from their entry intensities
// with the absorbed counts and the diagonal operator accumulated for the core
// shells, and the core shells' ALI solve (W of the full ray set).  Adds the
// marched ray-cell steps (per transition) to *steps.
template <typename TT>
miloc_status core_subiterations(miloc_ctx* c, double* steps)
{
    using T2 = typename V2<TT>::type;
    const bool fp64 = sizeof(TT) == sizeof(double);
    const int n = (int)c->nc;
    c->sub_last_k = -1;
    HIPCHK(c, launch_prepare(c->stream, n, c->d_mol.as<MolDev>(), c->T, c->d_x.as<double>(),
                             c->d_nmolLb.as<double>(), nullptr, c->d_ke.p, fp64));
    std::vector<T2> ke((size_t)n * c->T);
    HIPCHK(c, hipMemcpyAsync(ke.data(), c->d_ke.p, ke.size() * sizeof(T2), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // khat = kappa R_out / (b sqrt(pi)) and radii in units of R_out: the
    // line-centre depth of shell k is khat (R_k - R_k-1)
    int K = -1;
    std::vector<double> tau(c->T, 0.0);
    for (int k = n - 1; k >= 0 && K < 0; --k) {
        const double dr = c->Rn[k] - (k > 0 ? c->Rn[k - 1] : 0.0);
        for (int t = 0; t < c->T; ++t) {
            tau[t] += (double)ke[(size_t)k * c->T + t].x * dr;
            if (tau[t] >= c->sub_tau_min) K = k;
        }
    }
    c->sub_last_k = K;
    if (K < 0) return MILOC_OK;
    // the rays that reach the core (sorted by impact parameter: a prefix)
    int nr = 0;
    double core_steps = 0.0;
    while (nr < c->nrays && c->kmin_host[nr] <= K) {
        core_steps += 2.0 * (K - c->kmin_host[nr]) + 2.0;
        ++nr;
    }
    if (nr == 0) return MILOC_OK;
    HIPCHK(c, c->d_ient.ensure((size_t)c->T * nr * c->nch * sizeof(TT)));
    HIPCHK(c, c->d_sflags.ensure(16));
    HIPCHK(c, hipMemsetAsync(c->d_sflags.p, 0, 16, c->stream));
    March1DArgs<TT> a{};
    fill_march1d(c, c->T, 0, a);
    a.nrays = nr;
    a.core_k = K;
    a.seg = kSegEnvelopeIn;
    a.Iout = c->d_ient.as<TT>();
    HIPCHK(c, launch_march1d(c->stream, a, c->lanes, false));
    *steps += (double)nr * (n - 1 - K);
    a.seg = kSegCore;
    a.Iout = nullptr;
    a.Ient = c->d_ient.as<TT>();
    for (int m = 0; m < c->n_sub; ++m) {
        if (m > 0)
            HIPCHK(c, launch_prepare(c->stream, K + 1, c->d_mol.as<MolDev>(), c->T, c->d_x.as<double>(),
                                     c->d_nmolLb.as<double>(), nullptr, c->d_ke.p, fp64));
        HIPCHK(c, hipMemsetAsync(c->d_acc.p, 0, (size_t)(K + 1) * c->T * sizeof(double2), c->stream));
        HIPCHK(c, launch_march1d(c->stream, a, c->lanes, true));
        SEArgs se{};
        se.nc = K + 1;
        se.L = c->L;
        se.ntr = c->T;
        se.use_ali = 1;
        se.mol = c->d_mol.as<MolDev>();
        se.x_old = c->d_x.as<double>();
        se.x_new = c->d_xnew.as<double>();
        se.nH2 = c->d_nH2.as<double>();
        se.Tkin = c->d_T.as<double>();
        se.q = c->d_q.as<double>();
        se.acc = c->d_acc.as<double2>();
        se.delta_bits = c->d_sflags.as<unsigned long long>();
        se.bad = reinterpret_cast<unsigned int*>(c->d_sflags.as<char>() + 8);
        HIPCHK(c, launch_se(c->stream, se));
        HIPCHK(c, hipMemcpyAsync(c->d_x.p, c->d_xnew.p, (size_t)(K + 1) * c->L * sizeof(double),
                                 hipMemcpyDeviceToDevice, c->stream));
        *steps += core_steps;
    }
    unsigned long long fl[2] = {0, 0};
    unsigned maser = 0;
    HIPCHK(c, hipMemcpyAsync(fl, c->d_sflags.p, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&maser, maser_flag(c), sizeof maser, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (maser) return fail(c, MILOC_ENUMERIC, "maser: a step's line-centre optical depth fell below -40");
    if (fl[1] & 0xffffffffu)
        return fail(c, MILOC_ENUMERIC, "non-finite or negative populations from a core sub-iteration solve");
    return MILOC_OK;
}

// The channel base of every (direction, ray) of a regular grid and the
// largest span of a ray (ray_span_kernel), for the current lane count: an
// FP32 march then keeps only each ray's span in LDS.  span_w stays 0 when the
// span would not be shorter than the whole padded channel vector.
miloc_status ensure_spans(miloc_ctx* c)
{
    if (c->span_lanes == c->lanes) return MILOC_OK;
    const size_t rays = (size_t)c->N * c->N;
    HIPCHK(c, c->d_rbase.ensure((size_t)c->n_dir_dev * rays * sizeof(int)));
    HIPCHK(c, c->d_spanw.ensure(sizeof(int)));
    HIPCHK(c, hipMemsetAsync(c->d_spanw.p, 0, sizeof(int), c->stream));
    March3DArgs<float> a{};
    a.N = c->N;
    a.nc = (int)c->nc;
    a.nch = c->nch;
    a.rays_per_dir = (int)rays;
    a.n_dir = c->n_dir_dev;
    a.dirs = c->d_dirs.as<DirDev>();
    a.steps = c->d_steps.as<StepRec<float>>();
    a.win = c->d_win.as<float4>();
    const int reach = march_pass_reach(c->lanes);
    HIPCHK(c, launch_ray_spans(c->stream, a, reach, c->d_rbase.as<int>(), c->d_spanw.as<int>()));
    int w = 0;
    HIPCHK(c, hipMemcpyAsync(&w, c->d_spanw.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->span_w = (w + 31) / 32 * 32 + 8 < c->nch + reach && !std::getenv("MILOC_FULL_CHANNEL_VECTORS") ? w : 0;
    c->span_lanes = c->lanes;
    return MILOC_OK;
}

template <typename TT>
miloc_status launch_march(miloc_ctx* c, int ntr, int toff, bool accum, TT* Iout, bool zdir,
                          const DirDev* d_dirs_override, const void* steps_override, int nd_override,
                          const double* bimp_override, int nrays_override,
                          const void* win_override = nullptr, const DevBuf* ray_steps = nullptr,
                          const DevBuf* ray_off = nullptr, const DevBuf* ray_kmin = nullptr)
{
    hipError_t e;
    if (c->kind == 3) {
        March3DArgs<TT> a{};
        a.N = c->N;
        a.nc = (int)c->nc;
        a.nch = c->nch;
        a.ntr = ntr;
        a.trans_offset = toff;
        a.rays_per_dir = c->N * c->N;
        a.n_dir = zdir ? nd_override : c->n_dir_dev;
        a.dirs = zdir ? d_dirs_override : c->d_dirs.as<DirDev>();
        a.steps = zdir ? reinterpret_cast<const StepRec<TT>*>(steps_override) : c->d_steps.as<StepRec<TT>>();
        a.win = zdir ? reinterpret_cast<const typename V4<TT>::type*>(win_override)
                     : c->d_win.as<typename V4<TT>::type>();
        a.ke = c->d_ke.as<typename V2<TT>::type>();
        a.Ibg = accum ? c->d_Ibg.as<TT>() : c->d_zero.as<TT>();
        a.Iout = Iout;
        a.ntr_total = c->T;
        a.E = accum ? c->d_E.as<typename V2<TT>::type>() : nullptr;
        a.e_tstride = (size_t)c->total_steps * c->N * c->N;
        a.hf = c->hfk ? c->d_hf.as<typename V2<TT>::type>() : nullptr;
        a.hfk = c->hfk;
        a.maser = maser_flag(c);
        int max_steps = 0;
        if (zdir) {
            max_steps = c->N;
        } else {
            for (const DirDev& D : c->dir_host) max_steps = std::max(max_steps, D.nsteps);
        }
        if constexpr (std::is_same<TT, float>::value) {
            if (accum && !zdir && !c->hfk) {
                const miloc_status st = ensure_spans(c);
                if (st != MILOC_OK) return st;
                if (c->span_w > 0) {
                    a.rbase = c->d_rbase.as<int>();
                    a.span_w = c->span_w;
                }
            }
        }
        e = launch_march3d(c->stream, a, c->lanes, accum, max_steps);
    } else {
        March1DArgs<TT> a{};
        fill_march1d(c, ntr, toff, a);
        a.nrays = bimp_override ? nrays_override : c->nrays;
        if (ray_steps) {
            a.steps = reinterpret_cast<const typename V2<TT>::type*>(ray_steps->p);
            a.ray_off = ray_off->as<long long>();
            a.kmin = ray_kmin->as<int>();
        }
        if (bimp_override) a.area = bimp_override;
        a.Ibg = accum ? c->d_Ibg.as<TT>() : c->d_zero.as<TT>();
        a.Iout = Iout;
        if (accum && c->tbatch && !a.hf) {
            e = launch_march1d_all_transitions(c->stream, a);
        } else {
            // lines of sight run alone: 64 lanes shorten each step's channel loop
            e = launch_march1d(c->stream, a, accum ? c->lanes : 64, accum);
        }
    }
    HIPCHK(c, e);
    return MILOC_OK;
}

template <typename TT>
miloc_status launch_gathers(miloc_ctx* c, int toff, int nt)
{
    const int64_t stride[3] = {1, c->N, (int64_t)c->N * c->N};
    bool first = true;                    // writes every cell's sums of these transitions
    for (int g = 0; g < 3; ++g) {
        if (c->qcount[g] == 0) continue;
        Gather3DArgs<TT> a{};
        a.overwrite = first ? 1 : 0;
        first = false;
        a.N = c->N;
        a.ntr = nt;
        a.trans_offset = toff;
        a.ntr_total = c->T;
        a.nq = c->qcount[g];
        const int ax_a = g == 0 ? 1 : 0, ax_b = g == 2 ? 1 : 2;
        a.st_a = (int)stride[ax_a];
        a.st_b = (int)stride[ax_b];
        a.st_m = (int)stride[g];
        a.qlist = c->d_qlist.as<int>() + c->qoff[g];
        a.dirs = c->d_dirs.as<DirDev>();
        a.lstart = c->d_lstart.as<int>();
        a.moves = c->d_moves.as<int2>();
        a.E = c->d_E.as<typename V2<TT>::type>();
        a.e_tstride = (size_t)c->total_steps * c->N * c->N;
        a.acc = c->d_acc.as<double2>();
        HIPCHK(c, launch_gather3d(c->stream, a));
    }
    return MILOC_OK;
}

miloc_status check_ctx(miloc_ctx* c)
{
    if (!c) return MILOC_EINVAL;
    c->err.clear();
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(c, MILOC_EDEVICE, hipGetErrorString(e));
    return MILOC_OK;
}

}  // namespace

extern "C" {

const char* miloc_version(void) { return "miloc 0.1 gfx950"; }

miloc_status miloc_create(int hip_device, void* hip_stream, miloc_ctx** out)
{
    if (!out) return MILOC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MILOC_EDEVICE;
    if (hip_device < 0 || hip_device >= n) return MILOC_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return MILOC_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MILOC_EDEVICE;
    if (hipSetDevice(hip_device) != hipSuccess) return MILOC_EDEVICE;
    miloc_ctx* c = new (std::nothrow) miloc_ctx();
    if (!c) return MILOC_ENOMEM;
    c->device = hip_device;
    if (hip_stream) {
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) { delete c; return MILOC_EDEVICE; }
        c->own_stream = true;
    }
    for (auto& ev : c->ev)
        if (hipEventCreate(&ev) != hipSuccess) { miloc_destroy(c); return MILOC_EDEVICE; }
    c->dirs = healpix_directions(2);
    *out = c;
    return MILOC_OK;
}

void miloc_destroy(miloc_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* miloc_last_error(const miloc_ctx* c)
{
    return c ? c->err.c_str() : "";
}

miloc_status miloc_load_molecule(miloc_ctx* c, const miloc_molecule* m)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!m || !m->E_K || !m->g || !m->up || !m->lo || !m->A || !m->nu_Hz || !m->gamma_down)
        return fail(c, MILOC_EINVAL, "NULL molecule field");
    const int L = m->n_levels, T = m->n_trans;
    if (L < 2 || L > kMaxLevels) return fail(c, MILOC_EINVAL, "n_levels out of range 2..32");
    if (T < 1 || T > L * (L - 1) / 2) return fail(c, MILOC_EINVAL, "n_trans out of range");
    if (!finite_all(m->E_K, L) || !positive_all(m->g, L) || !finite_all(m->g, L))
        return fail(c, MILOC_EINVAL, "bad level energies or weights");
    if (!positive_all(m->A, T) || !positive_all(m->nu_Hz, T) || !finite_all(m->A, T) ||
        !finite_all(m->nu_Hz, T))
        return fail(c, MILOC_EINVAL, "A and nu must be positive and finite");
    if (!(m->mass_amu > 0) || !std::isfinite(m->mass_amu)) return fail(c, MILOC_EINVAL, "bad mass");
    std::vector<char> seen((size_t)L * L, 0);
    for (int t = 0; t < T; ++t) {
        const int u = m->up[t], l = m->lo[t];
        if (u < 0 || u >= L || l < 0 || l >= u) return fail(c, MILOC_EINVAL, "transition needs 0 <= lo < up < n_levels");
        if (seen[(size_t)u * L + l]) return fail(c, MILOC_EINVAL, "duplicate transition");
        seen[(size_t)u * L + l] = 1;
    }
    for (int u = 0; u < L; ++u)
        for (int l = 0; l < u; ++l) {
            const double gm = m->gamma_down[(size_t)u * L + l];
            if (!(gm >= 0) || !std::isfinite(gm)) return fail(c, MILOC_EINVAL, "bad collision coefficient");
        }
    c->L = L;
    c->T = T;
    c->E.assign(m->E_K, m->E_K + L);
    c->g.assign(m->g, m->g + L);
    c->up.assign(m->up, m->up + T);
    c->lo.assign(m->lo, m->lo + T);
    c->A.assign(m->A, m->A + T);
    c->nu.assign(m->nu_Hz, m->nu_Hz + T);
    c->gamma.assign(m->gamma_down, m->gamma_down + (size_t)L * L);
    c->mass_amu = m->mass_amu;
    c->hf_v.assign(T, {});
    c->hf_w.assign(T, {});
    c->has_mol = true;
    invalidate_model(c);
    return MILOC_OK;
}

miloc_status miloc_load_model_1d(miloc_ctx* c, const miloc_model1d* m)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!m || !m->r_out_cm || !m->n_H2 || !m->T_kin || !m->b_turb_cms || !m->v_r_cms || !m->abundance)
        return fail(c, MILOC_EINVAL, "NULL model field");
    const int n = m->n_shells;
    if (n < 1 || n > 65536) return fail(c, MILOC_EINVAL, "n_shells out of range 1..65536");
    if (m->n_rays < 1 || m->n_rays > 65536) return fail(c, MILOC_EINVAL, "n_rays out of range 1..65536");
    if (!positive_all(m->r_out_cm, n) || !finite_all(m->r_out_cm, n))
        return fail(c, MILOC_EINVAL, "radii must be positive and finite");
    for (int k = 1; k < n; ++k)
        if (!(m->r_out_cm[k] > m->r_out_cm[k - 1])) return fail(c, MILOC_EINVAL, "radii must increase");
    if (!nonneg_all(m->n_H2, n) || !finite_all(m->n_H2, n) || !positive_all(m->T_kin, n) ||
        !finite_all(m->T_kin, n) || !nonneg_all(m->b_turb_cms, n) || !finite_all(m->b_turb_cms, n) ||
        !finite_all(m->v_r_cms, n) || !nonneg_all(m->abundance, n) || !finite_all(m->abundance, n))
        return fail(c, MILOC_EINVAL, "negative or non-finite shell values");
    const double Rout = m->r_out_cm[n - 1];
    std::vector<double> imp(m->n_rays);
    if (m->impact_cm) {
        for (int j = 0; j < m->n_rays; ++j) {
            imp[j] = m->impact_cm[j];
            if (!(imp[j] > 0 && imp[j] < Rout) || (j > 0 && !(imp[j] > imp[j - 1])))
                return fail(c, MILOC_EINVAL, "impact parameters must increase inside (0, R)");
        }
    } else {
        for (int j = 0; j < m->n_rays; ++j) imp[j] = (j + 0.5) * Rout / m->n_rays;
    }
    c->kind = 1;
    c->nc = n;
    c->R.assign(m->r_out_cm, m->r_out_cm + n);
    c->nH2.assign(m->n_H2, m->n_H2 + n);
    c->Tk.assign(m->T_kin, m->T_kin + n);
    c->bt.assign(m->b_turb_cms, m->b_turb_cms + n);
    c->vr.assign(m->v_r_cms, m->v_r_cms + n);
    c->X.assign(m->abundance, m->abundance + n);
    c->nrays = m->n_rays;
    c->impact = imp;
    c->f_nH2.clear(); c->f_T.clear(); c->f_bt.clear(); c->f_vx.clear(); c->f_vy.clear();
    c->f_vz.clear(); c->f_X.clear();
    invalidate_model(c);
    return MILOC_OK;
}

miloc_status miloc_load_model_3d(miloc_ctx* c, const miloc_model3d* m)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!m || !m->n_H2 || !m->T_kin || !m->b_turb_cms || !m->vx || !m->vy || !m->vz || !m->abundance)
        return fail(c, MILOC_EINVAL, "NULL model field");
    if (m->n_oct_levels < 0) return fail(c, MILOC_EINVAL, "n_oct_levels must be >= 0");
    const int N = m->n0[0];
    const int Nmin = m->n_oct_levels > 0 ? 1 : 2;
    if (N < Nmin || N > 1024 || m->n0[1] != N || m->n0[2] != N)
        return fail(c, MILOC_EINVAL, "grid must be N^3 with 2 <= N <= 1024 (octree roots: 1 <= N)");
    if (!(m->root_cell_cm > 0) || !std::isfinite(m->root_cell_cm)) return fail(c, MILOC_EINVAL, "bad cell size");
    OctModel oct;
    int64_t nc = (int64_t)N * N * N;
    if (m->n_oct_levels > 0) {
        const std::string e = octree_from_levels(N, m->n_oct_levels, m->n_cells_per_level, m->first_child, oct);
        if (!e.empty()) return fail(c, MILOC_EINVAL, e);
        nc = oct.level_start.back();
    }
    if (!nonneg_all(m->n_H2, nc) || !finite_all(m->n_H2, nc) || !positive_all(m->T_kin, nc) ||
        !finite_all(m->T_kin, nc) || !nonneg_all(m->b_turb_cms, nc) || !finite_all(m->b_turb_cms, nc) ||
        !finite_all(m->vx, nc) || !finite_all(m->vy, nc) || !finite_all(m->vz, nc) ||
        !nonneg_all(m->abundance, nc) || !finite_all(m->abundance, nc))
        return fail(c, MILOC_EINVAL, "negative or non-finite cell values");
    c->kind = m->n_oct_levels > 0 ? 4 : 3;
    c->oct = std::move(oct);
    c->nc = nc;
    c->N = N;
    c->delta = m->root_cell_cm;
    c->f_nH2.assign(m->n_H2, m->n_H2 + nc);
    c->f_T.assign(m->T_kin, m->T_kin + nc);
    c->f_bt.assign(m->b_turb_cms, m->b_turb_cms + nc);
    c->f_vx.assign(m->vx, m->vx + nc);
    c->f_vy.assign(m->vy, m->vy + nc);
    c->f_vz.assign(m->vz, m->vz + nc);
    c->f_X.assign(m->abundance, m->abundance + nc);
    c->R.clear(); c->nH2.clear(); c->Tk.clear(); c->bt.clear(); c->vr.clear(); c->X.clear();
    invalidate_model(c);
    return MILOC_OK;
}

miloc_status miloc_octree_schedule(const miloc_model3d* m, int n_dir, const double* dirs, int plain,
                                   int64_t* n_steps, int64_t* n_trees, int* max_depth, uint32_t* steps_out,
                                   int64_t* trees_out)
{
    if (!m || m->n_oct_levels < 1 || !dirs || n_dir < 1 || n_dir > 1024) return MILOC_EINVAL;
    const int N = m->n0[0];
    if (N < 1 || N > 1024 || m->n0[1] != N || m->n0[2] != N) return MILOC_EINVAL;
    OctModel oct;
    if (!octree_from_levels(N, m->n_oct_levels, m->n_cells_per_level, m->first_child, oct).empty())
        return MILOC_EINVAL;
    std::vector<double> d(3 * (size_t)n_dir);
    for (int q = 0; q < n_dir; ++q) {
        const double x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
        const double nrm = std::sqrt(x * x + y * y + z * z);
        if (!(nrm > 0) || !std::isfinite(nrm)) return MILOC_EINVAL;
        d[3 * q] = x / nrm; d[3 * q + 1] = y / nrm; d[3 * q + 2] = z / nrm;
    }
    OctSchedule S;
    if (plain < 0 || plain > 2) return MILOC_EINVAL;
    if (!octree_schedule(oct, d, static_cast<OctRays>(plain), host_threads(), S).empty()) return MILOC_EINVAL;
    if (n_steps) *n_steps = S.n_steps;
    if (n_trees) *n_trees = (int64_t)S.trees.size();
    if (max_depth) *max_depth = S.max_depth;
    if (steps_out) std::memcpy(steps_out, S.rec.data(), S.rec.size() * sizeof(uint32_t));
    if (trees_out)
        for (size_t i = 0; i < S.trees.size(); ++i) {
            trees_out[4 * i] = S.trees[i].off;
            trees_out[4 * i + 1] = S.trees[i].n;
            trees_out[4 * i + 2] = S.trees[i].q;
            trees_out[4 * i + 3] = S.trees[i].r;
        }
    return MILOC_OK;
}

miloc_status miloc_model_footprint(const miloc_model1d* m1, const miloc_model3d* m3, int n_levels, int n_trans,
                                   int n_channels, int n_dir, const double* dirs, int precision, int64_t oct_steps,
                                   size_t* fixed_bytes, size_t* sums_bytes)
{
    if ((m1 == nullptr) == (m3 == nullptr) || !fixed_bytes || !sums_bytes) return MILOC_EINVAL;
    if (n_levels < 2 || n_levels > kMaxLevels || n_trans < 1 || n_trans > kMaxTrans || n_channels < 1)
        return MILOC_EINVAL;
    if (precision != MILOC_MARCH_FP32 && precision != MILOC_MARCH_FP64) return MILOC_EINVAL;
    const bool fp64 = precision == MILOC_MARCH_FP64;
    Footprint f;
    if (m1) {
        const int n = m1->n_shells;
        if (n < 1 || n > 65536 || !m1->r_out_cm || m1->n_rays < 1 || m1->n_rays > 65536) return MILOC_EINVAL;
        const double R = m1->r_out_cm[n - 1];
        if (!(R > 0)) return MILOC_EINVAL;
        std::vector<double> Rn(n), bn(m1->n_rays);
        for (int k = 0; k < n; ++k) Rn[k] = m1->r_out_cm[k] / R;
        Rn[n - 1] = 1.0;
        for (int j = 0; j < m1->n_rays; ++j)
            bn[j] = m1->impact_cm ? m1->impact_cm[j] / R : (j + 0.5) / m1->n_rays;
        std::vector<int64_t> off;
        std::vector<int> km;
        const int64_t steps = shell_ray_layout(n, Rn.data(), m1->n_rays, bn.data(), off, km);
        f = footprint_of(1, n, n_levels, n_trans, n_channels, 0, fp64, steps, m1->n_rays, 0);
    } else {
        const int N = m3->n0[0];
        if (N < 1 || N > 1024 || m3->n0[1] != N || m3->n0[2] != N || m3->n_oct_levels < 0) return MILOC_EINVAL;
        std::vector<double> dv = dirs ? std::vector<double>(dirs, dirs + 3 * (size_t)std::max(0, n_dir))
                                      : healpix_directions(2);
        const int nd = (int)dv.size() / 3;
        if (nd < 1 || nd > 1024) return MILOC_EINVAL;
        if (m3->n_oct_levels == 0) {
            if (N < 2) return MILOC_EINVAL;
            std::vector<DirDev> dd;
            std::vector<double> len;
            std::vector<int> fl;
            build_patterns(N, dv, dd, len, fl, nullptr);
            f = footprint_of(3, (int64_t)N * N * N, n_levels, n_trans, n_channels, nd, fp64, (int64_t)len.size(),
                             (int64_t)N * N, 0);
        } else {
            if (!m3->n_cells_per_level || oct_steps < 0) return MILOC_EINVAL;
            int64_t nc = 0;
            for (int l = 0; l < m3->n_oct_levels; ++l) nc += m3->n_cells_per_level[l];
            f = footprint_of(4, nc, n_levels, n_trans, n_channels, nd, fp64, oct_steps, 0, (int64_t)nd * N * N);
        }
    }
    *fixed_bytes = f.fixed;
    *sums_bytes = f.sums;
    return MILOC_OK;
}

miloc_status miloc_set_spectral(miloc_ctx* c, int n_channels, double v_min_cms, double dv_cms)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (n_channels < 8 || n_channels > 4096) return fail(c, MILOC_EINVAL, "n_channels out of range 8..4096");
    if (!std::isfinite(v_min_cms) || !(dv_cms > 0) || !std::isfinite(dv_cms))
        return fail(c, MILOC_EINVAL, "bad channel grid");
    c->nch = n_channels;
    c->vmin = v_min_cms;
    c->dv = dv_cms;
    c->has_spec = true;
    c->dirty = true;
    c->has_rad = false;
    return MILOC_OK;
}

miloc_status miloc_set_hyperfine(miloc_ctx* c, int trans, int n_comp, const double* dv_cms, const double* strength)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!c->has_mol) return fail(c, MILOC_ESTATE, "molecule must be loaded first");
    if (trans < 0 || trans >= c->T) return fail(c, MILOC_EINVAL, "transition index out of range");
    if (n_comp < 0 || n_comp > MILOC_MAX_HF_COMPONENTS)
        return fail(c, MILOC_EINVAL, "n_comp out of range 0..MILOC_MAX_HF_COMPONENTS");
    if (n_comp > 0 && (!dv_cms || !strength)) return fail(c, MILOC_EINVAL, "NULL component array");
    double sum = 0.0;
    for (int k = 0; k < n_comp; ++k) {
        if (!std::isfinite(dv_cms[k])) return fail(c, MILOC_EINVAL, "non-finite component offset");
        if (!(strength[k] > 0) || !std::isfinite(strength[k]))
            return fail(c, MILOC_EINVAL, "component strengths must be finite and > 0");
        sum += strength[k];
    }
    c->hf_v[trans].assign(dv_cms, dv_cms + n_comp);
    c->hf_w[trans].resize(n_comp);
    for (int k = 0; k < n_comp; ++k) c->hf_w[trans][k] = strength[k] / sum;
    c->dirty = true;
    c->has_rad = false;
    return MILOC_OK;
}

miloc_status miloc_set_octree_rays(miloc_ctx* c, int rays)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (rays != MILOC_OCT_RAYS_SCHEME && rays != MILOC_OCT_RAYS_LATTICE)
        return fail(c, MILOC_EINVAL, "rays must be MILOC_OCT_RAYS_SCHEME or MILOC_OCT_RAYS_LATTICE");
    const bool lat = rays == MILOC_OCT_RAYS_LATTICE;
    if (lat != c->oct_lattice) {
        c->oct_lattice = lat;
        c->dirty = true;
        c->has_rad = false;
    }
    return MILOC_OK;
}

miloc_status miloc_set_background(miloc_ctx* c, double T_bg_K)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!(T_bg_K >= 0) || !std::isfinite(T_bg_K)) return fail(c, MILOC_EINVAL, "T_bg must be >= 0");
    c->Tbg = T_bg_K;
    c->dirty = true;
    return MILOC_OK;
}

miloc_status miloc_set_directions_healpix(miloc_ctx* c, int nside)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (nside < 1 || nside > 8) return fail(c, MILOC_EINVAL, "nside out of range 1..8");
    c->dirs = healpix_directions(nside);
    c->dirty = true;
    return MILOC_OK;
}

miloc_status miloc_set_directions(miloc_ctx* c, int n_dir, const double* dirs)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (n_dir < 1 || n_dir > 1024 || !dirs) return fail(c, MILOC_EINVAL, "n_dir out of range 1..1024");
    std::vector<double> d(3 * (size_t)n_dir);
    for (int q = 0; q < n_dir; ++q) {
        const double x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
        const double nrm = std::sqrt(x * x + y * y + z * z);
        if (!(nrm > 0) || !std::isfinite(nrm)) return fail(c, MILOC_EINVAL, "zero or non-finite direction");
        d[3 * q] = x / nrm; d[3 * q + 1] = y / nrm; d[3 * q + 2] = z / nrm;
    }
    c->dirs = d;
    c->dirty = true;
    return MILOC_OK;
}

miloc_status miloc_set_subiterations(miloc_ctx* c, int n_sub, double tau_min)
{
    if (!c) return MILOC_EINVAL;
    c->err.clear();
    if (n_sub < 0 || n_sub > 1000) return fail(c, MILOC_EINVAL, "n_sub must be in 0..1000");
    if (!std::isfinite(tau_min)) return fail(c, MILOC_EINVAL, "tau_min must be finite");
    c->n_sub = n_sub;
    c->sub_tau_min = tau_min;
    return MILOC_OK;
}

miloc_status miloc_set_transition_batching(miloc_ctx* c, int on)
{
    if (!c) return MILOC_EINVAL;
    c->err.clear();
    if (on != 0 && on != 1) return fail(c, MILOC_EINVAL, "on must be 0 or 1");
    c->tbatch = on;
    return MILOC_OK;
}

miloc_status miloc_set_march_precision(miloc_ctx* c, int precision)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (precision != MILOC_MARCH_FP32 && precision != MILOC_MARCH_FP64)
        return fail(c, MILOC_EINVAL, "precision must be MILOC_MARCH_FP32 or MILOC_MARCH_FP64");
    if (precision != c->precision) {
        c->precision = precision;
        c->dirty = true;
    }
    return MILOC_OK;
}

miloc_status miloc_init_lte(miloc_ctx* c)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    s = ensure_base(c);
    if (s) return s;
    HIPCHK(c, launch_lte(c->stream, (int)c->nc, c->d_mol.as<MolDev>(), c->d_T.as<double>(), c->d_x.as<double>()));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_pops = true;
    c->has_rad = false;
    return MILOC_OK;
}

miloc_status miloc_set_populations(miloc_ctx* c, const double* x)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!x) return fail(c, MILOC_EINVAL, "NULL populations");
    s = ensure_base(c);
    if (s) return s;
    const size_t n = (size_t)c->nc * c->L;
    std::vector<double> h(x, x + n);
    for (int64_t k = 0; k < c->nc; ++k) {
        double sum = 0;
        for (int i = 0; i < c->L; ++i) {
            const double v = h[(size_t)k * c->L + i];
            if (!(v >= 0) || !std::isfinite(v)) return fail(c, MILOC_EINVAL, "populations must be finite and >= 0");
            sum += v;
        }
        if (!(sum > 0)) return fail(c, MILOC_EINVAL, "a cell has all-zero populations");
        for (int i = 0; i < c->L; ++i) h[(size_t)k * c->L + i] /= sum;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_x.p, h.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_pops = true;
    c->has_rad = false;
    return MILOC_OK;
}

miloc_status miloc_run(miloc_ctx* c, int max_iter, double tol, int use_ali, int* iters_done,
                       double* last_delta)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (max_iter < 1) return fail(c, MILOC_EINVAL, "max_iter must be >= 1");
    if (!std::isfinite(tol)) return fail(c, MILOC_EINVAL, "tol must be finite");
    if (c->n_sub > 0) {
        if (c->kind != 1) return fail(c, MILOC_EINVAL, "core sub-iterations are for 1D models");
        if (!use_ali) return fail(c, MILOC_EINVAL, "core sub-iterations need the ALI form (use_ali != 0)");
        for (int t = 0; t < c->T; ++t)
            if (!c->hf_v[t].empty())
                return fail(c, MILOC_EINVAL, "core sub-iterations are for single-Gaussian lines");
    }
    s = ensure_static(c);
    if (s) return s;
    if (!c->has_pops) {
        s = miloc_init_lte(c);
        if (s) return s;
    }
    const bool fp64 = c->precision == MILOC_MARCH_FP64;
    const int64_t nc = c->nc;
    double delta = INFINITY;
    int it = 0;
    bool converged = false;
    for (; it < max_iter; ++it) {
        // convergence maximum, failure counter and maser flag of this iteration
        HIPCHK(c, hipMemsetAsync(c->d_flags.p, 0, 16, c->stream));
        HIPCHK(c, ev_record(c, 0));
        HIPCHK(c, launch_prepare(c->stream, (int)nc, c->d_mol.as<MolDev>(), c->T, c->d_x.as<double>(),
                                 c->d_nmolLb.as<double>(), nullptr, c->d_ke.p, fp64));
        // the regular-grid and octree gathers write every cell's sums; the 1D
        // march adds into zeroed accumulators
        if (c->kind != 3 && c->kind != 4) HIPCHK(c, hipMemsetAsync(c->d_acc.p, 0, c->d_acc.bytes, c->stream));
        HIPCHK(c, ev_record(c, 1));
        float t_march = 0, t_gather = 0;
        if (c->kind == 3) {
            for (int t0 = 0; t0 < c->T; t0 += c->trans_chunk) {
                const int nt = std::min(c->trans_chunk, c->T - t0);
                if (t0 > 0) HIPCHK(c, ev_record(c, 1));
                s = fp64 ? launch_march<double>(c, nt, t0, true, nullptr, false, nullptr, nullptr, 0, nullptr, 0)
                         : launch_march<float>(c, nt, t0, true, nullptr, false, nullptr, nullptr, 0, nullptr, 0);
                if (s) return s;
                HIPCHK(c, ev_record(c, 4));
                s = fp64 ? launch_gathers<double>(c, t0, nt) : launch_gathers<float>(c, t0, nt);
                if (s) return s;
                HIPCHK(c, ev_record(c, 5));
                HIPCHK(c, ev_sync(c, 5));
                float a = 0, b = 0;
                HIPCHK(c, ev_elapsed(c, &a, 1, 4));
                HIPCHK(c, ev_elapsed(c, &b, 4, 5));
                t_march += a;
                t_gather += b;
                c->ctr.march_launches += 1;
            }
        } else if (c->kind == 4) {
            for (int t0 = 0; t0 < c->T; t0 += c->trans_chunk) {
                const int nt = std::min(c->trans_chunk, c->T - t0);
                if (t0 > 0) HIPCHK(c, ev_record(c, 1));
                s = fp64 ? launch_oct<double>(c, nt, t0, true, nullptr, c->d_osteps, c->d_otrees, c->oct_trees,
                                              c->d_oaw.as<double>(), c->d_win.p, c->oct_groups,
                                              c->d_olen64.as<double>())
                         : launch_oct<float>(c, nt, t0, true, nullptr, c->d_osteps, c->d_otrees, c->oct_trees,
                                             c->d_oaw.as<double>(), c->d_win.p, c->oct_groups, nullptr);
                if (s) return s;
                HIPCHK(c, ev_record(c, 4));
                if (fp64) {
                    GatherOctArgs<double> g{c->nc, nt, t0, c->T, c->d_ocell_off.as<long long>(),
                                            c->d_ocell_steps.as<unsigned>(), c->d_odir_off.as<unsigned>(),
                                            c->n_dir_dev, c->d_oE.as<double2>(),
                                            c->oct_estride, c->d_acc.as<double2>()};
                    HIPCHK(c, launch_gather_oct(c->stream, g));
                } else {
                    GatherOctArgs<float> g{c->nc, nt, t0, c->T, c->d_ocell_off.as<long long>(),
                                           c->d_ocell_steps.as<unsigned>(), c->d_odir_off.as<unsigned>(),
                                           c->n_dir_dev, c->d_oE.as<float2>(),
                                           c->oct_estride, c->d_acc.as<double2>()};
                    HIPCHK(c, launch_gather_oct(c->stream, g));
                }
                HIPCHK(c, ev_record(c, 5));
                HIPCHK(c, ev_sync(c, 5));
                float a = 0, b = 0;
                HIPCHK(c, ev_elapsed(c, &a, 1, 4));
                HIPCHK(c, ev_elapsed(c, &b, 4, 5));
                t_march += a;
                t_gather += b;
                c->ctr.march_launches += 1;
            }
        } else {
            s = fp64 ? launch_march<double>(c, c->T, 0, true, nullptr, false, nullptr, nullptr, 0, nullptr, 0)
                     : launch_march<float>(c, c->T, 0, true, nullptr, false, nullptr, nullptr, 0, nullptr, 0);
            if (s) return s;
            HIPCHK(c, ev_record(c, 4));
            HIPCHK(c, ev_sync(c, 4));
            HIPCHK(c, ev_elapsed(c, &t_march, 1, 4));
            c->ctr.march_launches += 1;
        }
        HIPCHK(c, ev_record(c, 2));
        SEArgs a{};
        a.nc = (int)nc;
        a.L = c->L;
        a.ntr = c->T;
        a.use_ali = use_ali ? 1 : 0;
        a.mol = c->d_mol.as<MolDev>();
        a.x_old = c->d_x.as<double>();
        a.x_new = c->d_xnew.as<double>();
        a.nH2 = c->d_nH2.as<double>();
        a.Tkin = c->d_T.as<double>();
        a.q = c->d_q.as<double>();
        a.acc = c->d_acc.as<double2>();
        a.delta_bits = c->d_flags.as<unsigned long long>();
        a.bad = reinterpret_cast<unsigned int*>(c->d_flags.as<char>() + 8);
        HIPCHK(c, launch_se(c->stream, a));
        HIPCHK(c, ev_record(c, 3));
        unsigned long long flags[2] = {0, 0};
        HIPCHK(c, hipMemcpyAsync(flags, c->d_flags.p, 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        float t01 = 0, t23 = 0;
        HIPCHK(c, ev_elapsed(c, &t01, 0, 1));
        HIPCHK(c, ev_elapsed(c, &t23, 2, 3));
        c->ctr.prepare_ms += t01;
        c->ctr.march_ms += t_march;
        c->ctr.accumulate_ms += t_gather;
        c->ctr.solve_ms += t23;
        c->ctr.ray_steps += c->steps_per_trans * c->T;
        c->ctr.channel_updates += c->steps_per_trans * c->T * c->nch;
        c->ctr.iterations += 1;
        c->has_rad = true;
        const unsigned int bad = (unsigned int)(flags[1] & 0xffffffffu);
        if (flags[1] >> 32) {
            if (iters_done) *iters_done = it;
            return fail(c, MILOC_ENUMERIC, "maser: a step's line-centre optical depth fell below -40 "
                                           "(populations left as before the iteration)");
        }
        if (bad) {
            if (iters_done) *iters_done = it;
            return fail(c, MILOC_ENUMERIC, "non-finite or negative populations from the equilibrium solve");
        }
        std::memcpy(&delta, &flags[0], sizeof(double));
        std::swap(c->d_x.p, c->d_xnew.p);
        if (c->n_sub > 0) {
            double sub_steps = 0.0;
            HIPCHK(c, ev_record(c, 0));
            s = fp64 ? core_subiterations<double>(c, &sub_steps) : core_subiterations<float>(c, &sub_steps);
            if (s) {
                if (iters_done) *iters_done = it;
                return s;
            }
            HIPCHK(c, ev_record(c, 1));
            HIPCHK(c, ev_sync(c, 1));
            float t_sub = 0;
            HIPCHK(c, ev_elapsed(c, &t_sub, 0, 1));
            c->ctr.march_ms += t_sub;
            c->ctr.ray_steps += sub_steps * c->T;
            c->ctr.channel_updates += sub_steps * c->T * c->nch;
        }
        if (tol > 0 && delta < tol) {
            converged = true;
            ++it;
            break;
        }
    }
    if (iters_done) *iters_done = it;
    if (last_delta) *last_delta = delta;
    if (tol > 0 && !converged) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "not converged after %d iterations (delta %.3e)", it, delta);
        return fail(c, MILOC_ENOTCONV, buf);
    }
    return MILOC_OK;
}

miloc_status miloc_get_sizes(const miloc_ctx* c, int64_t* n_cells, int* n_levels, int* n_trans,
                             int* n_channels)
{
    if (!c) return MILOC_EINVAL;
    if (n_cells) *n_cells = c->nc;
    if (n_levels) *n_levels = c->has_mol ? c->L : 0;
    if (n_trans) *n_trans = c->has_mol ? c->T : 0;
    if (n_channels) *n_channels = c->has_spec ? c->nch : 0;
    return MILOC_OK;
}

miloc_status miloc_get_populations(miloc_ctx* c, double* x_out)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!x_out) return fail(c, MILOC_EINVAL, "NULL output");
    if (!c->has_pops) return fail(c, MILOC_ESTATE, "no populations yet");
    const size_t n = (size_t)c->nc * c->L;
    std::vector<double> h(n);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->d_x.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memcpy(x_out, h.data(), n * sizeof(double));
    return MILOC_OK;
}

miloc_status miloc_get_radiation(miloc_ctx* c, double* J_out, double* lambda_out)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!c->has_rad) return fail(c, MILOC_ESTATE, "no iteration has run since the last change");
    const size_t n = (size_t)c->T * c->nc;
    std::vector<double2> h(n);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->d_acc.p, n * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int t = 0; t < c->T; ++t)
        for (int64_t k = 0; k < c->nc; ++k) {
            const size_t i = (size_t)t * c->nc + k;       // output: transition-major
            const size_t a = (size_t)k * c->T + t;        // device: cell-major
            const double qk = c->q_host[k] > 0 ? c->q_host[k] : 0.0;
            if (J_out) J_out[i] = h[a].x * qk * c->Iscale[t];
            if (lambda_out) lambda_out[i] = h[a].y * qk;
        }
    return MILOC_OK;
}

miloc_status miloc_get_spectra(miloc_ctx* c, int trans, int n_los, const double* impact_cm, double* dI_out)
{
    miloc_status s = check_ctx(c);
    if (s) return s;
    if (!dI_out) return fail(c, MILOC_EINVAL, "NULL output");
    if (!c->has_mol || c->kind == 0) return fail(c, MILOC_ESTATE, "no model");
    if (trans < 0 || trans >= c->T) return fail(c, MILOC_EINVAL, "transition index out of range");
    if (!c->has_pops) return fail(c, MILOC_ESTATE, "no populations yet");
    s = ensure_static(c);
    if (s) return s;
    const bool fp64 = c->precision == MILOC_MARCH_FP64;
    const size_t tsz = fp64 ? sizeof(double) : sizeof(float);
    DevBuf out, extra, extra2;
    // march I - I_bg from zero (see prepare_kernel)
    HIPCHK(c, hipMemsetAsync(maser_flag(c), 0, sizeof(unsigned), c->stream));
    HIPCHK(c, launch_prepare(c->stream, (int)c->nc, c->d_mol.as<MolDev>(), c->T, c->d_x.as<double>(),
                             c->d_nmolLb.as<double>(), c->d_Ibg64.as<double>(), c->d_ke.p, fp64));
    if (c->kind == 4) {
        if (impact_cm) return fail(c, MILOC_EINVAL, "3D spectra take no impact parameters");
        if (n_los != c->N * c->N) return fail(c, MILOC_EINVAL, "3D spectra need n_los = N*N");
        // +z lines of sight on the root ray lattice, traced without new rays
        const std::vector<double> zd = {0.0, 0.0, 1.0};
        OctSchedule S;
        const std::string e = octree_schedule(c->oct, zd, OctRays::Plain, host_threads(), S, fp64);
        if (!e.empty()) return fail(c, MILOC_EINVAL, e);
        DevBuf steps, trees, zdir, zaw, zwin, zlen;
        s = upload_oct_schedule(c, S, steps, trees);
        if (s) return s;
        if (fp64) {
            HIPCHK(c, zlen.ensure(std::max<size_t>(1, S.len64.size()) * sizeof(double)));
            HIPCHK(c, hipMemcpy(zlen.p, S.len64.data(), S.len64.size() * sizeof(double), hipMemcpyHostToDevice));
        }
        DirDev D{};
        D.d[2] = 1.0;
        D.m = 2;
        D.aw = 1.0;
        HIPCHK(c, zdir.ensure(sizeof(DirDev)));
        HIPCHK(c, hipMemcpy(zdir.p, &D, sizeof(DirDev), hipMemcpyHostToDevice));
        HIPCHK(c, zaw.ensure(sizeof(double)));
        HIPCHK(c, hipMemcpy(zaw.p, &D.aw, sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, zwin.ensure((size_t)c->nc * 4 * tsz));
        HIPCHK(c, launch_window_table(c->stream, (int)c->nc, 1, zdir.as<DirDev>(), c->d_vel.as<float4>(),
                                      c->d_bD.as<double>(), c->dv, c->chalf,
                                      fp64 ? kWindowK64 : kWindowK32, c->nch, c->hf_lo, c->hf_hi, zwin.p,
                                      fp64));
        HIPCHK(c, out.ensure((size_t)n_los * c->nch * tsz));
        const int gpb = 256 / c->lanes;
        const int groups = (int)std::min<int64_t>(c->oct_groups, ((int64_t)n_los + gpb - 1) / gpb * gpb);
        s = fp64 ? launch_oct<double>(c, 1, trans, false, out.as<double>(), steps, trees, (int64_t)S.trees.size(),
                                      zaw.as<double>(), zwin.p, groups, zlen.as<double>())
                 : launch_oct<float>(c, 1, trans, false, out.as<float>(), steps, trees, (int64_t)S.trees.size(),
                                     zaw.as<double>(), zwin.p, groups, nullptr);
        if (s) return s;
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else if (c->kind == 3) {
        if (impact_cm) return fail(c, MILOC_EINVAL, "3D spectra take no impact parameters");
        if (n_los != c->N * c->N) return fail(c, MILOC_EINVAL, "3D spectra need n_los = N*N");
        std::vector<double> zd = {0.0, 0.0, 1.0};
        std::vector<DirDev> dd;
        std::vector<double> len;
        std::vector<int> fl;
        build_patterns(c->N, zd, dd, len, fl, nullptr);
        HIPCHK(c, extra.ensure(sizeof(DirDev)));
        HIPCHK(c, hipMemcpy(extra.p, dd.data(), sizeof(DirDev), hipMemcpyHostToDevice));
        if (fp64) {
            std::vector<StepRec<double>> st(len.size());
            for (size_t i = 0; i < len.size(); ++i) { st[i].len = len[i]; st[i].flags = fl[i]; }
            HIPCHK(c, extra2.ensure(st.size() * sizeof(st[0])));
            HIPCHK(c, hipMemcpy(extra2.p, st.data(), st.size() * sizeof(st[0]), hipMemcpyHostToDevice));
        } else {
            std::vector<StepRec<float>> st(len.size());
            for (size_t i = 0; i < len.size(); ++i) { st[i].len = step_len_rec<float>(len[i]); st[i].flags = fl[i]; }
            HIPCHK(c, extra2.ensure(st.size() * sizeof(st[0])));
            HIPCHK(c, hipMemcpy(extra2.p, st.data(), st.size() * sizeof(st[0]), hipMemcpyHostToDevice));
        }
        HIPCHK(c, out.ensure((size_t)n_los * c->nch * tsz));
        DevBuf zwin;
        HIPCHK(c, zwin.ensure((size_t)c->nc * 4 * tsz));
        HIPCHK(c, launch_window_table(c->stream, (int)c->nc, 1, extra.as<DirDev>(), c->d_vel.as<float4>(),
                                      c->d_bD.as<double>(), c->dv, c->chalf,
                                      fp64 ? kWindowK64 : kWindowK32, c->nch, c->hf_lo, c->hf_hi, zwin.p,
                                      fp64));
        s = fp64 ? launch_march<double>(c, 1, trans, false, out.as<double>(), true, extra.as<DirDev>(), extra2.p, 1, nullptr, 0, zwin.p)
                 : launch_march<float>(c, 1, trans, false, out.as<float>(), true, extra.as<DirDev>(), extra2.p, 1, nullptr, 0, zwin.p);
        if (s) return s;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (s) return s;
    } else {
        const double Rout = c->R[c->nc - 1];
        std::vector<double> bn;
        if (impact_cm) {
            if (n_los < 1) return fail(c, MILOC_EINVAL, "n_los must be >= 1");
            bn.resize(n_los);
            for (int j = 0; j < n_los; ++j) {
                if (!(impact_cm[j] >= 0 && impact_cm[j] < Rout)) return fail(c, MILOC_EINVAL, "impact parameter outside [0, R)");
                bn[j] = impact_cm[j] / Rout;
            }
        } else {
            if (n_los != c->nrays) return fail(c, MILOC_EINVAL, "n_los must equal n_rays when impact_cm is NULL");
            bn.resize(n_los);
            for (int j = 0; j < n_los; ++j) bn[j] = c->impact[j] / Rout;
        }
        if (!(c->los_valid && c->los_fp64 == fp64 && c->los_b == bn)) {
            c->los_valid = false;
            HIPCHK(c, c->d_los_b.ensure(bn.size() * sizeof(double)));
            HIPCHK(c, hipMemcpy(c->d_los_b.p, bn.data(), bn.size() * sizeof(double), hipMemcpyHostToDevice));
            s = upload_ray_steps(c, bn, fp64, c->d_los_steps, c->d_los_off, c->d_los_kmin);
            if (s) return s;
            c->los_b = bn;
            c->los_fp64 = fp64;
            c->los_valid = true;
        }
        HIPCHK(c, c->d_los_out.ensure((size_t)n_los * c->nch * tsz));
        s = fp64 ? launch_march<double>(c, 1, trans, false, c->d_los_out.as<double>(), false, nullptr, nullptr, 0,
                                        c->d_los_b.as<double>(), n_los, nullptr, &c->d_los_steps, &c->d_los_off,
                                        &c->d_los_kmin)
                 : launch_march<float>(c, 1, trans, false, c->d_los_out.as<float>(), false, nullptr, nullptr, 0,
                                       c->d_los_b.as<double>(), n_los, nullptr, &c->d_los_steps, &c->d_los_off,
                                       &c->d_los_kmin);
        if (s) return s;
    }
    const size_t n = (size_t)n_los * c->nch;
    std::vector<char> h(n * tsz);
    const DevBuf& res = c->kind == 1 ? c->d_los_out : out;
    unsigned maser = 0;
    HIPCHK(c, hipMemcpyAsync(h.data(), res.p, n * tsz, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&maser, maser_flag(c), sizeof maser, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (maser)
        return fail(c, MILOC_ENUMERIC, "maser: a step's line-centre optical depth fell below -40");
    const double sc = c->Iscale[trans];
    for (size_t i = 0; i < n; ++i) {
        const double v = fp64 ? reinterpret_cast<double*>(h.data())[i] : (double)reinterpret_cast<float*>(h.data())[i];
        dI_out[i] = v * sc;
    }
    return MILOC_OK;
}

miloc_status miloc_get_counters(const miloc_ctx* c, miloc_counters* out)
{
    if (!c || !out) return MILOC_EINVAL;
    *out = c->ctr;
    out->march_lanes = c->lanes;
    out->reserved = 0;
    return MILOC_OK;
}

miloc_status miloc_reset_counters(miloc_ctx* c)
{
    if (!c) return MILOC_EINVAL;
    c->ctr = miloc_counters{};
    return MILOC_OK;
}

}  // extern "C"

// ------------------------------------------------------- allocation-free solve
// Device memory of miloc_solve_1d_noalloc: one copy of this array per GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to the device: the address each device gives for it is looked
// up once per device (hipGetSymbolAddress, with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[MILOC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The scratch array's device address on the current device `dev`.
hipError_t scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Installs a ScratchCarve on the calling thread for one call.
struct CarveScope {
    explicit CarveScope(ScratchCarve* sc) { tls_carve = sc; }
    ~CarveScope() { tls_carve = nullptr; }
};

}  // namespace

extern "C" {

miloc_status miloc_solve_1d_noalloc(int hip_device, void* hip_stream, const miloc_molecule* mol,
                                    const miloc_model1d* model, int n_channels, double v_min_cms, double dv_cms,
                                    double T_bg_K, int max_iter, double tol, int* iters_done, double* last_delta,
                                    double* x_out)
{
    if (!mol || !model || !x_out) return MILOC_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MILOC_EDEVICE;
    if (hip_device < 0 || hip_device >= n) return MILOC_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return MILOC_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MILOC_EDEVICE;
    if (hipSetDevice(hip_device) != hipSuccess) return MILOC_EDEVICE;
    void* base = nullptr;
    if (scratch_address(hip_device, &base) != hipSuccess) return MILOC_EDEVICE;
    ScratchCarve carve;
    carve.base = static_cast<char*>(base);
    carve.size = MILOC_NOALLOC_SCRATCH_BYTES;
    miloc_status s;
    int it = 0;
    double d = 0.0;
    {
        CarveScope scope(&carve);
        // a context of this call only: every device buffer carved from the
        // scratch, the caller's stream (NULL: the null stream), no events
        miloc_ctx c;
        c.device = hip_device;
        c.stream = reinterpret_cast<hipStream_t>(hip_stream);
        s = miloc_load_molecule(&c, mol);
        if (s == MILOC_OK) s = miloc_load_model_1d(&c, model);
        if (s == MILOC_OK) s = miloc_set_spectral(&c, n_channels, v_min_cms, dv_cms);
        if (s == MILOC_OK) s = miloc_set_background(&c, T_bg_K);
        if (s == MILOC_OK) s = miloc_run(&c, max_iter, tol, 1, &it, &d);
        if (s == MILOC_OK || s == MILOC_ENOTCONV) {
            const miloc_status g = miloc_get_populations(&c, x_out);
            if (g != MILOC_OK) s = g;
        }
        // nothing of this call may still run on the scratch when it returns
        (void)hipStreamSynchronize(c.stream);
    }
    if (carve.overflow) return MILOC_ENOMEM;
    if (s == MILOC_OK || s == MILOC_ENOTCONV) {
        if (iters_done) *iters_done = it;
        if (last_delta) *last_delta = d;
    }
    return s;
}

}  // extern "C"
