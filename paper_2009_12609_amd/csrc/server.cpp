// server.cpp -- 1D request loop (continuous batching) of libmiloc.
//
// Requests (a molecule, a shell model, a channel grid, a tolerance) are
// queued by miloc_server_submit and admitted by an admission thread when a
// slot is free and their device footprint fits the HBM budget (first fit in
// arrival order): host image, upload and admission kernels on a stream of its
// own, concurrently with the ticks.  Every tick advances every ready resident
// model by one ALI iteration (Sect. 2: march all transitions, then solve the
// statistical equilibrium of every shell): one captured HIP graph of four
// model-indexed kernels that walk device work lists, so models of different
// sizes, level counts and channel counts share the same launches and the
// graph never needs re-capturing.  Between ticks the worker thread reads each
// model's maximum relative change, retires converged or failed models (final
// spectra, populations to the host), frees their memory and takes in the
// admissions that have become ready.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "geometry.h"
#include "miloc.h"
#include "miloc_internal.h"

using namespace miloc;

namespace {

constexpr double kH = 6.62607015e-27;
constexpr double kK = 1.380649e-16;
constexpr double kC = 2.99792458e10;
constexpr double kAmu = 1.66053906660e-24;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtLog2e = 1.2011224087864498;
constexpr double kWindowK = 5.0;           // FP32 march: profile < e^-25 outside
constexpr int kMaxServeShells = 2048;      // per-shell LDS accumulators
constexpr int kMaxServeChannels = 512;
constexpr int kMaxServeLevels = 20;
constexpr int kRaysPerBlock = 16;          // 16 lanes per ray, 256 threads
constexpr int kSeBs = 16;
constexpr size_t kStageBytes = (size_t)64 << 20;   // pinned admission staging per round
constexpr size_t kResBytes = (size_t)64 << 20;     // pinned result area per tick
constexpr size_t kNoRes = ~(size_t)0;
// LDS tiers of the tick's march kernel (one captured graph each): the largest
// holds the FP64 per-shell accumulators of 2048 shells and 16 rays of 512
// channels; the smaller ones let more workgroups share a CU (160 KB of LDS:
// 8, 6, 5, 4, 3 and 2 workgroups) when the resident models are smaller.
constexpr int kLdsTiers = 6;
constexpr int kTierLds[kLdsTiers] = {20480, 27136, 32768, 40960, 53248, 65792};

// LDS bytes the tick's march kernel needs for one resident model.
constexpr int march_lds_need(int n, int nch)
{
    return (int)((((size_t)n * 2 * sizeof(double)) + 15) & ~(size_t)15) + kRaysPerBlock * nch * (int)sizeof(float) +
           kVecTailPadWords * (int)sizeof(float);
}
static_assert(march_lds_need(kMaxServeShells, kMaxServeChannels) <= kTierLds[kLdsTiers - 1],
              "the largest LDS tier must hold the largest served model");

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device allocation.
class Arena {
public:
    void init(size_t bytes) { free_[0] = bytes; size_ = bytes; }
    bool alloc(size_t n, size_t* off)
    {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) & ~(size_t)255;
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

// Host copy of one request and, once admitted, its device layout.
struct Request {
    uint64_t ticket = 0;
    // molecule
    int L = 0, T = 0;
    std::vector<double> E, g, A, nu, gamma;
    std::vector<int> up, lo;
    double mass = 0;
    // model
    int n = 0, nrays = 0;
    int64_t n_steps = 0;      // ray steps of the model's rays plus the centre line of sight
    std::vector<double> R, nH2, Tk, bt, vr, X, impact;
    int nch = 0;
    double vmin = 0, dv = 0, Tbg = 0, tol = 0;
    int max_iter = 0;
    // life cycle
    int state = 0;            // 0 queued, 1 active, 2 done, 3 failed, 4 cancelled
    bool cancel_req = false;  // cancel asked while active: the worker retires it
    bool ready = false;       // admitted on the device: the worker ticks it
    int iters = 0;
    double last_delta = INFINITY;
    double t_submit = 0, t_admit = 0, t_done = 0;
    miloc_status status = MILOC_OK;
    std::string error;
    // device
    size_t off = 0, bytes = 0;
    int slot = -1;
    ServeModel desc{};
    int phase = 0;              // 0: iterating, 1: spectra in the next tick, then retired
    std::vector<float> sp_host; // spectra copied back after the spectra tick (no room in the pinned area)
    size_t res_off = 0;         // offset of its results in the pinned result area, or kNoRes
    std::vector<double> Iscale, Ibg;
    // results
    std::vector<double> x, spectra;
};

// Arena block of one request: the regions filled from the host come first
// (one upload of [0, up_end)), then those the kernels fill.
struct Layout {
    size_t mol, roff, kmin, R, b, vrdv, area, shellv, x, nH2, Tk, nmolLb, Ibg, Ibg64, bsq, up_end;
    size_t steps, ke, acc, xn, q, spec, total;
};

Layout layout_of(const Request& r)
{
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t n) { const size_t at = o; o += (n + 255) & ~(size_t)255; return at; };
    l.mol = take(sizeof(MolDev));
    l.roff = take((size_t)(r.nrays + 1) * sizeof(int64_t));
    l.kmin = take((size_t)(r.nrays + 1) * sizeof(int));
    l.R = take(r.n * sizeof(double));
    l.b = take((size_t)(r.nrays + 1) * sizeof(double));
    l.vrdv = take(r.n * sizeof(double));
    l.area = take(r.nrays * sizeof(double));
    l.shellv = take(r.n * sizeof(float2));
    l.x = take((size_t)r.n * r.L * sizeof(double));
    l.nH2 = take(r.n * sizeof(double));
    l.Tk = take(r.n * sizeof(double));
    l.nmolLb = take(r.n * sizeof(double));
    l.Ibg = take(r.T * sizeof(float));
    l.Ibg64 = take(r.T * sizeof(double));
    l.bsq = take(r.n * sizeof(double));
    l.up_end = o;
    l.steps = take((size_t)r.n_steps * sizeof(float2));
    l.ke = take((size_t)r.n * r.T * sizeof(float2));
    l.acc = take((size_t)r.n * r.T * sizeof(double2));
    l.xn = take((size_t)r.n * r.L * sizeof(double));
    l.q = take(r.n * sizeof(double));
    l.spec = take((size_t)r.T * r.nch * sizeof(float));
    l.total = o;
    return l;
}

// Bytes of a request's results in the pinned result area (spectra, populations).
size_t result_bytes(const Request& r)
{
    return (((size_t)r.T * r.nch * sizeof(float) + 255) & ~(size_t)255) + (size_t)r.n * r.L * sizeof(double);
}

bool finite_pos(const double* a, int n, bool allow_zero)
{
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(a[i])) return false;
        if (allow_zero ? !(a[i] >= 0) : !(a[i] > 0)) return false;
    }
    return true;
}

}  // namespace

struct miloc_server {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    size_t budget = 0;
    int max_slots = 0;
    void* arena_mem = nullptr;
    Arena arena;

    // device tables
    ServeModel* d_models = nullptr;
    int4* d_march = nullptr;
    int2* d_cell = nullptr;
    int2* d_se = nullptr;
    int* d_counts = nullptr;             // n_march, n_cell, n_se
    unsigned long long* d_flags = nullptr;   // per slot: delta bits, bad
    size_t cap_march = 0, cap_cell = 0, cap_se = 0;
    ServeGrid grid{};
    hipGraph_t graph[kLdsTiers] = {};
    hipGraphExec_t graph_exec[kLdsTiers] = {};
    int tier = kLdsTiers - 1;            // LDS tier of the current resident set
    float* d_zero = nullptr;
    // pinned host areas: admission uploads, results of retiring models
    char* h_stage = nullptr;
    size_t stage_cap = 0;
    char* h_res = nullptr;
    size_t res_cap = 0;

    std::mutex mu;
    std::mutex err_mu;                   // guards err (set from caller and worker threads)
    std::condition_variable cv;
    std::deque<Request*> queue;
    std::vector<Request*> active;        // by slot (nullptr = free)
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool device_error = false;
    std::thread worker;
    std::thread admitter;
    hipStream_t adm_stream = nullptr;    // admission uploads and kernels
    bool adm_new = false;                // admissions became ready since the worker looked
    miloc_server_stats stats{};
};

namespace {

miloc_status sfail(miloc_server* s, miloc_status code, const std::string& m)
{
    if (s) {
        std::lock_guard<std::mutex> lk(s->err_mu);
        s->err = m;
    }
    return code;
}

// Admission, host part: the statics of a request (molecule table, ray layout,
// LTE start, per-shell values) written at their arena offsets into img, the
// host image of the block's first up_end bytes; independent per request.
// False with r->error set on failure.
bool admit_host(Request* r, char* img)
{
    const Layout lay = layout_of(*r);
    // molecule
    MolDev m;
    std::memset(&m, 0, sizeof(m));
    m.L = r->L;
    m.T = r->T;
    const double Emin = *std::min_element(r->E.begin(), r->E.end());
    for (int i = 0; i < r->L; ++i) { m.E[i] = r->E[i] - Emin; m.g[i] = r->g[i]; }
    for (int u = 0; u < r->L; ++u)
        for (int l = 0; l < u; ++l) m.gamma[u * r->L + l] = r->gamma[(size_t)u * r->L + l];
    for (int t = 0; t < r->T; ++t) {
        m.up[t] = r->up[t];
        m.lo[t] = r->lo[t];
        m.A[t] = r->A[t];
        m.gratio[t] = r->g[r->up[t]] / r->g[r->lo[t]];
        m.Ct[t] = kC * kC * kC * r->A[t] / (8.0 * kPi * r->nu[t] * r->nu[t] * r->nu[t]);
    }
    mol_pair_table(m);
    std::memcpy(img + lay.mol, &m, sizeof(m));
    // geometry and per-shell statics, in normalised radius units
    const int n = r->n;
    const double Rout = r->R[n - 1];
    double* Rn = reinterpret_cast<double*>(img + lay.R);
    double* b_all = reinterpret_cast<double*>(img + lay.b);   // the rays' impacts, then the centre line of sight
    double* an = reinterpret_cast<double*>(img + lay.area);
    for (int k = 0; k < n; ++k) Rn[k] = r->R[k] / Rout;
    Rn[n - 1] = 1.0;
    for (int j = 0; j < r->nrays; ++j) b_all[j] = r->impact[j] / Rout;
    b_all[r->nrays] = 0.0;
    for (int j = 0; j < r->nrays; ++j) {
        const double e0 = j == 0 ? 0.0 : 0.5 * (b_all[j] + b_all[j - 1]);
        const double e1 = j == r->nrays - 1 ? 1.0 : 0.5 * (b_all[j] + b_all[j + 1]);
        an[j] = kPi * (e1 * e1 - e0 * e0);
    }
    // ray layout of the model's rays and of the centre line of sight (spectra);
    // the step records themselves are computed on the device
    std::vector<int64_t> roff;
    std::vector<int> kmin;
    if (shell_ray_layout(n, Rn, r->nrays + 1, b_all, roff, kmin) != r->n_steps) {
        r->error = "ray step count mismatch";
        return false;
    }
    std::memcpy(img + lay.roff, roff.data(), roff.size() * sizeof(int64_t));
    std::memcpy(img + lay.kmin, kmin.data(), kmin.size() * sizeof(int));
    double* vrdv = reinterpret_cast<double*>(img + lay.vrdv);
    float2* sv = reinterpret_cast<float2*>(img + lay.shellv);
    double* xs = reinterpret_cast<double*>(img + lay.x);
    double* nmolLb = reinterpret_cast<double*>(img + lay.nmolLb);
    double* bsq = reinterpret_cast<double*>(img + lay.bsq);
    for (int k = 0; k < n; ++k) {
        vrdv[k] = r->vr[k] / r->dv;
        const double b = std::sqrt(2.0 * kK * r->Tk[k] / (r->mass * kAmu) + r->bt[k] * r->bt[k]);
        const double bs = b * std::sqrt(kPi);
        bsq[k] = bs;
        nmolLb[k] = r->nH2[k] * r->X[k] * Rout / bs;
        sv[k] = make_float2((float)(r->vr[k] / r->dv), (float)(r->dv * kSqrtLog2e / b));
        // LTE start at the local kinetic temperature (Sect. 3.3.2)
        double z = 0;
        for (int i = 0; i < r->L; ++i) z += m.g[i] * std::exp(-m.E[i] / r->Tk[k]);
        for (int i = 0; i < r->L; ++i) xs[(size_t)k * r->L + i] = m.g[i] * std::exp(-m.E[i] / r->Tk[k]) / z;
    }
    std::memcpy(img + lay.nH2, r->nH2.data(), n * sizeof(double));
    std::memcpy(img + lay.Tk, r->Tk.data(), n * sizeof(double));
    r->Iscale.resize(r->T);
    r->Ibg.resize(r->T);
    float* ibf = reinterpret_cast<float*>(img + lay.Ibg);
    for (int t = 0; t < r->T; ++t) {
        r->Iscale[t] = 2.0 * kH * std::pow(r->nu[t], 3) / (kC * kC);
        const double xx = r->Tbg > 0 ? kH * r->nu[t] / (kK * r->Tbg) : INFINITY;
        r->Ibg[t] = std::isfinite(xx) ? 1.0 / std::expm1(xx) : 0.0;
        ibf[t] = (float)r->Ibg[t];
    }
    std::memcpy(img + lay.Ibg64, r->Ibg.data(), r->T * sizeof(double));
    return true;
}

// Admission, device part, queued on the admission stream: one upload of the
// host image into the request's arena block, the ray steps and q (from the
// ray-sampled shell volumes) computed on the device, and the model
// descriptor.  img must stay untouched until the stream has drained.
bool admit_device(miloc_server* S, Request* r, const char* img)
{
    const Layout lay = layout_of(*r);
    char* base = static_cast<char*>(S->arena_mem) + r->off;
    auto dptr = [&](size_t o) { return static_cast<void*>(base + o); };
    const int n = r->n;
    if (hipMemcpyAsync(base, img, lay.up_end, hipMemcpyHostToDevice, S->adm_stream) != hipSuccess) {
        r->error = "upload failed";
        return false;
    }
    if (launch_ray_steps(S->adm_stream, n, static_cast<const double*>(dptr(lay.R)), r->nrays + 1,
                         static_cast<const double*>(dptr(lay.b)), static_cast<const int*>(dptr(lay.kmin)),
                         static_cast<const long long*>(dptr(lay.roff)), static_cast<const double*>(dptr(lay.vrdv)),
                         dptr(lay.steps), false) != hipSuccess ||
        launch_shell_weights(S->adm_stream, n, static_cast<const double*>(dptr(lay.R)), r->nrays,
                             static_cast<const double*>(dptr(lay.b)), static_cast<const double*>(dptr(lay.area)),
                             static_cast<double*>(dptr(lay.q)), static_cast<const double*>(dptr(lay.bsq)),
                             r->dv) != hipSuccess) {
        r->error = "admission kernel failed";
        return false;
    }
    ServeModel& d = r->desc;
    d = ServeModel{};
    March1DArgs<float>& a = d.m;
    a.n = n;
    a.nrays = r->nrays;
    a.nch = r->nch;
    a.ntr = r->T;
    a.steps = static_cast<const float2*>(dptr(lay.steps));
    a.ray_off = static_cast<const long long*>(dptr(lay.roff));
    a.kmin = static_cast<const int*>(dptr(lay.kmin));
    a.area = static_cast<const double*>(dptr(lay.area));
    a.shellv = static_cast<const float2*>(dptr(lay.shellv));
    a.ke = static_cast<const float2*>(dptr(lay.ke));
    a.Ibg = static_cast<const float*>(dptr(lay.Ibg));
    a.acc = static_cast<double2*>(dptr(lay.acc));
    a.chalf = 0.5 + r->vmin / r->dv;
    a.Kw = (float)(kWindowK * kSqrtLog2e);
    a.Iout = nullptr;
    a.trans_offset = 0;
    a.ntr_total = r->T;
    a.lds_acc = 1;
    a.acc_lds_bytes = (int)((((size_t)n * 2 * sizeof(double)) + 15) & ~(size_t)15);
    a.hf = nullptr;                      // requests carry single-Gaussian lines
    a.hfk = 0;
    a.hf_lo = a.hf_hi = 0.0;
    d.mol = static_cast<const MolDev*>(dptr(lay.mol));
    d.nmolLb = static_cast<const double*>(dptr(lay.nmolLb));
    d.ke_w = static_cast<float2*>(dptr(lay.ke));
    d.acc_w = static_cast<double2*>(dptr(lay.acc));
    d.x = static_cast<double*>(dptr(lay.x));
    d.xn = static_cast<double*>(dptr(lay.xn));
    d.nH2 = static_cast<const double*>(dptr(lay.nH2));
    d.Tk = static_cast<const double*>(dptr(lay.Tk));
    d.q = static_cast<const double*>(dptr(lay.q));
    d.delta_bits = S->d_flags + 2 * r->slot;
    d.bad = reinterpret_cast<unsigned int*>(S->d_flags + 2 * r->slot + 1);
    // a maser step fails the request like a failed solve (the tick's
    // prepare kernel clears the word before the march)
    a.maser = d.bad;
    d.nc = n;
    d.L = r->L;
    d.T = r->T;
    d.ibg64 = static_cast<const double*>(dptr(lay.Ibg64));
    d.spec = static_cast<float*>(dptr(lay.spec));
    d.zero = S->d_zero;
    d.mode = 0;
    return true;
}

// Upload the model table and the work lists of the ready resident set
// (res: by slot, nullptr where no ready model).
bool rebuild_tables(miloc_server* S, const std::vector<Request*>& res)
{
    std::vector<ServeModel> models(S->max_slots);
    std::vector<int4> march, spectra;
    std::vector<int2> cell, se;
    int need = 0;
    for (int sl = 0; sl < S->max_slots; ++sl) {
        Request* r = res[sl];
        if (!r) continue;
        need = std::max(need, march_lds_need(r->n, r->nch));
        models[sl] = r->desc;
        models[sl].mode = r->phase;
        if (r->phase == 0) {
            for (int t = 0; t < r->T; ++t)
                for (int j = 0; j < r->nrays; j += kRaysPerBlock) march.push_back(make_int4(sl, t, j, 0));
            for (int k = 0; k < r->n; k += kSeBs) se.push_back(make_int2(sl, k));
        } else {
            // centre spectra, four transitions per item; first in the list so
            // that these single-ray chains start at the beginning of the tick
            for (int t = 0; t < r->T; t += 4) spectra.push_back(make_int4(sl, t, 0, 1));
        }
        for (int k = 0; k < r->n; k += 256) cell.push_back(make_int2(sl, k));
    }
    march.insert(march.begin(), spectra.begin(), spectra.end());
    S->tier = kLdsTiers - 1;
    for (int t = kLdsTiers - 1; t >= 0 && kTierLds[t] >= need; --t) S->tier = t;
    if (march.size() > S->cap_march || cell.size() > S->cap_cell || se.size() > S->cap_se) return false;
    const int counts[3] = {(int)march.size(), (int)cell.size(), (int)se.size()};
    bool ok = hipMemcpyAsync(S->d_models, models.data(), models.size() * sizeof(ServeModel),
                             hipMemcpyHostToDevice, S->stream) == hipSuccess;
    ok = ok && (march.empty() || hipMemcpyAsync(S->d_march, march.data(), march.size() * sizeof(int4),
                                                hipMemcpyHostToDevice, S->stream) == hipSuccess);
    ok = ok && (cell.empty() || hipMemcpyAsync(S->d_cell, cell.data(), cell.size() * sizeof(int2),
                                               hipMemcpyHostToDevice, S->stream) == hipSuccess);
    ok = ok && (se.empty() || hipMemcpyAsync(S->d_se, se.data(), se.size() * sizeof(int2),
                                             hipMemcpyHostToDevice, S->stream) == hipSuccess);
    ok = ok && hipMemcpyAsync(S->d_counts, counts, sizeof(counts), hipMemcpyHostToDevice, S->stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(S->stream) == hipSuccess;
    return ok;
}

// Results of a model whose spectra ran in the last tick: host copies were
// queued after the tick; convert the spectra to CGS.
void take_results(Request* r, const float* sp)
{
    r->spectra.resize((size_t)r->T * r->nch);
    for (int t = 0; t < r->T; ++t)
        for (int c = 0; c < r->nch; ++c)
            r->spectra[(size_t)t * r->nch + c] = (double)sp[(size_t)t * r->nch + c] * r->Iscale[t];
}

// Admission thread: takes queued requests in arrival order while a slot,
// room in the arena and room in the pinned staging area are free, builds
// their host images (in parallel), uploads them and runs the admission
// kernels on its own stream, and hands them to the worker once the stream
// has drained.  It runs while the worker's ticks run, so a request arriving
// mid-tick is admitted during that tick rather than after it.
void admit_loop(miloc_server* S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<Request*> to_admit;
        std::vector<size_t> img_off;              // host images in the pinned staging area
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop || S->device_error) return;
            // a free slot and room in the arena, first fit in arrival order,
            // as many as the staging area holds this round; the slot is held
            // (not yet ready) while the admission runs
            size_t staged_bytes = 0;
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                Request* r = *it;
                if (r->state == 4) { it = S->queue.erase(it); continue; }
                int slot = -1;
                for (int i = 0; i < S->max_slots; ++i)
                    if (!S->active[i]) { slot = i; break; }
                size_t off = 0;
                if (slot < 0) break;
                const size_t up = (layout_of(*r).up_end + 255) & ~(size_t)255;
                if (staged_bytes + up > S->stage_cap) break;
                if (!S->arena.alloc(r->bytes, &off)) { ++it; continue; }
                img_off.push_back(staged_bytes);
                staged_bytes += up;
                r->off = off;
                r->slot = slot;
                r->state = 1;
                r->ready = false;
                r->t_admit = now_s();
                S->active[slot] = r;
                S->stats.admitted++;
                to_admit.push_back(r);
                it = S->queue.erase(it);
            }
            if (to_admit.empty()) {
                S->cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        auto fail_admission = [&](Request* r) {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->active[r->slot] != r) return;
            r->state = 3;
            r->status = MILOC_EDEVICE;
            r->t_done = now_s();
            S->arena.release(r->off, r->bytes);
            S->active[r->slot] = nullptr;
            S->stats.failed++;
        };
        // host images of all new requests in parallel, then one upload and
        // two kernels each, and a single synchronisation of the admission stream
        std::vector<char> host_ok(to_admit.size(), 0);
        {
            const size_t nw = std::min<size_t>(to_admit.size(),
                                               std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
            std::vector<std::thread> pool;
            std::atomic<size_t> next{0};
            for (size_t w = 0; w < nw; ++w)
                pool.emplace_back([&]() {
                    for (size_t i = next++; i < to_admit.size(); i = next++)
                        host_ok[i] = admit_host(to_admit[i], S->h_stage + img_off[i]) ? 1 : 0;
                });
            for (auto& t : pool) t.join();
        }
        for (size_t i = 0; i < to_admit.size(); ++i) {
            Request* r = to_admit[i];
            if (!host_ok[i] || !admit_device(S, r, S->h_stage + img_off[i])) {
                fail_admission(r);
                to_admit[i] = nullptr;
            }
        }
        const bool ok = hipStreamSynchronize(S->adm_stream) == hipSuccess;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (!ok) {
                S->device_error = true;
                sfail(S, MILOC_EDEVICE, "admission upload failed");
                S->stop = true;
                S->cv.notify_all();
                return;
            }
            for (Request* r : to_admit)
                if (r && S->active[r->slot] == r && r->state == 1) r->ready = true;
            S->adm_new = true;
        }
        S->cv.notify_all();
    }
}

// Worker thread: ticks over the ready resident models.
void worker_loop(miloc_server* S)
{
    (void)hipSetDevice(S->device);
    bool dirty = true;
    std::vector<unsigned long long> flags(2 * (size_t)S->max_slots);
    // the ready residents by slot, taken under the lock: the admission thread
    // fills free slots meanwhile, the worker alone retires ready ones
    std::vector<Request*> res(S->max_slots, nullptr);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->adm_new) {
                S->adm_new = false;
                dirty = true;
            }
            int n_active = 0, n_ready = 0;
            for (int sl = 0; sl < S->max_slots; ++sl) {
                Request* r = S->active[sl];
                res[sl] = r && r->ready ? r : nullptr;
                n_active += r ? 1 : 0;
                n_ready += res[sl] ? 1 : 0;
            }
            S->stats.active = n_active;
            S->stats.queued = (int64_t)S->queue.size();
            S->stats.peak_active = std::max<int64_t>(S->stats.peak_active, n_active);
            if (S->device_error) return;
            if (n_ready == 0) {
                // held slots are admissions in flight: wait for them
                if (S->stop && n_active == 0) return;
                S->cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        if (dirty) {
            if (!rebuild_tables(S, res)) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->device_error = true;
                sfail(S, MILOC_EDEVICE, "work-list upload failed");
                S->stop = true;
                S->cv.notify_all();
                return;
            }
            dirty = false;
        }
        // one tick = one ALI iteration of every iterating model and the centre
        // spectra of every model that finished in the previous tick
        const double t0 = now_s();
        hipError_t e = hipGraphLaunch(S->graph_exec[S->tier], S->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(flags.data(), S->d_flags, flags.size() * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, S->stream);
        // results of the models whose spectra run in this tick: into the
        // pinned result area while it has room, else into the request
        size_t res_used = 0;
        for (Request* r : res) {
            if (!r || r->phase != 1 || e != hipSuccess) continue;
            const size_t sp_bytes = (size_t)r->T * r->nch * sizeof(float);
            const size_t x_bytes = (size_t)r->n * r->L * sizeof(double);
            void* sp_dst;
            void* x_dst;
            if (res_used + result_bytes(*r) <= S->res_cap) {
                r->res_off = res_used;
                sp_dst = S->h_res + res_used;
                x_dst = S->h_res + res_used + ((sp_bytes + 255) & ~(size_t)255);
                res_used += (result_bytes(*r) + 255) & ~(size_t)255;
            } else {
                r->res_off = kNoRes;
                r->sp_host.resize((size_t)r->T * r->nch);
                r->x.resize((size_t)r->n * r->L);
                sp_dst = r->sp_host.data();
                x_dst = r->x.data();
            }
            e = hipMemcpyAsync(sp_dst, r->desc.spec, sp_bytes, hipMemcpyDeviceToHost, S->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(x_dst, r->desc.x, x_bytes, hipMemcpyDeviceToHost, S->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
        if (e != hipSuccess) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->device_error = true;
            sfail(S, MILOC_EDEVICE, std::string("tick failed: ") + hipGetErrorString(e));
            for (Request*& r : S->active)
                if (r) { r->state = 3; r->status = MILOC_EDEVICE; r->t_done = now_s(); r = nullptr; }
            S->stop = true;
            S->cv.notify_all();
            return;
        }
        bool retired = false;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.ticks++;
            S->stats.busy_s += now_s() - t0;
            auto retire = [&](Request* r) {
                r->t_done = now_s();
                if (r->cancel_req) {
                    r->state = 4;
                    S->stats.cancelled++;
                } else {
                    const bool good = r->status == MILOC_OK || r->status == MILOC_ENOTCONV;
                    if (good) {
                        if (r->res_off != kNoRes) {
                            const char* src = S->h_res + r->res_off;
                            const size_t sp_bytes = (size_t)r->T * r->nch * sizeof(float);
                            const double* xs = reinterpret_cast<const double*>(src + ((sp_bytes + 255) & ~(size_t)255));
                            r->x.assign(xs, xs + (size_t)r->n * r->L);
                            take_results(r, reinterpret_cast<const float*>(src));
                        } else {
                            take_results(r, r->sp_host.data());
                        }
                    }
                    r->state = good ? 2 : 3;
                    if (good) S->stats.completed++; else S->stats.failed++;
                }
                S->arena.release(r->off, r->bytes);
                S->active[r->slot] = nullptr;
                dirty = true;
                retired = true;
            };
            for (int sl = 0; sl < S->max_slots; ++sl) {
                Request* r = res[sl];
                if (!r) continue;
                if (r->phase == 1) {               // its spectra ran in this tick
                    retire(r);
                    continue;
                }
                r->iters++;
                double d;
                std::memcpy(&d, &flags[2 * sl], sizeof(double));
                r->last_delta = d;
                const unsigned bad = (unsigned)(flags[2 * sl + 1] & 0xffffffffu);
                if (r->cancel_req) {
                    retire(r);
                } else if (bad) {
                    r->status = MILOC_ENUMERIC;
                    retire(r);
                } else if ((r->tol > 0 && d < r->tol) || r->iters >= r->max_iter) {
                    r->status = (r->tol > 0 && !(d < r->tol)) ? MILOC_ENOTCONV : MILOC_OK;
                    r->phase = 1;
                    dirty = true;
                }
            }
        }
        if (retired) S->cv.notify_all();
    }
}

}  // namespace

extern "C" {

miloc_status miloc_server_create(int hip_device, size_t hbm_budget_bytes, int max_slots, miloc_server** out)
{
    if (!out) return MILOC_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096) return MILOC_EINVAL;
    if (hbm_budget_bytes < (1u << 20)) return MILOC_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return MILOC_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return MILOC_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MILOC_EDEVICE;
    if (hipSetDevice(hip_device) != hipSuccess) return MILOC_EDEVICE;
    std::unique_ptr<miloc_server> S(new (std::nothrow) miloc_server());
    if (!S) return MILOC_ENOMEM;
    S->device = hip_device;
    S->budget = hbm_budget_bytes;
    S->max_slots = max_slots;
    S->active.assign(max_slots, nullptr);
    // worst-case work lists: every slot holding a 19-transition model with
    // 4 * 2048 rays
    S->cap_march = (size_t)max_slots * 19 * ((kMaxServeShells * 4) / kRaysPerBlock + 1);
    S->cap_cell = (size_t)max_slots * (kMaxServeShells / 256 + 1);
    S->cap_se = (size_t)max_slots * (kMaxServeShells / kSeBs + 1);
    bool ok = hipStreamCreate(&S->stream) == hipSuccess;
    ok = ok && hipStreamCreate(&S->adm_stream) == hipSuccess;
    ok = ok && hipMalloc(&S->arena_mem, hbm_budget_bytes) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&S->d_models), max_slots * sizeof(ServeModel)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&S->d_march), S->cap_march * sizeof(int4)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&S->d_cell), S->cap_cell * sizeof(int2)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&S->d_se), S->cap_se * sizeof(int2)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&S->d_counts), 4 * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&S->d_flags), 2 * max_slots * sizeof(unsigned long long)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&S->d_zero), kMaxTrans * sizeof(float)) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&S->h_stage), kStageBytes) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&S->h_res), kResBytes) == hipSuccess;
    if (ok) {
        S->stage_cap = kStageBytes;
        S->res_cap = kResBytes;
    }
    if (!ok) {
        miloc_server_destroy(S.release());
        return MILOC_ENOMEM;
    }
    (void)hipMemset(S->d_counts, 0, 4 * sizeof(int));
    (void)hipMemset(S->d_flags, 0, 2 * max_slots * sizeof(unsigned long long));
    (void)hipMemset(S->d_zero, 0, kMaxTrans * sizeof(float));
    (void)hipMemset(S->d_models, 0, max_slots * sizeof(ServeModel));
    S->arena.init(hbm_budget_bytes);
    // grid of the persistent kernels and the captured tick graph
    S->grid.march_blocks = 2048;
    S->grid.cell_blocks = 512;
    S->grid.se_blocks = 2048;
    S->grid.se_bs = kSeBs;
    S->grid.march_lds = kTierLds[kLdsTiers - 1];
    S->grid.se_lds = kSeBs * (kMaxServeLevels * (kMaxServeLevels + 1) + kMaxServeLevels) * (int)sizeof(double);
    ServeTables tb{S->d_models, S->d_march, S->d_counts, S->d_cell, S->d_counts + 1, S->d_se, S->d_counts + 2};
    ok = serve_set_attributes(S->grid) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    for (int t = 0; t < kLdsTiers && ok; ++t) {
        ServeGrid g = S->grid;
        g.march_lds = kTierLds[t];
        ok = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const hipError_t le = launch_serve_tick(S->stream, tb, g);
            const hipError_t ce = hipStreamEndCapture(S->stream, &S->graph[t]);
            ok = le == hipSuccess && ce == hipSuccess;
        }
        ok = ok && hipGraphInstantiate(&S->graph_exec[t], S->graph[t], nullptr, nullptr, 0) == hipSuccess;
    }
    if (!ok) {
        miloc_server_destroy(S.release());
        return MILOC_EDEVICE;
    }
    miloc_server* raw = S.release();
    raw->worker = std::thread(worker_loop, raw);
    raw->admitter = std::thread(admit_loop, raw);
    *out = raw;
    return MILOC_OK;
}

void miloc_server_destroy(miloc_server* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Request* r : S->queue) r->state = 4;
        for (Request* r : S->active)
            if (r) r->cancel_req = true;
    }
    S->cv.notify_all();
    if (S->admitter.joinable()) S->admitter.join();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->device);
    if (S->adm_stream) (void)hipStreamSynchronize(S->adm_stream);
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    for (int t = 0; t < kLdsTiers; ++t) {
        if (S->graph_exec[t]) (void)hipGraphExecDestroy(S->graph_exec[t]);
        if (S->graph[t]) (void)hipGraphDestroy(S->graph[t]);
    }
    void* bufs[] = {S->arena_mem, S->d_models, S->d_march, S->d_cell, S->d_se, S->d_counts, S->d_flags,
                    S->d_zero};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (S->h_stage) (void)hipHostFree(S->h_stage);
    if (S->h_res) (void)hipHostFree(S->h_res);
    if (S->adm_stream) (void)hipStreamDestroy(S->adm_stream);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
}

const char* miloc_server_last_error(const miloc_server* S) { return S ? S->err.c_str() : ""; }

}  // extern "C"

namespace {

// Validates one request and copies it into host memory; r->bytes is its
// arena footprint.
miloc_status parse_request(miloc_server* S, const miloc_molecule* mol, const miloc_model1d* m, int n_channels,
                           double v_min_cms, double dv_cms, double T_bg_K, double tol, int max_iter,
                           std::unique_ptr<Request>& r)
{
    if (!mol || !m) return sfail(S, MILOC_EINVAL, "NULL molecule or model");
    r.reset(new Request());
    // molecule
    const int L = mol->n_levels, T = mol->n_trans;
    if (!mol->E_K || !mol->g || !mol->up || !mol->lo || !mol->A || !mol->nu_Hz || !mol->gamma_down)
        return sfail(S, MILOC_EINVAL, "NULL molecule field");
    if (L < 2 || L > kMaxServeLevels) return sfail(S, MILOC_EINVAL, "served models need 2..20 levels");
    if (T < 1 || T > L * (L - 1) / 2) return sfail(S, MILOC_EINVAL, "n_trans out of range");
    if (!finite_pos(mol->g, L, false) || !finite_pos(mol->A, T, false) || !finite_pos(mol->nu_Hz, T, false) ||
        !(mol->mass_amu > 0))
        return sfail(S, MILOC_EINVAL, "bad molecule values");
    for (int i = 0; i < L; ++i)
        if (!std::isfinite(mol->E_K[i])) return sfail(S, MILOC_EINVAL, "bad level energy");
    std::vector<char> seen((size_t)L * L, 0);
    for (int t = 0; t < T; ++t) {
        const int u = mol->up[t], l = mol->lo[t];
        if (u < 0 || u >= L || l < 0 || l >= u || seen[(size_t)u * L + l]) return sfail(S, MILOC_EINVAL, "bad transition");
        seen[(size_t)u * L + l] = 1;
    }
    for (int u = 0; u < L; ++u)
        for (int l = 0; l < u; ++l)
            if (!(mol->gamma_down[(size_t)u * L + l] >= 0) || !std::isfinite(mol->gamma_down[(size_t)u * L + l]))
                return sfail(S, MILOC_EINVAL, "bad collision coefficient");
    r->L = L;
    r->T = T;
    r->E.assign(mol->E_K, mol->E_K + L);
    r->g.assign(mol->g, mol->g + L);
    r->up.assign(mol->up, mol->up + T);
    r->lo.assign(mol->lo, mol->lo + T);
    r->A.assign(mol->A, mol->A + T);
    r->nu.assign(mol->nu_Hz, mol->nu_Hz + T);
    r->gamma.assign(mol->gamma_down, mol->gamma_down + (size_t)L * L);
    r->mass = mol->mass_amu;
    // model
    const int n = m->n_shells;
    if (!m->r_out_cm || !m->n_H2 || !m->T_kin || !m->b_turb_cms || !m->v_r_cms || !m->abundance)
        return sfail(S, MILOC_EINVAL, "NULL model field");
    if (n < 1 || n > kMaxServeShells) return sfail(S, MILOC_EINVAL, "served models need 1..2048 shells");
    if (m->n_rays < 1 || m->n_rays > 4 * kMaxServeShells) return sfail(S, MILOC_EINVAL, "n_rays out of range");
    if (!finite_pos(m->r_out_cm, n, false) || !finite_pos(m->n_H2, n, true) || !finite_pos(m->T_kin, n, false) ||
        !finite_pos(m->b_turb_cms, n, true) || !finite_pos(m->abundance, n, true))
        return sfail(S, MILOC_EINVAL, "negative or non-finite shell values");
    for (int k = 0; k < n; ++k) {
        if (!std::isfinite(m->v_r_cms[k])) return sfail(S, MILOC_EINVAL, "non-finite velocity");
        if (k > 0 && !(m->r_out_cm[k] > m->r_out_cm[k - 1])) return sfail(S, MILOC_EINVAL, "radii must increase");
    }
    if (n_channels < 8 || n_channels > kMaxServeChannels || !(dv_cms > 0) || !std::isfinite(v_min_cms) ||
        !std::isfinite(dv_cms))
        return sfail(S, MILOC_EINVAL, "bad channel grid (8..512 channels)");
    if (!(T_bg_K >= 0) || !std::isfinite(T_bg_K) || !std::isfinite(tol) || max_iter < 1)
        return sfail(S, MILOC_EINVAL, "bad background, tolerance or iteration cap");
    r->n = n;
    r->nrays = m->n_rays;
    r->R.assign(m->r_out_cm, m->r_out_cm + n);
    r->nH2.assign(m->n_H2, m->n_H2 + n);
    r->Tk.assign(m->T_kin, m->T_kin + n);
    r->bt.assign(m->b_turb_cms, m->b_turb_cms + n);
    r->vr.assign(m->v_r_cms, m->v_r_cms + n);
    r->X.assign(m->abundance, m->abundance + n);
    const double Rout = r->R[n - 1];
    r->impact.resize(r->nrays);
    for (int j = 0; j < r->nrays; ++j) {
        r->impact[j] = m->impact_cm ? m->impact_cm[j] : (j + 0.5) * Rout / r->nrays;
        if (!(r->impact[j] > 0 && r->impact[j] < Rout) || (j > 0 && !(r->impact[j] > r->impact[j - 1])))
            return sfail(S, MILOC_EINVAL, "impact parameters must increase inside (0, R)");
    }
    // ray steps: 2 (n - 1 - kmin) + 2 per ray, plus the centre line of sight
    {
        std::vector<double> Rn(n);
        for (int k = 0; k < n; ++k) Rn[k] = r->R[k] / Rout;
        Rn[n - 1] = 1.0;
        r->n_steps = 2 * (int64_t)n;
        for (int j = 0; j < r->nrays; ++j) {
            const double bj = r->impact[j] / Rout;
            const int km = std::min<int>(n - 1, (int)(std::upper_bound(Rn.begin(), Rn.end(), bj) - Rn.begin()));
            r->n_steps += 2 * (int64_t)(n - 1 - km) + 2;
        }
    }
    // band must hold every line out to 5 Doppler widths
    double maxu = 0;
    for (int k = 0; k < n; ++k) {
        const double b = std::sqrt(2.0 * kK * r->Tk[k] / (r->mass * kAmu) + r->bt[k] * r->bt[k]);
        maxu = std::max(maxu, std::fabs(r->vr[k]) + 5.0 * b);
    }
    if (-maxu < v_min_cms || maxu > v_min_cms + n_channels * dv_cms)
        return sfail(S, MILOC_EINVAL, "velocity band does not contain |v| + 5 b");
    r->nch = n_channels;
    r->vmin = v_min_cms;
    r->dv = dv_cms;
    r->Tbg = T_bg_K;
    r->tol = tol;
    r->max_iter = max_iter;
    if ((size_t)T * ((r->nrays + kRaysPerBlock - 1) / kRaysPerBlock) > S->cap_march / (size_t)S->max_slots)
        return sfail(S, MILOC_EINVAL, "too many transitions x rays for one serving slot");
    const Layout lay = layout_of(*r);
    if (lay.up_end > kStageBytes) return sfail(S, MILOC_EINVAL, "request too large for the staging area");
    r->bytes = lay.total;
    return MILOC_OK;
}

}  // namespace

extern "C" {

miloc_status miloc_server_footprint(miloc_server* S, const miloc_molecule* mol, const miloc_model1d* m,
                                    int n_channels, double v_min_cms, double dv_cms, double T_bg_K,
                                    size_t* bytes)
{
    if (!S || !bytes) return MILOC_EINVAL;
    std::unique_ptr<Request> r;
    const miloc_status st = parse_request(S, mol, m, n_channels, v_min_cms, dv_cms, T_bg_K, 0.0, 1, r);
    if (st != MILOC_OK) return st;
    *bytes = r->bytes;
    return MILOC_OK;
}

miloc_status miloc_server_submit(miloc_server* S, const miloc_molecule* mol, const miloc_model1d* m,
                                 int n_channels, double v_min_cms, double dv_cms, double T_bg_K, double tol,
                                 int max_iter, uint64_t* ticket)
{
    if (!S || !ticket) return MILOC_EINVAL;
    std::unique_ptr<Request> r;
    const miloc_status st = parse_request(S, mol, m, n_channels, v_min_cms, dv_cms, T_bg_K, tol, max_iter, r);
    if (st != MILOC_OK) return st;
    if (r->bytes > S->budget) return sfail(S, MILOC_EBUSY, "request larger than the whole HBM budget");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->device_error || S->stop) return sfail(S, MILOC_EDEVICE, "server stopped");
    r->ticket = S->next_ticket++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->all[r->ticket] = std::move(r);
    S->stats.submitted++;
    S->cv.notify_all();
    return MILOC_OK;
}

miloc_status miloc_server_poll(miloc_server* S, uint64_t ticket, int* done)
{
    if (!S || !done) return MILOC_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return sfail(S, MILOC_EINVAL, "unknown ticket");
    *done = it->second->state >= 2 ? 1 : 0;
    return MILOC_OK;
}

miloc_status miloc_server_wait(miloc_server* S, uint64_t ticket, double timeout_s, int* done)
{
    if (!S || !done) return MILOC_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return sfail(S, MILOC_EINVAL, "unknown ticket");
    Request* r = it->second.get();
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(0.0, timeout_s));
    while (r->state < 2 && !S->device_error) {
        if (S->cv.wait_until(lk, until) == std::cv_status::timeout) break;
    }
    *done = r->state >= 2 ? 1 : 0;
    return MILOC_OK;
}

miloc_status miloc_server_result_sizes(miloc_server* S, uint64_t ticket, int* n_shells, int* n_levels,
                                       int* n_trans, int* n_channels)
{
    if (!S) return MILOC_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return sfail(S, MILOC_EINVAL, "unknown ticket");
    const Request* r = it->second.get();
    if (n_shells) *n_shells = r->n;
    if (n_levels) *n_levels = r->L;
    if (n_trans) *n_trans = r->T;
    if (n_channels) *n_channels = r->nch;
    return MILOC_OK;
}

miloc_status miloc_server_take(miloc_server* S, uint64_t ticket, double* x_out, double* spectra_out,
                               miloc_result_info* info)
{
    if (!S) return MILOC_EINVAL;
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return sfail(S, MILOC_EINVAL, "unknown ticket");
        if (it->second->state < 2) return sfail(S, MILOC_ESTATE, "request not finished");
        r = std::move(it->second);
        S->all.erase(it);
    }
    if (info) {
        info->iterations = r->iters;
        info->last_delta = r->last_delta;
        info->latency_s = r->t_done - r->t_submit;
        info->queue_s = r->t_admit > 0 ? r->t_admit - r->t_submit : r->t_done - r->t_submit;
        info->status = r->state == 4 ? MILOC_ESTATE : r->status;
    }
    if (r->state == 2) {
        if (x_out) std::memcpy(x_out, r->x.data(), r->x.size() * sizeof(double));
        if (spectra_out) std::memcpy(spectra_out, r->spectra.data(), r->spectra.size() * sizeof(double));
        return r->status;
    }
    if (r->state == 4) return MILOC_ESTATE;
    return r->status == MILOC_OK ? MILOC_EDEVICE : r->status;
}

miloc_status miloc_server_cancel(miloc_server* S, uint64_t ticket)
{
    if (!S) return MILOC_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return sfail(S, MILOC_EINVAL, "unknown ticket");
    Request* r = it->second.get();
    if (r->state >= 2) return MILOC_OK;
    if (r->state == 0) {
        r->state = 4;
        r->t_done = now_s();
        auto q = std::find(S->queue.begin(), S->queue.end(), r);
        if (q != S->queue.end()) S->queue.erase(q);
        S->stats.cancelled++;
        S->cv.notify_all();
    } else {
        r->cancel_req = true;   // the worker retires it after the current tick
    }
    return MILOC_OK;
}

miloc_status miloc_server_get_stats(miloc_server* S, miloc_server_stats* out)
{
    if (!S || !out) return MILOC_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->arena_used = (int64_t)S->arena.used();
    return MILOC_OK;
}

}  // extern "C"
