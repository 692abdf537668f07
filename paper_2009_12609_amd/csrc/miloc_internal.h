// miloc_internal.h -- shared definitions of the host runtime and the gfx950 kernels.
//
// Internal units (chosen so that every FP32 quantity of the march is O(1)):
//   * intensities are photon occupation numbers, I' = I / (2 h nu^3 / c^2), so
//     B_ul J = A J' and B_lu J = (g_u/g_l) A J' in the equilibrium equations;
//   * lengths are in "march units": the cell size for 3D grids, the outer
//     radius for 1D models;
//   * velocities are in channel units (v / dv), and the line-profile argument is
//     carried as x * sqrt(log2 e) so that exp(-x^2) = exp2(-xs^2).
// With these, a step of length len in cell k contributes
//   tau_c = khat * len * e_c,  emission = ehat * len * e_c * beta_c,
//   e_c = exp(-((v_c + w)/b)^2),
// where khat, ehat carry kappa/(b sqrt(pi)) and eta/(b sqrt(pi)) times the
// length unit (Sect. 2, Eq. (3) in intensity form).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miloc {

constexpr int kMaxLevels = 32;
constexpr int kMaxTrans = kMaxLevels * (kMaxLevels - 1) / 2;

// Negative line-centre optical depth of one step (population inversion, a
// maser) below which a march raises its maser flag instead of marching on
// quietly: exp(40) = 2.4e17 of gain in a single step, and the FP32 exponential
// overflows near -88.
constexpr double kMaserTauMin = -40.0;

// Words of a march workgroup's LDS allocation that lie after each channel
// vector (the next vector, the queues or padding): the FP32 channel passes
// read up to this many words past the start of a step's window
// unconditionally and use only the values inside it.
constexpr int kVecTailPadWords = 64;

// Molecule constants on the device (read through uniform loads).
struct MolDev {
    int L, T;
    double E[kMaxLevels];        // E_i / k_B - min E  [K]
    double g[kMaxLevels];
    double gamma[kMaxLevels * kMaxLevels];   // [u*L + l], u > l
    int up[kMaxTrans], lo[kMaxTrans];
    double A[kMaxTrans];
    double gratio[kMaxTrans];    // g_u / g_l
    double Ct[kMaxTrans];        // c^3 A / (8 pi nu^3) [cm^3 s^-1 ... per unit n_mol]
    int pair_t[kMaxLevels * kMaxLevels];   // [u*kMaxLevels + l]: the transition u -> l, -1 if none
};

// Fills MolDev::pair_t from up/lo (the caller has rejected duplicate pairs).
inline void mol_pair_table(MolDev& m)
{
    for (int i = 0; i < kMaxLevels * kMaxLevels; ++i) m.pair_t[i] = -1;
    for (int t = 0; t < m.T; ++t) m.pair_t[m.up[t] * kMaxLevels + m.lo[t]] = t;
}

// One 3D ray direction of the regular-grid march.  All N*N rays of a
// direction share one crossing pattern (same fractional transverse offset),
// stored as a list of steps of the representative ray.
struct DirDev {
    double d[3];          // unit propagation vector
    double aw;            // |d_m|: ray cross-section per unit face area
    int sa, sb;           // move direction (+1/-1) along the transverse axes a, b
    int sta, stb;         // memory stride of one cell along a, b (positive)
    int stride_m;         // signed memory offset of one move along the main axis
    int start_off;        // memory offset of the start cell of ray (0, 0)
    int step0, nsteps;    // slice of the step table
    int m, fwd;           // main axis, 1 if d_m > 0
    int lstart0;          // offset of this direction's N+1 layer starts
    double maxlen;        // longest step of the pattern (cell units)
};

// One step of a regular-grid crossing pattern.  FP32 marches store log2 of
// the length (their profile exponent absorbs it), FP64 marches the length.
template <typename T>
struct StepRec {
    T len;                // path length in cell units (FP32: its base-2 logarithm)
    int flags;            // moves before this step: 1 = main axis, 2 = axis a, 4 = axis b
};

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };
template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

template <typename T>
struct March3DArgs {
    int N, nc, nch, ntr;
    int rays_per_dir, blocks_per_dir, n_dir;
    const DirDev* dirs;
    const StepRec<T>* steps;
    const typename V4<T>::type* win;     // [n_dir][nc] {x0, ibs, first channel, n channels}
    const typename V2<T>::type* ke;      // [nc][ntr_total] {khat, ehat}
    const T* Ibg;                        // [ntr], occupation units
    typename V2<T>::type* E;             // per-step partial sums [ntr][total steps][rays]
    size_t e_tstride;                    // total steps * rays (one transition of E)
    T* Iout;                             // spectra: [n_dir*rays][nch] or null
    int trans_offset;                    // first transition of this launch
    int step_lds_bytes;                  // LDS bytes reserved for the step list
    int ich;                             // LDS stride of one ray's channel vector
    int queue_lds_offset;                // LDS offset of the per-ray accumulation queues
    int ntr_total;                       // transitions in ke / acc (cell-major stride)
    const typename V2<T>::type* hf;      // hyperfine components [ntr_total][hfk] {offset / dv, strength}, or null
    int hfk;                             // components per transition (zero-strength padding)
    unsigned* maser;                     // set to 1 by a step with line-centre tau < kMaserTauMin
    // FP32 single-Gaussian accumulating march only: per (direction, ray) the
    // lowest channel any window of the ray starts at, or null; a ray's LDS
    // vector then holds channels base .. base + span_w - 1 only
    const int* rbase;
    int span_w;
};

// Per-cell gather of the per-step partial sums written by march3d, for the
// directions of one main axis.
template <typename T>
struct Gather3DArgs {
    int N, ntr, trans_offset, ntr_total, nq;
    int st_a, st_b, st_m;                // memory strides of the group's axes
    const int* qlist;                    // directions of this main axis
    const DirDev* dirs;
    const int* lstart;                   // layer starts
    const int2* moves;                   // cumulative (a, b) moves per step
    const typename V2<T>::type* E;
    size_t e_tstride;
    double2* acc;                        // [nc][ntr_total]
    int overwrite;                       // 1: the first gather of the launch's transitions writes the sums
};

template <typename T>
struct March1DArgs {
    int n, nrays, nch, ntr;
    const typename V2<T>::type* steps;   // per ray: 2 (n - 1 - kmin) + 2 steps {len / R_out, Doppler shift / dv}
    const long long* ray_off;            // first step of each ray
    const int* kmin;                     // innermost shell of each ray
    const double* area;                  // ray weights / R_out^2
    const typename V2<T>::type* shellv;  // {Ur, ibs} per shell
    const typename V2<T>::type* ke;      // [n][ntr_total]
    const T* Ibg;                        // [ntr_total]
    double2* acc;                        // [n][ntr_total]
    double chalf;
    T Kw;
    T* Iout;                             // spectra: [ntr][nrays][nch] or null
    int trans_offset;
    int ntr_total;                       // transitions in ke / acc (cell-major stride)
    int lds_acc;                         // per-shell LDS accumulators (set by the launcher)
    int acc_lds_bytes;                   // their size
    const typename V2<T>::type* hf;      // hyperfine components as in March3DArgs, or null
    int hfk;
    double hf_lo, hf_hi;                 // lowest / highest component offset (channels; <= 0, >= 0)
    unsigned* maser;                     // as in March3DArgs
    // Part of each ray marched (sub-iterations in an optically thick core of
    // shells 0..core_k; the launch then covers only rays that reach it):
    // kSegWhole the whole ray from I_bg; kSegEnvelopeIn its inward steps
    // outside the core, from I_bg, leaving in Iout the intensity it enters
    // the core with; kSegCore its steps inside the core, from Ient.
    int seg;
    int core_k;
    const T* Ient;                       // kSegCore: [ntr][nrays][nch] entry intensities
};

constexpr int kSegWhole = 0;
constexpr int kSegEnvelopeIn = 1;
constexpr int kSegCore = 2;

struct SEArgs {
    int nc, L, ntr, use_ali, bs;
    const MolDev* mol;
    const double* x_old;                 // [nc][L]
    double* x_new;                       // [nc][L]
    const double* nH2;                   // [nc]
    const double* Tkin;                  // [nc]
    const double* q;                     // [nc] dv / (b sqrt(pi) W); < 0: cell not solved
    const double2* acc;                  // [nc][ntr]
    unsigned long long* delta_bits;      // max relative change (as double bits)
    unsigned int* bad;                   // numeric-failure counter
};

// One resident model of the 1D request loop (device table entry).  All
// pointers point into the server's device arena.
struct ServeModel {
    March1DArgs<float> m;                // march of all transitions, FP32, LDS accumulators
    const MolDev* mol;
    const double* nmolLb;
    float2* ke_w;                        // = m.ke (writable)
    double2* acc_w;                      // = m.acc
    double* x;                           // populations [nc][L]
    double* xn;                          // solve output
    const double* nH2;
    const double* Tk;
    const double* q;
    unsigned long long* delta_bits;      // this model's max relative change of the tick
    unsigned int* bad;
    const double* ibg64;                 // background per transition (spectra: march I - I_bg)
    float* spec;                         // centre spectra [T][nch] (occupation units, I - I_bg)
    const float* zero;                   // T zeros
    int nc, L, T, mode;                  // mode 0: iterate, 1: final spectra this tick
};

// Device work lists of one tick.
struct ServeTables {
    const ServeModel* models;
    const int4* march_items;             // (model, transition, first ray, 1 = centre spectrum)
    const int* n_march;
    const int2* cell_items;              // (model, first cell), 256 cells each
    const int* n_cell;
    const int2* se_items;                // (model, first cell), se_bs cells each
    const int* n_se;
};

struct ServeGrid {
    int march_blocks, cell_blocks, se_blocks, se_bs;
    int march_lds, se_lds;
};

// Octree ray schedules.  Step record: word 0 = cell | flags, word 1 = the
// step length (root-cell units) as float bits.
constexpr uint32_t kOctCellMask = 0x0FFFFFFFu;
constexpr uint32_t kOctSave = 1u << 28;        // push the incoming intensity before the step
constexpr int kOctModeShift = 29;              // how the intensity starts at this step:
constexpr uint32_t kOctModeKeep = 0;           //   continue
constexpr uint32_t kOctModeBg = 1;             //   background (ray start or side re-entry)
constexpr uint32_t kOctModePeek = 2;           //   copy of the top saved vector
constexpr uint32_t kOctModePop = 3;            //   copy of the top saved vector, then drop it

// Per-cell sums of the octree march's per-step partial sums.
template <typename T>
struct GatherOctArgs {
    long long nc;
    int ntr, trans_offset, ntr_total;
    const long long* cell_off;           // [nc + 1]
    const unsigned* cell_steps;          // step indices grouped by cell, ascending
    const unsigned* dir_off;             // [n_dir + 1]: first step of each direction (steps are direction-major)
    int n_dir;
    const typename V2<T>::type* E;       // [step][estride]
    int estride;                         // row stride of E (>= ntr; even for FP32: 16-byte rows)
    double2* acc;                        // [nc][ntr_total]
};

// One work unit: every ray one root line gives rise to, in processing order.
struct OctTreeRec {
    int64_t off;     // first step record
    int32_t n;       // records
    int32_t q;       // direction
    int32_t r;       // root element (j N + i) on the upstream face
    int32_t depth;   // saved vectors alive at most
};

template <typename T>
struct OctMarchArgs {
    int nc, nch, ich;                    // cells, channels, stride of a channel vector (oct_stride)
    int ntr, trans_offset, ntr_total;    // transitions of this launch / in ke and acc
    long long n_items;                   // trees x ntr (transitions vary fastest)
    const OctTreeRec* trees;
    const uint2* steps;
    const double* len64;                 // FP64 step lengths (FP64 march), else null
    const double* aw;                    // |d_m| per direction
    const typename V4<T>::type* win;     // [n_dir][nc]
    const typename V2<T>::type* ke;      // [nc][ntr_total]
    const T* Ibg;                        // [ntr_total]
    typename V2<T>::type* E;             // per-step sums [step][estride] of this launch (with accumulation)
    int estride;                         // row stride of E (>= ntr; even for FP32: 16-byte rows)
    T* Iout;                             // no accumulation: [trees][nch] leaving intensity
    unsigned long long* counter;         // work counter, zero at launch
    T* stack;                            // [groups][depth][ich] saved vectors
    int depth;
    const typename V2<T>::type* hf;      // hyperfine components as in March3DArgs, or null
    int hfk;
    unsigned* maser;                     // as in March3DArgs
};

// Stride (elements) of an octree march channel vector, in LDS and in the
// saved-vector stacks: whole 16-byte units plus 64 bytes, so that vectors
// copy in 16-byte pieces and the lane groups of a wavefront start in
// different LDS banks.
inline int oct_stride(int nch, int elem_bytes)
{
    const int per = 16 / elem_bytes;
    return (nch + per - 1) / per * per + 64 / elem_bytes;
}

// Kernel launchers (kernels.hip).  All return hipError_t of the launch.
hipError_t launch_serve_tick(hipStream_t s, const ServeTables& tb, const ServeGrid& g);
hipError_t serve_set_attributes(const ServeGrid& g);
hipError_t launch_prepare(hipStream_t s, int nc, const MolDev* mol, int ntr, const double* x,
                          const double* nmolLb, const double* ibg_sub, void* ke, bool fp64);
hipError_t launch_lte(hipStream_t s, int nc, const MolDev* mol, const double* Tkin, double* x);
// Channel windows of every (direction, cell) of a regular grid.
hipError_t launch_window_table(hipStream_t s, int nc, int n_dir, const DirDev* dirs, const float4* vel,
                               const double* bD, double dv, double chalf, double K, int nch, double dlo,
                               double dhi, void* win,
                               bool fp64);
// max_steps: the longest step list of the launched directions (LDS staging).
// For every (direction, ray) of a.dirs: the lowest first channel of its
// steps' windows into rbase[q * rays_per_dir + r], and the largest span of a
// ray (its highest window start plus max(window, reach), minus the lowest)
// into *wmax with atomicMax (*wmax must start at 0).
hipError_t launch_ray_spans(hipStream_t s, const March3DArgs<float>& a, int reach, int* rbase, int* wmax);
// Channels the unrolled passes of one lane group of the FP32 march reach.
inline int march_pass_reach(int lanes) { return (lanes >= 64 ? 1 : (lanes >= 32 ? 2 : 4)) * lanes; }
hipError_t launch_march3d(hipStream_t s, const March3DArgs<float>& a, int lanes, bool accum,
                          int max_steps);
hipError_t launch_march3d(hipStream_t s, const March3DArgs<double>& a, int lanes, bool accum,
                          int max_steps);
// W_k = sum_j area_j * (path of ray j in shell k), normalised units; with
// bsq set, q_k = dv / (bsq_k W_k) is written instead of W_k.
hipError_t launch_shell_weights(hipStream_t s, int n, const double* R, int nrays, const double* b,
                                const double* area, double* W, const double* bsq = nullptr, double dv = 0.0);
// Step records of 1D rays (see ray_steps_kernel); R, b normalised to R_out,
// off[j] = first record of ray j, kmin[j] its innermost shell.
hipError_t launch_ray_steps(hipStream_t s, int n, const double* R, int nrays, const double* b, const int* kmin,
                            const long long* off, const double* vr_dv, void* out, bool fp64);
hipError_t launch_march1d(hipStream_t s, const March1DArgs<float>& a, int lanes, bool accum);
// All transitions of each ray in one pass (a wavefront per ray, four
// transitions per wavefront sharing the step's profile), with accumulation
// into acc by FP64 atomics; whole rays from I_bg only (seg = kSegWhole).
hipError_t launch_march1d_all_transitions(hipStream_t s, const March1DArgs<float>& a);
hipError_t launch_march1d_all_transitions(hipStream_t s, const March1DArgs<double>& a);
hipError_t launch_march1d(hipStream_t s, const March1DArgs<double>& a, int lanes, bool accum);
hipError_t launch_se(hipStream_t s, const SEArgs& a);
hipError_t launch_gather3d(hipStream_t s, const Gather3DArgs<float>& a);
hipError_t launch_gather3d(hipStream_t s, const Gather3DArgs<double>& a);
// groups: lane groups (8 or 16 lanes) of the persistent grid, a multiple of
// 256 / lanes; the work counter is cleared here.
hipError_t launch_march_oct(hipStream_t s, const OctMarchArgs<float>& a, int groups, bool accum, int lanes);
hipError_t launch_march_oct(hipStream_t s, const OctMarchArgs<double>& a, int groups, bool accum, int lanes);
hipError_t launch_gather_oct(hipStream_t s, const GatherOctArgs<float>& a);
hipError_t launch_gather_oct(hipStream_t s, const GatherOctArgs<double>& a);

}  // namespace miloc
