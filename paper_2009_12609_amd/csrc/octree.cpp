// octree.cpp -- host-side ray schedules through octree models (FP64 geometry).
//
// Sect. 2.2 of the paper lets the grid of rays follow the spatial
// discretisation.  For one direction the rays lie on nested lattices of
// lines parallel to it: working in axis coordinates flipped so that every
// direction component is >= 0 ("u"), the level-l lines pierce the upstream
// face u_m = 0 at o + i 2^-l root cells in both transverse axes, with
// o = 2^-(Lmax+1) (half a finest cell), so the level-l lattice contains every
// coarser one and the unrefined tree reproduces the regular grid's rays
// through cell centres.  A line is named by its finest-lattice indices; its
// level is the coarsest lattice holding it.
//
// The paper's rules, as traced here:
//   * a root line starts on every upstream surface element with the
//     background intensity;
//   * entering a leaf finer than its current level through the leaf's
//     upstream face, a ray starts, for each level in between, the three other
//     lines of that level crossing the same refined cell's upstream face, with
//     a copy of its intensity;
//   * the ray entering a leaf through its upstream face (the only line of the
//     leaf's level to do so) looks at the leaf's illuminated side faces: the
//     line of the leaf's level that enters through such a face is started
//     there if the neighbouring leaf is coarser than that line's level, with
//     the intensity the first ray had at the upstream face (background at the
//     model boundary, where the line comes from the opposite side);
//   * a ray is tagged with its line's level and ends on entering a leaf
//     coarser than the tag; otherwise it takes the leaf's level (the photon
//     count rescaling of the paper is the weight h_L^2 |d_m| in intensity
//     form);
//   * leaving through a side of the model a ray re-enters on the opposite
//     side at the same main-axis coordinate with the background intensity;
//     leaving through the downstream face it ends.
// Coinciding face crossings (within 1e-10 root cells) are ordered a-face,
// b-face, main-axis face: the lines behave as if shifted by an infinitesimal
// amount towards +a and a much smaller one towards +b.  Cells are half-open
// in u, and a point a crossing leaves exactly on a face of another axis is on
// the side that order puts it.  Per direction every leaf of level L then carries a total
// path of 2^-L / |d_m| over the lines of its level.
//
// The rays a root line gives rise to form one work unit (a "tree"); they are
// emitted depth first: the current ray runs to its end, then the most
// recently started pending ray.  Rays started at one point share one saved
// intensity vector; with this order the vector a starting ray needs is always
// the most recently saved one still in use, so the vectors form a stack and
// each record only says whether to push, peek or pop.
#include "octree.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "geometry.h"

namespace miloc {

std::string octree_from_levels(int N, int n_levels, const int64_t* n_cells_per_level,
                               const int32_t* const* first_child, OctModel& out)
{
    if (N < 1 || n_levels < 1 || n_levels > 12) return "octree: need N >= 1 and 1..12 levels";
    if (!n_cells_per_level) return "octree: NULL n_cells_per_level";
    if (n_cells_per_level[0] != (int64_t)N * N * N) return "octree: level 0 must hold N^3 cells";
    out.N = N;
    out.Lmax = n_levels - 1;
    out.level_start.assign(n_levels + 1, 0);
    for (int l = 0; l < n_levels; ++l) {
        if (n_cells_per_level[l] < 0) return "octree: negative cell count";
        out.level_start[l + 1] = out.level_start[l] + n_cells_per_level[l];
    }
    const int64_t total = out.level_start[n_levels];
    if (total > (int64_t)kOctCellMask) return "octree: too many cells (at most 2^28 - 1)";
    out.child.assign(total, -1);
    out.level.assign(total, 0);
    for (int l = 0; l < n_levels; ++l) {
        for (int64_t i = out.level_start[l]; i < out.level_start[l + 1]; ++i) out.level[i] = (int8_t)l;
        if (l == n_levels - 1) {
            if (n_cells_per_level[l] > 0 && first_child && first_child[l]) {
                for (int64_t i = 0; i < n_cells_per_level[l]; ++i)
                    if (first_child[l][i] >= 0) return "octree: cells of the last level cannot be refined";
            }
            break;
        }
        if (!first_child || !first_child[l]) return "octree: NULL first_child table";
        const int64_t nnext = n_cells_per_level[l + 1];
        if (nnext % 8 != 0) return "octree: a refined level must hold a multiple of 8 cells";
        std::vector<char> claimed(nnext / 8, 0);
        int64_t refined = 0;
        for (int64_t i = 0; i < n_cells_per_level[l]; ++i) {
            const int32_t fc = first_child[l][i];
            if (fc < 0) continue;
            if (fc % 8 != 0 || (int64_t)fc + 8 > nnext) return "octree: child block outside the next level";
            if (claimed[fc / 8]) return "octree: child block claimed twice";
            claimed[fc / 8] = 1;
            ++refined;
            out.child[out.level_start[l] + i] = (int32_t)(out.level_start[l + 1] + fc);
        }
        if (refined * 8 != nnext) return "octree: unclaimed cells in a level";
    }
    return std::string();
}

namespace {

constexpr double kTieTol = 1e-10;

// true if crossing (t1, axis r1) comes before crossing (t2, axis r2)
inline bool earlier(double t1, int r1, double t2, int r2)
{
    if (t1 < t2 - kTieTol) return true;
    if (t1 > t2 + kTieTol) return false;
    return r1 < r2;
}

struct Pending {
    int64_t line[2];       // finest-lattice indices (a, b) of the line
    int64_t cell[3];       // finest u-indices of the first cell (a, b, m)
    double t;              // path length at the start
    int entered;           // axis crossed to reach the first cell (2 = main axis)
    int tag, lev;
    int src;               // saved vector (stack position) or -1 for background
};

class DirTracer {
public:
    DirTracer(const OctModel& M, const double* d) : M_(M)
    {
        P_ = (int64_t)M.N << M.Lmax;
        h_ = std::ldexp(1.0, -M.Lmax);
        const int m = main_axis(d);
        ax_[2] = m;
        ax_[0] = m == 0 ? 1 : 0;
        ax_[1] = m == 2 ? 1 : 2;
        for (int s = 0; s < 3; ++s) neg_[s] = d[s] < 0.0;
        for (int u = 0; u < 3; ++u) du_[u] = std::fabs(d[ax_[u]]);
    }

    int32_t leaf(const int64_t* f, int& lev) const
    {
        int64_t s[3];
        for (int u = 0; u < 3; ++u) {
            const int a = ax_[u];
            s[a] = neg_[a] ? P_ - 1 - f[u] : f[u];
        }
        const int L = M_.Lmax;
        int64_t g = ((s[2] >> L) * M_.N + (s[1] >> L)) * M_.N + (s[0] >> L);
        int l = 0;
        while (M_.child[g] >= 0) {
            ++l;
            const int sh = L - l;
            g = M_.child[g] + ((s[0] >> sh) & 1) + 2 * ((s[1] >> sh) & 1) + 4 * ((s[2] >> sh) & 1);
        }
        lev = l;
        return (int32_t)g;
    }

    int line_level(int64_t la, int64_t lb) const
    {
        auto tz = [&](int64_t v) {
            v = ((v % P_) + P_) % P_;
            if (v == 0) return M_.Lmax;
            int z = 0;
            while (z < M_.Lmax && !(v & 1)) { v >>= 1; ++z; }
            return z;
        };
        return M_.Lmax - std::min(tz(la), tz(lb));
    }

    // transverse coordinate (root units) of a line at path length t
    double coord(int u, int64_t line, double t) const { return ((double)line + 0.5) * h_ + t * du_[u]; }

    // All rays of root element (i, j): appends step records to rec.  False if
    // the saved vectors do not follow stack order (not expected).
    bool tree(int i, int j, OctRays rays, std::vector<uint32_t>& rec, std::vector<double>* len64, int& max_depth,
              int64_t& n_rays);

private:
    const OctModel& M_;
    int64_t P_;
    double h_;
    int ax_[3];
    bool neg_[3];
    double du_[3];
};

inline int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Finest index along axis u of a point at coordinate pos (root units) that
// the crossing of axis 'by' has reached: on a face of axis u it lies below
// the face when that face's crossing comes later in the order a, b, m.
inline int64_t index_after(double pos, double h, int u, int by)
{
    const double x = pos / h;
    const double k = std::nearbyint(x);
    if (std::fabs(x - k) <= kTieTol / h) return (int64_t)k - (u > by ? 1 : 0);
    return (int64_t)std::floor(x);
}

bool DirTracer::tree(int i, int j, OctRays rays, std::vector<uint32_t>& rec, std::vector<double>* len64,
                     int& max_depth, int64_t& n_rays)
{
    const int L = M_.Lmax;
    const double dm = du_[2];
    const bool plain = rays != OctRays::Scheme;
    std::vector<Pending> todo;
    std::vector<int> users;          // rays still to start from each saved vector
    // the root line, or with the lattice all 4^L lines of the element (taken
    // from the back: the first line first)
    const int64_t nl = rays == OctRays::Lattice ? (int64_t)1 << L : 1;
    for (int64_t b = nl - 1; b >= 0; --b)
        for (int64_t a = nl - 1; a >= 0; --a) {
            Pending root;
            root.line[0] = ((int64_t)i << L) + a;
            root.line[1] = ((int64_t)j << L) + b;
            root.cell[0] = root.line[0];
            root.cell[1] = root.line[1];
            root.cell[2] = 0;
            root.t = 0.0;
            root.entered = 2;
            root.tag = 0;
            root.lev = 0;
            root.src = -1;
            todo.push_back(root);
        }
    while (!todo.empty()) {
        Pending R = todo.back();
        todo.pop_back();
        ++n_rays;
        uint32_t mode;
        if (R.src < 0) {
            mode = kOctModeBg;
        } else {
            // the vector of this ray is the top of the stack (see above)
            if (R.src != (int)users.size() - 1) return false;
            if (--users[R.src] == 0) {
                mode = kOctModePop;
                users.pop_back();
            } else {
                mode = kOctModePeek;
            }
        }
        for (;;) {
            int lev;
            const int32_t g = leaf(R.cell, lev);
            if (!plain && lev < R.tag) break;                 // coarser than the ray's tag: it ends
            const int64_t size = (int64_t)1 << (L - lev);
            const double side = (double)size * h_;
            int64_t lo[3];
            for (int u = 0; u < 3; ++u) lo[u] = R.cell[u] - R.cell[u] % size;
            uint32_t save = 0;
            if (!plain && R.entered == 2) {
                int saved = -1;
                auto vector_for_new_ray = [&]() {
                    if (saved < 0) {
                        users.push_back(0);
                        saved = (int)users.size() - 1;
                        save = kOctSave;
                        max_depth = std::max(max_depth, (int)users.size());
                    }
                    ++users[saved];
                    return saved;
                };
                std::vector<Pending> born;
                // upstream face of a refined cell: the other lines of each finer level
                for (int l = R.lev + 1; l <= lev; ++l) {
                    const int sh = L - l;
                    const int64_t step = (int64_t)1 << sh;
                    const int64_t qa = (R.cell[0] >> sh) & 1, qb = (R.cell[1] >> sh) & 1;
                    for (int64_t na = 0; na < 2; ++na)
                        for (int64_t nb = 0; nb < 2; ++nb) {
                            if (na == qa && nb == qb) continue;
                            Pending c = R;
                            c.line[0] += (na - qa) * step;
                            c.line[1] += (nb - qb) * step;
                            c.cell[0] += (na - qa) * step;
                            c.cell[1] += (nb - qb) * step;
                            c.entered = 2;
                            c.tag = l;
                            c.lev = l;
                            c.src = 0;
                            born.push_back(c);
                        }
                }
                // side faces: where the owner line would leave through the far
                // face of the leaf (on the leaf's own lattice period), the line one
                // period behind enters through the near face
                const double t_out_m = (double)(lo[2] + size) * h_ / dm;
                double t_wrap[2] = {INFINITY, INFINITY};
                for (int x = 0; x < 2; ++x)
                    if (du_[x] > 0.0) t_wrap[x] = R.t + (side - (coord(x, R.line[x], R.t) - (double)lo[x] * h_)) / du_[x];
                for (int x = 0; x < 2; ++x) {
                    if (!(du_[x] > 0.0) || !earlier(t_wrap[x], x, t_out_m, 2)) continue;
                    const int y = 1 - x;
                    int64_t nl[2];
                    nl[x] = R.line[x] - size;
                    nl[y] = R.line[y] - ((du_[y] > 0.0 && earlier(t_wrap[y], y, t_wrap[x], x)) ? size : 0);
                    const int nlev = line_level(nl[0], nl[1]);
                    const bool at_boundary = lo[x] == 0;
                    int64_t nb[3];
                    nb[x] = at_boundary ? P_ - 1 : lo[x] - 1;
                    nb[y] = lo[y];
                    nb[2] = lo[2];
                    int nblev;
                    (void)leaf(nb, nblev);
                    if (nblev >= lev || nblev >= nlev) continue;   // the line already arrives
                    Pending c;
                    c.line[0] = nl[0];
                    c.line[1] = nl[1];
                    c.t = t_wrap[x];
                    c.cell[x] = lo[x];
                    c.cell[y] = clamp64(index_after(coord(y, nl[y], c.t), h_, y, x), lo[y], lo[y] + size - 1);
                    c.cell[2] = clamp64(index_after(c.t * dm, h_, 2, x), lo[2], lo[2] + size - 1);
                    c.entered = x;
                    c.tag = nlev;
                    c.lev = lev;
                    c.src = at_boundary ? -2 : 0;
                    born.push_back(c);
                }
                for (Pending& c : born) {
                    if (c.src == -2) c.src = -1;
                    else c.src = vector_for_new_ray();
                    todo.push_back(c);
                }
            }
            R.lev = lev;
            // the step through this leaf
            double te[3];
            for (int x = 0; x < 2; ++x)
                te[x] = du_[x] > 0.0 ? ((double)(lo[x] + size) * h_ - ((double)R.line[x] + 0.5) * h_) / du_[x]
                                     : INFINITY;
            te[2] = (double)(lo[2] + size) * h_ / dm;
            int ex = 0;
            for (int u = 1; u < 3; ++u)
                if (earlier(te[u], u, te[ex], ex)) ex = u;
            const double s = std::max(0.0, te[ex] - R.t);
            const float sf = (float)s;
            uint32_t bits;
            std::memcpy(&bits, &sf, 4);
            rec.push_back((uint32_t)g | save | (mode << kOctModeShift));
            rec.push_back(bits);
            if (len64) len64->push_back(s);
            mode = kOctModeKeep;
            R.t = te[ex];
            for (int u = 0; u < 3; ++u) {
                if (u == ex) continue;
                const double pu = u == 2 ? R.t * dm : coord(u, R.line[u], R.t);
                R.cell[u] = clamp64(index_after(pu, h_, u, ex), lo[u], lo[u] + size - 1);
            }
            R.cell[ex] = lo[ex] + size;
            R.entered = ex;
            if (ex == 2) {
                if (R.cell[2] >= P_) break;                    // downstream face
            } else if (R.cell[ex] >= P_) {                     // model side: re-enter opposite
                R.cell[ex] -= P_;
                R.line[ex] -= P_;
                mode = kOctModeBg;
            }
        }
    }
    return users.empty();
}

}  // namespace

std::string octree_schedule(const OctModel& M, const std::vector<double>& dirs, OctRays rays, int n_threads,
                            OctSchedule& out, bool want_len64, int64_t n_cells)
{
    const int nd = (int)dirs.size() / 3;
    const int N = M.N;
    const int64_t nroot = (int64_t)N * N;
    if (rays == OctRays::Lattice) {
        // refuse before building what would not fit: a line of the finest
        // lattice takes at most 3 N 2^Lmax steps (one per finest cell along
        // each axis), 8 bytes each, and there are (N 2^Lmax)^2 per direction
        const double side = std::ldexp((double)N, M.Lmax);
        const double bound = (double)nd * side * side * 3.0 * side;
        if (bound > 4.0e9)
            return "octree: the brute-force lattice of this tree may take up to " + std::to_string(bound) +
                   " steps (limit 4e9); use the octree scheme";
    }
    struct Part {
        std::vector<uint32_t> rec;
        std::vector<double> len64;
        std::vector<OctTreeRec> trees;
        int max_depth = 0;
        int64_t n_rays = 0;
        bool ok = true;
    };
    std::vector<Part> parts(nd);
    const int nt = std::max(1, std::min(n_threads, nd));
    std::vector<std::thread> pool;
    for (int w = 0; w < nt; ++w)
        pool.emplace_back([&, w]() {
            for (int q = w; q < nd; q += nt) {
                Part& P = parts[q];
                DirTracer tr(M, &dirs[3 * (size_t)q]);
                P.trees.resize(nroot);
                for (int64_t r = 0; r < nroot; ++r) {
                    const int64_t off = (int64_t)P.rec.size() / 2;
                    int depth = 0;
                    if (!tr.tree((int)(r % N), (int)(r / N), rays, P.rec, want_len64 ? &P.len64 : nullptr, depth,
                                 P.n_rays))
                        P.ok = false;
                    OctTreeRec& T = P.trees[r];
                    T.off = off;
                    T.n = (int32_t)((int64_t)P.rec.size() / 2 - off);
                    T.q = q;
                    T.r = (int32_t)r;
                    T.depth = depth;
                    P.max_depth = std::max(P.max_depth, depth);
                }
            }
        });
    for (auto& t : pool) t.join();
    int64_t total = 0;
    for (const Part& P : parts) {
        if (!P.ok) return "octree: saved intensity vectors out of stack order";
        total += (int64_t)P.rec.size() / 2;
    }
    if (total > (int64_t)INT32_MAX * 64) return "octree: schedule too long";
    // the directions' records go to their offsets in one array, the parts
    // copied in parallel (the copy is gigabytes)
    out.dir_off.assign(nd, 0);
    {
        int64_t base = 0;
        for (int q = 0; q < nd; ++q) {
            out.dir_off[q] = base;
            base += (int64_t)parts[q].rec.size() / 2;
        }
    }
    out.rec.alloc(2 * (size_t)total);
    {
        std::vector<std::thread> cp;
        const int nc = std::max(1, std::min(n_threads, nd));
        for (int w = 0; w < nc; ++w)
            cp.emplace_back([&, w]() {
                for (int q = w; q < nd; q += nc) {
                    Part& P = parts[q];
                    if (!P.rec.empty())
                        std::memcpy(out.rec.data() + 2 * (size_t)out.dir_off[q], P.rec.data(),
                                    P.rec.size() * sizeof(uint32_t));
                    std::vector<uint32_t>().swap(P.rec);
                }
            });
        for (auto& t : cp) t.join();
    }
    out.len64.clear();
    if (want_len64) out.len64.reserve((size_t)total);
    out.trees.clear();
    out.trees.reserve((size_t)nd * nroot);
    out.max_depth = 0;
    out.n_rays = 0;
    for (int q = 0; q < nd; ++q) {
        Part& P = parts[q];
        const int64_t base = out.dir_off[q];
        out.len64.insert(out.len64.end(), P.len64.begin(), P.len64.end());
        std::vector<double>().swap(P.len64);
        for (OctTreeRec T : P.trees) {
            T.off += base;
            out.trees.push_back(T);
        }
        out.max_depth = std::max(out.max_depth, P.max_depth);
        out.n_rays += P.n_rays;
    }
    out.n_steps = total;
    out.dir_off.push_back(total);
    std::stable_sort(out.trees.begin(), out.trees.end(),
                     [](const OctTreeRec& a, const OctTreeRec& b) { return a.n > b.n; });
    out.cell_off.clear();
    out.cell_steps.clear();
    if (n_cells > 0) {
        if (total > (int64_t)UINT32_MAX) return "octree: more than 2^32 steps";
        // stable counting sort of the steps by cell: every thread counts the
        // cells of its own contiguous range of steps, a cell's entries are
        // laid out thread by thread, and each thread then places its steps in
        // order, so a cell's list keeps the schedule's step order (and the
        // per-cell sums their summation order from run to run)
        const int nf = std::max(1, std::min(n_threads, 16));
        std::vector<uint32_t> cnt((size_t)nf * (size_t)n_cells, 0u);
        auto range = [&](int w, int64_t& a, int64_t& b) {
            a = total * w / nf;
            b = total * (w + 1) / nf;
        };
        auto parallel = [&](auto&& fn) {
            std::vector<std::thread> th;
            for (int w = 0; w < nf; ++w) th.emplace_back(fn, w);
            for (auto& t : th) t.join();
        };
        parallel([&](int w) {
            int64_t a, b;
            range(w, a, b);
            uint32_t* cw = cnt.data() + (size_t)w * n_cells;
            for (int64_t i = a; i < b; ++i) ++cw[out.rec[2 * i] & kOctCellMask];
        });
        std::vector<int64_t>& off = out.cell_off;
        off.assign(n_cells + 1, 0);
        parallel([&](int w) {
            for (int64_t k = n_cells * w / nf; k < n_cells * (w + 1) / nf; ++k) {
                int64_t n = 0;
                for (int v = 0; v < nf; ++v) n += cnt[(size_t)v * n_cells + k];
                off[k + 1] = n;
            }
        });
        for (int64_t k = 0; k < n_cells; ++k) off[k + 1] += off[k];
        // per thread and cell, the first entry of that thread's steps in the cell
        parallel([&](int w) {
            for (int64_t k = n_cells * w / nf; k < n_cells * (w + 1) / nf; ++k) {
                int64_t run = off[k];
                for (int v = 0; v < nf; ++v) {
                    uint32_t& c = cnt[(size_t)v * n_cells + k];
                    const uint32_t n = c;
                    c = (uint32_t)run;
                    run += n;
                }
            }
        });
        out.cell_steps.resize(total);
        parallel([&](int w) {
            int64_t a, b;
            range(w, a, b);
            uint32_t* cw = cnt.data() + (size_t)w * n_cells;
            for (int64_t i = a; i < b; ++i) out.cell_steps[cw[out.rec[2 * i] & kOctCellMask]++] = (uint32_t)i;
        });
    }
    return std::string();
}

}  // namespace miloc
