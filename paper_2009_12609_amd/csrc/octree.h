// octree.h -- host-side octree ray schedules (see octree.cpp).
#pragma once

#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "miloc_internal.h"

namespace miloc {

// Host array of 32-bit words allocated without initialisation, for the
// schedule's step records (gigabytes, filled in parallel).
struct HostWords {
    std::unique_ptr<uint32_t[]> p;
    size_t n = 0;
    void alloc(size_t k)
    {
        p.reset(k ? new uint32_t[k] : nullptr);
        n = k;
    }
    uint32_t* data() { return p.get(); }
    const uint32_t* data() const { return p.get(); }
    size_t size() const { return n; }
    uint32_t operator[](size_t i) const { return p[i]; }
};

// An octree in global cell numbering: level-0 root cells (z N + y) N + x
// first, then each level in turn; child[g] is the global index of the first
// of the 8 children (offset cx + 2 cy + 4 cz) of cell g, -1 for a leaf.
struct OctModel {
    int N = 0;
    int Lmax = 0;
    std::vector<int32_t> child;
    std::vector<int8_t> level;
    std::vector<int64_t> level_start;   // first global index of each level (+ total)
};

// Builds the global numbering from per-level first-child tables and checks
// that every child block lies inside the next level and is claimed once.
// Returns an empty string on success, else the reason.
std::string octree_from_levels(int N, int n_levels, const int64_t* n_cells_per_level,
                               const int32_t* const* first_child, OctModel& out);

struct OctSchedule {
    HostWords rec;                    // 2 words per step
    std::vector<double> len64;        // FP64 step lengths (only when asked for)
    std::vector<int64_t> cell_off;    // per cell: first entry of its steps in cell_steps (+ total)
    std::vector<uint32_t> cell_steps; // step indices grouped by cell, ascending (only when asked for)
    std::vector<int64_t> dir_off;     // first step of each direction (+ total): steps are direction-major
    std::vector<OctTreeRec> trees;
    int max_depth = 0;
    int64_t n_steps = 0;
    int64_t n_rays = 0;
};

// Which rays a schedule holds: the octree scheme's created and terminated
// rays (Sect. 2.2), the root lines alone traced straight (lines of sight for
// maps), or the brute-force lattice of Sect. 2.2: every line of the finest
// lattice, 4^Lmax per root element, traced straight.
enum class OctRays { Scheme = 0, Plain = 1, Lattice = 2 };

// Ray schedule of every root element and direction.  Trees (one per root
// element: all of its rays in processing order) are ordered by decreasing
// length.  Uses up to n_threads host threads.
// want_len64 also keeps the FP64 step lengths (for the FP64 march).
// n_cells > 0 also lists, per cell, the steps that cross it (at most 2^32
// steps in all).
// Returns an empty string on success, else the reason.
std::string octree_schedule(const OctModel& M, const std::vector<double>& dirs, OctRays rays, int n_threads,
                            OctSchedule& out, bool want_len64 = false, int64_t n_cells = 0);

}  // namespace miloc
