// geometry.h -- host-side ray geometry (see geometry.cpp).
#pragma once

#include <stdint.h>

#include <vector>

namespace miloc {

// 12*nside^2 unit vectors (x, y, z interleaved), HEALPix RING order.
std::vector<double> healpix_directions(int nside);

// Axis (0, 1, 2) of the largest |component|; near-ties -> lowest index.
int main_axis(const double* d);

// Step list of the representative ray of one regular-grid direction.
struct DirPattern {
    int m = 2, a = 0, b = 1;          // main and transverse axes (a < b)
    double aw = 1.0;                  // |d_m|
    std::vector<double> len;          // step lengths (cell units)
    std::vector<int> flags;           // moves before each step: 1 m, 2 a, 4 b
    std::vector<double> layer_len;    // path length per layer (from the upstream face)
    std::vector<int> layer_start;     // first step of each layer, N+1 entries
    std::vector<int> na, nb;          // moves along a / b made up to and including each step
};
DirPattern regular_pattern(const double* d, int N);

// Innermost shell (first k with R[k] > b, R[n-1] = 1) and first step record
// of each 1D ray; each ray has 2 (n - 1 - kmin) + 2 steps.  Returns the total.
int64_t shell_ray_layout(int n, const double* R, int nrays, const double* b, std::vector<int64_t>& off,
                         std::vector<int>& kmin);

}  // namespace miloc
