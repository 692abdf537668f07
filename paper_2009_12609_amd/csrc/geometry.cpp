// geometry.cpp -- host-side ray geometry of the march (FP64).
//
//   * HEALPix RING pixel centres as ray directions (Sect. 2.2; Gorski et al. 2005)
//   * main direction = axis of the largest |component| (Sect. 2.2), components
//     equal within 1e-12 (relative) resolved to the lowest axis index
//   * crossing pattern of a regular-grid direction: the rays of one direction
//     start at the centres of the upstream surface cells and re-enter on the
//     opposite side after a side exit (Sect. 2.2), so in every layer all N*N
//     rays sit at the same fractional transverse offset and cross cell faces
//     in the same order.  One representative ray, traced analytically in FP64,
//     gives the step list every ray of the direction follows (translated).
//   * the step layout of 1D impact-parameter rays through shells (Sect. 2.1).
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace miloc {

std::vector<double> healpix_directions(int nside)
{
    std::vector<double> out;
    const double pi = 3.14159265358979323846;
    const int nring = 4 * nside - 1;
    for (int i = 1; i <= nring; ++i) {
        double z;
        int npix;
        double shift;      // phi_j = pi (j - shift) / (2 * ring_scale)
        int scale;
        if (i < nside) {
            z = 1.0 - (double)i * i / (3.0 * nside * nside);
            npix = 4 * i; shift = 0.5; scale = i;
        } else if (i <= 3 * nside) {
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside);
            npix = 4 * nside; shift = ((i - nside + 1) % 2) * 0.5; scale = nside;
        } else {
            const int ii = 4 * nside - i;
            z = -(1.0 - (double)ii * ii / (3.0 * nside * nside));
            npix = 4 * ii; shift = 0.5; scale = ii;
        }
        const double st = std::sqrt(std::max(0.0, 1.0 - z * z));
        for (int j = 1; j <= npix; ++j) {
            const double phi = pi * (j - shift) / (2.0 * scale);
            out.push_back(st * std::cos(phi));
            out.push_back(st * std::sin(phi));
            out.push_back(z);
        }
    }
    return out;
}

int main_axis(const double* d)
{
    const double ax[3] = {std::fabs(d[0]), std::fabs(d[1]), std::fabs(d[2])};
    const double mx = std::max(ax[0], std::max(ax[1], ax[2]));
    for (int i = 0; i < 3; ++i)
        if (ax[i] >= mx * (1.0 - 1e-12)) return i;
    return 2;
}

DirPattern regular_pattern(const double* d, int N)
{
    DirPattern P;
    P.m = main_axis(d);
    P.a = (P.m == 0) ? 1 : 0;
    P.b = (P.m == 2) ? 1 : 2;
    const double dm = std::fabs(d[P.m]), da = std::fabs(d[P.a]), db = std::fabs(d[P.b]);
    const double inf = std::numeric_limits<double>::infinity();
    P.layer_len.assign(N, 0.0);
    // Cumulative path parameter t (cell units) of the next face crossing of
    // each axis: the main axis crosses at n/|d_m|, the transverse axes (the
    // ray starts half a cell from their faces) at (n - 1/2)/|d|.
    long nm = 1, na = 1, nb = 1;
    double tprev = 0.0;
    int flags = 0;
    int layer = 0;
    const double tol = 1e-12;
    for (;;) {
        const double tm = (double)nm / dm;
        const double ta = da > 0 ? ((double)na - 0.5) / da : inf;
        const double tb = db > 0 ? ((double)nb - 0.5) / db : inf;
        const double tmin = std::min(tm, std::min(ta, tb));
        P.len.push_back(tmin - tprev);
        P.flags.push_back(flags);
        P.layer_len[layer] += tmin - tprev;
        int nf = 0;
        if (tm <= tmin + tol) {
            if (nm == N) break;            // downstream face: the ray ends
            nf |= 1;
            ++nm;
            ++layer;
        }
        if (ta <= tmin + tol) { nf |= 2; ++na; }
        if (tb <= tmin + tol) { nf |= 4; ++nb; }
        tprev = tmin;
        flags = nf;
    }
    P.aw = dm;
    // layer boundaries and cumulative transverse moves (used to find, for a
    // cell and a step, which ray of the direction was there)
    const int ns = (int)P.len.size();
    P.layer_start.assign(N + 1, ns);
    P.na.resize(ns);
    P.nb.resize(ns);
    int l = 0, ca = 0, cb = 0;
    P.layer_start[0] = 0;
    for (int s = 0; s < ns; ++s) {
        if (P.flags[s] & 1) P.layer_start[++l] = s;
        if (P.flags[s] & 2) ++ca;
        if (P.flags[s] & 4) ++cb;
        P.na[s] = ca;
        P.nb[s] = cb;
    }
    return P;
}

int64_t shell_ray_layout(int n, const double* R, int nrays, const double* b, std::vector<int64_t>& off,
                         std::vector<int>& kmin)
{
    off.resize(nrays);
    kmin.resize(nrays);
    int64_t total = 0;
    for (int j = 0; j < nrays; ++j) {
        const int km = std::min<int>(n - 1, (int)(std::upper_bound(R, R + n, b[j]) - R));
        kmin[j] = km;
        off[j] = total;
        total += 2 * (int64_t)(n - 1 - km) + 2;
    }
    return total;
}

}  // namespace miloc
