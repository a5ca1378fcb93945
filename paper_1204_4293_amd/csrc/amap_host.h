// Host-side helpers of the library: the device workspace and the filter
// functions of Sec. 4 used to tabulate the direct aperture-mass sum.
#pragma once

#include <cmath>
#include <cstddef>
#include <vector>

#include "amap.h"

namespace amap {

// A growable device buffer.  Growth waits for the device, since work already
// enqueued may still read the old buffer.
struct Workspace {
    void* ptr = nullptr;
    size_t size = 0;
    amap_status reserve(size_t bytes);
    void release();
};

// Starlet tangential-shear filter Q(eta), eta = vartheta/theta, as printed
// in Sec. 4.2 of the paper (the shear-space form of eq:splinewl).  The
// printed 1/eta^2 factor is removable at eta = 0, where Q = 0.
inline double starlet_Q(double eta) {
    if (eta == 0.0) return 0.0;
    const double e = eta, e2 = e * e;
    auto c3 = [](double v) { v = std::fabs(v); return v * v * v; };
    const double num = -279.0 * e2 * c3(e)
                     + 8.0 * (1.0 + 6.0 * e + 24.0 * e2) * c3(0.5 - e)
                     - 9.0 * (1.0 + 3.0 * e + 6.0 * e2) * c3(1.0 - e)
                     - 9.0 * (1.0 - 3.0 * e + 6.0 * e2) * c3(1.0 + e)
                     + (1.0 + 1.5 * e + 1.5 * e2) * c3(2.0 - e)
                     + (1.0 - 1.5 * e + 1.5 * e2) * c3(2.0 + e)
                     + 8.0 * (1.0 - 6.0 * e + 24.0 * e2) * c3(0.5 + e);
    return num / (45.0 * e2);
}

// Schneider et al. (1998) polynomial filter, eq:sch (Heaviside: 1 at vt = theta).
inline double s98_Q(double vt, double theta, double ell) {
    if (vt > theta) return 0.0;
    const double x2 = (vt / theta) * (vt / theta);
    return (1.0 + ell) * (2.0 + ell) / (M_PI * theta * theta) * x2 * std::pow(1.0 - x2, ell);
}

// Gaussian-type filter of eq:mexhat with normalisation A = 1.
inline double jbj04_Q(double vt, double theta, double b) {
    const double x2 = b * (vt / theta) * (vt / theta);
    return x2 * std::exp(-x2) / (theta * theta);
}

// Taps of the direct sum: rows dy = -R..R, dense weights [(2R+1)^2] indexed
// [(dy+R)(2R+1) + dx+R]; half[dy+R] is the largest |dx| inside the cut on
// that row (-1 if none).  wc = Q cos 2phi, ws = Q sin 2phi.
struct TapTable {
    int R = 0;
    std::vector<int> half;
    std::vector<double> wc, ws;
};

}  // namespace amap
