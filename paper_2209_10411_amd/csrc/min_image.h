// Minimum image on a periodic axis of length L without an FP64 division in
// the common case: the shift k(d) = floor(d / L + 0.5) is monotone in d, so
// for |d| < 1.25 L (where k is -1, 0 or 1) it is fixed by two thresholds,
// found once on the host by bisection over doubles with the same FP64
// operations.  The result is bit-identical to d - L k(d).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace mdl {

// up = the least d with k(d) >= 1, dn = the least d with k(d) >= 0.
inline void min_image_thresholds(int L, double &up, double &dn) {
    const double Ld = (double)L;
    auto k = [Ld](double d) { return std::floor(d / Ld + 0.5); };
    auto least = [&](double lo, double hi, double target) {  // k(lo) < target <= k(hi)
        for (;;) {
            const double mid = lo + (hi - lo) * 0.5;
            if (!(mid > lo && mid < hi)) return hi;
            if (k(mid) >= target) hi = mid;
            else lo = mid;
        }
    };
    up = least(0.0, Ld, 1.0);
    dn = least(-Ld, 0.0, 0.0);
}

__host__ __device__ inline double min_image_axis(double v, double L, double up, double dn) {
    if (fabs(v) < 1.25 * L) return v >= up ? v - L : (v < dn ? v + L : v);
    return v - L * floor(v / L + 0.5);
}

}  // namespace mdl
