// Host check of the division-free minimum image: for many axis lengths L,
// min_image_axis(d) must equal d - L floor(d / L + 0.5) bit for bit, at and
// around both thresholds, around +-L/2, at zero and at random d.  Prints the
// number of mismatches and exits 1 if any.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "../../paper_2209_10411_amd/csrc/min_image.h"

static bool same(double a, double b) { return std::memcmp(&a, &b, sizeof a) == 0; }

int main() {
    long bad = 0, checked = 0;
    std::mt19937_64 rng(12345);
    auto check = [&](double v, double L, double up, double dn) {
        const double want = v - L * std::floor(v / L + 0.5);
        const double got = mdl::min_image_axis(v, L, up, dn);
        ++checked;
        if (!same(want, got)) {
            if (bad < 10) std::printf("L=%g d=%.17g want %.17g got %.17g\n", L, v, want, got);
            ++bad;
        }
    };
    int lens[400];
    int nl = 0;
    for (int L = 3; L <= 300; ++L) lens[nl++] = L;
    for (int L : {333, 384, 500, 511, 512, 640, 1000, 1023, 1024, 1536, 4096, 10007, 65536}) lens[nl++] = L;
    for (int li = 0; li < nl; ++li) {
        const double L = lens[li];
        double up, dn;
        mdl::min_image_thresholds(lens[li], up, dn);
        for (double c : {up, dn, 0.5 * L, -0.5 * L, 0.0, -0.0, L, -L, 1.25 * L, -1.25 * L}) {
            double a = c, b = c;
            for (int k = 0; k < 6; ++k) {
                check(a, L, up, dn);
                check(b, L, up, dn);
                a = std::nextafter(a, 1e300);
                b = std::nextafter(b, -1e300);
            }
        }
        std::uniform_real_distribution<double> U(-1.3 * L, 1.3 * L);
        for (int r = 0; r < 20000; ++r) check(U(rng), L, up, dn);
        for (int r = 0; r < 2000; ++r) check(std::ldexp(U(rng), -40), L, up, dn);  // tiny |d|
    }
    std::printf("checked %ld values, %ld mismatches\n", checked, bad);
    return bad ? 1 : 0;
}
