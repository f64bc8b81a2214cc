// Host check of the bound behind the flag decision's fast path: a metaball
// sum whose terms use a reciprocal refined by two Newton steps from an
// estimate with relative error up to 2^-14 (worse than the hardware's) stays
// within 1e-13 C of the sum of exact quotients in index order, for bodies
// of 1..23 control points at points where C is near 1 (the decision falls
// back to the exact sum within 1e-12 of 1).  Prints the largest relative
// difference and exits 1 if it exceeds 1e-13.
#include <cmath>
#include <cstdio>
#include <random>

static double rcp_refined(double x, double rel_err) {
    double r = (1.0 / x) * (1.0 + rel_err);
    double e = std::fma(-x, r, 1.0);
    r = std::fma(e, r, r);
    e = std::fma(-x, r, 1.0);
    return std::fma(e, r, r);
}

int main() {
    std::mt19937_64 rng(2209);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double worst = 0.0;
    long evals = 0;
    for (int body = 0; body < 4000; ++body) {
        const int n = 1 + (int)(U(rng) * 23);
        double cp[23][3], k[23], ksum = 0.0;
        for (int i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) cp[i][a] = 100.0 + 6.0 * (U(rng) - 0.5);
            k[i] = 20.0 + 40.0 * U(rng);
            ksum += k[i];
        }
        for (int i = 0; i < n; ++i) k[i] *= 81.0 / ksum;  // sum k = R^2, R = 9
        auto exact = [&](const double x[3]) {
            double C = 0.0;
            for (int i = 0; i < n; ++i) {
                const double d0 = x[0] - cp[i][0], d1 = x[1] - cp[i][1], d2 = x[2] - cp[i][2];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                C += k[i] / r2;
            }
            return C;
        };
        auto fast = [&](const double x[3]) {
            double C = 0.0;
            for (int i = 0; i < n; ++i) {
                const double d0 = x[0] - cp[i][0], d1 = x[1] - cp[i][1], d2 = x[2] - cp[i][2];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const double rel = std::ldexp(2.0 * U(rng) - 1.0, -14);
                C += k[i] * rcp_refined(r2, rel);
            }
            return C;
        };
        for (int ray = 0; ray < 8; ++ray) {
            // a random direction from the mean control point: bisect to C = 1,
            // then sample around the surface
            double dir[3], nrm = 0.0;
            for (int a = 0; a < 3; ++a) { dir[a] = U(rng) - 0.5; nrm += dir[a] * dir[a]; }
            nrm = std::sqrt(nrm);
            double c0[3] = {0, 0, 0};
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < 3; ++a) c0[a] += cp[i][a] / n;
            double lo = 0.5, hi = 60.0;
            for (int it = 0; it < 80; ++it) {
                const double mid = 0.5 * (lo + hi);
                double x[3];
                for (int a = 0; a < 3; ++a) x[a] = c0[a] + mid * dir[a] / nrm;
                if (exact(x) >= 1.0) lo = mid; else hi = mid;
            }
            for (int j = 0; j < 16; ++j) {
                const double t = lo * (1.0 + 1e-3 * (2.0 * U(rng) - 1.0));
                double x[3];
                for (int a = 0; a < 3; ++a) x[a] = c0[a] + t * dir[a] / nrm;
                const double ce = exact(x), cf = fast(x);
                worst = std::fmax(worst, std::fabs(cf - ce) / ce);
                ++evals;
            }
        }
    }
    std::printf("evaluations %ld, largest relative difference %.3e\n", evals, worst);
    return worst < 1e-13 ? 0 : 1;
}
