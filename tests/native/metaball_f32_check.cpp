// Host check of the FP32 first decision of C(x) >= L used by the flagging and
// the link-fraction bracket: r = x - X and p - X rounded to FP32 (X the
// anchor), d = r - p, terms k * rcp(|d|^2) summed with fma, the reciprocal
// taken as the correctly rounded one moved by up to one ulp either way (the
// hardware's bound); the decision is made only when every |d|^2 >= 1 and the
// FP32 sum clears L by rel = 1.5 u (2.03 (|r|_1 + bp) + 9.5 + n) plus 1e-12
// (u = 2^-24, bp = max |p - X|_1).  Over random bodies of 1..20 control
// points far from the origin, at points near the surface (relative offsets
// down to 1e-8), deep inside, near control points and far out, every decision
// taken must equal the exact one (C in exact FP64 quotients, summed in
// order), and at lattice points (what the flagging evaluates) at least 95 %
// must be decided in FP32.  The same in periodic boxes for bodies near a
// face (the minimum image of x - X taken once, the exact sum's per point).  Prints the counts and exits 1 on any
// disagreement.
#include <cmath>
#include <cstdio>
#include <random>

static float rcp_hw(float x, std::mt19937_64 &rng) {
    float r = 1.0f / x;
    const int m = (int)(rng() % 3) - 1;  // -1, 0, +1 ulp
    if (m < 0) r = std::nextafter(r, 0.0f);
    if (m > 0) r = std::nextafter(r, INFINITY);
    return r;
}

int main() {
    std::mt19937_64 rng(20250);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    long decided = 0, undecided = 0, wrong = 0, lattice = 0, lattice_decided = 0;
    for (int body = 0; body < 6000; ++body) {
        const int n = 1 + (int)(U(rng) * 20);
        const int n4 = (n + 3) & ~3;
        const double R = 4.0 + 10.0 * U(rng);
        double cp[24][3], k[24], ksum = 0.0, X[3] = {0, 0, 0};
        const double base[3] = {256.0 * U(rng), 256.0 * U(rng), 640.0 * U(rng)};
        for (int i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) cp[i][a] = base[a] + 0.8 * R * (U(rng) - 0.5);
            k[i] = 20.0 + 40.0 * U(rng);
            ksum += k[i];
        }
        for (int i = 0; i < n; ++i) k[i] *= R * R / ksum;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) X[a] += cp[i][a] / n;
        const double L = U(rng) < 0.5 ? 1.0 : 0.5 + 0.5 * U(rng);  // 1, or a level c_0 < 1
        // FP32 staging (padding: weight 0 copies of point 0)
        float f[24][4], bp = 0.f;
        for (int i = 0; i < n4; ++i) {
            const int s = i < n ? i : 0;
            for (int a = 0; a < 3; ++a) f[i][a] = (float)(cp[s][a] - X[a]);
            f[i][3] = i < n ? (float)k[i] : 0.f;
            bp = std::fmax(bp, std::fabs(f[i][0]) + std::fabs(f[i][1]) + std::fabs(f[i][2]));
        }
        bp *= 1.f + 1e-6f;
        auto exact = [&](const double x[3]) -> double {
            double C = 0.0;
            for (int i = 0; i < n; ++i) {
                const double d0 = x[0] - cp[i][0], d1 = x[1] - cp[i][1], d2 = x[2] - cp[i][2];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                if (r2 == 0.0) return INFINITY;
                C += k[i] / r2;
            }
            return C;
        };
        // 1: >= L, 0: < L, -1: not decided
        auto f32 = [&](const double x[3]) {
            const float rx = (float)(x[0] - X[0]), ry = (float)(x[1] - X[1]), rz = (float)(x[2] - X[2]);
            float C = 0.f, rmin = 1.f;
            for (int i = 0; i < n4; ++i) {
                const float dx = rx - f[i][0], dy = ry - f[i][1], dz = rz - f[i][2];
                const float r2 = std::fma(dx, dx, std::fma(dy, dy, dz * dz));
                rmin = std::fmin(rmin, r2);
                C = std::fma(f[i][3], rcp_hw(r2, rng), C);
            }
            if (!(rmin >= 1.f)) return -1;
            const float ax = std::fabs(rx) + std::fabs(ry) + std::fabs(rz);
            const double rel = 1.5 * 5.9604644775390625e-8 * (2.03 * ((double)ax + (double)bp) + 9.5 + n4);
            const double Cd = (double)C;
            if (Cd * (1.0 - rel) > L * (1.0 + 1e-12)) return 1;
            if (Cd * (1.0 + rel) < L * (1.0 - 1e-12)) return 0;
            return -1;
        };
        auto check = [&](const double x[3]) {
            const int d = f32(x);
            if (d < 0) { ++undecided; return; }
            ++decided;
            const int e = exact(x) >= L ? 1 : 0;
            if (d != e) {
                ++wrong;
                std::printf("disagreement: body %d n %d x %.17g %.17g %.17g C %.17g L %g\n", body, n, x[0], x[1],
                            x[2], exact(x), L);
            }
        };
        for (int ray = 0; ray < 6; ++ray) {
            double dir[3], nrm = 0.0;
            for (int a = 0; a < 3; ++a) { dir[a] = U(rng) - 0.5; nrm += dir[a] * dir[a]; }
            nrm = std::sqrt(nrm);
            double lo = 0.0, hi = 4.0 * R;
            for (int it = 0; it < 90; ++it) {
                const double mid = 0.5 * (lo + hi);
                double x[3];
                for (int a = 0; a < 3; ++a) x[a] = X[a] + mid * dir[a] / nrm;
                if (exact(x) >= L) lo = mid; else hi = mid;
            }
            for (int j = 0; j < 40; ++j) {
                const double e = std::pow(10.0, -8.0 + 7.0 * U(rng)) * (U(rng) < 0.5 ? -1.0 : 1.0);
                double x[3];
                for (int a = 0; a < 3; ++a) x[a] = X[a] + lo * (1.0 + e) * dir[a] / nrm;
                check(x);
            }
        }
        for (int j = 0; j < 60; ++j) {  // anywhere in a ball of 2R, on lattice points, near control points
            double x[3];
            for (int a = 0; a < 3; ++a) x[a] = X[a] + 4.0 * R * (U(rng) - 0.5);
            check(x);
            for (int a = 0; a < 3; ++a) x[a] = std::floor(x[a]);
            const long before = decided;
            check(x);
            ++lattice;
            lattice_decided += decided - before;
            const int i = (int)(U(rng) * n);
            for (int a = 0; a < 3; ++a) x[a] = cp[i][a] + 2.0 * (U(rng) - 0.5);
            check(x);
        }
    }
    // Periodic boxes: bodies near a face, points on either side of it.  The
    // exact sum takes the minimum image of every x - p (floor(d / L + 0.5));
    // the FP32 form takes the minimum image of x - X once and uses r - (p - X)
    // where |r| + max |p - X|_1 < L/2 - 1 on every axis, else it leaves the
    // decision to FP64.
    long pdec = 0, pwrong = 0, pund = 0;
    for (int body = 0; body < 3000; ++body) {
        const int n = 1 + (int)(U(rng) * 20);
        const int n4 = (n + 3) & ~3;
        const double R = 4.0 + 10.0 * U(rng);
        const double Lb = 48.0 + 208.0 * U(rng);
        double cp[24][3], k[24], ksum = 0.0, X[3] = {0, 0, 0};
        double base[3];
        for (int a = 0; a < 3; ++a) base[a] = (U(rng) < 0.5 ? 0.3 * R * U(rng) : Lb - 0.3 * R * U(rng));
        for (int i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) cp[i][a] = base[a] + 0.8 * R * (U(rng) - 0.5);
            k[i] = 20.0 + 40.0 * U(rng);
            ksum += k[i];
        }
        for (int i = 0; i < n; ++i) k[i] *= R * R / ksum;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) X[a] += cp[i][a] / n;
        const double L = 1.0;
        float f[24][4], bp = 0.f;
        for (int i = 0; i < n4; ++i) {
            const int s = i < n ? i : 0;
            for (int a = 0; a < 3; ++a) f[i][a] = (float)(cp[s][a] - X[a]);
            f[i][3] = i < n ? (float)k[i] : 0.f;
            bp = std::fmax(bp, std::fabs(f[i][0]) + std::fabs(f[i][1]) + std::fabs(f[i][2]));
        }
        bp *= 1.f + 1e-6f;
        auto mi = [&](double d) { return d - Lb * std::floor(d / Lb + 0.5); };
        auto exact = [&](const double x[3]) -> double {
            double C = 0.0;
            for (int i = 0; i < n; ++i) {
                const double d0 = mi(x[0] - cp[i][0]), d1 = mi(x[1] - cp[i][1]), d2 = mi(x[2] - cp[i][2]);
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                if (r2 == 0.0) return INFINITY;
                C += k[i] / r2;
            }
            return C;
        };
        auto f32 = [&](const double x[3]) {
            double r[3] = {mi(x[0] - X[0]), mi(x[1] - X[1]), mi(x[2] - X[2])};
            for (int a = 0; a < 3; ++a)
                if (!(std::fabs(r[a]) + (double)bp < 0.5 * Lb - 1.0)) return -1;
            const float rx = (float)r[0], ry = (float)r[1], rz = (float)r[2];
            float C = 0.f, rmin = 1.f;
            for (int i = 0; i < n4; ++i) {
                const float dx = rx - f[i][0], dy = ry - f[i][1], dz = rz - f[i][2];
                const float r2 = std::fma(dx, dx, std::fma(dy, dy, dz * dz));
                rmin = std::fmin(rmin, r2);
                C = std::fma(f[i][3], rcp_hw(r2, rng), C);
            }
            if (!(rmin >= 1.f)) return -1;
            const float ax = std::fabs(rx) + std::fabs(ry) + std::fabs(rz);
            const double rel = 1.5 * 5.9604644775390625e-8 * (2.03 * ((double)ax + (double)bp) + 9.5 + n4);
            const double Cd = (double)C;
            if (Cd * (1.0 - rel) > L * (1.0 + 1e-12)) return 1;
            if (Cd * (1.0 + rel) < L * (1.0 - 1e-12)) return 0;
            return -1;
        };
        for (int j = 0; j < 300; ++j) {
            double x[3];
            for (int a = 0; a < 3; ++a) {
                double v = X[a] + 3.0 * R * (U(rng) - 0.5);
                v = v - Lb * std::floor(v / Lb);  // a point of the box
                x[a] = U(rng) < 0.5 ? std::floor(v) : v;
            }
            const int d = f32(x);
            if (d < 0) { ++pund; continue; }
            ++pdec;
            if (d != (exact(x) >= L ? 1 : 0)) ++pwrong;
        }
    }
    std::printf("periodic: decided %ld, undecided %ld, %ld disagreements\n", pdec, pund, pwrong);
    wrong += pwrong;
    std::printf("decided %ld, undecided %ld (to FP64), %ld disagreements; lattice points decided %ld of %ld\n",
                decided, undecided, wrong, lattice_decided, lattice);
    return wrong == 0 && lattice_decided >= 0.95 * lattice ? 0 : 1;
}
