// Shape descriptors of a metaball body (sec. 4): volume, surface area,
// principal dimensions and projected area on a grid, then sphericity,
// nominal and surface-equivalent diameters and the Corey shape factor.  C ABI
// in include/shape.h.  Grid points are formed without contraction (the same
// sums as written), the metaball in control-point order with exact
// quotients, so that the inside decisions are those of a plain evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/shape.h"

namespace {

constexpr int BLK = 256;
constexpr int MAXN = 64;

struct Body {
    double p[MAXN][3];
    double k[MAXN];
    int n;
};

// C(x) - 1 with exact quotients in control-point order (+inf on a control point).
__device__ double cm1(const Body &b, double x, double y, double z) {
#pragma clang fp contract(off)
    double c = 0.0;
    for (int j = 0; j < b.n; ++j) {
        const double dx = x - b.p[j][0], dy = y - b.p[j][1], dz = z - b.p[j][2];
        c += b.k[j] / ((dx * dx + dy * dy) + dz * dz);
    }
    return c - 1.0;
}

__device__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}
__device__ double block_min(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// Area of the zero surface of the linear interpolant in one tetrahedron.
__device__ double tet_area(const double P[4][3], const double g[4]) {
#pragma clang fp contract(off)
    int pos[4], neg[4], np = 0, nn = 0;
    for (int a = 0; a < 4; ++a) {
        if (g[a] >= 0.0) pos[np++] = a;
        else neg[nn++] = a;
    }
    if (np == 0 || nn == 0) return 0.0;
    auto cut = [&](int a, int b, double q[3]) {
        const double t = g[a] / (g[a] - g[b]);
        for (int c = 0; c < 3; ++c) q[c] = P[a][c] + t * (P[b][c] - P[a][c]);
    };
    auto tri = [](const double a[3], const double b[3], const double c[3]) {
        const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double x = u[1] * v[2] - u[2] * v[1], y = u[2] * v[0] - u[0] * v[2], z = u[0] * v[1] - u[1] * v[0];
        return 0.5 * sqrt((x * x + y * y) + z * z);
    };
    double q[4][3];
    if (np == 1 || np == 3) {
        const int lone = np == 1 ? pos[0] : neg[0];
        int o = 0;
        for (int a = 0; a < 4; ++a)
            if (a != lone) cut(lone, a, q[o++]);
        return tri(q[0], q[1], q[2]);
    }
    cut(pos[0], neg[0], q[0]);
    cut(pos[0], neg[1], q[1]);
    cut(pos[1], neg[1], q[2]);
    cut(pos[1], neg[0], q[3]);
    return tri(q[0], q[1], q[2]) + tri(q[0], q[2], q[3]);
}

struct Grid {
    double lo[3], h;
    int n[3];
};

__device__ __forceinline__ void centre(const Grid &G, long long t, double c[3], int idx[3]) {
#pragma clang fp contract(off)
    idx[0] = (int)(t % G.n[0]);
    const long long r = t / G.n[0];
    idx[1] = (int)(r % G.n[1]);
    idx[2] = (int)(r / G.n[1]);
    for (int a = 0; a < 3; ++a) c[a] = G.lo[a] + G.h * ((double)idx[a] + 0.5);
}

// Pass 1: inside count, first moments of the inside centres, surface area.
__global__ __launch_bounds__(BLK) void k_shape_grid(Body b, Grid G, long long cells, double *__restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    const long long t = blockIdx.x * (long long)BLK + threadIdx.x;
    double cnt = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, area = 0.0;
    if (t < cells) {
        double c[3];
        int idx[3];
        centre(G, t, c, idx);
        if (cm1(b, c[0], c[1], c[2]) >= 0.0) {
            cnt = 1.0;
            sx = c[0]; sy = c[1]; sz = c[2];
        }
        if (idx[0] < G.n[0] - 1 && idx[1] < G.n[1] - 1 && idx[2] < G.n[2] - 1) {
            double P[8][3], g[8];
            for (int q = 0; q < 8; ++q) {
                for (int a = 0; a < 3; ++a) P[q][a] = G.lo[a] + G.h * (double)(idx[a] + ((q >> a) & 1));
                g[q] = cm1(b, P[q][0], P[q][1], P[q][2]);
            }
            double gmin = g[0], gmax = g[0];
            for (int q = 1; q < 8; ++q) { gmin = fmin(gmin, g[q]); gmax = fmax(gmax, g[q]); }
            if (gmin < 0.0 && gmax >= 0.0) {
                const int tets[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};
                for (int e = 0; e < 6; ++e) {
                    double Pt[4][3], gt[4];
                    for (int v = 0; v < 4; ++v) {
                        gt[v] = g[tets[e][v]];
                        for (int a = 0; a < 3; ++a) Pt[v][a] = P[tets[e][v]][a];
                    }
                    area += tet_area(Pt, gt);
                }
            }
        }
    }
    const double v[5] = {cnt, sx, sy, sz, area};
    for (int q = 0; q < 5; ++q) {
        const double s = block_sum(v[q], red);
        if (threadIdx.x == 0) part[5 * blockIdx.x + q] = s;
    }
}

// Pass 2: second moments about the centroid c of the inside centres.
__global__ __launch_bounds__(BLK) void k_shape_moments(Body b, Grid G, long long cells, double cx, double cy,
                                                       double cz, double *__restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    const long long t = blockIdx.x * (long long)BLK + threadIdx.x;
    double m[6] = {0, 0, 0, 0, 0, 0};
    if (t < cells) {
        double c[3];
        int idx[3];
        centre(G, t, c, idx);
        if (cm1(b, c[0], c[1], c[2]) >= 0.0) {
            const double r[3] = {c[0] - cx, c[1] - cy, c[2] - cz};
            m[0] = r[0] * r[0]; m[1] = r[1] * r[1]; m[2] = r[2] * r[2];
            m[3] = r[0] * r[1]; m[4] = r[0] * r[2]; m[5] = r[1] * r[2];
        }
    }
    for (int q = 0; q < 6; ++q) {
        const double s = block_sum(m[q], red);
        if (threadIdx.x == 0) part[6 * blockIdx.x + q] = s;
    }
}

// Pass 3: min and max of the inside centres projected on the three axes
// (rows of ax), relative to the centroid.
__global__ __launch_bounds__(BLK) void k_shape_extent(Body b, Grid G, long long cells, double cx, double cy, double cz,
                                                      const double *__restrict__ ax, double *__restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    const long long t = blockIdx.x * (long long)BLK + threadIdx.x;
    double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, mhi[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL};
    if (t < cells) {
        double c[3];
        int idx[3];
        centre(G, t, c, idx);
        if (cm1(b, c[0], c[1], c[2]) >= 0.0) {
            const double r[3] = {c[0] - cx, c[1] - cy, c[2] - cz};
            for (int a = 0; a < 3; ++a) {
                const double pr = (r[0] * ax[3 * a] + r[1] * ax[3 * a + 1]) + r[2] * ax[3 * a + 2];
                lo[a] = pr;
                mhi[a] = -pr;
            }
        }
    }
    for (int a = 0; a < 3; ++a) {
        const double mn = block_min(lo[a], red), mx = block_min(mhi[a], red);
        if (threadIdx.x == 0) {
            part[6 * blockIdx.x + a] = mn;
            part[6 * blockIdx.x + 3 + a] = mx;
        }
    }
}

// Pass 4: columns along the shortest axis (aS) over the grid of the plane of
// the two longer ones (aL along u, aI along v) that hold an inside sample.
__global__ __launch_bounds__(BLK) void k_shape_project(Body b, double cx, double cy, double cz,
                                                       const double *__restrict__ ax, double hL, double hI, double hS,
                                                       double h, int nu, int nv, int nw, double *__restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    const long long t = blockIdx.x * (long long)BLK + threadIdx.x;
    double hit = 0.0;
    if (t < (long long)nu * nv) {
        const int iu = (int)(t / nv), iv = (int)(t - (long long)iu * nv);
        const double u = -hL + h * (double)iu, v = -hI + h * (double)iv;
        const double *aS = ax, *aI = ax + 3, *aL = ax + 6;
        for (int iw = 0; iw < nw && hit == 0.0; ++iw) {
            const double w = -hS + h * (double)iw;
            const double x = ((cx + u * aL[0]) + v * aI[0]) + w * aS[0];
            const double y = ((cy + u * aL[1]) + v * aI[1]) + w * aS[1];
            const double z = ((cz + u * aL[2]) + v * aI[2]) + w * aS[2];
            if (cm1(b, x, y, z) >= 0.0) hit = 1.0;
        }
    }
    const double s = block_sum(hit, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Eigenvectors of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (columns of V).
void jacobi3(double A[3][3], double V[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {  // A <- J^T A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
}

bool make_grid(const double *cp, const double *k, int n, double h, Grid &G, long long &cells) {
    double sk = 0.0;
    for (int j = 0; j < n; ++j) sk += k[j];
    const double r = std::sqrt(sk);
    for (int a = 0; a < 3; ++a) {
        double mn = cp[a], mx = cp[a];
        for (int j = 1; j < n; ++j) {
            mn = std::fmin(mn, cp[3 * j + a]);
            mx = std::fmax(mx, cp[3 * j + a]);
        }
        G.lo[a] = mn - r - h;
        const double hi = mx + r + h;
        const double na = std::ceil((hi - G.lo[a]) / h) + 1.0;
        if (!(na >= 2.0 && na < 2e6)) return false;
        G.n[a] = (int)na;
    }
    G.h = h;
    cells = (long long)G.n[0] * G.n[1] * G.n[2];
    return cells < (1ll << 31);
}

inline long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

}  // namespace

extern "C" {

size_t mb_shape_work_bytes(const double *cp, const double *k, int32_t n, double h) {
    if (!cp || !k || n < 1 || n > MAXN || !(h > 0.0)) return 0;
    Grid G;
    long long cells;
    if (!make_grid(cp, k, n, h, G, cells)) return 0;
    // per-block slots of the widest pass (6 doubles), and the three axes
    const long long blocks = cdiv(cells, BLK);
    return (size_t)(6 * blocks + 16) * sizeof(double);
}

lbm_status mb_shape_descriptors(const double *cp, const double *k, int32_t n, double h, void *work,
                                size_t work_bytes, void *hip_stream, mb_shape *out) {
    if (!cp || !k || !work || !out || n < 1 || n > MAXN || !(h > 0.0)) return LBM_E_INVALID;
    Body b;
    memset(&b, 0, sizeof b);
    b.n = n;
    for (int j = 0; j < n; ++j) {
        if (!(k[j] > 0.0) || !std::isfinite(k[j])) return LBM_E_INVALID;
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(cp[3 * j + a])) return LBM_E_INVALID;
            b.p[j][a] = cp[3 * j + a];
        }
        b.k[j] = k[j];
    }
    Grid G;
    long long cells;
    if (!make_grid(cp, k, n, h, G, cells)) return LBM_E_INVALID;
    const long long blocks = cdiv(cells, BLK);
    if (work_bytes < (size_t)(6 * blocks + 16) * sizeof(double)) return LBM_E_NOMEM;
    hipStream_t s = (hipStream_t)hip_stream;
    double *part = (double *)work, *axd = part + 6 * blocks;
    std::vector<double> hp((size_t)6 * blocks);
    auto fetch = [&](size_t count) {
        return hipMemcpyAsync(hp.data(), part, count * sizeof(double), hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    // pass 1
    k_shape_grid<<<(unsigned)blocks, BLK, 0, s>>>(b, G, cells, part);
    if (hipGetLastError() != hipSuccess || !fetch(5 * blocks)) return LBM_E_HIP;
    double cnt = 0, sx = 0, sy = 0, sz = 0, area = 0;
    for (long long q = 0; q < blocks; ++q) {
        cnt += hp[5 * q]; sx += hp[5 * q + 1]; sy += hp[5 * q + 2]; sz += hp[5 * q + 3]; area += hp[5 * q + 4];
    }
    if (!(cnt > 0.0)) return LBM_E_INVALID;
    const double c[3] = {sx / cnt, sy / cnt, sz / cnt};
    // pass 2
    k_shape_moments<<<(unsigned)blocks, BLK, 0, s>>>(b, G, cells, c[0], c[1], c[2], part);
    if (hipGetLastError() != hipSuccess || !fetch(6 * blocks)) return LBM_E_HIP;
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (long long q = 0; q < blocks; ++q)
        for (int a = 0; a < 6; ++a) m[a] += hp[6 * q + a];
    double A[3][3] = {{m[0], m[3], m[4]}, {m[3], m[1], m[5]}, {m[4], m[5], m[2]}}, V[3][3];
    jacobi3(A, V);
    double ax[9];
    for (int j = 0; j < 3; ++j) {  // axis j = column j, signed by its largest component
        int big = 0;
        for (int a = 1; a < 3; ++a)
            if (std::fabs(V[a][j]) > std::fabs(V[big][j])) big = a;
        const double sg = V[big][j] < 0 ? -1.0 : 1.0;
        for (int a = 0; a < 3; ++a) ax[3 * j + a] = sg * V[a][j];
    }
    // pass 3
    if (hipMemcpyAsync(axd, ax, sizeof ax, hipMemcpyHostToDevice, s) != hipSuccess) return LBM_E_HIP;
    k_shape_extent<<<(unsigned)blocks, BLK, 0, s>>>(b, G, cells, c[0], c[1], c[2], axd, part);
    if (hipGetLastError() != hipSuccess || !fetch(6 * blocks)) return LBM_E_HIP;
    double mn[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, mx[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL};
    for (long long q = 0; q < blocks; ++q)
        for (int a = 0; a < 3; ++a) {
            mn[a] = std::fmin(mn[a], hp[6 * q + a]);
            mx[a] = std::fmin(mx[a], hp[6 * q + 3 + a]);
        }
    double ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = -mx[a] - mn[a];
    int order[3] = {0, 1, 2};  // by increasing extent, stable
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && ext[order[j]] < ext[order[j - 1]]; --j) std::swap(order[j], order[j - 1]);
    double axs[9], dims[3];
    for (int a = 0; a < 3; ++a) {
        dims[a] = ext[order[a]] + h;
        for (int q = 0; q < 3; ++q) axs[3 * a + q] = ax[3 * order[a] + q];
    }
    // pass 4: the plane of the two longer axes
    double half[3];
    int cntax[3];
    for (int a = 0; a < 3; ++a) {
        half[a] = 0.5 * dims[a] + 2.0 * h;
        cntax[a] = (int)std::ceil(2.0 * half[a] / h) + 1;
    }
    const long long cols = (long long)cntax[2] * cntax[1];
    const long long pblocks = cdiv(cols, BLK);
    if (pblocks > 6 * blocks) return LBM_E_NOMEM;
    if (hipMemcpyAsync(axd, axs, sizeof axs, hipMemcpyHostToDevice, s) != hipSuccess) return LBM_E_HIP;
    k_shape_project<<<(unsigned)pblocks, BLK, 0, s>>>(b, c[0], c[1], c[2], axd, half[2], half[1], half[0], h,
                                                     cntax[2], cntax[1], cntax[0], part);
    if (hipGetLastError() != hipSuccess || !fetch(pblocks)) return LBM_E_HIP;
    double hits = 0;
    for (long long q = 0; q < pblocks; ++q) hits += hp[q];
    mb_shape &o = *out;
    o.V = cnt * h * h * h;
    o.S = area;
    o.A_p = hits * h * h;
    for (int a = 0; a < 3; ++a) {
        o.dims[a] = dims[a];
        o.centroid[a] = c[a];
    }
    memcpy(o.axes, axs, sizeof axs);
    o.d_n = std::cbrt(6.0 * o.V / M_PI);
    o.d_s = std::sqrt(4.0 * o.A_p / M_PI);
    o.Phi = M_PI * o.d_n * o.d_n / o.S;
    o.CSF = dims[0] / std::sqrt(dims[1] * dims[2]);
    o.cells_inside = (int64_t)cnt;
    o.columns_hit = (int64_t)hits;
    return LBM_OK;
}

}  // extern "C"
