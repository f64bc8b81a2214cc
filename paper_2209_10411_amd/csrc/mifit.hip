// Metaball-Imaging fit (sec. 2.2): the genetic algorithm's evaluation,
// mutation, crossover and selection, and the gradient search with the
// piecewise objective of Eq. GSloss and the anomaly cleaning.  C ABI in
// include/mifit.h.  Everything is FP64: the fitness decides the selection
// (an integer decision), and the gradient search runs 10^5 dependent
// steps.  Nothing here is a dense contraction (one reciprocal per hull
// point and control point), so it runs on the vector ALUs.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>
#include <mutex>

#include "../../include/mifit.h"

namespace {

constexpr int BLK = 256;         // threads of the fitness and gradient-search blocks (4 waves)
constexpr int CHUNK = 2048;      // hull points per fitness block
constexpr int SEL_BLK = 1024;    // threads of the selection sort
constexpr int SEL_MAX = 4096;    // pool size the one-block sort holds
constexpr double EPS_F = 1e-12;  // floor of f in the 1/f term of the objective

// Fixed-order sum over the block: butterfly within each wave, then the four
// wave sums in wave order.  Every thread returns the total.
__device__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();  // red may still be read from the previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// f(h) = sum_j k_j / |h - p_j|^2 with the model in LDS ([n][4]: k, x, y, z).
__device__ __forceinline__ double mb_value(const double *sM, int n, double hx, double hy, double hz) {
    double f = 0.0;
    for (int j = 0; j < n; ++j) {
        const double dx = hx - sM[4 * j + 1], dy = hy - sM[4 * j + 2], dz = hz - sM[4 * j + 3];
        f += sM[4 * j] / (dx * dx + dy * dy + dz * dz);
    }
    return f;
}

// The same sum with each quotient k / r^2 as k times the hardware reciprocal
// estimate of r^2 refined by two Newton steps (within a few ulp of the
// quotient; the fitness, a sum of squares of f - 1, is compared and ranked,
// not tested for equality).
__device__ __forceinline__ double mb_value_rcp(const double *sM, int n, double hx, double hy, double hz) {
    double f = 0.0;
    for (int j = 0; j < n; ++j) {
        const double dx = hx - sM[4 * j + 1], dy = hy - sM[4 * j + 2], dz = hz - sM[4 * j + 3];
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        double r = __builtin_amdgcn_rcp(r2);
        double e = fma(-r2, r, 1.0);
        r = fma(e, r, r);
        e = fma(-r2, r, 1.0);
        r = fma(e, r, r);
        f = fma(sM[4 * j], r, f);
    }
    return f;
}

// The per-point term of Eq. GSloss and its slope.
__device__ __forceinline__ double gs_term(double f) {
    if (f >= 2.0) return (f - 1.0) * (f - 1.0);
    if (f >= 1.0) return f - 1.0;
    const double fc = f > EPS_F ? f : EPS_F;
    return (f - 1.0) * (f - 1.0) + 1.0 / fc - 1.0;
}
__device__ __forceinline__ double gs_slope(double f) {
    if (f >= 2.0) return 2.0 * (f - 1.0);
    if (f >= 1.0) return 1.0;
    return 2.0 * (f - 1.0) - (f > EPS_F ? 1.0 / (f * f) : 0.0);
}

// ------------------------------------------------------------- evaluation
// Block (individual p, chunk c): sum over the chunk's hull points of
// (f - 1)^2, written to out[p * nch + c].
__global__ __launch_bounds__(BLK) void k_fitness(const double *__restrict__ hull, long long m,
                                                 const double *__restrict__ pop, int n, int nch,
                                                 double *__restrict__ out) {
    __shared__ double sM[MI_MAXCP * 4];
    __shared__ double red[4];
    const int p = blockIdx.x / nch, c = blockIdx.x - p * nch;
    const double *M = pop + (size_t)p * n * 4;
    for (int t = threadIdx.x; t < 4 * n; t += BLK) sM[t] = M[t];
    __syncthreads();
    const long long i0 = (long long)c * CHUNK;
    const long long i1 = i0 + CHUNK < m ? i0 + CHUNK : m;
    double s = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += BLK) {
        const double e = mb_value_rcp(sM, n, hull[3 * i], hull[3 * i + 1], hull[3 * i + 2]) - 1.0;
        s += e * e;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// F[p] = the chunk sums of individual p added in chunk order.
__global__ void k_fitness_sum(const double *__restrict__ part, int P, int nch, double *__restrict__ F) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(size_t)p * nch + c];
    F[p] = s;
}

// ------------------------------------------------------ genetic operators
// One mutant per individual (gene-wise; no contraction, so that each gene is
// exactly v + z * sigma).
__global__ void k_mutate(const double *__restrict__ pop, double *__restrict__ out, const double *__restrict__ U,
                         const double *__restrict__ Z, long long count, double C_m, double sx, double sk) {
#pragma clang fp contract(off)
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int g = (int)(i & 3);
    double v = pop[i];
    if (U[i] < C_m) v = v + Z[i] * (g == 0 ? sk : sx);
    if (g == 0 && v < 0.0) v = 0.0;
    out[i] = v;
}

// Children of the pairs (perm[2j], perm[2j+1]): control points from c on are
// exchanged; an odd last individual is copied.
__global__ void k_crossover(const double *__restrict__ pop, double *__restrict__ kids, const int *__restrict__ perm,
                            int N, int n, int c) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int g4 = 4 * n;
    if (i >= (long long)N * g4) return;
    const int a = (int)(i / g4), r = (int)(i - (long long)a * g4), j = r >> 2;
    int src;
    if ((N & 1) && a == N - 1) {
        src = perm[a];
    } else {
        const int first = perm[a & ~1], second = perm[a | 1];
        const bool head = j < c;
        src = (a & 1) ? (head ? second : first) : (head ? first : second);
    }
    if ((unsigned)src >= (unsigned)N) src = a;  // not a permutation entry: keep the index in range
    kids[i] = pop[(size_t)src * g4 + r];
}

// Indices of the N smallest of K pool fitness values, ties to the lower
// index: one block, bitonic sort of (F, index) pairs in LDS (NaN sorts as
// +inf, padding as +inf with indices past K).
__global__ __launch_bounds__(SEL_BLK) void k_select(const double *__restrict__ F, int K, int N, int *__restrict__ idx) {
    __shared__ double key[SEL_MAX];
    __shared__ int id[SEL_MAX];
    int L = 1;
    while (L < K) L <<= 1;
    for (int t = threadIdx.x; t < L; t += SEL_BLK) {
        const double v = t < K ? F[t] : HUGE_VAL;
        key[t] = v != v ? HUGE_VAL : v;
        id[t] = t;
    }
    __syncthreads();
    for (int size = 2; size <= L; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < L; t += SEL_BLK) {
                const int u = t ^ stride;
                if (u > t) {
                    const bool up = (t & size) == 0;
                    const double ka = key[t], kb = key[u];
                    const int ia = id[t], ib = id[u];
                    const bool gt = ka > kb || (ka == kb && ia > ib);
                    if (gt == up) {
                        key[t] = kb; key[u] = ka;
                        id[t] = ib; id[u] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int r = threadIdx.x; r < N; r += SEL_BLK) idx[r] = id[r];
}

__global__ void k_gather(const double *__restrict__ pool, const double *__restrict__ Fpool, const int *__restrict__ idx,
                         int N, int n, double *__restrict__ pop, double *__restrict__ F) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int g4 = 4 * n;
    if (i >= (long long)N * g4) return;
    const int a = (int)(i / g4), r = (int)(i - (long long)a * g4);
    pop[i] = pool[(size_t)idx[a] * g4 + r];
    if (r == 0) F[a] = Fpool[idx[a]];
}

// --------------------------------------------------------- gradient search
// n . p + d of a half-space (no contraction: the same sum as a plain dot product).
__device__ __forceinline__ double plane_side(const double *pl, double px, double py, double pz) {
#pragma clang fp contract(off)
    return ((px * pl[0] + py * pl[1]) + pz * pl[2]) + pl[3];
}

// Sum over the hull points of the Eq. GSloss terms for the model in LDS.
__device__ double gs_loss_block(const double *__restrict__ hull, long long m, const double *sM, int n, double *red) {
    double s = 0.0;
    for (long long i = threadIdx.x; i < m; i += BLK)
        s += gs_term(mb_value(sM, n, hull[3 * i], hull[3 * i + 1], hull[3 * i + 2]));
    return block_sum(s, red);
}

// One workgroup per model: E descent steps, cleaning, E steps.  Per step:
// pass 1, one hull point per lane: f and the objective's slope g_i (in
// LDS); pass 2, lanes over (control point j, chunk of points):
// dL/dk_j = sum g_i / r^2, dL/dp_j = sum g_i 2 k_j (h_i - p_j) / r^4 over the
// chunk; the chunks are added in order and the model updated in LDS.
__global__ __launch_bounds__(BLK) void k_gs(const double *__restrict__ hulls, const int64_t *__restrict__ hoff,
                                            const double *__restrict__ planes, const int64_t *__restrict__ poff,
                                            int n, int E, double eta, double *__restrict__ Mall,
                                            double *__restrict__ loss) {
    __shared__ double sM[MI_MAXCP * 4];
    __shared__ double part[BLK * 4];
    __shared__ double red[4];
    __shared__ double g[MI_GS_MAXPTS];  // the objective's slope at each hull point
    const int b = blockIdx.x;
    const long long h0 = hoff[b], m = hoff[b + 1] - h0;
    const double *hull = hulls + 3 * h0;
    double *M = Mall + (size_t)b * n * 4;
    for (int t = threadIdx.x; t < 4 * n; t += BLK) sM[t] = M[t];
    __syncthreads();
    double L = gs_loss_block(hull, m, sM, n, red);
    if (threadIdx.x == 0) loss[3 * b] = L;
    const int nch = BLK / n;                 // chunks of points in pass 2
    const int j = threadIdx.x % n, c = threadIdx.x / n;
    for (int phase = 0; phase < 2; ++phase) {
        for (int it = 0; it < E; ++it) {
            for (long long i = threadIdx.x; i < m; i += BLK)
                g[i] = gs_slope(mb_value(sM, n, hull[3 * i], hull[3 * i + 1], hull[3 * i + 2]));
            __syncthreads();
            double gk = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
            if (c < nch) {
                const double k = sM[4 * j], px = sM[4 * j + 1], py = sM[4 * j + 2], pz = sM[4 * j + 3];
                for (long long i = c; i < m; i += nch) {
                    const double dx = hull[3 * i] - px, dy = hull[3 * i + 1] - py, dz = hull[3 * i + 2] - pz;
                    const double y = 1.0 / (dx * dx + dy * dy + dz * dz);
                    const double gi = g[i];
                    gk += gi * y;
                    const double t = 2.0 * gi * k * y * y;
                    gx += t * dx; gy += t * dy; gz += t * dz;
                }
            }
            part[4 * threadIdx.x] = gk; part[4 * threadIdx.x + 1] = gx;
            part[4 * threadIdx.x + 2] = gy; part[4 * threadIdx.x + 3] = gz;
            __syncthreads();
            if (threadIdx.x < 4 * n) {  // gene t of control point t / 4, chunks in order
                const int jj = threadIdx.x >> 2, q = threadIdx.x & 3;
                double G = 0.0;
                for (int cc = 0; cc < nch; ++cc) G += part[4 * (cc * n + jj) + q];
                sM[threadIdx.x] -= eta * G;
            }
            __syncthreads();
        }
        if (phase == 0) {
            L = gs_loss_block(hull, m, sM, n, red);
            if (threadIdx.x == 0) loss[3 * b + 1] = L;
            // anomaly cleaning: negative weights and control points outside the hull
            if (threadIdx.x < n) {
                const int jj = threadIdx.x;
                bool out = sM[4 * jj] < 0.0;
                const double px = sM[4 * jj + 1], py = sM[4 * jj + 2], pz = sM[4 * jj + 3];
                for (long long q = poff[b]; q < poff[b + 1] && !out; ++q) out = plane_side(planes + 4 * q, px, py, pz) > 0.0;
                if (out) sM[4 * jj] = 0.0;
            }
            __syncthreads();
        }
    }
    L = gs_loss_block(hull, m, sM, n, red);
    if (threadIdx.x == 0) loss[3 * b + 2] = L;
    for (int t = threadIdx.x; t < 4 * n; t += BLK) M[t] = sM[t];
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int chunks(long long m) { return cdiv(m, CHUNK); }

lbm_status launched() { return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP; }

// Fitness of P individuals into F (partials in part when m spans chunks).
lbm_status fitness_launch(const double *hull, long long m, const double *pop, int P, int n, double *F, double *part,
                          hipStream_t s) {
    const int nch = chunks(m);
    if (nch == 1) {
        k_fitness<<<P, BLK, 0, s>>>(hull, m, pop, n, 1, F);
    } else {
        k_fitness<<<P * nch, BLK, 0, s>>>(hull, m, pop, n, nch, part);
        k_fitness_sum<<<cdiv(P, 256), 256, 0, s>>>(part, P, nch, F);
    }
    return launched();
}

struct GaLayout {
    size_t poolA, poolB, FA, FB, idx, part, total;
};
GaLayout ga_layout(long long m, int N, int n) {
    GaLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const size_t pool = (size_t)3 * N * n * 4 * sizeof(double);
    L.poolA = take(pool);
    L.poolB = take(pool);
    L.FA = take((size_t)3 * N * sizeof(double));
    L.FB = take((size_t)3 * N * sizeof(double));
    L.idx = take((size_t)N * sizeof(int));
    L.part = take(chunks(m) > 1 ? (size_t)2 * N * chunks(m) * sizeof(double) : 0);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

size_t mi_fitness_work_bytes(int64_t m, int32_t P) {
    if (m < 1 || P < 1) return 0;
    return chunks(m) > 1 ? (size_t)P * chunks(m) * sizeof(double) : 0;
}

lbm_status mi_fitness(const double *hull, int64_t m, const double *pop, int32_t P, int32_t n, double *F, void *work,
                      size_t work_bytes, void *hip_stream) {
    if (!hull || !pop || !F || m < 1 || P < 1 || n < 1 || n > MI_MAXCP) return LBM_E_INVALID;
    if ((long long)P * chunks(m) > 0x7fffffffll) return LBM_E_INVALID;
    const size_t need = mi_fitness_work_bytes(m, P);
    if (need && (!work || work_bytes < need)) return LBM_E_NOMEM;
    return fitness_launch(hull, m, pop, P, n, F, (double *)work, (hipStream_t)hip_stream);
}

size_t mi_ga_work_bytes(int64_t m, int32_t N_I, int32_t n) {
    if (m < 1 || N_I < 2 || n < 1 || n > MI_MAXCP) return 0;
    return ga_layout(m, N_I, n).total;
}

lbm_status mi_ga(const double *hull, int64_t m, int32_t N_I, int32_t n, int32_t E, double C_m, double C_c,
                 double sigma_x, double sigma_k, const double *U, const double *Z, const int32_t *PERM, double *pop,
                 double *F, void *work, size_t work_bytes, void *hip_stream) {
    if (!hull || !pop || !F || !work || m < 1 || n < 1 || n > MI_MAXCP || N_I < 2 || 3 * N_I > SEL_MAX || E < 0)
        return LBM_E_INVALID;
    if (E > 0 && (!U || !Z || !PERM)) return LBM_E_INVALID;
    if (!(C_c >= 0.0 && C_c <= 1.0) || !(sigma_x >= 0.0) || !(sigma_k >= 0.0)) return LBM_E_INVALID;
    const GaLayout Lw = ga_layout(m, N_I, n);
    if (work_bytes < Lw.total) return LBM_E_NOMEM;
    hipStream_t s = (hipStream_t)hip_stream;
    char *w = (char *)work;
    double *A = (double *)(w + Lw.poolA), *B = (double *)(w + Lw.poolB);
    double *FA = (double *)(w + Lw.FA), *FB = (double *)(w + Lw.FB);
    int *idx = (int *)(w + Lw.idx);
    double *part = (double *)(w + Lw.part);
    const long long genes = (long long)N_I * n * 4;
    const int c = (int)(C_c * n + 0.5);
    if (hipMemcpyAsync(A, pop, genes * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return LBM_E_HIP;
    lbm_status st = fitness_launch(hull, m, A, N_I, n, FA, part, s);
    if (st) return st;
    for (int e = 0; e < E; ++e) {
        k_mutate<<<cdiv(genes, 256), 256, 0, s>>>(A, A + genes, U + (size_t)e * genes, Z + (size_t)e * genes, genes,
                                                 C_m, sigma_x, sigma_k);
        k_crossover<<<cdiv(genes, 256), 256, 0, s>>>(A, A + 2 * genes, PERM + (size_t)e * N_I, N_I, n, c);
        if ((st = fitness_launch(hull, m, A + genes, 2 * N_I, n, FA + N_I, part, s))) return st;
        k_select<<<1, SEL_BLK, 0, s>>>(FA, 3 * N_I, N_I, idx);
        k_gather<<<cdiv(genes, 256), 256, 0, s>>>(A, FA, idx, N_I, n, B, FB);
        if ((st = launched())) return st;
        double *t = A; A = B; B = t;
        t = FA; FA = FB; FB = t;
    }
    if (hipMemcpyAsync(pop, A, genes * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(F, FA, N_I * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LBM_E_HIP;
    return launched();
}

lbm_status mi_gs(const double *hulls, const int64_t *hull_off, const double *planes, const int64_t *plane_off,
                 int32_t B, int32_t n, int32_t E, double eta, double *M, double *loss, void *hip_stream) {
    if (!hulls || !hull_off || !planes || !plane_off || !M || !loss || B < 1 || n < 1 || n > MI_MAXCP || E < 0 ||
        !(eta >= 0.0))
        return LBM_E_INVALID;
    // the offsets live on the device: read them to check every hull's size
    hipStream_t s = (hipStream_t)hip_stream;
    int64_t *ho = new int64_t[2 * (size_t)(B + 1)];
    if (hipMemcpyAsync(ho, hull_off, 8 * (size_t)(B + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(ho + B + 1, plane_off, 8 * (size_t)(B + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        delete[] ho;
        return LBM_E_HIP;
    }
    bool ok = ho[0] >= 0 && ho[B + 1] >= 0;
    for (int b = 0; b < B && ok; ++b)
        ok = ho[b + 1] - ho[b] >= 1 && ho[b + 1] - ho[b] <= MI_GS_MAXPTS && ho[B + 2 + b] >= ho[B + 1 + b];
    delete[] ho;
    if (!ok) return LBM_E_INVALID;
    k_gs<<<B, BLK, 0, s>>>(hulls, hull_off, planes, plane_off, n, E, eta, M, loss);
    return launched();
}

// ---------------------------------------------- fitness without allocation
// For callers that cannot allocate (graph capture, tight loops): the chunk
// sums live in this file-scope array, one copy per GPU, held until the
// process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t MI_SCRATCH_DOUBLES = size_t(1) << 17;  // 1 MiB: individuals x chunks <= 131072
__device__ __align__(256) double scratch[MI_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES];
}  // namespace

lbm_status mi_fitness_noalloc(const double *hull, int64_t m, const double *pop, int32_t P, int32_t n, double *F,
                              void *hip_stream) {
    if (!hull || !pop || !F || m < 1 || P < 1 || n < 1 || n > MI_MAXCP) return LBM_E_INVALID;
    if ((long long)P * chunks(m) > (long long)MI_SCRATCH_DOUBLES) return LBM_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return LBM_E_HIP;
    double *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch[dev]) {
            void *a = nullptr;
            if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return LBM_E_HIP;
            g_scratch[dev] = (double *)a;
        }
        ptr = g_scratch[dev];
    }
    return fitness_launch(hull, m, pop, P, n, F, ptr, (hipStream_t)hip_stream);
}

}  // extern "C"
