// Warm-start MLP: link features, batched forward/backward and Adam for
// training (own kernels, FP32 accumulation; one thread per output element,
// fixed-order sums so that every result is deterministic).  The one-link
// inference inside the link solver is in kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp_dev.h"

namespace mdl {

namespace {
__constant__ int m_ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int m_ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int m_ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

// Blob: theta, m, v (FP32 [P]); w16 (FP16 [P]); t; workspace for
// MLP_MAX_BATCH samples.
size_t mlp_blob_bytes() {
    size_t o = 0;
    o = al(o + 4 * (size_t)MLP_P);          // theta
    o = al(o + 4 * (size_t)MLP_P);          // m
    o = al(o + 4 * (size_t)MLP_P);          // v
    o = al(o + 2 * (size_t)MLP_P);          // w16
    o = al(o + 8);                          // t
    o = al(o + 4 * (size_t)MLP_MAX_BATCH * MLP_H);  // h1
    o = al(o + 4 * (size_t)MLP_MAX_BATCH * MLP_H);  // h2
    o = al(o + 4 * (size_t)MLP_MAX_BATCH * MLP_OUT);  // out
    o = al(o + 4 * (size_t)MLP_MAX_BATCH * MLP_OUT);  // dout
    o = al(o + 4 * (size_t)MLP_MAX_BATCH * MLP_H);  // dz1
    o = al(o + 4 * (size_t)MLP_MAX_BATCH * MLP_H);  // dz2
    o = al(o + 4 * (size_t)MLP_P);          // g
    o = al(o + 4);                          // loss
    o = al(o + 4 * (size_t)16 * (MLP_IN + 1) * MLP_H);  // weight-gradient slices
    return o;
}

MlpBlob mlp_blob(void *base) {
    char *b = (char *)base;
    MlpBlob r;
    size_t o = 0;
    auto take = [&](size_t bytes) { char *p = b + o; o = al(o + bytes); return p; };
    r.theta = (float *)take(4 * (size_t)MLP_P);
    r.m = (float *)take(4 * (size_t)MLP_P);
    r.v = (float *)take(4 * (size_t)MLP_P);
    r.w16 = (_Float16 *)take(2 * (size_t)MLP_P);
    r.t = (long long *)take(8);
    r.h1 = (float *)take(4 * (size_t)MLP_MAX_BATCH * MLP_H);
    r.h2 = (float *)take(4 * (size_t)MLP_MAX_BATCH * MLP_H);
    r.out = (float *)take(4 * (size_t)MLP_MAX_BATCH * MLP_OUT);
    r.dout = (float *)take(4 * (size_t)MLP_MAX_BATCH * MLP_OUT);
    r.dz1 = (float *)take(4 * (size_t)MLP_MAX_BATCH * MLP_H);
    r.dz2 = (float *)take(4 * (size_t)MLP_MAX_BATCH * MLP_H);
    r.g = (float *)take(4 * (size_t)MLP_P);
    r.loss = (float *)take(4);
    r.part = (float *)take(4 * (size_t)16 * (MLP_IN + 1) * MLP_H);
    return r;
}

__global__ void k_mlp_init(float *theta, float *m, float *v, _Float16 *w16, long long *t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_P) {
        m[i] = 0.f;
        v[i] = 0.f;
        w16[i] = (_Float16)theta[i];
    }
    if (i == 0) *t = 0;
}

// z = h_prev W + b for sample b, unit n; tanh (stored as TA) or linear (FP32 out)
template <typename TA, typename TW>
__global__ void k_mlp_layer(const TA *__restrict__ X, int K, const TW *__restrict__ W, int offW, int offB, int N,
                            int B, TA *__restrict__ H, float *__restrict__ out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * N) return;
    const int b = idx / N, n = idx - b * N;
    float z = (float)W[offB + n];
    for (int k = 0; k < K; ++k) z += (float)X[(long long)b * K + k] * (float)W[offW + k * N + n];
    if (H) H[idx] = (TA)tanhf(z);
    else out[idx] = z;
}

// loss gradient of the masked squared error (mean over the batch); the
// squared errors go to sq for the loss sum
template <typename TA>
__global__ void k_mlp_out_grad(const TA *__restrict__ X, const float *__restrict__ out,
                               const float *__restrict__ T, int B, float *__restrict__ dout,
                               float *__restrict__ sq) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * MLP_OUT) return;
    const int b = idx / MLP_OUT, j = idx - b * MLP_OUT;
    const bool task = (float)X[(long long)b * MLP_IN + 6] > 0.5f;
    const bool on = task ? j > 0 : j == 0;
    const float d = out[idx] - T[idx];
    dout[idx] = on ? 2.f * d / (float)B : 0.f;
    sq[idx] = on ? d * d : 0.f;
}

// fixed-order sum of the squared errors (one block of 256 threads)
__global__ void k_mlp_loss(const float *__restrict__ sq, int n, int B, float *__restrict__ loss) {
    __shared__ float s[256];
    float a = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) a += sq[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s[0] / (float)B;
}

// dZ_prev[b][k] = (sum_n dZ[b][n] W[k][n]) (1 - h[b][k]^2)
template <typename TA, typename TW>
__global__ void k_mlp_bwd_data(const float *__restrict__ dZ, int N, const TW *__restrict__ W, int offW, int K,
                               const TA *__restrict__ H, int B, float *__restrict__ dZp) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * K) return;
    const int b = idx / K, k = idx - b * K;
    float s = 0.f;
    for (int n = 0; n < N; ++n) s += dZ[(long long)b * N + n] * (float)W[offW + k * N + n];
    const float h = (float)H[idx];
    dZp[idx] = s * (1.f - h * h);
}

// Weight gradients in two fixed-order stages: slice s of the batch gives
// part[s][k][n] = sum_{b in slice} h[b][k] dZ[b][n] (row k = K: the bias,
// h = 1); then g = sum over the slices in order.
constexpr int MLP_SLICES = 16;
template <typename TA>
__global__ void k_mlp_bwd_weight_part(const TA *__restrict__ Hin, int K, const float *__restrict__ dZ, int N, int B,
                                      float *__restrict__ part) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = (K + 1) * N;
    if (idx >= MLP_SLICES * per) return;
    const int sl = idx / per, r = idx - sl * per, k = r / N, n = r - k * N;
    const int b0 = (int)((long long)B * sl / MLP_SLICES), b1 = (int)((long long)B * (sl + 1) / MLP_SLICES);
    float s = 0.f;
    if (k < K)
        for (int b = b0; b < b1; ++b) s += (float)Hin[(long long)b * K + k] * dZ[(long long)b * N + n];
    else
        for (int b = b0; b < b1; ++b) s += dZ[(long long)b * N + n];
    part[idx] = s;
}

__global__ void k_mlp_bwd_weight_sum(const float *__restrict__ part, int K, int N, float *__restrict__ g, int offW,
                                     int offB) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = (K + 1) * N;
    if (r >= per) return;
    float s = 0.f;
    for (int sl = 0; sl < MLP_SLICES; ++sl) s += part[sl * per + r];
    const int k = r / N, n = r - k * N;
    if (k < K) g[offW + k * N + n] = s;
    else g[offB + n] = s;
}

__global__ void k_mlp_adam(float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, _Float16 *__restrict__ w16, float lr, float b1, float b2,
                           float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    theta[i] = th;
    w16[i] = (_Float16)th;
}

// features and target (q, 0, 0, 0) of each link of the list
__global__ void k_mlp_collect(Params p, const DevParticle *__restrict__ P, const float *__restrict__ body,
                              const uint32_t *__restrict__ l_node, const uint32_t *__restrict__ l_do,
                              const double *__restrict__ l_q, int n, _Float16 *__restrict__ feat,
                              float *__restrict__ target) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const long long node = l_node[l];
    const int i = (int)(l_do[l] & 31u), pid = (int)(l_do[l] >> 8);
    _Float16 *f = feat + (long long)l * MLP_IN;
    float *t = target + (long long)l * MLP_OUT;
    if (node >= p.N || pid >= p.np || i < 1 || i >= 19) {  // never expected: an all-zero sample
        for (int a = 0; a < MLP_IN; ++a) f[a] = (_Float16)0.f;
        for (int a = 0; a < MLP_OUT; ++a) t[a] = 0.f;
        return;
    }
    const int x = (int)(node % p.nx), y = (int)((node / p.nx) % p.ny), z = (int)(node / ((long long)p.nx * p.ny));
    const int e[3] = {m_ex[i], m_ey[i], m_ez[i]};
    double head[7];
    mlp_link_head(p, P[pid], x, y, z, e, head);
    for (int a = 0; a < 7; ++a) f[a] = (_Float16)head[a];
    for (int c = 0; c < MLP_BODY; ++c) f[7 + c] = (_Float16)body[pid * MLP_BODY + c];
    t[0] = (float)l_q[l];
    t[1] = t[2] = t[3] = 0.f;
}

// Closest-point samples, one block scanning the pair slots in order: a
// converged pair (i < j) gets the next sample (block prefix of the flags),
// inputs from body i with the partner's centroid as the query point, target
// outputs 1..3 = the stationary point in body i's frame scaled by
// 1/sqrt(sum k) (output 0 untargeted).
__global__ __launch_bounds__(1024) void k_mlp_collect_contact(Params p, const DevParticle *__restrict__ P,
                                                              const float *__restrict__ body, ContactBufs cb,
                                                              int n_max, _Float16 *__restrict__ feat,
                                                              float *__restrict__ target, Counters *cnt) {
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int np = p.np;
    const long long np2 = (long long)np * np;
    int base = 0;
    for (long long q0 = 0; q0 < np2; q0 += 1024) {
        const long long q = q0 + t;
        int i = 0, j = 0;
        bool ok = false;
        if (q < np2) {
            i = (int)(q / np);
            j = (int)(q - (long long)i * np);
            ok = j > i && cb.pairOk[q];
        }
        int incl = ok ? 1 : 0;
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int wb = 0, tot = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < wv) wb += wsum[k];
            tot += wsum[k];
        }
        const int idx = base + wb + incl - (ok ? 1 : 0);
        if (ok && idx < n_max) {
            _Float16 *f = feat + (long long)idx * MLP_IN;
            float *tg = target + (long long)idx * MLP_OUT;
            double head[7];
            mlp_contact_head(p, P[i], P[j], head);
            for (int a = 0; a < 7; ++a) f[a] = (_Float16)head[a];
            for (int c = 0; c < MLP_BODY; ++c) f[7 + c] = (_Float16)body[i * MLP_BODY + c];
            const int zero[3] = {0, 0, 0};
            double off[7];
            mlp_point_head(p, P[i], cb.pairXm + 3 * q, zero, 1.0, off);
            tg[0] = 0.f;
            for (int a = 0; a < 3; ++a) tg[1 + a] = (float)off[a];
        }
        base += tot;
        __syncthreads();  // wsum is written again
    }
    if (t == 0) cnt->n_collect = min(base, n_max);
}

static int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

void launch_mlp_init(const MlpBlob &b, hipStream_t s) {
    k_mlp_init<<<cdiv(MLP_P, 256), 256, 0, s>>>(b.theta, b.m, b.v, b.w16, b.t);
}

template <typename TA, typename TW>
static void forward_t(const MlpBlob &b, const TA *X, const TW *W, int n, hipStream_t s) {
    TA *h1 = (TA *)b.h1, *h2 = (TA *)b.h2;
    k_mlp_layer<TA, TW><<<cdiv((long long)n * MLP_H, 256), 256, 0, s>>>(X, MLP_IN, W, MLP_OFF_W1, MLP_OFF_B1, MLP_H,
                                                                        n, h1, nullptr);
    k_mlp_layer<TA, TW><<<cdiv((long long)n * MLP_H, 256), 256, 0, s>>>(h1, MLP_H, W, MLP_OFF_W2, MLP_OFF_B2, MLP_H,
                                                                        n, h2, nullptr);
    k_mlp_layer<TA, TW><<<cdiv((long long)n * MLP_OUT, 256), 256, 0, s>>>(h2, MLP_H, W, MLP_OFF_W3, MLP_OFF_B3,
                                                                          MLP_OUT, n, nullptr, b.out);
}

// Forward pass of 32 samples per block with the matrix-core hidden layers
// (the link solver's form): outputs [n][4] into out.
// Wave inference: each wave loads the network once and takes tiles of 32
// samples (grid stride).
__global__ __launch_bounds__(256) void k_mlp_forward_mfma(const _Float16 *__restrict__ X,
                                                          const _Float16 *__restrict__ w, int n,
                                                          float *__restrict__ out) {
    const int lane = threadIdx.x & 63, s = lane & 31, h = lane >> 5;
    const int wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), nw = gridDim.x * (blockDim.x >> 6);
    if (wv * 32 >= n) return;  // wave-uniform; no block barrier in this kernel
    MlpWave W;
    mlp_wave_load(W, w);
    _Float16 w3[MLP_OUT][32];
    float b3[MLP_OUT];
#pragma unroll
    for (int o = 0; o < MLP_OUT; ++o) {
        mlp_wave_load_out(w3[o], w, o);
        b3[o] = (float)w[MLP_OFF_B3 + o];
    }
    for (int r0 = wv * 32; r0 < n; r0 += nw * 32) {
        const int r = r0 + s;
        const bool ok = r < n;
        const _Float16 *xr = X + (long long)(ok ? r : 0) * MLP_IN;
        mlp_h8 x[MLP_S1];
#pragma unroll
        for (int m = 0; m < MLP_S1; ++m)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = mlp_l1_input(2 * m + h, e);
                const _Float16 v = xr[k >= 0 ? k : 0];
                x[m][e] = k >= 0 ? (ok ? v : (_Float16)0.f) : (k == -1 ? (_Float16)1.f : (_Float16)0.f);
            }
        float z[MLP_OUT];
        mlp_wave_forward<MLP_OUT>(W, x, w3, b3, z);
#pragma unroll
        for (int o = 0; o < MLP_OUT; ++o)
            if (ok && h == (o & 1)) out[(long long)r * MLP_OUT + o] = z[o];
    }
}

void launch_mlp_forward(const MlpBlob &b, const void *X, int n, int precision, hipStream_t s) {
    if (precision == 1) forward_t<float, float>(b, (const float *)X, b.theta, n, s);
    else if (precision == 2) {
        if (n > 0) k_mlp_forward_mfma<<<min(cdiv(n, 128), 1024), 256, 0, s>>>((const _Float16 *)X, b.w16, n, b.out);
    } else forward_t<_Float16, _Float16>(b, (const _Float16 *)X, b.w16, n, s);
}

template <typename TA>
static void bwd_weight(const MlpBlob &b, const TA *Hin, int K, const float *dZ, int N, int n, int offW, int offB,
                       hipStream_t s) {
    k_mlp_bwd_weight_part<TA><<<cdiv((long long)MLP_SLICES * (K + 1) * N, 256), 256, 0, s>>>(Hin, K, dZ, N, n,
                                                                                            b.part);
    k_mlp_bwd_weight_sum<<<cdiv((K + 1) * N, 256), 256, 0, s>>>(b.part, K, N, b.g, offW, offB);
}

template <typename TA, typename TW>
static void grad_t(const MlpBlob &b, const TA *X, const TW *W, const float *T, int n, hipStream_t s) {
    forward_t<TA, TW>(b, X, W, n, s);
    const TA *h1 = (const TA *)b.h1, *h2 = (const TA *)b.h2;
    float *sq = b.dz1;  // squared errors, consumed before dz1 is written
    k_mlp_out_grad<TA><<<cdiv((long long)n * MLP_OUT, 256), 256, 0, s>>>(X, b.out, T, n, b.dout, sq);
    k_mlp_loss<<<1, 256, 0, s>>>(sq, n * MLP_OUT, n, b.loss);
    bwd_weight<TA>(b, h2, MLP_H, b.dout, MLP_OUT, n, MLP_OFF_W3, MLP_OFF_B3, s);
    k_mlp_bwd_data<TA, TW><<<cdiv((long long)n * MLP_H, 256), 256, 0, s>>>(b.dout, MLP_OUT, W, MLP_OFF_W3, MLP_H,
                                                                           h2, n, b.dz2);
    bwd_weight<TA>(b, h1, MLP_H, b.dz2, MLP_H, n, MLP_OFF_W2, MLP_OFF_B2, s);
    k_mlp_bwd_data<TA, TW><<<cdiv((long long)n * MLP_H, 256), 256, 0, s>>>(b.dz2, MLP_H, W, MLP_OFF_W2, MLP_H, h1,
                                                                           n, b.dz1);
    bwd_weight<TA>(b, X, MLP_IN, b.dz1, MLP_H, n, MLP_OFF_W1, MLP_OFF_B1, s);
}

void launch_mlp_loss_grad(const MlpBlob &b, const void *X, const float *T, int n, int precision, hipStream_t s) {
    if (precision == 1) grad_t<float, float>(b, (const float *)X, b.theta, T, n, s);
    else grad_t<_Float16, _Float16>(b, (const _Float16 *)X, b.w16, T, n, s);
}

void launch_mlp_adam(const MlpBlob &b, float lr, float beta1, float beta2, float eps, float bc1, float bc2,
                     hipStream_t s) {
    k_mlp_adam<<<cdiv(MLP_P, 256), 256, 0, s>>>(b.theta, b.g, b.m, b.v, b.w16, lr, beta1, beta2, eps, bc1, bc2);
}

void launch_mlp_collect_contact(const Params &p, const DevParticle *P, const float *body, const ContactBufs &cb,
                                int n_max, _Float16 *feat, float *target, Counters *cnt, hipStream_t s) {
    k_mlp_collect_contact<<<1, 1024, 0, s>>>(p, P, body, cb, n_max, feat, target, cnt);
}

void launch_mlp_collect(const Params &p, const DevParticle *P, const float *body, const uint32_t *l_node,
                        const uint32_t *l_do, const double *l_q, int n, _Float16 *feat, float *target,
                        hipStream_t s) {
    if (n > 0) k_mlp_collect<<<cdiv(n, 256), 256, 0, s>>>(p, P, body, l_node, l_do, l_q, n, feat, target);
}

}  // namespace mdl
