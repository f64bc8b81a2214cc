// Warm-start MLP of the link fractions: device-side feature map and the
// one-link inference used by the link solver.  87 inputs -> 64 -> 64 -> 4,
// tanh hidden layers, linear output; FP16 weights and activations, FP32
// accumulation.  Parameter order (P = 10052 values): W1 [87][64], b1 [64],
// W2 [64][64], b2 [64], W3 [64][4], b3 [4]; a layer computes
// z = h_prev W + b.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mdl {

constexpr int MLP_IN = 87, MLP_H = 64, MLP_OUT = 4;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = MLP_IN * MLP_H, MLP_OFF_W2 = MLP_OFF_B1 + MLP_H,
              MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H, MLP_OFF_W3 = MLP_OFF_B2 + MLP_H,
              MLP_OFF_B3 = MLP_OFF_W3 + MLP_H * MLP_OUT, MLP_P = MLP_OFF_B3 + MLP_OUT;
constexpr int MLP_BODY = 4 * MAXCP;  // constant per-body inputs

// Inputs of one link: the fluid node relative to the centroid (minimum image
// on periodic axes) and the direction, both in the body frame, the node
// scaled by 1/sqrt(sum k); the task bit (0: link fraction); then the body's
// constant block (control points sorted by weight, scaled), computed once
// at set-up.  This computes the first 7 entries (e: the link direction
// e_i); the caller appends the body block.
// The first 7 inputs of a query point pt (lab frame) with direction e_i and
// task bit 'task' for body B.
__device__ __forceinline__ void mlp_point_head(const Params &p, const DevParticle &B, const double pt[3],
                                               const int e_i[3], double task, double head[7]) {
    double d[3] = {pt[0] - B.X[0], pt[1] - B.X[1], pt[2] - B.X[2]};
    const int L[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a)
        if ((p.periodic >> a) & 1u) d[a] -= L[a] * floor(d[a] / L[a] + 0.5);
    double K = 0.0;
    for (int c = 0; c < B.n_cp; ++c) K += B.k[c];
    const double inv_s = 1.0 / sqrt(K);
    const double w = B.q[0], qx = B.q[1], qy = B.q[2], qz = B.q[3];
    // body -> lab rotation R; the body frame takes R^T
    const double R[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - w * qz), 2.0 * (qx * qz + w * qy),
                         2.0 * (qx * qy + w * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - w * qx),
                         2.0 * (qx * qz - w * qy), 2.0 * (qy * qz + w * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
    const double e[3] = {(double)e_i[0], (double)e_i[1], (double)e_i[2]};
    for (int a = 0; a < 3; ++a) {
        head[a] = (R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2]) * inv_s;
        head[3 + a] = R[a] * e[0] + R[3 + a] * e[1] + R[6 + a] * e[2];
    }
    head[6] = task;
}

__device__ __forceinline__ void mlp_link_head(const Params &p, const DevParticle &B, int x, int y, int z,
                                              const int e_i[3], double head[7]) {
    const double pt[3] = {(double)x, (double)y, (double)z};
    mlp_point_head(p, B, pt, e_i, 0.0, head);
}

// Closest-point task (task bit 1) of a body pair seen from body Bi: the
// partner's centroid as the query point, no direction.  Outputs 1..3 are
// the pair's stationary point relative to Bi's centroid, in Bi's frame,
// scaled by 1/sqrt(sum k of Bi).
__device__ __forceinline__ void mlp_contact_head(const Params &p, const DevParticle &Bi, const DevParticle &Bj,
                                                 double head[7]) {
    const int zero[3] = {0, 0, 0};
    mlp_point_head(p, Bi, Bj.X, zero, 1.0, head);
}

// Block inference on the matrix cores: the hidden layers of 32 samples at
// once, (32 x 88) x (88 x 64) and (32 x 64) x (64 x 64), as 32 x 32 x 8 FP16
// MFMA tiles with FP32 accumulation (waves 0 and 1 of a 256-thread block
// take the two 32-column halves), tanh on the accumulators, FP16
// activations.  Weights staged in LDS transposed (row = hidden unit, the
// reduction index contiguous), inputs padded to 88 with zeros.
constexpr int MLP_K1 = 88;                    // inputs padded to a multiple of 8
constexpr int MLP_ROW = MLP_K1 + 2 * MLP_H;  // one sample's LDS row: inputs, h1, h2
struct MlpLds {
    _Float16 w1t[MLP_H * MLP_K1];  // [unit][input]
    _Float16 w2t[MLP_H * MLP_H];   // [unit][h1]
    _Float16 b1[MLP_H], b2[MLP_H], w3[MLP_H * MLP_OUT], b3[MLP_OUT];
};

// All threads of the block; the caller synchronises before reading L.
// Global reads in parameter order (coalesced), transposed on the LDS side.
__device__ __forceinline__ void mlp_stage_lds(MlpLds &L, const _Float16 *__restrict__ w) {
    for (int e = threadIdx.x; e < MLP_IN * MLP_H; e += blockDim.x) {
        const int k = e / MLP_H, j = e - k * MLP_H;
        L.w1t[j * MLP_K1 + k] = w[MLP_OFF_W1 + e];
    }
    for (int j = threadIdx.x; j < MLP_H; j += blockDim.x) L.w1t[j * MLP_K1 + MLP_IN] = (_Float16)0.f;
    for (int e = threadIdx.x; e < MLP_H * MLP_H; e += blockDim.x) {
        const int k = e / MLP_H, j = e - k * MLP_H;
        L.w2t[j * MLP_H + k] = w[MLP_OFF_W2 + e];
    }
    for (int e = threadIdx.x; e < MLP_H; e += blockDim.x) {
        L.b1[e] = w[MLP_OFF_B1 + e];
        L.b2[e] = w[MLP_OFF_B2 + e];
    }
    for (int e = threadIdx.x; e < MLP_H * MLP_OUT; e += blockDim.x) L.w3[e] = w[MLP_OFF_W3 + e];
    for (int e = threadIdx.x; e < MLP_OUT; e += blockDim.x) L.b3[e] = w[MLP_OFF_B3 + e];
}

typedef _Float16 mlp_h4 __attribute__((ext_vector_type(4)));
typedef float mlp_f16 __attribute__((ext_vector_type(16)));

// One hidden layer for 32 rows: act[r][out0 + j] = tanh(sum_k act[r][in0 + k]
// wt[j][k] + b[j]), K a multiple of 8.  Waves 0 and 1 (columns 32w..32w+31).
// Operand layout of v_mfma_f32_32x32x8f16: lane l holds A[l % 32][k0 + 4 (l / 32) + e]
// and B[k0 + 4 (l / 32) + e][l % 32], e = 0..3; result register v of lane l is
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
__device__ __forceinline__ void mlp_layer_mfma(_Float16 (*act)[MLP_ROW], int in0, int K, const _Float16 *wt,
                                               const _Float16 *b, int out0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w >= 2) return;
    const int r = lane & 31, kq = (lane >> 5) * 4, j = 32 * w + (lane & 31);
    mlp_f16 acc = {};
    for (int k0 = 0; k0 < K; k0 += 8) {
        const mlp_h4 a = *(const mlp_h4 *)(&act[r][in0 + k0 + kq]);
        const mlp_h4 bb = *(const mlp_h4 *)(&wt[j * K + k0 + kq]);
        acc = __builtin_amdgcn_mfma_f32_32x32x8f16(a, bb, acc, 0, 0, 0);
    }
    const float bj = (float)b[j];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        act[row][out0 + j] = (_Float16)tanhf(acc[v] + bj);
    }
}

// Both hidden layers of the 32 rows of act (inputs in columns 0..86 written
// and synchronised by the caller); all threads of the 256-thread block.
// On return h1 = act[r][MLP_K1 ..], h2 = act[r][MLP_K1 + MLP_H ..] are
// visible to every thread.
__device__ __forceinline__ void mlp_block_hidden(const MlpLds &L, _Float16 (*act)[MLP_ROW]) {
    if (threadIdx.x < 32) act[threadIdx.x][MLP_IN] = (_Float16)0.f;  // the padding input
    __syncthreads();
    mlp_layer_mfma(act, 0, MLP_K1, L.w1t, L.b1, MLP_K1);
    __syncthreads();
    mlp_layer_mfma(act, MLP_K1, MLP_H, L.w2t, L.b2, MLP_K1 + MLP_H);
    __syncthreads();
}

// Output o of row r from h2 (FP32 sum of FP16 products).
__device__ __forceinline__ float mlp_block_output(const MlpLds &L, const _Float16 (*act)[MLP_ROW], int r, int o) {
    float z = (float)L.b3[o];
    for (int k = 0; k < MLP_H; ++k) z += (float)act[r][MLP_K1 + MLP_H + k] * (float)L.w3[k * MLP_OUT + o];
    return z;
}

// The same output split over an aligned group of 8 lanes (lane j of the group
// sums h2 entries 8j .. 8j+7, then a butterfly over the group); every lane of
// the wave calls it, and every lane of the group gets the sum.
__device__ __forceinline__ float mlp_group_output(const MlpLds &L, const _Float16 (*act)[MLP_ROW], int r, int o,
                                                  int j) {
    float z = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
        z += (float)act[r][MLP_K1 + MLP_H + 8 * j + u] * (float)L.w3[(8 * j + u) * MLP_OUT + o];
    z += __shfl_xor(z, 1);
    z += __shfl_xor(z, 2);
    z += __shfl_xor(z, 4);
    return z + (float)L.b3[o];
}

// Training and inference entry points (mlp.hip).  'precision' 0: FP16
// inputs, weights and activations; 1: FP32 throughout (test instantiation);
// 2 (forward only): FP16 with the hidden layers on the matrix cores, the
// form the link solver's warm start uses.
// Workspace for minibatches of at most MLP_MAX_BATCH samples.
constexpr int MLP_MAX_BATCH = 4096;
struct MlpBlob {
    float *theta, *m, *v;  // FP32 master parameters and Adam moments [P]
    _Float16 *w16;         // FP16 copy of the parameters [P]
    long long *t;          // Adam step count
    float *h1, *h2;        // [B][64] activations (FP16 or FP32 storage)
    float *out, *dout;     // [B][4]
    float *dz1, *dz2;      // [B][64]
    float *g;              // [P] gradient
    float *loss;           // [1]
    float *part;           // [16][88][64] weight-gradient slices
};
size_t mlp_blob_bytes();
MlpBlob mlp_blob(void *base);
void launch_mlp_init(const MlpBlob &b, hipStream_t s);  // m = v = 0, t = 0, w16 = theta
void launch_mlp_forward(const MlpBlob &b, const void *X, int n, int precision, hipStream_t s);
void launch_mlp_loss_grad(const MlpBlob &b, const void *X, const float *T, int n, int precision, hipStream_t s);
void launch_mlp_adam(const MlpBlob &b, float lr, float beta1, float beta2, float eps, float bc1, float bc2,
                     hipStream_t s);
void launch_mlp_collect(const Params &p, const DevParticle *P, const float *body, const uint32_t *l_node,
                        const uint32_t *l_do, const double *l_q, int n, _Float16 *feat, float *target,
                        hipStream_t s);
// Closest-point samples of the pairs whose last solve converged (pair order
// i < j, seen from body i), at most n_max; the count goes to cnt->n_collect.
void launch_mlp_collect_contact(const Params &p, const DevParticle *P, const float *body, const ContactBufs &cb,
                                int n_max, _Float16 *feat, float *target, Counters *cnt, hipStream_t s);

}  // namespace mdl
