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
    const double inv_s = B.rsk;
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

// Wave inference on the matrix cores: 32 samples per wave, every operand in
// registers.  With the transposed product Z^T = W^T X^T the weights are the A
// operands of v_mfma_f32_32x32x16_f16 (loaded once per wave and kept) and
// the samples the B operands; a 32 x 32 tile of units x samples per MFMA
// chain, FP32 accumulation, tanh on the accumulators, FP16 activations.
// Operand layout (32 x 32 x 16): lane l holds A[l % 32][8 (l / 32) + e] and
// B[8 (l / 32) + e][l % 32], e = 0..7; result register v of lane l is
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].  So lane l holds, for sample
// l % 32, sixteen units of each 32-unit tile, and those are the B operands
// of the next layer once its contraction index follows the same order
// (mlp_l2_unit); no activation leaves the registers.
// The order of a contraction is free, so layer 1 takes its inputs in chunks
// of 8 that a lane loads whole: chunk c = 2 m + h fills the slots of step m,
// lane half h: chunk 0 = inputs 0..6 and a constant 1 (carries b1), chunks
// 1..10 = the body block (inputs 7 + 8 (c - 1) + e), chunk 11 = zeros.
// Layer 2 takes b2 on a constant 1 in a fifth step.
constexpr int MLP_S1 = 6;  // K steps of layer 1 (12 chunks of 8)
constexpr int MLP_S2 = 5;  // K steps of layer 2: 64 units, then 1 and zeros
typedef _Float16 mlp_h8 __attribute__((ext_vector_type(8)));
typedef float mlp_f16 __attribute__((ext_vector_type(16)));

struct MlpWave {
    mlp_h8 w1[2][MLP_S1];  // A operands: tile t (units 32t..32t+31), step m
    mlp_h8 w2[2][MLP_S2];
};

// Input in slot e of chunk c (-1: the constant 1, -2: zero).
__device__ __forceinline__ int mlp_l1_input(int c, int e) {
    return c == 0 ? (e < 7 ? e : -1) : (c <= 10 ? 7 + 8 * (c - 1) + e : -2);
}
// Unit of layer 1 in slot e of layer-2 step m for lane half h: registers
// 8 (m % 2) + e of layer 1's tile m / 2.
__device__ __forceinline__ int mlp_l2_unit(int m, int h, int e) {
    return 32 * (m >> 1) + 16 * (m & 1) + 8 * (e >> 2) + 4 * h + (e & 3);
}
// Unit in register v of tile t of a layer's result, lane half h.
__device__ __forceinline__ int mlp_out_unit(int t, int v, int h) { return 32 * t + 8 * (v >> 2) + 4 * h + (v & 3); }

// tanh as 1 - 2 / (1 + e^(2x)) on the hardware exp2 and reciprocal (a few
// ulp of FP32 away from tanhf, below the FP16 rounding that follows).
__device__ __forceinline__ float mlp_tanh(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 / ln 2
    return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + e);
}

// The calling wave's A operands from the parameters w (FP16, parameter order).
__device__ __forceinline__ void mlp_wave_load(MlpWave &W, const _Float16 *__restrict__ w) {
    const int lane = threadIdx.x & 63, jl = lane & 31, h = lane >> 5;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int j = 32 * t + jl;
#pragma unroll
        for (int m = 0; m < MLP_S1; ++m)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = mlp_l1_input(2 * m + h, e);
                W.w1[t][m][e] = k >= 0 ? w[MLP_OFF_W1 + k * MLP_H + j]
                                       : (k == -1 ? w[MLP_OFF_B1 + j] : (_Float16)0.f);
            }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int e = 0; e < 8; ++e) W.w2[t][m][e] = w[MLP_OFF_W2 + mlp_l2_unit(m, h, e) * MLP_H + j];
#pragma unroll
        for (int e = 0; e < 8; ++e) W.w2[t][4][e] = (h == 0 && e == 0) ? w[MLP_OFF_B2 + j] : (_Float16)0.f;
    }
}

// Output o's weights of the lane's 32 units (tile t, register v at 16 t + v).
__device__ __forceinline__ void mlp_wave_load_out(_Float16 w3[32], const _Float16 *__restrict__ w, int o) {
    const int h = (threadIdx.x & 63) >> 5;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) w3[16 * t + v] = w[MLP_OFF_W3 + mlp_out_unit(t, v, h) * MLP_OUT + o];
}

// Both hidden layers of the wave's 32 samples and NO outputs.  x: the B
// operands of layer 1 (lane l: chunk 2 m + l / 32 of sample l % 32 in step
// m); w3[o]: mlp_wave_load_out's weights of output o, b3[o] its bias.  Every
// lane of the wave calls it; both lanes of a sample get its outputs.
// Activations are rounded to FP16 as stored ones are.
template <int NO>
__device__ __forceinline__ void mlp_wave_forward(const MlpWave &W, const mlp_h8 x[MLP_S1], const _Float16 (*w3)[32],
                                                 const float *b3, float out[NO]) {
    const int h = (threadIdx.x & 63) >> 5;
    mlp_f16 a0 = {}, a1 = {};
#pragma unroll
    for (int m = 0; m < MLP_S1; ++m) {
        a0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(W.w1[0][m], x[m], a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(W.w1[1][m], x[m], a1, 0, 0, 0);
    }
    mlp_h8 y[MLP_S2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int e = 0; e < 8; ++e) y[m][e] = (_Float16)mlp_tanh((m < 2 ? a0 : a1)[8 * (m & 1) + e]);
#pragma unroll
    for (int e = 0; e < 8; ++e) y[4][e] = (h == 0 && e == 0) ? (_Float16)1.f : (_Float16)0.f;
    a0 = mlp_f16{};
    a1 = mlp_f16{};
#pragma unroll
    for (int m = 0; m < MLP_S2; ++m) {
        a0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(W.w2[0][m], y[m], a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(W.w2[1][m], y[m], a1, 0, 0, 0);
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) out[o] = 0.f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const float y0 = (float)(_Float16)mlp_tanh(a0[v]), y1 = (float)(_Float16)mlp_tanh(a1[v]);
#pragma unroll
        for (int o = 0; o < NO; ++o) out[o] += y0 * (float)w3[o][v] + y1 * (float)w3[o][16 + v];
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) out[o] += __shfl_xor(out[o], 32) + b3[o];
}

// Training and inference entry points (mlp.hip).  'precision' 0: FP16
// inputs, weights and activations; 1: FP32 throughout (test instantiation);
// 2 (forward only): FP16 with the hidden layers on the matrix cores (the
// wave inference above, the form of the link solver's warm start).
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
