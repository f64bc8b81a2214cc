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

// Training and inference entry points (mlp.hip).  'precision' 0: FP16
// inputs, weights and activations; 1: FP32 throughout (test instantiation).
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
