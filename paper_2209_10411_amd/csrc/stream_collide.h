// Stream-collide of plain fluid nodes: storage forms of the populations,
// the BGK + Guo collision, and the one-system and batched stream-collide
// kernels (the HBM-bound part of a step, kept apart from the boundary
// kernels so that its hardware counters stay tied to this code).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace mdl {

// ------------------------------------------------------------------ storage
template <int S> struct Store;
template <> struct Store<0> {
    using T = float;
    __device__ static float ld(const T *p, long long i, float) { return p[i]; }
    __device__ static void st(T *p, long long i, float v, float) { p[i] = v; }
    __device__ static void st_nt(T *p, long long i, float v, float) { __builtin_nontemporal_store(v, p + i); }
};
template <> struct Store<1> {
    using T = _Float16;
    __device__ static float ld(const T *p, long long i, float inv) { return (float)p[i] * inv; }
    __device__ static void st(T *p, long long i, float v, float s) { p[i] = (_Float16)(v * s); }
    __device__ static void st_nt(T *p, long long i, float v, float s) {
        __builtin_nontemporal_store((_Float16)(v * s), p + i);
    }
};
template <> struct Store<2> {
    using T = uint16_t;
    __device__ static float ld(const T *p, long long i, float) {
        return __uint_as_float((uint32_t)p[i] << 16);
    }
    __device__ static uint16_t rne(float v) {
        uint32_t u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
        return (uint16_t)(u >> 16);
    }
    __device__ static void st(T *p, long long i, float v, float) { p[i] = rne(v); }
    __device__ static void st_nt(T *p, long long i, float v, float) { __builtin_nontemporal_store(rne(v), p + i); }
};

// ------------------------------------------------------------- lattice ops
// BGK + Guo on deviations d_i = f_i - w_i rho0 (FP32).  rho = rho0 + sum d,
// u = (sum e d + F/2)/rho with F = rho g; d+ = d + (deq - d)/tau + F_i.
__device__ __forceinline__ void collide(float d[Q], const Params &p) {
    float dr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        dr += d[i];
        if (EX[i]) jx += EX[i] > 0 ? d[i] : -d[i];
        if (EY[i]) jy += EY[i] > 0 ? d[i] : -d[i];
        if (EZ[i]) jz += EZ[i] > 0 ? d[i] : -d[i];
    }
    const float rho = p.rho0f + dr;
    const float Fx = rho * p.gx, Fy = rho * p.gy, Fz = rho * p.gz;
    const float inv = 1.0f / rho;
    const float ux = (jx + 0.5f * Fx) * inv, uy = (jy + 0.5f * Fy) * inv, uz = (jz + 0.5f * Fz) * inv;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float w = (float)WD[i];
        const float eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        const float eF = EX[i] * Fx + EY[i] * Fy + EZ[i] * Fz;
        const float deq = w * (dr + rho * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
        const float Fi = p.fcoef * w * (3.f * (eF - uF) + 9.f * eu * eF);
        d[i] = d[i] + p.omega * (deq - d[i]) + Fi;
    }
}

// Plain fluid node (skip mask clear: fluid with no solid neighbour at the
// start of the step): pull-stream (periodic wrap, resting halfway walls) and
// collide.  Results are written with non-temporal stores: they are not read
// again within the step.
template <int S>
__device__ __forceinline__ void bulk_update(const Params &p, const typename Store<S>::T *__restrict__ A,
                                            typename Store<S>::T *__restrict__ B, int x, int y, int z, int n) {
    using T = typename Store<S>::T;
    // source coordinates for e = -1, 0, +1 on each axis (wrapped), -1 = wall
    int sx[3], sy[3], sz[3];
    sx[1] = x; sy[1] = y; sz[1] = z;
    sx[2] = x - 1; sx[0] = x + 1;  // index by e + 1: source is x - e
    sy[2] = y - 1; sy[0] = y + 1;
    sz[2] = z - 1; sz[0] = z + 1;
    if (sx[2] < 0) sx[2] = (p.periodic & 1u) ? p.nx - 1 : -1;
    if (sx[0] >= p.nx) sx[0] = (p.periodic & 1u) ? 0 : -1;
    if (sy[2] < 0) sy[2] = (p.periodic & 2u) ? p.ny - 1 : -1;
    if (sy[0] >= p.ny) sy[0] = (p.periodic & 2u) ? 0 : -1;
    if (sz[2] < 0) sz[2] = (p.periodic & 4u) ? p.nz - 1 : -1;
    if (sz[0] >= p.nz) sz[0] = (p.periodic & 4u) ? 0 : -1;
    float d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int xs = sx[EX[i] + 1], ys = sy[EY[i] + 1], zs = sz[EZ[i] + 1];
        const bool wall = (xs | ys | zs) < 0;
        const T *Ai = wall ? A + (long long)OPP[i] * p.Ns : A + (long long)i * p.Ns;
        const int src = wall ? n : (zs * p.ny + ys) * p.nx + xs;
        d[i] = Store<S>::ld(Ai, src, p.inv_scale);
    }
    collide(d, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<S>::st_nt(B + (long long)i * p.Ns, n, d[i], p.scale);
}

// One system: one wave covers 64 consecutive x of one (y, z) row; a block of
// 8 waves takes consecutive rows in lattice order (the hardware spreads
// consecutive blocks over the XCDs).
constexpr int BULK_WAVES = 8;
template <int S>
__global__ __launch_bounds__(64 * BULK_WAVES) void k_bulk(Params p, const typename Store<S>::T *__restrict__ A,
                                                          typename Store<S>::T *__restrict__ B,
                                                          const uint8_t *__restrict__ skip, int nseg) {
    const int wave = blockIdx.x * BULK_WAVES + (threadIdx.x >> 6);
    const int seg = wave % nseg, row = wave / nseg;
    if (row >= p.ny * p.nz) return;
    const int x = seg * 64 + (threadIdx.x & 63);
    if (x >= p.nx) return;
    const int y = row % p.ny, z = row / p.ny;
    const int n = row * p.nx + x;
    if (skip[n]) return;
    bulk_update<S>(p, A, B, x, y, z, n);
}

// An ensemble of systems in one launch: the block table names each block's
// system; within a system a wave covers a tile of 2^tw_log2 consecutive x by
// 64 / 2^tw_log2 rows of y, or (TW_FLAT) 64 consecutive nodes in lattice
// order, which leaves no lane idle whatever nx (the tile shape is chosen per
// system by the autotuner), BW waves per block, tiles in lattice order.
template <int S, int BW>
__global__ __launch_bounds__(64 * BW) void k_bulk_batch(const BulkCase *__restrict__ cases,
                                                        const int *__restrict__ blk_case, int parity) {
    using T = typename Store<S>::T;
    const BulkCase &c = cases[blk_case[blockIdx.x]];
    const int wave = ((int)blockIdx.x - c.first_block) * BW + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    int x, y, z, n;
    if (c.tw_log2 == TW_FLAT) {
        n = wave * 64 + lane;
        if (n >= c.N) return;
        const unsigned row = (unsigned)n / (unsigned)c.nx;
        x = n - (int)row * c.nx;
        z = (int)(row / (unsigned)c.ny);
        y = (int)row - z * c.ny;
    } else {
        const int per_plane = c.nsx * c.nsy;
        z = wave / per_plane;
        if (z >= c.nz) return;
        const int r = wave - z * per_plane;
        const int ty = r / c.nsx, tx = r - ty * c.nsx;
        x = (tx << c.tw_log2) + (lane & ((1 << c.tw_log2) - 1));
        y = ty * (64 >> c.tw_log2) + (lane >> c.tw_log2);
        if (x >= c.nx || y >= c.ny) return;
        n = (z * c.ny + y) * c.nx + x;
    }
    if (c.skip[parity][n]) return;
    Params p;
    p.nx = c.nx; p.ny = c.ny; p.nz = c.nz; p.periodic = c.periodic; p.N = c.N; p.Ns = c.Ns;
    p.rho0f = c.rho0f; p.omega = c.omega; p.fcoef = c.fcoef;
    p.gx = c.gx; p.gy = c.gy; p.gz = c.gz;
    p.scale = c.scale; p.inv_scale = c.inv_scale;
    bulk_update<S>(p, (const T *)c.A[parity], (T *)c.B[parity], x, y, z, n);
}

}  // namespace mdl
