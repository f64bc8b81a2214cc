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

// c ? a : b without a branch.
__device__ __forceinline__ long long bsel(bool c, long long a, long long b) { return b ^ ((a ^ b) & -(long long)c); }

// 16-bit storage, nx even: a lane takes the node pair (x, x + 1), x even, and
// moves one aligned 32-bit word per population (twice the bytes of a 16-bit
// access per instruction).  The pulls along x shift a pair by one node: the
// missing value comes from the neighbouring lane's word (wave shift by one
// lane) or, where that lane holds no pair of the same row, from one extra
// 16-bit load (the next node, its periodic image, or the node's own opposite
// population at a wall).  Per node the arithmetic is bulk_update's.
// k_bulk_pair (nx a multiple of 128): a wave covers 128 consecutive x of a
// row.  k_bulk_pair_flat (other even nx): a wave covers 64 consecutive pairs
// in lattice order.
template <int S> struct Pair16;
// lo: the value in the low 16 bits of a word (callers shift the high half
// down first); one: a value's 16-bit storage code.
template <> struct Pair16<1> {
    __device__ static float lo(uint32_t w, float inv) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)) * inv;
    }
    __device__ static uint32_t one(float v, float s) {
        return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(v * s));
    }
};
template <> struct Pair16<2> {
    __device__ static float lo(uint32_t w, float) { return __uint_as_float(w << 16); }
    __device__ static uint32_t one(float v, float) { return (uint32_t)Store<2>::rne(v); }
};

template <int S>
__global__ __launch_bounds__(64 * BULK_WAVES) void k_bulk_pair(Params p, const typename Store<S>::T *__restrict__ A,
                                                               typename Store<S>::T *__restrict__ B,
                                                               const uint8_t *__restrict__ skip, int nseg) {
    using T = typename Store<S>::T;
    using W = Pair16<S>;
    // the wave's row and segment are uniform: scalar registers, scalar branches
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * BULK_WAVES + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int seg = wave % nseg, row = wave / nseg;
    if (row >= p.ny * p.nz) return;
    const int x0 = seg * 128 + 2 * lane;
    const bool act = x0 < p.nx;  // the pair exists (nx even: then so does x0 + 1)
    const int xc = act ? x0 : p.nx - 2;  // lanes past the row end read the row's last pair, unused
    const int y = row % p.ny, z = row / p.ny;
    const int n0 = row * p.nx + xc;
    const unsigned sk = act ? (unsigned)*(const uint16_t *)(skip + n0) : 0x0101u;  // 2-byte aligned
    const bool live0 = !(sk & 0xffu), live1 = !(sk >> 8);
    if (!__any(live0 || live1)) return;  // wave-uniform: every lane below takes part in the shifts
    int sy[3], sz[3];
    sy[1] = y; sz[1] = z;
    sy[2] = y - 1; sy[0] = y + 1;
    sz[2] = z - 1; sz[0] = z + 1;
    if (sy[2] < 0) sy[2] = (p.periodic & 2u) ? p.ny - 1 : -1;
    if (sy[0] >= p.ny) sy[0] = (p.periodic & 2u) ? 0 : -1;
    if (sz[2] < 0) sz[2] = (p.periodic & 4u) ? p.nz - 1 : -1;
    if (sz[0] >= p.nz) sz[0] = (p.periodic & 4u) ? 0 : -1;
    const bool perx = p.periodic & 1u;
    const float inv = p.inv_scale;
    const long long Ns = p.Ns;
    const int r0 = row * p.nx;  // this row's first node
    // The only lanes that pull along x from outside their wave's words: lane
    // 0 for e_x = +1 (the node before the segment), and for e_x = -1 lane 63
    // when the row continues past the segment, else the lane of the row's
    // last pair; either way one node per population, at a wave-uniform
    // address (periodic wrap, or the node's own opposite population at a wall).
    const bool more = (seg + 1) * 128 < p.nx;
    const bool edge_lo = lane == 0;
    const bool edge_hi = more ? lane == 63 : xc + 2 >= p.nx;
    // pass 1: every load at once, unconditionally (indices chosen by bitwise
    // selects, which stay selects: a branch here would hold each load back)
    uint32_t w[Q], eb[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ys = sy[EY[i] + 1], zs = sz[EZ[i] + 1];
        const bool rwall = (ys | zs) < 0;  // the source row lies beyond a wall: both nodes bounce
        const long long rb = (long long)(rwall ? 0 : (zs * p.ny + ys) * p.nx);  // source row
        const long long io = OPP[i] * Ns, ii = i * Ns + rb;
        w[i] = *(const uint32_t *)(A + bsel(rwall, io + n0, ii + xc));
        if (EX[i] > 0) {
            const long long e = bsel(seg > 0, ii + seg * 128 - 1, bsel(perx, ii + p.nx - 1, io + r0));
            eb[i] = *(const uint16_t *)(A + bsel(rwall, io + r0, e));
        } else if (EX[i] < 0) {
            const long long e = bsel(more, ii + (seg + 1) * 128, bsel(perx, ii, io + r0 + p.nx - 1));
            eb[i] = *(const uint16_t *)(A + bsel(rwall, io + r0, e));
        }
    }
    // pass 2: the pulls along x from the neighbouring lanes' words
    float d0[Q], d1[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ys = sy[EY[i] + 1], zs = sz[EZ[i] + 1];
        const bool rwall = (ys | zs) < 0;
        uint32_t b0 = w[i] & 0xffffu, b1 = w[i] >> 16;
        if (EX[i] > 0) {
            const uint32_t wl = (uint32_t)__shfl_up((int)w[i], 1);
            const uint32_t s0 = edge_lo ? eb[i] : wl >> 16;
            b1 = rwall ? b1 : b0;
            b0 = rwall ? b0 : s0;
        } else if (EX[i] < 0) {
            const uint32_t wr = (uint32_t)__shfl_down((int)w[i], 1);
            const uint32_t s1 = edge_hi ? eb[i] : wr & 0xffffu;
            b0 = rwall ? b0 : b1;
            b1 = rwall ? b1 : s1;
        }
        d0[i] = W::lo(b0, inv);
        d1[i] = W::lo(b1, inv);
    }
    if (!(live0 || live1)) return;
    collide(d0, p);
    collide(d1, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T *Bi = B + (long long)i * p.Ns;
        const uint32_t v0 = W::one(d0[i], p.scale), v1 = W::one(d1[i], p.scale);
        if (live0 && live1) {
            __builtin_nontemporal_store(v0 | (v1 << 16), (uint32_t *)(Bi + n0));
        } else if (live0) {
            __builtin_nontemporal_store((uint16_t)v0, (uint16_t *)(Bi + n0));
        } else {
            __builtin_nontemporal_store((uint16_t)v1, (uint16_t *)(Bi + n0 + 1));
        }
    }
}

// The same pair update with the pairs in lattice order: a wave takes 64
// consecutive pairs (128 nodes), rows wrap inside the wave, so no lane idles
// whatever the (even) nx.  A lane pulls from the neighbouring lane's word
// when that pair lies in its own row; at a row's ends and at the wave's ends
// it loads the one missing node itself (a per-lane index, loaded by every
// lane so that all loads stay unconditional).
template <int S>
__global__ __launch_bounds__(64 * BULK_WAVES) void k_bulk_pair_flat(Params p,
                                                                    const typename Store<S>::T *__restrict__ A,
                                                                    typename Store<S>::T *__restrict__ B,
                                                                    const uint8_t *__restrict__ skip) {
    using T = typename Store<S>::T;
    using W = Pair16<S>;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * BULK_WAVES + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int N = (int)p.N;  // even (nx even)
    if (wave * 128 >= N) return;  // wave-uniform
    const int nraw = wave * 128 + 2 * lane;
    const bool act = nraw < N;
    const int n0 = act ? nraw : N - 2;  // lanes past the end read the last pair, unused
    const unsigned sk = act ? (unsigned)*(const uint16_t *)(skip + n0) : 0x0101u;  // 2-byte aligned
    const bool live0 = !(sk & 0xffu), live1 = !(sk >> 8);
    if (!__any(live0 || live1)) return;  // wave-uniform: every lane below takes part in the shifts
    const unsigned row = (unsigned)n0 / (unsigned)p.nx;
    const int x0 = n0 - (int)row * p.nx;  // even
    const int z = (int)(row / (unsigned)p.ny), y = (int)row - z * p.ny;
    int sy[3], sz[3];
    sy[1] = y; sz[1] = z;
    sy[2] = y - 1; sy[0] = y + 1;
    sz[2] = z - 1; sz[0] = z + 1;
    if (sy[2] < 0) sy[2] = (p.periodic & 2u) ? p.ny - 1 : -1;
    if (sy[0] >= p.ny) sy[0] = (p.periodic & 2u) ? 0 : -1;
    if (sz[2] < 0) sz[2] = (p.periodic & 4u) ? p.nz - 1 : -1;
    if (sz[0] >= p.nz) sz[0] = (p.periodic & 4u) ? 0 : -1;
    const bool perx = p.periodic & 1u;
    const float inv = p.inv_scale;
    const long long Ns = p.Ns;
    // x0 - 1 is outside the lane-below's word at a row start or in lane 0;
    // x0 + 2 outside the lane-above's word at a row end or in lane 63
    const bool edge_lo = lane == 0 || x0 == 0;
    const bool edge_hi = lane == 63 || x0 + 2 >= p.nx;
    uint32_t w[Q], eb[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ys = sy[EY[i] + 1], zs = sz[EZ[i] + 1];
        const bool rwall = (ys | zs) < 0;  // the source row lies beyond a wall: both nodes bounce
        const long long rb = (long long)(rwall ? 0 : (zs * p.ny + ys) * p.nx);
        const long long io = OPP[i] * Ns, ii = i * Ns + rb;
        const long long wi = bsel(rwall, io + n0, ii + x0);
        w[i] = *(const uint32_t *)(A + wi);
        if (EX[i] > 0) {
            const long long e = bsel(x0 > 0, ii + x0 - 1, bsel(perx, ii + p.nx - 1, io + n0));
            eb[i] = *(const uint16_t *)(A + bsel(edge_lo && !rwall, e, wi));
        } else if (EX[i] < 0) {
            const long long e = bsel(x0 + 2 < p.nx, ii + x0 + 2, bsel(perx, ii, io + n0 + 1));
            eb[i] = *(const uint16_t *)(A + bsel(edge_hi && !rwall, e, wi));
        }
    }
    float d0[Q], d1[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ys = sy[EY[i] + 1], zs = sz[EZ[i] + 1];
        const bool rwall = (ys | zs) < 0;
        uint32_t b0 = w[i] & 0xffffu, b1 = w[i] >> 16;
        if (EX[i] > 0) {
            const uint32_t wl = (uint32_t)__shfl_up((int)w[i], 1);
            const uint32_t s0 = edge_lo ? eb[i] : wl >> 16;
            b1 = rwall ? b1 : b0;
            b0 = rwall ? b0 : s0;
        } else if (EX[i] < 0) {
            const uint32_t wr = (uint32_t)__shfl_down((int)w[i], 1);
            const uint32_t s1 = edge_hi ? eb[i] : wr & 0xffffu;
            b0 = rwall ? b0 : b1;
            b1 = rwall ? b1 : s1;
        }
        d0[i] = W::lo(b0, inv);
        d1[i] = W::lo(b1, inv);
    }
    if (!(live0 || live1)) return;
    collide(d0, p);
    collide(d1, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T *Bi = B + (long long)i * p.Ns;
        const uint32_t v0 = W::one(d0[i], p.scale), v1 = W::one(d1[i], p.scale);
        if (live0 && live1) {
            __builtin_nontemporal_store(v0 | (v1 << 16), (uint32_t *)(Bi + n0));
        } else if (live0) {
            __builtin_nontemporal_store((uint16_t)v0, (uint16_t *)(Bi + n0));
        } else {
            __builtin_nontemporal_store((uint16_t)v1, (uint16_t *)(Bi + n0 + 1));
        }
    }
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
