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
// Divergence sentinel: a fluid node whose velocity exceeds 0.3 lattice units
// (Mach 0.52), or whose moments are not finite, marks the context as
// diverged (ERR_FLUID; reported by the next synchronising call).
constexpr float U_MAX_SQ = 0.09f;

// Moments of the (possibly scaled) deviations and the BGK + Guo increments.
// rho = rho0 + sum d, u = (sum e d + F/2)/rho with F = rho g; the update
// d+ = d + (deq - d)/tau + F_i is evaluated per pair of opposite directions
// (i, ib) as d+_i = (1 - 1/tau) d_i + S + A, d+_ib = (1 - 1/tau) d_ib + S - A,
// with S the part of 1/tau deq_i + F_i even in e_i and A the odd part:
//   S = w [1/tau (dr + 4.5 rho (e.u)^2 - 1.5 rho u.u) + (1 - 1/2tau)(9 (e.u)(e.F) - 3 u.F)]
//   A = w [3/tau rho (e.u) + 3 (1 - 1/2tau) e.F]
// SCALED: the stored values are s d (s = p.scale, a power of two, so every
// scaling is exact): the moments are taken times 1/s and the increments
// applied times s, which leaves the same bits as scaling each value.
// Returns true when the node trips the sentinel (the comparison is false for
// a NaN, so non-finite moments trip it too).
template <bool SCALED = false>
__device__ __forceinline__ bool collide(float d[Q], const Params &p) {
    float sp[Q], dp[Q];
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        sp[i] = d[i] + d[i + 1];
        dp[i] = d[i] - d[i + 1];
    }
    float dr = d[0];
#pragma unroll
    for (int i = 1; i < Q; i += 2) dr += sp[i];
    float jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        if (EX[i]) jx += EX[i] > 0 ? dp[i] : -dp[i];
        if (EY[i]) jy += EY[i] > 0 ? dp[i] : -dp[i];
        if (EZ[i]) jz += EZ[i] > 0 ? dp[i] : -dp[i];
    }
    if (SCALED) {
        dr *= p.inv_scale;
        jx *= p.inv_scale;
        jy *= p.inv_scale;
        jz *= p.inv_scale;
    }
    const float rho = p.rho0f + dr;
    const float Fx = rho * p.gx, Fy = rho * p.gy, Fz = rho * p.gz;
    const float inv = __builtin_amdgcn_rcpf(rho);  // hardware reciprocal (1 ulp)
    const float ux = (jx + 0.5f * Fx) * inv, uy = (jy + 0.5f * Fy) * inv, uz = (jz + 0.5f * Fz) * inv;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
    const float om = p.omega, omc = 1.f - om;
    const float sc = SCALED ? p.scale : 1.f;
    const float g = sc * (om * (dr - 1.5f * rho * uu) - 3.f * p.fcoef * uF);
    const float r45 = sc * (4.5f * om * rho), r3 = sc * (3.f * om * rho);
    const float f9 = sc * (9.f * p.fcoef), f3 = sc * (3.f * p.fcoef);
    d[0] = omc * d[0] + (float)WD[0] * g;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const float w = (float)WD[i];
        const float eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        const float eF = EX[i] * Fx + EY[i] * Fy + EZ[i] * Fz;
        const float T = (w * r45) * eu + (w * f9) * eF;
        const float S = eu * T + w * g;
        const float A = (w * r3) * eu + (w * f3) * eF;
        d[i] = omc * d[i] + (S + A);
        d[i + 1] = omc * d[i + 1] + (S - A);
    }
    return !(uu <= U_MAX_SQ);
}

// Plain fluid node at (x, y, z), any layout of the launch (skip mask clear:
// fluid with no solid neighbour at the start of the step): pull-stream
// (periodic wrap, resting halfway walls) and collide; 64-bit offsets.
// Results are written with non-temporal stores: they are not read again
// within the step.
template <int S>
__device__ __forceinline__ bool bulk_update(const Params &p, const typename Store<S>::T *__restrict__ A,
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
        d[i] = Store<S>::ld(A, wall ? pidx(n, OPP[i]) : pidx((long long)(zs * p.ny + ys) * p.nx + xs, i),
                            p.inv_scale);
    }
    const bool bad = collide(d, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<S>::st_nt(B, pidx(n, i), d[i], p.scale);
    return bad;
}

// Waves per block of the one-system stream-collide kernels.
constexpr int BULK_WAVES = 4;

// Whether the short forms apply: every element offset into the population
// buffer, in bytes, fits 32 bits.
inline bool bulk_offsets_fit(const Params &p, int storage_bytes) {
    return (unsigned long long)Q * (unsigned long long)p.Ns * (unsigned long long)storage_bytes < (1ull << 32);
}

// One system, one node per lane (FP32; 16-bit storage with odd nx): a wave
// covers 64 consecutive x of one (y, z) row, so the source row of each
// population, and whether it lies beyond a wall, is wave-uniform (scalar);
// per lane only x and its two neighbours (wrapped, or the node's own opposite
// population at a resting wall).  Offsets are 32-bit (bulk_offsets_fit; the
// launcher takes k_bulk_wide otherwise).  Blocks take consecutive rows in
// lattice order (the hardware spreads consecutive blocks over the XCDs).
template <int S>
__global__ __launch_bounds__(64 * BULK_WAVES) void k_bulk(Params p, const typename Store<S>::T *__restrict__ A,
                                                          typename Store<S>::T *__restrict__ B,
                                                          const uint8_t *__restrict__ skip, int nseg,
                                                          int *__restrict__ err) {
    using T = typename Store<S>::T;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * BULK_WAVES + (threadIdx.x >> 6));
    const int seg = wave % nseg, row = wave / nseg;
    if (row >= p.ny * p.nz) return;
    const int x = seg * 64 + (threadIdx.x & 63);
    if (x >= p.nx) return;
    const int y = row % p.ny, z = row / p.ny;
    const uint32_t n = (uint32_t)(row * p.nx + x);
    if (skip[n]) return;
    int sy[3], sz[3];  // source rows (uniform) by e + 1; -1 = beyond a wall
    sy[1] = y; sz[1] = z;
    sy[2] = y - 1; sy[0] = y + 1;
    sz[2] = z - 1; sz[0] = z + 1;
    if (sy[2] < 0) sy[2] = (p.periodic & 2u) ? p.ny - 1 : -1;
    if (sy[0] >= p.ny) sy[0] = (p.periodic & 2u) ? 0 : -1;
    if (sz[2] < 0) sz[2] = (p.periodic & 4u) ? p.nz - 1 : -1;
    if (sz[0] >= p.nz) sz[0] = (p.periodic & 4u) ? 0 : -1;
    int xm = x - 1, xp = x + 1;  // sources for e_x = +1 and -1; -1 = wall
    if (xm < 0) xm = (p.periodic & 1u) ? p.nx - 1 : -1;
    if (xp >= p.nx) xp = (p.periodic & 1u) ? 0 : -1;
    const char *Ab = (const char *)A;
    float d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ys = sy[EY[i] + 1], zs = sz[EZ[i] + 1];
        const bool rwall = (ys | zs) < 0;  // uniform: the node's own opposite population
        const uint32_t rb = (uint32_t)((zs * p.ny + ys) * p.nx);  // source row (uniform)
        uint32_t off;
        if (rwall) {
            off = pidx32(n, OPP[i]);
        } else if (EX[i] == 0) {
            off = pidx32(rb + (uint32_t)x, i);
        } else {
            const int xs = EX[i] > 0 ? xm : xp;
            off = xs < 0 ? pidx32(n, OPP[i]) : pidx32(rb + (uint32_t)xs, i);
        }
        d[i] = Store<S>::ld((const T *)(Ab + off * (uint32_t)sizeof(T)), 0, p.inv_scale);
    }
    const bool bad = collide(d, p);
    char *Bb = (char *)B;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        Store<S>::st_nt((T *)(Bb + pidx32(n, i) * (uint32_t)sizeof(T)), 0, d[i], p.scale);
    if (bad) atomicOr(err, ERR_FLUID);
}

// The same launch shape with 64-bit offsets (lattices whose population
// buffer exceeds 4 GiB).
template <int S>
__global__ __launch_bounds__(64 * BULK_WAVES) void k_bulk_wide(Params p, const typename Store<S>::T *__restrict__ A,
                                                               typename Store<S>::T *__restrict__ B,
                                                               const uint8_t *__restrict__ skip, int nseg,
                                                               int *__restrict__ err) {
    const int wave = blockIdx.x * BULK_WAVES + (threadIdx.x >> 6);
    const int seg = wave % nseg, row = wave / nseg;
    if (row >= p.ny * p.nz) return;
    const int x = seg * 64 + (threadIdx.x & 63);
    if (x >= p.nx) return;
    const int y = row % p.ny, z = row / p.ny;
    const long long n = (long long)row * p.nx + x;
    if (skip[n]) return;
    if (bulk_update<S>(p, A, B, x, y, z, (int)n)) atomicOr(err, ERR_FLUID);
}

// Rows whose length is not a multiple of 64 (the row form would leave the
// last wave of every row partly idle: a third of it for nx = 160): a wave
// takes 64 consecutive nodes in lattice order, rows wrapping inside it, and
// each lane finds its own row.  Offsets as in bulk_update (node index below
// 2^31).
template <int S>
__global__ __launch_bounds__(64 * BULK_WAVES) void k_bulk_flat(Params p, const typename Store<S>::T *__restrict__ A,
                                                               typename Store<S>::T *__restrict__ B,
                                                               const uint8_t *__restrict__ skip,
                                                               int *__restrict__ err) {
    const uint32_t n = (blockIdx.x * (uint32_t)BULK_WAVES + (threadIdx.x >> 6)) * 64u + (threadIdx.x & 63);
    if (n >= (uint32_t)p.N || skip[n]) return;
    const uint32_t row = n / (uint32_t)p.nx;
    const int x = (int)(n - row * (uint32_t)p.nx);
    const int z = (int)(row / (uint32_t)p.ny), y = (int)row - z * p.ny;
    if (bulk_update<S>(p, A, B, x, y, z, (int)n)) atomicOr(err, ERR_FLUID);
}

// 16-bit storage, nx even: a lane takes the node pair (n0, n0 + 1), n0 even,
// and moves one 32-bit word per population (twice the bytes of a 16-bit
// access per instruction); a wave covers 64 consecutive pairs in lattice
// order, rows wrapping inside the wave, so no lane idles whatever nx.
// Fast path (every lane of the wave in a row whose y and z neighbours are
// inside the box, and not across a periodic seam): a lane loads, for every
// population i, the aligned 32-bit word of its own pair (x0, x0 + 1) in the
// source row (node n0 - e_y nx - e_z nx ny; a pair never straddles a run of
// the population layout).  An x-shifted
// population takes one of its two values from the neighbouring lane's word
// (lane - 1's high half for e_x = +1, lane + 1's low half for e_x = -1), moved
// across the wave by DPP, so every load covers whole cache lines.  Where that
// neighbour is not the right one (the first and last lanes of the wave, a
// row's ends: the periodic image in the same row, or the node's own opposite
// population at a resting wall) the value comes from one 16-bit load per
// x-shifted population, issued by every lane (at the word's own address
// where no fix is needed) so that all loads stay unconditional.  Other waves:
// every source by its coordinates.  The collision runs on the scaled stored
// values (collide<SCALED>).
template <int S> __device__ __forceinline__ float raw16(uint32_t b) {  // low 16 bits -> stored value, unscaled
    if constexpr (S == 1) return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
    else return __uint_as_float(b << 16);
}
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
template <int S> __device__ __forceinline__ uint32_t pack16(float a, float b) {  // RNE to two 16-bit codes
    const f32x2 v = {a, b};
    if constexpr (S == 1) return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
    else return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// DPP controls (gfx9 family): every lane takes the value of lane - 1
// (wave_shr:1) or lane + 1 (wave_shl:1); lanes without a source keep the
// given old value.
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;

template <int S>
__global__ __launch_bounds__(64 * BULK_WAVES) void k_bulk_pair(Params p, const typename Store<S>::T *__restrict__ A,
                                                               typename Store<S>::T *__restrict__ B,
                                                               const uint8_t *__restrict__ skip,
                                                               int *__restrict__ err) {
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * BULK_WAVES + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const uint32_t N = (uint32_t)p.N;  // even (nx even)
    if ((uint32_t)wave * 128u >= N) return;  // wave-uniform
    const uint32_t nraw = (uint32_t)wave * 128u + 2u * lane;
    const bool act = nraw < N;
    const uint32_t n0 = act ? nraw : N - 2;  // lanes past the end read the last pair, unused
    const unsigned sk = act ? (unsigned)*(const uint16_t *)(skip + n0) : 0x0101u;  // 2-byte aligned
    const bool live0 = !(sk & 0xffu), live1 = !(sk >> 8);
    if (!__any(live0 || live1)) return;
    const uint32_t row = n0 / (uint32_t)p.nx;
    const int x0 = (int)(n0 - row * (uint32_t)p.nx);  // even
    const int z = (int)(row / (uint32_t)p.ny), y = (int)row - z * p.ny;
    const int nx = p.nx, nxy = p.nx * p.ny;
    const bool interior = y >= 1 && y <= p.ny - 2 && z >= 1 && z <= p.nz - 2;
    const char *Ab = (const char *)A;
    float d0[Q], d1[Q];
    if (__all(interior)) {
        const bool perx = p.periodic & 1u;
        const bool lo_edge = x0 == 0, hi_edge = x0 + 2 == nx;
        // lanes whose x-shifted value lies outside the pair word of their
        // neighbour lane: the row's ends, and the wave's first and last lanes
        const bool lo_fix = lo_edge || lane == 0, hi_fix = hi_edge || lane == 63;
        uint32_t w[Q], fx[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            // the source row's pair (x0, x0 + 1): an even node, so both lie in one run
            const uint32_t ms = n0 - (uint32_t)(EY[i] * nx) - (uint32_t)(EZ[i] * nxy);
            w[i] = *(const uint32_t *)(Ab + 2u * pidx32(ms, i));
            if (EX[i] > 0) {  // node 0 pulls x0 - 1
                const uint32_t f = !lo_fix ? pidx32(ms, i)
                                   : !lo_edge ? pidx32(ms - 1u, i)
                                   : perx ? pidx32(ms + (uint32_t)(nx - 1), i) : pidx32(n0, OPP[i]);
                fx[i] = *(const uint16_t *)(Ab + 2u * f);
            } else if (EX[i] < 0) {  // node 1 pulls x0 + 2
                const uint32_t f = !hi_fix ? pidx32(ms, i)
                                   : !hi_edge ? pidx32(ms + 2u, i)
                                   : perx ? pidx32(ms + 2u - (uint32_t)nx, i) : pidx32(n0 + 1u, OPP[i]);
                fx[i] = *(const uint16_t *)(Ab + 2u * f);
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            uint32_t b0 = w[i], b1 = w[i] >> 16;
            if (EX[i] > 0) {  // (x0 - 1, x0): the neighbour lane's high half, then the own low half
                const uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w[i], DPP_WAVE_SHR1, 0xf, 0xf, false);
                b0 = lo_fix ? fx[i] : prev >> 16;
                b1 = w[i];
            } else if (EX[i] < 0) {  // (x0 + 1, x0 + 2): the own high half, then the neighbour lane's low half
                const uint32_t next = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w[i], DPP_WAVE_SHL1, 0xf, 0xf, false);
                b0 = w[i] >> 16;
                b1 = hi_fix ? fx[i] : next;
            }
            d0[i] = raw16<S>(b0);
            d1[i] = raw16<S>(b1);
        }
    } else {
        int sx[3][2], sy[3], sz[3];
        sy[1] = y; sz[1] = z;
        sy[2] = y - 1; sy[0] = y + 1;
        sz[2] = z - 1; sz[0] = z + 1;
        if (sy[2] < 0) sy[2] = (p.periodic & 2u) ? p.ny - 1 : -1;
        if (sy[0] >= p.ny) sy[0] = (p.periodic & 2u) ? 0 : -1;
        if (sz[2] < 0) sz[2] = (p.periodic & 4u) ? p.nz - 1 : -1;
        if (sz[0] >= p.nz) sz[0] = (p.periodic & 4u) ? 0 : -1;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int x = x0 + k;
            sx[1][k] = x;
            sx[2][k] = x - 1 < 0 ? ((p.periodic & 1u) ? nx - 1 : -1) : x - 1;
            sx[0][k] = x + 1 >= nx ? ((p.periodic & 1u) ? 0 : -1) : x + 1;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ys = sy[EY[i] + 1], zs = sz[EZ[i] + 1];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int xs = sx[EX[i] + 1][k];
                const bool wall = (xs | ys | zs) < 0;
                const uint32_t off = wall ? pidx32(n0 + (uint32_t)k, OPP[i])
                                          : pidx32((uint32_t)((zs * p.ny + ys) * nx + xs), i);
                const float v = raw16<S>((uint32_t)*(const uint16_t *)(Ab + off * 2u));
                if (k == 0) d0[i] = v;
                else d1[i] = v;
            }
        }
    }
    if (!(live0 || live1)) return;
    const bool bad0 = collide<S == 1>(d0, p), bad1 = collide<S == 1>(d1, p);
    char *Bb = (char *)B;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t v = pack16<S>(d0[i], d1[i]);
        char *q = Bb + 2u * pidx32(n0, i);
        if (live0 && live1) __builtin_nontemporal_store(v, (uint32_t *)q);
        else if (live0) __builtin_nontemporal_store((uint16_t)(v & 0xffffu), (uint16_t *)q);
        else __builtin_nontemporal_store((uint16_t)(v >> 16), (uint16_t *)(q + 2));
    }
    if ((bad0 && live0) || (bad1 && live1)) atomicOr(err, ERR_FLUID);
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
    if (bulk_update<S>(p, (const T *)c.A[parity], (T *)c.B[parity], x, y, z, n)) atomicOr(c.err, ERR_FLUID);
}

}  // namespace mdl
