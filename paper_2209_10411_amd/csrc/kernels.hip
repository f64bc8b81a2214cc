// HIP kernels of the coupled metaball / lattice Boltzmann step for CDNA4
// (gfx950).  The paper (arXiv 2209.10411) defines the operations; the GPU
// organisation is this library's own:
//   k_links          one thread per cut link: bounce-back value (simple or the
//                    paper's interpolated rule, sec. 2.3.2 Eqs. eqneq1-neqd)
//                    and the link's momentum exchange in FP64
//   k_reduce         one block per particle: fixed-order FP64 sum of the link
//                    momenta and, without contact, the body's rigid-body
//                    update (sec. 2.3.1)
//   k_rigid          one block (contact): sphero-metaball contacts and the
//                    Newton-Euler update of all particles over the sub-steps
//   k_region_*       per-particle cubes in 8x8x4 tiles, a block per tile:
//                    metaball flags (sec. 2.1), node classes and the
//                    boundary/uncovered update
//   k_bulk           every plain fluid node: pull-stream + BGK/Guo collide,
//                    branch-free apart from the one class byte (HBM-bound)
//   k_special        boundary and uncovered nodes: pull with bounce-back or
//                    refill (sec. 2.3.2, refilling equation), then collide
//   k_link_emit_*    cut-link list of the new geometry (masks and counts from
//                    the classification; a fixed grid visits the tiles with
//                    links)
//   k_link_q         link fractions q, eight lanes per link, by a safeguarded
//                    Newton iteration in FP64
// Populations are deviations f_i - w_i rho0 in FP32, FP16 or BF16 storage;
// collisions run in FP32, everything geometric or mechanical in FP64.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "launch.h"
#include "min_image.h"
#include "mlp_dev.h"
#include "stream_collide.h"

namespace mdl {

__device__ __forceinline__ void node_xyz(const Params &p, long long n, int &x, int &y, int &z) {
    if (p.N <= 0xffffffffLL) {  // 32-bit quotients (far shorter than 64-bit division)
        const unsigned u = (unsigned)n, r = u / (unsigned)p.nx;
        x = (int)(u - r * (unsigned)p.nx);
        y = (int)(r % (unsigned)p.ny);
        z = (int)(r / (unsigned)p.ny);
        return;
    }
    x = (int)(n % p.nx);
    long long r = n / p.nx;
    y = (int)(r % p.ny);
    z = (int)(r / p.ny);
}

// Neighbour (x + dx, ...) with periodic wrap; false outside a wall.
__device__ __forceinline__ bool nbr(const Params &p, int x, int y, int z, int dx, int dy, int dz,
                                    long long &out) {
    x += dx; y += dy; z += dz;
    if (x < 0 || x >= p.nx) { if (!(p.periodic & 1u)) return false; x = x < 0 ? x + p.nx : x - p.nx; }
    if (y < 0 || y >= p.ny) { if (!(p.periodic & 2u)) return false; y = y < 0 ? y + p.ny : y - p.ny; }
    if (z < 0 || z >= p.nz) { if (!(p.periodic & 4u)) return false; z = z < 0 ? z + p.nz : z - p.nz; }
    out = (long long)x + (long long)p.nx * ((long long)y + (long long)p.ny * z);
    return true;
}

// d - L floor(d / L + 0.5) per periodic axis (min_image_axis: the same
// result without a division within 1.25 L of zero).
__device__ __forceinline__ void min_image(const Params &p, double d[3]) {
    const double L[3] = {(double)p.nx, (double)p.ny, (double)p.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (p.periodic & (1u << a)) d[a] = min_image_axis(d[a], L[a], p.mi_up[a], p.mi_dn[a]);
}

// Control points of one body staged in LDS by the whole block, padded to a
// multiple of 4 with weight-0 copies of the first point (they add exactly
// zero) so that evaluation loops run 4 independent terms at a time.
// Orders the LDS accesses of the lanes of one wave (code motion and the
// memory model at wavefront scope; a wave's LDS operations run in order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Maximum over the 64 lanes of a wave (every lane gets it; all lanes take part).
__device__ __forceinline__ float wave_fmax(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

struct CPs {
    double x[MAXCP + 3][3];
    double k[MAXCP + 3];
    // the same points relative to the anchor (the body's centroid) and
    // weights in FP32, for the FP32 first decision of C >= L (metaball_ge32)
    float4 f[MAXCP + 3];
    double anc[3];
    float bp;  // max over the points of |p - anchor|_1
    int n;    // padded count
    int img;  // the body's img: 0 = the minimum image is the identity here
    double level;  // the link fractions' surface: C = level (1, or c_0 of the inner body)
};

// Point i of the staged set: lab position and weight in FP64, position
// relative to the anchor and weight in FP32.  Returns |p - anchor|_1 of the
// FP32 form.
__device__ __forceinline__ float stage_cp(CPs &c, int i, const double x[3], double k, const double anc[3]) {
    c.x[i][0] = x[0]; c.x[i][1] = x[1]; c.x[i][2] = x[2];
    c.k[i] = k;
    const float4 f = make_float4((float)(x[0] - anc[0]), (float)(x[1] - anc[1]), (float)(x[2] - anc[2]), (float)k);
    c.f[i] = f;
    return fabsf(f.x) + fabsf(f.y) + fabsf(f.z);
}

// Whole block: the body's points (padded to a multiple of 4 with weight-0
// copies of the first point) about the anchor X.
__device__ void stage_cps(CPs &c, const DevParticle &P) {
    const int n4 = (P.n_cp + 3) & ~3;
    const float b = threadIdx.x < n4 ? stage_cp(c, threadIdx.x, P.cpl[threadIdx.x < P.n_cp ? threadIdx.x : 0],
                                                threadIdx.x < P.n_cp ? P.k[threadIdx.x] : 0.0, P.X)
                                     : 0.f;
    const float bw = wave_fmax(b);  // n4 <= 24 points: all in the first wave
    if (threadIdx.x == 0) {
        c.anc[0] = P.X[0]; c.anc[1] = P.X[1]; c.anc[2] = P.X[2];
        c.n = n4;
        c.img = P.img;
        c.bp = bw * (1.f + 1e-6f);
    }
}

// Metaball function (Eq. metaballM) at a lab point, minimum image on
// periodic axes; a control point exactly on x gives +inf.  Terms k_i/r_i^2
// are exact quotients summed in index order.
__device__ double metaball(const Params &p, const CPs &P, const double x[3]) {
#pragma clang fp contract(off)
    double C = 0.0;
    for (int i0 = 0; i0 < P.n; i0 += 4) {
        double term[4];
        bool hit = false;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u;
            double d[3] = {x[0] - P.x[i][0], x[1] - P.x[i][1], x[2] - P.x[i][2]};
            if (P.img) min_image(p, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            hit |= r2 == 0.0;
            term[u] = P.k[i] / r2;
        }
        if (hit) return __builtin_inf();
        C += term[0];
        C += term[1];
        C += term[2];
        C += term[3];
    }
    return C;
}

// Reciprocal of x != 0: the hardware estimate and two Newton steps (a few
// ulps; the exact quotient costs about twice the instructions).
__device__ __forceinline__ double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(e, r, r);
    e = fma(-x, r, 1.0);
    return fma(e, r, r);
}

// C(x) with refined reciprocals in place of the quotients: each term within
// a few ulps, so the sum of at most 23 terms within 1e-14 C of metaball's.
__device__ double metaball_fast(const Params &p, const CPs &P, const double x[3]) {
#pragma clang fp contract(off)
    double C = 0.0;
    for (int i0 = 0; i0 < P.n; i0 += 4) {
        double term[4];
        bool hit = false;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u;
            double d[3] = {x[0] - P.x[i][0], x[1] - P.x[i][1], x[2] - P.x[i][2]};
            if (P.img) min_image(p, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            hit |= r2 == 0.0;
            term[u] = P.k[i] * rcp_refined(r2);
        }
        if (hit) return __builtin_inf();
        C += term[0];
        C += term[1];
        C += term[2];
        C += term[3];
    }
    return C;
}

// Whether C(x) >= L exactly as metaball decides it (exact quotients summed
// in index order): the fast sum decides unless it lies within 1e-12 L of L,
// where metaball is evaluated.  Cf: the fast value.
__device__ __forceinline__ bool metaball_ge(const Params &p, const CPs &P, const double x[3], double L, double &Cf) {
    Cf = metaball_fast(p, P, x);
    if (fabs(Cf - L) > 1e-12 * L) return Cf >= L;
    return metaball(p, P, x) >= L;
}
__device__ __forceinline__ bool metaball_ge1(const Params &p, const CPs &P, const double x[3], double &Cf) {
    return metaball_ge(p, P, x, 1.0, Cf);
}

// Whether C(x) >= L, decided first in FP32 where the FP32 sum is certain to
// fall on the same side as the exact one, else by metaball_ge.  FP32 form:
// r = x - X and the points' p - X rounded to FP32 (X the anchor), d = r - p,
// terms k * rcp(|d|^2) on the hardware reciprocal (1 ulp), summed with fma.
// With every |d|^2 >= 1 each component of d is off by at most
// u (|r_a| + |p_a| + |d_a|) (u = 2^-24), so |d|^2 by at most
// u (2.03 (|r|_1 + |p|_1) + 6.5) relative, a term by that plus 3 u, and the
// n-term sum by n u more: rel = u (2.03 (|r|_1 + bp) + 9.5 + n), taken with
// a factor 1.5.  The FP32 sum decides when it clears L by that bound plus
// 1e-12 (the exact sum's own rounding); points within 1 of a control point
// (|d|^2 < 1 in FP32), points whose differences could reach half a periodic
// box, and everything within the bound go to the FP64 forms.  Cf: the FP32
// sum when it decided, else metaball_fast's value.
__device__ __forceinline__ bool metaball_ge32(const Params &p, const CPs &P, const double x[3], double L,
                                              double &Cf) {
    double r[3] = {x[0] - P.anc[0], x[1] - P.anc[1], x[2] - P.anc[2]};
    bool ok = true;
    if (P.img) {
        // a body near a periodic face: the minimum image of x - X once; then
        // d = r - (p - X) is the minimum image of x - p for every point as
        // long as it stays below half the box on every periodic axis
        min_image(p, r);
        const double Lb[3] = {(double)p.nx, (double)p.ny, (double)p.nz};
        for (int a = 0; a < 3; ++a)
            if ((p.periodic >> a) & 1u) ok = ok && fabs(r[a]) + (double)P.bp < 0.5 * Lb[a] - 1.0;
    }
    if (ok) {
        const float rx = (float)r[0], ry = (float)r[1], rz = (float)r[2];
        float C = 0.f, rmin = 1.f;
        for (int i0 = 0; i0 < P.n; i0 += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 c = P.f[i0 + u];
                const float dx = rx - c.x, dy = ry - c.y, dz = rz - c.z;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                rmin = fminf(rmin, r2);
                C = fmaf(c.w, __builtin_amdgcn_rcpf(r2), C);
            }
        }
        if (rmin >= 1.f) {
            const float ax = fabsf(rx) + fabsf(ry) + fabsf(rz);
            const double rel = 1.5 * 5.9604644775390625e-8 * (2.03 * ((double)ax + (double)P.bp) + 9.5 + P.n);
            const double Cd = (double)C;
            if (Cd * (1.0 - rel) > L * (1.0 + 1e-12)) { Cf = Cd; return true; }
            if (Cd * (1.0 + rel) < L * (1.0 - 1e-12)) { Cf = Cd; return false; }
        }
    }
    return metaball_ge(p, P, x, L, Cf);
}

// A double from another lane of the same row by a DPP move (both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// Sum over an aligned group of eight lanes, the same bits in every lane:
// partners lane ^ 1, lane ^ 2 (quad permutations), then the mirror lane of
// the other quad (7 - lane), which holds the same quad sum as lane ^ 4.
constexpr int DPP_XOR1 = 0xb1, DPP_XOR2 = 0x4e, DPP_HALF_MIRROR = 0x141;
__device__ __forceinline__ double group8_sum(double v) {
    v += dpp_f64<DPP_XOR1>(v);
    v += dpp_f64<DPP_XOR2>(v);
    return v + dpp_f64<DPP_HALF_MIRROR>(v);
}
// Sum over the 64 lanes of a wave, the same bits in every lane: group8_sum,
// then the mirror lane of the other half-row (15 - lane), then lane ^ 16 and
// lane ^ 32 (IEEE addition commutes, so both partners form the same sum).
constexpr int DPP_ROW_MIRROR = 0x140;
__device__ __forceinline__ double wave_sum_fixed(double v) {
    v = group8_sum(v);
    v += dpp_f64<DPP_ROW_MIRROR>(v);
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
}

// C and dC/ds at x_f - s e_i for one link held by an aligned group of eight
// lanes: lane j sums control points j, j + 8, ... and the group adds its
// partial sums by a butterfly, which leaves the same bits in every lane.
// These values steer the Newton iteration and judge its residual to 1e-15 of
// the level, so they are formed with fused multiply-adds and refined
// reciprocals.
__device__ void metaball_ds8(const Params &p, const CPs &P, const double xf[3], const double e[3], double s,
                             double &C, double &dC) {
    double xs[3] = {xf[0] - s * e[0], xf[1] - s * e[1], xf[2] - s * e[2]};
    bool img = P.img;
    if (img) {
        // the image of the point nearest the centroid, once: then x - p needs
        // no image per point while it stays below half a periodic box
        double r[3] = {xs[0] - P.anc[0], xs[1] - P.anc[1], xs[2] - P.anc[2]};
        min_image(p, r);
        const double Lb[3] = {(double)p.nx, (double)p.ny, (double)p.nz};
        bool ok = true;
        for (int a = 0; a < 3; ++a)
            if ((p.periodic >> a) & 1u) ok = ok && fabs(r[a]) + (double)P.bp < 0.5 * Lb[a] - 1.0;
        if (ok) {
            for (int a = 0; a < 3; ++a) xs[a] = P.anc[a] + r[a];
            img = false;
        }
    }
    double c = 0.0, g = 0.0;
    for (int i = threadIdx.x & 7; i < P.n; i += 8) {
        double d[3] = {xs[0] - P.x[i][0], xs[1] - P.x[i][1], xs[2] - P.x[i][2]};
        if (img) min_image(p, d);
        const double r2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
        if (r2 == 0.0) {
            c = __builtin_inf();
            continue;
        }
        const double inv = rcp_refined(r2);
        const double kr = P.k[i] * inv;
        c += kr;
        g = fma(2.0 * kr * inv, fma(d[0], e[0], fma(d[1], e[1], d[2] * e[2])), g);
    }
    C = group8_sum(c);
    dC = group8_sum(g);
}

// Link fraction q (sec. 2.3.2): the first root of C(x_f - s e_i) = L on
// (0,1] (L = P.level: 1, or c_0 for the sphero-metaball's inner body), for
// one link by an aligned group of eight lanes (all active).
// Bracket: lane j decides C >= 1 at s = (j + 1)/8 exactly as the flagging
// does (metaball_ge1), and the first of the eight sub-interval ends with C >= 1 closes
// the bracket (none: q = 1).  Then a safeguarded Newton iteration
// (rtsafe-style: a Newton step that leaves the bracket or does not halve the
// step falls back to bisection) to |step| < 1e-13 or |C - 1| < 1e-15,
// started at the guess when it lies inside the bracket, else by regula
// falsi on the bracket ends, for at most it_max evaluations (conv:
// converged).  Every lane returns the same
// q and resid = C - 1 at the last evaluation; the return value is the
// number of evaluations of the iteration.
__device__ int link_fraction8(const Params &p, const CPs &P, int x, int y, int z, int i, double guess,
                              int it_max, double &q, double &resid, bool &conv) {
    const int lane = threadIdx.x & 63, j = lane & 7, base = lane & 56;
    const double xf[3] = {(double)x, (double)y, (double)z};
    const double e[3] = {(double)EX[i], (double)EY[i], (double)EZ[i]};
    const double sj = (double)(j + 1) / 8.0;
    const double xj[3] = {xf[0] - sj * e[0], xf[1] - sj * e[1], xf[2] - sj * e[2]};
    double Cj;
    const double L = P.level;
    const bool inj = metaball_ge32(p, P, xj, L, Cj);
    const unsigned grp = (unsigned)((__ballot(inj) >> base) & 0xffull);
    const int k0 = grp ? __ffs(grp) - 1 : 7;
    const double Chi = __shfl(Cj, base + k0), Clo = __shfl(Cj, base + (k0 > 0 ? k0 - 1 : 0));
    resid = 0.0;
    conv = true;
    if (!grp) {
        q = 1.0;
        return 0;
    }
    double lo = k0 / 8.0, hi = (k0 + 1) / 8.0;
    const double ghi = Chi - L, glo = Clo - L;
    double s;
    if (guess > lo && guess < hi) s = guess;
    else if (k0 > 0 && ghi < __builtin_inf()) s = lo + (hi - lo) * (-glo) / (ghi - glo);
    else s = 0.5 * (lo + hi);
    if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
    double dxold = hi - lo, dx = dxold;
    int it = 0;
    conv = false;
    while (it < it_max) {
        double C, dC;
        metaball_ds8(p, P, xf, e, s, C, dC);
        ++it;
        const double g = C - L;
        resid = g;
        if (fabs(g) < 1e-15 * L) {  // C = L to a few ulps: nothing left to resolve (tangent links get here
            conv = true;        // long before the step drops below 1e-13)
            break;
        }
        if (g >= 0.0) hi = s; else lo = s;
        const double sn = s - g * rcp_refined(dC);  // a zero or tiny slope leaves the bracket: bisection
        if (!(dC != 0.0) || !(sn > lo && sn < hi) || fabs(2.0 * g) > fabs(dxold * dC)) {
            dxold = dx;
            dx = 0.5 * (hi - lo);
            s = lo + dx;
        } else {
            dxold = dx;
            dx = s - sn;
            s = sn;
        }
        if (fabs(dx) < 1e-13) {
            conv = true;
            break;
        }
    }
    q = s;
    return it;
}

// Wave-aggregated append: one atomic per wave; returns this lane's slot.
__device__ __forceinline__ int wave_append(int *counter, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (!m) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    const unsigned long long below = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
    return pred ? base + __popcll(below) : -1;
}

// Sum over the lanes of a wave (all 64 lanes must take part).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}


// D3Q19 tables indexable by a runtime lane number.
__constant__ int c_ex[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int c_ey[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int c_ez[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__constant__ int c_opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
__constant__ float c_w[Q] = {1.f / 3, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                             1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                             1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
__constant__ double c_wd[Q] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                               1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                               1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Second-order equilibrium of a runtime direction in FP64.
__device__ __forceinline__ double feq64d(int i, double rho, const double u[3]) {
    const double eu = c_ex[i] * u[0] + c_ey[i] * u[1] + c_ez[i] * u[2];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return c_wd[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

// BGK + Guo for the one direction i a lane owns, given the node's moments:
// the same increments as collide (d+_i = (1 - 1/tau) d_i + S + A_i with S
// even and A_i odd in e_i).
__device__ __forceinline__ float collide_lane(float d, int i, float dr, float jx, float jy, float jz,
                                              const Params &p) {
    const float rho = p.rho0f + dr;
    const float Fx = rho * p.gx, Fy = rho * p.gy, Fz = rho * p.gz;
    const float inv = __builtin_amdgcn_rcpf(rho);
    const float ux = (jx + 0.5f * Fx) * inv, uy = (jy + 0.5f * Fy) * inv, uz = (jz + 0.5f * Fz) * inv;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
    const float om = p.omega;
    const float g = om * (dr - 1.5f * rho * uu) - 3.f * p.fcoef * uF;
    const float r45 = 4.5f * om * rho, r3 = 3.f * om * rho, f9 = 9.f * p.fcoef, f3 = 3.f * p.fcoef;
    const float ex = (float)c_ex[i], ey = (float)c_ey[i], ez = (float)c_ez[i], w = c_w[i];
    const float eu = ex * ux + ey * uy + ez * uz;
    const float eF = ex * Fx + ey * Fy + ez * Fz;
    const float T = (w * r45) * eu + (w * f9) * eF;
    const float S = eu * T + w * g;
    const float A = (w * r3) * eu + (w * f3) * eF;
    return (1.f - om) * d + (S + A);
}

// ------------------------------------------------------------------ kernels
// One thread per cut link (links come particle-major).  The thread forms the
// incoming population on the link -- simple bounce-back, or the paper's
// interpolated rule with the moments of x_f and x_f + e_i in FP64 -- and
// leaves it in B for the boundary-node pass, then the link's momentum
// exchange  dP = (e_ib - u_w) f+_ib(x_f) - (e_i - u_w) f_i(x_f, t+1) with
// both populations relative to w rho0, dT = (x_w - X) x dP.  Each wave's chunk of 64 links sums its links per
// body (a fixed butterfly) into part[chunk + body] (deterministic).
// Block bid of nblk (a whole grid, or one system's range of a batched grid).
template <int S>
__device__ __forceinline__ void links_body(const Params &p, const typename Store<S>::T *__restrict__ A,
                                           typename Store<S>::T *__restrict__ B,
                                           const int32_t *__restrict__ own,
                                           const DevParticle *__restrict__ P,
                                           const uint32_t *__restrict__ l_node,
                                           const uint32_t *__restrict__ l_do,
                                           const double *__restrict__ l_q, double *__restrict__ part,
                                           Counters *__restrict__ cnt, const int bid, const int nblk) {
    const int t = threadIdx.x, lane = t & 63;
    const int nl = cnt->n_links;
    const int nblock = (nl + 255) >> 8;  // 256 links per block and round, a chunk of 64 per wave
    for (int cb = bid; cb < nblock; cb += nblk) {
        const int l = (cb << 8) + t, ch = l >> 6;
        double dP[3] = {0, 0, 0}, dT[3] = {0, 0, 0};
        int pi = -1;
        bool ok = l < nl;
        long long n = 0;
        int i = 1;
        if (ok) {
            n = l_node[l];
            i = (int)(l_do[l] & 31u);
            pi = (int)(l_do[l] >> 8);
            if (n >= p.N || pi >= p.np || i < 1 || i >= Q) {  // never expected: report, do not touch memory
                atomicOr(&cnt->err, ERR_BAD_INDEX);
                ok = false;
                pi = -1;
            }
        }
        if (ok) {
            const int ib = c_opp[i];
            int x, y, z;
            node_xyz(p, n, x, y, z);
            long long ff = n;  // the node itself beyond a wall (its loads then go unused)
            const bool has_ff = nbr(p, x, y, z, c_ex[i], c_ey[i], c_ez[i], ff);
            // every load of the link is issued before the first is used: the
            // owner of x_f + e_i, the fraction, the body's motion, the population
            // leaving along e_ib, and both nodes' moments (which only the
            // interpolated rule uses)
            const int32_t own_ff = own[ff];
            const double ql = l_q[l];
            const DevParticle &Bd = P[pi];
            const double fbl = (double)Store<S>::ld(A, pidx(n, ib), p.inv_scale);
            double m0 = 0, m1 = 0, m2 = 0, m3 = 0, k0 = 0, k1 = 0, k2 = 0, k3 = 0;
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const double d0 = (double)Store<S>::ld(A, pidx(n, j), p.inv_scale);
                const double d1 = (double)Store<S>::ld(A, pidx(ff, j), p.inv_scale);
                m0 += d0; m1 += EX[j] * d0; m2 += EY[j] * d0; m3 += EZ[j] * d0;
                k0 += d1; k1 += EX[j] * d1; k2 += EY[j] * d1; k3 += EZ[j] * d1;
            }
            const bool ibb = p.bc == 1 && has_ff && own_ff == FLUID;
            const double q = ibb ? ql : 0.5;
            double r[3] = {x - q * c_ex[i] - Bd.X[0], y - q * c_ey[i] - Bd.X[1], z - q * c_ez[i] - Bd.X[2]};
            min_image(p, r);
            double uw[3];
            cross3(Bd.w, r, uw);
            for (int a = 0; a < 3; ++a) uw[a] += Bd.v[a];
            const double w = c_wd[i];
            const double fb = w * p.rho0 + fbl;
            const double mw = 6.0 * w * p.rho0 * (c_ex[i] * uw[0] + c_ey[i] * uw[1] + c_ez[i] * uw[2]);
            double val;
            if (!ibb) {
                val = fb + mw;
            } else {
                const double rf = p.rho0 + m0, rff = p.rho0 + k0;
                const double uf[3] = {m1 / rf - 0.5 * p.gfd[0], m2 / rf - 0.5 * p.gfd[1], m3 / rf - 0.5 * p.gfd[2]};
                const double uff[3] = {k1 / rff - 0.5 * p.gfd[0], k2 / rff - 0.5 * p.gfd[1], k3 / rff - 0.5 * p.gfd[2]};
                double ud[3];
                for (int a = 0; a < 3; ++a) {
                    const double us = q <= 0.5 ? 2.0 * q * uf[a] + (1.0 - 2.0 * q) * uff[a]
                                               : (1.0 - q) / q * uf[a] + (2.0 * q - 1.0) / q * uw[a];
                    const double uss = (1.0 - q) / (1.0 + q) * uff[a] + 2.0 * q / (1.0 + q) * uw[a];
                    ud[a] = us / 3.0 + 2.0 * uss / 3.0;
                }
                val = feq64d(ib, rf, ud) + fb - feq64d(ib, rf, uf) + mw;
            }
            Store<S>::st(B, pidx(n, i), (float)(val - w * p.rho0), p.scale);
            // exchanged populations relative to w rho0: the uniform reference
            // pressure exerts no force (its per-link terms cancel over a closed
            // surface; a surface touching a wall has no links there)
            const double fbd = fb - w * p.rho0, vald = val - w * p.rho0;
            dP[0] = (c_ex[ib] - uw[0]) * fbd - (c_ex[i] - uw[0]) * vald;
            dP[1] = (c_ey[ib] - uw[1]) * fbd - (c_ey[i] - uw[1]) * vald;
            dP[2] = (c_ez[ib] - uw[2]) * fbd - (c_ez[i] - uw[2]) * vald;
            cross3(r, dP, dT);
        }
        // the chunk's sum per body: links are listed body by body, so a wave
        // holds one run per body it touches; each run is summed over the wave
        // by a fixed butterfly (the same bits in every lane) and written by
        // the run's first lane
        const double v6[6] = {dP[0], dP[1], dP[2], dT[0], dT[1], dT[2]};
        const int prev = __shfl_up(pi, 1);
        unsigned long long heads = __ballot(pi >= 0 && (lane == 0 || prev != pi));
        while (heads) {
            const int h = __ffsll((long long)heads) - 1;
            heads &= heads - 1;
            const int b = __shfl(pi, h);
            const bool in = pi == b;
            double sum[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) sum[c] = wave_sum_fixed(in ? v6[c] : 0.0);
            if (lane == h) {
                double *o = part + 6ll * (ch + b);
                for (int c = 0; c < 6; ++c) o[c] = sum[c];
            }
        }
    }
}

template <int S>
__global__ __launch_bounds__(256) void k_links(Params p, const typename Store<S>::T *__restrict__ A,
                                               typename Store<S>::T *__restrict__ B,
                                               const int32_t *__restrict__ own,
                                               const DevParticle *__restrict__ P,
                                               const uint32_t *__restrict__ l_node,
                                               const uint32_t *__restrict__ l_do,
                                               const double *__restrict__ l_q, double *__restrict__ part,
                                               Counters *__restrict__ cnt) {
    links_body<S>(p, A, B, own, P, l_node, l_do, l_q, part, cnt, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------- rigid body (FP64)
__device__ void quat_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ void quat_mul(const double a[4], const double b[4], double o[4]) {
    const double r0 = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    const double r1 = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    const double r2 = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    const double r3 = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
}

__device__ void quat_of_rotvec(const double phi[3], double o[4]) {
    const double a = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (a == 0.0) { o[0] = 1.0; o[1] = o[2] = o[3] = 0.0; return; }
    const double s = sin(0.5 * a) / a;
    o[0] = cos(0.5 * a); o[1] = s * phi[0]; o[2] = s * phi[1]; o[3] = s * phi[2];
}

// Lab-frame control points and the region origin of the current pose, and
// whether the minimum image can shift anything here: the metaball is
// evaluated at points within half + 2 + sqrt 3 (+1 along a link) of X, the
// control points lie within rb of X; when on every periodic axis those points
// do not wrap and |x - cp| stays 1 below L/2, floor(d / L + 0.5) is 0 for every
// difference and the image is the identity (img = 0).
__device__ void refresh_pose(const Params &p, DevParticle &P) {
    double R[9];
    quat_rot(P.q, R);
    for (int i = 0; i < P.n_cp; ++i)
        for (int a = 0; a < 3; ++a)
            P.cpl[i][a] = P.X[a] + R[3 * a] * P.cpb[i][0] + R[3 * a + 1] * P.cpb[i][1] + R[3 * a + 2] * P.cpb[i][2];
    for (int a = 0; a < 3; ++a) P.lo[a] = P.full[a] ? 0 : (int)floor(P.X[a]) - P.half;
    const double reach = P.half + 2.0 + 1.7320508075688772 + 1.0;
    const double L[3] = {(double)p.nx, (double)p.ny, (double)p.nz};
    int img = 0;
    for (int a = 0; a < 3; ++a)
        if ((p.periodic >> a) & 1u)
            if (!(P.X[a] - reach >= 0.0 && P.X[a] + reach <= L[a] - 1.0 && reach + P.rb <= 0.5 * L[a] - 1.0)) img = 1;
    P.img = img;
}

// One block per particle: fixed-order FP64 sum of the link momenta (chunk
// partials from k_links) into the particle's hydrodynamic force and torque;
// with 'update' (no contact: bodies move independently) also the body's
// rigid-body update on an LDS copy of its record.  Block 0 also clears the
// per-step counters.
__device__ void body_substep(const Params &p, DevParticle &P, const double F[3], const double T[3], double dt);
__device__ void end_of_step(const Params &p, DevParticle &B, Counters *cnt);

// Fixed-order FP64 sum of the chunk partials of body pi (from k_links) into
// its hydrodynamic force and torque; with 'update' (no contact: bodies move
// independently) also its rigid-body update on an LDS copy of its record.
// Whole block, 256 threads; red and sp are LDS scratch.
__device__ void reduce_body(const Params &p, DevParticle *__restrict__ P, int pi, const int *__restrict__ l_off,
                            const double *__restrict__ part, Counters *__restrict__ cnt, int update,
                            double (*red)[256], DevParticle &sp) {
    const int t = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    const int a = max(0, l_off[pi]), b = min(l_off[pi + 1], p.link_cap);
    if (b > a)  // chunks of 64 links holding this body's links; slot = chunk + body
        for (int ch = (a >> 6) + t; ch <= ((b - 1) >> 6); ch += 256)
            for (int c = 0; c < 6; ++c) s[c] += part[6ll * (ch + pi) + c];
    for (int c = 0; c < 6; ++c) red[c][t] = s[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int c = 0; c < 6; ++c) red[c][t] += red[c][t + h];
        __syncthreads();
    }
    if (!update) {
        if (t == 0)
            for (int c = 0; c < 3; ++c) { P[pi].F[c] = red[c][0]; P[pi].T[c] = red[3 + c][0]; }
        __syncthreads();
        return;
    }
    constexpr int W = sizeof(DevParticle) / 4;
    for (int k = t; k < W; k += 256) ((int *)&sp)[k] = ((const int *)&P[pi])[k];
    __syncthreads();
    if (t == 0) {
        for (int c = 0; c < 3; ++c) { sp.F[c] = red[c][0]; sp.T[c] = red[3 + c][0]; sp.X0[c] = sp.X[c]; }
        const double dt = 1.0 / p.n_sub;
        for (int s2 = 0; s2 < p.n_sub; ++s2) body_substep(p, sp, sp.F, sp.T, dt);
        end_of_step(p, sp, cnt);
    }
    __syncthreads();
    for (int k = t; k < W; k += 256) ((int *)&P[pi])[k] = ((const int *)&sp)[k];
    __syncthreads();
}

__device__ void reset_step_counters(Counters *cnt) {
    cnt->n_special = 0;
}

// One block per particle: reduce_body.  Block 0 also clears the per-step
// counters.
__device__ __forceinline__ void reduce_case(const Params &p, DevParticle *__restrict__ P,
                                            const int *__restrict__ l_off, const double *__restrict__ part,
                                            Counters *__restrict__ cnt, int update, int *body_stats, const int pi) {
    __shared__ double red[6][256];
    __shared__ DevParticle sp;
    if (pi == 0 && threadIdx.x == 0) reset_step_counters(cnt);
    if (pi >= p.np) return;
    if (threadIdx.x < 4) body_stats[4 * pi + threadIdx.x] = 0;  // counts of the coming classification
    reduce_body(p, P, pi, l_off, part, cnt, update, red, sp);
}

__global__ __launch_bounds__(256) void k_reduce(Params p, DevParticle *__restrict__ P,
                                                const int *__restrict__ l_off,
                                                const double *__restrict__ part,
                                                Counters *__restrict__ cnt, int update, int *body_stats) {
    reduce_case(p, P, l_off, part, cnt, update, body_stats, blockIdx.x);
}


// ------------------------------------------------------ contact (sec. 2.3.1)
__device__ bool inv3d(const double A[9], double B[9]) {
    const double d = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(fabs(d) > 0.0)) return false;
    B[0] = (A[4] * A[8] - A[5] * A[7]) / d; B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / d; B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / d; B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / d; B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
    return true;
}

// Zoomed internal metaball of the sphero-metaball: the body shrunk about its
// centroid by s = 1 - R_s / sqrt(sum k) (points X + s (p - X), weights
// s^2 k), translated by 'shift' (periodic image).  Its points are formed
// from the body record where they are used (no per-thread copies, which
// would live in scratch memory).
struct InnerMB {
    const DevParticle *P;
    double s, s2;
    double shift[3];
    int n;
};

__device__ int inner_metaball(const Params &p, const DevParticle &P, const double shift[3], InnerMB &m) {
    double sk = 0.0;
    for (int i = 0; i < P.n_cp; ++i) sk += P.k[i];
    const double s = 1.0 - p.c_rs / sqrt(sk);
    if (!(s > 0.0)) return -1;
    m.P = &P;
    m.s = s;
    m.s2 = s * s;
    for (int a = 0; a < 3; ++a) m.shift[a] = shift[a];
    m.n = P.n_cp;
    return P.n_cp;
}

__device__ __forceinline__ double inner_cp(const InnerMB &m, int i, int a) {
    return m.P->X[a] + m.shift[a] + m.s * (m.P->cpl[i][a] - m.P->X[a]);
}
__device__ __forceinline__ double inner_k(const InnerMB &m, int i) { return m.s2 * m.P->k[i]; }

// f = sum k/r^2, gradient sum -2k d/r^4, Hessian sum 2k (4 d d^T/r^6 - I/r^4),
// from one reciprocal of r^2 per point (the powers and products follow; the
// Hessian's upper triangle is mirrored).
__device__ void mb_eval3(const InnerMB &m, const double x[3], double &f, double g[3], double H[9]) {
    double f_ = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0, h00 = 0.0, h01 = 0.0, h02 = 0.0, h11 = 0.0, h12 = 0.0, h22 = 0.0;
    for (int i = 0; i < m.n; ++i) {
        const double ki = inner_k(m, i);
        const double d0 = x[0] - inner_cp(m, i, 0), d1 = x[1] - inner_cp(m, i, 1), d2 = x[2] - inner_cp(m, i, 2);
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const double i2 = 1.0 / r2, i4 = i2 * i2;
        const double c1 = -2.0 * ki * i4, c2 = 8.0 * ki * i4 * i2;
        f_ += ki * i2;
        g0 += c1 * d0; g1 += c1 * d1; g2 += c1 * d2;
        h00 += c2 * d0 * d0 + c1; h01 += c2 * d0 * d1; h02 += c2 * d0 * d2;
        h11 += c2 * d1 * d1 + c1; h12 += c2 * d1 * d2; h22 += c2 * d2 * d2 + c1;
    }
    f = f_;
    g[0] = g0; g[1] = g1; g[2] = g2;
    H[0] = h00; H[1] = h01; H[2] = h02;
    H[3] = h01; H[4] = h11; H[5] = h12;
    H[6] = h02; H[7] = h12; H[8] = h22;
}

// Newton-Raphson for a stationary point of f0 + f1 from xm (in place), the
// step capped at L/4, for at most it_max iterations; true when the step
// fell below 1e-12 (1 + L).  iters: evaluations made.
__device__ bool pair_newton(const InnerMB &m0, const InnerMB &m1, double xm[3], double L, int it_max, int &iters) {
    for (int it = 0; it < it_max; ++it) {
        double f0, g0[3], H0[9], f1, g1[3], H1[9], H[9], Hi[9], dx[3];
        mb_eval3(m0, xm, f0, g0, H0);
        mb_eval3(m1, xm, f1, g1, H1);
        ++iters;
        for (int a = 0; a < 9; ++a) H[a] = H0[a] + H1[a];
        if (!inv3d(H, Hi)) return false;
        double st = 0.0;
        for (int a = 0; a < 3; ++a) {
            dx[a] = -(Hi[3 * a] * (g0[0] + g1[0]) + Hi[3 * a + 1] * (g0[1] + g1[1]) + Hi[3 * a + 2] * (g0[2] + g1[2]));
            st += dx[a] * dx[a];
        }
        st = sqrt(st);
        if (st > 0.25 * L)
            for (int a = 0; a < 3; ++a) dx[a] *= 0.25 * L / st;
        for (int a = 0; a < 3; ++a) xm[a] += dx[a];
        if (st < 1e-12 * (1.0 + L)) return true;
    }
    return false;
}

// Contact of two bodies (Eqs. CM_coreF, eq:grad, eq:cp, eq:contactprop):
// Newton-Raphson for the stationary point x_m of f0 + f1 between the inner
// metaballs from the point of the centroid segment dividing it in the ratio
// (K0/K1)^(1/3); Taylor projections x_c = x_m + q grad f, q = (1 - f)/|grad f|^2;
// n from body 1 to body 0; delta = 2 R_s - |x_c0 - x_c1| (signed form); contact
// point in the middle of the overlap.  1 = contact, 0 = none, -1 = iteration
// failed.  With a guess (warm start, finite), the iteration starts there for
// at most PAIR_WARM_MAX evaluations and its point is kept only if it
// converged to the kind of point the plain start finds between separate
// bodies: projection on the centroid segment inside it, outside both inner
// bodies (f0, f1 < 1), positive curvature of f0 + f1 along the segment;
// otherwise (also in deep contact) the plain start follows.  xm_out: the
// stationary point (body 0's frame), iters: evaluations.
constexpr int PAIR_WARM_MAX = 20, PAIR_NR_MAX = 60;
__device__ int pair_geometry(const Params &p, const DevParticle &P0, const DevParticle &P1, double xcp[3],
                             double nrm[3], double &delta, const double *guess, double xm_out[3], int &iters) {
    double d01[3] = {P1.X[0] - P0.X[0], P1.X[1] - P0.X[1], P1.X[2] - P0.X[2]};
    min_image(p, d01);
    const double sh0[3] = {0.0, 0.0, 0.0};
    const double sh1[3] = {P0.X[0] + d01[0] - P1.X[0], P0.X[1] + d01[1] - P1.X[1], P0.X[2] + d01[2] - P1.X[2]};
    InnerMB m0, m1;
    const int n0 = inner_metaball(p, P0, sh0, m0), n1 = inner_metaball(p, P1, sh1, m1);
    if (n0 < 0 || n1 < 0) return -1;
    double K0 = 0.0, K1 = 0.0;
    for (int i = 0; i < n0; ++i) K0 += inner_k(m0, i);
    for (int i = 0; i < n1; ++i) K1 += inner_k(m1, i);
    const double rho = cbrt(K0 / K1);
    double xm[3];
    const double L = sqrt(d01[0] * d01[0] + d01[1] * d01[1] + d01[2] * d01[2]);
    bool ok = false;
    double f0, g0[3], H0[9], f1, g1[3], H1[9];  // at the final point
    if (guess && isfinite(guess[0]) && isfinite(guess[1]) && isfinite(guess[2])) {
        for (int a = 0; a < 3; ++a) xm[a] = guess[a];
        ok = pair_newton(m0, m1, xm, L, PAIR_WARM_MAX, iters);
        if (ok) {  // the saddle between two separate bodies, as the plain start finds it
            const double t =
                ((xm[0] - P0.X[0]) * d01[0] + (xm[1] - P0.X[1]) * d01[1] + (xm[2] - P0.X[2]) * d01[2]) / (L * L);
            mb_eval3(m0, xm, f0, g0, H0);
            mb_eval3(m1, xm, f1, g1, H1);
            double curv = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) curv += d01[a] * (H0[3 * a + b] + H1[3 * a + b]) * d01[b];
            ok = t > 0.0 && t < 1.0 && f0 < 1.0 && f1 < 1.0 && curv > 0.0;
        }
    }
    const bool warm_kept = ok;
    if (!ok) {
        for (int a = 0; a < 3; ++a) xm[a] = P0.X[a] + d01[a] * rho / (1.0 + rho);
        ok = pair_newton(m0, m1, xm, L, PAIR_NR_MAX, iters);
    }
    for (int a = 0; a < 3; ++a) xm_out[a] = xm[a];
    if (!ok) return -1;
    if (!warm_kept) {
        mb_eval3(m0, xm, f0, g0, H0);
        mb_eval3(m1, xm, f1, g1, H1);
    }
    const double G0 = sqrt(g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2]);
    const double G1 = sqrt(g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]);
    if (!(G0 > 0.0 && G1 > 0.0)) return -1;
    // grad f0 = -grad f1 at x_m: x_c0 - x_c1 lies along n = grad f0/|grad f0|
    // with signed length (1 - f0)/|grad f0| + (1 - f1)/|grad f1| (< 0 when the
    // inner bodies overlap)
    const double q0 = (1.0 - f0) / (G0 * G0);
    delta = 2.0 * p.c_rs - ((1.0 - f0) / G0 + (1.0 - f1) / G1);
    for (int a = 0; a < 3; ++a) {
        nrm[a] = g0[a] / G0;
        xcp[a] = xm[a] + q0 * g0[a] - (p.c_rs - 0.5 * delta) * nrm[a];
    }
    return delta > 0.0 ? 1 : 0;
}

// The same pair geometry by an aligned group of eight lanes (all active,
// one pair): lane l sums the control points l, l + 8, ... of each inner
// body into f, grad f and the Hessian's six entries, and the group adds the
// partial sums (group8_sum: the same bits in every lane), so every lane
// follows the same iteration and returns the same result.  Reciprocals are
// refined hardware estimates.  Only the evaluations are shared out; the
// start, the Newton step and the projections are those of pair_geometry.
__device__ void mb_eval3_8(const InnerMB &m, const double x[3], double &f, double g[3], double H[9]) {
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x & 7; i < m.n; i += 8) {
        const double ki = inner_k(m, i);
        const double d0 = x[0] - inner_cp(m, i, 0), d1 = x[1] - inner_cp(m, i, 1), d2 = x[2] - inner_cp(m, i, 2);
        const double i2 = rcp_refined(fma(d0, d0, fma(d1, d1, d2 * d2))), i4 = i2 * i2;
        const double c1 = -2.0 * ki * i4, c2 = 8.0 * ki * i4 * i2;
        v[0] += ki * i2;
        v[1] += c1 * d0; v[2] += c1 * d1; v[3] += c1 * d2;
        v[4] += c2 * d0 * d0 + c1; v[5] += c2 * d0 * d1; v[6] += c2 * d0 * d2;
        v[7] += c2 * d1 * d1 + c1; v[8] += c2 * d1 * d2; v[9] += c2 * d2 * d2 + c1;
    }
#pragma unroll
    for (int a = 0; a < 10; ++a) v[a] = group8_sum(v[a]);
    f = v[0];
    g[0] = v[1]; g[1] = v[2]; g[2] = v[3];
    H[0] = v[4]; H[1] = v[5]; H[2] = v[6];
    H[3] = v[5]; H[4] = v[7]; H[5] = v[8];
    H[6] = v[6]; H[7] = v[8]; H[8] = v[9];
}

__device__ bool pair_newton8(const InnerMB &m0, const InnerMB &m1, double xm[3], double L, int it_max, int &iters) {
    for (int it = 0; it < it_max; ++it) {
        double f0, g0[3], H0[9], f1, g1[3], H1[9], H[9], Hi[9], dx[3];
        mb_eval3_8(m0, xm, f0, g0, H0);
        mb_eval3_8(m1, xm, f1, g1, H1);
        ++iters;
        for (int a = 0; a < 9; ++a) H[a] = H0[a] + H1[a];
        if (!inv3d(H, Hi)) return false;
        double st = 0.0;
        for (int a = 0; a < 3; ++a) {
            dx[a] = -(Hi[3 * a] * (g0[0] + g1[0]) + Hi[3 * a + 1] * (g0[1] + g1[1]) + Hi[3 * a + 2] * (g0[2] + g1[2]));
            st += dx[a] * dx[a];
        }
        st = sqrt(st);
        if (st > 0.25 * L)
            for (int a = 0; a < 3; ++a) dx[a] *= 0.25 * L / st;
        for (int a = 0; a < 3; ++a) xm[a] += dx[a];
        if (st < 1e-12 * (1.0 + L)) return true;
    }
    return false;
}

__device__ int pair_geometry8(const Params &p, const DevParticle &P0, const DevParticle &P1, double xcp[3],
                              double nrm[3], double &delta, const double *guess, double xm_out[3], int &iters) {
    double d01[3] = {P1.X[0] - P0.X[0], P1.X[1] - P0.X[1], P1.X[2] - P0.X[2]};
    min_image(p, d01);
    const double sh0[3] = {0.0, 0.0, 0.0};
    const double sh1[3] = {P0.X[0] + d01[0] - P1.X[0], P0.X[1] + d01[1] - P1.X[1], P0.X[2] + d01[2] - P1.X[2]};
    InnerMB m0, m1;
    const int n0 = inner_metaball(p, P0, sh0, m0), n1 = inner_metaball(p, P1, sh1, m1);
    if (n0 < 0 || n1 < 0) return -1;
    double K0 = 0.0, K1 = 0.0;
    for (int i = 0; i < n0; ++i) K0 += inner_k(m0, i);
    for (int i = 0; i < n1; ++i) K1 += inner_k(m1, i);
    const double rho = cbrt(K0 / K1);
    double xm[3];
    const double L = sqrt(d01[0] * d01[0] + d01[1] * d01[1] + d01[2] * d01[2]);
    bool ok = false;
    double f0, g0[3], H0[9], f1, g1[3], H1[9];  // at the final point
    if (guess && isfinite(guess[0]) && isfinite(guess[1]) && isfinite(guess[2])) {
        for (int a = 0; a < 3; ++a) xm[a] = guess[a];
        ok = pair_newton8(m0, m1, xm, L, PAIR_WARM_MAX, iters);
        if (ok) {
            const double t =
                ((xm[0] - P0.X[0]) * d01[0] + (xm[1] - P0.X[1]) * d01[1] + (xm[2] - P0.X[2]) * d01[2]) / (L * L);
            mb_eval3_8(m0, xm, f0, g0, H0);
            mb_eval3_8(m1, xm, f1, g1, H1);
            double curv = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) curv += d01[a] * (H0[3 * a + b] + H1[3 * a + b]) * d01[b];
            ok = t > 0.0 && t < 1.0 && f0 < 1.0 && f1 < 1.0 && curv > 0.0;
        }
    }
    const bool warm_kept = ok;
    if (!ok) {
        for (int a = 0; a < 3; ++a) xm[a] = P0.X[a] + d01[a] * rho / (1.0 + rho);
        ok = pair_newton8(m0, m1, xm, L, PAIR_NR_MAX, iters);
    }
    for (int a = 0; a < 3; ++a) xm_out[a] = xm[a];
    if (!ok) return -1;
    if (!warm_kept) {
        mb_eval3_8(m0, xm, f0, g0, H0);
        mb_eval3_8(m1, xm, f1, g1, H1);
    }
    const double G0 = sqrt(g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2]);
    const double G1 = sqrt(g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]);
    if (!(G0 > 0.0 && G1 > 0.0)) return -1;
    const double q0 = (1.0 - f0) / (G0 * G0);
    delta = 2.0 * p.c_rs - ((1.0 - f0) / G0 + (1.0 - f1) / G1);
    for (int a = 0; a < 3; ++a) {
        nrm[a] = g0[a] / G0;
        xcp[a] = xm[a] + q0 * g0[a] - (p.c_rs - 0.5 * delta) * nrm[a];
    }
    return delta > 0.0 ? 1 : 0;
}

// Contact with the halfway wall normal to axis ax (side 0 at -1/2, side 1 at
// L - 1/2) (Eqs. metawallcp, contactprop2): stationary point x_cw of f on the
// wall plane by 2-D Newton-Raphson from the projection of the control point
// where f on the plane is largest, x_cm =
// x_cw + q grad f, n = (x_cm - x_cw)/|...|, delta = R_s - |x_cm - x_cw|,
// x_cp = x_cw + delta/2 n.
__device__ int wall_geometry(const Params &p, const DevParticle &P, int ax, int side, double xcp[3],
                             double nrm[3], double &delta) {
    const int L = ax == 0 ? p.nx : (ax == 1 ? p.ny : p.nz);
    const double wpos = side ? L - 0.5 : -0.5;
    if (fabs(P.X[ax] - wpos) > P.rb + p.c_rs) return 0;
    const double sh[3] = {0.0, 0.0, 0.0};
    InnerMB m;
    const int n = inner_metaball(p, P, sh, m);
    if (n < 0) return -1;
    const int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
    // start at the projection of the control point where f on the plane is largest
    double xcw[3] = {P.X[0], P.X[1], P.X[2]};
    double best = -1.0;
    for (int i = 0; i < n; ++i) {
        double y[3] = {inner_cp(m, i, 0), inner_cp(m, i, 1), inner_cp(m, i, 2)}, fy, gy[3], Hy[9];
        y[ax] = wpos;
        mb_eval3(m, y, fy, gy, Hy);
        if (fy > best) {
            best = fy;
            for (int a = 0; a < 3; ++a) xcw[a] = y[a];
        }
    }
    bool ok = false;
    for (int it = 0; it < 60; ++it) {
        double f, g[3], H[9];
        mb_eval3(m, xcw, f, g, H);
        const double h11 = H[3 * a1 + a1], h12 = H[3 * a1 + a2], h22 = H[3 * a2 + a2];
        const double det = h11 * h22 - h12 * h12;
        if (!(fabs(det) > 0.0)) break;
        double d1 = -(h22 * g[a1] - h12 * g[a2]) / det, d2 = -(-h12 * g[a1] + h11 * g[a2]) / det;
        const double st = sqrt(d1 * d1 + d2 * d2);
        if (st > 0.25 * P.rb) { d1 *= 0.25 * P.rb / st; d2 *= 0.25 * P.rb / st; }
        xcw[a1] += d1;
        xcw[a2] += d2;
        if (st < 1e-12 * (1.0 + P.rb)) { ok = true; break; }
    }
    if (!ok) return -1;
    double f, g[3], H[9];
    mb_eval3(m, xcw, f, g, H);
    const double G = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (!(G > 0.0)) return -1;
    // grad f is normal to the plane at x_cw and points into the body: signed
    // length of x_cm - x_cw along n = grad f/|grad f| is (1 - f)/|grad f|
    delta = p.c_rs - (1.0 - f) / G;
    for (int a = 0; a < 3; ++a) {
        nrm[a] = g[a] / G;
        xcp[a] = xcw[a] + 0.5 * delta * nrm[a];
    }
    return delta > 0.0 ? 1 : 0;
}

// Linear spring-dashpot (sec. 2.3.1): F_n = k_n delta + eta_n (v_j - v_i).n,
// eta_n = 2 zeta sqrt(m_eff k_n) with zeta from the restitution; tangential
// spring xi (kept in the tangent plane) advanced by the tangential relative
// velocity, F_t = k_t xi + eta_n u_t, k_t = 2/7 k_n, capped at mu |F_n|.
__device__ void spring_dashpot(const Params &p, double meff, const double n[3], double delta,
                               const double vrel[3], double xi[3], double dt, double F[3]) {
    const double le = log(p.c_en);
    const double zeta = -le / sqrt(M_PI * M_PI + le * le);
    const double etan = 2.0 * zeta * sqrt(meff * p.c_kn), kt = 2.0 / 7.0 * p.c_kn;
    const double vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    const double Fn = p.c_kn * delta + etan * vn;
    const double xn = xi[0] * n[0] + xi[1] * n[1] + xi[2] * n[2];
    double Ft[3], ftn = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double ut = vrel[a] - vn * n[a];
        xi[a] = xi[a] - xn * n[a] + ut * dt;
        Ft[a] = kt * xi[a] + etan * ut;
        ftn += Ft[a] * Ft[a];
    }
    ftn = sqrt(ftn);
    const double cap = p.c_mu * fabs(Fn);
    if (ftn > cap && ftn > 0.0)
        for (int a = 0; a < 3; ++a) {
            Ft[a] *= cap / ftn;
            xi[a] = Ft[a] / kt;
        }
    for (int a = 0; a < 3; ++a) F[a] = Fn * n[a] + Ft[a];
}

__device__ void point_velocity(const Params &p, const DevParticle &P, const double x[3], double v[3],
                               double r[3]) {
    r[0] = x[0] - P.X[0]; r[1] = x[1] - P.X[1]; r[2] = x[2] - P.X[2];
    min_image(p, r);
    double wr[3];
    cross3(P.w, r, wr);
    for (int a = 0; a < 3; ++a) v[a] = P.v[a] + wr[a];
}

// One sub-step dt of the Newton-Euler update of a body under total force F
// and torque T (hydrodynamic + contact): semi-implicit Euler for v, X;
// body-frame Euler equation with the full inertia tensor for the spin; exact
// rotation of the sub-step spin for the attitude.  Kinematic bodies move with
// their given v, w.
__device__ void body_substep(const Params &p, DevParticle &P, const double F[3], const double T[3], double dt) {
    if (P.mode == 1) {
        const double phi[3] = {P.w[0] * dt, P.w[1] * dt, P.w[2] * dt};
        double dq[4];
        for (int a = 0; a < 3; ++a) P.X[a] += P.v[a] * dt;
        quat_of_rotvec(phi, dq);
        quat_mul(dq, P.q, P.q);
    } else {
        for (int a = 0; a < 3; ++a) {
            const double Ft = F[a] + (P.m - p.rho0 * P.V) * p.gp[a];
            P.v[a] += Ft / P.m * dt;
            P.X[a] += P.v[a] * dt;
        }
        double R[9], Tb[3], wb[3], Iw[3], gy[3];
        quat_rot(P.q, R);
        for (int a = 0; a < 3; ++a) {
            Tb[a] = R[a] * T[0] + R[3 + a] * T[1] + R[6 + a] * T[2];
            wb[a] = R[a] * P.w[0] + R[3 + a] * P.w[1] + R[6 + a] * P.w[2];
        }
        for (int a = 0; a < 3; ++a) Iw[a] = P.I[3 * a] * wb[0] + P.I[3 * a + 1] * wb[1] + P.I[3 * a + 2] * wb[2];
        cross3(wb, Iw, gy);
        const double rhs[3] = {Tb[0] - gy[0], Tb[1] - gy[1], Tb[2] - gy[2]};
        for (int a = 0; a < 3; ++a)
            wb[a] += dt * (P.Iinv[3 * a] * rhs[0] + P.Iinv[3 * a + 1] * rhs[1] + P.Iinv[3 * a + 2] * rhs[2]);
        for (int a = 0; a < 3; ++a) P.w[a] = R[3 * a] * wb[0] + R[3 * a + 1] * wb[1] + R[3 * a + 2] * wb[2];
        const double phi[3] = {wb[0] * dt, wb[1] * dt, wb[2] * dt};
        double dq[4];
        quat_of_rotvec(phi, dq);
        quat_mul(P.q, dq, P.q);
    }
    const double nq = sqrt(P.q[0] * P.q[0] + P.q[1] * P.q[1] + P.q[2] * P.q[2] + P.q[3] * P.q[3]);
    for (int a = 0; a < 4; ++a) P.q[a] /= nq;
    refresh_pose(p, P);
}

// All bodies over one lattice time unit in one block: n_sub sub-steps, each
// with the contact forces of every body pair (threads over pairs) and every
// walled face at the sub-step's poses, then each body advanced by its
// hydrodynamic load (held) plus its contacts summed in a fixed order
// (partners by index, then faces).  Finally end-of-step checks, periodic
// wrap of the centroid and the region origin.
constexpr int RIGID_LDS = 32;
// Contact of body pair q = i * np + j (i < j) at the sub-step's poses:
// force on i, torques on i and j, into the pair's slots (tangential spring
// of the pair updated).
// Whether bodies i and j are a candidate pair (bounding spheres overlap, not
// both kinematic).
__device__ __forceinline__ bool contact_candidate(const Params &p, const DevParticle &Pi, const DevParticle &Pj) {
    if (Pi.mode == 1 && Pj.mode == 1) return false;
    double d[3] = {Pj.X[0] - Pi.X[0], Pj.X[1] - Pi.X[1], Pj.X[2] - Pi.X[2]};
    min_image(p, d);
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) <= Pi.rb + Pj.rb;
}

// Contact of the pair q = i np + j (i < j) into its slots.  GROUP8: called by
// an aligned group of eight lanes for one pair (the geometry shared out,
// pair_geometry8); lane 0 writes the slots and counts.
template <bool GROUP8 = false>
__device__ __forceinline__ void contact_pair(const Params &p, const DevParticle *P, const ContactBufs &cb,
                                             Counters *__restrict__ cnt, int q, double dt, bool use_guess) {
    const int np = p.np;
    const int i = q / np, j = q - i * np;
    if (j <= i) return;
    double F[3] = {0, 0, 0}, Ti[3] = {0, 0, 0}, Tj[3] = {0, 0, 0};
    double *xi = cb.xiP + 3ll * q;
    const DevParticle &Pi = P[i], &Pj = P[j];
    uint8_t solved = 0;
    if (!(Pi.mode == 1 && Pj.mode == 1)) {
        int r = 0;
        double xcp[3], n[3], delta = 0.0;
        if (contact_candidate(p, Pi, Pj)) {
            double xm[3];
            int its = 0;
            const double *guess = use_guess ? cb.pairGuess + 4ll * q : nullptr;
            if constexpr (GROUP8) {
                r = pair_geometry8(p, Pi, Pj, xcp, n, delta, guess, xm, its);
                if (threadIdx.x & 7) return;  // the group's other lanes hold the same results
            } else {
                r = pair_geometry(p, Pi, Pj, xcp, n, delta, guess, xm, its);
            }
            atomicAdd(&cnt->n_contact_nr, 1ull);
            atomicAdd(&cnt->n_contact_it, (unsigned long long)its);
            for (int a = 0; a < 3; ++a) cb.pairXm[3ll * q + a] = xm[a];
            solved = r >= 0 ? 1 : 0;
        } else if (GROUP8 && (threadIdx.x & 7)) {
            return;
        }
        if (r < 0) atomicAdd(&cnt->n_contact_fail, 1ull);
        if (r <= 0) {
            xi[0] = xi[1] = xi[2] = 0.0;
        } else {
            atomicAdd(&cnt->n_contacts, 1ull);
            double vi[3], vj[3], ri[3], rj[3], vrel[3];
            point_velocity(p, Pi, xcp, vi, ri);
            point_velocity(p, Pj, xcp, vj, rj);
            for (int a = 0; a < 3; ++a) vrel[a] = vj[a] - vi[a];
            const double meff = Pi.mode == 1 ? Pj.m : (Pj.mode == 1 ? Pi.m : Pi.m * Pj.m / (Pi.m + Pj.m));
            spring_dashpot(p, meff, n, delta, vrel, xi, dt, F);
            const double Fm[3] = {-F[0], -F[1], -F[2]};
            cross3(ri, F, Ti);
            cross3(rj, Fm, Tj);
        }
    }
    if (GROUP8 && (threadIdx.x & 7)) return;
    for (int a = 0; a < 3; ++a) {
        cb.pairF[3ll * q + a] = F[a];
        cb.pairTi[3ll * q + a] = Ti[a];
        cb.pairTj[3ll * q + a] = Tj[a];
    }
    cb.pairOk[q] = solved;
    const uint8_t on = (F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0 || Ti[0] != 0.0 || Ti[1] != 0.0 || Ti[2] != 0.0 ||
                        Tj[0] != 0.0 || Tj[1] != 0.0 || Tj[2] != 0.0) ? 1 : 0;
    cb.pairOn[q] = on;
    cb.pairOn[(long long)j * np + i] = on;
}

// Contact of body i with face w = 2 * axis + side (q = 6 i + w), into its slots.
__device__ __forceinline__ void contact_wall(const Params &p, const DevParticle *P, const ContactBufs &cb,
                                             Counters *__restrict__ cnt, int q, double dt) {
    const int i = q / 6, w = q - 6 * i, ax = w >> 1, side = w & 1;
    double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
    double *xi = cb.xiW + 3ll * q;
    const DevParticle &Pi = P[i];
    if (Pi.mode != 1 && !((p.periodic >> ax) & 1u)) {
        double xcp[3], n[3], delta = 0.0;
        const int r = wall_geometry(p, Pi, ax, side, xcp, n, delta);
        if (r < 0) atomicAdd(&cnt->n_contact_fail, 1ull);
        if (r <= 0) {
            xi[0] = xi[1] = xi[2] = 0.0;
        } else {
            atomicAdd(&cnt->n_contacts, 1ull);
            double vi[3], ri[3], vrel[3];
            point_velocity(p, Pi, xcp, vi, ri);
            for (int a = 0; a < 3; ++a) vrel[a] = -vi[a];
            spring_dashpot(p, Pi.m, n, delta, vrel, xi, dt, F);
            for (int a = 0; a < 3; ++a) ri[a] = xcp[a] - Pi.X[a];
            cross3(ri, F, T);
        }
    }
    for (int a = 0; a < 3; ++a) { cb.wallF[3ll * q + a] = F[a]; cb.wallT[3ll * q + a] = T[a]; }
}

// Sub-step of body q: hydrodynamic load (held) plus its contacts summed in a
// fixed order (partners by index, then faces); partners whose pair slots hold
// only zeros are passed over (adding them changes no bit of the sums).
__device__ __forceinline__ void contact_body(const Params &p, DevParticle &B, int q, const ContactBufs &cb,
                                             double dt) {
    const int np = p.np;
    double F[3] = {B.F[0], B.F[1], B.F[2]}, T[3] = {B.T[0], B.T[1], B.T[2]};
    if (p.contact) {
        double Fc[3] = {0, 0, 0}, Tc[3] = {0, 0, 0};
        const uint8_t *on = cb.pairOn + (long long)q * np;
        for (int j = 0; j < np; ++j) {
            if (j == q || !on[j]) continue;
            if (j < q) {
                const long long k = (long long)j * np + q;
                for (int a = 0; a < 3; ++a) { Fc[a] -= cb.pairF[3 * k + a]; Tc[a] += cb.pairTj[3 * k + a]; }
            } else {
                const long long k = (long long)q * np + j;
                for (int a = 0; a < 3; ++a) { Fc[a] += cb.pairF[3 * k + a]; Tc[a] += cb.pairTi[3 * k + a]; }
            }
        }
        for (int w = 0; w < 6; ++w)
            for (int a = 0; a < 3; ++a) { Fc[a] += cb.wallF[3ll * (6 * q + w) + a]; Tc[a] += cb.wallT[3ll * (6 * q + w) + a]; }
        for (int a = 0; a < 3; ++a) { F[a] += Fc[a]; T[a] += Tc[a]; }
    }
    body_substep(p, B, F, T, dt);
}

__device__ __forceinline__ void rigid_case(const Params &p, DevParticle *__restrict__ Pg, const ContactBufs &cb,
                                           Counters *__restrict__ cnt) {
    __shared__ DevParticle sP[RIGID_LDS];
    const int t = threadIdx.x, np = p.np;
    const bool lds = np <= RIGID_LDS;
    DevParticle *P = lds ? sP : Pg;
    constexpr int W = sizeof(DevParticle) / 4;
    if (lds)
        for (int k = t; k < W * np; k += 256) ((int *)sP)[k] = ((const int *)Pg)[k];
    __syncthreads();
    for (int q = t; q < np; q += 256)
        for (int a = 0; a < 3; ++a) P[q].X0[a] = P[q].X[a];
    __syncthreads();
    const double dt = 1.0 / p.n_sub;
    for (int s = 0; s < p.n_sub; ++s) {
        if (p.contact) {
            // eight lanes per pair (aligned groups, all active: the branch is
            // group-uniform), then one thread per face
            for (int u = t; u < 8 * np * np + 6 * np; u += 256) {
                if (u < 8 * np * np) contact_pair<true>(p, P, cb, cnt, u >> 3, dt, false);
                else contact_wall(p, P, cb, cnt, u - 8 * np * np, dt);
            }
            __syncthreads();
        }
        for (int q = t; q < np; q += 256) contact_body(p, P[q], q, cb, dt);
        __syncthreads();
    }
    for (int q = t; q < np; q += 256) end_of_step(p, P[q], cnt);
    __syncthreads();
    if (lds)
        for (int k = t; k < W * np; k += 256) ((int *)Pg)[k] = ((const int *)sP)[k];
}

// The same sub-step over many blocks (many bodies): every pair and face in
// parallel, then every body (one thread each); the caller launches the pair
// kernel and then the body kernel once per sub-step.
__global__ __launch_bounds__(256) void k_contact_pairs(Params p, const DevParticle *__restrict__ P, ContactBufs cb,
                                                       Counters *__restrict__ cnt, int use_guess) {
    const int np2 = p.np * p.np;
    const double dt = 1.0 / p.n_sub;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 8 * np2) {  // eight lanes per pair (group-uniform branch)
        contact_pair<true>(p, P, cb, cnt, t >> 3, dt, use_guess != 0);
    } else {
        const int q = t - 8 * np2;
        if (q < 6 * p.np) contact_wall(p, P, cb, cnt, q, dt);
    }
}

// Warm start of the pair solves: the closest-point task of the MLP for every
// candidate pair (i < j), seen from body i, one wave per pair (four per
// block): inputs staged in LDS (FP16), hidden unit u on lane u (FP32 sums of
// FP16 products, FP16 activations), outputs 1..3 taken back to the lab frame
// as the starting stationary point; NaN where the pair is no candidate.
__global__ __launch_bounds__(256) void k_contact_guess(Params p, const DevParticle *__restrict__ P, ContactBufs cb,
                                                       const _Float16 *__restrict__ w, const float *__restrict__ body) {
    __shared__ _Float16 act[4][MLP_IN + 2 * MLP_H];  // inputs, h1, h2
    __shared__ float outs[4][MLP_OUT];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + wv;
    const int np = p.np;
    const int i = q / np, j = q - i * np;
    const bool cand = q < np * np && j > i && contact_candidate(p, P[i], P[j]);
    if (cand) {
        if (lane == 0) {
            double head[7];
            mlp_contact_head(p, P[i], P[j], head);
            for (int a = 0; a < 7; ++a) act[wv][a] = (_Float16)head[a];
        }
        for (int c = lane; c < MLP_BODY; c += 64) act[wv][7 + c] = (_Float16)body[i * MLP_BODY + c];
    }
    __syncthreads();
    if (cand) {
        float z = (float)w[MLP_OFF_B1 + lane];
        for (int k = 0; k < MLP_IN; ++k) z += (float)act[wv][k] * (float)w[MLP_OFF_W1 + k * MLP_H + lane];
        act[wv][MLP_IN + lane] = (_Float16)tanhf(z);
    }
    __syncthreads();
    if (cand) {
        float z = (float)w[MLP_OFF_B2 + lane];
        for (int k = 0; k < MLP_H; ++k) z += (float)act[wv][MLP_IN + k] * (float)w[MLP_OFF_W2 + k * MLP_H + lane];
        act[wv][MLP_IN + MLP_H + lane] = (_Float16)tanhf(z);
    }
    __syncthreads();
    if (cand && lane < MLP_OUT) {
        float o = (float)w[MLP_OFF_B3 + lane];
        for (int k = 0; k < MLP_H; ++k) o += (float)act[wv][MLP_IN + MLP_H + k] * (float)w[MLP_OFF_W3 + k * MLP_OUT + lane];
        outs[wv][lane] = o;
    }
    __syncthreads();
    if (q >= np * np || j <= i || lane != 0) return;
    double *g = cb.pairGuess + 4ll * q;
    if (!cand) {
        g[0] = __builtin_nan("");
        return;
    }
    // offset in body i's frame times sqrt(sum k), rotated to the lab frame
    const DevParticle &B = P[i];
    double K = 0.0;
    for (int c = 0; c < B.n_cp; ++c) K += B.k[c];
    const double s = sqrt(K);
    double R[9];
    quat_rot(B.q, R);
    const double ob[3] = {outs[wv][1] * s, outs[wv][2] * s, outs[wv][3] * s};
    for (int a = 0; a < 3; ++a) g[a] = B.X[a] + R[3 * a] * ob[0] + R[3 * a + 1] * ob[1] + R[3 * a + 2] * ob[2];
    g[3] = 0.0;
}

// One wave per body: lane l sums the pairs j = l, l + 64, ... in contact and
// wall l (< 6), the wave adds the partial sums by a butterfly (a fixed
// order), and lane 0 steps the body.
__global__ __launch_bounds__(256) void k_contact_bodies(Params p, DevParticle *__restrict__ P, ContactBufs cb,
                                                        Counters *__restrict__ cnt, int first, int last) {
    const int lane = threadIdx.x & 63, q = blockIdx.x * 4 + (threadIdx.x >> 6), np = p.np;
    if (q >= np) return;  // wave-uniform
    double s[6] = {0, 0, 0, 0, 0, 0};  // contact force, torque
    if (p.contact) {
        const uint8_t *on = cb.pairOn + (long long)q * np;
        for (int j = lane; j < np; j += 64) {
            if (j == q || !on[j]) continue;
            if (j < q) {
                const long long k = (long long)j * np + q;
                for (int a = 0; a < 3; ++a) { s[a] -= cb.pairF[3 * k + a]; s[3 + a] += cb.pairTj[3 * k + a]; }
            } else {
                const long long k = (long long)q * np + j;
                for (int a = 0; a < 3; ++a) { s[a] += cb.pairF[3 * k + a]; s[3 + a] += cb.pairTi[3 * k + a]; }
            }
        }
        if (lane < 6)
            for (int a = 0; a < 3; ++a) {
                s[a] += cb.wallF[3ll * (6 * q + lane) + a];
                s[3 + a] += cb.wallT[3ll * (6 * q + lane) + a];
            }
    }
    for (int c = 0; c < 6; ++c) s[c] = wave_sum64(s[c]);
    if (lane != 0) return;
    DevParticle &B = P[q];
    if (first)
        for (int a = 0; a < 3; ++a) B.X0[a] = B.X[a];
    const double F[3] = {B.F[0] + s[0], B.F[1] + s[1], B.F[2] + s[2]};
    const double T[3] = {B.T[0] + s[3], B.T[1] + s[4], B.T[2] + s[5]};
    body_substep(p, B, F, T, 1.0 / p.n_sub);
    if (last) end_of_step(p, B, cnt);
}

__global__ __launch_bounds__(256) void k_rigid(Params p, DevParticle *__restrict__ Pg, ContactBufs cb,
                                               Counters *__restrict__ cnt) {
    rigid_case(p, Pg, cb, cnt);
}

// End of a lattice step for one body: error checks (non-finite state, more
// than one lattice unit moved), periodic wrap of the centroid, pose refresh.
__device__ void end_of_step(const Params &p, DevParticle &B, Counters *cnt) {
    double d2 = 0.0;
    bool finite = true;
    for (int c = 0; c < 3; ++c) {
        d2 += (B.X[c] - B.X0[c]) * (B.X[c] - B.X0[c]);
        finite = finite && isfinite(B.X[c]) && isfinite(B.v[c]) && isfinite(B.w[c]);
    }
    if (!finite) atomicOr(&cnt->err, ERR_NONFINITE);
    else if (d2 > 1.0) atomicOr(&cnt->err, ERR_FAST_PARTICLE);
    // distance to the poses of the two previous flaggings (minimum image),
    // then this pose (flagged next) joins the history
    double reach = 1e30;
    if (B.hist >= 2 && finite) {
        reach = 0.0;
        for (int h = 0; h < 2; ++h) {
            double d[3] = {B.X[0] - B.Xf[h][0], B.X[1] - B.Xf[h][1], B.X[2] - B.Xf[h][2]};
            min_image(p, d);
            reach = fmax(reach, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
        }
    }
    B.reach = reach;
    const int L[3] = {p.nx, p.ny, p.nz};
    for (int c = 0; c < 3; ++c)  // keep the centroid inside a periodic box
        if ((p.periodic >> c) & 1u) {
            if (B.X[c] < 0.0) B.X[c] += L[c];
            else if (B.X[c] >= L[c]) B.X[c] -= L[c];
        }
    for (int a = 0; a < 3; ++a) { B.Xf[1][a] = B.Xf[0][a]; B.Xf[0][a] = B.X[a]; }
    B.hist = min(B.hist + 1, 2);
    refresh_pose(p, B);
}

// Pose refresh after a change from the host.  fresh = 0: the flag buffers
// may hold flags of unknown poses (no history: full regions); fresh = 1:
// the only flags are of the current pose (after a re-flag that cleared the
// other buffers).
__global__ void k_refresh_pose(Params p, DevParticle *P, int fresh) {
    const int pi = blockIdx.x * blockDim.x + threadIdx.x;
    if (pi >= p.np) return;
    DevParticle &B = P[pi];
    refresh_pose(p, B);
    for (int a = 0; a < 3; ++a) B.Xf[0][a] = B.Xf[1][a] = B.X[a];
    B.hist = fresh ? 2 : 0;
    B.reach = fresh ? 0.0 : 1e30;
}

// Region node of a region kernel thread; false if outside the region or the
// domain.
// Local region coordinates of thread t of tile f (tiles of TILE_X x TILE_Y
// x TILE_Z nodes over a region of dx x dy x ... nodes, x fastest).
__device__ __forceinline__ void tile_local(int f, int dx, int dy, int t, int &lx, int &ly, int &lz) {
    const int ntx = (dx + TILE_X - 1) / TILE_X, nty = (dy + TILE_Y - 1) / TILE_Y;
    const int tx = f % ntx, ty = (f / ntx) % nty, tz = f / (ntx * nty);
    lx = tx * TILE_X + (t % TILE_X);
    ly = ty * TILE_Y + (t / TILE_X) % TILE_Y;
    lz = tz * TILE_Z + t / (TILE_X * TILE_Y);
}

// Ball radii of the region kernels about the body's centroid: flagging
// (the C >= 1 set lies within re; half a node to spare), and classification
// and link build (a neighbour, sqrt 2, of the flags of this pose or of the
// two before, within reach).
__device__ __forceinline__ double flag_radius(const DevParticle &B) { return B.re + 0.5; }
__device__ __forceinline__ double class_radius(const DevParticle &B) { return B.re + 1.5 + B.reach; }

// True if no node of tile f of body B's region lies within rad of its
// centroid (block-uniform; never for a region spanning a periodic axis).
__device__ __forceinline__ bool tile_outside(const RegionMap &rm, const DevParticle &B, int pi, int f, double rad) {
    if (B.full[0] | B.full[1] | B.full[2]) return false;
    const int dx = rm.dims[3 * pi], dy = rm.dims[3 * pi + 1];
    int bx, by, bz;
    tile_local(f, dx, dy, 0, bx, by, bz);
    const int b0[3] = {B.lo[0] + bx, B.lo[1] + by, B.lo[2] + bz};
    const int w[3] = {TILE_X - 1, TILE_Y - 1, TILE_Z - 1};
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double g = fmax(0.0, fmax((double)b0[a] - B.X[a], B.X[a] - (double)(b0[a] + w[a])));
        d2 += g * g;
    }
    return d2 > rad * rad;
}

__device__ __forceinline__ bool region_node(const Params &p, const RegionMap &rm,
                                            const DevParticle *P, int bid, double rad, int &pi, int &x, int &y,
                                            int &z, long long &n) {
    pi = rm.part[bid];
    const int dx = rm.dims[3 * pi], dy = rm.dims[3 * pi + 1], dz = rm.dims[3 * pi + 2];
    int lx, ly, lz;
    tile_local(rm.first[bid], dx, dy, threadIdx.x, lx, ly, lz);
    if (lx >= dx || ly >= dy || lz >= dz) return false;
    const DevParticle &B = P[pi];
    if (!(B.full[0] | B.full[1] | B.full[2])) {
        // only the part of the cube within half + 2 of its centre floor(X):
        // what flagging, classification and link build touch lies within the
        // extent r_e of a centroid (at most two steps away, each step moving
        // less than one node), plus a neighbour (sqrt 2) and the offset of X
        // from the centre (sqrt 3): r_e + 5.15 < ceil(r_e) + 6 = half + 2
        const int ax = lx - B.half, ay = ly - B.half, az = lz - B.half, rr = B.half + 2;
        if (ax * ax + ay * ay + az * az > rr * rr) return false;
        // and within rad of the centroid itself
        const double ex = (double)(B.lo[0] + lx) - B.X[0], ey = (double)(B.lo[1] + ly) - B.X[1],
                     ez = (double)(B.lo[2] + lz) - B.X[2];
        if (ex * ex + ey * ey + ez * ez > rad * rad) return false;
    }
    int c[3] = {B.lo[0] + lx, B.lo[1] + ly, B.lo[2] + lz};
    const int L[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= L[a]) {
            if (!((p.periodic >> a) & 1u)) return false;
            c[a] = ((c[a] % L[a]) + L[a]) % L[a];
        }
    }
    x = c[0]; y = c[1]; z = c[2];
    n = (long long)x + (long long)p.nx * ((long long)y + (long long)p.ny * z);
    return true;
}

// Flags (sec. 2.1): C >= 1 is solid; the owner is the lowest body index
// (atomicMin).  own_new must hold FLUID on the region beforehand.
__device__ __forceinline__ void mark_body(const Params &p, const RegionMap &rm, const DevParticle *P,
                                          int32_t *own_new, const int bid) {
    __shared__ CPs cps;
    const int bp = rm.part[bid];
    const double rad = flag_radius(P[bp]);
    if (tile_outside(rm, P[bp], bp, rm.first[bid], rad)) return;  // the whole block
    stage_cps(cps, P[bp]);
    __syncthreads();
    int pi, x, y, z;
    long long n;
    if (!region_node(p, rm, P, bid, rad, pi, x, y, z, n)) return;
    const double xp[3] = {(double)x, (double)y, (double)z};
    double Cf;
    if (metaball_ge32(p, cps, xp, 1.0, Cf)) atomicMin(&own_new[n], pi);
}

__global__ __launch_bounds__(BLK) void k_region_mark(Params p, RegionMap rm, const DevParticle *P,
                                                     int32_t *own_new) {
    mark_body(p, rm, P, own_new, blockIdx.x);
}

// Integer sum over the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide integer sum (all BLK = 4 waves): wave sums, then the four
// totals through LDS (one barrier).  sh may be reused after a barrier.
static_assert(BLK == 256, "block reductions assume four waves");
__device__ __forceinline__ int block_sum(int v, int *sh) {
    v = wave_isum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// Three block-wide sums at once (all BLK threads; sh3 LDS scratch).
__device__ __forceinline__ void block_sum3(int &a, int &b, int &c, int (*sh3)[BLK]) {
    a = wave_isum(a);
    b = wave_isum(b);
    c = wave_isum(c);
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        sh3[0][w] = a; sh3[1][w] = b; sh3[2][w] = c;
    }
    __syncthreads();
    a = sh3[0][0] + sh3[0][1] + sh3[0][2] + sh3[0][3];
    b = sh3[1][0] + sh3[1][1] + sh3[1][2] + sh3[1][3];
    c = sh3[2][0] + sh3[2][1] + sh3[2][2] + sh3[2][3];
}

// Boundary or uncovered node n = (x, y, z), one thread: pull the 19
// populations -- a source outside a wall bounces off the resting wall, a
// source inside a body takes the bounce-back value that k_links left in B;
// for an uncovered node (solid before) populations from fluid sources are
// kept and a missing f_i becomes f_opp(i) + 6 w rho0 e_i.u_new if the
// opposite came from a fluid node, else feq_i(rho0, u_new) (sec. 2.3.2,
// refilling) -- then collide and store into B.  wall / solid: bit i set
// when the source x - e_i (i >= 1) lies outside the domain / in a body
// before the step; owner: the body that covered an uncovered node (FLUID
// otherwise).
template <int S>
__device__ void special_update(const Params &p, const typename Store<S>::T *__restrict__ A,
                               typename Store<S>::T *__restrict__ B, const DevParticle *__restrict__ P, int x,
                               int y, int z, long long n, uint32_t wall, uint32_t solid, int32_t owner) {
    const bool unc = owner != FLUID;
    // the rest population's source is the node itself: solid before for an
    // uncovered node
    if (unc) solid |= 1u;
    using T = typename Store<S>::T;
    float d[Q];
    uint32_t missing = 0u;
    // every population's load is issued whatever its case, its address
    // chosen by selects (the resting wall's own opposite population, the
    // bounce-back value in B, the pulled value), so that all 19 are in
    // flight together; a missing one's value is dropped
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const bool w = (wall >> i) & 1u, sd = (solid >> i) & 1u;
        if (unc && (w || sd)) missing |= 1u << i;
        long long src = n;  // kept beyond a wall
        nbr(p, x, y, z, -EX[i], -EY[i], -EZ[i], src);
        const T *base = sd && !w ? (const T *)B : A;
        const float v = Store<S>::ld(base, w ? pidx(n, OPP[i]) : pidx(sd ? n : src, i), p.inv_scale);
        d[i] = (unc && (w || sd)) ? 0.f : v;
    }
    if (missing) {
        const DevParticle &Bd = P[owner];
        double r[3] = {x - Bd.X[0], y - Bd.X[1], z - Bd.X[2]};
        min_image(p, r);
        double un[3];
        cross3(Bd.w, r, un);
        for (int a = 0; a < 3; ++a) un[a] += Bd.v[a];
        const double uu = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
        float f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = d[i];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (!((missing >> i) & 1u)) continue;
            const double eu = EX[i] * un[0] + EY[i] * un[1] + EZ[i] * un[2];
            const double w = WD[i];
            // the opposite direction's source is x + e_i: kept if it was fluid
            if (!((missing >> OPP[i]) & 1u))
                d[i] = (float)((double)f[OPP[i]] + 6.0 * w * p.rho0 * eu);
            else
                d[i] = (float)(w * p.rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
        }
    }
    collide(d, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<S>::st(B, pidx(n, i), d[i], p.scale);
}

// Node classification over the body regions.  Where regions overlap, one
// region decides each node without any claiming: a solid node by its owner
// after the step, an uncovered node by its owner before, a fluid node next to
// solid nodes by the lowest body index among those neighbours (old and new
// flags), whose region always contains it; a plain fluid node (no solid
// node around) only gets skip = 0, which any region may write.
//   - with do_special (a step), nodes fluid after the step that were solid
//     before (uncovered: refill) or had an in-domain solid neighbour before
//     (cut links: bounce-back) are updated right here (special_update);
//     without (a re-flag), k_uncovered lists the uncovered nodes for the
//     in-place refill over the whole domain;
//   - per-body counts of solid, uncovered and special nodes and of cut links
//     (a re-flag: solid and boundary nodes; k_uncovered adds the rest);
//   - only nodes within the body's classification ball (class_radius) are
//     visited;
//   - skip mask of the NEXT step's stream-collide: solid after, or with an
//     in-domain solid neighbour after (those nodes are left to the links and
//     special passes);
//   - with blk_cnt set, the block also counts the cut links of the new flags
//     for its body (first pass of the link build).
template <int S>
__device__ __forceinline__ void classify_body(const Params &p, const RegionMap &rm, const DevParticle *P,
                                              const int32_t *__restrict__ own_old,
                                              const int32_t *__restrict__ own_new,
                                              uint8_t *__restrict__ skip_next,
                                              uint32_t *special, Counters *cnt, int *blk_cnt,
                                              uint32_t *lmask, int *body_stats,
                                              const typename Store<S>::T *A,
                                              typename Store<S>::T *B, int do_special, int32_t *clear,
                                              const int bid) {
    __shared__ int sh[BLK];
    __shared__ int sh3[3][BLK];
    // owners before / after over the tile and a one-node halo (beyond a wall: OUTSIDE)
    constexpr int HX = TILE_X + 2, HY = TILE_Y + 2, HN = HX * HY * (TILE_Z + 2);
    constexpr int32_t OUTSIDE = -2;
    __shared__ int32_t h_old[HN], h_new[HN];
    const double rad = class_radius(P[rm.part[bid]]);
    if (tile_outside(rm, P[rm.part[bid]], rm.part[bid], rm.first[bid], rad)) {  // the whole block
        if (blk_cnt && threadIdx.x == 0) blk_cnt[bid] = 0;
        return;
    }
    {
        const int bp = rm.part[bid];
        const int dx = rm.dims[3 * bp], dy = rm.dims[3 * bp + 1];
        int bx, by, bz;
        tile_local(rm.first[bid], dx, dy, 0, bx, by, bz);
        const DevParticle &Bp = P[bp];
        const int L[3] = {p.nx, p.ny, p.nz};
        // all of a thread's halo loads are issued before the first is
        // written to LDS (one memory round trip, not one per slot)
        constexpr int HR = (HN + BLK - 1) / BLK;
        int32_t vo[HR], vn[HR];
#pragma unroll
        for (int r = 0; r < HR; ++r) {
            const int h = threadIdx.x + r * BLK;
            int c[3] = {Bp.lo[0] + bx - 1 + h % HX, Bp.lo[1] + by - 1 + (h / HX) % HY, Bp.lo[2] + bz - 1 + h / (HX * HY)};
            bool ok = h < HN;
            for (int a = 0; a < 3; ++a)
                if (c[a] < 0 || c[a] >= L[a]) {
                    if ((p.periodic >> a) & 1u) c[a] = ((c[a] % L[a]) + L[a]) % L[a];
                    else ok = false;
                }
            const long long g = ok ? (long long)c[0] + (long long)p.nx * ((long long)c[1] + (long long)p.ny * c[2]) : 0;
            vo[r] = ok ? own_old[g] : OUTSIDE;
            vn[r] = ok ? own_new[g] : OUTSIDE;
        }
#pragma unroll
        for (int r = 0; r < HR; ++r) {
            const int h = threadIdx.x + r * BLK;
            if (h < HN) {
                h_old[h] = vo[r];
                h_new[h] = vn[r];
            }
        }
    }
    __syncthreads();
    int pi, x, y, z;
    long long n;
    const bool in = region_node(p, rm, P, bid, rad, pi, x, y, z, n);
    if (in && clear) clear[n] = FLUID;  // the dead flag buffer (the flags before own_old) for the next flagging
    uint32_t m = 0u, wall = 0u, solid = 0u;
    // owners before / after, lowest owner among the neighbours before / after
    int32_t oo = FLUID, on = FLUID, mo = FLUID, mn = FLUID;
    if (in) {
        const int t = threadIdx.x;
        const int hc = (t % TILE_X + 1) + HX * ((t / TILE_X) % TILE_Y + 1) + HX * HY * (t / (TILE_X * TILE_Y) + 1);
        oo = h_old[hc];
        on = h_new[hc];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int hs = hc - EX[i] - HX * EY[i] - HX * HY * EZ[i];
            const int32_t vo = h_old[hs], vn = h_new[hs];
            if (vo == OUTSIDE) {
                wall |= 1u << i;
            } else {
                mo = min(mo, vo);
                mn = min(mn, vn);
                if (vo != FLUID) solid |= 1u << i;
                if (vn == pi) m |= 1u << i;
            }
        }
    }
    const bool so = oo != FLUID, sn = on != FLUID, nb_old = mo != FLUID, nb_new = mn != FLUID;
    const int32_t onb = min(mo, mn);
    if (sn) m = 0u;
    bool act = in;
    if (act) act = sn ? on == pi : so ? oo == pi : onb == FLUID || onb == pi;
    int c_solid = 0, c_refill = 0, c_spec = 0;
    if (act) {
        skip_next[n] = (uint8_t)((sn || nb_new) ? 1 : 0);
        const bool lo = !so && nb_old;
        const bool spec = !sn && (so || lo);
        c_solid = sn;
        // a re-flag (no boundary update) lists and counts its uncovered nodes
        // over the whole domain instead (k_uncovered): a body moved from
        // outside may leave them outside its new region
        c_refill = !sn && so && do_special;
        c_spec = do_special ? spec : lo && !sn;
        if (spec && do_special) {
            if (so && (oo < 0 || oo >= p.np)) atomicOr(&cnt->err, ERR_BAD_INDEX);  // never expected
            else special_update<S>(p, A, B, P, x, y, z, n, wall, solid, oo);
        }
    }
    // per-body node counts (one atomic per block and count, integers: order-free)
    block_sum3(c_solid, c_refill, c_spec, sh3);
    if (threadIdx.x == 0) {
        int *bs = body_stats + 4 * rm.part[bid];
        if (c_solid) atomicAdd(bs + 1, c_solid);
        if (c_refill) atomicAdd(bs + 2, c_refill);
        if (c_spec) atomicAdd(bs + 3, c_spec);
    }
    if (!blk_cnt) return;
    // first pass of the link build: this body's cut links of the new flags
    lmask[bid * BLK + threadIdx.x] = m;
    const int s = block_sum(__popc(m), sh);
    if (threadIdx.x == 0) {
        blk_cnt[bid] = s;
        if (s) atomicAdd(body_stats + 4 * rm.part[bid], s);
    }
}

template <int S>
__global__ __launch_bounds__(BLK) void k_region_classify(Params p, RegionMap rm, const DevParticle *P,
                                                         const int32_t *__restrict__ own_old,
                                                         const int32_t *__restrict__ own_new,
                                                         uint8_t *__restrict__ skip_next,
                                                         uint32_t *special, Counters *cnt, int *blk_cnt,
                                                         uint32_t *lmask, int *body_stats,
                                                         const typename Store<S>::T *A,
                                                         typename Store<S>::T *B, int do_special,
                                                         int32_t *clear) {
    classify_body<S>(p, rm, P, own_old, own_new, skip_next, special, cnt, blk_cnt, lmask, body_stats, A, B,
                     do_special, clear, blockIdx.x);
}

// Nodes uncovered by a re-flag (solid before, fluid after) anywhere in the
// domain: listed for the in-place refill and counted per body (uncovered and
// special).  The trip count is block-uniform, so a wave's lanes append
// together.
__global__ __launch_bounds__(256) void k_uncovered(Params p, const int32_t *__restrict__ own_old,
                                                   const int32_t *__restrict__ own_new, uint32_t *special,
                                                   Counters *cnt, int *body_stats) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long n0 = (long long)blockIdx.x * blockDim.x; n0 < p.N; n0 += stride) {
        const long long n = n0 + threadIdx.x;
        const int32_t oo = n < p.N ? own_old[n] : FLUID;
        const bool unc = n < p.N && oo != FLUID && own_new[n] == FLUID;
        const int k = wave_append(&cnt->n_special, unc);
        if (k < 0) continue;
        if (oo < 0 || oo >= p.np) {  // never expected: report, list nothing
            atomicOr(&cnt->err, ERR_BAD_INDEX);
            continue;
        }
        if (k < p.special_cap) special[k] = (uint32_t)n;
        else atomicOr(&cnt->err, ERR_SPECIAL_OVERFLOW);
        atomicAdd(body_stats + 4 * oo + 2, 1);
        atomicAdd(body_stats + 4 * oo + 3, 1);
    }
}

// Boundary and uncovered nodes, one wave per node, lane i < 19 owning
// direction i.  Boundary: a source inside a wall bounces off the resting
// wall, a source inside a body takes the bounce-back value that k_links left
// in B.  Uncovered (solid before): populations from fluid sources are kept, a
// missing f_i becomes f_opp(i) + 6 w rho0 e_i.u_new if the opposite came from
// a fluid node, else feq_i(rho0, u_new).  Then collide.  in_place (refill
// after an external re-flag): only uncovered nodes, A == B.
template <int S>
__global__ __launch_bounds__(256) void k_special(Params p, const typename Store<S>::T *A,
                                                 typename Store<S>::T *B,
                                                 const int32_t *__restrict__ own_old,
                                                 const DevParticle *__restrict__ P,
                                                 const uint32_t *__restrict__ list,
                                                 Counters *__restrict__ cnt, int in_place) {
    const int lane = threadIdx.x & 63;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    const int ns = min(cnt->n_special, p.special_cap);
    const int i = lane < Q ? lane : 0;
    for (int k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; k < ns; k += nw) {
        const long long n = list[k];
        if (n >= p.N) {  // never expected: report, do not touch memory
            if (lane == 0) atomicOr(&cnt->err, ERR_BAD_INDEX);
            continue;
        }
        const int own_n = own_old[n];
        if (own_n != FLUID && (own_n < 0 || own_n >= p.np)) {
            if (lane == 0) atomicOr(&cnt->err, ERR_BAD_INDEX);
            continue;
        }
        const bool unc = own_n != FLUID;
        if (in_place && !unc) continue;
        int x, y, z;
        node_xyz(p, n, x, y, z);
        float d = 0.f;
        bool missing = false;
        if (lane < Q) {
            long long s;
            if (!nbr(p, x, y, z, -c_ex[i], -c_ey[i], -c_ez[i], s)) {
                if (unc) missing = true;
                else d = Store<S>::ld(A, pidx(n, c_opp[i]), p.inv_scale);
            } else if (own_old[s] != FLUID) {
                if (unc) missing = true;
                else d = Store<S>::ld(B, pidx(n, i), p.inv_scale);
            } else {
                d = Store<S>::ld(A, pidx(s, i), p.inv_scale);
            }
        }
        if (unc) {
            const float dopp = __shfl(d, c_opp[i]);
            if (missing) {
                const DevParticle &Bd = P[own_n];
                double r[3] = {x - Bd.X[0], y - Bd.X[1], z - Bd.X[2]};
                min_image(p, r);
                double un[3];
                cross3(Bd.w, r, un);
                for (int a = 0; a < 3; ++a) un[a] += Bd.v[a];
                const double uu = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
                const double eu = c_ex[i] * un[0] + c_ey[i] * un[1] + c_ez[i] * un[2];
                const double w = c_wd[i];
                long long s2;
                if (nbr(p, x, y, z, c_ex[i], c_ey[i], c_ez[i], s2) && own_old[s2] == FLUID)
                    d = (float)((double)dopp + 6.0 * w * p.rho0 * eu);
                else
                    d = (float)(w * p.rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
            }
        }
        const float dv = lane < Q ? d : 0.f;
        const float dr = wave_sum(dv);
        const float jx = wave_sum(lane < Q ? c_ex[i] * dv : 0.f);
        const float jy = wave_sum(lane < Q ? c_ey[i] * dv : 0.f);
        const float jz = wave_sum(lane < Q ? c_ez[i] * dv : 0.f);
        if (lane < Q) Store<S>::st(B, pidx(n, i), collide_lane(d, i, dr, jx, jy, jz, p), p.scale);
    }
}

// Initial state: every fluid node holds the collided rest state.
template <int S>
__global__ void k_init_state(Params p, typename Store<S>::T *A, const int32_t *own) {
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < p.N;
         n += (long long)gridDim.x * blockDim.x) {
        float d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = 0.f;
        if (own[n] == FLUID) collide(d, p);
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<S>::st(A, pidx(n, i), d[i], p.scale);
    }
}

// Collides the stored populations of every fluid node in place (used when a
// post-stream state is handed in from the host).
template <int S>
__global__ void k_collide_stored(Params p, typename Store<S>::T *A, const int32_t *own) {
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < p.N;
         n += (long long)gridDim.x * blockDim.x) {
        if (own[n] != FLUID) continue;
        float d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = Store<S>::ld(A, pidx(n, i), p.inv_scale);
        collide(d, p);
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<S>::st(A, pidx(n, i), d[i], p.scale);
    }
}

__global__ void k_reset_counters(Counters *cnt) { reset_step_counters(cnt); }

__global__ void k_fill_i32(int32_t *a, long long n, int32_t v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}
__global__ void k_fill_u8(uint8_t *a, long long n, uint8_t v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}

// Link build, second pass: each block finds its offset in the particle-major
// list from the link totals of the bodies before its own and the counts of
// its body's earlier blocks (the first block of a body also records the
// body's offset, the last block the total) and lists
// its links (masks from the classification; thread order, then direction
// order).  The link fractions follow in k_link_q.
__device__ __forceinline__ void emit_body(const Params &p, const RegionMap &rm, const DevParticle *P,
                                          const uint32_t *__restrict__ lmask,
                                          const int *__restrict__ blk_cnt,
                                          const int *__restrict__ body_stats,
                                          const int *__restrict__ part_first_blk, int *__restrict__ l_off,
                                          uint32_t *__restrict__ l_node, uint32_t *__restrict__ l_do,
                                          Counters *cnt, int32_t *clear, const int bid, const int nblk) {
    __shared__ int sh[BLK];
    const int t = threadIdx.x;
    const int pid = rm.part[bid];
    const double rad = class_radius(P[pid]);
    // a block with no node in the ball lists nothing (its classification
    // counted none); the first block of a body and the last block still
    // record the offsets
    if (tile_outside(rm, P[pid], pid, rm.first[bid], rad) && part_first_blk[pid] != bid && bid != nblk - 1) return;
    // nor does a tile without links when the dead flags were cleared by the
    // classification (clear == NULL)
    if (!clear && blk_cnt[bid] == 0 && part_first_blk[pid] != bid && bid != nblk - 1) return;
    // the tile's own mask is loaded together with the counts before it (one
    // memory round trip for both)
    int pi, x, y, z;
    long long n;
    const bool in = region_node(p, rm, P, bid, rad, pi, x, y, z, n);
    const uint32_t m = in ? lmask[bid * BLK + t] : 0u;
    int before = 0;
    for (int q = t; q < pid; q += BLK) before += body_stats[4 * q];
    for (int b = part_first_blk[pid] + t; b < bid; b += BLK) before += blk_cnt[b];
    const int base = block_sum(before, sh);
    __syncthreads();  // every thread has read the sum before sh is reused
    if (t == 0) {
        if (part_first_blk[pid] == bid) l_off[pid] = min(base, p.link_cap);
        if (bid == nblk - 1) {
            const int total = base + blk_cnt[bid];
            if (total > p.link_cap) atomicOr(&cnt->err, ERR_LINK_OVERFLOW);
            cnt->n_links = min(total, p.link_cap);
            l_off[p.np] = min(total, p.link_cap);
        }
    }
    if (in && clear) clear[n] = FLUID;
    // exclusive prefix of the link counts over the block: inclusive scan
    // within the wave, plus the totals of the earlier waves
    const int c = __popc(m), lane = t & 63, w = t >> 6;
    int incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    int wbase = 0;
    for (int k = 0; k < w; ++k) wbase += sh[k];
    int o = base + wbase + incl - c;
    for (int i = 1; i < Q; ++i)
        if ((m >> i) & 1u) {
            if (o < p.link_cap) {
                l_node[o] = (uint32_t)n;
                l_do[o] = (uint32_t)i | ((uint32_t)pid << 8);
            }
            ++o;
        }
}

// The link list runs beside the stream-collide, which holds most of the
// compute units: a kernel there keeps few blocks resident, and one block per
// region tile (tens of thousands, nearly all without links) took the whole
// length of the stream-collide.  Here a block of a grid of G visits tiles b,
// b + G, b + 2G, ... ; per round, wave 0 tests 64 of them at once (one lane
// each) and the block then runs the per-tile body for the ones that pass,
// one after another.  (The flagging and the classification, which run alone
// and have work in a third of their tiles, are faster with a block per tile:
// this form took them from 122 to 191 and from 268 to 512 us.)
constexpr int REGION_GRID = 2048;
inline int region_grid(const Params &p) { return p.region_blocks < REGION_GRID ? p.region_blocks : REGION_GRID; }

template <class Test, class Body>
__device__ __forceinline__ void visit_tiles(int nblk, Test test, Body body) {
    __shared__ unsigned long long sel;
    const int G = gridDim.x;
    for (int base = blockIdx.x; base < nblk; base += 64 * G) {
        if (threadIdx.x < 64) {
            const int b = base + threadIdx.x * G;
            const unsigned long long m = __ballot(b < nblk && test(b));
            if (threadIdx.x == 0) sel = m;
        }
        __syncthreads();
        unsigned long long m = sel;
        __syncthreads();  // sel is rewritten in the next round
        while (m) {
            const int j = __ffsll((long long)m) - 1;
            m &= m - 1;
            body(base + j * G);
            __syncthreads();  // the body's LDS is restaged for the next tile
        }
    }
}

// The link list over the tiles with links, each body's first tile and the
// last tile (they record the offsets); the dead flags were cleared by the
// classification.
__global__ __launch_bounds__(BLK) void k_link_emit_tiles(Params p, RegionMap rm, const DevParticle *P,
                                                         const uint32_t *__restrict__ lmask,
                                                         const int *__restrict__ blk_cnt,
                                                         const int *__restrict__ body_stats,
                                                         const int *__restrict__ part_first_blk,
                                                         int *__restrict__ l_off, uint32_t *__restrict__ l_node,
                                                         uint32_t *__restrict__ l_do, Counters *cnt) {
    const int nblk = p.region_blocks;
    visit_tiles(
        nblk,
        [&](int b) {  // a body's tiles are consecutive: its first tile follows another body's
            return blk_cnt[b] > 0 || b == 0 || rm.part[b - 1] != rm.part[b] || b == nblk - 1;
        },
        [&](int b) {
            emit_body(p, rm, P, lmask, blk_cnt, body_stats, part_first_blk, l_off, l_node, l_do, cnt, nullptr, b,
                      nblk);
        });
}

// Link build, third pass: the link fractions of the whole list, eight lanes
// per link (32 links per block, blocks stride over the list), each wave
// staging one body's control points at a time in its LDS slot (a small slot
// per wave leaves room for several blocks per CU beside the stream-collide).
// With WARM the Newton iteration starts at the network's guess that the first
// pass (k_link_guess) left in l_q; a warm-started iteration that has not
// converged in NR_WARM_MAX evaluations is replaced by the plain one.  Per block: iteration histogram and largest
// final |C - 1|, added to the statistics.
constexpr int NR_WARM_MAX = 30, NR_MAX = 100;
// Warm start, first pass: the network's q for every link of the list, written
// to l_q as the solver's start (one wave per 32 links, the wave inference of
// mlp_dev.h; links with an invalid record get nothing, the solver reports
// them).  No block barrier: a wave without links returns at once.
__device__ __forceinline__ void link_guess_body(const Params &p, const DevParticle *__restrict__ P,
                                                const uint32_t *__restrict__ l_node,
                                                const uint32_t *__restrict__ l_do, const Counters *cnt,
                                                const _Float16 *__restrict__ wts, const float *__restrict__ body,
                                                double *__restrict__ l_q, const int bid, const int nblk) {
    const int lane = threadIdx.x & 63, s = lane & 31, h = lane >> 5;
    const int wv = bid * 4 + (threadIdx.x >> 6), nw = nblk * 4;  // 256-thread blocks
    const int nl = min(cnt->n_links, p.link_cap);
    if (wts == nullptr || p.np <= 0 || wv * 32 >= nl) return;
    MlpWave W;
    mlp_wave_load(W, wts);
    _Float16 w3[1][32];
    mlp_wave_load_out(w3[0], wts, 0);
    const float b3 = (float)wts[MLP_OFF_B3];
    for (int l0 = wv * 32; l0 < nl; l0 += nw * 32) {
        const int l = l0 + s;
        bool ok = l < nl;
        int pid = 0, i = 1;
        long long n = 0;
        if (ok) {
            n = l_node[l];
            i = (int)(l_do[l] & 31u);
            pid = (int)(l_do[l] >> 8);
            ok = n < p.N && pid < p.np && i >= 1 && i < Q;
        }
        if (!ok) pid = 0;  // loads stay inside body 0's block; the row is zeroed
        double head[7] = {};
        if (ok && h == 0) {  // chunk 0: inputs 0..6
            int x, y, z;
            node_xyz(p, n, x, y, z);
            const int e[3] = {c_ex[i], c_ey[i], c_ez[i]};
            mlp_link_head(p, P[pid], x, y, z, e, head);
        }
        // chunks 2m + h of the body block (chunk c = body entries 8 (c - 1) ..)
        const float4 *bb = (const float4 *)(body + (long long)pid * MLP_BODY);  // 320-byte rows
        mlp_h8 xin[MLP_S1];
#pragma unroll
        for (int m = 0; m < MLP_S1; ++m) {
            const int c = m == 0 ? 1 : (m == MLP_S1 - 1 ? 10 : 2 * m + h);  // a body chunk, 1..10
            const float4 u0 = bb[2 * (c - 1)], u1 = bb[2 * (c - 1) + 1];
            const float bv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
            const int cm = 2 * m + h;  // the chunk this slot takes
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                _Float16 v;
                if (m == 0) v = h == 0 ? (e < 7 ? (_Float16)head[e < 7 ? e : 0] : (_Float16)1.f) : (_Float16)bv[e];
                else v = cm <= 10 ? (_Float16)bv[e] : (_Float16)0.f;
                xin[m][e] = ok ? v : (_Float16)(cm == 0 && e == 7 ? 1.f : 0.f);
            }
        }
        float q[1];
        mlp_wave_forward<1>(W, xin, w3, &b3, q);
        if (ok && h == 0) l_q[l] = (double)q[0];
    }
}

__global__ __launch_bounds__(256) void k_link_guess(Params p, const DevParticle *__restrict__ P,
                                                    const uint32_t *__restrict__ l_node,
                                                    const uint32_t *__restrict__ l_do, const Counters *cnt,
                                                    const _Float16 *__restrict__ wts,
                                                    const float *__restrict__ body, double *__restrict__ l_q) {
    link_guess_body(p, P, l_node, l_do, cnt, wts, body, l_q, blockIdx.x, gridDim.x);
}

// Second pass (or the plain solve): WARM takes the start from l_q; a system
// without weights (wts NULL) takes the plain iteration in either form.
template <bool WARM>
__device__ __forceinline__ void link_q_body(const Params &p, const DevParticle *__restrict__ P,
                                            const uint32_t *__restrict__ l_node,
                                            const uint32_t *__restrict__ l_do, double *__restrict__ l_q,
                                            Counters *cnt, const NrStats &nrs, const _Float16 *__restrict__ wts,
                                            const int bid, const int nblk) {
    __shared__ CPs cps[4];  // one per wave
    __shared__ int sh[256];
    __shared__ unsigned hist[NR_HIST];
    __shared__ unsigned rmax;
    const int t = threadIdx.x, g = t >> 3, j = t & 7, w = t >> 6;
    const bool warm = WARM && wts != nullptr;  // block-uniform
    for (int b = t; b < NR_HIST; b += 256) hist[b] = 0u;
    if (t == 0) rmax = 0u;
    __syncthreads();
    // From here each wave runs its own eight groups through the rounds: the
    // wave's slot cps[w] is written and read only by its own lanes, so the
    // rounds need no block barrier (a wave does not wait for the slowest
    // link of the other three).
    const int nl = min(cnt->n_links, p.link_cap);
    int it_sum = 0, links = 0;
    // the next round's link record is loaded while this round solves
    uint32_t nx_node = 0, nx_do = 0;
    if (bid * 32 + g < nl) {
        nx_node = l_node[bid * 32 + g];
        nx_do = l_do[bid * 32 + g];
    }
    for (int l0 = bid * 32; l0 < nl; l0 += nblk * 32) {  // block-uniform trip count
        const int l = l0 + g;
        const bool ok0 = l < nl;
        const uint32_t cur_node = nx_node, cur_do = nx_do;
        if (l + nblk * 32 < nl) {
            nx_node = l_node[l + nblk * 32];
            nx_do = l_do[l + nblk * 32];
        }
        int pid = 0, i = 1;
        long long n = 0;
        if (ok0) {
            n = cur_node;
            i = (int)(cur_do & 31u);
            pid = (int)(cur_do >> 8);
            if (n >= p.N || pid >= p.np || i < 1 || i >= Q) {  // never expected: report, solve nothing
                if (j == 0) atomicOr(&cnt->err, ERR_BAD_INDEX);
            }
        }
        const bool ok = ok0 && n < p.N && pid < p.np && i >= 1 && i < Q;
        int x = 0, y = 0, z = 0;
        if (ok) node_xyz(p, n, x, y, z);
        double guess = -1.0;
        if (warm && ok) guess = l_q[l];  // the first pass's network output
        // The wave's links come body by body from the list, so its eight
        // groups nearly always share one body: the wave stages one body's
        // points at a time into its slot (lane k point k, padded to a
        // multiple of 4 with weight 0) and the groups of that body solve;
        // a wave across a body boundary takes a second turn.
        bool pending = ok;
        for (;;) {  // wave-uniform
            const unsigned long long pm = __ballot(pending);
            if (!pm) break;
            const int bpid = __shfl(pid, __ffsll((long long)pm) - 1);
            const DevParticle &B = P[bpid];
            const int n4 = (B.n_cp + 3) & ~3;
            // sphero-metaball level: the inner body (scaled by s about the
            // centroid, weights s^2 k) at the level c_0 = s^2
            const bool inner = p.link_c0 && p.c_rs > 0.0;
            const double sc = inner ? 1.0 - p.c_rs * B.rsk : 1.0;
            const int k = t & 63;
            float bmax = 0.f;
            if (k < n4) {
                const int src = k < B.n_cp ? k : 0;
                double xk[3];
                for (int a = 0; a < 3; ++a) xk[a] = inner ? B.X[a] + sc * (B.cpl[src][a] - B.X[a]) : B.cpl[src][a];
                bmax = stage_cp(cps[w], k, xk, k < B.n_cp ? (inner ? sc * sc * B.k[k] : B.k[k]) : 0.0, B.X);
            }
            bmax = wave_fmax(bmax);
            if (k == 0) {
                cps[w].anc[0] = B.X[0]; cps[w].anc[1] = B.X[1]; cps[w].anc[2] = B.X[2];
                cps[w].n = n4;
                cps[w].img = B.img;
                cps[w].level = sc * sc;
                cps[w].bp = bmax * (1.f + 1e-6f);
            }
            wave_sync();  // the slot is staged
            if (pending && pid == bpid) {  // group-uniform
                pending = false;
                double q, resid;
                bool conv;
                int its = link_fraction8(p, cps[w], x, y, z, i, guess, warm ? NR_WARM_MAX : NR_MAX, q, resid,
                                         conv);
                if (warm && !conv) {
                    its += link_fraction8(p, cps[w], x, y, z, i, -1.0, NR_MAX, q, resid, conv);
                }
                if (j == 0) {
                    l_q[l] = q;
                    it_sum += its;
                    ++links;
                    atomicAdd(&hist[min(its, NR_HIST - 1)], 1u);
                    atomicMax(&rmax, __float_as_uint((float)fabs(resid)));
                }
            }
            wave_sync();  // the slot is restaged next
        }
    }
    __syncthreads();
    const int its = block_sum(it_sum, sh);
    __syncthreads();
    const int nls = block_sum(links, sh);
    if (bid >= NR_BLOCKS) return;  // never: the launchers cap the grid
    if (t == 0 && nls > 0) {  // this block's own slot: plain read-modify-write
        nrs.work[2 * bid] += (unsigned long long)its;
        nrs.work[2 * bid + 1] += (unsigned long long)nls;
        nrs.resid[bid] = max(nrs.resid[bid], rmax);
    }
    for (int b = t; b < NR_HIST; b += 256)
        if (hist[b]) nrs.hist[bid * NR_HIST + b] += hist[b];
}

template <bool WARM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_link_q(Params p, const DevParticle *__restrict__ P,
                                                const uint32_t *__restrict__ l_node,
                                                const uint32_t *__restrict__ l_do, double *__restrict__ l_q,
                                                Counters *cnt, NrStats nrs, const _Float16 *__restrict__ wts) {
    link_q_body<WARM>(p, P, l_node, l_do, l_q, cnt, nrs, wts, blockIdx.x, gridDim.x);
}

// ------------------------------------------------- batched boundary kernels
// One launch of a kind for every system of an ensemble: block b works for
// system map[b] as its block b - first[kind] (the same code as the
// one-system launches above).
template <int S>
__global__ __launch_bounds__(256) void k_links_batch(const CaseArgs *__restrict__ cs, const int *__restrict__ map) {
    using T = typename Store<S>::T;
    const CaseArgs &a = cs[map[blockIdx.x]];
    links_body<S>(a.p, (const T *)a.A, (T *)a.B, a.own_old, a.P, a.l_node, a.l_do, a.l_q, a.part, a.cnt,
                  (int)blockIdx.x - a.first[BK_LINKS], a.nblk[BK_LINKS]);
}

__global__ __launch_bounds__(256) void k_reduce_batch(const CaseArgs *__restrict__ cs, const int *__restrict__ map) {
    const CaseArgs &a = cs[map[blockIdx.x]];
    reduce_case(a.p, a.P, a.l_off, a.part, a.cnt, a.update, a.body_stats, (int)blockIdx.x - a.first[BK_REDUCE]);
}

__global__ __launch_bounds__(256) void k_rigid_batch(const CaseArgs *__restrict__ cs, const int *__restrict__ map) {
    const CaseArgs &a = cs[map[blockIdx.x]];
    rigid_case(a.p, a.P, a.cb, a.cnt);
}

__global__ __launch_bounds__(BLK) void k_region_mark_batch(const CaseArgs *__restrict__ cs,
                                                           const int *__restrict__ map) {
    const CaseArgs &a = cs[map[blockIdx.x]];
    mark_body(a.p, a.rm, a.P, a.own_new, (int)blockIdx.x - a.first[BK_REGION]);
}

// with the boundary/uncovered update and the link count of the new flags
template <int S>
__global__ __launch_bounds__(BLK) void k_region_classify_batch(const CaseArgs *__restrict__ cs,
                                                               const int *__restrict__ map) {
    using T = typename Store<S>::T;
    const CaseArgs &a = cs[map[blockIdx.x]];
    classify_body<S>(a.p, a.rm, a.P, a.own_old, a.own_new, a.skip_next, a.special, a.cnt, a.blk_cnt, a.lmask,
                     a.body_stats, (const T *)a.A, (T *)a.B, 1, nullptr, (int)blockIdx.x - a.first[BK_REGION]);
}

__global__ __launch_bounds__(BLK) void k_link_emit_batch(const CaseArgs *__restrict__ cs,
                                                         const int *__restrict__ map) {
    const CaseArgs &a = cs[map[blockIdx.x]];
    emit_body(a.p, a.rm, a.P, a.lmask, a.blk_cnt, a.body_stats, a.part_first_blk, a.l_off, a.l_node, a.l_do, a.cnt,
              a.own_dead, (int)blockIdx.x - a.first[BK_REGION], a.nblk[BK_REGION]);
}

__global__ __launch_bounds__(256) void k_link_guess_batch(const CaseArgs *__restrict__ cs,
                                                          const int *__restrict__ map) {
    const CaseArgs &a = cs[map[blockIdx.x]];
    link_guess_body(a.p, a.P, a.l_node, a.l_do, a.cnt, a.warm, a.mlp_body, a.l_q,
                    (int)blockIdx.x - a.first[BK_LINKQ], a.nblk[BK_LINKQ]);
}

template <bool WARM>
__global__ __launch_bounds__(256) void k_link_q_batch(const CaseArgs *__restrict__ cs, const int *__restrict__ map) {
    const CaseArgs &a = cs[map[blockIdx.x]];
    link_q_body<WARM>(a.p, a.P, a.l_node, a.l_do, a.l_q, a.cnt, a.nrs, a.warm, (int)blockIdx.x - a.first[BK_LINKQ],
                      a.nblk[BK_LINKQ]);
}

// ------------------------------------------------------------ host launchers
static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// list kernels stride over their lists; size their grids for the expected lengths
static int expected_links(const Params &p) { return p.est_links > 0 ? min(p.est_links, p.link_cap) : p.link_cap; }
int link_grid(const Params &p) { return max(1, min(cdiv(expected_links(p), 256), 2048)); }
int link_q_grid(const Params &p) { return max(1, min(cdiv(expected_links(p), 32), NR_BLOCKS)); }
constexpr int LINK_GUESS_BLOCKS = 1024;  // 4096 waves, each loads the network once

// LDS reserved (and not used) by each stream-collide block, so that at most
// BULK_MAX_WAVES_PER_SIMD of its waves share a SIMD.  Its FP32 form needs 52
// VGPRs, so without a cap it fills all eight wave slots of every SIMD and the
// boundary kernels on the second stream (up to 128 VGPRs a wave) find no room
// until the stream-collide drains: the step becomes their sum instead of their
// maximum.  Six of eight slots leave two slots, 176 VGPRs and 22 KB of LDS per
// SIMD (CU) to the second stream; the stream-collide itself runs as fast with
// six waves per SIMD as with eight.  The LDS size per CU is read once per device.
constexpr int BULK_MAX_WAVES_PER_SIMD = 6;

static int bulk_lds_reserve(int waves_per_block, int max_blocks = 0) {
    static int lds_cu[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (lds_cu[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            v <= 0)
            v = -1;
        lds_cu[dev] = v;
    }
    if (lds_cu[dev] < 0) return 0;
    const int blocks = max_blocks > 0 ? max_blocks : BULK_MAX_WAVES_PER_SIMD * 4 / waves_per_block;  // 4 SIMDs per CU
    const int r = lds_cu[dev] / (blocks + 1) + 1;                        // blocks + 1 do not fit
    return (r + 511) & ~511;
}

template <int S>
static void launch_step_kernels_t(const StepArgs &a) {
    using T = typename Store<S>::T;
    const Params &p = a.p;
    T *A = (T *)a.A, *B = (T *)a.B;
    const int nspec = p.est_special > 0 ? min(p.est_special, p.special_cap) : p.special_cap;
    const int spec_grid = max(1, min(cdiv(nspec, 4), 2048));
    if (a.phase == PHASE_LINKS) {
        const int update = a.move && !p.contact;
        if (p.np > 0)
            k_links<S><<<link_grid(p), 256, 0, a.stream>>>(p, A, B, a.own_old, a.P, a.l_node, a.l_do, a.l_q,
                                                         a.part, a.cnt);
        k_reduce<<<max(p.np, 1), 256, 0, a.stream>>>(p, a.P, a.l_off, a.part, a.cnt, update, a.body_stats);
        if (a.move && p.contact && p.np > 0) {
            if (p.np <= RIGID_LDS && !a.warm) {  // few bodies: one block, records in LDS
                k_rigid<<<1, 256, 0, a.stream>>>(p, a.P, a.cb, a.cnt);
            } else {
                for (int s2 = 0; s2 < p.n_sub; ++s2) {
                    if (a.warm)
                        k_contact_guess<<<cdiv((long long)p.np * p.np, 4), 256, 0, a.stream>>>(p, a.P, a.cb, a.warm,
                                                                                            a.mlp_body);
                    k_contact_pairs<<<cdiv(8ll * p.np * p.np + 6 * p.np, 256), 256, 0, a.stream>>>(p, a.P, a.cb, a.cnt,
                                                                                                 a.warm ? 1 : 0);
                    k_contact_bodies<<<cdiv(p.np, 4), 256, 0, a.stream>>>(p, a.P, a.cb, a.cnt, s2 == 0,
                                                                          s2 == p.n_sub - 1);
                }
            }
        }
    } else if (a.phase == PHASE_FLAGS) {
        if (p.np > 0) {
            if (a.move) k_region_mark<<<p.region_blocks, BLK, 0, a.stream>>>(p, a.rm, a.P, a.own_new);
            hipExtLaunchKernelGGL(k_region_classify<S>, dim3(p.region_blocks), dim3(BLK), 0, a.stream, nullptr,
                                  a.ev_stop, 0, p, a.rm, (const DevParticle *)a.P, (const int32_t *)a.own_old,
                                  (const int32_t *)a.own_new, a.skip_next, a.special, a.cnt,
                                  a.move ? a.blk_cnt : (int *)nullptr, a.lmask, a.body_stats, (const T *)A, B,
                                  a.do_special, a.own_dead);
        } else if (a.ev_stop) {
            (void)hipEventRecord(a.ev_stop, a.stream);
        }
    } else if (a.phase == PHASE_BULK) {
        // events ride on the dispatch itself (no separate marker packets)
        const bool fits = bulk_offsets_fit(p, (int)sizeof(T));
        const int lds = bulk_lds_reserve(BULK_WAVES, a.bulk_blocks);
        if (S != 0 && p.nx % 2 == 0 && fits) {  // 16-bit storage: node pairs in lattice order
            hipExtLaunchKernelGGL(k_bulk_pair<S>, dim3(cdiv(cdiv(p.N, 128), BULK_WAVES)), dim3(64 * BULK_WAVES), lds,
                                  a.stream, a.ev_start, a.ev_stop, 0, p, (const T *)A, B, (const uint8_t *)a.skip,
                                  &a.cnt->err);
            return;
        }
        if (p.nx % 64 != 0 && p.N < (1ll << 31)) {  // rows not a multiple of a wave: lattice order
            hipExtLaunchKernelGGL(k_bulk_flat<S>, dim3(cdiv(cdiv(p.N, 64), BULK_WAVES)), dim3(64 * BULK_WAVES), lds,
                                  a.stream, a.ev_start, a.ev_stop, 0, p, (const T *)A, B, (const uint8_t *)a.skip,
                                  &a.cnt->err);
            return;
        }
        const int nseg = cdiv(p.nx, 64);
        const long long waves = (long long)nseg * p.ny * p.nz;
        if (fits)
            hipExtLaunchKernelGGL(k_bulk<S>, dim3(cdiv(waves, BULK_WAVES)), dim3(64 * BULK_WAVES), lds, a.stream,
                                  a.ev_start, a.ev_stop, 0, p, (const T *)A, B, (const uint8_t *)a.skip, nseg,
                                  &a.cnt->err);
        else
            hipExtLaunchKernelGGL(k_bulk_wide<S>, dim3(cdiv(waves, BULK_WAVES)), dim3(64 * BULK_WAVES), lds, a.stream,
                                  a.ev_start, a.ev_stop, 0, p, (const T *)A, B, (const uint8_t *)a.skip, nseg,
                                  &a.cnt->err);
    } else if (a.phase == PHASE_SPECIAL) {
        if (p.np > 0)
            hipExtLaunchKernelGGL(k_special<S>, dim3(spec_grid), dim3(256), 0, a.stream, a.ev_start, a.ev_stop, 0,
                                  p, (const T *)A, B, (const int32_t *)a.own_old, (const DevParticle *)a.P,
                                  (const uint32_t *)a.special, a.cnt, a.in_place);
        else if (a.ev_stop)
            (void)hipEventRecord(a.ev_stop, a.stream);
    } else if (a.phase == PHASE_LINKBUILD) {
        if (p.np > 0) {
            k_link_emit_tiles<<<region_grid(p), BLK, 0, a.stream>>>(p, a.rm, a.P, a.lmask, a.blk_cnt, a.body_stats,
                                                                     a.part_first_blk, a.l_off, a.l_node, a.l_do,
                                                                     a.cnt);
            const int qg = link_q_grid(p);
            if (a.warm) {  // the network's guesses over the list, then the solve
                k_link_guess<<<min(cdiv(expected_links(p), 128), LINK_GUESS_BLOCKS), 256, 0, a.stream>>>(
                    p, a.P, a.l_node, a.l_do, a.cnt, a.warm, a.mlp_body, a.l_q);
                k_link_q<true><<<qg, 256, 0, a.stream>>>(p, a.P, a.l_node, a.l_do, a.l_q, a.cnt, a.nrs, a.warm);
            } else
                k_link_q<false><<<qg, 256, 0, a.stream>>>(p, a.P, a.l_node, a.l_do, a.l_q, a.cnt, a.nrs, nullptr);
        }
    } else if (a.phase == PHASE_INIT_STATE) {
        k_init_state<S><<<2048, 256, 0, a.stream>>>(p, A, a.own_old);
    } else if (a.phase == PHASE_COLLIDE_STORED) {
        k_collide_stored<S><<<2048, 256, 0, a.stream>>>(p, A, a.own_old);
    }
}

void launch_phase(const StepArgs &a) {
    switch (a.p.storage) {
        case 0: launch_step_kernels_t<0>(a); break;
        case 1: launch_step_kernels_t<1>(a); break;
        default: launch_step_kernels_t<2>(a); break;
    }
}

void launch_fill_i32(int32_t *a, long long n, int32_t v, hipStream_t s) {
    k_fill_i32<<<2048, 256, 0, s>>>(a, n, v);
}
void launch_fill_u8(uint8_t *a, long long n, uint8_t v, hipStream_t s) {
    k_fill_u8<<<2048, 256, 0, s>>>(a, n, v);
}
template <int S>
static void launch_bulk_batch_t(int bw, const BulkCase *cases, const int *blk_case, int nblocks, int parity,
                                hipStream_t s) {
    if (nblocks <= 0) return;
    if (bw == 4) k_bulk_batch<S, 4><<<nblocks, 256, bulk_lds_reserve(4), s>>>(cases, blk_case, parity);
    else k_bulk_batch<S, 8><<<nblocks, 512, bulk_lds_reserve(8), s>>>(cases, blk_case, parity);
}

void launch_bulk_batch(int storage, int bw, const BulkCase *cases, const int *blk_case, int nblocks, int parity,
                       hipStream_t s) {
    if (storage == 1) launch_bulk_batch_t<1>(bw, cases, blk_case, nblocks, parity, s);
    else if (storage == 2) launch_bulk_batch_t<2>(bw, cases, blk_case, nblocks, parity, s);
    else launch_bulk_batch_t<0>(bw, cases, blk_case, nblocks, parity, s);
}

template <int S>
static void launch_case_batch_t(BatchOp op, const CaseArgs *cs, const int *map, int nblocks, hipStream_t s) {
    switch (op) {
        case OP_LINKS: k_links_batch<S><<<nblocks, 256, 0, s>>>(cs, map); break;
        case OP_REDUCE: k_reduce_batch<<<nblocks, 256, 0, s>>>(cs, map); break;
        case OP_RIGID: k_rigid_batch<<<nblocks, 256, 0, s>>>(cs, map); break;
        case OP_MARK: k_region_mark_batch<<<nblocks, BLK, 0, s>>>(cs, map); break;
        case OP_CLASSIFY: k_region_classify_batch<S><<<nblocks, BLK, 0, s>>>(cs, map); break;
        case OP_EMIT: k_link_emit_batch<<<nblocks, BLK, 0, s>>>(cs, map); break;
        case OP_LINKQ: k_link_q_batch<false><<<nblocks, 256, 0, s>>>(cs, map); break;
        case OP_LINKQ_WARM:  // guesses of the systems with a network, then every solve
            k_link_guess_batch<<<nblocks, 256, 0, s>>>(cs, map);
            k_link_q_batch<true><<<nblocks, 256, 0, s>>>(cs, map);
            break;
    }
}

void launch_case_batch(int storage, BatchOp op, const CaseArgs *cs, const int *map, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return;
    if (storage == 1) launch_case_batch_t<1>(op, cs, map, nblocks, s);
    else if (storage == 2) launch_case_batch_t<2>(op, cs, map, nblocks, s);
    else launch_case_batch_t<0>(op, cs, map, nblocks, s);
}

void launch_reset_counters(Counters *cnt, hipStream_t s) { k_reset_counters<<<1, 1, 0, s>>>(cnt); }
void launch_uncovered(const Params &p, const int32_t *own_old, const int32_t *own_new, uint32_t *special,
                      Counters *cnt, int *body_stats, hipStream_t s) {
    if (p.np > 0) k_uncovered<<<2048, 256, 0, s>>>(p, own_old, own_new, special, cnt, body_stats);
}
void launch_refresh_pose(const Params &p, DevParticle *P, int fresh, hipStream_t s) {
    if (p.np > 0) k_refresh_pose<<<cdiv(p.np, 64), 64, 0, s>>>(p, P, fresh);
}

}  // namespace mdl
