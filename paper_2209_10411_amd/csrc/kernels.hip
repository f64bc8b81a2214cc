// HIP kernels of the coupled metaball / lattice Boltzmann step for CDNA4
// (gfx950).  The paper (arXiv 2209.10411) defines the operations; the GPU
// organisation is this library's own:
//   k_links          one thread per cut link: bounce-back value (simple or the
//                    paper's interpolated rule, sec. 2.3.2 Eqs. eqneq1-neqd)
//                    and the link's momentum exchange in FP64
//   k_reduce_rigid   one block per particle: fixed-order FP64 sum of the link
//                    momenta, then the Newton-Euler update (sec. 2.3.1)
//   k_region_*       per-particle cubes: metaball flags (sec. 2.1), node
//                    classes and the list of nodes needing the slow path
//   k_bulk           every plain fluid node: pull-stream + BGK/Guo collide,
//                    branch-free apart from the one class byte (HBM-bound)
//   k_special        boundary and uncovered nodes: pull with bounce-back or
//                    refill (sec. 2.3.2, refilling equation), then collide
//   k_link_*         cut-link list of the new geometry, link fractions q by
//                    a safeguarded Newton iteration in FP64
// Populations are deviations f_i - w_i rho0 in FP32, FP16 or BF16 storage;
// collisions run in FP32, everything geometric or mechanical in FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "launch.h"

namespace mdl {

// ------------------------------------------------------------------ storage
template <int S> struct Store;
template <> struct Store<0> {
    using T = float;
    __device__ static float ld(const T *p, long long i, float) { return p[i]; }
    __device__ static void st(T *p, long long i, float v, float) { p[i] = v; }
};
template <> struct Store<1> {
    using T = _Float16;
    __device__ static float ld(const T *p, long long i, float inv) { return (float)p[i] * inv; }
    __device__ static void st(T *p, long long i, float v, float s) { p[i] = (_Float16)(v * s); }
};
template <> struct Store<2> {
    using T = uint16_t;
    __device__ static float ld(const T *p, long long i, float) {
        return __uint_as_float((uint32_t)p[i] << 16);
    }
    __device__ static void st(T *p, long long i, float v, float) {
        uint32_t u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
        p[i] = (uint16_t)(u >> 16);
    }
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

__device__ __forceinline__ void node_xyz(const Params &p, long long n, int &x, int &y, int &z) {
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

__device__ __forceinline__ void min_image(const Params &p, double d[3]) {
    const double L[3] = {(double)p.nx, (double)p.ny, (double)p.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (p.periodic & (1u << a)) d[a] -= L[a] * floor(d[a] / L[a] + 0.5);
}

// Metaball function (Eq. metaballM) of one body at a lab point, minimum
// image on periodic axes; a control point exactly on x gives +inf.
__device__ double metaball(const Params &p, const DevParticle &P, const double x[3]) {
#pragma clang fp contract(off)
    double C = 0.0;
    for (int i = 0; i < P.n_cp; ++i) {
        double d[3] = {x[0] - P.cpl[i][0], x[1] - P.cpl[i][1], x[2] - P.cpl[i][2]};
        min_image(p, d);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.0) return __builtin_inf();
        C += P.k[i] / r2;
    }
    return C;
}

// C and dC/ds along x(s) = xf - s e.
__device__ void metaball_ds(const Params &p, const DevParticle &P, const double xf[3], const int e[3],
                            double s, double &C, double &dC) {
#pragma clang fp contract(off)
    C = 0.0; dC = 0.0;
    for (int i = 0; i < P.n_cp; ++i) {
        double d[3] = {xf[0] - s * e[0] - P.cpl[i][0], xf[1] - s * e[1] - P.cpl[i][1],
                       xf[2] - s * e[2] - P.cpl[i][2]};
        min_image(p, d);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.0) { C = __builtin_inf(); dC = 0.0; return; }
        const double kr = P.k[i] / r2;
        C += kr;
        dC += 2.0 * kr / r2 * (d[0] * e[0] + d[1] * e[1] + d[2] * e[2]);
    }
}

// Link fraction (sec. 2.3.2): first root of g(s) = C(xf - s e) - 1 on (0,1].
// The root is bracketed in the first of 8 equal sub-intervals where g changes
// sign, then refined by Newton steps that fall back to bisection whenever a
// step leaves the bracket.  'guess' (in [0,1], or < 0 for none) replaces the
// regula-falsi start.  Returns the number of Newton/bisection iterations.
__device__ int link_fraction(const Params &p, const DevParticle &P, int x, int y, int z, int i,
                             double guess, double &q) {
    const double xf[3] = {(double)x, (double)y, (double)z};
    const int e[3] = {EX[i], EY[i], EZ[i]};
    double lo = 0.0, hi = 1.0, glo = -1.0, ghi = 0.0;
    {
        double C, dC;
        metaball_ds(p, P, xf, e, 0.0, C, dC);
        glo = C - 1.0;
    }
    for (int k = 1; k <= 8; ++k) {
        const double s = (double)k / 8.0;
        double C, dC;
        metaball_ds(p, P, xf, e, s, C, dC);
        if (C >= 1.0) { hi = s; ghi = C - 1.0; break; }
        lo = s; glo = C - 1.0;
    }
    double s;
    if (guess > lo && guess < hi) s = guess;
    else if (ghi < __builtin_inf()) s = lo + (hi - lo) * (-glo) / (ghi - glo);
    else s = 0.5 * (lo + hi);
    if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
    int it = 0;
    for (; it < 100; ++it) {
        double C, dC;
        metaball_ds(p, P, xf, e, s, C, dC);
        const double g = C - 1.0;
        if (g >= 0.0) hi = s; else lo = s;
        if (hi - lo <= 4e-16) break;
        double sn = (dC != 0.0) ? s - g / dC : 0.5 * (lo + hi);
        if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        if (fabs(sn - s) <= 1e-15) { s = sn; break; }
        s = sn;
    }
    q = s;
    return it + 1;
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double feq64(int i, double rho, const double u[3]) {
    const double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return WD[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

// Density and velocity of a stored (post-collision) node in FP64:
// rho = rho0 + sum d, u = sum e d / rho - g/2 (the collision added F).
template <int S>
__device__ void moments64(const Params &p, const typename Store<S>::T *A, long long n, double &rho,
                          double u[3]) {
    double dr = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double d = (double)Store<S>::ld(A, (long long)i * p.N + n, p.inv_scale);
        dr += d;
        j[0] += EX[i] * d; j[1] += EY[i] * d; j[2] += EZ[i] * d;
    }
    rho = p.rho0 + dr;
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho - 0.5 * p.gfd[a];
}

// ------------------------------------------------------------------ kernels
template <int S>
__global__ __launch_bounds__(256) void k_links(Params p, const typename Store<S>::T *__restrict__ A,
                                               typename Store<S>::T *__restrict__ B,
                                               const int32_t *__restrict__ own,
                                               const DevParticle *__restrict__ P,
                                               const uint32_t *__restrict__ l_node,
                                               const uint32_t *__restrict__ l_do,
                                               const double *__restrict__ l_q, double *__restrict__ lft,
                                               const Counters *__restrict__ cnt) {
    const int nl = cnt->n_links;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nl; l += gridDim.x * blockDim.x) {
        const long long n = l_node[l];
        const int i = (int)(l_do[l] & 31u), pi = (int)(l_do[l] >> 8);
        const int ib = OPP[i];
        const DevParticle &B0 = P[pi];
        int x, y, z;
        node_xyz(p, n, x, y, z);
        long long ff = -1;
        const bool ibb = p.bc == 1 && nbr(p, x, y, z, EX[i], EY[i], EZ[i], ff) && own[ff] == FLUID;
        const double q = ibb ? l_q[l] : 0.5;
        double r[3] = {x - q * EX[i] - B0.X[0], y - q * EY[i] - B0.X[1], z - q * EZ[i] - B0.X[2]};
        min_image(p, r);
        double uw[3];
        cross3(B0.w, r, uw);
        for (int a = 0; a < 3; ++a) uw[a] += B0.v[a];
        const double w = WD[i];
        const double fb = w * p.rho0 + (double)Store<S>::ld(A, (long long)ib * p.N + n, p.inv_scale);
        const double mw = 6.0 * w * p.rho0 * (EX[i] * uw[0] + EY[i] * uw[1] + EZ[i] * uw[2]);
        double val;
        if (!ibb) {
            val = fb + mw;
        } else {
            double rf, uf[3], rff, uff[3], ud[3];
            moments64<S>(p, A, n, rf, uf);
            moments64<S>(p, A, ff, rff, uff);
            for (int a = 0; a < 3; ++a) {
                const double us = q <= 0.5 ? 2.0 * q * uf[a] + (1.0 - 2.0 * q) * uff[a]
                                           : (1.0 - q) / q * uf[a] + (2.0 * q - 1.0) / q * uw[a];
                const double uss = (1.0 - q) / (1.0 + q) * uff[a] + 2.0 * q / (1.0 + q) * uw[a];
                ud[a] = us / 3.0 + 2.0 * uss / 3.0;
            }
            val = feq64(ib, rf, ud) + fb - feq64(ib, rf, uf) + mw;
        }
        Store<S>::st(B, (long long)i * p.N + n, (float)(val - w * p.rho0), p.scale);
        double dP[3], dT[3];
        dP[0] = (EX[ib] - uw[0]) * fb - (EX[i] - uw[0]) * val;
        dP[1] = (EY[ib] - uw[1]) * fb - (EY[i] - uw[1]) * val;
        dP[2] = (EZ[ib] - uw[2]) * fb - (EZ[i] - uw[2]) * val;
        cross3(r, dP, dT);
        double *o = lft + 6ll * l;
        o[0] = dP[0]; o[1] = dP[1]; o[2] = dP[2]; o[3] = dT[0]; o[4] = dT[1]; o[5] = dT[2];
    }
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

// Lab-frame control points and the region origin of the current pose.
__device__ void refresh_pose(const Params &p, DevParticle &P) {
    double R[9];
    quat_rot(P.q, R);
    for (int i = 0; i < P.n_cp; ++i)
        for (int a = 0; a < 3; ++a)
            P.cpl[i][a] = P.X[a] + R[3 * a] * P.cpb[i][0] + R[3 * a + 1] * P.cpb[i][1] + R[3 * a + 2] * P.cpb[i][2];
    const int L[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a)
        P.lo[a] = P.full[a] ? 0 : (int)floor(P.X[a]) - P.half;
    (void)L;
}

// Semi-implicit Euler over n_sub sub-steps with the hydrodynamic load held;
// spin by the body-frame Euler equation with the full inertia tensor; the
// attitude advances by the exact rotation of the sub-step's spin.
__device__ void rigid_update(const Params &p, DevParticle &P) {
    const double dt = 1.0 / p.n_sub;
    for (int s = 0; s < p.n_sub; ++s) {
        if (P.mode == 1) {
            const double phi[3] = {P.w[0] * dt, P.w[1] * dt, P.w[2] * dt};
            double dq[4];
            for (int a = 0; a < 3; ++a) P.X[a] += P.v[a] * dt;
            quat_of_rotvec(phi, dq);
            quat_mul(dq, P.q, P.q);
        } else {
            for (int a = 0; a < 3; ++a) {
                const double Ft = P.F[a] + (P.m - p.rho0 * P.V) * p.gp[a];
                P.v[a] += Ft / P.m * dt;
                P.X[a] += P.v[a] * dt;
            }
            double R[9], Tb[3], wb[3], Iw[3], gy[3];
            quat_rot(P.q, R);
            for (int a = 0; a < 3; ++a) {
                Tb[a] = R[a] * P.T[0] + R[3 + a] * P.T[1] + R[6 + a] * P.T[2];
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
    }
}

// One block per particle: fixed-order FP64 sum of the link momenta, then the
// rigid-body update (move != 0).  Block 0 also clears the per-step counters.
__global__ __launch_bounds__(256) void k_reduce_rigid(Params p, DevParticle *__restrict__ P,
                                                      const int *__restrict__ l_off,
                                                      const double *__restrict__ lft,
                                                      Counters *__restrict__ cnt, int move) {
    __shared__ double red[6][256];
    const int pi = blockIdx.x, t = threadIdx.x;
    if (pi == 0 && t == 0) { cnt->n_special = 0; cnt->n_refill = 0; cnt->n_solid = 0; }
    if (pi >= p.np) return;
    double s[6] = {0, 0, 0, 0, 0, 0};
    const int a = l_off[pi], b = l_off[pi + 1];
    for (int l = a + t; l < b; l += 256)
        for (int c = 0; c < 6; ++c) s[c] += lft[6ll * l + c];
    for (int c = 0; c < 6; ++c) red[c][t] = s[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int c = 0; c < 6; ++c) red[c][t] += red[c][t + h];
        __syncthreads();
    }
    if (t != 0) return;
    DevParticle &B = P[pi];
    for (int c = 0; c < 3; ++c) { B.F[c] = red[c][0]; B.T[c] = red[3 + c][0]; }
    if (!move) return;
    const double X0[3] = {B.X[0], B.X[1], B.X[2]};
    rigid_update(p, B);
    double d2 = 0.0;
    bool finite = true;
    for (int c = 0; c < 3; ++c) {
        d2 += (B.X[c] - X0[c]) * (B.X[c] - X0[c]);
        finite = finite && isfinite(B.X[c]) && isfinite(B.v[c]) && isfinite(B.w[c]);
    }
    if (!finite) atomicOr(&cnt->err, ERR_NONFINITE);
    else if (d2 > 1.0) atomicOr(&cnt->err, ERR_FAST_PARTICLE);
    // wrap the centroid into the box on periodic axes
    const int L[3] = {p.nx, p.ny, p.nz};
    for (int c = 0; c < 3; ++c)
        if ((p.periodic >> c) & 1u) {
            if (B.X[c] < 0.0) B.X[c] += L[c];
            else if (B.X[c] >= L[c]) B.X[c] -= L[c];
        }
    refresh_pose(p, B);
}

__global__ void k_refresh_pose(Params p, DevParticle *P) {
    const int pi = blockIdx.x * blockDim.x + threadIdx.x;
    if (pi < p.np) refresh_pose(p, P[pi]);
}

// Region node of a region kernel thread; false if outside the region or the
// domain.
__device__ __forceinline__ bool region_node(const Params &p, const RegionMap &rm,
                                            const DevParticle *P, int &pi, int &x, int &y, int &z,
                                            long long &n) {
    pi = rm.part[blockIdx.x];
    const int local = rm.first[blockIdx.x] + threadIdx.x;
    const int dx = rm.dims[3 * pi], dy = rm.dims[3 * pi + 1], dz = rm.dims[3 * pi + 2];
    if (local >= dx * dy * dz) return false;
    const int lx = local % dx, t = local / dx, ly = t % dy, lz = t / dy;
    const DevParticle &B = P[pi];
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

__global__ __launch_bounds__(BLK) void k_region_clear(Params p, RegionMap rm, const DevParticle *P,
                                                      int32_t *own_new) {
    int pi, x, y, z;
    long long n;
    if (region_node(p, rm, P, pi, x, y, z, n)) own_new[n] = FLUID;
}

__global__ __launch_bounds__(BLK) void k_region_mark(Params p, RegionMap rm, const DevParticle *P,
                                                     int32_t *own_new) {
    int pi, x, y, z;
    long long n;
    if (!region_node(p, rm, P, pi, x, y, z, n)) return;
    const double xp[3] = {(double)x, (double)y, (double)z};
    if (metaball(p, P[pi], xp) >= 1.0) atomicMin(&own_new[n], pi);
}

// Node classes: solid before / after, and "has cut links before" (a fluid
// node with an in-domain solid neighbour).  Fluid-after nodes that were solid
// or had links go to the special list.  Each node is handled once per pass
// (claimed through the stamp array) although regions may overlap.
__global__ __launch_bounds__(BLK) void k_region_classify(Params p, RegionMap rm, const DevParticle *P,
                                                         const int32_t *__restrict__ own_old,
                                                         const int32_t *__restrict__ own_new,
                                                         uint8_t *__restrict__ cls, uint32_t *stamp,
                                                         uint32_t tag, uint32_t *special,
                                                         Counters *cnt) {
    int pi, x, y, z;
    long long n;
    if (!region_node(p, rm, P, pi, x, y, z, n)) return;
    if (atomicExch(&stamp[n], tag) == tag) return;
    const bool so = own_old[n] != FLUID, sn = own_new[n] != FLUID;
    bool lo = false;
    if (!so) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long s;
            if (nbr(p, x, y, z, -EX[i], -EY[i], -EZ[i], s) && own_old[s] != FLUID) lo = true;
        }
    }
    cls[n] = (uint8_t)((so ? CLS_SOLID_OLD : 0) | (sn ? CLS_SOLID_NEW : 0) | (lo ? CLS_LINKS_OLD : 0));
    if (sn) atomicAdd(&cnt->n_solid, 1);
    if (!sn && (so || lo)) {
        const int k = atomicAdd(&cnt->n_special, 1);
        if (k < p.special_cap) special[k] = (uint32_t)n;
        else atomicOr(&cnt->err, ERR_SPECIAL_OVERFLOW);
        if (so) atomicAdd(&cnt->n_refill, 1);
    }
}

// Plain fluid nodes: pull-stream (periodic wrap, resting halfway walls) and
// collide.  One wave covers 64 consecutive x of one (y, z) row; blocks are
// remapped so that each XCD works through a contiguous slab of the lattice.
template <int S>
__global__ __launch_bounds__(256) void k_bulk(Params p, const typename Store<S>::T *__restrict__ A,
                                              typename Store<S>::T *__restrict__ B,
                                              const uint8_t *__restrict__ cls, int nseg, int nblk,
                                              int nblk8) {
    using T = typename Store<S>::T;
    const int b = blockIdx.x;
    const int lb = (b & 7) * nblk8 + (b >> 3);
    if (lb >= nblk) return;
    const int wave = lb * 4 + (threadIdx.x >> 6);
    const int seg = wave % nseg, row = wave / nseg;
    if (row >= p.ny * p.nz) return;
    const int x = seg * 64 + (threadIdx.x & 63);
    if (x >= p.nx) return;
    const int y = row % p.ny, z = row / p.ny;
    const int n = row * p.nx + x;
    if (cls[n]) return;
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
        const T *Ai = wall ? A + (long long)OPP[i] * p.N : A + (long long)i * p.N;
        const int src = wall ? n : (zs * p.ny + ys) * p.nx + xs;
        d[i] = Store<S>::ld(Ai, src, p.inv_scale);
    }
    collide(d, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<S>::st(B + (long long)i * p.N, n, d[i], p.scale);
}

// Boundary and uncovered nodes.  Boundary: a source inside a wall bounces off
// the resting wall, a source inside a body takes the bounce-back value that
// k_links left in B.  Uncovered (solid before): populations from fluid
// sources are kept, a missing f_i becomes f_opp(i) + 6 w rho0 e_i.u_new if the
// opposite came from a fluid node, else feq_i(rho0, u_new).  Then collide.
// in_place (refill after an external re-flag): only uncovered nodes, A == B.
template <int S>
__global__ __launch_bounds__(256) void k_special(Params p, const typename Store<S>::T *A,
                                                 typename Store<S>::T *B,
                                                 const int32_t *__restrict__ own_old,
                                                 const DevParticle *__restrict__ P,
                                                 const uint32_t *__restrict__ list,
                                                 const Counters *__restrict__ cnt, int in_place) {
    const int ns = min(cnt->n_special, p.special_cap);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ns; k += gridDim.x * blockDim.x) {
        const long long n = list[k];
        const int own_n = own_old[n];
        const bool unc = own_n != FLUID;
        if (in_place && !unc) continue;
        int x, y, z;
        node_xyz(p, n, x, y, z);
        float d[Q];
        uint32_t missing = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            long long s;
            if (!nbr(p, x, y, z, -EX[i], -EY[i], -EZ[i], s)) {
                if (unc) missing |= 1u << i;
                else d[i] = Store<S>::ld(A, (long long)OPP[i] * p.N + n, p.inv_scale);
            } else if (own_old[s] != FLUID) {
                if (unc) missing |= 1u << i;
                else d[i] = Store<S>::ld(B, (long long)i * p.N + n, p.inv_scale);
            } else {
                d[i] = Store<S>::ld(A, (long long)i * p.N + s, p.inv_scale);
            }
        }
        if (unc) {
            const DevParticle &Bd = P[own_n];
            double r[3] = {x - Bd.X[0], y - Bd.X[1], z - Bd.X[2]};
            min_image(p, r);
            double un[3];
            cross3(Bd.w, r, un);
            for (int a = 0; a < 3; ++a) un[a] += Bd.v[a];
            const double uu = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (!((missing >> i) & 1u)) continue;
                const double eu = EX[i] * un[0] + EY[i] * un[1] + EZ[i] * un[2];
                long long s2;
                if (nbr(p, x, y, z, EX[i], EY[i], EZ[i], s2) && own_old[s2] == FLUID)
                    d[i] = (float)((double)d[OPP[i]] + 6.0 * WD[i] * p.rho0 * eu);
                else
                    d[i] = (float)(WD[i] * p.rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
            }
        }
        collide(d, p);
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<S>::st(B, (long long)i * p.N + n, d[i], p.scale);
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
        for (int i = 0; i < Q; ++i) Store<S>::st(A, (long long)i * p.N + n, d[i], p.scale);
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
        for (int i = 0; i < Q; ++i) d[i] = Store<S>::ld(A, (long long)i * p.N + n, p.inv_scale);
        collide(d, p);
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<S>::st(A, (long long)i * p.N + n, d[i], p.scale);
    }
}

__global__ void k_reset_counters(Counters *cnt) {
    cnt->n_special = 0;
    cnt->n_refill = 0;
    cnt->n_solid = 0;
}

__global__ void k_fill_i32(int32_t *a, long long n, int32_t v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}
__global__ void k_fill_u8(uint8_t *a, long long n, uint8_t v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}

// Cut links of the new geometry: pass 1 counts per block.
__device__ __forceinline__ int links_of_node(const Params &p, const int32_t *own, int pi, int x, int y,
                                             int z, long long n) {
    if (own[n] != FLUID) return 0;
    int c = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        long long s;
        if (nbr(p, x, y, z, -EX[i], -EY[i], -EZ[i], s) && own[s] == pi) ++c;
    }
    return c;
}

__device__ __forceinline__ int block_sum(int v, int *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int h = BLK / 2; h > 0; h >>= 1) {
        if (t < h) sh[t] += sh[t + h];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(BLK) void k_link_count(Params p, RegionMap rm, const DevParticle *P,
                                                    const int32_t *__restrict__ own, int *blk_cnt) {
    __shared__ int sh[BLK];
    int pi, x, y, z;
    long long n;
    int c = 0;
    if (region_node(p, rm, P, pi, x, y, z, n)) c = links_of_node(p, own, pi, x, y, z, n);
    const int s = block_sum(c, sh);
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = s;
}

// Pass 2: one block scans the block counts; per-particle offsets follow from
// the first block of each particle.
__global__ __launch_bounds__(1024) void k_link_scan(Params p, const int *__restrict__ blk_cnt,
                                                    int *__restrict__ blk_off,
                                                    const int *__restrict__ part_first_blk,
                                                    int *__restrict__ l_off, Counters *cnt) {
    __shared__ int sh[1024];
    const int t = threadIdx.x, nb = p.region_blocks;
    const int per = (nb + 1023) / 1024;
    const int a = t * per, b = min(a + per, nb);
    int s = 0;
    for (int i = a; i < b; ++i) s += blk_cnt[i];
    sh[t] = s;
    __syncthreads();
    for (int h = 1; h < 1024; h <<= 1) {  // inclusive Hillis-Steele scan
        const int v = t >= h ? sh[t - h] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int run = sh[t] - s;
    for (int i = a; i < b; ++i) { blk_off[i] = run; run += blk_cnt[i]; }
    __syncthreads();
    if (t == 0) {
        const int total = sh[1023];
        if (total > p.link_cap) atomicOr(&cnt->err, ERR_LINK_OVERFLOW);
        cnt->n_links = min(total, p.link_cap);
    }
    for (int q = t; q < p.np; q += 1024) l_off[q] = min(blk_off[part_first_blk[q]], p.link_cap);
    if (t == 0) l_off[p.np] = min(sh[1023], p.link_cap);
}

// Pass 3: write the links in block order, thread order, direction order,
// with q from the safeguarded Newton iteration.
__global__ __launch_bounds__(BLK) void k_link_emit(Params p, RegionMap rm, const DevParticle *P,
                                                   const int32_t *__restrict__ own,
                                                   const int *__restrict__ blk_off,
                                                   uint32_t *__restrict__ l_node, uint32_t *__restrict__ l_do,
                                                   double *__restrict__ l_q, int *iters) {
    __shared__ int sh[BLK];
    int pi, x, y, z;
    long long n;
    int c = 0;
    const bool in = region_node(p, rm, P, pi, x, y, z, n);
    if (in) c = links_of_node(p, own, pi, x, y, z, n);
    const int t = threadIdx.x;
    sh[t] = c;
    __syncthreads();
    for (int h = 1; h < BLK; h <<= 1) {
        const int v = t >= h ? sh[t - h] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    if (!c) return;
    int o = blk_off[blockIdx.x] + sh[t] - c;
    const DevParticle &B = P[pi];
    int it_sum = 0;
#pragma unroll 1
    for (int i = 1; i < Q; ++i) {
        long long s;
        if (!(nbr(p, x, y, z, -EX[i], -EY[i], -EZ[i], s) && own[s] == pi)) continue;
        if (o < p.link_cap) {
            double q;
            it_sum += link_fraction(p, B, x, y, z, i, -1.0, q);
            l_node[o] = (uint32_t)n;
            l_do[o] = (uint32_t)i | ((uint32_t)pi << 8);
            l_q[o] = q;
        }
        ++o;
    }
    if (iters) atomicAdd(iters, it_sum);
}

// ------------------------------------------------------------ host launchers
static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

template <int S>
static void launch_step_kernels_t(const StepArgs &a) {
    using T = typename Store<S>::T;
    const Params &p = a.p;
    T *A = (T *)a.A, *B = (T *)a.B;
    const int link_grid = max(1, min(cdiv(p.link_cap, 256), 1024));
    const int spec_grid = max(1, min(cdiv(p.special_cap, 256), 1024));
    if (a.phase == PHASE_LINKS) {
        if (p.np > 0)
            k_links<S><<<link_grid, 256, 0, a.stream>>>(p, A, B, a.own_old, a.P, a.l_node, a.l_do, a.l_q,
                                                         a.lft, a.cnt);
        k_reduce_rigid<<<max(p.np, 1), 256, 0, a.stream>>>(p, a.P, a.l_off, a.lft, a.cnt, a.move);
    } else if (a.phase == PHASE_FLAGS) {
        if (p.np > 0) {
            if (a.move) {
                k_region_clear<<<p.region_blocks, BLK, 0, a.stream>>>(p, a.rm, a.P, a.own_new);
                k_region_mark<<<p.region_blocks, BLK, 0, a.stream>>>(p, a.rm, a.P, a.own_new);
            }
            k_region_classify<<<p.region_blocks, BLK, 0, a.stream>>>(p, a.rm, a.P, a.own_old, a.own_new,
                                                                      a.cls, a.stamp, a.tag, a.special,
                                                                      a.cnt);
        }
    } else if (a.phase == PHASE_BULK) {
        const int nseg = cdiv(p.nx, 64);
        const long long waves = (long long)nseg * p.ny * p.nz;
        const int nblk = cdiv(waves, 4);
        const int nblk8 = cdiv(nblk, 8);
        k_bulk<S><<<nblk8 * 8, 256, 0, a.stream>>>(p, A, B, a.cls, nseg, nblk, nblk8);
    } else if (a.phase == PHASE_SPECIAL) {
        if (p.np > 0)
            k_special<S><<<spec_grid, 256, 0, a.stream>>>(p, A, B, a.own_old, a.P, a.special, a.cnt,
                                                           a.in_place);
    } else if (a.phase == PHASE_LINKBUILD) {
        if (p.np > 0) {
            k_link_count<<<p.region_blocks, BLK, 0, a.stream>>>(p, a.rm, a.P, a.own_new, a.blk_cnt);
            k_link_scan<<<1, 1024, 0, a.stream>>>(p, a.blk_cnt, a.blk_off, a.part_first_blk, a.l_off, a.cnt);
            k_link_emit<<<p.region_blocks, BLK, 0, a.stream>>>(p, a.rm, a.P, a.own_new, a.blk_off,
                                                                a.l_node, a.l_do, a.l_q, a.iters);
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
void launch_reset_counters(Counters *cnt, hipStream_t s) { k_reset_counters<<<1, 1, 0, s>>>(cnt); }
void launch_refresh_pose(const Params &p, DevParticle *P, hipStream_t s) {
    if (p.np > 0) k_refresh_pose<<<cdiv(p.np, 64), 64, 0, s>>>(p, P);
}

}  // namespace mdl
