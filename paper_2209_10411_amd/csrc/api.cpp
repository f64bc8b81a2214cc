// Host side of the C ABI declared in include/midelbm.h: validation, body
// properties, arena layout, and the order in which the kernels of one
// coupled step are enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/midelbm.h"
#include "device.h"
#include "launch.h"
#include "min_image.h"
#include "mlp_dev.h"

using namespace mdl;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// value of "key": <number> in a small flat JSON text (false if absent)
bool json_num(const std::string &txt, const char *key, double &v) {
    const std::string pat = std::string("\"") + key + "\"";
    size_t at = txt.find(pat);
    if (at == std::string::npos) return false;
    at = txt.find(':', at + pat.size());
    if (at == std::string::npos) return false;
    char *end = nullptr;
    const double r = std::strtod(txt.c_str() + at + 1, &end);
    if (end == txt.c_str() + at + 1) return false;
    v = r;
    return true;
}

// Body properties by midpoint quadrature: cells of size h on a grid centred
// on the box [min p - sqrt(sum k), max p + sqrt(sum k)] (C >= 1 needs some
// |x - p_i|^2 <= sum k).  Volume, centroid (from exact integer index sums)
// and inertia tensor per unit density about the centroid.
struct BodyProps {
    double V, c[3], I[9];
    double re;  // radius about the centroid enclosing the inside cells, plus a cell diagonal and 1/2 lu
};

bool body_properties(int n_cp, const double *cp, const double *k, double h, BodyProps &out) {
    double sk = 0;
    for (int i = 0; i < n_cp; ++i) sk += k[i];
    const double rs = std::sqrt(sk);
    double lo[3];
    int n[3];
    for (int a = 0; a < 3; ++a) {
        double mn = cp[a], mx = cp[a];
        for (int i = 1; i < n_cp; ++i) {
            mn = std::min(mn, cp[3 * i + a]);
            mx = std::max(mx, cp[3 * i + a]);
        }
        mn -= rs; mx += rs;
        n[a] = (int)std::ceil((mx - mn) / h);
        lo[a] = 0.5 * (mn + mx) - 0.5 * n[a] * h;
    }
    auto inside = [&](double x, double y, double z) {
        double C = 0;
        for (int i = 0; i < n_cp; ++i) {
            const double dx = x - cp[3 * i], dy = y - cp[3 * i + 1], dz = z - cp[3 * i + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0) return true;
            C += k[i] / r2;
        }
        return C >= 1.0;
    };
    const int nth = 8;  // fixed chunking: results do not depend on the host
    std::vector<long long> cnt(nth, 0), sx(nth, 0), sy(nth, 0), sz(nth, 0);
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t] {
            for (int kz = t; kz < n[2]; kz += nth)
                for (int ky = 0; ky < n[1]; ++ky)
                    for (int kx = 0; kx < n[0]; ++kx)
                        if (inside(lo[0] + (kx + 0.5) * h, lo[1] + (ky + 0.5) * h, lo[2] + (kz + 0.5) * h)) {
                            ++cnt[t]; sx[t] += kx; sy[t] += ky; sz[t] += kz;
                        }
        });
    for (auto &x : th) x.join();
    th.clear();
    long long C = 0, S[3] = {0, 0, 0};
    for (int t = 0; t < nth; ++t) { C += cnt[t]; S[0] += sx[t]; S[1] += sy[t]; S[2] += sz[t]; }
    if (C == 0) return false;
    for (int a = 0; a < 3; ++a) out.c[a] = lo[a] + h * ((double)S[a] / (double)C + 0.5);
    std::vector<double> J(6 * nth, 0.0), R2(nth, 0.0);
    for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t] {
            double *j = &J[6 * t];
            double &rmax = R2[t];
            for (int kz = t; kz < n[2]; kz += nth)
                for (int ky = 0; ky < n[1]; ++ky)
                    for (int kx = 0; kx < n[0]; ++kx) {
                        const double x = lo[0] + (kx + 0.5) * h, y = lo[1] + (ky + 0.5) * h,
                                     z = lo[2] + (kz + 0.5) * h;
                        if (!inside(x, y, z)) continue;
                        const double r0 = x - out.c[0], r1 = y - out.c[1], r2 = z - out.c[2];
                        rmax = std::max(rmax, r0 * r0 + r1 * r1 + r2 * r2);
                        j[0] += r0 * r0; j[1] += r1 * r1; j[2] += r2 * r2;
                        j[3] += r0 * r1; j[4] += r0 * r2; j[5] += r1 * r2;
                    }
        });
    for (auto &x : th) x.join();
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int t = 0; t < nth; ++t)
        for (int c = 0; c < 6; ++c) s[c] += J[6 * t + c];
    double rm = 0.0;
    for (int t = 0; t < nth; ++t) rm = std::max(rm, R2[t]);
    out.re = std::sqrt(rm) + h * std::sqrt(3.0) + 0.5;
    const double h3 = h * h * h;
    out.V = (double)C * h3;
    out.I[0] = (s[1] + s[2]) * h3; out.I[4] = (s[0] + s[2]) * h3; out.I[8] = (s[0] + s[1]) * h3;
    out.I[1] = out.I[3] = -s[3] * h3;
    out.I[2] = out.I[6] = -s[4] * h3;
    out.I[5] = out.I[7] = -s[5] * h3;
    return true;
}

bool invert3(const double *A, double *B) {
    const double d = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(std::fabs(d) > 0)) return false;
    B[0] = (A[4] * A[8] - A[5] * A[7]) / d; B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / d; B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / d; B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / d; B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
    return true;
}

void rot_of_quat(const double *q, double *R) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

bool finite_all(const double *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// Everything the arena holds, in order.  Offsets are computed once from the
// configuration; lbm_arena_bytes and lbm_init share this plan.
struct Plan {
    long long N;
    long long Ns;  // N rounded up to POP_RUN (the population buffer holds Q * Ns elements)
    int np;
    int storage_bytes;
    int region_blocks;
    int link_cap, special_cap;
    std::vector<int> dims;            // [np][3]
    std::vector<int> part, first;     // [region_blocks]
    std::vector<int> part_first_blk;  // [np]
    std::vector<int> half;            // [np]
    size_t off_A, off_B, off_own[3], off_skip[2], off_P, off_part, off_first, off_dims,
        off_pfb, off_bcnt, off_blinks, off_loff, off_lnode, off_ldo, off_lq, off_lpart, off_special,
        off_cnt, total;
    bool contact;
    size_t off_lmask, off_nrs, off_mlpb;
    size_t off_pairF, off_pairTi, off_pairTj, off_wallF, off_wallT, off_xiP, off_xiW, off_pairOn, off_pairXm,
        off_pairOk, off_pairGuess;
};

struct HostParticle {
    DevParticle d;
};

lbm_status validate_config(const lbm_config *c) {
    if (!c) return fail(LBM_E_INVALID, "config is NULL");
    if (c->nx < 3 || c->ny < 3 || c->nz < 3) return fail(LBM_E_INVALID, "lattice sizes must be >= 3");
    const long long N = (long long)c->nx * c->ny * c->nz;
    if (N > 0x7fffffffll) return fail(LBM_E_INVALID, "lattice has more than 2^31-1 nodes");
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return fail(LBM_E_INVALID, "tau must be > 0.5");
    if (!(c->rho0 > 0) || !std::isfinite(c->rho0)) return fail(LBM_E_INVALID, "rho0 must be > 0");
    if (!finite_all(c->g_fluid, 3) || !finite_all(c->g_particle, 3))
        return fail(LBM_E_INVALID, "non-finite gravity");
    if (c->storage < 0 || c->storage > 2) return fail(LBM_E_INVALID, "unknown storage %d", c->storage);
    if (c->bc < 0 || c->bc > 1) return fail(LBM_E_INVALID, "unknown boundary rule %d", c->bc);
    if (c->n_sub < 1) return fail(LBM_E_INVALID, "n_sub must be >= 1");
    if (!(c->quad_h > 0) || !std::isfinite(c->quad_h)) return fail(LBM_E_INVALID, "quad_h must be > 0");
    if (c->contact_kn < 0.0 || !std::isfinite(c->contact_kn)) return fail(LBM_E_INVALID, "contact_kn must be >= 0");
    if (c->contact_kn > 0.0) {
        if (!(c->contact_rs > 0.0) || !std::isfinite(c->contact_rs)) return fail(LBM_E_INVALID, "contact_rs must be > 0");
        if (!(c->contact_en > 0.0 && c->contact_en <= 1.0)) return fail(LBM_E_INVALID, "contact_en must be in (0, 1]");
        if (!(c->contact_mu >= 0.0) || !std::isfinite(c->contact_mu)) return fail(LBM_E_INVALID, "contact_mu must be >= 0");
    }
    if (c->link_c0 != 0 && c->link_c0 != 1) return fail(LBM_E_INVALID, "link_c0 must be 0 or 1");
    if (c->link_c0 && (!(c->contact_rs > 0.0) || !std::isfinite(c->contact_rs)))
        return fail(LBM_E_INVALID, "link_c0 needs contact_rs > 0");
    if (c->storage == 1 && c->fp16_scale != 0.f) {
        int e;
        const float m = std::frexp(c->fp16_scale, &e);
        if (!(c->fp16_scale > 0) || m != 0.5f) return fail(LBM_E_INVALID, "fp16_scale must be a power of two");
    }
    return LBM_OK;
}

lbm_status validate_particle(const lbm_config *c, const lbm_particle *p, int idx) {
    if (p->n_cp < 1 || p->n_cp > MAXCP) return fail(LBM_E_INVALID, "particle %d: n_cp must be 1..%d", idx, MAXCP);
    if (!p->cp_xyz || !p->cp_k) return fail(LBM_E_INVALID, "particle %d: NULL control points", idx);
    if (!finite_all(p->cp_xyz, 3 * p->n_cp)) return fail(LBM_E_INVALID, "particle %d: non-finite control point", idx);
    for (int i = 0; i < p->n_cp; ++i)
        if (!(p->cp_k[i] > 0) || !std::isfinite(p->cp_k[i]))
            return fail(LBM_E_INVALID, "particle %d: k must be > 0", idx);
    if (!finite_all(p->x, 3) || !finite_all(p->quat, 4) || !finite_all(p->v, 3) || !finite_all(p->omega, 3))
        return fail(LBM_E_INVALID, "particle %d: non-finite state", idx);
    const double qn = p->quat[0] * p->quat[0] + p->quat[1] * p->quat[1] + p->quat[2] * p->quat[2] + p->quat[3] * p->quat[3];
    if (!(qn > 0)) return fail(LBM_E_INVALID, "particle %d: zero quaternion", idx);
    if (!(p->density > 0) || !std::isfinite(p->density)) return fail(LBM_E_INVALID, "particle %d: density must be > 0", idx);
    if (p->mode != LBM_MODE_FREE && p->mode != LBM_MODE_KINEMATIC)
        return fail(LBM_E_INVALID, "particle %d: unknown mode", idx);
    (void)c;
    return LBM_OK;
}

// Bounding radius of the body about its centroid.
double bounding_radius(int n_cp, const double *cp, const double *k, const double *cen) {
    double sk = 0, rm = 0;
    for (int i = 0; i < n_cp; ++i) {
        sk += k[i];
        double r2 = 0;
        for (int a = 0; a < 3; ++a) r2 += (cp[3 * i + a] - cen[a]) * (cp[3 * i + a] - cen[a]);
        rm = std::max(rm, std::sqrt(r2));
    }
    return rm + std::sqrt(sk);
}

// rb: bounding radius (capacities); re: extent of the C >= 1 set (regions).
lbm_status make_plan(const lbm_config *c, int np, const std::vector<double> &rb, const std::vector<double> &re,
                     Plan &pl) {
    pl.N = (long long)c->nx * c->ny * c->nz;
    pl.Ns = (pl.N + POP_RUN - 1) / POP_RUN * POP_RUN;
    pl.np = np;
    pl.storage_bytes = c->storage == 0 ? 4 : 2;
    pl.dims.assign(3 * np, 0);
    pl.half.assign(np, 0);
    pl.part.clear();
    pl.first.clear();
    pl.part_first_blk.assign(np, 0);
    const int L[3] = {c->nx, c->ny, c->nz};
    long long lcap = 0, scap = 0;
    for (int p = 0; p < np; ++p) {
        const int half = (int)std::ceil(std::min(re[p], rb[p])) + PAD;
        pl.half[p] = half;
        long long vol = 1;
        for (int a = 0; a < 3; ++a) {
            int d = 2 * half + 1;
            if (((c->periodic >> a) & 1u) && d >= L[a]) d = L[a];
            if (!((c->periodic >> a) & 1u)) d = std::min(d, L[a] + 2 * half + 1);
            pl.dims[3 * p + a] = d;
            vol *= d;
        }
        if (vol > 0x7fffffffll) return fail(LBM_E_INVALID, "particle %d is too large", p);
        // blocks are tiles of TILE_X x TILE_Y x TILE_Z nodes; tiles wholly
        // outside the ball the kernels visit (radius half + 2 about the
        // cube's centre) are left out unless the region spans a periodic axis
        pl.part_first_blk[p] = (int)pl.part.size();
        const int *d = &pl.dims[3 * p];
        const int nt[3] = {(d[0] + TILE_X - 1) / TILE_X, (d[1] + TILE_Y - 1) / TILE_Y, (d[2] + TILE_Z - 1) / TILE_Z};
        const int ts[3] = {TILE_X, TILE_Y, TILE_Z};
        bool full = false;
        for (int a = 0; a < 3; ++a) full = full || d[a] != 2 * half + 1;
        const long long rr = (long long)(half + 2) * (half + 2);
        for (int tz = 0; tz < nt[2]; ++tz)
            for (int ty = 0; ty < nt[1]; ++ty)
                for (int tx = 0; tx < nt[0]; ++tx) {
                    const int t3[3] = {tx, ty, tz};
                    long long r2 = 0;
                    for (int a = 0; a < 3; ++a) {
                        const int lo = t3[a] * ts[a], hi = lo + ts[a] - 1;
                        const int q = std::min(std::max(half, lo), hi);
                        r2 += (long long)(q - half) * (q - half);
                    }
                    if (!full && r2 > rr) continue;
                    pl.part.push_back(p);
                    pl.first.push_back(tx + nt[0] * (ty + nt[1] * tz));
                }
        const double area = 4.0 * M_PI * (rb[p] + 2.0) * (rb[p] + 2.0);
        lcap += (long long)(12.0 * area) + 4096;
        scap += (long long)(4.0 * area) + 4096;
    }
    if (lcap > 0x3fffffffll || scap > 0x3fffffffll) return fail(LBM_E_INVALID, "particles too large");
    pl.region_blocks = (int)pl.part.size();
    pl.link_cap = (int)lcap;
    pl.special_cap = (int)scap;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const size_t pop = (size_t)Q * pl.Ns * pl.storage_bytes;
    pl.off_A = take(pop);
    pl.off_B = take(pop);
    for (int k = 0; k < 3; ++k) pl.off_own[k] = take(4 * pl.N);
    pl.off_skip[0] = take(pl.N);
    pl.off_skip[1] = take(pl.N);
    pl.off_P = take(sizeof(DevParticle) * std::max(np, 1));
    pl.off_part = take(4 * std::max(pl.region_blocks, 1));
    pl.off_first = take(4 * std::max(pl.region_blocks, 1));
    pl.off_dims = take(4 * 3 * std::max(np, 1));
    pl.off_pfb = take(4 * std::max(np, 1));
    pl.off_bcnt = take(4 * std::max(pl.region_blocks, 1));
    pl.off_blinks = take(16 * (size_t)std::max(np, 1));
    pl.off_lmask = take(4 * (size_t)BLK * std::max(pl.region_blocks, 1));
    pl.off_loff = take(4 * (np + 1));
    pl.off_lnode = take(4 * (size_t)std::max(pl.link_cap, 1));
    pl.off_ldo = take(4 * (size_t)std::max(pl.link_cap, 1));
    pl.off_lq = take(8 * (size_t)std::max(pl.link_cap, 1));
    // per-chunk, per-body partial momentum sums: chunk + body < cap/256 + 1 + np
    pl.off_lpart = take(48 * ((size_t)pl.link_cap / 64 + 2 + np));  // a slot per (64-link chunk, body)
    pl.off_special = take(4 * (size_t)std::max(pl.special_cap, 1));
    pl.contact = c->contact_kn > 0.0 && np > 0;
    const size_t npp = pl.contact ? (size_t)np * np : 1, npw = pl.contact ? (size_t)np * 6 : 1;
    pl.off_pairF = take(24 * npp);
    pl.off_pairTi = take(24 * npp);
    pl.off_pairTj = take(24 * npp);
    pl.off_wallF = take(24 * npw);
    pl.off_wallT = take(24 * npw);
    pl.off_xiP = take(24 * npp);
    pl.off_xiW = take(24 * npw);
    pl.off_pairOn = take(npp);
    pl.off_pairXm = take(24 * npp);
    pl.off_pairOk = take(npp);
    pl.off_pairGuess = take(32 * npp);
    pl.off_cnt = take(sizeof(Counters));
    pl.off_nrs = take(4 * (size_t)NR_BLOCKS * NR_HIST + 16 * (size_t)NR_BLOCKS + 4 * (size_t)NR_BLOCKS);
    pl.off_mlpb = take(4 * (size_t)MLP_BODY * std::max(np, 1));
    pl.total = o;
    return LBM_OK;
}

}  // namespace

struct lbm_ctx {
    lbm_config cfg;
    Plan pl;
    Params p;
    hipStream_t stream;
    char *arena;
    void *A, *B;
    int32_t *own[3];
    int ic, in, id;  // current flags, next (all FLUID), dead (previous)
    uint8_t *skip[2];
    int is;          // skip mask of the coming step
    DevParticle *P;
    RegionMap rm;
    int *part_first_blk, *blk_cnt, *body_stats, *l_off;
    uint32_t *lmask;
    uint32_t *l_node, *l_do, *special;
    double *l_q, *lpart;
    Counters *cnt;
    ContactBufs cb;
    NrStats nrs;
    float *mlp_body;            // [np][80] constant warm-start inputs of each body
    const _Float16 *warm;       // warm-start MLP parameters, or NULL
    hipStream_t aux;              // second stream: link build overlapped with stream-collide
    hipEvent_t ev_main, ev_flags, ev_links, ev_bulk;
    bool pending_refill;
    bool timing;
    int timing_every;  // time the stream-collide of every timing_every-th step
    int bulk_blocks;  // stream-collide blocks per CU (0: the default cap), from the link count
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t ev_used;
    long long timed_launches;
    double timed_ms;
    long long steps;
};

namespace {

StepArgs base_args(lbm_ctx *c) {
    StepArgs a{};
    a.p = c->p;
    a.stream = c->stream;
    a.A = c->A; a.B = c->B;
    a.own_old = c->own[c->ic]; a.own_new = c->own[c->in]; a.own_dead = nullptr;
    a.skip = c->skip[c->is]; a.skip_next = c->skip[1 - c->is];
    a.P = c->P; a.rm = c->rm;
    a.part_first_blk = c->part_first_blk;
    a.blk_cnt = c->blk_cnt; a.body_stats = c->body_stats; a.l_off = c->l_off; a.lmask = c->lmask;
    a.l_node = c->l_node; a.l_do = c->l_do; a.l_q = c->l_q; a.part = c->lpart;
    a.special = c->special; a.cnt = c->cnt; a.cb = c->cb;
    a.nrs = c->nrs; a.warm = c->warm; a.mlp_body = c->mlp_body;
    a.bulk_blocks = c->bulk_blocks;
    return a;
}

lbm_status check_device(lbm_ctx *c) {
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    Counters h;
    HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
    if (h.err & ERR_NONFINITE) return fail(LBM_E_DIVERGED, "a particle state became non-finite");
    if (h.err & ERR_FAST_PARTICLE) return fail(LBM_E_DIVERGED, "a particle moved more than one lattice unit in a step");
    if (h.err & ERR_FLUID)
        return fail(LBM_E_DIVERGED, "the fluid diverged: a fluid node had non-finite moments or |u| > 0.3");
    if (h.err & ERR_LINK_OVERFLOW) return fail(LBM_E_NOMEM, "cut-link list exceeded its capacity (%d)", c->p.link_cap);
    if (h.err & ERR_SPECIAL_OVERFLOW) return fail(LBM_E_NOMEM, "boundary-node list exceeded its capacity (%d)", c->p.special_cap);
    if (h.err & ERR_BAD_INDEX) return fail(LBM_E_STATE, "an index list held an out-of-range entry (skipped)");
    return LBM_OK;
}

// Flags from scratch for the current poses into the next buffer, node
// classes against the current one, then the links of the new flags.  The
// old flags stay in the dead buffer until refill() has used them.
// Expected lengths of the link and boundary-node lists from the current ones
// (bodies are rigid: their surface changes little), with a margin; the list
// kernels stride over whatever the lists hold.  Synchronises.
lbm_status estimate_lists(lbm_ctx *c) {
    Counters h;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
    c->p.est_links = std::min(c->p.link_cap, (int)std::min<long long>(0x3fffffff, 3ll * h.n_links / 2 + 1024));
    // Where the boundary chain outweighs the stream-collide (many cut links
    // per node: on a 256^3 box with 200 bodies, 1.45 M links for 16.8 M
    // nodes), the stream-collide leaves it more of every CU: two blocks per
    // CU there gave 1.52 against 1.64 ms per step with six; with few links
    // (7.5 k for 6.3 M nodes) six blocks keep the stream-collide at full speed.
    // The 16-bit form (84 VGPRs, two nodes per lane) does best with four:
    // its step is the boundary chain's, which runs faster with the room
    // (settling 128x128x384: 0.118 -> 0.112 ms; two bodies 160x160x640:
    // 0.262 -> 0.252 ms), while the kernel itself loses 2-3 %.
    c->bulk_blocks = 50ll * h.n_links > (long long)c->p.N ? 2 : c->p.storage != 0 ? 4 : 0;
    // boundary nodes carry several cut links each (the special list is empty
    // right after set-up, when no previous flags exist)
    c->p.est_special = std::min(c->p.special_cap,
                                (int)std::min<long long>(0x3fffffff, std::max<long long>(3ll * h.n_special / 2,
                                                                                         h.n_links / 2) + 1024));
    return LBM_OK;
}

// Node counts of the last classification, summed over the bodies (solid,
// uncovered, boundary + uncovered); synchronises.
lbm_status body_counts(lbm_ctx *c, long long &solid, long long &refilled, long long &special) {
    solid = refilled = special = 0;
    if (c->p.np == 0) return LBM_OK;
    std::vector<int> bs(4 * (size_t)c->p.np);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(bs.data(), c->body_stats, 4 * bs.size(), hipMemcpyDeviceToHost));
    for (int q = 0; q < c->p.np; ++q) {
        solid += bs[4 * q + 1];
        refilled += bs[4 * q + 2];
        special += bs[4 * q + 3];
    }
    return LBM_OK;
}

lbm_status reflag(lbm_ctx *c) {
    launch_refresh_pose(c->p, c->P, 0, c->stream);
    launch_fill_i32(c->own[c->in], c->pl.N, FLUID, c->stream);
    launch_fill_i32(c->own[c->id], c->pl.N, FLUID, c->stream);
    launch_fill_u8(c->skip[0], c->pl.N, 0, c->stream);
    launch_fill_u8(c->skip[1], c->pl.N, 0, c->stream);
    launch_reset_counters(c->cnt, c->stream);
    if (c->p.np > 0) launch_fill_i32(c->body_stats, 4ll * c->p.np, 0, c->stream);
    StepArgs a = base_args(c);
    a.phase = PHASE_FLAGS;
    a.move = 1;
    launch_phase(a);
    launch_uncovered(c->p, a.own_old, a.own_new, c->special, c->cnt, c->body_stats, c->stream);
    a.phase = PHASE_LINKBUILD;
    launch_phase(a);
    // the next steps find the new flags only (the others are cleared, the
    // pre-flag ones go with the refill)
    launch_refresh_pose(c->p, c->P, 1, c->stream);
    const int old = c->ic;
    c->ic = c->in; c->in = c->id; c->id = old;
    c->is = 1 - c->is;
    c->pending_refill = true;
    return LBM_OK;
}

lbm_status do_refill(lbm_ctx *c) {
    StepArgs a = base_args(c);
    a.phase = PHASE_SPECIAL;
    a.in_place = 1;
    a.B = c->A;                  // in place on the stored state
    a.own_old = c->own[c->id];   // flags before the last re-flag
    launch_phase(a);
    launch_fill_i32(c->own[c->id], c->pl.N, FLUID, c->stream);
    c->pending_refill = false;
    return LBM_OK;
}

}  // namespace

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

// Constant warm-start inputs of each body: its control points in the body
// frame sorted by weight (largest first, ties by index), each as
// (p / sqrt(sum k), k / sum k), zero-padded to 20 points.
static std::vector<float> mlp_body_blocks(const std::vector<DevParticle> &hp) {
    std::vector<float> out(hp.size() * MLP_BODY, 0.f);
    for (size_t q = 0; q < hp.size(); ++q) {
        const DevParticle &d = hp[q];
        double K = 0.0;
        for (int i = 0; i < d.n_cp; ++i) K += d.k[i];
        const double s = std::sqrt(K);
        std::vector<int> order(d.n_cp);
        for (int i = 0; i < d.n_cp; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d.k[a] > d.k[b]; });
        for (int r = 0; r < d.n_cp; ++r) {
            const int i = order[r];
            for (int a = 0; a < 3; ++a) out[q * MLP_BODY + 4 * r + a] = (float)(d.cpb[i][a] / s);
            out[q * MLP_BODY + 4 * r + 3] = (float)(d.k[i] / K);
        }
    }
    return out;
}

static lbm_status prepare(const lbm_config *cfg, int32_t n_p, const lbm_particle *parts,
                          std::vector<DevParticle> *hp, Plan *pl) {
    lbm_status s = validate_config(cfg);
    if (s) return s;
    if (n_p < 0 || n_p > 65535) return fail(LBM_E_INVALID, "n_p must be 0..65535");
    if (n_p > 0 && !parts) return fail(LBM_E_INVALID, "particles is NULL");
    std::vector<double> rb(n_p), re(n_p);
    hp->assign(n_p, DevParticle{});
    const int L[3] = {cfg->nx, cfg->ny, cfg->nz};
    for (int p = 0; p < n_p; ++p) {
        const lbm_particle &q = parts[p];
        if ((s = validate_particle(cfg, &q, p))) return s;
        BodyProps bp;
        if (!body_properties(q.n_cp, q.cp_xyz, q.cp_k, cfg->quad_h, bp))
            return fail(LBM_E_INVALID, "particle %d has no volume at quad_h", p);
        DevParticle &d = (*hp)[p];
        d.n_cp = q.n_cp;
        d.mode = q.mode;
        const double qn = std::sqrt(q.quat[0] * q.quat[0] + q.quat[1] * q.quat[1] + q.quat[2] * q.quat[2] + q.quat[3] * q.quat[3]);
        for (int a = 0; a < 4; ++a) d.q[a] = q.quat[a] / qn;
        double R[9];
        rot_of_quat(d.q, R);
        double ksum = 0.0;
        for (int i = 0; i < q.n_cp; ++i) {
            d.k[i] = q.cp_k[i];
            ksum += d.k[i];
            for (int a = 0; a < 3; ++a) d.cpb[i][a] = q.cp_xyz[3 * i + a] - bp.c[a];
        }
        d.rsk = 1.0 / std::sqrt(ksum);
        for (int a = 0; a < 3; ++a) {
            d.X[a] = q.x[a] + R[3 * a] * bp.c[0] + R[3 * a + 1] * bp.c[1] + R[3 * a + 2] * bp.c[2];
            d.v[a] = q.v[a];
            d.w[a] = q.omega[a];
        }
        d.V = bp.V;
        d.m = q.density * bp.V;
        for (int a = 0; a < 9; ++a) d.I[a] = q.density * bp.I[a];
        if (!invert3(d.I, d.Iinv)) {
            if (q.mode == LBM_MODE_FREE) return fail(LBM_E_INVALID, "particle %d: singular inertia", p);
            for (int a = 0; a < 9; ++a) d.Iinv[a] = 0;
        }
        d.rb = bounding_radius(q.n_cp, q.cp_xyz, q.cp_k, bp.c);
        rb[p] = d.rb;
        re[p] = bp.re;
        d.re = std::min(bp.re, d.rb);
        d.reach = 1e30;
        d.hist = 0;
        for (int a = 0; a < 3; ++a)
            if (!((cfg->periodic >> a) & 1u) && (d.X[a] - d.rb < 0.0 || d.X[a] + d.rb > L[a] - 1.0))
                return fail(LBM_E_INVALID, "particle %d: bounding sphere crosses a wall on axis %d", p, a);
    }
    if (cfg->contact_kn > 0.0) {
        if (n_p > 1024) return fail(LBM_E_INVALID, "contact supports at most 1024 particles");
        for (int p = 0; p < n_p; ++p) {
            double sk = 0;
            for (int i = 0; i < parts[p].n_cp; ++i) sk += parts[p].cp_k[i];
            if (!(cfg->contact_rs < std::sqrt(sk))) return fail(LBM_E_INVALID, "particle %d: contact_rs >= sqrt(sum k)", p);
        }
    }
    if ((s = make_plan(cfg, n_p, rb, re, *pl))) return s;
    for (int p = 0; p < n_p; ++p) {
        DevParticle &d = (*hp)[p];
        d.half = pl->half[p];
        for (int a = 0; a < 3; ++a) d.full[a] = pl->dims[3 * p + a] == L[a] && ((cfg->periodic >> a) & 1u);
    }
    return LBM_OK;
}

lbm_status lbm_arena_bytes(const lbm_config *cfg, int32_t n_p, const lbm_particle *p, size_t *bytes) {
    if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
    std::vector<DevParticle> hp;
    Plan pl;
    lbm_status s = prepare(cfg, n_p, p, &hp, &pl);
    if (s) return s;
    *bytes = pl.total;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_config *cfg, int32_t n_p, const lbm_particle *parts, void *dev_arena,
                    size_t arena_bytes, void *hip_stream, lbm_ctx **out) {
    if (!out) return fail(LBM_E_INVALID, "out is NULL");
    *out = nullptr;
    std::vector<DevParticle> hp;
    Plan pl;
    lbm_status s = prepare(cfg, n_p, parts, &hp, &pl);
    if (s) return s;
    if (!dev_arena) return fail(LBM_E_INVALID, "arena is NULL");
    if (arena_bytes < pl.total) return fail(LBM_E_NOMEM, "arena holds %zu bytes, %zu needed", arena_bytes, pl.total);
    if ((uintptr_t)dev_arena & 255) return fail(LBM_E_INVALID, "arena must be 256-byte aligned");

    lbm_ctx *c = new lbm_ctx();
    c->cfg = *cfg;
    c->pl = pl;
    c->stream = (hipStream_t)hip_stream;
    c->arena = (char *)dev_arena;
    char *b = c->arena;
    c->A = b + pl.off_A; c->B = b + pl.off_B;
    for (int k = 0; k < 3; ++k) c->own[k] = (int32_t *)(b + pl.off_own[k]);
    c->ic = 0; c->in = 1; c->id = 2;
    c->skip[0] = (uint8_t *)(b + pl.off_skip[0]);
    c->skip[1] = (uint8_t *)(b + pl.off_skip[1]);
    c->is = 0;
    c->P = (DevParticle *)(b + pl.off_P);
    c->rm.part = (const int *)(b + pl.off_part);
    c->rm.first = (const int *)(b + pl.off_first);
    c->rm.dims = (const int *)(b + pl.off_dims);
    c->part_first_blk = (int *)(b + pl.off_pfb);
    c->blk_cnt = (int *)(b + pl.off_bcnt);
    c->body_stats = (int *)(b + pl.off_blinks);
    c->lmask = (uint32_t *)(b + pl.off_lmask);
    c->l_off = (int *)(b + pl.off_loff);
    c->l_node = (uint32_t *)(b + pl.off_lnode); c->l_do = (uint32_t *)(b + pl.off_ldo);
    c->l_q = (double *)(b + pl.off_lq); c->lpart = (double *)(b + pl.off_lpart);
    c->special = (uint32_t *)(b + pl.off_special);
    c->cnt = (Counters *)(b + pl.off_cnt);
    c->nrs.work = (unsigned long long *)(b + pl.off_nrs);
    c->nrs.hist = (unsigned int *)(b + pl.off_nrs + 16 * (size_t)NR_BLOCKS);
    c->nrs.resid = (unsigned int *)(b + pl.off_nrs + 16 * (size_t)NR_BLOCKS + 4 * (size_t)NR_BLOCKS * NR_HIST);
    c->mlp_body = (float *)(b + pl.off_mlpb);
    c->warm = nullptr;
    c->cb.pairF = (double *)(b + pl.off_pairF); c->cb.pairTi = (double *)(b + pl.off_pairTi);
    c->cb.pairTj = (double *)(b + pl.off_pairTj); c->cb.wallF = (double *)(b + pl.off_wallF);
    c->cb.wallT = (double *)(b + pl.off_wallT); c->cb.xiP = (double *)(b + pl.off_xiP);
    c->cb.xiW = (double *)(b + pl.off_xiW);
    c->cb.pairOn = (uint8_t *)(b + pl.off_pairOn);
    c->cb.pairXm = (double *)(b + pl.off_pairXm);
    c->cb.pairOk = (uint8_t *)(b + pl.off_pairOk);
    c->cb.pairGuess = (double *)(b + pl.off_pairGuess);
    c->aux = nullptr;
    c->ev_main = c->ev_flags = c->ev_links = c->ev_bulk = nullptr;
    c->timing = false;
    c->timing_every = 1;
    c->bulk_blocks = 0;
    c->ev_used = 0;
    c->timed_launches = 0;
    c->timed_ms = 0;
    c->steps = 0;

    Params &p = c->p;
    memset(&p, 0, sizeof p);
    p.nx = cfg->nx; p.ny = cfg->ny; p.nz = cfg->nz;
    p.periodic = cfg->periodic;
    p.N = pl.N;
    p.Ns = pl.Ns;
    p.np = n_p;
    p.bc = cfg->bc;
    p.n_sub = cfg->n_sub;
    p.storage = cfg->storage;
    p.rho0 = cfg->rho0;
    p.tau = cfg->tau;
    p.rho0f = (float)cfg->rho0;
    p.omega = (float)(1.0 / cfg->tau);
    p.fcoef = (float)(1.0 - 0.5 / cfg->tau);
    for (int a = 0; a < 3; ++a) { p.gfd[a] = cfg->g_fluid[a]; p.gp[a] = cfg->g_particle[a]; }
    p.scale = 1.f; p.inv_scale = 1.f;
    if (cfg->storage == 1) {
        p.scale = cfg->fp16_scale != 0.f ? cfg->fp16_scale : 1024.f;
        p.inv_scale = 1.f / p.scale;
    }
    p.contact = pl.contact ? 1 : 0;
    p.link_c0 = cfg->link_c0;
    p.c_rs = cfg->contact_rs; p.c_kn = cfg->contact_kn; p.c_en = cfg->contact_en; p.c_mu = cfg->contact_mu;
    p.link_cap = pl.link_cap;
    p.special_cap = pl.special_cap;
    p.region_blocks = pl.region_blocks;
    for (int a = 0; a < 3; ++a) min_image_thresholds(a == 0 ? p.nx : a == 1 ? p.ny : p.nz, p.mi_up[a], p.mi_dn[a]);

    auto bail = [&](lbm_status st) {
        if (c->ev_main) (void)hipEventDestroy(c->ev_main);
        if (c->ev_flags) (void)hipEventDestroy(c->ev_flags);
        if (c->ev_links) (void)hipEventDestroy(c->ev_links);
        if (c->ev_bulk) (void)hipEventDestroy(c->ev_bulk);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        delete c;
        return st;
    };
#define HIPCHK_C(expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return bail(fail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    if (n_p > 0) {
        HIPCHK_C(hipMemcpyAsync(c->P, hp.data(), sizeof(DevParticle) * n_p, hipMemcpyHostToDevice, c->stream));
        HIPCHK_C(hipMemcpyAsync((void *)c->rm.part, pl.part.data(), 4 * pl.part.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK_C(hipMemcpyAsync((void *)c->rm.first, pl.first.data(), 4 * pl.first.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK_C(hipMemcpyAsync((void *)c->rm.dims, pl.dims.data(), 4 * pl.dims.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK_C(hipMemcpyAsync(c->part_first_blk, pl.part_first_blk.data(), 4 * n_p, hipMemcpyHostToDevice, c->stream));
    }
    std::vector<int> zeros(n_p + 1, 0);
    HIPCHK_C(hipMemcpyAsync(c->l_off, zeros.data(), 4 * (n_p + 1), hipMemcpyHostToDevice, c->stream));
    Counters zc{};
    HIPCHK_C(hipMemcpyAsync(c->cnt, &zc, sizeof zc, hipMemcpyHostToDevice, c->stream));
    launch_fill_i32((int32_t *)c->nrs.work, (16 + 4 * (long long)NR_HIST + 4) * NR_BLOCKS / 4, 0, c->stream);
    std::vector<float> mb = mlp_body_blocks(hp);
    if (n_p > 0)
        HIPCHK_C(hipMemcpyAsync(c->mlp_body, mb.data(), 4 * mb.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK_C(hipStreamSynchronize(c->stream));  // host buffers above are released on return
    if (pl.contact) launch_fill_u8(c->cb.pairOk, (long long)n_p * n_p, 0, c->stream);  // no solve yet
    if (pl.contact) {  // tangential springs start relaxed
        std::vector<double> z((size_t)n_p * n_p * 3, 0.0);
        HIPCHK_C(hipMemcpyAsync(c->cb.xiP, z.data(), 24 * (size_t)n_p * n_p, hipMemcpyHostToDevice, c->stream));
        HIPCHK_C(hipMemcpyAsync(c->cb.xiW, z.data(), 24 * (size_t)n_p * 6, hipMemcpyHostToDevice, c->stream));
        HIPCHK_C(hipStreamSynchronize(c->stream));
    }
    HIPCHK_C(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIPCHK_C(hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming));
    // recorded with kernel dispatches (hipExtLaunchKernel): default flags
    HIPCHK_C(hipEventCreate(&c->ev_flags));
    HIPCHK_C(hipEventCreate(&c->ev_bulk));
    HIPCHK_C(hipEventCreateWithFlags(&c->ev_links, hipEventDisableTiming));
    for (int k = 0; k < 3; ++k) launch_fill_i32(c->own[k], pl.N, FLUID, c->stream);

    // counter-force: the fluid carries minus the net weight of free bodies
    if (cfg->counter_force && n_p > 0) {
        // needs the fluid volume, i.e. the flags: flag first, then read back
        reflag(c);
        long long n_solid, n_ref, n_spec;
        if (lbm_status st0 = body_counts(c, n_solid, n_ref, n_spec)) return bail(st0);
        const double nf = (double)(pl.N - n_solid);
        double W[3] = {0, 0, 0};
        for (int q = 0; q < n_p; ++q)
            if (hp[q].mode == LBM_MODE_FREE)
                for (int a = 0; a < 3; ++a) W[a] += (hp[q].m - cfg->rho0 * hp[q].V) * cfg->g_particle[a];
        for (int a = 0; a < 3; ++a) p.gfd[a] = cfg->g_fluid[a] - W[a] / (cfg->rho0 * nf);
    } else {
        reflag(c);
    }
    p.gx = (float)p.gfd[0]; p.gy = (float)p.gfd[1]; p.gz = (float)p.gfd[2];
    c->pending_refill = false;
    StepArgs a = base_args(c);
    a.phase = PHASE_INIT_STATE;
    launch_phase(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bail(fail(LBM_E_HIP, "kernel launch: %s", hipGetErrorString(e)));
    lbm_status st = check_device(c);
    if (st) return bail(st);
    st = estimate_lists(c);
    if (st) return bail(st);
#undef HIPCHK_C
    *out = c;
    return LBM_OK;
}

lbm_status metaball_flag(lbm_ctx *c, int64_t *n_solid, int64_t *n_links) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    if (c->pending_refill) do_refill(c);
    reflag(c);
    if (n_solid || n_links) {
        lbm_status s = check_device(c);
        if (s) return s;
        Counters h;
        HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
        long long ns, nr, nsp;
        if ((s = body_counts(c, ns, nr, nsp))) return s;
        if (n_solid) *n_solid = ns;
        if (n_links) *n_links = h.n_links;
        if ((s = estimate_lists(c))) return s;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

lbm_status refill(lbm_ctx *c, int64_t *n_refilled) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    if (!c->pending_refill) {
        if (n_refilled) *n_refilled = 0;
        return LBM_OK;
    }
    do_refill(c);
    if (n_refilled) {
        lbm_status s = check_device(c);
        if (s) return s;
        long long ns, nr, nsp;
        if ((s = body_counts(c, ns, nr, nsp))) return s;
        *n_refilled = nr;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int32_t n_steps, int32_t mode) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    if (n_steps < 0) return fail(LBM_E_INVALID, "n_steps must be >= 0");
    if (mode != LBM_STEP_COUPLED && mode != LBM_STEP_FLUID_ONLY) return fail(LBM_E_INVALID, "unknown step mode");
    if (c->pending_refill) do_refill(c);
    const bool move = mode == LBM_STEP_COUPLED;
    // Per step: the stream-collide of plain nodes runs on the caller's stream
    // while the second stream does bounce-back + momentum exchange, the
    // rigid-body update, flagging, classification with the boundary/uncovered
    // node update, and the link build.  The boundary pass writes other nodes of
    // the destination buffer than the stream-collide, so the two overlap; the
    // next step's stream-collide (which pulls from those nodes) waits for it,
    // and the next step's second-stream work starts after this step's
    // stream-collide (it overwrites the buffer that one reads).
    // the second stream's first step follows everything earlier on the caller's
    // stream; later steps follow the previous stream-collide (the event rides
    // on its dispatch)
    if (n_steps > 0) HIPCHK(hipEventRecord(c->ev_main, c->stream));
    hipEvent_t after = c->ev_main;
    for (int s = 0; s < n_steps; ++s) {
        StepArgs a = base_args(c);
        a.move = move;
        if (!move) a.own_new = a.own_old;  // geometry fixed
        HIPCHK(hipStreamWaitEvent(c->aux, after, 0));
        StepArgs b = a;
        b.stream = c->aux;
        b.phase = PHASE_LINKS;
        launch_phase(b);
        b.phase = PHASE_FLAGS;  // with the boundary/uncovered update
        b.do_special = 1;
        b.ev_stop = c->ev_flags;
        // flags of step n-1 are dead: cleared by the classification on its
        // balls, which cover them, for the next flagging
        b.own_dead = move ? c->own[c->id] : nullptr;
        launch_phase(b);
        b.ev_stop = nullptr;
        b.own_dead = nullptr;
        if (move) {
            b.phase = PHASE_LINKBUILD;
            launch_phase(b);
        }
        const bool t = c->timing && c->steps % c->timing_every == 0 && c->ev_used + 2 <= c->ev.size();
        a.phase = PHASE_BULK;
        a.ev_start = t ? c->ev[c->ev_used] : nullptr;
        a.ev_stop = t ? c->ev[c->ev_used + 1] : c->ev_bulk;
        after = a.ev_stop;
        launch_phase(a);
        if (t) c->ev_used += 2;
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_flags, 0));
        if (move) {
            const int old = c->ic;
            c->ic = c->in; c->in = c->id; c->id = old;
        }
        c->is = 1 - c->is;
        std::swap(c->A, c->B);
        c->steps++;
    }
    if (n_steps > 0) {  // everything on the second stream is done when the caller's stream is
        HIPCHK(hipEventRecord(c->ev_links, c->aux));
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_links, 0));
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx *c) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    return check_device(c);
}

lbm_status particle_forces(lbm_ctx *c, double *F, double *T) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    lbm_status s = check_device(c);
    if (s) return s;
    std::vector<DevParticle> hp(c->p.np);
    if (c->p.np) HIPCHK(hipMemcpy(hp.data(), c->P, sizeof(DevParticle) * c->p.np, hipMemcpyDeviceToHost));
    for (int p = 0; p < c->p.np; ++p)
        for (int a = 0; a < 3; ++a) {
            if (F) F[3 * p + a] = hp[p].F[a];
            if (T) T[3 * p + a] = hp[p].T[a];
        }
    return LBM_OK;
}

static lbm_status read_state(lbm_ctx *c, double *host) {
    lbm_status s = check_device(c);
    if (s) return s;
    const long long N = c->pl.N, Ns = c->pl.Ns;
    const size_t sb = c->pl.storage_bytes;
    std::vector<char> raw((size_t)Q * Ns * sb);
    HIPCHK(hipMemcpy(raw.data(), c->A, raw.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < Q; ++i)
        for (long long n = 0; n < N; ++n) {
            const size_t k = (size_t)pidx(n, i);  // device layout (pidx)
            double d;
            if (sb == 4) {
                d = ((const float *)raw.data())[k];
            } else if (c->p.storage == 1) {
                d = (double)(float)((const _Float16 *)raw.data())[k] * (double)c->p.inv_scale;
            } else {
                const uint32_t u = (uint32_t)((const uint16_t *)raw.data())[k] << 16;
                float f;
                memcpy(&f, &u, 4);
                d = f;
            }
            host[(size_t)i * N + n] = d + WD[i] * c->p.rho0;
        }
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx *c, double *f) {
    if (!c || !f) return fail(LBM_E_INVALID, "NULL argument");
    return read_state(c, f);
}

lbm_status lbm_set_populations(lbm_ctx *c, const double *f, int32_t post_collision) {
    if (!c || !f) return fail(LBM_E_INVALID, "NULL argument");
    lbm_status s = check_device(c);
    if (s) return s;
    const long long N = c->pl.N, Ns = c->pl.Ns;
    for (long long k = 0; k < (long long)Q * N; ++k)
        if (!std::isfinite(f[k])) return fail(LBM_E_INVALID, "non-finite population at %lld", k);
    std::vector<char> raw((size_t)Q * Ns * c->pl.storage_bytes, 0);
    for (int i = 0; i < Q; ++i)
        for (long long n = 0; n < N; ++n) {
            const size_t k = (size_t)pidx(n, i);  // device layout (pidx)
            const double d = f[(size_t)i * N + n] - WD[i] * c->p.rho0;
            if (c->pl.storage_bytes == 4) {
                ((float *)raw.data())[k] = (float)d;
            } else if (c->p.storage == 1) {
                ((_Float16 *)raw.data())[k] = (_Float16)(float)(d * c->p.scale);
            } else {
                const float x = (float)d;
                uint32_t u;
                memcpy(&u, &x, 4);
                u += 0x7fffu + ((u >> 16) & 1u);
                ((uint16_t *)raw.data())[k] = (uint16_t)(u >> 16);
            }
        }
    HIPCHK(hipMemcpy(c->A, raw.data(), raw.size(), hipMemcpyHostToDevice));
    if (!post_collision) {
        StepArgs a = base_args(c);
        a.phase = PHASE_COLLIDE_STORED;
        launch_phase(a);
    }
    c->pending_refill = false;
    return check_device(c);
}

lbm_status lbm_get_macros(lbm_ctx *c, double *rho, double *u) {
    if (!c || !rho || !u) return fail(LBM_E_INVALID, "NULL argument");
    const long long N = c->pl.N;
    std::vector<double> f((size_t)Q * N);
    lbm_status s = read_state(c, f.data());
    if (s) return s;
    for (long long n = 0; n < N; ++n) {
        double r = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q; ++i) {
            const double v = f[(size_t)i * N + n];
            r += v;
            j[0] += EX[i] * v; j[1] += EY[i] * v; j[2] += EZ[i] * v;
        }
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[3 * n + a] = j[a] / r - 0.5 * c->p.gfd[a];
    }
    return LBM_OK;
}

lbm_status lbm_get_flags(lbm_ctx *c, int32_t *owner) {
    if (!c || !owner) return fail(LBM_E_INVALID, "NULL argument");
    lbm_status s = check_device(c);
    if (s) return s;
    HIPCHK(hipMemcpy(owner, c->own[c->ic], 4 * c->pl.N, hipMemcpyDeviceToHost));
    for (long long n = 0; n < c->pl.N; ++n)
        if (owner[n] == FLUID) owner[n] = -1;
    return LBM_OK;
}

lbm_status lbm_get_links(lbm_ctx *c, int64_t *n_links, uint32_t *node, int32_t *dir, int32_t *owner, double *q) {
    if (!c || !n_links) return fail(LBM_E_INVALID, "NULL argument");
    lbm_status s = check_device(c);
    if (s) return s;
    Counters h;
    HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
    *n_links = h.n_links;
    if (!node && !dir && !owner && !q) return LBM_OK;
    const int nl = h.n_links;
    std::vector<uint32_t> nd(nl), d(nl);
    std::vector<double> qq(nl);
    if (nl) {
        HIPCHK(hipMemcpy(nd.data(), c->l_node, 4 * (size_t)nl, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(d.data(), c->l_do, 4 * (size_t)nl, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(qq.data(), c->l_q, 8 * (size_t)nl, hipMemcpyDeviceToHost));
    }
    for (int l = 0; l < nl; ++l) {
        if (node) node[l] = nd[l];
        if (dir) dir[l] = (int32_t)(d[l] & 31u);
        if (owner) owner[l] = (int32_t)(d[l] >> 8);
        if (q) q[l] = qq[l];
    }
    return LBM_OK;
}

lbm_status lbm_get_particles(lbm_ctx *c, lbm_particle_state *out) {
    if (!c || (!out && c->p.np)) return fail(LBM_E_INVALID, "NULL argument");
    lbm_status s = check_device(c);
    if (s) return s;
    std::vector<DevParticle> hp(c->p.np);
    if (c->p.np) HIPCHK(hipMemcpy(hp.data(), c->P, sizeof(DevParticle) * c->p.np, hipMemcpyDeviceToHost));
    for (int p = 0; p < c->p.np; ++p) {
        lbm_particle_state &o = out[p];
        const DevParticle &d = hp[p];
        memcpy(o.x, d.X, sizeof o.x); memcpy(o.quat, d.q, sizeof o.quat);
        memcpy(o.v, d.v, sizeof o.v); memcpy(o.omega, d.w, sizeof o.omega);
        memcpy(o.F, d.F, sizeof o.F); memcpy(o.T, d.T, sizeof o.T);
        o.mass = d.m; o.volume = d.V;
        memcpy(o.inertia, d.I, sizeof o.inertia);
    }
    return LBM_OK;
}

lbm_status lbm_set_particles(lbm_ctx *c, const lbm_particle_state *in) {
    if (!c || (!in && c->p.np)) return fail(LBM_E_INVALID, "NULL argument");
    lbm_status s = check_device(c);
    if (s) return s;
    std::vector<DevParticle> hp(c->p.np);
    if (c->p.np) HIPCHK(hipMemcpy(hp.data(), c->P, sizeof(DevParticle) * c->p.np, hipMemcpyDeviceToHost));
    const int L[3] = {c->p.nx, c->p.ny, c->p.nz};
    for (int p = 0; p < c->p.np; ++p) {
        const lbm_particle_state &o = in[p];
        if (!finite_all(o.x, 3) || !finite_all(o.quat, 4) || !finite_all(o.v, 3) || !finite_all(o.omega, 3))
            return fail(LBM_E_INVALID, "particle %d: non-finite state", p);
        DevParticle &d = hp[p];
        const double qn = std::sqrt(o.quat[0] * o.quat[0] + o.quat[1] * o.quat[1] + o.quat[2] * o.quat[2] + o.quat[3] * o.quat[3]);
        if (!(qn > 0)) return fail(LBM_E_INVALID, "particle %d: zero quaternion", p);
        for (int a = 0; a < 3; ++a) {
            d.X[a] = o.x[a]; d.v[a] = o.v[a]; d.w[a] = o.omega[a];
            if (!((c->p.periodic >> a) & 1u) && (d.X[a] - d.rb < 0.0 || d.X[a] + d.rb > L[a] - 1.0))
                return fail(LBM_E_INVALID, "particle %d: bounding sphere crosses a wall on axis %d", p, a);
        }
        for (int a = 0; a < 4; ++a) d.q[a] = o.quat[a] / qn;
    }
    if (c->p.np) HIPCHK(hipMemcpy(c->P, hp.data(), sizeof(DevParticle) * c->p.np, hipMemcpyHostToDevice));
    launch_refresh_pose(c->p, c->P, 0, c->stream);
    return check_device(c);
}

lbm_status lbm_get_gfluid(lbm_ctx *c, double *g3) {
    if (!c || !g3) return fail(LBM_E_INVALID, "NULL argument");
    for (int a = 0; a < 3; ++a) g3[a] = c->p.gfd[a];
    return LBM_OK;
}

lbm_status lbm_timing_enable(lbm_ctx *c, int32_t on) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    if (on && c->ev.empty()) {
        c->ev.resize(2 * 4096);
        for (auto &e : c->ev) HIPCHK(hipEventCreate(&e));
    }
    c->timing = on > 0;
    c->timing_every = on > 1 ? on : 1;
    return LBM_OK;
}

lbm_status lbm_timing_read(lbm_ctx *c, double *ms, int64_t *launches, int64_t *nodes_per_launch) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    HIPCHK(hipStreamSynchronize(c->stream));
    double tot = 0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]));
        tot += t;
    }
    if (ms) *ms = tot;
    if (launches) *launches = (int64_t)(c->ev_used / 2);
    if (nodes_per_launch) {
        // nodes the stream-collide kernel updated in the last step: all but
        // solid nodes and the boundary/uncovered nodes handled separately
        long long ns, nr, nsp;
        if (lbm_status s = body_counts(c, ns, nr, nsp)) return s;
        *nodes_per_launch = c->pl.N - ns - nsp;
    }
    c->ev_used = 0;
    return LBM_OK;
}

lbm_status lbm_nr_stats(lbm_ctx *c, int64_t *links, int64_t *iterations) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    lbm_status s = check_device(c);
    if (s) return s;
    std::vector<unsigned long long> w(2 * (size_t)NR_BLOCKS);
    HIPCHK(hipMemcpy(w.data(), c->nrs.work, 16 * (size_t)NR_BLOCKS, hipMemcpyDeviceToHost));
    unsigned long long it = 0, nl = 0;
    for (int b = 0; b < NR_BLOCKS; ++b) { it += w[2 * b]; nl += w[2 * b + 1]; }
    if (links) *links = (int64_t)nl;
    if (iterations) *iterations = (int64_t)it;
    launch_fill_i32((int32_t *)c->nrs.work, 4 * (long long)NR_BLOCKS, 0, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_nr_histogram(lbm_ctx *c, int64_t *hist, double *resid_max) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    lbm_status s = check_device(c);
    if (s) return s;
    std::vector<unsigned int> h((size_t)NR_BLOCKS * NR_HIST), r(NR_BLOCKS);
    HIPCHK(hipMemcpy(h.data(), c->nrs.hist, 4 * h.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(r.data(), c->nrs.resid, 4 * r.size(), hipMemcpyDeviceToHost));
    unsigned int rb = 0;
    for (int b = 0; b < NR_BLOCKS; ++b) rb = std::max(rb, r[b]);
    if (hist)
        for (int k = 0; k < NR_HIST; ++k) {
            long long t = 0;
            for (int b = 0; b < NR_BLOCKS; ++b) t += h[(size_t)b * NR_HIST + k];
            hist[k] = t;
        }
    if (resid_max) {
        float f;
        std::memcpy(&f, &rb, 4);
        *resid_max = f;
    }
    launch_fill_i32((int32_t *)c->nrs.hist, (long long)NR_BLOCKS * NR_HIST + NR_BLOCKS, 0, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_set_warmstart(lbm_ctx *c, const void *dev_weights) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    if (dev_weights && ((uintptr_t)dev_weights & 255)) return fail(LBM_E_INVALID, "weights must be 256-byte aligned");
    c->warm = dev_weights ? mlp_blob(const_cast<void *>(dev_weights)).w16 : nullptr;
    return LBM_OK;
}

size_t mlp_weights_bytes(void) { return mlp_blob_bytes(); }
int32_t mlp_param_count(void) { return MLP_P; }

lbm_status mlp_init(void *dev_weights, const float *params, void *hip_stream) {
    if (!dev_weights || !params) return fail(LBM_E_INVALID, "NULL argument");
    if ((uintptr_t)dev_weights & 255) return fail(LBM_E_INVALID, "weights must be 256-byte aligned");
    for (int i = 0; i < MLP_P; ++i)
        if (!std::isfinite(params[i])) return fail(LBM_E_INVALID, "parameter %d is not finite", i);
    hipStream_t st = (hipStream_t)hip_stream;
    const MlpBlob b = mlp_blob(dev_weights);
    HIPCHK(hipMemcpyAsync(b.theta, params, 4 * (size_t)MLP_P, hipMemcpyHostToDevice, st));
    launch_mlp_init(b, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return LBM_OK;
}

lbm_status mlp_get_params(const void *dev_weights, float *params, void *hip_stream) {
    if (!dev_weights || !params) return fail(LBM_E_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)hip_stream;
    const MlpBlob b = mlp_blob(const_cast<void *>(dev_weights));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(params, b.theta, 4 * (size_t)MLP_P, hipMemcpyDeviceToHost));
    return LBM_OK;
}

lbm_status mlp_collect(lbm_ctx *c, int64_t n_max, void *dev_feat, void *dev_target, int64_t *n_out) {
    if (!c || !dev_feat || !dev_target || !n_out) return fail(LBM_E_INVALID, "NULL argument");
    if (n_max < 0) return fail(LBM_E_INVALID, "n_max < 0");
    lbm_status s = check_device(c);
    if (s) return s;
    Counters h;
    HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
    const int n = (int)std::min<int64_t>(n_max, std::min(h.n_links, c->p.link_cap));
    launch_mlp_collect(c->p, c->P, c->mlp_body, c->l_node, c->l_do, c->l_q, n, (_Float16 *)dev_feat,
                       (float *)dev_target, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    *n_out = n;
    return LBM_OK;
}

lbm_status mlp_forward(void *dev_weights, const void *dev_feat, int64_t n, int32_t precision, float *dev_out,
                       void *hip_stream) {
    if (!dev_weights || !dev_feat || !dev_out) return fail(LBM_E_INVALID, "NULL argument");
    if (n < 0 || precision < 0 || precision > 2) return fail(LBM_E_INVALID, "bad n or precision");
    hipStream_t st = (hipStream_t)hip_stream;
    const MlpBlob b = mlp_blob(dev_weights);
    const size_t xb = precision == 1 ? 4 : 2;
    for (int64_t a = 0; a < n; a += MLP_MAX_BATCH) {
        const int m = (int)std::min<int64_t>(MLP_MAX_BATCH, n - a);
        launch_mlp_forward(b, (const char *)dev_feat + (size_t)a * MLP_IN * xb, m, precision, st);
        HIPCHK(hipMemcpyAsync(dev_out + (size_t)a * MLP_OUT, b.out, 4 * (size_t)m * MLP_OUT, hipMemcpyDeviceToDevice,
                              st));
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

lbm_status mlp_grad(void *dev_weights, const void *dev_feat, const void *dev_target, int64_t n, int32_t precision,
                    float *grad, double *loss, void *hip_stream) {
    if (!dev_weights || !dev_feat || !dev_target) return fail(LBM_E_INVALID, "NULL argument");
    if (n < 1 || n > MLP_MAX_BATCH) return fail(LBM_E_INVALID, "n must be 1..%d", MLP_MAX_BATCH);
    if (precision != 0 && precision != 1) return fail(LBM_E_INVALID, "precision must be 0 or 1");
    hipStream_t st = (hipStream_t)hip_stream;
    const MlpBlob b = mlp_blob(dev_weights);
    launch_mlp_loss_grad(b, dev_feat, (const float *)dev_target, (int)n, precision, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    if (grad) HIPCHK(hipMemcpy(grad, b.g, 4 * (size_t)MLP_P, hipMemcpyDeviceToHost));
    if (loss) {
        float l;
        HIPCHK(hipMemcpy(&l, b.loss, 4, hipMemcpyDeviceToHost));
        *loss = l;
    }
    return LBM_OK;
}

lbm_status mlp_train(void *dev_feat, void *dev_target, int64_t n, const char *hparams_json, void *dev_weights,
                     void *hip_stream) {
    if (!dev_weights || !dev_feat || !dev_target) return fail(LBM_E_INVALID, "NULL argument");
    if (n < 1) return fail(LBM_E_INVALID, "n must be >= 1");
    const std::string txt = hparams_json ? hparams_json : "";
    double lr = 1e-3, epochs = 1, batch = 256, b1 = 0.9, b2 = 0.999, eps = 1e-8, prec = 0;
    json_num(txt, "lr", lr);
    json_num(txt, "epochs", epochs);
    json_num(txt, "batch", batch);
    json_num(txt, "beta1", b1);
    json_num(txt, "beta2", b2);
    json_num(txt, "eps", eps);
    json_num(txt, "precision", prec);
    const int bs = (int)batch, ne = (int)epochs, pr = (int)prec;
    if (bs < 1 || bs > MLP_MAX_BATCH || ne < 0 || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) ||
        !(eps > 0) || (pr != 0 && pr != 1))
        return fail(LBM_E_INVALID, "bad hyper-parameters (batch 1..%d, epochs >= 0, lr > 0, 0 <= beta < 1, "
                                   "eps > 0, precision 0 or 1)", MLP_MAX_BATCH);
    hipStream_t st = (hipStream_t)hip_stream;
    const MlpBlob b = mlp_blob(dev_weights);
    long long t = 0;
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(&t, b.t, 8, hipMemcpyDeviceToHost));
    const size_t xb = pr == 1 ? 4 : 2;
    for (int e = 0; e < ne; ++e)
        for (int64_t a = 0; a < n; a += bs) {
            const int m = (int)std::min<int64_t>(bs, n - a);
            launch_mlp_loss_grad(b, (const char *)dev_feat + (size_t)a * MLP_IN * xb,
                                 (const float *)dev_target + (size_t)a * MLP_OUT, m, pr, st);
            ++t;
            const double bc1 = 1.0 - std::pow(b1, (double)t), bc2 = 1.0 - std::pow(b2, (double)t);
            launch_mlp_adam(b, (float)lr, (float)b1, (float)b2, (float)eps, (float)bc1, (float)bc2, st);
        }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(b.t, &t, 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return LBM_OK;
}

lbm_status lbm_contact_nr_stats(lbm_ctx *c, int64_t *solves, int64_t *iterations) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    lbm_status s = check_device(c);
    if (s) return s;
    Counters h;
    HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
    if (solves) *solves = (int64_t)h.n_contact_nr;
    if (iterations) *iterations = (int64_t)h.n_contact_it;
    const unsigned long long z[2] = {0ull, 0ull};
    HIPCHK(hipMemcpy((char *)c->cnt + offsetof(Counters, n_contact_nr), z, sizeof z, hipMemcpyHostToDevice));
    return LBM_OK;
}

lbm_status mlp_collect_contact(lbm_ctx *c, int64_t n_max, void *dev_feat, void *dev_target, int64_t *n_out) {
    if (!c || !dev_feat || !dev_target || !n_out) return fail(LBM_E_INVALID, "NULL argument");
    if (n_max < 0) return fail(LBM_E_INVALID, "n_max < 0");
    lbm_status s = check_device(c);
    if (s) return s;
    *n_out = 0;
    if (!c->pl.contact || n_max == 0) return LBM_OK;
    launch_mlp_collect_contact(c->p, c->P, c->mlp_body, c->cb, (int)std::min<int64_t>(n_max, 0x7fffffff),
                               (_Float16 *)dev_feat, (float *)dev_target, c->cnt, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    Counters h;
    HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
    *n_out = h.n_collect;
    return LBM_OK;
}

lbm_status lbm_contact_stats(lbm_ctx *c, int64_t *contacts, int64_t *failures) {
    if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
    lbm_status s = check_device(c);
    if (s) return s;
    Counters h;
    HIPCHK(hipMemcpy(&h, c->cnt, sizeof h, hipMemcpyDeviceToHost));
    if (contacts) *contacts = (int64_t)h.n_contacts;
    if (failures) *failures = (int64_t)h.n_contact_fail;
    return LBM_OK;
}

// ---------------------------------------------------------------- checkpoint
// File: a header (magic, version, the configuration, the particle count, the
// arena plan's offsets, the host-side step state and the kernel constants),
// then the arena's bytes [0, plan total) verbatim: populations in their
// storage type in both buffers, the three flag buffers, skip masks, particle
// records (FP64 state, control points, region history), cut links with q,
// contact springs, counters.  The arena holds no pointers, so a checkpoint
// loads into any arena of a context set up with the same configuration.
namespace {
constexpr char CKPT_MAGIC[8] = {'M', 'I', 'D', 'E', 'L', 'B', 'M', 0};
constexpr uint32_t CKPT_VERSION = 1;
struct CkptHeader {
    char magic[8];
    uint32_t version, n_sig;
    lbm_config cfg;
    int32_t n_p, ic, in, id, is, a_first, pending_refill, pad;
    int64_t steps;
    Params p;
};
std::vector<uint64_t> plan_signature(const Plan &pl) {
    std::vector<uint64_t> v = {(uint64_t)pl.N, (uint64_t)pl.Ns, (uint64_t)pl.np, (uint64_t)pl.storage_bytes,
                               (uint64_t)pl.region_blocks, (uint64_t)pl.link_cap, (uint64_t)pl.special_cap,
                               pl.off_A, pl.off_B, pl.off_own[0], pl.off_own[1], pl.off_own[2], pl.off_skip[0],
                               pl.off_skip[1], pl.off_P, pl.off_part, pl.off_first, pl.off_dims, pl.off_pfb,
                               pl.off_bcnt, pl.off_blinks, pl.off_loff, pl.off_lnode, pl.off_ldo, pl.off_lq,
                               pl.off_lpart, pl.off_special, pl.off_cnt, pl.off_lmask, pl.off_nrs, pl.off_mlpb,
                               pl.off_pairF, pl.off_pairTi, pl.off_pairTj, pl.off_wallF, pl.off_wallT, pl.off_xiP,
                               pl.off_xiW, pl.off_pairOn, pl.off_pairXm, pl.off_pairOk, pl.off_pairGuess, pl.total};
    return v;
}
constexpr size_t CKPT_CHUNK = size_t(64) << 20;
}  // namespace

lbm_status lbm_save(lbm_ctx *c, const char *path) {
    if (!c || !path) return fail(LBM_E_INVALID, "NULL argument");
    if (c->pending_refill) do_refill(c);
    lbm_status s = check_device(c);
    if (s) return s;
    CkptHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, CKPT_MAGIC, 8);
    h.version = CKPT_VERSION;
    const std::vector<uint64_t> sig = plan_signature(c->pl);
    h.n_sig = (uint32_t)sig.size();
    h.cfg = c->cfg;
    h.n_p = c->p.np;
    h.ic = c->ic; h.in = c->in; h.id = c->id; h.is = c->is;
    h.a_first = c->A == (void *)(c->arena + c->pl.off_A);
    h.pending_refill = 0;
    h.steps = c->steps;
    h.p = c->p;
    FILE *f = fopen(path, "wb");
    if (!f) return fail(LBM_E_INVALID, "cannot open %s for writing", path);
    bool ok = fwrite(&h, sizeof h, 1, f) == 1 && fwrite(sig.data(), 8, sig.size(), f) == sig.size();
    std::vector<char> buf(std::min(CKPT_CHUNK, c->pl.total));
    for (size_t o = 0; ok && o < c->pl.total; o += buf.size()) {
        const size_t n = std::min(buf.size(), c->pl.total - o);
        if (hipMemcpy(buf.data(), c->arena + o, n, hipMemcpyDeviceToHost) != hipSuccess) {
            fclose(f);
            return fail(LBM_E_HIP, "reading the arena for %s failed", path);
        }
        ok = fwrite(buf.data(), 1, n, f) == n;
    }
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(LBM_E_INVALID, "writing %s failed", path);
    return LBM_OK;
}

lbm_status lbm_load(lbm_ctx *c, const char *path) {
    if (!c || !path) return fail(LBM_E_INVALID, "NULL argument");
    lbm_status s = check_device(c);
    if (s) return s;
    FILE *f = fopen(path, "rb");
    if (!f) return fail(LBM_E_INVALID, "cannot open %s", path);
    CkptHeader h;
    if (fread(&h, sizeof h, 1, f) != 1 || memcmp(h.magic, CKPT_MAGIC, 8) != 0) {
        fclose(f);
        return fail(LBM_E_INVALID, "%s is not a checkpoint of this library", path);
    }
    if (h.version != CKPT_VERSION) {
        fclose(f);
        return fail(LBM_E_INVALID, "%s: checkpoint version %u, expected %u", path, h.version, CKPT_VERSION);
    }
    const std::vector<uint64_t> sig = plan_signature(c->pl);
    std::vector<uint64_t> fsig(h.n_sig);
    if (h.n_sig != sig.size() || fread(fsig.data(), 8, fsig.size(), f) != fsig.size() || fsig != sig ||
        memcmp(&h.cfg, &c->cfg, sizeof h.cfg) != 0 || h.n_p != c->p.np) {
        fclose(f);
        return fail(LBM_E_STATE, "%s was written by a context of another configuration", path);
    }
    std::vector<char> buf(std::min(CKPT_CHUNK, c->pl.total));
    for (size_t o = 0; o < c->pl.total; o += buf.size()) {
        const size_t n = std::min(buf.size(), c->pl.total - o);
        if (fread(buf.data(), 1, n, f) != n) {
            fclose(f);
            return fail(LBM_E_INVALID, "%s is truncated (the context's state is now undefined)", path);
        }
        if (hipMemcpy(c->arena + o, buf.data(), n, hipMemcpyHostToDevice) != hipSuccess) {
            fclose(f);
            return fail(LBM_E_HIP, "writing the arena from %s failed", path);
        }
    }
    fclose(f);
    char *b = c->arena;
    c->A = b + (h.a_first ? c->pl.off_A : c->pl.off_B);
    c->B = b + (h.a_first ? c->pl.off_B : c->pl.off_A);
    c->ic = h.ic; c->in = h.in; c->id = h.id; c->is = h.is;
    c->pending_refill = false;
    c->steps = h.steps;
    c->p = h.p;
    c->ev_used = 0;
    return check_device(c);
}

void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->ev) (void)hipEventDestroy(e);
    if (c->ev_main) (void)hipEventDestroy(c->ev_main);
    if (c->ev_flags) (void)hipEventDestroy(c->ev_flags);
    if (c->ev_links) (void)hipEventDestroy(c->ev_links);
    if (c->ev_bulk) (void)hipEventDestroy(c->ev_bulk);
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    delete c;
}


// ------------------------------------------------------------------ ensemble
// A batch of independent systems stepped together: one batched stream-collide
// launch over a table of equal tiles for all systems, one batched launch per
// kind of boundary kernel for all systems around it, and six consecutive
// steps (the period of the buffer rotation: A/B 2, flags 3) captured once
// into a HIP graph and replayed.

}  // extern "C"

namespace {
constexpr int GRAPH_PERIOD = 6;
constexpr int BATCH_AUX = 1;  // stream of the batched boundary kernels
constexpr int TW_CANDIDATES[4] = {6, 5, 4, TW_FLAT};  // wave tiles 64x1, 32x2, 16x4, 64 in lattice order
}  // namespace

struct lbm_batch {
    int n = 0;
    std::vector<lbm_ctx *> cs;
    hipStream_t caller = nullptr, main = nullptr, aux[BATCH_AUX] = {};
    hipEvent_t ev_in = nullptr, ev_main = nullptr, ev_out = nullptr;
    hipEvent_t ev_flags[BATCH_AUX] = {}, ev_links[BATCH_AUX] = {};
    int storage = 0, bw = 8;
    std::vector<int> tw;  // tile width log2 per system
    BulkCase *d_cases = nullptr;  // [n + 1]: the table, plus one slot for tuning runs
    int *d_blk = nullptr;         // [blk_cap]: block -> system
    int *d_blk1 = nullptr;        // [blk1_cap]: tuning runs of one system
    size_t blk_cap = 0, blk1_cap = 0;
    std::vector<BulkCase> h_cases;
    std::vector<int> h_blk;
    int nblocks = 0;
    int phase = 0;  // steps since the tables were written, modulo GRAPH_PERIOD
    // batched boundary kernels: argument blocks of the systems for each step
    // of a period from the tables' start, block -> system maps per kind
    CaseArgs *d_args = nullptr;  // [GRAPH_PERIOD][n]
    int *d_map = nullptr;
    size_t map_cap = 0;
    int map_off[BK_N] = {}, map_n[BK_N] = {};
    std::vector<CaseArgs> h_args;
    std::vector<Params> h_p;  // each system's constants when the tables were written (byte copies)
    bool any_rigid = false, any_warm = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> graph_key;
};

namespace {

long long tile_blocks(const lbm_config &c, int twl, int bw) {
    if (twl == TW_FLAT) return ((long long)c.nx * c.ny * c.nz + 64ll * bw - 1) / (64ll * bw);
    const long long nsx = (c.nx + (1 << twl) - 1) >> twl, th = 64 >> twl;
    const long long nsy = (c.ny + th - 1) / th;
    return (nsx * nsy * c.nz + bw - 1) / bw;
}

BulkCase bulk_case(const lbm_ctx *c, int twl, int bw, int first_block) {
    BulkCase b{};
    const Params &p = c->p;
    b.nx = p.nx; b.ny = p.ny; b.nz = p.nz; b.periodic = p.periodic; b.N = p.N; b.Ns = p.Ns;
    b.rho0f = p.rho0f; b.omega = p.omega; b.fcoef = p.fcoef;
    b.gx = p.gx; b.gy = p.gy; b.gz = p.gz; b.scale = p.scale; b.inv_scale = p.inv_scale;
    b.tw_log2 = twl;
    if (twl != TW_FLAT) {
        b.nsx = (p.nx + (1 << twl) - 1) >> twl;
        b.nsy = (p.ny + (64 >> twl) - 1) / (64 >> twl);
    }
    b.first_block = first_block;
    b.n_blocks = (int)tile_blocks(c->cfg, twl, bw);
    b.A[0] = c->A; b.B[0] = c->B; b.A[1] = c->B; b.B[1] = c->A;
    b.skip[0] = c->skip[c->is]; b.skip[1] = c->skip[1 - c->is];
    b.err = &c->cnt->err;
    return b;
}

// Block ranges of a system in the batched boundary launches (the one-system
// launch sizes; systems without bodies take no blocks but the force
// reduction's, whose block 0 clears the step counters).
void case_blocks(const lbm_ctx *c, int nb[BK_N]) {
    const Params &p = c->p;
    const bool bodies = p.np > 0;
    nb[BK_LINKS] = bodies ? link_grid(p) : 0;
    nb[BK_REDUCE] = std::max(p.np, 1);
    nb[BK_RIGID] = bodies && p.contact ? 1 : 0;
    nb[BK_REGION] = bodies ? p.region_blocks : 0;
    nb[BK_LINKQ] = bodies ? link_q_grid(p) : 0;
}

// Largest block ranges of a system (list grids at full capacity).
long long case_blocks_cap(const Params &p) {
    if (p.np <= 0) return 1;
    Params q = p;
    q.est_links = 0;  // 0: sized for the capacity
    return (long long)link_grid(q) + p.np + 1 + p.region_blocks + link_q_grid(q);
}

// Argument block of system c, k steps after its current state (buffer
// rotation: A/B swap each step, flag buffers old/new/dead cycle, skip masks
// swap), for the batched kernels of a step that moves the bodies.
CaseArgs case_args(const lbm_ctx *c, int k) {
    CaseArgs a{};
    int ic = c->ic, in = c->in, id = c->id, is = c->is;
    for (int s = 0; s < k; ++s) {
        const int old = ic;
        ic = in; in = id; id = old;
        is = 1 - is;
    }
    a.p = c->p;
    a.rm = c->rm;
    a.A = (k & 1) ? c->B : c->A;
    a.B = (k & 1) ? c->A : c->B;
    a.own_old = c->own[ic]; a.own_new = c->own[in]; a.own_dead = c->own[id];
    a.skip_next = c->skip[1 - is];
    a.P = c->P;
    a.part_first_blk = c->part_first_blk;
    a.blk_cnt = c->blk_cnt; a.l_off = c->l_off; a.body_stats = c->body_stats;
    a.lmask = c->lmask; a.l_node = c->l_node; a.l_do = c->l_do; a.special = c->special;
    a.l_q = c->l_q; a.part = c->lpart;
    a.cnt = c->cnt; a.cb = c->cb; a.nrs = c->nrs;
    a.warm = c->warm; a.mlp_body = c->mlp_body;
    a.update = !c->p.contact;
    return a;
}

void drop_graph(lbm_batch *b);

// Writes the launch tables for the systems' current state.  A captured graph
// holds launch sizes and table offsets of the old tables: it is dropped.
lbm_status write_table(lbm_batch *b) {
    drop_graph(b);
    b->h_cases.resize(b->n);
    b->h_blk.clear();
    int first = 0;
    for (int i = 0; i < b->n; ++i) {
        b->h_cases[i] = bulk_case(b->cs[i], b->tw[i], b->bw, first);
        for (int k = 0; k < b->h_cases[i].n_blocks; ++k) b->h_blk.push_back(i);
        first += b->h_cases[i].n_blocks;
    }
    if (b->h_blk.size() > b->blk_cap) return fail(LBM_E_NOMEM, "ensemble block table overflow");
    b->nblocks = first;
    // boundary kernels: block ranges, maps, argument blocks for a period
    std::vector<int> nb((size_t)b->n * BK_N);
    int tot[BK_N] = {};
    b->any_rigid = b->any_warm = false;
    for (int i = 0; i < b->n; ++i) {
        case_blocks(b->cs[i], &nb[(size_t)i * BK_N]);
        for (int k = 0; k < BK_N; ++k) tot[k] += nb[(size_t)i * BK_N + k];
        b->any_rigid = b->any_rigid || nb[(size_t)i * BK_N + BK_RIGID] > 0;
        b->any_warm = b->any_warm || b->cs[i]->warm != nullptr;
    }
    size_t need = 0;
    for (int k = 0; k < BK_N; ++k) {
        b->map_off[k] = (int)need;
        b->map_n[k] = tot[k];
        need += (size_t)tot[k];
    }
    if (need > b->map_cap) return fail(LBM_E_NOMEM, "ensemble boundary block map overflow");
    std::vector<int> map(need);
    int at[BK_N] = {};
    std::vector<CaseArgs> base(b->n);
    for (int i = 0; i < b->n; ++i) {
        for (int k = 0; k < BK_N; ++k) {
            const int m = nb[(size_t)i * BK_N + k];
            base[i].first[k] = at[k];
            base[i].nblk[k] = m;
            for (int j = 0; j < m; ++j) map[(size_t)b->map_off[k] + at[k] + j] = i;
            at[k] += m;
        }
    }
    b->h_args.resize((size_t)GRAPH_PERIOD * b->n);
    b->h_p.resize(b->n);
    for (int i = 0; i < b->n; ++i) {
        std::memcpy(&b->h_p[i], &b->cs[i]->p, sizeof(Params));
        for (int k = 0; k < GRAPH_PERIOD; ++k) {
            CaseArgs a = case_args(b->cs[i], k);
            std::memcpy(a.first, base[i].first, sizeof a.first);
            std::memcpy(a.nblk, base[i].nblk, sizeof a.nblk);
            b->h_args[(size_t)k * b->n + i] = a;
        }
    }
    HIPCHK(hipMemcpyAsync(b->d_cases, b->h_cases.data(), sizeof(BulkCase) * b->n, hipMemcpyHostToDevice, b->main));
    HIPCHK(hipMemcpyAsync(b->d_blk, b->h_blk.data(), 4 * b->h_blk.size(), hipMemcpyHostToDevice, b->main));
    HIPCHK(hipMemcpyAsync(b->d_args, b->h_args.data(), sizeof(CaseArgs) * b->h_args.size(), hipMemcpyHostToDevice,
                          b->main));
    if (need) HIPCHK(hipMemcpyAsync(b->d_map, map.data(), 4 * need, hipMemcpyHostToDevice, b->main));
    HIPCHK(hipStreamSynchronize(b->main));
    b->phase = 0;
    return LBM_OK;
}

bool table_valid(const lbm_batch *b) {
    if ((int)b->h_cases.size() != b->n || b->h_args.size() != (size_t)GRAPH_PERIOD * b->n) return false;
    for (int i = 0; i < b->n; ++i) {
        const BulkCase &h = b->h_cases[i];
        const lbm_ctx *c = b->cs[i];
        const int par = b->phase & 1;
        if (h.A[par] != c->A || h.skip[par] != c->skip[c->is] || h.tw_log2 != b->tw[i]) return false;
        const CaseArgs &a = b->h_args[(size_t)b->phase * b->n + i];
        if (a.A != c->A || a.own_old != c->own[c->ic] || a.own_new != c->own[c->in] || a.warm != c->warm)
            return false;
        if (std::memcmp(&b->h_p[i], &c->p, sizeof(Params)) != 0) return false;
    }
    return true;
}

// (after the stream has run any launch of the graph)
void drop_graph(lbm_batch *b) {
    if (b->exec && b->main) (void)hipStreamSynchronize(b->main);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
}

std::vector<uintptr_t> state_key(const lbm_batch *b) {
    std::vector<uintptr_t> k;
    k.push_back((uintptr_t)b->phase);
    for (auto *c : b->cs) {
        k.push_back((uintptr_t)c->A);
        k.push_back((uintptr_t)c->is);
        k.push_back((uintptr_t)c->ic);
    }
    return k;
}

// One coupled step of every system, enqueued on b->main and b->aux[0]: the
// batched stream-collide on the first stream; on the second, which starts
// after the first stream's previous work, the batched bounce-back and
// momentum exchange, force reduction (and rigid bodies), flags,
// classification with the boundary pass, then the link build.  The next
// step's stream-collide waits for the boundary pass.
lbm_status enqueue_batch_step(lbm_batch *b) {
    hipStream_t ax = b->aux[0];
    HIPCHK(hipEventRecord(b->ev_main, b->main));
    HIPCHK(hipStreamWaitEvent(ax, b->ev_main, 0));
    const CaseArgs *cs = b->d_args + (size_t)b->phase * b->n;
    auto run = [&](BatchOp op, int kind) {
        launch_case_batch(b->storage, op, cs, b->d_map + b->map_off[kind], b->map_n[kind], ax);
    };
    run(OP_LINKS, BK_LINKS);
    run(OP_REDUCE, BK_REDUCE);
    if (b->any_rigid) run(OP_RIGID, BK_RIGID);
    run(OP_MARK, BK_REGION);
    run(OP_CLASSIFY, BK_REGION);
    HIPCHK(hipEventRecord(b->ev_flags[0], ax));
    run(OP_EMIT, BK_REGION);
    run(b->any_warm ? OP_LINKQ_WARM : OP_LINKQ, BK_LINKQ);
    launch_bulk_batch(b->storage, b->bw, b->d_cases, b->d_blk, b->nblocks, b->phase & 1, b->main);
    HIPCHK(hipStreamWaitEvent(b->main, b->ev_flags[0], 0));
    for (int i = 0; i < b->n; ++i) {
        lbm_ctx *c = b->cs[i];
        const int old = c->ic;
        c->ic = c->in; c->in = c->id; c->id = old;
        c->is = 1 - c->is;
        std::swap(c->A, c->B);
        c->steps++;
    }
    b->phase = (b->phase + 1) % GRAPH_PERIOD;
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

lbm_status join_aux(lbm_batch *b) {
    for (int k = 0; k < BATCH_AUX; ++k) {
        HIPCHK(hipEventRecord(b->ev_links[k], b->aux[k]));
        HIPCHK(hipStreamWaitEvent(b->main, b->ev_links[k], 0));
    }
    return LBM_OK;
}

lbm_status capture_graph(lbm_batch *b) {
    drop_graph(b);
    std::vector<long long> steps0;
    for (auto *c : b->cs) steps0.push_back(c->steps);
    const std::vector<uintptr_t> key = state_key(b);
    HIPCHK(hipStreamBeginCapture(b->main, hipStreamCaptureModeThreadLocal));
    lbm_status st = LBM_OK;
    for (int s = 0; s < GRAPH_PERIOD && st == LBM_OK; ++s) st = enqueue_batch_step(b);
    if (st == LBM_OK) st = join_aux(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->main, &g);
    // the capture executed nothing: the host-side rotation has come full circle
    for (int i = 0; i < b->n; ++i) b->cs[i]->steps = steps0[i];
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(LBM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (state_key(b) != key) {
        (void)hipGraphDestroy(g);
        return fail(LBM_E_STATE, "ensemble state did not return to its start after %d steps", GRAPH_PERIOD);
    }
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_key = key;
    return LBM_OK;
}

void free_batch(lbm_batch *b) {
    if (!b) return;
    if (b->main) (void)hipStreamSynchronize(b->main);
    for (hipStream_t a : b->aux)
        if (a) (void)hipStreamSynchronize(a);
    drop_graph(b);
    for (auto *c : b->cs) lbm_destroy(c);
    for (hipEvent_t e : {b->ev_in, b->ev_main, b->ev_out})
        if (e) (void)hipEventDestroy(e);
    for (int k = 0; k < BATCH_AUX; ++k) {
        if (b->ev_flags[k]) (void)hipEventDestroy(b->ev_flags[k]);
        if (b->ev_links[k]) (void)hipEventDestroy(b->ev_links[k]);
    }
    if (b->main) (void)hipStreamDestroy(b->main);
    for (hipStream_t a : b->aux)
        if (a) (void)hipStreamDestroy(a);
    delete b;
}

struct BatchLayout {
    std::vector<size_t> off, bytes;
    size_t off_cases, off_blk, off_blk1, blk_cap, blk1_cap, off_args, off_map, map_cap, total;
};

lbm_status batch_layout(int32_t n, const lbm_config *cfgs, const int32_t *n_p, const lbm_particle *parts,
                        BatchLayout &L) {
    if (n < 1) return fail(LBM_E_INVALID, "n_cases must be >= 1");
    if (!cfgs || !n_p) return fail(LBM_E_INVALID, "cfgs and n_p must not be NULL");
    size_t o = 0;
    long long pofs = 0, cap = 0, cap1 = 0, mcap = 0;
    for (int i = 0; i < n; ++i) {
        if (n_p[i] < 0) return fail(LBM_E_INVALID, "case %d: n_p < 0", i);
        if (cfgs[i].storage != cfgs[0].storage) return fail(LBM_E_INVALID, "all cases must use one storage type");
        std::vector<DevParticle> hp;
        Plan pl;
        lbm_status s = prepare(&cfgs[i], n_p[i], parts ? parts + pofs : nullptr, &hp, &pl);
        if (s) {
            const std::string m = g_err;
            return fail(s, "case %d: %s", i, m.c_str());
        }
        const size_t by = pl.total;
        Params pc{};
        pc.np = pl.np;
        pc.link_cap = pl.link_cap;
        pc.region_blocks = pl.region_blocks;
        mcap += case_blocks_cap(pc);
        L.off.push_back(o);
        L.bytes.push_back(by);
        o = align256(o + by);
        pofs += n_p[i];
        long long mx = 0;
        for (int t : TW_CANDIDATES) mx = std::max(mx, tile_blocks(cfgs[i], t, 4));
        cap += mx;
        cap1 = std::max(cap1, mx);
    }
    if (cap > 0x7fffffffll || mcap > 0x7fffffffll) return fail(LBM_E_INVALID, "ensemble too large for one launch");
    L.blk_cap = (size_t)cap;
    L.blk1_cap = (size_t)cap1;
    L.off_cases = o; o = align256(o + sizeof(BulkCase) * (n + 1));
    L.off_blk = o; o = align256(o + 4 * L.blk_cap);
    L.off_blk1 = o; o = align256(o + 4 * L.blk1_cap);
    L.off_args = o; o = align256(o + sizeof(CaseArgs) * GRAPH_PERIOD * (size_t)n);
    L.map_cap = (size_t)mcap;
    L.off_map = o; o = align256(o + 4 * L.map_cap);
    L.total = o;
    return LBM_OK;
}

// tiny reader of the tuning cache written by lbm_autotune: {"bw": B, "tiles": {"key": t, ...}}
bool cache_int(const std::string &txt, const std::string &key, int &v) {
    const std::string pat = "\"" + key + "\":";
    const size_t at = txt.find(pat);
    if (at == std::string::npos) return false;
    return std::sscanf(txt.c_str() + at + pat.size(), " %d", &v) == 1;
}

std::string case_key(const lbm_ctx *c) {
    char k[96];
    std::snprintf(k, sizeof k, "%dx%dx%d/s%d/p%u", c->p.nx, c->p.ny, c->p.nz, c->p.storage, c->p.periodic);
    return k;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_arena_bytes(int32_t n_cases, const lbm_config *cfgs, const int32_t *n_p,
                                 const lbm_particle *parts, size_t *bytes) {
    if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
    BatchLayout L;
    lbm_status s = batch_layout(n_cases, cfgs, n_p, parts, L);
    if (s) return s;
    *bytes = L.total;
    return LBM_OK;
}

lbm_status lbm_batch_init(int32_t n_cases, const lbm_config *cfgs, const int32_t *n_p, const lbm_particle *parts,
                          void *dev_arena, size_t arena_bytes, void *hip_stream, lbm_batch **out) {
    if (!out) return fail(LBM_E_INVALID, "out is NULL");
    *out = nullptr;
    BatchLayout L;
    lbm_status s = batch_layout(n_cases, cfgs, n_p, parts, L);
    if (s) return s;
    if (!dev_arena) return fail(LBM_E_INVALID, "arena is NULL");
    if ((uintptr_t)dev_arena & 255) return fail(LBM_E_INVALID, "arena must be 256-byte aligned");
    if (arena_bytes < L.total) return fail(LBM_E_NOMEM, "arena holds %zu bytes, %zu needed", arena_bytes, L.total);
    lbm_batch *b = new lbm_batch();
    b->n = n_cases;
    b->caller = (hipStream_t)hip_stream;
    b->storage = cfgs[0].storage;
    b->tw.assign(n_cases, 6);
    char *base = (char *)dev_arena;
    b->d_cases = (BulkCase *)(base + L.off_cases);
    b->d_blk = (int *)(base + L.off_blk);
    b->d_blk1 = (int *)(base + L.off_blk1);
    b->blk_cap = L.blk_cap;
    b->blk1_cap = L.blk1_cap;
    b->d_args = (CaseArgs *)(base + L.off_args);
    b->d_map = (int *)(base + L.off_map);
    b->map_cap = L.map_cap;
    long long pofs = 0;
    for (int i = 0; i < n_cases; ++i) {
        lbm_ctx *c = nullptr;
        s = lbm_init(&cfgs[i], n_p[i], parts ? parts + pofs : nullptr, base + L.off[i], L.bytes[i], hip_stream, &c);
        if (s) {
            const std::string m = g_err;
            free_batch(b);
            return fail(s, "case %d: %s", i, m.c_str());
        }
        b->cs.push_back(c);
        pofs += n_p[i];
    }
    auto bail = [&](hipError_t e, const char *what) {
        free_batch(b);
        return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&b->main, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    for (int k = 0; k < BATCH_AUX; ++k) {
        if ((e = hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
        if ((e = hipEventCreateWithFlags(&b->ev_flags[k], hipEventDisableTiming)) != hipSuccess) return bail(e, "event");
        if ((e = hipEventCreateWithFlags(&b->ev_links[k], hipEventDisableTiming)) != hipSuccess) return bail(e, "event");
    }
    for (hipEvent_t *ev : {&b->ev_in, &b->ev_main, &b->ev_out})
        if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) return bail(e, "event");
    // the systems were initialised on the caller's stream
    if ((e = hipStreamSynchronize(b->caller)) != hipSuccess) return bail(e, "hipStreamSynchronize");
    s = write_table(b);
    if (s) {
        const std::string m = g_err;
        free_batch(b);
        return fail(s, "%s", m.c_str());
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_case(lbm_batch *b, int32_t i, lbm_ctx **ctx) {
    if (!b || !ctx) return fail(LBM_E_INVALID, "batch and ctx must not be NULL");
    if (i < 0 || i >= b->n) return fail(LBM_E_INVALID, "case %d out of range", i);
    *ctx = b->cs[i];
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int32_t n_steps, int32_t use_graph) {
    if (!b) return fail(LBM_E_INVALID, "batch is NULL");
    if (n_steps < 0) return fail(LBM_E_INVALID, "n_steps must be >= 0");
    if (n_steps == 0) return LBM_OK;
    for (auto *c : b->cs)
        if (c->pending_refill) do_refill(c);
    // the ensemble's streams follow the caller's
    HIPCHK(hipEventRecord(b->ev_in, b->caller));
    HIPCHK(hipStreamWaitEvent(b->main, b->ev_in, 0));
    if (!table_valid(b)) {
        lbm_status s = write_table(b);
        if (s) return s;
    }
    while (n_steps > 0) {
        if (use_graph && n_steps >= GRAPH_PERIOD) {
            if (!b->exec || state_key(b) != b->graph_key) {
                lbm_status s = capture_graph(b);
                if (s) return s;
            }
            HIPCHK(hipGraphLaunch(b->exec, b->main));
            for (auto *c : b->cs) c->steps += GRAPH_PERIOD;
            n_steps -= GRAPH_PERIOD;
        } else {
            lbm_status s = enqueue_batch_step(b);
            if (s) return s;
            n_steps -= 1;
        }
    }
    lbm_status s = join_aux(b);
    if (s) return s;
    HIPCHK(hipEventRecord(b->ev_out, b->main));
    HIPCHK(hipStreamWaitEvent(b->caller, b->ev_out, 0));
    return LBM_OK;
}

lbm_status lbm_batch_tiles(lbm_batch *b, int32_t *tw_log2, int32_t *waves_per_block) {
    if (!b) return fail(LBM_E_INVALID, "batch is NULL");
    if (tw_log2)
        for (int i = 0; i < b->n; ++i) tw_log2[i] = b->tw[i];
    if (waves_per_block) *waves_per_block = b->bw;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_batch *b, double budget_ms, const char *cache_path) {
    if (!b) return fail(LBM_E_INVALID, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->caller));
    HIPCHK(hipStreamSynchronize(b->main));
    drop_graph(b);
    std::string txt;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "rb")) {
            char buf[4096];
            size_t r;
            while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, r);
            std::fclose(f);
        }
    }
    bool complete = !txt.empty();
    if (complete) {
        int bw = 8;
        if (!cache_int(txt, "bw", bw) || (bw != 4 && bw != 8)) complete = false;
        std::vector<int> tw(b->n, 6);
        for (int i = 0; i < b->n && complete; ++i)
            if (!cache_int(txt, case_key(b->cs[i]), tw[i]) || tw[i] < 4 || tw[i] > TW_FLAT) complete = false;
        if (complete) {
            b->bw = bw;
            b->tw = tw;
            return write_table(b);
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const auto t_start = std::chrono::steady_clock::now();
    auto elapsed_ms = [&] {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    };
    auto time_launch = [&](const BulkCase *cases, const int *blk, int nblk, int bw, float &best) -> lbm_status {
        best = 1e30f;
        launch_bulk_batch(b->storage, bw, cases, blk, nblk, 0, b->main);  // warm-up
        for (int r = 0; r < 3; ++r) {
            HIPCHK(hipEventRecord(e0, b->main));
            launch_bulk_batch(b->storage, bw, cases, blk, nblk, 0, b->main);
            HIPCHK(hipEventRecord(e1, b->main));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return LBM_OK;
    };
    // per system: the wave tile (one system per launch; the result buffer is
    // overwritten by the next step at every node the kernel touches)
    std::vector<int> blk1;
    lbm_status st = LBM_OK;
    std::map<std::string, int> seen;
    for (int i = 0; i < b->n && st == LBM_OK; ++i) {
        const std::string key = case_key(b->cs[i]);
        if (seen.count(key)) { b->tw[i] = seen[key]; continue; }
        if (elapsed_ms() > budget_ms) break;
        float best_ms = 1e30f;
        int best_t = b->tw[i];
        for (int t : TW_CANDIDATES) {
            BulkCase h = bulk_case(b->cs[i], t, 8, 0);
            blk1.assign(h.n_blocks, b->n);
            if (blk1.size() > b->blk1_cap) continue;
            st = hipMemcpy(b->d_cases + b->n, &h, sizeof h, hipMemcpyHostToDevice) == hipSuccess ? LBM_OK
                 : fail(LBM_E_HIP, "hipMemcpy");
            if (st) break;
            st = hipMemcpy(b->d_blk1, blk1.data(), 4 * blk1.size(), hipMemcpyHostToDevice) == hipSuccess ? LBM_OK
                 : fail(LBM_E_HIP, "hipMemcpy");
            if (st) break;
            float ms;
            st = time_launch(b->d_cases, b->d_blk1, h.n_blocks, 8, ms);
            if (st) break;
            if (ms < best_ms) { best_ms = ms; best_t = t; }
        }
        b->tw[i] = best_t;
        seen[key] = best_t;
    }
    // whole ensemble: waves per block
    if (st == LBM_OK && elapsed_ms() <= budget_ms) {
        float best_ms = 1e30f;
        int best_bw = b->bw;
        for (int bw : {8, 4}) {
            b->bw = bw;
            st = write_table(b);
            if (st) break;
            float ms;
            st = time_launch(b->d_cases, b->d_blk, b->nblocks, bw, ms);
            if (st) break;
            if (ms < best_ms) { best_ms = ms; best_bw = bw; }
        }
        b->bw = best_bw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    st = write_table(b);
    if (st) return st;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "wb")) {
            std::fprintf(f, "{\"bw\": %d, \"tiles\": {", b->bw);
            std::map<std::string, int> all;
            for (int i = 0; i < b->n; ++i) all[case_key(b->cs[i])] = b->tw[i];
            bool first = true;
            for (auto &kv : all) {
                std::fprintf(f, "%s\"%s\": %d", first ? "" : ", ", kv.first.c_str(), kv.second);
                first = false;
            }
            std::fprintf(f, "}}\n");
            std::fclose(f);
        } else {
            return fail(LBM_E_INVALID, "cannot write %s", cache_path);
        }
    }
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b) { free_batch(b); }

}  // extern "C"
