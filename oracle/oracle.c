/*
 * oracle.c -- plain, slow FP64 CPU reference of the metaball-coupled
 * lattice Boltzmann time step of MI-DELBM (arXiv 2209.10411).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library: every constant below is written out here on its own.
 *
 * What it computes (paper section and equation cited at each function):
 *   - metaball flagging, C(x) = sum_i k_i/|x - p_i|^2, C >= 1 solid  (sec. 2.1, Eq. metaballM)
 *   - link fraction q of links cut by the C = 1 surface              (sec. 2.3.2, text after Eq. neqd)
 *   - D3Q19 BGK collision with Guo forcing                            (sec. 2.3.2; lattice and operator
 *                                                                      are not given by the paper: reading)
 *   - pull streaming with simple or interpolated bounce-back          (sec. 2.3.2, Eqs. eqneq1, eqneq2, neqd)
 *   - momentum-exchange force and torque, Galilean-invariant form     (sec. 2.3.2, MEM paragraph)
 *   - Newton-Euler rigid-body update with a unit quaternion           (sec. 2.3.1, Newton-Euler system)
 *   - local refilling of uncovered nodes                              (sec. 2.3.2, refilling equation)
 *
 * The canonical order of one step n -> n+1 (the paper gives the pieces but
 * not their order; this order is the reading used throughout):
 *   1 moments and collision at fluid nodes;  2 pull-stream into all nodes,
 *   cut links by bounce-back with the particle velocities at n;  3 momentum
 *   exchange over the cut links;  4 rigid-body update;  5 re-flag;  6 refill
 *   uncovered nodes with the particle state at n+1;  7 rebuild the links.
 *
 * All arithmetic is FP64 on full populations f_i (not deviations).
 * Loops over nodes may run under OpenMP; every reduction is serial and in a
 * fixed order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define MAX_CP 20
#define PI_D 3.14159265358979323846

/* D3Q19 velocities: rest, the six faces, the twelve edges; opposites are
 * adjacent (1/2, 3/4, ...). */
static const int EV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double WT[Q] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

typedef struct {
    int n_cp;
    double cpb[MAX_CP][3]; /* body frame, origin at the centroid */
    double k[MAX_CP];
    double cpl[MAX_CP][3]; /* lab frame at the current time */
    double X[3];           /* centroid, lab frame */
    double q[4];           /* body -> lab unit quaternion (w, x, y, z) */
    double v[3], w[3];     /* velocity, angular velocity (lab frame) */
    double m, V, I[3][3], Iinv[3][3];
    double rb;             /* bounding radius about X */
    int mode;              /* 0 free, 1 kinematic */
    double F[3], T[3];     /* hydrodynamic force and torque of the last step */
} orc_particle;

typedef struct orc_ctx {
    int nx, ny, nz;
    long N;
    unsigned periodic;
    double tau, rho0, gf[3], gp[3];
    int bc, n_sub, counter_force;
    /* contact (sec. 2.3.1): sphere radius R_s of the sphero-metaball, normal
     * stiffness k_n (0 disables contact), restitution e, friction mu_s */
    double c_rs, c_kn, c_en, c_mu;
    /* link fractions on the sphero-metaball level set (sec. 2.3.2: q solves
     * f = c_0 with c_0 depending on R_s): 0 = the C = 1 surface */
    int link_c0;
    double *xi_pair; /* [np][np][3] tangential springs of body pairs (i < j) */
    double *xi_wall; /* [np][6][3] tangential springs against the six faces */
    long n_contacts, n_contact_fail;
    int np, cap;
    orc_particle *P;
    double *f;      /* [Q][N] post-stream populations (the state) */
    double *fp;     /* [Q][N] post-collision scratch */
    double *rho;    /* [N]    density at time n */
    double *u;      /* [N][3] velocity at time n */
    int32_t *own;   /* [N] owner at the current time, -1 fluid */
    int32_t *own2;  /* [N] scratch for the next flags */
    /* links of the current time: node-major, direction-minor */
    long nl, lcap;
    int64_t *l_node;
    int32_t *l_dir, *l_own;
    double *l_q;
    int32_t *l_start; /* [N] first link of the node or -1 */
    uint8_t *l_cnt;   /* [N] number of links of the node */
    long n_refill, step;
} orc_ctx;

/* ------------------------------------------------------------ helpers */
static long idx(const orc_ctx *c, int x, int y, int z) {
    return (long)x + (long)c->nx * ((long)y + (long)c->ny * (long)z);
}

/* Neighbour of (x,y,z) displaced by d; 0 if it falls outside a wall. */
static int nbr(const orc_ctx *c, int x, int y, int z, int dx, int dy, int dz, long *out) {
    int p[3] = {x + dx, y + dy, z + dz};
    int L[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
        if (p[a] < 0 || p[a] >= L[a]) {
            if (!(c->periodic & (1u << a))) return 0;
            p[a] = (p[a] % L[a] + L[a]) % L[a];
        }
    }
    *out = idx(c, p[0], p[1], p[2]);
    return 1;
}

static void min_image(const orc_ctx *c, double d[3]) {
    double L[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a)
        if (c->periodic & (1u << a)) d[a] -= L[a] * floor(d[a] / L[a] + 0.5);
}

static void quat_to_rot(const double q[4], double R[3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

static void quat_mul(const double a[4], const double b[4], double o[4]) {
    double r[4];
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    memcpy(o, r, sizeof r);
}

/* Rotation quaternion for the rotation vector phi (angle |phi|). */
static void quat_exp(const double phi[3], double o[4]) {
    double a = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (a == 0.0) { o[0] = 1; o[1] = o[2] = o[3] = 0; return; }
    double s = sin(0.5 * a) / a;
    o[0] = cos(0.5 * a); o[1] = s * phi[0]; o[2] = s * phi[1]; o[3] = s * phi[2];
}

static void cross(const double a[3], const double b[3], double o[3]) {
    double r[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    memcpy(o, r, sizeof r);
}

static int inv3(const double A[3][3], double B[3][3]) {
    double d = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
             - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
             + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(fabs(d) > 0)) return -1;
    B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
    B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
    B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
    return 0;
}

/* -------------------------------------------------- metaball (sec. 2.1) */
/* Eq. metaballM on plain (non-periodic) coordinates; r = 0 gives +inf. */
double orc_metaball_eval(int n_cp, const double *cp, const double *k, const double x[3]) {
    double C = 0.0;
    for (int i = 0; i < n_cp; ++i) {
        double d0 = x[0] - cp[3 * i], d1 = x[1] - cp[3 * i + 1], d2 = x[2] - cp[3 * i + 2];
        double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (r2 == 0.0) return INFINITY;
        C += k[i] / r2;
    }
    return C;
}

/* Eq. metaballM for a particle in the lab frame, minimum image on periodic axes. */
static double metaball(const orc_ctx *c, const orc_particle *P, const double x[3]) {
    double C = 0.0;
    for (int i = 0; i < P->n_cp; ++i) {
        double d[3] = {x[0] - P->cpl[i][0], x[1] - P->cpl[i][1], x[2] - P->cpl[i][2]};
        min_image(c, d);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.0) return INFINITY;
        C += P->k[i] / r2;
    }
    return C;
}

/* Volume, centroid and inertia tensor (per unit density, about the
 * centroid) of the body C >= 1, by midpoint quadrature on cells of size h
 * over a grid centred on the box [min p - sqrt(sum k), max p + sqrt(sum k)];
 * the body lies in that box because C >= 1 needs some |x - p_i|^2 <= sum k.
 * Index sums are kept in integers so that symmetric bodies get an exactly
 * symmetric centroid. */
int orc_body_properties(int n_cp, const double *cp, const double *k, double h,
                        double *V, double c[3], double I[9], long *count) {
    double sk = 0.0;
    for (int i = 0; i < n_cp; ++i) sk += k[i];
    double rs = sqrt(sk), lo[3], hi[3];
    int n[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = cp[a]; hi[a] = cp[a];
        for (int i = 1; i < n_cp; ++i) {
            if (cp[3 * i + a] < lo[a]) lo[a] = cp[3 * i + a];
            if (cp[3 * i + a] > hi[a]) hi[a] = cp[3 * i + a];
        }
        lo[a] -= rs; hi[a] += rs;
        n[a] = (int)ceil((hi[a] - lo[a]) / h);
        lo[a] = 0.5 * (lo[a] + hi[a]) - 0.5 * n[a] * h; /* grid centred on the box */
    }
    /* pass 1: count and integer index sums (exact) for the centroid */
    long cnt = 0;
    int64_t s[3] = {0, 0, 0};
    for (int kz = 0; kz < n[2]; ++kz)
        for (int ky = 0; ky < n[1]; ++ky)
            for (int kx = 0; kx < n[0]; ++kx) {
                double x[3] = {lo[0] + (kx + 0.5) * h, lo[1] + (ky + 0.5) * h, lo[2] + (kz + 0.5) * h};
                if (orc_metaball_eval(n_cp, cp, k, x) >= 1.0) {
                    ++cnt; s[0] += kx; s[1] += ky; s[2] += kz;
                }
            }
    if (cnt == 0) return -1;
    for (int a = 0; a < 3; ++a) c[a] = lo[a] + h * ((double)s[a] / (double)cnt + 0.5);
    double J[6] = {0, 0, 0, 0, 0, 0}; /* sums of xx, yy, zz, xy, xz, yz */
    for (int kz = 0; kz < n[2]; ++kz)
        for (int ky = 0; ky < n[1]; ++ky)
            for (int kx = 0; kx < n[0]; ++kx) {
                double x[3] = {lo[0] + (kx + 0.5) * h, lo[1] + (ky + 0.5) * h, lo[2] + (kz + 0.5) * h};
                if (orc_metaball_eval(n_cp, cp, k, x) >= 1.0) {
                    double r0 = x[0] - c[0], r1 = x[1] - c[1], r2 = x[2] - c[2];
                    J[0] += r0 * r0; J[1] += r1 * r1; J[2] += r2 * r2;
                    J[3] += r0 * r1; J[4] += r0 * r2; J[5] += r1 * r2;
                }
            }
    double h3 = h * h * h;
    *V = (double)cnt * h3;
    I[0] = (J[1] + J[2]) * h3; I[4] = (J[0] + J[2]) * h3; I[8] = (J[0] + J[1]) * h3;
    I[1] = I[3] = -J[3] * h3; I[2] = I[6] = -J[4] * h3; I[5] = I[7] = -J[5] * h3;
    if (count) *count = cnt;
    return 0;
}

static void update_lab_cps(orc_particle *P) {
    double R[3][3];
    quat_to_rot(P->q, R);
    for (int i = 0; i < P->n_cp; ++i)
        for (int a = 0; a < 3; ++a)
            P->cpl[i][a] = P->X[a] + R[a][0] * P->cpb[i][0] + R[a][1] * P->cpb[i][1] + R[a][2] * P->cpb[i][2];
}

/* ------------------------------------------------------ lattice algebra */
/* Second-order equilibrium of direction i. */
static double feq(int i, double rho, const double u[3]) {
    double eu = EV[i][0] * u[0] + EV[i][1] * u[1] + EV[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return WT[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

void orc_feq(double rho, const double u[3], double out[Q]) {
    for (int i = 0; i < Q; ++i) out[i] = feq(i, rho, u);
}

/* Moments of a post-stream node: rho = sum f, u = (sum e f + F/2)/rho with
 * the body force F = rho g (Guo's half-force velocity). */
static void moments(const double f[Q], const double g[3], double *rho, double u[3]) {
    double r = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        j[0] += EV[i][0] * f[i]; j[1] += EV[i][1] * f[i]; j[2] += EV[i][2] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * r * g[a]) / r;
}

/* BGK collision with Guo forcing: f+ = f - (f - feq)/tau + F_i,
 * F_i = (1 - 1/(2 tau)) w_i [3 (e_i - u) + 9 (e_i . u) e_i] . F. */
void orc_collide_node(const double f[Q], const double g[3], double tau, double out[Q]) {
    double rho, u[3];
    moments(f, g, &rho, u);
    double F[3] = {rho * g[0], rho * g[1], rho * g[2]};
    for (int i = 0; i < Q; ++i) {
        double eu = EV[i][0] * u[0] + EV[i][1] * u[1] + EV[i][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += (3.0 * (EV[i][a] - u[a]) + 9.0 * eu * EV[i][a]) * F[a];
        double Fi = (1.0 - 0.5 / tau) * WT[i] * s;
        out[i] = f[i] - (f[i] - feq(i, rho, u)) / tau + Fi;
    }
}

/* ------------------------------------------------------------- context */
orc_ctx *orc_create(int nx, int ny, int nz, unsigned periodic, double tau, double rho0,
                    const double *gf, const double *gp, int bc, int n_sub, int counter_force) {
    if (nx < 3 || ny < 3 || nz < 3 || !(tau > 0.5) || n_sub < 1) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->nx = nx; c->ny = ny; c->nz = nz; c->N = (long)nx * ny * nz;
    c->periodic = periodic; c->tau = tau; c->rho0 = rho0;
    for (int a = 0; a < 3; ++a) { c->gf[a] = gf[a]; c->gp[a] = gp[a]; }
    c->bc = bc; c->n_sub = n_sub; c->counter_force = counter_force;
    c->f = (double *)malloc(sizeof(double) * Q * c->N);
    c->fp = (double *)malloc(sizeof(double) * Q * c->N);
    c->rho = (double *)malloc(sizeof(double) * c->N);
    c->u = (double *)malloc(sizeof(double) * 3 * c->N);
    c->own = (int32_t *)malloc(sizeof(int32_t) * c->N);
    c->own2 = (int32_t *)malloc(sizeof(int32_t) * c->N);
    c->l_start = (int32_t *)malloc(sizeof(int32_t) * c->N);
    c->l_cnt = (uint8_t *)malloc(c->N);
    if (!c->f || !c->fp || !c->rho || !c->u || !c->own || !c->own2 || !c->l_start || !c->l_cnt) {
        free(c->f); free(c->fp); free(c->rho); free(c->u); free(c->own); free(c->own2);
        free(c->l_start); free(c->l_cnt); free(c);
        return NULL;
    }
    return c;
}

void orc_destroy(orc_ctx *c) {
    if (!c) return;
    free(c->f); free(c->fp); free(c->rho); free(c->u); free(c->own); free(c->own2);
    free(c->l_start); free(c->l_cnt); free(c->l_node); free(c->l_dir); free(c->l_own);
    free(c->l_q); free(c->P); free(c->xi_pair); free(c->xi_wall); free(c);
}

/* Adds a body.  cp_xyz are in a body frame whose origin sits at x; the
 * centroid is computed here and becomes the reference point. */
int orc_add_particle(orc_ctx *c, int n_cp, const double *cp_xyz, const double *cp_k,
                     const double *x, const double *quat, const double *v, const double *w,
                     double density, int mode, double quad_h) {
    if (n_cp < 1 || n_cp > MAX_CP) return -1;
    for (int i = 0; i < n_cp; ++i) if (!(cp_k[i] > 0)) return -1;
    if (c->np == c->cap) {
        c->cap = c->cap ? 2 * c->cap : 4;
        c->P = (orc_particle *)realloc(c->P, sizeof(orc_particle) * c->cap);
    }
    orc_particle *P = &c->P[c->np];
    memset(P, 0, sizeof *P);
    P->n_cp = n_cp;
    double V, cen[3], I[9];
    if (orc_body_properties(n_cp, cp_xyz, cp_k, quad_h, &V, cen, I, NULL)) return -1;
    double nq = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    for (int a = 0; a < 4; ++a) P->q[a] = quat[a] / nq;
    double R[3][3];
    quat_to_rot(P->q, R);
    double sk = 0.0, rmax = 0.0;
    for (int i = 0; i < n_cp; ++i) {
        P->k[i] = cp_k[i]; sk += cp_k[i];
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            P->cpb[i][a] = cp_xyz[3 * i + a] - cen[a];
            r2 += P->cpb[i][a] * P->cpb[i][a];
        }
        if (sqrt(r2) > rmax) rmax = sqrt(r2);
    }
    for (int a = 0; a < 3; ++a) {
        P->X[a] = x[a] + R[a][0] * cen[0] + R[a][1] * cen[1] + R[a][2] * cen[2];
        P->v[a] = v[a]; P->w[a] = w[a];
    }
    P->rb = rmax + sqrt(sk);
    free(c->xi_pair);
    free(c->xi_wall);
    c->xi_pair = (double *)calloc(3 * (size_t)(c->np + 1) * (c->np + 1), sizeof(double));
    c->xi_wall = (double *)calloc(3 * 6 * (size_t)(c->np + 1), sizeof(double));
    P->V = V; P->m = density * V; P->mode = mode;
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) P->I[a][b] = density * I[3 * a + b];
    if (mode == 0 && inv3(P->I, P->Iinv)) return -1;
    update_lab_cps(P);
    c->np++;
    return c->np - 1;
}

/* Axis range of the cube around X of half-width rb (+1 node), wrapped or
 * clipped; a periodic axis shorter than the cube is covered once. */
static void cube_range(const orc_ctx *c, int a, double X, double rb, int *lo, int *hi, int *wrap) {
    int L = a == 0 ? c->nx : (a == 1 ? c->ny : c->nz);
    int l = (int)floor(X - rb) - 1, h = (int)ceil(X + rb) + 1;
    if (c->periodic & (1u << a)) {
        if (h - l + 1 >= L) { l = 0; h = L - 1; *wrap = 0; } else *wrap = 1;
    } else {
        if (l < 0) l = 0;
        if (h > L - 1) h = L - 1;
        *wrap = 0;
    }
    *lo = l; *hi = h;
}

/* Flags (sec. 2.1: C >= 1 inside).  Owner = the lowest-index body with
 * C >= 1 at the node, -1 for fluid.  Only nodes within the bounding radius
 * of a body can be inside it. */
static void flag_all(const orc_ctx *c, int32_t *own) {
    long N = c->N;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) own[n] = -1;
    for (int p = 0; p < c->np; ++p) {
        const orc_particle *P = &c->P[p];
        int lo[3], hi[3], wr[3];
        for (int a = 0; a < 3; ++a) cube_range(c, a, P->X[a], P->rb, &lo[a], &hi[a], &wr[a]);
        int L[3] = {c->nx, c->ny, c->nz};
#pragma omp parallel for schedule(static)
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    int q3[3] = {x, y, z};
                    for (int a = 0; a < 3; ++a)
                        if (wr[a]) q3[a] = (q3[a] % L[a] + L[a]) % L[a];
                    long n = idx(c, q3[0], q3[1], q3[2]);
                    if (own[n] >= 0) continue;
                    double xp[3] = {q3[0], q3[1], q3[2]};
                    if (metaball(c, P, xp) >= 1.0) own[n] = p;
                }
    }
}

/* Link fraction (sec. 2.3.2): along a cut link from the fluid node x_f
 * towards its solid neighbour x_f - e_i, q in (0, 1] is the first root of
 * g(s) = C_owner(x_f - s e_i) - 1 (g(0) < 0 <= g(1)).  The root is located in
 * the first of 8 equal sub-intervals where g changes sign and then refined
 * by bisection to full FP64 resolution.
 * With link_c0 (and a sphere radius R_s > 0), the surface the fluid sees is
 * the paper's level set f = c_0 of the sphero-metaball's zoomed inner body:
 * f_in(x) = sum s^2 k_j / |x - X - s (p_j - X)|^2 with s = 1 - R_s/sqrt(sum k),
 * and c_0 = s^2, the level at which f_in gives back a sphere's own radius
 * (the inner sphere of radius s sqrt(k) dilated by R_s).  Since
 * f_in(x) = C(X + (x - X)/s), g(s) = C(X + (x_f - s e_i - X)/s) - s^2.  When
 * this surface and C = 1 differ, g may keep one sign on (0, 1]: q = 1 when no
 * sample reaches the level, and q -> 0 when x_f itself lies inside. */
static double link_g(const orc_ctx *c, const orc_particle *P, const double xs[3], double *level) {
    if (!c->link_c0 || !(c->c_rs > 0.0)) {
        *level = 1.0;
        return metaball(c, P, xs);
    }
    double sk = 0.0;
    for (int j = 0; j < P->n_cp; ++j) sk += P->k[j];
    const double sc = 1.0 - c->c_rs / sqrt(sk);
    double r[3] = {xs[0] - P->X[0], xs[1] - P->X[1], xs[2] - P->X[2]};
    min_image(c, r);
    const double y[3] = {P->X[0] + r[0] / sc, P->X[1] + r[1] / sc, P->X[2] + r[2] / sc};
    *level = sc * sc;
    return metaball(c, P, y);
}

static double link_q(const orc_ctx *c, const orc_particle *P, int x, int y, int z, int i) {
    const int M = 8;
    double lo = 0.0, hi = 1.0, L;
    for (int k = 1; k <= M; ++k) {
        double s = (double)k / M;
        double xs[3] = {x - s * EV[i][0], y - s * EV[i][1], z - s * EV[i][2]};
        if (link_g(c, P, xs, &L) >= L) { lo = (double)(k - 1) / M; hi = s; break; }
    }
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double xs[3] = {x - mid * EV[i][0], y - mid * EV[i][1], z - mid * EV[i][2]};
        if (link_g(c, P, xs, &L) >= L) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

double orc_link_q(orc_ctx *c, int p, int x, int y, int z, int i) {
    return link_q(c, &c->P[p], x, y, z, i);
}

/* Cut links of the current flags: every fluid node x and direction i >= 1
 * whose source x - e_i is an in-domain solid node.  Node-major order. */
static void build_links(orc_ctx *c) {
    long N = c->N;
    int nz = c->nz;
    long *slab = (long *)calloc(nz + 1, sizeof(long));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        long cnt = 0;
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long n = idx(c, x, y, z);
                int k = 0;
                if (c->own[n] < 0)
                    for (int i = 1; i < Q; ++i) {
                        long s;
                        if (nbr(c, x, y, z, -EV[i][0], -EV[i][1], -EV[i][2], &s) && c->own[s] >= 0) ++k;
                    }
                c->l_cnt[n] = (uint8_t)k;
                cnt += k;
            }
        slab[z + 1] = cnt;
    }
    for (int z = 0; z < nz; ++z) slab[z + 1] += slab[z];
    c->nl = slab[nz];
    if (c->nl > c->lcap) {
        c->lcap = c->nl + c->nl / 2 + 16;
        c->l_node = (int64_t *)realloc(c->l_node, sizeof(int64_t) * c->lcap);
        c->l_dir = (int32_t *)realloc(c->l_dir, sizeof(int32_t) * c->lcap);
        c->l_own = (int32_t *)realloc(c->l_own, sizeof(int32_t) * c->lcap);
        c->l_q = (double *)realloc(c->l_q, sizeof(double) * c->lcap);
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        long o = slab[z];
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long n = idx(c, x, y, z);
                c->l_start[n] = c->l_cnt[n] ? (int32_t)o : -1;
                if (!c->l_cnt[n]) continue;
                for (int i = 1; i < Q; ++i) {
                    long s;
                    if (nbr(c, x, y, z, -EV[i][0], -EV[i][1], -EV[i][2], &s) && c->own[s] >= 0) {
                        c->l_node[o] = n; c->l_dir[o] = i; c->l_own[o] = c->own[s];
                        c->l_q[o] = link_q(c, &c->P[c->own[s]], x, y, z, i);
                        ++o;
                    }
                }
            }
    }
    (void)N;
    free(slab);
}

int orc_init(orc_ctx *c) {
    for (int p = 0; p < c->np; ++p) update_lab_cps(&c->P[p]);
    flag_all(c, c->own);
    if (c->counter_force) {
        /* periodic sedimentation: the fluid carries the opposite of the net
         * weight of the free bodies, spread over the fluid volume */
        long nf = 0;
        for (long n = 0; n < c->N; ++n) nf += c->own[n] < 0;
        double W[3] = {0, 0, 0};
        for (int p = 0; p < c->np; ++p)
            if (c->P[p].mode == 0)
                for (int a = 0; a < 3; ++a) W[a] += (c->P[p].m - c->rho0 * c->P[p].V) * c->gp[a];
        for (int a = 0; a < 3; ++a) c->gf[a] -= W[a] / (c->rho0 * (double)nf);
    }
    double u0[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        double fe = feq(i, c->rho0, u0);
        double *fi = c->f + (long)i * c->N;
        for (long n = 0; n < c->N; ++n) fi[n] = fe;
    }
    build_links(c);
    c->step = 0; c->n_refill = 0;
    return 0;
}

/* ------------------------------------------------------------ the step */
static void compute_macros(orc_ctx *c) {
    long N = c->N;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double fl[Q], r, u[3];
        for (int i = 0; i < Q; ++i) fl[i] = c->f[(long)i * N + n];
        moments(fl, c->gf, &r, u);
        c->rho[n] = r;
        c->u[3 * n] = u[0]; c->u[3 * n + 1] = u[1]; c->u[3 * n + 2] = u[2];
    }
}

static void collide_all(orc_ctx *c, double *out) {
    long N = c->N;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double fl[Q], fo[Q];
        for (int i = 0; i < Q; ++i) fl[i] = c->f[(long)i * N + n];
        if (c->own[n] < 0) orc_collide_node(fl, c->gf, c->tau, fo);
        else memcpy(fo, fl, sizeof fo);
        for (int i = 0; i < Q; ++i) out[(long)i * N + n] = fo[i];
    }
}

/* Surface velocity u = v + w x r of body p at lab point x (minimum image). */
static void surface_velocity(const orc_ctx *c, const orc_particle *P, const double x[3],
                             double uw[3], double r[3]) {
    r[0] = x[0] - P->X[0]; r[1] = x[1] - P->X[1]; r[2] = x[2] - P->X[2];
    min_image(c, r);
    double wr[3];
    cross(P->w, r, wr);
    for (int a = 0; a < 3; ++a) uw[a] = P->v[a] + wr[a];
}

/* Incoming population on a cut link (sec. 2.3.2, Eqs. eqneq1, eqneq2, neqd).
 * i arrives at the fluid node n = (x,y,z) from the solid side, ib = opp(i)
 * leaves towards the wall.  Simple bounce-back puts the wall halfway (q =
 * 1/2); interpolated bounce-back takes
 *   f_i = feq_ib(rho_f, u_d) + [f+_ib(x_f) - feq_ib(rho_f, u_f)] + 6 w rho0 e_i.u_w
 * with u_d = (1/3) u* + (2/3) u** from the paper's two linear interpolants, and
 * falls back to simple bounce-back when x_f + e_i is not a fluid node.
 * Returns the value; xw, uw, r receive the wall point, its velocity and the
 * lever arm about the centroid. */
static double bounce(const orc_ctx *c, long n, int x, int y, int z, int i, int p, double q,
                     double xw[3], double uw[3], double r[3]) {
    const orc_particle *P = &c->P[p];
    int ib = opp(i);
    long ff = -1;
    int ibb = c->bc == 1 && nbr(c, x, y, z, EV[i][0], EV[i][1], EV[i][2], &ff) && c->own[ff] < 0;
    double qq = ibb ? q : 0.5;
    xw[0] = x - qq * EV[i][0]; xw[1] = y - qq * EV[i][1]; xw[2] = z - qq * EV[i][2];
    surface_velocity(c, P, xw, uw, r);
    double eu = EV[i][0] * uw[0] + EV[i][1] * uw[1] + EV[i][2] * uw[2];
    double mw = 6.0 * WT[i] * c->rho0 * eu;
    double fb = c->fp[(long)ib * c->N + n];
    if (!ibb) return fb + mw;
    const double *uf = c->u + 3 * n, *uff = c->u + 3 * ff;
    double rf = c->rho[n], us[3], uss[3], ud[3];
    for (int a = 0; a < 3; ++a) {
        if (q <= 0.5) us[a] = 2.0 * q * uf[a] + (1.0 - 2.0 * q) * uff[a];
        else us[a] = (1.0 - q) / q * uf[a] + (2.0 * q - 1.0) / q * uw[a];
        uss[a] = (1.0 - q) / (1.0 + q) * uff[a] + 2.0 * q / (1.0 + q) * uw[a];
        ud[a] = us[a] / 3.0 + 2.0 * uss[a] / 3.0;
    }
    return feq(ib, rf, ud) + (fb - feq(ib, rf, uf)) + mw;
}

static void stream_all(orc_ctx *c) {
    long N = c->N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long n = idx(c, x, y, z);
                int fluid = c->own[n] < 0;
                for (int i = 0; i < Q; ++i) {
                    long s;
                    double val;
                    if (!nbr(c, x, y, z, -EV[i][0], -EV[i][1], -EV[i][2], &s)) {
                        val = c->fp[(long)opp(i) * N + n]; /* resting halfway wall */
                    } else if (fluid && c->own[s] >= 0) {
                        long l = c->l_start[n];
                        while (c->l_dir[l] != i) ++l;
                        double xw[3], uw[3], r[3];
                        val = bounce(c, n, x, y, z, i, c->l_own[l], c->l_q[l], xw, uw, r);
                    } else {
                        val = c->fp[(long)i * N + s];
                    }
                    c->f[(long)i * N + n] = val;
                }
            }
}

/* Momentum exchange over the cut links (sec. 2.3.2, MEM paragraph), in the
 * Galilean-invariant per-link form
 *   dP = (e_ib - u_w) f+_ib(x_f, t) - (e_i - u_w) f_i(x_f, t+1),
 *   dT = (x_w - X) x dP,
 * with both populations counted relative to w rho0.  Serial, link order. */
static void momentum_exchange(orc_ctx *c) {
    for (int p = 0; p < c->np; ++p)
        for (int a = 0; a < 3; ++a) c->P[p].F[a] = c->P[p].T[a] = 0.0;
    long N = c->N;
    for (long l = 0; l < c->nl; ++l) {
        long n = c->l_node[l];
        int i = c->l_dir[l], ib = opp(i), p = c->l_own[l];
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long)c->nx * c->ny));
        double xw[3], uw[3], r[3];
        /* exchanged populations taken relative to the rest state w rho0: the
         * uniform reference pressure then exerts no force, also on a body whose
         * surface touches a wall or another body and has no cut links there
         * (over a closed surface its per-link terms -2 w rho0 e_i cancel
         * exactly, since cut links come in opposite pairs of equal count) */
        double fin = bounce(c, n, x, y, z, i, p, c->l_q[l], xw, uw, r) - WT[i] * c->rho0;
        double fout = c->fp[(long)ib * N + n] - WT[ib] * c->rho0;
        double dP[3], dT[3];
        for (int a = 0; a < 3; ++a) dP[a] = (EV[ib][a] - uw[a]) * fout - (EV[i][a] - uw[a]) * fin;
        cross(r, dP, dT);
        for (int a = 0; a < 3; ++a) { c->P[p].F[a] += dP[a]; c->P[p].T[a] += dT[a]; }
    }
}

/* One sub-step dt of the Newton-Euler update (sec. 2.3.1) of one body
 * under total force F and torque T (lab frame, hydrodynamic + contact):
 * semi-implicit Euler for v and X; body-frame Euler equation
 * I dw_b/dt = T_b - w_b x I w_b for the spin; the attitude advances by the
 * exact rotation of w_b over the sub-step.  Weight minus buoyancy
 * (m - rho0 V) g acts on free bodies.  Kinematic bodies move with their given
 * v and w. */
static void body_substep(orc_ctx *c, orc_particle *P, const double F[3], const double T[3], double dt) {
    if (P->mode == 1) {
        double phi[3] = {P->w[0] * dt, P->w[1] * dt, P->w[2] * dt}, dq[4];
        for (int a = 0; a < 3; ++a) P->X[a] += P->v[a] * dt;
        quat_exp(phi, dq);
        quat_mul(dq, P->q, P->q);
    } else {
        double R[3][3], Tb[3], wb[3], Iw[3], g[3], rhs[3], dw[3];
        for (int a = 0; a < 3; ++a) {
            double Ft = F[a] + (P->m - c->rho0 * P->V) * c->gp[a];
            P->v[a] += Ft / P->m * dt;
            P->X[a] += P->v[a] * dt;
        }
        quat_to_rot(P->q, R);
        for (int a = 0; a < 3; ++a) {
            Tb[a] = R[0][a] * T[0] + R[1][a] * T[1] + R[2][a] * T[2];
            wb[a] = R[0][a] * P->w[0] + R[1][a] * P->w[1] + R[2][a] * P->w[2];
        }
        for (int a = 0; a < 3; ++a) Iw[a] = P->I[a][0] * wb[0] + P->I[a][1] * wb[1] + P->I[a][2] * wb[2];
        cross(wb, Iw, g);
        for (int a = 0; a < 3; ++a) rhs[a] = Tb[a] - g[a];
        for (int a = 0; a < 3; ++a) dw[a] = P->Iinv[a][0] * rhs[0] + P->Iinv[a][1] * rhs[1] + P->Iinv[a][2] * rhs[2];
        for (int a = 0; a < 3; ++a) wb[a] += dw[a] * dt;
        for (int a = 0; a < 3; ++a) P->w[a] = R[a][0] * wb[0] + R[a][1] * wb[1] + R[a][2] * wb[2];
        double phi[3] = {wb[0] * dt, wb[1] * dt, wb[2] * dt}, dq[4];
        quat_exp(phi, dq);
        quat_mul(P->q, dq, P->q);
    }
    double nq = sqrt(P->q[0] * P->q[0] + P->q[1] * P->q[1] + P->q[2] * P->q[2] + P->q[3] * P->q[3]);
    for (int a = 0; a < 4; ++a) P->q[a] /= nq;
    update_lab_cps(P);
}

/* ------------------------------------------------------ contact (sec. 2.3.1) */
/* Zoomed internal metaball of the sphero-metaball: the body scaled by
 * s = 1 - R_s / sqrt(sum k) about its centroid (control points
 * X + s (p - X), weights s^2 k), which is the same shape shrunk; dilating it
 * by a sphere of radius R_s approximates the body.  'shift' moves it to a
 * periodic image. */
static int inner_metaball(const orc_ctx *c, const orc_particle *P, const double shift[3],
                          double cp[][3], double k[]) {
    double sk = 0.0;
    for (int i = 0; i < P->n_cp; ++i) sk += P->k[i];
    double s = 1.0 - c->c_rs / sqrt(sk);
    if (!(s > 0.0)) return -1;
    for (int i = 0; i < P->n_cp; ++i) {
        for (int a = 0; a < 3; ++a) cp[i][a] = P->X[a] + shift[a] + s * (P->cpl[i][a] - P->X[a]);
        k[i] = s * s * P->k[i];
    }
    return P->n_cp;
}

/* f = sum k/r^2, its gradient sum -2 k d/r^4 and Hessian
 * sum 2 k (4 d d^T / r^6 - I / r^4) at x (d = x - p). */
static void mb_eval(int n, double cp[][3], const double k[], const double x[3], double *f, double g[3],
                    double H[3][3]) {
    *f = 0.0;
    for (int a = 0; a < 3; ++a) {
        g[a] = 0.0;
        for (int b = 0; b < 3; ++b) H[a][b] = 0.0;
    }
    for (int i = 0; i < n; ++i) {
        double d[3] = {x[0] - cp[i][0], x[1] - cp[i][1], x[2] - cp[i][2]};
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double r4 = r2 * r2, r6 = r4 * r2;
        *f += k[i] / r2;
        for (int a = 0; a < 3; ++a) {
            g[a] += -2.0 * k[i] * d[a] / r4;
            for (int b = 0; b < 3; ++b) H[a][b] += 2.0 * k[i] * (4.0 * d[a] * d[b] / r6 - (a == b ? 1.0 : 0.0) / r4);
        }
    }
}

/* Contact geometry of two bodies (Eqs. CM_coreF, eq:grad, eq:cp,
 * eq:contactprop): Newton-Raphson for the stationary point x_m of
 * f0 + f1 between the inner metaballs, started on the centroid segment at
 * the point dividing it in the ratio (K0/K1)^(1/3) (exact for single points);
 * Taylor projections x_c0 = x_m + q0 grad f0 with q0 = (1 - f0)/|grad f0|^2
 * (and likewise x_c1); n = (x_c0 - x_c1)/|x_c0 - x_c1| points from body 1 to
 * body 0; delta = 2 R_s - |x_c0 - x_c1| (in signed form, see below); the
 * contact point is the middle of the overlap on the line,
 * x_cp = x_c0 - (R_s - delta/2) n.  Returns 1 for a contact, 0 for none, -1
 * if the iteration failed. */
int orc_pair_geometry(orc_ctx *c, int i0, int i1, double xm[3], double xc0[3], double xc1[3],
                      double xcp[3], double nrm[3], double *delta) {
    const orc_particle *P0 = &c->P[i0], *P1 = &c->P[i1];
    double sh0[3] = {0, 0, 0}, sh1[3], d01[3];
    for (int a = 0; a < 3; ++a) d01[a] = P1->X[a] - P0->X[a];
    min_image(c, d01);
    for (int a = 0; a < 3; ++a) sh1[a] = P0->X[a] + d01[a] - P1->X[a];
    double cp0[MAX_CP][3], k0[MAX_CP], cp1[MAX_CP][3], k1[MAX_CP];
    int n0 = inner_metaball(c, P0, sh0, cp0, k0), n1 = inner_metaball(c, P1, sh1, cp1, k1);
    if (n0 < 0 || n1 < 0) return -1;
    double K0 = 0, K1 = 0;
    for (int i = 0; i < n0; ++i) K0 += k0[i];
    for (int i = 0; i < n1; ++i) K1 += k1[i];
    double rho = cbrt(K0 / K1);
    for (int a = 0; a < 3; ++a) xm[a] = P0->X[a] + d01[a] * rho / (1.0 + rho);
    double L = sqrt(d01[0] * d01[0] + d01[1] * d01[1] + d01[2] * d01[2]);
    int ok = 0;
    for (int it = 0; it < 60; ++it) {
        double f0, g0[3], H0[3][3], f1, g1[3], H1[3][3], H[3][3], Hi[3][3], dx[3];
        mb_eval(n0, cp0, k0, xm, &f0, g0, H0);
        mb_eval(n1, cp1, k1, xm, &f1, g1, H1);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) H[a][b] = H0[a][b] + H1[a][b];
        if (inv3(H, Hi)) break;
        double st = 0.0;
        for (int a = 0; a < 3; ++a) {
            dx[a] = -(Hi[a][0] * (g0[0] + g1[0]) + Hi[a][1] * (g0[1] + g1[1]) + Hi[a][2] * (g0[2] + g1[2]));
            st += dx[a] * dx[a];
        }
        st = sqrt(st);
        if (st > 0.25 * L) for (int a = 0; a < 3; ++a) dx[a] *= 0.25 * L / st;
        for (int a = 0; a < 3; ++a) xm[a] += dx[a];
        if (st < 1e-12 * (1.0 + L)) { ok = 1; break; }
    }
    if (!ok) return -1;
    double f0, g0[3], H0[3][3], f1, g1[3], H1[3][3];
    mb_eval(n0, cp0, k0, xm, &f0, g0, H0);
    mb_eval(n1, cp1, k1, xm, &f1, g1, H1);
    double G0 = sqrt(g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2]);
    double G1 = sqrt(g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]);
    if (!(G0 > 0.0 && G1 > 0.0)) return -1;
    double q0 = (1.0 - f0) / (G0 * G0), q1 = (1.0 - f1) / (G1 * G1);
    /* At the stationary point grad f0 = -grad f1, so x_c0 - x_c1 lies along
     * n = grad f0/|grad f0| (from body 1 towards body 0) and its signed length
     * is s = (1 - f0)/|grad f0| + (1 - f1)/|grad f1|, which stays meaningful
     * when the inner bodies overlap (s < 0). */
    double sgap = (1.0 - f0) / G0 + (1.0 - f1) / G1;
    *delta = 2.0 * c->c_rs - sgap;
    for (int a = 0; a < 3; ++a) {
        xc0[a] = xm[a] + q0 * g0[a];
        xc1[a] = xm[a] + q1 * g1[a];
        nrm[a] = g0[a] / G0;
        xcp[a] = xc0[a] - (c->c_rs - 0.5 * *delta) * nrm[a];
    }
    return *delta > 0.0;
}

/* Contact of a body with the halfway wall normal to axis ax (side 0: the
 * wall at -1/2, side 1: at L - 1/2) (Eqs. metawallcp, contactprop2): the
 * point x_cw of the wall plane where grad f is normal to the plane (2-D
 * Newton-Raphson on the in-plane gradient, started at the projection of the
 * control point where f on the plane is largest),
 * x_cm = x_cw + q grad f with q = (1 - f)/|grad f|^2, n = (x_cm - x_cw)/|...|
 * (into the domain), delta = R_s - |x_cm - x_cw|, x_cp = x_cw + delta/2 n. */
int orc_wall_geometry(orc_ctx *c, int ip, int ax, int side, double xcw[3], double xcm[3], double xcp[3],
                      double nrm[3], double *delta) {
    const orc_particle *P = &c->P[ip];
    int L = ax == 0 ? c->nx : (ax == 1 ? c->ny : c->nz);
    double wpos = side ? L - 0.5 : -0.5;
    if (fabs(P->X[ax] - wpos) > P->rb + c->c_rs) return 0;
    double sh[3] = {0, 0, 0}, cp[MAX_CP][3], k[MAX_CP];
    int n = inner_metaball(c, P, sh, cp, k);
    if (n < 0) return -1;
    int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
    /* start: the projection onto the plane of the control point where f on
     * the plane is largest (near the maximum of f over the plane) */
    double best = -1.0;
    for (int i = 0; i < n; ++i) {
        double y[3] = {cp[i][0], cp[i][1], cp[i][2]}, fy, gy[3], Hy[3][3];
        y[ax] = wpos;
        mb_eval(n, cp, k, y, &fy, gy, Hy);
        if (fy > best) {
            best = fy;
            for (int a = 0; a < 3; ++a) xcw[a] = y[a];
        }
    }
    int ok = 0;
    for (int it = 0; it < 60; ++it) {
        double f, g[3], H[3][3];
        mb_eval(n, cp, k, xcw, &f, g, H);
        double h11 = H[a1][a1], h12 = H[a1][a2], h22 = H[a2][a2];
        double det = h11 * h22 - h12 * h12;
        if (!(fabs(det) > 0)) break;
        double d1 = -(h22 * g[a1] - h12 * g[a2]) / det, d2 = -(-h12 * g[a1] + h11 * g[a2]) / det;
        double st = sqrt(d1 * d1 + d2 * d2);
        if (st > 0.25 * P->rb) { d1 *= 0.25 * P->rb / st; d2 *= 0.25 * P->rb / st; }
        xcw[a1] += d1;
        xcw[a2] += d2;
        if (st < 1e-12 * (1.0 + P->rb)) { ok = 1; break; }
    }
    if (!ok) return -1;
    double f, g[3], H[3][3];
    mb_eval(n, cp, k, xcw, &f, g, H);
    double G = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (!(G > 0.0)) return -1;
    double q = (1.0 - f) / (G * G);
    /* grad f is normal to the plane at x_cw and points into the body, so
     * x_cm - x_cw = q grad f has the signed length (1 - f)/|grad f| along
     * n = grad f/|grad f| (negative when the inner body crosses the plane). */
    *delta = c->c_rs - (1.0 - f) / G;
    for (int a = 0; a < 3; ++a) {
        xcm[a] = xcw[a] + q * g[a];
        nrm[a] = g[a] / G;
        xcp[a] = xcw[a] + 0.5 * *delta * nrm[a];
    }
    return *delta > 0.0;
}

/* Linear spring-dashpot with a Coulomb-capped tangential spring (sec. 2.3.1):
 * F_n = k_n delta + eta_n (v_j - v_i).n while delta > 0, eta_n from the
 * restitution e and the effective mass; tangential spring xi advanced by the
 * tangential relative velocity u_t (kept in the tangent plane), F_t =
 * k_t xi + eta_t u_t with k_t = 2/7 k_n, eta_t = eta_n, capped at mu_s F_n.
 * Returns the force on body i (along +n from j to i) in F. */
static void spring_dashpot(const orc_ctx *c, double meff, const double n[3], double delta,
                           const double vrel[3], double xi[3], double dt, double F[3]) {
    double le = log(c->c_en);
    double zeta = -le / sqrt(PI_D * PI_D + le * le);
    double etan = 2.0 * zeta * sqrt(meff * c->c_kn), kt = 2.0 / 7.0 * c->c_kn, etat = etan;
    double vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    double Fn = c->c_kn * delta + etan * vn;
    double ut[3], xn = xi[0] * n[0] + xi[1] * n[1] + xi[2] * n[2], Ft[3], ftn = 0.0;
    for (int a = 0; a < 3; ++a) {
        ut[a] = vrel[a] - vn * n[a];
        xi[a] = xi[a] - xn * n[a] + ut[a] * dt;
        Ft[a] = kt * xi[a] + etat * ut[a];
        ftn += Ft[a] * Ft[a];
    }
    ftn = sqrt(ftn);
    double cap = c->c_mu * fabs(Fn);
    if (ftn > cap && ftn > 0.0) {
        for (int a = 0; a < 3; ++a) {
            Ft[a] *= cap / ftn;
            xi[a] = Ft[a] / kt;
        }
    }
    for (int a = 0; a < 3; ++a) F[a] = Fn * n[a] + Ft[a];
}

static void point_velocity(const orc_ctx *c, const orc_particle *P, const double x[3], double v[3]) {
    double r[3] = {x[0] - P->X[0], x[1] - P->X[1], x[2] - P->X[2]}, wr[3];
    min_image(c, r);
    cross(P->w, r, wr);
    for (int a = 0; a < 3; ++a) v[a] = P->v[a] + wr[a];
}

/* Contact forces and torques on every body at the current poses: body
 * pairs whose bounding spheres overlap and bodies near walled faces.  Sums
 * in a fixed order (pairs by i then j). */
static void contact_forces(orc_ctx *c, double (*Fc)[3], double (*Tc)[3], double dt) {
    int np = c->np;
    for (int p = 0; p < np; ++p)
        for (int a = 0; a < 3; ++a) Fc[p][a] = Tc[p][a] = 0.0;
    if (!(c->c_kn > 0.0)) return;
    for (int i = 0; i < np; ++i)
        for (int j = i + 1; j < np; ++j) {
            orc_particle *Pi = &c->P[i], *Pj = &c->P[j];
            double *xi = c->xi_pair + 3 * ((long)i * np + j);
            if (Pi->mode == 1 && Pj->mode == 1) continue;
            double d[3] = {Pj->X[0] - Pi->X[0], Pj->X[1] - Pi->X[1], Pj->X[2] - Pi->X[2]};
            min_image(c, d);
            if (sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) > Pi->rb + Pj->rb) {
                xi[0] = xi[1] = xi[2] = 0.0;
                continue;
            }
            double xm[3], xc0[3], xc1[3], xcp[3], n[3], delta;
            int r = orc_pair_geometry(c, i, j, xm, xc0, xc1, xcp, n, &delta);
            if (r < 0) c->n_contact_fail++;
            if (r <= 0) { xi[0] = xi[1] = xi[2] = 0.0; continue; }
            c->n_contacts++;
            double vi[3], vj[3], vrel[3], F[3], ri[3], rj[3], Ti[3], Tj[3];
            point_velocity(c, Pi, xcp, vi);
            point_velocity(c, Pj, xcp, vj);
            for (int a = 0; a < 3; ++a) vrel[a] = vj[a] - vi[a];
            double meff = Pi->mode == 1 ? Pj->m : (Pj->mode == 1 ? Pi->m : Pi->m * Pj->m / (Pi->m + Pj->m));
            spring_dashpot(c, meff, n, delta, vrel, xi, dt, F);
            for (int a = 0; a < 3; ++a) { ri[a] = xcp[a] - Pi->X[a]; rj[a] = xcp[a] - Pj->X[a]; }
            min_image(c, ri);
            min_image(c, rj);
            double Fm[3] = {-F[0], -F[1], -F[2]};
            cross(ri, F, Ti);
            cross(rj, Fm, Tj);
            for (int a = 0; a < 3; ++a) {
                Fc[i][a] += F[a]; Tc[i][a] += Ti[a];
                Fc[j][a] += Fm[a]; Tc[j][a] += Tj[a];
            }
        }
    for (int i = 0; i < np; ++i) {
        orc_particle *Pi = &c->P[i];
        if (Pi->mode == 1) continue;
        for (int ax = 0; ax < 3; ++ax) {
            if (c->periodic & (1u << ax)) continue;
            for (int side = 0; side < 2; ++side) {
                double *xi = c->xi_wall + 3 * ((long)i * 6 + 2 * ax + side);
                double xcw[3], xcm[3], xcp[3], n[3], delta;
                int r = orc_wall_geometry(c, i, ax, side, xcw, xcm, xcp, n, &delta);
                if (r < 0) c->n_contact_fail++;
                if (r <= 0) { xi[0] = xi[1] = xi[2] = 0.0; continue; }
                c->n_contacts++;
                double vi[3], vrel[3], F[3], ri[3], Ti[3];
                point_velocity(c, Pi, xcp, vi);
                for (int a = 0; a < 3; ++a) vrel[a] = -vi[a];
                spring_dashpot(c, Pi->m, n, delta, vrel, xi, dt, F);
                for (int a = 0; a < 3; ++a) ri[a] = xcp[a] - Pi->X[a];
                cross(ri, F, Ti);
                for (int a = 0; a < 3; ++a) { Fc[i][a] += F[a]; Tc[i][a] += Ti[a]; }
            }
        }
    }
}

/* Rigid-body update of all bodies over one lattice time unit: n_sub
 * sub-steps, each with contact forces recomputed at the sub-step's poses and
 * the hydrodynamic load of the lattice step held. */
static void rigid_update_all(orc_ctx *c) {
    double dt = 1.0 / c->n_sub;
    int np = c->np;
    double (*Fc)[3] = malloc(sizeof(double[3]) * (np ? np : 1));
    double (*Tc)[3] = malloc(sizeof(double[3]) * (np ? np : 1));
    for (int s = 0; s < c->n_sub; ++s) {
        contact_forces(c, Fc, Tc, dt);
        for (int p = 0; p < np; ++p) {
            double F[3], T[3];
            for (int a = 0; a < 3; ++a) { F[a] = c->P[p].F[a] + Fc[p][a]; T[a] = c->P[p].T[a] + Tc[p][a]; }
            body_substep(c, &c->P[p], F, T, dt);
        }
    }
    free(Fc);
    free(Tc);
}

/* One lattice time unit of body p alone under a given hydrodynamic load (no
 * contact); used by tests. */
int orc_rigid_body_step(orc_ctx *c, int p, const double *F, const double *T) {
    if (p < 0 || p >= c->np) return -1;
    double dt = 1.0 / c->n_sub;
    for (int s = 0; s < c->n_sub; ++s) body_substep(c, &c->P[p], F, T, dt);
    return 0;
}

/* Bodies only (no fluid): n lattice time units of contact dynamics with the
 * hydrodynamic load set to zero; used by tests. */
int orc_dem_only(orc_ctx *c, int nsteps) {
    for (int p = 0; p < c->np; ++p)
        for (int a = 0; a < 3; ++a) c->P[p].F[a] = c->P[p].T[a] = 0.0;
    for (int t = 0; t < nsteps; ++t) rigid_update_all(c);
    return 0;
}

void orc_set_link_c0(orc_ctx *c, int on) { c->link_c0 = on; build_links(c); }

void orc_set_contact(orc_ctx *c, double rs, double kn, double en, double mu) {
    c->c_rs = rs; c->c_kn = kn; c->c_en = en; c->c_mu = mu;
}

long orc_n_contacts(const orc_ctx *c) { return c->n_contacts; }
long orc_n_contact_fail(const orc_ctx *c) { return c->n_contact_fail; }

/* Local refilling (sec. 2.3.2): a node solid at n and fluid at n+1 keeps the
 * populations that streamed in from nodes that were fluid; a missing f_i
 * takes the bounce-back of its opposite, f_ib + 6 w rho0 e_i . u_new, when
 * that opposite came from a fluid node, and the equilibrium at (rho0, u_new)
 * otherwise; u_new = v + w x (x - X) of the body that covered the node, at
 * n+1. */
static void refill(orc_ctx *c, const int32_t *own_old, const int32_t *own_new) {
    long N = c->N, cnt = 0;
#pragma omp parallel for schedule(static) reduction(+ : cnt)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long n = idx(c, x, y, z);
                if (!(own_old[n] >= 0 && own_new[n] < 0)) continue;
                ++cnt;
                const orc_particle *P = &c->P[own_old[n]];
                double xp[3] = {x, y, z}, un[3], r[3];
                surface_velocity(c, P, xp, un, r);
                for (int i = 0; i < Q; ++i) {
                    long s;
                    if (nbr(c, x, y, z, -EV[i][0], -EV[i][1], -EV[i][2], &s) && own_old[s] < 0) continue;
                    if (nbr(c, x, y, z, EV[i][0], EV[i][1], EV[i][2], &s) && own_old[s] < 0) {
                        double eu = EV[i][0] * un[0] + EV[i][1] * un[1] + EV[i][2] * un[2];
                        c->f[(long)i * N + n] = c->f[(long)opp(i) * N + n] + 6.0 * WT[i] * c->rho0 * eu;
                    } else {
                        c->f[(long)i * N + n] = feq(i, c->rho0, un);
                    }
                }
            }
    c->n_refill = cnt;
}

int orc_step(orc_ctx *c, int nsteps) {
    for (int t = 0; t < nsteps; ++t) {
        compute_macros(c);                 /* 1 */
        collide_all(c, c->fp);
        stream_all(c);                     /* 2 */
        momentum_exchange(c);              /* 3 */
        rigid_update_all(c);               /* 4 */
        flag_all(c, c->own2);              /* 5 */
        refill(c, c->own, c->own2);        /* 6 */
        int32_t *t2 = c->own; c->own = c->own2; c->own2 = t2;
        build_links(c);                    /* 7 */
        c->step++;
    }
    return 0;
}

/* ------------------------------------------------------------- access */
long orc_n_nodes(const orc_ctx *c) { return c->N; }
long orc_n_links(const orc_ctx *c) { return c->nl; }
long orc_n_refilled(const orc_ctx *c) { return c->n_refill; }
int orc_n_particles(const orc_ctx *c) { return c->np; }
void orc_get_gfluid(const orc_ctx *c, double *g) { memcpy(g, c->gf, 3 * sizeof(double)); }

void orc_get_f(const orc_ctx *c, double *out) { memcpy(out, c->f, sizeof(double) * Q * c->N); }
int orc_set_f(orc_ctx *c, const double *in) { memcpy(c->f, in, sizeof(double) * Q * c->N); return 0; }

/* Post-collision populations of the current state (collision at fluid
 * nodes only; solid nodes are copied). */
void orc_get_fpost(orc_ctx *c, double *out) { collide_all(c, out); }

void orc_get_macros(orc_ctx *c, double *rho, double *u) {
    compute_macros(c);
    memcpy(rho, c->rho, sizeof(double) * c->N);
    memcpy(u, c->u, sizeof(double) * 3 * c->N);
}

void orc_get_owner(const orc_ctx *c, int32_t *own) { memcpy(own, c->own, sizeof(int32_t) * c->N); }

void orc_get_links(const orc_ctx *c, int64_t *node, int32_t *dir, int32_t *own, double *q) {
    memcpy(node, c->l_node, sizeof(int64_t) * c->nl);
    memcpy(dir, c->l_dir, sizeof(int32_t) * c->nl);
    memcpy(own, c->l_own, sizeof(int32_t) * c->nl);
    memcpy(q, c->l_q, sizeof(double) * c->nl);
}

/* Particle record: X(3) q(4) v(3) w(3) F(3) T(3) m V I(9) rb n_cp = 32 doubles. */
int orc_get_particle(const orc_ctx *c, int p, double *o) {
    if (p < 0 || p >= c->np) return -1;
    const orc_particle *P = &c->P[p];
    memcpy(o, P->X, 3 * sizeof(double)); memcpy(o + 3, P->q, 4 * sizeof(double));
    memcpy(o + 7, P->v, 3 * sizeof(double)); memcpy(o + 10, P->w, 3 * sizeof(double));
    memcpy(o + 13, P->F, 3 * sizeof(double)); memcpy(o + 16, P->T, 3 * sizeof(double));
    o[19] = P->m; o[20] = P->V;
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) o[21 + 3 * a + b] = P->I[a][b];
    o[30] = P->rb; o[31] = P->n_cp;
    return 0;
}

int orc_set_particle_state(orc_ctx *c, int p, const double *X, const double *q,
                           const double *v, const double *w) {
    if (p < 0 || p >= c->np) return -1;
    orc_particle *P = &c->P[p];
    memcpy(P->X, X, 3 * sizeof(double)); memcpy(P->q, q, 4 * sizeof(double));
    memcpy(P->v, v, 3 * sizeof(double)); memcpy(P->w, w, 3 * sizeof(double));
    update_lab_cps(P);
    return 0;
}

int orc_get_cps(const orc_ctx *c, int p, double *lab, double *k) {
    if (p < 0 || p >= c->np) return -1;
    const orc_particle *P = &c->P[p];
    for (int i = 0; i < P->n_cp; ++i) {
        for (int a = 0; a < 3; ++a) lab[3 * i + a] = P->cpl[i][a];
        k[i] = P->k[i];
    }
    return P->n_cp;
}

/* Re-derives flags and links from the current particle state (used after
 * orc_set_particle_state). */
int orc_reflag(orc_ctx *c) { flag_all(c, c->own); build_links(c); return 0; }

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads the oracle's loops use (n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* The lattice table, for tests that check it against the D3Q19 definition. */
void orc_lattice(int32_t *e, double *w, int32_t *op) {
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = EV[i][a];
        w[i] = WT[i];
        op[i] = opp(i);
    }
}
