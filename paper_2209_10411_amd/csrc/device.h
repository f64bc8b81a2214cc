// Device-side data layout shared by the kernels and the host launcher.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mdl {

constexpr int Q = 19;
constexpr int MAXCP = 20;
constexpr int32_t FLUID = 0x7fffffff;  // owner value of a fluid node (atomicMin-friendly)
constexpr int PAD = 4;                  // region margin beyond the bounding radius
constexpr int BLK = 256;                // threads per block of the region kernels
constexpr int TILE_X = 8, TILE_Y = 8, TILE_Z = 4;  // a region block is a tile of BLK nodes

enum : int { ERR_LINK_OVERFLOW = 1, ERR_SPECIAL_OVERFLOW = 2, ERR_FAST_PARTICLE = 4,
             ERR_NONFINITE = 8, ERR_BAD_INDEX = 16, ERR_FLUID = 32 };

// Population layout: the nodes in runs of POP_RUN consecutive nodes, each
// run holding its Q populations one after another (POP_RUN elements each).
// A wave's load of one population covers a whole run segment, and the 19
// loads of a node range fall in one region of 19 x POP_RUN elements instead
// of 19 arrays far apart.  Node counts are padded to a multiple of POP_RUN
// (the array size Q * Ns).
constexpr int POP_RUN_LOG2 = 10, POP_RUN = 1 << POP_RUN_LOG2;
__host__ __device__ __forceinline__ long long pidx(long long n, int i) {
    return (((n >> POP_RUN_LOG2) * Q + i) << POP_RUN_LOG2) | (n & (POP_RUN - 1));
}
// The same in 32 bits (Q * Ns elements below 2^32).
__host__ __device__ __forceinline__ uint32_t pidx32(uint32_t n, int i) {
    return (((n >> POP_RUN_LOG2) * (uint32_t)Q + (uint32_t)i) << POP_RUN_LOG2) | (n & (uint32_t)(POP_RUN - 1));
}

// D3Q19 velocities in the order documented in midelbm.h.
constexpr int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
constexpr double WD[Q] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// FP64 particle record (one per body) living in device memory.
struct DevParticle {
    double X[3], q[4], v[3], w[3];  // centroid, body->lab quaternion, velocity, spin (lab)
    double m, V;
    double I[9], Iinv[9];           // body frame, about the centroid
    double F[3], T[3];              // hydrodynamic load of the last step
    double cpb[MAXCP][3];           // control points, body frame (origin = centroid)
    double k[MAXCP];
    double cpl[MAXCP][3];           // control points, lab frame, current pose
    double rb;                      // bounding radius about X
    int n_cp, mode;
    int half;                       // region half-width (ceil(rb) + PAD)
    int lo[3];                      // region origin (unwrapped), set from X each pose change
    int full[3];                    // 1: the region spans a whole periodic axis
    double X0[3];                   // centroid at the start of the current step
    // Region work is limited to balls about X: flags within re (extent of
    // the C >= 1 set), classification and link build within
    // re + sqrt 2 + reach, reach = distance to the centroids of the two
    // previous flaggings (Xf; hist = how many of them are known, reach
    // 1e30 until both are).
    double re;
    double reach;
    double Xf[2][3];
    int hist;
    int img;     // 0: no periodic image shifts any point evaluated near this body (see refresh_pose)
    double rsk;  // 1 / sqrt(sum k), the warm start's length scale (sum in point order)
};

// Small device-side counters, reset and read by the host at sync points.
struct Counters {
    int n_links;    // links of the current geometry
    int n_special;  // boundary and uncovered nodes listed this step
    int n_collect;  // samples written by the last contact-sample collection
    int pad2;
    int err;        // ERR_* bits
    uint32_t pad0;
    int pad[2];
    unsigned long long n_contacts;      // contacts resolved (pairs + walls, per sub-step)
    unsigned long long n_contact_fail;  // contact iterations that did not converge
    unsigned long long n_contact_nr;    // pair stationary-point solves (candidate pairs, per sub-step)
    unsigned long long n_contact_it;    // their Newton iterations
};

// Link-fraction solver statistics since the last read, one slot per block
// of the solver (no shared counters): histogram of the Newton evaluations per
// link (last bin: NR_HIST - 1 or more), evaluations and links, and the largest
// |C - 1| at a link's last evaluation (FP32 bits).  Summed on reading.
constexpr int NR_HIST = 65;
constexpr int NR_BLOCKS = 16384;  // largest grid of the solver
struct NrStats {
    unsigned int *hist;        // [NR_BLOCKS][NR_HIST]
    unsigned long long *work;  // [NR_BLOCKS][2]: evaluations, links
    unsigned int *resid;       // [NR_BLOCKS]
};

// Per-context constants, passed to kernels by value.
struct Params {
    int nx, ny, nz;
    unsigned periodic;
    long long N;
    long long Ns;  // N rounded up to POP_RUN (the population buffer holds Q * Ns elements, layout pidx)
    int np;
    int bc;
    int n_sub;
    int storage;
    float rho0f, omega, fcoef;  // 1/tau and 1 - 1/(2 tau)
    float gx, gy, gz;           // fluid body acceleration
    float scale, inv_scale;     // storage scale (FP16) and its inverse
    double rho0, tau;
    double gfd[3];              // fluid body acceleration, FP64
    double gp[3];               // particle gravity
    int link_cap, special_cap;
    int region_blocks;          // blocks of the region kernels
    int est_links, est_special; // expected list lengths (launch sizes of the list kernels; 0: capacities)
    int contact;                // contact enabled
    int link_c0;                // link fractions on the sphero-metaball level set (inner body, c_0 = s^2)
    double c_rs, c_kn, c_en, c_mu;
    // minimum image on a periodic axis of length L: for |d| < 1.25 L the
    // image shift k = floor(d / L + 0.5) (FP64) is +1 exactly when d >= mi_up
    // and -1 exactly when d < mi_dn (k is monotone in d; the host finds both
    // thresholds with the same FP64 operations)
    double mi_up[3], mi_dn[3];
};

// Per-sub-step contact results and tangential springs (arena), for bodies
// i < j at index i * np + j and walls at 6 * i + 2 * axis + side.
struct ContactBufs {
    double *pairF;   // [np*np][3] force on i
    double *pairTi;  // [np*np][3] torque on i
    double *pairTj;  // [np*np][3] torque on j
    double *wallF;   // [np*6][3]
    double *wallT;   // [np*6][3]
    double *xiP;     // [np*np][3] tangential springs, pairs
    double *xiW;     // [np*6][3] tangential springs, walls
    uint8_t *pairOn; // [np*np] 1 where the pair is in contact this sub-step (both (i,j) and (j,i))
    double *pairXm;     // [np*np][3] stationary point of the pair's last solve (i < j; frame of body i)
    uint8_t *pairOk;    // [np*np] 1 where that solve ran and converged
    double *pairGuess;  // [np*np][4] warm-start stationary point (x, y, z; NaN: none)
};

constexpr int TW_FLAT = 7;

// One system of an ensemble as seen by the batched stream-collide: sizes,
// collision constants, tile shape and block range, and the buffers of a step
// of either parity (parity 0: the assignment when the table was written).
struct BulkCase {
    int nx, ny, nz;
    unsigned periodic;
    long long N, Ns;
    float rho0f, omega, fcoef, gx, gy, gz, scale, inv_scale;
    int tw_log2;      // wave tile: 2^tw_log2 consecutive x by 64 >> tw_log2 rows of y (4..6), or
                      // TW_FLAT: 64 consecutive nodes in lattice order (rows wrap within a wave)
    int nsx, nsy;     // tiles along x and along y per z plane
    int first_block;  // first block of this system in the launch
    int n_blocks;     // blocks of this system
    void *A[2], *B[2];
    const uint8_t *skip[2];
    int *err;         // the system's error word (divergence sentinel)
};

// Region block map: block b of a region kernel works on particle part[b],
// tile first[b] of its region (tiles of TILE_X x TILE_Y x TILE_Z nodes, x
// fastest, then y, then z).
struct RegionMap {
    const int *part;
    const int *first;
    const int *dims;  // [np][3] region extent per axis
};

// Kernel kinds of the batched boundary launches (the three region kernels
// share one block range).
enum : int { BK_LINKS = 0, BK_REDUCE = 1, BK_RIGID = 2, BK_REGION = 3, BK_LINKQ = 4, BK_N = 5 };

// One system of an ensemble as seen by the batched boundary kernels: its
// constants and the buffers of one step, and its block range in each kind of
// launch (a block of a batched launch finds its system in a block -> system
// map and works as block  blockIdx.x - first[kind]  of a grid of nblk[kind]).
struct CaseArgs {
    Params p;
    RegionMap rm;
    void *A, *B;
    const int32_t *own_old;
    int32_t *own_new, *own_dead;
    uint8_t *skip_next;
    DevParticle *P;
    const int *part_first_blk;
    int *blk_cnt, *l_off, *body_stats;
    uint32_t *lmask, *l_node, *l_do, *special;
    double *l_q, *part;
    Counters *cnt;
    ContactBufs cb;
    NrStats nrs;
    const _Float16 *warm;   // warm-start MLP parameters, or NULL: plain Newton
    const float *mlp_body;  // [np][80] constant MLP inputs of each body
    int update;             // the force reduction also moves the bodies (no contact)
    int first[BK_N], nblk[BK_N];
};
// the host writes these tables for the device: one layout on both sides
static_assert(sizeof(Params) == 256 && sizeof(CaseArgs) == 600 && offsetof(CaseArgs, nrs) == 512 &&
                  offsetof(CaseArgs, first) == 556,
              "CaseArgs layout");

}  // namespace mdl
