/*
 * midelbm.h -- C ABI of the MI355X (gfx950) implementation of the per-step
 * hot path of the Metaball-Imaging Discrete Element Lattice Boltzmann
 * Method (MI-DELBM, arXiv 2209.10411).
 *
 * One call of lbm_step(..., LBM_STEP_COUPLED) advances the coupled system by
 * one lattice time unit:
 *   1. bounce-back on every link cut by a metaball surface (paper sec. 2.3.2,
 *      Eqs. eqneq1, eqneq2, neqd) and the momentum exchange on those links
 *      (sec. 2.3.2, MEM paragraph; Galilean-invariant per-link form);
 *   2. the FP64 Newton-Euler update of every particle (sec. 2.3.1);
 *   3. metaball flagging of the nodes near each particle (sec. 2.1,
 *      Eq. metaballM; C(x) >= 1 is solid);
 *   4. D3Q19 BGK stream-and-collide of every fluid node, with the local
 *      refilling of uncovered nodes (sec. 2.3.2, refilling equation) between
 *      streaming and collision;
 *   5. the cut-link list and link fractions q of the new geometry
 *      (sec. 2.3.2: q solves C(x_f - q e_i) = 1 along the link).
 * The paper gives no lattice, collision operator or forcing; this library
 * uses D3Q19 BGK with Guo forcing.
 *
 * Conventions
 *   - Lattice units.  Node (x, y, z) sits at integer coordinates; its linear
 *     index is x + nx*(y + ny*z).  Non-periodic faces are resting no-slip
 *     walls halfway outside the outermost nodes.
 *   - Populations are stored post-collision, as deviations f_i - w_i rho0,
 *     structure-of-arrays [19][N] in FP32, FP16 (times fp16_scale) or BF16,
 *     in two ping-pong buffers.  Velocity i = 0 is rest, 1..6 are +x,-x,+y,
 *     -y,+z,-z, 7..18 the edges (+x+y,-x-y,+x-y,-x+y,+x+z,-x-z,+x-z,-x+z,
 *     +y+z,-y-z,+y-z,-y+z); opposites are adjacent.
 *   - Particles: FP64 state on the device.  cp_xyz are control points in a
 *     body frame whose origin is placed at x with orientation quat
 *     (w, x, y, z); the library computes volume, centroid and inertia by
 *     midpoint quadrature with cell size quad_h and thereafter refers the
 *     particle to its centroid.  A node covered by several bodies belongs to
 *     the lowest-index one.
 *
 * Memory and ownership
 *   - Device memory is one caller-owned arena (any device allocation, e.g. a
 *     torch uint8 tensor) of at least lbm_arena_bytes() bytes, passed to
 *     lbm_init; the library sub-allocates it and never allocates device
 *     memory itself nor frees the arena.  Host input arrays are copied
 *     during the call and not retained.  lbm_destroy frees host state only.
 *   - All device work is enqueued on the caller's HIP stream given to
 *     lbm_init.  Calls that return data to the host synchronise that stream.
 *
 * Errors
 *   - Every call returns an lbm_status; lbm_last_error() gives a message for
 *     the last failure on the calling thread.  Device-side conditions (link
 *     list overflow, a particle moving more than one lattice unit per step,
 *     a non-finite particle state, and the fluid sentinel: a plain fluid node
 *     whose moments are not finite or whose velocity exceeds 0.3 lattice
 *     units, checked by the stream-collide at every node of every step) are
 *     recorded on the device, stay set, and are reported as LBM_E_DIVERGED or
 *     LBM_E_NOMEM by every later synchronising call.
 */
#ifndef MIDELBM_H
#define MIDELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

typedef enum {
    LBM_OK = 0,
    LBM_E_INVALID = -1,  /* argument out of range, NaN input, bad geometry        */
    LBM_E_NOMEM = -2,    /* arena too small, or a device list ran out of capacity */
    LBM_E_HIP = -3,      /* a HIP runtime call failed                             */
    LBM_E_DIVERGED = -4, /* non-finite or too fast particle state, or a fluid node
                            with non-finite moments or |u| > 0.3 (sentinel)      */
    LBM_E_STATE = -5     /* call not valid in the current state                   */
} lbm_status;

enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1, LBM_STORE_BF16 = 2 };
enum { LBM_BC_SBB = 0, LBM_BC_IBB = 1 };
enum { LBM_STEP_FLUID_ONLY = 0, LBM_STEP_COUPLED = 1 };
enum { LBM_MODE_FREE = 0, LBM_MODE_KINEMATIC = 1 };
enum { LBM_PERIODIC_X = 1, LBM_PERIODIC_Y = 2, LBM_PERIODIC_Z = 4 };

typedef struct {
    int32_t nx, ny, nz;   /* lattice size, each >= 3                              */
    uint32_t periodic;    /* LBM_PERIODIC_* bits; other faces are walls            */
    double tau;           /* BGK relaxation time, > 0.5                            */
    double rho0;          /* reference density, > 0                                */
    double g_fluid[3];    /* body acceleration of the fluid (Guo forcing, F = rho g) */
    double g_particle[3]; /* gravity on free particles, applied as (m - rho0 V) g  */
    int32_t storage;      /* LBM_STORE_*                                           */
    int32_t bc;           /* LBM_BC_SBB: halfway bounce-back; LBM_BC_IBB: paper's
                             interpolated bounce-back (Eqs. eqneq1-neqd)           */
    int32_t n_sub;        /* rigid-body sub-steps per lattice step, >= 1           */
    int32_t counter_force;/* 1: add to g_fluid minus the net weight of the free
                             particles spread over the fluid (periodic settling)   */
    double quad_h;        /* cell size of the body-property quadrature, > 0       */
    float fp16_scale;     /* FP16 storage multiplies deviations by this power of
                             two (0 selects 1024); ignored for FP32 and BF16       */
    int32_t link_c0;      /* 0: link fractions on the C = 1 surface that defines the
                             flags; 1: on the sphero-metaball's surface (sec. 2.3.2:
                             q solves f = c_0, c_0 depending on R_s): the level
                             c_0 = s^2 of the inner body (the body scaled by
                             s = 1 - contact_rs/sqrt(sum k) about its centroid,
                             weights s^2 k), which gives back a sphere's own radius;
                             needs contact_rs > 0.  Where that surface and C = 1
                             differ, q is 1 when the solid node lies outside it and
                             tends to 0 when the fluid node lies inside it        */
    /* contact (sec. 2.3.1): sphero-metaball of sphere radius contact_rs around
     * the body shrunk by 1 - contact_rs/sqrt(sum k); linear spring-dashpot with
     * stiffness contact_kn (0 disables contact), damping from the restitution
     * contact_en, tangential spring 2/7 contact_kn capped by contact_mu times
     * the normal force; recomputed every rigid-body sub-step.  Enabled contact
     * supports at most 1024 particles.                                       */
    double contact_rs, contact_kn, contact_en, contact_mu;
} lbm_config;

typedef struct {
    int32_t n_cp;         /* 1..20 control points                                  */
    int32_t mode;         /* LBM_MODE_FREE or LBM_MODE_KINEMATIC (moves with v, omega) */
    const double *cp_xyz; /* [n_cp][3] body frame                                  */
    const double *cp_k;   /* [n_cp] weights, > 0                                   */
    double x[3];          /* lab position of the body-frame origin                 */
    double quat[4];       /* body-to-lab rotation (w, x, y, z), normalised here    */
    double v[3];          /* initial velocity (lab)                                */
    double omega[3];      /* initial angular velocity (lab)                        */
    double density;       /* particle density (lattice units)                      */
} lbm_particle;

typedef struct {
    double x[3];          /* centroid (lab)                                        */
    double quat[4];       /* body-to-lab rotation                                  */
    double v[3], omega[3];/* velocity, angular velocity (lab)                      */
    double F[3], T[3];    /* hydrodynamic force and torque of the last step       */
    double mass, volume;
    double inertia[9];    /* body frame, about the centroid                       */
} lbm_particle_state;

/* Bytes of device arena needed for this configuration. */
lbm_status lbm_arena_bytes(const lbm_config *cfg, int32_t n_p, const lbm_particle *p, size_t *bytes);

/* Validates the configuration (tau > 0.5, sizes >= 3, 1..20 control points
 * with k > 0, finite inputs, each body's bounding sphere inside the walled
 * faces; overlapping bodies are not rejected, see the owner rule above),
 * computes body properties, uploads the state, flags the nodes, builds the
 * cut links and sets every fluid node to the collided rest state
 * f = feq(rho0, 0).  dev_arena must hold arena_bytes >= lbm_arena_bytes();
 * hip_stream is a hipStream_t (NULL = default stream). */
lbm_status lbm_init(const lbm_config *cfg, int32_t n_p, const lbm_particle *p, void *dev_arena,
                    size_t arena_bytes, void *hip_stream, lbm_ctx **out);

/* Metaball flagging (sec. 2.1): re-derives flags and owners of every node from
 * the current particle poses and rebuilds the cut-link list with its link
 * fractions.  Nodes uncovered by the change are remembered for refill().
 * n_solid and n_links are optional outputs (non-NULL makes the call sync). */
lbm_status metaball_flag(lbm_ctx *ctx, int64_t *n_solid, int64_t *n_links);

/* Advances n_steps steps.  LBM_STEP_COUPLED runs the full coupled step listed
 * at the top of this header; LBM_STEP_FLUID_ONLY keeps particles, flags and
 * links fixed (bounce-back and momentum exchange still use the particle
 * velocities).  Asynchronous on the context's stream. */
lbm_status lbm_step(lbm_ctx *ctx, int32_t n_steps, int32_t mode);

/* Hydrodynamic force and torque (about the centroid) on each particle from the
 * momentum exchange of the last step (sec. 2.3.2, MEM paragraph: per cut link
 * dP = (e_ib - u_w) f+_ib(x_f) - (e_i - u_w) f_i(x_f), both populations taken
 * relative to w_i rho0, and dT = (x_w - X) x dP with x_w = x_f - q e_i, summed
 * in a fixed order in FP64); F and T are [n_p][3] host arrays.  Synchronises. */
lbm_status particle_forces(lbm_ctx *ctx, double *F, double *T);

/* Local refilling (sec. 2.3.2) of the nodes uncovered by the last
 * metaball_flag() call: populations streaming in from fluid neighbours are
 * kept, a missing f_i takes f_opp(i) + 6 w_i rho0 e_i.u_new when its opposite
 * came from a fluid node and feq_i(rho0, u_new) otherwise, with u_new the
 * covering body's rigid velocity at the node; the node is then collided.
 * lbm_step in coupled mode does this internally every step.  n_refilled is
 * optional (non-NULL makes the call sync). */
lbm_status refill(lbm_ctx *ctx, int64_t *n_refilled);

/* ---- state access for tests and I/O (host FP64 arrays; all synchronise) ---- */
/* rho [N] and u [N][3] of the stored state (u excludes the half body force). */
lbm_status lbm_get_macros(lbm_ctx *ctx, double *rho, double *u);
/* Full post-collision populations f_i = w_i rho0 + deviation, [19][N]. */
lbm_status lbm_get_populations(lbm_ctx *ctx, double *f);
/* Sets the populations [19][N]; post_collision = 0 means f is a post-stream
 * state and fluid nodes are collided before storing. */
lbm_status lbm_set_populations(lbm_ctx *ctx, const double *f, int32_t post_collision);
/* owner [N]: -1 fluid, else the particle index. */
lbm_status lbm_get_flags(lbm_ctx *ctx, int32_t *owner);
/* Cut links of the current geometry in the library's order (particle-major):
 * node index, direction, owner and q.  Pass NULL arrays to get the count. */
lbm_status lbm_get_links(lbm_ctx *ctx, int64_t *n_links, uint32_t *node, int32_t *dir,
                         int32_t *owner, double *q);
lbm_status lbm_get_particles(lbm_ctx *ctx, lbm_particle_state *out /* [n_p] */);
/* Overwrites pose and velocities (x = centroid); call metaball_flag after. */
lbm_status lbm_set_particles(lbm_ctx *ctx, const lbm_particle_state *in /* [n_p] */);
/* Effective fluid body acceleration (includes the counter-force). */
lbm_status lbm_get_gfluid(lbm_ctx *ctx, double *g3);

/* ---- measurement ---- */
/* on > 0: the stream-collide kernel of every on-th step (the step count
 * since lbm_init a multiple of on; up to 4096 timed launches between reads)
 * is bracketed by HIP events on the context's stream (events on a launch add
 * a few microseconds to its step, so a stride above 1 keeps the steps
 * between timed ones free of them); on <= 0: off.  lbm_timing_read returns
 * the summed elapsed milliseconds and the count of timed launches since the
 * last read, and the number of nodes that kernel updated in the last step
 * (all nodes but solid, boundary and uncovered ones); it synchronises. */
lbm_status lbm_timing_enable(lbm_ctx *ctx, int32_t on);
lbm_status lbm_timing_read(lbm_ctx *ctx, double *ms, int64_t *launches, int64_t *nodes_per_launch);
/* Link fractions solved and Newton/bisection iterations spent on them since
 * the last call (resets the counts; synchronises). */
lbm_status lbm_nr_stats(lbm_ctx *ctx, int64_t *links, int64_t *iterations);
/* Contacts resolved (body pairs and walls, counted per rigid-body sub-step)
 * and contact iterations that did not converge, since lbm_init
 * (synchronises). */
lbm_status lbm_contact_stats(lbm_ctx *ctx, int64_t *contacts, int64_t *failures);
/* Stationary-point solves of candidate body pairs (bounding spheres
 * overlapping, per rigid-body sub-step) and their Newton evaluations since
 * the last call (resets the counts; synchronises). */
lbm_status lbm_contact_nr_stats(lbm_ctx *ctx, int64_t *solves, int64_t *iterations);
/* Waits for the context's stream and reports device-side errors. */
lbm_status lbm_sync(lbm_ctx *ctx);

/* ---- checkpoint / resume (not part of the paper's method: I/O around it) ----
 * lbm_save writes the context's whole state to the file at path: the
 * populations in their storage type (both buffers), flags and owners, skip
 * masks, cut links with their fractions, the FP64 particle records
 * (pose, velocities, loads, control points, region history), contact
 * springs, the step counter and the kernel constants.  A pending refill is
 * applied first.  Synchronises.  lbm_load replaces the state of ctx, which
 * must have been set up by lbm_init with the same configuration and the same
 * number of particles of the same sizes (the arena layout must match), with
 * the file's; the steps after it are bitwise those that would have followed
 * the save.  The warm-start network (lbm_set_warmstart) and the timing state
 * are not part of the file.  Errors: LBM_E_INVALID (NULL argument, file
 * cannot be opened, read or written, not a checkpoint), LBM_E_STATE (written
 * by a context of another configuration; ctx is unchanged), LBM_E_HIP. */
lbm_status lbm_save(lbm_ctx *ctx, const char *path);
lbm_status lbm_load(lbm_ctx *ctx, const char *path);

/* ---- measurement aid: streaming-copy ceiling ----
 * Times a plain copy with the stream-collide's access shape: the 19
 * populations of n nodes (elem_bytes 4 or 2) in the library's population
 * layout (runs of 1024 nodes, each run holding its 19 populations one after
 * another; stride = the padded node count, a multiple of 1024) are read from
 * dev_src and written to dev_dst with non-temporal stores, one node per lane.
 * One warm-up launch, then reps launches bracketed by HIP events on
 * hip_stream; *ms receives the mean duration of one launch, which moves
 * 2 * 19 * n * elem_bytes bytes.  Both buffers are caller-owned device memory
 * of at least 19 * stride elements (dev_dst is overwritten).  Synchronises.
 * Errors: LBM_E_INVALID (NULL pointer, n <= 0, stride < n or not a multiple
 * of 1024, reps < 1, other element size), LBM_E_HIP.  lbm_last_error() is not
 * set by this call. */
lbm_status lbm_copy_probe(const void *dev_src, void *dev_dst, int64_t n, int64_t stride, int32_t elem_bytes,
                          int32_t reps, void *hip_stream, double *ms);

void lbm_destroy(lbm_ctx *ctx);
const char *lbm_last_error(void);

/* ---- warm start of the link fractions (an extension beyond the paper: an
 * MLP trained on the method's own Newton solutions) ----
 * The link fraction q of a cut link is the first root of C(x_f - s e_i) = 1
 * on (0,1] (sec. 2.3.2), bracketed by eight samples and found by a
 * safeguarded Newton iteration.  A small MLP (87 inputs -> 64 -> 64 -> 4,
 * tanh hidden layers, linear output; FP16 weights and activations with FP32
 * sums) can supply the starting point.  Inputs of a link: the fluid node
 * relative to the centroid and the direction e_i, both in the body frame, the
 * node scaled by 1/sqrt(sum k); a task bit (0: link fraction); the body's
 * control points in the body frame sorted by weight (largest first), each
 * (p/sqrt(sum k), k/sum k), zero-padded to 20.  Output 0 is the q guess
 * (outputs 1..3 belong to a closest-point task, trained only when its bit
 * is set).  The guess is used only when it lies inside the bracket, and a
 * warm-started iteration not converged within 30 evaluations is redone from
 * the plain start, so the root found is the plain one (within the Newton
 * tolerance): the residual C - 1 judges the guess.
 *
 * Parameters: P = mlp_param_count() = 10052 FP32 values in the order
 * W1 [87][64], b1 [64], W2 [64][64], b2 [64], W3 [64][4], b3 [4] (a layer
 * computes z = h W + b).  A weights blob is caller-owned device memory of
 * mlp_weights_bytes() bytes, 256-byte aligned: FP32 parameters, Adam
 * moments and step count, the FP16 copy, and the training workspace. */
size_t mlp_weights_bytes(void);
int32_t mlp_param_count(void);
/* Loads the FP32 parameters (host [P]) and resets the Adam state; syncs. */
lbm_status mlp_init(void *dev_weights, const float *params, void *hip_stream);
/* Copies the FP32 parameters to the host [P]; synchronises the stream. */
lbm_status mlp_get_params(const void *dev_weights, float *params, void *hip_stream);
/* Training samples from the context's current cut links: features
 * dev_feat [n][87] FP16 and targets dev_target [n][4] FP32 (q, 0, 0, 0),
 * n = min(n_max, links); synchronises. */
lbm_status mlp_collect(lbm_ctx *ctx, int64_t n_max, void *dev_feat, void *dev_target, int64_t *n_out);
/* Closest-point samples (task bit 1) from the last contact sub-step: one per
 * candidate pair i < j whose stationary-point iteration converged, in pair
 * order, seen from body i -- the query point is body j's centroid, the
 * direction 0 -- with targets (0, p) where p = the stationary point relative
 * to body i's centroid in its frame, scaled by 1/sqrt(sum k) (outputs 1..3);
 * n = min(n_max, such pairs); none without contact.  With a warm start set
 * (lbm_set_warmstart), the same network's outputs 1..3 start each pair's
 * iteration, kept only if it converges within 20 evaluations to a point
 * between the two centroids, outside both inner bodies, with positive
 * curvature along the centroid segment (else the plain start follows).
 * Synchronises. */
lbm_status mlp_collect_contact(lbm_ctx *ctx, int64_t n_max, void *dev_feat, void *dev_target, int64_t *n_out);
/* Outputs [n][4] FP32 of the network for features [n][87]: precision 0 =
 * FP16 features/weights/activations (the production form), 1 = FP32
 * throughout (a test instantiation; features are then FP32), 2 = FP16 with
 * the hidden layers as matrix-core (MFMA) tiles of 32 samples, the form the
 * warm-started solvers use.  Enqueued on the stream; uses the blob's
 * workspace. */
lbm_status mlp_forward(void *dev_weights, const void *dev_feat, int64_t n, int32_t precision, float *dev_out,
                       void *hip_stream);
/* Gradient (host [P], FP32) and loss of one batch of n <= 4096 samples:
 * loss = (1/n) sum over samples of the squared errors of the targeted
 * outputs (output 0 when the task bit is 0, outputs 1..3 otherwise);
 * synchronises. */
lbm_status mlp_grad(void *dev_weights, const void *dev_feat, const void *dev_target, int64_t n,
                    int32_t precision, float *grad, double *loss, void *hip_stream);
/* Adam over sequential minibatches of the n samples (in the order given),
 * for the epochs given.  hparams_json: a flat object with any of "lr"
 * (1e-3), "epochs" (1), "batch" (256, at most 4096), "beta1" (0.9), "beta2"
 * (0.999), "eps" (1e-8), "precision" (0).  The step count persists in the
 * blob across calls.  Synchronises. */
lbm_status mlp_train(void *dev_feat, void *dev_target, int64_t n, const char *hparams_json, void *dev_weights,
                     void *hip_stream);
/* Warm-starts the link fractions of the context with the blob's FP16
 * weights from now on (the blob must stay alive); NULL: plain Newton. */
lbm_status lbm_set_warmstart(lbm_ctx *ctx, const void *dev_weights);
/* Histogram of Newton evaluations per solved link since the last call
 * (hist[65], last bin: 64 or more) and the largest |C - 1| at a link's last
 * evaluation; resets both; synchronises. */
lbm_status lbm_nr_histogram(lbm_ctx *ctx, int64_t *hist, double *resid_max);

/* ---- ensemble of independent systems ----
 * n_cases systems (each as lbm_init would set it up: configs cfgs[i],
 * particles parts[n_p[0] + ... + n_p[i-1] ...] concatenated) stepped
 * together: the stream-collide of all systems runs as one launch over a table
 * of equal tiles (a wave covers a tile of 64x1, 32x2 or 16x4 nodes, or 64
 * consecutive nodes in lattice order, chosen per system by lbm_autotune), each kind of boundary kernel runs as one
 * launch for all systems (a block finds its system in a block table) on a
 * second stream owned by the batch, and six consecutive coupled steps (the
 * period of the library's buffer rotation) are captured once into a HIP
 * graph and replayed.  Every system computes exactly what lbm_step computes
 * for it alone (same kernel code, same per-system order; a warm-started
 * system, lbm_set_warmstart on its context, keeps its network).  The launch
 * tables are rewritten, and the graph captured again, whenever a system's
 * buffers, constants or warm start changed from outside.  All systems must use
 * one storage type.  The arena layout is the library's: one 256-byte-aligned
 * device block of lbm_batch_arena_bytes bytes, owned by the caller.
 * Errors: LBM_E_INVALID for a bad case (the message names it), LBM_E_NOMEM
 * for a short arena, LBM_E_HIP for runtime failures. */
lbm_status lbm_batch_arena_bytes(int32_t n_cases, const lbm_config *cfgs, const int32_t *n_p,
                                 const lbm_particle *parts, size_t *bytes);
lbm_status lbm_batch_init(int32_t n_cases, const lbm_config *cfgs, const int32_t *n_p,
                          const lbm_particle *parts, void *dev_arena, size_t arena_bytes,
                          void *hip_stream, lbm_batch **out);
/* n_steps coupled steps of every system, enqueued after the caller's stream's
 * earlier work; the caller's stream waits for them.  use_graph = 1 replays
 * the captured graph for each whole block of six steps (captured on first
 * use and again whenever a system's buffers were rotated from outside, e.g.
 * by lbm_step on its context); the rest runs as plain launches. */
lbm_status lbm_batch_step(lbm_batch *b, int32_t n_steps, int32_t use_graph);
/* Context of system i, for the getters and setters above; owned by the batch
 * (do not destroy it). */
lbm_status lbm_batch_case(lbm_batch *b, int32_t i, lbm_ctx **ctx);
/* Chooses each system's wave tile (one launch per candidate, timed with HIP
 * events) and the waves per block of the batched launch (4 or 8), within
 * about budget_ms of host time (systems not reached keep 64x1).  Systems of
 * equal sizes, storage and periodicity share one choice.  With a cache path,
 * a complete cache file is read instead of measuring, and the choices are
 * written to it otherwise (a small JSON object).  Synchronises; the results
 * of the next step are unchanged by the tiles (only the launch shape is). */
lbm_status lbm_autotune(lbm_batch *b, double budget_ms, const char *cache_path /* nullable */);
/* Current choices: tw_log2[i] = log2 of the tile width of system i (6, 5 or
 * 4; 7: 64 consecutive nodes in lattice order), and the waves per block. */
lbm_status lbm_batch_tiles(lbm_batch *b, int32_t *tw_log2 /* [n_cases] */, int32_t *waves_per_block);
void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* MIDELBM_H */
