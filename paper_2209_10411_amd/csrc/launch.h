// Interface between the host-side C ABI (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mdl {

enum Phase {
    PHASE_LINKS = 0,       // bounce-back values + momentum exchange, force reduction, rigid body
    PHASE_FLAGS = 1,       // region flags (when move), node classes, optionally the boundary/uncovered update
    PHASE_BULK = 2,        // stream-collide of plain fluid nodes
    PHASE_SPECIAL = 3,     // boundary and uncovered nodes
    PHASE_LINKBUILD = 4,   // cut links and q of the new geometry
    PHASE_INIT_STATE = 5,     // collided rest state
    PHASE_COLLIDE_STORED = 6  // collide the stored populations of fluid nodes in place
};

struct StepArgs {
    Params p;
    int phase;
    int move;      // PHASE_LINKS: update particles; PHASE_FLAGS: re-flag
    int in_place;  // PHASE_SPECIAL: refill in place
    int do_special;  // PHASE_FLAGS: also update the boundary and uncovered nodes into B
    hipStream_t stream;
    void *A, *B;
    int32_t *own_old, *own_new;
    int32_t *own_dead;  // PHASE_FLAGS: flag buffer to reset to FLUID on the classification balls, or NULL
    uint8_t *skip;       // PHASE_BULK: skip mask of this step
    uint8_t *skip_next;  // PHASE_FLAGS: skip mask of the next step
    DevParticle *P;
    RegionMap rm;
    const int *part_first_blk;
    int *blk_cnt, *l_off;
    int *body_stats;  // [np][4] per body: cut links, solid, uncovered, special nodes of the classification
    uint32_t *lmask;  // per region thread: cut-link mask of the new flags
    uint32_t *l_node, *l_do;
    double *l_q, *part;
    uint32_t *special;
    Counters *cnt;
    ContactBufs cb;
    NrStats nrs;            // link-fraction solver statistics (per-block slots)
    const _Float16 *warm;   // warm-start MLP parameters (FP16), or NULL: plain Newton
    const float *mlp_body;  // [np][80] constant MLP inputs of each body
    hipEvent_t ev_start, ev_stop;  // PHASE_BULK / PHASE_SPECIAL: events recorded with the dispatch, or NULL
    int bulk_blocks;  // PHASE_BULK: stream-collide blocks allowed per CU (LDS reservation), 0: the default
};

void launch_phase(const StepArgs &a);
void launch_fill_i32(int32_t *a, long long n, int32_t v, hipStream_t s);
void launch_fill_u8(uint8_t *a, long long n, uint8_t v, hipStream_t s);
void launch_reset_counters(Counters *cnt, hipStream_t s);
// Re-flag: every node solid in own_old and fluid in own_new, listed for the
// in-place refill and counted per body.
void launch_uncovered(const Params &p, const int32_t *own_old, const int32_t *own_new, uint32_t *special,
                      Counters *cnt, int *body_stats, hipStream_t s);
// Batched stream-collide of an ensemble (bw: waves per block, 4 or 8).
void launch_bulk_batch(int storage, int bw, const BulkCase *cases, const int *blk_case, int nblocks, int parity,
                       hipStream_t s);
// fresh: the flag buffers hold flags of the current pose only (after a re-flag)
void launch_refresh_pose(const Params &p, DevParticle *P, int fresh, hipStream_t s);

// Batched boundary kernels of an ensemble: one launch of a kind for every
// system (cs: the systems' argument blocks, map: block -> system).
enum BatchOp { OP_LINKS, OP_REDUCE, OP_RIGID, OP_MARK, OP_CLASSIFY, OP_EMIT, OP_LINKQ, OP_LINKQ_WARM };
void launch_case_batch(int storage, BatchOp op, const CaseArgs *cs, const int *map, int nblocks, hipStream_t s);
// Launch sizes of the one-system boundary kernels (also the block ranges of
// a system in the batched launches).
int link_grid(const Params &p);
int link_q_grid(const Params &p);

}  // namespace mdl
