/*
 * hs.h -- Hierarchy-Scan on AMD Instinct MI355X (gfx950): C ABI.
 *
 * The library computes, for batches of skeletal characters, the three
 * per-frame steps of GPU skeletal animation (Sec. 1 of the paper):
 *   1. Simulation     -- sample and blend animation clips into local poses
 *                        (hs_pose_sample, or fused into hs_scan_forward);
 *   2. Hierarchy-Scan -- the tree prefix product of Eq. 1 (Sec. 3): every
 *                        joint's model-space transform is its parent's
 *                        transform times its own local transform,
 *                        G_j = G_parent(j) * L_j (hs_scan_forward);
 *   3. Bind MeshPose  -- skin matrices S_j = G_j * B_j^-1 (hs_skin, or fused
 *                        into hs_scan_forward);
 * plus the adjoint of step 2 (hs_scan_backward) for gradient-based use.
 *
 * Conventions
 *   - Matrices act on column vectors.  Outputs are 4x4 row-major fp32; the
 *     bottom row of every global matrix is written as exactly (0, 0, 0, 1).
 *   - A joint's local transform is L = T(t) * R(q) * diag(s) with the unit
 *     quaternion q = (x, y, z, w) turned into a rotation by the textbook
 *     polynomial (no renormalisation); s may be omitted (unit scale).
 *   - A batch is CSR: joint_offsets[C+1] (offsets[0] = 0, non-decreasing,
 *     offsets[C] = N) and parents[N], character-local indices, -1 for a
 *     root, each parent preceding its child (parents[j] < j), the ordering
 *     the paper obtains from a tree traversal (Sec. 3.2.1).  Several roots
 *     per character (a forest) and empty characters are allowed.
 *
 * Memory and streams
 *   - Every array argument of the per-frame calls is a caller-owned device
 *     pointer.  The library allocates only inside hs_context_create and
 *     hs_plan_create (and frees in the matching destroy call); the per-frame
 *     calls neither allocate nor synchronise, run asynchronously on the
 *     given stream, and may be captured into a HIP graph.
 *   - Outputs must not overlap inputs or each other.
 *   - A plan owns device workspaces (multipass tables, the status word, the
 *     chain path's publication records and its call counter): calls on one
 *     plan run in the order of their streams; calls on one plan that may
 *     run at the same time (unordered streams) race.
 *   - Arrays read or written as 16-byte vectors (quat, global_out, inv_bind,
 *     skin_out, grad_global, grad_quat, ckpt) must be 16-byte aligned; the
 *     others 4-byte aligned.
 *
 * Errors
 *   Every call returns an hs_status.  Argument, alignment, aliasing and
 *   topology errors are detected on the host before anything is launched;
 *   a failed launch returns HS_ERR_DEVICE.  What goes wrong inside a kernel
 *   is recorded in the plan's device status word, which hs_plan_status
 *   reads after synchronising (HS_ERR_DEVICE if any bit is set).
 *   hs_last_error() returns a thread-local description of the last failure
 *   on the calling thread.  NaN and Inf inputs are not errors: they
 *   propagate into the outputs.
 */
#ifndef HS_H_
#define HS_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hs_status;
#define HS_OK 0
#define HS_ERR_INVALID_ARG 1
#define HS_ERR_TOPOLOGY 2
#define HS_ERR_UNSUPPORTED 3
#define HS_ERR_DEVICE 4
#define HS_ERR_OOM 5

typedef struct hs_context hs_context;
typedef struct hs_plan hs_plan;
typedef struct hs_graph hs_graph;

/* Library version string (static storage). */
const char *hs_version(void);

/* Description of the last failure on this thread; valid until the next
 * failing call on the same thread.  Never NULL. */
const char *hs_last_error(void);

/* Create a context bound to HIP device `device`.  The context owns the
 * device properties and the autotuning cache (in memory; see
 * hs_context_load_tuning for the file form).  *out receives the
 * context; destroy it with hs_context_destroy after every plan made from it
 * has been destroyed. */
hs_status hs_context_create(int device, hs_context **out);
void hs_context_destroy(hs_context *ctx);

/* The autotuner's results on disk, as JSON: one entry per tuning key (the
 * device's gfx architecture, the size class of the batch -- log2 of its
 * joints and characters, its largest character, its longest chain of
 * 64-joint blocks -- instancing, strategy and schedule options) holding
 * the chosen launch shape:
 *   {"version": 1, "entries": {"<key>": {"tile_cap": 2048, "waves": 16,
 *    "grid_per_cu": 0, "chain_units": 0, "queue_waves": 4}, ...}}
 * hs_context_load_tuning merges a file's entries into the context's cache
 * (a missing file is HS_OK with nothing loaded; a malformed one is
 * HS_ERR_INVALID_ARG with the cache unchanged); plans created with
 * autotune then take a cached shape without timing candidates.
 * hs_context_save_tuning writes the context's whole cache (to a temporary
 * file renamed into place).  If the environment variable HS_TUNE_CACHE
 * names a file, hs_context_create loads it and every plan that tunes saves
 * the cache there.  Host calls; they touch no device memory. */
hs_status hs_context_load_tuning(hs_context *ctx, const char *path);
hs_status hs_context_save_tuning(const hs_context *ctx, const char *path);

/* ------------------------------------------------------------------------
 * Plans: topology analysis, done once per skeleton batch.
 * ------------------------------------------------------------------------ */

/* A batch of characters.  joint_offsets and parents may be host or device
 * pointers; hs_plan_create copies what it needs (a device pointer costs one
 * synchronous device-to-host copy) and keeps no reference to them. */
typedef struct hs_batch {
    int64_t num_characters;       /* C >= 0 */
    int64_t num_joints;           /* N = joint_offsets[C], 0 <= N < 2^31 */
    const int64_t *joint_offsets; /* [C+1] */
    const int32_t *parents;       /* [N] character-local, -1 = root, parents[j] < j */
} hs_batch;

/* Scan strategy. */
#define HS_STRATEGY_AUTO 0      /* tiles where a character fits, multipass beyond */
#define HS_STRATEGY_TILE 1      /* every character in an LDS tile (error if one does not fit) */
#define HS_STRATEGY_MULTIPASS 2 /* every character on the global multipass path */

typedef struct hs_plan_opts {
    int32_t strategy;       /* HS_STRATEGY_* */
    int32_t tile_joints;    /* tile capacity in joints (multiple of 64), 0 = choose */
    int32_t waves_per_tile; /* 64-lane waves per workgroup (1..16), 0 = choose */
    int32_t grid_tiles;     /* workgroups launched: 0 = one per tile; k > 0 = k per CU, each
                               looping over the cost-sorted tiles */
    int32_t autotune;       /* non-zero: time candidate launch shapes on the device when the
                               plan is created (result cached in the context) */
    int32_t chain_units;    /* non-zero: scan runs of up to four 64-joint blocks that consist of
                               whole chain segments with four joints per lane (a sequential
                               product per lane and a segmented scan across the wave) */
    int32_t algorithm;      /* HS_ALG_*: the scan that tiles run (forward, stored TRS poses) */
    int32_t adjoint;        /* HS_ADJ_*: the kernel that runs the adjoint of characters of up to
                               1024 joints */
    int32_t schedule;       /* HS_SCHED_*: how hs_scan_forward launches the tiles */
    int32_t adjoint_blocks_per_wave; /* HS_ADJ_ANCHORS: 64-joint blocks that each wave of the
                               two-level adjoint takes (1 or 2); 0 = choose: 2 when it lets
                               the batch's adjoint tiles run in fewer rounds of resident
                               workgroups, else 1 */
} hs_plan_opts;

/* Forward schedules (hs_scan_forward; the other tiled calls keep the size
 * classes).  HS_SCHED_QUEUE: every tile of the plan in one launch over the
 * plan's heaviest-first tile list: one workgroup per tile (grid_tiles 0,
 * the hardware dispatching them as CUs free up), or at most grid_tiles
 * resident workgroups per CU, each walking the list with a static stride;
 * LDS holds only the transforms of each tile's anchors (joints whose
 * children lie in another 64-joint block) and one staging slice per wave,
 * so large tiles do not cost occupancy.  Without tile_joints the queue's
 * tiles hold the largest character, at least 256 joints.  HS_SCHED_CLASSES:
 * one launch per size class (characters of up to 1024 joints, up to 1664,
 * the rest) with all of a tile's transforms in LDS.  HS_SCHED_AUTO takes the
 * queue where it applies (the library's scan, no chain units, not
 * instanced, a tile strategy, and each tile's anchors within the LDS) and
 * the classes elsewhere; HS_SCHED_QUEUE where it does not apply is
 * HS_ERR_UNSUPPORTED. */
#define HS_SCHED_AUTO 0
#define HS_SCHED_QUEUE 1
#define HS_SCHED_CLASSES 2

/* Adjoint kernels for characters of up to 1024 joints in recompute mode
 * (hs_scan_backward without checkpoints, hs_effector_backward,
 * hs_effector_step; larger characters always take the dataflow kernel up to
 * 1664 joints, then the multipass adjoint).  HS_ADJ_ROUNDS: tile-wide
 * synchronous reverse pointer-jumping rounds, one joint per thread,
 * workgroup barriers between rounds; recomputes every G_j on chip.
 * HS_ADJ_DATAFLOW: wave-level rounds per 64-joint block, blocks ordered by
 * LDS flags (no workgroup barriers between rounds).  HS_ADJ_ANCHORS: two
 * levels: every joint's seed goes straight to the nearest out-of-block
 * ancestor of its block path, those anchors pass their totals on to theirs
 * in decreasing order, then one wave-level reverse pointer jumping per
 * block over the seeds and the anchors' inflows (tiles whose anchors do not
 * fit the LDS fall back to HS_ADJ_ROUNDS).  HS_ADJ_AUTO resolves per call:
 * HS_ADJ_ANCHORS for end-effector seeds, HS_ADJ_ROUNDS for a dense
 * dLoss/dG (measured fastest for each: on a dense seed every joint of a
 * chain block sends to one anchor).  Given checkpoints, characters of up
 * to 1664 joints always run the dataflow kernel, which rebuilds each G_j
 * from them. */
#define HS_ADJ_AUTO 0
#define HS_ADJ_ROUNDS 1
#define HS_ADJ_DATAFLOW 2
#define HS_ADJ_ANCHORS 3

/* Tile algorithms.  HS_ALG_SCAN is this library's scan (wave-level pointer
 * jumping per 64-joint block, dataflow between blocks).  HS_ALG_WALK ..
 * HS_ALG_COMPRESSED are the paper's Algorithms 1-4 (per-joint walk to the
 * root, Sec. 2; barrier-synchronous pointer jumping, Sec. 3.1, Eq. 2;
 * 64-joint blocks with a walk over out-of-block partials, Sec. 3.2.1; the
 * 8-joint window and hops of 8, Sec. 3.2.2), one joint per thread on tiles
 * of at most 1024 joints, kept for comparison on this hardware.  They need
 * HS_POSE_TRS sources (HS_ERR_UNSUPPORTED otherwise) and no chain units;
 * characters larger than 1024 joints take the multipass path. */
#define HS_ALG_SCAN 0
#define HS_ALG_WALK 1
#define HS_ALG_JUMP 2
#define HS_ALG_BLOCKS 3
#define HS_ALG_COMPRESSED 4

typedef struct hs_plan_info {
    int64_t num_characters;
    int64_t num_joints;
    int64_t tiled_joints;      /* joints scanned in LDS tiles */
    int64_t multipass_joints;  /* joints on the multipass path */
    int32_t max_depth;         /* levels on the longest root-to-leaf path (root = 1) */
    int32_t max_character;     /* largest character, in joints */
    int32_t num_tiles;
    int32_t tile_joints;
    int32_t waves_per_tile;
    int32_t grid;              /* workgroups per tiled launch */
    int32_t multipass_rounds;  /* global jump rounds of the multipass path */
    int32_t max_block_chain;   /* longest chain of 64-joint blocks on any path */
    int32_t schedule;          /* HS_SCHED_QUEUE or HS_SCHED_CLASSES: the forward's launches */
    int32_t max_anchors;       /* queue: most anchors of one tile (LDS slots), else 0 */
    int32_t adjoint_blocks_per_wave; /* two-level adjoint of hs_effector_step: 64-joint blocks
                                  per wave (0: the plan has no such tiles) */
    int64_t chain_joints;      /* multipass joints of chain characters (every parent the previous
                                  joint), scanned in one pass over their poses */
} hs_plan_info;

/* Analyse a batch: validates the CSR topology (HS_ERR_TOPOLOGY if some
 * parents[j] is outside [-1, j)), packs whole characters into LDS tiles,
 * prepares the multipass path for characters larger than a tile, uploads
 * the device tables and, if asked, autotunes the launch shape.  opts may be
 * NULL.  Synchronises the device. */
hs_status hs_plan_create(hs_context *ctx, const hs_batch *batch, const hs_plan_opts *opts,
                         hs_plan **out);

/* Skeletons shared by many characters.  In the paper's pipeline (Sec. 1:
 * Simulation, Hierarchy-Scan, Bind MeshPose) characters of one kind share
 * the joint hierarchy and the bind pose; only the local poses differ.
 * Host arrays: skeleton k owns joints offsets[k] .. offsets[k+1]-1 of the
 * skeleton arrays (offsets[0] = 0, offsets[num_skeletons] = num_joints);
 * parents[] are skeleton-local as in hs_batch. */
typedef struct hs_skeleton_set {
    int32_t num_skeletons;
    int64_t num_joints;         /* joints over all skeletons */
    const int64_t *offsets;     /* host [num_skeletons + 1] */
    const int32_t *parents;     /* host [num_joints] */
} hs_skeleton_set;

/* A plan for num_characters instances: character c is a copy of skeleton
 * skeleton_id[c] (host array), so its joints are numbered as in hs_batch
 * with the skeleton's size.  The forward tiles read each joint's parent and
 * inverse bind through its skeleton (arrays small enough to stay in the
 * caches) instead of per-joint rows in HBM: hs_scan_forward's inv_bind is
 * then [skel->num_joints, 4, 4], one row per skeleton joint.  Everything
 * else (pose arrays, outputs, hs_pose_sample, hs_scan_backward) is per
 * joint as for hs_plan_create.  Chain units, the paper's algorithms and
 * the multipass strategy are not available (HS_ERR_UNSUPPORTED), and every
 * character must fit a tile (HS_ERR_UNSUPPORTED otherwise).  Errors:
 * HS_ERR_INVALID_ARG for bad offsets or a skeleton_id out of range,
 * HS_ERR_TOPOLOGY as hs_plan_create. */
hs_status hs_plan_create_instanced(hs_context *ctx, const hs_skeleton_set *skel, int32_t num_characters,
                                   const int32_t *skeleton_id, const hs_plan_opts *opts, hs_plan **out);
void hs_plan_destroy(hs_plan *plan);
hs_status hs_plan_get_info(const hs_plan *plan, hs_plan_info *out);

/* ------------------------------------------------------------------------
 * Device status.  The scan relies on the ordering the paper obtains from a
 * tree traversal (Sec. 3.2.1): every parent precedes its children, so a
 * block of the tile only ever waits for earlier blocks.  The plan checks
 * this on the host at creation; on the device two things are recorded in a
 * status word the plan owns (one per plan, shared by all its calls):
 *   HS_DEV_WAIT_TIMEOUT  a kernel's bounded wait for an earlier block gave
 *                        up (the ordering was broken, or the plan's wait
 *                        limit was lowered); the kernel went on with
 *                        whatever it held, so outputs since are unreliable;
 *   HS_DEV_TOPOLOGY      a call with HS_FLAG_VALIDATE found the plan's
 *                        device tables breaking the ordering: some joint's
 *                        parent outside [-1, j) of its character, or its
 *                        level not its parent's plus one.  That call's
 *                        kernels then do nothing (outputs unwritten).
 * ------------------------------------------------------------------------ */
#define HS_DEV_WAIT_TIMEOUT 1u
#define HS_DEV_TOPOLOGY 2u

/* Flag of hs_scan_forward and hs_scan_backward: re-check the plan's device
 * topology tables (one extra pass over parents and levels, on the call's
 * stream, ahead of the scan) into the status word. */
#define HS_FLAG_VALIDATE 1u

/* Synchronise the plan's device, then read its status word: *bits (if
 * non-NULL) receives the HS_DEV_* bits, *joint (if non-NULL) the lowest
 * global joint id that failed the topology check, or -1.  clear != 0 resets
 * the word.  Returns HS_OK when no bit is set, HS_ERR_DEVICE with a
 * description (hs_last_error) otherwise. */
hs_status hs_plan_status(const hs_plan *plan, uint32_t *bits, int64_t *joint, int32_t clear);

/* The number of polls after which a kernel's bounded wait gives up and
 * records HS_DEV_WAIT_TIMEOUT (default 4194304, far beyond any wait the
 * ordering allows).  For tests of the error path: with 0 every wait that
 * is needed at all gives up at once.  Every kernel still runs to its end.
 * Takes effect for calls made after it. */
hs_status hs_plan_set_wait_limit(hs_plan *plan, int32_t polls);

/* For tests of HS_FLAG_VALIDATE: overwrites joint's entry of the plan's
 * device parent table with the joint itself (a parent that does not
 * precede its child), as a stray device write might.  Synchronous.  Only
 * calls with HS_FLAG_VALIDATE should follow: they detect it and launch no
 * scan work; destroy the plan afterwards. */
hs_status hs_plan_debug_break_parent(hs_plan *plan, int64_t joint);

/* ------------------------------------------------------------------------
 * Simulation step (Sec. 1, step 1): looping clips, sampled and blended.
 * ------------------------------------------------------------------------ */

/* A library of clips, each num_keys keyframes at fps, every keyframe a pose
 * of joints_per_clip joints.  key_quat [clips][keys][J][4] (16-byte
 * aligned), key_trans [clips][keys][J][3].  Joint j of a character samples
 * joint j of the clip, so every character must have <= J joints. */
typedef struct hs_clip_lib {
    int32_t num_clips;
    int32_t num_keys;
    int32_t joints_per_clip;
    float fps;
    const float *key_quat;
    const float *key_trans;
} hs_clip_lib;

/* Per-character choices, each [C]: clip ids in [0, num_clips), time in
 * seconds (clips loop with period num_keys / fps), blend weight of clip b. */
typedef struct hs_clip_params {
    const int32_t *clip_a;
    const int32_t *clip_b;
    const float *time;
    const float *weight;
} hs_clip_params;

/* For each character: frame f = fps * time (one fp32 multiply), keys
 * k0 = floor(f) mod K and k1 = (k0 + 1) mod K, alpha = f - floor(f).  For
 * each clip, q = normalise((1 - alpha) q_k0 + alpha * sign * q_k1) where
 * sign is that of the dot product of the two keys (+1 when it is zero,
 * decided in fp64 from the exact fp32 products), t = (1 - alpha) t_k0 +
 * alpha t_k1.  The two clips are then blended the same way with the weight
 * (the sign decided on the fp32 clip quaternions).  Writes quat_out [N,4]
 * (16-byte aligned) and trans_out [N,3]; the scale is implicitly 1. */
hs_status hs_pose_sample(const hs_plan *plan, const hs_clip_lib *lib, const hs_clip_params *params,
                         float *quat_out, float *trans_out, hipStream_t stream);

/* Measurement reference, not part of the method: moves the bytes of a
 * forward scan of n joints and no arithmetic.  Reads quat [n,4] (16-byte
 * aligned), trans [n,3], scale [n,3] and table [n] (any 4-byte values, as
 * the scan reads one parent or code per joint) once each with streaming
 * loads, one joint per lane, and writes out [n,4,4] (16-byte aligned) as
 * the scan writes G: coalesced 16-byte rows through a per-wave LDS slice.
 * The rows hold the inputs (row 0: q.x q.y q.z t.x; row 1: q.w s.x s.y
 * t.y; row 2: s.z table-bits 0 t.z; row 3: 0 0 0 1).  Its speed is the
 * HBM rate this access pattern can reach on the device.  Asynchronous on
 * stream; allocates nothing; out must not overlap the inputs. */
hs_status hs_stream_probe(int64_t n, const float *quat, const float *trans, const float *scale,
                          const int32_t *table, float *out, hipStream_t stream);

/* Reverse mode of hs_pose_sample: given dLoss/dquat [N,4] (raw components,
 * 16-byte aligned) and dLoss/dtrans [N,3] of the sampled local poses,
 * writes dLoss/dkey_quat [num_clips, num_keys, joints_per_clip, 4] and
 * dLoss/dkey_trans [..., 3] (each the sum over every character and joint
 * that reads the key, summed per key row in a fixed order), dLoss/dtime [C]
 * and dLoss/dweight [C].  The
 * arc signs and the key index floor(f) are held fixed (the derivative away
 * from their switching points); d alpha / d time = fps.  Any output may be
 * NULL (not computed).  A character with an invalid clip id or a
 * non-finite time gets NaN time and weight gradients and adds nothing to
 * the keys.  workspace: NULL, or caller-owned device memory of 32 bytes per
 * joint ([N,2,4] fp32, 16-byte aligned, not overlapping any other array):
 * with it each joint's reverse step runs once (storing the adjoints of its
 * two clips' unnormalised key blends there) and the key gradients are
 * gathered from it; without it the gather recomputes each reader's reverse
 * step.  The results agree up to rounding (each route is bitwise
 * reproducible on its own).  Calls that
 * share a workspace must not overlap.  Asynchronous on stream; allocates
 * nothing. */
hs_status hs_pose_sample_backward(const hs_plan *plan, const hs_clip_lib *lib, const hs_clip_params *params,
                                  const float *grad_quat, const float *grad_trans, float *grad_key_quat,
                                  float *grad_key_trans, float *grad_time, float *grad_weight, float *workspace,
                                  hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * reverse mode of hs_pose_sample with hs_pose_sample_backward's workspace
 * route, the workspace being a static device array of the library
 * (HS_NOALLOC_MAX_JOINTS joints x 32 bytes = 16 MiB, one copy per device,
 * held until the process ends) instead of caller memory.  Arguments,
 * layouts and outputs are those of hs_pose_sample_backward without
 * `workspace`; the results equal that call's with a workspace, bit for bit
 * (the same kernels).  The call allocates nothing.  A plan of more than
 * HS_NOALLOC_MAX_JOINTS joints returns HS_ERR_INVALID_ARG with nothing
 * launched.  The array needs no clearing: each call writes every entry it
 * reads.  All calls on one device share that array, so calls that overlap
 * in time on one device (other streams, other threads) race; serialise
 * them. */
#define HS_NOALLOC_MAX_JOINTS (1 << 19)
hs_status hs_pose_sample_backward_noalloc(const hs_plan *plan, const hs_clip_lib *lib,
                                          const hs_clip_params *params, const float *grad_quat,
                                          const float *grad_trans, float *grad_key_quat, float *grad_key_trans,
                                          float *grad_time, float *grad_weight, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Hierarchy-Scan (Sec. 1 step 2; Eq. 1; Sec. 3) with optional fused skin.
 * ------------------------------------------------------------------------ */

#define HS_POSE_TRS 0   /* local poses given as quat/trans/scale arrays */
#define HS_POSE_CLIPS 1 /* local poses sampled on the fly (hs_pose_sample, fused) */

typedef struct hs_pose_src {
    int32_t kind;                  /* HS_POSE_TRS or HS_POSE_CLIPS */
    const float *quat;             /* TRS: [N,4] */
    const float *trans;            /* TRS: [N,3] */
    const float *scale;            /* TRS: [N,3] or NULL for unit scale */
    const hs_clip_lib *clips;      /* CLIPS */
    const hs_clip_params *params;  /* CLIPS */
} hs_pose_src;

/* Global transforms G_j = G_parent(j) L_j for every joint of the plan.
 *   global_out [N,4,4]  written if non-NULL;
 *   inv_bind   [N,4,4]  with skin_out [N,4,4]: if both are non-NULL the skin
 *                        S_j = G_j * inv_bind_j (full 4x4 product) is written
 *                        from the same pass (fused Bind MeshPose step);
 *   ckpt_out   [N,12]   if non-NULL (ckpt_k >= 1): rows 0-2 of G_j are stored
 *                        for joints whose level (root = 1) is a multiple of
 *                        ckpt_k, other rows untouched -- the checkpoints
 *                        hs_scan_backward may read instead of recomputing.
 * At least one of global_out, skin_out must be non-NULL.  flags: 0 or
 * HS_FLAG_VALIDATE. */
hs_status hs_scan_forward(const hs_plan *plan, const hs_pose_src *src, float *global_out,
                          const float *inv_bind, float *skin_out, float *ckpt_out, int32_t ckpt_k,
                          uint32_t flags, hipStream_t stream);

/* Bind MeshPose step on its own: S_j = G_j * inv_bind_j, full 4x4 products,
 * for n joints. */
hs_status hs_skin(int64_t n, const float *global, const float *inv_bind, float *skin_out,
                  hipStream_t stream);

/* ------------------------------------------------------------------------
 * HIP graphs: one frame's forward pass captured once, replayed per frame.
 * ------------------------------------------------------------------------ */

/* Capture one hs_scan_forward call, with exactly these arguments, into an
 * instantiated HIP graph (on a private stream of the plan's device).  The
 * pointers are baked into the graph: every replay reads the current contents
 * of the same input arrays and rewrites the same outputs.  The plan and the
 * arrays must outlive the graph.  Argument errors are those of
 * hs_scan_forward; capture or instantiation failures return HS_ERR_DEVICE. */
hs_status hs_graph_create_forward(const hs_plan *plan, const hs_pose_src *src, float *global_out,
                                  const float *inv_bind, float *skin_out, hs_graph **out);

/* Capture n hs_scan_forward calls, in order, into one graph: call i takes
 * srcs[i] and global_outs[i], inv_binds[i], skin_outs[i] (host arrays of n
 * entries each; a NULL array stands for n NULL pointers).  One replay runs
 * the n passes back to back for a single host call, e.g. several frames of
 * a serving loop, or ping-pong buffers.  n >= 1; otherwise the rules and
 * errors of hs_graph_create_forward, checked for every call before any
 * capture starts.  hs_graph_create_forward is the case n = 1. */
hs_status hs_graph_create_forward_n(const hs_plan *plan, int32_t n, const hs_pose_src *srcs,
                                    float *const *global_outs, const float *const *inv_binds,
                                    float *const *skin_outs, hs_graph **out);

/* Replay the captured work on `stream` (asynchronous, no allocation). */
hs_status hs_graph_launch(hs_graph *graph, hipStream_t stream);
void hs_graph_destroy(hs_graph *graph);

/* ------------------------------------------------------------------------
 * Adjoint of the Hierarchy-Scan.
 * ------------------------------------------------------------------------ */

/* Given dLoss/dG (grad_global [N,4,4]; its bottom rows are ignored since G's
 * bottom row is constant), writes dLoss/dq (grad_quat [N,4], derivative of
 * the rotation polynomial in the raw quaternion components), dLoss/dt
 * (grad_trans [N,3]) and, if non-NULL, dLoss/ds (grad_scale [N,3]).  The
 * global transforms the adjoint needs are recomputed (ckpt NULL: for
 * characters of up to 1024 joints as a by-product of the adjoint's own
 * doubling) or, for characters of up to 1664 joints, rebuilt from the
 * checkpoints that hs_scan_forward stored with the same ckpt_k, each G_j
 * as its nearest checkpointed ancestor's rows times at most ckpt_k - 1
 * local transforms (the dataflow kernel).  Larger characters get them from
 * one forward pass over their anchors, so ckpt is not read there.  The
 * results agree up to rounding either way.  Not bitwise reproducible
 * across runs where pushes collide (float atomics).
 * src must be HS_POSE_TRS.  flags: 0 or HS_FLAG_VALIDATE. */
hs_status hs_scan_backward(const hs_plan *plan, const hs_pose_src *src, const float *grad_global,
                           const float *ckpt, int32_t ckpt_k, float *grad_quat, float *grad_trans,
                           float *grad_scale, uint32_t flags, hipStream_t stream);

/* Gradient of the end-effector loss sum_e |b_e - y_e|^2, with b_e the
 * translation column of G_e (the loss of the adjoint's workload and of
 * IK-style loops): writes 2 (b_e - y_e) into column 3 of rows 0-2 of
 * grad_global[e] for every effector e (device int64 ids in [0,
 * num_joints), distinct; targets [num_effectors, 3]) and leaves the rest of
 * grad_global untouched (keep it zero).  Ids outside [0, num_joints) are
 * skipped.  Errors: HS_ERR_INVALID_ARG for NULL or misaligned arrays and
 * for grad_global overlapping an input.
 * Asynchronous; allocates nothing. */
hs_status hs_effector_loss_grad(int64_t num_joints, int64_t num_effectors, const int64_t *effectors,
                                const float *global, const float *targets, float *grad_global, hipStream_t stream);

/* The adjoint of an end-effector loss without a dense dLoss/dG.  With
 * loss = sum_e |b_e - y_e|^2 over a fixed set of joints e (b_e the
 * translation column of G_e), dLoss/dG is zero except in column 3 of rows
 * 0-2 of the effectors' rows; the adjoint's reverse accumulation
 * (X_j = D_j + sum over children c of X_c (.) L_c, derived for this library
 * from Eq. 1, since the paper has no backward) can start from those few
 * seeds.
 *
 * hs_effectors_create takes the effectors' global joint ids on the HOST
 * (num_effectors of them, distinct, in [0, num_joints); HS_ERR_INVALID_ARG
 * otherwise), sorts them and, when every adjoint tile of the plan runs the
 * synchronous-round kernel (characters of up to 1024 joints and the default
 * adjoint option), records each tile's share; hs_effectors_sparse then
 * returns 1.  Otherwise the set keeps a zeroed dense dLoss/dG buffer of
 * 64 bytes per joint.  It synchronises the device once; the set belongs to
 * the plan and must be destroyed before it.
 *
 * hs_effector_backward writes what hs_effector_loss_grad followed by
 * hs_scan_backward (recompute mode) would write, up to rounding: dLoss/dq,
 * dLoss/dt and, if grad_scale is non-NULL, dLoss/ds.  global is the
 * forward's output for the same pose ([N,4,4], 16-byte aligned), targets
 * [num_effectors, 3] the y_e in the order the ids were given.  On a sparse
 * set the synchronous-round tiles form each seed 2 (b_e - y_e) in LDS from
 * global and targets and dLoss/dG is never stored; otherwise the loss
 * gradient kernel fills the set's dense buffer and the general adjoint
 * reads it.  src must be HS_POSE_TRS.  Errors: HS_ERR_INVALID_ARG for NULL
 * or misaligned arrays, a set made for another plan or outputs overlapping
 * inputs.  Asynchronous; allocates nothing.  Calls with one dense set must
 * not overlap (they share its buffer). */
typedef struct hs_effectors hs_effectors;
hs_status hs_effectors_create(const hs_plan *plan, int64_t num_effectors, const int64_t *joint_ids,
                              hs_effectors **out);
void hs_effectors_destroy(hs_effectors *effectors);
int32_t hs_effectors_sparse(const hs_effectors *effectors);
hs_status hs_effector_backward(const hs_plan *plan, const hs_effectors *effectors, const hs_pose_src *src,
                               const float *global, const float *targets, float *grad_quat, float *grad_trans,
                               float *grad_scale, hipStream_t stream);

/* Forward scan and end-effector adjoint in one launch: each adjoint tile
 * first runs the forward scan of its characters in LDS (the blocks of
 * hs_scan_forward, Sec. 3.2.1), takes the seeds 2 (b_e - y_e) from it,
 * then runs the reverse rounds.  Writes what hs_scan_forward (global_out,
 * if non-NULL: G [N,4,4], 16-byte aligned) followed by hs_effector_backward
 * would write, up to rounding, without a separate forward launch or a
 * read of G.  Needs a sparse effector set (hs_effectors_sparse = 1):
 * HS_ERR_UNSUPPORTED otherwise.  src must be HS_POSE_TRS.  Other errors as
 * for hs_effector_backward.  Asynchronous; allocates nothing. */
hs_status hs_effector_step(const hs_plan *plan, const hs_effectors *effectors, const hs_pose_src *src,
                           const float *targets, float *global_out, float *grad_quat, float *grad_trans,
                           float *grad_scale, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Vertex skinning: the stage after Bind MeshPose.  The paper's pipeline
 * skins meshes with the skin matrices on the GPU (Sec. 3; Sec. 4 uses
 * meshes of 1000-3000 faces); each vertex moves by a weighted blend of the
 * S_j = G_j B_j^-1 of up to four joints of its character.
 * ------------------------------------------------------------------------ */

/* HS_SKIN_LINEAR: linear blend, p' = (sum_i w_i S_{j_i}) [p, 1], weights as
 * given.  HS_SKIN_DUAL_QUAT: dual quaternion skinning (Kavan, Collins,
 * Zara, O'Sullivan 2008): each S_j read as a rigid transform (its 3x3 block
 * as a rotation) and turned into a unit dual quaternion, the influences
 * summed with w_i times the sign of their rotation quaternion's dot product
 * with influence 0's (influence 0 is the pivot), normalised by the real
 * part, applied as a rigid transform; a row whose weights sum the real parts
 * to zero gives NaN. */
#define HS_SKIN_LINEAR 0
#define HS_SKIN_DUAL_QUAT 1

/* Meshes of a plan's characters.  Character c's skinned vertices are
 * output rows vertex_offsets[c] .. vertex_offsets[c+1]-1 (vertex_offsets[0]
 * = 0, non-decreasing); its k-th vertex is row mesh_first[c] + k of the mesh
 * arrays, so characters of one kind share their rows.  joints[] are
 * character-local joint ids (unused slots: any valid id with weight 0).
 * All pointers may be host or device memory; hs_mesh_create copies them. */
typedef struct hs_mesh_batch {
    const int64_t *vertex_offsets; /* [C+1] */
    const int32_t *mesh_first;     /* [C] */
    int64_t num_rows;              /* rows of the mesh arrays */
    const float *positions;        /* [num_rows, 3] bind-space positions */
    const int32_t *joints;         /* [num_rows, 4] */
    const float *weights;          /* [num_rows, 4] */
} hs_mesh_batch;

typedef struct hs_mesh hs_mesh;

/* Validate and copy a mesh batch for the plan's characters: mesh rows in
 * range, every joint id in [0, joints of its character), characters with
 * vertices at most 2048 joints (HS_ERR_UNSUPPORTED beyond), total vertices
 * below 2^31.  Errors: HS_ERR_INVALID_ARG.  Synchronises the device once. */
hs_status hs_mesh_create(const hs_plan *plan, const hs_mesh_batch *mesh, hs_mesh **out);
void hs_mesh_destroy(hs_mesh *mesh);

/* Skin every vertex: skin[N,4,4] (device, 16-byte aligned; rows 0-2 read)
 * from hs_scan_forward / hs_skin, out[V,3] (device, 4-byte aligned, V =
 * vertex_offsets[C]).  Asynchronous on stream; allocates nothing.  Errors:
 * HS_ERR_INVALID_ARG (NULL or misaligned arrays, unknown method, out
 * overlapping skin). */
hs_status hs_skin_vertices(const hs_mesh *mesh, const float *skin, int32_t method, float *out,
                           hipStream_t stream);

/* The whole pipeline in one pass per tile: local poses (TRS arrays or
 * clips, as hs_scan_forward), the scan, the skin matrices S_j = G_j B_j^-1
 * (inv_bind as in hs_scan_forward: per joint, or per skeleton joint for an
 * instanced plan) and vertex skinning of the mesh, which must have been
 * made for this plan.  S stays on chip; skin_out (nullable, [N,4,4]) also
 * writes it.  vertices_out [V,3] as hs_skin_vertices, bitwise the same
 * result as hs_scan_forward followed by hs_skin_vertices.  Every character
 * must be on a tile and tiles may hold at most 2048 joints
 * (HS_ERR_UNSUPPORTED otherwise: use the two calls).  Errors as
 * hs_scan_forward and hs_skin_vertices.  Asynchronous; allocates nothing. */
hs_status hs_scan_skin_vertices(const hs_plan *plan, const hs_pose_src *src, const float *inv_bind,
                                const hs_mesh *mesh, int32_t method, float *vertices_out, float *skin_out,
                                hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HS_H_ */
