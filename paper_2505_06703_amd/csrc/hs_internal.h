// hs_internal.h -- device-table layouts and kernel-launch entry points shared
// by the C-ABI host code (hs_capi.cpp) and the kernels (hs_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hs {

// Largest tile (joints) a workgroup can hold in the 160 KiB LDS of gfx950,
// including the per-character table of the fused sampler.
constexpr int kMaxTileJoints = 3072;

// Largest tile of the dataflow adjoint kernel, which keeps both the global
// transforms and the adjoint accumulators of the tile in LDS (96 bytes per
// joint).
constexpr int kMaxBwdTileJoints = 1664;

// Largest tile of the synchronous-round adjoint kernel: one joint per
// thread, 104 bytes of LDS per joint (jump product, inbox, pointer, owner
// word) and a flag per 64-joint block.
constexpr int kMaxSyncTileJoints = 1024;

// Most anchors of one in-LDS segment of the multipass anchor rounds (one
// thread each; 52 bytes of LDS per anchor).
constexpr int kAnchorSegCap = 1024;

// Device status word of a plan (two 32-bit words): word 0 collects the bits
// below, word 1 the lowest global joint id that failed the topology check
// (0xFFFFFFFF while none has).  The values equal HS_DEV_* of hs.h.
constexpr uint32_t kStatusWaitTimeout = 1u; // a bounded wait gave up
constexpr uint32_t kStatusTopology = 2u;    // the device topology check failed

// Polls a bounded wait makes before it gives up (the plan's default).
constexpr int kDefaultSpinLimit = 1 << 22;

// A tile: a contiguous range of global joint ids holding whole characters,
// scanned by one workgroup entirely in LDS.
struct TileDesc {
    int64_t begin;      // global id of the tile's first joint
    int32_t count;      // joints in the tile (<= tile capacity)
    int32_t first_char; // index of the tile's first character
    int32_t num_chars;  // characters in the tile (empty ones included)
    // bit b of (chain_hi:chain_lo) set: a chain unit of up to 4 blocks starts
    // at block b (every parent in it is the previous joint or before it)
    int32_t chain_lo;
    int32_t chain_hi;
    // pointer-jumping rounds that cover the deepest joint of the tile:
    // ceil(log2(max level)), the root at level 1
    int32_t rounds;
};
static_assert(sizeof(TileDesc) == 32, "TileDesc layout");

// A tile of the work-queue forward kernel: a contiguous range of global
// joint ids holding whole characters, whose joints find their parent
// through the plan's per-joint codes (QueueLaunch::code).
struct QTile {
    int64_t begin;       // global id of the tile's first joint
    int32_t count;       // joints in the tile
    int32_t first_char;  // index of the tile's first character
    int32_t num_chars;   // characters in the tile
    int32_t num_anchors; // anchors of the tile (their transforms stay in LDS)
    int32_t pad[2];
};
static_assert(sizeof(QTile) == 32, "QTile layout");

// Per-joint code of a queue tile (int32):
//   bits 0-11   parent reference: the in-block lane of the parent when bit
//               12 is set, else 1 + the anchor slot of the parent (0: root)
//   bit 12      the parent lies in the joint's own 64-joint block
//   bits 13-24  1 + the joint's own anchor slot (0: not an anchor)
// An anchor is a joint whose transform a later block of the tile needs:
// the parent of some joint of another block.
constexpr int kQRefBits = 12;
constexpr int kQInBlock = 1 << kQRefBits;
constexpr int kQOwnShift = kQRefBits + 1;
constexpr int kQMaxAnchors = (1 << kQRefBits) - 1;
constexpr int kQMaxTileJoints = 4096;

struct QueueLaunch {
    const QTile *tiles;       // heaviest first
    int32_t num_tiles;
    int32_t waves;            // 4, 8 or 16
    // persistent workgroups (<= num_tiles) by [poses sampled in the kernel]
    // [skin rows staged]: each instance and LDS layout has its own occupancy;
    // grid: the one launched (set by launch_forward_queue)
    int32_t grids[2][2];
    int32_t grid;
    int32_t max_anchors;      // LDS anchor slots (largest num_anchors)
    int32_t tile_cap;         // largest tile (the fused sampler's character table)
    const int32_t *code;      // [N] per-joint codes
    uint32_t *status;
    int32_t spin_limit;
    const uint32_t *gate;
};

// A 64-joint block of a character on the multipass path.  Blocks start at
// the character's first joint, so a block never spans two characters.
struct MPBlock {
    int64_t gbegin;  // global id of the block's first joint
    int64_t cbegin;  // index of that joint in the compact multipass arrays
    int32_t count;   // joints in the block (1..64)
    int32_t chr;     // character index
    int64_t pad;
};
static_assert(sizeof(MPBlock) == 32, "MPBlock layout");

// Where local poses come from.
struct PoseArgs {
    int32_t kind;          // 0 = TRS arrays, 1 = clips
    const float *quat;     // [N,4]
    const float *trans;    // [N,3]
    const float *scale;    // [N,3] or null
    // clips
    const int64_t *offsets; // [C+1] device copy of the CSR offsets
    int32_t num_clips, num_keys, joints_per_clip;
    float fps;
    const float *key_quat;  // [clips][keys][J][4]
    const float *key_trans; // [clips][keys][J][3]
    const int32_t *clip_a, *clip_b;
    const float *time, *weight;
};

// Outputs of a forward pass.
struct OutArgs {
    float *global_out;      // [N,16] or null
    const float *inv_bind;  // [N,16] or null ([skeleton joints,16] for instanced plans)
    float *skin_out;        // [N,16] or null
    float *ckpt;            // [N,12] or null
    int32_t ckpt_k;
    const int32_t *level;   // [N] level of each joint (root = 1), for checkpoints
};

// adjoint kernels for tiles of up to kMaxSyncTileJoints joints (the values
// of HS_ADJ_ROUNDS and HS_ADJ_DATAFLOW)
constexpr int32_t kAdjRounds = 1;
constexpr int32_t kAdjDataflow = 2;
constexpr int32_t kAdjAnchors = 3;

struct TileLaunch {
    const TileDesc *tiles;
    int32_t num_tiles;
    int32_t tile_cap;   // joints
    int32_t waves;      // 1..16
    int32_t grid;       // workgroups
    const int32_t *parent; // [N] global parent id or -1
    int32_t chain_units;   // tiles carry chain-unit marks
    int32_t algorithm;     // 0: this library's scan; 1-4: the paper's Algorithms 1-4
    int32_t adjoint;       // kAdjRounds or kAdjDataflow
    // instanced plans (non-null): characters share their skeleton's parents
    // and inverse binds; both are read through the skeleton's first joint
    const int32_t *skel_parent; // [skeleton joints] skeleton-local parent or -1
    const int32_t *char_skel;   // [C] first skeleton joint of each character's skeleton
    // the plan's status word and the polls of a bounded wait; gate (null
    // unless the call validates): the kernels do nothing once its topology
    // bit is set
    uint32_t *status;
    int32_t spin_limit;
    const uint32_t *gate;
    // the two-level adjoint (kAdjAnchors): per-joint anchor codes of the
    // adjoint tiles (the layout of QueueLaunch::code) and the most anchors
    // of one tile
    const int32_t *code;
    int32_t max_anchors;
    int32_t blocks_per_wave;  // the two-level adjoint: 64-joint blocks per wave (1 or 2)
};

// The one-pass path for chain characters on the multipass path (every
// joint's parent the previous joint): 64-joint blocks in chain order,
// grouped into superblocks of up to 64 consecutive blocks of one chain.
struct ChainBlock {
    int64_t gbegin;  // global id of the block's first joint
    int32_t count;   // joints in the block (1..64)
    int32_t sb;      // superblock
    int32_t k;       // index of the block in its superblock
    int32_t chr;     // character
    int64_t pad;
};
static_assert(sizeof(ChainBlock) == 32, "ChainBlock layout");

struct ChainSB {
    int32_t first;        // first block
    int32_t nblk;         // blocks (1..64)
    int32_t chain_first;  // the chain's first superblock
    int32_t pad;
};

struct ChainLaunch {
    const ChainBlock *blocks;
    int32_t num_blocks;
    const ChainSB *sbs;
    int32_t num_sb;
    int32_t grid;      // workgroups, all resident at once
    uint64_t *recs;    // [superblocks][12] tagged words: the product of the superblock's local
                       // transforms (kind 1), then G of its last joint (kind 2), tagged with
                       // the call's epoch; zeroed once when allocated
    uint32_t *epoch;   // [2]: the last call's epoch, and the count of its finished workgroups
    uint32_t *status;
    int32_t spin_limit;
    const uint32_t *gate;
};

struct MPLaunch {
    const MPBlock *blocks;
    int32_t num_blocks;
    int64_t nmp;              // joints on the multipass path (compact count)
    const int32_t *parent;    // [N] global parent id or -1
    // anchors: the joints that are some joint's nearest out-of-block
    // ancestor; the cross-block phase jumps over these only
    const int32_t *janc;      // [Nmp] anchor index of the joint's out-of-block ancestor, or -1
    const int32_t *aself;     // [Nmp] the joint's own anchor index, or -1
    int32_t num_anchors;
    int32_t rounds;           // anchor-level jump rounds
    float4 *A1;               // [num_anchors*3] anchors' in-block products (phase 1)
    int32_t *E1;              // [num_anchors] anchor index of each anchor's own anchor, or -1
    float4 *AP[2];            // [num_anchors*3] ping-pong anchor products
    int32_t *AE[2];           // [num_anchors] ping-pong anchor pointers
    // segments of at most kAnchorSegCap consecutive anchors that no anchor
    // points out of ([num_aseg + 1] offsets): each segment's rounds run in
    // one workgroup's LDS; num_aseg = 0: rounds over all anchors in HBM
    const int32_t *aseg;
    int32_t num_aseg;
    // adjoint workspace (NULL when the plan has none)
    float4 *S[2];             // [num_anchors*3] ping-pong anchor adjoints
    float4 *G;                // [Nmp*3] global transforms
    const uint32_t *gate;     // as TileLaunch::gate
};

struct BwdArgs {
    const float *grad_global; // [N,16]
    const float *ckpt;        // [N,12] or null
    int32_t ckpt_k;
    const int32_t *level;     // [N]
    float *grad_quat;         // [N,4]
    float *grad_trans;        // [N,3]
    float *grad_scale;        // [N,3] or null
    // Sparse end-effector loss sum_e |b_e - y_e|^2 (synchronous-round tiles
    // only; grad_global is then not read): the adjoint's seed is
    // 2 (b_e - y_e) in the translation column of each listed joint e, with
    // b_e read from the forward output, and zero elsewhere.
    const int64_t *eff_ids;   // [E] global joint ids, ascending, distinct; null = dense seed
    const int32_t *eff_row;   // [E] row of eff_target for each id
    const int32_t *eff_tile;  // [tiles][2] range [lo, hi) of eff_ids in each adjoint tile
    const float *eff_global;  // [N,16] forward output (not read when eff_forward)
    const float *eff_target;  // [E,3]
    // the forward scan runs inside each adjoint tile (blocks of the forward
    // kernel, G in LDS) and the seeds come from it; eff_global_out, if not
    // null, receives G [N,16]
    int32_t eff_forward;
    float *eff_global_out;
};

// Kernel launchers (hs_kernels.hip).  Each returns the hipError_t of the
// launch; none synchronises or allocates.
hipError_t launch_forward_tiles(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                                hipStream_t stream);
hipError_t launch_forward_queue(const QueueLaunch &ql, const PoseArgs &pose, const OutArgs &out,
                                hipStream_t stream);
size_t forward_queue_lds_bytes(int waves, int max_anchors, int tile_cap, bool sample, bool skin);
size_t backward_anchor_lds_bytes(int waves, int max_anchors, int tile_cap);
// Workgroups of the two-level adjoint (waves per workgroup, blocks per
// wave, seed kind 0 dense / 1 effectors / 2 forward in the tile) that fit
// one CU with `lds` bytes of LDS.
hipError_t anchor_blocks_per_cu(int waves, int bpw, int seed, size_t lds, int *out);
// Workgroups of the queue kernel (stored or sampled poses; G or skin
// output) that fit one CU with `lds` bytes of LDS.
hipError_t queue_blocks_per_cu(int waves, bool sample, bool skin, size_t lds, int *out);
hipError_t launch_forward_multipass(const MPLaunch &ml, const PoseArgs &pose, const OutArgs &out,
                                    hipStream_t stream);
// The one-pass chain path (clears its words, then one persistent launch).
hipError_t launch_forward_chains(const ChainLaunch &cl, const PoseArgs &pose, const OutArgs &out,
                                 hipStream_t stream);
// Workgroups of the chain kernel (stored or sampled poses) that fit one CU.
hipError_t chain_blocks_per_cu(bool sample, int *out);
constexpr int kChainWaves = 16;     // waves per workgroup of the chain kernel
constexpr int kChainSBBlocks = 64;  // 64-joint blocks per superblock of the chain kernel
hipError_t launch_backward_tiles(const TileLaunch &tl, const PoseArgs &pose, const BwdArgs &bwd,
                                 hipStream_t stream);
hipError_t launch_backward_multipass(const MPLaunch &ml, const PoseArgs &pose, const BwdArgs &bwd,
                                     hipStream_t stream);
hipError_t launch_pose_sample(const TileLaunch &tl, const MPLaunch &ml, const ChainLaunch &cl, const PoseArgs &pose,
                              float *quat_out, float *trans_out, hipStream_t stream);
hipError_t launch_skin(int64_t n, const float *global, const float *inv_bind, float *skin_out,
                       hipStream_t stream);

// Raise the dynamic-LDS limit of every tile kernel to what its largest tile
// needs (once per process and device, before any launch or capture).
hipError_t prepare_kernels();

// Topology check of a plan's device tables (HS_FLAG_VALIDATE): for every
// joint g of character c, parent[g] is -1 with level[g] = 1, or lies in
// [offsets[c], g) with level[g] = level[parent[g]] + 1; offsets must be
// non-decreasing.  Failures set kStatusTopology in status[0] and the lowest
// failing joint in status[1].
hipError_t launch_validate(const int64_t *offsets, int64_t num_chars, const int32_t *parent, const int32_t *level,
                           uint32_t *status, hipStream_t stream);

hipError_t launch_stream_probe(int64_t n, const float *quat, const float *trans, const float *scale,
                               const int32_t *table, float *out, hipStream_t stream);
hipError_t launch_effector_grad(int64_t n, int64_t ne, const int64_t *eff, const float *G, const float *target,
                                float *grad, hipStream_t stream);

// Reverse mode of the sampler (see hs_pose_sample_backward).
struct SampleBwdArgs {
    const float *grad_quat;    // [N,4]
    const float *grad_trans;   // [N,3]
    float *grad_key_quat;      // [clips*keys*J*4] or null
    float *grad_key_trans;     // [clips*keys*J*3] or null
    float *grad_time;          // [C] or null
    float *grad_weight;        // [C] or null
    int32_t C;
    // [N][2] adjoints of each joint's two unnormalised key blends, or null:
    // when given, the time/weight kernel stores them and the key gather
    // reads them instead of recomputing each reader's reverse step
    float4 *ws;
};
hipError_t launch_pose_sample_backward(const PoseArgs &pose, const SampleBwdArgs &A, hipStream_t stream);

// The allocation-free route of the sampler's reverse mode keeps its
// workspace ([N][2] float4) in a static device array of this many joints.
constexpr int64_t kNoAllocMaxJoints = 1 << 19;  // HS_NOALLOC_MAX_JOINTS
constexpr int kMaxDevices = 64;
// Device address of the calling thread's current device's copy of that
// array (looked up once per device, then cached); call with `device`
// current.
hipError_t noalloc_workspace(int device, float4 **out);

// Vertex skinning (after the Bind MeshPose step): character c's vertices
// are output rows voff[c] .. voff[c+1]-1; its k-th vertex reads mesh row
// mfirst[c] + k; joint ids are character-local (checked when the mesh is
// created: 0 <= id < the character's joint count <= kMaxSkinJoints).
constexpr int kMaxSkinJoints = 2048;
struct VertexLaunch {
    const int64_t *offsets;  // [C+1] joint CSR offsets
    const int64_t *voff;     // [C+1] vertex offsets
    const int32_t *mfirst;   // [C] first mesh row of each character
    const float *pos;        // [rows,3] bind-space positions
    const int32_t *joints;   // [rows,4]
    const float *weights;    // [rows,4]
    int32_t C;
    int32_t max_joints;      // largest character with vertices (LDS staging)
};
// method 0: linear blend; 1: dual quaternions
hipError_t launch_vertex_skin(const VertexLaunch &vl, int method, const float *skin, float *out,
                              hipStream_t stream);
// Scan + skin + vertex skinning per tile (tiles of at most
// kMaxVertexTileJoints joints; out.inv_bind required, out.skin_out optional).
constexpr int kMaxVertexTileJoints = 2048;
size_t forward_vertex_lds_bytes(int tile_cap);
hipError_t launch_forward_vertices(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                                   const VertexLaunch &vl, int method, float *vout, hipStream_t stream);

// Tiles of the paper's Algorithms 1-4 (one joint per thread).
constexpr int kPaperAlgTileJoints = 1024;

// LDS bytes one tiled-forward workgroup needs.
// char_map: the tile also holds its characters' start offsets (clip
// sampling, instanced plans)
size_t forward_tile_lds_bytes(int tile_cap, bool char_map);
size_t backward_tile_lds_bytes(int tile_cap);
size_t backward_sync_lds_bytes(int tile_cap);
size_t paper_alg_lds_bytes(int tile_cap, int alg);

} // namespace hs
