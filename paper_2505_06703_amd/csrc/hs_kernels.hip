// hs_kernels.hip -- CDNA4 (gfx950) kernels of the hierarchy scan.
//
// Data layout
//   Local poses are read as structure-of-arrays fields (quat [N,4] as one
//   16-byte vector per joint, trans/scale [N,3]); 64 consecutive joints are
//   handled by one 64-lane wave, so every load instruction of a wave reads
//   one contiguous span.  Affine transforms live in registers as 3x4
//   row-major fp32 (12 values); the constant bottom row (0,0,0,1) is never
//   stored or multiplied.
//
// Forward scan (tiled path, fwd_tile_kernel)
//   A workgroup owns a tile: a contiguous id range of whole characters.
//   The tile is cut into 64-joint blocks (the paper's blocks, Sec. 3.2.1),
//   one block per wave at a time.
//   Phase 1: pointer jumping restricted to in-block ancestors (Sec. 3.1 and
//     Eq. 2, applied inside the block as in Sec. 3.2), done with cross-lane
//     permutes: the 64 lanes of a wave run in lockstep, so the rounds need
//     no barrier and read the previous round's registers by construction.
//     The wave keeps jumping only while some lane still has an in-block
//     ancestor, i.e. ceil(log2(in-block depth)) rounds.  Each lane ends with
//     the product over its in-block path and its nearest out-of-block
//     ancestor (MaxParentOutBlock of Sec. 3.2.1).
//   Phase 2: instead of walking the out-of-block ancestors' partial
//     products (one composition per block crossed), each block waits on an
//     LDS flag until the block holding its out-of-block ancestor is final
//     and then needs exactly one composition: G_j = G_ext(j) * P_j.  Blocks
//     only depend on lower-numbered blocks and every wave processes its
//     blocks in increasing order, so the waits always drain.  Final 3x4
//     transforms are kept in LDS for later blocks and written to HBM as
//     contiguous 16-byte rows.
//
// Forward scan (multipass path) for characters larger than a tile:
//   the same phase 1 per 64-joint block into HBM, then ceil(log2 L)
//   rounds of global pointer jumping over the blocks' out-of-block
//   pointers (L = longest chain of blocks on a path), then one output pass.
//
// All arithmetic is fp32 on the vector ALUs with fused multiply-adds; the
// 3x4 compositions are far too small for matrix cores.

#include "hs_internal.h"

#include <algorithm>
#include <mutex>
#include <cmath>

namespace hs {
namespace {

constexpr int kWave = 64;

// Record status bits in the plan's status word (device scope).
__device__ __forceinline__ void note_status(uint32_t *status, uint32_t bits)
{
    __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True when the call validates and the device topology check has failed:
// the kernel then does nothing (the check ran earlier on the same stream,
// so every thread of the launch reads the same final value).
__device__ __forceinline__ bool gated(const uint32_t *gate)
{
    return gate && (__hip_atomic_load(gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kStatusTopology);
}

// ---------------------------------------------------------------------------
// 3x4 affine helpers (row-major, m[4*r + c], column 3 = translation)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void aff_identity(float m[12])
{
#pragma unroll
    for (int k = 0; k < 12; ++k) m[k] = (k % 5 == 0) ? 1.0f : 0.0f;
}

// L = [R(q) diag(s) | t] with the textbook polynomial of q = (x, y, z, w).
__device__ __forceinline__ void aff_from_trs(float4 q, float tx, float ty, float tz, float sx,
                                             float sy, float sz, float m[12])
{
    // every sum is written as an explicit fma so that the rounding does not
    // depend on how the compiler contracts the surrounding code: every
    // kernel forms bitwise the same local transform from the same pose
    const float x = q.x, y = q.y, z = q.z, w = q.w;
    const float yy = y * y, zz = z * z;
    const float wx = w * x, wy = w * y, wz = w * z;
    m[0] = fmaf(-2.0f, fmaf(y, y, zz), 1.0f) * sx;
    m[1] = 2.0f * fmaf(x, y, -wz) * sy;
    m[2] = 2.0f * fmaf(x, z, wy) * sz;
    m[3] = tx;
    m[4] = 2.0f * fmaf(x, y, wz) * sx;
    m[5] = fmaf(-2.0f, fmaf(x, x, zz), 1.0f) * sy;
    m[6] = 2.0f * fmaf(y, z, -wx) * sz;
    m[7] = ty;
    m[8] = 2.0f * fmaf(x, z, -wy) * sx;
    m[9] = 2.0f * fmaf(y, z, wx) * sy;
    m[10] = fmaf(-2.0f, fmaf(x, x, yy), 1.0f) * sz;
    m[11] = tz;
}

// o = a * b  ([A|u][B|v] = [AB | Av + u]): 36 FMA-class operations.
__device__ __forceinline__ void aff_mul(const float a[12], const float b[12], float o[12])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float a0 = a[4 * r], a1 = a[4 * r + 1], a2 = a[4 * r + 2], a3 = a[4 * r + 3];
        o[4 * r + 0] = fmaf(a0, b[0], fmaf(a1, b[4], a2 * b[8]));
        o[4 * r + 1] = fmaf(a0, b[1], fmaf(a1, b[5], a2 * b[9]));
        o[4 * r + 2] = fmaf(a0, b[2], fmaf(a1, b[6], a2 * b[10]));
        o[4 * r + 3] = fmaf(a0, b[3], fmaf(a1, b[7], fmaf(a2, b[11], a3)));
    }
}

__device__ __forceinline__ void aff_mul_left(const float a[12], float m[12])
{
    float o[12];
    aff_mul(a, m, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) m[k] = o[k];
}

__device__ __forceinline__ void aff_load(const float4 *p, float m[12])
{
    const float4 r0 = p[0], r1 = p[1], r2 = p[2];
    m[0] = r0.x; m[1] = r0.y; m[2] = r0.z; m[3] = r0.w;
    m[4] = r1.x; m[5] = r1.y; m[6] = r1.z; m[7] = r1.w;
    m[8] = r2.x; m[9] = r2.y; m[10] = r2.z; m[11] = r2.w;
}

// Streaming stores of outputs that no kernel of the call reads again (and
// streaming loads of inputs read once): the non-temporal hint keeps them
// from displacing cached inputs and tables.  Used only where a wave writes
// whole contiguous lines (coalesced 16-byte rows): per-lane rows 64 bytes
// apart measured slower with the hint (their partial lines are no longer
// merged in the cache before going to HBM).
typedef float native_float4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_stream(float4 *p, float4 v)
{
    const native_float4 n = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(n, reinterpret_cast<native_float4 *>(p));
}

__device__ __forceinline__ void aff_store(float4 *p, const float m[12])
{
    p[0] = make_float4(m[0], m[1], m[2], m[3]);
    p[1] = make_float4(m[4], m[5], m[6], m[7]);
    p[2] = make_float4(m[8], m[9], m[10], m[11]);
}

// Orders a wave's LDS accesses: every lane's earlier accesses complete
// before any lane's later ones.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float lane_read(float v, int byte_addr)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
}

// ---------------------------------------------------------------------------
// Simulation step: sample two looping clips and blend them.
// ---------------------------------------------------------------------------

// Normalised lerp of two key quaternions; the shorter-arc sign is taken from
// an fp64 sum of the exact fp32 products (x, y, z, w order) so that it is
// reproducible bit for bit on any implementation.
__device__ __forceinline__ float4 nlerp_keys(float4 a, float4 b, float alpha)
{
    double d = (double)a.x * (double)b.x;
    d = d + (double)a.y * (double)b.y;
    d = d + (double)a.z * (double)b.z;
    d = d + (double)a.w * (double)b.w;
    const float u = 1.0f - alpha;
    const float v = d < 0.0 ? -alpha : alpha;
    float4 r = make_float4(fmaf(u, a.x, v * b.x), fmaf(u, a.y, v * b.y), fmaf(u, a.z, v * b.z),
                           fmaf(u, a.w, v * b.w));
    const float inv = rsqrtf(fmaf(r.x, r.x, fmaf(r.y, r.y, fmaf(r.z, r.z, r.w * r.w))));
    return make_float4(r.x * inv, r.y * inv, r.z * inv, r.w * inv);
}

__device__ __forceinline__ float4 nlerp_blend(float4 a, float4 b, float wgt)
{
    const float d = fmaf(a.x, b.x, fmaf(a.y, b.y, fmaf(a.z, b.z, a.w * b.w)));
    const float u = 1.0f - wgt;
    const float v = d < 0.0f ? -wgt : wgt;
    float4 r = make_float4(fmaf(u, a.x, v * b.x), fmaf(u, a.y, v * b.y), fmaf(u, a.z, v * b.z),
                           fmaf(u, a.w, v * b.w));
    const float inv = rsqrtf(fmaf(r.x, r.x, fmaf(r.y, r.y, fmaf(r.z, r.z, r.w * r.w))));
    return make_float4(r.x * inv, r.y * inv, r.z * inv, r.w * inv);
}

// Keys and interpolation parameter of character chr: frame f = fps * time
// (one fp32 multiply), k0 = floor(f) mod K, k1 = k0 + 1 mod K, alpha =
// f - floor(f).  False for an out-of-range clip id or a non-finite time.
__device__ __forceinline__ bool sample_frame(const PoseArgs &P, int chr, int &k0, int &k1, float &alpha)
{
    const int ca = P.clip_a[chr], cb = P.clip_b[chr];
    const int K = P.num_keys;
    const float f = __fmul_rn(P.fps, P.time[chr]);
    const float fl = floorf(f);
    alpha = f - fl;
    k0 = k1 = 0;
    if (!(isfinite(fl) && ca >= 0 && ca < P.num_clips && cb >= 0 && cb < P.num_clips)) return false;
    float r = fmodf(fl, (float)K);
    if (r < 0.0f) r += (float)K;
    k0 = (int)r;
    if (k0 >= K) k0 = 0;
    k1 = (k0 + 1 == K) ? 0 : k0 + 1;
    return true;
}

// Sampled local pose of joint j (character-local) of character chr.  An
// out-of-range clip id or a non-finite time yields NaN poses (never an
// out-of-bounds read).
__device__ __forceinline__ void sample_pose(const PoseArgs &P, int chr, int j, float4 &q, float &tx,
                                            float &ty, float &tz)
{
    const int ca = P.clip_a[chr], cb = P.clip_b[chr];
    const float wgt = P.weight[chr];
    const int K = P.num_keys, J = P.joints_per_clip;
    int k0, k1;
    float alpha;
    if (!sample_frame(P, chr, k0, k1, alpha)) {
        const float nan = __int_as_float(0x7fc00000);
        q = make_float4(nan, nan, nan, nan);
        tx = ty = tz = nan;
        return;
    }
    const int64_t ia0 = ((int64_t)ca * K + k0) * J + j, ia1 = ((int64_t)ca * K + k1) * J + j;
    const int64_t ib0 = ((int64_t)cb * K + k0) * J + j, ib1 = ((int64_t)cb * K + k1) * J + j;
    const float4 *kq = reinterpret_cast<const float4 *>(P.key_quat);
    const float4 qa = nlerp_keys(kq[ia0], kq[ia1], alpha);
    const float4 qb = nlerp_keys(kq[ib0], kq[ib1], alpha);
    const float *kt = P.key_trans;
    const float u = 1.0f - alpha;
    const float ax = fmaf(u, kt[3 * ia0 + 0], alpha * kt[3 * ia1 + 0]);
    const float ay = fmaf(u, kt[3 * ia0 + 1], alpha * kt[3 * ia1 + 1]);
    const float az = fmaf(u, kt[3 * ia0 + 2], alpha * kt[3 * ia1 + 2]);
    const float bx = fmaf(u, kt[3 * ib0 + 0], alpha * kt[3 * ib1 + 0]);
    const float by = fmaf(u, kt[3 * ib0 + 1], alpha * kt[3 * ib1 + 1]);
    const float bz = fmaf(u, kt[3 * ib0 + 2], alpha * kt[3 * ib1 + 2]);
    q = nlerp_blend(qa, qb, wgt);
    const float uw = 1.0f - wgt;
    tx = fmaf(uw, ax, wgt * bx);
    ty = fmaf(uw, ay, wgt * by);
    tz = fmaf(uw, az, wgt * bz);
}

template <bool SAMPLE>
__device__ __forceinline__ void load_local(const PoseArgs &P, int64_t gid, int chr, int lj, float m[12])
{
    if constexpr (SAMPLE) {
        float4 q;
        float tx, ty, tz;
        sample_pose(P, chr, lj, q, tx, ty, tz);
        aff_from_trs(q, tx, ty, tz, 1.0f, 1.0f, 1.0f, m);
    } else {
        // each pose value is read once per call: streaming loads
        const native_float4 qn = __builtin_nontemporal_load(reinterpret_cast<const native_float4 *>(P.quat) + gid);
        const float4 q = make_float4(qn.x, qn.y, qn.z, qn.w);
        const float *t = P.trans + 3 * gid;
        float sx = 1.0f, sy = 1.0f, sz = 1.0f;
        if (P.scale) {
            const float *s = P.scale + 3 * gid;
            sx = __builtin_nontemporal_load(s);
            sy = __builtin_nontemporal_load(s + 1);
            sz = __builtin_nontemporal_load(s + 2);
        }
        aff_from_trs(q, __builtin_nontemporal_load(t), __builtin_nontemporal_load(t + 1),
                     __builtin_nontemporal_load(t + 2), sx, sy, sz, m);
    }
}

// ---------------------------------------------------------------------------
// Phase 1: in-block pointer jumping across the 64 lanes of a wave.
//   a : lane of the current in-block jump target, or -1
//   e : nearest out-of-block ancestor once known (caller's id space), or -1
// On return every lane holds the product over its in-block path.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_inblock_scan(float m[12], int &a, int &e, int lane)
{
    // Six rounds at most: a path inside one 64-joint block has at most 64
    // joints.  The rounds are unrolled so that no value is carried through a
    // loop back-edge (which would cost a register copy per round); the
    // update is a per-lane select rather than a branch.
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        if (!__any(a >= 0)) break;
        const bool act = a >= 0;
        const int src = (act ? a : lane) << 2;
        float ma[12], o[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) ma[k] = lane_read(m[k], src);
        const int aa = __builtin_amdgcn_ds_bpermute(src, a);
        const int ea = __builtin_amdgcn_ds_bpermute(src, e);
        aff_mul(ma, m, o);
#pragma unroll
        for (int k = 0; k < 12; ++k) m[k] = act ? o[k] : m[k];
        e = (act && aa < 0) ? ea : e;
        a = act ? aa : a;
    }
}

// The same scan with the rows moving through the wave's own LDS slice (X:
// [64][S] float4, S >= 3) with 16-byte accesses instead of 4-byte
// cross-lane permutes (measured faster on deep chains); the products and
// their order are those of wave_inblock_scan, so the results are bitwise
// equal.  xi: [64] int holding a and e packed (e < 2^24), or with xe
// non-null a in xi and e in xe ([64] int each).
__device__ __forceinline__ void wave_inblock_scan_lds(float m[12], int &a, int &e, int lane, float4 *X, int *xi,
                                                      int S = 3, int *xe = nullptr)
{
#pragma unroll 1
    for (int r = 0; r < 6; ++r) {
        if (!__any(a >= 0)) break;
        const bool act = a >= 0;
        wave_sync();  // the previous round's reads are done
        aff_store(X + S * lane, m);
        if (xe) {
            xi[lane] = a;
            xe[lane] = e;
        } else {
            xi[lane] = (a + 1) | ((e + 1) << 7);
        }
        wave_sync();
        if (act) {
            float ma[12];
            aff_load(X + S * a, ma);
            int aa, ea;
            if (xe) {
                aa = xi[a];
                ea = xe[a];
            } else {
                const int pk = xi[a];
                aa = (pk & 127) - 1;
                ea = (pk >> 7) - 1;
            }
            aff_mul_left(ma, m);
            if (aa < 0) e = ea;
            a = aa;
        }
    }
    wave_sync();  // the slice is free for the caller
}

// Find the character of tile-local joint jl: the largest i with cstart[i] <= jl.
__device__ __forceinline__ int tile_char_of(const int *cstart, int num_chars, int jl)
{
    int lo = 0, hi = num_chars - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= jl) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// bidx: row of the joint's inverse bind (gid, or the skeleton joint of an
// instanced plan)
__device__ __forceinline__ void write_skin_and_ckpt(const OutArgs &out, int64_t gid, int64_t bidx, const float m[12])
{
    if (out.skin_out) {
        const float4 *B = reinterpret_cast<const float4 *>(out.inv_bind) + 4 * bidx;
        const float4 b0 = B[0], b1 = B[1], b2 = B[2], b3 = B[3];
        float4 *S = reinterpret_cast<float4 *>(out.skin_out) + 4 * gid;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float g0 = m[4 * r], g1 = m[4 * r + 1], g2 = m[4 * r + 2], g3 = m[4 * r + 3];
            S[r] = make_float4(fmaf(g0, b0.x, fmaf(g1, b1.x, fmaf(g2, b2.x, g3 * b3.x))),
                               fmaf(g0, b0.y, fmaf(g1, b1.y, fmaf(g2, b2.y, g3 * b3.y))),
                               fmaf(g0, b0.z, fmaf(g1, b1.z, fmaf(g2, b2.z, g3 * b3.z))),
                               fmaf(g0, b0.w, fmaf(g1, b1.w, fmaf(g2, b2.w, g3 * b3.w))));
        }
        S[3] = b3;
    }
    if (out.ckpt && out.level[gid] % out.ckpt_k == 0)
        aff_store(reinterpret_cast<float4 *>(out.ckpt) + 3 * gid, m);
}

// ---------------------------------------------------------------------------
// Tiled forward kernel.
// LDS: G[cap][3] float4 | unit partials [cap/64][3] float4 | block flags,
// partial flags, partial anchors [cap/64] int | (SAMPLE) char starts [cap+1]
// ---------------------------------------------------------------------------
// LDS of the tiled forward kernel, and the bound of its waits.
struct FwdShared {
    float4 *G;       // [cap][3] final transforms (rows 0-2)
    float4 *part;    // [cap/64][3] partial product of a chain unit's last segment
    int *flags;      // [cap/64] block published its final transforms
    int *pflag;      // [cap/64] partial of the unit ending with this block published
    int *panc;       // [cap/64] anchor of that partial (tile-local id, or -1)
    int *cstart;     // (pose sampling) character starts
    uint32_t *status; // the plan's status word
    int spin;         // polls of a bounded wait
};

// Bounded wait until the block of tile-local joint e (if e >= 0) has
// published its final transforms.  The bound only guards against a broken
// invariant: after sh.spin polls (far beyond any legitimate wait) the wave
// records kStatusWaitTimeout in the plan's status word and proceeds with
// whatever the LDS holds instead of hanging the device.
__device__ __forceinline__ void wait_block_of(const FwdShared &sh, int e)
{
    const bool need = e >= 0;
    const int fb = need ? (e / kWave) : 0;
    bool done = !__any(need);
    for (int spin = 0; !done && spin < sh.spin; ++spin) {
        const int ok = need ? __hip_atomic_load(sh.flags + fb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 1;
        done = __all(ok);
        if (!done) __builtin_amdgcn_s_sleep(1);
    }
    if (!done) note_status(sh.status, kStatusWaitTimeout);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// m <- G_e m for tile-local joint e (no-op for e < 0), waiting (bounded, as
// above) until e's transform is known: either e's block has published, or
// e ends a chain unit that has published the partial product P of its last
// segment, in which case G_e = G_a P with a the segment's anchor, and the
// wait moves on to a.  Partials let a unit start as soon as the earlier
// unit's scan is done instead of after its final pass.
__device__ __forceinline__ void compose_final(const FwdShared &sh, int e, float m[12])
{
    for (int spin = 0; spin < sh.spin; ++spin) {
        if (__all(e < 0)) break;
        int fin = 0, step = 0;
        if (e >= 0) {
            const int be = e >> 6;
            fin = __hip_atomic_load(sh.flags + be, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (!fin && (e & (kWave - 1)) == kWave - 1)
                step = __hip_atomic_load(sh.pflag + be, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (fin) {
            float g[12];
            aff_load(sh.G + 3 * e, g);
            aff_mul_left(g, m);
            e = -1;
        } else if (step) {
            const int be = e >> 6;
            float pp[12];
            aff_load(sh.part + 3 * be, pp);
            aff_mul_left(pp, m);
            e = sh.panc[be];
        }
        if (!__any(fin | step)) __builtin_amdgcn_s_sleep(1);
    }
    if (__any(e >= 0)) note_status(sh.status, kStatusWaitTimeout);
}

// Publish blocks [b0, b0 + nb) of the tile: their final transforms are in LDS.
__device__ __forceinline__ void publish_blocks(int *flags, int b0, int nb, int lane)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane < nb) __hip_atomic_store(flags + b0 + lane, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Global matrices of tile-local joints [base, base + 64 * nb) leave as 16-byte
// rows, 4 per joint; each store instruction covers 1 KiB of contiguous output.
template <int MAXNB>
__device__ __forceinline__ void store_rows(const OutArgs &out, const float4 *Gs, int64_t tile_begin, int base,
                                           int nb, int n, int lane)
{
    const float4 bottom = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    float4 *dst = reinterpret_cast<float4 *>(out.global_out) + 4 * (tile_begin + base);
#pragma unroll
    for (int k = 0; k < 4 * MAXNB; ++k) {
        if (k >= 4 * nb) break;
        const int c = lane + kWave * k;
        const int jj = base + (c >> 2);
        const int r = c & 3;
        if (jj < n) {
            float4 v = Gs[3 * jj + (r == 3 ? 0 : r)];
            if (r == 3) v = bottom;
            store_stream(dst + c, v);
        }
    }
}

template <bool MAP>
__device__ __forceinline__ void char_of(const TileDesc &td, const int *cstart, int jl, int &chr, int &lj)
{
    chr = 0;
    lj = 0;
    if constexpr (MAP) {
        const int c = tile_char_of(cstart, td.num_chars, jl);
        chr = td.first_char + c;
        lj = jl - cstart[c];
    }
}

// One lane's joint of a 64-joint block: local transform, in-block ancestor
// lane a and nearest out-of-block ancestor e (tile-local), as the in-block
// scan expects them, and the joint's inverse-bind row.  INST: the parent
// comes from the character's skeleton (shared by many characters, so the
// reads hit the caches), as does the inverse bind.
template <bool SAMPLE, bool INST>
__device__ __forceinline__ void block_begin(const TileLaunch &tl, const PoseArgs &pose, const TileDesc &td, int n,
                                            int b, const FwdShared &sh, int lane, float m[12], int &a, int &e,
                                            int64_t &bidx)
{
    const int base = b * kWave;
    const int jl = base + lane;
    a = -1;
    e = -1;
    bidx = td.begin + jl;
    if (jl < n) {
        const int64_t gid = td.begin + jl;
        int chr, lj;
        char_of<SAMPLE || INST>(td, sh.cstart, jl, chr, lj);
        int pl;
        if constexpr (INST) {
            const int sj = tl.char_skel[chr] + lj;
            const int ps = tl.skel_parent[sj];
            pl = ps < 0 ? -1 : jl - lj + ps;
            bidx = sj;
        } else {
            const int p = tl.parent[gid];
            pl = p < 0 ? -1 : (int)(p - td.begin);
        }
        if (pl >= base) a = pl - base; else e = pl;
        load_local<SAMPLE>(pose, gid, chr, lj, m);
    } else {
        aff_identity(m);
    }
}

// After the in-block scan: one composition with the final transform of the
// nearest out-of-block ancestor once its block has published it, then the
// block's own publication and outputs.
__device__ __forceinline__ void block_finish(const OutArgs &out, const TileDesc &td, int n, int b,
                                             const FwdShared &sh, int lane, float m[12], int e, int64_t bidx)
{
    float4 *Gs = sh.G;
    const int base = b * kWave;
    const int jl = base + lane;
    const bool valid = jl < n;
    wait_block_of(sh, valid ? e : -1);
    if (valid && e >= 0) {
        float g[12];
        aff_load(Gs + 3 * e, g);
        aff_mul_left(g, m);
    }
    if (valid) aff_store(Gs + 3 * jl, m);
    publish_blocks(sh.flags, b, 1, lane);
    if (out.global_out) store_rows<1>(out, Gs, td.begin, base, 1, n, lane);
    if (valid) write_skin_and_ckpt(out, td.begin + jl, bidx, m);
}

// One 64-joint block: in-block pointer jumping across the wave, then the
// cross-block composition.
template <bool SAMPLE, bool INST>
__device__ __forceinline__ void fwd_block(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                                          const TileDesc &td, int n, int b, const FwdShared &sh, int lane)
{
    float m[12];
    int a, e;
    int64_t bidx;
    block_begin<SAMPLE, INST>(tl, pose, td, n, b, sh, lane, m, a, e, bidx);
    wave_inblock_scan(m, a, e, lane);
    block_finish(out, td, n, b, sh, lane, m, e, bidx);
}

// A block of the forward scan inside an adjoint tile (one block per wave,
// lane = the tile thread of the same joint): as fwd_block, and the joint's
// local transform also goes to L (the adjoint's first jump products) while
// its rotation and scale stay in the caller's registers for the gradients,
// so that each pose is read once.
__device__ __forceinline__ void fwd_block_keep(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                                               const TileDesc &td, int n, int b, const FwdShared &sh, int lane,
                                               float4 *L, float4 &q, float &sx, float &sy, float &sz)
{
    const int base = b * kWave;
    const int jl = base + lane;
    float m[12];
    int a = -1, e = -1;
    if (jl < n) {
        const int64_t gid = td.begin + jl;
        const int p = tl.parent[gid];
        const int pl = p < 0 ? -1 : (int)(p - td.begin);
        if (pl >= base) a = pl - base; else e = pl;
        const native_float4 qn = __builtin_nontemporal_load(reinterpret_cast<const native_float4 *>(pose.quat) + gid);
        q = make_float4(qn.x, qn.y, qn.z, qn.w);
        const float *t = pose.trans + 3 * gid;
        if (pose.scale) {
            const float *sp = pose.scale + 3 * gid;
            sx = __builtin_nontemporal_load(sp);
            sy = __builtin_nontemporal_load(sp + 1);
            sz = __builtin_nontemporal_load(sp + 2);
        }
        aff_from_trs(q, __builtin_nontemporal_load(t), __builtin_nontemporal_load(t + 1),
                     __builtin_nontemporal_load(t + 2), sx, sy, sz, m);
        aff_store(L + 3 * jl, m);
    } else {
        aff_identity(m);
    }
    wave_inblock_scan(m, a, e, lane);
    block_finish(out, td, n, b, sh, lane, m, e, td.begin + jl);
}

// The K local transforms of unit joints [i0, i0 + K) from the
// component-major staging area (stride S).  Lanes that own no joints read
// the first K slots instead; their values are never stored.
template <int K>
__device__ __forceinline__ void read_staged(const float *stage, int S, int i0, bool owns, float L[K][12])
{
    static_assert(K == 4, "one float4 per component");
    const int i = owns ? i0 : 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const float4 v = *reinterpret_cast<const float4 *>(stage + k * S + i);
        L[0][k] = v.x;
        L[1][k] = v.y;
        L[2][k] = v.z;
        L[3][k] = v.w;
    }
}

// A chain unit: kChainK * 64 consecutive joints (up to kChainK blocks) in
// which every joint's parent is either the previous joint or lies before
// the unit, i.e. the unit is a set of contiguous chain segments.  Lane l
// owns joints [kChainK l, kChainK l + kChainK) of the unit:
//   1. the lane's local transforms arrive through LDS (loaded coalesced,
//      staged component-major so that both the staging writes and each
//      lane's 16-byte reads of its kChainK joints are free of bank
//      conflicts) and stay in registers;
//   2. the product of the lane's open segment (kChainK - 1 compositions);
//   3. a segmented scan of those products across the wave (log2 64 rounds,
//      restarting at segment heads), carrying each segment's out-of-unit
//      anchor;
//   4. the transform preceding the lane's first joint (anchor's final
//      transform times the previous lanes' prefix, one composition), then
//      one composition per joint, in order.
// About 3.5 compositions per joint instead of 6 + 1 for a 64-deep block.
constexpr int kChainK = 4;

template <bool SAMPLE>
__device__ __forceinline__ void fwd_chain_unit(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                                               const TileDesc &td, int n, int b0, int nb, const FwdShared &sh,
                                               int lane)
{
    float4 *Gs = sh.G;
    const int *cstart = sh.cstart;
    const int ubase = b0 * kWave;
    const int S = nb * kWave;  // joints the unit spans; the staging stride
    float *stage = reinterpret_cast<float *>(Gs + 3 * ubase);  // 12 * S floats, the unit's own slots

    // 1. staging: component k of unit joint i at stage[k * S + i]
#pragma unroll
    for (int s = 0; s < kChainK; ++s) {
        if (s >= nb) break;
        const int i = s * kWave + lane;
        const int jl = ubase + i;
        float L[12];
        if (jl < n) {
            int chr, lj;
            char_of<SAMPLE>(td, cstart, jl, chr, lj);
            load_local<SAMPLE>(pose, td.begin + jl, chr, lj, L);
        } else {
            aff_identity(L);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) stage[k * S + i] = L[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const int i0 = kChainK * lane;
    const bool owns = i0 < S;
    // the lane's local transforms are read again after the scan (the
    // staging slots stay intact until step 4 writes) to keep register use low
    // 2. product of the lane's open segment.  anc: tile-local anchor of each
    // joint's segment (parent before the unit, or -1 for a root), or kOpen
    // while the segment continues from the previous lane.
    constexpr int kOpen = -2;
    bool valid[kChainK], head[kChainK];
    int par[kChainK], anc[kChainK];
    float T[12];
    float L[kChainK][12];
    read_staged<kChainK>(stage, S, i0, owns, L);
#pragma unroll
    for (int s = 0; s < kChainK; ++s) {
        const int jl = ubase + i0 + s;
        valid[s] = owns && jl < n;
        int p = -1;
        if (valid[s]) {
            const int pg = tl.parent[td.begin + jl];
            p = pg < 0 ? -1 : (int)(pg - td.begin);
        }
        par[s] = p;
        head[s] = !(valid[s] && p == jl - 1 && p >= ubase);
        if (s == 0) {
#pragma unroll
            for (int k = 0; k < 12; ++k) T[k] = L[0][k];
            anc[0] = head[0] ? p : kOpen;
        } else {
            float o[12];
            aff_mul(T, L[s], o);
#pragma unroll
            for (int k = 0; k < 12; ++k) T[k] = head[s] ? L[s][k] : o[k];
            anc[s] = head[s] ? p : anc[s - 1];
        }
    }

    // 3. segmented inclusive scan of the lane products; code = head flag |
    // (anchor + 1) << 1 for the segment open at the end of the lane
    int code = anc[kChainK - 1] == kOpen ? 0 : (1 | ((anc[kChainK - 1] + 1) << 1));
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const bool need = !(code & 1) && lane >= d;
        if (!__any(need)) break;
        const int src = (lane >= d ? lane - d : lane) << 2;
        float ta[12], o[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) ta[k] = lane_read(T[k], src);
        const int ca = __builtin_amdgcn_ds_bpermute(src, code);
        aff_mul(ta, T, o);
#pragma unroll
        for (int k = 0; k < 12; ++k) T[k] = need ? o[k] : T[k];
        code = need ? ca : code;
    }

    // the partial product of the segment open at the unit's last joint
    // lets the next unit go ahead before this one finishes
    const int last = S / kChainK - 1;
    if (lane == last && ubase + S <= n) {
        const int bl = b0 + nb - 1;
        aff_store(sh.part + 3 * bl, T);
        sh.panc[bl] = (code >> 1) - 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __hip_atomic_store(sh.pflag + bl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    // 4. the transform before the lane's first joint: the previous lane's
    // inclusive prefix (lane 0 always starts with a head) behind its anchor
    const int src = (lane > 0 ? lane - 1 : 0) << 2;
    float pre[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) pre[k] = lane_read(T[k], src);
    const int xa = (__builtin_amdgcn_ds_bpermute(src, code) >> 1) - 1;
    const bool open = owns && anc[0] == kOpen;
    compose_final(sh, open ? xa : -1, pre);
    read_staged<kChainK>(stage, S, i0, owns, L);
#pragma unroll
    for (int s = 0; s < kChainK; ++s) {
        const bool h = valid[s] && head[s];
        if (h) aff_identity(pre);
        compose_final(sh, h ? par[s] : -1, pre);
        float o[12];
        aff_mul(pre, L[s], o);
#pragma unroll
        for (int k = 0; k < 12; ++k) pre[k] = o[k];
        if (valid[s]) aff_store(Gs + 3 * (ubase + i0 + s), pre);
    }
    if (out.skin_out || out.ckpt) {
#pragma unroll 1
        for (int s = 0; s < kChainK; ++s) {
            const int jl = ubase + i0 + s;
            if (!owns || jl >= n) break;
            float g[12];
            aff_load(Gs + 3 * jl, g);
            write_skin_and_ckpt(out, td.begin + jl, td.begin + jl, g);
        }
    }
    publish_blocks(sh.flags, b0, nb, lane);
    if (out.global_out) store_rows<kChainK>(out, Gs, td.begin, ubase, nb, n, lane);
}

// ---------------------------------------------------------------------------
// Tiled forward kernel.
// LDS: G[cap][3] float4 | unit partials [cap/64][3] float4 | block flags,
// partial flags, partial anchors [cap/64] int | (SAMPLE) char starts [cap+1]
// The tile is cut into units -- single 64-joint blocks, or chain units of up
// to kChainK blocks where the plan found contiguous chain segments -- dealt
// to the waves round-robin; each wave processes its units in increasing
// order, and a unit only waits on blocks before it, so the waits drain.
// ---------------------------------------------------------------------------
// MODE 0: blocks; 1: chain units; 2: blocks of an instanced plan
template <int WAVES, bool SAMPLE, int MODE>
__global__ void __launch_bounds__(WAVES * kWave)
fwd_tile_kernel(TileLaunch tl, PoseArgs pose, OutArgs out)
{
    constexpr bool CHAIN = MODE == 1;
    constexpr bool INST = MODE == 2;
    extern __shared__ float4 lds[];
    if (gated(tl.gate)) return;
    const int cap = tl.tile_cap;
    const int nbk = cap >> 6;
    FwdShared sh;
    sh.G = lds;
    sh.part = lds + 3 * cap;
    sh.flags = reinterpret_cast<int *>(sh.part + 3 * nbk);
    sh.pflag = sh.flags + nbk;
    sh.panc = sh.pflag + nbk;
    sh.cstart = sh.panc + nbk;
    sh.status = tl.status;
    sh.spin = tl.spin_limit;
    int *cstart = sh.cstart;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;

    for (int tile = blockIdx.x; tile < tl.num_tiles; tile += gridDim.x) {
        const TileDesc td = tl.tiles[tile];
        const int n = td.count;
        const int nblk = (n + kWave - 1) / kWave;
        const uint64_t chain_starts = ((uint64_t)(uint32_t)td.chain_hi << 32) | (uint32_t)td.chain_lo;
        for (int i = threadIdx.x; i < nblk; i += WAVES * kWave) {
            sh.flags[i] = 0;
            sh.pflag[i] = 0;
        }
        if constexpr (SAMPLE || INST) {
            for (int i = threadIdx.x; i <= td.num_chars; i += WAVES * kWave)
                cstart[i] = (int)(pose.offsets[td.first_char + i] - td.begin);
        }
        __syncthreads();

        if constexpr (CHAIN) {
            int unit = 0;
            for (int b = 0; b < nblk; ++unit) {
                const bool chain = (chain_starts >> b) & 1;
                const int nb = chain ? min(kChainK, nblk - b) : 1;
                if (unit % WAVES == wave) {
                    if (chain)
                        fwd_chain_unit<SAMPLE>(tl, pose, out, td, n, b, nb, sh, lane);
                    else
                        fwd_block<SAMPLE, false>(tl, pose, out, td, n, b, sh, lane);
                }
                b += nb;
            }
        } else {
            for (int b = wave; b < nblk; b += WAVES) fwd_block<SAMPLE, INST>(tl, pose, out, td, n, b, sh, lane);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Work-queue forward kernel: every tile of the plan in one persistent
// launch.  The plan lists the tiles heaviest first; round r of the
// workgroups takes the next gridDim.x of them, in alternating directions
// (a static stride: a shared ticket counter serialised the workgroups on
// its atomics), so tiles of every size share the launch and no size class
// waits for another to drain.
//
// LDS holds only what other blocks read: the final transforms of the
// tile's anchors (the parents of joints in other blocks; the plan numbers
// them into slots) and a ready flag per slot, plus one staging slice per
// wave for the coalesced row stores.  A block scans its 64 joints across
// the wave as in the tiled kernel, carrying the slot of its nearest
// out-of-block ancestor instead of a joint id; it waits for that slot's
// flag, composes once, stores its anchors' transforms and raises their
// flags.  The LDS footprint therefore follows the anchor count, not the
// tile size, and large tiles keep several workgroups per CU.
// LDS: staging [WAVES][64][3 or 4] float4 (also the in-block scan's slices;
// 4 rows when skin rows are staged) |
// scan ints [WAVES][64] | anchors [max_anchors][3] float4 | flags
// [max_anchors] int | (SAMPLE) char starts [tile_cap + 1]
// ---------------------------------------------------------------------------
// Bounded wait (as wait_block_of) until anchor slot e (if e >= 0) is ready.
__device__ __forceinline__ void wait_slot(const int *flags, int e, uint32_t *status, int limit)
{
    const bool need = e >= 0;
    bool done = !__any(need);
    for (int spin = 0; !done && spin < limit; ++spin) {
        const int ok = need ? __hip_atomic_load(flags + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 1;
        done = __all(ok);
        if (!done) __builtin_amdgcn_s_sleep(1);
    }
    if (!done) note_status(status, kStatusWaitTimeout);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Rows of the block's 64 joints from the wave's slice X (stride S float4
// per joint; `rows` of them hold data: with 3 the fourth row is the
// constant (0, 0, 0, 1)) to dst (four 16-byte rows per joint, n joints at
// most): each store instruction covers 1 KiB of contiguous output, written
// with the streaming hint.
__device__ __forceinline__ void store_slice_rows(float4 *dst, const float4 *X, int S, int rows, int n, int lane)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = lane + kWave * k;
        const int jj = c >> 2, r = c & 3;
        if (jj < n) store_stream(dst + c, r < rows ? X[S * jj + r] : make_float4(0.0f, 0.0f, 0.0f, 1.0f));
    }
}

// SS: float4 rows per joint in the staging slice (3, or 4 when skin rows
// are staged too)
template <bool SAMPLE, bool SKIN>
__device__ __forceinline__ void queue_block(const QueueLaunch &ql, const PoseArgs &pose, const OutArgs &out,
                                            const QTile &td, int b, float4 *stage, int SS, int *xi, float4 *anc,
                                            int *flags, const int *cstart, int lane)
{
    const int base = b * kWave;
    const int jl = base + lane;
    const bool valid = jl < td.count;
    const int64_t gid = td.begin + jl;
    float m[12];
    int a = -1, e = -1, own = -1;
    if (valid) {
        const int code = ql.code[gid];
        const int ref = code & (kQInBlock - 1);
        if (code & kQInBlock) a = ref; else e = ref - 1;
        own = (code >> kQOwnShift) - 1;
        int chr = 0, lj = 0;
        if constexpr (SAMPLE) {
            const int c = tile_char_of(cstart, td.num_chars, jl);
            chr = td.first_char + c;
            lj = jl - cstart[c];
        }
        load_local<SAMPLE>(pose, gid, chr, lj, m);
    } else {
        aff_identity(m);
    }
    wave_inblock_scan_lds(m, a, e, lane, stage, xi, SS);
    wait_slot(flags, valid ? e : -1, ql.status, ql.spin_limit);
    if (valid && e >= 0) {
        float g[12];
        aff_load(anc + 3 * e, g);
        aff_mul_left(g, m);
    }
    if (own >= 0) aff_store(anc + 3 * own, m);
    aff_store(stage + SS * lane, m);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (own >= 0) __hip_atomic_store(flags + own, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nb = td.count - base;  // joints of this block (may exceed 64: clipped by the row stores)
    if (out.global_out)
        store_slice_rows(reinterpret_cast<float4 *>(out.global_out) + 4 * (td.begin + base), stage, SS, 3, nb, lane);
    if constexpr (SKIN) {
        // S = G B^-1 (the bottom row of S is B^-1's), staged like G so that
        // the rows leave as whole lines
        float4 srow[4];
        if (valid) {
            const float4 *B = reinterpret_cast<const float4 *>(out.inv_bind) + 4 * gid;
            const float4 b0 = B[0], b1 = B[1], b2 = B[2], b3 = B[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const float g0 = m[4 * r], g1 = m[4 * r + 1], g2 = m[4 * r + 2], g3 = m[4 * r + 3];
                srow[r] = make_float4(fmaf(g0, b0.x, fmaf(g1, b1.x, fmaf(g2, b2.x, g3 * b3.x))),
                                      fmaf(g0, b0.y, fmaf(g1, b1.y, fmaf(g2, b2.y, g3 * b3.y))),
                                      fmaf(g0, b0.z, fmaf(g1, b1.z, fmaf(g2, b2.z, g3 * b3.z))),
                                      fmaf(g0, b0.w, fmaf(g1, b1.w, fmaf(g2, b2.w, g3 * b3.w))));
            }
            srow[3] = b3;
        } else {
            srow[0] = srow[1] = srow[2] = srow[3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        wave_sync();  // the G rows have left the slice
#pragma unroll
        for (int r = 0; r < 4; ++r) stage[4 * lane + r] = srow[r];
        wave_sync();
        store_slice_rows(reinterpret_cast<float4 *>(out.skin_out) + 4 * (td.begin + base), stage, 4, 4, nb, lane);
    }
    if (valid && out.ckpt && out.level[gid] % out.ckpt_k == 0)
        aff_store(reinterpret_cast<float4 *>(out.ckpt) + 3 * gid, m);
    // the slice is written again by this wave's next block only after
    // every lane's reads above
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int WAVES, bool SAMPLE, bool SKIN>
__global__ void __launch_bounds__(WAVES * kWave)
fwd_queue_kernel(QueueLaunch ql, PoseArgs pose, OutArgs out)
{
    extern __shared__ float4 lds[];
    if (gated(ql.gate)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    constexpr int SS = SKIN ? 4 : 3;  // staged rows per joint
    float4 *stage = lds + wave * kWave * SS;
    int *xi = reinterpret_cast<int *>(lds + WAVES * kWave * SS) + wave * kWave;
    float4 *anc = lds + WAVES * kWave * SS + WAVES * kWave / 4;
    int *flags = reinterpret_cast<int *>(anc + 3 * ql.max_anchors);
    int *cstart = flags + ql.max_anchors;

    for (int r = 0;; ++r) {
        // round r takes tiles [r G, (r + 1) G) of the heaviest-first list,
        // in alternating directions, so that each workgroup's total stays
        // close to the others'
        const int G = (int)gridDim.x;
        const int tile = r * G + ((r & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (tile >= ql.num_tiles) break;  // uniform: every wave leaves together
        const QTile td = ql.tiles[tile];
        for (int i = threadIdx.x; i < td.num_anchors; i += WAVES * kWave) flags[i] = 0;
        if constexpr (SAMPLE) {
            for (int i = threadIdx.x; i <= td.num_chars; i += WAVES * kWave)
                cstart[i] = (int)(pose.offsets[td.first_char + i] - td.begin);
        }
        __syncthreads();
        const int nblk = (td.count + kWave - 1) / kWave;
        for (int b = wave; b < nblk; b += WAVES)
            queue_block<SAMPLE, SKIN>(ql, pose, out, td, b, stage, SS, xi, anc, flags, cstart, lane);
        __syncthreads();  // LDS is reused by the next tile
    }
}

// ---------------------------------------------------------------------------
// The paper's Algorithms 1-4 as tile kernels (plan option `algorithm`), for
// comparison with the scan above on this hardware.  One workgroup of 1024
// threads per tile, one joint per thread, the tile's local transforms in
// LDS, barriers where the algorithms synchronise, coalesced row stores at
// the end.  Rounds are synchronous (read phase, barrier, write phase), the
// reading under which the printed in-place updates do not race.
//   1 (Sec. 2): every joint walks to its root, multiplying the ancestors'
//     local transforms on the left.
//   2 (Sec. 3.1, Eq. 2): pointer jumping over the whole tile,
//     ceil(log2 depth) rounds.
//   3 (Sec. 3.2.1): blocks of 64; log2(64) = 6 rounds of pointer jumping over
//     in-block ancestors; then each joint walks its chain of nearest
//     out-of-block ancestors (MaxParentOutBlock), multiplying their in-block
//     partial products.
//   4 (Sec. 3.2.2): in-block, up to 7 single parent steps (a window of 8),
//     then up to 7 hops of 8 levels over those windows; then the walk of 3.
// LDS: A[cap][3] float4 | B[cap][3] float4 (Algorithm 4) | par, up, mpob [cap] int
// ---------------------------------------------------------------------------
template <int ALG>
__global__ void __launch_bounds__(1024)
paper_alg_kernel(TileLaunch tl, PoseArgs pose, OutArgs out)
{
    extern __shared__ float4 lds[];
    if (gated(tl.gate)) return;
    const int cap = tl.tile_cap;
    float4 *As = lds;
    float4 *Bs = lds + 3 * cap;
    int *par = reinterpret_cast<int *>(lds + (ALG == 4 ? 6 : 3) * cap);
    int *up = par + cap;
    int *mp = up + cap;
    const int jl = threadIdx.x;
    constexpr int kBlock = 64;

    for (int tile = blockIdx.x; tile < tl.num_tiles; tile += gridDim.x) {
        const TileDesc td = tl.tiles[tile];
        const bool live = jl < td.count;
        const int64_t gid = td.begin + jl;
        float L[12];
        int p = -1;
        if (live) {
            const int pg = tl.parent[gid];
            p = pg < 0 ? -1 : (int)(pg - td.begin);
            load_local<false>(pose, gid, 0, 0, L);
            aff_store(As + 3 * jl, L);
            par[jl] = p;
        } else {
            aff_identity(L);
        }
        __syncthreads();
        float m[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) m[k] = L[k];

        if constexpr (ALG == 1) {
            if (live) {
                int cur = p;
                for (int guard = 0; cur >= 0 && guard < cap; ++guard) {
                    float g[12];
                    aff_load(As + 3 * cur, g);
                    aff_mul_left(g, m);
                    cur = par[cur];
                }
            }
        } else if constexpr (ALG == 2) {
            int a = p;
            if (live) up[jl] = a;
            for (int r = 0; r < td.rounds; ++r) {
                __syncthreads();
                int aa = -1;
                if (a >= 0) {
                    float g[12];
                    aff_load(As + 3 * a, g);
                    aa = up[a];
                    aff_mul_left(g, m);
                }
                __syncthreads();
                if (a >= 0) {
                    a = aa;
                    aff_store(As + 3 * jl, m);
                    up[jl] = a;
                }
            }
        } else {
            // in-block parent pointer (-1 at a block boundary or a root) and
            // the nearest out-of-block ancestor (the parent of the topmost
            // in-block ancestor), found by the same rounds
            const int base = jl & ~(kBlock - 1);
            int a = (p >= base) ? p : -1;
            int e = (p >= 0 && p < base) ? p : -1;
            if (live) {
                up[jl] = a;
                mp[jl] = e;
            }
            if constexpr (ALG == 3) {
#pragma unroll 1
                for (int r = 0; r < 6; ++r) {
                    __syncthreads();
                    int aa = -1, ea = -1;
                    if (a >= 0) {
                        float g[12];
                        aff_load(As + 3 * a, g);
                        aa = up[a];
                        ea = mp[a];
                        aff_mul_left(g, m);
                    }
                    __syncthreads();
                    if (a >= 0) {
                        if (aa < 0) e = ea;
                        a = aa;
                        aff_store(As + 3 * jl, m);
                        up[jl] = a;
                        mp[jl] = e;
                    }
                }
            } else {
                // window: up to 7 single steps over the untouched locals
                int cur = a;
                for (int s = 0; s < 7 && cur >= 0; ++s) {
                    float g[12];
                    aff_load(As + 3 * cur, g);
                    aff_mul_left(g, m);
                    if (up[cur] < 0) e = mp[cur];
                    cur = up[cur];
                }
                // cur: the in-block ancestor 8 levels up (or -1)
                if (live) aff_store(Bs + 3 * jl, m);
                __syncthreads();
                // hops of 8 over the windows (read-only during this phase)
                for (int h = 0; h < 7 && cur >= 0; ++h) {
                    float g[12];
                    aff_load(Bs + 3 * cur, g);
                    aff_mul_left(g, m);
                    int nxt = cur;
                    for (int s = 0; s < 8 && nxt >= 0; ++s) {
                        if (up[nxt] < 0) e = mp[nxt];
                        nxt = up[nxt];
                    }
                    cur = nxt;
                }
                __syncthreads();
                if (live) {
                    aff_store(As + 3 * jl, m);
                    mp[jl] = e;
                }
            }
            // the walk over out-of-block ancestors' partials (a snapshot)
            __syncthreads();
            if (live) {
                int cur = e;
                for (int guard = 0; cur >= 0 && guard < cap; ++guard) {
                    float g[12];
                    aff_load(As + 3 * cur, g);
                    aff_mul_left(g, m);
                    cur = mp[cur];
                }
            }
        }
        // outputs: the final transforms through LDS for coalesced row stores
        __syncthreads();
        if (live) aff_store(As + 3 * jl, m);
        __syncthreads();
        if (out.global_out) {
            const float4 bottom = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            float4 *dst = reinterpret_cast<float4 *>(out.global_out) + 4 * td.begin;
            for (int c = jl; c < 4 * td.count; c += 1024) {
                const int r = c & 3;
                float4 v = As[3 * (c >> 2) + (r == 3 ? 0 : r)];
                if (r == 3) v = bottom;
                store_stream(dst + c, v);
            }
        }
        if (live) write_skin_and_ckpt(out, gid, gid, m);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the scan (tiled).
//
// For G_j = G_p L_j the adjoint X_j of G_j (rows 0-2, a 3x4 matrix; the
// constant bottom row carries no gradient) gathers the adjoints of all
// descendants pulled back through the path products between them:
//     X_j = D_j + sum over children c of  X_c (.) L_c,
//     X (.) [R'|t] = [X_A R'^T + X_b t^T | X_b],
// with D_j the incoming dLoss/dG_j.  The gradient of L_j is then
// [A_p^T X_A | A_p^T X_b] with A_p the parent's global rotation-scale block.
//
// Inside a 64-joint block the subtree sums are built by reverse pointer
// jumping: in round r every joint a adds its partial adjoint S_r(a), pulled
// back through the round-r jump product M_r(a) of the forward doubling
// (the product of the 2^r local transforms ending at a), into its 2^r-th
// in-block ancestor.  After ceil(log2 depth) rounds S(j) sums all in-block
// descendants.  Fan-in makes this a scatter: each pusher claims its target's
// owner word with a plain store, the pusher whose claim landed adds with a
// plain read-modify-write, the others with LDS float atomics after it.
// Blocks run in decreasing order; a block's top joints (parent in an
// earlier block) push X_c (.) L_c into the parent's LDS accumulator and
// bump that block's arrival counter, which the earlier block waits for.
// ---------------------------------------------------------------------------

// o = X (.) L  (36 FMA-class operations)
__device__ __forceinline__ void adj_pull(const float X[12], const float L[12], float o[12])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float x0 = X[4 * r], x1 = X[4 * r + 1], x2 = X[4 * r + 2], x3 = X[4 * r + 3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            o[4 * r + c] = fmaf(x0, L[4 * c], fmaf(x1, L[4 * c + 1], fmaf(x2, L[4 * c + 2], x3 * L[4 * c + 3])));
        o[4 * r + 3] = x3;
    }
}

__device__ __forceinline__ void lds_atomic_add12(float4 *dst, const float v[12])
{
    float *d = reinterpret_cast<float *>(dst);
#pragma unroll
    for (int k = 0; k < 12; ++k) atomicAdd(d + k, v[k]);
}

// Gradients of joint gid from its total adjoint X and the parent's global
// rotation-scale block Ap (row-major 3x3).
__device__ __forceinline__ void write_grads(const BwdArgs &B, int64_t gid, const float X[12], const float Ap[9],
                                            float4 q, float sx, float sy, float sz)
{
    float Rb[9], tb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int l = 0; l < 3; ++l)
            Rb[3 * i + l] = fmaf(Ap[i], X[l], fmaf(Ap[3 + i], X[4 + l], Ap[6 + i] * X[8 + l]));
        tb[i] = fmaf(Ap[i], X[3], fmaf(Ap[3 + i], X[7], Ap[6 + i] * X[11]));
    }
    const float x = q.x, y = q.y, z = q.z, w = q.w;
    const float sc[3] = {sx, sy, sz};
    if (B.grad_scale) {
        const float R[9] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y),
                            2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x),
                            2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)};
        float *gs = B.grad_scale + 3 * gid;
#pragma unroll
        for (int l = 0; l < 3; ++l) gs[l] = fmaf(Rb[l], R[l], fmaf(Rb[3 + l], R[3 + l], Rb[6 + l] * R[6 + l]));
    }
    // dLoss/dR = dLoss/dR' diag(s), then through the quaternion polynomial
    float G[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) G[3 * i + l] = Rb[3 * i + l] * sc[l];
    const float gx = 2.0f * (y * (G[1] + G[3]) + z * (G[2] + G[6]) + w * (G[7] - G[5])) - 4.0f * x * (G[4] + G[8]);
    const float gy = 2.0f * (x * (G[1] + G[3]) + w * (G[2] - G[6]) + z * (G[5] + G[7])) - 4.0f * y * (G[0] + G[8]);
    const float gz = 2.0f * (w * (G[3] - G[1]) + x * (G[2] + G[6]) + y * (G[5] + G[7])) - 4.0f * z * (G[0] + G[4]);
    const float gw = 2.0f * (z * (G[3] - G[1]) + y * (G[2] - G[6]) + x * (G[7] - G[5]));
    reinterpret_cast<float4 *>(B.grad_quat)[gid] = make_float4(gx, gy, gz, gw);
    float *gt = B.grad_trans + 3 * gid;
    gt[0] = tb[0];
    gt[1] = tb[1];
    gt[2] = tb[2];
}

// LDS: G[cap][3] | adjoint accumulators[cap][3] float4 | owner words[cap] uint16 |
// flags, expected, received [cap/64] int each
// 16-bit owner words of the dataflow adjoint: (round << 6) | lane, or
// kOwnFree.  Plain stores from several lanes to one word: one lands.
constexpr int kOwn16Shift = 6;
constexpr uint16_t kOwnFree = 0xFFFF;

__device__ __forceinline__ void own16_claim(uint16_t *w, uint16_t v)
{
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int own16_read(const uint16_t *w)
{
    return (int)__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int WAVES, bool CKPT>
__global__ void __launch_bounds__(WAVES * kWave)
bwd_tile_kernel(TileLaunch tl, PoseArgs pose, BwdArgs bwd)
{
    extern __shared__ float4 lds[];
    if (gated(tl.gate)) return;
    const int cap = tl.tile_cap;
    float4 *Gs = lds;
    float4 *Ds = lds + 3 * cap;
    uint16_t *Own = reinterpret_cast<uint16_t *>(lds + 6 * cap);
    int *flags = reinterpret_cast<int *>(Own + cap);
    int *expect = flags + cap / kWave;
    int *recv = expect + cap / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);

    for (int tile = blockIdx.x; tile < tl.num_tiles; tile += gridDim.x) {
        const TileDesc td = tl.tiles[tile];
        const int n = td.count;
        const int nblk = (n + kWave - 1) / kWave;
        for (int i = threadIdx.x; i < nblk; i += WAVES * kWave) {
            flags[i] = 0;
            expect[i] = 0;
            recv[i] = 0;
        }
        for (int i = threadIdx.x; i < 3 * n; i += WAVES * kWave) Ds[i] = zero4;
        __syncthreads();

        // ---- global transforms of the tile into Gs --------------------------
        if constexpr (!CKPT) {
            for (int b = wave; b < nblk; b += WAVES) {
                const int base = b * kWave;
                const int jl = base + lane;
                const bool valid = jl < n;
                const int64_t gid = td.begin + jl;
                float m[12];
                int a = -1, e = -1;
                if (valid) {
                    const int p = tl.parent[gid];
                    const int pl = p < 0 ? -1 : (int)(p - td.begin);
                    if (pl >= base) a = pl - base; else e = pl;
                    if (pl >= 0 && pl < base) atomicAdd(expect + pl / kWave, 1);
                    load_local<false>(pose, gid, 0, 0, m);
                } else {
                    aff_identity(m);
                }
                wave_inblock_scan(m, a, e, lane);
                const bool need = valid && e >= 0;
                const int fb = need ? (e / kWave) : 0;
                bool done = !__any(need);
                for (int spin = 0; !done && spin < tl.spin_limit; ++spin) {
                    const int ok = need ? __hip_atomic_load(flags + fb, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP)
                                        : 1;
                    done = __all(ok);
                    if (!done) __builtin_amdgcn_s_sleep(1);
                }
                if (!done) note_status(tl.status, kStatusWaitTimeout);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (need) {
                    float g[12];
                    aff_load(Gs + 3 * e, g);
                    aff_mul_left(g, m);
                }
                if (valid) aff_store(Gs + 3 * jl, m);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (lane == 0)
                    __hip_atomic_store(flags + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        } else {
            // Checkpoint mode: local transforms first (Gs as scratch) ...
            for (int jl = threadIdx.x; jl < n; jl += WAVES * kWave) {
                const int64_t gid = td.begin + jl;
                const int p = tl.parent[gid];
                const int pl = p < 0 ? -1 : (int)(p - td.begin);
                if (pl >= 0 && pl / kWave != jl / kWave) atomicAdd(expect + pl / kWave, 1);
                float m[12];
                load_local<false>(pose, gid, 0, 0, m);
                aff_store(Gs + 3 * jl, m);
            }
            __syncthreads();
            // ... then each joint multiplies the local transforms up to its
            // nearest checkpointed ancestor (at most ckpt_k - 1 of them) and
            // that ancestor's stored transform; results staged in Ds.
            for (int jl = threadIdx.x; jl < n; jl += WAVES * kWave) {
                const int64_t gid = td.begin + jl;
                float m[12];
                if (bwd.level[gid] % bwd.ckpt_k == 0) {
                    aff_load(reinterpret_cast<const float4 *>(bwd.ckpt) + 3 * gid, m);
                } else {
                    aff_load(Gs + 3 * jl, m);
                    int p = tl.parent[gid];
                    while (p >= 0) {
                        float g[12];
                        if (bwd.level[p] % bwd.ckpt_k == 0) {
                            aff_load(reinterpret_cast<const float4 *>(bwd.ckpt) + 3 * (int64_t)p, g);
                            aff_mul_left(g, m);
                            break;
                        }
                        aff_load(Gs + 3 * (int)(p - td.begin), g);
                        aff_mul_left(g, m);
                        p = tl.parent[p];
                    }
                }
                aff_store(Ds + 3 * jl, m);
            }
            __syncthreads();
            for (int i = threadIdx.x; i < 3 * n; i += WAVES * kWave) {
                Gs[i] = Ds[i];
                Ds[i] = zero4;
            }
        }
        __syncthreads();

        // ---- reverse sweep over the blocks ------------------------------------
        for (int idx = wave; idx < nblk; idx += WAVES) {
            const int b = nblk - 1 - idx;
            const int base = b * kWave;
            const int jl = base + lane;
            const bool valid = jl < n;
            const int64_t gid = td.begin + jl;
            // this block's inputs are fetched before the wait for the later
            // blocks' pushes, so their latency overlaps it
            float M[12], S[12];
            float4 q = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            float sx = 1.0f, sy = 1.0f, sz = 1.0f;
            int pl = -1, a = -1;
            if (valid) {
                const int p = tl.parent[gid];
                pl = p < 0 ? -1 : (int)(p - td.begin);
                if (pl >= base) a = pl - base;
                q = reinterpret_cast<const float4 *>(pose.quat)[gid];
                const float *t = pose.trans + 3 * gid;
                if (pose.scale) {
                    const float *sp = pose.scale + 3 * gid;
                    sx = sp[0]; sy = sp[1]; sz = sp[2];
                }
                aff_from_trs(q, t[0], t[1], t[2], sx, sy, sz, M);
                aff_load(reinterpret_cast<const float4 *>(bwd.grad_global) + 4 * gid, S);
            } else {
                aff_identity(M);
#pragma unroll
                for (int k = 0; k < 12; ++k) S[k] = 0.0f;
            }
            const int want = expect[b];
            bool done = want == 0;
            for (int spin = 0; !done && spin < tl.spin_limit; ++spin) {
                const int got = __hip_atomic_load(recv + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                done = __all(got >= want);
                if (!done) __builtin_amdgcn_s_sleep(1);
            }
            if (!done) note_status(tl.status, kStatusWaitTimeout);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (valid) {
                float acc[12];
                aff_load(Ds + 3 * jl, acc);
#pragma unroll
                for (int k = 0; k < 12; ++k) S[k] += acc[k];
                aff_store(Ds + 3 * jl, S);
            }

            // in-block reverse pointer jumping; colliding pushes resolved
            // with this block's owner words (touched by this wave only)
            Own[jl] = kOwnFree;
            wave_sync();
            if (a >= 0) own16_claim(Own + base + a, (uint16_t)lane);
            wave_sync();
#pragma unroll 1
            for (int r = 0; __any(a >= 0); ++r) {
                const bool act = a >= 0;
                const int tag = r << kOwn16Shift;
                bool lose = false;
                float c[12];
                if (act) {
                    adj_pull(S, M, c);
                    lose = own16_read(Own + base + a) != (tag | lane);
                    if (!lose) {
                        float acc[12];
                        aff_load(Ds + 3 * (base + a), acc);
#pragma unroll
                        for (int k = 0; k < 12; ++k) acc[k] += c[k];
                        aff_store(Ds + 3 * (base + a), acc);
                    }
                }
                wave_sync();
                if (lose) lds_atomic_add12(Ds + 3 * (base + a), c);
                // forward doubling: M_{r+1}(j) = M_r(a) M_r(j), a's values read
                // across lanes before any lane updates its own
                const int src = (act ? a : lane) << 2;
                float ma[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) ma[k] = lane_read(M[k], src);
                const int aa = __builtin_amdgcn_ds_bpermute(src, a);
                if (act) aff_mul_left(ma, M);
                const bool recv_r = valid && (own16_read(Own + jl) >> kOwn16Shift) == r;
                wave_sync();
                if (recv_r) aff_load(Ds + 3 * jl, S);
                if (act) {
                    a = aa;
                    if (a >= 0) own16_claim(Own + base + a, (uint16_t)(tag + (1 << kOwn16Shift) + lane));
                }
                wave_sync();
            }

            // heads push into their out-of-block parents and signal first;
            // the gradient stores follow, off the earlier blocks' critical path
            if (valid && pl >= 0 && pl < base) {
                const float *t = pose.trans + 3 * gid;  // the local transform again
                float L[12], c[12];
                aff_from_trs(q, t[0], t[1], t[2], sx, sy, sz, L);
                adj_pull(S, L, c);
                lds_atomic_add12(Ds + 3 * pl, c);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (valid && pl >= 0 && pl < base) atomicAdd(recv + pl / kWave, 1);
            if (valid) {
                float Ap[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
                if (pl >= 0) {
                    float g[12];
                    aff_load(Gs + 3 * pl, g);
                    Ap[0] = g[0]; Ap[1] = g[1]; Ap[2] = g[2];
                    Ap[3] = g[4]; Ap[4] = g[5]; Ap[5] = g[6];
                    Ap[6] = g[8]; Ap[7] = g[9]; Ap[8] = g[10];
                }
                write_grads(bwd, gid, S, Ap, q, sx, sy, sz);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the scan (tiled), recompute mode: tile-wide synchronous rounds.
//
// Every joint keeps, in registers, its partial adjoint S and the jump
// product M of the forward doubling; LDS holds M (for the jump targets), the
// adjoint accumulators and the jump pointers.  Round r moves S_r(j) (.) M_r(j)
// from each joint j to its jump target a = anc_r(j), while the forward
// doubling forms M_{r+1}(j) = M_r(a) M_r(j) and anc_{r+1}(j) = anc_r(a).
// After ceil(log2 L) rounds (L: deepest level of the tile, from the tile
// descriptor) S is the total adjoint X_j and M = G_j.  No block waits for
// later blocks' work, so the rounds of all joints of the tile run side by
// side.
//
// Several joints can push to one target in a round (the descendants of a
// at distance 2^r).  LDS float atomics are slow, so they are kept for
// those collisions only: every pusher first stores its id into the
// target's owner word (plain stores, one of them lands); the owner stores
// its contribution into the target's inbox with a plain store, the others
// add theirs with atomics one barrier later, and the target adds the inbox
// to the S it keeps in registers.  Owner words carry the round
// (id | r << 10), which also tells a joint whether anything arrived for it
// this round (an inbox is read only in a round that its owner wrote).
// LDS: M[cap][3] float4 | inboxes[cap][3] float4 | anc[cap] | owner[cap]
// ---------------------------------------------------------------------------
constexpr int kOwnerShift = 10;  // tile-local ids < 1024

__device__ __forceinline__ void owner_claim(int *w, int v)
{
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int owner_read(const int *w)
{
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// SEED: 0 dense dLoss/dG; 1 end-effector seeds from a given forward output;
// 2 end-effector seeds from the tile's own forward scan, run first with the
// forward kernel's blocks (one per wave: a tile has at most WAVES of them),
// G in the inbox array, which the seeds then overwrite in place.
constexpr int kSeedDense = 0, kSeedEffectors = 1, kSeedForward = 2;
constexpr int kOwnSeeded = -2;  // owner word of a seeded joint before the rounds

template <int WAVES, int SEED>
__global__ void __launch_bounds__(WAVES * kWave)
bwd_sync_kernel(TileLaunch tl, PoseArgs pose, BwdArgs bwd)
{
    constexpr bool EFF = SEED != kSeedDense;
    extern __shared__ float4 lds[];
    if (gated(tl.gate)) return;
    const int cap = tl.tile_cap;
    float4 *Ms = lds;
    float4 *In = lds + 3 * cap;
    int *Ac = reinterpret_cast<int *>(lds + 6 * cap);
    int *Own = Ac + cap;
    int *Fl = Own + cap;  // SEED 2: the forward's block flags [cap / 64]
    const int jl = threadIdx.x;

    for (int tile = blockIdx.x; tile < tl.num_tiles; tile += gridDim.x) {
        const TileDesc td = tl.tiles[tile];
        const bool live = jl < td.count;
        const int64_t gid = td.begin + jl;
        float M[12], S[12];
        int a = -1, p = -1;
        // the rotation and scale are kept for the gradient step: each pose
        // value is read from HBM once (streaming loads)
        float4 q = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
        float sx = 1.0f, sy = 1.0f, sz = 1.0f;
        if (live && SEED == kSeedForward) {
            // the pose comes with the tile's forward scan below
            p = tl.parent[gid];
            a = p < 0 ? -1 : (int)(p - td.begin);
#pragma unroll
            for (int k = 0; k < 12; ++k) S[k] = 0.0f;
            Ac[jl] = a;
            owner_claim(Own + jl, -1);
        } else if (live) {
            p = tl.parent[gid];
            a = p < 0 ? -1 : (int)(p - td.begin);
            const native_float4 qn =
                __builtin_nontemporal_load(reinterpret_cast<const native_float4 *>(pose.quat) + gid);
            q = make_float4(qn.x, qn.y, qn.z, qn.w);
            const float *t = pose.trans + 3 * gid;
            if (pose.scale) {
                const float *sp = pose.scale + 3 * gid;
                sx = __builtin_nontemporal_load(sp);
                sy = __builtin_nontemporal_load(sp + 1);
                sz = __builtin_nontemporal_load(sp + 2);
            }
            aff_from_trs(q, __builtin_nontemporal_load(t), __builtin_nontemporal_load(t + 1),
                         __builtin_nontemporal_load(t + 2), sx, sy, sz, M);
            if constexpr (EFF) {
#pragma unroll
                for (int k = 0; k < 12; ++k) S[k] = 0.0f;
                if constexpr (SEED == kSeedEffectors) aff_store(In + 3 * jl, S);
            } else {
                aff_load(reinterpret_cast<const float4 *>(bwd.grad_global) + 4 * gid, S);
            }
            aff_store(Ms + 3 * jl, M);
            Ac[jl] = a;
            owner_claim(Own + jl, -1);
        }
        if constexpr (SEED == kSeedForward) {
            // the tile's forward scan, G into the inbox array
            const int nblk = (td.count + kWave - 1) / kWave;
            if (jl < nblk) Fl[jl] = 0;
            __syncthreads();
            FwdShared sh{};
            sh.G = In;
            sh.flags = Fl;
            sh.status = tl.status;
            sh.spin = tl.spin_limit;
            OutArgs out{};
            out.global_out = bwd.eff_global_out;
            const int wave = jl / kWave;
            if (wave < nblk)
                fwd_block_keep(tl, pose, out, td, td.count, wave, sh, jl & (kWave - 1), Ms, q, sx, sy, sz);
            __syncthreads();
            if (live) aff_load(Ms + 3 * jl, M);
            // each effector's seed over its own row of G, marked in its owner word
            const int e1 = bwd.eff_tile[2 * tile + 1];
            for (int k = bwd.eff_tile[2 * tile] + jl; k < e1; k += WAVES * kWave) {
                const int le = (int)(bwd.eff_ids[k] - td.begin);
                const float *y = bwd.eff_target + 3 * (int64_t)bwd.eff_row[k];
                float g[12];
                aff_load(In + 3 * le, g);
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const float b = g[4 * r + 3];
                    g[4 * r] = g[4 * r + 1] = g[4 * r + 2] = 0.0f;
                    g[4 * r + 3] = 2.0f * (b - y[r]);
                }
                aff_store(In + 3 * le, g);
                owner_claim(Own + le, kOwnSeeded);
            }
            __syncthreads();
            if (live && owner_read(Own + jl) == kOwnSeeded) {
                aff_load(In + 3 * jl, S);
                owner_claim(Own + jl, -1);
            }
        }
        if constexpr (SEED == kSeedEffectors) {
            // the seeds of this tile's end effectors, through the inboxes
            __syncthreads();
            const int e1 = bwd.eff_tile[2 * tile + 1];
            for (int k = bwd.eff_tile[2 * tile] + jl; k < e1; k += WAVES * kWave) {
                const int64_t e = bwd.eff_ids[k];
                const float *g = bwd.eff_global + 16 * e;
                const float *y = bwd.eff_target + 3 * (int64_t)bwd.eff_row[k];
                float d[12];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    d[4 * r] = d[4 * r + 1] = d[4 * r + 2] = 0.0f;
                    d[4 * r + 3] = 2.0f * (g[4 * r + 3] - y[r]);
                }
                aff_store(In + 3 * (int)(e - td.begin), d);
            }
            __syncthreads();
            if (live) aff_load(In + 3 * jl, S);
        }
        __syncthreads();
        if (a >= 0) owner_claim(Own + a, jl);
        // the trip count comes from the tile descriptor, so it is uniform
        // across the workgroup and every wave meets the same barriers
        for (int r = 0; r < td.rounds; ++r) {
            __syncthreads();  // claims, products and pointers of round r
            const int tag = r << kOwnerShift;
            int aa = -1;
            bool lose = false;
            float c[12];
            if (a >= 0) {
                adj_pull(S, M, c);
                lose = owner_read(Own + a) != (tag | jl);
                if (!lose) aff_store(In + 3 * a, c);
                float ma[12];
                aff_load(Ms + 3 * a, ma);
                aa = Ac[a];
                aff_mul_left(ma, M);  // published after the barriers
            }
            __syncthreads();
            if (lose) lds_atomic_add12(In + 3 * a, c);
            const bool recv = live && (owner_read(Own + jl) >> kOwnerShift) == r;
            __syncthreads();
            if (recv) {
                float in[12];
                aff_load(In + 3 * jl, in);
#pragma unroll
                for (int k = 0; k < 12; ++k) S[k] += in[k];
            }
            if (a >= 0) {
                a = aa;
                aff_store(Ms + 3 * jl, M);
                Ac[jl] = a;
                if (a >= 0) owner_claim(Own + a, (tag + (1 << kOwnerShift)) | jl);
            }
        }
        __syncthreads();
        // M = G_j and S = X_j now; the gradients need the parent's G
        if (live) {
            float Ap[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
            if (p >= 0) {
                float g[12];
                aff_load(Ms + 3 * (int)(p - td.begin), g);
                Ap[0] = g[0]; Ap[1] = g[1]; Ap[2] = g[2];
                Ap[3] = g[4]; Ap[4] = g[5]; Ap[5] = g[6];
                Ap[6] = g[8]; Ap[7] = g[9]; Ap[8] = g[10];
            }
            write_grads(bwd, gid, S, Ap, q, sx, sy, sz);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Two-level adjoint (tiles of up to 1024 joints, one 64-joint block per
// wave, the anchor codes of the work-queue forward).
//
// With Y_j the sum over j's in-block descendants d of D_d pulled back
// through the in-block path products, and P_k the forward's in-block
// product of joint k (from the top of its in-block path), the inflow I_k
// of an anchor k (what its children in other blocks send) satisfies
//     I_k = sum over heads h with parent k of  Y_h (.) L_h
//         + sum over anchors k' whose nearest out-of-block ancestor is k
//           of  I_k' (.) P_k',
// and the total adjoint is the in-block reverse sum of the seeds D_j + I_j
// (I_j = 0 off the anchors).  Summed over a head's in-block subtree, the
// first term is sum_d D_d (.) P_d, so every seeded joint that is not an
// anchor sends D_d (.) P_d to its anchor at once, and every anchor, once
// its own inflow is complete, sends (D_k + I_k) (.) P_k: one composition
// per sender, anchors in decreasing order through LDS counters, no block
// waiting for another block's rounds.  Each block then runs one in-block
// reverse pointer jumping over D + I inside its wave (no workgroup
// barriers: pushes to in-block ancestors travel over per-wave lists built
// with LDS exchanges, values through the wave's own LDS slices).
// LDS per wave: stage [64][3] f4 (the block's G, then the scan's jump
// products), seeds [64][3] f4 (then the scan's contributions), jump
// targets, list heads and links [64] int each; per anchor slot: G, P, I [3]
// f4 each, flag, expected and received sends (int).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool any_nonzero12(const float v[12])
{
    bool nz = false;
#pragma unroll
    for (int k = 0; k < 12; ++k) nz |= v[k] != 0.0f;
    return nz;
}

// In-wave reverse pointer jumping over the block's in-block parents: S holds
// the seeds on entry and, on return, the sum over the lane's in-block
// descendants d of seed_d (.) (the local transforms on the path below the
// lane down to d).  L: the lane's local transform; a: in-block parent lane
// or -1.  Values move through the wave's own LDS slices with 16-byte
// accesses (cheaper than 4-byte cross-lane permutes for 12-float rows):
// Cx [64][3] the round's contributions, Mx [64][3] the jump products, and
// ints ax (jump targets), head and nxt (the list of the lanes that send to
// each lane in the round, built with LDS exchanges).
__device__ __forceinline__ void wave_reverse_scan(float S[12], const float L[12], int a, int lane, float4 *Cx,
                                                  float4 *Mx, int *ax, int *head, int *nxt)
{
    float M[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) M[k] = L[k];
    wave_sync();  // the caller's reads of these slices are done
    aff_store(Mx + 3 * lane, M);
    ax[lane] = a;
#pragma unroll 1
    for (int r = 0; r < 6; ++r) {  // an in-block path has at most 64 joints
        if (!__any(a >= 0)) break;
        const bool act = a >= 0;
        wave_sync();  // the previous round's reads are done
        if (act) {
            float c[12];
            adj_pull(S, M, c);  // what this lane sends to its 2^r-th in-block ancestor
            aff_store(Cx + 3 * lane, c);
        }
        head[lane] = -1;
        wave_sync();
        float ma[12];
        int aa = -1;
        if (act) {
            nxt[lane] = atomicExch(head + a, lane);  // the senders to a form a list
            aff_load(Mx + 3 * a, ma);
            aa = ax[a];
        }
        wave_sync();
        int h = head[lane];
        while (__any(h >= 0)) {
            if (h >= 0) {
                float cin[12];
                aff_load(Cx + 3 * h, cin);
#pragma unroll
                for (int k = 0; k < 12; ++k) S[k] += cin[k];
                h = nxt[h];
            }
        }
        // forward doubling: M_{r+1} = M_r(a) M_r, a <- a's ancestor; every
        // lane read round r's values before this point
        if (act) {
            aff_mul_left(ma, M);
            a = aa;
            aff_store(Mx + 3 * lane, M);
            ax[lane] = a;
        }
    }
}

// The stored TRS pose of joint gid (unit scale when the batch has none).
__device__ __forceinline__ void load_trs(const PoseArgs &pose, int64_t gid, float4 &q, float t[3], float s[3])
{
    const native_float4 qn = reinterpret_cast<const native_float4 *>(pose.quat)[gid];
    q = make_float4(qn.x, qn.y, qn.z, qn.w);
    const float *tp = pose.trans + 3 * gid;
    t[0] = tp[0];
    t[1] = tp[1];
    t[2] = tp[2];
    s[0] = s[1] = s[2] = 1.0f;
    if (pose.scale) {
        const float *sp = pose.scale + 3 * gid;
        s[0] = sp[0];
        s[1] = sp[1];
        s[2] = sp[2];
    }
}

// A wave takes BPW of the tile's blocks (wave, wave + WAVES, ...): with
// fewer, fuller waves a CU holds more tiles at once, so a batch of many
// tiles runs in fewer rounds of resident workgroups.  The forward handles
// the wave's blocks in increasing order and the anchor sends and reverse
// sums in decreasing order; forward waits only point to lower blocks and
// anchor waits only to higher ones, so the wave holding the lowest (resp.
// highest) unfinished block can always proceed.
template <int WAVES, int BPW, int SEED>
__global__ void __launch_bounds__(WAVES * kWave, 4)  // at most 128 VGPRs: four waves per SIMD
bwd_anchor_kernel(TileLaunch tl, PoseArgs pose, BwdArgs bwd)
{
    extern __shared__ float4 lds[];
    if (gated(tl.gate)) return;
    constexpr int T = WAVES * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int na = tl.max_anchors;
    float4 *stage = lds + wave * kWave * 3;                    // [WAVES][64][3]: a block's G, then jump products
    float4 *contrib = lds + (WAVES + wave) * kWave * 3;        // [WAVES][64][3]: the reverse scan's contributions
    float4 *AG = lds + WAVES * kWave * 6;
    float4 *AP = AG + 3 * na;
    float4 *AI = AP + 3 * na;
    int *aflag = reinterpret_cast<int *>(AI + 3 * na);
    int *expect = aflag + na;
    int *recv = expect + na;
    int *ax = recv + na + wave * kWave * 3;  // [WAVES][3][64]: jump targets, list heads, next
    int *head = ax + kWave;
    int *nxt = head + kWave;
    int *effk = recv + na + WAVES * kWave * 3;  // [tile_cap]: each joint's effector entry, or -1
    const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);

    for (int tile = blockIdx.x; tile < tl.num_tiles; tile += gridDim.x) {
        const TileDesc td = tl.tiles[tile];
        const int n = td.count;
        if (n == 0) continue;  // uniform: nothing to do, and no joint to read
        for (int i = threadIdx.x; i < na; i += T) {
            aflag[i] = 0;
            expect[i] = 0;
            recv[i] = 0;
        }
        for (int i = threadIdx.x; i < 3 * na; i += T) AI[i] = zero4;
        if constexpr (SEED != kSeedDense) {
            for (int i = threadIdx.x; i < n; i += T) effk[i] = -1;
            __syncthreads();
            const int e1 = bwd.eff_tile[2 * tile + 1];
            for (int k = bwd.eff_tile[2 * tile] + (int)threadIdx.x; k < e1; k += T)
                effk[(int)(bwd.eff_ids[k] - td.begin)] = k;
        }
        __syncthreads();

        // what each of the wave's blocks keeps from the forward for the
        // reverse: codes, the parent's rotation-scale block, the seed
        // (effector forms: its translation column); the reverse reads the
        // pose again (from the caches: the tile's poses were read just before)
        float Apb[BPW][9], Db[BPW][3];
        int ownb[BPW], eb[BPW], pab[BPW];

        // every block's codes and poses are loaded before the first scan
        int codeb[BPW];
        float4 qb[BPW];
        float tb[BPW][3], sb[BPW][3];
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int jl = (wave + b * WAVES) * kWave + lane;
            const int64_t gid = td.begin + min(jl, n - 1);  // past the tile: its last joint, not used
            codeb[b] = tl.code[gid];
            load_trs(pose, gid, qb[b], tb[b], sb[b]);
        }

        // ---- forward: the wave's blocks in increasing order (the queue
        // kernel's scheme); non-anchor seeded joints send D (.) P to their
        // anchor at once ----
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int base = (wave + b * WAVES) * kWave;
            ownb[b] = eb[b] = pab[b] = -1;
#pragma unroll
            for (int k = 0; k < 3; ++k) Db[b][k] = 0.0f;
            if (base >= n) continue;  // uniform across the wave
            const int jl = base + lane;
            const bool valid = jl < n;
            const int64_t gid = td.begin + jl;
            int a = -1, e = -1, own = -1, ps = -1;
            float m[12];
            if (valid) {
                const int code = codeb[b];
                const int ref = code & (kQInBlock - 1);
                if (code & kQInBlock) a = ref; else e = ps = ref - 1;
                own = (code >> kQOwnShift) - 1;
                aff_from_trs(qb[b], tb[b][0], tb[b][1], tb[b][2], sb[b][0], sb[b][1], sb[b][2], m);
            } else {
                aff_identity(m);
            }
            pab[b] = a;  // in-block parent lane, for the reverse sums
            wave_inblock_scan_lds(m, a, e, lane, stage, ax);
            float P[12];  // the in-block product from the top of the joint's in-block path
#pragma unroll
            for (int k = 0; k < 12; ++k) P[k] = m[k];
            if (own >= 0 && e >= 0) atomicAdd(expect + e, 1);  // k will send to its own anchor
            wait_slot(aflag, valid ? e : -1, tl.status, tl.spin_limit);
            if (valid && e >= 0) {
                float g[12];
                aff_load(AG + 3 * e, g);
                aff_mul_left(g, m);
            }
            if (own >= 0) {
                aff_store(AG + 3 * own, m);
                aff_store(AP + 3 * own, P);
            }
            aff_store(stage + 3 * lane, m);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (own >= 0) __hip_atomic_store(aflag + own, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            wave_sync();  // the block's G is staged
            if constexpr (SEED == kSeedForward) {
                if (bwd.eff_global_out) {
                    OutArgs out{};
                    out.global_out = bwd.eff_global_out;
                    store_rows<1>(out, stage, td.begin + base, 0, 1, n - base, lane);
                }
            }
            // the parent's global rotation-scale block, for the gradients (an
            // out-of-block parent is the anchor waited for above)
            float *Ap = Apb[b];
            Ap[0] = 1.0f; Ap[1] = 0.0f; Ap[2] = 0.0f;
            Ap[3] = 0.0f; Ap[4] = 1.0f; Ap[5] = 0.0f;
            Ap[6] = 0.0f; Ap[7] = 0.0f; Ap[8] = 1.0f;
            if (valid && (pab[b] >= 0 || ps >= 0)) {
                float g[12];
                aff_load(pab[b] >= 0 ? stage + 3 * pab[b] : AG + 3 * ps, g);
                Ap[0] = g[0]; Ap[1] = g[1]; Ap[2] = g[2];
                Ap[3] = g[4]; Ap[4] = g[5]; Ap[5] = g[6];
                Ap[6] = g[8]; Ap[7] = g[9]; Ap[8] = g[10];
            }
            // the seed
            float D[12];
            if constexpr (SEED == kSeedDense) {
                if (valid) {
                    const float4 *gg = reinterpret_cast<const float4 *>(bwd.grad_global) + 4 * gid;
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const float4 v = gg[r];
                        D[4 * r] = v.x;
                        D[4 * r + 1] = v.y;
                        D[4 * r + 2] = v.z;
                        D[4 * r + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 12; ++k) D[k] = 0.0f;
                }
            } else {
                const int k = valid ? effk[jl] : -1;
                if (k >= 0) {
                    const float *y = bwd.eff_target + 3 * (int64_t)bwd.eff_row[k];
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        float bt;
                        if constexpr (SEED == kSeedForward) bt = m[4 * r + 3];
                        else bt = bwd.eff_global[16 * gid + 4 * r + 3];
                        Db[b][r] = 2.0f * (bt - y[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    D[4 * r] = D[4 * r + 1] = D[4 * r + 2] = 0.0f;
                    D[4 * r + 3] = Db[b][r];
                }
            }
            if (own < 0 && e >= 0 && any_nonzero12(D)) {
                float c[12];
                adj_pull(D, P, c);
                lds_atomic_add12(AI + 3 * e, c);
            }
            ownb[b] = own;
            eb[b] = e;
        }
        __syncthreads();  // every direct send is in, every expected send counted

        // ---- the wave's blocks in decreasing order: once all its children
        // anchors have sent, an anchor sends (D_k + I_k) (.) P_k to its own
        // anchor; then the block's in-block reverse sums over D + I and its
        // gradients ----
#pragma unroll
        for (int b = BPW - 1; b >= 0; --b) {
            const int base = (wave + b * WAVES) * kWave;
            if (base >= n) continue;  // uniform across the wave
            const int jl = base + lane;
            const bool valid = jl < n;
            const int64_t gid = td.begin + jl;
            const int own = ownb[b], e = eb[b];
            // the pose again, issued before the wait for the anchor inflows
            float4 q = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            float t[3] = {0.0f, 0.0f, 0.0f}, sc[3] = {1.0f, 1.0f, 1.0f};
            if (valid) load_trs(pose, gid, q, t, sc);
            float X[12];
            if constexpr (SEED == kSeedDense) {
                if (valid) {
                    const float4 *gg = reinterpret_cast<const float4 *>(bwd.grad_global) + 4 * gid;
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const float4 v = gg[r];
                        X[4 * r] = v.x;
                        X[4 * r + 1] = v.y;
                        X[4 * r + 2] = v.z;
                        X[4 * r + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 12; ++k) X[k] = 0.0f;
                }
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    X[4 * r] = X[4 * r + 1] = X[4 * r + 2] = 0.0f;
                    X[4 * r + 3] = Db[b][r];
                }
            }
            {
                const bool need = own >= 0;
                const int want = need ? expect[own] : 0;
                bool done = !__any(need && want > 0);
                for (int spin = 0; !done && spin < tl.spin_limit; ++spin) {
                    const int got =
                        need ? __hip_atomic_load(recv + own, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0;
                    done = __all(got >= want);
                    if (!done) __builtin_amdgcn_s_sleep(1);
                }
                if (!done) note_status(tl.status, kStatusWaitTimeout);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (need) {
                    float I[12];
                    aff_load(AI + 3 * own, I);  // complete: every sender has arrived
#pragma unroll
                    for (int k = 0; k < 12; ++k) X[k] += I[k];
                    if (e >= 0) {
                        float Pk[12], c[12];
                        aff_load(AP + 3 * own, Pk);
                        adj_pull(X, Pk, c);
                        lds_atomic_add12(AI + 3 * e, c);
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                        atomicAdd(recv + e, 1);
                    }
                }
            }
            // X = D + I; the in-block reverse sums over it (the stage and
            // contribution slices carry the scan's jump products and sends)
            float L[12];
            if (valid) aff_from_trs(q, t[0], t[1], t[2], sc[0], sc[1], sc[2], L);
            else aff_identity(L);
            if (__any(any_nonzero12(X))) wave_reverse_scan(X, L, pab[b], lane, contrib, stage, ax, head, nxt);
            if (valid) write_grads(bwd, gid, X, Apb[b], q, sc[0], sc[1], sc[2]);
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

template <int W, int BPW>
const void *anchor_kernel_of(int seed)
{
    if (seed == kSeedForward) return reinterpret_cast<const void *>(bwd_anchor_kernel<W, BPW, kSeedForward>);
    if (seed == kSeedEffectors) return reinterpret_cast<const void *>(bwd_anchor_kernel<W, BPW, kSeedEffectors>);
    return reinterpret_cast<const void *>(bwd_anchor_kernel<W, BPW, kSeedDense>);
}

// ---------------------------------------------------------------------------
// Reverse mode of the Simulation step.  One workgroup per character; each
// thread takes joints, recomputes the two clips' key interpolations and the
// blend, and applies the reverse rules
//   q = v / |v|:            vbar = (qbar - q (q . qbar)) / |v|,
//   y = (1 - x) a + x b:    abar = (1 - x) ybar, bbar = x ybar, xbar = ybar . (b - a),
// with the arc signs and the key index held fixed.  Key gradients are
// summed over all readers with float atomics; the time and weight
// gradients are reduced over the character's joints in the workgroup.
// ---------------------------------------------------------------------------
constexpr int kSampleBwdThreads = 256;

__device__ __forceinline__ float4 unit_back(float4 q, float inv_norm, float4 qbar)
{
    const float d = q.x * qbar.x + q.y * qbar.y + q.z * qbar.z + q.w * qbar.w;
    return make_float4((qbar.x - q.x * d) * inv_norm, (qbar.y - q.y * d) * inv_norm,
                       (qbar.z - q.z * d) * inv_norm, (qbar.w - q.w * d) * inv_norm);
}

__device__ __forceinline__ void fma4(float4 &acc, float s, float4 v)
{
    acc.x = fmaf(s, v.x, acc.x);
    acc.y = fmaf(s, v.y, acc.y);
    acc.z = fmaf(s, v.z, acc.z);
    acc.w = fmaf(s, v.w, acc.w);
}

__device__ __forceinline__ float block_sum(float v, float *red)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x / kWave;
    __syncthreads();  // red is reused by consecutive calls
    if ((threadIdx.x & (kWave - 1)) == 0) red[wave] = v;
    __syncthreads();
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < kSampleBwdThreads / kWave; ++k) t += red[k];
    return t;
}

// Reverse mode of joint j of character c (its frame valid): the adjoints of
// the two clips' unnormalised key blends (vb[X]) and the factors of dLoss/dt
// in their translation lerps (tw[X]), the arc signs (sX[X]), and the joint's
// terms of dLoss/dalpha and dLoss/dw.
struct JointRev {
    float4 vb[2];
    float tw[2], sX[2];
    float gt[3];
    float g_alpha, g_w;
};

__device__ __forceinline__ void joint_reverse(const PoseArgs &P, const SampleBwdArgs &A, int64_t gid, int j,
                                              const int clip[2], int k0, int k1, float alpha, float w, JointRev &o)
{
    const int K = P.num_keys, J = P.joints_per_clip;
    const float4 *kq = reinterpret_cast<const float4 *>(P.key_quat);
    const float *kt = P.key_trans;
    const float uw = 1.0f - w, ua = 1.0f - alpha;
    const float4 gq = reinterpret_cast<const float4 *>(A.grad_quat)[gid];
    o.gt[0] = A.grad_trans[3 * gid];
    o.gt[1] = A.grad_trans[3 * gid + 1];
    o.gt[2] = A.grad_trans[3 * gid + 2];
    float4 qX[2], a[2], b[2];
    float invX[2], t0[2][3], t1[2][3];
#pragma unroll
    for (int X = 0; X < 2; ++X) {
        const int64_t r0 = ((int64_t)clip[X] * K + k0) * J + j, r1 = ((int64_t)clip[X] * K + k1) * J + j;
        a[X] = kq[r0];
        b[X] = kq[r1];
        double d = (double)a[X].x * (double)b[X].x;
        d = d + (double)a[X].y * (double)b[X].y;
        d = d + (double)a[X].z * (double)b[X].z;
        d = d + (double)a[X].w * (double)b[X].w;
        o.sX[X] = d < 0.0 ? -1.0f : 1.0f;
        const float v = alpha * o.sX[X];
        const float4 r = make_float4(fmaf(ua, a[X].x, v * b[X].x), fmaf(ua, a[X].y, v * b[X].y),
                                     fmaf(ua, a[X].z, v * b[X].z), fmaf(ua, a[X].w, v * b[X].w));
        invX[X] = 1.0f / sqrtf(fmaf(r.x, r.x, fmaf(r.y, r.y, fmaf(r.z, r.z, r.w * r.w))));
        qX[X] = make_float4(r.x * invX[X], r.y * invX[X], r.z * invX[X], r.w * invX[X]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            t0[X][i] = kt[3 * r0 + i];
            t1[X][i] = kt[3 * r1 + i];
        }
    }
    const float dab = qX[0].x * qX[1].x + qX[0].y * qX[1].y + qX[0].z * qX[1].z + qX[0].w * qX[1].w;
    const float sb = dab < 0.0f ? -1.0f : 1.0f;
    const float4 u = make_float4(fmaf(uw, qX[0].x, w * sb * qX[1].x), fmaf(uw, qX[0].y, w * sb * qX[1].y),
                                 fmaf(uw, qX[0].z, w * sb * qX[1].z), fmaf(uw, qX[0].w, w * sb * qX[1].w));
    const float inv_u = 1.0f / sqrtf(u.x * u.x + u.y * u.y + u.z * u.z + u.w * u.w);
    const float4 q = make_float4(u.x * inv_u, u.y * inv_u, u.z * inv_u, u.w * inv_u);
    const float4 ub = unit_back(q, inv_u, gq);
    // blend weight: d/dw of (1-w) qA + w sb qB and of (1-w) tA + w tB
    o.g_w = ub.x * (sb * qX[1].x - qX[0].x) + ub.y * (sb * qX[1].y - qX[0].y) + ub.z * (sb * qX[1].z - qX[0].z) +
            ub.w * (sb * qX[1].w - qX[0].w);
    o.g_alpha = 0.0f;
#pragma unroll
    for (int X = 0; X < 2; ++X) {
        const float sw = X == 0 ? uw : w * sb;  // the clip's factor in u
        o.tw[X] = X == 0 ? uw : w;              // and in t
        o.vb[X] = unit_back(qX[X], invX[X], make_float4(sw * ub.x, sw * ub.y, sw * ub.z, sw * ub.w));
#pragma unroll
        for (int i = 0; i < 3; ++i) o.g_alpha += o.tw[X] * o.gt[i] * (t1[X][i] - t0[X][i]);
        o.g_alpha += o.vb[X].x * (o.sX[X] * b[X].x - a[X].x) + o.vb[X].y * (o.sX[X] * b[X].y - a[X].y) +
                     o.vb[X].z * (o.sX[X] * b[X].z - a[X].z) + o.vb[X].w * (o.sX[X] * b[X].w - a[X].w);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float tA = fmaf(ua, t0[0][i], alpha * t1[0][i]), tB = fmaf(ua, t0[1][i], alpha * t1[1][i]);
        o.g_w += o.gt[i] * (tB - tA);
    }
}

// Time and weight gradients: one workgroup per character, the joints'
// terms reduced in the workgroup.
__global__ void __launch_bounds__(kSampleBwdThreads)
sample_bwd_kernel(PoseArgs P, SampleBwdArgs A)
{
    __shared__ float red[kSampleBwdThreads / kWave];
    for (int c = blockIdx.x; c < A.C; c += gridDim.x) {
        const int64_t base = P.offsets[c];
        const int n = (int)(P.offsets[c + 1] - base);
        int k0, k1;
        float alpha;
        const bool ok = sample_frame(P, c, k0, k1, alpha);  // uniform in the workgroup
        const int clip[2] = {P.clip_a[c], P.clip_b[c]};
        const float w = P.weight[c];
        float g_alpha = 0.0f, g_w = 0.0f;
        for (int j = ok ? (int)threadIdx.x : n; j < n; j += kSampleBwdThreads) {
            JointRev o;
            joint_reverse(P, A, base + j, j, clip, k0, k1, alpha, w, o);
            g_alpha += o.g_alpha;
            g_w += o.g_w;
            if (A.ws) {
                A.ws[2 * (base + j)] = o.vb[0];
                A.ws[2 * (base + j) + 1] = o.vb[1];
            }
        }
        const float sum_a = block_sum(g_alpha, red);
        const float sum_w = block_sum(g_w, red);
        if (threadIdx.x == 0) {
            const float nan = __int_as_float(0x7fc00000);
            if (A.grad_time) A.grad_time[c] = ok ? P.fps * sum_a : nan;
            if (A.grad_weight) A.grad_weight[c] = ok ? sum_w : nan;
        }
    }
}

// Keyframe gradients by gathering instead of scattering: one workgroup per
// (clip, key) block.  Its readers are the characters that read the block as
// clip A or B, at key k0 or k1 of their frame: up to four entries each.
// Every thread counts the entries of its characters (scan_key_readers) in
// one pass over the clip parameters; a workgroup prefix sum
// gives each thread the place of its first entry, and a second pass writes
// the entries there, so the list is in a fixed order (by thread, then by
// character) whatever the scheduling.  Each thread then sums, for its
// joints, every reader's contribution -- (1 - alpha) or alpha s times the
// adjoint of the key blend, (1 - alpha) or alpha times the weighted dLoss/dt
// -- and writes its key rows once.  No atomics on the gradients, no zero
// fill (blocks nobody reads get zeros), and the sums are bitwise
// reproducible.  A block with more readers than the list holds takes them
// in rounds of kKeyReaders.
constexpr int kKeyReaders = 1024;

// Calls emit(entry, alpha) for each entry of character c in block (clip,
// key), in a fixed order; entry = 4 c + 2 X + role (X: clip A or B, role:
// key k0 or k1 of the character's frame), alpha the frame's fraction.
template <typename Emit>
__device__ __forceinline__ void key_block_entries(const PoseArgs &P, int c, int clip, int key, Emit &&emit)
{
    const int cl[2] = {P.clip_a[c], P.clip_b[c]};
    if (cl[0] != clip && cl[1] != clip) return;  // most characters: two loads
    int k0, k1;
    float alpha;
    if (!sample_frame(P, c, k0, k1, alpha)) return;
#pragma unroll
    for (int X = 0; X < 2; ++X) {
        if (cl[X] != clip) continue;
        if (k0 == key) emit(4 * c + 2 * X, alpha);
        if (k1 == key) emit(4 * c + 2 * X + 1, alpha);
    }
}

// This thread's readers of block (clip, key), in a fixed order: characters
// c = seg + 256 k + thread, segment by segment.  The clip ids of a
// segment's 16 characters are loaded together (no branch between the
// loads, so one memory latency per segment), then only the characters
// that use the clip are examined.
constexpr int kScanPer = 16;

template <typename Emit>
__device__ __forceinline__ void scan_key_readers(const PoseArgs &P, int C, int clip, int key, Emit &&emit)
{
    for (int seg = 0; seg < C; seg += kSampleBwdThreads * kScanPer) {
        const int c0 = seg + (int)threadIdx.x;
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int c = c0 + k * kSampleBwdThreads;
            const int ca = c < C ? P.clip_a[c] : -1;
            const int cb = c < C ? P.clip_b[c] : -1;
            m |= (uint32_t)((ca == clip) | (cb == clip)) << k;
        }
        while (m) {
            const int k = __builtin_ctz(m);
            m &= m - 1;
            key_block_entries(P, c0 + k * kSampleBwdThreads, clip, key, emit);
        }
    }
}

// The block's reader list in LDS.  With the workspace (WS) each entry also
// carries the reader's first joint, joint count and its two factors, the
// key-blend factor ((1 - alpha), or alpha, which the k1 role multiplies by
// the arc sign) and the translation factor ((1 - alpha) or alpha, times
// 1 - w or w), so that summing an entry takes two loads.
template <bool WS>
struct KeyList {
    int entry[kKeyReaders];
    int64_t base[WS ? kKeyReaders : 1];
    int count[WS ? kKeyReaders : 1];
    float fq[WS ? kKeyReaders : 1], ft[WS ? kKeyReaders : 1];
};

// Entries [r0, r0 + kKeyReaders) of the block's list, this thread's share
// (its entries are numbered from `start` in the order of scan_key_readers).
template <bool WS>
__device__ __forceinline__ void fill_key_list(const PoseArgs &P, int C, int clip, int key, int start, int r0,
                                              KeyList<WS> &L)
{
    int idx = start;
    const int r1 = r0 + kKeyReaders;
    scan_key_readers(P, C, clip, key, [&](int e, float alpha) {
        if (idx >= r0 && idx < r1) {
            const int i = idx - r0;
            L.entry[i] = e;
            if constexpr (WS) {
                const int c = e >> 2, X = (e >> 1) & 1, role = e & 1;
                const int64_t b = P.offsets[c];
                L.base[i] = b;
                L.count[i] = (int)(P.offsets[c + 1] - b);
                const float w = P.weight[c];
                const float a = role == 0 ? 1.0f - alpha : alpha;
                L.fq[i] = a;
                L.ft[i] = a * (X ? w : 1.0f - w);
            }
        }
        ++idx;
    });
}

template <bool WS>
__global__ void __launch_bounds__(kSampleBwdThreads)
sample_bwd_keys_kernel(PoseArgs P, SampleBwdArgs A)
{
    __shared__ KeyList<WS> L;
    __shared__ int wsum[kSampleBwdThreads / kWave];
    const int K = P.num_keys, J = P.joints_per_clip;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t nblocks = (int64_t)P.num_clips * K;
    for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const int clip = (int)(blk / K), key = (int)(blk % K);
        // this thread's entries, then their place in the list
        int mine = 0;
        scan_key_readers(P, A.C, clip, key, [&](int, float) { ++mine; });
        int incl = mine;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        int start = incl - mine, total = 0;
#pragma unroll
        for (int w = 0; w < kSampleBwdThreads / kWave; ++w) {
            if (w < wave) start += wsum[w];
            total += wsum[w];
        }
        const bool once = total <= kKeyReaders;  // uniform in the workgroup
        if (once) fill_key_list<WS>(P, A.C, clip, key, start, 0, L);
        __syncthreads();
        for (int j0 = 0; j0 < J; j0 += kSampleBwdThreads) {
            const int j = j0 + (int)threadIdx.x;
            float4 gkq = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            float gkt[3] = {0.0f, 0.0f, 0.0f};
            // a reader of this block as its k1 has k0 = key - 1: the arc sign
            // of its clip blend depends on the two key rows alone (the same
            // fp64 decision as the reverse step's)
            float s1 = 1.0f;
            if (WS && j < J) {
                const float4 *kq = reinterpret_cast<const float4 *>(P.key_quat);
                const float4 a = kq[((int64_t)clip * K + (key == 0 ? K - 1 : key - 1)) * J + j];
                const float4 b = kq[((int64_t)clip * K + key) * J + j];
                double d = (double)a.x * (double)b.x;
                d = d + (double)a.y * (double)b.y;
                d = d + (double)a.z * (double)b.z;
                d = d + (double)a.w * (double)b.w;
                s1 = d < 0.0 ? -1.0f : 1.0f;
            }
            for (int r0 = 0; r0 < total; r0 += kKeyReaders) {
                if (!once) {
                    __syncthreads();  // the previous round's entries are read
                    fill_key_list<WS>(P, A.C, clip, key, start, r0, L);
                    __syncthreads();
                }
                const int nr = min(kKeyReaders, total - r0);
                for (int e = 0; e < nr; ++e) {
                    const int ent = L.entry[e];
                    const int X = (ent >> 1) & 1, role = ent & 1;
                    if constexpr (WS) {
                        // the reader's reverse step, stored by the time/weight kernel
                        if (j >= L.count[e]) continue;  // the character has no joint j
                        const int64_t g = L.base[e] + j;
                        const float4 vb = A.ws[2 * g + X];
                        const float f = role == 0 ? L.fq[e] : L.fq[e] * s1;
                        const float ft = L.ft[e];
                        fma4(gkq, f, vb);
#pragma unroll
                        for (int i = 0; i < 3; ++i) gkt[i] = fmaf(ft, A.grad_trans[3 * g + i], gkt[i]);
                    } else {
                        const int rc = ent >> 2;
                        const int64_t base = P.offsets[rc];
                        if (j >= (int)(P.offsets[rc + 1] - base)) continue;  // the character has no joint j
                        int k0, k1;
                        float alpha;
                        sample_frame(P, rc, k0, k1, alpha);
                        const int cl[2] = {P.clip_a[rc], P.clip_b[rc]};
                        JointRev o;
                        joint_reverse(P, A, base + j, j, cl, k0, k1, alpha, P.weight[rc], o);
                        // X is only known at run time: select, not index (no scratch)
                        const float4 vb = X ? o.vb[1] : o.vb[0];
                        const float sx = X ? o.sX[1] : o.sX[0], tw = X ? o.tw[1] : o.tw[0];
                        const float f = role == 0 ? 1.0f - alpha : alpha * sx;
                        const float ft = (role == 0 ? 1.0f - alpha : alpha) * tw;
                        fma4(gkq, f, vb);
#pragma unroll
                        for (int i = 0; i < 3; ++i) gkt[i] = fmaf(ft, o.gt[i], gkt[i]);
                    }
                }
            }
            if (j < J) {
                const int64_t row = blk * J + j;
                if (A.grad_key_quat) reinterpret_cast<float4 *>(A.grad_key_quat)[row] = gkq;
                if (A.grad_key_trans) {
                    A.grad_key_trans[3 * row] = gkt[0];
                    A.grad_key_trans[3 * row + 1] = gkt[1];
                    A.grad_key_trans[3 * row + 2] = gkt[2];
                }
            }
        }
        __syncthreads();  // the list and the wave sums are rewritten by the next block
    }
}

// ---------------------------------------------------------------------------
// Vertex skinning: each mesh vertex moves by a weighted blend of the skin
// matrices S_j of up to four joints of its character.
//   linear blend: p' = (sum_i w_i S_{j_i}) [p, 1];
//   dual quaternions (Kavan, Collins, Zara, O'Sullivan 2008): every rigid
//     S_j as a unit dual quaternion (q_r, q_d = 1/2 (t, 0) q_r); the
//     influences summed with w_i times the sign of q_r,i . q_r,0, divided by
//     the norm of the real part, applied as a rigid transform.
// One workgroup per character: its skin matrices (or their dual
// quaternions, converted once per joint) are staged in LDS, then every
// thread takes vertices; the mesh arrays are shared by the characters of
// a kind and stay in cache.
// LDS: [max_joints][3] float4 (linear) or [max_joints][2] float4 (dual)
// ---------------------------------------------------------------------------
constexpr int kSkinThreads = 256;

// Quaternion (x, y, z, w) of the rotation block of a rigid transform given
// by its rows (Shepperd's method: divide by the largest of the four
// 4 q_k^2 that the diagonal determines), then the dual part 1/2 (t, 0) q.
__device__ __forceinline__ void rigid_to_dual_quat(float4 r0, float4 r1, float4 r2, float4 &qr, float4 &qd)
{
    const float m00 = r0.x, m01 = r0.y, m02 = r0.z, m10 = r1.x, m11 = r1.y, m12 = r1.z;
    const float m20 = r2.x, m21 = r2.y, m22 = r2.z;
    const float tr = m00 + m11 + m22;
    float x, y, z, w;
    if (tr > 0.0f) {
        const float s = 2.0f * sqrtf(tr + 1.0f);
        const float is = 1.0f / s;
        w = 0.25f * s;
        x = (m21 - m12) * is;
        y = (m02 - m20) * is;
        z = (m10 - m01) * is;
    } else if (m00 > m11 && m00 > m22) {
        const float s = 2.0f * sqrtf(1.0f + m00 - m11 - m22);
        const float is = 1.0f / s;
        w = (m21 - m12) * is;
        x = 0.25f * s;
        y = (m01 + m10) * is;
        z = (m02 + m20) * is;
    } else if (m11 > m22) {
        const float s = 2.0f * sqrtf(1.0f + m11 - m00 - m22);
        const float is = 1.0f / s;
        w = (m02 - m20) * is;
        x = (m01 + m10) * is;
        y = 0.25f * s;
        z = (m12 + m21) * is;
    } else {
        const float s = 2.0f * sqrtf(1.0f + m22 - m00 - m11);
        const float is = 1.0f / s;
        w = (m10 - m01) * is;
        x = (m02 + m20) * is;
        y = (m12 + m21) * is;
        z = 0.25f * s;
    }
    const float n = 1.0f / sqrtf(x * x + y * y + z * z + w * w);
    x *= n; y *= n; z *= n; w *= n;
    qr = make_float4(x, y, z, w);
    const float tx = r0.w, ty = r1.w, tz = r2.w;
    qd = make_float4(0.5f * (tx * w + ty * z - tz * y), 0.5f * (-tx * z + ty * w + tz * x),
                     0.5f * (tx * y - ty * x + tz * w), -0.5f * (tx * x + ty * y + tz * z));
}

__device__ __forceinline__ float dot4(float4 a, float4 b) { return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w; }

// Dual quaternion blend of four influences (real part at X[STRIDE j], dual
// part at X[STRIDE j + 1]) applied to p: signs against influence 0, the
// normalised blend, then p + 2 r x (r x p + w p) + 2 (w_r d - w_d r + r x d).
template <int STRIDE>
__device__ __forceinline__ void dq_blend_apply(const float4 *X, const int jk[4], const float wk[4], float px, float py,
                                               float pz, float &ox, float &oy, float &oz)
{
    const float4 q0 = X[STRIDE * jk[0]];
    float4 br = make_float4(0.0f, 0.0f, 0.0f, 0.0f), bd = br;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 q = X[STRIDE * jk[k]], d = X[STRIDE * jk[k] + 1];
        const float s = dot4(q, q0) < 0.0f ? -wk[k] : wk[k];
        fma4(br, s, q);
        fma4(bd, s, d);
    }
    const float inv = 1.0f / sqrtf(dot4(br, br));
    const float rx = br.x * inv, ry = br.y * inv, rz = br.z * inv, rw = br.w * inv;
    const float dx = bd.x * inv, dy = bd.y * inv, dz = bd.z * inv, dw = bd.w * inv;
    const float cx = ry * pz - rz * py + rw * px;
    const float cy = rz * px - rx * pz + rw * py;
    const float cz = rx * py - ry * px + rw * pz;
    const float tx = 2.0f * (rw * dx - dw * rx + ry * dz - rz * dy);
    const float ty = 2.0f * (rw * dy - dw * ry + rz * dx - rx * dz);
    const float tz = 2.0f * (rw * dz - dw * rz + rx * dy - ry * dx);
    ox = px + 2.0f * (ry * cz - rz * cy) + tx;
    oy = py + 2.0f * (rz * cx - rx * cz) + ty;
    oz = pz + 2.0f * (rx * cy - ry * cx) + tz;
}

__device__ __forceinline__ void dq_apply2(const float4 *X, const int jk[4], const float wk[4], float px, float py,
                                          float pz, float &ox, float &oy, float &oz)
{
    dq_blend_apply<2>(X, jk, wk, px, py, pz, ox, oy, oz);
}

__device__ __forceinline__ void dq_apply(const float4 *X, const int jk[4], const float wk[4], float px, float py,
                                         float pz, float &ox, float &oy, float &oz)
{
    dq_blend_apply<3>(X, jk, wk, px, py, pz, ox, oy, oz);
}

template <int METHOD>
__global__ void __launch_bounds__(kSkinThreads)
vertex_skin_kernel(VertexLaunch vl, const float4 *skin, float *out)
{
    extern __shared__ float4 lds[];
    for (int c = blockIdx.x; c < vl.C; c += gridDim.x) {
        const int64_t v0 = vl.voff[c];
        const int nv = (int)(vl.voff[c + 1] - v0);
        if (nv == 0) continue;  // uniform across the workgroup
        const int64_t j0 = vl.offsets[c];
        const int nj = (int)(vl.offsets[c + 1] - j0);
        for (int j = threadIdx.x; j < nj; j += kSkinThreads) {
            const float4 *S = skin + 4 * (j0 + j);
            const float4 r0 = S[0], r1 = S[1], r2 = S[2];
            if constexpr (METHOD == 0) {
                lds[3 * j] = r0;
                lds[3 * j + 1] = r1;
                lds[3 * j + 2] = r2;
            } else {
                float4 qr, qd;
                rigid_to_dual_quat(r0, r1, r2, qr, qd);
                lds[2 * j] = qr;
                lds[2 * j + 1] = qd;
            }
        }
        __syncthreads();
        const int64_t m0 = vl.mfirst[c];
        for (int v = threadIdx.x; v < nv; v += kSkinThreads) {
            const int64_t m = m0 + v;
            const float px = vl.pos[3 * m], py = vl.pos[3 * m + 1], pz = vl.pos[3 * m + 2];
            const int4 ji = reinterpret_cast<const int4 *>(vl.joints)[m];
            const float4 wt = reinterpret_cast<const float4 *>(vl.weights)[m];
            const int jk[4] = {ji.x, ji.y, ji.z, ji.w};
            const float wk[4] = {wt.x, wt.y, wt.z, wt.w};
            float ox, oy, oz;
            if constexpr (METHOD == 0) {
                float4 a0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), a1 = a0, a2 = a0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    fma4(a0, wk[k], lds[3 * jk[k]]);
                    fma4(a1, wk[k], lds[3 * jk[k] + 1]);
                    fma4(a2, wk[k], lds[3 * jk[k] + 2]);
                }
                ox = fmaf(a0.x, px, fmaf(a0.y, py, fmaf(a0.z, pz, a0.w)));
                oy = fmaf(a1.x, px, fmaf(a1.y, py, fmaf(a1.z, pz, a1.w)));
                oz = fmaf(a2.x, px, fmaf(a2.y, py, fmaf(a2.z, pz, a2.w)));
            } else {
                // real parts staged at lds[2 j], dual parts at lds[2 j + 1]
                dq_apply2(lds, jk, wk, px, py, pz, ox, oy, oz);
            }
            float *dst = out + 3 * (v0 + v);
            dst[0] = ox;
            dst[1] = oy;
            dst[2] = oz;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Scan, skin matrices and vertex skinning in one pass per tile: the tile's
// blocks run the scan as in fwd_tile_kernel (G in LDS, no outputs); then
// each thread turns its joints' G_j into S_j = G_j B_j^-1 in place (or into
// S_j's unit dual quaternion), optionally writing S; then the threads take
// the vertices of the tile's characters and blend the staged transforms as
// vertex_skin_kernel does.  S never has to leave the chip.
// LDS: that of fwd_tile_kernel with the character map, plus the tile's
// vertex starts [cap + 1].
// ---------------------------------------------------------------------------
template <int WAVES, bool SAMPLE, bool INST, int METHOD>
__global__ void __launch_bounds__(WAVES * kWave)
fwd_vertex_kernel(TileLaunch tl, PoseArgs pose, OutArgs out, VertexLaunch vl, float *vout)
{
    extern __shared__ float4 lds[];
    if (gated(tl.gate)) return;
    constexpr int T = WAVES * kWave;
    const int cap = tl.tile_cap;
    const int nbk = cap >> 6;
    FwdShared sh;
    sh.G = lds;
    sh.part = lds + 3 * cap;
    sh.flags = reinterpret_cast<int *>(sh.part + 3 * nbk);
    sh.pflag = sh.flags + nbk;
    sh.panc = sh.pflag + nbk;
    sh.cstart = sh.panc + nbk;
    sh.status = tl.status;
    sh.spin = tl.spin_limit;
    int *cstart = sh.cstart;
    int *vstart = cstart + cap + 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const OutArgs none{};

    for (int tile = blockIdx.x; tile < tl.num_tiles; tile += gridDim.x) {
        const TileDesc td = tl.tiles[tile];
        const int n = td.count;
        const int nblk = (n + kWave - 1) / kWave;
        for (int i = threadIdx.x; i < nblk; i += T) {
            sh.flags[i] = 0;
            sh.pflag[i] = 0;
        }
        const int64_t vbase = vl.voff[td.first_char];
        for (int i = threadIdx.x; i <= td.num_chars; i += T) {
            cstart[i] = (int)(pose.offsets[td.first_char + i] - td.begin);
            vstart[i] = (int)(vl.voff[td.first_char + i] - vbase);
        }
        __syncthreads();
        for (int b = wave; b < nblk; b += WAVES) fwd_block<SAMPLE, INST>(tl, pose, none, td, n, b, sh, lane);
        __syncthreads();
        // G -> S (or its dual quaternion), in place
        for (int jl = threadIdx.x; jl < n; jl += T) {
            int64_t bidx = td.begin + jl;
            if constexpr (INST) {
                const int c = tile_char_of(cstart, td.num_chars, jl);
                bidx = tl.char_skel[td.first_char + c] + (jl - cstart[c]);
            }
            float m[12];
            aff_load(sh.G + 3 * jl, m);
            const float4 *B = reinterpret_cast<const float4 *>(out.inv_bind) + 4 * bidx;
            const float4 b0 = B[0], b1 = B[1], b2 = B[2], b3 = B[3];
            float4 S[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const float g0 = m[4 * r], g1 = m[4 * r + 1], g2 = m[4 * r + 2], g3 = m[4 * r + 3];
                S[r] = make_float4(fmaf(g0, b0.x, fmaf(g1, b1.x, fmaf(g2, b2.x, g3 * b3.x))),
                                   fmaf(g0, b0.y, fmaf(g1, b1.y, fmaf(g2, b2.y, g3 * b3.y))),
                                   fmaf(g0, b0.z, fmaf(g1, b1.z, fmaf(g2, b2.z, g3 * b3.z))),
                                   fmaf(g0, b0.w, fmaf(g1, b1.w, fmaf(g2, b2.w, g3 * b3.w))));
            }
            if (out.skin_out) {
                float4 *Sd = reinterpret_cast<float4 *>(out.skin_out) + 4 * (td.begin + jl);
                Sd[0] = S[0];
                Sd[1] = S[1];
                Sd[2] = S[2];
                Sd[3] = b3;
            }
            if constexpr (METHOD == 0) {
                sh.G[3 * jl] = S[0];
                sh.G[3 * jl + 1] = S[1];
                sh.G[3 * jl + 2] = S[2];
            } else {
                float4 qr, qd;
                rigid_to_dual_quat(S[0], S[1], S[2], qr, qd);
                sh.G[3 * jl] = qr;
                sh.G[3 * jl + 1] = qd;
            }
        }
        __syncthreads();
        const int nv = vstart[td.num_chars];
        for (int v = threadIdx.x; v < nv; v += T) {
            const int c = tile_char_of(vstart, td.num_chars, v);
            const int64_t mrow = vl.mfirst[td.first_char + c] + (v - vstart[c]);
            const float4 *X = sh.G + 3 * cstart[c];
            const float px = vl.pos[3 * mrow], py = vl.pos[3 * mrow + 1], pz = vl.pos[3 * mrow + 2];
            const int4 ji = reinterpret_cast<const int4 *>(vl.joints)[mrow];
            const float4 wt = reinterpret_cast<const float4 *>(vl.weights)[mrow];
            const int jk[4] = {ji.x, ji.y, ji.z, ji.w};
            const float wk[4] = {wt.x, wt.y, wt.z, wt.w};
            float ox, oy, oz;
            if constexpr (METHOD == 0) {
                float4 a0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), a1 = a0, a2 = a0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    fma4(a0, wk[k], X[3 * jk[k]]);
                    fma4(a1, wk[k], X[3 * jk[k] + 1]);
                    fma4(a2, wk[k], X[3 * jk[k] + 2]);
                }
                ox = fmaf(a0.x, px, fmaf(a0.y, py, fmaf(a0.z, pz, a0.w)));
                oy = fmaf(a1.x, px, fmaf(a1.y, py, fmaf(a1.z, pz, a1.w)));
                oz = fmaf(a2.x, px, fmaf(a2.y, py, fmaf(a2.z, pz, a2.w)));
            } else {
                dq_apply(X, jk, wk, px, py, pz, ox, oy, oz);
            }
            float *dst = vout + 3 * (vbase + v);
            dst[0] = ox;
            dst[1] = oy;
            dst[2] = oz;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// End-effector loss sum_e |b_e - y_e|^2 (b_e the translation of G_e): its
// gradient with respect to G is 2 (b_e - y_e) in column 3 of rows 0-2 of
// each effector's G and zero elsewhere.  One thread per effector writes
// those three values; the caller keeps the other entries zero.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
effector_grad_kernel(int64_t n, int64_t ne, const int64_t *eff, const float *G, const float *target, float *grad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int64_t e = eff[i];
    if (e < 0 || e >= n) return;  // ids outside the batch are skipped
#pragma unroll
    for (int r = 0; r < 3; ++r) grad[16 * e + 4 * r + 3] = 2.0f * (G[16 * e + 4 * r + 3] - target[3 * i + r]);
}

// ---------------------------------------------------------------------------
// Multipass path.
// ---------------------------------------------------------------------------
constexpr int kMPWaves = 4;

template <bool SAMPLE>
__global__ void __launch_bounds__(kMPWaves * kWave)
mp_local_kernel(MPLaunch ml, PoseArgs pose)
{
    __shared__ float4 slice[kMPWaves * kWave * 3];
    __shared__ int xs[2 * kMPWaves * kWave];
    if (gated(ml.gate)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int w = blockIdx.x * kMPWaves + wv;
    if (w >= ml.num_blocks) return;  // whole waves leave together
    const MPBlock bd = ml.blocks[w];
    const bool valid = lane < bd.count;
    const int64_t gid = bd.gbegin + lane;
    const int64_t cid = bd.cbegin + lane;
    float m[12];
    int a = -1, e = -1;
    if (valid) {
        const int p = ml.parent[gid];
        if (p >= 0) {
            const int64_t off = (int64_t)p - bd.gbegin;
            if (off >= 0) a = (int)off; else e = (int)(off + bd.cbegin);
        }
        int lj = 0;
        if constexpr (SAMPLE) lj = (int)(gid - pose.offsets[bd.chr]);
        load_local<SAMPLE>(pose, gid, bd.chr, lj, m);
    } else {
        aff_identity(m);
    }
    wave_inblock_scan_lds(m, a, e, lane, slice + wv * kWave * 3, xs + 2 * wv * kWave, 3,
                          xs + (2 * wv + 1) * kWave);
    // only the anchors' in-block products leave the kernel (the output pass
    // recomputes the others from the poses): anchor i starts the rounds from
    // its phase-1 product and the anchor index of its own anchor
    const int ai = valid ? ml.aself[cid] : -1;
    if (ai >= 0) {
        aff_store(ml.A1 + 3 * ai, m);
        ml.E1[ai] = ml.janc[cid];
    }
}

// One pointer-jumping round over the anchors (Eq. 2 applied to the anchor
// tree): product with the target's product, target's target.
__global__ void __launch_bounds__(256)
mp_anchor_round_kernel(int32_t na, const float4 *Pin, const int32_t *Ein, float4 *Pout, int32_t *Eout)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= na) return;
    float m[12];
    aff_load(Pin + 3 * i, m);
    int e = Ein[i];
    if (e >= 0) {
        float g[12];
        aff_load(Pin + 3 * e, g);
        aff_mul_left(g, m);
        e = Ein[e];
    }
    aff_store(Pout + 3 * i, m);
    Eout[i] = e;
}

// The same rounds for segments of at most kAnchorSegCap consecutive anchors
// that no anchor points out of (the plan cuts them, at character
// boundaries or inside a long chain's anchor list where allowed): one
// workgroup per segment, one thread per anchor, the products and pointers
// in LDS, read phase and write phase of each round separated by barriers.
// The trip count is the plan's, uniform across the workgroup.
__global__ void __launch_bounds__(kAnchorSegCap)
mp_anchor_seg_kernel(const int32_t *aseg, int32_t rounds, const float4 *Pin, const int32_t *Ein, float4 *Pout,
                     int32_t *Eout)
{
    __shared__ float4 M[kAnchorSegCap * 3];
    __shared__ int32_t E[kAnchorSegCap];
    const int s = aseg[blockIdx.x], n = aseg[blockIdx.x + 1] - s;
    const int t = threadIdx.x;
    const bool live = t < n;
    float m[12];
    int e = -1;
    if (live) {
        aff_load(Pin + 3 * (s + t), m);
        const int g = Ein[s + t];
        e = (g >= s && g < s + n) ? g - s : -1;  // the plan's cuts keep every pointer inside
        aff_store(M + 3 * t, m);
        E[t] = e;
    }
    for (int r = 0; r < rounds; ++r) {
        __syncthreads();  // products and pointers of round r
        float g[12];
        int ee = -1;
        if (e >= 0) {
            aff_load(M + 3 * e, g);
            ee = E[e];
        }
        __syncthreads();  // every read of round r done
        if (e >= 0) {
            aff_mul_left(g, m);
            e = ee;
            aff_store(M + 3 * t, m);
            E[t] = e;
        }
    }
    if (live) {
        aff_store(Pout + 3 * (s + t), m);
        Eout[s + t] = e < 0 ? -1 : s + e;
    }
}

// Final pass: the in-block scan again from the poses (cheaper than storing
// and re-reading every partial), then G_j = G_anchor P_j, one composition
// per joint.  Writes the outputs -- G through the wave's LDS slice as
// coalesced 16-byte rows -- or (Gc non-NULL) the compact global transforms
// the adjoint reads.  LDS: [kMPWaves][64][3] float4.
template <bool SAMPLE>
__global__ void __launch_bounds__(kMPWaves * kWave)
mp_out_kernel(MPLaunch ml, PoseArgs pose, const float4 *AP, OutArgs out, float4 *Gc)
{
    __shared__ float4 stage[kMPWaves * kWave * 3];
    __shared__ int xs[2 * kMPWaves * kWave];
    if (gated(ml.gate)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int w = blockIdx.x * kMPWaves + wv;
    if (w >= ml.num_blocks) return;  // whole waves leave together; no workgroup barriers here
    const MPBlock bd = ml.blocks[w];
    const bool valid = lane < bd.count;
    const int64_t gid = bd.gbegin + lane;
    const int64_t cid = bd.cbegin + lane;
    float m[12];
    int a = -1, e = -1;
    if (valid) {
        const int p = ml.parent[gid];
        if (p >= 0) {
            const int64_t off = (int64_t)p - bd.gbegin;
            if (off >= 0) a = (int)off; else e = (int)(off + bd.cbegin);
        }
        int lj = 0;
        if constexpr (SAMPLE) lj = (int)(gid - pose.offsets[bd.chr]);
        load_local<SAMPLE>(pose, gid, bd.chr, lj, m);
    } else {
        aff_identity(m);
    }
    wave_inblock_scan_lds(m, a, e, lane, stage + wv * kWave * 3, xs + 2 * wv * kWave, 3, xs + (2 * wv + 1) * kWave);
    const int an = valid ? ml.janc[cid] : -1;
    if (an >= 0) {
        float g[12];
        aff_load(AP + 3 * an, g);
        aff_mul_left(g, m);
    }
    if (Gc) {
        if (valid) aff_store(Gc + 3 * cid, m);
        return;
    }
    if (out.global_out) {
        float4 *st = stage + wv * kWave * 3;
        aff_store(st + 3 * lane, m);
        wave_sync();
        const float4 bottom = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
        float4 *dst = reinterpret_cast<float4 *>(out.global_out) + 4 * bd.gbegin;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = lane + kWave * k;
            if ((c >> 2) < bd.count) {
                const int r = c & 3;
                store_stream(dst + c, r == 3 ? bottom : st[3 * (c >> 2) + r]);
            }
        }
    }
    if (valid) write_skin_and_ckpt(out, gid, gid, m);
}

// ---------------------------------------------------------------------------
// One pass for chain characters beyond a tile (every joint's parent the
// previous joint): a reduce-then-scan over superblocks of up to 4096
// consecutive joints of one chain (64 of the plan's 64-joint blocks), one
// superblock per workgroup at a time.  Each of the 16 waves takes two
// segments of 128 consecutive joints (wave w: segments w and w + 16), two
// per lane: the lane multiplies its two local transforms in order
// (Q_0 = L_0, Q_1 = L_0 L_1), the wave scans the lanes' products (pointer
// jumping over lane - 1, six rounds for 128 joints) and keeps the
// inclusive products in its LDS slice.  The segments' totals meet in LDS,
// where one wave scans them (lane = segment), publishes the superblock's
// total, looks back over the chain's earlier superblocks (lane =
// superblock: the nearest final transform and the totals after it,
// composed by the same scan) for the transform entering the superblock,
// publishes its final transform, and leaves in LDS the transform entering
// each segment E; then G = (E W) Q_i, W the product of the segment's
// earlier lanes, staged in the slice a segment at a time and stored as
// coalesced rows.  Each pose is read once.  Workgroups take superblocks in
// increasing order (a static stride; the launch holds no more workgroups
// than are resident at once), and a superblock publishes its total before
// it looks back, so the look-backs only wait for publications that need no
// waiting.  Values cross workgroups as tagged agent-scope words (coherent
// across the XCDs' L2s).
// ---------------------------------------------------------------------------
// A superblock's record: 12 words, each a 32-bit value with its tag in the
// high half, (epoch << 2) | kind (kind 1 the superblock's total, 2 the
// final transform; the epoch numbers the calls, so that a word of an
// earlier call never reads as published), written as single 8-byte
// agent-scope stores (coherent across the XCDs' L2s).  A word read is then
// both the value and its own flag: a reader takes the record when all 12
// tags agree and carry this call's epoch, and reads again while they do
// not (not yet published, or a total being overwritten by the final
// transform), so no store has to complete before another.
// m: the 12 values in LDS (an affine row block); lane k < 12 stores word k.
__device__ __forceinline__ void publish12(uint64_t *rec, const float4 *m, unsigned epoch, unsigned kind, int lane)
{
    if (lane < 12) {
        const float v = reinterpret_cast<const float *>(m)[lane];
        const uint64_t tag = ((uint64_t)(epoch & 0x3fffffffu) << 2) | kind;
        __hip_atomic_store(rec + lane, (tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The record's kind when its 12 tags agree and carry this call's epoch,
// else 0; the values in m.
__device__ __forceinline__ unsigned read12(uint64_t *rec, unsigned epoch, float m[12])
{
    uint64_t w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = __hip_atomic_load(rec + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned tag = (unsigned)(w[0] >> 32);
    bool same = (tag >> 2) == (epoch & 0x3fffffffu);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        same &= (unsigned)(w[k] >> 32) == tag;
        m[k] = __uint_as_float((unsigned)w[k]);
    }
    return same ? (tag & 3u) : 0u;
}

// Wave 0 of the workgroup resolving superblock s: T [nt][3] the segments'
// totals (in; T[nt - 1] then holds the superblock's total), E [nt][3] the
// transforms entering the segments (out; first the products of the earlier
// segments' totals); X, xi the wave's scan slice.
__device__ __forceinline__ void resolve_superblock(const ChainLaunch &cl, unsigned epoch, int s, const ChainSB &sb,
                                                   int nt, int lane, float4 *T, float4 *E, float4 *X, int *xi)
{
    // inclusive products of the segments' totals, in chain order (lane = segment)
    const bool in = lane < nt;
    {
        float x[12];
        if (in) aff_load(T + 3 * lane, x);
        else aff_identity(x);
        int a = in && lane > 0 ? lane - 1 : -1, e = -1;
        wave_inblock_scan_lds(x, a, e, lane, X, xi);
        aff_store(X + 3 * lane, x);
        wave_sync();
        if (lane == nt - 1) aff_store(T + 3 * lane, x);  // the superblock's total
        if (in) {
            if (lane > 0) aff_load(X + 3 * (lane - 1), x);
            else aff_identity(x);
            aff_store(E + 3 * lane, x);
        }
        wave_sync();  // the slice is free; T and E written
    }
    float acc[12];  // the transform entering the superblock
    aff_identity(acc);
    uint64_t *rec = cl.recs + 12 * (int64_t)s;
    float4 *tot = T + 3 * (nt - 1);
    if (s == sb.chain_first) {
        publish12(rec, tot, epoch, 2, lane);
    } else {
        publish12(rec, tot, epoch, 1, lane);
        // look back, 64 superblocks at a time (lane k: superblock base - k)
        for (int base = s - 1;; base -= kWave) {
            const int q = base - lane;
            const bool lv = q >= sb.chain_first;
            unsigned st = 2;
            float v[12];
            for (int spin = 0;; ++spin) {
                if (lv) st = read12(cl.recs + 12 * (int64_t)q, epoch, v);
                if (__all(st > 0)) break;
                if (spin >= cl.spin_limit) {
                    note_status(cl.status, kStatusWaitTimeout);
                    st = 2;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            // the nearest final transform (the chain's first superblock always is one)
            const unsigned long long fin = __ballot(lv && st == 2);
            const int kf = fin ? __ffsll((long long)fin) - 1 : -1;
            const int nv = min(kWave, base - sb.chain_first + 1);  // lanes inside the chain
            if (!(lane < nv && (kf < 0 || lane <= kf))) aff_identity(v);
            const int top = kf >= 0 ? kf : nv - 1;  // the window's earliest superblock taken
            int pa = lane < top ? lane + 1 : -1, pe = -1;
            wave_inblock_scan_lds(v, pa, pe, lane, X, xi);  // lane 0: v(top) ... v(0)
            if (lane == 0) aff_store(X, v);
            wave_sync();
            float w[12];
            aff_load(X, w);
            wave_sync();
            aff_mul_left(w, acc);  // acc = w acc
            if (kf >= 0) break;    // uniform
        }
        float inc[12];
        aff_load(tot, inc);
        aff_mul_left(acc, inc);
        wave_sync();  // every lane has read the total
        if (lane == 0) aff_store(tot, inc);
        wave_sync();
        publish12(rec, tot, epoch, 2, lane);
    }
    if (in) {
        float x[12];
        aff_load(E + 3 * lane, x);
        aff_mul_left(acc, x);  // the transform entering segment `lane`
        aff_store(E + 3 * lane, x);
    }
}

constexpr int kChainPerLane = 2;                          // consecutive joints per lane
constexpr int kChainSeg = kChainPerLane * kWave;          // joints per segment
constexpr int kChainSegPerWave = 2;                       // a wave's segments: wave, wave + 16
constexpr int kChainSegs = kChainWaves * kChainSegPerWave;  // segments per superblock
static_assert(kChainSegs * kChainSeg == kChainSBBlocks * 64, "the segments cover a superblock");
static_assert(kChainSegs <= kWave, "the segments' totals are scanned by one wave");

// LDS of the chain kernel, in float4: per wave a slice of one segment's
// rows (the two segments' lane products after the forward half, then the
// staging of the rows), wave 0's parked products, the resolving wave's
// scan slice, the segments' totals and entering transforms, and the scans'
// int words (16 waves and the resolving wave).
constexpr int kChainSlice = kChainSeg * 3;
constexpr size_t kChainLdsF4 = (size_t)kChainWaves * kChainSlice + kChainSegPerWave * kChainPerLane * kWave * 3 +
                               kWave * 3 + 2 * kChainSegs * 3 + (kChainWaves + 1) * kWave / 4;
constexpr size_t kChainLdsBytes = kChainLdsF4 * sizeof(float4);

// The local transform of joint gid, the pose read with plain loads (a
// lane's joints share cache lines with its neighbours').
template <bool SAMPLE>
__device__ __forceinline__ void load_local_lane(const PoseArgs &P, int64_t gid, int chr, int lj, float m[12])
{
    if constexpr (SAMPLE) {
        float4 q;
        float tx, ty, tz;
        sample_pose(P, chr, lj, q, tx, ty, tz);
        aff_from_trs(q, tx, ty, tz, 1.0f, 1.0f, 1.0f, m);
    } else {
        const float4 q = reinterpret_cast<const float4 *>(P.quat)[gid];
        const float *t = P.trans + 3 * gid;
        float sx = 1.0f, sy = 1.0f, sz = 1.0f;
        if (P.scale) {
            const float *sp = P.scale + 3 * gid;
            sx = sp[0];
            sy = sp[1];
            sz = sp[2];
        }
        aff_from_trs(q, t[0], t[1], t[2], sx, sy, sz, m);
    }
}

template <bool SAMPLE>
__global__ void __launch_bounds__(kChainWaves * kWave, 4)  // at most 128 VGPRs: four waves per SIMD
mp_chain_kernel(ChainLaunch cl, PoseArgs pose, OutArgs out)
{
    extern __shared__ float4 lds[];
    if (gated(cl.gate)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform: branches on it stay scalar
    float4 *X = lds + wv * kChainSlice;                     // the wave's slice
    float4 *PS = lds + kChainWaves * kChainSlice;           // wave 0's products while it resolves
    float4 *R = PS + kChainSegPerWave * kChainPerLane * kWave * 3;  // the resolving wave's scan slice
    float4 *T = R + kWave * 3;                              // [segments][3] totals
    float4 *E = T + kChainSegs * 3;                         // [segments][3] entering transforms
    int *xs = reinterpret_cast<int *>(E + kChainSegs * 3);  // [17][64]
    int *xi = xs + wv * kWave;
    const float4 bottom = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    const int j0 = kChainPerLane * lane;  // the lane's first joint in a segment
    // this call's epoch: the last call's plus one (the last workgroup of a
    // call stores it, after every workgroup has read it)
    const unsigned epoch = (unsigned)__builtin_amdgcn_readfirstlane(
        (int)(__hip_atomic_load(cl.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u));  // uniform
    for (int s = blockIdx.x; s < cl.num_sb; s += gridDim.x) {  // uniform per workgroup
        const ChainSB sb = cl.sbs[s];
        const ChainBlock b0 = cl.blocks[sb.first];
        const int cnt = kWave * (sb.nblk - 1) + cl.blocks[sb.first + sb.nblk - 1].count;
        const int nt = (cnt + kChainSeg - 1) / kChainSeg;  // segments holding joints
        int lj0 = 0;
        if constexpr (SAMPLE) lj0 = (int)(b0.gbegin - pose.offsets[b0.chr]);
        float Q[kChainSegPerWave][kChainPerLane][12];
        wave_sync();  // the previous superblock's reads of the slice are done
#pragma unroll
        for (int h = 0; h < kChainSegPerWave; ++h) {
            const int gs = wv + kChainWaves * h;               // the segment
            const int n = min(kChainSeg, cnt - gs * kChainSeg);  // its joints (<= 0: none)
            if (n <= 0) break;                                 // uniform per wave
            const int sj = gs * kChainSeg + j0;                // the lane's first joint in the superblock
#pragma unroll
            for (int i = 0; i < kChainPerLane; ++i) {
                if (j0 + i < n) load_local_lane<SAMPLE>(pose, b0.gbegin + sj + i, b0.chr, lj0 + sj + i, Q[h][i]);
                else aff_identity(Q[h][i]);
                if (i > 0) aff_mul_left(Q[h][i - 1], Q[h][i]);  // Q_i = L_0 ... L_i
            }
            float x[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) x[k] = Q[h][kChainPerLane - 1][k];
            int a = lane > 0 && j0 < n ? lane - 1 : -1, e = -1;
            float4 *Xh = X + h * (kWave * 3);
            wave_inblock_scan_lds(x, a, e, lane, Xh, xi);  // x: the product over lanes 0..lane
            aff_store(Xh + 3 * lane, x);                   // read back once E is known
            if (lane == (n - 1) / kChainPerLane) aff_store(T + 3 * gs, x);  // the segment's total
        }
        __syncthreads();  // every segment's total
        if (wv == 0) {
            // the products wait in LDS (registers for the resolution)
#pragma unroll
            for (int h = 0; h < kChainSegPerWave; ++h)
#pragma unroll
                for (int i = 0; i < kChainPerLane; ++i)
                    aff_store(PS + 3 * (kWave * (kChainPerLane * h + i) + lane), Q[h][i]);
            resolve_superblock(cl, epoch, s, sb, nt, lane, T, E, R, xs + kChainWaves * kWave);
#pragma unroll
            for (int h = 0; h < kChainSegPerWave; ++h)
#pragma unroll
                for (int i = 0; i < kChainPerLane; ++i)
                    aff_load(PS + 3 * (kWave * (kChainPerLane * h + i) + lane), Q[h][i]);
        }
        __syncthreads();  // the transforms entering the segments
        // G = (E W) Q_i, W the product over the segment's earlier lanes
#pragma unroll
        for (int h = 0; h < kChainSegPerWave; ++h) {
            const int gs = wv + kChainWaves * h;
            if (gs * kChainSeg >= cnt) break;
            float W[12], F[12];
            if (lane > 0) aff_load(X + h * (kWave * 3) + 3 * (lane - 1), W);
            else aff_identity(W);
            aff_load(E + 3 * gs, F);
#pragma unroll
            for (int k = 0; k < 12; ++k)  // the same for every lane: scalar registers
                F[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(F[k])));
            aff_mul_left(F, W);
#pragma unroll
            for (int i = 0; i < kChainPerLane; ++i) aff_mul_left(W, Q[h][i]);
        }
#pragma unroll
        for (int h = 0; h < kChainSegPerWave; ++h) {
            const int gs = wv + kChainWaves * h;
            const int n = min(kChainSeg, cnt - gs * kChainSeg);
            if (n <= 0) break;
            const int64_t gb = b0.gbegin + gs * kChainSeg;  // the segment's first joint
            if (out.global_out) {
                wave_sync();  // the slice's last readers are done
#pragma unroll
                for (int i = 0; i < kChainPerLane; ++i) aff_store(X + 3 * (j0 + i), Q[h][i]);
                wave_sync();
                // lane: row r of joints lane / 4 + 16 k
                const int r = lane & 3;
                float4 *dst = reinterpret_cast<float4 *>(out.global_out) + 4 * gb + lane;
                const float4 *src = X + 3 * (lane >> 2) + min(r, 2);
#pragma unroll 1
                for (int jr = lane >> 2; jr < n; jr += kWave / 4) {
                    const float4 v = *src;
                    store_stream(dst, r == 3 ? bottom : v);
                    dst += kWave;
                    src += 3 * (kWave / 4);
                }
            }
#pragma unroll
            for (int i = 0; i < kChainPerLane; ++i)
                if (j0 + i < n) write_skin_and_ckpt(out, gb + j0 + i, gb + j0 + i, Q[h][i]);
        }
        // no barrier here: a wave's next writes are to its own slice, to T
        // (read by the resolution before the second barrier) and, for wave
        // 0, to PS, R and its words; E is rewritten only after every wave
        // has reached the next superblock's first barrier.  A wave that is
        // done storing starts the next superblock's loads.
    }
    // the last workgroup to finish (every workgroup has read the epoch)
    // stores it for the next call and resets the count
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned done = __hip_atomic_fetch_add(cl.epoch + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(cl.epoch + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(cl.epoch, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint on the multipass path (characters larger than an adjoint tile).
//
// With D the incoming dLoss/dG, the in-block adjoint Z = R_B(Y) of a block
// sums Y over in-block subtrees (Z_j = Y_j + sum over in-block children c of
// Z_c (.) L_c).  A head h (parent outside the block, an anchor e) hands
// X_h (.) L_h to e.  Writing U_e for what anchor e receives from all its
// out-of-block children, and P_a for an anchor's phase-1 product (the local
// transforms from its own anchor e_a, exclusive, down to a):
//     U_e = B_e + sum over anchors a with e_a = e of  U_a (.) P_a,
//     B_e = sum over heads h with parent e of  R_B(D)_h (.) L_h,
// the adjoint recursion again, on the anchor tree with P as the locals; and
// X = R_B(D + U) block by block.  So: R_B(D) with heads pushing into B
// (global float atomics, one push per head), reverse pointer jumping over
// the anchors, then R_B(D + U) and the gradients.
// ---------------------------------------------------------------------------
// R_B for one 64-joint block held by one wave: S in (Y_j), S out (Z_j).
// a: lane of the in-block parent, or -1.  Reverse pointer jumping over the
// in-block ancestors with the forward doubling alongside, collisions
// resolved with owner words as in the tiled adjoint.  Wave-private LDS:
// Ms[64][3], Sa[64][3] float4, Ac[64], Own[64] int.
__device__ __forceinline__ void wave_block_reverse(float S[12], const float L[12], int a, int lane, float4 *Ms,
                                                   float4 *Sa, int *Ac, int *Own)
{
    float M[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) M[k] = L[k];
    aff_store(Ms + 3 * lane, M);
    aff_store(Sa + 3 * lane, S);
    Ac[lane] = a;
    owner_claim(Own + lane, -1);
    wave_sync();
    if (a >= 0) owner_claim(Own + a, lane);
    wave_sync();
#pragma unroll 1
    for (int r = 0; r < 6; ++r) {
        if (!__any(a >= 0)) break;
        const int tag = r << kOwnerShift;
        int aa = -1;
        bool lose = false;
        float c[12];
        if (a >= 0) {
            adj_pull(S, M, c);
            lose = owner_read(Own + a) != (tag | lane);
            if (!lose) {
                float acc[12];
                aff_load(Sa + 3 * a, acc);
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] += c[k];
                aff_store(Sa + 3 * a, acc);
            }
            float ma[12];
            aff_load(Ms + 3 * a, ma);
            aa = Ac[a];
            aff_mul_left(ma, M);
        }
        wave_sync();
        if (lose) lds_atomic_add12(Sa + 3 * a, c);
        const bool recv = (owner_read(Own + lane) >> kOwnerShift) == r;
        wave_sync();
        if (recv) aff_load(Sa + 3 * lane, S);
        if (a >= 0) {
            a = aa;
            aff_store(Ms + 3 * lane, M);
            Ac[lane] = a;
            if (a >= 0) owner_claim(Own + a, (tag + (1 << kOwnerShift)) | lane);
        }
        wave_sync();
    }
}

constexpr int kRevWaveFloat4 = 64 * 6 + 32;  // per-wave LDS of wave_block_reverse, in float4

// FINAL = false: R_B(D) per block, heads push into the anchor accumulators
// Sanc.  FINAL = true: R_B(D + U) with U = Sanc injected at the anchors, then
// the gradients (the parent's global transform from the compact table G).
template <bool FINAL>
__global__ void __launch_bounds__(kMPWaves * kWave)
mpr_block_kernel(MPLaunch ml, PoseArgs pose, BwdArgs bwd, float4 *Sanc)
{
    extern __shared__ float4 lds[];
    if (gated(ml.gate)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    float4 *Ms = lds + wv * kRevWaveFloat4;
    float4 *Sa = Ms + 3 * kWave;
    int *Ac = reinterpret_cast<int *>(Sa + 3 * kWave);
    int *Own = Ac + kWave;
    const int w = blockIdx.x * kMPWaves + wv;
    if (w >= ml.num_blocks) return;  // whole waves leave together; no workgroup barriers here
    const MPBlock bd = ml.blocks[w];
    const bool valid = lane < bd.count;
    const int64_t gid = bd.gbegin + lane;
    const int64_t cid = bd.cbegin + lane;
    int a = -1, p = -1;
    bool head = false;
    float L[12], S[12];
    if (valid) {
        p = ml.parent[gid];
        if (p >= 0) {
            if (p >= bd.gbegin) a = (int)(p - bd.gbegin); else head = true;
        }
        load_local<false>(pose, gid, 0, 0, L);
        aff_load(reinterpret_cast<const float4 *>(bwd.grad_global) + 4 * gid, S);
        if constexpr (FINAL) {
            const int ai = ml.aself[cid];
            if (ai >= 0) {
                float u[12];
                aff_load(Sanc + 3 * ai, u);
#pragma unroll
                for (int k = 0; k < 12; ++k) S[k] += u[k];
            }
        }
    } else {
        aff_identity(L);
#pragma unroll
        for (int k = 0; k < 12; ++k) S[k] = 0.0f;
    }
    wave_block_reverse(S, L, a, lane, Ms, Sa, Ac, Own);
    if constexpr (!FINAL) {
        if (valid && head) {
            float c[12];
            adj_pull(S, L, c);
            float *dst = reinterpret_cast<float *>(Sanc + 3 * (int64_t)ml.janc[cid]);
#pragma unroll
            for (int k = 0; k < 12; ++k) atomicAdd(dst + k, c[k]);
        }
    } else if (valid) {
        float Ap[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
        if (p >= 0) {
            float g[12];
            aff_load(ml.G + 3 * (bd.cbegin + (p - bd.gbegin)), g);  // same character
            Ap[0] = g[0]; Ap[1] = g[1]; Ap[2] = g[2];
            Ap[3] = g[4]; Ap[4] = g[5]; Ap[5] = g[6];
            Ap[6] = g[8]; Ap[7] = g[9]; Ap[8] = g[10];
        }
        const float4 q = reinterpret_cast<const float4 *>(pose.quat)[gid];
        float sx = 1.0f, sy = 1.0f, sz = 1.0f;
        if (pose.scale) {
            const float *sp = pose.scale + 3 * gid;
            sx = sp[0]; sy = sp[1]; sz = sp[2];
        }
        write_grads(bwd, gid, S, Ap, q, sx, sy, sz);
    }
}

__global__ void __launch_bounds__(256)
mpr_fill_zero_kernel(int64_t n4, float4 *dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) dst[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ void __launch_bounds__(256)
mpr_copy_kernel(int64_t n4, const float4 *src, float4 *dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) dst[i] = src[i];
}

// One reverse round over the anchor tree: anchor i adds S_r(i) (.) M_r(i)
// into its current target (global float atomics into the next buffer,
// which starts as a copy of S_r), while M and the targets double.
__global__ void __launch_bounds__(256)
mpr_anchor_round_kernel(int32_t na, const float4 *S, const float4 *M, const int32_t *A, float4 *Snext,
                        float4 *Mnext, int32_t *Anext)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= na) return;
    float m[12];
    aff_load(M + 3 * i, m);
    const int t = A[i];
    if (t >= 0) {
        float x[12], c[12], g[12];
        aff_load(S + 3 * i, x);
        adj_pull(x, m, c);
        float *dst = reinterpret_cast<float *>(Snext + 3 * t);
#pragma unroll
        for (int k = 0; k < 12; ++k) atomicAdd(dst + k, c[k]);
        aff_load(M + 3 * t, g);
        aff_mul_left(g, m);
        Anext[i] = A[t];
    } else {
        Anext[i] = -1;
    }
    aff_store(Mnext + 3 * i, m);
}

// The reverse rounds for one segment of anchors that no anchor points out
// of (the segments of the forward's anchor rounds): one workgroup, one
// thread per anchor, inboxes, jump products, pointers and owner words in
// LDS.  Each round every pusher sends S (.) M to its current target the
// way the synchronous tile adjoint does: the target's owner word names one
// pusher, which stores into the inbox; the others (fan-in) add to it
// atomically after a barrier; the target adds its inbox to S in registers.
// S holds the anchors' adjoints before the rounds and receives them after.
// LDS: inbox [cap][3] | M [cap][3] float4 | pointers [cap] | owners [cap]
size_t mpr_seg_lds_bytes() { return (size_t)kAnchorSegCap * (6 * sizeof(float4) + 2 * sizeof(int32_t)); }

__global__ void __launch_bounds__(kAnchorSegCap)
mpr_anchor_seg_kernel(const int32_t *aseg, int32_t rounds, float4 *S, const float4 *M0, const int32_t *A0)
{
    static_assert(kAnchorSegCap <= (1 << kOwnerShift), "owner words hold a segment-local id");
    extern __shared__ float4 lds[];
    float4 *In = lds;
    float4 *Ms = lds + 3 * kAnchorSegCap;
    int32_t *As = reinterpret_cast<int32_t *>(lds + 6 * kAnchorSegCap);
    int32_t *Own = As + kAnchorSegCap;
    const int s = aseg[blockIdx.x], n = aseg[blockIdx.x + 1] - s;
    const int t = threadIdx.x;
    const bool live = t < n;
    float x[12], m[12];
    int a = -1;
    if (live) {
        aff_load(S + 3 * (s + t), x);
        aff_load(M0 + 3 * (s + t), m);
        const int g = A0[s + t];
        a = (g >= s && g < s + n) ? g - s : -1;  // the plan's cuts keep every pointer inside
        aff_store(Ms + 3 * t, m);
        As[t] = a;
        owner_claim(Own + t, -1);
    }
    __syncthreads();
    if (a >= 0) owner_claim(Own + a, t);
    for (int r = 0; r < rounds; ++r) {
        __syncthreads();  // claims, products and pointers of round r
        const int tag = r << kOwnerShift;
        int aa = -1;
        bool lose = false;
        float c[12];
        if (a >= 0) {
            adj_pull(x, m, c);
            lose = owner_read(Own + a) != (tag | t);
            if (!lose) aff_store(In + 3 * a, c);
            float g[12];
            aff_load(Ms + 3 * a, g);
            aa = As[a];
            aff_mul_left(g, m);  // published after the barriers
        }
        __syncthreads();
        if (lose) lds_atomic_add12(In + 3 * a, c);
        const bool recv = live && (owner_read(Own + t) >> kOwnerShift) == r;
        __syncthreads();
        if (recv) {
            float in[12];
            aff_load(In + 3 * t, in);
#pragma unroll
            for (int k = 0; k < 12; ++k) x[k] += in[k];
        }
        if (a >= 0) {
            a = aa;
            aff_store(Ms + 3 * t, m);
            As[t] = a;
            if (a >= 0) owner_claim(Own + a, (tag + (1 << kOwnerShift)) | t);
        }
    }
    if (live) aff_store(S + 3 * (s + t), x);
}

// ---------------------------------------------------------------------------
// Standalone Simulation step and Bind MeshPose step.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
sample_tile_kernel(TileLaunch tl, PoseArgs pose, float *quat_out, float *trans_out)
{
    extern __shared__ float4 lds[];
    int *cstart = reinterpret_cast<int *>(lds);
    for (int tile = blockIdx.x; tile < tl.num_tiles; tile += gridDim.x) {
        const TileDesc td = tl.tiles[tile];
        for (int i = threadIdx.x; i <= td.num_chars; i += blockDim.x)
            cstart[i] = (int)(pose.offsets[td.first_char + i] - td.begin);
        __syncthreads();
        for (int jl = threadIdx.x; jl < td.count; jl += blockDim.x) {
            const int c = tile_char_of(cstart, td.num_chars, jl);
            const int64_t gid = td.begin + jl;
            float4 q;
            float tx, ty, tz;
            sample_pose(pose, td.first_char + c, jl - cstart[c], q, tx, ty, tz);
            reinterpret_cast<float4 *>(quat_out)[gid] = q;
            trans_out[3 * gid + 0] = tx;
            trans_out[3 * gid + 1] = ty;
            trans_out[3 * gid + 2] = tz;
        }
        __syncthreads();
    }
}

template <class BLOCK>
__global__ void __launch_bounds__(256)
sample_mp_kernel(const BLOCK *blocks, int32_t num_blocks, PoseArgs pose, float *quat_out, float *trans_out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = blockIdx.x * kMPWaves + threadIdx.x / kWave;
    if (w >= num_blocks) return;
    const BLOCK bd = blocks[w];
    if (lane >= bd.count) return;
    const int64_t gid = bd.gbegin + lane;
    float4 q;
    float tx, ty, tz;
    sample_pose(pose, bd.chr, (int)(gid - pose.offsets[bd.chr]), q, tx, ty, tz);
    reinterpret_cast<float4 *>(quat_out)[gid] = q;
    trans_out[3 * gid + 0] = tx;
    trans_out[3 * gid + 1] = ty;
    trans_out[3 * gid + 2] = tz;
}

__global__ void __launch_bounds__(256)
skin_kernel(int64_t n, const float4 *G, const float4 *B, float4 *S)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 b0 = B[4 * i], b1 = B[4 * i + 1], b2 = B[4 * i + 2], b3 = B[4 * i + 3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float4 g = G[4 * i + r];
        S[4 * i + r] = make_float4(fmaf(g.x, b0.x, fmaf(g.y, b1.x, fmaf(g.z, b2.x, g.w * b3.x))),
                                   fmaf(g.x, b0.y, fmaf(g.y, b1.y, fmaf(g.z, b2.y, g.w * b3.y))),
                                   fmaf(g.x, b0.z, fmaf(g.y, b1.z, fmaf(g.z, b2.z, g.w * b3.z))),
                                   fmaf(g.x, b0.w, fmaf(g.y, b1.w, fmaf(g.z, b2.w, g.w * b3.w))));
    }
}

template <int WAVES, bool SAMPLE, int MODE>
hipError_t launch_fwd_tiles_t(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                              hipStream_t stream)
{
    const size_t lds = forward_tile_lds_bytes(tl.tile_cap, SAMPLE || MODE == 2);
    auto kern = fwd_tile_kernel<WAVES, SAMPLE, MODE>;
    hipLaunchKernelGGL(kern, dim3(tl.grid), dim3(WAVES * kWave), lds, stream, tl, pose, out);
    return hipGetLastError();
}

template <bool SAMPLE, int MODE>
hipError_t launch_fwd_tiles_w(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                              hipStream_t stream)
{
    switch (tl.waves) {
    case 1: return launch_fwd_tiles_t<1, SAMPLE, MODE>(tl, pose, out, stream);
    case 2: return launch_fwd_tiles_t<2, SAMPLE, MODE>(tl, pose, out, stream);
    case 4: return launch_fwd_tiles_t<4, SAMPLE, MODE>(tl, pose, out, stream);
    case 8: return launch_fwd_tiles_t<8, SAMPLE, MODE>(tl, pose, out, stream);
    case 16: return launch_fwd_tiles_t<16, SAMPLE, MODE>(tl, pose, out, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int WAVES, bool SAMPLE, bool INST>
hipError_t set_vertex_lds_limits()
{
    const int bytes = (int)forward_vertex_lds_bytes(kMaxVertexTileJoints);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(fwd_vertex_kernel<WAVES, SAMPLE, INST, 0>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (err != hipSuccess) return err;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fwd_vertex_kernel<WAVES, SAMPLE, INST, 1>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int WAVES>
hipError_t set_vertex_lds_limits_all()
{
    hipError_t err;
    if ((err = set_vertex_lds_limits<WAVES, false, false>()) != hipSuccess) return err;
    if ((err = set_vertex_lds_limits<WAVES, false, true>()) != hipSuccess) return err;
    if ((err = set_vertex_lds_limits<WAVES, true, false>()) != hipSuccess) return err;
    return set_vertex_lds_limits<WAVES, true, true>();
}

template <int WAVES>
hipError_t set_lds_limits()
{
    const int fwd = (int)forward_tile_lds_bytes(kMaxTileJoints, true);
    const int bwd = (int)backward_tile_lds_bytes(kMaxBwdTileJoints);
    const void *fk[6] = {reinterpret_cast<const void *>(fwd_tile_kernel<WAVES, false, 0>),
                         reinterpret_cast<const void *>(fwd_tile_kernel<WAVES, true, 0>),
                         reinterpret_cast<const void *>(fwd_tile_kernel<WAVES, false, 1>),
                         reinterpret_cast<const void *>(fwd_tile_kernel<WAVES, true, 1>),
                         reinterpret_cast<const void *>(fwd_tile_kernel<WAVES, false, 2>),
                         reinterpret_cast<const void *>(fwd_tile_kernel<WAVES, true, 2>)};
    for (const void *k : fk) {
        hipError_t err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, fwd);
        if (err != hipSuccess) return err;
    }
    const void *bk[2] = {reinterpret_cast<const void *>(bwd_tile_kernel<WAVES, false>),
                         reinterpret_cast<const void *>(bwd_tile_kernel<WAVES, true>)};
    for (const void *k : bk) {
        hipError_t err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bwd);
        if (err != hipSuccess) return err;
    }
    const int bs = (int)backward_sync_lds_bytes(std::min(kMaxSyncTileJoints, WAVES * kWave));
    const void *sk[3] = {reinterpret_cast<const void *>(bwd_sync_kernel<WAVES, kSeedDense>),
                         reinterpret_cast<const void *>(bwd_sync_kernel<WAVES, kSeedEffectors>),
                         reinterpret_cast<const void *>(bwd_sync_kernel<WAVES, kSeedForward>)};
    hipError_t err = hipSuccess;
    for (const void *k : sk)
        if (err == hipSuccess) err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bs);
    if (err != hipSuccess) return err;
    {
        // the two-level adjoint: up to the whole LDS (the plan checks its need)
        int dev = 0, lds_max = 0;
        if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
        if ((err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
            return err;
        for (int seed = 0; seed < 3; ++seed) {
            if (err == hipSuccess)
                err = hipFuncSetAttribute(anchor_kernel_of<WAVES, 1>(seed), hipFuncAttributeMaxDynamicSharedMemorySize,
                                          lds_max);
            if constexpr (WAVES <= 8) {
                if (err == hipSuccess)
                    err = hipFuncSetAttribute(anchor_kernel_of<WAVES, 2>(seed),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
            }
        }
    }
    if (err != hipSuccess || WAVES != 16) return err;
    const void *pk[4] = {reinterpret_cast<const void *>(paper_alg_kernel<1>),
                         reinterpret_cast<const void *>(paper_alg_kernel<2>),
                         reinterpret_cast<const void *>(paper_alg_kernel<3>),
                         reinterpret_cast<const void *>(paper_alg_kernel<4>)};
    for (int k = 0; k < 4; ++k) {
        err = hipFuncSetAttribute(pk[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)paper_alg_lds_bytes(kPaperAlgTileJoints, k + 1));
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

} // namespace

// Workspace of the allocation-free reverse mode of the sampler
// (hs_pose_sample_backward_noalloc): 2 float4 per joint for at most
// kNoAllocMaxJoints joints.  Each device that loads the library holds its
// own copy until the process ends; host code reaches it only through the
// device address that noalloc_workspace() looks up (the symbol itself is
// a host-side stand-in, not a device address).
static __device__ __align__(256) float4 scratch[2 * (size_t)kNoAllocMaxJoints];

hipError_t noalloc_workspace(int device, float4 **out)
{
    static std::mutex mu;
    static float4 *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
        if (err != hipSuccess) return err;
        addr[device] = static_cast<float4 *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

template <int WAVES>
void queue_kernels(const void **k, int &n)
{
    k[n++] = reinterpret_cast<const void *>(fwd_queue_kernel<WAVES, false, false>);
    k[n++] = reinterpret_cast<const void *>(fwd_queue_kernel<WAVES, false, true>);
    k[n++] = reinterpret_cast<const void *>(fwd_queue_kernel<WAVES, true, false>);
    k[n++] = reinterpret_cast<const void *>(fwd_queue_kernel<WAVES, true, true>);
}

hipError_t prepare_kernels()
{
    hipError_t err;
    {
        // the queue kernels: up to the whole LDS of a CU (the plan checks
        // its own need against the device's limit)
        int dev = 0, lds_max = 0;
        if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
        if ((err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
            return err;
        const void *qk[20];
        int nq = 0;
        queue_kernels<1>(qk, nq);
        queue_kernels<2>(qk, nq);
        queue_kernels<4>(qk, nq);
        queue_kernels<8>(qk, nq);
        queue_kernels<16>(qk, nq);
        for (int i = 0; i < nq; ++i)
            if ((err = hipFuncSetAttribute(qk[i], hipFuncAttributeMaxDynamicSharedMemorySize, lds_max)) != hipSuccess)
                return err;
    }
    if ((err = set_vertex_lds_limits_all<4>()) != hipSuccess || (err = set_vertex_lds_limits_all<8>()) != hipSuccess ||
        (err = set_vertex_lds_limits_all<16>()) != hipSuccess)
        return err;
    if ((err = hipFuncSetAttribute(reinterpret_cast<const void *>(vertex_skin_kernel<0>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, kMaxSkinJoints * 48)) != hipSuccess ||
        (err = hipFuncSetAttribute(reinterpret_cast<const void *>(vertex_skin_kernel<1>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, kMaxSkinJoints * 32)) != hipSuccess)
        return err;
    if ((err = hipFuncSetAttribute(reinterpret_cast<const void *>(mpr_anchor_seg_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)mpr_seg_lds_bytes())) != hipSuccess)
        return err;
    if ((err = hipFuncSetAttribute(reinterpret_cast<const void *>(mp_chain_kernel<false>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kChainLdsBytes)) != hipSuccess ||
        (err = hipFuncSetAttribute(reinterpret_cast<const void *>(mp_chain_kernel<true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kChainLdsBytes)) != hipSuccess)
        return err;
    if ((err = set_lds_limits<1>()) != hipSuccess) return err;
    if ((err = set_lds_limits<2>()) != hipSuccess) return err;
    if ((err = set_lds_limits<4>()) != hipSuccess) return err;
    if ((err = set_lds_limits<8>()) != hipSuccess) return err;
    return set_lds_limits<16>();
}

size_t forward_queue_lds_bytes(int waves, int max_anchors, int tile_cap, bool sample, bool skin)
{
    size_t bytes = (size_t)waves * kWave * (skin ? 68 : 52) + (size_t)max_anchors * 52;
    if (sample) bytes += (size_t)(tile_cap + 1) * 4;
    return bytes;
}

size_t forward_tile_lds_bytes(int tile_cap, bool char_map)
{
    size_t bytes = (size_t)tile_cap * 48 + (size_t)(tile_cap / kWave) * (48 + 3 * 4);
    if (char_map) bytes += (size_t)(tile_cap + 1) * 4;
    return bytes;
}

size_t paper_alg_lds_bytes(int tile_cap, int alg)
{
    return (size_t)tile_cap * ((alg == 4 ? 96 : 48) + 3 * 4);
}

hipError_t launch_paper_alg(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out, hipStream_t stream)
{
    if (tl.tile_cap > kPaperAlgTileJoints || pose.kind != 0) return hipErrorInvalidValue;
    const size_t lds = paper_alg_lds_bytes(tl.tile_cap, tl.algorithm);
    const dim3 grid(tl.grid), blk(1024);
    switch (tl.algorithm) {
    case 1: hipLaunchKernelGGL(paper_alg_kernel<1>, grid, blk, lds, stream, tl, pose, out); break;
    case 2: hipLaunchKernelGGL(paper_alg_kernel<2>, grid, blk, lds, stream, tl, pose, out); break;
    case 3: hipLaunchKernelGGL(paper_alg_kernel<3>, grid, blk, lds, stream, tl, pose, out); break;
    case 4: hipLaunchKernelGGL(paper_alg_kernel<4>, grid, blk, lds, stream, tl, pose, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward_tiles(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                                hipStream_t stream)
{
    if (tl.num_tiles == 0) return hipSuccess;
    if (tl.algorithm != 0) return launch_paper_alg(tl, pose, out, stream);
    const bool sample = pose.kind == 1;
    // tiles that map joints to characters read the CSR offsets
    if ((sample || tl.skel_parent) && !pose.offsets) return hipErrorInvalidValue;
    if (tl.skel_parent) {
        if (tl.chain_units || !tl.char_skel) return hipErrorInvalidValue;
        return sample ? launch_fwd_tiles_w<true, 2>(tl, pose, out, stream)
                      : launch_fwd_tiles_w<false, 2>(tl, pose, out, stream);
    }
    if (tl.chain_units)
        return sample ? launch_fwd_tiles_w<true, 1>(tl, pose, out, stream)
                      : launch_fwd_tiles_w<false, 1>(tl, pose, out, stream);
    return sample ? launch_fwd_tiles_w<true, 0>(tl, pose, out, stream)
                  : launch_fwd_tiles_w<false, 0>(tl, pose, out, stream);
}

// Phase 1 per block, anchor rounds, final pass; Gc non-NULL: compact global
// transforms for the adjoint instead of the outputs.
hipError_t run_multipass(const MPLaunch &ml, const PoseArgs &pose, const OutArgs &out, float4 *Gc,
                         hipStream_t stream)
{
    const dim3 blk(kMPWaves * kWave);
    const dim3 grid((ml.num_blocks + kMPWaves - 1) / kMPWaves);
    if (pose.kind == 1)
        hipLaunchKernelGGL(mp_local_kernel<true>, grid, blk, 0, stream, ml, pose);
    else
        hipLaunchKernelGGL(mp_local_kernel<false>, grid, blk, 0, stream, ml, pose);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    // rounds over the anchors, from the phase-1 products (A1, E1) into the
    // ping-pong buffers; with no rounds the phase-1 products are final
    const float4 *pin = ml.A1;
    const int32_t *ein = ml.E1;
    if (ml.num_anchors > 0 && ml.num_aseg > 0) {
        hipLaunchKernelGGL(mp_anchor_seg_kernel, dim3((unsigned)ml.num_aseg), dim3(kAnchorSegCap), 0, stream,
                           ml.aseg, ml.rounds, ml.A1, ml.E1, ml.AP[0], ml.AE[0]);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        pin = ml.AP[0];
    } else if (ml.num_anchors > 0) {
        const dim3 agrid((unsigned)((ml.num_anchors + 255) / 256));
        for (int r = 0; r < ml.rounds; ++r) {
            hipLaunchKernelGGL(mp_anchor_round_kernel, agrid, dim3(256), 0, stream, ml.num_anchors, pin, ein,
                               ml.AP[r & 1], ml.AE[r & 1]);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            pin = ml.AP[r & 1];
            ein = ml.AE[r & 1];
        }
    }
    if (pose.kind == 1)
        hipLaunchKernelGGL(mp_out_kernel<true>, grid, blk, 0, stream, ml, pose, pin, out, Gc);
    else
        hipLaunchKernelGGL(mp_out_kernel<false>, grid, blk, 0, stream, ml, pose, pin, out, Gc);
    return hipGetLastError();
}

hipError_t chain_blocks_per_cu(bool sample, int *out)
{
    *out = 0;
    return sample ? hipOccupancyMaxActiveBlocksPerMultiprocessor(out, mp_chain_kernel<true>, kChainWaves * kWave,
                                                                 kChainLdsBytes)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(out, mp_chain_kernel<false>, kChainWaves * kWave,
                                                                 kChainLdsBytes);
}

hipError_t launch_forward_chains(const ChainLaunch &cl, const PoseArgs &pose, const OutArgs &out,
                                 hipStream_t stream)
{
    if (cl.num_blocks == 0) return hipSuccess;
    if (cl.grid < 1 || cl.num_sb < 1) return hipErrorInvalidValue;
    if (pose.kind == 1)
        hipLaunchKernelGGL(mp_chain_kernel<true>, dim3(cl.grid), dim3(kChainWaves * kWave), kChainLdsBytes, stream,
                           cl, pose, out);
    else
        hipLaunchKernelGGL(mp_chain_kernel<false>, dim3(cl.grid), dim3(kChainWaves * kWave), kChainLdsBytes, stream,
                           cl, pose, out);
    return hipGetLastError();
}

hipError_t launch_forward_multipass(const MPLaunch &ml, const PoseArgs &pose, const OutArgs &out,
                                    hipStream_t stream)
{
    if (ml.num_blocks == 0) return hipSuccess;
    return run_multipass(ml, pose, out, nullptr, stream);
}

hipError_t launch_pose_sample(const TileLaunch &tl, const MPLaunch &ml, const ChainLaunch &cl, const PoseArgs &pose,
                              float *quat_out, float *trans_out, hipStream_t stream)
{
    if (tl.num_tiles > 0) {
        const size_t lds = (size_t)(tl.tile_cap + 1) * 4;
        hipLaunchKernelGGL(sample_tile_kernel, dim3(tl.num_tiles), dim3(256), lds, stream, tl, pose,
                           quat_out, trans_out);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (ml.num_blocks > 0) {
        hipLaunchKernelGGL(sample_mp_kernel<MPBlock>, dim3((ml.num_blocks + kMPWaves - 1) / kMPWaves),
                           dim3(kMPWaves * kWave), 0, stream, ml.blocks, ml.num_blocks, pose, quat_out, trans_out);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (cl.num_blocks > 0) {
        hipLaunchKernelGGL(sample_mp_kernel<ChainBlock>, dim3((cl.num_blocks + kMPWaves - 1) / kMPWaves),
                           dim3(kMPWaves * kWave), 0, stream, cl.blocks, cl.num_blocks, pose, quat_out, trans_out);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_pose_sample_backward(const PoseArgs &pose, const SampleBwdArgs &A, hipStream_t stream)
{
    hipError_t err = hipSuccess;
    const bool keys = A.grad_key_quat || A.grad_key_trans;
    SampleBwdArgs a = A;
    if (!keys) a.ws = nullptr;  // nothing would read it
    if (A.C > 0 && (A.grad_time || A.grad_weight || a.ws)) {
        hipLaunchKernelGGL(sample_bwd_kernel, dim3((unsigned)A.C), dim3(kSampleBwdThreads), 0, stream, pose, a);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if (keys) {
        const int64_t blocks = (int64_t)pose.num_clips * pose.num_keys;
        const dim3 grid((unsigned)std::min<int64_t>(blocks, 1 << 20));
        if (a.ws)
            hipLaunchKernelGGL(sample_bwd_keys_kernel<true>, grid, dim3(kSampleBwdThreads), 0, stream, pose, a);
        else
            hipLaunchKernelGGL(sample_bwd_keys_kernel<false>, grid, dim3(kSampleBwdThreads), 0, stream, pose, a);
        err = hipGetLastError();
    }
    return err;
}

// The forward's memory traffic without its arithmetic: per joint the same
// reads (quat 16, trans 12, scale 12, a 4-byte table entry: streaming
// loads, one joint per lane) and the same 64-byte output rows (coalesced
// 16-byte stores, four per joint, through a per-wave LDS slice as the
// scan's blocks store them), the rows holding the inputs so that nothing
// can be dropped.
__global__ void __launch_bounds__(256)
stream_probe_kernel(int64_t n, const float *quat, const float *trans, const float *scale, const int32_t *table,
                    float *out)
{
    __shared__ float4 slice[4][kWave * 3];
    const int lane = threadIdx.x & (kWave - 1);
    float4 *X = slice[threadIdx.x / kWave];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~(int64_t)(kWave - 1); base < n;
         base += stride) {
        const int64_t g = base + lane;
        float m[12];
        if (g < n) {
            const native_float4 q = __builtin_nontemporal_load(reinterpret_cast<const native_float4 *>(quat) + g);
            const float *t = trans + 3 * g, *sc = scale + 3 * g;
            m[0] = q.x; m[1] = q.y; m[2] = q.z; m[3] = __builtin_nontemporal_load(t);
            m[4] = q.w; m[5] = __builtin_nontemporal_load(sc); m[6] = __builtin_nontemporal_load(sc + 1);
            m[7] = __builtin_nontemporal_load(t + 1);
            m[8] = __builtin_nontemporal_load(sc + 2); m[9] = __int_as_float(__builtin_nontemporal_load(table + g));
            m[10] = 0.0f; m[11] = __builtin_nontemporal_load(t + 2);
        } else {
            aff_identity(m);
        }
        wave_sync();
        aff_store(X + 3 * lane, m);
        wave_sync();
        OutArgs o{};
        o.global_out = out;
        store_rows<1>(o, X, base, 0, 1, (int)std::min<int64_t>(kWave, n - base), lane);
    }
}

hipError_t launch_stream_probe(int64_t n, const float *quat, const float *trans, const float *scale,
                               const int32_t *table, float *out, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int64_t waves = (n + kWave - 1) / kWave;
    const dim3 grid((unsigned)std::min<int64_t>((waves + 3) / 4, 1 << 20));
    hipLaunchKernelGGL(stream_probe_kernel, grid, dim3(256), 0, stream, n, quat, trans, scale, table, out);
    return hipGetLastError();
}

hipError_t launch_effector_grad(int64_t n, int64_t ne, const int64_t *eff, const float *G, const float *target,
                                float *grad, hipStream_t stream)
{
    if (ne == 0) return hipSuccess;
    hipLaunchKernelGGL(effector_grad_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, stream, n, ne, eff,
                       G, target, grad);
    return hipGetLastError();
}

// Device topology check (HS_FLAG_VALIDATE): one workgroup per character,
// its threads over the character's joints.
__global__ void __launch_bounds__(256)
validate_kernel(const int64_t *offsets, int64_t num_chars, const int32_t *parent, const int32_t *level,
                uint32_t *status)
{
    for (int64_t c = blockIdx.x; c < num_chars; c += gridDim.x) {
        const int64_t b = offsets[c], e = offsets[c + 1];
        if (e < b) {
            if (threadIdx.x == 0) {
                note_status(status, kStatusTopology);
                atomicMin(status + 1, (uint32_t)b);
            }
            continue;
        }
        for (int64_t g = b + threadIdx.x; g < e; g += blockDim.x) {
            const int32_t p = parent[g];
            const bool ok = p < 0 ? (p == -1 && level[g] == 1)
                                  : ((int64_t)p >= b && (int64_t)p < g && level[g] == level[p] + 1);
            if (!ok) {
                note_status(status, kStatusTopology);
                atomicMin(status + 1, (uint32_t)g);
            }
        }
    }
}

hipError_t launch_validate(const int64_t *offsets, int64_t num_chars, const int32_t *parent, const int32_t *level,
                           uint32_t *status, hipStream_t stream)
{
    if (num_chars <= 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>(num_chars, 65536);
    hipLaunchKernelGGL(validate_kernel, dim3(grid), dim3(256), 0, stream, offsets, num_chars, parent, level, status);
    return hipGetLastError();
}

hipError_t launch_skin(int64_t n, const float *global, const float *inv_bind, float *skin_out,
                       hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(skin_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n,
                       reinterpret_cast<const float4 *>(global),
                       reinterpret_cast<const float4 *>(inv_bind),
                       reinterpret_cast<float4 *>(skin_out));
    return hipGetLastError();
}

size_t forward_vertex_lds_bytes(int tile_cap)
{
    return forward_tile_lds_bytes(tile_cap, true) + (size_t)(tile_cap + 1) * 4;
}

template <int WAVES, bool SAMPLE>
hipError_t launch_queue_t(const QueueLaunch &ql, const PoseArgs &pose, const OutArgs &out, hipStream_t stream)
{
    const bool skin = out.skin_out != nullptr;
    const size_t lds = forward_queue_lds_bytes(WAVES, ql.max_anchors, ql.tile_cap, SAMPLE, skin);
    if (skin)
        hipLaunchKernelGGL((fwd_queue_kernel<WAVES, SAMPLE, true>), dim3(ql.grid), dim3(WAVES * kWave), lds, stream,
                           ql, pose, out);
    else
        hipLaunchKernelGGL((fwd_queue_kernel<WAVES, SAMPLE, false>), dim3(ql.grid), dim3(WAVES * kWave), lds, stream,
                           ql, pose, out);
    return hipGetLastError();
}

template <int WAVES>
hipError_t queue_occupancy_t(bool sample, bool skin, size_t lds, int *out)
{
    const void *k[4];
    int n = 0;
    queue_kernels<WAVES>(k, n);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k[2 * (sample ? 1 : 0) + (skin ? 1 : 0)], WAVES * kWave,
                                                        lds);
}

hipError_t queue_blocks_per_cu(int waves, bool sample, bool skin, size_t lds, int *out)
{
    *out = 1;
    switch (waves) {
    case 1: return queue_occupancy_t<1>(sample, skin, lds, out);
    case 2: return queue_occupancy_t<2>(sample, skin, lds, out);
    case 4: return queue_occupancy_t<4>(sample, skin, lds, out);
    case 8: return queue_occupancy_t<8>(sample, skin, lds, out);
    case 16: return queue_occupancy_t<16>(sample, skin, lds, out);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward_queue(const QueueLaunch &ql, const PoseArgs &pose, const OutArgs &out,
                                hipStream_t stream)
{
    if (ql.num_tiles == 0) return hipSuccess;
    if (ql.max_anchors > kQMaxAnchors || ql.tile_cap > kQMaxTileJoints)
        return hipErrorInvalidValue;
    const bool sample = pose.kind == 1;
    if (sample && !pose.offsets) return hipErrorInvalidValue;
    QueueLaunch q = ql;
    q.grid = ql.grids[sample ? 1 : 0][out.skin_out ? 1 : 0];
    if (q.grid < 1) return hipErrorInvalidValue;
    switch (ql.waves) {
    case 1: return sample ? launch_queue_t<1, true>(q, pose, out, stream) : launch_queue_t<1, false>(q, pose, out, stream);
    case 2: return sample ? launch_queue_t<2, true>(q, pose, out, stream) : launch_queue_t<2, false>(q, pose, out, stream);
    case 4: return sample ? launch_queue_t<4, true>(q, pose, out, stream) : launch_queue_t<4, false>(q, pose, out, stream);
    case 8: return sample ? launch_queue_t<8, true>(q, pose, out, stream) : launch_queue_t<8, false>(q, pose, out, stream);
    case 16:
        return sample ? launch_queue_t<16, true>(q, pose, out, stream) : launch_queue_t<16, false>(q, pose, out, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int WAVES, bool SAMPLE, bool INST>
hipError_t launch_fwd_vertex_t(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                               const VertexLaunch &vl, int method, float *vout, hipStream_t stream)
{
    const size_t lds = forward_vertex_lds_bytes(tl.tile_cap);
    const dim3 grid(tl.grid), blk(WAVES * kWave);
    if (method == 0)
        hipLaunchKernelGGL((fwd_vertex_kernel<WAVES, SAMPLE, INST, 0>), grid, blk, lds, stream, tl, pose, out, vl, vout);
    else
        hipLaunchKernelGGL((fwd_vertex_kernel<WAVES, SAMPLE, INST, 1>), grid, blk, lds, stream, tl, pose, out, vl, vout);
    return hipGetLastError();
}

template <bool SAMPLE, bool INST>
hipError_t launch_fwd_vertex_w(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                               const VertexLaunch &vl, int method, float *vout, hipStream_t stream)
{
    // 4 to 16 waves: at least one block per wave in the scan when the tile
    // allows, and enough threads for the vertex phase
    int waves = 4;
    while (waves < 16 && waves * 2 * kWave <= tl.tile_cap) waves *= 2;
    switch (waves) {
    case 4: return launch_fwd_vertex_t<4, SAMPLE, INST>(tl, pose, out, vl, method, vout, stream);
    case 8: return launch_fwd_vertex_t<8, SAMPLE, INST>(tl, pose, out, vl, method, vout, stream);
    default: return launch_fwd_vertex_t<16, SAMPLE, INST>(tl, pose, out, vl, method, vout, stream);
    }
}

hipError_t launch_forward_vertices(const TileLaunch &tl, const PoseArgs &pose, const OutArgs &out,
                                   const VertexLaunch &vl, int method, float *vout, hipStream_t stream)
{
    if (tl.num_tiles == 0) return hipSuccess;
    if (tl.tile_cap > kMaxVertexTileJoints || !pose.offsets || !out.inv_bind || (method != 0 && method != 1))
        return hipErrorInvalidValue;
    const bool sample = pose.kind == 1, inst = tl.skel_parent != nullptr;
    if (inst && !tl.char_skel) return hipErrorInvalidValue;
    if (sample)
        return inst ? launch_fwd_vertex_w<true, true>(tl, pose, out, vl, method, vout, stream)
                    : launch_fwd_vertex_w<true, false>(tl, pose, out, vl, method, vout, stream);
    return inst ? launch_fwd_vertex_w<false, true>(tl, pose, out, vl, method, vout, stream)
                : launch_fwd_vertex_w<false, false>(tl, pose, out, vl, method, vout, stream);
}

hipError_t launch_vertex_skin(const VertexLaunch &vl, int method, const float *skin, float *out,
                              hipStream_t stream)
{
    if (vl.C == 0) return hipSuccess;
    if (vl.max_joints > kMaxSkinJoints || (method != 0 && method != 1)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)vl.C), blk(kSkinThreads);
    const float4 *S = reinterpret_cast<const float4 *>(skin);
    if (method == 0)
        hipLaunchKernelGGL(vertex_skin_kernel<0>, grid, blk, (size_t)vl.max_joints * 48, stream, vl, S, out);
    else
        hipLaunchKernelGGL(vertex_skin_kernel<1>, grid, blk, (size_t)vl.max_joints * 32, stream, vl, S, out);
    return hipGetLastError();
}

size_t backward_anchor_lds_bytes(int waves, int max_anchors, int tile_cap)
{
    return (size_t)waves * kWave * (2 * 48 + 3 * 4) + (size_t)max_anchors * (3 * 48 + 12) + (size_t)tile_cap * 4;
}

size_t backward_sync_lds_bytes(int tile_cap)
{
    return (size_t)tile_cap * 104 + (size_t)(tile_cap / kWave + 1) * 4;
}

size_t backward_tile_lds_bytes(int tile_cap)
{
    return (size_t)tile_cap * 98 + (size_t)(tile_cap / kWave) * 12;
}

template <int WAVES, bool CKPT>
hipError_t launch_bwd_tiles_t(const TileLaunch &tl, const PoseArgs &pose, const BwdArgs &bwd,
                              hipStream_t stream)
{
    const size_t lds = backward_tile_lds_bytes(tl.tile_cap);
    auto kern = bwd_tile_kernel<WAVES, CKPT>;
    hipLaunchKernelGGL(kern, dim3(tl.grid), dim3(WAVES * kWave), lds, stream, tl, pose, bwd);
    return hipGetLastError();
}

template <bool CKPT>
hipError_t launch_bwd_tiles_w(const TileLaunch &tl, const PoseArgs &pose, const BwdArgs &bwd,
                              hipStream_t stream)
{
    switch (tl.waves) {
    case 1: return launch_bwd_tiles_t<1, CKPT>(tl, pose, bwd, stream);
    case 2: return launch_bwd_tiles_t<2, CKPT>(tl, pose, bwd, stream);
    case 4: return launch_bwd_tiles_t<4, CKPT>(tl, pose, bwd, stream);
    case 8: return launch_bwd_tiles_t<8, CKPT>(tl, pose, bwd, stream);
    case 16: return launch_bwd_tiles_t<16, CKPT>(tl, pose, bwd, stream);
    default: return hipErrorInvalidValue;
    }
}

// The two-level adjoint with W waves of BPW blocks each (W * BPW blocks
// cover the tile).
template <int W, int BPW>
hipError_t launch_bwd_anchor_t(const TileLaunch &tl, const PoseArgs &pose, const BwdArgs &bwd, hipStream_t stream)
{
    if (tl.tile_cap > W * BPW * kWave || !tl.code) return hipErrorInvalidValue;
    const size_t lds = backward_anchor_lds_bytes(W, tl.max_anchors, tl.tile_cap);
    const dim3 grid(tl.grid), blk(W * kWave);
    if (bwd.eff_ids && bwd.eff_forward)
        hipLaunchKernelGGL((bwd_anchor_kernel<W, BPW, kSeedForward>), grid, blk, lds, stream, tl, pose, bwd);
    else if (bwd.eff_ids)
        hipLaunchKernelGGL((bwd_anchor_kernel<W, BPW, kSeedEffectors>), grid, blk, lds, stream, tl, pose, bwd);
    else
        hipLaunchKernelGGL((bwd_anchor_kernel<W, BPW, kSeedDense>), grid, blk, lds, stream, tl, pose, bwd);
    return hipGetLastError();
}

// WAVES: the tile's blocks (a power of two); tl.blocks_per_wave 2 halves
// the waves.
template <int WAVES>
hipError_t launch_bwd_anchor_w(const TileLaunch &tl, const PoseArgs &pose, const BwdArgs &bwd, hipStream_t stream)
{
    if constexpr (WAVES >= 2) {
        if (tl.blocks_per_wave == 2) return launch_bwd_anchor_t<WAVES / 2, 2>(tl, pose, bwd, stream);
    }
    return launch_bwd_anchor_t<WAVES, 1>(tl, pose, bwd, stream);
}


template <int W, int BPW>
hipError_t anchor_occupancy_t(int seed, size_t lds, int *out)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, anchor_kernel_of<W, BPW>(seed), W * kWave, lds);
}

hipError_t anchor_blocks_per_cu(int waves, int bpw, int seed, size_t lds, int *out)
{
    *out = 0;
    if (bpw == 2) {
        switch (waves) {
        case 1: return anchor_occupancy_t<1, 2>(seed, lds, out);
        case 2: return anchor_occupancy_t<2, 2>(seed, lds, out);
        case 4: return anchor_occupancy_t<4, 2>(seed, lds, out);
        case 8: return anchor_occupancy_t<8, 2>(seed, lds, out);
        default: return hipErrorInvalidValue;
        }
    }
    switch (waves) {
    case 1: return anchor_occupancy_t<1, 1>(seed, lds, out);
    case 2: return anchor_occupancy_t<2, 1>(seed, lds, out);
    case 4: return anchor_occupancy_t<4, 1>(seed, lds, out);
    case 8: return anchor_occupancy_t<8, 1>(seed, lds, out);
    case 16: return anchor_occupancy_t<16, 1>(seed, lds, out);
    default: return hipErrorInvalidValue;
    }
}

template <int WAVES>
hipError_t launch_bwd_sync_w(const TileLaunch &tl, const PoseArgs &pose, const BwdArgs &bwd, hipStream_t stream)
{
    if (tl.tile_cap > WAVES * kWave) return hipErrorInvalidValue;
    if (tl.adjoint == kAdjAnchors) return launch_bwd_anchor_w<WAVES>(tl, pose, bwd, stream);
    const size_t lds = backward_sync_lds_bytes(tl.tile_cap);
    if (bwd.eff_ids && bwd.eff_forward)
        hipLaunchKernelGGL((bwd_sync_kernel<WAVES, kSeedForward>), dim3(tl.grid), dim3(WAVES * kWave), lds, stream,
                           tl, pose, bwd);
    else if (bwd.eff_ids)
        hipLaunchKernelGGL((bwd_sync_kernel<WAVES, kSeedEffectors>), dim3(tl.grid), dim3(WAVES * kWave), lds, stream,
                           tl, pose, bwd);
    else
        hipLaunchKernelGGL((bwd_sync_kernel<WAVES, kSeedDense>), dim3(tl.grid), dim3(WAVES * kWave), lds, stream, tl,
                           pose, bwd);
    return hipGetLastError();
}

hipError_t launch_backward_tiles(const TileLaunch &tl, const PoseArgs &pose, const BwdArgs &bwd,
                                 hipStream_t stream)
{
    if (tl.num_tiles == 0) return hipSuccess;
    if (tl.tile_cap > kMaxBwdTileJoints) return hipErrorInvalidValue;
    if (tl.tile_cap > kMaxSyncTileJoints || tl.adjoint == kAdjDataflow) {
        if (bwd.eff_ids) return hipErrorInvalidValue;  // sparse seeds: synchronous tiles only
        return bwd.ckpt ? launch_bwd_tiles_w<true>(tl, pose, bwd, stream)
                        : launch_bwd_tiles_w<false>(tl, pose, bwd, stream);
    }
    // tiles of up to 1024 joints: one joint per thread; the jump products
    // give every G_j on chip, so checkpoints are not read here
    TileLaunch t2 = tl;
    t2.waves = 1;
    while (t2.waves < 16 && t2.tile_cap > kWave * t2.waves) t2.waves *= 2;
    switch (t2.waves) {
    case 1: return launch_bwd_sync_w<1>(t2, pose, bwd, stream);
    case 2: return launch_bwd_sync_w<2>(t2, pose, bwd, stream);
    case 4: return launch_bwd_sync_w<4>(t2, pose, bwd, stream);
    case 8: return launch_bwd_sync_w<8>(t2, pose, bwd, stream);
    case 16: return launch_bwd_sync_w<16>(t2, pose, bwd, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward_multipass(const MPLaunch &ml, const PoseArgs &pose, const BwdArgs &bwd,
                                     hipStream_t stream)
{
    if (ml.num_blocks == 0) return hipSuccess;
    if (!ml.G || !ml.aself || (ml.num_anchors > 0 && !ml.S[0])) return hipErrorNotSupported;
    if (bwd.eff_ids) return hipErrorInvalidValue;  // sparse seeds: synchronous tiles only
    const dim3 blk(kMPWaves * kWave);
    const dim3 grid((ml.num_blocks + kMPWaves - 1) / kMPWaves);
    const size_t lds = (size_t)kMPWaves * kRevWaveFloat4 * sizeof(float4);
    hipError_t err;
    // global transforms of the multipass characters (compact), and P
    if ((err = run_multipass(ml, pose, OutArgs{}, ml.G, stream)) != hipSuccess) return err;
    const int na = ml.num_anchors;
    const dim3 agrid((unsigned)((na + 255) / 256));
    const dim3 cgrid((unsigned)((3 * (int64_t)na + 255) / 256));
    int cur = 0;
    if (na > 0) {
        hipLaunchKernelGGL(mpr_fill_zero_kernel, cgrid, dim3(256), 0, stream, 3 * (int64_t)na, ml.S[0]);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    hipLaunchKernelGGL(mpr_block_kernel<false>, grid, blk, lds, stream, ml, pose, bwd, ml.S[0]);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (na > 0 && ml.num_aseg > 0) {
        // per segment in one workgroup's LDS, from the phase-1 products and
        // pointers (A1, E1, left by the forward pass above); in place in S[0]
        hipLaunchKernelGGL(mpr_anchor_seg_kernel, dim3((unsigned)ml.num_aseg), dim3(kAnchorSegCap),
                           mpr_seg_lds_bytes(), stream, ml.aseg, ml.rounds, ml.S[0], ml.A1, ml.E1);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    } else if (na > 0) {
        // the anchors' phase-1 products and pointers (A1, E1, left by the
        // forward pass above) start the reverse rounds
        const float4 *min = ml.A1;
        const int32_t *ein = ml.E1;
        for (int r = 0; r < ml.rounds; ++r) {
            hipLaunchKernelGGL(mpr_copy_kernel, cgrid, dim3(256), 0, stream, 3 * (int64_t)na, ml.S[cur], ml.S[cur ^ 1]);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            hipLaunchKernelGGL(mpr_anchor_round_kernel, agrid, dim3(256), 0, stream, na, ml.S[cur], min, ein,
                               ml.S[cur ^ 1], ml.AP[r & 1], ml.AE[r & 1]);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            min = ml.AP[r & 1];
            ein = ml.AE[r & 1];
            cur ^= 1;
        }
    }
    hipLaunchKernelGGL(mpr_block_kernel<true>, grid, blk, lds, stream, ml, pose, bwd, ml.S[cur]);
    return hipGetLastError();
}

} // namespace hs
