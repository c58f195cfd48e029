// hs_capi.cpp -- the C ABI of include/hs.h: argument validation, topology
// analysis and tiling (plans), launch-shape autotuning, and dispatch of the
// HIP kernels in hs_kernels.hip.
#include "hs.h"
#include "hs_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

static_assert(hs::kNoAllocMaxJoints == HS_NOALLOC_MAX_JOINTS, "static workspace size");

using hs::MPBlock;
using hs::TileDesc;

namespace {

thread_local std::string g_last_error = "no error";

hs_status fail(hs_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

hs_status fail_hip(hipError_t err, const char *what)
{
    if (err == hipErrorOutOfMemory)
        return fail(HS_ERR_OOM, "%s: out of device memory", what);
    return fail(HS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(err));
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

struct Range {
    const void *p;
    size_t bytes;
    const char *name;
};

bool overlap(const Range &a, const Range &b)
{
    if (!a.p || !b.p || a.bytes == 0 || b.bytes == 0) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a.p), b0 = reinterpret_cast<uintptr_t>(b.p);
    return a0 < b0 + b.bytes && b0 < a0 + a.bytes;
}

// Every output must be disjoint from every input and from the other outputs.
hs_status check_aliasing(const std::vector<Range> &outs, const std::vector<Range> &ins)
{
    for (size_t i = 0; i < outs.size(); ++i) {
        for (const Range &in : ins)
            if (overlap(outs[i], in))
                return fail(HS_ERR_INVALID_ARG, "output %s overlaps input %s", outs[i].name, in.name);
        for (size_t k = i + 1; k < outs.size(); ++k)
            if (overlap(outs[i], outs[k]))
                return fail(HS_ERR_INVALID_ARG, "outputs %s and %s overlap", outs[i].name, outs[k].name);
    }
    return HS_OK;
}

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t err = hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T));
    if (err != hipSuccess) return err;
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Copy n elements from a host or device pointer into a host vector.
template <class T>
hipError_t fetch(std::vector<T> &dst, const T *src, size_t n)
{
    dst.resize(n);
    if (n == 0) return hipSuccess;
    hipPointerAttribute_t attr;
    bool device = false;
    if (hipPointerGetAttributes(&attr, src) == hipSuccess)
        device = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
    (void)hipGetLastError();  // clear the error left for unregistered host memory
    if (!device) {
        std::memcpy(dst.data(), src, n * sizeof(T));
        return hipSuccess;
    }
    return hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost);
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

int ceil_log2(int64_t v)
{
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

static_assert(hs::kAdjRounds == HS_ADJ_ROUNDS && hs::kAdjDataflow == HS_ADJ_DATAFLOW &&
                  hs::kAdjAnchors == HS_ADJ_ANCHORS,
              "adjoint kinds");
static_assert(hs::kStatusWaitTimeout == HS_DEV_WAIT_TIMEOUT && hs::kStatusTopology == HS_DEV_TOPOLOGY, "status bits");

struct Shape {
    int tile_cap = 0;
    int waves = 0;
    int grid_per_cu = 0;  // 0 = one workgroup per tile
    bool chain_units = false;
    int algorithm = HS_ALG_SCAN;
    int adjoint = HS_ADJ_ROUNDS;
    int queue_waves = 0;  // > 0: the forward runs as one work-queue launch with this many waves
    int queue_cap = 0;    // work queue: tile capacity when it differs from tile_cap (0: tile_cap)
};

} // namespace

struct hs_context {
    int device = 0;
    int num_cu = 0;
    size_t max_lds = 0;
    std::string arch;
    std::mutex mu;
    std::map<std::string, Shape> tuned;  // autotuning cache keyed by arch + size class
    std::string tune_file;               // HS_TUNE_CACHE: where tuning results persist
    float4 *noalloc_ws = nullptr;        // this device's static workspace (hs_pose_sample_backward_noalloc)
};

namespace {

// ---------------------------------------------------------------------------
// The autotuning cache as JSON (hs_context_load_tuning / _save_tuning).  A
// small reader for the one shape the file has: an object whose "entries"
// member maps keys to objects of integer fields; unknown members are
// skipped.
// ---------------------------------------------------------------------------
struct JsonReader {
    const std::string &t;
    size_t i = 0;
    explicit JsonReader(const std::string &text) : t(text) {}
    void ws()
    {
        while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\r' || t[i] == '\t')) ++i;
    }
    bool eat(char c)
    {
        ws();
        if (i < t.size() && t[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string &out)
    {
        ws();
        if (i >= t.size() || t[i] != '"') return false;
        out.clear();
        for (++i; i < t.size() && t[i] != '"'; ++i) {
            if (t[i] == '\\') {
                if (++i >= t.size()) return false;
            }
            out.push_back(t[i]);
        }
        return i++ < t.size();
    }
    bool integer(long long &v)
    {
        ws();
        const char *b = t.c_str() + i;
        char *e = nullptr;
        v = std::strtoll(b, &e, 10);
        if (e == b) return false;
        i += (size_t)(e - b);
        return true;
    }
    // skips one value of any kind
    bool skip()
    {
        ws();
        if (i >= t.size()) return false;
        if (t[i] == '"') {
            std::string d;
            return str(d);
        }
        if (t[i] == '{' || t[i] == '[') {
            const char close = t[i] == '{' ? '}' : ']';
            ++i;
            if (eat(close)) return true;
            do {
                if (close == '}') {
                    std::string k;
                    if (!str(k) || !eat(':')) return false;
                }
                if (!skip()) return false;
            } while (eat(','));
            return eat(close);
        }
        while (i < t.size() && std::strchr(",}] \n\r\t", t[i]) == nullptr) ++i;
        return true;
    }
};

bool parse_shape(JsonReader &r, Shape &sh)
{
    if (!r.eat('{')) return false;
    if (r.eat('}')) return false;
    bool cap = false;
    do {
        std::string k;
        long long v = 0;
        if (!r.str(k) || !r.eat(':')) return false;
        if (k == "tile_cap" || k == "waves" || k == "grid_per_cu" || k == "chain_units" || k == "queue_waves") {
            if (!r.integer(v)) return false;
            if (k == "tile_cap") {
                if (v < 64 || v > hs::kMaxTileJoints || v % 64) return false;
                sh.tile_cap = (int)v;
                cap = true;
            } else if (k == "waves" || k == "queue_waves") {
                if (v < (k == "waves" ? 1 : 0) || v > 16 || (v & (v - 1))) return false;
                (k == "waves" ? sh.waves : sh.queue_waves) = (int)v;
            } else if (k == "grid_per_cu") {
                if (v < 0 || v > 64) return false;
                sh.grid_per_cu = (int)v;
            } else {
                if (v != 0 && v != 1) return false;
                sh.chain_units = v != 0;
            }
        } else if (!r.skip()) {
            return false;
        }
    } while (r.eat(','));
    return r.eat('}') && cap && sh.waves >= 1 && !(sh.chain_units && sh.queue_waves);
}

// Parses a cache file's text; false (and nothing in `out`) if malformed.
bool parse_tuning(const std::string &text, std::map<std::string, Shape> &out)
{
    JsonReader r(text);
    std::map<std::string, Shape> got;
    if (!r.eat('{')) return false;
    if (!r.eat('}')) {
        do {
            std::string k;
            if (!r.str(k) || !r.eat(':')) return false;
            if (k == "entries") {
                if (!r.eat('{')) return false;
                if (!r.eat('}')) {
                    do {
                        std::string key;
                        Shape sh;
                        if (!r.str(key) || !r.eat(':') || !parse_shape(r, sh)) return false;
                        got[key] = sh;
                    } while (r.eat(','));
                    if (!r.eat('}')) return false;
                }
            } else if (!r.skip()) {
                return false;
            }
        } while (r.eat(','));
        if (!r.eat('}')) return false;
    }
    r.ws();
    if (r.i != text.size()) return false;
    out = got;
    return true;
}

std::string format_tuning(const std::map<std::string, Shape> &tuned)
{
    std::string o = "{\"version\": 1, \"entries\": {";
    bool first = true;
    char buf[256];
    for (const auto &kv : tuned) {
        std::string key;
        for (char c : kv.first) {
            if (c == '"' || c == '\\') key.push_back('\\');
            key.push_back(c);
        }
        const Shape &sh = kv.second;
        snprintf(buf, sizeof buf,
                 "\"tile_cap\": %d, \"waves\": %d, \"grid_per_cu\": %d, \"chain_units\": %d, \"queue_waves\": %d",
                 sh.tile_cap, sh.waves, sh.grid_per_cu, sh.chain_units ? 1 : 0, sh.queue_waves);
        o += (first ? "\n  \"" : ",\n  \"") + key + "\": {" + buf + "}";
        first = false;
    }
    o += first ? "}}\n" : "\n}}\n";
    return o;
}

hs_status load_tuning_file(hs_context *ctx, const char *path)
{
    FILE *f = std::fopen(path, "rb");
    if (!f) return HS_OK;  // nothing tuned yet
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    std::map<std::string, Shape> got;
    if (!parse_tuning(text, got)) return fail(HS_ERR_INVALID_ARG, "tuning cache %s is malformed", path);
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const auto &kv : got) ctx->tuned[kv.first] = kv.second;
    return HS_OK;
}

hs_status save_tuning_file(const hs_context *ctx, const char *path)
{
    std::string text;
    {
        std::lock_guard<std::mutex> lk(const_cast<hs_context *>(ctx)->mu);
        text = format_tuning(ctx->tuned);
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(HS_ERR_INVALID_ARG, "cannot write tuning cache %s", tmp.c_str());
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(HS_ERR_INVALID_ARG, "cannot write tuning cache %s", path);
    }
    return HS_OK;
}

} // namespace

// Device tables and workspace of the multipass path.
struct MPSet {
    MPBlock *d_blocks = nullptr;
    int32_t num_blocks = 0;
    int64_t nmp = 0;
    int32_t *d_janc = nullptr;
    int32_t *d_aself = nullptr;  // each joint's own anchor index, or -1
    int32_t *d_aseg = nullptr;   // in-LDS segments of the anchor rounds (offsets)
    int32_t num_aseg = 0;
    int32_t num_anchors = 0;
    int32_t rounds = 0;        // anchor-level jump rounds
    float4 *A1 = nullptr;      // anchors' phase-1 products
    int32_t *E1 = nullptr;
    float4 *AP[2] = {nullptr, nullptr};
    int32_t *AE[2] = {nullptr, nullptr};
    // adjoint: anchor adjoints, compact G
    float4 *S[2] = {nullptr, nullptr};
    float4 *G = nullptr;
    // the one-pass chain path (forward set only): chain characters' blocks
    // and superblocks, their workspace, and the resident grid per pose kind
    hs::ChainBlock *d_cblocks = nullptr;
    int32_t num_cblocks = 0;
    hs::ChainSB *d_csb = nullptr;
    int32_t num_csb = 0;
    int64_t chain_joints = 0;
    uint64_t *c_recs = nullptr;
    uint32_t *c_epoch = nullptr;
    int32_t c_grid[2] = {0, 0};
};

void free_mpset(MPSet &m)
{
    (void)hipFree(m.d_blocks);
    (void)hipFree(m.d_janc);
    (void)hipFree(m.d_aself);
    (void)hipFree(m.d_aseg);
    (void)hipFree(m.A1);
    (void)hipFree(m.E1);
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(m.AP[i]);
        (void)hipFree(m.AE[i]);
        (void)hipFree(m.S[i]);
    }
    (void)hipFree(m.G);
    (void)hipFree(m.d_cblocks);
    (void)hipFree(m.d_csb);
    (void)hipFree(m.c_recs);
    (void)hipFree(m.c_epoch);
    m = MPSet{};
}

struct hs_plan {
    hs_context *ctx = nullptr;
    int64_t C = 0, N = 0;
    std::vector<int64_t> h_offsets;
    std::vector<int32_t> h_parents;  // character-local
    std::vector<int32_t> h_gparent;  // global parent id or -1
    hs_plan_info info{};
    Shape shape;
    // device tables
    int64_t *d_offsets = nullptr;
    int32_t *d_parent = nullptr;  // global parent id or -1
    int32_t *d_level = nullptr;
    TileDesc *d_tiles = nullptr;
    std::vector<TileDesc> h_tiles;
    int32_t main_grid = 0;
    // smaller characters on smaller tiles of their own (more workgroups per
    // CU), launched before the main set: {tiles, count, cap, waves, grid}
    struct ClassSet {
        TileDesc *d_tiles = nullptr;
        int32_t num_tiles = 0, cap = 0, waves = 0, grid = 0;
    };
    std::vector<ClassSet> small;
    // adjoint tiles: characters of up to 1024 joints (synchronous-round
    // kernel) and larger ones up to the dataflow kernel's limit
    TileDesc *d_btiles = nullptr;
    std::vector<TileDesc> h_btiles;
    int32_t num_btiles = 0;
    int32_t bwd_cap = 0;
    TileDesc *d_bbig = nullptr;
    int32_t num_bbig = 0;
    int32_t *d_bcode = nullptr;  // anchor codes of the adjoint tiles' joints
    int32_t b_max_anchors = 0;
    bool b_anchor_ok = false;    // the two-level adjoint fits the LDS
    int b_bpw_opt = 0;           // the two-level adjoint's blocks per wave as asked (0 = choose)
    int b_bpw[3] = {1, 1, 1};    // ... as chosen, per seed kind (dense, effectors, forward in the tile)
    int64_t bwd_untiled = 0;  // joints the adjoint's tiles do not cover
    int32_t max_units = 0;
    // multipass: characters larger than the forward tile (mp) and than the
    // adjoint tile (bmp, with the adjoint workspace)
    MPSet mp, bmp;
    std::vector<int32_t> h_level;
    // instanced plans: skeleton-local parents and each character's first
    // skeleton joint (the forward tiles read these instead of d_parent)
    bool inst = false;
    int64_t skel_joints = 0;
    int32_t *d_skel_parent = nullptr;
    int32_t *d_char_skel = nullptr;
    // device status word (bits, lowest failing joint) and the polls of the
    // kernels' bounded waits
    uint32_t *d_status = nullptr;
    int32_t spin_limit = hs::kDefaultSpinLimit;
    // the forward's work queue (schedule HS_SCHED_QUEUE): tiles heaviest
    // first and per-joint codes; num_tiles = 0 when the forward launches the
    // size classes instead
    struct QueueSet {
        hs::QTile *d_tiles = nullptr;
        int32_t num_tiles = 0, grid = 0, waves = 0, max_anchors = 0, cap = 0;
        int32_t grids[2][2] = {{0, 0}, {0, 0}};  // by [sampled poses][skin rows]
        int32_t *d_code = nullptr;
    } q;
    int sched_opt = HS_SCHED_AUTO;
};

namespace {

void free_plan(hs_plan *p)
{
    if (!p) return;
    (void)hipFree(p->d_offsets);
    (void)hipFree(p->d_parent);
    (void)hipFree(p->d_level);
    (void)hipFree(p->d_tiles);
    for (auto &c : p->small) (void)hipFree(c.d_tiles);
    (void)hipFree(p->d_btiles);
    (void)hipFree(p->d_bbig);
    free_mpset(p->mp);
    free_mpset(p->bmp);
    (void)hipFree(p->d_skel_parent);
    (void)hipFree(p->d_char_skel);
    (void)hipFree(p->d_status);
    (void)hipFree(p->q.d_tiles);
    (void)hipFree(p->q.d_code);
    (void)hipFree(p->d_bcode);
    delete p;
}

// RAII guard that makes the plan's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Length of the longest chain of 64-joint blocks along any root-to-joint path
// of one character (ids relative to `base`, blocks aligned to `align0`).
int block_chain_length(const int32_t *par, int64_t n, int64_t align0, std::vector<int32_t> &top,
                       std::vector<int32_t> &chain)
{
    top.resize(n);
    chain.resize(n);
    int best = 0;
    for (int64_t j = 0; j < n; ++j) {
        const int32_t p = par[j];
        const int64_t bj = (j + align0) / 64;
        if (p >= 0 && (p + align0) / 64 == bj) {
            top[j] = top[p];
            chain[j] = chain[p];
        } else {
            top[j] = (int32_t)j;
            chain[j] = p < 0 ? 1 : chain[p] + 1;
        }
        best = std::max(best, (int)chain[j]);
    }
    return best;
}

// Mark the chain units of a tile: runs of up to 4 blocks (at least 2) in
// which every joint's parent is the previous joint or lies before the run,
// and whose longest chain segment has at least 16 joints (below that the
// per-block doubling needs no more than 4 rounds and is cheaper).
int mark_chain_units(const std::vector<int32_t> &gparent, TileDesc &t)
{
    int units = 0;
    const int n = t.count;
    const int nblk = (n + 63) / 64;
    uint64_t mask = 0;
    for (int b = 0; b < nblk;) {
        const int e = std::min(b + 4, nblk);
        bool ok = e - b >= 2;
        int longest = 0, seg = 0;
        for (int j = 64 * b; ok && j < std::min(64 * e, n); ++j) {
            const int32_t pg = gparent[t.begin + j];
            const int64_t p = pg < 0 ? -1 : (int64_t)pg - t.begin;
            if (p == j - 1 && p >= 64 * b) {
                ++seg;
            } else if (p < 64 * b) {
                seg = 1;
            } else {
                ok = false;
            }
            longest = std::max(longest, seg);
        }
        if (ok && longest >= 16) {
            mask |= uint64_t(1) << b;
            b = e;
        } else {
            ++b;
        }
        ++units;
    }
    t.chain_lo = (int32_t)(uint32_t)(mask & 0xffffffffu);
    t.chain_hi = (int32_t)(uint32_t)(mask >> 32);
    return units;
}

struct Packing {
    std::vector<TileDesc> tiles;  // sorted, heaviest first
    std::vector<MPBlock> mpb;
    std::vector<int64_t> chains;  // one-pass chain characters (when asked for)
    int64_t nmp = 0, tiled = 0;
    int max_chain_tiles = 0, max_chain_mp = 0;
    int max_units = 0;  // most work units (blocks or chain units) in one tile
};

// Pack whole characters, in order, into tiles of at most `cap` joints; the
// characters that do not fit go to the multipass path.  Only characters of
// lo..hi joints are taken; the others are left out (another packing covers
// them).
Packing pack_tiles(const hs_plan *plan, int cap, int strategy, bool chain_units, int64_t lo = 0,
                   int64_t hi = INT64_MAX, bool chain_pass = false)
{
    const int64_t C = plan->C;
    const auto &off = plan->h_offsets;
    const auto &par = plan->h_parents;
    Packing pk;
    std::vector<TileDesc> tiles;
    std::vector<int64_t> tile_cost;
    std::vector<int32_t> top, chain;

    TileDesc cur{};
    bool open = false;
    int cur_chain = 0;
    int32_t cur_level = 1;
    auto flush = [&]() {
        if (open && cur.count > 0) {
            cur.rounds = ceil_log2(cur_level);
            tiles.push_back(cur);
            tile_cost.push_back((int64_t)cur.count + 48 * (int64_t)cur_chain);
            pk.max_chain_tiles = std::max(pk.max_chain_tiles, cur_chain);
        }
        open = false;
        cur_chain = 0;
        cur_level = 1;
    };
    for (int64_t c = 0; c < C; ++c) {
        const int64_t n = off[c + 1] - off[c];
        if (n < lo || n > hi) {
            flush();  // tiles are contiguous id ranges
            continue;
        }
        const bool to_mp = strategy == HS_STRATEGY_MULTIPASS || n > cap;
        if (to_mp) {
            flush();
            if (n == 0) continue;
            if (chain_pass) {
                // every parent the previous joint: the one-pass chain path
                const int32_t *pc = par.data() + off[c];
                bool chain = pc[0] == -1;
                for (int64_t j = 1; j < n && chain; ++j) chain = pc[j] == j - 1;
                if (chain) {
                    pk.chains.push_back(c);
                    continue;
                }
            }
            const int L = block_chain_length(par.data() + off[c], n, 0, top, chain);
            pk.max_chain_mp = std::max(pk.max_chain_mp, L);
            for (int64_t k = 0; k < n; k += 64) {
                MPBlock b{};
                b.gbegin = off[c] + k;
                b.cbegin = pk.nmp + k;
                b.count = (int32_t)std::min<int64_t>(64, n - k);
                b.chr = (int32_t)c;
                pk.mpb.push_back(b);
            }
            pk.nmp += n;
            continue;
        }
        if (!open) {
            if (n == 0) continue;
            cur = TileDesc{};
            cur.begin = off[c];
            cur.first_char = (int32_t)c;
            open = true;
        } else if (cur.count + n > cap || cur.num_chars + 1 > cap) {
            // a tile holds at most `cap` joints and `cap` characters (empty
            // characters inside a tile still take a slot of its LDS table)
            flush();
            cur = TileDesc{};
            cur.begin = off[c];
            cur.first_char = (int32_t)c;
            open = true;
        }
        if (n > 0) {
            const int L = block_chain_length(par.data() + off[c], n, cur.count, top, chain);
            cur_chain = std::max(cur_chain, L);
            for (int64_t j = off[c]; j < off[c + 1]; ++j) cur_level = std::max(cur_level, plan->h_level[j]);
        }
        cur.count += (int32_t)n;
        cur.num_chars += 1;
        pk.tiled += n;
    }
    flush();

    // heaviest tiles first: the hardware dispatches workgroups in order, so
    // long serial block chains start early instead of trailing the launch
    std::vector<size_t> order(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return tile_cost[a] > tile_cost[b]; });
    pk.tiles.resize(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) pk.tiles[i] = tiles[order[i]];
    for (TileDesc &t : pk.tiles) {
        const int units = chain_units ? mark_chain_units(plan->h_gparent, t) : (t.count + 63) / 64;
        pk.max_units = std::max(pk.max_units, units);
    }
    return pk;
}

// Upload a packing's multipass blocks and allocate the path's workspace
// (and the adjoint's, if asked).
// Anchors of the multipass characters: e(c), the nearest out-of-block
// ancestor of compact joint c (one pass in joint order: the parent's own
// e when the parent lies in the same block); the anchors are the distinct
// e values, janc(c) is the index of e(c) among them, and the anchor-level
// rounds cover the longest anchor chain.
void build_anchors(const hs_plan *plan, const Packing &pk, std::vector<int32_t> &janc,
                   std::vector<int32_t> &anchors, int &rounds)
{
    const auto &gpar = plan->h_gparent;
    std::vector<int32_t> e((size_t)pk.nmp, -1);
    for (const MPBlock &bd : pk.mpb)
        for (int l = 0; l < bd.count; ++l) {
            const int64_t g = bd.gbegin + l, c = bd.cbegin + l;
            const int64_t p = gpar[g];
            if (p < 0) e[c] = -1;
            else if (p >= bd.gbegin) e[c] = e[bd.cbegin + (p - bd.gbegin)];
            else e[c] = (int32_t)(bd.cbegin + (p - bd.gbegin));  // same character, earlier block
        }
    std::vector<int32_t> aidx((size_t)pk.nmp, -1);
    for (int64_t c = 0; c < pk.nmp; ++c)
        if (e[c] >= 0) aidx[e[c]] = 0;
    anchors.clear();
    for (int64_t c = 0; c < pk.nmp; ++c)
        if (aidx[c] == 0) {
            aidx[c] = (int32_t)anchors.size();
            anchors.push_back((int32_t)c);
        }
    janc.assign((size_t)pk.nmp, -1);
    for (int64_t c = 0; c < pk.nmp; ++c) janc[c] = e[c] >= 0 ? aidx[e[c]] : -1;
    // anchors come in joint order and e(a) < a, so a chain's depth is known
    // when its anchor is reached
    std::vector<int32_t> depth(anchors.size(), 1);
    int maxd = 1;
    for (size_t i = 0; i < anchors.size(); ++i) {
        const int32_t j = janc[anchors[i]];
        depth[i] = j < 0 ? 1 : depth[j] + 1;
        maxd = std::max(maxd, depth[i]);
    }
    rounds = ceil_log2(maxd);
}

// Upload a packing's multipass blocks and anchors and allocate the path's
// workspace (and the adjoint's, if asked).
// The one-pass chain path's tables and workspace: each chain character in
// 64-joint blocks, up to 64 consecutive blocks of one chain per
// superblock; the grid is the workgroups resident at once.
hs_status make_chains(MPSet &m, const hs_plan *plan, const Packing &pk)
{
    if (pk.chains.empty()) return HS_OK;
    std::vector<hs::ChainBlock> cb;
    std::vector<hs::ChainSB> sbs;
    for (int64_t c : pk.chains) {
        const int64_t b0 = plan->h_offsets[c], n = plan->h_offsets[c + 1] - b0;
        const int32_t first_sb = (int32_t)sbs.size();
        for (int64_t k = 0; k < n; k += 64) {
            const int64_t blk = k / 64;
            if (blk % hs::kChainSBBlocks == 0) sbs.push_back(hs::ChainSB{(int32_t)cb.size(), 0, first_sb, 0});
            hs::ChainBlock b{};
            b.gbegin = b0 + k;
            b.count = (int32_t)std::min<int64_t>(64, n - k);
            b.sb = (int32_t)sbs.size() - 1;
            b.k = sbs.back().nblk++;
            b.chr = (int32_t)c;
            cb.push_back(b);
        }
        m.chain_joints += n;
    }
    if (cb.size() > (size_t)INT32_MAX / 4) return fail(HS_ERR_UNSUPPORTED, "too many chain blocks");
    m.num_cblocks = (int32_t)cb.size();
    m.num_csb = (int32_t)sbs.size();
    for (int smp = 0; smp < 2; ++smp) {
        int per_cu = 0;
        hipError_t e = hs::chain_blocks_per_cu(smp != 0, &per_cu);
        if (e != hipSuccess) return fail_hip(e, "hs_plan_create (chain occupancy)");
        if (per_cu < 1) return fail(HS_ERR_UNSUPPORTED, "the chain kernel does not fit a CU");
        m.c_grid[smp] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(m.num_csb, (int64_t)per_cu * plan->ctx->num_cu));
    }
    const size_t ns = (size_t)m.num_csb;
    hipError_t err = upload(&m.d_cblocks, cb);
    if (err == hipSuccess) err = upload(&m.d_csb, sbs);
    if (err == hipSuccess) err = hipMalloc(&m.c_recs, ns * 12 * sizeof(uint64_t));
    if (err == hipSuccess) err = hipMalloc(&m.c_epoch, 2 * sizeof(uint32_t));
    // records and epoch start at zero once; each call then tags its
    // publications with the next epoch (no clearing per call)
    if (err == hipSuccess) err = hipMemset(m.c_recs, 0, ns * 12 * sizeof(uint64_t));
    if (err == hipSuccess) err = hipMemset(m.c_epoch, 0, 2 * sizeof(uint32_t));
    if (err == hipSuccess) err = hipDeviceSynchronize();
    if (err != hipSuccess) return fail_hip(err, "hs_plan_create (chain workspace)");
    return HS_OK;
}

hs_status make_mpset(MPSet &m, const hs_plan *plan, const Packing &pk, bool adjoint)
{
    free_mpset(m);
    m.num_blocks = (int32_t)pk.mpb.size();
    m.nmp = pk.nmp;
    if (!adjoint) {
        hs_status rc = make_chains(m, plan, pk);
        if (rc != HS_OK) {
            free_mpset(m);
            return rc;
        }
    }
    if (pk.nmp == 0) return HS_OK;
    std::vector<int32_t> janc, anchors;
    build_anchors(plan, pk, janc, anchors, m.rounds);
    m.num_anchors = (int32_t)anchors.size();
    std::vector<int32_t> aself((size_t)pk.nmp, -1);
    for (size_t i = 0; i < anchors.size(); ++i) aself[anchors[i]] = (int32_t)i;
    // Segments for the in-LDS anchor rounds: a cut before anchor k is valid
    // when no anchor from k on points below k (anchors point to earlier
    // anchors of their character); segments take the furthest valid cut
    // within kAnchorSegCap anchors.  If some stretch has no valid cut that
    // close, the rounds stay global.
    std::vector<int32_t> aseg;
    {
        const int64_t na = (int64_t)anchors.size();
        std::vector<int64_t> sufmin((size_t)na + 1, INT64_MAX);
        for (int64_t i = na - 1; i >= 0; --i) {
            const int32_t pa = janc[anchors[i]];
            sufmin[i] = std::min<int64_t>(sufmin[i + 1], pa < 0 ? INT64_MAX : pa);
        }
        aseg.push_back(0);
        int64_t s = 0;
        while (s < na) {
            int64_t k = std::min<int64_t>(na, s + hs::kAnchorSegCap);
            while (k > s && !(k == na || sufmin[k] >= k)) --k;
            if (k == s) {
                aseg.clear();
                break;
            }
            aseg.push_back((int32_t)k);
            s = k;
        }
        if (aseg.size() < 2 || m.rounds == 0) aseg.clear();
        m.num_aseg = aseg.empty() ? 0 : (int32_t)aseg.size() - 1;
    }
    hipError_t err = upload(&m.d_blocks, pk.mpb);
    if (err == hipSuccess) err = upload(&m.d_aseg, aseg);
    if (err == hipSuccess) err = upload(&m.d_janc, janc);
    if (err == hipSuccess) err = upload(&m.d_aself, aself);
    const size_t n = (size_t)pk.nmp, na = std::max<size_t>(1, anchors.size());
    if (err == hipSuccess) err = hipMalloc(&m.A1, na * 3 * sizeof(float4));
    if (err == hipSuccess) err = hipMalloc(&m.E1, na * sizeof(int32_t));
    for (int i = 0; i < 2 && err == hipSuccess; ++i) {
        err = hipMalloc(&m.AP[i], na * 3 * sizeof(float4));
        if (err == hipSuccess) err = hipMalloc(&m.AE[i], na * sizeof(int32_t));
        if (adjoint && err == hipSuccess) err = hipMalloc(&m.S[i], na * 3 * sizeof(float4));
    }
    if (adjoint && err == hipSuccess) err = hipMalloc(&m.G, n * 3 * sizeof(float4));
    // anchor pointers start as "none": the rounds index with them, so they
    // never hold uninitialised values (even if a validating call's check
    // keeps the first pass from writing them)
    if (err == hipSuccess) err = hipMemset(m.E1, 0xFF, na * sizeof(int32_t));
    for (int i = 0; i < 2 && err == hipSuccess; ++i) err = hipMemset(m.AE[i], 0xFF, na * sizeof(int32_t));
    if (err != hipSuccess) {
        free_mpset(m);
        return fail_hip(err, "hs_plan_create (multipass workspace)");
    }
    return HS_OK;
}

// The forward's work queue: every character of at most `cap` joints, in
// id order, on tiles of at most `cap` joints, heaviest first.  A tile's
// anchors are the parents of its joints that lie in another 64-joint
// block; they get LDS slots in joint order, and every joint a code naming
// its in-block parent lane or its parent's slot, and its own slot.
// Returns false (nothing built) when the anchors of some tile would not
// fit the LDS.
// Anchor slots and per-joint codes (the layout of hs::QueueLaunch::code) of
// a tile: the anchors are the parents of the tile's joints that lie in
// another 64-joint block (blocks counted from the tile's first joint),
// numbered in joint order.  Writes the codes of the tile's joints into
// `code` and returns the tile's anchor count.
int tile_codes(const hs_plan *plan, const TileDesc &t, std::vector<int32_t> &code, std::vector<int32_t> &slot)
{
    const auto &gpar = plan->h_gparent;
    slot.assign((size_t)t.count, 0);
    for (int jl = 0; jl < t.count; ++jl) {
        const int32_t pg = gpar[t.begin + jl];
        if (pg >= 0 && (pg - t.begin) / 64 != jl / 64) slot[pg - t.begin] = 1;
    }
    int na = 0;
    for (int jl = 0; jl < t.count; ++jl) slot[jl] = slot[jl] ? ++na : 0;  // 1 + slot, or 0
    for (int jl = 0; jl < t.count; ++jl) {
        const int32_t pg = gpar[t.begin + jl];
        const int base = jl & ~63;
        int c = 0;
        if (pg >= 0) {
            const int pl = (int)(pg - t.begin);
            c = pl >= base ? (hs::kQInBlock | (pl - base)) : slot[pl];
        }
        code[t.begin + jl] = c | (slot[jl] << hs::kQOwnShift);
    }
    return na;
}

hs_status build_queue(hs_plan *plan, const Shape &shape, int strategy, bool *built)
{
    *built = false;
    auto &Q = plan->q;
    (void)hipFree(Q.d_tiles);
    (void)hipFree(Q.d_code);
    Q.d_tiles = nullptr;
    Q.d_code = nullptr;
    Q.num_tiles = Q.grid = Q.max_anchors = 0;
    const int cap = shape.queue_cap > 0 ? shape.queue_cap : shape.tile_cap;
    const Packing pk = pack_tiles(plan, cap, strategy, false, 0, cap);
    std::vector<hs::QTile> qt(pk.tiles.size());
    std::vector<int32_t> code((size_t)plan->N, 0), slot;
    int max_anchors = 0;
    for (size_t i = 0; i < pk.tiles.size(); ++i) {
        const TileDesc &t = pk.tiles[i];
        const int na = tile_codes(plan, t, code, slot);
        hs::QTile &q = qt[i];
        q = hs::QTile{};
        q.begin = t.begin;
        q.count = t.count;
        q.first_char = t.first_char;
        q.num_chars = t.num_chars;
        q.num_anchors = na;
        max_anchors = std::max(max_anchors, na);
    }
    const int waves = shape.queue_waves;
    const size_t lds_max = hs::forward_queue_lds_bytes(waves, max_anchors, cap, true, true);
    if (max_anchors > hs::kQMaxAnchors || cap > hs::kQMaxTileJoints || lds_max > plan->ctx->max_lds) return HS_OK;
    hipError_t err = upload(&Q.d_tiles, qt);
    if (err == hipSuccess) err = upload(&Q.d_code, code);
    if (err != hipSuccess) return fail_hip(err, "hs_plan_create (work queue)");
    Q.num_tiles = (int32_t)qt.size();
    Q.max_anchors = max_anchors;
    Q.cap = cap;
    Q.waves = waves;
    // as many workgroups as fit the CUs at once (each pose source has its
    // own instance, registers and LDS)
    for (int smp = 0; smp < 2; ++smp)
        for (int skin = 0; skin < 2; ++skin) {
            int per_cu = 1;
            const size_t lds = hs::forward_queue_lds_bytes(waves, max_anchors, cap, smp != 0, skin != 0);
            if ((err = hs::queue_blocks_per_cu(waves, smp != 0, skin != 0, lds, &per_cu)) != hipSuccess)
                return fail_hip(err, "hs_plan_create (work-queue occupancy)");
            // grid_per_cu 0: one workgroup per tile, dispatched by the
            // hardware as CUs free up; k > 0: at most k resident workgroups
            // per CU, each walking the list
            per_cu = std::max(1, std::min(per_cu, std::max(1, shape.grid_per_cu)));
            Q.grids[smp][skin] =
                shape.grid_per_cu > 0
                    ? (int32_t)std::max<int64_t>(1, std::min<int64_t>(Q.num_tiles, (int64_t)per_cu * plan->ctx->num_cu))
                    : std::max<int32_t>(1, Q.num_tiles);
        }
    Q.grid = Q.grids[0][0];
    *built = true;
    return HS_OK;
}

hs_status build_tables(hs_plan *plan, const Shape &shape, int strategy)
{
    const int cap = shape.tile_cap;
    const int ncu = plan->ctx->num_cu;
    auto grid_of = [&](size_t ntiles) {
        return shape.grid_per_cu > 0 ? (int32_t)std::min<int64_t>(ntiles, (int64_t)shape.grid_per_cu * ncu)
                                     : (int32_t)ntiles;
    };
    // Size classes: with tiles larger than 1024 joints, characters of up to
    // 1024 joints get 1024-joint tiles (8 waves; three workgroups fit a CU)
    // and, under 1664-joint tiles or larger, characters of 1025-1664 joints
    // get 1664-joint tiles (16 waves; two per CU).  The main set holds the
    // rest.  Each set is one launch with its own LDS size.
    for (auto &c : plan->small) (void)hipFree(c.d_tiles);
    plan->small.clear();
    int64_t main_lo = 0;
    int64_t small_tiled = 0;
    int32_t small_tiles = 0, small_grid = 0;
    if (strategy != HS_STRATEGY_MULTIPASS && cap > 1024) {
        struct Cls { int64_t lo, hi; int cap, waves; };
        std::vector<Cls> cls = {{0, 1024, 1024, 8}};
        if (cap > 1664) cls.push_back({1025, 1664, 1664, 16});
        for (const Cls &c : cls) {
            Packing ps = pack_tiles(plan, c.cap, strategy, shape.chain_units, c.lo, c.hi);
            main_lo = c.hi + 1;
            if (ps.tiles.empty()) continue;
            hs_plan::ClassSet cs;
            cs.num_tiles = (int32_t)ps.tiles.size();
            cs.cap = c.cap;
            cs.waves = c.waves;
            cs.grid = grid_of(ps.tiles.size());
            hipError_t e0 = upload(&cs.d_tiles, ps.tiles);
            if (e0 != hipSuccess) return fail_hip(e0, "hs_plan_create");
            plan->small.push_back(cs);
            small_tiled += ps.tiled;
            small_tiles += cs.num_tiles;
            small_grid += cs.grid;
        }
    }
    Packing pk = pack_tiles(plan, cap, strategy, shape.chain_units, main_lo, INT64_MAX, true);
    std::vector<TileDesc> &sorted = pk.tiles;
    const int64_t nmp = pk.nmp, tiled = pk.tiled + small_tiled;
    const int max_chain_tiles = pk.max_chain_tiles, max_chain_mp = pk.max_chain_mp;

    // The adjoint gets tiles of its own.  Characters of up to 1024 joints go
    // to the synchronous-round kernel, on tiles just large enough for the
    // largest of them but at least 256 joints (4 waves: many workgroups per
    // CU; measured against 512 joints: 179 vs 195 us on 10 000 x 256 joints,
    // 12 vs 20 us on 64 x 64); characters of up to 1664 joints to the
    // dataflow kernel; the rest to the multipass adjoint.
    (void)hipFree(plan->d_btiles);
    (void)hipFree(plan->d_bbig);
    plan->d_btiles = plan->d_bbig = nullptr;
    plan->num_btiles = plan->num_bbig = 0;
    {
        int64_t m_sync = 0;
        for (int64_t c = 0; c < plan->C; ++c) {
            const int64_t n = plan->h_offsets[c + 1] - plan->h_offsets[c];
            if (n <= hs::kMaxSyncTileJoints) m_sync = std::max(m_sync, n);
        }
        plan->bwd_cap = std::max(256, round_up((int)m_sync, 64));
        const bool mp_all = strategy == HS_STRATEGY_MULTIPASS;
        Packing ps, pb;
        if (!mp_all) ps = pack_tiles(plan, plan->bwd_cap, strategy, false, 0, hs::kMaxSyncTileJoints);
        pb = pack_tiles(plan, hs::kMaxBwdTileJoints, strategy, false, mp_all ? 0 : hs::kMaxSyncTileJoints + 1);
        plan->num_btiles = (int32_t)ps.tiles.size();
        plan->h_btiles = ps.tiles;
        // anchor codes of the adjoint tiles (the two-level adjoint)
        (void)hipFree(plan->d_bcode);
        plan->d_bcode = nullptr;
        plan->b_max_anchors = 0;
        plan->b_anchor_ok = false;
        if (!ps.tiles.empty()) {
            std::vector<int32_t> code((size_t)plan->N, 0), slot;
            for (const TileDesc &t : ps.tiles)
                plan->b_max_anchors = std::max(plan->b_max_anchors, tile_codes(plan, t, code, slot));
            int w = 1;
            while (w * 64 < plan->bwd_cap) w *= 2;
            const size_t lds1 = hs::backward_anchor_lds_bytes(w, plan->b_max_anchors, plan->bwd_cap);
            const size_t lds2 = hs::backward_anchor_lds_bytes(std::max(1, w / 2), plan->b_max_anchors, plan->bwd_cap);
            const int64_t tiles = (int64_t)ps.tiles.size();
            const int nc = std::max(1, plan->ctx->num_cu);
            plan->b_anchor_ok = plan->b_max_anchors <= hs::kQMaxAnchors && lds1 <= plan->ctx->max_lds;
            // blocks per wave, per seed kind: two when the resident
            // workgroups then cover the tiles in fewer rounds (the adjoint
            // is latency-bound, so a round costs about one tile's time)
            for (int kind = 0; kind < 3 && plan->b_anchor_ok; ++kind) {
                int occ1 = 0, occ2 = 0;
                hipError_t e4 = hs::anchor_blocks_per_cu(w, 1, kind, lds1, &occ1);
                if (e4 == hipSuccess && w >= 2) e4 = hs::anchor_blocks_per_cu(w / 2, 2, kind, lds2, &occ2);
                if (e4 != hipSuccess) return fail_hip(e4, "hs_plan_create (adjoint occupancy)");
                const int64_t r1 = occ1 > 0 ? (tiles + (int64_t)occ1 * nc - 1) / ((int64_t)occ1 * nc) : INT64_MAX;
                const int64_t r2 = occ2 > 0 ? (tiles + (int64_t)occ2 * nc - 1) / ((int64_t)occ2 * nc) : INT64_MAX;
                int bpw = r2 < r1 ? 2 : 1;
                if (plan->b_bpw_opt == 2 && w >= 2 && occ2 > 0) bpw = 2;
                if (plan->b_bpw_opt == 1 && occ1 > 0) bpw = 1;
                if (bpw == 1 && occ1 == 0) plan->b_anchor_ok = false;
                plan->b_bpw[kind] = bpw;
            }
            hipError_t e3 = upload(&plan->d_bcode, code);
            if (e3 != hipSuccess) return fail_hip(e3, "hs_plan_create (adjoint codes)");
        }
        plan->num_bbig = (int32_t)pb.tiles.size();
        hipError_t e2 = upload(&plan->d_btiles, ps.tiles);
        if (e2 == hipSuccess) e2 = upload(&plan->d_bbig, pb.tiles);
        if (e2 != hipSuccess) return fail_hip(e2, "hs_plan_create");
        plan->bwd_untiled = pb.nmp;
        hs_status rc2 = make_mpset(plan->bmp, plan, pb, true);
        if (rc2 != HS_OK) return rc2;
    }

    hipError_t err;
    (void)hipFree(plan->d_tiles);
    plan->d_tiles = nullptr;
    if ((err = upload(&plan->d_tiles, sorted)) != hipSuccess) return fail_hip(err, "hs_plan_create");
    plan->h_tiles = sorted;
    hs_status rc = make_mpset(plan->mp, plan, pk, false);
    if (rc != HS_OK) return rc;
    plan->max_units = pk.max_units;
    plan->shape = shape;

    plan->main_grid = grid_of(sorted.size());

    hs_plan_info &I = plan->info;
    I.tiled_joints = tiled;
    I.multipass_joints = nmp + plan->mp.chain_joints;
    I.chain_joints = plan->mp.chain_joints;
    I.num_tiles = (int32_t)sorted.size() + small_tiles;
    I.tile_joints = cap;
    I.waves_per_tile = shape.waves;
    I.grid = plan->main_grid + small_grid;
    I.multipass_rounds = plan->mp.rounds;
    I.max_block_chain = std::max(max_chain_tiles, max_chain_mp);
    I.schedule = HS_SCHED_CLASSES;
    I.max_anchors = 0;
    I.adjoint_blocks_per_wave = plan->num_btiles > 0 && plan->b_anchor_ok ? plan->b_bpw[2] : 0;
    bool queued = false;
    if (shape.queue_waves > 0 && strategy != HS_STRATEGY_MULTIPASS && !plan->inst && !shape.chain_units &&
        shape.algorithm == HS_ALG_SCAN) {
        if ((rc = build_queue(plan, shape, strategy, &queued)) != HS_OK) return rc;
    } else {
        (void)hipFree(plan->q.d_tiles);
        (void)hipFree(plan->q.d_code);
        plan->q.d_tiles = nullptr;
        plan->q.d_code = nullptr;
        plan->q.num_tiles = 0;
    }
    if (queued) {
        I.schedule = HS_SCHED_QUEUE;
        I.max_anchors = plan->q.max_anchors;
        I.num_tiles = plan->q.num_tiles;
        I.tile_joints = plan->q.cap;
        I.waves_per_tile = plan->q.waves;
        I.grid = plan->q.grid;
    } else if (plan->sched_opt == HS_SCHED_QUEUE) {
        return fail(HS_ERR_UNSUPPORTED, "the work-queue schedule does not fit this plan (tile anchors beyond the LDS)");
    }
    return HS_OK;
}

// The main tile set (k < 0) or size class k.  validate: the call checked
// the topology on the device first; its kernels then do nothing if the
// check failed.
hs::TileLaunch tile_launch(const hs_plan *p, int k = -1, bool validate = false)
{
    hs::TileLaunch tl{};
    if (k < 0) {
        tl.tiles = p->d_tiles;
        tl.num_tiles = (int32_t)p->h_tiles.size();
        tl.tile_cap = p->shape.tile_cap;
        tl.waves = p->shape.waves;
        tl.grid = std::max(1, p->main_grid);
    } else {
        const auto &c = p->small[k];
        tl.tiles = c.d_tiles;
        tl.num_tiles = c.num_tiles;
        tl.tile_cap = c.cap;
        tl.waves = c.waves;
        tl.grid = std::max(1, c.grid);
    }
    tl.parent = p->d_parent;
    tl.chain_units = p->shape.chain_units ? 1 : 0;
    tl.algorithm = p->shape.algorithm;
    if (p->inst) {
        tl.skel_parent = p->d_skel_parent;
        tl.char_skel = p->d_char_skel;
    }
    tl.status = p->d_status;
    tl.spin_limit = p->spin_limit;
    tl.gate = validate ? p->d_status : nullptr;
    return tl;
}

hs::MPLaunch mp_launch(const hs_plan *p, const MPSet &m, bool validate = false)
{
    hs::MPLaunch ml{};
    ml.blocks = m.d_blocks;
    ml.num_blocks = m.num_blocks;
    ml.nmp = m.nmp;
    ml.parent = p->d_parent;
    ml.janc = m.d_janc;
    ml.A1 = m.A1;
    ml.E1 = m.E1;
    ml.num_anchors = m.num_anchors;
    ml.rounds = m.rounds;
    ml.aself = m.d_aself;
    ml.aseg = m.d_aseg;
    ml.num_aseg = m.num_aseg;
    ml.G = m.G;
    for (int i = 0; i < 2; ++i) {
        ml.AP[i] = m.AP[i];
        ml.AE[i] = m.AE[i];
        ml.S[i] = m.S[i];
    }
    ml.gate = validate ? p->d_status : nullptr;
    return ml;
}

hs::ChainLaunch chain_launch(const hs_plan *p, bool sample, bool validate = false)
{
    const MPSet &m = p->mp;
    hs::ChainLaunch cl{};
    cl.blocks = m.d_cblocks;
    cl.num_blocks = m.num_cblocks;
    cl.sbs = m.d_csb;
    cl.num_sb = m.num_csb;
    cl.grid = m.c_grid[sample ? 1 : 0];
    cl.recs = m.c_recs;
    cl.epoch = m.c_epoch;
    cl.status = p->d_status;
    cl.spin_limit = p->spin_limit;
    cl.gate = validate ? p->d_status : nullptr;
    return cl;
}

// HS_FLAG_VALIDATE: the topology check of the plan's device tables, on the
// call's stream ahead of its kernels.
hs_status launch_validate(const hs_plan *plan, hipStream_t stream, const char *what)
{
    hipError_t err = hs::launch_validate(plan->d_offsets, plan->C, plan->d_parent, plan->d_level, plan->d_status,
                                         stream);
    if (err != hipSuccess) return fail_hip(err, what);
    return HS_OK;
}

hs_status check_pose_src(const hs_plan *plan, const hs_pose_src *src, hs::PoseArgs &pa,
                         std::vector<Range> &ins, bool allow_clips)
{
    if (!src) return fail(HS_ERR_INVALID_ARG, "pose source is NULL");
    const size_t N = (size_t)plan->N;
    pa = hs::PoseArgs{};
    pa.kind = src->kind;
    pa.offsets = plan->d_offsets;
    if (src->kind == HS_POSE_TRS) {
        if (!src->quat || !src->trans) return fail(HS_ERR_INVALID_ARG, "quat and trans must be non-NULL");
        if (!aligned(src->quat, 16)) return fail(HS_ERR_INVALID_ARG, "quat must be 16-byte aligned");
        if (!aligned(src->trans, 4) || (src->scale && !aligned(src->scale, 4)))
            return fail(HS_ERR_INVALID_ARG, "trans/scale must be 4-byte aligned");
        pa.quat = src->quat;
        pa.trans = src->trans;
        pa.scale = src->scale;
        ins.push_back({src->quat, N * 16, "quat"});
        ins.push_back({src->trans, N * 12, "trans"});
        ins.push_back({src->scale, src->scale ? N * 12 : 0, "scale"});
        return HS_OK;
    }
    if (src->kind != HS_POSE_CLIPS) return fail(HS_ERR_INVALID_ARG, "unknown pose source kind %d", src->kind);
    if (!allow_clips) return fail(HS_ERR_UNSUPPORTED, "this call needs HS_POSE_TRS poses");
    const hs_clip_lib *L = src->clips;
    const hs_clip_params *P = src->params;
    if (!L || !P) return fail(HS_ERR_INVALID_ARG, "clip library and parameters must be non-NULL");
    if (L->num_clips <= 0 || L->num_keys <= 0 || L->joints_per_clip <= 0)
        return fail(HS_ERR_INVALID_ARG, "clip library sizes must be positive");
    if (!std::isfinite(L->fps)) return fail(HS_ERR_INVALID_ARG, "fps must be finite");
    if (L->joints_per_clip < plan->info.max_character)
        return fail(HS_ERR_INVALID_ARG, "clips hold %d joints but a character has %d",
                    L->joints_per_clip, plan->info.max_character);
    if (!L->key_quat || !L->key_trans || !P->clip_a || !P->clip_b || !P->time || !P->weight)
        return fail(HS_ERR_INVALID_ARG, "clip arrays must be non-NULL");
    if (!aligned(L->key_quat, 16)) return fail(HS_ERR_INVALID_ARG, "key_quat must be 16-byte aligned");
    pa.num_clips = L->num_clips;
    pa.num_keys = L->num_keys;
    pa.joints_per_clip = L->joints_per_clip;
    pa.fps = L->fps;
    pa.key_quat = L->key_quat;
    pa.key_trans = L->key_trans;
    pa.clip_a = P->clip_a;
    pa.clip_b = P->clip_b;
    pa.time = P->time;
    pa.weight = P->weight;
    const size_t keys = (size_t)L->num_clips * L->num_keys * L->joints_per_clip;
    const size_t C = (size_t)plan->C;
    ins.push_back({L->key_quat, keys * 16, "key_quat"});
    ins.push_back({L->key_trans, keys * 12, "key_trans"});
    ins.push_back({P->clip_a, C * 4, "clip_a"});
    ins.push_back({P->clip_b, C * 4, "clip_b"});
    ins.push_back({P->time, C * 4, "time"});
    ins.push_back({P->weight, C * 4, "weight"});
    return HS_OK;
}

hs_status run_forward(const hs_plan *plan, const hs::PoseArgs &pa, const hs::OutArgs &oa,
                      hipStream_t stream, bool validate = false)
{
    if (validate) {
        hs_status rc = launch_validate(plan, stream, "hs_scan_forward (validate)");
        if (rc != HS_OK) return rc;
    }
    hipError_t err = hipSuccess;
    if (plan->q.num_tiles > 0) {
        hs::QueueLaunch ql{};
        ql.tiles = plan->q.d_tiles;
        ql.num_tiles = plan->q.num_tiles;
        ql.waves = plan->q.waves;
        ql.grid = plan->q.grid;
        std::memcpy(ql.grids, plan->q.grids, sizeof ql.grids);
        ql.max_anchors = plan->q.max_anchors;
        ql.tile_cap = plan->q.cap;
        ql.code = plan->q.d_code;
        ql.status = plan->d_status;
        ql.spin_limit = plan->spin_limit;
        ql.gate = validate ? plan->d_status : nullptr;
        err = hs::launch_forward_queue(ql, pa, oa, stream);
    } else {
        for (int k = 0; k < (int)plan->small.size() && err == hipSuccess; ++k)
            err = hs::launch_forward_tiles(tile_launch(plan, k, validate), pa, oa, stream);
        if (err == hipSuccess) err = hs::launch_forward_tiles(tile_launch(plan, -1, validate), pa, oa, stream);
    }
    if (err != hipSuccess) return fail_hip(err, "hs_scan_forward (tiles)");
    err = hs::launch_forward_multipass(mp_launch(plan, plan->mp, validate), pa, oa, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_scan_forward (multipass)");
    err = hs::launch_forward_chains(chain_launch(plan, pa.kind == 1, validate), pa, oa, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_scan_forward (chains)");
    return HS_OK;
}

// ---------------------------------------------------------------------------
// Launch-shape autotuning: time the candidates on scratch poses of the
// plan's own topology and keep the fastest.
// ---------------------------------------------------------------------------
std::string tune_key(const hs_plan *p, int strategy)
{
    // size class: number of joints (log2), largest character and deepest
    // block chain, rounded so that similar batches share an entry; the
    // strategy and the instancing decide which candidates are allowed
    char buf[160];
    snprintf(buf, sizeof buf, "%s|N%d|maxc%d|chain%d|chars%d|inst%d|strat%d|sched%d", p->ctx->arch.c_str(),
             ceil_log2(std::max<int64_t>(1, p->N)), round_up(std::max(1, p->info.max_character), 64),
             ceil_log2(std::max(1, p->info.max_block_chain)), ceil_log2(std::max<int64_t>(1, p->C)),
             p->inst ? 1 : 0, strategy, p->sched_opt);
    return buf;
}

hs_status autotune(hs_plan *plan, const Shape &base, int strategy)
{
    const std::string key = tune_key(plan, strategy);
    {
        std::lock_guard<std::mutex> lk(plan->ctx->mu);
        auto it = plan->ctx->tuned.find(key);
        if (it != plan->ctx->tuned.end()) {
            Shape sh = it->second;  // the forward's launch shape; the adjoint kind is this plan's
            sh.adjoint = base.adjoint;
            sh.algorithm = base.algorithm;
            if (plan->inst) sh.chain_units = false;
            if (plan->inst || plan->sched_opt == HS_SCHED_CLASSES || sh.chain_units) sh.queue_waves = 0;
            return build_tables(plan, sh, strategy);
        }
    }
    const size_t N = (size_t)plan->N;
    std::vector<Shape> cands;
    const int min_cap = round_up(std::max(1, plan->info.max_character), 64);
    if (base.queue_waves > 0) {
        // the work queue: tile size and waves; one workgroup per tile, or
        // the resident workgroups looping over the tiles (measured on the
        // heterogeneous batch: 175.7 against 180.5 us)
        for (int cap : {256, 512, 1024, 2048, 3072}) {
            if (cap < min_cap && strategy == HS_STRATEGY_TILE) continue;
            for (int w : {2, 4, 8, 16}) {
                if (w * 64 > cap) continue;
                for (int g : {0, 64}) {
                    Shape c = base;
                    c.tile_cap = cap;
                    c.queue_cap = 0;
                    c.queue_waves = w;
                    c.grid_per_cu = g;
                    while (c.waves > 1 && c.waves * 64 > cap) c.waves >>= 1;  // the size-class tiles' waves
                    cands.push_back(c);
                }
            }
        }
    }
    for (int cap : {64, 128, 256, 512, 1024, 2048}) {
        if (plan->sched_opt == HS_SCHED_QUEUE) break;  // the size classes are not candidates then
        // every character must stay on a tile for the tile strategy and for
        // instanced plans (which have no multipass path)
        if (cap < min_cap && (strategy == HS_STRATEGY_TILE || plan->inst)) continue;
        if (hs::forward_tile_lds_bytes(cap, true) > plan->ctx->max_lds) continue;
        for (int w : {1, 2, 4, 8, 16}) {
            if (w * 64 > cap) continue;
            if (cap / (w * 64) > 4) continue;  // at most 4 blocks per wave
            for (int g : {0, 2, 4})
                for (bool cu : {false, true}) {
                    if (cu && plan->inst) continue;  // instanced tiles run whole blocks
                    Shape c = base;
                    c.tile_cap = cap;
                    c.waves = w;
                    c.grid_per_cu = g;
                    c.chain_units = cu;
                    c.queue_waves = 0;
                    cands.push_back(c);
                }
        }
    }
    if (cands.empty()) return build_tables(plan, base, strategy);

    float *q = nullptr, *t = nullptr, *G = nullptr;
    hipError_t err;
    if ((err = hipMalloc(&q, N * 16)) != hipSuccess || (err = hipMalloc(&t, N * 12)) != hipSuccess ||
        (err = hipMalloc(&G, N * 64)) != hipSuccess) {
        (void)hipFree(q); (void)hipFree(t); (void)hipFree(G);
        return fail_hip(err, "hs_plan_create (autotune scratch)");
    }
    // identity rotations, zero offsets: values do not affect the timing
    std::vector<float> hq(N * 4, 0.0f);
    for (size_t i = 0; i < N; ++i) hq[4 * i + 3] = 1.0f;
    (void)hipMemcpy(q, hq.data(), N * 16, hipMemcpyHostToDevice);
    (void)hipMemset(t, 0, N * 12);
    hipStream_t s;
    (void)hipStreamCreate(&s);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hs::PoseArgs pa{};
    pa.kind = 0;
    pa.quat = q;
    pa.trans = t;
    pa.offsets = plan->d_offsets;  // the character map of instanced tiles reads these
    hs::OutArgs oa{};
    oa.global_out = G;
    // median of 10 timed runs after 3 warm-up runs per candidate; the
    // default shape (timed first) is kept unless a candidate beats it by 3%
    auto time_shape = [&](const Shape &sh, float &ms_out) -> hs_status {
        hs_status rc2 = build_tables(plan, sh, strategy);
        if (rc2 != HS_OK) return rc2;
        std::vector<float> ms;
        for (int it = 0; it < 13; ++it) {
            (void)hipEventRecord(e0, s);
            rc2 = run_forward(plan, pa, oa, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            if (rc2 != HS_OK) return rc2;
            float m = 0.0f;
            (void)hipEventElapsedTime(&m, e0, e1);
            if (it >= 3) ms.push_back(m);
        }
        std::sort(ms.begin(), ms.end());
        ms_out = ms[ms.size() / 2];
        return HS_OK;
    };
    Shape best = base;
    float best_ms = 1e30f;
    hs_status rc = time_shape(base, best_ms);
    const float default_ms = best_ms;
    for (size_t i = 0; rc == HS_OK && i < cands.size(); ++i) {
        float ms = 0.0f;
        if ((rc = time_shape(cands[i], ms)) != HS_OK) break;
        if (ms < best_ms && ms < 0.97f * default_ms) {
            best_ms = ms;
            best = cands[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    (void)hipFree(q);
    (void)hipFree(t);
    (void)hipFree(G);
    if (rc != HS_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(plan->ctx->mu);
        plan->ctx->tuned[key] = best;
    }
    if (!plan->ctx->tune_file.empty()) {
        hs_status rc2 = save_tuning_file(plan->ctx, plan->ctx->tune_file.c_str());
        if (rc2 != HS_OK) return rc2;
    }
    return build_tables(plan, best, strategy);
}

// Validation of a forward call and its kernel arguments; HS_OK with
// *empty set when there is nothing to launch (an empty batch).
hs_status prepare_forward(const hs_plan *plan, const hs_pose_src *src, float *global_out, const float *inv_bind,
                          float *skin_out, float *ckpt_out, int32_t ckpt_k, uint32_t flags, hs::PoseArgs &pa,
                          hs::OutArgs &oa, bool *empty)
{
    *empty = true;
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_scan_forward: plan is NULL");
    if (flags & ~HS_FLAG_VALIDATE) return fail(HS_ERR_INVALID_ARG, "hs_scan_forward: unknown flags 0x%x", flags);
    if (ckpt_out && ckpt_k < 1) return fail(HS_ERR_INVALID_ARG, "hs_scan_forward: ckpt_k must be >= 1");
    if (plan->N == 0) return HS_OK;  // zero-size arrays may be NULL
    if (!global_out && !skin_out) return fail(HS_ERR_INVALID_ARG, "hs_scan_forward: no output requested");
    if ((skin_out != nullptr) != (inv_bind != nullptr))
        return fail(HS_ERR_INVALID_ARG, "hs_scan_forward: inv_bind and skin_out go together");
    for (const void *p : {(const void *)global_out, (const void *)inv_bind, (const void *)skin_out,
                          (const void *)ckpt_out})
        if (p && !aligned(p, 16)) return fail(HS_ERR_INVALID_ARG, "hs_scan_forward: outputs and inv_bind must be 16-byte aligned");
    std::vector<Range> ins;
    hs_status rc = check_pose_src(plan, src, pa, ins, true);
    if (rc != HS_OK) return rc;
    if (plan->shape.algorithm != HS_ALG_SCAN && src->kind != HS_POSE_TRS)
        return fail(HS_ERR_UNSUPPORTED, "hs_scan_forward: the paper's algorithms take stored TRS poses only");
    const size_t N = (size_t)plan->N;
    ins.push_back({inv_bind, (plan->inst ? (size_t)plan->skel_joints : N) * 64, "inv_bind"});
    std::vector<Range> outs = {{global_out, N * 64, "global_out"}, {skin_out, N * 64, "skin_out"},
                               {ckpt_out, N * 48, "ckpt_out"}};
    if ((rc = check_aliasing(outs, ins)) != HS_OK) return rc;
    oa = hs::OutArgs{};
    oa.global_out = global_out;
    oa.inv_bind = inv_bind;
    oa.skin_out = skin_out;
    oa.ckpt = ckpt_out;
    oa.ckpt_k = ckpt_out ? ckpt_k : 1;
    oa.level = plan->d_level;
    *empty = false;
    return HS_OK;
}

} // namespace

extern "C" {

const char *hs_version(void) { return "hs 0.1.0 (gfx950)"; }

const char *hs_last_error(void) { return g_last_error.c_str(); }

hs_status hs_context_create(int device, hs_context **out)
{
    if (!out) return fail(HS_ERR_INVALID_ARG, "hs_context_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t err = hipGetDeviceCount(&count);
    if (err != hipSuccess) return fail_hip(err, "hs_context_create");
    if (device < 0 || device >= count)
        return fail(HS_ERR_INVALID_ARG, "hs_context_create: device %d not in [0, %d)", device, count);
    hipDeviceProp_t prop;
    if ((err = hipGetDeviceProperties(&prop, device)) != hipSuccess) return fail_hip(err, "hs_context_create");
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0)
        return fail(HS_ERR_UNSUPPORTED, "hs_context_create: device %d is %s; this library targets gfx950",
                    device, arch.c_str());
    float4 *noalloc_ws = nullptr;
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        if ((err = hipSetDevice(device)) != hipSuccess) return fail_hip(err, "hs_context_create");
        err = hs::prepare_kernels();
        if (err == hipSuccess) err = hs::noalloc_workspace(device, &noalloc_ws);
        if (prev >= 0) (void)hipSetDevice(prev);
        if (err != hipSuccess) return fail_hip(err, "hs_context_create (kernel attributes, static workspace)");
    }
    hs_context *ctx = new hs_context();
    ctx->noalloc_ws = noalloc_ws;
    if (const char *tf = std::getenv("HS_TUNE_CACHE")) {
        if (*tf) {
            ctx->tune_file = tf;
            ctx->device = device;
            ctx->arch = arch.substr(0, arch.find(':'));
            hs_status rc = load_tuning_file(ctx, tf);
            if (rc != HS_OK) {
                delete ctx;
                return rc;
            }
        }
    }
    ctx->device = device;
    ctx->num_cu = prop.multiProcessorCount;
    ctx->max_lds = prop.sharedMemPerBlock;
    ctx->arch = arch.substr(0, arch.find(':'));
    *out = ctx;
    return HS_OK;
}

void hs_context_destroy(hs_context *ctx) { delete ctx; }

hs_status hs_context_load_tuning(hs_context *ctx, const char *path)
{
    if (!ctx || !path) return fail(HS_ERR_INVALID_ARG, "hs_context_load_tuning: NULL argument");
    return load_tuning_file(ctx, path);
}

hs_status hs_context_save_tuning(const hs_context *ctx, const char *path)
{
    if (!ctx || !path) return fail(HS_ERR_INVALID_ARG, "hs_context_save_tuning: NULL argument");
    return save_tuning_file(ctx, path);
}

} // extern "C"

namespace {

// Skeleton tables of an instanced plan (host arrays): skeleton-local
// parents and each character's first skeleton joint.
struct SkelTables {
    const std::vector<int32_t> *parents;
    const std::vector<int32_t> *char_first;
};

hs_status create_plan(hs_context *ctx, const hs_batch *batch, const hs_plan_opts *opts, hs_plan **out,
                      const SkelTables *inst);

} // namespace

extern "C" {

hs_status hs_plan_create(hs_context *ctx, const hs_batch *batch, const hs_plan_opts *opts, hs_plan **out)
{
    return create_plan(ctx, batch, opts, out, nullptr);
}

hs_status hs_plan_create_instanced(hs_context *ctx, const hs_skeleton_set *skel, int32_t num_characters,
                                   const int32_t *skeleton_id, const hs_plan_opts *opts, hs_plan **out)
{
    if (!out) return fail(HS_ERR_INVALID_ARG, "hs_plan_create_instanced: out is NULL");
    *out = nullptr;
    if (!ctx || !skel) return fail(HS_ERR_INVALID_ARG, "hs_plan_create_instanced: context and skeletons must be non-NULL");
    const int32_t S = skel->num_skeletons;
    const int64_t NS = skel->num_joints;
    if (S < 0 || NS < 0 || NS >= (int64_t(1) << 31) - 1)
        return fail(HS_ERR_INVALID_ARG, "skeleton counts out of range");
    if (num_characters < 0) return fail(HS_ERR_INVALID_ARG, "num_characters must be >= 0");
    if (!skel->offsets || (NS > 0 && !skel->parents) || (num_characters > 0 && !skeleton_id))
        return fail(HS_ERR_INVALID_ARG, "skeleton offsets, parents and skeleton_id must be non-NULL");
    const int64_t *so = skel->offsets;
    if (so[0] != 0 || so[S] != NS) return fail(HS_ERR_INVALID_ARG, "skeleton offsets must run from 0 to num_joints");
    for (int32_t k = 0; k < S; ++k)
        if (so[k + 1] < so[k]) return fail(HS_ERR_INVALID_ARG, "skeleton offsets must be non-decreasing");
    hs_plan_opts o{};
    if (opts) o = *opts;
    if (o.chain_units || o.algorithm != HS_ALG_SCAN || o.strategy == HS_STRATEGY_MULTIPASS)
        return fail(HS_ERR_UNSUPPORTED, "instanced plans run the library's block scan on tiles "
                                        "(no chain units, paper algorithms or multipass strategy)");
    // the batch the instances make: character c is a copy of skeleton skeleton_id[c]
    std::vector<int64_t> off((size_t)num_characters + 1, 0);
    std::vector<int32_t> first((size_t)num_characters);
    for (int32_t c = 0; c < num_characters; ++c) {
        const int32_t k = skeleton_id[c];
        if (k < 0 || k >= S) return fail(HS_ERR_INVALID_ARG, "skeleton_id[%d] = %d out of range", c, k);
        first[c] = (int32_t)so[k];
        off[c + 1] = off[c] + (so[k + 1] - so[k]);
        if (off[c + 1] >= (int64_t(1) << 31) - 1) return fail(HS_ERR_UNSUPPORTED, "instances exceed 2^31-1 joints");
    }
    std::vector<int32_t> par((size_t)off[num_characters]);
    for (int32_t c = 0; c < num_characters; ++c)
        std::copy(skel->parents + first[c], skel->parents + first[c] + (off[c + 1] - off[c]), par.begin() + off[c]);
    std::vector<int32_t> sp(skel->parents, skel->parents + NS);
    const hs_batch b{num_characters, off[num_characters], off.data(), par.data()};
    const SkelTables t{&sp, &first};
    return create_plan(ctx, &b, &o, out, &t);
}

} // extern "C"

namespace {

hs_status create_plan(hs_context *ctx, const hs_batch *batch, const hs_plan_opts *opts, hs_plan **out,
                      const SkelTables *inst)
{
    if (!out) return fail(HS_ERR_INVALID_ARG, "hs_plan_create: out is NULL");
    *out = nullptr;
    if (!ctx || !batch) return fail(HS_ERR_INVALID_ARG, "hs_plan_create: context and batch must be non-NULL");
    const int64_t C = batch->num_characters, N = batch->num_joints;
    if (C < 0 || C >= (int64_t(1) << 31)) return fail(HS_ERR_INVALID_ARG, "num_characters %lld out of range", (long long)C);
    if (N < 0 || N >= (int64_t(1) << 31) - 1) return fail(HS_ERR_UNSUPPORTED, "num_joints %lld out of range [0, 2^31-1)", (long long)N);
    if (!batch->joint_offsets) return fail(HS_ERR_INVALID_ARG, "joint_offsets is NULL");
    if (N > 0 && !batch->parents) return fail(HS_ERR_INVALID_ARG, "parents is NULL");
    hs_plan_opts o{};
    if (opts) o = *opts;
    if (o.schedule < HS_SCHED_AUTO || o.schedule > HS_SCHED_CLASSES)
        return fail(HS_ERR_INVALID_ARG, "unknown schedule %d", o.schedule);
    if (o.strategy < HS_STRATEGY_AUTO || o.strategy > HS_STRATEGY_MULTIPASS)
        return fail(HS_ERR_INVALID_ARG, "unknown strategy %d", o.strategy);
    if (o.tile_joints < 0 || o.tile_joints % 64 != 0)
        return fail(HS_ERR_INVALID_ARG, "tile_joints must be a non-negative multiple of 64");
    if (o.waves_per_tile != 0 && o.waves_per_tile != 1 && o.waves_per_tile != 2 && o.waves_per_tile != 4 &&
        o.waves_per_tile != 8 && o.waves_per_tile != 16)
        return fail(HS_ERR_INVALID_ARG, "waves_per_tile must be 0, 1, 2, 4, 8 or 16");
    if (o.grid_tiles < 0 || o.grid_tiles > 64) return fail(HS_ERR_INVALID_ARG, "grid_tiles must be in [0, 64]");
    if (o.algorithm < HS_ALG_SCAN || o.algorithm > HS_ALG_COMPRESSED)
        return fail(HS_ERR_INVALID_ARG, "unknown algorithm %d", o.algorithm);
    if (o.adjoint < HS_ADJ_AUTO || o.adjoint > HS_ADJ_ANCHORS)
        return fail(HS_ERR_INVALID_ARG, "unknown adjoint kernel %d", o.adjoint);
    if (o.adjoint_blocks_per_wave < 0 || o.adjoint_blocks_per_wave > 2)
        return fail(HS_ERR_INVALID_ARG, "adjoint_blocks_per_wave must be 0, 1 or 2");
    if (o.algorithm != HS_ALG_SCAN && o.chain_units)
        return fail(HS_ERR_INVALID_ARG, "chain units belong to the library's own scan (algorithm 0)");
    if (o.schedule == HS_SCHED_QUEUE &&
        (o.algorithm != HS_ALG_SCAN || o.chain_units || o.strategy == HS_STRATEGY_MULTIPASS))
        return fail(HS_ERR_UNSUPPORTED, "the work-queue schedule runs the library's scan on tiles, without chain units");

    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_plan_create: cannot select device %d", ctx->device);

    hs_plan *plan = new hs_plan();
    plan->ctx = ctx;
    plan->C = C;
    plan->N = N;
    hipError_t err;
    if ((err = fetch(plan->h_offsets, batch->joint_offsets, (size_t)C + 1)) != hipSuccess ||
        (err = fetch(plan->h_parents, batch->parents, (size_t)N)) != hipSuccess) {
        free_plan(plan);
        return fail_hip(err, "hs_plan_create (reading topology)");
    }
    const auto &off = plan->h_offsets;
    const auto &par = plan->h_parents;
    if (off[0] != 0) {
        free_plan(plan);
        return fail(HS_ERR_INVALID_ARG, "joint_offsets[0] must be 0");
    }
    int max_char = 0, max_depth = 0;
    std::vector<int32_t> level((size_t)N), gparent((size_t)N);
    for (int64_t c = 0; c < C; ++c) {
        if (off[c + 1] < off[c] || off[c + 1] > N) {
            free_plan(plan);
            return fail(HS_ERR_INVALID_ARG, "joint_offsets must be non-decreasing and end at num_joints");
        }
        const int64_t n = off[c + 1] - off[c];
        max_char = std::max<int64_t>(max_char, n);
        for (int64_t j = 0; j < n; ++j) {
            const int64_t g = off[c] + j;
            const int32_t p = par[g];
            if (p < -1 || (int64_t)p >= j) {
                free_plan(plan);
                return fail(HS_ERR_TOPOLOGY, "character %lld joint %lld has parent %d (need -1 <= parent < %lld)",
                            (long long)c, (long long)j, p, (long long)j);
            }
            gparent[g] = p < 0 ? -1 : (int32_t)(off[c] + p);
            level[g] = p < 0 ? 1 : level[off[c] + p] + 1;
            max_depth = std::max(max_depth, level[g]);
        }
    }
    if (off[C] != N) {
        free_plan(plan);
        return fail(HS_ERR_INVALID_ARG, "joint_offsets[C] = %lld but num_joints = %lld", (long long)off[C], (long long)N);
    }
    plan->h_gparent = gparent;
    plan->h_level = level;
    plan->info.num_characters = C;
    plan->info.num_joints = N;
    plan->info.max_depth = max_depth;
    plan->info.max_character = max_char;
    if ((err = upload(&plan->d_offsets, off)) != hipSuccess || (err = upload(&plan->d_parent, gparent)) != hipSuccess ||
        (err = upload(&plan->d_level, level)) != hipSuccess) {
        free_plan(plan);
        return fail_hip(err, "hs_plan_create (upload)");
    }

    {
        // status word: no bits, no failing joint
        const std::vector<uint32_t> st = {0u, 0xFFFFFFFFu};
        if ((err = upload(&plan->d_status, st)) != hipSuccess) {
            free_plan(plan);
            return fail_hip(err, "hs_plan_create (status word)");
        }
    }
    if (inst) {
        plan->inst = true;
        plan->skel_joints = (int64_t)inst->parents->size();
        if ((err = upload(&plan->d_skel_parent, *inst->parents)) != hipSuccess ||
            (err = upload(&plan->d_char_skel, *inst->char_first)) != hipSuccess) {
            free_plan(plan);
            return fail_hip(err, "hs_plan_create_instanced (upload)");
        }
    }

    // default launch shape
    const int lds_cap = hs::kMaxTileJoints;
    const int min_cap = round_up(std::max(1, max_char), 64);
    Shape sh;
    if (o.tile_joints > 0) {
        sh.tile_cap = o.tile_joints;
    } else {
        const int64_t target = (N + 2 * (int64_t)ctx->num_cu - 1) / (2 * (int64_t)ctx->num_cu);
        sh.tile_cap = (int)std::min<int64_t>(1024, round_up((int)std::max<int64_t>(64, target), 64));
        sh.tile_cap = std::max(sh.tile_cap, std::min(min_cap, 2048));
    }
    if (hs::forward_tile_lds_bytes(sh.tile_cap, true) > ctx->max_lds || sh.tile_cap > lds_cap) {
        free_plan(plan);
        return fail(HS_ERR_UNSUPPORTED, "tile of %d joints exceeds the %zu-byte LDS", sh.tile_cap, ctx->max_lds);
    }
    if (o.strategy == HS_STRATEGY_TILE && min_cap > sh.tile_cap) {
        free_plan(plan);
        return fail(HS_ERR_UNSUPPORTED, "a character of %d joints does not fit a %d-joint tile", max_char,
                    sh.tile_cap);
    }
    sh.waves = o.waves_per_tile > 0 ? o.waves_per_tile : std::min(16, sh.tile_cap / 64);
    while (sh.waves > 1 && (sh.waves * 64 > sh.tile_cap || (sh.waves & (sh.waves - 1)) != 0))
        --sh.waves;  // a power of two with at least one block per wave

    sh.grid_per_cu = o.grid_tiles;
    sh.chain_units = o.chain_units != 0;
    sh.algorithm = o.algorithm;
    sh.adjoint = o.adjoint;  // AUTO is resolved per call (the seeds decide)
    plan->sched_opt = o.schedule;
    plan->b_bpw_opt = o.adjoint_blocks_per_wave;
    if (inst && o.schedule == HS_SCHED_QUEUE) {
        free_plan(plan);
        return fail(HS_ERR_UNSUPPORTED, "the work-queue schedule does not take instanced plans");
    }
    if (o.schedule != HS_SCHED_CLASSES && sh.algorithm == HS_ALG_SCAN && !sh.chain_units && !inst &&
        o.strategy != HS_STRATEGY_MULTIPASS) {
        // four waves (measured against eight and sixteen on the deep,
        // heterogeneous and fused workloads: more workgroups per CU), fewer
        // on tiles of fewer blocks
        // default tiles: the largest character's size, at least 256 joints
        // (one workgroup per tile; measured on 10 000 x 256 joints with
        // sampled poses: 88.4 us on 256-joint tiles against 93.9 us on
        // 1024-joint ones)
        if (o.tile_joints == 0 && sh.tile_cap > 256) sh.queue_cap = std::max(256, std::min(min_cap, sh.tile_cap));
        const int qcap = sh.queue_cap > 0 ? sh.queue_cap : sh.tile_cap;
        int w = o.waves_per_tile > 0 ? o.waves_per_tile : 4;
        while (w > 1 && w * 64 > qcap) w >>= 1;
        sh.queue_waves = w;
    }
    if (sh.algorithm != HS_ALG_SCAN) {
        // the paper's algorithms: one joint per thread, 1024-thread workgroups
        if (o.strategy == HS_STRATEGY_TILE && min_cap > hs::kPaperAlgTileJoints) {
            free_plan(plan);
            return fail(HS_ERR_UNSUPPORTED, "the paper's algorithms tile characters of at most %d joints",
                        hs::kPaperAlgTileJoints);
        }
        sh.tile_cap = std::min(sh.tile_cap, hs::kPaperAlgTileJoints);
        sh.waves = 16;
    }

    hs_status rc = build_tables(plan, sh, o.strategy);
    if (rc == HS_OK && sh.algorithm == HS_ALG_SCAN && o.waves_per_tile == 0 && plan->max_units > 0) {
        // no more waves than work units in the largest tile; tiles small
        // enough for three workgroups per CU take 8 waves (measured faster
        // than 16 on the deep workload: more workgroups overlap their phases)
        const int wmax = sh.tile_cap <= 1024 ? 8 : 16;
        int w = 1;
        while (w * 2 <= std::min(wmax, plan->max_units)) w *= 2;
        if (w != sh.waves) {
            sh.waves = w;
            rc = build_tables(plan, sh, o.strategy);
        }
    }
    if (rc == HS_OK && o.autotune && N > 0 && sh.algorithm == HS_ALG_SCAN) rc = autotune(plan, sh, o.strategy);
    if (rc == HS_OK && plan->inst && (plan->mp.nmp > 0 || plan->mp.chain_joints > 0))
        rc = fail(HS_ERR_UNSUPPORTED, "instanced plans need every character on a tile (%d joints at most here)",
                  plan->shape.tile_cap);
    if (rc != HS_OK) {
        free_plan(plan);
        return rc;
    }
    *out = plan;
    return HS_OK;
}

} // namespace

extern "C" {

void hs_plan_destroy(hs_plan *plan) { free_plan(plan); }

hs_status hs_plan_get_info(const hs_plan *plan, hs_plan_info *out)
{
    if (!plan || !out) return fail(HS_ERR_INVALID_ARG, "hs_plan_get_info: NULL argument");
    *out = plan->info;
    return HS_OK;
}

hs_status hs_plan_status(const hs_plan *plan, uint32_t *bits, int64_t *joint, int32_t clear)
{
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_plan_status: plan is NULL");
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_plan_status: cannot select device");
    hipError_t err = hipDeviceSynchronize();
    if (err != hipSuccess) return fail_hip(err, "hs_plan_status (synchronize)");
    uint32_t st[2];
    if ((err = hipMemcpy(st, plan->d_status, sizeof st, hipMemcpyDeviceToHost)) != hipSuccess)
        return fail_hip(err, "hs_plan_status (read)");
    if (bits) *bits = st[0];
    if (joint) *joint = st[1] == 0xFFFFFFFFu ? -1 : (int64_t)st[1];
    if (clear && st[0] != 0) {
        const uint32_t fresh[2] = {0u, 0xFFFFFFFFu};
        if ((err = hipMemcpy(plan->d_status, fresh, sizeof fresh, hipMemcpyHostToDevice)) != hipSuccess)
            return fail_hip(err, "hs_plan_status (clear)");
    }
    if (st[0] == 0) return HS_OK;
    std::string msg;
    if (st[0] & HS_DEV_TOPOLOGY) {
        char buf[160];
        snprintf(buf, sizeof buf, "device topology check failed (first bad joint %lld)",
                 st[1] == 0xFFFFFFFFu ? -1LL : (long long)st[1]);
        msg += buf;
    }
    if (st[0] & HS_DEV_WAIT_TIMEOUT) {
        if (!msg.empty()) msg += "; ";
        msg += "a kernel's bounded wait gave up (outputs of the calls since the last clear are unreliable)";
    }
    return fail(HS_ERR_DEVICE, "hs_plan_status: %s", msg.c_str());
}

hs_status hs_plan_set_wait_limit(hs_plan *plan, int32_t polls)
{
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_plan_set_wait_limit: plan is NULL");
    if (polls < 0) return fail(HS_ERR_INVALID_ARG, "hs_plan_set_wait_limit: polls must be >= 0");
    plan->spin_limit = polls;
    return HS_OK;
}

hs_status hs_plan_debug_break_parent(hs_plan *plan, int64_t joint)
{
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_plan_debug_break_parent: plan is NULL");
    if (joint < 0 || joint >= plan->N)
        return fail(HS_ERR_INVALID_ARG, "hs_plan_debug_break_parent: joint %lld outside [0, %lld)",
                    (long long)joint, (long long)plan->N);
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_plan_debug_break_parent: cannot select device");
    const int32_t self = (int32_t)joint;
    hipError_t err = hipMemcpy(plan->d_parent + joint, &self, sizeof self, hipMemcpyHostToDevice);
    if (err != hipSuccess) return fail_hip(err, "hs_plan_debug_break_parent");
    return HS_OK;
}

struct hs_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" hs_status hs_graph_create_forward(const hs_plan *plan, const hs_pose_src *src, float *global_out,
                                             const float *inv_bind, float *skin_out, hs_graph **out)
{
    if (!src) {
        if (out) *out = nullptr;
        return fail(HS_ERR_INVALID_ARG, "hs_graph_create_forward: src is NULL");
    }
    return hs_graph_create_forward_n(plan, 1, src, &global_out, &inv_bind, &skin_out, out);
}

extern "C" hs_status hs_graph_create_forward_n(const hs_plan *plan, int32_t n, const hs_pose_src *srcs,
                                               float *const *global_outs, const float *const *inv_binds,
                                               float *const *skin_outs, hs_graph **out)
{
    if (!out) return fail(HS_ERR_INVALID_ARG, "hs_graph_create_forward: out is NULL");
    *out = nullptr;
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_graph_create_forward: plan is NULL");
    if (n < 1) return fail(HS_ERR_INVALID_ARG, "hs_graph_create_forward_n: n = %d, need n >= 1", n);
    if (!srcs) return fail(HS_ERR_INVALID_ARG, "hs_graph_create_forward_n: srcs is NULL");
    auto gout = [&](int i) { return global_outs ? global_outs[i] : nullptr; };
    auto ibind = [&](int i) { return inv_binds ? inv_binds[i] : nullptr; };
    auto sout = [&](int i) { return skin_outs ? skin_outs[i] : nullptr; };
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_graph_create_forward: cannot select device");
    // argument errors surface before a capture is opened: a validation-only
    // pass (no launch) per call
    for (int i = 0; i < n; ++i) {
        hs::PoseArgs pa;
        hs::OutArgs oa;
        bool empty = true;
        hs_status rc0 = prepare_forward(plan, &srcs[i], gout(i), ibind(i), sout(i), nullptr, 0, 0, pa, oa, &empty);
        if (rc0 != HS_OK) return rc0;
    }
    hipStream_t s = nullptr;
    hipError_t err = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (err != hipSuccess) return fail_hip(err, "hs_graph_create_forward (stream)");
    hs_graph *g = new hs_graph();
    g->device = plan->ctx->device;
    err = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) {
        (void)hipStreamDestroy(s);
        delete g;
        return fail_hip(err, "hs_graph_create_forward (begin capture)");
    }
    hs_status rc = HS_OK;
    for (int i = 0; i < n && rc == HS_OK; ++i)
        rc = hs_scan_forward(plan, &srcs[i], gout(i), ibind(i), sout(i), nullptr, 0, 0, s);
    err = hipStreamEndCapture(s, &g->graph);
    if (rc == HS_OK && err != hipSuccess) rc = fail_hip(err, "hs_graph_create_forward (end capture)");
    if (rc == HS_OK) {
        err = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (err != hipSuccess) rc = fail_hip(err, "hs_graph_create_forward (instantiate)");
    }
    (void)hipStreamDestroy(s);
    if (rc != HS_OK) {
        hs_graph_destroy(g);
        return rc;
    }
    *out = g;
    return HS_OK;
}

extern "C" hs_status hs_graph_launch(hs_graph *graph, hipStream_t stream)
{
    if (!graph || !graph->exec) return fail(HS_ERR_INVALID_ARG, "hs_graph_launch: graph is NULL");
    DeviceGuard dg(graph->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_graph_launch: cannot select device");
    hipError_t err = hipGraphLaunch(graph->exec, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_graph_launch");
    return HS_OK;
}

extern "C" void hs_graph_destroy(hs_graph *graph)
{
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

hs_status hs_scan_forward(const hs_plan *plan, const hs_pose_src *src, float *global_out, const float *inv_bind,
                          float *skin_out, float *ckpt_out, int32_t ckpt_k, uint32_t flags, hipStream_t stream)
{
    hs::PoseArgs pa;
    hs::OutArgs oa;
    bool empty = true;
    hs_status rc = prepare_forward(plan, src, global_out, inv_bind, skin_out, ckpt_out, ckpt_k, flags, pa, oa, &empty);
    if (rc != HS_OK || empty) return rc;
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_scan_forward: cannot select device");
    return run_forward(plan, pa, oa, stream, (flags & HS_FLAG_VALIDATE) != 0);
}

hs_status hs_pose_sample(const hs_plan *plan, const hs_clip_lib *lib, const hs_clip_params *params,
                         float *quat_out, float *trans_out, hipStream_t stream)
{
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_pose_sample: plan is NULL");
    if (plan->N == 0) return HS_OK;  // zero-size arrays may be NULL
    if (!quat_out || !trans_out) return fail(HS_ERR_INVALID_ARG, "hs_pose_sample: outputs must be non-NULL");
    if (!aligned(quat_out, 16) || !aligned(trans_out, 4))
        return fail(HS_ERR_INVALID_ARG, "hs_pose_sample: quat_out must be 16-byte aligned");
    hs_pose_src src{};
    src.kind = HS_POSE_CLIPS;
    src.clips = lib;
    src.params = params;
    hs::PoseArgs pa;
    std::vector<Range> ins;
    hs_status rc = check_pose_src(plan, &src, pa, ins, true);
    if (rc != HS_OK) return rc;
    const size_t N = (size_t)plan->N;
    std::vector<Range> outs = {{quat_out, N * 16, "quat_out"}, {trans_out, N * 12, "trans_out"}};
    if ((rc = check_aliasing(outs, ins)) != HS_OK) return rc;
    if (N == 0) return HS_OK;
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_pose_sample: cannot select device");
    hipError_t err = hipSuccess;
    for (int k = 0; k < (int)plan->small.size() && err == hipSuccess; ++k)
        err = hs::launch_pose_sample(tile_launch(plan, k), hs::MPLaunch{}, hs::ChainLaunch{}, pa, quat_out,
                                     trans_out, stream);
    if (err == hipSuccess)
        err = hs::launch_pose_sample(tile_launch(plan), mp_launch(plan, plan->mp), chain_launch(plan, true), pa,
                                     quat_out, trans_out, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_pose_sample");
    return HS_OK;
}

} // extern "C"

namespace {

// Both routes of the sampler's reverse mode: `workspace` is caller memory
// (hs_pose_sample_backward) or the device's static array
// (hs_pose_sample_backward_noalloc, `noalloc`), in which case the batch
// must fit the array.
hs_status sample_backward(const char *name, const hs_plan *plan, const hs_clip_lib *lib,
                          const hs_clip_params *params, const float *grad_quat, const float *grad_trans,
                          float *grad_key_quat, float *grad_key_trans, float *grad_time, float *grad_weight,
                          float *workspace, bool noalloc, hipStream_t stream)
{
    if (!plan) return fail(HS_ERR_INVALID_ARG, "%s: plan is NULL", name);
    if (noalloc) {
        if (plan->N > hs::kNoAllocMaxJoints)
            return fail(HS_ERR_INVALID_ARG,
                        "%s: %lld joints exceed the static workspace of %lld joints (HS_NOALLOC_MAX_JOINTS); "
                        "use hs_pose_sample_backward with a caller workspace",
                        name, (long long)plan->N, (long long)hs::kNoAllocMaxJoints);
        if (!plan->ctx->noalloc_ws) return fail(HS_ERR_DEVICE, "%s: no static workspace on this device", name);
        workspace = reinterpret_cast<float *>(plan->ctx->noalloc_ws);
    }
    hs_pose_src src{};
    src.kind = HS_POSE_CLIPS;
    src.clips = lib;
    src.params = params;
    hs::PoseArgs pa;
    std::vector<Range> ins;
    hs_status rc = check_pose_src(plan, &src, pa, ins, true);
    if (rc != HS_OK) return rc;
    const size_t N = (size_t)plan->N, C = (size_t)plan->C;
    if (N > 0 && (!grad_quat || !grad_trans))
        return fail(HS_ERR_INVALID_ARG, "%s: grad_quat and grad_trans must be non-NULL", name);
    if (!aligned(grad_quat, 16) || !aligned(grad_trans, 4) || !aligned(grad_key_quat, 4) ||
        !aligned(grad_key_trans, 4) || !aligned(grad_time, 4) || !aligned(grad_weight, 4) ||
        !aligned(workspace, 16))
        return fail(HS_ERR_INVALID_ARG, "%s: grad_quat and workspace must be 16-byte aligned, the rest 4", name);
    ins.push_back({grad_quat, N * 16, "grad_quat"});
    ins.push_back({grad_trans, N * 12, "grad_trans"});
    const size_t keys = (size_t)lib->num_clips * lib->num_keys * lib->joints_per_clip;
    std::vector<Range> outs = {{grad_key_quat, grad_key_quat ? keys * 16 : 0, "grad_key_quat"},
                               {grad_key_trans, grad_key_trans ? keys * 12 : 0, "grad_key_trans"},
                               {grad_time, grad_time ? C * 4 : 0, "grad_time"},
                               {grad_weight, grad_weight ? C * 4 : 0, "grad_weight"},
                               {workspace, workspace ? N * 32 : 0, "workspace"}};
    if ((rc = check_aliasing(outs, ins)) != HS_OK) return rc;
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "%s: cannot select device", name);
    hs::SampleBwdArgs A{grad_quat, grad_trans, grad_key_quat, grad_key_trans, grad_time, grad_weight,
                        (int32_t)plan->C, reinterpret_cast<float4 *>(workspace)};
    hipError_t err = hs::launch_pose_sample_backward(pa, A, stream);
    if (err != hipSuccess) return fail_hip(err, name);
    return HS_OK;
}

} // namespace

extern "C" {

hs_status hs_pose_sample_backward(const hs_plan *plan, const hs_clip_lib *lib, const hs_clip_params *params,
                                  const float *grad_quat, const float *grad_trans, float *grad_key_quat,
                                  float *grad_key_trans, float *grad_time, float *grad_weight, float *workspace,
                                  hipStream_t stream)
{
    return sample_backward("hs_pose_sample_backward", plan, lib, params, grad_quat, grad_trans, grad_key_quat,
                           grad_key_trans, grad_time, grad_weight, workspace, false, stream);
}

hs_status hs_pose_sample_backward_noalloc(const hs_plan *plan, const hs_clip_lib *lib,
                                          const hs_clip_params *params, const float *grad_quat,
                                          const float *grad_trans, float *grad_key_quat, float *grad_key_trans,
                                          float *grad_time, float *grad_weight, hipStream_t stream)
{
    return sample_backward("hs_pose_sample_backward_noalloc", plan, lib, params, grad_quat, grad_trans,
                           grad_key_quat, grad_key_trans, grad_time, grad_weight, nullptr, true, stream);
}

hs_status hs_stream_probe(int64_t n, const float *quat, const float *trans, const float *scale,
                          const int32_t *table, float *out, hipStream_t stream)
{
    if (n < 0) return fail(HS_ERR_INVALID_ARG, "hs_stream_probe: n must be >= 0");
    if (n == 0) return HS_OK;
    if (!quat || !trans || !scale || !table || !out)
        return fail(HS_ERR_INVALID_ARG, "hs_stream_probe: arrays must be non-NULL");
    if (!aligned(quat, 16) || !aligned(out, 16) || !aligned(trans, 4) || !aligned(scale, 4) || !aligned(table, 4))
        return fail(HS_ERR_INVALID_ARG, "hs_stream_probe: quat and out must be 16-byte aligned, the rest 4");
    const size_t N = (size_t)n;
    std::vector<Range> ins = {{quat, N * 16, "quat"}, {trans, N * 12, "trans"}, {scale, N * 12, "scale"},
                              {table, N * 4, "table"}};
    hs_status rc = check_aliasing({{out, N * 64, "out"}}, ins);
    if (rc != HS_OK) return rc;
    hipError_t err = hs::launch_stream_probe(n, quat, trans, scale, table, out, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_stream_probe");
    return HS_OK;
}

hs_status hs_effector_loss_grad(int64_t num_joints, int64_t num_effectors, const int64_t *effectors,
                                const float *global, const float *targets, float *grad_global, hipStream_t stream)
{
    if (num_joints < 0 || num_effectors < 0)
        return fail(HS_ERR_INVALID_ARG, "hs_effector_loss_grad: sizes must be >= 0");
    if (num_effectors == 0) return HS_OK;
    if (!effectors || !global || !targets || !grad_global)
        return fail(HS_ERR_INVALID_ARG, "hs_effector_loss_grad: NULL array");
    if (!aligned(effectors, 8) || !aligned(global, 4) || !aligned(targets, 4) || !aligned(grad_global, 4))
        return fail(HS_ERR_INVALID_ARG, "hs_effector_loss_grad: misaligned array");
    const size_t N = (size_t)num_joints, E = (size_t)num_effectors;
    hs_status rc = check_aliasing({{grad_global, N * 64, "grad_global"}},
                                  {{global, N * 64, "global"}, {targets, E * 12, "targets"}, {effectors, E * 8, "effectors"}});
    if (rc != HS_OK) return rc;
    hipError_t err = hs::launch_effector_grad(num_joints, num_effectors, effectors, global, targets, grad_global,
                                              stream);
    if (err != hipSuccess) return fail_hip(err, "hs_effector_loss_grad");
    return HS_OK;
}

hs_status hs_skin(int64_t n, const float *global, const float *inv_bind, float *skin_out, hipStream_t stream)
{
    if (n < 0) return fail(HS_ERR_INVALID_ARG, "hs_skin: n must be >= 0");
    if (n == 0) return HS_OK;
    if (!global || !inv_bind || !skin_out) return fail(HS_ERR_INVALID_ARG, "hs_skin: NULL array");
    if (!aligned(global, 16) || !aligned(inv_bind, 16) || !aligned(skin_out, 16))
        return fail(HS_ERR_INVALID_ARG, "hs_skin: arrays must be 16-byte aligned");
    hs_status rc = check_aliasing({{skin_out, (size_t)n * 64, "skin_out"}},
                                  {{global, (size_t)n * 64, "global"}, {inv_bind, (size_t)n * 64, "inv_bind"}});
    if (rc != HS_OK) return rc;
    hipError_t err = hs::launch_skin(n, global, inv_bind, skin_out, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_skin");
    return HS_OK;
}

} // extern "C"

struct hs_mesh {
    const hs_plan *plan = nullptr;  // the plan it was made for
    int device = 0;
    int64_t N = 0, V = 0, rows = 0;
    hs::VertexLaunch vl{};
    int64_t *d_offsets = nullptr, *d_voff = nullptr;
    int32_t *d_mfirst = nullptr, *d_joints = nullptr;
    float *d_pos = nullptr, *d_weights = nullptr;
};

namespace {

void free_mesh(hs_mesh *m)
{
    if (!m) return;
    (void)hipFree(m->d_offsets);
    (void)hipFree(m->d_voff);
    (void)hipFree(m->d_mfirst);
    (void)hipFree(m->d_joints);
    (void)hipFree(m->d_pos);
    (void)hipFree(m->d_weights);
    delete m;
}

} // namespace

namespace {

// The adjoint's launches: synchronous-round (or dataflow) tiles, the large
// dataflow tiles, then the multipass characters.
hs_status run_backward(const hs_plan *plan, const hs::PoseArgs &pa, const hs::BwdArgs &ba, hipStream_t stream,
                       const char *what, bool validate = false)
{
    if (validate) {
        hs_status rc = launch_validate(plan, stream, what);
        if (rc != HS_OK) return rc;
    }
    hs::TileLaunch tl = tile_launch(plan, -1, validate);
    tl.chain_units = 0;
    hipError_t err = hipSuccess;
    if (plan->num_btiles > 0) {
        tl.tiles = plan->d_btiles;
        tl.num_tiles = plan->num_btiles;
        tl.tile_cap = plan->bwd_cap;
        // with checkpoints the dataflow kernel rebuilds every G_j from its
        // nearest checkpointed ancestor; without, the plan's kernel
        // recomputes them (the synchronous rounds: as their jump products)
        tl.adjoint = ba.ckpt ? hs::kAdjDataflow : plan->shape.adjoint;
        // AUTO: the two-level kernel for end-effector seeds (measured on
        // the differentiable workload: 40 against 49 us per step), the
        // synchronous rounds for dense seeds (37 against 73 us: every joint
        // of a chain block sends to the same anchor)
        if (tl.adjoint == 0) tl.adjoint = ba.eff_ids ? hs::kAdjAnchors : hs::kAdjRounds;
        if (tl.adjoint == hs::kAdjAnchors && !plan->b_anchor_ok) tl.adjoint = hs::kAdjRounds;
        tl.code = plan->d_bcode;
        tl.max_anchors = plan->b_max_anchors;
        tl.blocks_per_wave = plan->b_bpw[ba.eff_ids ? (ba.eff_forward ? 2 : 1) : 0];
        tl.grid = plan->num_btiles;
        tl.waves = 1;  // dataflow: a power of two, at most one wave per block
        while (tl.waves < 16 && tl.waves * 2 * 64 <= plan->bwd_cap) tl.waves *= 2;
        err = hs::launch_backward_tiles(tl, pa, ba, stream);
        if (err != hipSuccess) return fail_hip(err, (std::string(what) + " (tiles)").c_str());
    }
    if (plan->num_bbig > 0) {
        tl.tiles = plan->d_bbig;
        tl.num_tiles = plan->num_bbig;
        tl.tile_cap = hs::kMaxBwdTileJoints;
        tl.waves = 16;
        tl.grid = plan->num_bbig;
        err = hs::launch_backward_tiles(tl, pa, ba, stream);
        if (err != hipSuccess) return fail_hip(err, (std::string(what) + " (large tiles)").c_str());
    }
    err = hs::launch_backward_multipass(mp_launch(plan, plan->bmp, validate), pa, ba, stream);
    if (err != hipSuccess) return fail_hip(err, (std::string(what) + " (multipass)").c_str());
    return HS_OK;
}

} // namespace

extern "C" {

hs_status hs_mesh_create(const hs_plan *plan, const hs_mesh_batch *mb, hs_mesh **out)
{
    if (!out) return fail(HS_ERR_INVALID_ARG, "hs_mesh_create: out is NULL");
    *out = nullptr;
    if (!plan || !mb) return fail(HS_ERR_INVALID_ARG, "hs_mesh_create: plan and mesh must be non-NULL");
    const int64_t C = plan->C, R = mb->num_rows;
    if (R < 0 || R >= (int64_t(1) << 31)) return fail(HS_ERR_INVALID_ARG, "num_rows %lld out of range", (long long)R);
    if (!mb->vertex_offsets || (C > 0 && !mb->mesh_first) ||
        (R > 0 && (!mb->positions || !mb->joints || !mb->weights)))
        return fail(HS_ERR_INVALID_ARG, "hs_mesh_create: NULL mesh array");
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_mesh_create: cannot select device");
    std::vector<int64_t> voff;
    std::vector<int32_t> mfirst, joints;
    std::vector<float> pos, wts;
    hipError_t err;
    if ((err = fetch(voff, mb->vertex_offsets, (size_t)C + 1)) != hipSuccess ||
        (err = fetch(mfirst, mb->mesh_first, (size_t)C)) != hipSuccess ||
        (err = fetch(joints, mb->joints, (size_t)R * 4)) != hipSuccess ||
        (err = fetch(pos, mb->positions, (size_t)R * 3)) != hipSuccess ||
        (err = fetch(wts, mb->weights, (size_t)R * 4)) != hipSuccess)
        return fail_hip(err, "hs_mesh_create (reading the mesh)");
    if (voff[0] != 0) return fail(HS_ERR_INVALID_ARG, "vertex_offsets[0] must be 0");
    if (voff[C] >= (int64_t(1) << 31)) return fail(HS_ERR_INVALID_ARG, "more than 2^31-1 vertices");
    // joint-id range of each distinct run of mesh rows, computed once
    std::map<std::pair<int64_t, int64_t>, std::pair<int32_t, int32_t>> ranges;
    int max_joints = 0;
    for (int64_t c = 0; c < C; ++c) {
        const int64_t nv = voff[c + 1] - voff[c];
        if (nv < 0) return fail(HS_ERR_INVALID_ARG, "vertex_offsets must be non-decreasing");
        if (nv == 0) continue;
        if (mfirst[c] < 0 || mfirst[c] + nv > R)
            return fail(HS_ERR_INVALID_ARG, "character %lld: mesh rows [%d, %lld) outside [0, %lld)", (long long)c,
                        mfirst[c], (long long)(mfirst[c] + nv), (long long)R);
        const int64_t nj = plan->h_offsets[c + 1] - plan->h_offsets[c];
        if (nj > hs::kMaxSkinJoints)
            return fail(HS_ERR_UNSUPPORTED, "character %lld has %lld joints; vertex skinning stages at most %d",
                        (long long)c, (long long)nj, hs::kMaxSkinJoints);
        max_joints = std::max<int>(max_joints, (int)nj);
        auto key = std::make_pair((int64_t)mfirst[c], nv);
        auto it = ranges.find(key);
        if (it == ranges.end()) {
            int32_t lo = INT32_MAX, hi = INT32_MIN;
            for (int64_t k = 4 * (int64_t)mfirst[c]; k < 4 * (mfirst[c] + nv); ++k) {
                lo = std::min(lo, joints[k]);
                hi = std::max(hi, joints[k]);
            }
            it = ranges.emplace(key, std::make_pair(lo, hi)).first;
        }
        if (it->second.first < 0 || it->second.second >= nj)
            return fail(HS_ERR_INVALID_ARG, "character %lld: joint ids in [%d, %d] but it has %lld joints",
                        (long long)c, it->second.first, it->second.second, (long long)nj);
    }
    hs_mesh *m = new hs_mesh();
    m->plan = plan;
    m->device = plan->ctx->device;
    m->N = plan->N;
    m->V = voff[C];
    m->rows = R;
    if ((err = upload(&m->d_offsets, plan->h_offsets)) != hipSuccess || (err = upload(&m->d_voff, voff)) != hipSuccess ||
        (err = upload(&m->d_mfirst, mfirst)) != hipSuccess || (err = upload(&m->d_joints, joints)) != hipSuccess ||
        (err = upload(&m->d_pos, pos)) != hipSuccess || (err = upload(&m->d_weights, wts)) != hipSuccess) {
        free_mesh(m);
        return fail_hip(err, "hs_mesh_create (upload)");
    }
    hs::VertexLaunch &vl = m->vl;
    vl.offsets = m->d_offsets;
    vl.voff = m->d_voff;
    vl.mfirst = m->d_mfirst;
    vl.pos = m->d_pos;
    vl.joints = m->d_joints;
    vl.weights = m->d_weights;
    vl.C = (int32_t)C;
    vl.max_joints = max_joints;
    *out = m;
    return HS_OK;
}

void hs_mesh_destroy(hs_mesh *mesh) { free_mesh(mesh); }

hs_status hs_skin_vertices(const hs_mesh *mesh, const float *skin, int32_t method, float *out, hipStream_t stream)
{
    if (!mesh) return fail(HS_ERR_INVALID_ARG, "hs_skin_vertices: mesh is NULL");
    if (method != HS_SKIN_LINEAR && method != HS_SKIN_DUAL_QUAT)
        return fail(HS_ERR_INVALID_ARG, "hs_skin_vertices: unknown method %d", method);
    if (mesh->V == 0) return HS_OK;
    if (!skin || !out) return fail(HS_ERR_INVALID_ARG, "hs_skin_vertices: skin and out must be non-NULL");
    if (!aligned(skin, 16) || !aligned(out, 4))
        return fail(HS_ERR_INVALID_ARG, "hs_skin_vertices: skin must be 16-byte and out 4-byte aligned");
    hs_status rc = check_aliasing({{out, (size_t)mesh->V * 12, "out"}}, {{skin, (size_t)mesh->N * 64, "skin"}});
    if (rc != HS_OK) return rc;
    DeviceGuard dg(mesh->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_skin_vertices: cannot select device");
    hipError_t err = hs::launch_vertex_skin(mesh->vl, method, skin, out, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_skin_vertices");
    return HS_OK;
}

hs_status hs_scan_skin_vertices(const hs_plan *plan, const hs_pose_src *src, const float *inv_bind,
                                const hs_mesh *mesh, int32_t method, float *vertices_out, float *skin_out,
                                hipStream_t stream)
{
    if (!plan || !mesh) return fail(HS_ERR_INVALID_ARG, "hs_scan_skin_vertices: plan and mesh must be non-NULL");
    if (mesh->plan != plan) return fail(HS_ERR_INVALID_ARG, "hs_scan_skin_vertices: the mesh was made for another plan");
    if (method != HS_SKIN_LINEAR && method != HS_SKIN_DUAL_QUAT)
        return fail(HS_ERR_INVALID_ARG, "hs_scan_skin_vertices: unknown method %d", method);
    if (plan->mp.nmp > 0 || plan->mp.chain_joints > 0)
        return fail(HS_ERR_UNSUPPORTED, "hs_scan_skin_vertices: every character must be on a tile (no multipass)");
    if (plan->shape.tile_cap > hs::kMaxVertexTileJoints)
        return fail(HS_ERR_UNSUPPORTED, "hs_scan_skin_vertices: tiles of at most %d joints (plan has %d)",
                    hs::kMaxVertexTileJoints, plan->shape.tile_cap);
    hs::PoseArgs pa;
    std::vector<Range> ins;
    hs_status rc = check_pose_src(plan, src, pa, ins, true);
    if (rc != HS_OK) return rc;
    const size_t N = (size_t)plan->N, V = (size_t)mesh->V;
    if (N == 0) return HS_OK;
    if (!inv_bind || (V > 0 && !vertices_out))
        return fail(HS_ERR_INVALID_ARG, "hs_scan_skin_vertices: inv_bind and vertices_out must be non-NULL");
    if (!aligned(inv_bind, 16) || !aligned(skin_out, 16) || !aligned(vertices_out, 4))
        return fail(HS_ERR_INVALID_ARG, "hs_scan_skin_vertices: inv_bind and skin_out must be 16-byte aligned");
    ins.push_back({inv_bind, (plan->inst ? (size_t)plan->skel_joints : N) * 64, "inv_bind"});
    std::vector<Range> outs = {{vertices_out, V * 12, "vertices_out"}, {skin_out, skin_out ? N * 64 : 0, "skin_out"}};
    if ((rc = check_aliasing(outs, ins)) != HS_OK) return rc;
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_scan_skin_vertices: cannot select device");
    hs::OutArgs oa{};
    oa.inv_bind = inv_bind;
    oa.skin_out = skin_out;
    hipError_t err = hipSuccess;
    for (int k = 0; k < (int)plan->small.size() && err == hipSuccess; ++k)
        err = hs::launch_forward_vertices(tile_launch(plan, k), pa, oa, mesh->vl, method, vertices_out, stream);
    if (err == hipSuccess)
        err = hs::launch_forward_vertices(tile_launch(plan), pa, oa, mesh->vl, method, vertices_out, stream);
    if (err != hipSuccess) return fail_hip(err, "hs_scan_skin_vertices");
    return HS_OK;
}

hs_status hs_scan_backward(const hs_plan *plan, const hs_pose_src *src, const float *grad_global, const float *ckpt,
                           int32_t ckpt_k, float *grad_quat, float *grad_trans, float *grad_scale, uint32_t flags,
                           hipStream_t stream)
{
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_scan_backward: plan is NULL");
    if (flags & ~HS_FLAG_VALIDATE) return fail(HS_ERR_INVALID_ARG, "hs_scan_backward: unknown flags 0x%x", flags);
    if (ckpt && ckpt_k < 1) return fail(HS_ERR_INVALID_ARG, "hs_scan_backward: ckpt_k must be >= 1");
    if (plan->N == 0) return HS_OK;  // zero-size arrays may be NULL
    if (!grad_global || !grad_quat || !grad_trans)
        return fail(HS_ERR_INVALID_ARG, "hs_scan_backward: grad_global, grad_quat and grad_trans must be non-NULL");
    if (ckpt && ckpt_k < 1) return fail(HS_ERR_INVALID_ARG, "hs_scan_backward: ckpt_k must be >= 1");
    for (const void *p : {(const void *)grad_global, (const void *)grad_quat, (const void *)ckpt})
        if (p && !aligned(p, 16)) return fail(HS_ERR_INVALID_ARG, "hs_scan_backward: grad_global, grad_quat and ckpt must be 16-byte aligned");
    if (!aligned(grad_trans, 4) || (grad_scale && !aligned(grad_scale, 4)))
        return fail(HS_ERR_INVALID_ARG, "hs_scan_backward: grad_trans/grad_scale must be 4-byte aligned");
    hs::PoseArgs pa;
    std::vector<Range> ins;
    hs_status rc = check_pose_src(plan, src, pa, ins, false);
    if (rc != HS_OK) return rc;
    const size_t N = (size_t)plan->N;
    ins.push_back({grad_global, N * 64, "grad_global"});
    ins.push_back({ckpt, ckpt ? N * 48 : 0, "ckpt"});
    std::vector<Range> outs = {{grad_quat, N * 16, "grad_quat"}, {grad_trans, N * 12, "grad_trans"},
                               {grad_scale, grad_scale ? N * 12 : 0, "grad_scale"}};
    if ((rc = check_aliasing(outs, ins)) != HS_OK) return rc;
    if (N == 0) return HS_OK;
    hs::BwdArgs ba{};
    ba.grad_global = grad_global;
    ba.ckpt = ckpt;
    ba.ckpt_k = ckpt ? ckpt_k : 1;
    ba.level = plan->d_level;
    ba.grad_quat = grad_quat;
    ba.grad_trans = grad_trans;
    ba.grad_scale = grad_scale;
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_scan_backward: cannot select device");
    return run_backward(plan, pa, ba, stream, "hs_scan_backward", (flags & HS_FLAG_VALIDATE) != 0);
}

} // extern "C"

// ---------------------------------------------------------------------------
// End-effector losses: the adjoint seeded from a list of joints.
// ---------------------------------------------------------------------------
struct hs_effectors {
    const hs_plan *plan = nullptr;  // the plan it was made for
    int device = 0;
    int64_t E = 0;
    // every adjoint tile runs the synchronous-round kernel: the seeds are
    // formed inside it from these tables
    bool sparse = false;
    int64_t *d_ids = nullptr;   // ascending (sparse) or in the caller's order (dense)
    int32_t *d_row = nullptr;   // target row of each sorted id
    int32_t *d_tile = nullptr;  // [num_btiles][2]: each tile's range of d_ids
    float *d_dense = nullptr;   // dense seed [N,16], zero outside the effector rows
};

namespace {

void free_effectors(hs_effectors *e)
{
    if (!e) return;
    (void)hipFree(e->d_ids);
    (void)hipFree(e->d_row);
    (void)hipFree(e->d_tile);
    (void)hipFree(e->d_dense);
    delete e;
}

} // namespace

extern "C" {

hs_status hs_effectors_create(const hs_plan *plan, int64_t num_effectors, const int64_t *joint_ids,
                              hs_effectors **out)
{
    if (!out) return fail(HS_ERR_INVALID_ARG, "hs_effectors_create: out is NULL");
    *out = nullptr;
    if (!plan) return fail(HS_ERR_INVALID_ARG, "hs_effectors_create: plan is NULL");
    if (num_effectors < 0 || num_effectors >= (int64_t(1) << 31))
        return fail(HS_ERR_INVALID_ARG, "hs_effectors_create: num_effectors %lld out of range",
                    (long long)num_effectors);
    if (num_effectors > 0 && !joint_ids) return fail(HS_ERR_INVALID_ARG, "hs_effectors_create: joint_ids is NULL");
    const int64_t E = num_effectors, N = plan->N;
    std::vector<int64_t> ids(joint_ids, joint_ids + E);
    std::vector<int32_t> order((size_t)E);
    for (int64_t i = 0; i < E; ++i) {
        if (ids[i] < 0 || ids[i] >= N)
            return fail(HS_ERR_INVALID_ARG, "hs_effectors_create: joint id %lld outside [0, %lld)",
                        (long long)ids[i], (long long)N);
        order[i] = (int32_t)i;
    }
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ids[a] < ids[b]; });
    for (int64_t i = 1; i < E; ++i)
        if (ids[order[i]] == ids[order[i - 1]])
            return fail(HS_ERR_INVALID_ARG, "hs_effectors_create: joint %lld listed twice", (long long)ids[order[i]]);
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_effectors_create: cannot select device");
    hs_effectors *e = new hs_effectors();
    e->plan = plan;
    e->device = plan->ctx->device;
    e->E = E;
    e->sparse = plan->num_btiles > 0 && plan->num_bbig == 0 && plan->bmp.num_blocks == 0 &&
                plan->bwd_untiled == 0 && plan->shape.adjoint != hs::kAdjDataflow;
    hipError_t err = hipSuccess;
    if (e->sparse) {
        std::vector<int64_t> sorted((size_t)std::max<int64_t>(E, 1), 0);  // never an empty (NULL) table
        std::vector<int32_t> row((size_t)std::max<int64_t>(E, 1), 0);
        for (int64_t i = 0; i < E; ++i) {
            sorted[i] = ids[order[i]];
            row[i] = order[i];
        }
        // each adjoint tile's range [lo, hi) of the sorted ids
        std::vector<int32_t> tile(2 * plan->h_btiles.size(), 0);
        int64_t covered = 0;
        for (size_t t = 0; t < plan->h_btiles.size(); ++t) {
            const hs::TileDesc &td = plan->h_btiles[t];
            const auto lo = std::lower_bound(sorted.begin(), sorted.begin() + E, td.begin);
            const auto hi = std::lower_bound(sorted.begin(), sorted.begin() + E, td.begin + td.count);
            tile[2 * t] = (int32_t)(lo - sorted.begin());
            tile[2 * t + 1] = (int32_t)(hi - sorted.begin());
            covered += hi - lo;
        }
        if (covered != E) {  // the adjoint's tiles cover every joint of such a plan
            free_effectors(e);
            return fail(HS_ERR_DEVICE, "hs_effectors_create: %lld ids outside the adjoint's tiles",
                        (long long)(E - covered));
        }
        if ((err = upload(&e->d_ids, sorted)) != hipSuccess || (err = upload(&e->d_row, row)) != hipSuccess ||
            (err = upload(&e->d_tile, tile)) != hipSuccess) {
            free_effectors(e);
            return fail_hip(err, "hs_effectors_create (upload)");
        }
    } else if (N > 0) {
        // the general adjoint reads a dense seed: the loss gradient kernel
        // writes the effector rows of this zeroed buffer on every call
        if ((err = upload(&e->d_ids, ids)) != hipSuccess ||
            (err = hipMalloc(reinterpret_cast<void **>(&e->d_dense), (size_t)N * 64)) != hipSuccess ||
            (err = hipMemset(e->d_dense, 0, (size_t)N * 64)) != hipSuccess ||
            (err = hipDeviceSynchronize()) != hipSuccess) {
            free_effectors(e);
            return fail_hip(err, "hs_effectors_create (dense seed)");
        }
    }
    *out = e;
    return HS_OK;
}

void hs_effectors_destroy(hs_effectors *effectors) { free_effectors(effectors); }

int32_t hs_effectors_sparse(const hs_effectors *effectors) { return effectors && effectors->sparse ? 1 : 0; }

hs_status hs_effector_backward(const hs_plan *plan, const hs_effectors *effectors, const hs_pose_src *src,
                               const float *global, const float *targets, float *grad_quat, float *grad_trans,
                               float *grad_scale, hipStream_t stream)
{
    if (!plan || !effectors) return fail(HS_ERR_INVALID_ARG, "hs_effector_backward: plan and effectors must be non-NULL");
    if (effectors->plan != plan)
        return fail(HS_ERR_INVALID_ARG, "hs_effector_backward: the effectors were made for another plan");
    if (plan->N == 0) return HS_OK;
    const size_t N = (size_t)plan->N, E = (size_t)effectors->E;
    if (!global || !grad_quat || !grad_trans || (E > 0 && !targets))
        return fail(HS_ERR_INVALID_ARG, "hs_effector_backward: global, targets, grad_quat and grad_trans must be non-NULL");
    if (!aligned(global, 16) || !aligned(grad_quat, 16))
        return fail(HS_ERR_INVALID_ARG, "hs_effector_backward: global and grad_quat must be 16-byte aligned");
    if (!aligned(targets, 4) || !aligned(grad_trans, 4) || (grad_scale && !aligned(grad_scale, 4)))
        return fail(HS_ERR_INVALID_ARG, "hs_effector_backward: targets/grad_trans/grad_scale must be 4-byte aligned");
    hs::PoseArgs pa;
    std::vector<Range> ins;
    hs_status rc = check_pose_src(plan, src, pa, ins, false);
    if (rc != HS_OK) return rc;
    ins.push_back({global, N * 64, "global"});
    ins.push_back({targets, E * 12, "targets"});
    std::vector<Range> outs = {{grad_quat, N * 16, "grad_quat"}, {grad_trans, N * 12, "grad_trans"},
                               {grad_scale, grad_scale ? N * 12 : 0, "grad_scale"}};
    if ((rc = check_aliasing(outs, ins)) != HS_OK) return rc;
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_effector_backward: cannot select device");
    hs::BwdArgs ba{};
    ba.ckpt_k = 1;
    ba.level = plan->d_level;
    ba.grad_quat = grad_quat;
    ba.grad_trans = grad_trans;
    ba.grad_scale = grad_scale;
    if (effectors->sparse) {
        ba.eff_ids = effectors->d_ids;
        ba.eff_row = effectors->d_row;
        ba.eff_tile = effectors->d_tile;
        ba.eff_global = global;
        ba.eff_target = targets;
    } else {
        hipError_t err = hs::launch_effector_grad(plan->N, effectors->E, effectors->d_ids, global, targets,
                                                  effectors->d_dense, stream);
        if (err != hipSuccess) return fail_hip(err, "hs_effector_backward (seed)");
        ba.grad_global = effectors->d_dense;
    }
    return run_backward(plan, pa, ba, stream, "hs_effector_backward");
}

hs_status hs_effector_step(const hs_plan *plan, const hs_effectors *effectors, const hs_pose_src *src,
                           const float *targets, float *global_out, float *grad_quat, float *grad_trans,
                           float *grad_scale, hipStream_t stream)
{
    if (!plan || !effectors) return fail(HS_ERR_INVALID_ARG, "hs_effector_step: plan and effectors must be non-NULL");
    if (effectors->plan != plan)
        return fail(HS_ERR_INVALID_ARG, "hs_effector_step: the effectors were made for another plan");
    if (!effectors->sparse)
        return fail(HS_ERR_UNSUPPORTED, "hs_effector_step: the plan's adjoint does not run on synchronous tiles only "
                                        "(characters over 1024 joints, the dataflow option or multipass); use "
                                        "hs_scan_forward and hs_effector_backward");
    if (plan->N == 0) return HS_OK;
    const size_t N = (size_t)plan->N, E = (size_t)effectors->E;
    if (!grad_quat || !grad_trans || (E > 0 && !targets))
        return fail(HS_ERR_INVALID_ARG, "hs_effector_step: targets, grad_quat and grad_trans must be non-NULL");
    if (!aligned(global_out, 16) || !aligned(grad_quat, 16))
        return fail(HS_ERR_INVALID_ARG, "hs_effector_step: global_out and grad_quat must be 16-byte aligned");
    if (!aligned(targets, 4) || !aligned(grad_trans, 4) || (grad_scale && !aligned(grad_scale, 4)))
        return fail(HS_ERR_INVALID_ARG, "hs_effector_step: targets/grad_trans/grad_scale must be 4-byte aligned");
    hs::PoseArgs pa;
    std::vector<Range> ins;
    hs_status rc = check_pose_src(plan, src, pa, ins, false);
    if (rc != HS_OK) return rc;
    ins.push_back({targets, E * 12, "targets"});
    std::vector<Range> outs = {{global_out, global_out ? N * 64 : 0, "global_out"},
                               {grad_quat, N * 16, "grad_quat"}, {grad_trans, N * 12, "grad_trans"},
                               {grad_scale, grad_scale ? N * 12 : 0, "grad_scale"}};
    if ((rc = check_aliasing(outs, ins)) != HS_OK) return rc;
    DeviceGuard dg(plan->ctx->device);
    if (!dg.ok) return fail(HS_ERR_DEVICE, "hs_effector_step: cannot select device");
    hs::BwdArgs ba{};
    ba.ckpt_k = 1;
    ba.level = plan->d_level;
    ba.grad_quat = grad_quat;
    ba.grad_trans = grad_trans;
    ba.grad_scale = grad_scale;
    ba.eff_ids = effectors->d_ids;
    ba.eff_row = effectors->d_row;
    ba.eff_tile = effectors->d_tile;
    ba.eff_target = targets;
    ba.eff_forward = 1;
    ba.eff_global_out = global_out;
    return run_backward(plan, pa, ba, stream, "hs_effector_step");
}

} // extern "C"
