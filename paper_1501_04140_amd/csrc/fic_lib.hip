// Host runtime and C ABI of libfic (see include/fic.h).
//
// Every entry point validates its arguments on the host, then queues kernels
// on the caller's stream. Per-level counts that depend on the data (pool size,
// active ranges, codes) stay in a device control block. Kernels are launched
// with worst-case grids and read those counts themselves, so the quadtree
// runs with no host synchronisation between levels.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fic_internal.h"
#include "fic_kernels.hip"
#include "fic_mlp_kernels.hip"
#include "fic_persist.hip"
#include "fic_peaks.hip"

#define FIC_API extern "C" __attribute__((visibility("default")))

namespace fic {
namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(FIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK()                                                                    \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess) return fail(FIC_EDEVICE, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

// Domain-side buffers of one quadtree level: they depend only on the image,
// so the pools of all levels are built concurrently.
struct PoolBufs {
    Buf key, pool, hl, sd, ad, jd, blk;
    Buf dh, dl, wd;  // MFMA grid matchers (B = 8): exact and normalized columns, 40 / A'
};

constexpr int kLevels = 4;

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    Ctrl* ctrl = nullptr;  // [1 + kLevels]: the quadtree's control, then each level's pool control
    int64_t* T = nullptr;  // entropy table, kMaxWindow + 1 entries
    PoolBufs pl[kLevels];
    Buf arow, sr, cr, part, blk, act0, act1, tmpc, dec, codes, map, imgA, imgB, acc, mr;
    Buf ar, srp, gb, rc;  // MFMA grid matchers (B = 8): rows, sum r', shared bounds, int8 row offsets
    Buf plan;     // bitstream section offsets
    hipStream_t side[kLevels] = {};  // one per level's pool phase (default priority)
    hipEvent_t ev_fork = nullptr, ev_pool[kLevels] = {};
    // device copy of one image's level arguments (the pool steps of several
    // levels share launches through it) and its host mirror
    Lvl* dlv = nullptr;
    Lvl hlv[kLevels];
    int nlv = 0;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

const std::vector<int64_t>& entropy_table() {
    static const std::vector<int64_t> t = [] {
        std::vector<int64_t> v(kMaxWindow + 1, 0);
        for (int c = 2; c <= kMaxWindow; ++c)
            v[c] = llround((double)c * std::log2((double)c) * std::ldexp(1.0, kEntFrac));
        return v;
    }();
    return t;
}

// Fixed-point form of Nw * (log2 Nw - theta): entropy > theta iff key < M.
int64_t entropy_cut(int nw, double theta) {
    double v = (double)nw * (std::log2((double)nw) - theta) * std::ldexp(1.0, kEntFrac);
    if (v <= 0) return 0;
    return llround(v);
}

// A new workspace bound to stream s: control block and entropy table.
int new_ws(int dev, hipStream_t s, Workspace** out) {
    Workspace* ws = new Workspace();
    ws->device = dev;
    ws->stream = s;
    if (hipMalloc(&ws->ctrl, sizeof(Ctrl) * (1 + kLevels)) != hipSuccess) {
        delete ws;
        return fail(FIC_ENOMEM, "hipMalloc of the control block failed");
    }
    if (hipMalloc(&ws->T, sizeof(int64_t) * (kMaxWindow + 1)) != hipSuccess) {
        (void)hipFree(ws->ctrl);
        delete ws;
        return fail(FIC_ENOMEM, "hipMalloc of the entropy table failed");
    }
    const std::vector<int64_t>& t = entropy_table();
    HIP_TRY(hipMemcpy(ws->T, t.data(), sizeof(int64_t) * t.size(), hipMemcpyHostToDevice));
    std::vector<Ctrl> init(1 + kLevels);  // zero counters, empty histograms, no floor bound yet
    std::memset(init.data(), 0, sizeof(Ctrl) * init.size());
    for (Ctrl& c : init) c.cut_bound = ~0ull;
    HIP_TRY(hipMemcpy(ws->ctrl, init.data(), sizeof(Ctrl) * init.size(), hipMemcpyHostToDevice));
    *out = ws;
    return FIC_OK;
}

// Level streams and events of a workspace that forks the pool phases (made on first use).
int ensure_fork(Workspace& ws) {
    if (ws.ev_fork) return FIC_OK;
    for (int l = 0; l < kLevels; ++l) {
        HIP_TRY(hipStreamCreateWithFlags(&ws.side[l], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ws.ev_pool[l], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&ws.ev_fork, hipEventDisableTiming));
    if (hipMalloc(&ws.dlv, sizeof(Lvl) * kLevels) != hipSuccess) {
        ws.dlv = nullptr;
        return fail(FIC_ENOMEM, "hipMalloc of the level table failed");
    }
    return FIC_OK;
}

// Device copy of an image's level arguments, rewritten only when they change
// (after the work that may still read the old copy has finished).
int upload_levels(Workspace& ws, const std::vector<Lvl>& t) {
    const int n = (int)t.size();
    if (n == ws.nlv && std::memcmp(ws.hlv, t.data(), sizeof(Lvl) * n) == 0) return FIC_OK;
    HIP_TRY(hipStreamSynchronize(ws.stream));
    for (hipStream_t sd : ws.side)
        if (sd) HIP_TRY(hipStreamSynchronize(sd));
    std::memcpy(ws.hlv, t.data(), sizeof(Lvl) * n);
    ws.nlv = n;
    HIP_TRY(hipMemcpy(ws.dlv, ws.hlv, sizeof(Lvl) * n, hipMemcpyHostToDevice));
    return FIC_OK;
}

int get_ws(hipStream_t s, Workspace** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find({dev, s});
    if (it != g_ws.end()) {
        *out = it->second;
        return FIC_OK;
    }
    Workspace* ws;
    int rc = new_ws(dev, s, &ws);
    if (rc) return rc;
    g_ws[{dev, s}] = ws;
    *out = ws;
    return FIC_OK;
}

void free_ws(Workspace* ws) {
    Buf* bufs[] = {&ws->arow, &ws->sr, &ws->cr, &ws->part, &ws->blk, &ws->act0, &ws->act1,
                   &ws->tmpc, &ws->dec, &ws->codes, &ws->map, &ws->imgA, &ws->imgB, &ws->acc,
                   &ws->mr, &ws->ar, &ws->srp, &ws->gb, &ws->rc, &ws->plan};
    for (Buf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (PoolBufs& pb : ws->pl) {
        Buf* pbs[] = {&pb.key, &pb.pool, &pb.hl, &pb.sd, &pb.ad, &pb.jd, &pb.blk, &pb.dh, &pb.dl, &pb.wd};
        for (Buf* b : pbs)
            if (b->p) (void)hipFree(b->p);
    }
    for (int l = 0; l < kLevels; ++l) {
        if (ws->side[l]) (void)hipStreamDestroy(ws->side[l]);
        if (ws->ev_pool[l]) (void)hipEventDestroy(ws->ev_pool[l]);
    }
    if (ws->ev_fork) (void)hipEventDestroy(ws->ev_fork);
    if (ws->dlv) (void)hipFree(ws->dlv);
    (void)hipFree(ws->ctrl);
    (void)hipFree(ws->T);
    delete ws;
}

int ensure(Workspace& ws, Buf& b, size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (b.cap >= bytes) return FIC_OK;
    if (b.p) {
        // the buffer may still be in use on the caller's stream or a level's stream
        HIP_TRY(hipStreamSynchronize(ws.stream));
        for (hipStream_t sd : ws.side)
            if (sd) HIP_TRY(hipStreamSynchronize(sd));
        HIP_TRY(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 255) & ~(size_t)255;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FIC_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    b.cap = want;
    return FIC_OK;
}

template <typename T>
T* P(Buf& b) {
    return reinterpret_cast<T*>(b.p);
}

// ---------------------------------------------------------------- profiling
// While on, each launch of a library kernel is bracketed by two HIP events on
// its stream; fic_profile_end sums the intervals per kernel label.
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};
struct Prof {
    std::mutex mu;
    bool on = false;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> spare;
} g_prof;

// Set while a call that must not create events (fic_encode_level_noalloc) queues work.
thread_local bool g_prof_off = false;

hipEvent_t prof_event() {
    if (!g_prof.spare.empty()) {
        hipEvent_t e = g_prof.spare.back();
        g_prof.spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

class ProfScope {
  public:
    ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
        if (g_prof_off) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.on) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        a_ = prof_event();
        b_ = prof_event();
        if (a_ && b_) (void)hipEventRecord(a_, s_);
    }
    ~ProfScope() {
        if (!a_ || !b_) return;
        (void)hipEventRecord(b_, s_);
        std::lock_guard<std::mutex> lk(g_prof.mu);
        g_prof.recs.push_back({name_, a_, b_});
    }

  private:
    const char* name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// Profile label of a per-level pool or quadtree step: "<step>_b<B>".
const char* level_label(const char* step, int B) {
    static const char* const names[][4] = {
        {"pool_score_b2", "pool_score_b4", "pool_score_b8", "pool_score_b16"},
        {"pool_bound_b2", "pool_bound_b4", "pool_bound_b8", "pool_bound_b16"},
        {"pool_count_b2", "pool_count_b4", "pool_count_b8", "pool_count_b16"},
        {"pool_scatter_b2", "pool_scatter_b4", "pool_scatter_b8", "pool_scatter_b16"},
        {"pool_select_b2", "pool_select_b4", "pool_select_b8", "pool_select_b16"},
        {"pool_prep_b2", "pool_prep_b4", "pool_prep_b8", "pool_prep_b16"},
        {"reduce_quad_b2", "reduce_quad_b4", "reduce_quad_b8", "reduce_quad_b16"},
        {"quad_compact_b2", "quad_compact_b4", "quad_compact_b8", "quad_compact_b16"}};
    static const char* const steps[] = {"pool_score", "pool_bound", "pool_count", "pool_scatter",
                                        "pool_select", "pool_prep", "reduce_quad", "quad_compact"};
    const int b = B == 2 ? 0 : B == 4 ? 1 : B == 8 ? 2 : 3;
    for (int i = 0; i < 8; ++i)
        if (std::strcmp(step, steps[i]) == 0) return names[i][b];
    return step;
}

// Whether kernel profiling is on (the one-image encode then queues on one stream).
bool prof_active() {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    return g_prof.on;
}

const char* match_label(int B) {
    switch (B) {
        case 2: return "match_b2";
        case 4: return "match_b4";
        case 8: return "match_b8";
        default: return "match_b16";
    }
}

// ---------------------------------------------------------------- validation
int check_kset(const int8_t* k, int n, KSet* ks) {
    if (!k) return fail(FIC_EINVAL, "contrast set is NULL");
    if (n < 1 || n > FIC_MAX_S) return fail(FIC_EINVAL, "contrast set size %d not in 1..%d", n, FIC_MAX_S);
    std::memset(ks, 0, sizeof *ks);
    ks->n = n;
    ks->consecutive = 1;
    for (int i = 0; i < n; ++i) {
        if (k[i] < 0 || k[i] > 10) return fail(FIC_EINVAL, "contrast k=%d not in 0..10", (int)k[i]);
        if (i > 0 && k[i] <= k[i - 1]) return fail(FIC_EINVAL, "contrast set not strictly increasing");
        ks->k[i] = k[i];
        if (k[i] != k[0] + i) ks->consecutive = 0;
    }
    ks->k0 = k[0];
    ks->k1 = k[n - 1];
    return FIC_OK;
}

bool valid_B(int B) { return B == 2 || B == 4 || B == 8 || B == 16; }

// Matcher mode for a contrast set (kt_match's MODE).
int match_mode(const KSet& ks) {
    return ks.n <= kSmallMax ? kModeSmall : (ks.consecutive ? kModeGrid : kModeList);
}

// ---------------------------------------------------------------- one level
// Matcher selected for a level (fic_encode_level_ex's variant).

// The int8 MFMA matcher serves B = 8 with a contrast grid 0..k1 (k1 >= 2) on
// domain grids it can index (fewer than kM8MaxPool domains).
bool mfma_eligible(int B, const KSet& ks, int64_t total = 0) {
    return B == 8 && ks.consecutive && ks.k0 == 0 && ks.n >= 3 && total < kM8MaxPool;
}

// Nonzero values of a contrast set.
int nonzero_values(const KSet& ks) {
    int c = 0;
    for (int u = 0; u < ks.n; ++u) c += ks.k[u] != 0;
    return c;
}

// The FP16 MFMA matcher for small sets serves B = 4, 8 and 16 with one or two
// values, at least one of them nonzero, on grids below kMqMaxPool domains.
bool mfq_eligible(int B, const KSet& ks, int64_t total = 0) {
    return (B == 4 || B == 8 || B == 16) && match_mode(ks) == kModeSmall && nonzero_values(ks) >= 1 &&
           total < kMqMaxPool;
}

// Matcher a level gets by default.
int auto_var(int B, const KSet& ks, int64_t total) {
    if (mfma_eligible(B, ks, total)) return kVarMfma;
    if (mfq_eligible(B, ks, total)) return kVarMfq;
    return kVarValu;
}

// Host plan of one level of one image.
struct Level {
    int lv, B, L, gy, gx, total;  // domain grid
    int max_act;                  // worst-case active ranges
    int nc;                       // pool chunks of the matcher
    int cg;                       // domains per pool chunk
    int var;                      // kVarValu, kVarMfma, kVarFp32, kVarMfma16 or kVarMfq
    KSet ks;
};

bool is_mfma8(int var) { return var == kVarMfma || var == kVarMfma16; }

int default_cg(int B, int var) {
    if (is_mfma8(var)) return kM8Chunk;
    // several LDS stages per workgroup: its range staging, A operands and
    // the final merge across column lanes are paid once per chunk
    if (var == kVarMfq) return B == 16 ? 4 * mq_cols(B) : 256;
    if (var == kVarFp32) return 256;
    return match_chunk_domains(B);
}

Level make_level(int lv, int H, int W, int B, int L, int max_act, const KSet& ks, int variant = 0,
                 int cg = 0) {
    Level v;
    v.var = variant != 0 ? variant : auto_var(B, ks, (int64_t)((H - 2 * B) / L + 1) * ((W - 2 * B) / L + 1));
    v.lv = lv;
    v.B = B;
    v.L = L;
    v.gy = (H - 2 * B) / L + 1;
    v.gx = (W - 2 * B) / L + 1;
    v.total = v.gy * v.gx;
    v.max_act = max_act;
    v.ks = ks;
    v.cg = cg > 0 ? cg : default_cg(B, v.var);
    // enough workgroups to fill the chip when the pool is large, at most one
    // chunk per cg domains and 64 chunks
    const int rows_per_block = is_mfma8(v.var) ? m8_rows(v.var == kVarMfma16)
                               : v.var == kVarMfq ? mq_rows(B)
                               : v.var == kVarFp32 ? kBlock
                                                   : 8 * match_ranges_per_block(B, match_mode(ks));
    const int row_blocks = cdiv((int64_t)8 * max_act, rows_per_block);
    int nc = cdiv(2048, row_blocks);
    nc = std::max(1, std::min(nc, 64));
    nc = std::min(nc, std::max(1, cdiv(v.total, v.cg)));
    v.nc = nc;
    return v;
}

struct Sizes {
    size_t rng = 0, part = 0, blk = 0, act = 0, ar = 0;                // range side, all levels
    size_t key[kLevels] = {}, hl[kLevels] = {}, dom[kLevels] = {};      // domain side, per level
    size_t pblk[kLevels] = {}, dcol[kLevels] = {};
    size_t dq[kLevels] = {};  // FP16 pool columns of the small-set MFMA matcher, bytes
};

void grow(Sizes& s, const Level& v) {
    const int n = v.B * v.B;
    const int l = v.lv;
    s.key[l] = std::max(s.key[l], (size_t)v.total * 8);
    s.hl[l] = std::max(s.hl[l], (size_t)v.total * (n / 2) * 4);
    s.dom[l] = std::max(s.dom[l], (size_t)v.total);
    s.pblk[l] = std::max(s.pblk[l], (size_t)cdiv(v.total, kBlock * kPoolItems) * sizeof(int2));
    s.rng = std::max(s.rng, (size_t)v.max_act);
    s.part = std::max(s.part, (size_t)v.max_act * v.nc * sizeof(Partial));
    s.blk = std::max(s.blk, (size_t)cdiv(v.max_act, kRqRanges) * sizeof(int2));
    s.act = std::max(s.act, (size_t)v.max_act);
    if (is_mfma8(v.var)) {
        s.ar = std::max(s.ar, (size_t)v.max_act * 8 * 64 * 2);  // int8 rows, or FP16 (2 bytes)
        s.dcol[l] = std::max(s.dcol[l], (size_t)v.total);
    }
    if (v.var == kVarMfq) s.dq[l] = std::max(s.dq[l], (size_t)v.total * n * 2);
}

// Every workspace buffer a plan of these sizes needs, in a fixed order:
// get(buffer, bytes) for each. Sizing through the allocator (ensure_sizes)
// and placing in the fixed device scratch (carve_sizes) both walk this list.
template <typename Get>
int visit_sizes(Workspace& ws, const Sizes& s, Get get) {
    int rc;
    for (int l = 0; l < kLevels; ++l) {
        if (!s.dom[l]) continue;
        PoolBufs& pb = ws.pl[l];
        if ((rc = get(pb.key, s.key[l]))) return rc;
        if ((rc = get(pb.pool, s.dom[l] * 4))) return rc;
        if ((rc = get(pb.hl, s.hl[l]))) return rc;
        if ((rc = get(pb.sd, s.dom[l] * 4))) return rc;
        if ((rc = get(pb.ad, s.dom[l] * 8))) return rc;
        if ((rc = get(pb.jd, s.dom[l] * 4))) return rc;
        if ((rc = get(pb.blk, s.pblk[l]))) return rc;
        if (s.dq[l] && (rc = get(pb.dh, s.dq[l]))) return rc;
        if (s.dcol[l]) {
            if ((rc = get(pb.dh, s.dcol[l] * 128))) return rc;  // h rows, or FP16 columns
            if ((rc = get(pb.dl, s.dcol[l] * 128))) return rc;  // l rows, or normalized FP16 columns
            if ((rc = get(pb.wd, s.dcol[l] * 4))) return rc;
        }
    }
    if ((rc = get(ws.sr, s.rng * 4))) return rc;
    if ((rc = get(ws.cr, s.rng * 8))) return rc;
    if ((rc = get(ws.part, s.part))) return rc;
    if ((rc = get(ws.blk, s.blk))) return rc;
    if ((rc = get(ws.act0, s.act * 4))) return rc;
    if ((rc = get(ws.act1, s.act * 4))) return rc;
    if ((rc = get(ws.tmpc, s.act * sizeof(fic_code)))) return rc;
    if ((rc = get(ws.dec, s.act))) return rc;
    if (s.ar) {
        if ((rc = get(ws.ar, s.ar))) return rc;
        if ((rc = get(ws.srp, s.rng * 4))) return rc;
        if ((rc = get(ws.gb, s.rng * 8))) return rc;
        if ((rc = get(ws.rc, s.rng * 8))) return rc;
    }
    return FIC_OK;
}

int ensure_sizes(Workspace& ws, const Sizes& s) {
    return visit_sizes(ws, s, [&ws](Buf& b, size_t bytes) { return ensure(ws, b, bytes); });
}

// Kernel arguments of one image at one level.
Lvl make_lvl(Workspace& ws, const Level& v, const uint8_t* img, int H, int W, int pitch,
             int entropy_mode, float entropy_bits, int min_pool, int32_t* act, int32_t* act_next,
             int last, int64_t thr, fic_code* codes, int capacity, fic_level_stats* stats) {
    Lvl a;
    std::memset(&a, 0, sizeof a);
    a.img = img;
    a.pitch = pitch;
    a.H = H;
    a.W = W;
    a.B = v.B;
    a.L = v.L;
    a.gx = v.gx;
    a.gy = v.gy;
    a.total = v.total;
    a.max_act = v.max_act;
    a.lv = v.lv;
    a.last = last;
    a.nc = v.nc;
    a.cg = v.cg;
    a.var = v.var;
    a.min_pool = min_pool;
    a.rank = std::min(min_pool, v.total);
    const int side = 2 * v.B;
    a.pmode = entropy_mode;
    a.M = entropy_mode == 1 ? entropy_cut(side * side, (double)entropy_bits) : 0;
    if (entropy_mode == 2) {
        // keep iff V' > t N^2, i.e. V' > floor(t N^2) (exact in double: t is a float, N^2 <= 2^20)
        const double nn = (double)side * side * side * side;
        a.kv = (int64_t)(side * side) * (side * side) * 16257;  // > N^2 * 127.5^2 >= V'
        const double cut = std::floor((double)entropy_bits * nn);
        const double m = (double)a.kv - cut;
        a.M = m <= 0.0 ? 0 : (m > (double)a.kv + 1.0 ? a.kv + 1 : (int64_t)m);
    }
    {
        const int64_t maxkey = entropy_mode == 2 ? a.kv + 1 : entropy_table()[side * side] + 1;
        int shift = 0;
        while ((maxkey >> shift) >= kSelBins) ++shift;
        a.sel_shift = shift;
        a.bound_chunk = std::max(8192, cdiv(v.total, 64));
    }
    a.thr = thr;
    a.capacity = capacity;
    PoolBufs& pb = ws.pl[v.lv];
    a.ctrl = ws.ctrl;
    a.pctrl = ws.ctrl + 1 + v.lv;
    a.key = P<int64_t>(pb.key);
    a.pool = P<int32_t>(pb.pool);
    a.hl = P<uint32_t>(pb.hl);
    a.sd = P<uint32_t>(pb.sd);
    a.ad = P<int64_t>(pb.ad);
    a.jd = P<int32_t>(pb.jd);
    a.pblk = P<int2>(pb.blk);
    a.part = P<Partial>(ws.part);
    a.sr = P<int32_t>(ws.sr);
    a.cr = P<int64_t>(ws.cr);
    a.act = act;
    a.act_next = act_next;
    a.tmpc = P<fic_code>(ws.tmpc);
    a.dec = P<uint8_t>(ws.dec);
    a.blk = P<int2>(ws.blk);
    a.codes = codes;
    a.stats = stats;
    a.ar = P<int8_t>(ws.ar);
    a.srp = P<int32_t>(ws.srp);
    a.gb = P<int64_t>(ws.gb);
    a.rc = P<int2>(ws.rc);
    a.dh = P<int8_t>(pb.dh);
    a.dl = P<int8_t>(pb.dl);
    a.gd = P<float>(pb.wd);
    a.ks = v.ks;
    return a;
}

// keep iff E <= T^2 n  <=>  1600 n E <= 1600 T^2 n^2
int64_t keep_threshold(float rms, int B) {
    const double n = (double)B * B;
    const double thr = std::floor(1600.0 * (double)rms * (double)rms * n * n);
    return thr >= 9.0e18 ? INT64_MAX : (int64_t)thr;
}

template <typename F>
int max_over(const std::vector<Lvl>& h, F f) {
    int m = 1;
    for (const Lvl& a : h) m = std::max(m, f(a));
    return m;
}

// Domains at or above which the entropy keys come from cell histograms.
// (every such grid: at 512^2 the per-window kernel took 13 us at levels 0 and 1, where the
// cell kernel scores level 3's 259081 domains in 5 us)
constexpr int kScoreCellsMin = 0;

// Whether the score step of this level runs the cell kernel (which can also
// write level 0's active list).
bool score_by_cells(const Lvl& a) { return a.pmode != 2 && 4 * a.L == 2 * a.B; }

template <int SIDE, bool TAB>
void launch_score(const Lvl* dt, const std::vector<Lvl>& h, const int64_t* T, hipStream_t st,
                  bool fill_act = false) {
    if (h[0].pmode == 2) {
        const int gx = max_over(h, [](const Lvl& a) { return cdiv((int64_t)a.total * ScoreShape<SIDE>::TPD, kBlock); });
        kt_pool_var<SIDE, TAB><<<dim3(gx, 1, h.size()), kBlock, 0, st>>>(h[0], dt);
        return;
    }
    // large grids with stride L = SIDE / 4: keys from cell histograms
    constexpr int L = SIDE / 4;
    const bool cells = max_over(h, [](const Lvl& a) { return a.total; }) >= kScoreCellsMin &&
                       std::all_of(h.begin(), h.end(), [](const Lvl& a) { return a.L == L; });
    if (cells) {
        const int bx = max_over(h, [](const Lvl& a) { return cdiv(a.gx, sc_tx(L)); });
        const int by = max_over(h, [](const Lvl& a) { return cdiv(a.gy, kScTY); });
        kt_pool_score_cells<L, TAB><<<dim3(bx, by, h.size()), kBlock, 0, st>>>(h[0], dt, T, fill_act ? 1 : 0);
        return;
    }
    const int gx = max_over(h, [](const Lvl& a) { return cdiv((int64_t)a.total * ScoreShape<SIDE>::TPD, kBlock); });
    kt_pool_score<SIDE, TAB><<<dim3(gx, 1, h.size()), kBlock, 0, st>>>(h[0], dt, T);
}

// Domain-side moments of the level's pool (they depend only on the image).
template <int B, bool TAB>
void launch_pool_prep(const Lvl* dt, const std::vector<Lvl>& h, bool filtered, hipStream_t st) {
    const int n = (int)h.size();
    ProfScope ps(level_label("pool_prep", B), st);
    if (B == 8 && is_mfma8(h[0].var)) {
        const int gx = max_over(h, [](const Lvl& a) { return cdiv((int64_t)a.total * 4, kBlock); });
        kt_pool_prep_i8<TAB><<<dim3(gx, 1, n), kBlock, 0, st>>>(h[0], dt, filtered ? 1 : 0);
        return;
    }
    if constexpr (B == 4 || B == 8 || B == 16) {
        if (h[0].var == kVarMfq) {
            const int gx = max_over(h, [](const Lvl& a) { return cdiv((int64_t)a.total * (B * B / 16), kBlock); });
            kt_pool_prep_mq<B, TAB><<<dim3(gx, 1, n), kBlock, 0, st>>>(h[0], dt, filtered ? 1 : 0);
            return;
        }
    }
    const int gx = max_over(h, [](const Lvl& a) { return cdiv((int64_t)a.total * PrepShape<B>::TPD, kBlock); });
    kt_pool_prep<B, TAB><<<dim3(gx, 1, n), kBlock, 0, st>>>(h[0], dt, filtered ? 1 : 0);
}

// The matcher over the level's active ranges (after its pool is ready).
template <int B, bool TAB>
void launch_match(const Lvl* dt, const std::vector<Lvl>& h, hipStream_t st) {
    const int n = (int)h.size();
    const Lvl& a0 = h[0];
    const int max_act = max_over(h, [](const Lvl& a) { return a.max_act; });
    const int max_nc = max_over(h, [](const Lvl& a) { return a.nc; });
    if (B == 8 && is_mfma8(a0.var)) {
        {
            ProfScope ps("range_prep", st);
            kt_range_prep_i8<TAB><<<dim3(cdiv((int64_t)8 * max_act, kBlock), 1, n), kBlock, 0, st>>>(h[0], dt);
        }
        const dim3 grid(cdiv((int64_t)8 * max_act, m8_rows(a0.var == kVarMfma16)), max_nc, n);
        if (a0.var == kVarMfma16) {
            ProfScope ps("match_b8_mfma16", st);
            kt_match_mfma8<true, TAB><<<grid, kM8Waves * 64, 0, st>>>(h[0], dt);
        } else {
            ProfScope ps("match_b8_mfma", st);
            kt_match_mfma8<false, TAB><<<grid, kM8Waves * 64, 0, st>>>(h[0], dt);
        }
        return;
    }
    if (B == 8 && a0.var == kVarFp32) {
        ProfScope ps("match_b8_fp32", st);
        kt_match_fp32<TAB><<<dim3(cdiv(max_act, kBlock / 8), max_nc, n), kBlock, 0, st>>>(h[0], dt);
        return;
    }
    if constexpr (B == 4 || B == 8 || B == 16) {
        if (a0.var == kVarMfq) {
            ProfScope ps(B == 4 ? "match_b4_mfq" : (B == 8 ? "match_b8_mfq" : "match_b16_mfq"), st);
            const dim3 grid(cdiv((int64_t)8 * max_act, mq_rows(B)), max_nc, n);
            if (nonzero_values(a0.ks) > 1) kt_match_mfq<B, 2, TAB><<<grid, kMqWaves * 64, 0, st>>>(h[0], dt);
            else kt_match_mfq<B, 1, TAB><<<grid, kMqWaves * 64, 0, st>>>(h[0], dt);
            return;
        }
    }
    ProfScope ps(match_label(B), st);
    const int mode = match_mode(a0.ks);
    const dim3 grid(cdiv(max_act, match_ranges_per_block(B, mode)), max_nc, n);
    if (mode == kModeSmall) kt_match<B, kModeSmall, TAB><<<grid, kBlock, 0, st>>>(h[0], dt);
    else if (mode == kModeGrid) kt_match<B, kModeGrid, TAB><<<grid, kBlock, 0, st>>>(h[0], dt);
    else kt_match<B, kModeList, TAB><<<grid, kBlock, 0, st>>>(h[0], dt);
}

// Pool of one level: the entropy (or variance) filter of Section 3, or the
// whole grid, and the pool's moments, for h.size() images whose arguments are
// at dt (by value when dt is NULL). Three steps: the keys, the selection
// (which reads only the level's arguments, so levels of different B can share
// its launches), and the moments.
template <bool TAB>
void launch_score_step(const Lvl* dt, const std::vector<Lvl>& h, const int64_t* T, hipStream_t st,
                       bool fill_act = false) {
    ProfScope ps(level_label("pool_score", h[0].B), st);
    switch (2 * h[0].B) {
        case 4: launch_score<4, TAB>(dt, h, T, st, fill_act); break;
        case 8: launch_score<8, TAB>(dt, h, T, st, fill_act); break;
        case 16: launch_score<16, TAB>(dt, h, T, st, fill_act); break;
        default: launch_score<32, TAB>(dt, h, T, st, fill_act); break;
    }
}

template <bool TAB>
void launch_select_steps(const Lvl* dt, const std::vector<Lvl>& h, hipStream_t st) {
    const int n = (int)h.size();
    // small grids: one workgroup stages every key and builds the pool itself
    const bool direct = max_over(h, [](const Lvl& a) { return a.total; }) <= kSelDirect;
    if (!direct) {
        {
            ProfScope ps(level_label("pool_bound", h[0].B), st);
            const int gx = max_over(h, [](const Lvl& a) { return cdiv(a.total, a.bound_chunk); });
            kt_floor_bound<TAB><<<dim3(gx, 1, n), kBlock, 0, st>>>(h[0], dt);
        }
        const int gx = max_over(h, [](const Lvl& a) { return cdiv(a.total, kBlock * kPoolItems); });
        {
            ProfScope ps(level_label("pool_count", h[0].B), st);
            kt_pool_count<TAB><<<dim3(gx, 1, n), kBlock, 0, st>>>(h[0], dt);
        }
        {
            ProfScope ps(level_label("pool_scatter", h[0].B), st);
            kt_pool_scatter<TAB><<<dim3(gx, 1, n), kBlock, 0, st>>>(h[0], dt);
        }
    }
    {
        ProfScope ps(level_label("pool_select", h[0].B), st);
        kt_floor_select<TAB><<<dim3(1, 1, n), 1024, 0, st>>>(h[0], dt, direct ? 1 : 0);
    }
    if (std::any_of(h.begin(), h.end(), [](const Lvl& a) { return a.pools_out != nullptr; })) {
        const int gx = max_over(h, [](const Lvl& a) { return std::min(cdiv(a.total, kBlock), 1024); });
        kt_copy_pool<TAB><<<dim3(gx, 1, n), kBlock, 0, st>>>(h[0], dt);
    }
}

template <bool TAB>
void launch_prep_step(const Lvl* dt, const std::vector<Lvl>& h, bool filtered, hipStream_t st) {
    switch (h[0].B) {
        case 2: launch_pool_prep<2, TAB>(dt, h, filtered, st); break;
        case 4: launch_pool_prep<4, TAB>(dt, h, filtered, st); break;
        case 8: launch_pool_prep<8, TAB>(dt, h, filtered, st); break;
        default: launch_pool_prep<16, TAB>(dt, h, filtered, st); break;
    }
}

template <bool TAB>
int launch_pool_phase_t(const Lvl* dt, const std::vector<Lvl>& h, const int64_t* T, bool filtered,
                        hipStream_t st, bool fill_act = false) {
    if (filtered) {
        launch_score_step<TAB>(dt, h, T, st, fill_act);
        launch_select_steps<TAB>(dt, h, st);
    }
    launch_prep_step<TAB>(dt, h, filtered, st);
    LAUNCH_CHECK();
    return FIC_OK;
}

template <bool TAB>
int launch_match_phase_t(const Lvl* dt, const std::vector<Lvl>& h, hipStream_t st) {
    switch (h[0].B) {
        case 2: launch_match<2, TAB>(dt, h, st); break;
        case 4: launch_match<4, TAB>(dt, h, st); break;
        case 8: launch_match<8, TAB>(dt, h, st); break;
        default: launch_match<16, TAB>(dt, h, st); break;
    }
    LAUNCH_CHECK();
    return FIC_OK;
}

int launch_pool_phase(const Lvl* dt, const std::vector<Lvl>& h, const int64_t* T, bool filtered,
                      hipStream_t st, bool fill_act = false) {
    return dt ? launch_pool_phase_t<true>(dt, h, T, filtered, st, fill_act)
              : launch_pool_phase_t<false>(dt, h, T, filtered, st, fill_act);
}

int launch_match_phase(const Lvl* dt, const std::vector<Lvl>& h, hipStream_t st) {
    return dt ? launch_match_phase_t<true>(dt, h, st) : launch_match_phase_t<false>(dt, h, st);
}

// Pool, moments and matcher of one level, in order on one stream.
int launch_level(const Lvl* dt, const std::vector<Lvl>& h, const int64_t* T, bool filtered,
                 hipStream_t st) {
    int rc = launch_pool_phase(dt, h, T, filtered, st);
    if (rc) return rc;
    return launch_match_phase(dt, h, st);
}

// Keep/split decisions and compaction for a quadtree level.
template <bool TAB>
int launch_quad_t(const Lvl* dt, const std::vector<Lvl>& h, hipStream_t st) {
    const int gr = max_over(h, [](const Lvl& a) { return cdiv(a.max_act, kRqRanges); });
    const int gx = max_over(h, [](const Lvl& a) { return cdiv(a.max_act, kBlock * kQuadItems); });
    {
        ProfScope ps(level_label("reduce_quad", h[0].B), st);
        kt_reduce_quad<TAB><<<dim3(gr, 1, h.size()), kBlock, 0, st>>>(h[0], dt);
    }
    {
        ProfScope ps(level_label("quad_compact", h[0].B), st);
        kt_quad_scatter<TAB><<<dim3(gx, 1, h.size()), kBlock, 0, st>>>(h[0], dt);
    }
    LAUNCH_CHECK();
    return FIC_OK;
}

int launch_quad(const Lvl* dt, const std::vector<Lvl>& h, hipStream_t st) {
    return dt ? launch_quad_t<true>(dt, h, st) : launch_quad_t<false>(dt, h, st);
}

int check_image(const uint8_t* img, int H, int W, int pitch, int B) {
    if (!img) return fail(FIC_EINVAL, "image pointer is NULL");
    if (!valid_B(B)) return fail(FIC_EINVAL, "range side %d not in {2,4,8,16}", B);
    if (H < 2 * B || W < 2 * B) return fail(FIC_EINVAL, "image %dx%d smaller than a domain (%d)", H, W, 2 * B);
    if (H > FIC_MAX_SIDE || W > FIC_MAX_SIDE) return fail(FIC_EINVAL, "image side above %d", FIC_MAX_SIDE);
    if (H % B || W % B) return fail(FIC_EINVAL, "image %dx%d not a multiple of %d", H, W, B);
    if (pitch < W) return fail(FIC_EINVAL, "pitch %d < width %d", pitch, W);
    return FIC_OK;
}

int check_params(const fic_params* p, std::vector<KSet>& ks) {
    if (!p) return fail(FIC_EINVAL, "params pointer is NULL");
    if (p->n_levels < 1 || p->n_levels > 4) return fail(FIC_EINVAL, "n_levels %d not in 1..4", p->n_levels);
    if (!valid_B(p->B0)) return fail(FIC_EINVAL, "B0 %d not in {2,4,8,16}", p->B0);
    if ((p->B0 >> (p->n_levels - 1)) < 2) return fail(FIC_EINVAL, "last level range side below 2");
    if (!(p->rms_thresh >= 0.0f) || !std::isfinite(p->rms_thresh))
        return fail(FIC_EINVAL, "rms_thresh must be finite and >= 0");
    if (p->entropy_mode < 0 || p->entropy_mode > 2) return fail(FIC_EINVAL, "entropy_mode %d not 0, 1 or 2", p->entropy_mode);
    if (p->entropy_mode != 0 && !std::isfinite(p->entropy_bits)) return fail(FIC_EINVAL, "entropy_bits not finite");
    if (p->min_pool < 1) return fail(FIC_EINVAL, "min_pool must be >= 1");
    ks.resize(p->n_levels);
    for (int l = 0; l < p->n_levels; ++l) {
        if (p->L[l] < 1) return fail(FIC_EINVAL, "L[%d] = %d < 1", l, p->L[l]);
        int rc = check_kset(p->s_k[l], p->n_s[l], &ks[l]);
        if (rc) return rc;
    }
    return FIC_OK;
}

// Per-level plans of one image's quadtree.
std::vector<Level> quad_levels(int H, int W, const fic_params* p, const std::vector<KSet>& ks,
                               const int* cg = nullptr, const int* var = nullptr) {
    std::vector<Level> lv;
    for (int l = 0; l < p->n_levels; ++l) {
        const int B = p->B0 >> l;
        lv.push_back(make_level(l, H, W, B, p->L[l], (H / B) * (W / B), ks[l], var ? var[l] : 0,
                                cg ? cg[l] : 0));
    }
    return lv;
}

// Argument tables of one image's quadtree (one entry per level).
std::vector<Lvl> quad_tables(Workspace& ws, const std::vector<Level>& lv, const uint8_t* img,
                             int H, int W, int pitch, const fic_params* p, fic_code* codes,
                             int capacity, fic_level_stats* stats, uint32_t* flags = nullptr,
                             int32_t* pools = nullptr) {
    std::vector<Lvl> t;
    int64_t pool_off = 0;
    for (size_t l = 0; l < lv.size(); ++l) {
        const Level& v = lv[l];
        int32_t* cur = P<int32_t>((l % 2) ? ws.act1 : ws.act0);
        int32_t* nxt = P<int32_t>((l % 2) ? ws.act0 : ws.act1);
        const int last = l + 1 == lv.size();
        t.push_back(make_lvl(ws, v, img, H, W, pitch, p->entropy_mode, p->entropy_bits, p->min_pool,
                             cur, nxt, last, keep_threshold(p->rms_thresh, v.B), codes, capacity,
                             stats));
        t.back().flags = last ? nullptr : flags;
        t.back().pools_out = (pools && p->entropy_mode != 0) ? pools + pool_off : nullptr;
        pool_off += v.total;
    }
    return t;
}

// Queue the whole quadtree of one image (tables at dt, host copies t).
// Images [start, start + count) of a batch table launch together; a batch sorted
// by size launches each size class with grids sized for it.
struct Group {
    int start, count;
};

// One image with its level arguments also on the device (fork->dlv): level
// 0's pool and matcher on the caller's stream; level 1's pool on a side
// stream of its own (its matcher comes next); the pools of levels 2.. on a
// second side stream, their selection steps shared by those levels (level =
// blockIdx.z). Fewer launches and events than a stream per level: the host
// queues the encode sooner.
int launch_quadtree_one(const std::vector<Lvl>& t, const int64_t* T, bool filtered, hipStream_t st,
                        Workspace& fork) {
    const int nl = (int)t.size();
    int rc;
    // Every level scored by the cell kernel: one launch scores them all (and
    // writes level 0's active list) before the streams fork.
    const bool all_cells =
        filtered && nl <= 4 && std::all_of(t.begin(), t.end(), [](const Lvl& a) { return score_by_cells(a); });
    // otherwise level 0's active list is written by its score kernel when that is the cell kernel
    const bool fill = filtered && !all_cells && score_by_cells(t[0]);
    if (all_cells) {
        int end[4];
        for (int l = 0; l < 4; ++l)
            end[l] = (l ? end[l - 1] : 0) + (l < nl ? cdiv(t[l].gx, sc_tx(t[l].L)) * cdiv(t[l].gy, kScTY) : 0);
        kt_pool_score_cells_levels<<<end[nl - 1], kBlock, 0, st>>>(fork.dlv, make_int4(end[0], end[1], end[2], end[3]),
                                                                   T);
    } else if (!fill) {
        const int gx = cdiv((t[0].H / t[0].B) * (t[0].W / t[0].B), kBlock);
        kt_act_full<false><<<gx, kBlock, 0, st>>>(t[0], nullptr, 1);
    }
    HIP_TRY(hipEventRecord(fork.ev_fork, st));
    const std::vector<Lvl> h0{t[0]};
    if (all_cells) {
        launch_select_steps<false>(nullptr, h0, st);
        launch_prep_step<false>(nullptr, h0, true, st);
        LAUNCH_CHECK();
    } else if ((rc = launch_pool_phase(nullptr, h0, T, filtered, st, fill))) {
        return rc;
    }
    if ((rc = launch_match_phase(nullptr, h0, st))) return rc;
    if ((rc = launch_quad(nullptr, h0, st))) return rc;
    // level 1
    hipStream_t p1 = fork.side[1];
    HIP_TRY(hipStreamWaitEvent(p1, fork.ev_fork, 0));
    const std::vector<Lvl> h1{t[1]};
    if (all_cells) {
        launch_select_steps<false>(nullptr, h1, p1);
        launch_prep_step<false>(nullptr, h1, true, p1);
        LAUNCH_CHECK();
    } else if ((rc = launch_pool_phase(nullptr, h1, T, filtered, p1))) {
        return rc;
    }
    HIP_TRY(hipEventRecord(fork.ev_pool[1], p1));
    // levels 2..
    if (nl > 2) {
        hipStream_t p2 = fork.side[2];
        HIP_TRY(hipStreamWaitEvent(p2, fork.ev_fork, 0));
        const std::vector<Lvl> rest(t.begin() + 2, t.end());
        if (filtered) {
            if (!all_cells)
                for (const Lvl& a : rest) launch_score_step<false>(nullptr, {a}, T, p2);
            launch_select_steps<true>(fork.dlv + 2, rest, p2);
        }
        for (const Lvl& a : rest) launch_prep_step<false>(nullptr, {a}, filtered, p2);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(fork.ev_pool[2], p2));
    }
    for (int l = 1; l < nl; ++l) {
        if (l <= 2) HIP_TRY(hipStreamWaitEvent(st, fork.ev_pool[l], 0));
        const std::vector<Lvl> h{t[l]};
        if ((rc = launch_match_phase(nullptr, h, st))) return rc;
        if ((rc = launch_quad(nullptr, h, st))) return rc;
    }
    return FIC_OK;
}

// The quadtree of n_images images whose level arguments are t ([level][image],
// also at dt when not NULL). With `fork` (one image, its level arguments
// uploaded to fork->dlv) the pools run on side streams (launch_quadtree_one);
// otherwise everything runs on st, level by level.
int launch_quadtree(const Lvl* dt, const std::vector<Lvl>& t, int n_images, const int64_t* T,
                    bool filtered, hipStream_t st, const std::vector<Group>* groups = nullptr,
                    Workspace* fork = nullptr) {
    const int nl = (int)t.size() / n_images;
    // (while profiling, everything stays on st, so that each kernel's event interval is its own)
    if (fork && dt == nullptr && n_images == 1 && nl > 1 && nl <= kLevels && fork->dlv &&
        fork->nlv == nl && !prof_active())
        return launch_quadtree_one(t, T, filtered, st, *fork);
    const std::vector<Group> all{{0, n_images}};
    const std::vector<Group>& gs = groups ? *groups : all;
    for (const Group& g : gs) {
        std::vector<Lvl> h0(t.begin() + g.start, t.begin() + g.start + g.count);
        const int gx = max_over(h0, [](const Lvl& a) { return cdiv((a.H / a.B) * (a.W / a.B), kBlock); });
        if (dt)
            kt_act_full<true><<<dim3(gx, 1, g.count), kBlock, 0, st>>>(h0[0], dt + g.start, 1);
        else
            kt_act_full<false><<<dim3(gx, 1, g.count), kBlock, 0, st>>>(h0[0], dt, 1);
    }
    for (int l = 0; l < nl; ++l) {
        // every group's pool, then every group's matcher and decisions
        for (int phase = 0; phase < 2; ++phase)
            for (const Group& g : gs) {
                std::vector<Lvl> h(t.begin() + l * n_images + g.start,
                                   t.begin() + l * n_images + g.start + g.count);
                const Lvl* dl = dt ? dt + l * n_images + g.start : nullptr;
                int rc = phase == 0 ? launch_pool_phase(dl, h, T, filtered, st)
                                    : launch_match_phase(dl, h, st);
                if (rc) return rc;
                if (phase == 1 && (rc = launch_quad(dl, h, st))) return rc;
            }
    }
    return FIC_OK;
}

// Quadtree encode of one image into `codes` (device); counters in ws.ctrl.
// Words of the split-flag bitmap: one bit per possible active range of every level but the last.
int64_t flag_words(int H, int W, const fic_params* p) {
    int64_t bits = 0;
    for (int l = 0; l + 1 < p->n_levels; ++l) {
        const int B = p->B0 >> l;
        bits += (int64_t)(H / B) * (W / B);
    }
    return (bits + 31) / 32;
}

int encode_image_impl(Workspace& ws, const uint8_t* img, int H, int W, int pitch,
                      const fic_params* p, const std::vector<KSet>& ks, fic_code* codes,
                      int capacity, fic_level_stats* stats, uint32_t* flags = nullptr,
                      int32_t* pools = nullptr, int32_t* n_out = nullptr) {
    std::vector<Level> lv = quad_levels(H, W, p, ks);
    Sizes sz;
    for (const Level& v : lv) grow(sz, v);
    int rc = ensure_sizes(ws, sz);
    if (rc) return rc;
    if (flags) {
        const int64_t nw = flag_words(H, W, p);
        if (nw > 0)
            k_fill_i32<<<cdiv(nw, kBlock), kBlock, 0, ws.stream>>>(reinterpret_cast<int32_t*>(flags), (int)nw, 0);
    }
    std::vector<Lvl> t = quad_tables(ws, lv, img, H, W, pitch, p, codes, capacity, stats, flags, pools);
    t.back().n_out = n_out;
    if ((rc = ensure_fork(ws))) return rc;
    if ((rc = upload_levels(ws, t))) return rc;
    return launch_quadtree(nullptr, t, 1, ws.T, p->entropy_mode != 0, ws.stream, nullptr, &ws);
}

}  // namespace
}  // namespace fic

using namespace fic;

FIC_API int fic_version(void) { return 100; }

FIC_API const char* fic_last_error(void) { return g_err.c_str(); }

namespace fic {
namespace {

// Host checks of one level's arguments (fic_encode_level_ex); *ks and *var
// receive the contrast set and the matcher.
int check_level(const uint8_t* img, int H, int W, int pitch, int B, int L, const int8_t* s_k, int n_s,
                int entropy_mode, float entropy_bits, int min_pool, const int32_t* range_yx, int n_ranges,
                const fic_match* out, int variant, KSet* ks, int* var) {
    int rc = check_image(img, H, W, pitch, B);
    if (rc) return rc;
    if (L < 1) return fail(FIC_EINVAL, "domain step L=%d < 1", L);
    if ((rc = check_kset(s_k, n_s, ks))) return rc;
    if (entropy_mode < 0 || entropy_mode > 2) return fail(FIC_EINVAL, "entropy_mode %d not 0, 1 or 2", entropy_mode);
    if (entropy_mode != 0 && !std::isfinite(entropy_bits)) return fail(FIC_EINVAL, "entropy_bits not finite");
    if (min_pool < 1) return fail(FIC_EINVAL, "min_pool must be >= 1");
    if (n_ranges < 0) return fail(FIC_EINVAL, "n_ranges < 0");
    if (!range_yx && n_ranges != (H / B) * (W / B))
        return fail(FIC_EINVAL, "range_yx is NULL but n_ranges %d != %d", n_ranges, (H / B) * (W / B));
    if (n_ranges > 0 && !out) return fail(FIC_EINVAL, "out is NULL");
    if (variant < FIC_MATCH_AUTO || variant > FIC_MATCH_MFMA_F16)
        return fail(FIC_EINVAL, "matcher variant %d unknown", variant);
    const int64_t grid_total = (int64_t)((H - 2 * B) / L + 1) * ((W - 2 * B) / L + 1);
    // FP16 MFMA: the grid form (B = 8, 0..k1) or the small-set form (B = 4, 8, 16)
    const bool f16_small = variant == FIC_MATCH_MFMA_F16 && !mfma_eligible(B, *ks) && mfq_eligible(B, *ks);
    const bool mf = variant == FIC_MATCH_MFMA_I8 || (variant == FIC_MATCH_MFMA_F16 && !f16_small);
    if ((mf || variant == FIC_MATCH_FP32) && !mfma_eligible(B, *ks))
        return fail(FIC_EINVAL,
                    variant == FIC_MATCH_MFMA_F16
                        ? "matcher variant %d needs B = 8 and contrast set 0..k1 (k1 >= 2), or B = 4, 8 or 16 "
                          "and one or two values, one of them nonzero"
                        : "matcher variant %d needs B = 8 and contrast set 0..k1 (k1 >= 2)",
                    variant);
    if (mf && !mfma_eligible(B, *ks, grid_total))
        return fail(FIC_EINVAL, "the MFMA matchers take domain grids below %d domains", kM8MaxPool);
    if (f16_small && !mfq_eligible(B, *ks, grid_total))
        return fail(FIC_EINVAL, "the small-set MFMA matcher takes domain grids below %d domains", kMqMaxPool);
    *var = variant == FIC_MATCH_VALU ? kVarValu
           : variant == FIC_MATCH_MFMA_I8 ? kVarMfma
           : variant == FIC_MATCH_MFMA_F16 ? (f16_small ? kVarMfq : kVarMfma16)
           : variant == FIC_MATCH_FP32 ? kVarFp32 : 0;
    return FIC_OK;
}

// Queue one level's search on ws.stream; every buffer of plan v is in place.
int encode_level_run(Workspace& ws, const Level& v, const uint8_t* img, int H, int W, int pitch,
                     int entropy_mode, float entropy_bits, int min_pool, const int32_t* range_yx,
                     int n_ranges, fic_match* out, int32_t* pool_out, int32_t* pool_count) {
    int rc;
    hipStream_t st = ws.stream;
    int32_t* act = P<int32_t>(ws.act0);
    std::vector<Lvl> t{make_lvl(ws, v, img, H, W, pitch, entropy_mode, entropy_bits, min_pool, act,
                                P<int32_t>(ws.act1), 1, 0, nullptr, 0, nullptr)};
    const Lvl* dt = nullptr;  // one image: arguments by value
    const std::vector<Lvl>& h = t;
    if (range_yx)
        kt_act_from_yx<false><<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(h[0], dt, range_yx, n_ranges);
    else
        kt_act_full<false><<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(h[0], dt, 0);
    if ((rc = launch_level(dt, t, ws.T, entropy_mode != 0, st))) return rc;
    {
        ProfScope ps("reduce_level", st);
        if (v.var == kVarFp32)
            kt_reduce_fp32<false><<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(h[0], dt, out);
        else
            kt_reduce_level<false><<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(h[0], dt, out);
    }
    LAUNCH_CHECK();
    if (pool_count)
        HIP_TRY(hipMemcpyAsync(pool_count, &(ws.ctrl + 1)->pool_count, sizeof(int32_t),
                               hipMemcpyDeviceToDevice, st));
    if (pool_out) {
        if (entropy_mode != 0)
            HIP_TRY(hipMemcpyAsync(pool_out, ws.pl[0].pool.p, sizeof(int32_t) * v.total,
                                   hipMemcpyDeviceToDevice, st));
        else
            HIP_TRY(hipMemcpyAsync(pool_out, ws.pl[0].jd.p, sizeof(int32_t) * v.total,
                                   hipMemcpyDeviceToDevice, st));
    }
    return FIC_OK;
}

}  // namespace
}  // namespace fic

FIC_API int fic_encode_level_ex(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t B,
                                int32_t L, const int8_t* s_k, int32_t n_s, int32_t entropy_mode,
                                float entropy_bits, int32_t min_pool, const int32_t* range_yx,
                                int32_t n_ranges, fic_match* out, int32_t* pool_out,
                                int32_t* pool_count, int32_t variant, void* stream) {
    KSet ks;
    int var = 0;
    int rc = check_level(img, H, W, pitch, B, L, s_k, n_s, entropy_mode, entropy_bits, min_pool,
                         range_yx, n_ranges, out, variant, &ks, &var);
    if (rc) return rc;
    if (n_ranges == 0) return FIC_OK;
    Workspace* ws;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    Level v = make_level(0, H, W, B, L, n_ranges, ks, var);
    Sizes sz;
    grow(sz, v);
    if ((rc = ensure_sizes(*ws, sz))) return rc;
    return encode_level_run(*ws, v, img, H, W, pitch, entropy_mode, entropy_bits, min_pool, range_yx,
                            n_ranges, out, pool_out, pool_count);
}

FIC_API int fic_encode_level(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t B,
                             int32_t L, const int8_t* s_k, int32_t n_s, int32_t entropy_mode,
                             float entropy_bits, int32_t min_pool, const int32_t* range_yx,
                             int32_t n_ranges, fic_match* out, int32_t* pool_out,
                             int32_t* pool_count, void* stream) {
    return fic_encode_level_ex(img, H, W, pitch, B, L, s_k, n_s, entropy_mode, entropy_bits,
                               min_pool, range_yx, n_ranges, out, pool_out, pool_count,
                               FIC_MATCH_AUTO, stream);
}

// ---------------------------------------------------------------- fixed scratch
// The workspace of fic_encode_level_noalloc: one array in each device's
// memory for the life of the process. In host code its name is a host-side
// stand-in, not a device address: the address comes from hipGetSymbolAddress,
// once per device, and only that address is ever handed to kernels or copies.
// Layout: the control blocks, the entropy table, then the level's buffers.
static __device__ __align__(256) uint8_t scratch[FIC_NOALLOC_SCRATCH_BYTES];

namespace fic {
namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kScratchCtrl = ((sizeof(Ctrl) * (1 + kLevels)) + 255) & ~(size_t)255;
constexpr size_t kScratchHead = kScratchCtrl + (((kMaxWindow + 1) * sizeof(int64_t) + 255) & ~(size_t)255);

std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// This device's scratch address; the first call on a device resolves it and
// uploads the entropy table (a synchronous copy).
int scratch_address(int dev, uint8_t** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FIC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        const std::vector<int64_t>& t = entropy_table();
        HIP_TRY(hipMemcpy(static_cast<uint8_t*>(ptr) + kScratchCtrl, t.data(), sizeof(int64_t) * t.size(),
                          hipMemcpyHostToDevice));
        g_scratch[dev] = static_cast<uint8_t*>(ptr);
    }
    *out = g_scratch[dev];
    return FIC_OK;
}

// Place every buffer of sz in the scratch after its head; *need receives the
// bytes the plan takes in all.
int carve_sizes(Workspace& ws, uint8_t* base, const Sizes& sz, size_t* need) {
    size_t off = kScratchHead;
    const int rc = visit_sizes(ws, sz, [&](Buf& b, size_t bytes) {
        if (bytes == 0) bytes = 1;
        if (b.p && b.cap >= bytes) return FIC_OK;
        const size_t want = (bytes + 255) & ~(size_t)255;
        b.p = base ? base + off : nullptr;
        b.cap = want;
        off += want;
        return FIC_OK;
    });
    *need = off;
    return rc;
}

struct NoProfile {
    NoProfile() { g_prof_off = true; }
    ~NoProfile() { g_prof_off = false; }
};

}  // namespace
}  // namespace fic

FIC_API int fic_encode_level_noalloc(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t B,
                                     int32_t L, const int8_t* s_k, int32_t n_s, int32_t entropy_mode,
                                     float entropy_bits, int32_t min_pool, const int32_t* range_yx,
                                     int32_t n_ranges, fic_match* out, int32_t* pool_out,
                                     int32_t* pool_count, void* stream) {
    KSet ks;
    int var = 0;
    int rc = check_level(img, H, W, pitch, B, L, s_k, n_s, entropy_mode, entropy_bits, min_pool,
                         range_yx, n_ranges, out, FIC_MATCH_AUTO, &ks, &var);
    if (rc) return rc;
    if (n_ranges == 0) return FIC_OK;
    const Level v = make_level(0, H, W, B, L, n_ranges, ks, var);
    Sizes sz;
    grow(sz, v);
    {
        Workspace probe;
        size_t need = 0;
        carve_sizes(probe, nullptr, sz, &need);
        if (need > (size_t)FIC_NOALLOC_SCRATCH_BYTES)
            return fail(FIC_EINVAL,
                        "this level needs %zu bytes of device scratch; fic_encode_level_noalloc holds %zu "
                        "(use fic_encode_level)",
                        need, (size_t)FIC_NOALLOC_SCRATCH_BYTES);
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FIC_EINVAL, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    uint8_t* base = nullptr;
    if ((rc = scratch_address(dev, &base))) return rc;
    Workspace ws;  // every buffer in the scratch; nothing here is freed
    ws.device = dev;
    ws.stream = (hipStream_t)stream;
    ws.ctrl = reinterpret_cast<Ctrl*>(base);
    ws.T = reinterpret_cast<int64_t*>(base + kScratchCtrl);
    size_t need = 0;
    carve_sizes(ws, base, sz, &need);
    NoProfile np;
    {
        const int words = (int)(sizeof(Ctrl) / 4) * (1 + kLevels);
        k_ctrl_reset<<<cdiv(words, kBlock), kBlock, 0, ws.stream>>>(ws.ctrl, 1 + kLevels);
    }
    LAUNCH_CHECK();
    return encode_level_run(ws, v, img, H, W, pitch, entropy_mode, entropy_bits, min_pool, range_yx,
                            n_ranges, out, pool_out, pool_count);
}

FIC_API int fic_encode_image(const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                             const fic_params* p, fic_code* codes, int32_t capacity,
                             int32_t* n_codes, fic_level_stats* stats, void* stream) {
    std::vector<KSet> ks;
    int rc = check_params(p, ks);
    if (rc) return rc;
    if ((rc = check_image(img, H, W, pitch, p->B0))) return rc;
    if (!codes || !n_codes) return fail(FIC_EINVAL, "codes or n_codes is NULL");
    const int lower = (H / p->B0) * (W / p->B0);
    if (capacity < lower)
        return fail(FIC_ECAPACITY, "capacity %d below the %d codes of the first level", capacity, lower);
    Workspace* ws;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    return encode_image_impl(*ws, img, H, W, pitch, p, ks, codes, capacity, stats, nullptr, nullptr,
                             n_codes);
}

FIC_API int fic_encode_image_ex(const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                                const fic_params* p, fic_code* codes, int32_t capacity,
                                int32_t* n_codes, fic_level_stats* stats, uint32_t* flags,
                                int32_t* pools, void* stream) {
    std::vector<KSet> ks;
    int rc = check_params(p, ks);
    if (rc) return rc;
    if ((rc = check_image(img, H, W, pitch, p->B0))) return rc;
    if (!codes || !n_codes) return fail(FIC_EINVAL, "codes or n_codes is NULL");
    const int lower = (H / p->B0) * (W / p->B0);
    if (capacity < lower)
        return fail(FIC_ECAPACITY, "capacity %d below the %d codes of the first level", capacity, lower);
    Workspace* ws;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    return encode_image_impl(*ws, img, H, W, pitch, p, ks, codes, capacity, stats, flags, pools,
                             n_codes);
}

FIC_API int fic_decode(const fic_code* codes, int32_t n_codes, int32_t H, int32_t W, int32_t iters,
                       uint8_t* out, int32_t out_pitch, void* stream) {
    if (!out) return fail(FIC_EINVAL, "out is NULL");
    if (H < 1 || W < 1 || H > FIC_MAX_SIDE || W > FIC_MAX_SIDE) return fail(FIC_EINVAL, "bad image size");
    if (out_pitch < W) return fail(FIC_EINVAL, "out_pitch < W");
    if (iters < 0) return fail(FIC_EINVAL, "iters < 0");
    if (n_codes < 1 || !codes) return fail(FIC_EINVAL, "no codes");
    Workspace* ws;
    int rc;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    const int npx = H * W;
    if ((rc = ensure(*ws, ws->map, (size_t)npx * 4))) return rc;
    if ((rc = ensure(*ws, ws->imgA, (size_t)npx))) return rc;
    if ((rc = ensure(*ws, ws->imgB, (size_t)npx))) return rc;
    if ((rc = ensure(*ws, ws->acc, 64))) return rc;
    hipStream_t st = ws->stream;
    int* err = P<int>(ws->acc);
    k_fill_i32<<<1, 64, 0, st>>>(err, 1, 0);
    k_fill_i32<<<cdiv(npx, kBlock), kBlock, 0, st>>>(P<int32_t>(ws->map), npx, -1);
    k_decode_map<<<cdiv(n_codes, kBlock), kBlock, 0, st>>>(codes, n_codes, H, W, P<int32_t>(ws->map), err);
    k_check_map<<<cdiv(npx, kBlock), kBlock, 0, st>>>(P<int32_t>(ws->map), npx, err);
    LAUNCH_CHECK();
    int herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (herr) return fail(FIC_EINVAL, "codes do not tile the image or leave it (flags %d)", herr);
    uint8_t* a = P<uint8_t>(ws->imgA);
    uint8_t* b = P<uint8_t>(ws->imgB);
    k_fill_u8<<<cdiv(npx, kBlock), kBlock, 0, st>>>(iters == 0 ? out : a, H, W, iters == 0 ? out_pitch : W, 128);
    for (int it = 0; it < iters; ++it) {
        const bool lastit = it == iters - 1;
        uint8_t* dst = lastit ? out : b;
        ProfScope ps("decode_iter", st);
        k_decode_iter<<<cdiv(npx, kBlock), kBlock, 0, st>>>(codes, P<int32_t>(ws->map), a, W, dst,
                                                           lastit ? out_pitch : W, H, W);
        std::swap(a, b);
    }
    LAUNCH_CHECK();
    HIP_TRY(hipStreamSynchronize(st));
    return FIC_OK;
}

FIC_API int fic_sse(const uint8_t* a, int32_t pitch_a, const uint8_t* b, int32_t pitch_b, int32_t H,
                    int32_t W, uint64_t* sse, void* stream) {
    if (!a || !b || !sse) return fail(FIC_EINVAL, "NULL pointer");
    if (H < 1 || W < 1 || pitch_a < W || pitch_b < W) return fail(FIC_EINVAL, "bad shape");
    hipStream_t st = (hipStream_t)stream;
    k_fill_i32<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(sse), 2, 0);
    int blocks = std::min(cdiv((int64_t)H * W, kBlock), 1024);
    k_sse<<<blocks, kBlock, 0, st>>>(a, pitch_a, b, pitch_b, H, W,
                                     reinterpret_cast<unsigned long long*>(sse));
    LAUNCH_CHECK();
    return FIC_OK;
}

FIC_API int fic_calibrate_s(const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                            const fic_params* p, int8_t* k_out, void* stream) {
    if (!k_out) return fail(FIC_EINVAL, "k_out is NULL");
    fic_params q;
    if (!p) return fail(FIC_EINVAL, "params pointer is NULL");
    q = *p;
    q.entropy_mode = 0;
    for (int l = 0; l < 4; ++l) {
        q.n_s[l] = 11;
        for (int k = 0; k <= 10; ++k) q.s_k[l][k] = (int8_t)k;
    }
    std::vector<KSet> ks;
    int rc = check_params(&q, ks);
    if (rc) return rc;
    if (!std::isfinite(p->entropy_bits)) return fail(FIC_EINVAL, "entropy_bits not finite");
    if ((rc = check_image(img, H, W, pitch, q.B0))) return rc;
    Workspace* ws;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    const int Blast = q.B0 >> (q.n_levels - 1);
    const int capacity = (H / Blast) * (W / Blast);
    if ((rc = ensure(*ws, ws->codes, (size_t)capacity * sizeof(fic_code)))) return rc;
    if ((rc = ensure(*ws, ws->acc, 64))) return rc;
    if ((rc = ensure(*ws, ws->mr, 64))) return rc;
    if ((rc = encode_image_impl(*ws, img, H, W, pitch, &q, ks, P<fic_code>(ws->codes), capacity, nullptr)))
        return rc;
    hipStream_t st = ws->stream;
    int64_t mr[4] = {0, 0, 0, 0};
    for (int l = 0; l < q.n_levels; ++l) {
        int B = q.B0 >> l;
        mr[l] = entropy_cut(B * B, (double)p->entropy_bits);
    }
    HIP_TRY(hipMemcpyAsync(ws->mr.p, mr, sizeof mr, hipMemcpyHostToDevice, st));
    k_fill_i32<<<1, 64, 0, st>>>(P<int32_t>(ws->acc), 16, 0);
    k_calib_accum<<<cdiv(capacity, kBlock), kBlock, 0, st>>>(
        img, pitch, P<fic_code>(ws->codes), ws->ctrl, capacity, ws->T, P<int64_t>(ws->mr),
        P<unsigned long long>(ws->acc));
    LAUNCH_CHECK();
    unsigned long long acc[8];
    HIP_TRY(hipMemcpyAsync(acc, ws->acc.p, sizeof acc, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int l = 0; l < q.n_levels; ++l) {
        unsigned long long tot = acc[2 * l], cnt = acc[2 * l + 1];
        k_out[l] = cnt ? (int8_t)((2 * tot + cnt) / (2 * cnt)) : (int8_t)-1;
    }
    return FIC_OK;
}

FIC_API int fic_s_histogram(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, const fic_params* p,
                            int32_t low_entropy_only, uint64_t* hist, void* stream) {
    if (!hist) return fail(FIC_EINVAL, "hist is NULL");
    if (!p) return fail(FIC_EINVAL, "params pointer is NULL");
    fic_params q = *p;
    q.entropy_mode = 0;
    for (int l = 0; l < 4; ++l) {
        q.n_s[l] = 11;
        for (int k = 0; k <= 10; ++k) q.s_k[l][k] = (int8_t)k;
    }
    std::vector<KSet> ks;
    int rc = check_params(&q, ks);
    if (rc) return rc;
    if (low_entropy_only && !std::isfinite(p->entropy_bits)) return fail(FIC_EINVAL, "entropy_bits not finite");
    if ((rc = check_image(img, H, W, pitch, q.B0))) return rc;
    Workspace* ws;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    const int Blast = q.B0 >> (q.n_levels - 1);
    const int capacity = (H / Blast) * (W / Blast);
    if ((rc = ensure(*ws, ws->codes, (size_t)capacity * sizeof(fic_code)))) return rc;
    if ((rc = ensure(*ws, ws->mr, 64))) return rc;
    if ((rc = encode_image_impl(*ws, img, H, W, pitch, &q, ks, P<fic_code>(ws->codes), capacity, nullptr)))
        return rc;
    hipStream_t st = ws->stream;
    int64_t mr[4] = {0, 0, 0, 0};
    for (int l = 0; l < q.n_levels; ++l) {
        const int B = q.B0 >> l;
        mr[l] = low_entropy_only ? entropy_cut(B * B, (double)p->entropy_bits) : 0;
    }
    HIP_TRY(hipMemcpyAsync(ws->mr.p, mr, sizeof mr, hipMemcpyHostToDevice, st));
    k_calib_hist<<<cdiv(capacity, kBlock), kBlock, 0, st>>>(img, pitch, P<fic_code>(ws->codes), ws->ctrl,
                                                          capacity, ws->T, P<int64_t>(ws->mr),
                                                          low_entropy_only ? 1 : 0,
                                                          reinterpret_cast<unsigned long long*>(hist));
    LAUNCH_CHECK();
    HIP_TRY(hipStreamSynchronize(st));  // the host copy of mr must outlive the upload
    return FIC_OK;
}

FIC_API int fic_select_s(const uint64_t* hist, int32_t n_levels, float second_frac, int8_t* s_k,
                         int32_t* n_s) {
    if (!hist || !s_k || !n_s) return fail(FIC_EINVAL, "NULL argument");
    if (n_levels < 1 || n_levels > 4) return fail(FIC_EINVAL, "n_levels %d not in 1..4", n_levels);
    if (!(second_frac >= 0.0f) || !(second_frac <= 1.0f)) return fail(FIC_EINVAL, "second_frac not in [0, 1]");
    for (int l = 0; l < n_levels; ++l) {
        const uint64_t* h = hist + 11 * l;
        int a = -1, b = -1;  // most and second most frequent k (ties to the smaller k)
        for (int k = 0; k <= 10; ++k) {
            if (h[k] == 0) continue;
            if (a < 0 || h[k] > h[a]) {
                b = a;
                a = k;
            } else if (b < 0 || h[k] > h[b]) {
                b = k;
            }
        }
        n_s[l] = 0;
        if (a < 0) continue;
        const bool two = b >= 0 && (double)h[b] >= (double)second_frac * (double)h[a];
        s_k[2 * l] = (int8_t)(two ? std::min(a, b) : a);
        s_k[2 * l + 1] = (int8_t)(two ? std::max(a, b) : 0);
        n_s[l] = two ? 2 : 1;
    }
    return FIC_OK;
}

FIC_API int fic_peak_probe(int32_t what, void* stream, double* rate) {
    if (!rate) return fail(FIC_EINVAL, "rate is NULL");
    if (what < FIC_PEAK_VALU_FMA || what > FIC_PEAK_HBM_COPY) return fail(FIC_EINVAL, "probe %d unknown", what);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    void* out = nullptr;
    void* src = nullptr;
    void* dst = nullptr;
    const size_t copy_bytes = (size_t)1 << 30;
    if (hipMalloc(&out, 256) != hipSuccess) return fail(FIC_ENOMEM, "hipMalloc failed");
    if (what == FIC_PEAK_HBM_COPY) {
        if (hipMalloc(&src, copy_bytes) != hipSuccess || hipMalloc(&dst, copy_bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (src) (void)hipFree(src);
            (void)hipFree(out);
            return fail(FIC_ENOMEM, "hipMalloc of the copy buffers failed");
        }
    }
    const int grid = cus * 8;
    auto launch = [&]() {
        switch (what) {
            case FIC_PEAK_VALU_FMA: k_peak_fma<<<grid, 256, 0, st>>>(1.0f, static_cast<float*>(out)); break;
            case FIC_PEAK_DOT2: k_peak_dot2<<<grid, 256, 0, st>>>(3, static_cast<int*>(out)); break;
            case FIC_PEAK_MFMA_F16: k_peak_mfma_f16<<<grid, 256, 0, st>>>(0.5f, static_cast<float*>(out)); break;
            case FIC_PEAK_MFMA_I8: k_peak_mfma_i8<<<grid, 256, 0, st>>>(3, static_cast<int*>(out)); break;
            default:
                k_peak_copy<<<cus * 16, 256, 0, st>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst),
                                                      copy_bytes / 16);
        }
    };
    const double lanes = (double)grid * 256, waves = (double)grid * 4;
    const double work = what == FIC_PEAK_VALU_FMA ? lanes * 8 * kPeakIters * 2
                        : what == FIC_PEAK_DOT2 ? lanes * 8 * kPeakIters * 4
                        : what == FIC_PEAK_MFMA_F16 ? waves * kPeakIters * (2.0 * 16 * 16 * 32)
                        : what == FIC_PEAK_MFMA_I8 ? waves * kPeakIters * (2.0 * 16 * 16 * 64)
                                                   : 2.0 * (double)copy_bytes;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int reps = 5;
    if (e == hipSuccess) {
        launch();  // warm-up
        launch();
        e = hipEventRecord(e0, st);
    }
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (e != hipSuccess) return fail(FIC_EDEVICE, "peak probe: %s", hipGetErrorString(e));
    *rate = work * reps / (ms * 1e-3);
    return FIC_OK;
}

FIC_API int fic_profile_begin(void) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (auto& r : g_prof.recs) {
        g_prof.spare.push_back(r.a);
        g_prof.spare.push_back(r.b);
    }
    g_prof.recs.clear();
    g_prof.on = true;
    return FIC_OK;
}

FIC_API int fic_profile_end(fic_kernel_time* out, int32_t max, int32_t* n_out) {
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        g_prof.on = false;
        recs.swap(g_prof.recs);
    }
    std::vector<fic_kernel_time> agg;
    int rc = FIC_OK;
    for (auto& r : recs) {
        if (rc == FIC_OK) {
            hipError_t e = hipEventSynchronize(r.b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess) {
                rc = fail(FIC_EDEVICE, "profiling event: %s", hipGetErrorString(e));
            } else {
                fic_kernel_time* t = nullptr;
                for (auto& x : agg)
                    if (std::strncmp(x.name, r.name, sizeof x.name) == 0) t = &x;
                if (!t) {
                    fic_kernel_time z;
                    std::memset(&z, 0, sizeof z);
                    std::strncpy(z.name, r.name, sizeof z.name - 1);
                    agg.push_back(z);
                    t = &agg.back();
                }
                t->launches += 1;
                t->total_ms += ms;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        for (auto& r : recs) {
            g_prof.spare.push_back(r.a);
            g_prof.spare.push_back(r.b);
        }
    }
    if (rc) return rc;
    std::sort(agg.begin(), agg.end(),
              [](const fic_kernel_time& x, const fic_kernel_time& y) { return x.total_ms > y.total_ms; });
    if (n_out) *n_out = (int32_t)agg.size();
    if (out)
        for (int i = 0; i < (int)agg.size() && i < max; ++i) out[i] = agg[i];
    return FIC_OK;
}

// ================================================================ batched quadtree
// n images, each with its own workspace; every level of every image runs in
// the same launches (image = blockIdx.z), captured once into a hipGraph.
namespace fic {
namespace {

// n_codes of table entry i (an image in size order) goes to the caller's slot orig[i]
__global__ void kt_copy_counts(const Lvl* __restrict__ tab, int n, const int32_t* __restrict__ orig,
                               int32_t* __restrict__ n_codes) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) n_codes[orig[i]] = tab[i].ctrl->n_codes;
}

struct BatchImage {
    const uint8_t* img;
    int H, W, pitch;
    int64_t code_off;
    int capacity;
    Workspace* ws;
    int orig;  // index in the caller's arrays
};

}  // namespace
}  // namespace fic

struct fic_batch {
    int device = 0;
    hipStream_t st = nullptr;
    fic_params p;
    std::vector<fic::KSet> ks;
    std::vector<fic::BatchImage> im;
    fic_code* codes = nullptr;
    int32_t* n_codes = nullptr;
    fic_level_stats* stats = nullptr;
    std::vector<int> cg;  // per level; 0 = default
    std::vector<fic::Lvl> htab;  // host copy of the [level][image] argument table
    std::vector<fic::Group> groups;  // runs of images of equal size (images sorted by size)
    int32_t* dorig = nullptr;        // device: caller index of each image
    void* dtab = nullptr;
    size_t dtab_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t matches_hint = 0;
    // persistent form
    int form = FIC_BATCH_LEVELS;
    std::vector<int> tiles;  // per level: ranges per tile (0 = default)
    int wgs = 0;             // resident workgroups (0 = every one that fits)
    void* pq_mem = nullptr;
    size_t pq_bytes = 0;
    fic::PqArgs pa{};
    int32_t* blk_seg = nullptr;
    int32_t* blk_z0 = nullptr;
    int32_t* blk_first = nullptr;
    int32_t* blko = nullptr;
    int2* blkc = nullptr;
    int n_blk = 0;
    int pq_grid = 0;
};

namespace fic {
namespace {

// ---------------------------------------------------------------- persistent form
// Matcher of a level inside the persistent kernel.
int pq_kind(int var, const KSet& ks) {
    if (var == kVarMfq) return nonzero_values(ks) > 1 ? kPqMfq2 : kPqMfq1;
    const int mode = match_mode(ks);
    return mode == kModeSmall ? kPqValuSmall : (mode == kModeGrid ? kPqValuGrid : kPqValuList);
}

// Ranges per tile a level takes by default: one matcher call at level 0 (so
// that a single image's first level spreads over many workgroups), about 64
// below it.
int pq_default_tile(int B, int kind, int l) {
    const int per = pq_block_ranges(B, kind);
    return l == 0 ? per : per * std::max(1, 64 / per);
}

int pq_tile(const fic_batch* b, int l, int kind) {
    const int B = b->p.B0 >> l;
    return (b->tiles.size() > (size_t)l && b->tiles[l] > 0) ? b->tiles[l] : pq_default_tile(B, kind, l);
}

// Sizes, tile and slot tables, the device buffers (zeroed once: every queue
// word then carries an old epoch) and the launch shape of the persistent form.
int pq_build(fic_batch* b, const std::vector<int>& var) {
    const int n = (int)b->im.size(), nl = b->p.n_levels;
    PqArgs pa{};
    pa.n_img = n;
    pa.n_levels = nl;
    pa.B0 = b->p.B0;
    for (int l = 0; l < nl; ++l) {
        pa.kind[l] = pq_kind(var[l], b->ks[l]);
        pa.R[l] = pq_tile(b, l, pa.kind[l]);
        const int per = pq_block_ranges(b->p.B0 >> l, pa.kind[l]);
        if (pa.R[l] % per != 0 || pa.R[l] > kPqMaxTile)
            return fail(FIC_EINVAL, "level %d: %d ranges per tile is not a multiple of %d up to %d", l, pa.R[l],
                        per, kPqMaxTile);
    }
    std::vector<int32_t> tile_base((size_t)nl * n), blk_first((size_t)nl * n + 1);
    std::vector<int64_t> slot_base((size_t)nl * n);
    std::vector<int32_t> blk_seg, blk_z0;
    int64_t tiles = 0, slots = 0;
    for (int l = 0; l < nl; ++l) {
        if (l == 1) pa.T0 = (int32_t)tiles;
        for (int i = 0; i < n; ++i) {
            const int B = b->p.B0 >> l;
            const int64_t N = (int64_t)(b->im[i].H / B) * (b->im[i].W / B);
            const size_t seg = (size_t)l * n + i;
            tile_base[seg] = (int32_t)tiles;
            slot_base[seg] = slots;
            blk_first[seg] = (int32_t)blk_seg.size();
            tiles += (N + pa.R[l] - 1) / pa.R[l];
            slots += N;
            for (int64_t z = 0; z < N; z += kPqEmitSlots) {
                blk_seg.push_back((int32_t)seg);
                blk_z0.push_back((int32_t)z);
            }
        }
    }
    if (nl == 1) pa.T0 = (int32_t)tiles;
    blk_first[(size_t)nl * n] = (int32_t)blk_seg.size();
    if (tiles >= INT32_MAX || blk_seg.size() >= (size_t)INT32_MAX)
        return fail(FIC_EINVAL, "batch too large for the persistent form");
    pa.T = (int32_t)tiles;
    // launch shape: every workgroup that fits, or the caller's count
    int dev_cus = 0, per_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, b->device));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kt_pq, kBlock, 0));
    const int fit = std::max(1, dev_cus * std::max(1, per_cu));
    b->pq_grid = b->wgs > 0 ? std::min(b->wgs, fit) : fit;
    pa.gq_cap = (int32_t)(tiles - pa.T0) + b->pq_grid + 1;
    // one allocation, carved
    const size_t nb = blk_seg.size();
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_ctl = take(sizeof(PqCtl)), o_tb = take(4 * tile_base.size()), o_sb = take(8 * slot_base.size());
    const size_t o_rec = take(sizeof(PqRec) * slots), o_st = take(slots), o_qe = take(8 * slots);
    const size_t o_fill = take(4 * (size_t)tiles), o_gq = take(8 * (size_t)pa.gq_cap);
    const size_t o_enq = take(16 * (size_t)n), o_rem = take(16 * (size_t)n);
    const size_t o_bs = take(4 * nb), o_bz = take(4 * nb), o_bf = take(4 * blk_first.size());
    const size_t o_bc = take(8 * nb), o_bo = take(4 * nb);
    if (b->pq_bytes < off) {
        if (b->pq_mem) (void)hipFree(b->pq_mem);
        b->pq_mem = nullptr;
        b->pq_bytes = 0;
        if (hipMalloc(&b->pq_mem, off) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FIC_ENOMEM, "hipMalloc(%zu) for the persistent form failed", off);
        }
        b->pq_bytes = off;
    }
    uint8_t* m = static_cast<uint8_t*>(b->pq_mem);
    HIP_TRY(hipMemset(m, 0, off));
    HIP_TRY(hipMemcpy(m + o_tb, tile_base.data(), 4 * tile_base.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m + o_sb, slot_base.data(), 8 * slot_base.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m + o_bs, blk_seg.data(), 4 * nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m + o_bz, blk_z0.data(), 4 * nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m + o_bf, blk_first.data(), 4 * blk_first.size(), hipMemcpyHostToDevice));
    pa.ctl = reinterpret_cast<PqCtl*>(m + o_ctl);
    pa.tile_base = reinterpret_cast<const int32_t*>(m + o_tb);
    pa.slot_base = reinterpret_cast<const int64_t*>(m + o_sb);
    pa.rec = reinterpret_cast<PqRec*>(m + o_rec);
    pa.state = m + o_st;
    pa.qe = reinterpret_cast<uint64_t*>(m + o_qe);
    pa.fill = reinterpret_cast<int32_t*>(m + o_fill);
    pa.gq = reinterpret_cast<uint64_t*>(m + o_gq);
    pa.enq = reinterpret_cast<int32_t*>(m + o_enq);
    pa.rem = reinterpret_cast<int32_t*>(m + o_rem);
    b->pa = pa;
    b->blk_seg = reinterpret_cast<int32_t*>(m + o_bs);
    b->blk_z0 = reinterpret_cast<int32_t*>(m + o_bz);
    b->blk_first = reinterpret_cast<int32_t*>(m + o_bf);
    b->blkc = reinterpret_cast<int2*>(m + o_bc);
    b->blko = reinterpret_cast<int32_t*>(m + o_bo);
    b->n_blk = (int)nb;
    return FIC_OK;
}

// Every kernel of the persistent form, in order, on stream st: the pools of
// every level (they depend only on the images), the reset, the persistent
// kernel, the ordered compaction.
int batch_launch_pq(fic_batch* b, hipStream_t st) {
    const Lvl* dt = static_cast<const Lvl*>(b->dtab);
    const int n = (int)b->im.size(), nl = b->p.n_levels;
    const bool filtered = b->p.entropy_mode != 0;
    for (int l = 0; l < nl; ++l)
        for (const Group& g : b->groups) {
            std::vector<Lvl> h(b->htab.begin() + l * n + g.start, b->htab.begin() + l * n + g.start + g.count);
            int rc = launch_pool_phase(dt + l * n + g.start, h, b->im[0].ws->T, filtered, st);
            if (rc) return rc;
        }
    const PqArgs& pa = b->pa;
    {
        ProfScope ps("pq_reset", st);
        const int grid = std::max(1, std::min(1024, cdiv(std::max<int64_t>(pa.T, 4 * (int64_t)n), kBlock)));
        kt_pq_reset<<<grid, kBlock, 0, st>>>(dt, pa);
    }
    {
        ProfScope ps("pq_quadtree", st);
        kt_pq<<<b->pq_grid, kBlock, 0, st>>>(dt, pa);
    }
    {
        ProfScope ps("pq_emit", st);
        kt_pq_count<<<b->n_blk, kBlock, 0, st>>>(dt, pa, b->blk_seg, b->blk_z0, b->blkc);
        kt_pq_scan<<<n, kBlock, 0, st>>>(dt, pa, b->blk_first, b->blkc, b->blko, b->dorig, b->n_codes);
        kt_pq_scatter<<<b->n_blk, kBlock, 0, st>>>(dt, pa, b->blk_seg, b->blk_z0, b->blko);
    }
    LAUNCH_CHECK();
    return FIC_OK;
}

void batch_drop_graph(fic_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Every kernel of the batch, in order, on stream st.
int batch_launch_pq(fic_batch* b, hipStream_t st);

int batch_launch(fic_batch* b, hipStream_t st) {
    if (b->form == FIC_BATCH_PERSISTENT) return batch_launch_pq(b, st);
    const Lvl* dt = static_cast<const Lvl*>(b->dtab);
    const int n = (int)b->im.size();
    // Single stream: the batch graph is captured without the per-level pool streams.
    int rc = launch_quadtree(dt, b->htab, n, b->im[0].ws->T, b->p.entropy_mode != 0, st, &b->groups,
                             nullptr);
    if (rc) return rc;
    kt_copy_counts<<<cdiv(n, kBlock), kBlock, 0, st>>>(dt, n, b->dorig, b->n_codes);
    LAUNCH_CHECK();
    return FIC_OK;
}

// (Re)build the argument table and the captured graph of a batch.
int batch_build(fic_batch* b) {
    // a replay may still run on a caller stream while buffers are regrown
    HIP_TRY(hipDeviceSynchronize());
    batch_drop_graph(b);
    const int n = (int)b->im.size(), nl = b->p.n_levels;
    std::vector<Lvl> tab((size_t)nl * n);
    // one matcher per level for the whole batch: the one the largest image (first) gets
    std::vector<int> var(nl);
    {
        const std::vector<Level> lv0 = quad_levels(b->im[0].H, b->im[0].W, &b->p, b->ks, b->cg.data());
        for (int l = 0; l < nl; ++l) var[l] = lv0[l].var;
    }
    // the persistent kernel holds the VALU and small-set MFMA matchers
    if (b->form == FIC_BATCH_PERSISTENT)
        for (int l = 0; l < nl; ++l)
            if (var[l] != kVarMfq) var[l] = kVarValu;
    for (int i = 0; i < n; ++i) {
        BatchImage& m = b->im[i];
        std::vector<Level> lv = quad_levels(m.H, m.W, &b->p, b->ks, b->cg.data(), var.data());
        Sizes sz;
        for (const Level& v : lv) grow(sz, v);
        int rc = ensure_sizes(*m.ws, sz);
        if (rc) return rc;
        std::vector<Lvl> t = quad_tables(*m.ws, lv, m.img, m.H, m.W, m.pitch, &b->p,
                                         b->codes + m.code_off, m.capacity,
                                         b->stats ? b->stats + (size_t)m.orig * nl : nullptr);
        for (int l = 0; l < nl; ++l) tab[(size_t)l * n + i] = t[l];
    }
    const size_t bytes = sizeof(Lvl) * tab.size();
    if (b->dtab_bytes < bytes) {
        if (b->dtab) (void)hipFree(b->dtab);
        b->dtab = nullptr;
        b->dtab_bytes = 0;
        if (hipMalloc(&b->dtab, bytes) != hipSuccess) return fail(FIC_ENOMEM, "hipMalloc(%zu) failed", bytes);
        b->dtab_bytes = bytes;
    }
    HIP_TRY(hipMemcpy(b->dtab, tab.data(), bytes, hipMemcpyHostToDevice));
    b->htab = tab;
    if (b->form == FIC_BATCH_PERSISTENT) {
        int rc = pq_build(b, var);
        if (rc) return rc;
    }
    HIP_TRY(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    int rc = batch_launch(b, b->st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->st, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(FIC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return FIC_OK;
}

int batch_time(fic_batch* b, hipStream_t s, int reps, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(b->exec, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(FIC_EDEVICE, "timing the batch: %s", hipGetErrorString(e));
    *ms = t / reps;
    return FIC_OK;
}

// Chunk size level l actually uses (a 0 entry means the library default).
int batch_chunk(const fic_batch* b, int l) {
    if (b->cg[l] > 0) return b->cg[l];
    const int B = b->p.B0 >> l;
    return default_cg(B, auto_var(B, b->ks[l], 0));
}

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Cache key: GPU architecture, HIP runtime version, the batch's image sizes and parameters.
std::string batch_key(const fic_batch* b) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    uint64_t h = 1469598103934665603ull;
    for (const BatchImage& m : b->im) {
        h = fnv1a(h, &m.H, sizeof m.H);
        h = fnv1a(h, &m.W, sizeof m.W);
    }
    h = fnv1a(h, &b->p, sizeof b->p);
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|hip%d|n%zu|%016llx", arch.c_str(), rt, b->im.size(),
                  (unsigned long long)h);
    return buf;
}

}  // namespace
}  // namespace fic

FIC_API int fic_batch_create(int32_t n, const uint8_t* const* imgs, const int32_t* H,
                             const int32_t* W, const int32_t* pitch, const fic_params* p,
                             fic_code* codes, const int64_t* code_offset, int32_t* n_codes,
                             fic_level_stats* stats, fic_batch** out) {
    if (!out) return fail(FIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 65535) return fail(FIC_EINVAL, "batch size %d not in 1..65535", n);
    if (!imgs || !H || !W || !pitch || !code_offset) return fail(FIC_EINVAL, "NULL host array");
    if (!codes || !n_codes) return fail(FIC_EINVAL, "codes or n_codes is NULL");
    std::vector<KSet> ks;
    int rc = check_params(p, ks);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        if ((rc = check_image(imgs[i], H[i], W[i], pitch[i], p->B0)))
            return fail(rc, "image %d: %s", i, g_err.c_str());
        const int64_t cap = code_offset[i + 1] - code_offset[i];
        const int64_t lower = (int64_t)(H[i] / p->B0) * (W[i] / p->B0);
        if (code_offset[i] < 0 || cap < lower)
            return fail(FIC_ECAPACITY, "image %d: code capacity %lld below %lld", i, (long long)cap,
                        (long long)lower);
        if (cap > INT32_MAX) return fail(FIC_EINVAL, "image %d: code capacity too large", i);
    }
    fic_batch* b = new fic_batch();
    b->p = *p;
    b->ks = ks;
    b->codes = codes;
    b->n_codes = n_codes;
    b->stats = stats;
    b->cg.assign(p->n_levels, 0);
    auto bail = [&](int code) {
        fic_batch_destroy(b);
        return code;
    };
    if (hipGetDevice(&b->device) != hipSuccess) return bail(fail(FIC_EDEVICE, "hipGetDevice failed"));
    if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(FIC_EDEVICE, "hipStreamCreateWithFlags failed"));
    for (int i = 0; i < n; ++i) {
        BatchImage m;
        m.img = imgs[i];
        m.H = H[i];
        m.W = W[i];
        m.pitch = pitch[i];
        m.code_off = code_offset[i];
        m.capacity = (int)(code_offset[i + 1] - code_offset[i]);
        m.ws = nullptr;
        m.orig = i;
        if ((rc = new_ws(b->device, b->st, &m.ws))) return bail(rc);
        b->im.push_back(m);
    }
    // largest images first; equal sizes form one launch group
    std::stable_sort(b->im.begin(), b->im.end(), [](const BatchImage& x, const BatchImage& y) {
        return (int64_t)x.H * x.W != (int64_t)y.H * y.W ? (int64_t)x.H * x.W > (int64_t)y.H * y.W
                                                          : (x.H != y.H ? x.H > y.H : false);
    });
    for (int i = 0; i < n; ++i) {
        if (i == 0 || b->im[i].H != b->im[i - 1].H || b->im[i].W != b->im[i - 1].W)
            b->groups.push_back({i, 0});
        b->groups.back().count++;
    }
    {
        std::vector<int32_t> orig(n);
        for (int i = 0; i < n; ++i) orig[i] = b->im[i].orig;
        if (hipMalloc(&b->dorig, sizeof(int32_t) * n) != hipSuccess) return bail(fail(FIC_ENOMEM, "hipMalloc failed"));
        if (hipMemcpy(b->dorig, orig.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(FIC_EDEVICE, "upload of the image order failed"));
    }
    if ((rc = batch_build(b))) return bail(rc);
    *out = b;
    return FIC_OK;
}

FIC_API int fic_batch_run(fic_batch* b, void* stream) {
    if (!b || !b->exec) return fail(FIC_EINVAL, "batch is NULL or not built");
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return FIC_OK;
}

FIC_API int fic_batch_run_eager(fic_batch* b, void* stream) {
    if (!b || !b->exec) return fail(FIC_EINVAL, "batch is NULL or not built");
    return batch_launch(b, (hipStream_t)stream);
}

FIC_API int fic_batch_set_chunks(fic_batch* b, const int32_t* cg) {
    if (!b) return fail(FIC_EINVAL, "batch is NULL");
    for (int l = 0; l < b->p.n_levels; ++l) {
        const int v = cg ? cg[l] : 0;
        if (v < 0 || v > (1 << 20)) return fail(FIC_EINVAL, "chunk %d not in 0..2^20", v);
        b->cg[l] = v;
    }
    return batch_build(b);
}

FIC_API int fic_batch_get_chunks(const fic_batch* b, int32_t* cg) {
    if (!b || !cg) return fail(FIC_EINVAL, "NULL argument");
    for (int l = 0; l < b->p.n_levels; ++l) cg[l] = fic::batch_chunk(b, l);
    return FIC_OK;
}

FIC_API int fic_batch_set_form(fic_batch* b, int32_t form, const int32_t* tiles, int32_t workgroups) {
    if (!b) return fail(FIC_EINVAL, "batch is NULL");
    if (form != FIC_BATCH_LEVELS && form != FIC_BATCH_PERSISTENT) return fail(FIC_EINVAL, "form %d unknown", form);
    if (workgroups < 0) return fail(FIC_EINVAL, "workgroups < 0");
    const int nl = b->p.n_levels;
    std::vector<int> t(nl, 0);
    for (int l = 0; l < nl && tiles; ++l) {
        if (tiles[l] < 0 || tiles[l] > fic::kPqMaxTile)
            return fail(FIC_EINVAL, "tile of %d ranges not in 0..%d", tiles[l], fic::kPqMaxTile);
        t[l] = tiles[l];
    }
    const int keep_form = b->form, keep_wgs = b->wgs;
    const std::vector<int> keep_tiles = b->tiles;
    b->form = form;
    b->tiles = t;
    b->wgs = workgroups;
    const int rc = fic::batch_build(b);
    if (rc) {
        // restore the previous form (its graph is rebuilt)
        const std::string msg = fic::g_err;
        b->form = keep_form;
        b->tiles = keep_tiles;
        b->wgs = keep_wgs;
        (void)fic::batch_build(b);
        return fail(rc, "%s", msg.c_str());
    }
    return FIC_OK;
}

FIC_API int fic_batch_get_form(const fic_batch* b, int32_t* form, int32_t* tiles, int32_t* workgroups) {
    if (!b) return fail(FIC_EINVAL, "batch is NULL");
    if (form) *form = b->form;
    if (workgroups) *workgroups = b->form == FIC_BATCH_PERSISTENT ? b->pq_grid : 0;
    if (tiles)
        for (int l = 0; l < b->p.n_levels; ++l) tiles[l] = b->form == FIC_BATCH_PERSISTENT ? b->pa.R[l] : 0;
    return FIC_OK;
}

namespace fic {
namespace {

// Persistent form: coordinate descent over each level's ranges per tile (1,
// 2, 4 or 8 matcher calls) and then the resident workgroups per compute unit.
int pq_autotune(fic_batch* b, hipStream_t s, int reps, float* best_out) {
    const int nl = b->p.n_levels;
    float best;
    int rc = batch_time(b, s, reps, &best);
    if (rc) return rc;
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    const int fit = b->pq_grid;
    b->tiles.assign(nl, 0);
    for (int l = 0; l < nl; ++l) b->tiles[l] = b->pa.R[l];
    for (int l = 0; l < nl; ++l) {
        const int per = pq_block_ranges(b->p.B0 >> l, b->pa.kind[l]);
        const int keep = b->tiles[l];
        int best_t = keep;
        for (int m : {1, 2, 4, 8}) {
            const int t = per * m;
            if (t == keep || t > kPqMaxTile) continue;
            b->tiles[l] = t;
            if ((rc = batch_build(b))) return rc;
            float ms;
            if ((rc = batch_time(b, s, reps, &ms))) return rc;
            if (ms < best) {
                best = ms;
                best_t = t;
            }
        }
        b->tiles[l] = best_t;
    }
    const int keep_w = b->wgs;
    int best_w = keep_w;
    for (int per_cu = 1; per_cu * cus < fit; ++per_cu) {
        b->wgs = per_cu * cus;
        if ((rc = batch_build(b))) return rc;
        float ms;
        if ((rc = batch_time(b, s, reps, &ms))) return rc;
        if (ms < best) {
            best = ms;
            best_w = b->wgs;
        }
    }
    b->wgs = best_w;
    if ((rc = batch_build(b))) return rc;
    *best_out = best;
    return FIC_OK;
}

}  // namespace
}  // namespace fic

namespace fic {
namespace {

// Integers of the JSON list that follows `tag` in line ln (at most want of them).
std::vector<int> parse_list(const std::string& ln, const std::string& tag, int want) {
    std::vector<int> out;
    const size_t q = ln.find(tag);
    if (q == std::string::npos) return out;
    const char* c = ln.c_str() + q + tag.size();
    for (int l = 0; l < want; ++l) {
        char* end = nullptr;
        const long v = std::strtol(c, &end, 10);
        if (end == c) break;
        out.push_back((int)v);
        c = end;
        while (*c == ',' || *c == ' ') ++c;
    }
    return out;
}

}  // namespace
}  // namespace fic

FIC_API int fic_batch_autotune(fic_batch* b, void* stream, int32_t reps, const char* cache_path,
                               float* best_ms) {
    if (!b) return fail(FIC_EINVAL, "batch is NULL");
    if (reps < 1) return fail(FIC_EINVAL, "reps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const bool pq = b->form == FIC_BATCH_PERSISTENT;
    const std::string key = batch_key(b) + (pq ? "|persistent" : "|levels");
    const int nl = b->p.n_levels;
    int rc;
    // cached choice?
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[1024];
            std::vector<int> found, wg;
            while (std::fgets(line, sizeof line, f)) {
                std::string ln(line);
                if (ln.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
                found = parse_list(ln, pq ? "\"tiles\": [" : "\"chunks\": [", nl);
                wg = parse_list(ln, "\"workgroups\": ", 1);
            }
            std::fclose(f);
            if ((int)found.size() == nl && (!pq || wg.size() == 1)) {
                rc = pq ? fic_batch_set_form(b, FIC_BATCH_PERSISTENT, found.data(), wg[0])
                        : fic_batch_set_chunks(b, found.data());
                if (rc) return rc;
                if (best_ms) {
                    float ms;
                    if ((rc = batch_time(b, s, reps, &ms))) return rc;
                    *best_ms = ms;
                }
                return FIC_OK;
            }
        }
    }
    float best;
    if (pq) {
        if ((rc = pq_autotune(b, s, reps, &best))) return rc;
    } else {
        // coordinate descent over the matcher chunk of each level
        static const int cand[] = {32, 64, 128, 256, 512, 1024, 2048, 4096};
        if ((rc = batch_time(b, s, reps, &best))) return rc;
        for (int l = 0; l < nl; ++l) b->cg[l] = batch_chunk(b, l);
        for (int l = 0; l < nl; ++l) {
            const int keep = b->cg[l];
            int best_cg = keep;
            for (int c : cand) {
                b->cg[l] = c;
                if ((rc = batch_build(b))) return rc;
                float ms;
                if ((rc = batch_time(b, s, reps, &ms))) return rc;
                if (ms < best) {
                    best = ms;
                    best_cg = c;
                }
            }
            b->cg[l] = best_cg;
        }
        if ((rc = batch_build(b))) return rc;
    }
    if (best_ms) *best_ms = best;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "{\"key\": \"%s\", \"%s\": [", key.c_str(), pq ? "tiles" : "chunks");
            for (int l = 0; l < nl; ++l) std::fprintf(f, "%s%d", l ? ", " : "", pq ? b->pa.R[l] : b->cg[l]);
            std::fprintf(f, "]");
            if (pq) std::fprintf(f, ", \"workgroups\": %d", b->wgs);
            std::fprintf(f, ", \"ms\": %.4f}\n", best);
            std::fclose(f);
        }
    }
    return FIC_OK;
}

FIC_API int fic_batch_destroy(fic_batch* b) {
    if (!b) return FIC_OK;
    (void)hipDeviceSynchronize();
    fic::batch_drop_graph(b);
    for (fic::BatchImage& m : b->im)
        if (m.ws) fic::free_ws(m.ws);
    if (b->dtab) (void)hipFree(b->dtab);
    if (b->dorig) (void)hipFree(b->dorig);
    if (b->pq_mem) (void)hipFree(b->pq_mem);
    if (b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return FIC_OK;
}

#include "fic_learned_api.hip"
#include "fic_stream.hip"
