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

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    Ctrl* ctrl = nullptr;
    int64_t* T = nullptr;  // entropy table, kMaxWindow + 1 entries
    Buf key, pool, hl, sd, ad, jd, arow, sr, cr, part, blk, act0, act1, tmpc, dec, codes, map,
        imgA, imgB, acc, mr;
    Buf ar, srp, dh, dl, wd, cw;  // int8 MFMA matcher (B = 8)
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

int get_ws(hipStream_t s, Workspace** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find({dev, s});
    if (it != g_ws.end()) {
        *out = it->second;
        return FIC_OK;
    }
    Workspace* ws = new Workspace();
    ws->device = dev;
    ws->stream = s;
    if (hipMalloc(&ws->ctrl, sizeof(Ctrl)) != hipSuccess) {
        delete ws;
        return fail(FIC_ENOMEM, "hipMalloc of the control block failed");
    }
    if (hipMalloc(&ws->T, sizeof(int64_t) * (kMaxWindow + 1)) != hipSuccess) {
        (void)hipFree(ws->ctrl);
        delete ws;
        return fail(FIC_ENOMEM, "hipMalloc of the entropy table failed");
    }
    const std::vector<int64_t>& t = entropy_table();
    HIP_TRY(hipMemcpyAsync(ws->T, t.data(), sizeof(int64_t) * t.size(), hipMemcpyHostToDevice, s));
    {
        static Ctrl init;  // zero counters, empty histogram, no floor bound yet
        std::memset(&init, 0, sizeof init);
        init.cut_bound = ~0ull;
        HIP_TRY(hipMemcpyAsync(ws->ctrl, &init, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    g_ws[{dev, s}] = ws;
    *out = ws;
    return FIC_OK;
}

int ensure(Workspace& ws, Buf& b, size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (b.cap >= bytes) return FIC_OK;
    if (b.p) {
        HIP_TRY(hipStreamSynchronize(ws.stream));
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
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.on) return;
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

// ---------------------------------------------------------------- one level
// Matcher selected for a level (fic_encode_level_ex's variant).
enum { kVarValu = 1, kVarMfma = 2, kVarFp32 = 3 };

struct Level {
    int lv, B, L, gy, gx, total;  // domain grid
    int max_act;                  // worst-case active ranges
    int nc;                       // pool chunks of the matcher
    int var;                      // kVarValu, kVarMfma or kVarFp32
    KSet ks;
};

// The int8 MFMA matcher serves B = 8 with a contrast grid 0..k1 (k1 >= 2).
bool mfma_eligible(int B, const KSet& ks) {
    return B == 8 && ks.consecutive && ks.k0 == 0 && ks.n >= 3;
}

// Pool domains per chunk of the level's matcher (its partials per range).
int chunk_domains(const Level& v);

Level make_level(int lv, int H, int W, int B, int L, int max_act, const KSet& ks, int variant = 0) {
    Level v;
    v.var = variant != 0 ? variant : (mfma_eligible(B, ks) ? kVarMfma : kVarValu);
    v.lv = lv;
    v.B = B;
    v.L = L;
    v.gy = (H - 2 * B) / L + 1;
    v.gx = (W - 2 * B) / L + 1;
    v.total = v.gy * v.gx;
    v.max_act = max_act;
    v.ks = ks;
    int row_blocks = cdiv((int64_t)8 * max_act, kBlock);
    int nc = cdiv(2048, row_blocks);
    nc = std::max(1, std::min(nc, 64));
    nc = std::min(nc, std::max(1, cdiv(v.total, 64)));
    v.nc = nc;
    return v;
}

int chunk_domains(const Level& v) {
    if (v.var == kVarMfma) return kM8Chunk;
    if (v.var == kVarFp32) return 256;
    return match_chunk_domains(v.B);
}

struct Sizes {
    size_t key = 0, pool = 0, hl = 0, dom = 0, arow = 0, rng = 0, part = 0, blk = 0, act = 0;
    size_t ar = 0, dcol = 0;  // int8 MFMA matcher
};

void grow(Sizes& s, const Level& v) {
    const int n = v.B * v.B;
    s.key = std::max(s.key, (size_t)v.total * 8);
    s.pool = std::max(s.pool, (size_t)v.total * 4);
    s.hl = std::max(s.hl, (size_t)v.total * (n / 2) * 4);
    s.dom = std::max(s.dom, (size_t)v.total);
    s.arow = std::max(s.arow, (size_t)v.max_act * 8 * n);
    s.rng = std::max(s.rng, (size_t)v.max_act);
    s.part = std::max(s.part, (size_t)v.max_act * v.nc * sizeof(Partial));
    size_t nblk = (size_t)std::max(cdiv(v.total, kBlock * kPoolItems), cdiv(v.max_act, kBlock * kQuadItems));
    s.blk = std::max(s.blk, nblk * sizeof(int2));
    s.act = std::max(s.act, (size_t)v.max_act);
    if (v.var == kVarMfma) {
        s.ar = std::max(s.ar, (size_t)v.max_act * 8 * 64);
        s.dcol = std::max(s.dcol, (size_t)v.total);
    }
}

int ensure_sizes(Workspace& ws, const Sizes& s) {
    int rc;
    if ((rc = ensure(ws, ws.key, s.key))) return rc;
    if ((rc = ensure(ws, ws.pool, s.pool))) return rc;
    if ((rc = ensure(ws, ws.hl, s.hl))) return rc;
    if ((rc = ensure(ws, ws.sd, s.dom * 4))) return rc;
    if ((rc = ensure(ws, ws.ad, s.dom * 8))) return rc;
    if ((rc = ensure(ws, ws.jd, s.dom * 4))) return rc;
    if ((rc = ensure(ws, ws.arow, s.arow))) return rc;
    if ((rc = ensure(ws, ws.sr, s.rng * 4))) return rc;
    if ((rc = ensure(ws, ws.cr, s.rng * 8))) return rc;
    if ((rc = ensure(ws, ws.part, s.part))) return rc;
    if ((rc = ensure(ws, ws.blk, s.blk))) return rc;
    if ((rc = ensure(ws, ws.act0, s.act * 4))) return rc;
    if ((rc = ensure(ws, ws.act1, s.act * 4))) return rc;
    if ((rc = ensure(ws, ws.tmpc, s.act * sizeof(fic_code)))) return rc;
    if ((rc = ensure(ws, ws.dec, s.act))) return rc;
    if (s.ar) {
        if ((rc = ensure(ws, ws.ar, s.ar))) return rc;
        if ((rc = ensure(ws, ws.srp, s.rng * 4))) return rc;
        if ((rc = ensure(ws, ws.dh, s.dcol * 64))) return rc;
        if ((rc = ensure(ws, ws.dl, s.dcol * 64))) return rc;
        if ((rc = ensure(ws, ws.wd, s.dcol * 4))) return rc;
        if ((rc = ensure(ws, ws.cw, s.dcol * 4))) return rc;
    }
    return FIC_OK;
}

void launch_mfma8(Workspace& ws, const Level& v, const uint8_t* img, int pitch, bool filtered,
                  const int32_t* act) {
    hipStream_t st = ws.stream;
    const int32_t* act_count = ws.ctrl->act_count + v.lv;
    {
        ProfScope ps("pool_prep", st);
        k_pool_prep_i8<<<cdiv((int64_t)v.total * 4, kBlock), kBlock, 0, st>>>(
            img, pitch, v.L, v.gx, P<int32_t>(ws.pool), filtered ? -1 : v.total, ws.ctrl,
            P<int8_t>(ws.dh), P<int8_t>(ws.dl), P<uint32_t>(ws.sd), P<int64_t>(ws.ad),
            P<int32_t>(ws.jd), P<float>(ws.wd), P<float>(ws.cw));
    }
    {
        ProfScope ps("range_prep", st);
        k_range_prep_i8<<<cdiv((int64_t)8 * v.max_act, kBlock), kBlock, 0, st>>>(
            img, pitch, act, act_count, P<int8_t>(ws.ar), P<int32_t>(ws.sr), P<int32_t>(ws.srp),
            P<int64_t>(ws.cr));
    }
    ProfScope ps("match_b8_mfma", st);
    dim3 grid(cdiv((int64_t)8 * v.max_act, kM8Rows), v.nc);
    k_match_mfma8<<<grid, kM8Waves * 64, 0, st>>>(
        P<int8_t>(ws.ar), P<int32_t>(ws.srp), act_count, P<int8_t>(ws.dh), P<int8_t>(ws.dl),
        P<uint32_t>(ws.sd), P<int64_t>(ws.ad), P<float>(ws.wd), P<float>(ws.cw), P<int32_t>(ws.jd),
        ws.ctrl, v.ks.k1, v.nc, P<Partial>(ws.part));
}

template <int B>
void launch_level_kernels(Workspace& ws, const Level& v, const uint8_t* img, int pitch,
                          bool filtered, const int32_t* act) {
    hipStream_t st = ws.stream;
    const int32_t* act_count = ws.ctrl->act_count + v.lv;
    if (B == 8 && v.var == kVarMfma) {
        launch_mfma8(ws, v, img, pitch, filtered, act);
        return;
    }
    {
        ProfScope ps("pool_prep", st);
        k_pool_prep<B><<<cdiv((int64_t)v.total * PrepShape<B>::TPD, kBlock), kBlock, 0, st>>>(
            img, pitch, v.L, v.gx, P<int32_t>(ws.pool), filtered ? -1 : v.total, ws.ctrl,
            P<uint32_t>(ws.hl), P<uint32_t>(ws.sd), P<int64_t>(ws.ad), P<int32_t>(ws.jd));
    }
    if (B == 8 && v.var == kVarFp32) {
        ProfScope ps("match_b8_fp32", st);
        dim3 g32(cdiv(v.max_act, kBlock / 8), v.nc);
        k_match_fp32<<<g32, kBlock, 0, st>>>(img, pitch, act, act_count, img, v.L, v.gx,
                                             P<int32_t>(ws.jd), ws.ctrl, v.ks.k1, v.nc,
                                             P<Partial>(ws.part));
        return;
    }
    ProfScope ps(match_label(B), st);
    dim3 grid(cdiv(v.max_act, kBlock / 8), v.nc);
    const int mode = v.ks.n <= kSmallMax ? kModeSmall : (v.ks.consecutive ? kModeGrid : kModeList);
#define FIC_MATCH_ARGS                                                                          \
    img, pitch, act, act_count, P<uint32_t>(ws.hl), P<uint32_t>(ws.sd), P<int64_t>(ws.ad),      \
        P<int32_t>(ws.jd), ws.ctrl, v.ks, v.nc, P<Partial>(ws.part), P<int32_t>(ws.sr),          \
        P<int64_t>(ws.cr)
    if (mode == kModeSmall)
        k_match<B, kModeSmall><<<grid, kBlock, 0, st>>>(FIC_MATCH_ARGS);
    else if (mode == kModeGrid)
        k_match<B, kModeGrid><<<grid, kBlock, 0, st>>>(FIC_MATCH_ARGS);
    else
        k_match<B, kModeList><<<grid, kBlock, 0, st>>>(FIC_MATCH_ARGS);
#undef FIC_MATCH_ARGS
}

// Radix-select digits (shift, width) covering the bits of keys below maxkey.
std::vector<std::pair<int, int>> select_digits(int64_t maxkey) {
    int bits = 1;
    while (bits < 63 && ((int64_t)1 << bits) <= maxkey) ++bits;
    std::vector<std::pair<int, int>> d;
    for (int hi = bits; hi > 0; hi -= kSelBits) {
        int w = std::min(kSelBits, hi);
        d.push_back({hi - w, w});
    }
    return d;
}

// Pool of one level (entropy filter of Section 3, or the whole grid), then the
// pool moments and the matcher. The level's active list and count must
// already be on the device.
int run_level(Workspace& ws, const Level& v, const uint8_t* img, int pitch, int entropy_mode,
              float entropy_bits, int min_pool, const int32_t* act) {
    hipStream_t st = ws.stream;
    const bool filtered = entropy_mode == 1;
    if (filtered) {
        const int side = 2 * v.B;
        const int64_t M = entropy_cut(side * side, (double)entropy_bits);
        {
            ProfScope ps("pool_score", st);
            switch (side) {
                case 4:
                    k_pool_score<4><<<cdiv((int64_t)v.total * ScoreShape<4>::TPD, kBlock), kBlock, 0, st>>>(
                        img, pitch, v.L, v.gx, v.total, ws.T, M, P<int64_t>(ws.key), ws.ctrl);
                    break;
                case 8:
                    k_pool_score<8><<<cdiv((int64_t)v.total * ScoreShape<8>::TPD, kBlock), kBlock, 0, st>>>(
                        img, pitch, v.L, v.gx, v.total, ws.T, M, P<int64_t>(ws.key), ws.ctrl);
                    break;
                case 16:
                    k_pool_score<16><<<cdiv((int64_t)v.total * ScoreShape<16>::TPD, kBlock), kBlock, 0, st>>>(
                        img, pitch, v.L, v.gx, v.total, ws.T, M, P<int64_t>(ws.key), ws.ctrl);
                    break;
                default:
                    k_pool_score<32><<<cdiv((int64_t)v.total * ScoreShape<32>::TPD, kBlock), kBlock, 0, st>>>(
                        img, pitch, v.L, v.gx, v.total, ws.T, M, P<int64_t>(ws.key), ws.ctrl);
                    break;
            }
        }
        const int rank = std::min(min_pool, v.total);
        {
            // floor: an upper bound on the rank-th smallest key
            ProfScope ps("pool_select", st);
            const int64_t maxkey = entropy_table()[side * side] + 1;
            int shift = 0;
            while ((maxkey >> shift) >= kSelBins) ++shift;
            const int chunk = std::max(8192, cdiv(v.total, 64));
            k_floor_bound<<<cdiv(v.total, chunk), kBlock, 0, st>>>(P<int64_t>(ws.key), v.total,
                                                                   min_pool, rank, shift, chunk,
                                                                   ws.ctrl);
        }
        {
            ProfScope ps("pool_compact", st);
            CompactArgs a{};
            a.kind = 0;
            a.total = v.total;
            a.min_pool = min_pool;
            a.M = M;
            a.key = P<int64_t>(ws.key);
            const int nblk = cdiv(v.total, kBlock * kPoolItems);
            k_pool_count<<<nblk, kBlock, 0, st>>>(a, ws.ctrl, P<int2>(ws.blk));
            k_pool_scatter<<<nblk, kBlock, 0, st>>>(a, ws.ctrl, P<int2>(ws.blk), P<int32_t>(ws.pool));
        }
        {
            ProfScope ps("pool_select", st);
            k_floor_select<<<1, 1024, 0, st>>>(P<int64_t>(ws.key), v.total, min_pool, rank,
                                               P<int32_t>(ws.pool), ws.ctrl);
        }
    }
    switch (v.B) {
        case 2: launch_level_kernels<2>(ws, v, img, pitch, filtered, act); break;
        case 4: launch_level_kernels<4>(ws, v, img, pitch, filtered, act); break;
        case 8: launch_level_kernels<8>(ws, v, img, pitch, filtered, act); break;
        default: launch_level_kernels<16>(ws, v, img, pitch, filtered, act); break;
    }
    LAUNCH_CHECK();
    return FIC_OK;
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

int check_params(const fic_params* p, int H, int W, std::vector<KSet>& ks) {
    if (!p) return fail(FIC_EINVAL, "params pointer is NULL");
    if (p->n_levels < 1 || p->n_levels > 4) return fail(FIC_EINVAL, "n_levels %d not in 1..4", p->n_levels);
    if (!valid_B(p->B0)) return fail(FIC_EINVAL, "B0 %d not in {2,4,8,16}", p->B0);
    if ((p->B0 >> (p->n_levels - 1)) < 2) return fail(FIC_EINVAL, "last level range side below 2");
    if (!(p->rms_thresh >= 0.0f) || !std::isfinite(p->rms_thresh))
        return fail(FIC_EINVAL, "rms_thresh must be finite and >= 0");
    if (p->entropy_mode != 0 && p->entropy_mode != 1) return fail(FIC_EINVAL, "entropy_mode %d not 0 or 1", p->entropy_mode);
    if (p->entropy_mode == 1 && !std::isfinite(p->entropy_bits)) return fail(FIC_EINVAL, "entropy_bits not finite");
    if (p->min_pool < 1) return fail(FIC_EINVAL, "min_pool must be >= 1");
    ks.resize(p->n_levels);
    for (int l = 0; l < p->n_levels; ++l) {
        if (p->L[l] < 1) return fail(FIC_EINVAL, "L[%d] = %d < 1", l, p->L[l]);
        int rc = check_kset(p->s_k[l], p->n_s[l], &ks[l]);
        if (rc) return rc;
    }
    (void)H;
    (void)W;
    return FIC_OK;
}

// Quadtree encode into `codes` (device), counters in the control block.
int encode_image_impl(Workspace& ws, const uint8_t* img, int H, int W, int pitch,
                      const fic_params* p, const std::vector<KSet>& ks, fic_code* codes,
                      int capacity, fic_level_stats* stats) {
    hipStream_t st = ws.stream;
    std::vector<Level> lv;
    Sizes sz;
    for (int l = 0; l < p->n_levels; ++l) {
        int B = p->B0 >> l;
        lv.push_back(make_level(l, H, W, B, p->L[l], (H / B) * (W / B), ks[l]));
        grow(sz, lv.back());
    }
    int rc = ensure_sizes(ws, sz);
    if (rc) return rc;
    k_act_full<<<cdiv(lv[0].max_act, kBlock), kBlock, 0, st>>>(P<int32_t>(ws.act0), H / p->B0,
                                                             W / p->B0, p->B0, ws.ctrl, 0, 1);
    Buf* cur = &ws.act0;
    Buf* nxt = &ws.act1;
    for (int l = 0; l < p->n_levels; ++l) {
        const Level& v = lv[l];
        rc = run_level(ws, v, img, pitch, p->entropy_mode, p->entropy_bits, p->min_pool,
                       P<int32_t>(*cur));
        if (rc) return rc;
        const int n = v.B * v.B;
        const bool last = l == p->n_levels - 1;
        // keep iff E <= T^2 n  <=>  1600 n E <= 1600 T^2 n^2
        double thr_d = std::floor(1600.0 * (double)p->rms_thresh * (double)p->rms_thresh *
                                  (double)n * (double)n);
        int64_t thr = thr_d >= 9.0e18 ? INT64_MAX : (int64_t)thr_d;
        const int nblk = cdiv(v.max_act, kBlock * kQuadItems);
        {
            ProfScope ps("reduce_quad", st);
            k_reduce_quad<<<nblk, kBlock, 0, st>>>(
                v.B, v.L, v.gx, l, last ? 1 : 0, thr, P<int32_t>(*cur), ws.ctrl, P<Partial>(ws.part),
                v.nc, chunk_domains(v), P<int64_t>(ws.cr), P<int32_t>(ws.sr), v.ks,
                P<fic_code>(ws.tmpc), P<uint8_t>(ws.dec), P<int2>(ws.blk), stats);
        }
        {
            ProfScope ps("quad_compact", st);
            CompactArgs a{};
            a.kind = 1;
            a.act_count = ws.ctrl->act_count + l;
            a.decision = P<uint8_t>(ws.dec);
            k_quad_scatter<<<nblk, kBlock, 0, st>>>(a, ws.ctrl, P<int2>(ws.blk),
                                                    P<fic_code>(ws.tmpc), codes, capacity,
                                                    P<int32_t>(*cur), P<int32_t>(*nxt), v.B / 2);
        }
        LAUNCH_CHECK();
        std::swap(cur, nxt);
    }
    return FIC_OK;
}

}  // namespace
}  // namespace fic

using namespace fic;

FIC_API int fic_version(void) { return 100; }

FIC_API const char* fic_last_error(void) { return g_err.c_str(); }

FIC_API int fic_encode_level_ex(const uint8_t* img, int32_t H, int32_t W, int32_t pitch, int32_t B,
                                int32_t L, const int8_t* s_k, int32_t n_s, int32_t entropy_mode,
                                float entropy_bits, int32_t min_pool, const int32_t* range_yx,
                                int32_t n_ranges, fic_match* out, int32_t* pool_out,
                                int32_t* pool_count, int32_t variant, void* stream) {
    int rc = check_image(img, H, W, pitch, B);
    if (rc) return rc;
    if (L < 1) return fail(FIC_EINVAL, "domain step L=%d < 1", L);
    KSet ks;
    if ((rc = check_kset(s_k, n_s, &ks))) return rc;
    if (entropy_mode != 0 && entropy_mode != 1) return fail(FIC_EINVAL, "entropy_mode %d not 0 or 1", entropy_mode);
    if (entropy_mode == 1 && !std::isfinite(entropy_bits)) return fail(FIC_EINVAL, "entropy_bits not finite");
    if (min_pool < 1) return fail(FIC_EINVAL, "min_pool must be >= 1");
    if (n_ranges < 0) return fail(FIC_EINVAL, "n_ranges < 0");
    if (!range_yx && n_ranges != (H / B) * (W / B))
        return fail(FIC_EINVAL, "range_yx is NULL but n_ranges %d != %d", n_ranges, (H / B) * (W / B));
    if (n_ranges > 0 && !out) return fail(FIC_EINVAL, "out is NULL");
    if (variant < FIC_MATCH_AUTO || variant > FIC_MATCH_FP32)
        return fail(FIC_EINVAL, "matcher variant %d unknown", variant);
    if ((variant == FIC_MATCH_MFMA_I8 || variant == FIC_MATCH_FP32) && !mfma_eligible(B, ks))
        return fail(FIC_EINVAL, "matcher variant %d needs B = 8 and contrast set 0..k1 (k1 >= 2)",
                    variant);
    if (n_ranges == 0) return FIC_OK;
    Workspace* ws;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    const int var = variant == FIC_MATCH_VALU ? kVarValu
                    : variant == FIC_MATCH_MFMA_I8 ? kVarMfma
                    : variant == FIC_MATCH_FP32 ? kVarFp32 : 0;
    Level v = make_level(0, H, W, B, L, n_ranges, ks, var);
    Sizes sz;
    grow(sz, v);
    if ((rc = ensure_sizes(*ws, sz))) return rc;
    hipStream_t st = ws->stream;
    int32_t* act = P<int32_t>(ws->act0);
    if (range_yx)
        k_act_from_yx<<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(act, range_yx, n_ranges, H, W, B,
                                                                 ws->ctrl);
    else
        k_act_full<<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(act, H / B, W / B, B, ws->ctrl, 0, 0);
    if ((rc = run_level(*ws, v, img, pitch, entropy_mode, entropy_bits, min_pool, act)))
        return rc;
    {
        ProfScope ps("reduce_level", st);
        if (v.var == kVarFp32)
            k_reduce_fp32<<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(
                img, pitch, L, v.gx, act, ws->ctrl->act_count, P<Partial>(ws->part), v.nc, ws->ctrl,
                out);
        else
            k_reduce_level<<<cdiv(n_ranges, kBlock), kBlock, 0, st>>>(
                B, L, v.gx, act, ws->ctrl->act_count, P<Partial>(ws->part), v.nc, chunk_domains(v),
                ws->ctrl, P<int64_t>(ws->cr), P<int32_t>(ws->sr), ks, out);
    }
    LAUNCH_CHECK();
    if (pool_count)
        HIP_TRY(hipMemcpyAsync(pool_count, &ws->ctrl->pool_count, sizeof(int32_t),
                               hipMemcpyDeviceToDevice, st));
    if (pool_out) {
        if (entropy_mode == 1)
            HIP_TRY(hipMemcpyAsync(pool_out, ws->pool.p, sizeof(int32_t) * v.total,
                                   hipMemcpyDeviceToDevice, st));
        else
            HIP_TRY(hipMemcpyAsync(pool_out, ws->jd.p, sizeof(int32_t) * v.total,
                                   hipMemcpyDeviceToDevice, st));
    }
    return FIC_OK;
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

FIC_API int fic_encode_image(const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                             const fic_params* p, fic_code* codes, int32_t capacity,
                             int32_t* n_codes, fic_level_stats* stats, void* stream) {
    std::vector<KSet> ks;
    int rc = check_params(p, H, W, ks);
    if (rc) return rc;
    if ((rc = check_image(img, H, W, pitch, p->B0))) return rc;
    if (!codes || !n_codes) return fail(FIC_EINVAL, "codes or n_codes is NULL");
    const int lower = (H / p->B0) * (W / p->B0);
    if (capacity < lower)
        return fail(FIC_ECAPACITY, "capacity %d below the %d codes of the first level", capacity, lower);
    Workspace* ws;
    if ((rc = get_ws((hipStream_t)stream, &ws))) return rc;
    if ((rc = encode_image_impl(*ws, img, H, W, pitch, p, ks, codes, capacity, stats))) return rc;
    HIP_TRY(hipMemcpyAsync(n_codes, &ws->ctrl->n_codes, sizeof(int32_t), hipMemcpyDeviceToDevice,
                           ws->stream));
    return FIC_OK;
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
    int rc = check_params(&q, H, W, ks);
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
