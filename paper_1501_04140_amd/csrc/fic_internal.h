// Shared declarations of the libfic kernels and host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fic.h"

namespace fic {

constexpr int kBlock = 256;    // threads per workgroup (4 wavefronts of 64)
constexpr int kItems = 8;      // items per thread in the compaction kernels
constexpr int kSelBits = 12;   // radix-select digit width
constexpr int kSelBins = 1 << kSelBits;
constexpr int kEntFrac = 32;   // fixed-point fraction bits of the entropy table
constexpr int kMaxWindow = 1024;  // largest histogram window (32 x 32 domain)

// Device-resident control block of one workspace.
struct Ctrl {
    int32_t act_count[5];  // active ranges per quadtree level (index = level)
    int32_t pool_count;    // domains in the current level's pool
    int32_t pass_count;    // running count of the entropy score kernel (reset by it)
    int32_t passed;        // domains above the entropy threshold at this level
    int32_t n_codes;       // codes emitted so far (may exceed capacity)
    int32_t lvl_base[5];   // codes emitted before each quadtree level
    int32_t err;
    int32_t sel_rank;      // rank still to find inside the current key prefix
    uint64_t sel_prefix;   // unused, kept for layout
    uint64_t cut_bound;    // floor mode: upper bound on the min_pool-th smallest key
    uint32_t ghist[kSelBins];
};

// Contrast set of a level: s = k / 10.
struct KSet {
    int n;            // number of values
    int consecutive;  // 1 iff k = k0, k0+1, ..., k1
    int k0, k1;
    int k[12];
};

// Best candidate of one range over one chunk of the pool.
struct Partial {
    int64_t F;    // k^2 A' - 80 k B'  (= 1600 n E minus the range constant 1600 C)
    int64_t key;  // (domain << 8) | (iso << 4) | contrast index
};

// Arguments of the quadtree kernels for one image at one level. Kernels read
// tab[blockIdx.z]: a table of one for a single image, one entry per image for
// a batch.
// Matcher of a level: dot4 VALU, int8 MFMA (hi/lo split), FP32 comparator,
// FP16 MFMA (exact for B = 8).
// kVarMfq: the FP16 MFMA matcher of B = 8 and 16 levels with one or two contrast values
enum { kVarValu = 1, kVarMfma = 2, kVarFp32 = 3, kVarMfma16 = 4, kVarMfq = 5 };

struct Lvl {
    const uint8_t* img;
    int32_t pitch, H, W;
    int32_t B, L, gx, gy, total;  // domain grid
    int32_t max_act;              // worst-case active ranges
    int32_t lv, last;             // quadtree level; 1 on the last level
    int32_t nc, cg;               // matcher: pool chunks launched, domains per chunk
    int32_t min_pool, rank;       // entropy floor: pool size wanted, min(min_pool, total)
    int32_t sel_shift, bound_chunk;
    int32_t capacity;
    int32_t var;                  // matcher: kVarValu, kVarMfma, kVarFp32, kVarMfma16 or kVarMfq
    int32_t pmode;                // pool filter: 0 none, 1 entropy, 2 variance
    int64_t M;                    // filter cut (keep iff key < M)
    int64_t kv;                   // variance filter: key = kv - (N sum p^2 - (sum p)^2)
    int64_t thr;                  // keep iff 1600 n E <= thr
    Ctrl* ctrl;                   // quadtree control: active counts, codes
    Ctrl* pctrl;                  // this level's pool control: pool size, filter counters
    int2* pblk;                   // pool compaction: per-workgroup counts
    int64_t* key;
    int32_t* pool;
    uint32_t* hl;
    uint32_t* sd;
    int64_t* ad;
    int32_t* jd;
    Partial* part;
    int32_t* sr;
    int64_t* cr;
    int32_t* act;
    int32_t* act_next;
    fic_code* tmpc;
    uint8_t* dec;
    int2* blk;
    fic_code* codes;
    fic_level_stats* stats;
    int8_t* ar;  // int8 MFMA matcher (B = 8)
    int32_t* srp;
    int64_t* gb;  // MFMA grid matchers: each range's best F so far over all pool chunks
    int2* rc;     // int8 MFMA grid matcher: each range's row offset c and sum |r' - c|
    // optional, MFMA grid matchers: per range of the grid (grid order), a match
    // already reached (e_num >= 0) whose F starts the range's bound gb
    const fic_match* gbseed;
    int8_t* dh;
    int8_t* dl;
    float* gd;
    uint32_t* flags;    // optional: split flags, one bit per active range, levels in order
    int32_t* pools_out; // optional: this level's pool list
    int32_t* n_out;     // optional, last level: the number of codes, written by the compaction
    KSet ks;
};

}  // namespace fic
