// Persistent quadtree: one kernel matches, decides and splits every level of
// every image of a batch (Section 2's quadtree, with the predefined contrast
// values of Section 3.1 or any other contrast set).
//
// Work is a queue of range tiles. A tile is (image, level, up to R ranges of
// that level's active list). Resident workgroups claim tiles in order from a
// device counter; the level-0 tiles of every image are known in advance, the
// tiles of deeper levels are pushed as they fill. A workgroup stages its
// tile's ranges, runs the level's matcher over the whole of the level's pool,
// decides keep or split per range (RMS threshold, Section 2), writes the
// range's result, and appends the four children of each split range to the
// next level's queue of the same image. No host launch happens between
// levels, and a child range is matched as soon as its tile fills, while other
// ranges of its parent's level are still being searched.
//
// Cross-workgroup traffic is single words only, so no device-scope fence (an
// L2 write-back on this chip) is needed:
//  * queue entries and ready-tile slots are 64-bit words (run epoch << 32 |
//    value) written once with agent-scope atomic stores; a reader spins until
//    the word carries the current run's epoch, so stale words from earlier
//    runs are never taken;
//  * counters are atomic read-modify-writes: per (image, level) the entries
//    queued (enq) and the ranges not yet decided (rem, plus kPqOpen until the
//    level above has finished); per tile the entries written (fill); the
//    claim and push positions; the images finished.
// A level finishes when its rem reaches 0. The workgroup that sees this
// pushes the next level's last, partial tile, closes that level (rem -=
// kPqOpen) and, if that reaches 0 too, carries on down; after the last level
// it counts the image as finished. Where one atomic must be performed before
// the next (a push before the decrement that can end the run), the wave
// waits for its memory operations in between.
//
// Results go to dense per-level arrays indexed by the range's quadtree slot
// z (level-0 raster index, then two bits per level: 0 TL, 1 TR, 2 BL, 3 BR).
// Slot order at a level is the order of the level-synchronous active list
// (children follow their parents), so a final ordered compaction over the
// slots (kt_pq_count / kt_pq_scan / kt_pq_scatter) emits the codes in exactly
// the order fic_encode_image documents. A slot is a leaf iff every ancestor
// was split in this run and the slot was kept; states of slots that were not
// active in this run are never read.

namespace fic {

#ifndef FIC_PQ_WAVES
#define FIC_PQ_WAVES 4  // waves per SIMD the persistent kernel is compiled for
#endif
constexpr int kPqMaxTile = 256;         // ranges per tile, at most
constexpr int32_t kPqOpen = 1 << 30;    // in a level's rem while the level above runs
constexpr int kPqEmitItems = 8;         // slots per thread in the compaction
constexpr int kPqEmitSlots = kBlock * kPqEmitItems;
// Polls of one wait before the kernel gives up and flags the run (seconds at
// the sleep between polls; every wait ends even if the protocol were broken).
constexpr int kPqSpinLimit = 1 << 24;

// Matchers the persistent kernel holds: VALU small set, grid, list; FP16 MFMA
// small set with one or two nonzero values.
enum { kPqValuSmall = 0, kPqValuGrid = 1, kPqValuList = 2, kPqMfq1 = 3, kPqMfq2 = 4 };

struct PqRec {           // the best transform of one range (16 bytes)
    int64_t e_num;
    int32_t dom;
    int16_t q_o;
    uint8_t iso_s;       // iso | s_idx << 3
    uint8_t pad;
};

struct PqCtl {
    uint32_t epoch;      // this run's tag (the reset kernel increments it)
    int32_t ghead;       // tiles claimed
    int32_t gtail;       // tiles pushed (levels >= 1)
    int32_t done;        // images whose last level has finished
    int32_t err;         // set when a wait ran past kPqSpinLimit (the run's results are void)
};

struct PqArgs {
    int32_t n_img, n_levels, B0;
    int32_t R[4];        // ranges per tile, per level
    int32_t kind[4];     // matcher per level
    int32_t T0;          // tiles of level 0 over all images
    int32_t T;           // tiles over all levels
    int32_t gq_cap;      // ready-tile slots (pushable tiles + one per workgroup)
    const int32_t* tile_base;  // [level * n_img + image] first tile, ascending
    const int64_t* slot_base;  // [level * n_img + image] first slot of rec / state / qe
    PqRec* rec;
    uint8_t* state;      // 1 kept, 0 split
    uint64_t* qe;        // queued ranges: epoch << 32 | slot
    int32_t* fill;       // [tile] entries written
    uint64_t* gq;        // pushed tiles: epoch << 32 | tile
    int32_t* enq;        // [image * 4 + level]
    int32_t* rem;        // [image * 4 + level]
    PqCtl* ctl;
};

__device__ inline void pq_wait_memory() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ inline uint64_t pq_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t pq_load32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void pq_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t pq_add(int32_t* p, int32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last index with base[index] <= v (base ascending, base[0] <= v).
__device__ inline int pq_find(const int32_t* base, int n, int v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Packed corner (y << 16 | x) of slot z at level l.
__device__ inline int pq_yx(int z, int l, int gx0, int B0) {
    const int r0 = z >> (2 * l);
    int y = (r0 / gx0) * B0, x = (r0 % gx0) * B0;
    for (int k = 1; k <= l; ++k) {
        const int c = (z >> (2 * (l - k))) & 3;
        y += (c >> 1) * (B0 >> k);
        x += (c & 1) * (B0 >> k);
    }
    return (y << 16) | x;
}

__device__ inline void pq_push(const PqArgs& pa, uint32_t epoch, int tile) {
    const int slot = pq_add(&pa.ctl->gtail, 1);
    pq_store(pa.gq + slot, ((uint64_t)epoch << 32) | (uint32_t)tile);
}

// LDS of every matcher the kernel holds, overlaid.
// The B = 16 matchers take half their usual LDS stages here, so that four
// or five workgroups fit on a compute unit.
constexpr int kPqTn16 = MatchTile<16>::TN / 2;
constexpr int kPqCols16 = mq_cols(16) / 2;
union PqSmem {
    MatchSmem<2, kModeSmall> v2s;
    MatchSmem<2, kModeGrid> v2g;
    MatchSmem<2, kModeList> v2l;
    MatchSmem<4, kModeSmall> v4s;
    MatchSmem<4, kModeGrid> v4g;
    MatchSmem<4, kModeList> v4l;
    MatchSmem<8, kModeSmall> v8s;
    MatchSmem<8, kModeGrid> v8g;
    MatchSmem<8, kModeList> v8l;
    MatchSmem<16, kModeSmall, kPqTn16> v16s;
    MatchSmem<16, kModeGrid, kPqTn16> v16g;
    MatchSmem<16, kModeList, kPqTn16> v16l;
    MqSmem<4, 1> q41;
    MqSmem<4, 2> q42;
    MqSmem<8, 1> q81;
    MqSmem<8, 2> q82;
    MqSmem<16, 1, kPqCols16> q161;
    MqSmem<16, 2, kPqCols16> q162;
};

// The persistent kernel's LDS (namespace scope, so that each matcher's own
// non-inlined function addresses it directly).
__shared__ PqSmem g_pq_u;
__shared__ int32_t g_pq_act[kPqMaxTile];
__shared__ int32_t g_pq_z[kPqMaxTile];
__shared__ Partial g_pq_part[64];
__shared__ int32_t g_pq_sr[64];
__shared__ int64_t g_pq_cr[64];
__shared__ int32_t g_pq_n;
__shared__ uint8_t g_pq_split[kPqMaxTile];

// Ranges one matcher call takes (its workgroup's share).
__host__ __device__ constexpr int pq_block_ranges(int B, int kind) {
    return kind >= kPqMfq1 ? mq_rows(B) / 8 : match_ranges_per_block(B, kind == kPqValuSmall ? kModeSmall : kModeGrid);
}

// A pointer the whole wave holds, in scalar registers (function arguments
// arrive in vector registers; loads through a scalar base are scalar loads).
template <typename T>
__device__ inline T* pq_uniform(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// One matcher call per function, each compiled (and register-allocated) on
// its own: ranges g_pq_act[s0 ..] (g_pq_n of them) of level tab[idx].
template <int B, int MODE>
__device__ __noinline__ void pq_valu(const Lvl* __restrict__ tab, int idx, int s0) {
    constexpr int TN = B == 16 ? kPqTn16 : MatchTile<B>::TN;
    const Lvl& a = pq_uniform(tab)[__builtin_amdgcn_readfirstlane(idx)];
    MatchSmem<B, MODE, TN>* sm = reinterpret_cast<MatchSmem<B, MODE, TN>*>(&g_pq_u);
    k_match_body<B, MODE, TN>(*sm, 0, 0, a.img, a.pitch, g_pq_act + __builtin_amdgcn_readfirstlane(s0), &g_pq_n,
                          a.hl, a.sd, a.ad, a.jd, a.pctrl, a.ks, 1, g_pq_part, g_pq_sr, g_pq_cr, 1 << 30);
}

template <int B, int NK>
__device__ __noinline__ void pq_mfq(const Lvl* __restrict__ tab, int idx, int s0) {
    constexpr int COLS = B == 16 ? kPqCols16 : mq_cols(B);
    const Lvl& a = pq_uniform(tab)[__builtin_amdgcn_readfirstlane(idx)];
    MqSmem<B, NK, COLS>* sm = reinterpret_cast<MqSmem<B, NK, COLS>*>(&g_pq_u);
    k_match_mfq_body<B, NK, COLS>(*sm, 0, 0, a.img, a.pitch, g_pq_act + __builtin_amdgcn_readfirstlane(s0), &g_pq_n,
                            reinterpret_cast<const _Float16*>(a.dh), a.sd, a.ad, a.jd, a.pctrl, a.ks, 1, 1 << 30,
                            g_pq_part, g_pq_sr, g_pq_cr);
}

// Best (F, key) of each of the g_pq_n ranges at g_pq_act + s0 over the level's whole pool.
__device__ __forceinline__ void pq_match(int B, int kind, const Lvl* tab, int idx, int s0) {
    switch (B * 8 + kind) {
        case 2 * 8 + kPqValuSmall: pq_valu<2, kModeSmall>(tab, idx, s0); break;
        case 2 * 8 + kPqValuGrid: pq_valu<2, kModeGrid>(tab, idx, s0); break;
        case 2 * 8 + kPqValuList: pq_valu<2, kModeList>(tab, idx, s0); break;
        case 4 * 8 + kPqValuSmall: pq_valu<4, kModeSmall>(tab, idx, s0); break;
        case 4 * 8 + kPqValuGrid: pq_valu<4, kModeGrid>(tab, idx, s0); break;
        case 4 * 8 + kPqValuList: pq_valu<4, kModeList>(tab, idx, s0); break;
        case 8 * 8 + kPqValuSmall: pq_valu<8, kModeSmall>(tab, idx, s0); break;
        case 8 * 8 + kPqValuGrid: pq_valu<8, kModeGrid>(tab, idx, s0); break;
        case 8 * 8 + kPqValuList: pq_valu<8, kModeList>(tab, idx, s0); break;
        case 16 * 8 + kPqValuSmall: pq_valu<16, kModeSmall>(tab, idx, s0); break;
        case 16 * 8 + kPqValuGrid: pq_valu<16, kModeGrid>(tab, idx, s0); break;
        case 16 * 8 + kPqValuList: pq_valu<16, kModeList>(tab, idx, s0); break;
        case 4 * 8 + kPqMfq1: pq_mfq<4, 1>(tab, idx, s0); break;
        case 4 * 8 + kPqMfq2: pq_mfq<4, 2>(tab, idx, s0); break;
        case 8 * 8 + kPqMfq1: pq_mfq<8, 1>(tab, idx, s0); break;
        case 8 * 8 + kPqMfq2: pq_mfq<8, 2>(tab, idx, s0); break;
        case 16 * 8 + kPqMfq1: pq_mfq<16, 1>(tab, idx, s0); break;
        default: pq_mfq<16, 2>(tab, idx, s0); break;
    }
}

// The per-run reset: a new epoch, empty queues, level 0 of every image open
// with all its ranges pending, deeper levels closed (kPqOpen) until their
// parents finish.
__global__ __launch_bounds__(kBlock) void kt_pq_reset(const Lvl* __restrict__ tab, PqArgs pa) {
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g == 0) {
        pa.ctl->epoch += 1;
        pa.ctl->ghead = 0;
        pa.ctl->gtail = 0;
        pa.ctl->done = 0;
        pa.ctl->err = 0;
    }
    if (g < pa.n_img * 4) {
        const int i = g >> 2, l = g & 3;
        const Lvl& a = tab[i];
        pa.enq[g] = 0;
        pa.rem[g] = l == 0 ? (a.H / a.B) * (a.W / a.B) : kPqOpen;
    }
    for (int t = g; t < pa.T; t += gridDim.x * kBlock) pa.fill[t] = 0;
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(FIC_PQ_WAVES, 8))) void kt_pq(const Lvl* __restrict__ tab, PqArgs pa) {
    int32_t* const sAct = g_pq_act;
    int32_t* const sZ = g_pq_z;
    Partial* const sPart = g_pq_part;
    int32_t* const sSR = g_pq_sr;
    int64_t* const sCR = g_pq_cr;
    uint8_t* const sSplit = g_pq_split;
    __shared__ int32_t sTask[4];
    const uint32_t epoch = pa.ctl->epoch;
    const int nl = pa.n_levels, n_img = pa.n_img;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (;;) {
        // claim the next tile (thread 0), or stop when every image has finished
        if (threadIdx.x == 0) {
            const int h = pq_add(&pa.ctl->ghead, 1);
            int tau = -1;
            if (h < pa.T0) {
                tau = h;
            } else if (h - pa.T0 < pa.gq_cap) {
                const uint64_t* slot = pa.gq + (h - pa.T0);
                for (int spins = 0;; ++spins) {
                    const uint64_t v = pq_load(slot);
                    if ((uint32_t)(v >> 32) == epoch) {
                        tau = (int)(uint32_t)v;
                        break;
                    }
                    if (pq_load32(&pa.ctl->done) >= n_img) {
                        const uint64_t w = pq_load(slot);
                        if ((uint32_t)(w >> 32) == epoch) tau = (int)(uint32_t)w;
                        break;
                    }
                    if (pq_load32(&pa.ctl->err) != 0) break;
                    if (spins >= kPqSpinLimit) {
                        pq_add(&pa.ctl->err, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
            }
            sTask[0] = tau;
            if (tau >= 0) {
                const int idx = pq_find(pa.tile_base, nl * n_img, tau);
                const int l = idx / n_img, i = idx % n_img;
                const Lvl& a = tab[idx];
                const int start = (tau - pa.tile_base[idx]) * pa.R[l];
                const int total = l == 0 ? (a.H / a.B) * (a.W / a.B) : pq_load32(&pa.enq[i * 4 + l]);
                sTask[1] = idx;
                sTask[2] = start;
                sTask[3] = min(pa.R[l], total - start);
            }
        }
        __syncthreads();
        // the task is the same for the whole workgroup: scalar registers
        const int tau = __builtin_amdgcn_readfirstlane(sTask[0]);
        if (tau < 0) return;
        const int idx = __builtin_amdgcn_readfirstlane(sTask[1]);
        const int start = __builtin_amdgcn_readfirstlane(sTask[2]);
        const int cnt = __builtin_amdgcn_readfirstlane(sTask[3]);
        const int l = idx / n_img, i = idx % n_img;
        const Lvl& a = tab[idx];
        const int B = a.B, kind = pa.kind[l];
        const int gx0 = tab[i].W / pa.B0;
        const int64_t sb = pa.slot_base[idx];
        // the tile's ranges: slots and packed corners
        for (int k = threadIdx.x; k < cnt; k += kBlock) {
            int z;
            if (l == 0) {
                z = start + k;
            } else {
                const uint64_t* e = pa.qe + sb + start + k;
                uint64_t v = pq_load(e);
                for (int spins = 0; (uint32_t)(v >> 32) != epoch; ++spins) {
                    if (spins >= kPqSpinLimit) {
                        pq_add(&pa.ctl->err, 1);
                        v = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    v = pq_load(e);
                }
                z = (int)(uint32_t)v;
            }
            sZ[k] = z;
            sAct[k] = pq_yx(z, l, gx0, pa.B0);
        }
        __syncthreads();
        const int per = pq_block_ranges(B, kind);
        for (int s0 = 0; s0 < cnt; s0 += per) {
            const int nsub = min(per, cnt - s0);
            if (threadIdx.x == 0) g_pq_n = nsub;
            __syncthreads();
            pq_match(B, kind, tab, idx, s0);
            __syncthreads();
            if (wave == 0 && lane < nsub) {
                // the decision of each range (one per lane) and its result
                const int z = sZ[s0 + lane];
                fic_match m;
                int dy, dx;
                const Partial pr = sPart[lane];
                finish_best(sAct[s0 + lane], B, a.L, a.gx, pr.F, pr.key, sCR[lane], sSR[lane], a.ks, m, dy, dx);
                const bool keep = a.last || m.e_num <= a.thr;
                PqRec r;
                r.e_num = m.e_num;
                r.dom = m.dom;
                r.q_o = m.q_o;
                r.iso_s = (uint8_t)(m.iso | (m.s_idx << 3));
                r.pad = 0;
                pa.rec[sb + z] = r;
                pa.state[sb + z] = keep ? 1 : 0;
                sSplit[s0 + lane] = keep ? 0 : 1;
            }
            __syncthreads();
        }
        // commit the tile: the children of its split ranges, then the counters
        int my = 0;
#pragma unroll
        for (int u = 0; u < kPqMaxTile / kBlock; ++u) {
            const int k = threadIdx.x * (kPqMaxTile / kBlock) + u;
            my += (k < cnt && sSplit[k]) ? 1 : 0;
        }
        int before, e1, splits, t1;
        block_scan2(my, 0, before, e1, splits, t1);
        if (splits > 0) {
            if (threadIdx.x == 0) {
                // the reservation and the next level's pending count, both performed before
                // this level's count is lowered below
                const int base = pq_add(&pa.enq[i * 4 + l + 1], 4 * splits);
                pq_add(&pa.rem[i * 4 + l + 1], 4 * splits);
                sTask[0] = base;
                pq_wait_memory();
            }
            __syncthreads();
            const int64_t sbn = pa.slot_base[idx + n_img];
            uint64_t* e = pa.qe + sbn + sTask[0] + 4 * before;
#pragma unroll
            for (int u = 0; u < kPqMaxTile / kBlock; ++u) {
                const int k = threadIdx.x * (kPqMaxTile / kBlock) + u;
                if (k < cnt && sSplit[k]) {
                    const int z = sZ[k];
#pragma unroll
                    for (int c = 0; c < 4; ++c) pq_store(e + c, ((uint64_t)epoch << 32) | (uint32_t)(4 * z + c));
                    e += 4;
                }
            }
        }
        if (threadIdx.x == 0) {
            if (splits > 0) {
                // entries per tile of the next level; a tile that fills is pushed
                const int base = sTask[0];
                const int Rn = pa.R[l + 1], tb = pa.tile_base[idx + n_img];
                for (int p = base, end = base + 4 * splits; p < end;) {
                    const int t = p / Rn, te = min(end, (t + 1) * Rn), add = te - p;
                    if (pq_add(&pa.fill[tb + t], add) + add == Rn) pq_push(pa, epoch, tb + t);
                    p = te;
                }
                pq_wait_memory();  // pushes visible before the count that may end the run
            }
            int left = pq_add(&pa.rem[i * 4 + l], -cnt) - cnt;
            // finished levels: push the next level's partial tile, close it, go on down
            int lv = l;
            while (left == 0) {
                if (lv + 1 >= nl) {
                    pq_add(&pa.ctl->done, 1);
                    break;
                }
                const int nidx = (lv + 1) * n_img + i;
                const int en = pq_load32(&pa.enq[i * 4 + lv + 1]);
                const int Rn = pa.R[lv + 1];
                if (en % Rn != 0) pq_push(pa, epoch, pa.tile_base[nidx] + en / Rn);
                pq_wait_memory();
                left = pq_add(&pa.rem[i * 4 + lv + 1], -kPqOpen) - kPqOpen;
                ++lv;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- ordered compaction of the results
// A slot is active iff every ancestor was split in this run (level 0: all).
__device__ inline bool pq_active(const PqArgs& pa, int i, int l, int z) {
    for (int k = 0; k < l; ++k)
        if (pa.state[pa.slot_base[k * pa.n_img + i] + (z >> (2 * (l - k)))] != 0) return false;
    return true;
}

// Per compaction block: (leaves, active ranges) among its slots.
__global__ __launch_bounds__(kBlock) void kt_pq_count(const Lvl* __restrict__ tab, PqArgs pa,
                                                       const int32_t* __restrict__ blk_seg,
                                                       const int32_t* __restrict__ blk_z0, int2* blkc) {
    const int b = blockIdx.x, seg = blk_seg[b];
    const int l = seg / pa.n_img, i = seg % pa.n_img;
    const Lvl& a = tab[seg];
    const int N = (a.H / a.B) * (a.W / a.B);
    const int64_t sb = pa.slot_base[seg];
    int leaves = 0, act = 0;
    const int z0 = blk_z0[b] + threadIdx.x * kPqEmitItems;
#pragma unroll
    for (int u = 0; u < kPqEmitItems; ++u) {
        const int z = z0 + u;
        if (z < N && pq_active(pa, i, l, z)) {
            ++act;
            leaves += (a.last || pa.state[sb + z] == 1) ? 1 : 0;
        }
    }
    int e0, e1, t0, t1;
    block_scan2(leaves, act, e0, e1, t0, t1);
    if (threadIdx.x == 0) blkc[b] = make_int2(t0, t1);
}

// One workgroup per image: code offsets of its blocks (levels in order, slot
// order within a level), the per-level statistics and the code count.
__global__ __launch_bounds__(kBlock) void kt_pq_scan(const Lvl* __restrict__ tab, PqArgs pa,
                                                      const int32_t* __restrict__ blk_first,
                                                      const int2* __restrict__ blkc, int32_t* blko,
                                                      const int32_t* __restrict__ orig, int32_t* n_codes) {
    const int i = blockIdx.x, nl = pa.n_levels;
    int running = 0;
    for (int l = 0; l < nl; ++l) {
        const int seg = l * pa.n_img + i;
        const int b0 = blk_first[seg], b1 = blk_first[seg + 1];
        int lvl_leaves = 0, lvl_act = 0;
        for (int c = b0; c < b1; c += kBlock) {
            const int b = c + threadIdx.x;
            const int2 v = b < b1 ? blkc[b] : make_int2(0, 0);
            int e0, e1, t0, t1;
            block_scan2(v.x, v.y, e0, e1, t0, t1);
            if (b < b1) blko[b] = running + lvl_leaves + e0;
            lvl_leaves += t0;
            lvl_act += t1;
            __syncthreads();
        }
        const Lvl& a = tab[seg];
        if (threadIdx.x == 0 && a.stats) {
            fic_level_stats st;
            const int pool = a.pctrl->pool_count;
            st.matches = (int64_t)lvl_act * pool * 8;
            st.pool = pool;
            st.passed = a.pctrl->passed;
            st.active = lvl_act;
            st.accepted = lvl_leaves;
            a.stats[l] = st;
        }
        running += lvl_leaves;
    }
    if (threadIdx.x == 0) {
        // a run whose waits gave up reports -1 codes (its results are void)
        const int total = pa.ctl->err != 0 ? -1 : running;
        tab[i].ctrl->n_codes = total;
        if (n_codes) n_codes[orig ? orig[i] : i] = total;
    }
}

// The codes: each leaf's record expanded at its place.
__global__ __launch_bounds__(kBlock) void kt_pq_scatter(const Lvl* __restrict__ tab, PqArgs pa,
                                                         const int32_t* __restrict__ blk_seg,
                                                         const int32_t* __restrict__ blk_z0,
                                                         const int32_t* __restrict__ blko) {
    const int b = blockIdx.x, seg = blk_seg[b];
    const int l = seg / pa.n_img, i = seg % pa.n_img;
    const Lvl& a = tab[seg];
    const int N = (a.H / a.B) * (a.W / a.B);
    const int64_t sb = pa.slot_base[seg];
    const int gx0 = tab[i].W / pa.B0;
    const int z0 = blk_z0[b] + threadIdx.x * kPqEmitItems;
    bool leaf[kPqEmitItems];
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < kPqEmitItems; ++u) {
        const int z = z0 + u;
        leaf[u] = z < N && pq_active(pa, i, l, z) && (a.last || pa.state[sb + z] == 1);
        cnt += leaf[u] ? 1 : 0;
    }
    int e0, e1, t0, t1;
    block_scan2(cnt, 0, e0, e1, t0, t1);
    int pos = blko[b] + e0;
    const int log2B = 31 - __clz(a.B);
#pragma unroll
    for (int u = 0; u < kPqEmitItems; ++u) {
        if (!leaf[u]) continue;
        const int z = z0 + u;
        if (pos < a.capacity) {
            const PqRec r = pa.rec[sb + z];
            const int yx = pq_yx(z, l, gx0, pa.B0);
            const int j = r.dom, s_idx = r.iso_s >> 3;
            const uint64_t w0 = (uint64_t)r.e_num;
            const uint64_t w1 = (uint64_t)(uint32_t)j | ((uint64_t)(uint32_t)(yx >> 16) << 32) |
                                ((uint64_t)(yx & 0xffff) << 48);
            const uint64_t w2 = (uint64_t)(uint16_t)((j / a.gx) * a.L) | ((uint64_t)(uint16_t)((j % a.gx) * a.L) << 16) |
                                ((uint64_t)(uint16_t)r.q_o << 32) | ((uint64_t)log2B << 48) |
                                ((uint64_t)(r.iso_s & 7) << 56);
            const uint64_t w3 = (uint64_t)kset_value(a.ks, s_idx) | ((uint64_t)s_idx << 8) | ((uint64_t)l << 16);
            uint64_t* dst = reinterpret_cast<uint64_t*>(a.codes + pos);
            dst[0] = w0;
            dst[1] = w1;
            dst[2] = w2;
            dst[3] = w3;
        }
        ++pos;
    }
}

}  // namespace fic
