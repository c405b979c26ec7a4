// Device kernels of libfic: exhaustive range-domain matching for fractal
// image encoding on gfx950 (CDNA4, 64-wide wavefronts).
//
// The hot loop correlates every range row (a range block under one of the 8
// isometries) with every domain of the pool (Section 2). Each thread owns one
// range row held in registers as packed bytes. Each workgroup stages a tile of
// decimated domains in LDS; every lane of a wave reads the same domain, so the
// LDS reads are broadcasts. The 2x2 sums (0..1020) are split into a high byte
// and a low byte, so each inner product is two v_dot4_u32_u8 chains per 4
// pixels, exact in 32 bits. The distance is decided in exact 64-bit integers:
//   16 Q^2 n E(k) = k^2 A' - 8 Q k B' + 16 Q^2 C     (Q = 10, s = k/Q)
// with A' = n sum d'^2 - (sum d')^2, B' = n <r, d'> - sum r sum d',
// C = n sum r^2 - (sum r)^2 and d' = 4 d, the integer 2x2 sum. This is eq. (1)
// with o from eq. (3) expanded in the moments of R and D.
#include <limits>
#include <type_traits>

#include "fic_internal.h"

namespace fic {

// ---------------------------------------------------------------- isometries
// T_t(D)[i][c] = D[iso_src(B, t, i, c)]; t=1 is 90 degrees clockwise, t=2 180,
// t=3 270, t=4+u the left-right mirror of t=u (Section 2).
__host__ __device__ inline int iso_src(int B, int t, int i, int c) {
    if (t >= 4) {
        c = B - 1 - c;
        t -= 4;
    }
    switch (t) {
        case 0: return i * B + c;
        case 1: return (B - 1 - c) * B + i;
        case 2: return (B - 1 - i) * B + (B - 1 - c);
        default: return c * B + (B - 1 - i);
    }
}

// Isometry u with T_u o T_t = identity: rotations invert, mirrors are involutions.
__host__ __device__ inline int iso_inverse(int t) { return t == 1 ? 3 : (t == 3 ? 1 : t); }

__device__ inline int64_t floordiv64(int64_t a, int64_t b) {  // b > 0
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

__device__ inline int floordiv32(int a, int b) {  // b > 0
    const int q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

// ---------------------------------------------------------------- active range lists
// Packed corner: (y << 16) | x. Block 0 also sets the level's active count
// and, when asked, clears the code counter of a new quadtree.
__device__ __forceinline__ void k_act_full_body(int32_t* act, int gy, int gx, int B, Ctrl* ctrl, int lv, int reset) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        ctrl->act_count[lv] = gy * gx;
        if (reset) {
            ctrl->n_codes = 0;
            ctrl->lvl_base[lv] = 0;
        }
    }
    if (q >= gy * gx) return;
    int ry = q / gx, rx = q - ry * gx;
    act[q] = ((ry * B) << 16) | (rx * B);
}

// Caller-supplied corners; an invalid corner is stored as -1.
__device__ __forceinline__ void k_act_from_yx_body(int32_t* act, const int32_t* yx, int n, int H, int W, int B,
                              Ctrl* ctrl) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) ctrl->act_count[0] = n;
    if (q >= n) return;
    int y = yx[2 * q], x = yx[2 * q + 1];
    bool ok = y >= 0 && x >= 0 && y + B <= H && x + B <= W && (y % B) == 0 && (x % B) == 0;
    act[q] = ok ? ((y << 16) | x) : -1;
}

// ---------------------------------------------------------------- entropy score (Section 3)
// key[j] = sum_b T[c_b] over the 8-bin (p >> 5) histogram of the 2B x 2B
// domain j, where T[c] = round(c log2 c * 2^32). Entropy in bits is
// log2 Nw - key / (Nw 2^32), so the domain passes iff key < M.
// TPD lanes of one wavefront share a domain; each lane counts 16 pixels into
// eight 8-bit counters packed in a 64-bit word. ctrl->pass_count accumulates
// the domains that pass (k_floor_select clears it after the pool is built).
template <int SIDE>
struct ScoreShape {
    static constexpr int NPIX = SIDE * SIDE;
    static constexpr int PER = 16;  // pixels per lane
    static constexpr int TPD = NPIX / PER;
};

template <int SIDE>
__device__ __forceinline__ void k_pool_score_body(const uint8_t* __restrict__ img, int pitch,
                                                       int L, int gx, int total,
                                                       const int64_t* __restrict__ T, int64_t M,
                                                       int64_t* __restrict__ key, Ctrl* ctrl) {
    using S = ScoreShape<SIDE>;
    constexpr int TPD = S::TPD, PER = S::PER;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = g / TPD, sub = g % TPD;
    const bool ok = j < total;
    uint64_t acc = 0;
    if (ok) {
        const int y = (j / gx) * L, x = (j % gx) * L;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int m = sub * PER + q;
            const int i = m / SIDE, c = m % SIDE;
            const uint32_t b = img[(int64_t)(y + i) * pitch + x + c] >> 5;
            acc += 1ull << (8 * b);
        }
    }
    // widen to 16-bit counters (4 bins per word) and add over the domain's lanes
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        lo |= ((acc >> (8 * b)) & 0xffull) << (16 * b);
        hi |= ((acc >> (8 * (b + 4))) & 0xffull) << (16 * b);
    }
#pragma unroll
    for (int m = 1; m < TPD; m <<= 1) {
        lo += __shfl_xor(lo, m, 64);
        hi += __shfl_xor(hi, m, 64);
    }
    int pass = 0;
    if (ok && sub == 0) {
        int64_t s = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            s += T[(lo >> (16 * b)) & 0xffff];
            s += T[(hi >> (16 * b)) & 0xffff];
        }
        key[j] = s;
        pass = s < M;
    }
    int cnt = __syncthreads_count(pass);
    if (threadIdx.x == 0 && cnt) atomicAdd(&ctrl->pass_count, cnt);
}

// The same keys by cells. With stride L and side 4L, domain (dy, dx) is the
// 4 x 4 block of L x L cells starting at cell (dy, dx). A workgroup scores a
// tile of kScTY x TX domains (TX = sc_tx(L)) from the histograms of the
// (kScTY + 3) x (TX + 3) cells they cover: a wave reads 64 consecutive pixels of a row
// (L lanes per cell, 8-bit counters over the cell's L rows), cells are widened
// to 16-bit counters, summed 4 at a time along x, then 4 rows at a time along y.
// Each cell is read once per tile instead of once per domain that covers it.
constexpr int kScTY = 4;
// Tile width at cell side L: 16 domains at L = 8 (the coarsest level has few
// domains, so narrower tiles give it more workgroups and each fewer cells),
// else 64. Threads beyond the tile's domains only help load the cells.
__host__ __device__ constexpr int sc_tx(int L) { return L == 8 ? 16 : 64; }
static_assert(kScTY * 64 == kBlock, "one thread per domain of the widest tile");

// LDS of the cell kernel at cell side L.
template <int L>
struct CellSmem {
    static constexpr int TX = sc_tx(L);
    static constexpr int CX = TX + 3, CY = kScTY + 3;  // cells of the tile
    uint64_t sc[CY * CX * 2];                           // cells: bins 0-3 | bins 4-7, 16 bits each
    uint64_t sh[CY * TX * 2];                           // sums of 4 cells along x
    int64_t sT[16 * L * L + 1];                            // the entropy table up to a domain's pixels
};
union CellSmemAny {
    CellSmem<1> l1;
    CellSmem<2> l2;
    CellSmem<4> l4;
    CellSmem<8> l8;
};

// Tile (tbx, tby) of the level's domain grid.
template <int L>
__device__ __forceinline__ void k_pool_score_cells_body(CellSmem<L>& sm, int tbx, int tby,
                                                             const uint8_t* __restrict__ img, int pitch,
                                                             int gx, int gy,
                                                             const int64_t* __restrict__ T, int64_t M,
                                                             int64_t* __restrict__ key, Ctrl* ctrl) {
    constexpr int CX = CellSmem<L>::CX, CY = CellSmem<L>::CY;
    constexpr int NPIX = 16 * L * L;               // pixels of a domain
    constexpr int CPW = 64 / L;                    // cells across a wave's 64 pixels
    constexpr int XCH = (CX + CPW - 1) / CPW;      // wave chunks per row of cells
    constexpr int NCH = CY * XCH;
    uint64_t* const sc = sm.sc;
    uint64_t* const sh = sm.sh;
    int64_t* const sT = sm.sT;
    constexpr int TX = CellSmem<L>::TX;
    const int dx0 = tbx * TX, dy0 = tby * kScTY;
    if (dx0 >= gx || dy0 >= gy) return;
    for (int i = threadIdx.x; i <= NPIX; i += kBlock) sT[i] = T[i];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // kChunks chunks per wave at a time, their loads all in flight. Cells
    // (cy, cx) with cy < gy + 3 and cx < gx + 3 lie inside the image ((gy + 3) L
    // = H), so a chunk's addresses are clamped to such a cell and every load is
    // issued; cells outside the tile or the grid count zero.
    constexpr int kChunks = 4, NWV = kBlock / 64;
    for (int t0 = wid; t0 < NCH; t0 += kChunks * NWV) {
        uint32_t v[kChunks][L];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int t = t0 + c * NWV;
            const int cr = t / XCH, lc = (t % XCH) * CPW + lane / L;
            const int cy = min(dy0 + cr, gy + 2), cx = min(dx0 + lc, gx + 2);
            const uint8_t* p = img + (int64_t)cy * L * pitch + (int64_t)cx * L + lane % L;
#pragma unroll
            for (int r = 0; r < L; ++r) v[c][r] = p[(int64_t)r * pitch];
        }
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int t = t0 + c * NWV;
            const int cr = t / XCH, lc = (t % XCH) * CPW + lane / L;
            const int cy = dy0 + cr, cx = dx0 + lc;
            uint64_t acc = 0;
#pragma unroll
            for (int r = 0; r < L; ++r) acc += 1ull << (8 * (v[c][r] >> 5));
            if (!(t < NCH && lc < CX && cy < gy + 3 && cx < gx + 3)) acc = 0;
#pragma unroll
            for (int m = 1; m < L; m <<= 1) acc += __shfl_xor(acc, m, 64);
            if (t < NCH && lane % L == 0 && lc < CX) {
                uint64_t lo = 0, hi = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    lo |= ((acc >> (8 * b)) & 0xffull) << (16 * b);
                    hi |= ((acc >> (8 * (b + 4))) & 0xffull) << (16 * b);
                }
                sc[(cr * CX + lc) * 2] = lo;
                sc[(cr * CX + lc) * 2 + 1] = hi;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < CY * TX; i += kBlock) {
        const int r = i / TX, c = i % TX;
        uint64_t lo = 0, hi = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lo += sc[(r * CX + c + k) * 2];
            hi += sc[(r * CX + c + k) * 2 + 1];
        }
        sh[i * 2] = lo;
        sh[i * 2 + 1] = hi;
    }
    __syncthreads();
    const int ty = threadIdx.x / TX, tx = threadIdx.x % TX;
    const int dy = dy0 + ty, dx = dx0 + tx;
    int pass = 0;
    if (ty < kScTY && dy < gy && dx < gx) {
        uint64_t lo = 0, hi = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lo += sh[((ty + k) * TX + tx) * 2];
            hi += sh[((ty + k) * TX + tx) * 2 + 1];
        }
        int64_t s = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            s += sT[(lo >> (16 * b)) & 0xffff];
            s += sT[(hi >> (16 * b)) & 0xffff];
        }
        key[(int64_t)dy * gx + dx] = s;
        pass = s < M;
    }
    const int cnt = __syncthreads_count(pass);
    if (threadIdx.x == 0 && cnt) atomicAdd(&ctrl->pass_count, cnt);
}

// Variance filter (an alternative to the entropy filter of Section 3): key[j]
// = kv - V' with V' = N sum p^2 - (sum p)^2 over the N = SIDE^2 pixels of the
// domain (N^2 times its variance, exact), so smaller keys mean higher variance
// and the floor keeps the highest-variance domains. Passes iff key < M.
template <int SIDE>
__device__ __forceinline__ void k_pool_var_body(const uint8_t* __restrict__ img, int pitch, int L,
                                                int gx, int total, int64_t kv, int64_t M,
                                                int64_t* __restrict__ key, Ctrl* ctrl) {
    using S = ScoreShape<SIDE>;
    constexpr int TPD = S::TPD, PER = S::PER;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = g / TPD, sub = g % TPD;
    const bool ok = j < total;
    int s1 = 0, s2 = 0;
    if (ok) {
        const int y = (j / gx) * L, x = (j % gx) * L;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int m = sub * PER + q;
            const int v = img[(int64_t)(y + m / SIDE) * pitch + x + m % SIDE];
            s1 += v;
            s2 += v * v;
        }
    }
#pragma unroll
    for (int m = 1; m < TPD; m <<= 1) {
        s1 += __shfl_xor(s1, m, 64);
        s2 += __shfl_xor(s2, m, 64);
    }
    int pass = 0;
    if (ok && sub == 0) {
        const int64_t vp = (int64_t)S::NPIX * s2 - (int64_t)s1 * s1;
        const int64_t k = kv - vp;
        key[j] = k;
        pass = k < M;
    }
    int cnt = __syncthreads_count(pass);
    if (threadIdx.x == 0 && cnt) atomicAdd(&ctrl->pass_count, cnt);
}

// Pool mode for a level: 0 = threshold passers, 1 = floor (lowest keys), 2 = all.
__device__ inline int pool_mode(int passed, int total, int min_pool) {
    if (total <= min_pool) return 2;
    return passed >= min_pool ? 0 : 1;
}

// Calls f(i, key[i]) for i = i0 + t, i0 + t + nt, ... below i1 (t = this
// thread's index among nt), issuing KLD loads before the first call, so that a
// thread waits for one load latency per KLD keys instead of one per key.
template <int KLD, typename F>
__device__ __forceinline__ void for_each_key(const int64_t* __restrict__ key, int i0, int i1, int t,
                                             int nt, F f) {
    for (int b = i0 + t; b < i1; b += KLD * nt) {
        uint64_t v[KLD];
#pragma unroll
        for (int u = 0; u < KLD; ++u) {
            const int i = b + u * nt;
            v[u] = i < i1 ? (uint64_t)key[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < KLD; ++u)
            if (b + u * nt < i1) f(b + u * nt, v[u]);
    }
}

// Floor, step 1. Workgroup b takes keys [b*chunk, (b+1)*chunk) and finds the
// bucket of key >> shift (shift puts every key below 2^(shift+12)) holding its
// own r-th smallest key. The chunk alone has r keys not above that bucket's
// largest key, so the global r-th smallest key is not above it either.
__device__ __forceinline__ void k_floor_bound_body(const int64_t* __restrict__ key, int total,
                                                        int min_pool, int r, int shift, int chunk,
                                                        Ctrl* ctrl) {
    if (pool_mode(ctrl->pass_count, total, min_pool) != 1) return;
    const int lo = blockIdx.x * chunk, hi = min(total, lo + chunk);
    if (hi - lo < r) return;
    __shared__ uint32_t h[kSelBins];
    __shared__ uint32_t part[kBlock];
    __shared__ int s_t;
    __shared__ uint32_t s_cum;
    for (int i = threadIdx.x; i < kSelBins; i += kBlock) h[i] = 0u;
    if (threadIdx.x == 0) {
        s_t = 0;
        s_cum = 0;
    }
    __syncthreads();
    for_each_key<8>(key, lo, hi, threadIdx.x, kBlock, [&](int, uint64_t u) {
        atomicAdd(&h[min(u >> shift, (uint64_t)(kSelBins - 1))], 1u);
    });
    __syncthreads();
    constexpr int per = kSelBins / kBlock;
    uint32_t mine = 0;
    for (int b = 0; b < per; ++b) mine += h[threadIdx.x * per + b];
    part[threadIdx.x] = mine;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        uint32_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    const uint32_t incl = part[threadIdx.x], excl = incl - mine;
    if (excl < (uint32_t)r && (uint32_t)r <= incl) {
        s_t = threadIdx.x;
        s_cum = excl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t cum = s_cum;
        int b = s_t * per;
        for (; b < s_t * per + per - 1; ++b) {
            if (cum + h[b] >= (uint32_t)r) break;
            cum += h[b];
        }
        const unsigned long long bound = (((unsigned long long)b + 1) << shift) - 1;
        atomicMin(reinterpret_cast<unsigned long long*>(&ctrl->cut_bound), bound);
    }
}

// ---------------------------------------------------------------- order-preserving compaction
// Two flags per item (f0, f1). Pool: f0 = domain kept (threshold mode), a
// floor candidate (key <= bound) or any domain (all mode). Quadtree: f0 =
// range kept, f1 = range split.
struct CompactArgs {
    int kind;  // 0 pool, 1 quadtree
    int total;
    int min_pool;
    int64_t M;
    const int64_t* key;
    const int32_t* act_count;  // quadtree: number of items
    const uint8_t* decision;   // quadtree: 1 kept, 0 split, 2 invalid
};

constexpr int kPoolItems = 8;   // domains per thread in the pool compaction
constexpr int kQuadItems = 4;   // ranges per thread in the quadtree compaction
constexpr int kRqLanes = 4;     // lanes per range in the quadtree decision step
constexpr int kRqRanges = kBlock / kRqLanes;  // ranges per workgroup of that step

__device__ inline void item_flags(const CompactArgs& a, const Ctrl* ctrl, int mode, int i, int& f0,
                                  int& f1) {
    f0 = 0;
    f1 = 0;
    if (a.kind == 0) {
        if (i >= a.total) return;
        const int64_t k = a.key[i];
        if (mode == 2) f0 = 1;
        else if (mode == 0) f0 = k < a.M;
        else f0 = (uint64_t)k <= ctrl->cut_bound;
    } else {
        if (i >= *a.act_count) return;
        const uint8_t d = a.decision[i];
        f0 = d == 1;
        f1 = d == 0;
    }
}

// Exclusive scan over a 256-thread block of two counters; also returns totals.
__device__ inline void block_scan2(int v0, int v1, int& e0, int& e1, int& t0, int& t1) {
    __shared__ int w0[kBlock / 64], w1[kBlock / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int s0 = v0, s1 = v1;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int a0 = __shfl_up(s0, d, 64), a1 = __shfl_up(s1, d, 64);
        if (lane >= d) {
            s0 += a0;
            s1 += a1;
        }
    }
    if (lane == 63) {
        w0[wid] = s0;
        w1[wid] = s1;
    }
    __syncthreads();
    int b0 = 0, b1 = 0;
    t0 = 0;
    t1 = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) {
            b0 += w0[w];
            b1 += w1[w];
        }
        t0 += w0[w];
        t1 += w1[w];
    }
    e0 = b0 + s0 - v0;
    e1 = b1 + s1 - v1;
    __syncthreads();
}

// Sums of the per-workgroup counts blk[0..n) over the whole workgroup: the
// offsets of the workgroup that follows them. Each thread issues its loads
// together. Every thread gets the sums.
__device__ inline int2 counts_before(const int2* blk, int n) {
    int s0 = 0, s1 = 0;
    for (int i = threadIdx.x; i < n; i += 4 * kBlock) {
        int2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = i + u * kBlock;
            v[u] = k < n ? blk[k] : make_int2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s0 += v[u].x;
            s1 += v[u].y;
        }
    }
    int e0, e1, t0, t1;
    block_scan2(s0, s1, e0, e1, t0, t1);
    return make_int2(t0, t1);
}

// Pool compaction. A workgroup covers kBlock * kPoolItems consecutive
// domains; thread t reads domains base + u * kBlock + t (u < kPoolItems), so
// every load of a wave is contiguous, and keeps the kept flags as a bit mask.
__device__ inline uint32_t pool_flag_bits(const CompactArgs& a, const Ctrl* ctrl, int mode, int base) {
    const uint64_t cut = ctrl->cut_bound;
    uint32_t bits = 0;
#pragma unroll 8
    for (int u = 0; u < kPoolItems; ++u) {
        const int i = base + u * kBlock + (int)threadIdx.x;
        int f = 0;
        if (i < a.total) {
            if (mode == 2) {
                f = 1;
            } else {
                const int64_t k = a.key[i];
                f = mode == 0 ? (k < a.M) : ((uint64_t)k <= cut);
            }
        }
        bits |= (uint32_t)f << u;
    }
    return bits;
}

// Pass 1: per-workgroup counts of kept domains.
__device__ __forceinline__ void k_pool_count_body(CompactArgs a, const Ctrl* ctrl, int2* blk) {
    const int mode = pool_mode(ctrl->pass_count, a.total, a.min_pool);
    const int base = blockIdx.x * kBlock * kPoolItems;
    const uint32_t bits = pool_flag_bits(a, ctrl, mode, base);
    int e0, e1, t0, t1;
    block_scan2(__popc(bits), 0, e0, e1, t0, t1);
    if (threadIdx.x == 0) blk[blockIdx.x] = make_int2(t0, 0);
}

// Pass 2: kept domains in ascending index order. Items are ordered (u, wave,
// lane); the per-(u, wave) counts come from wave ballots, the workgroup's
// offset from the counts of the workgroups before it. The last workgroup sets
// pool_count (the pool, or the floor candidates).
__device__ __forceinline__ void k_pool_scatter_body(CompactArgs a, Ctrl* ctrl, const int2* blk,
                                                         int nblk, int32_t* pool_out) {
    constexpr int NW = kBlock / 64;
    __shared__ int s_off[kPoolItems * NW + 1];
    const int boff = counts_before(blk, blockIdx.x).x;
    const int mode = pool_mode(ctrl->pass_count, a.total, a.min_pool);
    const int base = blockIdx.x * kBlock * kPoolItems;
    const uint32_t bits = pool_flag_bits(a, ctrl, mode, base);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll 8
    for (int u = 0; u < kPoolItems; ++u) {
        const uint64_t m = __ballot((bits >> u) & 1u);
        if (lane == 0) s_off[u * NW + wid] = __popcll(m);
    }
    __syncthreads();
    if (wid == 0) {  // exclusive scan of the kPoolItems * NW counts in (u, wave) order
        constexpr int NE = kPoolItems * NW;
        constexpr int PER = NE >= 64 ? NE / 64 : 1;
        static_assert(NE < 64 || NE % 64 == 0, "scan layout");
        int v[PER], sum = 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            v[e] = lane * PER + e < NE ? s_off[lane * PER + e] : 0;
            sum += v[e];
        }
        int incl = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(incl, d, 64);
            if (lane >= d) incl += t;
        }
        int run = incl - sum;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            if (lane * PER + e < NE) s_off[lane * PER + e] = run;
            run += v[e];
        }
        if (lane == 63) s_off[NE] = incl;  // the workgroup's total
    }
    __syncthreads();
    if ((int)blockIdx.x == nblk - 1 && threadIdx.x == 0) ctrl->pool_count = boff + s_off[kPoolItems * NW];
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll 8
    for (int u = 0; u < kPoolItems; ++u) {
        const bool f = (bits >> u) & 1u;
        const uint64_t m = __ballot(f);
        if (f) pool_out[boff + s_off[u * NW + wid] + __popcll(m & below)] = base + u * kBlock + threadIdx.x;
    }
}

// Exclusive scan of one int per thread over a 1024-thread workgroup (16
// waves); returns this thread's offset and sets the total. s_w: 16 ints of LDS.
__device__ inline int scan1024(int v, int* s_w, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int s = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(s, d, 64);
        if (lane >= d) s += t;
    }
    if (lane == 63) s_w[wid] = s;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const int x = s_w[w];
        base += w < wid ? x : 0;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return base + s - v;
}

// The same without the closing barrier: callers alternate between two s_w
// buffers, so a barrier of their own always separates two uses of one buffer.
__device__ inline int scan1024_open(int v, int* s_w, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int s = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(s, d, 64);
        if (lane >= d) s += t;
    }
    if (lane == 63) s_w[wid] = s;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const int x = s_w[w];
        base += w < wid ? x : 0;
        tot += x;
    }
    total = tot;
    return base + s - v;
}

constexpr int kSelStage = 8192;    // floor candidates (key and index) held in LDS by the select
constexpr int kSelDirect = 16384;  // grid domains the select takes directly (keys only in LDS)

// Floor, step 3 (one workgroup of 1024): exact radix select of the r-th
// smallest key among the C candidates (all keys <= cut_bound), then
// compaction to the keys below it plus the first ties in index order. The
// candidates are staged in LDS when they fit; the digits start at the highest
// bit a candidate can have, and the select stops as soon as the chosen bucket
// is taken whole. Staged candidates are compacted in one pass per wave over a
// contiguous segment (ballot ranks, 64 candidates a step), with one barrier
// for the waves' totals. Always launched: it also publishes the number of
// domains that passed the threshold and clears the per-level counters.
// direct (grids of at most kSelDirect domains, launched without the bound and
// compaction steps): every domain is a candidate (its index is its place, so
// only keys are staged), and the threshold and whole-grid pools are compacted
// here too.
__device__ __forceinline__ void k_floor_select_body(const int64_t* __restrict__ key, int total,
                                                       int min_pool, int r, int shift,
                                                       int32_t* __restrict__ pool, Ctrl* ctrl,
                                                       bool direct, int64_t M) {
    // staged keys; indices (non-direct candidates only) in the upper part
    __shared__ uint64_t sk[kSelDirect];
    int32_t* const sj = reinterpret_cast<int32_t*>(sk + kSelStage);
    static_assert(kSelStage * 12 <= kSelDirect * 8, "keys and indices share the stage");
    __shared__ uint32_t h[kSelBins];
    __shared__ int s_w[2][16];
    __shared__ int s_wl[16], s_wt[16];
    __shared__ uint64_t s_prefix;
    __shared__ uint32_t s_rank;
    __shared__ int s_lo, s_done, s_c0, s_c1;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
    const int passed = ctrl->pass_count;
    const int mode = pool_mode(passed, total, min_pool);
    const uint64_t below = (1ull << lane) - 1ull;
    if (direct && mode != 1) {
        // every domain (mode 2) or the threshold passers (mode 0), in index
        // order: wave w counts, then writes, its own contiguous segment
        const int S = (total + 15) / 16, wb = min(total, wid * S), we = min(total, wb + S);
        int cnt = 0;
        for (int i0 = wb; i0 < we; i0 += 64) {
            const int i = i0 + lane;
            cnt += __popcll(__ballot(i < we && (mode == 2 || key[i] < M)));
        }
        if (lane == 0) s_wl[wid] = cnt;
        __syncthreads();
        int off = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            off += w < wid ? s_wl[w] : 0;
            tot += s_wl[w];
        }
        for (int i0 = wb; i0 < we; i0 += 64) {
            const int i = i0 + lane;
            const bool f = i < we && (mode == 2 || key[i] < M);
            const uint64_t m = __ballot(f);
            if (f) pool[off + __popcll(m & below)] = i;
            off += __popcll(m);
        }
        if (tid == 0) ctrl->pool_count = tot;
    }
    if (mode == 1) {
        const int C = direct ? total : ctrl->pool_count;
        const bool staged = direct || C <= kSelStage;
        // The first digit's range is known before staging: every key of a
        // whole grid is below 2^(shift + kSelBits), every candidate is at most
        // cut_bound. So the first histogram is taken while staging.
        const uint64_t ub = direct ? (1ull << min(shift + kSelBits, 63)) - 1ull : ctrl->cut_bound;
        const int top = min(62, ub ? 63 - __clzll((long long)ub) : 0);
        {
            for (int i = tid; i < kSelBins; i += nt) h[i] = 0u;
            if (tid == 0) {
                s_prefix = 0;
                s_rank = (uint32_t)r;
                s_done = 0;
                s_lo = 0;
            }
            __syncthreads();
            const int p0 = top - (kSelBits - 1), lo0 = max(p0, 0), hs0 = p0 + kSelBits;
            const uint32_t dmask0 = (1u << (hs0 - lo0)) - 1u;
            const auto first_digit = [&](uint64_t u) {
                if ((u >> hs0) == 0) atomicAdd(&h[(uint32_t)(u >> lo0) & dmask0], 1u);
            };
            if (staged && direct) {
                for_each_key<8>(key, 0, C, tid, nt, [&](int i, uint64_t u) {
                    sk[i] = u;
                    first_digit(u);
                });
            } else if (staged) {
                // the candidates' indices first (8 loads in flight), then their keys
                constexpr int KLD = 8;
                for (int b = tid; b < C; b += KLD * nt) {
                    int j[KLD];
                    uint64_t v[KLD];
#pragma unroll
                    for (int u = 0; u < KLD; ++u) j[u] = b + u * nt < C ? pool[b + u * nt] : 0;
#pragma unroll
                    for (int u = 0; u < KLD; ++u) v[u] = b + u * nt < C ? (uint64_t)key[j[u]] : 0ull;
#pragma unroll
                    for (int u = 0; u < KLD; ++u)
                        if (b + u * nt < C) {
                            sj[b + u * nt] = j[u];
                            sk[b + u * nt] = v[u];
                            first_digit(v[u]);
                        }
                }
            }
            __syncthreads();
        }
        int par = 0;
        for (int p = top - (kSelBits - 1);; p -= kSelBits, par ^= 1) {
            const int lo = max(p, 0);
            const int hs = p + kSelBits;  // bits >= hs are already decided
            const uint32_t dmask = (1u << (hs - lo)) - 1u;
            const uint64_t prefix = s_prefix;
            if (staged && p == top - (kSelBits - 1)) {
                // first digit: histogram taken while staging
            } else if (staged) {
                // 4 LDS reads in flight per thread
                for (int b = tid; b < C; b += 4 * nt) {
                    uint64_t v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = b + u * nt < C ? sk[b + u * nt] : 0ull;
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (b + u * nt < C && (v[u] >> hs) == (prefix >> hs))
                            atomicAdd(&h[(uint32_t)(v[u] >> lo) & dmask], 1u);
                }
            } else {
                for (int i = tid; i < C; i += nt) {
                    const uint64_t u = (uint64_t)key[pool[i]];
                    if ((u >> hs) == (prefix >> hs)) atomicAdd(&h[(uint32_t)(u >> lo) & dmask], 1u);
                }
            }
            __syncthreads();
            const uint32_t rank = s_rank;
            uint32_t c4[4], mine = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                c4[b] = h[tid * 4 + b];
                mine += c4[b];
            }
            // only this thread reads these bins: clear them for the next digit
#pragma unroll
            for (int b = 0; b < 4; ++b) h[tid * 4 + b] = 0u;
            int tot;
            const uint32_t excl = (uint32_t)scan1024_open((int)mine, s_w[par], tot);
            if (excl < rank && rank <= excl + mine) {
                uint32_t cum = excl;
                int b = 0;
                for (; b < 3; ++b) {
                    if (cum + c4[b] >= rank) break;
                    cum += c4[b];
                }
                s_prefix = prefix | ((uint64_t)(tid * 4 + b) << lo);
                s_rank = rank - cum;
                s_lo = lo;
                s_done = (c4[b] == rank - cum) || lo == 0;
            }
            __syncthreads();
            if (s_done) break;
        }
        // keep keys whose bits >= s_lo are below the chosen prefix, and the
        // first s_rank (in index order) of those equal to it; a kept key's
        // place is (keys below before it) + min(ties before it, s_rank)
        const uint64_t hmask = ~((1ull << s_lo) - 1ull);
        const uint64_t cut = s_prefix;
        const int take = (int)s_rank;
        if (staged) {
            // wave w takes a contiguous segment: its counts of keys below
            // and equal to the cut, then (after the waves' totals) its writes
            const int S = (C + 15) / 16, wb = min(C, wid * S), we = min(C, wb + S);
            int nl = 0, ntie = 0;
            for (int i0 = wb; i0 < we; i0 += 4 * 64) {
                uint64_t v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * 64 + lane;
                    v[u] = i < we ? sk[i] & hmask : ~0ull;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool in = i0 + u * 64 + lane < we;
                    nl += __popcll(__ballot(in && v[u] < cut));
                    ntie += __popcll(__ballot(in && v[u] == cut));
                }
            }
            if (lane == 0) {
                s_wl[wid] = nl;
                s_wt[wid] = ntie;
            }
            __syncthreads();
            int lr = 0, tr = 0;
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                lr += w < wid ? s_wl[w] : 0;
                tr += w < wid ? s_wt[w] : 0;
            }
            for (int i0 = wb; i0 < we; i0 += 4 * 64) {
                uint64_t v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * 64 + lane;
                    v[u] = i < we ? sk[i] & hmask : ~0ull;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * 64 + lane;
                    const bool less = i < we && v[u] < cut, tie = i < we && v[u] == cut;
                    const uint64_t bl = __ballot(less), bt = __ballot(tie);
                    const int l = lr + __popcll(bl & below), t = tr + __popcll(bt & below);
                    if (less) pool[l + min(t, take)] = direct ? i : sj[i];
                    if (tie && t < take) pool[l + t] = direct ? i : sj[i];
                    lr += __popcll(bl);
                    tr += __popcll(bt);
                }
            }
        } else {
            // more candidates than LDS holds: rounds of 1024 in index order,
            // compacted in place (a round writes only below its own reads)
            if (tid == 0) {
                s_c0 = 0;
                s_c1 = 0;
            }
            __syncthreads();
            for (int base = 0; base < C; base += nt) {
                const int i = base + tid;
                int j = 0, less = 0, tie = 0;
                if (i < C) {
                    j = pool[i];
                    const uint64_t u = (uint64_t)key[j] & hmask;
                    less = u < cut;
                    tie = u == cut;
                }
                int tot;
                const int packed = scan1024(less | (tie << 16), s_w[par ^ 1], tot);
                const int lr = s_c0 + (packed & 0xffff), tr = s_c1 + (packed >> 16);
                if (i < C && (less || (tie && tr < take))) pool[lr + min(tr, take)] = j;
                __syncthreads();
                if (tid == 0) {
                    s_c0 += tot & 0xffff;
                    s_c1 += tot >> 16;
                }
                __syncthreads();
            }
        }
        if (tid == 0) ctrl->pool_count = r;
    }
    if (tid == 0) {
        ctrl->passed = passed;
        ctrl->pass_count = 0;
        ctrl->cut_bound = ~0ull;
    }
}

// Quadtree compaction: kept leaves to the code list (after the codes of the
// earlier levels), the four children of each split range to the next active
// list, in order. A workgroup's offsets are the sums of the decision step's
// per-workgroup counts before its first range; the last workgroup, which also
// sees the totals, sets the next level's code base and active count.
__device__ __forceinline__ void k_quad_scatter_body(CompactArgs a, Ctrl* ctrl, const Ctrl* pctrl,
                                                         int lv, int nblk,
                                                         const int2* blk, const fic_code* tmp_codes,
                                                         fic_code* codes, int capacity,
                                                         const int32_t* act, int32_t* act_next,
                                                         int half, fic_level_stats* stats,
                                                         int32_t* n_out) {
    const int base = blockIdx.x * kBlock * kQuadItems + threadIdx.x * kQuadItems;
    int f0[kQuadItems], f1[kQuadItems];
    int c0 = 0, c1 = 0;
#pragma unroll
    for (int u = 0; u < kQuadItems; ++u) {
        item_flags(a, ctrl, 0, base + u, f0[u], f1[u]);
        c0 += f0[u];
        c1 += f1[u];
    }
    // kept and split ranges before this workgroup
    constexpr int kPer = kBlock * kQuadItems / kRqRanges;  // decision workgroups per workgroup
    const int2 off = counts_before(blk, blockIdx.x * kPer);
    const int off0 = off.x, off1 = off.y;
    int e0, e1, t0, t1;
    block_scan2(c0, c1, e0, e1, t0, t1);
    int r0 = off0 + e0, r1 = off1 + e1;
    const int cb = ctrl->lvl_base[lv];
#pragma unroll
    for (int u = 0; u < kQuadItems; ++u) {
        const int i = base + u;
        if (f0[u]) {
            const int pos = cb + r0;
            if (pos < capacity) codes[pos] = tmp_codes[i];
            ++r0;
        }
        if (f1[u]) {
            const int yx = act[i];
            const int y = yx >> 16, x = yx & 0xffff;
            int32_t* dst = act_next + 4 * r1;
            dst[0] = (y << 16) | x;
            dst[1] = (y << 16) | (x + half);
            dst[2] = ((y + half) << 16) | x;
            dst[3] = ((y + half) << 16) | (x + half);
            ++r1;
        }
    }
    if ((int)blockIdx.x == nblk - 1 && threadIdx.x == 0) {
        const int tot0 = off0 + t0, tot1 = off1 + t1;
        const int nact = *a.act_count;
        ctrl->lvl_base[lv + 1] = cb + tot0;
        ctrl->n_codes = cb + tot0;
        if (n_out) *n_out = cb + tot0;
        ctrl->act_count[lv + 1] = 4 * tot1;
        if (stats) {
            const int pool = pctrl->pool_count;
            fic_level_stats st;
            st.matches = (int64_t)nact * pool * 8;
            st.pool = pool;
            st.passed = pctrl->passed;
            st.active = nact;
            st.accepted = tot0;
            stats[lv] = st;
        }
    }
}

// ---------------------------------------------------------------- pool preparation
// Per pool entry p: the decimated domain d' (2x2 sums) as packed high and low
// bytes, S = sum d', A' = n sum d'^2 - S^2 and the grid index j. TPD lanes
// share a domain, 16 decimated values each. identity_total >= 0 means the
// pool is the whole grid (no filter); block 0 then publishes its size.
template <int B>
struct PrepShape {
    static constexpr int n = B * B;
    static constexpr int PER = n < 16 ? n : 16;
    static constexpr int TPD = n / PER;
};

template <int B>
__device__ __forceinline__ void k_pool_prep_body(const uint8_t* __restrict__ img, int pitch,
                                                      int L, int gx, const int32_t* __restrict__ pool,
                                                      int identity_total, Ctrl* ctrl,
                                                      uint32_t* __restrict__ HL,
                                                      uint32_t* __restrict__ Sd,
                                                      int64_t* __restrict__ Ad,
                                                      int32_t* __restrict__ Jd) {
    using S = PrepShape<B>;
    constexpr int n = B * B, NW = n / 4, PER = S::PER, TPD = S::TPD;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (identity_total >= 0 && g == 0) {
        ctrl->pool_count = identity_total;
        ctrl->passed = identity_total;
    }
    const int count = identity_total >= 0 ? identity_total : ctrl->pool_count;
    const int p = g / TPD, sub = g % TPD;
    const bool ok = p < count;
    uint32_t s = 0;
    uint64_t q = 0;
    int j = 0;
    if (ok) {
        j = identity_total >= 0 ? p : pool[p];
        const int y = (j / gx) * L, x = (j % gx) * L;
        uint32_t* hl = HL + (int64_t)p * 2 * NW;
#pragma unroll
        for (int w = 0; w < PER / 4; ++w) {
            uint32_t hw = 0, lw = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int m = sub * PER + 4 * w + b, i = m / B, c = m % B;
                const uint8_t* px = img + (int64_t)(y + 2 * i) * pitch + x + 2 * c;
                const uint32_t d = (uint32_t)px[0] + px[1] + px[pitch] + px[pitch + 1];
                s += d;
                q += (uint64_t)d * d;
                hw |= (d >> 8) << (8 * b);
                lw |= (d & 255u) << (8 * b);
            }
            hl[sub * (PER / 4) + w] = hw;
            hl[NW + sub * (PER / 4) + w] = lw;
        }
    }
#pragma unroll
    for (int m = 1; m < TPD; m <<= 1) {
        s += __shfl_xor(s, m, 64);
        q += __shfl_xor(q, m, 64);
    }
    if (ok && sub == 0) {
        Sd[p] = s;
        Ad[p] = (int64_t)n * (int64_t)q - (int64_t)s * (int64_t)s;
        Jd[p] = j;
    }
}

// ---------------------------------------------------------------- the matcher
// Candidate key: (domain << 27) | (iso << 24) | (contrast index << 20) | sum d'.
// Ordering keys orders (domain, iso, contrast index); the low 20 bits carry the
// domain sum (< 2^18), a function of the domain, for the offset of eq. (3).
__device__ inline int64_t make_key(int64_t j, int t, int s, uint32_t S) {
    return (j << 27) | ((int64_t)t << 24) | ((int64_t)s << 20) | (int64_t)S;
}

__device__ inline bool pair_less(int64_t fa, int64_t ka, int64_t fb, int64_t kb) {
    return fa < fb || (fa == fb && ka < kb);
}

// Best contrast for one (row, domain) element. F = k^2 A' - 8Q k B' is
// 16 Q^2 n E(k) minus the row constant 16 Q^2 C. For a consecutive set
// k0..k1 the minimiser is the smallest k with (2k+1) A' >= 8Q B' (F is a
// convex quadratic in k); an FP32 estimate is corrected exactly.
__device__ inline void best_contrast_grid(int64_t Bp, int64_t Ap, int k0, int k1, int64_t& F, int& s) {
    int k = k0;
    if (Ap > 0) {
        float xf = (float)Bp * (40.0f / (float)Ap);
        float kf = fminf(fmaxf(rintf(xf), (float)k0), (float)k1);
        k = (int)kf;
        const int64_t b80 = 80 * Bp;
        while (k > k0 && (int64_t)(2 * k - 1) * Ap >= b80) --k;
        while (k < k1 && (int64_t)(2 * k + 1) * Ap < b80) ++k;
    }
    F = (int64_t)(k * k) * Ap - (int64_t)(80 * k) * Bp;
    s = k - k0;
}

// Every value of the set in turn; ks refers to the kernel argument (a local
// copy indexed in a loop would live in scratch memory).
__device__ inline void best_contrast_list(int64_t Bp, int64_t Ap, const KSet& ks, int64_t& F, int& s) {
    F = INT64_MAX;
    s = 0;
    for (int i = 0; i < ks.n; ++i) {
        const int k = ks.k[i];
        const int64_t f = (int64_t)(k * k) * Ap - (int64_t)(80 * k) * Bp;
        if (f < F) {
            F = f;
            s = i;
        }
    }
}

__device__ inline void best_contrast(int64_t Bp, int64_t Ap, const KSet& ks, int64_t& F, int& s) {
    if (ks.consecutive) best_contrast_grid(Bp, Ap, ks.k0, ks.k1, F, s);
    else best_contrast_list(Bp, Ap, ks, F, s);
}

template <int B>
struct MatchTile {
    static constexpr int n = B * B;
    static constexpr int NW = n / 4;
    // domains per LDS tile: 8-34 KiB of LDS
    static constexpr int TN = B == 16 ? 64 : (B == 8 ? 128 : 256);
    // target domains per pool chunk (one workgroup's share of the pool)
    static constexpr int CG = B == 16 ? 16 : (B == 8 ? 32 : (B == 4 ? 64 : 128));
    // exact integer widths (bounds by Cauchy-Schwarz: |B'| <= sqrt(A' C))
    using BpT = typename std::conditional<(B <= 8), int32_t, int64_t>::type;   // B'
    using GT = typename std::conditional<(B <= 4), int32_t, int64_t>::type;    // k A' - 80 B'
};

// Contrast-set modes of the matcher.
enum { kModeSmall = 0, kModeGrid = 1, kModeList = 2 };
constexpr int kSmallMax = 2;

// Isometries per thread: 2 for small sets at B <= 4, where a domain's LDS
// record would otherwise cost more LDS bandwidth than its arithmetic; the
// workgroup then covers 64 ranges instead of 32.
constexpr int match_isos_per_thread(int B, int mode) { return mode == kModeSmall && B <= 4 ? 2 : 1; }
constexpr int match_ranges_per_block(int B, int mode) { return kBlock * match_isos_per_thread(B, mode) / 8; }

// Number of pool chunks actually used: about one LDS tile each, at most the
// chunks the grid was launched with.
__device__ inline int active_chunks(int P, int TN, int n_chunks) {
    return max(1, min(n_chunks, (P + TN - 1) / TN));
}

// Domain loop of the B = 2 small-set matcher for IT isometries of one range.
// Records {d'0 | d'1 << 16, d'2 | d'3 << 16, kf A', p} with p the pool position
// and kf the first contrast value in use; TWO adds the second value through
// (k1 - k0) A'. G = 80 sum_i d'_i w_i + kf A' with |sum_i d'_i w_i| <= 4 * 1020
// * 765 < 2^22, so one 24-bit multiply-add is exact whatever the pool size.
// Running minimum of G and the pool position of its first occurrence, per
// isometry.
template <int IT, bool TWO>
__device__ __forceinline__ void match_b2_loop(const int4* sRec, const int32_t* sE1, int cnt,
                                              const uint32_t* w01, const uint32_t* w23, int* g0,
                                              int* p0, int* g1, int* p1) {
    typedef short s2 __attribute__((ext_vector_type(2)));
    s2 a01[IT], a23[IT];
    int bg0[IT], bp0[IT], bg1[IT], bp1[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        a01[i] = __builtin_bit_cast(s2, w01[i]);
        a23[i] = __builtin_bit_cast(s2, w23[i]);
        bg0[i] = g0[i];
        bp0[i] = p0[i];
        bg1[i] = g1[i];
        bp1[i] = p1[i];
    }
#pragma unroll 4
    for (int d = 0; d < cnt; ++d) {
        const int4 rec = sRec[d];
        const int e1 = TWO ? sE1[d] : 0;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            int dsum = __builtin_amdgcn_sdot2(__builtin_bit_cast(s2, rec.x), a01[i], 0, false);
            dsum = __builtin_amdgcn_sdot2(__builtin_bit_cast(s2, rec.y), a23[i], dsum, false);
            const int g = __mul24(dsum, 80) + rec.z;
            const bool lt = g < bg0[i];
            bp0[i] = lt ? rec.w : bp0[i];
            bg0[i] = lt ? g : bg0[i];
            if constexpr (TWO) {
                const int h = g + e1;
                const bool lt1 = h < bg1[i];
                bp1[i] = lt1 ? rec.w : bp1[i];
                bg1[i] = lt1 ? h : bg1[i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        g0[i] = bg0[i];
        p0[i] = bp0[i];
        g1[i] = bg1[i];
        p1[i] = bp1[i];
    }
}

// grid: x = row blocks of RPB ranges (RPB = 32, or 64 with two isometries
// per thread), y = pool chunks. The workgroup stages its range blocks in LDS;
// thread (range q, isometry t) keeps row[m] = R[iso_src(inverse(t), m)] in
// registers as packed bytes, so that <row, d'> = <R, T_t(d')>. With IT
// isometries per thread, thread j of a range takes t = j, j + 8 / IT, ...
//  kModeSmall: at most kSmallMax contrast values. For each value k > 0 the
//    thread keeps the smallest G = k A' - 80 B' (F = k G), in 32-bit integers
//    for B <= 4; k = 0 gives F = 0 everywhere, so its best is the first domain.
//  kModeGrid: consecutive k0..k1, closed-form minimiser, exact in int64.
//  kModeList: any set, every value evaluated in int64.
// LDS of the VALU matcher (one struct, so that a kernel holding several
// matchers can overlay them).
template <int B, int MODE, int TN_ = MatchTile<B>::TN>
struct MatchSmem {
    using Tl = MatchTile<B>;
    static constexpr int TN = TN_, NW = Tl::NW, n = Tl::n;
    static constexpr int RPB = match_ranges_per_block(B, MODE);
    static constexpr int NKA = MODE == kModeSmall ? kSmallMax : 1;
    static constexpr bool kFast = MODE == kModeSmall && B <= 4;
    uint32_t sHL[TN * 2 * NW];
    uint32_t sS[kFast ? 1 : TN];
    int64_t sA[MODE == kModeSmall ? 1 : TN];
    float sAf[MODE == kModeSmall ? 1 : TN];  // A' in FP32, for the screen
    typename Tl::GT sKA[NKA][kFast ? 1 : TN];
    int4 sRec[kFast ? TN : 1];
    int32_t sE1[kFast && B == 2 ? TN : 1];
    uint8_t sR[RPB * n];
};

// TN_: pool domains per LDS stage (the level default, or fewer where LDS is short).
template <int B, int MODE, int TN_ = MatchTile<B>::TN>
__device__ __forceinline__ void k_match_body(MatchSmem<B, MODE, TN_>& sm, int bx, int by,
                                                  const uint8_t* __restrict__ img, int pitch,
                                                  const int32_t* __restrict__ act,
                                                  const int32_t* act_count,
                                                  const uint32_t* __restrict__ HL,
                                                  const uint32_t* __restrict__ Sd,
                                                  const int64_t* __restrict__ Ad,
                                                  const int32_t* __restrict__ Jd, const Ctrl* ctrl,
                                                  const KSet& ks, int n_chunks, Partial* __restrict__ part,
                                                  int32_t* __restrict__ SRout,
                                                  int64_t* __restrict__ CRout, int cg) {
    using Tl = MatchTile<B>;
    using BpT = typename Tl::BpT;
    using GT = typename Tl::GT;
    constexpr int n = Tl::n, NW = Tl::NW, TN = TN_;
    constexpr int IT = match_isos_per_thread(B, MODE), TPR = 8 / IT;
    constexpr int RPB = match_ranges_per_block(B, MODE);
    constexpr int NKA = MODE == kModeSmall ? kSmallMax : 1;
    // small sets at B <= 4: per domain (S, k0 A', k1 A') in one 16-byte record
    constexpr bool kFast = MODE == kModeSmall && B <= 4;
    static_assert(NKA == MatchSmem<B, MODE, TN_>::NKA, "LDS layout");
    auto& sHL = sm.sHL;
    auto& sS = sm.sS;
    auto& sA = sm.sA;
    auto& sAf = sm.sAf;
    auto& sKA = sm.sKA;
    auto& sRec = sm.sRec;
    auto& sE1 = sm.sE1;
    auto& sR = sm.sR;

    const int nact = *act_count;
    const int q0 = bx * RPB;
    if (q0 >= nact) return;
    const int P = ctrl->pool_count;
    const int c = by;
    if (c >= active_chunks(P, cg, n_chunks)) return;
    const int nca = active_chunks(P, cg, n_chunks);

#pragma unroll
    for (int e = threadIdx.x; e < RPB * n; e += kBlock) {
        const int lq = e / n, m = e % n, q = q0 + lq;
        uint8_t v = 0;
        if (q < nact) {
            const int yx = act[q];
            if (yx >= 0) v = img[(int64_t)((yx >> 16) + m / B) * pitch + (yx & 0xffff) + m % B];
        }
        sR[e] = v;
    }
    __syncthreads();
    const int lq = threadIdx.x / TPR, tsub = threadIdx.x % TPR, q = q0 + lq;
    const bool valid = q < nact;
    const uint8_t* rr = sR + lq * n;
    uint32_t rI[IT][NW];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        // T_u is affine in (i, c): source index = a0 + a1 i + a2 c
        const int u = iso_inverse(tsub + it * TPR);
        const int a0 = iso_src(B, u, 0, 0);
        const int a1 = iso_src(B, u, 1, 0) - a0, a2 = iso_src(B, u, 0, 1) - a0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int m = 4 * w + b;
                v |= (uint32_t)rr[a0 + a1 * (m / B) + a2 * (m % B)] << (8 * b);
            }
            rI[it][w] = v;
        }
    }
    uint32_t* r = rI[0];
    // sum r and sum r^2 (the same for every isometry)
    uint32_t srum = 0, sq = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        srum = __builtin_amdgcn_udot4(r[w], 0x01010101u, srum, false);
        sq = __builtin_amdgcn_udot4(r[w], r[w], sq, false);
    }
    if (valid && tsub == 0 && c == 0) {
        SRout[q] = (int32_t)srum;
        CRout[q] = (int64_t)n * sq - (int64_t)srum * srum;
    }
    const BpT sr = (BpT)srum;
    const int lo = (int)((int64_t)P * c / nca);
    const int hi = (int)((int64_t)P * (c + 1) / nca);

    // kModeSmall state, per isometry of the thread
    GT bestG[IT][kSmallMax];
    int bestPs[IT][kSmallMax];
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int u = 0; u < kSmallMax; ++u) {
            bestG[it][u] = std::numeric_limits<GT>::max();
            bestPs[it][u] = lo;  // k = 0: every domain ties, the first one wins
        }
    // other modes
    int64_t bestF = INT64_MAX;
    int bestP = -1, bestS = 0;
    // screen: over real k, F >= -1600 B'^2 / A', so an element can go below a best
    // F_b <= 0 only if B' > 0 and 1600 B'^2 > -F_b A'. thrF = -F_b / 1600 shrunk by
    // 2^-18 (below the FP32 roundings of B'^2, A' and the product), so no element that
    // could win is skipped; while F_b > 0 (no candidate yet, or a set without 0)
    // every element goes to the exact step.
    float thrF = 0.0f;

    for (int base = lo; base < hi; base += TN) {
        const int cnt = min(TN, hi - base);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * 2 * NW; i += kBlock) sHL[i] = HL[(int64_t)base * 2 * NW + i];
        for (int i = threadIdx.x; i < cnt; i += kBlock) {
            const int64_t a = Ad[base + i];
            if constexpr (kFast && B == 2) {
                // B = 2: the 4 sums d' as two pairs of 16-bit values (from the high and
                // low bytes), k0 A', the pool position, and (k1 - k0) A' aside
                const uint32_t h = HL[(int64_t)(base + i) * 2], l = HL[(int64_t)(base + i) * 2 + 1];
                // the first value in use is kf (kf A' <= 10 * 4 * 4 * 1020^2 < 2^28)
                const int k0 = ks.n > 0 ? ks.k[0] : 0, k1 = ks.n > 1 ? ks.k[1] : 0;
                const int kf = k0 != 0 ? k0 : k1;
                int4 rec;
                rec.x = (int)__builtin_amdgcn_perm(h, l, 0x05010400u);  // d0 | d1 << 16
                rec.y = (int)__builtin_amdgcn_perm(h, l, 0x07030602u);  // d2 | d3 << 16
                rec.z = (int)((int64_t)kf * a);
                rec.w = base + i;
                sRec[i] = rec;
                sE1[i] = (int)((int64_t)(k1 - k0) * a);
            } else if constexpr (kFast) {
                // k A' may wrap in 32 bits; G = k A' - 80 B' fits (|G| < 2^31) and is
                // computed modulo 2^32
                int4 rec;
                rec.x = (int)Sd[base + i];
                rec.y = (int)((uint32_t)(ks.n > 0 ? ks.k[0] : 0) * (uint32_t)a);
                rec.z = (int)((uint32_t)(ks.n > 1 ? ks.k[1] : 0) * (uint32_t)a);
                rec.w = 0;
                sRec[i] = rec;
            } else {
                sS[i] = Sd[base + i];
                if (MODE == kModeSmall) {
#pragma unroll
                    for (int u = 0; u < kSmallMax; ++u) sKA[u][i] = (GT)(u < ks.n ? ks.k[u] : 0) * (GT)a;
                } else {
                    sA[i] = a;
                    sAf[i] = (float)a;
                }
            }
        }
        __syncthreads();
        if constexpr (kFast) {
            // G_u = k_u A' + 80 sum r S - 80 n (256 P_hi + P_lo); every 24-bit operand is
            // below 2^23 for B <= 4, so three 24-bit multiply-adds at full rate
            const bool use0 = ks.n > 0 && ks.k[0] != 0, use1 = ks.n > 1 && ks.k[1] != 0;
            const int c1 = 80 * (int)srum;
            constexpr int kPh = 80 * n * 256, kPl = 80 * n;
            if constexpr (B == 2) {
                // G_u = k_u A' + 80 sum_i d'_i (sum r - 4 r_i): the weights sum r - 4 r_i
                // lie in [-765, 765], so two v_dot2_i32_i16 give the sum exactly, and
                // |sum| < 2^22 leaves one 24-bit multiply-add for G
                uint32_t w01[IT], w23[IT];
                int g0[IT], p0[IT], g1[IT], p1[IT];
#pragma unroll
                for (int it = 0; it < IT; ++it) {
                    const uint32_t rw = rI[it][0];
                    const int r0 = rw & 0xff, r1 = (rw >> 8) & 0xff, r2 = (rw >> 16) & 0xff, r3 = rw >> 24;
                    const int sr4 = r0 + r1 + r2 + r3;
                    w01[it] = (uint32_t)(uint16_t)(sr4 - 4 * r0) | ((uint32_t)(uint16_t)(sr4 - 4 * r1) << 16);
                    w23[it] = (uint32_t)(uint16_t)(sr4 - 4 * r2) | ((uint32_t)(uint16_t)(sr4 - 4 * r3) << 16);
                    // the slot of the first value in use comes first
                    const int f = use0 ? 0 : 1;
                    g0[it] = bestG[it][f];
                    p0[it] = bestPs[it][f];
                    g1[it] = bestG[it][1 - f];
                    p1[it] = bestPs[it][1 - f];
                }
                if (use0 && use1) match_b2_loop<IT, true>(sRec, sE1, cnt, w01, w23, g0, p0, g1, p1);
                else if (use0 || use1) match_b2_loop<IT, false>(sRec, sE1, cnt, w01, w23, g0, p0, g1, p1);
#pragma unroll
                for (int it = 0; it < IT; ++it) {
                    const int f = use0 ? 0 : 1;
                    bestG[it][f] = g0[it];
                    bestPs[it][f] = p0[it];
                    bestG[it][1 - f] = g1[it];
                    bestPs[it][1 - f] = p1[it];
                }
                continue;
            }
#pragma unroll 2
            for (int d = 0; d < cnt; ++d) {
                const uint32_t* hl = sHL + d * 2 * NW;
                const int4 rec = sRec[d];
                const uint32_t cs = (uint32_t)__mul24(c1, rec.x);
                const int dd = base + d;
#pragma unroll
                for (int it = 0; it < IT; ++it) {
                    uint32_t ph = 0, pl = 0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        ph = __builtin_amdgcn_udot4(rI[it][w], hl[w], ph, false);
                        pl = __builtin_amdgcn_udot4(rI[it][w], hl[NW + w], pl, false);
                    }
                    const uint32_t pt = (uint32_t)__mul24(kPh, (int)ph) + (uint32_t)__mul24(kPl, (int)pl);
                    if (use0) {
                        const int g = (int)((uint32_t)rec.y + cs - pt);
                        const bool lt = g < bestG[it][0];
                        bestG[it][0] = lt ? g : bestG[it][0];
                        bestPs[it][0] = lt ? dd : bestPs[it][0];
                    }
                    if (use1) {
                        const int g = (int)((uint32_t)rec.z + cs - pt);
                        const bool lt = g < bestG[it][1];
                        bestG[it][1] = lt ? g : bestG[it][1];
                        bestPs[it][1] = lt ? dd : bestPs[it][1];
                    }
                }
            }
            continue;
        }
        for (int d = 0; d < cnt; ++d) {
            const uint32_t* hl = sHL + d * 2 * NW;
            uint32_t ph = 0, pl = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                ph = __builtin_amdgcn_udot4(r[w], hl[w], ph, false);
                pl = __builtin_amdgcn_udot4(r[w], hl[NW + w], pl, false);
            }
            const BpT Pv = (BpT)((ph << 8) + pl);
            const BpT Bp = Pv * (BpT)n - sr * (BpT)sS[d];
            if (MODE == kModeSmall) {
                const GT b80 = (GT)80 * (GT)Bp;
#pragma unroll
                for (int u = 0; u < kSmallMax; ++u) {
                    if (u < ks.n && ks.k[u] != 0) {
                        const GT g = sKA[u][d] - b80;
                        if (g < bestG[0][u]) {
                            bestG[0][u] = g;
                            bestPs[0][u] = base + d;
                        }
                    }
                }
            } else {
                const float bf = (float)Bp;
                if (bestF > 0 || (Bp > 0 && bf * bf >= thrF * sAf[d])) {
                    int64_t F;
                    int sidx;
                    if (MODE == kModeGrid) best_contrast_grid((int64_t)Bp, sA[d], ks.k0, ks.k1, F, sidx);
                    else best_contrast_list((int64_t)Bp, sA[d], ks, F, sidx);
                    if (F < bestF) {
                        bestF = F;
                        bestP = base + d;
                        bestS = sidx;
                        thrF = bestF > 0 ? 0.0f : (float)(-bestF) * (1.0f / 1600.0f) * (1.0f - 1.0f / 262144.0f);
                    }
                }
            }
        }
    }
    int64_t outF = INT64_MAX, outK = INT64_MAX;
    if (lo < hi) {
        if (MODE == kModeSmall) {
#pragma unroll
            for (int it = 0; it < IT; ++it)
#pragma unroll
                for (int u = 0; u < kSmallMax; ++u) {
                    if (u >= ks.n) continue;
                    const int k = ks.k[u];
                    if (k != 0 && bestG[it][u] == std::numeric_limits<GT>::max()) continue;
                    const int64_t F = k == 0 ? 0 : (int64_t)k * (int64_t)bestG[it][u];
                    const int p = bestPs[it][u];
                    const int64_t K = make_key(Jd[p], tsub + it * TPR, u, Sd[p]);
                    if (pair_less(F, K, outF, outK)) {
                        outF = F;
                        outK = K;
                    }
                }
        } else if (bestP >= 0) {
            outF = bestF;
            outK = make_key(Jd[bestP], tsub, bestS, Sd[bestP]);
        }
    }
    // reduce over the TPR consecutive lanes of each range
#pragma unroll
    for (int m = 1; m < TPR; m <<= 1) {
        const int64_t of = __shfl_xor(outF, m, 64);
        const int64_t ok = __shfl_xor(outK, m, 64);
        if (pair_less(of, ok, outF, outK)) {
            outF = of;
            outK = ok;
        }
    }
    if (valid && tsub == 0) {
        Partial pr;
        pr.F = outF;
        pr.key = outK;
        part[(int64_t)q * n_chunks + c] = pr;
    }
}

// ---------------------------------------------------------------- per-range result
// Contrast numerator at position s of a set. Callers pass the set by
// reference to the kernel argument: a by-value copy indexed per lane would be
// placed in LDS, one copy per thread.
__device__ inline int kset_value(const KSet& ks, int s) {
    return ks.consecutive ? ks.k0 + s : ks.k[s];
}

// Fill the match of a range from its best (F, key) over all pool chunks.
__device__ inline bool finish_best(int yx, int B, int L, int gx, int64_t F, int64_t K, int64_t CRq,
                                   int32_t SRq, const KSet& ks, fic_match& m, int& dy, int& dx) {
    m.flags = 0;
    m.pad_ = 0;
    if (yx < 0 || K == INT64_MAX) {
        m.e_num = -1;
        m.dom = -1;
        m.iso = 0;
        m.s_idx = 0;
        m.k = 0;
        m.q_o = 0;
        m.E = -1.0f;
        dy = dx = 0;
        return false;
    }
    const int n = B * B;
    const int j = (int)(K >> 27), t = (int)((K >> 24) & 7), s = (int)((K >> 20) & 15);
    const int64_t sd = K & 0xfffff;
    const int k = kset_value(ks, s);
    dy = (j / gx) * L;
    dx = (j % gx) * L;
    m.e_num = F + 1600 * CRq;
    m.dom = j;
    m.iso = (uint8_t)t;
    m.s_idx = (uint8_t)s;
    m.k = (uint8_t)k;
    // |numerator| < 2^24 for n <= 256 (sum r <= 255 n, sum d' <= 1020 n, k <= 10)
    m.q_o = (int16_t)floordiv32(2 * (40 * SRq - k * (int)sd) + 40 * n, 80 * n);
    m.E = (float)m.e_num / (1600.0f * (float)n);
    return true;
}

__device__ inline bool finish_range(int yx, int B, int L, int gx, const Partial* pr, int nca,
                                    int64_t CRq, int32_t SRq, const KSet& ks, fic_match& m,
                                    int& dy, int& dx) {
    int64_t F = INT64_MAX, K = INT64_MAX;
    for (int c = 0; c < nca; ++c)
        if (pair_less(pr[c].F, pr[c].key, F, K)) {
            F = pr[c].F;
            K = pr[c].key;
        }
    return finish_best(yx, B, L, gx, F, K, CRq, SRq, ks, m, dy, dx);
}

__device__ __forceinline__ void k_reduce_level_body(int B, int L, int gx,
                                                         const int32_t* __restrict__ act,
                                                         const int32_t* act_count,
                                                         const Partial* __restrict__ part,
                                                         int n_chunks, int CG, const Ctrl* ctrl,
                                                         const int64_t* __restrict__ CR,
                                                         const int32_t* __restrict__ SR, const KSet& ks,
                                                         fic_match* __restrict__ out) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= *act_count) return;
    fic_match m;
    int dy, dx;
    const int nca = active_chunks(ctrl->pool_count, CG, n_chunks);
    finish_range(act[q], B, L, gx, part + (int64_t)q * n_chunks, nca, CR[q], SR[q], ks, m, dy, dx);
    out[q] = m;
}

// Quadtree step: the leaf record and the keep/split decision of each active
// range. kRqLanes lanes share a range: they take its pool chunks in turn (all
// loads of a workgroup in flight together), combine their bests, and each
// stores a quarter of the range's 32-byte code. Per-workgroup counts of kept
// and split ranges go to blk (the compaction that follows sums them).
__device__ __forceinline__ void k_reduce_quad_body(
    int B, int L, int gx, int lv, int last, int64_t thr, const int32_t* __restrict__ act,
    const Ctrl* ctrl, const Ctrl* pctrl, const Partial* __restrict__ part, int n_chunks, int CG,
    const int64_t* __restrict__ CR, const int32_t* __restrict__ SR, const KSet& ks,
    fic_code* __restrict__ tmp, uint8_t* __restrict__ dec, int2* blk,
    uint32_t* __restrict__ flags) {
    static_assert(sizeof(fic_code) == 32 && kRqLanes == 4, "one 8-byte word of a code per lane");
    static_assert(offsetof(fic_code, dom) == 8 && offsetof(fic_code, y) == 12 &&
                      offsetof(fic_code, x) == 14 && offsetof(fic_code, dy) == 16 &&
                      offsetof(fic_code, q_o) == 20 && offsetof(fic_code, log2B) == 22 &&
                      offsetof(fic_code, k) == 24 && offsetof(fic_code, level) == 26,
                  "fic_code layout");
    const int lane = threadIdx.x % kRqLanes;
    const int q = blockIdx.x * kRqRanges + threadIdx.x / kRqLanes;
    const int nact = ctrl->act_count[lv];
    int fbase = 0;  // first flag bit of this level
    if (flags)
        for (int l = 0; l < lv; ++l) fbase += ctrl->act_count[l];
    const int nca = active_chunks(pctrl->pool_count, CG, n_chunks);
    const bool valid = q < nact;
    int64_t bF = INT64_MAX, bK = INT64_MAX;
    if (valid) {
        const Partial* pr = part + (int64_t)q * n_chunks;
#pragma unroll 4
        for (int c = lane; c < nca; c += kRqLanes) {
            const Partial v = pr[c];
            if (pair_less(v.F, v.key, bF, bK)) {
                bF = v.F;
                bK = v.key;
            }
        }
    }
#pragma unroll
    for (int m = 1; m < kRqLanes; m <<= 1) {
        const int64_t of = __shfl_xor(bF, m, 64), ok = __shfl_xor(bK, m, 64);
        if (pair_less(of, ok, bF, bK)) {
            bF = of;
            bK = ok;
        }
    }
    int kept = 0, split = 0;
    if (valid) {
        fic_match m;
        int dy, dx;
        const int yx = act[q];
        const bool ok = finish_best(yx, B, L, gx, bF, bK, CR[q], SR[q], ks, m, dy, dx);
        uint8_t d = 2;
        if (ok) {
            // the code's 8-byte words (little-endian fic_code layout): e_num |
            // dom, y, x | dy, dx, q_o, log2B, iso | k, s_idx, level, zero padding
            const uint64_t w0 = (uint64_t)m.e_num;
            const uint64_t w1 = (uint64_t)(uint32_t)m.dom | ((uint64_t)(uint32_t)(yx >> 16) << 32) |
                                ((uint64_t)(yx & 0xffff) << 48);
            const uint64_t w2 = (uint64_t)(uint16_t)dy | ((uint64_t)(uint16_t)dx << 16) |
                                ((uint64_t)(uint16_t)m.q_o << 32) |
                                ((uint64_t)(31 - __clz(B)) << 48) | ((uint64_t)m.iso << 56);
            const uint64_t w3 = (uint64_t)m.k | ((uint64_t)m.s_idx << 8) | ((uint64_t)lv << 16);
            const uint64_t w = lane == 0 ? w0 : lane == 1 ? w1 : lane == 2 ? w2 : w3;
            reinterpret_cast<uint64_t*>(tmp + q)[lane] = w;
            d = (last || m.e_num <= thr) ? 1 : 0;
        }
        if (lane == 0) {
            dec[q] = d;
            kept = d == 1;
            split = d == 0;
            if (flags && d == 0) atomicOr(&flags[(fbase + q) >> 5], 1u << ((fbase + q) & 31));
        }
    }
    int e0, e1, t0, t1;
    block_scan2(kept, split, e0, e1, t0, t1);
    if (threadIdx.x == 0) blk[blockIdx.x] = make_int2(t0, t1);
}

// ---------------------------------------------------------------- decoder
// map[pixel] = index of the code covering it (-1 if none); err set on overlap.
__global__ void k_decode_map(const fic_code* __restrict__ codes, int n_codes, int H, int W,
                             int32_t* __restrict__ map, int* err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_codes) return;
    fic_code c = codes[i];
    int B = 1 << c.log2B;
    bool ok = c.log2B >= 1 && c.log2B <= 4 && c.iso < 8 && c.k <= 10 && c.y >= 0 && c.x >= 0 &&
              c.y + B <= H && c.x + B <= W && c.dy >= 0 && c.dx >= 0 && c.dy + 2 * B <= H &&
              c.dx + 2 * B <= W;
    if (!ok) {
        atomicOr(err, 1);
        return;
    }
    for (int a = 0; a < B; ++a)
        for (int b = 0; b < B; ++b) {
            int old = atomicExch(&map[(c.y + a) * W + c.x + b], i);
            if (old != -1) atomicOr(err, 2);
        }
}

__global__ void k_fill_i32(int32_t* p, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Control blocks in their starting state: every counter zero, no floor bound.
__global__ void k_ctrl_reset(Ctrl* c, int n) {
    constexpr int kWords = (int)(sizeof(Ctrl) / 4);
    constexpr int kCut = (int)(offsetof(Ctrl, cut_bound) / 4);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kWords) return;
    const int w = i % kWords;
    reinterpret_cast<uint32_t*>(c)[i] = (w == kCut || w == kCut + 1) ? 0xffffffffu : 0u;
}

__global__ void k_fill_u8(uint8_t* p, int H, int W, int pitch, uint8_t v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < H * W) p[(i / W) * pitch + i % W] = v;
}

__global__ void k_check_map(const int32_t* map, int n, int* err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && map[i] < 0) atomicOr(err, 4);
}

// One Jacobi step: every pixel is rebuilt from the previous image.
__global__ void k_decode_iter(const fic_code* __restrict__ codes, const int32_t* __restrict__ map,
                              const uint8_t* __restrict__ src, int src_pitch,
                              uint8_t* __restrict__ dst, int dst_pitch, int H, int W) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= H * W) return;
    int py = p / W, px = p - py * W;
    int ci = map[p];
    if (ci < 0) return;
    fic_code c = codes[ci];
    int B = 1 << c.log2B;
    int i = py - c.y, col = px - c.x;
    int sidx = iso_src(B, c.iso, i, col);
    int si = sidx / B, sc = sidx - si * B;
    const uint8_t* s0 = src + (c.dy + 2 * si) * src_pitch + c.dx + 2 * sc;
    int d = (int)s0[0] + s0[1] + s0[src_pitch] + s0[src_pitch + 1];
    // (k/10)(d/4) + q_o rounded half up: floor((k d + 40 q_o + 20) / 40)
    int num = c.k * d + 40 * (int)c.q_o + 20;
    int v = num >= 0 ? num / 40 : -((-num + 39) / 40);
    dst[py * dst_pitch + px] = (uint8_t)min(max(v, 0), 255);
}

__global__ void k_sse(const uint8_t* __restrict__ a, int pa, const uint8_t* __restrict__ b, int pb,
                      int H, int W, unsigned long long* out) {
    unsigned long long acc = 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < H * W; p += gridDim.x * blockDim.x) {
        int y = p / W, x = p - y * W;
        int d = (int)a[y * pa + x] - (int)b[y * pb + x];
        acc += (unsigned long long)(d * d);
    }
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

// ---------------------------------------------------------------- calibration
// For every kept leaf whose B x B range has 8-bin entropy <= theta
// (key >= Mr), add k to the level's sum and count.
__global__ void k_calib_accum(const uint8_t* __restrict__ img, int pitch,
                              const fic_code* __restrict__ codes, const Ctrl* ctrl, int capacity,
                              const int64_t* __restrict__ T, const int64_t* __restrict__ Mr,
                              unsigned long long* acc /* [2*levels] */) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = min(ctrl->n_codes, capacity);
    if (i >= nc) return;
    fic_code c = codes[i];
    int B = 1 << c.log2B;
    int h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < B; ++a)
        for (int b = 0; b < B; ++b) {
            int v = img[(c.y + a) * pitch + c.x + b] >> 5;
#pragma unroll
            for (int q = 0; q < 8; ++q) h[q] += (v == q);
        }
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += T[h[q]];
    if (s >= Mr[c.level]) {
        atomicAdd(&acc[2 * c.level], (unsigned long long)c.k);
        atomicAdd(&acc[2 * c.level + 1], 1ull);
    }
}



// Histogram of the optimal contrast numerator k over kept leaves (all of them,
// or only those whose B x B range has 8-bin entropy <= theta): hist[level][k].
__global__ void k_calib_hist(const uint8_t* __restrict__ img, int pitch,
                             const fic_code* __restrict__ codes, const Ctrl* ctrl, int capacity,
                             const int64_t* __restrict__ T, const int64_t* __restrict__ Mr,
                             int low_only, unsigned long long* __restrict__ hist /* [4][11] */) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = min(ctrl->n_codes, capacity);
    if (i >= nc) return;
    const fic_code c = codes[i];
    if (c.k > 10 || c.level > 3) return;
    if (low_only) {
        const int B = 1 << c.log2B;
        int h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int a = 0; a < B; ++a)
            for (int b = 0; b < B; ++b) {
                const int v = img[(c.y + a) * pitch + c.x + b] >> 5;
#pragma unroll
                for (int q = 0; q < 8; ++q) h[q] += (v == q);
            }
        int64_t s = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s += T[h[q]];
        if (s < Mr[c.level]) return;
    }
    atomicAdd(&hist[c.level * 11 + c.k], 1ull);
}

// ================================================================ int8 MFMA matcher (B = 8)
// The correlation of every range row with every pool domain as an integer
// GEMM on the matrix cores: rows are r' = r - 128 (int8), columns split the
// 2x2 sums as d' = 128 h + l with h in 0..7 and l in 0..127 (both int8), so
//   X = sum r' d' = 128 sum r' h + sum r' l
// is exact in int32 after two v_mfma_i32_16x16x64_i8 (K = 64 = n). Then
//   B' = n P - sumR sumD' = 64 X - sumR' S,   sumR' = sumR - 128 n,
// also exact in int32. An FP32 screen (below) discards elements that cannot
// beat the row's best; the rest are decided exactly in int64, keeping the
// result identical to the exhaustive definition.
typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kM8Waves = 4;                            // wavefronts per workgroup
// 16-row MFMA tiles per wavefront: 4 for the int8 form, 2 for FP16 (whose
// register budget would otherwise halve its occupancy)
constexpr int m8_row_tiles(bool) { return 4; }
constexpr int m8_rows(bool f16) { return kM8Waves * 16 * m8_row_tiles(f16); }  // rows per workgroup
constexpr int kM8RowBits = 6;                           // queue entry: row | position << kM8RowBits
constexpr int kM8ColTiles = 6;                         // 16-column tiles per LDS stage
constexpr int kM8Cols = 16 * kM8ColTiles;              // 96 pool domains per LDS stage
constexpr int kM8Chunk = 1024;                         // target pool domains per chunk
// (1 - 2^-18): a factor that puts an FP32 square root or product (a few ulps
// of error each) safely below the exact real value.
constexpr float kM8Shrink = 1.0f - 1.0f / 262144.0f;
// The int8 screen's column scale: its normalized columns are at most 8 * 4079
// < 2^15 in size, two int8 halves.
constexpr float kI8Scale = 4079.0f;

// Rows r' = r - 128 of the 8 inverse-isometry arrangements of each range:
// Ar[(8q + t) * 64 + m] = R[iso_src(8, inverse(t), m)] - 128, as int8 or (F16)
// as FP16 (exact: integers of 8 bits). Thread per row.
template <bool F16>
__device__ __forceinline__ void k_range_prep_m8_body(const uint8_t* __restrict__ img, int pitch,
                                                          const int32_t* __restrict__ act,
                                                          const int32_t* act_count,
                                                          int8_t* __restrict__ Ar,
                                                          int32_t* __restrict__ SR,
                                                          int32_t* __restrict__ SRp,
                                                          int64_t* __restrict__ CR,
                                                          int64_t* __restrict__ GB,
                                                          int2* __restrict__ RC,
                                                          const fic_match* __restrict__ seed, int W) {
    constexpr int B = 8, n = 64;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= 8 * *act_count) return;
    const int q = row >> 3, t = row & 7;
    const int yx = act[q];
    if (t == 0) GB[q] = 0;  // the matcher's shared bound: F = 0 (k = 0) is always reached
    uint32_t* dst = reinterpret_cast<uint32_t*>(Ar + (int64_t)row * n * (F16 ? 2 : 1));
    if (yx < 0) {
        // r = 0 -> r' = -128 (0xd800 as FP16; int8: r' - c = 0 with c = -128)
        for (int w = 0; w < (F16 ? n / 2 : n / 4); ++w) dst[w] = F16 ? 0xd800d800u : 0u;
        if (t == 0) {
            SR[q] = 0;
            SRp[q] = -128 * n;
            CR[q] = 0;
            if constexpr (!F16) RC[q] = make_int2(-128, 0);
        }
        return;
    }
    const uint8_t* r = img + (int64_t)(yx >> 16) * pitch + (yx & 0xffff);
    // int8 rows are r' - c with c the range's mean of r' rounded, moved into
    // [max r' - 127, min r' + 128] so that every r' - c fits in int8 (a range's
    // values span at most 255)
    int cc = 0;
    if constexpr (!F16) {
        int s = 0, mn = 255, mx = 0;
        for (int i = 0; i < B; ++i)
            for (int c = 0; c < B; ++c) {
                const int v = r[i * pitch + c];
                s += v;
                mn = min(mn, v);
                mx = max(mx, v);
            }
        cc = min(max((s - 128 * n + 32) >> 6, mx - 255), mn);
        if (t == 0) {
            int sa = 0;
            for (int i = 0; i < B; ++i)
                for (int c = 0; c < B; ++c) sa += abs((int)r[i * pitch + c] - 128 - cc);
            RC[q] = make_int2(cc, sa);
        }
    }
    const int u = iso_inverse(t);
    const int a0 = iso_src(B, u, 0, 0);
    const int a1 = iso_src(B, u, 1, 0) - a0, a2 = iso_src(B, u, 0, 1) - a0;
    if constexpr (F16) {
#pragma unroll
        for (int w = 0; w < n / 2; ++w) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int m = 2 * w + b;
                const int src = a0 + a1 * (m / B) + a2 * (m % B);
                const _Float16 h = (_Float16)((int)r[(src / B) * pitch + src % B] - 128);
                v |= (uint32_t)__builtin_bit_cast(uint16_t, h) << (16 * b);
            }
            dst[w] = v;
        }
    } else {
#pragma unroll
        for (int w = 0; w < n / 4; ++w) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int m = 4 * w + b;
                const int src = a0 + a1 * (m / B) + a2 * (m % B);
                v |= (uint32_t)(uint8_t)((int)r[(src / B) * pitch + src % B] - 128 - cc) << (8 * b);
            }
            dst[w] = v;
        }
    }
    if (t == 0) {
        int s = 0;
        int64_t s2 = 0;
        for (int i = 0; i < B; ++i)
            for (int c = 0; c < B; ++c) {
                const int v = r[i * pitch + c];
                s += v;
                s2 += v * v;
            }
        SR[q] = s;
        SRp[q] = s - 128 * n;
        const int64_t cr = (int64_t)n * s2 - (int64_t)s * s;
        CR[q] = cr;
        if (seed) {
            // a match already reached for this range (e_num = F + 1600 C) bounds
            // its best F from the start: the screen still passes every element
            // with F at or below it, so the search's result is unchanged
            const int64_t e = seed[(int64_t)((yx >> 16) / B) * (W / B) + (yx & 0xffff) / B].e_num;
            if (e >= 0) GB[q] = min((int64_t)0, e - 1600 * cr);
        }
    }
}

// Columns for the MFMA matchers, 128 bytes per domain in each of two arrays:
// at Dh the exact sums d' (FP16, exact: integers below 2^11; or int8 as
// d' = 128 h + l with h in 0..7 and l in 0..127), at Dl their normalized form
// for the screen (below); in FP32 G = 40 / A' (0 for a constant domain). Four
// lanes share a domain, 16 decimated values each.
template <bool F16>
__device__ __forceinline__ void k_pool_prep_m8_body(const uint8_t* __restrict__ img, int pitch,
                                                         int L, int gx, const int32_t* __restrict__ pool,
                                                         int identity_total, Ctrl* ctrl,
                                                         int8_t* __restrict__ Dh, int8_t* __restrict__ Dl,
                                                         uint32_t* __restrict__ Sd, int64_t* __restrict__ Ad,
                                                         int32_t* __restrict__ Jd, float* __restrict__ Gd) {
    constexpr int B = 8, n = 64, TPD = 4, PER = 16;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (identity_total >= 0 && g == 0) {
        ctrl->pool_count = identity_total;
        ctrl->passed = identity_total;
    }
    const int count = identity_total >= 0 ? identity_total : ctrl->pool_count;
    const int p = g / TPD, sub = g % TPD;
    const bool ok = p < count;
    uint32_t s = 0;
    uint64_t q = 0;
    int j = 0;
    int dv[PER];  // the lane's d', normalized once the domain's moments are known
    if (ok) {
        j = identity_total >= 0 ? p : pool[p];
        const int y = (j / gx) * L, x = (j % gx) * L;
        // FP16: d' at Dh + 128 p; int8: h at Dh + 128 p, l 64 bytes further
        uint32_t* hd = reinterpret_cast<uint32_t*>(Dh + (int64_t)p * 128 + sub * PER * (F16 ? 2 : 1));
        uint32_t* ld = reinterpret_cast<uint32_t*>(Dh + (int64_t)p * 128 + 64 + sub * PER);
#pragma unroll
        for (int w = 0; w < PER / 4; ++w) {
            uint32_t hw = 0, lw = 0, f16w[2] = {0u, 0u};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int m = sub * PER + 4 * w + b, i = m / B, c = m % B;
                const uint8_t* px = img + (int64_t)(y + 2 * i) * pitch + x + 2 * c;
                const uint32_t d = (uint32_t)px[0] + px[1] + px[pitch] + px[pitch + 1];
                dv[4 * w + b] = (int)d;
                s += d;
                q += (uint64_t)d * d;
                hw |= (d >> 7) << (8 * b);
                lw |= (d & 127u) << (8 * b);
                f16w[b >> 1] |= (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(int)d) << (16 * (b & 1));
            }
            if constexpr (F16) {
                hd[2 * w] = f16w[0];
                hd[2 * w + 1] = f16w[1];
            } else {
                hd[w] = hw;
                ld[w] = lw;
            }
        }
    }
#pragma unroll
    for (int m = 1; m < TPD; m <<= 1) {
        s += __shfl_xor(s, m, 64);
        q += __shfl_xor(q, m, 64);
    }
    // the screen's normalized columns d^_i = (64 d'_i - S) s at Dl + 128 p, s =
    // 1 / Q (FP16) or 4079 / Q (int8: rounded to integers, |d^| <= 32632, as
    // 256 h + l with h, l in -128..127: h at Dl + 128 p, l 64 bytes further),
    // Q = sqrt(A') rounded below; s = 0 for a constant domain
    if (ok) {
        const int64_t A = (int64_t)n * (int64_t)q - (int64_t)s * (int64_t)s;
        const float sc = A > 0 ? (F16 ? 1.0f : kI8Scale) / (sqrtf((float)A) * kM8Shrink) : 0.0f;
        if constexpr (F16) {
            uint32_t* nd = reinterpret_cast<uint32_t*>(Dl + (int64_t)p * 128 + sub * PER * 2);
#pragma unroll
            for (int w = 0; w < PER / 2; ++w) {
                const _Float16 h0 = (_Float16)((float)(64 * dv[2 * w] - (int)s) * sc);
                const _Float16 h1 = (_Float16)((float)(64 * dv[2 * w + 1] - (int)s) * sc);
                nd[w] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
            }
        } else {
            uint32_t* nh = reinterpret_cast<uint32_t*>(Dl + (int64_t)p * 128 + sub * PER);
            uint32_t* nl = reinterpret_cast<uint32_t*>(Dl + (int64_t)p * 128 + 64 + sub * PER);
#pragma unroll
            for (int w = 0; w < PER / 4; ++w) {
                uint32_t hw = 0, lw = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int v = (int)rintf((float)(64 * dv[4 * w + b] - (int)s) * sc);
                    const int h = (v + 128) >> 8, l = v - 256 * h;
                    hw |= (uint32_t)(uint8_t)h << (8 * b);
                    lw |= (uint32_t)(uint8_t)l << (8 * b);
                }
                nh[w] = hw;
                nl[w] = lw;
            }
        }
    }
    if (ok && sub == 0) {
        const int64_t A = (int64_t)n * (int64_t)q - (int64_t)s * (int64_t)s;
        Sd[p] = s;
        Ad[p] = A;
        Jd[p] = j;
        Gd[p] = A > 0 ? 40.0f / (float)A : 0.0f;
    }
}

// Smallest k in [0, k1] with (2k+1) A' >= 80 B' (the exact minimiser of F).
__device__ inline int grid_k(int64_t Bp, int64_t Ap, int k1) {
    if (Ap <= 0 || Bp <= 0) return 0;
    int k = (int)fminf(fmaxf(rintf((float)Bp * (40.0f / (float)Ap)), 0.0f), (float)k1);
    const int64_t b80 = 80 * Bp;
    while (k > 0 && (int64_t)(2 * k - 1) * Ap >= b80) --k;
    while (k < k1 && (int64_t)(2 * k + 1) * Ap < b80) ++k;
    return k;
}

__device__ inline void lex_min_shfl(int64_t& F, int64_t& K, int mask) {
    const int64_t of = __shfl_xor(F, mask, 64);
    const int64_t ok = __shfl_xor(K, mask, 64);
    if (pair_less(of, ok, F, K)) {
        F = of;
        K = ok;
    }
}

// grid: x = workgroups of m8_rows rows, y = pool chunks. The contrast set is
// k = 0..k1. Each wavefront keeps 16 RT rows; each lane holds 4 rows x 1
// column of every 16x16 output tile: lane group g = lane / 16 holds rows
// 4g..4g+3 of a tile, so groups g and g ^ 1 hold the 8 rows of one range.
// Screen: for any k, F = k^2 A' - 80 k B' is at least the continuous minimum
// -1600 B'^2 / A', so an element can match or beat a best F_b <= 0 only if
// B' >= s_b sqrt(A'), s_b = sqrt(-F_b / 1600). A range's code is the minimum
// over its 8 rows, so every row is screened against the smallest F_b among its
// range's rows (the largest s_b), rounded below. The bound is not strict, so
// ties stay candidates. How the matchers evaluate it on normalized columns is
// described with them below. Candidates go to a per-wavefront queue in LDS and
// are decided exactly in int64, one per lane (the FP32 k corrected by one
// step).
// F = 0 never improves a row: its best starts at (F = 0, the chunk's first
// position, k = 0) and positions only grow. So a row of a constant range
// (C = 0, hence B' = 0 and F >= 0 everywhere) and a padded row start from the
// mark kM8Excl in place of F = 0 (s_b near 9300: no element reaches its bound)
// and report F = 0 at the end. Each row's best is one packed word
// (F + 2^37) << 26 | position << 4 | k, which orders as (F, key) does within a
// row (0 >= F >= -1600 C > -2^37 for n = 64, positions below kM8MaxPool); lanes
// lower it with an LDS atomic minimum.
constexpr int kM8Queue = 64 + 4 * 64;  // a flush at 16 entries, then up to one tile's 256
constexpr int kM8MaxPool = 1 << 22;    // pool positions the packed best can hold
// F of a row that never queues (below every real F >= -1600 C > -2^37)
constexpr int64_t kM8Excl = -(1ll << 37) + 1;

__device__ inline uint64_t m8_pack(int64_t F, int pos, int k) {
    return ((uint64_t)(F + (1ll << 37)) << 26) | ((uint64_t)pos << 4) | (uint64_t)k;
}

__device__ inline int64_t m8_unpack_F(uint64_t v) { return (int64_t)(v >> 26) - (1ll << 37); }

// The exact decision of one candidate (row, pool position) given X = sum r' d'.
__device__ inline void m8_decide(int row, int pos, int X, const int32_t* nsr, uint64_t* best,
                                 const int64_t* __restrict__ Ad, const uint32_t* __restrict__ Sd,
                                 const float* __restrict__ Gd, int k1) {
    const int64_t Ap = Ad[pos];
    const int bi = (X << 6) + nsr[row] * (int)Sd[pos];  // B' = 64 X - sum r' S, exact
    const int64_t Bp = bi, b80 = 80 * Bp;
    int k = (int)__builtin_amdgcn_fmed3f(rintf((float)bi * Gd[pos]), 0.0f, (float)k1);
    if (Ap <= 0) k = 0;
    else if (k > 0 && (int64_t)(2 * k - 1) * Ap >= b80) --k;
    else if (k < k1 && (int64_t)(2 * k + 1) * Ap < b80) ++k;
    const int64_t F = (int64_t)(k * k) * Ap - (int64_t)(80 * k) * Bp;
    if (F <= 0) atomicMin(reinterpret_cast<unsigned long long*>(best + row), (unsigned long long)m8_pack(F, pos, k));
}

// ================================================================ MFMA grid matchers, normalized screen (B = 8)
// The grid matchers screen on normalized operands. Each pool domain's column
// holds d^_i = (64 d'_i - S) s with s = 1 / Q (FP16 form) or 4079 / Q (int8
// form, rounded to integers: |d^| <= 4079 sqrt(63) < 2^15, split as 256 h + l
// with h, l in -128..127), Q = sqrt(A') rounded below (s = 0 for a constant
// domain). The rows are r^ = r' - c with c the range's mean of r' rounded
// (FP16: |r^| <= 255, exact), for int8 moved into [max r' - 127, min r' + 128]
// so that every r^ fits in int8. In exact arithmetic
//   X^ = sum r^_i d^_i = s (64 sum r' d' - S sum r') = s B'
// (the d^ of a column sum to zero, so a shift of the rows changes nothing),
// and an element can match or beat a range's best F_b <= 0, which needs
// B' >= s_b sqrt(A'), only if X^ >= s_b s sqrt(A') >= s_b (FP16) or 4079 s_b
// (int8): a bound of the range alone. Computed X^ differ from the exact one by
// at most E per range:
//  * FP16: the FP16 roundings of d^ (relative 2^-11, the FP32 product 2^-23)
//    move it by at most 2^-10.99 ||r^|| ||d^|| + 2^-25 sum |r^| with ||d^|| = 8
//    sqrt(A') / Q, about 8, and the FP32 accumulation of 64 products and the
//    start value by below 0.3: E = ||r^|| / 120 + 0.5;
//  * int8: the rounding to integers moves each d^ by at most 0.5, the FP32
//    arithmetic before it by below 0.01: E = 0.51 sum |r^| + 2; the int32 sums
//    are exact.
// The bound enters the accumulators. The FP16 form's start at 2^15 - (s_b - E)
// and hold 2^15 + X^ - (s_b - E) in (0, 2^16) (|X^| and s_b are at most
// sqrt(C) <= 8160), compared as FP32 bit patterns with that of 2^15 (positive
// floats order as their bit patterns). The int8 form takes T = floor(4079 s_b
// - E - 8) and screens in two steps: one MFMA over the h parts alone, started
// at -Th with Th = ceil((T - 128 sum |r^|) / 256) (|sum r^ l| is at most 128
// sum |r^|), rules a tile out when every Xh - Th < 0; a tile that passes is
// redone with its second MFMA started at 256 Xh - T, and an element is a
// candidate iff the result is >= 0 (|values| < 2^29). The screen of a
// 16-column tile is one maximum over the lane's elements. Candidates are then
// decided exactly from the integer data: X = sum r' d' (FP16 dot products of
// integers with partial sums below 2^24), or int8 dot products of r^ with the
// columns d' = 128 h + l, X = sum r^ d' + c S.
// A pool stage (kM8Cols normalized columns) is copied from global memory
// straight into LDS (global_load_lds, 16 bytes a lane, no registers on the
// way) while the previous stage is matched: 8 chunks of 16 bytes per domain
// (FP16: the values 8u..8u+7; int8: u < 4 the h values 16u.., u >= 4 the l
// values 16(u - 4)..), chunk u of column c at c * 8 + (u ^ ((c >> 1) & 7)), so
// that 16 consecutive columns read one chunk each from distinct banks.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr float kN16Off = 32768.0f;      // 2^15
constexpr int kN16OffBits = 0x47000000;  // its FP32 bit pattern

__device__ inline int m8_chunk(int c, int u) { return c * 8 + (u ^ ((c >> 1) & 7)); }

// One copy of 16 bytes a lane from base + off (off per lane) into LDS: lane
// i's 16 bytes land at lds + 16 i (base and lds the same in every lane; lds
// passed in m0). The compiler's builtin for this instruction makes every
// later LDS read of the kernel wait for the copy to land, which would stall
// each stage on its successor's copy; issued here, nothing waits for it but
// the explicit vmcnt before the barrier that publishes the stage. It has no
// register results (its only outputs are in LDS), and its address registers
// are read when it issues. It writes m0, a register the compiler reserves and
// does not restore after inline assembly: the kernels that use it must not use
// m0 otherwise (none of their other instructions reads it: a test checks their
// assembly).
__device__ __forceinline__ void m8_copy_to_lds(const void* base, uint32_t off,
                                               const void __attribute__((address_space(3)))* lds) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
                 :
                 : "v"(off), "s"(base), "s"((uint32_t)(uintptr_t)lds)
                 : "memory");
}

// Exact decision of the wavefront's queued candidates (entry: row | position
// << kM8RowBits), one per lane, with X = sum r' d' from the integer rows (Ar,
// row wrow0 + row) and columns (Dx): FP16 r' and d' (dot products of pairs;
// partial sums below 2^24, exact), or int8 r' - c and the h | l halves of d' =
// 128 h + l (dot products of fours; X = sum (r' - c) d' + c S). Pairs and fours are read as whole words:
// a bit cast of one element of a wider vector register is not reliable here.
template <bool I8>
__device__ inline void m8_flush(int n, const uint2* q, const int32_t* nsr, uint64_t* best,
                                const void* __restrict__ Ar, int wrow0, const void* __restrict__ Dx,
                                const int64_t* __restrict__ Ad, const uint32_t* __restrict__ Sd,
                                const float* __restrict__ Gd, const int2* __restrict__ RC, int k1, int lane) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int i = lane; i < n; i += 64) {
        const uint2 en = q[i];
        const int row = (int)(en.x & ((1u << kM8RowBits) - 1u)), pos = (int)(en.x >> kM8RowBits);
        int X;
        if constexpr (I8) {
            const int* r = reinterpret_cast<const int*>(static_cast<const int8_t*>(Ar) + (int64_t)(wrow0 + row) * 64);
            const int* d = reinterpret_cast<const int*>(static_cast<const int8_t*>(Dx) + (int64_t)pos * 128);
            int xh = 0, xl = 0;
#pragma unroll 4
            for (int c = 0; c < 16; ++c) {
                const int rv = r[c];
                xh = __builtin_amdgcn_sdot4(rv, d[c], xh, false);
                xl = __builtin_amdgcn_sdot4(rv, d[16 + c], xl, false);
            }
            X = (xh << 7) + xl + RC[(wrow0 + row) >> 3].x * (int)Sd[pos];  // rows are r' - c
        } else {
            const h2* r = reinterpret_cast<const h2*>(static_cast<const _Float16*>(Ar) + (int64_t)(wrow0 + row) * 64);
            const h2* d = reinterpret_cast<const h2*>(static_cast<const _Float16*>(Dx) + (int64_t)pos * 64);
            float x = 0.0f;
#pragma unroll 4
            for (int c = 0; c < 32; ++c) x = __builtin_amdgcn_fdot2(r[c], d[c], x, false);
            X = (int)x;
        }
        m8_decide(row, pos, X, nsr, best, Ad, Sd, Gd, k1);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// grid: x = workgroups of m8_rows rows, y = pool chunks. Ar: the rows r' (FP16
// or int8); Dx: the exact columns (FP16 d', or int8 h | l); Dn: the normalized
// columns.
template <bool I8>
__device__ __forceinline__ void k_match_grid_body(
    const void* __restrict__ Ar, const int32_t* __restrict__ SR, const int32_t* __restrict__ SRp,
    const int64_t* __restrict__ CR, const int32_t* act_count, const void* __restrict__ Dx,
    const void* __restrict__ Dn, const uint32_t* __restrict__ Sd, const int64_t* __restrict__ Ad,
    const float* __restrict__ Gd, const int32_t* __restrict__ Jd, const Ctrl* ctrl, int k1, int n_chunks,
    Partial* __restrict__ part, int cg, int64_t* __restrict__ GB, const int2* __restrict__ RC) {
    constexpr int RT = m8_row_tiles(!I8), WR = 16 * RT;
    constexpr int kLoads = kM8Cols * 8 / (kM8Waves * 64);
    static_assert(WR <= (1 << kM8RowBits), "row index of a queue entry");
    static_assert(kM8Waves * kLoads * 64 == kM8Cols * 8, "a stage is whole 16-byte chunks per lane");
    __shared__ v4i sD[2][kM8Cols * 8];
    __shared__ uint2 sQueue[kM8Waves][kM8Queue];
    __shared__ uint64_t sBest[kM8Waves][WR];
    __shared__ int32_t sNsr[kM8Waves][WR];

    const int nrows = 8 * *act_count;
    const int row_blk = blockIdx.x * m8_rows(!I8);
    if (row_blk >= nrows) return;
    const int P = ctrl->pool_count;
    const int nca = active_chunks(P, cg, n_chunks);
    const int c = blockIdx.y;
    if (c >= nca) return;
    const int lo = (int)((int64_t)P * c / nca), hi = (int)((int64_t)P * (c + 1) / nca);

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane >> 4, c16 = lane & 15;
    const int wrow0 = row_blk + wave * WR;
    uint2* queue = sQueue[wave];
    uint64_t* best = sBest[wave];
    int32_t* nsr = sNsr[wave];

    // A operands: FP16 r^ = r' - c (c = the row's range mean of r', rounded), 8
    // values of each K half; int8 r^ as the rows were prepared, 16 values
    v8h af[RT][2];
    v4i a8[RT];
    float E[RT];    // error bound of X^ for the lane's output range
    int Lr[RT];     // int8: 128 sum |r' - c| of the lane's output range (the l part's largest size)
    float sig[RT];  // s_b of the lane's range
    int cw[RT];     // c of the lane's output range
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int arow = wrow0 + 16 * rt + c16;
        const v4i z = {0, 0, 0, 0};
        if constexpr (I8) {
            a8[rt] = arow < nrows
                         ? *reinterpret_cast<const v4i*>(static_cast<const int8_t*>(Ar) + (int64_t)arow * 64 + 16 * g)
                         : z;
        } else {
            const _Float16 ca =
                arow < nrows ? (_Float16)rintf((float)SRp[arow >> 3] * (1.0f / 64.0f)) : (_Float16)0.0f;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const v8h v = __builtin_bit_cast(
                    v8h, arow < nrows ? *reinterpret_cast<const v4i*>(static_cast<const _Float16*>(Ar) +
                                                                    (int64_t)arow * 64 + 32 * h + 8 * g)
                                      : z);
                af[rt][h] = v - ca;
            }
        }
        const int orow = wrow0 + 16 * rt + 4 * g;
        E[rt] = 0.0f;
        Lr[rt] = 0;
        cw[rt] = 0;
        if (orow < nrows) {
            const int q = orow >> 3;
            // sum r'^2 from sum r and C = 64 sum r^2 - (sum r)^2
            const int64_t s = SR[q], sp = SRp[q];
            const int64_t r2 = (CR[q] + s * s) / 64 - 256 * s + 64 * 16384;
            if constexpr (I8) {
                const int2 rc = RC[q];
                cw[rt] = rc.x;
                E[rt] = 0.51f * (float)rc.y + 2.0f;
                Lr[rt] = 128 * rc.y;
                (void)r2;
            } else {
                // ||r^||^2 = sum r'^2 - 2 c sum r' + 64 c^2
                const int64_t co = (int64_t)rintf((float)sp * (1.0f / 64.0f));
                cw[rt] = (int)co;
                E[rt] = sqrtf((float)(r2 - 2 * co * sp + 64 * co * co)) * (1.0f / 120.0f) + 0.5f;
            }
        }
    }
    for (int i = lane; i < WR; i += 64) {
        // k = 0 gives F = 0 for every domain; its smallest key is the chunk's first domain
        const int r = wrow0 + i;
        const bool live = r < nrows && CR[r >> 3] != 0;
        best[i] = m8_pack(live ? 0 : kM8Excl, lo, 0);
        nsr[i] = r < nrows ? -SRp[r >> 3] : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // A first bound before the search: 4 tiles of 16 domains spread over the
    // chunk, decided exactly (FP16: X = sum r^ d' + c S, products of integers
    // with partial sums below 64 * 255 * 1020 < 2^24; int8: X = 128 sum r^ h +
    // sum r^ l + c S). Without it every chunk would open with half of its first
    // elements queued.
    if (lo < hi) {
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            const int pos = lo + (int)((int64_t)(hi - lo) * (16 * st + c16) / 64);
            if constexpr (I8) {
                const int8_t* d = static_cast<const int8_t*>(Dx) + (int64_t)pos * 128 + 16 * g;
                const v4i bh = *reinterpret_cast<const v4i*>(d), bl = *reinterpret_cast<const v4i*>(d + 64);
                const int S = (int)Sd[pos];
                const v4i z = {0, 0, 0, 0};
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const v4i xh = __builtin_amdgcn_mfma_i32_16x16x64_i8(a8[rt], bh, z, 0, 0, 0);
                    const v4i xl = __builtin_amdgcn_mfma_i32_16x16x64_i8(a8[rt], bl, z, 0, 0, 0);
                    if (wrow0 + 16 * rt + 4 * g < nrows) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            m8_decide(16 * rt + 4 * g + e, pos, (xh[e] << 7) + xl[e] + cw[rt] * S, nsr, best, Ad, Sd,
                                      Gd, k1);
                    }
                }
            } else {
                const _Float16* d = static_cast<const _Float16*>(Dx) + (int64_t)pos * 64 + 8 * g;
                const v8h b0 = __builtin_bit_cast(v8h, *reinterpret_cast<const v4i*>(d));
                const v8h b1 = __builtin_bit_cast(v8h, *reinterpret_cast<const v4i*>(d + 32));
                const int S = (int)Sd[pos];
                const v4f z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    v4f x = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[rt][0], b0, z, 0, 0, 0);
                    x = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[rt][1], b1, x, 0, 0, 0);
                    if (wrow0 + 16 * rt + 4 * g < nrows) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            m8_decide(16 * rt + 4 * g + e, pos, (int)x[e] + cw[rt] * S, nsr, best, Ad, Sd, Gd, k1);
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    // accumulator start values: FP16 2^15 - (s_b - E) in four lanes of a tile
    // row; int8 -T (fine screen: 256 Xh + Xl - T >= 0) and -Th (coarse screen
    // on the h part alone: Xh - Th >= 0, Th = ceil((T - Lr) / 256), since
    // |Xl| <= 128 sum |r' - c| = Lr)
    v4f C[RT];
    int Ci[RT], Ch[RT];
    // A range's bound is the smallest F found for it so far, here or in any
    // other pool chunk: after each batch of decisions a workgroup publishes its
    // ranges' best F (real matches) with an atomic minimum and reads the
    // others' back, so chunks do not each rediscover what one has found. A
    // value read late is only looser.
    auto set_bounds = [&] {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const uint64_t* bb = best + 16 * rt + 8 * (g >> 1);
            uint64_t mb = bb[0];
#pragma unroll
            for (int e = 1; e < 8; ++e) mb = bb[e] < mb ? bb[e] : mb;
            int64_t F = m8_unpack_F(mb);
            const int orow = wrow0 + 16 * rt + 4 * g;
            if (orow < nrows && F != kM8Excl) {
                int64_t* gp = GB + (orow >> 3);
                if (F < 0 && c16 == 0 && (g & 1) == 0)
                    __hip_atomic_fetch_min(gp, F, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int64_t Fg = __hip_atomic_load(gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                F = Fg < F ? Fg : F;
            }
            sig[rt] = F < 0 ? __builtin_amdgcn_sqrtf((float)(-F) * (1.0f / 1600.0f)) * kM8Shrink : 0.0f;
            if constexpr (I8) {
                // 4079 s_b - E in FP32 (values below 2^25: roundings below 4, and
                // 8 taken off), then integers: Th = ceil((T - Lr) / 256)
                const int T = (int)floorf(kI8Scale * sig[rt] - E[rt] - 8.0f);
                Ci[rt] = -T;
                Ch[rt] = -((T - Lr[rt] + 255) >> 8);
            } else {
                const float c0 = kN16Off - (sig[rt] - E[rt]);
                C[rt] = v4f{c0, c0, c0, c0};
            }
        }
    };
    set_bounds();
    int qn = 0;  // queued candidates (the same in every lane)

    // this wavefront's share of a stage: chunks (kLoads wave + l) * 64 + lane
    // (columns past the chunk's end copy its last domain and are never queued)
    uint32_t off[kLoads];  // byte offsets of a full stage's chunks, from the stage's first column
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
        const int i = (kLoads * wave + l) * 64 + lane, col = i >> 3, u = (i & 7) ^ ((col >> 1) & 7);
        off[l] = (uint32_t)(col * 128 + 16 * u);
    }
    auto stage_dma = [&](v4i* dD, int b0, int n) {
        // the same in every lane; read from the first so that it sits in SGPRs
        const uint64_t bu = (uint64_t)(uintptr_t)(static_cast<const int8_t*>(Dn) + (int64_t)b0 * 128);
        const void* base = (const void*)(uintptr_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(bu >> 32)) << 32) |
                                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)bu));
        if (n == kM8Cols) {
#pragma unroll
            for (int l = 0; l < kLoads; ++l)
                m8_copy_to_lds(base, off[l], (const __attribute__((address_space(3))) void*)(dD + (kLoads * wave + l) * 64));
        } else {  // the chunk's last stage: columns past its end copy its last one
#pragma unroll
            for (int l = 0; l < kLoads; ++l) {
                const uint32_t o = (uint32_t)(min((int)(off[l] >> 7), n - 1) * 128) + (off[l] & 127u);
                m8_copy_to_lds(base, o, (const __attribute__((address_space(3))) void*)(dD + (kLoads * wave + l) * 64));
            }
        }
    };
    auto dma_wait = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };  // vmcnt(0)

    // nothing of the set-up may still be in flight in the loop
    dma_wait();
    if (lo < hi) {
        stage_dma(sD[0], lo, min(kM8Cols, hi - lo));
        dma_wait();
    }
    __syncthreads();
    // one 16-column tile for every row tile: the screen's value per element
    // (FP16: FP32 bits of 2^15 + X^ - (s_b - E); int8 fine: X^ - T; int8
    // coarse, the h part only: Xh - Th)
    auto tile = [&](const v4i* cD, int ct, bool coarse, v4i (&acc)[RT]) {
        const int col = 16 * ct + c16;
        const v4i q0 = cD[m8_chunk(col, g)];
        if constexpr (I8) {
            if (coarse) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const v4i ch = {Ch[rt], Ch[rt], Ch[rt], Ch[rt]};
                    acc[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a8[rt], q0, ch, 0, 0, 0);
                }
            } else {
                const v4i q1 = cD[m8_chunk(col, 4 + g)];
                const v4i z = {0, 0, 0, 0};
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const v4i xh = __builtin_amdgcn_mfma_i32_16x16x64_i8(a8[rt], q0, z, 0, 0, 0);
                    acc[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a8[rt], q1, (xh << 8) + Ci[rt], 0, 0, 0);
                }
            }
        } else {
            const v4i q1 = cD[m8_chunk(col, 4 + g)];
            const v8h b0 = __builtin_bit_cast(v8h, q0), b1 = __builtin_bit_cast(v8h, q1);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                v4f x = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[rt][0], b0, C[rt], 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[rt][1], b1, x, 0, 0, 0);
                acc[rt] = __builtin_bit_cast(v4i, x);
            }
        }
    };
    constexpr int kPass = I8 ? 0 : kN16OffBits;  // a candidate's screen value is at least this
    auto stage = [&](const v4i* cD, v4i* nD, int base) {
        const int nb = base + kM8Cols;
        if (nb < hi) stage_dma(nD, nb, min(kM8Cols, hi - nb));  // lands while this stage is matched
        // the start values as the stage begins, kept in registers (not rebuilt
        // from constants at every tile); a bound raised within the stage takes
        // effect at the next: the older one is looser, so the screen stays safe
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            if constexpr (I8) asm volatile("" : "+v"(Ch[rt]));
            else asm volatile("" : "+v"(C[rt]));
        }
        // the screen of every tile, without a branch: a bit per tile with a candidate
        uint32_t hits = 0;
#pragma unroll
        for (int ct = 0; ct < kM8ColTiles; ++ct) {
            v4i acc[RT];
            tile(cD, ct, true, acc);
            int mx = max(max(acc[0][0], acc[0][1]), acc[0][2]);
            mx = max(mx, acc[0][3]);
#pragma unroll
            for (int rt = 1; rt < RT; ++rt) {
                mx = max(max(mx, acc[rt][0]), acc[rt][1]);
                mx = max(max(mx, acc[rt][2]), acc[rt][3]);
            }
            hits |= __ballot(mx >= kPass) ? 1u << ct : 0u;
        }
        if (!hits) return;
        // slow path: the tiles with a candidate again, every element queued by ballot
        bool flushed = false;
        for (int ct = 0; ct < kM8ColTiles; ++ct) {
            if (!(hits & (1u << ct))) continue;
            v4i acc[RT];
            tile(cD, ct, false, acc);
            const int col = 16 * ct + c16;
            const bool colok = base + col < hi;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                bool cand[4];
                uint64_t m[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    cand[e] = colok && acc[rt][e] >= kPass;
                    m[e] = __ballot(cand[e]);
                }
                if ((m[0] | m[1] | m[2] | m[3]) == 0) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (m[e]) {
                        const int slot = qn + __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(m[e] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[e], 0u));
                        if (cand[e])
                            queue[slot] = make_uint2((uint32_t)(16 * rt + 4 * g + e) |
                                                         ((uint32_t)(base + col) << kM8RowBits),
                                                     0u);
                        qn += __popcll(m[e]);
                    }
                }
                // decided every 16 candidates: the bounds tighten early, so fewer
                // tiles take this path
                if (qn >= 16) {
                    m8_flush<I8>(qn, queue, nsr, best, Ar, wrow0, Dx, Ad, Sd, Gd, RC, k1, lane);
                    qn = 0;
                    flushed = true;
                }
            }
        }
        if (flushed) set_bounds();  // for the next stage
    };
    int buf = 0;
    for (int base = lo; base < hi; base += kM8Cols, buf ^= 1) {
        stage(sD[buf], sD[buf ^ 1], base);
        dma_wait();
        __syncthreads();
    }
    if (qn > 0) m8_flush<I8>(qn, queue, nsr, best, Ar, wrow0, Dx, Ad, Sd, Gd, RC, k1, lane);
    // per range: rows 8q..8q+7 are the 4 rows of lane group g and of g ^ 1
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int orow = wrow0 + 16 * rt + 4 * g;
        int64_t F = INT64_MAX, K = INT64_MAX;
        if (lo < hi && orow < nrows && c16 == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint64_t v = best[16 * rt + 4 * g + e];
                const int pos = (int)((v >> 4) & (uint64_t)(kM8MaxPool - 1)), k = (int)(v & 15u);
                const int64_t Fe = m8_unpack_F(v) == kM8Excl ? 0 : m8_unpack_F(v);
                const int64_t key = make_key(Jd[pos], (orow + e) & 7, k, Sd[pos]);
                if (pair_less(Fe, key, F, K)) {
                    F = Fe;
                    K = key;
                }
            }
        }
        lex_min_shfl(F, K, 16);
        if (c16 == 0 && (g & 1) == 0 && orow < nrows) {
            Partial pr;
            pr.F = F;
            pr.key = K;
            part[(int64_t)(orow >> 3) * n_chunks + c] = pr;
        }
    }
}

// ================================================================ FP32-FMA comparator (B = 8)
// The same search with the correlation in FP32 FMAs (exact: every partial sum
// is an integer below 2^24) and E decided in FP32, with no exact rescoring:
// it shows what plain single precision gets right and wrong.
__device__ inline int64_t ordered_float(float f) {
    const int32_t b = __float_as_int(f);
    return (int64_t)(b >= 0 ? b : (b ^ 0x7fffffff));
}

__device__ inline float float_from_ordered(int64_t o) {
    const int32_t b = (int32_t)o;
    return __int_as_float(b >= 0 ? b : (b ^ 0x7fffffff));
}

constexpr int kF32Tile = 64;  // domains per LDS stage

__device__ __forceinline__ void k_match_fp32_body(const uint8_t* __restrict__ img, int pitch,
                                                       const int32_t* __restrict__ act,
                                                       const int32_t* act_count,
                                                       const uint8_t* __restrict__ DDimg, int L,
                                                       int gx, const int32_t* __restrict__ Jd,
                                                       const Ctrl* ctrl, int k1, int n_chunks,
                                                       Partial* __restrict__ part, int cg) {
    constexpr int B = 8, n = 64, RPB = kBlock / 8;
    __shared__ float sD[kF32Tile * n];
    __shared__ float sS[kF32Tile], sA[kF32Tile];
    __shared__ uint8_t sR[RPB * n];
    const int nact = *act_count;
    const int q0 = blockIdx.x * RPB;
    if (q0 >= nact) return;
    const int P = ctrl->pool_count;
    const int nca = active_chunks(P, cg, n_chunks);
    const int c = blockIdx.y;
    if (c >= nca) return;
    const int lo = (int)((int64_t)P * c / nca), hi = (int)((int64_t)P * (c + 1) / nca);
#pragma unroll
    for (int e = threadIdx.x; e < RPB * n; e += kBlock) {
        const int lq = e / n, m = e % n, q = q0 + lq;
        uint8_t v = 0;
        if (q < nact) {
            const int yx = act[q];
            if (yx >= 0) v = img[(int64_t)((yx >> 16) + m / B) * pitch + (yx & 0xffff) + m % B];
        }
        sR[e] = v;
    }
    __syncthreads();
    const int lq = threadIdx.x >> 3, t = threadIdx.x & 7, q = q0 + lq;
    const uint8_t* rr = sR + lq * n;
    float r[n];
    float sr = 0.0f;
    {
        const int u = iso_inverse(t);
        const int a0 = iso_src(B, u, 0, 0);
        const int a1 = iso_src(B, u, 1, 0) - a0, a2 = iso_src(B, u, 0, 1) - a0;
#pragma unroll
        for (int m = 0; m < n; ++m) {
            r[m] = (float)rr[a0 + a1 * (m / B) + a2 * (m % B)];
            sr += r[m];
        }
    }
    float bestF = INFINITY;
    int bestP = lo, bestK = 0;
    for (int base = lo; base < hi; base += kF32Tile) {
        const int cnt = min(kF32Tile, hi - base);
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * n; e += kBlock) {
            const int d = e / n, m = e % n;
            const int j = Jd[base + d];
            const int y = (j / gx) * L, x = (j % gx) * L;
            const uint8_t* px = DDimg + (int64_t)(y + 2 * (m / B)) * pitch + x + 2 * (m % B);
            sD[e] = (float)((int)px[0] + px[1] + px[pitch] + px[pitch + 1]);
        }
        __syncthreads();
        for (int d = threadIdx.x; d < cnt; d += kBlock) {
            float s = 0.0f, s2 = 0.0f;
            for (int m = 0; m < n; ++m) {
                const float v = sD[d * n + m];
                s += v;
                s2 = fmaf(v, v, s2);
            }
            sS[d] = s;
            sA[d] = fmaf((float)n, s2, -s * s);
        }
        __syncthreads();
        for (int d = 0; d < cnt; ++d) {
            float p = 0.0f;
#pragma unroll
            for (int m = 0; m < n; ++m) p = fmaf(r[m], sD[d * n + m], p);
            const float Bp = fmaf((float)n, p, -sr * sS[d]);
            const float Ap = sA[d];
            float kf = Ap > 0.0f ? fminf(fmaxf(rintf(40.0f * Bp / Ap), 0.0f), (float)k1) : 0.0f;
            const float F = kf * fmaf(kf, Ap, -80.0f * Bp);
            if (F < bestF) {
                bestF = F;
                bestP = base + d;
                bestK = (int)kf;
            }
        }
    }
    int64_t outF = INT64_MAX, outK = INT64_MAX;
    if (lo < hi) {
        outF = ordered_float(bestF);
        outK = make_key(Jd[bestP], t, bestK, 0);
    }
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) lex_min_shfl(outF, outK, m);
    if (q < nact && t == 0) {
        Partial pr;
        pr.F = outF;
        pr.key = outK;
        part[(int64_t)q * n_chunks + c] = pr;
    }
}

// Result of the FP32 comparator: its own argmin and FP32 E, plus the exact
// e_num of the candidate it chose (recomputed in integers for reporting).
__device__ __forceinline__ void k_reduce_fp32_body(const uint8_t* __restrict__ img, int pitch,
                                                        int L, int gx, const int32_t* __restrict__ act,
                                                        const int32_t* act_count,
                                                        const Partial* __restrict__ part,
                                                        int n_chunks, int cg, const Ctrl* ctrl,
                                                        fic_match* __restrict__ out) {
    constexpr int B = 8, n = 64;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= *act_count) return;
    const int nca = active_chunks(ctrl->pool_count, cg, n_chunks);
    int64_t F = INT64_MAX, K = INT64_MAX;
    for (int c = 0; c < nca; ++c)
        if (pair_less(part[(int64_t)q * n_chunks + c].F, part[(int64_t)q * n_chunks + c].key, F, K)) {
            F = part[(int64_t)q * n_chunks + c].F;
            K = part[(int64_t)q * n_chunks + c].key;
        }
    fic_match m;
    m.flags = 0;
    m.pad_ = 0;
    const int yx = act[q];
    if (yx < 0 || K == INT64_MAX) {
        m.e_num = -1;
        m.dom = -1;
        m.iso = m.s_idx = m.k = 0;
        m.q_o = 0;
        m.E = -1.0f;
        out[q] = m;
        return;
    }
    const int j = (int)(K >> 27), t = (int)((K >> 24) & 7), k = (int)((K >> 20) & 15);
    const int dy = (j / gx) * L, dx = (j % gx) * L;
    const uint8_t* R = img + (int64_t)(yx >> 16) * pitch + (yx & 0xffff);
    int64_t sr = 0, sr2 = 0, sd = 0, sd2 = 0, pr = 0;
    for (int i = 0; i < B; ++i)
        for (int cc = 0; cc < B; ++cc) {
            const int src = iso_src(B, t, i, cc);
            const uint8_t* px = img + (int64_t)(dy + 2 * (src / B)) * pitch + dx + 2 * (src % B);
            const int64_t d = (int64_t)px[0] + px[1] + px[pitch] + px[pitch + 1];
            const int64_t r = R[i * pitch + cc];
            sr += r;
            sr2 += r * r;
            sd += d;
            sd2 += d * d;
            pr += r * d;
        }
    const int64_t Ap = n * sd2 - sd * sd, Bp = n * pr - sr * sd, C = n * sr2 - sr * sr;
    m.e_num = (int64_t)(k * k) * Ap - (int64_t)(80 * k) * Bp + 1600 * C;
    m.dom = j;
    m.iso = (uint8_t)t;
    m.s_idx = (uint8_t)k;
    m.k = (uint8_t)k;
    m.q_o = (int16_t)floordiv64(2 * (40 * sr - k * sd) + 40 * n, 80 * (int64_t)n);
    m.E = (float_from_ordered(F) + 1600.0f * (float)C) / (1600.0f * (float)n);
    out[q] = m;
}


// ================================================================ FP16 MFMA matcher for small contrast sets
// The 4 x 4, 8 x 8 and 16 x 16 quadtree levels with one or two predefined
// contrast values (Section 3.1), on FP16 MFMA. Operands are centred:
// r' = r - 128 in [-128, 127] and d'' = d' - 510 in [-510, 510] are exact in
// FP16, and every partial sum of X = sum r' d'' is an integer of magnitude at
// most n * 128 * 510 < 2^24 (n <= 256), so the FP32 accumulator holds X
// exactly whatever the order of the additions. B' is a covariance, so
// B' = n X - (sum r')(sum d''), and for each nonzero value k of the set
// G = k A' - 80 B' = (k A' + 80 (sum r')(sum d'')) - 80 n X is an integer:
// |G| < 2^31 at B = 4 (Cauchy-Schwarz, |B'| <= sqrt(A' C)), so it is computed
// in 32-bit integers there, and in 64-bit integers (one multiply-add of the
// converted X into a per-column term) at B = 8 and 16. The 4 rows a lane
// holds are isometries of one range, so the per-column term k A' + 80 (sum
// r')(sum d'') is formed once per column. F = k G orders like G for a fixed
// k > 0, so each lane keeps, per row and per nonzero value, the running
// minimum of G and its position, visiting positions in ascending order with
// strict compares (the first occurrence wins); the values and the 16 lanes of
// a row are merged lexicographically on (F, position, contrast index) at the
// end. k = 0 gives F = 0 for every domain: a set holding 0 (its first value,
// the set being increasing) adds the candidate (0, the chunk's first
// position, 0). The pool is short at these levels (a few hundred domains),
// where a screen would send a large share of the elements to an exact
// decision; this epilogue is a handful of integer instructions per element.
// The range blocks are staged in LDS and turned into the inverse-isometry
// rows in registers by the kernel itself.
constexpr int kMqWaves = 4;
constexpr int mq_row_tiles(int B) { return B == 16 ? 1 : 2; }
constexpr int mq_rows(int B) { return kMqWaves * 16 * mq_row_tiles(B); }  // rows per workgroup
constexpr int mq_cols(int B) { return B == 16 ? 32 : (B == 8 ? 64 : 128); }  // pool domains per LDS stage
constexpr int kMqMaxPool = 1 << 21;
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

// Operand shapes: B = 8, 16 take v_mfma_f32_16x16x32_f16 (K = 32 per
// instruction, 8 halves per lane); B = 4 (n = 16) takes
// v_mfma_f32_16x16x16_f16 (K = 16, 4 halves per lane). LDS holds each column
// in U-byte units, one unit of padding per column.
template <int B> struct MqShape {
    static constexpr int KW = 32, KG = B * B / 32, U = 16;
    using AF = v8h;
    using LU = v4i;
    __device__ static v4f mfma(AF a, AF b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <> struct MqShape<4> {
    static constexpr int KW = 16, KG = 1, U = 8;
    using AF = v4h;
    using LU = uint2;
    __device__ static v4f mfma(AF a, AF b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
};

// Columns of the small-set MFMA matcher: the n values d'' = d' - 510 of each
// pool domain in FP16 at Dh (2n bytes per domain), and S, A', j as for the
// VALU matcher. n / 16 lanes per domain, 16 values each.
template <int B>
__device__ __forceinline__ void k_pool_prep_mq_body(const uint8_t* __restrict__ img, int pitch, int L,
                                                         int gx, const int32_t* __restrict__ pool,
                                                         int identity_total, Ctrl* ctrl,
                                                         _Float16* __restrict__ Dh, uint32_t* __restrict__ Sd,
                                                         int64_t* __restrict__ Ad, int32_t* __restrict__ Jd) {
    constexpr int n = B * B, PER = 16, TPD = n / PER;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (identity_total >= 0 && g == 0) {
        ctrl->pool_count = identity_total;
        ctrl->passed = identity_total;
    }
    const int count = identity_total >= 0 ? identity_total : ctrl->pool_count;
    const int p = g / TPD, sub = g % TPD;
    const bool ok = p < count;
    uint32_t s = 0;
    uint64_t q = 0;
    int j = 0;
    if (ok) {
        j = identity_total >= 0 ? p : pool[p];
        const int y = (j / gx) * L, x = (j % gx) * L;
        uint32_t* hd = reinterpret_cast<uint32_t*>(Dh + (int64_t)p * n + sub * PER);
#pragma unroll
        for (int w = 0; w < PER / 2; ++w) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int m = sub * PER + 2 * w + b, i = m / B, c = m % B;
                const uint8_t* px = img + (int64_t)(y + 2 * i) * pitch + x + 2 * c;
                const uint32_t d = (uint32_t)px[0] + px[1] + px[pitch] + px[pitch + 1];
                s += d;
                q += (uint64_t)d * d;
                v |= (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)((int)d - 510)) << (16 * b);
            }
            hd[w] = v;
        }
    }
#pragma unroll
    for (int m = 1; m < TPD; m <<= 1) {
        s += __shfl_xor(s, m, 64);
        q += __shfl_xor(q, m, 64);
    }
    if (ok && sub == 0) {
        Sd[p] = s;
        Ad[p] = (int64_t)n * (int64_t)q - (int64_t)s * (int64_t)s;
        Jd[p] = j;
    }
}

// LDS of the small-set MFMA matcher (one struct, so that a kernel holding
// several matchers can overlay them).
template <int B, int NK, int COLS_ = mq_cols(B)>
struct MqSmem {
    static constexpr int n = B * B, COLS = COLS_, CH = 2 * n / MqShape<B>::U + 1;
    static constexpr int NR = mq_rows(B) / 8;
    using GT = typename std::conditional<(B <= 4), int32_t, int64_t>::type;
    typename MqShape<B>::LU sB[2][COLS * CH];
    GT sKA[2][NK][COLS];      // k A' per column and nonzero value
    int32_t sSdd[2][COLS];    // sum d'' = S - 510 n
    uint8_t sPix[NR * n];
    int32_t sSR[NR];
};

// Workgroup (bx, by): rows bx * mq_rows(B) .. (8 per range), pool chunk by.
// NK: the number of nonzero values in the set (1 or 2).
// COLS_: pool domains per LDS stage (the level default, or fewer where LDS is short).
template <int B, int NK, int COLS_ = mq_cols(B)>
__device__ __forceinline__ void k_match_mfq_body(
    MqSmem<B, NK, COLS_>& sm, int bx, int by, const uint8_t* __restrict__ img, int pitch,
    const int32_t* __restrict__ act, const int32_t* act_count, const _Float16* __restrict__ Dh,
    const uint32_t* __restrict__ Sd, const int64_t* __restrict__ Ad, const int32_t* __restrict__ Jd,
    const Ctrl* ctrl, const KSet& ks, int n_chunks, int cg, Partial* __restrict__ part,
    int32_t* __restrict__ SRout, int64_t* __restrict__ CRout) {
    using Sh = MqShape<B>;
    using AF = typename Sh::AF;
    using GT = typename MqSmem<B, NK, COLS_>::GT;
    constexpr int n = B * B, KG = Sh::KG, KW = Sh::KW, RT = mq_row_tiles(B), ROWS = mq_rows(B);
    constexpr int NR = ROWS / 8;                // ranges per workgroup
    constexpr int COLS = COLS_, CT = COLS / 16;
    constexpr int CPC = n / 8;                  // 16-byte chunks per column in memory
    constexpr int CH = MqSmem<B, NK, COLS_>::CH;  // LDS stride per column (one unit of padding)
    constexpr int NT = kMqWaves * 64;
    constexpr int NLD = COLS * CPC / NT;        // chunks per thread per stage
    static_assert(COLS * CPC % NT == 0 && COLS <= NT, "stage split over the workgroup");
    auto& sB = sm.sB;
    auto& sKA = sm.sKA;
    auto& sSdd = sm.sSdd;
    auto& sPix = sm.sPix;
    auto& sSR = sm.sSR;

    const int nact = *act_count, nrows = 8 * nact;
    const int row_blk = bx * ROWS;
    if (row_blk >= nrows) return;
    const int P = ctrl->pool_count;
    const int nca = active_chunks(P, cg, n_chunks);
    const int c = by;
    if (c >= nca) return;
    const int lo = (int)((int64_t)P * c / nca), hi = (int)((int64_t)P * (c + 1) / nca);

    // the set: its nonzero values in order (with their indices), and whether it holds 0
    int kz0 = 0, kz1 = 0, u0 = 0, u1 = 0;
    bool zero_in = false, have0 = false;
#pragma unroll
    for (int u = 0; u < kSmallMax; ++u) {
        if (u < ks.n) {
            const int k = ks.k[u];
            if (k == 0) {
                zero_in = true;
            } else if (!have0) {
                kz0 = k;
                u0 = u;
                have0 = true;
            } else {
                kz1 = k;
                u1 = u;
            }
        }
    }

    // a thread's share of one stage: NLD 16-byte chunks, and (first COLS threads)
    // its column's A' and S
    v4i ld[NLD];
    int64_t ldA = 0;
    uint32_t ldS = 0;
    auto load_stage = [&](int b0, int cnt) {
        const v4i zz = {0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int ci = threadIdx.x + NT * i, col = ci / CPC, uu = ci % CPC;
            ld[i] = col < cnt ? *reinterpret_cast<const v4i*>(Dh + (int64_t)(b0 + col) * n + 8 * uu) : zz;
        }
        if (threadIdx.x < COLS) {
            ldA = (int)threadIdx.x < cnt ? Ad[b0 + threadIdx.x] : 0;
            ldS = (int)threadIdx.x < cnt ? Sd[b0 + threadIdx.x] : 0u;
        }
    };
    auto store_stage = [&](int bf) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int ci = threadIdx.x + NT * i, col = ci / CPC, uu = ci % CPC;
            if constexpr (Sh::U == 16) {
                sB[bf][col * CH + uu] = ld[i];
            } else {  // two 8-byte units per 16-byte chunk
                sB[bf][col * CH + 2 * uu] = make_uint2((uint32_t)ld[i][0], (uint32_t)ld[i][1]);
                sB[bf][col * CH + 2 * uu + 1] = make_uint2((uint32_t)ld[i][2], (uint32_t)ld[i][3]);
            }
        }
        if (threadIdx.x < COLS) {
            const int t = threadIdx.x;
            // k A' <= 10 n^2 510^2: below 2^31 for n = 16
#pragma unroll
            for (int m = 0; m < NK; ++m) sKA[bf][m][t] = (GT)(m == 0 ? kz0 : kz1) * (GT)ldA;
            sSdd[bf][t] = (int)ldS - 510 * n;
        }
    };
    // the first stage's loads are in flight while the ranges are staged
    if (lo < hi) load_stage(lo, min(COLS, hi - lo));

    // the workgroup's range blocks, their sums and C (written out by chunk 0):
    // each thread stages SPT consecutive pixels of one range row, all its loads
    // issued together
    const int q0 = row_blk >> 3;
    {
        constexpr int SPT = NR * n / NT;
        static_assert(B % SPT == 0 && NR * n == SPT * NT, "a thread's pixels lie in one row");
        const int lq = threadIdx.x / (n / SPT), m0 = (threadIdx.x % (n / SPT)) * SPT, q = q0 + lq;
        const int yx = q < nact ? act[q] : -1;
        uint8_t v[SPT];
        const uint8_t* src = img + (yx >= 0 ? (int64_t)((yx >> 16) + m0 / B) * pitch + (yx & 0xffff) + m0 % B : 0);
#pragma unroll
        for (int i = 0; i < SPT; ++i) v[i] = yx >= 0 ? src[i] : 0;
#pragma unroll
        for (int i = 0; i < SPT; ++i) sPix[lq * n + m0 + i] = v[i];
    }
    __syncthreads();
    {
        constexpr int TPQ = NT / NR, PPT = n / TPQ;  // threads per range, pixels per thread
        static_assert(64 % TPQ == 0, "a range's threads share a wavefront");
        const int lq = threadIdx.x / TPQ, sub = threadIdx.x % TPQ;
        int s = 0, s2 = 0;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int v = sPix[lq * n + sub * PPT + i];
            s += v;
            s2 += v * v;
        }
#pragma unroll
        for (int m = 1; m < TPQ; m <<= 1) {
            s += __shfl_xor(s, m, 64);
            s2 += __shfl_xor(s2, m, 64);
        }
        if (sub == 0) {
            sSR[lq] = s;
            const int q = q0 + lq;
            if (c == 0 && q < nact) {
                SRout[q] = s;
                CRout[q] = (int64_t)n * s2 - (int64_t)s * s;
            }
        }
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const int wrow0 = row_blk + wave * 16 * RT;

    // A operands: row 16 rt + c16 of the wave, K = KW kg + (KW / 4) g + e
    AF af[RT][KG];
    int srd80[RT];  // 80 sum r' of the range of the lane's 4 output rows
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int arow = wrow0 + 16 * rt + c16;
        const int lq = (arow - row_blk) >> 3, t = arow & 7;
        const int u = iso_inverse(t);
        const int a0 = iso_src(B, u, 0, 0);
        const int a1 = iso_src(B, u, 1, 0) - a0, a2 = iso_src(B, u, 0, 1) - a0;
        const uint8_t* rr = sPix + lq * n;
#pragma unroll
        for (int kg = 0; kg < KG; ++kg)
#pragma unroll
            for (int e = 0; e < KW / 4; ++e) {
                const int m = KW * kg + (KW / 4) * g + e;
                af[rt][kg][e] = (_Float16)((int)rr[a0 + a1 * (m / B) + a2 * (m % B)] - 128);
            }
        const int orow = wrow0 + 16 * rt + 4 * g;
        srd80[rt] = 80 * (sSR[(orow - row_blk) >> 3] - 128 * n);
    }
    // running minimum of G per row of the lane and nonzero value, with its position
    GT bG[RT][4][NK];
    int bP[RT][4][NK];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int m = 0; m < NK; ++m) {
                bG[rt][e][m] = std::numeric_limits<GT>::max();
                bP[rt][e][m] = lo;
            }
    constexpr int kN80 = 80 * n;

    if (lo < hi) store_stage(0);
    __syncthreads();
    int buf = 0;
    for (int base = lo; base < hi; base += COLS, buf ^= 1) {
        const int nb = base + COLS;
        if (nb < hi) load_stage(nb, min(COLS, hi - nb));  // in flight while this stage is matched
        const int cnt = min(COLS, hi - base);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int col = 16 * ct + c16;
            AF bq[KG];
#pragma unroll
            for (int kg = 0; kg < KG; ++kg) bq[kg] = __builtin_bit_cast(AF, sB[buf][col * CH + 4 * kg + g]);
            v4f acc[RT];
            const v4f zf = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                v4f x = zf;
#pragma unroll
                for (int kg = 0; kg < KG; ++kg) x = Sh::mfma(af[rt][kg], bq[kg], x);
                acc[rt] = x;
            }
            if (col < cnt) {
                GT ka[NK];
#pragma unroll
                for (int m = 0; m < NK; ++m) ka[m] = sKA[buf][m][col];
                const int sdd = sSdd[buf][col];
                const int pos = base + col;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    GT yc[NK];  // k A' + 80 (sum r')(sum d'')
#pragma unroll
                    for (int m = 0; m < NK; ++m) {
                        if constexpr (B <= 4)
                            yc[m] = (GT)((uint32_t)ka[m] + (uint32_t)srd80[rt] * (uint32_t)sdd);
                        else
                            yc[m] = ka[m] + (int64_t)srd80[rt] * (int64_t)sdd;
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int x = (int)acc[rt][e];  // an exact integer below 2^24
#pragma unroll
                        for (int m = 0; m < NK; ++m) {
                            GT gv;
                            if constexpr (B <= 4)
                                gv = (GT)((uint32_t)yc[m] - (uint32_t)kN80 * (uint32_t)x);
                            else
                                gv = yc[m] - (int64_t)kN80 * (int64_t)x;
                            if (gv < bG[rt][e][m]) {
                                bG[rt][e][m] = gv;
                                bP[rt][e][m] = pos;
                            }
                        }
                    }
                }
            }
        }
        // the other buffer was last read in the previous stage, before its barrier
        if (nb < hi) store_stage(buf ^ 1);
        __syncthreads();
    }
    // per row: the lane's best (F, position << 1 | contrast index) over its values,
    // then over the 16 column lanes of the row, lexicographic
    int64_t bF[RT][4];
    int bPU[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            bF[rt][e] = zero_in ? 0 : INT64_MAX;
            bPU[rt][e] = lo << 1;
#pragma unroll
            for (int m = 0; m < NK; ++m) {
                if (bG[rt][e][m] == std::numeric_limits<GT>::max()) continue;
                const int64_t F = (int64_t)(m == 0 ? kz0 : kz1) * (int64_t)bG[rt][e][m];
                const int pu = (bP[rt][e][m] << 1) | (m == 0 ? u0 : u1);
                if (F < bF[rt][e] || (F == bF[rt][e] && pu < bPU[rt][e])) {
                    bF[rt][e] = F;
                    bPU[rt][e] = pu;
                }
            }
#pragma unroll
            for (int m = 1; m < 16; m <<= 1) {
                const int64_t of = __shfl_xor(bF[rt][e], m, 64);
                const int op = __shfl_xor(bPU[rt][e], m, 64);
                if (of < bF[rt][e] || (of == bF[rt][e] && op < bPU[rt][e])) {
                    bF[rt][e] = of;
                    bPU[rt][e] = op;
                }
            }
        }
    // per range: rows 8q..8q+7 are the 4 rows of lane group g and of g ^ 1
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int orow = wrow0 + 16 * rt + 4 * g;
        int64_t F = INT64_MAX, K = INT64_MAX;
        if (lo < hi && orow < nrows && c16 == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (bF[rt][e] == INT64_MAX) continue;
                const int pos = bPU[rt][e] >> 1, u = bPU[rt][e] & 1;
                const int64_t key = make_key(Jd[pos], (orow + e) & 7, u, Sd[pos]);
                if (pair_less(bF[rt][e], key, F, K)) {
                    F = bF[rt][e];
                    K = key;
                }
            }
        }
        lex_min_shfl(F, K, 16);
        if (c16 == 0 && (g & 1) == 0 && orow < nrows) {
            Partial pr;
            pr.F = F;
            pr.key = K;
            part[(int64_t)(orow >> 3) * n_chunks + c] = pr;
        }
    }
}

// ================================================================ table-driven launches
// Every quadtree kernel reads its image's arguments from tab[blockIdx.z] (a
// batch, TAB = true) or from the by-value a0 (one image, TAB = false). The
// choice is a template parameter so that either source stays a uniform
// (scalar) load. Workgroups beyond an image's own grid return at once.
template <bool TAB>
__device__ inline const Lvl& lvl_of(const Lvl& a0, const Lvl* __restrict__ tab) {
    if constexpr (TAB)
        return tab[blockIdx.z];
    else
        return a0;
}
#define FIC_LV const Lvl& a = lvl_of<TAB>(a0, tab)

// Default matcher chunk (domains per pool chunk) for a level.
int match_chunk_domains(int B) {
    switch (B) {
        case 2: return MatchTile<2>::CG;
        case 4: return MatchTile<4>::CG;
        case 8: return MatchTile<8>::CG;
        default: return MatchTile<16>::CG;
    }
}

template <bool TAB>
__global__ void kt_act_full(Lvl a0, const Lvl* __restrict__ tab, int reset) {
    FIC_LV;
    k_act_full_body(a.act, a.H / a.B, a.W / a.B, a.B, a.ctrl, a.lv, reset);
}

template <bool TAB>
__global__ void kt_act_from_yx(Lvl a0, const Lvl* __restrict__ tab, const int32_t* yx, int n) {
    FIC_LV;
    k_act_from_yx_body(a.act, yx, n, a.H, a.W, a.B, a.ctrl);
}

// The level's active list (every range of the grid) and the encode's
// counters, as kt_act_full writes them, from thread t0 of nthr.
__device__ __forceinline__ void act_full_part(const Lvl& a, int t0, int nthr) {
    const int gxr = a.W / a.B, n = (a.H / a.B) * gxr;
    if (t0 == 0) {
        a.ctrl->act_count[a.lv] = n;
        a.ctrl->n_codes = 0;
        a.ctrl->lvl_base[a.lv] = 0;
    }
    for (int q = t0; q < n; q += nthr) {
        const int ry = q / gxr, rx = q - ry * gxr;
        a.act[q] = ((ry * a.B) << 16) | (rx * a.B);
    }
}

template <int L, bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_score_cells(Lvl a0, const Lvl* __restrict__ tab,
                                                              const int64_t* __restrict__ T, int fill_act) {
    FIC_LV;
    __shared__ CellSmem<L> sm;
    // also level 0's active list: one launch fewer
    if (fill_act)
        act_full_part(a, (blockIdx.y * gridDim.x + blockIdx.x) * kBlock + threadIdx.x,
                      gridDim.x * gridDim.y * kBlock);
    k_pool_score_cells_body<L>(sm, blockIdx.x, blockIdx.y, a.img, a.pitch, a.gx, a.gy, T, a.M, a.key, a.pctrl);
}

// Every level of one image in one launch (levels at tab[0..], each with cell
// side L = B / 2 in 1, 2, 4, 8): workgroups [end[l - 1], end[l]) score level
// l's tiles, row by row of tiles; level 0's also write its active list.
__global__ __launch_bounds__(kBlock) void kt_pool_score_cells_levels(const Lvl* __restrict__ tab, int4 end,
                                                                     const int64_t* __restrict__ T) {
    __shared__ CellSmemAny sm;
    const int b = blockIdx.x;
    const int l = (b >= end.x) + (b >= end.y) + (b >= end.z);
    const int base = l == 0 ? 0 : l == 1 ? end.x : l == 2 ? end.y : end.z;
    const Lvl& a = tab[l];
    const int tw = sc_tx(a.L), lb = b - base, nbx = (a.gx + tw - 1) / tw;
    const int tbx = lb % nbx, tby = lb / nbx;
    if (l == 0) act_full_part(a, lb * kBlock + threadIdx.x, end.x * kBlock);
    switch (a.L) {
        case 1: k_pool_score_cells_body<1>(sm.l1, tbx, tby, a.img, a.pitch, a.gx, a.gy, T, a.M, a.key, a.pctrl); break;
        case 2: k_pool_score_cells_body<2>(sm.l2, tbx, tby, a.img, a.pitch, a.gx, a.gy, T, a.M, a.key, a.pctrl); break;
        case 4: k_pool_score_cells_body<4>(sm.l4, tbx, tby, a.img, a.pitch, a.gx, a.gy, T, a.M, a.key, a.pctrl); break;
        default: k_pool_score_cells_body<8>(sm.l8, tbx, tby, a.img, a.pitch, a.gx, a.gy, T, a.M, a.key, a.pctrl); break;
    }
}

template <int SIDE, bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_score(Lvl a0, const Lvl* __restrict__ tab,
                                                        const int64_t* __restrict__ T) {
    FIC_LV;
    if ((int64_t)blockIdx.x * kBlock >= (int64_t)a.total * ScoreShape<SIDE>::TPD) return;
    k_pool_score_body<SIDE>(a.img, a.pitch, a.L, a.gx, a.total, T, a.M, a.key, a.pctrl);
}

template <int SIDE, bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_var(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    if ((int64_t)blockIdx.x * kBlock >= (int64_t)a.total * ScoreShape<SIDE>::TPD) return;
    k_pool_var_body<SIDE>(a.img, a.pitch, a.L, a.gx, a.total, a.kv, a.M, a.key, a.pctrl);
}

// Copy of the level's final pool list (for the bitstream).
template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_copy_pool(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    if (!a.pools_out) return;
    const int n = a.pctrl->pool_count;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) a.pools_out[i] = a.pool[i];
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_floor_bound(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    k_floor_bound_body(a.key, a.total, a.min_pool, a.rank, a.sel_shift, a.bound_chunk, a.pctrl);
}

__device__ inline CompactArgs pool_args(const Lvl& a) {
    CompactArgs c{};
    c.kind = 0;
    c.total = a.total;
    c.min_pool = a.min_pool;
    c.M = a.M;
    c.key = a.key;
    return c;
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_count(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    const int nblk = (a.total + kBlock * kPoolItems - 1) / (kBlock * kPoolItems);
    if ((int)blockIdx.x >= nblk) return;
    k_pool_count_body(pool_args(a), a.pctrl, a.pblk);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_scatter(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    const int nblk = (a.total + kBlock * kPoolItems - 1) / (kBlock * kPoolItems);
    if ((int)blockIdx.x >= nblk) return;
    k_pool_scatter_body(pool_args(a), a.pctrl, a.pblk, nblk, a.pool);
}

template <bool TAB>
__global__ __launch_bounds__(1024) void kt_floor_select(Lvl a0, const Lvl* __restrict__ tab, int direct) {
    FIC_LV;
    k_floor_select_body(a.key, a.total, a.min_pool, a.rank, a.sel_shift, a.pool, a.pctrl,
                        direct && a.total <= kSelDirect, a.M);
}

template <int B, bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_prep(Lvl a0, const Lvl* __restrict__ tab, int filtered) {
    FIC_LV;
    if ((int64_t)blockIdx.x * kBlock >= (int64_t)a.total * PrepShape<B>::TPD) return;
    k_pool_prep_body<B>(a.img, a.pitch, a.L, a.gx, a.pool, filtered ? -1 : a.total, a.pctrl, a.hl,
                        a.sd, a.ad, a.jd);
}

template <int B, int MODE, bool TAB>
__global__ __launch_bounds__(kBlock) void kt_match(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    __shared__ MatchSmem<B, MODE> sm;
    k_match_body<B, MODE>(sm, blockIdx.x, blockIdx.y, a.img, a.pitch, a.act, a.ctrl->act_count + a.lv, a.hl, a.sd, a.ad, a.jd,
                          a.pctrl, a.ks, a.nc, a.part, a.sr, a.cr, a.cg);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_prep_i8(Lvl a0, const Lvl* __restrict__ tab, int filtered) {
    FIC_LV;
    if ((int64_t)blockIdx.x * kBlock >= (int64_t)a.total * 4) return;
    if (a.var == kVarMfma16)
        k_pool_prep_m8_body<true>(a.img, a.pitch, a.L, a.gx, a.pool, filtered ? -1 : a.total, a.pctrl,
                                  a.dh, a.dl, a.sd, a.ad, a.jd, a.gd);
    else
        k_pool_prep_m8_body<false>(a.img, a.pitch, a.L, a.gx, a.pool, filtered ? -1 : a.total, a.pctrl,
                                   a.dh, a.dl, a.sd, a.ad, a.jd, a.gd);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_range_prep_i8(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    if (a.var == kVarMfma16)
        k_range_prep_m8_body<true>(a.img, a.pitch, a.act, a.ctrl->act_count + a.lv, a.ar, a.sr, a.srp, a.cr, a.gb,
                                   a.rc, a.gbseed, a.W);
    else
        k_range_prep_m8_body<false>(a.img, a.pitch, a.act, a.ctrl->act_count + a.lv, a.ar, a.sr, a.srp, a.cr, a.gb,
                                    a.rc, a.gbseed, a.W);
}

template <int B, bool TAB>
__global__ __launch_bounds__(kBlock) void kt_pool_prep_mq(Lvl a0, const Lvl* __restrict__ tab, int filtered) {
    FIC_LV;
    if ((int64_t)blockIdx.x * kBlock >= (int64_t)a.total * (B * B / 16)) return;
    k_pool_prep_mq_body<B>(a.img, a.pitch, a.L, a.gx, a.pool, filtered ? -1 : a.total, a.pctrl,
                           reinterpret_cast<_Float16*>(a.dh), a.sd, a.ad, a.jd);
}

template <int B, int NK, bool TAB>
__global__ __launch_bounds__(kMqWaves * 64) void kt_match_mfq(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    __shared__ MqSmem<B, NK> sm;
    k_match_mfq_body<B, NK>(sm, blockIdx.x, blockIdx.y, a.img, a.pitch, a.act, a.ctrl->act_count + a.lv,
                            reinterpret_cast<const _Float16*>(a.dh), a.sd, a.ad, a.jd, a.pctrl, a.ks, a.nc,
                            a.cg, a.part, a.sr, a.cr);
}

template <bool F16, bool TAB>
__global__ __launch_bounds__(kM8Waves * 64) void kt_match_mfma8(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    k_match_grid_body<!F16>(a.ar, a.sr, a.srp, a.cr, a.ctrl->act_count + a.lv, a.dh, a.dl, a.sd, a.ad, a.gd, a.jd,
                            a.pctrl, a.ks.k1, a.nc, a.part, a.cg, a.gb, a.rc);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_match_fp32(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    k_match_fp32_body(a.img, a.pitch, a.act, a.ctrl->act_count + a.lv, a.img, a.L, a.gx, a.jd,
                      a.pctrl, a.ks.k1, a.nc, a.part, a.cg);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_reduce_level(Lvl a0, const Lvl* __restrict__ tab,
                                                          fic_match* __restrict__ out) {
    FIC_LV;
    k_reduce_level_body(a.B, a.L, a.gx, a.act, a.ctrl->act_count + a.lv, a.part, a.nc, a.cg,
                        a.pctrl, a.cr, a.sr, a.ks, out);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_reduce_fp32(Lvl a0, const Lvl* __restrict__ tab,
                                                         fic_match* __restrict__ out) {
    FIC_LV;
    k_reduce_fp32_body(a.img, a.pitch, a.L, a.gx, a.act, a.ctrl->act_count + a.lv, a.part, a.nc,
                       a.cg, a.pctrl, out);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_reduce_quad(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    const int nblk = (a.max_act + kRqRanges - 1) / kRqRanges;
    if ((int)blockIdx.x >= nblk) return;
    k_reduce_quad_body(a.B, a.L, a.gx, a.lv, a.last, a.thr, a.act, a.ctrl, a.pctrl, a.part, a.nc,
                       a.cg, a.cr, a.sr, a.ks, a.tmpc, a.dec, a.blk, a.flags);
}

template <bool TAB>
__global__ __launch_bounds__(kBlock) void kt_quad_scatter(Lvl a0, const Lvl* __restrict__ tab) {
    FIC_LV;
    const int nblk = (a.max_act + kBlock * kQuadItems - 1) / (kBlock * kQuadItems);
    if ((int)blockIdx.x >= nblk) return;
    CompactArgs c{};
    c.kind = 1;
    c.act_count = a.ctrl->act_count + a.lv;
    c.decision = a.dec;
    k_quad_scatter_body(c, a.ctrl, a.pctrl, a.lv, nblk, a.blk, a.tmpc, a.codes, a.capacity, a.act,
                        a.act_next, a.B / 2, a.stats, a.n_out);
}

#undef FIC_LV

}  // namespace fic
