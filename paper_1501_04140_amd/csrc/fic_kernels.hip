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

// ---------------------------------------------------------------- control block
__global__ void k_level_init(Ctrl* ctrl, int lv, int act_count_init, int pool_identity_count,
                             int min_pool_rank) {
    int tid = threadIdx.x;
    for (int i = tid; i < kSelBins; i += blockDim.x) ctrl->ghist[i] = 0u;
    if (tid == 0) {
        if (act_count_init >= 0) ctrl->act_count[lv] = act_count_init;
        ctrl->pass_count = pool_identity_count >= 0 ? pool_identity_count : 0;
        ctrl->pool_count = pool_identity_count >= 0 ? pool_identity_count : 0;
        ctrl->sel_prefix = 0ull;
        ctrl->sel_rank = min_pool_rank;
        ctrl->ticket = 0u;
    }
}

__global__ void k_ctrl_reset(Ctrl* ctrl) {
    if (threadIdx.x == 0) {
        for (int i = 0; i < 5; ++i) ctrl->act_count[i] = 0;
        ctrl->n_codes = 0;
        ctrl->code_base = 0;
        ctrl->err = 0;
    }
}

// ---------------------------------------------------------------- active range lists
// Packed corner: (y << 16) | x.
__global__ void k_act_full(int32_t* act, int gy, int gx, int B) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= gy * gx) return;
    int ry = q / gx, rx = q - ry * gx;
    act[q] = ((ry * B) << 16) | (rx * B);
}

// Caller-supplied corners; an invalid corner is stored as -1.
__global__ void k_act_from_yx(int32_t* act, const int32_t* yx, int n, int H, int W, int B) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int y = yx[2 * q], x = yx[2 * q + 1];
    bool ok = y >= 0 && x >= 0 && y + B <= H && x + B <= W && (y % B) == 0 && (x % B) == 0;
    act[q] = ok ? ((y << 16) | x) : -1;
}

// ---------------------------------------------------------------- entropy score (Section 3)
// key[j] = sum_b T[c_b] over the 8-bin (p >> 5) histogram of the 2B x 2B
// domain j, where T[c] = round(c log2 c * 2^32). Entropy in bits is
// log2 Nw - key / (Nw 2^32), so the domain passes iff key < M.
__global__ void k_pool_score(const uint8_t* __restrict__ img, int pitch, int side, int L, int gx,
                             int total, const int64_t* __restrict__ T, int64_t M,
                             int64_t* __restrict__ key, Ctrl* ctrl) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int pass = 0;
    if (j < total) {
        int y = (j / gx) * L, x = (j % gx) * L;
        int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i < side; ++i) {
            const uint8_t* row = img + (int64_t)(y + i) * pitch + x;
            for (int u = 0; u < side; ++u) {
                int b = row[u] >> 5;
#pragma unroll
                for (int q = 0; q < 8; ++q) c[q] += (b == q);
            }
        }
        int64_t s = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s += T[c[q]];
        key[j] = s;
        pass = s < M;
    }
    int cnt = __syncthreads_count(pass);
    if (threadIdx.x == 0 && cnt) atomicAdd(&ctrl->pass_count, cnt);
}

// Pool mode for a level: 0 = threshold passers, 1 = floor (lowest keys), 2 = all.
__device__ inline int pool_mode(const Ctrl* ctrl, int total, int min_pool) {
    if (total <= min_pool) return 2;
    return ctrl->pass_count >= min_pool ? 0 : 1;
}

// One 12-bit digit of a radix select for the min_pool-th smallest key
// (keys < 2^48). The last workgroup to finish picks the digit.
__global__ void k_select_pass(const int64_t* __restrict__ key, int total, int min_pool, int shift,
                              Ctrl* ctrl) {
    if (pool_mode(ctrl, total, min_pool) != 1) return;
    __shared__ uint32_t h[kSelBins];
    __shared__ int s_last;
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const uint64_t prefix = ctrl->sel_prefix;
    const int hs = shift + kSelBits;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        uint64_t u = (uint64_t)key[i];
        if ((u >> hs) == (prefix >> hs)) atomicAdd(&h[(u >> shift) & (kSelBins - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x)
        if (h[i]) atomicAdd(&ctrl->ghist[i], h[i]);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&ctrl->ticket, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // last workgroup: find the digit holding rank sel_rank (1-based)
    __shared__ uint32_t part[256];
    const int per = kSelBins / 256;
    uint32_t sum = 0;
    if (threadIdx.x < 256)
        for (int b = 0; b < per; ++b) sum += atomicAdd(&ctrl->ghist[threadIdx.x * per + b], 0u);
    if (threadIdx.x < 256) part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t rank = (uint32_t)ctrl->sel_rank, cum = 0;
        int t = 0;
        while (t < 255 && cum + part[t] < rank) cum += part[t++];
        int b = t * per;
        for (;; ++b) {
            uint32_t hb = atomicAdd(&ctrl->ghist[b], 0u);
            if (cum + hb >= rank || b == t * per + per - 1) break;
            cum += hb;
        }
        ctrl->sel_prefix = prefix | ((uint64_t)b << shift);
        ctrl->sel_rank = (int)(rank - cum);
        ctrl->ticket = 0u;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) ctrl->ghist[i] = 0u;
}

// ---------------------------------------------------------------- order-preserving compaction
// Two flags per item (f0, f1). Used for the pool (f0 = below the cut, f1 = tied
// at the cut) and for the quadtree (f0 = kept, f1 = split).
struct CompactArgs {
    int kind;  // 0 pool, 1 quadtree
    int total;
    int min_pool;
    int64_t M;
    const int64_t* key;
    const int32_t* act_count;  // quadtree: number of items
    const uint8_t* decision;   // quadtree: 1 kept, 0 split, 2 invalid
};

__device__ inline void item_flags(const CompactArgs& a, const Ctrl* ctrl, int mode, int i, int& f0,
                                  int& f1) {
    f0 = 0;
    f1 = 0;
    if (a.kind == 0) {
        if (i >= a.total) return;
        int64_t k = a.key[i];
        if (mode == 2) f0 = 1;
        else if (mode == 0) f0 = k < a.M;
        else {
            int64_t cut = (int64_t)ctrl->sel_prefix;
            f0 = k < cut;
            f1 = k == cut;
        }
    } else {
        if (i >= *a.act_count) return;
        uint8_t d = a.decision[i];
        f0 = d == 1;
        f1 = d == 0;
    }
}

__device__ inline int compact_mode(const CompactArgs& a, const Ctrl* ctrl) {
    return a.kind == 0 ? pool_mode(ctrl, a.total, a.min_pool) : 0;
}

// Inclusive scan over a 256-thread block of two counters; returns exclusive values.
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

__global__ __launch_bounds__(kBlock) void k_compact_count(CompactArgs a, const Ctrl* ctrl,
                                                          int2* blk) {
    int mode = compact_mode(a, ctrl);
    int base = blockIdx.x * kBlock * kItems + threadIdx.x * kItems;
    int c0 = 0, c1 = 0;
    for (int u = 0; u < kItems; ++u) {
        int f0, f1;
        item_flags(a, ctrl, mode, base + u, f0, f1);
        c0 += f0;
        c1 += f1;
    }
    int e0, e1, t0, t1;
    block_scan2(c0, c1, e0, e1, t0, t1);
    if (threadIdx.x == 0) blk[blockIdx.x] = make_int2(t0, t1);
}

// Single workgroup: exclusive scan of the per-block counts, then the totals.
__global__ __launch_bounds__(kBlock) void k_compact_scan(CompactArgs a, Ctrl* ctrl, int2* blk,
                                                         int nblk, int lv, fic_level_stats* stats,
                                                         int codes_capacity) {
    __shared__ int carry0, carry1;
    if (threadIdx.x == 0) {
        carry0 = 0;
        carry1 = 0;
    }
    __syncthreads();
    for (int base = 0; base < nblk; base += kBlock) {
        int i = base + threadIdx.x;
        int2 v = i < nblk ? blk[i] : make_int2(0, 0);
        int e0, e1, t0, t1;
        block_scan2(v.x, v.y, e0, e1, t0, t1);
        if (i < nblk) blk[i] = make_int2(carry0 + e0, carry1 + e1);
        __syncthreads();
        if (threadIdx.x == 0) {
            carry0 += t0;
            carry1 += t1;
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (a.kind == 0) {
        int mode = pool_mode(ctrl, a.total, a.min_pool);
        ctrl->pool_count = mode == 1 ? carry0 + min(carry1, ctrl->sel_rank) : carry0;
    } else {
        int act = *a.act_count;
        int pool = ctrl->pool_count;
        ctrl->code_base = ctrl->n_codes;
        ctrl->n_codes += carry0;
        ctrl->act_count[lv + 1] = 4 * carry1;
        if (stats) {
            fic_level_stats s;
            s.matches = (int64_t)act * pool * 8;
            s.pool = pool;
            s.passed = ctrl->pass_count;
            s.active = act;
            s.accepted = carry0;
            stats[lv] = s;
        }
    }
    (void)codes_capacity;
}

__global__ __launch_bounds__(kBlock) void k_compact_scatter(
    CompactArgs a, const Ctrl* ctrl, const int2* blk, int32_t* pool_out,
    // quadtree outputs
    const fic_code* tmp_codes, fic_code* codes, int capacity, const int32_t* act,
    int32_t* act_next, int half) {
    int mode = compact_mode(a, ctrl);
    int base = blockIdx.x * kBlock * kItems + threadIdx.x * kItems;
    int f0[kItems], f1[kItems];
    int c0 = 0, c1 = 0;
    for (int u = 0; u < kItems; ++u) {
        item_flags(a, ctrl, mode, base + u, f0[u], f1[u]);
        c0 += f0[u];
        c1 += f1[u];
    }
    int e0, e1, t0, t1;
    block_scan2(c0, c1, e0, e1, t0, t1);
    int2 off = blk[blockIdx.x];
    int r0 = off.x + e0, r1 = off.y + e1;
    if (a.kind == 0) {
        int take = mode == 1 ? ctrl->sel_rank : 0;
        for (int u = 0; u < kItems; ++u) {
            int keep = f0[u] || (f1[u] && r1 < take);
            if (keep) pool_out[r0 + min(r1, take)] = base + u;
            r0 += f0[u];
            r1 += f1[u];
        }
    } else {
        int cb = ctrl->code_base;
        for (int u = 0; u < kItems; ++u) {
            int i = base + u;
            if (f0[u]) {
                int pos = cb + r0;
                if (pos < capacity) codes[pos] = tmp_codes[i];
            }
            if (f1[u]) {
                int yx = act[i];
                int y = yx >> 16, x = yx & 0xffff;
                int32_t* dst = act_next + 4 * r1;
                dst[0] = (y << 16) | x;
                dst[1] = (y << 16) | (x + half);
                dst[2] = ((y + half) << 16) | x;
                dst[3] = ((y + half) << 16) | (x + half);
            }
            r0 += f0[u];
            r1 += f1[u];
        }
    }
}

// ---------------------------------------------------------------- pool and range preparation
// Per pool entry p: the decimated domain d' (2x2 sums) as packed high and low
// bytes, S = sum d', A' = n sum d'^2 - S^2 and the grid index j.
template <int B>
__global__ __launch_bounds__(kBlock) void k_pool_prep(const uint8_t* __restrict__ img, int pitch,
                                                      int L, int gx, const int32_t* __restrict__ pool,
                                                      const Ctrl* ctrl, uint32_t* __restrict__ HL,
                                                      uint32_t* __restrict__ Sd,
                                                      int64_t* __restrict__ Ad,
                                                      int32_t* __restrict__ Jd) {
    constexpr int n = B * B, NW = n / 4;
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ctrl->pool_count) return;
    int j = pool ? pool[p] : p;
    int y = (j / gx) * L, x = (j % gx) * L;
    uint32_t s = 0;
    uint64_t q = 0;
    uint32_t* hl = HL + (int64_t)p * 2 * NW;
    for (int w = 0; w < NW; ++w) {
        uint32_t hw = 0, lw = 0;
        for (int b = 0; b < 4; ++b) {
            int m = 4 * w + b, i = m / B, c = m % B;
            const uint8_t* px = img + (int64_t)(y + 2 * i) * pitch + x + 2 * c;
            uint32_t d = (uint32_t)px[0] + px[1] + px[pitch] + px[pitch + 1];
            s += d;
            q += (uint64_t)d * d;
            hw |= (d >> 8) << (8 * b);
            lw |= (d & 255u) << (8 * b);
        }
        hl[w] = hw;
        hl[NW + w] = lw;
    }
    Sd[p] = s;
    Ad[p] = (int64_t)n * (int64_t)q - (int64_t)s * (int64_t)s;
    Jd[p] = j;
}

// Row q*8+t holds the range block R of active range q rearranged so that
// <row, d'> = <R, T_t(d')>: row[m] = R[iso_src(inverse(t), m)].
template <int B>
__global__ __launch_bounds__(kBlock) void k_range_prep(const uint8_t* __restrict__ img, int pitch,
                                                       const int32_t* __restrict__ act,
                                                       const int32_t* act_count,
                                                       uint32_t* __restrict__ Arow,
                                                       int32_t* __restrict__ SR,
                                                       int64_t* __restrict__ CR) {
    constexpr int n = B * B, NW = n / 4;
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= 8 * *act_count) return;
    int q = row >> 3, t = row & 7;
    int yx = act[q];
    uint32_t* dst = Arow + (int64_t)row * NW;
    if (yx < 0) {
        for (int w = 0; w < NW; ++w) dst[w] = 0u;
        if (t == 0) {
            SR[q] = 0;
            CR[q] = 0;
        }
        return;
    }
    int y = yx >> 16, x = yx & 0xffff;
    int u = iso_inverse(t);
    for (int w = 0; w < NW; ++w) {
        uint32_t v = 0;
        for (int b = 0; b < 4; ++b) {
            int src = iso_src(B, u, (4 * w + b) / B, (4 * w + b) % B);
            v |= (uint32_t)img[(int64_t)(y + src / B) * pitch + x + src % B] << (8 * b);
        }
        dst[w] = v;
    }
    if (t == 0) {
        int s = 0;
        int64_t s2 = 0;
        for (int i = 0; i < B; ++i)
            for (int c = 0; c < B; ++c) {
                int v = img[(int64_t)(y + i) * pitch + x + c];
                s += v;
                s2 += v * v;
            }
        SR[q] = s;
        CR[q] = (int64_t)n * s2 - (int64_t)s * s;
    }
}

// ---------------------------------------------------------------- the matcher
// Best contrast for one (row, domain) element. F = k^2 A' - 8Q k B' is
// 16 Q^2 n E(k) minus the row constant 16 Q^2 C. For a consecutive set
// k0..k1 the minimiser is the smallest k with (2k+1) A' >= 8Q B' (F is a
// convex quadratic in k); an FP32 estimate is corrected exactly.
__device__ inline void best_contrast(int64_t Bp, int64_t Ap, const KSet& ks, int64_t& F, int& s) {
    if (ks.consecutive) {
        int k = ks.k0;
        if (Ap > 0) {
            float xf = (float)Bp * (40.0f / (float)Ap);
            float kf = fminf(fmaxf(rintf(xf), (float)ks.k0), (float)ks.k1);
            k = (int)kf;
            const int64_t b80 = 80 * Bp;
            while (k > ks.k0 && (int64_t)(2 * k - 1) * Ap >= b80) --k;
            while (k < ks.k1 && (int64_t)(2 * k + 1) * Ap < b80) ++k;
        }
        F = (int64_t)(k * k) * Ap - (int64_t)(80 * k) * Bp;
        s = k - ks.k0;
    } else {
        F = INT64_MAX;
        s = 0;
        for (int i = 0; i < ks.n; ++i) {
            const int k = ks.k[i];
            int64_t f = (int64_t)(k * k) * Ap - (int64_t)(80 * k) * Bp;
            if (f < F) {
                F = f;
                s = i;
            }
        }
    }
}

__device__ inline bool pair_less(int64_t fa, int64_t ka, int64_t fb, int64_t kb) {
    return fa < fb || (fa == fb && ka < kb);
}

template <int B>
struct MatchTile {
    static constexpr int n = B * B;
    static constexpr int NW = n / 4;
    // domains per LDS tile: about 24-36 KiB of LDS
    static constexpr int TN = B == 16 ? 64 : (B == 8 ? 128 : 256);
};

// grid: x = row blocks of 256 rows (32 ranges x 8 isometries), y = pool chunks.
template <int B>
__global__ __launch_bounds__(kBlock) void k_match(const uint32_t* __restrict__ Arow,
                                                  const int32_t* __restrict__ SR,
                                                  const int32_t* act_count,
                                                  const uint32_t* __restrict__ HL,
                                                  const uint32_t* __restrict__ Sd,
                                                  const int64_t* __restrict__ Ad,
                                                  const int32_t* __restrict__ Jd, const Ctrl* ctrl,
                                                  KSet ks, int n_chunks, Partial* __restrict__ part) {
    using T = MatchTile<B>;
    constexpr int n = T::n, NW = T::NW, TN = T::TN;
    __shared__ uint32_t sHL[TN * 2 * NW];
    __shared__ uint32_t sS[TN];
    __shared__ int64_t sA[TN];
    __shared__ int32_t sJ[TN];

    const int nrows = 8 * *act_count;
    const int row0 = blockIdx.x * kBlock;
    if (row0 >= nrows) return;
    const int row = row0 + threadIdx.x;
    const bool valid = row < nrows;
    const int t = row & 7;

    uint32_t r[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) r[w] = valid ? Arow[(int64_t)row * NW + w] : 0u;
    const int64_t sr = valid ? SR[row >> 3] : 0;

    const int P = ctrl->pool_count;
    const int c = blockIdx.y;
    const int lo = (int)((int64_t)P * c / n_chunks);
    const int hi = (int)((int64_t)P * (c + 1) / n_chunks);

    int64_t bestF = INT64_MAX, bestK = INT64_MAX;
    for (int base = lo; base < hi; base += TN) {
        const int cnt = min(TN, hi - base);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * 2 * NW; i += kBlock) sHL[i] = HL[(int64_t)base * 2 * NW + i];
        for (int i = threadIdx.x; i < cnt; i += kBlock) {
            sS[i] = Sd[base + i];
            sA[i] = Ad[base + i];
            sJ[i] = Jd[base + i];
        }
        __syncthreads();
        for (int d = 0; d < cnt; ++d) {
            const uint32_t* hl = sHL + d * 2 * NW;
            uint32_t ph = 0, pl = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                ph = __builtin_amdgcn_udot4(r[w], hl[w], ph, false);
                pl = __builtin_amdgcn_udot4(r[w], hl[NW + w], pl, false);
            }
            const int64_t Pv = ((int64_t)ph << 8) + pl;
            const int64_t Bp = Pv * n - sr * (int64_t)sS[d];
            int64_t F;
            int s;
            best_contrast(Bp, sA[d], ks, F, s);
            if (F < bestF) {
                bestF = F;
                bestK = ((int64_t)sJ[d] << 8) | (t << 4) | s;
            }
        }
    }
    // reduce the 8 isometry rows of each range (8 consecutive lanes)
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
        int64_t of = __shfl_xor(bestF, m, 64);
        int64_t ok = __shfl_xor(bestK, m, 64);
        if (pair_less(of, ok, bestF, bestK)) {
            bestF = of;
            bestK = ok;
        }
    }
    if (valid && t == 0) {
        Partial pr;
        pr.F = bestF;
        pr.key = bestK;
        part[(int64_t)(row >> 3) * n_chunks + c] = pr;
    }
}

// ---------------------------------------------------------------- per-range result
__device__ inline bool finish_range(const uint8_t* img, int pitch, int yx, int B, int L, int gx,
                                    const Partial* pr, int n_chunks, int64_t CRq, int32_t SRq,
                                    const KSet& ks, fic_match& m, int& dy, int& dx) {
    int64_t F = INT64_MAX, K = INT64_MAX;
    for (int c = 0; c < n_chunks; ++c)
        if (pair_less(pr[c].F, pr[c].key, F, K)) {
            F = pr[c].F;
            K = pr[c].key;
        }
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
    const int j = (int)(K >> 8), t = (int)((K >> 4) & 15), s = (int)(K & 15);
    const int k = ks.consecutive ? ks.k0 + s : ks.k[s];
    dy = (j / gx) * L;
    dx = (j % gx) * L;
    int64_t sd = 0;
    for (int i = 0; i < 2 * B; ++i) {
        const uint8_t* row = img + (int64_t)(dy + i) * pitch + dx;
        for (int u = 0; u < 2 * B; ++u) sd += row[u];
    }
    m.e_num = F + 1600 * CRq;
    m.dom = j;
    m.iso = (uint8_t)t;
    m.s_idx = (uint8_t)s;
    m.k = (uint8_t)k;
    // o = (4Q sumR - k sumD') / (4Q n), rounded half up
    m.q_o = (int16_t)floordiv64(2 * (40 * (int64_t)SRq - k * sd) + 40 * n, 80 * (int64_t)n);
    m.E = (float)m.e_num / (1600.0f * (float)n);
    return true;
}

__global__ __launch_bounds__(kBlock) void k_reduce_level(const uint8_t* __restrict__ img, int pitch,
                                                         int B, int L, int gx,
                                                         const int32_t* __restrict__ act,
                                                         const int32_t* act_count,
                                                         const Partial* __restrict__ part,
                                                         int n_chunks, const int64_t* __restrict__ CR,
                                                         const int32_t* __restrict__ SR, KSet ks,
                                                         fic_match* __restrict__ out) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= *act_count) return;
    fic_match m;
    int dy, dx;
    finish_range(img, pitch, act[q], B, L, gx, part + (int64_t)q * n_chunks, n_chunks, CR[q], SR[q],
                 ks, m, dy, dx);
    out[q] = m;
}

// Quadtree step: the leaf record and the keep/split decision of each active range.
__global__ __launch_bounds__(kBlock) void k_reduce_quad(
    const uint8_t* __restrict__ img, int pitch, int B, int L, int gx, int lv, int last,
    int64_t thr, const int32_t* __restrict__ act, const int32_t* act_count,
    const Partial* __restrict__ part, int n_chunks, const int64_t* __restrict__ CR,
    const int32_t* __restrict__ SR, KSet ks, fic_code* __restrict__ tmp, uint8_t* __restrict__ dec) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= *act_count) return;
    fic_match m;
    int dy, dx;
    const int yx = act[q];
    bool ok = finish_range(img, pitch, yx, B, L, gx, part + (int64_t)q * n_chunks, n_chunks, CR[q],
                           SR[q], ks, m, dy, dx);
    if (!ok) {
        dec[q] = 2;
        return;
    }
    fic_code c;
    c.e_num = m.e_num;
    c.dom = m.dom;
    c.y = (int16_t)(yx >> 16);
    c.x = (int16_t)(yx & 0xffff);
    c.dy = (int16_t)dy;
    c.dx = (int16_t)dx;
    c.q_o = m.q_o;
    c.log2B = (uint8_t)(31 - __clz(B));
    c.iso = m.iso;
    c.k = m.k;
    c.s_idx = m.s_idx;
    c.level = (uint8_t)lv;
    for (int i = 0; i < 5; ++i) c.pad_[i] = 0;
    tmp[q] = c;
    dec[q] = (last || m.e_num <= thr) ? 1 : 0;
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

// ---------------------------------------------------------------- launch helpers
int match_tile_domains(int B) {
    switch (B) {
        case 2: return MatchTile<2>::TN;
        case 4: return MatchTile<4>::TN;
        case 8: return MatchTile<8>::TN;
        default: return MatchTile<16>::TN;
    }
}

}  // namespace fic
