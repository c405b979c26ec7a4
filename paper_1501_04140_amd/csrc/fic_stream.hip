// Bitstream of a quadtree encode: device packer and host reader (included by
// fic_lib.hip). The paper reports compression ratios (Section 4) without a bit
// allocation; the fixed-length layout is documented in include/fic.h.

namespace fic {
namespace {

constexpr uint32_t kStreamMagic = 0xF1C5;
constexpr uint32_t kStreamVersion = 1;

__host__ __device__ inline int bits_for(int64_t x) {  // ceil(log2 x) for x >= 2, else 0
    int b = 0;
    while (b < 62 && (1ll << b) < x) ++b;
    return b;
}

struct StreamLevel {
    int32_t listed, P, g, pbits, sbits, len;
    int32_t nflags, nleaves, first_leaf;
    int64_t pool_off, pool_bit, leaf_bit;
};

struct StreamPlan {
    StreamLevel lv[4];
    int64_t flag_bit, nflag_total, total_bits;
};

// OR `width` (<= 32) bits of v into the stream at bit pos (below cap bits).
__device__ inline void put_bits(uint32_t* w, int64_t pos, uint32_t v, int width, int64_t cap) {
    if (width <= 0 || pos + width > cap) return;
    if (width < 32) v &= (1u << width) - 1u;
    const int64_t word = pos >> 5;
    const int off = (int)(pos & 31);
    atomicOr(&w[word], v << off);
    if (off + width > 32) atomicOr(&w[word + 1], v >> (32 - off));
}

__device__ inline int level_grid(const fic_params& p, int H, int W, int l) {
    const int B = p.B0 >> l;
    return ((H - 2 * B) / p.L[l] + 1) * ((W - 2 * B) / p.L[l] + 1);
}

// Section offsets from the encode's per-level counts (one thread).
__global__ void k_stream_plan(fic_params p, int H, int W, const fic_level_stats* __restrict__ stats,
                              StreamPlan* __restrict__ plan, int64_t* __restrict__ n_bytes) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    StreamPlan q;
    int64_t pos = 64;
    int64_t poff = 0;
    for (int l = 0; l < p.n_levels; ++l) {
        StreamLevel& v = q.lv[l];
        const int grid = level_grid(p, H, W, l);
        pos += 16 + 4 + 4 * p.n_s[l] + 1;
        v.pool_off = poff;
        v.g = bits_for(grid);
        {
            // list the pool only where it shortens the level
            const int64_t P = stats[l].pool, nl = stats[l].accepted;
            v.listed = p.entropy_mode != 0 && stats[l].active > 0 && nl > 0 &&
                       24 + P * v.g + nl * bits_for(P) < nl * v.g;
        }
        v.P = v.listed ? stats[l].pool : grid;
        v.pool_bit = 0;
        if (v.listed) {
            pos += 24;
            v.pool_bit = pos;
            pos += (int64_t)v.P * v.g;
        }
        poff += grid;
    }
    q.flag_bit = pos;
    q.nflag_total = 0;
    for (int l = 0; l < p.n_levels; ++l) {
        q.lv[l].nflags = l + 1 < p.n_levels ? stats[l].active : 0;
        q.nflag_total += q.lv[l].nflags;
    }
    pos += q.nflag_total;
    int first = 0;
    for (int l = 0; l < p.n_levels; ++l) {
        StreamLevel& v = q.lv[l];
        v.pbits = bits_for(v.P);
        v.sbits = bits_for(p.n_s[l]);
        v.len = v.pbits + 3 + v.sbits + 9;
        v.nleaves = stats[l].accepted;
        v.first_leaf = first;
        v.leaf_bit = pos;
        pos += (int64_t)v.nleaves * v.len;
        first += v.nleaves;
    }
    q.total_bits = pos;
    *plan = q;
    *n_bytes = (pos + 7) / 8;
}

// Header fields (one thread).
__global__ void k_stream_header(fic_params p, int H, int W, const StreamPlan* __restrict__ plan,
                                uint32_t* __restrict__ out, int64_t cap) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t pos = 0;
    auto put = [&](uint32_t v, int width) {
        put_bits(out, pos, v, width, cap);
        pos += width;
    };
    put(kStreamMagic, 16);
    put(kStreamVersion, 8);
    put((uint32_t)H, 16);
    put((uint32_t)W, 16);
    put((uint32_t)p.B0, 5);
    put((uint32_t)p.n_levels, 3);
    for (int l = 0; l < p.n_levels; ++l) {
        const StreamLevel& v = plan->lv[l];
        put((uint32_t)p.L[l], 16);
        put((uint32_t)p.n_s[l], 4);
        for (int i = 0; i < p.n_s[l]; ++i) put((uint32_t)p.s_k[l][i], 4);
        put((uint32_t)v.listed, 1);
        if (v.listed) {
            put((uint32_t)v.P, 24);
            pos += (int64_t)v.P * v.g;  // the pool list, written by k_stream_pools
        }
    }
}

// Pool lists: thread t is entry t of the concatenated per-level pools.
__global__ void k_stream_pools(fic_params p, const StreamPlan* __restrict__ plan,
                               const int32_t* __restrict__ pools, int64_t n_all,
                               uint32_t* __restrict__ out, int64_t cap) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_all) return;
    int l = 0;
    while (l + 1 < p.n_levels && t >= plan->lv[l + 1].pool_off) ++l;
    const StreamLevel& v = plan->lv[l];
    const int64_t i = t - v.pool_off;
    if (!v.listed || i >= v.P) return;
    put_bits(out, v.pool_bit + i * v.g, (uint32_t)pools[t], v.g, cap);
}

// Split flags: bit t of the encoder's bitmap goes to the flag section at t.
__global__ void k_stream_flags(const StreamPlan* __restrict__ plan, const uint32_t* __restrict__ flags,
                               uint32_t* __restrict__ out, int64_t cap) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= plan->nflag_total) return;
    if ((flags[t >> 5] >> (t & 31)) & 1u) put_bits(out, plan->flag_bit + t, 1u, 1, cap);
}

// Leaves: code i (codes are level by level) at its level's section.
__global__ void k_stream_leaves(const fic_code* __restrict__ codes, int n_codes,
                                const StreamPlan* __restrict__ plan, const int32_t* __restrict__ pools,
                                uint32_t* __restrict__ out, int64_t cap, int n_levels) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_codes) return;
    const fic_code c = codes[i];
    const int l = c.level;
    if (l >= n_levels) return;
    const StreamLevel& v = plan->lv[l];
    const int j = i - v.first_leaf;
    if (j < 0 || j >= v.nleaves) return;
    int64_t pos = v.leaf_bit + (int64_t)j * v.len;
    uint32_t dpos = (uint32_t)c.dom;
    if (v.listed) {  // position of the domain in the ascending pool
        const int32_t* pl = pools + v.pool_off;
        int lo = 0, hi = v.P;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (pl[mid] < c.dom) lo = mid + 1;
            else hi = mid;
        }
        dpos = (uint32_t)lo;
    }
    put_bits(out, pos, dpos, v.pbits, cap);
    pos += v.pbits;
    put_bits(out, pos, c.iso, 3, cap);
    pos += 3;
    put_bits(out, pos, c.s_idx, v.sbits, cap);
    pos += v.sbits;
    put_bits(out, pos, (uint32_t)c.q_o & 0x1ffu, 9, cap);
}

int64_t stream_bound_bits(int H, int W, const fic_params* p) {
    int64_t bits = 64;
    for (int l = 0; l < p->n_levels; ++l) {
        const int B = p->B0 >> l;
        const int64_t grid = (int64_t)((H - 2 * B) / p->L[l] + 1) * ((W - 2 * B) / p->L[l] + 1);
        const int64_t ranges = (int64_t)(H / B) * (W / B);
        bits += 16 + 4 + 4 * p->n_s[l] + 1 + 24 + grid * bits_for(grid);
        bits += l + 1 < p->n_levels ? ranges : 0;
        bits += ranges * (bits_for(grid) + 3 + bits_for(p->n_s[l]) + 9);
    }
    return bits;
}

// Host reader (bounds-checked).
struct BitReader {
    const uint8_t* d;
    int64_t nbits, pos = 0;
    bool bad = false;
    uint32_t get(int width) {
        if (width <= 0) return 0;
        if (pos + width > nbits) {
            bad = true;
            return 0;
        }
        uint32_t v = 0;
        for (int i = 0; i < width; ++i, ++pos) v |= (uint32_t)((d[pos >> 3] >> (pos & 7)) & 1) << i;
        return v;
    }
};

}  // namespace
}  // namespace fic

FIC_API int64_t fic_stream_bound(int32_t H, int32_t W, const fic_params* p) {
    std::vector<KSet> ks;
    if (check_params(p, ks) || H < 2 * p->B0 || W < 2 * p->B0) return -1;
    return (stream_bound_bits(H, W, p) + 31) / 32 * 4;
}

FIC_API int fic_pack_stream(const fic_code* codes, int32_t n_codes, int32_t H, int32_t W,
                            const fic_params* p, const fic_level_stats* stats, const uint32_t* flags,
                            const int32_t* pools, uint8_t* out, int64_t capacity, int64_t* n_bytes,
                            void* stream) {
    std::vector<KSet> ks;
    int rc = check_params(p, ks);
    if (rc) return rc;
    if (H < 2 * p->B0 || W < 2 * p->B0 || H % p->B0 || W % p->B0 || H > FIC_MAX_SIDE || W > FIC_MAX_SIDE)
        return fail(FIC_EINVAL, "image %dx%d does not fit the parameters", H, W);
    if (n_codes < 0 || (n_codes > 0 && !codes)) return fail(FIC_EINVAL, "bad codes");
    if (!stats || !out || !n_bytes) return fail(FIC_EINVAL, "stats, out or n_bytes is NULL");
    if (p->n_levels > 1 && !flags) return fail(FIC_EINVAL, "flags is NULL (needed for n_levels > 1)");
    if (p->entropy_mode != 0 && !pools) return fail(FIC_EINVAL, "pools is NULL (needed with a pool filter)");
    if (capacity < 4 || capacity % 4 || ((uintptr_t)out & 3))
        return fail(FIC_EINVAL, "out must be 4-byte aligned with a capacity that is a multiple of 4");
    Workspace* ws;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = get_ws(st, &ws))) return rc;
    if ((rc = ensure(*ws, ws->plan, sizeof(StreamPlan)))) return rc;
    StreamPlan* plan = P<StreamPlan>(ws->plan);
    uint32_t* w = reinterpret_cast<uint32_t*>(out);
    const int64_t cap = capacity * 8;
    const int64_t nw = capacity / 4;
    k_fill_i32<<<cdiv(nw, kBlock), kBlock, 0, st>>>(reinterpret_cast<int32_t*>(w), (int)nw, 0);
    k_stream_plan<<<1, 1, 0, st>>>(*p, H, W, stats, plan, n_bytes);
    k_stream_header<<<1, 1, 0, st>>>(*p, H, W, plan, w, cap);
    if (p->entropy_mode != 0) {
        int64_t n_all = 0;
        for (int l = 0; l < p->n_levels; ++l) {
            const int B = p->B0 >> l;
            n_all += (int64_t)((H - 2 * B) / p->L[l] + 1) * ((W - 2 * B) / p->L[l] + 1);
        }
        k_stream_pools<<<cdiv(n_all, kBlock), kBlock, 0, st>>>(*p, plan, pools, n_all, w, cap);
    }
    if (p->n_levels > 1) {
        int64_t nf = 0;
        for (int l = 0; l + 1 < p->n_levels; ++l) {
            const int B = p->B0 >> l;
            nf += (int64_t)(H / B) * (W / B);
        }
        k_stream_flags<<<cdiv(nf, kBlock), kBlock, 0, st>>>(plan, flags, w, cap);
    }
    if (n_codes > 0)
        k_stream_leaves<<<cdiv(n_codes, kBlock), kBlock, 0, st>>>(codes, n_codes, plan, pools, w, cap,
                                                                p->n_levels);
    LAUNCH_CHECK();
    return FIC_OK;
}

FIC_API int fic_unpack_stream(const uint8_t* data, int64_t n_bytes, fic_code* codes, int32_t capacity,
                              int32_t* n_codes, int32_t* H_out, int32_t* W_out) {
    if (!data || n_bytes < 8 || !n_codes) return fail(FIC_EINVAL, "no stream");
    BitReader r{data, n_bytes * 8};
    if (r.get(16) != kStreamMagic || r.get(8) != kStreamVersion) return fail(FIC_EINVAL, "not a stream of this format");
    const int H = (int)r.get(16), W = (int)r.get(16);
    const int B0 = (int)r.get(5), nl = (int)r.get(3);
    if (nl < 1 || nl > 4 || !valid_B(B0) || (B0 >> (nl - 1)) < 2 || H < 2 * B0 || W < 2 * B0 || H % B0 || W % B0)
        return fail(FIC_EINVAL, "bad stream header");
    int L[4], ns[4], kk[4][16];
    std::vector<std::vector<int32_t>> pools(nl);
    bool listed[4];
    for (int l = 0; l < nl; ++l) {
        L[l] = (int)r.get(16);
        ns[l] = (int)r.get(4);
        for (int i = 0; i < ns[l]; ++i) kk[l][i] = (int)r.get(4);
        const int B = B0 >> l;
        if (L[l] < 1 || ns[l] < 1 || H < 2 * B || W < 2 * B) return fail(FIC_EINVAL, "bad stream level %d", l);
        const int64_t grid = (int64_t)((H - 2 * B) / L[l] + 1) * ((W - 2 * B) / L[l] + 1);
        listed[l] = r.get(1) != 0;
        if (listed[l]) {
            const int64_t P = r.get(24);
            if (P < 1 || P > grid) return fail(FIC_EINVAL, "bad pool size at level %d", l);
            const int g = bits_for(grid);
            pools[l].resize(P);
            for (int64_t i = 0; i < P; ++i) pools[l][i] = (int32_t)r.get(g);
        }
        if (r.bad) return fail(FIC_EINVAL, "stream truncated");
    }
    // rebuild the active lists from the split flags
    std::vector<std::vector<std::pair<int, int>>> act(nl);
    std::vector<std::vector<uint8_t>> split(nl);
    for (int y = 0; y < H / B0; ++y)
        for (int x = 0; x < W / B0; ++x) act[0].push_back({y * B0, x * B0});
    for (int l = 0; l < nl; ++l) {
        split[l].assign(act[l].size(), 0);
        if (l + 1 == nl) break;
        const int h = (B0 >> l) / 2;
        for (size_t q = 0; q < act[l].size(); ++q) {
            split[l][q] = (uint8_t)r.get(1);
            if (split[l][q]) {
                const int y = act[l][q].first, x = act[l][q].second;
                act[l + 1].push_back({y, x});
                act[l + 1].push_back({y, x + h});
                act[l + 1].push_back({y + h, x});
                act[l + 1].push_back({y + h, x + h});
            }
        }
        if (r.bad) return fail(FIC_EINVAL, "stream truncated");
    }
    int count = 0;
    for (int l = 0; l < nl; ++l) {
        const int B = B0 >> l;
        const int gx = (W - 2 * B) / L[l] + 1;
        const int64_t grid = (int64_t)((H - 2 * B) / L[l] + 1) * gx;
        const int pb = listed[l] ? bits_for((int64_t)pools[l].size()) : bits_for(grid);
        const int sb = bits_for(ns[l]);
        for (size_t q = 0; q < act[l].size(); ++q) {
            if (split[l][q]) continue;
            const uint32_t dp = r.get(pb);
            const int iso = (int)r.get(3);
            const int si = (int)r.get(sb);
            int qo = (int)r.get(9);
            if (r.bad) return fail(FIC_EINVAL, "stream truncated");
            if (qo >= 256) qo -= 512;
            int64_t dom = dp;
            if (listed[l]) {
                if (dp >= pools[l].size()) return fail(FIC_EINVAL, "bad pool position");
                dom = pools[l][dp];
            }
            if (dom < 0 || dom >= grid || si >= ns[l]) return fail(FIC_EINVAL, "bad leaf");
            if (count < capacity && codes) {
                fic_code c;
                std::memset(&c, 0, sizeof c);
                c.e_num = -1;
                c.dom = (int32_t)dom;
                c.y = (int16_t)act[l][q].first;
                c.x = (int16_t)act[l][q].second;
                c.dy = (int16_t)((dom / gx) * L[l]);
                c.dx = (int16_t)((dom % gx) * L[l]);
                c.q_o = (int16_t)qo;
                c.log2B = (uint8_t)bits_for(B);
                c.iso = (uint8_t)iso;
                c.k = (uint8_t)kk[l][si];
                c.s_idx = (uint8_t)si;
                c.level = (uint8_t)l;
                codes[count] = c;
            }
            ++count;
        }
    }
    *n_codes = count;
    if (H_out) *H_out = H;
    if (W_out) *W_out = W;
    if (count > capacity) return fail(FIC_ECAPACITY, "stream holds %d codes, capacity %d", count, capacity);
    return FIC_OK;
}
