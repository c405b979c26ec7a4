// Device kernels of the learned domain proposal (an extension of the
// exhaustive search of Section 2): a 64-256-256-64 network embeds 8 x 8 range
// blocks and 2x2-summed domain blocks, the k most similar domains of each
// range are rescored exactly with the moment form of eq. (1), and ranges whose
// best proposal fails the RMS test fall back to the exhaustive matcher.
//
// Matrix products run on the fp16 MFMA (v_mfma_f32_16x16x32_f16, fp32
// accumulation). Operand layout of that instruction on a 64-wide wave:
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + e], e = 0..7
//   B (32 x 16): lane l holds B[8 (l / 16) + e][l % 16]
//   C (16 x 16): lane l holds C[4 (l / 16) + e][l % 16], e = 0..3
// Every product here is C = A * B^T with both operands stored K-contiguous
// ("NT"), so each lane's fragment is one 16-byte load.
#include "fic_internal.h"

namespace fic {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Parameter layout (fp32 master copy): W1 [256][64], b1, W2 [256][256], b2,
// W3 [64][256], b3 -- each W stored (out, in).
constexpr int kMlpIn = 64, kMlpHid = 256, kMlpOut = 64;
constexpr int kOffW1 = 0, kOffB1 = 16384, kOffW2 = 16640, kOffB2 = 82176, kOffW3 = 82432,
              kOffB3 = 98816, kMlpParams = 98880;
// fp16 copies: W1, W2, W3 as above, then their transposes W1t [64][256],
// W2t [256][256], W3t [256][64] (the operands of the backward products).
constexpr int kH16W1 = 0, kH16W2 = 16384, kH16W3 = 81920, kH16W1t = 98304, kH16W2t = 114688,
              kH16W3t = 180224, kH16Total = 196608;

__device__ inline f4 mfma16(h8 a, h8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ inline int wave_sum_i32(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline float wave_sum_f32(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline float wave_max_f32(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int o) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, o, 64);
    hi = __shfl_xor(hi, o, 64);
    return ((uint64_t)hi << 32) | lo;
}

// LDS writes by some lanes of a wave, then reads of them by other lanes.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- block vectors
// One wave per block; lane e holds element e (row e / 8, column e % 8). The
// block's 64 values (range pixels, or the 2x2 sums of a domain) are centred
// and scaled to unit norm -- exactly up to the final division: 64 v - sum v
// and its squared norm are integers -- and written as the 8 rows T_t x,
// t = 0..7 (row 8 q + t). A constant or out-of-image block gives zero rows.
__global__ __launch_bounds__(256) void k_block_rows(const uint8_t* __restrict__ img, int pitch,
                                                    int H, int W, int kind, int L, int gx,
                                                    int total, const int32_t* __restrict__ list,
                                                    int n, _Float16* __restrict__ X) {
    const int q = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= n) return;
    int y, x;
    bool ok;
    if (kind == 0) {
        const int rgx = W / 8;
        if (list) {
            y = list[2 * q];
            x = list[2 * q + 1];
        } else {
            y = (q / rgx) * 8;
            x = (q % rgx) * 8;
        }
        ok = y >= 0 && x >= 0 && y + 8 <= H && x + 8 <= W;
    } else {
        const int j = list ? list[q] : q;
        ok = j >= 0 && j < total;
        y = ok ? (j / gx) * L : 0;
        x = ok ? (j % gx) * L : 0;
        ok = ok && y + 16 <= H && x + 16 <= W;
    }
    const int i = lane >> 3, c = lane & 7;
    int v = 0;
    if (ok) {
        if (kind == 0) {
            v = img[(int64_t)(y + i) * pitch + x + c];
        } else {
            const uint8_t* p = img + (int64_t)(y + 2 * i) * pitch + x + 2 * c;
            v = p[0] + p[1] + p[pitch] + p[pitch + 1];
        }
    }
    const int s = wave_sum_i32(v);
    const int cen = 64 * v - s;
    const int64_t nn = wave_sum_i64((int64_t)cen * cen);
    const float xv = nn > 0 ? (float)cen / sqrtf((float)nn) : 0.0f;
    _Float16* out = X + (int64_t)q * 8 * 64 + lane;
#pragma unroll
    for (int t = 0; t < 8; ++t) out[t * 64] = (_Float16)__shfl(xv, iso_src(8, t, i, c), 64);
}

// ---------------------------------------------------------------- matrix product
enum { kEpiRelu16 = 0, kEpiF32 = 1, kEpiMask16 = 2, kEpiPart32 = 3 };

// C[m][n] = alpha * sum_k A[m][k] B[n][k] over k in this split's chunk, then
//   kEpiRelu16: C16 = max(C + bias[n], 0)          (forward hidden layers)
//   kEpiF32:    C32 = C + bias[n] (bias may be NULL)
//   kEpiMask16: C16 = C if mask[m][n] > 0 else 0   (ReLU derivative)
//   kEpiPart32: C32[split][m][n] = C               (split-K partial sums)
// Workgroup tile 64 x 64 (2 x 2 waves of 32 x 32), the column blocks of a row
// block in consecutive workgroups. Rows and columns past M, N
// read the last valid row and are not stored. The K range of every split must
// be a multiple of 32, and lda, ldb multiples of 8.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(const _Float16* __restrict__ A, int lda,
                                                 const _Float16* __restrict__ B, int ldb, int M,
                                                 int N, int kchunk, int ktot, float alpha,
                                                 const float* __restrict__ bias,
                                                 const _Float16* __restrict__ mask, int ldm,
                                                 void* __restrict__ C, int ldc) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nbn = (N + 63) / 64;  // column blocks; blockIdx.x = row block * nbn + column block
    const int m0 = (int)(blockIdx.x / nbn) * 64 + (wave & 1) * 32;
    const int n0 = (int)(blockIdx.x % nbn) * 64 + (wave >> 1) * 32;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(ktot, kb + kchunk);
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const _Float16* a0 = A + (int64_t)min(m0 + r, M - 1) * lda + kq;
    const _Float16* a1 = A + (int64_t)min(m0 + 16 + r, M - 1) * lda + kq;
    const _Float16* b0 = B + (int64_t)min(n0 + r, N - 1) * ldb + kq;
    const _Float16* b1 = B + (int64_t)min(n0 + 16 + r, N - 1) * ldb + kq;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k = kb; k < ke; k += 32) {
        const h8 fa0 = *reinterpret_cast<const h8*>(a0 + k);
        const h8 fa1 = *reinterpret_cast<const h8*>(a1 + k);
        const h8 fb0 = *reinterpret_cast<const h8*>(b0 + k);
        const h8 fb1 = *reinterpret_cast<const h8*>(b1 + k);
        acc[0][0] = mfma16(fa0, fb0, acc[0][0]);
        acc[0][1] = mfma16(fa0, fb1, acc[0][1]);
        acc[1][0] = mfma16(fa1, fb0, acc[1][0]);
        acc[1][1] = mfma16(fa1, fb1, acc[1][1]);
    }
    if constexpr (EPI == kEpiRelu16 || EPI == kEpiF32) {
        // full 64-column tiles: the workgroup's 64 x 64 outputs go through LDS and
        // out as whole rows, 16 bytes per store
        const int bm = (int)(blockIdx.x / nbn) * 64, bn = (int)(blockIdx.x % nbn) * 64;
        if (bn + 64 <= N && ldc % 8 == 0 && ((uintptr_t)C & 15) == 0) {
            constexpr int ES = EPI == kEpiRelu16 ? 2 : 4;   // output bytes per element
            constexpr int RB = 64 * ES + 16;                // LDS row stride in bytes (padded)
            __shared__ __align__(16) unsigned char tile[64 * RB];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int cl = (wave >> 1) * 32 + 16 * j + (lane & 15);
                    const float bv = bias ? bias[bn + cl] : 0.0f;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int rl = (wave & 1) * 32 + 16 * i + 4 * (lane >> 4) + e;
                        const float v = alpha * acc[i][j][e] + bv;
                        if constexpr (EPI == kEpiRelu16)
                            reinterpret_cast<_Float16*>(tile + rl * RB)[cl] = (_Float16)fmaxf(v, 0.0f);
                        else
                            reinterpret_cast<float*>(tile + rl * RB)[cl] = v;
                    }
                }
            __syncthreads();
            constexpr int CPR = 64 * ES / 16;  // 16-byte chunks per row
#pragma unroll
            for (int c = threadIdx.x; c < 64 * CPR; c += 256) {
                const int rl = c / CPR, ch = c % CPR, row = bm + rl;
                if (row < M)
                    *reinterpret_cast<uint4*>(static_cast<unsigned char*>(C) + ((int64_t)row * ldc + bn) * ES +
                                              16 * ch) = *reinterpret_cast<const uint4*>(tile + rl * RB + 16 * ch);
            }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + 16 * j + (lane & 15);
            if (col >= N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + 16 * i + 4 * (lane >> 4) + e;
                if (row >= M) continue;
                const float v = alpha * acc[i][j][e];
                const int64_t at = (int64_t)row * ldc + col;
                if (EPI == kEpiRelu16) {
                    static_cast<_Float16*>(C)[at] = (_Float16)fmaxf(v + bias[col], 0.0f);
                } else if (EPI == kEpiF32) {
                    static_cast<float*>(C)[at] = v + (bias ? bias[col] : 0.0f);
                } else if (EPI == kEpiMask16) {
                    const bool on = (float)mask[(int64_t)row * ldm + col] > 0.0f;
                    static_cast<_Float16*>(C)[at] = (_Float16)(on ? v : 0.0f);
                } else {
                    static_cast<float*>(C)[(int64_t)blockIdx.z * M * ldc + at] = v;
                }
            }
        }
}

// ---------------------------------------------------------------- fused forward
// The whole network on tiles of 64 rows with the hidden layers in LDS only:
// the encode path, which keeps no activations for a backward pass. The same
// MFMAs in the same order as the three k_gemm_nt launches (16x16x32 over k in
// ascending steps of 32 from zero) and the same epilogues, so Y is bit for
// bit theirs. A workgroup of 8 waves holds every weight fragment it uses in
// registers for the whole launch (wave w: layer 1 and 2 columns [32 w, 32 w +
// 32), layer 3 columns [16 (w & 3), + 16) for rows [32 (w >> 2), + 32)) and
// walks over the row tiles, so the weights leave L2 once per workgroup rather
// than once per tile; the next tile's rows are loaded while the current one
// runs layers 2 and 3. Rows past M read the last row and are not stored. The
// 64 rows are 8 blocks of 8 isometry rows: the layer-3 tile goes through LDS
// and each wave finishes one block's sum and norm with the arithmetic of
// k_iso_norm, in the same order, so the embeddings G16 are bit for bit those
// of k_iso_norm on Y.
constexpr int kFuseRows = 64;
constexpr int kFuseWaves = 8;
constexpr int kFuseLd = kMlpHid + 8;  // LDS row stride of a hidden layer in halves (16 bytes of padding)

__global__ __launch_bounds__(kFuseWaves * 64) void k_mlp_forward(const _Float16* __restrict__ X, int M,
                                                                 const _Float16* __restrict__ w16,
                                                                 const float* __restrict__ w,
                                                                 _Float16* __restrict__ G16) {
    __shared__ __align__(16) _Float16 sH1[kFuseRows * kFuseLd];
    __shared__ __align__(16) _Float16 sH2[kFuseRows * kFuseLd];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4, kq = g * 8;
    const int ntiles = (M + kFuseRows - 1) / kFuseRows;
    if ((int)blockIdx.x >= ntiles) return;
    const _Float16* W1 = w16 + kH16W1;
    const _Float16* W2 = w16 + kH16W2;
    const _Float16* W3 = w16 + kH16W3;
    constexpr int K1 = kMlpIn / 32, K2 = kMlpHid / 32;
    const int c0 = 32 * wave;                                 // layers 1, 2: this wave's first column
    const int c3 = 16 * (wave & 3), r3 = 32 * (wave >> 2);  // layer 3: its columns and rows

    // the weight fragments and biases of this wave, for every tile
    h8 fb1[K1][2], fb2[K2][2], fb3[K2];
#pragma unroll
    for (int kk = 0; kk < K1; ++kk)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            fb1[kk][j] = *reinterpret_cast<const h8*>(W1 + (c0 + 16 * j + r) * kMlpIn + 32 * kk + kq);
#pragma unroll
    for (int kk = 0; kk < K2; ++kk) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
            fb2[kk][j] = *reinterpret_cast<const h8*>(W2 + (c0 + 16 * j + r) * kMlpHid + 32 * kk + kq);
        fb3[kk] = *reinterpret_cast<const h8*>(W3 + (c3 + r) * kMlpHid + 32 * kk + kq);
    }
    float bias1[2], bias2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        bias1[j] = w[kOffB1 + c0 + 16 * j + r];
        bias2[j] = w[kOffB2 + c0 + 16 * j + r];
    }
    const float bias3 = w[kOffB3 + c3 + r];

    auto load_rows = [&](int m0, h8 (&fa)[K1][4]) {
#pragma unroll
        for (int kk = 0; kk < K1; ++kk)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                fa[kk][i] = *reinterpret_cast<const h8*>(X + (int64_t)min(m0 + 16 * i + r, M - 1) * kMlpIn + 32 * kk + kq);
    };
    h8 fa[K1][4];
    load_rows((int)blockIdx.x * kFuseRows, fa);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int m0 = tile * kFuseRows;
        f4 acc[4][2];

        // layer 1: H1 = max(X W1^T + b1, 0), K = 64
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < K1; ++kk)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(fa[kk][i], fb1[kk][j], acc[i][j]);
        // the next tile's rows, in flight during layers 2 and 3
        if (tile + (int)gridDim.x < ntiles) load_rows((tile + gridDim.x) * kFuseRows, fa);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = c0 + 16 * j + r;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    sH1[(16 * i + 4 * g + e) * kFuseLd + col] = (_Float16)fmaxf(1.0f * acc[i][j][e] + bias1[j], 0.0f);
        }
        __syncthreads();

        // layer 2: H2 = max(H1 W2^T + b2, 0), K = 256
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < K2; ++kk) {
            h8 a[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const h8*>(sH1 + (16 * i + r) * kFuseLd + 32 * kk + kq);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(a[i], fb2[kk][j], acc[i][j]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = c0 + 16 * j + r;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    sH2[(16 * i + 4 * g + e) * kFuseLd + col] = (_Float16)fmaxf(1.0f * acc[i][j][e] + bias2[j], 0.0f);
        }
        __syncthreads();

        // layer 3: Y = H2 W3^T + b3, K = 256; rows [r3, r3 + 32), columns [c3, c3 + 16)
        f4 out[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) out[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < K2; ++kk)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const h8 a = *reinterpret_cast<const h8*>(sH2 + (r3 + 16 * i + r) * kFuseLd + 32 * kk + kq);
                out[i] = mfma16(a, fb3[kk], out[i]);
            }
        // Y tile in LDS (H1's space: every read of H1 is before the barrier above)
        constexpr int kYLd = kMlpOut + 4;
        float* tY = reinterpret_cast<float*>(sH1);
        static_assert(kFuseRows * kYLd * 4 <= kFuseRows * kFuseLd * 2, "Y tile fits in H1's space");
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) tY[(r3 + 16 * i + 4 * g + e) * kYLd + c3 + r] = 1.0f * out[i][e] + bias3;
        __syncthreads();
        // S_q = sum_t Y[8 q + t], G_q = S_q / |S_q|: wave w takes block w
        {
            const int q = wave, row0 = m0 + 8 * q;
            float sum = 0.0f;
#pragma unroll
            for (int t = 0; t < 8; ++t) sum += tY[(8 * q + t) * kYLd + lane];
            const float nn = sqrtf(wave_sum_f32(sum * sum));
            const float gq = nn > 0.0f ? sum / nn : 0.0f;
            if (row0 < M) G16[(int64_t)(row0 / 8) * 64 + lane] = (_Float16)gq;
        }
        __syncthreads();  // the Y tile is read before the next tile's H1 overwrites it
    }
}

// ---------------------------------------------------------------- embedding
// S_q = sum_t Y[8 q + t]; G_q = S_q / |S_q| (0 if S_q = 0). One wave per block.
__global__ __launch_bounds__(256) void k_iso_norm(const float* __restrict__ Y, int n,
                                                  float* __restrict__ G32, float* __restrict__ nrm,
                                                  _Float16* __restrict__ G16) {
    const int q = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= n) return;
    const float* y = Y + (int64_t)q * 8 * 64 + lane;
    float s = 0.0f;
#pragma unroll
    for (int t = 0; t < 8; ++t) s += y[t * 64];
    const float nn = sqrtf(wave_sum_f32(s * s));
    const float g = nn > 0.0f ? s / nn : 0.0f;
    if (G32) G32[(int64_t)q * 64 + lane] = g;
    if (nrm && lane == 0) nrm[q] = nn;
    G16[(int64_t)q * 64 + lane] = (_Float16)g;
}

// ---------------------------------------------------------------- loss
// One workgroup per range: z = Z[r][0..nd) (similarities / tau), label y.
// loss[r] = logsumexp(z) - z_y; P[r][j] = softmax(z)_j - [j = y] (fp16), zero
// for nd <= j < ldp. A label outside 0..nd-1 zeroes the row (no loss).
__global__ __launch_bounds__(256) void k_softmax_ce(const float* __restrict__ Z, int ldz, int nd,
                                                    const int32_t* __restrict__ labels,
                                                    _Float16* __restrict__ P, int ldp,
                                                    float* __restrict__ loss) {
    __shared__ float red[4];
    const int r = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const float* z = Z + (int64_t)r * ldz;
    _Float16* p = P + (int64_t)r * ldp;
    const int y = labels[r];
    if (y < 0 || y >= nd) {
        for (int j = tid; j < ldp; j += 256) p[j] = (_Float16)0.0f;
        if (tid == 0) loss[r] = 0.0f;
        return;
    }
    float m = -INFINITY;
    for (int j = tid; j < nd; j += 256) m = fmaxf(m, z[j]);
    m = wave_max_f32(m);
    if (lane == 0) red[wave] = m;
    __syncthreads();
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    float s = 0.0f;
    for (int j = tid; j < nd; j += 256) s += __expf(z[j] - m);
    s = wave_sum_f32(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    s = red[0] + red[1] + red[2] + red[3];
    const float lse = m + __logf(s);
    for (int j = tid; j < ldp; j += 256) {
        float v = 0.0f;
        if (j < nd) v = __expf(z[j] - lse) - (j == y ? 1.0f : 0.0f);
        p[j] = (_Float16)v;
    }
    if (tid == 0) loss[r] = lse - z[y];
}

// mean of n values (one workgroup)
__global__ __launch_bounds__(256) void k_mean(const float* __restrict__ v, int n, float* __restrict__ out) {
    __shared__ float red[4];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += v[i];
    s = wave_sum_f32(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1] + red[2] + red[3]) / (float)max(n, 1);
}

// out[c][r] = in[r][c] for r < rows, c < cols; zero for rows <= r < rows_pad.
__global__ __launch_bounds__(256) void k_transpose16(const _Float16* __restrict__ in, int ldi,
                                                     int rows, int cols,
                                                     _Float16* __restrict__ out, int ldo,
                                                     int rows_pad) {
    __shared__ _Float16 tile[64][65];
    const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < rows && c < cols) ? in[(int64_t)r * ldi + c] : (_Float16)0.0f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int c = c0 + i, r = r0 + tx;
        if (c < cols && r < rows_pad) out[(int64_t)c * ldo + r] = tile[tx][i];
    }
}

// dS = (dG - G (G . dG)) / |S| for each block; records max |dS| (float bits).
__global__ __launch_bounds__(256) void k_norm_bwd(const float* __restrict__ dG,
                                                  const float* __restrict__ G,
                                                  const float* __restrict__ nrm, int n,
                                                  float* __restrict__ dS,
                                                  uint32_t* __restrict__ maxbits) {
    const int q = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= n) return;
    const int64_t at = (int64_t)q * 64 + lane;
    const float g = G[at], dg = dG[at], nn = nrm[q];
    const float dot = wave_sum_f32(g * dg);
    const float v = nn > 0.0f ? (dg - g * dot) / nn : 0.0f;
    dS[at] = v;
    const float mx = wave_max_f32(fabsf(v));
    if (lane == 0) atomicMax(maxbits, __float_as_uint(mx));
}

// Power-of-two scale that brings max |dS| near 2^10 for the fp16 backward.
__device__ inline float grad_scale(uint32_t maxbits) {
    const float mx = __uint_as_float(maxbits);
    if (!(mx > 0.0f) || !isfinite(mx)) return 1.0f;
    const int e = 10 - (int)ceilf(log2f(mx));
    return ldexpf(1.0f, max(-60, min(60, e)));
}

// dY16[8 q + t] = fp16(dS_q * scale) for every isometry t.
__global__ __launch_bounds__(256) void k_expand_grad(const float* __restrict__ dS, int n,
                                                     const uint32_t* __restrict__ maxbits,
                                                     _Float16* __restrict__ dY) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)n * 8 * 64) return;
    const int64_t q = i >> 9;
    const int e = (int)(i & 63);
    dY[i] = (_Float16)(dS[q * 64 + e] * grad_scale(*maxbits));
}

// out[c] = sum_r At[c][r] (one workgroup per c)
__global__ __launch_bounds__(256) void k_row_sums(const _Float16* __restrict__ At, int ld, int len,
                                                  float* __restrict__ out) {
    __shared__ float red[4];
    const _Float16* a = At + (int64_t)blockIdx.x * ld;
    float s = 0.0f;
    for (int r = threadIdx.x; r < len; r += 256) s += (float)a[r];
    s = wave_sum_f32(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// grad[i] = (sum over splits of part[s][i]) * scale / grad_scale
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ part, int splits,
                                                     int count, float scale,
                                                     const uint32_t* __restrict__ maxbits,
                                                     float* __restrict__ grad) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + i];
    grad[i] = s * scale / grad_scale(*maxbits);
}

// bias gradients: grad[i] = sums[i] * scale / grad_scale
__global__ void k_scale_into(const float* __restrict__ sums, int count, float scale,
                             const uint32_t* __restrict__ maxbits, float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) grad[i] = sums[i] * scale / grad_scale(*maxbits);
}

// Adam with bias correction (bc1 = 1 - beta1^t, bc2 = 1 - beta2^t); writes
// the fp16 weight copies and their transposes.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ g, float lr, float beta1,
                                              float beta2, float eps, float bc1, float bc2,
                                              _Float16* __restrict__ w16) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    const _Float16 h = (_Float16)wi;
    if (i >= kOffW1 && i < kOffB1) {
        const int o = (i - kOffW1) / kMlpIn, k = (i - kOffW1) % kMlpIn;
        w16[kH16W1 + o * kMlpIn + k] = h;
        w16[kH16W1t + k * kMlpHid + o] = h;
    } else if (i >= kOffW2 && i < kOffB2) {
        const int o = (i - kOffW2) / kMlpHid, k = (i - kOffW2) % kMlpHid;
        w16[kH16W2 + o * kMlpHid + k] = h;
        w16[kH16W2t + k * kMlpHid + o] = h;
    } else if (i >= kOffW3 && i < kOffB3) {
        const int o = (i - kOffW3) / kMlpHid, k = (i - kOffW3) % kMlpHid;
        w16[kH16W3 + o * kMlpHid + k] = h;
        w16[kH16W3t + k * kMlpOut + o] = h;
    }
}

// fp16 copies (and transposes) of the master weights
__global__ __launch_bounds__(256) void k_weights16(const float* __restrict__ w, _Float16* __restrict__ w16) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams) return;
    const _Float16 h = (_Float16)w[i];
    if (i < kOffB1) {
        const int o = i / kMlpIn, k = i % kMlpIn;
        w16[kH16W1 + o * kMlpIn + k] = h;
        w16[kH16W1t + k * kMlpHid + o] = h;
    } else if (i >= kOffW2 && i < kOffB2) {
        const int o = (i - kOffW2) / kMlpHid, k = (i - kOffW2) % kMlpHid;
        w16[kH16W2 + o * kMlpHid + k] = h;
        w16[kH16W2t + k * kMlpHid + o] = h;
    } else if (i >= kOffW3 && i < kOffB3) {
        const int o = (i - kOffW3) / kMlpHid, k = (i - kOffW3) % kMlpHid;
        w16[kH16W3 + o * kMlpHid + k] = h;
        w16[kH16W3t + k * kMlpOut + o] = h;
    }
}

// ---------------------------------------------------------------- top-k similarity
// Proposals: the k best keys (domain embeddings) of each query (range
// embedding) by similarity, ties to the lower key index. The similarity is the
// dot product of int8 codes of the embeddings, q = rint(x s) with one scale s
// = 127 / max |x| over the queries and the keys together (fp32 arithmetic),
// so scores are integers (|score| <= 64 * 127^2), exact in int32 in any
// summation order; one v_mfma_i32_16x16x64_i8 gives a 16 x 16 tile. Two
// passes over the keys, split into nc chunks:
//  1. per query, the largest score of each group of keys, a group being the
//     keys of one chunk and one column lane (index mod 16 within the chunk's
//     stages): 16 nc disjoint groups. Each maximum is the score of a key of
//     its group, so at least 32 keys score at least theta, the 32nd largest
//     maximum (of the lanes' maxima when there are more than 64 groups; below
//     every score with fewer than 32): no key scoring below theta is among
//     the best 32;
//  2. the keys scoring at least theta: the MFMA started at -theta gives
//     score - theta exactly, so a tile's screen is one maximum and a sign;
//     passing elements whose key (score, then lower index) is above the
//     list's threshold enter a list per (query, chunk). A list that could
//     overflow keeps its best 32 and takes the 32nd as its threshold.
// A merge sorts each query's lists. With theta near the 32nd best score a
// query keeps a few dozen keys; a running top-32 admits every key that beats
// the keys seen before it, hundreds per query.
constexpr int kTopK = 32;    // largest proposal count
constexpr int kTkRT = 4;     // 16-row tiles per wave: 64 queries
constexpr int kTkWaves = 4;  // waves per workgroup
constexpr int kTkQ = kTkWaves * 16 * kTkRT;
constexpr int kTkCap = 48;   // list slots per (query, chunk)
constexpr int kTkCols = 128;  // keys per LDS stage (64 bytes each)
constexpr int kTkTiles = kTkCols / 16;
constexpr int kTkScoreCap = 1 << 21;  // above every |score| (64 * 127^2 < 2^20)

// Ordered key: larger key = larger score, then lower domain index.
__device__ inline uint64_t tk_key(float s, int d) {
    uint32_t u = __float_as_uint(s);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)u << 32) | (uint32_t)(~(uint32_t)d);
}

__device__ inline float tk_score(uint64_t key) {
    uint32_t u = (uint32_t)(key >> 32);
    u = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    return __uint_as_float(u);
}

__device__ inline int tk_index(uint64_t key) { return (int)(~(uint32_t)key); }

// A 64-bit value moved by a DPP lane pattern (CTRL: quad_perm = 0x00..0xff,
// row_ror:n = 0x120 + n); every pattern used here reads a lane of the same row.
template <int CTRL>
__device__ inline uint64_t dpp_u64(uint64_t v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// v of lane ^ j. Distances 1 and 2 are quad permutations and 8 the rotation
// of a 16-lane row by 8 (DPP: no LDS round trip). Distance 4 takes the
// rotation by 4 or by 12, whichever came from lane ^ 4 (from4, found once by
// rotating the lane ids). 16 and 32 go through ds_bpermute.
__device__ inline uint64_t xor_lane_u64(uint64_t v, int j, bool from4) {
    switch (j) {
        case 1: return dpp_u64<0xb1>(v);  // quad_perm [1, 0, 3, 2]
        case 2: return dpp_u64<0x4e>(v);  // quad_perm [2, 3, 0, 1]
        case 4: {
            const uint64_t a = dpp_u64<0x124>(v), b = dpp_u64<0x12c>(v);
            return from4 ? a : b;
        }
        case 8: return dpp_u64<0x128>(v);
        default: return shfl_xor_u64(v, j);
    }
}

// Bitonic sort of one key per lane, descending across the wave.
__device__ inline uint64_t wave_sort_desc(uint64_t v, int lane) {
    const bool from4 = __builtin_amdgcn_update_dpp(0, lane, 0x124, 0xf, 0xf, false) == (lane ^ 4);
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t o = xor_lane_u64(v, j, from4);
            const bool take_max = ((lane & j) == 0) == ((lane & k) == 0);
            v = take_max ? (v > o ? v : o) : (v < o ? v : o);
        }
    return v;
}

// Ordered bits of a score (the high word of its key).
__device__ inline uint32_t tk_ord(float s) {
    const uint32_t u = __float_as_uint(s);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// max |x| over fp16 arrays a [na] and b [nb] (multiples of 8 values), as
// float bits (non-negative floats order as unsigned integers); *out starts at 0
__global__ __launch_bounds__(256) void k_tk_absmax(const _Float16* __restrict__ a, int64_t na,
                                                   const _Float16* __restrict__ b, int64_t nb,
                                                   uint32_t* __restrict__ out) {
    float m = 0.0f;
    const int64_t n8 = (na + nb) / 8;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n8; t += (int64_t)gridDim.x * 256) {
        const h8 v = t < na / 8 ? reinterpret_cast<const h8*>(a)[t] : reinterpret_cast<const h8*>(b)[t - na / 8];
#pragma unroll
        for (int e = 0; e < 8; ++e) m = fmaxf(m, fabsf((float)v[e]));
    }
    m = wave_max_f32(m);
    if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(out, __float_as_uint(m));
}

// int8 codes q = rint(x s), s = 127 / m (m = *mbits as a float; s = 0 when m = 0),
// 8 values per thread
__global__ __launch_bounds__(256) void k_tk_quant(const _Float16* __restrict__ x, int64_t n8,
                                                  const uint32_t* __restrict__ mbits, int8_t* __restrict__ q) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n8) return;
    const float m = __uint_as_float(*mbits);
    const float sc = m > 0.0f ? 127.0f / m : 0.0f;
    const h8 v = reinterpret_cast<const h8*>(x)[t];
    uint32_t w[2] = {0u, 0u};
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e >> 2] |= (uint32_t)(uint8_t)(int8_t)(int)rintf((float)v[e] * sc) << (8 * (e & 3));
    reinterpret_cast<uint2*>(q)[t] = make_uint2(w[0], w[1]);
}

// Shared by the two passes: the query codes as A operands, the stage copies
// and the tiles. grid: x = blocks of kTkQ queries, y = key chunks; the keys of
// a chunk stream through LDS in stages of kTkCols codes (64 bytes each),
// copied straight from global memory in 16-byte chunks (no registers on the
// way, as the MFMA grid matchers copy their columns): chunk u (values 16 u ..
// 16 u + 15) of key c at c * 4 + (u ^ ((c >> 2) & 3)), so that the 16 keys of
// a tile read one chunk each from distinct banks.
constexpr int kTkLoads = kTkCols * 4 / (kTkWaves * 64);
static_assert(kTkWaves * kTkLoads * 64 == kTkCols * 4, "a stage is whole 16-byte chunks per lane");

__device__ inline int tk_swz(int c) { return (c >> 2) & 3; }
__device__ inline int tk_chunk(int c, int u) { return c * 4 + (u ^ tk_swz(c)); }

struct TkWave {
    int nq, lo, hi, wave, lane, g, c16, wq0;
    v4i af[kTkRT];
    uint32_t off[kTkLoads];  // byte offsets of a full stage's chunks, from the stage's first key
};

__device__ __forceinline__ bool tk_setup(TkWave& w, const int8_t* __restrict__ QR, int nq, int nk) {
    const int q0 = blockIdx.x * kTkQ;
    if (q0 >= nq) return false;
    const int nc = gridDim.y, c = blockIdx.y;
    w.nq = nq;
    w.lo = (int)((int64_t)nk * c / nc);
    w.hi = (int)((int64_t)nk * (c + 1) / nc);
    w.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    w.lane = threadIdx.x & 63;
    w.g = w.lane >> 4;
    w.c16 = w.lane & 15;
    w.wq0 = q0 + w.wave * 16 * kTkRT;
    // query rows past the end read the last row and are never written
#pragma unroll
    for (int rt = 0; rt < kTkRT; ++rt)
        w.af[rt] = *reinterpret_cast<const v4i*>(QR + (int64_t)min(w.wq0 + 16 * rt + w.c16, nq - 1) * 64 + 16 * w.g);
#pragma unroll
    for (int l = 0; l < kTkLoads; ++l) {
        const int i = (kTkLoads * w.wave + l) * 64 + w.lane, col = i >> 2, u = (i & 3) ^ tk_swz(col);
        w.off[l] = (uint32_t)(col * 64 + 16 * u);
    }
    return true;
}

// Copy keys b0 .. b0 + n - 1 (n <= kTkCols; keys past n copy key n - 1) into dD.
__device__ __forceinline__ void tk_stage_copy(const TkWave& w, const int8_t* __restrict__ QD, v4i* dD, int b0,
                                              int n) {
    // the same in every lane: read from the first so that they sit in SGPRs
    const uint64_t bu = (uint64_t)(uintptr_t)(QD + (int64_t)b0 * 64);
    const void* base = (const void*)(uintptr_t)(
        ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(bu >> 32)) << 32) |
        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)bu));
#pragma unroll
    for (int l = 0; l < kTkLoads; ++l) {
        const uint32_t o =
            n == kTkCols ? w.off[l] : (uint32_t)(min((int)(w.off[l] >> 6), n - 1) * 64) + (w.off[l] & 63u);
        const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uintptr_t)(
            (const __attribute__((address_space(3))) void*)(dD + (kTkLoads * w.wave + l) * 64)));
        m8_copy_to_lds(base, o, (const __attribute__((address_space(3))) void*)(uintptr_t)la);
    }
}

__device__ __forceinline__ void tk_wait_copies() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// One 16-key tile (ct) for every row tile, the accumulators started at c0.
__device__ __forceinline__ void tk_tile(const TkWave& w, const v4i* cD, int ct, const v4i (&c0)[kTkRT],
                                        v4i (&acc)[kTkRT]) {
    const v4i b = cD[tk_chunk(16 * ct + w.c16, w.g)];
#pragma unroll
    for (int rt = 0; rt < kTkRT; ++rt) acc[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(w.af[rt], b, c0[rt], 0, 0, 0);
}

// The chunk's stages, double-buffered: fn(buffer, first key) on each while
// the next one is copied in.
template <class Fn>
__device__ __forceinline__ void tk_stages(const TkWave& w, const int8_t* __restrict__ QD, v4i (*sD)[kTkCols * 4],
                                          Fn&& fn) {
    tk_wait_copies();
    if (w.lo < w.hi) {
        tk_stage_copy(w, QD, sD[0], w.lo, min(kTkCols, w.hi - w.lo));
        tk_wait_copies();
    }
    __syncthreads();
    int buf = 0;
    for (int base = w.lo; base < w.hi; base += kTkCols, buf ^= 1) {
        const int nb = base + kTkCols;
        if (nb < w.hi) tk_stage_copy(w, QD, sD[buf ^ 1], nb, min(kTkCols, w.hi - nb));
        fn(sD[buf], base);
        tk_wait_copies();
        __syncthreads();
    }
}

// Pass 1: GM [nq][16 nc], the largest score of each (chunk, column lane) group
// of keys per query (INT_MIN for an empty group).
__global__ __launch_bounds__(kTkWaves * 64) void k_tk_max(const int8_t* __restrict__ QR, int nq,
                                                          const int8_t* __restrict__ QD, int nk,
                                                          int32_t* __restrict__ GM) {
    __shared__ v4i sD[2][kTkCols * 4];
    TkWave w;
    if (!tk_setup(w, QR, nq, nk)) return;
    constexpr int RT = kTkRT;
    const v4i zero[RT] = {};
    int m[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) m[rt][e] = INT_MIN;
    // fold a stage into m, two tiles at a time (keys past the chunk's end count as INT_MIN)
    tk_stages(w, QD, sD, [&](const v4i* cD, int base) {
        const bool tail = base + kTkCols > w.hi;
#pragma unroll 2
        for (int ct = 0; ct < kTkTiles; ct += 2) {
            v4i x0[RT], x1[RT];
            tk_tile(w, cD, ct, zero, x0);
            tk_tile(w, cD, ct + 1, zero, x1);
            if (tail) {
                const bool ok0 = base + 16 * ct + w.c16 < w.hi, ok1 = base + 16 * ct + 16 + w.c16 < w.hi;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        x0[rt][e] = ok0 ? x0[rt][e] : INT_MIN;
                        x1[rt][e] = ok1 ? x1[rt][e] : INT_MIN;
                    }
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int e = 0; e < 4; ++e) m[rt][e] = max(max(m[rt][e], x0[rt][e]), x1[rt][e]);
        }
    });
    const int c = blockIdx.y, G = 16 * gridDim.y;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = w.wq0 + 16 * rt + 4 * w.g + e;
            if (q < nq) GM[(int64_t)q * G + 16 * c + w.c16] = m[rt][e];
        }
}

// Per query (one wave): theta, the 32nd largest group maximum (of the lanes'
// maxima over groups lane, lane + 64, ... when there are more than 64), or
// -kTkScoreCap (below every score) when fewer than 32 groups hold a key.
__global__ __launch_bounds__(256) void k_tk_theta(const int32_t* __restrict__ GM, int nq, int G,
                                                  int32_t* __restrict__ theta) {
    const int q = (int)((blockIdx.x * 256u + threadIdx.x) >> 6), lane = threadIdx.x & 63;
    if (q >= nq) return;
    int m = INT_MIN;
    for (int j = lane; j < G; j += 64) m = max(m, GM[(int64_t)q * G + j]);
    const uint64_t v = wave_sort_desc((uint64_t)((uint32_t)m ^ 0x80000000u) << 32, lane);
    const int t = (int)((uint32_t)(shfl_u64(v, kTopK - 1) >> 32) ^ 0x80000000u);
    if (lane == 0) theta[q] = max(t, -kTkScoreCap);
}

// Pass 2: per (query, chunk) the list [kTkCap] of keys scoring at least
// theta, and its count.
__global__ __launch_bounds__(kTkWaves * 64) void k_tk_collect(const int8_t* __restrict__ QR, int nq,
                                                              const int8_t* __restrict__ QD, int nk,
                                                              const int32_t* __restrict__ th_in,
                                                              uint64_t* __restrict__ list,
                                                              int32_t* __restrict__ lcount) {
    constexpr int RT = kTkRT, WR = 16 * RT;
    static_assert(WR == 64, "one query per lane in the list bookkeeping");
    __shared__ v4i sD[2][kTkCols * 4];
    __shared__ uint64_t sThr[kTkWaves][WR];  // keys above this enter the query's list
    __shared__ __align__(16) int32_t sTh[kTkWaves][WR];  // its score
    __shared__ int32_t sCnt[kTkWaves][WR];
    // list entries on their way to global memory: stored in batches, because
    // the wait for a stage's copy would also wait for every store before it
    // (room for a row tile's elements, 4 per lane, beyond the flush mark)
    constexpr int kQ = 128 + 4 * 64;
    __shared__ uint32_t sQi[kTkWaves][kQ];  // list position (row * kTkCap + slot)
    __shared__ uint64_t sQk[kTkWaves][kQ];  // key
    __shared__ int32_t sQn[kTkWaves];       // queued entries
    TkWave w;
    if (!tk_setup(w, QR, nq, nk)) return;
    const int c = blockIdx.y, wave = w.wave, lane = w.lane, g = w.g, c16 = w.c16;
    {
        const int q = w.wq0 + lane;
        const int t = q < nq ? th_in[q] : kTkScoreCap;  // padded rows: above every score
        // keys of scores >= t: ord(t) << 32 and above
        sThr[wave][lane] = ((uint64_t)tk_ord((float)t) << 32) - 1u;
        sTh[wave][lane] = t;
        sCnt[wave][lane] = 0;
    }
    wave_lds_sync();
    v4i cs[RT];  // per row 16 rt + 4 g + e: the screen start -theta
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) cs[rt] = -*reinterpret_cast<const v4i*>(&sTh[wave][16 * rt + 4 * g]);
    uint64_t* wlist = list + ((int64_t)c * nq + w.wq0) * kTkCap;
    if (lane == 0) sQn[wave] = 0;
    wave_lds_sync();
    auto flush = [&] {
        wave_lds_sync();
        const int qn = sQn[wave];
        for (int j = lane; j < qn; j += 64) wlist[sQi[wave][j]] = sQk[wave][j];
        wave_lds_sync();
        if (lane == 0) sQn[wave] = 0;
        wave_lds_sync();
    };
    // the rows whose list could overflow keep their best 32
    auto prune = [&] {
        flush();
        const int nl = sCnt[wave][lane];
        uint64_t need = __ballot(nl > kTkCap - 16);
        tk_wait_copies();  // this wave's list stores have landed
        while (need) {
            const int i = __ffsll((unsigned long long)need) - 1;
            need &= need - 1;
            const int n = __shfl(nl, i, 64);
            uint64_t* L = wlist + (int64_t)i * kTkCap;
            // read from L2, past this CU's vector cache
            uint64_t v = lane < n ? __hip_atomic_load(L + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
            v = wave_sort_desc(v, lane);
            if (lane < kTopK) L[lane] = v;
            const uint64_t t = shfl_u64(v, kTopK - 1);
            if (lane == 0) {
                sCnt[wave][i] = kTopK;
                sThr[wave][i] = t;
                sTh[wave][i] = (int)tk_score(t);
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) cs[rt] = -*reinterpret_cast<const v4i*>(&sTh[wave][16 * rt + 4 * g]);
    };
    // a stage: the screen of every tile without a branch (one maximum per
    // lane and one ballot: a bit per tile with an element at or above theta;
    // a branch per tile would keep the next tile's LDS reads from being issued
    // early), then the flagged tiles again and their elements above the list
    // threshold queued. (LDS operations of one wave take effect in program
    // order, so the counts and thresholds need no fence here.)
    tk_stages(w, QD, sD, [&](const v4i* cD, int base) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) asm volatile("" : "+v"(cs[rt]));
        uint32_t hits = 0;  // bit ct: tile ct has an element at or above theta
#pragma unroll
        for (int ct = 0; ct < kTkTiles; ++ct) {
            v4i acc[RT];
            tk_tile(w, cD, ct, cs, acc);
            int mm = max(max(acc[0][0], acc[0][1]), acc[0][2]);
            mm = max(mm, acc[0][3]);
#pragma unroll
            for (int rt = 1; rt < RT; ++rt) {
                mm = max(max(mm, acc[rt][0]), acc[rt][1]);
                mm = max(max(mm, acc[rt][2]), acc[rt][3]);
            }
            hits |= __ballot(mm >= 0) ? 1u << ct : 0u;
        }
        while (hits) {
            const int ct = __builtin_ffs(hits) - 1;
            hits &= hits - 1;
            const int col = 16 * ct + c16;
            const v4i b = cD[tk_chunk(col, g)];
            const int kc = base + col;
            const bool colok = kc < w.hi;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const v4i x = __builtin_amdgcn_mfma_i32_16x16x64_i8(w.af[rt], b, cs[rt], 0, 0, 0);  // score - theta
                // each lane lists its own elements at or above theta whose key is
                // above the row's threshold: slots and queue places from LDS atomics
                const bool has = colok && max(max(x[0], x[1]), max(x[2], x[3])) >= 0;
                if (has) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (x[e] < 0) continue;
                        const int i = 16 * rt + 4 * g + e;
                        const uint64_t key = tk_key((float)(x[e] - cs[rt][e]), kc);
                        if (key <= sThr[wave][i]) continue;
                        const int slot = atomicAdd(&sCnt[wave][i], 1);
                        const int qp = atomicAdd(&sQn[wave], 1);
                        sQi[wave][qp] = (uint32_t)(i * kTkCap + slot);
                        sQk[wave][qp] = key;
                    }
                }
                // a row tile adds at most 4 entries per lane to the queue
                if (__ballot(has)) {
                    wave_lds_sync();
                    if (sQn[wave] > kQ - 4 * 64) flush();
                }
            }
            // a tile adds at most 16 entries to a row
            if (__ballot(sCnt[wave][lane] > kTkCap - 16)) prune();
        }
    });
    flush();
    if (w.wq0 + lane < nq) lcount[(int64_t)c * nq + w.wq0 + lane] = sCnt[wave][lane];
}

// Best k of a query's lists, best first (one wave per query): the lists'
// entries in order, the first 64 sorted, then 32 at a time into the upper
// lanes, sorted with the best 32 so far.
__global__ __launch_bounds__(256) void k_tk_merge(const uint64_t* __restrict__ list,
                                                  const int32_t* __restrict__ lcount, int nc, int nq, int k,
                                                  int32_t* __restrict__ idx, float* __restrict__ score) {
    const int q = (int)((blockIdx.x * 256u + threadIdx.x) >> 6), lane = threadIdx.x & 63;
    if (q >= nq) return;
    // chunk counts in lanes 0..nc-1, their exclusive prefix sums
    const int cn = lane < nc ? lcount[(int64_t)lane * nq + q] : 0;
    int incl = cn;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    const int excl = incl - cn, total = __shfl(incl, 63, 64);
    int start[16];  // first entry of each chunk (nc <= 16), in every lane
#pragma unroll
    for (int l = 0; l < 16; ++l) start[l] = __shfl(excl, l, 64);
    auto fetch = [&](int p) -> uint64_t {  // entry p of the chunks' lists in order
        int cc = 0, o = p;
#pragma unroll
        for (int l = 1; l < 16; ++l)
            if (l < nc && start[l] <= p) {
                cc = l;
                o = p - start[l];
            }
        return list[((int64_t)cc * nq + q) * kTkCap + o];
    };
    uint64_t v = lane < total ? fetch(lane) : 0ull;
    v = wave_sort_desc(v, lane);
    for (int p = 64; p < total; p += 32) {
        if (lane >= 32) v = p + lane - 32 < total ? fetch(p + lane - 32) : 0ull;
        v = wave_sort_desc(v, lane);
    }
    if (lane < k) {
        idx[(int64_t)q * k + lane] = v ? tk_index(v) : -1;
        if (score) score[(int64_t)q * k + lane] = v ? tk_score(v) : -INFINITY;
    }
}

// ---------------------------------------------------------------- exact rescoring
// One workgroup per 8 x 8 range of the grid; thread (c = tid / 8, t = tid % 8)
// takes isometry t of proposals c, c + 16. Evaluates the distance of eq. (1) exactly over the
// range's proposals, isometries and contrast values (same moment form and tie
// order as the exhaustive matcher) and writes the match; e_num = -1 when the
// range has no proposal. The domains' 2x2 sums d' come from the image (COLS
// 0) or (COLS 1) from the columns that the int8 grid matcher's pool
// preparation already holds for every domain of the level (h and l, d' =
// 128 h + l), with S and A'.
constexpr int kRsThreads = 128;               // threads per range
constexpr int kRsPairs = kTopK * 8 / kRsThreads;  // (proposal, isometry) pairs per thread

template <int COLS>
__global__ __launch_bounds__(kRsThreads) void k_rescore(const uint8_t* __restrict__ img, int pitch,
                                                        int W, int L, int gx, int total,
                                                        const int8_t* __restrict__ Dh, const uint32_t* __restrict__ Sd,
                                                        const int64_t* __restrict__ Ad,
                                                        const int32_t* __restrict__ cand, int kc,
                                                        int nr, KSet ks, fic_match* __restrict__ out) {
    constexpr int NW = kRsThreads / 64;
    __shared__ int sr[64];
    __shared__ __align__(16) int srp[8][64];  // <srp[t], d> = <R, T_t d>
    __shared__ __align__(16) int sd[kTopK][64];
    __shared__ int64_t redF[NW], redK[NW];
    const int q = blockIdx.x, tid = threadIdx.x;
    if (q >= nr) return;
    const int rgx = W / 8;
    const int y = (q / rgx) * 8, x = (q % rgx) * 8;
    if (tid < 64) sr[tid] = img[(int64_t)(y + (tid >> 3)) * pitch + x + (tid & 7)];
    // thread (c0, t) takes the pairs (c0 + 16 u, t), u < kRsPairs
    const int c0 = tid >> 3, t = tid & 7;
    int jv[kRsPairs];
#pragma unroll
    for (int u = 0; u < kRsPairs; ++u) {
        const int c = c0 + (kRsThreads / 8) * u;
        jv[u] = c < kc ? cand[(int64_t)q * kc + c] : -1;
    }
    if constexpr (COLS == 0) {
        for (int e = tid; e < kTopK * 64; e += kRsThreads) {
            const int cc = e >> 6, m = e & 63;
            const int jj = cc < kc ? cand[(int64_t)q * kc + cc] : -1;
            int v = 0;
            if (jj >= 0 && jj < total) {
                const uint8_t* p = img + (int64_t)((jj / gx) * L + 2 * (m >> 3)) * pitch + (jj % gx) * L + 2 * (m & 7);
                v = p[0] + p[1] + p[pitch] + p[pitch + 1];
            }
            sd[cc][m] = v;
        }
    } else {
        // values 8 t .. 8 t + 7 of each of the thread's proposals
#pragma unroll
        for (int u = 0; u < kRsPairs; ++u) {
            const int c = c0 + (kRsThreads / 8) * u, j = jv[u];
            int v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (j >= 0 && j < total) {
                const uint2 hw = *reinterpret_cast<const uint2*>(Dh + (int64_t)j * 128 + 8 * t);
                const uint2 lw = *reinterpret_cast<const uint2*>(Dh + (int64_t)j * 128 + 64 + 8 * t);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t hh = (e < 4 ? hw.x : hw.y) >> (8 * (e & 3)), ll = (e < 4 ? lw.x : lw.y) >> (8 * (e & 3));
                    v[e] = 128 * (int)(hh & 255u) + (int)(ll & 255u);
                }
            }
            *reinterpret_cast<int4*>(&sd[c][8 * t]) = make_int4(v[0], v[1], v[2], v[3]);
            *reinterpret_cast<int4*>(&sd[c][8 * t + 4]) = make_int4(v[4], v[5], v[6], v[7]);
        }
    }
    __syncthreads();
    // the range permuted once per isometry: T_t d takes d[src_t(e)] to place e,
    // so R[e] goes to place src_t(e) of copy t
    for (int i = tid; i < 8 * 64; i += kRsThreads) {
        const int tt = i >> 6, e = i & 63;
        srp[tt][iso_src(8, tt, e >> 3, e & 7)] = sr[e];
    }
    __syncthreads();
    int64_t F = INT64_MAX, K = INT64_MAX;
    // the 8 threads of a proposal group (consecutive lanes) each sum one eighth
    // of the range, then combine; every sum is exact in 32 bits (S2 <= 64 *
    // 1020^2, |Pc| <= 64 * 255 * 1020)
    int SR = 0, SR2 = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = sr[8 * t + u];
        SR += r;
        SR2 += r * r;
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
        SR += __shfl_xor(SR, o, 64);
        SR2 += __shfl_xor(SR2, o, 64);
    }
#pragma unroll
    for (int u = 0; u < kRsPairs; ++u) {
        const int c = c0 + (kRsThreads / 8) * u, j = jv[u];
        int S = 0, S2 = 0;
        if constexpr (COLS == 0) {
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                const int d = sd[c][8 * t + w];
                S += d;
                S2 += d * d;
            }
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                S += __shfl_xor(S, o, 64);
                S2 += __shfl_xor(S2, o, 64);
            }
        }
        if (j >= 0 && j < total) {
            int Pc = 0;
            const int4* pr = reinterpret_cast<const int4*>(srp[t]);
            const int4* pd = reinterpret_cast<const int4*>(sd[c]);
#pragma unroll 4
            for (int e = 0; e < 16; ++e) {
                const int4 a = pr[e], b = pd[e];
                Pc += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
            }
            int64_t Ap;
            if constexpr (COLS == 0) {
                Ap = 64 * (int64_t)S2 - (int64_t)S * S;
            } else {
                S = (int)Sd[j];
                Ap = Ad[j];
            }
            const int64_t Bp = 64 * (int64_t)Pc - (int64_t)SR * S;
            int64_t Fu;
            int s;
            best_contrast(Bp, Ap, ks, Fu, s);
            const int64_t Ku = make_key(j, t, s, (uint32_t)S);
            if (pair_less(Fu, Ku, F, K)) {
                F = Fu;
                K = Ku;
            }
        }
    }
    // workgroup argmin of (F, K)
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t f2 = __shfl_xor(F, o, 64), k2 = __shfl_xor(K, o, 64);
        if (pair_less(f2, k2, F, K)) {
            F = f2;
            K = k2;
        }
    }
    if ((tid & 63) == 0) {
        redF[tid >> 6] = F;
        redK[tid >> 6] = K;
    }
    __syncthreads();
    if (tid != 0) return;
    for (int w = 1; w < NW; ++w)
        if (pair_less(redF[w], redK[w], F, K)) {
            F = redF[w];
            K = redK[w];
        }
    fic_match m;
    m.flags = 0;
    m.pad_ = 0;
    if (K == INT64_MAX) {  // no proposal at all: exhaustive search decides
        m.e_num = -1;
        m.dom = -1;
        m.iso = 0;
        m.s_idx = 0;
        m.k = 0;
        m.q_o = 0;
        m.E = -1.0f;
    } else {
        const int64_t CR = 64 * (int64_t)SR2 - (int64_t)SR * SR;
        const int jj = (int)(K >> 27), tt = (int)((K >> 24) & 7), ss = (int)((K >> 20) & 15);
        const int64_t sdom = K & 0xfffff;
        const int k = ks.consecutive ? ks.k0 + ss : ks.k[ss];
        m.e_num = F + 1600 * CR;
        m.dom = jj;
        m.iso = (uint8_t)tt;
        m.s_idx = (uint8_t)ss;
        m.k = (uint8_t)k;
        m.q_o = (int16_t)floordiv64(2 * (40 * (int64_t)SR - k * sdom) + 40 * 64, 80 * 64);
        m.E = (float)m.e_num / (1600.0f * 64.0f);
    }
    out[q] = m;
}

// The fallback list: ranges with no proposal or with 1600 n E > thr, in grid
// order (so that neighbouring ranges, which cost the exhaustive matcher alike,
// share its workgroups). One workgroup, rounds of 1024 ranges.
__global__ __launch_bounds__(1024) void k_fallback_list(const fic_match* __restrict__ m, int nr, int W,
                                                        int64_t thr, int32_t* __restrict__ fb_act,
                                                        int32_t* __restrict__ fb_q,
                                                        int32_t* __restrict__ fb_count) {
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, rgx = W / 8;
    int done = 0;
    for (int b = 0; b < nr; b += 1024) {
        const int q = b + tid;
        bool f = false;
        if (q < nr) {
            const int64_t e = m[q].e_num;
            f = e < 0 || e > thr;
        }
        const uint64_t bal = __ballot(f);
        if (lane == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        int before = done, tot = 0;
        for (int i = 0; i < 16; ++i) {
            const int c = wsum[i];
            before += i < w ? c : 0;
            tot += c;
        }
        if (f) {
            const int pos = before + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            fb_act[pos] = (((q / rgx) * 8) << 16) | ((q % rgx) * 8);
            fb_q[pos] = q;
        }
        done += tot;
        __syncthreads();  // wsum is rewritten next round
    }
    if (tid == 0) *fb_count = done;
}

// out[fb_q[p]] = exhaustive match p, flagged as a fallback
__global__ void k_fallback_scatter(const fic_match* __restrict__ tmp, const int32_t* __restrict__ fb_q,
                                   const int32_t* __restrict__ fb_count, fic_match* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *fb_count) return;
    fic_match m = tmp[p];
    m.flags |= FIC_FLAG_FALLBACK;
    out[fb_q[p]] = m;
}

// Level codes of a full range grid (single-level encodes, for the decoder).
__global__ void k_level_codes(const fic_match* __restrict__ m, int nr, int W, int B, int L, int gx,
                              fic_code* __restrict__ codes) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nr) return;
    const fic_match a = m[q];
    const int rgx = W / B;
    fic_code c;
    c.e_num = a.e_num;
    c.dom = a.dom;
    c.y = (int16_t)((q / rgx) * B);
    c.x = (int16_t)((q % rgx) * B);
    c.dy = (int16_t)(a.dom >= 0 ? (a.dom / gx) * L : 0);
    c.dx = (int16_t)(a.dom >= 0 ? (a.dom % gx) * L : 0);
    c.q_o = a.q_o;
    c.log2B = (uint8_t)(31 - __clz(B));
    c.iso = a.iso;
    c.k = a.k;
    c.s_idx = a.s_idx;
    c.level = 0;
    for (int i = 0; i < 5; ++i) c.pad_[i] = 0;
    codes[q] = c;
}

}  // namespace fic
