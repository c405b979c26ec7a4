// Peak-rate probes: the rates the roofline fractions are read against,
// measured on the device at hand. Each kernel keeps its unit busy with
// independent chains and stores one value only if it is impossible, so the
// work is not removed.

namespace fic {

constexpr int kPeakIters = 4096;

// 32-bit multiply-add (fp32 FMA, unpacked): 8 chains per lane, 2 ops each.
__global__ __launch_bounds__(256) void k_peak_fma(float seed, float* out) {
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = seed + (float)(threadIdx.x + i);
    const float b = 1.0000001f, c = 1e-7f;
    for (int it = 0; it < kPeakIters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = __builtin_fmaf(a[i], b, c);
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += a[i];
    if (s == -1.0f) out[0] = s;
}

// v_dot2_i32_i16 (the 2 x 2 matcher's instruction): 4 ops per lane.
__global__ __launch_bounds__(256) void k_peak_dot2(int seed, int* out) {
    typedef short s2 __attribute__((ext_vector_type(2)));
    int a[8];
    const s2 x = __builtin_bit_cast(s2, seed | 0x00030000), y = __builtin_bit_cast(s2, seed ^ 0x00050007);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = (int)threadIdx.x + i;
    for (int it = 0; it < kPeakIters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_sdot2(x, y, a[i], false);
    int s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s ^= a[i];
    if (s == 0x7fffffff) out[0] = s;
}

// v_mfma_f32_16x16x32_f16: 2 * 16 * 16 * 32 flops per wave instruction, 4 chains.
__global__ __launch_bounds__(256) void k_peak_mfma_f16(float seed, float* out) {
    typedef _Float16 h8 __attribute__((ext_vector_type(8)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    h8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (_Float16)(seed + (float)i);
        b[i] = (_Float16)(seed - (float)i);
    }
    f4 c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = f4{0.0f, 0.0f, 0.0f, (float)threadIdx.x};
    for (int it = 0; it < kPeakIters / 4; ++it)
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c[i], 0, 0, 0);
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
    if (s == -1.0f) out[0] = s;
}

// v_mfma_i32_16x16x64_i8: 2 * 16 * 16 * 64 ops per wave instruction, 4 chains.
__global__ __launch_bounds__(256) void k_peak_mfma_i8(int seed, int* out) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 a = {seed, seed + 1, seed + 2, seed + 3}, b = {seed ^ 5, seed ^ 6, seed ^ 7, seed ^ 9};
    i4 c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = i4{0, 0, 0, (int)threadIdx.x};
    for (int it = 0; it < kPeakIters / 4; ++it)
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c[i], 0, 0, 0);
    int s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) s ^= c[i][0] ^ c[i][1] ^ c[i][2] ^ c[i][3];
    if (s == 0x7fffffff) out[0] = s;
}

// Device-to-device copy, 16 bytes per lane per step: read + write bytes.
__global__ __launch_bounds__(256) void k_peak_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace fic
