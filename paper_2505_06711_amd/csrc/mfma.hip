// Matrix-core dense layers for gfx950.
//
// One workgroup (4 waves) computes a 64 x 64 tile of C = A * Wt^T; each wave owns a
// 32 x 32 quarter as 2 x 2 MFMA 16x16 accumulators.  K advances in chunks of 32: the A
// chunk (FP32 in memory) is rounded to the operand type while it is written to LDS, the
// Wt chunk is copied as stored.  Instructions (operand K per instruction):
//   FP32  v_mfma_f32_16x16x4_f32    lane l supplies A[l%16][k0 + l/16]
//   BF16  v_mfma_f32_16x16x32_bf16  lane l supplies A[l%16][k0 + 8(l/16) .. +7]
//   FP8   v_mfma_f32_16x16x32_fp8   lane l supplies A[l%16][k0 + 8(l/16) .. +7]
// and likewise for B = Wt^T; the 16x16 result holds C[4(l/16) + r][l%16] in register r.
#include "mfma.hpp"

namespace reann {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

template <OpType OP> struct OpT;
template <> struct OpT<OpType::F32> { using T = float; static constexpr int LDT = 36; };
template <> struct OpT<OpType::BF16> { using T = uint16_t; static constexpr int LDT = 40; };
template <> struct OpT<OpType::FP8> { using T = uint8_t; static constexpr int LDT = 40; };

__device__ inline uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline uint8_t f2fp8(float f) {   // OCP e4m3, |f| <= 448 by construction of the scale
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(f, 0.0f, 0, false) & 0xff);
}

template <OpType OP> __device__ inline typename OpT<OP>::T to_op(float v, float inv_scale) {
    if constexpr (OP == OpType::F32) return v;
    else if constexpr (OP == OpType::BF16) return f2bf(v);
    else return f2fp8(v * inv_scale);
}

__device__ inline float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

template <OpType OP, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int64_t rows, int in, int out, const float *__restrict__ A, int lda,
                                              const typename OpT<OP>::T *__restrict__ Wt, int ldw,
                                              const float *__restrict__ bias, float *__restrict__ Z, int ldz,
                                              float *__restrict__ C, int ldc, const float *__restrict__ sA,
                                              const float *__restrict__ sW) {
    using T = typename OpT<OP>::T;
    constexpr int BM = 64, BN = 64, KC = kMfmaKC, LDT = OpT<OP>::LDT;
    __shared__ __attribute__((aligned(16))) T As[BM * LDT];
    __shared__ __attribute__((aligned(16))) T Ws[BN * LDT];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t m0 = (int64_t)blockIdx.x * BM;
    const int n0 = blockIdx.y * BN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const float inv_sa = (OP == OpType::FP8) ? 1.0f / sA[0] : 1.0f;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int lr = tid >> 2, lk = (tid & 3) * 8;   // loader: row, first of 8 k
    const int64_t ar = m0 + lr;
    const int wr = n0 + lr;
    const int li = lane & 15, lg = lane >> 4;
    for (int k0 = 0; k0 < in; k0 += KC) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = k0 + lk + q;
            const float v = (ar < rows && k < in) ? A[ar * lda + k] : 0.0f;
            As[lr * LDT + lk + q] = to_op<OP>(v, inv_sa);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) Ws[lr * LDT + lk + q] = wr < out ? Wt[(int64_t)wr * ldw + k0 + lk + q] : T(0);
        __syncthreads();
        if constexpr (OP == OpType::F32) {
#pragma unroll
            for (int s = 0; s < KC / 4; ++s) {
                float a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[(wm + i * 16 + li) * LDT + s * 4 + lg];
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = Ws[(wn + j * 16 + li) * LDT + s * 4 + lg];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        } else if constexpr (OP == OpType::BF16) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&As[(wm + i * 16 + li) * LDT + 8 * lg]));
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&Ws[(wn + j * 16 + li) * LDT + 8 * lg]));
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
            long a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const long *>(&As[(wm + i * 16 + li) * LDT + 8 * lg]);
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const long *>(&Ws[(wn + j * 16 + li) * LDT + 8 * lg]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    const float scale = (OP == OpType::FP8) ? sA[0] * sW[0] : 1.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm + i * 16 + 4 * lg + r;
                const int col = n0 + wn + j * 16 + li;
                if (row >= rows || col >= out) continue;
                float v = acc[i][j][r] * scale;
                if (EPI == EPI_BIAS_SILU) {
                    v += bias[col];
                    Z[row * ldz + col] = v;
                    v = silu_f(v);
                } else if (EPI == EPI_BIAS) {
                    v += bias[col];
                } else if (EPI == EPI_DSILU) {
                    v *= dsilu_f(Z[row * ldz + col]);
                }
                C[row * ldc + col] = v;
            }
}

void gemm_mfma(hipStream_t st, OpType op, Epi epi, int64_t rows, int in, int out, const float *A, int lda,
               const void *Wt, int ldw, const float *bias, float *Z, int ldz, float *C, int ldc, const float *sA,
               const float *sW) {
    if (rows <= 0) return;
    if (ldw % kMfmaKC != 0 || ldw < in) fail(REANN_E_DEVICE, "gemm_mfma: weight rows must be padded to 32");
    dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((out + 63) / 64));
#define G_(OPV, E)                                                                                               \
    hipLaunchKernelGGL((k_gemm<OPV, E>), grid, dim3(256), 0, st, rows, in, out, A, lda,                          \
                       (const typename OpT<OPV>::T *)Wt, ldw, bias, Z, ldz, C, ldc, sA, sW)
#define GE_(OPV)                                                     \
    switch (epi) {                                                   \
    case EPI_BIAS_SILU: G_(OPV, EPI_BIAS_SILU); break;               \
    case EPI_BIAS: G_(OPV, EPI_BIAS); break;                         \
    case EPI_DSILU: G_(OPV, EPI_DSILU); break;                       \
    default: G_(OPV, EPI_NONE); break;                               \
    }
    if (op == OpType::F32) { GE_(OpType::F32) }
    else if (op == OpType::BF16) { GE_(OpType::BF16) }
    else { GE_(OpType::FP8) }
#undef GE_
#undef G_
    LAUNCH_OK("k_gemm");
}

// ------------------------------------------------------------- FP8 scaling --

__global__ void k_amax(const float *__restrict__ A, int64_t rows, int cols, int lda, uint32_t *__restrict__ out) {
    float m = 0.0f;
    const int64_t tot = rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cols;
        const int c = (int)(t % cols);
        m = fmaxf(m, fabsf(A[r * lda + c]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    // max is order-independent, so the atomic keeps the result deterministic
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void k_scale_from_amax(const uint32_t *__restrict__ a, float *__restrict__ s) {
    const float v = __uint_as_float(*a);
    *s = v > 0.0f ? v / 448.0f : 1.0f;
}

void amax_scale(hipStream_t st, const float *A, int64_t rows, int cols, int lda, float *d_scale, uint32_t *d_tmp) {
    zero(st, d_tmp, 4);
    const int64_t tot = rows * cols;
    const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (tot + 255) / 256));
    hipLaunchKernelGGL(k_amax, dim3(nb), dim3(256), 0, st, A, rows, cols, lda, d_tmp);
    LAUNCH_OK("k_amax");
    hipLaunchKernelGGL(k_scale_from_amax, dim3(1), dim3(1), 0, st, d_tmp, d_scale);
    LAUNCH_OK("k_scale_from_amax");
}

template <OpType OP>
__global__ void k_convert(const float *__restrict__ src, int rows, int cols, int ld_src, typename OpT<OP>::T *dst,
                          int ld_dst, const float *__restrict__ scale) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * ld_dst) return;
    const int64_t r = t / ld_dst;
    const int c = (int)(t % ld_dst);
    const float inv = (OP == OpType::FP8) ? 1.0f / scale[0] : 1.0f;
    dst[t] = c < cols ? to_op<OP>(src[r * ld_src + c], inv) : typename OpT<OP>::T(0);
}

void convert_operand(hipStream_t st, OpType op, const float *src, int rows, int cols, int ld_src, void *dst,
                     int ld_dst, const float *scale) {
    const int64_t tot = (int64_t)rows * ld_dst;
    if (tot == 0) return;
    if (op == OpType::F32)
        hipLaunchKernelGGL(k_convert<OpType::F32>, dim3(grid_for(tot, 256)), dim3(256), 0, st, src, rows, cols, ld_src,
                           (float *)dst, ld_dst, scale);
    else if (op == OpType::BF16)
        hipLaunchKernelGGL(k_convert<OpType::BF16>, dim3(grid_for(tot, 256)), dim3(256), 0, st, src, rows, cols,
                           ld_src, (uint16_t *)dst, ld_dst, scale);
    else
        hipLaunchKernelGGL(k_convert<OpType::FP8>, dim3(grid_for(tot, 256)), dim3(256), 0, st, src, rows, cols,
                           ld_src, (uint8_t *)dst, ld_dst, scale);
    LAUNCH_OK("k_convert");
}

}  // namespace reann
