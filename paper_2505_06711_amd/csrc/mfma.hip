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

#include <type_traits>

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

__device__ inline uint8_t f2fp8(float f) {   // OCP e4m3; values beyond the largest finite one (448) saturate
    f = fminf(fmaxf(f, -448.0f), 448.0f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(f, 0.0f, 0, false) & 0xff);
}

template <OpType OP> __device__ inline typename OpT<OP>::T to_op(float v, float inv_scale) {
    if constexpr (OP == OpType::F32) return v;
    else if constexpr (OP == OpType::BF16) return f2bf(v);
    else return f2fp8(v * inv_scale);
}

// SiLU and its derivative in FP32 from the hardware base-2 exponential and reciprocal:
// sigma(z) = 1 / (1 + 2^(-z log2(e))), silu = z sigma, silu' = sigma (1 + z (1 - sigma)).
// For z below -126 / log2(e) the exponential overflows to +inf and sigma is 0, the limit.
__device__ inline float sigm_f(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}
__device__ inline float silu_f(float z) { return z * sigm_f(z); }
// The forward's SiLU with the exponential of the library (argument reduction in extended
// precision, so the rounding of -z log2(e) is not amplified by |z|); the activation is rounded
// once more than an exact SiLU, not several times.
__device__ inline float silu_fwd(float z) { return z * __builtin_amdgcn_rcpf(1.0f + expf(-z)); }
__device__ inline float dsilu_f(float z) {
    const float s = sigm_f(z);
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
                    v = silu_fwd(v);
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

// ------------------------------------------------------- fused atomic NNs --
//
// One workgroup takes kFuseBM rows of one element's NN through every layer; the activations
// stay in LDS between layers and only the pre-activations Z_k (needed by the adjoint) and
// the outputs reach HBM.  Each of the 4 waves owns every row of the tile and the column
// blocks j = wave + 4 jj of the layer output; its weight fragments come straight from
// global memory (every tile reads the same weights, so they stay in cache) one K chunk
// ahead of the matrix instructions.
//
// Operand order inside a K chunk: lane l (row or column l % 16, group g = l / 16) holds a
// contiguous run of k; for FP32 the run is 4 long and sub-step s of the chunk uses element s,
// so the instruction's k index g stands for k0 + 4 g + s on both operands (the contraction
// is a sum over k, so any common order of k gives the same product).

namespace {

constexpr int kFuseWaves = 4;
constexpr int kOutParts = 8;   // threads per row in the output layer (kFuseBM * kOutParts = 256)
static_assert(kFuseBM * kOutParts == 256, "output layer mapping");

template <OpType OP> struct Fuse;
template <> struct Fuse<OpType::F32> {
    using T = float;
    static constexpr int KC = 16;    // k per chunk
    static constexpr int PAD = 4;    // LDS row padding (elements): row stride = 4 banks mod 64
};
template <> struct Fuse<OpType::BF16> {
    using T = uint16_t;
    static constexpr int KC = 32;
    static constexpr int PAD = 8;
};
template <> struct Fuse<OpType::FP8> {
    using T = uint8_t;
    static constexpr int KC = 32;
    static constexpr int PAD = 16;
};

typedef float fl4 __attribute__((ext_vector_type(4)));

// Lane permutations within rows of 16 lanes (DPP; registers only, no LDS round trip).  The
// permutations used here read an active lane of the same row for every lane, so the moves
// need no old value.
template <int CTRL> __device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- lane 7 - i within each group of 8

template <int CTRL> __device__ inline float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over each group of 8 consecutive lanes (every lane gets the same value: the quad sums
// are formed in the same order everywhere and the last step adds two of them, which
// commutes exactly).
template <typename A> __device__ inline A sum8(A v) {
    if constexpr (sizeof(A) == 8) {
        v += dpp_f64<kDppXor1>(v);
        v += dpp_f64<kDppXor2>(v);
        return v + dpp_f64<kDppHalfMirror>(v);
    } else {
        v += dpp_f32<kDppXor1>(v);
        v += dpp_f32<kDppXor2>(v);
        return v + dpp_f32<kDppHalfMirror>(v);
    }
}

// Output layer of the forward (FP32 data, accumulation in A): kOutParts threads share a row,
// each takes H / kOutParts hidden units for all DOUT outputs, and the partial sums are
// combined across the row's threads; thread `part` writes outputs part, part + kOutParts, ...
// The energy NN (one output) accumulates in FP64 with FP64 weights and bias: its output is a
// sum of H terms that can cancel to a small atomic energy, so the FP32 rounding of its weights
// would be amplified by that cancellation.  The message NNs accumulate in FP32 with FP32 weights,
// like their hidden layers.  H (the hidden width) is a compile-time constant, so the loops
// unroll without branches.
template <int DOUT, typename A, int H, typename WT>
__device__ inline void out_layer(const float *hl, int ldl, const WT *wo, const WT *bo, const FusedNN &p, int64_t m0,
                                 int tid) {
    constexpr int QN = H / kOutParts;
    const int row = tid / kOutParts, part = tid % kOutParts;
    A hv[QN];
#pragma unroll
    for (int j = 0; j < QN; ++j) hv[j] = (A)hl[row * ldl + part * QN + j];
    A s[DOUT];
#pragma unroll
    for (int o = 0; o < DOUT; ++o) {
        const WT *w = wo + o * H + part * QN;
        A a = A(0);
#pragma unroll
        for (int j = 0; j < QN; ++j) a += hv[j] * (A)w[j];
        s[o] = a;
    }
#pragma unroll
    for (int o = 0; o < DOUT; ++o) s[o] = sum8(s[o]);
    const int64_t grow = m0 + row;
    if (grow < p.rows) {
#pragma unroll
        for (int o = 0; o < DOUT; ++o)
            if (o % kOutParts == part) p.C[grow * p.ldc + o] = (float)(s[o] + (A)bo[o]);
    }
}

// acc[rb][cb] = sum_k X[16 rb + i][k] Wt[16 (wave + 4 cb) + j][k] over k < kin (a multiple of
// the chunk).  Columns at or past `out` read row 0 of Wt; the caller never stores them.
template <OpType OP, int NCB, bool SPLIT>
__device__ inline void fused_layer(const typename Fuse<OP>::T *X, int ldx, const typename Fuse<OP>::T *__restrict__ Wt,
                                   int ldw, int kin, int out, int wave, int lane, f4 (&acc)[kFuseBM / 16][NCB]) {
    constexpr int RB = kFuseBM / 16, KC = Fuse<OP>::KC;
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    const typename Fuse<OP>::T *wrow[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int col = 16 * (wave + kFuseWaves * cb) + li;
        wrow[cb] = Wt + (size_t)(col < out ? col : 0) * ldw;
    }
    // weight fragments in two register sets used in turn: the set for chunk k0 + KC is
    // requested before the matrix instructions of chunk k0 are issued (the scheduling
    // barriers keep the compiler from moving the requests next to their use)
    using T = typename Fuse<OP>::T;
    using V = typename std::conditional<OP == OpType::F32, fl4,
                                        typename std::conditional<OP == OpType::BF16, u16x8, long>::type>::type;
    constexpr int RUN = OP == OpType::F32 ? 4 : 8;   // k per lane per chunk
    auto load_b = [&](V (&b)[NCB], int k0) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[cb] = *reinterpret_cast<const V *>(wrow[cb] + k0 + RUN * lg);
    };
    auto load_a = [&](V (&a)[RB], int k0) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) a[rb] = *reinterpret_cast<const V *>(X + (16 * rb + li) * ldx + k0 + RUN * lg);
    };
    // SPLIT (the forward, whose rounding reaches the energy): even chunks accumulate into acc,
    // odd chunks into acc2, summed at the end, so each FP32 accumulation chain is half as long.
    // The adjoint keeps one chain (its rounding reaches only the forces, and the registers of a
    // second chain would spill).
    f4 acc2[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc2[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    f4 (&accb)[RB][NCB] = SPLIT ? acc2 : acc;
    auto mma = [&](f4 (&c)[RB][NCB], const V (&a)[RB], const V (&b)[NCB]) {
        if constexpr (OP == OpType::F32) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        c[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][s], b[cb][s], c[rb][cb], 0, 0, 0);
        } else if constexpr (OP == OpType::BF16) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    c[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, a[rb]), __builtin_bit_cast(bf16x8, b[cb]), c[rb][cb], 0, 0, 0);
        } else {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    c[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[rb], b[cb], c[rb][cb], 0, 0, 0);
        }
    };
    // pairs of chunks per trip, so that a trip is one basic block and the requests cannot be
    // sunk into a later block next to their use; both operands of chunk k0 + KC (weights from
    // global memory, the activation tile from LDS) are requested before chunk k0 is multiplied
    V a0[RB], a1[RB], b0[NCB], b1[NCB];
    const int nck = kin / KC, klast = kin - KC;
    load_b(b0, 0);
    load_a(a0, 0);
    int k0 = 0;
    for (int pr = 0; pr + 2 <= nck; pr += 2) {
        load_b(b1, k0 + KC);
        load_a(a1, k0 + KC);
        __builtin_amdgcn_sched_barrier(0);
        mma(acc, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        const int k2 = min(k0 + 2 * KC, klast);
        load_b(b0, k2);
        load_a(a0, k2);
        __builtin_amdgcn_sched_barrier(0);
        mma(accb, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        k0 += 2 * KC;
    }
    if (nck & 1) mma(acc, a0, b0);   // a0, b0 hold the last chunk
    if constexpr (SPLIT) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] += acc2[rb][cb];
    }
}

}  // namespace

// Density features of order l of tile row r for the pairs (a, b >= a) with a in [A0, A1):
// X[r][l P + idx(a, b)] = sum over the components q of order l of w_q S[q][a] S[q][b].
// A tile row past the segment's end takes the segment's last row (its results are never
// stored), so every load is unconditional.
template <OpType OP, int L, int K, int l, int A0, int A1>
__device__ inline void density_part(const FusedNN &p, typename Fuse<OP>::T *X, int ldx, int64_t m0, int r) {
    constexpr int NLK = n_lambda(L) * K, P = K * (K + 1) / 2;
    constexpr int q0 = l * (l + 1) * (l + 2) / 6, nq = (l + 1) * (l + 2) / 2;
    const int64_t row = min(m0 + r, p.rows - 1);
    const float4 *Sg = reinterpret_cast<const float4 *>(p.S + row * NLK + q0 * K);
    float sv[nq][K], w[nq];
#pragma unroll
    for (int q = 0; q < nq; ++q) {
        w[q] = (float)p.dc.w[q0 + q];
#pragma unroll
        for (int m4 = 0; m4 < K / 4; ++m4) {
            const float4 v4 = Sg[q * (K / 4) + m4];
            sv[q][4 * m4] = v4.x; sv[q][4 * m4 + 1] = v4.y; sv[q][4 * m4 + 2] = v4.z; sv[q][4 * m4 + 3] = v4.w;
        }
    }
    typename Fuse<OP>::T *xr = X + r * ldx + l * P;
#pragma unroll
    for (int a = A0; a < A1; ++a)
#pragma unroll
        for (int b = a; b < K; ++b) {
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < nq; ++q) acc += w[q] * sv[q][a] * sv[q][b];
            const int f = a * K - a * (a - 1) / 2 + (b - a);
            xr[f] = to_op<OP>(acc, OP == OpType::FP8 ? p.xinv[l * P + f] : 1.0f);
        }
}

// Split of the pairs a <= b of K channels into a < A and a >= A with about half on each side.
constexpr int pair_split(int K) {
    int A = 0, n = 0;
    while (2 * n < K * (K + 1) / 2) n += K - A++;
    return A;
}

// Forward of one element's NN over rows [0, rows): C = out_layer(SiLU(... SiLU(rho W_0^T + b_0) ...))
// with rho the density of S.  NCB = H / 64 column blocks per wave; (L, K) fix the density.
// L = 0 is the radial message form: its features are the K orbital sums S[0] themselves.
template <OpType OP, int NCB, int L, int K>
__device__ __forceinline__ void mlp_fwd_body(const FusedNN &p, const int64_t m0) {
    using T = typename Fuse<OP>::T;
    constexpr int BM = kFuseBM, RB = BM / 16;
    constexpr int NLK = n_lambda(L) * K, P = K * (K + 1) / 2;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    // layer 0 contracts over F rounded up to the chunk size only (the weight rows are padded
    // further, with zeros, which the product does not need)
    const int F = p.F, H = p.H, Fk = (F + Fuse<OP>::KC - 1) / Fuse<OP>::KC * Fuse<OP>::KC;
    const int ldx = (Fk > H ? Fk : H) + Fuse<OP>::PAD, ldf = H + 4;
    // LDS, addressed from `smem` by offset arithmetic only (a pointer picked from an array
    // would lose its address space and turn every LDS access into a flat one): X [BM][ldx]
    // holds the layer-0 input and then, in place, every hidden layer's output; non-FP32
    // operands add an FP32 copy of the last hidden layer; W_out [dout][H].  One region for
    // the activations keeps four workgroups per CU.
    const int offf = BM * ldx * (int)sizeof(T);
    const int offw = offf + (OP == OpType::F32 ? 0 : BM * ldf * 4);
    T *X = reinterpret_cast<T *>(smem);
    float *hf = reinterpret_cast<float *>(smem + offf);
    float *wo = reinterpret_cast<float *>(smem + offw);
    double *wo64 = reinterpret_cast<double *>(smem + offw);   // the energy NN's FP64 W_out instead
    if (p.dout == 1)
        for (int e = tid; e < H; e += 256) wo64[e] = p.Wout64[e];
    else
        for (int e = tid; e < p.dout * H; e += 256) wo[e] = p.Wout[e];
    // layer-0 input: the density of this tile's orbital sums, rounded to the operand type and
    // zero padded to Fk columns.  One task per wave (lanes 0..31 take the tile's rows): the
    // orders l < L whole, and order L (the most components) split in two halves of its pairs,
    // so that no wave runs divergent code and the longest task is about half of order L.
    // The radial form (L = 0) copies the sums.
    static_assert(L <= 2, "density tasks are laid out for L <= 2");
    if constexpr (L == 0) {
        for (int it = tid; it < BM * K; it += 256) {
            const int r = it / K, f = it % K;
            const int64_t row = min(m0 + r, p.rows - 1);
            X[r * ldx + f] = to_op<OP>(p.S[row * K + f], OP == OpType::FP8 ? p.xinv[f] : 1.0f);
        }
    } else if (lane < BM) {
        constexpr int AS = pair_split(K);
        if (wave == 0) density_part<OP, L, K, 0, 0, (L == 1 ? K : K)>(p, X, ldx, m0, lane);
        if constexpr (L == 2) {
            if (wave == 1) density_part<OP, L, K, 1, 0, K>(p, X, ldx, m0, lane);
            if (wave == 2) density_part<OP, L, K, 2, 0, AS>(p, X, ldx, m0, lane);
            if (wave == 3) density_part<OP, L, K, 2, AS, K>(p, X, ldx, m0, lane);
        } else {
            if (wave == 1) density_part<OP, L, K, 1, 0, AS>(p, X, ldx, m0, lane);
            if (wave == 2) density_part<OP, L, K, 1, AS, K>(p, X, ldx, m0, lane);
        }
    }
    for (int it = tid; it < BM * (Fk - F); it += 256)
        X[(it / (Fk - F)) * ldx + F + it % (Fk - F)] = to_op<OP>(0.0f, 1.0f);
    __syncthreads();
    for (int k = 0; k < p.nh; ++k) {
        float bias[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) bias[cb] = p.b[k][16 * (wave + kFuseWaves * cb) + li];
        f4 acc[RB][NCB];
        fused_layer<OP, NCB, true>(X, ldx, reinterpret_cast<const T *>(p.W[k]), p.ldw[k], k == 0 ? Fk : H, H, wave, lane,
                             acc);
        __syncthreads();   // every wave has read this layer's input
        const bool last = k + 1 == p.nh;
        float *Zk = p.Z[k];
        // FP8: the product carries the operands' scales; the next layer's input is stored scaled
        const float zs = OP == OpType::FP8 ? p.zscale[k] : 1.0f;
        const float hin = (OP == OpType::FP8 && !last) ? p.hinv[k + 1] : 1.0f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int col = 16 * (wave + kFuseWaves * cb) + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = 16 * rb + 4 * lg + r;
                    const int64_t row = m0 + rr;
                    const float z = acc[rb][cb][r] * zs + bias[cb];
                    if (row < p.rows) Zk[row * p.ldz + col] = z;
                    const float h = silu_fwd(z);
                    X[rr * ldx + col] = to_op<OP>(h, hin);
                    if (OP != OpType::F32 && last) hf[rr * ldf + col] = h;
                }
            }
        __syncthreads();
    }
    // output layer: dout is K (message NNs) or 1 (energy NN)
    const float *hl = (OP == OpType::F32) ? reinterpret_cast<const float *>(X) : hf;
    const int ldl = (OP == OpType::F32) ? ldx : ldf;
    if (p.dout == K) out_layer<K, float, 64 * NCB, float>(hl, ldl, wo, p.bout, p, m0, tid);
    else out_layer<1, double, 64 * NCB, double>(hl, ldl, wo64, p.bout64, p, m0, tid);
}

// Output layer of the adjoint: Ga[r][q] = (sum_o G[r][o] Wout[o][q]) * SiLU'(z) for column
// q = tid % H of rows r0, r0 + 256 / H, ... (z holds those NR = kFuseBM H / 256 rows'
// pre-activations); the thread keeps its column of Wout in registers and reads each G row as
// vectors.  H is a compile-time constant.
template <OpType OP, int DOUT, int H>
__device__ inline void out_adjoint(const FusedNN &p, const float *wo, const float *gs,
                                   const float (&z)[kFuseBM * H / 256], typename Fuse<OP>::T *Ga, int ldh, int64_t m0,
                                   int tid) {
    constexpr int NR = kFuseBM * H / 256, rstep = 256 / H;
    const int q = tid % H, r0 = tid / H;
    float wq[DOUT];
#pragma unroll
    for (int o = 0; o < DOUT; ++o) wq[o] = wo[o * H + q];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int r = r0 + rstep * i;
        float s = 0.0f;
        if constexpr (DOUT % 4 == 0) {
#pragma unroll
            for (int o = 0; o < DOUT; o += 4) {
                const float4 g4 = *reinterpret_cast<const float4 *>(gs + r * DOUT + o);
                s += g4.x * wq[o] + g4.y * wq[o + 1] + g4.z * wq[o + 2] + g4.w * wq[o + 3];
            }
        } else {
#pragma unroll
            for (int o = 0; o < DOUT; ++o) s += gs[r * DOUT + o] * wq[o];
        }
        const float v = m0 + r < p.rows ? s * dsilu_f(z[i]) : 0.0f;
        Ga[r * ldh + q] = to_op<OP>(v, 1.0f);
    }
}

// Adjoint of one element's NN: C = dE/dS from G = dE/d(output), using the stored Z_k.
template <OpType OP, int NCB, int L, int K>
__device__ __forceinline__ void mlp_bwd_body(const FusedNN &p, const int64_t m0) {
    constexpr int NCBF = (L + 1) * K * (K + 1) / 2 > 128 ? 4 : 2;   // column blocks per wave, first layer
    using T = typename Fuse<OP>::T;
    constexpr int BM = kFuseBM, RB = BM / 16;
    constexpr int NLK = n_lambda(L) * K, P = K * (K + 1) / 2, NL = n_lambda(L);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    const int F = p.F, H = p.H, dout = p.dout;
    const int ldh = H + Fuse<OP>::PAD, ldr = F + 4;
    // LDS from `smem` by offset arithmetic only (see the forward kernel).  Region A holds the
    // adjoint tile, updated in place layer by layer, and finally dE/drho; region B holds W_out
    // and the G tile.
    const int offB = max(BM * ldh * (int)sizeof(T), BM * ldr * 4);
    T *Ga = reinterpret_cast<T *>(smem);
    float *Rb = reinterpret_cast<float *>(smem);          // dE/drho [BM][ldr]
    float *wo = reinterpret_cast<float *>(smem + offB);   // W_out [dout][H]
    float *gs = wo + dout * H;                             // G tile [BM][dout]
    // output layer: zbar[r][q] = (sum_o G[r][o] Wout[o][q]) * SiLU'(Z_{nh-1}[r][q]); thread tid
    // takes column q = tid % H of rows r0, r0 + 256 / H, ...
    {
        for (int e = tid; e < dout * H; e += 256) wo[e] = p.Wout[e];
        for (int e = tid; e < BM * dout; e += 256) {
            const int r = e / dout, o = e % dout;
            gs[e] = m0 + r < p.rows ? p.G[(m0 + r) * p.ldg + o] : 0.0f;
        }
        constexpr int HC = 64 * NCB, NR = BM * HC / 256, rstep = 256 / HC;   // HC = H
        const int q = tid % HC, r0 = tid / HC;
        const float *Zl = p.Z[p.nh - 1];
        float z[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) {   // rows past the end: as above (out_adjoint zeroes them)
            const int64_t row = min(m0 + r0 + rstep * i, p.rows - 1);
            z[i] = Zl[row * p.ldz + q];
        }
        __syncthreads();
        if (dout == K) out_adjoint<OP, K, HC>(p, wo, gs, z, Ga, ldh, m0, tid);
        else out_adjoint<OP, 1, HC>(p, wo, gs, z, Ga, ldh, m0, tid);
    }
    __syncthreads();
    for (int k = p.nh - 1; k >= 1; --k) {
        const float *Zk = p.Z[k - 1];
        float zp[RB][NCB][4];   // issued before the matrix loop so their latency is hidden
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // rows past the end read the last row; their adjoints are set to 0 below
                    const int64_t row = min(m0 + 16 * rb + 4 * lg + r, p.rows - 1);
                    const int col = 16 * (wave + kFuseWaves * cb) + li;
                    zp[rb][cb][r] = Zk[row * p.ldz + col];
                }
        f4 acc[RB][NCB];
        fused_layer<OP, NCB, false>(Ga, ldh, reinterpret_cast<const T *>(p.W[k]), p.ldw[k], H, H, wave, lane, acc);
        __syncthreads();   // every wave has read the tile
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int col = 16 * (wave + kFuseWaves * cb) + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = 16 * rb + 4 * lg + r;
                    const float v = m0 + rr < p.rows ? acc[rb][cb][r] * dsilu_f(zp[rb][cb][r]) : 0.0f;
                    Ga[rr * ldh + col] = to_op<OP>(v, 1.0f);
                }
            }
        __syncthreads();
    }
    // first layer: dE/drho = zbar_0 W_0 (F columns), into region A once every wave is done
    // reading the adjoint tile
    f4 acc[RB][NCBF];
    fused_layer<OP, NCBF, false>(Ga, ldh, reinterpret_cast<const T *>(p.W[0]), p.ldw[0], H, F, wave, lane, acc);
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCBF; ++cb) {
            const int col = 16 * (wave + kFuseWaves * cb) + li;
            if (col >= F) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) Rb[(16 * rb + 4 * lg + r) * ldr + col] = acc[rb][cb][r];
        }
    __syncthreads();
    // the radial form (L = 0): dE/dS = dE/dx
    if constexpr (L == 0) {
        for (int it = tid; it < BM * K; it += 256) {
            const int r = it / K, f = it % K;
            if (m0 + r < p.rows) p.C[(m0 + r) * K + f] = Rb[r * ldr + f];
        }
        return;
    }
    // density adjoint: dE/dS[lambda][a] = w_lambda sum_b M_l[a][b] S[lambda][b] for lambda of
    // order l, with M_l the symmetric matrix of dE/drho[l] (doubled on the diagonal); one
    // thread per (row, lambda), S read from global
    for (int it = tid; it < BM * NL; it += 256) {
        const int r = it / NL, lam = it % NL;
        const int64_t row = m0 + r;
        if (row >= p.rows) continue;
        const int l = lam == 0 ? 0 : (lam < 4 ? 1 : (lam < 10 ? 2 : 3));
        const float *rb = Rb + r * ldr + l * P;
        const float4 *Sg = reinterpret_cast<const float4 *>(p.S + row * NLK + lam * K);
        float sl[K];
#pragma unroll
        for (int m4 = 0; m4 < K / 4; ++m4) {
            const float4 v4 = Sg[m4];
            sl[4 * m4] = v4.x; sl[4 * m4 + 1] = v4.y; sl[4 * m4 + 2] = v4.z; sl[4 * m4 + 3] = v4.w;
        }
        const float wl = (float)p.dc.w[lam];
        // each of the K (K + 1) / 2 distinct matrix entries is read once and used for both
        // (a, b) and (b, a); every acc[a] still receives its terms in the order b = 0 .. K - 1
        float acc2[K];
#pragma unroll
        for (int a = 0; a < K; ++a) acc2[a] = 0.0f;
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = a; b < K; ++b) {
                const float m = rb[a * K - a * (a - 1) / 2 + (b - a)];
                if (a == b) {
                    acc2[a] += 2.0f * m * sl[a];
                } else {
                    acc2[a] += m * sl[b];
                    acc2[b] += m * sl[a];
                }
            }
#pragma unroll
        for (int a = 0; a < K; ++a) p.C[row * NLK + lam * K + a] = wl * acc2[a];
    }
}

// The kernels: one element's rows (blocks of kFuseBM rows), or several segments of the same NN
// shape in one launch (block b runs segment s for tile0[s] <= b < tile0[s + 1]).
template <OpType OP, int NCB, int L, int K>
__global__ __launch_bounds__(256, 4) void k_mlp_fwd(FusedNN p) {
    mlp_fwd_body<OP, NCB, L, K>(p, (int64_t)blockIdx.x * kFuseBM);
}
template <OpType OP, int NCB, int L, int K>
__global__ __launch_bounds__(256, 4) void k_mlp_bwd(FusedNN p) {
    mlp_bwd_body<OP, NCB, L, K>(p, (int64_t)blockIdx.x * kFuseBM);
}
__device__ __forceinline__ int fused_segment(const FusedMulti &pm) {
    int s = 0;
    while (s + 1 < pm.n && (int64_t)blockIdx.x >= pm.tile0[s + 1]) ++s;
    return s;
}
template <OpType OP, int NCB, int L, int K>
__global__ __launch_bounds__(256, 4) void k_mlp_fwd_multi(FusedMulti pm) {
    const int s = fused_segment(pm);
    mlp_fwd_body<OP, NCB, L, K>(pm.seg[s], ((int64_t)blockIdx.x - pm.tile0[s]) * kFuseBM);
}
template <OpType OP, int NCB, int L, int K>
__global__ __launch_bounds__(256, 4) void k_mlp_bwd_multi(FusedMulti pm) {
    const int s = fused_segment(pm);
    mlp_bwd_body<OP, NCB, L, K>(pm.seg[s], ((int64_t)blockIdx.x - pm.tile0[s]) * kFuseBM);
}

bool fused_nn_ok(OpType op, int F, int H, int nh, int dout, int NLK) {
    (void)op;
    return (H == 64 || H == 128) && F >= 1 && F <= kFuseMaxF && nh >= 1 && nh <= kFuseMaxNh &&
           dout >= 1 && dout <= kFuseMaxOut && NLK >= 1 && NLK <= kFuseMaxNLK;
}

// ---------------------------------------------------------- FP8 calibration --

__device__ inline void atomic_max_pos(float *a, float v) {   // v >= 0: order as unsigned
    atomicMax(reinterpret_cast<unsigned int *>(a), __float_as_uint(v));
}

// block y = feature f; the blocks along x split the rows
__global__ void k_density_absmax(int L, int K, int64_t rows, DensityConsts dc, const float *__restrict__ S,
                                 float *__restrict__ out) {
    const int P = K * (K + 1) / 2, NLK = dc.lstart[L + 1] * K;
    const int f = blockIdx.y, l = f / P;
    int rem = f % P, a = 0;
    while (rem >= K - a) { rem -= K - a; ++a; }
    const int b = a + rem;
    float m = 0.0f;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        const float *Sr = S + r * NLK;
        float acc = 0.0f;
        for (int q = dc.lstart[l]; q < dc.lstart[l + 1]; ++q) acc += (float)dc.w[q] * Sr[q * K + a] * Sr[q * K + b];
        m = fmaxf(m, fabsf(acc));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomic_max_pos(out + f, m);
}

__global__ void k_silu_absmax(int64_t rows, int H, int ld, const float *__restrict__ Z, float *__restrict__ out) {
    float m = 0.0f;
    const int64_t tot = rows * H;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(silu_fwd(Z[(t / H) * ld + t % H])));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomic_max_pos(out, m);
}

void density_absmax(hipStream_t st, int L, int K, int64_t rows, const DensityConsts &dc, const float *S, float *out) {
    if (rows <= 0) return;
    const int F = (L + 1) * K * (K + 1) / 2;
    const int bx = (int)std::min<int64_t>(64, (rows + 255) / 256);
    hipLaunchKernelGGL(k_density_absmax, dim3(bx, F), dim3(256), 0, st, L, K, rows, dc, S, out);
    LAUNCH_OK("k_density_absmax");
}

void silu_absmax(hipStream_t st, int64_t rows, int H, int ld, const float *Z, float *out) {
    if (rows <= 0) return;
    const int nb = (int)std::min<int64_t>(1024, (rows * H + 255) / 256);
    hipLaunchKernelGGL(k_silu_absmax, dim3(nb), dim3(256), 0, st, rows, H, ld, Z, out);
    LAUNCH_OK("k_silu_absmax");
}

static size_t fused_smem(OpType op, bool fwd, int F, int H, int dout, int NLK) {
    (void)NLK;
    const size_t eb = op_bytes(op), pad = op == OpType::F32 ? 4 : (op == OpType::BF16 ? 8 : 16);
    const size_t Fp = pad_k(F), ldh = H + pad;
    if (!fwd) {
        const size_t a = std::max<size_t>(kFuseBM * ldh * eb, (size_t)kFuseBM * (F + 4) * 4);
        return a + (size_t)(dout * H + kFuseBM * dout) * 4;
    }
    const size_t kc = op == OpType::F32 ? 16 : 32, Fk = (F + kc - 1) / kc * kc;
    const size_t ldx = std::max<size_t>(Fk, H) + pad;
    size_t b = kFuseBM * ldx * eb;
    if (op != OpType::F32) b += (size_t)kFuseBM * (H + 4) * 4;
    return b + (size_t)dout * H * (dout == 1 ? 8 : 4);   // W_out: FP64 for the energy NN
}

// Launch the fused kernel over nseg segments of the same NN shape: one segment with the
// per-element kernel, several with the segment-table kernel.
static void launch_fused(hipStream_t st, OpType op, bool fwd, const FusedNN *segs, int nseg) {
    const FusedNN &p = segs[0];
    const int NLK = p.dc.lstart[p.L + 1] * p.K;
    const int Fwant = p.L == 0 ? p.K : (p.L + 1) * p.K * (p.K + 1) / 2;   // L = 0: the radial form
    if (!fused_nn_ok(op, p.F, p.H, p.nh, p.dout, NLK) || p.F != Fwant || (p.dout != p.K && p.dout != 1))
        fail(REANN_E_DEVICE, "mlp_fused: unsupported layer shape");
    FusedMulti pm{};
    int64_t tiles = 0;
    if (nseg > 1) {
        if (nseg > kFuseMaxSeg) fail(REANN_E_DEVICE, "mlp_fused: too many segments");
        pm.n = nseg;
        for (int s = 0; s < nseg; ++s) {
            const FusedNN &q = segs[s];
            if (q.F != p.F || q.H != p.H || q.nh != p.nh || q.dout != p.dout || q.L != p.L || q.K != p.K)
                fail(REANN_E_DEVICE, "mlp_fused: segments of different shapes");
            pm.seg[s] = q;
            pm.tile0[s] = tiles;
            tiles += (q.rows + kFuseBM - 1) / kFuseBM;
        }
        pm.tile0[nseg] = tiles;
    } else {
        tiles = (p.rows + kFuseBM - 1) / kFuseBM;
    }
    if (tiles <= 0) return;
    const size_t smem = fused_smem(op, fwd, p.F, p.H, p.dout, NLK);
    const dim3 grid((unsigned)tiles);
    const bool h128 = p.H == 128;   // the kernels take H = 64 NCB as a compile-time constant
    const bool multi = nseg > 1;
#define LK_(OPV, NC, LL, KK)                                                                                  \
    if (fwd) {                                                                                              \
        if (multi) hipLaunchKernelGGL((k_mlp_fwd_multi<OPV, NC, LL, KK>), grid, dim3(256), smem, st, pm);   \
        else hipLaunchKernelGGL((k_mlp_fwd<OPV, NC, LL, KK>), grid, dim3(256), smem, st, p);                \
    } else {                                                                                                \
        if (multi) hipLaunchKernelGGL((k_mlp_bwd_multi<OPV, NC, LL, KK>), grid, dim3(256), smem, st, pm);   \
        else hipLaunchKernelGGL((k_mlp_bwd<OPV, NC, LL, KK>), grid, dim3(256), smem, st, p);                \
    }
#define NC_(OPV, LL, KK)                       \
    if (h128) { LK_(OPV, 2, LL, KK) }          \
    else { LK_(OPV, 1, LL, KK) }
#define ALL_(OPV)                                                                       \
    if (p.L == 2 && p.K == 8) { NC_(OPV, 2, 8) }                                        \
    else if (p.L == 2 && p.K == 12) { NC_(OPV, 2, 12) }                                 \
    else if (p.L == 1 && p.K == 4) { NC_(OPV, 1, 4) }                                   \
    else if (p.L == 2 && p.K == 4) { NC_(OPV, 2, 4) }                                   \
    else if (p.L == 0 && p.K == 12) { NC_(OPV, 0, 12) }                                 \
    else if (p.L == 0 && p.K == 8) { NC_(OPV, 0, 8) }                                   \
    else fail(REANN_E_UNSUPPORTED, "mlp_fused: no kernel compiled for this (L, K)");
    if (op == OpType::F32) { ALL_(OpType::F32) }
    else if (op == OpType::BF16) { ALL_(OpType::BF16) }
    else {
        if (!fwd) fail(REANN_E_DEVICE, "mlp_fused: FP8 runs the forward only (its adjoint takes BF16 operands)");
#undef LK_
#define LK_(OPV, NC, LL, KK)                                                                                  \
    if (multi) hipLaunchKernelGGL((k_mlp_fwd_multi<OPV, NC, LL, KK>), grid, dim3(256), smem, st, pm);       \
    else hipLaunchKernelGGL((k_mlp_fwd<OPV, NC, LL, KK>), grid, dim3(256), smem, st, p);
        ALL_(OpType::FP8)
#undef LK_
    }
#undef ALL_
#undef NC_
#undef LK_
    LAUNCH_OK(fwd ? "k_mlp_fwd" : "k_mlp_bwd");
}

void mlp_fused(hipStream_t st, OpType op, bool fwd, const FusedNN &p) {
    if (p.rows <= 0) return;
    launch_fused(st, op, fwd, &p, 1);
}

int mlp_fused_segments(hipStream_t st, OpType op, bool fwd, const FusedNN *segs, int nseg) {
    int launches = 0;
    for (int s0 = 0; s0 < nseg; s0 += kFuseMaxSeg) {
        const int k = std::min(kFuseMaxSeg, nseg - s0);
        launch_fused(st, op, fwd, segs + s0, k);
        ++launches;
    }
    return launches;
}

}  // namespace reann
