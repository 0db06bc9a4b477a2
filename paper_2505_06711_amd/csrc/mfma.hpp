// Matrix-core (MFMA) dense layers for the hidden layers of the atomic NNs and their
// vector-Jacobian products: C[rows x out] = A[rows x in] * Wt^T with FP32 accumulation.
// Operands are FP32, bfloat16 or OCP FP8 e4m3 (per-tensor scales); A is FP32 in memory and
// is rounded to the operand type while it is staged to LDS.
#pragma once

#include "mlp.hpp"

namespace reann {

enum class OpType { F32 = 0, BF16 = 1, FP8 = 2 };

constexpr int kMfmaKC = 32;   // K chunk staged per iteration; weight rows are padded to it

__host__ __device__ inline int pad_k(int in) { return (in + kMfmaKC - 1) / kMfmaKC * kMfmaKC; }

// Wt: operand-typed [out][ldw] (ldw = pad_k(in), zero padded).  FP8 only: sA / sW are the
// device scales of A (amax/448, see amax_scale) and of Wt; the product is rescaled by both.
void gemm_mfma(hipStream_t st, OpType op, Epi epi, int64_t rows, int in, int out, const float *A, int lda,
               const void *Wt, int ldw, const float *bias, float *Z, int ldz, float *C, int ldc, const float *sA,
               const float *sW);

// *d_scale = max(|A|) / 448 over rows x cols (row stride lda), or 1 if A is all zero.
void amax_scale(hipStream_t st, const float *A, int64_t rows, int cols, int lda, float *d_scale, uint32_t *d_tmp);

// Convert FP32 [rows][cols] (row stride ld_src) into operand type [rows][ld_dst] (zero padded);
// for FP8 the values are divided by *scale first.
void convert_operand(hipStream_t st, OpType op, const float *src, int rows, int cols, int ld_src, void *dst,
                     int ld_dst, const float *scale);

// Fused atomic NN (every layer of one element's NN in one launch, FP32 or BF16 operands).
constexpr int kFuseBM = 32;      // rows per workgroup
constexpr int kFuseMaxH = 128;   // hidden width (64 or 128)
constexpr int kFuseMaxF = 256;   // input width
constexpr int kFuseMaxNh = 4;    // hidden layers
constexpr int kFuseMaxOut = 16;  // output width
constexpr int kFuseMaxNLK = 160; // orbital sums per row (NL * K)

struct FusedNN {
    int64_t rows;                 // rows of this element's segment
    int F, H, nh, dout;           // input width, hidden width, hidden layers, output width
    int L, K;                     // angular order and radial channels of the density input
    DensityConsts dc;             // its multinomial weights and component ranges
    const float *S;               // orbital sums [rows][NL*K] (the NN input is their density)
    // forward: W[k] = layer k as [out][ldw] (gemm_mfma's forward operand)
    // adjoint: W[k] = layer k transposed, [in][ldw]
    const void *W[kFuseMaxNh];
    int ldw[kFuseMaxNh];
    const float *b[kFuseMaxNh];   // forward: hidden-layer biases
    float *Z[kFuseMaxNh];         // pre-activations [rows][ldz]: written by forward, read by adjoint
    int ldz;
    const float *Wout, *bout;     // output layer [dout][H], [dout] (FP32)
    const double *Wout64, *bout64;   // forward with dout = 1 (the energy NN): the same in FP64
    // FP8 forward only (1 / 1 / NULL otherwise): layer k's product is multiplied by zscale[k]
    // before its bias; the input of hidden layer k >= 1 is stored as h * hinv[k]; the layer-0
    // input (the density) as rho_f * xinv[f] (the calibrated per-feature scales, whose inverses
    // are folded into the layer-0 operand)
    float zscale[kFuseMaxNh];
    float hinv[kFuseMaxNh];
    const float *xinv;
    const float *G;               // adjoint: output adjoint [rows][ldg]
    int ldg;
    float *C;                     // forward: outputs [rows][ldc]; adjoint: dE/dS [rows][NL*K]
    int ldc;
};

// Segments of the same NN shape (the elements' rows of one layer, or locals and ghosts) for
// one launch of the fused kernels.  Kernel arguments stay well under 4 KiB.
constexpr int kFuseMaxSeg = 4;
struct FusedMulti {
    int n;
    int64_t tile0[kFuseMaxSeg + 1];   // first block of each segment; tile0[n] = total blocks
    FusedNN seg[kFuseMaxSeg];
};
static_assert(sizeof(FusedMulti) < 3072, "kernel arguments");

// Whether the fused kernels take these shapes (every operand type: FP8 runs the forward only,
// its adjoint takes BF16 operands).
bool fused_nn_ok(OpType op, int F, int H, int nh, int dout, int NLK);

// FP8 calibration from FP32 activations: out[f] = max over the rows of |rho_f| of the density of
// S [rows][NL*K] (f = (l, a <= b) in the feature order); out[F] must be zero on entry.
void density_absmax(hipStream_t st, int L, int K, int64_t rows, const DensityConsts &dc, const float *S, float *out);
// out[0] = max(out[0], max |SiLU(z)|) over Z [rows][ld], H columns; out must be zero initially.
void silu_absmax(hipStream_t st, int64_t rows, int H, int ld, const float *Z, float *out);
// Forward (fwd = true: density of S, hidden layers, Z stores, output layer with FP64
// accumulation) or adjoint (fwd = false: output layer, hidden layers, first layer, density
// adjoint to dE/dS) of one element's NN.
void mlp_fused(hipStream_t st, OpType op, bool fwd, const FusedNN &p);
// The same over nseg segments of one NN shape, kFuseMaxSeg to a launch; returns the launches.
int mlp_fused_segments(hipStream_t st, OpType op, bool fwd, const FusedNN *segs, int nseg);

inline size_t op_bytes(OpType op) { return op == OpType::F32 ? 4 : (op == OpType::BF16 ? 2 : 1); }

}  // namespace reann
