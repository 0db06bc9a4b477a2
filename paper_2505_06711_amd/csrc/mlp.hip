// Density contraction, dense layers of the atomic NNs and the small reductions around them.
//
// Density (Sec. 2.1, Eq. (1) with the pairwise features that give the stated
// (L+1) K (K+1)/2 count): rho[l,(a,b)] = sum_{|lambda|=l} w_lambda S[lambda][a] S[lambda][b].
// Atomic NN (Eq. (2)): hidden layers Linear + SiLU, linear output, one NN per element.
#include "mlp.hpp"

#include <type_traits>

namespace reann {

__device__ inline float d_expm(float x) { return expf(x); }
__device__ inline double d_expm(double x) { return exp(x); }

template <typename R> __device__ inline R silu(R z) { return z / (R(1) + d_expm(-z)); }
template <typename R> __device__ inline R dsilu(R z) {
    const R sg = R(1) / (R(1) + d_expm(-z));
    return sg * (R(1) + z * (R(1) - sg));
}

// ------------------------------------------------------------------ density --

// one thread per (atom i, angular order l): the K(K+1)/2 pair features of that l
template <typename R, int K>
__global__ void k_density(int64_t n, int L, DensityConsts dc, const R *__restrict__ S, R *__restrict__ rho) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * (L + 1)) return;
    const int64_t i = t / (L + 1);
    const int l = (int)(t % (L + 1));
    const int NL = dc.lstart[L + 1], P = K * (K + 1) / 2, F = (L + 1) * P;
    const int k0 = dc.lstart[l], k1 = dc.lstart[l + 1];
    const R *Si = S + i * NL * K;
    R *out = rho + i * F + l * P;
    // at most 6 Cartesian components share one l when L <= 2 (the dispatcher enforces L <= 2);
    // unused slots hold zero so every index below is static
    R v[6][K], w[6];
    const int nk = k1 - k0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        w[q] = q < nk ? R(dc.w[k0 + q]) : R(0);
#pragma unroll
        for (int m = 0; m < K; ++m) v[q][m] = q < nk ? Si[(k0 + q) * K + m] : R(0);
    }
    int f = 0;
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = a; b < K; ++b) {
            R s = R(0);
#pragma unroll
            for (int q = 0; q < 6; ++q) s += w[q] * v[q][a] * v[q][b];
            out[f++] = s;
        }
}

// one thread per (atom i, l): Sbar[lambda][a] = w_lambda sum_b coef(a,b) S[lambda][b] for
// lambda of order l, with coef the symmetric matrix of rhobar[l] (doubled on the diagonal)
template <typename R, int K>
__global__ void k_density_vjp(int64_t n, int L, DensityConsts dc, const R *__restrict__ S, const R *__restrict__ rb,
                              R *__restrict__ Sbar) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * (L + 1)) return;
    const int64_t i = t / (L + 1);
    const int l = (int)(t % (L + 1));
    const int NL = dc.lstart[L + 1], P = K * (K + 1) / 2, F = (L + 1) * P;
    const int k0 = dc.lstart[l], k1 = dc.lstart[l + 1];
    R C[K][K];
    const R *rbi = rb + i * F + l * P;
    int f = 0;
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = a; b < K; ++b) {
            const R v = rbi[f++];
            C[a][b] = a == b ? R(2) * v : v;
            C[b][a] = C[a][b];
        }
    for (int k = k0; k < k1; ++k) {
        const R *Sk = S + i * NL * K + k * K;
        R sv[K];
#pragma unroll
        for (int m = 0; m < K; ++m) sv[m] = Sk[m];
        R *out = Sbar + i * NL * K + k * K;
        const R w = R(dc.w[k]);
#pragma unroll
        for (int a = 0; a < K; ++a) {
            R s = R(0);
#pragma unroll
            for (int b = 0; b < K; ++b) s += C[a][b] * sv[b];
            out[a] = w * s;
        }
    }
}

// The literal reading of Eq. (1): only the squares, rho[l][a] = sum_{|lambda|=l} w_lambda
// S[lambda][a]^2 (F = (L+1) K); one thread per feature.
template <typename R>
__global__ void k_density_sq(int64_t n, int L, int K, DensityConsts dc, const R *__restrict__ S, R *__restrict__ rho) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int F = (L + 1) * K, NL = dc.lstart[L + 1];
    if (t >= n * F) return;
    const int64_t i = t / F;
    const int l = (int)(t % F) / K, a = (int)(t % K);
    R s = R(0);
    for (int k = dc.lstart[l]; k < dc.lstart[l + 1]; ++k) {
        const R v = S[(i * NL + k) * K + a];
        s += R(dc.w[k]) * v * v;
    }
    rho[t] = s;
}

// its adjoint: Sbar[lambda][a] = 2 w_lambda S[lambda][a] rhobar[l(lambda)][a]; one thread per value
template <typename R>
__global__ void k_density_sq_vjp(int64_t n, int L, int K, DensityConsts dc, const R *__restrict__ S,
                                 const R *__restrict__ rb, R *__restrict__ Sbar) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int NL = dc.lstart[L + 1];
    if (t >= n * NL * K) return;
    const int64_t i = t / (NL * K);
    const int k = (int)(t % (NL * K)) / K, a = (int)(t % K);
    int l = 0;
    while (dc.lstart[l + 1] <= k) ++l;
    Sbar[t] = R(2) * R(dc.w[k]) * S[t] * rb[i * (L + 1) * K + l * K + a];
}

void density_sq(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S,
                void *rho) {
    const int64_t tot = n * (L + 1) * K;
    if (tot == 0) return;
    if (fp64) hipLaunchKernelGGL(k_density_sq<double>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, L, K, dc, (const double *)S, (double *)rho);
    else hipLaunchKernelGGL(k_density_sq<float>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, L, K, dc, (const float *)S, (float *)rho);
    LAUNCH_OK("k_density_sq");
}

void density_sq_vjp(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S,
                    const void *rhobar, void *Sbar) {
    const int64_t tot = n * dc.lstart[L + 1] * K;
    if (tot == 0) return;
    if (fp64) hipLaunchKernelGGL(k_density_sq_vjp<double>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, L, K, dc, (const double *)S, (const double *)rhobar, (double *)Sbar);
    else hipLaunchKernelGGL(k_density_sq_vjp<float>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, L, K, dc, (const float *)S, (const float *)rhobar, (float *)Sbar);
    LAUNCH_OK("k_density_sq_vjp");
}

#define REANN_K_DISPATCH(K, CALL)                                                      \
    do {                                                                               \
        if ((K) == 8) { CALL(8); }                                                     \
        else if ((K) == 12) { CALL(12); }                                              \
        else if ((K) == 4) { CALL(4); }                                                \
        else fail(REANN_E_UNSUPPORTED, "no density kernel compiled for this K");       \
    } while (0)

void density(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S, void *rho) {
    const int64_t tot = n * (L + 1);
    if (tot == 0) return;
    if (L > 2) fail(REANN_E_UNSUPPORTED, "density kernel supports L <= 2");
#define DEN(KK)                                                                                                   \
    if (fp64) hipLaunchKernelGGL((k_density<double, KK>), dim3(grid_for(tot, 128)), dim3(128), 0, st, n, L, dc,  \
                                 (const double *)S, (double *)rho);                                              \
    else hipLaunchKernelGGL((k_density<float, KK>), dim3(grid_for(tot, 128)), dim3(128), 0, st, n, L, dc,        \
                            (const float *)S, (float *)rho);
    REANN_K_DISPATCH(K, DEN);
#undef DEN
    LAUNCH_OK("k_density");
}

void density_vjp(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S,
                 const void *rhobar, void *Sbar) {
    const int64_t tot = n * (L + 1);
    if (tot == 0) return;
    if (L > 2) fail(REANN_E_UNSUPPORTED, "density kernel supports L <= 2");
#define DVJ(KK)                                                                                                     \
    if (fp64) hipLaunchKernelGGL((k_density_vjp<double, KK>), dim3(grid_for(tot, 128)), dim3(128), 0, st, n, L, dc, \
                                 (const double *)S, (const double *)rhobar, (double *)Sbar);                        \
    else hipLaunchKernelGGL((k_density_vjp<float, KK>), dim3(grid_for(tot, 128)), dim3(128), 0, st, n, L, dc,       \
                            (const float *)S, (const float *)rhobar, (float *)Sbar);
    REANN_K_DISPATCH(K, DVJ);
#undef DVJ
    LAUNCH_OK("k_density_vjp");
}

// -------------------------------------------------------------- dense layer --

constexpr int TM = 64, TN = 64, TK = 16;

template <typename R, int EPI, bool TRANS>
__global__ __launch_bounds__(256) void k_dense(int64_t rows, int in, int out, const R *__restrict__ A, int lda,
                                               const R *__restrict__ W, const R *__restrict__ bias, R *__restrict__ Z,
                                               int ldz, R *__restrict__ C, int ldc) {
    __shared__ R As[TK][TM + 1];
    __shared__ R Ws[TK][TN + 1];
    // output layers (EPI_BIAS) accumulate in FP64: their few outputs per row are sums of
    // large terms with cancellation, and the cost is negligible
    using Acc = typename std::conditional<EPI == EPI_BIAS, double, R>::type;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t r0 = (int64_t)blockIdx.x * TM;
    const int o0 = blockIdx.y * TN;
    Acc acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = Acc(0);
    for (int k0 = 0; k0 < in; k0 += TK) {
        for (int e = threadIdx.x; e < TM * TK; e += 256) {
            const int rr = e / TK, kk = e % TK;
            const int64_t r = r0 + rr;
            const int k = k0 + kk;
            As[kk][rr] = (r < rows && k < in) ? A[r * lda + k] : R(0);
        }
        for (int e = threadIdx.x; e < TN * TK; e += 256) {
            int oo, kk;
            if (TRANS) { oo = e / TK; kk = e % TK; }
            else { kk = e / TN; oo = e % TN; }
            const int o = o0 + oo, k = k0 + kk;
            R v = R(0);
            if (o < out && k < in) v = TRANS ? W[(int64_t)o * in + k] : W[(int64_t)k * out + o];
            Ws[kk][oo] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            R a[4], w[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) a[p] = As[kk][ty + 16 * p];
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] = Ws[kk][tx + 16 * q];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] += Acc(a[p]) * Acc(w[q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int64_t r = r0 + ty + 16 * p;
        if (r >= rows) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = o0 + tx + 16 * q;
            if (o >= out) continue;
            R v = R(acc[p][q]);
            if (EPI == EPI_BIAS_SILU) {
                v += bias[o];
                Z[r * ldz + o] = v;
                v = silu(v);
            } else if (EPI == EPI_BIAS) {
                v = R(acc[p][q] + Acc(bias[o]));
            } else if (EPI == EPI_DSILU) {
                v *= dsilu(Z[r * ldz + o]);
            }
            C[r * ldc + o] = v;
        }
    }
}

template <typename R>
static void dense_t(hipStream_t st, Epi epi, bool trans, int64_t rows, int in, int out, const R *A, int lda, const R *W,
                    const R *b, R *Z, int ldz, R *C, int ldc) {
    if (rows <= 0) return;
    dim3 grid((unsigned)((rows + TM - 1) / TM), (unsigned)((out + TN - 1) / TN));
#define L_(E, T) hipLaunchKernelGGL((k_dense<R, E, T>), grid, dim3(256), 0, st, rows, in, out, A, lda, W, b, Z, ldz, C, ldc)
    if (trans) {
        switch (epi) {
        case EPI_BIAS_SILU: L_(EPI_BIAS_SILU, true); break;
        case EPI_BIAS: L_(EPI_BIAS, true); break;
        case EPI_DSILU: L_(EPI_DSILU, true); break;
        default: L_(EPI_NONE, true); break;
        }
    } else {
        switch (epi) {
        case EPI_BIAS_SILU: L_(EPI_BIAS_SILU, false); break;
        case EPI_BIAS: L_(EPI_BIAS, false); break;
        case EPI_DSILU: L_(EPI_DSILU, false); break;
        default: L_(EPI_NONE, false); break;
        }
    }
#undef L_
    LAUNCH_OK("k_dense");
}

void dense(hipStream_t st, bool fp64, Epi epi, bool trans_w, int64_t rows, int in, int out, const void *A, int lda,
           const void *W, const void *b, void *Z, int ldz, void *C, int ldc) {
    if (fp64)
        dense_t<double>(st, epi, trans_w, rows, in, out, (const double *)A, lda, (const double *)W, (const double *)b,
                        (double *)Z, ldz, (double *)C, ldc);
    else
        dense_t<float>(st, epi, trans_w, rows, in, out, (const float *)A, lda, (const float *)W, (const float *)b,
                       (float *)Z, ldz, (float *)C, ldc);
}

// ------------------------------------------------------------- reductions --

constexpr int kRedBlock = 256;

template <typename R>
__global__ void k_energy(int64_t n, double scale, const R *__restrict__ y, const int32_t *__restrict__ perm,
                         const double *__restrict__ w, double *__restrict__ Eat, double *__restrict__ part) {
    __shared__ double sm[kRedBlock];
    const int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
    double e = 0.0, we = 0.0;
    if (i < n) {
        e = scale * (double)y[i];
        if (Eat) Eat[perm[i]] = e;
        we = w ? w[perm[i]] * e : e;
    }
    sm[threadIdx.x] = we;
    __syncthreads();
    for (int h = kRedBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// The same for a small system in one block, which also forms the total: thread t takes atoms
// t, t + 256, ... in order, then a tree over the threads.
template <typename R>
__global__ __launch_bounds__(kRedBlock) void k_energy_total(int64_t n, double scale, const R *__restrict__ y,
                                                            const int32_t *__restrict__ perm, const double *__restrict__ w,
                                                            double *__restrict__ Eat, double *__restrict__ total) {
    __shared__ double sm[kRedBlock];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kRedBlock) {
        const double e = scale * (double)y[i];
        if (Eat) Eat[perm[i]] = e;
        acc += w ? w[perm[i]] * e : e;
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kRedBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = sm[0];
}

void energy_total(hipStream_t st, bool fp64, int64_t n, double scale, const void *y, const int32_t *perm,
                  const double *w_user, double *Eat_user, double *partials, double *total) {
    if (n <= kEnergyOneBlock) {
        if (fp64) hipLaunchKernelGGL(k_energy_total<double>, dim3(1), dim3(kRedBlock), 0, st, n, scale, (const double *)y, perm, w_user, Eat_user, total);
        else hipLaunchKernelGGL(k_energy_total<float>, dim3(1), dim3(kRedBlock), 0, st, n, scale, (const float *)y, perm, w_user, Eat_user, total);
        LAUNCH_OK("k_energy_total");
        return;
    }
    const int nb = energy_finalize(st, fp64, n, scale, y, perm, w_user, Eat_user, partials);
    sum_rows(st, partials, nb, 1, total, false);
}

int energy_finalize(hipStream_t st, bool fp64, int64_t n, double scale, const void *y, const int32_t *perm,
                    const double *w_user, double *Eat_user, double *partials) {
    const int nb = grid_for(n, kRedBlock);
    if (fp64) hipLaunchKernelGGL(k_energy<double>, dim3(nb), dim3(kRedBlock), 0, st, n, scale, (const double *)y, perm, w_user, Eat_user, partials);
    else hipLaunchKernelGGL(k_energy<float>, dim3(nb), dim3(kRedBlock), 0, st, n, scale, (const float *)y, perm, w_user, Eat_user, partials);
    LAUNCH_OK("k_energy");
    return nb;
}

__global__ void k_sum_rows(const double *__restrict__ part, int nb, int width, double *__restrict__ out, int acc) {
    // block q sums column q over the rows in a fixed order (strided per thread, then a tree)
    // eight independent running sums per thread keep eight loads in flight
    __shared__ double sm[256];
    const int q = blockIdx.x;
    double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int r = threadIdx.x;
    for (; r + 7 * 256 < nb; r += 8 * 256)
#pragma unroll
        for (int u = 0; u < 8; ++u) s8[u] += part[(int64_t)(r + u * 256) * width + q];
    for (; r < nb; r += 256) s8[0] += part[(int64_t)r * width + q];
    const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = acc ? out[q] + sm[0] : sm[0];
}

void sum_rows(hipStream_t st, const double *partials, int nb, int width, double *out, bool accumulate) {
    hipLaunchKernelGGL(k_sum_rows, dim3(width), dim3(256), 0, st, partials, nb, width, out, accumulate ? 1 : 0);
    LAUNCH_OK("k_sum_rows");
}

// ------------------------------------------------------------ output layers --
// The last layer of an atomic NN has few outputs (K messages or one energy), too narrow for a
// 64-wide tile.  64 rows per block: the activations are staged in LDS, W [out][in] too, and
// every output accumulates in FP64 (these are sums of large terms with cancellation).
constexpr int kOutRows = 64, kOutMaxIn = 128, kOutMaxOut = 16;

template <typename WT>
__global__ __launch_bounds__(256) void k_out_fwd(int64_t rows, int in, int out, const float *__restrict__ A, int lda,
                                                 const WT *__restrict__ W, const WT *__restrict__ b,
                                                 float *__restrict__ C, int ldc) {
    __shared__ float sA[kOutRows][kOutMaxIn + 1];
    __shared__ WT sW[kOutMaxOut][kOutMaxIn];
    const int64_t r0 = (int64_t)blockIdx.x * kOutRows;
    for (int e = threadIdx.x; e < kOutRows * in; e += 256) {
        const int rr = e / in, k = e % in;
        sA[rr][k] = r0 + rr < rows ? A[(r0 + rr) * lda + k] : 0.0f;
    }
    for (int e = threadIdx.x; e < out * in; e += 256) sW[e / in][e % in] = W[e];
    __syncthreads();
    const int rr = threadIdx.x >> 2, q0 = threadIdx.x & 3;
    const int64_t r = r0 + rr;
    if (r >= rows) return;
    for (int o = q0; o < out; o += 4) {
        double s = 0.0;
        for (int k = 0; k < in; ++k) s += (double)sA[rr][k] * (double)sW[o][k];
        C[r * ldc + o] = (float)(s + (double)b[o]);
    }
}

// The energy NN's output layer on the per-layer path: one output per row, FP64 weights and
// bias, FP64 accumulation in order k = 0 .. in - 1 (one thread per row; any width up to 1024).
constexpr int kOutEnMaxIn = 1024;
__global__ __launch_bounds__(256) void k_out_energy(int64_t rows, int in, const float *__restrict__ A, int lda,
                                                    const double *__restrict__ W, const double *__restrict__ b,
                                                    float *__restrict__ C, int ldc) {
    __shared__ double sW[kOutEnMaxIn];
    for (int k = threadIdx.x; k < in; k += 256) sW[k] = W[k];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    double s = 0.0;
    for (int k = 0; k < in; ++k) s += (double)A[r * lda + k] * sW[k];
    C[r * ldc] = (float)(s + b[0]);
}

// zbar[r][q] = (sum_o ybar[r][o] W[o][q]) * SiLU'(Z[r][q])
__global__ void k_out_vjp(int64_t rows, int out, int in, const float *__restrict__ G, int ldg,
                          const float *__restrict__ W, const float *__restrict__ Z, int ldz, float *__restrict__ C,
                          int ldc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * in) return;
    const int64_t r = t / in;
    const int q = (int)(t % in);
    float s = 0.0f;
    for (int o = 0; o < out; ++o) s += G[r * ldg + o] * W[(int64_t)o * in + q];
    C[r * ldc + q] = s * dsilu(Z[r * ldz + q]);
}

void out_layer_fwd(hipStream_t st, int64_t rows, int in, int out, const float *A, int lda, const float *W,
                   const float *b, float *C, int ldc) {
    if (rows <= 0) return;
    if (in > kOutMaxIn || out > kOutMaxOut) {   // wide layers: the tiled kernel (also FP64-accumulated)
        dense(st, false, EPI_BIAS, true, rows, in, out, A, lda, W, b, nullptr, 0, C, ldc);
        return;
    }
    hipLaunchKernelGGL(k_out_fwd<float>, dim3(grid_for(rows, kOutRows)), dim3(256), 0, st, rows, in, out, A, lda, W, b,
                       C, ldc);
    LAUNCH_OK("k_out_fwd");
}

void out_layer_energy(hipStream_t st, int64_t rows, int in, const float *A, int lda, const double *W, const double *b,
                      float *C, int ldc) {
    if (rows <= 0) return;
    if (in > kOutEnMaxIn) fail(REANN_E_UNSUPPORTED, "energy NN output layer wider than 1024");
    hipLaunchKernelGGL(k_out_energy, dim3(grid_for(rows, 256)), dim3(256), 0, st, rows, in, A, lda, W, b, C, ldc);
    LAUNCH_OK("k_out_energy");
}

void out_layer_vjp(hipStream_t st, int64_t rows, int out, int in, const float *G, int ldg, const float *W,
                   const float *Z, int ldz, float *C, int ldc) {
    if (rows <= 0) return;
    const int64_t tot = rows * in;
    hipLaunchKernelGGL(k_out_vjp, dim3(grid_for(tot, 256)), dim3(256), 0, st, rows, out, in, G, ldg, W, Z, ldz, C, ldc);
    LAUNCH_OK("k_out_vjp");
}

// The backward's start: the energy adjoint of every atom, and (nz > 0) zeros in z[0, nz).
template <typename R>
__global__ void k_seed(int64_t n, double scale, const double *__restrict__ g, const int32_t *__restrict__ perm,
                       const double *__restrict__ w, R *__restrict__ ybar, int64_t nz, R *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ybar[i] = R(scale * (g ? *g : 1.0) * (w ? w[perm[i]] : 1.0));
    if (i < nz) z[i] = R(0);
}

void fill_energy_seed(hipStream_t st, bool fp64, int64_t n, double scale, const double *g, const int32_t *perm,
                      const double *w_user, void *ybar, int64_t nzero, void *zero_out) {
    const int64_t nt = std::max<int64_t>(n, nzero);
    if (fp64)
        hipLaunchKernelGGL(k_seed<double>, dim3(grid_for(nt, 256)), dim3(256), 0, st, n, scale, g, perm, w_user,
                           (double *)ybar, nzero, (double *)zero_out);
    else
        hipLaunchKernelGGL(k_seed<float>, dim3(grid_for(nt, 256)), dim3(256), 0, st, n, scale, g, perm, w_user,
                           (float *)ybar, nzero, (float *)zero_out);
    LAUNCH_OK("k_seed");
}

// Blocks [0, 9): virial component q = the sum over the nw rows of Wpart[.][q] (in the order of
// sum_rows), times g, to Wout (when asked for); the other blocks: forces in caller order, times g.
__device__ inline double virial_column(const double *__restrict__ part, int nw, int q) {
    __shared__ double sm[256];
    double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int r = threadIdx.x;
    for (; r + 7 * 256 < nw; r += 8 * 256)
#pragma unroll
        for (int u = 0; u < 8; ++u) s8[u] += part[(int64_t)(r + u * 256) * 9 + q];
    for (; r < nw; r += 256) s8[0] += part[(int64_t)r * 9 + q];
    sm[threadIdx.x] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    return sm[0];
}

template <typename R>
__global__ __launch_bounds__(256) void k_forces_out(int64_t n, const R *__restrict__ F, const int32_t *__restrict__ perm,
                                                    const double *__restrict__ g, double *__restrict__ out,
                                                    const double *__restrict__ Wpart, int nw, double *__restrict__ Wout) {
    const double gs = g ? *g : 1.0;
    if (blockIdx.x < 9) {
        if (!Wout) return;   // uniform over the block
        const double w = virial_column(Wpart, nw, (int)blockIdx.x);
        if (threadIdx.x == 0) Wout[blockIdx.x] = gs * w;
        return;
    }
    const int64_t t = (int64_t)(blockIdx.x - 9) * blockDim.x + threadIdx.x;
    if (t < n * 3) {
        const int64_t i = t / 3, a = t % 3;
        out[(int64_t)perm[i] * 3 + a] = gs * (double)F[t];
    }
}

void forces_out(hipStream_t st, bool fp64, int64_t n, const void *F, const int32_t *perm, const double *g,
                double *forces_user, const double *Wpart, int nw, double *virial_out) {
    const unsigned nb = 9u + (unsigned)grid_for(n * 3, 256);
    if (fp64) hipLaunchKernelGGL(k_forces_out<double>, dim3(nb), dim3(256), 0, st, n, (const double *)F, perm, g, forces_user, Wpart, nw, virial_out);
    else hipLaunchKernelGGL(k_forces_out<float>, dim3(nb), dim3(256), 0, st, n, (const float *)F, perm, g, forces_user, Wpart, nw, virial_out);
    LAUNCH_OK("k_forces_out");
}

__global__ void k_zero(uint32_t *__restrict__ p, int64_t nwords) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nwords) p[t] = 0u;
}

// A fill kernel rather than hipMemsetAsync, so the step can be captured in a HIP graph.
void zero(hipStream_t st, void *p, size_t bytes) {
    const int64_t nw = (int64_t)((bytes + 3) / 4);
    if (nw == 0) return;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(nw, 256)), dim3(256), 0, st, (uint32_t *)p, nw);
    LAUNCH_OK("k_zero");
}

// dst[t] += src[t] (and copy: dst[t] = src[t]) for t < count, in the working type; kernels, so
// that the step can be captured in a HIP graph.
template <typename R, bool ADD>
__global__ void k_axpy1(int64_t count, R *__restrict__ dst, const R *__restrict__ src) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = ADD ? dst[t] + src[t] : src[t];
}

void add_into(hipStream_t st, bool fp64, int64_t count, void *dst, const void *src) {
    if (count <= 0) return;
    if (fp64) hipLaunchKernelGGL((k_axpy1<double, true>), dim3(grid_for(count, 256)), dim3(256), 0, st, count, (double *)dst, (const double *)src);
    else hipLaunchKernelGGL((k_axpy1<float, true>), dim3(grid_for(count, 256)), dim3(256), 0, st, count, (float *)dst, (const float *)src);
    LAUNCH_OK("k_axpy1");
}

void copy_into(hipStream_t st, bool fp64, int64_t count, void *dst, const void *src) {
    if (count <= 0) return;
    if (fp64) hipLaunchKernelGGL((k_axpy1<double, false>), dim3(grid_for(count, 256)), dim3(256), 0, st, count, (double *)dst, (const double *)src);
    else hipLaunchKernelGGL((k_axpy1<float, false>), dim3(grid_for(count, 256)), dim3(256), 0, st, count, (float *)dst, (const float *)src);
    LAUNCH_OK("k_axpy1");
}

}  // namespace reann
