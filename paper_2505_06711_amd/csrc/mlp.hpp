// Atomic neural networks (Sec. 2.1, Eq. (2) and the energy readout) and the density
// contraction of Eq. (1) that feeds them, with their vector-Jacobian products.
#pragma once

#include "common.hpp"

namespace reann {

struct DensityConsts {
    double w[35];    // multinomial weight l!/(lx! ly! lz!) per Cartesian component
    int lstart[6];   // first component of each l (lstart[L+1] = NL)
};

// rho[i][f], f = (l, a, b >= a), from S[i][NL][K]; rows [0, n).
void density(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S, void *rho);
// Sbar[i][lambda][a] from rhobar[i][F] and S (overwrites Sbar).
// The literal reading of Eq. (1) (only the squares, rho[i][l K + a], F = (L+1) K) and its adjoint.
void density_sq(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S, void *rho);
void density_sq_vjp(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S,
                    const void *rhobar, void *Sbar);
void density_vjp(hipStream_t st, bool fp64, int L, int K, int64_t n, const DensityConsts &dc, const void *S,
                 const void *rhobar, void *Sbar);

enum Epi { EPI_BIAS_SILU = 0, EPI_BIAS = 1, EPI_DSILU = 2, EPI_NONE = 3 };

// Dense layer over `rows` rows (row-major, leading dims lda / ldc):
//   trans_w = true : C = A W^T (+ epilogue), W [out][in]   (forward)
//   trans_w = false: C = A W   (+ epilogue), W [in][out]   (vector-Jacobian product)
// EPI_BIAS_SILU: Z = acc + b (stored to Z), C = SiLU(Z);  EPI_BIAS: C = acc + b;
// EPI_DSILU: C = acc * SiLU'(Z) with Z read;  EPI_NONE: C = acc.
void dense(hipStream_t st, bool fp64, Epi epi, bool trans_w, int64_t rows, int in, int out, const void *A, int lda,
           const void *W, const void *b, void *Z, int ldz, void *C, int ldc);

// Output layer of an atomic NN (FP32 data, FP64 accumulation): C = A W^T + b, W [out][in].
void out_layer_fwd(hipStream_t st, int64_t rows, int in, int out, const float *A, int lda, const float *W,
                   const float *b, float *C, int ldc);
// The energy NN's output layer (one output): FP64 weights [in] and bias, FP64 accumulation.
void out_layer_energy(hipStream_t st, int64_t rows, int in, const float *A, int lda, const double *W, const double *b,
                      float *C, int ldc);
// Its adjoint into the last hidden layer: C[r][q] = (sum_o G[r][o] W[o][q]) * SiLU'(Z[r][q]).
void out_layer_vjp(hipStream_t st, int64_t rows, int out, int in, const float *G, int ldg, const float *W,
                   const float *Z, int ldz, float *C, int ldc);

// Eat[perm[i]] = scale * y[i] (FP64), and per-block partial sums of w[perm[i]] Eat[perm[i]] in
// local order (w_user: caller-order weights, NULL = 1).
int energy_finalize(hipStream_t st, bool fp64, int64_t n, double scale, const void *y, const int32_t *perm,
                    const double *w_user, double *Eat_user, double *partials);
// total[0] = sum of w[perm[i]] Eat[perm[i]], with Eat written as above: a system of at most
// kEnergyOneBlock atoms in one launch (one block, fixed order), a larger one by energy_finalize
// and sum_rows (partials: grid_for(n, 256) doubles)
constexpr int64_t kEnergyOneBlock = 8192;
void energy_total(hipStream_t st, bool fp64, int64_t n, double scale, const void *y, const int32_t *perm,
                  const double *w_user, double *Eat_user, double *partials, double *total);
// out[0] = sum of partials[0..nb) (single block, fixed order); if accumulate, out[q] += ...
void sum_rows(hipStream_t st, const double *partials, int nb, int width, double *out, bool accumulate);
// ybar[i] = scale * g * w[perm[i]]  (g = device scalar or NULL = 1; w_user = caller-order weights
// or NULL = 1), and zero_out[0, nzero) = 0 in the same launch (working type)
void fill_energy_seed(hipStream_t st, bool fp64, int64_t n, double scale, const double *g, const int32_t *perm,
                      const double *w_user, void *ybar, int64_t nzero = 0, void *zero_out = nullptr);
// forces_user[perm[i]][a] = gscale * F[i][a]; virial_out[q] = gscale * sum_r Wpart[r][q] over the
// nw rows of partials (virial_out NULL: not formed); one launch
void forces_out(hipStream_t st, bool fp64, int64_t n, const void *F, const int32_t *perm, const double *g,
                double *forces_user, const double *Wpart, int nw, double *virial_out);
void zero(hipStream_t st, void *p, size_t bytes);
// dst += src, and dst = src, over `count` elements of the working type (FP64 or FP32)
void add_into(hipStream_t st, bool fp64, int64_t count, void *dst, const void *src);
void copy_into(hipStream_t st, bool fp64, int64_t count, void *dst, const void *src);

}  // namespace reann
