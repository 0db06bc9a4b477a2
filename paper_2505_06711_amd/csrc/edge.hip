// Edge passes of one message-passing layer and the per-layer ghost exchange.
//
// Forward (Sec. 2.1, Eq. (1) inner sum): for every local atom i,
//   S_i[lambda][m] = sum_{j in N(i), r_ij < r_c} c_j[m] A_lambda(d_ij) R_m(r_ij) f_c(r_ij),
// with d_ij = x_j - x_i formed in FP64 from FP64 positions, then rounded to the working type.
//
// Backward (Sec. 2.2, Eqs. (3)-(5)): given Sbar_i = dE/dS_i, each directed edge i->j has
//   g_ij = d/dd [ f_c sum_lambda A_lambda(d) sum_m Sbar_i[lambda][m] c_j[m] R_m(r) ],
// contributing +g_ij to F_i, -g_ij to F_j, -d (x) g_ij to the virial and
//   f_c R_m sum_lambda Sbar_i[lambda][m] A_lambda(d)  to  cbar_j[m] = dE/dc_j[m].
// No atomics: every ext row k gathers what lands on k -- as centre (its own edges) and
// as neighbour (the edges j->k of its local neighbours j, whose Sbar it reads).  Each
// edge is therefore evaluated at both ends; results are deterministic.
#include "edge.hpp"

namespace reann {

template <int L> struct LamTab {
    static constexpr int N = n_lambda(L);
    int lx[N], ly[N], lz[N];
    constexpr LamTab() : lx(), ly(), lz() {
        int k = 0;
        for (int l = 0; l <= L; ++l)
            for (int a = l; a >= 0; --a)
                for (int b = l - a; b >= 0; --b) {
                    lx[k] = a; ly[k] = b; lz[k] = l - a - b;
                    ++k;
                }
    }
};

__device__ inline float d_exp(float x) { return expf(x); }
__device__ inline double d_exp(double x) { return exp(x); }
__device__ inline float d_cospi(float x) { return cospif(x); }
__device__ inline double d_cospi(double x) { return cospi(x); }
__device__ inline float d_sinpi(float x) { return sinpif(x); }
__device__ inline double d_sinpi(double x) { return sinpi(x); }
__device__ inline float d_sqrt(float x) { return sqrtf(x); }
__device__ inline double d_sqrt(double x) { return sqrt(x); }

// A_lambda(u) with u = s d, and optionally dA_lambda/dd (= s * dA/du).
template <int L, typename R, bool GRAD>
__device__ inline void angular(R ux, R uy, R uz, R s, R *A, R (*dA)[3]) {
    constexpr LamTab<L> T{};
    constexpr int N = LamTab<L>::N;
    R px[L + 1], py[L + 1], pz[L + 1];
    px[0] = py[0] = pz[0] = R(1);
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        px[k] = px[k - 1] * ux;
        py[k] = py[k - 1] * uy;
        pz[k] = pz[k - 1] * uz;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int lx = T.lx[k], ly = T.ly[k], lz = T.lz[k];
        A[k] = px[lx] * py[ly] * pz[lz];
        if constexpr (GRAD) {
            dA[k][0] = lx ? s * R(lx) * px[lx > 0 ? lx - 1 : 0] * py[ly] * pz[lz] : R(0);
            dA[k][1] = ly ? s * R(ly) * px[lx] * py[ly > 0 ? ly - 1 : 0] * pz[lz] : R(0);
            dA[k][2] = lz ? s * R(lz) * px[lx] * py[ly] * pz[lz > 0 ? lz - 1 : 0] : R(0);
        }
    }
}

template <int L, int K, typename R>
__global__ __launch_bounds__(256) void k_edge_fwd(EdgeArgs a, EdgeConsts ec, const R *__restrict__ c,
                                                  R *__restrict__ S) {
    constexpr int NL = n_lambda(L);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    R acc[NL][K];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int m = 0; m < K; ++m) acc[l][m] = R(0);
    const double xi = a.px[i], yi = a.py[i], zi = a.pz[i];
    const R inv_rc = R(1.0 / ec.r_c);
    const R s = R(ec.ang_scale);
    for (int64_t k = a.row[i]; k < a.row[i + 1]; ++k) {
        const int64_t j = a.col[k];
        const double dx = a.px[j] - xi, dy = a.py[j] - yi, dz = a.pz[j] - zi;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 >= ec.rc2) continue;
        const R r = d_sqrt(R(d2));
        const R u = R(0.5) * d_cospi(r * inv_rc) + R(0.5);
        const R fc = u * u;
        R A[NL];
        angular<L, R, false>(R(ec.ang_scale * dx), R(ec.ang_scale * dy), R(ec.ang_scale * dz), s, A, nullptr);
        const R *cj = c + j * K;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const R xm = r - R(ec.centres[m]);
            const R w = cj[m] * d_exp(-R(ec.alphas[m]) * xm * xm) * fc;
#pragma unroll
            for (int l = 0; l < NL; ++l) acc[l][m] += w * A[l];
        }
    }
    R *out = S + i * NL * K;
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int m = 0; m < K; ++m) out[l * K + m] = acc[l][m];
}

constexpr int kBwdBlock = 128;

template <int L, int K, typename R, bool CBAR>
__global__ __launch_bounds__(kBwdBlock) void k_edge_bwd(EdgeArgs a, EdgeConsts ec, const R *__restrict__ c,
                                                        const R *__restrict__ Sbar, R *__restrict__ F,
                                                        R *__restrict__ cbar, double *__restrict__ Wpart) {
    constexpr int NL = n_lambda(L);
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double W[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) W[q] = 0.0;
    if (x < a.n_ext) {
        const bool loc = x < a.n;
        R sb[NL][K];
#pragma unroll
        for (int l = 0; l < NL; ++l)
#pragma unroll
            for (int m = 0; m < K; ++m) sb[l][m] = loc ? Sbar[x * NL * K + l * K + m] : R(0);
        R ck[K];
#pragma unroll
        for (int m = 0; m < K; ++m) ck[m] = c[x * K + m];
        R f[3] = {R(0), R(0), R(0)};
        R cb[K];
#pragma unroll
        for (int m = 0; m < K; ++m) cb[m] = R(0);
        const double xi = a.px[x], yi = a.py[x], zi = a.pz[x];
        const R inv_rc = R(1.0 / ec.r_c);
        const R s = R(ec.ang_scale);
        const R pi_rc = R(M_PI / ec.r_c);
        for (int64_t k = a.row[x]; k < a.row[x + 1]; ++k) {
            const int64_t j = a.col[k];
            const bool jloc = j < a.n;
            const double dx = a.px[j] - xi, dy = a.py[j] - yi, dz = a.pz[j] - zi;
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 >= ec.rc2) continue;
            const R r = d_sqrt(R(d2));
            const R rinv = R(1) / r;
            const R t = r * inv_rc;
            const R u = R(0.5) * d_cospi(t) + R(0.5);
            const R fc = u * u;
            const R dfc = -u * pi_rc * d_sinpi(t);
            R Rm[K], dRm[K];
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const R xm = r - R(ec.centres[m]);
                const R al = R(ec.alphas[m]);
                Rm[m] = d_exp(-al * xm * xm);
                dRm[m] = R(-2) * al * xm * Rm[m];
            }
            const R ex = R(dx) * rinv, ey = R(dy) * rinv, ez = R(dz) * rinv;   // unit vector k -> j
            const R ux = R(ec.ang_scale * dx), uy = R(ec.ang_scale * dy), uz = R(ec.ang_scale * dz);
            if (loc) {   // edge x -> j, x the centre
                R A[NL], dA[NL][3];
                angular<L, R, true>(ux, uy, uz, s, A, dA);
                const R *cj = c + j * K;
                R w[K], v[K];
#pragma unroll
                for (int m = 0; m < K; ++m) { w[m] = cj[m] * Rm[m]; v[m] = cj[m] * dRm[m]; }
                R g0 = R(0), g1 = R(0), g2 = R(0), sAP = R(0), sAQ = R(0);
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    R P = R(0), Q = R(0);
#pragma unroll
                    for (int m = 0; m < K; ++m) { P += sb[l][m] * w[m]; Q += sb[l][m] * v[m]; }
                    g0 += P * dA[l][0]; g1 += P * dA[l][1]; g2 += P * dA[l][2];
                    sAP += A[l] * P; sAQ += A[l] * Q;
                }
                const R rad = dfc * sAP + fc * sAQ;
                const R gx = fc * g0 + rad * ex, gy = fc * g1 + rad * ey, gz = fc * g2 + rad * ez;
                f[0] += gx; f[1] += gy; f[2] += gz;
                const double gd[3] = {double(gx), double(gy), double(gz)};
                const double dd[3] = {dx, dy, dz};
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int q = 0; q < 3; ++q) W[3 * p + q] -= dd[p] * gd[q];
            }
            if (jloc) {   // edge j -> x, j the centre: displacement -d
                R A[NL], dA[NL][3];
                angular<L, R, true>(-ux, -uy, -uz, s, A, dA);
                const R *sbj = Sbar + j * NL * K;
                R w[K], v[K];
#pragma unroll
                for (int m = 0; m < K; ++m) { w[m] = ck[m] * Rm[m]; v[m] = ck[m] * dRm[m]; }
                R g0 = R(0), g1 = R(0), g2 = R(0), sAP = R(0), sAQ = R(0);
                R cacc[K];
#pragma unroll
                for (int m = 0; m < K; ++m) cacc[m] = R(0);
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    R P = R(0), Q = R(0);
#pragma unroll
                    for (int m = 0; m < K; ++m) {
                        const R sv = sbj[l * K + m];
                        P += sv * w[m];
                        Q += sv * v[m];
                        if constexpr (CBAR) cacc[m] += sv * A[l];
                    }
                    g0 += P * dA[l][0]; g1 += P * dA[l][1]; g2 += P * dA[l][2];
                    sAP += A[l] * P; sAQ += A[l] * Q;
                }
                const R rad = dfc * sAP + fc * sAQ;
                // the unit vector of this edge is -e
                f[0] -= fc * g0 - rad * ex;
                f[1] -= fc * g1 - rad * ey;
                f[2] -= fc * g2 - rad * ez;
                if constexpr (CBAR) {
#pragma unroll
                    for (int m = 0; m < K; ++m) cb[m] += fc * Rm[m] * cacc[m];
                }
            }
        }
        F[3 * x] += f[0];
        F[3 * x + 1] += f[1];
        F[3 * x + 2] += f[2];
        if constexpr (CBAR) {
#pragma unroll
            for (int m = 0; m < K; ++m) cbar[x * K + m] = cb[m];
        }
    }
    __shared__ double sw[9][kBwdBlock];
#pragma unroll
    for (int q = 0; q < 9; ++q) sw[q][threadIdx.x] = W[q];
    __syncthreads();
    for (int h = kBwdBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 9; ++q) sw[q][threadIdx.x] += sw[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 9) Wpart[(int64_t)blockIdx.x * 9 + threadIdx.x] = sw[threadIdx.x][0];
}

#define REANN_LK_DISPATCH(L, K, CALL)                                              \
    do {                                                                           \
        if ((L) == 2 && (K) == 8) { CALL(2, 8); }                                  \
        else if ((L) == 2 && (K) == 12) { CALL(2, 12); }                           \
        else if ((L) == 1 && (K) == 4) { CALL(1, 4); }                             \
        else if ((L) == 2 && (K) == 4) { CALL(2, 4); }                             \
        else fail(REANN_E_UNSUPPORTED, "no edge kernel compiled for this (L, K)"); \
    } while (0)

void edge_forward(hipStream_t st, bool fp64, int L, int K, const EdgeArgs &a, const EdgeConsts &ec, const void *c,
                  void *S) {
    const int B = 128;
#define FWD(LL, KK)                                                                                        \
    if (fp64)                                                                                              \
        hipLaunchKernelGGL((k_edge_fwd<LL, KK, double>), dim3(grid_for(a.n, B)), dim3(B), 0, st, a, ec,    \
                           (const double *)c, (double *)S);                                                \
    else                                                                                                   \
        hipLaunchKernelGGL((k_edge_fwd<LL, KK, float>), dim3(grid_for(a.n, B)), dim3(B), 0, st, a, ec,     \
                           (const float *)c, (float *)S);
    REANN_LK_DISPATCH(L, K, FWD);
#undef FWD
    LAUNCH_OK("k_edge_fwd");
}

int edge_backward_blocks(int64_t n_ext) { return grid_for(n_ext, kBwdBlock); }

int edge_backward(hipStream_t st, bool fp64, int L, int K, const EdgeArgs &a, const EdgeConsts &ec, const void *c,
                  const void *Sbar, bool want_cbar, void *F, void *cbar, double *Wpart) {
    const int nb = edge_backward_blocks(a.n_ext);
#define BWD(LL, KK)                                                                                          \
    if (fp64) {                                                                                              \
        if (want_cbar)                                                                                       \
            hipLaunchKernelGGL((k_edge_bwd<LL, KK, double, true>), dim3(nb), dim3(kBwdBlock), 0, st, a, ec,  \
                               (const double *)c, (const double *)Sbar, (double *)F, (double *)cbar, Wpart); \
        else                                                                                                 \
            hipLaunchKernelGGL((k_edge_bwd<LL, KK, double, false>), dim3(nb), dim3(kBwdBlock), 0, st, a, ec, \
                               (const double *)c, (const double *)Sbar, (double *)F, (double *)cbar, Wpart); \
    } else {                                                                                                 \
        if (want_cbar)                                                                                       \
            hipLaunchKernelGGL((k_edge_bwd<LL, KK, float, true>), dim3(nb), dim3(kBwdBlock), 0, st, a, ec,   \
                               (const float *)c, (const float *)Sbar, (float *)F, (float *)cbar, Wpart);     \
        else                                                                                                 \
            hipLaunchKernelGGL((k_edge_bwd<LL, KK, float, false>), dim3(nb), dim3(kBwdBlock), 0, st, a, ec,  \
                               (const float *)c, (const float *)Sbar, (float *)F, (float *)cbar, Wpart);     \
    }
    REANN_LK_DISPATCH(L, K, BWD);
#undef BWD
    LAUNCH_OK("k_edge_bwd");
    return nb;
}

// ------------------------------------------------------------- ghost exchange --

template <typename R>
__global__ void k_gather(int64_t n, int64_t n_gh, int K, const int32_t *__restrict__ owner, R *__restrict__ c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_gh * K) return;
    const int64_t g = t / K, m = t % K;
    c[(n + g) * K + m] = c[(int64_t)owner[g] * K + m];
}

template <typename R>
__global__ void k_reduce(int64_t n, int width, const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                         R *__restrict__ v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * width) return;
    const int64_t o = t / width, m = t % width;
    R s = v[o * width + m];
    for (int32_t q = ptr[o]; q < ptr[o + 1]; ++q) s += v[(n + idx[q]) * width + m];
    v[o * width + m] = s;
}

template <typename R>
__global__ void k_init_c(int64_t n_ext, int K, const int8_t *__restrict__ spec, const R *__restrict__ c0,
                         R *__restrict__ c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ext * K) return;
    const int64_t x = t / K, m = t % K;
    c[t] = c0[(int64_t)spec[x] * K + m];
}

void ghost_gather(hipStream_t st, bool fp64, int64_t n, int64_t n_gh, int K, const int32_t *owner, void *c) {
    if (n_gh == 0) return;
    const int64_t tot = n_gh * K;
    if (fp64) hipLaunchKernelGGL(k_gather<double>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, n_gh, K, owner, (double *)c);
    else hipLaunchKernelGGL(k_gather<float>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, n_gh, K, owner, (float *)c);
    LAUNCH_OK("k_gather");
}

void ghost_reduce(hipStream_t st, bool fp64, int64_t n, int width, const int32_t *copy_ptr, const int32_t *copy_idx,
                  void *v) {
    const int64_t tot = n * width;
    if (fp64) hipLaunchKernelGGL(k_reduce<double>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, width, copy_ptr, copy_idx, (double *)v);
    else hipLaunchKernelGGL(k_reduce<float>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n, width, copy_ptr, copy_idx, (float *)v);
    LAUNCH_OK("k_reduce");
}

void init_messages(hipStream_t st, bool fp64, int64_t n_ext, int K, const int8_t *spec, const void *c0, void *c) {
    const int64_t tot = n_ext * K;
    if (fp64) hipLaunchKernelGGL(k_init_c<double>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n_ext, K, spec, (const double *)c0, (double *)c);
    else hipLaunchKernelGGL(k_init_c<float>, dim3(grid_for(tot, 256)), dim3(256), 0, st, n_ext, K, spec, (const float *)c0, (float *)c);
    LAUNCH_OK("k_init_c");
}

}  // namespace reann
