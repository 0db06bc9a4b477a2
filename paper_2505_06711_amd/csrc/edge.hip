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
// No atomics: the centre-role kernel evaluates each edge i->j once (Sbar_i staged in LDS)
// and keeps +g_ij for F_i and the virial; what lands on j (-g_ij and the cbar_j terms) is
// written as a record at the edge's compacted slot.  The neighbour-role kernel then gives
// every ext row k the sum of the records of its edges j->k, found through a per-step map of
// each entry to the compacted slot of its reverse.  Sums over a row's edges are taken across the lanes of a half-wave in a fixed
// order, so results are deterministic.
#include "edge.hpp"

namespace reann {

// Workgroup b is dispatched to XCD b % 8.  Give each XCD one contiguous range of row tiles
// (atoms are ordered by spatial bin, so neighbouring rows share their neighbours' data and
// that data then stays in one XCD's L2).  A bijection on [0, nb).
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb) {
    constexpr int64_t kXcd = 8;
    const int64_t x = b % kXcd, q = b / kXcd, per = nb / kXcd, rem = nb % kXcd;
    return x * per + (x < rem ? x : rem) + q;
}

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

// Radial Gaussian exp(-alpha x^2).  FP32: 2^(-alpha log2(e) x^2) with the hardware base-2
// exponential (a single instruction; the exponent carries the same FP32 rounding as the
// product it replaces).  FP64: exp.  `a` is the matching constant of EdgeConsts.
__device__ inline float gauss(float a2, float x) { return __builtin_amdgcn_exp2f(-a2 * x * x); }
__device__ inline double gauss(double a, double x) { return exp(-a * x * x); }
template <typename R> __device__ inline R gauss_const(const EdgeConsts &ec, int m) {
    return sizeof(R) == 4 ? R(ec.alphas2[m]) : R(ec.alphas[m]);
}
__device__ inline float d_cospi(float x) { return cospif(x); }
__device__ inline double d_cospi(double x) { return cospi(x); }
__device__ inline float d_sinpi(float x) { return sinpif(x); }
__device__ inline double d_sinpi(double x) { return sinpi(x); }
__device__ inline float d_sqrt(float x) { return sqrtf(x); }
__device__ inline double d_sqrt(double x) { return sqrt(x); }

// r / r_c, the argument of the cutoff function.  FP32: a product with 1/r_c rounded to FP32
// would carry that constant's rounding (a relative bias of up to 3e-8, the same sign for every
// edge), which the steep tail of f_c amplifies ~10x near r_c and every atom of a crystal repeats
// coherently; 1/r_c is taken as a sum of two floats instead, so the quotient is within about one
// rounding of the exact one.  FP64: the product with 1/r_c.
__device__ inline float over_rc(float r, double r_c) {
    const double inv = 1.0 / r_c;
    const float hi = (float)inv, lo = (float)(inv - (double)hi);
    return fmaf(r, hi, r * lo);
}
__device__ inline double over_rc(double r, double r_c) { return r * (1.0 / r_c); }

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

// In-cutoff compaction of the (r_c + skin) list for the current positions: each row's
// in-cutoff local neighbours are packed at the front of its slot range and its in-cutoff
// ghost neighbours at the back (reverse order).  Every later pass of the step reads only
// these entries.  fslot maps a compacted slot to its list slot and cpos the other way (cpos
// is written for in-cutoff entries only).
constexpr int kCompactPasses = 8;   // passes of 16 entries whose loads are issued together

__global__ void k_compact(EdgeArgs a, double rc2, int32_t *__restrict__ col2, int32_t *__restrict__ fslot,
                          int32_t *__restrict__ cpos, int32_t *__restrict__ nloc, int32_t *__restrict__ ngh) {
    // 16 lanes per row take the row's entries 16 at a time (a pass); a ballot gives each
    // in-cutoff entry its rank, so the packed order equals a sequential scan of the row.  The
    // entries of up to kCompactPasses passes are loaded at once, then their neighbours'
    // positions, and only then are the passes tested in order, so that a lane has that many
    // independent loads in flight instead of one dependent load per pass.
    constexpr int CH = kCompactPasses;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t x = t >> 4;
    const int g = threadIdx.x & 15, gbase = threadIdx.x & 48;
    const bool active = x < a.n_ext;
    const int64_t lo = active ? a.row[x] : 0, hi = active ? a.row[x + 1] : 0;
    const double4 pi = active ? a.p4[x] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    int64_t front = lo, back = hi;
    const uint32_t below = (1u << g) - 1u;
    const int64_t last = hi - 1;   // indices past the row's end are clamped to its last entry
    for (int64_t base = lo; base < hi; base += 16 * CH) {
        int32_t j[CH];
        double dx[CH], dy[CH], dz[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) j[u] = base + 16 * u < hi ? a.col[min(base + 16 * u + g, last)] : 0;
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const double4 q = base + 16 * u < hi ? a.p4[j[u]] : pi;
            dx[u] = q.x - xi; dy[u] = q.y - yi; dz[u] = q.z - zi;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (base + 16 * u >= hi) break;   // uniform over the row's lanes
            const int64_t k = base + 16 * u + g;
            const bool in = k < hi && dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u] < rc2;
            const bool isl = in && j[u] < a.n, isg = in && j[u] >= a.n;
            const uint32_t ml = (uint32_t)(__ballot(isl) >> gbase) & 0xffffu;
            const uint32_t mg = (uint32_t)(__ballot(isg) >> gbase) & 0xffffu;
            if (isl) {
                const int64_t d = front + __popc(ml & below);
                col2[d] = j[u];
                fslot[d] = (int32_t)k;
                cpos[k] = (int32_t)d;
            }
            if (isg) {
                const int64_t d = back - 1 - __popc(mg & below);
                col2[d] = j[u];
                fslot[d] = (int32_t)k;
                cpos[k] = (int32_t)d;
            }
            front += __popc(ml);
            back -= __popc(mg);
        }
    }
    if (active && g == 0) {
        nloc[x] = (int32_t)(front - lo);
        ngh[x] = (int32_t)(hi - back);
    }
}

// Forward edge pass: the 4 lanes of a quad own one row, lane q the channels
// m = q K/4 .. (q+1) K/4 - 1 (a contiguous block, so a neighbour's message block is one
// vector load and the lane's part of S is written with vector stores).
// The row's edges are taken in groups of 4: lane q evaluates the geometry of edge 4g + q
// (r, f_c and the angular terms, from one position gather), and the quad exchanges these
// with DPP quad broadcasts, so that every lane accumulates all 4 edges into its channels.
// The list entries, positions and messages of group g + 1 are loaded while group g is
// evaluated (indices clamped to the row's last edge; a lane past the end contributes 0).
constexpr int kFwdLanes = 4;

// DPP lane moves within rows of 16 lanes.  The controls used here make every lane read an
// active lane of its own row, so no lane keeps an old value (and none reads an out-of-range
// lane, which would give 0): the move needs no prior register initialisation.
template <int CTRL> __device__ inline int dpp_move(int v) { return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true); }
template <int CTRL> __device__ inline float dpp_move(float v) { return __int_as_float(dpp_move<CTRL>(__float_as_int(v))); }
template <int CTRL> __device__ inline double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_move<CTRL>((int)(uint32_t)(b & 0xffffffffll)), hi = dpp_move<CTRL>((int)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int kDppRowHalfMirror = 0x141;   // lane i <- lane 7 - i within each group of 8
constexpr int kDppRowMirror = 0x140;       // lane i <- lane 15 - i within each row of 16

// value of lane SRC of this lane's quad (all 4 lanes must be active)
template <int SRC, typename V> __device__ inline V quad_bcast(V v) { return dpp_move<SRC * 0x55>(v); }

template <int L, int K, typename R>
__global__ __launch_bounds__(256) void k_edge_fwd(EdgeArgs a, CutList cl, EdgeConsts ec, const R *__restrict__ c,
                                                  R *__restrict__ S) {
    constexpr int NL = n_lambda(L);
    constexpr int G = kFwdLanes, KG = K / G;
    static_assert(K % G == 0, "K must be a multiple of the lanes per row");
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / G;
    const int q = (int)(t % G);
    if (i >= a.n) return;   // the whole quad leaves together
    R acc[NL][KG];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int u = 0; u < KG; ++u) acc[l][u] = R(0);
    R cen[KG], alp[KG];
#pragma unroll
    for (int u = 0; u < KG; ++u) { cen[u] = R(ec.centres[KG * q + u]); alp[u] = gauss_const<R>(ec, KG * q + u); }
    const double4 pi = a.p4[i];
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const R s = R(ec.ang_scale);
    const int nl = cl.nloc[i], cnt = nl + cl.ngh[i], last = cnt - 1;
    const int64_t lo = cl.row[i], gb = cl.row[i + 1] - cl.ngh[i];
    auto slot = [&](int e) -> int64_t { return e < nl ? lo + e : gb + (e - nl); };
    const int ngroups = (cnt + G - 1) / G;
    // group 0 in registers, and the own list entry of group 1
    double xo = 0.0, yo = 0.0, zo = 0.0;
    R cg[G][KG];
    int32_t jnext = 0;
    if (ngroups > 0) {
        const int32_t j0 = cl.col[slot(min(q, last))];
        jnext = cl.col[slot(min(G + q, last))];
        { const double4 q = a.p4[j0]; xo = q.x; yo = q.y; zo = q.z; }
        const int32_t js[G] = {quad_bcast<0>(j0), quad_bcast<1>(j0), quad_bcast<2>(j0), quad_bcast<3>(j0)};
#pragma unroll
        for (int sl = 0; sl < G; ++sl)
#pragma unroll
            for (int u = 0; u < KG; ++u) cg[sl][u] = c[(int64_t)js[sl] * K + KG * q + u];
    }
    for (int g = 0; g < ngroups; ++g) {
        const double dx = xo - xi, dy = yo - yi, dz = zo - zi;
        const bool live = g * G + q <= last;
        R cur[G][KG];
#pragma unroll
        for (int sl = 0; sl < G; ++sl)
#pragma unroll
            for (int u = 0; u < KG; ++u) cur[sl][u] = cg[sl][u];
        {   // group g + 1: own position, the quad's messages, and the own entry of group g + 2
            const int32_t j1 = jnext;
            { const double4 q = a.p4[j1]; xo = q.x; yo = q.y; zo = q.z; }
            const int32_t js[G] = {quad_bcast<0>(j1), quad_bcast<1>(j1), quad_bcast<2>(j1), quad_bcast<3>(j1)};
#pragma unroll
            for (int sl = 0; sl < G; ++sl)
#pragma unroll
                for (int u = 0; u < KG; ++u) cg[sl][u] = c[(int64_t)js[sl] * K + KG * q + u];
            jnext = cl.col[slot(min((g + 2) * G + q, last))];
        }
        // own edge: geometry
        const double d2 = dx * dx + dy * dy + dz * dz;
        const R r = d_sqrt(R(d2));
        const R uc = R(0.5) * d_cospi(over_rc(r, ec.r_c)) + R(0.5);
        const R fc = live ? uc * uc : R(0);
        R A[NL];
        angular<L, R, false>(R(ec.ang_scale * dx), R(ec.ang_scale * dy), R(ec.ang_scale * dz), s, A, nullptr);
        // the quad's 4 edges into this lane's channels
        auto edge = [&](const R rs, const R fs, const R (&As)[NL], const R (&cs)[KG]) {
#pragma unroll
            for (int u = 0; u < KG; ++u) {
                const R xm = rs - cen[u];
                const R w = cs[u] * gauss(alp[u], xm) * fs;
#pragma unroll
                for (int l = 0; l < NL; ++l) acc[l][u] += w * As[l];
            }
        };
#define REANN_FWD_SRC(SRC)                                                          \
        {                                                                           \
            R As[NL];                                                               \
            _Pragma("unroll") for (int l = 0; l < NL; ++l) As[l] = quad_bcast<SRC>(A[l]); \
            edge(quad_bcast<SRC>(r), quad_bcast<SRC>(fc), As, cur[SRC]);            \
        }
        REANN_FWD_SRC(0)
        REANN_FWD_SRC(1)
        REANN_FWD_SRC(2)
        REANN_FWD_SRC(3)
#undef REANN_FWD_SRC
    }
    R *out = S + i * NL * K + KG * q;
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int u = 0; u < KG; ++u) out[l * K + u] = acc[l][u];
}

// Per-edge radial/cutoff factors shared by both adjoint roles.
template <int K, typename R> struct EdgeGeo {
    R r, ex, ey, ez, fc, dfc;
    R Rm[K], dRm[K];
};

template <int K, typename R>
__device__ inline void edge_geo(const EdgeConsts &ec, double dx, double dy, double dz, EdgeGeo<K, R> &g) {
    const double d2 = dx * dx + dy * dy + dz * dz;
    g.r = d_sqrt(R(d2));
    const R rinv = R(1) / g.r;
    const R t = over_rc(g.r, ec.r_c);
    const R u = R(0.5) * d_cospi(t) + R(0.5);
    g.fc = u * u;
    g.dfc = -u * R(M_PI / ec.r_c) * d_sinpi(t);
    g.ex = R(dx) * rinv; g.ey = R(dy) * rinv; g.ez = R(dz) * rinv;
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const R xm = g.r - R(ec.centres[m]);
        const R al = R(ec.alphas[m]);
        g.Rm[m] = gauss(gauss_const<R>(ec, m), xm);
        g.dRm[m] = R(-2) * al * xm * g.Rm[m];
    }
}

// 16-byte vector stores / loads of 4 consecutive values (edge records are 16-byte aligned)
__device__ inline void st4(float *p, float a, float b, float c, float d) {
    *reinterpret_cast<float4 *>(p) = make_float4(a, b, c, d);
}
__device__ inline void st4(double *p, double a, double b, double c, double d) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(a, b);
    reinterpret_cast<double2 *>(p)[1] = make_double2(c, d);
}
__device__ inline void add4(const float *p, float (&v)[4]) {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    v[0] += t.x; v[1] += t.y; v[2] += t.z; v[3] += t.w;
}
__device__ inline void add4(const double *p, double (&v)[4]) {
    const double2 t0 = reinterpret_cast<const double2 *>(p)[0], t1 = reinterpret_cast<const double2 *>(p)[1];
    v[0] += t0.x; v[1] += t0.y; v[2] += t1.x; v[3] += t1.y;
}

constexpr int kRowsPerBlock = 8;   // 256 threads = 8 half-waves, one row each

// Centre role: for local row k and each in-cutoff neighbour j (edge k -> j),
//   g = d/dd [ f_c sum_lambda A_lambda(d) sum_m Sbar_k[lambda][m] c_j[m] R_m(r) ]
// adds +g to F_k and the symmetric part of -d (x) g to the virial; the edge's record gets g
// and (CBAR) the terms
//   f_c R_m sum_lambda Sbar_k[lambda][m] A_lambda(d)  of  cbar_j[m].
// kCentreLanes lanes share a row and take its edges in turn; Sbar_k is staged in LDS and
// read by all of them.  Each lane runs a two-stage pipeline: the list entry of its edge after
// next and the position and message of its next edge are loaded while the current edge is
// evaluated.  The record of edge k -> j is stored at the edge's compacted slot f (so a row's
// records are contiguous): rec[f * RS + 0..2] = g, rec[f * RS + 4 + m] = terms (RS = 4 + K
// with CBAR, 4 without).
constexpr int kCentreLanes = 16;
constexpr int kCentreRows = 256 / kCentreLanes;

// Sum over the kCentreLanes = 16 lanes of a row (one DPP row, all lanes active): the quad
// sums, then each lane adds the mirrored lane's value within its group of 8 (the other quad)
// and within the row (the other half), so every lane ends with the row's total.
static_assert(kCentreLanes == 16, "row sums are formed within a DPP row of 16 lanes");
template <typename R> __device__ inline R row_sum(R v) {
    v += dpp_move<kDppQuadXor1>(v);
    v += dpp_move<kDppQuadXor2>(v);
    v += dpp_move<kDppRowHalfMirror>(v);
    return v + dpp_move<kDppRowMirror>(v);
}

template <int L, int K, typename R, bool CBAR>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 3 : 1) void k_adj_centre(EdgeArgs a, CutList cl, EdgeConsts ec, const R *__restrict__ c,
                                                    const R *__restrict__ Sbar, R *__restrict__ F,
                                                    double *__restrict__ Wpart, R *__restrict__ rec) {
    constexpr int NL = n_lambda(L), LPR = kCentreLanes;
    constexpr int RS = CBAR ? 4 + K : 4;
    constexpr LamTab<L> LT{};
    __shared__ R sS[kCentreRows][NL * K];
    __shared__ double sW[kCentreRows][9];
    const int grp = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t row0 = tile * kCentreRows;
    for (int t = threadIdx.x; t < kCentreRows * NL * K; t += 256) {
        const int64_t rr = row0 + t / (NL * K);
        sS[t / (NL * K)][t % (NL * K)] = rr < a.n ? Sbar[row0 * NL * K + t] : R(0);
    }
    __syncthreads();
    const int64_t x = row0 + grp;
    R f0 = R(0), f1 = R(0), f2 = R(0);
    // virial: the total over all edges of a rotation-invariant energy is symmetric, so the
    // symmetric part of each -d (x) g is accumulated (xx, yy, zz, xy, xz, yz); a lane's few
    // edges in the working type, the row and block sums in FP64
    R W[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) W[q] = R(0);
    if (x < a.n) {
        const double4 pi = a.p4[x];
        const double xi = pi.x, yi = pi.y, zi = pi.z;
        const R s = R(ec.ang_scale);
        const R *sb = sS[grp];
        const int nl = cl.nloc[x], cnt = nl + cl.ngh[x];
        const int64_t lo = cl.row[x], gb = cl.row[x + 1] - cl.ngh[x];
        auto slot = [&](int e) -> int64_t { return e < nl ? lo + e : gb + (e - nl); };
        // two-stage pipeline without branches: the next edge's position and message and the
        // list entry after it are loaded (indices clamped to the row's last edge) while the
        // current edge is evaluated
        int e = lane;
        const int last = cnt - 1;
        double xc = 0.0, yc = 0.0, zc = 0.0;
        R cc[K];
        int32_t jn = 0;
        if (e < cnt) {
            const int64_t s0 = slot(e), s1 = slot(min(e + LPR, last));
            const int32_t j0 = cl.col[s0];
            jn = cl.col[s1];
            { const double4 q = a.p4[j0]; xc = q.x; yc = q.y; zc = q.z; }
#pragma unroll
            for (int m = 0; m < K; ++m) cc[m] = c[(int64_t)j0 * K + m];
        }
        for (; e < cnt; e += LPR) {
            // keep Sbar_k in LDS: without this the compiler hoists the NL*K reads out of the
            // loop into registers, which caps occupancy
            asm volatile("" ::: "memory");
            const double dx = xc - xi, dy = yc - yi, dz = zc - zi;
            const int64_t f = slot(e);
            EdgeGeo<K, R> g;
            edge_geo<K, R>(ec, dx, dy, dz, g);
            R u[K], cacc[K];
#pragma unroll
            for (int m = 0; m < K; ++m) {
                u[m] = cc[m] * g.Rm[m];
                cacc[m] = R(0);
            }
            {
                const int64_t jj = jn, s2 = slot(min(e + 2 * LPR, last));
                { const double4 q = a.p4[jj]; xc = q.x; yc = q.y; zc = q.z; }
#pragma unroll
                for (int m = 0; m < K; ++m) cc[m] = c[jj * K + m];
                jn = cl.col[s2];
            }
            // powers of the scaled displacement; A_lambda and its gradient are formed per lambda
            const R ux = R(ec.ang_scale * dx), uy = R(ec.ang_scale * dy), uz = R(ec.ang_scale * dz);
            R px[L + 1], py[L + 1], pz[L + 1];
            px[0] = py[0] = pz[0] = R(1);
#pragma unroll
            for (int k = 1; k <= L; ++k) { px[k] = px[k - 1] * ux; py[k] = py[k - 1] * uy; pz[k] = pz[k - 1] * uz; }
            // P_lambda = sum_m Sbar[lambda][m] u_m for the angular gradient, and
            // cacc_m = sum_lambda Sbar[lambda][m] A_lambda; the two radial contractions then
            // follow as sum_lambda A_lambda P_lambda = cacc . u and
            // sum_lambda A_lambda sum_m Sbar[lambda][m] v_m = cacc . v
            R gx = R(0), gy = R(0), gz = R(0);
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                // one row of Sbar_k at a time (the compiler would otherwise load them all ahead)
                asm volatile("" ::: "memory");
                const int lx = LT.lx[l], ly = LT.ly[l], lz = LT.lz[l];
                const R Al = px[lx] * py[ly] * pz[lz];
                R P = R(0);
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    const R w = sb[l * K + m];
                    P += w * u[m];
                    cacc[m] += w * Al;
                }
                if (lx) gx += P * (s * R(lx) * px[lx > 0 ? lx - 1 : 0] * py[ly] * pz[lz]);
                if (ly) gy += P * (s * R(ly) * px[lx] * py[ly > 0 ? ly - 1 : 0] * pz[lz]);
                if (lz) gz += P * (s * R(lz) * px[lx] * py[ly] * pz[lz > 0 ? lz - 1 : 0]);
            }
            // c_m dR_m/dr = -2 alpha_m (r - r_m) u_m, formed here rather than kept through the loop
            R sAP = R(0), sAQ = R(0);
#pragma unroll
            for (int m = 0; m < K; ++m) {
                sAP += cacc[m] * u[m];
                sAQ += cacc[m] * (R(-2) * R(ec.alphas[m]) * (g.r - R(ec.centres[m])) * u[m]);
            }
            const R rad = g.dfc * sAP + g.fc * sAQ;
            gx = g.fc * gx + rad * g.ex; gy = g.fc * gy + rad * g.ey; gz = g.fc * gz + rad * g.ez;
            f0 += gx; f1 += gy; f2 += gz;
            R *out = rec + f * RS;
            st4(out, gx, gy, gz, R(0));
            if constexpr (CBAR) {
#pragma unroll
                for (int m = 0; m < K; m += 4)
                    st4(out + 4 + m, g.fc * g.Rm[m] * cacc[m], g.fc * g.Rm[m + 1] * cacc[m + 1],
                        g.fc * g.Rm[m + 2] * cacc[m + 2], g.fc * g.Rm[m + 3] * cacc[m + 3]);
            }
            const R ddx = R(dx), ddy = R(dy), ddz = R(dz);
            W[0] -= ddx * gx;
            W[1] -= ddy * gy;
            W[2] -= ddz * gz;
            W[3] -= R(0.5) * (ddx * gy + ddy * gx);
            W[4] -= R(0.5) * (ddx * gz + ddz * gx);
            W[5] -= R(0.5) * (ddy * gz + ddz * gy);
        }
    }
    f0 = row_sum(f0); f1 = row_sum(f1); f2 = row_sum(f2);
    double Wd[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) Wd[q] = row_sum(double(W[q]));
    if (lane == 0) {
        if (x < a.n) { F[3 * x] += f0; F[3 * x + 1] += f1; F[3 * x + 2] += f2; }
        sW[grp][0] = Wd[0]; sW[grp][4] = Wd[1]; sW[grp][8] = Wd[2];
        sW[grp][1] = sW[grp][3] = Wd[3];
        sW[grp][2] = sW[grp][6] = Wd[4];
        sW[grp][5] = sW[grp][7] = Wd[5];
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double t = 0.0;
        for (int h = 0; h < kCentreRows; ++h) t += sW[h][threadIdx.x];
        Wpart[tile * 9 + threadIdx.x] = t;
    }
}

// Neighbour role: ext row k (local or ghost) sums the records of the edges j -> k over its
// in-cutoff local neighbours j (at the compacted slot of the reverse of each entry k -> j):
// F_k -= sum g and, with CBAR, cbar_k[m] = sum of the terms.  The reverse of an in-cutoff
// entry is in cutoff (its displacement is the exact negation), so its compacted slot is set.
// MAKE (the step's first gather) finds that slot through fslot, rev and cpos and stores it in
// rslot; the later gathers read rslot.  With CBAR 4 lanes share an edge record (one group
// of 4 values each, 8 edges per pass of the half-wave); without it a lane takes an edge.
template <int K, typename R, bool CBAR, bool MAKE>
__global__ __launch_bounds__(256) void k_adj_gather(EdgeArgs a, CutList cl, const R *__restrict__ rec,
                                                    R *__restrict__ F, R *__restrict__ cbar) {
    constexpr int RS = CBAR ? 4 + K : 4;
    constexpr int NP = RS / 4;              // groups of 4 values per record
    constexpr int LPE = CBAR ? 4 : 1;       // lanes per edge
    constexpr int EPP = 32 / LPE;           // edges per pass
    static_assert(K % 4 == 0 && (NP <= LPE || !CBAR), "record layout");
    const int hw = threadIdx.x >> 5, lane = threadIdx.x & 31;
    const int64_t x = xcd_tile(blockIdx.x, gridDim.x) * kRowsPerBlock + hw;
    if (x >= a.n_ext) return;   // whole half-wave leaves together
    const int part = lane % LPE, eg = lane / LPE;
    R acc[4] = {R(0), R(0), R(0), R(0)};
    const int cnt = cl.nloc[x], last = cnt - 1;
    const int64_t lo = cl.row[x];
    // U passes at a time, so that each lane has U independent (reverse slot -> record) loads
    // in flight; indices past the row's end are clamped to its last edge and their records
    // are not added
    constexpr int U = 8;
    const int pc = part < NP ? 4 * part : 0;
    for (int e0 = eg; e0 < cnt; e0 += U * EPP) {
        int32_t rv[U];
        if constexpr (MAKE) {
            // first gather of a step: the reverse compacted slot from the list slot, its
            // reverse and that one's compacted slot, kept in rslot for the later gathers
#pragma unroll
            for (int u = 0; u < U; ++u) rv[u] = cl.fslot[lo + min(e0 + u * EPP, last)];
#pragma unroll
            for (int u = 0; u < U; ++u) rv[u] = cl.rev[rv[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) rv[u] = cl.cpos[rv[u]];
            if (part == 0) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (e0 + u * EPP < cnt) cl.rslot[lo + e0 + u * EPP] = rv[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) rv[u] = cl.rslot[lo + min(e0 + u * EPP, last)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            R v[4] = {R(0), R(0), R(0), R(0)};
            add4(rec + (int64_t)rv[u] * RS + pc, v);
            if (e0 + u * EPP < cnt && part < NP) {
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] += v[q];
            }
        }
    }
#pragma unroll
    for (int o = LPE; o < 32; o <<= 1)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += __shfl_xor(acc[q], o, 32);
    if (eg == 0) {
        if (part == 0) {
            F[3 * x] -= acc[0]; F[3 * x + 1] -= acc[1]; F[3 * x + 2] -= acc[2];
        } else if (CBAR && part < NP) {
#pragma unroll
            for (int q = 0; q < 4; ++q) cbar[x * K + 4 * (part - 1) + q] = acc[q];
        }
    }
}

#define REANN_LK_DISPATCH(L, K, CALL)                                              \
    do {                                                                           \
        if ((L) == 2 && (K) == 8) { CALL(2, 8); }                                  \
        else if ((L) == 2 && (K) == 12) { CALL(2, 12); }                           \
        else if ((L) == 1 && (K) == 4) { CALL(1, 4); }                             \
        else if ((L) == 2 && (K) == 4) { CALL(2, 4); }                             \
        else if ((L) == 0 && (K) == 12) { CALL(0, 12); }                           \
        else if ((L) == 0 && (K) == 8) { CALL(0, 8); }                             \
        else fail(REANN_E_UNSUPPORTED, "no edge kernel compiled for this (L, K)"); \
    } while (0)

void compact_cutoff(hipStream_t st, const EdgeArgs &a, double r_c, CutList &cl) {
    hipLaunchKernelGGL(k_compact, dim3(grid_for(a.n_ext * 16, 256)), dim3(256), 0, st, a, r_c * r_c, cl.col, cl.fslot,
                       cl.cpos, cl.nloc, cl.ngh);
    LAUNCH_OK("k_compact");
}


void edge_forward(hipStream_t st, bool fp64, int L, int K, const EdgeArgs &a, const CutList &cl, const EdgeConsts &ec,
                  const void *c, void *S) {
    const int B = 256;
    const int64_t nt = a.n * kFwdLanes;
#define FWD(LL, KK)                                                                                       \
    if (fp64)                                                                                             \
        hipLaunchKernelGGL((k_edge_fwd<LL, KK, double>), dim3(grid_for(nt, B)), dim3(B), 0, st, a, cl, ec, \
                           (const double *)c, (double *)S);                                               \
    else                                                                                                  \
        hipLaunchKernelGGL((k_edge_fwd<LL, KK, float>), dim3(grid_for(nt, B)), dim3(B), 0, st, a, cl, ec,  \
                           (const float *)c, (float *)S);
    REANN_LK_DISPATCH(L, K, FWD);
#undef FWD
    LAUNCH_OK("k_edge_fwd");
}

int edge_backward_blocks(int64_t n_ext) { return grid_for(n_ext, kCentreRows); }

int edge_adjoint_centre(hipStream_t st, bool fp64, int L, int K, const EdgeArgs &a, const CutList &cl,
                        const EdgeConsts &ec, const void *c, const void *Sbar, bool want_cbar, void *F, double *Wpart,
                        void *rec) {
    const int nbc = grid_for(a.n, kCentreRows);
#define CEN_T(LL, KK, R, CB)                                                                                       \
    hipLaunchKernelGGL((k_adj_centre<LL, KK, R, CB>), dim3(nbc), dim3(256), 0, st, a, cl, ec, (const R *)c,      \
                       (const R *)Sbar, (R *)F, Wpart, (R *)rec);
#define CEN(LL, KK)                                             \
    if (fp64) {                                                 \
        if (want_cbar) { CEN_T(LL, KK, double, true) }          \
        else { CEN_T(LL, KK, double, false) }                   \
    } else {                                                    \
        if (want_cbar) { CEN_T(LL, KK, float, true) }           \
        else { CEN_T(LL, KK, float, false) }                    \
    }
    REANN_LK_DISPATCH(L, K, CEN);
#undef CEN
#undef CEN_T
    LAUNCH_OK("k_adj_centre");
    return nbc;
}

void edge_adjoint_gather(hipStream_t st, bool fp64, int K, const EdgeArgs &a, const CutList &cl, bool want_cbar,
                         bool make_rslot, const void *rec, void *F, void *cbar) {
    const int nbn = grid_for(a.n_ext, kRowsPerBlock);
#define GAT_T(KK, R, CB)                                                                                          \
    if (make_rslot)                                                                                               \
        hipLaunchKernelGGL((k_adj_gather<KK, R, CB, true>), dim3(nbn), dim3(256), 0, st, a, cl, (const R *)rec,   \
                           (R *)F, (R *)cbar);                                                                    \
    else                                                                                                          \
        hipLaunchKernelGGL((k_adj_gather<KK, R, CB, false>), dim3(nbn), dim3(256), 0, st, a, cl, (const R *)rec,  \
                           (R *)F, (R *)cbar);
#define GAT(KK)                                                 \
    if (fp64) {                                                 \
        if (want_cbar) { GAT_T(KK, double, true) }              \
        else { GAT_T(KK, double, false) }                       \
    } else {                                                    \
        if (want_cbar) { GAT_T(KK, float, true) }               \
        else { GAT_T(KK, float, false) }                        \
    }
    if (K == 4) { GAT(4) }
    else if (K == 8) { GAT(8) }
    else if (K == 12) { GAT(12) }
    else fail(REANN_E_UNSUPPORTED, "no edge kernel compiled for this K");
#undef GAT
#undef GAT_T
    LAUNCH_OK("k_adj_gather");
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
