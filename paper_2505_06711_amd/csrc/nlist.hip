// GPU neighbour-list build for the subdomain-extended system.
//
// Every FP64 position operation here is written without contraction so that the pair
// predicate is exactly  d = y_j - w_i,  fma(dz,dz, fma(dy,dy, dx*dx)) < (r_c+skin)^2,
// with w the wrapped position and y = w + shift*L the copy position.
#include "nlist.hpp"

#include <cstring>

#include <algorithm>
#include <cmath>

#pragma clang fp contract(off)

namespace reann {

// ------------------------------------------------------------------ geometry --

void geom_init(Geom &g, const double cell[9], const int32_t pbc[3], const int32_t P[3], double r_c, double skin) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (a != b && cell[3 * a + b] != 0.0) fail(REANN_E_UNSUPPORTED, "only orthorhombic cells are supported");
    g.ndom = 1;
    for (int a = 0; a < 3; ++a) {
        g.L[a] = cell[4 * a];
        g.per[a] = pbc[a] ? 1 : 0;
        g.P[a] = P ? (P[a] > 0 ? P[a] : 1) : 1;
        if (g.P[a] > kMaxSplit) fail(REANN_E_UNSUPPORTED, "at most 16 subdomains per axis");
        if (!g.per[a] && g.P[a] != 1) fail(REANN_E_INVALID, "a non-periodic axis cannot be split");
        if (g.per[a] && !(g.L[a] > 0.0 && std::isfinite(g.L[a]))) fail(REANN_E_INVALID, "periodic cell length must be > 0");
        g.ndom *= g.P[a];
        if (g.per[a]) {
            double h = g.L[a] / g.P[a];
            for (int k = 0; k < g.P[a]; ++k) {
                g.lo[a][k] = k * h;
                g.hi[a][k] = (k == g.P[a] - 1) ? g.L[a] : (k + 1) * h;
            }
        } else {
            g.lo[a][0] = -INFINITY;
            g.hi[a][0] = INFINITY;
        }
    }
    g.rcut = r_c + skin;
    g.rc2 = g.rcut * g.rcut;
    g.shell = g.rcut + 1e-6;
    for (int a = 0; a < 3; ++a) g.nm[a] = g.per[a] ? (int)std::floor(g.shell / g.L[a]) + 1 : 0;
}

__device__ inline double wrap_coord(double x, double L, int &qe) {
    double q = floor(x / L);
    double t = q * L;
    double w = x - t;
    int k = (int)q;
    if (w < 0.0) { w = w + L; k -= 1; }
    if (w >= L) { w = w - L; k += 1; }
    qe = k;
    return w;
}

// Domains along axis a whose shell contains coordinate y: bitmask (P <= 16).
__device__ inline unsigned axis_domains(const Geom &g, int a, double y) {
    if (!g.per[a]) return 1u;
    unsigned m = 0;
    for (int k = 0; k < g.P[a]; ++k)
        if (y >= g.lo[a][k] - g.shell && y < g.hi[a][k] + g.shell) m |= 1u << k;
    return m;
}

__global__ void k_wrap_count(Geom g, int64_t n, const double *__restrict__ pos, double *__restrict__ w,
                             int32_t *__restrict__ q, int32_t *__restrict__ dom, int64_t *__restrict__ gcount,
                             int32_t *__restrict__ bad) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int c[3];
    double wu[3];
    bool finite = true;
    for (int a = 0; a < 3; ++a) finite = finite && isfinite(pos[3 * u + a]) && fabs(pos[3 * u + a]) < 1e9;
    if (!finite) {
        // flagged for the host; the atom gets no copies so every offset stays in range
        atomicOr(bad, 1);
        for (int a = 0; a < 3; ++a) { w[3 * u + a] = 0.0; q[3 * u + a] = 0; }
        dom[u] = 0;
        gcount[u] = 0;
        return;
    }
    for (int a = 0; a < 3; ++a) {
        double x = pos[3 * u + a];
        int qe = 0;
        double ww = g.per[a] ? wrap_coord(x, g.L[a], qe) : x;
        wu[a] = ww;
        w[3 * u + a] = ww;
        q[3 * u + a] = qe;
        c[a] = 0;
        for (int k = 0; k < g.P[a]; ++k)
            if (ww >= g.lo[a][k] && ww < g.hi[a][k]) c[a] = k;
    }
    dom[u] = (c[0] * g.P[1] + c[1]) * g.P[2] + c[2];
    int64_t cnt = 0;
    for (int s0 = -g.nm[0]; s0 <= g.nm[0]; ++s0)
        for (int s1 = -g.nm[1]; s1 <= g.nm[1]; ++s1)
            for (int s2 = -g.nm[2]; s2 <= g.nm[2]; ++s2) {
                int s[3] = {s0, s1, s2};
                unsigned m[3];
                for (int a = 0; a < 3; ++a) {
                    double y = g.per[a] ? wu[a] + (double)s[a] * g.L[a] : wu[a];
                    m[a] = axis_domains(g, a, y);
                }
                int k = __popc(m[0]) * __popc(m[1]) * __popc(m[2]);
                if (s0 == 0 && s1 == 0 && s2 == 0) k -= 1;   // the atom itself in its own subdomain
                cnt += k;
            }
    gcount[u] = cnt;
}

__global__ void k_ghost_gen(Geom g, int64_t n, const double *__restrict__ w, const int32_t *__restrict__ dom,
                            const int64_t *__restrict__ goff, int32_t *__restrict__ g_owner, int32_t *__restrict__ g_shift,
                            int32_t *__restrict__ g_dom, double *__restrict__ g_pos) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int64_t o = goff[u];
    if (goff[u + 1] == o) return;   // no copies (also the case of a flagged atom)
    double wu[3] = {w[3 * u], w[3 * u + 1], w[3 * u + 2]};
    int own = dom[u];
    for (int s0 = -g.nm[0]; s0 <= g.nm[0]; ++s0)
        for (int s1 = -g.nm[1]; s1 <= g.nm[1]; ++s1)
            for (int s2 = -g.nm[2]; s2 <= g.nm[2]; ++s2) {
                int s[3] = {s0, s1, s2};
                unsigned m[3];
                double y[3];
                for (int a = 0; a < 3; ++a) {
                    y[a] = g.per[a] ? wu[a] + (double)s[a] * g.L[a] : wu[a];
                    m[a] = axis_domains(g, a, y[a]);
                }
                for (int k0 = 0; k0 < g.P[0]; ++k0) {
                    if (!(m[0] >> k0 & 1u)) continue;
                    for (int k1 = 0; k1 < g.P[1]; ++k1) {
                        if (!(m[1] >> k1 & 1u)) continue;
                        for (int k2 = 0; k2 < g.P[2]; ++k2) {
                            if (!(m[2] >> k2 & 1u)) continue;
                            int p = (k0 * g.P[1] + k1) * g.P[2] + k2;
                            if (s0 == 0 && s1 == 0 && s2 == 0 && p == own) continue;
                            g_owner[o] = (int32_t)u;
                            g_shift[3 * o] = s0; g_shift[3 * o + 1] = s1; g_shift[3 * o + 2] = s2;
                            g_dom[o] = p;
                            g_pos[3 * o] = y[0]; g_pos[3 * o + 1] = y[1]; g_pos[3 * o + 2] = y[2];
                            ++o;
                        }
                    }
                }
            }
}

struct Bins {
    double mn[3], bs[3];
    int nb[3];
    int64_t nbin;
};

__device__ inline int bin_of(const Bins &b, const double *y) {
    int c[3];
    for (int a = 0; a < 3; ++a) {
        int k = (int)((y[a] - b.mn[a]) / b.bs[a]);
        c[a] = k < 0 ? 0 : (k >= b.nb[a] ? b.nb[a] - 1 : k);
    }
    return (c[0] * b.nb[1] + c[1]) * b.nb[2] + c[2];
}

// Key of a pre-ext element: locals (slot = species) then ghosts (slot = n_species, or with
// ghosts_by_species n_species + the owner's species).
__global__ void k_keys(Bins b, int ndom, int n_species, int64_t n, int64_t n_gh, const double *__restrict__ w,
                       const int32_t *__restrict__ dom, const int32_t *__restrict__ species, const double *__restrict__ g_pos,
                       const int32_t *__restrict__ g_dom, const int32_t *__restrict__ g_owner, int ghosts_by_species,
                       int64_t *__restrict__ key, int32_t *__restrict__ count) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n + n_gh) return;
    int slot, p;
    int bn;
    if (e < n) {
        slot = species[e]; p = dom[e]; bn = bin_of(b, w + 3 * e);
    } else {
        int64_t gi = e - n;
        slot = n_species + (ghosts_by_species ? species[g_owner[gi]] : 0);
        p = g_dom[gi];
        bn = bin_of(b, g_pos + 3 * gi);
    }
    int64_t k = ((int64_t)slot * ndom + p) * b.nbin + bn;
    key[e] = k;
    atomicAdd(&count[k], 1);
}

__global__ void k_i32_to_i64(const int32_t *__restrict__ a, int64_t *__restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_scatter(int64_t m, const int64_t *__restrict__ key, const int64_t *__restrict__ kstart,
                          int32_t *__restrict__ cursor, int32_t *__restrict__ order) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int64_t k = key[e];
    int64_t pos = kstart[k] + atomicAdd(&cursor[k], 1);
    order[pos] = (int32_t)e;
}

// Sort each segment [start[k], start[k+1]) of distinct values ascending.  One wave per
// segment: every value's rank is the number of smaller values in the segment, taken against
// an LDS copy; a segment longer than kSegLds is sorted by one lane (insertion sort) instead.
constexpr int kSegLds = 1024;

__global__ __launch_bounds__(256) void k_sort_segments(int64_t nseg, const int64_t *__restrict__ start,
                                                       int32_t *__restrict__ v) {
    __shared__ int32_t sv[4][kSegLds];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * 4 + w;
    const bool valid = k < nseg;
    const int64_t a = valid ? start[k] : 0;
    const int m = valid ? (int)(start[k + 1] - a) : 0;
    const bool in_lds = m <= kSegLds;
    if (in_lds)
        for (int e = lane; e < m; e += 64) sv[w][e] = v[a + e];
    __syncthreads();
    if (in_lds) {
        for (int e = lane; e < m; e += 64) {
            const int32_t x = sv[w][e];
            int rank = 0;
            for (int q = 0; q < m; ++q) rank += sv[w][q] < x;
            v[a + rank] = x;
        }
    } else if (lane == 0) {
        for (int64_t i = a + 1; i < a + m; ++i) {
            const int32_t x = v[i];
            int64_t j = i - 1;
            while (j >= a && v[j] > x) { v[j + 1] = v[j]; --j; }
            v[j + 1] = x;
        }
    }
}

__global__ void k_sort_segments32(int64_t nseg, const int32_t *__restrict__ start, int32_t *__restrict__ v) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    int32_t a = start[k], e = start[k + 1];
    for (int32_t i = a + 1; i < e; ++i) {
        int32_t x = v[i];
        int32_t j = i - 1;
        while (j >= a && v[j] > x) { v[j + 1] = v[j]; --j; }
        v[j + 1] = x;
    }
}

// rev[f] for the entry f = (x -> j) of a sorted list: the slot of (j -> x) in row j.  Every
// entry has one: rows of locals list every ext atom in range, rows of ghosts every local in
// range, and a row of a ghost only holds locals.  Each pair is resolved once, from its entry
// with x < j (a binary search for x in row j), which writes both slots; rev starts at -1, and
// k_reverse_check then sets *bad if a slot was not written (an entry without its reverse).
__global__ void k_reverse(int64_t n_ext, const int64_t *__restrict__ row, const int32_t *__restrict__ col,
                          int32_t *__restrict__ rev, int32_t *__restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t x = t >> 4;
    const int g = (int)(t & 15);
    if (x >= n_ext) return;
    const int64_t hi = row[x + 1];
    for (int64_t f = row[x] + g; f < hi; f += 16) {
        const int32_t j = col[f];
        if (j < x) continue;   // resolved from (j -> x)
        int64_t a = row[j], b = row[j + 1];
        const int64_t end = b;
        while (a < b) {
            const int64_t mid = (a + b) >> 1;
            if (col[mid] < x) a = mid + 1;
            else b = mid;
        }
        if (a < end && col[a] == (int32_t)x) {
            rev[f] = (int32_t)a;
            rev[a] = (int32_t)f;
        } else {
            atomicOr(bad, 1);
        }
    }
}

__global__ void k_reverse_check(int64_t n_pairs, const int32_t *__restrict__ rev, int32_t *__restrict__ bad) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < n_pairs && rev[f] < 0) atomicOr(bad, 1);
}

__global__ void k_build_ext(Bins b, int64_t n, int64_t n_ext, const int32_t *__restrict__ order,
                            const double *__restrict__ w, const int32_t *__restrict__ dom, const int32_t *__restrict__ species,
                            const double *__restrict__ g_pos, const int32_t *__restrict__ g_dom,
                            const int32_t *__restrict__ g_owner_user, const int32_t *__restrict__ g_shift_in,
                            int32_t *__restrict__ perm, int32_t *__restrict__ inv_perm, double *__restrict__ pext,
                            int32_t *__restrict__ dom_ext, int32_t *__restrict__ bin_ext, int8_t *__restrict__ spec_ext,
                            int32_t *__restrict__ gh_owner_user, int32_t *__restrict__ gh_shift) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_ext) return;
    int64_t pre = order[x];
    const double *y;
    if (pre < n) {
        perm[x] = (int32_t)pre;
        inv_perm[pre] = (int32_t)x;
        y = w + 3 * pre;
        dom_ext[x] = dom[pre];
        spec_ext[x] = (int8_t)species[pre];
    } else {
        int64_t gi = pre - n, go = x - n;
        y = g_pos + 3 * gi;
        dom_ext[x] = g_dom[gi];
        int32_t ou = g_owner_user[gi];
        gh_owner_user[go] = ou;
        spec_ext[x] = (int8_t)species[ou];
        for (int a = 0; a < 3; ++a) gh_shift[3 * go + a] = g_shift_in[3 * gi + a];
    }
    pext[x] = y[0];
    pext[n_ext + x] = y[1];
    pext[2 * n_ext + x] = y[2];
    bin_ext[x] = bin_of(b, y);
}

__global__ void k_ghost_owner(int64_t n_gh, const int32_t *__restrict__ owner_user, const int32_t *__restrict__ inv_perm,
                              int32_t *__restrict__ owner) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n_gh) owner[g] = inv_perm[owner_user[g]];
}

// Candidate scan over the 27 bins around atom x of its subdomain.  Locals see every ext atom
// of the subdomain; ghosts see only locals.  A half-wave (32 lanes) takes a row: the keys in
// increasing order (slot, then the stencil's bins by index), and each key's atoms 32 at a
// time, one per lane, so that the atoms' positions are read contiguously.  Ext atoms are
// numbered in key order, so the row comes out with its columns ascending.  The count pass
// keeps each 32-atom chunk's hits as one word (up to cap_words chunks per row) and the fill
// replays them; a row with more chunks is measured again by the fill.
constexpr int kRowsPerBlk = 8;   // 256 threads, a half-wave per row

template <bool FILL>
__global__ __launch_bounds__(256) void k_rows_group(Bins b, Geom g, int n_species, int n_ghost_slots, int64_t n, int64_t n_ext,
                                              const double *__restrict__ pext, const int32_t *__restrict__ dom_ext,
                                              const int32_t *__restrict__ bin_ext, const int64_t *__restrict__ kstart,
                                              int64_t *__restrict__ rowcnt, const int64_t *__restrict__ row,
                                              int32_t *__restrict__ col, int32_t *__restrict__ coincident,
                                              uint32_t *__restrict__ mask, int32_t *__restrict__ nchunk, int cap_words) {
    const int64_t x = (int64_t)blockIdx.x * kRowsPerBlk + (threadIdx.x >> 5);
    const int lane = threadIdx.x & 31, half = threadIdx.x & 32;
    if (x >= n_ext) return;   // the whole half-wave
    const double xi = pext[x], yi = pext[n_ext + x], zi = pext[2 * n_ext + x];
    const int p = dom_ext[x];
    const int bx = bin_ext[x];
    const int c2 = bx % b.nb[2], c1 = (bx / b.nb[2]) % b.nb[1], c0 = bx / (b.nb[2] * b.nb[1]);
    const int nslot = (x < n) ? n_species + n_ghost_slots : n_species;
    uint32_t *mrow = mask + x * cap_words;
    const int nkept = FILL ? nchunk[x] : 0;
    const bool replay = FILL && nkept <= cap_words;
    int64_t cnt = 0, o = FILL ? row[x] : 0;
    int q = 0;   // chunks so far
    // replay: the row's words are read 32 at a time, one per lane, and passed round by shuffles
    uint32_t wbuf = 0;
    int wbase = -32;
    for (int slot = 0; slot < nslot; ++slot) {
        for (int d0 = -1; d0 <= 1; ++d0) {
            const int a0 = c0 + d0;
            if (a0 < 0 || a0 >= b.nb[0]) continue;
            for (int d1 = -1; d1 <= 1; ++d1) {
                const int a1 = c1 + d1;
                if (a1 < 0 || a1 >= b.nb[1]) continue;
                for (int d2 = -1; d2 <= 1; ++d2) {
                    const int a2 = c2 + d2;
                    if (a2 < 0 || a2 >= b.nb[2]) continue;
                    const int64_t bn = ((int64_t)a0 * b.nb[1] + a1) * b.nb[2] + a2;
                    const int64_t k = ((int64_t)slot * g.ndom + p) * b.nbin + bn;
                    const int64_t s0 = kstart[k], s1 = kstart[k + 1];
                    for (int64_t t0 = s0; t0 < s1; t0 += 32, ++q) {
                        const int64_t e = t0 + lane;
                        uint32_t bits;
                        if (replay) {
                            if (q >= wbase + 32) {
                                wbase = q;
                                wbuf = q + lane < nkept ? mrow[q + lane] : 0u;
                            }
                            bits = (uint32_t)__shfl((int)wbuf, q - wbase, 32);
                        } else {
                            bool hit = false;
                            if (e < s1 && e != x) {
                                const double dx = pext[e] - xi, dy = pext[n_ext + e] - yi, dz = pext[2 * n_ext + e] - zi;
                                const double dd = fma(dz, dz, fma(dy, dy, dx * dx));
                                hit = dd < g.rc2;
                                // two copies closer than 1e-6 A: the pair direction is undefined
                                if (!FILL && dd < 1e-12) atomicOr(coincident, 1);
                            }
                            bits = (uint32_t)(__ballot(hit) >> half);
                        }
                        if (FILL) {
                            if ((bits >> lane) & 1u) col[o + __popc(bits & ((1u << lane) - 1u))] = (int32_t)e;
                            o += __popc(bits);
                        } else {
                            cnt += __popc(bits);
                            if (lane == 0 && q < cap_words) mrow[q] = bits;
                        }
                    }
                }
            }
        }
    }
    if (!FILL && lane == 0) {
        rowcnt[x] = cnt;
        nchunk[x] = q;
    }
}

// The candidate scan (see k_rows_group) with a thread per row, each taking its candidates one
// by one: the count pass keeps the hits as bits over the row's candidates (up to 32 cap_words),
// and the fill replays them.  Suits rows whose keys hold few atoms (several elements, small
// bins), where most lanes of a group would idle.
template <bool FILL>
__global__ void k_rows_thread(Bins b, Geom g, int n_species, int n_ghost_slots, int64_t n, int64_t n_ext, const double *__restrict__ pext,
                       const int32_t *__restrict__ dom_ext, const int32_t *__restrict__ bin_ext,
                       const int64_t *__restrict__ kstart, int64_t *__restrict__ rowcnt, const int64_t *__restrict__ row,
                       int32_t *__restrict__ col, int32_t *__restrict__ coincident, uint32_t *__restrict__ mask,
                       int32_t *__restrict__ ncand, int cap_words) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_ext) return;
    const double xi = pext[x], yi = pext[n_ext + x], zi = pext[2 * n_ext + x];
    const int p = dom_ext[x];
    const int bx = bin_ext[x];
    const int c2 = bx % b.nb[2], c1 = (bx / b.nb[2]) % b.nb[1], c0 = bx / (b.nb[2] * b.nb[1]);
    const int nslot = (x < n) ? n_species + n_ghost_slots : n_species;
    const int64_t cap_bits = (int64_t)cap_words * 32;
    uint32_t *mrow = mask + x * cap_words;
    // the fill replays the count pass's hits from its bits when they fitted, else it measures
    // the distances again
    const bool replay = FILL && ncand[x] <= cap_bits;
    int64_t cnt = 0, o = FILL ? row[x] : 0, ci = 0;
    uint32_t word = 0;
    // keys in increasing order (slot, then the stencil's bins by index): ext atoms are numbered
    // in key order, so a row comes out with its columns ascending; ci numbers the candidates in
    // this order
    for (int slot = 0; slot < nslot; ++slot) {
        for (int d0 = -1; d0 <= 1; ++d0) {
            int a0 = c0 + d0;
            if (a0 < 0 || a0 >= b.nb[0]) continue;
            for (int d1 = -1; d1 <= 1; ++d1) {
                int a1 = c1 + d1;
                if (a1 < 0 || a1 >= b.nb[1]) continue;
                for (int d2 = -1; d2 <= 1; ++d2) {
                    int a2 = c2 + d2;
                    if (a2 < 0 || a2 >= b.nb[2]) continue;
                    int64_t bn = ((int64_t)a0 * b.nb[1] + a1) * b.nb[2] + a2;
                    int64_t k = ((int64_t)slot * g.ndom + p) * b.nbin + bn;
                    for (int64_t e = kstart[k]; e < kstart[k + 1]; ++e, ++ci) {
                        if (replay) {
                            if ((ci & 31) == 0) word = mrow[ci >> 5];
                            if ((word >> (ci & 31)) & 1u) col[o++] = (int32_t)e;
                            continue;
                        }
                        bool hit = false;
                        if (e != x) {
                            double dx = pext[e] - xi, dy = pext[n_ext + e] - yi, dz = pext[2 * n_ext + e] - zi;
                            double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
                            hit = d2 < g.rc2;
                            // two copies closer than 1e-6 A: the pair direction is undefined
                            if (!FILL && d2 < 1e-12) atomicOr(coincident, 1);
                        }
                        if (FILL) {
                            if (hit) col[o++] = (int32_t)e;
                        } else {
                            if (hit) {
                                ++cnt;
                                word |= 1u << (ci & 31);
                            }
                            if ((ci & 31) == 31) {
                                if ((ci >> 5) < cap_words) mrow[ci >> 5] = word;
                                word = 0;
                            }
                        }
                    }
                }
            }
        }
    }
    if (!FILL) {
        if ((ci & 31) != 0 && (ci >> 5) < cap_words) mrow[ci >> 5] = word;   // the last, partial word
        rowcnt[x] = cnt;
        ncand[x] = ci < INT32_MAX ? (int32_t)ci : INT32_MAX;
    }
}

__global__ void k_copy_count(int64_t n_gh, const int32_t *__restrict__ owner, int32_t *__restrict__ cnt) {
    int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi < n_gh) atomicAdd(&cnt[owner[gi]], 1);
}

__global__ void k_copy_fill(int64_t n_gh, const int32_t *__restrict__ owner, const int64_t *__restrict__ start,
                            int32_t *__restrict__ cursor, int32_t *__restrict__ idx) {
    int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n_gh) return;
    int32_t o = owner[gi];
    idx[start[o] + atomicAdd(&cursor[o], 1)] = (int32_t)gi;
}

__global__ void k_i64_to_i32(const int64_t *__restrict__ a, int32_t *__restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (int32_t)a[i];
}

// Bounds of the wrapped positions (needed along open axes only): per-block minima and maxima of
// the three coordinates over a grid-strided share of the atoms (stride = blocks x 256), then
// one block combines the blocks' values.  Min and max do not depend on the order.
constexpr int kMinmaxBlocks = 256;

__global__ __launch_bounds__(256) void k_minmax_part(int64_t n, const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double smin[3][256], smax[3][256];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        for (int a = 0; a < 3; ++a) {
            double v = w[3 * i + a];
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
        }
    for (int a = 0; a < 3; ++a) { smin[a][threadIdx.x] = mn[a]; smax[a][threadIdx.x] = mx[a]; }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + s]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) { part[6 * blockIdx.x + a] = smin[a][0]; part[6 * blockIdx.x + 3 + a] = smax[a][0]; }
}

__global__ __launch_bounds__(256) void k_minmax(int nb, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double smin[3][256], smax[3][256];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int a = 0; a < 3; ++a) {
            mn[a] = fmin(mn[a], part[6 * b + a]);
            mx[a] = fmax(mx[a], part[6 * b + 3 + a]);
        }
    for (int a = 0; a < 3; ++a) { smin[a][threadIdx.x] = mn[a]; smax[a][threadIdx.x] = mx[a]; }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + s]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) { out[a] = smin[a][0]; out[3 + a] = smax[a][0]; }
}

__global__ void k_xref(int64_t n, const double *__restrict__ pos, const int32_t *__restrict__ perm,
                       double *__restrict__ xref) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t u = perm[i];
    for (int a = 0; a < 3; ++a) xref[3 * i + a] = pos[3 * u + a];
}

// ---------------------------------------------------------------------- scan --

__global__ void k_scan_block(int64_t *__restrict__ d, int64_t n, int64_t *__restrict__ sums) {
    __shared__ int64_t s[1024];
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int64_t v = i < n ? d[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) d[i] = s[threadIdx.x] - v;   // exclusive
    if (threadIdx.x == 1023) sums[blockIdx.x] = s[1023];
}

__global__ void k_scan_add(int64_t *__restrict__ d, int64_t n, const int64_t *__restrict__ sums) {
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) d[i] += sums[blockIdx.x];
}

static void scan_rec(hipStream_t st, int64_t *d, int64_t n, int64_t *tmp) {
    int64_t nb = (n + 1023) / 1024;
    int64_t *sums = tmp;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(1024), 0, st, d, n, sums);
    LAUNCH_OK("k_scan_block");
    if (nb > 1) {
        scan_rec(st, sums, nb, tmp + nb + 1);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(1024), 0, st, d, n, sums);
        LAUNCH_OK("k_scan_add");
    }
}

// d holds n counts in [0, n); on return d[0..n] are exclusive offsets, d[n] = total.  Enqueued
// only: the total stays on the device.
static void scan_exclusive_async(hipStream_t st, int64_t *d, int64_t n, DevBuf &tmp) {
    // last element + its count = total: scan n+1 values where d[n] was set to 0 by the caller
    int64_t m = n + 1;
    int64_t need = 0, k = m;
    while (k > 1) { k = (k + 1023) / 1024; need += k + 1; }
    int64_t *t = static_cast<int64_t *>(tmp.ensure((size_t)(need + 16) * sizeof(int64_t)));
    scan_rec(st, d, m, t);
}

int64_t scan_exclusive_i64(hipStream_t st, int64_t *d, int64_t n, DevBuf &tmp) {
    scan_exclusive_async(st, d, n, tmp);
    int64_t total = 0;
    HIP_OK(hipMemcpyAsync(&total, d + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return total;
}

// Scattered device scalars the host needs (counts for allocation sizes, bounds, check flags),
// gathered by one tiny kernel into one block and read with one copy: every read is a wait for
// the stream, which behind other streams' work sharing a hardware queue can take far longer
// than the work itself.
constexpr int kPickMax = 160;
struct Pick {
    const void *p[kPickMax];
    int8_t is32[kPickMax];   // 1: int32 (sign-extended); 0: eight bytes (int64, or a double's bits)
    int n;
};

__global__ void k_pick(Pick pk, int64_t *__restrict__ out) {
    for (int t = threadIdx.x; t < pk.n; t += blockDim.x)
        out[t] = pk.is32[t] ? (int64_t) * static_cast<const int32_t *>(pk.p[t]) : *static_cast<const int64_t *>(pk.p[t]);
}

struct Picker {
    Pick pk{};
    int add(const void *p, bool is32) {
        if (pk.n >= kPickMax) fail(REANN_E_UNSUPPORTED, "neighbour build: too many values to read back");
        pk.p[pk.n] = p;
        pk.is32[pk.n] = is32 ? 1 : 0;
        return pk.n++;
    }
    // enqueue the gather, copy to `host` and wait
    void read(hipStream_t st, DevBuf &dev, int64_t *host) {
        int64_t *d = static_cast<int64_t *>(dev.ensure(kPickMax * sizeof(int64_t)));
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(128), 0, st, pk, d);
        LAUNCH_OK("k_pick");
        HIP_OK(hipMemcpyAsync(host, d, pk.n * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
    }
};

// --------------------------------------------------------------------- build --

void build_nlist(hipStream_t st, const double *d_pos, const int32_t *d_species, int64_t n, int n_species,
                 const Geom &g, double r_c, double skin, NList &nl, NListScratch &s, bool ghosts_by_species,
                 bool defer_check) {
    if (n <= 0) fail(REANN_E_INVALID, "n must be > 0");
    if (n >= (int64_t)1 << 30) fail(REANN_E_UNSUPPORTED, "too many atoms");
    const int B = 256;
    nl.g = g;
    nl.n = n;
    nl.n_species = n_species;
    nl.skin = skin;
    nl.r_c = r_c;
    double *w = static_cast<double *>(s.a.ensure(n * 3 * sizeof(double)));
    int32_t *q = nl.q.resize(n * 3);
    int32_t *dom = static_cast<int32_t *>(s.b.ensure(n * sizeof(int32_t)));
    int64_t *goff = static_cast<int64_t *>(s.c.ensure((n + 1) * sizeof(int64_t)));
    int32_t *bad = static_cast<int32_t *>(s.i.ensure(64));
    HIP_OK(hipMemsetAsync(goff + n, 0, sizeof(int64_t), st));
    HIP_OK(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_wrap_count, dim3(grid_for(n, B)), dim3(B), 0, st, g, n, d_pos, w, q, dom, goff, bad);
    LAUNCH_OK("k_wrap_count");
    scan_exclusive_async(st, goff, n, s.m);
    // the bounds of the wrapped locals set the bins along open axes only
    const bool open_axis = !(g.per[0] && g.per[1] && g.per[2]);
    double *d_mm = static_cast<double *>(s.mm.ensure((6 + 6 * kMinmaxBlocks) * sizeof(double)));
    if (open_axis) {
        const int nb = (int)std::min<int64_t>(kMinmaxBlocks, (n + 255) / 256);
        hipLaunchKernelGGL(k_minmax_part, dim3(nb), dim3(256), 0, st, n, w, d_mm + 6);
        LAUNCH_OK("k_minmax_part");
        hipLaunchKernelGGL(k_minmax, dim3(1), dim3(256), 0, st, nb, d_mm + 6, d_mm);
        LAUNCH_OK("k_minmax");
    }
    // first read: ghost count, the invalid-position flag and (open axes) the bounds
    int64_t hv[kPickMax];
    double bb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    {
        Picker pk;
        pk.add(goff + n, false);
        pk.add(bad, true);
        if (open_axis)
            for (int a = 0; a < 6; ++a) pk.add(d_mm + a, false);
        pk.read(st, s.chk, hv);
        if (open_axis) std::memcpy(bb, hv + 2, sizeof bb);
    }
    check_deferred(s);   // a previous build's deferred check (the wait above covered its copy)
    const int64_t n_gh = hv[0];
    if (hv[1]) fail(REANN_E_INVALID, "positions contain NaN, Inf or |x| >= 1e9");
    if (n + n_gh >= ((int64_t)1 << 31) - 1) fail(REANN_E_UNSUPPORTED, "extended system too large");
    nl.n_gh = n_gh;
    nl.n_ext = n + n_gh;
    const int64_t n_ext = nl.n_ext;
    int32_t *g_owner = static_cast<int32_t *>(s.d.ensure((n_gh + 1) * sizeof(int32_t)));
    int32_t *g_shift = static_cast<int32_t *>(s.e.ensure((n_gh + 1) * 3 * sizeof(int32_t)));
    int32_t *g_dom = static_cast<int32_t *>(s.f.ensure((n_gh + 1) * sizeof(int32_t)));
    double *g_pos = static_cast<double *>(s.g.ensure((n_gh + 1) * 3 * sizeof(double)));
    hipLaunchKernelGGL(k_ghost_gen, dim3(grid_for(n, B)), dim3(B), 0, st, g, n, w, dom, goff, g_owner, g_shift, g_dom,
                       g_pos);
    LAUNCH_OK("k_ghost_gen");

    // spatial bins of size >= r_c + skin over the region holding every copy
    Bins b{};
    b.nbin = 1;
    for (int a = 0; a < 3; ++a) {
        double lo = g.per[a] ? -g.shell : bb[a];
        double hi = g.per[a] ? g.L[a] + g.shell : bb[3 + a];
        double ext = hi - lo;
        if (!(ext >= 0.0 && ext < 1e8)) fail(REANN_E_INVALID, "system extent out of range");
        int nb = (int)std::floor(ext / (g.rcut * 1.000000001));
        nb = std::max(1, std::min(nb, 1024));
        b.nb[a] = nb;
        b.mn[a] = lo;
        b.bs[a] = nb > 1 ? ext / nb : 1.0;
        b.nbin *= nb;
    }
    const int nghs = ghosts_by_species ? n_species : 1;   // ghost key slots
    const int64_t nkeys = (int64_t)(n_species + nghs) * g.ndom * b.nbin;
    if (nkeys > ((int64_t)1 << 28)) fail(REANN_E_UNSUPPORTED, "bin table too large");

    int64_t *key = static_cast<int64_t *>(s.h.ensure(n_ext * sizeof(int64_t)));
    int32_t *cnt32 = static_cast<int32_t *>(s.i.ensure((nkeys + 1) * sizeof(int32_t)));
    int64_t *kstart = static_cast<int64_t *>(s.j.ensure((nkeys + 1) * sizeof(int64_t)));
    HIP_OK(hipMemsetAsync(cnt32, 0, (nkeys + 1) * sizeof(int32_t), st));
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n_ext, B)), dim3(B), 0, st, b, g.ndom, n_species, n, n_gh, w, dom,
                       d_species, g_pos, g_dom, g_owner, ghosts_by_species ? 1 : 0, key, cnt32);
    LAUNCH_OK("k_keys");
    hipLaunchKernelGGL(k_i32_to_i64, dim3(grid_for(nkeys + 1, B)), dim3(B), 0, st, cnt32, kstart, nkeys + 1);
    LAUNCH_OK("k_i32_to_i64");
    // every ext atom adds one to exactly one key, so the total is n_ext by construction; it is
    // read back (and checked) with the pair count below
    scan_exclusive_async(st, kstart, nkeys, s.m);
    int32_t *order = static_cast<int32_t *>(s.k.ensure(n_ext * sizeof(int32_t)));
    HIP_OK(hipMemsetAsync(cnt32, 0, (nkeys + 1) * sizeof(int32_t), st));
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n_ext, B)), dim3(B), 0, st, n_ext, key, kstart, cnt32, order);
    LAUNCH_OK("k_scatter");
    hipLaunchKernelGGL(k_sort_segments, dim3(grid_for(nkeys, 4)), dim3(256), 0, st, nkeys, kstart, order);
    LAUNCH_OK("k_sort_segments");

    int32_t *perm = nl.perm.resize(n);
    int32_t *inv_perm = nl.inv_perm.resize(n);
    double *pext = static_cast<double *>(s.l.ensure(3 * n_ext * sizeof(double)));
    int32_t *d_dom_ext = static_cast<int32_t *>(s.dext.ensure(n_ext * sizeof(int32_t)));
    int32_t *d_bin_ext = static_cast<int32_t *>(s.bext.ensure(n_ext * sizeof(int32_t)));
    int32_t *gh_owner_user = static_cast<int32_t *>(s.gou.ensure((n_gh + 1) * sizeof(int32_t)));
    int8_t *spec_ext = nl.spec_ext.resize(n_ext);
    int32_t *gh_shift = nl.gh_shift.resize((n_gh + 1) * 3);
    hipLaunchKernelGGL(k_build_ext, dim3(grid_for(n_ext, B)), dim3(B), 0, st, b, n, n_ext, order, w, dom, d_species,
                       g_pos, g_dom, g_owner, g_shift, perm, inv_perm, pext, d_dom_ext, d_bin_ext, spec_ext,
                       gh_owner_user, gh_shift);
    LAUNCH_OK("k_build_ext");
    int32_t *gh_owner = nl.gh_owner.resize(n_gh + 1);
    if (n_gh > 0) {
        hipLaunchKernelGGL(k_ghost_owner, dim3(grid_for(n_gh, B)), dim3(B), 0, st, n_gh, gh_owner_user, inv_perm,
                           gh_owner);
        LAUNCH_OK("k_ghost_owner");
    }

    // rows: count (keeping the hits), scan, fill.  A bin holds about n_ext / nbin atoms (a
    // subdomain's atoms fill about its own share of the bins), so a row has about
    // 27 n_ext / nbin candidates; the hits are kept for up to about twice that (as bits per
    // candidate, or one word per 32-atom chunk of a key).  Keys of 24 or more atoms on average
    // take a half-wave per row, smaller ones a thread per row.
    int64_t *row = nl.row.resize(n_ext + 1);
    HIP_OK(hipMemsetAsync(row + n_ext, 0, sizeof(int64_t), st));
    int32_t *coinc = static_cast<int32_t *>(s.coinc.ensure(64));
    HIP_OK(hipMemsetAsync(coinc, 0, sizeof(int32_t), st));
    const double per_bin = (double)n_ext / (double)b.nbin, mean_cand = 27.0 * per_bin;
    const bool group = per_bin / n_species >= 24.0;
    const double words = std::ceil(2.0 * mean_cand / 32.0) + 2.0 + (group ? 27.0 * (n_species + nghs) : 0.0);
    const int cap_words = (int)std::min<double>(4096.0, words);
    uint32_t *mask = static_cast<uint32_t *>(s.mask.ensure((size_t)n_ext * cap_words * sizeof(uint32_t)));
    int32_t *nkept = static_cast<int32_t *>(s.ncand.ensure((size_t)n_ext * sizeof(int32_t)));
    if (group)
        hipLaunchKernelGGL(k_rows_group<false>, dim3(grid_for(n_ext, kRowsPerBlk)), dim3(256), 0, st, b, g, n_species,
                           nghs, n, n_ext, pext, d_dom_ext, d_bin_ext, kstart, row, nullptr, nullptr, coinc, mask, nkept,
                           cap_words);
    else
        hipLaunchKernelGGL(k_rows_thread<false>, dim3(grid_for(n_ext, 128)), dim3(128), 0, st, b, g, n_species, nghs, n,
                           n_ext, pext, d_dom_ext, d_bin_ext, kstart, row, nullptr, nullptr, coinc, mask, nkept, cap_words);
    LAUNCH_OK("k_rows<count>");
    scan_exclusive_async(st, row, n_ext, s.m);
    // second read: pair counts, the key total and the species segments of the locals
    {
        Picker pk;
        pk.add(row + n_ext, false);
        pk.add(row + n, false);
        pk.add(kstart + nkeys, false);
        pk.add(coinc, true);
        for (int sp = 0; sp <= n_species; ++sp) pk.add(kstart + (int64_t)sp * g.ndom * b.nbin, false);
        if (ghosts_by_species)
            for (int sp = 1; sp <= n_species; ++sp) pk.add(kstart + (int64_t)(n_species + sp) * g.ndom * b.nbin, false);
        pk.read(st, s.chk, hv);
    }
    const int64_t n_pairs = hv[0];
    if (hv[2] != n_ext) fail(REANN_E_DEVICE, "neighbour build: key count mismatch");
    if (hv[3]) fail(REANN_E_INVALID, "two atoms (or an atom and a periodic copy) closer than 1e-6 A");
    nl.seg.assign(hv + 4, hv + 4 + n_species + 1);
    // ghost species segments: [gseg[s], gseg[s+1]) are the ghosts of element s (ghosts_by_species),
    // else one segment of every ghost
    if (ghosts_by_species) {
        nl.gseg.assign(1, n);
        nl.gseg.insert(nl.gseg.end(), hv + 4 + n_species + 1, hv + 4 + 2 * n_species + 1);
    } else {
        nl.gseg = {n, n_ext};
    }
    if (nl.gseg.back() != n_ext) fail(REANN_E_DEVICE, "neighbour build: ghost segments mismatch");
    if (nl.seg[n_species] != n) fail(REANN_E_DEVICE, "neighbour build: species segments mismatch");
    if (n_pairs >= ((int64_t)1 << 31) - 1) fail(REANN_E_UNSUPPORTED, "too many neighbour pairs");
    nl.n_pairs = n_pairs;
    nl.n_local_pairs = hv[1];
    int32_t *col = nl.col.resize(n_pairs + 1);
    if (group)
        hipLaunchKernelGGL(k_rows_group<true>, dim3(grid_for(n_ext, kRowsPerBlk)), dim3(256), 0, st, b, g, n_species,
                           nghs, n, n_ext, pext, d_dom_ext, d_bin_ext, kstart, nullptr, row, col, nullptr, mask, nkept,
                           cap_words);
    else
        hipLaunchKernelGGL(k_rows_thread<true>, dim3(grid_for(n_ext, 128)), dim3(128), 0, st, b, g, n_species, nghs, n,
                           n_ext, pext, d_dom_ext, d_bin_ext, kstart, nullptr, row, col, nullptr, mask, nkept, cap_words);
    LAUNCH_OK("k_rows<fill>");
    // the rows are ascending as filled; the reverse slot of every entry
    {
        int32_t *rev = nl.rev.resize(n_pairs + 1);
        int32_t *flag = static_cast<int32_t *>(s.flag.ensure(64));
        HIP_OK(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
        HIP_OK(hipMemsetAsync(rev, 0xff, (n_pairs + 1) * sizeof(int32_t), st));   // -1: not resolved
        hipLaunchKernelGGL(k_reverse, dim3(grid_for(n_ext * 16, B)), dim3(B), 0, st, n_ext, row, col, rev, flag);
        LAUNCH_OK("k_reverse");
        if (n_pairs > 0) {
            hipLaunchKernelGGL(k_reverse_check, dim3(grid_for(n_pairs, B)), dim3(B), 0, st, n_pairs, rev, flag);
            LAUNCH_OK("k_reverse_check");
        }
    }

    // owner -> ghost copies
    int32_t *copy_ptr = nl.copy_ptr.resize(n + 1);
    int32_t *copy_idx = nl.copy_idx.resize(n_gh + 1);
    {
        int32_t *c32 = static_cast<int32_t *>(s.i.ensure((n + 1) * sizeof(int32_t)));
        int64_t *c64 = static_cast<int64_t *>(s.j.ensure((n + 1) * sizeof(int64_t)));
        HIP_OK(hipMemsetAsync(c32, 0, (n + 1) * sizeof(int32_t), st));
        if (n_gh > 0) {
            hipLaunchKernelGGL(k_copy_count, dim3(grid_for(n_gh, B)), dim3(B), 0, st, n_gh, gh_owner, c32);
            LAUNCH_OK("k_copy_count");
        }
        hipLaunchKernelGGL(k_i32_to_i64, dim3(grid_for(n + 1, B)), dim3(B), 0, st, c32, c64, n + 1);
        LAUNCH_OK("k_i32_to_i64");
        scan_exclusive_async(st, c64, n, s.m);
        hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(n + 1, B)), dim3(B), 0, st, c64, copy_ptr, n + 1);
        LAUNCH_OK("k_i64_to_i32");
        if (n_gh > 0) {
            HIP_OK(hipMemsetAsync(c32, 0, (n + 1) * sizeof(int32_t), st));
            hipLaunchKernelGGL(k_copy_fill, dim3(grid_for(n_gh, B)), dim3(B), 0, st, n_gh, gh_owner, c64, c32, copy_idx);
            LAUNCH_OK("k_copy_fill");
            hipLaunchKernelGGL(k_sort_segments32, dim3(grid_for(n, B)), dim3(B), 0, st, n, copy_ptr, copy_idx);
            LAUNCH_OK("k_sort_segments32");
        }
    }
    double *xref = nl.xref.resize(n * 3);
    hipLaunchKernelGGL(k_xref, dim3(grid_for(n, B)), dim3(B), 0, st, n, d_pos, perm, xref);
    LAUNCH_OK("k_xref");
    // last read (the list is complete when it returns): the symmetry check of the reverse slots
    if (defer_check) {
        HIP_OK(hipMemcpyAsync(s.sym.get(), s.flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        s.sym_pending = true;
        return;
    }
    {
        Picker pk;
        pk.add(s.flag.p, true);
        pk.read(st, s.chk, hv);
    }
    if (hv[0]) fail(REANN_E_DEVICE, "neighbour build: list is not symmetric");
}

void check_deferred(NListScratch &s) {
    if (!s.sym_pending) return;
    s.sym_pending = false;
    if (*s.sym.get()) fail(REANN_E_DEVICE, "neighbour build: list is not symmetric");
}

// ------------------------------------------------------------ per-step work --

__global__ void k_refresh(Geom g, int64_t n, int64_t n_ext, const double *__restrict__ pos, const int32_t *__restrict__ perm,
                          const int32_t *__restrict__ q, const int32_t *__restrict__ gh_owner,
                          const int32_t *__restrict__ gh_shift, double4 *__restrict__ p4) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_ext) return;
    int64_t i = x < n ? x : gh_owner[x - n];
    int64_t u = perm[i];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        double v = pos[3 * u + a];
        if (g.per[a]) {
            double t = (double)q[3 * u + a] * g.L[a];   // q is stored per caller index
            v = v - t;
        }
        w[a] = v;
    }
    if (x >= n) {
        int64_t gi = x - n;
        for (int a = 0; a < 3; ++a)
            if (g.per[a]) w[a] = w[a] + (double)gh_shift[3 * gi + a] * g.L[a];
    }
    p4[x] = make_double4(w[0], w[1], w[2], 0.0);
}

void refresh_positions(hipStream_t st, const NList &nl, const double *d_pos, double4 *p4) {
    hipLaunchKernelGGL(k_refresh, dim3(grid_for(nl.n_ext, 256)), dim3(256), 0, st, nl.g, nl.n, nl.n_ext, d_pos,
                       nl.perm.ptr(), nl.q.ptr(), nl.gh_owner.ptr(), nl.gh_shift.ptr(), p4);
    LAUNCH_OK("k_refresh");
}

__device__ inline double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

// Per-block maxima of |x_i - xref_i|^2 (NaN counts as too far), then one block combines them.
__global__ void k_maxdisp_part(int64_t n, const double *__restrict__ pos, const int32_t *__restrict__ perm,
                               const double *__restrict__ xref, double *__restrict__ part) {
    __shared__ double sm[256];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = perm[i];
        const double dx = pos[3 * u] - xref[3 * i], dy = pos[3 * u + 1] - xref[3 * i + 1],
                     dz = pos[3 * u + 2] - xref[3 * i + 2];
        m = nan_max(m, dx * dx + dy * dy + dz * dz);
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = nan_max(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_maxdisp_final(int nb, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double sm[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) m = nan_max(m, part[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = nan_max(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sm[0];
}

// d_out must hold 1 + 1024 doubles (result, then per-block partials).
void max_displacement2(hipStream_t st, const NList &nl, const double *d_pos, double *d_out) {
    const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nl.n + 255) / 256));
    hipLaunchKernelGGL(k_maxdisp_part, dim3(nb), dim3(256), 0, st, nl.n, d_pos, nl.perm.ptr(), nl.xref.ptr(),
                       d_out + 1);
    LAUNCH_OK("k_maxdisp_part");
    hipLaunchKernelGGL(k_maxdisp_final, dim3(1), dim3(256), 0, st, nb, d_out + 1, d_out);
    LAUNCH_OK("k_maxdisp_final");
}

}  // namespace reann
