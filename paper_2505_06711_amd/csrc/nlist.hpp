// Neighbour list of the subdomain-extended system (Sec. 2.2): locals of every subdomain,
// their ghost copies, and one CSR list for cutoff r_c + skin that every MP layer reuses.
#pragma once

#include "common.hpp"

namespace reann {

constexpr int kMaxSplit = 16;   // subdomains per axis

struct Geom {
    double L[3];
    int per[3];
    int P[3];
    double lo[3][kMaxSplit], hi[3][kMaxSplit];
    double rcut, rc2, shell;
    int nm[3];
    int ndom;
};

// Extended-atom layout: [0, n) are the local atoms of all subdomains, ordered by
// (species, subdomain, spatial bin, caller index); [n, n_ext) are the ghost copies,
// ordered by (subdomain, spatial bin, generation order), or with ghosts_by_species by
// (species, subdomain, spatial bin, generation order).  Rows of locals list every
// ext atom of the same subdomain within r_c + skin; rows of ghosts list only the
// locals of their subdomain within r_c + skin (used by the atomics-free backward).
// Every row is sorted ascending, so its locals come before its ghosts.
struct NList {
    Geom g{};
    int64_t n = 0, n_gh = 0, n_ext = 0, n_pairs = 0, n_local_pairs = 0;
    int n_species = 0;
    double skin = 0, r_c = 0;
    std::vector<int64_t> seg;    // host: species segments over the locals, [n_species + 1]
    std::vector<int64_t> gseg;   // host: species segments over the ghosts ([n, n_ext) if not by species)
    DArr<int32_t> perm;          // [n]   local -> caller index
    DArr<int32_t> inv_perm;      // [n]   caller -> local index
    DArr<int32_t> q;             // [n*3] integer wrap per axis, caller order: w = x - q L
    DArr<int32_t> gh_owner;      // [n_gh] local index of the owner
    DArr<int32_t> gh_shift;      // [n_gh*3] lattice shift of the copy
    DArr<int32_t> copy_ptr;      // [n+1]  owner -> its ghost copies (CSR)
    DArr<int32_t> copy_idx;      // [n_gh] ghost indices in increasing order per owner
    DArr<int64_t> row;           // [n_ext+1]
    DArr<int32_t> col;           // [n_pairs] ext indices
    DArr<int32_t> rev;           // [n_pairs] slot of the reverse entry (j -> x) of entry (x -> j)
    DArr<int8_t> spec_ext;       // [n_ext]
    DArr<double> xref;           // [n*3] caller positions at build time, local order
};

// Scratch reused between builds.
struct NListScratch {
    DevBuf a, b, c, d, e, f, g, h, i, j, k, l, m, flag, mm, chk, dext, bext, gou, coinc, mask, ncand;
    PinnedWord sym;             // deferred symmetry check: the flag, copied back
    bool sym_pending = false;
};

void geom_init(Geom &g, const double cell[9], const int32_t pbc[3], const int32_t P[3], double r_c, double skin);

// d_pos: device FP64 [n][3] (caller order); d_species: device int32 [n].  The build reads its
// counts back in two waits; a third waits for the end of the build and checks that every entry
// has its reverse.  defer_check: that last check is copied back with the build instead, and
// read by check_deferred after the caller has waited for the stream for other reasons.
void build_nlist(hipStream_t st, const double *d_pos, const int32_t *d_species, int64_t n, int n_species,
                 const Geom &g, double r_c, double skin, NList &nl, NListScratch &s, bool ghosts_by_species = false,
                 bool defer_check = false);
// REANN_E_DEVICE if a deferred check failed (the stream of the build must have been waited for).
void check_deferred(NListScratch &s);

// Exclusive scan of n int64 values in place; returns the total (synchronises).
int64_t scan_exclusive_i64(hipStream_t st, int64_t *d, int64_t n, DevBuf &tmp);

// Positions of the extended system from caller positions: w_i = x_{perm i} - q_i L for
// locals, owner position + shift L for ghosts.  SoA output px/py/pz [n_ext].
// Wrapped positions of all ext atoms (locals then ghost copies) as (x, y, z, 0), one 32-byte
// record per atom so that a neighbour's position is a single cache line.
void refresh_positions(hipStream_t st, const NList &nl, const double *d_pos, double4 *p4);

// max_i |x_i - xref_i|^2 over locals -> d_out[0]; d_out holds 1 + 1024 doubles (partials after it).
void max_displacement2(hipStream_t st, const NList &nl, const double *d_pos, double *d_out);

}  // namespace reann
