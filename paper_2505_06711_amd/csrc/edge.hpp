// Edge passes of one MP layer (Sec. 2.1 Eq. (1) inner sum, and its adjoint, Eqs. (3)-(5))
// plus the per-layer ghost exchange (Sec. 2.2): gather of messages, reduction of adjoints.
#pragma once

#include "common.hpp"

namespace reann {

struct EdgeConsts {
    double centres[16];
    double alphas[16];
    double alphas2[16];   // alphas * log2(e): the FP32 kernels evaluate exp(-a x^2) as 2^(-a2 x^2)
    double r_c;
    double rc2;       // r_c^2 in FP64: in-cutoff test of a list entry
    double ang_scale;
};

struct EdgeArgs {
    int64_t n, n_ext;
    const int64_t *row;
    const int32_t *col;
    const double4 *p4;   // ext positions (x, y, z, 0)
};

// In-cutoff entries of the list for the current positions (same slot ranges as the list):
// row x's in-cutoff local neighbours at col[row[x] .. row[x] + nloc[x]), its in-cutoff
// ghost neighbours at col[row[x+1] - ngh[x] .. row[x+1]).
// fslot[s]: the list slot of the entry compacted into s; cpos[f]: the compacted slot of the
// in-cutoff list entry f; rev: the list's reverse slots; rslot[s] (for the in-cutoff local
// neighbours of each row, filled by the step's first adjoint gather): the compacted slot of
// the reverse of entry s.
struct CutList {
    const int64_t *row;
    int32_t *col;
    int32_t *nloc, *ngh;
    int32_t *fslot, *cpos, *rslot;
    const int32_t *rev;
};
void compact_cutoff(hipStream_t st, const EdgeArgs &a, double r_c, CutList &cl);

// S[i][lambda][m] for the n local rows.  c: messages of all ext atoms, [n_ext][K].
void edge_forward(hipStream_t st, bool fp64, int L, int K, const EdgeArgs &a, const CutList &cl, const EdgeConsts &ec,
                  const void *c, void *S);

// Atomics-free adjoint of one layer in two launches.  Centre role (local rows): evaluates
// every in-cutoff edge once, adds its gradient to F of the centre and the virial, and
// writes at the edge's compacted slot the record of what it gives the neighbour end.
// Neighbour role (every ext row): sums the records of the row's incoming edges through
// rslot.
//   Sbar [n][NL][K] (locals), c [n_ext][K]; F [n_ext][3] is accumulated;
//   cbar [n_ext][K] is overwritten when want_cbar; Wpart receives one FP64 [9] per block
// of the centre-role launch (the return value is that block count); rec holds
// edge_record_elems(K) working-type values per (compacted) list slot.
int edge_adjoint_centre(hipStream_t st, bool fp64, int L, int K, const EdgeArgs &a, const CutList &cl,
                        const EdgeConsts &ec, const void *c, const void *Sbar, bool want_cbar, void *F, double *Wpart,
                        void *rec);
// make_rslot: the first gather after compact_cutoff (fills rslot; later gathers read it).
void edge_adjoint_gather(hipStream_t st, bool fp64, int K, const EdgeArgs &a, const CutList &cl, bool want_cbar,
                         bool make_rslot, const void *rec, void *F, void *cbar);
// Values per edge record: the edge gradient (3, padded to 4) and K adjoint-message terms.
inline int edge_record_elems(int K) { return 4 + K; }
int edge_backward_blocks(int64_t n_ext);

// c[n + g][:] = c[owner[g]][:]
void ghost_gather(hipStream_t st, bool fp64, int64_t n, int64_t n_gh, int K, const int32_t *owner, void *c);
// v[o][:] += sum over ghost copies g of o of v[n + g][:], in increasing g
void ghost_reduce(hipStream_t st, bool fp64, int64_t n, int width, const int32_t *copy_ptr, const int32_t *copy_idx,
                  void *v);
// c^0 of every ext atom from its species
void init_messages(hipStream_t st, bool fp64, int64_t n_ext, int K, const int8_t *spec, const void *c0, void *c);

}  // namespace reann
