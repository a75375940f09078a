// Host layout builder for libsccs: validation of an SCCS problem and the
// index structures the persistent CCD kernel walks.
//
// Ownership.  The G persistent workgroups each own a contiguous patient range
// [pb[b], pb[b+1]) (balanced by era count), for every column.  All state of a
// patient (den_i) and of its eras (w_k) is only ever read or written by its
// owner, so consecutive coordinates need no device-wide synchronisation
// beyond the reduction of the two partial sums of Eqs. 7 and 9.
//
// Column groups.  Consecutive columns that share no patient are independent
// coordinates: the Newton step of one does not depend on the update of the
// other (the update of column j changes only the state of column j's
// patients), so a run of such columns can be visited with ONE device-wide
// reduction carrying all their partial sums, with results identical to
// visiting them one by one.  Columns are cut greedily, in order, into groups
// of at most max_group pairwise patient-disjoint columns (gcol[g] is the
// first column of group g).  max_group = 1 gives one column per group.
//
// Tiles.  The nonzeros of a group (compressed column storage, Section 2.4
// "Representation in Memory") are reordered group by group, then by owning
// workgroup, then column by column in CSC order, and cut into tiles of at
// most tile_nnz entries -- one wavefront each -- that hold whole (column,
// patient) segments and never straddle an ownership boundary.  A segment
// longer than tile_nnz gets a tile of its own (a "long" tile, walked in
// 64-wide chunks).  Tile t is [tile_start[t], tile_start[t+1]) of that
// order.  own[g*(G+1) + b] is the first tile of group g owned by workgroup
// b; own[g*(G+1) + G] closes group g.  rp[e] = (row, patient | c << 28)
// with c the column's index within its group.
//
// Pass descriptors.  gdesc[g] packs what the sweep needs to decide, at run
// time, whether group g can join a pass that starts with earlier groups (see
// sccs_kernels.hpp): g's first column j0 (bits 0-12), its width (bits
// 13-15) and a link mask (kLinkCols bits from bit 16) whose bit i is set
// when column j0 - kLinkCols + i (>= 0) shares a patient with some column of
// g.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "sccs.h"
#include "sccs_limits.hpp"

namespace sccs {


struct Layout {
  int32_t N = 0, J = 0, G = 0, tile_nnz = kTile;
  int64_t K = 0, nnz = 0;
  int64_t tiles_cap = 0;            // workspace room for tile_start (>= tiles + 1)
  std::vector<int32_t> pb;          // [G+1] patient bounds per workgroup
  std::vector<uint32_t> rp;         // [2*nnz] (row, patient) per nonzero, CSC order
  std::vector<int32_t> tile_start;  // [T+1]
  std::vector<int32_t> own;         // [n_groups*(G+1)]
  int32_t n_groups = 0;
  std::vector<int32_t> gcol;        // [n_groups+1] first column of each group
  std::vector<uint32_t> gdesc;      // [n_groups] pass descriptors
  std::vector<int32_t> pptr;        // [N+1] patient_ptr as int32
  std::vector<int32_t> era_ptr;     // [K+1] compressed row storage of X
  std::vector<int32_t> era_col;     // [nnz]
  std::vector<double> val;          // [nnz] covariate values in rp order (empty: binary)
  std::vector<double> era_val;      // [nnz] covariate values in era_col order (empty: binary)
  int32_t n_tiles() const { return (int32_t)tile_start.size() - 1; }
  int32_t max_tiles_per_wg = 0;     // over all (column, workgroup) pairs
};

// Check every rule stated for sccs_problem.  Returns SCCS_OK or
// SCCS_ERR_INVALID_ARG with a message in err.
sccs_status validate_problem(const sccs_problem* p, std::string& err);

// Upper bound on the number of tiles (see the .cpp for the argument), so
// that workspace sizes can be computed without building the layout.
int64_t tile_bound(int64_t nnz, int32_t J, int32_t G, int32_t tile_nnz);

// Dimensions only (vectors empty): enough to size the workspace.
inline void layout_dims(const sccs_problem* p, int32_t G, int32_t tile_nnz, Layout& L) {
  L.N = p->n_patients; L.J = p->n_cols; L.G = G; L.K = p->n_rows; L.nnz = p->nnz; L.tile_nnz = tile_nnz;
  L.tiles_cap = tile_bound(p->nnz, p->n_cols, G, tile_nnz) + 1;
}

// Build the layout for G workgroups, tiles of at most tile_nnz nonzeros
// (except single-segment tiles) and column groups of at most max_group
// columns.  The problem must have been validated.
void build_layout(const sccs_problem* p, int32_t G, Layout& L, int32_t tile_nnz = kTile, int32_t max_group = 1);

// Relabelling of the columns for independent coordinates.  Columns are
// visited in decreasing order of nonzeros (ties: smaller index first); each
// joins the first group, in creation order, that has fewer than width
// columns and shares no patient with it, or else opens a new group at the
// end.  order[k] is the column that takes position k: the groups in creation
// order, each group's columns in the order they joined.  Algorithm 1 visits
// coordinates in a fixed cyclic order; which drug is numbered first is the
// caller's choice, and under this numbering consecutive runs of pairwise
// patient-disjoint columns (column groups) are long.
void independent_order(const sccs_problem* p, int32_t width, std::vector<int32_t>& order);

// Copy of a problem with its columns in the order given (column k of the
// copy is column order[k] of src); row-indexed arrays are shared with src.
struct PermutedProblem {
  sccs_problem p{};
  std::vector<int64_t> col_ptr;
  std::vector<int32_t> row_idx;
  std::vector<double> value;
};
void permute_columns(const sccs_problem* src, const std::vector<int32_t>& order, PermutedProblem& out);

// Y'X_j with patient weights (NULL = 1), summed on the host in compressed
// column order; for binary problems the terms are integers, so the sum is
// exact in any order.
void host_ytx(const sccs_problem* p, const int32_t* weight, std::vector<double>& ytx);

}  // namespace sccs
