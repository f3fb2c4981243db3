// Internal data structures shared by the host analysis, the launch code and
// the C ABI.  Not installed; the public interface is include/pexsi_hip.h.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pxs {

// Pole table (poles.cpp).  shifts_ri: 2*P doubles, weights_ri: 2*nsets*P.
int pole_table(double beta, double dE, double mu, int P, int nsets, double* shifts_ri,
               double* weights_ri);

struct Panel {
  int32_t J;   // supernode
  int32_t p0;  // first column, as a position in the supernode's row list
  int32_t wp;  // width
  int32_t nb_rows;  // rows below the panel's diagonal block (= ld_J - p0 - wp)
};

// Multiply-adds per shift on the exact column structure of L that each
// kernel of one panel performs (symbolic.cpp: they partition
// sum_k c_k (c_k + 1) / 2 for the factorization and sum_k (c_k^2 + c_k) for
// selected inversion).  The stored (relaxed supernodal) structure can hold
// explicit zeros, which the kernels multiply but which are not counted here.
struct PanelMacs {
  double intu = 0.0;   // left-looking update from the earlier panels of the supernode
  double diag = 0.0;   // LDL^T of the diagonal block
  double trsm = 0.0;   // rows below the diagonal block
  double off = 0.0;    // SelInv: Z_BB times L-hat
  double sdiag = 0.0;  // SelInv: diagonal-block partials
  double sfinal = 0.0; // SelInv: diagonal block in LDS (incl. the diagonal terms)
};

// Result of the symbolic analysis (symbolic.cpp).  All indices are 0-based;
// "new" indices are positions after the fill-reducing permutation.
struct Symbolic {
  int32_t n = 0;
  int64_t nnz_lower = 0;
  int32_t panel_width = 64;
  double pivot_tol = 1e-14;

  std::vector<int32_t> perm;   // new -> old column
  std::vector<int32_t> iperm;  // old -> new column

  // Supernodes: columns [sfirst[J], sfirst[J+1]) in the new order.
  int32_t nsuper = 0;
  std::vector<int32_t> sfirst;
  std::vector<int32_t> sparent;          // -1 for roots
  std::vector<int64_t> rowptr;           // row list E_J = rows[rowptr[J] .. rowptr[J+1])
  std::vector<int32_t> rows;             // own columns first, then the rows below
  std::vector<int64_t> off;              // storage offset (elements) of supernode J
  std::vector<int32_t> ld;               // leading dimension = |E_J|
  std::vector<int32_t> snode_of_col;     // new column -> supernode
  int64_t nnzL_store = 0;                // sum ld_J * w_J
  int64_t nnzL_stored_lower = 0;         // sum over J of lower part incl. diagonal
  int64_t nnzL_exact = 0;
  double flops_factor = 0.0, flops_selinv = 0.0;
  int32_t max_front = 0;

  // Gather/scatter maps (host copies, uploaded by pxs_symbolic_bind).
  //   address of element (row position i, column position q) of supernode
  //   J's row list, i >= q:  colmap[rowptr[J] + q] + relpos[colseg[rowptr[J] + q] + i]
  std::vector<int64_t> colmap;
  std::vector<int64_t> colseg;
  std::vector<int32_t> relpos;
  std::vector<int64_t> entry_off;    // input entry -> element offset
  std::vector<int32_t> entry_diag;   // 1 on the diagonal; 2 if the storage holds the entry's transpose; else 0

  std::vector<Panel> panels;        // factor order; selected inversion runs backwards
  std::vector<PanelMacs> xm_panel;  // exact multiply-adds per shift, one per panel
  std::vector<double> xm_update;    // exact multiply-adds per shift of each supernode's ancestor update
  int64_t max_below = 0;            // max nb_rows over panels
  int32_t max_split = 1;            // split-K pieces of the diagonal SelInv update

  // Device copies (inside the caller's map buffer).
  void* dmaps = nullptr;
  int64_t map_bytes = 0;
  int64_t o_colmap = 0, o_colseg = 0, o_entry_off = 0, o_relpos = 0, o_entry_diag = 0, o_diagoff = 0;
  std::vector<int64_t> diagoff;     // new column -> element offset of its diagonal entry

  // Workspace layout per batch: work_fixed, then work_per_shift for every
  // shift, then gather_per_shift (dense Z_CC of one supernode) for each shift
  // of a SelInv chunk (selinv_chunk shifts, 0 = the whole batch).
  int64_t work_fixed = 0, work_per_shift = 0, gather_per_shift = 0;
  int32_t selinv_chunk = 0;
  int32_t tile_rows = 64;           // rows per workgroup tile of the panel products (64 or 128)

  // Selected inversion runs independent subtrees on separate streams:
  // sel_stream[J] in [0, sel_nstreams); a supernode waits for its parent
  // when they are on different streams.  Each stream has its own per-shift
  // region (work_per_shift) and dense Z_CC region (gather_bytes[s] per shift).
  int32_t sel_nstreams = 1;
  int32_t fused_lanes = 0;   // factor panel work and SelInv: the sel_stream lanes fused on one stream
  std::vector<int32_t> sel_stream;
  std::vector<int64_t> gather_bytes;
  std::vector<uint8_t> cross_child;  // J has a child on another stream
  int32_t max_below_super = 0;      // max over supernodes of ld - w

  // Factorization with the same subtree streams: supernodes are issued by
  // height in the supernodal tree (leaves first, column order within a
  // height), the panel work of J on stream sel_stream[J], every ancestor
  // scatter on the caller's stream in that order.  fac_child[J] is the child
  // of J issued last (-1 for a leaf): its scatter ends the scatters into J.
  std::vector<int32_t> fac_order;
  std::vector<int32_t> fac_child;
};

struct AnalyzeOptions {
  int selinv_streams = 4;
  int selinv_chunk = 0;
  int tile_rows = 64;
  int ordering = 0;
  int leaf_cols = 128;
  int sep_cols = 0;        // 0: every separator is one supernode
  int fused_lanes = 0;    // 1: subtree lanes fused on one stream (factor and SelInv), -1: never, 0: by structure
  int panel_width = 64;
  double pivot_tol = 1e-14;
};

// Automatic lane fusion (AnalyzeOptions.fused_lanes = 0) below this many
// flops per supernode and shift.
constexpr double FUSE_FLOPS_PER_SUPER = 1e8;

// Returns 0 on success, -1 on invalid input (msg set).
int analyze(int32_t n, const int64_t* colptr, const int32_t* rowind, int32_t nblk,
            const int32_t* blkptr, const double* coords, const AnalyzeOptions& opt,
            Symbolic& S, std::string& msg);

// Rows of one split-K piece of the diagonal-block SelInv update, and the
// number of pieces for a panel with `below` rows beneath it.
constexpr int64_t SPLIT_ROWS = 256;
inline int32_t split_count(int64_t below) {
  int64_t s = (below + SPLIT_ROWS - 1) / SPLIT_ROWS;
  if (s < 1) s = 1;
  return (int32_t)s;
}

}  // namespace pxs
