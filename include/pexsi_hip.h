/*
 * pexsi_hip.h -- C ABI of the MI355X hot path of the PEXSI method
 * (pole expansion and selected inversion, arXiv:1405.0194).
 *
 * What the library computes (paper, Sec. II.A-II.C):
 *   for a real symmetric pencil (H, S), S positive definite, given on the
 *   lower triangle of the union pattern of H and S,
 *     - the pole table {z_l, omega_l^g} of eq. polerho / eq. gammaF,
 *     - for each shift w_l = z_l + mu: a supernodal LDL^T factorization of
 *       the complex symmetric A_l = H - w_l S (Sec. II.A "selected inversion"
 *       and Sec. II.B steps 1-3), without pivoting,
 *     - selected inversion: the entries of A_l^{-1} on the pattern of L
 *       (Sec. II.B step 4),
 *     - the pole sums Gamma^g = Im sum_l omega_l^g A_l^{-1} on the pattern
 *       of H and S (eqs. gammapole, gammaF) and the traces Tr(Gamma^g S),
 *       Tr(Gamma^g H) (eq. Nmu),
 *     - inertia counts #{negative d_k} of H - eps S in real arithmetic
 *       (Sec. II.C, Sylvester's law of inertia);
 *   for a complex Hermitian pencil (S Hermitian positive definite; the
 *   variant the paper's conclusion names for k-point sampling) the same
 *   steps with an L D U factorization, two-sided selected inversion, the
 *   density matrix as the matrix imaginary part (M - M^H) / 2i of the pole
 *   sum M, and inertia from the real pivots at real shifts (the *_hermitian
 *   functions).
 *
 * Conventions
 *   - Every function returns a pxs_status; nothing throws across the ABI.
 *     Negative codes are usage/system errors and leave outputs untouched
 *     unless stated.  PXS_TINY_PIVOT (> 0) is numeric: see info[].
 *   - Host pointers are marked (host); device pointers (device) must be
 *     device memory of the current HIP device.  The caller owns every array
 *     passed in.  The library owns only the opaque handles and their host
 *     metadata; it allocates no device memory on its own: the symbolic maps,
 *     the factor storage and the workspace all live in caller buffers whose
 *     sizes pxs_symbolic_info reports.
 *   - Matrices are given as the lower triangle (row >= column, diagonal
 *     included) in 0-based CSC: colptr (int64, n+1), rowind (int32, sorted
 *     within each column).  Value arrays are aligned with rowind.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work on it and return without synchronising, except where an output
 *     is a host array (traces, counts, info), which synchronises the stream.
 *   - Complex numbers are pxs_c64 {re, im}, layout-compatible with C99
 *     double complex and numpy/torch complex128.
 *   - Threads: a bound symbolic handle is read-only and may serve calls on
 *     several streams.  Eager factorization and selected inversion with more
 *     than one subtree stream (pxs_factor, pxs_inertia, pxs_selinv,
 *     pxs_density_matrix, pxs_factor_hermitian, pxs_inertia_hermitian) run
 *     independent subtrees on a process-wide pool of streams and events per
 *     device: issue such calls from one host thread at a time.  The results
 *     do not depend on the number of streams (bit-identical).  Graph plans
 *     use only the stream passed to pxs_plan_run.
 */
#ifndef PEXSI_HIP_H
#define PEXSI_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PXS_OK = 0,
  PXS_EINVAL = -1,     /* bad argument (null pointer, size, malformed CSC) */
  PXS_ENOMEM = -2,     /* host allocation failed */
  PXS_EHIP = -3,       /* a HIP runtime call failed */
  PXS_ESTATE = -4,     /* handle in the wrong state (e.g. maps not bound) */
  PXS_TINY_PIVOT = 1   /* some |d_k| fell below the pivot threshold; info[] */
} pxs_status;

typedef struct { double re, im; } pxs_c64;

typedef struct pxs_symbolic_s* pxs_symbolic;
typedef struct pxs_numeric_s* pxs_numeric;

/* Weight sets of the pole table, in this order (Sec. II.A, II.C). */
enum { PXS_SET_RHO = 0, PXS_SET_E = 1, PXS_SET_F = 2, PXS_SET_D = 3 };

typedef struct {
  int32_t ordering;     /* 0: nested dissection (default), 1: natural order */
  int32_t leaf_cols;    /* max columns of a nested-dissection leaf (0: 128) */
  int32_t panel_width;  /* columns per numeric panel, 1..64 (0: 64) */
  int32_t selinv_chunk; /* shifts per selected-inversion pass (0: the whole
                           batch); bounds the dense Z_CC workspace */
  double pivot_tol;     /* |d_k| < pivot_tol * (max|H| + |w| max|S|) flags a
                           tiny pivot (0: 1e-14) */
  int32_t tile_rows;    /* rows per workgroup tile of the panel products:
                           64 or 128 (0: 64) */
  int32_t selinv_streams; /* streams for independent subtrees in selected
                           inversion, 1..8 (0: 4); the library creates them
                           (default priority) on first use */
  int32_t sep_cols;     /* max columns of a separator supernode: a wider
                           nested-dissection separator is cut into pieces of
                           at most this many columns, each a supernode whose
                           rows below are the union of its own columns'
                           structures (fewer stored zeros); 0: no cut */
  int32_t fused_lanes; /* 1: the factorization's panel work and selected
                           inversion run the subtrees of the selinv_streams
                           assignment as lanes of the caller's stream, each
                           launch taking the next operation of every lane
                           that has one of its kind ready (one grid, no
                           library streams, also inside stream captures;
                           fewer, fuller launches: about half the time of a
                           small-supernode system such as a 1D chain);
                           -1: one stream per subtree; 0 (default): lanes
                           when the average supernode holds under 1e8 flops
                           per shift, else streams.  Complex-symmetric
                           pencils and inertia counts; the Hermitian path
                           keeps its streams */
  double reserved1[2];
} pxs_options;

typedef struct {
  int64_t n;                   /* matrix dimension */
  int64_t nnz_lower;           /* entries of the lower input pattern */
  int64_t nnz_L;               /* stored entries of L (supernodal, incl. the
                                  dense diagonal blocks' lower triangles) */
  int64_t nnz_L_exact;         /* entries of the exact pattern of L */
  int64_t nsuper;              /* supernodes */
  int64_t npanel;              /* numeric panels (supernodes cut into
                                  panel_width-wide column blocks) */
  int64_t bytes_per_shift;     /* factor storage per complex shift (bytes);
                                  a real (inertia) shift needs half */
  int64_t work_bytes;          /* workspace for one shift (pxs_workspace_size
                                  gives it for a batch) */
  int64_t work_fixed;
  int64_t work_per_shift;
  int64_t gather_per_shift;    /* dense Z_CC copy, per shift of a SelInv chunk */
  int64_t selinv_chunk;        /* as in pxs_options (0: whole batch) */
  int64_t map_bytes;           /* device bytes of the symbolic maps */
  int64_t max_front;           /* largest row count of a supernode */
  double flops_factor;         /* algorithmic flops per complex shift:
                                  8 * sum_k c_k (c_k + 1) / 2 */
  double flops_selinv;         /* 8 * sum_k (c_k^2 + c_k) */
  /* c_k = off-diagonal nonzeros of column k in the exact pattern of L */
  double macs_exact[8];        /* the same multiply-adds per shift split by
                                  the kernel class (pxs_profile_begin numbers)
                                  that performs them: [1] factor updates,
                                  [2] SelInv off-diagonal product, [3] panel
                                  TRSM, [4] SelInv diagonal-block partials,
                                  [6] diagonal-block LDL^T; [0] the SelInv
                                  diagonal blocks finished in LDS; [5] (L-hat,
                                  a by-product of the blocked algorithm) and
                                  [7] are 0.  [1]+[3]+[6] = flops_factor / 8,
                                  [0]+[2]+[4] = flops_selinv / 8. */
  int64_t fused_lanes;         /* 1 if the subtree lanes run fused on one
                                  stream (pxs_options.fused_lanes), else 0 */
  int64_t sel_lanes;           /* subtree streams or lanes (at most
                                  selinv_streams; 1: everything in order) */
} pxs_syminfo;

/* ---------------------------------------------------------------------- */
/* Pole table (Sec. II.A, eq. polerho; eq. gammaF; Sec. II.C).
 * beta: inverse temperature (1/Ha); dE: bound on max|eps - mu| over the
 * pencil's spectrum; mu: chemical potential; P: number of poles (even, >= 2).
 * Out (host): shifts[P] = z_l + mu (all with positive imaginary part) and
 * weights[nsets * P] (set-major: weights[g * P + l]) for the first nsets of
 * {rho, E, F, d}, 1 <= nsets <= 4, such that
 *   g(eps - mu) ~= Im sum_l weights[g*P+l] / (eps - shifts[l]).
 * Errors: PXS_EINVAL for P odd or < 2, beta/dE <= 0, nsets out of range. */
pxs_status pxs_poles(double beta, double dE, double mu, int32_t P, int32_t nsets,
                     pxs_c64* shifts, pxs_c64* weights);

/* ---------------------------------------------------------------------- */
/* Symbolic analysis (Sec. II.B steps 1-2; eq. parent).  Host only.
 * n, colptr, rowind (host): lower CSC of the union pattern of H and S.
 * nblk, blkptr (host, nullable): atom blocks, blkptr[0]=0 .. blkptr[nblk]=n;
 *   columns of a block stay together and are treated as one graph vertex.
 *   NULL: every column is its own block.
 * coords (host, nullable): nblk x 3 block positions, used for geometric
 *   nested dissection; NULL: graph (level-structure) nested dissection.
 * opt (host, nullable): NULL = defaults.
 * Out: *out, an immutable handle; free with pxs_free_symbolic.
 * Errors: PXS_EINVAL for a malformed pattern (unsorted or upper entries,
 *   missing diagonal, bad blkptr), PXS_ENOMEM. */
pxs_status pxs_analyze(int32_t n, const int64_t* colptr, const int32_t* rowind,
                       int32_t nblk, const int32_t* blkptr, const double* coords,
                       const pxs_options* opt, pxs_symbolic* out);

/* Sizes and work of an analysis (Sec. II.B steps 1-2: the pattern of L
 * found by the symbolic factorization sets the storage, the workspace and
 * the flop counts; Sec. II.A: the cost grows like nnz(L) and the dense
 * products on the supernodes).  info (host) receives the fields of
 * pxs_syminfo; the sizes are those every later call of this handle needs.
 * Errors: PXS_EINVAL for a null argument. */
pxs_status pxs_symbolic_info(pxs_symbolic sym, pxs_syminfo* info);

/* Workspace bytes for a batch of nshift shifts (`real`: an inertia batch,
 * which runs no selected inversion and needs less). */
pxs_status pxs_workspace_size(pxs_symbolic sym, int32_t nshift, int32_t real, int64_t* bytes);

/* Export of the analysis, for tests and tools (host arrays, any may be NULL):
 * perm[n] (new -> old column), super_ptr[nsuper+1] (first new column of each
 * supernode), super_parent[nsuper] (-1 for roots), row_ptr[nsuper+1] and
 * rows[row_ptr[nsuper]] (the sorted new row indices of each supernode, its
 * own columns first). */
pxs_status pxs_symbolic_export(pxs_symbolic sym, int32_t* perm, int32_t* super_ptr,
                               int32_t* super_parent, int64_t* row_ptr, int32_t* rows);

/* Copies the symbolic maps into `maps` (device, info.map_bytes bytes,
 * 256-byte aligned) on `stream` and records that buffer in the handle.
 * Must precede any numeric call; the buffer must outlive the handle's use. */
pxs_status pxs_symbolic_bind(pxs_symbolic sym, void* maps, void* stream);

/* ---------------------------------------------------------------------- */
/* Numeric LDL^T of A_l = H - shifts[l] S for l < nshift (Sec. II.B step 3):
 * assembles every shift into Lbuf and factors it in place.
 * Hval, Sval (device, nnz_lower doubles): values on the input pattern.
 * shifts (host, nshift): complex shifts w_l; Im w_l > 0 guarantees that
 *   the factorization exists (Im A_l is negative definite).
 * Lbuf (device, nshift * bytes_per_shift), work (device,
 *   pxs_workspace_size(sym, nshift, 0) bytes): caller buffers, 256-byte
 *   aligned, kept by the numeric handle.
 * info (host, nshift, nullable): 0, or the 1-based new column index of the
 *   first pivot below the threshold (the factor continues regardless).
 * Returns PXS_TINY_PIVOT if any info[l] != 0 (then synchronises stream). */
pxs_status pxs_factor(pxs_symbolic sym, const double* Hval, const double* Sval,
                      int32_t nshift, const pxs_c64* shifts, void* Lbuf, void* work,
                      int64_t* info, void* stream, pxs_numeric* out);

/* Complex Hermitian H and S (k-point Hamiltonians; the structurally
 * symmetric, non-symmetric variant named as future work in the paper's
 * conclusion): A_l = H - shifts[l] S is factored as L D U without pivoting.
 * Hval, Sval (device, nnz_lower complex): the lower triangle on the input
 * pattern (the upper triangle is its conjugate; diagonal entries real).
 * Lbuf and work sizes come from pxs_hermitian_sizes (Lbuf holds per shift
 * the L region and a U^T region of the same layout).  The returned handle
 * works with pxs_selinv (selected inverse of both triangles), pxs_pole_sum
 * (complex output, see there), pxs_get_selected (lower triangle Z_l[i][j],
 * i >= j), pxs_get_selected_upper (Z_l[j][i] at the same entries) and
 * pxs_get_diag.  SelInv of a Hermitian handle runs independent subtrees on
 * the library's streams as for real pencils (one stream inside a capture);
 * selinv_chunk does not apply: the workspace covers the whole batch.
 * Errors and info as for pxs_factor. */
pxs_status pxs_hermitian_sizes(pxs_symbolic sym, int32_t nshift, int64_t* lbuf_bytes, int64_t* work_bytes);
pxs_status pxs_factor_hermitian(pxs_symbolic sym, const pxs_c64* Hval, const pxs_c64* Sval,
                                int32_t nshift, const pxs_c64* shifts, void* Lbuf, void* work,
                                int64_t* info, void* stream, pxs_numeric* out);

/* Selected inversion in place (Sec. II.B step 4): afterwards Lbuf holds
 * Z_l = A_l^{-1} on the (supernodal) pattern of L for every shift. */
pxs_status pxs_selinv(pxs_numeric num, void* stream);

/* Pole sums (eqs. gammapole, gammaF): for every input entry k and set g < nsets,
 * out[g * nnz_lower + k] = Im sum_l weights[g * nshift + l] * Z_l[k]
 * (device output, input ordering).  traces (host, 2 * nsets, nullable):
 * traces[2g] = Tr(Gamma^g S), traces[2g+1] = Tr(Gamma^g H) over the full
 * symmetric matrices (two traces per set: no reserved third slot).
 * Requires pxs_selinv first.
 * Hermitian handles: Gamma^g = (M - M^H) / 2i with M = sum_l w_{g,l} Z_l
 * (the matrix imaginary part; entrywise Im for real pencils); out then holds
 * nsets * nnz_lower complex values (2 doubles each, Gamma_ij for i >= j) and
 * the traces are Re Tr(Gamma S), Re Tr(Gamma H). */
pxs_status pxs_pole_sum(pxs_numeric num, int32_t nsets, const pxs_c64* weights,
                        double* out, double* traces, void* stream);

/* The selected elements of Z_l = A_l^{-1} (Sec. II.A: selected inversion
 * returns the entries of the inverse on the pattern of H and S, which the
 * pattern of L contains) at the input entries: out (device, nnz_lower
 * complex, input ordering) after pxs_selinv; used by tests and for the LDOS
 * of Sec. II.D.  Errors: PXS_EINVAL for a null handle or output or a shift
 * outside 0..nshift-1. */
pxs_status pxs_get_selected(pxs_numeric num, int32_t shift, pxs_c64* out, void* stream);
/* Z_l[j][i] for every input entry (i, j), i >= j (equal to pxs_get_selected
 * for real pencils). */
pxs_status pxs_get_selected_upper(pxs_numeric num, int32_t shift, pxs_c64* out, void* stream);

/* D of shift l after pxs_factor (device out[n], new ordering). */
pxs_status pxs_get_diag(pxs_numeric num, int32_t shift, pxs_c64* out, void* stream);

/* Inertia counts (Sec. II.C): real LDL^T of H - eps[q] S for q < nshift and
 * neg_count[q] = #{k : d_k < 0} (host).  Lbuf needs nshift * bytes_per_shift
 * / 2 bytes, work as for pxs_factor.  info as for pxs_factor: a tiny pivot
 * makes the count unreliable; shift eps slightly and retry.  Synchronises. */
pxs_status pxs_inertia(pxs_symbolic sym, const double* Hval, const double* Sval,
                       int32_t nshift, const double* eps, void* Lbuf, void* work,
                       int64_t* neg_count, int64_t* info, void* stream);

/* Inertia counts (Sec. II.C) enqueued on `stream` without waiting for the
 * device, for callers that overlap counts with other work (a serving
 * loop): eps (device, nshift doubles) holds the real shifts; after the
 * stream reaches this point neg_count (device, nshift int64) holds
 * #{k : d_k < 0} of H - eps[q] S and info (device, nshift int64) the
 * 1-based column of a tiny pivot or 0 (a flagged count is unreliable: shift
 * eps slightly and count again).  Every launch runs on `stream` (no library
 * streams).  Lbuf and work as for pxs_inertia; the arrays must stay valid
 * until the stream has passed this call. */
pxs_status pxs_inertia_async(pxs_symbolic sym, const double* Hval, const double* Sval,
                             int32_t nshift, const double* eps, void* Lbuf, void* work,
                             int64_t* neg_count, int64_t* info, void* stream);

/* Inertia counts of a complex Hermitian pencil (Sec. II.C for Hermitian H,
 * S): the L D U factorization of H - eps[q] S (a Hermitian matrix at a real
 * shift, so D is real up to rounding) and neg_count[q] = #{k : Re d_k < 0}
 * (host), which by Sylvester's law is the number of eigenvalues of the
 * pencil below eps[q].  Hval, Sval: device complex values on the input
 * pattern as for pxs_factor_hermitian; Lbuf and work sized by
 * pxs_hermitian_sizes(nshift).  info and errors as for pxs_inertia.
 * Synchronises. */
pxs_status pxs_inertia_hermitian(pxs_symbolic sym, const pxs_c64* Hval, const pxs_c64* Sval,
                                 int32_t nshift, const double* eps, void* Lbuf, void* work,
                                 int64_t* neg_count, int64_t* info, void* stream);

/* The density matrix of Sec. II.B in one call: the pole table of eq.
 * polerho for (beta, dE, mu, P) and nsets weight sets (eq. gammaF), the
 * factorization and selected inversion of every shift, and the pole sums
 * Gamma^g = Im sum_l omega_l^g Z_l with their traces (eqs. gammapole, Nmu).
 * Buffers and outputs as for pxs_factor and pxs_pole_sum (out: device
 * nsets * nnz_lower; traces: host 2 * nsets; info: host P, nullable);
 * shifts/weights (host, nullable) receive the pole table used.  Errors: as
 * pxs_poles, pxs_factor, pxs_pole_sum; PXS_TINY_PIVOT as pxs_factor. */
pxs_status pxs_density_matrix(pxs_symbolic sym, const double* Hval, const double* Sval,
                              double beta, double dE, double mu, int32_t P, int32_t nsets,
                              void* Lbuf, void* work, double* out, double* traces,
                              int64_t* info, pxs_c64* shifts, pxs_c64* weights,
                              void* stream);

/* Allocation-free variant of pxs_density_matrix, for callers that cannot
 * allocate device memory (tight serving loops, code that must not call
 * hipMalloc): the same computation and results (bit for bit), with the
 * workspace in a device array inside the library (64 MiB per device, held
 * until the process ends) instead of a caller buffer.  The caller still
 * passes the bound symbolic handle, H and S values, Lbuf (P *
 * bytes_per_shift bytes) and out (device nsets * nnz_lower doubles).
 * Every launch runs on `stream` (no library streams); the call synchronises
 * it.  Calls on one device share the array: calls that overlap in time on
 * one device (several host threads or streams) race and must be serialised
 * by the caller.  Errors: PXS_EINVAL, before any device work, when the
 * system and P need more workspace than the array holds (pxs_last_error
 * gives both sizes), and for the arguments pxs_density_matrix rejects. */
pxs_status pxs_density_matrix_noalloc(pxs_symbolic sym, const double* Hval, const double* Sval,
                                      double beta, double dE, double mu, int32_t P, int32_t nsets,
                                      void* Lbuf, double* out, double* traces, int64_t* info,
                                      pxs_c64* shifts, pxs_c64* weights, void* stream);

/* ---------------------------------------------------------------------- */
/* Graph-captured density matrix (the batched execution of all shifts as one
 * replayable HIP graph).  pxs_plan_create captures assembly, LDL^T, selected
 * inversion and the pole sums of nsets weight sets for nshift shifts, bound
 * to these buffers (same conventions as pxs_factor / pxs_pole_sum; out is
 * device nsets * nnz_lower).  Shifts and weights are read from the workspace
 * when the graph runs, so one plan serves every pole table of the same size
 * and new H/S values on the same pattern (SCF-style repeats).  The capture
 * uses a private stream; creating a plan runs nothing.
 * pxs_plan_run uploads shifts[nshift] and weights[nsets * nshift] (host) on
 * `stream` and replays the graph there; traces (host, 2 * nsets) and info
 * (host, nshift) are optional and synchronise the stream.  Calls on one plan
 * must not overlap (they share the buffers).
 * flags: 0, or PXS_PLAN_ACCUMULATE: the pole sums are added to `out`
 * instead of overwriting it, so a system too large for one batch can run its
 * poles in chunks into one output (the traces then cover the last chunk). */
typedef struct pxs_plan_s* pxs_plan;
enum { PXS_PLAN_ACCUMULATE = 1 };
pxs_status pxs_plan_create(pxs_symbolic sym, const double* Hval, const double* Sval,
                           int32_t nshift, int32_t nsets, void* Lbuf, void* work, double* out,
                           int32_t flags, pxs_plan* plan);
/* The same for a complex Hermitian pencil (Hval, Sval, Lbuf, work as for
 * pxs_factor_hermitian): captures the L D U, the two-sided selected inversion
 * (on the capturing stream) and the pole sums Gamma^g = (M - M^H) / 2i;
 * out is device complex nsets * nnz_lower.  flags must be 0.  Run, results
 * and free as for pxs_plan_create. */
pxs_status pxs_plan_create_hermitian(pxs_symbolic sym, const pxs_c64* Hval, const pxs_c64* Sval,
                                     int32_t nshift, int32_t nsets, void* Lbuf, void* work, pxs_c64* out,
                                     int32_t flags, pxs_plan* plan);
pxs_status pxs_plan_run(pxs_plan plan, const pxs_c64* shifts, const pxs_c64* weights,
                        double* traces, int64_t* info, void* stream);
/* Traces (host, 2 * nsets, nullable) and info (host, nshift, nullable) of
 * the last run of the plan, after synchronising `stream` (the stream the run
 * was enqueued on, or one ordered after it). */
pxs_status pxs_plan_results(pxs_plan plan, double* traces, int64_t* info, void* stream);
/* pxs_plan_run with the pole table already on the device: shifts (device,
 * nshift) and weights (device, nsets * nshift, set-major) are copied into
 * the workspace on `stream` and the graph replayed there; nothing waits for
 * the device (the shifts are not checked for finiteness).  With
 * pxs_plan_copy_results a caller can queue several runs of one plan (pole
 * chunks of one request, PXS_PLAN_ACCUMULATE) back to back. */
pxs_status pxs_plan_run_device(pxs_plan plan, const pxs_c64* shifts, const pxs_c64* weights,
                               void* stream);
/* Enqueues copies of the last run's traces (device, 2 * nsets doubles,
 * nullable) and tiny-pivot info (device, nshift int64, nullable) on
 * `stream`, without waiting: a later run of the same plan overwrites the
 * workspace values, the copies do not change. */
pxs_status pxs_plan_copy_results(pxs_plan plan, double* traces, int64_t* info, void* stream);
void pxs_plan_free(pxs_plan plan);

/* ---------------------------------------------------------------------- */
/* Fused batch of systems (Sec. II.B: the poles of one system and separate
 * systems are independent, so their panel operations can share launches).
 * The density matrices of nsys real symmetric systems, each with its own
 * bound symbolic handle (no SelInv shift chunk), values, nshift[i] shifts
 * and caller buffers as for pxs_plan_create (Lbuf[i], work[i], out[i]:
 * device nsets * nnz_lower doubles), run as one sequence of launches: each
 * launch takes the next panel operation of every system whose next
 * operation uses the same kernel, as one grid.  Every system's operations
 * keep the order of its single-stream run, so its factors, selected
 * inverses and pole sums are the same bits as an eager run of it alone.
 * pxs_batch_create plans the launches (host only); pxs_batch_info reports
 * the device bytes of the launch table (table_bytes) and the number of
 * fused launches; pxs_batch_bind copies the table into `table` (device,
 * 256-byte aligned, kept until pxs_batch_free) and captures the whole
 * sequence (assembly, factorizations, selected inversions, pole sums) as
 * one HIP graph on a private stream.  pxs_batch_run uploads the pole tables
 * (host: shifts concatenated over the systems, sum nshift; weights
 * concatenated over the systems, each nsets * nshift[i] set-major) on
 * `stream` and replays the graph there; pxs_batch_results synchronises
 * `stream` and returns traces (host, nsys * 2 * nsets, nullable: system i's
 * Tr(G^g S), Tr(G^g H) at 2 * nsets * i + 2g) and info (host, sum nshift,
 * nullable).  Calls on one batch must not overlap (shared buffers). */
typedef struct pxs_batch_s* pxs_batch;
pxs_status pxs_batch_create(int32_t nsys, const pxs_symbolic* syms, const double* const* Hval,
                            const double* const* Sval, const int32_t* nshift, int32_t nsets,
                            void* const* Lbuf, void* const* work, double* const* out, pxs_batch* batch);
pxs_status pxs_batch_info(pxs_batch batch, int64_t* table_bytes, int64_t* launches);
pxs_status pxs_batch_bind(pxs_batch batch, void* table, void* stream);
pxs_status pxs_batch_run(pxs_batch batch, const pxs_c64* shifts, const pxs_c64* weights, void* stream);
pxs_status pxs_batch_results(pxs_batch batch, double* traces, int64_t* info, void* stream);
void pxs_batch_free(pxs_batch batch);

/* Kernel timing for benchmarks: while a profile is open, every launch of the
 * selected kernel class is bracketed by HIP events on its launch stream.
 * kernel: 1 factor update, 2 SelInv off-diagonal product, 3 panel TRSM,
 *         4 SelInv diagonal-block product, 5 L-hat product, 6 diagonal-block
 *         LDL^T, 7 assembly, 8 pole sum, 9 SelInv gather of Z_CC.
 * pxs_profile_end synchronises those events and returns the summed kernel
 * time (ms), the number of launches, their algorithmic flops (complex
 * multiply-add = 8 flops, real = 2, counted on the exact column structure
 * of L as in pxs_syminfo.macs_exact; for kernels 7, 8 and 9 their
 * algorithmic HBM bytes instead), in `bytes` (nullable) their algorithmic
 * HBM bytes (every operand of the stored structure read once and every
 * result written once) and in `stored` (nullable) their flops on the stored
 * (relaxed supernodal) structure, explicit zeros included, no tile padding.
 * Process-wide state; not thread safe.  PXS_ESTATE if no profile is open;
 * PXS_EHIP (and no totals) if an event could not be created or recorded
 * during the profile. */
pxs_status pxs_profile_begin(int32_t kernel);
pxs_status pxs_profile_end(double* total_ms, int64_t* launches, double* work, double* bytes,
                           double* stored);

/* Text of the last HIP or validation error seen by this thread (diagnostics). */
const char* pxs_last_error(void);

void pxs_free_symbolic(pxs_symbolic sym);
void pxs_free_numeric(pxs_numeric num);
const char* pxs_status_string(pxs_status s);

#ifdef __cplusplus
}
#endif
#endif /* PEXSI_HIP_H */
