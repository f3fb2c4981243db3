// Launch entry points of the numeric phases (numeric.hip) and the layout of
// the fixed part of the workspace.
#pragma once
#include <hip/hip_runtime.h>

#include "pxs_internal.h"

namespace pxs {

constexpr int MAX_SHIFTS = 4096;
constexpr int ABSMAX_BLOCKS = 512;
constexpr int POLESUM_BLOCKS = 1024;

// byte offsets inside the fixed workspace region (work_fixed = 1 MiB)
constexpr int64_t WK_ABSMAX = 0;             // 2 doubles: max|H|, max|S|
constexpr int64_t WK_ABSMAX_PART = 256;      // ABSMAX_BLOCKS x 2 doubles
constexpr int64_t WK_POLESUM_PART = 16384;   // POLESUM_BLOCKS x 8 doubles
constexpr int64_t WK_TRACES = 90112;         // 8 doubles
constexpr int64_t WK_SHIFTS = 131072;        // MAX_SHIFTS complex
constexpr int64_t WK_INFO = 196608;          // MAX_SHIFTS int64
constexpr int64_t WK_NEGC = WK_INFO + 8 * MAX_SHIFTS;   // MAX_SHIFTS int64
constexpr int64_t WK_WEIGHTS = 262144;       // 4 x MAX_SHIFTS complex
constexpr int64_t WK_FIXED_BYTES = 1 << 20;

// kernel-class timing with HIP events (pxs_profile_begin / _end)
enum KernelClass { KC_NONE = 0, KC_UPDATE = 1, KC_SELINV_OFF = 2, KC_TRSM = 3, KC_SELINV_DIAG = 4,
                   KC_LHAT = 5, KC_DIAG = 6, KC_ASSEMBLE = 7, KC_POLESUM = 8, KC_GATHER = 9 };
int profile_begin(int kernel);
int profile_end(double* ms, int64_t* launches, double* work, double* bytes, double* stored);

// inorder: every launch on the caller's stream (no library streams), as
// inside a stream capture; the results are the same bits either way.
template <bool CPLX>
int run_factor(const Symbolic& S, const double* H, const double* Sv, int nshift,
               const double* shifts_host, void* L, void* work, hipStream_t st, bool inorder = false);
// Kernel-only parts (no host copies), capturable into a HIP graph; the
// shifts and weights are read from the workspace.
template <bool CPLX>
int run_factor_kernels(const Symbolic& S, const double* H, const double* Sv, int nshift, void* L,
                       void* work, hipStream_t st, bool inorder = false);
int run_pole_sum_kernels(const Symbolic& S, int nshift, const void* L, void* work, const double* H,
                         const double* Sv, int nsets, double* out, int accumulate, hipStream_t st);
int upload_shifts(int nshift, const double* shifts_host, void* work, hipStream_t st);
int upload_weights(int nshift, int nsets, const double* weights_host, void* work, hipStream_t st);
// the same from device arrays (stream-ordered, no host involvement)
int upload_shifts_device(int nshift, const double* shifts_dev, void* work, hipStream_t st);
int upload_weights_device(int nshift, int nsets, const double* weights_dev, void* work, hipStream_t st);
// Inertia counts enqueued without host synchronisation: real shifts from a
// device array, the real LDL^T on the caller's stream, the negative-pivot
// counts and tiny-pivot columns copied to device arrays.
int run_inertia_async(const Symbolic& S, const double* H, const double* Sv, int nshift, const double* eps_dev,
                      void* L, void* work, int64_t* neg_dev, int64_t* info_dev, hipStream_t st);
// events: nullptr (library pool) or selinv_event_count(S) events owned by
// the caller (a graph plan).
int run_selinv(const Symbolic& S, int nshift, void* L, void* work, hipStream_t st,
               hipEvent_t* events = nullptr, bool inorder = false);
int selinv_event_count(const Symbolic& S);
// creates the subtree streams (call outside any stream capture)
int selinv_streams_ready(const Symbolic& S);
// workspace bytes a batch of nshift complex shifts needs (factor + SelInv)
int64_t selinv_work_bytes(const Symbolic& S, int nshift);
// the same when every launch runs on one stream (inorder, or a capture)
int64_t selinv_work_bytes_inorder(const Symbolic& S, int nshift);

// Workspace of the allocation-free density matrix: a device array of this
// size in the library's code object (one per device, for the life of the
// process), shared by every call on that device.
constexpr int64_t NOALLOC_SCRATCH_BYTES = int64_t(64) << 20;
// Its device address on the current device (looked up once per device).
int noalloc_scratch(void** ptr);
int run_pole_sum(const Symbolic& S, int nshift, const void* L, void* work, const double* H,
                 const double* Sv, int nsets, const double* weights_host, double* out,
                 hipStream_t st);
int run_gather(const Symbolic& S, int shift, const void* L, void* out, hipStream_t st);
int run_get_diag(const Symbolic& S, int shift, bool cplx, const void* L, void* out, hipStream_t st);

// Fused execution of several systems' density matrices (batch.inc).
struct BatchSys {
  const Symbolic* S;
  const double* H;
  const double* Sv;
  int32_t nshift;
  void* L;
  void* work;
  double* out;
};
struct BatchPlan;   // the schedule and its item table (host), opaque here
// Builds the schedule (host only); nullptr and *err set on failure.
BatchPlan* batch_create(const std::vector<BatchSys>& sys, int nsets, int* err);
void batch_destroy(BatchPlan* b);
int64_t batch_table_bytes(const BatchPlan* b);
int64_t batch_launches(const BatchPlan* b);
// Copies the item table to `table` (device, batch_table_bytes) on st and
// keeps the address for the launches.
int batch_bind(BatchPlan* b, void* table, hipStream_t st);
// Assembly, the fused factorization and SelInv, the pole sums (kernels
// only; the shifts and weights are read from each system's workspace).
int run_batch_kernels(const BatchPlan* b, hipStream_t st);

// Complex Hermitian pencils (hermitian.inc): L region + U^T region per shift.
int64_t herm_storage_bytes(const Symbolic& S, int nshift);
int64_t herm_work_bytes(const Symbolic& S, int nshift);
int run_factor_h(const Symbolic& S, const double* H, const double* Sv, int nshift, const double* shifts_host,
                 void* L, void* work, hipStream_t st);
int run_factor_kernels_h(const Symbolic& S, const double* H, const double* Sv, int nshift, void* L, void* work,
                         hipStream_t st);
int run_selinv_h(const Symbolic& S, int nshift, void* L, void* work, hipStream_t st);
int run_pole_sum_kernels_h(const Symbolic& S, int nshift, const void* L, void* work, const double* H,
                           const double* Sv, int nsets, double* out, hipStream_t st);
int run_pole_sum_h(const Symbolic& S, int nshift, const void* L, void* work, const double* H, const double* Sv,
                   int nsets, const double* weights_host, double* out, hipStream_t st);
int run_gather_h(const Symbolic& S, int shift, bool upper, const void* L, void* out, hipStream_t st);
int run_get_diag_h(const Symbolic& S, int shift, const void* L, void* out, hipStream_t st);

}  // namespace pxs
