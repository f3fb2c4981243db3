// C ABI (include/pexsi_hip.h): argument checking, handle management and the
// sequencing of the numeric phases.  No device memory is allocated here: the
// maps, factor storage and workspace are caller buffers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pexsi_hip.h"
#include "numeric.h"
#include "pxs_internal.h"

struct pxs_symbolic_s {
  pxs::Symbolic S;
};

struct pxs_numeric_s {
  const pxs::Symbolic* S = nullptr;
  const double* H = nullptr;
  const double* Sv = nullptr;
  int32_t nshift = 0;
  std::vector<double> shifts;   // 2 per shift (host copy, source of the async upload)
  std::vector<double> weights;  // host staging for pole sums
  void* L = nullptr;
  void* work = nullptr;
  bool selinv_done = false;
  bool herm = false;            // complex Hermitian factorization (L + U^T regions)
};

extern "C" void pxs_plan_free(struct pxs_plan_s* plan);

struct pxs_plan_s {
  const pxs::Symbolic* S = nullptr;
  int32_t nshift = 0, nsets = 0;
  void* work = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<double> shifts, weights;   // host staging (sources of the uploads)
  std::vector<hipEvent_t> events;        // fork/join events recorded in the capture
};

namespace {

thread_local std::string g_last_error;

pxs_status hip_fail(int e) {
  g_last_error = hipGetErrorString((hipError_t)e);
  return PXS_EHIP;
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

template <class T>
void append_bytes(std::vector<char>& buf, int64_t& off, const std::vector<T>& v) {
  off = (int64_t)((buf.size() + 255) / 256 * 256);
  buf.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
}

// Packs the device maps of a symbolic handle; also fills S.map_bytes and the
// offsets (deterministic, so info and bind agree).
void pack_maps(pxs::Symbolic& S, std::vector<char>* out) {
  std::vector<char> buf;
  if (S.diagoff.empty()) {
    S.diagoff.resize(S.n);
    for (int32_t J = 0; J < S.nsuper; ++J)
      for (int32_t c = S.sfirst[J]; c < S.sfirst[J + 1]; ++c) {
        const int64_t q = c - S.sfirst[J];
        S.diagoff[c] = S.off[J] + q * S.ld[J] + q;
      }
  }
  append_bytes(buf, S.o_colmap, S.colmap);
  append_bytes(buf, S.o_colseg, S.colseg);
  append_bytes(buf, S.o_entry_off, S.entry_off);
  append_bytes(buf, S.o_diagoff, S.diagoff);
  append_bytes(buf, S.o_relpos, S.relpos);
  append_bytes(buf, S.o_entry_diag, S.entry_diag);
  S.map_bytes = (int64_t)((buf.size() + 255) / 256 * 256);
  if (out) out->swap(buf);
}

}  // namespace

extern "C" {

const char* pxs_status_string(pxs_status s) {
  switch (s) {
    case PXS_OK: return "ok";
    case PXS_EINVAL: return "invalid argument";
    case PXS_ENOMEM: return "out of host memory";
    case PXS_EHIP: return "HIP runtime error";
    case PXS_ESTATE: return "handle in the wrong state";
    case PXS_TINY_PIVOT: return "tiny pivot (see info)";
  }
  return "unknown status";
}

const char* pxs_last_error(void) { return g_last_error.c_str(); }

pxs_status pxs_poles(double beta, double dE, double mu, int32_t P, int32_t nsets, pxs_c64* shifts,
                     pxs_c64* weights) {
  if (!shifts || !weights) return PXS_EINVAL;
  if (pxs::pole_table(beta, dE, mu, P, nsets, (double*)shifts, (double*)weights) != 0) return PXS_EINVAL;
  return PXS_OK;
}

pxs_status pxs_analyze(int32_t n, const int64_t* colptr, const int32_t* rowind, int32_t nblk,
                       const int32_t* blkptr, const double* coords, const pxs_options* opt,
                       pxs_symbolic* out) {
  if (!out || !colptr || !rowind || n <= 0) return PXS_EINVAL;
  *out = nullptr;
  pxs::AnalyzeOptions o;
  if (opt) {
    o.ordering = opt->ordering;
    if (opt->leaf_cols > 0) o.leaf_cols = opt->leaf_cols;
    if (opt->sep_cols < 0) return PXS_EINVAL;
    o.sep_cols = opt->sep_cols;
    if (opt->panel_width > 0) o.panel_width = opt->panel_width;
    if (opt->pivot_tol > 0) o.pivot_tol = opt->pivot_tol;
    if (opt->selinv_chunk < 0) return PXS_EINVAL;
    o.selinv_chunk = opt->selinv_chunk;
    if (opt->tile_rows != 0 && opt->tile_rows != 64 && opt->tile_rows != 128) return PXS_EINVAL;
    if (opt->tile_rows) o.tile_rows = opt->tile_rows;
    if (opt->selinv_streams < 0 || opt->selinv_streams > 8) return PXS_EINVAL;
    if (opt->selinv_streams) o.selinv_streams = opt->selinv_streams;
    if (opt->fused_lanes < -1 || opt->fused_lanes > 1) return PXS_EINVAL;
    o.fused_lanes = opt->fused_lanes;
    if (o.ordering != 0 && o.ordering != 1) return PXS_EINVAL;
    if (o.panel_width > 64) return PXS_EINVAL;
  }
  pxs_symbolic_s* h = new (std::nothrow) pxs_symbolic_s;
  if (!h) return PXS_ENOMEM;
  std::string msg;
  try {
    if (pxs::analyze(n, colptr, rowind, nblk, blkptr, coords, o, h->S, msg) != 0) {
      g_last_error = msg;
      delete h;
      return PXS_EINVAL;
    }
    h->S.work_fixed = pxs::WK_FIXED_BYTES;
    pack_maps(h->S, nullptr);
  } catch (const std::bad_alloc&) {
    delete h;
    return PXS_ENOMEM;
  }
  *out = h;
  return PXS_OK;
}

pxs_status pxs_symbolic_info(pxs_symbolic sym, pxs_syminfo* info) {
  if (!sym || !info) return PXS_EINVAL;
  const pxs::Symbolic& S = sym->S;
  std::memset(info, 0, sizeof(*info));
  info->n = S.n;
  info->nnz_lower = S.nnz_lower;
  info->nnz_L = S.nnzL_stored_lower;
  info->nnz_L_exact = S.nnzL_exact;
  info->nsuper = S.nsuper;
  info->npanel = (int64_t)S.panels.size();
  info->bytes_per_shift = 16 * S.nnzL_store;
  info->work_fixed = S.work_fixed;
  info->work_per_shift = S.work_per_shift;
  info->work_bytes = pxs::selinv_work_bytes(S, 1);
  info->gather_per_shift = S.gather_per_shift;
  info->selinv_chunk = S.selinv_chunk;
  info->map_bytes = S.map_bytes;
  info->max_front = S.max_front;
  info->flops_factor = S.flops_factor;
  info->flops_selinv = S.flops_selinv;
  for (const pxs::PanelMacs& m : S.xm_panel) {
    info->macs_exact[pxs::KC_UPDATE] += m.intu;
    info->macs_exact[pxs::KC_DIAG] += m.diag;
    info->macs_exact[pxs::KC_TRSM] += m.trsm;
    info->macs_exact[pxs::KC_SELINV_OFF] += m.off;
    info->macs_exact[pxs::KC_SELINV_DIAG] += m.sdiag;
    info->macs_exact[0] += m.sfinal;
  }
  for (double u : S.xm_update) info->macs_exact[pxs::KC_UPDATE] += u;
  info->fused_lanes = S.fused_lanes;
  info->sel_lanes = S.sel_nstreams;
  return PXS_OK;
}

pxs_status pxs_workspace_size(pxs_symbolic sym, int32_t nshift, int32_t real, int64_t* bytes) {
  if (!sym || !bytes || nshift < 1 || nshift > pxs::MAX_SHIFTS) return PXS_EINVAL;
  const pxs::Symbolic& S = sym->S;
  *bytes = real ? S.work_fixed + (int64_t)nshift * S.work_per_shift : pxs::selinv_work_bytes(S, nshift);
  return PXS_OK;
}

pxs_status pxs_symbolic_export(pxs_symbolic sym, int32_t* perm, int32_t* super_ptr,
                               int32_t* super_parent, int64_t* row_ptr, int32_t* rows) {
  if (!sym) return PXS_EINVAL;
  const pxs::Symbolic& S = sym->S;
  if (perm) std::memcpy(perm, S.perm.data(), sizeof(int32_t) * S.n);
  if (super_ptr) std::memcpy(super_ptr, S.sfirst.data(), sizeof(int32_t) * (S.nsuper + 1));
  if (super_parent) std::memcpy(super_parent, S.sparent.data(), sizeof(int32_t) * S.nsuper);
  if (row_ptr) std::memcpy(row_ptr, S.rowptr.data(), sizeof(int64_t) * (S.nsuper + 1));
  if (rows) std::memcpy(rows, S.rows.data(), sizeof(int32_t) * S.rows.size());
  return PXS_OK;
}

pxs_status pxs_symbolic_bind(pxs_symbolic sym, void* maps, void* stream) {
  if (!sym || !maps || !aligned256(maps)) return PXS_EINVAL;
  std::vector<char> buf;
  try {
    pack_maps(sym->S, &buf);
  } catch (const std::bad_alloc&) {
    return PXS_ENOMEM;
  }
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(maps, buf.data(), buf.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e);
  // the host staging buffer dies here: wait for the copy
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  sym->S.dmaps = maps;
  const int k = pxs::selinv_streams_ready(sym->S);
  if (k != 0) return hip_fail(k);
  return PXS_OK;
}

static pxs_status check_numeric_args(pxs_symbolic sym, const double* H, const double* Sv, int32_t nshift,
                                     void* Lbuf, void* work) {
  if (!sym || !H || !Sv || !Lbuf || !work) return PXS_EINVAL;
  if (nshift < 1 || nshift > pxs::MAX_SHIFTS) return PXS_EINVAL;
  if (!aligned256(Lbuf) || !aligned256(work)) return PXS_EINVAL;
  if (!sym->S.dmaps) return PXS_ESTATE;
  return PXS_OK;
}

pxs_status pxs_factor(pxs_symbolic sym, const double* Hval, const double* Sval, int32_t nshift,
                      const pxs_c64* shifts, void* Lbuf, void* work, int64_t* info, void* stream,
                      pxs_numeric* out) {
  pxs_status s0 = check_numeric_args(sym, Hval, Sval, nshift, Lbuf, work);
  if (s0 != PXS_OK) return s0;
  if (!shifts || !out) return PXS_EINVAL;
  for (int32_t l = 0; l < nshift; ++l)
    if (!std::isfinite(shifts[l].re) || !std::isfinite(shifts[l].im)) return PXS_EINVAL;
  pxs_numeric_s* h = new (std::nothrow) pxs_numeric_s;
  if (!h) return PXS_ENOMEM;
  h->S = &sym->S;
  h->H = Hval;
  h->Sv = Sval;
  h->nshift = nshift;
  h->shifts.assign((const double*)shifts, (const double*)shifts + 2 * nshift);
  h->L = Lbuf;
  h->work = work;
  hipStream_t st = (hipStream_t)stream;
  int e = pxs::run_factor<true>(sym->S, Hval, Sval, nshift, h->shifts.data(), Lbuf, work, st);
  if (e != 0) {
    delete h;
    return hip_fail(e);
  }
  *out = h;
  if (info) {
    hipError_t he = hipMemcpyAsync(info, (char*)work + pxs::WK_INFO, sizeof(int64_t) * nshift,
                                   hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(he);
    for (int32_t l = 0; l < nshift; ++l)
      if (info[l] != 0) return PXS_TINY_PIVOT;
  }
  return PXS_OK;
}

pxs_status pxs_hermitian_sizes(pxs_symbolic sym, int32_t nshift, int64_t* lbuf_bytes, int64_t* work_bytes) {
  if (!sym || nshift < 1 || nshift > pxs::MAX_SHIFTS) return PXS_EINVAL;
  if (lbuf_bytes) *lbuf_bytes = pxs::herm_storage_bytes(sym->S, nshift);
  if (work_bytes) *work_bytes = pxs::herm_work_bytes(sym->S, nshift);
  return PXS_OK;
}

pxs_status pxs_factor_hermitian(pxs_symbolic sym, const pxs_c64* Hval, const pxs_c64* Sval, int32_t nshift,
                                const pxs_c64* shifts, void* Lbuf, void* work, int64_t* info, void* stream,
                                pxs_numeric* out) {
  pxs_status s0 = check_numeric_args(sym, (const double*)Hval, (const double*)Sval, nshift, Lbuf, work);
  if (s0 != PXS_OK) return s0;
  if (!shifts || !out) return PXS_EINVAL;
  for (int32_t l = 0; l < nshift; ++l)
    if (!std::isfinite(shifts[l].re) || !std::isfinite(shifts[l].im)) return PXS_EINVAL;
  pxs_numeric_s* h = new (std::nothrow) pxs_numeric_s;
  if (!h) return PXS_ENOMEM;
  h->S = &sym->S;
  h->H = (const double*)Hval;
  h->Sv = (const double*)Sval;
  h->nshift = nshift;
  h->herm = true;
  h->shifts.assign((const double*)shifts, (const double*)shifts + 2 * nshift);
  h->L = Lbuf;
  h->work = work;
  hipStream_t st = (hipStream_t)stream;
  int e = pxs::run_factor_h(sym->S, h->H, h->Sv, nshift, h->shifts.data(), Lbuf, work, st);
  if (e != 0) {
    delete h;
    return hip_fail(e);
  }
  *out = h;
  if (info) {
    hipError_t he = hipMemcpyAsync(info, (char*)work + pxs::WK_INFO, sizeof(int64_t) * nshift,
                                   hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(he);
    for (int32_t l = 0; l < nshift; ++l)
      if (info[l] != 0) return PXS_TINY_PIVOT;
  }
  return PXS_OK;
}

pxs_status pxs_selinv(pxs_numeric num, void* stream) {
  if (!num) return PXS_EINVAL;
  if (num->selinv_done) return PXS_ESTATE;
  int e = num->herm ? pxs::run_selinv_h(*num->S, num->nshift, num->L, num->work, (hipStream_t)stream)
                    : pxs::run_selinv(*num->S, num->nshift, num->L, num->work, (hipStream_t)stream);
  if (e != 0) return hip_fail(e);
  num->selinv_done = true;
  return PXS_OK;
}

pxs_status pxs_pole_sum(pxs_numeric num, int32_t nsets, const pxs_c64* weights, double* out,
                        double* traces, void* stream) {
  if (!num || !weights || !out || nsets < 1 || nsets > 4) return PXS_EINVAL;
  if (!num->selinv_done) return PXS_ESTATE;
  num->weights.assign((const double*)weights, (const double*)weights + 2 * nsets * num->nshift);
  hipStream_t st = (hipStream_t)stream;
  int e = num->herm ? pxs::run_pole_sum_h(*num->S, num->nshift, num->L, num->work, num->H, num->Sv, nsets,
                                           num->weights.data(), out, st)
                    : pxs::run_pole_sum(*num->S, num->nshift, num->L, num->work, num->H, num->Sv, nsets,
                                        num->weights.data(), out, st);
  if (e != 0) return hip_fail(e);
  if (traces) {
    double t8[8];
    hipError_t he = hipMemcpyAsync(t8, (char*)num->work + pxs::WK_TRACES, sizeof(t8),
                                   hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(he);
    for (int g = 0; g < 2 * nsets; ++g) traces[g] = t8[g];
  }
  return PXS_OK;
}

pxs_status pxs_get_selected(pxs_numeric num, int32_t shift, pxs_c64* out, void* stream) {
  if (!num || !out || shift < 0 || shift >= num->nshift) return PXS_EINVAL;
  int e = num->herm ? pxs::run_gather_h(*num->S, shift, false, num->L, out, (hipStream_t)stream)
                    : pxs::run_gather(*num->S, shift, num->L, out, (hipStream_t)stream);
  if (e != 0) return hip_fail(e);
  return PXS_OK;
}

pxs_status pxs_get_selected_upper(pxs_numeric num, int32_t shift, pxs_c64* out, void* stream) {
  if (!num || !out || shift < 0 || shift >= num->nshift) return PXS_EINVAL;
  int e = num->herm ? pxs::run_gather_h(*num->S, shift, true, num->L, out, (hipStream_t)stream)
                    : pxs::run_gather(*num->S, shift, num->L, out, (hipStream_t)stream);
  if (e != 0) return hip_fail(e);
  return PXS_OK;
}

pxs_status pxs_get_diag(pxs_numeric num, int32_t shift, pxs_c64* out, void* stream) {
  if (!num || !out || shift < 0 || shift >= num->nshift) return PXS_EINVAL;
  if (num->selinv_done) return PXS_ESTATE;
  int e = num->herm ? pxs::run_get_diag_h(*num->S, shift, num->L, out, (hipStream_t)stream)
                    : pxs::run_get_diag(*num->S, shift, true, num->L, out, (hipStream_t)stream);
  if (e != 0) return hip_fail(e);
  return PXS_OK;
}

pxs_status pxs_inertia(pxs_symbolic sym, const double* Hval, const double* Sval, int32_t nshift,
                       const double* eps, void* Lbuf, void* work, int64_t* neg_count, int64_t* info,
                       void* stream) {
  pxs_status s0 = check_numeric_args(sym, Hval, Sval, nshift, Lbuf, work);
  if (s0 != PXS_OK) return s0;
  if (!eps || !neg_count) return PXS_EINVAL;
  std::vector<double> sh(2 * nshift, 0.0);
  for (int32_t q = 0; q < nshift; ++q) {
    if (!std::isfinite(eps[q])) return PXS_EINVAL;
    sh[2 * q] = eps[q];
  }
  hipStream_t st = (hipStream_t)stream;
  int e = pxs::run_factor<false>(sym->S, Hval, Sval, nshift, sh.data(), Lbuf, work, st);
  if (e != 0) return hip_fail(e);
  std::vector<int64_t> tmp(2 * pxs::MAX_SHIFTS);
  hipError_t he = hipMemcpyAsync(tmp.data(), (char*)work + pxs::WK_INFO, sizeof(int64_t) * 2 * pxs::MAX_SHIFTS,
                                 hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(he);
  bool tiny = false;
  for (int32_t q = 0; q < nshift; ++q) {
    neg_count[q] = tmp[pxs::MAX_SHIFTS + q];
    if (info) info[q] = tmp[q];
    tiny = tiny || tmp[q] != 0;
  }
  return tiny ? PXS_TINY_PIVOT : PXS_OK;
}

pxs_status pxs_inertia_async(pxs_symbolic sym, const double* Hval, const double* Sval, int32_t nshift,
                             const double* eps, void* Lbuf, void* work, int64_t* neg_count, int64_t* info,
                             void* stream) {
  pxs_status s0 = check_numeric_args(sym, Hval, Sval, nshift, Lbuf, work);
  if (s0 != PXS_OK) return s0;
  if (!eps || !neg_count || !info) return PXS_EINVAL;
  const int e = pxs::run_inertia_async(sym->S, Hval, Sval, nshift, eps, Lbuf, work, neg_count, info,
                                       (hipStream_t)stream);
  if (e != 0) return hip_fail(e);
  return PXS_OK;
}

pxs_status pxs_inertia_hermitian(pxs_symbolic sym, const pxs_c64* Hval, const pxs_c64* Sval, int32_t nshift,
                                 const double* eps, void* Lbuf, void* work, int64_t* neg_count, int64_t* info,
                                 void* stream) {
  pxs_status s0 = check_numeric_args(sym, (const double*)Hval, (const double*)Sval, nshift, Lbuf, work);
  if (s0 != PXS_OK) return s0;
  if (!eps || !neg_count) return PXS_EINVAL;
  std::vector<double> sh(2 * nshift, 0.0);
  for (int32_t q = 0; q < nshift; ++q) {
    if (!std::isfinite(eps[q])) return PXS_EINVAL;
    sh[2 * q] = eps[q];
  }
  hipStream_t st = (hipStream_t)stream;
  int e = pxs::run_factor_h(sym->S, (const double*)Hval, (const double*)Sval, nshift, sh.data(), Lbuf, work, st);
  if (e != 0) return hip_fail(e);
  std::vector<int64_t> tmp(2 * pxs::MAX_SHIFTS);
  hipError_t he = hipMemcpyAsync(tmp.data(), (char*)work + pxs::WK_INFO, sizeof(int64_t) * 2 * pxs::MAX_SHIFTS,
                                 hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(he);
  bool tiny = false;
  for (int32_t q = 0; q < nshift; ++q) {
    neg_count[q] = tmp[pxs::MAX_SHIFTS + q];
    if (info) info[q] = tmp[q];
    tiny = tiny || tmp[q] != 0;
  }
  return tiny ? PXS_TINY_PIVOT : PXS_OK;
}

pxs_status pxs_density_matrix(pxs_symbolic sym, const double* Hval, const double* Sval, double beta,
                              double dE, double mu, int32_t P, int32_t nsets, void* Lbuf, void* work,
                              double* out, double* traces, int64_t* info, pxs_c64* shifts,
                              pxs_c64* weights, void* stream) {
  if (nsets < 1 || nsets > 4 || P < 2 || (P & 1) || P > pxs::MAX_SHIFTS) return PXS_EINVAL;
  std::vector<pxs_c64> sh(P), wt((size_t)nsets * P);
  pxs_status s = pxs_poles(beta, dE, mu, P, nsets, sh.data(), wt.data());
  if (s != PXS_OK) return s;
  pxs_numeric num = nullptr;
  s = pxs_factor(sym, Hval, Sval, P, sh.data(), Lbuf, work, info, stream, &num);
  if (s < 0) return s;
  pxs_status piv = s;
  s = pxs_selinv(num, stream);
  if (s == PXS_OK) s = pxs_pole_sum(num, nsets, wt.data(), out, traces, stream);
  pxs_free_numeric(num);
  if (s != PXS_OK) return s;
  if (shifts) std::memcpy(shifts, sh.data(), sizeof(pxs_c64) * P);
  if (weights) std::memcpy(weights, wt.data(), sizeof(pxs_c64) * nsets * P);
  return piv;
}

pxs_status pxs_density_matrix_noalloc(pxs_symbolic sym, const double* Hval, const double* Sval, double beta,
                                      double dE, double mu, int32_t P, int32_t nsets, void* Lbuf, double* out,
                                      double* traces, int64_t* info, pxs_c64* shifts, pxs_c64* weights,
                                      void* stream) {
  if (!sym || nsets < 1 || nsets > 4 || P < 2 || (P & 1) || P > pxs::MAX_SHIFTS) return PXS_EINVAL;
  const pxs::Symbolic& S = sym->S;
  // the size limit is checked before anything touches the device
  const int64_t need = pxs::selinv_work_bytes_inorder(S, P);
  if (need > pxs::NOALLOC_SCRATCH_BYTES) {
    g_last_error = "pxs_density_matrix_noalloc: this system and pole count need " + std::to_string(need) +
                   " bytes of workspace; the library's scratch array holds " +
                   std::to_string(pxs::NOALLOC_SCRATCH_BYTES) + " (use pxs_density_matrix with a workspace)";
    return PXS_EINVAL;
  }
  if (!Hval || !Sval || !Lbuf || !out || !aligned256(Lbuf)) return PXS_EINVAL;
  if (!S.dmaps) return PXS_ESTATE;
  std::vector<pxs_c64> sh(P), wt((size_t)nsets * P);
  pxs_status s = pxs_poles(beta, dE, mu, P, nsets, sh.data(), wt.data());
  if (s != PXS_OK) return s;
  void* work = nullptr;
  int e = pxs::noalloc_scratch(&work);
  if (e != 0) return hip_fail(e);
  hipStream_t st = (hipStream_t)stream;
  // every launch on the caller's stream: no library streams or events
  e = pxs::run_factor<true>(S, Hval, Sval, P, (const double*)sh.data(), Lbuf, work, st, true);
  if (e == 0) e = pxs::run_selinv(S, P, Lbuf, work, st, nullptr, true);
  if (e == 0) e = pxs::run_pole_sum(S, P, Lbuf, work, Hval, Sval, nsets, (const double*)wt.data(), out, st);
  if (e != 0) return hip_fail(e);
  // the shift and weight uploads read sh and wt: finish before they go
  double t8[8];
  std::vector<int64_t> inf(P);
  hipError_t he = hipMemcpyAsync(t8, (char*)work + pxs::WK_TRACES, sizeof(t8), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess)
    he = hipMemcpyAsync(inf.data(), (char*)work + pxs::WK_INFO, sizeof(int64_t) * P, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(he);
  if (traces)
    for (int g = 0; g < 2 * nsets; ++g) traces[g] = t8[g];
  bool tiny = false;
  for (int32_t l = 0; l < P; ++l) {
    if (info) info[l] = inf[l];
    tiny = tiny || inf[l] != 0;
  }
  if (shifts) std::memcpy(shifts, sh.data(), sizeof(pxs_c64) * P);
  if (weights) std::memcpy(weights, wt.data(), sizeof(pxs_c64) * nsets * P);
  return tiny ? PXS_TINY_PIVOT : PXS_OK;
}

// One capture for both kinds of pencil: herm selects the L D U kernels (no
// accumulation into out for those).
static pxs_status plan_create(pxs_symbolic sym, const double* Hval, const double* Sval, int32_t nshift,
                              int32_t nsets, void* Lbuf, void* work, double* out, int32_t flags, bool herm,
                              pxs_plan* plan) {
  pxs_status s0 = check_numeric_args(sym, Hval, Sval, nshift, Lbuf, work);
  if (s0 != PXS_OK) return s0;
  if (!out || !plan || nsets < 1 || nsets > 4 || (flags & ~PXS_PLAN_ACCUMULATE)) return PXS_EINVAL;
  if (herm && (flags & PXS_PLAN_ACCUMULATE)) return PXS_EINVAL;
  *plan = nullptr;
  pxs_plan_s* p = new (std::nothrow) pxs_plan_s;
  if (!p) return PXS_ENOMEM;
  p->S = &sym->S;
  p->nshift = nshift;
  p->nsets = nsets;
  p->work = work;
  // everything the capture needs is created before it starts
  int k = pxs::selinv_streams_ready(sym->S);
  for (int q = 0; k == 0 && q < pxs::selinv_event_count(sym->S); ++q) {
    hipEvent_t ev;
    k = (int)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (k == 0) p->events.push_back(ev);
  }
  hipStream_t cs = nullptr;
  if (k == 0) k = (int)hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (k == 0) {
    k = (int)hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (k == 0) {
      if (herm) {
        // inside a capture the Hermitian SelInv stays on the capturing stream
        k = pxs::run_factor_kernels_h(sym->S, Hval, Sval, nshift, Lbuf, work, cs);
        if (k == 0) k = pxs::run_selinv_h(sym->S, nshift, Lbuf, work, cs);
        if (k == 0) k = pxs::run_pole_sum_kernels_h(sym->S, nshift, Lbuf, work, Hval, Sval, nsets, out, cs);
      } else {
        k = pxs::run_factor_kernels<true>(sym->S, Hval, Sval, nshift, Lbuf, work, cs);
        if (k == 0) k = pxs::run_selinv(sym->S, nshift, Lbuf, work, cs, p->events.data());
        if (k == 0)
          k = pxs::run_pole_sum_kernels(sym->S, nshift, Lbuf, work, Hval, Sval, nsets, out,
                                        (flags & PXS_PLAN_ACCUMULATE) ? 1 : 0, cs);
      }
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(cs, &g);
      if (e2 == hipSuccess) p->graph = g;   // only a graph the capture produced is kept
      if (k == 0 && e2 != hipSuccess) k = (int)e2;
    }
  }
  if (k == 0) k = (int)hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);   // cleanup: the capture's status decides
  if (k != 0) {
    pxs_plan_free(p);
    return hip_fail(k);
  }
  *plan = p;
  return PXS_OK;
}

pxs_status pxs_plan_create(pxs_symbolic sym, const double* Hval, const double* Sval, int32_t nshift,
                           int32_t nsets, void* Lbuf, void* work, double* out, int32_t flags,
                           pxs_plan* plan) {
  return plan_create(sym, Hval, Sval, nshift, nsets, Lbuf, work, out, flags, false, plan);
}

pxs_status pxs_plan_create_hermitian(pxs_symbolic sym, const pxs_c64* Hval, const pxs_c64* Sval, int32_t nshift,
                                     int32_t nsets, void* Lbuf, void* work, pxs_c64* out, int32_t flags,
                                     pxs_plan* plan) {
  return plan_create(sym, (const double*)Hval, (const double*)Sval, nshift, nsets, Lbuf, work, (double*)out,
                     flags, true, plan);
}

pxs_status pxs_plan_run(pxs_plan plan, const pxs_c64* shifts, const pxs_c64* weights, double* traces,
                        int64_t* info, void* stream) {
  if (!plan || !shifts || !weights) return PXS_EINVAL;
  for (int32_t l = 0; l < plan->nshift; ++l)
    if (!std::isfinite(shifts[l].re) || !std::isfinite(shifts[l].im)) return PXS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  plan->shifts.assign((const double*)shifts, (const double*)shifts + 2 * plan->nshift);
  plan->weights.assign((const double*)weights, (const double*)weights + 2 * plan->nsets * plan->nshift);
  int k = pxs::upload_shifts(plan->nshift, plan->shifts.data(), plan->work, st);
  if (k == 0) k = pxs::upload_weights(plan->nshift, plan->nsets, plan->weights.data(), plan->work, st);
  if (k == 0) k = (int)hipGraphLaunch(plan->exec, st);
  if (k != 0) return hip_fail(k);
  if (traces || info) return pxs_plan_results(plan, traces, info, stream);
  return PXS_OK;
}

pxs_status pxs_plan_run_device(pxs_plan plan, const pxs_c64* shifts, const pxs_c64* weights, void* stream) {
  if (!plan || !shifts || !weights) return PXS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int k = pxs::upload_shifts_device(plan->nshift, (const double*)shifts, plan->work, st);
  if (k == 0) k = pxs::upload_weights_device(plan->nshift, plan->nsets, (const double*)weights, plan->work, st);
  if (k == 0) k = (int)hipGraphLaunch(plan->exec, st);
  if (k != 0) return hip_fail(k);
  return PXS_OK;
}

pxs_status pxs_plan_copy_results(pxs_plan plan, double* traces, int64_t* info, void* stream) {
  if (!plan) return PXS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t he = hipSuccess;
  if (traces)
    he = hipMemcpyAsync(traces, (char*)plan->work + pxs::WK_TRACES, sizeof(double) * 2 * plan->nsets,
                        hipMemcpyDeviceToDevice, st);
  if (he == hipSuccess && info)
    he = hipMemcpyAsync(info, (char*)plan->work + pxs::WK_INFO, sizeof(int64_t) * plan->nshift,
                        hipMemcpyDeviceToDevice, st);
  if (he != hipSuccess) return hip_fail(he);
  return PXS_OK;
}

pxs_status pxs_plan_results(pxs_plan plan, double* traces, int64_t* info, void* stream) {
  if (!plan) return PXS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  double t8[8];
  std::vector<int64_t> inf(plan->nshift);
  hipError_t he = hipMemcpyAsync(t8, (char*)plan->work + pxs::WK_TRACES, sizeof(t8), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess)
    he = hipMemcpyAsync(inf.data(), (char*)plan->work + pxs::WK_INFO, sizeof(int64_t) * plan->nshift,
                        hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(he);
  if (traces)
    for (int g = 0; g < 2 * plan->nsets; ++g) traces[g] = t8[g];
  bool tiny = false;
  for (int32_t l = 0; l < plan->nshift; ++l) {
    if (info) info[l] = inf[l];
    tiny = tiny || inf[l] != 0;
  }
  return tiny ? PXS_TINY_PIVOT : PXS_OK;
}

void pxs_plan_free(pxs_plan plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  for (hipEvent_t e : plan->events) hipEventDestroy(e);
  delete plan;
}

struct pxs_batch_s {
  pxs::BatchPlan* plan = nullptr;
  std::vector<pxs::BatchSys> sys;
  int32_t nsets = 0;
  int64_t total_shifts = 0;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<double> shifts, weights;   // host staging (sources of the uploads)
};

pxs_status pxs_batch_create(int32_t nsys, const pxs_symbolic* syms, const double* const* Hval,
                            const double* const* Sval, const int32_t* nshift, int32_t nsets, void* const* Lbuf,
                            void* const* work, double* const* out, pxs_batch* batch) {
  if (!batch || nsys < 1 || !syms || !Hval || !Sval || !nshift || !Lbuf || !work || !out) return PXS_EINVAL;
  if (nsets < 1 || nsets > 4) return PXS_EINVAL;
  *batch = nullptr;
  std::vector<pxs::BatchSys> sys;
  int64_t total = 0;
  try {
    for (int32_t i = 0; i < nsys; ++i) {
      pxs_status s0 = check_numeric_args(syms[i], Hval[i], Sval[i], nshift[i], Lbuf[i], work[i]);
      if (s0 != PXS_OK) return s0;
      const pxs::Symbolic& S = syms[i]->S;
      // the fused path runs SelInv on all shifts at once, on one stream
      if (S.selinv_chunk > 0 && S.selinv_chunk < nshift[i]) {
        g_last_error = "pxs_batch_create: system " + std::to_string(i) + " has a SelInv shift chunk";
        return PXS_EINVAL;
      }
      if (!out[i]) return PXS_EINVAL;
      sys.push_back(pxs::BatchSys{&S, Hval[i], Sval[i], nshift[i], Lbuf[i], work[i], out[i]});
      total += nshift[i];
    }
  } catch (const std::bad_alloc&) {
    return PXS_ENOMEM;
  }
  pxs_batch_s* b = new (std::nothrow) pxs_batch_s;
  if (!b) return PXS_ENOMEM;
  int err = 0;
  b->plan = pxs::batch_create(sys, nsets, &err);
  if (!b->plan) {
    delete b;
    return err == (int)hipErrorOutOfMemory ? PXS_ENOMEM : hip_fail(err);
  }
  b->sys = sys;
  b->nsets = nsets;
  b->total_shifts = total;
  *batch = b;
  return PXS_OK;
}

pxs_status pxs_batch_info(pxs_batch batch, int64_t* table_bytes, int64_t* launches) {
  if (!batch) return PXS_EINVAL;
  if (table_bytes) *table_bytes = pxs::batch_table_bytes(batch->plan);
  if (launches) *launches = pxs::batch_launches(batch->plan);
  return PXS_OK;
}

pxs_status pxs_batch_bind(pxs_batch batch, void* table, void* stream) {
  if (!batch || batch->bound) return batch ? PXS_ESTATE : PXS_EINVAL;
  if (!table || !aligned256(table)) return PXS_EINVAL;
  int k = pxs::batch_bind(batch->plan, table, (hipStream_t)stream);
  hipStream_t cs = nullptr;
  if (k == 0) k = (int)hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (k == 0) {
    k = (int)hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (k == 0) {
      k = pxs::run_batch_kernels(batch->plan, cs);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(cs, &g);
      if (e2 == hipSuccess) batch->graph = g;
      if (k == 0 && e2 != hipSuccess) k = (int)e2;
    }
  }
  if (k == 0) k = (int)hipGraphInstantiate(&batch->exec, batch->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (k != 0) return hip_fail(k);
  batch->bound = true;
  return PXS_OK;
}

pxs_status pxs_batch_run(pxs_batch batch, const pxs_c64* shifts, const pxs_c64* weights, void* stream) {
  if (!batch || !shifts || !weights) return PXS_EINVAL;
  if (!batch->bound) return PXS_ESTATE;
  for (int64_t l = 0; l < batch->total_shifts; ++l)
    if (!std::isfinite(shifts[l].re) || !std::isfinite(shifts[l].im)) return PXS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  batch->shifts.assign((const double*)shifts, (const double*)shifts + 2 * batch->total_shifts);
  batch->weights.assign((const double*)weights, (const double*)weights + 2 * batch->nsets * batch->total_shifts);
  int k = 0;
  int64_t o = 0;
  for (const pxs::BatchSys& y : batch->sys) {
    k = pxs::upload_shifts(y.nshift, batch->shifts.data() + 2 * o, y.work, st);
    if (k == 0) k = pxs::upload_weights(y.nshift, batch->nsets, batch->weights.data() + 2 * batch->nsets * o,
                                        y.work, st);
    if (k != 0) return hip_fail(k);
    o += y.nshift;
  }
  k = (int)hipGraphLaunch(batch->exec, st);
  if (k != 0) return hip_fail(k);
  return PXS_OK;
}

pxs_status pxs_batch_results(pxs_batch batch, double* traces, int64_t* info, void* stream) {
  if (!batch) return PXS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const size_t nb = batch->sys.size();
  std::vector<double> t8(8 * nb);
  std::vector<int64_t> inf(batch->total_shifts);
  hipError_t he = hipSuccess;
  int64_t o = 0;
  for (size_t i = 0; i < nb && he == hipSuccess; ++i) {
    const pxs::BatchSys& y = batch->sys[i];
    he = hipMemcpyAsync(t8.data() + 8 * i, (char*)y.work + pxs::WK_TRACES, 8 * sizeof(double),
                        hipMemcpyDeviceToHost, st);
    if (he == hipSuccess)
      he = hipMemcpyAsync(inf.data() + o, (char*)y.work + pxs::WK_INFO, sizeof(int64_t) * y.nshift,
                          hipMemcpyDeviceToHost, st);
    o += y.nshift;
  }
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(he);
  if (traces)
    for (size_t i = 0; i < nb; ++i)
      for (int g = 0; g < 2 * batch->nsets; ++g) traces[2 * batch->nsets * i + g] = t8[8 * i + g];
  bool tiny = false;
  for (int64_t l = 0; l < batch->total_shifts; ++l) {
    if (info) info[l] = inf[l];
    tiny = tiny || inf[l] != 0;
  }
  return tiny ? PXS_TINY_PIVOT : PXS_OK;
}

void pxs_batch_free(pxs_batch batch) {
  if (!batch) return;
  if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
  if (batch->graph) (void)hipGraphDestroy(batch->graph);
  pxs::batch_destroy(batch->plan);
  delete batch;
}

pxs_status pxs_profile_begin(int32_t kernel) {
  if (kernel < 1 || kernel > 9) return PXS_EINVAL;
  pxs::profile_begin(kernel);
  return PXS_OK;
}

pxs_status pxs_profile_end(double* total_ms, int64_t* launches, double* work, double* bytes,
                           double* stored) {
  if (!total_ms || !launches || !work) return PXS_EINVAL;
  double b = 0.0, sw = 0.0;
  int e = pxs::profile_end(total_ms, launches, work, &b, &sw);
  if (e == -1) {
    g_last_error = "pxs_profile_end: no profile is open";
    return PXS_ESTATE;
  }
  if (bytes) *bytes = b;
  if (stored) *stored = sw;
  if (e != 0) return hip_fail(e);
  return PXS_OK;
}

void pxs_free_symbolic(pxs_symbolic sym) { delete sym; }
void pxs_free_numeric(pxs_numeric num) { delete num; }

}  // extern "C"
