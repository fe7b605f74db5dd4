// C-ABI entry points of librosko.so: argument checks on the host, then
// kernel launches on the caller's stream.  See include/rosko.h.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "internal.h"
#include "pack_batch.h"

namespace rosko {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = '\0'; }

}  // namespace rosko

using namespace rosko;

#define RK_REQUIRE(cond, code, ...) \
  do {                              \
    if (!(cond)) {                  \
      set_error(__VA_ARGS__);       \
      return (code);                \
    }                               \
  } while (0)

static int32_t check_dense(const void* A, int64_t M, int64_t K, int64_t lda, const char* name) {
  RK_REQUIRE(M >= 0 && K >= 0, ROSKO_EINVAL, "%s: negative size (%lld x %lld)", name,
             (long long)M, (long long)K);
  RK_REQUIRE(lda >= K && lda >= 1, ROSKO_EINVAL, "%s: leading dimension %lld < %lld", name,
             (long long)lda, (long long)K);
  RK_REQUIRE(A != nullptr || M == 0 || K == 0, ROSKO_EINVAL, "%s: null pointer", name);
  return ROSKO_OK;
}

static int32_t check_mr(int32_t mr) {
  RK_REQUIRE(mr >= 1 && mr <= 256, ROSKO_EINVAL, "mr %d outside 1..256", mr);
  return ROSKO_OK;
}

static int32_t check_packed_for_write(const rosko_packed* out, int64_t R, int64_t S, int32_t mr,
                                      int32_t dt) {
  RK_REQUIRE(out != nullptr, ROSKO_EINVAL, "packed output is null");
  RK_REQUIRE(out->M == R && out->K == S && out->mr == mr, ROSKO_EINVAL,
             "packed output shape (%lld x %lld, mr %d) does not match (%lld x %lld, mr %d)",
             (long long)out->M, (long long)out->K, out->mr, (long long)R, (long long)S, mr);
  RK_REQUIRE(dt == ROSKO_F32 || dt == ROSKO_BF16 || dt == ROSKO_FP8_E4M3, ROSKO_EUNSUPPORTED,
             "value dtype %d not supported", dt);
  RK_REQUIRE(out->nnz_cap >= 0 && out->ncols_cap >= 0 && out->nrec_cap >= 0, ROSKO_EINVAL,
             "negative capacity");
  RK_REQUIRE(S < (int64_t(1) << 24), ROSKO_EUNSUPPORTED, "K = %lld >= 2^24 columns",
             (long long)S);
  RK_REQUIRE(out->nrec_cap == 0 || out->rec, ROSKO_EINVAL, "record array is null");
  RK_REQUIRE(out->panel_nz_ptr && out->panel_col_ptr && out->col_ptr, ROSKO_EINVAL,
             "packed pointer arrays are null");
  RK_REQUIRE(out->ncols_cap == 0 || (out->col_ind && out->col_nnz), ROSKO_EINVAL,
             "packed column arrays are null");
  RK_REQUIRE(out->nnz_cap == 0 || (out->loc && out->val), ROSKO_EINVAL,
             "packed value arrays are null");
  RK_REQUIRE(dt != ROSKO_FP8_E4M3 || R == 0 || out->row_scale, ROSKO_EINVAL,
             "FP8 packing needs row_scale");
  RK_REQUIRE(R == 0 || out->kblk_ptr, ROSKO_EINVAL, "kblk_ptr is null");
  return ROSKO_OK;
}

static hipStream_t s_of(void* stream) { return static_cast<hipStream_t>(stream); }

static int32_t check_packed_for_read(const rosko_packed* A) {
  RK_REQUIRE(A != nullptr, ROSKO_EINVAL, "packed matrix is null");
  RK_REQUIRE(A->M >= 0 && A->K >= 0, ROSKO_EINVAL, "packed matrix has a negative size");
  int32_t st = check_mr(A->mr);
  if (st) return st;
  RK_REQUIRE(A->n_panels == ceil_div(A->M, A->mr), ROSKO_EINVAL,
             "n_panels %d != ceil(M / mr) = %lld", A->n_panels,
             (long long)ceil_div(A->M, A->mr));
  RK_REQUIRE(A->val_dtype == ROSKO_F32 || A->val_dtype == ROSKO_BF16 ||
                 A->val_dtype == ROSKO_FP8_E4M3,
             ROSKO_EUNSUPPORTED, "value dtype %d not supported", A->val_dtype);
  RK_REQUIRE(A->M == 0 || (A->panel_nz_ptr && A->panel_col_ptr && A->col_ptr), ROSKO_EINVAL,
             "packed pointer arrays are null");
  RK_REQUIRE(A->ncols_cap == 0 || (A->col_ind && A->col_nnz), ROSKO_EINVAL,
             "packed column arrays are null");
  RK_REQUIRE(A->nnz_cap == 0 || (A->loc && A->val), ROSKO_EINVAL,
             "packed value arrays are null");
  RK_REQUIRE(A->val_dtype != ROSKO_FP8_E4M3 || A->M == 0 || A->row_scale, ROSKO_EINVAL,
             "FP8 values need row_scale");
  RK_REQUIRE(A->M == 0 || A->kblk_ptr, ROSKO_EINVAL, "kblk_ptr is null");
  RK_REQUIRE(A->nrec_cap == 0 || A->rec, ROSKO_EINVAL, "record array is null");
  return ROSKO_OK;
}

extern "C" {

int32_t rosko_abi_version(void) { return 11; }

const char* rosko_last_error(void) { return g_err; }

const char* rosko_status_str(int32_t s) {
  switch (s) {
    case ROSKO_OK: return "ROSKO_OK";
    case ROSKO_EINVAL: return "ROSKO_EINVAL";
    case ROSKO_EUNSUPPORTED: return "ROSKO_EUNSUPPORTED";
    case ROSKO_ESMALLBUF: return "ROSKO_ESMALLBUF";
    case ROSKO_EHIP: return "ROSKO_EHIP";
    case ROSKO_EINTERNAL: return "ROSKO_EINTERNAL";
    default: return "ROSKO_UNKNOWN";
  }
}

int32_t rosko_pack_workspace_size(int64_t M, int64_t K, int32_t mr, int32_t transpose,
                                  size_t* bytes) {
  clear_error();
  RK_REQUIRE(bytes != nullptr, ROSKO_EINVAL, "bytes is null");
  RK_REQUIRE(M >= 0 && K >= 0, ROSKO_EINVAL, "negative size");
  int32_t st = check_mr(mr);
  if (st) return st;
  // transpose packing packs the K x M matrix A^T
  const PackWs L = transpose ? pack_ws_layout(K, M, mr, true) : pack_ws_layout(M, K, mr, false);
  *bytes = L.bytes;
  return ROSKO_OK;
}

int32_t rosko_pack_query(const float* A, int64_t M, int64_t K, int64_t lda, int32_t mr,
                         void* ws, size_t ws_bytes, void* stream, int64_t* nnz,
                         int64_t* ncols, int64_t* nrec) {
  clear_error();
  int32_t st = check_dense(A, M, K, lda, "A");
  if (st) return st;
  if ((st = check_mr(mr))) return st;
  RK_REQUIRE(nnz && ncols && nrec, ROSKO_EINVAL, "nnz / ncols / nrec outputs are null");
  RK_REQUIRE(K < (int64_t(1) << 24), ROSKO_EUNSUPPORTED, "K = %lld >= 2^24 columns",
             (long long)K);
  const PackWs L = pack_ws_layout(M, K, mr, false);
  RK_REQUIRE(ws != nullptr && ws_bytes >= L.bytes, ROSKO_ESMALLBUF,
             "workspace %zu bytes < %zu", ws_bytes, L.bytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  if ((st = launch_pack_count_scan(A, M, K, lda, mr, ws, L, nullptr, s))) return st;
  int64_t tot[4];
  ROSKO_HIP_CHECK(hipMemcpyAsync(tot, static_cast<char*>(ws) + L.totals, sizeof(tot),
                                 hipMemcpyDeviceToHost, s));
  ROSKO_HIP_CHECK(hipStreamSynchronize(s));
  *nnz = tot[0];
  *ncols = tot[1];
  *nrec = tot[3];
  return ROSKO_OK;
}

int32_t rosko_pack_transpose_query(const float* A, int64_t M, int64_t K, int64_t lda,
                                   int32_t mr, void* ws, size_t ws_bytes, void* stream,
                                   int64_t* nnz, int64_t* ncols, int64_t* nrec) {
  clear_error();
  int32_t st = check_dense(A, M, K, lda, "A");
  if (st) return st;
  if ((st = check_mr(mr))) return st;
  RK_REQUIRE(nnz && ncols && nrec, ROSKO_EINVAL, "nnz / ncols / nrec outputs are null");
  RK_REQUIRE(M < (int64_t(1) << 24), ROSKO_EUNSUPPORTED, "M = %lld >= 2^24 columns of A^T",
             (long long)M);
  const PackWs L = pack_ws_layout(K, M, mr, true);
  RK_REQUIRE(ws != nullptr && ws_bytes >= L.bytes, ROSKO_ESMALLBUF,
             "workspace %zu bytes < %zu", ws_bytes, L.bytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* At = reinterpret_cast<float*>(static_cast<char*>(ws) + L.transposed);
  (void)hipGetLastError();
  if ((st = launch_transpose(A, M, K, lda, At, s))) return st;
  if ((st = launch_pack_count_scan(At, K, M, M > 0 ? M : 1, mr, ws, L, nullptr, s))) return st;
  int64_t tot[4];
  ROSKO_HIP_CHECK(hipMemcpyAsync(tot, static_cast<char*>(ws) + L.totals, sizeof(tot),
                                 hipMemcpyDeviceToHost, s));
  ROSKO_HIP_CHECK(hipStreamSynchronize(s));
  *nnz = tot[0];
  *ncols = tot[1];
  *nrec = tot[3];
  return ROSKO_OK;
}

static int32_t pack_common(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                           int32_t val_dtype, void* ws, const PackWs& L, rosko_packed* out,
                           hipStream_t s) {
  int32_t st;
  out->n_panels = (int32_t)L.P;
  out->val_dtype = val_dtype;
  out->nnz = -1;
  out->ncols = -1;
  out->nrec = -1;
  (void)hipGetLastError();
  if (val_dtype == ROSKO_FP8_E4M3) {
    if ((st = launch_row_scale(A, R, S, lda, out->row_scale, s))) return st;
  }
  return launch_pack(A, R, S, lda, mr, val_dtype, ws, L, out, s);
}

int32_t rosko_pack(const float* A, int64_t M, int64_t K, int64_t lda, int32_t mr,
                   int32_t val_dtype, void* ws, size_t ws_bytes, rosko_packed* out,
                   void* stream) {
  clear_error();
  int32_t st = check_dense(A, M, K, lda, "A");
  if (st) return st;
  if ((st = check_mr(mr))) return st;
  if ((st = check_packed_for_write(out, M, K, mr, val_dtype))) return st;
  RK_REQUIRE(out->row_perm == nullptr, ROSKO_EUNSUPPORTED,
             "the dense packer keeps the row order: row_perm must be NULL");
  const PackWs L = pack_ws_layout(M, K, mr, false);
  RK_REQUIRE(L.P <= INT32_MAX, ROSKO_EUNSUPPORTED, "too many panels");
  RK_REQUIRE(ws != nullptr && ws_bytes >= L.bytes, ROSKO_ESMALLBUF,
             "workspace %zu bytes < %zu", ws_bytes, L.bytes);
  return pack_common(A, M, K, lda, mr, val_dtype, ws, L, out, static_cast<hipStream_t>(stream));
}

int32_t rosko_pack_batch(int32_t n, const rosko_pack_job* jobs, void* stream) {
  clear_error();
  RK_REQUIRE(n >= 0 && n <= ROSKO_PACK_BATCH_MAX, ROSKO_EINVAL, "batch of %d jobs (0..%d)", n,
             ROSKO_PACK_BATCH_MAX);
  RK_REQUIRE(n == 0 || jobs != nullptr, ROSKO_EINVAL, "jobs is null");
  PackTask t[ROSKO_PACK_BATCH_MAX];
  for (int32_t i = 0; i < n; ++i) {
    const rosko_pack_job& J = jobs[i];
    const bool tr = J.transpose != 0;
    // the packed matrix: A, or A^T (K x M) for a transpose job
    const int64_t R = tr ? J.K : J.M, S = tr ? J.M : J.K;
    int32_t st = check_dense(J.A, J.M, J.K, J.lda, "A");
    if (st) return st;
    if ((st = check_mr(J.mr))) return st;
    if ((st = check_packed_for_write(J.out, R, S, J.mr, J.val_dtype))) return st;
    RK_REQUIRE(J.out->row_perm == nullptr, ROSKO_EUNSUPPORTED,
               "job %d: the dense packer keeps the row order: row_perm must be NULL", i);
    const PackWs L = pack_ws_layout(R, S, J.mr, tr);
    RK_REQUIRE(L.P <= INT32_MAX, ROSKO_EUNSUPPORTED, "job %d: too many panels", i);
    RK_REQUIRE(J.ws != nullptr && J.ws_bytes >= L.bytes, ROSKO_ESMALLBUF,
               "job %d: workspace %zu bytes < %zu", i, J.ws_bytes, L.bytes);
    // a transpose job packs the dense transpose it writes into its workspace
    const float* src =
        tr ? reinterpret_cast<const float*>(static_cast<const char*>(J.ws) + L.transposed) : J.A;
    t[i] = PackTask{src, R, S, tr ? (J.M > 0 ? J.M : 1) : J.lda, J.mr, J.val_dtype, J.ws, L,
                    J.out};
  }
  for (int32_t i = 0; i < n; ++i) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(t[i].ws), a1 = a0 + t[i].L.bytes;
    for (int32_t j = i + 1; j < n; ++j) {
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(t[j].ws), b1 = b0 + t[j].L.bytes;
      RK_REQUIRE(t[i].out != t[j].out, ROSKO_EINVAL, "jobs %d and %d share their packed output",
                 i, j);
      RK_REQUIRE(a1 <= b0 || b1 <= a0, ROSKO_EINVAL, "jobs %d and %d share workspace bytes", i,
                 j);
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  for (int32_t i = 0; i < n; ++i) {
    if (jobs[i].transpose) {
      float* At = reinterpret_cast<float*>(static_cast<char*>(jobs[i].ws) + t[i].L.transposed);
      int32_t st = launch_transpose(jobs[i].A, jobs[i].M, jobs[i].K, jobs[i].lda, At, s);
      if (st) return st;
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    rosko_packed* out = t[i].out;
    out->n_panels = (int32_t)t[i].L.P;
    out->val_dtype = t[i].val_dtype;
    out->nnz = -1;
    out->ncols = -1;
    out->nrec = -1;
    if (t[i].val_dtype == ROSKO_FP8_E4M3) {
      int32_t st = launch_row_scale(t[i].A, t[i].R, t[i].S, t[i].lda, out->row_scale, s);
      if (st) return st;
    }
  }
  return launch_pack_batch(t, n, s);
}

int32_t rosko_pack_transpose(const float* A, int64_t M, int64_t K, int64_t lda, int32_t mr,
                             int32_t val_dtype, void* ws, size_t ws_bytes, rosko_packed* out,
                             void* stream) {
  clear_error();
  int32_t st = check_dense(A, M, K, lda, "A");
  if (st) return st;
  if ((st = check_mr(mr))) return st;
  if ((st = check_packed_for_write(out, K, M, mr, val_dtype))) return st;
  RK_REQUIRE(out->row_perm == nullptr, ROSKO_EUNSUPPORTED,
             "the dense packer keeps the row order: row_perm must be NULL");
  const PackWs L = pack_ws_layout(K, M, mr, true);
  RK_REQUIRE(L.P <= INT32_MAX, ROSKO_EUNSUPPORTED, "too many panels");
  RK_REQUIRE(ws != nullptr && ws_bytes >= L.bytes, ROSKO_ESMALLBUF,
             "workspace %zu bytes < %zu", ws_bytes, L.bytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* At = reinterpret_cast<float*>(static_cast<char*>(ws) + L.transposed);
  (void)hipGetLastError();
  if ((st = launch_transpose(A, M, K, lda, At, s))) return st;
  return pack_common(At, K, M, M > 0 ? M : 1, mr, val_dtype, ws, L, out, s);
}

int32_t rosko_pack_result(const void* ws, size_t ws_bytes, rosko_packed* packed, void* stream) {
  clear_error();
  RK_REQUIRE(packed != nullptr, ROSKO_EINVAL, "packed is null");
  int32_t st = check_mr(packed->mr);
  if (st) return st;
  const PackWs L = pack_ws_layout(packed->M, packed->K, packed->mr, false);
  RK_REQUIRE(ws != nullptr && ws_bytes >= L.totals + 4 * sizeof(int64_t), ROSKO_ESMALLBUF,
             "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t tot[4];
  ROSKO_HIP_CHECK(hipMemcpyAsync(tot, static_cast<const char*>(ws) + L.totals, sizeof(tot),
                                 hipMemcpyDeviceToHost, s));
  ROSKO_HIP_CHECK(hipStreamSynchronize(s));
  packed->nnz = tot[0];
  packed->ncols = tot[1];
  packed->nrec = tot[3];
  RK_REQUIRE(tot[2] == 0, ROSKO_ESMALLBUF,
             "packing needs %lld values / %lld columns / %lld records, capacities are "
             "%lld / %lld / %lld",
             (long long)tot[0], (long long)tot[1], (long long)tot[3],
             (long long)packed->nnz_cap, (long long)packed->ncols_cap,
             (long long)packed->nrec_cap);
  return ROSKO_OK;
}

int32_t rosko_pack_set_mode(int32_t mode) {
  clear_error();
  return set_pack_mode(mode);
}

// ------------------------------------------------------- CSR packing

static int32_t check_csr_sizes(int64_t M, int64_t K, int64_t nnz_in, int32_t mr) {
  RK_REQUIRE(M >= 0 && K >= 0 && nnz_in >= 0, ROSKO_EINVAL, "negative size");
  int32_t st = check_mr(mr);
  if (st) return st;
  RK_REQUIRE(M < (int64_t(1) << 31) && nnz_in < (int64_t(1) << 31), ROSKO_EUNSUPPORTED,
             "CSR packing takes M and nnz below 2^31");
  RK_REQUIRE(K < (int64_t(1) << 24), ROSKO_EUNSUPPORTED, "K = %lld >= 2^24 columns",
             (long long)K);
  return ROSKO_OK;
}

static int32_t check_csr(const int64_t* row_ptr, const int32_t* col_idx, const float* val,
                         int64_t M, int64_t K, int64_t nnz_in, int32_t mr) {
  int32_t st = check_csr_sizes(M, K, nnz_in, mr);
  if (st) return st;
  RK_REQUIRE(M == 0 || row_ptr != nullptr, ROSKO_EINVAL, "row_ptr is null");
  RK_REQUIRE(nnz_in == 0 || (col_idx && val), ROSKO_EINVAL, "col_idx / val is null");
  return ROSKO_OK;
}

static int32_t csr_ws_need(int64_t M, int64_t K, int64_t nnz_in, int32_t mr, hipStream_t s,
                           size_t* need) {
  const CsrWs L = csr_ws_layout(M, nnz_in, mr);
  size_t temp = 0;
  if (M > 0) {
    int32_t st = csr_temp_bytes(L, M, K, &temp, s);
    if (st) return st;
  }
  *need = L.bytes + (size_t)round_up((int64_t)temp, 256);
  return ROSKO_OK;
}

int32_t rosko_pack_csr_workspace_size(int64_t M, int64_t K, int64_t nnz_in, int32_t mr,
                                      size_t* bytes) {
  clear_error();
  RK_REQUIRE(bytes != nullptr, ROSKO_EINVAL, "bytes is null");
  *bytes = 0;
  int32_t st = check_csr_sizes(M, K, nnz_in, mr);
  if (st) return st;
  return csr_ws_need(M, K, nnz_in, mr, nullptr, bytes);
}

int32_t rosko_pack_csr_query(const int64_t* row_ptr, const int32_t* col_idx, const float* val,
                             const int32_t* row_perm, int64_t M, int64_t K, int64_t nnz_in,
                             int32_t mr, void* ws, size_t ws_bytes, void* stream, int64_t* nnz,
                             int64_t* ncols, int64_t* nrec) {
  clear_error();
  int32_t st = check_csr(row_ptr, col_idx, val, M, K, nnz_in, mr);
  if (st) return st;
  RK_REQUIRE(nnz && ncols && nrec, ROSKO_EINVAL, "nnz / ncols / nrec outputs are null");
  hipStream_t s = s_of(stream);
  size_t need = 0;
  if ((st = csr_ws_need(M, K, nnz_in, mr, s, &need))) return st;
  RK_REQUIRE(ws != nullptr && ws_bytes >= need, ROSKO_ESMALLBUF, "workspace %zu bytes < %zu",
             ws_bytes, need);
  (void)hipGetLastError();
  if ((st = launch_pack_csr(row_ptr, col_idx, val, row_perm, M, K, nnz_in, mr, ROSKO_F32, ws,
                            ws_bytes, nullptr, s)))
    return st;
  int64_t tot[kCsrTotals];
  ROSKO_HIP_CHECK(hipMemcpyAsync(tot, ws, sizeof(tot), hipMemcpyDeviceToHost, s));
  ROSKO_HIP_CHECK(hipStreamSynchronize(s));
  RK_REQUIRE(tot[kCsrTotBad] == 0, ROSKO_EINVAL,
             "invalid CSR input (flags 0x%llx: 1 row_perm entry out of range, 2 row_perm "
             "repeats a row, 4 bad row pointers, 8 column out of range, 16 repeated entry)",
             (unsigned long long)tot[kCsrTotBad]);
  *nnz = tot[kCsrTotNnz];
  *ncols = tot[kCsrTotNcols];
  *nrec = tot[kCsrTotNrec];
  return ROSKO_OK;
}

int32_t rosko_pack_csr(const int64_t* row_ptr, const int32_t* col_idx, const float* val,
                       int64_t M, int64_t K, int64_t nnz_in, int32_t mr, int32_t val_dtype,
                       void* ws, size_t ws_bytes, rosko_packed* out, void* stream) {
  clear_error();
  int32_t st = check_csr(row_ptr, col_idx, val, M, K, nnz_in, mr);
  if (st) return st;
  if ((st = check_packed_for_write(out, M, K, mr, val_dtype))) return st;
  hipStream_t s = s_of(stream);
  size_t need = 0;
  if ((st = csr_ws_need(M, K, nnz_in, mr, s, &need))) return st;
  RK_REQUIRE(ws != nullptr && ws_bytes >= need, ROSKO_ESMALLBUF, "workspace %zu bytes < %zu",
             ws_bytes, need);
  RK_REQUIRE(ceil_div(M, mr) <= INT32_MAX, ROSKO_EUNSUPPORTED, "too many panels");
  out->n_panels = (int32_t)ceil_div(M, mr);
  out->val_dtype = val_dtype;
  out->nnz = -1;
  out->ncols = -1;
  out->nrec = -1;
  (void)hipGetLastError();
  return launch_pack_csr(row_ptr, col_idx, val, out->row_perm, M, K, nnz_in, mr, val_dtype, ws,
                         ws_bytes, out, s);
}

int32_t rosko_pack_csr_result(const void* ws, size_t ws_bytes, rosko_packed* packed,
                              void* stream) {
  clear_error();
  RK_REQUIRE(packed != nullptr, ROSKO_EINVAL, "packed is null");
  RK_REQUIRE(ws != nullptr && ws_bytes >= sizeof(int64_t) * kCsrTotals, ROSKO_ESMALLBUF,
             "workspace too small");
  hipStream_t s = s_of(stream);
  int64_t tot[kCsrTotals];
  ROSKO_HIP_CHECK(hipMemcpyAsync(tot, ws, sizeof(tot), hipMemcpyDeviceToHost, s));
  ROSKO_HIP_CHECK(hipStreamSynchronize(s));
  packed->nnz = tot[kCsrTotNnz];
  packed->ncols = tot[kCsrTotNcols];
  packed->nrec = tot[kCsrTotNrec];
  RK_REQUIRE(tot[kCsrTotBad] == 0, ROSKO_EINVAL,
             "invalid CSR input (flags 0x%llx: 1 row_perm entry out of range, 2 row_perm "
             "repeats a row, 4 bad row pointers, 8 column out of range, 16 repeated entry)",
             (unsigned long long)tot[kCsrTotBad]);
  RK_REQUIRE(tot[kCsrTotOverflow] == 0, ROSKO_ESMALLBUF,
             "packing needs %lld values / %lld columns / %lld records, capacities are "
             "%lld / %lld / %lld",
             (long long)tot[kCsrTotNnz], (long long)tot[kCsrTotNcols],
             (long long)tot[kCsrTotNrec], (long long)packed->nnz_cap,
             (long long)packed->ncols_cap, (long long)packed->nrec_cap);
  return ROSKO_OK;
}

int32_t rosko_row_order_workspace_size(int64_t M, size_t* bytes) {
  clear_error();
  RK_REQUIRE(bytes != nullptr, ROSKO_EINVAL, "bytes is null");
  *bytes = 0;
  RK_REQUIRE(M >= 0, ROSKO_EINVAL, "negative size");
  RK_REQUIRE(M < (int64_t(1) << 31), ROSKO_EUNSUPPORTED, "M >= 2^31");
  if (M == 0) return ROSKO_OK;
  size_t temp = 0;
  int32_t st = order_temp_bytes(M, &temp, nullptr);
  if (st) return st;
  *bytes = order_ws_bytes_fixed(M) + (size_t)round_up((int64_t)temp, 256);
  return ROSKO_OK;
}

int32_t rosko_row_order(const int64_t* row_ptr, int64_t M, int32_t mr, int32_t mode, void* ws,
                        size_t ws_bytes, int32_t* perm, void* stream) {
  clear_error();
  RK_REQUIRE(M >= 0, ROSKO_EINVAL, "negative size");
  int32_t st = check_mr(mr);
  if (st) return st;
  RK_REQUIRE(mode == ROSKO_ORDER_DEGREE || mode == ROSKO_ORDER_BALANCED, ROSKO_EINVAL,
             "unknown row order mode %d", mode);
  RK_REQUIRE(M < (int64_t(1) << 31), ROSKO_EUNSUPPORTED, "M >= 2^31");
  if (M == 0) return ROSKO_OK;
  RK_REQUIRE(row_ptr != nullptr && perm != nullptr, ROSKO_EINVAL, "null argument");
  hipStream_t s = s_of(stream);
  size_t temp = 0;
  if ((st = order_temp_bytes(M, &temp, s))) return st;
  const size_t need = order_ws_bytes_fixed(M) + (size_t)round_up((int64_t)temp, 256);
  RK_REQUIRE(ws != nullptr && ws_bytes >= need, ROSKO_ESMALLBUF, "workspace %zu bytes < %zu",
             ws_bytes, need);
  (void)hipGetLastError();
  return launch_row_order(row_ptr, M, mr, mode, ws, ws_bytes, perm, s);
}

int32_t rosko_spmm_workspace_size(const rosko_packed* A, int64_t N, const rosko_plan* plan,
                                  size_t* bytes) {
  clear_error();
  RK_REQUIRE(A != nullptr && bytes != nullptr, ROSKO_EINVAL, "null argument");
  RK_REQUIRE(A->M >= 0 && A->K >= 0 && N >= 0, ROSKO_EINVAL, "negative size");
  int32_t st = check_mr(A->mr);
  if (st) return st;
  rosko_plan p = plan ? *plan : auto_plan(A, N);
  if ((st = normalize_plan(A, N, &p))) return st;
  *bytes = spmm_ws_bytes(A, N, p);
  return ROSKO_OK;
}

int32_t rosko_spmm(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N,
                   int64_t ldb, float* C, int64_t ldc, int32_t beta, const rosko_plan* plan,
                   void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int32_t st = check_packed_for_read(A);
  if (st) return st;
  RK_REQUIRE(b_dtype == ROSKO_F32 || b_dtype == ROSKO_BF16, ROSKO_EUNSUPPORTED,
             "B dtype %d not supported", b_dtype);
  RK_REQUIRE(N >= 0, ROSKO_EINVAL, "negative N");
  RK_REQUIRE(ldb >= N && ldb >= 1, ROSKO_EINVAL, "ldb %lld < N %lld", (long long)ldb,
             (long long)N);
  RK_REQUIRE(ldc >= N && ldc >= 1, ROSKO_EINVAL, "ldc %lld < N %lld", (long long)ldc,
             (long long)N);
  RK_REQUIRE(beta == 0 || beta == 1, ROSKO_EINVAL, "beta must be 0 or 1");
  RK_REQUIRE(B != nullptr || A->K == 0 || N == 0, ROSKO_EINVAL, "B is null");
  RK_REQUIRE(C != nullptr || A->M == 0 || N == 0, ROSKO_EINVAL, "C is null");
  rosko_plan p = plan ? *plan : auto_plan(A, N);
  if ((st = normalize_plan(A, N, &p))) return st;
  if (A->M == 0 || N == 0) return ROSKO_OK;
  (void)hipGetLastError();
  if (p.path == ROSKO_PATH_DENSE) {
    if (A->K == 0) return beta ? ROSKO_OK : launch_fill_zero(C, A->M, N, ldc, s_of(stream));
    return launch_spmm_dense(A, B, b_dtype, N, ldb, C, ldc, beta, ws, ws_bytes,
                             static_cast<hipStream_t>(stream));
  }
  return launch_spmm_sparse(A, B, b_dtype, N, ldb, C, ldc, beta, p, static_cast<float*>(ws),
                            ws_bytes, static_cast<hipStream_t>(stream));
}

int32_t rosko_spmm_backward_workspace_size(const rosko_packed* A, const rosko_packed* At,
                                           int64_t N, size_t* bytes) {
  clear_error();
  RK_REQUIRE(bytes != nullptr, ROSKO_EINVAL, "bytes is null");
  *bytes = 0;
  RK_REQUIRE(N >= 0, ROSKO_EINVAL, "negative N");
  int32_t st;
  if (At != nullptr) {
    RK_REQUIRE(At->M >= 0 && At->K >= 0, ROSKO_EINVAL, "negative size");
    if ((st = check_mr(At->mr))) return st;
    rosko_plan p = auto_plan(At, N);
    *bytes = spmm_ws_bytes(At, N, p);
  }
  if (A != nullptr) {
    RK_REQUIRE(A->M >= 0 && A->K >= 0 && A->nnz_cap >= 0, ROSKO_EINVAL, "negative size");
    if ((st = check_mr(A->mr))) return st;
    // dB's SpMM and dA's SDDMM run one after the other on the stream: they
    // share the workspace
    *bytes = std::max(*bytes, sddmm_ws_bytes(A, N));
  }
  return ROSKO_OK;
}

int32_t rosko_spmm_backward(const rosko_packed* A, const rosko_packed* At, const float* B,
                            int64_t ldb, const float* dC, int64_t lddc, int64_t N, float* dB,
                            int64_t lddb, float* dA_val, int64_t dA_cap, void* ws,
                            size_t ws_bytes, void* stream) {
  clear_error();
  int32_t st = check_packed_for_read(A);
  if (st) return st;
  RK_REQUIRE(N >= 0, ROSKO_EINVAL, "negative N");
  RK_REQUIRE(lddc >= N && lddc >= 1, ROSKO_EINVAL, "lddc < N");
  RK_REQUIRE(dC != nullptr || A->M == 0 || N == 0, ROSKO_EINVAL, "dC is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dB) {
    if ((st = check_packed_for_read(At))) return st;
    RK_REQUIRE(At->M == A->K && At->K == A->M, ROSKO_EINVAL,
               "At is %lld x %lld, expected %lld x %lld", (long long)At->M, (long long)At->K,
               (long long)A->K, (long long)A->M);
    RK_REQUIRE(At->val_dtype == ROSKO_F32, ROSKO_EUNSUPPORTED, "At must hold FP32 values");
    RK_REQUIRE(lddb >= N && lddb >= 1, ROSKO_EINVAL, "lddb < N");
    if (At->M > 0 && N > 0) {
      rosko_plan p = auto_plan(At, N);
      (void)hipGetLastError();
      if ((st = launch_spmm_sparse(At, dC, ROSKO_F32, N, lddc, dB, lddb, 0, p,
                                   static_cast<float*>(ws), ws_bytes, s)))
        return st;
    }
  }
  if (dA_val) {
    RK_REQUIRE(ldb >= N && ldb >= 1, ROSKO_EINVAL, "ldb < N");
    RK_REQUIRE(B != nullptr || A->K == 0 || N == 0, ROSKO_EINVAL, "B is null");
    RK_REQUIRE(dA_cap >= 0, ROSKO_EINVAL, "negative dA capacity");
    (void)hipGetLastError();
    if ((st = launch_sddmm(A, dC, lddc, B, ldb, N, dA_val, dA_cap, static_cast<float*>(ws),
                             ws_bytes, s)))
      return st;
  }
  return ROSKO_OK;
}

int32_t rosko_scatter_dense(const rosko_packed* A, const float* vals, int64_t n_vals,
                            float* out, int64_t ldo, void* stream) {
  clear_error();
  int32_t st = check_packed_for_read(A);
  if (st) return st;
  RK_REQUIRE(n_vals >= 0, ROSKO_EINVAL, "negative value count");
  RK_REQUIRE(ldo >= A->K && ldo >= 1, ROSKO_EINVAL, "ldo %lld < K %lld", (long long)ldo,
             (long long)A->K);
  if (A->M == 0 || A->K == 0 || n_vals == 0) return ROSKO_OK;
  RK_REQUIRE(vals != nullptr && out != nullptr, ROSKO_EINVAL, "null argument");
  (void)hipGetLastError();
  return launch_scatter_dense(A, vals, n_vals, out, ldo, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------- direct convolution

static int32_t check_conv_shape(int64_t C_in, int64_t H, int64_t W) {
  RK_REQUIRE(C_in >= 1 && H >= 1 && W >= 1, ROSKO_EINVAL, "convolution sizes must be >= 1");
  RK_REQUIRE(C_in < (int64_t(1) << 20) && H < (int64_t(1) << 20) && W < (int64_t(1) << 20),
             ROSKO_EUNSUPPORTED, "convolution sizes too large");
  const ConvGeom g = conv_geometry(C_in, H, W);
  RK_REQUIRE(4 * g.T < (int64_t(1) << 24), ROSKO_EUNSUPPORTED,
             "the padded input (4 x %lld elements) exceeds the records' 24-bit column field",
             (long long)g.T);
  return ROSKO_OK;
}

int32_t rosko_conv_geometry(int32_t C_in, int32_t H, int32_t W, int64_t* Wq, int64_t* T) {
  clear_error();
  RK_REQUIRE(Wq && T, ROSKO_EINVAL, "null argument");
  int32_t st = check_conv_shape(C_in, H, W);
  if (st) return st;
  const ConvGeom g = conv_geometry(C_in, H, W);
  *Wq = g.Wq;
  *T = g.T;
  return ROSKO_OK;
}

int32_t rosko_conv_input(const float* X, int32_t C_in, int32_t H, int32_t W, float* Bc,
                         void* stream) {
  clear_error();
  int32_t st = check_conv_shape(C_in, H, W);
  if (st) return st;
  RK_REQUIRE(X && Bc, ROSKO_EINVAL, "null argument");
  (void)hipGetLastError();
  return launch_conv_input(X, C_in, H, W, Bc, s_of(stream));
}

int32_t rosko_conv_records(const rosko_packed* A, int32_t C_in, int32_t H, int32_t W,
                           uint32_t* rec_out, int64_t rec_cap, void* stream) {
  clear_error();
  int32_t st = check_packed_for_read(A);
  if (st) return st;
  if ((st = check_conv_shape(C_in, H, W))) return st;
  RK_REQUIRE(A->K == 9 * (int64_t)C_in, ROSKO_EINVAL, "A has %lld columns, expected 9 x %d",
             (long long)A->K, C_in);
  RK_REQUIRE(A->nrec >= 0, ROSKO_EINVAL, "A's record count is not known (pack result first)");
  const int64_t nrec = std::min(A->nrec, A->nrec_cap);
  RK_REQUIRE(rec_cap >= nrec, ROSKO_ESMALLBUF, "rec_out holds %lld records < %lld",
             (long long)rec_cap, (long long)nrec);
  RK_REQUIRE(nrec == 0 || rec_out != nullptr, ROSKO_EINVAL, "rec_out is null");
  (void)hipGetLastError();
  return launch_conv_records(A, nrec, C_in, H, W, rec_out, s_of(stream));
}

int32_t rosko_conv_workspace_size(const rosko_packed* A, int32_t H, int32_t W,
                                  const rosko_plan* plan, size_t* bytes) {
  clear_error();
  RK_REQUIRE(A != nullptr && bytes != nullptr, ROSKO_EINVAL, "null argument");
  *bytes = 0;
  int32_t st = check_mr(A->mr);
  if (st) return st;
  RK_REQUIRE(A->K % 9 == 0 && A->K > 0, ROSKO_EINVAL, "A's columns are not 9 x C_in");
  if ((st = check_conv_shape(A->K / 9, H, W))) return st;
  const int64_t N = conv_geometry(A->K / 9, H, W).N;
  rosko_plan p = plan ? *plan : auto_plan(A, N);
  RK_REQUIRE(p.path != ROSKO_PATH_DENSE, ROSKO_EUNSUPPORTED,
             "the direct convolution runs on the sparse path");
  if ((st = normalize_plan(A, N, &p))) return st;
  *bytes = spmm_ws_bytes(A, N, p);
  return ROSKO_OK;
}

int32_t rosko_conv(const rosko_packed* A, const uint32_t* rec_conv, const float* Bc,
                   int32_t C_in, int32_t H, int32_t W, float* Yq, int64_t ldy, int32_t beta,
                   const rosko_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int32_t st = check_packed_for_read(A);
  if (st) return st;
  if ((st = check_conv_shape(C_in, H, W))) return st;
  RK_REQUIRE(A->K == 9 * (int64_t)C_in, ROSKO_EINVAL, "A has %lld columns, expected 9 x %d",
             (long long)A->K, C_in);
  RK_REQUIRE(beta == 0 || beta == 1, ROSKO_EINVAL, "beta must be 0 or 1");
  const ConvGeom g = conv_geometry(C_in, H, W);
  RK_REQUIRE(ldy >= g.N, ROSKO_EINVAL, "ldy %lld < H * Wq = %lld", (long long)ldy,
             (long long)g.N);
  RK_REQUIRE(A->M == 0 || (Yq && Bc && (rec_conv || A->nrec_cap == 0)), ROSKO_EINVAL,
             "null argument");
  rosko_plan p = plan ? *plan : auto_plan(A, g.N);
  RK_REQUIRE(p.path != ROSKO_PATH_DENSE, ROSKO_EUNSUPPORTED,
             "the direct convolution runs on the sparse path");
  if ((st = normalize_plan(A, g.N, &p))) return st;
  if (A->M == 0) return ROSKO_OK;
  (void)hipGetLastError();
  return launch_spmm_sparse_flat(A, rec_conv, Bc, 4 * g.T, g.N, Yq, ldy, beta, p,
                                 static_cast<float*>(ws), ws_bytes, s_of(stream));
}

int32_t rosko_conv_unpad(const float* Yq, int64_t ldy, int64_t C_out, int32_t H, int32_t W,
                         float* Y, void* stream) {
  clear_error();
  RK_REQUIRE(C_out >= 0 && H >= 1 && W >= 1, ROSKO_EINVAL, "bad size");
  const int64_t Wq = conv_geometry(1, H, W).Wq;
  RK_REQUIRE(ldy >= H * Wq, ROSKO_EINVAL, "ldy < H * Wq");
  if (C_out == 0) return ROSKO_OK;
  RK_REQUIRE(Yq && Y, ROSKO_EINVAL, "null argument");
  (void)hipGetLastError();
  return launch_conv_unpad(Yq, ldy, C_out, H, W, Wq, Y, s_of(stream));
}

// ---------------------------------------------------------- scheduler

int32_t rosko_features_workspace_size(int64_t M, int64_t K, size_t* bytes) {
  clear_error();
  RK_REQUIRE(bytes != nullptr, ROSKO_EINVAL, "bytes is null");
  RK_REQUIRE(M >= 0 && K >= 0, ROSKO_EINVAL, "negative size");
  *bytes = features_ws_bytes(M, K);
  return ROSKO_OK;
}

int32_t rosko_features(const float* A, int64_t M, int64_t K, int64_t lda, int64_t N, void* ws,
                       size_t ws_bytes, float* features, void* stream) {
  clear_error();
  int32_t st = check_dense(A, M, K, lda, "A");
  if (st) return st;
  RK_REQUIRE(M >= 1 && K >= 1 && N >= 1, ROSKO_EINVAL, "features need M, K, N >= 1");
  RK_REQUIRE(M <= (int64_t(1) << 21), ROSKO_EUNSUPPORTED, "M = %lld > 2^21", (long long)M);
  RK_REQUIRE(features != nullptr, ROSKO_EINVAL, "features is null");
  const size_t need = features_ws_bytes(M, K);
  RK_REQUIRE(ws != nullptr && ws_bytes >= need, ROSKO_ESMALLBUF,
             "features workspace %zu bytes < %zu", ws_bytes, need);
  RK_REQUIRE((uintptr_t)ws % 256 == 0, ROSKO_EINVAL, "features workspace must be 256-byte aligned");
  (void)hipGetLastError();
  return launch_features(A, M, K, lda, N, ws, features, static_cast<hipStream_t>(stream));
}

static int32_t check_mlp_dims(int32_t F, int32_t H, int32_t C) {
  RK_REQUIRE(F >= 1 && H >= 1 && C >= 1 && F <= 4096 && H <= 4096 && C <= 4096, ROSKO_EINVAL,
             "network sizes F=%d H=%d C=%d outside 1..4096", F, H, C);
  return ROSKO_OK;
}

int32_t rosko_mlp_param_count(int32_t F, int32_t H, int32_t C, int64_t* n) {
  clear_error();
  int32_t st = check_mlp_dims(F, H, C);
  if (st) return st;
  RK_REQUIRE(n != nullptr, ROSKO_EINVAL, "n is null");
  *n = (int64_t)F * H + H + (int64_t)H * H + H + (int64_t)H * C + C;
  return ROSKO_OK;
}

int32_t rosko_mlp_normalize(const float* X, int64_t batch, int32_t F, const float* mu,
                            const float* sigma, float* Xn, void* stream) {
  clear_error();
  RK_REQUIRE(batch >= 0 && F >= 1, ROSKO_EINVAL, "bad sizes");
  if (batch == 0) return ROSKO_OK;
  RK_REQUIRE(X && mu && sigma && Xn, ROSKO_EINVAL, "null argument");
  (void)hipGetLastError();
  return launch_normalize(X, batch, F, mu, sigma, Xn, static_cast<hipStream_t>(stream));
}

int32_t rosko_mlp_forward(const float* params, int32_t F, int32_t H, int32_t C, const float* X,
                          int64_t batch, float* H1, float* H2, float* Y, void* stream) {
  clear_error();
  int32_t st = check_mlp_dims(F, H, C);
  if (st) return st;
  RK_REQUIRE(batch >= 0, ROSKO_EINVAL, "negative batch");
  if (batch == 0) return ROSKO_OK;
  RK_REQUIRE(params && X && H1 && H2 && Y, ROSKO_EINVAL, "null argument");
  (void)hipGetLastError();
  return launch_mlp_forward(params, F, H, C, X, batch, H1, H2, Y,
                            static_cast<hipStream_t>(stream));
}

int32_t rosko_mlp_backward(const float* params, int32_t F, int32_t H, int32_t C, const float* X,
                           const float* H1, const float* H2, const float* Y, const float* T,
                           const float* mask, int64_t batch, float* grads, float* ws,
                           float* loss, void* stream) {
  clear_error();
  int32_t st = check_mlp_dims(F, H, C);
  if (st) return st;
  RK_REQUIRE(batch >= 1, ROSKO_EINVAL, "batch must be >= 1");
  RK_REQUIRE(params && X && H1 && H2 && Y && T && mask && grads && ws && loss, ROSKO_EINVAL,
             "null argument");
  (void)hipGetLastError();
  return launch_mlp_backward(params, F, H, C, X, H1, H2, Y, T, mask, batch, grads, ws, loss,
                             static_cast<hipStream_t>(stream));
}

int32_t rosko_adam_step(float* params, const float* grads, float* m, float* v, int64_t n,
                        float lr, float beta1, float beta2, float eps, int32_t t, void* stream) {
  clear_error();
  RK_REQUIRE(n >= 0 && t >= 1, ROSKO_EINVAL, "need n >= 0 and t >= 1");
  RK_REQUIRE(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f,
             ROSKO_EINVAL, "bad Adam constants");
  if (n == 0) return ROSKO_OK;
  RK_REQUIRE(params && grads && m && v, ROSKO_EINVAL, "null argument");
  (void)hipGetLastError();
  return launch_adam(params, grads, m, v, n, lr, beta1, beta2, eps, t,
                     static_cast<hipStream_t>(stream));
}

int32_t rosko_argmin_rows(const float* Y, int64_t batch, int32_t C, int32_t* out, void* stream) {
  clear_error();
  RK_REQUIRE(batch >= 0 && C >= 1, ROSKO_EINVAL, "bad sizes");
  if (batch == 0) return ROSKO_OK;
  RK_REQUIRE(Y && out, ROSKO_EINVAL, "null argument");
  (void)hipGetLastError();
  return launch_argmin(Y, batch, C, out, static_cast<hipStream_t>(stream));
}

int32_t rosko_sched_candidate(int32_t index, int32_t* mr, rosko_plan* plan) {
  clear_error();
  static const int32_t kMr[ROSKO_SCHED_CANDIDATES] = {8, 16, 32, 32, 64, 128, 32};
  static const int32_t kV[ROSKO_SCHED_CANDIDATES] = {4, 4, 4, 2, 2, 1, 0};
  RK_REQUIRE(index >= 0 && index < ROSKO_SCHED_CANDIDATES, ROSKO_EINVAL,
             "candidate %d outside 0..%d", index, ROSKO_SCHED_CANDIDATES - 1);
  RK_REQUIRE(mr && plan, ROSKO_EINVAL, "null argument");
  *mr = kMr[index];
  plan->path = kV[index] ? ROSKO_PATH_SPARSE : ROSKO_PATH_DENSE;
  plan->cols_per_lane = kV[index];
  plan->waves_per_tile = 0;
  plan->k_split = 0;
  plan->depth = 0;
  return ROSKO_OK;
}

int32_t rosko_sched_analytic(const float* f, int32_t* index) {
  clear_error();
  RK_REQUIRE(f && index, ROSKO_EINVAL, "null argument");
  // A 3 x 3 table over density d = f[3] (bands at 0.02 and 0.3) and log2 N
  // = f[2] (bands at 6 and 11), each cell the candidate with the smallest
  // geometric-mean time (repack + SpMM) over the training problems of the
  // random-shape corpus in that cell: short columns (few values per record)
  // take shorter panels, wide B on dense-ish matrices the matrix cores.
  static const int32_t kTable[3][3] = {{0, 1, 3}, {1, 3, 3}, {1, 3, 6}};
  const float d = f[3], lN = f[2];
  const int db = d < 0.02f ? 0 : (d < 0.3f ? 1 : 2);
  const int nb = lN < 6.0f ? 0 : (lN < 11.0f ? 1 : 2);
  *index = kTable[db][nb];
  return ROSKO_OK;
}

// The value-type rule (see rosko.h): products the BF16 matrix cores can
// take (BF16 or FP8 values times a BF16 B) go dense from this density up.
constexpr float kBf16DenseDensity = 0.015f;
constexpr int32_t kDenseCandidate = ROSKO_SCHED_CANDIDATES - 1;

int32_t rosko_sched_precision(const float* f, int32_t val_dtype, int32_t b_dtype,
                              int32_t* index) {
  clear_error();
  RK_REQUIRE(f && index, ROSKO_EINVAL, "null argument");
  RK_REQUIRE(val_dtype == ROSKO_F32 || val_dtype == ROSKO_BF16 ||
                 val_dtype == ROSKO_FP8_E4M3,
             ROSKO_EINVAL, "value dtype %d", val_dtype);
  RK_REQUIRE(b_dtype == ROSKO_F32 || b_dtype == ROSKO_BF16, ROSKO_EINVAL, "B dtype %d",
             b_dtype);
  if (val_dtype != ROSKO_F32 && b_dtype == ROSKO_BF16 && f[3] >= kBf16DenseDensity)
    *index = kDenseCandidate;
  return ROSKO_OK;
}

// Host forward pass of the plan network and its arg-min (see rosko.h).
int32_t rosko_plan_select(const float* f, const float* params, const float* mu,
                          const float* sigma, int32_t val_dtype, int32_t b_dtype,
                          int32_t* index, int32_t* mr, rosko_plan* plan) {
  clear_error();
  RK_REQUIRE(f && index && mr && plan, ROSKO_EINVAL, "null argument");
  int32_t c = 0;
  if (params == nullptr) {
    int32_t st = rosko_sched_analytic(f, &c);
    if (st) return st;
  } else {
    RK_REQUIRE(mu && sigma, ROSKO_EINVAL, "network given without its normalisation");
    constexpr int F = ROSKO_NFEAT, H = 64, Cn = ROSKO_SCHED_CANDIDATES;
    const float* W1 = params;
    const float* b1 = W1 + F * H;
    const float* W2 = b1 + H;
    const float* b2 = W2 + H * H;
    const float* W3 = b2 + H;
    const float* b3 = W3 + H * Cn;
    float x[F], h1[H], h2[H];
    for (int i = 0; i < F; ++i) x[i] = (f[i] - mu[i]) / sigma[i];
    for (int j = 0; j < H; ++j) {
      float a = b1[j];
      for (int i = 0; i < F; ++i) a += x[i] * W1[i * H + j];
      h1[j] = a > 0.0f ? a : 0.0f;
    }
    for (int j = 0; j < H; ++j) {
      float a = b2[j];
      for (int i = 0; i < H; ++i) a += h1[i] * W2[i * H + j];
      h2[j] = a > 0.0f ? a : 0.0f;
    }
    float best = 0.0f;
    for (int j = 0; j < Cn; ++j) {
      float a = b3[j];
      for (int i = 0; i < H; ++i) a += h2[i] * W3[i * Cn + j];
      if (j == 0 || a < best) {
        best = a;
        c = j;
      }
    }
  }
  int32_t st = rosko_sched_precision(f, val_dtype, b_dtype, &c);
  if (st) return st;
  *index = c;
  return rosko_sched_candidate(c, mr, plan);
}

}  // extern "C"
