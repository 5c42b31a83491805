// C entry points that are not tied to one kernel family: workspace sizing,
// the factorization and general solve wrappers, error strings.
#include "common.h"

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>

namespace hp {

namespace {
thread_local char g_last_error[256] = "";
std::mutex g_lds_mu;
std::map<const void *, size_t> g_lds_set;
}  // namespace

void note_hip_error(hipError_t e, const char *file, int line) {
  const char *base = file;
  for (const char *p = file; *p; ++p)
    if (*p == '/') base = p + 1;
  snprintf(g_last_error, sizeof(g_last_error), "%s:%d: %s", base, line, hipGetErrorString(e));
}

int ensure_dynamic_lds(const void *func, size_t bytes) {
  if (bytes <= 64 * 1024) return HP_OK;
  std::lock_guard<std::mutex> lk(g_lds_mu);
  size_t &cur = g_lds_set[func];
  if (cur >= bytes) return HP_OK;
  HP_CHECK_HIP(hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  cur = bytes;
  return HP_OK;
}

Workspace plan_workspace(int n, int nrhs, int prec) {
  Workspace w{};
  const size_t A = 256;
  const size_t elt = is_c64(prec) ? sizeof(cplx<float>) : sizeof(cplx<double>);
  size_t off = 0;
  w.sync_off = off;
  w.sync_bytes = align_up(factor_sync_bytes(std::max(n, 1)), A);
  off += w.sync_bytes;
  w.slot_off = off;
  w.slot_bytes = align_up(factor_slot_bytes(), A);
  off += w.slot_bytes;
  w.flag_off = off;
  off += A;
  w.rhs_off = off;
  w.rhs_bytes = align_up((size_t)n * std::max(nrhs, 1) * std::max(elt, sizeof(cplx<double>)), A);
  off += w.rhs_bytes;
  w.res_off = off;
  w.res_bytes = align_up((size_t)n * std::max(nrhs, 1) * sizeof(cplx<double>), A);
  off += w.res_bytes;
  w.aux_off = off;
  w.aux_bytes = align_up((size_t)std::max(nrhs, 1) * std::max(nrhs, 1) * sizeof(cplx<double>), A);
  off += w.aux_bytes;
  w.red_off = off;
  w.red_bytes = align_up((size_t)std::max(nrhs, 1) * 64 + 4096, A);
  off += w.red_bytes;
  w.inv_off = off;
  w.inv_bytes = align_up(inverse_bytes(n, prec), A);
  off += w.inv_bytes;
  if (is_c64(prec)) {
    w.u12_off = off;
    w.u12_bytes = align_up((size_t)kInvBlock * n * sizeof(cplx<float>), A);
    off += w.u12_bytes;
  }
  if (is_c64(prec) && nrhs > 0) {
    w.wv_off = off;
    w.wv_bytes = align_up(wform_bytes(n), A);
    off += w.wv_bytes;
    w.inv2_off = off;
    w.inv2_bytes = align_up(wform_inv_bytes(n), A);
    off += w.inv2_bytes;
    w.z_off = off;
    w.z_bytes = align_up((size_t)n * nrhs * sizeof(cplx<float>), A);
    off += w.z_bytes;
    w.wtmp_off = off;
    w.wtmp_bytes = align_up(wform_tmp_bytes(n), A);
    off += w.wtmp_bytes;
  }
  w.h3 = prec == HP_C64H;
  if (w.h3) {  // the trailing update's operands: at most n rows of L21 and n columns of U12, K = kOuterBlock
    w.h3_bytes = h3_operand_bytes(n, kOuterBlock);
    w.h3a_off = off;
    off += w.h3_bytes;
    w.h3b_off = off;
    off += w.h3_bytes;
  }
  w.total = off;
  return w;
}

}  // namespace hp

using namespace hp;

extern "C" size_t hp_workspace_bytes(int n, int nrhs, int prec) {
  if (n < 1 || nrhs < 0 || !prec_ok(prec)) return 0;
  return plan_workspace(n, nrhs, prec).total;
}

extern "C" int hp_factor(int n, int prec, void *A, long lda, int *ipiv, int *perm, int *info, void *work,
                         size_t work_bytes, void *stream) {
  if (n < 1 || !A || !ipiv || !perm || !info || !work || lda < n) return HP_ERR_ARG;
  if (!prec_ok(prec)) return HP_ERR_ARG;
  Workspace ws = plan_workspace(n, 0, prec);
  if (work_bytes < ws.total) return HP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (prec == HP_C128)
    return lu_factor<double>(n, (cplx<double> *)A, lda, ipiv, perm, info, (char *)work, ws, st);
  return lu_factor<float>(n, (cplx<float> *)A, lda, ipiv, perm, info, (char *)work, ws, st);
}

extern "C" int hp_lu_solve(int n, int nrhs, int prec, const void *LU, long lda, const int *perm, void *X, long ldx,
                           void *work, size_t work_bytes, void *stream) {
  if (n < 1 || nrhs < 1 || !LU || !perm || !X || !work || lda < n || ldx < nrhs) return HP_ERR_ARG;
  if (!prec_ok(prec)) return HP_ERR_ARG;
  Workspace ws = plan_workspace(n, nrhs, prec);
  if (work_bytes < ws.total) return HP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)work;
  if (prec == HP_C128)
    return lu_solve<double>(n, nrhs, (const cplx<double> *)LU, lda, perm, (cplx<double> *)X, ldx,
                            (cplx<double> *)(w + ws.rhs_off), nullptr, st);
  return lu_solve<float>(n, nrhs, (const cplx<float> *)LU, lda, perm, (cplx<float> *)X, ldx,
                         (cplx<float> *)(w + ws.rhs_off), (cplx<float> *)(w + ws.inv_off), st);
}

extern "C" const char *hp_strerror(int code) {
  switch (code) {
    case HP_OK: return "ok";
    case HP_ERR_ARG: return "invalid argument";
    case HP_ERR_HIP: return "HIP runtime error";
    case HP_ERR_SINGULAR: return "exactly zero pivot";
    case HP_ERR_NOCONV: return "iterative refinement did not converge";
    case HP_ERR_WORKSPACE: return "workspace too small";
    case HP_ERR_UNSUPPORTED: return "unsupported case";
    case HP_ERR_SYNC: return "bounded inter-workgroup wait expired";
    default: return "unknown error";
  }
}

extern "C" const char *hp_last_error(void) { return g_last_error; }

extern "C" const char *hp_build_info(void) {
  return "hprmat gfx950: blocked right-looking complex LU (co-resident panel grid, MFMA trailing update: "
         "4M in FP64, 3M in FP32, split-FP16 4M x 3 in the FP16 variant), FP64/FP32 factors, device FP64 "
         "refinement; batched stepped LU for many small systems (no grid-wide waits)";
}
