// Refinement solves with an FP32 factor: the forward substitution in the
// transformed ("W") form.
//
// The refinement of Sec. 3.2 applies the same working-precision factors to a
// new right-hand side many times.  A blocked forward solve with 256-row blocks
// alternates a diagonal-block step (latency-bound: a few dozen workgroups)
// with a trailing GEMM that needs its result.  Here each block column of L
// below the diagonal is multiplied once, per hp_solve call, by the inverse of
// its diagonal block,
//   W_b = L[below b, b] Linv_b,
// and then, with Y holding P B,
//   Y[below b] -= W_b Y_b    for b = 0, 1, ...   (Y_b as it stands), then
//   Z_b = Linv_b Y_b         for every b at once,
// since L[below b, b] (Linv_b Y_b) = W_b Y_b.  The chain of the forward solve
// is then GEMMs only (K = 256) and its diagonal-block products one batched
// GEMM.  Building W costs about half a solve; the refinement runs many.
// L is unit lower triangular with entries of modulus <= 1 (partial pivoting),
// so W_b and Linv_b stay moderate.  The same transformation of U (whose
// diagonal blocks carry the pivots and can be far worse conditioned) raised
// the error of an unrefined FP32 solve by up to 2-4x on the optical-model
// systems, so the backward substitution keeps the inverted-block form
// (lu_solve_upper).
// Linv_b is assembled from the 128-row inverses of the factor's diagonal
// blocks: [[Lf, 0], [M, Ls]]^-1 = [[Lf^-1, 0], [-Ls^-1 M Lf^-1, Ls^-1]].
#include "common.h"

#include <algorithm>

namespace hp {

constexpr int kWBlock = 2 * kInvBlock;  // rows of a diagonal block of the transformed form

// W is stored packed: block column b (rows below it, 256 columns, leading
// dimension 256) after block column b - 1.  Only full 256-column blocks have
// rows below them.
static long w_offset(int n, int bi) {
  long off = 0;
  for (int j = 0; j < bi; ++j) off += (long)(n - (j + 1) * kWBlock) * kWBlock;
  return off;
}
size_t wform_bytes(int n) {
  const int nb2 = (n + kWBlock - 1) / kWBlock;
  return (size_t)w_offset(n, std::max(nb2 - 1, 0)) * sizeof(cplx<float>);
}
size_t wform_inv_bytes(int n) {
  const size_t nb = (size_t)(n + kWBlock - 1) / kWBlock;
  return nb * kWBlock * kWBlock * sizeof(cplx<float>);
}
size_t wform_tmp_bytes(int n) {
  const size_t nb = (size_t)(n + kWBlock - 1) / kWBlock;
  return nb * kInvBlock * kInvBlock * sizeof(cplx<float>);
}

// Diagonal quadrants of every 256-row inverse of L from the 128-row inverses
// (zero beyond the factor); the off-diagonal quadrants cleared (the GEMMs of
// wform_build fill the lower one).  One workgroup per 256-row block.
__global__ void inv256_fill_kernel(int nbt, const cplx<float> *__restrict__ inv, cplx<float> *__restrict__ inv2) {
  const int bi = blockIdx.x;
  const size_t iblk = (size_t)kInvBlock * kInvBlock;
  cplx<float> *out = inv2 + (size_t)bi * kWBlock * kWBlock;
  const int f = 2 * bi, s = 2 * bi + 1;  // 128-row blocks of this 256-row block
  const cplx<float> *If = inv + f * iblk;
  const cplx<float> *Is = s < nbt ? inv + s * iblk : nullptr;
  for (int e = threadIdx.x; e < kWBlock * kWBlock; e += blockDim.x) {
    const int r = e / kWBlock, c = e - r * kWBlock;
    cplx<float> v{0.f, 0.f};
    if (r < kInvBlock && c < kInvBlock)
      v = If[r * kInvBlock + c];
    else if (r >= kInvBlock && c >= kInvBlock && Is)
      v = Is[(r - kInvBlock) * kInvBlock + c - kInvBlock];
    out[e] = v;
  }
}

// From the 128-row inverses of L (inv: the output of solve_inverses for this
// factor, L blocks first) assembles the 256-row inverses (inv2,
// wform_inv_bytes) and forms W (wform_bytes).  tmp: wform_tmp_bytes.
int wform_build(int n, const cplx<float> *LU, long lda, const cplx<float> *inv, cplx<float> *inv2,
                cplx<float> *tmp, cplx<float> *W, hipStream_t st) {
  int rc;
  const int nbt = (n + kInvBlock - 1) / kInvBlock;
  const int nb2 = (n + kWBlock - 1) / kWBlock;
  const long iblk = (long)kInvBlock * kInvBlock, blk2 = (long)kWBlock * kWBlock;
  const int h = kInvBlock;
  hipLaunchKernelGGL(inv256_fill_kernel, dim3(nb2), dim3(256), 0, st, nbt, inv, inv2);
  HP_CHECK_LAUNCH();
  // lower quadrant -Ls^-1 (M Lf^-1): full 256-row blocks batched, a ragged last block alone
  const int nfull = n / kWBlock;
  if (nfull > 0) {
    const long sA = (long)kWBlock * lda + kWBlock;  // from one diagonal block of LU to the next
    if ((rc = gemm_set_batched<float>(h, h, h, 1.f, LU + (long)h * lda, lda, sA, inv, h, 2 * iblk, tmp, h, iblk,
                                      nfull, st)))
      return rc;
    if ((rc = gemm_set_batched<float>(h, h, h, -1.f, inv + iblk, h, 2 * iblk, tmp, h, iblk, inv2 + (long)h * kWBlock,
                                      kWBlock, blk2, nfull, st)))
      return rc;
  }
  if (nfull < nb2) {
    const int b = nfull * kWBlock, bs = n - b, b1 = std::min(h, bs), b2 = bs - b1;
    if (b2 > 0) {
      const long fb = 2L * nfull;  // 128-row block index of the first half
      if ((rc = gemm_set_batched<float>(b2, b1, b1, 1.f, LU + (long)(b + b1) * lda + b, lda, 0, inv + fb * iblk, h, 0,
                                        tmp, h, 0, 1, st)))
        return rc;
      if ((rc = gemm_set_batched<float>(b2, b1, b2, -1.f, inv + (fb + 1) * iblk, h, 0, tmp, h, 0,
                                        inv2 + nfull * blk2 + (long)h * kWBlock, kWBlock, 0, 1, st)))
        return rc;
    }
  }
  // W_b = L[below b, b] Linv_b
  for (int bi = 0; bi + 1 < nb2; ++bi) {
    const int b = bi * kWBlock;
    if ((rc = gemm_set_batched<float>(n - b - kWBlock, kWBlock, kWBlock, 1.f, LU + (long)(b + kWBlock) * lda + b, lda,
                                      0, inv2 + bi * blk2, kWBlock, 0, W + w_offset(n, bi), kWBlock, 0, 1, st)))
      return rc;
  }
  return HP_OK;
}

// Z (n x nrhs, leading dimension ldz) <- U^-1 L^-1 Y for Y (leading dimension
// ldy) holding P B; Y is overwritten (intermediate values).  LU, lda and inv
// (the 128-row inverses of L and U) are those given to wform_build, W and
// inv2 its outputs.
int wform_solve(int n, int nrhs, const cplx<float> *LU, long lda, const cplx<float> *inv, const cplx<float> *W,
                const cplx<float> *inv2, cplx<float> *Y, long ldy, cplx<float> *Z, long ldz, hipStream_t st) {
  int rc;
  const int nb2 = (n + kWBlock - 1) / kWBlock;
  const long blk2 = (long)kWBlock * kWBlock;
  for (int bi = 0; bi + 1 < nb2; ++bi) {
    const int b = bi * kWBlock;
    if ((rc = gemm_sub<float>(n - b - kWBlock, nrhs, kWBlock, W + w_offset(n, bi), kWBlock, Y + (long)b * ldy, ldy,
                              Y + (long)(b + kWBlock) * ldy, ldy, st)))
      return rc;
  }
  // Z_b = Linv_b Y_b for every block
  const int nfull = n / kWBlock;
  if (nfull > 0 && (rc = gemm_set_batched<float>(kWBlock, nrhs, kWBlock, 1.f, inv2, kWBlock, blk2, Y, ldy,
                                                 (long)kWBlock * ldy, Z, ldz, (long)kWBlock * ldz, nfull, st)))
    return rc;
  const int b = nfull * kWBlock, bs = n - b;
  if (bs > 0 && (rc = gemm_set_batched<float>(bs, nrhs, bs, 1.f, inv2 + nfull * blk2, kWBlock, 0, Y + (long)b * ldy,
                                              ldy, 0, Z + (long)b * ldz, ldz, 0, 1, st)))
    return rc;
  return lu_solve_upper<float>(n, nrhs, LU, lda, Z, ldz, inv, st);
}

}  // namespace hp
