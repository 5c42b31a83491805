// The Woodbury-kinetic matrix S(E) = I + K_diag^-1 V (Sec. 3.3, Type 3) in
// the channel-major order of C(E):
//
//   S[(c,i),(c',j)] = delta_cc' delta_ij + (1/h) kinv_ij Vd_cc'(r_j),
//   Vd_cc'(r_j) = V_cc'(r_j) + delta_cc' (h l_c(l_c+1)/r_j^2 + eps_c - E).
//
// Every element is non-zero in general (a dense matrix, like C(E) only in
// its diagonal blocks).  One workgroup per (row channel c, tile of kTileC
// column channels): the tile's Vd_cc'(r_j) for all j are staged in LDS by
// coalesced reads along c' (V is stored [j][c][c']), then the workgroup
// writes rows (c, 0..nr-1), each a contiguous run of kTileC * nr elements,
// in 256-element strips.  Bound by HBM writes (N^2 elements), like the
// assembly of C(E).
#include "common.h"

namespace hp {

constexpr int kTileC = 8;

template <typename T>
__global__ __launch_bounds__(256) void schur_build_kernel(int nc, int nr, double h, double E,
                                                          const double *__restrict__ kinv,
                                                          const double *__restrict__ r,
                                                          const int *__restrict__ l,
                                                          const double *__restrict__ eps,
                                                          const double *__restrict__ v,
                                                          cplx<T> *__restrict__ S, long lds) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<double> *vd = reinterpret_cast<cplx<double> *>(smem_raw);  // [nr][kTileC]
  const int c = blockIdx.y;
  const int c0 = blockIdx.x * kTileC;
  const int tc = min(kTileC, nc - c0);
  const int lc = l[c];
  const double shift = eps[c] - E;
  const double inv_h = 1.0 / h;
  for (int e = threadIdx.x; e < nr * kTileC; e += 256) {
    const int j = e / kTileC, k = e - j * kTileC;
    cplx<double> x{0.0, 0.0};
    if (k < tc) {
      const long o = 2 * (((long)j * nc + c) * nc + c0 + k);
      x = cplx<double>{v[o], v[o + 1]};
      if (c0 + k == c) {
        const double rj = r[j];
        x.re += h * (double)lc * (double)(lc + 1) / (rj * rj) + shift;
      }
    }
    vd[e] = cplx<double>{x.re * inv_h, x.im * inv_h};
  }
  __syncthreads();
  const int width = tc * nr;  // columns (c0.., all j) of this tile
  for (int i = 0; i < nr; ++i) {
    const double *krow = kinv + (long)i * nr;
    cplx<T> *out = S + ((long)c * nr + i) * lds + (long)c0 * nr;
    for (int e = threadIdx.x; e < width; e += 256) {
      const int k = e / nr, j = e - k * nr;
      const double kij = krow[j];
      const cplx<double> d = vd[j * kTileC + k];
      double re = kij * d.re, im = kij * d.im;
      if (c0 + k == c && j == i) re += 1.0;
      out[e] = cplx<T>{(T)re, (T)im};
    }
  }
}

}  // namespace hp

using namespace hp;

extern "C" int hp_build_schur(const hp_system *sys, double E, int prec, const double *kinv, void *S, long lds,
                              void *stream) {
  if (!sys || !S || !kinv || !sys->r || !sys->l || !sys->eps || !sys->v) return HP_ERR_ARG;
  if (sys->nc < 1 || sys->nr < 1 || !prec_ok(prec) || !(sys->hbar2_2mu != 0.0)) return HP_ERR_ARG;
  if (sys->vnl) return HP_ERR_UNSUPPORTED;  // the form needs local potentials
  const long n = (long)sys->nc * sys->nr;
  if (lds < n) return HP_ERR_ARG;
  const size_t shm = (size_t)sys->nr * kTileC * sizeof(cplx<double>);
  if (shm > 150 * 1024) return HP_ERR_UNSUPPORTED;
  if (sys->nc > 65535) return HP_ERR_UNSUPPORTED;  // grid y
  hipStream_t st = (hipStream_t)stream;
  dim3 grid((unsigned)((sys->nc + kTileC - 1) / kTileC), (unsigned)sys->nc), block(256);
  const double elt = is_c64(prec) ? 8.0 : 16.0;
  TraceScope ts(TR_ASSEMBLE, st, 0.0, elt * (double)n * (double)n);
  int rc;
  if (prec == HP_C128) {
    if ((rc = ensure_dynamic_lds((const void *)schur_build_kernel<double>, shm))) return rc;
    hipLaunchKernelGGL(schur_build_kernel<double>, grid, block, shm, st, sys->nc, sys->nr, sys->hbar2_2mu, E, kinv,
                       sys->r, sys->l, sys->eps, sys->v, (cplx<double> *)S, lds);
  } else {
    if ((rc = ensure_dynamic_lds((const void *)schur_build_kernel<float>, shm))) return rc;
    hipLaunchKernelGGL(schur_build_kernel<float>, grid, block, shm, st, sys->nc, sys->nr, sys->hbar2_2mu, E, kinv,
                       sys->r, sys->l, sys->eps, sys->v, (cplx<float> *)S, lds);
  }
  HP_CHECK_LAUNCH();
  return HP_OK;
}
