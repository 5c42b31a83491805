// Coulomb functions and the collision matrix.
//
// F_l(eta, rho), G_l(eta, rho) and their rho-derivatives for the matching at
// the channel radius (the role of the paper's Coulomb routine, Sec. 4.1).
// Method (Steed's algorithm as used by Barnett's COULFG, with an inward
// integration below the barrier):
//  * CF1: f = F'/F by backward recurrence of the ratio of the minimal
//    solution in l (from the Abramowitz & Stegun 14.2 recurrences),
//      f_n = S_{n+1} - R_{n+1}^2 / (S_{n+1} + f_{n+1}),
//      S_n = n/rho + eta/n,  R_n^2 = 1 + eta^2/n^2,
//    started far above l; the signs of S_{n+1} + f_{n+1} = R_{n+1} F_n/F_{n+1}
//    give the sign of F_l.
//  * CF2: p + iq = (G' + iF')/(G + iF) as the continued fraction
//      i(1 - eta/rho) + (i/rho) K_n (a_n / b_n),
//      a_n = (i eta - l + n - 1)(i eta + l + n),  b_n = 2(rho - eta + n i),
//    by the modified Lentz method.
//  * With the Wronskian F'G - FG' = 1: F = w / sqrt(q (1 + g^2)),
//    g = (f - p)/q, G = g F, F' = f F, G' = (p g - q) F.
//  * Inside the Coulomb + centrifugal barrier (rho below the turning point
//    rho_t = eta + sqrt(eta^2 + l(l+1))), q is too small to carry F, so G and
//    G' are taken from Steed at rho_t + 2 and carried inward by Taylor
//    series of the Coulomb equation (G grows inward: stable), and
//    F = 1 / (f G - G') from the Wronskian with CF1 at rho.
//
// Collision matrix (matching u(a) = R a u'(a) with u_c = k_c^-1/2 (I_c delta -
// U O_c)):  U = (O - Rt O')^-1 (I - Rt I'),  Rt = rho^1/2 R rho^1/2.
#include "common.h"

#include <climits>
#include <cmath>
#include <mutex>
#include <vector>

namespace hp {

struct CoulombOut {
  double F, Fp, G, Gp;
  int status;  // 0 ok, 1 a continued fraction did not converge or a value left double range
};

// Far below the Coulomb barrier (large eta, rho well inside the turning
// point) F underflows and G overflows double range: reported, never returned
// as a value.
__host__ __device__ static void check_range(CoulombOut &o) {
  const bool finite = __builtin_isfinite(o.F) && __builtin_isfinite(o.Fp) && __builtin_isfinite(o.G) &&
                      __builtin_isfinite(o.Gp);
  if (!finite || o.F == 0.0) o.status = 1;
}

__host__ __device__ static double cf1_ratio(int L, double eta, double rho, double *sign) {
  const int ltop = L + (int)rho + 60;
  auto S = [&](int n) { return n / rho + eta / n; };
  auto R2 = [&](int n) { return 1.0 + (eta / n) * (eta / n); };
  double f = S(ltop + 1);
  double sg = 1.0;
  for (int n = ltop - 1; n >= L; --n) {
    double d = S(n + 1) + f;
    if (d == 0.0) d = 1e-300;
    if (d < 0.0) sg = -sg;
    f = S(n + 1) - R2(n + 1) / d;
  }
  *sign = sg;
  return f;
}

__host__ __device__ static int cf2_pq(int L, double eta, double rho, double *p, double *q) {
  // Lentz on K(a_n / b_n), complex arithmetic written out
  const double tiny = 1e-300;
  const cplx<double> a{-(double)L, eta}, b{(double)L + 1.0, eta};
  cplx<double> f{tiny, 0.0}, C = f, D{0.0, 0.0};
  int ok = 1;
  for (int n = 1; n < 200000; ++n) {
    const cplx<double> an = cmul(cplx<double>{a.re + n - 1, a.im}, cplx<double>{b.re + n - 1, b.im});
    const cplx<double> bn{2.0 * (rho - eta), 2.0 * n};
    D = cadd(bn, cmul(an, D));
    if (D.re == 0.0 && D.im == 0.0) D.re = tiny;
    C = cadd(bn, cdiv(an, C));
    if (C.re == 0.0 && C.im == 0.0) C.re = tiny;
    D = crcp(D);
    const cplx<double> delta = cmul(C, D);
    f = cmul(f, delta);
    const double dr = delta.re - 1.0, di = delta.im;
    if (dr * dr + di * di < 1e-32) {
      ok = 0;
      break;
    }
  }
  // i(1 - eta/rho) + (i/rho) f
  *p = -f.im / rho;
  *q = (1.0 - eta / rho) + f.re / rho;
  return ok;
}

__host__ __device__ static void steed(int L, double eta, double rho, CoulombOut &o) {
  double w;
  const double f = cf1_ratio(L, eta, rho, &w);
  double p, q;
  o.status = cf2_pq(L, eta, rho, &p, &q);
  const double g = (f - p) / q;
  const double F = w / sqrt(q * (1.0 + g * g));
  o.F = F;
  o.Fp = f * F;
  o.G = g * F;
  o.Gp = (p * g - q) * F;
}

// one Taylor step of u'' = (L(L+1)/x^2 + 2 eta/x + sigma) u from x0 to x0 + h
// (sigma = -1: the Coulomb equation of an open channel, x = rho; sigma = +1:
// a closed channel, x = kappa r).  With u = sum c_n t^n, t = x - x0, the
// equation times x^2 gives the three-term recurrence below.
__host__ __device__ static void taylor_step(double LL, double eta, double x0, double h, double &u, double &up,
                                            double sigma = -1.0) {
  double cm2 = 0.0, cm1 = 0.0, c0 = u, c1 = up;
  double s = u + up * h, sp = up;
  double hp = h;  // h^(n+1)
  const double A = LL + 2.0 * eta * x0 + sigma * x0 * x0;
  const double B = 2.0 * eta + 2.0 * sigma * x0;
  for (int n = 0; n < 300; ++n) {
    const double c2 = (A * c0 + B * cm1 + sigma * cm2 - 2.0 * x0 * (n + 1) * n * c1 - (double)n * (n - 1) * c0) /
                      (x0 * x0 * (n + 2.0) * (n + 1.0));
    const double dterm = (n + 2.0) * c2 * hp;  // (n+2) c_{n+2} h^(n+1)
    hp *= h;
    const double term = c2 * hp;               // c_{n+2} h^(n+2)
    s += term;
    sp += dterm;
    cm2 = cm1;
    cm1 = c0;
    c0 = c1;
    c1 = c2;
    if (n > 8 && fabs(term) <= 1e-18 * fabs(s) && fabs(dterm) <= 1e-18 * fabs(sp)) break;
  }
  u = s;
  up = sp;
}

// With scale: far inside the turning point G grows beyond double range on
// the way in; whenever |G| passes 1e150 the pair (G, G') is divided by |G|
// and the logarithm added to *scale, so the values returned are
// G~ = G e^-scale, G~' likewise and F~ = F e^scale = 1/(f G~ - G~') (the
// Wronskian with the scaled G).  Channels that never pass 1e150 come out
// exactly as unscaled, with *scale = 0.
__host__ __device__ static CoulombOut coulomb_fg_scaled(int L, double eta, double rho, double *scale) {
  CoulombOut o;
  *scale = 0.0;
  const double LL = (double)L * (L + 1);
  const double rtp = eta + sqrt(eta * eta + LL);
  if (rho >= rtp) {
    steed(L, eta, rho, o);
    check_range(o);
    return o;
  }
  double x = rtp + 2.0;
  steed(L, eta, x, o);
  double G = o.G, Gp = o.Gp, th = 0.0;
  while (x > rho) {
    double h = -fmin(1.0, fmin(0.25 * x, x - rho));
    taylor_step(LL, eta, x, h, G, Gp);
    x += h;
    const double m = fabs(G);
    if (m > 1e150) {
      G /= m;
      Gp /= m;
      th += log(m);
    }
  }
  double sg;
  const double f = cf1_ratio(L, eta, rho, &sg);
  const double F = 1.0 / (f * G - Gp);
  o.F = F;
  o.Fp = f * F;
  o.G = G;
  o.Gp = Gp;
  check_range(o);
  *scale = th;
  return o;
}

// Unscaled values; status 1 where they leave double range.
__host__ __device__ static CoulombOut coulomb_fg(int L, double eta, double rho) {
  double th;
  CoulombOut o = coulomb_fg_scaled(L, eta, rho, &th);
  if (th > 0.0) o.status = 1;
  return o;
}

// Closed channel: x W'(x) / W(x) at x = kappa a for the solution of
// u'' = (1 + L(L+1)/x^2 + 2 eta/x) u that decays outward (the Whittaker
// function W_{-eta, L+1/2}(2x)).  For eta >= 0 the coefficient is >= 1
// everywhere, so integrated inward that solution dominates the growing one
// by at least e^(2 dx): started kClosedSpan units further out with the local
// log-derivative -sqrt(coefficient) and carried inward by Taylor steps (the
// pair (u, u') renormalized after each step), the start's error is damped by
// e^(-2 kClosedSpan) at x.  Status 1 if the input is out of range.
constexpr double kClosedSpan = 40.0;
__host__ __device__ static double closed_logderiv(int L, double eta, double x, int *status) {
  *status = (x > 0.0 && eta >= 0.0) ? 0 : 1;
  if (*status) return 0.0;
  const double LL = (double)L * (L + 1);
  double xc = x + kClosedSpan;
  double u = 1.0, up = -sqrt(1.0 + LL / (xc * xc) + 2.0 * eta / xc);
  while (xc > x) {
    const double h = -fmin(1.0, fmin(0.25 * xc, xc - x));
    taylor_step(LL, eta, xc, h, u, up, 1.0);
    xc += h;
    const double m = fabs(u);
    u /= m;
    up /= m;
  }
  return x * up / u;
}

__global__ void coulomb_kernel(int nch, const int *__restrict__ l, const double *__restrict__ eta,
                               const double *__restrict__ rho, double *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  CoulombOut o = coulomb_fg(l[c], eta[c], rho[c]);
  out[4 * c + 0] = o.F;
  out[4 * c + 1] = o.Fp;
  out[4 * c + 2] = o.G;
  out[4 * c + 3] = o.Gp;
}

// Per channel: k, eta, rho, then (F, F', G, G'); status per channel in st[c]
// (0 ok, 2 continued fraction did not converge, 3 closed channel with its
// log-derivative L_c = a u'(a)/u(a) in fg[4c], 4 at a threshold or out of
// range, 6 open but far below its Coulomb barrier: fg holds the values
// scaled by e^-+theta[c] as coulomb_fg_scaled returns them).
__global__ void channel_kernel(int nc, double E, double h, double z1z2e2, double a, const int *__restrict__ l,
                               const double *__restrict__ eps, double *__restrict__ fg, double *__restrict__ sqrho,
                               double *__restrict__ theta, int *__restrict__ stat) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double ec = E - eps[c];
  theta[c] = 0.0;
  if (!(ec > 0.0)) {
    fg[4 * c] = fg[4 * c + 1] = fg[4 * c + 2] = fg[4 * c + 3] = 0.0;
    sqrho[c] = 0.0;
    if (!(ec < 0.0)) {
      stat[c] = 4;
      return;
    }
    const double kappa = sqrt(-ec / h);
    const double eta = z1z2e2 / (2.0 * h * kappa);
    int bad = 0;
    fg[4 * c] = closed_logderiv(l[c], eta, kappa * a, &bad);
    stat[c] = bad ? 4 : 3;
    return;
  }
  const double k = sqrt(ec / h);
  const double eta = z1z2e2 / (2.0 * h * k);
  const double rho = k * a;
  double th;
  CoulombOut o = coulomb_fg_scaled(l[c], eta, rho, &th);
  fg[4 * c + 0] = o.F;
  fg[4 * c + 1] = o.Fp;
  fg[4 * c + 2] = o.G;
  fg[4 * c + 3] = o.Gp;
  sqrho[c] = sqrt(rho);
  theta[c] = th;
  stat[c] = o.status ? 2 : (th > 0.0 ? 6 : 0);
}

// The matching with scaled channel values (some open channel far below its
// Coulomb barrier): with O = e^theta O~, O~ = G~ + i F~ e^-2theta (likewise
// O', I, I'), ZO = (diag O~ - Rt diag O~') E and ZI = ZO - 2i Q E with
// Q = diag F~ - Rt diag F~' and E = diag(e^theta), so
//   U = ZO^-1 ZI = I - 2i E^-1 (diag O~ - Rt diag O~')^-1 Q E^-1,
// every factor e^-theta <= 1.  This kernel writes ZO~ and Q E^-1 over the
// no open channels (oidx: their channel numbers, null for all; R at stride
// ldr indexed by open position).
__global__ void zmat_scaled_kernel(int no, const cplx<double> *__restrict__ R, long ldr, const double *__restrict__ fg,
                                   const double *__restrict__ sqrho, const double *__restrict__ theta,
                                   const int *__restrict__ oidx, cplx<double> *__restrict__ ZO,
                                   cplx<double> *__restrict__ ZQ) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)no * no) return;
  const int i = (int)(e / no), j = (int)(e - (long)i * no);
  const int c = oidx ? oidx[i] : i, cp = oidx ? oidx[j] : j;
  const double s = sqrho[c] * sqrho[cp];
  const cplx<double> r = R[(long)i * ldr + j];
  const cplx<double> rt{s * r.re, s * r.im};
  const double sc = exp(-2.0 * theta[cp]);
  const double Fp = fg[4 * cp + 1], Gp = fg[4 * cp + 3];
  cplx<double> zo = cmul(rt, cplx<double>{Gp, Fp * sc});
  zo = cplx<double>{-zo.re, -zo.im};
  cplx<double> q{-rt.re * Fp, -rt.im * Fp};
  if (i == j) {  // c == cp
    zo.re += fg[4 * c + 2];
    zo.im += fg[4 * c] * sc;
    q.re += fg[4 * c];
  }
  const double ej = exp(-theta[cp]);
  ZO[e] = zo;
  ZQ[e] = cplx<double>{q.re * ej, q.im * ej};
}

// U = I - 2i E^-1 Y in place (Y = ZO~^-1 Q E^-1, no x no).
__global__ void u_scaled_kernel(int no, const double *__restrict__ theta, const int *__restrict__ oidx,
                                cplx<double> *__restrict__ Y) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)no * no) return;
  const int i = (int)(e / no), j = (int)(e - (long)i * no);
  const double ei = exp(-theta[oidx ? oidx[i] : i]);
  const cplx<double> y = Y[e];
  // -2i ei y = (2 ei y.im, -2 ei y.re)
  cplx<double> u{2.0 * ei * y.im, -2.0 * ei * y.re};
  if (i == j) u.re += 1.0;
  Y[e] = u;
}

// ZO = diag(O) - Rt diag(O'), ZI = diag(I) - Rt diag(I'), both nc x nc row-major.
__global__ void zmat_kernel(int nc, const cplx<double> *__restrict__ R, const double *__restrict__ fg,
                            const double *__restrict__ sqrho, cplx<double> *__restrict__ ZO,
                            cplx<double> *__restrict__ ZI) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)nc * nc) return;
  const int c = (int)(e / nc), cp = (int)(e - (long)c * nc);
  const double s = sqrho[c] * sqrho[cp];
  const cplx<double> rt{s * R[e].re, s * R[e].im};
  const double F = fg[4 * cp], Fp = fg[4 * cp + 1], G = fg[4 * cp + 2], Gp = fg[4 * cp + 3];
  // Rt * O'_c' with O' = G' + i F', I' = G' - i F'
  cplx<double> zo = cmul(rt, cplx<double>{Gp, Fp});
  cplx<double> zi = cmul(rt, cplx<double>{Gp, -Fp});
  zo = cplx<double>{-zo.re, -zo.im};
  zi = cplx<double>{-zi.re, -zi.im};
  if (c == cp) {
    zo.re += G;
    zo.im += F;
    zi.re += G;
    zi.im -= F;
  }
  ZO[e] = zo;
  ZI[e] = zi;
}

// Closed channels (E < eps_c) are eliminated from u(a) = R a u'(a) through
// the open channels' effective R-matrix
//   R_eff = R_oo + R_oc L (I - R_cc L)^-1 R_co,   L = diag(a u_c'(a) / u_c(a)),
// the log-derivatives of the decaying external solutions (channel_kernel);
// U then follows over the open channels as above.  oidx / cidx list the open
// and closed channels; matrices packed row-major.
// Mcc = I - R_cc L (ncl x ncl) and Y = R_co (ncl x no).
__global__ void closed_mats_kernel(int nc, int ncl, int no, const cplx<double> *__restrict__ R,
                                   const double *__restrict__ fg, const int *__restrict__ cidx,
                                   const int *__restrict__ oidx, cplx<double> *__restrict__ Mcc,
                                   cplx<double> *__restrict__ Y) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nm = (long)ncl * ncl, ny = (long)ncl * no;
  if (e < nm) {
    const int i = (int)(e / ncl), j = (int)(e - (long)i * ncl);
    const double Lj = fg[4 * cidx[j]];
    const cplx<double> r = R[(long)cidx[i] * nc + cidx[j]];
    cplx<double> m{-r.re * Lj, -r.im * Lj};
    if (i == j) m.re += 1.0;
    Mcc[e] = m;
  } else if (e < nm + ny) {
    const long f = e - nm;
    const int i = (int)(f / no), j = (int)(f - (long)i * no);
    Y[f] = R[(long)cidx[i] * nc + oidx[j]];
  }
}

// R_eff = R_oo + R_oc L Y (no x no), Y = (I - R_cc L)^-1 R_co.
__global__ void reff_kernel(int nc, int ncl, int no, const cplx<double> *__restrict__ R,
                            const double *__restrict__ fg, const int *__restrict__ cidx,
                            const int *__restrict__ oidx, const cplx<double> *__restrict__ Y,
                            cplx<double> *__restrict__ Reff) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)no * no) return;
  const int i = (int)(e / no), j = (int)(e - (long)i * no);
  cplx<double> acc = R[(long)oidx[i] * nc + oidx[j]];
  for (int k = 0; k < ncl; ++k) {
    const double Lk = fg[4 * cidx[k]];
    const cplx<double> r = R[(long)oidx[i] * nc + cidx[k]];
    const cplx<double> y = Y[(long)k * no + j];
    acc.re += Lk * (r.re * y.re - r.im * y.im);
    acc.im += Lk * (r.re * y.im + r.im * y.re);
  }
  Reff[e] = acc;
}

// zmat_kernel over the open channels, from R_eff.
__global__ void zmat_open_kernel(int no, const cplx<double> *__restrict__ Reff, const double *__restrict__ fg,
                                 const double *__restrict__ sqrho, const int *__restrict__ oidx,
                                 cplx<double> *__restrict__ ZO, cplx<double> *__restrict__ ZI) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)no * no) return;
  const int i = (int)(e / no), j = (int)(e - (long)i * no);
  const int c = oidx[i], cp = oidx[j];
  const double s = sqrho[c] * sqrho[cp];
  const cplx<double> rt{s * Reff[e].re, s * Reff[e].im};
  const double F = fg[4 * cp], Fp = fg[4 * cp + 1], G = fg[4 * cp + 2], Gp = fg[4 * cp + 3];
  cplx<double> zo = cmul(rt, cplx<double>{Gp, Fp});
  cplx<double> zi = cmul(rt, cplx<double>{Gp, -Fp});
  zo = cplx<double>{-zo.re, -zo.im};
  zi = cplx<double>{-zi.re, -zi.im};
  if (i == j) {
    zo.re += G;
    zo.im += F;
    zi.re += G;
    zi.im -= F;
  }
  ZO[e] = zo;
  ZI[e] = zi;
}

__global__ void zero_c128_kernel(long n, cplx<double> *__restrict__ p) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = cplx<double>{0.0, 0.0};
}

// S[oidx[i]][oidx[j]] = U[i][j] (the rest of S was cleared).
__global__ void scatter_open_kernel(int nc, int no, const int *__restrict__ oidx, const cplx<double> *__restrict__ U,
                                    cplx<double> *__restrict__ S) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)no * no) return;
  const int i = (int)(e / no), j = (int)(e - (long)i * no);
  S[(long)oidx[i] * nc + oidx[j]] = U[e];
}

}  // namespace hp

using namespace hp;

extern "C" int hp_coulomb(int l, double eta, double rho, double *out) {
  if (l < 0 || !(rho > 0.0) || !(eta >= 0.0) || !out) return HP_ERR_ARG;
  CoulombOut o = coulomb_fg(l, eta, rho);
  out[0] = o.F;
  out[1] = o.Fp;
  out[2] = o.G;
  out[3] = o.Gp;
  return o.status ? HP_ERR_NOCONV : HP_OK;
}

extern "C" int hp_coulomb_device(int nch, const int *l, const double *eta, const double *rho, double *out,
                                 void *stream) {
  if (nch < 0 || (nch > 0 && (!l || !eta || !rho || !out))) return HP_ERR_ARG;
  if (nch == 0) return HP_OK;
  hipLaunchKernelGGL(coulomb_kernel, dim3((nch + 63) / 64), dim3(64), 0, (hipStream_t)stream, nch, l, eta, rho,
                     out);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

namespace hp {

// Gaussian elimination with partial pivoting (largest |Re| + |Im|, smallest
// row on ties) of the first n columns of the row-major n x w matrix z, the
// other columns carried along; all 256 threads of the workgroup take part.
// Returns 1 on an exactly zero pivot.
__device__ static int block_eliminate(cplx<double> *z, int n, int w, double *sv, int *sr) {
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int brow = INT_MAX;
    for (int r = k + tid; r < n; r += 256) {
      const double v = cabs1(z[(long)r * w + k]);
      if (v > best || (v == best && r < brow)) {
        best = v;
        brow = r;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int orow = __shfl_xor(brow, off);
      if (ov > best || (ov == best && orow < brow)) {
        best = ov;
        brow = orow;
      }
    }
    if ((tid & 63) == 0) {
      sv[tid >> 6] = best;
      sr[tid >> 6] = brow;
    }
    __syncthreads();
    best = sv[0];
    brow = sr[0];
    for (int q = 1; q < 4; ++q)
      if (sv[q] > best || (sv[q] == best && sr[q] < brow)) {
        best = sv[q];
        brow = sr[q];
      }
    __syncthreads();
    if (!(best > 0.0)) return 1;
    if (brow != k)
      for (int j = k + tid; j < w; j += 256) {
        const cplx<double> x = z[(long)k * w + j];
        z[(long)k * w + j] = z[(long)brow * w + j];
        z[(long)brow * w + j] = x;
      }
    __syncthreads();
    const cplx<double> inv = crcp(z[(long)k * w + k]);
    // rows below k: l = z_ik / z_kk, z_ij -= l z_kj (j > k); one thread per (i, j)
    const int rows = n - k - 1, cols = w - k - 1;
    for (int e = tid; e < rows * cols; e += 256) {
      const int i = k + 1 + e / cols, j = k + 1 + e % cols;
      const cplx<double> l = cmul(z[(long)i * w + k], inv);
      z[(long)i * w + j] = cfms(z[(long)i * w + j], l, z[(long)k * w + j]);
    }
    __syncthreads();
  }
  return 0;
}

// Back substitution after block_eliminate: out = U^-1 (right part of z,
// nrhs columns), one right-hand column per thread; row i / column cp of the
// result is stored at out[rmap[i] * ldo + cmap[cp]] (maps may be null for
// the identity).
__device__ static void block_back_substitute(const cplx<double> *z, int n, int w, int nrhs, cplx<double> *out,
                                             long ldo, const int *rmap, const int *cmap) {
  for (int cp = threadIdx.x; cp < nrhs; cp += 256) {
    const long oc = cmap ? cmap[cp] : cp;
    for (int i = n - 1; i >= 0; --i) {
      cplx<double> acc = z[(long)i * w + n + cp];
      for (int j = i + 1; j < n; ++j) acc = cfms(acc, z[(long)i * w + j], out[(rmap ? rmap[j] : j) * ldo + oc]);
      out[(rmap ? rmap[i] : i) * ldo + oc] = cdiv(acc, z[(long)i * w + i]);
    }
  }
}

// Collision matrices of a batch of systems (see hp_batch_smatrix), one
// workgroup per system: the channel functions into LDS (Coulomb functions of
// the open channels, decaying-solution log-derivatives L_c of the closed
// ones); with closed channels, Y = (I - R_cc L)^-1 R_co by elimination in the
// workspace and R_eff = R_oo + R_oc L Y into S's block (compact, no x no);
// then Z = [ZO | ZI] over the open channels from R (or R_eff) in the
// workspace at 2 r_off, Gaussian elimination with partial pivoting, and back
// substitution into S (at r_off), whose closed rows and columns are zero.
// status[s]: 0 ok, 1 no open channel or E at a threshold, 2 a continued
// fraction or a closed channel's integration failed, 3 an exactly zero pivot,
// 4 more than 512 channels.
constexpr int kBatchSmatMaxChannels = 512;

__global__ __launch_bounds__(256) void batch_smatrix_kernel(int count, const hp_batch_item *__restrict__ items,
                                                            const cplx<double> *__restrict__ R,
                                                            cplx<double> *__restrict__ S, cplx<double> *__restrict__ Z,
                                                            int *__restrict__ status) {
  __shared__ double fg[4 * kBatchSmatMaxChannels];
  __shared__ double sqrho[kBatchSmatMaxChannels];
  __shared__ double thl[kBatchSmatMaxChannels];  // scales of channels far below their barrier
  __shared__ int oidx[kBatchSmatMaxChannels], cidx[kBatchSmatMaxChannels];
  __shared__ double sv[4];
  __shared__ int sr[4];
  __shared__ int s_bad, s_no, s_ncl, s_scaled;
  const int sidx = blockIdx.x;
  if (sidx >= count) return;
  const hp_batch_item it = items[sidx];
  const hp_system &sys = it.sys;
  const int nc = sys.nc, tid = threadIdx.x;
  if (nc > kBatchSmatMaxChannels) {  // the channel table would not fit
    if (tid == 0) status[sidx] = 4;
    return;
  }
  if (tid == 0) s_bad = s_scaled = 0;
  __syncthreads();
  for (int c = tid; c < nc; c += 256) {
    const double ec = it.E - sys.eps[c];
    fg[4 * c] = fg[4 * c + 1] = fg[4 * c + 2] = fg[4 * c + 3] = 0.0;
    sqrho[c] = 0.0;
    thl[c] = 0.0;
    if (!(ec > 0.0)) {
      if (!(ec < 0.0)) {  // at the threshold (or NaN)
        atomicMax(&s_bad, 1);
        continue;
      }
      const double kappa = sqrt(-ec / sys.hbar2_2mu);
      const double eta = sys.z1z2e2 / (2.0 * sys.hbar2_2mu * kappa);
      int bad = 0;
      fg[4 * c] = closed_logderiv(sys.l[c], eta, kappa * sys.a, &bad);
      if (bad) atomicMax(&s_bad, 2);
      continue;
    }
    const double k = sqrt(ec / sys.hbar2_2mu);
    const double eta = sys.z1z2e2 / (2.0 * sys.hbar2_2mu * k);
    const double rho = k * sys.a;
    double th;
    const CoulombOut o = coulomb_fg_scaled(sys.l[c], eta, rho, &th);
    fg[4 * c + 0] = o.F;
    fg[4 * c + 1] = o.Fp;
    fg[4 * c + 2] = o.G;
    fg[4 * c + 3] = o.Gp;
    sqrho[c] = sqrt(rho);
    thl[c] = th;
    if (th > 0.0) atomicMax(&s_scaled, 1);
    if (o.status) atomicMax(&s_bad, 2);
  }
  __syncthreads();
  if (tid == 0) {  // open and closed channel lists, in channel order
    int no = 0, ncl = 0;
    for (int c = 0; c < nc; ++c) {
      if (it.E - sys.eps[c] > 0.0)
        oidx[no++] = c;
      else
        cidx[ncl++] = c;
    }
    s_no = no;
    s_ncl = ncl;
    if (no == 0) s_bad = max(s_bad, 1);
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) status[sidx] = s_bad;
    return;
  }
  const int no = s_no, ncl = s_ncl;
  const cplx<double> *Rs = R + it.r_off;
  cplx<double> *Ss = S + it.r_off;
  cplx<double> *z = Z + 2 * it.r_off;  // 2 nc^2 complex values of workspace
  // the open channels' R: R itself, or R_eff in S's block (ld no)
  const cplx<double> *Ro = Rs;
  long ldr = nc;
  if (ncl > 0) {
    // [I - R_cc L | R_co] (ncl x (ncl + no)), then Y after it (ncl x no)
    const int wa = ncl + no;
    for (int e = tid; e < ncl * wa; e += 256) {
      const int i = e / wa, j = e - i * wa;
      cplx<double> m;
      if (j < ncl) {
        const double Lj = fg[4 * cidx[j]];
        const cplx<double> r = Rs[(long)cidx[i] * nc + cidx[j]];
        m = cplx<double>{-r.re * Lj, -r.im * Lj};
        if (i == j) m.re += 1.0;
      } else {
        m = Rs[(long)cidx[i] * nc + oidx[j - ncl]];
      }
      z[e] = m;
    }
    __syncthreads();
    if (block_eliminate(z, ncl, wa, sv, sr)) {
      if (tid == 0) status[sidx] = 3;
      return;
    }
    cplx<double> *Y = z + (long)ncl * wa;
    block_back_substitute(z, ncl, wa, no, Y, no, nullptr, nullptr);
    __syncthreads();
    for (int e = tid; e < no * no; e += 256) {
      const int i = e / no, j = e - i * no;
      cplx<double> acc = Rs[(long)oidx[i] * nc + oidx[j]];
      for (int k = 0; k < ncl; ++k) {
        const double Lk = fg[4 * cidx[k]];
        const cplx<double> r = Rs[(long)oidx[i] * nc + cidx[k]];
        const cplx<double> y = Y[(long)k * no + j];
        acc.re += Lk * (r.re * y.re - r.im * y.im);
        acc.im += Lk * (r.re * y.im + r.im * y.re);
      }
      Ss[e] = acc;
    }
    __syncthreads();
    Ro = Ss;
    ldr = no;
  }
  // Z over the open channels (zmat_kernel's formula)
  const int w2 = 2 * no;
  for (int e = tid; e < no * no; e += 256) {
    const int i = e / no, j = e - i * no;
    const int c = ncl ? oidx[i] : i, cp = ncl ? oidx[j] : j;
    const double sc = sqrho[c] * sqrho[cp];
    const cplx<double> rr = Ro[(long)i * ldr + j];
    const cplx<double> rt{sc * rr.re, sc * rr.im};
    const double F = fg[4 * cp], Fp = fg[4 * cp + 1], G = fg[4 * cp + 2], Gp = fg[4 * cp + 3];
    if (s_scaled) {  // zmat_scaled_kernel's form: [ZO~ | Q E^-1]
      const double sc = exp(-2.0 * thl[cp]);
      cplx<double> zo = cmul(rt, cplx<double>{Gp, Fp * sc});
      zo = cplx<double>{-zo.re, -zo.im};
      cplx<double> q{-rt.re * Fp, -rt.im * Fp};
      if (i == j) {
        zo.re += G;
        zo.im += F * sc;
        q.re += F;
      }
      const double ej = exp(-thl[cp]);
      z[(long)i * w2 + j] = zo;
      z[(long)i * w2 + no + j] = cplx<double>{q.re * ej, q.im * ej};
      continue;
    }
    cplx<double> zo = cmul(rt, cplx<double>{Gp, Fp});
    cplx<double> zi = cmul(rt, cplx<double>{Gp, -Fp});
    zo = cplx<double>{-zo.re, -zo.im};
    zi = cplx<double>{-zi.re, -zi.im};
    if (i == j) {
      zo.re += G;
      zo.im += F;
      zi.re += G;
      zi.im -= F;
    }
    z[(long)i * w2 + j] = zo;
    z[(long)i * w2 + no + j] = zi;
  }
  __syncthreads();  // R_eff (in S) is consumed
  if (ncl > 0)
    for (int e = tid; e < nc * nc; e += 256) Ss[e] = cplx<double>{0.0, 0.0};
  __syncthreads();
  if (block_eliminate(z, no, w2, sv, sr)) {
    if (tid == 0) status[sidx] = 3;
    return;
  }
  // back substitution: S_oo = U^-1 (right half), scattered to the open rows and columns
  block_back_substitute(z, no, w2, no, Ss, nc, ncl ? oidx : nullptr, ncl ? oidx : nullptr);
  if (s_scaled) {  // U = I - 2i E^-1 Y over the open channels
    __syncthreads();
    for (int e = tid; e < no * no; e += 256) {
      const int i = e / no, j = e - i * no;
      const int ci = ncl ? oidx[i] : i, cj = ncl ? oidx[j] : j;
      const double ei = exp(-thl[ci]);
      const cplx<double> y = Ss[(long)ci * nc + cj];
      cplx<double> u{2.0 * ei * y.im, -2.0 * ei * y.re};
      if (i == j) u.re += 1.0;
      Ss[(long)ci * nc + cj] = u;
    }
  }
  if (tid == 0) status[sidx] = 0;
}

// The collision matrix from R (see hp_smatrix), on workspace w laid out by ws;
// hstat, hidx: host arrays of nc ints.
static int smatrix_impl(const hp_system *sys, double E, const double *R, double *S, int *nopen, char *w,
                        const Workspace &ws, int *hstat, int *hidx, hipStream_t st) {
  const int nc = sys->nc;
  cplx<double> *ZO = (cplx<double> *)(w + ws.aux_off);
  cplx<double> *tmp = (cplx<double> *)(w + ws.rhs_off);
  double *fg = (double *)(w + ws.red_off);
  double *sqrho = fg + 4 * (size_t)nc;
  double *theta = sqrho + nc;
  int *stat = (int *)(theta + nc);
  int *ipiv = stat + nc;
  int *perm = ipiv + nc;
  int *finfo = (int *)(w + ws.flag_off);
  TraceScope ts(TR_SMATRIX, st, 8.0 / 3.0 * (double)nc * nc * nc, 0.0);
  hipLaunchKernelGGL(channel_kernel, dim3((nc + 63) / 64), dim3(64), 0, st, nc, E, sys->hbar2_2mu, sys->z1z2e2,
                     sys->a, sys->l, sys->eps, fg, sqrho, theta, stat);
  HP_CHECK_LAUNCH();
  const long cnt = (long)nc * nc;
  hipLaunchKernelGGL(zmat_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, nc,
                     (const cplx<double> *)R, fg, sqrho, ZO, (cplx<double> *)S);
  HP_CHECK_LAUNCH();
  int rc;
  if ((rc = lu_factor<double>(nc, ZO, nc, ipiv, perm, finfo, w, ws, st))) return rc;
  if ((rc = lu_solve<double>(nc, nc, ZO, nc, perm, (cplx<double> *)S, nc, tmp, nullptr, st))) return rc;
  int hinfo = 0;
  HP_CHECK_HIP(hipMemcpyAsync(&hinfo, finfo, sizeof(int), hipMemcpyDeviceToHost, st));
  HP_CHECK_HIP(hipMemcpyAsync(hstat, stat, sizeof(int) * nc, hipMemcpyDeviceToHost, st));
  HP_CHECK_HIP(hipStreamSynchronize(st));
  int open = 0, closed = 0, bad = 0, edge = 0, scaled = 0;
  for (int c = 0; c < nc; ++c) {
    if (hstat[c] == 0 || hstat[c] == 6) {
      ++open;
      if (hstat[c] == 6) scaled = 1;
    } else if (hstat[c] == 3) {
      ++closed;
    } else if (hstat[c] == 2) {
      bad = 1;
    } else {
      edge = 1;
    }
  }
  if (nopen) *nopen = open;
  if (bad) return HP_ERR_NOCONV;
  if (edge || open == 0) return HP_ERR_UNSUPPORTED;  // at a threshold, or no open channel
  if (closed == 0 && !scaled) {
    if (hinfo == -1) return HP_ERR_SYNC;
    if (hinfo > 0) return HP_ERR_SINGULAR;
    return HP_OK;
  }
  if (closed == 0) {
    // some open channel far below its Coulomb barrier: the pass above is
    // discarded; U = I - 2i E^-1 ZO~^-1 Q E^-1 (zmat_scaled_kernel)
    hipLaunchKernelGGL(zmat_scaled_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, nc,
                       (const cplx<double> *)R, (long)nc, fg, sqrho, theta, (const int *)nullptr, ZO,
                       (cplx<double> *)S);
    HP_CHECK_LAUNCH();
    if ((rc = lu_factor<double>(nc, ZO, nc, ipiv, perm, finfo, w, ws, st))) return rc;
    if ((rc = lu_solve<double>(nc, nc, ZO, nc, perm, (cplx<double> *)S, nc, tmp, nullptr, st))) return rc;
    hipLaunchKernelGGL(u_scaled_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, nc, theta,
                       (const int *)nullptr, (cplx<double> *)S);
    HP_CHECK_LAUNCH();
    HP_CHECK_HIP(hipMemcpyAsync(&hinfo, finfo, sizeof(int), hipMemcpyDeviceToHost, st));
    HP_CHECK_HIP(hipStreamSynchronize(st));
    if (hinfo == -1) return HP_ERR_SYNC;
    if (hinfo > 0) return HP_ERR_SINGULAR;
    return HP_OK;
  }
  // closed channels: the pass above is discarded; eliminate them through
  // R_eff and match over the open channels
  const int no = open, ncl = closed;
  for (int c = 0, io = 0, ic = 0; c < nc; ++c) {
    if (hstat[c] == 0 || hstat[c] == 6)
      hidx[io++] = c;
    else
      hidx[no + ic++] = c;
  }
  int *oidx = perm + nc, *cidx = oidx + no;
  cplx<double> *Y = (cplx<double> *)S;                 // ncl x no, then the open channels' ZI and U
  cplx<double> *Reff = (cplx<double> *)(w + ws.res_off);  // no x no
  HP_CHECK_HIP(hipMemcpyAsync(oidx, hidx, sizeof(int) * (size_t)nc, hipMemcpyHostToDevice, st));
  {
    const long cnt2 = (long)ncl * ncl + (long)ncl * no;
    hipLaunchKernelGGL(closed_mats_kernel, dim3((unsigned)((cnt2 + 255) / 256)), dim3(256), 0, st, nc, ncl, no,
                       (const cplx<double> *)R, fg, cidx, oidx, ZO, Y);
    HP_CHECK_LAUNCH();
  }
  if ((rc = lu_factor<double>(ncl, ZO, ncl, ipiv, perm, finfo + 1, w, ws, st))) return rc;
  if ((rc = lu_solve<double>(ncl, no, ZO, ncl, perm, Y, no, tmp, nullptr, st))) return rc;
  const long cnt_o = (long)no * no;
  hipLaunchKernelGGL(reff_kernel, dim3((unsigned)((cnt_o + 255) / 256)), dim3(256), 0, st, nc, ncl, no,
                     (const cplx<double> *)R, fg, cidx, oidx, Y, Reff);
  HP_CHECK_LAUNCH();
  if (scaled)  // an open channel far below its Coulomb barrier: the scaled form over the open channels
    hipLaunchKernelGGL(zmat_scaled_kernel, dim3((unsigned)((cnt_o + 255) / 256)), dim3(256), 0, st, no,
                       (const cplx<double> *)Reff, (long)no, fg, sqrho, theta, (const int *)oidx, ZO,
                       (cplx<double> *)S);
  else
    hipLaunchKernelGGL(zmat_open_kernel, dim3((unsigned)((cnt_o + 255) / 256)), dim3(256), 0, st, no, Reff, fg,
                       sqrho, oidx, ZO, (cplx<double> *)S);
  HP_CHECK_LAUNCH();
  if ((rc = lu_factor<double>(no, ZO, no, ipiv, perm, finfo, w, ws, st))) return rc;
  if ((rc = lu_solve<double>(no, no, ZO, no, perm, (cplx<double> *)S, no, tmp, nullptr, st))) return rc;
  if (scaled) {
    hipLaunchKernelGGL(u_scaled_kernel, dim3((unsigned)((cnt_o + 255) / 256)), dim3(256), 0, st, no, theta,
                       (const int *)oidx, (cplx<double> *)S);
    HP_CHECK_LAUNCH();
  }
  // U (no x no, packed at the start of S) to its place in S, zeros elsewhere
  HP_CHECK_HIP(hipMemcpyAsync(Reff, S, sizeof(cplx<double>) * (size_t)cnt_o, hipMemcpyDeviceToDevice, st));
  {
    const long cnt_s = (long)nc * nc;
    hipLaunchKernelGGL(zero_c128_kernel, dim3((unsigned)((cnt_s + 255) / 256)), dim3(256), 0, st, cnt_s,
                       (cplx<double> *)S);
    HP_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(scatter_open_kernel, dim3((unsigned)((cnt_o + 255) / 256)), dim3(256), 0, st, nc, no, oidx,
                     Reff, (cplx<double> *)S);
  HP_CHECK_LAUNCH();
  int hinfo2[2] = {0, 0};
  HP_CHECK_HIP(hipMemcpyAsync(hinfo2, finfo, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HP_CHECK_HIP(hipStreamSynchronize(st));
  if (hinfo2[0] == -1 || hinfo2[1] == -1) return HP_ERR_SYNC;
  if (hinfo2[0] > 0 || hinfo2[1] > 0) return HP_ERR_SINGULAR;
  return HP_OK;
}

// Scratch of hp_smatrix_noalloc: file-scope device memory, one copy per GPU,
// held until the process ends.  In host code the array's name is not a
// device address: kernels get the address hipGetSymbolAddress returns for
// the current device, looked up once per device.
constexpr int kSmatNoallocMaxChannels = 256;
constexpr size_t kSmatScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kSmatScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch[kMaxDevices] = {};
}  // namespace

static int scratch_for_device(char **out) {
  int dev = 0;
  HP_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HP_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HP_ERR_HIP;
    g_scratch[dev] = (char *)p;
  }
  *out = g_scratch[dev];
  return HP_OK;
}

static bool smatrix_args_ok(const hp_system *sys, const double *R, const double *S) {
  return sys && sys->nc >= 1 && sys->a > 0 && sys->hbar2_2mu > 0 && sys->l && sys->eps && R && S;
}

}  // namespace hp

extern "C" int hp_smatrix(const hp_system *sys, double E, const double *R, double *S, int *nopen, void *work,
                          size_t work_bytes, void *stream) {
  if (!smatrix_args_ok(sys, R, S) || !work) return HP_ERR_ARG;
  const int nc = sys->nc;
  Workspace ws = plan_workspace(nc, nc, HP_C128);
  if (work_bytes < ws.total) return HP_ERR_WORKSPACE;
  std::vector<int> hstat(nc), hidx(nc);
  return smatrix_impl(sys, E, R, S, nopen, (char *)work, ws, hstat.data(), hidx.data(), (hipStream_t)stream);
}

extern "C" int hp_smatrix_noalloc(const hp_system *sys, double E, const double *R, double *S, int *nopen,
                                  void *stream) {
  if (!smatrix_args_ok(sys, R, S)) return HP_ERR_ARG;
  const int nc = sys->nc;
  if (nc > kSmatNoallocMaxChannels) return HP_ERR_UNSUPPORTED;
  Workspace ws = plan_workspace(nc, nc, HP_C128);
  if (ws.total > kSmatScratchBytes) return HP_ERR_UNSUPPORTED;
  char *w = nullptr;
  int rc = scratch_for_device(&w);
  if (rc) return rc;
  int hstat[kSmatNoallocMaxChannels], hidx[kSmatNoallocMaxChannels];
  return smatrix_impl(sys, E, R, S, nopen, w, ws, hstat, hidx, (hipStream_t)stream);
}

extern "C" int hp_batch_smatrix(int count, const hp_batch_item *items, const double *R, double *S, int *status,
                                long sum_nc2, int nc_max, void *work, size_t work_bytes, void *stream) {
  if (count < 1 || !items || !R || !S || !status || !work || sum_nc2 < 1 || nc_max < 1) return HP_ERR_ARG;
  if (nc_max > kBatchSmatMaxChannels) return HP_ERR_UNSUPPORTED;
  if (work_bytes < 2 * sizeof(cplx<double>) * (size_t)sum_nc2) return HP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  TraceScope ts(TR_SMATRIX, st, 0.0, 0.0);
  hipLaunchKernelGGL(batch_smatrix_kernel, dim3(count), dim3(256), 0, st, count, items, (const cplx<double> *)R,
                     (cplx<double> *)S, (cplx<double> *)work, status);
  HP_CHECK_LAUNCH();
  return HP_OK;
}
