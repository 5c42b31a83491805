/*
 * hprmat.h -- C ABI of the MI355X coupled-channel R-matrix internal-region solver.
 *
 * The library solves, on one AMD Instinct MI355X (gfx950), the dense complex
 * symmetric system of the Lagrange-mesh R-matrix method (arXiv 2512.11590,
 * Sec. 2, Eqs. linear_system and block_structure):
 *
 *     C(E) X = B,   C = T + L(Bloch) + centrifugal + V + thresholds - E,
 *
 * on nc channels x nr Lagrange-Legendre points (N = nc * nr), with B the nc
 * surface vectors q_i = f_i(a) (Sec. 3.1, step 2), then extracts the
 * R-matrix (Sec. 3.1, step 4) and the collision matrix.
 *
 * Conventions for every entry point
 *  - Matrices are row-major.  Because C is complex symmetric (C = C^T), the
 *    row-major array is also the column-major array of the same matrix.
 *  - Complex values are interleaved (re, im) pairs of double (complex128) or
 *    float (complex64); "ld" arguments count complex elements.
 *  - Pointers named d_* or documented "device" must be device memory from the
 *    caller (hipMalloc or equivalent); the library allocates nothing on the
 *    device.  Host pointers are documented as such.
 *  - `stream` is a hipStream_t (passed as void*; NULL = the null stream).
 *    All work is enqueued on it; entry points that must read a device-side
 *    result (the refinement loop, the singular-pivot check) synchronize it.
 *  - Return value: HP_OK or a negative HP_ERR_* code.  Argument errors are
 *    detected before any work is enqueued.
 *  - Channel-major unknown index: (c, i) -> c * nr + i  (Sec. 3.1, step 4).
 */
#ifndef HPRMAT_H
#define HPRMAT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HP_OK 0
#define HP_ERR_ARG (-1)         /* invalid argument (sizes, null pointers, precision) */
#define HP_ERR_HIP (-2)         /* a HIP runtime call or kernel launch failed */
#define HP_ERR_SINGULAR (-3)    /* the factorization met an exactly zero pivot */
#define HP_ERR_NOCONV (-4)      /* iterative refinement did not reach the tolerance */
#define HP_ERR_WORKSPACE (-5)   /* workspace smaller than hp_workspace_bytes() */
#define HP_ERR_UNSUPPORTED (-6) /* outside what the library implements (e.g. no open channel, sizes beyond a kernel's limits) */
#define HP_ERR_SYNC (-7)        /* a bounded inter-workgroup wait expired (no hang: reported) */

/* Working precision of the matrix and its LU factors. */
#define HP_C128 0 /* complex FP64 */
#define HP_C64 1  /* complex FP32 (factor); refinement residual stays FP64 */
/* complex FP32 factor whose trailing updates run on the FP16 matrix cores
 * under row and column scaling (split FP16 operands, FP32 accumulation;
 * Sec. 3.2 / 3.4 mixed precision, the optional FP16 variant); the matrix and
 * the factors are stored as with HP_C64, and every entry point that takes
 * HP_C64 takes HP_C64H (only hp_factor computes differently) */
#define HP_C64H 2

/* Description of one coupled-channel system.  Scalars by value; arrays in
 * device memory, owned by the caller, read-only for the library. */
typedef struct hp_system {
  int nc;            /* number of channels, >= 1 */
  int nr;            /* Lagrange-Legendre points per channel, >= 1 */
  double a;          /* channel radius a (fm) */
  double hbar2_2mu;  /* hbar^2 / 2 mu (MeV fm^2), common to all channels */
  double z1z2e2;     /* Z1 Z2 e^2 (MeV fm) of the external Coulomb field */
  const double *r;   /* device [nr]: mesh points r_i */
  const double *q;   /* device [nr]: surface values q_i = f_i(a) */
  const double *tl;  /* device [nr*nr]: (T + L)_ij / (hbar^2/2mu), row-major */
  const int *l;      /* device [nc]: orbital angular momentum per channel */
  const double *eps; /* device [nc]: threshold energy per channel (MeV) */
  const double *v;   /* device [nr*nc*nc] complex128: V[i][c][c'] = V_cc'(r_i) (MeV) */
  /* Optional non-local potential (Sec. 2: the coupling blocks D become full
   * matrices).  NULL for a local system.  Otherwise device [n*n] complex128,
   * n = nc*nr, row-major in the channel-major index:
   * vnl[(c*nr+i)*n + c'*nr+j] = W_cc'(r_i, r_j) (MeV/fm), the kernel at the
   * mesh-point pairs.  The library adds the Lagrange-mesh matrix element
   * sqrt(w_i w_j) W_cc'(r_i, r_j) (Gauss quadrature) to element
   * ((c,i),(c',j)) of C(E) (batched entry points too). */
  const double *w;   /* device [nr]: mesh weights w_i on (0, a); required when vnl != NULL */
  const double *vnl;
} hp_system;

/* Outcome of hp_solve (host struct, written by the library). */
typedef struct hp_solve_info {
  int iterations;        /* refinement corrections applied */
  int converged;         /* 1 if refinement converged (or no refinement was asked) */
  double correction;     /* max over columns of |d|_inf / |x|_inf of the last correction */
  double residual;       /* backward error of the returned X: max over columns of
                            |b - C x|_inf / (|C|_inf |x|_inf + |b|_inf), norms of |Re|+|Im| */
} hp_solve_info;

/* ---- host-side precompute ---------------------------------------------- */

/* Lagrange-Legendre mesh on (0, a) (Sec. 2): points r[i], weights w[i]
 * (summing to a), surface values q[i] = f_i(a) and the kinetic + Bloch
 * matrix tl[i*nr + j] = (T + L)_ij / (hbar^2/2mu) in closed form.  All
 * four arrays are HOST memory of nr (tl: nr*nr) doubles; any may be NULL.
 * Errors: HP_ERR_ARG if nr < 1 or a <= 0. */
int hp_mesh(int nr, double a, double *r, double *w, double *q, double *tl);

/* Inverse of the kinetic + Bloch matrix tl of hp_mesh (the shared kinetic
 * block K = (hbar^2/2mu) tl of the Woodbury-kinetic form, Sec. 3.3, step 1,
 * without the factor hbar^2/2mu): kinv[i*nr + j] = (tl^-1)_ij for the rounded
 * tl that hp_mesh returns, by Gauss-Jordan elimination with partial pivoting
 * in binary128, rounded once.  Energy-independent: once per mesh.  Runs on
 * the calling host thread: about 2 nr^3 binary128 operations in software
 * arithmetic (0.08 s at nr = 100, 4 s at nr = 400 on one core).  kinv:
 * HOST nr*nr doubles.  Errors: HP_ERR_ARG (nr < 1, a <= 0, kinv NULL),
 * HP_ERR_SINGULAR. */
int hp_kinetic_inverse(int nr, double a, double *kinv);

/* Device workspace (bytes) that hp_factor, hp_solve and hp_smatrix need for
 * an n x n factorization with nrhs right-hand sides in precision prec.  One
 * workspace may serve all three calls on one stream in sequence.  With
 * prec == HP_C64 and nrhs > 0 it includes the transformed FP32 L factor
 * that hp_solve's refinement solves use (about 4 n^2 bytes); hp_factor alone
 * needs only hp_workspace_bytes(n, 0, prec). */
size_t hp_workspace_bytes(int n, int nrhs, int prec);

/* ---- the hot path ----------------------------------------------------- */

/* Assemble C(E) (Eq. block_structure) into device matrix C (n x n, n =
 * nc*nr, leading dimension ldc >= n, complex128 if prec == HP_C128, complex64
 * if HP_C64, converted from FP64 values), overwriting every element:
 *   C[(c,i),(c',j)] = delta_cc' [ h tl_ij + delta_ij (h l_c(l_c+1)/r_i^2 + eps_c - E) ]
 *                     + delta_ij V_cc'(r_i)
 *                     [ + sqrt(w_i w_j) W_cc'(r_i, r_j)  if sys->vnl != NULL ],
 * h = hbar2_2mu.
 * Errors: HP_ERR_ARG (null pointer, vnl without w, ldc < n, bad prec),
 * HP_ERR_HIP. */
int hp_build_matrix(const hp_system *sys, double E, int prec, void *C, long ldc, void *stream);

/* LU factorization with partial pivoting in place, P A = L U (Sec. 3.1,
 * Type 1; Type 2/4 in FP32).  A: device n x n, leading dimension lda >= n,
 * precision prec; on return the strict lower triangle holds L (unit diagonal
 * implied) and the upper triangle U.  ipiv: device [n], ipiv[k] = row
 * exchanged with row k at step k (0-based, LAPACK order).  perm: device [n],
 * perm[i] = original row now in row i (used by hp_solve).  info: device int,
 * set to 0, or k+1 for the first exactly zero pivot column k, or -1 if a
 * bounded inter-workgroup wait expired.  work: device workspace of at least
 * hp_workspace_bytes(n, 0, prec) bytes.  Asynchronous: does not synchronize;
 * read *info after the stream completes.  Internally, block k+1 is factored
 * on a second stream (one per device and caller stream, created on first
 * use, default priority) while block k's trailing update runs on `stream`;
 * all of it is ordered before work enqueued on `stream` afterwards.
 * Errors: HP_ERR_ARG, HP_ERR_WORKSPACE, HP_ERR_UNSUPPORTED (n too large for
 * the co-resident panel grid), HP_ERR_HIP. */
int hp_factor(int n, int prec, void *A, long lda, int *ipiv, int *perm, int *info,
              void *work, size_t work_bytes, void *stream);

/* Solve C(E) X = B for the nc surface right-hand sides (Sec. 3.1, steps 2-3)
 * with the factors of hp_factor (LU, lda, perm, precision prec).  X: device
 * n x nc complex128 (leading dimension nc), overwritten with the solution.
 * The factors give X0 (prec == HP_C64: FP32 factors, X0 widened to FP64).
 * With max_refine > 0, iterative refinement follows (Sec. 3.2 and Sec. 3.4
 * step 7, here entirely on the device): r = B - C X in FP64 from the block
 * structure of sys (no N x N FP64 matrix of the local part; a non-local
 * system adds one FP64 product with its n x n kernel values, the X rows and
 * the result scaled by sqrt(w)), correction from the factors,
 * X += d in FP64.  The relative correction max_c |d_c| / |x_c| tracks the
 * forward error: refinement stops converged when it is <= tol (tol <= 0:
 * 2^-29 = u64/u32: the error left after such a correction, about kappa u32
 * times it, is below the FP64 floor kappa u64) or when it stops shrinking (a
 * correction larger than half the previous one) with that correction itself
 * <= max(tol, 2^-26), and reports non-convergence (HP_ERR_NOCONV) when it
 * stops shrinking above that (Performance Results, Accuracy Validation,
 * Fig. illcond: the single-precision factor is then too inaccurate to
 * contract; the caller then solves in FP64, the paper's fallback mechanism)
 * or after max_refine corrections.  info (host, may
 * be NULL) receives the outcome, including the normwise backward error.
 * Synchronizes the stream once per refinement pass.  With FP32 factors the
 * call first multiplies every block column of L below the diagonal by the
 * inverse of its 256-row diagonal block (kept in work, the factors are not
 * modified), so that the forward substitution of each solve of the
 * refinement is a chain of GEMMs.
 * Errors: HP_ERR_ARG, HP_ERR_WORKSPACE, HP_ERR_NOCONV (X holds the last
 * iterate), HP_ERR_SINGULAR (zero pivot reported by hp_factor), HP_ERR_SYNC,
 * HP_ERR_HIP. */
int hp_solve(const hp_system *sys, double E, int prec, const void *LU, long lda,
             const int *perm, const int *info_factor, double *X, int max_refine, double tol,
             void *work, size_t work_bytes, hp_solve_info *info, void *stream);

/* ---- Woodbury-kinetic form (Sec. 3.3, Type 3) ---------------------------
 * M = K_diag (I + K_diag^-1 V) with K = h tl shared by every channel, so
 * M c = b becomes S c = K_diag^-1 b with S = I + K_diag^-1 V.  The library
 * keeps the channel-major unknown order of C(E) (the paper lists S in
 * radial-major order: the same matrix up to one symmetric permutation), so
 * S[(c,i),(c',j)] = delta_cc' delta_ij + (1/h) kinv_ij Vd_cc'(r_j) with
 * Vd_cc'(r_j) = V_cc'(r_j) + delta_cc' (h l_c(l_c+1)/r_j^2 + eps_c - E) (every
 * term of C(E) that is diagonal in the radial index).  S is factored by
 * hp_factor like C(E) (it is not symmetric; the factorization does not
 * assume symmetry).  Local systems only (HP_ERR_UNSUPPORTED if sys->vnl). */

/* Workspace of hp_solve_schur: hp_workspace_bytes(n, nrhs, prec) plus room for
 * the transformed residual (n*nrhs complex128), the complex copy of kinv/h
 * and K^-1 q; nr = n / nrhs.  0 on bad arguments. */
size_t hp_schur_workspace_bytes(int n, int nrhs, int prec);

/* Assemble S(E) into device matrix S (n x n, leading dimension lds >= n,
 * complex128 for HP_C128, complex64 for HP_C64/HP_C64H, from FP64 values).
 * kinv: device nr*nr doubles from hp_kinetic_inverse.
 * Errors: HP_ERR_ARG, HP_ERR_UNSUPPORTED (non-local system), HP_ERR_HIP. */
int hp_build_schur(const hp_system *sys, double E, int prec, const double *kinv, void *S, long lds,
                   void *stream);

/* Solve C(E) X = B through the factors of S(E) (hp_factor on hp_build_schur's
 * matrix): X0 from S X0 = K_diag^-1 B; with max_refine > 0 the FP64 residual
 * r = B - C X of C(E) itself (as in hp_solve) is transformed, S d =
 * K_diag^-1 r, X += d, with hp_solve's stop rule and reported figures (the
 * backward error is C(E)'s).  max_refine = 0 with FP32 factors is the paper's
 * single-precision Type 3 solve.  Arguments, X layout and errors as
 * hp_solve, plus kinv (device, as for hp_build_schur); work: at least
 * hp_schur_workspace_bytes(n, nc, prec) bytes. */
int hp_solve_schur(const hp_system *sys, double E, int prec, const double *kinv, const void *LU, long lda,
                   const int *perm, const int *info_factor, double *X, int max_refine, double tol, void *work,
                   size_t work_bytes, hp_solve_info *info, void *stream);

/* General solve with the factors: X (device n x nrhs, leading dimension ldx,
 * precision prec) holds B on entry and X = A^-1 B on return. */
int hp_lu_solve(int n, int nrhs, int prec, const void *LU, long lda, const int *perm,
                void *X, long ldx, void *work, size_t work_bytes, void *stream);

/* The trailing-update kernel on its own: C -= A B for complex matrices
 * (device, row-major, interleaved, precision prec), A M x K (lda >= K),
 * B K x N (ldb >= N), C M x N (ldc >= N); the block operation of Sec. 3.1's
 * LU and substitutions.  Exposed for tests and tuning.  Asynchronous. */
int hp_gemm_sub(int M, int N, int K, int prec, const void *A, long lda, const void *B, long ldb, void *C,
                long ldc, void *stream);

/* The HP_C64H trailing update on its own: C -= A B (complex FP32, row-major)
 * with A's rows and B's columns scaled by powers of two into [-1, 1], split
 * into two FP16 words each and multiplied on the FP16 matrix cores with FP32
 * accumulation (three products per real product).  K a multiple of 32, at
 * most 256 (HP_ERR_UNSUPPORTED otherwise).  work: device, at least
 * 8 K (M + N) + 4 (M + N) + 512 bytes for the converted operands
 * (HP_ERR_WORKSPACE otherwise).  Exposed for tests and tuning; asynchronous. */
int hp_gemm_h3_sub(int M, int N, int K, const void *A, long lda, const void *B, long ldb, void *C, long ldc,
                   void *work, size_t work_bytes, void *stream);

/* R-matrix (Sec. 3.1, step 4, with the factor hbar^2/(2 mu a)):
 *   R[c][c'] = (hbar2_2mu / a) sum_i q_i X[(c,i)][c'],
 * X device n x nc complex128, R device nc x nc complex128 (row-major). */
int hp_rmatrix(const hp_system *sys, const double *X, double *R, void *stream);

/* Collision matrix U from R by matching to Coulomb functions at r = a in
 * every channel (the Coulomb-asymptotics step the paper performs with its
 * Coulomb routine, Sec. 4.1): with rho_c = k_c a, k_c = sqrt((E - eps_c)/h),
 * eta_c = z1z2e2 / (2 h k_c), O = G + iF, I = G - iF,
 *   U = (O - Rt O')^-1 (I - Rt I'),   Rt = rho^1/2 R rho^1/2.
 * Closed channels (E < eps_c) end in decaying Whittaker functions
 * W_{-eta_c, l_c + 1/2}(2 kappa_c r), kappa_c = sqrt((eps_c - E)/h),
 * eta_c = z1z2e2 / (2 h kappa_c) (the special functions of Sec. 4.1): with
 * L_c = a u_c'(a)/u_c(a) they are eliminated through the open channels'
 * effective R-matrix R_eff = R_oo + R_oc L (I - R_cc L)^-1 R_co, from which U
 * follows over the open channels as above.
 * R, S: device nc x nc complex128; S receives U on the open-open entries and
 * zeros in the closed channels' rows and columns.  nopen (host, may be NULL)
 * receives the number of open channels.  An open channel so far below its
 * Coulomb barrier that F and G leave double range is carried with scaled
 * values F~ = F e^theta, G~ = G e^-theta, and U is formed as
 *   U = I - 2i E^-1 (diag O~ - Rt diag O~')^-1 (diag F~ - Rt diag F~') E^-1,
 * E = diag(e^theta), O~ = G~ + i F~ e^-2theta (the same U; every factor
 * e^-theta <= 1; with closed channels, over the open ones from R_eff).
 * HP_ERR_UNSUPPORTED if no channel is open or E equals a threshold;
 * HP_ERR_NOCONV if a continued fraction did not converge.  Uses work
 * (hp_workspace_bytes(nc, nc, HP_C128)).  Synchronizes the stream. */
int hp_smatrix(const hp_system *sys, double E, const double *R, double *S, int *nopen,
               void *work, size_t work_bytes, void *stream);

/* hp_smatrix for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation with the same kernels and the same result, but its
 * workspace is a fixed 4 MiB array of device memory inside the library (one
 * copy per GPU, looked up once per device on first use and held until the
 * process ends) instead of a caller's buffer.  At most 256 channels
 * (HP_ERR_UNSUPPORTED beyond).  The call allocates nothing (no hipMalloc,
 * no stream or event creation; with hp_trace enabled the timers still
 * create their events).  Every call on one GPU uses that GPU's array, and
 * everything in it that must start cleared is cleared by the call itself:
 * calls that overlap on one GPU (from several host threads or streams) race
 * for the array and must be serialized by the caller.  Synchronizes the
 * stream, like hp_smatrix.  Errors: as hp_smatrix, plus HP_ERR_UNSUPPORTED
 * for nc > 256. */
int hp_smatrix_noalloc(const hp_system *sys, double E, const double *R, double *S, int *nopen,
                       void *stream);

/* ---- helpers ------------------------------------------------------------ */

/* Coulomb functions F_l, F_l', G_l, G_l' (d/drho) at (eta, rho), computed on
 * the HOST with the same routine the device uses (for tests).  out: host [4].
 * Errors: HP_ERR_ARG if l < 0, rho <= 0 or eta < 0; HP_ERR_NOCONV if a
 * continued fraction did not converge or the functions leave double range
 * (far below the Coulomb barrier: F underflows, G overflows). */
int hp_coulomb(int l, double eta, double rho, double *out);

/* Same routine on the device for nch channels: device arrays l[nch],
 * eta[nch], rho[nch] -> out[nch*4]. */
int hp_coulomb_device(int nch, const int *l, const double *eta, const double *rho,
                      double *out, void *stream);

/* ---- batched uneven systems ---------------------------------------------- */

/* Many independent systems (one per (J^pi, energy) label, n of a few hundred
 * to a few thousand) solved side by side, one workgroup per system, with no
 * inter-workgroup synchronisation.  The caller lays the systems out in shared
 * device buffers and describes each by an hp_batch_item in DEVICE memory;
 * listing the largest systems first balances the persistent grid.
 * Offsets are in elements of the buffer they index. */
typedef struct hp_batch_item {
  hp_system sys;  /* this system's data (device pointers) */
  double E;       /* its energy (MeV) */
  long a_off;     /* its n x n matrix in A (leading dimension n) */
  long x_off;     /* its n x nc block in X (leading dimension nc) */
  long p_off;     /* its n entries of ipiv and perm */
  long r_off;     /* its nc x nc block of R */
  long c_off;     /* its nc entries of per-column arrays: sum of nc over the systems before it */
} hp_batch_item;

/* Workspace of the batched solves: sum_nc = sum of nc, sum_xn = sum of n*nc
 * over the systems, nmax = the largest n.  0 on bad arguments. */
size_t hp_batch_workspace_bytes(int count, long sum_nc, long sum_xn, int nmax, int prec);

/* C(E) of every system into A (precision prec), as hp_build_matrix does for one
 * (Eq. block_structure, with the non-local term of an item whose sys.vnl is
 * set).  64 workgroups per system. */
int hp_batch_build(int count, const hp_batch_item *items, int prec, void *A, void *stream);

/* LU with partial pivoting of every system (Sec. 3.1), in place, as
 * hp_factor: ipiv/perm per system at p_off, info[s] = 0 or k+1 for the first
 * exactly zero pivot column k.  A persistent grid of `groups` workgroups takes
 * systems in list order from a counter in `work` (>= 256 bytes); each
 * workgroup factors its system in panels of `panel` (1..32) columns: column
 * steps with full-row interchanges, the panel's block row, and the trailing
 * update as MFMA complex tiles (3M in FP32, 4M in FP64).
 * Errors: HP_ERR_ARG, HP_ERR_HIP. */
int hp_batch_factor(int count, const hp_batch_item *items, int prec, void *A, int *ipiv, int *perm,
                    int *info, int panel, int groups, void *work, size_t work_bytes, void *stream);

/* The same factorization in steps, for batches of larger systems, blocked
 * in two levels: outer blocks of `block` columns (a multiple of `panel`, at
 * most 64), each factored as panels of `panel` (1..32) columns whose updates
 * stay inside the block, then the block's row U12 = L11^-1 A12 and one
 * trailing update with K = block (Sec. 3.1's blocked LU with the update
 * deferred to the end of each outer block).  Each step is one launch over
 * every system still factoring: the panels' column steps one workgroup per
 * system (interchanges inside the panel), then each panel's interchanges on
 * the other columns with its block row, the outer block rows and the
 * updates as column chunks and tiles of all systems, so the device is
 * filled by tiles rather than by systems.  block == panel is the one-level
 * form.  n_host: HOST array of the systems' n, which must be listed largest
 * first (HP_ERR_ARG otherwise).  work: at least 256 + 4 * (2 ceil(nmax /
 * panel) + 2 ceil(nmax / block)) * (count + 1) bytes (the batch
 * workspace of hp_batch_workspace_bytes is enough).  Errors: HP_ERR_ARG,
 * HP_ERR_WORKSPACE, HP_ERR_HIP. */
int hp_batch_factor_stepped(int count, const hp_batch_item *items, const int *n_host, int prec, void *A,
                            int *ipiv, int *perm, int *info, int panel, int block, void *work,
                            size_t work_bytes, void *stream);

/* Solves every system for its nc surface right-hand sides with the factors:
 * X (FP64, per system at x_off) = C^-1 B.  With refine != 0 (FP32 factors
 * only), the per-system refinement state is reset for hp_batch_refine_step;
 * systems with a zero pivot (info_factor) are marked and left alone.
 * shape_host: NULL (one workgroup solves each system) or the HOST (n, nc)
 * pairs of the systems, largest n first, for the stepped form (per block of
 * 64 rows one launch of every system's diagonal block and one of all update
 * tiles).  No host synchronisation.  work: hp_batch_workspace_bytes(...). */
int hp_batch_solve_init(int count, const hp_batch_item *items, const int *shape_host, int prec, const void *LU,
                        const int *perm, const int *info_factor, double *X, int refine, long sum_nc,
                        long sum_xn, void *work, size_t work_bytes, void *stream);

/* One FP64 refinement step of FP32 factors for every system still refining
 * (Sec. 3.2): r = B - C X from the block structure (plus, for a non-local
 * system, its kernel product, one output per thread), d from the factors
 * (column-scaled; solves as chosen by shape_host), X += d, and the stop rule
 * of hp_solve per system (relative correction <= tol, tol <= 0: 2^-29; a
 * correction larger than half the previous one: converged if it is itself
 * <= max(tol, 2^-26), else not converged; not converged after max_refine
 * steps).  A
 * fixed sequence of launches, no host synchronisation: it may be captured
 * in a graph and replayed. */
int hp_batch_refine_step(int count, const hp_batch_item *items, const int *shape_host, const void *LU,
                         const int *perm, double *X, int max_refine, double tol, long sum_nc, long sum_xn,
                         void *work, size_t work_bytes, void *stream);

/* Whether hp_batch_factor_stepped takes FP32 panels of 8 columns on at most
 * 4096 rows with the panel held in registers (one 1024-thread workgroup per
 * system; default 1) or through memory (0).  The arithmetic, and so the
 * factors, are the same.  Returns the previous setting.  For tests and
 * tuning; not to be changed while a factorization is in flight. */
int hp_set_batch_reg_panel(int on);

/* Number of systems still refining after the last step (host *active);
 * synchronizes the stream. */
int hp_batch_active(const void *work, unsigned *active, void *stream);

/* Per-system outcome (host arrays of count): status 1 converged (or no
 * refinement), 2 not converged, 3 zero pivot, 4 a non-local system with
 * more than 1024 mesh points in a refined batch (not supported: its X is
 * not a solution), 0 still refining; iters =
 * corrections applied (may be NULL).  Synchronizes the stream. */
int hp_batch_status(int count, const void *work, int *status, int *iters, void *stream);

/* Collision matrix of every system from its R (R and S: device, nc x nc
 * complex128 blocks at r_off), by the matching of hp_smatrix, one workgroup
 * per system, all in FP64: channel functions (Coulomb functions of the open
 * channels, decaying-solution log-derivatives L_c of the closed ones, as
 * hp_smatrix); with closed channels the open channels' effective R-matrix
 * R_eff = R_oo + R_oc L (I - R_cc L)^-1 R_co by Gaussian elimination with
 * partial pivoting; then Z = [O - Rt O' | I - Rt I'] over the open channels,
 * elimination with partial pivoting (largest |Re| + |Im|) and back
 * substitution.  S is zero in closed rows and columns.  status: device
 * int[count], per system 0 ok, 1 no open channel or E exactly at a
 * threshold, 2 a Coulomb continued fraction (or a closed channel's
 * integration) did not converge (channels far below their Coulomb barrier
 * are matched in the scaled form of hp_smatrix), 3 an exactly zero pivot, 4 more than 512 channels; S of a system with
 * status 1, 2 or 4 is not written, with status 3 it holds no result.
 * sum_nc2 = sum of nc^2 over the systems (host), nc_max = the largest nc
 * (host, at most 512, else HP_ERR_UNSUPPORTED).  work: device, at least
 * 32 * sum_nc2 bytes.  Asynchronous, no host synchronisation (may be
 * captured in a graph). */
int hp_batch_smatrix(int count, const hp_batch_item *items, const double *R, double *S, int *status,
                     long sum_nc2, int nc_max, void *work, size_t work_bytes, void *stream);

/* R of every system (Sec. 3.1 step 4), FP64 complex at r_off of R. */
int hp_batch_rmatrix(int count, const hp_batch_item *items, const double *X, double *R, void *stream);

/* ---- concurrency ------------------------------------------------------- */

/* Number of factorizations that may be requested at the same time on one
 * device, from different streams (process-wide, default 1).  A panel grid's
 * workgroups wait for each other at every column, so they must be resident
 * together.  With 1, each factorization runs on its caller's stream (plus the
 * look-ahead stream) with panel workgroups of up to ~150 KB of LDS.  With
 * k > 1, factorizations of n > 256 are serialized on one device-wide stream
 * (the caller's stream hands over and waits by events; its other work still
 * overlaps with other streams), and panel workgroups hold 64 KB of rows, or
 * the ceil(n / 128) rows that a grid of 128 workgroups needs when that is
 * more, so that they find room beside other streams' kernels (up to ~150 KB
 * of rows per workgroup, beyond which hp_factor fails with
 * HP_ERR_UNSUPPORTED).  Factorizations that must overlap each other use the
 * batched entry points, which have no grid-wide waits.  Returns the previous
 * setting, or HP_ERR_ARG if k is outside [1, 256].  Host-side setting; takes
 * effect for factorizations enqueued afterwards. */
int hp_set_concurrency(int k);

/* Whether hp_solve replays the refinement solves of FP32 factors from a HIP
 * graph (1, the default) or launches them one by one (0).  The graph is
 * captured on an internal stream at the first refinement solve of each call
 * and replayed on the caller's stream; the results are identical.  Launches
 * inside the graph are not timed by hp_trace.  Returns the previous setting,
 * or HP_ERR_ARG if on is not 0 or 1.  Host-side setting. */
int hp_set_solve_graphs(int on);

/* ---- instrumentation ---------------------------------------------------- */

/* Per-stage device timers.  hp_trace_enable(mask) clears the record and starts
 * bracketing the kernel launches of the selected stages with HIP events on
 * their stream: mask < 0 selects every stage, otherwise bit s selects stage s
 * (the order of the names below: assemble, panel, laswp, trsm, gemm_c128,
 * gemm_c64, residual, refine, rmatrix, smatrix, gemm_f16x3); hp_trace_enable(0) stops.  hp_trace_read() waits for the recorded events,
 * fills out[0 .. HP_TRACE_STAGES-1] (host array) with, per stage, the launch
 * count, summed kernel time (ms) and summed algorithmic flops and bytes of
 * those launches, clears the record and returns HP_TRACE_STAGES.
 * Errors: HP_ERR_ARG if max_stats < HP_TRACE_STAGES, HP_ERR_HIP. */
#define HP_TRACE_STAGES 11
typedef struct hp_trace_stat {
  const char *name; /* stage name, owned by the library */
  long launches;
  double ms;
  double flops;
  double bytes;
} hp_trace_stat;
int hp_trace_enable(int mask);
int hp_trace_read(hp_trace_stat *out, int max_stats);

/* Static description of the build: string owned by the library. */
const char *hp_build_info(void);

/* The last failing HIP call on this host thread ("file:line: HIP error
 * text"), or "" if none; string owned by the library. */
const char *hp_last_error(void);

/* Human-readable text for an HP_* code. */
const char *hp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* HPRMAT_H */
