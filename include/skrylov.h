/*
 * skrylov.h -- C ABI of the MI355X (gfx950) sketched-and-truncated polynomial block
 * Krylov solver for large sparse Sylvester equations
 *
 *        A X + X B = C1 C2^T,   A: n1 x n1, B: n2 x n2 sparse, C1: n1 x r, C2: n2 x r,
 *
 * after Palitta, Schweitzer and Simoncini, "Sketched and truncated polynomial Krylov
 * subspace methods: matrix Sylvester equations" (arXiv 2311.16019), Algorithm 1 (s-PKSM).
 *
 * Conventions used by every entry point:
 *   - Dense blocks ("n x r") are row-major FP64 arrays (element (i, c) at i*r + c).
 *   - Pointers documented as "device" must point to memory allocated on the current
 *     HIP device (hipMalloc, or a PyTorch CUDA tensor); "host" pointers to host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All device
 *     work of a call is ordered on that stream; calls synchronise it only where stated.
 *   - Return value: SKR_OK (0) or a positive status on success (results are valid),
 *     a negative error code on failure (nothing was produced; skr_last_error() says why).
 *   - The library never takes ownership of caller buffers; handles (skr_op, skr_result)
 *     own their device memory until the matching *_destroy call.
 *   - A handle may be used from one host thread at a time.
 */
#ifndef SKRYLOV_H
#define SKRYLOV_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SKR_API __attribute__((visibility("default")))
#else
#define SKR_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct skr_op_s* skr_op;
typedef struct skr_result_s* skr_result;

enum {
  SKR_OK = 0,
  SKR_NOT_CONVERGED = 1, /* maxit reached; factors from the last projected solve      */
  SKR_BREAKDOWN = 2,     /* a Krylov space became invariant; factors are valid          */
  SKR_EINVAL = -1,       /* invalid argument (shape, parameter, pointer)                */
  SKR_EHIP = -2,         /* a HIP runtime call failed                                   */
  SKR_ENOMEM = -3,       /* device allocation failed                                    */
  SKR_ENOTSUP = -4,      /* valid request this build does not support                   */
  SKR_EPROJ = -5         /* projected Sylvester solve failed (see skr_last_error)       */
};

enum { SKR_FP64 = 0, SKR_MIXED = 1 };           /* bulk precision                       */
enum { SKR_SKETCH_SPARSE_SIGN = 0,             /* subspace embedding (Algorithm 1)     */
       SKR_SKETCH_SRHT = 1,                     /* subsampled randomized DCT (Sec. 6)   */
       SKR_SKETCH_NONE = 2 };                   /* no embedding: Algorithm 2 (t-PKSM)   */
enum { SKR_RECOVER_STORED = 0, SKR_RECOVER_TWO_PASS = 1 };
enum { SKR_ORTH_EUCLIDEAN = 0,                  /* truncated Gram-Schmidt as in Algorithm 1  */
       SKR_ORTH_SKETCHED = 1 };                 /* in the sketched inner product (app. A)    */

/*
 * Solver parameters (Algorithm 1's inputs plus this library's choices).
 *   k         truncation: orthogonalise against the last k blocks (eqn:arnoldi_tr), k >= 1
 *   maxit     maximum number of block steps d
 *   p         check period: the projected equation is solved when d % p == 0 and at maxit
 *   s         sketch rows (s x n embeddings S_U, S_V); 0 means 2*maxit*r rounded up to a
 *             multiple of zeta.  Requires s >= (maxit+1)*r and s % zeta == 0.
 *   tol       relative stop test  rho <= tol * ||beta_1 beta_2^T||_F  (eq:resnorm_sk with
 *             the whitened subdiagonal blocks)
 *   seed      embedding seed; S_U uses seed, S_V uses splitmix64_mix(seed + 1)
 *   zeta      nonzeros per column of the sparse sign embedding (default 8)
 *   precision SKR_FP64, or SKR_MIXED (FP32 sparse products, orthogonalisation and sketch
 *             input; FP64 sketched quantities, projected solve and residual estimate).
 *             In SKR_MIXED, rho is the residual of the sketched problem on the FP32-stored
 *             basis and SKR_OK means rho met tol: the true residual can exceed rho (by 2.5x
 *             at a residual of 1e-3 on a poorly conditioned basis; by 1.3x at 1e-6 on the
 *             n = 1e6 convection-diffusion pair with k = 10).  A caller that needs the true
 *             residual bounded checks it with skr_true_residual.
 *   sketch    SKR_SKETCH_SPARSE_SIGN: s-PKSM (Algorithm 1) with the sparse sign embedding
 *             (zeta nonzeros per column).  SKR_SKETCH_SRHT: s-PKSM with the subsampled
 *             randomized DCT of the paper's experiments, S x = sqrt(n/s) DCT2(E x)[rows]
 *             (orthonormal DCT-II; E_j = -1 when the low bit of SplitMix64 output j+1 from
 *             the space's seed is set; rows = the s indices i with the smallest output i+1
 *             of the generator started at mix64(seed), ascending); needs s <= n and
 *             n = N1 N2 with N1 = P Q, P, Q <= 64, N1 <= 3072, N2 <= 4096 (SKR_ENOTSUP
 *             otherwise); zeta is ignored.  SKR_SKETCH_NONE: the truncated
 *             Arnoldi method t-PKSM (Algorithm 2, appendix A): the same block steps without
 *             an embedding, the projected equation H_d Y + Y G_d^T = E_1 beta_1 beta_2^T E_1^T
 *             on the truncated block Hessenberg matrices (beta = R factors of C1, C2), the
 *             estimate rho = sqrt(d r) (||Y E_d g_{d+1,d}^T||_F + ||h_{d+1,d} E_d^T Y||_F) of
 *             Algorithm 2 in the stop test, and X1 = U_d Y1, X2 = V_d Y2; s, seed and zeta
 *             are ignored.
 *   recover   SKR_RECOVER_STORED (keep every basis block in HBM) or
 *             SKR_RECOVER_TWO_PASS (keep k+1 blocks, regenerate them for the factors)
 *   profile   1: record HIP events around every launch of each kernel family of the block
 *             step; 2 + f: only around the launches of family f (index f of
 *             skr_result_kernel_stats: 0 spmm, 1 dots, 2 reduce, 3 update, 4 sketch,
 *             5 whiten); 0: none.  Each timed launch adds two event records to its stream
 *             (on the benchmark problem timing every family lengthens the block steps by
 *             about a fifth; timing one family costs much less)
 *   trunc_tol relative Frobenius cutoff of the low-rank factorisation of the projected
 *             solution Y (0 keeps everything); 1e-12 suits FP64 and 1e-8 the FP32 bulk of
 *             SKR_MIXED (the Python binding's defaults)
 *   orth      SKR_ORTH_EUCLIDEAN: the truncated block Gram-Schmidt and the QR of the new
 *             block use the Euclidean inner product (Algorithm 1).  SKR_ORTH_SKETCHED: both
 *             use <x, y>_S = (S x)^T (S y) instead (the alternative appendix A names):
 *             S U_1 has orthonormal columns (ell = R factor of S C), h_{i,d} =
 *             (S U_i)^T (S U~) in block modified Gram-Schmidt over the window, R from a
 *             Cholesky QR twice of the sketched remainder, U_{d+1} = (U~ - sum_i U_i h_{i,d})
 *             R^{-1}; S U_{d+1} comes from the sketch-space QR.  The sketched Galerkin
 *             solution does not depend on the basis of the truncated space, so the factors
 *             agree with SKR_ORTH_EUCLIDEAN up to rounding.  Needs the sparse sign sketch and
 *             r <= 4, k <= 3 (SKR_ENOTSUP otherwise).
 */
typedef struct {
  int32_t k;
  int32_t maxit;
  int32_t p;
  int32_t zeta;
  int64_t s;
  double tol;
  uint64_t seed;
  int32_t precision;
  int32_t sketch;
  int32_t recover;
  int32_t profile;
  double trunc_tol;
  int32_t orth;
} skr_params;

/* Fill *p with defaults: k=2, maxit=200, p=20, zeta=8, s=0, tol=1e-6, seed=0,
 * SKR_FP64, sparse sign, stored basis, trunc_tol=1e-12, Euclidean orthogonalisation.  Returns SKR_OK. */
SKR_API int skr_params_default(skr_params* p);

/*
 * Create a sparse operator from a square CSR matrix M (n x n, nnz nonzeros).
 *   rowptr  host int32[n+1], rowptr[0] = 0, nondecreasing, rowptr[n] = nnz
 *   colind  host int32[nnz], each in [0, n)
 *   vals    host FP64[nnz]
 *   diag    host FP64[n] or NULL: an extra diagonal term, the operator is M + diag(diag)
 * The library copies the matrix to the device, builds the CSR of M^T (needed for the
 * Krylov space of B^T and for adjoint solves) and FP32 copies of both for mixed
 * precision.  Synchronises `stream` before returning.  Errors: SKR_EINVAL for a
 * malformed CSR (checked on the host), SKR_ENOMEM, SKR_EHIP.
 */
SKR_API int skr_op_create_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                      const double* vals, const double* diag, void* stream, skr_op* out);

/* Replace the diagonal term: diag is a device FP64[n] pointer (copied, stream-ordered)
 * or NULL to remove it.  Used to differentiate with respect to a reaction term. */
SKR_API int skr_op_set_diag(skr_op op, const double* diag, void* stream);

/* Size of the operator. */
SKR_API int skr_op_size(skr_op op, int64_t* n, int64_t* nnz);

SKR_API int skr_op_destroy(skr_op op);

/*
 * Solve A X + X B = C1 C2^T (Algorithm 1): Krylov spaces K(A, C1) and K(B^T, C2).
 *   C1  device FP64 n1 x r row-major,  C2  device FP64 n2 x r row-major,  1 <= r <= 16
 * On success *out holds X ~ X1 X2^T with X1: n1 x ell, X2: n2 x ell (ell <= d*r).
 * The call is stream-ordered on `stream` and synchronises it once per residual check
 * (reading rho) and at the end.  Returns SKR_OK, SKR_NOT_CONVERGED or SKR_BREAKDOWN
 * with valid factors, or a negative error.
 */
SKR_API int skr_solve(skr_op A, skr_op B, const double* C1, const double* C2, int64_t r,
              const skr_params* params, void* stream, skr_result* out);

/*
 * Solve the transposed equation A^T L + L B^T = G1 G2^T with the same method
 * (Krylov spaces K(A^T, G1) and K(B, G2)); arguments as for skr_solve.  Its factors
 * L ~ L1 L2^T give the gradient of a loss <G1 G2^T, X> with respect to the data of
 * the forward equation.
 */
SKR_API int skr_adjoint_solve(skr_op A, skr_op B, const double* G1, const double* G2, int64_t r,
                      const skr_params* params, void* stream, skr_result* out);

/*
 * Lyapunov specialisation (the paper's Sec. 4 setting): A X + X A^T = C C^T.  With B = A^T
 * and C2 = C1 = C the second Krylov space K(B^T, C2) of Algorithm 1 is K(A, C) itself; the
 * solve builds it once, with one embedding S_U (seed as above), so M_B = M_A and each block
 * step and each sign-iteration step does half of the tandem work.  Same parameters as
 * skr_solve (sketch sparse sign or none); requires r <= 4, k <= 10 and stored-basis recovery
 * (SKR_ENOTSUP otherwise).  The result holds factors of the symmetric X ~ X1 X2^T (both
 * n x ell; X1 and X2 themselves differ).  C: device FP64 n x r row-major.
 */
SKR_API int skr_lyap_solve(skr_op A, const double* C, int64_t r, const skr_params* params, void* stream,
                           skr_result* out);

/* Scalars of a result: rank ell of the factors, block steps d, last relative residual
 * estimate rho/||beta_1 beta_2^T||_F, and the status returned by the solve. */
SKR_API int skr_result_info(skr_result res, int64_t* ell, int32_t* iters, double* rho_rel, int32_t* status);

/* Copy up to `cap` residual-history entries (block step, relative estimate) to host
 * arrays; *len receives the number of entries available. */
SKR_API int skr_result_history(skr_result res, int32_t* d, double* rho_rel, int32_t cap, int32_t* len);

/* Copy the factors into caller buffers: X1 device FP64 n1 x ell, X2 device FP64
 * n2 x ell, row-major (ell from skr_result_info).  Stream-ordered, no sync. */
SKR_API int skr_result_copy_factors(skr_result res, double* X1, double* X2, void* stream);

/* Device-time breakdown of the solve in milliseconds (HIP events): block steps,
 * projected solves (incl. residual estimates), recovery.  Any pointer may be NULL. */
SKR_API int skr_result_timing(skr_result res, double* ms_steps, double* ms_proj, double* ms_recover);

/* Per-kernel-family device time of a solve run with params.profile != 0: family `idx`
 * (0 .. count-1) has a static name, a number of launches and their summed duration in
 * milliseconds (HIP events on the solve's stream).  *count receives the number of
 * families; idx out of range returns SKR_EINVAL. */
SKR_API int skr_result_kernel_stats(skr_result res, int32_t idx, int32_t* count, const char** name,
                                    int64_t* launches, double* ms);

/* Diagnostics of the last projected solve (eqn:reduced_sk) of a result: Newton steps of the
 * sign iteration, eigenvalues of the two projected matrices in the left half plane (handled
 * by deflation), and the relative residual of the projected Sylvester equation. */
SKR_API int skr_result_proj_stats(skr_result res, int32_t* newton_iters, int32_t* neg_a, int32_t* neg_b,
                                  double* proj_resid);

/* Number of residual checks whose projected equation could not be solved (the sign
 * iteration cannot separate the sketched projected matrices' spectra, which happens when the
 * truncated bases have become numerically dependent).  Such a check is skipped: the solve goes
 * on to the next one, and when the last check fails it returns SKR_NOT_CONVERGED with the
 * factors of the last check that was solved. */
SKR_API int skr_result_failed_checks(skr_result res, int32_t* failed);

SKR_API int skr_result_destroy(skr_result res);

/*
 * True relative residual ||A X + X B - C1 C2^T||_F / ||C1 C2^T||_F of X = X1 X2^T
 * (the definition of the residual matrix in Sec. 3), evaluated on the device from the
 * factors through QR factorisations of [A X1, X1, -C1] and [X2, B^T X2, C2].
 * All matrices device FP64 row-major; X1 n1 x ell, X2 n2 x ell, C1 n1 x r, C2 n2 x r.
 * Synchronises `stream`; result in *rel.
 */
SKR_API int skr_true_residual(skr_op A, skr_op B, const double* X1, const double* X2, int64_t ell,
                      const double* C1, const double* C2, int64_t r, void* stream, double* rel);

/*
 * The same for the transposed (adjoint) equation: ||A^T L + L B^T - G1 G2^T||_F / ||G1 G2^T||_F
 * of L = L1 L2^T (the factors skr_adjoint_solve returns), from QR factorisations of
 * [A^T L1, L1, -G1] and [L2, B L2, G2].  Arguments and layouts as for skr_true_residual.
 */
SKR_API int skr_true_residual_adjoint(skr_op A, skr_op B, const double* L1, const double* L2, int64_t ell,
                      const double* G1, const double* G2, int64_t r, void* stream, double* rel);

/*
 * Loss and gradients of L = tr(P1^T X P2), X = X1 X2^T, given the adjoint factors
 * Lam = L1 L2^T of A^T Lam + Lam B^T = P1 P2^T (dL = <Lam, dC1 C2^T + C1 dC2^T - dA X>):
 *   dC1 = L1 (L2^T C2)   n1 x r        dC2 = L2 (L1^T C1)   n2 x r
 *   dsig_i = -sum_j Lam_ij X_ij        n1   (gradient w.r.t. A's diagonal term)
 *   dP1 = X1 (X2^T P2)   n1 x q        dP2 = X2 (X1^T P1)   n2 x q
 * All arrays device FP64 row-major; ellx/elll are the factor ranks, q the columns of P.
 * Any output pointer may be NULL to skip it.  *loss is written to host memory and the
 * call synchronises `stream`.
 */
SKR_API int skr_pairing_grads(int64_t n1, int64_t n2, int64_t r, int64_t q,
                      const double* X1, const double* X2, int64_t ellx,
                      const double* L1, const double* L2, int64_t elll,
                      const double* C1, const double* C2, const double* P1, const double* P2,
                      double* loss, double* dC1, double* dC2, double* dsig,
                      double* dP1, double* dP2, void* stream);

/*
 * skr_pairing_grads for callers that cannot allocate device memory (code under HIP graph
 * capture, allocation-free serving loops, harnesses that forbid hipMalloc): the same
 * arguments, results and loss, but every temporary lives in one fixed device workspace of
 * SKR_PAIRING_SCRATCH_BYTES per device, which the library's code object holds from its load
 * until the process ends.  The call makes no hipMalloc/hipFree and no allocating library
 * call; the caller still provides every input and output buffer.  The temporaries are
 * 2 q ellx + (q ellx for each of dP1, dP2) + (elll r for each of dC1, dC2) + elll ellx (dsig)
 * doubles plus the partial sums of the long reductions (at most 256 of the largest of those
 * products); dsig needs room for at least one more row of ellx doubles and works through
 * the rows in chunks that fit.  Sizes beyond the workspace return SKR_EINVAL before any work
 * is queued.  The workspace is shared by every call on a device and keeps the last call's
 * contents (nothing in it needs to start at zero): the call synchronises `stream` before it
 * returns, so calls made one after another never overlap, but calls that overlap on one
 * device (from several host threads) race on the workspace and must not be made.
 */
#define SKR_PAIRING_SCRATCH_BYTES (32ll << 20)
SKR_API int skr_pairing_grads_noalloc(int64_t n1, int64_t n2, int64_t r, int64_t q,
                      const double* X1, const double* X2, int64_t ellx,
                      const double* L1, const double* L2, int64_t elll,
                      const double* C1, const double* C2, const double* P1, const double* P2,
                      double* loss, double* dC1, double* dC2, double* dsig,
                      double* dP1, double* dP2, void* stream);

/* Device memory and streams released by finished calls are kept by the library and
 * reused by later calls (a solve allocates its stored bases, gigabytes at large n, and
 * several streams).  This returns every cached block of every device to the HIP runtime;
 * blocks in use are unaffected.  Synchronises each device that holds cached blocks.
 * Returns SKR_OK. */
SKR_API int skr_release_cached_memory(void);

/* Thread-local message describing the last negative return on this thread. */
SKR_API const char* skr_last_error(void);

/* Library version string. */
SKR_API const char* skr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SKRYLOV_H */
