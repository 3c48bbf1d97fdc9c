/*
 * rss.h -- C ABI of librss: strong recursive skeletonization factorization (RS-S)
 * of kernel integral-equation matrices on one AMD Instinct MI355X (gfx950).
 *
 * Method: Minden, Ho, Damle, Ying, "A recursive skeletonization factorization
 * based on strong admissibility" (arXiv:1609.08130).
 *
 * Problem statement (Section 1, eqs. bie, linear, discbie): given N distinct points
 * x_i in the plane, the matrix is
 *     A_ii = diag,    A_ij = weight * K(x_i - x_j)  (i != j),
 *     K(z) = -log|z| / (2 pi)                       (2D Laplace, Section 3.2).
 * rss_factor_create builds F ~ A (eq. rss, Algorithm 1) to tolerance tol;
 * rss_solve applies F^{-1} (Section 3.3, the F^{-1} product), rss_apply applies F,
 * rss_logdet returns log|det D| (Section 3.3), rss_sqrt_apply applies the generalized
 * square root F^{1/2} or its adjoint (Section 3.3), rss_matvec applies A exactly and
 * rss_gmres solves A x = b by GMRES preconditioned with F^{-1} (Section 4 uses F
 * as a preconditioner for an outer Krylov iteration).
 *
 * Conventions
 *  - Pointers named d_* are DEVICE pointers (hipMalloc'd or torch CUDA tensors on
 *    the current device).  The caller owns them; the library never keeps them
 *    after a call returns.  rss_factor_create copies the points.
 *  - Points: N x 2 FP64, row-major (x0, y0, x1, y1, ...).  DOF i is point i.
 *  - Vectors: FP64, column-major N x nrhs with leading dimension ld >= N.
 *  - `stream` is a hipStream_t (NULL = default stream).  solve / apply / matvec
 *    are asynchronous on it; factor_create, gmres, logdet, info and the query calls
 *    synchronize it.
 *  - Every call returns an rss_status and never throws or aborts across the ABI.
 *    On failure rss_last_error() (thread-local) describes the cause; a failed
 *    rss_factor_create stores NULL in *out and leaks nothing.
 *  - One factor may be used by one thread at a time (internal workspaces); distinct
 *    factors are independent.
 */
#ifndef RSS_H
#define RSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rss_factor_s* rss_factor;

typedef enum {
    RSS_OK = 0,
    RSS_E_ARG = 1,          /* invalid argument (sizes, tolerance, non-finite or duplicate points) */
    RSS_E_NOMEM = 2,        /* device allocation failed */
    RSS_E_DEVICE = 3,       /* a HIP runtime call or kernel failed */
    RSS_E_SINGULAR = 4,     /* an exactly singular pivot block (X_RR or the top block) */
    RSS_E_UNSUPPORTED = 5,  /* a size or mode the library does not handle (e.g. |B| > 256) */
    RSS_E_NOCONV = 6        /* rss_gmres reached maxit before rtol */
} rss_status;

typedef enum { RSS_FP64 = 0, RSS_MIXED = 1 } rss_precision;

typedef struct {
    uint32_t struct_size;   /* sizeof(rss_params); checked as an ABI guard */
    int32_t  dim;           /* 2 */
    double   diag;          /* A_ii */
    double   weight;        /* w in A_ij = w * K(x_i - x_j) */
    double   tol;           /* ID tolerance epsilon >= 0 (Definition 1) */
    int32_t  leaf_size;     /* n_occ: the tree is refined uniformly until no leaf box holds more */
    int32_t  n_proxy;       /* proxy points on the circle Gamma (Section 3.2), 1..64 */
    double   proxy_radius;  /* radius of Gamma in box side lengths, in (0.5*sqrt(2), 2.5] */
    double   root_lo[2];    /* lower corner of the root box */
    double   root_side;     /* side of the root box; <= 0: bounding square of the points */
    int32_t  precision;     /* rss_precision: RSS_MIXED computes the Schur-complement
                               products in FP32, keeps an FP32 copy of the factor for
                               rss_solve and, when tol >= 16 * 2^-24 (~9.5e-7), keeps the
                               block store (the current A_{B_a,B_b} blocks) in FP32; the
                               ID (double-double Gram and pivoted Cholesky), the
                               eliminations, the LU factors and the FP64 records stay
                               FP64.  The factor is then accurate to ~1e-7; rss_gmres
                               refines to any rtol */
} rss_params;

/* Fill *p with the defaults: dim 2, diag 1, weight 1, tol 1e-6, leaf 64, 16 proxies at
 * radius 1.25, root box [0,1]^2, FP64. */
void rss_params_default(rss_params* p);

/* Build F ~ A (Algorithm 1).  d_points: device, n x 2 FP64 row-major.  Synchronizes
 * `stream`.  Errors: RSS_E_ARG (n < 1, bad params, point outside the root box,
 * non-finite or duplicate points), RSS_E_UNSUPPORTED (tree deeper than 12 levels or a
 * box with more than 256 active DOFs), RSS_E_SINGULAR, RSS_E_NOMEM, RSS_E_DEVICE. */
rss_status rss_factor_create(const double* d_points, int64_t n, const rss_params* p,
                             void* stream, rss_factor* out);

/* x = F^{-1} b (Section 3.3).  d_b, d_x: device, N x nrhs, leading dimension ld.
 * d_x == d_b is allowed.  Uses the FP32 factor copy when the factor is RSS_MIXED and
 * use_fp32 != 0; otherwise FP64. */
rss_status rss_solve(rss_factor f, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                     int32_t use_fp32, void* stream);

/* y = F x (eq. rss).  d_x and d_y must not alias. */
rss_status rss_apply(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld,
                     void* stream);

/* y = A x exactly (d_x, d_y must not alias): by FFT convolution when the points form a
 * uniform n x n grid in DOF order i + n j (detected at factor creation; the matrix minus
 * its diagonal is then block Toeplitz), otherwise by direct summation. */
rss_status rss_matvec(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld,
                      void* stream);

/* Solve A x = b (one right-hand side) by restarted GMRES(restart) with modified
 * Gram-Schmidt, right-preconditioned by F^{-1}, x0 = 0, until the true residual
 * |b - A x| / |b| <= rtol.  FP64 throughout except the preconditioner, which uses the
 * FP32 factor copy when use_fp32 != 0 on a mixed factor.  Synchronizes.  Returns
 * RSS_E_NOCONV when maxit iterations do not reach rtol (x holds the last iterate). */
rss_status rss_gmres(rss_factor f, const double* d_b, double* d_x, double rtol, int32_t maxit,
                     int32_t restart, int32_t use_fp32, void* stream, int32_t* iters,
                     double* relres);

/* sign * exp(logabs) = det D = det F (the V_i, W_i are unit triangular). */
rss_status rss_logdet(rss_factor f, double* sign, double* logabs);

/* Generalized square root of F for a positive definite matrix (Section 3.3):
 *     C = F^{1/2} = (prod V_i) P_t D^{1/2},   F = C C^*,
 * with D^{1/2} the lower Cholesky factor of each diagonal block of D (X_RR of every
 * skeletonization step and the top block) and C^* = D^{1/2 *} P_t^* (prod' W_i), which
 * uses V_i = W_i^* (a symmetric kernel).  adjoint == 0: y = C x; otherwise y = C^* x.
 * d_x, d_y: device, N x nrhs, leading dimension ld, must not alias.  FP64 records.  The
 * first call on a factor computes the Cholesky factors (one more N-sized set of blocks,
 * kept until rss_factor_destroy) and synchronizes the stream; RSS_E_SINGULAR when a
 * block is not positive definite (then no square root exists and nothing is written). */
rss_status rss_sqrt_apply(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld,
                          int32_t adjoint, void* stream);

/* Tree depth D (leaves at depth D; levels D..2 are skeletonized) and the number of
 * DOFs in the top block. */
rss_status rss_shape(rss_factor f, int32_t* depth, int64_t* n_top);

/* Skeleton and redundant DOFs (global indices, ascending) of box `box` (linear index
 * bx + 2^depth * by) at tree depth `depth`, as decided by its strong skeletonization.
 * A box without redundant DOFs reports all its DOFs as skeleton and *nr = 0.
 * Capacities too small: RSS_E_ARG with the needed sizes in *ns, *nr. */
rss_status rss_box_sets(rss_factor f, int32_t depth, int64_t box, int64_t* skel, int32_t cap_s,
                        int32_t* ns, int64_t* red, int32_t cap_r, int32_t* nr);

/* The remaining active DOFs (global indices, ascending) that form the top block. */
rss_status rss_top_set(rss_factor f, int64_t* idx, int64_t cap, int64_t* count);

/* JSON text with per-level statistics, memory use and the algorithmic flop/byte
 * counts of the factorization; NUL-terminated, truncated to cap bytes. */
rss_status rss_info(rss_factor f, char* buf, int64_t cap);

/* Release all device memory of f to the library's block cache.  NULL-safe.
 * Synchronizes the device (any stream may still be using the factor). */
rss_status rss_factor_destroy(rss_factor f);

/* Return every cached device block to the device.  The library keeps released blocks
 * for reuse by later factorizations (repeated factorizations then allocate nothing);
 * call this to hand the memory back, e.g. before other large allocations. */
rss_status rss_trim(void);

/* Description of the last failure on the calling thread ("" if none). */
const char* rss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RSS_H */
