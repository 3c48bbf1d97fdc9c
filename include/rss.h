/*
 * rss.h -- C ABI of librss: strong recursive skeletonization factorization (RS-S)
 * of kernel integral-equation matrices on one AMD Instinct MI355X (gfx950).
 *
 * Method: Minden, Ho, Damle, Ying, "A recursive skeletonization factorization
 * based on strong admissibility" (arXiv:1609.08130).
 *
 * Problem statement (Section 1, eqs. bie, linear, discbie): given N distinct points
 * x_i, the matrix is
 *     A_ii = diag,    A_ij = weight * K(x_i - x_j)  (i != j),
 *     K(z) = -log|z| / (2 pi)                       (2D Laplace, Section 3.2).
 * rss_factor_create builds F ~ A (eq. rss, Algorithm 1) to tolerance tol;
 * rss_solve applies F^{-1} (Section 3.3, the F^{-1} product), rss_apply applies F,
 * rss_logdet returns log det D (Section 3.3), rss_sqrt_apply applies the generalized
 * square root F^{1/2} or its adjoint (Section 3.3), rss_matvec applies A exactly and
 * rss_gmres solves A x = b by GMRES preconditioned with F^{-1} (Section 4 uses F
 * as a preconditioner for an outer Krylov iteration).
 *
 * Conventions
 *  - Pointers named d_* are DEVICE pointers (hipMalloc'd or torch CUDA tensors on
 *    the current device).  The caller owns them; the library never keeps them
 *    after a call returns.  rss_factor_create copies the points.  Pointers named h_*
 *    (and the plain output pointers of the query calls) are HOST pointers.
 *  - Points: N x dim FP64, row-major (x0, y0, x1, y1, ...).  DOF i is point i.
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
    RSS_E_UNSUPPORTED = 5,  /* a kernel, dimension, size or mode this version does not handle */
    RSS_E_NOCONV = 6,       /* rss_gmres reached maxit before rtol */
    RSS_E_ARENA = 7         /* the factorization needs more device memory than arena_bytes */
} rss_status;

/* Kernel K of the integral operator (Section 1 eq. discbie; Section 4 Examples 1 and 2).
 * This version factors RSS_K_LAPLACE2D; the others return RSS_E_UNSUPPORTED. */
typedef enum { RSS_K_LAPLACE2D = 0, RSS_K_LAPLACE3D = 1, RSS_K_HELMHOLTZ2D = 2 } rss_kernel;

typedef enum { RSS_FP64 = 0, RSS_MIXED = 1 } rss_precision;

/* The factorization: RS-S (strong skeletonization at every level, Algorithm 1) or RS-WS
 * (Section 3.4, Algorithm 2: at every level a weak skeletonization pass, which compresses
 * each box against everything outside it and eliminates its redundant DOFs against its own
 * skeleton, then the strong pass on what remains; one more weak pass after the last level,
 * eq. rws).  RS-WS stores less (Section 3.4). */
typedef enum { RSS_METHOD_STRONG = 0, RSS_METHOD_HYBRID = 1 } rss_method;

/* Most DOFs the top block (Section 3.3, the final dense factorization) may hold. */
#define RSS_MAX_TOP 16384

typedef struct {
    uint32_t struct_size;   /* sizeof(rss_params); checked as an ABI guard */
    int32_t  dim;           /* spatial dimension d of the points: 2 */
    int32_t  kernel;        /* rss_kernel */
    int32_t  symmetric;     /* 1: K real symmetric, so A_BF^* = A_FB and the ID of the far
                               field is one-sided with T^T on the row side (Section 3.2);
                               0 (the two-sided stack of eq. skelid): RSS_E_UNSUPPORTED */
    double   diag;          /* A_ii */
    double   weight;        /* w in A_ij = w * K(x_i - x_j) */
    double   kappa;         /* wavenumber of RSS_K_HELMHOLTZ2D (ignored otherwise) */
    double   tol;           /* ID tolerance epsilon >= 0 (Definition 1) */
    int32_t  leaf_size;     /* n_occ: the tree is refined uniformly until no leaf box holds more */
    int32_t  n_proxy;       /* proxy points on the circle Gamma (Section 3.2), 1..64 */
    double   proxy_radius;  /* radius of Gamma in box side lengths, in (0.5*sqrt(d), 2.5] */
    double   root_lo[3];    /* lower corner of the root box (first dim entries used) */
    double   root_side;     /* side of the root box; <= 0: bounding box of the points */
    int32_t  precision;     /* rss_precision: RSS_MIXED computes the Schur-complement
                               products between different boxes in FP32, keeps an FP32
                               copy of the factor for rss_solve and, when tol >= 16 *
                               2^-24 (~9.5e-7), keeps the blocks A_{B_a,B_b} with a != b
                               of the block store in FP32.  The self blocks A_{B_a,B_a}
                               and the skeleton-skeleton products (O(1) entries), the ID
                               (double-double Gram and pivoted Cholesky), the
                               eliminations, the LU factors and the records stay FP64, so
                               |A - F| matches the FP64 factor's; rss_solve with the FP32
                               copy is accurate to a few 2^-24 and rss_gmres refines to
                               any rtol */
    int32_t  method;        /* rss_method */
    int32_t  level_graphs;  /* 1: the launches of each pass over a level (the ID, elimination
                               and Schur kernels of all its colours, Section 5's colouring
                               making the boxes of one colour independent) are captured into
                               one HIP graph and launched as one; a thread reuses the
                               executable graph of the same level and pass of its previous
                               factorization, updated in place.  0: launched one by one
                               (the per-phase times of rss_info are split by kernel then) */
    int32_t  max_box;       /* largest box the recursion compresses, in active DOFs: when a box
                               of the next level up would hold more, Algorithm 1 ends after the
                               current level and every active DOF left forms the top block
                               (its upper levels left uncompressed, so F is no less accurate;
                               the RS-WS weak step at depth 1 is skipped likewise).  0: the
                               kernels' limit, 256.  Otherwise 1..256.  A top block of more
                               than RSS_MAX_TOP DOFs fails with RSS_E_UNSUPPORTED */
    uint64_t arena_bytes;   /* 0: no limit; otherwise the most device memory the factor may
                               hold at any time (store, records, workspaces), failing with
                               RSS_E_ARENA (nothing leaked) when the build needs more */
} rss_params;

/* Fill *p with the defaults for dimension `dim` and kernel `kernel`: diag 1, weight 1,
 * kappa 0, tol 1e-6, leaf 64, 16 proxies at radius 1.25 sides, root box [0,1]^dim,
 * symmetric 1, FP64, RS-S, no arena limit (Section 4 Example 1 settings, with the leaf size and
 * proxy count of the workloads here).  Leaves *p untouched when p is NULL. */
void rss_params_default(rss_params* p, int32_t dim, int32_t kernel);

/* Build F ~ A (Section 3.3, Algorithm 1).  d_points: device, n x dim FP64 row-major.
 * Synchronizes `stream`.  Errors: RSS_E_ARG (n < 1, bad params, point outside the root
 * box, non-finite or duplicate points), RSS_E_UNSUPPORTED (kernel, dim or symmetric mode
 * not built, tree deeper than 12 levels), RSS_E_SINGULAR, RSS_E_ARENA, RSS_E_NOMEM,
 * RSS_E_DEVICE. */
rss_status rss_factor_create(const double* d_points, int64_t n, const rss_params* p,
                             void* stream, rss_factor* out);

/* x = F^{-1} b (Section 3.3, F^{-1} = (prod W_i^{-1}) P_t D^{-1} P_t^* (prod' V_i^{-1})).
 * d_b, d_x: device, N x nrhs, leading dimension ld.  d_x == d_b is allowed.  Uses the
 * FP32 factor copy when the factor is RSS_MIXED and use_fp32 != 0; otherwise FP64. */
rss_status rss_solve(rss_factor f, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                     int32_t use_fp32, void* stream);

/* y = F x (Section 3.3 eq. rss, F = (prod V_i) P_t D P_t^* (prod' W_i)).  d_x and d_y
 * must not alias. */
rss_status rss_apply(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld,
                     void* stream);

/* y = A x exactly, the operator of Section 1 eq. discbie that Section 4 applies by FFT or
 * a fast multipole method (d_x, d_y must not alias): by FFT convolution when the points
 * form a uniform n x n grid in DOF order i + n j (detected at factor creation; the matrix
 * minus its diagonal is then block Toeplitz), otherwise by direct summation. */
rss_status rss_matvec(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld,
                      void* stream);

/* Solve A x = b (one right-hand side) by restarted GMRES(restart) with modified
 * Gram-Schmidt, right-preconditioned by F^{-1} (Section 4 preconditions its Krylov
 * iteration with F), x0 = 0, until the true residual |b - A x| / |b| <= rtol.  FP64
 * throughout except the preconditioner, which uses the FP32 factor copy when
 * use_fp32 != 0 on a mixed factor.  Synchronizes.  Returns RSS_E_NOCONV when maxit
 * iterations do not reach rtol (x holds the last iterate, *iters and *relres are set). */
rss_status rss_gmres(rss_factor f, const double* d_b, double* d_x, double rtol, int32_t maxit,
                     int32_t restart, int32_t use_fp32, void* stream, int32_t* iters,
                     double* relres);

/* rss_gmres for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same iteration, bit for bit,
 * with its Krylov basis and work vectors in a device array of the library instead of memory
 * allocated per call.  The array holds RSS_GMRES_NOALLOC_BYTES (256 MiB); every GPU the
 * library runs on holds its own copy until the process ends.  Limits: restart <= 64 and
 * (2 restart + 3) N + 1024 <= RSS_GMRES_NOALLOC_BYTES / 8 doubles (N = 1048576 allows
 * restart <= 14), else RSS_E_ARG with nothing written.  All calls on one GPU share the
 * array, which keeps the last call's contents (each call writes every entry before reading
 * it): calls that overlap in time on one GPU race, and the caller must serialize them. */
#define RSS_GMRES_NOALLOC_BYTES ((uint64_t)256 << 20)
rss_status rss_gmres_noalloc(rss_factor f, const double* d_b, double* d_x, double rtol, int32_t maxit,
                             int32_t restart, int32_t use_fp32, void* stream, int32_t* iters,
                             double* relres);

/* log det F = log det D (Section 3.3: the V_i, W_i are unit triangular, and log|D|
 * approximates log|K|) as a complex number re + i im with im in (-pi, pi]: for a real
 * matrix re = log|det F| and im = 0 (det > 0) or pi (det < 0). */
rss_status rss_logdet(rss_factor f, double* re, double* im);

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

/* Tree depth D of the uniform tree (Section 3: leaves at depth D; Algorithm 1
 * skeletonizes depths D..2, the paper's levels 1..L-2) and the number of DOFs of the
 * top block B_t of the final factorization (Section 3.3). */
rss_status rss_shape(rss_factor f, int32_t* depth, int64_t* n_top);

/* Skeleton and redundant DOFs (host arrays of global indices, ascending) of box `box`
 * (linear index bx + 2^depth * by) at tree depth `depth`: the partition B = S u R that
 * its interpolative decomposition (Section 2.2, Definition 1; Section 3.1 eq. skelid)
 * chose, in the strong step (weak == 0) or, for RS-WS, the weak step (weak == 1,
 * Section 3.4 eq. weakskel).  A box without redundant DOFs reports all its DOFs as
 * skeleton and *nr = 0.  Capacities too small: RSS_E_ARG with the needed sizes in *ns,
 * *nr; no such step: RSS_E_ARG. */
rss_status rss_box_sets(rss_factor f, int32_t depth, int64_t box, int32_t weak, int64_t* skel,
                        int32_t cap_s, int32_t* ns, int64_t* red, int32_t cap_r, int32_t* nr);

/* The factored operators of one strong skeletonization step (Section 3.1: eqs. skelid,
 * zab, skelop; the block elimination of Section 2.1 eq. landu with I = R, J = S u N),
 * copied to host arrays, FP64 column-major:
 *   h_T   |S| x |R|  interpolation matrix T (A_{:,R} ~ A_{:,S} T),
 *   h_XRR |R| x |R|  X_RR after the two triangular operations U_T, L_T,
 *   h_XJR |J| x |R|  X_JR (rows S, then the active near field N in box order),
 *   h_G   |R| x |J|  X_RR^{-1} X_RJ,
 *   h_J   |J|        global DOF indices of J in the row order of h_XJR;
 * weak selects the step as for rss_box_sets (a weak step has J = S).
 * *ns, *nr, *nj receive |S|, |R|, |J| (0, 0, 0 when the box has no record); any output
 * pointer may be NULL to skip it, and `cap` is the entries available in each non-NULL
 * array (RSS_E_ARG, nothing copied, when one is too small). */
rss_status rss_box_record(rss_factor f, int32_t depth, int64_t box, int32_t weak, double* h_T,
                          double* h_XRR, double* h_XJR, double* h_G, int64_t* h_J, int64_t cap,
                          int32_t* ns, int32_t* nr, int32_t* nj);

/* The remaining active DOFs (global indices, ascending) that form the top block B_t of
 * the final factorization (Section 3.3). */
rss_status rss_top_set(rss_factor f, int64_t* idx, int64_t cap, int64_t* count);

/* JSON text of the measured quantities of Section 4 (t_f with a per-phase split, m_f as
 * device bytes) and the per-level realized sizes (sum and maximum of |S|, |R|, |J|) with
 * the algorithmic flop and byte counts of Theorem 2's terms; NUL-terminated, truncated to
 * cap bytes. */
rss_status rss_info(rss_factor f, char* buf, int64_t cap);

/* Release all device memory of f to the library's block cache.  NULL-safe.
 * Synchronizes the device (any stream may still be using the factor).  (Library
 * plumbing; no passage of the paper.) */
rss_status rss_factor_destroy(rss_factor f);

/* Return every cached device block to the device.  The library keeps released blocks
 * for reuse by later factorizations (repeated factorizations then allocate nothing);
 * call this to hand the memory back, e.g. before other large allocations.  (Library
 * plumbing; no passage of the paper.) */
rss_status rss_trim(void);

/* Description of the last failure on the calling thread ("" if none).  (Library
 * plumbing; no passage of the paper.) */
const char* rss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RSS_H */
