// Using the factorization (Section 3.3, eq. rss and the F^{-1} product after it).
//
//   F^{-1} = (prod W_i^{-1}) P_t D^{-1} P_t^* (prod' V_i^{-1})
//   V_i^{-1} z : z_R -= T^T z_S ; z_J -= E z_R          (E = X_JR X_RR^{-1})
//   W_i^{-1} z : z_R -= G z_J   ; z_S -= T z_R
//   D^{-1}     : z_R <- X_RR^{-1} z_R per record, z_top <- A_top^{-1} z_top
// Forward sweeps run in factor order (levels fine to coarse, colours ascending), the
// backward sweep in reverse order.  D^{-1} on R_i is applied right after V_i^{-1}: no
// later step reads or writes R_i.  Same-colour boxes touch disjoint entries of z, so one
// workgroup per box of a colour runs without atomics.
//
//   F = (prod V_i) P_t D P_t^* (prod' W_i)
//   W_i z : z_S += T z_R ; z_R += G z_J     (then D: z_R <- X_RR z_R)
//   V_i z : z_J += E z_R ; z_R += T^T z_S
#include "rss_internal.h"

namespace rss {

struct SweepArgs {
    int nmax, ldJ;
    const int* cnt;
    const int* krank;
    const int* nJ;
    const int* Sg;
    const int* Rg;
    const int* Jg;
    const void* T;
    const void* XJR;
    const void* G;
    const void* Xinv;
    const double* XRR;
};

template <typename TT>
__global__ void __launch_bounds__(256) k_solve_fwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    __shared__ double zS[kMaxBox], zR[kMaxBox], w[kMaxBox];
    __shared__ int sg[kMaxBox], rg[kMaxBox];
    const int tid = threadIdx.x;
    const int c = boxes[blockIdx.x];
    const int nj = a.nJ[c];
    if (nj == 0) return;
    const int n = a.cnt[c], k = a.krank[c], r = n - k;
    const int nmax = a.nmax, ldJ = a.ldJ;
    const int64_t bsz = (int64_t)nmax * nmax;
    const TT* T = (const TT*)a.T + c * bsz;
    const TT* Xi = (const TT*)a.Xinv + c * bsz;
    const TT* E = (const TT*)a.XJR + (int64_t)c * ldJ * nmax;
    const int* J = a.Jg + (int64_t)c * ldJ;
    for (int i = tid; i < k; i += 256) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += 256) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    for (int h = 0; h < nrhs; ++h) {
        double* zc = z + (int64_t)h * ld;
        for (int i = tid; i < k; i += 256) zS[i] = zc[sg[i]];
        for (int i = tid; i < r; i += 256) zR[i] = zc[rg[i]];
        __syncthreads();
        for (int b = tid; b < r; b += 256) {
            double s = zR[b];
            for (int q = 0; q < k; ++q) s -= (double)T[q + (int64_t)b * nmax] * zS[q];
            zR[b] = s;
        }
        __syncthreads();
        for (int b = tid; b < r; b += 256) {
            double s = 0.0;
            for (int q = 0; q < r; ++q) s += (double)Xi[b + (int64_t)q * nmax] * zR[q];
            w[b] = s;
        }
        __syncthreads();
        for (int jj = tid; jj < nj; jj += 256) {
            double s = 0.0;
            for (int b = 0; b < r; ++b) s += (double)E[jj + (int64_t)b * ldJ] * w[b];
            zc[J[jj]] -= s;
        }
        for (int b = tid; b < r; b += 256) zc[rg[b]] = w[b];
        __syncthreads();
    }
}

template <typename TT>
__global__ void __launch_bounds__(256) k_solve_bwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    __shared__ double zR[kMaxBox];
    __shared__ double part[4][kMaxBox];
    __shared__ int sg[kMaxBox], rg[kMaxBox];
    const int tid = threadIdx.x;
    const int c = boxes[blockIdx.x];
    const int nj = a.nJ[c];
    if (nj == 0) return;
    const int n = a.cnt[c], k = a.krank[c], r = n - k;
    const int nmax = a.nmax, ldJ = a.ldJ;
    const int64_t bsz = (int64_t)nmax * nmax;
    const TT* T = (const TT*)a.T + c * bsz;
    const TT* G = (const TT*)a.G + (int64_t)c * nmax * ldJ;
    const int* J = a.Jg + (int64_t)c * ldJ;
    for (int i = tid; i < k; i += 256) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += 256) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    const int wv = tid >> 6, lane = tid & 63;
    for (int h = 0; h < nrhs; ++h) {
        double* zc = z + (int64_t)h * ld;
        // z_R -= G z_J : wave wv sums over jj = wv, wv+4, ...; lanes over rows b
        for (int b0 = 0; b0 < r; b0 += 64) {
            int b = b0 + lane;
            double s = 0.0;
            if (b < r)
                for (int jj = wv; jj < nj; jj += 4) s += (double)G[b + (int64_t)jj * nmax] * zc[J[jj]];
            if (b < r) part[wv][b] = s;
        }
        __syncthreads();
        for (int b = tid; b < r; b += 256) {
            double v = zc[rg[b]] - (part[0][b] + part[1][b] + part[2][b] + part[3][b]);
            zR[b] = v;
            zc[rg[b]] = v;
        }
        __syncthreads();
        for (int q = tid; q < k; q += 256) {
            double s = 0.0;
            for (int b = 0; b < r; ++b) s += (double)T[q + (int64_t)b * nmax] * zR[b];
            zc[sg[q]] -= s;
        }
        __syncthreads();
    }
}

// y = F x: W_i then D on R_i (factor order)
__global__ void __launch_bounds__(256) k_apply_fwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    __shared__ double zR[kMaxBox], w[kMaxBox];
    __shared__ double part[4][kMaxBox];
    __shared__ int sg[kMaxBox], rg[kMaxBox];
    const int tid = threadIdx.x;
    const int c = boxes[blockIdx.x];
    const int nj = a.nJ[c];
    if (nj == 0) return;
    const int n = a.cnt[c], k = a.krank[c], r = n - k;
    const int nmax = a.nmax, ldJ = a.ldJ;
    const int64_t bsz = (int64_t)nmax * nmax;
    const double* T = (const double*)a.T + c * bsz;
    const double* G = (const double*)a.G + (int64_t)c * nmax * ldJ;
    const double* X = a.XRR + c * bsz;
    const int* J = a.Jg + (int64_t)c * ldJ;
    for (int i = tid; i < k; i += 256) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += 256) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    const int wv = tid >> 6, lane = tid & 63;
    for (int h = 0; h < nrhs; ++h) {
        double* zc = z + (int64_t)h * ld;
        for (int b = tid; b < r; b += 256) zR[b] = zc[rg[b]];
        __syncthreads();
        for (int q = tid; q < k; q += 256) {           // z_S += T z_R
            double s = 0.0;
            for (int b = 0; b < r; ++b) s += T[q + (int64_t)b * nmax] * zR[b];
            zc[sg[q]] += s;
        }
        __syncthreads();
        for (int b0 = 0; b0 < r; b0 += 64) {           // z_R += G z_J
            int b = b0 + lane;
            double s = 0.0;
            if (b < r)
                for (int jj = wv; jj < nj; jj += 4) s += G[b + (int64_t)jj * nmax] * zc[J[jj]];
            if (b < r) part[wv][b] = s;
        }
        __syncthreads();
        for (int b = tid; b < r; b += 256) zR[b] += part[0][b] + part[1][b] + part[2][b] + part[3][b];
        __syncthreads();
        for (int b = tid; b < r; b += 256) {           // z_R <- X_RR z_R
            double s = 0.0;
            for (int q = 0; q < r; ++q) s += X[b + (int64_t)q * nmax] * zR[q];
            w[b] = s;
        }
        __syncthreads();
        for (int b = tid; b < r; b += 256) zc[rg[b]] = w[b];
        __syncthreads();
    }
}

// y = F x: V_i (reverse order)
__global__ void __launch_bounds__(256) k_apply_bwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    __shared__ double zR[kMaxBox], w[kMaxBox];
    __shared__ int sg[kMaxBox], rg[kMaxBox];
    const int tid = threadIdx.x;
    const int c = boxes[blockIdx.x];
    const int nj = a.nJ[c];
    if (nj == 0) return;
    const int n = a.cnt[c], k = a.krank[c], r = n - k;
    const int nmax = a.nmax, ldJ = a.ldJ;
    const int64_t bsz = (int64_t)nmax * nmax;
    const double* T = (const double*)a.T + c * bsz;
    const double* Xi = (const double*)a.Xinv + c * bsz;
    const double* E = (const double*)a.XJR + (int64_t)c * ldJ * nmax;
    const int* J = a.Jg + (int64_t)c * ldJ;
    for (int i = tid; i < k; i += 256) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += 256) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    for (int h = 0; h < nrhs; ++h) {
        double* zc = z + (int64_t)h * ld;
        for (int b = tid; b < r; b += 256) zR[b] = zc[rg[b]];
        __syncthreads();
        for (int b = tid; b < r; b += 256) {           // w = X_RR^{-1} z_R
            double s = 0.0;
            for (int q = 0; q < r; ++q) s += Xi[b + (int64_t)q * nmax] * zR[q];
            w[b] = s;
        }
        __syncthreads();
        for (int jj = tid; jj < nj; jj += 256) {       // z_J += X_JR w
            double s = 0.0;
            for (int b = 0; b < r; ++b) s += E[jj + (int64_t)b * ldJ] * w[b];
            zc[J[jj]] += s;
        }
        __syncthreads();
        for (int b = tid; b < r; b += 256) {           // z_R += T^T z_S
            double s = 0.0;
            for (int q = 0; q < k; ++q) s += T[q + (int64_t)b * nmax] * zc[sg[q]];
            zc[rg[b]] = zR[b] + s;
        }
        __syncthreads();
    }
}

static SweepArgs sweep_args(const Level& L, int use32) {
    SweepArgs a;
    a.nmax = L.nmax; a.ldJ = L.ldJ; a.cnt = L.cnt; a.krank = L.krank; a.nJ = L.nJ;
    a.Sg = L.Sg; a.Rg = L.Rg; a.Jg = L.Jg; a.XRR = L.XRR;
    if (use32) { a.T = L.T32; a.XJR = L.XJR32; a.G = L.G32; a.Xinv = L.Xinv32; }
    else { a.T = L.T; a.XJR = L.XJR; a.G = L.G; a.Xinv = L.Xinv; }
    return a;
}

void launch_solve_fwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld, int use32,
                      hipStream_t s) {
    if (nboxes <= 0) return;
    SweepArgs a = sweep_args(L, use32);
    if (use32) k_solve_fwd<float><<<dim3(nboxes), dim3(256), 0, s>>>(a, boxes, z, nrhs, ld);
    else k_solve_fwd<double><<<dim3(nboxes), dim3(256), 0, s>>>(a, boxes, z, nrhs, ld);
}

void launch_solve_bwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld, int use32,
                      hipStream_t s) {
    if (nboxes <= 0) return;
    SweepArgs a = sweep_args(L, use32);
    if (use32) k_solve_bwd<float><<<dim3(nboxes), dim3(256), 0, s>>>(a, boxes, z, nrhs, ld);
    else k_solve_bwd<double><<<dim3(nboxes), dim3(256), 0, s>>>(a, boxes, z, nrhs, ld);
}

void launch_apply_fwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      hipStream_t s) {
    if (nboxes <= 0) return;
    k_apply_fwd<<<dim3(nboxes), dim3(256), 0, s>>>(sweep_args(L, 0), boxes, z, nrhs, ld);
}

void launch_apply_bwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      hipStream_t s) {
    if (nboxes <= 0) return;
    k_apply_bwd<<<dim3(nboxes), dim3(256), 0, s>>>(sweep_args(L, 0), boxes, z, nrhs, ld);
}

// ---- top block ------------------------------------------------------------------------
__global__ void k_gather_top(const int* __restrict__ idx, int64_t ntop, const double* __restrict__ z, int nrhs,
                             int64_t ld, double* __restrict__ tmp) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntop * nrhs) return;
    int64_t i = e % ntop, h = e / ntop;
    tmp[e] = z[h * ld + idx[i]];
}

template <typename TT>
__global__ void k_top_gemv(const int* __restrict__ idx, int64_t ntop, const TT* __restrict__ M,
                           const double* __restrict__ tmp, int nrhs, double* __restrict__ z, int64_t ld) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int h = blockIdx.y;
    if (i >= ntop) return;
    const double* x = tmp + (int64_t)h * ntop;
    double s = 0.0;
    for (int64_t j = 0; j < ntop; ++j) s += (double)M[i + j * ntop] * x[j];
    z[(int64_t)h * ld + idx[i]] = s;
}

void launch_top_apply(const int* top_idx, int64_t ntop, const double* M, const float* M32, double* z, int nrhs,
                      int64_t ld, double* tmp, hipStream_t s) {
    if (ntop <= 0) return;
    int64_t tot = ntop * nrhs;
    k_gather_top<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(top_idx, ntop, z, nrhs, ld, tmp);
    dim3 grid((unsigned)((ntop + 255) / 256), nrhs);
    if (M32) k_top_gemv<float><<<grid, dim3(256), 0, s>>>(top_idx, ntop, M32, tmp, nrhs, z, ld);
    else k_top_gemv<double><<<grid, dim3(256), 0, s>>>(top_idx, ntop, M, tmp, nrhs, z, ld);
}

__global__ void k_convert_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

void launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
    k_convert_f32<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(src, dst, n);
}

__global__ void k_copy_cols(const double* __restrict__ src, int64_t lds, double* __restrict__ dst, int64_t ldd,
                            int64_t n, int nrhs) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    int64_t i = e % n, h = e / n;
    dst[h * ldd + i] = src[h * lds + i];
}

void launch_copy_cols(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int nrhs,
                      hipStream_t s) {
    int64_t tot = n * nrhs;
    k_copy_cols<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(src, lds, dst, ldd, n, nrhs);
}

// Dense LU with partial pivoting of the top block (one workgroup), log|det|, then the
// explicit inverse by solves against identity columns (many workgroups).
__global__ void __launch_bounds__(1024) k_top_lu(double* __restrict__ A, int64_t n, int* __restrict__ piv,
                                                 int* flag, double* logdet, int* sign) {
    __shared__ int piv_idx;
    __shared__ double piv_val;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    double lds = 0.0;
    int sgn = 1;
    for (int64_t j = 0; j < n; ++j) {
        if (wv == 0) {
            double best = -1.0;
            int64_t bi = INT64_MAX;
            for (int64_t i = j + lane; i < n; i += 64) {
                double v = fabs(A[i + j * n]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                double v2 = __shfl_xor(best, o, 64);
                int64_t i2 = __shfl_xor(bi, o, 64);
                if (v2 > best || (v2 == best && i2 < bi)) { best = v2; bi = i2; }
            }
            if (lane == 0) { piv_idx = (int)bi; piv_val = best; }
        }
        __syncthreads();
        const int64_t p = piv_idx;
        const double pv = piv_val;
        if (!(pv > 0.0)) {
            if (tid == 0) atomicOr(flag, 8);
            return;
        }
        if (tid == 0) piv[j] = (int)p;
        if (p != j) {
            for (int64_t l = tid; l < n; l += 1024) {
                double t0 = A[j + l * n];
                A[j + l * n] = A[p + l * n];
                A[p + l * n] = t0;
            }
            sgn = -sgn;
        }
        __syncthreads();
        const double d = A[j + j * n];
        lds += log(fabs(d));
        if (d < 0) sgn = -sgn;
        const double rinv = 1.0 / d;
        for (int64_t i = j + 1 + tid; i < n; i += 1024) A[i + j * n] *= rinv;
        __syncthreads();
        {
            // trailing update, 64 rows x 16 columns of threads (no integer division)
            const int ni = (int)n, jj = (int)j;
            for (int l = jj + 1 + wv; l < ni; l += 16) {
                const double ajl = A[jj + (int64_t)l * n];
                for (int i = jj + 1 + lane; i < ni; i += 64) A[i + (int64_t)l * n] -= A[i + j * n] * ajl;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        *logdet = lds;
        *sign = sgn;
        // row permutation of P A = L U: row i of P A is row perm[i] of A
        int* perm = piv + n;
        for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
        for (int64_t j = 0; j < n; ++j) {
            int p = piv[j];
            int t0 = perm[j]; perm[j] = perm[p]; perm[p] = t0;
        }
    }
}

// Columns [c0, c0 + NC) of A^{-1} from P A = L U, solved in LDS (n <= 1024).
template <int NC>
__global__ void __launch_bounds__(256) k_top_inverse_lds(const double* __restrict__ LU, const int* __restrict__ perm,
                                                         int64_t n, double* __restrict__ Ainv) {
    extern __shared__ double xs[];   // n x NC, xs[i * NC + c]
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * NC;
    for (int64_t e = tid; e < n * NC; e += 256) {
        int64_t i = e / NC, c = e % NC;
        xs[e] = (perm[i] == c0 + c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int64_t j = 0; j < n; ++j) {          // L y = P e (unit lower)
        const int64_t m = n - j - 1;
        for (int64_t e = tid; e < m * NC; e += 256) {
            int64_t i = j + 1 + e / NC, c = e % NC;
            xs[i * NC + c] -= LU[i + j * n] * xs[j * NC + c];
        }
        __syncthreads();
    }
    for (int64_t j = n - 1; j >= 0; --j) {     // U x = y
        if (tid < NC) xs[j * NC + tid] /= LU[j + j * n];
        __syncthreads();
        for (int64_t e = tid; e < j * NC; e += 256) {
            int64_t i = e / NC, c = e % NC;
            xs[i * NC + c] -= LU[i + j * n] * xs[j * NC + c];
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < n * NC; e += 256) {
        int64_t i = e % n, c = e / n;
        if (c0 + c < n) Ainv[(c0 + c) * n + i] = xs[i * NC + c];
    }
}

__global__ void k_top_inverse(const double* __restrict__ LU, const int* __restrict__ piv, int64_t n,
                              double* __restrict__ Ainv) {
    int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n) return;
    double* x = Ainv + col * n;
    for (int64_t i = 0; i < n; ++i) x[i] = (i == col) ? 1.0 : 0.0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t p = piv[j];
        if (p != j) { double t0 = x[j]; x[j] = x[p]; x[p] = t0; }
    }
    for (int64_t j = 0; j < n; ++j) {
        double xj = x[j];
        if (xj != 0.0)
            for (int64_t i = j + 1; i < n; ++i) x[i] -= LU[i + j * n] * xj;
    }
    for (int64_t j = n - 1; j >= 0; --j) {
        double xj = x[j] / LU[j + j * n];
        x[j] = xj;
        for (int64_t i = 0; i < j; ++i) x[i] -= LU[i + j * n] * xj;
    }
}

void launch_lu_inverse(double* A, double* Ainv, int64_t n, int* piv, double* work, int* flag, double* logdet,
                       int* sign, hipStream_t s) {
    (void)work;
    if (n <= 0) return;
    k_top_lu<<<dim3(1), dim3(1024), 0, s>>>(A, n, piv, flag, logdet, sign);
    constexpr int NC = 8;
    if (n <= 1024) {
        size_t lds = sizeof(double) * (size_t)n * NC;
        k_top_inverse_lds<NC><<<dim3((unsigned)((n + NC - 1) / NC)), dim3(256), lds, s>>>(A, piv + n, n, Ainv);
    } else {
        k_top_inverse<<<dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s>>>(A, piv, n, Ainv);
    }
}

}  // namespace rss
