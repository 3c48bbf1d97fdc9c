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
//
//   F^{1/2} = (prod V_i) P_t D^{1/2}, D^{1/2} = Cholesky factors L of the blocks of D;
//   (F^{1/2})^* = D^{1/2 *} P_t^* (prod' W_i) (V_i = W_i^* for a symmetric matrix): the
//   F sweeps with L (before V_i) or L^T (after W_i) in place of X_RR.
//
// Several right-hand sides of one solve go through in groups of four per launch, each
// loaded entry of a record used for all of them.
#include <algorithm>

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
    const double* Lc;   // Cholesky factors of X_RR (square-root sweeps) or nullptr
};

// sum_{t < cnt} M[t * stride] v[t] in eight partial sums, with sixteen loads of M in
// flight at a time (eight for the tail).
template <typename TT>
__device__ inline double dot_strided(const TT* __restrict__ M, int64_t stride, const double* v, int cnt) {
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int t = 0;
    for (; t + 16 <= cnt; t += 16) {
        TT m[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) m[u] = M[(int64_t)(t + u) * stride];
#pragma unroll
        for (int u = 0; u < 16; ++u) s[u & 7] += (double)m[u] * v[t + u];
    }
    for (; t + 8 <= cnt; t += 8) {
        TT m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m[u] = M[(int64_t)(t + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += (double)m[u] * v[t + u];
    }
    for (; t < cnt; ++t) s[0] += (double)M[(int64_t)t * stride] * v[t];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// NR dot products sharing the loads of M: out[h] = sum_{t < cnt} M[t * stride] v[h * ldv + t].
// Per h the partial sums, their order and the final combination are those of
// dot_strided, so each result is bit for bit the single-vector one.
template <typename TT, int NR>
__device__ inline void dot_strided_m(const TT* __restrict__ M, int64_t stride, const double* v, int ldv, int cnt,
                                     double (&out)[NR], int vs = 1) {
    double s[NR][8];
#pragma unroll
    for (int h = 0; h < NR; ++h)
#pragma unroll
        for (int u = 0; u < 8; ++u) s[h][u] = 0.0;
    // loads in flight: sixteen, or eight for several FP64 vectors (registers); the
    // sequence of terms each partial sum receives is the same either way
    constexpr int UL = (sizeof(TT) == 8 && NR > 1) ? 8 : 16;
    int t = 0;
    for (; t + 16 <= cnt; t += 16) {
#pragma unroll
        for (int u0 = 0; u0 < 16; u0 += UL) {
            TT m[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) m[u] = M[(int64_t)(t + u0 + u) * stride];
#pragma unroll
            for (int u = 0; u < UL; ++u)
#pragma unroll
                for (int h = 0; h < NR; ++h) s[h][(u0 + u) & 7] += (double)m[u] * v[h * ldv + (t + u0 + u) * vs];
        }
    }
    for (; t + 8 <= cnt; t += 8) {
        TT m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m[u] = M[(int64_t)(t + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int h = 0; h < NR; ++h) s[h][u] += (double)m[u] * v[h * ldv + (t + u) * vs];
    }
    for (; t < cnt; ++t) {
        const TT m = M[(int64_t)t * stride];
#pragma unroll
        for (int h = 0; h < NR; ++h) s[h][0] += (double)m * v[h * ldv + t * vs];
    }
#pragma unroll
    for (int h = 0; h < NR; ++h)
        out[h] = ((s[h][0] + s[h][1]) + (s[h][2] + s[h][3])) + ((s[h][4] + s[h][5]) + (s[h][6] + s[h][7]));
}

// The value of another lane moved bit for bit by a DPP control that reaches every lane
// (quad permutations, half-row mirror).
template <int CTRL>
__device__ inline double dpp_double(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)((unsigned long long)b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Lanes per output for `outs` outputs on NTH threads: the largest of 8, 4, 2, 1 that still
// covers every output in one pass (1 when there are more outputs than threads).
template <int NTH>
__device__ inline int lanes_per_output(int outs) {
    int g = 8;
    while (g > 1 && outs * g > NTH) g >>= 1;
    return g;
}

// Outputs o < outs of y_o = sum_t M_o[t * stride] v_t, each split over G adjacent lanes
// (lane g of the group takes t = g, g + G, ...; the G parts are then added by a
// butterfly), NR vectors at once.  mrow(o) is the first entry of output o's terms.
// Called by every thread of the block (the butterfly needs whole groups).
template <typename TT, int NTH, int NR, class MRow, class Out>
__device__ inline void split_dots(int outs, int cnt, int64_t stride, const double* v, int ldv, MRow mrow, Out out) {
    const int tid = threadIdx.x;
    // FP32 records only: split FP64 rows measured slower (8-byte loads G rows apart)
    const int G = sizeof(TT) == 4 ? lanes_per_output<NTH>(outs) : 1;
    const int g = tid % G;
    for (int o0 = 0; o0 < outs; o0 += NTH / G) {
        const int o = o0 + tid / G;
        double res[NR];
        if (o < outs && g < cnt) {
            dot_strided_m<TT, NR>(mrow(o) + (int64_t)g * stride, stride * G, v + g, ldv, (cnt - g + G - 1) / G, res,
                                  G);
        } else {
#pragma unroll
            for (int h = 0; h < NR; ++h) res[h] = 0.0;
        }
#pragma unroll
        for (int h = 0; h < NR; ++h) {
            if (G >= 2) res[h] += dpp_double<0xB1>(res[h]);    // lane ^ 1 (quad permutation)
            if (G >= 4) res[h] += dpp_double<0x4E>(res[h]);    // lane ^ 2
            if (G >= 8) res[h] += dpp_double<0x141>(res[h]);   // the other quad of 8 (half-row mirror)
        }
        if (o < outs && g == 0) out(o, res);
    }
}

// NR = 1: the right-hand sides one after the other (nrhs of them).  NR > 1: nrhs <= NR
// right-hand sides together, so every entry of the record is loaded once for all of
// them.
template <typename TT, int NTH, int NR>
__global__ void __launch_bounds__(NTH) k_solve_fwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    constexpr int PL = kMaxBox;
    __shared__ double zS[NR * PL], zR[NR * PL], w[NR * PL];
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
    for (int i = tid; i < k; i += NTH) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += NTH) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    const int nh = NR == 1 ? 1 : nrhs;          // right-hand sides per pass
    const int npass = NR == 1 ? nrhs : 1;
    for (int pass = 0; pass < npass; ++pass) {
        double* z0 = z + (int64_t)pass * ld;
        for (int h = 0; h < nh; ++h) {
            const double* zc = z0 + (int64_t)h * ld;
            for (int i = tid; i < k; i += NTH) zS[h * PL + i] = zc[sg[i]];
            for (int i = tid; i < r; i += NTH) zR[h * PL + i] = zc[rg[i]];
        }
        __syncthreads();
        split_dots<TT, NTH, NR>(   // z_R -= T^T z_S
            r, k, 1, zS, PL, [&](int b) { return T + (int64_t)b * nmax; },
            [&](int b, const double(&o)[NR]) {
#pragma unroll
                for (int h = 0; h < NR; ++h) zR[h * PL + b] -= o[h];
            });
        __syncthreads();
        split_dots<TT, NTH, NR>(   // X_RR^{-1} z_R
            r, r, nmax, zR, PL, [&](int b) { return Xi + b; },
            [&](int b, const double(&o)[NR]) {
#pragma unroll
                for (int h = 0; h < NR; ++h) w[h * PL + b] = o[h];
            });
        __syncthreads();
        for (int jj = tid; jj < nj; jj += NTH) {   // z_J -= E w
            const int g = J[jj];
            double o[NR];
            dot_strided_m<TT, NR>(E + jj, ldJ, w, PL, r, o);
#pragma unroll
            for (int h = 0; h < NR; ++h)
                if (h < nh) z0[(int64_t)h * ld + g] -= o[h];
        }
        for (int b = tid; b < r; b += NTH)
            for (int h = 0; h < nh; ++h) z0[(int64_t)h * ld + rg[b]] = w[h * PL + b];
        __syncthreads();
    }
}

// Dynamic LDS: zJ[NR * ldJ], and for NR > 1 the wave partial sums part[NW][NR][nmax].
template <typename TT, int NTH, int NR>
__global__ void __launch_bounds__(NTH) k_solve_bwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    constexpr int NW = NTH / 64;
    extern __shared__ double dyn[];
    __shared__ double zR[NR * kMaxBox];
    __shared__ double part_s[NR == 1 ? NW * kMaxBox : 1];
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
    double* zJ = dyn;
    double* part = NR == 1 ? part_s : dyn + (int64_t)NR * ldJ;
    const int PL = NR == 1 ? kMaxBox : nmax;   // part[(w * NR + h) * PL + b]
    for (int i = tid; i < k; i += NTH) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += NTH) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    const int wv = tid >> 6, lane = tid & 63;
    const int q4 = (nj + NW - 1) / NW;   // J entries per wave
    const int nh = NR == 1 ? 1 : nrhs;
    const int npass = NR == 1 ? nrhs : 1;
    for (int pass = 0; pass < npass; ++pass) {
        double* z0 = z + (int64_t)pass * ld;
        for (int h = 0; h < nh; ++h)
            for (int jj = tid; jj < nj; jj += NTH) zJ[h * ldJ + jj] = z0[(int64_t)h * ld + J[jj]];
        __syncthreads();
        // z_R -= G z_J : wave wv takes a contiguous 1/NW of J, lanes take rows b
        const int j0 = wv * q4, j1 = min(nj, j0 + q4);
        for (int b0 = 0; b0 < r; b0 += 64) {
            const int b = b0 + lane;
            if (b < r) {
                double o[NR];
                if (j1 > j0) {
                    dot_strided_m<TT, NR>(G + b + (int64_t)j0 * nmax, nmax, zJ + j0, ldJ, j1 - j0, o);
                } else {
#pragma unroll
                    for (int h = 0; h < NR; ++h) o[h] = 0.0;
                }
#pragma unroll
                for (int h = 0; h < NR; ++h) part[(wv * NR + h) * PL + b] = o[h];
            }
        }
        __syncthreads();
        for (int b = tid; b < r; b += NTH)
            for (int h = 0; h < nh; ++h) {
                double sp = 0.0;
#pragma unroll
                for (int u = 0; u < NW; ++u) sp += part[(u * NR + h) * PL + b];
                double* zc = z0 + (int64_t)h * ld;
                const double v = zc[rg[b]] - sp;
                zR[h * kMaxBox + b] = v;
                zc[rg[b]] = v;
            }
        __syncthreads();
        split_dots<TT, NTH, NR>(   // z_S -= T z_R
            k, r, nmax, zR, kMaxBox, [&](int q) { return T + q; },
            [&](int q, const double(&o)[NR]) {
#pragma unroll
                for (int h = 0; h < NR; ++h)
                    if (h < nh) z0[(int64_t)h * ld + sg[q]] -= o[h];
            });
        __syncthreads();
    }
}

// y = F x: W_i then D on R_i (factor order).  z_S is updated before z_J is gathered (S is
// the first part of J).  Dynamic LDS: zJ[ldJ].
template <int NTH>
__global__ void __launch_bounds__(NTH) k_apply_fwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    constexpr int NW = NTH / 64;
    extern __shared__ double zJ[];
    __shared__ double zR[kMaxBox], w[kMaxBox];
    __shared__ double part[NW][kMaxBox];
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
    for (int i = tid; i < k; i += NTH) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += NTH) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    const int wv = tid >> 6, lane = tid & 63;
    const int q4 = (nj + NW - 1) / NW;   // J entries per wave
    for (int h = 0; h < nrhs; ++h) {
        double* zc = z + (int64_t)h * ld;
        for (int b = tid; b < r; b += NTH) zR[b] = zc[rg[b]];
        __syncthreads();
        for (int q = tid; q < k; q += NTH) zc[sg[q]] += dot_strided(T + q, nmax, zR, r);   // z_S += T z_R
        __syncthreads();
        for (int jj = tid; jj < nj; jj += NTH) zJ[jj] = zc[J[jj]];
        __syncthreads();
        // z_R += G z_J: wave wv takes a contiguous 1/NW of J, lanes take rows b
        const int j0 = wv * q4, j1 = min(nj, j0 + q4);
        for (int b0 = 0; b0 < r; b0 += 64) {
            const int b = b0 + lane;
            if (b < r) part[wv][b] = j1 > j0 ? dot_strided(G + b + (int64_t)j0 * nmax, nmax, zJ + j0, j1 - j0) : 0.0;
        }
        __syncthreads();
        for (int b = tid; b < r; b += NTH) {
            double sp = 0.0;
#pragma unroll
            for (int u = 0; u < NW; ++u) sp += part[u][b];
            zR[b] += sp;
        }
        __syncthreads();
        if (a.Lc) {   // z_R <- L^T z_R (L lower, column-major)
            const double* Lb = a.Lc + c * bsz;
            for (int b = tid; b < r; b += NTH) w[b] = dot_strided(Lb + (int64_t)b * nmax + b, 1, zR + b, r - b);
        } else {
            for (int b = tid; b < r; b += NTH) w[b] = dot_strided(X + b, nmax, zR, r);   // z_R <- X_RR z_R
        }
        __syncthreads();
        for (int b = tid; b < r; b += NTH) zc[rg[b]] = w[b];
        __syncthreads();
    }
}

// y = F x: V_i (reverse order).  z_J is updated before z_S is read (S is part of J).
template <int NTH>
__global__ void __launch_bounds__(NTH) k_apply_bwd(SweepArgs a, const int* __restrict__ boxes, double* z,
                                                   int nrhs, int64_t ld) {
    __shared__ double zR[kMaxBox], w[kMaxBox], zS[kMaxBox];
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
    for (int i = tid; i < k; i += NTH) sg[i] = a.Sg[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += NTH) rg[i] = a.Rg[(int64_t)c * nmax + i];
    __syncthreads();
    for (int h = 0; h < nrhs; ++h) {
        double* zc = z + (int64_t)h * ld;
        for (int b = tid; b < r; b += NTH) zR[b] = zc[rg[b]];
        __syncthreads();
        if (a.Lc) {   // z_R <- L z_R first (the square root of this record's block of D)
            const double* Lb = a.Lc + c * bsz;
            for (int b = tid; b < r; b += NTH) w[b] = dot_strided(Lb + b, nmax, zR, b + 1);
            __syncthreads();
            for (int b = tid; b < r; b += NTH) zR[b] = w[b];
            __syncthreads();
        }
        for (int b = tid; b < r; b += NTH) w[b] = dot_strided(Xi + b, nmax, zR, r);   // w = X_RR^{-1} z_R
        __syncthreads();
        for (int jj = tid; jj < nj; jj += NTH) zc[J[jj]] += dot_strided(E + jj, ldJ, w, r);   // z_J += X_JR w
        __syncthreads();
        for (int q = tid; q < k; q += NTH) zS[q] = zc[sg[q]];
        __syncthreads();
        for (int b = tid; b < r; b += NTH) zc[rg[b]] = zR[b] + dot_strided(T + (int64_t)b * nmax, 1, zS, k);   // z_R += T^T z_S
        __syncthreads();
    }
}

static SweepArgs sweep_args(const Level& L, int use32) {
    SweepArgs a;
    a.nmax = L.nmax; a.ldJ = L.ldJ; a.cnt = L.cnt; a.krank = L.krank; a.nJ = L.nJ;
    a.Sg = L.Sg; a.Rg = L.Rg; a.Jg = L.Jg; a.XRR = L.XRR; a.Lc = nullptr;
    if (use32) { a.T = L.T32; a.XJR = L.XJR32; a.G = L.G32; a.Xinv = L.Xinv32; }
    else { a.T = L.T; a.XJR = L.XJR; a.G = L.G; a.Xinv = L.Xinv; }
    return a;
}

// Several right-hand sides go through the sweeps in groups of kSolveGroup, each group in
// one launch per colour (the record is read once per group); one right-hand side, or a
// box size whose group buffers do not fit in LDS, takes the one-at-a-time kernels.
constexpr int kSolveGroup = 4;

template <typename TT, int NTH, int NR>
static void solve_fwd_k(const SweepArgs& a, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                        hipStream_t s) {
    k_solve_fwd<TT, NTH, NR><<<dim3(nboxes), dim3(NTH), 0, s>>>(a, boxes, z, nrhs, ld);
}

template <typename TT, int NTH, int NR>
static void solve_bwd_k(const SweepArgs& a, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                        size_t lds, hipStream_t s) {
    if (lds > 65536)
        hipFuncSetAttribute((const void*)k_solve_bwd<TT, NTH, NR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_solve_bwd<TT, NTH, NR><<<dim3(nboxes), dim3(NTH), lds, s>>>(a, boxes, z, nrhs, ld);
}

template <typename TT, int NTH>
static void solve_fwd_t(const SweepArgs& a, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                        hipStream_t s) {
    note_shape("solve_fwd_" + std::to_string(NTH) + (sizeof(TT) == 4 ? "_f32" : "_f64") + (nrhs > 1 ? "_multi" : ""));
    if (nrhs == 1) {
        solve_fwd_k<TT, NTH, 1>(a, boxes, nboxes, z, 1, ld, s);
        return;
    }
    for (int h0 = 0; h0 < nrhs; h0 += kSolveGroup)
        solve_fwd_k<TT, NTH, kSolveGroup>(a, boxes, nboxes, z + (int64_t)h0 * ld, std::min(kSolveGroup, nrhs - h0),
                                          ld, s);
}

template <typename TT, int NTH>
static void solve_bwd_t(const SweepArgs& a, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                        hipStream_t s) {
    constexpr int NW = NTH / 64;
    const size_t lds1 = sizeof(double) * (size_t)a.ldJ;
    const size_t ldsg = sizeof(double) * ((size_t)kSolveGroup * a.ldJ + (size_t)NW * kSolveGroup * a.nmax);
    const size_t stat = sizeof(double) * kSolveGroup * kMaxBox + 2 * sizeof(int) * kMaxBox + 1024;
    note_shape("solve_bwd_" + std::to_string(NTH) + (sizeof(TT) == 4 ? "_f32" : "_f64") + (nrhs > 1 ? "_multi" : ""));
    if (nrhs == 1 || ldsg + stat > (size_t)elim_lds_limit()) {
        solve_bwd_k<TT, NTH, 1>(a, boxes, nboxes, z, nrhs, ld, lds1, s);
        return;
    }
    for (int h0 = 0; h0 < nrhs; h0 += kSolveGroup)
        solve_bwd_k<TT, NTH, kSolveGroup>(a, boxes, nboxes, z + (int64_t)h0 * ld, std::min(kSolveGroup, nrhs - h0),
                                          ld, ldsg, s);
}

void launch_solve_fwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld, int use32,
                      hipStream_t s) {
    if (nboxes <= 0) return;
    SweepArgs a = sweep_args(L, use32);
    // few boxes: a large workgroup per box keeps more loads of the record in flight
    if (plan_params(nboxes).sweep_threads == 1024) {
        if (use32) solve_fwd_t<float, 1024>(a, boxes, nboxes, z, nrhs, ld, s);
        else solve_fwd_t<double, 1024>(a, boxes, nboxes, z, nrhs, ld, s);
    } else {
        if (use32) solve_fwd_t<float, 256>(a, boxes, nboxes, z, nrhs, ld, s);
        else solve_fwd_t<double, 256>(a, boxes, nboxes, z, nrhs, ld, s);
    }
}

void launch_solve_bwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld, int use32,
                      hipStream_t s) {
    if (nboxes <= 0) return;
    SweepArgs a = sweep_args(L, use32);
    if (plan_params(nboxes).sweep_threads == 1024) {
        if (use32) solve_bwd_t<float, 1024>(a, boxes, nboxes, z, nrhs, ld, s);
        else solve_bwd_t<double, 1024>(a, boxes, nboxes, z, nrhs, ld, s);
    } else {
        if (use32) solve_bwd_t<float, 256>(a, boxes, nboxes, z, nrhs, ld, s);
        else solve_bwd_t<double, 256>(a, boxes, nboxes, z, nrhs, ld, s);
    }
}

void launch_apply_fwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      const double* Lroot, hipStream_t s) {
    if (nboxes <= 0) return;
    const size_t lds = sizeof(double) * (size_t)L.ldJ;
    SweepArgs a = sweep_args(L, 0);
    a.Lc = Lroot;
    if (plan_params(nboxes).sweep_threads == 1024) k_apply_fwd<1024><<<dim3(nboxes), dim3(1024), lds, s>>>(a, boxes, z, nrhs, ld);
    else k_apply_fwd<256><<<dim3(nboxes), dim3(256), lds, s>>>(a, boxes, z, nrhs, ld);
}

void launch_apply_bwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      const double* Lroot, hipStream_t s) {
    if (nboxes <= 0) return;
    SweepArgs a = sweep_args(L, 0);
    a.Lc = Lroot;
    if (plan_params(nboxes).sweep_threads == 1024) k_apply_bwd<1024><<<dim3(nboxes), dim3(1024), 0, s>>>(a, boxes, z, nrhs, ld);
    else k_apply_bwd<256><<<dim3(nboxes), dim3(256), 0, s>>>(a, boxes, z, nrhs, ld);
}

// ---- generalized square root (Section 3.3): Cholesky factors of the blocks of D --------

// In-place lower Cholesky factor of the n x n block at L (column-major, leading dimension
// ld; only the lower triangle is read), right-looking, one column per step.  Every thread
// of the workgroup calls it; a pivot that is not positive (or NaN) sets bit 16 of *flag and
// ends the factorization (the same decision on every thread).
template <int NTH>
__device__ void chol_inplace(double* L, int n, int64_t ld, int* flag) {
    const int tid = threadIdx.x;
    for (int j = 0; j < n; ++j) {
        __syncthreads();
        const double d = L[j + ld * j];
        if (!(d > 0.0)) {
            if (tid == 0) atomicOr(flag, 16);
            return;
        }
        const double sd = sqrt(d), inv = 1.0 / sd;
        for (int i = j + 1 + tid; i < n; i += NTH) L[i + ld * j] *= inv;
        __syncthreads();
        if (tid == 0) L[j + ld * j] = sd;
        const int m = n - j - 1;
        for (int e = tid; e < m * m; e += NTH) {
            const int ii = e % m, ll = e / m;
            if (ii >= ll) {
                const int i = j + 1 + ii, l = j + 1 + ll;
                L[i + ld * l] -= L[i + ld * j] * L[l + ld * j];
            }
        }
    }
    __syncthreads();
}

// One workgroup per record: L.Lc of the box <- lower Cholesky factor of X_RR (upper
// triangle zero).
__global__ void __launch_bounds__(256) k_chol_records(const int* __restrict__ boxes, const int* __restrict__ cnt,
                                                      const int* __restrict__ krank, const int* __restrict__ nJ,
                                                      const double* __restrict__ XRR, double* Lc, int nmax,
                                                      int* flag) {
    const int c = boxes[blockIdx.x];
    if (nJ[c] == 0) return;
    const int r = cnt[c] - krank[c];
    const int64_t bsz = (int64_t)nmax * nmax;
    const double* X = XRR + c * bsz;
    double* L = Lc + c * bsz;
    for (int e = threadIdx.x; e < r * r; e += 256) {
        const int i = e % r, j = e / r;
        L[i + (int64_t)nmax * j] = i >= j ? X[i + (int64_t)nmax * j] : 0.0;
    }
    chol_inplace<256>(L, r, nmax, flag);
}

// One workgroup: Lt <- lower Cholesky factor of the dense top block A, LT <- its transpose.
__global__ void __launch_bounds__(1024) k_chol_top(const double* __restrict__ A, int n, double* Lt, double* LT,
                                                   int* flag) {
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += 1024) {
        const int i = (int)(e % n), j = (int)(e / n);
        Lt[e] = i >= j ? A[e] : 0.0;
    }
    chol_inplace<1024>(Lt, n, n, flag);
    if (*flag & 16) return;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += 1024) {
        const int i = (int)(e % n), j = (int)(e / n);
        LT[(int64_t)j + (int64_t)n * i] = Lt[e];
    }
}

void launch_chol_records(const Level& L, const int* boxes, int nboxes, int* flag, hipStream_t s) {
    if (nboxes <= 0) return;
    k_chol_records<<<dim3(nboxes), dim3(256), 0, s>>>(boxes, L.cnt, L.krank, L.nJ, L.XRR, L.Lc, L.nmax, flag);
}

void launch_chol_top(const double* A, int64_t n, double* Lt, double* LT, int* flag, hipStream_t s) {
    if (n <= 0) return;
    k_chol_top<<<dim3(1), dim3(1024), 0, s>>>(A, (int)n, Lt, LT, flag);
}

// ---- top block ------------------------------------------------------------------------
__global__ void k_gather_top(const int* __restrict__ idx, int64_t ntop, const double* __restrict__ z, int nrhs,
                             int64_t ld, double* __restrict__ tmp) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntop * nrhs) return;
    int64_t i = e % ntop, h = e / ntop;
    tmp[e] = z[h * ld + idx[i]];
}

// z[idx[i]] = sum_j M[i][j] tmp[j]: 64 rows per workgroup, one lane per row, the four
// waves take quarters of j and add their partial sums in LDS.
template <typename TT>
__global__ void __launch_bounds__(256) k_top_gemv(const int* __restrict__ idx, int64_t ntop, const TT* __restrict__ M,
                                                  const double* __restrict__ tmp, int nrhs, double* __restrict__ z,
                                                  int64_t ld) {
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const int h = blockIdx.y;
    const double* x = tmp + (int64_t)h * ntop;
    const int64_t q4 = (ntop + 3) / 4;
    const int64_t j0 = wv * q4, j1 = j0 + q4 < ntop ? j0 + q4 : ntop;
    double s = 0.0;
    if (i < ntop && j1 > j0) s = dot_strided(M + i + j0 * ntop, ntop, x + j0, (int)(j1 - j0));
    part[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && i < ntop) z[(int64_t)h * ld + idx[i]] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

void launch_top_apply(const int* top_idx, int64_t ntop, const double* M, const float* M32, double* z, int nrhs,
                      int64_t ld, double* tmp, hipStream_t s) {
    if (ntop <= 0) return;
    int64_t tot = ntop * nrhs;
    k_gather_top<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(top_idx, ntop, z, nrhs, ld, tmp);
    dim3 grid((unsigned)((ntop + 63) / 64), nrhs);
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

// Dense LU with partial pivoting of the top block, blocked right-looking (panels of
// kNB columns): the panel is factored by one workgroup (in LDS when it fits), then the
// row interchanges, the triangular solve for U12 and the trailing update A22 -= L21 U12
// run over many workgroups.  Pivots: largest magnitude, lowest row on ties.  The
// explicit inverse follows by blocked triangular solves against identity columns.
constexpr int kNB = 32;
constexpr int kPanelTall = 4096;   // panel rows from which the panel takes the wide-row form

// Panel [k0, k0 + nb): ipiv[k0 + j] = global pivot row of step j.  Also publishes the
// net row permutation of the panel's interchanges restricted to the rows it moves:
// sw[0] = count, then pairs (row, source row) meaning new A[row, :] = old A[source, :].
template <bool INLDS, bool TALL>
__global__ void __launch_bounds__(1024) k_lu_panel(double* __restrict__ A, int n, int k0, int* __restrict__ ipiv,
                                                   int* __restrict__ sw, int* flag, double* logdet, int* sign) {
    extern __shared__ double pl[];
    __shared__ int piv_idx;
    __shared__ double piv_val;
    __shared__ int sp[kNB];
    __shared__ int cnt;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    if (*flag & 8) return;
    const int m = n - k0, nb = min(kNB, m);
    const int ld = INLDS ? m : n;
    double* P = INLDS ? pl : A + k0 + (int64_t)k0 * n;
    if (INLDS) {
        for (int e = tid; e < m * nb; e += 1024) {
            int i = e % m, j = e / m;
            P[e] = A[(k0 + i) + (int64_t)(k0 + j) * n];
        }
        __syncthreads();
    }
    __shared__ double wbest[16], rowj[kNB];
    __shared__ int wbi[16];
    // TALL (panels of kPanelTall rows or more): the pivot search over all 16 waves and one
    // row per thread in the update; otherwise one wave searches and each wave updates whole
    // columns (fewer steps per thread).  Same pivots and the same operations either way.
    constexpr bool tall = TALL;
    double lsum = 0.0;
    int sgn = 1;
    if constexpr (INLDS) {
        // Panel in LDS: two barriers per column.  Wave 0 updates column j + 1 and finds its
        // pivot while doing so; the multipliers of column j are formed on the fly in the
        // update and stored scaled in the next step, beside the row interchange.  Same
        // pivots and the same operations as the steps below.
        if (wv == 0) {
            double best = -1.0;
            int bi = m;
            for (int i = lane; i < m; i += 64) {
                double v = fabs(P[i]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            wave_argmax(best, bi);
            if (lane == 0) { piv_idx = bi; piv_val = best; }
        }
        __syncthreads();
        double rprev = 0.0;   // 1 / pivot of column j - 1
        for (int j = 0; j < nb; ++j) {
            const int p = piv_idx;
            if (!(piv_val > 0.0) || p >= m) {
                if (tid == 0) atomicOr(flag, 8);
                return;
            }
            if (tid == 0) { ipiv[k0 + j] = k0 + p; sp[j] = p; }
            // column j - 1's multipliers below row j - 1; rows j and p go with the interchange
            if (j > 0)
                for (int i = j + tid; i < m; i += 1024)
                    if (i != j && i != p) P[i + (int64_t)(j - 1) * ld] *= rprev;
            if (p != j) {
                for (int l = tid; l < nb; l += 1024) {
                    double a = P[j + (int64_t)l * ld], b = P[p + (int64_t)l * ld];
                    if (l == j - 1) { a *= rprev; b *= rprev; }
                    P[j + (int64_t)l * ld] = b;
                    P[p + (int64_t)l * ld] = a;
                }
                sgn = -sgn;
            } else if (j > 0 && tid == 0) {
                P[j + (int64_t)(j - 1) * ld] *= rprev;
            }
            __syncthreads();
            const double d = P[j + (int64_t)j * ld];
            if (wv == 15) lsum += log(fabs(d));   // off wave 0's pivot chain
            if (d < 0) sgn = -sgn;
            const double rinv = 1.0 / d;
            double best = -1.0;
            int bi = m;
            for (int l = j + 1 + wv; l < nb; l += 16) {
                const double ajl = P[j + (int64_t)l * ld];
                for (int i = j + 1 + lane; i < m; i += 64) {
                    const double mult = P[i + (int64_t)j * ld] * rinv;
                    const double v = P[i + (int64_t)l * ld] - mult * ajl;
                    P[i + (int64_t)l * ld] = v;
                    if (l == j + 1) {
                        const double a = fabs(v);
                        if (a > best || (a == best && i < bi)) { best = a; bi = i; }
                    }
                }
            }
            if (wv == 0 && j + 1 < nb) {
                wave_argmax(best, bi);
                if (lane == 0) { piv_idx = bi; piv_val = best; }
            }
            rprev = rinv;
            __syncthreads();
        }
        for (int i = nb + tid; i < m; i += 1024) P[i + (int64_t)(nb - 1) * ld] *= rprev;
        __syncthreads();
    } else
    for (int j = 0; j < nb; ++j) {
        if constexpr (tall) {
            // largest magnitude, lowest row on ties: per wave, then across the waves
            double best = -1.0;
            int bi = m;
            for (int i = j + tid; i < m; i += 1024) {
                double v = fabs(P[i + (int64_t)j * ld]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            wave_argmax(best, bi);
            if (lane == 0) { wbest[wv] = best; wbi[wv] = bi; }
            __syncthreads();
            if (tid == 0) {
                best = wbest[0];
                bi = wbi[0];
                for (int w = 1; w < 16; ++w)
                    if (wbest[w] > best || (wbest[w] == best && wbi[w] < bi)) { best = wbest[w]; bi = wbi[w]; }
                piv_idx = bi;
                piv_val = best;
            }
        } else if (wv == 0) {
            double best = -1.0;
            int bi = m;
            for (int i = j + lane; i < m; i += 64) {
                double v = fabs(P[i + (int64_t)j * ld]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            wave_argmax(best, bi);
            if (lane == 0) { piv_idx = bi; piv_val = best; }
        }
        __syncthreads();
        const int p = piv_idx;
        if (!(piv_val > 0.0) || p >= m) {
            if (tid == 0) atomicOr(flag, 8);
            return;
        }
        if (tid == 0) { ipiv[k0 + j] = k0 + p; sp[j] = p; }
        if (p != j) {
            for (int l = tid; l < nb; l += 1024) {
                double t0 = P[j + (int64_t)l * ld];
                P[j + (int64_t)l * ld] = P[p + (int64_t)l * ld];
                P[p + (int64_t)l * ld] = t0;
            }
            sgn = -sgn;
        }
        __syncthreads();
        const double d = P[j + (int64_t)j * ld];
        lsum += log(fabs(d));
        if (d < 0) sgn = -sgn;
        const double rinv = 1.0 / d;
        if constexpr (!tall) {
            for (int i = j + 1 + tid; i < m; i += 1024) P[i + (int64_t)j * ld] *= rinv;
            __syncthreads();
            for (int l = j + 1 + wv; l < nb; l += 16) {
                const double ajl = P[j + (int64_t)l * ld];
                for (int i = j + 1 + lane; i < m; i += 64) P[i + (int64_t)l * ld] -= P[i + (int64_t)j * ld] * ajl;
            }
            __syncthreads();
            continue;
        }
        if (tid < nb) rowj[tid] = P[j + (int64_t)tid * ld];
        __syncthreads();
        // one row per thread: the multiplier, then the row's update right of column j, eight
        // of the row's entries loaded together at a time
        for (int i = j + 1 + tid; i < m; i += 1024) {
            double* Pi = P + i;
            const double mult = Pi[(int64_t)j * ld] * rinv;
            Pi[(int64_t)j * ld] = mult;
#pragma unroll
            for (int l0 = 0; l0 < kNB; l0 += 8) {
                if (l0 + 7 <= j || l0 >= nb) continue;
                double* col = Pi + (int64_t)l0 * ld;
                double r[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) r[q] = (l0 + q > j && l0 + q < nb) ? col[(int64_t)q * ld] : 0.0;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (l0 + q > j && l0 + q < nb) col[(int64_t)q * ld] = r[q] - mult * rowj[l0 + q];
            }
        }
        __syncthreads();
    }
    if (INLDS) {
        for (int e = tid; e < m * nb; e += 1024) {
            int i = e % m, j = e / m;
            A[(k0 + i) + (int64_t)(k0 + j) * n] = P[e];
        }
    }
    if (tid == (INLDS ? 1023 : 0)) {   // a thread that summed the logarithms
        *logdet = (k0 == 0 ? 0.0 : *logdet) + lsum;
        *sign = (k0 == 0 ? 1 : *sign) * sgn;
    }
    if (tid == 0) cnt = 0;
    __syncthreads();
    // net permutation: candidate rows are the panel rows and the pivot rows below it
    if (wv == 0) {
        int r = -1;
        if (lane < nb) {
            r = lane;
        } else if (lane < 2 * nb) {
            int q = sp[lane - nb];
            bool dup = q < nb;
            for (int i = 0; i < lane - nb && !dup; ++i) dup = sp[i] == q;
            if (!dup) r = q;
        }
        int src = r;
        if (r >= 0)
            for (int j = nb - 1; j >= 0; --j) {
                if (src == j) src = sp[j];
                else if (src == sp[j]) src = j;
            }
        const bool moved = r >= 0 && src != r;
        const unsigned long long mask = __ballot(moved);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (moved) {
            sw[1 + 2 * before] = k0 + r;
            sw[2 + 2 * before] = k0 + src;
        }
        if (lane == 0) sw[0] = __popcll(mask);
    }
}

// Row interchanges of panel k0 on every column block outside the panel, then
// U12 = L11^{-1} A12 for the blocks right of it.  One workgroup per kNB columns.
__global__ void __launch_bounds__(256) k_lu_swap_trsm(double* __restrict__ A, int n, int k0,
                                                      const int* __restrict__ sw, const int* flag) {
    __shared__ double vs[2 * kNB * kNB];
    __shared__ double Ls[kNB * kNB];
    __shared__ double Xs[kNB * kNB];
    const int tid = threadIdx.x;
    if (*flag & 8) return;
    const int c0 = blockIdx.x * kNB;
    if (c0 == k0) return;                      // the panel swapped its own rows
    const int nc = min(kNB, n - c0);
    const int ns = sw[0];
    for (int e = tid; e < ns * nc; e += 256) {
        int q = e % ns, c = e / ns;
        vs[q + 2 * kNB * c] = A[sw[2 + 2 * q] + (int64_t)(c0 + c) * n];
    }
    __syncthreads();
    for (int e = tid; e < ns * nc; e += 256) {
        int q = e % ns, c = e / ns;
        A[sw[1 + 2 * q] + (int64_t)(c0 + c) * n] = vs[q + 2 * kNB * c];
    }
    if (c0 < k0) return;
    __syncthreads();
    const int nb = min(kNB, n - k0);
    for (int e = tid; e < nb * nb; e += 256) {
        int i = e % nb, j = e / nb;
        Ls[e] = A[(k0 + i) + (int64_t)(k0 + j) * n];
    }
    for (int e = tid; e < nb * nc; e += 256) {
        int i = e % nb, c = e / nb;
        Xs[e] = A[(k0 + i) + (int64_t)(c0 + c) * n];
    }
    __syncthreads();
    for (int j = 0; j < nb - 1; ++j) {
        for (int e = tid; e < (nb - 1 - j) * nc; e += 256) {
            int i = j + 1 + e % (nb - 1 - j), c = e / (nb - 1 - j);
            Xs[i + nb * c] -= Ls[i + nb * j] * Xs[j + nb * c];
        }
        __syncthreads();
    }
    for (int e = tid; e < nb * nc; e += 256) {
        int i = e % nb, c = e / nb;
        A[(k0 + i) + (int64_t)(c0 + c) * n] = Xs[e];
    }
}

// A22 -= L21 U12 for rows and columns >= k0 + nb, 64 x 64 tiles, 4 x 4 per thread.
__global__ void __launch_bounds__(256) k_lu_gemm(double* __restrict__ A, int n, int k0, const int* flag) {
    __shared__ double Ls[64 * kNB];
    __shared__ double Us[(kNB + 1) * 64];
    const int tid = threadIdx.x;
    if (*flag & 8) return;
    const int nb = min(kNB, n - k0);
    const int s0 = k0 + nb;
    const int r0 = s0 + blockIdx.y * 64, c0 = s0 + blockIdx.x * 64;
    const int nr = min(64, n - r0), nc = min(64, n - c0);
    for (int e = tid; e < 64 * nb; e += 256) {
        int i = e % 64, q = e / 64;
        Ls[e] = i < nr ? A[(r0 + i) + (int64_t)(k0 + q) * n] : 0.0;
    }
    for (int e = tid; e < nb * 64; e += 256) {
        int q = e % nb, c = e / nb;
        Us[q + (kNB + 1) * c] = c < nc ? A[(k0 + q) + (int64_t)(c0 + c) * n] : 0.0;
    }
    __syncthreads();
    const int ti = tid % 16, tc = tid / 16;
    double acc[4][4] = {};
    for (int q = 0; q < nb; ++q) {
        double a[4], b[4];
        for (int u = 0; u < 4; ++u) a[u] = Ls[(ti + 16 * u) + 64 * q];
        for (int v = 0; v < 4; ++v) b[v] = Us[q + (kNB + 1) * (tc + 16 * v)];
        for (int u = 0; u < 4; ++u)
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            int i = ti + 16 * u, c = tc + 16 * v;
            if (i < nr && c < nc) A[(r0 + i) + (int64_t)(c0 + c) * n] -= acc[u][v];
        }
}

// perm[i] = source row of row i of P A, from the sequence of interchanges ipiv.
__global__ void k_lu_perm(const int* __restrict__ ipiv, int n, int* __restrict__ perm, const int* flag, int in_lds) {
    extern __shared__ int pm[];
    if (threadIdx.x != 0 || (*flag & 8)) return;
    int* w = in_lds ? pm : perm;
    for (int i = 0; i < n; ++i) w[i] = i;
    for (int j = 0; j < n; ++j) {
        int p = ipiv[j];
        int t0 = w[j]; w[j] = w[p]; w[p] = t0;
    }
    if (in_lds)
        for (int i = 0; i < n; ++i) perm[i] = w[i];
}

// Columns [c0, c0 + NC) of A^{-1} = U^{-1} L^{-1} P: X = P e_c in LDS, then blocked
// forward and backward substitution (a kNB x kNB diagonal block in LDS, then one
// rectangular update per block).
// Inverses of the kNB x kNB diagonal blocks of the LU factors: block b < nblk of the unit
// lower L, block nblk + b of U.  One thread per column of the block, by substitution.
// Dinv[(which * nblk + b) * kNB * kNB + i + kNB c].
__global__ void __launch_bounds__(kNB) k_tri_diag_inv(const double* __restrict__ LU, int n, int nblk,
                                                       double* __restrict__ Dinv, const int* flag) {
    __shared__ double D[kNB * kNB];
    __shared__ double X[kNB * kNB];   // X[i * kNB + c]: row i of column c of the inverse
    if (*flag & 8) return;
    const int upper = blockIdx.x >= nblk;
    const int b = blockIdx.x - (upper ? nblk : 0);
    const int jb = b * kNB, bs = min(kNB, n - jb);
    const int c = threadIdx.x;
    for (int e = c; e < bs * bs; e += kNB) D[e] = LU[(jb + e % bs) + (int64_t)(jb + e / bs) * n];
    __syncthreads();
    double* out = Dinv + (int64_t)(upper * nblk + b) * kNB * kNB;
    if (c >= bs) return;
    if (!upper) {
        for (int i = 0; i < bs; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int j = c; j < i; ++j) v -= D[i + bs * j] * X[j * kNB + c];
            X[i * kNB + c] = v;
        }
    } else {
        for (int i = bs - 1; i >= 0; --i) {
            double v = i == c ? 1.0 : 0.0;
            for (int j = i + 1; j <= c; ++j) v -= D[i + bs * j] * X[j * kNB + c];
            X[i * kNB + c] = v / D[i + bs * i];
        }
    }
    for (int i = 0; i < bs; ++i) out[i + kNB * c] = X[i * kNB + c];
}

template <int NC>
__global__ void __launch_bounds__(256) k_top_inverse_blk(const double* __restrict__ LU, const int* __restrict__ perm,
                                                         int n, double* __restrict__ Ainv, const double* __restrict__ Dinv,
                                                         const int* flag) {
    extern __shared__ double xs[];   // n x NC, xs[i * NC + c]
    __shared__ double D[kNB * kNB];
    __shared__ double yt[kNB * NC];
    const int nblk = (n + kNB - 1) / kNB;
    const int tid = threadIdx.x;
    if (*flag & 8) return;
    const int c0 = blockIdx.x * NC;
    for (int e = tid; e < n * NC; e += 256) {
        int i = e / NC, c = e % NC;
        xs[e] = (perm[i] == c0 + c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // x_blk <- (inverse of the diagonal block) x_blk, lower or upper triangular
    auto diag_apply = [&](int jb, int bs, bool lower) {
        for (int e = tid; e < bs * NC; e += 256) {
            const int i = e / NC, c = e % NC;
            double v = 0.0;
            if (lower) for (int j = 0; j <= i; ++j) v += D[i + kNB * j] * xs[(jb + j) * NC + c];
            else for (int j = i; j < bs; ++j) v += D[i + kNB * j] * xs[(jb + j) * NC + c];
            yt[e] = v;
        }
        __syncthreads();
        for (int e = tid; e < bs * NC; e += 256) xs[(jb + e / NC) * NC + e % NC] = yt[e];
        __syncthreads();
    };
    // rows i0 <= i < i1: x_i -= LU(i, jb .. jb + bs) x_blk for all NC columns; a thread takes
    // a row, with the bs entries of LU loaded at once (one read of L2 per row and block)
    auto offdiag = [&](int i0, int i1, int jb, int bs) {
        for (int i = i0 + tid; i < i1; i += 256) {
            double l[kNB];
#pragma unroll
            for (int j = 0; j < kNB; ++j) l[j] = j < bs ? LU[i + (int64_t)(jb + j) * n] : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < kNB; ++j) v += l[j] * xs[min(jb + j, n - 1) * NC + c];
                xs[i * NC + c] -= v;
            }
        }
    };
    for (int jb = 0; jb < n; jb += kNB) {            // L y = P e (unit lower)
        const int bs = min(kNB, n - jb);
        const double* Di = Dinv + (int64_t)(jb / kNB) * kNB * kNB;
        for (int e = tid; e < kNB * kNB; e += 256) D[e] = Di[e];
        __syncthreads();
        diag_apply(jb, bs, true);
        offdiag(jb + bs, n, jb, bs);
        __syncthreads();
    }
    for (int b = nblk - 1; b >= 0; --b) {            // U x = y
        const int jb = b * kNB, bs = min(kNB, n - jb);
        const double* Di = Dinv + (int64_t)(nblk + b) * kNB * kNB;
        for (int e = tid; e < kNB * kNB; e += 256) D[e] = Di[e];
        __syncthreads();
        diag_apply(jb, bs, false);
        offdiag(0, jb, jb, bs);
        __syncthreads();
    }
    for (int e = tid; e < n * NC; e += 256) {
        int i = e % n, c = e / n;
        if (c0 + c < n) Ainv[(int64_t)(c0 + c) * n + i] = xs[i * NC + c];
    }
}

// The same solves for n beyond what an LDS column block holds: NC columns per workgroup,
// kept in their own output columns of Ainv (global memory), the solved rows of the current
// diagonal block staged in LDS.  Each workgroup reads the LU factors once for its NC
// columns (the one-column form read them once per column).  Same operations in the same
// order as k_top_inverse_blk.
template <int NC>
__global__ void __launch_bounds__(256) k_top_inverse_glb(const double* __restrict__ LU, const int* __restrict__ perm,
                                                         int n, double* __restrict__ Ainv, const double* __restrict__ Dinv,
                                                         const int* flag) {
    __shared__ double D[kNB * kNB];
    __shared__ double xb[kNB * NC];   // xb[i * NC + c]: row jb + i of the current block
    const int nblk = (n + kNB - 1) / kNB;
    const int tid = threadIdx.x;
    if (*flag & 8) return;
    const int c0 = blockIdx.x * NC;
    const int nc = min(NC, n - c0);
    double* X = Ainv + (int64_t)c0 * n;   // X[i + n c], c < nc
    for (int64_t e = tid; e < (int64_t)n * nc; e += 256) {
        const int i = (int)(e % n), c = (int)(e / n);
        X[e] = (perm[i] == c0 + c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // x_blk <- (inverse of the diagonal block) x_blk; xb keeps the result (zero beyond bs)
    auto diag_apply = [&](int jb, int bs, bool lower) {
        for (int e = tid; e < kNB * NC; e += 256) {
            const int i = e / NC, c = e % NC;
            double v = 0.0;
            if (i < bs && c < nc) {
                const double* x = X + (int64_t)n * c + jb;
                if (lower) for (int j = 0; j <= i; ++j) v += D[i + kNB * j] * x[j];
                else for (int j = i; j < bs; ++j) v += D[i + kNB * j] * x[j];
            }
            xb[e] = v;
        }
        __syncthreads();
        for (int e = tid; e < bs * NC; e += 256) {
            const int i = e / NC, c = e % NC;
            if (c < nc) X[(int64_t)n * c + jb + i] = xb[e];
        }
        __syncthreads();
    };
    auto offdiag = [&](int i0, int i1, int jb, int bs) {
        for (int i = i0 + tid; i < i1; i += 256) {
            double l[kNB];
#pragma unroll
            for (int j = 0; j < kNB; ++j) l[j] = j < bs ? LU[i + (int64_t)(jb + j) * n] : 0.0;
            for (int c = 0; c < nc; ++c) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < kNB; ++j) v += l[j] * xb[j * NC + c];
                X[(int64_t)n * c + i] -= v;
            }
        }
    };
    for (int jb = 0; jb < n; jb += kNB) {            // L y = P e (unit lower)
        const int bs = min(kNB, n - jb);
        const double* Di = Dinv + (int64_t)(jb / kNB) * kNB * kNB;
        for (int e = tid; e < kNB * kNB; e += 256) D[e] = Di[e];
        __syncthreads();
        diag_apply(jb, bs, true);
        offdiag(jb + bs, n, jb, bs);
        __syncthreads();
    }
    for (int b = nblk - 1; b >= 0; --b) {            // U x = y
        const int jb = b * kNB, bs = min(kNB, n - jb);
        const double* Di = Dinv + (int64_t)(nblk + b) * kNB * kNB;
        for (int e = tid; e < kNB * kNB; e += 256) D[e] = Di[e];
        __syncthreads();
        diag_apply(jb, bs, false);
        offdiag(0, jb, jb, bs);
        __syncthreads();
    }
}

int64_t lu_piv_ints(int64_t n) { return 2 * n + 4 * kNB + 1; }
int64_t lu_work_doubles(int64_t n) { return 2 * ((n + kNB - 1) / kNB) * kNB * kNB; }

void launch_lu_inverse(double* A, double* Ainv, int64_t n64, int* piv, double* work, int* flag, double* logdet,
                       int* sign, hipStream_t s) {
    if (n64 <= 0) return;
    const int n = (int)n64;
    int* ipiv = piv;
    int* perm = piv + n;
    int* sw = piv + 2 * n;
    const int lim = elim_lds_limit();
    const int nblk = (n + kNB - 1) / kNB;
    for (int k0 = 0; k0 < n; k0 += kNB) {
        const int m = n - k0, nb = std::min(kNB, m);
        const size_t pl = sizeof(double) * (size_t)m * nb;
        if ((long)pl + 1024 <= lim)
            k_lu_panel<true, false><<<dim3(1), dim3(1024), pl, s>>>(A, n, k0, ipiv, sw, flag, logdet, sign);
        else if (m >= kPanelTall)
            k_lu_panel<false, true><<<dim3(1), dim3(1024), 0, s>>>(A, n, k0, ipiv, sw, flag, logdet, sign);
        else
            k_lu_panel<false, false><<<dim3(1), dim3(1024), 0, s>>>(A, n, k0, ipiv, sw, flag, logdet, sign);
        if (nblk > 1) k_lu_swap_trsm<<<dim3(nblk), dim3(256), 0, s>>>(A, n, k0, sw, flag);
        const int rest = n - k0 - nb;
        if (rest > 0) {
            const unsigned g = (unsigned)((rest + 63) / 64);
            k_lu_gemm<<<dim3(g, g), dim3(256), 0, s>>>(A, n, k0, flag);
        }
    }
    const bool pl = (size_t)n * sizeof(int) + 1024 <= (size_t)lim;
    k_lu_perm<<<dim3(1), dim3(64), pl ? sizeof(int) * (size_t)n : 0, s>>>(ipiv, n, perm, flag, pl ? 1 : 0);
    k_tri_diag_inv<<<dim3(2 * nblk), dim3(kNB), 0, s>>>(A, n, nblk, work, flag);
    constexpr int NC = 8;
    const size_t lds = sizeof(double) * (size_t)n * NC;
    if ((long)lds + (long)sizeof(double) * kNB * (kNB + NC) + 1024 > lim) {
        // n beyond what one LDS column block holds (about 2000 DOFs)
        // columns per workgroup: as many as keep at least 256 workgroups (one per CU)
        if (n >= 256 * 32)
            k_top_inverse_glb<32><<<dim3((unsigned)((n + 31) / 32)), dim3(256), 0, s>>>(A, perm, n, Ainv,
                                                                                        (const double*)work, flag);
        else if (n >= 256 * 16)
            k_top_inverse_glb<16><<<dim3((unsigned)((n + 15) / 16)), dim3(256), 0, s>>>(A, perm, n, Ainv,
                                                                                        (const double*)work, flag);
        else
            k_top_inverse_glb<8><<<dim3((unsigned)((n + 7) / 8)), dim3(256), 0, s>>>(A, perm, n, Ainv,
                                                                                      (const double*)work, flag);
    } else {
        k_top_inverse_blk<NC><<<dim3((unsigned)((n + NC - 1) / NC)), dim3(256), lds, s>>>(A, perm, n, Ainv,
                                                                                          (const double*)work, flag);
    }
}

}  // namespace rss
