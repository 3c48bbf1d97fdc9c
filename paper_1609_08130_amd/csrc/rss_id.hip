// Interpolative decomposition of one box per wavefront (Section 2.2, Definition 1;
// Section 3.2, eq. smallid).
//
// The ID input of box c is M = [A(O, B_c); w K(Gamma, B_c)]: the current blocks of the
// active DOFs of the boxes at Chebyshev distance 2 (the boxes inside the proxy circle)
// stacked over the kernel evaluated at n_p proxy points on the circle Gamma of radius
// proxy_radius * side around the box centre.
//
// Greedy column-pivoted Householder QR of M is mathematically determined by M^T M, so
// it is carried out on the triangular factor R0 of an unpivoted QR of M instead:
//   1. TSQR: rows of M are streamed in chunks of BR rows; each chunk is annihilated
//      into R0 by n structured Householder reflectors acting on [R0; chunk].
//   2. Pivoted QR of R0 with trailing column norms recomputed at every step; the pivot
//      is the lowest B-position among columns whose norm is within tau * |R_00| of the
//      largest; stop at step j > 0 once the largest norm is <= tol * |R_00|.
//   3. T = R11^{-1} R12 by back substitution, re-indexed to ascending skeleton /
//      redundant positions.
// Lane q owns column q (and q + 64, ... for CPT > 1), so every column of R0 is private
// to one lane except for the broadcast of the current reflector through LDS.
#include "rss_internal.h"

namespace rss {

__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_min_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

template <int CPT, int BR, bool RLDS>
__global__ void __launch_bounds__(64) k_id(const double* __restrict__ store, int nb, int nmax,
                                           const int* __restrict__ cnt, const int* __restrict__ gidx,
                                           const int* __restrict__ nact, const int* __restrict__ apos,
                                           const int* __restrict__ boxes, const double* __restrict__ pts,
                                           const double* __restrict__ ptmpl, KernelParams kp, int t,
                                           int* __restrict__ krank, int* __restrict__ spos,
                                           int* __restrict__ rpos, double* __restrict__ Tout,
                                           int* __restrict__ mrows, double* __restrict__ work) {
    constexpr int NP = 64 * CPT;
    extern __shared__ double R0s[];   // RLDS: nmax x NP
    __shared__ double vbuf[NP > BR ? NP : BR];
    __shared__ double taubuf;
    __shared__ const double* obase[16];
    __shared__ const int* oap[16];
    __shared__ int obeg[17];
    __shared__ int nO;
    __shared__ const double* rowptr[BR];
    __shared__ int rowprox[BR];
    __shared__ double pxs[kMaxProxy], pys[kMaxProxy];
    __shared__ int piv[NP];
    __shared__ int srank_s[NP];
    __shared__ int pivsel;

    const int lane = threadIdx.x;
    const int c = boxes[blockIdx.x];
    const int n = cnt[c];
    double* R0 = RLDS ? R0s : (work + (int64_t)blockIdx.x * NP * NP);
    if (n == 0) {
        if (lane == 0) { krank[c] = 0; mrows[c] = 0; }
        return;
    }
    const int cx = c % nb, cy = c / nb;
    const int64_t bsz = (int64_t)nmax * nmax;

    // O ring: boxes at distance exactly 2, ascending linear index.
    if (lane == 0) {
        int cntO = 0;
        obeg[0] = 0;
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                if (max(abs(dx), abs(dy)) != 2) continue;
                int ox = cx + dx, oy = cy + dy;
                if (ox < 0 || oy < 0 || ox >= nb || oy >= nb) continue;
                int o = ox + nb * oy;
                obase[cntO] = store + ((int64_t)o * kNbr + nbr_slot(-dx, -dy)) * bsz;   // block (o, c)
                oap[cntO] = apos + (int64_t)o * nmax;
                obeg[cntO + 1] = obeg[cntO] + nact[o];
                ++cntO;
            }
        nO = cntO;
    }
    // proxy points y_p = centre + radius * (cos, sin)(2 pi p / n_p)
    {
#pragma clang fp contract(off)
        double side_t = kp.side / (double)(1 << t);
        double ccx = kp.lo_x + ((double)cx + 0.5) * side_t;
        double ccy = kp.lo_y + ((double)cy + 0.5) * side_t;
        double rr = kp.proxy_radius * side_t;
        for (int p = lane; p < kp.n_proxy; p += 64) {
            pxs[p] = ccx + rr * ptmpl[2 * p];
            pys[p] = ccy + rr * ptmpl[2 * p + 1];
        }
    }
    double colx[CPT], coly[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
        int q = lane + 64 * cc;
        colx[cc] = 0.0; coly[cc] = 0.0;
        if (q < n) {
            int g = gidx[(int64_t)c * nmax + q];
            colx[cc] = pts[2 * (int64_t)g];
            coly[cc] = pts[2 * (int64_t)g + 1];
        }
    }
    for (int i = 0; i < n; ++i) {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) R0[i * NP + lane + 64 * cc] = 0.0;
    }
    __syncthreads();
    const int mO = obeg[nO];
    const int m = mO + kp.n_proxy;

    // ---- 1. TSQR ----------------------------------------------------------------
    for (int r0 = 0; r0 < m; r0 += BR) {
        if (lane < BR) {
            int row = r0 + lane;
            const double* ptr = nullptr;
            int kind = -2;
            if (row < mO) {
                int s = 0;
                while (obeg[s + 1] <= row) ++s;
                ptr = obase[s] + oap[s][row - obeg[s]];
                kind = -1;
            } else if (row < m) {
                kind = row - mO;
            }
            rowptr[lane] = ptr;
            rowprox[lane] = kind;
        }
        __syncthreads();
        double cv[CPT][BR];
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            const int kind = rowprox[i];
            const double* ptr = rowptr[i];
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) {
                int q = lane + 64 * cc;
                double v = 0.0;
                if (q < n) {
                    if (kind == -1) {
                        v = ptr[(int64_t)q * nmax];
                    } else if (kind >= 0) {
#pragma clang fp contract(off)
                        double dx = pxs[kind] - colx[cc];
                        double dy = pys[kind] - coly[cc];
                        v = kp.coef * log(dx * dx + dy * dy);
                    }
                }
                cv[cc][i] = v;
            }
        }
#pragma unroll
        for (int cj = 0; cj < CPT; ++cj) {
            for (int jj = 0; jj < 64; ++jj) {
                const int j = cj * 64 + jj;
                if (j >= n) break;
                if (lane == jj) {
                    double alpha = R0[j * NP + j];
                    double sigma = 0.0;
#pragma unroll
                    for (int i = 0; i < BR; ++i) sigma += cv[cj][i] * cv[cj][i];
                    double tau = 0.0;
                    if (sigma != 0.0) {
                        double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
                        tau = (beta - alpha) / beta;
                        double sc = 1.0 / (alpha - beta);
#pragma unroll
                        for (int i = 0; i < BR; ++i) vbuf[i] = cv[cj][i] * sc;
                        R0[j * NP + j] = beta;
                    }
                    taubuf = tau;
                }
                __syncthreads();
                const double tau = taubuf;
                if (tau != 0.0) {
#pragma unroll
                    for (int cc = 0; cc < CPT; ++cc) {
                        int q = lane + 64 * cc;
                        if (q > j && q < n) {
                            double w = R0[j * NP + q];
#pragma unroll
                            for (int i = 0; i < BR; ++i) w += vbuf[i] * cv[cc][i];
                            double tw = tau * w;
                            R0[j * NP + q] -= tw;
#pragma unroll
                            for (int i = 0; i < BR; ++i) cv[cc][i] -= tw * vbuf[i];
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    // ---- 2. pivoted QR of R0 ------------------------------------------------------
    bool done[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) done[cc] = (lane + 64 * cc) >= n;
    const int kmax = min(m, n);
    double rnorm0 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        double nu[CPT];
        double lmax = -1.0;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            nu[cc] = -1.0;
            if (!done[cc]) {
                int q = lane + 64 * cc;
                double s = 0.0;
                for (int i = j; i < n; ++i) {
                    double v = R0[i * NP + q];
                    s += v * v;
                }
                nu[cc] = s;
                lmax = fmax(lmax, s);
            }
        }
        const double numax = wave_max(lmax);
        const double mu = sqrt(numax);
        if (!(mu == mu)) break;   // no finite trailing norm left
        if (j == 0) {
            if (!(mu > 0.0)) break;
            rnorm0 = mu;
        } else if (mu <= kp.tol * rnorm0) {
            break;
        }
        const double thr = mu - kp.tau * rnorm0;
        int lmin = 1 << 30;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc)
            if (!done[cc] && sqrt(nu[cc]) >= thr) lmin = min(lmin, lane + 64 * cc);
        const int p = wave_min_int(lmin);
        if (p >= n) break;        // no candidate (non-finite norms): stop the ID here
        if (lane == (p & 63)) {
            double alpha = R0[j * NP + p];
            double sigma = 0.0;
            for (int i = j + 1; i < n; ++i) {
                double v = R0[i * NP + p];
                sigma += v * v;
            }
            double tau = 0.0;
            if (sigma != 0.0) {
                double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
                tau = (beta - alpha) / beta;
                double sc = 1.0 / (alpha - beta);
                for (int i = j + 1; i < n; ++i) vbuf[i] = R0[i * NP + p] * sc;
                R0[j * NP + p] = beta;
            }
            taubuf = tau;
            piv[j] = p;
            pivsel = p;
        }
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc)
            if (lane + 64 * cc == p) done[cc] = true;
        const double tau = taubuf;
        if (tau != 0.0) {
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) {
                if (done[cc]) continue;
                int q = lane + 64 * cc;
                double w = R0[j * NP + q];
                for (int i = j + 1; i < n; ++i) w += vbuf[i] * R0[i * NP + q];
                double tw = tau * w;
                R0[j * NP + q] -= tw;
                for (int i = j + 1; i < n; ++i) R0[i * NP + q] -= tw * vbuf[i];
            }
        }
        __syncthreads();
        k = j + 1;
    }

    // ---- 3. sorted sets and T = R11^{-1} R12 -----------------------------------------
    int srank[CPT];
    {
        int below = 0;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            bool isS = (lane + 64 * cc < n) && done[cc];
            unsigned long long mask = __ballot(isS);
            srank[cc] = below + __popcll(mask & ((1ull << lane) - 1ull));
            below += __popcll(mask);
            if (isS) srank_s[lane + 64 * cc] = srank[cc];
        }
    }
    __syncthreads();
    if (lane == 0) { krank[c] = k; mrows[c] = m; }
    const int64_t boff = (int64_t)c * nmax;
    double* Tb = Tout + (int64_t)c * nmax * nmax;
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
        int q = lane + 64 * cc;
        if (q >= n) continue;
        if (done[cc]) {
            spos[boff + srank[cc]] = q;
        } else {
            int rr = q - srank[cc];
            rpos[boff + rr] = q;
            // back substitution, in place in the lane's own column
            for (int a = k - 1; a >= 0; --a) {
                double s = R0[a * NP + q];
                for (int b = a + 1; b < k; ++b) s -= R0[a * NP + piv[b]] * R0[b * NP + q];
                s = s / R0[a * NP + piv[a]];
                R0[a * NP + q] = s;
            }
            for (int a = 0; a < k; ++a) Tb[srank_s[piv[a]] + (int64_t)rr * nmax] = R0[a * NP + q];
        }
    }
}

int elim_lds_limit();

void launch_id(const Level& L, const int* boxes, int nboxes, const double* pts, const double* ptmpl,
               const KernelParams& kp, double* work, hipStream_t s) {
    // R0 (rows < nmax, row stride NP = 64 * CPT) lives in LDS when it fits, else in
    // `work` (nboxes * NP * NP doubles).
    if (nboxes <= 0) return;
    dim3 grid(nboxes), block(64);
    const int lim = elim_lds_limit();
    if (L.nmax <= 64) {
        size_t lds = sizeof(double) * (size_t)L.nmax * 64;
        k_id<1, 32, true><<<grid, block, lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                   pts, ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows,
                                                   work);
    } else if (L.nmax <= 128) {
        size_t lds = sizeof(double) * (size_t)L.nmax * 128;
        if ((int)(lds + 4096) <= lim) {
            hipFuncSetAttribute((const void*)k_id<2, 32, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            k_id<2, 32, true><<<grid, block, lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                       pts, ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows,
                                                       work);
        } else {
            k_id<2, 32, false><<<grid, block, 0, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                      pts, ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows,
                                                      work);
        }
    } else {
        k_id<4, 16, false><<<grid, block, 0, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes, pts,
                                                  ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows, work);
    }
}

}  // namespace rss
