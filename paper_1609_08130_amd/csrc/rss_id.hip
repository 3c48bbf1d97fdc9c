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

// Thread layout: NWC column waves x RG row groups, RPT chunk rows per thread.  Thread (rg, q) owns column q of B
// (n <= 64 NWC) and rows rg*RPT .. rg*RPT+RPT-1 of each TSQR chunk of RG*RPT rows.
// R0 (n rows, row stride NT = 64 NWC) is private per column; rows of the chunk are
// combined across the row groups through LDS (two barriers per reflector).
template <int NWC, int RG, int RPT, bool RLDS>
__global__ void __launch_bounds__(64 * NWC * RG) k_id(const double* __restrict__ store, int nb, int nmax,
                                                      const int* __restrict__ cnt, const int* __restrict__ gidx,
                                                      const int* __restrict__ nact, const int* __restrict__ apos,
                                                      const int* __restrict__ boxes, const double* __restrict__ pts,
                                                      const double* __restrict__ ptmpl, KernelParams kp, int t,
                                                      int* __restrict__ krank, int* __restrict__ spos,
                                                      int* __restrict__ rpos, double* __restrict__ Tout,
                                                      int* __restrict__ mrows, double* __restrict__ work) {
    constexpr int NT = 64 * NWC;          // column threads
    constexpr int BR = RG * RPT;          // chunk rows
    constexpr int VB = NT > BR ? NT : BR;
    // keep the reflector rows in registers across the second barrier unless a
    // 1024-thread group would run out of registers (then re-read them from LDS)
    constexpr bool CACHE_V = NWC * RG * 64 <= 512 && RPT <= 32;
    extern __shared__ double R0s[];       // RLDS: nmax x NT
    __shared__ double vraw[2][VB];
    __shared__ double part[2][RG];
    __shared__ double dpart[2][RG][NT];
    __shared__ double taubuf[2];
    __shared__ double scbuf[2];
    __shared__ double rjq[2][NT];
    __shared__ const double* obase[16];
    __shared__ const int* oap[16];
    __shared__ int obeg[17];
    __shared__ int nO;
    __shared__ const double* rowptr[BR];
    __shared__ int rowprox[BR];
    __shared__ double pxs[kMaxProxy], pys[kMaxProxy];
    __shared__ int piv[NT];
    __shared__ int srank_s[NT];
    __shared__ double redv[2][NWC];
    __shared__ int redi[2][NWC];
    __shared__ unsigned long long smask[NWC];

    const int tid = threadIdx.x;
    const int q = tid % NT;               // column
    const int rg = tid / NT;              // row group
    const int wv = q >> 6, lane = q & 63; // column wave (within row group 0)
    const int c = boxes[blockIdx.x];
    const int n = cnt[c];
    double* R0 = RLDS ? R0s : (work + (int64_t)blockIdx.x * NT * NT);
    if (n == 0) {
        if (tid == 0) { krank[c] = 0; mrows[c] = 0; }
        return;
    }
    const int cx = c % nb, cy = c / nb;
    const int64_t bsz = (int64_t)nmax * nmax;

    if (tid == 0) {
        // O ring: boxes at distance exactly 2, ascending linear index
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
    {
        // proxy points y_p = centre + radius * (cos, sin)(2 pi p / n_p)
#pragma clang fp contract(off)
        double side_t = kp.side / (double)(1 << t);
        double ccx = kp.lo_x + ((double)cx + 0.5) * side_t;
        double ccy = kp.lo_y + ((double)cy + 0.5) * side_t;
        double rr = kp.proxy_radius * side_t;
        for (int p = tid; p < kp.n_proxy; p += 64 * NWC * RG) {
            pxs[p] = ccx + rr * ptmpl[2 * p];
            pys[p] = ccy + rr * ptmpl[2 * p + 1];
        }
    }
    double colx = 0.0, coly = 0.0;
    if (q < n) {
        int g = gidx[(int64_t)c * nmax + q];
        colx = pts[2 * (int64_t)g];
        coly = pts[2 * (int64_t)g + 1];
    }
    for (int i = rg; i < n; i += RG) R0[i * NT + q] = 0.0;
    __syncthreads();
    const int mO = obeg[nO];
    const int m = mO + kp.n_proxy;

    // ---- 1. TSQR: [R0; chunk] -> R0, BR rows at a time ----------------------------------
    int step = 0;
    for (int r0 = 0; r0 < m; r0 += BR) {
        for (int i = tid; i < BR; i += 64 * NWC * RG) {
            int row = r0 + i;
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
            rowptr[i] = ptr;
            rowprox[i] = kind;
        }
        __syncthreads();
        double cv[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int ri = rg * RPT + i;
            const int kind = rowprox[ri];
            double v = 0.0;
            if (q < n) {
                if (kind == -1) {
                    v = rowptr[ri][(int64_t)q * nmax];
                } else if (kind >= 0) {
#pragma clang fp contract(off)
                    double dx = pxs[kind] - colx;
                    double dy = pys[kind] - coly;
                    v = kp.coef * log(dx * dx + dy * dy);
                }
            }
            cv[i] = v;
        }
        for (int j = 0; j < n; ++j, ++step) {
            const int buf = step & 1;
            // A: the threads of column j publish their rows and partial sums of squares
            if (q == j) {
                double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    s4[i & 3] += cv[i] * cv[i];
                    vraw[buf][rg * RPT + i] = cv[i];
                }
                part[buf][rg] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            }
            __syncthreads();
            // B: the owner forms the reflector scalars; every other column forms its
            //    partial product with the unscaled reflector rows
            if (q == j && rg == 0) {
                double sigma = 0.0;
#pragma unroll
                for (int g = 0; g < RG; ++g) sigma += part[buf][g];
                const double alpha = R0[j * NT + j];
                double tau = 0.0, sc = 0.0;
                if (sigma != 0.0) {
                    const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
                    tau = (beta - alpha) / beta;
                    sc = 1.0 / (alpha - beta);
                    R0[j * NT + j] = beta;
                }
                taubuf[buf] = tau;
                scbuf[buf] = sc;
            }
            const bool col = q > j && q < n;
            const double* v = vraw[buf] + rg * RPT;
            double vv[CACHE_V ? RPT : 1];
            if (col) {
                double w4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const double vi = v[i];
                    if (CACHE_V) vv[CACHE_V ? i : 0] = vi;
                    w4[i & 3] += vi * cv[i];
                }
                dpart[buf][rg][q] = (w4[0] + w4[1]) + (w4[2] + w4[3]);
                if (rg == 0) rjq[buf][q] = R0[j * NT + q];
            }
            __syncthreads();
            // C: rank-one update of the chunk rows; row group 0 updates row j of R0
            const double tau = taubuf[buf];
            if (col && tau != 0.0) {
                const double sc = scbuf[buf];
                double sdot = 0.0;
#pragma unroll
                for (int g = 0; g < RG; ++g) sdot += dpart[buf][g][q];
                const double rj = rjq[buf][q];
                const double tw = tau * (rj + sc * sdot);
                const double fct = tw * sc;
#pragma unroll
                for (int i = 0; i < RPT; ++i) cv[i] -= fct * (CACHE_V ? vv[CACHE_V ? i : 0] : v[i]);
                if (rg == 0) R0[j * NT + q] = rj - tw;
            }
        }
    }
    __syncthreads();

    // ---- 2. pivoted QR of R0 with fresh trailing norms (row group 0) -----------------------
    bool done = q >= n;
    const int kmax = min(m, n);
    double rnorm0 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j, ++step) {
        const int buf = step & 1;
        double nu = -1.0;
        if (rg == 0) {
            if (!done) {
                double s4[4] = {0.0, 0.0, 0.0, 0.0};
                for (int i = j; i < n; ++i) {
                    double vv = R0[i * NT + q];
                    s4[(i - j) & 3] += vv * vv;
                }
                nu = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            }
            double wmax = wave_max(nu);
            if (lane == 0) redv[buf][wv] = wmax;
        }
        __syncthreads();
        double numax = redv[buf][0];
#pragma unroll
        for (int w = 1; w < NWC; ++w) numax = fmax(numax, redv[buf][w]);
        const double mu = sqrt(numax);
        if (!(mu == mu)) break;
        if (j == 0) {
            if (!(mu > 0.0)) break;
            rnorm0 = mu;
        } else if (mu <= kp.tol * rnorm0) {
            break;
        }
        const double thr = mu - kp.tau * rnorm0;
        if (rg == 0) {
            int cand = (!done && sqrt(nu) >= thr) ? q : (1 << 30);
            int wmin = wave_min_int(cand);
            if (lane == 0) redi[buf][wv] = wmin;
        }
        __syncthreads();
        int p = redi[buf][0];
#pragma unroll
        for (int w = 1; w < NWC; ++w) p = min(p, redi[buf][w]);
        if (p >= n) break;
        if (q == p && rg == 0) {
            double alpha = R0[j * NT + p];
            double sigma = 0.0;
            for (int i = j + 1; i < n; ++i) {
                double vv = R0[i * NT + p];
                sigma += vv * vv;
            }
            double tau = 0.0;
            if (sigma != 0.0) {
                double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
                tau = (beta - alpha) / beta;
                double sc = 1.0 / (alpha - beta);
                for (int i = j + 1; i < n; ++i) vraw[buf][i] = R0[i * NT + p] * sc;
                R0[j * NT + p] = beta;
            }
            taubuf[buf] = tau;
            piv[j] = p;
        }
        if (q == p) done = true;
        __syncthreads();
        const double tau = taubuf[buf];
        if (rg == 0 && tau != 0.0 && !done) {
            const double* v = vraw[buf];
            double w4[4] = {R0[j * NT + q], 0.0, 0.0, 0.0};
            for (int i = j + 1; i < n; ++i) w4[(i - j) & 3] += v[i] * R0[i * NT + q];
            double tw = tau * ((w4[0] + w4[1]) + (w4[2] + w4[3]));
            R0[j * NT + q] -= tw;
            for (int i = j + 1; i < n; ++i) R0[i * NT + q] -= tw * v[i];
        }
        k = j + 1;
    }
    __syncthreads();

    // ---- 3. sorted sets and T = R11^{-1} R12 (row group 0) -------------------------------
    const bool isS = (q < n) && done;
    if (rg == 0) {
        const unsigned long long mask = __ballot(isS);
        if (lane == 0) smask[wv] = mask;
    }
    __syncthreads();
    int below = 0;
    for (int w = 0; w < wv; ++w) below += __popcll(smask[w]);
    const int srank = below + __popcll(smask[wv] & ((1ull << lane) - 1ull));
    if (rg == 0 && isS) srank_s[q] = srank;
    __syncthreads();
    if (rg != 0) return;
    if (q == 0) { krank[c] = k; mrows[c] = m; }
    const int64_t boff = (int64_t)c * nmax;
    double* Tb = Tout + (int64_t)c * nmax * nmax;
    if (q < n) {
        if (isS) {
            spos[boff + srank] = q;
        } else {
            int rr = q - srank;
            rpos[boff + rr] = q;
            for (int a = k - 1; a >= 0; --a) {
                double sacc = R0[a * NT + q];
                for (int b = a + 1; b < k; ++b) sacc -= R0[a * NT + piv[b]] * R0[b * NT + q];
                sacc = sacc / R0[a * NT + piv[a]];
                R0[a * NT + q] = sacc;
            }
            for (int a = 0; a < k; ++a) Tb[srank_s[piv[a]] + (int64_t)rr * nmax] = R0[a * NT + q];
        }
    }
}

int elim_lds_limit();

void launch_id(const Level& L, const int* boxes, int nboxes, const double* pts, const double* ptmpl,
               const KernelParams& kp, double* work, hipStream_t s) {
    // R0 (n rows, row stride 64 NWC) lives in LDS when it fits, else in `work`
    // (nboxes * (64 NWC)^2 doubles).  Chunks of 256 rows for |B| <= 64, else 128 (64 for |B| > 128).
    if (nboxes <= 0) return;
    dim3 grid(nboxes), block(512);
    const int lim = elim_lds_limit() - 32768;   // room for the static LDS arrays
    if (L.nmax <= 64) {
        size_t lds = sizeof(double) * (size_t)L.nmax * 64;
        k_id<1, 4, 32, true><<<grid, dim3(256), lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                       pts, ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows,
                                                       work);
    } else if (L.nmax <= 128 && (int)(sizeof(double) * (size_t)L.nmax * 128) <= lim) {
        size_t lds = sizeof(double) * (size_t)L.nmax * 128;
        hipFuncSetAttribute((const void*)k_id<2, 4, 32, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_id<2, 4, 32, true><<<grid, block, lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                       pts, ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows,
                                                       work);
    } else if (L.nmax <= 128) {
        k_id<2, 4, 32, false><<<grid, block, 0, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                      pts, ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows,
                                                      work);
    } else {
        k_id<4, 2, 32, false><<<grid, block, 0, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                      pts, ptmpl, kp, L.t, L.krank, L.spos, L.rpos, L.T, L.mrows,
                                                      work);
    }
}

}  // namespace rss
