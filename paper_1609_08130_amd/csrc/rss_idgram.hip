// Interpolative decomposition of the boxes of one colour through the Gram matrix
// (Section 2.2, Definition 1, by greedy column-pivoted QR; Section 3.2, eq. smallid).
//
// Greedy column-pivoted QR of M depends on M only through G = M^T M: the trailing
// squared column norms after j steps are the diagonal of the Schur complement of the
// pivoted leading j x j block of G, and the R factor is the pivoted Cholesky factor of G
// (up to row signs, which T = R11^{-1} R12 does not see).  Forming G in FP64 would lose
// the trailing norms below sqrt(u) |M|, so
//   1. k_gram  : G is accumulated with compensated products and sums (double-double,
//                error ~ u^2 |M|^2), the rows of M split over several workgroups per box;
//   2. k_pchol : pivoted Cholesky of G in double-double, left-looking, with the pivot
//                rule of the oracle (fresh trailing norms = Schur diagonal; lowest
//                B-position among columns within tau |R_00| of the largest; stop at step
//                j > 0 once the largest is <= tol |R_00|), then T = R11^{-1} R12 in FP64.
// The ID input of box c is M = [A(O, B_c); w K(Gamma, B_c)] (O = boxes at Chebyshev
// distance 2, Gamma = n_p proxy points on the circle of radius proxy_radius * side).
#include "rss_internal.h"

namespace rss {

// ---- double-double arithmetic: Knuth's TwoSum, FMA-based TwoProd --------------------------
struct dd {
    double hi, lo;
};

__device__ inline void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
    s = a + b;
    double z = s - a;
    e = (a - (s - z)) + (b - z);
}

__device__ inline void fast_two_sum(double a, double b, double& s, double& e) {   // |a| >= |b|
#pragma clang fp contract(off)
    s = a + b;
    e = b - (s - a);
}

__device__ inline dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
    double s1, s2, t1, t2;
    two_sum(a.hi, b.hi, s1, s2);
    two_sum(a.lo, b.lo, t1, t2);
    s2 += t1;
    fast_two_sum(s1, s2, s1, s2);
    s2 += t2;
    fast_two_sum(s1, s2, s1, s2);
    return {s1, s2};
}

__device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, {-b.hi, -b.lo}); }

__device__ inline dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
    double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    double s, t;
    fast_two_sum(p, e, s, t);
    return {s, t};
}

__device__ inline dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul({q1, 0.0}, b));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul({q2, 0.0}, b));
    double q3 = r.hi / b.hi;
    double s, t;
    fast_two_sum(q1, q2, s, t);
    return dd_add({s, t}, {q3, 0.0});
}

__device__ inline dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
    if (!(a.hi > 0.0)) return {0.0, 0.0};
    double x = sqrt(a.hi);
    dd d = dd_sub(a, dd_mul({x, 0.0}, {x, 0.0}));   // a - x^2
    double corr = d.hi / (2.0 * x);                  // one Newton step
    double s, t;
    two_sum(x, corr, s, t);
    return {s, t};
}

__device__ inline double wave_max_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int kSliceRows = 256;   // rows of M per Gram workgroup
constexpr int kChunk = 32;        // rows staged in LDS at a time

// Number of Gram slices per box and workspace of one colour batch (doubles).
int id_slices(int nmax, int n_proxy) { return (16 * nmax + n_proxy + kSliceRows - 1) / kSliceRows; }

size_t id_work_doubles(int nmax, int n_proxy, size_t nboxes) {
    const size_t nn = (size_t)nmax * nmax;
    return nboxes * ((size_t)id_slices(nmax, n_proxy) * nn * 2 + nn * 2);
}

struct ORing {
    const double* base[16];
    const int* ap[16];
    int beg[17];
    int cnt;
};

__device__ inline void build_oring(ORing& o, const double* store, const int* nact, const int* apos, int c, int nb,
                                   int nmax) {
    const int64_t bsz = (int64_t)nmax * nmax;
    const int cx = c % nb, cy = c / nb;
    int cntO = 0;
    o.beg[0] = 0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            if (max(abs(dx), abs(dy)) != 2) continue;
            int ox = cx + dx, oy = cy + dy;
            if (ox < 0 || oy < 0 || ox >= nb || oy >= nb) continue;
            int ob = ox + nb * oy;
            o.base[cntO] = store + ((int64_t)ob * kNbr + nbr_slot(-dx, -dy)) * bsz;   // block (o, c)
            o.ap[cntO] = apos + (int64_t)ob * nmax;
            o.beg[cntO + 1] = o.beg[cntO] + nact[ob];
            ++cntO;
        }
    o.cnt = cntO;
}

// ---- 1. partial Gram matrices -------------------------------------------------------------
// grid (slices, boxes); thread owns TPT 2x2 tiles of the upper triangle of G.
template <int NTH, int TPT>
__global__ void __launch_bounds__(NTH) k_gram(const double* __restrict__ store, int nb, int nmax,
                                              const int* __restrict__ cnt, const int* __restrict__ gidx,
                                              const int* __restrict__ nact, const int* __restrict__ apos,
                                              const int* __restrict__ boxes, const double* __restrict__ pts,
                                              const double* __restrict__ ptmpl, KernelParams kp, int t,
                                              double* __restrict__ gpart, int nslice) {
#pragma clang fp contract(off)
    extern __shared__ double Ms[];   // kChunk x (nmax + 1)
    __shared__ ORing oring;
    __shared__ double pxs[kMaxProxy], pys[kMaxProxy];
    __shared__ double colx[kMaxBox], coly[kMaxBox];
    const int tid = threadIdx.x;
    const int c = boxes[blockIdx.y];
    const int sl = blockIdx.x;
    const int n = cnt[c];
    if (n == 0) return;
    if (tid == 0) build_oring(oring, store, nact, apos, c, nb, nmax);
    {
#pragma clang fp contract(off)
        const int cx = c % nb, cy = c / nb;
        double side_t = kp.side / (double)(1 << t);
        double ccx = kp.lo_x + ((double)cx + 0.5) * side_t;
        double ccy = kp.lo_y + ((double)cy + 0.5) * side_t;
        double rr = kp.proxy_radius * side_t;
        for (int p = tid; p < kp.n_proxy; p += NTH) {
            pxs[p] = ccx + rr * ptmpl[2 * p];
            pys[p] = ccy + rr * ptmpl[2 * p + 1];
        }
    }
    for (int q = tid; q < n; q += NTH) {
        int g = gidx[(int64_t)c * nmax + q];
        colx[q] = pts[2 * (int64_t)g];
        coly[q] = pts[2 * (int64_t)g + 1];
    }
    __syncthreads();
    const int mO = oring.beg[oring.cnt];
    const int m = mO + kp.n_proxy;
    const int r_begin = sl * kSliceRows;
    if (r_begin >= m) return;
    const int r_end = min(m, r_begin + kSliceRows);
    const int ld = nmax + 1;
    const int nt = (n + 1) >> 1;                  // 2x2 tiles per dimension
    const int ntiles = nt * (nt + 1) / 2;
    int tp[TPT], tq[TPT];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        int id = tid + u * NTH;
        tp[u] = -1;
        tq[u] = -1;
        if (id < ntiles) {
            // id -> (a, b) with a <= b over the upper triangle, row-major
            int a = 0, rem = id;
            while (rem >= nt - a) { rem -= nt - a; ++a; }
            tp[u] = 2 * a;
            tq[u] = 2 * (a + rem);
        }
    }
    double s[TPT][4], e[TPT][4];
#pragma unroll
    for (int u = 0; u < TPT; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) { s[u][v] = 0.0; e[u][v] = 0.0; }

    for (int r0 = r_begin; r0 < r_end; r0 += kChunk) {
        const int rows = min(kChunk, r_end - r0);
        __syncthreads();
        for (int idx = tid; idx < kChunk * ld; idx += NTH) {
            int i = idx % kChunk, q = idx / kChunk;
            double v = 0.0;
            if (i < rows && q < n) {
                int row = r0 + i;
                if (row < mO) {
                    int o = 0;
                    while (oring.beg[o + 1] <= row) ++o;
                    v = oring.base[o][oring.ap[o][row - oring.beg[o]] + (int64_t)q * nmax];
                } else {
#pragma clang fp contract(off)
                    int pp = row - mO;
                    double dx = pxs[pp] - colx[q];
                    double dy = pys[pp] - coly[q];
                    v = kp.coef * log(dx * dx + dy * dy);
                }
            }
            Ms[i * ld + q] = v;
        }
        __syncthreads();
        for (int i = 0; i < rows; ++i) {
            const double* row = Ms + i * ld;
#pragma unroll
            for (int u = 0; u < TPT; ++u) {
                if (tp[u] < 0) continue;
                const double a0 = row[tp[u]], a1 = row[tp[u] + 1];
                const double b0 = row[tq[u]], b1 = row[tq[u] + 1];
                const double av[4] = {a0 * b0, a0 * b1, a1 * b0, a1 * b1};
                const double aa[4] = {a0, a0, a1, a1};
                const double bb[4] = {b0, b1, b0, b1};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // compensated accumulation of the product aa*bb (TwoProd + TwoSum)
                    const double p = av[v];
                    const double pe = fma(aa[v], bb[v], -p);
                    double sn, te;
                    two_sum(s[u][v], p, sn, te);
                    s[u][v] = sn;
                    e[u][v] += te + pe;
                }
            }
        }
    }
    // write the slice's partial Gram (upper triangle, double-double)
    double2* G = (double2*)gpart + ((int64_t)blockIdx.y * nslice + sl) * nmax * nmax;
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        if (tp[u] < 0) continue;
        const int ps[4] = {tp[u], tp[u], tp[u] + 1, tp[u] + 1};
        const int qs[4] = {tq[u], tq[u] + 1, tq[u], tq[u] + 1};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (ps[v] < n && qs[v] < n && ps[v] <= qs[v]) {
                double hi, lo;
                fast_two_sum(s[u][v], e[u][v], hi, lo);
                G[(int64_t)ps[v] * nmax + qs[v]] = make_double2(hi, lo);
            }
        }
    }
}

// ---- 2. pivoted Cholesky of G in double-double, then T ------------------------------------
__device__ inline dd gram_entry(const double2* G, int nsl, int nmax, int64_t sstride, int a, int b) {
#pragma clang fp contract(off)
    if (a > b) { int t0 = a; a = b; b = t0; }
    dd acc = {0.0, 0.0};
    for (int s = 0; s < nsl; ++s) {
        double2 v = G[s * sstride + (int64_t)a * nmax + b];
        acc = dd_add(acc, {v.x, v.y});
    }
    return acc;
}

template <int NTH>
__global__ void __launch_bounds__(NTH) k_pchol(const int* __restrict__ cnt, const int* __restrict__ nact,
                                               const int* __restrict__ boxes, int nb, int nmax, KernelParams kp,
                                               const double* __restrict__ gpart, int nslice,
                                               double* __restrict__ rwork, int* __restrict__ krank,
                                               int* __restrict__ spos, int* __restrict__ rpos,
                                               double* __restrict__ Tout, int* __restrict__ mrows) {
#pragma clang fp contract(off)
    constexpr int NW = NTH / 64;
    __shared__ int piv[kMaxBox];
    __shared__ int srank_s[kMaxBox];
    __shared__ double rjj_hi, rjj_lo;
    __shared__ double redv[2][NW];
    __shared__ int redi[2][NW];
    __shared__ unsigned long long smask[NW];
    __shared__ int mrow_s;
    const int q = threadIdx.x;
    const int wv = q >> 6, lane = q & 63;
    const int c = boxes[blockIdx.x];
    const int n = cnt[c];
    if (n == 0) {
        if (q == 0) { krank[c] = 0; mrows[c] = 0; }
        return;
    }
    if (q == 0) {
        // rows of the ID input: active DOFs of the distance-2 boxes plus the proxies
        const int cx = c % nb, cy = c / nb;
        int mO = 0;
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                if (max(abs(dx), abs(dy)) != 2) continue;
                int ox = cx + dx, oy = cy + dy;
                if (ox < 0 || oy < 0 || ox >= nb || oy >= nb) continue;
                mO += nact[ox + nb * oy];
            }
        mrow_s = mO + kp.n_proxy;
    }
    __syncthreads();
    const int m = mrow_s;
    const int nsl = (m + kSliceRows - 1) / kSliceRows;
    const int64_t sstride = (int64_t)nmax * nmax;
    const double2* G = (const double2*)gpart + (int64_t)blockIdx.x * nslice * sstride;
    double2* R = (double2*)rwork + (int64_t)blockIdx.x * sstride;   // R[j * nmax + q]
    dd d = {0.0, 0.0};
    if (q < n) d = gram_entry(G, nsl, nmax, sstride, q, q);
    bool done = q >= n;
    const int kmax = min(m, n);
    double rnorm0 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        const int buf = j & 1;
        const double nu = done ? -1.0 : d.hi + d.lo;
        double wmax = wave_max_d(nu);
        if (lane == 0) redv[buf][wv] = wmax;
        __syncthreads();
        double numax = redv[buf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) numax = fmax(numax, redv[buf][w]);
        const double mu = sqrt(fmax(numax, 0.0));
        if (!(numax == numax)) break;
        if (j == 0) {
            if (!(mu > 0.0)) break;
            rnorm0 = mu;
        } else if (mu <= kp.tol * rnorm0) {
            break;
        }
        const double thr = mu - kp.tau * rnorm0;
        int cand = (!done && nu >= 0.0 && sqrt(nu) >= thr) ? q : (1 << 30);
        int wmin = wave_min_i(cand);
        if (lane == 0) redi[buf][wv] = wmin;
        __syncthreads();
        int p = redi[buf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) p = min(p, redi[buf][w]);
        if (p >= n) break;
        if (q == p) {
            dd r = dd_sqrt(d);
            rjj_hi = r.hi;
            rjj_lo = r.lo;
            piv[j] = p;
            R[(int64_t)j * nmax + p] = make_double2(r.hi, r.lo);
            done = true;
        }
        __syncthreads();
        if (!done) {
            // r_jq = (G_pq - sum_{i<j} r_ip r_iq) / r_jj ; d_q -= r_jq^2
            dd acc = gram_entry(G, nsl, nmax, sstride, p, q);
            for (int i = 0; i < j; ++i) {
                const double2 rip = R[(int64_t)i * nmax + p];
                const double2 riq = R[(int64_t)i * nmax + q];
                acc = dd_sub(acc, dd_mul({rip.x, rip.y}, {riq.x, riq.y}));
            }
            const dd rjq = dd_div(acc, {rjj_hi, rjj_lo});
            R[(int64_t)j * nmax + q] = make_double2(rjq.hi, rjq.lo);
            d = dd_sub(d, dd_mul(rjq, rjq));
        }
        __syncthreads();
        k = j + 1;
    }

    // ---- sorted sets and T = R11^{-1} R12 (FP64 back substitution) ----------------------
    const bool isS = (q < n) && done;
    const unsigned long long mask = __ballot(isS);
    if (lane == 0) smask[wv] = mask;
    __syncthreads();
    int below = 0;
    for (int w = 0; w < wv; ++w) below += __popcll(smask[w]);
    const int srank = below + __popcll(mask & ((1ull << lane) - 1ull));
    if (isS) srank_s[q] = srank;
    __syncthreads();
    if (q == 0) { krank[c] = k; mrows[c] = m; }
    const int64_t boff = (int64_t)c * nmax;
    double* Tb = Tout + (int64_t)c * nmax * nmax;
    if (q < n) {
        if (isS) {
            spos[boff + srank] = q;
        } else {
            const int rr = q - srank;
            rpos[boff + rr] = q;
            // in place in row-major R: R[a][q] <- t_a
            for (int a = k - 1; a >= 0; --a) {
                double acc = R[(int64_t)a * nmax + q].x;
                for (int b = a + 1; b < k; ++b) acc -= R[(int64_t)a * nmax + piv[b]].x * R[(int64_t)b * nmax + q].x;
                acc = acc / R[(int64_t)a * nmax + piv[a]].x;
                R[(int64_t)a * nmax + q].x = acc;
            }
            for (int a = 0; a < k; ++a) Tb[srank_s[piv[a]] + (int64_t)rr * nmax] = R[(int64_t)a * nmax + q].x;
        }
    }
}

void launch_id_gram(const Level& L, const int* boxes, int nboxes, const double* pts, const double* ptmpl,
                    const KernelParams& kp, double* work, hipStream_t s) {
    if (nboxes <= 0) return;
    const int nsl = id_slices(L.nmax, kp.n_proxy);
    const size_t nn = (size_t)L.nmax * L.nmax;
    double* gpart = work;
    double* rwork = work + (size_t)nboxes * nsl * nn * 2;
    const size_t lds = sizeof(double) * (size_t)kChunk * (L.nmax + 1);
    dim3 ggrid(nsl, nboxes);
    const int nt = (L.nmax + 1) / 2, ntiles = nt * (nt + 1) / 2;
    if (ntiles <= 3 * 256) {
        k_gram<256, 3><<<ggrid, dim3(256), lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes, pts,
                                                     ptmpl, kp, L.t, gpart, nsl);
    } else if (ntiles <= 5 * 256) {
        k_gram<256, 5><<<ggrid, dim3(256), lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes, pts,
                                                     ptmpl, kp, L.t, gpart, nsl);
    } else if (ntiles <= 9 * 256) {
        k_gram<256, 9><<<ggrid, dim3(256), lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes, pts,
                                                     ptmpl, kp, L.t, gpart, nsl);
    } else {
        k_gram<1024, 9><<<ggrid, dim3(1024), lds, s>>>(L.store, L.nb, L.nmax, L.cnt, L.gidx, L.nact, L.apos, boxes,
                                                       pts, ptmpl, kp, L.t, gpart, nsl);
    }
    if (L.nmax <= 64) {
        k_pchol<64><<<dim3(nboxes), dim3(64), 0, s>>>(L.cnt, L.nact, boxes, L.nb, L.nmax, kp, gpart, nsl, rwork,
                                                     L.krank, L.spos, L.rpos, L.T, L.mrows);
    } else if (L.nmax <= 128) {
        k_pchol<128><<<dim3(nboxes), dim3(128), 0, s>>>(L.cnt, L.nact, boxes, L.nb, L.nmax, kp, gpart, nsl, rwork,
                                                       L.krank, L.spos, L.rpos, L.T, L.mrows);
    } else {
        k_pchol<256><<<dim3(nboxes), dim3(256), 0, s>>>(L.cnt, L.nact, boxes, L.nb, L.nmax, kp, gpart, nsl, rwork,
                                                       L.krank, L.spos, L.rpos, L.T, L.mrows);
    }
}

}  // namespace rss
