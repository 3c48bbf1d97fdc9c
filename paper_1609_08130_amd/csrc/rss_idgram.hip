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
#include <algorithm>
#include <type_traits>

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

// 1 / b in double-double: one FP64 division and one Newton correction.
__device__ inline dd dd_recip(dd b) {
#pragma clang fp contract(off)
    const double q1 = 1.0 / b.hi;
    const dd r = dd_sub({1.0, 0.0}, dd_mul({q1, 0.0}, b));   // 1 - q1 b
    double s, t;
    fast_two_sum(q1, r.hi * q1, s, t);
    return {s, t};
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

// Largest value of the wave (fmax semantics), on every lane: DPP row shifts within rows
// of 16 lanes, then the row broadcasts of lanes 15 and 31, read back from lane 63.  Lanes
// without a source contribute +0.0 (the values reduced here are >= 0 or -1 for "none",
// and a result of 0 and one of -1 lead to the same decision).
template <int CTRL, int ROWS>
__device__ inline double dpp_fmax_step(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), CTRL, ROWS, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)((unsigned long long)b >> 32), CTRL, ROWS, 0xf, true);
    return fmax(v, __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo)));
}

__device__ inline double wave_max_d(double v) {
    v = dpp_fmax_step<0x111, 0xf>(v);   // row_shr:1
    v = dpp_fmax_step<0x112, 0xf>(v);   // row_shr:2
    v = dpp_fmax_step<0x114, 0xf>(v);   // row_shr:4
    v = dpp_fmax_step<0x118, 0xf>(v);   // row_shr:8
    v = dpp_fmax_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_fmax_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int kChunk = 32;        // rows staged in LDS at a time

// Launch shape of the Gram kernel for one colour.  With many boxes, one workgroup takes a
// 256-row slice of M and the whole upper triangle of G; with few boxes (the upper levels)
// the rows are cut into shorter slices and the triangle into groups of 256 2x2 tiles, so
// that the colour still spreads over the whole chip.  The partial Gram matrices of the
// slices are then summed by k_gram_reduce.
// With an FP32 store and plan field gram_i8, k_gram_i8 (exact sums on the int8 matrix
// cores, below) takes 256-row slices instead.
struct GramPlan {
    int slice_rows, nsl, groups, tpt, nth, i8;
};

constexpr int kI8Rows = 256;   // most rows of M per slice of the int8 Gram kernel
constexpr int kI8Pitch = 80;   // LDS bytes per column of a 64-row digit chunk (+16: no bank conflicts)
constexpr int kI8MaxN = 96;    // largest box of the int8 path
constexpr int kI8L = 5;        // base-128 digits per entry
constexpr int kI8Tpw = 3;      // 16 x 16 tiles of G per wave
constexpr int kI8It = 4;       // columns per thread in a 64-row chunk (16 npad <= 4 * 64 NW)

// waves of k_gram_i8 for boxes of at most nmax <= kI8MaxN DOFs: 4 or 8 (kI8Tpw tiles each)
static int gram_i8_waves(int nmax) {
    const int np16 = (nmax + 15) / 16, ntile = np16 * (np16 + 1) / 2;
    return ntile <= 4 * kI8Tpw ? 4 : 8;
}

static GramPlan gram_plan(int nmax, int n_proxy, size_t nboxes, int weak, bool store32) {
    // rows of M: <= 16 boxes at distance 2 (24 at distance 1 or 2 in a weak pass), plus proxies
    const int mmax = (weak ? 24 : 16) * nmax + n_proxy;
    const int nt = (nmax + 1) / 2, ntiles = nt * (nt + 1) / 2;
    GramPlan g;
    g.i8 = 0;
    const PlanParams pp = plan_params((int)nboxes);
    if (store32 && pp.gram_i8 && nmax <= kI8MaxN) {
        // 256-row slices; few-box colours halve them (down to one 64-row chunk) until the
        // colour has gram_min_wg workgroups
        g.i8 = 1;
        g.slice_rows = kI8Rows;
        g.groups = 1;
        g.tpt = 1;
        g.nth = 64 * gram_i8_waves(nmax);
        if (!pp.gram_many)
            while (g.slice_rows > 64 && nboxes * (size_t)((mmax + g.slice_rows - 1) / g.slice_rows) < (size_t)pp.gram_min_wg)
                g.slice_rows >>= 1;
    } else if (pp.gram_many) {
        // fewest tile slots (idle threads) over 192- and 256-thread workgroups with 3, 5 or
        // 9 tiles per thread, the fewer tiles per thread on a tie
        g.slice_rows = 256;
        int best = 1 << 30;
        for (int tpt : {3, 5, 9})
            for (int nth : {192, 256}) {
                const int groups = (ntiles + nth * tpt - 1) / (nth * tpt);
                if (groups * nth * tpt < best) {
                    best = groups * nth * tpt;
                    g.tpt = tpt;
                    g.nth = nth;
                    g.groups = groups;
                }
            }
    } else {
        g.nth = 256;
        g.tpt = 1;
        g.groups = (ntiles + 255) / 256;
        g.slice_rows = 128;
        while (g.slice_rows > kChunk &&
               nboxes * (size_t)((mmax + g.slice_rows - 1) / g.slice_rows) * g.groups < (size_t)pp.gram_min_wg)
            g.slice_rows >>= 1;
    }
    g.nsl = (mmax + g.slice_rows - 1) / g.slice_rows;
    return g;
}

// Rows of R kept in LDS by the pivoted Cholesky of a colour with few boxes (the rest stay
// in the workspace).
static int pchol_lds_rows(int nmax) { return std::max(1, std::min(nmax, 49152 / (16 * nmax))); }

// Workspace (doubles) for any colour of at most nboxes boxes: the plan, and with it the
// number of slices, depends on the colour's box count.
size_t id_work_doubles(int nmax, int n_proxy, size_t nboxes, int weak, bool store32) {
    const size_t nn = (size_t)nmax * nmax;
    size_t slices = 0;
    for (size_t b = 1; b <= nboxes; ++b)
        slices = std::max(slices, b * (size_t)gram_plan(nmax, n_proxy, b, weak, store32).nsl);
    return slices * nn * 2 + nboxes * nn * 2;
}

constexpr int kRingMax = 24;   // boxes of the ID rows: 16 at distance 2, 24 at distance 1 or 2

template <typename ST>
struct ORing {
    const ST* base[kRingMax];
    const int* ap[kRingMax];
    int beg[kRingMax + 1];
    int cnt;
};

// Offset (dx, dy) of ring slot s in ascending (dy, dx) order.  Strong pass: the 16 offsets at
// distance 2 (5 on the row dy = -2, then pairs dx = -2, 2 on the rows -1, 0, 1, then 5 on
// dy = 2).  Weak pass: the 24 offsets of the 5 x 5 window but its centre.
__device__ inline void ring_offset(int s, int weak, int& dx, int& dy) {
    if (weak) {
        const int i = s < 12 ? s : s + 1;
        dx = i % 5 - 2;
        dy = i / 5 - 2;
        return;
    }
    if (s < 5) { dx = s - 2; dy = -2; }
    else if (s < 11) { dy = (s - 5) / 2 - 1; dx = ((s - 5) & 1) ? 2 : -2; }
    else { dx = s - 13; dy = 2; }
}

// Threads 0..15 (0..23 in a weak pass) look up one ring slot each (the active counts load in
// parallel); after a barrier, thread 0 lists the boxes that exist in ring order.  Ends with
// a barrier.
template <typename ST>
__device__ inline void build_oring(ORing<ST>& o, int* ring_box, int* ring_nact, const ST* store, const int* nact,
                                   const int* apos, int c, int nb, int nmax, int weak) {
    const int64_t bsz = (int64_t)nmax * nmax;
    const int tid = threadIdx.x;
    const int nslot = weak ? 24 : 16;
    if (tid < nslot) {
        int dx, dy;
        ring_offset(tid, weak, dx, dy);
        const int ox = c % nb + dx, oy = c / nb + dy;
        const bool in = ox >= 0 && oy >= 0 && ox < nb && oy < nb;
        ring_box[tid] = in ? ox + nb * oy : -1;
        ring_nact[tid] = in ? nact[ox + nb * oy] : 0;
    }
    __syncthreads();
    if (tid == 0) {
        int cntO = 0;
        o.beg[0] = 0;
        for (int s = 0; s < nslot; ++s) {
            const int ob = ring_box[s];
            if (ob < 0) continue;
            int dx, dy;
            ring_offset(s, weak, dx, dy);
            o.base[cntO] = store + ((int64_t)ob * kNbr + nbr_slot(-dx, -dy)) * bsz;   // block (o, c)
            o.ap[cntO] = apos + (int64_t)ob * nmax;
            o.beg[cntO + 1] = o.beg[cntO] + ring_nact[s];
            ++cntO;
        }
        o.cnt = cntO;
    }
    __syncthreads();
}

// ---- 1. partial Gram matrices -------------------------------------------------------------
// One row of M into the thread's TPT 2x2 tiles: compensated accumulation of each product
// (TwoSum into s, its error into e); TWOPROD adds the product's own rounding error.
template <int TPT, bool TWOPROD>
__device__ inline void gram_row(const double* row, const int (&tp)[TPT], const int (&tq)[TPT], double (&s)[TPT][4],
                                double (&e)[TPT][4]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        if (tp[u] < 0) continue;
        const double2 ap = *(const double2*)(row + tp[u]);
        const double2 bq = *(const double2*)(row + tq[u]);
        const double a0 = ap.x, a1 = ap.y, b0 = bq.x, b1 = bq.y;
        const double aa[4] = {a0, a0, a1, a1};
        const double bb[4] = {b0, b1, b0, b1};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double p = aa[v] * bb[v];
            double sn, te;
            two_sum(s[u][v], p, sn, te);
            s[u][v] = sn;
            if constexpr (TWOPROD) e[u][v] += te + fma(aa[v], bb[v], -p);
            else e[u][v] += te;
        }
    }
}

// Rows of M of box c: active DOFs of the distance-2 boxes (distance 1 or 2 in a weak pass)
// plus the proxies.
__device__ inline int id_rows(const int* nact, int c, int nb, int n_proxy, int weak) {
    const int cx = c % nb, cy = c / nb;
    int mO = 0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            const int d = max(abs(dx), abs(dy));
            if (d == 0 || (d == 1 && !weak)) continue;
            int ox = cx + dx, oy = cy + dy;
            if (ox < 0 || oy < 0 || ox >= nb || oy >= nb) continue;
            mO += nact[ox + nb * oy];
        }
    return mO + n_proxy;
}

// grid (slices x tile groups, boxes); thread owns TPT 2x2 tiles of the upper triangle of G.
template <int NTH, int TPT, typename ST>
__global__ void __launch_bounds__(NTH) k_gram(const ST* __restrict__ store, int nb, int nmax,
                                              const int* __restrict__ cnt, const int* __restrict__ gidx,
                                              const int* __restrict__ nact, const int* __restrict__ apos,
                                              const int* __restrict__ boxes, const double* __restrict__ pts,
                                              const double* __restrict__ ptmpl, KernelParams kp, int t,
                                              double* __restrict__ gpart, int nslice, int slice_rows) {
#pragma clang fp contract(off)
    // kChunk rows of M, leading dimension nmax + 2: even, so that the column pairs of a
    // 2x2 tile are 16-byte aligned and read as one double2
    extern __shared__ double2 Ms2[];
    double* Ms = (double*)Ms2;
    __shared__ ORing<ST> oring;
    __shared__ int ring_box[kRingMax], ring_nact[kRingMax];
    __shared__ double pxs[kMaxProxy], pys[kMaxProxy];
    __shared__ double colx[kMaxBox], coly[kMaxBox];
    __shared__ const ST* rowsrc[kChunk];
    const int tid = threadIdx.x;
    const int c = boxes[blockIdx.y];
    const int sl = blockIdx.x % nslice;
    const int grp = blockIdx.x / nslice;
    const int n = cnt[c];
    if (n == 0) return;
    // slices past the box's rows and tile groups past its triangle leave before the set-up
    if (sl * slice_rows >= id_rows(nact, c, nb, kp.n_proxy, kp.weak)) return;
    {
        const int nt0 = (n + 1) >> 1;
        if (grp * NTH * TPT >= nt0 * (nt0 + 1) / 2) return;
    }
    build_oring(oring, ring_box, ring_nact, store, nact, apos, c, nb, nmax, kp.weak);
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
    const int r_begin = sl * slice_rows;
    if (r_begin >= m) return;
    const int r_end = min(m, r_begin + slice_rows);
    const int ld = nmax + 2;
    const int nt = (n + 1) >> 1;                  // 2x2 tiles per dimension
    const int ntiles = nt * (nt + 1) / 2;
    if (grp * NTH * TPT >= ntiles) return;        // this box has no tiles in the group
    int tp[TPT], tq[TPT];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        int id = tid + u * NTH + grp * NTH * TPT;
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
        // source row of each chunk line (one lookup per line), then the chunk with GU
        // loads in flight per thread
        constexpr int GU = 4;
        if (tid < kChunk) {
            const ST* src = nullptr;
            const int row = r0 + tid;
            if (tid < rows && row < mO) {
                int o = 0;
                while (oring.beg[o + 1] <= row) ++o;
                src = oring.base[o] + oring.ap[o][row - oring.beg[o]];
            }
            rowsrc[tid] = src;
        }
        __syncthreads();
        for (int idx0 = tid; idx0 < kChunk * ld; idx0 += NTH * GU) {
            double v[GU];
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int idx = idx0 + u * NTH;
                const int i = idx & (kChunk - 1), q = idx / kChunk;
                const ST* src = rowsrc[i];
                v[u] = (idx < kChunk * ld && i < rows && q < n && src) ? (double)src[(int64_t)q * nmax] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int idx = idx0 + u * NTH;
                const int i = idx & (kChunk - 1), q = idx / kChunk;
                // proxy entries are written by the loop below, not here
                const bool proxy = i < rows && q < n && !rowsrc[i];
                if (idx < kChunk * ld && !proxy) Ms[i * ld + q] = v[u];
            }
        }
        // proxy rows (the last rows of M) from the kernel
        if (r0 + rows > mO) {
            const int i0 = max(0, mO - r0);
            for (int idx = tid; idx < (rows - i0) * n; idx += NTH) {
#pragma clang fp contract(off)
                const int i = i0 + idx % (rows - i0), q = idx / (rows - i0);
                const int pp = r0 + i - mO;
                const double dx = pxs[pp] - colx[q];
                const double dy = pys[pp] - coly[q];
                Ms[i * ld + q] = kp.coef * log(dx * dx + dy * dy);
            }
        }
        __syncthreads();
        // Rows copied from an FP32 store hold FP32 values, whose products are exact in FP64:
        // their rounding error term is zero and is not formed (the sums are unchanged).
        const int exact_end = std::is_same<ST, float>::value ? min(max(mO - r0, 0), rows) : 0;
        int i = 0;
        for (; i < exact_end; ++i) gram_row<TPT, false>(Ms + i * ld, tp, tq, s, e);
        for (; i < rows; ++i) gram_row<TPT, true>(Ms + i * ld, tp, tq, s, e);
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

// ---- 1b. exact Gram sums of FP32 rows on the int8 matrix cores ---------------------------
// In a slice of M, the rows copied from an FP32 store are fixed-point numbers column by
// column: with E_q the largest binary exponent of column q over the slice (x = f 2^E,
// f in [1/2, 1)) and U_q = E_q - 7 L + 1, every entry is an integer X = x 2^-U_q with
// |X| < 2^(7 L - 1), exactly so when the column's exponents span at most 7 L - 25 (the last
// mantissa bit of its smallest entry is then >= 2^U_q).  With L = 5 (spreads up to 10),
// X splits into digits d_0 .. d_3 in [-64, 64] and a last one with |d| <= 64, and
//     sum_k X_kp X_kq = sum_s 128^s S_s,   S_s = sum_{u+v=s} sum_k d_u(k,p) d_v(k,q),
// every S_s an exact int32 sum (|S_s| <= 5 * 256 * 64^2 < 2^23) formed by
// v_mfma_i32_16x16x64_i8, one 64-row chunk (one K step) at a time.  The 2L - 1 sums give the
// slice's entry exactly as two int64 words (S_0..S_4 and S_5..S_8, each below 2^53 in
// magnitude), hence as a double-double by one TwoSum, scaled by 2^(U_p + U_q).  The slice's
// proxy rows (FP64 kernel values) add their products with TwoProd.  A slice with a wider
// exponent spread sums on the vector units in double-double instead.  Output: k_gram's slice layout (upper triangle, hi and lo), for k_pchol.
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Row and column of the 16 x 16 int32 result of v_mfma_i32_16x16x64_i8 held in element v of
// lane l.
__device__ inline void i8_out(int l, int v, int& i, int& j) {
    i = 4 * (l >> 4) + v;
    j = l & 15;
}

// The wave's tiles (P, Q) of one 64-row chunk: kI8L digit operands of each side, kI8L^2
// products into the 2 kI8L - 1 sums of each tile.
__device__ inline void i8_chunk_mma(const signed char* dig, int limb, const int (&tP)[kI8Tpw],
                                    const int (&tQ)[kI8Tpw], i32x4 (&acc)[kI8Tpw][2 * kI8L - 1]) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, koff = 16 * (lane >> 4);
#pragma unroll
    for (int t = 0; t < kI8Tpw; ++t) {
        if (tP[t] < 0) continue;   // the same on the whole wave
        i32x4 a[kI8L], b[kI8L];
#pragma unroll
        for (int u = 0; u < kI8L; ++u) {
            a[u] = *(const i32x4*)(dig + u * limb + (16 * tP[t] + r) * kI8Pitch + koff);
            b[u] = *(const i32x4*)(dig + u * limb + (16 * tQ[t] + r) * kI8Pitch + koff);
        }
#pragma unroll
        for (int u = 0; u < kI8L; ++u)
#pragma unroll
            for (int v = 0; v < kI8L; ++v)
                acc[t][u + v] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[u], b[v], acc[t][u + v], 0, 0, 0);
    }
}

// One thread's share of a 64-row chunk: for each of its kI8It columns q = (tid >> 4) +
// (NTH / 16) j, the rows i4 + 16 e (i4 = tid & 15, e < 4) of the chunk, already loaded
// (zero past the slice's O-ring rows or past column n).  Their digits go to LDS packed four
// to a 32-bit word, dig[u][q][4 i4 + e]: the rows of a chunk sit in LDS in the order
// (i4, e), the same for every column, so the products over a chunk are unchanged.
template <int NTH>
__device__ inline void i8_digits(signed char* dig, int limb, int npad_box, const float (&x)[kI8It][4],
                                 const int* ucol) {
    const int i4 = threadIdx.x & 15, qb = threadIdx.x >> 4;
#pragma unroll
    for (int j = 0; j < kI8It; ++j) {
        const int q = qb + (NTH / 16) * j;
        if (q >= npad_box) break;
        int w[kI8L];
#pragma unroll
        for (int u = 0; u < kI8L; ++u) w[u] = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // x 2^-U_q is an integer below 2^34 in magnitude: exact in FP32, and so is every
            // step below (rint of an exact quotient by 128; the remainder is an integer <= 64)
            float y = ldexpf(x[j][e], -ucol[q]);
#pragma unroll
            for (int u = 0; u < kI8L; ++u) {
                float d = y;
                if (u < kI8L - 1) {
                    const float r = rintf(y * 0.0078125f);
                    d = fmaf(r, -128.0f, y);
                    y = r;
                }
                w[u] |= ((int)d & 255) << (8 * e);
            }
        }
#pragma unroll
        for (int u = 0; u < kI8L; ++u) *(int*)(dig + u * limb + q * kI8Pitch + 4 * i4) = w[u];
    }
}

// grid (slices of slice_rows <= kI8Rows rows, boxes), 64 NW threads; wave w owns tiles
// w, w + NW, w + 2 NW of the upper triangle of 16 x 16 tiles of G.  Every thread holds its
// share of the slice (kI8Rows / 64 chunks x kI8It columns x 4 rows) in registers from one
// batch of loads, used by the exponent pass and then by the digits of each chunk.
template <int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) k_gram_i8(const float* __restrict__ store, int nb, int nmax,
                                                     const int* __restrict__ cnt, const int* __restrict__ gidx,
                                                     const int* __restrict__ nact, const int* __restrict__ apos,
                                                     const int* __restrict__ boxes, const double* __restrict__ pts,
                                                     const double* __restrict__ ptmpl, KernelParams kp, int t,
                                                     double* __restrict__ gpart, int nslice, int slice_rows,
                                                     int* __restrict__ flag) {
#pragma clang fp contract(off)
    constexpr int NTH = 64 * NW;
    // one chunk's digits [L][npad][kI8Pitch]; after the products, the proxy rows [k][npad]
    extern __shared__ double2 i8_lds[];
    signed char* dig = (signed char*)i8_lds;
    double* prox = (double*)i8_lds;
    __shared__ ORing<float> oring;
    __shared__ int ring_box[kRingMax], ring_nact[kRingMax];
    __shared__ double pxs[kMaxProxy], pys[kMaxProxy];
    __shared__ double colx[kI8MaxN], coly[kI8MaxN];
    __shared__ int emax[kI8MaxN], emin[kI8MaxN], ucol[kI8MaxN];
    __shared__ const float* rsrc[kI8Rows];
    __shared__ int wide_s;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int c = boxes[blockIdx.y];
    const int sl = blockIdx.x;
    const int n = cnt[c];
    if (n == 0) return;
    if (sl * slice_rows >= id_rows(nact, c, nb, kp.n_proxy, kp.weak)) return;
    build_oring(oring, ring_box, ring_nact, store, nact, apos, c, nb, nmax, kp.weak);
    {
        const int cx = c % nb, cy = c / nb;
        const double side_t = kp.side / (double)(1 << t);
        const double ccx = kp.lo_x + ((double)cx + 0.5) * side_t;
        const double ccy = kp.lo_y + ((double)cy + 0.5) * side_t;
        const double rr = kp.proxy_radius * side_t;
        for (int p = tid; p < kp.n_proxy; p += NTH) {
            pxs[p] = ccx + rr * ptmpl[2 * p];
            pys[p] = ccy + rr * ptmpl[2 * p + 1];
        }
    }
    for (int q = tid; q < n; q += NTH) {
        const int g = gidx[(int64_t)c * nmax + q];
        colx[q] = pts[2 * (int64_t)g];
        coly[q] = pts[2 * (int64_t)g + 1];
    }
    const int mO = oring.beg[oring.cnt];
    const int m = mO + kp.n_proxy;
    const int r0 = sl * slice_rows, r1 = min(m, r0 + slice_rows);
    const int nro = max(min(r1, mO) - r0, 0);   // O-ring rows of the slice: [r0, r0 + nro)
    const int p0 = max(r0, mO), npr = max(r1 - p0, 0);   // its proxy rows: [p0, p0 + npr)
    for (int i = tid; i < kI8Rows; i += NTH) {
        const float* src = nullptr;
        if (i < nro) {
            const int row = r0 + i;
            int o = 0;
            while (oring.beg[o + 1] <= row) ++o;
            src = oring.base[o] + oring.ap[o][row - oring.beg[o]];
        }
        rsrc[i] = src;
    }
    __syncthreads();
    // The slice's O-ring values, all loads issued at once: chunk ch, column j of the thread,
    // rows 64 ch + i4 + 16 e (16 lanes read 16 consecutive rows of one column).
    const int i4 = tid & 15, qb = tid >> 4;
    constexpr int NCH = kI8Rows / 64;
    float xv[NCH][kI8It][4];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int j = 0; j < kI8It; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 64 * ch + i4 + 16 * e, q = qb + (NTH / 16) * j;
                xv[ch][j][e] = (row < nro && q < n) ? rsrc[row][(int64_t)q * nmax] : 0.0f;
            }
    // exponent range of each column (zeros aside): the 16 lanes of a column reduce by
    // quarter-wave shuffles
#pragma unroll
    for (int j = 0; j < kI8It; ++j) {
        int hi = -100000, lo = 100000;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (xv[ch][j][e] != 0.0f) {
                    int ex;
                    (void)frexpf(xv[ch][j][e], &ex);
                    hi = max(hi, ex);
                    lo = min(lo, ex);
                }
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) {
            hi = max(hi, __shfl_xor(hi, o, 64));
            lo = min(lo, __shfl_xor(lo, o, 64));
        }
        const int q = qb + (NTH / 16) * j;
        if (i4 == 0 && q < n) {
            emax[q] = hi;
            emin[q] = lo;
        }
    }
    if (tid == 0) wide_s = 0;
    __syncthreads();
    for (int q = tid; q < n; q += NTH)
        if (emax[q] > -100000 && emax[q] - emin[q] > 7 * kI8L - 25) wide_s = 1;
    __syncthreads();
    double2* G = (double2*)gpart + ((int64_t)blockIdx.y * nslice + sl) * nmax * nmax;
    if (wide_s) {
        // exponent spread too wide for the digits: compensated sums on the vector units
        if (tid == 0) atomicOr(flag, 128);   // records that this form ran
        for (int e = tid; e < n * n; e += NTH) {
            const int p = e / n, q = e % n;
            if (p > q) continue;
            double sh = 0.0, se = 0.0;
            for (int i = 0; i < nro; ++i) {
                const double a = (double)rsrc[i][(int64_t)p * nmax], b = (double)rsrc[i][(int64_t)q * nmax];
                double sn, te;
                two_sum(sh, a * b, sn, te);   // FP32 products are exact in FP64
                sh = sn;
                se += te;
            }
            for (int k = 0; k < npr; ++k) {
                const int pp = p0 - mO + k;
                const double dxp = pxs[pp] - colx[p], dyp = pys[pp] - coly[p];
                const double dxq = pxs[pp] - colx[q], dyq = pys[pp] - coly[q];
                const double a = kp.coef * log(dxp * dxp + dyp * dyp), b = kp.coef * log(dxq * dxq + dyq * dyq);
                const double pr = a * b;
                double sn, te;
                two_sum(sh, pr, sn, te);
                sh = sn;
                se += te + fma(a, b, -pr);
            }
            double hi, lo;
            fast_two_sum(sh, se, hi, lo);
            G[(int64_t)p * nmax + q] = make_double2(hi, lo);
        }
        return;
    }
    const int npad_box = (n + 15) & ~15, np16 = npad_box >> 4;
    const int limb = ((nmax + 15) & ~15) * kI8Pitch;
    for (int q = tid; q < npad_box; q += NTH) ucol[q] = q < n && emax[q] > -100000 ? emax[q] - 7 * kI8L + 1 : 0;
    int tP[kI8Tpw], tQ[kI8Tpw];
    {
        const int ntile = np16 * (np16 + 1) / 2;
#pragma unroll
        for (int u = 0; u < kI8Tpw; ++u) {
            const int tt = wv + NW * u;
            tP[u] = -1;
            tQ[u] = -1;
            if (tt < ntile) {
                int P = 0, rem = tt;
                while (rem >= np16 - P) { rem -= np16 - P; ++P; }
                tP[u] = P;
                tQ[u] = P + rem;
            }
        }
    }
    i32x4 acc[kI8Tpw][2 * kI8L - 1];
#pragma unroll
    for (int u = 0; u < kI8Tpw; ++u)
#pragma unroll
        for (int s2 = 0; s2 < 2 * kI8L - 1; ++s2) acc[u][s2] = i32x4{0, 0, 0, 0};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        if (64 * ch >= nro) break;
        __syncthreads();   // ucol written; the previous chunk's operands read
        i8_digits<NTH>(dig, limb, npad_box, xv[ch], ucol);
        __syncthreads();
        i8_chunk_mma(dig, limb, tP, tQ, acc);
    }
    __syncthreads();
    // the slice's proxy rows, FP64, over the digits
    for (int e = tid; e < npr * n; e += NTH) {
        const int k = e / n, q = e % n;
        const int pp = p0 - mO + k;
        const double dx = pxs[pp] - colx[q], dy = pys[pp] - coly[q];
        prox[k * npad_box + q] = kp.coef * log(dx * dx + dy * dy);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kI8Tpw; ++u) {
        if (tP[u] < 0) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int i, j;
            i8_out(lane, v, i, j);
            const int p = 16 * tP[u] + i, q = 16 * tQ[u] + j;
            if (q >= n || p > q) continue;
            // sum_s 128^s S_s = w1 2^35 + w0, both words exact in FP64
            long long w0 = 0, w1 = 0;
#pragma unroll
            for (int s2 = 2 * kI8L - 2; s2 >= 0; --s2) {
                if (s2 >= 5) w1 = w1 * 128 + acc[u][s2][v];
                else w0 = w0 * 128 + acc[u][s2][v];
            }
            dd a;
            two_sum(ldexp((double)w1, 35), (double)w0, a.hi, a.lo);
            a.hi = ldexp(a.hi, ucol[p] + ucol[q]);
            a.lo = ldexp(a.lo, ucol[p] + ucol[q]);
            for (int k = 0; k < npr; ++k) {
                const double x = prox[k * npad_box + p], y = prox[k * npad_box + q];
                const double pr = x * y;
                a = dd_add(a, {pr, fma(x, y, -pr)});
            }
            G[(int64_t)p * nmax + q] = make_double2(a.hi, a.lo);
        }
    }
}

// ---- 2. sum of the partial Gram matrices (few-box colours) ---------------------------------

// grid (nmax^2 / 256, boxes): slice 0 <- sum over the slices that hold rows, in slice order.
__global__ void __launch_bounds__(256) k_gram_reduce(const int* __restrict__ cnt, const int* __restrict__ nact,
                                                     const int* __restrict__ boxes, int nb, int nmax, int n_proxy,
                                                     int weak, double* __restrict__ gpart, int nslice,
                                                     int slice_rows) {
#pragma clang fp contract(off)
    const int c = boxes[blockIdx.y];
    const int n = cnt[c];
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int pa = e / nmax, qa = e % nmax;
    if (pa >= n || qa >= n || pa > qa) return;
    const int m = id_rows(nact, c, nb, n_proxy, weak);
    const int nsl = (m + slice_rows - 1) / slice_rows;
    const int64_t sstride = (int64_t)nmax * nmax;
    double2* G = (double2*)gpart + (int64_t)blockIdx.y * nslice * sstride + e;
    dd acc = {0.0, 0.0};
    for (int sl = 0; sl < nsl; ++sl) {
        double2 v = G[sl * sstride];
        acc = dd_add(acc, {v.x, v.y});
    }
    G[0] = make_double2(acc.hi, acc.lo);
}

// ---- 3. pivoted Cholesky of G in double-double, then T ------------------------------------
__device__ inline dd gram_entry(const double2* G, int nsl, int nmax, int64_t sstride, int a, int b) {
#pragma clang fp contract(off)
    if (a > b) { int t0 = a; a = b; b = t0; }
    const double2* g = G + (int64_t)a * nmax + b;
    // the first kGramPf slices are loaded together, then summed in slice order (one load
    // latency per entry instead of one per slice)
    constexpr int kGramPf = 6;
    double2 v[kGramPf];
#pragma unroll
    for (int s = 0; s < kGramPf; ++s) v[s] = s < nsl ? g[s * sstride] : make_double2(0.0, 0.0);
    dd acc = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kGramPf; ++s)
        if (s < nsl) acc = dd_add(acc, {v[s].x, v[s].y});
    for (int s = kGramPf; s < nsl; ++s) {
        const double2 w = g[s * sstride];
        acc = dd_add(acc, {w.x, w.y});
    }
    return acc;
}

// Sum of v over the SUB adjacent lanes of a column group, identical on all of them
// (double-double addition is commutative bit for bit, so both orders agree).
// The value of lane l ^ O (O = 1 or 2: a DPP quad permutation; otherwise an LDS-crossbar
// shuffle), moved bit for bit.
template <int O>
__device__ inline double xor_lane(double v) {
    if constexpr (O == 1 || O == 2) {
        constexpr int ctrl = O == 1 ? 0xB1 : 0x4E;   // quad_perm [1,0,3,2] and [2,3,0,1]
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), ctrl, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)((unsigned long long)b >> 32), ctrl, 0xf, 0xf, false);
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    } else {
        return __shfl_xor(v, O, 64);
    }
}

template <int SUB, int O = 1>
__device__ inline dd group_sum_dd(dd v) {
#pragma clang fp contract(off)
    if constexpr (O < SUB) {
        const dd w = {xor_lane<O>(v.hi), xor_lane<O>(v.lo)};
        return group_sum_dd<SUB, 2 * O>(dd_add(v, w));
    } else {
        return v;
    }
}

template <int SUB, int O = 1>
__device__ inline double group_sum(double v) {
    if constexpr (O < SUB) return group_sum<SUB, 2 * O>(v + xor_lane<O>(v));
    else return v;
}

// One workgroup per box; the SUB adjacent threads 4 q .. 4 q + SUB - 1 own column q and
// split its dot products (every one of them then holds the same values).  The pivot of a
// step is chosen by every wave from the trailing norms in LDS, so that one barrier per
// step suffices.  Rows j < kc of
// R live in LDS (hi and lo parts apart), later rows in the workspace; every thread of a
// column writes the same value to the same entry, so each reads back only what it wrote
// itself or what other columns wrote before a barrier.  nsl_fixed > 0: the slices are
// already summed into slice 0 (nsl_fixed = 1); otherwise every entry is summed over the
// box's slices here.
template <int NTH, int SUB>
__global__ void __launch_bounds__(NTH) k_pchol(const int* __restrict__ cnt, const int* __restrict__ nact,
                                               const int* __restrict__ boxes, int nb, int nmax, KernelParams kp,
                                               const double* __restrict__ gpart, int nslice, int slice_rows,
                                               int nsl_fixed, double* __restrict__ rwork, int kc,
                                               int* __restrict__ krank, int* __restrict__ spos,
                                               int* __restrict__ rpos, double* __restrict__ Tout,
                                               int* __restrict__ mrows) {
#pragma clang fp contract(off)
    constexpr int NW = NTH / 64;
    constexpr int NQ = NTH / SUB;    // columns the workgroup can hold (n <= NQ)
    extern __shared__ double rl[];   // Rh[kc * nmax] | Rl[kc * nmax]
    __shared__ int piv[NQ];
    __shared__ int srank_s[NQ];
    __shared__ double dh[2][NQ], dl[2][NQ];   // trailing norms^2, by step parity
    __shared__ double nuv[2][NQ];             // their sum (-1: column done)
    __shared__ unsigned long long smask[NW];
    const int tid = threadIdx.x;
    const int q = tid / SUB, sub = tid % SUB;
    const int wv = tid >> 6, lane = tid & 63;
    const int c = boxes[blockIdx.x];
    const int n = cnt[c];
    if (n == 0) {
        if (tid == 0) { krank[c] = 0; mrows[c] = 0; }
        return;
    }
    const int m = id_rows(nact, c, nb, kp.n_proxy, kp.weak);
    const int nsl = nsl_fixed > 0 ? nsl_fixed : (m + slice_rows - 1) / slice_rows;
    const int64_t sstride = (int64_t)nmax * nmax;
    const double2* G = (const double2*)gpart + (int64_t)blockIdx.x * nslice * sstride;
    double2* Rg = (double2*)rwork + (int64_t)blockIdx.x * sstride;   // rows >= kc: Rg[j * nmax + q]
    double* Rh = rl;
    double* Rl = rl + (int64_t)kc * nmax;
    auto rget = [&](int j, int col) -> dd {
        if (j < kc) return {Rh[j * nmax + col], Rl[j * nmax + col]};
        const double2 v = Rg[(int64_t)j * nmax + col];
        return {v.x, v.y};
    };
    auto rput = [&](int j, int col, dd v) {
        if (j < kc) {
            Rh[j * nmax + col] = v.hi;
            Rl[j * nmax + col] = v.lo;
        } else {
            Rg[(int64_t)j * nmax + col] = make_double2(v.hi, v.lo);
        }
    };
    auto rhi = [&](int j, int col) -> double { return j < kc ? Rh[j * nmax + col] : Rg[(int64_t)j * nmax + col].x; };
    auto rset_hi = [&](int j, int col, double v) {
        if (j < kc) Rh[j * nmax + col] = v;
        else Rg[(int64_t)j * nmax + col].x = v;
    };
    dd d = {0.0, 0.0};
    if (q < n) d = gram_entry(G, nsl, nmax, sstride, q, q);
    bool done = q >= n;
    const int kmax = min(m, n);
    double rnorm0 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        const int buf = j & 1;
        if (q < n && sub == 0) {
            dh[buf][q] = d.hi;
            dl[buf][q] = d.lo;
            nuv[buf][q] = done ? -1.0 : d.hi + d.lo;
        }
        __syncthreads();
        // largest trailing norm, then the lowest column within tau rnorm0 of it; the lane's
        // norms stay in registers for the second pass
        constexpr int NU = (NQ + 63) / 64;
        double nul[NU];
        double wm = -1.0;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int t = lane + 64 * u;
            nul[u] = t < n ? nuv[buf][t] : -1.0;
            wm = fmax(wm, nul[u]);
        }
        const double numax = wave_max_d(wm);
        const double mu = sqrt(fmax(numax, 0.0));
        if (!(numax == numax)) break;
        if (j == 0) {
            if (!(mu > 0.0)) break;
            rnorm0 = mu;
        } else if (mu <= kp.tol * rnorm0) {
            break;
        }
        // candidates: norm >= thr, compared as nu >= thr^2 (every column when thr <= 0)
        const double thr = mu - kp.tau * rnorm0;
        const double thr2 = thr > 0.0 ? thr * thr : 0.0;
        int p = 1 << 30;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const unsigned long long b = __ballot(nul[u] >= 0.0 && nul[u] >= thr2);
            if (b && p == (1 << 30)) p = 64 * u + __ffsll((long long)b) - 1;
        }
        if (p >= n) break;
        // the pivot row's Gram entry is requested before r_jj is formed, so that its load
        // overlaps the square root and the reciprocal (every thread forms r_jj itself: no
        // extra barrier)
        const bool active = !done && q != p;
        dd gpq = {0.0, 0.0};
        if (active) gpq = gram_entry(G, nsl, nmax, sstride, p, q);
        const dd rjj = dd_sqrt({dh[buf][p], dl[buf][p]});
        if (q == p) {
            if (sub == 0) piv[j] = p;
            rput(j, p, rjj);
            done = true;
        }
        if (active) {
            // r_jq = (G_pq - sum_{i<j} r_ip r_iq) / r_jj ; d_q -= r_jq^2.  Thread sub of the
            // column takes i = sub, sub + SUB, ... in two partial sums.
            const dd rinv = dd_recip(rjj);
            // term t (row i = sub + SUB t) goes to s0 for even t, s1 for odd t, each in
            // increasing t; rows < kc from LDS, then rows >= kc from the workspace, four
            // terms per pass with all their loads issued first
            dd s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
            const int jl = min(j, kc);
            int i = sub;
            for (; i + 3 * SUB < jl; i += 4 * SUB) {
                dd a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = {Rh[(i + u * SUB) * nmax + p], Rl[(i + u * SUB) * nmax + p]};
                    b[u] = {Rh[(i + u * SUB) * nmax + q], Rl[(i + u * SUB) * nmax + q]};
                }
                s0 = dd_add(s0, dd_mul(a[0], b[0]));
                s1 = dd_add(s1, dd_mul(a[1], b[1]));
                s0 = dd_add(s0, dd_mul(a[2], b[2]));
                s1 = dd_add(s1, dd_mul(a[3], b[3]));
            }
            for (; i + SUB < jl; i += 2 * SUB) {
                s0 = dd_add(s0, dd_mul(rget(i, p), rget(i, q)));
                s1 = dd_add(s1, dd_mul(rget(i + SUB, p), rget(i + SUB, q)));
            }
            bool odd = false;   // the next term goes to s1
            if (i < jl) {
                s0 = dd_add(s0, dd_mul(rget(i, p), rget(i, q)));
                i += SUB;
                odd = true;
            }
            if (i < j) {
                if (odd) { const dd t0 = s0; s0 = s1; s1 = t0; }
                for (; i + 3 * SUB < j; i += 4 * SUB) {
                    double2 a[4], b[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a[u] = Rg[(int64_t)(i + u * SUB) * nmax + p];
                        b[u] = Rg[(int64_t)(i + u * SUB) * nmax + q];
                    }
#pragma unroll
                    for (int u = 0; u < 4; u += 2) {
                        s0 = dd_add(s0, dd_mul({a[u].x, a[u].y}, {b[u].x, b[u].y}));
                        s1 = dd_add(s1, dd_mul({a[u + 1].x, a[u + 1].y}, {b[u + 1].x, b[u + 1].y}));
                    }
                }
                for (; i + SUB < j; i += 2 * SUB) {
                    s0 = dd_add(s0, dd_mul(rget(i, p), rget(i, q)));
                    s1 = dd_add(s1, dd_mul(rget(i + SUB, p), rget(i + SUB, q)));
                }
                if (i < j) s0 = dd_add(s0, dd_mul(rget(i, p), rget(i, q)));
                if (odd) { const dd t0 = s0; s0 = s1; s1 = t0; }
            }
            const dd sum = group_sum_dd<SUB>(dd_add(s0, s1));
            const dd rjq = dd_mul(dd_sub(gpq, sum), rinv);
            rput(j, q, rjq);
            d = dd_sub(d, dd_mul(rjq, rjq));
        }
        k = j + 1;
    }

    // ---- sorted sets and T = R11^{-1} R12 (FP64 back substitution) ----------------------
    __syncthreads();
    const bool isS = (q < n) && done;
    const unsigned long long mask = __ballot(isS && sub == 0);
    if (lane == 0) smask[wv] = mask;
    __syncthreads();
    int below = 0;
    for (int w = 0; w < wv; ++w) below += __popcll(smask[w]);
    const int srank = below + __popcll(mask & ((1ull << lane) - 1ull));
    if (isS && sub == 0) srank_s[q] = srank;
    __syncthreads();
    if (tid == 0) { krank[c] = k; mrows[c] = m; }
    const int64_t boff = (int64_t)c * nmax;
    double* Tb = Tout + (int64_t)c * nmax * nmax;
    if (q < n) {
        if (isS) {
            if (sub == 0) spos[boff + srank] = q;
        } else {
            const int rr = q - srank;
            if (sub == 0) rpos[boff + rr] = q;
            // in place in column q of R: R[a][q] <- t_a, last row first; the sum over b is
            // split over the column's threads
            for (int a = k - 1; a >= 0; --a) {
                double part = 0.0;
                int b = a + 1 + sub;
                if (a < kc) {
                    // rows a and b in LDS: four terms per pass, their loads issued first
                    const double* ra = Rh + (int64_t)a * nmax;
                    const int bl = min(k, kc);
                    for (; b + 3 * SUB < bl; b += 4 * SUB) {
                        int pb[4];
                        double xa[4], yb[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            pb[u] = piv[b + u * SUB];
                            yb[u] = Rh[(int64_t)(b + u * SUB) * nmax + q];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) xa[u] = ra[pb[u]];
#pragma unroll
                        for (int u = 0; u < 4; ++u) part += xa[u] * yb[u];
                    }
                }
                for (; b < k; b += SUB) part += rhi(a, piv[b]) * rhi(b, q);
                const double acc = rhi(a, q) - group_sum<SUB>(part);
                rset_hi(a, q, acc / rhi(a, piv[a]));
            }
            for (int a = sub; a < k; a += SUB) Tb[srank_s[piv[a]] + (int64_t)rr * nmax] = rhi(a, q);
        }
    }
}

template <int NTH, int TPT>
static void gram_launch(const Level& L, const int* boxes, int nboxes, const double* pts, const double* ptmpl,
                        const KernelParams& kp, double* gpart, const GramPlan& g, size_t lds, hipStream_t s) {
    const dim3 grid(g.nsl * g.groups, nboxes);
    note_shape("gram_" + std::to_string(NTH) + "x" + std::to_string(TPT) + "_rows" + std::to_string(g.slice_rows));
    // the chunk exceeds the default 64 KB of dynamic LDS only for nmax > 254
    if (L.store32)
        hipFuncSetAttribute((const void*)k_gram<NTH, TPT, float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    else
        hipFuncSetAttribute((const void*)k_gram<NTH, TPT, double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (L.store32)
        k_gram<NTH, TPT, float><<<grid, dim3(NTH), lds, s>>>((const float*)L.store, L.nb, L.nmax, L.cnt, L.gidx,
                                                              L.nact, L.apos, boxes, pts, ptmpl, kp, L.t, gpart,
                                                              g.nsl, g.slice_rows);
    else
        k_gram<NTH, TPT, double><<<grid, dim3(NTH), lds, s>>>((const double*)L.store, L.nb, L.nmax, L.cnt, L.gidx,
                                                               L.nact, L.apos, boxes, pts, ptmpl, kp, L.t, gpart,
                                                               g.nsl, g.slice_rows);
}

template <int NW>
static void gram_i8_launch(const Level& L, const int* boxes, int nboxes, const double* pts, const double* ptmpl,
                           const KernelParams& kp, double* gpart, const GramPlan& g, int* flag, hipStream_t s) {
    const int npad = (L.nmax + 15) & ~15;
    const size_t lds = std::max((size_t)kI8L * npad * kI8Pitch, sizeof(double) * kMaxProxy * npad);
    note_shape("gram_i8_w" + std::to_string(NW) + "_rows" + std::to_string(g.slice_rows));
    k_gram_i8<NW><<<dim3(g.nsl, nboxes), dim3(64 * NW), lds, s>>>((const float*)L.store, L.nb, L.nmax, L.cnt, L.gidx,
                                                                   L.nact, L.apos, boxes, pts, ptmpl, kp, L.t, gpart,
                                                                   g.nsl, g.slice_rows, flag);
}

template <int NTH, int SUB>
static void pchol_launch(const Level& L, const int* boxes, int nboxes, const KernelParams& kp, double* gpart,
                         const GramPlan& g, int nsl_fixed, double* rwork, hipStream_t s) {
    // many boxes: the first 16 rows of R in LDS (16 KB at nmax 64 keeps ~10 workgroups per
    // CU; measured 0.4 ms faster per leaf level than none), later rows in the workspace
    const PlanParams pp = plan_params(nboxes);
    const int kc = pp.pchol_kc > 0 ? std::min(pp.pchol_kc, L.nmax) : pchol_lds_rows(L.nmax);
    const size_t lds = sizeof(double) * 2 * (size_t)kc * L.nmax;
    note_shape("pchol_" + std::to_string(NTH) + "x" + std::to_string(SUB) + "_kc" + std::to_string(kc));
    k_pchol<NTH, SUB><<<dim3(nboxes), dim3(NTH), lds, s>>>(L.cnt, L.nact, boxes, L.nb, L.nmax, kp, gpart, g.nsl,
                                                          g.slice_rows, nsl_fixed, rwork, kc, L.krank, L.spos,
                                                          L.rpos, L.T, L.mrows);
}

int launch_id_gram(const Level& L, const int* boxes, int nboxes, const double* pts, const double* ptmpl,
                   const KernelParams& kp, double* work, int* flag, hipStream_t s) {
    if (nboxes <= 0) return 0;
    const GramPlan g = gram_plan(L.nmax, kp.n_proxy, nboxes, kp.weak, L.store32);
    const size_t nn = (size_t)L.nmax * L.nmax;
    double* gpart = work;
    double* rwork = work + (size_t)nboxes * g.nsl * nn * 2;
    const size_t lds = sizeof(double) * (size_t)kChunk * (L.nmax + 2);
    int launches = 2;
    if (g.i8) {
        if (g.nth == 256) gram_i8_launch<4>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, flag, s);
        else gram_i8_launch<8>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, flag, s);
    } else if (g.tpt == 1) gram_launch<256, 1>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, lds, s);
    else if (g.tpt == 3 && g.nth == 192) gram_launch<192, 3>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, lds, s);
    else if (g.tpt == 3) gram_launch<256, 3>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, lds, s);
    else if (g.tpt == 5 && g.nth == 192) gram_launch<192, 5>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, lds, s);
    else if (g.tpt == 5) gram_launch<256, 5>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, lds, s);
    else if (g.nth == 192) gram_launch<192, 9>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, lds, s);
    else gram_launch<256, 9>(L, boxes, nboxes, pts, ptmpl, kp, gpart, g, lds, s);
    int nsl_fixed = 0;
    // few-box colours sum the slices once before the pivoted Cholesky (its steps are the
    // critical path; the many-box form sums each entry as it reads it)
    if (g.groups > 1 || g.slice_rows < 256 || (g.i8 && !plan_params(nboxes).gram_many)) {
        k_gram_reduce<<<dim3((unsigned)((nn + 255) / 256), nboxes), dim3(256), 0, s>>>(
            L.cnt, L.nact, boxes, L.nb, L.nmax, kp.n_proxy, kp.weak, gpart, g.nsl, g.slice_rows);
        nsl_fixed = 1;
        ++launches;
        note_shape("gram_reduce");
    }
    // many boxes: one thread per column; few boxes: four threads per column
    if (plan_params(nboxes).gram_many) {
        if (L.nmax <= 64) pchol_launch<64, 1>(L, boxes, nboxes, kp, gpart, g, nsl_fixed, rwork, s);
        else if (L.nmax <= 128) pchol_launch<128, 1>(L, boxes, nboxes, kp, gpart, g, nsl_fixed, rwork, s);
        else pchol_launch<256, 1>(L, boxes, nboxes, kp, gpart, g, nsl_fixed, rwork, s);
    } else {
        if (L.nmax <= 64) pchol_launch<256, 4>(L, boxes, nboxes, kp, gpart, g, nsl_fixed, rwork, s);
        else if (L.nmax <= 128) pchol_launch<512, 4>(L, boxes, nboxes, kp, gpart, g, nsl_fixed, rwork, s);
        else pchol_launch<1024, 4>(L, boxes, nboxes, kp, gpart, g, nsl_fixed, rwork, s);
    }
    return launches;
}

}  // namespace rss
