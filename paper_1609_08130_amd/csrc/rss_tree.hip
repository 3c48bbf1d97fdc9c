// Uniform quadtree, block store generation, level transition and top-block assembly.
//
// Tree (Section 3, Figure 2): the root box is refined uniformly; a point at depth t
// lies in box (floor((x - lo) * 2^t / side), floor((y - lo) * 2^t / side)), clamped,
// with linear index bx + 2^t * by.  DOFs inside a box are kept in ascending global
// index.  The block store of a level holds A(B_a, B_b) for every ordered pair of boxes
// at Chebyshev distance <= 2; pairs further apart are never modified (Theorem 1,
// Corollary 1) and are evaluated from the kernel when needed.
#include <climits>

#include "rss_internal.h"

namespace rss {

__device__ inline double kernel_entry(double xi, double yi, double xj, double yj, double coef) {
#pragma clang fp contract(off)
    double dx = xi - xj;
    double dy = yi - yj;
    return coef * log(dx * dx + dy * dy);
}

// log x (x > 0) to ~1.3e-12 relative: x = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// log m = 2 atanh(t), t = (m - 1) / (m + 1), |t| <= 0.172, by the odd series of atanh up to
// t^13 (the first omitted term is below 5e-13).  Used for entries stored in FP32, whose
// rounding (3e-8 relative) it leaves unchanged in all but rare ties; about a third of the
// cost of the full-precision FP64 logarithm, which bounds the store kernels.
__device__ inline double log_for_f32(double x) {
    int e;
    double m = frexp(x, &e);   // m in [1/2, 1)
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double t = (m - 1.0) / (m + 1.0);
    const double t2 = t * t;
    double p = 1.0 / 13.0;
    p = fma(p, t2, 1.0 / 11.0);
    p = fma(p, t2, 1.0 / 9.0);
    p = fma(p, t2, 1.0 / 7.0);
    p = fma(p, t2, 1.0 / 5.0);
    p = fma(p, t2, 1.0 / 3.0);
    p = fma(p, t2, 1.0);
    return fma((double)e, 0.69314718055994531, 2.0 * t * p);
}

// A store entry w K(x_i - x_j) in the store's type: FP64 entries take the full-precision
// logarithm, FP32 entries the series above.
template <typename ST>
__device__ inline double store_entry(double xi, double yi, double xj, double yj, double coef) {
    if constexpr (sizeof(ST) == 8) {
        return kernel_entry(xi, yi, xj, yj, coef);
    } else {
#pragma clang fp contract(off)
        const double dx = xi - xj;
        const double dy = yi - yj;
        return coef * log_for_f32(dx * dx + dy * dy);
    }
}

__device__ inline void box_coord(double x, double y, double lo_x, double lo_y, double s, int nb,
                                 int& cx, int& cy) {
#pragma clang fp contract(off)
    double fx = floor((x - lo_x) * s);
    double fy = floor((y - lo_y) * s);
    cx = fx < 0 ? 0 : (fx > nb - 1 ? nb - 1 : (int)fx);
    cy = fy < 0 ? 0 : (fy > nb - 1 ? nb - 1 : (int)fy);
}

// ------------------------------------------------------------------------------------
__global__ void k_validate_points(const double* __restrict__ pts, int64_t n, double lo_x, double lo_y,
                                  double side, int* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = pts[2 * i], y = pts[2 * i + 1];
    bool ok = isfinite(x) && isfinite(y) && x >= lo_x && y >= lo_y && x <= lo_x + side && y <= lo_y + side;
    if (!ok) atomicOr(flag, 1);
}

void launch_validate_points(const double* pts, int64_t n, double lo_x, double lo_y, double side,
                            int* flag, hipStream_t s) {
    int64_t nb = (n + 255) / 256;
    k_validate_points<<<dim3((unsigned)nb), dim3(256), 0, s>>>(pts, n, lo_x, lo_y, side, flag);
}

// counts[box] += 1 for every point; counts[nbox] = max count (atomicMax)
// Runs of equal boxes among the lanes of a wave (consecutive points mostly share a box):
// bit l of the result is set when lane l starts a run.  Lanes past the end carry box -1.
__device__ inline unsigned long long run_heads(int b) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(b, 1, 64);
    return __ballot(lane == 0 || prev != b);
}

// Length of the run that lane `lane` starts (heads: run_heads).
__device__ inline int run_length(unsigned long long heads, int lane) {
    const unsigned long long later = lane == 63 ? 0ull : heads >> (lane + 1);
    return later ? __ffsll((long long)later) : 64 - lane;
}

__global__ void k_count_boxes(const double* __restrict__ pts, int64_t n, int nb, double lo_x, double lo_y,
                              double s, int* counts) {
    // one atomic per run of equal boxes in a wave instead of one per point
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int b = -1;
    if (i < n) {
        int cx, cy;
        box_coord(pts[2 * i], pts[2 * i + 1], lo_x, lo_y, s, nb, cx, cy);
        b = cx + nb * cy;
    }
    const unsigned long long heads = run_heads(b);
    if (b >= 0 && ((heads >> lane) & 1ull)) atomicAdd(&counts[b], run_length(heads, lane));
}

__global__ void k_max_count(const int* __restrict__ counts, int64_t nbox, int* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = i < nbox ? counts[i] : 0;
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, v);
}

void launch_count_boxes(const double* pts, int64_t n, int t, double lo_x, double lo_y, double side,
                        int* counts, hipStream_t s) {
    int nb = 1 << t;
    int64_t nbox = (int64_t)nb * nb;
    double sc = ldexp(1.0, t) / side;
    hipMemsetAsync(counts, 0, sizeof(int) * (nbox + 1), s);
    k_count_boxes<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(pts, n, nb, lo_x, lo_y, sc, counts);
    k_max_count<<<dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, s>>>(counts, nbox, counts + nbox);
}

__global__ void k_leaf_scatter(const double* __restrict__ pts, int64_t n, int nb, double lo_x, double lo_y,
                               double s, int* fill, int* gidx, int nmax) {
    // the head of each run of equal boxes reserves the run's slots with one atomic; the
    // order inside a box is made ascending afterwards (k_leaf_sort)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int b = -1;
    if (i < n) {
        int cx, cy;
        box_coord(pts[2 * i], pts[2 * i + 1], lo_x, lo_y, s, nb, cx, cy);
        b = cx + nb * cy;
    }
    const unsigned long long heads = run_heads(b);
    const bool head = (heads >> lane) & 1ull;
    int base = 0;
    if (b >= 0 && head) base = atomicAdd(&fill[b], run_length(heads, lane));
    const int h = 63 - __clzll((long long)(heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull))));
    base = __shfl(base, h, 64);
    if (b >= 0) gidx[(int64_t)b * nmax + base + (lane - h)] = (int)i;
}

// Sort each box's DOF list ascending (rank sort in LDS); fill[] holds the counts.
__global__ void k_leaf_sort(const int* __restrict__ fill, int* gidx, int nmax) {
    __shared__ int v[kMaxBox];
    int b = blockIdx.x;
    int c = fill[b];
    int64_t base = (int64_t)b * nmax;
    for (int i = threadIdx.x; i < c; i += blockDim.x) v[i] = gidx[base + i];
    __syncthreads();
    for (int i = threadIdx.x; i < c; i += blockDim.x) {
        int x = v[i], r = 0;
        for (int j = 0; j < c; ++j) r += v[j] < x;
        gidx[base + r] = x;
    }
}

void launch_leaf_lists(const double* pts, int64_t n, int t, double lo_x, double lo_y, double side,
                       int* fill, int* gidx, int nmax, int nbox, hipStream_t s) {
    int nb = 1 << t;
    double sc = ldexp(1.0, t) / side;
    hipMemsetAsync(fill, 0, sizeof(int) * nbox, s);
    k_leaf_scatter<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(pts, n, nb, lo_x, lo_y, sc, fill,
                                                                            gidx, nmax);
    k_leaf_sort<<<dim3(nbox), dim3(256), 0, s>>>(fill, gidx, nmax);
}

// ------------------------------------------------------------------------------------
// Leaf store: A(B_a, B_b) = diag on coincident DOFs, w K(x_i - x_j) otherwise.
// One block per (box a, neighbour slot).  flag |= 2 on duplicate points.
// The kernel is symmetric (K(x - y) = K(y - x), exactly in floating point since the
// differences only change sign), so A(B_b, B_a) = A(B_a, B_b)^T: one workgroup per box a
// and per offset of the self block or the 12 offsets (dx, dy) with dy > 0 or (dy = 0,
// dx > 0).  Each 64 x 64 tile is evaluated once into LDS and written to both blocks,
// coalesced in both orientations.
template <typename ST>
__global__ void __launch_bounds__(256) k_leaf_store(ST* __restrict__ store, double* __restrict__ dstore,
                                                    const int* __restrict__ cnt, const int* __restrict__ gidx,
                                                    const double* __restrict__ pts, int nb, int nmax, double coef,
                                                    double diag, int* flag) {
    // the row point of a thread comes from registers, the column points (the same for the
    // whole wave) from LDS; the transposing tile holds entries in the store's type
    __shared__ double xb[kMaxBox], yb[kMaxBox];
    __shared__ int gb[kMaxBox];
    __shared__ ST tile[64][65];
    const int a = blockIdx.x / 13, oi = blockIdx.x % 13;
    // oi = 0: self; oi = 1..12: the offsets after (0, 0) in row-major order of the 5x5 window
    const int o = 12 + oi;
    const int dx = o % 5 - 2, dy = o / 5 - 2;
    const int ax = a % nb, ay = a / nb;
    const int bx = ax + dx, by = ay + dy;
    if (bx < 0 || by < 0 || bx >= nb || by >= nb) return;
    const int b = bx + nb * by;
    const int na = cnt[a], nbb = cnt[b];
    for (int i = threadIdx.x; i < nbb; i += blockDim.x) {
        int g = gidx[(int64_t)b * nmax + i];
        gb[i] = g; xb[i] = pts[2 * (int64_t)g]; yb[i] = pts[2 * (int64_t)g + 1];
    }
    __syncthreads();
    ST* blk_ab = store + ((int64_t)a * kNbr + o) * nmax * nmax;                  // A(B_a, B_b)
    ST* blk_ba = store + ((int64_t)b * kNbr + (24 - o)) * nmax * nmax;           // A(B_b, B_a)
    const bool self = oi == 0;
    // self block of an FP32 store: full-precision FP64 entries in the separate array
    double* dblk = (self && dstore) ? dstore + (int64_t)a * nmax * nmax : nullptr;
    bool dup = false;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i0 = 0; i0 < na; i0 += 64) {
        const int ti = min(64, na - i0);
        int gi = -1;
        double xi = 0.0, yi = 0.0;
        if (lane < ti) {
            gi = gidx[(int64_t)a * nmax + i0 + lane];
            xi = pts[2 * (int64_t)gi];
            yi = pts[2 * (int64_t)gi + 1];
        }
        for (int j0 = 0; j0 < nbb; j0 += 64) {
            const int tj = min(64, nbb - j0);
            // rows i0 + lane, columns j0 + wv + 4 t
            for (int jj = wv; jj < tj; jj += 4) {
                const int j = j0 + jj;
                ST v = (ST)0;
                if (lane < ti) {
                    const int i = i0 + lane;
                    if (dblk) {
                        dblk[i + (int64_t)j * nmax] = gi == gb[j] ? diag : kernel_entry(xi, yi, xb[j], yb[j], coef);
                        dup |= gi != gb[j] && (xi == xb[j] && yi == yb[j]);
                    } else {
                        if (gi == gb[j]) {
                            v = (ST)diag;
                        } else {
                            v = (ST)store_entry<ST>(xi, yi, xb[j], yb[j], coef);
                            dup |= (xi == xb[j] && yi == yb[j]);
                        }
                        blk_ab[i + (int64_t)j * nmax] = v;
                    }
                }
                tile[jj][lane] = v;
            }
            if (!self) {
                __syncthreads();
                // A(B_b, B_a)(j, i) = A(B_a, B_b)(i, j): rows j0 + lane, columns i0 + wv + 4 t
                for (int ii = wv; ii < ti; ii += 4)
                    if (lane < tj) blk_ba[(j0 + lane) + (int64_t)(i0 + ii) * nmax] = tile[lane][ii];
                __syncthreads();
            }
        }
    }
    if (dup) atomicOr(flag, 2);
}

void launch_leaf_store(const Level& L, const double* pts, const KernelParams& kp, int* flag, hipStream_t s) {
    if (L.store32)
        k_leaf_store<float><<<dim3(L.nbox * 13), dim3(256), 0, s>>>((float*)L.store, L.dstore, L.cnt, L.gidx, pts,
                                                                    L.nb, L.nmax, kp.coef, kp.diag, flag);
    else
        k_leaf_store<double><<<dim3(L.nbox * 13), dim3(256), 0, s>>>((double*)L.store, nullptr, L.cnt, L.gidx, pts,
                                                                     L.nb, L.nmax, kp.coef, kp.diag, flag);
}

// ------------------------------------------------------------------------------------
// Level transition (Section 3.3, subsequent levels): B_P = union of the children's
// active DOFs, ascending.  pmap[P*nmaxP + p] = (child slot << 16) | position of the DOF
// in the child's level-start list (the child store is indexed by those positions).

__global__ void __launch_bounds__(256) k_parent_lists(const int* __restrict__ cnact, const int* __restrict__ capos,
                                                      const int* __restrict__ cgidx, int cnb, int cnmax,
                                                      int* __restrict__ pgidx, int* __restrict__ pmap, int pnb,
                                                      int pnmax) {
    __shared__ int vals[4][kMaxBox];
    __shared__ int posn[4][kMaxBox];
    __shared__ int len[4];
    int P = blockIdx.x;
    int px = P % pnb, py = P / pnb;
    if (threadIdx.x < 4) {
        int ix = threadIdx.x & 1, iy = threadIdx.x >> 1;
        len[threadIdx.x] = cnact[(2 * px + ix) + cnb * (2 * py + iy)];
    }
    __syncthreads();
    for (int c = 0; c < 4; ++c) {
        int ch = (2 * px + (c & 1)) + cnb * (2 * py + (c >> 1));
        for (int i = threadIdx.x; i < len[c]; i += blockDim.x) {
            int p = capos[(int64_t)ch * cnmax + i];
            posn[c][i] = p;
            vals[c][i] = cgidx[(int64_t)ch * cnmax + p];
        }
    }
    __syncthreads();
    for (int c = 0; c < 4; ++c) {
        for (int i = threadIdx.x; i < len[c]; i += blockDim.x) {
            int g = vals[c][i];
            int rank = i;
            for (int c2 = 0; c2 < 4; ++c2) {
                if (c2 == c) continue;
                int lo = 0, hi = len[c2];
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (vals[c2][mid] < g) lo = mid + 1; else hi = mid;
                }
                rank += lo;
            }
            pgidx[(int64_t)P * pnmax + rank] = g;
            pmap[(int64_t)P * pnmax + rank] = (c << 16) | posn[c][i];
        }
    }
}

void launch_parent_lists(const Level& C, Level& P, int* pmap, hipStream_t s) {
    k_parent_lists<<<dim3(P.nbox), dim3(256), 0, s>>>(C.nact, C.apos, C.gidx, C.nb, C.nmax, P.gidx, pmap, P.nb,
                                                      P.nmax);
}


template <typename ST>
__global__ void __launch_bounds__(256) k_parent_store(const ST* __restrict__ cstore,
                                                      const double* __restrict__ cdstore, int cnb, int cnmax,
                                                      ST* __restrict__ pstore, double* __restrict__ pdstore,
                                                      const int* __restrict__ pcnt,
                                                      const int* __restrict__ pgidx, const int* __restrict__ pmap,
                                                      int pnb, int pnmax, const double* __restrict__ pts,
                                                      double coef) {
    __shared__ int mp[kMaxBox], mq[kMaxBox];
    __shared__ double xp[kMaxBox], yp[kMaxBox], xq[kMaxBox], yq[kMaxBox];
    __shared__ ST tile[64][65];
    const int tid = threadIdx.x;
    const int P = blockIdx.x / kNbr, o = blockIdx.x % kNbr;
    const int dx = o % 5 - 2, dy = o / 5 - 2;
    // Parent offsets with |dx| = 2 or |dy| = 2: every child pair is at distance >= 3, so the
    // whole block is kernel entries, and A(B_Q, B_P) is its transpose bit for bit; the
    // workgroup of the upper offset writes both, the lower one has nothing to do.
    const bool far_only = abs(dx) == 2 || abs(dy) == 2;
    if (far_only && o < 12) return;
    const int Px = P % pnb, Py = P / pnb;
    const int Qx = Px + dx, Qy = Py + dy;
    if (Qx < 0 || Qy < 0 || Qx >= pnb || Qy >= pnb) return;
    const int Q = Qx + pnb * Qy;
    const int np = pcnt[P], nq = pcnt[Q];
    for (int i = tid; i < np; i += blockDim.x) {
        mp[i] = pmap[(int64_t)P * pnmax + i];
        int g = pgidx[(int64_t)P * pnmax + i];
        xp[i] = pts[2 * (int64_t)g]; yp[i] = pts[2 * (int64_t)g + 1];
    }
    for (int i = tid; i < nq; i += blockDim.x) {
        mq[i] = pmap[(int64_t)Q * pnmax + i];
        int g = pgidx[(int64_t)Q * pnmax + i];
        xq[i] = pts[2 * (int64_t)g]; yq[i] = pts[2 * (int64_t)g + 1];
    }
    __syncthreads();
    ST* blk = pstore + ((int64_t)P * kNbr + o) * pnmax * pnmax;
    if (far_only) {
        ST* blk_t = pstore + ((int64_t)Q * kNbr + (24 - o)) * pnmax * pnmax;
        const int lane = tid & 63, wv = tid >> 6;
        for (int i0 = 0; i0 < np; i0 += 64)
            for (int j0 = 0; j0 < nq; j0 += 64) {
                const int ti = min(64, np - i0), tj = min(64, nq - j0);
                // rows i0 + lane, columns j0 + wv + 4 t; the tile goes out transposed
                for (int jj = wv; jj < tj; jj += 4) {
                    ST v = (ST)0;
                    if (lane < ti) {
                        v = (ST)store_entry<ST>(xp[i0 + lane], yp[i0 + lane], xq[j0 + jj], yq[j0 + jj], coef);
                        blk[(i0 + lane) + (int64_t)(j0 + jj) * pnmax] = v;
                    }
                    tile[jj][lane] = v;
                }
                __syncthreads();
                for (int ii = wv; ii < ti; ii += 4)
                    if (lane < tj) blk_t[(j0 + lane) + (int64_t)(i0 + ii) * pnmax] = tile[lane][ii];
                __syncthreads();
            }
        return;
    }
    // the parent's self block goes to the FP64 array when there is one (its child pairs are
    // within distance 1: the children's self blocks come from their FP64 array)
    double* dblk = (o == 12 && pdstore) ? pdstore + (int64_t)P * pnmax * pnmax : nullptr;
    // Adjacent parents: child pairs within distance 2 copy their entry of the child store,
    // the others (distance 3) are kernel entries.  Element e = i + np j, taken U at a time
    // per thread with every load issued before the first store; (i, j) advance by a fixed
    // step instead of a division per element.
    constexpr int U = 4;
    const int tot = np * nq;
    if (tot == 0) return;
    const int di = 256 % np, dj = 256 / np;
    int i = tid % np, j = tid / np;
    for (int e0 = tid; e0 < tot; e0 += 256 * U) {
        double v[U];
        int iu[U], ju[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            iu[u] = i;
            ju[u] = j;
            i += di;
            j += dj;
            if (i >= np) { i -= np; ++j; }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = 0.0;
            if (e0 + 256 * u >= tot) continue;
            const int ii = iu[u], jj = ju[u];
            const int sa = mp[ii] >> 16, pa = mp[ii] & 0xffff;
            const int sb = mq[jj] >> 16, qb = mq[jj] & 0xffff;
            const int ax = 2 * Px + (sa & 1), ay = 2 * Py + (sa >> 1);
            const int bx = 2 * Qx + (sb & 1), by = 2 * Qy + (sb >> 1);
            const int ddx = bx - ax, ddy = by - ay;
            if (cdstore && ddx == 0 && ddy == 0) {
                v[u] = cdstore[(int64_t)(ax + cnb * ay) * cnmax * cnmax + pa + (int64_t)qb * cnmax];
            } else if (ddx >= -2 && ddx <= 2 && ddy >= -2 && ddy <= 2) {
                const ST* cb = cstore + ((int64_t)(ax + cnb * ay) * kNbr + nbr_slot(ddx, ddy)) * cnmax * cnmax;
                v[u] = (double)cb[pa + (int64_t)qb * cnmax];
            } else {
                v[u] = store_entry<ST>(xp[ii], yp[ii], xq[jj], yq[jj], coef);
            }
        }
        if (dblk) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e0 + 256 * u < tot) dblk[iu[u] + (int64_t)ju[u] * pnmax] = v[u];
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e0 + 256 * u < tot) blk[iu[u] + (int64_t)ju[u] * pnmax] = (ST)v[u];
        }
    }
}

void launch_parent_store(const Level& C, const Level& P, const int* pmap, const double* pts,
                         const KernelParams& kp, hipStream_t s) {
    if (C.store32)
        k_parent_store<float><<<dim3(P.nbox * kNbr), dim3(256), 0, s>>>(
            (const float*)C.store, C.dstore, C.nb, C.nmax, (float*)P.store, P.dstore, P.cnt, P.gidx, pmap, P.nb,
            P.nmax, pts, kp.coef);
    else
        k_parent_store<double><<<dim3(P.nbox * kNbr), dim3(256), 0, s>>>(
            (const double*)C.store, nullptr, C.nb, C.nmax, (double*)P.store, nullptr, P.cnt, P.gidx, pmap, P.nb,
            P.nmax, pts, kp.coef);
}

__global__ void k_level_sizes(const int* __restrict__ nact, int nb, int group, int* __restrict__ pc,
                              int* __restrict__ out) {
    const int pnb = nb / group;
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    int v = 0;
    if (P < pnb * pnb) {
        const int px = P % pnb, py = P / pnb;
        for (int iy = 0; iy < group; ++iy)
            for (int ix = 0; ix < group; ++ix) v += nact[(group * px + ix) + nb * (group * py + iy)];
        if (pc) pc[P] = v;
    }
    int mx = v, sm = v;
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(out, mx);
        atomicAdd(out + 1, sm);
    }
}

void launch_level_sizes(const int* nact, int nb, int group, int* pc, int* out, hipStream_t s) {
    const int pn = (nb / group) * (nb / group);
    k_level_sizes<<<dim3((unsigned)((pn + 255) / 256)), dim3(256), 0, s>>>(nact, nb, group, pc, out);
}

// ------------------------------------------------------------------------------------
// RS-WS (Section 3.4): after the weak pass of a level the strong pass restarts on the DOFs
// that remain active.  Box P's new list is its active DOFs in ascending order,
// list'(P)[i] = list(P)[apos(P)[i]], and every stored block is restricted to the active
// rows and columns (the self blocks from and to the FP64 arrays when there are some).

__global__ void k_compact_lists(const int* __restrict__ nact, const int* __restrict__ apos,
                                const int* __restrict__ gidx, int nmax, int* __restrict__ cgidx, int cnmax) {
    const int P = blockIdx.x;
    const int n = nact[P];
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        cgidx[(int64_t)P * cnmax + i] = gidx[(int64_t)P * nmax + apos[(int64_t)P * nmax + i]];
}

template <typename ST>
__global__ void __launch_bounds__(256) k_compact_store(const ST* __restrict__ st, const double* __restrict__ ds,
                                                       int nb, int nmax, const int* __restrict__ nact,
                                                       const int* __restrict__ apos, ST* __restrict__ cst,
                                                       double* __restrict__ cds, int cnmax) {
    __shared__ int ap[kMaxBox], aq[kMaxBox];
    const int P = blockIdx.x / kNbr, o = blockIdx.x % kNbr;
    const int dx = o % 5 - 2, dy = o / 5 - 2;
    const int Qx = P % nb + dx, Qy = P / nb + dy;
    if (Qx < 0 || Qy < 0 || Qx >= nb || Qy >= nb) return;
    const int Q = Qx + nb * Qy;
    const int np = nact[P], nq = nact[Q];
    for (int i = threadIdx.x; i < np; i += 256) ap[i] = apos[(int64_t)P * nmax + i];
    for (int i = threadIdx.x; i < nq; i += 256) aq[i] = apos[(int64_t)Q * nmax + i];
    __syncthreads();
    const int64_t bsz = (int64_t)nmax * nmax, cbsz = (int64_t)cnmax * cnmax;
    const bool self = o == 12 && ds;
    const ST* src = st + ((int64_t)P * kNbr + o) * bsz;
    const double* dsrc = self ? ds + (int64_t)P * bsz : nullptr;
    ST* dst = cst + ((int64_t)P * kNbr + o) * cbsz;
    double* ddst = self ? cds + (int64_t)P * cbsz : nullptr;
    for (int e = threadIdx.x; e < np * nq; e += 256) {
        const int i = e % np, j = e / np;
        const int64_t from = ap[i] + (int64_t)aq[j] * nmax, to = i + (int64_t)j * cnmax;
        if (self) ddst[to] = dsrc[from];
        else dst[to] = src[from];
    }
}

void launch_compact(const Level& L, Level& C, hipStream_t s) {
    k_compact_lists<<<dim3(L.nbox), dim3(256), 0, s>>>(L.nact, L.apos, L.gidx, L.nmax, C.gidx, C.nmax);
    if (L.store32)
        k_compact_store<float><<<dim3(L.nbox * kNbr), dim3(256), 0, s>>>(
            (const float*)L.store, L.dstore, L.nb, L.nmax, L.nact, L.apos, (float*)C.store, C.dstore, C.nmax);
    else
        k_compact_store<double><<<dim3(L.nbox * kNbr), dim3(256), 0, s>>>(
            (const double*)L.store, nullptr, L.nb, L.nmax, L.nact, L.apos, (double*)C.store, nullptr, C.nmax);
}

// ------------------------------------------------------------------------------------
// Top block (Section 3.3, final factorization): the remaining active DOFs of the last
// level, ascending; tmap[p] = (box << 8) | position in the box's level-start list (as
// unsigned: positions < kMaxBox = 256, boxes < 2^24).
static_assert(kMaxBox <= 256, "top map packs a box position into 8 bits");

__global__ void __launch_bounds__(1024) k_top_lists(const int* __restrict__ nact, const int* __restrict__ apos,
                                                   const int* __restrict__ gidx, int nbox, int nmax, int* top_idx,
                                                   int* tmap) {
    // one block; nbox <= 16 boxes of <= kMaxBox DOFs.  The boxes' active global indices
    // (ascending in each box) and positions are staged in LDS first, so the rank searches
    // below read no global memory.
    __shared__ int ag[16 * kMaxBox], ap[16 * kMaxBox];
    __shared__ int off[17];
    if (threadIdx.x == 0) {
        off[0] = 0;
        for (int b = 0; b < nbox; ++b) off[b + 1] = off[b] + nact[b];
    }
    __syncthreads();
    const int tot = off[nbox];
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        int b = 0;
        while (off[b + 1] <= e) ++b;
        const int p = apos[(int64_t)b * nmax + (e - off[b])];
        ap[e] = p;
        ag[e] = gidx[(int64_t)b * nmax + p];
    }
    __syncthreads();
    // rank of entry e of box b: its place in b plus, in every other box, the number of
    // indices below its own (a binary search)
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        int b = 0;
        while (off[b + 1] <= e) ++b;
        const int g = ag[e];
        int rank = e - off[b];
        for (int c = 0; c < nbox; ++c) {
            if (c == b) continue;
            int lo = off[c], hi = off[c + 1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ag[mid] < g) lo = mid + 1; else hi = mid;
            }
            rank += lo - off[c];
        }
        top_idx[rank] = g;
        tmap[rank] = (int)(((unsigned)b << 8) | (unsigned)ap[e]);
    }
}

// Any number of boxes (a recursion that ended above depth 2): the active entries are first
// gathered in box order (one workgroup, a scan of the per-box counts), then each entry's
// rank is the number of entries with a smaller global index.
__global__ void __launch_bounds__(1024) k_top_gather(const int* __restrict__ nact, const int* __restrict__ apos,
                                                    const int* __restrict__ gidx, int nbox, int nmax,
                                                    int* __restrict__ eg, int* __restrict__ etm) {
    __shared__ int sc[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nbox; b0 += 1024) {
        const int b = b0 + (int)threadIdx.x;
        const int c = b < nbox ? nact[b] : 0;
        sc[threadIdx.x] = c;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {   // inclusive scan (Hillis-Steele)
            const int v = threadIdx.x >= (unsigned)d ? sc[threadIdx.x - d] : 0;
            __syncthreads();
            sc[threadIdx.x] += v;
            __syncthreads();
        }
        const int off = carry + sc[threadIdx.x] - c;
        for (int i = 0; i < c; ++i) {
            const int pos = apos[(int64_t)b * nmax + i];
            eg[off + i] = gidx[(int64_t)b * nmax + pos];
            etm[off + i] = (int)(((unsigned)b << 8) | (unsigned)pos);
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry += sc[1023];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_top_rank(const int* __restrict__ eg, const int* __restrict__ etm,
                                                  int ntop, int* __restrict__ top_idx, int* __restrict__ tmap) {
    __shared__ int chunk[256];
    const int e = (int)(blockIdx.x * 256 + threadIdx.x);
    const int g = e < ntop ? eg[e] : 0;
    int rank = 0;
    for (int j0 = 0; j0 < ntop; j0 += 256) {
        const int j = j0 + (int)threadIdx.x;
        chunk[threadIdx.x] = j < ntop ? eg[j] : INT_MAX;
        __syncthreads();
        const int m = min(256, ntop - j0);
        for (int q = 0; q < m; ++q) rank += chunk[q] < g ? 1 : 0;
        __syncthreads();
    }
    if (e < ntop) {
        top_idx[rank] = g;
        tmap[rank] = etm[e];
    }
}

void launch_top_lists(const Level& L, int* top_idx, int* tmap, int64_t ntop, int* work, hipStream_t s) {
    if (ntop <= 0) return;
    if (L.nbox <= 16) {
        k_top_lists<<<dim3(1), dim3(1024), 0, s>>>(L.nact, L.apos, L.gidx, L.nbox, L.nmax, top_idx, tmap);
        return;
    }
    int* eg = work;
    int* etm = work + ntop;
    k_top_gather<<<dim3(1), dim3(1024), 0, s>>>(L.nact, L.apos, L.gidx, L.nbox, L.nmax, eg, etm);
    k_top_rank<<<dim3((unsigned)((ntop + 255) / 256)), dim3(256), 0, s>>>(eg, etm, (int)ntop, top_idx, tmap);
}

template <typename ST>
__global__ void k_top_assemble(const ST* __restrict__ store, const double* __restrict__ dstore, int nb, int nmax,
                               const int* __restrict__ tmap,
                               const int* __restrict__ top_idx, int64_t ntop, const double* __restrict__ pts,
                               double coef, double* __restrict__ A) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntop * ntop) return;
    int64_t i = e % ntop, j = e / ntop;
    const int a = (int)((unsigned)tmap[i] >> 8), pa = tmap[i] & 0xff;
    const int b = (int)((unsigned)tmap[j] >> 8), qb = tmap[j] & 0xff;
    int dx = b % nb - a % nb, dy = b / nb - a / nb;
    double v;
    if (dstore && a == b) {
        v = dstore[(int64_t)a * nmax * nmax + pa + (int64_t)qb * nmax];
    } else if (dx >= -2 && dx <= 2 && dy >= -2 && dy <= 2) {
        v = (double)store[((int64_t)a * kNbr + nbr_slot(dx, dy)) * nmax * nmax + pa + (int64_t)qb * nmax];
    } else {
        int gi = top_idx[i], gj = top_idx[j];
        v = kernel_entry(pts[2 * (int64_t)gi], pts[2 * (int64_t)gi + 1], pts[2 * (int64_t)gj],
                         pts[2 * (int64_t)gj + 1], coef);
    }
    A[e] = v;
}

void launch_top_assemble(const Level& L, const int* tmap, const int* top_idx, int64_t ntop, const double* pts,
                         const KernelParams& kp, double* A, hipStream_t s) {
    int64_t tot = ntop * ntop;
    const dim3 g((unsigned)((tot + 255) / 256));
    if (L.store32)
        k_top_assemble<float><<<g, dim3(256), 0, s>>>((const float*)L.store, L.dstore, L.nb, L.nmax, tmap, top_idx,
                                                      ntop, pts, kp.coef, A);
    else
        k_top_assemble<double><<<g, dim3(256), 0, s>>>((const double*)L.store, nullptr, L.nb, L.nmax, tmap, top_idx,
                                                       ntop, pts, kp.coef, A);
}

}  // namespace rss
