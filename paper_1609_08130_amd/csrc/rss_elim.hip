// Decoupling and elimination of the redundant DOFs of one box per workgroup
// (Section 3.1, the U_T / L_T pair and eq. zab; Section 2.1, eqs. landu and
// block_elimination with I = R, J = S u N, K = F).
//
// With the box's ID (S, R, T) and the current blocks of the store:
//   Z_X  = A_XR - A_XS T                   X in {S, N}     (column operation L_T)
//   X_RR = A_RR - A_RS T - T^T Z_S                         (both operations)
//   X_RJ = A_RJ - T^T A_SJ                 J = S u N       (row operation U_T)
//   X_JR = [Z_S; Z_N]
// X_RR^{-1} comes from in-place Gauss-Jordan elimination with partial pivoting (largest
// |.|, lowest row on ties; its pivots are those of LU with partial pivoting and give
// log|det X_RR|), and G = X_RR^{-1} X_RJ is formed tile by tile.  The record keeps T,
// X_JR, G, X_RR and X_RR^{-1}; the Schur complement A_JJ -= X_JR G is applied by the
// Schur kernel.  J lists S first, then the active DOFs of the adjacent boxes in
// ascending box index.
//
// Three launches per colour: k_elim_rows forms X_JR and Y_RR = A_RR - A_RS T tile by
// tile over many workgroups per box, k_elim_inv forms X_RR = Y_RR - T^T Z_S and its
// inverse (one workgroup per box), and k_elim_g forms G tile by tile over many
// workgroups per box.
#include "rss_internal.h"

namespace rss {

struct ElimArgs {
    const void* store;   // FP64 or FP32 entries (the kernels' ST)
    const double* dstore;   // self blocks of an FP32 store (FP64), or nullptr
    int* tl_cnt;         // Schur tile lists of the colour (TileList)
    int* tl_tiles;
    int* tl_info;
    int tl_capx;
    int nb, nmax, ldJ;
    const int* cnt;
    const int* gidx;
    int* nact;
    int* apos;
    const int* krank;
    int* nJ;
    const int* spos;
    const int* rpos;
    int* Jg;
    int* jmap;           // J row -> (3x3 slot << 16) | position in its box, for the Schur kernel
    int* jseg;           // per 3x3 slot: (first J row << 16) | rows, for the self-block update
    int* Sg;
    int* Rg;
    const double* T;
    double* XJR;
    double* G;
    double* XRR;
    double* Xinv;
    float* XJR32;
    float* G32;
    float* Xinv32;
    float* T32;
    double* logdet_part;
    int* sign_part;
    int* flag;           // error and status bits (bit 64: the LDS Gauss-Jordan ran)
    int weak;            // RS-WS weak pass: J = S (no adjacent boxes)
};

constexpr int kTileMax = 32;   // rows (or columns) of J per tile, at most
constexpr int kLineMax = 128;  // lines of the tiles one row workgroup takes, at most
constexpr int kElimGLds = 98304;   // LDS bytes of k_elim_g with X_RR^{-1} held for all its tiles

// Workgroups are dealt to the 8 XCDs round-robin in launch order.  With a grid of
// 8 * ntile * ceil(nbox / 8) workgroups, id = x + 8 s takes box x + 8 (s / ntile) and
// tile s % ntile, so all tiles of a box (and its one-workgroup kernels, launched with
// id = box) run on XCD x and share its L2.
__device__ inline bool xcd_tile(int ntile, int nbox, int& bi, int& tile) {
    const int x = blockIdx.x & 7, s = blockIdx.x >> 3;
    bi = x + 8 * (s / ntile);
    tile = s % ntile;
    return bi < nbox;
}

static inline unsigned xcd_grid(int ntile, int nbox) { return (unsigned)(8 * ntile * ((nbox + 7) / 8)); }

// dst(i, j) = src(i, j) for i < rows, j < cols, taken in the order e = i + rows j: thread t
// handles e = t, t + NTH, ... and issues U loads before its first store.  The (i, j) of
// successive elements advance by the fixed step (NTH % rows, NTH / rows), so no division
// is done per element.
template <int NTH, int U = 8, typename Load, typename Store>
__device__ inline void stage2d(int rows, int cols, Load load, Store store) {
    const int total = rows * cols;
    if (total <= 0) return;
    const int di = NTH % rows, dj = NTH / rows;
    int i = threadIdx.x % rows, j = threadIdx.x / rows;
    auto advance = [&](int& a, int& b) {
        a += di;
        b += dj;
        if (a >= rows) { a -= rows; ++b; }
    };
    for (int e0 = threadIdx.x; e0 < total; e0 += NTH * U) {
        double v[U];
        const int i0 = i, j0 = j;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = e0 + u * NTH < total ? load(i, j) : 0.0;
            advance(i, j);
        }
        int a = i0, b = j0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e0 + u * NTH < total) store(a, b, v[u]);
            advance(a, b);
        }
    }
}

// Per-workgroup tables of box c in LDS (ST: entry type of the block store).
typedef double f64x4 __attribute__((ext_vector_type(4)));   // accumulator of one FP64 MFMA block

template <typename ST>
struct ElimShared {
    int sp[kMaxBox], rp[kMaxBox];   // B positions of S and R
    const ST* blk_nc[8];            // A(B_o, B_c) of the adjacent boxes o
    const ST* blk_cn[8];            // A(B_c, B_o)
    const int* nap[8];              // active positions of o
    int nbox[8];
    int joff[9];                    // J segments: [0, k) is S, then one per adjacent box
    int nN;
    const void* srcp[kLineMax];     // source block and row/column of each tile line ...
    int srcpos[kLineMax];
    unsigned char src64[kLineMax];  // ... and whether that block holds FP64 entries
};

// Entry idx of the source block of tile line `line`.
template <typename ST>
__device__ inline double src_entry(const ElimShared<ST>& sh, int line, int64_t idx) {
    return sh.src64[line] ? ((const double*)sh.srcp[line])[idx] : (double)((const ST*)sh.srcp[line])[idx];
}

// The self block A(B_c, B_c): in the FP64 array when the store is FP32 and has one.
template <typename ST>
__device__ inline const void* self_block(const ElimArgs& a, int c, bool& is64) {
    const int64_t bsz = (int64_t)a.nmax * a.nmax;
    is64 = a.dstore != nullptr || sizeof(ST) == 8;
    if (a.dstore) return a.dstore + (int64_t)c * bsz;
    return (const ST*)a.store + ((int64_t)c * kNbr + 12) * bsz;
}

// sp, rp, the adjacent-box tables and T (Ts[b + r q] = T[q][b]).  The caller synchronizes.
template <int NTH, typename ST>
__device__ void elim_setup(ElimShared<ST>& sh, const ElimArgs& a, int c, int k, int r, double* Ts) {
    const int tid = threadIdx.x, nmax = a.nmax, nb = a.nb;
    const int64_t bsz = (int64_t)nmax * nmax;
    for (int i = tid; i < k; i += NTH) sh.sp[i] = a.spos[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += NTH) sh.rp[i] = a.rpos[(int64_t)c * nmax + i];
    // adjacent boxes in ascending index: thread t < 8 looks at offset t (centre skipped),
    // then thread 0 compacts and forms the segment offsets
    const int cx = c % nb, cy = c / nb;
    if (tid < 8) {
        const int t = tid < 4 ? tid : tid + 1;
        const int dx = t % 3 - 1, dy = t / 3 - 1;
        const int ox = cx + dx, oy = cy + dy;
        const bool in = !a.weak && ox >= 0 && oy >= 0 && ox < nb && oy < nb;
        sh.nbox[tid] = in ? ox + nb * oy : -1;
        sh.srcpos[tid] = in ? a.nact[ox + nb * oy] : 0;
    }
    const double* Tg = a.T + (int64_t)c * bsz;
    stage2d<NTH>(
        k, r, [&](int q, int b) { return Tg[q + (int64_t)b * nmax]; }, [&](int q, int b, double v) { Ts[b + r * q] = v; });
    __syncthreads();
    if (tid == 0) {
        int cntN = 0;
        sh.joff[0] = k;
        for (int t = 0; t < 8; ++t) {
            const int o = sh.nbox[t];
            if (o < 0) continue;
            const int tt = t < 4 ? t : t + 1;
            const int dx = tt % 3 - 1, dy = tt / 3 - 1;
            sh.blk_nc[cntN] = (const ST*)a.store + ((int64_t)o * kNbr + nbr_slot(-dx, -dy)) * bsz;   // A(B_o, B_c)
            sh.blk_cn[cntN] = (const ST*)a.store + ((int64_t)c * kNbr + nbr_slot(dx, dy)) * bsz;     // A(B_c, B_o)
            sh.nap[cntN] = a.apos + (int64_t)o * nmax;
            sh.nbox[cntN] = o;
            sh.joff[cntN + 1] = sh.joff[cntN] + sh.srcpos[t];
            ++cntN;
        }
        sh.nN = cntN;
    }
}

// Global index of J entry jj.
template <typename ST>
__device__ inline int j_global(const ElimShared<ST>& sh, const ElimArgs& a, int c, int jj, int k) {
    if (jj < k) return a.gidx[(int64_t)c * a.nmax + sh.sp[jj]];
    int i = 0;
    while (sh.joff[i + 1] <= jj) ++i;
    return a.gidx[(int64_t)sh.nbox[i] * a.nmax + sh.nap[i][jj - sh.joff[i]]];
}

// Store position of J entry jj: (slot << 16) | position in its box, slot = (dy + 1) 3 +
// (dx + 1) of the box in the 3x3 neighbourhood of c (4: c itself, whose J rows are S).
template <typename ST>
__device__ inline int j_map(const ElimShared<ST>& sh, const ElimArgs& a, int c, int jj, int k) {
    if (jj < k) return (4 << 16) | sh.sp[jj];
    int i = 0;
    while (sh.joff[i + 1] <= jj) ++i;
    const int o = sh.nbox[i], nb = a.nb;
    const int slot = (o / nb - c / nb + 1) * 3 + (o % nb - c % nb + 1);
    return (slot << 16) | sh.nap[i][jj - sh.joff[i]];
}

// Rows [r0, r0 + tr) of E = [J; R] against the columns R: rows of J give X_JR (and its
// FP32 copy when XJR32 != nullptr), rows past J give Y_RR = A_RR - A_RS T (into Y, ld nmax).
// tA: tw x n.
// Source of lines l < nl of [J; R] starting at row r0 (J rows r0 + l < nj, then R rows):
// the block holding the line, its row there and the block's entry type.  The caller
// synchronizes.
template <int NTH, typename ST>
__device__ void elim_rows_src(ElimShared<ST>& sh, const ElimArgs& a, int c, int k, int nj, int r0, int nl) {
    bool acc64;
    const void* Acc = self_block<ST>(a, c, acc64);
    for (int l = threadIdx.x; l < nl; l += NTH) {
        const int jj = r0 + l;
        if (jj < k) {
            sh.srcp[l] = Acc;
            sh.src64[l] = acc64;
            sh.srcpos[l] = sh.sp[jj];
        } else if (jj < nj) {
            int s = 0;
            while (sh.joff[s + 1] <= jj) ++s;
            sh.srcp[l] = sh.blk_nc[s];
            sh.src64[l] = sizeof(ST) == 8;
            sh.srcpos[l] = sh.nap[s][jj - sh.joff[s]];
        } else {
            sh.srcp[l] = Acc;
            sh.src64[l] = acc64;
            sh.srcpos[l] = sh.rp[jj - nj];
        }
    }
}

// The products of a tile of tr lines starting at row r0, its lines in tA[i + tw col] (col
// a B position: col < k ? sp[col] : rp[col - k]).  The transposed tile (r x tr) on the FP64
// matrix cores, so that the 16 lanes of a result row hold 16 consecutive lines:
// D = A_(tile, R)^T - T^T A_(tile, S)^T with A = -T^T (A[b][q] = -Ts[b + r q]) and
// B[q][i] = tA[i + tw q]; D starts at the R columns of the tile.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[l / 16 + 4 v][l % 16].  16 x 16
// blocks are dealt to the waves.  Rows of J go to X_JR (and its FP32 copy), rows of R to Y.
template <int NTH>
__device__ void elim_rows_product(const ElimArgs& a, int k, int r, int nj, int r0, int tr, int tw, const double* Ts,
                                  const double* tA, double* XJR, float* XJR32, double* Y) {
    const int tid = threadIdx.x, nmax = a.nmax, ldJ = a.ldJ;
    const int lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int nrb = (r + 15) / 16, nblk = nrb * ((tr + 15) / 16);
    for (int blk = wv; blk < nblk; blk += NTH / 64) {
        const int rb = (blk % nrb) * 16, i = (blk / nrb) * 16 + l16;
        f64x4 x;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int b = rb + l4 + 4 * v;
            x[v] = (b < r && i < tr) ? tA[i + tw * (k + b)] : 0.0;
        }
        const int ar = rb + l16;
        for (int q0 = 0; q0 < k; q0 += 4) {
            const int q = q0 + l4;
            const double av = (ar < r && q < k) ? -Ts[ar + r * q] : 0.0;
            const double bv = (q < k && i < tr) ? tA[i + tw * q] : 0.0;
            x = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, x, 0, 0, 0);
        }
        if (i < tr) {
            const int row = r0 + i;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = rb + l4 + 4 * v;
                if (b >= r) break;
                if (row < nj) {
                    XJR[row + (int64_t)b * ldJ] = x[v];
                    if (XJR32) XJR32[row + (int64_t)b * ldJ] = (float)x[v];
                } else {
                    Y[(row - nj) + (int64_t)b * nmax] = x[v];
                }
            }
        }
    }
}

// One tile of tr lines starting at row r0: sources, lines staged into tA, products.
template <int NTH, typename ST>
__device__ void elim_rows_tile(ElimShared<ST>& sh, const ElimArgs& a, int c, int k, int r, int nj, int r0, int tr,
                               int tw, const double* Ts, double* tA, double* XJR, float* XJR32, double* Y) {
    const int nmax = a.nmax;
    const int n = k + r;
    elim_rows_src<NTH, ST>(sh, a, c, k, nj, r0, tr);
    __syncthreads();
    // tA[i + tw col]: line i of the tile at B position (col < k ? sp[col] : rp[col - k])
    stage2d<NTH>(
        tr, n,
        [&](int i, int col) {
            const int pos = col < k ? sh.sp[col] : sh.rp[col - k];
            return src_entry(sh, i, sh.srcpos[i] + (int64_t)pos * nmax);
        },
        [&](int i, int col, double v) { tA[i + tw * col] = v; });
    __syncthreads();
    elim_rows_product<NTH>(a, k, r, nj, r0, tr, tw, Ts, tA, XJR, XJR32, Y);
    __syncthreads();
}

// Columns [c0, c0 + tc) of G = X_RR^{-1} X_RJ.  The kernel is real symmetric and so is
// every stored update, so X_RJ = A_RJ - T^T A_SJ is the transpose of X_JR = A_JR - A_JS T
// (the record k_elim_rows wrote): the tile is X_JR's rows c0 .. c0 + tc - 1, read into
// tX[b + ldt col] (ldt = nmax + 1, odd: 16 lanes reading one row of 16 columns hit 16
// banks).  X_RR^{-1} (ld ldw) is read from W when the workgroup holds it in LDS
// (xi_lds); otherwise it is staged through Wst, tw columns at a time.  r <= 64 HB.
template <int NTH, int HB>
__device__ void elim_g_tile(const ElimArgs& a, int c, int r, int c0, int tc, int tw, double* tX, double* Wst,
                            const double* Xi, const double* W, bool xi_lds, double* G, float* G32) {
    constexpr int NW = NTH / 64;
    const int tid = threadIdx.x, nmax = a.nmax, ldJ = a.ldJ;
    const int lane = tid & 63, jg = tid >> 6;
    const int ldt = nmax + 1;
    const double* XJR = a.XJR + (int64_t)c * ldJ * nmax;
    stage2d<NTH>(
        tc, r, [&](int col, int b) { return XJR[(c0 + col) + (int64_t)b * ldJ]; },
        [&](int col, int b, double v) { tX[b + ldt * col] = v; });
    __syncthreads();
    // G^T = X_RJ^T X_RR^{-T} on the FP64 matrix cores (tc x r results, so that the 16 lanes
    // of a result row hold 16 consecutive rows of G): 16 x 16 blocks dealt to the waves,
    // one v_mfma_f64_16x16x4 per 4 values of the inner index; lane l supplies
    // A[l % 16][l / 16] = tX[q + ldt col] and B[l / 16][l % 16] = X_RR^{-1}[b][q] and
    // receives D[l / 16 + 4 v][l % 16] for v < 4.
    constexpr int MB = 2 * HB;   // blocks per wave: r <= 64 HB, tc <= 32, 4 waves
    static_assert(NW == 4 && kTileMax <= 32, "block count per wave assumes 4 waves and <= 32 columns");
    const int ncb = (tc + 15) / 16, nblk = ncb * ((r + 15) / 16);
    const int l16 = lane & 15, l4 = lane >> 4;
    f64x4 acc[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[m] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int qc = xi_lds ? r : tw;
    for (int q0 = 0; q0 < r; q0 += qc) {
        const int qn = min(qc, r - q0);
        const double* Wq = W + (int64_t)q0 * ldt;
        if (!xi_lds) {
            stage2d<NTH>(
                r, qn, [&](int b, int q) { return Xi[b + (int64_t)(q0 + q) * nmax]; },
                [&](int b, int q, double v) { Wst[b + ldt * q] = v; });
            __syncthreads();
            Wq = Wst;
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int blk = jg + NW * m;
            if (blk >= nblk) break;
            const int acol = (blk % ncb) * 16 + l16, b = (blk / ncb) * 16 + l16;
            for (int qq = 0; qq < qn; qq += 4) {
                const int kk = qq + l4;
                const double av = (acol < tc && kk < qn) ? tX[(q0 + kk) + ldt * acol] : 0.0;
                const double bv = (kk < qn && b < r) ? Wq[b + ldt * kk] : 0.0;
                acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[m], 0, 0, 0);
            }
        }
        if (!xi_lds) __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int blk = jg + NW * m;
        if (blk >= nblk) break;
        const int b = (blk / ncb) * 16 + l16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = (blk % ncb) * 16 + l4 + 4 * v;
            if (b < r && col < tc) {
                G[b + (int64_t)(c0 + col) * nmax] = acc[m][v];
                if (G32) G32[b + (int64_t)(c0 + col) * nmax] = (float)acc[m][v];
            }
        }
    }
    __syncthreads();
}

// X_RR^{-1} of the r x r matrix Xs (ld ldx) in place: Gauss-Jordan with partial pivoting
// (largest |.|, lowest row on ties), then the row interchanges undone on the columns.
// Each step: one wave picks the pivot; the pivot column (after the interchange) and rows j
// and p are copied to sc; then each wave updates whole columns, every element by the lane
// that owns it (interchange, pivot-row scaling and rank-1 update in one pass).
// sc: 4 * ldx doubles of LDS.  Returns false when a pivot column is exactly zero.
template <int NTH>
__device__ bool gj_inverse(double* Xs, int ldx, int r, int* colswap, double* sc, int& piv_idx, double& piv_val,
                           double& ld_sum, int& sgn) {
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    double* fvec = sc;
    double* rowj = sc + ldx;
    double* rowp = sc + 2 * ldx;
    double* pivs = sc + 3 * ldx;
    for (int j = 0; j < r; ++j) {
        if (wv == 0) {
            double best = -1.0;
            int bi = 1 << 30;
            for (int i = j + lane; i < r; i += 64) {
                double v = fabs(Xs[i + j * ldx]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            wave_argmax(best, bi);
            if (lane == 0) {
                piv_idx = bi;
                piv_val = (bi < r && best > 0.0) ? Xs[bi + j * ldx] : 0.0;
            }
        }
        __syncthreads();
        const int p = piv_idx;
        const double d = piv_val;
        if (!(fabs(d) > 0.0) || p >= r) return false;
        for (int i = tid; i < r; i += NTH) {
            fvec[i] = (i == j) ? 0.0 : Xs[(i == p ? j : i) + j * ldx];   // column j after the interchange
            rowj[i] = Xs[j + i * ldx];
            rowp[i] = Xs[p + i * ldx];
        }
        if (tid == 0) { colswap[j] = p; pivs[j] = d; }
        __syncthreads();
        const double rinv = 1.0 / d;
        // each wave takes 4 columns per pass and each lane rows lane and lane + 64, all loads
        // issued before the first store (every element is read and written by its owner only)
        for (int l0 = 4 * wv; l0 < r; l0 += 4 * (NTH / 64)) {
            double xjl[4], xjo[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int l = min(l0 + u, r - 1);
                xjl[u] = (l == j ? 1.0 : rowp[l]) * rinv;   // new pivot row
                xjo[u] = rowj[l];                            // old row j, now row p
            }
            for (int i0 = lane; i0 < r; i0 += 128) {
                double x[2][4], fv[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = min(i0 + 64 * h, r - 1);
                    fv[h] = fvec[i];
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[h][u] = Xs[i + min(l0 + u, r - 1) * ldx];
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = i0 + 64 * h;
                    if (i >= r) continue;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int l = l0 + u;
                        if (l >= r) continue;
                        double v;
                        if (i == j) v = xjl[u];
                        else v = ((l == j) ? 0.0 : (i == p ? xjo[u] : x[h][u])) - fv[h] * xjl[u];
                        Xs[i + l * ldx] = v;
                    }
                }
            }
        }
        __syncthreads();
    }
    for (int j = r - 1; j >= 0; --j) {
        int p = colswap[j];
        if (p != j)
            for (int i = tid; i < r; i += NTH) {
                double t0 = Xs[i + j * ldx];
                Xs[i + j * ldx] = Xs[i + p * ldx];
                Xs[i + p * ldx] = t0;
            }
        __syncthreads();
    }
    // log|det| and sign: one log per thread, summed in pivot order
    for (int i = tid; i < r; i += NTH) fvec[i] = log(fabs(pivs[i]));
    __syncthreads();
    ld_sum = 0.0;
    sgn = 1;
    for (int i = 0; i < r; ++i) {
        ld_sum += fvec[i];
        if (pivs[i] < 0) sgn = -sgn;
        if (colswap[i] != i) sgn = -sgn;
    }
    return true;
}

// Value of v held by lane `ln` of the wave (ln wave-uniform).
__device__ inline double lane_read(double v, int ln) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffff), ln);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), ln);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Register-resident variant of gj_inverse: thread (wave w, lane) holds X[lane + 64 h][w + NW c]
// for h < RB, c < CB, which covers r <= 64 RB and r <= NW CB.  The pivot rows are not
// interchanged: step j takes as pivot the unused row p of largest |x_pj| (an unsigned 64-bit
// key, lowest row among equal keys), scales row p, subtracts its multiples from every other
// row and replaces column j; the per-step arithmetic of each element is that of the
// interchanging form.  At the end row p_j of the array holds row j of the interchanging form,
// and the column interchanges of that form (the transposition of j with the position row p_j
// had reached there) are undone on the way out.  One barrier per step: the wave that owns
// column j picks the pivot and publishes column j (through a buffer of two halves used in
// alternate steps), p and 1 / x_pj, so the other waves load all three together; every wave
// reads row p of its own columns from the lane holding it.
// x holds the matrix on entry (zero outside r x r); the inverse is written to Xs (ld ldx).
// sc: 4 * ldx doubles of LDS.
template <int NTH, int RB, int CB>
__device__ bool gj_inverse_reg(double (&x)[RB][CB], double* Xs, int ldx, float* Xs32, int r, int* colswap,
                               double* sc, double& ld_sum, int& sgn) {
    constexpr int NW = NTH / 64;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    double* colj = sc;                  // two halves of ldx
    double* pivs = sc + 2 * ldx;
    double* rinvs = sc + 3 * ldx;       // 1 / pivot, by step parity
    unsigned used = 0;   // bit h: row lane + 64 h has been a pivot row
    for (int j = 0; j < r; ++j) {
        double* cb = colj + (j & 1) * ldx;
        const int cj = j / NW;
        if (wv == j % NW) {
            unsigned long long kb = 0;
            int hb = 0;
            double vc[RB];
#pragma unroll
            for (int h = 0; h < RB; ++h) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c == cj) v = x[h][c];
                vc[h] = v;
                const int i = lane + 64 * h;
                if (i < r) cb[i] = v;
                const bool cand = i < r && !((used >> h) & 1u);
                const unsigned long long key = cand ? (unsigned long long)__double_as_longlong(fabs(v)) : 0ull;
                if (key > kb) { kb = key; hb = h; }
            }
            const unsigned long long km = wave_max_u64(kb);
            int p = -1;
            if (km > 0) {
#pragma unroll
                for (int h = RB - 1; h >= 0; --h) {
                    const unsigned long long b = __ballot(kb == km && hb == h);
                    if (b) p = 64 * h + __ffsll((long long)b) - 1;
                }
            }
            // the pivot and its reciprocal go out with p (-1: no usable pivot)
            double d = 0.0;
            if (p >= 0) {
#pragma unroll
                for (int h = 0; h < RB; ++h)
                    if (h == (p >> 6)) d = lane_read(vc[h], p & 63);
            }
            if (!(fabs(d) > 0.0)) p = -1;
            if (lane == 0) {
                colswap[j] = p;
                pivs[j] = d;
                rinvs[j & 1] = 1.0 / d;
            }
        }
        __syncthreads();
        const int p = __builtin_amdgcn_readfirstlane(colswap[j]);
        if (p < 0) return false;
        const double rinv = rinvs[j & 1];
        const int pl = p & 63, ph = p >> 6;
        double fv[RB];
#pragma unroll
        for (int h = 0; h < RB; ++h) {
            const int i = lane + 64 * h;
            fv[h] = (i == p || i >= r) ? 0.0 : cb[i];
        }
        // new pivot row, from the lane that holds row p (slot ph is wave-uniform)
        double xj[CB];
#pragma unroll
        for (int h = 0; h < RB; ++h)
            if (h == ph) {
#pragma unroll
                for (int c = 0; c < CB; ++c) xj[c] = lane_read(x[h][c], pl) * rinv;
            }
        // every row but p (rows and columns >= r hold values that are never read back)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int h = 0; h < RB; ++h) x[h][c] -= fv[h] * xj[c];
#pragma unroll
        for (int h = 0; h < RB; ++h)
            if (h == ph && lane == pl) {
#pragma unroll
                for (int c = 0; c < CB; ++c) x[h][c] = xj[c];
                used |= 1u << h;
            }
        if (wv == j % NW) {
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c == cj) {
#pragma unroll
                    for (int h = 0; h < RB; ++h) x[h][c] = (lane + 64 * h == p) ? rinv : -fv[h] * rinv;
                }
        }
    }
    // The interchanging form would have moved row p_j to position j (so its row j is row p_j
    // of the array) and then moved column j of its result to column p_j: the product of
    // its row transpositions, applied to the columns in reverse order, is the permutation
    // j -> p_j itself.  So entry (i, l) of the array goes to (j with p_j = i, p_l).
    __syncthreads();
    int* lpos = (int*)colj;   // array row -> row of the inverse
    for (int j = tid; j < r; j += NTH) lpos[colswap[j]] = j;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < RB; ++h)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = lane + 64 * h, l = wv + NW * c;
            if (i < r && l < r) {
                Xs[lpos[i] + colswap[l] * ldx] = x[h][c];
                if (Xs32) Xs32[lpos[i] + colswap[l] * ldx] = (float)x[h][c];
            }
        }
    // log|det|: the sum of log|pivot| (wave 0, by lanes then across the wave); sign: the
    // negative pivots and the parity of j -> p_j (number of inversions)
    ld_sum = 0.0;
    sgn = 1;
    if (wv == 0) {
        double ls = 0.0;
        int odd = 0;
        for (int t = lane; t < r; t += 64) {
            ls += log(fabs(pivs[t]));
            const int pt = colswap[t];
            int inv = pivs[t] < 0 ? 1 : 0;
            for (int u = t + 1; u < r; ++u) inv += colswap[u] < pt ? 1 : 0;
            odd ^= inv & 1;
        }
        for (int o = 32; o > 0; o >>= 1) {
            ls += __shfl_xor(ls, o, 64);
            odd ^= __shfl_xor(odd, o, 64);
        }
        ld_sum = ls;
        sgn = odd ? -1 : 1;
    }
    __syncthreads();
    return true;
}

// X_RR = Y_RR - T^T Z_S straight into the registers of gj_inverse_reg (thread (wave w, lane)
// forms X[lane + 64 h][w + NW c], reading T for its rows and Z_S for its columns once per q),
// also written to XRR; then the inverse straight into Xinv (and its FP32 copy).
template <int NTH, int RB, int CB>
__device__ bool xrr_gj_reg(const double* Yg, int nmax, const double* Ts, const double* zs, int ldz, int k, int r,
                           double* XRR, double* Xinv, float* Xinv32, int* colswap, double* sc, double& ld_sum,
                           int& sgn) {
    constexpr int NW = NTH / 64;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double x[RB][CB];
#pragma unroll
    for (int h = 0; h < RB; ++h)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = lane + 64 * h, l = wv + NW * c;
            x[h][c] = (i < r && l < r) ? Yg[i + (int64_t)l * nmax] : 0.0;
        }
#pragma unroll 2
    for (int q = 0; q < k; ++q) {
        double t[RB], z[CB];
#pragma unroll
        for (int h = 0; h < RB; ++h) t[h] = Ts[min(lane + 64 * h, r - 1) + r * q];
#pragma unroll
        for (int c = 0; c < CB; ++c) z[c] = zs[q + (int64_t)min(wv + NW * c, r - 1) * ldz];
#pragma unroll
        for (int h = 0; h < RB; ++h)
#pragma unroll
            for (int c = 0; c < CB; ++c) x[h][c] -= t[h] * z[c];
    }
#pragma unroll
    for (int h = 0; h < RB; ++h)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = lane + 64 * h, l = wv + NW * c;
            if (i < r && l < r) XRR[i + (int64_t)l * nmax] = x[h][c];
            else x[h][c] = 0.0;
        }
    return gj_inverse_reg<NTH, RB, CB>(x, Xinv, nmax, Xinv32, r, colswap, sc, ld_sum, sgn);
}

// X_RR = Y_RR - T^T Z_S (Y_RR read from Yg, formed by the row tiles),
// then its inverse, log|det| and the per-box records.  Returns false when X_RR is singular.
template <int NTH, typename ST>
__device__ bool elim_xrr_inverse(ElimShared<ST>& sh, const ElimArgs& a, int c, int k, int r, int nj, const double* Ts,
                                 const double* Yg, double* Xs, double* xsr, int mixed, int* colswap, double* sc,
                                 int& piv_idx, double& piv_val) {
    const int tid = threadIdx.x, nmax = a.nmax, ldJ = a.ldJ;
    const int64_t bsz = (int64_t)nmax * nmax;
    const double* XJR = a.XJR + (int64_t)c * ldJ * nmax;
    double* XRR = a.XRR + (int64_t)c * bsz;
    // Z_S = rows S of X_JR, staged in LDS (xsr[q + k b2]) when a buffer is given
    const double* zs = XJR;
    int ldz = ldJ;
    if (xsr) {
        for (int e = tid; e < k * r; e += NTH) {
            int q = e % k, b2 = e / k;
            xsr[e] = XJR[q + (int64_t)b2 * ldJ];
        }
        __syncthreads();
        zs = xsr;
        ldz = k;
    }
    double ld_sum;
    int sgn;
    bool ok;
    // Register Gauss-Jordan when 64 RB rows and NW CB columns cover r (256 threads: r <= 64,
    // X_RR through XRR; 1024 threads: r <= 128, X_RR formed in the registers); the inverse
    // goes straight to Xinv.  Otherwise X_RR goes through Xs to the LDS form.
    double* Xinv = a.Xinv + (int64_t)c * bsz;
    float* Xinv32 = mixed ? a.Xinv32 + (int64_t)c * bsz : nullptr;
    if ((NTH == 1024 && r <= 128) || (NTH == 256 && r <= 64)) {
        if constexpr (NTH == 1024) {
            if (r <= 64) ok = xrr_gj_reg<NTH, 1, 4>(Yg, nmax, Ts, zs, ldz, k, r, XRR, Xinv, Xinv32, colswap, sc, ld_sum, sgn);
            else if (r <= 96) ok = xrr_gj_reg<NTH, 2, 6>(Yg, nmax, Ts, zs, ldz, k, r, XRR, Xinv, Xinv32, colswap, sc, ld_sum, sgn);
            else ok = xrr_gj_reg<NTH, 2, 8>(Yg, nmax, Ts, zs, ldz, k, r, XRR, Xinv, Xinv32, colswap, sc, ld_sum, sgn);
        } else if constexpr (NTH == 256) {
            // X_RR element by element into XRR, then into the registers from there (the
            // workgroup's own writes are visible to it after the barrier)
            for (int e = tid; e < r * r; e += NTH) {
                int b = e % r, b2 = e / r;
                double v = Yg[b + (int64_t)b2 * nmax];
                for (int q = 0; q < k; ++q) v -= Ts[b + r * q] * zs[q + (int64_t)b2 * ldz];
                XRR[b + (int64_t)b2 * nmax] = v;
            }
            __syncthreads();
            constexpr int CB = 16;
            double x[1][CB];
            const int wv = tid >> 6, lane = tid & 63;
#pragma unroll
            for (int cc = 0; cc < CB; ++cc) {
                const int l = wv + 4 * cc;
                x[0][cc] = (lane < r && l < r) ? XRR[lane + (int64_t)l * nmax] : 0.0;
            }
            ok = gj_inverse_reg<NTH, 1, CB>(x, Xinv, nmax, Xinv32, r, colswap, sc, ld_sum, sgn);
        }
    } else {
        for (int e = tid; e < r * r; e += NTH) {
            int b = e % r, b2 = e / r;
            double v = Yg[b + (int64_t)b2 * nmax];
            for (int q = 0; q < k; ++q) v -= Ts[b + r * q] * zs[q + (int64_t)b2 * ldz];
            XRR[b + (int64_t)b2 * nmax] = v;
            Xs[b + b2 * nmax] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) atomicOr(a.flag, 64);   // records that the LDS form ran
        ok = gj_inverse<NTH>(Xs, nmax, r, colswap, sc, piv_idx, piv_val, ld_sum, sgn);
        if (ok)
            for (int e = tid; e < r * r; e += NTH) {
                int b = e % r, b2 = e / r;
                Xinv[b + (int64_t)b2 * nmax] = Xs[b + b2 * nmax];
                if (mixed) Xinv32[b + (int64_t)b2 * nmax] = (float)Xs[b + b2 * nmax];
            }
    }
    if (!ok) return false;
    if (tid == 0) {
        a.logdet_part[c] = ld_sum;
        a.sign_part[c] = sgn;
    }
    if (mixed)
        for (int e = tid; e < k * r; e += NTH) {
            int b = e % r, q = e / r;
            a.T32[(int64_t)c * bsz + q + (int64_t)b * nmax] = (float)Ts[e];
        }
    for (int i = tid; i < k; i += NTH) a.Sg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + sh.sp[i]];
    for (int i = tid; i < r; i += NTH) a.Rg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + sh.rp[i]];
    return true;
}

// ---- the three launches of a colour ------------------------------------------------------
// grid (row tiles of [J; R], boxes).  Dynamic LDS: Ts[tsz] | tA[nmax tw]
template <int NTH, typename ST>
__global__ void __launch_bounds__(NTH) k_elim_rows(ElimArgs a, const int* __restrict__ boxes, int nbox, int ntile,
                                                   int mixed, double* __restrict__ work, int tsz, int tw, int tpw) {
    extern __shared__ double dyn[];
    __shared__ ElimShared<ST> sh;
    const int tid = threadIdx.x;
    int bi, tile;
    if (!xcd_tile(ntile, nbox, bi, tile)) return;
    const int c = boxes[bi];
    const int n = a.cnt[c];
    const int k = a.krank[c];
    const int r = n - k;
    if (n == 0 || r == 0) return;
    if (tile > 0) {
        // |J| + |R| from the active counts of the adjacent boxes: workgroups whose rows all
        // lie beyond it leave before the set-up
        const int nb = a.nb, cx = c % nb, cy = c / nb;
        int njr = k + r;
        for (int t = 0; t < (a.weak ? 0 : 9); ++t) {
            const int ox = cx + t % 3 - 1, oy = cy + t / 3 - 1;
            if (t != 4 && ox >= 0 && oy >= 0 && ox < nb && oy < nb) njr += a.nact[ox + nb * oy];
        }
        if (tile * tpw * tw >= njr) return;
    }
    const int nmax = a.nmax, ldJ = a.ldJ;
    double* Ts = dyn;
    double* tA = dyn + tsz;
    elim_setup<NTH, ST>(sh, a, c, k, r, Ts);
    __syncthreads();
    const int nj = sh.joff[sh.nN];
    double* XJR = a.XJR + (int64_t)c * ldJ * nmax;
    float* XJR32 = mixed ? a.XJR32 + (int64_t)c * ldJ * nmax : nullptr;
    double* Y = work + (int64_t)bi * nmax * nmax;
    // tpw consecutive tiles share the set-up: rows [rlo, rhi) of [J; R]
    const int rlo = tile * tpw * tw, rhi = min((tile + 1) * tpw * tw, nj + r);
    if (rlo >= rhi) return;
    for (int jj = rlo + tid; jj < min(nj, rhi); jj += NTH) {
        a.Jg[(int64_t)c * ldJ + jj] = j_global(sh, a, c, jj, k);
        a.jmap[(int64_t)c * ldJ + jj] = j_map(sh, a, c, jj, k);
    }
    constexpr int PF = 8;   // tile entries per thread held in registers
    if (rhi - rlo > kLineMax || tw * n > PF * NTH) {
        for (int r0 = rlo; r0 < rhi; r0 += tw)
            elim_rows_tile<NTH, ST>(sh, a, c, k, r, nj, r0, min(tw, rhi - r0), tw, Ts, tA, XJR, XJR32, Y);
        return;
    }
    // The sources of all lines at once; then the lines of tile t + 1 are loaded into
    // registers while the products of tile t run (one barrier after each landing and
    // after each product, as the tile form)
    elim_rows_src<NTH, ST>(sh, a, c, k, nj, rlo, rhi - rlo);
    __syncthreads();
    double v[PF];
    auto issue = [&](int r0) {
        const int tr = min(tw, rhi - r0), total = tr * n, l0 = r0 - rlo;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int e = tid + NTH * u;
            v[u] = 0.0;
            if (e < total) {
                const int i = e % tr, col = e / tr;
                const int pos = col < k ? sh.sp[col] : sh.rp[col - k];
                v[u] = src_entry(sh, l0 + i, sh.srcpos[l0 + i] + (int64_t)pos * nmax);
            }
        }
    };
    auto land = [&](int r0) {
        const int tr = min(tw, rhi - r0), total = tr * n;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int e = tid + NTH * u;
            if (e < total) tA[e % tr + tw * (e / tr)] = v[u];
        }
    };
    issue(rlo);
    for (int r0 = rlo; r0 < rhi; r0 += tw) {
        land(r0);
        __syncthreads();
        if (r0 + tw < rhi) issue(r0 + tw);
        elim_rows_product<NTH>(a, k, r, nj, r0, min(tw, rhi - r0), tw, Ts, tA, XJR, XJR32, Y);
        __syncthreads();
    }
}

// grid (boxes).  Dynamic LDS: Ts[tsz] | sc[4 nmax] | Z_S[tsz] (when use_zs) | Xs[nmax^2]
// (when XLDS; else X_RR is inverted in place of Y_RR in the workspace)
template <bool XLDS, int NTH, typename ST>
__global__ void __launch_bounds__(NTH) k_elim_inv(ElimArgs a, const int* __restrict__ boxes, int mixed,
                                                  double* __restrict__ work, int* flag, int tsz, int use_zs) {
    extern __shared__ double dyn[];
    __shared__ ElimShared<ST> sh;
    __shared__ int colswap[kMaxBox];
    __shared__ int piv_idx;
    __shared__ double piv_val;
    const int tid = threadIdx.x;
    const int c = boxes[blockIdx.x];
    const int n = a.cnt[c];
    const int k = a.krank[c];
    const int r = n - k;
    if (n == 0 || r == 0) {
        if (tid == 0) a.nJ[c] = 0;
        return;
    }
    const int nmax = a.nmax;
    double* Ts = dyn;
    double* sc = dyn + tsz;
    double* xsr = use_zs ? sc + 4 * nmax : nullptr;
    double* Y = work + (int64_t)blockIdx.x * nmax * nmax;
    double* Xs = XLDS ? sc + 4 * nmax + (use_zs ? tsz : 0) : Y;
    elim_setup<NTH, ST>(sh, a, c, k, r, Ts);
    __syncthreads();
    const int nj = sh.joff[sh.nN];
    if (!elim_xrr_inverse<NTH, ST>(sh, a, c, k, r, nj, Ts, Y, Xs, xsr, mixed, colswap, sc, piv_idx, piv_val)) {
        if (tid == 0) { atomicOr(flag, 4); a.nJ[c] = 0; }
        return;
    }
    if (tid == 0) {
        a.nJ[c] = nj;
        a.nact[c] = k;
    }
    for (int i = tid; i < k; i += NTH) a.apos[(int64_t)c * nmax + i] = sh.sp[i];
    if (tid < 64) {
        // the box's ceil(|J| / 64)^2 Schur tiles, appended to the list of its XCD by wave 0
        const int nt1 = (nj + 63) >> 6, ntl = nt1 * nt1, x = blockIdx.x & 7;
        int off = 0;
        if (tid == 0) off = atomicAdd(a.tl_cnt + x, ntl);
        off = __shfl(off, 0, 64);
        const int64_t o = (int64_t)x * a.tl_capx + off;
        for (int t = tid; t < ntl; t += 64) {
            a.tl_tiles[o + t] = (int)(((unsigned)c << 12) | ((t % nt1) << 6) | (t / nt1));
            a.tl_info[o + t] = (int)(((unsigned)(c >> 20) << 21) | ((unsigned)nj << 9) | (unsigned)r);
        }
    } else if (tid < 64 + 9) {
        // J rows of the box at 3x3 slot s = (dy + 1) 3 + (dx + 1) (slot 4: S of c)
        const int sl = tid - 64;
        int v = 0;
        if (sl == 4) {
            v = k;
        } else {
            const int ox = c % a.nb + sl % 3 - 1, oy = c / a.nb + sl / 3 - 1;
            for (int i = 0; i < sh.nN; ++i)
                if (sh.nbox[i] == ox + a.nb * oy) v = (sh.joff[i] << 16) | (sh.joff[i + 1] - sh.joff[i]);
            if ((v & 0xffff) == 0) v = 0;
        }
        a.jseg[(int64_t)c * 9 + sl] = v;
    }
}

// grid (column tiles of J, boxes).  Dynamic LDS: tX[(nmax + 1) tw] | W: X_RR^{-1}
// [(nmax + 1) nmax] when xi_lds (loaded once for the workgroup's tiles), else a staging
// buffer [(nmax + 1) tw].
template <int NTH, int HB>
__global__ void __launch_bounds__(NTH) k_elim_g(ElimArgs a, const int* __restrict__ boxes, int nbox, int ntile,
                                                int mixed, int* flag, int tw, int tpw, int xi_lds) {
    extern __shared__ double dyn[];
    int bi, tile;
    if (!xcd_tile(ntile, nbox, bi, tile)) return;
    const int c = boxes[bi];
    const int n = a.cnt[c];
    const int k = a.krank[c];
    const int r = n - k;
    if (n == 0 || r == 0 || (*flag & 4)) return;
    // |J| is known from the inverse kernel: workgroups whose tiles all lie beyond it leave
    // before the set-up
    const int nj = a.nJ[c];
    if (tile * tpw * tw >= nj) return;
    const int nmax = a.nmax, ldJ = a.ldJ, ldt = nmax + 1;
    double* tX = dyn;
    double* W = dyn + (int64_t)ldt * tw;
    const double* Xi = a.Xinv + (int64_t)c * nmax * nmax;
    if (xi_lds)
        stage2d<NTH>(
            r, r, [&](int b, int q) { return Xi[b + (int64_t)q * nmax]; },
            [&](int b, int q, double v) { W[b + ldt * q] = v; });
    double* G = a.G + (int64_t)c * nmax * ldJ;
    float* G32 = mixed ? a.G32 + (int64_t)c * nmax * ldJ : nullptr;
    for (int t = tile * tpw; t < (tile + 1) * tpw; ++t) {   // tpw consecutive tiles share the set-up
        const int c0 = t * tw;
        if (c0 >= nj) break;
        elim_g_tile<NTH, HB>(a, c, r, c0, min(tw, nj - c0), tw, tX, W, Xi, W, xi_lds != 0, G, G32);
    }
}

// Tiles of one box handled in turn by one workgroup of the row and column tile kernels:
// several when the launch has work groups to spare (the per-box setup is then paid once
// for them), one otherwise so that small colours still spread over all compute units.
static int tiles_per_wg(int ntile, int nboxes) { return min(ntile, plan_params(nboxes).elim_tpw); }

static int g_max_lds = -1;

int elim_lds_limit() {
    if (g_max_lds < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            g_max_lds = v;
        else
            g_max_lds = 65536;
    }
    return g_max_lds;
}

template <typename K>
static void set_lds(K kernel, size_t bytes) {
    hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename ST>
static int launch_elim_t(const Level& L, const int* boxes, int nboxes, int mixed, int weak, double* work, int* flag,
                         const TileList& tl, hipStream_t s) {
    if (nboxes <= 0) return 0;
    ElimArgs a;
    a.weak = weak;
    a.tl_cnt = tl.cnt; a.tl_tiles = tl.tiles; a.tl_info = tl.info; a.tl_capx = tl.capx;
    a.jseg = L.jseg;
    a.store = L.store; a.dstore = L.dstore; a.nb = L.nb; a.nmax = L.nmax; a.ldJ = L.ldJ;
    a.cnt = L.cnt; a.gidx = L.gidx; a.nact = L.nact; a.apos = L.apos; a.krank = L.krank; a.nJ = L.nJ;
    a.spos = L.spos; a.rpos = L.rpos; a.Jg = L.Jg; a.jmap = L.jmap; a.Sg = L.Sg; a.Rg = L.Rg; a.T = L.T;
    a.XJR = L.XJR; a.G = L.G; a.XRR = L.XRR; a.Xinv = L.Xinv;
    a.XJR32 = L.XJR32; a.G32 = L.G32; a.Xinv32 = L.Xinv32; a.T32 = L.T32;
    a.logdet_part = L.logdet_part; a.sign_part = L.sign_part; a.flag = flag;
    const size_t D = sizeof(double);
    const size_t nm = (size_t)L.nmax;
    const size_t tsz = nm * nm / 4 + 1;                    // |S| |R| <= n^2 / 4
    const size_t lim = (size_t)elim_lds_limit() - 8192;    // room for the static tables
    // widest tile (32, 16, 8 or 4 lines) whose buffers fit beside `fixed` doubles
    auto tile_w = [&](size_t fixed, size_t bufs) {
        for (int tw = kTileMax; tw >= 4; tw >>= 1)
            if (D * (fixed + bufs * nm * tw) <= lim) return tw;
        return 0;
    };
    // at most 16 lines per tile: the smaller LDS footprint keeps more workgroups per CU,
    // which measured faster than 32-line tiles (leaf colours: 8.4 -> 8.0 ms per level)
    const PlanParams pp = plan_params(nboxes);
    const int twr = std::min(pp.elim_tw, tile_w(tsz, 1));
    const int twg = std::min(pp.elim_tw, tile_w(2 * kTileMax, 2));   // column tiles: ld nmax + 1
    if (twr == 0 || twg == 0) return -1;
    const size_t lr = D * (tsz + nm * twr);
    set_lds(k_elim_rows<256, ST>, lr);
    const int ntr = (L.ldJ + L.nmax + twr - 1) / twr;
    const int pr = tiles_per_wg(ntr, nboxes), gr = (ntr + pr - 1) / pr;
    note_shape("elim_rows_w" + std::to_string(twr) + "_tpw" + std::to_string(pr));
    k_elim_rows<256, ST><<<dim3(xcd_grid(gr, nboxes)), dim3(256), lr, s>>>(a, boxes, nboxes, gr, mixed, work,
                                                                      (int)tsz, twr, pr);
    const size_t base = tsz + 4 * nm;
    // X_RR in LDS only for the LDS Gauss-Jordan: not when every r fits the register form
    // (r <= nmax <= 64 with 256 threads, <= 128 with 1024)
    const bool wide_inv = pp.inv_threads == 1024;
    const bool reg_only = wide_inv ? L.nmax <= 128 : L.nmax <= 64;
    const bool xl = !reg_only && D * (base + nm * nm) <= lim;
    const int zs = D * (base + tsz + (xl ? nm * nm : 0)) <= lim ? 1 : 0;
    const size_t li = D * (base + (zs ? tsz : 0) + (xl ? nm * nm : 0));
    // many boxes: small workgroups, several per CU; few boxes: one large workgroup each
    note_shape(std::string("elim_inv_") + (wide_inv ? "1024" : "256") + (xl ? "_xlds" : "") + (zs ? "_zs" : ""));
    if (!wide_inv) {
        if (xl) {
            set_lds(k_elim_inv<true, 256, ST>, li);
            k_elim_inv<true, 256, ST><<<dim3(nboxes), dim3(256), li, s>>>(a, boxes, mixed, work, flag, (int)tsz, zs);
        } else {
            set_lds(k_elim_inv<false, 256, ST>, li);
            k_elim_inv<false, 256, ST><<<dim3(nboxes), dim3(256), li, s>>>(a, boxes, mixed, work, flag, (int)tsz, zs);
        }
    } else if (xl) {
        set_lds(k_elim_inv<true, 1024, ST>, li);
        k_elim_inv<true, 1024, ST><<<dim3(nboxes), dim3(1024), li, s>>>(a, boxes, mixed, work, flag, (int)tsz, zs);
    } else {
        set_lds(k_elim_inv<false, 1024, ST>, li);
        k_elim_inv<false, 1024, ST><<<dim3(nboxes), dim3(1024), li, s>>>(a, boxes, mixed, work, flag, (int)tsz, zs);
    }
    const int ntg = (L.ldJ + twg - 1) / twg;
    const int pg = tiles_per_wg(ntg, nboxes), gt = (ntg + pg - 1) / pg;
    const dim3 gg(xcd_grid(gt, nboxes));
    // X_RR^{-1} held in LDS for all tiles of the workgroup when it fits beside the tile
    const int xi = D * (nm + 1) * (twg + nm) <= (size_t)kElimGLds ? 1 : 0;
    const size_t lg = D * (nm + 1) * (twg + (xi ? nm : (size_t)twg));
    note_shape("elim_g_hb" + std::to_string(L.nmax <= 64 ? 1 : (L.nmax <= 128 ? 2 : 4)) + "_w" + std::to_string(twg) +
               "_tpw" + std::to_string(pg) + (xi ? "_xi" : ""));
    if (L.nmax <= 64) {
        set_lds(k_elim_g<256, 1>, lg);
        k_elim_g<256, 1><<<gg, dim3(256), lg, s>>>(a, boxes, nboxes, gt, mixed, flag, twg, pg, xi);
    } else if (L.nmax <= 128) {
        set_lds(k_elim_g<256, 2>, lg);
        k_elim_g<256, 2><<<gg, dim3(256), lg, s>>>(a, boxes, nboxes, gt, mixed, flag, twg, pg, xi);
    } else {
        set_lds(k_elim_g<256, 4>, lg);
        k_elim_g<256, 4><<<gg, dim3(256), lg, s>>>(a, boxes, nboxes, gt, mixed, flag, twg, pg, xi);
    }
    return 3;
}

int launch_elim(const Level& L, const int* boxes, int nboxes, int mixed, int weak, double* work, int* flag,
                const TileList& tl, hipStream_t s) {
    return L.store32 ? launch_elim_t<float>(L, boxes, nboxes, mixed, weak, work, flag, tl, s)
                     : launch_elim_t<double>(L, boxes, nboxes, mixed, weak, work, flag, tl, s);
}

}  // namespace rss
