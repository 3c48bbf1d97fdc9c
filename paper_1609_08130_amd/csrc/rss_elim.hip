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
#include "rss_internal.h"

namespace rss {

struct ElimArgs {
    double* store;
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
};

constexpr int kTile = 32;   // rows (or columns) of J per tile

// Dynamic LDS: Ts[tsz] | Xs[nmax*nmax] (when XLDS) | tile[nmax*kTile]
template <bool XLDS, int NTH>
__global__ void __launch_bounds__(NTH) k_elim(ElimArgs a, const int* __restrict__ boxes, int mixed,
                                              double* __restrict__ work, int* flag, int tsz) {
    extern __shared__ double dyn[];
    __shared__ int sp[kMaxBox], rp[kMaxBox];
    __shared__ const double* blk_nc[8];
    __shared__ const double* blk_cn[8];
    __shared__ const int* nap[8];
    __shared__ int nbox_[8];
    __shared__ int joff[9];
    __shared__ int nN;
    __shared__ int colswap[kMaxBox];
    __shared__ double fvec[kMaxBox];
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
    const int nmax = a.nmax, ldJ = a.ldJ, nb = a.nb;
    const int64_t bsz = (int64_t)nmax * nmax;
    const int cx = c % nb, cy = c / nb;
    double* Ts = dyn;
    double* Xs = XLDS ? dyn + tsz : work + (int64_t)blockIdx.x * bsz;
    double* tile = dyn + tsz + (XLDS ? bsz : 0);
    const int ldx = nmax;

    for (int i = tid; i < k; i += NTH) sp[i] = a.spos[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += NTH) rp[i] = a.rpos[(int64_t)c * nmax + i];
    if (tid == 0) {
        int cntN = 0;
        joff[0] = k;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0) continue;
                int ox = cx + dx, oy = cy + dy;
                if (ox < 0 || oy < 0 || ox >= nb || oy >= nb) continue;
                int o = ox + nb * oy;
                blk_nc[cntN] = a.store + ((int64_t)o * kNbr + nbr_slot(-dx, -dy)) * bsz;   // A(B_o, B_c)
                blk_cn[cntN] = a.store + ((int64_t)c * kNbr + nbr_slot(dx, dy)) * bsz;     // A(B_c, B_o)
                nap[cntN] = a.apos + (int64_t)o * nmax;
                nbox_[cntN] = o;
                joff[cntN + 1] = joff[cntN] + a.nact[o];
                ++cntN;
            }
        nN = cntN;
    }
    const double* Tg = a.T + (int64_t)c * bsz;
    for (int e = tid; e < k * r; e += NTH) Ts[e] = Tg[(e % k) + (int64_t)(e / k) * nmax];   // Ts[q + b*k]
    __syncthreads();
    const int nj = joff[nN];
    const double* Acc = a.store + ((int64_t)c * kNbr + 12) * bsz;

    // J list (global indices)
    for (int jj = tid; jj < nj; jj += NTH) {
        int g;
        if (jj < k) {
            g = a.gidx[(int64_t)c * nmax + sp[jj]];
        } else {
            int i = 0;
            while (joff[i + 1] <= jj) ++i;
            g = a.gidx[(int64_t)nbox_[i] * nmax + nap[i][jj - joff[i]]];
        }
        a.Jg[(int64_t)c * ldJ + jj] = g;
    }

    // ---- X_JR = A_JR - A_JS T, kTile rows at a time (rows staged in LDS) ----
    double* XJR = a.XJR + (int64_t)c * ldJ * nmax;
    for (int r0 = 0; r0 < nj; r0 += kTile) {
        const int tr = min(kTile, nj - r0);
        // stage the rows' S columns then R columns: tile[i + kTile * col], col < n
        for (int e = tid; e < tr * n; e += NTH) {
            int i = e % tr, col = e / tr;
            int jj = r0 + i;
            const double* blk;
            int row;
            if (jj < k) {
                blk = Acc;
                row = sp[jj];
            } else {
                int s = 0;
                while (joff[s + 1] <= jj) ++s;
                blk = blk_nc[s];
                row = nap[s][jj - joff[s]];
            }
            int pos = col < k ? sp[col] : rp[col - k];
            tile[i + kTile * col] = blk[row + (int64_t)pos * nmax];
        }
        __syncthreads();
        for (int e = tid; e < tr * r; e += NTH) {
            int i = e % tr, b = e / tr;
            double v = tile[i + kTile * (k + b)];
            const double* tb = Ts + b * k;
            for (int q = 0; q < k; ++q) v -= tile[i + kTile * q] * tb[q];
            XJR[(r0 + i) + (int64_t)b * ldJ] = v;
        }
        __syncthreads();
    }

    // ---- X_RR = A_RR - A_RS T - T^T Z_S -----------------------------------------
    double* XRR = a.XRR + (int64_t)c * bsz;
    for (int e = tid; e < r * r; e += NTH) {
        int b = e % r, b2 = e / r;
        double v = Acc[rp[b] + (int64_t)rp[b2] * nmax];
        const double* t2 = Ts + b2 * k;
        const double* t1 = Ts + b * k;
        for (int q = 0; q < k; ++q) v -= Acc[rp[b] + (int64_t)sp[q] * nmax] * t2[q];
        for (int q = 0; q < k; ++q) v -= t1[q] * XJR[q + (int64_t)b2 * ldJ];
        XRR[b + (int64_t)b2 * nmax] = v;
        Xs[b + b2 * ldx] = v;
    }
    __syncthreads();

    // ---- X_RR^{-1} by in-place Gauss-Jordan with partial pivoting ---------------------
    double ld_sum = 0.0;
    int sgn = 1;
    bool singular = false;
    const int wv = tid >> 6, lane = tid & 63;
    for (int j = 0; j < r; ++j) {
        if (wv == 0) {
            double best = -1.0;
            int bi = 1 << 30;
            for (int i = j + lane; i < r; i += 64) {
                double v = fabs(Xs[i + j * ldx]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                double v2 = __shfl_xor(best, o, 64);
                int i2 = __shfl_xor(bi, o, 64);
                if (v2 > best || (v2 == best && i2 < bi)) { best = v2; bi = i2; }
            }
            if (lane == 0) { piv_idx = bi; piv_val = best; }
        }
        __syncthreads();
        const int p = piv_idx;
        if (!(piv_val > 0.0)) { singular = true; break; }
        if (p != j) {
            for (int l = tid; l < r; l += NTH) {
                double t0 = Xs[j + l * ldx];
                Xs[j + l * ldx] = Xs[p + l * ldx];
                Xs[p + l * ldx] = t0;
            }
            sgn = -sgn;
        }
        if (tid == 0) colswap[j] = p;
        __syncthreads();
        const double d = Xs[j + j * ldx];
        ld_sum += log(fabs(d));
        if (d < 0) sgn = -sgn;
        const double rinv = 1.0 / d;
        for (int i = tid; i < r; i += NTH) fvec[i] = (i == j) ? 0.0 : Xs[i + j * ldx];
        __syncthreads();
        for (int l = tid; l < r; l += NTH) Xs[j + l * ldx] = (l == j ? 1.0 : Xs[j + l * ldx]) * rinv;
        __syncthreads();
        for (int e = tid; e < r * r; e += NTH) {
            int i = e % r, l = e / r;
            if (i == j) continue;
            double base = (l == j) ? 0.0 : Xs[i + l * ldx];
            Xs[i + l * ldx] = base - fvec[i] * Xs[j + l * ldx];
        }
        __syncthreads();
    }
    if (singular) {
        if (tid == 0) { atomicOr(flag, 4); a.nJ[c] = 0; }
        return;
    }
    // undo the row interchanges on the columns of the inverse
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
    if (tid == 0) {
        a.logdet_part[c] = ld_sum;
        a.sign_part[c] = sgn;
    }
    double* Xinv = a.Xinv + (int64_t)c * bsz;
    for (int e = tid; e < r * r; e += NTH) {
        int b = e % r, b2 = e / r;
        Xinv[b + (int64_t)b2 * nmax] = Xs[b + b2 * ldx];
    }

    // ---- G = X_RR^{-1} X_RJ, kTile columns of J at a time ------------------------------
    double* G = a.G + (int64_t)c * nmax * ldJ;
    for (int c0 = 0; c0 < nj; c0 += kTile) {
        const int tc = min(kTile, nj - c0);
        // tile[b + r * j'] = X_RJ[b, c0 + j']
        for (int e = tid; e < tc * r; e += NTH) {
            int b = e % r, jp = e / r;
            int jj = c0 + jp;
            const double* blk;
            int col;
            if (jj < k) {
                blk = Acc;
                col = sp[jj];
            } else {
                int s = 0;
                while (joff[s + 1] <= jj) ++s;
                blk = blk_cn[s];
                col = nap[s][jj - joff[s]];
            }
            const double* bc = blk + (int64_t)col * nmax;
            double v = bc[rp[b]];
            const double* tb = Ts + b * k;
            for (int q = 0; q < k; ++q) v -= tb[q] * bc[sp[q]];
            tile[b + r * jp] = v;
        }
        __syncthreads();
        for (int e = tid; e < tc * r; e += NTH) {
            int b = e % r, jp = e / r;
            const double* tcol = tile + r * jp;
            double v = 0.0;
            for (int q = 0; q < r; ++q) v += Xs[b + q * ldx] * tcol[q];
            G[b + (int64_t)(c0 + jp) * nmax] = v;
        }
        __syncthreads();
    }

    // ---- bookkeeping: record sets, FP32 copies, active list of c becomes S ---------------
    for (int i = tid; i < k; i += NTH) a.Sg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + sp[i]];
    for (int i = tid; i < r; i += NTH) a.Rg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + rp[i]];
    if (mixed) {
        __syncthreads();
        for (int e = tid; e < nj * r; e += NTH) {
            int jj = e % nj, b = e / nj;
            a.XJR32[(int64_t)c * ldJ * nmax + jj + (int64_t)b * ldJ] = (float)XJR[jj + (int64_t)b * ldJ];
        }
        for (int e = tid; e < r * nj; e += NTH) {
            int b = e % r, jj = e / r;
            a.G32[(int64_t)c * nmax * ldJ + b + (int64_t)jj * nmax] = (float)G[b + (int64_t)jj * nmax];
        }
        for (int e = tid; e < r * r; e += NTH) {
            int b = e % r, b2 = e / r;
            a.Xinv32[(int64_t)c * bsz + b + (int64_t)b2 * nmax] = (float)Xs[b + b2 * ldx];
        }
        for (int e = tid; e < k * r; e += NTH) {
            int q = e % k, b = e / k;
            a.T32[(int64_t)c * bsz + q + (int64_t)b * nmax] = (float)Ts[q + b * k];
        }
    }
    if (tid == 0) {
        a.nJ[c] = nj;
        a.nact[c] = k;
    }
    for (int i = tid; i < k; i += NTH) a.apos[(int64_t)c * nmax + i] = sp[i];
}

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

void launch_elim(const Level& L, const int* boxes, int nboxes, int mixed, double* work, int* flag,
                 hipStream_t s) {
    if (nboxes <= 0) return;
    ElimArgs a;
    a.store = L.store; a.nb = L.nb; a.nmax = L.nmax; a.ldJ = L.ldJ;
    a.cnt = L.cnt; a.gidx = L.gidx; a.nact = L.nact; a.apos = L.apos; a.krank = L.krank; a.nJ = L.nJ;
    a.spos = L.spos; a.rpos = L.rpos; a.Jg = L.Jg; a.Sg = L.Sg; a.Rg = L.Rg; a.T = L.T;
    a.XJR = L.XJR; a.G = L.G; a.XRR = L.XRR; a.Xinv = L.Xinv;
    a.XJR32 = L.XJR32; a.G32 = L.G32; a.Xinv32 = L.Xinv32; a.T32 = L.T32;
    a.logdet_part = L.logdet_part; a.sign_part = L.sign_part;
    const int tsz = (L.nmax * L.nmax) / 4 + 1;            // |S| |R| <= n^2 / 4
    const size_t tile = (size_t)L.nmax * kTile;
    const size_t with_x = sizeof(double) * (tsz + (size_t)L.nmax * L.nmax + tile);
    const size_t without_x = sizeof(double) * (tsz + tile);
    // few boxes in a colour (upper levels): one large workgroup per box to cut latency
    const bool big = nboxes < 512;
    if ((int)with_x <= elim_lds_limit()) {
        if (big) {
            hipFuncSetAttribute((const void*)k_elim<true, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)with_x);
            k_elim<true, 1024><<<dim3(nboxes), dim3(1024), with_x, s>>>(a, boxes, mixed, work, flag, tsz);
        } else {
            hipFuncSetAttribute((const void*)k_elim<true, 256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)with_x);
            k_elim<true, 256><<<dim3(nboxes), dim3(256), with_x, s>>>(a, boxes, mixed, work, flag, tsz);
        }
    } else {
        if (big) {
            hipFuncSetAttribute((const void*)k_elim<false, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)without_x);
            k_elim<false, 1024><<<dim3(nboxes), dim3(1024), without_x, s>>>(a, boxes, mixed, work, flag, tsz);
        } else {
            hipFuncSetAttribute((const void*)k_elim<false, 256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)without_x);
            k_elim<false, 256><<<dim3(nboxes), dim3(256), without_x, s>>>(a, boxes, mixed, work, flag, tsz);
        }
    }
}

}  // namespace rss
