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

// Dynamic LDS: Ts[tsz] (T, b-fastest) | Xs[nmax*nmax] (when XLDS) | tA[nmax*kTile] | tX[nmax*kTile]
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
    __shared__ const double* srcp[kTile];
    __shared__ int srcpos[kTile];

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
    double* Ts = dyn;                                              // Ts[b + r q] = T[q][b]
    double* Xs = XLDS ? dyn + tsz : work + (int64_t)blockIdx.x * bsz;
    double* tA = dyn + tsz + (XLDS ? bsz : 0);
    double* tX = tA + (int64_t)nmax * kTile;
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
    for (int e = tid; e < k * r; e += NTH) {
        int b = e % r, q = e / r;
        Ts[e] = Tg[q + (int64_t)b * nmax];
    }
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

    // ---- X_JR = A_JR - A_JS T, kTile rows of J at a time ------------------------------
    double* XJR = a.XJR + (int64_t)c * ldJ * nmax;
    for (int r0 = 0; r0 < nj; r0 += kTile) {
        const int tr = min(kTile, nj - r0);
        if (tid < tr) {
            const int jj = r0 + tid;
            if (jj < k) {
                srcp[tid] = Acc;
                srcpos[tid] = sp[jj];
            } else {
                int s = 0;
                while (joff[s + 1] <= jj) ++s;
                srcp[tid] = blk_nc[s];
                srcpos[tid] = nap[s][jj - joff[s]];
            }
        }
        __syncthreads();
        // tA[i + kTile * col]: row i of the tile at B position (col < k ? sp[col] : rp[col - k])
        for (int e = tid; e < tr * n; e += NTH) {
            int i = e % tr, col = e / tr;
            int pos = col < k ? sp[col] : rp[col - k];
            tA[i + kTile * col] = srcp[i][srcpos[i] + (int64_t)pos * nmax];
        }
        __syncthreads();
        const int rh = (r + 1) >> 1;
        for (int e = tid; e < tr * rh; e += NTH) {
            const int i = e % tr, b = 2 * (e / tr);
            const bool two = b + 1 < r;
            double v0 = tA[i + kTile * (k + b)];
            double v1 = two ? tA[i + kTile * (k + b + 1)] : 0.0;
            for (int q = 0; q < k; ++q) {
                const double x = tA[i + kTile * q];
                v0 -= x * Ts[b + r * q];
                if (two) v1 -= x * Ts[b + 1 + r * q];
            }
            XJR[(r0 + i) + (int64_t)b * ldJ] = v0;
            if (two) XJR[(r0 + i) + (int64_t)(b + 1) * ldJ] = v1;
        }
        __syncthreads();
    }

    // ---- X_RR = A_RR - A_RS T - T^T Z_S ------------------------------------------------
    double* XRR = a.XRR + (int64_t)c * bsz;
    for (int e = tid; e < r * r; e += NTH) {
        int b = e % r, b2 = e / r;
        double v = Acc[rp[b] + (int64_t)rp[b2] * nmax];
        for (int q = 0; q < k; ++q) v -= Acc[rp[b] + (int64_t)sp[q] * nmax] * Ts[b2 + r * q];
        for (int q = 0; q < k; ++q) v -= Ts[b + r * q] * XJR[q + (int64_t)b2 * ldJ];
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
        for (int l = wv; l < r; l += NTH / 64) {
            const double xjl = Xs[j + l * ldx];
            for (int i = lane; i < r; i += 64) {
                if (i == j) continue;
                double base = (l == j) ? 0.0 : Xs[i + l * ldx];
                Xs[i + l * ldx] = base - fvec[i] * xjl;
            }
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

    // ---- G = X_RR^{-1} X_RJ, X_RJ = A_RJ - T^T A_SJ, kTile columns of J at a time ------
    double* G = a.G + (int64_t)c * nmax * ldJ;
    for (int c0 = 0; c0 < nj; c0 += kTile) {
        const int tc = min(kTile, nj - c0);
        if (tid < tc) {
            const int jj = c0 + tid;
            if (jj < k) {
                srcp[tid] = Acc;
                srcpos[tid] = sp[jj];
            } else {
                int s = 0;
                while (joff[s + 1] <= jj) ++s;
                srcp[tid] = blk_cn[s];
                srcpos[tid] = nap[s][jj - joff[s]];
            }
        }
        __syncthreads();
        // tA[pos + nmax * jp] = A(B_c position pos, J column c0 + jp)
        for (int e = tid; e < tc * n; e += NTH) {
            int pos = e % n, jp = e / n;
            tA[pos + nmax * jp] = srcp[jp][pos + (int64_t)srcpos[jp] * nmax];
        }
        __syncthreads();
        for (int e = tid; e < tc * r; e += NTH) {
            const int b = e % r, jp = e / r;
            const double* col = tA + nmax * jp;
            double v = col[rp[b]];
            for (int q = 0; q < k; ++q) v -= Ts[b + r * q] * col[sp[q]];
            tX[b + nmax * jp] = v;
        }
        __syncthreads();
        const int th = (tc + 1) >> 1;
        for (int e = tid; e < th * r; e += NTH) {
            const int b = e % r, jp = 2 * (e / r);
            const bool two = jp + 1 < tc;
            const double* x0 = tX + nmax * jp;
            const double* x1 = x0 + nmax;
            double v0 = 0.0, v1 = 0.0;
            for (int q = 0; q < r; ++q) {
                const double w = Xs[b + q * ldx];
                v0 += w * x0[q];
                if (two) v1 += w * x1[q];
            }
            G[b + (int64_t)(c0 + jp) * nmax] = v0;
            if (two) G[b + (int64_t)(c0 + jp + 1) * nmax] = v1;
        }
        __syncthreads();
    }

    // ---- bookkeeping: record sets, FP32 copies, active list of c becomes S ---------------
    for (int i = tid; i < k; i += NTH) a.Sg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + sp[i]];
    for (int i = tid; i < r; i += NTH) a.Rg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + rp[i]];
    if (mixed) {
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
            int b = e % r, q = e / r;
            a.T32[(int64_t)c * bsz + q + (int64_t)b * nmax] = (float)Ts[e];
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
    const size_t tile = 2 * (size_t)L.nmax * kTile;
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
