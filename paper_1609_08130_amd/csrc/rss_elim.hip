// Decoupling and elimination of the redundant DOFs of one box per workgroup
// (Section 3.1, the U_T / L_T pair and eq. zab; Section 2.1, eqs. landu and
// block_elimination with I = R, J = S u N, K = F).
//
// With the box's ID (S, R, T) and the current blocks of the store:
//   Z_X  = A_XR - A_XS T                   X in {S, N}     (column operation L_T)
//   X_RR = A_RR - A_RS T - T^T (A_SR - A_SS T)             (both operations)
//   X_RJ = A_RJ - T^T A_SJ                 J = S u N       (row operation U_T)
//   X_JR = [Z_S; Z_N]
// then X_RR = P L U (partial pivoting), G = X_RR^{-1} X_RJ and the explicit X_RR^{-1}.
// The record keeps T, X_JR, G, X_RR and X_RR^{-1}; the Schur complement
// A_JJ -= X_JR G is applied by the Schur kernel.  J lists S first, then the active
// DOFs of the adjacent boxes in ascending box index.
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

constexpr int kTLds = 4096;   // T kept in LDS when |S| |R| <= kTLds

__global__ void __launch_bounds__(256) k_elim(ElimArgs a, const int* __restrict__ boxes, int mixed,
                                              double* __restrict__ work, int* flag) {
    __shared__ int sp[kMaxBox], rp[kMaxBox];
    __shared__ double Ts[kTLds];
    __shared__ const double* blk_nc[8];
    __shared__ const double* blk_cn[8];
    __shared__ const int* nap[8];
    __shared__ int nbox_[8];
    __shared__ int joff[9];
    __shared__ int nN;
    __shared__ int piv[kMaxBox];
    __shared__ double red_v[256];
    __shared__ int red_i[256];
    __shared__ int singular;

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
    for (int i = tid; i < k; i += 256) sp[i] = a.spos[(int64_t)c * nmax + i];
    for (int i = tid; i < r; i += 256) rp[i] = a.rpos[(int64_t)c * nmax + i];
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
        singular = 0;
    }
    const double* Tg = a.T + (int64_t)c * bsz;
    const bool tl = k * r <= kTLds;
    if (tl)
        for (int e = tid; e < k * r; e += 256) Ts[e] = Tg[(e % k) + (int64_t)(e / k) * nmax];
    __syncthreads();
    const int ldT = tl ? k : nmax;
    const double* Tp = tl ? (const double*)Ts : Tg;
    const int nj = joff[nN];
    const double* Acc = a.store + ((int64_t)c * kNbr + 12) * bsz;

    // J list (global indices)
    for (int jj = tid; jj < nj; jj += 256) {
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
    // X_JR = A_JR - A_JS T
    double* XJR = a.XJR + (int64_t)c * ldJ * nmax;
    for (int e = tid; e < nj * r; e += 256) {
        int jj = e % nj, b = e / nj;
        const double* blk;
        int row;
        if (jj < k) {
            blk = Acc;
            row = sp[jj];
        } else {
            int i = 0;
            while (joff[i + 1] <= jj) ++i;
            blk = blk_nc[i];
            row = nap[i][jj - joff[i]];
        }
        double v = blk[row + (int64_t)rp[b] * nmax];
        for (int q = 0; q < k; ++q) v -= blk[row + (int64_t)sp[q] * nmax] * Tp[q + b * ldT];
        XJR[jj + (int64_t)b * ldJ] = v;
    }
    // X_RJ = A_RJ - T^T A_SJ, written into G's storage (r x |J|, ld nmax)
    double* G = a.G + (int64_t)c * nmax * ldJ;
    for (int e = tid; e < r * nj; e += 256) {
        int b = e % r, jj = e / r;
        const double* blk;
        int col;
        if (jj < k) {
            blk = Acc;
            col = sp[jj];
        } else {
            int i = 0;
            while (joff[i + 1] <= jj) ++i;
            blk = blk_cn[i];
            col = nap[i][jj - joff[i]];
        }
        const double* bc = blk + (int64_t)col * nmax;
        double v = bc[rp[b]];
        for (int q = 0; q < k; ++q) v -= Tp[q + b * ldT] * bc[sp[q]];
        G[b + (int64_t)jj * nmax] = v;
    }
    __syncthreads();
    // X_RR = A_RR - A_RS T - T^T Z_S   (Z_S = first k rows of X_JR)
    double* LU = work + (int64_t)blockIdx.x * bsz;
    double* XRR = a.XRR + (int64_t)c * bsz;
    for (int e = tid; e < r * r; e += 256) {
        int b = e % r, b2 = e / r;
        double v = Acc[rp[b] + (int64_t)rp[b2] * nmax];
        for (int q = 0; q < k; ++q) v -= Acc[rp[b] + (int64_t)sp[q] * nmax] * Tp[q + b2 * ldT];
        for (int q = 0; q < k; ++q) v -= Tp[q + b * ldT] * XJR[q + (int64_t)b2 * ldJ];
        XRR[b + (int64_t)b2 * nmax] = v;
        LU[b + (int64_t)b2 * nmax] = v;
    }
    __syncthreads();
    // LU with partial pivoting (largest |.|, lowest row on ties)
    double ld_sum = 0.0;
    int sgn = 1;
    for (int j = 0; j < r; ++j) {
        double best = -1.0;
        int bi = 1 << 30;
        for (int i = j + tid; i < r; i += 256) {
            double v = fabs(LU[i + (int64_t)j * nmax]);
            if (v > best || (v == best && i < bi)) { best = v; bi = i; }
        }
        red_v[tid] = best;
        red_i[tid] = bi;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) {
                double v2 = red_v[tid + s];
                int i2 = red_i[tid + s];
                if (v2 > red_v[tid] || (v2 == red_v[tid] && i2 < red_i[tid])) { red_v[tid] = v2; red_i[tid] = i2; }
            }
            __syncthreads();
        }
        const int p = red_i[0];
        const double pv = red_v[0];
        __syncthreads();
        if (!(pv > 0.0)) {
            if (tid == 0) singular = 1;
            break;
        }
        if (tid == 0) piv[j] = p;
        if (p != j) {
            for (int l = tid; l < r; l += 256) {
                double t0 = LU[j + (int64_t)l * nmax];
                LU[j + (int64_t)l * nmax] = LU[p + (int64_t)l * nmax];
                LU[p + (int64_t)l * nmax] = t0;
            }
            sgn = -sgn;
        }
        __syncthreads();
        const double d = LU[j + (int64_t)j * nmax];
        ld_sum += log(fabs(d));
        if (d < 0) sgn = -sgn;
        const double rinv = 1.0 / d;
        for (int i = j + 1 + tid; i < r; i += 256) LU[i + (int64_t)j * nmax] *= rinv;
        __syncthreads();
        const int m2 = r - j - 1;
        for (int e = tid; e < m2 * m2; e += 256) {
            int i = j + 1 + e % m2, l = j + 1 + e / m2;
            LU[i + (int64_t)l * nmax] -= LU[i + (int64_t)j * nmax] * LU[j + (int64_t)l * nmax];
        }
        __syncthreads();
    }
    if (singular) {
        if (tid == 0) atomicOr(flag, 4);
        if (tid == 0) a.nJ[c] = 0;
        return;
    }
    if (tid == 0) {
        a.logdet_part[c] = ld_sum;
        a.sign_part[c] = sgn;
    }
    // G = X_RR^{-1} X_RJ, column by column; X_RR^{-1} from the identity
    double* Xinv = a.Xinv + (int64_t)c * bsz;
    for (int col = tid; col < nj + r; col += 256) {
        double* x;
        if (col < nj) {
            x = G + (int64_t)col * nmax;
        } else {
            x = Xinv + (int64_t)(col - nj) * nmax;
            for (int i = 0; i < r; ++i) x[i] = (i == col - nj) ? 1.0 : 0.0;
        }
        for (int j = 0; j < r; ++j) {
            int p = piv[j];
            if (p != j) { double t0 = x[j]; x[j] = x[p]; x[p] = t0; }
        }
        for (int j = 0; j < r; ++j) {
            double xj = x[j];
            for (int i = j + 1; i < r; ++i) x[i] -= LU[i + (int64_t)j * nmax] * xj;
        }
        for (int j = r - 1; j >= 0; --j) {
            double xj = x[j] / LU[j + (int64_t)j * nmax];
            x[j] = xj;
            for (int i = 0; i < j; ++i) x[i] -= LU[i + (int64_t)j * nmax] * xj;
        }
    }
    // bookkeeping: record sets, active list of c becomes S
    for (int i = tid; i < k; i += 256) a.Sg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + sp[i]];
    for (int i = tid; i < r; i += 256) a.Rg[(int64_t)c * nmax + i] = a.gidx[(int64_t)c * nmax + rp[i]];
    __syncthreads();
    if (mixed) {
        for (int e = tid; e < nj * r; e += 256) {
            int jj = e % nj, b = e / nj;
            a.XJR32[(int64_t)c * ldJ * nmax + jj + (int64_t)b * ldJ] = (float)XJR[jj + (int64_t)b * ldJ];
        }
        for (int e = tid; e < r * nj; e += 256) {
            int b = e % r, jj = e / r;
            a.G32[(int64_t)c * nmax * ldJ + b + (int64_t)jj * nmax] = (float)G[b + (int64_t)jj * nmax];
        }
        for (int e = tid; e < r * r; e += 256) {
            int b = e % r, b2 = e / r;
            a.Xinv32[(int64_t)c * bsz + b + (int64_t)b2 * nmax] = (float)Xinv[b + (int64_t)b2 * nmax];
        }
        for (int e = tid; e < k * r; e += 256) {
            int q = e % k, b = e / k;
            a.T32[(int64_t)c * bsz + q + (int64_t)b * nmax] = (float)Tg[q + (int64_t)b * nmax];
        }
    }
    if (tid == 0) {
        a.nJ[c] = nj;
        a.nact[c] = k;
    }
    for (int i = tid; i < k; i += 256) a.apos[(int64_t)c * nmax + i] = sp[i];
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
    k_elim<<<dim3(nboxes), dim3(256), 0, s>>>(a, boxes, mixed, work, flag);
}

}  // namespace rss
