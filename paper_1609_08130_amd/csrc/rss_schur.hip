// Schur complement update of one skeletonization step (Section 2.1,
// S_JJ = A_JJ - A_JR A_RR^{-1} A_RJ, here A_JJ -= X_JR G with G = X_RR^{-1} X_RJ).
//
// The |J| x |J| update is computed in 64 x 64 tiles and subtracted in place from the
// block store: J row jj lies in box slot s (the 3x3 neighbourhood of c) at position p of
// that box's level-start list, so entry (jj, ll) lives in block (box(s_jj), box(s_ll)) of
// the store.  Boxes of one colour have disjoint neighbourhoods, so no two workgroups of
// a launch write the same entry and no atomics are needed.
//
// TT = double: FP64 products subtracted from the FP64 store.  TT = float (mixed
// precision): the products of the FP32 copies of X_JR and G are accumulated in FP32 and
// subtracted from the store of entry type ST (FP32 in mixed factorizations).
#include <type_traits>

#include "rss_internal.h"

namespace rss {

struct SchurArgs {
    void* store;   // entries of type ST
    double* dstore;   // self blocks of an FP32 store (FP64), or nullptr
    int nb, nmax, ldJ;
    const int* cnt;
    const int* nact;
    const int* apos;
    const int* krank;
    const int* nJ;
    const int* spos;
    const void* XJR;
    const void* G;
};

typedef double f64x4 __attribute__((ext_vector_type(4)));   // accumulator of one FP64 MFMA block

template <typename TT, typename ST, bool ATOM>
__global__ void __launch_bounds__(256) k_schur(SchurArgs a, const int* __restrict__ boxes,
                                               const int* __restrict__ tl_cnt, const int* __restrict__ tl_tiles,
                                               int tl_capx) {
    constexpr int TM = 64, TK = 16;
    __shared__ TT As[TK][TM + 1];
    __shared__ TT Bs[TK][TM + 1];
    __shared__ int rslot[TM], rpos_[TM], cslot[TM], cpos_[TM];
    __shared__ int slot_box[9];
    __shared__ int slot_nact[9];
    __shared__ int joff[10];
    __shared__ int jslot[9];
    __shared__ int64_t blkoff[81];   // [row slot * 9 + column slot]: first entry of that block
                                     // (in dstore for the self blocks, slot pairs s s, when set)

    const int tid = threadIdx.x;
    // Workgroups are dealt to the 8 XCDs round-robin in launch order: workgroup x + 8 s
    // takes entry s of tile list x, which holds the active tiles of the boxes at positions
    // bi = x mod 8 of the colour, so all tiles of a box run on one XCD and its X_JR and G
    // stay in one L2.  Workgroups past the end of their list leave after one load.
    const int xcd = blockIdx.x & 7, sidx = blockIdx.x >> 3;
    if (sidx >= tl_cnt[xcd]) return;
    const int ent = tl_tiles[(int64_t)xcd * tl_capx + sidx];
    const int bi = ent >> 12, ti = (ent >> 6) & 63, tj = ent & 63;
    const int c = boxes[bi];
    const int nj = a.nJ[c];
    if (nj == 0 || ti * TM >= nj || tj * TM >= nj) return;
    const int n = a.cnt[c], k = a.krank[c], r = n - k;
    if (r <= 0) return;
    const int nmax = a.nmax, ldJ = a.ldJ, nb = a.nb;
    const int64_t bsz = (int64_t)nmax * nmax;
    const int cx = c % nb, cy = c / nb;
    const int row0 = ti * TM, col0 = tj * TM;
    const TT* XJR = (const TT*)a.XJR + (int64_t)c * ldJ * nmax;
    const TT* G = (const TT*)a.G + (int64_t)c * nmax * ldJ;
    // slab k0 of X_JR (rows row0..) and G (columns col0..) into registers; the loads of
    // the first slab are in flight during the set-up below, those of slab s + 1 during
    // the products of slab s
    constexpr int PER = TM * TK / 256;
    TT va[PER], vb[PER];
    auto load_slab = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            const int i = e % TM, kk = e / TM;
            const int row = row0 + i, kc = k0 + kk;
            va[u] = (row < nj && kc < r) ? XJR[row + (int64_t)kc * ldJ] : (TT)0;
            const int kb = e % TK, j = e / TK;
            const int col = col0 + j, kc2 = k0 + kb;
            vb[u] = (col < nj && kc2 < r) ? G[kc2 + (int64_t)col * nmax] : (TT)0;
        }
    };
    load_slab(0);
    if (tid < 9) {
        // slot s = (dy + 1) 3 + (dx + 1) of the 3x3 neighbourhood; the active counts are
        // loaded by nine threads at once
        const int ox = cx + tid % 3 - 1, oy = cy + tid / 3 - 1;
        const int box = (ox < 0 || oy < 0 || ox >= nb || oy >= nb) ? -1 : ox + nb * oy;
        slot_box[tid] = box;
        slot_nact[tid] = box < 0 ? 0 : a.nact[box];
    }
    __syncthreads();
    if (tid == 0) {
        // J segments: S of c (slot 4), then adjacent boxes in ascending index
        joff[0] = 0;
        jslot[0] = 4;
        joff[1] = k;
        int cntS = 1;
        for (int s = 0; s < 9; ++s) {
            if (s == 4 || slot_box[s] < 0) continue;
            jslot[cntS] = s;
            joff[cntS + 1] = joff[cntS] + slot_nact[s];
            ++cntS;
        }
    } else if (tid >= 64 && tid < 64 + 81) {
        // block (row box of slot sa, column box of slot sb): offset (sb - sa) in the 3x3 grid
        const int sa = (tid - 64) / 9, sb = (tid - 64) % 9;
        const int abox = slot_box[sa];
        blkoff[tid - 64] = (abox < 0 || slot_box[sb] < 0) ? (int64_t)-1
                           : (sa == sb && a.dstore)     ? (int64_t)abox * bsz
                                                        : ((int64_t)abox * kNbr + nbr_slot(sb % 3 - sa % 3, sb / 3 - sa / 3)) * bsz;
    }
    __syncthreads();
    if (tid < 2 * TM) {
        int i = tid & (TM - 1);
        int jj = (tid < TM ? ti : tj) * TM + i;
        int sl = -1, ps = 0;
        if (jj < nj) {
            int seg = 0;
            while (joff[seg + 1] <= jj) ++seg;
            sl = jslot[seg];
            int box = slot_box[sl];
            int loc = jj - joff[seg];
            ps = (seg == 0) ? a.spos[(int64_t)c * nmax + loc] : a.apos[(int64_t)box * nmax + loc];
        }
        if (tid < TM) { rslot[i] = sl; rpos_[i] = ps; }
        else { cslot[i] = sl; cpos_[i] = ps; }
    }
    // The 64 x 64 product, 16 entries per thread.  FP64 (TT = double): on the matrix cores,
    // transposed (D[col][row] = sum_k G[k][col] X_JR[row][k]) so that the 16 lanes of a result
    // row cover 16 consecutive J rows; wave w takes the 32 x 32 quadrant (rows 32 (w % 2),
    // columns 32 (w / 2)) as 2 x 2 blocks of 16 x 16, one 16x16x4 MFMA per block and 4
    // values of k, lane l supplying A[l % 16][l / 16] = G[k][col] and B[l / 16][l % 16] =
    // X_JR[row][k] and receiving D[l / 16 + 4 v][l % 16] as value v.  FP32 (mixed): vector
    // FMAs on a 4 x 4 register tile per thread (rows tx + 16 u, columns ty + 16 v), which
    // measured faster here than the FP32 matrix-core form.
    constexpr bool kMfma = std::is_same<TT, double>::value;
    const int lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int qr = (wv & 1) * 32, qc = (wv >> 1) * 32;
    const int tx = tid & 15, ty = tid >> 4;
    // entry e < 16 of the thread: tile row and column
    auto erow = [&](int e) -> int {
        if constexpr (kMfma) return qr + 16 * ((e >> 2) & 1) + l16;
        else return tx + 16 * (e & 3);
    };
    auto ecol = [&](int e) -> int {
        if constexpr (kMfma) return qc + 16 * (e >> 3) + l4 + 4 * (e & 3);
        else return ty + 16 * (e >> 2);
    };
    f64x4 macc[2][2];   // [column block][row block] (matrix-core form)
    TT vacc[16];        // [e] (vector form)
#pragma unroll
    for (int e = 0; e < 16; ++e) vacc[e] = 0;
#pragma unroll
    for (int ci = 0; ci < 2; ++ci)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) macc[ci][ri] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < r; k0 += TK) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            As[e / TM][e % TM] = va[u];
            Bs[e % TK][e / TK] = vb[u];
        }
        __syncthreads();
        if (k0 + TK < r) load_slab(k0 + TK);
        if constexpr (kMfma) {
#pragma unroll
            for (int kk = 0; kk < TK; kk += 4) {
                double ga[2], xb[2];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) ga[ci] = Bs[kk + l4][qc + 16 * ci + l16];
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) xb[ri] = As[kk + l4][qr + 16 * ri + l16];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                    for (int ri = 0; ri < 2; ++ri)
                        macc[ci][ri] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[ci], xb[ri], macc[ci][ri], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < TK; ++kk) {
                TT av[4], bv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) av[u] = As[kk][tx + 16 * u];
#pragma unroll
                for (int v = 0; v < 4; ++v) bv[v] = Bs[kk][ty + 16 * v];
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int u = 0; u < 4; ++u) vacc[u + 4 * v] += av[u] * bv[v];
            }
        }
    }
    auto eval = [&](int e) -> TT {
        if constexpr (kMfma) return macc[e >> 3][(e >> 2) & 1][e & 3];
        else return vacc[e];
    };
    // read-modify-write of the 16 entries: all loads are issued, without branches, before
    // the first store; an entry outside J reads entry 0 of the store and is not written
    ST* st = (ST*)a.store;
    auto entry = [&](int e) -> int64_t {
        const int i = erow(e), j = ecol(e);
        const int sa = rslot[i], sb = cslot[j];
        const bool in = (sa | sb) >= 0;
        const int64_t off = blkoff[in ? sa * 9 + sb : 0] + rpos_[i] + (int64_t)cpos_[j] * nmax;
        return in ? off : (int64_t)-1;
    };
    if constexpr (ATOM) {
        // Every entry has one writer per launch (the neighbourhoods of one colour are
        // disjoint), so a no-return atomic add of -(X_JR G)_e rounds once, exactly as the
        // load-subtract-store below, and the workgroup waits for no load.
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t off = entry(e);
            if (off < 0) continue;
            if (a.dstore && rslot[erow(e)] == cslot[ecol(e)]) unsafeAtomicAdd(a.dstore + off, -(double)eval(e));
            else unsafeAtomicAdd(st + off, -(ST)eval(e));
        }
        return;
    }
    if (a.dstore) {
        // FP32 store with FP64 self blocks: an entry of a self block (row and column slot
        // equal) is updated in FP64, every other entry in ST as below
        double* ds = a.dstore;
        auto self = [&](int e) -> bool { return rslot[erow(e)] == cslot[ecol(e)]; };
        double old[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t off = max(entry(e), (int64_t)0);
            old[e] = self(e) ? ds[off] : (double)st[off];
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) asm volatile("" ::"v"(old[e]));
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t off = entry(e);
            if (off < 0) continue;
            if (self(e)) ds[off] = old[e] - (double)eval(e);
            else st[off] = (ST)old[e] - (ST)eval(e);
        }
        return;
    }
    ST old[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) old[e] = st[max(entry(e), (int64_t)0)];
    // keep every load here, ahead of the stores (the compiler would otherwise move a load
    // into the conditional store below and wait for it there)
#pragma unroll
    for (int e = 0; e < 16; ++e) asm volatile("" ::"v"(old[e]));
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t off = entry(e);
        if (off >= 0) st[off] = old[e] - (ST)eval(e);
    }
}

int schur_tile_capx(int nboxes, int maxJ) {
    const int tpd = (maxJ + 63) / 64;
    return tpd * tpd * ((nboxes + 7) / 8);
}

int launch_schur(const Level& L, const int* boxes, int nboxes, int maxJ, int mixed, int fp64_tiles,
                 const TileList& tl, hipStream_t s) {
    if (nboxes <= 0) return 0;
    if (tl.capx < schur_tile_capx(nboxes, maxJ)) return -1;
    SchurArgs a;
    a.store = L.store; a.dstore = L.dstore; a.nb = L.nb; a.nmax = L.nmax; a.ldJ = L.ldJ;
    a.cnt = L.cnt; a.nact = L.nact; a.apos = L.apos; a.krank = L.krank; a.nJ = L.nJ; a.spos = L.spos;
    const int tpd = (maxJ + 63) / 64;
    const int64_t nwg = 8 * (int64_t)tpd * tpd * ((nboxes + 7) / 8);   // 8 lists of at most capx entries
    dim3 grid((unsigned)nwg), block(256);
    const bool atom = plan_params(nboxes).schur_atomic != 0;
    const std::string form = atom ? "_atomic" : "";
    if (mixed && !fp64_tiles) {
        note_shape(std::string("schur_f32") + (L.store32 ? "_store32" : "_store64") + form);
        a.XJR = L.XJR32; a.G = L.G32;
        if (L.store32) {
            if (atom) k_schur<float, float, true><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
            else k_schur<float, float, false><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
        } else {
            if (atom) k_schur<float, double, true><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
            else k_schur<float, double, false><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
        }
    } else {
        note_shape(std::string(fp64_tiles ? "schur_f64_sxs" : "schur_f64") + (L.store32 ? "_store32" : "_store64") + form);
        a.XJR = L.XJR; a.G = L.G;
        if (L.store32) {
            if (atom) k_schur<double, float, true><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
            else k_schur<double, float, false><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
        } else {
            if (atom) k_schur<double, double, true><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
            else k_schur<double, double, false><<<grid, block, 0, s>>>(a, boxes, tl.cnt, tl.tiles, tl.capx);
        }
    }
    return 0;
}

}  // namespace rss
