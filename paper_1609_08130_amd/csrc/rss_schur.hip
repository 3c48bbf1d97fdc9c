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
// subtracted from the store of entry type ST (FP32 in mixed factorizations).  Mixed
// precision keeps the self blocks A(B_a, B_a) in FP64 beside an FP32 store (dstore), and
// forms the S x S products of each step in FP64: the tile kernel leaves S x S to
// k_schur_self and updates the other self-block entries in a second read-modify-write pass
// (FP64 words), run only by tiles that hold such entries, so that no load of the first pass
// waits inside a branch on the entry type.
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
    const int* jmap;   // J row -> (3x3 slot << 16) | position in its box (written by k_elim_rows)
    const int* jseg;   // per 3x3 slot: (first J row << 16) | rows (written by k_elim_inv)
    const void* XJR;
    const void* G;
};

typedef double f64x4 __attribute__((ext_vector_type(4)));   // accumulator of one FP64 MFMA block
typedef float f32x4 __attribute__((ext_vector_type(4)));    // accumulator of one FP32 MFMA block

// MF (TT = float only): the FP32 products on the matrix cores (v_mfma_f32_16x16x4f32) instead
// of vector FMAs.
template <typename TT, typename ST, bool ATOM, bool MF = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(std::is_same<TT, double>::value ? 4 : 7))) k_schur(SchurArgs a, const int* __restrict__ tl_cnt,
                                               const int* __restrict__ tl_tiles, const int* __restrict__ tl_info,
                                               int tl_capx) {
    constexpr int TM = 64, TK = 16;
    __shared__ TT As[TK][TM + 1];
    __shared__ TT Bs[TK][TM + 1];
    __shared__ int rslot[TM], rpos_[TM], cslot[TM], cpos_[TM];
    __shared__ int64_t blkoff[81];   // [row slot * 9 + column slot]: first entry of that block
                                     // (-1: no such box, or S x S of a mixed factorization;
                                     // self blocks in dstore when set)
    __shared__ int slotmask[2];      // slots present among the tile's rows, columns

    const int tid = threadIdx.x;
    // Workgroups are dealt to the 8 XCDs round-robin in launch order: workgroup x + 8 s
    // takes entry s of tile list x, which holds the active tiles of the boxes at positions
    // bi = x mod 8 of the colour, so all tiles of a box run on one XCD and its X_JR and G
    // stay in one L2.  The list count, the entry (box, tile) and the box's |J| and |R| are
    // loaded together (every workgroup index is below the list capacity), so the slab loads
    // wait for one load latency; workgroups past the end of their list leave there.
    const int xcd = blockIdx.x & 7, sidx = blockIdx.x >> 3;
    const int64_t li = (int64_t)xcd * tl_capx + sidx;
    const int lcnt = tl_cnt[xcd], ent = tl_tiles[li], inf = tl_info[li];
    if (sidx >= lcnt) return;
    const int c = (int)(((unsigned)ent >> 12) | (((unsigned)inf >> 21) << 20)), ti = (ent >> 6) & 63, tj = ent & 63;
    const int nj = (inf >> 9) & 0xfff, r = inf & 0x1ff;
    if (nj == 0 || r <= 0 || ti * TM >= nj || tj * TM >= nj) return;
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
    // the tile's row and column maps (one load each) and the store offsets of the 81 blocks of
    // the neighbourhood, from the box coordinates alone (slot s = (dy + 1) 3 + (dx + 1))
    if (tid < 2) slotmask[tid] = 0;
    __syncthreads();
    if (tid < 2 * TM) {
        const int i = tid & (TM - 1);
        const int jj = (tid < TM ? ti : tj) * TM + i;
        const int m = jj < nj ? a.jmap[(int64_t)c * ldJ + jj] : -1;
        const int sl = m < 0 ? -1 : m >> 16, ps = m & 0xffff;
        if (tid < TM) { rslot[i] = sl; rpos_[i] = ps; }
        else { cslot[i] = sl; cpos_[i] = ps; }
        if (sl >= 0) atomicOr(&slotmask[tid >= TM], 1 << sl);
    } else if (tid < 2 * TM + 81) {
        const int sa = (tid - 2 * TM) / 9, sb = (tid - 2 * TM) % 9;
        const int ax = cx + sa % 3 - 1, ay = cy + sa / 3 - 1, bx = cx + sb % 3 - 1, by = cy + sb / 3 - 1;
        const bool in = ax >= 0 && ay >= 0 && ax < nb && ay < nb && bx >= 0 && by >= 0 && bx < nb && by < nb;
        const int64_t abox = ax + (int64_t)nb * ay;
        // mixed precision: S x S belongs to k_schur_self
        const bool sxs = !std::is_same<TT, double>::value && sa == 4 && sb == 4;
        blkoff[tid - 2 * TM] = (!in || sxs)             ? (int64_t)-1
                               : (sa == sb && a.dstore) ? abox * bsz
                                                        : (abox * kNbr + nbr_slot(sb % 3 - sa % 3, sb / 3 - sa / 3)) * bsz;
    }
    __syncthreads();
    // The 64 x 64 product, 16 entries per thread.  FP64 (TT = double): on the matrix cores,
    // transposed (D[col][row] = sum_k G[k][col] X_JR[row][k]) so that the 16 lanes of a result
    // row cover 16 consecutive J rows; wave w takes the 32 x 32 quadrant (rows 32 (w % 2),
    // columns 32 (w / 2)) as 2 x 2 blocks of 16 x 16, one 16x16x4 MFMA per block and 4
    // values of k, lane l supplying A[l % 16][l / 16] = G[k][col] and B[l / 16][l % 16] =
    // X_JR[row][k] and receiving D[l / 16 + 4 v][l % 16] as value v.  FP32 (mixed), MF: the
    // same blocks on v_mfma_f32_16x16x4f32, which returns D[4 (l / 16) + v][l % 16] as value v;
    // otherwise vector FMAs on a 4 x 4 register tile per thread (rows tx + 16 u, columns
    // ty + 16 v).
    constexpr bool kF64 = std::is_same<TT, double>::value;
    constexpr bool kMfma = kF64 || MF;
    const int lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int qr = (wv & 1) * 32, qc = (wv >> 1) * 32;
    const int tx = tid & 15, ty = tid >> 4;
    // entry e < 16 of the thread: tile row and column
    auto erow = [&](int e) -> int {
        if constexpr (kMfma) return qr + 16 * ((e >> 2) & 1) + l16;
        else return tx + 16 * (e & 3);
    };
    // FP64 blocks: lane l holds D[l / 16 + 4 v][l % 16] as value v; FP32 blocks: D[4 (l / 16) + v][l % 16]
    auto ecol = [&](int e) -> int {
        if constexpr (kF64) return qc + 16 * (e >> 3) + l4 + 4 * (e & 3);
        else if constexpr (kMfma) return qc + 16 * (e >> 3) + 4 * l4 + (e & 3);
        else return ty + 16 * (e >> 2);
    };
    typedef typename std::conditional<kF64, f64x4, f32x4>::type accv;
    accv macc[2][2];    // [column block][row block] (matrix-core form)
    TT vacc[16];        // [e] (vector form)
#pragma unroll
    for (int e = 0; e < 16; ++e) vacc[e] = 0;
#pragma unroll
    for (int ci = 0; ci < 2; ++ci)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) macc[ci][ri] = accv{0, 0, 0, 0};
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
                TT ga[2], xb[2];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) ga[ci] = Bs[kk + l4][qc + 16 * ci + l16];
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) xb[ri] = As[kk + l4][qr + 16 * ri + l16];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                    for (int ri = 0; ri < 2; ++ri) {
                        if constexpr (kF64)
                            macc[ci][ri] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[ci], xb[ri], macc[ci][ri], 0, 0, 0);
                        else
                            macc[ci][ri] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[ci], xb[ri], macc[ci][ri], 0, 0, 0);
                    }
            }
        } else {
            // the last slab stops at the first multiple of 4 not below |R| (its zero padding
            // would add only zero products)
            const int kn = min(TK, r - k0);
            for (int k4 = 0; k4 < kn; k4 += 4) {
#pragma unroll
                for (int kk = k4; kk < k4 + 4; ++kk) {
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
    }
    auto eval = [&](int e) -> TT {
        if constexpr (kMfma) return macc[e >> 3][(e >> 2) & 1][e & 3];
        else return vacc[e];
    };
    // read-modify-write of the 16 entries: all loads are issued, without branches, before
    // the first store; an entry outside J reads entry 0 of the store and is not written
    ST* st = (ST*)a.store;
    // entries in dstore: self blocks (row and column slot equal) when the store has one
    const bool ds = a.dstore != nullptr;
    auto entry = [&](int e, bool want_self) -> int64_t {
        const int i = erow(e), j = ecol(e);
        const int sa = rslot[i], sb = cslot[j];
        const int64_t bo = (sa | sb) >= 0 ? blkoff[sa * 9 + sb] : (int64_t)-1;
        return (bo < 0 || (ds && sa == sb) != want_self) ? (int64_t)-1 : bo + rpos_[i] + (int64_t)cpos_[j] * nmax;
    };
    // second pass: the FP64 self-block entries (only in tiles whose rows and columns share a
    // slot), loaded together at their offsets or at entry 0 without a branch
    auto self_pass = [&]() {
        if (!ds || !(slotmask[0] & slotmask[1])) return;
        double o64[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) o64[e] = a.dstore[max(entry(e, true), (int64_t)0)];
#pragma unroll
        for (int e = 0; e < 16; ++e) asm volatile("" ::"v"(o64[e]));
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t off = entry(e, true);
            if (off >= 0) a.dstore[off] = o64[e] - (double)eval(e);
        }
    };
    if constexpr (ATOM) {
        // Every entry has one writer per launch (the neighbourhoods of one colour are
        // disjoint), so a no-return atomic add of -(X_JR G)_e rounds once, exactly as the
        // load-subtract-store below, and the workgroup waits for no load.
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t off = entry(e, false);
            if (off >= 0) unsafeAtomicAdd(st + off, -(ST)eval(e));
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t off = ds ? entry(e, true) : (int64_t)-1;
            if (off >= 0) unsafeAtomicAdd(a.dstore + off, -(double)eval(e));
        }
        return;
    }
    ST old[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) old[e] = st[max(entry(e, false), (int64_t)0)];
    // keep every load here, ahead of the stores (the compiler would otherwise move a load
    // into the conditional store below and wait for it there)
#pragma unroll
    for (int e = 0; e < 16; ++e) asm volatile("" ::"v"(old[e]));
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t off = entry(e, false);
        if (off >= 0) st[off] = old[e] - (ST)eval(e);
    }
    self_pass();
}

// The S x S block of a step of a mixed factorization, with FP64 products: one workgroup per
// (box, 64 x 64 sub-tile of S x S), A(S, S) -= X_SR G_RS into the FP64 entries of the box's
// self block (dstore, or the FP64 store).  Same tile arithmetic and lane layout as k_schur;
// the slot-generic form (the J segment of any 3x3 slot, jseg) keeps TT and the slot as
// parameters.
template <typename TT>
__global__ void __launch_bounds__(256) k_schur_self(SchurArgs a, const int* __restrict__ boxes, int sl, int nsub) {
    constexpr int TM = 64, TK = 16, PER = TM * TK / 256;
    constexpr bool kF64 = std::is_same<TT, double>::value;
    __shared__ TT As[TK][TM + 1];
    __shared__ TT Bs[TK][TM + 1];
    __shared__ int rpos_[TM], cpos_[TM];
    const int tid = threadIdx.x;
    const int sub = blockIdx.x % (nsub * nsub);
    const int c = boxes[blockIdx.x / (nsub * nsub)];
    if (a.nJ[c] == 0) return;   // no elimination (the segment table is not written)
    const int seg = a.jseg[(int64_t)c * 9 + sl];
    const int j0 = seg >> 16, len = seg & 0xffff;
    const int u = sub % nsub, v = sub / nsub;
    if (seg == 0 || u * TM >= len || v * TM >= len) return;
    const int n = a.cnt[c], k = a.krank[c], r = n - k;
    const int nmax = a.nmax, ldJ = a.ldJ, nb = a.nb;
    const int64_t bsz = (int64_t)nmax * nmax;
    const int64_t abox = (c % nb + sl % 3 - 1) + (int64_t)nb * (c / nb + sl / 3 - 1);
    double* blk = a.dstore ? a.dstore + abox * bsz : (double*)a.store + (abox * kNbr + 12) * bsz;
    const int row0 = j0 + u * TM, col0 = j0 + v * TM;
    const int rl = min(TM, len - u * TM), cl = min(TM, len - v * TM);
    const TT* XJR = (const TT*)a.XJR + (int64_t)c * ldJ * nmax;
    const TT* G = (const TT*)a.G + (int64_t)c * nmax * ldJ;
    TT va[PER], vb[PER];
    auto load_slab = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            const int i = e % TM, kk = e / TM;
            va[q] = (i < rl && k0 + kk < r) ? XJR[row0 + i + (int64_t)(k0 + kk) * ldJ] : (TT)0;
            const int kb = e % TK, j = e / TK;
            vb[q] = (j < cl && k0 + kb < r) ? G[k0 + kb + (int64_t)(col0 + j) * nmax] : (TT)0;
        }
    };
    load_slab(0);
    if (tid < TM) rpos_[tid] = tid < rl ? (a.jmap[(int64_t)c * ldJ + row0 + tid] & 0xffff) : 0;
    else if (tid < 2 * TM) cpos_[tid - TM] = tid - TM < cl ? (a.jmap[(int64_t)c * ldJ + col0 + tid - TM] & 0xffff) : 0;
    const int lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int qr = (wv & 1) * 32, qc = (wv >> 1) * 32;
    typedef typename std::conditional<kF64, f64x4, f32x4>::type accv;
    accv macc[2][2];
#pragma unroll
    for (int ci = 0; ci < 2; ++ci)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) macc[ci][ri] = accv{0, 0, 0, 0};
    for (int k0 = 0; k0 < r; k0 += TK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            As[e / TM][e % TM] = va[q];
            Bs[e % TK][e / TK] = vb[q];
        }
        __syncthreads();
        if (k0 + TK < r) load_slab(k0 + TK);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
            TT ga[2], xb[2];
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) ga[ci] = Bs[kk + l4][qc + 16 * ci + l16];
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) xb[ri] = As[kk + l4][qr + 16 * ri + l16];
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    if constexpr (kF64)
                        macc[ci][ri] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[ci], xb[ri], macc[ci][ri], 0, 0, 0);
                    else
                        macc[ci][ri] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[ci], xb[ri], macc[ci][ri], 0, 0, 0);
                }
        }
    }
    // entry e: row qr + 16 ((e >> 2) & 1) + l16; column qc + 16 (e >> 3) + l4 + 4 (e & 3) (FP64
    // blocks) or qc + 16 (e >> 3) + 4 l4 + (e & 3) (FP32 blocks)
    auto erow = [&](int e) -> int { return qr + 16 * ((e >> 2) & 1) + l16; };
    auto ecol = [&](int e) -> int {
        return kF64 ? qc + 16 * (e >> 3) + l4 + 4 * (e & 3) : qc + 16 * (e >> 3) + 4 * l4 + (e & 3);
    };
    auto entry = [&](int e) -> int64_t {
        const int i = erow(e), j = ecol(e);
        return (i < rl && j < cl) ? rpos_[i] + (int64_t)cpos_[j] * nmax : (int64_t)-1;
    };
    double old[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) old[e] = blk[max(entry(e), (int64_t)0)];
#pragma unroll
    for (int e = 0; e < 16; ++e) asm volatile("" ::"v"(old[e]));
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t off = entry(e);
        if (off >= 0) blk[off] = old[e] - (double)macc[e >> 3][(e >> 2) & 1][e & 3];
    }
}

int schur_tile_capx(int nboxes, int maxJ) {
    const int tpd = (maxJ + 63) / 64;
    return tpd * tpd * ((nboxes + 7) / 8);
}

int launch_schur(const Level& L, const int* boxes, int nboxes, int maxJ, int mixed, const TileList& tl, hipStream_t s) {
    if (nboxes <= 0) return 0;
    if (tl.capx < schur_tile_capx(nboxes, maxJ)) return -1;
    SchurArgs a;
    a.store = L.store; a.dstore = L.dstore; a.nb = L.nb; a.nmax = L.nmax; a.ldJ = L.ldJ;
    a.cnt = L.cnt; a.nact = L.nact; a.apos = L.apos; a.krank = L.krank; a.nJ = L.nJ; a.spos = L.spos;
    a.jmap = L.jmap; a.jseg = L.jseg;
    const int tpd = (maxJ + 63) / 64;
    const int64_t nwg = 8 * (int64_t)tpd * tpd * ((nboxes + 7) / 8);   // 8 lists of at most capx entries
    dim3 grid((unsigned)nwg), block(256);
    const PlanParams pp = plan_params(nboxes);
    const bool atom = pp.schur_atomic != 0;
    std::string form = atom ? "_atomic" : "";
    if (mixed) {
        // FP32 products: vector FMAs (schur_form 0) or matrix cores (1)
        const int sf = pp.schur_form;
        form += sf == 1 ? "_mfma" : "";
        note_shape(std::string("schur_f32") + (L.store32 ? "_store32" : "_store64") + form);
        a.XJR = L.XJR32; a.G = L.G32;
        if (L.store32) {
            if (sf == 1 && atom) k_schur<float, float, true, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else if (sf == 1) k_schur<float, float, false, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else if (atom) k_schur<float, float, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else k_schur<float, float, false><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
        } else {
            if (sf == 1 && atom) k_schur<float, double, true, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else if (sf == 1) k_schur<float, double, false, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else if (atom) k_schur<float, double, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else k_schur<float, double, false><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
        }
    } else {
        note_shape(std::string("schur_f64") + (L.store32 ? "_store32" : "_store64") + form);
        a.XJR = L.XJR; a.G = L.G;
        if (L.store32) {
            if (atom) k_schur<double, float, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else k_schur<double, float, false><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
        } else {
            if (atom) k_schur<double, double, true><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
            else k_schur<double, double, false><<<grid, block, 0, s>>>(a, tl.cnt, tl.tiles, tl.info, tl.capx);
        }
    }
    return 0;
}

int launch_schur_self(const Level& L, const int* boxes, int nboxes, hipStream_t s) {
    if (nboxes <= 0) return 0;
    SchurArgs a;
    a.store = L.store; a.dstore = L.dstore; a.nb = L.nb; a.nmax = L.nmax; a.ldJ = L.ldJ;
    a.cnt = L.cnt; a.nact = L.nact; a.apos = L.apos; a.krank = L.krank; a.nJ = L.nJ; a.spos = L.spos;
    a.jmap = L.jmap; a.jseg = L.jseg;
    const int nsub = (L.nmax + 63) / 64;
    // S x S (slot 4) with the FP64 records
    a.XJR = L.XJR; a.G = L.G;
    note_shape("schur_self_sxs_f64");
    k_schur_self<double><<<dim3((unsigned)((int64_t)nboxes * nsub * nsub)), dim3(256), 0, s>>>(a, boxes, 4, nsub);
    return 1;
}

}  // namespace rss
