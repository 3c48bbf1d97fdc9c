// Internal declarations of librss: level data, factor records and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rss.h"

namespace rss {

constexpr int kMaxDepth = 12;      // deepest uniform tree level (4^12 leaf boxes)
constexpr int kMaxBox = 256;       // largest active DOF count of one box
static_assert(kMaxBox < 512 && 9 * kMaxBox < 4096, "Schur tile-list info packs |R| in 9 and |J| in 12 bits");
constexpr int kMaxProxy = 64;
constexpr int kNbr = 25;           // stored block pairs per box: offsets (dx, dy) in [-2, 2]^2
constexpr double kTau = 1e-11;     // pivot tie window relative to the first pivot norm
int elim_lds_limit();

// offset slot of box b seen from box a: (dy + 2) * 5 + (dx + 2)
__host__ __device__ inline int nbr_slot(int dx, int dy) { return (dy + 2) * 5 + (dx + 2); }

struct KernelParams {
    double coef;     // w K(z) = coef * log|z|^2, coef = -w / (4 pi)
    double diag;
    double tol;
    double tau;
    int n_proxy;
    double proxy_radius;
    double lo_x, lo_y, side;   // root box
    int weak = 0;              // 1: the weak pass of RS-WS (ID rows from distance 1 and 2, J = S)
};

// One tree level: active lists at the start of the level, the block store, and the
// strong-skeletonization records of its boxes.
struct Level {
    int t = 0, nb = 0, nbox = 0;
    int nmax = 0;        // max |B| at level start; leading dimension of store blocks
    int ldJ = 0;         // 9 * nmax: capacity of J lists
    void* store = nullptr;     // nbox * 25 * nmax * nmax entries: FP64, or FP32 when store32
    int store32 = 0;           // mixed precision: the block store holds FP32 entries
    int weak = 0;              // RS-WS: the records of this level are those of its weak pass
    size_t store_bytes() const { return (size_t)nbox * kNbr * nmax * nmax * (store32 ? 4 : 8); }
    // With an FP32 store the self blocks A(B_a, B_a) (offset (0, 0)) live in this FP64 array
    // instead: after a box's elimination its skeleton-skeleton entries are O(1), and FP32
    // rounding of them would dominate |A - F|.  nullptr with an FP64 store.
    double* dstore = nullptr;
    size_t dstore_bytes() const { return store32 ? (size_t)nbox * nmax * nmax * 8 : 0; }
    int* cnt = nullptr;        // |B| at level start
    int* gidx = nullptr;       // nbox * nmax global DOF indices (ascending)
    int* nact = nullptr;       // current active count
    int* apos = nullptr;       // nbox * nmax active positions in B (ascending)
    // records
    int* krank = nullptr;      // |S| (= |B| when nothing was eliminated)
    int* nJ = nullptr;         // |J|
    int* spos = nullptr;       // nbox * nmax
    int* rpos = nullptr;       // nbox * nmax
    int* Jg = nullptr;         // nbox * ldJ global indices of J = S then active near field
    int* jmap = nullptr;       // nbox * ldJ: J row -> (3x3 neighbourhood slot << 16) | position in its box
    int* jseg = nullptr;       // nbox * 9: J rows of the box at each 3x3 slot, (first << 16) | count
                               // (0: no such box or no active DOFs); slot 4 is S
    int* Sg = nullptr;         // nbox * nmax
    int* Rg = nullptr;         // nbox * nmax
    double* T = nullptr;       // nbox * nmax * nmax, |S| x |R| col-major (ld nmax)
    double* XJR = nullptr;     // nbox * ldJ * nmax, |J| x |R| (ld ldJ)
    double* G = nullptr;       // nbox * nmax * ldJ, |R| x |J| (ld nmax)
    double* XRR = nullptr;     // nbox * nmax * nmax
    double* Xinv = nullptr;    // nbox * nmax * nmax
    double* Lc = nullptr;      // nbox * nmax * nmax: lower Cholesky factor of X_RR (built on first use)
    float* XJR32 = nullptr;    // mixed: FP32 copies
    float* G32 = nullptr;
    float* Xinv32 = nullptr;
    float* T32 = nullptr;
    int* mrows = nullptr;            // per box: rows of its ID input
    double* logdet_part = nullptr;   // per box: log|det X_RR|
    int* sign_part = nullptr;        // per box: sign of det X_RR (+-1)
    // host-side schedule
    std::vector<int> h_cnt, h_k;
    std::vector<std::vector<int>> colour_boxes;   // ascending box ids per colour
    std::vector<int*> d_colour_boxes;
    std::vector<std::vector<int>> rec_boxes;      // boxes with a record, per colour
    std::vector<int*> d_rec_boxes;
    std::vector<hipEvent_t> pass_ev;              // timing events of the pass (read at the end)
    int graphed = 0;                              // the pass ran as one HIP graph (pass_ev: start, end)
};

// FFT plan of the exact operator on a uniform n x n grid (L x L circulant embedding).
struct FFTPlan {
    bool ready = false;
    int n = 0, L = 0, logL = 0;
    double h = 0;
    void* chat = nullptr;   // FFT2 of the circulant generator, L x L complex
    void* work = nullptr;   // L x L complex scratch
    void* tw = nullptr;     // L / 2 twiddles
};

// Realized sizes and algorithmic counts of one skeletonized level: F_ID = 2 m n^2 - 2/3 n^3,
// F_X = 4 |J| |R| |S| + 4 |R|^2 |S|, F_LU = 2/3 |R|^3, F_G = 2 |R|^2 |J| + 4/3 |R|^3,
// F_Schur = 2 |J|^2 |R|; Schur bytes = 16 |J|^2 (FP64 target read + write) plus the two
// operands; solve bytes = factor data streamed by one solve.
struct LevelStats {
    int depth = 0, weak = 0, boxes = 0, nmax = 0, records = 0, max_k = 0, max_J = 0;
    double sum_k = 0, sum_r = 0, sum_J = 0;
    double flops_id = 0, flops_x = 0, flops_lu = 0, flops_g = 0, flops_schur = 0;
    double bytes_schur = 0, bytes_solve64 = 0, bytes_solve32 = 0;
    // mixed precision: the S x S tiles run in their own FP64 launch (flops, bytes, time);
    // flops_schur, bytes_schur and ms_schur then count the main (FP32) launch only
    double flops_schur_self = 0, bytes_schur_self = 0, ms_schur_self = 0;
    double ms_id = 0, ms_elim = 0, ms_schur = 0, ms_transition = 0;
    double ms_graph = 0;   // the whole pass, when it ran as one HIP graph (the split above is then 0)
};

}  // namespace rss

struct rss_factor_s {
    rss_params params;
    rss::KernelParams kp;
    int64_t n = 0;
    int depth = 0;
    double* pts = nullptr;          // n x 2
    std::vector<rss::Level> levels; // levels[i] = depth D - i (skeletonized levels only)
    // top block
    hipStream_t stream = nullptr;   // stream of rss_factor_create (allocations of the factor)
    rss::FFTPlan fft;               // exact operator by FFT when the points form a grid
    int lds_limit = 0;
    int top_depth = 0;              // level whose remaining active DOFs form the top block
    int64_t ntop = 0;
    int* top_idx = nullptr;
    double* top_A = nullptr;        // ntop x ntop
    double* top_inv = nullptr;      // explicit inverse
    float* top_inv32 = nullptr;
    double* top_L = nullptr;        // lower Cholesky factor of top_A (built on first use) ...
    double* top_LT = nullptr;       // ... and its transpose, both dense ntop x ntop
    int sqrt_ready = 0;
    double top_logdet = 0;
    int top_sign = 1;
    // workspaces
    double* work = nullptr;         // solve / gmres scratch
    size_t work_elems = 0;
    int* flag = nullptr;            // device error flags
    std::vector<void*> allocs;
    void* hpin = nullptr;          // pinned host staging for small device-to-host copies
    size_t hpin_bytes = 0;
    void* hup = nullptr;           // pinned host staging of host-to-device uploads since the last sync
    size_t hup_bytes = 0, hup_used = 0;
    std::vector<std::pair<void*, size_t>> pending_free;   // released at the next synchronization
    std::vector<rss::LevelStats> stats;
    std::vector<std::string> shapes;   // launch shapes taken (note_shape)
    std::vector<double> phase_ms;   // tree, leaf store, id, elim, schur, transition, top, total
    std::vector<int> kernel_launches;
    double wall_ms = 0;
    size_t bytes_device = 0;
};

namespace rss {

// Largest 64-bit key of the wave, on every lane: within each row of 16 lanes by DPP row
// shifts (1, 2, 4, 8), then across rows by the row broadcasts of lanes 15 and 31, so that
// lane 63 ends with the maximum; lanes without a source take 0 (the identity).
template <int CTRL, int ROWS>
__device__ inline unsigned long long dpp_max_step(unsigned long long k) {
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(k & 0xffffffffull), CTRL, ROWS, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(k >> 32), CTRL, ROWS, 0xf, true);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    return o > k ? o : k;
}

__device__ inline unsigned long long wave_max_u64(unsigned long long k) {
    k = dpp_max_step<0x111, 0xf>(k);   // row_shr:1
    k = dpp_max_step<0x112, 0xf>(k);   // row_shr:2
    k = dpp_max_step<0x114, 0xf>(k);   // row_shr:4
    k = dpp_max_step<0x118, 0xf>(k);   // row_shr:8
    k = dpp_max_step<0x142, 0xa>(k);   // row_bcast:15 into rows 1 and 3
    k = dpp_max_step<0x143, 0xc>(k);   // row_bcast:31 into rows 2 and 3
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k & 0xffffffffull), 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// Smallest unsigned value of the wave, on every lane (DPP as above; lanes without a
// source keep the identity 0xffffffff).
template <int CTRL, int ROWS>
__device__ inline unsigned dpp_min_step(unsigned v) {
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)0xffffffffu, (int)v, CTRL, ROWS, 0xf, false);
    return o < v ? o : v;
}

__device__ inline unsigned wave_min_u32(unsigned v) {
    v = dpp_min_step<0x111, 0xf>(v);   // row_shr:1
    v = dpp_min_step<0x112, 0xf>(v);   // row_shr:2
    v = dpp_min_step<0x114, 0xf>(v);   // row_shr:4
    v = dpp_min_step<0x118, 0xf>(v);   // row_shr:8
    v = dpp_min_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_min_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Partial-pivoting choice over the wave: the largest best (each lane's largest |entry|,
// >= 0, or -1 for none) and, among lanes that hold it, the lowest index bi; the result on
// every lane.  Non-negative doubles order like their bit patterns.
__device__ inline void wave_argmax(double& best, int& bi) {
    const unsigned long long key = best >= 0.0 ? (unsigned long long)__double_as_longlong(best) + 1ull : 0ull;
    const unsigned long long km = wave_max_u64(key);
    bi = (int)wave_min_u32(key == km ? (unsigned)bi : 0xffffffffu);
    best = km == 0 ? -1.0 : __longlong_as_double((long long)(km - 1ull));
}

// Launch-plan parameters of the kernels of one colour, by the colour's box count (buckets
// with lower bounds kPlanBucketLo).  The table in tuned_plans.inc is written by the
// autotuner (paper_1609_08130_amd/tune.py), which times the factorization and the solve
// with candidate values set through the environment variable RSS_TUNE
// ("b<bucket>.<field>=<value>,..."), read at every rss_factor_create.  Every value is
// correct for any box count; only the speed differs.
struct PlanParams {
    int gram_many;       // 1: Gram matrices of 256-row slices with the whole triangle per workgroup
    int gram_min_wg;     // few-box Gram plan: rows are sliced until the colour has this many workgroups
    int pchol_kc;        // many-box pivoted Cholesky: rows of R kept in LDS (0: as many as fit)
    int elim_tpw;        // elimination row / column tiles per workgroup
    int elim_tw;         // widest elimination tile (lines of J)
    int inv_threads;     // workgroup of the X_RR inverse: 256 or 1024 threads
    int sweep_threads;   // workgroup of the solve / apply sweeps: 256 or 1024 threads
    int gram_i8;         // 1: with an FP32 store, exact Gram sums on the int8 matrix cores
    int schur_atomic;    // 1: Schur entries updated by no-return atomic adds (same rounding)
    int schur_form;      // FP32 Schur products: 0 vector FMAs, 1 matrix cores
};
constexpr int kPlanBuckets = 5;
extern const int kPlanBucketLo[kPlanBuckets];
PlanParams plan_params(int nboxes);
// Re-reads RSS_TUNE (rss_factor_create calls it once).
void reload_plan_overrides();

// Launch shapes (the kernel variants chosen by box counts and sizes) are collected by name
// into the log of the factor whose entry point is running, for rss_info; a launcher calls
// note_shape once per variant it launches.  No log set: nothing is recorded.
void set_shape_log(std::vector<std::string>* log);
void note_shape(const std::string& name);

// ---- launchers (each enqueues on `s`) -------------------------------------------------
// tree / store (rss_tree.hip)
void launch_validate_points(const double* pts, int64_t n, double lo_x, double lo_y, double side,
                            int* flag, hipStream_t s);
void launch_count_boxes(const double* pts, int64_t n, int t, double lo_x, double lo_y, double side,
                        int* counts, hipStream_t s);
void launch_leaf_lists(const double* pts, int64_t n, int t, double lo_x, double lo_y, double side,
                       int* fill, int* gidx, int nmax, int nbox, hipStream_t s);
void launch_leaf_store(const Level& L, const double* pts, const KernelParams& kp, int* flag,
                       hipStream_t s);
void launch_parent_lists(const Level& C, Level& P, int* pmap, hipStream_t s);
void launch_parent_store(const Level& C, const Level& P, const int* pmap, const double* pts,
                         const KernelParams& kp, hipStream_t s);
// Sizes of the next level from the active counts after a pass, on the device: with group 2
// (level transition) pc[P] = sum of the active counts of P's 2 x 2 children, with group 1
// pc = nact (pc may be nullptr); out[0] = max pc, out[1] = sum pc (zeroed by the caller).
void launch_level_sizes(const int* nact, int nb, int group, int* pc, int* out, hipStream_t s);
// RS-WS: C (same depth, lists and store allocated for C.nmax = the largest active count)
// <- the active DOFs of L after its weak pass, lists and blocks compacted.
void launch_compact(const Level& L, Level& C, hipStream_t s);
void launch_top_assemble(const Level& L, const int* tmap, const int* top_idx, int64_t ntop,
                         const double* pts, const KernelParams& kp, double* A, hipStream_t s);
// work: 2 ntop ints (used when the level has more than 16 boxes)
void launch_top_lists(const Level& L, int* top_idx, int* tmap, int64_t ntop, int* work, hipStream_t s);

// skeletonization (rss_idgram.hip, rss_elim.hip, rss_schur.hip)
// Returns the number of kernels launched.  flag: the factor's device flag word; bit 128
// records that the int8 Gram kernel summed a slice in double-double (wide exponent spread).
int launch_id_gram(const Level& L, const int* boxes, int nboxes, const double* pts, const double* ptmpl,
                   const KernelParams& kp, double* work, int* flag, hipStream_t s);
size_t id_work_doubles(int nmax, int n_proxy, size_t nboxes, int weak, bool store32);
// Returns the number of kernels launched, or -1 when the box size leaves no LDS tile.
// Active 64 x 64 tiles of the Schur updates of one colour, in 8 lists (one per XCD: the
// boxes with position bi = x mod 8 in the colour's list go to list x).  An entry packs
// (bi << 12) | (tile row << 6) | tile column; cnt[x] counts the entries of list x, which
// start at tiles + x * capx.  Filled by launch_elim, read by launch_schur.
struct TileList {
    int* cnt = nullptr;     // 8 counters, zero before the colour's elimination
    int* tiles = nullptr;   // 8 * capx entries: (box mod 2^20 << 12) | (tile row << 6) | tile column
    int* info = nullptr;    // 8 * capx entries beside tiles: (box / 2^20 << 21) | (|J| << 9) | |R|
                            // (|J| <= 9 kMaxBox < 4096, |R| <= kMaxBox < 512)
    int capx = 0;           // ceil(boxes / 8) * ceil(ldJ / 64)^2
};
// Every active tile goes to tl; the J segment of each 3x3 slot goes to L.jseg.
// weak: the RS-WS weak pass (J = S, no adjacent boxes).
int launch_elim(const Level& L, const int* boxes, int nboxes, int mixed, int weak, double* work, int* flag,
                const TileList& tl, hipStream_t s);
// Entries per tile list for a colour of nboxes boxes with |J| <= maxJ.
int schur_tile_capx(int nboxes, int maxJ);
// The Schur update of the tiles of tl with the factorization's product type.  Mixed
// precision leaves out S x S of each step (launch_schur_self).  Returns -1 when tl.capx is
// below schur_tile_capx(nboxes, maxJ) (nothing launched).
int launch_schur(const Level& L, const int* boxes, int nboxes, int maxJ, int mixed, const TileList& tl, hipStream_t s);
// Mixed precision: the S x S block of each step with FP64 products into its FP64 entries.
// Returns the number of kernels launched.
int launch_schur_self(const Level& L, const int* boxes, int nboxes, hipStream_t s);

// dense top block (rss_solve.hip)
// piv: lu_piv_ints(n) ints (interchanges, row permutation, panel swap lists)
int64_t lu_piv_ints(int64_t n);
// work: lu_work_doubles(n) doubles (inverses of the diagonal blocks of L and U)
int64_t lu_work_doubles(int64_t n);
void launch_lu_inverse(double* A, double* Ainv, int64_t n, int* piv, double* work, int* flag,
                       double* logdet, int* sign, hipStream_t s);

// solve / apply sweeps (rss_solve.hip)
void launch_solve_fwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      int use32, hipStream_t s);
void launch_solve_bwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      int use32, hipStream_t s);
// Lroot == nullptr: F x.  Lroot == L.Lc: the generalized square root, with the block
// Cholesky factors in place of X_RR (forward sweep: L^T after W_i; backward: L before V_i).
void launch_apply_fwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      const double* Lroot, hipStream_t s);
void launch_apply_bwd(const Level& L, const int* boxes, int nboxes, double* z, int nrhs, int64_t ld,
                      const double* Lroot, hipStream_t s);
// Cholesky factors: of X_RR for the listed records (into L.Lc), and of the dense top block
// (L and its transpose LT).  A block that is not positive definite sets bit 16 of *flag.
void launch_chol_records(const Level& L, const int* boxes, int nboxes, int* flag, hipStream_t s);
void launch_chol_top(const double* A, int64_t n, double* Lt, double* LT, int* flag, hipStream_t s);
void launch_top_apply(const int* top_idx, int64_t ntop, const double* M, const float* M32, double* z,
                      int nrhs, int64_t ld, double* tmp, hipStream_t s);
void launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t s);
void launch_copy_cols(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int nrhs,
                      hipStream_t s);

// exact operator and BLAS-1 (rss_matvec.hip)
void launch_matvec_direct(const double* pts, int64_t n, const KernelParams& kp, const double* x,
                          double* y, hipStream_t s);
bool fft_grid_detect(FFTPlan& P, const double* pts, int64_t N, int* dflag, hipStream_t s);
bool fft_plan_init(FFTPlan& P, const KernelParams& kp, hipStream_t s);
void launch_matvec_fft(const FFTPlan& P, const KernelParams& kp, const double* x, double* y, hipStream_t s);
void launch_dot_partial(const double* x, const double* y, int64_t n, double* part, hipStream_t s);
int dot_partial_blocks(int64_t n);
void launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t s);
void launch_scal_copy(double a, const double* x, double* y, int64_t n, hipStream_t s);
// y[i] = v for i < n (a kernel, not hipMemsetAsync, so that it may sit in a captured graph)
void launch_fill(double* y, double v, int64_t n, hipStream_t s);

}  // namespace rss
