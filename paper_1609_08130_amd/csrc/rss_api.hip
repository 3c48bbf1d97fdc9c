// C ABI of librss and the host-side driver of Algorithm 1 (Section 3.3).
//
// rss_factor_create: tree -> leaf block store -> for every skeletonized level (leaves
// first): for every colour of the 3x3 colouring, one launch each of the ID, elimination
// and Schur kernels over all boxes of that colour -> level transition (B_parent = union
// of child skeletons) -> top block LU.  The host synchronizes once per level to size the
// next level's store and to collect statistics.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sstream>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "rss_internal.h"

namespace rss {
int elim_lds_limit();

#include "tuned_plans.inc"

static std::mutex g_plan_mu;
static PlanParams g_plan[kPlanBuckets];
static bool g_plan_ready = false;

void reload_plan_overrides() {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (int b = 0; b < kPlanBuckets; ++b) g_plan[b] = kPlanTable[b];
    const char* env = std::getenv("RSS_TUNE");
    if (env) {
        std::string all(env);
        size_t pos = 0;
        while (pos < all.size()) {
            size_t end = all.find(',', pos);
            if (end == std::string::npos) end = all.size();
            const std::string item = all.substr(pos, end - pos);
            pos = end + 1;
            const size_t dot = item.find('.'), eq = item.find('=');
            if (item.size() < 4 || item[0] != 'b' || dot == std::string::npos || eq == std::string::npos || eq < dot)
                continue;
            const int b = std::atoi(item.substr(1, dot - 1).c_str());
            if (b < 0 || b >= kPlanBuckets) continue;
            const std::string key = item.substr(dot + 1, eq - dot - 1);
            const int v = std::atoi(item.substr(eq + 1).c_str());
            PlanParams& q = g_plan[b];
            if (key == "gram_many") q.gram_many = v != 0;
            else if (key == "gram_min_wg" && v > 0) q.gram_min_wg = v;
            else if (key == "pchol_kc" && v >= 0) q.pchol_kc = v;
            else if (key == "elim_tpw" && v >= 1 && v <= 8) q.elim_tpw = v;
            else if (key == "elim_tw" && (v == 4 || v == 8 || v == 16 || v == 32)) q.elim_tw = v;
            else if (key == "inv_threads" && (v == 256 || v == 1024)) q.inv_threads = v;
            else if (key == "sweep_threads" && (v == 256 || v == 1024)) q.sweep_threads = v;
            else if (key == "gram_i8") q.gram_i8 = v != 0;
            else if (key == "schur_atomic") q.schur_atomic = v != 0;
            else if (key == "schur_form" && v >= 0 && v <= 1) q.schur_form = v;
        }
    }
    g_plan_ready = true;
}

PlanParams plan_params(int nboxes) {
    if (!g_plan_ready) reload_plan_overrides();
    int b = 0;
    while (b + 1 < kPlanBuckets && nboxes >= kPlanBucketLo[b + 1]) ++b;
    return g_plan[b];
}

static thread_local std::vector<std::string>* g_shape_log = nullptr;

void set_shape_log(std::vector<std::string>* log) { g_shape_log = log; }

void note_shape(const std::string& name) {
    if (!g_shape_log) return;
    if (std::find(g_shape_log->begin(), g_shape_log->end(), name) == g_shape_log->end()) g_shape_log->push_back(name);
}

// Sets the shape log of factor f for the lifetime of the guard.
struct ShapeLogScope {
    explicit ShapeLogScope(rss_factor f) { set_shape_log(&f->shapes); }
    ~ShapeLogScope() { set_shape_log(nullptr); }
};
}

namespace {

thread_local std::string g_err;

struct Fail {
    rss_status st;
};

[[noreturn]] void fail(rss_status st, const std::string& msg) {
    g_err = msg;
    throw Fail{st};
}

#define HIPCHK(x)                                                                                 \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) fail(RSS_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(RSS_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

// Device memory comes from a process-wide cache: a freed block is kept (per device) and
// handed to a later request of at most its size and at least half of it, so repeated
// factorizations of similar problems run without mapping or unmapping memory.
// rss_trim() returns the cached blocks to the device.
struct CachedBlock {
    int dev;
    size_t bytes;
    void* ptr;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;
std::unordered_map<void*, std::pair<int, size_t>> g_live;   // ptr -> (device, block bytes)

size_t round_block(size_t b) {
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

template <class T>
T* dalloc(rss_factor f, size_t n, hipStream_t s) {
    (void)s;
    if (n == 0) n = 1;
    if (f->params.arena_bytes && f->bytes_device + n * sizeof(T) > f->params.arena_bytes)
        fail(RSS_E_ARENA, "the factorization needs more than arena_bytes = " + std::to_string(f->params.arena_bytes) +
                              " bytes of device memory (" + std::to_string(f->bytes_device + n * sizeof(T)) +
                              " requested)");
    const size_t want = round_block(n * sizeof(T));
    int dev = 0;
    (void)hipGetDevice(&dev);
    void* p = nullptr;
    size_t got = 0;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        size_t best = SIZE_MAX;
        int bi = -1;
        for (int i = 0; i < (int)g_cache.size(); ++i) {
            const CachedBlock& b = g_cache[i];
            if (b.dev == dev && b.bytes >= want && b.bytes <= 2 * want && b.bytes < best) { best = b.bytes; bi = i; }
        }
        if (bi >= 0) {
            p = g_cache[bi].ptr;
            got = g_cache[bi].bytes;
            g_cache.erase(g_cache.begin() + bi);
        }
    }
    if (!p) {
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            // give cached memory back and retry once
            rss_trim();
            e = hipMalloc(&p, want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                fail(RSS_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
            }
        }
        got = want;
    }
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_live[p] = {dev, got};
    }
    f->allocs.push_back(p);
    f->bytes_device += n * sizeof(T);
    return (T*)p;
}

template <class T>
T* dalloc(rss_factor f, size_t n) {
    return dalloc<T>(f, n, f->stream);
}

// Return a block to the cache.  The caller guarantees that no queued work still uses it
// (the library synchronizes the stream before releasing memory a kernel may touch).
void release_block(void* p) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    g_cache.push_back({it->second.first, it->second.second, p});
    g_live.erase(it);
}

void dfree(rss_factor f, void* p, size_t bytes, hipStream_t s) {
    if (!p) return;
    auto it = std::find(f->allocs.begin(), f->allocs.end(), p);
    if (it != f->allocs.end()) f->allocs.erase(it);
    f->bytes_device -= bytes;
    (void)hipStreamSynchronize(s);
    release_block(p);
}

void dfree(rss_factor f, void* p, size_t bytes) { dfree(f, p, bytes, f->stream); }

template <class T>
std::vector<T> d2h(const T* d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) {
        HIPCHK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return h;
}

// Everything queued on `s` has completed: blocks whose release was deferred go back to the
// cache and the upload staging is free again.
void after_sync(rss_factor f) {
    for (auto& pb : f->pending_free) release_block(pb.first);
    f->pending_free.clear();
    f->hup_used = 0;
}

// Release a block once the work queued so far has completed (at the next after_sync).
void defer_free(rss_factor f, void* p, size_t bytes) {
    if (!p) return;
    auto it = std::find(f->allocs.begin(), f->allocs.end(), p);
    if (it != f->allocs.end()) f->allocs.erase(it);
    f->bytes_device -= bytes;
    f->pending_free.push_back({p, bytes});
}

// Copy host data to the device without waiting: the data goes through pinned staging that
// stays untouched until the next synchronization (a full staging buffer forces one).
void upload(rss_factor f, void* d, const void* h, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    const size_t need = (bytes + 255) / 256 * 256;
    if (f->hup_used + need > f->hup_bytes) {
        HIPCHK(hipStreamSynchronize(s));
        after_sync(f);
        if (need > f->hup_bytes) {
            if (f->hup) (void)hipHostFree(f->hup);
            f->hup = nullptr;
            f->hup_bytes = 0;
            const size_t nb = std::max(need, (size_t)4 << 20);
            HIPCHK(hipHostMalloc(&f->hup, nb));
            f->hup_bytes = nb;
        }
    }
    unsigned char* st = (unsigned char*)f->hup + f->hup_used;
    std::memcpy(st, h, bytes);
    f->hup_used += need;
    HIPCHK(hipMemcpyAsync(d, st, bytes, hipMemcpyHostToDevice, s));
}

template <class T>
T* h2d(rss_factor f, const std::vector<T>& h, hipStream_t s) {
    T* d = dalloc<T>(f, h.size());
    upload(f, d, h.data(), h.size() * sizeof(T), s);
    return d;
}

// Several box lists in one device allocation and one copy; returns a pointer per list.
std::vector<int*> h2d_lists(rss_factor f, const std::vector<std::vector<int>>& lists, hipStream_t s) {
    std::vector<int> all;
    std::vector<size_t> off;
    for (auto& v : lists) {
        off.push_back(all.size());
        all.insert(all.end(), v.begin(), v.end());
    }
    int* d = dalloc<int>(f, std::max<size_t>(all.size(), 1));
    upload(f, d, all.data(), all.size() * sizeof(int), s);
    std::vector<int*> ptrs;
    for (size_t o : off) ptrs.push_back(d + o);
    return ptrs;
}

// Several device int arrays copied through pinned host memory with one synchronization.
std::vector<std::vector<int>> d2h_many(rss_factor f, const std::vector<std::pair<const int*, size_t>>& src,
                                       hipStream_t s) {
    size_t tot = 0;
    for (auto& p : src) tot += p.second;
    const size_t bytes = std::max<size_t>(tot, 1) * sizeof(int);
    if (bytes > f->hpin_bytes) {
        if (f->hpin) (void)hipHostFree(f->hpin);
        f->hpin = nullptr;
        f->hpin_bytes = 0;
        HIPCHK(hipHostMalloc(&f->hpin, bytes));
        f->hpin_bytes = bytes;
    }
    int* h = (int*)f->hpin;
    size_t o = 0;
    for (auto& p : src) {
        if (p.second) HIPCHK(hipMemcpyAsync(h + o, p.first, p.second * sizeof(int), hipMemcpyDeviceToHost, s));
        o += p.second;
    }
    HIPCHK(hipStreamSynchronize(s));
    after_sync(f);
    std::vector<std::vector<int>> out;
    o = 0;
    for (auto& p : src) {
        out.emplace_back(h + o, h + o + p.second);
        o += p.second;
    }
    return out;
}

int colour_of(int b, int nb) { return (b % nb) % 3 + 3 * ((b / nb) % 3); }

__global__ void k_init_active(const int* cnt, int* nact, int* apos, int nbox, int nmax) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nbox * nmax) return;
    int b = (int)(e / nmax), i = (int)(e % nmax);
    apos[e] = i;
    if (i == 0) nact[b] = cnt[b];
}

void init_active(rss::Level& L, hipStream_t s) {
    int64_t tot = (int64_t)L.nbox * L.nmax;
    k_init_active<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(L.cnt, L.nact, L.apos, L.nbox, L.nmax);
    check_launch();
}

void alloc_level_lists(rss_factor f, rss::Level& L) {
    L.cnt = dalloc<int>(f, L.nbox);
    L.gidx = dalloc<int>(f, (size_t)L.nbox * L.nmax);
    L.nact = dalloc<int>(f, L.nbox);
    L.apos = dalloc<int>(f, (size_t)L.nbox * L.nmax);
    L.store = dalloc<unsigned char>(f, L.store_bytes());
    if (L.store32) L.dstore = dalloc<double>(f, (size_t)L.nbox * L.nmax * L.nmax);
}

void alloc_level_records(rss_factor f, rss::Level& L, bool mixed) {
    size_t nbox = L.nbox, nm = L.nmax, ldJ = L.ldJ;
    L.krank = dalloc<int>(f, nbox);
    L.nJ = dalloc<int>(f, nbox);
    L.spos = dalloc<int>(f, nbox * nm);
    L.rpos = dalloc<int>(f, nbox * nm);
    L.Sg = dalloc<int>(f, nbox * nm);
    L.Rg = dalloc<int>(f, nbox * nm);
    L.Jg = dalloc<int>(f, nbox * ldJ);
    L.jmap = dalloc<int>(f, nbox * ldJ);
    L.jseg = dalloc<int>(f, nbox * 9);
    L.T = dalloc<double>(f, nbox * nm * nm);
    L.XJR = dalloc<double>(f, nbox * ldJ * nm);
    L.G = dalloc<double>(f, nbox * nm * ldJ);
    L.XRR = dalloc<double>(f, nbox * nm * nm);
    L.Xinv = dalloc<double>(f, nbox * nm * nm);
    L.mrows = dalloc<int>(f, nbox);
    L.logdet_part = dalloc<double>(f, nbox);
    L.sign_part = dalloc<int>(f, nbox);
    if (mixed) {
        L.XJR32 = dalloc<float>(f, nbox * ldJ * nm);
        L.G32 = dalloc<float>(f, nbox * nm * ldJ);
        L.Xinv32 = dalloc<float>(f, nbox * nm * nm);
        L.T32 = dalloc<float>(f, nbox * nm * nm);
    }
}

void free_store(rss_factor f, rss::Level& L) {
    dfree(f, L.store, L.store_bytes());
    L.store = nullptr;
    if (L.dstore) dfree(f, L.dstore, L.dstore_bytes());
    L.dstore = nullptr;
}

struct EvTimer {
    std::vector<hipEvent_t> ev;
    hipEvent_t rec(hipStream_t s) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        HIPCHK(hipEventRecord(e, s));
        ev.push_back(e);
        return e;
    }
    ~EvTimer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

float ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    return ms;
}

void destroy_all(rss_factor f) {
    // any stream may still use the factor's memory: wait for the device first
    (void)hipDeviceSynchronize();
    for (void* p : f->allocs) release_block(p);
    f->allocs.clear();
    if (f->hpin) (void)hipHostFree(f->hpin);
    f->hpin = nullptr;
    f->hpin_bytes = 0;
    if (f->hup) (void)hipHostFree(f->hup);
    f->hup = nullptr;
    f->hup_bytes = f->hup_used = 0;
    for (auto& pb : f->pending_free) release_block(pb.first);
    f->pending_free.clear();
}

// Executable graphs of the level passes (level_graphs = 1), per thread and keyed by (device,
// depth, pass, precision): a thread's factorizations run one after another and each
// synchronizes before it returns, so an executable graph is never updated while a launch of
// it is in flight.  A new capture updates the cached graph in place when its topology
// matches (same kernels, new arguments), else replaces it.  rss_trim releases the calling
// thread's graphs; the others live until the process ends.
struct GraphKey {
    int dev, depth, weak, mixed;
    bool operator<(const GraphKey& o) const {
        return std::tie(dev, depth, weak, mixed) < std::tie(o.dev, o.depth, o.weak, o.mixed);
    }
};
static thread_local std::map<GraphKey, hipGraphExec_t>* g_graph_exec = nullptr;

hipGraphExec_t graph_exec_for(const GraphKey& key, hipGraph_t g) {
    if (!g_graph_exec) g_graph_exec = new std::map<GraphKey, hipGraphExec_t>();
    auto it = g_graph_exec->find(key);
    if (it != g_graph_exec->end()) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        if (hipGraphExecUpdate(it->second, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess)
            return it->second;
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(it->second);
        g_graph_exec->erase(it);
    }
    hipGraphExec_t ex = nullptr;
    HIPCHK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    (*g_graph_exec)[key] = ex;
    return ex;
}

void release_thread_graphs() {
    if (!g_graph_exec) return;
    for (auto& kv : *g_graph_exec) (void)hipGraphExecDestroy(kv.second);
    g_graph_exec->clear();
}

// The stream the level passes are captured on (capture records launches; nothing runs on it),
// one per thread and device, at the default priority.
static thread_local std::map<int, hipStream_t>* g_capture_streams = nullptr;

hipStream_t capture_stream() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (!g_capture_streams) g_capture_streams = new std::map<int, hipStream_t>();
    auto it = g_capture_streams->find(dev);
    if (it != g_capture_streams->end()) return it->second;
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    (*g_capture_streams)[dev] = cs;
    return cs;
}

// phase indices of rss_factor_s::phase_ms
// schur: the Schur-update tile launches with the factorization's product type; schur_self:
// the launches of the self blocks a mixed factorization keeps in FP64
// level_graphs: the passes launched as HIP graphs (their split by kernel is not measured)
enum { PH_TREE = 0, PH_KGEN, PH_ID, PH_ELIM, PH_SCHUR, PH_SCHUR_SELF, PH_GRAPH, PH_TRANS, PH_TOP, PH_TOTAL, PH_N };
const char* kPhaseName[PH_N] = {"tree", "leaf_store", "id", "elim", "schur", "schur_self", "level_graphs",
                                "transition", "top", "total"};

void factor_impl(rss_factor f, const double* d_points, hipStream_t s) {
    const rss_params& p = f->params;
    auto t_start = std::chrono::steady_clock::now();
    EvTimer evs;
    hipEvent_t e0 = evs.rec(s);
    f->phase_ms.assign(PH_N, 0.0);
    f->kernel_launches.assign(PH_N, 0);

    f->pts = dalloc<double>(f, (size_t)f->n * 2);
    HIPCHK(hipMemcpyAsync(f->pts, d_points, sizeof(double) * 2 * f->n, hipMemcpyDeviceToDevice, s));
    f->flag = dalloc<int>(f, 16);   // [0]: error bits; [4 + c]: largest |J| of colour c in the level
    HIPCHK(hipMemsetAsync(f->flag, 0, sizeof(int) * 16, s));

    // root box
    double lo_x = p.root_lo[0], lo_y = p.root_lo[1], side = p.root_side;
    if (!(side > 0)) {
        std::vector<double> hp = d2h(f->pts, (size_t)f->n * 2, s);
        double mnx = hp[0], mny = hp[1], mxx = hp[0], mxy = hp[1];
        for (int64_t i = 0; i < f->n; ++i) {
            mnx = std::min(mnx, hp[2 * i]); mxx = std::max(mxx, hp[2 * i]);
            mny = std::min(mny, hp[2 * i + 1]); mxy = std::max(mxy, hp[2 * i + 1]);
        }
        lo_x = mnx; lo_y = mny;
        side = std::max(mxx - mnx, mxy - mny);
        if (!(side > 0)) side = 1.0;
        if (!std::isfinite(side)) fail(RSS_E_ARG, "non-finite point");
    }
    f->kp.lo_x = lo_x; f->kp.lo_y = lo_y; f->kp.side = side;
    rss::launch_validate_points(f->pts, f->n, lo_x, lo_y, side, f->flag, s);
    check_launch();

    // depth: shallowest uniform level whose boxes hold <= leaf_size points
    int* counts = nullptr;
    size_t counts_n = 0;
    int depth = -1, maxcount = 0;
    int t0 = 0;
    while (t0 < rss::kMaxDepth && (double)p.leaf_size * std::pow(4.0, t0 + 1) < (double)f->n) ++t0;
    for (int t = t0; t <= rss::kMaxDepth; ++t) {
        size_t nbox = (size_t)1 << (2 * t);
        if (counts_n < nbox + 1) {
            if (counts) dfree(f, counts, counts_n * sizeof(int));
            counts = dalloc<int>(f, nbox + 1);
            counts_n = nbox + 1;
        }
        rss::launch_count_boxes(f->pts, f->n, t, lo_x, lo_y, side, counts, s);
        check_launch();
        int mx = 0, flag = 0;
        HIPCHK(hipMemcpyAsync(&mx, counts + nbox, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&flag, f->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (flag & 1) fail(RSS_E_ARG, "non-finite point or point outside the root box");
        if (mx <= p.leaf_size) {
            depth = t;
            maxcount = mx;
            break;
        }
    }
    if (depth < 0) fail(RSS_E_UNSUPPORTED, "tree deeper than 12 levels (clustered or duplicate points)");
    f->depth = depth;

    // leaf level
    rss::Level L;
    L.t = depth; L.nb = 1 << depth; L.nbox = L.nb * L.nb;
    L.nmax = std::max(maxcount, 1);
    L.ldJ = 9 * L.nmax;
    // FP32 store in mixed precision when its rounding (u32 = 2^-24) sits at least 16x below
    // the ID tolerance; tighter tolerances keep an FP64 store (the Schur products stay FP32)
    L.store32 = (p.precision == RSS_MIXED && p.tol >= 16.0 * 0x1.0p-24) ? 1 : 0;
    alloc_level_lists(f, L);
    rss::launch_leaf_lists(f->pts, f->n, depth, lo_x, lo_y, side, L.cnt, L.gidx, L.nmax, L.nbox, s);
    check_launch();
    dfree(f, counts, counts_n * sizeof(int));
    hipEvent_t e1 = evs.rec(s);
    rss::launch_leaf_store(L, f->pts, f->kp, f->flag, s);
    check_launch();
    hipEvent_t e2 = evs.rec(s);
    init_active(L, s);

    // proxy template (unit circle, equispaced from angle 0)
    std::vector<double> tmpl(2 * p.n_proxy);
    for (int i = 0; i < p.n_proxy; ++i) {
        double th = 2.0 * M_PI * (double)i / (double)p.n_proxy;
        tmpl[2 * i] = std::cos(th);
        tmpl[2 * i + 1] = std::sin(th);
    }
    double* ptmpl = h2d(f, tmpl, s);
    // The level boundaries synchronize once each, for the one number the host needs to size
    // the next level (its largest box) and the error flags; the per-level statistics, the
    // solve schedule and the phase times are read once, after the top block.
    std::vector<std::pair<hipEvent_t, hipEvent_t>> trans_ev;   // transitions and compactions
    bool checked_points = false;

    const bool mixed = p.precision == RSS_MIXED;
    double* work = nullptr;
    size_t work_n = 0;
    int* tl_cnt = nullptr;
    int* tl_tiles = nullptr;
    size_t tl_n = 0;

    // Error bits of the device flag: 1 points outside the root box, 2 duplicate points,
    // 4 singular X_RR.  Bits 64 and 128 only record kernel forms that ran (rss_info shapes).
    auto check_flag = [&](int fl) {
        if (!checked_points) {
            checked_points = true;
            if (fl & 2) fail(RSS_E_ARG, "duplicate points");
        }
        if (fl & 4) fail(RSS_E_SINGULAR, "singular redundant block X_RR");
    };

    // Largest and total active counts of the next level (see launch_level_sizes): the
    // boundary's one synchronization.
    auto level_sizes = [&](const rss::Level& L, int group, int* pc) -> std::pair<int, int64_t> {
        HIPCHK(hipMemsetAsync(f->flag + 8, 0, sizeof(int) * 2, s));
        rss::launch_level_sizes(L.nact, L.nb, group, pc, f->flag + 8, s);
        check_launch();
        auto hv = d2h_many(f, {{f->flag, 1}, {f->flag + 8, 2}}, s);
        check_flag(hv[0][0]);
        return {hv[1][0], (int64_t)hv[1][1]};
    };

    // One pass over the colours of level L: the ID, elimination and Schur launches of every
    // colour (strong skeletonization, or with weak = 1 the weak skeletonization of RS-WS).
    auto run_pass = [&](rss::Level& L, int weak) {
        L.weak = weak;
        if (weak) L.ldJ = L.nmax;   // J = S
        rss::KernelParams kpw = f->kp;
        kpw.weak = weak;
        const int nb = L.nb;
        L.colour_boxes.assign(9, {});
        for (int b = 0; b < L.nbox; ++b) L.colour_boxes[colour_of(b, nb)].push_back(b);
        size_t maxc = 0;
        for (auto& v : L.colour_boxes) maxc = std::max(maxc, v.size());
        L.d_colour_boxes = h2d_lists(f, L.colour_boxes, s);
        alloc_level_records(f, L, mixed);
        size_t need = std::max(maxc * (size_t)L.nmax * L.nmax, rss::id_work_doubles(L.nmax, p.n_proxy, maxc, weak, L.store32));
        if (need > work_n) {
            if (work) defer_free(f, work, work_n * sizeof(double));
            work = dalloc<double>(f, need);
            work_n = need;
        }
        // Schur tile lists: 8 counters per colour, zero at the level start; one entry buffer
        // reused by the colours in turn
        // the tile-list entries and the per-tile box sizes share one buffer
        const int capx = rss::schur_tile_capx((int)maxc, L.ldJ);
        if (!tl_cnt) tl_cnt = dalloc<int>(f, 9 * 8);
        if ((size_t)capx * 16 > tl_n) {
            if (tl_tiles) defer_free(f, tl_tiles, tl_n * sizeof(int));
            tl_n = (size_t)capx * 16;
            tl_tiles = dalloc<int>(f, tl_n);
        }
        HIPCHK(hipMemsetAsync(tl_cnt, 0, sizeof(int) * 9 * 8, s));
        std::vector<hipEvent_t>& ev = L.pass_ev;
        ev.clear();
        ev.push_back(evs.rec(s));
        // level_graphs: the colour loop below is captured (no event, memset or host
        // synchronization inside it) on the thread's capture stream and the graph is launched
        // on s, which may be the null stream (not capturable)
        const bool graphs = p.level_graphs != 0;
        L.graphed = graphs ? 1 : 0;
        const hipStream_t sl = graphs ? capture_stream() : s;
        auto mark = [&]() {
            if (!graphs) ev.push_back(evs.rec(s));
        };
        if (graphs) HIPCHK(hipStreamBeginCapture(sl, hipStreamCaptureModeThreadLocal));
        try {
            for (int col = 0; col < 9; ++col) {
                int nbx = (int)L.colour_boxes[col].size();
                if (nbx == 0) continue;
                const int* bx = L.d_colour_boxes[col];
                const int ni = rss::launch_id_gram(L, bx, nbx, f->pts, ptmpl, kpw, work, f->flag, sl);
                check_launch();
                mark();
                rss::TileList tl;
                tl.cnt = tl_cnt + 8 * col;
                tl.tiles = tl_tiles;
                tl.info = tl_tiles + (size_t)8 * capx;
                tl.capx = capx;
                const int ne = rss::launch_elim(L, bx, nbx, mixed ? 1 : 0, weak, work, f->flag, tl, sl);
                if (ne < 0) fail(RSS_E_UNSUPPORTED, "box too large for the elimination kernel's LDS tiles");
                check_launch();
                mark();
                // mixed: S x S in FP64 first (its own event pair), then the tiles
                if (mixed) {
                    f->kernel_launches[PH_SCHUR_SELF] += rss::launch_schur_self(L, bx, nbx, sl);
                    check_launch();
                }
                mark();
                if (rss::launch_schur(L, bx, nbx, L.ldJ, mixed ? 1 : 0, tl, sl) < 0)
                    fail(RSS_E_DEVICE, "Schur tile list too small");
                check_launch();
                mark();
                f->kernel_launches[PH_ID] += ni;
                f->kernel_launches[PH_ELIM] += ne;
                f->kernel_launches[PH_SCHUR] += 1;
            }
        } catch (...) {
            if (graphs) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(sl, &g);
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
            }
            throw;
        }
        if (graphs) {
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamEndCapture(sl, &g));
            int dev = 0;
            (void)hipGetDevice(&dev);
            hipGraphExec_t ex = nullptr;
            try {
                ex = graph_exec_for(GraphKey{dev, L.t, weak, mixed ? 1 : 0}, g);
            } catch (...) {
                (void)hipGraphDestroy(g);
                throw;
            }
            (void)hipGraphDestroy(g);
            HIPCHK(hipGraphLaunch(ex, s));
            ev.push_back(evs.rec(s));
            f->kernel_launches[PH_GRAPH] += 1;
        }
    };

    // Level transition to the parent level (B_parent = union of the children's active DOFs);
    // L goes to the factor's levels.  When a parent box would hold more than max_box active
    // DOFs nothing is built, L stays, and the returned level has t = -1: the recursion ends
    // and L's active DOFs form the top block.
    const int max_box = p.max_box > 0 ? p.max_box : rss::kMaxBox;
    auto transition = [&](rss::Level& L) -> rss::Level {
        hipEvent_t et0 = evs.rec(s);
        rss::Level P;
        P.t = L.t - 1; P.nb = L.nb / 2; P.nbox = P.nb * P.nb;
        P.cnt = dalloc<int>(f, P.nbox);
        const int pmax = std::max(1, level_sizes(L, 2, P.cnt).first);
        if (pmax > max_box) {
            defer_free(f, P.cnt, sizeof(int) * (size_t)P.nbox);
            trans_ev.push_back({et0, evs.rec(s)});
            rss::Level none;
            none.t = -1;
            return none;
        }
        P.nmax = pmax;
        P.ldJ = 9 * P.nmax;
        P.gidx = dalloc<int>(f, (size_t)P.nbox * P.nmax);
        P.nact = dalloc<int>(f, P.nbox);
        P.apos = dalloc<int>(f, (size_t)P.nbox * P.nmax);
        P.store32 = L.store32;
        P.store = dalloc<unsigned char>(f, P.store_bytes());
        if (P.store32) P.dstore = dalloc<double>(f, (size_t)P.nbox * P.nmax * P.nmax);
        int* pmap = dalloc<int>(f, (size_t)P.nbox * P.nmax);
        rss::launch_parent_lists(L, P, pmap, s);
        check_launch();
        rss::launch_parent_store(L, P, pmap, f->pts, f->kp, s);
        check_launch();
        init_active(P, s);
        trans_ev.push_back({et0, evs.rec(s)});
        defer_free(f, pmap, sizeof(int) * (size_t)P.nbox * P.nmax);
        defer_free(f, L.store, L.store_bytes());
        L.store = nullptr;
        if (L.dstore) defer_free(f, L.dstore, L.dstore_bytes());
        L.dstore = nullptr;
        f->levels.push_back(std::move(L));
        return P;
    };

    // RS-WS: the strong pass of a level restarts on the DOFs its weak pass left active (the
    // lists and the store compacted at the same depth); L, with the weak records, goes to
    // the factor's levels.
    auto compact = [&](rss::Level& L) -> rss::Level {
        hipEvent_t ec0 = evs.rec(s);
        rss::Level C;
        C.t = L.t; C.nb = L.nb; C.nbox = L.nbox;
        C.cnt = dalloc<int>(f, C.nbox);
        C.nmax = std::max(1, level_sizes(L, 1, C.cnt).first);
        C.ldJ = 9 * C.nmax;
        C.store32 = L.store32;
        C.gidx = dalloc<int>(f, (size_t)C.nbox * C.nmax);
        C.nact = dalloc<int>(f, C.nbox);
        C.apos = dalloc<int>(f, (size_t)C.nbox * C.nmax);
        C.store = dalloc<unsigned char>(f, C.store_bytes());
        if (C.store32) C.dstore = dalloc<double>(f, (size_t)C.nbox * C.nmax * C.nmax);
        rss::launch_compact(L, C, s);
        check_launch();
        init_active(C, s);
        trans_ev.push_back({ec0, evs.rec(s)});
        defer_free(f, L.store, L.store_bytes());
        L.store = nullptr;
        if (L.dstore) defer_free(f, L.dstore, L.dstore_bytes());
        L.dstore = nullptr;
        f->levels.push_back(std::move(L));
        return C;
    };

    const bool hybrid = p.method == RSS_METHOD_HYBRID;
    while (L.t >= 2) {
        if (hybrid) {
            run_pass(L, 1);
            L = compact(L);
        }
        run_pass(L, 0);
        if (L.t == 2) break;
        rss::Level P = transition(L);
        if (P.t < 0) break;
        L = std::move(P);
    }
    if (hybrid && L.t == 2) {
        // the final weak step at depth 1 (Section 3.4)
        rss::Level P = transition(L);
        if (P.t >= 0) {
            L = std::move(P);
            run_pass(L, 1);
        }
    }
    f->top_depth = L.t;
    if (work) defer_free(f, work, work_n * sizeof(double));
    if (tl_tiles) defer_free(f, tl_tiles, tl_n * sizeof(int));
    if (tl_cnt) defer_free(f, tl_cnt, sizeof(int) * 9 * 8);

    // top block
    hipEvent_t eT0 = evs.rec(s);
    const int64_t ntop = level_sizes(L, 1, nullptr).second;
    if (ntop > RSS_MAX_TOP)
        fail(RSS_E_UNSUPPORTED, "the top block at depth " + std::to_string(L.t) + " holds " + std::to_string(ntop) +
                                    " DOFs (limit " + std::to_string(RSS_MAX_TOP) + "): boxes above it exceed max_box");
    f->ntop = ntop;
    f->top_idx = dalloc<int>(f, ntop);
    int* tmap = dalloc<int>(f, ntop);
    f->top_A = dalloc<double>(f, (size_t)ntop * ntop);
    double* LU = dalloc<double>(f, (size_t)ntop * ntop);
    f->top_inv = dalloc<double>(f, (size_t)ntop * ntop);
    int* piv = dalloc<int>(f, (size_t)rss::lu_piv_ints(ntop));
    double* dlog = dalloc<double>(f, 1);
    int* dsign = dalloc<int>(f, 1);
    int* tw = L.nbox > 16 ? dalloc<int>(f, (size_t)2 * ntop) : nullptr;
    rss::launch_top_lists(L, f->top_idx, tmap, ntop, tw, s);
    check_launch();
    if (tw) defer_free(f, tw, sizeof(int) * (size_t)2 * ntop);
    rss::launch_top_assemble(L, tmap, f->top_idx, ntop, f->pts, f->kp, f->top_A, s);
    check_launch();
    HIPCHK(hipMemcpyAsync(LU, f->top_A, sizeof(double) * ntop * ntop, hipMemcpyDeviceToDevice, s));
    double* luw = dalloc<double>(f, (size_t)rss::lu_work_doubles(ntop));
    rss::launch_lu_inverse(LU, f->top_inv, ntop, piv, luw, f->flag, dlog, dsign, s);
    check_launch();
    if (mixed && ntop > 0) {
        f->top_inv32 = dalloc<float>(f, (size_t)ntop * ntop);
        rss::launch_convert_f32(f->top_inv, f->top_inv32, ntop * ntop, s);
        check_launch();
    }
    hipEvent_t eT1 = evs.rec(s);
    HIPCHK(hipStreamSynchronize(s));
    after_sync(f);
    f->phase_ms[PH_TOP] += ev_ms(eT0, eT1);
    {
        int flag = 0;
        HIPCHK(hipMemcpy(&flag, f->flag, sizeof(int), hipMemcpyDeviceToHost));
        if (flag & 8) fail(RSS_E_SINGULAR, "singular top block");
        double lg = 0;
        int sg = 1;
        if (ntop > 0) {
            HIPCHK(hipMemcpy(&lg, dlog, sizeof(double), hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(&sg, dsign, sizeof(int), hipMemcpyDeviceToHost));
        }
        f->top_logdet = lg;
        f->top_sign = sg;
    }
    dfree(f, LU, sizeof(double) * ntop * ntop);
    dfree(f, tmap, sizeof(int) * ntop);
    dfree(f, piv, sizeof(int) * (size_t)rss::lu_piv_ints(ntop));
    free_store(f, L);
    if (L.krank) f->levels.push_back(std::move(L));
    else {
        // unskeletonized final level: lists are no longer needed
        dfree(f, L.cnt, sizeof(int) * L.nbox);
        dfree(f, L.gidx, sizeof(int) * (size_t)L.nbox * L.nmax);
        dfree(f, L.nact, sizeof(int) * L.nbox);
        dfree(f, L.apos, sizeof(int) * (size_t)L.nbox * L.nmax);
    }
    // Per-level statistics, the solve schedule (boxes with a record, per colour) and the phase
    // times: one read of every level's counts.
    {
        std::vector<std::pair<const int*, size_t>> src = {{f->flag, 1}};
        for (auto& Lv : f->levels) {
            const size_t nbx = (size_t)Lv.nbox;
            src.push_back({Lv.cnt, nbx});
            src.push_back({Lv.krank, nbx});
            src.push_back({Lv.nJ, nbx});
            src.push_back({Lv.mrows, nbx});
            src.push_back({Lv.jseg, mixed ? nbx * 9 : (size_t)0});
        }
        auto hv = d2h_many(f, src, s);
        if (hv[0][0] & 64) rss::note_shape("elim_inv_gauss_jordan_lds");
        if (hv[0][0] & 128) rss::note_shape("gram_i8_wide");
        f->phase_ms[PH_TREE] += ev_ms(e0, e1);
        f->phase_ms[PH_KGEN] += ev_ms(e1, e2);
        for (auto& te : trans_ev) f->phase_ms[PH_TRANS] += ev_ms(te.first, te.second);
        for (size_t li = 0; li < f->levels.size(); ++li) {
            rss::Level& Lv = f->levels[li];
            const std::vector<hipEvent_t>& ev = Lv.pass_ev;
            double lv_id = 0, lv_elim = 0, lv_schur = 0, lv_self = 0, lv_graph = 0;
            if (Lv.graphed && ev.size() >= 2) lv_graph = ev_ms(ev.front(), ev.back());
            for (size_t i = 1; !Lv.graphed && i + 2 < ev.size(); i += 4) {
                lv_id += ev_ms(ev[i - 1], ev[i]);
                lv_elim += ev_ms(ev[i], ev[i + 1]);
                lv_self += ev_ms(ev[i + 1], ev[i + 2]);
                lv_schur += ev_ms(ev[i + 2], ev[i + 3]);
            }
            f->phase_ms[PH_ID] += lv_id;
            f->phase_ms[PH_ELIM] += lv_elim;
            f->phase_ms[PH_SCHUR] += lv_schur;
            f->phase_ms[PH_SCHUR_SELF] += lv_self;
            f->phase_ms[PH_GRAPH] += lv_graph;
            Lv.h_cnt = std::move(hv[1 + 5 * li]);
            Lv.h_k = std::move(hv[2 + 5 * li]);
            const std::vector<int>& hJ = hv[3 + 5 * li];
            const std::vector<int>& hm = hv[4 + 5 * li];
            const std::vector<int>& hseg = hv[5 + 5 * li];
            Lv.rec_boxes.assign(9, {});
            for (int col = 0; col < 9; ++col)
                for (int b : Lv.colour_boxes[col])
                    if (hJ[b] > 0) Lv.rec_boxes[col].push_back(b);
            Lv.d_rec_boxes = h2d_lists(f, Lv.rec_boxes, s);
            rss::LevelStats st;
            st.depth = Lv.t; st.weak = Lv.weak; st.boxes = Lv.nbox; st.nmax = Lv.nmax;
            st.ms_id = lv_id; st.ms_elim = lv_elim; st.ms_schur = lv_schur; st.ms_schur_self = lv_self;
            st.ms_graph = lv_graph;
            for (int b = 0; b < Lv.nbox; ++b) {
                double n = Lv.h_cnt[b], k = Lv.h_k[b], r = n - k, J = hJ[b], m = hm[b];
                if (n > 0) st.flops_id += 2.0 * m * n * n - 2.0 / 3.0 * n * n * n;
                if (J <= 0) continue;
                st.records += 1;
                st.sum_k += k; st.sum_r += r; st.sum_J += J;
                st.max_k = std::max(st.max_k, (int)k);
                st.max_J = std::max(st.max_J, (int)J);
                st.flops_x += 4.0 * J * r * k + 4.0 * r * r * k;
                st.flops_lu += 2.0 / 3.0 * r * r * r;
                st.flops_g += 2.0 * r * r * J + 4.0 / 3.0 * r * r * r;
                // target read + write of the store entries and the two operands once
                if (mixed) {
                    // S x S with FP64 products (k_schur_self), the rest with FP32 products: into
                    // the store, and with an FP32 store the adjacent boxes' self blocks into
                    // their FP64 entries
                    double adj = 0;
                    if (Lv.store32)
                        for (int sl = 0; sl < 9; ++sl) {
                            const double len = hseg[(size_t)b * 9 + sl] & 0xffff;
                            if (sl != 4) adj += len * len;
                        }
                    st.flops_schur_self += 2.0 * k * k * r;
                    st.bytes_schur_self += 16.0 * k * k + 8.0 * 2.0 * k * r;
                    st.flops_schur += 2.0 * (J * J - k * k) * r;
                    st.bytes_schur += (Lv.store32 ? 8.0 : 16.0) * (J * J - k * k - adj) + 16.0 * adj + 4.0 * 2.0 * J * r;
                } else {
                    st.flops_schur += 2.0 * J * J * r;
                    st.bytes_schur += 16.0 * J * J + 8.0 * 2.0 * J * r;
                }
                st.bytes_solve64 += 8.0 * (2.0 * J * r + 2.0 * k * r + r * r);
                st.bytes_solve32 += 4.0 * (2.0 * J * r + 2.0 * k * r + r * r);
            }
            f->stats.push_back(st);
        }
    }
    f->work_elems = (size_t)f->n * 4 + (size_t)ntop * 8 + 4096;
    f->work = dalloc<double>(f, f->work_elems);
    // exact operator: FFT on uniform grids, direct summation otherwise
    if (rss::fft_grid_detect(f->fft, f->pts, f->n, f->flag, s)) {
        const size_t LL = (size_t)f->fft.L * f->fft.L;
        f->fft.chat = dalloc<double>(f, 2 * LL);
        f->fft.work = dalloc<double>(f, 2 * LL);
        f->fft.tw = dalloc<double>(f, (size_t)f->fft.L);
        if (!rss::fft_plan_init(f->fft, f->kp, s)) fail(RSS_E_DEVICE, "FFT plan initialization failed");
    }
    (void)hipGetLastError();
    hipEvent_t eE = evs.rec(s);
    HIPCHK(hipStreamSynchronize(s));
    f->phase_ms[PH_TOTAL] = ev_ms(e0, eE);
    f->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
}

rss_status guard_factor(rss_factor f) {
    if (!f) {
        g_err = "NULL factor";
        return RSS_E_ARG;
    }
    return RSS_OK;
}

}  // namespace

static void exact_matvec(rss_factor f, const double* x, double* y, hipStream_t s);

// ---------------------------------------------------------------------------------------
extern "C" {

void rss_params_default(rss_params* p, int32_t dim, int32_t kernel) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(rss_params);
    p->dim = dim;
    p->kernel = kernel;
    p->symmetric = 1;
    p->diag = 1.0;
    p->weight = 1.0;
    p->tol = 1e-6;
    p->leaf_size = 64;
    p->n_proxy = 16;
    p->proxy_radius = 1.25;
    p->root_side = 1.0;
    p->precision = RSS_FP64;
    p->arena_bytes = 0;
}

const char* rss_last_error(void) { return g_err.c_str(); }

rss_status rss_trim(void) {
    std::vector<CachedBlock> blocks;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        blocks.swap(g_cache);
    }
    for (auto& b : blocks) (void)hipFree(b.ptr);
    release_thread_graphs();
    return RSS_OK;
}

rss_status rss_factor_create(const double* d_points, int64_t n, const rss_params* p, void* stream,
                             rss_factor* out) {
    g_err.clear();
    if (out) *out = nullptr;
    if (!out || !p || !d_points) {
        g_err = "NULL argument";
        return RSS_E_ARG;
    }
    if (p->struct_size != sizeof(rss_params)) {
        g_err = "rss_params.struct_size mismatch (header/library version)";
        return RSS_E_ARG;
    }
    if (p->kernel != RSS_K_LAPLACE2D && p->kernel != RSS_K_LAPLACE3D && p->kernel != RSS_K_HELMHOLTZ2D) {
        g_err = "unknown kernel";
        return RSS_E_ARG;
    }
    if (p->dim != 2 && p->dim != 3) { g_err = "dim must be 2 or 3"; return RSS_E_ARG; }
    if (p->kernel != RSS_K_LAPLACE2D || p->dim != 2) {
        g_err = "this version factors the 2D Laplace kernel only (dim 2, RSS_K_LAPLACE2D)";
        return RSS_E_UNSUPPORTED;
    }
    if (p->symmetric != 1) {
        g_err = "the two-sided ID of a non-symmetric kernel (symmetric = 0) is not built";
        return RSS_E_UNSUPPORTED;
    }
    if (p->method != RSS_METHOD_STRONG && p->method != RSS_METHOD_HYBRID) { g_err = "bad method"; return RSS_E_ARG; }
    if (n < 1 || n > (int64_t)1 << 30) { g_err = "n out of range"; return RSS_E_ARG; }
    if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) { g_err = "tol must be finite and >= 0"; return RSS_E_ARG; }
    if (p->leaf_size < 1 || p->leaf_size > rss::kMaxBox) { g_err = "leaf_size must be in [1, 256]"; return RSS_E_ARG; }
    if (p->n_proxy < 1 || p->n_proxy > rss::kMaxProxy) { g_err = "n_proxy must be in [1, 64]"; return RSS_E_ARG; }
    if (!(p->proxy_radius > 0.5 * std::sqrt(2.0)) || !(p->proxy_radius <= 2.5)) {
        g_err = "proxy_radius must be in (0.5*sqrt(2), 2.5] box sides";
        return RSS_E_ARG;
    }
    if (!std::isfinite(p->diag) || !std::isfinite(p->weight)) { g_err = "diag/weight not finite"; return RSS_E_ARG; }
    if (p->precision != RSS_FP64 && p->precision != RSS_MIXED) { g_err = "bad precision"; return RSS_E_ARG; }
    if (p->level_graphs != 0 && p->level_graphs != 1) { g_err = "level_graphs must be 0 or 1"; return RSS_E_ARG; }
    if (p->max_box < 0 || p->max_box > rss::kMaxBox) { g_err = "max_box must be in [0, 256]"; return RSS_E_ARG; }
    rss_factor f = new (std::nothrow) rss_factor_s();
    if (!f) { g_err = "host allocation failed"; return RSS_E_NOMEM; }
    f->params = *p;
    f->n = n;
    f->kp.coef = -p->weight / (4.0 * M_PI);
    f->kp.diag = p->diag;
    f->kp.tol = p->tol;
    f->kp.tau = rss::kTau;
    f->kp.n_proxy = p->n_proxy;
    f->kp.proxy_radius = p->proxy_radius;
    hipStream_t s = (hipStream_t)stream;
    f->stream = s;
    rss::ShapeLogScope shape_scope(f);
    rss::reload_plan_overrides();
    try {
        factor_impl(f, d_points, s);
    } catch (const Fail& e) {
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        destroy_all(f);
        delete f;
        return e.st;
    } catch (const std::bad_alloc&) {
        (void)hipStreamSynchronize(s);
        destroy_all(f);
        delete f;
        g_err = "host allocation failed";
        return RSS_E_NOMEM;
    }
    *out = f;
    return RSS_OK;
}

rss_status rss_factor_destroy(rss_factor f) {
    if (!f) return RSS_OK;
    destroy_all(f);
    delete f;
    return RSS_OK;
}

static void solve_impl(rss_factor f, double* z, int nrhs, int64_t ld, int use32, hipStream_t s) {
    for (auto& L : f->levels)
        for (int col = 0; col < 9; ++col) {
            rss::launch_solve_fwd(L, L.d_rec_boxes[col], (int)L.rec_boxes[col].size(), z, nrhs, ld, use32, s);
            check_launch();
        }
    if ((size_t)f->ntop * nrhs > f->work_elems) fail(RSS_E_ARG, "nrhs too large for the top workspace");
    rss::launch_top_apply(f->top_idx, f->ntop, f->top_inv, use32 ? f->top_inv32 : nullptr, z, nrhs, ld, f->work, s);
    check_launch();
    for (auto it = f->levels.rbegin(); it != f->levels.rend(); ++it)
        for (int col = 8; col >= 0; --col) {
            rss::launch_solve_bwd(*it, it->d_rec_boxes[col], (int)it->rec_boxes[col].size(), z, nrhs, ld, use32, s);
            check_launch();
        }
}

rss_status rss_solve(rss_factor f, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, int32_t use_fp32,
                     void* stream) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    rss::ShapeLogScope shape_scope(f);
    if (!d_b || !d_x || nrhs < 1 || ld < f->n) { g_err = "bad solve arguments"; return RSS_E_ARG; }
    hipStream_t s = (hipStream_t)stream;
    const int use32 = (use_fp32 && f->params.precision == RSS_MIXED) ? 1 : 0;
    try {
        if (d_x != d_b) rss::launch_copy_cols(d_b, ld, d_x, ld, f->n, nrhs, s);
        check_launch();
        solve_impl(f, d_x, nrhs, ld, use32, s);
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

rss_status rss_apply(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld, void* stream) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    rss::ShapeLogScope shape_scope(f);
    if (!d_x || !d_y || nrhs < 1 || ld < f->n || d_x == d_y) { g_err = "bad apply arguments"; return RSS_E_ARG; }
    hipStream_t s = (hipStream_t)stream;
    try {
        rss::launch_copy_cols(d_x, ld, d_y, ld, f->n, nrhs, s);
        check_launch();
        for (auto& L : f->levels)
            for (int col = 0; col < 9; ++col) {
                rss::launch_apply_fwd(L, L.d_rec_boxes[col], (int)L.rec_boxes[col].size(), d_y, nrhs, ld, nullptr, s);
                check_launch();
            }
        if ((size_t)f->ntop * nrhs > f->work_elems) fail(RSS_E_ARG, "nrhs too large for the top workspace");
        rss::launch_top_apply(f->top_idx, f->ntop, f->top_A, nullptr, d_y, nrhs, ld, f->work, s);
        check_launch();
        for (auto it = f->levels.rbegin(); it != f->levels.rend(); ++it)
            for (int col = 8; col >= 0; --col) {
                rss::launch_apply_bwd(*it, it->d_rec_boxes[col], (int)it->rec_boxes[col].size(), d_y, nrhs, ld, nullptr, s);
                check_launch();
            }
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

// Cholesky factors of the blocks of D, built once per factor on the first square-root
// call (synchronizes).  Throws RSS_E_SINGULAR when a block is not positive definite.
static void ensure_sqrt(rss_factor f, hipStream_t s) {
    if (f->sqrt_ready) return;
    int* fl = f->flag + 15;
    HIPCHK(hipMemsetAsync(fl, 0, sizeof(int), s));
    for (auto& L : f->levels) {
        if (!L.Lc) L.Lc = dalloc<double>(f, (size_t)L.nbox * L.nmax * L.nmax, s);
        for (int col = 0; col < 9; ++col) {
            rss::launch_chol_records(L, L.d_rec_boxes[col], (int)L.rec_boxes[col].size(), fl, s);
            check_launch();
        }
    }
    if (f->ntop > 0) {
        if (!f->top_L) f->top_L = dalloc<double>(f, (size_t)f->ntop * f->ntop, s);
        if (!f->top_LT) f->top_LT = dalloc<double>(f, (size_t)f->ntop * f->ntop, s);
        rss::launch_chol_top(f->top_A, f->ntop, f->top_L, f->top_LT, fl, s);
        check_launch();
    }
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, fl, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag & 16) fail(RSS_E_SINGULAR, "a diagonal block of D is not positive definite: no square root");
    f->sqrt_ready = 1;
}

rss_status rss_sqrt_apply(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld, int32_t adjoint,
                          void* stream) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (!d_x || !d_y || nrhs < 1 || ld < f->n || d_x == d_y) { g_err = "bad sqrt_apply arguments"; return RSS_E_ARG; }
    hipStream_t s = (hipStream_t)stream;
    try {
        if ((size_t)f->ntop * nrhs > f->work_elems) fail(RSS_E_ARG, "nrhs too large for the top workspace");
        ensure_sqrt(f, s);
        rss::launch_copy_cols(d_x, ld, d_y, ld, f->n, nrhs, s);
        check_launch();
        if (!adjoint) {
            // (prod V_i) P_t D^{1/2}: the top block first, then each record's L just before its V_i
            rss::launch_top_apply(f->top_idx, f->ntop, f->top_L, nullptr, d_y, nrhs, ld, f->work, s);
            check_launch();
            for (auto it = f->levels.rbegin(); it != f->levels.rend(); ++it)
                for (int col = 8; col >= 0; --col) {
                    rss::launch_apply_bwd(*it, it->d_rec_boxes[col], (int)it->rec_boxes[col].size(), d_y, nrhs, ld,
                                          it->Lc, s);
                    check_launch();
                }
        } else {
            // D^{1/2 *} P_t^* (prod' W_i): each W_i followed by its record's L^T, the top last
            for (auto& L : f->levels)
                for (int col = 0; col < 9; ++col) {
                    rss::launch_apply_fwd(L, L.d_rec_boxes[col], (int)L.rec_boxes[col].size(), d_y, nrhs, ld, L.Lc,
                                          s);
                    check_launch();
                }
            rss::launch_top_apply(f->top_idx, f->ntop, f->top_LT, nullptr, d_y, nrhs, ld, f->work, s);
            check_launch();
        }
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

rss_status rss_matvec(rss_factor f, const double* d_x, double* d_y, int32_t nrhs, int64_t ld, void* stream) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (!d_x || !d_y || nrhs < 1 || ld < f->n || d_x == d_y) { g_err = "bad matvec arguments"; return RSS_E_ARG; }
    hipStream_t s = (hipStream_t)stream;
    try {
        for (int h = 0; h < nrhs; ++h) {
            exact_matvec(f, d_x + h * ld, d_y + h * ld, s);
            check_launch();
        }
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

static void exact_matvec(rss_factor f, const double* x, double* y, hipStream_t s) {
    if (f->fft.ready) rss::launch_matvec_fft(f->fft, f->kp, x, y, s);
    else rss::launch_matvec_direct(f->pts, f->n, f->kp, x, y, s);
}

// Host side of the dot products: the partial sums of the blocks are copied into `hpart`
// (dot_partial_blocks(n) <= 1024 entries, caller-owned) and added in order.
static double ddot(rss_factor f, const double* x, const double* y, double* part, double* hpart, hipStream_t s) {
    const int nbk = rss::dot_partial_blocks(f->n);
    rss::launch_dot_partial(x, y, f->n, part, s);
    check_launch();
    HIPCHK(hipMemcpyAsync(hpart, part, sizeof(double) * nbk, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double acc = 0.0;
    for (int i = 0; i < nbk; ++i) acc += hpart[i];
    return acc;
}

// Device and host work arrays of one GMRES(restart) run on a factor of n DOFs.
struct GmresWork {
    double* V;      // n (restart + 1): Arnoldi basis
    double* Z;      // n restart: F^{-1} V (right preconditioning)
    double* rvec;   // n
    double* wvec;   // n
    double* part;   // 1024 partial dot products
    double* H;      // host (restart + 1) restart
    double* cs;     // host restart
    double* sn;     // host restart
    double* g;      // host restart + 1
    double* y;      // host restart
    double* hpart;  // host 1024
};

static size_t gmres_device_doubles(int64_t n, int restart) { return (size_t)n * (2 * (size_t)restart + 3) + 1024; }

// Right-preconditioned restarted GMRES(restart) with modified Gram-Schmidt, x0 = 0, stopping
// on the recomputed true residual; allocates nothing (every array comes in `w`).  Returns
// RSS_OK or RSS_E_NOCONV; throws Fail on device errors.
static rss_status gmres_run(rss_factor f, const double* d_b, double* d_x, double rtol, int maxit, int restart,
                            int use32, hipStream_t s, const GmresWork& w, int* iters, double* relres) {
    const int64_t n = f->n;
    const int ldh = restart + 1;
    int it = 0;
    double rr = 1.0;
    rss::launch_fill(d_x, 0.0, n, s);
    check_launch();
    const double nb = std::sqrt(ddot(f, d_b, d_b, w.part, w.hpart, s));
    if (nb == 0.0) {
        rr = 0.0;
    } else {
        rss::launch_scal_copy(1.0, d_b, w.rvec, n, s);
        check_launch();
        while (true) {
            const double beta = std::sqrt(ddot(f, w.rvec, w.rvec, w.part, w.hpart, s));
            rr = beta / nb;
            if (rr <= rtol || it >= maxit) break;
            rss::launch_scal_copy(1.0 / beta, w.rvec, w.V, n, s);
            check_launch();
            std::fill(w.H, w.H + (size_t)ldh * restart, 0.0);
            std::fill(w.g, w.g + ldh, 0.0);
            w.g[0] = beta;
            int m = 0;
            for (int j = 0; j < restart; ++j) {
                double* vj = w.V + (size_t)j * n;
                double* zj = w.Z + (size_t)j * n;
                rss::launch_scal_copy(1.0, vj, zj, n, s);
                check_launch();
                solve_impl(f, zj, 1, n, use32, s);
                exact_matvec(f, zj, w.wvec, s);
                check_launch();
                for (int i = 0; i <= j; ++i) {
                    const double hij = ddot(f, w.wvec, w.V + (size_t)i * n, w.part, w.hpart, s);
                    w.H[i + (size_t)j * ldh] = hij;
                    rss::launch_axpy(-hij, w.V + (size_t)i * n, w.wvec, n, s);
                    check_launch();
                }
                const double hn = std::sqrt(ddot(f, w.wvec, w.wvec, w.part, w.hpart, s));
                w.H[j + 1 + (size_t)j * ldh] = hn;
                for (int i = 0; i < j; ++i) {
                    const double a = w.H[i + (size_t)j * ldh], c2 = w.H[i + 1 + (size_t)j * ldh];
                    w.H[i + (size_t)j * ldh] = w.cs[i] * a + w.sn[i] * c2;
                    w.H[i + 1 + (size_t)j * ldh] = -w.sn[i] * a + w.cs[i] * c2;
                }
                const double hjj = w.H[j + (size_t)j * ldh], hj1 = w.H[j + 1 + (size_t)j * ldh];
                const double den = std::hypot(hjj, hj1);
                w.cs[j] = hjj / den;
                w.sn[j] = hj1 / den;
                w.H[j + (size_t)j * ldh] = den;
                w.H[j + 1 + (size_t)j * ldh] = 0.0;
                w.g[j + 1] = -w.sn[j] * w.g[j];
                w.g[j] = w.cs[j] * w.g[j];
                ++it;
                m = j + 1;
                if (std::fabs(w.g[j + 1]) / nb <= rtol || hn == 0.0 || it >= maxit) break;
                rss::launch_scal_copy(1.0 / hn, w.wvec, w.V + (size_t)(j + 1) * n, n, s);
                check_launch();
            }
            for (int i = m - 1; i >= 0; --i) {
                double acc = w.g[i];
                for (int l = i + 1; l < m; ++l) acc -= w.H[i + (size_t)l * ldh] * w.y[l];
                w.y[i] = acc / w.H[i + (size_t)i * ldh];
            }
            for (int i = 0; i < m; ++i) {
                rss::launch_axpy(w.y[i], w.Z + (size_t)i * n, d_x, n, s);
                check_launch();
            }
            exact_matvec(f, d_x, w.wvec, s);
            check_launch();
            rss::launch_scal_copy(1.0, d_b, w.rvec, n, s);
            check_launch();
            rss::launch_axpy(-1.0, w.wvec, w.rvec, n, s);
            check_launch();
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (rr > rtol) {
        g_err = "gmres did not reach rtol within maxit";
        return RSS_E_NOCONV;
    }
    return RSS_OK;
}

static GmresWork gmres_work_on(double* d, int64_t n, int restart) {
    GmresWork w{};
    w.V = d;
    w.Z = w.V + (size_t)n * (restart + 1);
    w.rvec = w.Z + (size_t)n * restart;
    w.wvec = w.rvec + n;
    w.part = w.wvec + n;
    return w;
}

rss_status rss_gmres(rss_factor f, const double* d_b, double* d_x, double rtol, int32_t maxit, int32_t restart,
                     int32_t use_fp32, void* stream, int32_t* iters, double* relres) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (!d_b || !d_x || d_b == d_x || !(rtol > 0) || maxit < 1 || restart < 1 || restart > 200) {
        g_err = "bad gmres arguments";
        return RSS_E_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int use32 = (use_fp32 && f->params.precision == RSS_MIXED) ? 1 : 0;
    const size_t nd = gmres_device_doubles(f->n, restart);
    double* d = nullptr;
    rss_status st = RSS_OK;
    try {
        d = dalloc<double>(f, nd, s);
        GmresWork w = gmres_work_on(d, f->n, restart);
        std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), y(restart),
            hpart(1024);
        w.H = H.data(); w.cs = cs.data(); w.sn = sn.data(); w.g = g.data(); w.y = y.data(); w.hpart = hpart.data();
        st = gmres_run(f, d_b, d_x, rtol, maxit, restart, use32, s, w, iters, relres);
    } catch (const Fail& e) {
        st = e.st;
    }
    if (d) dfree(f, d, sizeof(double) * nd, s);
    (void)hipStreamSynchronize(s);
    return st;
}

// ---- the entry point that allocates nothing ------------------------------------------------
// Work arrays of rss_gmres_noalloc: one array in the code object, so that the entry point
// never allocates; every GPU that runs the library holds its own copy, at its own address,
// from the module's load on that GPU until the process ends.  In host code `scratch` names
// a host-side stand-in, not device memory: host code uses only the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[RSS_GMRES_NOALLOC_BYTES / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per device).
double* scratch_on_current_device() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(RSS_E_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(RSS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (double*)p;
    }
    return g_scratch_dev[dev];
}
}  // namespace

rss_status rss_gmres_noalloc(rss_factor f, const double* d_b, double* d_x, double rtol, int32_t maxit,
                             int32_t restart, int32_t use_fp32, void* stream, int32_t* iters, double* relres) {
    constexpr int kMaxRestart = 64;
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (!d_b || !d_x || d_b == d_x || !(rtol > 0) || maxit < 1 || restart < 1 || restart > kMaxRestart) {
        g_err = "bad gmres arguments (rss_gmres_noalloc takes restart <= 64)";
        return RSS_E_ARG;
    }
    const size_t nd = gmres_device_doubles(f->n, restart);
    if (nd > RSS_GMRES_NOALLOC_BYTES / sizeof(double)) {
        g_err = "rss_gmres_noalloc needs (2 restart + 3) N + 1024 = " + std::to_string(nd) +
                " doubles, more than its " + std::to_string(RSS_GMRES_NOALLOC_BYTES / sizeof(double)) +
                " (lower restart, or use rss_gmres)";
        return RSS_E_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int use32 = (use_fp32 && f->params.precision == RSS_MIXED) ? 1 : 0;
    double H[(kMaxRestart + 1) * kMaxRestart], cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart],
        hpart[1024];
    try {
        GmresWork w = gmres_work_on(scratch_on_current_device(), f->n, restart);
        w.H = H; w.cs = cs; w.sn = sn; w.g = g; w.y = y; w.hpart = hpart;
        return gmres_run(f, d_b, d_x, rtol, maxit, restart, use32, s, w, iters, relres);
    } catch (const Fail& e) {
        (void)hipStreamSynchronize(s);
        return e.st;
    }
}

rss_status rss_logdet(rss_factor f, double* re, double* im) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (!re || !im) { g_err = "NULL argument"; return RSS_E_ARG; }
    try {
        double total = f->top_logdet;
        int sg = f->top_sign;
        for (auto& L : f->levels) {
            std::vector<double> ld = d2h(L.logdet_part, L.nbox, nullptr);
            std::vector<int> sgs = d2h(L.sign_part, L.nbox, nullptr);
            std::vector<int> hJ = d2h(L.nJ, L.nbox, nullptr);
            for (int b = 0; b < L.nbox; ++b)
                if (hJ[b] > 0) {
                    total += ld[b];
                    sg *= sgs[b];
                }
        }
        *re = total;
        *im = sg < 0 ? M_PI : 0.0;
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

rss_status rss_shape(rss_factor f, int32_t* depth, int64_t* n_top) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (depth) *depth = f->depth;
    if (n_top) *n_top = f->ntop;
    return RSS_OK;
}

rss_status rss_box_sets(rss_factor f, int32_t depth, int64_t box, int32_t weak, int64_t* skel, int32_t cap_s,
                        int32_t* ns, int64_t* red, int32_t cap_r, int32_t* nr) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    const rss::Level* L = nullptr;
    for (auto& l : f->levels)
        if (l.t == depth && l.weak == (weak ? 1 : 0)) L = &l;
    if (!L || box < 0 || box >= L->nbox || !ns || !nr) {
        g_err = "no skeletonized level / box with these indices";
        return RSS_E_ARG;
    }
    try {
        int n = L->h_cnt[box], k = L->h_k[box];
        int nJ = 0;
        HIPCHK(hipMemcpy(&nJ, L->nJ + box, sizeof(int), hipMemcpyDeviceToHost));
        int r = nJ > 0 ? n - k : 0;
        int s_cnt = nJ > 0 ? k : n;
        *ns = s_cnt;
        *nr = r;
        if (s_cnt > cap_s || r > cap_r || (s_cnt && !skel) || (r && !red)) {
            g_err = "capacity too small";
            return RSS_E_ARG;
        }
        std::vector<int> hs(std::max(s_cnt, 1)), hr(std::max(r, 1));
        if (nJ > 0) {
            if (k) HIPCHK(hipMemcpy(hs.data(), L->Sg + (size_t)box * L->nmax, sizeof(int) * k, hipMemcpyDeviceToHost));
            if (r) HIPCHK(hipMemcpy(hr.data(), L->Rg + (size_t)box * L->nmax, sizeof(int) * r, hipMemcpyDeviceToHost));
        } else if (n) {
            HIPCHK(hipMemcpy(hs.data(), L->gidx + (size_t)box * L->nmax, sizeof(int) * n, hipMemcpyDeviceToHost));
        }
        for (int i = 0; i < s_cnt; ++i) skel[i] = hs[i];
        for (int i = 0; i < r; ++i) red[i] = hr[i];
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

rss_status rss_box_record(rss_factor f, int32_t depth, int64_t box, int32_t weak, double* h_T, double* h_XRR,
                          double* h_XJR, double* h_G, int64_t* h_J, int64_t cap, int32_t* ns, int32_t* nr,
                          int32_t* nj) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    const rss::Level* L = nullptr;
    for (auto& l : f->levels)
        if (l.t == depth && l.weak == (weak ? 1 : 0)) L = &l;
    if (!L || box < 0 || box >= L->nbox || !ns || !nr || !nj) {
        g_err = "no skeletonized level / box with these indices";
        return RSS_E_ARG;
    }
    try {
        int nJ = 0;
        HIPCHK(hipMemcpy(&nJ, L->nJ + box, sizeof(int), hipMemcpyDeviceToHost));
        const int n = L->h_cnt[box], k = nJ > 0 ? L->h_k[box] : 0, r = nJ > 0 ? n - k : 0;
        *ns = k;
        *nr = r;
        *nj = nJ;
        if (nJ <= 0) return RSS_OK;
        const int64_t need_T = (int64_t)k * r, need_X = (int64_t)r * r, need_J = (int64_t)nJ * r;
        if ((h_T && need_T > cap) || (h_XRR && need_X > cap) || ((h_XJR || h_G) && need_J > cap) ||
            (h_J && nJ > cap)) {
            g_err = "capacity too small";
            return RSS_E_ARG;
        }
        const size_t nm = (size_t)L->nmax, ldJ = (size_t)L->ldJ;
        // column-major copies with the record's leading dimension removed
        auto get = [&](const double* src, size_t ld, int rows, int cols, double* dst) {
            if (!dst || rows == 0 || cols == 0) return;
            std::vector<double> h(ld * (size_t)cols);
            HIPCHK(hipMemcpy(h.data(), src, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
            for (int j = 0; j < cols; ++j)
                for (int i = 0; i < rows; ++i) dst[i + (size_t)rows * j] = h[i + ld * j];
        };
        get(L->T + (size_t)box * nm * nm, nm, k, r, h_T);
        get(L->XRR + (size_t)box * nm * nm, nm, r, r, h_XRR);
        get(L->XJR + (size_t)box * ldJ * nm, ldJ, nJ, r, h_XJR);
        get(L->G + (size_t)box * nm * ldJ, nm, r, nJ, h_G);
        if (h_J) {
            std::vector<int> hj(nJ);
            HIPCHK(hipMemcpy(hj.data(), L->Jg + (size_t)box * ldJ, sizeof(int) * nJ, hipMemcpyDeviceToHost));
            for (int i = 0; i < nJ; ++i) h_J[i] = hj[i];
        }
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

rss_status rss_top_set(rss_factor f, int64_t* idx, int64_t cap, int64_t* count) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (!count) { g_err = "NULL count"; return RSS_E_ARG; }
    *count = f->ntop;
    if (cap < f->ntop || (f->ntop && !idx)) { g_err = "capacity too small"; return RSS_E_ARG; }
    try {
        std::vector<int> h = d2h(f->top_idx, f->ntop, nullptr);
        for (int64_t i = 0; i < f->ntop; ++i) idx[i] = h[i];
    } catch (const Fail& e) {
        return e.st;
    }
    return RSS_OK;
}

rss_status rss_info(rss_factor f, char* buf, int64_t cap) {
    g_err.clear();
    if (guard_factor(f) != RSS_OK) return RSS_E_ARG;
    if (!buf || cap < 1) { g_err = "bad buffer"; return RSS_E_ARG; }
    std::ostringstream o;
    o.precision(17);
    o << "{\"n\":" << f->n << ",\"depth\":" << f->depth << ",\"top_depth\":" << f->top_depth
      << ",\"n_top\":" << f->ntop
      << ",\"precision\":\"" << (f->params.precision == RSS_MIXED ? "mixed" : "fp64") << "\""
      << ",\"method\":\"" << (f->params.method == RSS_METHOD_HYBRID ? "rs-ws" : "rs-s") << "\""
      << ",\"level_graphs\":" << f->params.level_graphs
      << ",\"exact_operator\":\"" << (f->fft.ready ? "fft" : "direct") << "\""
      << ",\"bytes_device\":" << f->bytes_device << ",\"lds_limit\":" << rss::elim_lds_limit() << ",\"wall_ms\":" << f->wall_ms << ",\"phase_ms\":{";
    for (int i = 0; i < PH_N; ++i) o << (i ? "," : "") << "\"" << kPhaseName[i] << "\":" << f->phase_ms[i];
    o << "},\"launches\":{";
    for (int i = 0; i < PH_N; ++i) o << (i ? "," : "") << "\"" << kPhaseName[i] << "\":" << f->kernel_launches[i];
    o << "},\"shapes\":[";
    for (size_t i = 0; i < f->shapes.size(); ++i) o << (i ? "," : "") << "\"" << f->shapes[i] << "\"";
    o << "],\"levels\":[";
    for (size_t i = 0; i < f->stats.size(); ++i) {
        const auto& s = f->stats[i];
        o << (i ? "," : "") << "{\"depth\":" << s.depth << ",\"pass\":\"" << (s.weak ? "weak" : "strong")
          << "\",\"boxes\":" << s.boxes << ",\"nmax\":" << s.nmax
          << ",\"records\":" << s.records << ",\"sum_k\":" << s.sum_k << ",\"sum_r\":" << s.sum_r
          << ",\"sum_J\":" << s.sum_J << ",\"max_k\":" << s.max_k << ",\"max_J\":" << s.max_J
          << ",\"flops_id\":" << s.flops_id << ",\"flops_x\":" << s.flops_x << ",\"flops_lu\":" << s.flops_lu
          << ",\"flops_g\":" << s.flops_g << ",\"flops_schur\":" << s.flops_schur
          << ",\"bytes_schur\":" << s.bytes_schur << ",\"bytes_solve64\":" << s.bytes_solve64
          << ",\"bytes_solve32\":" << s.bytes_solve32 << ",\"ms_id\":" << s.ms_id << ",\"ms_elim\":" << s.ms_elim
          << ",\"ms_schur\":" << s.ms_schur << ",\"flops_schur_self\":" << s.flops_schur_self
          << ",\"bytes_schur_self\":" << s.bytes_schur_self << ",\"ms_schur_self\":" << s.ms_schur_self
          << ",\"ms_graph\":" << s.ms_graph << "}";
    }
    o << "]}";
    std::string js = o.str();
    int64_t m = std::min<int64_t>(cap - 1, (int64_t)js.size());
    std::memcpy(buf, js.data(), m);
    buf[m] = 0;
    return RSS_OK;
}

}  // extern "C"
