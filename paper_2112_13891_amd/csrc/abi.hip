// abi.hip -- the C ABI of libfms and the host control of the method:
// argument checking, seed selection (SplitMix64 + partial Fisher-Yates on
// pool positions), the round loop of Algorithm 2 with the seed-count control
// of Section II-D, merge resolution and workspace management.
//
// Per round the host crosses to the device twice: once after the batch has
// iterated and the merge passes ran (status, merge state and positions come
// back), once after the pool was updated (its new length comes back).
// Within the batch the iterations are enqueued in chunks and the host only
// polls a pinned copy of the device control block between chunks.

#include <algorithm>
#include <atomic>
#include <immintrin.h>
#include <map>
#include <memory>
#include <mutex>
#include <sys/syscall.h>
#include <unistd.h>
#include <tuple>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "fms_internal.h"

// Device scratch of ms_step_noalloc: every workspace buffer of that call is
// carved out of it, so the call allocates nothing.  Each GPU the library runs
// on holds its own copy until the process ends.  In host code this name is
// only a handle for hipGetSymbolAddress: the device address it returns, kept
// per device, is the one passed to kernels.
static constexpr size_t kScratchBytes = 32ull << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace fms {

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? MS_E_NOMEM : MS_E_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define FMS_HIP(expr)                                              \
    do {                                                           \
        hipError_t _e = (expr);                                    \
        if (_e != hipSuccess) return hip_fail(_e, #expr);          \
    } while (0)

#define FMS_CHECK(expr)              \
    do {                             \
        int _rc = (expr);            \
        if (_rc != MS_OK) return _rc; \
    } while (0)

// ---- seed selection ---------------------------------------------------------

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).
struct SplitMix64 {
    uint64_t state;
    uint64_t next() {
        state += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
};

// Partial Fisher-Yates over positions 0..len-1, simulated sparsely: only the
// touched positions are stored.  pos[t] receives the position that ends up in
// slot t (slot t is final after its own swap, since later swaps only touch
// slots > t).  Swap partner of slot t: t + floor(r * (len - t) / 2^64).
// The touched positions live in an open-addressing table (linear probing,
// at most 2 * count keys in at least 4 * count entries), reused per thread.
struct TouchedPositions {
    std::vector<uint64_t> slot;   // (key << 32 | value), kEmpty when unused
    uint32_t mask = 0;
    static constexpr uint64_t kEmpty = ~0ull;
    void reset(int32_t count) {
        size_t cap = 16;
        while (cap < (size_t)count * 4) cap <<= 1;
        slot.assign(cap, kEmpty);
        mask = (uint32_t)cap - 1;
    }
    uint64_t* find(int32_t key) {
        uint32_t i = ((uint32_t)key * 0x9E3779B1u) & mask;
        for (;;) {
            uint64_t& e = slot[i];
            if (e == kEmpty || (int32_t)(uint32_t)(e >> 32) == key) return &e;
            i = (i + 1) & mask;
        }
    }
    int32_t get(int32_t key) {
        const uint64_t e = *find(key);
        return e == kEmpty ? key : (int32_t)(uint32_t)e;
    }
    void put(int32_t key, int32_t v) { *find(key) = ((uint64_t)(uint32_t)key << 32) | (uint32_t)v; }
};

void draw_positions(uint64_t* state, int32_t len, int32_t count, int32_t* pos) {
    SplitMix64 g{*state};
    static thread_local TouchedPositions moved;
    moved.reset(count);
    for (int32_t t = 0; t < count; ++t) {
        const uint64_t r = g.next();
        const int32_t j =
            t + (int32_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)(len - t)) >> 64);
        const int32_t vt = moved.get(t), vj = moved.get(j);
        moved.put(j, vt);
        moved.put(t, vj);
        pos[t] = vj;
    }
    *state = g.state;
}

// ---- device memory ------------------------------------------------------------

// Test hook: FMS_FAIL_ALLOC_AFTER=k makes the (k+1)-th allocation of a call fail.
struct AllocBudget {
    long long left = -1;
    AllocBudget() {
        const char* e = std::getenv("FMS_FAIL_ALLOC_AFTER");
        if (e && *e) left = std::atoll(e);
    }
    bool take() {
        if (left < 0) return true;
        if (left == 0) return false;
        --left;
        return true;
    }
};

// Stream-ordered device buffers owned by one call; freed on scope exit.
class Workspace {
   public:
    explicit Workspace(hipStream_t s) : s_(s) {}
    ~Workspace() {
        for (void* p : bufs_) (void)hipFreeAsync(p, s_);
    }
    template <typename T>
    int alloc(T** out, size_t count) {
        size_t bytes = std::max<size_t>(count * sizeof(T), 256);
        void* p = nullptr;
        if (!budget_.take()) return fail(MS_E_NOMEM, "device workspace allocation failed (test hook)");
        hipError_t e = hipMallocAsync(&p, bytes, s_);
        if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorOutOfMemory : e, "hipMallocAsync");
        bufs_.push_back(p);
        bytes_ += bytes;
        peak_ = std::max(peak_, bytes_);
        *out = (T*)p;
        return MS_OK;
    }
    template <typename T>
    void release(T* p) {
        for (size_t i = 0; i < bufs_.size(); ++i)
            if (bufs_[i] == (void*)p) {
                (void)hipFreeAsync(p, s_);
                bufs_.erase(bufs_.begin() + i);
                return;
            }
    }
    long long peak() const { return peak_; }

   private:
    hipStream_t s_;
    std::vector<void*> bufs_;
    AllocBudget budget_;
    long long bytes_ = 0, peak_ = 0;
};

// True on the process's initial thread.  Its thread-local caches are left to
// the end of the process (the HIP runtime may already be shutting down when
// they are destroyed).
bool on_initial_thread() { return (pid_t)syscall(SYS_gettid) == getpid(); }

// Buffers of host threads that have exited.  A thread's caches cannot be
// freed from its own exit (measured: hipFree / hipHostFree called from a
// thread-local destructor returned only part of the memory), so the exiting
// thread hands them here, and the next ms_fit or ms_fit_batched call on any
// thread, or ms_release_workspace, frees them: memory held for exited
// threads never outlives the next call.
std::mutex g_orphan_mu;
std::vector<void*> g_orphan_dev, g_orphan_host;

void free_orphans() {
    std::vector<void*> dev, host;
    {
        std::lock_guard<std::mutex> lock(g_orphan_mu);
        dev.swap(g_orphan_dev);
        host.swap(g_orphan_host);
    }
    for (void* q : dev) (void)hipFree(q);
    for (void* q : host) (void)hipHostFree(q);
}

// Pinned host staging, per thread, grown on demand and kept for reuse; handed
// to the orphan list when the thread exits, freed by ms_release_workspace.
struct Pinned {
    void* p = nullptr;
    size_t cap = 0;
    Pinned() = default;
    Pinned(const Pinned&) = delete;
    Pinned& operator=(const Pinned&) = delete;
    ~Pinned() {
        if (p && !on_initial_thread()) {
            std::lock_guard<std::mutex> lock(g_orphan_mu);
            g_orphan_host.push_back(p);
        }
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
    int ensure(size_t bytes) {
        if (bytes <= cap) return MS_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(bytes, 1 << 16);
        FMS_HIP(hipHostMalloc(&p, want, hipHostMallocDefault));
        cap = want;
        return MS_OK;
    }
};
thread_local Pinned g_pin_ctl, g_pin_pos, g_pin_rb, g_pin_modes;


int ensure_pool_release_threshold() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    FMS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (dev >= 0 && dev < 64 && !done[dev]) {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        done[dev] = true;
    }
    return MS_OK;
}

// ---- argument checks -------------------------------------------------------------

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

int check_common(const float* X, int64_t n, int32_t d) {
    if (!X) return fail(MS_E_INVALID, "X is NULL");
    if (n < 1 || n > INT_MAX) return fail(MS_E_INVALID, "n must be in [1, 2^31-1]");
    if (d < 1 || d > 256) return fail(MS_E_INVALID, "d must be in [1, 256]");
    if ((long long)n * step_shape(d).DP > (1LL << 40))
        return fail(MS_E_INVALID, "n*d too large");
    return MS_OK;
}

int check_params(const ms_params* p, bool for_fit) {
    if (!p) return fail(MS_E_INVALID, "params is NULL");
    if (!finite_pos(p->h)) return fail(MS_E_INVALID, "h must be finite and > 0");
    if (p->kernel != MS_KERNEL_FLAT && p->kernel != MS_KERNEL_GAUSSIAN)
        return fail(MS_E_INVALID, "unknown kernel");
    if (p->precision != MS_PREC_FP32 && p->precision != MS_PREC_BF16_REFINE)
        return fail(MS_E_INVALID, "unknown precision");
    if (!finite_pos(p->tol)) return fail(MS_E_INVALID, "tol must be finite and > 0");
    if (!std::isfinite(p->tol * p->h) || p->tol * p->h <= 0.0f)
        return fail(MS_E_INVALID, "tol*h must be a positive finite float");
    if (p->precision == MS_PREC_BF16_REFINE && !(std::isfinite(p->refine_radius) && p->refine_radius >= 0.0f))
        return fail(MS_E_INVALID, "refine_radius must be finite and >= 0");
    if (p->metric != MS_METRIC_EUCLIDEAN && p->metric != MS_METRIC_COSINE)
        return fail(MS_E_INVALID, "unknown metric");
    if (p->graph != 0 && p->graph != 1) return fail(MS_E_INVALID, "graph must be 0 or 1");
    if (p->tile_R != 0 && p->tile_R != 1 && p->tile_R != 2 && p->tile_R != 4)
        return fail(MS_E_INVALID, "tile_R must be 0, 1, 2 or 4");
    if (p->plain != 0 && p->plain != 1) return fail(MS_E_INVALID, "plain must be 0 or 1");
    if (p->tile_chunk != 0 && (p->tile_chunk < 64 || p->tile_chunk > 65536))
        return fail(MS_E_INVALID, "tile_chunk must be 0 or in [64, 65536]");
    if (p->tile_grid < 0 || p->tile_grid > 65536) return fail(MS_E_INVALID, "tile_grid must be in [0, 65536]");
    if (p->reserved[0] != 0) return fail(MS_E_INVALID, "reserved fields must be 0");
    if (!for_fit) return MS_OK;
    if (p->max_iter < 1 || p->max_iter > kMaxIterCap)
        return fail(MS_E_INVALID, "max_iter must be in [1, 4096]");
    if (!(std::isfinite(p->merge_radius) && p->merge_radius >= 0.0f))
        return fail(MS_E_INVALID, "merge_radius must be finite and >= 0");
    if (!(std::isfinite(p->cover_radius) && p->cover_radius >= 0.0f))
        return fail(MS_E_INVALID, "cover_radius must be finite and >= 0");
    if (!(p->gamma > 0.0f && p->gamma <= 1.0f)) return fail(MS_E_INVALID, "gamma must be in (0, 1]");
    if (p->n_initial < 1) return fail(MS_E_INVALID, "n_initial must be >= 1");
    if (p->L < 1) return fail(MS_E_INVALID, "L must be >= 1");
    return MS_OK;
}

float packed_scale(const ms_params* p) {
    if (p->kernel != MS_KERNEL_GAUSSIAN) return 1.0f;
    // w = exp(-q/(2h^2)) = exp2(-|c x - c s|^2) with c^2 = log2(e)/(2h^2)
    return (float)std::sqrt(1.4426950408889634 / (2.0 * (double)p->h * (double)p->h));
}

// ---- cached device workspace of ms_fit ----------------------------------------------

// ms_fit is host-synchronous, so one thread never has two fits in flight: its
// device buffers can be kept and reused by the next fit on the same thread
// and device (grown on demand, never shrunk).
enum Slot {
    SL_XP, SL_RB, SL_POOL0, SL_POOL1, SL_REMOVED, SL_BLOCKS, SL_MODES, SL_ACT0, SL_ACT1,
    SL_SHIFT2, SL_PART, SL_POS, SL_FLAG, SL_XS, SL_PERM, SL_GEOM, SL_SORTWS, SL_FEAT, SL_XN,
    SL_JPTS, SL_JSEEDS, SL_JMODES, SL_COVERED, SL_CAND,
    // ms_fit_batched's rounds and the batched steps they run
    SL_BCONV, SL_BITERS, SL_BS, SL_BSH2, SL_BNM, SL_BSTATE, SL_BSTEP_S, SL_BSTEP_ACT0, SL_BSTEP_ACT1, SL_BSTEP_STATUS,
    SL_BSTEP_ITERS, SL_BSTEP_SHIFT2, SL_BSTEP_CNT, SL_BSTEP_PLAN, SL_BSTEP_ITEMC, SL_BSTEP_SLOTC, SL_BSTEP_PART,
    SL_COUNT
};

// Handed to the orphan list when the thread exits (freed by the next call on
// any thread), freed by ms_release_workspace.
struct DevCache {
    int dev = -1;
    void* p[SL_COUNT] = {};
    size_t cap[SL_COUNT] = {};
    long long held = 0;
    DevCache() = default;
    DevCache(const DevCache&) = delete;
    DevCache& operator=(const DevCache&) = delete;
    ~DevCache() {
        if (on_initial_thread()) return;
        std::lock_guard<std::mutex> lock(g_orphan_mu);
        for (int i = 0; i < SL_COUNT; ++i)
            if (p[i]) g_orphan_dev.push_back(p[i]);
    }
    void release() {
        for (int i = 0; i < SL_COUNT; ++i) {
            if (p[i]) (void)hipFree(p[i]);
            p[i] = nullptr;
            cap[i] = 0;
        }
        held = 0;
    }
};
thread_local std::vector<std::unique_ptr<DevCache>> g_cache;

DevCache& cache_for_device(int dev) {
    for (auto& c : g_cache)
        if (c->dev == dev) return *c;
    g_cache.emplace_back(new DevCache());
    g_cache.back()->dev = dev;
    return *g_cache.back();
}

template <typename T>
int cache_get(DevCache& c, AllocBudget& budget, Slot sl, size_t count, T** out,
              bool keep_contents = false, hipStream_t s = nullptr) {
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (c.cap[sl] < bytes) {
        if (!budget.take()) return fail(MS_E_NOMEM, "device workspace allocation failed (test hook)");
        const size_t want = std::max(bytes, c.cap[sl] + c.cap[sl] / 2);
        void* np = nullptr;
        hipError_t e = hipMalloc(&np, want);
        if (e != hipSuccess || !np) return hip_fail(e == hipSuccess ? hipErrorOutOfMemory : e, "hipMalloc");
        if (c.p[sl]) {
            if (keep_contents) {
                hipError_t e2 = hipMemcpyAsync(np, c.p[sl], c.cap[sl], hipMemcpyDeviceToDevice, s);
                if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
                if (e2 != hipSuccess) {
                    (void)hipFree(np);
                    return hip_fail(e2, "workspace grow copy");
                }
            }
            (void)hipFree(c.p[sl]);
            c.held -= (long long)c.cap[sl];
        }
        c.p[sl] = np;
        c.cap[sl] = want;
        c.held += (long long)want;
    }
    *out = (T*)c.p[sl];
    return MS_OK;
}

// Layout of the per-round readback buffer: the control block first, then the
// batch arrays the host needs, sized for the current batch B so that one
// contiguous copy brings everything back.
struct RbLayout {
    size_t state, ids, iters, status, S, total;
};

RbLayout rb_layout(int B, int DP) {
    auto up = [](size_t v, size_t a) { return (v + a - 1) / a * a; };
    RbLayout L;
    size_t o = up(sizeof(Ctl), 256);
    L.state = o; o += (size_t)B * 4;
    L.ids = o; o += (size_t)B * 4;
    L.iters = o; o += (size_t)B * 4;
    L.status = o; o += (size_t)B;
    o = up(o, 16);
    L.S = o; o += (size_t)B * DP * 4;
    L.total = up(o, 256);
    return L;
}

// Host-mapped progress word of this thread's fits: the step kernel of
// iteration t stores (t << 32 | active seeds) into it.
struct ProgressWord {
    unsigned long long* host = nullptr;
    unsigned long long* dev = nullptr;
    int ensure() {
        if (host) return MS_OK;
        void* p = nullptr;
        FMS_HIP(hipHostMalloc(&p, 64, hipHostMallocMapped | hipHostMallocCoherent));
        void* d = nullptr;
        hipError_t e = hipHostGetDevicePointer(&d, p, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(p);
            return hip_fail(e, "hipHostGetDevicePointer");
        }
        host = (unsigned long long*)p;
        dev = (unsigned long long*)d;
        return MS_OK;
    }
    ~ProgressWord() {
        if (host) (void)hipHostFree(host);
    }
};
thread_local ProgressWord g_prog;

// Waits for the work queued on the stream by polling it.  The fit's host
// decisions wait on short device tails, where the wake-up of a blocking wait
// costs more than the tail itself.  Only for work whose host-side results are
// in pinned memory (copies to pageable memory keep hipStreamSynchronize).
hipError_t wait_stream(hipStream_t s) {
    for (;;) {
        const hipError_t q = hipStreamQuery(s);
        if (q != hipErrorNotReady) return q;
        for (int i = 0; i < 64; ++i) _mm_pause();
    }
}

// Enqueue iterations, keeping at most kAhead of them queued beyond the one the
// device last reported starting, until an iteration reports no active seed
// (every later one would find none either) or max_iter were enqueued.  If the
// stream drains without a new report, the control block is read back instead.
int iterate_batch(Batch& b, int max_iter, hipStream_t s, Ctl* mirror) {
    // one iteration queued behind the running one: an iteration lasts longer
    // than the host needs to see it start and enqueue the next
    constexpr int kAhead = 1;
    constexpr unsigned long long kNone = ~0ull;
    volatile unsigned long long* word = g_prog.host;
    *word = kNone;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    b.prog = g_prog.dev;
    int launched = 0;
    for (;;) {
        const unsigned long long w = *word;
        const int t_obs = w == kNone ? -1 : (int)(w >> 32);
        const int m_obs = (int)(w & 0xffffffffu);
        if (t_obs >= 0 && m_obs == 0) break;
        if (launched >= max_iter) break;
        if (launched - (t_obs + 1) < kAhead) {
            FMS_HIP(launch_iteration(b, launched, s));
            ++launched;
            continue;
        }
        // wait for the device to start another iteration
        bool moved = false;
        for (int spin = 0; spin < 4096 && !moved; ++spin) {
            if (*word != w) moved = true;
            else _mm_pause();
        }
        if (moved) continue;
        const hipError_t q = hipStreamQuery(s);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return hip_fail(q, "hipStreamQuery");
        if (*word != w) continue;
        // drained with no newer report: decide from the control block
        FMS_HIP(hipMemcpyAsync(mirror, b.ctl, offsetof(Ctl, conv_it) + (size_t)(launched + 1) * 4,
                               hipMemcpyDeviceToHost, s));
        FMS_HIP(wait_stream(s));
        int conv = 0;
        for (int u = 0; u < launched; ++u) conv += mirror->conv_it[u];
        if (conv >= mirror->need || mirror->count[launched % 3] == 0) break;
        FMS_HIP(launch_iteration(b, launched, s));
        ++launched;
    }
    b.prog = nullptr;
    return MS_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// The executable graph of ms_step_batched's iterations and its capture
// stream, per host thread (released by ms_release_workspace; a thread that
// exits keeps its handles, a few kilobytes of host state, to the end of the
// process).
struct GraphCache {
    int dev = -1;
    hipStream_t cs = nullptr;
    hipGraphExec_t ge = nullptr;
    long long instantiations = 0, updates = 0;
    void clear() {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (cs) (void)hipStreamDestroy(cs);
        ge = nullptr;
        cs = nullptr;
        dev = -1;
    }
};
thread_local GraphCache g_graph;

struct Events {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Events() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
    int create() {
        for (auto& x : e)
            if (!x) FMS_HIP(hipEventCreate(&x));
        return MS_OK;
    }
};
thread_local Events g_events;

bool log_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("MS_LOG");
        return e && *e && *e != '0';
    }();
    return on;
}

// FP32 squared distance with the same operation order as the device kernels.
float host_dist2(const float* a, const float* b, int d) {
    float q = 0.0f;
    for (int k = 0; k < d; ++k) {
        float t = a[k] - b[k];
        q = std::fmaf(t, t, q);
    }
    return q;
}

// Refine threshold of the BF16 form on E = -|x - s|^2 in packed units.  For
// D <= 4 pairs within refine_radius * h are recomputed exactly (at least h for
// the flat window, whose non-refined pairs get weight 0); for larger D every
// pair whose Gaussian weight may exceed 2^-127 (every pair that may lie in the
// flat window) is computed exactly and the others contribute nothing.
float bf16_e_thr(const ms_params* p, int D) {
    if (D > 4) {
        if (p->kernel == MS_KERNEL_GAUSSIAN) return -127.0f;
        return -(float)((double)p->h * p->h);
    }
    if (p->kernel == MS_KERNEL_GAUSSIAN)
        return -(float)((double)p->refine_radius * p->refine_radius * 1.4426950408889634 / 2.0);
    const double rr = std::max(1.0, (double)p->refine_radius) * p->h;
    return -(float)(rr * rr);
}

// Distance (original units) within which the BF16 form computes every pair
// exactly in FP32: its refine threshold.  Directions are at most a chord of 2
// apart, so for the cosine metric a reach of 2 or more means every pair is
// computed exactly -- the plain FP32 step, which then runs in its place.
double bf16_exact_reach(const ms_params* p, int D) {
    const double e = -(double)bf16_e_thr(p, D);
    return std::sqrt(std::max(0.0, e)) / (double)packed_scale(p);
}

bool bf16_form(const ms_params* p, int d) {
    if (p->precision != MS_PREC_BF16_REFINE) return false;
    return !(p->metric == MS_METRIC_COSINE && bf16_exact_reach(p, step_shape(d).D) >= 2.0);
}

// Pairs from which the merge and the pool coverage take the block join
// instead of the brute-force passes (MS_JOIN_PAIRS overrides both, e.g. 0 to
// take the join whenever the sides are large enough).
constexpr long long kJoinMergePairs = 1LL << 27;
constexpr long long kJoinCoverPairs = 1LL << 28;
long long join_pairs_min(long long dflt) {
    const char* e = std::getenv("MS_JOIN_PAIRS");
    if (e && *e) return std::atoll(e);
    return dflt;
}

struct SortedPoints {
    float* Xs = nullptr;
    int32_t* perm = nullptr;
    void* sws = nullptr;   // sort workspace (holds the point bounds)
    float* geom = nullptr;
    char* feat = nullptr;
};

void fill_batch(Batch& b, int n, int d, int B, const StepShape& sh, const ms_params* p,
                float scale, const float* Xp, Ctl* ctl, const SortedPoints* sp = nullptr) {
    const float tolh = p->tol * p->h;
    b.prec = bf16_form(p, d) ? MS_PREC_BF16_REFINE : MS_PREC_FP32;   // the form that runs
    b.Xs = sp ? sp->Xs : nullptr;
    b.geom = sp ? sp->geom : nullptr;
    b.pf = sp ? sp->feat : nullptr;
    b.xv = (sp && sp->feat && sh.D <= 4) ? sp->feat + (size_t)((n + 255) / 256) * 256 * 16 * 2 : nullptr;
    b.shift = (sp && sh.D > 4) ? sort_frame_shift(sp->sws) : nullptr;
    b.e_thr = bf16_e_thr(p, sh.D);
    b.kappa = 1.0f / 1024.0f;
    b.n = n;
    b.d = d;
    b.n_seeds = B;
    b.sh = sh;
    b.kernel = p->kernel;
    b.h = p->h;
    b.scale = scale;
    b.inv_scale = 1.0f / scale;
    b.thr2 = tolh * tolh;
    b.Xp = Xp;
    b.grid = step_grid(sh, B, n);
    b.metric = p->metric;
    b.ctl = ctl;
}

int fit_impl(const ms_params* p, const float* X, int n, int d, float* modes, int32_t max_modes,
             int32_t* k_out, int32_t* labels, ms_diag* diag, hipStream_t s) {
    const auto t_start = std::chrono::steady_clock::now();
    free_orphans();
    const bool trace = log_enabled();
    int dev = 0;
    FMS_HIP(hipGetDevice(&dev));
    DevCache& C = cache_for_device(dev);
    AllocBudget budget;
    FMS_CHECK(g_events.create());
    hipEvent_t* ev = g_events.e;

    if (p->check_finite) {
        int32_t* flag;
        FMS_CHECK(cache_get(C, budget, SL_FLAG, 1, &flag));
        FMS_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
        FMS_HIP(launch_check_finite(X, (long long)n * d, flag, s));
        int32_t hflag = 0;
        FMS_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMS_HIP(hipStreamSynchronize(s));   // pageable destination: the blocking wait
        if (hflag) return fail(MS_E_NONFINITE, "X contains NaN or Inf");
    }
    if (p->metric == MS_METRIC_COSINE) {
        // the method runs on the directions of the rows
        float* Xn;
        int32_t* flag;
        FMS_CHECK(cache_get(C, budget, SL_XN, (size_t)n * d, &Xn));
        FMS_CHECK(cache_get(C, budget, SL_FLAG, 1, &flag));
        FMS_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
        FMS_HIP(launch_normalize_rows(X, n, d, Xn, flag, s));
        int32_t hflag = 0;
        FMS_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMS_HIP(hipStreamSynchronize(s));   // pageable destination: the blocking wait
        if (hflag) return fail(MS_E_INVALID, "cosine metric: a row of X has no direction (length 0 or not finite)");
        X = Xn;
    }

    const StepShape base = step_shape(d);
    const int DP = base.DP;
    const bool all = p->all_points_as_seeds != 0;
    const float scale = packed_scale(p);
    const float rm = p->merge_radius * p->h, rc = p->cover_radius * p->h;
    const float r2m = rm * rm, r2c = rc * rc;

    float* Xp;
    FMS_CHECK(cache_get(C, budget, SL_XP, (size_t)n * DP, &Xp));
    FMS_HIP(launch_pack_points(X, n, d, DP, scale, Xp, s));
    const bool bf16 = bf16_form(p, d);
    // FP32 on enough points: spatially ordered points and block culling
    // (directions are at most 2 apart: nothing to cull when the reach is 2)
    const bool cull = !bf16 && !p->plain && cull_supported(d, n) &&
                      !(p->metric == MS_METRIC_COSINE && cull_reach(p->kernel, p->h) >= 2.0);
    const bool sorted = bf16 || cull;
    SortedPoints sp;
    if (sorted) {
        FMS_CHECK(cache_get(C, budget, SL_XS, (size_t)n * DP, &sp.Xs));
        FMS_CHECK(cache_get(C, budget, SL_PERM, n, &sp.perm));
        FMS_CHECK(cache_get(C, budget, SL_GEOM, (size_t)((n + 255) / 256) * geom_stride(base.D), &sp.geom));
        FMS_CHECK(cache_get(C, budget, SL_SORTWS, sort_workspace_bytes(n), (char**)&sp.sws));
        FMS_HIP(launch_spatial_sort(Xp, n, DP, base.D, sp.Xs, sp.perm, sp.geom, sp.sws, s));
    }
    if (bf16) {
        FMS_CHECK(cache_get(C, budget, SL_FEAT, base.D <= 4 ? bf16_feature_bytes(n)
                                                           : bf16_wide_feature_bytes(n, base.D, p->kernel),
                            &sp.feat));
        if (base.D <= 4) FMS_HIP(launch_bf16_features(sp.Xs, n, d, sp.geom, sp.feat, s));
        else FMS_HIP(launch_bf16_wide_features(sp.Xs, n, base.D, sp.geom, sp.feat, p->kernel, s));
    }

    int32_t* pool[2] = {nullptr, nullptr};
    uint8_t* removed = nullptr;
    int32_t* block_tmp = nullptr;
    int pool_len = n;
    if (!all) {
        FMS_CHECK(cache_get(C, budget, SL_POOL0, n, &pool[0]));
        FMS_CHECK(cache_get(C, budget, SL_POOL1, n, &pool[1]));
        FMS_CHECK(cache_get(C, budget, SL_REMOVED, n, &removed));
        FMS_CHECK(cache_get(C, budget, SL_BLOCKS, pool_compact_blocks(n) + 1, &block_tmp));
        FMS_HIP(launch_iota(pool[0], n, s));
        FMS_HIP(launch_fill_u8(removed, n, 0, s));   // kept clear by each compaction
    }

    // block join (spatially ordered sides) for the round epilogue and the
    // labels once the modes are many; the points are indexed when first needed
    const bool join_ok = join_shape_ok(base.D);
    JoinIndex jpts{};
    bool have_jpts = false;
    auto points_index = [&]() -> int {
        if (have_jpts) return MS_OK;
        char* w;
        FMS_CHECK(cache_get(C, budget, SL_JPTS, join_layout(n, DP, base.D).total, &w));
        FMS_HIP(launch_join_index(X, n, d, d, DP, base.D, scale, w, &jpts, s));
        have_jpts = true;
        return MS_OK;
    };

    // device mode store (DP stride), grown on demand
    int Kcap = std::min(n, 1024);
    float* modes_ws;
    FMS_CHECK(cache_get(C, budget, SL_MODES, (size_t)Kcap * DP, &modes_ws));
    std::vector<int32_t> counts;
    // the mode each drawn point's seed ended in: a start for the labels' join
    std::vector<int32_t> cand;

    FMS_CHECK(g_pin_ctl.ensure(2 * sizeof(Ctl)));
    Ctl* mirror = (Ctl*)g_pin_ctl.p;
    FMS_CHECK(g_prog.ensure());

    uint64_t rng = p->rng_seed;
    long long N = p->n_initial;
    int K = 0, rounds = 0;
    long long pairs = 0, refined = 0, drawn_total = 0;
    double iterate_ms = 0.0, merge_ms = 0.0;
    int cur = 0;
    if (trace) std::fprintf(stderr, "[fms] fit n=%d d=%d setup %.3f ms\n", n, d, ms_since(t_start));

    for (;;) {
        const auto t_round = std::chrono::steady_clock::now();
        const int B = all ? n : (int)std::min<long long>(N, pool_len);
        const StepShape sh = bf16 ? step_shape_bf16(d, B)
                                  : (cull ? step_shape_cull(d, B, n) : step_shape_for(d, B));
        Batch b;
        fill_batch(b, n, d, B, sh, p, scale, Xp, nullptr, sorted ? &sp : nullptr);
        const long long part_floats = step_part_floats(sh, B, b.grid);
        const RbLayout L = rb_layout(B, DP);
        char* rbuf;
        FMS_CHECK(cache_get(C, budget, SL_RB, L.total, &rbuf));
        Ctl* ctl = (Ctl*)rbuf;
        b.ctl = ctl;
        // the pool length lives in the control block across rounds; keep it
        int32_t* bstate = (int32_t*)(rbuf + L.state);
        int32_t* bids = (int32_t*)(rbuf + L.ids);
        b.iters = (int32_t*)(rbuf + L.iters);
        b.status = (uint8_t*)(rbuf + L.status);
        b.S = (float*)(rbuf + L.S);
        FMS_CHECK(cache_get(C, budget, SL_ACT0, B, &b.act[0]));
        FMS_CHECK(cache_get(C, budget, SL_ACT1, B, &b.act[1]));
        FMS_CHECK(cache_get(C, budget, SL_SHIFT2, B, &b.shift2));
        FMS_CHECK(cache_get(C, budget, SL_PART, (size_t)part_floats, &b.part));

        const int need = (int)std::ceil((double)p->gamma * (double)B);
        int32_t* dpos = nullptr;
        if (!all) {
            FMS_CHECK(cache_get(C, budget, SL_POS, B, &dpos));
            FMS_CHECK(g_pin_pos.ensure((size_t)B * sizeof(int32_t)));
            int32_t* hpos = (int32_t*)g_pin_pos.p;
            draw_positions(&rng, pool_len, B, hpos);
            FMS_HIP(hipMemcpyAsync(dpos, hpos, (size_t)B * sizeof(int32_t), hipMemcpyHostToDevice, s));
        }
        FMS_HIP(launch_round_init(X, d, DP, all ? nullptr : pool[cur], dpos, B, bids, removed,
                                  bstate, b, need, p->max_iter, s));
        if (sorted) {
            // seeds that are close in space share waves (refine work, culled blocks)
            if (all)
                FMS_HIP(hipMemcpyAsync(b.act[0], sp.perm, (size_t)B * 4, hipMemcpyDeviceToDevice, s));
            else
                FMS_HIP(launch_seed_order(b.S, DP, b.sh.D, B, scale, b.status, sp.sws, b.act[0], Xp, n, s));
        }

        FMS_HIP(hipEventRecord(ev[2], s));
        FMS_CHECK(iterate_batch(b, p->max_iter, s, mirror));
        FMS_HIP(hipEventRecord(ev[3], s));
        const auto t_merge = std::chrono::steady_clock::now();

        // merge ("prune modes"): old modes first, then parallel decision
        // passes; if they decide every seed, the founders are numbered and
        // appended to the mode store on the device, so that pool coverage and
        // compaction follow without a host round trip
        const int K_old = K;
        if ((long long)K_old + B > Kcap) {
            int newcap = std::max(Kcap * 2, K_old + B);
            newcap = std::min(newcap, n);
            FMS_CHECK(cache_get(C, budget, SL_MODES, (size_t)newcap * DP, &modes_ws, true, s));
            Kcap = newcap;
        }
        const int kPasses = 3;
        // many seeds: their final positions are indexed once, for the merge
        // (against the old modes, then the decision passes among the seeds)
        // and, as the new modes, for the pool coverage
        // (only when the brute-force passes would compare many pairs: the
        // index builds cost about a millisecond, the brute-force decision and
        // coverage passes run 1e8 pairs in a fraction of one).  The coverage
        // compares the pool with the round's founders, estimated from the
        // founders per drawn seed so far
        const long long est_founders =
            drawn_total > 0 ? ((long long)B * K_old + drawn_total - 1) / drawn_total : (long long)B;
        const bool join_merge =
            join_ok && B >= kJoinMin && (long long)B * ((long long)K_old + B) >= join_pairs_min(kJoinMergePairs);
        const bool join_cover = join_ok && !all && B >= kJoinMin && n >= kJoinMin &&
                                (long long)pool_len * est_founders >= join_pairs_min(kJoinCoverPairs);
        JoinIndex jseeds{};
        if (join_merge || join_cover) {
            char* w;
            FMS_CHECK(cache_get(C, budget, SL_JSEEDS, join_layout(B, DP, base.D).total, &w));
            FMS_HIP(launch_join_index(b.S, B, DP, d, DP, base.D, scale, w, &jseeds, s));
        }
        if (join_merge) {
            if (K_old > 0) {
                char* w;
                JoinIndex jmodes{};
                FMS_CHECK(cache_get(C, budget, SL_JMODES, join_layout(K_old, DP, base.D).total, &w));
                FMS_HIP(launch_join_index(modes_ws, K_old, DP, d, DP, base.D, scale, w, &jmodes, s));
                FMS_HIP(launch_join(JOIN_FIRST, jseeds, jmodes, DP, base.D, r2m, nullptr, nullptr, b.status, bstate,
                                    nullptr, nullptr, 0, nullptr, s));
            }
            for (int q = 0; q < kPasses; ++q)
                FMS_HIP(launch_join(JOIN_DECIDE, jseeds, jseeds, DP, base.D, r2m, nullptr, nullptr, b.status,
                                    bstate, nullptr, nullptr, 0, nullptr, s, K_old, q == 0, &ctl->und[q]));
        } else {
            for (int q = 0; q < kPasses; ++q)
                FMS_HIP(launch_merge_decide_pass(b.S, DP, d, b.status, B, modes_ws, K_old, K_old, r2m, bstate,
                                                 &ctl->und[q], q == 0, s));
        }
        FMS_HIP(launch_merge_founders(b.S, DP, B, K_old, bstate, modes_ws, ctl, kPasses - 1, block_tmp, s));
        if (!all) {
            // seed pool: drop the drawn seeds and the points the new modes
            // cover, keep the rest in ascending order
            if (join_cover) {
                uint8_t* covered;
                FMS_CHECK(points_index());
                FMS_CHECK(cache_get(C, budget, SL_COVERED, n, &covered));
                FMS_HIP(launch_fill_u8(covered, n, 0, s));
                FMS_HIP(launch_join(JOIN_ANY, jpts, jseeds, DP, base.D, r2c, nullptr, nullptr, nullptr, nullptr,
                                    bstate, ctl, kPasses - 1, covered, s));
                FMS_HIP(launch_pool_mark(pool[cur], pool_len, covered, removed, block_tmp, s));
            } else {
                FMS_HIP(launch_cover(X, d, pool[cur], pool_len, modes_ws, K_old, 0, ctl, r2c, removed,
                                     block_tmp, s));
            }
            FMS_HIP(launch_pool_compact(pool[cur], removed, pool_len, pool[cur ^ 1], block_tmp, ctl, s));
        }

        // one copy brings back the control block and the batch
        FMS_CHECK(g_pin_rb.ensure(L.total));
        char* hrb = (char*)g_pin_rb.p;
        FMS_HIP(hipMemcpyAsync(hrb, rbuf, L.total, hipMemcpyDeviceToHost, s));
        FMS_HIP(wait_stream(s));
        const Ctl& cs = *(const Ctl*)hrb;
        const int32_t* h_state = (const int32_t*)(hrb + L.state);
        const int32_t* h_ids = (const int32_t*)(hrb + L.ids);
        const int32_t* h_iters = (const int32_t*)(hrb + L.iters);
        const uint8_t* h_status = (const uint8_t*)(hrb + L.status);
        const float* h_S = (const float*)(hrb + L.S);
        {
            float ms = 0.0f;
            FMS_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
            iterate_ms += ms;
        }
        pairs += cs.pairs;
        refined += ctl_refined(cs);
        if (!all) pool_len = cs.pool_len;
        const bool host_merge = cs.merge_host != 0;

        // number the founders in seed order; with host_merge, a seed the
        // device passes left undecided gets the same rule here (all earlier
        // seeds are decided by the time it is reached, so this is exact)
        std::vector<int32_t> mode_of(B, -1);
        std::vector<int32_t> founders;
        for (int i = 0; i < B; ++i) {
            int st = h_state[i];
            if (st == MG_SKIP) continue;
            if (st == MG_UNDECIDED) {
                st = MG_FOUNDER;
                const float* si = h_S + (size_t)i * DP;
                for (int j : founders) {   // increasing seed order
                    if (host_dist2(si, h_S + (size_t)j * DP, d) <= r2m) {
                        st = K_old + j;
                        break;
                    }
                }
            }
            if (st == MG_FOUNDER) {
                mode_of[i] = K;
                founders.push_back(i);
                counts.push_back(1);
                ++K;
            } else if (st >= K_old) {
                mode_of[i] = mode_of[st - K_old];
                counts[mode_of[i]] += 1;
            } else {
                mode_of[i] = st;
                counts[st] += 1;
            }
        }
        if (!host_merge && K != cs.k_new)
            return fail(MS_E_HIP, "merge: device and host founder counts differ");
        if (join_ok && n >= kJoinMin) {
            if (cand.empty()) cand.assign(n, -1);
            for (int i = 0; i < B; ++i)
                if (mode_of[i] >= 0) cand[h_ids[i]] = mode_of[i];
        }
        if (host_merge && K > K_old) {
            FMS_CHECK(g_pin_modes.ensure((size_t)(K - K_old) * DP * 4));
            float* hm = (float*)g_pin_modes.p;
            for (int q = 0; q < K - K_old; ++q)
                std::memcpy(hm + (size_t)q * DP, h_S + (size_t)founders[q] * DP, (size_t)DP * 4);
            FMS_HIP(hipMemcpyAsync(modes_ws + (size_t)K_old * DP, hm, (size_t)(K - K_old) * DP * 4,
                                   hipMemcpyHostToDevice, s));
            if (!all && pool_len > 0) {
                // the device covered nothing new: cover the compacted pool now
                // and compact it back into the current buffer
                FMS_HIP(launch_cover(X, d, pool[cur ^ 1], pool_len, modes_ws, K_old, K, nullptr, r2c,
                                     removed, block_tmp, s));
                FMS_HIP(launch_pool_compact(pool[cur ^ 1], removed, pool_len, pool[cur], block_tmp, ctl, s));
                FMS_HIP(hipMemcpyAsync(mirror, ctl, offsetof(Ctl, conv_it), hipMemcpyDeviceToHost, s));
                FMS_HIP(wait_stream(s));
                pool_len = mirror->pool_len;
                cur ^= 1;   // undone below: the pool is back in pool[cur]
            }
        }

        if (diag) {
            if (rounds < MS_DIAG_MAX_ROUNDS) {
                diag->round_N[rounds] = all ? B : (int32_t)std::min<long long>(N, INT_MAX);
                diag->round_B[rounds] = B;
                diag->round_M[rounds] = K;
                diag->round_T[rounds] = cs.iters_run;
                int conv = 0;
                for (int u = 0; u < cs.iters_run; ++u) conv += cs.conv_it[u];
                diag->round_converged[rounds] = conv;
            }
            for (int i = 0; i < B; ++i) {
                const long long o = drawn_total + i;
                if (diag->drawn) diag->drawn[o] = h_ids[i];
                if (diag->drawn_iters) diag->drawn_iters[o] = h_iters[i];
                if (diag->drawn_status)
                    diag->drawn_status[o] = h_status[i] == ST_CONVERGED ? 1 : (h_status[i] == ST_FAILED ? 2 : 0);
                if (diag->drawn_final)
                    for (int k = 0; k < d; ++k) diag->drawn_final[o * d + k] = h_S[(size_t)i * DP + k];
            }
        }
        drawn_total += B;
        rounds += 1;
        merge_ms += ms_since(t_merge);
        if (all) break;
        cur ^= 1;
        if (trace)
            std::fprintf(stderr, "[fms] round %d B=%d T=%d K=%d pool=%d%s round %.3f ms (merge+pool %.3f)\n",
                         rounds, B, cs.iters_run, K, pool_len, host_merge ? " (host merge)" : "",
                         ms_since(t_round), ms_since(t_merge));
        if (pool_len == 0 || N >= (long long)p->L * K) break;
        N *= 2;
    }

    *k_out = K;
    if (diag) {
        diag->rounds = rounds;
        diag->pairs = pairs;
        diag->refined_pairs = refined;
        diag->iterate_ms = iterate_ms;
        diag->merge_ms = merge_ms;
        if (diag->counts)
            for (int j = 0; j < std::min(K, max_modes); ++j) diag->counts[j] = counts[j];
    }
    if (K == 0) return fail(MS_E_NO_MODES, "no seed converged");
    if (K > max_modes) return fail(MS_E_CAPACITY, "more modes than max_modes (k_out holds the required K)");

    FMS_HIP(hipMemcpy2DAsync(modes, (size_t)d * 4, modes_ws, (size_t)DP * 4, (size_t)d * 4, K,
                             hipMemcpyDeviceToDevice, s));
    if (labels) {
        FMS_HIP(hipEventRecord(ev[2], s));
        if (join_ok && K >= kJoinMin && n >= kJoinMin) {
            // many modes: nearest mode by the block join (the same distances
            // and ties as the brute-force labelling)
            char* w;
            JoinIndex jm{};
            FMS_CHECK(points_index());
            FMS_CHECK(cache_get(C, budget, SL_JMODES, join_layout(K, DP, base.D).total, &w));
            FMS_HIP(launch_join_index(modes_ws, K, DP, d, DP, base.D, scale, w, &jm, s));
            int32_t* dcand = nullptr;
            if (!cand.empty()) {
                FMS_CHECK(cache_get(C, budget, SL_CAND, n, &dcand));
                FMS_CHECK(g_pin_pos.ensure((size_t)n * sizeof(int32_t)));
                std::memcpy(g_pin_pos.p, cand.data(), (size_t)n * sizeof(int32_t));
                FMS_HIP(hipMemcpyAsync(dcand, g_pin_pos.p, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s));
            }
            FMS_HIP(launch_join(JOIN_NEAREST, jpts, jm, DP, base.D, 0.0f, labels, nullptr, nullptr, nullptr,
                                nullptr, nullptr, 0, nullptr, s, 0, false, nullptr, dcand, modes_ws));
        } else {
            FMS_HIP(launch_assign(X, n, d, modes, K, labels, nullptr, s));
        }
        FMS_HIP(hipEventRecord(ev[3], s));
    }
    FMS_HIP(wait_stream(s));
    if (diag) {
        float ms = 0.0f;
        if (labels) FMS_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
        diag->assign_ms = ms;
        diag->workspace_bytes = C.held;
        diag->total_ms = ms_since(t_start);
    }
    if (trace) std::fprintf(stderr, "[fms] fit done K=%d total %.3f ms\n", K, ms_since(t_start));
    return MS_OK;
}

// Bump allocation out of one device buffer of fixed size, with no allocation
// call: every request is rounded up to 256 bytes.  With a NULL base it only
// counts, so that a dry run can size a call before anything is launched.
class Arena {
   public:
    Arena(char* base, size_t cap) : base_(base), cap_(cap) {}
    template <typename T>
    int alloc(T** out, size_t count) {
        const size_t bytes = (std::max<size_t>(count * sizeof(T), 256) + 255) / 256 * 256;
        if (base_ && (off_ > cap_ || bytes > cap_ - off_))
            return fail(MS_E_INVALID, "scratch buffer too small for this call");
        *out = base_ ? (T*)(base_ + off_) : nullptr;
        off_ += bytes;
        return MS_OK;
    }
    size_t used() const { return off_; }

   private:
    char* base_;
    size_t cap_;
    size_t off_ = 0;
};

// The body of ms_step over device buffers taken from `ws` (a Workspace or an
// Arena).  With run = false only the buffers are requested (nothing is
// launched): the dry run that sizes an Arena.
template <class A>
int step_core(A& ws, bool run, const ms_params* p, const float* X, int n, int d, float* seeds, int m,
              int n_iter, uint8_t* converged, int32_t* iters, float* shift2, hipStream_t s) {
#define FMS_RUN(expr)                   \
    do {                                \
        if (run) FMS_HIP(expr);         \
    } while (0)
    const bool bf16 = bf16_form(p, d);
    const bool cull = !bf16 && !p->plain && cull_supported(d, n) &&
                      !(p->metric == MS_METRIC_COSINE && cull_reach(p->kernel, p->h) >= 2.0);
    const bool sorted = bf16 || cull;
    const StepShape sh = bf16 ? step_shape_bf16(d, m)
                              : (cull ? step_shape_cull(d, m, n) : step_shape_for(d, m));
    const float scale = packed_scale(p);
    if (p->metric == MS_METRIC_COSINE) {
        // the directions of the rows (a row of length 0 gives NaN directions,
        // and every seed that sees it fails)
        float* Xn;
        FMS_CHECK(ws.alloc(&Xn, (size_t)n * d));
        FMS_RUN(launch_normalize_rows(X, n, d, Xn, nullptr, s));
        X = Xn;
    }
    float* Xp;
    FMS_CHECK(ws.alloc(&Xp, (size_t)n * sh.DP));
    FMS_RUN(launch_pack_points(X, n, d, sh.DP, scale, Xp, s));
    SortedPoints sp;
    if (sorted) {
        char* sws;
        FMS_CHECK(ws.alloc(&sp.Xs, (size_t)n * sh.DP));
        FMS_CHECK(ws.alloc(&sp.perm, n));
        FMS_CHECK(ws.alloc(&sp.geom, (size_t)((n + 255) / 256) * geom_stride(sh.D)));
        FMS_CHECK(ws.alloc(&sws, sort_workspace_bytes(n > m ? n : m)));
        sp.sws = sws;
        FMS_RUN(launch_spatial_sort(Xp, n, sh.DP, sh.D, sp.Xs, sp.perm, sp.geom, sws, s));
    }
    if (bf16) {
        FMS_CHECK(ws.alloc(&sp.feat, sh.D <= 4 ? bf16_feature_bytes(n)
                                               : bf16_wide_feature_bytes(n, sh.D, p->kernel)));
        if (sh.D <= 4) FMS_RUN(launch_bf16_features(sp.Xs, n, d, sp.geom, sp.feat, s));
        else FMS_RUN(launch_bf16_wide_features(sp.Xs, n, sh.D, sp.geom, sp.feat, p->kernel, s));
    }
    Ctl* ctl;
    FMS_CHECK(ws.alloc(&ctl, 1));
    Batch b;
    fill_batch(b, n, d, m, sh, p, scale, Xp, ctl, sorted ? &sp : nullptr);
    FMS_CHECK(ws.alloc(&b.S, (size_t)m * sh.DP));
    FMS_CHECK(ws.alloc(&b.act[0], m));
    FMS_CHECK(ws.alloc(&b.act[1], m));
    FMS_CHECK(ws.alloc(&b.status, m));
    FMS_CHECK(ws.alloc(&b.iters, m));
    FMS_CHECK(ws.alloc(&b.shift2, m));
    FMS_CHECK(ws.alloc(&b.part, (size_t)step_part_floats(sh, m, b.grid)));
    if (!run) return MS_OK;
    FMS_HIP(launch_ctl_reset(ctl, 0, INT_MAX, n_iter, s));
    FMS_HIP(launch_seed_init_from_array(seeds, converged, d, m, b, s));
    if (sorted)   // seeds that are close in space share waves (refine work, culled blocks)
        FMS_HIP(launch_seed_order(b.S, sh.DP, sh.D, m, scale, b.status, sp.sws, b.act[0], Xp, n, s));
    for (int t = 0; t < n_iter; ++t) FMS_HIP(launch_iteration(b, t, s));
    FMS_HIP(launch_seed_export(b, m, seeds, converged, iters, shift2, s));
    return MS_OK;
#undef FMS_RUN
}

int step_impl(const ms_params* p, const float* X, int n, int d, float* seeds, int m, int n_iter,
              uint8_t* converged, int32_t* iters, float* shift2, hipStream_t s) {
    FMS_CHECK(ensure_pool_release_threshold());
    Workspace ws(s);
    return step_core(ws, true, p, X, n, d, seeds, m, n_iter, converged, iters, shift2, s);
}

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
int scratch_base(char** out) {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static char* base[kMaxDev] = {};
    int dev = 0;
    FMS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(MS_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!base[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(MS_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        base[dev] = (char*)ptr;
    }
    *out = base[dev];
    return MS_OK;
}

// ms_step with every buffer in the fixed device scratch: a dry run sizes the
// call, a call that needs more than the scratch holds is rejected before
// anything is launched, and the kernels are those of ms_step.
int step_noalloc_impl(const ms_params* p, const float* X, int n, int d, float* seeds, int m, int n_iter,
                      uint8_t* converged, int32_t* iters, float* shift2, hipStream_t s) {
    Arena need(nullptr, 0);
    FMS_CHECK(step_core(need, false, p, X, n, d, seeds, m, n_iter, converged, iters, shift2, s));
    if (need.used() > kScratchBytes)
        return fail(MS_E_INVALID, "ms_step_noalloc: this call needs " + std::to_string(need.used()) +
                                      " bytes of device scratch, more than the fixed " +
                                      std::to_string(kScratchBytes));
    char* base = nullptr;
    FMS_CHECK(scratch_base(&base));
    Arena ws(base, kScratchBytes);
    return step_core(ws, true, p, X, n, d, seeds, m, n_iter, converged, iters, shift2, s);
}

// Seeds per lane that the batched step is built for, by padded dimension.
bool batched_R_ok(int D, int R) {
    if (R == 1) return true;
    if (R == 2) return D <= 16;
    if (R == 4) return D <= 4;
    return false;
}

// Tuned launch shape (seeds per lane, points per chunk, step grid), by input
// kind (padded dimension, floor(log2) of the mean points and of the mean
// seeds per cloud), for the whole process.
using TuneKey = std::tuple<int, int, int, int>;
struct TuneShape {
    int R, chunk, grid;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneShape> g_tune;
constexpr int kBatchedChunk = 1024;   // points per chunk unless set or tuned
constexpr int kBatchedGrid = 2048;    // workgroups of the step unless set or tuned

int ilog2_ll(long long v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

TuneKey tune_key(int d, long long n, long long M, int ncl, int precision) {
    return TuneKey(step_shape(d).D, ilog2_ll(std::max(1LL, n / ncl)), ilog2_ll(std::max(1LL, M / ncl)), precision);
}

// R_force = 0: the tuned shape for this kind of input, else seeds per lane
// from the mean seeds per cloud (small clouds waste fewer lanes).  With
// ev != NULL the iterations are bracketed by ev[0] and ev[1].
// Points of a batch already packed (DP columns, packed units of the call's
// parameters) with the point and seed offsets on the device: a caller that
// runs several step calls over the same clouds packs them once.
struct BatchedBf16;
struct BatchedPrepared {
    const float* Xp;
    int DP;
    const long long* xo_dev;
    const int32_t* so_dev;
    DevCache* cache;          // the calling fit's cache for the step's buffers (kept across calls), or NULL
    const BatchedBf16* bb;    // the BF16 form: the points' order and features (prepared once), else NULL
};

// The BF16 form over many clouds (Gaussian, padded D in {8, 16, 32}): each
// cloud's points in the spatial order of the one-cloud form (its own pivots),
// their block features, and the per-cloud offsets the kernels use.  The
// point part depends on the clouds only; the seed part (stpre, soff,
// stiles) on each call's seed offsets.
struct BatchedBf16 {
    float* Xs = nullptr;
    void* feat = nullptr;
    void* sws = nullptr;
    int32_t* poff = nullptr;     // pivots before each cloud
    int32_t* boff = nullptr;     // 256-point blocks before each cloud
    int32_t* stpre = nullptr;    // 256-seed tiles before each cloud
    long long* soff = nullptr;   // seed offsets (64-bit, for the seed order)
    float* zero = nullptr;       // frame of the sorted points (no shift)
    int ptot = 0, nblk = 0, stiles = 0, count = 0;
};

bool batched_bf16_ok(const ms_params* p, int d) {
    const int D = step_shape(d).D;
    return p->kernel == MS_KERNEL_GAUSSIAN && (D == 8 || D == 16 || D == 32);
}

// Sorts the packed points Xp of the clouds and builds their features (the
// workspace comes from ws); the offsets are xo (host) and xo_dev.  count
// sizes the sort workspace: at least the points and every later call's seeds.
int prepare_batched_bf16_points(Workspace& ws, const float* Xp, int n, int D, const std::vector<long long>& xo,
                                const long long* xo_dev, int ncl, int count, BatchedBf16& bb, hipStream_t s) {
    std::vector<int32_t> poff(ncl + 1, 0), boff(ncl + 1, 0);
    for (int c = 0; c < ncl; ++c) {
        const long long nc = xo[c + 1] - xo[c];
        poff[c + 1] = poff[c] + batched_pivot_count(nc);
        boff[c + 1] = boff[c] + (int)((nc + 255) / 256);
    }
    bb.ptot = poff[ncl];
    bb.nblk = boff[ncl];
    bb.count = std::max(std::max(n, count), 1);
    FMS_CHECK(ws.alloc(&bb.poff, (size_t)ncl + 1));
    FMS_CHECK(ws.alloc(&bb.boff, (size_t)ncl + 1));
    FMS_CHECK(ws.alloc(&bb.zero, (size_t)D));
    FMS_CHECK(ws.alloc(&bb.Xs, (size_t)std::max(n, 1) * D));
    char* feat;
    FMS_CHECK(ws.alloc(&feat, bf16f_feature_bytes_blocks(std::max(bb.nblk, 1), D)));
    bb.feat = feat;
    char* sws;
    FMS_CHECK(ws.alloc(&sws, batched_sort_workspace_bytes(bb.count, bb.ptot)));
    bb.sws = sws;
    const size_t ob = (size_t)(ncl + 1) * sizeof(int32_t);
    FMS_HIP(hipMemcpyAsync(bb.poff, poff.data(), ob, hipMemcpyHostToDevice, s));
    FMS_HIP(hipMemcpyAsync(bb.boff, boff.data(), ob, hipMemcpyHostToDevice, s));
    FMS_HIP(hipMemsetAsync(bb.zero, 0, (size_t)D * 4, s));
    FMS_HIP(hipStreamSynchronize(s));   // the host copies go out of scope
    const CloudRows pts{ncl, xo_dev, bb.boff, bb.nblk};
    FMS_HIP(launch_batched_sort(Xp, n, D, pts, bb.poff, bb.ptot, bb.Xs, bb.sws, bb.count, s));
    FMS_HIP(launch_bf16f_features_batched(bb.Xs, D, xo_dev, bb.boff, ncl, bb.nblk, bb.feat, s));
    return MS_OK;
}

// The seed part of bb for the seed offsets so (host), from ws.
int prepare_batched_bf16_seeds(Workspace& ws, const std::vector<int32_t>& so, int ncl, BatchedBf16& bb,
                               hipStream_t s) {
    std::vector<int32_t> stpre(ncl + 1, 0);
    std::vector<long long> soff(ncl + 1, 0);
    for (int c = 0; c < ncl; ++c) {
        stpre[c + 1] = stpre[c] + (so[c + 1] - so[c] + 255) / 256;
        soff[c + 1] = so[c + 1];
    }
    if (so[ncl] > bb.count) return fail(MS_E_HIP, "more seeds than the prepared sort workspace holds");
    bb.stiles = stpre[ncl];
    FMS_CHECK(ws.alloc(&bb.stpre, (size_t)ncl + 1));
    FMS_CHECK(ws.alloc(&bb.soff, (size_t)ncl + 1));
    FMS_HIP(hipMemcpyAsync(bb.stpre, stpre.data(), (size_t)(ncl + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    FMS_HIP(hipMemcpyAsync(bb.soff, soff.data(), (size_t)(ncl + 1) * sizeof(long long), hipMemcpyHostToDevice, s));
    FMS_HIP(hipStreamSynchronize(s));   // the host copies go out of scope
    return MS_OK;
}

int step_batched_impl(const ms_params* p, const float* X, const int64_t* x_off, float* seeds,
                      const int64_t* s_off, int ncl, int d, int n_iter, uint8_t* converged,
                      int32_t* iters, float* shift2, hipStream_t s, int R_force = 0,
                      hipEvent_t* ev = nullptr, const BatchedPrepared* pre = nullptr) {
    FMS_CHECK(ensure_pool_release_threshold());
    const int n = (int)x_off[ncl];
    const int M = (int)s_off[ncl];
    const bool bf = p->precision == MS_PREC_BF16_REFINE;
    if (bf && !batched_bf16_ok(p, d))
        return fail(MS_E_INVALID, "the batched BF16 form is built for the Gaussian kernel at 5 <= d <= 32");
    if (bf && pre && !pre->bb) return fail(MS_E_HIP, "the batched BF16 form needs its prepared points");
    StepShape sh = step_shape_for(d, std::max(1, M / ncl));
    // default: at most two seeds per lane up to D = 8 and one above (timed on
    // 512 uneven clouds: more seeds per lane cost occupancy here, and the
    // work queue already balances the items)
    const int r_cap = sh.D <= 8 ? 2 : 1;
    if (sh.R > r_cap) {
        sh.R = r_cap;
        sh.TS = 64 * r_cap;
    }
    int R = R_force;
    int chunk = p->tile_chunk, grid_cap = p->tile_grid;
    if (R == 0 || chunk == 0 || grid_cap == 0) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune.find(tune_key(d, n, M, ncl, p->precision));
        if (it != g_tune.end()) {
            if (R == 0) R = it->second.R;
            if (chunk == 0) chunk = it->second.chunk;
            if (grid_cap == 0) grid_cap = it->second.grid;
        }
    }
    if (chunk == 0) chunk = kBatchedChunk;
    if (grid_cap == 0) grid_cap = kBatchedGrid;
    if (bf) {
        // seed tiles of 128 (the finalize's two slots per lane), chunks of
        // whole 256-point blocks
        sh.R = 2;
        sh.TS = kBf16fTile;
        chunk = (chunk + 255) / 256 * 256;
    } else if (R != 0) {
        if (!batched_R_ok(sh.D, R)) return fail(MS_E_INVALID, "tile_R is not built for this dimension");
        sh.R = R;
        sh.TS = 64 * R;
    }
    const float scale = packed_scale(p);
    std::vector<long long> xo(ncl + 1);
    std::vector<int32_t> so(ncl + 1);
    for (int c = 0; c <= ncl; ++c) {
        xo[c] = x_off[c];
        so[c] = (int32_t)s_off[c];
    }
    const long long max_items = batched_max_items(xo.data(), so.data(), ncl, sh.TS, chunk);
    if (max_items > INT_MAX / 2) return fail(MS_E_INVALID, "too many work items for one batch");
    Workspace ws(s);
    const float* Xp;
    const long long* xo_dev;
    const int32_t* so_dev;
    if (pre) {
        if (pre->DP != sh.DP) return fail(MS_E_HIP, "prepared points have another row width");
        Xp = pre->Xp;
        xo_dev = pre->xo_dev;
        so_dev = pre->so_dev;
    } else {
        float* xp;
        long long* xod;
        int32_t* sod;
        FMS_CHECK(ws.alloc(&xp, (size_t)n * sh.DP));
        FMS_HIP(launch_pack_points(X, n, d, sh.DP, scale, xp, s));
        FMS_CHECK(ws.alloc(&xod, (size_t)ncl + 1));
        FMS_CHECK(ws.alloc(&sod, (size_t)ncl + 1));
        FMS_HIP(hipMemcpyAsync(xod, xo.data(), (size_t)(ncl + 1) * sizeof(long long), hipMemcpyHostToDevice, s));
        FMS_HIP(hipMemcpyAsync(sod, so.data(), (size_t)(ncl + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
        FMS_HIP(hipStreamSynchronize(s));   // the host copies of the offsets go out of scope
        Xp = xp;
        xo_dev = xod;
        so_dev = sod;
    }
    BatchedBf16 bb;
    if (bf) {
        if (pre) bb = *pre->bb;
        else FMS_CHECK(prepare_batched_bf16_points(ws, Xp, n, sh.D, xo, xo_dev, ncl, M, bb, s));
        FMS_CHECK(prepare_batched_bf16_seeds(ws, so, ncl, bb, s));
    }
    Batch b;
    fill_batch(b, n, d, M, sh, p, scale, Xp, nullptr);
    b.grid = (int)std::min<long long>(INT_MAX, std::max(1LL, max_items));   // capped by the launcher
    b.chunk_points = chunk;
    b.grid_cap = grid_cap;
    if (bf) {
        b.Xs = bb.Xs;
        b.pf = bb.feat;
        b.feat_blocks = bb.nblk;
        b.boff = bb.boff;
        b.shift = bb.zero;
    }
    // the step's buffers: from the calling fit's cache (kept from one step
    // call of the fit to the next), else stream-ordered for this call
    AllocBudget budget;
    DevCache* cache = pre ? pre->cache : nullptr;
    auto get = [&](auto** out, size_t count, Slot sl) {
        return cache ? cache_get(*cache, budget, sl, count, out) : ws.alloc(out, count);
    };
    FMS_CHECK(get(&b.S, (size_t)M * sh.DP, SL_BSTEP_S));
    FMS_CHECK(get(&b.act[0], (size_t)M, SL_BSTEP_ACT0));
    FMS_CHECK(get(&b.act[1], (size_t)M, SL_BSTEP_ACT1));
    FMS_CHECK(get(&b.status, (size_t)M, SL_BSTEP_STATUS));
    FMS_CHECK(get(&b.iters, (size_t)M, SL_BSTEP_ITERS));
    FMS_CHECK(get(&b.shift2, (size_t)M, SL_BSTEP_SHIFT2));
    int32_t *cnt, *plan, *item_cloud, *slot_cloud;
    FMS_CHECK(get(&cnt, (size_t)2 * ncl, SL_BSTEP_CNT));
    FMS_CHECK(get(&plan, (size_t)4 * ncl + 3, SL_BSTEP_PLAN));   // + the work-item queue head
    FMS_CHECK(get(&item_cloud, (size_t)std::max(1LL, max_items), SL_BSTEP_ITEMC));
    FMS_CHECK(get(&slot_cloud, (size_t)M, SL_BSTEP_SLOTC));
    FMS_CHECK(get(&b.part, (size_t)std::max(1LL, max_items) * sh.TS * (sh.D + 1), SL_BSTEP_PART));
    FMS_HIP(launch_batched_init(seeds, converged, d, M, so_dev, ncl, cnt, b, s));
    if (bf) {
        // each cloud's active list in the spatial order of its seeds
        const CloudRows pts{ncl, xo_dev, bb.boff, bb.nblk};
        const CloudRows sds{ncl, bb.soff, bb.stpre, bb.stiles};
        FMS_HIP(launch_batched_seed_order(b.S, sh.DP, sh.D, M, scale, b.status, sds, Xp, pts, bb.poff, bb.sws,
                                          bb.count, bb.ptot, b.act[0], s));
    }
    if (ev) FMS_HIP(hipEventRecord(ev[0], s));
    if (p->graph && n_iter > 0) {
        // every iteration captured on a private stream (capture is not allowed
        // on the null stream), then one graph launch on the caller's stream.
        // The executable graph is kept (per host thread and device) and
        // updated in place when a later call captures the same topology, so
        // that it is instantiated once per shape.
        int dev = 0;
        FMS_HIP(hipGetDevice(&dev));
        GraphCache& gc = g_graph;
        if (gc.dev != dev) gc.clear();
        gc.dev = dev;
        if (!gc.cs) FMS_HIP(hipStreamCreateWithFlags(&gc.cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(gc.cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int t = 0; t < n_iter && e == hipSuccess; ++t)
                e = launch_batched_iteration(b, xo_dev, so_dev, ncl, cnt, plan, item_cloud, slot_cloud, t, gc.cs);
            const hipError_t e2 = hipStreamEndCapture(gc.cs, &g);
            if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess && gc.ge) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            const hipError_t eu = hipGraphExecUpdate(gc.ge, g, &bad, &res);
            if (eu != hipSuccess || res != hipGraphExecUpdateSuccess) {
                (void)hipGetLastError();   // another topology: instantiate anew
                (void)hipGraphExecDestroy(gc.ge);
                gc.ge = nullptr;
            } else {
                gc.updates += 1;
            }
        }
        if (e == hipSuccess && !gc.ge) {
            e = hipGraphInstantiate(&gc.ge, g, nullptr, nullptr, 0);
            if (e == hipSuccess) gc.instantiations += 1;
            else gc.ge = nullptr;
        }
        if (e == hipSuccess) e = hipGraphLaunch(gc.ge, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // the workspace outlives the launch
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "batched iterations as a graph");
    } else {
        for (int t = 0; t < n_iter; ++t)
            FMS_HIP(launch_batched_iteration(b, xo_dev, so_dev, ncl, cnt, plan, item_cloud, slot_cloud, t, s));
    }
    if (ev) FMS_HIP(hipEventRecord(ev[1], s));
    FMS_HIP(launch_seed_export(b, M, seeds, converged, iters, shift2, s));
    return MS_OK;
}

// Runs f(c) for every cloud c, on up to 16 host threads when the round has
// enough work (clouds are taken from a shared counter; each cloud's work is
// sequential, so the results do not depend on the thread count).  If a thread
// cannot be started the ones running finish the clouds.
template <class F>
void for_each_cloud(int ncl, long long work, F&& f) {
    const unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1u, 16u);
    nt = std::min(nt, ncl);
    if (work < (1LL << 14) || nt <= 1) {
        for (int c = 0; c < ncl; ++c) f(c);
        return;
    }
    std::atomic<int> next{0};
    auto worker = [&]() {
        for (int c = next.fetch_add(1); c < ncl; c = next.fetch_add(1)) f(c);
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nt; ++i) {
        try {
            th.emplace_back(worker);
        } catch (...) {
            break;
        }
    }
    worker();
    for (auto& t : th) t.join();
}

// Host staging of ms_fit_batched, sized by each round's seeds and modes
// (grown on demand, kept for the thread).
thread_local Pinned g_pin_bpos, g_pin_bso, g_pin_bso32, g_pin_bconv, g_pin_bmoff, g_pin_blen, g_pin_bk;

// The whole method (Algorithm 2 with the seed pool of Section II-D; with
// all_points_as_seeds, Algorithm 1) for every cloud of a CSR batch, the
// clouds' rounds advancing together: per round, the host draws each active
// cloud's seeds from its pool (SplitMix64 state rng_seed + c for cloud c),
// the device gathers them and runs the batched fused step for all clouds
// until every seed of the round converged, failed or max_iter updates were
// made; the device merges each cloud's converged seeds into that cloud's
// modes in draw order (first mode within merge_radius h, else a new mode;
// decision passes until none is undecided, the modes kept per cloud at the
// cloud's own rows of a mode store), removes covered points from each pool
// and compacts the pools, and the host applies each cloud's seed-count rule
// (stop when its pool is empty or N >= L M, else N <- 2N) from the mode
// counts it reads back.  Labels: nearest mode within the cloud.
int fit_batched_impl(const ms_params* p, const float* X, const int64_t* x_off, int ncl, int d, float* modes,
                     int64_t max_modes, int64_t* k_off, int32_t* labels, int32_t* rounds_out, hipStream_t s) {
    const auto t_start = std::chrono::steady_clock::now();
    free_orphans();
    FMS_CHECK(ensure_pool_release_threshold());
    const long long n = x_off[ncl];
    const bool all = p->all_points_as_seeds != 0;
    const float rm = p->merge_radius * p->h, rc = p->cover_radius * p->h;
    const float r2m = rm * rm, r2c = rc * rc;
    Workspace ws(s);
    long long* xo_dev;
    long long* so_dev;
    int32_t *pool[2], *pos_dev, *plen_dev, *moff_dev, *it_dev;
    uint8_t *removed, *conv_dev;
    float *S_dev, *sh2_dev, *nm_dev;
    // the point-sized buffers come from this thread's cache (kept across
    // calls); the small per-cloud ones are stream-ordered
    int dev = 0;
    FMS_HIP(hipGetDevice(&dev));
    DevCache& C = cache_for_device(dev);
    AllocBudget budget;
    FMS_CHECK(ws.alloc(&xo_dev, (size_t)ncl + 1));
    FMS_CHECK(ws.alloc(&so_dev, (size_t)ncl + 1));
    FMS_CHECK(cache_get(C, budget, SL_POOL0, (size_t)n, &pool[0]));
    FMS_CHECK(cache_get(C, budget, SL_POOL1, (size_t)n, &pool[1]));
    FMS_CHECK(cache_get(C, budget, SL_POS, (size_t)n, &pos_dev));
    FMS_CHECK(ws.alloc(&plen_dev, (size_t)ncl));
    FMS_CHECK(ws.alloc(&moff_dev, (size_t)ncl + 1));
    FMS_CHECK(cache_get(C, budget, SL_REMOVED, (size_t)n, &removed));
    FMS_CHECK(cache_get(C, budget, SL_BCONV, (size_t)n, &conv_dev));
    FMS_CHECK(cache_get(C, budget, SL_BITERS, (size_t)n, &it_dev));
    FMS_CHECK(cache_get(C, budget, SL_BS, (size_t)n * d, &S_dev));
    FMS_CHECK(cache_get(C, budget, SL_BSH2, (size_t)n, &sh2_dev));
    FMS_CHECK(cache_get(C, budget, SL_BNM, (size_t)n * d, &nm_dev));   // the mode store
    int32_t *state_dev, *kcnt_dev, *kold_dev, *und_dev;
    FMS_CHECK(cache_get(C, budget, SL_BSTATE, (size_t)n, &state_dev));
    FMS_CHECK(ws.alloc(&kcnt_dev, (size_t)ncl));
    FMS_CHECK(ws.alloc(&kold_dev, (size_t)ncl));
    FMS_CHECK(ws.alloc(&und_dev, (size_t)1));
    FMS_CHECK(g_pin_bso.ensure((size_t)(ncl + 1) * 8));
    FMS_CHECK(g_pin_bso32.ensure((size_t)(ncl + 1) * 4));
    FMS_CHECK(g_pin_bmoff.ensure((size_t)(ncl + 1) * 4));
    FMS_CHECK(g_pin_blen.ensure((size_t)ncl * 4));
    FMS_CHECK(g_pin_bk.ensure((size_t)(ncl + 1) * 4));
    int64_t* hso = (int64_t*)g_pin_bso.p;
    int32_t* hso32 = (int32_t*)g_pin_bso32.p;
    int32_t* hmoff = (int32_t*)g_pin_bmoff.p;
    int32_t* hlen = (int32_t*)g_pin_blen.p;
    int32_t* hk = (int32_t*)g_pin_bk.p;   // [0, ncl): modes per cloud; [ncl]: undecided seeds

    std::vector<long long> xo(x_off, x_off + ncl + 1);
    FMS_HIP(hipMemcpyAsync(xo_dev, xo.data(), (size_t)(ncl + 1) * 8, hipMemcpyHostToDevice, s));
    // the points packed once for every step call of the fit
    ms_params q = *p;
    q.graph = 0;
    q.tile_R = 0;
    const int DP = step_shape(d).DP;
    float* Xp;
    int32_t* so32_dev;
    FMS_CHECK(cache_get(C, budget, SL_XP, (size_t)n * DP, &Xp));
    FMS_CHECK(ws.alloc(&so32_dev, (size_t)ncl + 1));
    FMS_HIP(launch_pack_points(X, (int)n, d, DP, packed_scale(&q), Xp, s));
    // the BF16 form: the clouds' spatial order and block features, once per
    // call (a round's seeds are never more than the points)
    BatchedBf16 bb;
    const bool bf = p->precision == MS_PREC_BF16_REFINE;
    if (bf) FMS_CHECK(prepare_batched_bf16_points(ws, Xp, (int)n, step_shape(d).D, xo, xo_dev, ncl, (int)n, bb, s));
    const BatchedPrepared pre{Xp, DP, xo_dev, so32_dev, &C, bf ? &bb : nullptr};
    FMS_HIP(launch_bf_iota(xo_dev, ncl, pool[0], n, s));
    FMS_HIP(launch_bf_fill_i32(kcnt_dev, ncl, 0, s));
    FMS_HIP(launch_fill_u8(removed, (int)n, 0, s));
    std::vector<uint64_t> rng(ncl);
    std::vector<long long> N(ncl, p->n_initial);
    std::vector<int32_t> plen(ncl);
    std::vector<char> active(ncl);
    for (int c = 0; c < ncl; ++c) {
        rng[c] = p->rng_seed + (uint64_t)c;
        plen[c] = (int32_t)(x_off[c + 1] - x_off[c]);
        active[c] = plen[c] > 0;
        hlen[c] = plen[c];
    }
    FMS_HIP(hipMemcpyAsync(plen_dev, hlen, (size_t)ncl * 4, hipMemcpyHostToDevice, s));
    // iterations between checks for a finished round (an iteration with no
    // active seed is a few microseconds of empty launches)
    constexpr int kChunk = 8;
    int cur = 0, rounds = 0;
    const bool trace = log_enabled();
    if (trace) {
        FMS_HIP(wait_stream(s));
        std::fprintf(stderr, "[fms] fit_batched %d clouds, %lld points: setup %.3f ms\n", ncl, n, ms_since(t_start));
    }
    for (;;) {
        const auto t_round = std::chrono::steady_clock::now();
        double t_draw = 0.0, t_iter = 0.0, t_merge = 0.0;
        int iters_run = 0;
        // draws (the staging buffers hold no copy in flight: every round ends
        // with a wait on the stream)
        int64_t M = 0;
        hso[0] = 0;
        for (int c = 0; c < ncl; ++c) {
            if (active[c]) M += all ? plen[c] : (int32_t)std::min<long long>(N[c], plen[c]);
            hso[c + 1] = M;
        }
        if (M == 0) break;
        FMS_CHECK(g_pin_bpos.ensure((size_t)M * 4));
        FMS_CHECK(g_pin_bconv.ensure((size_t)M));
        int32_t* hpos = (int32_t*)g_pin_bpos.p;
        uint8_t* hconv = (uint8_t*)g_pin_bconv.p;
        for_each_cloud(ncl, M, [&](int c) {
            const int32_t B = (int32_t)(hso[c + 1] - hso[c]);
            if (B == 0) return;
            if (all)
                for (int32_t t = 0; t < B; ++t) hpos[hso[c] + t] = t;
            else
                draw_positions(&rng[c], plen[c], B, hpos + hso[c]);
        });
        FMS_HIP(hipMemcpyAsync(pos_dev, hpos, (size_t)M * 4, hipMemcpyHostToDevice, s));
        FMS_HIP(hipMemcpyAsync(so_dev, hso, (size_t)(ncl + 1) * 8, hipMemcpyHostToDevice, s));
        for (int c = 0; c <= ncl; ++c) hso32[c] = (int32_t)hso[c];
        FMS_HIP(hipMemcpyAsync(so32_dev, hso32, (size_t)(ncl + 1) * 4, hipMemcpyHostToDevice, s));
        FMS_HIP(launch_bf_gather(X, d, xo_dev, so_dev, ncl, pos_dev, pool[cur], removed, S_dev, (int)M, s));
        FMS_HIP(launch_fill_u8(conv_dev, (int)M, 0, s));
        t_draw = ms_since(t_round);
        // iterations until the round is over for every seed
        for (int done = 0; done < p->max_iter;) {
            const int k = std::min(kChunk, p->max_iter - done);
            FMS_CHECK(step_batched_impl(&q, X, x_off, S_dev, hso, ncl, d, k, conv_dev, it_dev, sh2_dev, s, 0,
                                        nullptr, &pre));
            done += k;
            iters_run = done;
            FMS_HIP(hipMemcpyAsync(hconv, conv_dev, (size_t)M, hipMemcpyDeviceToHost, s));
            FMS_HIP(wait_stream(s));
            bool open = false;
            for (long long g = 0; g < M && !open; ++g) open = hconv[g] == ST_ACTIVE;
            if (!open) break;
        }
        t_iter = ms_since(t_round) - t_draw;
        rounds += 1;
        // merge on the device, cloud by cloud in draw order: decision passes
        // until no seed is undecided (each pass settles at least the first
        // undecided seed of each cloud), then the founders become modes
        FMS_HIP(launch_bf_merge_init(state_dev, (int)M, s));
        int passes = 0;
        for (;;) {
            FMS_HIP(launch_bf_decide_pass(S_dev, d, conv_dev, so_dev, ncl, nm_dev, xo_dev, kcnt_dev, r2m, state_dev,
                                          und_dev, (int)M, passes == 0, s));
            ++passes;
            FMS_HIP(hipMemcpyAsync(hk + ncl, und_dev, 4, hipMemcpyDeviceToHost, s));
            FMS_HIP(wait_stream(s));
            if (hk[ncl] == 0) break;
        }
        FMS_HIP(launch_bf_founders(S_dev, d, so_dev, ncl, state_dev, xo_dev, nm_dev, kcnt_dev, kold_dev, s));
        t_merge = ms_since(t_round) - t_draw - t_iter;
        if (trace)
            std::fprintf(stderr, "[fms] fit_batched round %d: %lld seeds, %d iterations, %d merge passes; draws "
                                 "%.3f, iterations %.3f, merge %.3f ms\n",
                         rounds, (long long)M, iters_run, passes, t_draw, t_iter, t_merge);
        if (all) {
            FMS_HIP(hipMemcpyAsync(hk, kcnt_dev, (size_t)ncl * 4, hipMemcpyDeviceToHost, s));
            FMS_HIP(wait_stream(s));
            break;
        }
        // pools: coverage by the new modes, compaction, seed-count control
        FMS_HIP(launch_bf_cover(X, d, xo_dev, ncl, pool[cur], plen_dev, nm_dev, kold_dev, kcnt_dev, r2c, removed, n,
                                s));
        FMS_HIP(launch_bf_compact(xo_dev, ncl, pool[cur], removed, plen_dev, pool[cur ^ 1], s));
        cur ^= 1;
        FMS_HIP(hipMemcpyAsync(hlen, plen_dev, (size_t)ncl * 4, hipMemcpyDeviceToHost, s));
        FMS_HIP(hipMemcpyAsync(hk, kcnt_dev, (size_t)ncl * 4, hipMemcpyDeviceToHost, s));
        FMS_HIP(wait_stream(s));
        if (trace)
            std::fprintf(stderr, "[fms] fit_batched round %d: coverage and pools %.3f ms, round %.3f ms\n", rounds,
                         ms_since(t_round) - t_draw - t_iter - t_merge, ms_since(t_round));
        bool any = false;
        for (int c = 0; c < ncl; ++c) {
            if (!active[c]) continue;
            plen[c] = hlen[c];
            const long long K = hk[c];
            if (plen[c] == 0 || N[c] >= (long long)p->L * K) active[c] = 0;
            else N[c] *= 2;
            any = any || active[c];
        }
        if (!any) break;
    }
    if (rounds_out) *rounds_out = rounds;

    // modes and labels
    long long K = 0;
    k_off[0] = 0;
    for (int c = 0; c < ncl; ++c) {
        K += hk[c];
        k_off[c + 1] = K;
    }
    if (K > max_modes) return fail(MS_E_CAPACITY, "more modes than max_modes (k_off holds the required counts)");
    for (int c = 0; c < ncl; ++c)
        if (x_off[c + 1] > x_off[c] && hk[c] == 0) return fail(MS_E_NO_MODES, "a cloud has no converged seed");
    for (int c = 0; c <= ncl; ++c) hmoff[c] = (int32_t)k_off[c];
    FMS_HIP(hipMemcpyAsync(moff_dev, hmoff, (size_t)(ncl + 1) * 4, hipMemcpyHostToDevice, s));
    if (K > 0) FMS_HIP(launch_bf_modes_out(nm_dev, d, xo_dev, ncl, moff_dev, modes, s));
    if (labels) FMS_HIP(launch_bf_assign(X, d, xo_dev, ncl, modes, moff_dev, labels, n, s));
    FMS_HIP(wait_stream(s));
    if (trace) std::fprintf(stderr, "[fms] fit_batched done: %lld modes, %.3f ms\n", K, ms_since(t_start));
    return MS_OK;
}

// Times each candidate R on private copies of the seeds; records the fastest.
int tune_batched_impl(const ms_params* p, const float* X, const int64_t* x_off, const float* seeds,
                      const int64_t* s_off, int ncl, int d, int trials, int32_t* best_R,
                      float* ms_per_iter, int32_t* best_chunk, int32_t* best_grid, hipStream_t s) {
    const long long n = x_off[ncl], M = s_off[ncl];
    const int D = step_shape(d).D;
    Workspace ws(s);
    float* S;
    uint8_t* conv;
    int32_t* it;
    float* sh2;
    FMS_CHECK(ws.alloc(&S, (size_t)M * d));
    FMS_CHECK(ws.alloc(&conv, (size_t)M));
    FMS_CHECK(ws.alloc(&it, (size_t)M));
    FMS_CHECK(ws.alloc(&sh2, (size_t)M));
    FMS_CHECK(g_events.create());
    hipEvent_t* ev = g_events.e;
    ms_params q = *p;
    q.graph = 0;
    q.tile_R = 0;
    const int candR[3] = {1, 2, 4};
    const int candC[4] = {512, 1024, 2048, 4096};
    const int candG[3] = {1024, 2048, 4096};
    TuneShape best{0, kBatchedChunk, kBatchedGrid};
    float best_ms = 0.0f;
    for (int c = 0; c < 3; ++c) {
        if (ms_per_iter) ms_per_iter[c] = -1.0f;
        if (!batched_R_ok(D, candR[c])) continue;
        if (p->precision == MS_PREC_BF16_REFINE && candR[c] != 2) continue;   // tiles of 128 only
        for (int ci = 0; ci < 4; ++ci)
            for (int gi = 0; gi < 3; ++gi) {
                q.tile_chunk = candC[ci];
                q.tile_grid = candG[gi];
                float ms = 0.0f;
                // one untimed pass (first launch of the shape), then the timed one
                for (int pass = 0; pass < 2; ++pass) {
                    FMS_HIP(hipMemcpyAsync(S, seeds, (size_t)M * d * 4, hipMemcpyDeviceToDevice, s));
                    FMS_HIP(launch_fill_u8(conv, (int)M, 0, s));
                    FMS_CHECK(step_batched_impl(&q, X, x_off, S, s_off, ncl, d, pass ? trials : 1, conv, it, sh2,
                                                s, candR[c], pass ? ev : nullptr));
                }
                FMS_HIP(hipEventSynchronize(ev[1]));
                FMS_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
                ms /= (float)trials;
                if (ms_per_iter && (ms_per_iter[c] < 0.0f || ms < ms_per_iter[c])) ms_per_iter[c] = ms;
                if (best.R == 0 || ms < best_ms) {
                    best = TuneShape{candR[c], candC[ci], candG[gi]};
                    best_ms = ms;
                }
            }
    }
    FMS_HIP(hipStreamSynchronize(s));
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[tune_key(d, n, M, ncl, p->precision)] = best;
    }
    if (best_R) *best_R = best.R;
    if (best_chunk) *best_chunk = best.chunk;
    if (best_grid) *best_grid = best.grid;
    return MS_OK;
}

}  // namespace
}  // namespace fms

using namespace fms;

namespace {

// Arguments of ms_step_batched and ms_tune_batched.
int check_batched_args(const ms_params* p, const float* X, const int64_t* x_off, const int64_t* s_off,
                       int32_t ncl, int32_t d) {
    FMS_CHECK(check_params(p, false));
    if (p->precision != MS_PREC_FP32 && p->precision != MS_PREC_BF16_REFINE)
        return fail(MS_E_INVALID, "unknown precision");
    if (p->precision == MS_PREC_BF16_REFINE && !batched_bf16_ok(p, d))
        return fail(MS_E_INVALID, "the batched BF16 form is built for the Gaussian kernel at 5 <= d <= 32");
    if (p->metric != MS_METRIC_EUCLIDEAN)
        return fail(MS_E_INVALID, "ms_step_batched computes the Euclidean metric only");
    if (!x_off || !s_off) return fail(MS_E_INVALID, "offsets are NULL");
    if (ncl < 1 || ncl > batched_max_clouds()) return fail(MS_E_INVALID, "ncl must be in [1, 8192]");
    if (d < 1 || d > 64) return fail(MS_E_INVALID, "the batched calls take d in [1, 64]");
    if (x_off[0] != 0 || s_off[0] != 0) return fail(MS_E_INVALID, "offsets must start at 0");
    for (int c = 0; c < ncl; ++c) {
        if (x_off[c + 1] < x_off[c] || s_off[c + 1] < s_off[c])
            return fail(MS_E_INVALID, "offsets must be nondecreasing");
        if (s_off[c + 1] > s_off[c] && x_off[c + 1] == x_off[c])
            return fail(MS_E_INVALID, "a cloud with seeds has no points");
    }
    if (x_off[ncl] > INT_MAX || s_off[ncl] > INT_MAX)
        return fail(MS_E_INVALID, "total points and seeds must be <= 2^31-1");
    if (s_off[ncl] > 0) FMS_CHECK(check_common(X, x_off[ncl], d));
    return MS_OK;
}

}  // namespace

extern "C" {

void ms_default_params(ms_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->rng_seed = 0;
    p->h = 1.0f;
    p->kernel = MS_KERNEL_GAUSSIAN;
    p->precision = MS_PREC_FP32;
    p->tol = 1e-3f;
    p->max_iter = 100;
    p->merge_radius = 1.0f;
    p->cover_radius = 1.0f;
    p->gamma = 1.0f;
    p->n_initial = 128;
    p->L = 8;
    p->refine_radius = 3.0f;
    p->all_points_as_seeds = 0;
    p->check_finite = 0;
}

int ms_fit(const ms_params* p, const float* X, int64_t n, int32_t d, float* modes,
           int32_t max_modes, int32_t* k_out, int32_t* labels, ms_diag* diag, void* stream) {
    g_err.clear();
    FMS_CHECK(check_params(p, true));
    FMS_CHECK(check_common(X, n, d));
    if (!modes) return fail(MS_E_INVALID, "modes is NULL");
    if (!k_out) return fail(MS_E_INVALID, "k_out is NULL");
    if (max_modes < 1) return fail(MS_E_INVALID, "max_modes must be >= 1");
    if (p->precision == MS_PREC_BF16_REFINE && !bf16_supported(d))
        return fail(MS_E_INVALID, "precision MS_PREC_BF16_REFINE supports 1 <= d <= 32");
    *k_out = 0;
    return fit_impl(p, X, (int)n, d, modes, max_modes, k_out, labels, diag, (hipStream_t)stream);
}

int ms_step(const ms_params* p, const float* X, int64_t n, int32_t d, float* seeds, int32_t m,
            int32_t n_iter, uint8_t* converged, int32_t* iters, float* shift2, void* stream) {
    g_err.clear();
    FMS_CHECK(check_params(p, false));
    FMS_CHECK(check_common(X, n, d));
    if (m < 0) return fail(MS_E_INVALID, "m must be >= 0");
    if (n_iter < 0 || n_iter > kMaxIterCap) return fail(MS_E_INVALID, "n_iter must be in [0, 4096]");
    if (m == 0) return MS_OK;
    if (!seeds || !converged || !iters || !shift2) return fail(MS_E_INVALID, "NULL seed array");
    if (p->precision == MS_PREC_BF16_REFINE && !bf16_supported(d))
        return fail(MS_E_INVALID, "precision MS_PREC_BF16_REFINE supports 1 <= d <= 32");
    return step_impl(p, X, (int)n, d, seeds, m, n_iter, converged, iters, shift2, (hipStream_t)stream);
}

int ms_step_noalloc(const ms_params* p, const float* X, int64_t n, int32_t d, float* seeds, int32_t m,
                    int32_t n_iter, uint8_t* converged, int32_t* iters, float* shift2, void* stream) {
    g_err.clear();
    FMS_CHECK(check_params(p, false));
    FMS_CHECK(check_common(X, n, d));
    if (m < 0) return fail(MS_E_INVALID, "m must be >= 0");
    if (n_iter < 0 || n_iter > kMaxIterCap) return fail(MS_E_INVALID, "n_iter must be in [0, 4096]");
    if (m == 0) return MS_OK;
    if (!seeds || !converged || !iters || !shift2) return fail(MS_E_INVALID, "NULL seed array");
    if (p->precision == MS_PREC_BF16_REFINE && !bf16_supported(d))
        return fail(MS_E_INVALID, "precision MS_PREC_BF16_REFINE supports 1 <= d <= 32");
    return step_noalloc_impl(p, X, (int)n, d, seeds, m, n_iter, converged, iters, shift2,
                             (hipStream_t)stream);
}

int ms_step_batched(const ms_params* p, const float* X, const int64_t* x_off, float* seeds,
                    const int64_t* s_off, int32_t ncl, int32_t d, int32_t n_iter, uint8_t* converged,
                    int32_t* iters, float* shift2, void* stream) {
    g_err.clear();
    FMS_CHECK(check_batched_args(p, X, x_off, s_off, ncl, d));
    if (n_iter < 0 || n_iter > kMaxIterCap) return fail(MS_E_INVALID, "n_iter must be in [0, 4096]");
    if (s_off[ncl] == 0) return MS_OK;
    if (!seeds || !converged || !iters || !shift2) return fail(MS_E_INVALID, "NULL seed array");
    return step_batched_impl(p, X, x_off, seeds, s_off, ncl, d, n_iter, converged, iters, shift2,
                             (hipStream_t)stream, p->tile_R);
}

int ms_fit_batched(const ms_params* p, const float* X, const int64_t* x_off, int32_t ncl, int32_t d,
                   float* modes, int64_t max_modes, int64_t* k_off, int32_t* labels, int32_t* rounds,
                   void* stream) {
    g_err.clear();
    FMS_CHECK(check_params(p, true));
    FMS_CHECK(check_batched_args(p, X, x_off, x_off, ncl, d));
    if (p->gamma != 1.0f) return fail(MS_E_INVALID, "ms_fit_batched runs every round to convergence: gamma must be 1");
    if (!k_off) return fail(MS_E_INVALID, "k_off is NULL");
    if (!modes) return fail(MS_E_INVALID, "modes is NULL");
    if (max_modes < 1) return fail(MS_E_INVALID, "max_modes must be >= 1");
    if (x_off[ncl] == 0) return fail(MS_E_INVALID, "no cloud has points");
    return fit_batched_impl(p, X, x_off, ncl, d, modes, max_modes, k_off, labels, rounds, (hipStream_t)stream);
}

int ms_tune_batched(const ms_params* p, const float* X, const int64_t* x_off, const float* seeds,
                    const int64_t* s_off, int32_t ncl, int32_t d, int32_t trials, int32_t* best_R,
                    float* ms_per_iter, int32_t* best_chunk, int32_t* best_grid, void* stream) {
    g_err.clear();
    FMS_CHECK(check_batched_args(p, X, x_off, s_off, ncl, d));
    if (trials < 1 || trials > 64) return fail(MS_E_INVALID, "trials must be in [1, 64]");
    if (s_off[ncl] == 0) return fail(MS_E_INVALID, "no cloud has seeds");
    if (!seeds) return fail(MS_E_INVALID, "seeds is NULL");
    return tune_batched_impl(p, X, x_off, seeds, s_off, ncl, d, trials, best_R, ms_per_iter, best_chunk,
                             best_grid, (hipStream_t)stream);
}

int ms_assign(const float* X, int64_t n, int32_t d, const float* modes, int32_t k, int32_t* labels,
              float* margin, void* stream) {
    g_err.clear();
    FMS_CHECK(check_common(X, n, d));
    if (!modes) return fail(MS_E_INVALID, "modes is NULL");
    if (!labels) return fail(MS_E_INVALID, "labels is NULL");
    if (k < 1) return fail(MS_E_INVALID, "k must be >= 1");
    FMS_HIP(launch_assign(X, (int)n, d, modes, k, labels, margin, (hipStream_t)stream));
    return MS_OK;
}

static int check_diff(const void* X, int32_t nbatch, int64_t n, const void* S, int64_t m, int32_t d,
                      double h, int32_t bytes) {
    if (!X || !S) return fail(MS_E_INVALID, "NULL array");
    if (bytes != 4 && bytes != 8) return fail(MS_E_INVALID, "dtype_bytes must be 4 or 8");
    if (nbatch < 1 || nbatch > 65535) return fail(MS_E_INVALID, "nbatch must be in [1, 65535]");
    if (n < 1 || m < 1 || n > INT_MAX / 2 || m > INT_MAX / 2) return fail(MS_E_INVALID, "bad n or m");
    if (d < 1 || d > 64) return fail(MS_E_INVALID, "the differentiable calls take d in [1, 64]");
    if (!(std::isfinite(h) && h > 0.0)) return fail(MS_E_INVALID, "h must be finite and > 0");
    return MS_OK;
}

int ms_forward_update(const void* X, int32_t nbatch, int64_t n, const void* S_in, int64_t m, int32_t d,
                      double h, void* S_out, int32_t dtype_bytes, void* stream) {
    g_err.clear();
    FMS_CHECK(check_diff(X, nbatch, n, S_in, m, d, h, dtype_bytes));
    if (!S_out) return fail(MS_E_INVALID, "S_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    FMS_CHECK(ensure_pool_release_threshold());
    Workspace ws(s);
    char* w;
    FMS_CHECK(ws.alloc(&w, adjoint_workspace_bytes(nbatch, (int)n, (int)m, d, dtype_bytes)));
    FMS_HIP(launch_forward_update(X, nbatch, (int)n, S_in, (int)m, d, h, S_out, dtype_bytes, w, s));
    return MS_OK;
}

int ms_step_adjoint(const void* X, int32_t nbatch, int64_t n, const void* S, int64_t m, int32_t d,
                    double h, const void* G, void* dS, void* dX, int32_t dtype_bytes, void* stream) {
    g_err.clear();
    FMS_CHECK(check_diff(X, nbatch, n, S, m, d, h, dtype_bytes));
    if (!G || !dS || !dX) return fail(MS_E_INVALID, "NULL gradient array");
    hipStream_t s = (hipStream_t)stream;
    FMS_CHECK(ensure_pool_release_threshold());
    Workspace ws(s);
    char* w;
    FMS_CHECK(ws.alloc(&w, adjoint_workspace_bytes(nbatch, (int)n, (int)m, d, dtype_bytes)));
    FMS_HIP(launch_step_adjoint(X, nbatch, (int)n, S, (int)m, d, h, G, dS, dX, dtype_bytes, w, s));
    return MS_OK;
}

int ms_seed_draw(uint64_t* state, const int32_t* pool, int32_t len, int32_t count, int32_t* out) {
    g_err.clear();
    if (!state || !pool || !out) return fail(MS_E_INVALID, "NULL argument");
    if (len < 0 || count < 0 || count > len) return fail(MS_E_INVALID, "need 0 <= count <= len");
    std::vector<int32_t> pos((size_t)count);
    draw_positions(state, len, count, pos.data());
    for (int32_t t = 0; t < count; ++t) out[t] = pool[pos[t]];
    return MS_OK;
}

int ms_seed_count_next(int32_t n_last, int32_t modes, int32_t H, int32_t* n_next) {
    g_err.clear();
    if (!n_next) return fail(MS_E_INVALID, "NULL argument");
    if (n_last < 1 || modes < 0 || H < 1) return fail(MS_E_INVALID, "need n_last >= 1, modes >= 0, H >= 1");
    // Section II-D, frame sequences: a count above H times the mode count is
    // too expensive and shrinks by one mode count per frame
    long long next = n_last;
    if ((long long)n_last > (long long)H * modes) next = (long long)n_last - modes;
    *n_next = (int32_t)std::max(1LL, next);
    return MS_OK;
}

int ms_release_workspace(void) {
    g_err.clear();
    free_orphans();
    g_graph.clear();
    for (auto& c : g_cache) c->release();
    g_cache.clear();
    for (Pinned* q : {&g_pin_ctl, &g_pin_pos, &g_pin_rb, &g_pin_modes, &g_pin_bpos, &g_pin_bso, &g_pin_bso32,
                      &g_pin_bconv, &g_pin_bmoff, &g_pin_blen, &g_pin_bk})
        q->release();
    return MS_OK;
}

int ms_graph_stats(int64_t* instantiations, int64_t* updates) {
    if (instantiations) *instantiations = g_graph.instantiations;
    if (updates) *updates = g_graph.updates;
    return MS_OK;
}

const char* ms_last_error(void) { return g_err.c_str(); }

const char* ms_version(void) { return "libfms 0.1 (gfx950)"; }

}  // extern "C"
