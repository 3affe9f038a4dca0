// Host driver of the C ABI declared in include/rhif.h: the level loop of the factorization
// (Sec. 3.1 / 3.2 of the paper), the factor apply (eq. (3.2)) and the PCG solve (Sec. 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rhif.h"
#include "devstructs.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_last_error;

struct Failure {
    rhif_status st;
    std::string msg;
};

[[noreturn]] void fail(rhif_status st, const std::string& msg) { throw Failure{st, msg}; }

void hipcheck(hipError_t e, const char* what, int line) {
    if (e != hipSuccess) {
        char buf[256];
        std::snprintf(buf, sizeof(buf), "%s failed at line %d: %s", what, line, hipGetErrorString(e));
        fail(e == hipErrorOutOfMemory ? RHIF_ENOMEM : RHIF_EDEVICE, buf);
    }
}
#define HIPCHK(x) hipcheck((x), #x, __LINE__)

constexpr int kLdsBudgetDoubles = 8192;      // 64 KiB of LDS per workgroup (default kernels)
constexpr int kLdsMaxDoubles = 20480;        // 160 KiB: the gfx950 per-workgroup limit
constexpr int kApplyCap = kLdsBudgetDoubles - rhif::kApplyDiagDoubles - rhif::kApplyExtDoubles - 32;
// largest leading block k_chol_lead factors in LDS ((p|1) p + kPotrfSmemFixed <= 20480 doubles;
// k_trsm_rows then needs 4 * 17 * 144 doubles)
constexpr int kCholLdsPmax = 139;
constexpr int kElimPanel = 128;   // panel width of the elimination of large interiors
constexpr int kStaticLdsReserve = 32;         // doubles of static LDS a kernel may declare
constexpr int kRedBlocks = 1024;              // fixed partial-sum layout of the CG reductions
constexpr int32_t kRemovedFlags = 4;          // option bits that no longer exist
constexpr int64_t kBigSkelElems = 1 << 18;    // M (rows x columns) from which the ID spreads over
                                              // many workgroups per group
constexpr int kBigCheck = 16;                 // steps between the host's checks for active groups
constexpr int kScaleRowsPerWG = 128;          // strips of a group pair's two-sided scaling per workgroup
constexpr int kPrecondPanelMinN = 256;        // larger groups: block-Jacobi Cholesky by the panel kernels

// Planner state of one problem of a factorization call: scratch, level plans and the
// host tables of the skeleton apply. The sets are kept for reuse (PlanPool); the level-0 plan
// depends on the grid and the leaf size alone (every unknown is active at the leaf level) and
// is reused by the next factorization of the same geometry that takes the set.
struct PlanSet {
    rhif::PlanScratch scr;
    std::vector<rhif::LevelPlan*> plans;
    bool plan0_ok = false;
    int plan0_key[3] = {0, 0, 0};
    std::vector<rhif::ApplyDesc> sk_ad;
    std::vector<int32_t> sk_dofs;
    std::vector<rhif::GroupApplyDesc> gad;
    std::vector<int32_t> skel_of;
    rhif::LevelPlan& plan(int lvl) {
        while (static_cast<int>(plans.size()) <= lvl) plans.push_back(new rhif::LevelPlan());
        return *plans[lvl];
    }
};

// The planner states not in use, shared by all host threads: a factorization takes one per
// problem, preferring one whose level-0 plan is of the problem's geometry, and gives them
// back when it ends.
class PlanPool {
public:
    static PlanPool& get() {
        static PlanPool* p = new PlanPool();
        return *p;
    }
    // keys[i] = (dim, side, leaf) of problem i
    std::vector<PlanSet*> take(const std::vector<std::array<int, 3>>& keys) {
        std::lock_guard<std::mutex> lk(mu_);
        std::vector<PlanSet*> out(keys.size(), nullptr);
        for (size_t i = 0; i < keys.size(); ++i)
            for (size_t j = 0; j < free_.size(); ++j) {
                PlanSet* ps = free_[j];
                if (ps->plan0_ok && ps->plan0_key[0] == keys[i][0] && ps->plan0_key[1] == keys[i][1] &&
                    ps->plan0_key[2] == keys[i][2]) {
                    out[i] = ps;
                    free_.erase(free_.begin() + j);
                    break;
                }
            }
        for (auto& ps : out) {
            if (ps) continue;
            if (!free_.empty()) {
                ps = free_.back();
                free_.pop_back();
            } else {
                ps = new PlanSet();
            }
        }
        return out;
    }
    void give(const std::vector<PlanSet*>& sets) {
        std::lock_guard<std::mutex> lk(mu_);
        for (PlanSet* ps : sets)
            if (ps) free_.push_back(ps);
    }

private:
    std::mutex mu_;
    std::vector<PlanSet*> free_;
};

// The planner states of one factorization call, given back however the call ends.
struct PlanLease {
    std::vector<PlanSet*> sets;
    ~PlanLease() { PlanPool::get().give(sets); }
};

// The descriptor tables of one level concatenated over the problems of a factorization
// call, every offset moved to the problem's share of the level-wide arrays.
struct MergedTables {
    std::vector<rhif::CellRef> cref;
    std::vector<rhif::FrontDesc> pot[2];   // cell eliminations below the root, at the root
    std::vector<rhif::SepDesc> sep;
    std::vector<rhif::CellGroup> cg;
    std::vector<rhif::CellScaleDesc> cs;
    std::vector<rhif::SkelDesc> skd;
    std::vector<int32_t> cgptr, cgl, cgoff;
};

// Waits for an event by polling it (short waits wake the host sooner than a blocking
// synchronization); a wait longer than kPollMs blocks.
void poll_event(hipEvent_t ev) {
    constexpr auto kPollMs = std::chrono::milliseconds(2);
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) HIPCHK(e);
        if (std::chrono::steady_clock::now() - t0 > kPollMs) break;
    }
    HIPCHK(hipEventSynchronize(ev));
}

// Per-thread host state reused across factorizations: pinned staging buffers for the
// uploads (a ring, each slot fenced by the event of its last copy), a pinned buffer for
// the small read-backs and the merged tables (so that repeated factorizations do not pay
// for fresh allocations and page faults). Kept for the life of the process.
struct HostCache {
    MergedTables mt;
    static constexpr int kSlots = 3;
    char* up[kSlots] = {};
    size_t up_bytes[kSlots] = {};
    hipEvent_t up_ev[kSlots] = {};
    bool up_pending[kSlots] = {};
    int next = 0;
    char* down = nullptr;
    size_t down_bytes = 0;

    char* get_up(size_t b, int& slot) {
        slot = next;
        next = (next + 1) % kSlots;
        if (up_pending[slot]) {
            HIPCHK(hipEventSynchronize(up_ev[slot]));
            up_pending[slot] = false;
        }
        if (b > up_bytes[slot]) {
            if (up[slot]) (void)hipHostFree(up[slot]);
            up[slot] = nullptr;
            const size_t nb = std::max(b, 2 * up_bytes[slot]);
            up_bytes[slot] = 0;
            HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&up[slot]), nb, hipHostMallocDefault));
            up_bytes[slot] = nb;
        }
        return up[slot];
    }
    void fence(int slot, hipStream_t s) {
        if (!up_ev[slot]) HIPCHK(hipEventCreateWithFlags(&up_ev[slot], hipEventDisableTiming));
        HIPCHK(hipEventRecord(up_ev[slot], s));
        up_pending[slot] = true;
    }
    // per device: a stream for table uploads that may overlap the kernels of the factor's
    // stream, and events that order them (round robin)
    std::vector<hipStream_t> side;
    std::vector<std::array<hipEvent_t, 4>> side_ev;
    std::vector<int> side_next;
    hipStream_t side_stream(int dev, hipEvent_t& ev) {
        if (static_cast<int>(side.size()) <= dev) {
            side.resize(dev + 1, nullptr);
            side_ev.resize(dev + 1);
            side_next.resize(dev + 1, 0);
        }
        if (!side[dev]) {
            HIPCHK(hipStreamCreateWithFlags(&side[dev], hipStreamNonBlocking));
            for (auto& e : side_ev[dev]) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        ev = side_ev[dev][side_next[dev]];
        side_next[dev] = (side_next[dev] + 1) % 4;
        return side[dev];
    }
    // pinned word for the error read-backs
    unsigned long long* errw = nullptr;
    unsigned long long* err_word() {
        if (!errw) HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&errw), 64, hipHostMallocDefault));
        return errw;
    }
    // Waits for the work queued on s so far, by polling (the waits of the level loop are
    // short: the rank read-back after a level's last kernel).
    std::vector<hipEvent_t> wait_ev;
    void wait(hipStream_t s, int dev) {
        if (static_cast<int>(wait_ev.size()) <= dev) wait_ev.resize(dev + 1, nullptr);
        if (!wait_ev[dev]) HIPCHK(hipEventCreateWithFlags(&wait_ev[dev], hipEventDisableTiming));
        HIPCHK(hipEventRecord(wait_ev[dev], s));
        poll_event(wait_ev[dev]);
    }
    // s waits for every upload queued so far on the device's upload stream
    std::vector<hipEvent_t> join_ev;
    void side_join(hipStream_t s, int dev) {
        hipEvent_t unused = nullptr;
        const hipStream_t cs = side_stream(dev, unused);
        if (static_cast<int>(join_ev.size()) <= dev) join_ev.resize(dev + 1, nullptr);
        if (!join_ev[dev]) HIPCHK(hipEventCreateWithFlags(&join_ev[dev], hipEventDisableTiming));
        HIPCHK(hipEventRecord(join_ev[dev], cs));
        HIPCHK(hipStreamWaitEvent(s, join_ev[dev], 0));
    }
    char* get_down(size_t b) {
        if (b > down_bytes) {
            if (down) (void)hipHostFree(down);
            down = nullptr;
            const size_t nb = std::max<size_t>(b, std::max<size_t>(2 * down_bytes, 1 << 16));
            down_bytes = 0;
            HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&down), nb, hipHostMallocDefault));
            down_bytes = nb;
        }
        return down;
    }
};
HostCache& host_cache() {
    thread_local HostCache* c = new HostCache();
    return *c;
}

// Host threads for the per-problem planning of a factorization call with several problems
// (the planner's work on different problems is independent). The threads live for the
// life of the process and wait between calls; the caller's thread takes part.
class HostPool {
public:
    static HostPool& get() {
        static HostPool* p = new HostPool();
        return *p;
    }
    // fn(i) for every i in [0, n); returns when all calls have returned, rethrowing the
    // first exception any of them threw. One call at a time (others wait).
    void run(int n, const std::function<void(int)>& fn) {
        if (n <= 1 || nthreads_ == 0) {
            for (int i = 0; i < n; ++i) fn(i);
            return;
        }
        std::lock_guard<std::mutex> one(run_mu_);
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            n_ = n;
            next_.store(0);
            pending_ = nthreads_;
            err_ = nullptr;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return pending_ == 0; });
        fn_ = nullptr;
        if (err_) std::rethrow_exception(err_);
    }

private:
    HostPool() {
        const unsigned hw = std::thread::hardware_concurrency();
        nthreads_ = static_cast<int>(std::min(15u, hw > 1 ? hw - 1 : 0u));
        for (int t = 0; t < nthreads_; ++t) std::thread([this] { loop(); }).detach();
    }
    void work() {
        for (;;) {
            const int i = next_.fetch_add(1);
            if (i >= n_) break;
            try {
                (*fn_)(i);
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu_);
                if (!err_) err_ = std::current_exception();
            }
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
            }
            work();
            std::lock_guard<std::mutex> lk(mu_);
            if (--pending_ == 0) done_cv_.notify_one();
        }
    }
    int nthreads_ = 0;
    std::mutex run_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)>* fn_ = nullptr;
    int n_ = 0;
    std::atomic<int> next_{0};
    int pending_ = 0;
    uint64_t gen_ = 0;
    std::exception_ptr err_;
};

// Packs host arrays into one upload; every sub-array is 256-byte aligned.
struct Packer {
    std::vector<std::pair<const void*, size_t>> parts;
    std::vector<size_t> offs;
    size_t total = 0;
    size_t add(const void* p, size_t bytes) {
        total = (total + 255) / 256 * 256;
        offs.push_back(total);
        parts.emplace_back(p, bytes);
        total += bytes;
        return offs.back();
    }
    template <class T>
    size_t add(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
};

struct LevelDev {
    bool root = false;
    bool leaf_banded = false;   // cells factored by k_leaf_elim (block-bidiagonal L)
    bool precond = false;   // block Jacobi applied at this level
    double* front = nullptr;
    double* lg = nullptr;
    double* tp = nullptr;
    double* gp = nullptr;
    int32_t* ext = nullptr;    // per-panel nonzero row ends of the cells' L
    double* linv = nullptr;    // inverses of the 16 x 16 diagonal blocks: cells' L,
    double* li = nullptr;      //   the block-Jacobi factors L_g,
    double* skli = nullptr;    //   and the skeleton eliminations' L~
    // device views into the uploaded tables
    int32_t* cdofs = nullptr;
    rhif::CellRef* cref = nullptr;
    rhif::Tile* tiles = nullptr;
    int32_t* src = nullptr;
    int32_t* cg2 = nullptr;       // per frontal unknown: its group and position at the level below
    int32_t* ct2 = nullptr;
    int32_t* gslot_cnt = nullptr; // per group: the cells containing it and its frontal offsets there
    int32_t* gslot_cell = nullptr;
    int32_t* gslot_off = nullptr;
    rhif::ApplyDesc* cell_ad = nullptr;
    rhif::ApplyDesc* sep_ad = nullptr;
    rhif::GatherDesc* gat = nullptr;
    int32_t* sepdofs = nullptr;
    rhif::ApplyDesc* skel_ad = nullptr;
    int32_t* skeldofs = nullptr;
    rhif::GroupApplyDesc* grp_ad = nullptr;   // fused per-group apply (gather, L_g, skeleton)
    int32_t* permd = nullptr;                 // group-local pivot orders of the level's IDs
    int n_grp = 0, mn_grp = 0;
    int tk_cap = 0;               // largest k (n - k) of the level's skeletonized groups, if staged
    int tk_raw = 0;               // the same, staged or not
    int n_cell_ad = 0, n_sep_ad = 0, n_gather = 0, n_skel_ad = 0;
    size_t lds_cell = 0, lds_sep = 0, lds_skel = 0;
    // largest n_I / n_B of each block family (split apply when n_I is small enough)
    int mi_cell = 0, mb_cell = 0, mi_sep = 0, mi_skel = 0, mb_skel = 0;
    // algorithmic bytes of one apply sweep over each block family
    double b_cell = 0.0, b_sep = 0.0, b_gather = 0.0, b_skel = 0.0;
    int64_t bytes = 0;   // device bytes of the factor held for this level
    // ID choices (host)
    std::vector<int32_t> k, perm, first_dof, gsize;
    // a factorization call with several problems: this problem's share of the level-wide
    // arrays (element offsets) and host copies of its apply tables, from which the solves
    // over all the call's problems build their merged tables
    int64_t o_front = 0, o_ext = 0, o_lg = 0, o_li = 0, o_t = 0, o_g = 0, o_skli = 0;
    int64_t o_cdofs = 0, o_sepdofs = 0, o_skeldofs = 0, o_perm = 0;
    std::vector<rhif::ApplyDesc> h_cell_ad, h_sep_ad, h_skel_ad;
    std::vector<rhif::GatherDesc> h_gat;
    std::vector<rhif::GroupApplyDesc> h_gad;
};

void apply_max(const std::vector<rhif::ApplyDesc>& v, int& mi, int& mb) {
    mi = mb = 0;
    for (const auto& d : v) {
        mi = std::max(mi, d.nI);
        mb = std::max(mb, d.nB);
    }
}

size_t apply_lds(const std::vector<rhif::ApplyDesc>& v) {
    int m = 0;
    for (const auto& d : v)
        if (d.wsoff < 0) m = std::max(m, d.nI + d.nB);
    return static_cast<size_t>(rhif::kApplyDiagDoubles + rhif::kApplyExtDoubles + m) * sizeof(double);
}

int grid_for(int64_t N) {
    const int64_t b = (N + 255) / 256;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, kRedBlocks)));
}

}  // namespace

// Pinned host words for the PCG scalars of a handle: 64-byte slots carved from pages that
// are allocated once and recycled between handles (no pinned allocation per handle).
class PinnedSlots {
public:
    static PinnedSlots& get() {
        static PinnedSlots* p = new PinnedSlots();
        return *p;
    }
    double* take() {
        std::lock_guard<std::mutex> lk(mu_);
        if (free_.empty()) {
            char* page = nullptr;
            if (hipHostMalloc(reinterpret_cast<void**>(&page), kPage, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            for (size_t o = 0; o < kPage; o += kSlot) free_.push_back(reinterpret_cast<double*>(page + o));
        }
        double* p = free_.back();
        free_.pop_back();
        return p;
    }
    void give(double* p) {
        std::lock_guard<std::mutex> lk(mu_);
        free_.push_back(p);
    }

private:
    static constexpr size_t kPage = 4096, kSlot = 64;
    std::mutex mu_;
    std::vector<double*> free_;
};

// Device memory of factor handles. Every handle bump-allocates from chunks that it takes
// from a per-device cache of freed chunks (hipMalloc only on a miss) and returns them when
// it is destroyed, after the device has finished with them: a factorization then performs
// no allocation call once the cache holds chunks of the sizes it needs.
class ChunkCache {
public:
    static ChunkCache& of_device(int dev) {
        static std::mutex mu;
        static std::map<int, ChunkCache*> all;
        std::lock_guard<std::mutex> lk(mu);
        ChunkCache*& c = all[dev];
        if (!c) c = new ChunkCache();
        return *c;
    }
    // A chunk of at least `want` bytes (and at most twice as large if taken from the cache).
    void* take(size_t want, size_t& got) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(want);
            if (it != free_.end() && it->first <= 2 * want) {
                got = it->first;
                void* p = it->second;
                free_.erase(it);
                cached_ -= got;
                return p;
            }
        }
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            trim(0);   // give the cached chunks back to the device and try once more
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        got = want;
        return p;
    }
    void give(void* p, size_t bytes) {
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(bytes, p);
        cached_ += bytes;
        if (cached_ > kMaxCached) trim_locked(kMaxCached);
    }
    void trim(size_t keep) {
        std::lock_guard<std::mutex> lk(mu_);
        trim_locked(keep);
    }

private:
    static constexpr size_t kMaxCached = size_t(64) << 30;   // bytes kept for reuse per device
    void trim_locked(size_t keep) {
        while (cached_ > keep && !free_.empty()) {
            auto it = std::prev(free_.end());   // largest first
            (void)hipFree(it->second);
            cached_ -= it->first;
            free_.erase(it);
        }
    }
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    size_t cached_ = 0;
};

constexpr int kGroupStageMax = 8192;   // doubles of T and G blocks a group apply stages in LDS
constexpr int kKbufHead = 4;   // ints before the ID outputs: the 64-bit error word, padded

// Device memory of the handles made by one factorization call (one handle, or every handle
// of a batch): bump-allocated from chunks of the per-device cache, and given back to the
// cache when the last of those handles is destroyed (each has waited for its own work).
struct Arena {
    struct Chunk {
        void* p;
        size_t bytes;
    };
    static constexpr size_t kChunkBytes = size_t(64) << 20;
    int device = 0;
    std::mutex mu;
    std::vector<Chunk> chunks;
    char* cur = nullptr;
    size_t left = 0;

    void* dalloc(size_t bytes) {
        std::lock_guard<std::mutex> lk(mu);
        const size_t b = (std::max<size_t>(bytes, 256) + 255) / 256 * 256;
        if (b > left) {
            size_t got = 0;
            void* p = ChunkCache::of_device(device).take(std::max(b, kChunkBytes), got);
            if (!p) fail(RHIF_ENOMEM, "device allocation failed");
            chunks.push_back({p, got});
            cur = static_cast<char*>(p);
            left = got;
        }
        void* ptr = cur;
        cur += b;
        left -= b;
        return ptr;
    }
    ~Arena() {
        ChunkCache& cc = ChunkCache::of_device(device);
        for (const Chunk& c : chunks) cc.give(c.p, c.bytes);
    }
};

// Level-wide arrays of one level of a factorization call with several problems (each
// problem's share lies inside them at the offsets its LevelDev records).
struct BatchLevelBase {
    double *front = nullptr, *linv = nullptr, *lg = nullptr, *li = nullptr, *tp = nullptr, *gp = nullptr,
           *skli = nullptr;
    int32_t *ext = nullptr, *cdofs = nullptr, *sepdofs = nullptr, *skeldofs = nullptr, *perm = nullptr;
};

// A merged launch set of apply blocks of several problems, all taking the same kernels.
struct MFam {
    const rhif::ApplyDesc* ad = nullptr;
    int n = 0, mi = 0, mb = 0;
    size_t lds = 0;
    int kind = 0;   // 0 fused, 1 split, 2 big
    bool band = false;
    const double* pool = nullptr;
    const double* lip = nullptr;
    const double* tp = nullptr;
    const int32_t* dofs = nullptr;
    const int32_t* ext = nullptr;
};

// One level of the merged apply: cell blocks below the root and at the root, and the group
// blocks (fused per-group kernels, or gather, block Jacobi and skeleton blocks), each family
// split by the kernels its problems take alone ([0] fused, [1] split solve and product,
// [2] panel by panel over many workgroups).
struct MLevel {
    MFam cells[3], roots[3], seps[3], skels[3];
    const rhif::GroupApplyDesc* grp = nullptr;
    int n_grp = 0, mn_grp = 0, tk = 0;
    const rhif::GatherDesc* gat = nullptr;
    int n_gat = 0;
    const BatchLevelBase* b = nullptr;
};

// The applies and PCG solves over all problems of a factorization call with several problems:
// one launch per kernel and level over the blocks of all problems, vectors concatenated.
struct BatchSolve {
    std::mutex mu;                          // one solve at a time
    std::vector<rhif_factor_s*> fs;         // the call's handles (an entry is cleared when destroyed)
    std::vector<BatchLevelBase> base;       // per level
    std::vector<int64_t> zoff;              // each problem's first unknown in the vectors
    int64_t ntot = 0;
    double* ybuf = nullptr;                 // the problems' apply scratch (their shares)
    double* ws = nullptr;
    // built at the first solve
    bool ready = false;
    bool precond = true;
    std::vector<MLevel> lev;
    rhif::BatchSeg* seg = nullptr;
    int32_t* blk = nullptr;
    int nblk = 0;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *u = nullptr, *part = nullptr, *sc = nullptr;
    int32_t* active = nullptr;
    double* hsc = nullptr;                  // pinned host copies of the scalars
    int32_t* hact = nullptr;                // pinned host copy of the active flags
    ~BatchSolve() {
        if (hsc) (void)hipHostFree(hsc);
        if (hact) (void)hipHostFree(hact);
    }
};

struct rhif_factor_s {
    rhif::GridInfo g;
    rhif_opts o{};
    int L = 0;        // skeletonization levels of the paper's level loop (the root is level L)
    int Lskel = 0;    // the same count (kept for the ID getter)
    int64_t nnz = 0;
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    double* val = nullptr;
    std::vector<LevelDev> lev;
    double* ybuf = nullptr;
    int64_t y_elems = 0;
    double* ws = nullptr;
    int64_t ws_elems = 0;
    // PCG workspace
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *part = nullptr, *sc = nullptr;
    double* hsc = nullptr;                 // pinned host scalars of the PCG (read back by the graphs)
    hipEvent_t sc_ev = nullptr;            // recorded after a scalar's copy to hsc
    const double* graph_u = nullptr;       // solution vector the PCG graphs were captured with
    // HIP graphs of the solve phase, captured on first use on an internal stream:
    // [0] z <- F^-1 z;  [1] the first CG update;  [2] one PCG iteration (apply .. next update)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
    bool graphs_off = false;

    rhif_stats_t stats{};
    std::shared_ptr<Arena> arena;   // device memory (shared with the other handles of a batch)
    std::shared_ptr<BatchSolve> bsolve;   // a call with several problems: their joint solves
    int bidx = -1;                        // this problem's place in that call
    int64_t o_ybuf = 0, o_ws = 0;         // its share of the call-wide apply scratch
    // the last work of the handle on every stream it was used on (its memory may be reused
    // once these have completed)
    std::vector<std::pair<hipStream_t, hipEvent_t>> done_ev;
    void mark(hipStream_t st) {
        hipEvent_t e = nullptr;
        for (auto& p : done_ev)
            if (p.first == st) e = p.second;
        if (!e) {
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            done_ev.emplace_back(st, e);
        }
        HIPCHK(hipEventRecord(e, st));
    }
    int device = 0;
    // per-launch device timing (RHIF_FLAG_KERNEL_TIMES)
    bool ktimes = false;
    uint32_t kmask = 0xffffu;
    struct Pend {
        hipEvent_t a, b;
        int cls;
        double fl, by;
    };
    std::vector<Pend> pend;
    std::vector<hipEvent_t> evpool;
    std::vector<Pend> gpend[3];   // timing events recorded inside the graphs (read after every replay)

    hipEvent_t ev() {
        if (!evpool.empty()) {
            hipEvent_t e = evpool.back();
            evpool.pop_back();
            return e;
        }
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        return e;
    }
    // After a replay of graph g has completed: add its recorded kernel times.
    void resolve_graph(int g) {
        for (const Pend& q : gpend[g]) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, q.a, q.b));
            stats.kernel_ms[q.cls] += ms;
            stats.kernel_launches[q.cls] += 1;
            stats.kernel_flops[q.cls] += q.fl;
            stats.kernel_bytes[q.cls] += q.by;
        }
    }
    void resolve() {
        for (const Pend& q : pend) {
            HIPCHK(hipEventSynchronize(q.b));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, q.a, q.b));
            stats.kernel_ms[q.cls] += ms;
            stats.kernel_launches[q.cls] += 1;
            stats.kernel_flops[q.cls] += q.fl;
            stats.kernel_bytes[q.cls] += q.by;
            evpool.push_back(q.a);
            evpool.push_back(q.b);
        }
        pend.clear();
    }

    void* dalloc(size_t bytes) { return arena->dalloc(bytes); }
    void release() {
        // the memory goes back to the cache only once no work of this handle can still use it
        for (auto& p : done_ev) {
            (void)hipEventSynchronize(p.second);
            (void)hipEventDestroy(p.second);
        }
        done_ev.clear();
        for (int g = 0; g < 3; ++g) {
            if (gexec[g]) (void)hipGraphExecDestroy(gexec[g]);
            if (graph[g]) (void)hipGraphDestroy(graph[g]);
            gexec[g] = nullptr;
            graph[g] = nullptr;
            for (const Pend& q : gpend[g]) {
                evpool.push_back(q.a);
                evpool.push_back(q.b);
            }
            gpend[g].clear();
        }
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
        if (sc_ev) (void)hipEventDestroy(sc_ev);
        sc_ev = nullptr;
        if (hsc) PinnedSlots::get().give(hsc);
        hsc = nullptr;
        for (const Pend& q : pend) {
            (void)hipEventSynchronize(q.b);
            evpool.push_back(q.a);
            evpool.push_back(q.b);
        }
        pend.clear();
        for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
        evpool.clear();
        if (bsolve) {
            std::lock_guard<std::mutex> lk(bsolve->mu);
            bsolve->fs[bidx] = nullptr;
        }
        bsolve.reset();
        arena.reset();
    }
};

namespace {

// Launch with optional HIP-event bracketing on the launch stream.
#define KTIMED(f, s, cls, fl, by, ...)                                       \
    do {                                                                     \
        hipEvent_t ea_ = nullptr;                                            \
        if ((f)->ktimes && (((f)->kmask >> (cls)) & 1u)) {                   \
            ea_ = (f)->ev();                                                 \
            HIPCHK(hipEventRecord(ea_, (s)));                                \
        }                                                                    \
        __VA_ARGS__;                                                         \
        HIPCHK(hipGetLastError());                                           \
        if (ea_) {                                                           \
            hipEvent_t eb_ = (f)->ev();                                      \
            HIPCHK(hipEventRecord(eb_, (s)));                                \
            (f)->pend.push_back({ea_, eb_, (cls), (fl), (by)});              \
        }                                                                    \
    } while (0)

void validate_grid(const rhif_grid* g) {
    if (!g) fail(RHIF_EINVAL, "grid is NULL");
    if (g->dim != 2 && g->dim != 3) fail(RHIF_EINVAL, "grid dim must be 2 or 3");
    const int s = g->n[0];
    if (s < 1) fail(RHIF_EINVAL, "grid side must be >= 1");
    for (int k = 1; k < g->dim; ++k)
        if (g->n[k] != s) fail(RHIF_EINVAL, "only cubic grids (equal sides) are supported");
    int64_t N = 1;
    for (int k = 0; k < g->dim; ++k) N *= s;
    if (N >= (int64_t(1) << 31)) fail(RHIF_EINVAL, "grid too large for 32-bit indices");
}

int64_t fd_nnz(int d, int64_t s) {
    int64_t sp = 1;
    for (int k = 0; k < d - 1; ++k) sp *= s;
    return sp * s + 2 * d * sp * (s - 1);
}

std::string step_name(int st) {
    switch (st) {
        case 0: return "E (cell elimination)";
        case 1: return "C (block-Jacobi)";
        case 2: return "K (skeleton elimination)";
        case 3: return "root";
        case 6: return "extend-add source table";
        default: return "?";
    }
}

// Turns the device error word (~0: no error) into an error return. batch: the call
// factors several problems (their blocks are numbered over all of them).
void raise_err(unsigned long long h, bool batch) {
    if (h != ~0ull) {
        const int ilevel = static_cast<int>(h >> 40);
        const int step = static_cast<int>((h >> 32) & 0xff);
        const int block = static_cast<int>(h & 0xffffffffu);
        const char* in = batch ? " (one of the batch's problems; blocks numbered over the batch)" : "";
        char buf[320];
        if (step == 6) {
            std::snprintf(buf, sizeof(buf), "internal error: extend-add sources of cell %d at level %d disagree "
                          "with the plan%s", block, ilevel, in);
            fail(RHIF_EDEVICE, buf);
        }
        if (step == 7) {
            std::snprintf(buf, sizeof(buf), "internal error: skeleton row table of group %d at level %d disagrees "
                          "with the plan%s", block, ilevel, in);
            fail(RHIF_EDEVICE, buf);
        }
        std::snprintf(buf, sizeof(buf), "not SPD: Cholesky pivot <= 0 or not finite at level %d, step %s, block %d%s",
                      ilevel, step_name(step).c_str(), block, in);
        fail(RHIF_ENOTSPD, buf);
    }
}

void check_err(const unsigned long long* err, bool batch, hipStream_t s, int dev) {
    HostCache& hc = host_cache();
    unsigned long long* h = hc.err_word();
    HIPCHK(hipMemcpyAsync(h, err, sizeof(*h), hipMemcpyDeviceToHost, s));
    hc.wait(s, dev);
    raise_err(*h, batch);
}

template <class T>
T* view(char* base, size_t off) { return reinterpret_cast<T*>(base + off); }

// Copies the packed tables to a new device buffer, asynchronously on the stream.
// extra: bytes of device memory after the tables that the device fills itself.
char* upload(rhif_factor_s* f, Packer& pk, hipStream_t s, size_t extra = 0) {
    if (pk.total == 0 && extra == 0) return nullptr;
    char* dst = static_cast<char*>(f->dalloc(pk.total + extra));
    if (pk.total == 0) return dst;
    HostCache& hc = host_cache();
    int slot = 0;
    char* h = hc.get_up(pk.total, slot);
    for (size_t e = 0; e < pk.parts.size(); ++e)
        if (pk.parts[e].second) std::memcpy(h + pk.offs[e], pk.parts[e].first, pk.parts[e].second);
    HIPCHK(hipMemcpyAsync(dst, h, pk.total, hipMemcpyHostToDevice, s));
    hc.fence(slot, s);
    return dst;
}

// The same on the upload stream, so that the copy overlaps the kernels already queued on s;
// s waits for it before anything queued after this call, or (join = false) the caller makes
// s wait later with HostCache::side_join. (The destination is fresh memory of the handle, so
// the copy depends on nothing queued before.)
char* upload_side(rhif_factor_s* f, Packer& pk, hipStream_t s, bool join = true) {
    if (pk.total == 0) return nullptr;
    HostCache& hc = host_cache();
    hipEvent_t ev = nullptr;
    hipStream_t cs = hc.side_stream(f->device, ev);
    int slot = 0;
    char* h = hc.get_up(pk.total, slot);
    for (size_t e = 0; e < pk.parts.size(); ++e)
        if (pk.parts[e].second) std::memcpy(h + pk.offs[e], pk.parts[e].first, pk.parts[e].second);
    char* dst = static_cast<char*>(f->dalloc(pk.total));
    HIPCHK(hipMemcpyAsync(dst, h, pk.total, hipMemcpyHostToDevice, cs));
    hc.fence(slot, cs);
    if (join) {
        HIPCHK(hipEventRecord(ev, cs));
        HIPCHK(hipStreamWaitEvent(s, ev, 0));
    }
    return dst;
}

int panel_cap_for(int nmax, int reserved_doubles) {
    const int cap = (kLdsBudgetDoubles - reserved_doubles - rhif::kPotrfSmemFixed) / 17;
    return std::max(0, std::min(cap, nmax));
}

size_t potrf_lds(int cap, int reserved) {
    return static_cast<size_t>(reserved + rhif::kPotrfSmemFixed + cap * 17) * sizeof(double);
}

using SkelKernel = decltype(&rhif::k_skeletonize<0, double, 16>);

// the k_skeletonize instance of a storage form, register form (rows per thread) and precision
template <typename MR>
SkelKernel skel_kernel_of(int staged, int rm) {
    using namespace rhif;
    if (staged == 4) return k_skeletonize<4, MR, 16>;
    if (rm <= 16)
        return staged == 3 ? k_skeletonize<3, MR, 16> : staged == 1 ? k_skeletonize<1, MR, 16> : k_skeletonize<0, MR, 16>;
    if (rm <= 32)
        return staged == 3 ? k_skeletonize<3, MR, 32> : staged == 1 ? k_skeletonize<1, MR, 32> : k_skeletonize<0, MR, 32>;
    return staged == 3 ? k_skeletonize<3, MR, 96> : staged == 1 ? k_skeletonize<1, MR, 96> : k_skeletonize<0, MR, 96>;
}

SkelKernel skel_kernel(int staged, int rm, bool f32) {
    return f32 ? skel_kernel_of<float>(staged, rm) : skel_kernel_of<double>(staged, rm);
}

// rows of M per thread that the register ID needs for the level's groups (the largest over
// groups with n <= 64; the same chunking as the kernel's)
int skel_rows_per_thread(const std::vector<rhif::SkelDesc>& groups) {
    int cs_max = 0;
    for (const auto& sk : groups) {
        if (sk.n > 64) continue;
        int cw = 1;
        while (cw < sk.n && cw < 64) cw <<= 1;
        const int nrc = 256 / cw;
        cs_max = std::max(cs_max, (sk.r + nrc - 1) / nrc);
    }
    return cs_max;
}

void set_kernel_attributes() {
    static std::once_flag once;
    std::call_once(once, [] {
        const int bytes = kLdsMaxDoubles * static_cast<int>(sizeof(double));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_precond_scale),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        for (const void* k : {reinterpret_cast<const void*>(&rhif::k_big_trisolve<double>),
                              reinterpret_cast<const void*>(&rhif::k_big_trisolve<float>),
                              reinterpret_cast<const void*>(&rhif::k_skeletonize<4, double, 16>),
                              reinterpret_cast<const void*>(&rhif::k_skeletonize<4, float, 16>)})
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        for (int staged : {0, 1, 3})
            for (int rm : rhif::kSkelRegForms)
                for (bool f32 : {false, true})
                    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(skel_kernel(staged, rm, f32)),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_apply_group_up),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_apply_group_dn),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_chol_lead),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_leaf_elim<false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_leaf_elim<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        // k_precond_groups also holds a few static LDS words
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_precond_groups),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kStaticLdsReserve * 8);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rhif::k_trsm_rows),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        for (const void* k : {reinterpret_cast<const void*>(&rhif::k_apply_trsv_up),
                              reinterpret_cast<const void*>(&rhif::k_apply_trsv_dn),
                              reinterpret_cast<const void*>(&rhif::k_apply_gemv_up),
                              reinterpret_cast<const void*>(&rhif::k_apply_gemv_dn)})
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipGetLastError();   // an attribute a runtime does not take must not linger
    });
}

// Caller's CSR of one problem of a factorization call.
struct CsrIn {
    const int32_t* rp;
    const int32_t* ci;
    const double* val;
};

// One problem of a factorization call while the level loop runs.
struct Prob {
    rhif_factor_s* f = nullptr;
    PlanSet* ps = nullptr;
    int64_t n_active = 0;      // unknowns active at the current level
    bool reuse0 = false;       // the level-0 plan of the slot's last factorization is reused
    int pending_skel = -1;     // level whose skeleton apply tables are still to be uploaded
    double sk_fl = 0.0;        // their skeletonization flops
    // the problem's share of the level-wide arrays (element or entry offsets)
    int64_t o_front = 0, o_ext = 0, o_lg = 0, o_li = 0, o_t = 0, o_g = 0, o_skli = 0, o_m = 0;
    int32_t o_cell = 0, o_cs = 0, o_cg = 0, o_k = 0, o_p = 0;
};

// The level loop of the factorization (Sec. 3.1 / 3.2) for one or several independent
// problems with the same options (cells and groups of different problems are as
// independent as those of one problem: Sec. 2.1, and the simultaneous skeletonization of
// Sec. 2.2). The problems advance level by level together. Their plans are made on the host
// pool; every kernel of a level that works from descriptor tables (cell elimination, block
// Jacobi, skeletonization) runs as one launch over the blocks of all problems, whose tables
// are concatenated with every offset moved to the problem's share of level-wide arrays. Only
// the frontal assembly, which reads each problem's own matrix and plan, is launched per
// problem. One read-back per level brings every problem's ranks to the host. With one
// problem the shares are the whole arrays and the launches are those of a lone factorization.
void do_factor(const std::vector<rhif_factor_s*>& fs, const CsrIn* in, hipStream_t s) {
    using namespace rhif;
    const int B = static_cast<int>(fs.size());
    const bool batch = B > 1;
    rhif_factor_s* f0 = fs[0];
    const rhif_opts& o = f0->o;
    const int d = f0->g.d;
    const int W = 1 << d;
    const int leaf = o.leaf;
    // precision 1: the interpolative decompositions in FP32; precision 2: also the Schur
    // products of the cell eliminations (level 0 and the upper levels' final
    // S = A_BB - W^T W) on the FP32 matrix cores. Cholesky factors, block Jacobi and every
    // stored factor value stay FP64.
    const bool f32 = o.precision >= 1;
    const bool f32schur = o.precision == 2;
    HostCache& hc = host_cache();
    MergedTables& mt = hc.mt;
    HostPool& pool = HostPool::get();
    // The skeleton apply tables are copied on the upload stream and read by no kernel of the
    // factorization, so the factor's stream joins those copies once, at the end. If the call
    // fails before that, the guard waits for them before the handles' memory is released.
    struct SideGuard {
        HostCache& hc;
        int dev;
        bool armed = false;
        ~SideGuard() {
            if (!armed) return;
            hipEvent_t unused = nullptr;
            (void)hipStreamSynchronize(hc.side_stream(dev, unused));
        }
    } side_guard{hc, f0->device};

    // the error word leads the block of the ID outputs, so that one copy reads back both
    int32_t* kbuf = static_cast<int32_t*>(f0->dalloc(kKbufHead * sizeof(int32_t)));
    unsigned long long* err = reinterpret_cast<unsigned long long*>(kbuf);
    int64_t kp_elems = 0;
    double* mp = nullptr;   // ID scratch (the largest level)
    int64_t mp_elems = 0;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, err, ~0ull);

    std::vector<Prob> pr(B);
    PlanLease lease;
    {
        std::vector<std::array<int, 3>> keys(B);
        for (int p = 0; p < B; ++p) keys[p] = {d, fs[p]->g.s, leaf};
        lease.sets = PlanPool::get().take(keys);
    }
    int Lmax = 0;
    for (int p = 0; p < B; ++p) {
        rhif_factor_s* f = fs[p];
        Prob& q = pr[p];
        q.f = f;
        q.ps = lease.sets[p];
        q.n_active = f->g.N;
        Lmax = std::max(Lmax, f->L);
        f->lev.resize(f->L + 1);
        // every handle keeps its own copy of A
        f->nnz = fd_nnz(d, f->g.s);
        f->rp = static_cast<int32_t*>(f->dalloc((f->g.N + 1) * sizeof(int32_t)));
        f->ci = static_cast<int32_t*>(f->dalloc(f->nnz * sizeof(int32_t)));
        f->val = static_cast<double*>(f->dalloc(f->nnz * sizeof(double)));
        HIPCHK(hipMemcpyAsync(f->rp, in[p].rp, (f->g.N + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(f->ci, in[p].ci, f->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(f->val, in[p].val, f->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    pool.run(B, [&](int p) { pr[p].ps->scr.reserve(fs[p]->g.N); });
    // several problems: what their solves over all of them need is kept as the levels go
    std::shared_ptr<BatchSolve> bs;
    if (batch) {
        bs = std::make_shared<BatchSolve>();
        bs->fs = fs;
        bs->base.resize(Lmax + 1);
        for (int p = 0; p < B; ++p) {
            fs[p]->bsolve = bs;
            fs[p]->bidx = p;
        }
    }

    const bool timing = (o.flags & RHIF_FLAG_PHASE_TIMES) != 0;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto phase = [&](int idx, std::chrono::steady_clock::time_point t0) {
        if (!timing) return;
        HIPCHK(hipStreamSynchronize(s));
        const double ms = std::chrono::duration<double, std::milli>(now() - t0).count();
        for (rhif_factor_s* f : fs) f->stats.t_phase_ms[idx] += ms;
    };

    // The skeleton apply tables of a problem's level lv (ranks and pivots known): descriptors
    // and the fused per-group apply table, on the host. Nothing of the next level depends on
    // them, so they are built while the next level's first kernels run.
    auto skel_tables_host = [&](Prob& q) {
        const int lv = q.pending_skel;
        rhif_factor_s* f = q.f;
        PlanSet& ps = *q.ps;
        LevelDev& LD = f->lev[lv];
        const LevelPlan& P = ps.plan(lv);
        const int nsk = static_cast<int>(LD.k.size());
        double fl = 0.0, sby = 0.0;
        skel_apply_tables(P, LD.k.data(), LD.perm.data(), kApplyCap, ps.sk_ad, ps.sk_dofs, f->ws_elems, fl, sby);
        validate_skel_apply(P, ps.sk_ad, ps.sk_dofs, f->g.N);
        LD.b_skel = sby;
        f->stats.flops[lv] += fl;
        q.sk_fl = fl;
        // per separator group: gather, block Jacobi and skeleton elimination in one launch
        std::vector<GroupApplyDesc>& gad = ps.gad;
        gad.assign(P.sep_desc.size(), GroupApplyDesc{});
        LD.mn_grp = 0;
        LD.tk_cap = 0;
        std::vector<int32_t>& skel_of = ps.skel_of;
        skel_of.assign(P.gptr.size(), -1);
        for (int e = 0; e < nsk; ++e) skel_of[P.skels[e]] = e;
        for (size_t e = 0; e < P.sep_desc.size(); ++e) {
            const SepDesc& sd = P.sep_desc[e];
            const GatherDesc& gt = P.gather[e];
            GroupApplyDesc& x = gad[e];
            x.n = sd.n;
            x.dofs = sd.dofs;
            x.nslot = gt.nslot;
            for (int sl = 0; sl < gt.nslot; ++sl) x.yoff[sl] = gt.yoff[sl];
            x.precond = LD.precond ? 1 : 0;
            x.loff = sd.loff;
            x.li = sd.lioff;
            const int se = skel_of[P.seps[e]];
            if (se >= 0) {
                const SkelDesc& sk = P.skel_desc[se];
                const int kk = LD.k[sk.gid];
                if (kk < sk.n) {
                    x.nr = sk.n - kk;
                    x.k = kk;
                    x.poff = sk.poff;
                    x.goff = sk.goff;
                    x.toff = sk.toff;
                    x.skli = sk.lioff;
                }
            }
            LD.mn_grp = std::max(LD.mn_grp, sd.n);
            LD.tk_cap = std::max(LD.tk_cap, x.k * x.nr);
        }
        LD.n_grp = static_cast<int>(gad.size());
        // T and G's off-diagonal block of a group go through LDS when the largest fit
        LD.tk_raw = LD.tk_cap;
        if (2 * LD.tk_cap > kGroupStageMax) LD.tk_cap = 0;
        if (bs) {
            LD.h_skel_ad = ps.sk_ad;
            LD.h_gad = gad;
        }
        LD.n_skel_ad = static_cast<int>(ps.sk_ad.size());
        LD.lds_skel = apply_lds(ps.sk_ad);
        apply_max(ps.sk_ad, LD.mi_skel, LD.mb_skel);
    };
    // ... and their upload, one copy for all problems with tables pending
    std::vector<int> skel_rec(Lmax + 1, -1);   // per level: its (last) skeletonization timing record
    auto skel_tables_upload = [&](const std::vector<int>& which) {
        if (which.empty()) return;
        const int lv = pr[which[0]].pending_skel;   // every problem waiting has the same level
        Packer pk;
        std::vector<std::array<size_t, 4>> off(which.size());
        double fl = 0.0;
        for (size_t i = 0; i < which.size(); ++i) {
            Prob& q = pr[which[i]];
            PlanSet& ps = *q.ps;
            off[i] = {pk.add(ps.sk_ad), pk.add(ps.sk_dofs), pk.add(ps.gad), pk.add(q.f->lev[q.pending_skel].perm)};
            fl += q.sk_fl;
        }
        char* T = upload_side(f0, pk, s, false);
        side_guard.armed = side_guard.armed || T != nullptr;
        for (size_t i = 0; i < which.size(); ++i) {
            Prob& q = pr[which[i]];
            LevelDev& LD = q.f->lev[q.pending_skel];
            if (T) {
                LD.skel_ad = view<ApplyDesc>(T, off[i][0]);
                LD.skeldofs = view<int32_t>(T, off[i][1]);
                LD.grp_ad = view<GroupApplyDesc>(T, off[i][2]);
                LD.permd = view<int32_t>(T, off[i][3]);
                LD.o_skeldofs = static_cast<int64_t>(off[i][1] / sizeof(int32_t));
                LD.o_perm = static_cast<int64_t>(off[i][3] / sizeof(int32_t));
            }
            if (bs) {
                BatchLevelBase& b = bs->base[q.pending_skel];
                b.skeldofs = b.perm = reinterpret_cast<int32_t*>(T);
            }
            q.pending_skel = -1;
        }
        // the level's skeletonization launch gets its algorithmic flops now that they are known
        if (f0->ktimes && skel_rec[lv] >= 0) f0->pend[skel_rec[lv]].fl = fl;
    };

    std::vector<int> act, nonroot, pend;
    for (int lvl = 0; lvl <= Lmax; ++lvl) {
        act.clear();
        for (int p = 0; p < B; ++p)
            if (lvl <= fs[p]->L) act.push_back(p);
        const int na = static_cast<int>(act.size());

        // ---- plan the cell half of every problem ----
        auto t0 = now();
        // the largest per-unknown table is built by the device: at level 0 the cells' frontal
        // unknowns (closed form; the host fills the groups' lists while the first kernels
        // run), above it the extend-add sources
        pool.run(na, [&](int i) {
            Prob& q = pr[act[i]];
            rhif_factor_s* f = q.f;
            PlanSet& ps = *q.ps;
            LevelPlan& P = ps.plan(lvl);
            const LevelPlan* prevP = lvl > 0 ? &ps.plan(lvl - 1) : nullptr;
            q.reuse0 = lvl == 0 && ps.plan0_ok && ps.plan0_key[0] == d && ps.plan0_key[1] == f->g.s &&
                       ps.plan0_key[2] == leaf;
            if (lvl == 0 && !q.reuse0) ps.plan0_ok = false;
            if (!q.reuse0) {
                build_cells(f->g, lvl, leaf, lvl == f->L, q.n_active, prevP, ps.scr, kApplyCap, P, true);
                validate_cells(P, prevP, d);
            }
            if (P.max_nf > 16 * kPotrfMaxTiles) fail(RHIF_ENOMEM, "a frontal matrix is too large for this version");
        });

        // ---- the problems' shares of the level-wide arrays; merged cell tables ----
        int64_t n_front = 0, n_ext = 0;
        int32_t n_cell = 0;
        mt.cref.clear();
        mt.pot[0].clear();
        mt.pot[1].clear();
        double alg_elim[2] = {0.0, 0.0};
        for (int p : act) {
            Prob& q = pr[p];
            rhif_factor_s* f = q.f;
            const LevelPlan& P = q.ps->plan(lvl);
            LevelDev& LD = f->lev[lvl];
            const int kind = lvl == f->L ? 1 : 0;
            LD.root = kind == 1;
            LD.precond = o.precond != 0;
            f->stats.n_active[lvl] = q.n_active;
            f->stats.n_cells[lvl] = P.ncells;
            f->stats.max_front[lvl] = P.max_nf;
            q.o_front = n_front;
            q.o_ext = n_ext;
            q.o_cell = n_cell;
            for (CellRef c : P.cell_ref) {
                c.off += q.o_front;
                mt.cref.push_back(c);
            }
            for (FrontDesc fd : P.cell_potrf) {
                fd.off += q.o_front;
                if (fd.ext >= 0) fd.ext += static_cast<int32_t>(q.o_ext);
                mt.pot[kind].push_back(fd);
            }
            alg_elim[kind] += P.alg_elim_flops;
            n_front += P.front_elems;
            n_ext += P.ext_elems;
            n_cell += P.ncells;
        }
        if (n_ext >= (int64_t(1) << 31)) fail(RHIF_ENOMEM, "too many cells in one level of the call");
        double* front = static_cast<double*>(f0->dalloc(std::max<int64_t>(n_front, 1) * sizeof(double)));
        int32_t* ext = static_cast<int32_t*>(f0->dalloc(std::max<int64_t>(n_ext, 1) * sizeof(int32_t)));
        // ---- upload: every problem's cell tables and the merged ones, one copy ----
        const rhif::CellRef* cref_all = nullptr;
        const rhif::FrontDesc* pot_dev[2] = {nullptr, nullptr};
        {
            Packer pk;
            std::vector<std::array<size_t, 7>> off(na);
            for (int i = 0; i < na; ++i) {
                const LevelPlan& P = pr[act[i]].ps->plan(lvl);
                off[i] = {pk.add(P.c_dofs), pk.add(P.cell_ref), pk.add(P.tiles), pk.add(P.src),
                          pk.add(P.cell_apply), pk.add(P.c_g2), pk.add(P.c_t2)};
            }
            const size_t o_cref = pk.add(mt.cref), o_pot0 = pk.add(mt.pot[0]), o_pot1 = pk.add(mt.pot[1]);
            // the frontal unknowns the device writes go after the tables, in the same buffer
            const size_t tail = (pk.total + 255) / 256 * 256;
            std::vector<size_t> o_dev(na, 0);
            size_t extra = tail - pk.total;
            for (int i = 0; i < na; ++i) {
                const LevelPlan& P = pr[act[i]].ps->plan(lvl);
                if (!P.dofs_on_device) continue;
                o_dev[i] = pk.total + extra;
                extra += static_cast<size_t>(std::max<int64_t>(P.c_dptr[P.ncells], 1)) * sizeof(int32_t);
            }
            char* T = upload(f0, pk, s, extra);
            if (bs) {
                BatchLevelBase& b = bs->base[lvl];
                b.front = front;
                b.ext = ext;
                b.cdofs = reinterpret_cast<int32_t*>(T);
            }
            cref_all = view<CellRef>(T, o_cref);
            pot_dev[0] = view<FrontDesc>(T, o_pot0);
            pot_dev[1] = view<FrontDesc>(T, o_pot1);
            for (int i = 0; i < na; ++i) {
                Prob& q = pr[act[i]];
                rhif_factor_s* f = q.f;
                const LevelPlan& P = q.ps->plan(lvl);
                LevelDev& LD = f->lev[lvl];
                LD.cg2 = view<int32_t>(T, off[i][5]);
                LD.ct2 = view<int32_t>(T, off[i][6]);
                const size_t o_cd = P.dofs_on_device ? o_dev[i] : off[i][0];
                LD.cdofs = view<int32_t>(T, o_cd);
                LD.o_cdofs = static_cast<int64_t>(o_cd / sizeof(int32_t));
                LD.cref = view<CellRef>(T, off[i][1]);
                LD.tiles = view<Tile>(T, off[i][2]);
                LD.src = P.src_on_device ? static_cast<int32_t*>(f0->dalloc(
                                               std::max<int64_t>(P.c_dptr[P.ncells], 1) * 2 * W * sizeof(int32_t)))
                                         : view<int32_t>(T, off[i][3]);
                LD.cell_ad = view<ApplyDesc>(T, off[i][4]);
                LD.n_cell_ad = static_cast<int>(P.cell_apply.size());
                LD.lds_cell = apply_lds(P.cell_apply);
                apply_max(P.cell_apply, LD.mi_cell, LD.mb_cell);
                LD.b_cell = P.alg_apply_cell_bytes;
                LD.front = front + q.o_front;
                LD.ext = ext + q.o_ext;
                LD.o_front = q.o_front;
                LD.o_ext = q.o_ext;
                LD.bytes = P.front_elems * 8 + P.ext_elems * 4;
                if (bs) LD.h_cell_ad = P.cell_apply;
                f->y_elems = std::max(f->y_elems, P.y_elems);
                f->ws_elems = std::max(f->ws_elems, P.ws_elems);
            }
        }
        phase(5, t0);

        // ---- frontal assembly, per problem ----
        t0 = now();
        for (int p : act) {
            rhif_factor_s* f = pr[p].f;
            const GridInfo& g = f->g;
            const LevelPlan& P = pr[p].ps->plan(lvl);
            const LevelPlan* prevP = lvl > 0 ? &pr[p].ps->plan(lvl - 1) : nullptr;
            LevelDev& LD = f->lev[lvl];
            const LevelDev* prev = lvl > 0 ? &f->lev[lvl - 1] : nullptr;
            if (P.dofs_on_device && P.ncells > 0)
                KTIMED(f0, s, RHIF_K_FRONT_CSR, 0.0, 4.0 * P.c_dptr[P.ncells],
                       hipLaunchKernelGGL(k_leaf_dofs, dim3(P.ncells), dim3(256), 0, s, LD.cref, d, g.s, P.w, P.nc1,
                                          LD.cdofs));
            if (P.tiles.empty()) continue;
            if (lvl == 0) {
                const double by = P.alg_front_bytes + 12.0 * f->nnz + 4.0 * (g.N + 1);
                KTIMED(f0, s, RHIF_K_FRONT_CSR, 0.0, by,
                       hipLaunchKernelGGL(k_front_csr, dim3(P.tiles.size()), dim3(256), 0, s, LD.tiles, LD.cref,
                                          LD.cdofs, d, g.s, P.w, P.nc1, f->rp, f->ci, f->val, LD.front));
            } else {
                if (P.src_on_device)
                    KTIMED(f0, s, RHIF_K_FRONT_EXTEND, 0.0, 4.0 * (2.0 + 2.0 * W) * P.c_dptr[P.ncells],
                           hipLaunchKernelGGL(k_extend_src, dim3(P.ncells), dim3(256), 0, s, LD.cref, LD.cg2, LD.ct2,
                                              static_cast<int>(prevP->gptr.size()) - 1, prev->gslot_cnt,
                                              prev->gslot_cell, prev->gslot_off, prev->cref, prevP->ncells, d,
                                              prevP->nc1, P.nc1, W, lvl, LD.src, err));
                double rd = 0.0;
                for (int c = 0; c < prevP->ncells; ++c)
                    rd += 8.0 * static_cast<double>(prevP->c_nB[c]) * prevP->c_nB[c];
                KTIMED(f0, s, RHIF_K_FRONT_EXTEND, 0.0, P.alg_front_bytes + rd,
                       hipLaunchKernelGGL(k_front_extend, dim3(P.tiles.size()), dim3(256), 0, s, LD.tiles, LD.cref,
                                          LD.src, W, d, prevP->nc1, prev->cref, prev->front, LD.front));
            }
        }
        phase(0, t0);

        // ---- cell elimination (E_l; at a problem's root: B_L = chol(A_L)), one launch
        //      sequence for the cells below the root and one for the roots ----
        double* linv = nullptr;
        if (!mt.pot[0].empty() || !mt.pot[1].empty()) {
            linv = static_cast<double*>(f0->dalloc(std::max<int64_t>(n_ext, 1) * 256 * sizeof(double)));
            for (int p : act) pr[p].f->lev[lvl].linv = linv + 256 * pr[p].o_ext;
            if (bs) bs->base[lvl].linv = linv;
        }
        for (int kind = 0; kind < 2; ++kind) {
            const std::vector<FrontDesc>& pot = mt.pot[kind];
            if (pot.empty()) continue;
            t0 = now();
            const bool root = kind == 1;
            const FrontDesc* potd = pot_dev[kind];
            int nmax = 0, pmax = 0, mmax = 0;
            for (const auto& fd : pot) {
                nmax = std::max(nmax, fd.n - std::min(fd.n, 1));
                pmax = std::max(pmax, fd.p);
                mmax = std::max(mmax, fd.n - fd.p);
            }
            const int cls = root ? RHIF_K_ROOT : (lvl == 0 ? RHIF_K_ELIM_LEAF : RHIF_K_ELIM_UPPER);
            const unsigned ncell = static_cast<unsigned>(pot.size());
            const int w = leaf << lvl;
            // the frontal tiles of such cells skip what the banded elimination never reads
            if (leaf_interior_banded(d, lvl, root, w)) {
                // leaf interiors: block-bidiagonal Cholesky factors
                for (int p : act)
                    if ((lvl == pr[p].f->L) == root) pr[p].f->lev[lvl].leaf_banded = true;
                const int nt = (mmax + 15) / 16;
                const int tpw = (nt + 3) / 4;
                const size_t lds0 =
                    static_cast<size_t>((10 + 4 * std::max(tpw, 1) + 2 * (2 + nt)) * 16 * 17) * sizeof(double);
                KTIMED(f0, s, cls, alg_elim[kind], 0.0,
                       hipLaunchKernelGGL(f32schur ? k_leaf_elim<true> : k_leaf_elim<false>, dim3(ncell), dim3(256),
                                          lds0, s, potd, front, linv, std::max(tpw, 1), lvl, err, ext));
            } else if (pmax > kCholLdsPmax) {
                // large interiors (3D upper levels, roots): panel by panel, each panel's
                // Cholesky, row solves and trailing update as three launches over all cells
                const int nq = (pmax + kElimPanel - 1) / kElimPanel;
                std::vector<rhif::FrontDesc> pd;
                std::vector<int32_t> pd_off(nq + 1, 0), pd_mrow(nq, 0);
                std::vector<int32_t> ext_all(std::max<int64_t>(n_ext, 1), 0);
                for (int q = 0; q < nq; ++q) {
                    const int j0 = q * kElimPanel;
                    for (const auto& fd : pot) {
                        if (fd.p <= j0) continue;
                        rhif::FrontDesc e = fd;
                        e.off = fd.off + j0 + static_cast<int64_t>(j0) * fd.ld;
                        e.n = fd.n - j0;
                        e.p = std::min(kElimPanel, fd.p - j0);
                        e.ext = fd.ext + j0 / 16;
                        pd.push_back(e);
                        pd_mrow[q] = std::max(pd_mrow[q], e.n - e.p);
                    }
                    pd_off[q + 1] = static_cast<int32_t>(pd.size());
                }
                // the apply's row extents of L: every panel column block runs to the interior's end
                for (const auto& fd : pot)
                    for (int t = 0; t < (fd.p + 15) / 16; ++t) ext_all[fd.ext + t] = fd.p;
                Packer pk;
                const size_t o_pd = pk.add(pd), o_ea = pk.add(ext_all);
                char* T = upload(f0, pk, s);
                // only the shares of this sequence's problems (the other sequence's kernels
                // write their own)
                for (int p : act) {
                    const Prob& q = pr[p];
                    const int64_t ne = q.ps->plan(lvl).ext_elems;
                    if ((lvl == q.f->L) != root || ne == 0) continue;
                    HIPCHK(hipMemcpyAsync(ext + q.o_ext, T + o_ea + q.o_ext * sizeof(int32_t),
                                          ne * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
                }
                const rhif::FrontDesc* pdd = view<rhif::FrontDesc>(T, o_pd);
                const size_t lds1 =
                    static_cast<size_t>(rhif::kPotrfSmemFixed + (kElimPanel | 1) * kElimPanel) * sizeof(double);
                const int pstride = 17 * kElimPanel;
                for (int q = 0; q < nq; ++q) {
                    const unsigned nc = static_cast<unsigned>(pd_off[q + 1] - pd_off[q]);
                    const rhif::FrontDesc* dq = pdd + pd_off[q];
                    KTIMED(f0, s, cls, q == 0 ? alg_elim[kind] : 0.0, 0.0,
                           hipLaunchKernelGGL(k_chol_lead, dim3(nc), dim3(256), lds1, s, dq, front, linv, kElimPanel,
                                              lvl, root ? 3 : 0, err, nullptr));
                    const int mr = pd_mrow[q];
                    if (mr > 0) {
                        KTIMED(f0, s, cls, 0.0, 0.0,
                               hipLaunchKernelGGL(k_trsm_rows, dim3(nc, (mr + 63) / 64), dim3(256),
                                                  static_cast<size_t>(4 * pstride) * sizeof(double), s, dq, front,
                                                  linv, pstride));
                        const int nb = (mr + kSyrkBlock - 1) / kSyrkBlock;
                        KTIMED(f0, s, cls, 0.0, 0.0,
                               hipLaunchKernelGGL(k_syrk_schur<false>, dim3(nc, nb * (nb + 1) / 2), dim3(256), 0, s,
                                                  dq, front));
                    }
                }
            } else if (!root && lvl > 0) {
                // small interiors: Cholesky, row solves and Schur update as three wide launches
                const size_t lds1 = static_cast<size_t>(rhif::kPotrfSmemFixed + (pmax | 1) * pmax) * sizeof(double);
                KTIMED(f0, s, cls, alg_elim[kind], 0.0,
                       hipLaunchKernelGGL(k_chol_lead, dim3(ncell), dim3(256), lds1, s, potd, front, linv,
                                          kCholLdsPmax, lvl, 0, err, ext));
                if (mmax > 0) {
                    const int pstride = 17 * ((pmax + 15) / 16) * 16;
                    KTIMED(f0, s, cls, 0.0, 0.0,
                           hipLaunchKernelGGL(k_trsm_rows, dim3(ncell, (mmax + 63) / 64), dim3(256),
                                              static_cast<size_t>(4 * pstride) * sizeof(double), s, potd, front, linv,
                                              pstride));
                    const int nb = (mmax + kSyrkBlock - 1) / kSyrkBlock;
                    KTIMED(f0, s, cls, 0.0, 0.0,
                           hipLaunchKernelGGL(f32schur ? k_syrk_schur<true> : k_syrk_schur<false>,
                                              dim3(ncell, nb * (nb + 1) / 2), dim3(256), 0, s, potd, front));
                }
            } else {
                const int cap = panel_cap_for(nmax, 0);
                KTIMED(f0, s, cls, alg_elim[kind], 0.0,
                       hipLaunchKernelGGL(k_potrf_batch, dim3(ncell), dim3(256), potrf_lds(cap, 0), s, potd, front,
                                          cap, lvl, root ? 3 : 0, err, ext, linv));
            }
            phase(root ? 6 : 1, t0);
        }

        // ---- host, overlapping the elimination: the leaf groups' lists and the separator
        //      half of this level's plans ----
        t0 = now();
        nonroot.clear();
        pend.clear();
        for (int p : act) {
            if (lvl < pr[p].f->L) nonroot.push_back(p);
            if (pr[p].pending_skel >= 0) pend.push_back(p);
        }
        pool.run(na, [&](int i) {
            Prob& q = pr[act[i]];
            rhif_factor_s* f = q.f;
            PlanSet& ps = *q.ps;
            LevelPlan& P = ps.plan(lvl);
            if (P.lists_pending) fill_leaf_lists(f->g, ps.scr, P);
            if (lvl == f->L) return;
            if (!q.reuse0) {
                build_separators(f->g, ps.scr, kApplyCap, P);
                validate_separators(P);
            }
            if (lvl == 0) {
                ps.plan0_ok = true;
                ps.plan0_key[0] = d;
                ps.plan0_key[1] = f->g.s;
                ps.plan0_key[2] = leaf;
            }
        });
        // the skeleton apply tables of the level below are needed by no kernel of this level:
        // they are built while this level's skeletonization runs
        auto finish_pending = [&] {
            pool.run(static_cast<int>(pend.size()), [&](int i) { skel_tables_host(pr[pend[i]]); });
            skel_tables_upload(pend);
        };
        for (int p : act)
            if (lvl == pr[p].f->L) pr[p].f->stats.flops[lvl] += pr[p].ps->plan(lvl).flops;
        if (nonroot.empty()) {
            finish_pending();
            continue;
        }

        // ---- the separator half: shares, merged tables, one upload ----
        int64_t n_lg = 0, n_t = 0, n_g = 0, n_li = 0, n_skli = 0, n_m = 0;
        int32_t n_cs = 0, n_cg = 0, n_k = 0, n_p = 0;
        int max_sep_n = 0, max_cell_groups = 0, max_skel_n = 0;
        double alg_pchol = 0.0, alg_pscale = 0.0;
        mt.sep.clear();
        mt.cg.clear();
        mt.cs.clear();
        mt.skd.clear();
        mt.cgl.clear();
        mt.cgoff.clear();
        mt.cgptr.clear();
        for (int p : act) {
            Prob& q = pr[p];
            const LevelPlan& P = q.ps->plan(lvl);
            const int32_t o_cgl = static_cast<int32_t>(mt.cgl.size());
            if (lvl == q.f->L) {
                // a root among the merged cells: no boundary groups
                for (int c = 0; c < P.ncells; ++c) mt.cgptr.push_back(o_cgl);
                continue;
            }
            q.f->stats.flops[lvl] += P.flops;
            q.o_lg = n_lg;
            q.o_t = n_t;
            q.o_g = n_g;
            q.o_li = n_li;
            q.o_skli = n_skli;
            q.o_m = n_m;
            q.o_cs = n_cs;
            q.o_cg = n_cg;
            q.o_k = n_k;
            q.o_p = n_p;
            for (SepDesc sd : P.sep_desc) {
                for (int sl = 0; sl < sd.nslot; ++sl) sd.slot_cell[sl] += q.o_cell;
                sd.loff += q.o_lg;
                sd.lioff += static_cast<int32_t>(q.o_li);
                mt.sep.push_back(sd);
            }
            for (CellGroup cg : P.cell_groups) {
                cg.loff += q.o_lg;
                cg.lioff += static_cast<int32_t>(q.o_li);
                cg.cell += q.o_cs;
                mt.cg.push_back(cg);
            }
            for (CellScaleDesc cs : P.cell_scale) {
                cs.off += q.o_front;
                cs.g_begin += q.o_cg;
                mt.cs.push_back(cs);
            }
            for (SkelDesc sk : P.skel_desc) {
                for (int sl = 0; sl < sk.nslot; ++sl) sk.cell[sl] += q.o_cell;
                sk.moff += q.o_m;
                sk.toff += q.o_t;
                sk.goff += q.o_g;
                sk.gid += q.o_k;
                sk.poff += q.o_p;
                sk.lioff += static_cast<int32_t>(q.o_skli);
                mt.skd.push_back(sk);
            }
            for (int c = 0; c < P.ncells; ++c) mt.cgptr.push_back(P.c_gptr[c] + o_cgl);
            mt.cgl.insert(mt.cgl.end(), P.c_g.begin(), P.c_g.end());
            mt.cgoff.insert(mt.cgoff.end(), P.c_goff.begin(), P.c_goff.end());
            n_lg += P.lg_elems;
            n_t += P.t_elems;
            n_g += P.g_elems;
            n_li += P.li_elems;
            n_skli += P.skli_elems;
            n_m += P.m_elems;
            n_cs += static_cast<int32_t>(P.cell_scale.size());
            n_cg += static_cast<int32_t>(P.cell_groups.size());
            n_k += static_cast<int32_t>(P.skel_desc.size());
            n_p += P.skel_ntotal;
            max_sep_n = std::max(max_sep_n, P.max_sep_n);
            max_cell_groups = std::max(max_cell_groups, P.max_cell_groups);
            max_skel_n = std::max(max_skel_n, P.max_skel_n);
            alg_pchol += P.alg_prec_chol_flops;
            alg_pscale += P.alg_prec_scale_flops;
        }
        mt.cgptr.push_back(static_cast<int32_t>(mt.cgl.size()));
        if (n_li >= (int64_t(1) << 31) || n_skli >= (int64_t(1) << 31))
            fail(RHIF_ENOMEM, "too many groups in one level of the call");
        const rhif::SepDesc* sep_all = nullptr;
        const rhif::CellGroup* cg_all = nullptr;
        const rhif::CellScaleDesc* cs_all = nullptr;
        const rhif::SkelDesc* skd_all = nullptr;
        const int32_t *cgptr_all = nullptr, *cgl_all = nullptr, *cgoff_all = nullptr;
        {
            Packer pk;
            const int nn = static_cast<int>(nonroot.size());
            std::vector<std::array<size_t, 6>> off(nn);
            for (int i = 0; i < nn; ++i) {
                const LevelPlan& P = pr[nonroot[i]].ps->plan(lvl);
                off[i] = {pk.add(P.sep_apply), pk.add(P.gather), pk.add(P.sep_dofs),
                          pk.add(P.gslot_cnt), pk.add(P.gslot_cell), pk.add(P.gslot_off)};
            }
            const size_t o_sep = pk.add(mt.sep), o_cg = pk.add(mt.cg), o_cs = pk.add(mt.cs), o_skd = pk.add(mt.skd),
                         o_cgp = pk.add(mt.cgptr), o_cgl = pk.add(mt.cgl), o_cgo = pk.add(mt.cgoff);
            char* T = upload_side(f0, pk, s);
            if (bs) bs->base[lvl].sepdofs = reinterpret_cast<int32_t*>(T);
            sep_all = view<SepDesc>(T, o_sep);
            cg_all = view<CellGroup>(T, o_cg);
            cs_all = view<CellScaleDesc>(T, o_cs);
            skd_all = view<SkelDesc>(T, o_skd);
            cgptr_all = view<int32_t>(T, o_cgp);
            cgl_all = view<int32_t>(T, o_cgl);
            cgoff_all = view<int32_t>(T, o_cgo);
            for (int i = 0; i < nn; ++i) {
                rhif_factor_s* f = pr[nonroot[i]].f;
                const LevelPlan& P = pr[nonroot[i]].ps->plan(lvl);
                LevelDev& LD = f->lev[lvl];
                LD.sep_ad = view<ApplyDesc>(T, off[i][0]);
                LD.gat = view<GatherDesc>(T, off[i][1]);
                LD.sepdofs = view<int32_t>(T, off[i][2]);
                LD.o_sepdofs = static_cast<int64_t>(off[i][2] / sizeof(int32_t));
                if (bs) {
                    LD.h_sep_ad = P.sep_apply;
                    LD.h_gat = P.gather;
                }
                LD.gslot_cnt = view<int32_t>(T, off[i][3]);
                LD.gslot_cell = view<int32_t>(T, off[i][4]);
                LD.gslot_off = view<int32_t>(T, off[i][5]);
                LD.n_sep_ad = static_cast<int>(P.sep_apply.size());
                int mb = 0;
                apply_max(P.sep_apply, LD.mi_sep, mb);
                LD.n_gather = static_cast<int>(P.gather.size());
                LD.lds_sep = apply_lds(P.sep_apply);
                LD.b_sep = P.alg_apply_sep_bytes;
                LD.b_gather = P.alg_gather_bytes;
                f->ws_elems = std::max(f->ws_elems, P.ws_elems);
            }
        }
        double* lg = static_cast<double*>(f0->dalloc(std::max<int64_t>(n_lg, 1) * sizeof(double)));
        double* tp = static_cast<double*>(f0->dalloc(std::max<int64_t>(n_t, 1) * sizeof(double)));
        double* gp = static_cast<double*>(f0->dalloc(std::max<int64_t>(n_g, 1) * sizeof(double)));
        for (int p : nonroot) {
            const Prob& q = pr[p];
            const LevelPlan& P = q.ps->plan(lvl);
            LevelDev& LD = q.f->lev[lvl];
            LD.lg = lg + q.o_lg;
            LD.tp = tp + q.o_t;
            LD.gp = gp + q.o_g;
            LD.o_lg = q.o_lg;
            LD.o_t = q.o_t;
            LD.o_g = q.o_g;
            LD.o_li = q.o_li;
            LD.o_skli = q.o_skli;
            LD.bytes += (P.lg_elems + P.t_elems + P.g_elems) * 8;
        }
        if (bs) {
            BatchLevelBase& b = bs->base[lvl];
            b.lg = lg;
            b.tp = tp;
            b.gp = gp;
        }
        if (n_m > mp_elems) {
            mp = static_cast<double*>(f0->dalloc(n_m * sizeof(double)));
            mp_elems = n_m;
        }
        const int nsk = static_cast<int>(mt.skd.size());
        const int64_t kp = static_cast<int64_t>(n_k) + n_p + 1;
        if (kp > kp_elems) {
            // a larger block: the error word so far moves along (stream-ordered after every
            // kernel that may have set it)
            int32_t* nb = static_cast<int32_t*>(f0->dalloc((kKbufHead + kp) * sizeof(int32_t)));
            HIPCHK(hipMemcpyAsync(nb, kbuf, sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
            kbuf = nb;
            err = reinterpret_cast<unsigned long long*>(nb);
            kp_elems = kp;
        }
        // ranks, then the pivot orders, right after the error word
        int32_t* kout = kbuf + kKbufHead;
        int32_t* pout = kout + n_k;
        phase(5, t0);

        // ---- block Jacobi (C_l) ----
        t0 = now();
        const int nsep = static_cast<int>(mt.sep.size());
        if (o.precond && nsep > 0) {
            const int cap = panel_cap_for(max_sep_n, 0);
            double* li = static_cast<double*>(f0->dalloc(std::max<int64_t>(n_li, 1) * sizeof(double)));
            for (int p : nonroot) pr[p].f->lev[lvl].li = li + pr[p].o_li;
            if (bs) bs->base[lvl].li = li;
            // L_g is factored in LDS when the largest group fits
            const int nm = max_sep_n;
            const bool gstage = (o.flags & RHIF_FLAG_GLOBAL_STAGING) != 0;
            const bool staged = !gstage && rhif::kPotrfSmemFixed + nm * nm <= kLdsMaxDoubles - kStaticLdsReserve;
            const size_t lds_pg = staged ? static_cast<size_t>(rhif::kPotrfSmemFixed + nm * nm) * sizeof(double)
                                         : potrf_lds(cap, 0);
            if (nm <= kPrecondPanelMinN) {
                KTIMED(f0, s, RHIF_K_PRECOND_CHOL, alg_pchol, 0.0,
                       hipLaunchKernelGGL(k_precond_groups, dim3(nsep), dim3(256), lds_pg, s, sep_all, cref_all, front,
                                          lg, li, cap, staged ? nm : 0, lvl, err));
            } else {
                // large groups: A_gg gathered by many workgroups per group, L_g by the panel
                // kernels of the cell elimination (one launch per 128-column panel for all groups)
                KTIMED(f0, s, RHIF_K_PRECOND_CHOL, alg_pchol, 0.0,
                       hipLaunchKernelGGL(k_precond_gather, dim3(nsep, (nm + 15) / 16), dim3(256), 0, s, sep_all,
                                          cref_all, front, lg));
                const int nq = (nm + kElimPanel - 1) / kElimPanel;
                std::vector<rhif::FrontDesc> pd;
                std::vector<int32_t> pd_off(nq + 1, 0), pd_mrow(nq, 0);
                for (int q = 0; q < nq; ++q) {
                    const int j0 = q * kElimPanel;
                    for (int e = 0; e < nsep; ++e) {
                        const SepDesc& sd = mt.sep[e];
                        if (sd.n <= j0) continue;
                        rhif::FrontDesc fd{};
                        fd.off = sd.loff + j0 + static_cast<int64_t>(j0) * sd.n;
                        fd.ld = sd.n;
                        fd.n = sd.n - j0;
                        fd.p = std::min(kElimPanel, sd.n - j0);
                        fd.id = e;
                        fd.ext = sd.lioff / 256 + j0 / 16;
                        pd.push_back(fd);
                        pd_mrow[q] = std::max(pd_mrow[q], fd.n - fd.p);
                    }
                    pd_off[q + 1] = static_cast<int32_t>(pd.size());
                }
                Packer pk;
                const size_t o_pd = pk.add(pd);
                char* T = upload(f0, pk, s);
                const rhif::FrontDesc* pdd = view<rhif::FrontDesc>(T, o_pd);
                const size_t lds1 =
                    static_cast<size_t>(rhif::kPotrfSmemFixed + (kElimPanel | 1) * kElimPanel) * sizeof(double);
                const int pstride = 17 * kElimPanel;
                for (int q = 0; q < nq; ++q) {
                    const unsigned nc = static_cast<unsigned>(pd_off[q + 1] - pd_off[q]);
                    if (nc == 0) continue;
                    const rhif::FrontDesc* dq = pdd + pd_off[q];
                    KTIMED(f0, s, RHIF_K_PRECOND_CHOL, 0.0, 0.0,
                           hipLaunchKernelGGL(k_chol_lead, dim3(nc), dim3(256), lds1, s, dq, lg, li, kElimPanel, lvl,
                                              1, err, nullptr));
                    const int mr = pd_mrow[q];
                    if (mr > 0) {
                        KTIMED(f0, s, RHIF_K_PRECOND_CHOL, 0.0, 0.0,
                               hipLaunchKernelGGL(k_trsm_rows, dim3(nc, (mr + 63) / 64), dim3(256),
                                                  static_cast<size_t>(4 * pstride) * sizeof(double), s, dq, lg, li,
                                                  pstride));
                        const int nb = (mr + kSyrkBlock - 1) / kSyrkBlock;
                        KTIMED(f0, s, RHIF_K_PRECOND_CHOL, 0.0, 0.0,
                               hipLaunchKernelGGL(k_syrk_schur<false>, dim3(nc, nb * (nb + 1) / 2), dim3(256), 0, s,
                                                  dq, lg));
                    }
                }
            }
            if (!mt.cs.empty()) {
                // per wave a strip of finished panels in LDS, or (larger groups) one 16 x 17 tile
                int pstride = 17 * ((max_sep_n + 15) / 16) * 16;
                if (gstage || 4 * pstride > kLdsMaxDoubles) pstride = 0;
                const size_t lds_sc = static_cast<size_t>(pstride > 0 ? 4 * pstride : 4 * 16 * 17) * sizeof(double);
                const int gc = max_cell_groups;
                // large groups: each pair's strips over several workgroups, the two one-sided
                // solves as two launches
                const int nz = (max_sep_n + kScaleRowsPerWG - 1) / kScaleRowsPerWG;
                if (nz <= 1) {
                    KTIMED(f0, s, RHIF_K_PRECOND_SCALE, alg_pscale, 0.0,
                           hipLaunchKernelGGL(k_precond_scale, dim3(mt.cs.size(), gc * (gc + 1) / 2), dim3(256),
                                              lds_sc, s, cs_all, cg_all, lg, li, front, pstride, 0));
                } else {
                    for (int ph = 1; ph <= 2; ++ph)
                        KTIMED(f0, s, RHIF_K_PRECOND_SCALE, ph == 1 ? alg_pscale : 0.0, 0.0,
                               hipLaunchKernelGGL(k_precond_scale, dim3(mt.cs.size(), gc * (gc + 1) / 2, nz),
                                                  dim3(256), lds_sc, s, cs_all, cg_all, lg, li, front, pstride, ph));
                }
            }
        }
        for (int p : nonroot)
            pr[p].f->stats.n_groups[lvl] =
                o.precond ? static_cast<int32_t>(pr[p].ps->plan(lvl).sep_desc.size()) : 0;
        phase(2, t0);

        // ---- skeletonization (K_l) ----
        t0 = now();
        int32_t* hk = nullptr;
        int32_t* hp = nullptr;
        if (nsk > 0) {
            const int n = max_skel_n;
            int rmax = 1;
            for (const auto& sk : mt.skd) rmax = std::max(rmax, sk.r);
            // must match the LDS layout of k_skeletonize
            const int base = (2 * n + 1) / 2 + 1 + rmax + 2 * 256 * std::max(1, (n + 63) / 64) + rhif::kCpqrRegExtra;
            // M in doubles of LDS (FP32 values take half)
            const int msz = f32 ? (rmax * (n | 1) + 1) / 2 : rmax * (n | 1);
            const int full = kPotrfSmemFixed + 17 * n;        // potrf scratch with the whole panel
            int staged = 0, cap = 0;
            size_t lds = 0;
            if (o.flags & RHIF_FLAG_GLOBAL_STAGING) {
                cap = panel_cap_for(n, base);
                lds = potrf_lds(cap, base);
            } else if (base + msz + n * n + full <= kLdsMaxDoubles) {
                staged = 3;
                cap = n;
                lds = static_cast<size_t>(base + msz + n * n + full) * sizeof(double);
                // far more groups than the 256 CUs hold at two per CU: the form that keeps more
                // of them resident per CU, when their LDS allows it and every group's ID fits
                // its registers (so that each group takes the same ID code in any form)
                if (nsk > 2 * 256 && kSkelWavesMany * lds <= kLdsMaxDoubles * sizeof(double) &&
                    skel_rows_per_thread(mt.skd) <= 16)
                    staged = 4;
            } else if (base + msz + kPotrfSmemFixed <= kLdsMaxDoubles) {
                staged = 1;
                cap = std::min(n, (kLdsMaxDoubles - base - msz - kPotrfSmemFixed) / 17);
                lds = static_cast<size_t>(base + msz + kPotrfSmemFixed + 17 * cap) * sizeof(double);
            } else {
                cap = panel_cap_for(n, base);
                lds = potrf_lds(cap, base);
            }
            double* skli = static_cast<double*>(f0->dalloc(std::max<int64_t>(n_skli, 1) * sizeof(double)));
            for (int p : nonroot) pr[p].f->lev[lvl].skli = skli + pr[p].o_skli;
            if (bs) bs->base[lvl].skli = skli;
            // groups whose M is too large for LDS and has many rows (the upper 3D levels): the
            // ID spread over row blocks of kBigRowsHost rows, one launch per step for all groups
            const bool big = (o.flags & RHIF_FLAG_SKEL_MULTI) ||
                             (staged == 0 && !(o.flags & RHIF_FLAG_GLOBAL_STAGING) &&
                              static_cast<int64_t>(rmax) * n >= kBigSkelElems);
            if (big) {
                const int nblk = (rmax + kBigRowsHost - 1) / kBigRowsHost;
                double* nrm = static_cast<double*>(f0->dalloc(static_cast<size_t>(nsk) * nblk * n * sizeof(double)));
                double* wpart = static_cast<double*>(f0->dalloc(static_cast<size_t>(nsk) * nblk * n * sizeof(double)));
                int32_t* posb = static_cast<int32_t*>(f0->dalloc(static_cast<size_t>(nsk) * n * sizeof(int32_t)));
                BigState* bst = static_cast<BigState*>(f0->dalloc(static_cast<size_t>(nsk) * sizeof(BigState)));
                double* csum = static_cast<double*>(f0->dalloc(static_cast<size_t>(nsk) * n * sizeof(double)));
                int jmax = 0;
                for (const auto& sk : mt.skd) jmax = std::max(jmax, std::min(sk.r, sk.n));
                const dim3 gb2(nsk, nblk), gcs(nsk, (n + 255) / 256);
                auto colsum = [&](const double* part) {
                    KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                           hipLaunchKernelGGL(f32 ? k_big_colsum<float> : k_big_colsum<double>, gcs, dim3(256), 0, s,
                                              skd_all, bst, part, csum, n, nblk));
                };
                KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                       hipLaunchKernelGGL(f32 ? k_big_gather<float> : k_big_gather<double>, gb2, dim3(256), 0, s,
                                          skd_all, cgptr_all, cgl_all, cgoff_all, cref_all, front, mp, nrm, posb,
                                          pout, bst, n, nblk, lvl, err));
                colsum(nrm);
                BigState* hst = reinterpret_cast<BigState*>(hc.get_down(static_cast<size_t>(nsk) * sizeof(BigState) + 64));
                // every group takes at most jmax steps (the last one only records the rank); the
                // host checks every kBigCheck steps whether any group is still active
                for (int j = 0; j <= jmax; ++j) {
                    KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                           hipLaunchKernelGGL(f32 ? k_big_pivot<float> : k_big_pivot<double>, dim3(nsk), dim3(256), 0,
                                              s, skd_all, mp, csum, posb, pout, bst, o.eps, j, n, kout));
                    if (j == jmax) break;
                    KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                           hipLaunchKernelGGL(f32 ? k_big_dot<float> : k_big_dot<double>, gb2, dim3(256), 0, s,
                                              skd_all, mp, posb, bst, wpart, j, n, nblk));
                    colsum(wpart);
                    KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                           hipLaunchKernelGGL(f32 ? k_big_update<float> : k_big_update<double>, gb2, dim3(256), 0, s,
                                              skd_all, mp, nrm, posb, bst, csum, j, n, nblk));
                    colsum(nrm);
                    if ((j + 1) % kBigCheck == 0) {
                        HIPCHK(hipMemcpyAsync(hst, bst, static_cast<size_t>(nsk) * sizeof(BigState),
                                              hipMemcpyDeviceToHost, s));
                        hc.wait(s, f0->device);
                        bool any = false;
                        for (int e = 0; e < nsk; ++e) any = any || hst[e].active;
                        if (!any) break;
                    }
                }
                // a group still active after jmax steps took every column: its rank is set by
                // the last pivot launch (j == min(r, n))
                // the ranks to the host: they size the substitution's LDS and the tables of the
                // skeleton eliminations
                int32_t* hkk = reinterpret_cast<int32_t*>(hc.get_down(static_cast<size_t>(n_k) * sizeof(int32_t) + 64));
                HIPCHK(hipMemcpyAsync(hkk, kout, static_cast<size_t>(n_k) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                hc.wait(s, f0->device);
                int nrmax = 0, kmax = 0;
                for (const auto& sk : mt.skd) {
                    nrmax = std::max(nrmax, sk.n - hkk[sk.gid]);
                    kmax = std::max(kmax, hkk[sk.gid]);
                }
                if (nrmax > 0 && kmax > 0) {
                    const size_t mrb = f32 ? sizeof(float) : sizeof(double);
                    int ncol = kTrisolveColsHost;
                    while (ncol > 1 && ncol * kmax * mrb > kLdsMaxDoubles * sizeof(double)) --ncol;
                    if (kmax * mrb > kLdsMaxDoubles * sizeof(double))
                        fail(RHIF_ENOMEM, "a skeleton rank is too large for this version");
                    KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                           hipLaunchKernelGGL(f32 ? k_big_trisolve<float> : k_big_trisolve<double>,
                                              dim3(nsk, (nrmax + ncol - 1) / ncol), dim3(256), ncol * kmax * mrb, s,
                                              skd_all, mp, pout, bst, tp, ncol));
                }
                // the skeleton eliminations spread over many workgroups per group: G and its
                // zeroed blocks, the partial Cholesky of G by the panel kernels of the cell
                // elimination, the write-back
                const dim3 gcol(nsk, (n + 15) / 16);
                auto elim = [&](int ph) {
                    KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                           hipLaunchKernelGGL(f32 ? k_big_elim<float> : k_big_elim<double>, gcol, dim3(256), 0, s,
                                              skd_all, cref_all, front, mp, gp, kout, pout, ph));
                };
                for (int ph = 0; ph < 3; ++ph) elim(ph);
                const int nq = (nrmax + kElimPanel - 1) / kElimPanel;
                std::vector<rhif::FrontDesc> pd;
                std::vector<int32_t> pd_off(nq + 1, 0), pd_mrow(std::max(nq, 1), 0);
                for (int q = 0; q < nq; ++q) {
                    const int j0 = q * kElimPanel;
                    for (const auto& sk : mt.skd) {
                        const int nr = sk.n - hkk[sk.gid];
                        if (nr <= j0) continue;
                        rhif::FrontDesc e{};
                        e.off = sk.goff + j0 + static_cast<int64_t>(j0) * sk.n;
                        e.ld = sk.n;
                        e.n = sk.n - j0;
                        e.p = std::min(kElimPanel, nr - j0);
                        e.id = sk.gid;
                        e.ext = sk.lioff / 256 + j0 / 16;
                        pd.push_back(e);
                        pd_mrow[q] = std::max(pd_mrow[q], e.n - e.p);
                    }
                    pd_off[q + 1] = static_cast<int32_t>(pd.size());
                }
                if (!pd.empty()) {
                    Packer pk;
                    const size_t o_pd = pk.add(pd);
                    char* T = upload(f0, pk, s);
                    const rhif::FrontDesc* pdd = view<rhif::FrontDesc>(T, o_pd);
                    const size_t lds1 =
                        static_cast<size_t>(rhif::kPotrfSmemFixed + (kElimPanel | 1) * kElimPanel) * sizeof(double);
                    const int pstride = 17 * kElimPanel;
                    for (int q = 0; q < nq; ++q) {
                        const unsigned nc = static_cast<unsigned>(pd_off[q + 1] - pd_off[q]);
                        if (nc == 0) continue;
                        const rhif::FrontDesc* dq = pdd + pd_off[q];
                        KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                               hipLaunchKernelGGL(k_chol_lead, dim3(nc), dim3(256), lds1, s, dq, gp, skli, kElimPanel,
                                                  lvl, 2, err, nullptr));
                        const int mr = pd_mrow[q];
                        if (mr > 0) {
                            KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                                   hipLaunchKernelGGL(k_trsm_rows, dim3(nc, (mr + 63) / 64), dim3(256),
                                                      static_cast<size_t>(4 * pstride) * sizeof(double), s, dq, gp,
                                                      skli, pstride));
                            const int nb = (mr + kSyrkBlock - 1) / kSyrkBlock;
                            KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                                   hipLaunchKernelGGL(k_syrk_schur<false>, dim3(nc, nb * (nb + 1) / 2), dim3(256), 0,
                                                      s, dq, gp));
                        }
                    }
                }
                elim(3);
            } else {
                KTIMED(f0, s, RHIF_K_SKELETONIZE, 0.0, 0.0,
                       hipLaunchKernelGGL(skel_kernel(staged, skel_rows_per_thread(mt.skd), f32), dim3(nsk),
                                          dim3(256), lds, s, skd_all, cgptr_all, cgl_all, cgoff_all, cref_all, front,
                                          mp, tp, gp, skli, o.eps, kout, pout, cap, n, rmax, lvl, err));
            }
            if (f0->ktimes) skel_rec[lvl] = static_cast<int>(f0->pend.size()) - 1;
            finish_pending();
            // error word, ranks and pivot orders in one copy; synchronizes: the ranks are on
            // the host now
            const size_t nb = (kKbufHead + static_cast<size_t>(n_k) + static_cast<size_t>(n_p)) * sizeof(int32_t);
            char* h = hc.get_down(nb + 64);
            HIPCHK(hipMemcpyAsync(h, kbuf, nb, hipMemcpyDeviceToHost, s));
            hk = reinterpret_cast<int32_t*>(h) + kKbufHead;
            hp = hk + n_k;
            hc.wait(s, f0->device);
            unsigned long long e = 0;
            std::memcpy(&e, h, sizeof(e));
            raise_err(e, batch);
        } else {
            finish_pending();
            check_err(err, batch, s, f0->device);
        }
        phase(3, t0);

        // ---- every problem's next active unknowns; this level's skeleton apply tables are
        //      built after the next level's first launches ----
        t0 = now();
        for (int p : nonroot) {
            const Prob& q = pr[p];
            const LevelPlan& P = q.ps->plan(lvl);
            LevelDev& LD = q.f->lev[lvl];
            const int ns = static_cast<int>(P.skel_desc.size());
            if (ns > 0) {
                LD.k.assign(hk + q.o_k, hk + q.o_k + ns);
                LD.perm.assign(hp + q.o_p, hp + q.o_p + P.skel_ntotal);
            } else {
                LD.k.clear();
                LD.perm.clear();
            }
        }
        pool.run(static_cast<int>(nonroot.size()), [&](int i) {
            Prob& q = pr[nonroot[i]];
            rhif_factor_s* f = q.f;
            const LevelPlan& P = q.ps->plan(lvl);
            LevelDev& LD = f->lev[lvl];
            const int ns = static_cast<int>(LD.k.size());
            LD.first_dof.resize(ns);
            LD.gsize.resize(ns);
            int64_t sum_rank = 0;
            int max_rank = 0;
            for (int e = 0; e < ns; ++e) {
                const int gidx = P.skels[e];
                LD.first_dof[e] = P.gdofs[P.gptr[gidx]];
                LD.gsize[e] = P.gptr[gidx + 1] - P.gptr[gidx];
                sum_rank += LD.k[e];
                max_rank = std::max(max_rank, LD.k[e]);
            }
            f->stats.n_skel[lvl] = ns;
            f->stats.sum_skel_n[lvl] = P.skel_ntotal;
            f->stats.sum_rank[lvl] = sum_rank;
            f->stats.max_rank[lvl] = max_rank;
            q.n_active = next_active_set(P, LD.k.data(), LD.perm.data(), q.ps->scr);
            q.pending_skel = lvl;
        });
        phase(5, t0);
    }
    // every problem finished its last skeleton tables at its root level
    check_err(err, batch, s, f0->device);
    if (bs) {
        // the problems' apply scratch in two call-wide arrays, each problem's vector at its
        // place in the concatenated vectors of the solves over all of them
        int64_t ny = 0, nw = 0;
        bs->zoff.resize(B);
        for (int p = 0; p < B; ++p) {
            bs->zoff[p] = bs->ntot;
            bs->ntot += fs[p]->g.N;
            fs[p]->o_ybuf = ny;
            fs[p]->o_ws = nw;
            ny += std::max<int64_t>(fs[p]->y_elems, 1);
            nw += fs[p]->ws_elems;
        }
        bs->ybuf = static_cast<double*>(f0->dalloc(ny * sizeof(double)));
        bs->ws = nw > 0 ? static_cast<double*>(f0->dalloc(nw * sizeof(double))) : nullptr;
    }
    for (Prob& q : pr) {
        rhif_factor_s* f = q.f;
        f->stats.levels = f->L;
        f->stats.root_size = static_cast<int32_t>(q.n_active);
        f->stats.n_active[f->L] = q.n_active;
        if (bs) {
            f->ybuf = bs->ybuf + f->o_ybuf;
            if (f->ws_elems > 0) f->ws = bs->ws + f->o_ws;
        } else {
            f->ybuf = static_cast<double*>(f->dalloc(std::max<int64_t>(f->y_elems, 1) * sizeof(double)));
            if (f->ws_elems > 0) f->ws = static_cast<double*>(f->dalloc(f->ws_elems * sizeof(double)));
        }
        int64_t bytes = 0;
        for (const auto& LD : f->lev) bytes += LD.bytes;
        f->stats.factor_bytes = bytes;
    }
    if (side_guard.armed) hc.side_join(s, f0->device);
    hc.wait(s, f0->device);
    side_guard.armed = false;
    f0->resolve();
}

void launch_up(rhif_factor_s* f, double by, const rhif::ApplyDesc* ad, int n, size_t lds, const double* pool,
               const double* tp, const int32_t* dofs, double* z, double* ybuf, double* ws, hipStream_t s,
               const int32_t* ext = nullptr) {
    if (n <= 0) return;
    KTIMED(f, s, RHIF_K_APPLY_UP, 0.0, by,
           hipLaunchKernelGGL(rhif::k_apply_up, dim3(n), dim3(256), lds, s, ad, pool, tp, dofs, z, ybuf, ws, ext));
}

void launch_down(rhif_factor_s* f, double by, const rhif::ApplyDesc* ad, int n, size_t lds, const double* pool,
                 const double* tp, const int32_t* dofs, double* z, double* ws, hipStream_t s,
                 const int32_t* ext = nullptr) {
    if (n <= 0) return;
    KTIMED(f, s, RHIF_K_APPLY_DOWN, 0.0, by,
           hipLaunchKernelGGL(rhif::k_apply_down, dim3(n), dim3(256), lds, s, ad, pool, tp, dofs, z, ws, ext));
}

// Split apply (solve and product launches) when every block of the family has
// n_I <= kSplitApplyMaxI and the inverses of the diagonal blocks are there; else the
// fused kernels.
bool split_ok(int mi, int mb, const double* lip) {
    return lip != nullptr && mi <= rhif::kSplitApplyMaxI && 64 * 65 + mb + 256 <= kLdsMaxDoubles &&
           16 * ((mi + 15) / 16) + mb + (mi + 15) / 16 + 1 <= kLdsMaxDoubles;
}

size_t trsv_lds(int mi, int mb) {
    return static_cast<size_t>(16 * ((mi + 15) / 16) + mb + (mi + 15) / 32 + 1) * sizeof(double);
}

// The fused per-group kernels when every group fits the one-row-per-thread solves and the
// inverses of the diagonal blocks are there.
bool group_ok(const LevelDev& LD) {
    if (LD.n_grp <= 0 || LD.grp_ad == nullptr || LD.mn_grp > rhif::kSplitApplyMaxI) return false;
    if (LD.precond && LD.li == nullptr) return false;
    if (LD.n_skel_ad > 0 && LD.skli == nullptr) return false;
    return true;
}

size_t group_lds(const LevelDev& LD) {
    return static_cast<size_t>(2 * 16 * ((LD.mn_grp + 15) / 16) + 2 * LD.tk_cap) * sizeof(double);
}

// LDS of k_apply_band for interiors of up to mi unknowns.
size_t band_lds(int mi) {
    return static_cast<size_t>(16 * ((mi + 15) / 16) + 2 * 16 * 17 + 16) * sizeof(double);
}

// Families with an interior above kBigApplyMinI: panel by panel over many workgroups per
// block (their vectors staged in the workspace, which the planner gives every such block).
bool big_ok(int mi, const double* lip) { return lip != nullptr && mi > rhif::kBigApplyMinI; }

void big_up(rhif_factor_s* f, double by, const rhif::ApplyDesc* ad, int n, int mi, int mb, const double* pool,
            const double* lip, const double* tp, const int32_t* dofs, const int32_t* ext, double* z, double* ybuf,
            double* ws, hipStream_t s) {
    const int P = rhif::kBigApplyPanel;
    const int np = (mi + P - 1) / P;
    const dim3 grid(n, (mi + mb + P - 1) / P);
    auto launch = [&](int phase, int j, double b) {
        KTIMED(f, s, RHIF_K_APPLY_UP, 0.0, b,
               hipLaunchKernelGGL(rhif::k_apply_big_up, grid, dim3(256), 0, s, ad, phase, j, pool, lip, tp, dofs, ext,
                                  z, ybuf, ws));
    };
    launch(0, 0, by);
    if (tp != nullptr) launch(1, 0, 0.0);
    for (int j = 0; j <= np; ++j) launch(2, j, 0.0);
    launch(3, 0, 0.0);
}

void big_down(rhif_factor_s* f, double by, const rhif::ApplyDesc* ad, int n, int mi, int mb, const double* pool,
              const double* lip, const double* tp, const int32_t* dofs, const int32_t* ext, double* z, double* ws,
              hipStream_t s) {
    const int P = rhif::kBigApplyPanel;
    const int np = (mi + P - 1) / P;
    const dim3 grid(n, (mi + mb + P - 1) / P);
    auto launch = [&](int phase, int j, double b) {
        KTIMED(f, s, RHIF_K_APPLY_DOWN, 0.0, b,
               hipLaunchKernelGGL(rhif::k_apply_big_dn, grid, dim3(256), 0, s, ad, phase, j, pool, lip, tp, dofs, ext,
                                  z, ws));
    };
    launch(0, 0, by);
    launch(1, 0, 0.0);
    for (int j = np - 1; j >= 1; --j) launch(2, j, 0.0);
    launch(3, 0, 0.0);
}

void apply_up_block(rhif_factor_s* f, double by, const rhif::ApplyDesc* ad, int n, int mi, int mb, size_t lds,
                    const double* pool, const double* lip, const double* tp, const int32_t* dofs, double* z,
                    double* ybuf, hipStream_t s, const int32_t* ext = nullptr, bool band = false) {
    if (n <= 0) return;
    if (big_ok(mi, lip)) {
        big_up(f, by, ad, n, mi, mb, pool, lip, tp, dofs, ext, z, ybuf, f->ws, s);
        return;
    }
    if (!split_ok(mi, mb, lip)) {
        launch_up(f, by, ad, n, lds, pool, tp, dofs, z, ybuf, f->ws, s, ext);
        return;
    }
    if (band)
        KTIMED(f, s, RHIF_K_APPLY_UP, 0.0, by,
               hipLaunchKernelGGL(rhif::k_apply_band<true>, dim3(n), dim3(256), band_lds(mi), s, ad, pool, lip, dofs,
                                  z));
    else
        KTIMED(f, s, RHIF_K_APPLY_UP, 0.0, by,
               hipLaunchKernelGGL(rhif::k_apply_trsv_up, dim3(n), dim3(256), trsv_lds(mi, mb), s, ad, pool, lip, tp,
                                  dofs, z, ext));
    if (mb > 0)
        KTIMED(f, s, RHIF_K_APPLY_UP, 0.0, 0.0,
               hipLaunchKernelGGL(rhif::k_apply_gemv_up, dim3(n, (mb + 63) / 64), dim3(256),
                                  static_cast<size_t>(mi + 256) * sizeof(double), s, ad, pool, dofs, z, ybuf));
}

void apply_down_block(rhif_factor_s* f, double by, const rhif::ApplyDesc* ad, int n, int mi, int mb, size_t lds,
                      const double* pool, const double* lip, const double* tp, const int32_t* dofs, double* z,
                      hipStream_t s, const int32_t* ext = nullptr, bool band = false) {
    if (n <= 0) return;
    if (big_ok(mi, lip)) {
        big_down(f, by, ad, n, mi, mb, pool, lip, tp, dofs, ext, z, f->ws, s);
        return;
    }
    if (!split_ok(mi, mb, lip)) {
        launch_down(f, by, ad, n, lds, pool, tp, dofs, z, f->ws, s, ext);
        return;
    }
    if (mb > 0)
        KTIMED(f, s, RHIF_K_APPLY_DOWN, 0.0, by,
               hipLaunchKernelGGL(rhif::k_apply_gemv_dn, dim3(n, (mi + 63) / 64), dim3(256),
                                  static_cast<size_t>(64 * 65 + mb + 256) * sizeof(double), s, ad, pool, dofs, z));
    if (band)
        KTIMED(f, s, RHIF_K_APPLY_DOWN, 0.0, mb > 0 ? 0.0 : by,
               hipLaunchKernelGGL(rhif::k_apply_band<false>, dim3(n), dim3(256), band_lds(mi), s, ad, pool, lip, dofs,
                                  z));
    else
        KTIMED(f, s, RHIF_K_APPLY_DOWN, 0.0, mb > 0 ? 0.0 : by,
               hipLaunchKernelGGL(rhif::k_apply_trsv_dn, dim3(n), dim3(256), trsv_lds(mi, mb), s, ad, pool, lip, tp,
                                  dofs, z, ext));
}

// z <- G^-1 z: the up-sweep of every level, then the forward solve with the root factor.
void do_apply_up(rhif_factor_s* f, double* z, hipStream_t s) {
    const int L = f->L;
    for (int lvl = 0; lvl < L; ++lvl) {
        LevelDev& LD = f->lev[lvl];
        apply_up_block(f, LD.b_cell, LD.cell_ad, LD.n_cell_ad, LD.mi_cell, LD.mb_cell, LD.lds_cell, LD.front, LD.linv,
                       nullptr, LD.cdofs, z, f->ybuf, s, LD.ext, LD.leaf_banded);
        if (group_ok(LD)) {
            KTIMED(f, s, RHIF_K_APPLY_GATHER, 0.0, LD.b_gather + LD.b_sep + LD.b_skel,
                   hipLaunchKernelGGL(rhif::k_apply_group_up, dim3(LD.n_grp), dim3(256), group_lds(LD), s, LD.grp_ad,
                                      LD.sepdofs, f->ybuf, z, LD.lg, LD.li, LD.gp, LD.tp, LD.skli, LD.permd,
                                      LD.tk_cap));
            continue;
        }
        if (LD.n_gather > 0)
            KTIMED(f, s, RHIF_K_APPLY_GATHER, 0.0, LD.b_gather,
                   hipLaunchKernelGGL(rhif::k_sep_gather, dim3(LD.n_gather), dim3(256), 0, s, LD.gat, LD.sepdofs,
                                      f->ybuf, z));
        if (LD.precond)
            apply_up_block(f, LD.b_sep, LD.sep_ad, LD.n_sep_ad, LD.mi_sep, 0, LD.lds_sep, LD.lg, LD.li, nullptr,
                           LD.sepdofs, z, nullptr, s);
        apply_up_block(f, LD.b_skel, LD.skel_ad, LD.n_skel_ad, LD.mi_skel, LD.mb_skel, LD.lds_skel, LD.gp, LD.skli,
                       LD.tp, LD.skeldofs, z, nullptr, s);
    }
    LevelDev& LD = f->lev[L];
    apply_up_block(f, LD.b_cell, LD.cell_ad, LD.n_cell_ad, LD.mi_cell, LD.mb_cell, LD.lds_cell, LD.front, LD.linv,
                   nullptr, LD.cdofs, z, f->ybuf, s, LD.ext);
}

// z <- G^-T z: the backward solve with the root factor, then the down-sweep of every level.
void do_apply_down(rhif_factor_s* f, double* z, hipStream_t s) {
    const int L = f->L;
    {
        LevelDev& LD = f->lev[L];
        apply_down_block(f, LD.b_cell, LD.cell_ad, LD.n_cell_ad, LD.mi_cell, LD.mb_cell, LD.lds_cell, LD.front,
                         LD.linv, nullptr, LD.cdofs, z, s, LD.ext);
    }
    for (int lvl = L - 1; lvl >= 0; --lvl) {
        LevelDev& LD = f->lev[lvl];
        if (group_ok(LD)) {
            KTIMED(f, s, RHIF_K_APPLY_GATHER, 0.0, LD.b_sep + LD.b_skel,
                   hipLaunchKernelGGL(rhif::k_apply_group_dn, dim3(LD.n_grp), dim3(256), group_lds(LD), s, LD.grp_ad,
                                      LD.sepdofs, z, LD.lg, LD.li, LD.gp, LD.tp, LD.skli, LD.permd, LD.tk_cap));
        } else {
            apply_down_block(f, LD.b_skel, LD.skel_ad, LD.n_skel_ad, LD.mi_skel, LD.mb_skel, LD.lds_skel, LD.gp,
                             LD.skli, LD.tp, LD.skeldofs, z, s);
            if (LD.precond)
                apply_down_block(f, LD.b_sep, LD.sep_ad, LD.n_sep_ad, LD.mi_sep, 0, LD.lds_sep, LD.lg, LD.li, nullptr,
                                 LD.sepdofs, z, s);
        }
        apply_down_block(f, LD.b_cell, LD.cell_ad, LD.n_cell_ad, LD.mi_cell, LD.mb_cell, LD.lds_cell, LD.front,
                         LD.linv, nullptr, LD.cdofs, z, s, LD.ext, LD.leaf_banded);
    }
}

// z <- F^-1 z = G^-T G^-1 z (eq. (3.2))
void do_apply_inplace(rhif_factor_s* f, double* z, hipStream_t s) {
    do_apply_up(f, z, s);
    do_apply_down(f, z, s);
}

// z <- F z = G G^T z (eq. (3.3)): G^T undoes the down-sweep (levels 0 .. L-1: E, C, K) and the
// backward root solve; G undoes the forward root solve and the up-sweep (levels L-1 .. 0: K, C,
// then E with the cells' boundary contributions gathered into the shared unknowns).
void do_forward_inplace(rhif_factor_s* f, double* z, hipStream_t s) {
    const int L = f->L;
    auto gt = [&](const rhif::ApplyDesc* ad, int n, const double* pool, const double* tp, const int32_t* dofs,
                  const int32_t* ext) {
        if (n > 0) hipLaunchKernelGGL(rhif::k_fwd_gt, dim3(n), dim3(256), 0, s, ad, pool, tp, dofs, ext, z);
    };
    auto gg = [&](const rhif::ApplyDesc* ad, int n, const double* pool, const double* tp, const int32_t* dofs,
                  const int32_t* ext) {
        if (n > 0) hipLaunchKernelGGL(rhif::k_fwd_g, dim3(n), dim3(256), 0, s, ad, pool, tp, dofs, ext, z, f->ybuf);
    };
    for (int lvl = 0; lvl < L; ++lvl) {
        const LevelDev& LD = f->lev[lvl];
        gt(LD.cell_ad, LD.n_cell_ad, LD.front, nullptr, LD.cdofs, LD.ext);
        if (LD.precond) gt(LD.sep_ad, LD.n_sep_ad, LD.lg, nullptr, LD.sepdofs, nullptr);
        gt(LD.skel_ad, LD.n_skel_ad, LD.gp, LD.tp, LD.skeldofs, nullptr);
    }
    const LevelDev& R = f->lev[L];
    gt(R.cell_ad, R.n_cell_ad, R.front, nullptr, R.cdofs, R.ext);
    gg(R.cell_ad, R.n_cell_ad, R.front, nullptr, R.cdofs, R.ext);
    for (int lvl = L - 1; lvl >= 0; --lvl) {
        const LevelDev& LD = f->lev[lvl];
        gg(LD.skel_ad, LD.n_skel_ad, LD.gp, LD.tp, LD.skeldofs, nullptr);
        if (LD.precond) gg(LD.sep_ad, LD.n_sep_ad, LD.lg, nullptr, LD.sepdofs, nullptr);
        gg(LD.cell_ad, LD.n_cell_ad, LD.front, nullptr, LD.cdofs, LD.ext);
        if (LD.n_gather > 0)
            hipLaunchKernelGGL(rhif::k_fwd_gather, dim3(LD.n_gather), dim3(256), 0, s, LD.gat, LD.sepdofs, f->ybuf, z);
    }
    HIPCHK(hipGetLastError());
}

// ||op||_2 of a symmetric operator by power iteration on op^2 from the unit vector along v0:
// the estimate sqrt(||op(op(v))||) after each normalized step, until it changes by at most rtol
// (relative) or after maxit steps. op(x, y) writes y = op x; uses f->p, f->q, f->r.
template <class Op>
double power_norm(rhif_factor_s* f, const double* v0, int maxit, double rtol, Op op, int* iters, hipStream_t s) {
    const int64_t N = f->g.N;
    const int gb = grid_for(N);
    double* v = f->p;
    double* w = f->q;
    double* hsc = f->hsc;
    auto norm2 = [&](const double* x) {
        hipLaunchKernelGGL(rhif::k_dot, dim3(gb), dim3(256), 0, s, N, x, x, f->part);
        hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(256), 0, s, f->part, gb, 3, f->sc, nullptr);
        HIPCHK(hipMemcpyAsync(hsc, f->sc, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return hsc[0];
    };
    const double n0 = norm2(v0);
    if (!(n0 > 0.0)) fail(RHIF_EINVAL, "start vector is zero");
    hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, s, N, v0, v);
    hipLaunchKernelGGL(rhif::k_axpby, dim3(gb), dim3(256), 0, s, N, 0.0, v, 1.0 / std::sqrt(n0), v);
    double est = 0.0;
    int it = 0;
    while (it < maxit) {
        ++it;
        op(v, f->r);
        op(f->r, w);
        const double nw = norm2(w);
        const double now = std::sqrt(std::sqrt(nw));
        if (nw == 0.0) {
            est = 0.0;
            break;
        }
        hipLaunchKernelGGL(rhif::k_axpby, dim3(gb), dim3(256), 0, s, N, 0.0, v, 1.0 / std::sqrt(nw), w);
        std::swap(v, w);
        const bool done = est > 0.0 && std::fabs(now - est) <= rtol * now;
        est = now;
        if (done) break;
    }
    HIPCHK(hipGetLastError());
    if (iters) *iters = it;
    return est;
}

void ensure_pcg(rhif_factor_s* f) {
    if (f->r) return;
    const size_t vb = f->g.N * sizeof(double);
    f->r = static_cast<double*>(f->dalloc(vb));
    f->z = static_cast<double*>(f->dalloc(vb));
    f->p = static_cast<double*>(f->dalloc(vb));
    f->q = static_cast<double*>(f->dalloc(vb));
    f->part = static_cast<double*>(f->dalloc(2 * kRedBlocks * sizeof(double)));
    f->sc = static_cast<double*>(f->dalloc(16 * sizeof(double)));
    f->hsc = PinnedSlots::get().take();
    if (f->hsc == nullptr)
        fail(RHIF_ENOMEM, "pinned host allocation failed");
    HIPCHK(hipEventCreateWithFlags(&f->sc_ev, hipEventDisableTiming));
}

void drop_graph(rhif_factor_s* f, int g) {
    if (f->gexec[g]) (void)hipGraphExecDestroy(f->gexec[g]);
    if (f->graph[g]) (void)hipGraphDestroy(f->graph[g]);
    f->gexec[g] = nullptr;
    f->graph[g] = nullptr;
    for (const auto& q : f->gpend[g]) {
        f->evpool.push_back(q.a);
        f->evpool.push_back(q.b);
    }
    f->gpend[g].clear();
}

// Runs body(stream) as graph g: captured once on the internal stream, then replayed on s.
// Returns false (nothing launched) if graphs are unavailable or the kernels inside are
// being timed, and the caller runs body(s) directly.
// Whether the solve phase runs as HIP graphs (the flag is set, capture works, and none of
// the kernels inside is being timed).
bool graphs_wanted(const rhif_factor_s* f) {
    if (f->graphs_off || !(f->o.flags & RHIF_FLAG_SOLVE_GRAPHS)) return false;
    constexpr uint32_t in_graphs = (1u << RHIF_K_APPLY_UP) | (1u << RHIF_K_APPLY_DOWN) | (1u << RHIF_K_APPLY_GATHER) |
                                   (1u << RHIF_K_SPMV) | (1u << RHIF_K_VECTOR);
    return !(f->ktimes && (f->kmask & in_graphs));
}

template <class Body>
bool run_graph(rhif_factor_s* f, int g, hipStream_t s, Body body) {
    if (f->graphs_off || !(f->o.flags & RHIF_FLAG_SOLVE_GRAPHS)) return false;
    // kernels timed with HIP events run as direct launches (event times of graph nodes are
    // not available)
    constexpr uint32_t in_graphs = (1u << RHIF_K_APPLY_UP) | (1u << RHIF_K_APPLY_DOWN) | (1u << RHIF_K_APPLY_GATHER) |
                                   (1u << RHIF_K_SPMV) | (1u << RHIF_K_VECTOR);
    if (f->ktimes && (f->kmask & in_graphs)) return false;
    if (!f->gexec[g]) {
        if (!f->cap_stream && hipStreamCreateWithFlags(&f->cap_stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            f->graphs_off = true;
            return false;
        }
        const size_t np = f->pend.size();
        hipError_t e = hipStreamBeginCapture(f->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            try {
                body(f->cap_stream);
            } catch (...) {
                e = hipErrorUnknown;
            }
            hipGraph_t gr = nullptr;
            const hipError_t e2 = hipStreamEndCapture(f->cap_stream, &gr);
            f->graph[g] = gr;
            if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&f->gexec[g], f->graph[g], nullptr, nullptr, 0);
        f->gpend[g].assign(f->pend.begin() + np, f->pend.end());
        f->pend.resize(np);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            drop_graph(f, g);
            f->graphs_off = true;
            return false;
        }
    }
    HIPCHK(hipGraphLaunch(f->gexec[g], s));
    return true;
}

void apply_z(rhif_factor_s* f, hipStream_t s, bool& used) {
    used = run_graph(f, 0, s, [&](hipStream_t cs) { do_apply_inplace(f, f->z, cs); });
    if (!used) do_apply_inplace(f, f->z, s);
}

struct PcgWs {
    double *r, *z, *p, *q, *part, *sc;
    double* hsc;   // pinned host scalars, or nullptr
};

// Workspace of rhif_pcg_solve_noalloc: the CG vectors r, z, p, q (N doubles each), the
// partial sums of the reductions and the scalar slots, for N <= RHIF_NOALLOC_MAX_N. It is a
// file-scope device array, so calling the entry point allocates nothing; each GPU holds its
// own copy for the life of the process. Host code reaches it only through the address that
// hipGetSymbolAddress returns per device (the array's name is not a device address on the
// host).
constexpr int64_t kNoAllocDoubles = 4 * int64_t(RHIF_NOALLOC_MAX_N) + 2 * kRedBlocks + 16;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

double* noalloc_scratch(int dev) {
    static std::mutex mu;
    static std::map<int, double*> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(RHIF_EDEVICE, "hipGetSymbolAddress returned no address for the workspace");
    addr[dev] = static_cast<double*>(ptr);
    return static_cast<double*>(ptr);
}

// The PCG of rhif_pcg_solve on the workspace w (r, z, p, q: N doubles each; part: 2 kRedBlocks
// doubles of partial sums; sc: 16 scalars). With w.hsc (pinned host scalars) the host waits on
// events and looks ahead; without it (the no-allocation entry point) every scalar is read
// with a copy to host memory of the caller's thread and a stream synchronization, and no
// graph is used.
void pcg_run(rhif_factor_s* f, const PcgWs& w, const double* rhs, double* u, double rtol, int32_t maxit,
             int32_t* iters, double* relres, hipStream_t s) {
    const int64_t N = f->g.N;
    const int gb = grid_for(N);
    // a factor computed partly in FP32 is applied as a slightly inexact preconditioner: the
    // flexible (Polak-Ribiere) beta keeps CG robust to that, with the residual and every
    // inner product in FP64
    const bool flex = f->o.precision >= 1;
    double host_sc[2] = {0.0, 0.0};
    const bool pinned = w.hsc != nullptr;
    double* hsc = pinned ? w.hsc : host_sc;
    const double NB = 8.0 * static_cast<double>(N);
    const double spmv_by = 12.0 * f->nnz + 4.0 * (N + 1) + 3.0 * NB;
#define VEC(by, ...) KTIMED(f, cs, RHIF_K_VECTOR, 0.0, (by), __VA_ARGS__)
    // the graphs hold the solution pointer: capture again for another one
    if (pinned && f->graph_u != u) {
        drop_graph(f, 1);
        drop_graph(f, 2);
        f->graph_u = u;
    }
    // q = A p; alpha; u += alpha p, r -= alpha q; |r|^2 -> host
    auto update = [&](hipStream_t cs) {
        KTIMED(f, cs, RHIF_K_SPMV, 2.0 * f->nnz + 2.0 * N, spmv_by,
               hipLaunchKernelGGL(rhif::k_spmv_dot, dim3(gb), dim3(256), 0, cs, N, f->rp, f->ci, f->val, w.p, w.q,
                                  w.part));
        VEC(0.0, hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(256), 0, cs, w.part, gb, 1, w.sc, nullptr));
        VEC((flex ? 7 : 6) * NB, hipLaunchKernelGGL(rhif::k_axpy2, dim3(gb), dim3(256), 0, cs, N, w.sc, w.p, w.q, u,
                                                    w.r, w.part, flex ? w.z : nullptr, w.part + kRedBlocks));
        VEC(0.0, hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(256), 0, cs, w.part, gb, 2, w.sc, nullptr));
        if (flex)
            VEC(0.0, hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(256), 0, cs, w.part + kRedBlocks, gb, 5, w.sc,
                                        nullptr));
        HIPCHK(hipMemcpyAsync(hsc + 1, w.sc + 3, sizeof(double), hipMemcpyDeviceToHost, cs));
        if (!pinned) HIPCHK(hipStreamSynchronize(cs));
    };
    // z = F^-1 r; rho = r.z; beta (touches neither u, r nor p)
    auto precondition = [&](hipStream_t cs) {
        VEC(2 * NB, hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, cs, N, w.r, w.z));
        do_apply_inplace(f, w.z, cs);
        VEC(2 * NB, hipLaunchKernelGGL(rhif::k_dot, dim3(gb), dim3(256), 0, cs, N, w.r, w.z, w.part));
        VEC(0.0, hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(256), 0, cs, w.part, gb, flex ? 6 : 4, w.sc,
                                    nullptr));
    };
    // p = z + beta p; then the next update
    auto advance = [&](hipStream_t cs) {
        VEC(3 * NB, hipLaunchKernelGGL(rhif::k_update_p, dim3(gb), dim3(256), 0, cs, N, w.sc, w.z, w.p));
        update(cs);
    };
    auto iterate = [&](hipStream_t cs) {
        precondition(cs);
        advance(cs);
    };
    {
        hipStream_t cs = s;
        // r = f, u = 0, ||f||^2
        VEC(2 * NB, hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, cs, N, rhs, w.r));
        VEC(NB, hipLaunchKernelGGL(rhif::k_fill, dim3(gb), dim3(256), 0, cs, N, 0.0, u));
        VEC(NB, hipLaunchKernelGGL(rhif::k_dot, dim3(gb), dim3(256), 0, cs, N, rhs, rhs, w.part));
        VEC(0.0, hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(256), 0, cs, w.part, gb, 0, w.sc, nullptr));
        HIPCHK(hipMemcpyAsync(hsc, w.sc + 6, sizeof(double), hipMemcpyDeviceToHost, cs));
        if (pinned) HIPCHK(hipEventRecord(f->sc_ev, cs));
        else HIPCHK(hipStreamSynchronize(cs));
        // z = F^-1 r, rho = r.z, p = z
        VEC(2 * NB, hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, cs, N, w.r, w.z));
    }
    bool g0 = false;
    if (pinned) apply_z(f, s, g0);
    else do_apply_inplace(f, w.z, s);
    {
        hipStream_t cs = s;
        VEC(2 * NB, hipLaunchKernelGGL(rhif::k_dot, dim3(gb), dim3(256), 0, cs, N, w.r, w.z, w.part));
        VEC(0.0, hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(256), 0, cs, w.part, gb, 3, w.sc, nullptr));
        VEC(2 * NB, hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, cs, N, w.z, w.p));
    }
    int it = 0;
    double rel = 0.0;
    bool conv = false;
    if (!pinned) {
        // plain loop: every scalar read synchronizes the stream
        const double ff = hsc[0];
        const double fnorm = std::sqrt(ff);
        conv = (ff == 0.0);
        while (!conv && it < maxit) {
            update(s);
            ++it;
            rel = std::sqrt(hsc[1]) / fnorm;
            if (rel <= rtol) {
                conv = true;
                break;
            }
            if (it >= maxit) break;
            precondition(s);
            hipStream_t cs = s;
            VEC(3 * NB, hipLaunchKernelGGL(rhif::k_update_p, dim3(gb), dim3(256), 0, cs, N, w.sc, w.z, w.p));
        }
    } else if (g0 || graphs_wanted(f)) {
        HIPCHK(hipStreamSynchronize(s));
        if (g0) f->resolve_graph(0);
        const double ff = hsc[0];
        const double fnorm = std::sqrt(ff);
        conv = (ff == 0.0);
        int last = -1;   // graph whose replay the next synchronization completes
        if (!conv && maxit > 0) {
            if (run_graph(f, 1, s, update)) last = 1;
            else update(s);
        }
        while (!conv && it < maxit) {
            HIPCHK(hipStreamSynchronize(s));
            if (last >= 0) f->resolve_graph(last);
            last = -1;
            ++it;
            rel = std::sqrt(hsc[1]) / fnorm;
            if (rel <= rtol) {
                conv = true;
                break;
            }
            if (it >= maxit) break;
            if (run_graph(f, 2, s, iterate)) last = 2;
            else iterate(s);
        }
    } else {
        // Direct launches. The host waits only for the residual norm (an event after its
        // copy); while it decides, the stream already preconditions the new residual
        // (z = F^-1 r and r.z change neither u, r nor p, so an iteration that turns out not
        // to be needed leaves the solution untouched). The look-ahead is skipped when the
        // observed rate predicts convergence at the next check (within 10x of rtol), so that
        // a finished solve rarely leaves an unneeded apply behind. The stream runs the same
        // kernels in the same order as without look-ahead.
        HIPCHK(hipEventSynchronize(f->sc_ev));   // ||f||^2, copied before the first apply
        const double ff = hsc[0];
        const double fnorm = std::sqrt(ff);
        conv = (ff == 0.0);
        if (!conv && maxit > 0) {
            update(s);
            HIPCHK(hipEventRecord(f->sc_ev, s));
            bool ahead = maxit > 1;
            if (ahead) precondition(s);
            double prev = 1.0;   // ||r_0|| / ||f||
            while (true) {
                HIPCHK(hipEventSynchronize(f->sc_ev));
                ++it;
                rel = std::sqrt(hsc[1]) / fnorm;
                if (rel <= rtol) {
                    conv = true;
                    break;
                }
                if (it >= maxit) break;
                if (!ahead) precondition(s);
                advance(s);
                HIPCHK(hipEventRecord(f->sc_ev, s));
                const double predicted = prev > 0.0 ? rel * (rel / prev) : rel;
                prev = rel;
                ahead = it + 1 < maxit && !(predicted <= 10.0 * rtol);
                if (ahead) precondition(s);
            }
        }
    }
#undef VEC
    if (pinned) f->resolve();
    HIPCHK(hipGetLastError());
    f->mark(s);
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (!conv) fail(RHIF_ENOCONV, "PCG did not reach the tolerance within maxit iterations");
}

// ---------------------------------------------------------------------------------------
// Solves over all problems of a factorization call with several problems. The apply of
// eq. (3.2) runs level by level over the blocks of every problem in one launch per kernel;
// each block carries its problem's place in the concatenated vectors, and the problems of a
// family are split by the kernels they take alone, so that every block is computed as in its
// own problem's apply. The PCG's vector kernels give every problem its own scalars and the
// partial sums of its lone grid, so that each problem's iterates are those of its own solve.
// ---------------------------------------------------------------------------------------

// The merged tables, the vector segments and the workspace, at the first solve.
void batch_prepare(BatchSolve& b, hipStream_t s) {
    using namespace rhif;
    if (b.ready) return;
    rhif_factor_s* f0 = nullptr;
    int Lmax = 0;
    for (rhif_factor_s* f : b.fs) {
        if (!f) fail(RHIF_EINVAL, "a handle of the factorization call has been destroyed");
        if (!f0) f0 = f;
        Lmax = std::max(Lmax, f->L);
    }
    const int B = static_cast<int>(b.fs.size());
    const bool precond = f0->o.precond != 0;
    b.precond = precond;
    // merged tables, [level][family][fused / split]
    struct Fam {
        std::vector<ApplyDesc> ad;
        int mi = 0, mb = 0;
        size_t lds = 0;
        int band = -1;
    };
    std::vector<std::array<std::array<Fam, 3>, 4>> fam(Lmax + 1);
    // the kernels a family of one problem takes alone: 0 fused, 1 split, 2 big
    auto kind_of = [](int mi, int mb, const double* lip) {
        return split_ok(mi, mb, lip) ? 1 : big_ok(mi, lip) ? 2 : 0;
    };
    std::vector<std::vector<GroupApplyDesc>> grp(Lmax + 1);
    std::vector<std::vector<GatherDesc>> gat(Lmax + 1);
    b.lev.assign(Lmax + 1, MLevel{});
    auto add = [&](Fam& F, const std::vector<ApplyDesc>& src, int64_t o_pool, int64_t o_li, int64_t o_t,
                   int64_t o_dofs, int64_t o_ext, int64_t o_y, int64_t o_w, int64_t zo, int mi, int mb, size_t lds,
                   bool band) {
        for (ApplyDesc a : src) {
            a.off += o_pool;
            if (a.toff >= 0) a.toff += o_t;
            if (a.yoff >= 0) a.yoff += o_y;
            if (a.wsoff >= 0) a.wsoff += o_w;
            a.dofs += static_cast<int32_t>(o_dofs);
            if (a.ext >= 0) a.ext += static_cast<int32_t>(o_ext);
            a.li += static_cast<int32_t>(o_li);
            a.zoff = zo;
            F.ad.push_back(a);
        }
        F.mi = std::max(F.mi, mi);
        F.mb = std::max(F.mb, mb);
        F.lds = std::max(F.lds, lds);
        if (F.band < 0) F.band = band ? 1 : 0;
        else if (F.band != (band ? 1 : 0)) fail(RHIF_EINVAL, "internal error: mixed banded and full cell blocks");
    };
    std::vector<int> tkr(Lmax + 1, 0);
    for (int p = 0; p < B; ++p) {
        rhif_factor_s* f = b.fs[p];
        const int64_t zo = b.zoff[p];
        for (int lvl = 0; lvl <= f->L; ++lvl) {
            const LevelDev& LD = f->lev[lvl];
            const bool root = lvl == f->L;
            const int sp = kind_of(LD.mi_cell, LD.mb_cell, LD.linv);
            add(fam[lvl][root ? 1 : 0][sp], LD.h_cell_ad, LD.o_front, 256 * LD.o_ext, 0, LD.o_cdofs, LD.o_ext,
                f->o_ybuf, f->o_ws, zo, LD.mi_cell, LD.mb_cell, LD.lds_cell, LD.leaf_banded);
            if (root) continue;
            if (group_ok(LD)) {
                for (GroupApplyDesc x : LD.h_gad) {
                    x.dofs += static_cast<int32_t>(LD.o_sepdofs);
                    for (int sl = 0; sl < x.nslot; ++sl) x.yoff[sl] += f->o_ybuf;
                    x.loff += LD.o_lg;
                    x.li += static_cast<int32_t>(LD.o_li);
                    x.poff += static_cast<int32_t>(LD.o_perm);
                    x.goff += LD.o_g;
                    x.toff += LD.o_t;
                    x.skli += static_cast<int32_t>(LD.o_skli);
                    x.zoff = zo;
                    grp[lvl].push_back(x);
                }
                MLevel& M = b.lev[lvl];
                M.mn_grp = std::max(M.mn_grp, LD.mn_grp);
                tkr[lvl] = std::max(tkr[lvl], LD.tk_raw);
            } else {
                for (GatherDesc g : LD.h_gat) {
                    g.dofs += static_cast<int32_t>(LD.o_sepdofs);
                    for (int sl = 0; sl < g.nslot; ++sl) g.yoff[sl] += f->o_ybuf;
                    g.zoff = zo;
                    gat[lvl].push_back(g);
                }
                if (precond)
                    add(fam[lvl][2][kind_of(LD.mi_sep, 0, LD.li)], LD.h_sep_ad, LD.o_lg, LD.o_li, 0,
                        LD.o_sepdofs, 0, f->o_ybuf, f->o_ws, zo, LD.mi_sep, 0, LD.lds_sep, false);
                add(fam[lvl][3][kind_of(LD.mi_skel, LD.mb_skel, LD.skli)], LD.h_skel_ad, LD.o_g, LD.o_skli,
                    LD.o_t, LD.o_skeldofs, 0, f->o_ybuf, f->o_ws, zo, LD.mi_skel, LD.mb_skel, LD.lds_skel, false);
            }
        }
    }
    // one upload of every merged table
    Packer pk;
    std::vector<std::array<std::array<size_t, 3>, 4>> off(Lmax + 1);
    std::vector<size_t> o_grp(Lmax + 1), o_gat(Lmax + 1);
    for (int lvl = 0; lvl <= Lmax; ++lvl) {
        for (int k = 0; k < 4; ++k)
            for (int sp = 0; sp < 3; ++sp) off[lvl][k][sp] = pk.add(fam[lvl][k][sp].ad);
        o_grp[lvl] = pk.add(grp[lvl]);
        o_gat[lvl] = pk.add(gat[lvl]);
    }
    // vector segments: each problem's blocks as its lone solve lays them out
    std::vector<BatchSeg> seg(B);
    std::vector<int32_t> blk;
    for (int p = 0; p < B; ++p) {
        rhif_factor_s* f = b.fs[p];
        BatchSeg& g = seg[p];
        g.rp = f->rp;
        g.ci = f->ci;
        g.val = f->val;
        g.zoff = b.zoff[p];
        g.n = f->g.N;
        g.b0 = static_cast<int32_t>(blk.size());
        g.nb = grid_for(f->g.N);
        for (int e = 0; e < g.nb; ++e) blk.push_back(p);
    }
    const size_t o_seg = pk.add(seg), o_blk = pk.add(blk);
    char* T = upload(f0, pk, s);
    for (int lvl = 0; lvl <= Lmax; ++lvl) {
        MLevel& M = b.lev[lvl];
        M.b = &b.base[lvl];
        const BatchLevelBase& bb = b.base[lvl];
        MFam* dst[4] = {M.cells, M.roots, M.seps, M.skels};
        for (int k = 0; k < 4; ++k)
            for (int sp = 0; sp < 3; ++sp) {
                const Fam& F = fam[lvl][k][sp];
                MFam& m = dst[k][sp];
                m.n = static_cast<int>(F.ad.size());
                if (m.n == 0) continue;
                m.ad = view<ApplyDesc>(T, off[lvl][k][sp]);
                m.mi = F.mi;
                m.mb = F.mb;
                m.lds = F.lds;
                m.kind = sp;
                m.band = F.band == 1;
                if (k < 2) {
                    m.pool = bb.front;
                    m.lip = bb.linv;
                    m.dofs = bb.cdofs;
                    m.ext = bb.ext;
                } else if (k == 2) {
                    m.pool = bb.lg;
                    m.lip = bb.li;
                    m.dofs = bb.sepdofs;
                } else {
                    m.pool = bb.gp;
                    m.lip = bb.skli;
                    m.tp = bb.tp;
                    m.dofs = bb.skeldofs;
                }
                // a split set whose largest blocks together overflow the split kernels' LDS:
                // never the case for the blocks this library makes; refuse rather than guess
                if (m.kind == 1 && !split_ok(m.mi, m.mb, m.lip))
                    fail(RHIF_EINVAL, "internal error: merged split apply blocks exceed the LDS");
            }
        M.n_grp = static_cast<int>(grp[lvl].size());
        if (M.n_grp > 0) M.grp = view<GroupApplyDesc>(T, o_grp[lvl]);
        // T and G's off-diagonal blocks through LDS when the level's largest fit (as alone)
        M.tk = 2 * tkr[lvl] > kGroupStageMax ? 0 : tkr[lvl];
        M.n_gat = static_cast<int>(gat[lvl].size());
        if (M.n_gat > 0) M.gat = view<GatherDesc>(T, o_gat[lvl]);
    }
    b.seg = view<BatchSeg>(T, o_seg);
    b.blk = view<int32_t>(T, o_blk);
    b.nblk = static_cast<int>(blk.size());
    const size_t vb = static_cast<size_t>(std::max<int64_t>(b.ntot, 1)) * sizeof(double);
    b.r = static_cast<double*>(f0->dalloc(vb));
    b.z = static_cast<double*>(f0->dalloc(vb));
    b.p = static_cast<double*>(f0->dalloc(vb));
    b.q = static_cast<double*>(f0->dalloc(vb));
    b.u = static_cast<double*>(f0->dalloc(vb));
    b.part = static_cast<double*>(f0->dalloc(2 * static_cast<size_t>(b.nblk) * sizeof(double)));
    b.sc = static_cast<double*>(f0->dalloc(16 * static_cast<size_t>(B) * sizeof(double)));
    b.active = static_cast<int32_t*>(f0->dalloc(static_cast<size_t>(B) * sizeof(int32_t)));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&b.hsc), 16 * static_cast<size_t>(B) * sizeof(double),
                         hipHostMallocDefault));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&b.hact), static_cast<size_t>(B) * sizeof(int32_t),
                         hipHostMallocDefault));
    b.ready = true;
}

void mfam_up(rhif_factor_s* f, const MFam& m, double* z, double* ybuf, double* ws, hipStream_t s) {
    if (m.n <= 0) return;
    if (m.kind == 2) {
        big_up(f, 0.0, m.ad, m.n, m.mi, m.mb, m.pool, m.lip, m.tp, m.dofs, m.ext, z, ybuf, ws, s);
        return;
    }
    if (m.kind == 0) {
        hipLaunchKernelGGL(rhif::k_apply_up, dim3(m.n), dim3(256), m.lds, s, m.ad, m.pool, m.tp, m.dofs, z, ybuf, ws,
                           m.ext);
        return;
    }
    if (m.band)
        hipLaunchKernelGGL(rhif::k_apply_band<true>, dim3(m.n), dim3(256), band_lds(m.mi), s, m.ad, m.pool, m.lip,
                           m.dofs, z);
    else
        hipLaunchKernelGGL(rhif::k_apply_trsv_up, dim3(m.n), dim3(256), trsv_lds(m.mi, m.mb), s, m.ad, m.pool, m.lip,
                           m.tp, m.dofs, z, m.ext);
    if (m.mb > 0)
        hipLaunchKernelGGL(rhif::k_apply_gemv_up, dim3(m.n, (m.mb + 63) / 64), dim3(256),
                           static_cast<size_t>(m.mi + 256) * sizeof(double), s, m.ad, m.pool, m.dofs, z, ybuf);
}

void mfam_down(rhif_factor_s* f, const MFam& m, double* z, double* ws, hipStream_t s) {
    if (m.n <= 0) return;
    if (m.kind == 2) {
        big_down(f, 0.0, m.ad, m.n, m.mi, m.mb, m.pool, m.lip, m.tp, m.dofs, m.ext, z, ws, s);
        return;
    }
    if (m.kind == 0) {
        hipLaunchKernelGGL(rhif::k_apply_down, dim3(m.n), dim3(256), m.lds, s, m.ad, m.pool, m.tp, m.dofs, z, ws,
                           m.ext);
        return;
    }
    if (m.mb > 0)
        hipLaunchKernelGGL(rhif::k_apply_gemv_dn, dim3(m.n, (m.mi + 63) / 64), dim3(256),
                           static_cast<size_t>(64 * 65 + m.mb + 256) * sizeof(double), s, m.ad, m.pool, m.dofs, z);
    if (m.band)
        hipLaunchKernelGGL(rhif::k_apply_band<false>, dim3(m.n), dim3(256), band_lds(m.mi), s, m.ad, m.pool, m.lip,
                           m.dofs, z);
    else
        hipLaunchKernelGGL(rhif::k_apply_trsv_dn, dim3(m.n), dim3(256), trsv_lds(m.mi, m.mb), s, m.ad, m.pool, m.lip,
                           m.tp, m.dofs, z, m.ext);
}

// z <- F^-1 z for every problem at once (z: the concatenated vectors).
void batch_apply(BatchSolve& b, double* z, hipStream_t s) {
    const int Lmax = static_cast<int>(b.lev.size()) - 1;
    const bool precond = b.precond;
    rhif_factor_s* f0 = b.fs[0];   // launches are not timed (the joint calls refuse timing flags)
    for (int lvl = 0; lvl <= Lmax; ++lvl) {
        const MLevel& M = b.lev[lvl];
        const BatchLevelBase& bb = *M.b;
        for (int k = 0; k < 3; ++k) mfam_up(f0, M.cells[k], z, b.ybuf, b.ws, s);
        if (M.n_grp > 0)
            hipLaunchKernelGGL(rhif::k_apply_group_up, dim3(M.n_grp), dim3(256),
                               static_cast<size_t>(2 * 16 * ((M.mn_grp + 15) / 16) + 2 * M.tk) * sizeof(double), s,
                               M.grp, bb.sepdofs, b.ybuf, z, bb.lg, bb.li, bb.gp, bb.tp, bb.skli, bb.perm, M.tk);
        if (M.n_gat > 0)
            hipLaunchKernelGGL(rhif::k_sep_gather, dim3(M.n_gat), dim3(256), 0, s, M.gat, bb.sepdofs, b.ybuf, z);
        if (precond)
            for (int k = 0; k < 3; ++k) mfam_up(f0, M.seps[k], z, nullptr, b.ws, s);
        for (int k = 0; k < 3; ++k) mfam_up(f0, M.skels[k], z, nullptr, b.ws, s);
        for (int k = 0; k < 3; ++k) mfam_up(f0, M.roots[k], z, b.ybuf, b.ws, s);
    }
    for (int lvl = Lmax; lvl >= 0; --lvl) {
        const MLevel& M = b.lev[lvl];
        const BatchLevelBase& bb = *M.b;
        for (int k = 0; k < 3; ++k) mfam_down(f0, M.roots[k], z, b.ws, s);
        if (M.n_grp > 0)
            hipLaunchKernelGGL(rhif::k_apply_group_dn, dim3(M.n_grp), dim3(256),
                               static_cast<size_t>(2 * 16 * ((M.mn_grp + 15) / 16) + 2 * M.tk) * sizeof(double), s,
                               M.grp, bb.sepdofs, z, bb.lg, bb.li, bb.gp, bb.tp, bb.skli, bb.perm, M.tk);
        for (int k = 0; k < 3; ++k) mfam_down(f0, M.skels[k], z, b.ws, s);
        if (precond)
            for (int k = 0; k < 3; ++k) mfam_down(f0, M.seps[k], z, b.ws, s);
        for (int k = 0; k < 3; ++k) mfam_down(f0, M.cells[k], z, b.ws, s);
    }
    HIPCHK(hipGetLastError());
}

// The handles of one factorization call with several problems, all of them, in the call's
// order; returns its joint solve state, locked.
BatchSolve& batch_of(int32_t count, const rhif_factor_t* hs, std::unique_lock<std::mutex>& lk) {
    if (count < 2 || !hs) fail(RHIF_EINVAL, "count must be >= 2 and handles not NULL");
    for (int32_t i = 0; i < count; ++i)
        if (!hs[i]) fail(RHIF_EINVAL, "NULL handle");
    BatchSolve* b = hs[0]->bsolve.get();
    if (!b) fail(RHIF_EINVAL, "the handles do not come from one rhif_factor_batch call with several problems");
    lk = std::unique_lock<std::mutex>(b->mu);
    if (static_cast<int32_t>(b->fs.size()) != count)
        fail(RHIF_EINVAL, "pass every handle of the rhif_factor_batch call, in its order");
    for (int32_t i = 0; i < count; ++i)
        if (b->fs[i] != hs[i]) fail(RHIF_EINVAL, "pass every handle of the rhif_factor_batch call, in its order");
    return *b;
}

// PCG over every problem at once: each problem takes the iterations of its own rhif_pcg_solve
// (same kernels' arithmetic, same partial sums) and stops at its own convergence; the loop ends
// when all have converged or after maxit iterations.
void batch_pcg(BatchSolve& b, const double* const* rhs, double* const* u, double rtol, int32_t maxit,
               int32_t* iters, double* relres, hipStream_t s) {
    using namespace rhif;
    const int B = static_cast<int>(b.fs.size());
    const bool flex = b.fs[0]->o.precision >= 1;
    const int nb = b.nblk;
    const int64_t Nt = b.ntot;
    const int gt = grid_for(Nt);
    // r = f, u = 0, ||f||^2
    for (int p = 0; p < B; ++p)
        HIPCHK(hipMemcpyAsync(b.r + b.zoff[p], rhs[p], b.fs[p]->g.N * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<int32_t> act(B, 1);
    for (int p = 0; p < B; ++p) b.hact[p] = 1;
    HIPCHK(hipMemcpyAsync(b.active, b.hact, B * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill, dim3(gt), dim3(256), 0, s, Nt, 0.0, b.u);
    hipLaunchKernelGGL(k_bdot, dim3(nb), dim3(256), 0, s, b.seg, b.blk, b.r, b.r, b.part);
    hipLaunchKernelGGL(k_bfinalize, dim3(B), dim3(256), 0, s, b.seg, b.part, 0, b.sc, b.active);
    // z = F^-1 r, rho = r.z, p = z
    hipLaunchKernelGGL(k_copy, dim3(gt), dim3(256), 0, s, Nt, b.r, b.z);
    batch_apply(b, b.z, s);
    hipLaunchKernelGGL(k_bdot, dim3(nb), dim3(256), 0, s, b.seg, b.blk, b.r, b.z, b.part);
    hipLaunchKernelGGL(k_bfinalize, dim3(B), dim3(256), 0, s, b.seg, b.part, 3, b.sc, b.active);
    hipLaunchKernelGGL(k_copy, dim3(gt), dim3(256), 0, s, Nt, b.z, b.p);
    HIPCHK(hipMemcpyAsync(b.hsc, b.sc, 16 * B * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<double> fnorm(B);
    int nact = 0;
    for (int p = 0; p < B; ++p) {
        const double ff = b.hsc[16 * p + 6];
        fnorm[p] = std::sqrt(ff);
        iters[p] = 0;
        relres[p] = 0.0;
        if (ff == 0.0) act[p] = 0;
        nact += act[p];
    }
    bool changed = nact < B;
    int it = 0;
    while (nact > 0 && it < maxit) {
        if (changed) {
            for (int p = 0; p < B; ++p) b.hact[p] = act[p];
            HIPCHK(hipMemcpyAsync(b.active, b.hact, B * sizeof(int32_t), hipMemcpyHostToDevice, s));
            changed = false;
        }
        // q = A p; alpha; u += alpha p, r -= alpha q; |r|^2
        hipLaunchKernelGGL(k_bspmv_dot, dim3(nb), dim3(256), 0, s, b.seg, b.blk, b.p, b.q, b.part);
        hipLaunchKernelGGL(k_bfinalize, dim3(B), dim3(256), 0, s, b.seg, b.part, 1, b.sc, b.active);
        hipLaunchKernelGGL(k_baxpy2, dim3(nb), dim3(256), 0, s, b.seg, b.blk, b.sc, b.p, b.q, b.u, b.r, b.part,
                           flex ? b.z : nullptr, b.part + nb);
        hipLaunchKernelGGL(k_bfinalize, dim3(B), dim3(256), 0, s, b.seg, b.part, 2, b.sc, b.active);
        if (flex) hipLaunchKernelGGL(k_bfinalize, dim3(B), dim3(256), 0, s, b.seg, b.part + nb, 5, b.sc, b.active);
        HIPCHK(hipMemcpyAsync(b.hsc, b.sc, 16 * B * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ++it;
        for (int p = 0; p < B; ++p) {
            if (!act[p]) continue;
            iters[p] = it;
            relres[p] = std::sqrt(b.hsc[16 * p + 3]) / fnorm[p];
            if (relres[p] <= rtol) {
                act[p] = 0;
                --nact;
                changed = true;
            }
        }
        if (nact == 0 || it >= maxit) break;
        if (changed) {
            for (int p = 0; p < B; ++p) b.hact[p] = act[p];
            HIPCHK(hipMemcpyAsync(b.active, b.hact, B * sizeof(int32_t), hipMemcpyHostToDevice, s));
            changed = false;
        }
        // z = F^-1 r; rho = r.z; beta; p = z + beta p
        hipLaunchKernelGGL(k_copy, dim3(gt), dim3(256), 0, s, Nt, b.r, b.z);
        batch_apply(b, b.z, s);
        hipLaunchKernelGGL(k_bdot, dim3(nb), dim3(256), 0, s, b.seg, b.blk, b.r, b.z, b.part);
        hipLaunchKernelGGL(k_bfinalize, dim3(B), dim3(256), 0, s, b.seg, b.part, flex ? 6 : 4, b.sc, b.active);
        hipLaunchKernelGGL(k_bupdate_p, dim3(nb), dim3(256), 0, s, b.seg, b.blk, b.sc, b.z, b.p);
    }
    for (int p = 0; p < B; ++p)
        HIPCHK(hipMemcpyAsync(u[p], b.u + b.zoff[p], b.fs[p]->g.N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipGetLastError());
    for (rhif_factor_s* f : b.fs) f->mark(s);
    if (nact > 0) fail(RHIF_ENOCONV, "PCG did not reach the tolerance within maxit iterations for every problem");
}


}  // namespace

extern "C" {

const char* rhif_last_error(void) { return g_last_error.c_str(); }

const char* rhif_version(void) { return "rhif 0.2 (gfx950; FP64 and FP32-mixed factorizations)"; }

#define API_BEGIN try {
#define API_END                                                   \
    }                                                             \
    catch (const Failure& e) {                                    \
        g_last_error = e.msg;                                     \
        return e.st;                                              \
    }                                                             \
    catch (const std::bad_alloc&) {                               \
        g_last_error = "host allocation failed";                  \
        return RHIF_ENOMEM;                                       \
    }                                                             \
    catch (const std::exception& e) {                             \
        g_last_error = std::string("internal error: ") + e.what(); \
        return RHIF_EINVAL;                                       \
    }                                                             \
    g_last_error.clear();                                         \
    return RHIF_OK;

rhif_status rhif_fd_nnz(const rhif_grid* g, int64_t* nnz) {
    API_BEGIN
    validate_grid(g);
    if (!nnz) fail(RHIF_EINVAL, "nnz is NULL");
    *nnz = fd_nnz(g->dim, g->n[0]);
    API_END
}

rhif_status rhif_assemble_fd(const rhif_grid* g, const double* a_cells, const double* b, int32_t* row_ptr,
                             int32_t* col, double* val, hipStream_t s) {
    API_BEGIN
    validate_grid(g);
    if (!a_cells || !row_ptr || !col || !val) fail(RHIF_EINVAL, "NULL device pointer");
    const int d = g->dim, sd = g->n[0];
    int64_t N = 1;
    for (int k = 0; k < d; ++k) N *= sd;
    hipLaunchKernelGGL(rhif::k_fd_rowptr, dim3(static_cast<int>(std::min<int64_t>(N / 256 + 1, 65535))), dim3(256), 0,
                       s, d, sd, row_ptr);
    const double h = 1.0 / (sd + 1);
    const double inv_h2 = 1.0 / (h * h);
    const int grid = static_cast<int>(std::min<int64_t>((N + 255) / 256, 65535));
    hipLaunchKernelGGL(rhif::k_assemble_fd, dim3(grid), dim3(256), 0, s, d, sd, inv_h2, a_cells, b, row_ptr, col, val);
    HIPCHK(hipGetLastError());
    API_END
}

rhif_status rhif_factor(const rhif_grid* g, const rhif_opts* o, const int32_t* row_ptr, const int32_t* col,
                        const double* val, hipStream_t s, rhif_factor_t* out) {
    if (!out) {
        g_last_error = "out is NULL";
        return RHIF_EINVAL;
    }
    return rhif_factor_batch(1, g, o, &row_ptr, &col, &val, s, out);
}

rhif_status rhif_factor_batch(int32_t count, const rhif_grid* grids, const rhif_opts* o,
                              const int32_t* const* row_ptr, const int32_t* const* col, const double* const* val,
                              hipStream_t s, rhif_factor_t* out) {
    std::vector<rhif_factor_s*> fs;
    auto drop = [&] {
        if (fs.empty()) return;
        (void)hipStreamSynchronize(s);
        for (rhif_factor_s* f : fs) {
            f->release();
            delete f;
        }
        fs.clear();
    };
    try {
        if (!out) fail(RHIF_EINVAL, "out is NULL");
        if (count < 1) fail(RHIF_EINVAL, "count must be >= 1");
        for (int32_t i = 0; i < count; ++i) out[i] = nullptr;
        if (!grids) fail(RHIF_EINVAL, "grids is NULL");
        if (!o) fail(RHIF_EINVAL, "opts is NULL");
        if (o->leaf < 2) fail(RHIF_EINVAL, "leaf must be >= 2");
        if (!(o->eps >= 0.0) || !(o->eps < 1.0)) fail(RHIF_EINVAL, "eps must be in [0, 1)");
        if (o->precond != 0 && o->precond != 1) fail(RHIF_EINVAL, "precond must be 0 or 1");
        if (o->precision < 0 || o->precision > 2)
            fail(RHIF_EINVAL, "precision must be 0 (FP64), 1 (FP32 ID) or 2 (FP32 ID and Schur products)");
        if (o->flags & kRemovedFlags) fail(RHIF_EINVAL, "flag bit 2 (leaf sublevels) is not supported");
        if (count > 1 && (o->flags & (RHIF_FLAG_KERNEL_TIMES | RHIF_FLAG_PHASE_TIMES)))
            fail(RHIF_EINVAL, "kernel and phase times are recorded for single factorizations only");
        if (!row_ptr || !col || !val) fail(RHIF_EINVAL, "NULL CSR pointer array");
        std::vector<CsrIn> in(count);
        for (int32_t i = 0; i < count; ++i) {
            validate_grid(&grids[i]);
            if (grids[i].dim != grids[0].dim) fail(RHIF_EINVAL, "every grid of a batch must have the same dim");
            if (!row_ptr[i] || !col[i] || !val[i]) fail(RHIF_EINVAL, "NULL CSR pointer");
            in[i] = {row_ptr[i], col[i], val[i]};
        }
        set_kernel_attributes();
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        auto arena = std::make_shared<Arena>();
        arena->device = dev;
        for (int32_t i = 0; i < count; ++i) {
            rhif_factor_s* f = new rhif_factor_s();
            fs.push_back(f);
            f->device = dev;
            f->arena = arena;
            const rhif_grid* g = &grids[i];
            f->g.d = g->dim;
            f->g.s = g->n[0];
            f->g.N = 1;
            for (int k = 0; k < g->dim; ++k) f->g.N *= g->n[0];
            f->o = *o;
            f->ktimes = (o->flags & RHIF_FLAG_KERNEL_TIMES) != 0;
            {
                const uint32_t m = (static_cast<uint32_t>(o->flags) >> RHIF_KERNEL_MASK_SHIFT) & 0xffffu;
                f->kmask = m ? m : 0xffffu;
            }
            f->L = rhif::num_levels(f->g.s, o->leaf);
            f->Lskel = f->L;
            f->stats.sublevels = 0;
            if (f->L > RHIF_MAX_LEVELS) fail(RHIF_EINVAL, "too many levels");
        }
        const auto t0 = std::chrono::steady_clock::now();
        do_factor(fs, in.data(), s);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int32_t i = 0; i < count; ++i) {
            fs[i]->mark(s);
            fs[i]->stats.t_total_ms = ms;
            out[i] = fs[i];
        }
        g_last_error.clear();
        return RHIF_OK;
    } catch (const Failure& e) {
        g_last_error = e.msg;
        drop();
        return e.st;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        drop();
        return RHIF_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = std::string("internal error: ") + e.what();
        drop();
        return RHIF_EINVAL;
    }
}

rhif_status rhif_apply(rhif_factor_t f, const double* r, double* z, int32_t nrhs, hipStream_t s) {
    API_BEGIN
    if (!f || !r || !z) fail(RHIF_EINVAL, "NULL argument");
    if (nrhs < 0) fail(RHIF_EINVAL, "nrhs < 0");
    ensure_pcg(f);
    const int64_t N = f->g.N;
    bool used = false;
    for (int c = 0; c < nrhs; ++c) {
        double* zc = z + c * N;
        const double* rc = r + c * N;
        hipLaunchKernelGGL(rhif::k_copy, dim3(grid_for(N)), dim3(256), 0, s, N, rc, f->z);
        apply_z(f, s, used);
        hipLaunchKernelGGL(rhif::k_copy, dim3(grid_for(N)), dim3(256), 0, s, N, f->z, zc);
    }
    HIPCHK(hipGetLastError());
    f->mark(s);
    if (used && !f->gpend[0].empty()) {
        HIPCHK(hipStreamSynchronize(s));
        f->resolve_graph(0);
    }
    API_END
}

rhif_status rhif_apply_batch(int32_t count, const rhif_factor_t* f, const double* const* r, double* const* z,
                             hipStream_t s) {
    API_BEGIN
    std::unique_lock<std::mutex> lk;
    BatchSolve& b = batch_of(count, f, lk);
    if (!r || !z) fail(RHIF_EINVAL, "NULL vector array");
    for (int32_t i = 0; i < count; ++i)
        if (!r[i] || !z[i]) fail(RHIF_EINVAL, "NULL vector");
    batch_prepare(b, s);
    for (int32_t i = 0; i < count; ++i)
        HIPCHK(hipMemcpyAsync(b.z + b.zoff[i], r[i], f[i]->g.N * sizeof(double), hipMemcpyDeviceToDevice, s));
    batch_apply(b, b.z, s);
    for (int32_t i = 0; i < count; ++i)
        HIPCHK(hipMemcpyAsync(z[i], b.z + b.zoff[i], f[i]->g.N * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (int32_t i = 0; i < count; ++i) f[i]->mark(s);
    API_END
}

rhif_status rhif_pcg_solve_batch(int32_t count, const rhif_factor_t* f, const double* const* rhs, double* const* u,
                                 double rtol, int32_t maxit, int32_t* iters, double* relres, hipStream_t s) {
    API_BEGIN
    std::unique_lock<std::mutex> lk;
    BatchSolve& b = batch_of(count, f, lk);
    if (!rhs || !u || !iters || !relres) fail(RHIF_EINVAL, "NULL argument");
    for (int32_t i = 0; i < count; ++i)
        if (!rhs[i] || !u[i]) fail(RHIF_EINVAL, "NULL vector");
    if (maxit < 0 || !(rtol >= 0.0)) fail(RHIF_EINVAL, "bad maxit or rtol");
    batch_prepare(b, s);
    batch_pcg(b, rhs, u, rtol, maxit, iters, relres, s);
    API_END
}

rhif_status rhif_apply_half(rhif_factor_t f, const double* r, double* z, int32_t which, hipStream_t s) {
    API_BEGIN
    if (!f || !r || !z) fail(RHIF_EINVAL, "NULL argument");
    if (which != 0 && which != 1) fail(RHIF_EINVAL, "which must be 0 (G^-1) or 1 (G^-T)");
    ensure_pcg(f);
    const int64_t N = f->g.N;
    hipLaunchKernelGGL(rhif::k_copy, dim3(grid_for(N)), dim3(256), 0, s, N, r, f->z);
    if (which == 0) do_apply_up(f, f->z, s);
    else do_apply_down(f, f->z, s);
    hipLaunchKernelGGL(rhif::k_copy, dim3(grid_for(N)), dim3(256), 0, s, N, f->z, z);
    HIPCHK(hipGetLastError());
    f->resolve();
    f->mark(s);
    API_END
}

rhif_status rhif_estimate_es(rhif_factor_t f, const double* v0, int32_t maxit, double rtol, double* es,
                             int32_t* iters, hipStream_t s) {
    API_BEGIN
    if (!f || !v0 || !es) fail(RHIF_EINVAL, "NULL argument");
    if (maxit < 1 || !(rtol >= 0.0)) fail(RHIF_EINVAL, "bad maxit or rtol");
    ensure_pcg(f);
    const int64_t N = f->g.N;
    const int gb = grid_for(N);
    double* t = f->z;
    // y = x - G^-1 A G^-T x
    auto op = [&](const double* x, double* y) {
        hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, s, N, x, t);
        do_apply_down(f, t, s);
        hipLaunchKernelGGL(rhif::k_spmv_dot, dim3(gb), dim3(256), 0, s, N, f->rp, f->ci, f->val, t, y, f->part);
        do_apply_up(f, y, s);
        hipLaunchKernelGGL(rhif::k_axpby, dim3(gb), dim3(256), 0, s, N, 1.0, x, -1.0, y);
    };
    int it = 0;
    *es = power_norm(f, v0, maxit, rtol, op, &it, s);
    f->resolve();
    f->mark(s);
    if (iters) *iters = it;
    API_END
}

rhif_status rhif_apply_forward(rhif_factor_t f, const double* x, double* y, hipStream_t s) {
    API_BEGIN
    if (!f || !x || !y) fail(RHIF_EINVAL, "NULL argument");
    ensure_pcg(f);
    const int64_t N = f->g.N;
    hipLaunchKernelGGL(rhif::k_copy, dim3(grid_for(N)), dim3(256), 0, s, N, x, f->z);
    do_forward_inplace(f, f->z, s);
    hipLaunchKernelGGL(rhif::k_copy, dim3(grid_for(N)), dim3(256), 0, s, N, f->z, y);
    HIPCHK(hipGetLastError());
    f->mark(s);
    API_END
}

rhif_status rhif_estimate_ea(rhif_factor_t f, const double* v0, int32_t maxit, double rtol, double* ea,
                             int32_t* iters, hipStream_t s) {
    API_BEGIN
    if (!f || !v0 || !ea) fail(RHIF_EINVAL, "NULL argument");
    if (maxit < 1 || !(rtol >= 0.0)) fail(RHIF_EINVAL, "bad maxit or rtol");
    ensure_pcg(f);
    const int64_t N = f->g.N;
    const int gb = grid_for(N);
    double* t = f->z;
    auto opA = [&](const double* x, double* y) {
        hipLaunchKernelGGL(rhif::k_spmv_dot, dim3(gb), dim3(256), 0, s, N, f->rp, f->ci, f->val, x, y, f->part);
    };
    // y = A x - F x
    auto opD = [&](const double* x, double* y) {
        hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, s, N, x, t);
        do_forward_inplace(f, t, s);
        hipLaunchKernelGGL(rhif::k_spmv_dot, dim3(gb), dim3(256), 0, s, N, f->rp, f->ci, f->val, x, y, f->part);
        hipLaunchKernelGGL(rhif::k_axpby, dim3(gb), dim3(256), 0, s, N, -1.0, t, 1.0, y);
    };
    int ia = 0, id = 0;
    const double na = power_norm(f, v0, maxit, rtol, opA, &ia, s);
    const double nd = power_norm(f, v0, maxit, rtol, opD, &id, s);
    *ea = na > 0.0 ? nd / na : 0.0;
    f->resolve();
    f->mark(s);
    if (iters) *iters = std::max(ia, id);
    API_END
}

rhif_status rhif_grad_log_a(const rhif_grid* g, const double* a_cells, const double* u, const double* lam,
                            double* grad, hipStream_t s) {
    API_BEGIN
    validate_grid(g);
    if (!a_cells || !u || !lam || !grad) fail(RHIF_EINVAL, "NULL device pointer");
    const int d = g->dim, sd = g->n[0];
    int64_t nc = 1;
    for (int k = 0; k < d; ++k) nc *= (sd + 1);
    const double h = 1.0 / (sd + 1);
    const int grid = static_cast<int>(std::min<int64_t>((nc + 255) / 256, 65535));
    hipLaunchKernelGGL(rhif::k_grad_log_a, dim3(grid), dim3(256), 0, s, d, sd, 1.0 / (h * h), a_cells, u, lam, grad);
    HIPCHK(hipGetLastError());
    API_END
}

rhif_status rhif_matvec(rhif_factor_t f, const double* x, double* y, hipStream_t s) {
    API_BEGIN
    if (!f || !x || !y) fail(RHIF_EINVAL, "NULL argument");
    ensure_pcg(f);
    const int64_t N = f->g.N;
    hipLaunchKernelGGL(rhif::k_spmv_dot, dim3(grid_for(N)), dim3(256), 0, s, N, f->rp, f->ci, f->val, x, y, f->part);
    HIPCHK(hipGetLastError());
    f->mark(s);
    API_END
}

rhif_status rhif_pcg_solve(rhif_factor_t f, const double* rhs, double* u, double rtol, int32_t maxit,
                           int32_t* iters, double* relres, hipStream_t s) {
    API_BEGIN
    if (!f || !rhs || !u) fail(RHIF_EINVAL, "NULL argument");
    if (maxit < 0 || !(rtol >= 0.0)) fail(RHIF_EINVAL, "bad maxit or rtol");
    ensure_pcg(f);
    const PcgWs w{f->r, f->z, f->p, f->q, f->part, f->sc, f->hsc};
    pcg_run(f, w, rhs, u, rtol, maxit, iters, relres, s);
    API_END
}

rhif_status rhif_pcg_solve_noalloc(rhif_factor_t f, const double* rhs, double* u, double rtol, int32_t maxit,
                                   int32_t* iters, double* relres, hipStream_t s) {
    API_BEGIN
    if (!f || !rhs || !u) fail(RHIF_EINVAL, "NULL argument");
    if (maxit < 0 || !(rtol >= 0.0)) fail(RHIF_EINVAL, "bad maxit or rtol");
    if (f->g.N > RHIF_NOALLOC_MAX_N) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "rhif_pcg_solve_noalloc: N = %lld exceeds RHIF_NOALLOC_MAX_N = %d",
                      static_cast<long long>(f->g.N), RHIF_NOALLOC_MAX_N);
        fail(RHIF_EINVAL, buf);
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev != f->device) fail(RHIF_EINVAL, "rhif_pcg_solve_noalloc: the current device is not the handle's");
    double* base = noalloc_scratch(dev);
    const int64_t N = f->g.N;
    const PcgWs w{base, base + N, base + 2 * N, base + 3 * N, base + 4 * N, base + 4 * N + 2 * kRedBlocks, nullptr};
    // the scalar slots start cleared (a fill kernel, not a memset node, so that a caller may
    // capture the call); the vectors are written before they are read
    hipLaunchKernelGGL(rhif::k_fill, dim3(1), dim3(256), 0, s, int64_t(16), 0.0, w.sc);
    HIPCHK(hipGetLastError());
    // no kernel timing here: its events would be created on demand
    const bool kt = f->ktimes;
    f->ktimes = false;
    try {
        pcg_run(f, w, rhs, u, rtol, maxit, iters, relres, s);
    } catch (...) {
        f->ktimes = kt;
        throw;
    }
    f->ktimes = kt;
    API_END
}

rhif_status rhif_stats(rhif_factor_t f, rhif_stats_t* out) {
    API_BEGIN
    if (!f || !out) fail(RHIF_EINVAL, "NULL argument");
    f->resolve();
    *out = f->stats;
    API_END
}

rhif_status rhif_skeletons(rhif_factor_t f, int32_t level, int32_t* ngroups, int64_t* total, int32_t* first_dof,
                           int32_t* size, int32_t* rank, int32_t* perm) {
    API_BEGIN
    if (!f || !ngroups || !total) fail(RHIF_EINVAL, "NULL argument");
    if (level < 0 || level >= f->Lskel) fail(RHIF_EINVAL, "level out of range");
    const LevelDev& LD = f->lev[level];
    *ngroups = static_cast<int32_t>(LD.k.size());
    *total = static_cast<int64_t>(LD.perm.size());
    if (first_dof) std::copy(LD.first_dof.begin(), LD.first_dof.end(), first_dof);
    if (size) std::copy(LD.gsize.begin(), LD.gsize.end(), size);
    if (rank) std::copy(LD.k.begin(), LD.k.end(), rank);
    if (perm) std::copy(LD.perm.begin(), LD.perm.end(), perm);
    API_END
}

void rhif_destroy(rhif_factor_t f) {
    if (!f) return;
    f->release();
    delete f;
}

}  // extern "C"
