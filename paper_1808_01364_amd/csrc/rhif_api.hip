// Host driver of the C ABI declared in include/rhif.h: the level loop of the factorization
// (Sec. 3.1 / 3.2 of the paper), the factor apply (eq. (eqAinv)) and the PCG solve (Sec. 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
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

constexpr int kLdsBudgetDoubles = 8192;      // 64 KiB of LDS per workgroup
constexpr int kApplyCap = kLdsBudgetDoubles - rhif::kApplyDiagDoubles - 32;
constexpr int kRedBlocks = 1024;              // fixed partial-sum layout of the CG reductions

// Pinned host staging shared by all handles of the process (grow-only).
struct Pinned {
    std::mutex mu;
    char* up = nullptr;
    size_t up_bytes = 0;
    char* down = nullptr;
    size_t down_bytes = 0;
    char* get_up(size_t b) {
        if (b > up_bytes) {
            if (up) (void)hipHostFree(up);
            up = nullptr;
            up_bytes = 0;
            const size_t nb = std::max(b, up_bytes * 2);
            HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&up), nb, hipHostMallocDefault));
            up_bytes = nb;
        }
        return up;
    }
    char* get_down(size_t b) {
        if (b > down_bytes) {
            if (down) (void)hipHostFree(down);
            down = nullptr;
            down_bytes = 0;
            const size_t nb = std::max<size_t>(b, 1 << 16);
            HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&down), nb, hipHostMallocDefault));
            down_bytes = nb;
        }
        return down;
    }
};
Pinned& pinned() {
    static Pinned* p = new Pinned();
    return *p;
}

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
    rhif::LevelPlan plan;
    double* front = nullptr;
    double* lg = nullptr;
    double* tp = nullptr;
    double* gp = nullptr;
    char* tab = nullptr;
    char* tab2 = nullptr;
    // device views into tab / tab2
    int32_t* cdofs = nullptr;
    rhif::CellRef* cref = nullptr;
    rhif::FrontDesc* potrf = nullptr;
    rhif::Tile* tiles = nullptr;
    int32_t* src = nullptr;
    rhif::SepDesc* sep = nullptr;
    rhif::CellGroup* cg = nullptr;
    rhif::CellScaleDesc* cs = nullptr;
    rhif::SkelDesc* skd = nullptr;
    int32_t* rows = nullptr;
    rhif::ApplyDesc* cell_ad = nullptr;
    rhif::ApplyDesc* sep_ad = nullptr;
    rhif::GatherDesc* gat = nullptr;
    int32_t* sepdofs = nullptr;
    rhif::ApplyDesc* skel_ad = nullptr;
    int32_t* skeldofs = nullptr;
    int n_skel_ad = 0;
    size_t lds_cell = 0, lds_sep = 0, lds_skel = 0;
    // ID choices (host)
    std::vector<int32_t> k, perm, first_dof, gsize;
};

size_t apply_lds(const std::vector<rhif::ApplyDesc>& v) {
    int m = 0;
    for (const auto& d : v)
        if (d.wsoff < 0) m = std::max(m, d.nI + d.nB);
    return static_cast<size_t>(rhif::kApplyDiagDoubles + m) * sizeof(double);
}

int grid_for(int64_t N) {
    const int64_t b = (N + 255) / 256;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, kRedBlocks)));
}

}  // namespace

struct rhif_factor_s {
    rhif::GridInfo g;
    rhif_opts o{};
    int L = 0;
    int64_t nnz = 0;
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    double* val = nullptr;
    std::vector<LevelDev> lev;
    unsigned long long* err = nullptr;
    double* mp = nullptr;     // ID scratch (largest level)
    int64_t mp_elems = 0;
    double* ybuf = nullptr;
    int64_t y_elems = 0;
    double* ws = nullptr;
    int64_t ws_elems = 0;
    int32_t* kout = nullptr;  // per-level ID outputs (largest level)
    int32_t* pout = nullptr;
    int64_t kp_elems = 0;
    // PCG workspace
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *part = nullptr, *sc = nullptr;
    rhif_stats_t stats{};
    std::vector<void*> allocs;
    hipStream_t alloc_stream = nullptr;

    void* dalloc(size_t bytes) {
        void* ptr = nullptr;
        HIPCHK(hipMallocAsync(&ptr, std::max<size_t>(bytes, 256), alloc_stream));
        allocs.push_back(ptr);
        return ptr;
    }
    void release() {
        (void)hipStreamSynchronize(alloc_stream);
        for (void* ptr : allocs) (void)hipFree(ptr);
        allocs.clear();
    }
};

namespace {

void set_pool_threshold() {
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    });
}

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
        default: return "?";
    }
}

void check_err(rhif_factor_s* f, hipStream_t s) {
    unsigned long long h = 0;
    HIPCHK(hipMemcpyAsync(&h, f->err, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h != ~0ull) {
        const int level = static_cast<int>(h >> 40);
        const int step = static_cast<int>((h >> 32) & 0xff);
        const int block = static_cast<int>(h & 0xffffffffu);
        char buf[256];
        std::snprintf(buf, sizeof(buf), "not SPD: Cholesky pivot <= 0 or not finite at level %d, step %s, block %d",
                      level, step_name(step).c_str(), block);
        fail(RHIF_ENOTSPD, buf);
    }
}

template <class T>
T* view(char* base, size_t off) { return reinterpret_cast<T*>(base + off); }

void upload(rhif_factor_s* f, Packer& pk, char*& dst, hipStream_t s) {
    if (pk.total == 0) return;
    Pinned& pn = pinned();
    std::lock_guard<std::mutex> lk(pn.mu);
    char* h = pn.get_up(pk.total);
    for (size_t e = 0; e < pk.parts.size(); ++e)
        if (pk.parts[e].second) std::memcpy(h + pk.offs[e], pk.parts[e].first, pk.parts[e].second);
    dst = static_cast<char*>(f->dalloc(pk.total));
    HIPCHK(hipMemcpyAsync(dst, h, pk.total, hipMemcpyHostToDevice, s));
    // the staging buffer is reused by the next upload: wait for this copy
    HIPCHK(hipStreamSynchronize(s));
}

int panel_cap_for(int nmax, int reserved_doubles) {
    const int cap = (kLdsBudgetDoubles - reserved_doubles - 16 * 17) / 17;
    return std::max(0, std::min(cap, nmax));
}

size_t potrf_lds(int cap, int reserved) { return static_cast<size_t>(reserved + 16 * 17 + cap * 17) * sizeof(double); }

void do_factor(rhif_factor_s* f, const int32_t* row_ptr, const int32_t* col, const double* val, hipStream_t s) {
    using namespace rhif;
    const GridInfo& g = f->g;
    const int d = g.d;
    const int W = 1 << d;
    const int leaf = f->o.leaf;
    f->nnz = fd_nnz(d, g.s);
    f->err = static_cast<unsigned long long*>(f->dalloc(sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, f->err, ~0ull);
    // the handle keeps its own copy of A
    f->rp = static_cast<int32_t*>(f->dalloc((g.N + 1) * sizeof(int32_t)));
    f->ci = static_cast<int32_t*>(f->dalloc(f->nnz * sizeof(int32_t)));
    f->val = static_cast<double*>(f->dalloc(f->nnz * sizeof(double)));
    HIPCHK(hipMemcpyAsync(f->rp, row_ptr, (g.N + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(f->ci, col, f->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(f->val, val, f->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));

    PlanScratch scr;
    scr.init(g.N);
    std::vector<int32_t> active(g.N), next;
    for (int64_t i = 0; i < g.N; ++i) active[i] = static_cast<int32_t>(i);
    f->lev.resize(f->L + 1);
    const bool timing = (f->o.flags & RHIF_FLAG_PHASE_TIMES) != 0;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms_since = [&](std::chrono::steady_clock::time_point t0) {
        return std::chrono::duration<double, std::milli>(now() - t0).count();
    };
    auto phase = [&](int idx, std::chrono::steady_clock::time_point t0) {
        if (!timing) return;
        HIPCHK(hipStreamSynchronize(s));
        f->stats.t_phase_ms[idx] += ms_since(t0);
    };

    for (int lvl = 0; lvl <= f->L; ++lvl) {
        const bool root = (lvl == f->L);
        LevelDev& LD = f->lev[lvl];
        LevelPlan& P = LD.plan;
        const LevelDev* prev = lvl > 0 ? &f->lev[lvl - 1] : nullptr;
        auto t0 = now();
        build_level(g, lvl, leaf, root, active, prev ? &prev->plan : nullptr, scr, kApplyCap, P);
        validate_level(P, prev ? &prev->plan : nullptr, d);
        f->stats.n_active[lvl] = static_cast<int64_t>(active.size());
        f->stats.n_cells[lvl] = P.ncells;
        f->stats.max_front[lvl] = P.max_nf;

        Packer pk;
        const size_t o_cdofs = pk.add(P.c_dofs), o_cref = pk.add(P.cell_ref), o_potrf = pk.add(P.cell_potrf),
                     o_tiles = pk.add(P.tiles), o_src = pk.add(P.src), o_sep = pk.add(P.sep_desc),
                     o_cg = pk.add(P.cell_groups), o_cs = pk.add(P.cell_scale), o_skd = pk.add(P.skel_desc),
                     o_rows = pk.add(P.skel_rows), o_cad = pk.add(P.cell_apply), o_sad = pk.add(P.sep_apply),
                     o_gat = pk.add(P.gather), o_sdofs = pk.add(P.sep_dofs);
        upload(f, pk, LD.tab, s);
        char* T = LD.tab;
        LD.cdofs = view<int32_t>(T, o_cdofs);
        LD.cref = view<CellRef>(T, o_cref);
        LD.potrf = view<FrontDesc>(T, o_potrf);
        LD.tiles = view<Tile>(T, o_tiles);
        LD.src = view<int32_t>(T, o_src);
        LD.sep = view<SepDesc>(T, o_sep);
        LD.cg = view<CellGroup>(T, o_cg);
        LD.cs = view<CellScaleDesc>(T, o_cs);
        LD.skd = view<SkelDesc>(T, o_skd);
        LD.rows = view<int32_t>(T, o_rows);
        LD.cell_ad = view<ApplyDesc>(T, o_cad);
        LD.sep_ad = view<ApplyDesc>(T, o_sad);
        LD.gat = view<GatherDesc>(T, o_gat);
        LD.sepdofs = view<int32_t>(T, o_sdofs);
        LD.lds_cell = apply_lds(P.cell_apply);
        LD.lds_sep = apply_lds(P.sep_apply);

        LD.front = static_cast<double*>(f->dalloc(P.front_elems * sizeof(double)));
        if (!root) {
            LD.lg = static_cast<double*>(f->dalloc(P.lg_elems * sizeof(double)));
            LD.tp = static_cast<double*>(f->dalloc(P.t_elems * sizeof(double)));
            LD.gp = static_cast<double*>(f->dalloc(P.g_elems * sizeof(double)));
            if (P.m_elems > f->mp_elems) {
                f->mp = static_cast<double*>(f->dalloc(P.m_elems * sizeof(double)));
                f->mp_elems = P.m_elems;
            }
            const int64_t kp = static_cast<int64_t>(P.skel_desc.size()) + P.skel_ntotal + 1;
            if (kp > f->kp_elems) {
                f->kout = static_cast<int32_t*>(f->dalloc(kp * sizeof(int32_t)));
                f->pout = static_cast<int32_t*>(f->dalloc(kp * sizeof(int32_t)));
                f->kp_elems = kp;
            }
        }
        f->y_elems = std::max(f->y_elems, P.y_elems);
        f->ws_elems = std::max(f->ws_elems, P.ws_elems);
        phase(5, t0);

        // ---- frontal assembly ----
        t0 = now();
        if (!P.tiles.empty()) {
            if (lvl == 0)
                hipLaunchKernelGGL(k_front_csr, dim3(P.tiles.size()), dim3(256), 0, s, LD.tiles, LD.cref, LD.cdofs, d,
                                   g.s, P.w, P.nc1, f->rp, f->ci, f->val, LD.front);
            else
                hipLaunchKernelGGL(k_front_extend, dim3(P.tiles.size()), dim3(256), 0, s, LD.tiles, LD.cref, LD.src, W,
                                   prev->cref, prev->front, LD.front);
            HIPCHK(hipGetLastError());
        }
        phase(0, t0);

        // ---- cell elimination (E_l; at the root: B_L = chol(A_L)) ----
        t0 = now();
        if (!P.cell_potrf.empty()) {
            int nmax = 0;
            for (const auto& fd : P.cell_potrf) nmax = std::max(nmax, fd.n - std::min(fd.n, 1));
            const int cap = panel_cap_for(nmax, 0);
            hipLaunchKernelGGL(k_potrf_batch, dim3(P.cell_potrf.size()), dim3(256), potrf_lds(cap, 0), s, LD.potrf,
                               LD.front, cap, lvl, root ? 3 : 0, f->err);
            HIPCHK(hipGetLastError());
            f->stats.flops[lvl] += P.flops;
        }
        phase(root ? 6 : 1, t0);
        if (root) break;

        // ---- block Jacobi (C_l) ----
        t0 = now();
        if (f->o.precond && !P.sep_desc.empty()) {
            const int cap = panel_cap_for(P.max_sep_n, 0);
            hipLaunchKernelGGL(k_precond_groups, dim3(P.sep_desc.size()), dim3(256), potrf_lds(cap, 0), s, LD.sep,
                               LD.cref, LD.front, LD.lg, cap, lvl, f->err);
            HIPCHK(hipGetLastError());
            if (!P.cell_scale.empty()) {
                hipLaunchKernelGGL(k_precond_scale, dim3(P.cell_scale.size()), dim3(256), 0, s, LD.cs, LD.cg, LD.lg,
                                   LD.front);
                HIPCHK(hipGetLastError());
            }
        }
        f->stats.n_groups[lvl] = f->o.precond ? static_cast<int32_t>(P.sep_desc.size()) : 0;
        phase(2, t0);

        // ---- skeletonization (K_l) ----
        t0 = now();
        const int nsk = static_cast<int>(P.skel_desc.size());
        Pinned& pn = pinned();
        std::unique_lock<std::mutex> lk(pn.mu);
        int32_t* hk = nullptr;
        int32_t* hp = nullptr;
        if (nsk > 0) {
            const int n = P.max_skel_n;
            const int base = (n + 1) / 2 + 1;
            const int cap = panel_cap_for(n, base + 2);
            const size_t lds = std::max(static_cast<size_t>(base + n + 2) * sizeof(double), potrf_lds(cap, base));
            hipLaunchKernelGGL(k_skeletonize, dim3(nsk), dim3(256), lds, s, LD.skd, LD.rows, LD.cref, LD.front, f->mp,
                               LD.tp, LD.gp, f->o.eps, f->kout, f->pout, cap, lvl, f->err);
            HIPCHK(hipGetLastError());
            char* h = pn.get_down((nsk + P.skel_ntotal) * sizeof(int32_t) + 64);
            hk = reinterpret_cast<int32_t*>(h);
            hp = hk + nsk;
            HIPCHK(hipMemcpyAsync(hk, f->kout, nsk * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(hp, f->pout, P.skel_ntotal * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        }
        check_err(f, s);   // synchronizes: ranks are on the host now
        phase(3, t0);

        t0 = now();
        LD.k.assign(hk, hk + nsk);
        LD.perm.assign(hp, hp + P.skel_ntotal);
        lk.unlock();
        LD.first_dof.resize(nsk);
        LD.gsize.resize(nsk);
        int64_t sum_rank = 0;
        int max_rank = 0;
        for (int e = 0; e < nsk; ++e) {
            const int gidx = P.skels[e];
            LD.first_dof[e] = P.gdofs[P.gptr[gidx]];
            LD.gsize[e] = P.gptr[gidx + 1] - P.gptr[gidx];
            sum_rank += LD.k[e];
            max_rank = std::max(max_rank, LD.k[e]);
        }
        f->stats.n_skel[lvl] = nsk;
        f->stats.sum_skel_n[lvl] = P.skel_ntotal;
        f->stats.sum_rank[lvl] = sum_rank;
        f->stats.max_rank[lvl] = max_rank;
        std::vector<ApplyDesc> sk_ad;
        std::vector<int32_t> sk_dofs;
        double fl = 0.0;
        finish_level(P, LD.k.data(), LD.perm.data(), kApplyCap, sk_ad, sk_dofs, f->ws_elems, active, next, scr, fl);
        validate_skel_apply(P, sk_ad, sk_dofs, g.N);
        f->stats.flops[lvl] += P.flops + fl;
        Packer pk2;
        const size_t o_ad = pk2.add(sk_ad), o_dofs = pk2.add(sk_dofs);
        upload(f, pk2, LD.tab2, s);
        if (LD.tab2) {
            LD.skel_ad = view<ApplyDesc>(LD.tab2, o_ad);
            LD.skeldofs = view<int32_t>(LD.tab2, o_dofs);
        }
        LD.n_skel_ad = static_cast<int>(sk_ad.size());
        LD.lds_skel = apply_lds(sk_ad);
        active.swap(next);
        phase(5, t0);
    }
    check_err(f, s);
    f->stats.levels = f->L;
    f->stats.root_size = static_cast<int32_t>(active.size());
    f->stats.n_active[f->L] = static_cast<int64_t>(active.size());
    f->ybuf = static_cast<double*>(f->dalloc(std::max<int64_t>(f->y_elems, 1) * sizeof(double)));
    if (f->ws_elems > 0) f->ws = static_cast<double*>(f->dalloc(f->ws_elems * sizeof(double)));
    int64_t bytes = 0;
    for (const auto& LD : f->lev) {
        const auto& P = LD.plan;
        bytes += (P.front_elems + (P.root ? 0 : P.lg_elems + P.t_elems + P.g_elems)) * 8;
    }
    f->stats.factor_bytes = bytes;
    HIPCHK(hipStreamSynchronize(s));
}

void launch_up(const rhif::ApplyDesc* ad, int n, size_t lds, const double* pool, const double* tp,
               const int32_t* dofs, double* z, double* ybuf, double* ws, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(rhif::k_apply_up, dim3(n), dim3(256), lds, s, ad, pool, tp, dofs, z, ybuf, ws);
}

void launch_down(const rhif::ApplyDesc* ad, int n, size_t lds, const double* pool, const double* tp,
                 const int32_t* dofs, double* z, double* ws, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(rhif::k_apply_down, dim3(n), dim3(256), lds, s, ad, pool, tp, dofs, z, ws);
}

void do_apply_inplace(rhif_factor_s* f, double* z, hipStream_t s) {
    const int L = f->L;
    for (int lvl = 0; lvl < L; ++lvl) {
        LevelDev& LD = f->lev[lvl];
        const auto& P = LD.plan;
        launch_up(LD.cell_ad, static_cast<int>(P.cell_apply.size()), LD.lds_cell, LD.front, nullptr, LD.cdofs, z,
                  f->ybuf, f->ws, s);
        if (!P.gather.empty())
            hipLaunchKernelGGL(rhif::k_sep_gather, dim3(P.gather.size()), dim3(256), 0, s, LD.gat, LD.sepdofs,
                               f->ybuf, z);
        if (f->o.precond)
            launch_up(LD.sep_ad, static_cast<int>(P.sep_apply.size()), LD.lds_sep, LD.lg, nullptr, LD.sepdofs, z,
                      nullptr, f->ws, s);
        launch_up(LD.skel_ad, LD.n_skel_ad, LD.lds_skel, LD.gp, LD.tp, LD.skeldofs, z, nullptr, f->ws, s);
    }
    {
        LevelDev& LD = f->lev[L];
        const auto& P = LD.plan;
        launch_up(LD.cell_ad, static_cast<int>(P.cell_apply.size()), LD.lds_cell, LD.front, nullptr, LD.cdofs, z,
                  f->ybuf, f->ws, s);
        launch_down(LD.cell_ad, static_cast<int>(P.cell_apply.size()), LD.lds_cell, LD.front, nullptr, LD.cdofs, z,
                    f->ws, s);
    }
    for (int lvl = L - 1; lvl >= 0; --lvl) {
        LevelDev& LD = f->lev[lvl];
        const auto& P = LD.plan;
        launch_down(LD.skel_ad, LD.n_skel_ad, LD.lds_skel, LD.gp, LD.tp, LD.skeldofs, z, f->ws, s);
        if (f->o.precond)
            launch_down(LD.sep_ad, static_cast<int>(P.sep_apply.size()), LD.lds_sep, LD.lg, nullptr, LD.sepdofs, z,
                        f->ws, s);
        launch_down(LD.cell_ad, static_cast<int>(P.cell_apply.size()), LD.lds_cell, LD.front, nullptr, LD.cdofs, z,
                    f->ws, s);
    }
    HIPCHK(hipGetLastError());
}

void ensure_pcg(rhif_factor_s* f) {
    if (f->r) return;
    const size_t vb = f->g.N * sizeof(double);
    f->r = static_cast<double*>(f->dalloc(vb));
    f->z = static_cast<double*>(f->dalloc(vb));
    f->p = static_cast<double*>(f->dalloc(vb));
    f->q = static_cast<double*>(f->dalloc(vb));
    f->part = static_cast<double*>(f->dalloc(kRedBlocks * sizeof(double)));
    f->sc = static_cast<double*>(f->dalloc(16 * sizeof(double)));
}

}  // namespace

extern "C" {

const char* rhif_last_error(void) { return g_last_error.c_str(); }

const char* rhif_version(void) { return "rhif 0.1 (gfx950, FP64)"; }

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
    std::vector<int32_t> rp(N + 1);
    rp[0] = 0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t r = i;
        int cnt = 1;
        for (int k = 0; k < d; ++k) {
            const int x = static_cast<int>(r % sd) + 1;
            r /= sd;
            cnt += (x > 1) + (x < sd);
        }
        rp[i + 1] = rp[i] + cnt;
    }
    {
        Pinned& pn = pinned();
        std::lock_guard<std::mutex> lk(pn.mu);
        char* h = pn.get_up((N + 1) * sizeof(int32_t));
        std::memcpy(h, rp.data(), (N + 1) * sizeof(int32_t));
        HIPCHK(hipMemcpyAsync(row_ptr, h, (N + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    const double h = 1.0 / (sd + 1);
    const double inv_h2 = 1.0 / (h * h);
    const int grid = static_cast<int>(std::min<int64_t>((N + 255) / 256, 65535));
    hipLaunchKernelGGL(rhif::k_assemble_fd, dim3(grid), dim3(256), 0, s, d, sd, inv_h2, a_cells, b, row_ptr, col, val);
    HIPCHK(hipGetLastError());
    API_END
}

rhif_status rhif_factor(const rhif_grid* g, const rhif_opts* o, const int32_t* row_ptr, const int32_t* col,
                        const double* val, hipStream_t s, rhif_factor_t* out) {
    rhif_factor_s* f = nullptr;
    try {
        if (!out) fail(RHIF_EINVAL, "out is NULL");
        *out = nullptr;
        validate_grid(g);
        if (!o) fail(RHIF_EINVAL, "opts is NULL");
        if (o->leaf < 2) fail(RHIF_EINVAL, "leaf must be >= 2");
        if (!(o->eps >= 0.0) || !(o->eps < 1.0)) fail(RHIF_EINVAL, "eps must be in [0, 1)");
        if (o->precond != 0 && o->precond != 1) fail(RHIF_EINVAL, "precond must be 0 or 1");
        if (o->precision != 0) fail(RHIF_EINVAL, "only precision 0 (FP64) is available");
        if (!row_ptr || !col || !val) fail(RHIF_EINVAL, "NULL CSR pointer");
        set_pool_threshold();
        f = new rhif_factor_s();
        f->alloc_stream = s;
        f->g.d = g->dim;
        f->g.s = g->n[0];
        f->g.N = 1;
        for (int k = 0; k < g->dim; ++k) f->g.N *= g->n[0];
        f->o = *o;
        f->L = rhif::num_levels(f->g.s, o->leaf);
        if (f->L > RHIF_MAX_LEVELS) fail(RHIF_EINVAL, "too many levels");
        const auto t0 = std::chrono::steady_clock::now();
        do_factor(f, row_ptr, col, val, s);
        f->stats.t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = f;
        g_last_error.clear();
        return RHIF_OK;
    } catch (const Failure& e) {
        g_last_error = e.msg;
        if (f) {
            (void)hipStreamSynchronize(s);
            f->release();
            delete f;
        }
        return e.st;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        if (f) {
            f->release();
            delete f;
        }
        return RHIF_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = std::string("internal error: ") + e.what();
        if (f) {
            f->release();
            delete f;
        }
        return RHIF_EINVAL;
    }
}

rhif_status rhif_apply(rhif_factor_t f, const double* r, double* z, int32_t nrhs, hipStream_t s) {
    API_BEGIN
    if (!f || !r || !z) fail(RHIF_EINVAL, "NULL argument");
    if (nrhs < 0) fail(RHIF_EINVAL, "nrhs < 0");
    const int64_t N = f->g.N;
    for (int c = 0; c < nrhs; ++c) {
        double* zc = z + c * N;
        const double* rc = r + c * N;
        if (zc != rc) {
            hipLaunchKernelGGL(rhif::k_copy, dim3(grid_for(N)), dim3(256), 0, s, N, rc, zc);
        }
        do_apply_inplace(f, zc, s);
    }
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
    API_END
}

rhif_status rhif_pcg_solve(rhif_factor_t f, const double* rhs, double* u, double rtol, int32_t maxit,
                           int32_t* iters, double* relres, hipStream_t s) {
    API_BEGIN
    if (!f || !rhs || !u) fail(RHIF_EINVAL, "NULL argument");
    if (maxit < 0 || !(rtol >= 0.0)) fail(RHIF_EINVAL, "bad maxit or rtol");
    ensure_pcg(f);
    const int64_t N = f->g.N;
    const int gb = grid_for(N);
    Pinned& pn = pinned();
    double* hsc = nullptr;
    {
        std::lock_guard<std::mutex> lk(pn.mu);
        hsc = reinterpret_cast<double*>(pn.get_down(64));
    }
    // r = f, u = 0, ||f||^2
    hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, s, N, rhs, f->r);
    hipLaunchKernelGGL(rhif::k_fill, dim3(gb), dim3(256), 0, s, N, 0.0, u);
    hipLaunchKernelGGL(rhif::k_dot, dim3(gb), dim3(256), 0, s, N, rhs, rhs, f->part);
    hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(64), 0, s, f->part, gb, 0, f->sc, nullptr);
    HIPCHK(hipMemcpyAsync(hsc, f->sc + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    // z = F^-1 r, rho = r.z, p = z
    hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, s, N, f->r, f->z);
    do_apply_inplace(f, f->z, s);
    hipLaunchKernelGGL(rhif::k_dot, dim3(gb), dim3(256), 0, s, N, f->r, f->z, f->part);
    hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(64), 0, s, f->part, gb, 3, f->sc, nullptr);
    hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, s, N, f->z, f->p);
    HIPCHK(hipStreamSynchronize(s));
    const double ff = hsc[0];
    const double fnorm = std::sqrt(ff);
    int it = 0;
    double rel = 0.0;
    bool conv = (ff == 0.0);
    while (!conv && it < maxit) {
        hipLaunchKernelGGL(rhif::k_spmv_dot, dim3(gb), dim3(256), 0, s, N, f->rp, f->ci, f->val, f->p, f->q, f->part);
        hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(64), 0, s, f->part, gb, 1, f->sc, nullptr);
        hipLaunchKernelGGL(rhif::k_axpy2, dim3(gb), dim3(256), 0, s, N, f->sc, f->p, f->q, u, f->r, f->part);
        hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(64), 0, s, f->part, gb, 2, f->sc, nullptr);
        HIPCHK(hipMemcpyAsync(hsc + 1, f->sc + 3, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ++it;
        rel = std::sqrt(hsc[1]) / fnorm;
        if (rel <= rtol) {
            conv = true;
            break;
        }
        hipLaunchKernelGGL(rhif::k_copy, dim3(gb), dim3(256), 0, s, N, f->r, f->z);
        do_apply_inplace(f, f->z, s);
        hipLaunchKernelGGL(rhif::k_dot, dim3(gb), dim3(256), 0, s, N, f->r, f->z, f->part);
        hipLaunchKernelGGL(rhif::k_finalize, dim3(1), dim3(64), 0, s, f->part, gb, 4, f->sc, nullptr);
        hipLaunchKernelGGL(rhif::k_update_p, dim3(gb), dim3(256), 0, s, N, f->sc, f->z, f->p);
    }
    HIPCHK(hipGetLastError());
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (!conv) fail(RHIF_ENOCONV, "PCG did not reach the tolerance within maxit iterations");
    API_END
}

rhif_status rhif_stats(rhif_factor_t f, rhif_stats_t* out) {
    API_BEGIN
    if (!f || !out) fail(RHIF_EINVAL, "NULL argument");
    *out = f->stats;
    API_END
}

rhif_status rhif_skeletons(rhif_factor_t f, int32_t level, int32_t* ngroups, int64_t* total, int32_t* first_dof,
                           int32_t* size, int32_t* rank, int32_t* perm) {
    API_BEGIN
    if (!f || !ngroups || !total) fail(RHIF_EINVAL, "NULL argument");
    if (level < 0 || level >= f->L) fail(RHIF_EINVAL, "level out of range");
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
