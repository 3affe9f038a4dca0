// HIP kernels for gfx950 (CDNA4, 64-wide wavefronts) of the recursively preconditioned
// hierarchical interpolative factorization and its PCG solve.
//
// Every batched kernel runs one 256-thread workgroup (4 waves) per block of the batch and
// works on dense FP64 column-major matrices in HBM; small operands are staged in LDS.
// The dense Schur-complement updates use the FP64 matrix cores
// (v_mfma_f64_16x16x4f64). Nothing uses floating-point atomics: every sum that several
// blocks contribute to is formed by one thread in a fixed order, so results are bitwise
// repeatable run to run.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "devstructs.hpp"
#include "kernels.hpp"
#include "leafgeom.hpp"

namespace rhif {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kWG = 256;
constexpr int kWaves = kWG / 64;
constexpr int kSyrkBatch = 2;   // Schur tiles accumulated per wave at a time
constexpr int kLeafTilesPerWave = 4;   // Schur tiles a wave of the leaf kernel accumulates in registers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void report(unsigned long long* err, unsigned long long code) {
    atomicMin(err, code);
}

__device__ __forceinline__ unsigned long long err_code(int level, int step, int block) {
    return (static_cast<unsigned long long>(level) << 40) |
           (static_cast<unsigned long long>(step) << 32) |
           static_cast<unsigned long long>(static_cast<uint32_t>(block));
}

// Broadcast of lane l's double (l uniform) through scalar registers.
__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(v), l);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Cholesky factorization and inversion of a 16 x 16 SPD block held by one wave in registers:
// lane i < 16 holds row i in a[0..i]. On return a[c] = L[i][c] (c <= i; the entries above
// the diagonal are left undefined: the rank-1 updates run unmasked, since the rows above a
// pivot only change entries above their diagonal, which are never read) and li[r] =
// (L^-1)[r][lane] for lane < 16. A pivot <= 0 or NaN reports `code` and continues with 1.
__device__ __forceinline__ void wave_chol_inv16(double (&a)[16], double (&li)[16], int lane,
                                                unsigned long long* err, unsigned long long code) {
    double rinv[16];   // 1 / L[c][c], the same in every lane
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        double dcc = readlane_d(a[c], c);
        if (!(dcc > 0.0) || !(dcc < INFINITY)) {
            if (lane == 0) report(err, code);
            dcc = 1.0;
        }
        const double lcc = sqrt(dcc);
        rinv[c] = 1.0 / lcc;
        const double lic = a[c] * rinv[c];
        a[c] = (lane == c) ? lcc : lic;
#pragma unroll
        for (int q = c + 1; q < 16; ++q) a[q] -= a[c] * readlane_d(a[c], q);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        double v = (lane == i) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) v -= readlane_d(a[k], i) * li[k];
        li[i] = v * rinv[i];
    }
}

// ---------------------------------------------------------------------------------------
// Workgroup-collective partial Cholesky (right-looking over the pivots, 16-column panels).
//
// On entry the lower triangle of the n x n matrix A (column-major, ld) holds the
// symmetric matrix [[D, X^T], [X, S]] with D of order p. On exit
//   A[0:p, 0:p]  = L  with D = L L^T                       (Sec. 2.1: L_I = chol(A_II))
//   A[p:n, 0:p]  = X L^-T = W^T                             (W = L^-1 A_BI^T)
//   A[p:n, p:n]  = S - W^T W, stored in full (both triangles)  (the Schur complement)
// The panel loop updates only the pivot columns (rows j1..n-1, columns j1..p-1); the
// Schur complement is formed once at the end, S -= W^T W. Both products run on the FP64
// matrix cores, one 16 x 16 tile per wave at a time. Row tiles of a panel that are exactly
// zero (structural zeros, e.g. outside the band of a grid interior) are skipped. If ext is
// given, ext[t] receives the end of the nonzero rows (< p) of panel t, for the apply; if
// linv is given, linv[256 t + 16 i + j] receives the inverse of the t-th 16 x 16 diagonal
// block of L (padded with the identity).
// A pivot <= 0 or NaN reports `code` (the smallest code wins) and the factorization
// continues with pivot 1 so that every wave still finishes.
// smem: kPotrfSmemFixed doubles (diagonal block and tile flags), then panel_cap*17
// doubles for the panel.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void wg_potrf_partial(double* __restrict__ A, int ld, int n, int p, double* smem,
                                                 int panel_cap, unsigned long long* err, unsigned long long code,
                                                 int32_t* __restrict__ ext, double* __restrict__ linv = nullptr) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* Li = smem + 16 * 17;                           // inverse of the diagonal block
    int* tnz = reinterpret_cast<int*>(smem + 2 * 16 * 17); // kPotrfMaxTiles flags
    double* Pl = smem + kPotrfSmemFixed;
    // the diagonal block at c0 is factored and inverted by wave 0 in registers (lane i < 16
    // holds row i of the block; rows past the last pivot are padded with the identity)
    auto factor_diag = [&](int c0) {
        const int j0 = c0, jb = min(16, p - c0);
        if (wave == 0) {
            double a[16], li[16];
#pragma unroll
            for (int c = 0; c < 16; ++c)
                a[c] = (lane < jb && c <= lane) ? A[(j0 + lane) + static_cast<size_t>(j0 + c) * ld]
                                                : (lane == c ? 1.0 : 0.0);
            wave_chol_inv16(a, li, lane, err, code);
            if (lane < jb) {
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c <= lane) A[(j0 + lane) + static_cast<size_t>(j0 + c) * ld] = a[c];
            }
            if (lane < 16) {
#pragma unroll
                for (int i = 0; i < 16; ++i) Li[i * 17 + lane] = li[i];
                if (linv != nullptr) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) linv[(j0 >> 4) * 256 + i * 16 + lane] = li[i];
                }
            }
        }
    };
    // one 16 x 16 tile (ti, tj) of the update A[j1:n, j1:p] -= P P[0:mi]^T (lower part) after the
    // panel at j0 (jb columns)
    auto update_tile = [&](int j0, int jb, int ti, int tj, bool lds_panel) {
        const int j1 = j0 + jb, m = n - j1, mi = p - j1;
        const int ra = ti * 16 + (lane & 15);
        const int rb = tj * 16 + (lane & 15);
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const int k = kk + (lane >> 4);
            double av = 0.0, bv = 0.0;
            if (k < jb) {
                if (lds_panel) {
                    if (ra < m) av = Pl[ra * 17 + k];
                    if (rb < m) bv = Pl[rb * 17 + k];
                } else {
                    if (ra < m) av = A[(j1 + ra) + static_cast<size_t>(j0 + k) * ld];
                    if (rb < m) bv = A[(j1 + rb) + static_cast<size_t>(j0 + k) * ld];
                }
            }
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        // lane holds D[lane/16 + 4 q][lane % 16], q = 0..3
        const int col = tj * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = ti * 16 + (lane >> 4) + 4 * q;
            if (row < m && col < mi && row >= col) A[(j1 + row) + static_cast<size_t>(j1 + col) * ld] -= acc[q];
        }
    };
    // Right-looking over 16-column blocks with look-ahead: after the panel of a block, its
    // update first covers the next block column; then wave 0 factors the next diagonal block
    // while the other waves update the rest. Every tile is computed as without look-ahead.
    int jp = -1, jbp = 0, ntp = 0, ntip = 0;   // the previous block and its update's tile counts
    bool ldsp = false;
    for (int j0 = 0;; j0 += 16) {
        if (wave == 0) {
            if (j0 < p) factor_diag(j0);
        } else if (jp >= 0) {
            for (int t = wave - 1; t < ntp * ntip; t += kWaves - 1) {
                const int tj = t % ntip, ti = t / ntip;
                if (tj == 0 || ti < tj || !tnz[ti] || !tnz[tj]) continue;
                update_tile(jp, jbp, ti, tj, ldsp);
            }
        }
        __syncthreads();
        if (j0 >= p) break;
        const int jb = min(16, p - j0);
        const int j1 = j0 + jb;
        const int m = n - j1;       // rows below the diagonal block
        const int mi = p - j1;      // pivot columns still to come
        // (2) panel: the rows below the diagonal block solve  x L_blk^T = a.
        const bool lds_panel = (m <= panel_cap);
        const int nt = (m + 15) >> 4;
        for (int e = tid; e < nt; e += kWG) tnz[e] = 0;
        __syncthreads();
        // rows below the block become  P = A_panel L_blk^-T  (16-row tiles on the matrix
        // cores; lane holds P[lane/16 + 4 q][lane % 16])
        for (int ti = wave; ti < nt; ti += kWaves) {
            const int ra = ti * 16 + (lane & 15);
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const int k = kk + (lane >> 4);
                const double av = (ra < m && k < jb) ? A[(j1 + ra) + static_cast<size_t>(j0 + k) * ld] : 0.0;
                const double bv = Li[(lane & 15) * 17 + k];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
            const int c = lane & 15;
            bool nz = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = ti * 16 + (lane >> 4) + 4 * q;
                if (r < m && c < jb) {
                    A[(j1 + r) + static_cast<size_t>(j0 + c) * ld] = acc[q];
                    nz = nz || acc[q] != 0.0;
                }
                if (lds_panel && r < m) Pl[r * 17 + c] = (c < jb) ? acc[q] : 0.0;
            }
            if (__any(nz) && lane == 0) tnz[ti] = 1;
        }
        __syncthreads();
        if (ext != nullptr && tid == 0) {
            int e = j1;
            for (int t = 0; t < (mi + 15) / 16; ++t)
                if (tnz[t]) e = min(p, j1 + 16 * (t + 1));
            ext[j0 >> 4] = e;
        }
        // (3) update of the remaining pivot columns A[j1:n, j1:p] -= P P[0:mi]^T: here the next
        //     block column (tj = 0), the rest at the top of the next round
        const int nti = (mi + 15) >> 4;
        if (nti > 0) {
            for (int ti = wave; ti < nt; ti += kWaves)
                if (tnz[ti] && tnz[0]) update_tile(j0, jb, ti, 0, lds_panel);
            __syncthreads();
        }
        jp = j0;
        jbp = jb;
        ntp = nt;
        ntip = nti;
        ldsp = lds_panel;
    }
    // (4) the Schur complement, S -= W^T W over the p pivots, lower tiles on the matrix cores.
    //     16-column blocks of W^T are staged in LDS (when its rows fit the panel buffer);
    //     every wave accumulates a batch of kSyrkBatch tiles over all pivots.
    const int ms = n - p;
    const int nts = (ms + 15) >> 4;
    const int ntl = nts * (nts + 1) / 2;
    const bool lds_w = ms <= panel_cap;
    for (int base = 0; base < ntl; base += kWaves * kSyrkBatch) {
        v4d acc[kSyrkBatch];
        int tiq[kSyrkBatch], tjq[kSyrkBatch];
#pragma unroll
        for (int q = 0; q < kSyrkBatch; ++q) {
            acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
            const int t = base + wave * kSyrkBatch + q;
            int ti = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
            while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
            while (ti * (ti + 1) / 2 > t) --ti;
            tiq[q] = t < ntl ? ti : -1;
            tjq[q] = t - ti * (ti + 1) / 2;
        }
        for (int k0 = 0; k0 < p; k0 += 16) {
            const int kb = min(16, p - k0);
            if (lds_w) {
                __syncthreads();
                for (int e = tid; e < ms * 16; e += kWG) {
                    const int r = e % ms, c = e / ms;
                    Pl[r * 17 + c] = (c < kb) ? A[(p + r) + static_cast<size_t>(k0 + c) * ld] : 0.0;
                }
                __syncthreads();
            }
#pragma unroll
            for (int q = 0; q < kSyrkBatch; ++q) {
                if (tiq[q] < 0) continue;
                const int ra = tiq[q] * 16 + (lane & 15);
                const int rb = tjq[q] * 16 + (lane & 15);
#pragma unroll
                for (int kk = 0; kk < 16; kk += 4) {
                    const int k = kk + (lane >> 4);
                    double av = 0.0, bv = 0.0;
                    if (k < kb) {
                        if (lds_w) {
                            if (ra < ms) av = Pl[ra * 17 + k];
                            if (rb < ms) bv = Pl[rb * 17 + k];
                        } else {
                            if (ra < ms) av = A[(p + ra) + static_cast<size_t>(k0 + k) * ld];
                            if (rb < ms) bv = A[(p + rb) + static_cast<size_t>(k0 + k) * ld];
                        }
                    }
                    acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kSyrkBatch; ++q) {
            if (tiq[q] < 0) continue;
            const int col = tjq[q] * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = tiq[q] * 16 + (lane >> 4) + 4 * r;
                if (row < ms && col < ms && row >= col)
                    A[(p + row) + static_cast<size_t>(p + col) * ld] -= acc[q][r];
            }
        }
    }
    __syncthreads();
    // the Schur complement in full
    for (int e = tid; e < ms * ms; e += kWG) {
        const int i = e % ms, j = e / ms;
        if (i < j) A[(p + i) + static_cast<size_t>(p + j) * ld] = A[(p + j) + static_cast<size_t>(p + i) * ld];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Workgroup-collective column-pivoted Householder QR for the interpolative decomposition
// (Sec. 2.2). M (r x n) is row-major with row stride ldr, in LDS or global memory.
// Thread t owns column slot t % cw over row chunk t / cw, cw = min(64, the next power of
// two >= n); with n > 64 it owns the columns slot, slot + 64, ... Columns are never moved:
// pos[c] is the current position of column c in the pivoted order and perm[j] the column at
// position j, kept as a QR that swaps columns would keep them. Step j takes, among the
// columns not chosen yet, the largest 2-norm over rows j.. (recomputed from the current
// values every step; ties to the lowest current position) and continues while
// R_jj > eps R_11. Returns the rank k; row i <= j of column perm[j] then holds R[i][j].
// part: 2 * 256 * ceil(n / cw) doubles.
// ---------------------------------------------------------------------------------------
template <int UR, typename MR>
__device__ __forceinline__ int wg_cpqr_rows(MR* __restrict__ M, int ldr, int r, int n, double eps, int* pos,
                                            int* perm, double* part_) {
    MR* part = reinterpret_cast<MR*>(part_);
    const int tid = threadIdx.x, lane = tid & 63;
    int cw = 1;
    while (cw < n && cw < 64) cw <<= 1;
    const int nrc = kWG / cw;
    const int cl = tid % cw, rc = tid / cw;
    const int cs = (r + nrc - 1) / nrc;
    const int i0 = rc * cs, i1 = min(r, i0 + cs);
    const int nblk = (n + cw - 1) / cw;
    MR* pd = part;                 // dot partials  [blk][rc][cl]
    MR* pn = part + nblk * kWG;    // norm partials [blk][rc][cl]
    for (int c = tid; c < n; c += kWG) {
        pos[c] = c;
        perm[c] = c;
    }
    for (int blk = 0; blk < nblk; ++blk) {
        const int c = blk * cw + cl;
        MR sq = 0.0, sq1 = 0.0;
        if (c < n) {
            int i = i0;
            for (; i + 1 < i1; i += 2) {
                const MR v = M[static_cast<size_t>(i) * ldr + c], u = M[static_cast<size_t>(i + 1) * ldr + c];
                sq += v * v;
                sq1 += u * u;
            }
            if (i < i1) sq += M[static_cast<size_t>(i) * ldr + c] * M[static_cast<size_t>(i) * ldr + c];
        }
        pn[blk * kWG + tid] = sq + sq1;
    }
    __syncthreads();
    const int kmax = min(r, n);
    MR r11 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        // (a) pivot among the columns with pos >= j; every wave reduces the same partials in
        //     the same order, so all of them reach the same choice without a barrier
        MR best = -1;
        int bpos = 0x7fffffff, bc = -1;
        for (int c = lane; c < n; c += 64) {
            const int pp = pos[c];
            if (pp < j) continue;
            const int blk = c / cw, sl = c % cw;
            MR v = 0.0;
            for (int q = 0; q < nrc; ++q) v += pn[blk * kWG + q * cw + sl];
            if (v > best || (v == best && pp < bpos)) {
                best = v;
                bpos = pp;
                bc = c;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const MR ob = __shfl_xor(best, off, 64);
            const int op = __shfl_xor(bpos, off, 64);
            const int oc = __shfl_xor(bc, off, 64);
            if (ob > best || (ob == best && op < bpos)) {
                best = ob;
                bpos = op;
                bc = oc;
            }
        }
        const MR nrm = sqrt(best);
        const int pc = bc;
        if (j == 0) r11 = nrm;
        if (!(nrm > static_cast<MR>(eps) * r11)) break;
        // (b) reflector of column pc over rows j..: v = (x0 - alpha, x1, ...), beta = 2 / v^T v
        const MR x0 = M[static_cast<size_t>(j) * ldr + pc];
        const MR alpha = -copysign(nrm, x0);
        const MR v0 = x0 - alpha;
        const MR beta = MR(1) / (nrm * (nrm + fabs(x0)));
        // rows of this thread's chunk below row j (row j itself is handled apart)
        const bool has_j = (i0 <= j && j < i1);
        const int ib = max(i0, j + 1);
        // (c) w_c = v^T M[j:, c] for the columns still to choose (the test below gives the
        //     same answer before and after the position update of this step)
        for (int blk = 0; blk < nblk; ++blk) {
            const int c = blk * cw + cl;
            MR w = 0.0;
            if (c < n && c != pc && pos[c] >= j) {
                MR w1 = 0.0, w2 = 0.0, w3 = 0.0;
                if (has_j) w = v0 * M[static_cast<size_t>(j) * ldr + c];
                // rows by rounds of UR (then at most one of eight), every load of a round issued
                // before its products; row i goes to the accumulator of i mod 4
                auto round = [&](auto cu, int i) {
                    constexpr int R = decltype(cu)::value;
                    const MR* Mi = M + static_cast<size_t>(i) * ldr;
                    MR a[R], b[R];
#pragma unroll
                    for (int u = 0; u < R; ++u) {
                        a[u] = Mi[u * ldr + pc];
                        b[u] = Mi[u * ldr + c];
                    }
#pragma unroll
                    for (int u = 0; u < R; u += 4) {
                        w += a[u] * b[u];
                        w1 += a[u + 1] * b[u + 1];
                        w2 += a[u + 2] * b[u + 2];
                        w3 += a[u + 3] * b[u + 3];
                    }
                };
                int i = ib;
                for (; i + UR - 1 < i1; i += UR) round(std::integral_constant<int, UR>{}, i);
                if (UR > 8 && i + 7 < i1) {
                    round(std::integral_constant<int, 8>{}, i);
                    i += 8;
                }
                for (; i < i1; ++i) w += M[static_cast<size_t>(i) * ldr + pc] * M[static_cast<size_t>(i) * ldr + c];
                w += (w1 + w2) + w3;
            }
            pd[blk * kWG + tid] = w;
        }
        __syncthreads();
        // (d) M[j:, c] -= beta w_c v, and the new squared norms over rows j+1..
        for (int blk = 0; blk < nblk; ++blk) {
            const int c = blk * cw + cl;
            if (c < n && c != pc && pos[c] >= j) {
                MR f = 0.0;
                for (int q = 0; q < nrc; ++q) f += pd[blk * kWG + q * cw + cl];
                f *= beta;
                if (has_j) M[static_cast<size_t>(j) * ldr + c] -= f * v0;
                MR sq = 0.0, sq1 = 0.0, sq2 = 0.0, sq3 = 0.0;
                auto round = [&](auto cu, int i) {
                    constexpr int R = decltype(cu)::value;
                    MR* Mi = M + static_cast<size_t>(i) * ldr;
                    MR a[R], b[R];
#pragma unroll
                    for (int u = 0; u < R; ++u) {
                        a[u] = Mi[u * ldr + pc];
                        b[u] = Mi[u * ldr + c];
                    }
#pragma unroll
                    for (int u = 0; u < R; ++u) {
                        b[u] -= f * a[u];
                        Mi[u * ldr + c] = b[u];
                    }
#pragma unroll
                    for (int u = 0; u < R; u += 4) {
                        sq += b[u] * b[u];
                        sq1 += b[u + 1] * b[u + 1];
                        sq2 += b[u + 2] * b[u + 2];
                        sq3 += b[u + 3] * b[u + 3];
                    }
                };
                int i = ib;
                for (; i + UR - 1 < i1; i += UR) round(std::integral_constant<int, UR>{}, i);
                if (UR > 8 && i + 7 < i1) {
                    round(std::integral_constant<int, 8>{}, i);
                    i += 8;
                }
                for (; i < i1; ++i) {
                    const MR nv = M[static_cast<size_t>(i) * ldr + c] - f * M[static_cast<size_t>(i) * ldr + pc];
                    M[static_cast<size_t>(i) * ldr + c] = nv;
                    sq += nv * nv;
                }
                pn[blk * kWG + tid] = sq + ((sq1 + sq2) + sq3);
            }
        }
        if (tid == 0) {
            M[static_cast<size_t>(j) * ldr + pc] = alpha;
            const int q = pos[pc], cj = perm[j];
            perm[j] = pc;
            perm[q] = cj;
            pos[cj] = q;
            pos[pc] = j;
        }
        __syncthreads();
        k = j + 1;
    }
    __syncthreads();
    return k;
}

// ---------------------------------------------------------------------------------------
// The same column-pivoted Householder QR as wg_cpqr_rows (pivot rule, ties, stopping test,
// reflector, R left in M) for n <= 64, with the matrix in registers: thread t owns column
// t % cw over row chunk t / cw (the layout above) and holds its cs <= RPT entries, so that a
// step reads no matrix entry from memory. Row j, the row a step works on, is kept apart: at
// the end of step j - 1 the chunk holding row j moves it to LDS (rowj) and shifts its registers
// down by one, so the registers hold exactly the rows below j (and zeros) and the row loops
// run over all of them with no bounds. Then
//   w_c = v0 rowj[c] + sum over the registers of piv_i x_i(c),   x_i(c) -= beta w_c piv_i,
// piv being the pivot column's entry of the same row (read from the lane that holds it: a lane
// read when cw = 64, one chunk per wave; a wave shuffle otherwise), and row j of R follows from
// rowj. Column sums are reduced over the wave's chunks by butterflies and over the four waves
// through LDS in a fixed order, so every thread holds the same sums and takes the same pivot.
// part: 9 * 64 values of MR (per-wave dot and norm sums, rowj).
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T lane_value(T v, int l) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b), l));
        const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), l));
        return __builtin_bit_cast(T, (static_cast<unsigned long long>(hi) << 32) | lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    }
}

// v of the lane given by the DPP pattern CTRL (within a row of 16 lanes)
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_value(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
        return __builtin_bit_cast(T, (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                         static_cast<unsigned>(lo));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF,
                                                                 false));
    }
}

template <int RPT, typename MR, bool UNI>
__device__ __forceinline__ int wg_cpqr_regs(MR* __restrict__ M, int ldr, int r, int n, double eps, int* pos,
                                            int* perm, double* part_) {
    MR* part = reinterpret_cast<MR*>(part_);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int cw = 64;
    if constexpr (!UNI) {
        cw = 1;
        while (cw < n && cw < 64) cw <<= 1;
    }
    const int nrc = kWG / cw;
    const int cl = UNI ? lane : tid % cw;
    const int rc = UNI ? wave : tid / cw;
    const int cs = (r + nrc - 1) / nrc;
    const int i0 = rc * cs, i1 = min(r, i0 + cs);
    const bool own = cl < n;
    const int base = UNI ? 0 : (lane & ~(cw - 1));   // first lane of this thread's chunk in the wave
    MR* pw = part;                                   // [wave][64] dot sums
    MR* pq = part + 4 * 64;                          // [wave][64] squared-norm sums
    MR* rowj = part + 8 * 64;                        // row j of every column
    auto wave_col_sum = [&](MR v) {
        if constexpr (!UNI)
            for (int off = 32; off >= cw; off >>= 1) v += __shfl_xor(v, off, 64);
        return v;
    };
    auto piv = [&](MR xu, int src) -> MR {
        if constexpr (UNI) return lane_value(xu, src);
        else return __shfl(xu, base + src, 64);
    };
    MR x[RPT];
    // row `row` to rowj: its chunk's registers hold it first and shift down by one
    auto take = [&](int row) {
        if (rc == row / cs) {
            if (own) rowj[cl] = x[0];
#pragma unroll
            for (int u = 0; u + 1 < RPT; ++u) x[u] = x[u + 1];
            x[RPT - 1] = MR(0);
        }
    };
    MR s0 = 0, s1 = 0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int i = i0 + u;
        x[u] = (own && i < i1) ? M[static_cast<size_t>(i) * ldr + cl] : MR(0);
        if (u & 1) s1 += x[u] * x[u];
        else s0 += x[u] * x[u];
    }
    {
        const MR sq = wave_col_sum(s0 + s1);
        if (lane < cw) pq[wave * 64 + cl] = sq;
    }
    if (r > 0) take(0);
    for (int c = tid; c < n; c += kWG) {
        pos[c] = c;
        perm[c] = c;
    }
    int mypos = cl;
    __syncthreads();
    const int kmax = min(r, n);
    MR r11 = 0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        // (a) pivot: the largest squared norm among columns at positions >= j, ties to the
        //     lowest position; the same in every lane of every wave
        const MR nrm2 = (pq[cl] + pq[64 + cl]) + (pq[128 + cl] + pq[192 + cl]);
        const bool cand = own && mypos >= j;
        MR best = cand ? nrm2 : MR(-1);
        int bpos = cand ? mypos : 0x7fffffff, bc = cl;
        auto keep_max = [&](MR ob, int op, int oc) {
            const bool tk = ob > best || (ob == best && op < bpos);
            best = tk ? ob : best;
            bpos = tk ? op : bpos;
            bc = tk ? oc : bc;
        };
        // butterfly over the cw lanes of a chunk: lane ^ 1, lane ^ 2 (quad permutes), the
        // mirrored lane in the half row and in the row (DPP), then lane ^ 16, lane ^ 32
        if (cw > 1) keep_max(dpp_value<0xB1>(best), dpp_value<0xB1>(bpos), dpp_value<0xB1>(bc));
        if (cw > 2) keep_max(dpp_value<0x4E>(best), dpp_value<0x4E>(bpos), dpp_value<0x4E>(bc));
        if (cw > 4) keep_max(dpp_value<0x141>(best), dpp_value<0x141>(bpos), dpp_value<0x141>(bc));
        if (cw > 8) keep_max(dpp_value<0x140>(best), dpp_value<0x140>(bpos), dpp_value<0x140>(bc));
        if (cw > 16) keep_max(__shfl_xor(best, 16, 64), __shfl_xor(bpos, 16, 64), __shfl_xor(bc, 16, 64));
        if (cw > 32) keep_max(__shfl_xor(best, 32, 64), __shfl_xor(bpos, 32, 64), __shfl_xor(bc, 32, 64));
        const int pc = __builtin_amdgcn_readfirstlane(bc);
        const int q = __builtin_amdgcn_readfirstlane(bpos);
        const MR nrm = sqrt(lane_value(best, 0));
        if (j == 0) r11 = nrm;
        if (!(nrm > static_cast<MR>(eps) * r11)) break;
        if (tid == 0) {
            const int qq = pos[pc], cj = perm[j];
            perm[j] = pc;
            perm[qq] = cj;
            pos[cj] = qq;
            pos[pc] = j;
        }
        // (b) reflector of column pc over rows j..: v = (x0 - alpha, x1, ...), beta = 2 / v^T v
        const MR xj = rowj[cl];
        const MR x0 = lane_value(rowj[pc], 0);
        const MR alpha = -copysign(nrm, x0);
        const MR v0 = x0 - alpha;
        const MR beta = MR(1) / (nrm * (nrm + fabs(x0)));
        const bool act = own && cl != pc && mypos >= j;
        // (c) w_c = v^T M[j:, c]: rows > j from the registers, row j from rowj
        MR wa = 0, wb = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            if (u & 1) wb += piv(x[u], pc) * x[u];
            else wa += piv(x[u], pc) * x[u];
        }
        {
            const MR ws = wave_col_sum(wa + wb);
            if (lane < cw) pw[wave * 64 + cl] = ws;
        }
        __syncthreads();
        // (d) M[j:, c] -= beta w_c v (columns not chosen yet), and the new squared norms over
        //     rows j+1..; the pivot is read back from perm so that no copy of its entries stays
        //     live across the barrier
        const int pcu = __builtin_amdgcn_readfirstlane(perm[j]);
        const MR f = beta * (((pw[cl] + pw[64 + cl]) + (pw[128 + cl] + pw[192 + cl])) + v0 * xj);
        const MR fa = act ? f : MR(0);
        MR n0 = 0, n1 = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            x[u] -= fa * piv(x[u], pcu);
            if (u & 1) n1 += x[u] * x[u];
            else n0 += x[u] * x[u];
        }
        {
            const MR sq = wave_col_sum(n0 + n1);
            if (lane < cw) pq[wave * 64 + cl] = sq;
            // row j of R: final after this step
            if (tid < n) M[static_cast<size_t>(j) * ldr + cl] = act ? xj - f * v0 : (cl == pc ? alpha : xj);
        }
        // row j + 1 to rowj (its reads of this step came before the first barrier)
        if (j + 1 < r) take(j + 1);
        if (cl == pc) mypos = j;
        else if (mypos == j) mypos = q;
        __syncthreads();
        k = j + 1;
    }
    __syncthreads();
    return k;
}

// ---------------------------------------------------------------------------------------
// Adjoint of the solve with respect to the log-coefficients theta = log a (one thread per
// grid cell). A depends on a_c through the cell's share of the stencil (eq. (1.1) with the
// edge rule of the assembly below): every grid edge (x, x + e_k) of cell c carries
// a_c 2^(1-d) / h^2 of its edge coefficient, so
//   lambda^T (dA/da_c) u = 2^(1-d) h^-2 sum over the cell's edges of
//                          (lambda(x + e_k) - lambda(x)) (u(x + e_k) - u(x))
// (values at the Dirichlet ghosts are 0) and the gradient of a loss L(u) with
// A lambda = dL/du is dL/dtheta_c = -a_c lambda^T (dA/da_c) u. Cell c = (c_1..c_d),
// c_k in 0..s, x_1 fastest, has corners x_k in {c_k, c_k + 1}.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double grid_value(const double* v, int d, int s, const int* x) {
    int64_t lin = 0, mul = 1;
    for (int k = 0; k < d; ++k) {
        if (x[k] < 1 || x[k] > s) return 0.0;
        lin += static_cast<int64_t>(x[k] - 1) * mul;
        mul *= s;
    }
    return v[lin];
}

__global__ __launch_bounds__(256) void k_grad_log_a(int d, int s, double inv_h2, const double* __restrict__ a,
                                                    const double* __restrict__ u, const double* __restrict__ lam,
                                                    double* __restrict__ g) {
    int64_t nc = 1;
    for (int k = 0; k < d; ++k) nc *= (s + 1);
    for (int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; c < nc;
         c += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int cc[3] = {0, 0, 0};
        int64_t r = c;
        for (int k = 0; k < d; ++k) {
            cc[k] = static_cast<int>(r % (s + 1));
            r /= (s + 1);
        }
        double acc = 0.0;
        for (int k = 0; k < d; ++k) {
            // the 2^(d-1) edges along axis k: the other coordinates at c_j or c_j + 1
            for (int t = 0; t < (1 << (d - 1)); ++t) {
                int x[3], y[3];
                int bit = 0;
                for (int j = 0; j < d; ++j) {
                    if (j == k) {
                        x[j] = cc[j];
                        y[j] = cc[j] + 1;
                    } else {
                        x[j] = y[j] = cc[j] + ((t >> bit) & 1);
                        ++bit;
                    }
                }
                const double du = grid_value(u, d, s, y) - grid_value(u, d, s, x);
                const double dl = grid_value(lam, d, s, y) - grid_value(lam, d, s, x);
                acc += dl * du;
            }
        }
        g[c] = -a[c] * acc * inv_h2 / static_cast<double>(1 << (d - 1));
    }
}

// ---------------------------------------------------------------------------------------
// Assembly of A = h^-2 K(a) + diag(b) (5-point / 7-point, Sec. 3.1 / 3.2): one thread per
// row; the row pointer was filled on the host.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double edge_coef(const double* a, int d, int s, int k, const int* x, int xk) {
#pragma clang fp contract(off)
    // mean of the 2^(d-1) cells containing the grid edge from (.., xk, ..) to (.., xk+1, ..)
    // along axis k: cell c_k = xk, c_j in {x_j - 1, x_j} for j != k (last other axis fastest)
    const int s1 = s + 1;
    double acc = 0.0;
    int oth[2];
    int no = 0;
    for (int j = 0; j < d; ++j)
        if (j != k) oth[no++] = j;
    const int combos = 1 << no;
    for (int t = 0; t < combos; ++t) {
        int64_t lin = 0, mul = 1;
        for (int j = 0; j < d; ++j) {
            int cj;
            if (j == k) {
                cj = xk;
            } else {
                const int which = (j == oth[0]) ? (no == 2 ? ((t >> 1) & 1) : (t & 1)) : (t & 1);
                cj = x[j] - 1 + which;
            }
            lin += cj * mul;
            mul *= s1;
        }
        acc += a[lin];
    }
    return acc / static_cast<double>(combos);
}

// Row pointer of the 5-/7-point matrix in closed form: row i holds 1 + sum_k [x_k > 1] + [x_k < s]
// entries, so the rows before i hold i (1 + 2d) entries less, per axis k, one for every row
// j < i on the first plane x_k = 1 and one for every row on the last plane x_k = s; with
// stride t = s^k such rows come in runs of t every s t rows.
__global__ __launch_bounds__(256) void k_fd_rowptr(int d, int s, int32_t* __restrict__ row_ptr) {
    int64_t N = 1;
    for (int k = 0; k < d; ++k) N *= s;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i <= N;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t v = i * (1 + 2 * d), t = 1;
        for (int k = 0; k < d; ++k) {
            const int64_t q = i / (t * s), r = i % (t * s);
            const int64_t first = q * t + (r < t ? r : t);
            const int64_t last = q * t + (r > (s - 1) * t ? r - (s - 1) * t : 0);
            v -= first + last;
            t *= s;
        }
        row_ptr[i] = static_cast<int32_t>(v);
    }
}

__global__ __launch_bounds__(256) void k_assemble_fd(int d, int s, double inv_h2, const double* __restrict__ a,
                                                     const double* __restrict__ b, const int32_t* __restrict__ row_ptr,
                                                     int32_t* __restrict__ col, double* __restrict__ val) {
#pragma clang fp contract(off)
    const int64_t N = (d == 2) ? static_cast<int64_t>(s) * s : static_cast<int64_t>(s) * s * s;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int x[3];
        int64_t r = i;
        for (int k = 0; k < d; ++k) {
            x[k] = static_cast<int>(r % s) + 1;
            r /= s;
        }
        double diag = 0.0;
        double off_lo[3], off_hi[3];
        for (int k = 0; k < d; ++k) {
            const double lo = edge_coef(a, d, s, k, x, x[k] - 1) * inv_h2;
            const double hi = edge_coef(a, d, s, k, x, x[k]) * inv_h2;
            diag = diag + (lo + hi);
            off_lo[k] = -lo;
            off_hi[k] = -hi;
        }
        if (b != nullptr) diag = diag + b[i];
        int64_t stride[3] = {1, s, static_cast<int64_t>(s) * s};
        int e = row_ptr[i];
        for (int k = d - 1; k >= 0; --k)
            if (x[k] > 1) {
                col[e] = static_cast<int32_t>(i - stride[k]);
                val[e] = off_lo[k];
                ++e;
            }
        col[e] = static_cast<int32_t>(i);
        val[e] = diag;
        ++e;
        for (int k = 0; k < d; ++k)
            if (x[k] < s) {
                col[e] = static_cast<int32_t>(i + stride[k]);
                val[e] = off_hi[k];
                ++e;
            }
    }
}

// ---------------------------------------------------------------------------------------
// Level-0 frontal unknowns: position p of cell c gets its grid index from the closed form
// leaf_frontal_dof (interior box, then the boundary boxes by slot code), one thread per
// position.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_leaf_dofs(const CellRef* __restrict__ cells, int d, int s, int w, int nc1,
                                                   int32_t* __restrict__ cdofs) {
    const CellRef cr = cells[blockIdx.x];
    for (int p = threadIdx.x; p < cr.nf; p += kWG)
        cdofs[cr.dptr + p] = leaf_frontal_dof(d, s, w, nc1, static_cast<int>(blockIdx.x), p);
}

// ---------------------------------------------------------------------------------------
// Level-0 frontal assembly: frontal element (p, q) of cell c is A[i, j] (i, j its unknowns)
// when c is the first cell (lowest index) whose closure contains both i and j, else 0.
// Every entry of A lands in exactly one frontal, so the frontals add up to A.
// One workgroup per tile (Tile::shape); with kTileBand only the elements of the diagonal
// and first subdiagonal 16 x 16 blocks are written. The coordinates and the range of cells
// whose closure holds each of the tile's column unknowns are staged in LDS once per tile.
// ---------------------------------------------------------------------------------------
// Coordinates x_k (1-based) of unknown i and, per axis, the cells lo_k..hi_k whose
// closure holds it (a coordinate on a cell boundary belongs to both neighbours).
__device__ __forceinline__ void unknown_cells(int i, int d, int s, int w, int nc1, int* x, int* lo, int* hi) {
    int rr = i;
    for (int k = 0; k < 3; ++k) {
        x[k] = 0;
        lo[k] = hi[k] = 0;
        if (k < d) {
            const int a = rr % s + 1;
            rr /= s;
            x[k] = a;
            const int c = a / w;
            const bool on = (a % w) == 0;
            lo[k] = on ? max(c - 1, 0) : c;
            hi[k] = on ? min(c, nc1 - 1) : c;
        }
    }
}

__global__ __launch_bounds__(256) void k_front_csr(const Tile* __restrict__ tiles, const CellRef* __restrict__ cells,
                                                   const int32_t* __restrict__ cdofs, int d, int s, int w, int nc1,
                                                   const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, double* __restrict__ F) {
    __shared__ int cq_info[64 * 10];   // per tile column: unknown, x[3], lo[3], hi[3]
    const Tile t = tiles[blockIdx.x];
    const CellRef cr = cells[t.cell];
    const int nf = cr.nf;
    const int nrow = t.shape ? (t.shape >> 8) & 0xff : 64, ncol = t.shape ? t.shape & 0xff : 64;
    const bool band = (t.shape & kTileBand) != 0;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        const int q = t.c0 + lane;
        int* ci = cq_info + lane * 10;
        if (lane < ncol && q < nf) {
            const int j = cdofs[cr.dptr + q];
            ci[0] = j;
            unknown_cells(j, d, s, w, nc1, ci + 1, ci + 4, ci + 7);
        }
    }
    const int p = t.r0 + lane;
    const bool prow = lane < nrow && p < nf;
    int i = 0, xi[3], alo[3], ahi[3];
    // the row's matrix entries (a stencil row has at most 2d + 1 <= 7), held in registers;
    // longer rows are searched in memory
    int rc[7];
    double rv[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        rc[k] = -1;
        rv[k] = 0.0;
    }
    bool longrow = false;
    if (prow) {
        i = cdofs[cr.dptr + p];
        unknown_cells(i, d, s, w, nc1, xi, alo, ahi);
        const int e0 = row_ptr[i], ne = row_ptr[i + 1] - e0;
        longrow = ne > 7;
#pragma unroll
        for (int k = 0; k < 7; ++k)
            if (k < ne) {
                rc[k] = col[e0 + k];
                rv[k] = val[e0 + k];
            }
    }
    __syncthreads();
    if (!prow) return;
    for (int cq = threadIdx.x >> 6; cq < ncol; cq += 4) {
        const int q = t.c0 + cq;
        if (q >= nf) break;
        if (band) {
            const int db = (p >> 4) - (q >> 4);
            if (db < 0 || db > 1) continue;
        }
        const int* ci = cq_info + cq * 10;
        int dist = 0;
        for (int k = 0; k < d; ++k) dist += abs(ci[1 + k] - xi[k]);
        double v = 0.0;
        if (dist <= 1) {
            // first common cell, axis by axis
            int64_t own = 0, mul = 1;
            bool ok = true;
            for (int k = 0; k < d; ++k) {
                const int lo = max(alo[k], ci[4 + k]), hi = min(ahi[k], ci[7 + k]);
                if (lo > hi) ok = false;
                own += lo * mul;
                mul *= nc1;
            }
            if (ok && own == t.cell) {
                const int j = ci[0];
                if (longrow) {
                    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                        if (col[e] == j) {
                            v = val[e];
                            break;
                        }
                } else {
#pragma unroll
                    for (int k = 6; k >= 0; --k)
                        if (rc[k] == j) v = rv[k];
                }
            }
        }
        F[cr.off + p + static_cast<size_t>(q) * cr.ld] = v;
    }
}

// ---------------------------------------------------------------------------------------
// Level >= 1 frontal assembly ("extend-add"): frontal element (p, q) of cell c is the sum,
// over the children of c whose closures contain both unknowns (ascending child index),
// of the children's Schur-complement shares.
// ---------------------------------------------------------------------------------------
// A child cell's place among its parent's children (bit k: its coordinate's parity on axis k).
__device__ __forceinline__ int child_rank(int c, int d, int pnc1) {
    int rel = 0;
    for (int k = 0; k < d; ++k) {
        rel |= ((c % pnc1) & 1) << k;
        c /= pnc1;
    }
    return rel;
}

__global__ __launch_bounds__(256) void k_front_extend(const Tile* __restrict__ tiles, const CellRef* __restrict__ cells,
                                                      const int32_t* __restrict__ src, int W, int d, int pnc1,
                                                      const CellRef* __restrict__ child, const double* __restrict__ Fc,
                                                      double* __restrict__ F) {
    // per column of the tile, its position in each child's frontal by the child's place among
    // the cell's children (-1: not in that child), staged once (W <= 8)
    __shared__ int32_t qt[64 * 8];
    const Tile t = tiles[blockIdx.x];
    const CellRef cr = cells[t.cell];
    const int nf = cr.nf;
    const int ncol = t.shape ? t.shape & 0xff : min(64, nf - t.c0);   // 64 x 64, or the tile's shape
    const int32_t* sc = src + static_cast<size_t>(cr.dptr + t.c0) * 2 * W;
    for (int e = threadIdx.x; e < ncol * W; e += kWG) qt[e] = -1;
    __syncthreads();
    for (int e = threadIdx.x; e < ncol * W; e += kWG) {
        const int c = sc[2 * e];
        if (c >= 0) qt[(e / W) * W + child_rank(c, d, pnc1)] = sc[2 * e + 1];
    }
    // the row's sources: child place, and the element offset of the row in that child's frontal
    const int p = t.r0 + (threadIdx.x & 63);
    const bool prow = p < nf;
    int pr[8], cld[8];
    int64_t coff[8];
    int np = 0;
    if (prow) {
        const int32_t* sp = src + static_cast<size_t>(cr.dptr + p) * 2 * W;
        for (int a = 0; a < W; ++a) {
            const int c = sp[2 * a];
            if (c < 0) break;
            const CellRef ch = child[c];
            pr[np] = child_rank(c, d, pnc1);
            coff[np] = ch.off + sp[2 * a + 1];
            cld[np] = ch.ld;
            ++np;
        }
    }
    __syncthreads();
    if (!prow) return;
    // four columns per thread and pass, every load of the pass issued before the sums; the
    // shares are added in the row's child order
    const int wave = threadIdx.x >> 6;
    for (int cq0 = wave; cq0 < ncol; cq0 += 16) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int cq = cq0 + 4 * u;
            v[u] = 0.0;
            if (cq >= ncol) continue;
            const int32_t* qc = qt + cq * W;
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                if (a >= np) break;
                const int off = qc[pr[a]];
                if (off >= 0) v[u] += Fc[coff[a] + static_cast<size_t>(off) * cld[a]];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int cq = cq0 + 4 * u;
            if (cq < ncol) F[cr.off + p + static_cast<size_t>(t.c0 + cq) * cr.ld] = v[u];
        }
    }
}

// ---------------------------------------------------------------------------------------
// Extend-add source table of a level >= 1 (read by k_front_extend): for frontal position p of
// cell c, the children of c whose closures hold the unknown (the cells of the level below
// that contain its group g2 there, in slot order) and the unknown's position t2 + the
// group's offset in each child's frontal; unused pairs are -1. One thread per position.
// Entries that contradict the plan (group out of range, no child or more than W, a position
// outside the child's boundary block) are reported as step 6 and left at -1.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_extend_src(const CellRef* __restrict__ cells, const int32_t* __restrict__ g2,
                                                    const int32_t* __restrict__ t2, int ngroups2,
                                                    const int32_t* __restrict__ gslot_cnt,
                                                    const int32_t* __restrict__ gslot_cell,
                                                    const int32_t* __restrict__ gslot_off,
                                                    const CellRef* __restrict__ child, int nchild, int d, int pnc1,
                                                    int nc1, int W, int level, int32_t* __restrict__ src,
                                                    unsigned long long* err) {
    const int c = blockIdx.x;
    const CellRef cr = cells[c];
    for (int p = threadIdx.x; p < cr.nf; p += kWG) {
        const int64_t e = static_cast<int64_t>(cr.dptr) + p;
        int32_t* o = src + e * 2 * W;
        for (int q = 0; q < 2 * W; ++q) o[q] = -1;
        const int g = g2[e], t = t2[e];
        if (g < 0 || g >= ngroups2) {
            report(err, err_code(level, 6, c));
            continue;
        }
        const int nsl = min(gslot_cnt[g], kMaxSlots);
        int nq = 0;
        bool ok = true;
        for (int sl = 0; sl < nsl; ++sl) {
            const int cc = gslot_cell[g * kMaxSlots + sl];
            if (cc < 0 || cc >= nchild) {
                ok = false;
                break;
            }
            // parent of child cc: its coordinates halved
            int rr = cc, par = 0, mul = 1;
            for (int k = 0; k < d; ++k) {
                par += ((rr % pnc1) >> 1) * mul;
                rr /= pnc1;
                mul *= nc1;
            }
            if (par != c) continue;
            const int pos = gslot_off[g * kMaxSlots + sl] + t;
            const CellRef ch = child[cc];
            if (nq >= W || pos < ch.nI || pos >= ch.nf) {
                ok = false;
                break;
            }
            o[2 * nq] = cc;
            o[2 * nq + 1] = pos;
            ++nq;
        }
        if (!ok || nq == 0) {
            for (int q = 0; q < 2 * W; ++q) o[q] = -1;
            report(err, err_code(level, 6, c));
        }
    }
}

// Batched partial Cholesky of cell frontals (cell elimination, Sec. 2.1) or of the root.
__global__ __launch_bounds__(256) void k_potrf_batch(const FrontDesc* __restrict__ desc, double* __restrict__ pool,
                                                     int panel_cap, int level, int step, unsigned long long* err,
                                                     int32_t* __restrict__ ext, double* __restrict__ linv) {
    extern __shared__ double smem[];
    const FrontDesc fd = desc[blockIdx.x];
    const bool has = fd.ext >= 0;
    wg_potrf_partial(pool + fd.off, fd.ld, fd.n, fd.p, smem, panel_cap, err, err_code(level, step, fd.id),
                     (ext != nullptr && has) ? ext + fd.ext : nullptr,
                     (linv != nullptr && has) ? linv + static_cast<size_t>(fd.ext) * 256 : nullptr);
}

// ---------------------------------------------------------------------------------------
// Leaf-cell elimination (eq. (2.1)) when A_II is banded with bandwidth <= 16 in its natural
// order (the interior box of a leaf cell: bandwidth = the box's row length), so that L is
// block bidiagonal in 16 x 16 blocks. For J = 0, 1, ...:
//   L_JJ = chol(D_JJ - L_J,J-1 L_J,J-1^T),  Li_J = L_JJ^-1,  L_J+1,J = D_J+1,J Li_J^T   (wave 0)
//   W^T_J = (X_J - W^T_J-1 L_J,J-1^T) Li_J^T        (16 boundary rows per wave and tile)
// then S = A_BB - W^T W on the matrix cores, both triangles written. These are the factors
// of the dense partial Cholesky; only the structural zeros outside the band are skipped.
// LDS (dynamic): L_J,J-1 double buffer (2 x 272), Li_J and L_JJ by parity (4 x 272), per
// wave a transfer tile (272) and tpw tiles of W^T_J-1 (tpw x 272), then two buffers of
// (2 + row tiles) x 272 for the next block's operands, loaded by waves 1..3 while wave 0
// factors the current block. Waves 1..3 also store block J's L_JJ and Li_J from LDS during
// round J + 1, so that wave 0 only factors.
// ---------------------------------------------------------------------------------------
// F32: the Schur product W^T W on the FP32 matrix cores with FP32 accumulation (operands
// rounded to FP32; L, W^T and S stay FP64).
template <bool F32>
__global__ __launch_bounds__(256) void k_leaf_elim(const FrontDesc* __restrict__ desc, double* __restrict__ pool,
                                                   double* __restrict__ linv, int tpw, int level,
                                                   unsigned long long* err, int32_t* __restrict__ ext) {
    extern __shared__ double smem[];
    constexpr int TS = 16 * 17;
    const FrontDesc fd = desc[blockIdx.x];
    double* A = pool + fd.off;
    const int ld = fd.ld, p = fd.p, m = fd.n - fd.p;
    const int nb = (p + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lh = lane >> 4;
    const int ntile = (m + 15) / 16;
    double* Lsb = smem;                 // [2][TS]: L_J,J-1 by parity of J
    double* Lis0 = smem + 2 * TS;       // [2][TS]: Li_J by parity of J, row-major
    double* Ljj0 = smem + 4 * TS;       // [2][TS]: L_JJ by parity of J, row-major
    double* Tw = smem + 6 * TS + wave * TS;                  // this wave's transfer tile
    double* Pw = smem + 10 * TS + static_cast<size_t>(wave) * tpw * TS;  // this wave's W^T_J-1 tiles
    // operands of block J, loaded during the previous block by waves 1..3 (by parity of J):
    // D_JJ (row-major), D_J+1,J (row-major) and the X_J row tiles (row-major per tile)
    double* Buf = smem + (10 + 4 * tpw) * TS;
    const int bufsz = (2 + ntile) * TS;
    double* lv = linv + static_cast<size_t>(fd.ext) * 256;
    const unsigned long long code = err_code(level, 0, fd.id);
    // S -= W^T W accumulated block by block in registers of waves 1..3 while wave 0 factors
    // the next diagonal block (up to kLeafTilesPerWave lower tiles per wave); otherwise
    // formed at the end from W^T in memory
    const int ntl = ntile * (ntile + 1) / 2;
    const bool inc = ntl <= 3 * kLeafTilesPerWave;
    v4d sacc[kLeafTilesPerWave];
    v4f saccf[kLeafTilesPerWave];
#pragma unroll
    for (int u = 0; u < kLeafTilesPerWave; ++u) {
        sacc[u] = v4d{0.0, 0.0, 0.0, 0.0};
        saccf[u] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }
    // row of register q of a 16 x 16 product tile (FP32: 4 (lane / 16) + q; FP64: lane / 16 + 4 q)
    auto prow = [&](int q) { return F32 ? 4 * lh + q : lh + 4 * q; };
    auto tile_ij = [](int t, int& ti, int& tj) {
        ti = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    };
    // rank-16 update with the W^T tiles of the block just finished (P tiles of every wave)
    auto syrk_step = [&]() {
#pragma unroll
        for (int u = 0; u < kLeafTilesPerWave; ++u) {
            const int t = (wave - 1) + 3 * u;
            if (t >= ntl) break;
            int ti, tj;
            tile_ij(t, ti, tj);
            const double* Pa = smem + 10 * TS + static_cast<size_t>(ti & 3) * tpw * TS + (ti >> 2) * TS;
            const double* Pb = smem + 10 * TS + static_cast<size_t>(tj & 3) * tpw * TS + (tj >> 2) * TS;
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                if constexpr (F32)
                    saccf[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(static_cast<float>(Pa[lr * 17 + kk + lh]),
                                                                   static_cast<float>(Pb[lr * 17 + kk + lh]),
                                                                   saccf[u], 0, 0, 0);
                else
                    sacc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(Pa[lr * 17 + kk + lh], Pb[lr * 17 + kk + lh],
                                                                  sacc[u], 0, 0, 0);
            }
        }
    };
    auto prefetch = [&](int J, int t0, int stride) {
        double* B = Buf + (J & 1) * bufsz;
        const int j0 = 16 * J, jb = min(16, p - j0), rb = min(16, p - j0 - 16);
        // 256 elements per 16 x 16 tile: element e = row * 16 + col
        for (int e = t0; e < (2 + ntile) * 256; e += stride) {
            const int tile = e >> 8, r = (e >> 4) & 15, c = e & 15;
            double v;
            if (tile == 0) v = (r < jb && c <= r) ? A[(j0 + r) + static_cast<size_t>(j0 + c) * ld] : 0.0;
            else if (tile == 1) v = (r < rb && c < jb) ? A[(j0 + 16 + r) + static_cast<size_t>(j0 + c) * ld] : 0.0;
            else {
                const int rr = 16 * (tile - 2) + r;
                v = (rr < m && c < jb) ? A[(p + rr) + static_cast<size_t>(j0 + c) * ld] : 0.0;
            }
            B[tile * TS + r * 17 + c] = v;
        }
    };
    // block K's L_KK (lower part) and Li_K from LDS to the frontal and linv, by waves 1..3
    auto store_diag = [&](int K) {
        const int k0 = 16 * K, kb = min(16, p - k0);
        const double* Lk = Ljj0 + (K & 1) * TS;
        const double* Ik = Lis0 + (K & 1) * TS;
        for (int e = threadIdx.x - 64; e < 256; e += kWG - 64) {
            const int r = e >> 4, c = e & 15;
            if (r < kb && c <= r) A[(k0 + r) + static_cast<size_t>(k0 + c) * ld] = Lk[r * 17 + c];
            lv[K * 256 + e] = Ik[r * 17 + c];
        }
        if (threadIdx.x == 64) ext[fd.ext + K] = min(p, k0 + 32);
    };
    prefetch(0, threadIdx.x, kWG);
    __syncthreads();
    for (int J = 0; J < nb; ++J) {
        const int j0 = 16 * J, jb = min(16, p - j0);
        const double* Lprev = Lsb + (J & 1) * TS;
        const double* B = Buf + (J & 1) * bufsz;
        double* Lis = Lis0 + (J & 1) * TS;
        double* Ljj = Ljj0 + (J & 1) * TS;
        if (wave == 0) {
            double a[16], li[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) a[c] = (lane < 16) ? B[lane * 17 + c] : 0.0;
            if (lane >= jb && lane < 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c) a[c] = (lane == c) ? 1.0 : 0.0;
            }
            if (J > 0) {
                // D_JJ -= L_J,J-1 L_J,J-1^T (rows and columns < jb are real)
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 16; kk += 4) {
                    const double x = Lprev[lr * 17 + kk + lh];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) Tw[(lh + 4 * q) * 17 + lr] = acc[q];
                __builtin_amdgcn_wave_barrier();
                if (lane < jb) {
#pragma unroll
                    for (int c = 0; c < 16; ++c)
                        if (c <= lane) a[c] -= Tw[lane * 17 + c];
                }
                __builtin_amdgcn_wave_barrier();
            }
            wave_chol_inv16(a, li, lane, err, code);
            if (lane < 16) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    Lis[i * 17 + lane] = li[i];
                    Ljj[lane * 17 + i] = a[i];
                }
            }
        } else {
            if (inc && J > 0) syrk_step();
            if (J > 0) store_diag(J - 1);
            if (J + 1 < nb) prefetch(J + 1, threadIdx.x - 64, kWG - 64);
        }
        __syncthreads();
        // W^T_J for this wave's row tiles
        int slot = 0;
        for (int t = wave; t < ntile; t += kWaves, ++slot) {
            const int r0 = 16 * t;
            double* P = Pw + slot * TS;
            const double* X = B + (2 + t) * TS;
            v4d acc;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = X[(lh + 4 * q) * 17 + lr];
            if (J > 0) {
#pragma unroll
                for (int kk = 0; kk < 16; kk += 4) {
                    const double av = -P[lr * 17 + kk + lh];
                    const double bv = Lprev[lr * 17 + kk + lh];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) Tw[(lh + 4 * q) * 17 + lr] = acc[q];
            __builtin_amdgcn_wave_barrier();
            v4d out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const double av = Tw[lr * 17 + kk + lh];
                const double bv = Lis[lr * 17 + kk + lh];
                out = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, out, 0, 0, 0);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + lh + 4 * q;
                P[(lh + 4 * q) * 17 + lr] = out[q];
                if (r < m && lr < jb) A[(p + r) + static_cast<size_t>(j0 + lr) * ld] = out[q];
            }
            __builtin_amdgcn_wave_barrier();
        }
        // L_J+1,J = D_J+1,J Li_J^T by wave 0, into the other buffer
        if (wave == 0 && J + 1 < nb) {
            const int rb = min(16, p - j0 - 16);
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            const double* Dsub = B + TS;
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const double av = Dsub[lr * 17 + kk + lh];
                const double bv = Lis[lr * 17 + kk + lh];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
            double* Lnext = Lsb + ((J + 1) & 1) * TS;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = lh + 4 * q;
                Lnext[r * 17 + lr] = acc[q];
                if (r < rb && lr < jb) A[(j0 + 16 + r) + static_cast<size_t>(j0 + lr) * ld] = acc[q];
            }
        }
        __syncthreads();
    }
    if (wave != 0 && nb > 0) store_diag(nb - 1);
    // S = A_BB - W^T W, each lower element written with its mirror by one lane (S stays
    // exactly symmetric)
    double* S = A + p + static_cast<size_t>(p) * ld;
    if (inc) {
        if (wave == 0) return;
        syrk_step();   // the last block
#pragma unroll
        for (int u = 0; u < kLeafTilesPerWave; ++u) {
            const int t = (wave - 1) + 3 * u;
            if (t >= ntl) break;
            int ti, tj;
            tile_ij(t, ti, tj);
            const int c = tj * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = ti * 16 + prow(q);
                const double sq = F32 ? static_cast<double>(saccf[u][q]) : sacc[u][q];
                if (r < m && c < m && r >= c) {
                    const double v = S[r + static_cast<size_t>(c) * ld] - sq;
                    S[r + static_cast<size_t>(c) * ld] = v;
                    S[c + static_cast<size_t>(r) * ld] = v;
                }
            }
        }
        return;
    }
    const double* Wt = A + p;
    for (int t = wave; t < ntl; t += kWaves) {
        int ti, tj;
        tile_ij(t, ti, tj);
        const int c = tj * 16 + lr;
        v4d s0 = {0.0, 0.0, 0.0, 0.0}, acc = {0.0, 0.0, 0.0, 0.0};
        v4f accf = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ti * 16 + prow(q);
            if (r < m && c < m) s0[q] = S[max(r, c) + static_cast<size_t>(min(r, c)) * ld];
        }
        const int ra = ti * 16 + lr, rb = tj * 16 + lr;
        const double* Wa = Wt + ra;
        const double* Wb = Wt + rb;
        const bool oka = ra < m, okb = rb < m;
        auto mac = [&](double av, double bv) {
            if constexpr (F32)
                accf = __builtin_amdgcn_mfma_f32_16x16x4f32(static_cast<float>(av), static_cast<float>(bv), accf, 0,
                                                           0, 0);
            else
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        };
        int k0 = 0;
        for (; k0 + 16 <= p; k0 += 16) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t col = static_cast<size_t>(k0 + 4 * u + lh) * ld;
                av[u] = oka ? Wa[col] : 0.0;
                bv[u] = okb ? Wb[col] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) mac(av[u], bv[u]);
        }
        for (; k0 < p; k0 += 4) {
            const int kq = k0 + lh;
            const double av = (oka && kq < p) ? Wa[static_cast<size_t>(kq) * ld] : 0.0;
            const double bv = (okb && kq < p) ? Wb[static_cast<size_t>(kq) * ld] : 0.0;
            mac(av, bv);
        }
        if constexpr (F32) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = static_cast<double>(accf[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ti * 16 + prow(q);
            if (r < m && c < m && r >= c) {
                const double v = s0[q] - acc[q];
                S[r + static_cast<size_t>(c) * ld] = v;
                S[c + static_cast<size_t>(r) * ld] = v;
            }
        }
    }
}

template __global__ void k_leaf_elim<false>(const FrontDesc*, double*, double*, int, int, unsigned long long*,
                                            int32_t*);
template __global__ void k_leaf_elim<true>(const FrontDesc*, double*, double*, int, int, unsigned long long*,
                                           int32_t*);

// ---------------------------------------------------------------------------------------
// The cell elimination of eq. (2.1) in three launches, for levels with few cells (one
// workgroup per cell would leave most of the chip idle and wait on memory latency):
//   k_chol_lead:  A_II = L L^T, one workgroup per cell, A_II staged in LDS when it fits;
//                 also stores the inverses of L's 16 x 16 diagonal blocks;
//   k_trsm_rows:  W^T = A_BI L^-T, 16 rows per wave, independent across rows;
//   k_syrk_schur: S = A_BB - W^T W on 32 x 32 blocks, both triangles written.
// Large interiors are eliminated panel by panel with the same three kernels (right-looking
// blocked Cholesky): for a panel of columns j0..j0+b, each is given the trailing frontal
// A[j0:n, j0:n] with p = b, so the TRSM covers every row below the panel and the SYRK
// updates the whole trailing matrix (interior rows included).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol_lead(const FrontDesc* __restrict__ desc, double* __restrict__ pool,
                                                   double* __restrict__ linv, int lds_pmax, int level, int step,
                                                   unsigned long long* err, int32_t* __restrict__ ext) {
    extern __shared__ double smem[];
    const FrontDesc fd = desc[blockIdx.x];
    const int p = fd.p, ld = fd.ld;
    double* A = pool + fd.off;
    double* lv = linv + static_cast<size_t>(fd.ext) * 256;
    int32_t* ex = ext != nullptr ? ext + fd.ext : nullptr;
    const unsigned long long code = err_code(level, step, fd.id);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (p <= lds_pmax) {
        const int ls = p | 1;
        double* D = smem + kPotrfSmemFixed;
        // lower triangle into LDS, eight loads in flight per thread before their stores
        const int pp = p * p;
        for (int e0 = threadIdx.x; e0 < pp; e0 += 8 * kWG) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kWG, i = e % p, j = e / p;
                v[u] = (e < pp && i >= j) ? A[i + static_cast<size_t>(j) * ld] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kWG, i = e % p, j = e / p;
                if (e < pp && i >= j) D[i + j * ls] = v[u];
            }
        }
        __syncthreads();
        wg_potrf_partial(D, ls, p, p, smem, 0, err, code, ex, lv);
        for (int j = wave; j < p; j += kWaves)
            for (int i = j + lane; i < p; i += 64) A[i + static_cast<size_t>(j) * ld] = D[i + j * ls];
    } else {
        wg_potrf_partial(A, ld, p, p, smem, 0, err, code, ex, lv);
    }
}

// Wave-level triangular solves with a lower-triangular L (n x n, column-major, ld ldl)
// whose 16 x 16 diagonal blocks have stored inverses li (256 doubles per block, padded with
// the identity), on the FP64 matrix cores:
//   wave_trsm_rlt: rows r0..r0+15 of the column-major m x n block X become X L^-T, by
//                  16-column panels P_j = (X_j - P_<j L_j,<j^T) Li_j^T;
//   wave_trsm_ll:  columns c0..c0+15 of the column-major n x nc block Y become L^-1 Y, by
//                  16-row blocks Y_I = Li_I (Y_I - L_I,<I Y_<I); optionally also written
//                  transposed to YT (ld ldt).
// Pw: the wave's LDS scratch, 17 * roundup16(n) doubles (finished panels / row blocks);
// with HL = false only one 16 x 17 tile, and the finished panels are read back from X / Y in
// global memory (each wave reads only what it wrote itself, after a device-scope fence).
// Lane l holds output rows l/16 + 4q, column l % 16 of a 16 x 16 tile.
template <bool HL = true>
__device__ __forceinline__ void wave_trsm_rlt(double* __restrict__ X, int ldx, int m, int r0, int n,
                                              const double* __restrict__ L, int ldl, const double* __restrict__ li,
                                              double* Pw) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lh = lane >> 4;
    for (int j0 = 0; j0 < n; j0 += 16) {
        const int jb = min(16, n - j0);
        double* Pt = HL ? Pw + j0 * 17 : Pw;
        v4d acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + lh + 4 * q;
            acc[q] = (r < m && lr < jb) ? X[r + static_cast<size_t>(j0 + lr) * ldx] : 0.0;
        }
        // 16 columns (four products) per step, their operands loaded before the products (j0 is
        // a multiple of 16); the products accumulate in column order
        auto ld16 = [&](int kc, double (&av)[4], double (&bv)[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k0 = kc + 4 * u;
                if constexpr (HL)
                    av[u] = -Pw[(k0 + lh) * 17 + lr];
                else
                    av[u] = (r0 + lr < m) ? -X[(r0 + lr) + static_cast<size_t>(k0 + lh) * ldx] : 0.0;
                bv[u] = (lr < jb) ? L[(j0 + lr) + static_cast<size_t>(k0 + lh) * ldl] : 0.0;
            }
        };
#pragma nounroll
        for (int kc = 0; kc < j0; kc += 16) {
            double ca[4], cb[4];
            ld16(kc, ca, cb);
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u], cb[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Pt[lr * 17 + lh + 4 * q] = acc[q];
        __builtin_amdgcn_wave_barrier();
        v4d out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const double av = Pt[(kk + lh) * 17 + lr];
            const double bv = li[(j0 >> 4) * 256 + lr * 16 + kk + lh];
            out = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, out, 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + lh + 4 * q;
            if constexpr (HL) Pt[lr * 17 + lh + 4 * q] = out[q];
            if (r < m && lr < jb) X[r + static_cast<size_t>(j0 + lr) * ldx] = out[q];
        }
        if constexpr (!HL) __threadfence();
        __builtin_amdgcn_wave_barrier();
    }
}

template <bool HL = true>
__device__ __forceinline__ void wave_trsm_ll(double* __restrict__ Y, int ldy, int n, int c0, int nc,
                                             const double* __restrict__ L, int ldl, const double* __restrict__ li,
                                             double* Yb, double* __restrict__ YT, int ldt) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lh = lane >> 4;
    const int cb = min(16, nc - c0);
    for (int i0 = 0; i0 < n; i0 += 16) {
        double* Yt = HL ? Yb + i0 * 17 : Yb;
        v4d acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = i0 + lh + 4 * q;
            acc[q] = (r < n && lr < cb) ? Y[r + static_cast<size_t>(c0 + lr) * ldy] : 0.0;
        }
        // as in wave_trsm_rlt: 16 rows of Y (four products) per step, operands loaded first
        auto ld16 = [&](int kc, double (&av)[4], double (&bv)[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k0 = kc + 4 * u;
                av[u] = (i0 + lr < n) ? -L[(i0 + lr) + static_cast<size_t>(k0 + lh) * ldl] : 0.0;
                if constexpr (HL)
                    bv[u] = Yb[(k0 + lh) * 17 + lr];
                else
                    bv[u] = (lr < cb) ? Y[(k0 + lh) + static_cast<size_t>(c0 + lr) * ldy] : 0.0;
            }
        };
#pragma nounroll
        for (int kc = 0; kc < i0; kc += 16) {
            double ca[4], cv[4];
            ld16(kc, ca, cv);
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u], cv[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Yt[(lh + 4 * q) * 17 + lr] = acc[q];
        __builtin_amdgcn_wave_barrier();
        v4d out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const double av = li[(i0 >> 4) * 256 + lr * 16 + kk + lh];
            const double bv = Yt[(kk + lh) * 17 + lr];
            out = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, out, 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = i0 + lh + 4 * q;
            if constexpr (HL) Yt[(lh + 4 * q) * 17 + lr] = out[q];
            if (r < n && lr < cb) {
                Y[r + static_cast<size_t>(c0 + lr) * ldy] = out[q];
                if (YT != nullptr) YT[(c0 + lr) + static_cast<size_t>(r) * ldt] = out[q];
            }
        }
        if constexpr (!HL) __threadfence();
        __builtin_amdgcn_wave_barrier();
    }
}

// Rows p.. of the cell: W^T = X L^-T, wave w of block y owning rows p + 16 (4 y + w) ..
// (pstride doubles of LDS per wave). The waves never wait for each other.
__global__ __launch_bounds__(256) void k_trsm_rows(const FrontDesc* __restrict__ desc, double* __restrict__ pool,
                                                   const double* __restrict__ linv, int pstride) {
    extern __shared__ double smem[];
    const FrontDesc fd = desc[blockIdx.x];
    const int p = fd.p, m = fd.n - fd.p;
    const int wave = threadIdx.x >> 6;
    const int r0 = (static_cast<int>(blockIdx.y) * kWaves + wave) * 16;
    if (r0 >= m || p == 0) return;
    double* A = pool + fd.off;
    wave_trsm_rlt(A + p, fd.ld, m, r0, p, A, fd.ld, linv + static_cast<size_t>(fd.ext) * 256,
                  smem + static_cast<size_t>(wave) * pstride);
}

// S = A_BB - W^T W on the kSyrkBlock x kSyrkBlock block (bi, bj), bi >= bj (block y of the
// cell, row-major over the lower triangle); each wave a 32 x 32 quarter of it, as 2 x 2 tiles of
// 16 x 16 on the matrix cores (each operand load feeds two products); every tile accumulates
// over k in ascending order. The old values are read from the lower triangle; each lower
// element is written with its mirror.
// F32: the product W^T W on the FP32 matrix cores with FP32 accumulation (operands rounded
// to FP32; S and the subtraction stay FP64). The FP32 16 x 16 x 4 product leaves row
// 4 (lane / 16) + q of its tile in register q; the FP64 one row lane / 16 + 4 q.
template <bool F32>
__global__ __launch_bounds__(256) void k_syrk_schur(const FrontDesc* __restrict__ desc, double* __restrict__ pool) {
    static_assert(kSyrkBlock == 64, "four 32 x 32 quarters per block");
    const FrontDesc fd = desc[blockIdx.x];
    const int p = fd.p, ms = fd.n - fd.p, ld = fd.ld;
    const int nb = (ms + kSyrkBlock - 1) / kSyrkBlock;
    const int t = blockIdx.y;
    if (t >= nb * (nb + 1) / 2) return;
    int bi = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    while (bi * (bi + 1) / 2 > t) --bi;
    const int bj = t - bi * (bi + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lh = lane >> 4;
    // tiles ti0, ti0 + 1 (rows) by tj0, tj0 + 1 (columns)
    const int ti0 = 4 * bi + 2 * (wave >> 1), tj0 = 4 * bj + 2 * (wave & 1);
    if (ti0 + 1 < tj0 || ti0 * 16 >= ms) return;   // above the diagonal, or past the last row
    double* A = pool + fd.off;
    double* S = A + p + static_cast<size_t>(p) * ld;
    const double* Wt = A + p;
    auto act = [&](int a, int b) { return (ti0 + a) * 16 < ms && (tj0 + b) * 16 < ms && ti0 + a >= tj0 + b; };
    auto row_of = [&](int a, int q) { return F32 ? (ti0 + a) * 16 + 4 * lh + q : (ti0 + a) * 16 + lh + 4 * q; };
    v4d s0[2][2], acc[2][2];
    v4f accf[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            s0[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
            acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
            accf[a][b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            const int c = (tj0 + b) * 16 + lr;
            if (act(a, b)) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = row_of(a, q);
                    if (r < ms && c < ms) s0[a][b][q] = S[max(r, c) + static_cast<size_t>(min(r, c)) * ld];
                }
            }
        }
    const int ra0 = ti0 * 16 + lr, rb0 = tj0 * 16 + lr;
    for (int k0 = 0; k0 < p; k0 += 4) {
        const int k = k0 + lh;
        double av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            av[a] = (ra0 + 16 * a < ms && k < p) ? Wt[ra0 + 16 * a + static_cast<size_t>(k) * ld] : 0.0;
            bv[a] = (rb0 + 16 * a < ms && k < p) ? Wt[rb0 + 16 * a + static_cast<size_t>(k) * ld] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if constexpr (F32)
                    accf[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(static_cast<float>(av[a]),
                                                                      static_cast<float>(bv[b]), accf[a][b], 0, 0, 0);
                else
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
    }
    // each lower element (r >= c) is written with its mirror by the one lane that read it
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if (!act(a, b)) continue;
            const int c = (tj0 + b) * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = row_of(a, q);
                const double pr = F32 ? static_cast<double>(accf[a][b][q]) : acc[a][b][q];
                if (r < ms && c < ms && r >= c) {
                    const double v = s0[a][b][q] - pr;
                    S[r + static_cast<size_t>(c) * ld] = v;
                    S[c + static_cast<size_t>(r) * ld] = v;
                }
            }
        }
}
template __global__ void k_syrk_schur<false>(const FrontDesc*, double*);
template __global__ void k_syrk_schur<true>(const FrontDesc*, double*);

// ---------------------------------------------------------------------------------------
// Block-Jacobi step (Sec. 2.3), part 1: for every separator group g, gather its diagonal
// block from every cell that holds a share of it and factor it, A_gg = L_g L_g^T.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_precond_groups(const SepDesc* __restrict__ sd, const CellRef* __restrict__ cells,
                                                        const double* __restrict__ F, double* __restrict__ Lg,
                                                        double* __restrict__ Li, int panel_cap, int lds_n, int level,
                                                        unsigned long long* err) {
    extern __shared__ double smem[];
    __shared__ int64_t s_off[kMaxSlots];
    __shared__ int32_t s_ld[kMaxSlots];
    const SepDesc& gr = sd[blockIdx.x];   // slot arrays indexed through memory
    const int n = gr.n, ns = gr.nslot;
    if (threadIdx.x < ns) {
        const int sl = threadIdx.x;
        const CellRef c = cells[gr.slot_cell[sl]];
        s_off[sl] = c.off + gr.slot_off[sl] + static_cast<int64_t>(gr.slot_off[sl]) * c.ld;
        s_ld[sl] = c.ld;
    }
    __syncthreads();
    double* L = Lg + gr.loff;
    const unsigned long long code = err_code(level, 1, blockIdx.x);
    double* lv = Li + gr.lioff;
    if (n <= lds_n) {
        double* D = smem + kPotrfSmemFixed;
        for (int e = threadIdx.x; e < n * n; e += kWG) {
            const int a = e % n, b = e / n;
            double v = 0.0;
            for (int sl = 0; sl < ns; ++sl) v += F[s_off[sl] + a + static_cast<size_t>(b) * s_ld[sl]];
            D[e] = v;
        }
        __syncthreads();
        wg_potrf_partial(D, n, n, n, smem, 0, err, code, nullptr, lv);
        for (int e = threadIdx.x; e < n * n; e += kWG) L[e] = D[e];
    } else {
        for (int e = threadIdx.x; e < n * n; e += kWG) {
            const int a = e % n, b = e / n;
            double v = 0.0;
            for (int sl = 0; sl < ns; ++sl) v += F[s_off[sl] + a + static_cast<size_t>(b) * s_ld[sl]];
            L[e] = v;
        }
        __syncthreads();
        wg_potrf_partial(L, n, n, n, smem, panel_cap, err, code, nullptr, lv);
    }
}

// Block-Jacobi step, part 1 for levels with large groups: A_gg gathered from the group's
// cells into L_g, 16 columns per workgroup; the Cholesky factor then comes from the panel
// kernels of the cell elimination.
__global__ __launch_bounds__(256) void k_precond_gather(const SepDesc* __restrict__ sd,
                                                        const CellRef* __restrict__ cells,
                                                        const double* __restrict__ F, double* __restrict__ Lg) {
    const SepDesc& gr = sd[blockIdx.x];
    const int n = gr.n, ns = gr.nslot;
    const int y0 = blockIdx.y * 16;
    if (y0 >= n) return;
    const int y1 = min(n, y0 + 16);
    int64_t off[kMaxSlots];
    int32_t ld[kMaxSlots];
    for (int sl = 0; sl < ns; ++sl) {
        const CellRef c = cells[gr.slot_cell[sl]];
        off[sl] = c.off + gr.slot_off[sl] + static_cast<int64_t>(gr.slot_off[sl]) * c.ld;
        ld[sl] = c.ld;
    }
    double* L = Lg + gr.loff;
    for (int e = threadIdx.x; e < (y1 - y0) * n; e += kWG) {
        const int a = e % n, b = y0 + e / n;
        double v = 0.0;
        for (int sl = 0; sl < ns; ++sl) v += F[off[sl] + a + static_cast<size_t>(b) * ld[sl]];
        L[a + static_cast<size_t>(b) * n] = v;
    }
}

// Block-Jacobi step, part 2: every cell's share S of the separator matrix becomes
// Lambda^-1 S Lambda^-T with Lambda = blockdiag(L_g) over the cell's boundary groups; the
// diagonal blocks become I in the group's first cell and 0 in the others, so that the
// assembled matrix has unit block diagonal. One workgroup per block (g, h) of a cell with g
// after h in the cell's group order: S_gh := L_g^-1 S_gh L_h^-T (rows, then columns, by
// blocked substitution with the stored inverses of the 16 x 16 diagonal blocks), written
// also transposed into the (h, g) block. Workgroups with g = h set the diagonal block.
// phase 0: both one-sided solves in one launch; 1: only X <- X L_h^-T (its 16-row strips are
// independent); 2: only X <- L_g^-1 X (16-column strips), and the diagonal blocks. The strips of
// a pair are spread over the workgroups of the grid's third dimension.
__global__ __launch_bounds__(256) void k_precond_scale(const CellScaleDesc* __restrict__ cd,
                                                       const CellGroup* __restrict__ cg, const double* __restrict__ Lg,
                                                       const double* __restrict__ Li, double* __restrict__ F,
                                                       int pstride, int phase) {
    extern __shared__ double smem[];
    const CellScaleDesc c = cd[blockIdx.x];
    const int gc = c.g_count;
    const int t = blockIdx.y;
    if (t >= gc * (gc + 1) / 2) return;
    int eg = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((eg + 1) * (eg + 2) / 2 <= t) ++eg;
    while (eg * (eg + 1) / 2 > t) --eg;
    const int eh = t - eg * (eg + 1) / 2;
    const CellGroup G = cg[c.g_begin + eg], H = cg[c.g_begin + eh];
    double* Fc = F + c.off;
    const int ld = c.ld;
    const int z = blockIdx.z, nz = gridDim.z;
    if (eg == eh) {
        if (phase == 1) return;
        for (int e = z * kWG + threadIdx.x; e < G.n * G.n; e += nz * kWG) {
            const int a = e % G.n, b = e / G.n;
            Fc[(G.off + a) + static_cast<size_t>(G.off + b) * ld] = (G.owner && a == b) ? 1.0 : 0.0;
        }
        return;
    }
    const int wave = threadIdx.x >> 6;
    const int s0 = (z * kWaves + wave) * 16, ss = nz * kWaves * 16;
    double* X = Fc + G.off + static_cast<size_t>(H.off) * ld;
    double* XT = Fc + H.off + static_cast<size_t>(G.off) * ld;
    if (pstride > 0) {
        double* Pw = smem + static_cast<size_t>(wave) * pstride;
        if (phase != 2)
            for (int r0 = s0; r0 < G.n; r0 += ss) wave_trsm_rlt(X, ld, G.n, r0, H.n, Lg + H.loff, H.n, Li + H.lioff, Pw);
        if (phase == 0) __syncthreads();
        if (phase != 1)
            for (int c0 = s0; c0 < H.n; c0 += ss)
                wave_trsm_ll(X, ld, G.n, c0, H.n, Lg + G.loff, G.n, Li + G.lioff, Pw, XT, ld);
    } else {
        // groups too large for LDS strips: finished panels are read back from the frontal
        double* Pw = smem + wave * 16 * 17;
        if (phase != 2)
            for (int r0 = s0; r0 < G.n; r0 += ss)
                wave_trsm_rlt<false>(X, ld, G.n, r0, H.n, Lg + H.loff, H.n, Li + H.lioff, Pw);
        if (phase == 0) {
            __threadfence();
            __syncthreads();
        }
        if (phase != 1)
            for (int c0 = s0; c0 < H.n; c0 += ss)
                wave_trsm_ll<false>(X, ld, G.n, c0, H.n, Lg + G.loff, G.n, Li + G.lioff, Pw, XT, ld);
    }
}

// ---------------------------------------------------------------------------------------
// Skeletonization of one edge (2D) / face (3D) (Sec. 2.2), all groups of a level from the
// same matrix:
//   1. M = A[R_g, g]: the group's columns over the other boundary unknowns of its one or
//      two cells, the shares of both cells added;
//   2. ID by column-pivoted QR -> rank k, pivot order, T = R11^-1 R12;
//   3. the zeroed blocks of eq. (2.2) in the order (redundant, skeleton):
//        G = [[A~_tt, A~_ht^T], [A~_ht, A_hh]] with
//        A~_tt = A_tt - T^T A_ht - A_ht^T T + T^T A_hh T,  A~_ht = A_ht - A_hh T;
//   4. partial Cholesky of G over the n-k redundant unknowns: L~, W~^T and the new
//      skeleton block A_hh - W~^T W~;
//   5. the new skeleton block goes to the group's first cell, the other cell's share of
//      the group's diagonal block is cleared. Couplings of the redundant unknowns to R are
//      dropped simply by not carrying them to the next level.
// ---------------------------------------------------------------------------------------
// The row table of M = A[R_g, g] (Sec. 2.2): R_g is the other boundary groups of the
// group's first cell (with the second cell's position where the group is shared), then the
// second cell's groups not in the first. rwl[2 i], rwl[2 i + 1] receive row i's position in
// either cell (-1: none). The cells' group lists are staged in LDS by all threads, then the
// first wave builds the segments (first row, count, positions), one lane per list entry; a
// row count that disagrees with the plan is reported. scratch: 4 * kMaxSkelSegs + 2 + 4 * kMaxCellGroups ints.
// Frontal rows p1 (first cell), p2 (second cell) of row i of M from the row segments (-1: the
// cell holds no share of that row).
__device__ __forceinline__ void seg_row(const int* seg, int ns, int i, int& p1, int& p2) {
    p1 = p2 = -1;
    for (int q = 0; q < ns; ++q) {
        const int t = i - seg[4 * q];
        if (t >= 0 && t < seg[4 * q + 1]) {
            p1 = seg[4 * q + 2] >= 0 ? seg[4 * q + 2] + t : -1;
            p2 = seg[4 * q + 3] >= 0 ? seg[4 * q + 3] + t : -1;
        }
    }
}

__device__ __forceinline__ void build_row_table(const SkelDesc& g, const int32_t* __restrict__ cgptr,
                                                const int32_t* __restrict__ cgl, const int32_t* __restrict__ cgoff,
                                                int nf0, int nf1, int r, int* rwl, int* scratch, int level,
                                                unsigned long long* err) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    int* seg = scratch;
    int* nseg = seg + 4 * kMaxSkelSegs;
    int* lst = nseg + 2;   // [4][kMaxCellGroups]: groups and offsets of cell 0, then of cell 1
    const int a0 = cgptr[g.cell[0]], na = min(cgptr[g.cell[0] + 1] - a0, kMaxCellGroups);
    const int b0 = g.nslot > 1 ? cgptr[g.cell[1]] : 0;
    const int nbl = g.nslot > 1 ? min(cgptr[g.cell[1] + 1] - b0, kMaxCellGroups) : 0;
    const bool fits = (cgptr[g.cell[0] + 1] - a0) <= kMaxCellGroups &&
                      (g.nslot < 2 || cgptr[g.cell[1] + 1] - b0 <= kMaxCellGroups);
    for (int e = tid; e < na; e += nthr) {
        lst[e] = cgl[a0 + e];
        lst[kMaxCellGroups + e] = cgoff[a0 + e];
    }
    for (int e = tid; e < nbl; e += nthr) {
        lst[2 * kMaxCellGroups + e] = cgl[b0 + e];
        lst[3 * kMaxCellGroups + e] = cgoff[b0 + e];
    }
    __syncthreads();
    if (tid < 64) {
        // wave 0, one lane per list entry: lanes 0..31 the first cell's groups in order, lanes
        // 32..63 the second cell's; a wave prefix sum places every kept group's rows
        const int lane = tid;
        const int* ga = lst;
        const int* oa = lst + kMaxCellGroups;
        const int* gb = lst + 2 * kMaxCellGroups;
        const int* ob = lst + 3 * kMaxCellGroups;
        bool keep = false;
        int nh = 0, p1 = -1, p2 = -1;
        if (lane < 32) {
            const int e = lane;
            if (e < na && ga[e] != g.grp) {
                const int h = ga[e];
                keep = true;
                nh = ((e + 1 < na) ? oa[e + 1] : nf0) - oa[e];
                p1 = oa[e];
                for (int f2 = 0; f2 < nbl; ++f2)
                    if (gb[f2] == h) p2 = ob[f2];
            }
        } else {
            const int f2 = lane - 32;
            if (f2 < nbl && gb[f2] != g.grp) {
                const int h = gb[f2];
                bool shared = false;
                for (int e = 0; e < na; ++e) shared = shared || (ga[e] == h);
                if (!shared) {
                    keep = true;
                    nh = ((f2 + 1 < nbl) ? ob[f2 + 1] : nf1) - ob[f2];
                    p2 = ob[f2];
                }
            }
        }
        const unsigned long long km = __ballot(keep);
        const int idx = __popcll(km & ((1ull << lane) - 1ull));
        const int ns = __popcll(km);
        int incl = nh;   // inclusive prefix sum of the kept groups' sizes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        const int total = __shfl(incl, 63, 64);
        if (keep && idx < kMaxSkelSegs) {
            seg[4 * idx] = incl - nh;
            seg[4 * idx + 1] = nh;
            seg[4 * idx + 2] = p1;
            seg[4 * idx + 3] = p2;
        }
        if (lane == 0) {
            const bool ok = fits && ns <= kMaxSkelSegs && total == r;
            if (!ok) report(err, err_code(level, 7, blockIdx.x));
            *nseg = ok ? ns : 0;
        }
    }
    __syncthreads();
    if (rwl == nullptr) return;   // segments only (in scratch; their count at scratch[4 kMaxSkelSegs])
    const int ns = *nseg;
    for (int i = tid; i < r; i += nthr) {
        int p1 = -1, p2 = -1;
        seg_row(seg, ns, i, p1, p2);
        rwl[2 * i] = p1;
        rwl[2 * i + 1] = p2;
    }
    __syncthreads();
}

// LDS: pos, perm ints | row table (2 rmax ints) | QR partials |
//      [M (rmax x (nmax|1))] | [G (nmax^2)] | potrf scratch
// SM / SG: M / G staged in LDS (else in the global pools), fixed at compile time so that
// every access has a known address space.
// Steps 3-5 of the skeletonization of one group, after its ID (rank k, pivot order perm in
// LDS, T = R11^-1 R12 held in rows 0..k-1 of M at the redundant columns): the zeroed blocks of
// eq. (2.2), the elimination of the redundant unknowns (partial Cholesky of G) and the write-
// back of the new skeleton block. G (n x n, ld n) is Gw, in LDS (SG) or the global pool.
template <bool SG, typename MR>
__device__ __forceinline__ void skel_eliminate(const SkelDesc& g, int k, const int* perm, const MR* __restrict__ M,
                                               int ldr, const CellRef* __restrict__ cells, double* __restrict__ F,
                                               double* __restrict__ Gpool, double* __restrict__ Gw, double* psmem,
                                               double* __restrict__ skli, int panel_cap, int level,
                                               unsigned long long* err, int block_id) {
    const int n = g.n, nr = n - k;
    const int tid = threadIdx.x;
    const CellRef c0 = cells[g.cell[0]];
    CellRef c1 = c0;
    if (g.nslot > 1) c1 = cells[g.cell[1]];
    const double* f0 = F + c0.off + static_cast<size_t>(g.off[0]) * c0.ld;
    const double* f1 = F + c1.off + static_cast<size_t>(g.off[1]) * c1.ld;
    // 3. the zeroed blocks of eq. (2.2) in the order (redundant, skeleton). G first holds the
    //    whole permuted A_gg; then V = A_ht - A_hh T replaces the lower (h, t) block (A_ht
    //    stays in the upper one), then A~_tt = A_tt - T^T V - A_ht^T T (lower part).
    const int nn = n * n;
    for (int e0 = tid; e0 < nn; e0 += 4 * kWG) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kWG;
            v[u] = 0.0;
            if (e < nn) {
                const int x = e % n, y = e / n;
                const int qx = x < nr ? perm[k + x] : perm[x - nr];
                const int qy = y < nr ? perm[k + y] : perm[y - nr];
                v[u] = f0[g.off[0] + qx + static_cast<size_t>(qy) * c0.ld];
                if (g.nslot > 1) v[u] += f1[g.off[1] + qx + static_cast<size_t>(qy) * c1.ld];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + u * kWG < nn) Gw[e0 + u * kWG] = v[u];
    }
    __syncthreads();
    for (int e = tid; e < k * nr; e += kWG) {
        const int c = e % k, a = e / k;
        const int pa = perm[k + a];
        const double* Gc = Gw + (nr + c) + static_cast<size_t>(nr) * n;
        double v = Gw[(nr + c) + static_cast<size_t>(a) * n], v1 = 0.0;
        int q = 0;
        for (; q + 1 < k; q += 2) {
            v -= Gc[static_cast<size_t>(q) * n] * static_cast<double>(M[static_cast<size_t>(q) * ldr + pa]);
            v1 -= Gc[static_cast<size_t>(q + 1) * n] * static_cast<double>(M[static_cast<size_t>(q + 1) * ldr + pa]);
        }
        if (q < k) v -= Gc[static_cast<size_t>(q) * n] * static_cast<double>(M[static_cast<size_t>(q) * ldr + pa]);
        Gw[(nr + c) + static_cast<size_t>(a) * n] = v + v1;
    }
    __syncthreads();
    for (int e = tid; e < nr * nr; e += kWG) {
        const int a = e % nr, b = e / nr;
        if (a < b) continue;
        const int pa = perm[k + a], pb = perm[k + b];
        double v = Gw[a + static_cast<size_t>(b) * n], v1 = 0.0;
        for (int c = 0; c < k; ++c) {
            const MR* Tc = M + static_cast<size_t>(c) * ldr;
            v -= static_cast<double>(Tc[pa]) * Gw[(nr + c) + static_cast<size_t>(b) * n];
            v1 -= Gw[a + static_cast<size_t>(nr + c) * n] * static_cast<double>(Tc[pb]);
        }
        Gw[a + static_cast<size_t>(b) * n] = v + v1;
    }
    __syncthreads();
    // 4. eliminate the redundant unknowns
    wg_potrf_partial(Gw, n, n, nr, psmem, panel_cap, err, err_code(level, 2, block_id), nullptr, skli + g.lioff);
    // 5. write back the skeleton block (and keep G for the apply)
    double* Gout = Gpool + g.goff;
    for (int e = tid; e < nn; e += kWG) {
        const int a = e % n, b = e / n;
        if (SG) Gout[e] = Gw[e];
        if (a < k && b < k) {
            // skeleton a, b sit at positions perm[a], perm[b] of the group's ascending order
            F[c0.off + (g.off[0] + perm[a]) + static_cast<size_t>(g.off[0] + perm[b]) * c0.ld] =
                Gw[(nr + a) + static_cast<size_t>(nr + b) * n];
        }
        if (g.nslot > 1) F[c1.off + (g.off[1] + a) + static_cast<size_t>(g.off[1] + b) * c1.ld] = 0.0;
    }
}

// The ID of one group: from registers (wg_cpqr_regs) when n <= 64 and a thread's rows fit the
// largest register form compiled in (RMAX per thread; 32 when a wave holds several chunks),
// else wg_cpqr_rows. The register form used is the smallest that holds the rows.
template <int RMAX, int UR, typename MR>
__device__ __forceinline__ int cpqr_any(MR* M, int ldr, int r, int n, double eps, int* pos, int* perm,
                                        double* part) {
    int cw = 1;
    while (cw < n && cw < 64) cw <<= 1;
    const int cs = (r + kWG / cw - 1) / (kWG / cw);
    if (n > 64 || cs > (cw < 64 ? (RMAX < 32 ? RMAX : 32) : RMAX))
        return wg_cpqr_rows<UR, MR>(M, ldr, r, n, eps, pos, perm, part);
    if (cw < 64) {
        if (cs <= 8) return wg_cpqr_regs<8, MR, false>(M, ldr, r, n, eps, pos, perm, part);
        if constexpr (RMAX >= 32)
            if (cs > 16) return wg_cpqr_regs<32, MR, false>(M, ldr, r, n, eps, pos, perm, part);
        return wg_cpqr_regs<16, MR, false>(M, ldr, r, n, eps, pos, perm, part);
    }
    if constexpr (RMAX >= 32) {
        if (cs > 16) {
            if constexpr (RMAX >= 64) {
                if (cs > 32) {
                    if constexpr (RMAX > 64)
                        if (cs > 64) return wg_cpqr_regs<RMAX, MR, true>(M, ldr, r, n, eps, pos, perm, part);
                    return wg_cpqr_regs<64, MR, true>(M, ldr, r, n, eps, pos, perm, part);
                }
            }
            return wg_cpqr_regs<32, MR, true>(M, ldr, r, n, eps, pos, perm, part);
        }
    }
    return wg_cpqr_regs<16, MR, true>(M, ldr, r, n, eps, pos, perm, part);
}

// MR: arithmetic of the ID (M, its QR and T); double, or float in the mixed-precision form.
// RMAX: the most rows of M per thread for which the ID runs from registers (cpqr_any).
template <bool SM, bool SG, typename MR, int RMAX>
__device__ __forceinline__ void skeletonize_one(const SkelDesc& g, const int32_t* __restrict__ cgptr,
                                                const int32_t* __restrict__ cgl, const int32_t* __restrict__ cgoff,
                                                const CellRef* __restrict__ cells, double* __restrict__ F,
                                                double* __restrict__ Mpool, double* __restrict__ Tpool,
                                                double* __restrict__ Gpool, double* __restrict__ skli, double eps,
                                                int32_t* __restrict__ kout, int32_t* __restrict__ pout, int panel_cap,
                                                int nmax, int rmax, int level, unsigned long long* err,
                                                double* smem) {
    const int n = g.n, r = g.r, ldr = n | 1;
    const int tid = threadIdx.x;
    const int ipd = (2 * nmax + 1) / 2 + 1;
    const int nbm = max(1, (nmax + 63) / 64);
    int* pos = reinterpret_cast<int*>(smem);
    int* perm = pos + nmax;
    int* rwl = reinterpret_cast<int*>(smem + ipd);
    double* part = smem + ipd + rmax;
    double* after = part + 2 * kWG * nbm + kCpqrRegExtra;
    MR* __restrict__ M = SM ? reinterpret_cast<MR*>(after) : reinterpret_cast<MR*>(Mpool + g.moff);
    // M occupies rmax (nmax | 1) values of MR, rounded up to whole doubles
    const size_t m_doubles = (static_cast<size_t>(rmax) * (nmax | 1) * sizeof(MR) + sizeof(double) - 1) / sizeof(double);
    double* gl = SM ? after + m_doubles : after;
    double* __restrict__ Gw = SG ? gl : Gpool + g.goff;
    double* psmem = SG ? gl + static_cast<size_t>(nmax) * nmax : gl;
    const CellRef c0 = cells[g.cell[0]];
    CellRef c1 = c0;
    if (g.nslot > 1) c1 = cells[g.cell[1]];
    const double* f0 = F + c0.off + static_cast<size_t>(g.off[0]) * c0.ld;
    const double* f1 = F + c1.off + static_cast<size_t>(g.off[1]) * c1.ld;
    build_row_table(g, cgptr, cgl, cgoff, c0.nf, c1.nf, r, rwl, reinterpret_cast<int*>(part), level, err);
    // 1. M = A[R_g, g] (row-major), the shares of both cells added; eight independent
    //    loads in flight per thread
    const int rn = r * n;
    for (int e0 = tid; e0 < rn; e0 += 8 * kWG) {
        double v[8];
        int dst[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kWG;
            v[u] = 0.0;
            dst[u] = -1;
            if (e < rn) {
                const int i = e % r, j = e / r;
                const int p1 = rwl[2 * i], p2 = rwl[2 * i + 1];
                if (p1 >= 0) v[u] += f0[p1 + static_cast<size_t>(j) * c0.ld];
                if (p2 >= 0) v[u] += f1[p2 + static_cast<size_t>(j) * c1.ld];
                dst[u] = i * ldr + j;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (dst[u] >= 0) M[dst[u]] = static_cast<MR>(v[u]);
    }
    __syncthreads();
    // 2. ID: rank k, pivot order, and T = R11^-1 R12 solved in place over R12
    const int k = cpqr_any<RMAX, SM ? 8 : 16, MR>(M, ldr, r, n, eps, pos, perm, part);
    const int nr = n - k;
    // column-oriented back substitution, every (row, column) update of a step in parallel:
    // t_i = x_i / R_ii, then x_e -= R_ei t_i for e < i
    for (int i = k - 1; i >= 0; --i) {
        const MR* Ri = M + static_cast<size_t>(i) * ldr;
        const int pi = perm[i];
        for (int a = tid; a < nr; a += kWG) {
            const int pa = perm[k + a];
            M[static_cast<size_t>(i) * ldr + pa] = Ri[pa] / Ri[pi];
        }
        __syncthreads();
        for (int idx = tid; idx < i * nr; idx += kWG) {
            const int e = idx % i, a = idx / i;
            const int pa = perm[k + a];
            M[static_cast<size_t>(e) * ldr + pa] -= M[static_cast<size_t>(e) * ldr + pi] * Ri[pa];
        }
        __syncthreads();
    }
    if (tid == 0) kout[g.gid] = k;
    for (int e = tid; e < n; e += kWG) pout[g.poff + e] = perm[e];
    __syncthreads();
    double* T = Tpool + g.toff;
    for (int e = tid; e < k * nr; e += kWG) {
        const int i = e % k, a = e / k;
        T[e] = static_cast<double>(M[static_cast<size_t>(i) * ldr + perm[k + a]]);
    }
    skel_eliminate<SG, MR>(g, k, perm, M, ldr, cells, F, Gpool, Gw, psmem, skli, panel_cap, level, err,
                           blockIdx.x);
}

// STAGED: 3 = M and G in LDS, 1 = M in LDS, 0 = both in the global pools; 4 = the layout of 3
// compiled for kSkelWavesMany waves per SIMD (fewer registers), for launches with many more
// groups than compute units, where more resident groups per CU hide the latency of each.
// One kernel per form, so that each keeps the register budget of its own code. RMAX (16, 32 or
// 96; 16 for form 4): the largest register form of the ID compiled in, chosen per level from
// its groups' sizes, since the registers of the largest form bound the groups resident per CU.
template <int STAGED, typename MR, int RMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STAGED == 4 ? kSkelWavesMany : 1))) void k_skeletonize(const SkelDesc* __restrict__ sd, const int32_t* __restrict__ cgptr,
                                                     const int32_t* __restrict__ cgl, const int32_t* __restrict__ cgoff,
                                                     const CellRef* __restrict__ cells, double* __restrict__ F,
                                                     double* __restrict__ Mpool, double* __restrict__ Tpool,
                                                     double* __restrict__ Gpool, double* __restrict__ skli, double eps,
                                                     int32_t* __restrict__ kout, int32_t* __restrict__ pout,
                                                     int panel_cap, int nmax, int rmax, int level,
                                                     unsigned long long* err) {
    extern __shared__ double smem[];
    const SkelDesc g = sd[blockIdx.x];
    skeletonize_one<STAGED != 0, STAGED >= 3, MR, RMAX>(g, cgptr, cgl, cgoff, cells, F, Mpool, Tpool, Gpool, skli, eps, kout,
                                              pout, panel_cap, nmax, rmax, level, err, smem);
}

#define RHIF_SKEL_INST(S, MR, RM)                                                                                  \
    template __global__ void k_skeletonize<S, MR, RM>(const SkelDesc*, const int32_t*, const int32_t*,             \
                                                      const int32_t*, const CellRef*, double*, double*, double*,   \
                                                      double*, double*, double, int32_t*, int32_t*, int, int, int, \
                                                      int, unsigned long long*);
#define RHIF_SKEL_INST3(S, MR) RHIF_SKEL_INST(S, MR, 16) RHIF_SKEL_INST(S, MR, 32) RHIF_SKEL_INST(S, MR, 96)
RHIF_SKEL_INST3(0, double)
RHIF_SKEL_INST3(1, double)
RHIF_SKEL_INST3(3, double)
RHIF_SKEL_INST(4, double, 16)
RHIF_SKEL_INST3(0, float)
RHIF_SKEL_INST3(1, float)
RHIF_SKEL_INST3(3, float)
RHIF_SKEL_INST(4, float, 16)
#undef RHIF_SKEL_INST3
#undef RHIF_SKEL_INST

// ---------------------------------------------------------------------------------------
// Interpolative decompositions of large groups across many workgroups (the faces of the upper
// 3D levels: M = A[R_g, g] of thousands of rows and hundreds of columns, in the global pool).
// The same column-pivoted Householder QR as wg_cpqr_rows (Sec. 2.2, the recomputed trailing
// norms, ties to the lowest position, rank test |R_jj| > eps |R_11|), but every step is spread
// over the row blocks of kBigRows rows of every group of the level: k_big_pivot (one
// workgroup per group) picks the pivot from the blocks' norm partials and forms the reflector,
// k_big_dot forms the blocks' partials of v^T M, and k_big_update sums them (fixed order),
// updates its rows and leaves the new norm partials. The host launches the three per step.
// Then k_big_trisolve solves T = R11^-1 R12 in place (one thread per redundant column), and
// k_big_elim with the panel kernels of the cell elimination performs the zeroing and the
// elimination of the redundant unknowns.
// ---------------------------------------------------------------------------------------
constexpr int kBigRows = 64;
static_assert(kBigRows == kBigRowsHost, "row blocks of the multi-workgroup ID");

template <typename MR>
__global__ __launch_bounds__(256) void k_big_gather(const SkelDesc* __restrict__ sd, const int32_t* __restrict__ cgptr,
                                                    const int32_t* __restrict__ cgl, const int32_t* __restrict__ cgoff,
                                                    const CellRef* __restrict__ cells, const double* __restrict__ F,
                                                    double* __restrict__ Mpool, double* __restrict__ nrm,
                                                    int32_t* __restrict__ pos, int32_t* __restrict__ pout,
                                                    BigState* __restrict__ st, int nmax, int nblk, int level,
                                                    unsigned long long* err) {
    __shared__ int seg[4 * kMaxSkelSegs + 2 + 4 * kMaxCellGroups];
    __shared__ int rows[2 * kBigRows];
    const int gi = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const SkelDesc g = sd[gi];
    const int n = g.n, r = g.r, ldr = n | 1;
    const CellRef c0 = cells[g.cell[0]];
    CellRef c1 = c0;
    if (g.nslot > 1) c1 = cells[g.cell[1]];
    build_row_table(g, cgptr, cgl, cgoff, c0.nf, c1.nf, r, nullptr, seg, level, err);
    const int ns = seg[4 * kMaxSkelSegs];
    const double* f0 = F + c0.off + static_cast<size_t>(g.off[0]) * c0.ld;
    const double* f1 = F + c1.off + static_cast<size_t>(g.off[1]) * c1.ld;
    MR* M = reinterpret_cast<MR*>(Mpool + g.moff);
    const int i0 = b * kBigRows, i1 = min(r, i0 + kBigRows);
    double* np = nrm + (static_cast<size_t>(gi) * nblk + b) * nmax;
    for (int i = i0 + tid; i < i1; i += kWG) {
        int p1, p2;
        seg_row(seg, ns, i, p1, p2);
        rows[2 * (i - i0)] = p1;
        rows[2 * (i - i0) + 1] = p2;
    }
    __syncthreads();
    for (int c = tid; c < n; c += kWG) {
        MR sq = 0;
        for (int i = i0; i < i1; ++i) {
            const int p1 = rows[2 * (i - i0)], p2 = rows[2 * (i - i0) + 1];
            double v = 0.0;
            if (p1 >= 0) v += f0[p1 + static_cast<size_t>(c) * c0.ld];
            if (p2 >= 0) v += f1[p2 + static_cast<size_t>(c) * c1.ld];
            const MR x = static_cast<MR>(v);
            M[static_cast<size_t>(i) * ldr + c] = x;
            sq += x * x;
        }
        np[c] = static_cast<double>(sq);
    }
    if (b == 0) {
        for (int c = tid; c < n; c += kWG) {
            pos[static_cast<size_t>(gi) * nmax + c] = c;
            pout[g.poff + c] = c;
        }
        if (tid == 0) {
            BigState z{};
            z.active = 1;
            st[gi] = z;
        }
    }
}

template <typename MR>
__global__ __launch_bounds__(256) void k_big_pivot(const SkelDesc* __restrict__ sd, const double* __restrict__ Mpool,
                                                   const double* __restrict__ nsum, int32_t* __restrict__ pos,
                                                   int32_t* __restrict__ pout, BigState* __restrict__ st, double eps,
                                                   int j, int nmax, int32_t* __restrict__ kout) {
    __shared__ double rb[kWaves];
    __shared__ int rp[kWaves], rc[kWaves];
    const int gi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (!st[gi].active) return;
    const SkelDesc g = sd[gi];
    const int n = g.n, r = g.r, ldr = n | 1;
    if (j >= min(r, n)) {   // every column taken
        if (tid == 0) {
            st[gi].active = 0;
            st[gi].k = j;
            kout[g.gid] = j;
        }
        return;
    }
    const int32_t* pg = pos + static_cast<size_t>(gi) * nmax;
    double best = -1.0;
    int bpos = 0x7fffffff, bc = -1;
    for (int c = tid; c < n; c += kWG) {
        const int pp = pg[c];
        if (pp < j) continue;
        const double vd = static_cast<double>(static_cast<MR>(nsum[static_cast<size_t>(gi) * nmax + c]));
        if (vd > best || (vd == best && pp < bpos)) {
            best = vd;
            bpos = pp;
            bc = c;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int op = __shfl_xor(bpos, off, 64);
        const int oc = __shfl_xor(bc, off, 64);
        if (ob > best || (ob == best && op < bpos)) {
            best = ob;
            bpos = op;
            bc = oc;
        }
    }
    if (lane == 0) {
        rb[wave] = best;
        rp[wave] = bpos;
        rc[wave] = bc;
    }
    __syncthreads();
    if (tid != 0) return;
    for (int w = 1; w < kWaves; ++w)
        if (rb[w] > best || (rb[w] == best && rp[w] < bpos)) {
            best = rb[w];
            bpos = rp[w];
            bc = rc[w];
        }
    BigState s = st[gi];
    const MR nv = sqrt(static_cast<MR>(best));
    if (j == 0) s.r11 = static_cast<double>(nv);
    if (!(nv > static_cast<MR>(eps) * static_cast<MR>(s.r11))) {
        s.active = 0;
        s.k = j;
        kout[g.gid] = j;
        st[gi] = s;
        return;
    }
    const MR* M = reinterpret_cast<const MR*>(Mpool + g.moff);
    const MR x0 = M[static_cast<size_t>(j) * ldr + bc];
    const MR alpha = -copysign(nv, x0);
    s.pc = bc;
    s.v0 = static_cast<double>(x0 - alpha);
    s.alpha = static_cast<double>(alpha);
    s.beta = static_cast<double>(MR(1) / (nv * (nv + fabs(x0))));
    s.k = j + 1;
    st[gi] = s;
    // the pivot order: column bc moves to position j
    int32_t* pw = pos + static_cast<size_t>(gi) * nmax;
    const int q = pw[bc], cj = pout[g.poff + j];
    pout[g.poff + j] = bc;
    pout[g.poff + q] = cj;
    pw[cj] = q;
    pw[bc] = j;
}

template <typename MR>
__global__ __launch_bounds__(256) void k_big_dot(const SkelDesc* __restrict__ sd, const double* __restrict__ Mpool,
                                                 const int32_t* __restrict__ pos, const BigState* __restrict__ st,
                                                 double* __restrict__ wpart, int j, int nmax, int nblk) {
    const int gi = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const BigState s = st[gi];
    if (!s.active) return;
    const SkelDesc g = sd[gi];
    const int n = g.n, r = g.r, ldr = n | 1;
    const int i0 = max(j, b * kBigRows), i1 = min(r, b * kBigRows + kBigRows);
    if (b * kBigRows >= r) return;
    const MR* M = reinterpret_cast<const MR*>(Mpool + g.moff);
    const int32_t* pg = pos + static_cast<size_t>(gi) * nmax;
    double* wp = wpart + (static_cast<size_t>(gi) * nblk + b) * nmax;
    const MR v0 = static_cast<MR>(s.v0);
    for (int c = tid; c < n; c += kWG) {
        if (pg[c] <= j) continue;
        MR w0 = 0, w1 = 0;
        int i = i0;
        if (i == j && i < i1) {   // row j lies in this block
            w0 = v0 * M[static_cast<size_t>(j) * ldr + c];
            ++i;
        }
        for (; i + 7 < i1; i += 8) {   // the order of the two-row loop below, loads first
            MR a[8], pv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                pv[u] = M[static_cast<size_t>(i + u) * ldr + s.pc];
                a[u] = M[static_cast<size_t>(i + u) * ldr + c];
            }
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
                w0 += pv[u] * a[u];
                w1 += pv[u + 1] * a[u + 1];
            }
        }
        for (; i + 1 < i1; i += 2) {
            w0 += M[static_cast<size_t>(i) * ldr + s.pc] * M[static_cast<size_t>(i) * ldr + c];
            w1 += M[static_cast<size_t>(i + 1) * ldr + s.pc] * M[static_cast<size_t>(i + 1) * ldr + c];
        }
        if (i < i1) w0 += M[static_cast<size_t>(i) * ldr + s.pc] * M[static_cast<size_t>(i) * ldr + c];
        wp[c] = static_cast<double>(w0 + w1);
    }
}

// The row blocks' partial sums of every column (norms after k_big_gather / k_big_update, v^T M
// after k_big_dot), summed once per step in block order (in the ID's arithmetic), so that
// k_big_pivot and the blocks of k_big_update read one value per column.
template <typename MR>
__global__ __launch_bounds__(256) void k_big_colsum(const SkelDesc* __restrict__ sd, const BigState* __restrict__ st,
                                                    const double* __restrict__ part, double* __restrict__ sum, int nmax,
                                                    int nblk) {
    const int gi = blockIdx.x, c = blockIdx.y * kWG + threadIdx.x;
    if (!st[gi].active) return;
    const SkelDesc g = sd[gi];
    if (c >= g.n) return;
    const int nb = (g.r + kBigRows - 1) / kBigRows;
    MR v = 0;
    for (int b = 0; b < nb; ++b) v += static_cast<MR>(part[(static_cast<size_t>(gi) * nblk + b) * nmax + c]);
    sum[static_cast<size_t>(gi) * nmax + c] = static_cast<double>(v);
}

template <typename MR>
__global__ __launch_bounds__(256) void k_big_update(const SkelDesc* __restrict__ sd, double* __restrict__ Mpool,
                                                    double* __restrict__ nrm, const int32_t* __restrict__ pos,
                                                    const BigState* __restrict__ st, const double* __restrict__ wsum,
                                                    int j, int nmax, int nblk) {
    const int gi = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const BigState s = st[gi];
    if (!s.active) return;
    const SkelDesc g = sd[gi];
    const int n = g.n, r = g.r, ldr = n | 1;
    if (b * kBigRows >= r) return;
    const int i0 = max(j, b * kBigRows), i1 = min(r, b * kBigRows + kBigRows);
    MR* M = reinterpret_cast<MR*>(Mpool + g.moff);
    const int32_t* pg = pos + static_cast<size_t>(gi) * nmax;
    double* np = nrm + (static_cast<size_t>(gi) * nblk + b) * nmax;
    const MR v0 = static_cast<MR>(s.v0), beta = static_cast<MR>(s.beta);
    for (int c = tid; c < n; c += kWG) {
        if (pg[c] <= j) continue;
        const MR w = static_cast<MR>(wsum[static_cast<size_t>(gi) * nmax + c]);
        const MR f = beta * w;
        MR sq = 0;
        int i = i0;
        if (i == j && i < i1) {   // row j lies in this block
            M[static_cast<size_t>(j) * ldr + c] -= f * v0;
            ++i;
        }
        // eight rows' loads in flight before their updates (the pivot column is never written
        // here); the norm sums in row order
        for (; i + 7 < i1; i += 8) {
            MR a[8], pv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a[u] = M[static_cast<size_t>(i + u) * ldr + c];
                pv[u] = M[static_cast<size_t>(i + u) * ldr + s.pc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const MR nvv = a[u] - f * pv[u];
                M[static_cast<size_t>(i + u) * ldr + c] = nvv;
                sq += nvv * nvv;
            }
        }
        for (; i < i1; ++i) {
            const MR nvv = M[static_cast<size_t>(i) * ldr + c] - f * M[static_cast<size_t>(i) * ldr + s.pc];
            M[static_cast<size_t>(i) * ldr + c] = nvv;
            sq += nvv * nvv;
        }
        np[c] = static_cast<double>(sq);
    }
    // R[j][pc] = alpha, by the block holding row j (no block reads it during this step)
    if (tid == 0 && b * kBigRows <= j && j < b * kBigRows + kBigRows)
        M[static_cast<size_t>(j) * ldr + s.pc] = static_cast<MR>(s.alpha);
}

// T = R11^-1 R12 in place over R12 (and copied to the T pool): back substitution for `ncol`
// redundant columns per workgroup, held in LDS; at each step every thread updates its rows of
// all of them with one entry of the pivot column of R11 (the operations and order of a column
// by column substitution).
constexpr int kTrisolveCols = kTrisolveColsHost;   // most redundant columns per workgroup

template <typename MR>
__global__ __launch_bounds__(256) void k_big_trisolve(const SkelDesc* __restrict__ sd, double* __restrict__ Mpool,
                                                      const int32_t* __restrict__ pout, const BigState* __restrict__ st,
                                                      double* __restrict__ Tpool, int ncol) {
    extern __shared__ double smem[];
    const int gi = blockIdx.x, tid = threadIdx.x;
    const SkelDesc g = sd[gi];
    const int n = g.n, ldr = n | 1, k = st[gi].k, nr = n - k;
    const int a0 = blockIdx.y * ncol;
    if (a0 >= nr || k == 0) return;
    const int nc = min(ncol, nr - a0);
    MR* M = reinterpret_cast<MR*>(Mpool + g.moff);
    const int32_t* perm = pout + g.poff;
    MR* x = reinterpret_cast<MR*>(smem);   // [ncol][k]
    for (int e = tid; e < nc * k; e += kWG) {
        const int c = e / k, i = e % k;
        x[e] = M[static_cast<size_t>(i) * ldr + perm[k + a0 + c]];
    }
    __syncthreads();
    for (int i = k - 1; i > 0; --i) {
        const int pi = perm[i];
        const MR rii = M[static_cast<size_t>(i) * ldr + pi];
        MR t[kTrisolveCols];   // row i is final: every thread forms the step's multipliers
#pragma unroll
        for (int c = 0; c < kTrisolveCols; ++c) t[c] = c < nc ? x[c * k + i] / rii : MR(0);
        for (int e = tid; e < i; e += kWG) {
            const MR r = M[static_cast<size_t>(e) * ldr + pi];
#pragma unroll
            for (int c = 0; c < kTrisolveCols; ++c)
                if (c < nc) x[c * k + e] -= r * t[c];
        }
        __syncthreads();
    }
    double* T = Tpool + g.toff;
    for (int e = tid; e < nc * k; e += kWG) {
        const int c = e / k, i = e % k;
        const MR ti = x[e] / M[static_cast<size_t>(i) * ldr + perm[i]];
        M[static_cast<size_t>(i) * ldr + perm[k + a0 + c]] = ti;
        T[i + static_cast<size_t>(a0 + c) * k] = static_cast<double>(ti);
    }
}

// The skeleton elimination of the large groups spread over many workgroups per group (the
// partial Cholesky of G then goes by the panel kernels of the cell elimination):
//   phase 0: G = the group's permuted diagonal block (redundant unknowns first), 16 columns of
//            G per workgroup;
//   phase 1: V = A_ht - A_hh T over the lower (skeleton, redundant) block;
//   phase 2: A~_tt = A_tt - T^T V - A_ht^T T on the lower triangle of the redundant block;
//   phase 3: the skeleton block of the Schur complement back to the first cell's frontal, the
//            second cell's share of the group cleared.
// Each entry is formed with the operations and order of skel_eliminate.
template <typename MR>
__global__ __launch_bounds__(256) void k_big_elim(const SkelDesc* __restrict__ sd, const CellRef* __restrict__ cells,
                                                  double* __restrict__ F, const double* __restrict__ Mpool,
                                                  double* __restrict__ Gpool, const int32_t* __restrict__ kout,
                                                  const int32_t* __restrict__ pout, int phase) {
    const SkelDesc g = sd[blockIdx.x];
    const int n = g.n, k = kout[g.gid], nr = n - k, ldr = n | 1, tid = threadIdx.x;
    const int y0 = blockIdx.y * 16;
    if (y0 >= n) return;
    const int y1 = min(n, y0 + 16);
    const int32_t* perm = pout + g.poff;
    const MR* M = reinterpret_cast<const MR*>(Mpool + g.moff);
    double* Gw = Gpool + g.goff;
    const CellRef c0 = cells[g.cell[0]];
    CellRef c1 = c0;
    if (g.nslot > 1) c1 = cells[g.cell[1]];
    const double* f0 = F + c0.off + static_cast<size_t>(g.off[0]) * c0.ld;
    const double* f1 = F + c1.off + static_cast<size_t>(g.off[1]) * c1.ld;
    if (phase == 0) {
        for (int e = tid; e < (y1 - y0) * n; e += kWG) {
            const int x = e % n, y = y0 + e / n;
            const int qx = x < nr ? perm[k + x] : perm[x - nr];
            const int qy = y < nr ? perm[k + y] : perm[y - nr];
            double v = f0[g.off[0] + qx + static_cast<size_t>(qy) * c0.ld];
            if (g.nslot > 1) v += f1[g.off[1] + qx + static_cast<size_t>(qy) * c1.ld];
            Gw[x + static_cast<size_t>(y) * n] = v;
        }
        return;
    }
    if (phase == 1) {   // columns a in [y0, y1) of the redundant block
        for (int e = tid; e < k * (min(y1, nr) - y0); e += kWG) {
            const int c = e % k, a = y0 + e / k;
            const int pa = perm[k + a];
            const double* Gc = Gw + (nr + c) + static_cast<size_t>(nr) * n;
            double v = Gw[(nr + c) + static_cast<size_t>(a) * n], v1 = 0.0;
            int q = 0;
            for (; q + 1 < k; q += 2) {
                v -= Gc[static_cast<size_t>(q) * n] * static_cast<double>(M[static_cast<size_t>(q) * ldr + pa]);
                v1 -= Gc[static_cast<size_t>(q + 1) * n] * static_cast<double>(M[static_cast<size_t>(q + 1) * ldr + pa]);
            }
            if (q < k) v -= Gc[static_cast<size_t>(q) * n] * static_cast<double>(M[static_cast<size_t>(q) * ldr + pa]);
            Gw[(nr + c) + static_cast<size_t>(a) * n] = v + v1;
        }
        return;
    }
    if (phase == 2) {   // columns b in [y0, y1), rows a >= b of the redundant block
        for (int e = tid; e < nr * (min(y1, nr) - y0); e += kWG) {
            const int a = e % nr, b = y0 + e / nr;
            if (a < b) continue;
            const int pa = perm[k + a], pb = perm[k + b];
            double v = Gw[a + static_cast<size_t>(b) * n], v1 = 0.0;
            for (int c = 0; c < k; ++c) {
                const MR* Tc = M + static_cast<size_t>(c) * ldr;
                v -= static_cast<double>(Tc[pa]) * Gw[(nr + c) + static_cast<size_t>(b) * n];
                v1 -= Gw[a + static_cast<size_t>(nr + c) * n] * static_cast<double>(Tc[pb]);
            }
            Gw[a + static_cast<size_t>(b) * n] = v + v1;
        }
        return;
    }
    // phase 3
    for (int e = tid; e < (y1 - y0) * n; e += kWG) {
        const int a = e % n, b = y0 + e / n;
        if (a < k && b < k)
            F[c0.off + (g.off[0] + perm[a]) + static_cast<size_t>(g.off[0] + perm[b]) * c0.ld] =
                Gw[(nr + a) + static_cast<size_t>(nr + b) * n];
        if (g.nslot > 1) F[c1.off + (g.off[1] + a) + static_cast<size_t>(g.off[1] + b) * c1.ld] = 0.0;
    }
}

#define RHIF_BIG_INST(MR)                                                                                          \
    template __global__ void k_big_gather<MR>(const SkelDesc*, const int32_t*, const int32_t*, const int32_t*,     \
                                              const CellRef*, const double*, double*, double*, int32_t*, int32_t*, \
                                              BigState*, int, int, int, unsigned long long*);                     \
    template __global__ void k_big_pivot<MR>(const SkelDesc*, const double*, const double*, int32_t*, int32_t*,    \
                                             BigState*, double, int, int, int32_t*);                              \
    template __global__ void k_big_colsum<MR>(const SkelDesc*, const BigState*, const double*, double*, int, int); \
    template __global__ void k_big_dot<MR>(const SkelDesc*, const double*, const int32_t*, const BigState*,        \
                                           double*, int, int, int);                                               \
    template __global__ void k_big_update<MR>(const SkelDesc*, double*, double*, const int32_t*, const BigState*,  \
                                              const double*, int, int, int);                                      \
    template __global__ void k_big_trisolve<MR>(const SkelDesc*, double*, const int32_t*, const BigState*,         \
                                                double*, int);                                                    \
    template __global__ void k_big_elim<MR>(const SkelDesc*, const CellRef*, double*, const double*, double*,      \
                                            const int32_t*, const int32_t*, int);
RHIF_BIG_INST(double)
RHIF_BIG_INST(float)
#undef RHIF_BIG_INST


// ---------------------------------------------------------------------------------------
// The forward product F x = G G^T x (eq. (3.3)) for the apply error e_a = ||A - F|| / ||A||
// (Sec. 4): every block of the apply (a cell's E: L and W^T in its frontal; a group's C: L_g;
// a skeleton's K: L~, W~^T and T) undone with products instead of solves, in the reverse
// order of the sweeps. One workgroup per block, operands read from HBM (a diagnostic, not a
// hot path). Rows of L past the panel extents (banded leaf interiors) are structural zeros
// and are skipped, as in the apply.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int l_rows_end(const ApplyDesc& d, const int32_t* ext, int col) {
    return (d.ext >= 0 && ext != nullptr) ? min(d.nI, static_cast<int>(ext[d.ext + col / 16])) : d.nI;
}

// Undo of a down-sweep block (part of G^T x): with T (a skeleton block), z_B += T z_I first;
// then z_I <- L^T z_I + W z_B.
__global__ __launch_bounds__(256) void k_fwd_gt(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                const double* __restrict__ Tp, const int32_t* __restrict__ dofs,
                                                const int32_t* __restrict__ ext, double* __restrict__ z) {
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nB = d.nB, ld = d.ld, tid = threadIdx.x;
    const double* A = pool + d.off;
    const int32_t* di = dofs + d.dofs;
    const int32_t* db = di + nI;
    if (d.toff >= 0) {
        const double* T = Tp + d.toff;
        for (int h = tid; h < nB; h += kWG) {
            double acc = 0.0;
            for (int t = 0; t < nI; ++t) acc += T[h + static_cast<size_t>(t) * nB] * z[di[t]];
            z[db[h]] += acc;
        }
        __syncthreads();
    }
    // rows in increasing chunks: the new z_I[i] reads the old z_I[e], e >= i
    for (int c0 = 0; c0 < nI; c0 += kWG) {
        const int i = c0 + tid;
        double acc = 0.0;
        if (i < nI) {
            const double* col = A + static_cast<size_t>(i) * ld;
            const int e1 = l_rows_end(d, ext, i);
            for (int e = i; e < e1; ++e) acc += col[e] * z[di[e]];
            for (int b = 0; b < nB; ++b) acc += col[nI + b] * z[db[b]];
        }
        __syncthreads();
        if (i < nI) z[di[i]] = acc;
        __syncthreads();
    }
}

// Undo of an up-sweep block (part of G y): y = W^T z_I (to the scratch at yoff, summed into the
// shared z_B by k_fwd_gather; or added to z_B in place), z_I <- L z_I, and with T (a skeleton
// block) z_I += T^T z_B last.
__global__ __launch_bounds__(256) void k_fwd_g(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                               const double* __restrict__ Tp, const int32_t* __restrict__ dofs,
                                               const int32_t* __restrict__ ext, double* __restrict__ z,
                                               double* __restrict__ ybuf) {
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nB = d.nB, ld = d.ld, tid = threadIdx.x;
    const double* A = pool + d.off;
    const int32_t* di = dofs + d.dofs;
    const int32_t* db = di + nI;
    for (int b = tid; b < nB; b += kWG) {
        double acc = 0.0;
        for (int i = 0; i < nI; ++i) acc += A[(nI + b) + static_cast<size_t>(i) * ld] * z[di[i]];
        if (d.yoff >= 0) ybuf[d.yoff + b] = acc;
        else z[db[b]] += acc;
    }
    __syncthreads();
    // rows in decreasing chunks: the new z_I[i] reads the old z_I[e], e <= i
    for (int c1 = nI; c1 > 0; c1 -= kWG) {
        const int i = c1 - kWG + tid;
        double acc = 0.0;
        if (i >= 0) {
            for (int e = 0; e <= i; ++e)
                if (i < l_rows_end(d, ext, e)) acc += A[i + static_cast<size_t>(e) * ld] * z[di[e]];
        }
        __syncthreads();
        if (i >= 0) z[di[i]] = acc;
        __syncthreads();
    }
    if (d.toff >= 0) {
        const double* T = Tp + d.toff;
        for (int t = tid; t < nI; t += kWG) {
            double acc = 0.0;
            for (int h = 0; h < nB; ++h) acc += T[h + static_cast<size_t>(t) * nB] * z[db[h]];
            z[di[t]] += acc;
        }
    }
}

// z_g += the cells' contributions y of every separator group (the shared boundary unknowns).
__global__ __launch_bounds__(256) void k_fwd_gather(const GatherDesc* __restrict__ gd, const int32_t* __restrict__ dofs,
                                                    const double* __restrict__ ybuf, double* __restrict__ z) {
    const GatherDesc g = gd[blockIdx.x];
    z += g.zoff;   // the block's problem within the vector
    for (int t = threadIdx.x; t < g.n; t += kWG) {
        const int i = dofs[g.dofs + t];
        double v = z[i];
        for (int sl = 0; sl < g.nslot; ++sl) v += ybuf[g.yoff[sl] + t];
        z[i] = v;
    }
}

// ---------------------------------------------------------------------------------------
// Factor apply (eq. (3.2)). One workgroup per block; z_I and z_B are staged in LDS (or
// in a global workspace for oversized blocks). Triangular solves go by 32-row blocks: the
// diagonal block is solved by one wave from LDS, the rest is a GEMV by all threads.
// ---------------------------------------------------------------------------------------
constexpr int kTB = 32;

// ext (LDS, may be null): per 16-column panel of L, the end of its nonzero rows.
__device__ void wg_trsv_lower(const double* __restrict__ L, int ld, int n, double* z, double* Dg, const int* ext) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j0 = 0; j0 < n; j0 += kTB) {
        const int jb = min(kTB, n - j0);
        for (int e = tid; e < jb * jb; e += kWG) {
            const int a = e % jb, b = e / jb;
            Dg[a * (kTB + 1) + b] = L[(j0 + a) + static_cast<size_t>(j0 + b) * ld];
        }
        __syncthreads();
        if (wave == 0) {
            double x = (lane < jb) ? z[j0 + lane] : 0.0;
            for (int c = 0; c < jb; ++c) {
                const double xc = __shfl(x, c, 64) / Dg[c * (kTB + 1) + c];
                if (lane == c) x = xc;
                else if (lane > c && lane < jb) x -= Dg[lane * (kTB + 1) + c] * xc;
            }
            if (lane < jb) z[j0 + lane] = x;
        }
        __syncthreads();
        int iend = n;
        if (ext != nullptr) {
            iend = ext[j0 >> 4];
            if (jb > 16) iend = max(iend, ext[(j0 >> 4) + 1]);
        }
        for (int i = j0 + jb + tid; i < iend; i += kWG) {
            double acc = 0.0;
            for (int c = 0; c < jb; ++c) acc += L[i + static_cast<size_t>(j0 + c) * ld] * z[j0 + c];
            z[i] -= acc;
        }
        __syncthreads();
    }
}

__device__ void wg_trsv_lower_t(const double* __restrict__ L, int ld, int n, double* z, double* Dg, const int* ext) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + kTB - 1) / kTB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int j0 = bi * kTB;
        const int jb = min(kTB, n - j0);
        for (int e = tid; e < jb * jb; e += kWG) {
            const int a = e % jb, b = e / jb;
            Dg[a * (kTB + 1) + b] = L[(j0 + a) + static_cast<size_t>(j0 + b) * ld];
        }
        __syncthreads();
        if (wave == 0) {
            double x = (lane < jb) ? z[j0 + lane] : 0.0;
            for (int c = jb - 1; c >= 0; --c) {
                const double xc = __shfl(x, c, 64) / Dg[c * (kTB + 1) + c];
                if (lane == c) x = xc;
                else if (lane < c) x -= Dg[c * (kTB + 1) + lane] * xc;
            }
            if (lane < jb) z[j0 + lane] = x;
        }
        __syncthreads();
        for (int i = tid; i < j0; i += kWG) {
            if (ext != nullptr && ext[i >> 4] <= j0) continue;   // L[j0.., i] is zero
            double acc = 0.0;
            const double* Li = L + static_cast<size_t>(i) * ld + j0;
            for (int c = 0; c < jb; ++c) acc += Li[c] * z[j0 + c];
            z[i] -= acc;
        }
        __syncthreads();
    }
}

// Up-sweep block: [z_I -= T^T z_B]; z_I <- L^-1 z_I; y = W^T z_I -> scratch or z_B -= y.
__global__ __launch_bounds__(256) void k_apply_up(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                  const double* __restrict__ Tp, const int32_t* __restrict__ dofs,
                                                  double* __restrict__ z, double* __restrict__ ybuf,
                                                  double* __restrict__ ws, const int32_t* __restrict__ extp) {
    extern __shared__ double smem[];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    double* Dg = smem;
    int* ext = (extp != nullptr && d.ext >= 0 && (d.nI + 15) / 16 <= 2 * kApplyExtDoubles)
                   ? reinterpret_cast<int*>(smem + kApplyDiagDoubles)
                   : nullptr;
    if (ext != nullptr)
        for (int t = threadIdx.x; t < (d.nI + 15) / 16; t += kWG) ext[t] = extp[d.ext + t];
    double* zI = (d.wsoff >= 0) ? ws + d.wsoff : smem + kApplyDiagDoubles + kApplyExtDoubles;
    double* zB = zI + d.nI;
    const int32_t* di = dofs + d.dofs;
    const int32_t* db = di + d.nI;
    const bool needB = (d.toff >= 0) || (d.yoff < 0);
    for (int i = threadIdx.x; i < d.nI; i += kWG) zI[i] = z[di[i]];
    if (needB)
        for (int i = threadIdx.x; i < d.nB; i += kWG) zB[i] = z[db[i]];
    __syncthreads();
    if (d.toff >= 0) {
        const double* T = Tp + d.toff;
        for (int a = threadIdx.x; a < d.nI; a += kWG) {
            double acc = 0.0;
            for (int c = 0; c < d.nB; ++c) acc += T[c + static_cast<size_t>(a) * d.nB] * zB[c];
            zI[a] -= acc;
        }
        __syncthreads();
    }
    const double* A = pool + d.off;
    wg_trsv_lower(A, d.ld, d.nI, zI, Dg, ext);
    for (int i = threadIdx.x; i < d.nI; i += kWG) z[di[i]] = zI[i];
    // y = W^T z_I: lanes run over 64 outputs, the 4 waves over quarters of the sum
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q0 = (d.nI * wave) / kWaves, q1 = (d.nI * (wave + 1)) / kWaves;
    for (int b0 = 0; b0 < d.nB; b0 += 64) {
        const int b = b0 + lane;
        double acc = 0.0;
        if (b < d.nB) {
            const double* Wb = A + d.nI + b;
            int i = q0;
            for (; i + 3 < q1; i += 4)
                acc += Wb[static_cast<size_t>(i) * d.ld] * zI[i] + Wb[static_cast<size_t>(i + 1) * d.ld] * zI[i + 1] +
                       Wb[static_cast<size_t>(i + 2) * d.ld] * zI[i + 2] + Wb[static_cast<size_t>(i + 3) * d.ld] * zI[i + 3];
            for (; i < q1; ++i) acc += Wb[static_cast<size_t>(i) * d.ld] * zI[i];
        }
        __syncthreads();
        Dg[wave * 64 + lane] = acc;
        __syncthreads();
        if (wave == 0 && b < d.nB) {
            const double y = Dg[lane] + Dg[64 + lane] + Dg[128 + lane] + Dg[192 + lane];
            if (d.yoff >= 0) ybuf[d.yoff + b] = y;
            else z[db[b]] = zB[b] - y;
        }
    }
}

// Down-sweep block: z_I <- L^-T (z_I - W z_B); [z_B -= T z_I].
__global__ __launch_bounds__(256) void k_apply_down(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                    const double* __restrict__ Tp, const int32_t* __restrict__ dofs,
                                                    double* __restrict__ z, double* __restrict__ ws,
                                                    const int32_t* __restrict__ extp) {
    extern __shared__ double smem[];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    double* Dg = smem;
    int* ext = (extp != nullptr && d.ext >= 0 && (d.nI + 15) / 16 <= 2 * kApplyExtDoubles)
                   ? reinterpret_cast<int*>(smem + kApplyDiagDoubles)
                   : nullptr;
    if (ext != nullptr)
        for (int t = threadIdx.x; t < (d.nI + 15) / 16; t += kWG) ext[t] = extp[d.ext + t];
    double* zI = (d.wsoff >= 0) ? ws + d.wsoff : smem + kApplyDiagDoubles + kApplyExtDoubles;
    double* zB = zI + d.nI;
    const int32_t* di = dofs + d.dofs;
    const int32_t* db = di + d.nI;
    for (int i = threadIdx.x; i < d.nI; i += kWG) zI[i] = z[di[i]];
    for (int i = threadIdx.x; i < d.nB; i += kWG) zB[i] = z[db[i]];
    __syncthreads();
    const double* A = pool + d.off;
    for (int i = threadIdx.x; i < d.nI; i += kWG) {
        double acc = 0.0;
        const double* Wi = A + static_cast<size_t>(i) * d.ld + d.nI;
        for (int b = 0; b < d.nB; ++b) acc += Wi[b] * zB[b];
        zI[i] -= acc;
    }
    __syncthreads();
    wg_trsv_lower_t(A, d.ld, d.nI, zI, Dg, ext);
    for (int i = threadIdx.x; i < d.nI; i += kWG) z[di[i]] = zI[i];
    if (d.toff >= 0) {
        const double* T = Tp + d.toff;
        for (int c = threadIdx.x; c < d.nB; c += kWG) {
            double acc = 0.0;
            for (int a = 0; a < d.nI; ++a) acc += T[c + static_cast<size_t>(a) * d.nB] * zI[a];
            z[db[c]] = zB[c] - acc;
        }
    }
}

// ---------------------------------------------------------------------------------------
// Factor apply, split form for blocks with n_I <= kSplitApplyMaxI: the triangular solves
// (one workgroup per block) and the W products (one workgroup per 64 rows or columns of a
// block) are separate launches. The solves go by 16-column panels of L with the stored
// inverses Li of its diagonal blocks; the next panel's entries of L and rows of Li are
// loaded into registers while the current panel is processed:
//   forward  (L z = b):   z_J = Li_J z_J, then z_i -= L[i, J] z_J for the rows below;
//   backward (L^T z = b): z_J = Li_J^T z_J, then z_k -= L[J, k]^T z_J for k before J.
// Each thread owns one row (forward) or one column (backward) of a panel.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void stage_apply_vectors(const ApplyDesc& d, const int32_t* __restrict__ dofs,
                                                    const double* __restrict__ z, double* zI, double* zB, bool needB,
                                                    int* ex, const int32_t* __restrict__ extp) {
    const int32_t* di = dofs + d.dofs;
    const int nt = (d.nI + 15) / 16;
    for (int i = threadIdx.x; i < nt * 16; i += kWG) zI[i] = (i < d.nI) ? z[di[i]] : 0.0;
    if (needB)
        for (int c = threadIdx.x; c < d.nB; c += kWG) zB[c] = z[di[d.nI + c]];
    for (int t = threadIdx.x; t < nt; t += kWG) ex[t] = (extp != nullptr && d.ext >= 0) ? extp[d.ext + t] : d.nI;
}

// Workgroup forward solve z <- L^-1 z (z in LDS, n <= kSplitApplyMaxI; ex: per-panel
// nonzero row ends of L in LDS, or null when L is dense).
template <bool PREFETCH = true>
__device__ __forceinline__ void wg_trsv_fwd(const double* __restrict__ L, int ld, int n,
                                            const double* __restrict__ li, double* zI, const int* ex) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = (n + 15) / 16;
    const bool solver = (wave == 0 && lane < 16);
    double lv[16], lr[16], lvn[16], lrn[16];
    auto load = [&](int t, double (&v)[16], double (&r)[16]) {
        const int j0 = 16 * t, jb = min(16, n - j0);
        const int i = j0 + 16 + tid;
        const bool ok = i < (ex != nullptr ? ex[t] : n);
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = (ok && c < jb) ? L[i + static_cast<size_t>(j0 + c) * ld] : 0.0;
        if (solver) {
#pragma unroll
            for (int k = 0; k < 16; ++k) r[k] = li[t * 256 + lane * 16 + k];
        }
    };
    if (PREFETCH) load(0, lvn, lrn);
    for (int t = 0; t < nt; ++t) {
        if (PREFETCH) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                lv[c] = lvn[c];
                lr[c] = lrn[c];
            }
            if (t + 1 < nt) load(t + 1, lvn, lrn);
        } else {
            load(t, lv, lr);
        }
        const int j0 = 16 * t;
        if (solver) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += lr[k] * zI[j0 + k];
            zI[j0 + lane] = acc;
        }
        __syncthreads();
        const int i = j0 + 16 + tid;
        if (i < (ex != nullptr ? ex[t] : n)) {
            double acc = zI[i];
#pragma unroll
            for (int c = 0; c < 16; ++c) acc -= lv[c] * zI[j0 + c];
            zI[i] = acc;
        }
        __syncthreads();
    }
}

// Workgroup backward solve z <- L^-T z (same conventions).
template <bool PREFETCH = true>
__device__ __forceinline__ void wg_trsv_bwd(const double* __restrict__ L, int ld, int n,
                                            const double* __restrict__ li, double* zI, const int* ex) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = (n + 15) / 16;
    const bool solver = (wave == 0 && lane < 16);
    double lv[16], lr[16], lvn[16], lrn[16];
    // thread k owns column k < j0 of the row panel J (rows j0..j0+15)
    auto load = [&](int t, double (&v)[16], double (&r)[16]) {
        const int j0 = 16 * t, jb = min(16, n - j0);
        const int k = tid;
        const bool ok = k < j0 && (ex == nullptr || ex[k >> 4] > j0);
        const double* Lk = L + static_cast<size_t>(k) * ld + j0;
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (ok && q < jb) ? Lk[q] : 0.0;
        if (solver) {
#pragma unroll
            for (int q = 0; q < 16; ++q) r[q] = li[t * 256 + q * 16 + lane];
        }
    };
    if (PREFETCH) load(nt - 1, lvn, lrn);
    for (int t = nt - 1; t >= 0; --t) {
        if (PREFETCH) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                lv[c] = lvn[c];
                lr[c] = lrn[c];
            }
            if (t > 0) load(t - 1, lvn, lrn);
        } else {
            load(t, lv, lr);
        }
        const int j0 = 16 * t;
        if (solver) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) acc += lr[q] * zI[j0 + q];
            zI[j0 + lane] = acc;
        }
        __syncthreads();
        if (tid < j0) {
            double acc = zI[tid];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc -= lv[q] * zI[j0 + q];
            zI[tid] = acc;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// Factor apply of blocks with large interiors (n_I > kBigApplyMinI: the upper 3D levels and
// large roots), spread over many workgroups per block. The block's vectors are staged in the
// global workspace at wsoff ([z_I | z_B]); the solves go by panels of kBigApplyPanel columns of
// L, one launch per panel over every block of the family:
//   up   (L z_I = b; y = W^T z_I): launch j updates rows [P t, P t + P) of every block (the rows
//        of L below panel j - 1 and the rows of W^T) with panel j - 1, solved by the previous
//        launch, and workgroup t = j then solves its diagonal block (panel j);
//   down (z_I -= W z_B; L^T z_I = b): launch j updates the columns of panel t < j with panel j,
//        and workgroup t = j - 1 then solves its diagonal block.
// The diagonal blocks go through the stored inverses of their 16 x 16 diagonal blocks (the
// solves of the split kernels). phase: 0 gather, 1 T (skeleton blocks), 2 panel step j,
// 3 scatter. Workgroup (b, t) of grid (blocks, ceil((max n_I + n_B) / P)).
// ---------------------------------------------------------------------------------------
constexpr int kBP = kBigApplyPanel;
static_assert(kWG == 2 * kBP, "two threads per row or column of a panel chunk");

// Dot product of two contiguous vectors of length n by one wave: lane l takes the elements
// l, l + 64, ..., eight loads of each vector in flight, into eight partial sums; the total
// is returned to every lane.
__device__ __forceinline__ double wave_dot(const double* __restrict__ x, const double* __restrict__ y, int n,
                                           int lane) {
    double p8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = lane;
    for (; b + 7 * 64 < n; b += 8 * 64) {
        double xv[8], yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            xv[u] = x[b + 64 * u];
            yv[u] = y[b + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) p8[u] += xv[u] * yv[u];
    }
    for (; b < n; b += 64) p8[0] += x[b] * y[b];
    return wave_sum(((p8[0] + p8[1]) + (p8[2] + p8[3])) + ((p8[4] + p8[5]) + (p8[6] + p8[7])));
}

// Rows of panel column block q (16 columns) below which L is structurally zero.
__device__ __forceinline__ int big_rows_end(const ApplyDesc& d, const int32_t* __restrict__ extp, int q) {
    return (extp != nullptr && d.ext >= 0) ? static_cast<int>(extp[d.ext + q]) : d.nI;
}

// Solve the diagonal block of panel j in place (w: the block's staged z_I); TRANS: L^T.
template <bool TRANS>
__device__ __forceinline__ void big_diag_solve(const ApplyDesc& d, const double* __restrict__ A,
                                               const double* __restrict__ li, const int32_t* __restrict__ extp,
                                               double* w, int j, double* zl, int* ex) {
    const int j0 = j * kBP, nb = min(kBP, d.nI - j0);
    // the solves read whole 16-blocks: pad the last one with zeros
    for (int e = threadIdx.x; e < 16 * ((nb + 15) / 16); e += kWG) zl[e] = e < nb ? w[j0 + e] : 0.0;
    for (int q = threadIdx.x; q < (nb + 15) / 16; q += kWG)
        ex[q] = min(nb, max(0, big_rows_end(d, extp, j0 / 16 + q) - j0));
    __syncthreads();
    const double* Ajj = A + j0 + static_cast<size_t>(j0) * d.ld;
    if (TRANS) wg_trsv_bwd(Ajj, d.ld, nb, li + d.li + 256 * (j0 / 16), zl, ex);
    else wg_trsv_fwd(Ajj, d.ld, nb, li + d.li + 256 * (j0 / 16), zl, ex);
    for (int e = threadIdx.x; e < nb; e += kWG) w[j0 + e] = zl[e];
}

__global__ __launch_bounds__(256) void k_apply_big_up(const ApplyDesc* __restrict__ ad, int phase, int j,
                                                      const double* __restrict__ pool, const double* __restrict__ li,
                                                      const double* __restrict__ Tp, const int32_t* __restrict__ dofs,
                                                      const int32_t* __restrict__ extp, double* __restrict__ z,
                                                      double* __restrict__ ybuf, double* __restrict__ ws) {
    __shared__ double xs[kBP], part[kWG], zl[kBP];
    __shared__ int ex[kBP / 16];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nrows = d.nI + d.nB, t = blockIdx.y, tid = threadIdx.x;
    const int r0 = t * kBP;
    if (r0 >= nrows) return;
    const int r1 = min(r0 + kBP, nrows);
    double* w = ws + d.wsoff;
    const int32_t* di = dofs + d.dofs;   // z_I's unknowns, then z_B's
    const double* A = pool + d.off;
    const int np = (nI + kBP - 1) / kBP;
    if (phase == 0) {
        const bool needB = d.toff >= 0 || d.yoff < 0;
        for (int r = r0 + tid; r < r1; r += kWG) w[r] = (r < nI || needB) ? z[di[r]] : 0.0;
        return;
    }
    if (phase == 1) {   // z_I -= T z_B: a wave per row of T, lanes over its (contiguous) columns
        if (d.toff < 0 || r0 >= nI) return;
        const double* T = Tp + d.toff;
        const int lane = tid & 63, wave = tid >> 6;
        for (int a = r0 + wave; a < min(r1, nI); a += kWaves) {
            const double acc = wave_dot(T + static_cast<size_t>(a) * d.nB, w + nI, d.nB, lane);
            if (lane == 0) w[a] -= acc;
        }
        return;
    }
    if (phase == 3) {
        for (int r = r0 + tid; r < r1; r += kWG) {
            if (r < nI) z[di[r]] = w[r];
            else if (d.yoff >= 0) ybuf[d.yoff + (r - nI)] = -w[r];
            else z[di[r]] = w[r];
        }
        return;
    }
    // phase 2: the rows of chunk t below panel j - 1 (rows of L, then of W^T) -= A[rows, panel
    // j - 1] x_{j-1}; then panel j's solve
    const int c0 = (j - 1) * kBP, nc = min(kBP, nI - c0);
    if (j >= 1 && j - 1 < np && r1 > c0 + nc) {
        // padded with zeros: the 16-column steps below read whole column blocks
        for (int c = tid; c < kBP; c += kWG) xs[c] = c < nc ? w[c0 + c] : 0.0;
        __syncthreads();
        // two threads per row, each over half of the panel's columns, 16 at a time (the
        // structural zeros of L below a column block's row end are skipped)
        const int rr = tid & (kBP - 1), h = tid / kBP;
        const int r = r0 + rr;
        double acc = 0.0;
        if (r < r1 && r >= c0 + nc) {
            const int ca = h * (kBP / 2), cb = min(nc, ca + kBP / 2);
            for (int q0 = ca; q0 < cb; q0 += 16) {
                if (r < nI && r >= big_rows_end(d, extp, (c0 + q0) >> 4)) continue;
                const double* Ar = A + r + static_cast<size_t>(c0 + q0) * d.ld;
                const int qn = min(16, cb - q0);
                double v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = u < qn ? Ar[static_cast<size_t>(u) * d.ld] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) acc += v[u] * xs[q0 + u];
            }
        }
        part[tid] = acc;
        __syncthreads();
        if (h == 0 && r < r1 && r >= c0 + nc) w[r] -= part[tid] + part[tid + kBP];
        __syncthreads();
    }
    if (t == j && j < np) big_diag_solve<false>(d, A, li, extp, w, j, zl, ex);
}

__global__ __launch_bounds__(256) void k_apply_big_dn(const ApplyDesc* __restrict__ ad, int phase, int j,
                                                      const double* __restrict__ pool, const double* __restrict__ li,
                                                      const double* __restrict__ Tp, const int32_t* __restrict__ dofs,
                                                      const int32_t* __restrict__ extp, double* __restrict__ z,
                                                      double* __restrict__ ws) {
    __shared__ double xs[kBP], zl[kBP];
    __shared__ int ex[kBP / 16];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nB = d.nB, nrows = nI + nB, t = blockIdx.y, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r0 = t * kBP;
    if (r0 >= nrows) return;
    const int r1 = min(r0 + kBP, nrows);
    double* w = ws + d.wsoff;
    const int32_t* di = dofs + d.dofs;
    const double* A = pool + d.off;
    const int np = (nI + kBP - 1) / kBP;
    if (phase == 0) {
        for (int r = r0 + tid; r < r1; r += kWG) w[r] = z[di[r]];
        return;
    }
    if (phase == 3) {   // scatter z_I; z_B -= T z_I
        for (int r = r0 + tid; r < min(r1, nI); r += kWG) z[di[r]] = w[r];
        if (d.toff >= 0 && r0 < nB) {
            // two threads per column of this chunk, each over half of z_I, eight loads in flight
            __shared__ double half[kBP];
            const double* T = Tp + d.toff;
            const int c = r0 + (tid & (kBP - 1)), h = tid / kBP;
            const int a0 = h == 0 ? 0 : nI / 2, a1 = h == 0 ? nI / 2 : nI;
            double acc = 0.0;
            if (c < nB) {
                double p8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                int a = a0;
                for (; a + 7 < a1; a += 8) {
                    double t8[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) t8[u] = T[c + static_cast<size_t>(a + u) * nB];
#pragma unroll
                    for (int u = 0; u < 8; ++u) p8[u] += t8[u] * w[a + u];
                }
                for (; a < a1; ++a) p8[0] += T[c + static_cast<size_t>(a) * nB] * w[a];
                acc = ((p8[0] + p8[1]) + (p8[2] + p8[3])) + ((p8[4] + p8[5]) + (p8[6] + p8[7]));
            }
            if (h == 1) half[tid - kBP] = acc;
            __syncthreads();
            if (h == 0 && c < nB) z[di[nI + c]] = w[nI + c] - (acc + half[tid]);
        }
        return;
    }
    if (t >= np) return;   // the remaining phases work on the columns of z_I
    const int col0 = t * kBP, ncol = min(kBP, nI - col0);
    if (phase == 1) {
        // z_I -= W z_B on this chunk's columns (a wave per column, lanes over the rows of W^T);
        // then the last panel's solve
        for (int c = wave; c < ncol; c += kWaves) {
            const double acc = wave_dot(A + nI + static_cast<size_t>(col0 + c) * d.ld, w + nI, nB, lane);
            if (lane == 0) w[col0 + c] -= acc;
        }
        __syncthreads();
        if (t == np - 1) big_diag_solve<true>(d, A, li, extp, w, t, zl, ex);
        return;
    }
    // phase 2: columns of chunk t < j -= L[panel j rows, columns]^T x_j; then panel j - 1's solve
    if (j >= np || t >= j) return;
    const int j0 = j * kBP, nr = min(kBP, nI - j0);
    // padded with zeros: every lane reads its kBP / 16 rows below
    for (int e = tid; e < kBP; e += kWG) xs[e] = e < nr ? w[j0 + e] : 0.0;
    __syncthreads();
    // four columns per wave at a time, 16 lanes per column, each lane over kBP / 16 rows
    // (all loads of a column issued before its products)
    const int sub = lane >> 4, le = lane & 15;
    for (int c0 = 4 * wave; c0 < ncol; c0 += 4 * kWaves) {
        const int c = c0 + sub;
        double acc = 0.0;
        if (c < ncol) {
            const int col = col0 + c;
            const int rend = min(nr, big_rows_end(d, extp, col >> 4) - j0);
            const double* Lc = A + j0 + static_cast<size_t>(col) * d.ld;
            double v[kBP / 16];
#pragma unroll
            for (int m = 0; m < kBP / 16; ++m) v[m] = le + 16 * m < rend ? Lc[le + 16 * m] : 0.0;
#pragma unroll
            for (int m = 0; m < kBP / 16; ++m) acc += v[m] * xs[le + 16 * m];
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (le == 0 && c < ncol) w[col0 + c] -= acc;
    }
    __syncthreads();
    if (t == j - 1) big_diag_solve<true>(d, A, li, extp, w, t, zl, ex);
}

// ---------------------------------------------------------------------------------------
// Triangular solves of the apply for banded leaf cells, whose L (from k_leaf_elim) is block
// bidiagonal in 16 x 16 blocks: in steps of 16 rows,
//   up   (L z = b):   z_J = Li_J (b_J - L_J,J-1 z_J-1),            J = 0, 1, ...
//   down (L^T z = b): z_J = Li_J^T (b_J - L_J+1,J^T z_J+1),        J = nb-1, ..., 0
// with the stored inverses Li_J of the diagonal blocks. Each step's two 16 x 16 blocks are
// streamed kBandDepth steps ahead by all threads (one element of each per thread) and
// staged in LDS, so that the chain of steps waits on LDS rather than on memory.
// ---------------------------------------------------------------------------------------
constexpr int kBandDepth = 4;

template <bool UP>
__global__ __launch_bounds__(256) void k_apply_band(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                    const double* __restrict__ lip, const int32_t* __restrict__ dofs,
                                                    double* __restrict__ z) {
    extern __shared__ double smem[];
    constexpr int TS = 16 * 17;
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nb = (nI + 15) / 16, ld = d.ld;
    const double* A = pool + d.off;
    const double* li = lip + d.li;
    const int tid = threadIdx.x, er = tid >> 4, ec = tid & 15;
    double* zI = smem;               // 16 nb
    double* Lt = zI + 16 * nb;       // the step's off-diagonal block, [row][col]
    double* Lit = Lt + TS;           // the step's diagonal-block inverse, [row][col]
    double* yv = Lit + TS;           // 16
    const int32_t* di = dofs + d.dofs;
    for (int i = tid; i < 16 * nb; i += kWG) zI[i] = i < nI ? z[di[i]] : 0.0;
    // operands of step q: UP L_J,J-1 (rows 16J.., cols 16J-16..), DOWN L_J+1,J; and Li_J
    auto blk = [&](int q, double& lv, double& liv) {
        lv = 0.0;
        liv = 0.0;
        if (q >= nb) return;
        const int J = UP ? q : nb - 1 - q, j0 = 16 * J;
        if (UP) {
            if (J > 0 && j0 + er < nI) lv = A[(j0 + er) + static_cast<size_t>(j0 - 16 + ec) * ld];
        } else {
            if (j0 + 16 + er < nI) lv = A[(j0 + 16 + er) + static_cast<size_t>(j0 + ec) * ld];
        }
        liv = li[J * 256 + tid];
    };
    double lr[kBandDepth], lir[kBandDepth];
#pragma unroll
    for (int sl = 0; sl < kBandDepth; ++sl) blk(sl, lr[sl], lir[sl]);
    for (int q0 = 0; q0 < nb; q0 += kBandDepth) {
#pragma unroll
        for (int sl = 0; sl < kBandDepth; ++sl) {
            const int q = q0 + sl;
            if (q >= nb) break;
            Lt[er * 17 + ec] = lr[sl];
            Lit[er * 17 + ec] = lir[sl];
            blk(q + kBandDepth, lr[sl], lir[sl]);
            __syncthreads();
            if (tid < 16) {
                const int i = tid;
                const int J = UP ? q : nb - 1 - q, j0 = 16 * J;
                double acc = zI[j0 + i];
                if (UP && J > 0) {
#pragma unroll
                    for (int c = 0; c < 16; ++c) acc -= Lt[i * 17 + c] * zI[j0 - 16 + c];
                } else if (!UP && J + 1 < nb) {
#pragma unroll
                    for (int c = 0; c < 16; ++c) acc -= Lt[c * 17 + i] * zI[j0 + 16 + c];
                }
                yv[i] = acc;
                __builtin_amdgcn_wave_barrier();
                double v = 0.0;
#pragma unroll
                for (int k = 0; k < 16; ++k) v += (UP ? Lit[i * 17 + k] : Lit[k * 17 + i]) * yv[k];
                zI[j0 + i] = v;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < nI; i += kWG) z[di[i]] = zI[i];
}

template __global__ void k_apply_band<true>(const ApplyDesc*, const double*, const double*, const int32_t*, double*);
template __global__ void k_apply_band<false>(const ApplyDesc*, const double*, const double*, const int32_t*, double*);

// Up-sweep solve: [z_I -= T^T z_B]; z_I <- L^-1 z_I.
__global__ __launch_bounds__(256) void k_apply_trsv_up(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                       const double* __restrict__ lip, const double* __restrict__ Tp,
                                                       const int32_t* __restrict__ dofs, double* __restrict__ z,
                                                       const int32_t* __restrict__ extp) {
    extern __shared__ double smem[];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nB = d.nB;
    const int nt = (nI + 15) / 16;
    const int tid = threadIdx.x;
    double* zI = smem;
    double* zB = zI + nt * 16;
    const bool hasT = d.toff >= 0;
    int* ex = reinterpret_cast<int*>(zB + (hasT ? nB : 0));
    stage_apply_vectors(d, dofs, z, zI, zB, hasT, ex, extp);
    __syncthreads();
    if (hasT) {
        const double* T = Tp + d.toff;
        for (int a = tid; a < nI; a += kWG) {
            double acc = 0.0, acc1 = 0.0;
            const double* Ta = T + static_cast<size_t>(a) * nB;
            int c = 0;
            for (; c + 1 < nB; c += 2) {
                acc += Ta[c] * zB[c];
                acc1 += Ta[c + 1] * zB[c + 1];
            }
            if (c < nB) acc += Ta[c] * zB[c];
            zI[a] -= acc + acc1;
        }
        __syncthreads();
    }
    wg_trsv_fwd(pool + d.off, d.ld, nI, lip + d.li, zI, ex);
    const int32_t* di = dofs + d.dofs;
    for (int i = tid; i < nI; i += kWG) z[di[i]] = zI[i];
}

// Down-sweep solve: z_I <- L^-T z_I; [z_B -= T z_I].
__global__ __launch_bounds__(256) void k_apply_trsv_dn(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                       const double* __restrict__ lip, const double* __restrict__ Tp,
                                                       const int32_t* __restrict__ dofs, double* __restrict__ z,
                                                       const int32_t* __restrict__ extp) {
    extern __shared__ double smem[];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nB = d.nB;
    const int nt = (nI + 15) / 16;
    const int tid = threadIdx.x;
    double* zI = smem;
    double* zB = zI + nt * 16;
    const bool hasT = d.toff >= 0;
    int* ex = reinterpret_cast<int*>(zB + (hasT ? nB : 0));
    stage_apply_vectors(d, dofs, z, zI, zB, hasT, ex, extp);
    __syncthreads();
    wg_trsv_bwd(pool + d.off, d.ld, nI, lip + d.li, zI, ex);
    const int32_t* di = dofs + d.dofs;
    for (int i = tid; i < nI; i += kWG) z[di[i]] = zI[i];
    if (hasT) {
        const double* T = Tp + d.toff;
        for (int c = tid; c < nB; c += kWG) {
            double acc = 0.0, acc1 = 0.0;
            int a = 0;
            for (; a + 1 < nI; a += 2) {
                acc += T[c + static_cast<size_t>(a) * nB] * zI[a];
                acc1 += T[c + static_cast<size_t>(a + 1) * nB] * zI[a + 1];
            }
            if (a < nI) acc += T[c + static_cast<size_t>(a) * nB] * zI[a];
            z[di[nI + c]] = zB[c] - (acc + acc1);
        }
    }
}

// Separator groups of one level, one workgroup per group, all on the group's own unknowns
// staged in LDS (zl in ascending order; zp in the skeleton elimination's order: redundant
// perm[k..n), then skeletons perm[0..k)).
//   up:   z_g -= sum of the cells' y shares; [z_g <- L_g^-1 z_g];
//         [z_r -= T^T z_s; z_r <- L~^-1 z_r; z_s -= W~^T z_r]
//   down: [z_r -= W~ z_s; z_r <- L~^-T z_r; z_s -= T z_r]; [z_g <- L_g^-T z_g]
// T (k x nr, column-major) and G's off-diagonal block G[nr + c, a] (as gk[c + a k]) of a
// skeletonized group into LDS, eight loads in flight per thread.
__device__ __forceinline__ void stage_tg(const double* __restrict__ T, const double* __restrict__ G, int n, int nr,
                                         int k, double* tk, double* gk) {
    const int kn = k * nr;
    for (int e0 = threadIdx.x; e0 < 2 * kn; e0 += 8 * kWG) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kWG;
            v[u] = 0.0;
            if (e < kn) v[u] = T[e];
            else if (e < 2 * kn) {
                const int f = e - kn, c = f % k, a = f / k;
                v[u] = G[(nr + c) + static_cast<size_t>(a) * n];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kWG;
            if (e < kn) tk[e] = v[u];
            else if (e < 2 * kn) gk[e - kn] = v[u];
        }
    }
}

__global__ __launch_bounds__(256) void k_apply_group_up(const GroupApplyDesc* __restrict__ gd,
                                                        const int32_t* __restrict__ gdofs,
                                                        const double* __restrict__ ybuf, double* __restrict__ z,
                                                        const double* __restrict__ Lg, const double* __restrict__ lig,
                                                        const double* __restrict__ Gp, const double* __restrict__ Tp,
                                                        const double* __restrict__ skli,
                                                        const int32_t* __restrict__ perm, int tkcap) {
    extern __shared__ double smem[];
    const GroupApplyDesc g = gd[blockIdx.x];
    z += g.zoff;   // the block's problem within the vector
    const int n = g.n, tid = threadIdx.x;
    const int np = 16 * ((n + 15) / 16);
    double* zl = smem;
    double* zp = smem + np;
    // T and G's off-diagonal block staged in LDS (when the level's largest fit), loaded first
    const bool stg = g.nr > 0 && tkcap > 0;
    double* tk = smem + 2 * np;
    double* gk = tk + g.k * g.nr;
    if (stg) stage_tg(Tp + g.toff, Gp + g.goff, n, g.nr, g.k, tk, gk);
    const int32_t* di = gdofs + g.dofs;
    const int64_t* yoff = gd[blockIdx.x].yoff;   // indexed through memory, not a private copy
    for (int t = tid; t < np; t += kWG) {
        double v = 0.0;
        if (t < n) {
            v = z[di[t]];
            for (int sl = 0; sl < g.nslot; ++sl) v -= ybuf[yoff[sl] + t];
        }
        zl[t] = v;
    }
    __syncthreads();
    if (g.precond) wg_trsv_fwd<false>(Lg + g.loff, n, n, lig + g.li, zl, nullptr);
    if (g.nr > 0) {
        const int nr = g.nr, k = g.k;
        const int32_t* pv = perm + g.poff;
        for (int q = tid; q < np; q += kWG) zp[q] = (q < nr) ? zl[pv[k + q]] : (q < n ? zl[pv[q - nr]] : 0.0);
        __syncthreads();
        const double* T = stg ? tk : Tp + g.toff;
        for (int a = tid; a < nr; a += kWG) {
            double acc = 0.0;
            for (int c = 0; c < k; ++c) acc += T[c + static_cast<size_t>(a) * k] * zp[nr + c];
            zp[a] -= acc;
        }
        __syncthreads();
        const double* G = Gp + g.goff;
        wg_trsv_fwd<false>(G, n, nr, skli + g.skli, zp, nullptr);
        for (int c = tid; c < k; c += kWG) {
            double acc = 0.0;
            if (stg)
                for (int a = 0; a < nr; ++a) acc += gk[c + a * k] * zp[a];
            else
                for (int a = 0; a < nr; ++a) acc += G[(nr + c) + static_cast<size_t>(a) * n] * zp[a];
            zp[nr + c] -= acc;
        }
        __syncthreads();
        for (int q = tid; q < n; q += kWG) zl[q < nr ? pv[k + q] : pv[q - nr]] = zp[q];
        __syncthreads();
    }
    for (int t = tid; t < n; t += kWG) z[di[t]] = zl[t];
}

__global__ __launch_bounds__(256) void k_apply_group_dn(const GroupApplyDesc* __restrict__ gd,
                                                        const int32_t* __restrict__ gdofs, double* __restrict__ z,
                                                        const double* __restrict__ Lg, const double* __restrict__ lig,
                                                        const double* __restrict__ Gp, const double* __restrict__ Tp,
                                                        const double* __restrict__ skli,
                                                        const int32_t* __restrict__ perm, int tkcap) {
    extern __shared__ double smem[];
    const GroupApplyDesc g = gd[blockIdx.x];
    z += g.zoff;   // the block's problem within the vector
    const int n = g.n, tid = threadIdx.x;
    const int np = 16 * ((n + 15) / 16);
    double* zl = smem;
    double* zp = smem + np;
    const bool stg = g.nr > 0 && tkcap > 0;
    double* tk = smem + 2 * np;
    double* gk = tk + g.k * g.nr;
    if (stg) stage_tg(Tp + g.toff, Gp + g.goff, n, g.nr, g.k, tk, gk);
    const int32_t* di = gdofs + g.dofs;
    for (int t = tid; t < np; t += kWG) zl[t] = (t < n) ? z[di[t]] : 0.0;
    __syncthreads();
    if (g.nr > 0) {
        const int nr = g.nr, k = g.k;
        const int32_t* pv = perm + g.poff;
        for (int q = tid; q < np; q += kWG) zp[q] = (q < nr) ? zl[pv[k + q]] : (q < n ? zl[pv[q - nr]] : 0.0);
        __syncthreads();
        const double* G = Gp + g.goff;
        for (int a = tid; a < nr; a += kWG) {
            double acc = 0.0;
            if (stg)
                for (int c = 0; c < k; ++c) acc += gk[c + a * k] * zp[nr + c];
            else {
                const double* Ga = G + static_cast<size_t>(a) * n + nr;
                for (int c = 0; c < k; ++c) acc += Ga[c] * zp[nr + c];
            }
            zp[a] -= acc;
        }
        __syncthreads();
        wg_trsv_bwd<false>(G, n, nr, skli + g.skli, zp, nullptr);
        const double* T = stg ? tk : Tp + g.toff;
        for (int c = tid; c < k; c += kWG) {
            double acc = 0.0;
            for (int a = 0; a < nr; ++a) acc += T[c + static_cast<size_t>(a) * k] * zp[a];
            zp[nr + c] -= acc;
        }
        __syncthreads();
        for (int q = tid; q < n; q += kWG) zl[q < nr ? pv[k + q] : pv[q - nr]] = zp[q];
        __syncthreads();
    }
    if (g.precond) wg_trsv_bwd<false>(Lg + g.loff, n, n, lig + g.li, zl, nullptr);
    for (int t = tid; t < n; t += kWG) z[di[t]] = zl[t];
}

// Up-sweep product y = W^T z_I for 64 rows b of W^T per workgroup (lanes over b, waves
// over quarters of the sum, eight loads in flight); y goes to the gather scratch or is
// subtracted from z_B.
__global__ __launch_bounds__(256) void k_apply_gemv_up(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                       const int32_t* __restrict__ dofs, double* __restrict__ z,
                                                       double* __restrict__ ybuf) {
    extern __shared__ double smem[];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nB = d.nB, ld = d.ld;
    const int b0 = 64 * static_cast<int>(blockIdx.y);
    if (b0 >= nB) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* zI = smem;
    double* red = smem + nI;
    const int32_t* di = dofs + d.dofs;
    for (int i = tid; i < nI; i += kWG) zI[i] = z[di[i]];
    __syncthreads();
    const int b = b0 + lane;
    const int q0 = (nI * wave) / kWaves, q1 = (nI * (wave + 1)) / kWaves;
    double acc = 0.0;
    if (b < nB) {
        const double* Wb = pool + d.off + nI + b;
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int i = q0;
        // sixteen loads in flight, two rounds of the eight partial sums
        for (; i + 15 < q1; i += 16) {
            double x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) x[u] = Wb[static_cast<size_t>(i + u) * ld];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += x[u] * zI[i + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += x[8 + u] * zI[i + 8 + u];
        }
        for (; i + 7 < q1; i += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += Wb[static_cast<size_t>(i + u) * ld] * zI[i + u];
        }
        for (; i < q1; ++i) a[0] += Wb[static_cast<size_t>(i) * ld] * zI[i];
        acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    red[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave == 0 && b < nB) {
        const double y = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
        if (d.yoff >= 0) ybuf[d.yoff + b] = y;
        else z[di[nI + b]] -= y;
    }
}

// Down-sweep product z_I -= W z_B for 64 unknowns i of z_I per workgroup: 64 x 64 tiles of
// W^T are read coalesced (along b) into LDS and summed along b by (i, quarter) threads.
__global__ __launch_bounds__(256) void k_apply_gemv_dn(const ApplyDesc* __restrict__ ad, const double* __restrict__ pool,
                                                       const int32_t* __restrict__ dofs, double* __restrict__ z) {
    extern __shared__ double smem[];
    const ApplyDesc d = ad[blockIdx.x];
    z += d.zoff;   // the block's problem within the vector
    const int nI = d.nI, nB = d.nB, ld = d.ld;
    const int i0 = 64 * static_cast<int>(blockIdx.y);
    if (i0 >= nI || nB == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* tile = smem;                 // [i][b], stride 65
    double* zB = smem + 64 * 65;
    double* red = zB + nB;
    const int32_t* di = dofs + d.dofs;
    for (int c = tid; c < nB; c += kWG) zB[c] = z[di[nI + c]];
    const double* Wt = pool + d.off + nI;
    double acc = 0.0;
    for (int bc = 0; bc < nB; bc += 64) {
        __syncthreads();
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + u * kWG;
            const int br = e & 63, ir = e >> 6;
            const int b = bc + br, i = i0 + ir;
            v[u] = (b < nB && i < nI) ? Wt[b + static_cast<size_t>(i) * ld] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + u * kWG;
            tile[(e >> 6) * 65 + (e & 63)] = v[u];
        }
        __syncthreads();
        const int bl = min(64, nB - bc);
        for (int br = wave * 16; br < min(bl, wave * 16 + 16); ++br) acc += tile[lane * 65 + br] * zB[bc + br];
    }
    red[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave == 0 && i0 + lane < nI) {
        const double s = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
        z[di[i0 + lane]] -= s;
    }
}

// Up-sweep gather: z_g -= sum over the cells containing g (ascending) of their y share.
__global__ __launch_bounds__(256) void k_sep_gather(const GatherDesc* __restrict__ gd, const int32_t* __restrict__ dofs,
                                                    const double* __restrict__ ybuf, double* __restrict__ z) {
    const GatherDesc g = gd[blockIdx.x];
    z += g.zoff;   // the block's problem within the vector
    for (int t = threadIdx.x; t < g.n; t += kWG) {
        const int i = dofs[g.dofs + t];
        double v = z[i];
        for (int sl = 0; sl < g.nslot; ++sl) v -= ybuf[g.yoff[sl] + t];
        z[i] = v;
    }
}

// ---------------------------------------------------------------------------------------
// CG building blocks. Reductions are two-stage with a fixed grid: kRedBlocks partial sums
// in a fixed layout, then one block adds them in a fixed order.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kWaves; ++w) s += red[w];
    __syncthreads();
    return s;
}

// q = A p and partial sums of p . q
__global__ __launch_bounds__(256) void k_spmv_dot(int64_t N, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                  const double* __restrict__ v, const double* __restrict__ p,
                                                  double* __restrict__ q, double* __restrict__ part) {
    __shared__ double red[kWaves];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; i < N; i += static_cast<int64_t>(gridDim.x) * kWG) {
        double s = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * p[ci[e]];
        q[i] = s;
        acc += s * p[i];
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_dot(int64_t N, const double* __restrict__ x, const double* __restrict__ y,
                                             double* __restrict__ part) {
    __shared__ double red[kWaves];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; i < N; i += static_cast<int64_t>(gridDim.x) * kWG)
        acc += x[i] * y[i];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// scalar slots: 0 rho, 1 pq, 2 alpha, 3 rr, 4 rho_new, 5 beta, 6 ff
// mode 0: sc[6] = sum;   mode 1: sc[1] = sum, alpha = rho / pq;   mode 2: sc[3] = sum;
// mode 3: rho = sum (initial);   mode 4: beta = sum / rho, rho = sum.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ part, int nparts, int mode,
                                                  double* __restrict__ sc, double* __restrict__ host_out) {
    __shared__ double red[kWaves];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) acc += part[b];
    const double s = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    switch (mode) {
        case 0: sc[6] = s; if (host_out) host_out[0] = s; break;
        case 1: sc[1] = s; sc[2] = sc[0] / s; break;
        case 2: sc[3] = s; if (host_out) host_out[0] = s; break;
        case 3: sc[0] = s; break;
        case 4: sc[4] = s; sc[5] = s / sc[0]; sc[0] = s; break;
        case 5: sc[7] = s; break;                                        // r_new . z_old
        case 6: sc[4] = s; sc[5] = (s - sc[7]) / sc[0]; sc[0] = s; break;  // Polak-Ribiere beta
        default: break;
    }
}

// u += alpha p ; r -= alpha q ; partial sums of r . r
// With zold (the flexible, Polak-Ribiere form of the iteration), also partial sums of
// r_new . zold into part2.
__global__ __launch_bounds__(256) void k_axpy2(int64_t N, const double* __restrict__ sc, const double* __restrict__ p,
                                               const double* __restrict__ q, double* __restrict__ u, double* __restrict__ r,
                                               double* __restrict__ part, const double* __restrict__ zold,
                                               double* __restrict__ part2) {
    __shared__ double red[kWaves];
    const double alpha = sc[2];
    double acc = 0.0, acc2 = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; i < N; i += static_cast<int64_t>(gridDim.x) * kWG) {
        u[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
        if (zold != nullptr) acc2 += ri * zold[i];
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    if (zold != nullptr) {
        const double t2 = block_sum(acc2, red);
        if (threadIdx.x == 0) part2[blockIdx.x] = t2;
    }
}

// p = z + beta p
__global__ __launch_bounds__(256) void k_update_p(int64_t N, const double* __restrict__ sc, const double* __restrict__ z,
                                                  double* __restrict__ p) {
    const double beta = sc[5];
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; i < N; i += static_cast<int64_t>(gridDim.x) * kWG)
        p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(256) void k_copy(int64_t N, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; i < N; i += static_cast<int64_t>(gridDim.x) * kWG)
        y[i] = x[i];
}

// y = a x + b y
__global__ __launch_bounds__(256) void k_axpby(int64_t N, double a, const double* __restrict__ x, double b,
                                               double* __restrict__ y) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; i < N; i += static_cast<int64_t>(gridDim.x) * kWG)
        y[i] = a * x[i] + b * y[i];
}
__global__ __launch_bounds__(256) void k_fill(int64_t N, double v, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kWG) + threadIdx.x; i < N; i += static_cast<int64_t>(gridDim.x) * kWG)
        y[i] = v;
}

// ---------------------------------------------------------------------------------------
// The same vector kernels for a PCG over several problems at once: block b works for problem
// blk[b] exactly as block b - b0 of that problem's lone grid would (same rows, same partial
// sums), every problem with its own scalars (16 slots each). An inactive problem (converged)
// gets alpha = beta = 0, which leaves its solution and residual as they are.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bspmv_dot(const BatchSeg* __restrict__ seg, const int32_t* __restrict__ blk,
                                                   const double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ part) {
    __shared__ double red[kWaves];
    const BatchSeg g = seg[blk[blockIdx.x]];
    const double* pp = p + g.zoff;
    double* qq = q + g.zoff;
    double acc = 0.0;
    for (int64_t i = (blockIdx.x - g.b0) * static_cast<int64_t>(kWG) + threadIdx.x; i < g.n;
         i += static_cast<int64_t>(g.nb) * kWG) {
        double s = 0.0;
        for (int e = g.rp[i]; e < g.rp[i + 1]; ++e) s += g.val[e] * pp[g.ci[e]];
        qq[i] = s;
        acc += s * pp[i];
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_bdot(const BatchSeg* __restrict__ seg, const int32_t* __restrict__ blk,
                                              const double* __restrict__ x, const double* __restrict__ y,
                                              double* __restrict__ part) {
    __shared__ double red[kWaves];
    const BatchSeg g = seg[blk[blockIdx.x]];
    const double* xx = x + g.zoff;
    const double* yy = y + g.zoff;
    double acc = 0.0;
    for (int64_t i = (blockIdx.x - g.b0) * static_cast<int64_t>(kWG) + threadIdx.x; i < g.n;
         i += static_cast<int64_t>(g.nb) * kWG)
        acc += xx[i] * yy[i];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// One workgroup per problem: its partial sums in the order of k_finalize, the modes of
// k_finalize on its 16 scalar slots.
__global__ __launch_bounds__(256) void k_bfinalize(const BatchSeg* __restrict__ seg, const double* __restrict__ part,
                                                   int mode, double* __restrict__ sc, const int32_t* __restrict__ active) {
    __shared__ double red[kWaves];
    const BatchSeg g = seg[blockIdx.x];
    double acc = 0.0;
    for (int b = threadIdx.x; b < g.nb; b += blockDim.x) acc += part[g.b0 + b];
    const double s = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    double* c = sc + 16 * blockIdx.x;
    const bool on = active[blockIdx.x] != 0;
    switch (mode) {
        case 0: c[6] = s; break;
        case 1: c[1] = s; c[2] = on ? c[0] / s : 0.0; break;
        case 2: c[3] = s; break;
        case 3: c[0] = s; break;
        case 4: c[4] = s; c[5] = on ? s / c[0] : 0.0; c[0] = s; break;
        case 5: c[7] = s; break;
        case 6: c[4] = s; c[5] = on ? (s - c[7]) / c[0] : 0.0; c[0] = s; break;
        default: break;
    }
}

__global__ __launch_bounds__(256) void k_baxpy2(const BatchSeg* __restrict__ seg, const int32_t* __restrict__ blk,
                                                const double* __restrict__ sc, const double* __restrict__ p,
                                                const double* __restrict__ q, double* __restrict__ u,
                                                double* __restrict__ r, double* __restrict__ part,
                                                const double* __restrict__ zold, double* __restrict__ part2) {
    __shared__ double red[kWaves];
    const int pb = blk[blockIdx.x];
    const BatchSeg g = seg[pb];
    const double alpha = sc[16 * pb + 2];
    const int64_t o = g.zoff;
    double acc = 0.0, acc2 = 0.0;
    for (int64_t i = (blockIdx.x - g.b0) * static_cast<int64_t>(kWG) + threadIdx.x; i < g.n;
         i += static_cast<int64_t>(g.nb) * kWG) {
        u[o + i] += alpha * p[o + i];
        const double ri = r[o + i] - alpha * q[o + i];
        r[o + i] = ri;
        acc += ri * ri;
        if (zold != nullptr) acc2 += ri * zold[o + i];
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    if (zold != nullptr) {
        const double t2 = block_sum(acc2, red);
        if (threadIdx.x == 0) part2[blockIdx.x] = t2;
    }
}

__global__ __launch_bounds__(256) void k_bupdate_p(const BatchSeg* __restrict__ seg, const int32_t* __restrict__ blk,
                                                   const double* __restrict__ sc, const double* __restrict__ z,
                                                   double* __restrict__ p) {
    const int pb = blk[blockIdx.x];
    const BatchSeg g = seg[pb];
    const double beta = sc[16 * pb + 5];
    const int64_t o = g.zoff;
    for (int64_t i = (blockIdx.x - g.b0) * static_cast<int64_t>(kWG) + threadIdx.x; i < g.n;
         i += static_cast<int64_t>(g.nb) * kWG)
        p[o + i] = z[o + i] + beta * p[o + i];
}

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace rhif
