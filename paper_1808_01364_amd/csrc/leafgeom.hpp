// Level-0 groups and frontal unknowns in closed form.
//
// At level 0 every unknown is active, so the groups of Sec. 3.1 / 3.2 are boxes of the grid:
// along each axis a cell of width w contributes either its open slab or one of its two
// bounding planes. The host planner enumerates these boxes to build its tables; a device
// kernel evaluates the same functions to write the frontal unknowns of every leaf cell
// directly, so that the host does not have to build and upload them. Both are constexpr and
// therefore usable on the host and on the device.
#pragma once
#include <cstdint>

namespace rhif {

// The group of the cell with coordinates c[0..d-1] selected by slot code t: digit k of t in
// base 3 picks, along axis k, the plane x_k = c_k w (0), the open slab c_k w < x_k < (c_k+1) w
// clipped to x_k <= s (1) or the plane x_k = (c_k+1) w (2). Returns its number of grid points,
// 0 if a plane lies outside 1..s or the slab is empty; lo and n receive the box's lowest
// corner and extents (axes >= d: lo = n = 1).
constexpr int64_t leaf_group_box(int d, int s, int w, const int* c, int t, int* lo, int* n) {
    for (int k = 0; k < 3; ++k) {
        lo[k] = 1;
        n[k] = 1;
    }
    int64_t cnt = 1;
    for (int k = 0; k < d; ++k) {
        const int dk = t % 3;
        t /= 3;
        if (dk == 1) {
            const int64_t a = static_cast<int64_t>(c[k]) * w + 1;
            const int64_t top = static_cast<int64_t>(c[k] + 1) * w - 1;
            const int64_t b = top < s ? top : s;
            if (a > b) return 0;
            lo[k] = static_cast<int>(a);
            n[k] = static_cast<int>(b - a + 1);
        } else {
            const int64_t x = static_cast<int64_t>(c[k] + (dk == 2 ? 1 : 0)) * w;
            if (x < 1 || x > s) return 0;
            lo[k] = static_cast<int>(x);
        }
        cnt *= n[k];
    }
    return cnt;
}

// Global index (x_1 fastest, 0-based) of frontal position p of leaf cell `cell` (cells
// numbered with the first axis fastest, nc1 per axis): the interior box first, then the
// boundary groups by ascending slot code, each box in ascending order. -1 if p >= the
// frontal size.
constexpr int32_t leaf_frontal_dof(int d, int s, int w, int nc1, int cell, int p) {
    int c[3] = {0, 0, 0};
    int r = cell;
    for (int k = 0; k < d; ++k) {
        c[k] = r % nc1;
        r /= nc1;
    }
    int n3 = 1;
    for (int k = 0; k < d; ++k) n3 *= 3;
    const int t_int = (n3 - 1) / 2;   // every digit 1: the interior
    int lo[3] = {1, 1, 1}, n[3] = {1, 1, 1};
    int64_t q = p;
    for (int e = -1; e < n3; ++e) {
        if (e == t_int) continue;
        const int64_t cnt = leaf_group_box(d, s, w, c, e < 0 ? t_int : e, lo, n);
        if (q < cnt) {
            const int64_t x0 = lo[0] + q % n[0];
            const int64_t x1 = lo[1] + (q / n[0]) % n[1];
            const int64_t x2 = lo[2] + q / (static_cast<int64_t>(n[0]) * n[1]);
            int64_t i = x0 - 1;
            if (d > 1) i += (x1 - 1) * s;
            if (d > 2) i += (x2 - 1) * static_cast<int64_t>(s) * s;
            return static_cast<int32_t>(i);
        }
        q -= cnt;
    }
    return -1;
}

}  // namespace rhif
