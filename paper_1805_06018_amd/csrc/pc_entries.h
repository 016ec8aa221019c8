// Matrix entries of the product-convolution operator (Sec. 3.1):
//   A~[y, x] = sum_{k : x in U_k} w_k[x] phi_k^E[y - x].
// w_k vanishes on every leaf not containing p_k, so the sum runs over the
// points of one leaf containing x (any one: on a shared facet the other
// leaf's extra points have zero weight there).  Shared by the GPU kernel and
// the CPU emulation.
#pragma once
#include <stdint.h>
#include "pc_internal.h"

namespace pc {

// Tables in the planes x prow x cols view of Omega (d < 3: one plane).
struct EntryTables {
    int d;
    int planes, prow, cols;
    const int32_t* leaf_of;   // [N] a leaf containing each grid point
    const int32_t* lp_off;    // [L+1] CSR of the points on each closed leaf
    const int32_t* lp;
    const int64_t* wbase;     // [r] weight table offset, -1 if the term is not kept
    const int32_t* ubox;      // [r][6] bbox(U_k): origin, extents
    const int64_t* eoff;      // [r] offset of phi_k^E
    const int32_t* ebox;      // [r][6] box of phi_k^E: offset origin, extents
};

// Omega coordinates (d of them) -> (plane, row, col); false if outside.
__host__ __device__ inline bool view_coords(const EntryTables& E, const int64_t* c, int64_t* v) {
    v[0] = E.d == 3 ? c[0] : 0;
    v[1] = E.d == 3 ? c[1] : (E.d == 2 ? c[0] : 0);
    v[2] = c[E.d - 1];
    return v[0] >= 0 && v[0] < E.planes && v[1] >= 0 && v[1] < E.prow && v[2] >= 0 && v[2] < E.cols;
}

// One entry in FP64 (terms added in ascending k); NaN if y or x is outside
// Omega.
template <class T>
__host__ __device__ inline double entry_value(const EntryTables& E, const T* wts, const T* phiE, const int64_t* y,
                                              const int64_t* x) {
    int64_t yv[3], xv[3];
    if (!view_coords(E, y, yv) || !view_coords(E, x, xv)) return __builtin_nan("");
    const int32_t leaf = E.leaf_of[(xv[0] * E.prow + xv[1]) * E.cols + xv[2]];
    double acc = 0.0;
    for (int32_t j = E.lp_off[leaf]; j < E.lp_off[leaf + 1]; ++j) {
        const int32_t k = E.lp[j];
        const int64_t wb = E.wbase[k];
        if (wb < 0) continue;
        const int32_t* u = E.ubox + 6 * (int64_t)k;
        const double w =
            (double)wts[wb + ((xv[0] - u[0]) * u[4] + (xv[1] - u[1])) * (int64_t)u[5] + (xv[2] - u[2])];
        const int32_t* e = E.ebox + 6 * (int64_t)k;
        const int64_t z0 = yv[0] - xv[0] - e[0], z1 = yv[1] - xv[1] - e[1], z2 = yv[2] - xv[2] - e[2];
        if (z0 < 0 || z0 >= e[3] || z1 < 0 || z1 >= e[4] || z2 < 0 || z2 >= e[5]) continue;
        acc += w * (double)phiE[E.eoff[k] + (z0 * e[4] + z1) * (int64_t)e[5] + z2];
    }
    return acc;
}

}  // namespace pc
