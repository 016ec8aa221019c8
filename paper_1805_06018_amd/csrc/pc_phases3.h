// Steps of the 3-D work items (Item3), shared by the GPU kernels and the
// CPU emulation like the 2-D phases.
//
// A patch's FFT box nz x n1 x 2m is transformed in three launches:
//   plane-forward: every gathered plane (axis-0 index) runs phases A-C and
//     the forward column pass 2 along axis 1, then its n1 x (m + 1) spectrum
//     goes to the item's scratch area (plane-major, row stride m + 1);
//   axis-0: a block takes a range of flattened (axis-1, axis-2) frequency
//     columns, loads the gathered planes of those columns into LDS and runs
//     phases C, D (product with the 3-D spectrum) and E along axis 0, then
//     writes the planes the output needs back to scratch;
//   plane-inverse: every written plane loads its spectrum from scratch and
//     runs the inverse column pass 2 and phases E-H into its staging plane.
// The 3-D spectrum is stored as nz x n1 x (m + 1) in the permuted slot order
// of each axis, so the axis-0 block reads column c of axis-0 slot s at
// spec[s * n1 (m + 1) + c].
#pragma once
#include "pc_phases.h"

namespace pc {

// Axis-0 planes (FFT coordinates) gathered (s) and written (d).
struct Planes {
    int s_off, s_n, d_off, d_n;
};

__host__ __device__ inline Planes planes_of(const Item3& I, bool adj) {
    if (!adj) return Planes{I.in_offz, I.in_nz, I.out_offz, I.out_nz};
    return Planes{I.out_offz, I.out_nz, I.in_offz, I.in_nz};
}

__host__ __device__ inline int64_t plane_elems(const Item3& I) { return (int64_t)I.p.n0 * (I.p.m + 1); }

// Scratch of one item and vector in a launch over a contiguous item range
// whose first item has scratch offset 'base' and B vectors: layout
// [item][vector][nz][n1][m + 1].
template <class T>
__host__ __device__ inline cx<T>* item_scratch(cx<T>* scratch, int64_t base, const Item3& I, int B, int rhs) {
    return scratch + (I.scratch_off - base) * B + (int64_t)rhs * I.nz * plane_elems(I);
}

// Context of the q-th gathered plane: source rows in that Omega plane,
// forward weights of that plane of the patch box.
template <class T>
__host__ __device__ inline Ctx<T> plane_ctx_gather(const Item3& I, bool adj, int q, const T* in_vec, T* slot_vec,
                                                   const T* wts, const cx<T>* spec, const cx<T>* tw, int64_t pitch,
                                                   int64_t plane_pitch) {
    const Planes pl = planes_of(I, adj);
    Ctx<T> c = make_ctx<T>(I.p, adj, in_vec + (int64_t)(I.gz + pl.s_off + q) * plane_pitch, slot_vec, wts, spec, tw,
                           pitch);
    if (!adj) c.w += (int64_t)q * I.w_plane;
    return c;
}

// Context of the q-th written plane: its staging plane, adjoint weights of
// that plane of the patch box.
template <class T>
__host__ __device__ inline Ctx<T> plane_ctx_write(const Item3& I, bool adj, int q, const T* in_vec, T* slot_vec,
                                                  const T* wts, const cx<T>* spec, const cx<T>* tw, int64_t pitch) {
    Ctx<T> c = make_ctx<T>(I.p, adj, in_vec, slot_vec, wts, spec, tw, pitch);
    c.dst += (int64_t)q * c.d_n0 * c.dst_rs;
    if (adj) c.w += (int64_t)q * I.w_plane;
    return c;
}

// Copies between LDS and scratch move copy_batch<T>() elements per thread
// per step: all reads of a step are issued before its writes.  Measured on
// the 128^3 workload: FP32 gains from 8 in flight (28.7 -> 24.4 ms per
// apply); the FP64 kernels, at two waves per SIMD, lose from any batching
// (66.8 / 73.5 / 82.0 / 93.3 ms for 1 / 2 / 4 / 8).
template <class T>
__host__ __device__ constexpr int copy_batch() { return sizeof(T) == 8 ? 1 : 8; }

// LDS plane (n1 rows of m + 1 complex, row stride ld) <-> scratch plane
// (row stride m + 1); consecutive threads on consecutive elements.  Scratch
// is written once and read once, by the next kernel: the stores are
// non-temporal (128^3 workload: 24.3 -> 23.5 ms per apply).
template <class T>
__host__ __device__ inline void plane_store(const Ctx<T>& c, const cx<T>* buf, cx<T>* dst, int tid, int nth) {
    constexpr int U = copy_batch<T>();
    const int NC = c.it.m + 1, n = c.it.n0 * NC;
    for (int t0 = tid; t0 < n; t0 += U * nth) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * nth;
            if (t < n) {
                const int row = fdiv(t, c.inv_nc), col = t - imul24(row, NC);
                v[u] = buf[imul24(row, c.it.ld) + col];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + u * nth < n) {
                __builtin_nontemporal_store(v[u].x, &dst[t0 + u * nth].x);
                __builtin_nontemporal_store(v[u].y, &dst[t0 + u * nth].y);
            }
    }
}

template <class T>
__host__ __device__ inline void plane_load(const Ctx<T>& c, cx<T>* buf, const cx<T>* src, int tid, int nth) {
    constexpr int U = copy_batch<T>();
    const int NC = c.it.m + 1, n = c.it.n0 * NC;
    for (int t0 = tid; t0 < n; t0 += U * nth) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * nth;
            if (t < n) v[u] = src[t];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * nth;
            if (t < n) {
                const int row = fdiv(t, c.inv_nc), col = t - imul24(row, NC);
                buf[imul24(row, c.it.ld) + col] = v[u];
            }
        }
    }
}

// Context of the axis-0 block over columns [c_lo, c_lo + ncols): phases C-E
// see an nz x ncols box (it.m + 1 = ncols) with LDS row stride ld.
template <class T>
__host__ __device__ inline Ctx<T> axis_ctx(const Item3& I, bool adj, int c_lo, int ncols, int ld, const cx<T>* spec,
                                           const cx<T>* tw) {
    Ctx<T> c;
    Item it = I.p;
    it.n0 = I.nz;
    it.a0 = I.az;
    it.b0 = I.bz;
    it.m = ncols - 1;
    it.ld = ld;
    c.it = it;
    c.adj = adj;
    const Planes pl = planes_of(I, adj);
    c.s_off0 = pl.s_off;
    c.s_n0 = pl.s_n;
    c.d_off0 = pl.d_off;
    c.d_n0 = pl.d_n;
    c.s_off1 = 0;
    c.s_n1 = ncols;
    c.d_off1 = 0;
    c.d_n1 = ncols;
    c.inv_bm = 1.0f;
    c.inv_b0 = 1.0f / (float)I.bz;
    c.inv_nc = 1.0f / (float)ncols;
    c.inv_sn0 = 1.0f / (float)pl.s_n;
    c.inv_dn0 = 1.0f / (float)pl.d_n;
    c.src = nullptr;
    c.dst = nullptr;
    c.dst_rs = 0;
    c.add = false;
    c.w = nullptr;
    c.spec = spec + I.p.spec_off + c_lo;
    c.spec_ld = (int)plane_elems(I);
    c.tw0 = tw + I.twz;
    c.twm = c.tw0;
    c.tw2m = c.tw0;
    c.pitch = 0;
    return c;
}

// Gathered planes of the block's columns: scratch (plane stride pe) -> LDS.
template <class T>
__host__ __device__ inline void axis_load(const Ctx<T>& c, cx<T>* buf, const cx<T>* sc, int64_t pe, int tid, int nth) {
    constexpr int U = copy_batch<T>();
    const int NC = c.it.m + 1, n = c.s_n0 * NC;
    for (int t0 = tid; t0 < n; t0 += U * nth) {
        cx<T> v[U];
        int li[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * nth;
            li[u] = -1;
            if (t < n) {
                const int q = fdiv(t, c.inv_nc), col = t - imul24(q, NC);
                const int row = c.s_off0 + q;
                li[u] = imul24(row, c.it.ld) + col;
                v[u] = sc[(int64_t)row * pe + col];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (li[u] >= 0) buf[li[u]] = v[u];
    }
}

// Written planes of the block's columns: LDS -> scratch.
template <class T>
__host__ __device__ inline void axis_store(const Ctx<T>& c, const cx<T>* buf, cx<T>* sc, int64_t pe, int tid, int nth) {
    constexpr int U = copy_batch<T>();
    const int NC = c.it.m + 1, n = c.d_n0 * NC;
    for (int t0 = tid; t0 < n; t0 += U * nth) {
        cx<T> v[U];
        int64_t gi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * nth;
            gi[u] = -1;
            if (t < n) {
                const int q = fdiv(t, c.inv_nc), col = t - imul24(q, NC);
                const int row = c.d_off0 + q;
                gi[u] = (int64_t)row * pe + col;
                v[u] = buf[imul24(row, c.it.ld) + col];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (gi[u] >= 0) {
                __builtin_nontemporal_store(v[u].x, &sc[gi[u]].x);
                __builtin_nontemporal_store(v[u].y, &sc[gi[u]].y);
            }
    }
}

// Axis-0 pass-1 twiddles (bz (az - 1) complex, runs per task) copied into
// LDS after the block's box.
template <class T>
__host__ __device__ inline void axis_twiddles_to_lds(Ctx<T>& c, cx<T>* dst, int tid, int nth) {
    const int n = c.it.b0 * (c.it.a0 - 1);
    for (int t = tid; t < n; t += nth) dst[t] = c.tw0[t];
    c.tw0 = dst;
    c.twm = dst;
    c.tw2m = dst;
}

// LDS row stride of the axis-0 block (odd, at least the column count + 1).
__host__ __device__ constexpr int axis_ld(int cols) { return (cols + 1) % 2 ? cols + 1 : cols + 2; }

}  // namespace pc
