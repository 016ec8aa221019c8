// The nine phases of one convolution work item (a patch or row piece of the
// product-convolution sum, eq. 2.3, or of its adjoint, eq. 1.4).
//
// Work item layout: an n0 x n1 FFT box (n1 = 2m) lives in LDS as n0 rows of
// m + 1 complex columns (row stride ld).  Each real row of length 2m is
// transformed as a complex length-m FFT of (even, odd) sample pairs plus a
// post-processing step; every 1-D FFT of length n = a * b runs as two
// in-place register passes:
//   pass 1: for each j0 < b, DFT_a over x[b j1 + j0], times w_n^(j0 k1);
//   pass 2: for each k1 < a, DFT_b over slots b k1 + (0..b-1).
// Frequency k = k1 + a k0 ends in slot b k1 + k0 (permuted order).  The
// kernel spectra are stored in the same permuted order, and the inverse
// transform undoes the passes in reverse, so no reordering pass is needed.
//
// Phases (one barrier between consecutive phases):
//   1 gather (weighted for the forward sum) + row pass 1
//   2 row pass 2
//   3 real-row post-processing (thread-private, in place)
//   4 column pass 1 (only the gathered rows are non-zero)
//   5 column pass 2, product with the spectrum (conjugate for the adjoint),
//     inverse column pass 2
//   6 inverse column pass 1 (only rows needed by the output are kept)
//   7 real-row pre-processing for the inverse
//   8 inverse row pass 2
//   9 inverse row pass 1 + write of the output box (weighted for the adjoint)
//
// All functions are __host__ __device__: the GPU kernel runs them with a
// barrier in between; a host-only build can run them thread by thread.
#pragma once
#include "pc_fft.h"
#include "pc_internal.h"

namespace pc {

template <class T>
struct Ctx {
    Item it;
    bool adj;
    int s_off0, s_n0, s_off1, s_n1;   // gathered box (FFT coordinates)
    int d_off0, d_n0, d_off1, d_n1;   // written box
    const T* src;                     // input vector, Omega origin
    T* dst;                           // staging box of this item and vector
    const T* w;                       // weight table of the item's input box
    const cx<T>* spec;
    const cx<T>* tw0;                 // w_{n0}^e
    const cx<T>* twm;                 // w_m^e
    const cx<T>* tw2m;                // w_{2m}^e
    int64_t pitch;                    // Omega row pitch (elements)
};

template <class T>
__host__ __device__ inline Ctx<T> make_ctx(const Item& it, bool adj, const T* in_vec, T* slot_vec,
                                           const T* wts, const cx<T>* spec, const cx<T>* tw, int64_t pitch) {
    Ctx<T> c;
    c.it = it;
    c.adj = adj;
    if (!adj) {
        c.s_off0 = it.in_off0; c.s_n0 = it.in_n0; c.s_off1 = it.in_off1; c.s_n1 = it.in_n1;
        c.d_off0 = 0; c.d_n0 = it.out_n0; c.d_off1 = 0; c.d_n1 = it.out_n1;
        c.dst = slot_vec + it.slot_fwd;
    } else {
        c.s_off0 = 0; c.s_n0 = it.out_n0; c.s_off1 = 0; c.s_n1 = it.out_n1;
        c.d_off0 = it.in_off0; c.d_n0 = it.in_n0; c.d_off1 = it.in_off1; c.d_n1 = it.in_n1;
        c.dst = slot_vec + it.slot_adj;
    }
    c.src = in_vec;
    c.w = wts + it.w_off;
    c.spec = spec + it.spec_off;
    c.tw0 = tw + it.tw0;
    c.twm = tw + it.twm;
    c.tw2m = tw + it.tw2m;
    c.pitch = pitch;
    return c;
}

// 1: gather + row pass 1 (forward DFT_am, twiddle w_m^(j0 k1))
template <class T>
__host__ __device__ inline void ph1(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int am = c.it.am, bm = c.it.bm, ld = c.it.ld;
    const int ntask = c.s_n0 * bm;
    for (int t = tid; t < ntask; t += nth) {
        const int j0 = t % bm, q = t / bm;
        const int row = c.s_off0 + q;
        const T* srow = c.src + (int64_t)(c.it.g0 + row) * c.pitch + c.it.g1;
        const T* wrow = c.w + (int64_t)q * c.s_n1;
        cx<T> x[kMaxRadix];
#pragma unroll
        for (int j1 = 0; j1 < kMaxRadix; ++j1) {
            if (j1 < am) {
                const int j = bm * j1 + j0;
                const int e0 = 2 * j - c.s_off1, e1 = e0 + 1;
                T v0 = T(0), v1 = T(0);
                if ((unsigned)e0 < (unsigned)c.s_n1) {
                    v0 = srow[2 * j];
                    if (!c.adj) v0 *= wrow[e0];
                }
                if ((unsigned)e1 < (unsigned)c.s_n1) {
                    v1 = srow[2 * j + 1];
                    if (!c.adj) v1 *= wrow[e1];
                }
                x[j1] = {v0, v1};
            }
        }
        dft_rt<-1>(am, x);
        cx<T>* out = buf + (int64_t)row * ld + j0;
#pragma unroll
        for (int k1 = 0; k1 < kMaxRadix; ++k1)
            if (k1 < am) out[bm * k1] = cmul(x[k1], c.twm[j0 * k1]);
    }
}

// 2 (forward) / 8 (inverse): row pass 2 over rows [r_off, r_off + r_n)
template <int S, class T>
__host__ __device__ inline void ph_rows2(const Ctx<T>& c, cx<T>* buf, int tid, int nth, int r_off, int r_n) {
    const int am = c.it.am, bm = c.it.bm, ld = c.it.ld;
    const int ntask = r_n * am;
    for (int t = tid; t < ntask; t += nth) {
        const int r = t % r_n, k1 = t / r_n;
        cx<T>* p = buf + (int64_t)(r_off + r) * ld + bm * k1;
        cx<T> x[kMaxRadix];
#pragma unroll
        for (int k0 = 0; k0 < kMaxRadix; ++k0)
            if (k0 < bm) x[k0] = p[k0];
        dft_rt<S>(bm, x);
#pragma unroll
        for (int k0 = 0; k0 < kMaxRadix; ++k0)
            if (k0 < bm) p[k0] = x[k0];
    }
}

__host__ __device__ inline int slot_of(int k, int a, int b) { return b * (k % a) + k / a; }

// 3: Z = DFT_m(x_even + i x_odd)  ->  X = DFT_2m(x) for k in [0, m]
//    (X[m] goes to the extra column m), thread-private in place.
template <class T>
__host__ __device__ inline void ph3(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int M = c.it.m, am = c.it.am, bm = c.it.bm, ld = c.it.ld;
    const int H = M / 2 + 1;
    const int ntask = c.s_n0 * H;
    const T half = T(0.5);
    for (int t = tid; t < ntask; t += nth) {
        const int r = t % c.s_n0, k = t / c.s_n0;
        cx<T>* p = buf + (int64_t)(c.s_off0 + r) * ld;
        const int sk = slot_of(k, am, bm);
        const cx<T> Zk = p[sk];
        if (k == 0) {
            p[sk] = {Zk.x + Zk.y, T(0)};
            p[M] = {Zk.x - Zk.y, T(0)};
        } else {
            const int skm = slot_of(M - k, am, bm);
            const cx<T> Zm = p[skm];
            const cx<T> E = {(Zk.x + Zm.x) * half, (Zk.y - Zm.y) * half};
            const cx<T> O = {(Zk.y + Zm.y) * half, (Zm.x - Zk.x) * half};
            const cx<T> wO = cmul(c.tw2m[k], O);
            p[sk] = E + wO;
            if (2 * k != M) p[skm] = conj(E - wO);
        }
    }
}

// 4: column pass 1 (forward), columns 0..m
template <class T>
__host__ __device__ inline void ph4(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int a0 = c.it.a0, b0 = c.it.b0, ld = c.it.ld, NC = c.it.m + 1;
    const int ntask = NC * b0;
    for (int t = tid; t < ntask; t += nth) {
        const int col = t % NC, j0 = t / NC;
        cx<T> x[kMaxRadix];
#pragma unroll
        for (int j1 = 0; j1 < kMaxRadix; ++j1) {
            if (j1 < a0) {
                const int row = b0 * j1 + j0;
                x[j1] = ((unsigned)(row - c.s_off0) < (unsigned)c.s_n0) ? buf[(int64_t)row * ld + col]
                                                                        : cx<T>{T(0), T(0)};
            }
        }
        dft_rt<-1>(a0, x);
#pragma unroll
        for (int k1 = 0; k1 < kMaxRadix; ++k1)
            if (k1 < a0) buf[(int64_t)(b0 * k1 + j0) * ld + col] = cmul(x[k1], c.tw0[j0 * k1]);
    }
}

// 5: column pass 2, spectral product, inverse column pass 2
template <class T>
__host__ __device__ inline void ph5(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int a0 = c.it.a0, b0 = c.it.b0, ld = c.it.ld, NC = c.it.m + 1;
    const int ntask = NC * a0;
    for (int t = tid; t < ntask; t += nth) {
        const int col = t % NC, k1 = t / NC;
        cx<T>* p = buf + (int64_t)(b0 * k1) * ld + col;
        const cx<T>* sp = c.spec + (int64_t)(b0 * k1) * NC + col;
        cx<T> x[kMaxRadix];
#pragma unroll
        for (int k0 = 0; k0 < kMaxRadix; ++k0)
            if (k0 < b0) x[k0] = p[(int64_t)k0 * ld];
        dft_rt<-1>(b0, x);
#pragma unroll
        for (int k0 = 0; k0 < kMaxRadix; ++k0) {
            if (k0 < b0) {
                const cx<T> s = sp[(int64_t)k0 * NC];
                x[k0] = c.adj ? cmulc(x[k0], s) : cmul(x[k0], s);
            }
        }
        dft_rt<1>(b0, x);
#pragma unroll
        for (int k0 = 0; k0 < kMaxRadix; ++k0)
            if (k0 < b0) p[(int64_t)k0 * ld] = x[k0];
    }
}

// 6: inverse column pass 1; keeps the rows of the written box
template <class T>
__host__ __device__ inline void ph6(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int a0 = c.it.a0, b0 = c.it.b0, ld = c.it.ld, NC = c.it.m + 1;
    const int ntask = NC * b0;
    for (int t = tid; t < ntask; t += nth) {
        const int col = t % NC, j0 = t / NC;
        cx<T> x[kMaxRadix];
#pragma unroll
        for (int k1 = 0; k1 < kMaxRadix; ++k1)
            if (k1 < a0) x[k1] = cmulc(buf[(int64_t)(b0 * k1 + j0) * ld + col], c.tw0[j0 * k1]);
        dft_rt<1>(a0, x);
#pragma unroll
        for (int j1 = 0; j1 < kMaxRadix; ++j1) {
            if (j1 < a0) {
                const int row = b0 * j1 + j0;
                if ((unsigned)(row - c.d_off0) < (unsigned)c.d_n0) buf[(int64_t)row * ld + col] = x[j1];
            }
        }
    }
}

// 7: X (k in [0, m]) -> Z = DFT_m(y_even + i y_odd), thread-private in place
template <class T>
__host__ __device__ inline void ph7(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int M = c.it.m, am = c.it.am, bm = c.it.bm, ld = c.it.ld;
    const int H = M / 2 + 1;
    const int ntask = c.d_n0 * H;
    const T half = T(0.5);
    for (int t = tid; t < ntask; t += nth) {
        const int r = t % c.d_n0, k = t / c.d_n0;
        cx<T>* p = buf + (int64_t)(c.d_off0 + r) * ld;
        const int sk = slot_of(k, am, bm);
        const int skm = (k == 0) ? M : slot_of(M - k, am, bm);
        const cx<T> Xk = p[sk], Xm = p[skm];
        const cx<T> E = {(Xk.x + Xm.x) * half, (Xk.y - Xm.y) * half};
        const cx<T> D = {(Xk.x - Xm.x) * half, (Xk.y + Xm.y) * half};
        const cx<T> O = cmulc(D, c.tw2m[k]);
        p[sk] = {E.x - O.y, E.y + O.x};
        if (k != 0 && 2 * k != M) p[skm] = {E.x + O.y, O.x - E.y};
    }
}

// 9: inverse row pass 1 + write of the output box
template <class T>
__host__ __device__ inline void ph9(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int am = c.it.am, bm = c.it.bm, ld = c.it.ld;
    const int ntask = c.d_n0 * bm;
    for (int t = tid; t < ntask; t += nth) {
        const int j0 = t % bm, q = t / bm;
        const int row = c.d_off0 + q;
        const cx<T>* in = buf + (int64_t)row * ld + j0;
        cx<T> x[kMaxRadix];
#pragma unroll
        for (int k1 = 0; k1 < kMaxRadix; ++k1)
            if (k1 < am) x[k1] = cmulc(in[bm * k1], c.twm[j0 * k1]);
        dft_rt<1>(am, x);
        T* drow = c.dst + (int64_t)q * c.d_n1;
        const T* wrow = c.w + (int64_t)q * c.d_n1;
#pragma unroll
        for (int j1 = 0; j1 < kMaxRadix; ++j1) {
            if (j1 < am) {
                const int j = bm * j1 + j0;
                const int e0 = 2 * j - c.d_off1, e1 = e0 + 1;
                if ((unsigned)e0 < (unsigned)c.d_n1) drow[e0] = c.adj ? x[j1].x * wrow[e0] : x[j1].x;
                if ((unsigned)e1 < (unsigned)c.d_n1) drow[e1] = c.adj ? x[j1].y * wrow[e1] : x[j1].y;
            }
        }
    }
}

// Deterministic reduction of one output tile for one vector: contributors in
// ascending item order (ascending patch index k).
template <class T>
__host__ __device__ inline void reduce_tile(const Tile& t, int col_in_tile, const int32_t* contrib,
                                            const Box* boxes, const T* slots, T* out, int64_t pitch) {
    if (col_in_tile >= t.nc) return;
    const int col = t.c0 + col_in_tile;
    T acc[kReduceRows];
#pragma unroll
    for (int rr = 0; rr < kReduceRows; ++rr) acc[rr] = T(0);
    for (int ci = t.beg; ci < t.end; ++ci) {
        const Box b = boxes[contrib[ci]];
        const int cc = col - b.lo1;
        if ((unsigned)cc >= (unsigned)b.n1) continue;
        const T* s = slots + b.off + cc;
#pragma unroll
        for (int rr = 0; rr < kReduceRows; ++rr) {
            const int r2 = t.r0 + rr - b.lo0;
            if (rr < t.nr && (unsigned)r2 < (unsigned)b.n0) acc[rr] += s[(int64_t)r2 * b.n1];
        }
    }
#pragma unroll
    for (int rr = 0; rr < kReduceRows; ++rr)
        if (rr < t.nr) out[(int64_t)(t.r0 + rr) * pitch + col] = acc[rr];
}

}  // namespace pc
