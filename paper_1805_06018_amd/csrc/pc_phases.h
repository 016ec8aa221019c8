// The phases of one convolution work item (a patch or row piece of the
// product-convolution sum, eq. (2.5), or of its adjoint, eq. (1.6)).
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
//   A0 coalesced gather into LDS (weighted for the forward sum)
//   A  row pass 1 in place
//   B row pass 2 fused with the real-row post-processing: a task owns the
//     slot groups k1 and m-k1's group, which hold every pair Z[k], Z[m-k]
//   C column pass 1 (only the gathered rows are non-zero)
//   D column pass 2, product with the spectrum (conjugate for the adjoint),
//     inverse column pass 2
//   E inverse column pass 1 (only rows needed by the output are kept)
//   F real-row pre-processing fused with inverse row pass 2
//   G inverse row pass 1 in place (rows end in natural order)
//   H coalesced copy of the output box to staging (weighted for the adjoint)
//
// Every phase is templated on its radix (dispatched once per phase) and all
// functions are __host__ __device__: the GPU kernel runs them with a barrier
// in between; a host-only build runs them thread by thread.
#pragma once
#include "pc_fft.h"
#include "pc_internal.h"

namespace pc {

// a * b for operands below 2^23: one full-rate 24-bit multiply on the GPU
// (a 32-bit product is a quarter-rate instruction there).
__host__ __device__ __forceinline__ int imul24(int a, int b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __mul24(a, b);
#else
    return a * b;
#endif
}

// floor(x / d) for 0 <= x < 2^22 with inv = 1.0f / d (exact: the fraction
// (x + 1/2) / d stays at least 1/(2d) away from an integer).
__host__ __device__ inline int fdiv(int x, float inv) { return (int)(((float)x + 0.5f) * inv); }

// w[k1] = w_n^(j0 k1) for 1 <= k1 < A: the twiddles of pass-1 task j0,
// stored as one run per task (entry j0 (A - 1) + k1 - 1 of the table), so
// one multiply finds the run and the reads take immediate offsets; w[0] = 1
// is never read.  All of a task's twiddles are read before any of its
// results is written back to LDS: the compiler cannot tell the twiddle
// table from the box, so a read placed after a store would wait for it.
template <int A, class T>
__host__ __device__ __forceinline__ void twiddle_run(const cx<T>* tw, int j0, cx<T>* w) {
    const cx<T>* q = tw + imul24(j0, A - 1) - 1;
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) w[k1] = q[k1];
}

template <class T>
struct Ctx {
    Item it;
    bool adj;
    int s_off0, s_n0, s_off1, s_n1;   // gathered box (FFT coordinates)
    int d_off0, d_n0, d_off1, d_n1;   // written box
    float inv_bm, inv_b0, inv_nc, inv_sn0, inv_dn0;
    const T* src;                     // input vector, Omega origin
    T* dst;                           // written box: staging box of this item and vector, or
                                      // (add) the output vector at the box's Omega origin
    int64_t dst_rs;                   // row stride of dst (box width, or the Omega pitch)
    bool add;                         // add into the output instead of storing to staging
    const T* w;                       // weight table of the item's input box
    const cx<T>* spec;
    int spec_ld;                      // spectrum row stride (m + 1 for 2-D items)
    const cx<T>* tw0;                 // column pass-1 twiddles (runs per task, see twiddle_run)
    const cx<T>* twm;                 // row pass-1 twiddles (the same layout)
    const cx<T>* tw2m;                // w_2m^(k1 + am k0) at k1 bm + k0 (post-/pre-processing)
    int64_t pitch;                    // Omega row pitch (elements)
};

// out_vec: null to store the written box to the item's staging box in
// slot_vec; else the output vector (Omega origin) that the written box is
// added into, in place.
template <class T>
__host__ __device__ inline Ctx<T> make_ctx(const Item& it, bool adj, const T* in_vec, T* slot_vec,
                                           const T* wts, const cx<T>* spec, const cx<T>* tw, int64_t pitch,
                                           T* out_vec = nullptr) {
    Ctx<T> c;
    c.it = it;
    c.adj = adj;
    if (!adj) {
        c.s_off0 = it.in_off0; c.s_n0 = it.in_n0; c.s_off1 = it.in_off1; c.s_n1 = it.in_n1;
        c.d_off0 = it.out_off0; c.d_n0 = it.out_n0; c.d_off1 = it.out_off1; c.d_n1 = it.out_n1;
    } else {
        c.s_off0 = it.out_off0; c.s_n0 = it.out_n0; c.s_off1 = it.out_off1; c.s_n1 = it.out_n1;
        c.d_off0 = it.in_off0; c.d_n0 = it.in_n0; c.d_off1 = it.in_off1; c.d_n1 = it.in_n1;
    }
    c.add = out_vec != nullptr;
    if (c.add) {
        c.dst = out_vec + (int64_t)(it.g0 + c.d_off0) * pitch + it.g1 + c.d_off1;
        c.dst_rs = pitch;
    } else {
        c.dst = slot_vec + (adj ? it.slot_adj : it.slot_fwd);
        c.dst_rs = c.d_n1;
    }
    c.inv_bm = 1.0f / (float)it.bm;
    c.inv_b0 = 1.0f / (float)it.b0;
    c.inv_nc = 1.0f / (float)(it.m + 1);
    c.inv_sn0 = 1.0f / (float)c.s_n0;
    c.inv_dn0 = 1.0f / (float)c.d_n0;
    c.src = in_vec;
    c.w = wts + it.w_off;
    c.spec = spec + it.spec_off;
    c.spec_ld = it.m + 1;
    c.tw0 = tw + it.tw0;
    c.twm = tw + it.twm;
    c.tw2m = tw + it.tw2m;
    c.pitch = pitch;
    return c;
}

// The item's twiddle tables (column pass 1: b0 (a0 - 1), row pass 1:
// bm (am - 1), pairs: (am / 2 + 1) bm complex) are copied into LDS right
// after the FFT box, cooperatively and before the first barrier; the phases
// then read their twiddles from LDS.
__host__ __device__ inline int64_t tw_lds_elems(const Item& it) {
    return (int64_t)it.b0 * (it.a0 - 1) + (int64_t)it.bm * (it.am - 1) + (int64_t)(it.am / 2 + 1) * it.bm;
}

// With copy false the tables are already there (only the pointers are set).
template <class T>
__host__ __device__ inline void twiddles_to_lds(Ctx<T>& c, cx<T>* dst, int tid, int nth, bool copy = true) {
    const int l0 = c.it.b0 * (c.it.a0 - 1), lm = c.it.bm * (c.it.am - 1);
    const int n = copy ? (int)tw_lds_elems(c.it) : 0;
    for (int t = tid; t < n; t += nth) {
        cx<T> v;
        if (t < l0)
            v = c.tw0[t];
        else if (t < l0 + lm)
            v = c.twm[t - l0];
        else
            v = c.tw2m[t - l0 - lm];
        dst[t] = v;
    }
    c.tw0 = dst;
    c.twm = dst + l0;
    c.tw2m = dst + l0 + lm;
}

#define PC_RADIX_SWITCH(R, FN, ...)               \
    switch (R) {                                  \
        case 1: FN<1>(__VA_ARGS__); break;        \
        case 2: FN<2>(__VA_ARGS__); break;        \
        case 3: FN<3>(__VA_ARGS__); break;        \
        case 4: FN<4>(__VA_ARGS__); break;        \
        case 5: FN<5>(__VA_ARGS__); break;        \
        case 6: FN<6>(__VA_ARGS__); break;        \
        case 7: FN<7>(__VA_ARGS__); break;        \
        case 8: FN<8>(__VA_ARGS__); break;        \
        case 9: FN<9>(__VA_ARGS__); break;        \
        case 10: FN<10>(__VA_ARGS__); break;      \
        case 12: FN<12>(__VA_ARGS__); break;      \
        case 14: FN<14>(__VA_ARGS__); break;      \
        case 15: FN<15>(__VA_ARGS__); break;      \
        case 16: FN<16>(__VA_ARGS__); break;      \
        default: break;                           \
    }

// Row pass-2 radices: m <= 128 and the larger factor goes first, so bm <= 10.
#define PC_RADIX_SWITCH_ROW2(R, FN, ...)          \
    switch (R) {                                  \
        case 1: FN<1>(__VA_ARGS__); break;        \
        case 2: FN<2>(__VA_ARGS__); break;        \
        case 3: FN<3>(__VA_ARGS__); break;        \
        case 4: FN<4>(__VA_ARGS__); break;        \
        case 5: FN<5>(__VA_ARGS__); break;        \
        case 6: FN<6>(__VA_ARGS__); break;        \
        case 7: FN<7>(__VA_ARGS__); break;        \
        case 8: FN<8>(__VA_ARGS__); break;        \
        case 9: FN<9>(__VA_ARGS__); break;        \
        case 10: FN<10>(__VA_ARGS__); break;      \
        default: break;                           \
    }
constexpr int kMaxRowPass2Radix = 10;

// ---------------------------------------------------------------- phase A
// A0: coalesced copy of the gathered box into LDS, weighted for the forward
// sum: each gathered row holds the real samples 0..2m-1 (zero outside the
// box) as m complex (even, odd) pairs.  A fixed set of threads owns each
// column, so consecutive lanes read consecutive input columns.
// U: rows whose loads are in flight together (registers allowing: 8 in the
// 1024-thread kernel, 16 in the 256-thread plane kernels).
template <int U = 8, class T>
__host__ __device__ inline void phA0(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int n = 2 * c.it.m;            // real samples per row
    const int rps = nth / n;             // rows per sweep (n <= 256 <= nth)
    const int r0 = tid / n, col = tid - r0 * n;
    if (r0 >= rps) return;
    const int e = col - c.s_off1;        // column inside the gathered box
    const bool live = (unsigned)e < (unsigned)c.s_n1;
    const bool wgt = live && !c.adj;
    const int rstride = 2 * c.it.ld, rstep = rps * rstride;
    T* rows = reinterpret_cast<T*>(buf) + (c.s_off0 + r0) * rstride + col;
    // Global addresses: a workgroup-uniform base plus a 32-bit byte offset
    // per lane, which the loads take as scalar base + vector offset (the
    // rows of a box are fewer than 256 and pc_create limits every extent of
    // Omega to 2^20, so the offsets stay below 2^31); a batch's rows are a
    // uniform stride apart.
    const char* sbase = reinterpret_cast<const char*>(c.src + (int64_t)(c.it.g0 + c.s_off0) * c.pitch + c.it.g1);
    const char* wbase = reinterpret_cast<const char*>(c.w);
    uint32_t soff = (uint32_t)(r0 * c.pitch + col) * (uint32_t)sizeof(T);
    uint32_t woff = (uint32_t)(r0 * c.it.w_ld + e) * (uint32_t)sizeof(T);
    const uint32_t sstep = (uint32_t)(rps * c.pitch) * (uint32_t)sizeof(T);
    const uint32_t wstep = (uint32_t)(rps * c.it.w_ld) * (uint32_t)sizeof(T);
    // predicated batches: every row of a batch is loaded before any is used
    for (int q = r0; q < c.s_n0; q += U * rps) {
        T v[U], f[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = (live && q + u * rps < c.s_n0) ? *reinterpret_cast<const T*>(sbase + (soff + u * sstep)) : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            f[u] = (wgt && q + u * rps < c.s_n0) ? *reinterpret_cast<const T*>(wbase + (woff + u * wstep)) : T(1);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (q + u * rps < c.s_n0) rows[u * rstep] = v[u] * f[u];
        soff += U * sstep;
        woff += U * wstep;
        rows += U * rstep;
    }
}

// A1: row pass 1 in place on the gathered rows: the thread that reads slots
// bm j1 + j0 writes the twiddled DFT_am outputs back to slots bm k1 + j0.
template <int A, class T>
__host__ __device__ inline void phA_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int bm = c.it.bm, ld = c.it.ld;
    const int ntask = c.s_n0 * bm;
    for (int t = tid; t < ntask; t += nth) {
        const int q = fdiv(t, c.inv_bm), j0 = t - imul24(q, bm);
        cx<T>* p = buf + (imul24(c.s_off0 + q, ld) + j0);
        cx<T> x[A], w[A];
#pragma unroll
        for (int j1 = 0; j1 < A; ++j1) x[j1] = p[bm * j1];
        twiddle_run<A>(c.twm, j0, w);
        Dft<A, -1>::run(x);
        p[0] = x[0];   // twiddle w^0 = 1
#pragma unroll
        for (int k1 = 1; k1 < A; ++k1) p[bm * k1] = cmul(x[k1], w[k1]);
    }
}
template <class T>
__host__ __device__ inline void phA(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH(c.it.am, phA_r, c, buf, tid, nth);
}

// Real-row post-processing of one frequency pair: from Z[k], Z[m-k] of
// Z = DFT_m(x_even + i x_odd) to 2 X[k] and 2 X[m-k] of X = DFT_2m(x).
// The factor 1/2 of the even/odd split is left out here and in pre_pair
// (so every row spectrum is 2 X and every pre-processed row 2 Z); the
// spectra carry the product 1/4 instead.  Scaling by powers of two is
// exact, so the results are bit for bit those of the halved formulas.
template <class T>
__host__ __device__ inline void post_pair(cx<T> Zk, cx<T> Zm, cx<T> w, cx<T>& Xk, cx<T>& Xm) {
    const cx<T> E = {Zk.x + Zm.x, Zk.y - Zm.y};
    const cx<T> O = {Zk.y + Zm.y, Zm.x - Zk.x};
    const cx<T> wO = cmul(w, O);
    Xk = E + wO;
    Xm = conj(E - wO);
}
// Inverse: from X[k], X[m-k] back to 2 Z[k], 2 Z[m-k].
template <class T>
__host__ __device__ inline void pre_pair(cx<T> Xk, cx<T> Xm, cx<T> w, cx<T>& Zk, cx<T>& Zm) {
    const cx<T> E = {Xk.x + Xm.x, Xk.y - Xm.y};
    const cx<T> D = {Xk.x - Xm.x, Xk.y + Xm.y};
    const cx<T> O = cmulc(D, w);
    Zk = {E.x - O.y, E.y + O.x};
    Zm = {E.x + O.y, O.x - E.y};
}

// ---------------------------------------------------------------- phase B
// Task (row, k1) with k1 in [0, am/2]: groups k1 and k1b = (am - k1) mod am.
// Frequencies k = k1 + am k0 and m - k = k1b + am (bm - 1 - k0) for k1 > 0;
// for k1 = 0 the partner of am k0 is am (bm - k0); slot(k) = bm k1 + k0 and
// X[m] goes to the extra column m.
template <int Bm, class T>
__host__ __device__ inline void phB_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int am = c.it.am, ld = c.it.ld, M = c.it.m;
    const int H = am / 2 + 1;
    const int ntask = c.s_n0 * H;
    for (int t = tid; t < ntask; t += nth) {
        const int k1 = fdiv(t, c.inv_sn0), r = t - imul24(k1, c.s_n0);
        cx<T>* p = buf + imul24(c.s_off0 + r, ld);
        const int k1b = (k1 == 0) ? 0 : am - k1;
        cx<T>* pa = p + imul24(Bm, k1);
        cx<T>* pb = p + imul24(Bm, k1b);
        cx<T> za[Bm], zb[Bm], w[Bm];
#pragma unroll
        for (int k0 = 0; k0 < Bm; ++k0) za[k0] = pa[k0];
        if (k1b != k1) {
#pragma unroll
            for (int k0 = 0; k0 < Bm; ++k0) zb[k0] = pb[k0];
        }
        // w[k0] = w_2m^(k1 + am k0): the twiddles of every branch below
        const cx<T>* tq = c.tw2m + imul24(k1, Bm);
#pragma unroll
        for (int k0 = 0; k0 < Bm; ++k0) w[k0] = tq[k0];
        Dft<Bm, -1>::run(za);
        if (k1b != k1) {
            Dft<Bm, -1>::run(zb);
#pragma unroll
            for (int k0 = 0; k0 < Bm; ++k0) {
                cx<T> Xk, Xm;
                post_pair(za[k0], zb[Bm - 1 - k0], w[k0], Xk, Xm);
                za[k0] = Xk;
                zb[Bm - 1 - k0] = Xm;
            }
#pragma unroll
            for (int k0 = 0; k0 < Bm; ++k0) pb[k0] = zb[k0];
        } else if (k1 == 0) {
            // k = am k0 pairs with am (bm - k0); k0 = 0 gives X[0] and X[m]
            const cx<T> z0 = za[0];
#pragma unroll
            for (int k0 = 1; 2 * k0 <= Bm; ++k0) {
                cx<T> Xk, Xm;
                post_pair(za[k0], za[Bm - k0], w[k0], Xk, Xm);
                za[k0] = Xk;
                if (2 * k0 != Bm) za[Bm - k0] = Xm;
            }
            za[0] = {(z0.x + z0.y) * T(2), T(0)};   // 2 X[0] and 2 X[m], as post_pair
            p[M] = {(z0.x - z0.y) * T(2), T(0)};
        } else {
            // am even, k1 = am/2: k0 pairs with bm - 1 - k0
#pragma unroll
            for (int k0 = 0; 2 * k0 < Bm; ++k0) {
                cx<T> Xk, Xm;
                post_pair(za[k0], za[Bm - 1 - k0], w[k0], Xk, Xm);
                za[k0] = Xk;
                if (2 * k0 != Bm - 1) za[Bm - 1 - k0] = Xm;
            }
        }
#pragma unroll
        for (int k0 = 0; k0 < Bm; ++k0) pa[k0] = za[k0];
    }
}
template <class T>
__host__ __device__ inline void phB(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH_ROW2(c.it.bm, phB_r, c, buf, tid, nth);
}

// ---------------------------------------------------------------- phase C
template <int A0, class T>
__host__ __device__ inline void phC_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int b0 = c.it.b0, ld = c.it.ld, NC = c.it.m + 1;
    const int ntask = NC * b0;
    for (int t = tid; t < ntask; t += nth) {
        const int j0 = fdiv(t, c.inv_nc), col = t - imul24(j0, NC);
        cx<T>* p = buf + (imul24(j0, ld) + col);
        const int step = b0 * ld;
        cx<T> x[A0], w[A0];
#pragma unroll
        for (int j1 = 0; j1 < A0; ++j1) {
            const int row = b0 * j1 + j0;
            x[j1] = ((unsigned)(row - c.s_off0) < (unsigned)c.s_n0) ? p[j1 * step] : cx<T>{T(0), T(0)};
        }
        twiddle_run<A0>(c.tw0, j0, w);
        Dft<A0, -1>::run(x);
        p[0] = x[0];
#pragma unroll
        for (int k1 = 1; k1 < A0; ++k1) p[k1 * step] = cmul(x[k1], w[k1]);
    }
}
template <class T>
__host__ __device__ inline void phC(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH(c.it.a0, phC_r, c, buf, tid, nth);
}

// ---------------------------------------------------------------- phase D
// MODE 0: column pass 2, product with the spectrum, inverse column pass 2;
// MODE 1: column pass 2 only (forward 2-D FFT of a plane);
// MODE 2: inverse column pass 2 only (inverse 2-D FFT of a plane).
template <int MODE, int B0, class T>
__host__ __device__ inline void phD_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int a0 = c.it.a0, ld = c.it.ld, NC = c.it.m + 1;
    const int ntask = NC * a0;
    for (int t = tid; t < ntask; t += nth) {
        const int k1 = fdiv(t, c.inv_nc), col = t - imul24(k1, NC);
        cx<T>* p = buf + (imul24(k1, B0 * ld) + col);
        cx<T> x[B0];
        if (MODE == 0) {
            // spectrum: a uniform base plus a 32-bit byte offset per lane
            // (a scalar-base load); rows k0 a uniform stride apart
            const uint32_t sstride = (uint32_t)c.spec_ld * (uint32_t)sizeof(cx<T>);
            const uint32_t so = (uint32_t)(imul24(k1, B0 * c.spec_ld) + col) * (uint32_t)sizeof(cx<T>);
            const char* sb = reinterpret_cast<const char*>(c.spec);
            cx<T> s[B0];
#pragma unroll
            for (int k0 = 0; k0 < B0; ++k0) s[k0] = *reinterpret_cast<const cx<T>*>(sb + (so + k0 * sstride));
#pragma unroll
            for (int k0 = 0; k0 < B0; ++k0) x[k0] = p[k0 * ld];
            Dft<B0, -1>::run(x);
            if (c.adj) {
#pragma unroll
                for (int k0 = 0; k0 < B0; ++k0) x[k0] = cmulc(x[k0], s[k0]);
            } else {
#pragma unroll
                for (int k0 = 0; k0 < B0; ++k0) x[k0] = cmul(x[k0], s[k0]);
            }
            Dft<B0, 1>::run(x);
        } else {
#pragma unroll
            for (int k0 = 0; k0 < B0; ++k0) x[k0] = p[k0 * ld];
            if (MODE == 1)
                Dft<B0, -1>::run(x);
            else
                Dft<B0, 1>::run(x);
        }
#pragma unroll
        for (int k0 = 0; k0 < B0; ++k0) p[k0 * ld] = x[k0];
    }
}
template <int B0, class T>
__host__ __device__ inline void phD0_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) { phD_r<0, B0>(c, buf, tid, nth); }
template <int B0, class T>
__host__ __device__ inline void phD1_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) { phD_r<1, B0>(c, buf, tid, nth); }
template <int B0, class T>
__host__ __device__ inline void phD2_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) { phD_r<2, B0>(c, buf, tid, nth); }
template <class T>
__host__ __device__ inline void phD(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH(c.it.b0, phD0_r, c, buf, tid, nth);
}
template <class T>
__host__ __device__ inline void phD_fwd(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH(c.it.b0, phD1_r, c, buf, tid, nth);
}
template <class T>
__host__ __device__ inline void phD_inv(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH(c.it.b0, phD2_r, c, buf, tid, nth);
}

// ---------------------------------------------------------------- phase E
template <int A0, class T>
__host__ __device__ inline void phE_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int b0 = c.it.b0, ld = c.it.ld, NC = c.it.m + 1;
    const int ntask = NC * b0;
    for (int t = tid; t < ntask; t += nth) {
        const int j0 = fdiv(t, c.inv_nc), col = t - imul24(j0, NC);
        cx<T>* p = buf + (imul24(j0, ld) + col);
        const int step = b0 * ld;
        cx<T> x[A0], w[A0];
#pragma unroll
        for (int k1 = 0; k1 < A0; ++k1) x[k1] = p[k1 * step];
        twiddle_run<A0>(c.tw0, j0, w);
#pragma unroll
        for (int k1 = 1; k1 < A0; ++k1) x[k1] = cmulc(x[k1], w[k1]);
        Dft<A0, 1>::run(x);
#pragma unroll
        for (int j1 = 0; j1 < A0; ++j1) {
            const int row = b0 * j1 + j0;
            if ((unsigned)(row - c.d_off0) < (unsigned)c.d_n0) p[j1 * step] = x[j1];
        }
    }
}
template <class T>
__host__ __device__ inline void phE(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH(c.it.a0, phE_r, c, buf, tid, nth);
}

// ---------------------------------------------------------------- phase F
// Mirror of phase B on the written rows: pre-processing of the frequency
// pairs, then the inverse DFT_bm of groups k1 and k1b.
template <int Bm, class T>
__host__ __device__ inline void phF_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int am = c.it.am, ld = c.it.ld, M = c.it.m;
    const int H = am / 2 + 1;
    const int ntask = c.d_n0 * H;
    for (int t = tid; t < ntask; t += nth) {
        const int k1 = fdiv(t, c.inv_dn0), r = t - imul24(k1, c.d_n0);
        cx<T>* p = buf + imul24(c.d_off0 + r, ld);
        const int k1b = (k1 == 0) ? 0 : am - k1;
        cx<T>* pa = p + imul24(Bm, k1);
        cx<T>* pb = p + imul24(Bm, k1b);
        cx<T> za[Bm], zb[Bm], w[Bm];
#pragma unroll
        for (int k0 = 0; k0 < Bm; ++k0) za[k0] = pa[k0];
        if (k1b != k1) {
#pragma unroll
            for (int k0 = 0; k0 < Bm; ++k0) zb[k0] = pb[k0];
        }
        // w[k0] = w_2m^(k1 + am k0): the twiddles of every branch below
        const cx<T>* tq = c.tw2m + imul24(k1, Bm);
#pragma unroll
        for (int k0 = 0; k0 < Bm; ++k0) w[k0] = tq[k0];
        if (k1b != k1) {
#pragma unroll
            for (int k0 = 0; k0 < Bm; ++k0) {
                cx<T> Zk, Zm;
                pre_pair(za[k0], zb[Bm - 1 - k0], w[k0], Zk, Zm);
                za[k0] = Zk;
                zb[Bm - 1 - k0] = Zm;
            }
            Dft<Bm, 1>::run(zb);
#pragma unroll
            for (int k0 = 0; k0 < Bm; ++k0) pb[k0] = zb[k0];
        } else if (k1 == 0) {
            const cx<T> X0 = za[0], XM = p[M];
#pragma unroll
            for (int k0 = 1; 2 * k0 <= Bm; ++k0) {
                cx<T> Zk, Zm;
                pre_pair(za[k0], za[Bm - k0], w[k0], Zk, Zm);
                za[k0] = Zk;
                if (2 * k0 != Bm) za[Bm - k0] = Zm;
            }
            cx<T> Z0, Zunused;
            pre_pair(X0, XM, cx<T>{T(1), T(0)}, Z0, Zunused);
            za[0] = Z0;
        } else {
#pragma unroll
            for (int k0 = 0; 2 * k0 < Bm; ++k0) {
                cx<T> Zk, Zm;
                pre_pair(za[k0], za[Bm - 1 - k0], w[k0], Zk, Zm);
                za[k0] = Zk;
                if (2 * k0 != Bm - 1) za[Bm - 1 - k0] = Zm;
            }
        }
        Dft<Bm, 1>::run(za);
#pragma unroll
        for (int k0 = 0; k0 < Bm; ++k0) pa[k0] = za[k0];
    }
}
template <class T>
__host__ __device__ inline void phF(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH_ROW2(c.it.bm, phF_r, c, buf, tid, nth);
}

// ---------------------------------------------------------------- phase G
// Inverse row pass 1, in place: the thread that reads slots bm k1 + j0 writes
// z[bm j1 + j0] back to the same slots, so each LDS row ends in natural order
// and, read as reals, is the real output row.
template <int A, class T>
__host__ __device__ inline void phG_r(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    const int bm = c.it.bm, ld = c.it.ld;
    const int ntask = c.d_n0 * bm;
    for (int t = tid; t < ntask; t += nth) {
        const int q = fdiv(t, c.inv_bm), j0 = t - imul24(q, bm);
        cx<T>* p = buf + (imul24(c.d_off0 + q, ld) + j0);
        cx<T> x[A], w[A];
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) x[k1] = p[bm * k1];
        twiddle_run<A>(c.twm, j0, w);
#pragma unroll
        for (int k1 = 1; k1 < A; ++k1) x[k1] = cmulc(x[k1], w[k1]);
        Dft<A, 1>::run(x);
#pragma unroll
        for (int j1 = 0; j1 < A; ++j1) p[bm * j1] = x[j1];
    }
}
template <class T>
__host__ __device__ inline void phG(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
    PC_RADIX_SWITCH(c.it.am, phG_r, c, buf, tid, nth);
}

// *p += v as one device atomic whose result is not used (the add is done
// where the line lives, nothing returns to the wave, so no load latency is
// exposed at the end of the workgroup).  Only the workgroups of one colour
// launch touch a given element, and only once, so the atomic never races;
// it rounds like a plain add (round to nearest even).
template <class T>
__host__ __device__ __forceinline__ void add_to(T* p, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
    unsafeAtomicAdd(p, v);
#else
    *p = *p + v;
#endif
}

// ---------------------------------------------------------------- phase H
// The written box leaves LDS (weighted for the adjoint), either to the
// item's staging box or, when the launch holds items of one colour (their
// written boxes are disjoint), added straight into the output vector.  A
// fixed set of threads owns each column of the box, so consecutive lanes
// touch consecutive elements and no index is divided per element.
// Staging stores are non-temporal: staging is read once, by the reduction
// after the launch, and streaming it past the L2 keeps the spectra and
// inputs that the item's other vectors reuse (measured on the 1024^2
// workload: 5.17 -> 5.03 ms per apply, mostly in the reduction).
// The weighted value is rounded before it is added (no fused multiply-add),
// as the staged value is before the reduction adds it, so both ways give
// the same bits.
// OUT: kOutStage (staged kernel: stores only), kOutAdd (colour launches:
// adds only) or kOutEither (the CPU emulation: c.add decides).
enum { kOutStage = 0, kOutAdd = 1, kOutEither = 2 };
template <int U = 4, int OUT = kOutEither, class T>
__host__ __device__ inline void phH(const Ctx<T>& c, cx<T>* buf, int tid, int nth) {
#pragma clang fp contract(off)
    const int n1 = c.d_n1;
    const int rps = nth / n1;            // rows per sweep (n1 <= 256 <= nth)
    const int r0 = tid / n1, e = tid - r0 * n1;
    if (r0 >= rps) return;
    // the thread's first row; consecutive rows of a batch are a uniform
    // stride apart, so every address is one add from these pointers
    const int rstride = 2 * c.it.ld, rstep = rps * rstride;
    const T* rows = reinterpret_cast<const T*>(buf) + (c.d_off0 + r0) * rstride + c.d_off1 + e;
    // global addresses: uniform bases plus 32-bit byte offsets per lane, as
    // in the gather (the staging box or the output rows of the box)
    char* dbase = reinterpret_cast<char*>(c.dst);
    const char* wbase = reinterpret_cast<const char*>(c.w);
    uint32_t doff = (uint32_t)(r0 * c.dst_rs + e) * (uint32_t)sizeof(T);
    uint32_t woff = (uint32_t)(r0 * c.it.w_ld + e) * (uint32_t)sizeof(T);
    const uint32_t dstep = (uint32_t)(rps * c.dst_rs) * (uint32_t)sizeof(T);
    const uint32_t wstep = (uint32_t)(rps * c.it.w_ld) * (uint32_t)sizeof(T);
    if (OUT == kOutAdd || (OUT == kOutEither && c.add)) {
        // one atomic add per element; nothing returns, so no batching
        for (int r = r0; r < c.d_n0; r += rps) {
            const T p = rows[0] * (c.adj ? *reinterpret_cast<const T*>(wbase + woff) : T(1));
            add_to(reinterpret_cast<T*>(dbase + doff), p);
            rows += rstep;
            woff += wstep;
            doff += dstep;
        }
        return;
    }
    // predicated batches of U rows: LDS reads (and adjoint weights) first
    for (int q = r0; q < c.d_n0; q += U * rps) {
        T v[U], f[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = q + u * rps < c.d_n0 ? rows[u * rstep] : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            f[u] = (c.adj && q + u * rps < c.d_n0) ? *reinterpret_cast<const T*>(wbase + (woff + u * wstep)) : T(1);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (q + u * rps < c.d_n0)
                __builtin_nontemporal_store(v[u] * f[u], reinterpret_cast<T*>(dbase + (doff + u * dstep)));
        rows += U * rstep;
        woff += U * wstep;
        doff += U * dstep;
    }
}

// Deterministic reduction of one output tile for one vector: contributors in
// ascending item order (ascending patch index k).  cboxes[ci] is the staging
// box of the tile's ci-th contributor.  Contributors are taken four at a time:
// their loads are issued together and then added in ascending order, so the
// sum order is the same as one at a time.  With accumulate, out += alpha * sum.
template <class T>
__host__ __device__ inline void reduce_tile(const Tile& t, int col_in_tile, const Box* cboxes, const T* slots,
                                            T* out, int64_t pitch, bool accumulate = false, T alpha = T(1)) {
    if (col_in_tile >= t.nc) return;
    const int col = t.c0 + col_in_tile;
    constexpr int U = 4;
    T acc[kReduceRows];
#pragma unroll
    for (int rr = 0; rr < kReduceRows; ++rr) acc[rr] = T(0);
    for (int c0 = t.beg; c0 < t.end; c0 += U) {
        T x[U][kReduceRows];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ci = c0 + u;
            Box b;
            if (ci < t.end) {
                b = cboxes[ci];
            } else {
                b.lo0 = b.lo1 = 0;
                b.n0 = b.n1 = 0;
                b.off = 0;
            }
            const int cc = col - b.lo1;
            const bool colok = (unsigned)cc < (unsigned)b.n1;
            const T* s = slots + b.off + cc;
            const int r_lo = t.r0 - b.lo0;
#pragma unroll
            for (int rr = 0; rr < kReduceRows; ++rr) {
                const int r2 = r_lo + rr;
                x[u][rr] = (colok && (unsigned)r2 < (unsigned)b.n0) ? s[(int64_t)r2 * b.n1] : T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int rr = 0; rr < kReduceRows; ++rr) acc[rr] += x[u][rr];
    }
#pragma unroll
    for (int rr = 0; rr < kReduceRows; ++rr)
        if (rr < t.nr) {
            T* o = out + (int64_t)(t.r0 + rr) * pitch + col;
            *o = accumulate ? *o + alpha * acc[rr] : acc[rr];
        }
}

}  // namespace pc
