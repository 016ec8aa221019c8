// HIP kernels of the product-convolution apply for gfx950.
#include "pc_kernels.h"
#include "pc_phases.h"

namespace pc {

template <class T>
struct ConvArgs {
    const Item* items;
    int item_lo, n_items;   // items [item_lo, item_lo + n_items)
    int B;
    int adj;
    const cx<T>* spec;
    const T* wts;
    const cx<T>* tw;
    const T* in;
    int64_t ld_in;
    T* slots;
    int64_t slot_stride;
    int64_t pitch;
};

// One workgroup per (item, vector).  Blocks are dealt round-robin to the 8
// XCDs (block id mod 8); the mapping below gives every XCD whole items with
// all their vectors in sequence, so a patch's spectrum is fetched into one
// XCD's L2 and reused there by every vector.
template <class T>
__global__ __launch_bounds__(threads_for<T>()) void conv_kernel(ConvArgs<T> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    constexpr int NT = threads_for<T>();
    const int bid = blockIdx.x;
    const int xcd = bid & 7, l = bid >> 3;
    const int item = xcd + 8 * (l / A.B);
    const int rhs = l % A.B;
    if (item >= A.n_items) return;
    const Item it = A.items[A.item_lo + item];
    const Ctx<T> c = make_ctx<T>(it, A.adj != 0, A.in + (int64_t)rhs * A.ld_in, A.slots + (int64_t)rhs * A.slot_stride,
                                 A.wts, A.spec, A.tw, A.pitch);
    const int tid = threadIdx.x;
    phA(c, buf, tid, NT);
    __syncthreads();
    phB(c, buf, tid, NT);
    __syncthreads();
    phC(c, buf, tid, NT);
    __syncthreads();
    phD(c, buf, tid, NT);
    __syncthreads();
    phE(c, buf, tid, NT);
    __syncthreads();
    phF(c, buf, tid, NT);
    __syncthreads();
    phG(c, buf, tid, NT);
    __syncthreads();
    phH(c, buf, tid, NT);
}

template <class T>
__global__ __launch_bounds__(kReduceCols) void reduce_kernel(const Tile* tiles, const Box* cboxes, const T* slots,
                                                             int64_t slot_stride, T* out, int64_t ldo, int64_t pitch) {
    const Tile t = tiles[blockIdx.x];
    const int rhs = blockIdx.y;
    reduce_tile<T>(t, threadIdx.x, cboxes, slots + (int64_t)rhs * slot_stride, out + (int64_t)rhs * ldo, pitch);
}

// ---------------------------------------------------------------- estimator
constexpr int kEstThreads = 256;

__device__ inline double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = kEstThreads / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// One block per leaf: sum over probes i and leaf points x of (Yt - Y)^2, in
// FP64, in a fixed order (thread-strided loop, then a fixed tree).
template <class T>
__global__ __launch_bounds__(kEstThreads) void est_leaf_kernel(const int32_t* leaf_box, int q, const T* Yt, int64_t ldt,
                                                               const T* Y, int64_t ldy, int64_t pitch, double* leaf_sq) {
    __shared__ double sh[kEstThreads];
    const int c = blockIdx.x;
    const int lo0 = leaf_box[4 * c], lo1 = leaf_box[4 * c + 1], n0 = leaf_box[4 * c + 2], n1 = leaf_box[4 * c + 3];
    const int64_t cnt = (int64_t)n0 * n1;
    double acc = 0.0;
    for (int i = 0; i < q; ++i) {
        const T* a = Yt + (int64_t)i * ldt;
        const T* b = Y + (int64_t)i * ldy;
        for (int64_t e = threadIdx.x; e < cnt; e += kEstThreads) {
            const int64_t idx = (int64_t)(lo0 + e / n1) * pitch + lo1 + e % n1;
            const double dv = (double)a[idx] - (double)b[idx];
            acc += dv * dv;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) leaf_sq[c] = s;
}

// Row blocks of Omega: partial sums of (Yt - Y)^2 and Y^2 (each point once).
template <class T>
__global__ __launch_bounds__(kEstThreads) void est_total_kernel(int q, const T* Yt, int64_t ldt, const T* Y, int64_t ldy,
                                                                int64_t n_total, int n_part, double* partials) {
    __shared__ double sh[kEstThreads];
    const int64_t chunk = (n_total + n_part - 1) / n_part;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n_total ? beg + chunk : n_total;
    double dd = 0.0, yy = 0.0;
    for (int i = 0; i < q; ++i) {
        const T* a = Yt + (int64_t)i * ldt;
        const T* b = Y + (int64_t)i * ldy;
        for (int64_t e = beg + threadIdx.x; e < end; e += kEstThreads) {
            const double bv = (double)b[e];
            const double dv = (double)a[e] - bv;
            dd += dv * dv;
            yy += bv * bv;
        }
    }
    const double s0 = block_sum(dd, sh);
    const double s1 = block_sum(yy, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s0;
        partials[2 * blockIdx.x + 1] = s1;
    }
}

// ---------------------------------------------------------------- launchers
template <class T>
static hipError_t conv_t(const DevPlan& P, bool adj, int item_lo, int item_hi, int B, const void* in, int64_t ld_in,
                         void* slots, int64_t slot_stride, hipStream_t s) {
    ConvArgs<T> A;
    A.items = P.items;
    A.item_lo = item_lo;
    A.n_items = item_hi - item_lo;
    A.B = B;
    A.adj = adj ? 1 : 0;
    A.spec = static_cast<const cx<T>*>(P.spec);
    A.wts = static_cast<const T*>(P.wts);
    A.tw = static_cast<const cx<T>*>(P.tw);
    A.in = static_cast<const T*>(in);
    A.ld_in = ld_in;
    A.slots = static_cast<T*>(slots);
    A.slot_stride = slot_stride;
    A.pitch = P.cols;
    if (A.n_items <= 0 || B <= 0) return hipSuccess;
    const int64_t per_xcd = (int64_t)((A.n_items + 7) / 8) * B;
    const int64_t nblk = 8 * per_xcd;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(conv_kernel<T>, dim3((unsigned)nblk), dim3(threads_for<T>()), P.max_lds, s, A);
    return hipGetLastError();
}

hipError_t launch_conv(const DevPlan& P, bool adjoint, int item_lo, int item_hi, int B, const void* in, int64_t ld_in,
                       void* slots, int64_t slot_stride, hipStream_t s) {
    if (P.dtype == 1) return conv_t<double>(P, adjoint, item_lo, item_hi, B, in, ld_in, slots, slot_stride, s);
    return conv_t<float>(P, adjoint, item_lo, item_hi, B, in, ld_in, slots, slot_stride, s);
}

hipError_t launch_reduce(const DevPlan& P, bool adjoint, int B, const void* slots, int64_t slot_stride, void* out,
                         int64_t ldo, hipStream_t s) {
    const int nt = adjoint ? P.n_tiles_adj : P.n_tiles_fwd;
    if (nt <= 0 || B <= 0) return hipSuccess;
    const Tile* tiles = adjoint ? P.tiles_adj : P.tiles_fwd;
    const Box* cboxes = adjoint ? P.cboxes_adj : P.cboxes_fwd;
    dim3 grid((unsigned)nt, (unsigned)B);
    if (P.dtype == 1)
        hipLaunchKernelGGL(reduce_kernel<double>, grid, dim3(kReduceCols), 0, s, tiles, cboxes,
                           static_cast<const double*>(slots), slot_stride, static_cast<double*>(out), ldo,
                           (int64_t)P.cols);
    else
        hipLaunchKernelGGL(reduce_kernel<float>, grid, dim3(kReduceCols), 0, s, tiles, cboxes,
                           static_cast<const float*>(slots), slot_stride, static_cast<float*>(out), ldo,
                           (int64_t)P.cols);
    return hipGetLastError();
}

hipError_t launch_est(int dtype, const int32_t* leaf_box, int n_leaves, int q, const void* Yt, int64_t ldt,
                      const void* Y, int64_t ldy, int rows, int cols, double* leaf_sq, double* partials, int n_part,
                      hipStream_t s) {
    const int64_t n_total = (int64_t)rows * cols;
    if (dtype == 1) {
        hipLaunchKernelGGL(est_leaf_kernel<double>, dim3(n_leaves), dim3(kEstThreads), 0, s, leaf_box, q,
                           static_cast<const double*>(Yt), ldt, static_cast<const double*>(Y), ldy, (int64_t)cols,
                           leaf_sq);
        hipLaunchKernelGGL(est_total_kernel<double>, dim3(n_part), dim3(kEstThreads), 0, s, q,
                           static_cast<const double*>(Yt), ldt, static_cast<const double*>(Y), ldy, n_total, n_part,
                           partials);
    } else {
        hipLaunchKernelGGL(est_leaf_kernel<float>, dim3(n_leaves), dim3(kEstThreads), 0, s, leaf_box, q,
                           static_cast<const float*>(Yt), ldt, static_cast<const float*>(Y), ldy, (int64_t)cols,
                           leaf_sq);
        hipLaunchKernelGGL(est_total_kernel<float>, dim3(n_part), dim3(kEstThreads), 0, s, q,
                           static_cast<const float*>(Yt), ldt, static_cast<const float*>(Y), ldy, n_total, n_part,
                           partials);
    }
    return hipGetLastError();
}

hipError_t set_kernel_attributes() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&conv_kernel<float>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&conv_kernel<double>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
}

}  // namespace pc
