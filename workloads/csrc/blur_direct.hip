// Exact spatially varying Gaussian blur on the GPU (the black-box operator A
// whose impulse responses feed the product-convolution approximation; it is
// not part of the approximation itself).
//
// A[y, x] = exp(-sum_i (y_i - x_i)^2 / (2 s_i(x)^2)) / Z(x) for |y_i - x_i| <=
// R_i(x) = ceil(4 s_i(x)), Z(x) the sum of the same Gaussian over the full box.
// blur_adjoint computes (A^T v)[x] = sum_z g_x(z) v[x + z] over x + z in Omega
// for B vectors (the exact adjoint the error estimator needs).  2-D domains
// (d = 1 is a single row).  Widths and radii come from the host so that the
// radii match the supplied impulse responses exactly.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kVec = 8;   // vectors per pass over the taps

template <class T>
__device__ inline T gauss_norm(T s, int R) {
    T z = T(0);
    for (int t = -R; t <= R; ++t) z += exp(-(T)(t * t) / (2 * s * s));
    return z;
}

template <class T>
__global__ __launch_bounds__(kThreads) void blur_adjoint_kernel(const T* s0, const T* s1, const int32_t* r0,
                                                                const int32_t* r1, int n0, int n1, const T* in,
                                                                int64_t ldin, T* out, int64_t ldout, int B) {
    const int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (x >= (int64_t)n0 * n1) return;
    const int x0 = (int)(x / n1), x1 = (int)(x % n1);
    const T sa = s0[x], sb = s1[x];
    const int Ra = r0[x], Rb = r1[x];
    const T inv = T(1) / (gauss_norm(sa, Ra) * gauss_norm(sb, Rb));
    for (int v0 = 0; v0 < B; v0 += kVec) {
        T acc[kVec];
        for (int v = 0; v < kVec; ++v) acc[v] = T(0);
        for (int z0 = -Ra; z0 <= Ra; ++z0) {
            const int y0 = x0 + z0;
            if (y0 < 0 || y0 >= n0) continue;
            const T w0 = exp(-(T)(z0 * z0) / (2 * sa * sa));
            for (int z1 = -Rb; z1 <= Rb; ++z1) {
                const int y1 = x1 + z1;
                if (y1 < 0 || y1 >= n1) continue;
                const T w = w0 * exp(-(T)(z1 * z1) / (2 * sb * sb));
                const int64_t y = (int64_t)y0 * n1 + y1;
#pragma unroll
                for (int v = 0; v < kVec; ++v)
                    if (v0 + v < B) acc[v] += w * in[(int64_t)(v0 + v) * ldin + y];
            }
        }
        for (int v = 0; v < kVec; ++v)
            if (v0 + v < B) out[(int64_t)(v0 + v) * ldout + x] = acc[v] * inv;
    }
}

}  // namespace

extern "C" {

// s0, s1: per-point widths along axes 0 and 1 (device, n0*n1 each, dtype);
// r0, r1: per-point radii (device int32).  in/out: B device vectors with
// leading dimensions ldin/ldout.  dtype 0 = f32, 1 = f64.  Returns 0 on success.
int blur_adjoint(int dtype, const void* s0, const void* s1, const int32_t* r0, const int32_t* r1, int n0, int n1,
                 const void* in, int64_t ldin, void* out, int64_t ldout, int B, hipStream_t stream) {
    const int64_t N = (int64_t)n0 * n1;
    const unsigned grid = (unsigned)((N + kThreads - 1) / kThreads);
    if (dtype == 1)
        hipLaunchKernelGGL(blur_adjoint_kernel<double>, dim3(grid), dim3(kThreads), 0, stream,
                           static_cast<const double*>(s0), static_cast<const double*>(s1), r0, r1, n0, n1,
                           static_cast<const double*>(in), ldin, static_cast<double*>(out), ldout, B);
    else
        hipLaunchKernelGGL(blur_adjoint_kernel<float>, dim3(grid), dim3(kThreads), 0, stream,
                           static_cast<const float*>(s0), static_cast<const float*>(s1), r0, r1, n0, n1,
                           static_cast<const float*>(in), ldin, static_cast<float*>(out), ldout, B);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // extern "C"
