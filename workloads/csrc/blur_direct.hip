// Exact spatially varying Gaussian blur on the GPU (the black-box operator A
// whose impulse responses feed the product-convolution approximation; it is
// not part of the approximation itself).
//
// A[y, x] = exp(-sum_i (y_i - x_i)^2 / (2 s_i(x)^2)) / Z(x) for |y_i - x_i| <=
// R_i(x) = ceil(4 s_i(x)), Z(x) the sum of the same Gaussian over the full box.
// blur_adjoint computes (A^T v)[x] = sum_z g_x(z) v[x + z] over x + z in Omega
// for B vectors (the exact adjoint the error estimator needs).  blur_adjoint
// takes 2-D domains (d = 1 is a single row), blur_adjoint3 3-D ones.  Widths
// and radii come from the host so that the radii match the supplied impulse
// responses exactly.
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

// Forward blur, 2-D: (A u)[y] = sum_x A[y, x] u[x].  One thread per y
// gathers over the x with |y_i - x_i| <= rmax_i (the largest radii) and
// keeps those with |y_i - x_i| <= R_i(x); inv_z[x] = 1 / Z(x) comes from the
// host.
template <class T>
__global__ __launch_bounds__(kThreads) void blur_forward_kernel(const T* s0, const T* s1, const int32_t* r0,
                                                                const int32_t* r1, const T* inv_z, int n0, int n1,
                                                                int rmax0, int rmax1, const T* in, int64_t ldin,
                                                                T* out, int64_t ldout, int B) {
    const int64_t y = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (y >= (int64_t)n0 * n1) return;
    const int y0 = (int)(y / n1), y1 = (int)(y % n1);
    for (int v0 = 0; v0 < B; v0 += kVec) {
        T acc[kVec];
        for (int v = 0; v < kVec; ++v) acc[v] = T(0);
        for (int x0 = y0 - rmax0; x0 <= y0 + rmax0; ++x0) {
            if (x0 < 0 || x0 >= n0) continue;
            const int d0 = y0 - x0;
            for (int x1 = y1 - rmax1; x1 <= y1 + rmax1; ++x1) {
                if (x1 < 0 || x1 >= n1) continue;
                const int64_t x = (int64_t)x0 * n1 + x1;
                const int d1 = y1 - x1;
                if (abs(d0) > r0[x] || abs(d1) > r1[x]) continue;
                const T sa = s0[x], sb = s1[x];
                const T w = exp(-(T)(d0 * d0) / (2 * sa * sa) - (T)(d1 * d1) / (2 * sb * sb)) * inv_z[x];
#pragma unroll
                for (int v = 0; v < kVec; ++v)
                    if (v0 + v < B) acc[v] += w * in[(int64_t)(v0 + v) * ldin + x];
            }
        }
        for (int v = 0; v < kVec; ++v)
            if (v0 + v < B) out[(int64_t)(v0 + v) * ldout + y] = acc[v];
    }
}

// 3-D: one thread per x; the axis-2 Gaussian factors come from the exact
// recurrence g(z+1) = g(z) r(z), r(z+1) = r(z) exp(-1/s^2) in FP64 (no exp
// per tap), the axis-0 and axis-1 factors from exp.
template <class T>
__global__ __launch_bounds__(kThreads) void blur_adjoint3_kernel(const T* s0, const T* s1, const T* s2,
                                                                 const int32_t* r0, const int32_t* r1,
                                                                 const int32_t* r2, int n0, int n1, int n2,
                                                                 const T* in, int64_t ldin, T* out, int64_t ldout,
                                                                 int B) {
    const int64_t plane = (int64_t)n1 * n2;
    const int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (x >= (int64_t)n0 * plane) return;
    const int x0 = (int)(x / plane);
    const int64_t rem = x - (int64_t)x0 * plane;
    const int x1 = (int)(rem / n2), x2 = (int)(rem - (int64_t)x1 * n2);
    const double sa = (double)s0[x], sb = (double)s1[x], sc = (double)s2[x];
    const int Ra = r0[x], Rb = r1[x], Rc = r2[x];
    const double inv = 1.0 / (gauss_norm(sa, Ra) * gauss_norm(sb, Rb) * gauss_norm(sc, Rc));
    const int z2lo = -x2 > -Rc ? -x2 : -Rc;
    const int z2hi = n2 - 1 - x2 < Rc ? n2 - 1 - x2 : Rc;
    const double g_lo = exp(-(double)z2lo * z2lo / (2 * sc * sc));
    const double r_lo = exp(-(double)(2 * z2lo + 1) / (2 * sc * sc));
    const double q2 = exp(-1.0 / (sc * sc));
    for (int v0 = 0; v0 < B; v0 += kVec) {
        T acc[kVec];
        for (int v = 0; v < kVec; ++v) acc[v] = T(0);
        for (int z0 = -Ra; z0 <= Ra; ++z0) {
            const int y0 = x0 + z0;
            if (y0 < 0 || y0 >= n0) continue;
            const double w0 = exp(-(double)(z0 * z0) / (2 * sa * sa));
            for (int z1 = -Rb; z1 <= Rb; ++z1) {
                const int y1 = x1 + z1;
                if (y1 < 0 || y1 >= n1) continue;
                const double w01 = w0 * exp(-(double)(z1 * z1) / (2 * sb * sb));
                const int64_t ybase = (int64_t)y0 * plane + (int64_t)y1 * n2 + x2;
                double g = g_lo, r = r_lo;
                for (int z2 = z2lo; z2 <= z2hi; ++z2) {
                    const T w = (T)(w01 * g);
                    const int64_t y = ybase + z2;
#pragma unroll
                    for (int v = 0; v < kVec; ++v)
                        if (v0 + v < B) acc[v] += w * in[(int64_t)(v0 + v) * ldin + y];
                    g *= r;
                    r *= q2;
                }
            }
        }
        for (int v = 0; v < kVec; ++v)
            if (v0 + v < B) out[(int64_t)(v0 + v) * ldout + x] = (T)((double)acc[v] * inv);
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

// Forward blur, 2-D (d = 1 as one row): out = A in.  inv_z: 1 / Z(x) per x
// (device, dtype); rmax0, rmax1: the largest radii along each axis.
int blur_forward(int dtype, const void* s0, const void* s1, const int32_t* r0, const int32_t* r1, const void* inv_z,
                 int n0, int n1, int rmax0, int rmax1, const void* in, int64_t ldin, void* out, int64_t ldout, int B,
                 hipStream_t stream) {
    const int64_t N = (int64_t)n0 * n1;
    const unsigned grid = (unsigned)((N + kThreads - 1) / kThreads);
    if (dtype == 1)
        hipLaunchKernelGGL(blur_forward_kernel<double>, dim3(grid), dim3(kThreads), 0, stream,
                           static_cast<const double*>(s0), static_cast<const double*>(s1), r0, r1,
                           static_cast<const double*>(inv_z), n0, n1, rmax0, rmax1, static_cast<const double*>(in),
                           ldin, static_cast<double*>(out), ldout, B);
    else
        hipLaunchKernelGGL(blur_forward_kernel<float>, dim3(grid), dim3(kThreads), 0, stream,
                           static_cast<const float*>(s0), static_cast<const float*>(s1), r0, r1,
                           static_cast<const float*>(inv_z), n0, n1, rmax0, rmax1, static_cast<const float*>(in),
                           ldin, static_cast<float*>(out), ldout, B);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

// 3-D: s0, s1, s2 widths and r0, r1, r2 radii along axes 0, 1, 2 (device,
// n0*n1*n2 each); otherwise as blur_adjoint.
int blur_adjoint3(int dtype, const void* s0, const void* s1, const void* s2, const int32_t* r0, const int32_t* r1,
                  const int32_t* r2, int n0, int n1, int n2, const void* in, int64_t ldin, void* out, int64_t ldout,
                  int B, hipStream_t stream) {
    const int64_t N = (int64_t)n0 * n1 * n2;
    const unsigned grid = (unsigned)((N + kThreads - 1) / kThreads);
    if (dtype == 1)
        hipLaunchKernelGGL(blur_adjoint3_kernel<double>, dim3(grid), dim3(kThreads), 0, stream,
                           static_cast<const double*>(s0), static_cast<const double*>(s1),
                           static_cast<const double*>(s2), r0, r1, r2, n0, n1, n2, static_cast<const double*>(in),
                           ldin, static_cast<double*>(out), ldout, B);
    else
        hipLaunchKernelGGL(blur_adjoint3_kernel<float>, dim3(grid), dim3(kThreads), 0, stream,
                           static_cast<const float*>(s0), static_cast<const float*>(s1),
                           static_cast<const float*>(s2), r0, r1, r2, n0, n1, n2, static_cast<const float*>(in),
                           ldin, static_cast<float*>(out), ldout, B);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // extern "C"
