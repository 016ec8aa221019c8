// Register-resident DFT codelets for the convolution kernels (gfx950).
//
// Dft<R, S>::run(x) replaces x[0..R) by X[k] = sum_j x[j] w^(j k) with
// w = exp(S 2 pi i / R): S = -1 is the forward transform, S = +1 the
// unnormalised inverse.  Primes 2, 3, 5, 7 and radix 4 are written out;
// composite radices split as R = P * Q (decimation in time) with the inner
// twiddles as compile-time constants.  Those constants come from a constexpr
// evaluation in FP64 (exact integer reduction of the angle to [0, pi/4], then
// Taylor series) and are rounded once to the working precision.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace pc {

template <class T>
struct cx {
    T x, y;
};

template <class T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <class T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <class T>
__host__ __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// (S i) * a
template <int S, class T>
__host__ __device__ __forceinline__ cx<T> mul_si(cx<T> a) {
    if constexpr (S > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
}

// ---------------------------------------------------------------- constants
constexpr double kTwoPi = 6.28318530717958647692528676655900577;

constexpr double series_cos(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k <= 14; ++k) {
        term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
constexpr double series_sin(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k <= 14; ++k) {
        term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
// cos(2 pi num / den) with the fraction reduced exactly in integers.
constexpr double cos_turn(long num, long den) {
    long n = num % den;
    if (n < 0) n += den;
    if (2 * n > den) n = den - n;              // cos is even: fraction in [0, 1/2]
    double sign = 1.0;
    if (4 * n > den) {                         // fraction in (1/4, 1/2]: cos(pi - x) = -cos x
        sign = -1.0;
        long nn = den - 2 * n;                 // (den - 2n) / (2 den) in [0, 1/4)
        den = 2 * den;
        n = nn;
    }
    if (8 * n > den)                           // (1/8, 1/4]: cos x = sin(pi/2 - x)
        return sign * series_sin(kTwoPi * (double)(den - 4 * n) / (double)(4 * den));
    return sign * series_cos(kTwoPi * (double)n / (double)den);
}
// sin(2 pi num / den) = cos(2 pi (num/den - 1/4))
constexpr double sin_turn(long num, long den) { return cos_turn(4 * num - den, 4 * den); }

// v * w^E, w = exp(S 2 pi i / R), E a compile-time constant.
template <int R, int E, int S, class T>
__host__ __device__ __forceinline__ cx<T> twc(cx<T> v) {
    constexpr int e = ((E % R) + R) % R;
    if constexpr (e == 0) {
        return v;
    } else if constexpr (2 * e == R) {
        return {-v.x, -v.y};
    } else if constexpr (4 * e == R) {
        return mul_si<S>(v);
    } else if constexpr (4 * e == 3 * R) {
        return mul_si<-S>(v);
    } else {
        constexpr T c = (T)cos_turn(e, R);
        constexpr T s = (T)((double)S * sin_turn(e, R));
        return {v.x * c - v.y * s, v.x * s + v.y * c};
    }
}

template <int I, int N, class F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

constexpr int smallest_factor(int n) {
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}
constexpr bool is_prime(int n) { return n >= 2 && smallest_factor(n) == n; }

template <int R, int S>
struct Dft;

template <int S>
struct Dft<1, S> {
    template <class T>
    __host__ __device__ __forceinline__ static void run(cx<T>*) {}
};

template <int S>
struct Dft<2, S> {
    template <class T>
    __host__ __device__ __forceinline__ static void run(cx<T>* x) {
        cx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    }
};

template <int S>
struct Dft<4, S> {
    template <class T>
    __host__ __device__ __forceinline__ static void run(cx<T>* x) {
        cx<T> t0 = x[0] + x[2], t1 = x[0] - x[2];
        cx<T> t2 = x[1] + x[3], t3 = mul_si<S>(x[1] - x[3]);
        x[0] = t0 + t2;
        x[2] = t0 - t2;
        x[1] = t1 + t3;
        x[3] = t1 - t3;
    }
};

// Odd primes: pair x_m with x_{P-m}.
template <int P, int S>
struct DftOddPrime {
    template <class T>
    __host__ __device__ __forceinline__ static void run(cx<T>* x) {
        constexpr int H = (P - 1) / 2;
        cx<T> a[H + 1], b[H + 1];
        cx<T> x0 = x[0];
        cx<T> sum = x0;
        static_for<1, H + 1>([&](auto mm) {
            constexpr int m = decltype(mm)::value;
            a[m] = x[m] + x[P - m];
            b[m] = x[m] - x[P - m];
            sum = sum + a[m];
        });
        cx<T> out[P];
        out[0] = sum;
        static_for<1, H + 1>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            cx<T> re = x0, im = {T(0), T(0)};
            static_for<1, H + 1>([&](auto mm) {
                constexpr int m = decltype(mm)::value;
                constexpr T c = (T)cos_turn((long)k * m, P);
                constexpr T s = (T)sin_turn((long)k * m, P);
                re = {re.x + a[m].x * c, re.y + a[m].y * c};
                im = {im.x + b[m].x * s, im.y + b[m].y * s};
            });
            cx<T> sim = mul_si<S>(im);
            out[k] = re + sim;
            out[P - k] = re - sim;
        });
        static_for<0, P>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            x[k] = out[k];
        });
    }
};

template <int S> struct Dft<3, S> : DftOddPrime<3, S> {};
template <int S> struct Dft<5, S> : DftOddPrime<5, S> {};
template <int S> struct Dft<7, S> : DftOddPrime<7, S> {};

// Composite radix R = P * Q, decimation in time:
//   X[k1 + P k0] = sum_j0 w_Q^(j0 k0) [ w_R^(j0 k1) sum_j1 x[Q j1 + j0] w_P^(j1 k1) ].
template <int R, int S>
struct DftComposite {
    static constexpr int P = (R % 4 == 0 && R > 4) ? 4 : smallest_factor(R);
    static constexpr int Q = R / P;
    template <class T>
    __host__ __device__ __forceinline__ static void run(cx<T>* x) {
        cx<T> y[R];
        static_for<0, Q>([&](auto jj0) {
            constexpr int j0 = decltype(jj0)::value;
            cx<T> t[P];
            static_for<0, P>([&](auto jj1) {
                constexpr int j1 = decltype(jj1)::value;
                t[j1] = x[Q * j1 + j0];
            });
            Dft<P, S>::run(t);
            static_for<0, P>([&](auto kk1) {
                constexpr int k1 = decltype(kk1)::value;
                y[j0 * P + k1] = twc<R, j0 * k1, S>(t[k1]);
            });
        });
        static_for<0, P>([&](auto kk1) {
            constexpr int k1 = decltype(kk1)::value;
            cx<T> t[Q];
            static_for<0, Q>([&](auto jj0) {
                constexpr int j0 = decltype(jj0)::value;
                t[j0] = y[j0 * P + k1];
            });
            Dft<Q, S>::run(t);
            static_for<0, Q>([&](auto kk0) {
                constexpr int k0 = decltype(kk0)::value;
                x[k1 + P * k0] = t[k0];
            });
        });
    }
};

template <int S> struct Dft<6, S> : DftComposite<6, S> {};
template <int S> struct Dft<8, S> : DftComposite<8, S> {};
template <int S> struct Dft<9, S> : DftComposite<9, S> {};
template <int S> struct Dft<10, S> : DftComposite<10, S> {};
template <int S> struct Dft<12, S> : DftComposite<12, S> {};
template <int S> struct Dft<14, S> : DftComposite<14, S> {};
template <int S> struct Dft<15, S> : DftComposite<15, S> {};
template <int S> struct Dft<16, S> : DftComposite<16, S> {};

// Runtime radix dispatch on a register array of kMaxRadix elements.
template <int S, class T>
__host__ __device__ __forceinline__ void dft_rt(int r, cx<T>* x) {
    switch (r) {
        case 2: Dft<2, S>::run(x); break;
        case 3: Dft<3, S>::run(x); break;
        case 4: Dft<4, S>::run(x); break;
        case 5: Dft<5, S>::run(x); break;
        case 6: Dft<6, S>::run(x); break;
        case 7: Dft<7, S>::run(x); break;
        case 8: Dft<8, S>::run(x); break;
        case 9: Dft<9, S>::run(x); break;
        case 10: Dft<10, S>::run(x); break;
        case 12: Dft<12, S>::run(x); break;
        case 14: Dft<14, S>::run(x); break;
        case 15: Dft<15, S>::run(x); break;
        case 16: Dft<16, S>::run(x); break;
        default: break;   // radix 1: identity
    }
}

}  // namespace pc
