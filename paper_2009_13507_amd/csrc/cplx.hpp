// cplx.hpp -- complex arithmetic and small-argument trigonometric series for
// the gfx950 kernels.  Real type R is double (complex128 states) or float
// (complex64 states).
#pragma once
#include <hip/hip_runtime.h>

namespace ssgp {

__host__ __device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }

template <typename R> struct alignas(2 * sizeof(R)) cx {
    R x, y;
};

template <typename R> __host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R> __host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
template <typename R> __host__ __device__ __forceinline__ R abs2(cx<R> a) { return a.x * a.x + a.y * a.y; }
// a * b + c
template <typename R> __host__ __device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
    return {fma_(a.x, b.x, fma_(-a.y, b.y, c.x)), fma_(a.x, b.y, fma_(a.y, b.x, c.y))};
}
// i * a
template <typename R> __host__ __device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.y, a.x}; }
// Crank-Nicolson right-hand side (I - sT) u / o at one point from the
// diagonal coefficient d = (1 - s/h^2) / o, the point's value u and the sum
// of its two neighbours: the off-diagonal s/(2h^2) / o is exactly -1, so
// the value is d u - (u_{i-1} + u_{i+1}).
template <typename R> __host__ __device__ __forceinline__ cx<R> cn_rhs(cx<R> d, cx<R> u, cx<R> nsum) {
    return {fma_(d.x, u.x, fma_(-d.y, u.y, -nsum.x)), fma_(d.x, u.y, fma_(d.y, u.x, -nsum.y))};
}
template <typename R> __host__ __device__ __forceinline__ cx<R> czero() { return {R(0), R(0)}; }

// Lane shuffles of a complex value across the 64-lane wavefront.
template <typename R> __device__ __forceinline__ cx<R> shfl_up(cx<R> v, int d) {
    return {__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64)};
}
template <typename R> __device__ __forceinline__ cx<R> shfl_down(cx<R> v, int d) {
    return {__shfl_down(v.x, d, 64), __shfl_down(v.y, d, 64)};
}

// Taylor series in q = u^2 (u real), summed by Horner from the highest
// term.  Ten terms each; for q <= (pi/4)^2 the first omitted term is below
// 2e-18 relative, so the series are correctly rounded to a few ulp in FP64.
//   sinc_q(q)   = sin(u)/u   = sum_k (-q)^k / (2k+1)!
//   cos_q(q)    = cos(u)     = sum_k (-q)^k / (2k)!
//   sinhc_q(q)  = sinh(u)/u  = sum_k q^k / (2k+1)!
//   cosh_q(q)   = cosh(u)    = sum_k q^k / (2k)!
// The coefficients are the reciprocals 1/n!, folded at compile time.
__host__ __device__ constexpr double inv_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return 1.0 / f;
}

template <typename R, bool ALT, int ODD, int NT = 10>
__host__ __device__ __forceinline__ R series_q(R q) {
    // sum_{k=0}^{NT-1} s^k q^k / (2k+ODD)!, s = -1 if ALT
    R acc = R(inv_fact(2 * (NT - 1) + ODD));
#pragma unroll
    for (int k = NT - 2; k >= 0; --k) {
        const R c = R(inv_fact(2 * k + ODD));
        acc = ALT ? fma_(-q, acc, c) : fma_(q, acc, c);
    }
    return acc;
}
template <typename R> __host__ __device__ __forceinline__ R sinc_q(R q) { return series_q<R, true, 1>(q); }
template <typename R> __host__ __device__ __forceinline__ R cos_q(R q) { return series_q<R, true, 0>(q); }
template <typename R> __host__ __device__ __forceinline__ R sinhc_q(R q) { return series_q<R, false, 1>(q); }
template <typename R> __host__ __device__ __forceinline__ R cosh_q(R q) { return series_q<R, false, 0>(q); }

// Largest u^2 for which the series above are used.
template <typename R> struct SeriesLimit { static constexpr R q = R(0.6168502750680849); };  // (pi/4)^2
// Shorter series: with q <= SERIES_Qn the first omitted term of the n-term
// series, q^n / (2n)!, is below 2^-60 relative (the sums are >= 0.99 there).
// A wavefront takes the shortest series valid for all its lanes.
constexpr double SERIES_Q2 = 4e-9, SERIES_Q3 = 8e-6, SERIES_Q4 = 4e-4, SERIES_Q5 = 4.5e-3, SERIES_Q6 = 2.5e-2;

} // namespace ssgp
