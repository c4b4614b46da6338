// cplx.hpp -- complex arithmetic on HIP vector types (float2 / double2) for gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace fcn {

template <typename R>
struct vec2;
template <>
struct vec2<float> {
    using type = float2;
};
template <>
struct vec2<double> {
    using type = double2;
};
template <typename R>
using c2 = typename vec2<R>::type;

template <typename R>
__device__ __forceinline__ c2<R> mk(R x, R y) {
    c2<R> r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename R>
__device__ __forceinline__ c2<R> cadd(c2<R> a, c2<R> b) {
    return mk<R>(a.x + b.x, a.y + b.y);
}
template <typename R>
__device__ __forceinline__ c2<R> csub(c2<R> a, c2<R> b) {
    return mk<R>(a.x - b.x, a.y - b.y);
}
template <typename R>
__device__ __forceinline__ c2<R> cmul(c2<R> a, c2<R> b) {
    return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__device__ __forceinline__ c2<R> cmulc(c2<R> a, c2<R> b) {  // a * conj(b)
    return mk<R>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// a * (h + l) and a * conj(h + l) for a constant carried as a hi + lo pair (|l| <= ulp(h)/2):
// the small product a * l is added into the fused products of a * h.
template <typename R>
__device__ __forceinline__ c2<R> cmul_pair(c2<R> a, c2<R> h, c2<R> l) {
    const R px = a.x * l.x - a.y * l.y, py = a.x * l.y + a.y * l.x;
    return mk<R>(fma(a.x, h.x, fma(-a.y, h.y, px)), fma(a.x, h.y, fma(a.y, h.x, py)));
}
template <typename R>
__device__ __forceinline__ c2<R> cmulc_pair(c2<R> a, c2<R> h, c2<R> l) {
    const R px = a.x * l.x + a.y * l.y, py = a.y * l.x - a.x * l.y;
    return mk<R>(fma(a.x, h.x, fma(a.y, h.y, px)), fma(a.y, h.x, fma(-a.x, h.y, py)));
}
template <typename R>
__device__ __forceinline__ c2<R> cscale(c2<R> a, R s) {
    return mk<R>(a.x * s, a.y * s);
}
// a * (i s), s real
template <typename R>
__device__ __forceinline__ c2<R> cmul_i(c2<R> a, R s) {
    return mk<R>(-a.y * s, a.x * s);
}
// 1 / a
template <typename R>
__device__ __forceinline__ c2<R> crcp(c2<R> a) {
    R d = R(1) / (a.x * a.x + a.y * a.y);
    return mk<R>(a.x * d, -a.y * d);
}
template <typename R>
__device__ __forceinline__ c2<R> czero() {
    return mk<R>(R(0), R(0));
}
// conversion between storage and arithmetic precision (round to nearest when narrowing)
template <typename To, typename From>
__device__ __forceinline__ c2<To> ccast(c2<From> a) {
    return mk<To>(To(a.x), To(a.y));
}

}  // namespace fcn
