// cx.h -- plain complex value type shared by host and device code of libcsg.
#pragma once

#include <hip/hip_runtime.h>

namespace csg {

// Interleaved complex (re, im) with natural vector alignment, so a complex128
// element moves as one 16-byte access and a complex64 element as one 8-byte one.
template <typename T>
struct alignas(2 * sizeof(T)) Cx {
    T re, im;
};
using zc = Cx<double>;
using cf = Cx<float>;

template <typename T>
__host__ __device__ __forceinline__ Cx<T> mkc(T re, T im) { Cx<T> r; r.re = re; r.im = im; return r; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return mkc<T>(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return mkc<T>(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b)
{
    return mkc<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) { return mkc<T>(s * a.re, s * a.im); }
// a * b + c
template <typename T>
__host__ __device__ __forceinline__ Cx<T> cfma(Cx<T> a, Cx<T> b, Cx<T> c)
{
    return mkc<T>(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}
// conj(a) * b + c
template <typename T>
__host__ __device__ __forceinline__ Cx<T> cjfma(Cx<T> a, Cx<T> b, Cx<T> c)
{
    return mkc<T>(fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.re, b.im, fma(-a.im, b.re, c.im)));
}
template <typename T>
__host__ __device__ __forceinline__ T cabs2(Cx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename TO, typename TI>
__host__ __device__ __forceinline__ Cx<TO> cvt(Cx<TI> a) { return mkc<TO>((TO)a.re, (TO)a.im); }

}  // namespace csg
