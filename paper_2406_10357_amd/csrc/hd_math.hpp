// hd_math.hpp -- small device vector math and precision traits for the HIP
// library. Everything is templated on the scalar type T (float or double);
// one code path serves FP32 and FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HD_HD __host__ __device__ __forceinline__
#define HD_D __device__ __forceinline__

namespace hd {

template <class T> struct V3 {
    T x, y, z;
};

template <class T> HD_HD V3<T> mk(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> HD_HD V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> HD_HD V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> HD_HD V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> HD_HD T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> HD_HD V3<T> cross(V3<T> a, V3<T> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> HD_HD T norm2(V3<T> a) { return dot(a, a); }
template <class T> HD_HD T hmin(T a, T b) { return a < b ? a : b; }
template <class T> HD_HD T hmax(T a, T b) { return a > b ? a : b; }
template <class T> HD_HD T clamp01(T t) { return hmin(hmax(t, T(0)), T(1)); }
// a[k] for k in 0..2 as selects between values. A run-time index into a
// register array (or a ?: between two array elements, which selects an
// address) makes the compiler keep the array in private (scratch) memory.
template <class X> HD_HD X pick3(X a0, X a1, X a2, int k) {
    X r = a2;
    if (k == 0) r = a0;
    if (k == 1) r = a1;
    return r;
}
template <class T> HD_HD T clampab(T t, T a, T b) { return hmin(hmax(t, a), b); }

HD_D float hsqrt(float x) { return __builtin_sqrtf(x); }
HD_D double hsqrt(double x) { return __builtin_sqrt(x); }

template <class To, class From> HD_HD V3<To> cvt(V3<From> a) { return {To(a.x), To(a.y), To(a.z)}; }

// Unit roundoff of round-to-nearest arithmetic.
template <class T> struct Prec;
template <> struct Prec<float> { static constexpr double u = 5.9604644775390625e-08; };  // 2^-24
template <> struct Prec<double> { static constexpr double u = 1.1102230246251565e-16; }; // 2^-53

// Order-preserving maps between non-negative IEEE floats and unsigned ints
// (so atomicMax on the bits is a max on the values).
HD_HD uint32_t f2ord(float f) {
    uint32_t b = __builtin_bit_cast(uint32_t, f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
HD_HD float ord2f(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __builtin_bit_cast(float, b);
}
HD_HD unsigned long long d2ord(double f) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, f);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
HD_HD double ord2d(unsigned long long o) {
    unsigned long long b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __builtin_bit_cast(double, b);
}

} // namespace hd

namespace hd {
// neighbouring floats (finite inputs)
HD_HD float next_down(float f) {
    uint32_t b = __builtin_bit_cast(uint32_t, f);
    if (f > 0.0f) b -= 1;
    else if (f < 0.0f) b += 1;
    else b = 0x80000001u;
    return __builtin_bit_cast(float, b);
}
HD_HD float next_up(float f) {
    uint32_t b = __builtin_bit_cast(uint32_t, f);
    if (f > 0.0f) b += 1;
    else if (f < 0.0f) b -= 1;
    else b = 0x00000001u;
    return __builtin_bit_cast(float, b);
}
} // namespace hd
