// m2p_dual.h -- forward-mode dual numbers (value + one tangent) for the
// adjoint kernels.  The stage's device functions are templates on the scalar
// type, so instantiating them on Dual<T> yields directional derivatives of
// exactly the arithmetic the forward kernels execute.  Comparisons and
// selects act on values (minmod, max, clamps take the derivative of the
// selected branch); sqrt at 0 takes derivative 0.
#pragma once

#include <hip/hip_runtime.h>

namespace m2p {

template <typename T>
struct Dual {
    T v, d;
    __host__ __device__ Dual() : v(0), d(0) {}
    __host__ __device__ Dual(double x) : v(T(x)), d(0) {}
    __host__ __device__ Dual(T x, T dx) : v(x), d(dx) {}
    __device__ Dual operator-() const { return Dual(-v, -d); }
    __device__ Dual& operator+=(const Dual& b)
    {
        v += b.v;
        d += b.d;
        return *this;
    }
};

template <typename T> __device__ __forceinline__ Dual<T> operator+(const Dual<T>& a, const Dual<T>& b) { return Dual<T>(a.v + b.v, a.d + b.d); }
template <typename T> __device__ __forceinline__ Dual<T> operator-(const Dual<T>& a, const Dual<T>& b) { return Dual<T>(a.v - b.v, a.d - b.d); }
template <typename T> __device__ __forceinline__ Dual<T> operator*(const Dual<T>& a, const Dual<T>& b) { return Dual<T>(a.v * b.v, a.d * b.v + a.v * b.d); }
template <typename T> __device__ __forceinline__ Dual<T> operator/(const Dual<T>& a, const Dual<T>& b)
{
    const T q = a.v / b.v;
    return Dual<T>(q, (a.d - q * b.d) / b.v);
}
template <typename T> __device__ __forceinline__ bool operator>(const Dual<T>& a, const Dual<T>& b) { return a.v > b.v; }
template <typename T> __device__ __forceinline__ bool operator<(const Dual<T>& a, const Dual<T>& b) { return a.v < b.v; }
template <typename T> __device__ __forceinline__ bool operator>=(const Dual<T>& a, const Dual<T>& b) { return a.v >= b.v; }
template <typename T> __device__ __forceinline__ bool operator<=(const Dual<T>& a, const Dual<T>& b) { return a.v <= b.v; }
template <typename T> __device__ __forceinline__ Dual<T> sqrt(const Dual<T>& a)
{
    const T s = ::sqrt(a.v);
    return Dual<T>(s, s > T(0) ? a.d / (T(2) * s) : T(0));
}
template <typename T> __device__ __forceinline__ Dual<T> fabs(const Dual<T>& a) { return a.v < T(0) ? -a : a; }

template <typename T> __device__ __forceinline__ T val(const T& x) { return x; }
template <typename T> __device__ __forceinline__ T val(const Dual<T>& x) { return x.v; }

}  // namespace m2p
