// Forward-mode dual number (value, derivative along one parameter direction).
// Instantiating the operator and energy kernels on this type gives, with the
// displacement held fixed, the derivative of A u and of the energy density with
// respect to the seeded material constants or element thicknesses: the
// linearisation the adjoint gradient needs, consistent with the forward
// operator by construction.
#pragma once

#include <hip/hip_runtime.h>

namespace dgtn {

struct Dual {
    double v, d;
    Dual() = default;
    __host__ __device__ constexpr Dual(double x) : v(x), d(0.0) {}
    __host__ __device__ constexpr Dual(double x, double dx) : v(x), d(dx) {}
    // found by argument-dependent lookup only, so the plain overloads stay visible
    friend __device__ inline Dual sqrt(Dual a) {
        const double s = ::sqrt(a.v);
        return Dual(s, s > 0 ? 0.5 * a.d / s : 0.0);
    }
    friend __device__ inline Dual min(Dual a, Dual b) { return a.v <= b.v ? a : b; }
};

__host__ __device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__host__ __device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__host__ __device__ inline Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__host__ __device__ inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
__host__ __device__ inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
__host__ __device__ inline Dual& operator*=(Dual& a, Dual b) { return a = a * b; }
__host__ __device__ inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
__host__ __device__ inline bool operator>(Dual a, Dual b) { return a.v > b.v; }

}  // namespace dgtn
