// Double-double arithmetic: a value held as the unevaluated sum hi + lo of two
// doubles with |lo| <= ulp(hi) / 2, about 106 significant bits.  Instantiating
// the operator kernels on this type evaluates A u of a double u, with the
// operator's double coefficients, without the cancellation that limits the FP64
// residual b - A u (the interior-penalty terms sigma [u], sigma = C N^2 / h, are
// large and cancel in the residual of an accurate solution): the extended-
// precision residual of iterative refinement in three precisions (Carson and
// Higham, SIAM J. Sci. Comput. 40 (2018) A817).
//
// The building blocks are the error-free transformations: Knuth's two-sum
// (s + e = a + b exactly) and the product with a fused multiply-add
// (p + e = a * b exactly).  Contraction of a * b + c into one fused operation is
// switched off inside them, since it would change the roundings the error terms
// account for.
#pragma once

#include <hip/hip_runtime.h>

namespace dgtn {

struct DD;
__device__ inline DD dd_sqrt(DD a);

struct DD {
    double hi, lo;
    DD() = default;
    __host__ __device__ constexpr DD(double x) : hi(x), lo(0.0) {}
    __host__ __device__ constexpr DD(double h, double l) : hi(h), lo(l) {}
    // hidden friends, found by argument-dependent lookup only, so that the plain
    // overloads for double stay visible inside the namespace
    friend __device__ inline DD sqrt(DD a) { return dd_sqrt(a); }
    friend __device__ inline DD min(DD a, DD b) { return (a.hi < b.hi || (a.hi == b.hi && a.lo <= b.lo)) ? a : b; }
};

// s + e == a + b exactly (any a, b)
__host__ __device__ inline DD two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return DD(s, e);
}

// s + e == a + b exactly, given |a| >= |b| or a == 0
__host__ __device__ inline DD quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    return DD(s, b - (s - a));
}

// p + e == a * b exactly
__host__ __device__ inline DD two_prod(double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    return DD(p, __builtin_fma(a, b, -p));
}

__host__ __device__ inline DD operator+(DD a, DD b) {
#pragma clang fp contract(off)
    DD s = two_sum(a.hi, b.hi);
    const DD t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__host__ __device__ inline DD operator-(DD a) { return DD(-a.hi, -a.lo); }
__host__ __device__ inline DD operator-(DD a, DD b) { return a + (-b); }

__host__ __device__ inline DD operator*(DD a, DD b) {
#pragma clang fp contract(off)
    DD p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

// quotient: the double quotient, its remainder in double-double, one correction
__host__ __device__ inline DD operator/(DD a, DD b) {
#pragma clang fp contract(off)
    const double q1 = a.hi / b.hi;
    const DD r = a - b * DD(q1);
    const double q2 = r.hi / b.hi;
    const DD r2 = r - b * DD(q2);
    const double q3 = r2.hi / b.hi;
    const DD q = quick_two_sum(q1, q2);
    return q + DD(q3);
}

__device__ inline DD dd_sqrt(DD a) {
#pragma clang fp contract(off)
    if (!(a.hi > 0)) return DD(0.0);
    const double s = ::sqrt(a.hi);
    const DD r = a - two_prod(s, s);
    return quick_two_sum(s, r.hi / (2.0 * s));
}

__host__ __device__ inline DD& operator+=(DD& a, DD b) { return a = a + b; }
__host__ __device__ inline DD& operator-=(DD& a, DD b) { return a = a - b; }
__host__ __device__ inline DD& operator*=(DD& a, DD b) { return a = a * b; }
__host__ __device__ inline bool operator<(DD a, DD b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__host__ __device__ inline bool operator>(DD a, DD b) { return b < a; }
__host__ __device__ inline bool operator<=(DD a, DD b) { return !(b < a); }
__host__ __device__ inline bool operator>=(DD a, DD b) { return !(a < b); }
__host__ __device__ inline bool operator==(DD a, DD b) { return a.hi == b.hi && a.lo == b.lo; }
__host__ __device__ inline bool operator!=(DD a, DD b) { return !(a == b); }

}  // namespace dgtn
