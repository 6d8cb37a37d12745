// The quotient of Eq. 1, a / c for a neighbour count c >= 1, correctly
// rounded, from a multiplication and two fused multiply-adds.  Host and
// device code: the library's kernels call it, and a CPU test compares it
// with IEEE division.
//
// With p the precision in bits (53 or 24) and y = RN(1/c) (a table of one
// division per count):
//   q  = RN(a * y)        within two units in the last place (ulp) of a / c;
//   r  = RN(a - c * q)    exact, by a fused multiply-add: a - c*q is a
//                         multiple of half an ulp of a / c, at most 4c of them;
//   q' = RN(q + r * y)    (fused) = RN(a / c).
// The last step is Markstein's correction.  q + r*y differs from a / c by at
// most 2^(1-p) ulp, while a / c lies at least ulp / (2c) from every rounding
// boundary: for odd c, a / c is never a midpoint, and its distance to one is
// a nonzero multiple of half an ulp divided by c; an even c reduces to an odd
// one by a power of two, exactly.  So for c < 2^(p-2) the rounding cannot
// change.  The argument needs no underflow or overflow in q and r: outside
// [lo, hi] (zero, subnormal or tiny |a|, infinities, NaN) the function
// divides.
#pragma once

#include <hip/hip_runtime.h>

namespace lms {

template <typename T>
struct CountDivRange;
template <>
struct CountDivRange<double> {
    static constexpr double lo = 0x1p-960, hi = 0x1.fffffffffffffp+1023;
};
template <>
struct CountDivRange<float> {
    static constexpr float lo = 0x1p-100f, hi = 0x1.fffffep+127f;
};

// a / c, correctly rounded; y must be RN(1/c) and 1 <= c <= 2^20.
template <typename T>
__host__ __device__ __forceinline__ T div_by_count(T a, T c, T y) {
    const T m = fabs(a);
    if (m >= CountDivRange<T>::lo && m <= CountDivRange<T>::hi) {
        const T q = a * y;
        const T r = fma(-q, c, a);
        return fma(r, y, q);
    }
    return a / c;
}

}  // namespace lms
