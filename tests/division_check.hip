// CPU check of div_by_count (the sweep kernels' quotient) against IEEE
// division, bit for bit: counts 1..16 and some larger ones, random bit
// patterns over every exponent, coordinate-like values, and the edges of the
// range where the function switches to division.  Built by hipcc and run on
// the host only; exit status 0 when every case agrees.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "lms_divide.hpp"

template <typename T, typename U>
long check(long per_count, uint64_t seed) {
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> unit(-4.0, 4.0);
    const T lo = lms::CountDivRange<T>::lo, hi = lms::CountDivRange<T>::hi;
    const T eps = std::numeric_limits<T>::epsilon();
    std::vector<T> special = {T(0), -T(0), std::numeric_limits<T>::denorm_min(), std::numeric_limits<T>::min(),
                              lo, lo * (T(1) - eps), lo * (T(1) + eps), hi, -hi, std::numeric_limits<T>::infinity(),
                              -std::numeric_limits<T>::infinity(), T(1), T(3), T(0.1), T(1) - eps, T(2) - 2 * eps};
    const int counts[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 31, 100, 1000, 1 << 20};
    long bad = 0, n = 0;
    for (int ci : counts) {
        const T c = T(ci), y = T(1) / c;
        auto one = [&](T a) {
            const T got = lms::div_by_count(a, c, y), want = a / c;
            ++n;
            if (std::isnan(want) ? !std::isnan(got) : std::memcmp(&got, &want, sizeof(T)) != 0) {
                if (bad < 8) std::printf("c=%d a=%a: %a, division %a\n", ci, double(a), double(got), double(want));
                ++bad;
            }
        };
        for (T a : special) {
            one(a);
            one(-a);
        }
        for (long i = 0; i < per_count; ++i) {
            U bits = U(g());
            T a;
            std::memcpy(&a, &bits, sizeof(T));
            one(a);
            one(T(unit(g)));
            one(T(ci) * T(unit(g)));  // sums of about c coordinates
        }
    }
    std::printf("%s: %ld cases, %ld differ\n", sizeof(T) == 8 ? "float64" : "float32", n, bad);
    return bad;
}

int main() {
    const long bad = check<double, uint64_t>(400000, 1) + check<float, uint32_t>(400000, 2);
    return bad == 0 ? 0 : 1;
}
