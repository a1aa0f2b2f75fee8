// Host construction of the packed inverse elevation table (Dong et al.,
// Sec. 3.2, Eq. (4)); the entry layout and the lookup are in rir_device.h
// (SensorTab::ebin, elev_row).  Plain C++, no HIP.
#pragma once

#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace rir {

// Order-preserving integer key of a float or double (-0 sorts just below +0).
template <typename T>
struct KeyOf;
template <>
struct KeyOf<float> {
    using U = uint32_t;
};
template <>
struct KeyOf<double> {
    using U = uint64_t;
};
template <typename T>
inline typename KeyOf<T>::U to_key(T x)
{
    using U = typename KeyOf<T>::U;
    const U sign = U(1) << (8 * sizeof(U) - 1);
    U b;
    std::memcpy(&b, &x, sizeof b);
    return (b & sign) ? ~b : (b | sign);
}
template <typename T>
inline T from_key(typename KeyOf<T>::U k)
{
    using U = typename KeyOf<T>::U;
    const U sign = U(1) << (8 * sizeof(U) - 1);
    const U b = (k & sign) ? (k & ~sign) : ~k;
    T x;
    std::memcpy(&x, &b, sizeof x);
    return x;
}

// The bin of sz exactly as the kernels compute it (elev_row in rir_device.h).
template <typename T>
inline long bin_of(T sz, T lo, T sc, T bmax)
{
#pragma clang fp contract(off)
    const T d = sz - lo;
    T f = d * sc;
    f = f >= (T)0 ? f : (T)0;
    f = f < bmax ? f : bmax;
    return (long)(int)f;
}

// Packed inverse elevation table of one level in arithmetic type T (entry
// layout in rir_device.h).  The exact lower edge a_b of every bin (the least
// T value the kernels' bin formula maps to bin b or above) is found by
// bisection over the ordered T values; then each bin lists the midpoints above
// its upper edge (c) and those strictly inside it, which must all be equal (k
// of them).  Returns false when some bin holds two distinct midpoints.
template <typename T>
inline bool build_ebin(const std::vector<double> &mu, const std::vector<double> &uoff, long nb, double lo, double hi,
                std::vector<T> &out)
{
    using U = typename KeyOf<T>::U;
    const T lo_t = (T)lo, sc_t = (T)((double)nb / (hi - lo)), bmax = (T)(nb - 1);
    const T inf = std::numeric_limits<T>::infinity();
    std::vector<U> edge(nb + 1);
    edge[0] = to_key(-inf);
    edge[nb] = to_key(inf);
    for (long b = 1; b < nb; ++b) {
        U a = to_key(-inf), z = to_key(inf);  // bin_of(a) < b <= bin_of(z)
        while (z - a > 1) {
            const U m = a + (z - a) / 2;
            if (bin_of(from_key<T>(m), lo_t, sc_t, bmax) >= b)
                z = m;
            else
                a = m;
        }
        edge[b] = z;
    }
    std::vector<T> m_t(mu.size());
    for (size_t k = 0; k < mu.size(); ++k)
        m_t[k] = (T)mu[k];
    out.assign(4 * nb, (T)0);
    for (long b = 0; b < nb; ++b) {
        const T a_lo = from_key<T>(edge[b]);
        const bool last = b == nb - 1;
        const T a_hi = from_key<T>(edge[b + 1]);
        int c = 0, k = 0;
        T mid = (T)0;
        for (size_t q = 0; q < m_t.size(); ++q) {
            const T m = m_t[q];
            if (!last && m >= a_hi) {
                ++c;
            } else if ((b == 0 || m > a_lo) && (last || m < a_hi)) {
                if (k > 0 && m != mid)
                    return false;
                mid = m;
                ++k;
            }
        }
        if (c + k > 0xffff)
            return false;
        const uint64_t ck = (uint32_t)c | ((uint32_t)(c + k) << 16);
        std::memcpy(&out[4 * b], &ck, sizeof(T) == 4 ? 4 : 8);
        out[4 * b + 1] = mid;
        out[4 * b + 2] = (T)uoff[c];
        out[4 * b + 3] = (T)uoff[c + k];
    }
    return true;
}

}  // namespace rir
