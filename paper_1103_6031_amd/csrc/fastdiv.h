// Division by a run-time constant with a multiply and a shift (round-up method,
// Granlund & Montgomery 1994): for 1 <= d < 2^31 and 0 <= n < 2^31,
//   s = ceil(log2 d),  m = floor(2^32 (2^s - d) / d) + 1,  n / d = (mulhi32(n, m) + n) >> s.
// The constants are computed once on the host; kernels then split a linear cell index into
// coordinates without integer division instructions.
#pragma once

#if defined(__HIPCC__)
#define MGIC_HD __host__ __device__
#else
#define MGIC_HD
#endif

namespace mgic {

struct FastDiv {
    unsigned d = 1, m = 1, s = 0;

    FastDiv() = default;
    MGIC_HD explicit FastDiv(unsigned dd) : d(dd) {
        s = 0;
        while ((1u << s) < d) ++s;
        m = (unsigned)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    }
    MGIC_HD unsigned div(unsigned n) const {
#if defined(__HIP_DEVICE_COMPILE__)
        const unsigned t = __umulhi(n, m);
#else
        const unsigned t = (unsigned)(((unsigned long long)n * m) >> 32);
#endif
        return (t + n) >> s;
    }
    MGIC_HD unsigned mod(unsigned n) const { return n - div(n) * d; }
};

}  // namespace mgic
