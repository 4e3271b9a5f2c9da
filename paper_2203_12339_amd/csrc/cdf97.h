// CDF 9/7 biorthogonal wavelet (the 9/7 filter pair of Sec. 5) in the
// lifting form of Daubechies and Sweldens, as used by JPEG 2000: two
// predict/update pairs and a final scaling.  Scaled here so that the
// low-pass has DC gain sqrt(2) and the high-pass Nyquist gain sqrt(2)
// (near-orthonormal, so coefficient energy tracks signal energy).
//
// One analysis level on x[0..n), n >= 8, even samples low / odd samples high,
// whole-sample symmetric ends (x[-1] = x[1], x[n] = x[n-2]):
//   odd  += A (left + right);  even += B (left + right)
//   odd  += G (left + right);  even += D (left + right)
//   low[i] = x[2i] * ZLO, high[i] = x[2i+1] * ZHI
// and the inverse runs the same steps backwards with opposite signs.
// Levels repeat on the low band while it has at least 8 entries (or for a
// requested count); coefficients are laid out coarse to fine
//   [ low_J, high_J, high_{J-1}, ..., high_1 ].
#pragma once

#if defined(__HIP__)
#define TLT_HD __host__ __device__
#else
#define TLT_HD
#endif

namespace tlt {
namespace cdf97 {

constexpr double A = -1.586134342059924;
constexpr double B = -0.052980118572961;
constexpr double G = 0.882911075530934;
constexpr double D = 0.443506852043971;
constexpr double KS = 1.230174104914001;
constexpr double SQRT2 = 1.4142135623730950488;
constexpr double ZLO = SQRT2 / KS;   // low-band scale
constexpr double ZHI = KS / SQRT2;   // high-band scale
constexpr int MIN_SPLIT = 8;
constexpr int MAX_LEVELS = 32;

// symmetric neighbours of sample i in a list of n >= 2
TLT_HD inline int left_of(int i) { return i > 0 ? i - 1 : 1; }
TLT_HD inline int right_of(int i, int n) { return i + 1 < n ? i + 1 : i - 1; }

}  // namespace cdf97
}  // namespace tlt
