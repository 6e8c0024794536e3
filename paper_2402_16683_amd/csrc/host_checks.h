// Host-side argument checks of the ABI that need no device: plain C++, also compiled
// on its own by the CPU tests.
#ifndef ICR_HOST_CHECKS_H
#define ICR_HOST_CHECKS_H

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace icr {

inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return na && nb && pa < pb + nb && pb < pa + na;
}

inline int64_t floor_div(int64_t a, int64_t b) { return a / b - ((a % b != 0) && ((a < 0) != (b < 0))); }

// Do the batched views {a + i*sa + [0, na)} and {b + j*sb + [0, nb)}, 0 <= i, j < batch
// (all in bytes), share a byte? Exact when both views have the same stride and rows no
// longer than it (interleaved per-level slices of one workspace); otherwise the bounding
// ranges decide, which may reject views that only interleave.
inline bool overlaps_batched(const void* a, int64_t sa, int64_t na, const void* b, int64_t sb, int64_t nb,
                             int64_t batch) {
  if (na <= 0 || nb <= 0 || batch <= 0) return false;
  if (!overlaps(a, size_t((batch - 1) * sa + na), b, size_t((batch - 1) * sb + nb))) return false;
  if (batch == 1 || sa != sb || na > sa || nb > sb) return true;
  // rows i of a and j of b meet iff -nb < d + k*s < na with k = j - i, |k| < batch
  const int64_t d = static_cast<const char*>(b) - static_cast<const char*>(a), st = sa;
  const int64_t kmin = floor_div(-nb - d, st) + 1;
  const int64_t kmax = -floor_div(d - na, st) - 1;   // ceil((na - d) / st) - 1
  return std::max(kmin, -(batch - 1)) <= std::min(kmax, batch - 1);
}

}  // namespace icr

#endif  // ICR_HOST_CHECKS_H
