// Host-side helpers shared by the single-problem and the ensemble front ends.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

namespace atfd {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Text of the calling thread's most recent failure (at_last_error(NULL)).
std::string& thread_error();

// Integer-only cumulative thresholds floor(2^53 * W_j / W_total) of the
// delay bins (the generator in include/atfd.h).
inline bool make_thresholds(int L, const uint32_t* weights, uint64_t* thr) {
  unsigned __int128 total = 0;
  for (int j = 0; j < L; ++j) total += weights ? weights[j] : 1u;
  if (total == 0) return false;
  unsigned __int128 cum = 0;
  for (int j = 0; j < L; ++j) {
    cum += weights ? weights[j] : 1u;
    thr[j] = static_cast<uint64_t>((cum << 53) / total);
  }
  return true;
}

// Central-difference taps of Sec. 2 eq. general_deriv (the synchronous parts
// of Tables atschemes-left/right and the textbook sixth-order first
// derivative), indexed o = -s..s.
inline bool cd_taps(int d, int order, double* t) {
  static const double d1_2[] = {-0.5, 0.0, 0.5};
  static const double d1_4[] = {1.0 / 12, -8.0 / 12, 0.0, 8.0 / 12, -1.0 / 12};
  static const double d1_6[] = {-1.0 / 60, 9.0 / 60, -45.0 / 60, 0.0, 45.0 / 60, -9.0 / 60, 1.0 / 60};
  static const double d2_2[] = {1.0, -2.0, 1.0};
  static const double d2_4[] = {-1.0 / 12, 16.0 / 12, -30.0 / 12, 16.0 / 12, -1.0 / 12};
  static const double d2_6[] = {2.0 / 180, -27.0 / 180, 270.0 / 180, -490.0 / 180, 270.0 / 180, -27.0 / 180, 2.0 / 180};
  const double* src = nullptr;
  if (d == 1) src = order == 2 ? d1_2 : order == 4 ? d1_4 : order == 6 ? d1_6 : nullptr;
  if (d == 2) src = order == 2 ? d2_2 : order == 4 ? d2_4 : order == 6 ? d2_6 : nullptr;
  if (!src) return false;
  for (int i = 0; i <= order; ++i) t[i] = src[i];
  return true;
}

// Taps of the space-expanded single-level schemes at the point next to a low
// face, o = -3..3 (Tables atschemes-left/right; the right-boundary rows are
// the mirror images): first derivative (1,2,2)a, second derivative (2,1,2)
// (scheme 1) or (2,2,2)a (scheme 2). Offsets o < 0 are the buffer points at
// the delayed level. The printed left (1,2,2)a row has -U_{i-1} where the
// order conditions, and the mirror of the right row, give +U_{i-1}.
inline bool space_taps(int d, int scheme, double* t) {
  static const double d1_122a[7] = {0.0, -0.25, 0.25, -0.75, 0.75, 0.0, 0.0};
  static const double d2_212[7] = {0.0, 0.5, -0.5, -0.5, 0.5, 0.0, 0.0};
  static const double d2_222a[7] = {1.0 / 3, -2.0 / 3, 1.0 / 3, 2.0 / 3, -4.0 / 3, 2.0 / 3, 0.0};
  const double* src = nullptr;
  if (d == 1 && (scheme == 1 || scheme == 2)) src = d1_122a;
  if (d == 2 && scheme == 1) src = d2_212;
  if (d == 2 && scheme == 2) src = d2_222a;
  if (!src) return false;
  for (int i = 0; i < 7; ++i) t[i] = src[i];
  return true;
}

}  // namespace atfd
