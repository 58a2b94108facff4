// Exact derivation of finite-difference and AT coefficients from a chosen
// stencil, and a search over stencil extents.
//
// Sec. 3.1: the Taylor expansion of u_{i+j}^{n-l} about (i, n) (eq. exp) and
// the order conditions (eq. cond): with dt ~ dx^r every term u^{(p,q)} with
// p + r q < d + a must vanish, except (p, q) = (d, 0), whose coefficient is
// one. Dividing the row of (p, q) by its common factor dx^p dt^q / (p! q!)
// leaves integer entries j^p (-l)^q and right-hand side d! on the (d, 0) row.
// The rank test of the derivation recipe: rank(A) < rank(A|b) means no
// scheme, rank(A) = rank(A|b) = unknowns a unique one, otherwise a family.
// Sec. 3.2 eq. general_deriv_at2: a stencil is a set of (point, level) pairs.
//
// Arithmetic is exact: reduced fractions of 128-bit integers, every product
// and sum checked for overflow (a stencil too large for that range is
// rejected, never rounded).

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "atfd.h"
#include "host_common.hpp"

namespace {

using i128 = __int128;

constexpr int kMaxUnknowns = 48;
constexpr int kMaxOffset = 32;
constexpr int kMaxLevel = 64;
constexpr int kMaxDeriv = 4;
constexpr int kMaxOrder = 12;

at_status derr(const char* fmt, int v = 0) {
  char buf[256];
  snprintf(buf, sizeof(buf), fmt, v);
  atfd::thread_error() = buf;
  return AT_EINVAL;
}

i128 gcd128(i128 a, i128 b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b != 0) {
    i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

struct Q {
  i128 n = 0, d = 1;  // d > 0, gcd(|n|, d) = 1
};

// Overflow-checked rational arithmetic; `ok` turns false on overflow.
struct Arith {
  bool ok = true;

  Q make(i128 n, i128 d) {
    if (d < 0) { n = -n; d = -d; }
    i128 g = gcd128(n, d);
    if (g > 1) { n /= g; d /= g; }
    Q q;
    q.n = n;
    q.d = d;
    return q;
  }
  i128 mul(i128 a, i128 b) {
    i128 r;
    if (__builtin_mul_overflow(a, b, &r)) { ok = false; return 0; }
    return r;
  }
  i128 sub(i128 a, i128 b) {
    i128 r;
    if (__builtin_sub_overflow(a, b, &r)) { ok = false; return 0; }
    return r;
  }
  Q mulq(const Q& x, const Q& y) {
    if (x.n == 0 || y.n == 0) return Q();
    // cross-reduce first to keep the magnitudes down
    i128 g1 = gcd128(x.n, y.d), g2 = gcd128(y.n, x.d);
    return make(mul(x.n / g1, y.n / g2), mul(x.d / g2, y.d / g1));
  }
  Q divq(const Q& x, const Q& y) {
    Q inv;
    inv.n = y.d;
    inv.d = y.n;
    if (inv.d < 0) {
      inv.n = sub(0, inv.n);
      inv.d = sub(0, inv.d);
    }
    return mulq(x, inv);
  }
  Q subq(const Q& x, const Q& y) {
    if (y.n == 0) return x;
    i128 g = gcd128(x.d, y.d);
    i128 l = mul(x.d / g, y.d);
    i128 a = mul(x.n, l / x.d), b = mul(y.n, l / y.d);
    return make(sub(a, b), l);
  }
  Q power(i128 base, int e) {
    i128 r = 1;
    for (int i = 0; i < e; ++i) r = mul(r, base);
    Q q;
    q.n = r;
    return q;
  }
};

// The (p, q) terms constrained by eq. cond for (d, a, r): p + r q < d + a.
std::vector<std::pair<int, int>> cond_terms(int d, int a, int r) {
  std::vector<std::pair<int, int>> t;
  for (int q = 0; r * q < d + a; ++q)
    for (int p = 0; p + r * q < d + a; ++p) t.emplace_back(p, q);
  return t;
}

struct Result {
  int status = AT_DERIVE_NONE;
  int n_cond = 0, rank_a = 0, rank_ab = 0;
  std::vector<Q> c;   // a solution when consistent (free unknowns zero)
};

// Builds eq. cond for the stencil and reduces [A | b] to row-echelon form.
// Returns false on overflow.
bool derive(int d, int a, int r, int n, const int* j, const int* l, Result& out) {
  Arith ar;
  auto terms = cond_terms(d, a, r);
  const int m = static_cast<int>(terms.size());
  std::vector<std::vector<Q>> M(m, std::vector<Q>(n + 1));
  i128 dfact = 1;
  for (int i = 2; i <= d; ++i) dfact *= i;
  for (int row = 0; row < m; ++row) {
    const int p = terms[row].first, q = terms[row].second;
    for (int col = 0; col < n; ++col)
      M[row][col] = ar.mulq(ar.power(j[col], p), ar.power(-static_cast<i128>(l[col]), q));
    M[row][n].n = (p == d && q == 0) ? dfact : 0;
  }
  if (!ar.ok) return false;
  // Gauss-Jordan elimination over the rationals.
  std::vector<int> piv_col;
  int rk = 0;
  for (int col = 0; col <= n && rk < m; ++col) {
    int piv = -1;
    for (int row = rk; row < m; ++row)
      if (M[row][col].n != 0) { piv = row; break; }
    if (piv < 0) continue;
    std::swap(M[rk], M[piv]);
    const Q pv = M[rk][col];
    for (int c2 = col; c2 <= n; ++c2) M[rk][c2] = ar.divq(M[rk][c2], pv);
    for (int row = 0; row < m; ++row) {
      if (row == rk || M[row][col].n == 0) continue;
      const Q f = M[row][col];
      for (int c2 = col; c2 <= n; ++c2) M[row][c2] = ar.subq(M[row][c2], ar.mulq(f, M[rk][c2]));
    }
    if (!ar.ok) return false;
    piv_col.push_back(col);
    ++rk;
  }
  out.n_cond = m;
  out.rank_ab = rk;
  out.rank_a = rk;
  if (!piv_col.empty() && piv_col.back() == n) out.rank_a = rk - 1;  // the b column took a pivot
  out.c.assign(n, Q());
  if (out.rank_a < out.rank_ab) {
    out.status = AT_DERIVE_NONE;
    return true;
  }
  out.status = out.rank_a == n ? AT_DERIVE_UNIQUE : AT_DERIVE_INFINITE;
  for (int i = 0; i < out.rank_a; ++i) out.c[piv_col[i]] = M[i][n];
  return true;
}

bool fits_i64(const Q& q) {
  return q.n >= INT64_MIN && q.n <= INT64_MAX && q.d <= INT64_MAX;
}

at_status check_dar(int d, int a, int r) {
  if (d < 1 || d > kMaxDeriv) return derr("derivative order d must be 1..%d", kMaxDeriv);
  if (a < 1 || a > kMaxOrder) return derr("accuracy a must be 1..%d", kMaxOrder);
  if (r < 1 || r > 4) return derr("dt ~ dx^r needs r in 1..%d", 4);
  return AT_OK;
}

at_status derive_checked(int d, int a, int r, int n, const int* j, const int* l, Result& res) {
  if (!derive(d, a, r, n, j, l, res))
    return derr("exact arithmetic overflow: stencil offsets, levels or order too large (%d unknowns)", n);
  for (const Q& q : res.c)
    if (!fits_i64(q)) return derr("a coefficient does not fit 64-bit numerator/denominator (%d unknowns)", n);
  return AT_OK;
}

void store(const Result& res, int a_used, int n, int64_t* num, int64_t* den, at_derivation* info) {
  for (int i = 0; i < n; ++i) {
    num[i] = static_cast<int64_t>(res.c[i].n);
    den[i] = static_cast<int64_t>(res.c[i].d);
  }
  info->status = res.status;
  info->order = a_used;
  info->n_cond = res.n_cond;
  info->n_unknown = n;
  info->rank_a = res.rank_a;
  info->rank_ab = res.rank_ab;
}

}  // namespace

extern "C" {

at_status at_derive_scheme(int32_t d, int32_t a, int32_t r, int32_t n, const int32_t* j, const int32_t* l,
                           int64_t* num, int64_t* den, at_derivation* info) {
  if (at_status st = check_dar(d, a, r)) return st;
  if (n < 1 || n > kMaxUnknowns) return derr("stencil size must be 1..%d", kMaxUnknowns);
  if (!j || !l || !num || !den || !info) return derr("null pointer argument");
  for (int i = 0; i < n; ++i) {
    if (j[i] < -kMaxOffset || j[i] > kMaxOffset) return derr("point offsets must lie in [-%d, %d]", kMaxOffset);
    if (l[i] < 0 || l[i] > kMaxLevel) return derr("time-level delays must lie in [0, %d]", kMaxLevel);
    for (int i2 = 0; i2 < i; ++i2)
      if (j[i2] == j[i] && l[i2] == l[i]) return derr("stencil entry %d repeats an earlier (j, l) pair", i);
  }
  Result res;
  if (at_status st = derive_checked(d, a, r, n, j, l, res)) return st;
  store(res, a, n, num, den, info);
  return AT_OK;
}

at_status at_search_scheme(int32_t d, int32_t a, int32_t r, int32_t s_min, int32_t with_centre, int32_t k,
                           int32_t T, int32_t side, int32_t max_extent, int32_t cap, int32_t* n_out,
                           int32_t* j_out, int32_t* l_out, int64_t* num, int64_t* den, at_derivation* info) {
  if (at_status st = check_dar(d, a, r)) return st;
  if (s_min < 0 || s_min > kMaxOffset) return derr("s_min must be 0..%d", kMaxOffset);
  if (T < 1 || k < 0 || k + T - 1 > kMaxLevel) return derr("levels k..k+T-1 must lie in [0, %d]", kMaxLevel);
  if (side != -1 && side != 1) return derr("side must be +1 (buffer on the right) or -1 (left)");
  if (max_extent < 1 || max_extent > kMaxOffset) return derr("max_extent must be 1..%d", kMaxOffset);
  if (!n_out || !j_out || !l_out || !num || !den || !info) return derr("null pointer argument");
  *n_out = 0;
  info->status = AT_DERIVE_NONE;
  info->order = a;
  info->n_cond = info->n_unknown = info->rank_a = info->rank_ab = 0;
  std::vector<int> jj, ll;
  // Accepts a unique scheme that uses at least one buffer point.
  auto accept = [&](const std::vector<int>& js, const std::vector<int>& ls, Result& res, int a_used,
                    bool& done) -> at_status {
    const int n = static_cast<int>(js.size());
    bool uses_buffer = false;
    for (int i = 0; i < n; ++i) uses_buffer |= (js[i] >= 1 && res.c[i].n != 0);
    if (res.status != AT_DERIVE_UNIQUE || !uses_buffer) return AT_OK;
    if (n > cap) return derr("output capacity too small: the scheme has %d entries", n);
    const bool flip = side < 0 && (d & 1);
    for (int i = 0; i < n; ++i) {
      j_out[i] = side * js[i];
      l_out[i] = ls[i];
      if (flip) res.c[i].n = -res.c[i].n;
    }
    store(res, a_used, n, num, den, info);
    *n_out = n;
    done = true;
    return AT_OK;
  };
  for (int s_max = 1; s_max <= max_extent; ++s_max) {
    jj.clear();
    ll.clear();
    for (int x = -s_min; x <= 0; ++x)
      if (x != 0 || with_centre) { jj.push_back(x); ll.push_back(0); }
    for (int x = 1; x <= s_max; ++x)
      for (int t = 0; t < T; ++t) { jj.push_back(x); ll.push_back(k + t); }
    const int n = static_cast<int>(jj.size());
    if (n > kMaxUnknowns) break;
    bool done = false;
    Result res;
    if (at_status st = derive_checked(d, a, r, n, jj.data(), ll.data(), res)) return st;
    if (at_status st = accept(jj, ll, res, a, done)) return st;
    if (done) return AT_OK;
    if (res.status != AT_DERIVE_INFINITE) continue;  // no scheme here: widen the stencil
    // Recipe step 3, a consistent system with a family of solutions: first
    // impose further conditions (higher accuracy) while the family persists.
    bool determined = false;
    for (int a2 = a + 1; a2 <= kMaxOrder && !determined; ++a2) {
      Result r2;
      // conditions beyond exact 128-bit range end the escalation (the
      // reduction below may still find a scheme)
      if (!derive(d, a2, r, n, jj.data(), ll.data(), r2)) break;
      bool fits = true;
      for (const Q& q : r2.c) fits = fits && fits_i64(q);
      if (!fits) break;
      if (r2.status == AT_DERIVE_INFINITE) continue;
      determined = true;
      if (at_status st = accept(jj, ll, r2, a2, done)) return st;
      if (done) return AT_OK;
    }
    // ... else reduce the system: drop one buffer entry, the oldest level of
    // the farthest point first, and keep the first unique scheme.
    std::vector<int> order;
    for (int i = 0; i < n; ++i)
      if (jj[i] >= 1) order.push_back(i);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      return ll[x] != ll[y] ? ll[x] > ll[y] : jj[x] > jj[y];
    });
    for (int drop : order) {
      std::vector<int> j2, l2;
      for (int i = 0; i < n; ++i)
        if (i != drop) { j2.push_back(jj[i]); l2.push_back(ll[i]); }
      Result r3;
      if (at_status st = derive_checked(d, a, r, n - 1, j2.data(), l2.data(), r3)) return st;
      if (at_status st = accept(j2, l2, r3, a, done)) return st;
      if (done) return AT_OK;
    }
  }
  return AT_OK;
}

}  // extern "C"
