"""Exact (rational) derivation of finite-difference and AT coefficients.

Test infrastructure (oracle). Everything here is exact arithmetic on
``fractions.Fraction``.

Paper passages followed:
- Sec. 3.1, eq. taylor_series_async / eq. exp: the Taylor expansion of
  u_{i+j}^{n-l} about (i, n) in dx and dt.
- Sec. 3.1, eq. cond: the order conditions. With dt ~ dx^r, every term
  u^{(p,q)} with p + r q < d + a must vanish except (p, q) = (d, 0), whose
  coefficient must be one.
- Sec. 3.1 (derivation recipe): rank(A) vs rank(A|b) decides between a
  unique solution, no solution and infinitely many.
- Sec. 3.3 / Sec. 3.4 Example 3: the step-by-step route. First the symmetric
  synchronous central difference (eq. general_deriv_cds); then a small system
  over successive delayed time levels k, k+1, ..., k+T-1 that cancels the
  asynchrony terms (the third linear system of Example 3).

A stencil is a list of (j, l) pairs: spatial offset j and time-level delay l
(the value used is u_{i+j}^{n-l}). Coefficients returned are dimensionless:
the derivative is sum_c c_{j,l} u_{i+j}^{n-l} / dx^d.
"""
from fractions import Fraction
from math import factorial


def order_condition_terms(d, a, r):
    """The (p, q) pairs constrained by eq. cond: p + r q < d + a."""
    terms = []
    for q in range(0, d + a + 1):
        for p in range(0, d + a + 1):
            if p + r * q < d + a:
                terms.append((p, q))
    if (d, 0) not in terms:
        terms.append((d, 0))
    return terms


def condition_row(p, q, stencil):
    """Row of eq. cond for term u^{(p,q)}, divided by dx^p dt^q.

    Entry for (j, l): j^p (-l)^q / (p! q!).
    """
    den = factorial(p) * factorial(q)
    return [Fraction(j) ** p * Fraction(-l) ** q / den for (j, l) in stencil]


def rank(mat):
    """Rank of a rational matrix by Gaussian elimination."""
    m = [list(row) for row in mat]
    nrow = len(m)
    ncol = len(m[0]) if nrow else 0
    rk = 0
    for col in range(ncol):
        piv = None
        for r_ in range(rk, nrow):
            if m[r_][col] != 0:
                piv = r_
                break
        if piv is None:
            continue
        m[rk], m[piv] = m[piv], m[rk]
        for r_ in range(nrow):
            if r_ != rk and m[r_][col] != 0:
                f = m[r_][col] / m[rk][col]
                m[r_] = [x - f * y for x, y in zip(m[r_], m[rk])]
        rk += 1
    return rk


def solve_consistent(A, b):
    """Solve A c = b for a consistent system of full column rank.

    Returns (status, c): status is 'unique', 'none' or 'infinite' following the
    rank test of Sec. 3.1. ``c`` is only returned for 'unique'.
    """
    ncol = len(A[0])
    rA = rank(A)
    rAb = rank([row + [bi] for row, bi in zip(A, b)])
    if rA != rAb:
        return "none", None
    if rA < ncol:
        return "infinite", None
    # Reduce the augmented matrix and read off the solution.
    m = [list(row) + [bi] for row, bi in zip(A, b)]
    nrow = len(m)
    piv_cols = []
    rk = 0
    for col in range(ncol):
        piv = None
        for r_ in range(rk, nrow):
            if m[r_][col] != 0:
                piv = r_
                break
        if piv is None:
            continue
        m[rk], m[piv] = m[piv], m[rk]
        pv = m[rk][col]
        m[rk] = [x / pv for x in m[rk]]
        for r_ in range(nrow):
            if r_ != rk and m[r_][col] != 0:
                f = m[r_][col]
                m[r_] = [x - f * y for x, y in zip(m[r_], m[rk])]
        piv_cols.append(col)
        rk += 1
    c = [Fraction(0)] * ncol
    for i, col in enumerate(piv_cols):
        c[col] = m[i][ncol]
    return "unique", c


def derive_scheme(stencil, d, a, r):
    """Single-system derivation of Sec. 3.1 for an explicit (j, l) stencil.

    Builds eq. cond for all p + r q < d + a and solves it exactly. Returns
    (status, {(j, l): c}).
    """
    terms = order_condition_terms(d, a, r)
    A = [condition_row(p, q, stencil) for (p, q) in terms]
    b = [Fraction(1) if (p, q) == (d, 0) else Fraction(0) for (p, q) in terms]
    status, c = solve_consistent(A, b)
    if status != "unique":
        return status, None
    return status, dict(zip(stencil, c))


def central_difference(d, a):
    """Synchronous central difference taps c_{-s..s} (Sec. 3.3, eq. general_deriv_cds).

    Step one of Example 3: use the symmetric combination u_{i+j} + (-1)^d u_{i-j}
    for j = 0..s (s = a/2, d = 1 or 2) and impose the q = 0 conditions
    p < d + a. Returns the 2s+1 taps for offsets j = -s..s.
    """
    s = a // 2
    # unknowns: phi_j for j = 1..s, plus phi_0 (the centre) for even d
    js = list(range(0 if d % 2 == 0 else 1, s + 1))
    rows = []
    rhs = []
    for p in range(d + a):
        row = []
        for j in js:
            if j == 0:
                # phi_0 multiplies u_i alone: only the p = 0 term survives
                row.append(Fraction(1) if p == 0 else Fraction(0))
            else:
                # Taylor coefficient of u^{(p,0)} in u_{i+j} + (-1)^d u_{i-j}
                row.append((Fraction(j) ** p + (-1) ** d * Fraction(-j) ** p) / factorial(p))
        if all(v == 0 for v in row):
            continue
        rows.append(row)
        rhs.append(Fraction(1) if p == d else Fraction(0))
    status, phi = solve_consistent(rows, rhs)
    if status != "unique":
        raise ValueError(f"central difference d={d} a={a}: {status}")
    taps = {o: Fraction(0) for o in range(-s, s + 1)}
    for j, ph in zip(js, phi):
        if j == 0:
            taps[0] += ph
        else:
            taps[j] += ph
            taps[-j] += (-1) ** d * ph
    return [taps[o] for o in range(-s, s + 1)]


def time_level_weights(k, T):
    """Weights c_m, m = 0..T-1, over delayed levels n-k-m (Sec. 3.4 Example 3).

    The third system of Example 3: after the spatial step, the asynchrony
    terms with the same power q of dt are all equivalent, so one condition per
    q remains. Written for T levels:
        sum_m c_m = 1,   sum_m c_m (k+m)^q = 0   for q = 1..T-1.
    (Example 3 prints the T = 3 case; its rows carry constant factors
    -5 dt / 4 dx^2 and 5 dt^2 / 8 dx^2 that do not change the solution.)
    """
    k = Fraction(k)
    A = [[Fraction(1)] * T]
    b = [Fraction(1)]
    for q in range(1, T):
        A.append([(k + m) ** q for m in range(T)])
        b.append(Fraction(0))
    status, c = solve_consistent(A, b)
    if status != "unique":
        raise ValueError(f"time-level system k={k} T={T}: {status}")
    return c


def time_expanded_at_stencil(d, a, k, T, side):
    """Full (j, l) stencil of a time-expanded AT scheme at the point next to a face.

    Tables atschemes-left/right, rows (1,2,2)b, (2,2,2)b, (1,4,2), (2,4,2),
    (2,6,2): the derivative at the point adjacent to the face is
    sum_m c_m(k) * CD_a(stencil with the buffer-side taps at level n-k-m).
    side = 'left' puts the buffer points at j < 0, 'right' at j > 0.
    Returns {(j, l): coefficient}.
    """
    taps = central_difference(d, a)
    s = (len(taps) - 1) // 2
    w = time_level_weights(k, T)
    out = {}
    for m in range(T):
        for idx, c in enumerate(taps):
            j = idx - s
            buffer = (j < 0) if side == "left" else (j > 0)
            key = (j, k + m) if buffer else (j, 0)
            out[key] = out.get(key, Fraction(0)) + w[m] * c
    return {key: v for key, v in out.items() if v != 0 or key[1] == 0}


def condition_residuals(coefs, d, a, r, extra=0):
    """Evaluate eq. cond for a given stencil: returns {(p, q): value}.

    ``extra`` widens the range to p + r q < d + a + extra to expose the leading
    truncation terms.
    """
    res = {}
    for q in range(0, d + a + extra + 1):
        for p in range(0, d + a + extra + 1):
            if p + r * q < d + a + extra:
                den = factorial(p) * factorial(q)
                res[(p, q)] = sum(
                    (c * Fraction(j) ** p * Fraction(-l) ** q / den for (j, l), c in coefs.items()),
                    Fraction(0),
                )
    return res


def n_time_levels(d, a, r):
    """T = ceil((d + a) / r): successive delayed levels needed to cancel the
    asynchrony terms u^{(0,q)}, q < (d + a) / r (eq. cond with p = 0)."""
    return -(-(d + a) // r)


# Footprints of the space-expanded single-level AT schemes (Tables
# atschemes-left/right, rows (2,1,2), (1,2,2)a, (2,2,2)a): at the point next to
# a face, own points at level n on one side and buffer points at the single
# delayed level n-k on the other. Left boundary: buffer at j < 0.
_SPACE_FOOTPRINTS = {
    # (d, scheme): (own offsets, buffer offsets, a) for the left boundary
    (1, "space212"): ((1, 0), (-1, -2), 2),     # (1,2,2)a
    (1, "space222"): ((1, 0), (-1, -2), 2),     # (1,2,2)a
    (2, "space212"): ((1, 0), (-1, -2), 1),     # (2,1,2)
    (2, "space222"): ((2, 1, 0), (-1, -2, -3), 2),   # (2,2,2)a
}


def space_expanded_at_stencil(d, scheme, side):
    """Coefficients of a space-expanded AT scheme at the point next to a face.

    Solves eq. cond (Sec. 3.1, r = 2) exactly for the scheme's footprint with
    the buffer points at delay k. The solution does not depend on k >= 1 (the
    rows with q > 0 scale by powers of k), and the paper uses the same
    coefficients for every k, k = 0 included (Sec. 5.1: these schemes do not
    reduce to the central difference at k = 0). Returns {(j, 'k' or 0): c}
    with 'k' marking buffer points; side 'right' mirrors the footprint.
    """
    own, buf, a = _SPACE_FOOTPRINTS[(d, scheme)]
    sgn = 1 if side == "left" else -1
    sols = []
    for k in (1, 2, 3):
        st = [(sgn * j, 0) for j in own] + [(sgn * j, k) for j in buf]
        status, c = derive_scheme(st, d, a, 2)
        if status != "unique":
            raise ValueError(f"space-expanded d={d} {scheme}: {status}")
        sols.append([c[x] for x in st])
    if sols[0] != sols[1] or sols[0] != sols[2]:
        raise ValueError("space-expanded coefficients depend on k")
    keys = [(sgn * j, 0) for j in own] + [(sgn * j, "k") for j in buf]
    return dict(zip(keys, sols[0]))

