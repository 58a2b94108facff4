"""Scheme derivation in the library (at_derive_scheme, at_search_scheme)
against the oracle's exact derivation and the schemes printed in the paper.

Host code only: these run without a GPU. The oracle solves eq. cond with its
own Fraction elimination; the library with 128-bit exact rationals. Results
must agree exactly: status, rank(A), rank(A|b) and every coefficient.
"""
import json
import os
import random
from fractions import Fraction

import pytest

from oracle import coeffs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_schemes.json")))


def _derive():
    if not os.path.exists(os.path.join(ROOT, "paper_1702_00496_amd", "libatfd.so")):
        pytest.fail("libatfd.so is not built (python -m paper_1702_00496_amd.build)")
    from paper_1702_00496_amd import derive
    return derive


def _oracle_ranks(stencil, d, a, r):
    terms = coeffs.order_condition_terms(d, a, r)
    A = [coeffs.condition_row(p, q, stencil) for (p, q) in terms]
    b = [Fraction(1) if t == (d, 0) else Fraction(0) for t in terms]
    return len(terms), coeffs.rank(A), coeffs.rank([row + [bi] for row, bi in zip(A, b)]), A, b


def _random_stencils(seed, count):
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        d = rng.choice((1, 2))
        a = rng.choice((1, 2, 3, 4))
        r = rng.choice((1, 2))
        n = rng.randint(2, 9)
        pairs = set()
        while len(pairs) < n:
            j = rng.randint(-4, 4)
            l = 0 if j <= 0 and rng.random() < 0.7 else rng.randint(0, 5)
            pairs.add((j, l))
        out.append((sorted(pairs), d, a, r))
    return out


def test_random_stencils_match_the_oracle_exactly():
    derive = _derive()
    seen = {"unique": 0, "none": 0, "infinite": 0}
    for stencil, d, a, r in _random_stencils(1702, 400):
        status, c, info = derive.derive_scheme(stencil, d, a, r)
        ostatus, oc = coeffs.derive_scheme(stencil, d, a, r)
        ncond, ra, rab, A, b = _oracle_ranks(stencil, d, a, r)
        assert status == ostatus, (stencil, d, a, r)
        assert (info["n_cond"], info["rank_a"], info["rank_ab"]) == (ncond, ra, rab)
        seen[status] += 1
        if status == "unique":
            assert c == oc
        elif status == "infinite":
            # one member of the family: it satisfies every condition
            vec = [c[x] for x in stencil]
            for row, bi in zip(A, b):
                assert sum(x * y for x, y in zip(row, vec)) == bi
    assert min(seen.values()) >= 20, seen


def test_example1_nonuniform_delays_and_its_singular_set():
    """Sec. 3.4 Example 1, eq. ex1-0: coefficients ((-4k1+k2), 3k1, -k2, k1) /
    (2 (3k1 - k2)); the system is singular on 3 k1 = k2, and at k1 = k2 = 0 it
    has no scheme (eq. ex1-1 is used there)."""
    derive = _derive()
    for k1 in range(0, 6):
        for k2 in range(0, 6):
            st = [(-1, 0), (0, 0), (1, k1), (2, k2)]
            status, c, info = derive.derive_scheme(st, 1, 2, 2)
            if 3 * k1 == k2:
                assert status != "unique" and info["rank_a"] < 4
                continue
            den = 2 * (3 * k1 - k2)
            assert status == "unique"
            assert [c[x] for x in st] == [Fraction(-4 * k1 + k2, den), Fraction(3 * k1, den),
                                          Fraction(-k2, den), Fraction(k1, den)]


def test_example2_printed_scheme_from_derive_and_search():
    """Sec. 3.4 Example 2, eq. ex2-1: the 11-point one-sided scheme for d = 2,
    a = 4, r = 1 with a uniform delay on the right; the search with interior
    extent 5 and no centre point finds it first at s_max = 6."""
    derive = _derive()
    g = GOLD["example2"]
    want = [Fraction(v, g["den"]) for v in g["num"]]
    for k in (1, 2, 5):
        st = [(j, 0) for j in g["stencil_sync"]] + [(j, k) for j in g["stencil_delayed"]]
        status, c, info = derive.derive_scheme(st, g["d"], g["a"], g["r"])
        assert status == "unique" and info["n_cond"] == 21 and info["rank_a"] == 11, g["cite"]
        assert [c[x] for x in st] == want
        found, info = derive.search_scheme(g["d"], g["a"], g["r"], s_min=5, k=k, with_centre=False)
        assert found is not None and info["order"] == 4
        assert sorted(found) == sorted(st) and [found[x] for x in st] == want


def test_search_recovers_example1_uniform_scheme():
    derive = _derive()
    g = GOLD["example1_uniform"]
    for k in (1, 3):
        found, info = derive.search_scheme(1, 2, 2, s_min=1, k=k)
        st = [(j, k if l == "k" else l) for j, l in g["stencil"]]
        assert sorted(found) == sorted(st), g["cite"]
        assert [found[x] for x in st] == [Fraction(v, g["den"]) for v in g["num"]]


@pytest.mark.parametrize("name", sorted(k for k in GOLD["space_expanded"] if not k.startswith("_")))
def test_space_expanded_table_rows(name):
    derive = _derive()
    g = GOLD["space_expanded"][name]
    for k in (1, 2, 4):
        st = [(j, k if l == "k" else l) for j, l in g["stencil"]]
        status, c, _ = derive.derive_scheme(st, g["d"], g["a"], g["r"])
        assert status == "unique"
        assert [c[x] for x in st] == [Fraction(v, g["den"]) for v in g["num"]], g["cite"]


@pytest.mark.parametrize("d,a", [(1, 2), (2, 2), (2, 4)])
@pytest.mark.parametrize("side", ["left", "right"])
def test_search_with_T_levels_gives_the_time_expanded_rows(d, a, side):
    """Interior extent s = a/2 with the centre and T successive delayed levels
    (T from the p = 0 rows of eq. cond): where the CD footprint determines the
    system, the search returns the time-expanded table rows (1,2,2)b, (2,2,2)b,
    (2,4,2) of the oracle at every delay."""
    derive = _derive()
    s = a // 2
    T = coeffs.n_time_levels(d, a, 2)
    for k in (1, 2, 3):
        found, info = derive.search_scheme(d, a, 2, s_min=s, k=k, T=T, side=side)
        want = coeffs.time_expanded_at_stencil(d, a, k, T, side)
        assert found is not None and info["status"] == "unique"
        assert {x: v for x, v in found.items() if v != 0} == {x: v for x, v in want.items() if v != 0}
        assert max(abs(j) for j, _ in found) == s


@pytest.mark.parametrize("d,a", [(1, 4), (2, 6)])
def test_time_expanded_rows_are_members_of_a_family_and_the_search_reduces_it(d, a):
    """(1,4,2) and (2,6,2): on the full CD footprint with T levels the system
    is consistent but rank deficient by one; the table row (the structured
    member of Sec. 3.3) solves it, and the search's reduced stencil (one
    buffer entry fewer) is a unique scheme of the same accuracy."""
    derive = _derive()
    s = a // 2
    T = coeffs.n_time_levels(d, a, 2)
    for k in (1, 2):
        full = [(j, 0) for j in range(-s, 1)] + [(j, k + t) for j in range(1, s + 1) for t in range(T)]
        status, member, info = derive.derive_scheme(full, d, a, 2)
        assert status == "infinite" and info["rank_a"] == info["rank_ab"] == len(full) - 1
        row = coeffs.time_expanded_at_stencil(d, a, k, T, "right")
        res = coeffs.condition_residuals(row, d, a, 2)
        assert all(v == (1 if pq == (d, 0) else 0) for pq, v in res.items())
        found, info = derive.search_scheme(d, a, 2, s_min=s, k=k, T=T)
        assert found is not None and len(found) == len(full) - 1 and info["order"] == a
        assert (s, k + T - 1) not in found       # the oldest level of the farthest point went first
        assert coeffs.derive_scheme(sorted(found), d, a, 2) == ("unique", found)


def test_search_result_is_the_smallest_extent():
    """Brute force with the oracle: no smaller buffer extent gives a scheme
    (at the requested or any higher accuracy reached through the recipe)."""
    derive = _derive()
    for d, a, r, s_min, k, T, centre in ((2, 4, 1, 5, 2, 1, False), (1, 2, 2, 1, 2, 1, True),
                                         (2, 2, 2, 2, 1, 1, True), (1, 4, 2, 2, 3, 1, True),
                                         (2, 4, 2, 2, 2, 2, True)):
        found, info = derive.search_scheme(d, a, r, s_min=s_min, k=k, T=T, with_centre=centre)
        assert found is not None
        s_max = max(j for j, _ in found)
        own = [(j, 0) for j in range(-s_min, 1) if j != 0 or centre]
        for smaller in range(1, s_max):
            st = own + [(j, k + t) for j in range(1, smaller + 1) for t in range(T)]
            for a2 in range(a, 13):
                status, c = coeffs.derive_scheme(st, d, a2, r)
                if status == "infinite":
                    continue
                assert status == "none" or all(c[x] == 0 for x in st if x[0] >= 1), (d, a, smaller, a2)
                break
        # and the result satisfies eq. cond at the accuracy reported
        res = coeffs.condition_residuals(found, d, info["order"], r)
        assert all(v == (1 if pq == (d, 0) else 0) for pq, v in res.items())


def test_infinite_family_raises_the_accuracy():
    """Recipe step 3: the symmetric 5-point synchronous stencil with a = 2 has
    a family of first-derivative schemes; imposing further conditions gives the
    unique CD4, reported with accuracy 4."""
    derive = _derive()
    st = [(j, 0) for j in range(-2, 3)]
    status, c, info = derive.derive_scheme(st, 1, 2, 2)
    assert status == "infinite" and info["rank_a"] == info["rank_ab"] < 5
    status, c, info = derive.derive_scheme(st, 1, 4, 2)
    assert status == "unique"
    cd4 = coeffs.central_difference(1, 4)
    assert [c[(j, 0)] for j in range(-2, 3)] == cd4


def test_derivation_rejects_bad_arguments_and_overflow():
    derive = _derive()
    from paper_1702_00496_amd import ATError
    with pytest.raises(ATError, match="repeats"):
        derive.derive_scheme([(0, 0), (1, 1), (0, 0)], 1, 2, 2)
    with pytest.raises(ATError, match="derivative order"):
        derive.derive_scheme([(0, 0), (1, 0)], 0, 2, 2)
    with pytest.raises(ATError, match="offsets"):
        derive.derive_scheme([(0, 0), (40, 0)], 1, 2, 2)
    with pytest.raises(ATError, match="overflow|64-bit"):
        derive.derive_scheme([(j, (j * 37) % 65) for j in range(-32, 8)], 4, 12, 1)


def test_search_rejects_bad_arguments_and_reports_no_scheme():
    derive = _derive()
    from paper_1702_00496_amd import ATError
    with pytest.raises(ATError, match="side"):
        derive.search_scheme(1, 2, 2, s_min=1, k=1, side="up")
    with pytest.raises(ATError, match="levels"):
        derive.search_scheme(1, 2, 2, s_min=1, k=-1)
    with pytest.raises(ATError, match="s_min"):
        derive.search_scheme(1, 2, 2, s_min=40, k=1)
    with pytest.raises(ATError, match="max_extent"):
        derive.search_scheme(1, 2, 2, s_min=1, k=1, max_extent=0)
    # order 12 first derivative with one interior point and one buffer point
    # per extent: the buffer alone never satisfies the conditions up to 2 points
    found, info = derive.search_scheme(1, 12, 1, s_min=0, k=1, with_centre=False, max_extent=2)
    assert found is None and info["status"] == "none"


def test_search_left_side_is_the_mirror_image():
    """side='left' puts the buffer at j < 0: j -> -j, coefficients times (-1)^d,
    and the mirrored stencil is again the oracle's unique solution."""
    derive = _derive()
    for d, a in ((1, 2), (2, 2), (2, 4)):
        right, _ = derive.search_scheme(d, a, 2, s_min=a // 2, k=2, T=coeffs.n_time_levels(d, a, 2))
        left, _ = derive.search_scheme(d, a, 2, s_min=a // 2, k=2, T=coeffs.n_time_levels(d, a, 2), side="left")
        assert left == {(-j, l): (-1) ** d * c for (j, l), c in right.items()}
        assert coeffs.derive_scheme(sorted(left), d, a, 2) == ("unique", left)
