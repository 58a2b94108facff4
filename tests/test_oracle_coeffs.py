"""Pins of the oracle's coefficient derivation against what the paper prints.

Fixture: tests/golden/paper_schemes.json (each entry cites its passage).
"""
import json
import os
from fractions import Fraction

import pytest

from oracle import coeffs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_schemes.json")))


@pytest.mark.parametrize("name", sorted(GOLD["central_differences"]))
def test_central_difference_matches_printed_taps(name):
    g = GOLD["central_differences"][name]
    d = int(name[1])
    a = int(name.split("_a")[1])
    got = coeffs.central_difference(d, a)
    want = [Fraction(v, g["den"]) for v in g["num"]]
    assert got == want, g["cite"]


def test_cd6_first_derivative_satisfies_order_conditions():
    """CD6 D1 is not printed; eq. cond with l = 0 pins it: exact for p < 7."""
    taps = coeffs.central_difference(1, 6)
    st = {(j, 0): c for j, c in zip(range(-3, 4), taps)}
    res = coeffs.condition_residuals(st, 1, 6, 2)
    for (p, q), v in res.items():
        assert v == (1 if (p, q) == (1, 0) else 0), (p, q)
    # the next term is non-zero: sixth order, not more
    assert coeffs.condition_residuals(st, 1, 6, 2, extra=1)[(7, 0)] != 0


@pytest.mark.parametrize("T", [2, 3, 4])
def test_time_level_weights_match_printed_polynomials(T):
    g = GOLD["time_level_weights"][f"T{T}"]
    for k in range(0, 9):
        got = coeffs.time_level_weights(k, T)
        want = [Fraction(sum(c * k ** i for i, c in enumerate(poly)), den)
                for poly, den in zip(g["poly"], g["den"])]
        assert got == want, (k, g["cite"])


def test_time_level_weights_reduce_to_synchronous_at_k0():
    """Sec. 3.4 Example 3: with k = 0 the AT scheme is the standard CD."""
    for T in (1, 2, 3, 4):
        assert coeffs.time_level_weights(0, T) == [1] + [0] * (T - 1)


def test_example2_one_sided_scheme():
    g = GOLD["example2"]
    for k in (1, 2, 5):
        st = [(j, 0) for j in g["stencil_sync"]] + [(j, k) for j in g["stencil_delayed"]]
        status, c = coeffs.derive_scheme(st, g["d"], g["a"], g["r"])
        assert status == "unique"
        assert [c[x] for x in st] == [Fraction(v, g["den"]) for v in g["num"]], g["cite"]


def test_example1_uniform_and_nonuniform_delays():
    g = GOLD["example1_uniform"]
    for k in (1, 2, 3):
        st = [(-1, 0), (0, 0), (1, k), (2, k)]
        status, c = coeffs.derive_scheme(st, 1, 2, 2)
        assert status == "unique"
        assert [c[x] for x in st] == [Fraction(v, g["den"]) for v in g["num"]], g["cite"]
    # eq. ex1-0: coefficients ((-4k1+k2), 3k1, -k2, k1) / (2 (3k1 - k2)); singular at 3k1 = k2
    for k1 in range(0, 4):
        for k2 in range(0, 4):
            st = [(-1, 0), (0, 0), (1, k1), (2, k2)]
            status, c = coeffs.derive_scheme(st, 1, 2, 2)
            if 3 * k1 == k2:
                assert status != "unique"
                continue
            den = 2 * (3 * k1 - k2)
            assert [c[x] for x in st] == [Fraction(-4 * k1 + k2, den), Fraction(3 * k1, den),
                                          Fraction(-k2, den), Fraction(k1, den)]


@pytest.mark.parametrize("name", sorted(k for k in GOLD["space_expanded"] if not k.startswith("_")))
def test_space_expanded_table_schemes(name):
    g = GOLD["space_expanded"][name]
    for k in (1, 2, 3):
        st = [(j, k if l == "k" else l) for j, l in g["stencil"]]
        status, c = coeffs.derive_scheme(st, g["d"], g["a"], g["r"])
        assert status == "unique", name
        assert [c[x] for x in st] == [Fraction(v, g["den"]) for v in g["num"]], g["cite"]


def test_printed_left_122a_is_inconsistent_and_mirror_is_the_scheme():
    """Table atschemes-left prints (1,2,2)a as (3U_{i+1} - 3U_i - U_{i-1} - U_{i-2})/4dx, whose
    coefficients sum to -2/4 (not a derivative). The mirror of the right-boundary
    scheme, with +U_{i-1}, is what eq. cond yields."""
    printed = {(1, 0): Fraction(3, 4), (0, 0): Fraction(-3, 4), (-1, 1): Fraction(-1, 4), (-2, 1): Fraction(-1, 4)}
    assert sum(printed.values()) != 0
    st = [(1, 0), (0, 0), (-1, 1), (-2, 1)]
    status, c = coeffs.derive_scheme(st, 1, 2, 2)
    assert status == "unique"
    assert c == {(1, 0): Fraction(3, 4), (0, 0): Fraction(-3, 4), (-1, 1): Fraction(1, 4), (-2, 1): Fraction(-1, 4)}


@pytest.mark.parametrize("name", ["(1,2,2)b", "(2,2,2)b", "(1,4,2)", "(2,4,2)", "(2,6,2)"])
@pytest.mark.parametrize("side", ["left", "right"])
def test_time_expanded_schemes_meet_order_conditions_and_printed_error(name, side):
    g = GOLD["leading_terms"][name]
    d, a, T = g["d"], g["a"], g["T"]
    for k in range(0, 8):
        st = coeffs.time_expanded_at_stencil(d, a, k, T, side)
        res = coeffs.condition_residuals(st, d, a, 2)
        for (p, q), v in res.items():
            assert v == (1 if (p, q) == (d, 0) else 0), (name, side, k, p, q)
        wide = coeffs.condition_residuals(st, d, a, 2, extra=a + 2)
        sp = g["space"]
        assert abs(wide[(sp["p"], 0)]) == Fraction(*sp["coef"]), g["cite"]
        if "time" in g:
            tm = g["time"]
            kp = 1
            for r_ in tm["kroots"]:
                kp *= (k + r_)
            assert abs(wide[(0, tm["q"])]) == Fraction(*tm["coef"]) * kp, (g["cite"], k)


@pytest.mark.parametrize("name", ["(1,2,2)a_right", "(2,2,2)a_right", "(2,1,2)_right"])
def test_space_expanded_printed_leading_terms(name):
    g = GOLD["space_expanded"][name]
    lead = GOLD["space_expanded_leading"][name]
    for k in (1, 2, 3):
        st = [(j, k if l == "k" else l) for j, l in g["stencil"]]
        _, c = coeffs.derive_scheme(st, g["d"], g["a"], g["r"])
        wide = coeffs.condition_residuals(c, g["d"], g["a"], 2, extra=3)
        sp, tm = lead["space"], lead["time"]
        assert abs(wide[(sp["p"], sp["q"])]) == Fraction(*sp["coef"]), lead["cite"]
        assert abs(wide[(tm["p"], tm["q"])]) == Fraction(*tm["coef"]) * k, lead["cite"]


def test_levels_needed():
    assert [coeffs.n_time_levels(d, a, 2) for d, a in [(1, 2), (2, 2), (1, 4), (2, 4), (1, 6), (2, 6)]] == [2, 2, 3, 3, 4, 4]


def test_moment_laws_for_uniform_delays():
    """Sec. 4.2 eq. te-async1 / Sec. 5.2 eq. aveE_scaling_gen_L with p_k = 1/L."""
    laws = GOLD["moment_laws"]
    for L in range(1, 12):
        m2 = sum(Fraction(k * (k + 1), L) for k in range(L))
        m3 = sum(Fraction(k * (k + 1) * (k + 2), L) for k in range(L))
        g2, g3 = laws["T2_uniform"], laws["T3_uniform"]
        assert m2 == Fraction(sum(c * L ** i for i, c in enumerate(g2["poly_in_L"])), g2["scale"][1])
        assert m3 == Fraction(sum(c * L ** i for i, c in enumerate(g3["poly_in_L"])), g3["scale"][1])
