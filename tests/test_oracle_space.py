"""Pins of the oracle's space-expanded single-level AT family (Tables
atschemes-left/right, rows (2,1,2), (1,2,2)a, (2,2,2)a; Sec. 5.1 Cases 2
and 3), against what the paper and the mathematics fix:

- the delayed-level wiring: on an exact travelling wave the AT derivative
  minus the same stencil on undelayed data is linear in k with the paper's
  leading time term (fixture tests/golden/paper_schemes.json,
  ``space_expanded_leading``);
- the spatial order of the boundary derivative (1, 2 or 2 by the tables);
- k = 0 keeps the standard CD2 (a zero-delay run equals the synchronous run);
- the asymptotic second-order convergence of the whole solver with random
  delays, and its larger error, reported for Cases 2 and 3.
"""
import json
import math
import os

import pytest
import torch

from oracle import analytic
from oracle.solver import DelayModel, Oracle, Problem

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_schemes.json")))
LEAD = GOLD["space_expanded_leading"]

# (scheme, derivative order) -> table row whose leading terms apply
ROWS = {("space212", 1): "(1,2,2)a_right", ("space222", 1): "(1,2,2)a_right",
        ("space212", 2): "(2,1,2)_right", ("space222", 2): "(2,2,2)a_right"}


def wave(prob, t):
    """u = sin(3 (x - t)): exact for pure advection with c = 1."""
    return analytic.advected_modes(prob, [((3, 0, 0), 1.0, 0.0)], t)


def mixed_derivative(x, t, p, q):
    """d^p/dx^p d^q/dt^q of sin(3 (x - t))."""
    th = 3.0 * (x - t)
    # each x-derivative multiplies by 3 and each t-derivative by -3, both
    # advancing the phase by pi/2
    return (3.0 ** p) * ((-3.0) ** q) * torch.sin(th + (p + q) * math.pi / 2)


def boundary_derivative(scheme, d, N, dt, k, history="exact"):
    prob = Problem(ndim=1, n=(N,), pe=(4,), dt=dt, order=2, c=(1.0,), alpha=0.0)
    o = Oracle(prob, DelayModel(L=4, mode="rng", scheme=scheme), wave(prob, 0.0))
    n = 3
    o.n = n
    if history == "exact":
        o.hist = {l: wave(prob, l * dt) for l in range(0, n + 1)}
    else:   # every level holds u^n: the same stencil on undelayed data
        o.hist = {l: wave(prob, n * dt) for l in range(0, n + 1)}
    K = torch.full((prob.n_pe, 1, 2), k, dtype=torch.long)
    taps = o.taps1 if d == 1 else o.taps2
    D = o.axis_derivative(o.hist[n], K, 0, taps) / prob.dx[0] ** d
    b = prob.b[0]
    idx = torch.cat([torch.arange(4) * b, torch.arange(4) * b + b - 1])
    x = torch.arange(N, dtype=torch.float64) * prob.dx[0]
    return prob, D.reshape(-1)[idx], x[idx], n * dt


@pytest.mark.parametrize("scheme,d", sorted(ROWS))
def test_delay_error_is_the_printed_leading_time_term(scheme, d):
    lead = LEAD[ROWS[(scheme, d)]]
    N, dt = 1024, 2e-4
    _, D0, x, t = boundary_derivative(scheme, d, N, dt, 1, history="frozen")
    dx = 2 * math.pi / N
    tm = lead["time"]
    pred_unit = mixed_derivative(x, t, tm["p"], tm["q"]).abs() * dt * dx ** (tm["p"] - d) \
        * tm["coef"][0] / tm["coef"][1]
    _, D1, _, _ = boundary_derivative(scheme, d, N, dt, 1)
    delta1 = D1 - D0
    big = pred_unit > 0.3 * pred_unit.max()
    assert big.sum() >= 2
    rel = (delta1.abs()[big] - pred_unit[big]).abs() / pred_unit[big]
    assert float(rel.max()) < 0.05, lead["cite"]
    for k in (2, 3):
        _, Dk, _, _ = boundary_derivative(scheme, d, N, dt, k)
        lin = ((Dk - D0) - k * delta1).abs()[big] / (k * delta1.abs()[big])
        assert float(lin.max()) < 0.05, (k, lead["cite"])


@pytest.mark.parametrize("scheme,d,order", [("space212", 1, 2), ("space212", 2, 1),
                                            ("space222", 1, 2), ("space222", 2, 2)])
def test_boundary_derivative_order_with_delayed_data(scheme, d, order):
    errs = []
    for N in (128, 256, 512):
        dx = 2 * math.pi / N
        _, D, x, t = boundary_derivative(scheme, d, N, 0.05 * dx * dx, 2)
        errs.append(float((D - mixed_derivative(x, t, d, 0)).abs().max()))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.2 for r in rates), (errs, rates)


@pytest.mark.parametrize("scheme", ["space212", "space222"])
def test_zero_delays_keep_the_standard_cd2(scheme):
    prob = Problem(ndim=2, n=(32, 24), pe=(4, 3), dt=1e-3, order=2, c=(1.0, 0.5), alpha=0.1)
    u0 = analytic.advected_modes(prob, [((1, 2, 0), 1.0, 0.3), ((3, 1, 0), 0.5, 1.1)], 0.0)
    a = Oracle(prob, DelayModel(L=3, mode="zero", scheme=scheme), u0).run(5)
    b = Oracle(prob, DelayModel(L=3, mode="sync"), u0).run(5)
    assert torch.equal(a, b)
    c = Oracle(prob, DelayModel(L=3, mode="rng", seed=4, scheme=scheme), u0).run(5)
    assert not torch.equal(a, c)


@pytest.mark.parametrize("scheme,c", [("space212", 0.0), ("space222", 1.0)])
def test_cases_2_and_3_converge_at_second_order_with_delays(scheme, c):
    """Sec. 5.1 (figure of Cases 2-5, parts (a) and (b)): with delays drawn
    from p = {0.5, 0.3, 0.2} (L = 3) the average error still falls with slope
    -2, and asynchrony raises its magnitude."""
    modes = [((3, 0, 0), 2.0, 0.0), ((4, 0, 0), 0.5, 0.0), ((5, 0, 0), 1.5, 0.0)]
    errs = {}
    for mode in ("rng", "zero"):
        errs[mode] = []
        for N in (64, 128, 256):
            alpha = 0.1
            dx = 2 * math.pi / N
            dt = 0.05 * dx * dx / alpha
            prob = Problem(ndim=1, n=(N,), pe=(16,), dt=dt, order=2, c=(c,), alpha=alpha)
            u0 = analytic.advected_modes(prob, modes, 0.0)
            o = Oracle(prob, DelayModel(L=3, mode=mode, seed=7, weights=[5, 3, 2], scheme=scheme), u0)
            o.run(int(round(0.05 / dt)))
            errs[mode].append(float((o.u - analytic.advected_modes(prob, modes, o.t)).abs().mean()))
    rates = [math.log2(errs["rng"][i] / errs["rng"][i + 1]) for i in range(2)]
    assert all(r > 1.8 for r in rates), (errs, rates)
    assert all(e1 > 1.2 * e0 for e1, e0 in zip(errs["rng"], errs["zero"]))


def test_space_schemes_reject_other_orders_and_thin_pes():
    prob4 = Problem(ndim=1, n=(32,), pe=(4,), dt=1e-3, order=4)
    with pytest.raises(ValueError):
        Oracle(prob4, DelayModel(L=2, scheme="space222"), torch.zeros(prob4.shape, dtype=torch.float64))
    thin = Problem(ndim=1, n=(16,), pe=(8,), dt=1e-3, order=2)
    with pytest.raises(ValueError):
        Oracle(thin, DelayModel(L=2, scheme="space222"), torch.zeros(thin.shape, dtype=torch.float64))
    Oracle(thin, DelayModel(L=2, scheme="space212"), torch.zeros(thin.shape, dtype=torch.float64))
