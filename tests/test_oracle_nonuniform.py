"""Pins of the oracle's non-uniform-delay scheme (Sec. 3.4 Example 1, eq.
ex1-0, with its second-derivative counterpart on the (2,1,2) footprint):
the two buffer points next to a face carry their own delays k1 (nearest) and
k2. Checked against what the paper and the mathematics fix:

- equal delays reduce it to the uniform-delay schemes (the paper: eq. ex1-0
  becomes eq. ex1-1 = (1,2,2)a; the (2,2)-footprint row becomes (2,1,2)), so a
  run whose second-point delays are forced equal to the face delays is the
  space212 run;
- on an exact travelling wave the spatial error of the face derivative is the
  Taylor residual dx^2 (6k1 - k2) / (6 (3k1 - k2)) u_xxx printed with eq.
  ex1-0, and the delayed-minus-undelayed part is dt k1 k2 / (2 (3k1 - k2))
  u_xt with a minus sign (reading: the printed time coefficient is twice
  this), including the singular set 3 k1 = k2, where k1 + 1 is used;
- zero delays keep the standard CD2 (equal to the synchronous run bitwise);
- the whole solver converges at second order with random per-point delays.
"""
import math

import pytest
import torch

from oracle import analytic, solver
from oracle.solver import DelayModel, Oracle, Problem, nonuniform_delays


def wave(prob, t):
    return analytic.advected_modes(prob, [((3, 0, 0), 1.0, 0.0)], t)


def mixed_derivative(x, t, p, q):
    """d^p/dx^p d^q/dt^q of sin(3 (x - t))."""
    return (3.0 ** p) * ((-3.0) ** q) * torch.sin(3.0 * (x - t) + (p + q) * math.pi / 2)


def face_derivative(d, N, dt, k1, k2, history):
    """Derivative d at every face-adjacent point with per-face delays (k1, k2)."""
    prob = Problem(ndim=1, n=(N,), pe=(4,), dt=dt, order=2, c=(1.0,), alpha=0.0)
    o = Oracle(prob, DelayModel(L=8, mode="rng", scheme="nonuniform212"), wave(prob, 0.0))
    n = 12
    o.n = n
    if history == "exact":
        o.hist = {l: wave(prob, l * dt) for l in range(0, n + 1)}
    else:    # every level holds u^n: the same stencil on undelayed data
        o.hist = {l: wave(prob, n * dt) for l in range(0, n + 1)}
    K = torch.full((prob.n_pe, 1, 2), k1, dtype=torch.long)
    o.K2 = torch.full((prob.n_pe, 1, 2), k2, dtype=torch.long)
    taps = o.taps1 if d == 1 else o.taps2
    D = o.axis_derivative(o.hist[n], K, 0, taps) / prob.dx[0] ** d
    b = prob.b[0]
    idx = torch.cat([torch.arange(4) * b, torch.arange(4) * b + b - 1])
    x = torch.arange(N, dtype=torch.float64) * prob.dx[0]
    return D.reshape(-1)[idx], x[idx], n * dt


PAIRS = [(1, 2), (2, 1), (3, 1), (1, 5), (2, 7), (1, 3), (2, 6)]
N_WAVE, DT_WAVE = 2048, 2e-5


def close_where_large(got, pred, tol=0.05):
    """|got - pred| <= tol |pred| wherever |pred| is at least 0.3 of its max."""
    big = pred.abs() > 0.3 * pred.abs().max()
    assert int(big.sum()) >= 2
    return float(((got - pred).abs()[big] / pred.abs()[big]).max()) < tol


@pytest.mark.parametrize("k1,k2", PAIRS)
def test_first_derivative_error_terms(k1, k2):
    e1, e2 = nonuniform_delays(k1, k2)
    den = 3 * e1 - e2
    N, dt = N_WAVE, DT_WAVE
    dx = 2 * math.pi / N
    D0, x, t = face_derivative(1, N, dt, k1, k2, "frozen")
    D1, _, _ = face_derivative(1, N, dt, k1, k2, "exact")
    # spatial part: the dx^2 coefficient printed with eq. ex1-0
    space = D0 - mixed_derivative(x, t, 1, 0)
    pred_s = dx ** 2 * (6 * e1 - e2) / (6 * den) * mixed_derivative(x, t, 3, 0)
    assert close_where_large(space, pred_s)
    # time part: u_xt dt sum c j (-l)
    pred_t = -dt * e1 * e2 / (2 * den) * mixed_derivative(x, t, 1, 1)
    assert close_where_large(D1 - D0, pred_t)


@pytest.mark.parametrize("k1,k2", PAIRS)
def test_second_derivative_error_terms(k1, k2):
    e1, e2 = nonuniform_delays(k1, k2)
    den = 3 * e1 - e2
    N, dt = N_WAVE, DT_WAVE
    dx = 2 * math.pi / N
    D0, x, t = face_derivative(2, N, dt, k1, k2, "frozen")
    D1, _, _ = face_derivative(2, N, dt, k1, k2, "exact")
    space = D0 - mixed_derivative(x, t, 2, 0)
    # first order in space, like the (2,1,2) row it generalises; the mirror
    # image at the left face flips the sign of the odd term
    sgn = torch.cat([-torch.ones(4), torch.ones(4)]).double()
    pred_s = sgn * dx * e1 / den * mixed_derivative(x, t, 3, 0)
    assert close_where_large(space, pred_s)
    pred_t = -sgn * (dt / dx) * e1 * e2 / den * mixed_derivative(x, t, 1, 1)
    assert close_where_large(D1 - D0, pred_t)


def test_singular_set_and_synchronous_points():
    """Eq. ex1-0 has no solution where 3 k1 = k2 (k1 >= 1): the nearest point
    then takes the next older level; both delays zero: the CD2."""
    assert nonuniform_delays(1, 3) == (2, 3)
    assert nonuniform_delays(2, 6) == (3, 6)
    assert nonuniform_delays(0, 0) is None
    assert nonuniform_delays(0, 4) == (0, 4)
    assert nonuniform_delays(2, 1) == (2, 1)


def test_equal_point_delays_reduce_to_the_space212_scheme(monkeypatch):
    prob = Problem(ndim=2, n=(32, 24), pe=(4, 3), dt=1e-3, order=2, c=(1.0, 0.5), alpha=0.1)
    u0 = analytic.advected_modes(prob, [((1, 2, 0), 1.0, 0.3), ((3, 1, 0), 0.5, 1.1)], 0.0)
    ref = Oracle(prob, DelayModel(L=4, mode="rng", seed=9, scheme="space212"), u0).run(6)
    monkeypatch.setattr(solver, "point_delay_table", solver.delay_table)
    got = Oracle(prob, DelayModel(L=4, mode="rng", seed=9, scheme="nonuniform212"), u0).run(6)
    assert torch.allclose(got, ref, rtol=0, atol=1e-13)


def test_zero_delays_keep_the_standard_cd2():
    prob = Problem(ndim=2, n=(32, 24), pe=(4, 3), dt=1e-3, order=2, c=(1.0, 0.5), alpha=0.1)
    u0 = analytic.advected_modes(prob, [((1, 2, 0), 1.0, 0.3), ((3, 1, 0), 0.5, 1.1)], 0.0)
    a = Oracle(prob, DelayModel(L=3, mode="zero", scheme="nonuniform212"), u0).run(5)
    b = Oracle(prob, DelayModel(L=3, mode="sync"), u0).run(5)
    assert torch.equal(a, b)
    c = Oracle(prob, DelayModel(L=3, mode="rng", seed=4, scheme="nonuniform212"), u0).run(5)
    d = Oracle(prob, DelayModel(L=3, mode="rng", seed=4, scheme="space212"), u0).run(5)
    assert not torch.equal(a, c) and not torch.equal(c, d)


def test_second_point_delays_are_their_own_draws():
    prob = Problem(ndim=2, n=(16, 16), pe=(4, 4), dt=1e-3, order=2)
    dm = DelayModel(L=8, mode="rng", seed=11, scheme="nonuniform212")
    K1 = torch.stack([solver.delay_table(prob, dm, n) for n in range(20, 40)])
    K2 = torch.stack([solver.point_delay_table(prob, dm, n) for n in range(20, 40)])
    assert K1.min() >= 0 and K2.max() <= 7
    assert float((K1 == K2).double().mean()) < 0.3      # about 1/8 for independent uniform draws
    assert float(K2.double().mean()) == pytest.approx(3.5, abs=0.4)


@pytest.mark.parametrize("c", [0.0, 1.0])
def test_solver_converges_at_second_order_with_per_point_delays(c):
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
            o = Oracle(prob, DelayModel(L=4, mode=mode, seed=7, scheme="nonuniform212"), u0)
            o.run(int(round(0.05 / dt)))
            errs[mode].append(float((o.u - analytic.advected_modes(prob, modes, o.t)).abs().mean()))
    rates = [math.log2(errs["rng"][i] / errs["rng"][i + 1]) for i in range(2)]
    assert rates[-1] > 1.9 and rates[0] > 1.6, (errs, rates)
    assert all(e1 > 1.2 * e0 for e1, e0 in zip(errs["rng"], errs["zero"]))


def test_nonuniform_scheme_rejects_other_orders_and_host_tables():
    z = lambda p: torch.zeros(p.shape, dtype=torch.float64)
    prob4 = Problem(ndim=1, n=(32,), pe=(4,), dt=1e-3, order=4)
    with pytest.raises(ValueError):
        Oracle(prob4, DelayModel(L=2, scheme="nonuniform212"), z(prob4))
    ok = Problem(ndim=1, n=(32,), pe=(4,), dt=1e-3, order=2)
    with pytest.raises(ValueError):
        Oracle(ok, DelayModel(L=2, mode="host", scheme="nonuniform212"), z(ok))
