"""Pins of the oracle's AT time step against what the paper and mathematics fix.

- k = 0 everywhere reproduces the synchronous scheme bit for bit (Sec. 3.4,
  remark after eq. cd4-at).
- The synchronous scheme equals the exact discrete Fourier solution built
  from the printed central-difference taps (closed form).
- Polynomials x^p t^q with p <= a+d-1, q <= T-1 are differentiated exactly
  by the AT operator for every delay (eq. cond).
- The boundary truncation error tends to the printed leading term (Tables
  atschemes-left/right).
- Observed convergence orders (Sec. 5.2: slopes -2, -4 for AT, -1 for
  standard schemes used asynchronously).
- Burgers against the Cole-Hopf exact solution.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import rng
from oracle.analytic import advected_modes
from oracle.norms import error_norms
from oracle.solver import DelayModel, Oracle, Problem, boundary_mask, delay_table

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_schemes.json")))


def _taps(d, a):
    if (d, a) == (1, 6):
        # not printed in the paper: the textbook sixth-order first derivative
        # (Fornberg, Math. Comp. 51, 1988, Table 1)
        return np.array([-1, 9, -45, 0, 45, -9, 1], dtype=np.float64) / 60
    g = GOLD["central_differences"][f"d{d}_a{a}"]
    return np.array(g["num"], dtype=np.float64) / g["den"]


def _run(prob, dm, u0, steps):
    o = Oracle(prob, dm, u0)
    o.run(steps)
    return o


CASES = [
    dict(ndim=1, n=(64,), pe=(4,), order=2, integrator="euler", equation="advdiff", c=(1.0,)),
    dict(ndim=1, n=(96,), pe=(4,), order=4, integrator="ab2", equation="advdiff", c=(1.0,)),
    dict(ndim=1, n=(96,), pe=(4,), order=6, integrator="rk2", equation="burgers", c=(0.0,)),
    dict(ndim=1, n=(60,), pe=(5,), order=4, integrator="ab3", equation="advdiff", c=(0.7,)),
    dict(ndim=2, n=(32, 24), pe=(4, 3), order=4, integrator="ab2", equation="advdiff", c=(1.0, -0.5)),
    dict(ndim=3, n=(16, 16, 24), pe=(2, 2, 3), order=4, integrator="ab2", equation="advdiff", c=(1.0, 1.0, 1.0)),
    dict(ndim=3, n=(24, 12, 12), pe=(2, 2, 2), order=6, integrator="rk2", equation="burgers", c=(0.0, 0.0, 0.0)),
]


def _prob(case, dt=2e-3, alpha=0.1):
    return Problem(dt=dt, alpha=alpha, **case)


def _ic(prob, seed=5):
    modes = W.make_modes([(1, 2, 1), (2, 1, 3)][:2], [0.6, 0.3], seed=seed)
    return torch.from_numpy(W.eval_modes(modes, prob.n, prob.ndim))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['ndim']}d_o{c['order']}_{c['integrator']}_{c['equation']}")
def test_zero_delays_reproduce_synchronous_bitwise(case):
    prob = _prob(case)
    u0 = _ic(prob)
    L = 4
    a = _run(prob, DelayModel(L=L, mode="sync"), u0, 12).u
    b = _run(prob, DelayModel(L=L, mode="zero"), u0, 12).u
    assert torch.equal(a, b)
    c = _run(prob, DelayModel(L=L, mode="rng", seed=3), u0, 12).u
    assert not torch.equal(a, c)


def _discrete_fourier_sync(prob, kappa, steps):
    """Exact discrete solution of the synchronous scheme for u0 = sin(kappa . x):
    every Fourier mode e^{i kappa . x} is an eigenvector of CD_a; the
    integrator is a linear recurrence in its eigenvalue lambda."""
    lam = 0.0 + 0.0j
    for ax in range(prob.ndim):
        dx = prob.dx[ax]
        s = prob.s
        ph = np.exp(1j * kappa[ax] * dx * np.arange(-s, s + 1))
        d1 = (_taps(1, prob.order) * ph).sum() / dx
        d2 = (_taps(2, prob.order) * ph).sum() / dx ** 2
        lam += -prob.c[ax] * d1 + prob.alpha * d2
    z = prob.dt * lam
    if prob.integrator == "euler":
        g = (1 + z) ** steps
    elif prob.integrator == "rk2":
        g = (1 + z + z * z / 2) ** steps
    elif prob.integrator == "ab2":
        u_prev, u_cur = 1.0 + 0j, 1 + z
        for _ in range(steps - 1):
            u_prev, u_cur = u_cur, u_cur + z * (1.5 * u_cur - 0.5 * u_prev)
        g = u_cur
    elif prob.integrator == "ab3":
        # start-up (reading S4): one Euler step, one AB2 step, then AB3
        g_hist = [1.0 + 0j]
        for n in range(steps):
            f = [z * v for v in g_hist[::-1]]      # z * g^n, z * g^{n-1}, ...
            if n == 0:
                inc = f[0]
            elif n == 1:
                inc = 1.5 * f[0] - 0.5 * f[1]
            else:
                inc = (23.0 * f[0] - 16.0 * f[1] + 5.0 * f[2]) / 12.0
            g_hist.append(g_hist[-1] + inc)
        g = g_hist[-1]
    xs = np.meshgrid(*[np.arange(prob.n[a]) * prob.dx[a] for a in range(3)][::-1], indexing="ij")
    phase = sum(kappa[a] * xs[2 - a] for a in range(3))
    return np.imag(g * np.exp(1j * phase))


@pytest.mark.parametrize("integ,order,ndim", [("euler", 2, 1), ("ab2", 4, 1), ("rk2", 6, 1), ("ab2", 4, 3), ("ab2", 4, 2),
                                               ("ab3", 4, 1), ("ab3", 6, 2), ("ab3", 2, 3)])
def test_synchronous_scheme_equals_discrete_fourier_solution(integ, order, ndim):
    n = {1: (64,), 2: (32, 16), 3: (16, 16, 16)}[ndim]
    pe = {1: (4,), 2: (2, 2), 3: (2, 2, 2)}[ndim]
    c = (1.0, -0.5, 0.25)[:ndim]
    prob = Problem(ndim=ndim, n=n, pe=pe, dt=1e-3, order=order, integrator=integ, c=c, alpha=0.1)
    kappa = (3, 1, 2)[:ndim] + (0,) * (3 - ndim)
    u0 = torch.from_numpy(W.eval_modes(W.make_modes([kappa], [1.0], phis=[0.0]), prob.n, ndim))
    steps = 40
    got = _run(prob, DelayModel(mode="sync"), u0, steps).u.numpy()
    want = _discrete_fourier_sync(prob, kappa, steps)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("order,d", [(2, 1), (2, 2), (4, 1), (4, 2), (6, 1), (6, 2)])
def test_polynomials_are_differentiated_exactly_for_every_delay(order, d):
    """eq. cond: u = x^p t^q with p <= a + d - 1, q <= T - 1 is reproduced for
    all k. Evaluated at the boundary layers of an interior PE face (the
    periodic wrap is far away)."""
    s = order // 2
    T = s + 1
    L = 5
    b = 2 * s + 2
    npe = 4
    N = b * npe
    h = 0.37            # grid spacing
    dt = 0.11
    prob = Problem(ndim=1, n=(N,), pe=(npe,), dt=dt, order=order, length=N * h)
    x0 = 2 * b * h      # interior face between PE 1 and PE 2
    x = torch.arange(N, dtype=torch.float64) * h - x0
    n_now = L + T
    for p in range(0, order + d):
        for q in range(0, T):
            o = Oracle(prob, DelayModel(L=L, T=T, mode="zero"), torch.zeros(prob.shape))
            o.n = n_now
            t = lambda l: (n_now - l) * dt - 0.5   # shift t so that t^q is not trivial
            o.hist = {l: (x ** p * t(l) ** q).reshape(prob.shape) for l in range(0, n_now + 1)}
            centre = o.hist[n_now]
            # exact derivative at time t_n
            if p >= d:
                exact = math.factorial(p) / math.factorial(p - d) * x ** (p - d) * t(n_now) ** q
            else:
                exact = torch.zeros_like(x)
            taps = o.taps1 if d == 1 else o.taps2
            for k in range(L):
                K = torch.full((prob.n_pe, 1, 2), k, dtype=torch.long)
                D = o.axis_derivative(centre, K, 0, taps).reshape(-1) / h ** d
                sl = slice(b + 1, 3 * b - 1)   # both sides of the interior face x0
                err = (D[sl] - exact[sl]).abs().max()
                scale = 1.0 + exact[sl].abs().max() + (x[sl].abs().max() ** p) * abs(t(n_now + L + T)) ** q
                assert err <= 1e-9 * scale, (p, q, k, float(err))


@pytest.mark.parametrize("order,scheme", [(4, "(2,4,2)"), (6, "(2,6,2)"), (2, "(2,2,2)b")])
def test_boundary_truncation_error_tends_to_printed_term(order, scheme):
    """Apply the AT second derivative once to u = sin(x - t) at the point next to
    a low face, with a fixed delay k and dt = dx. (D - u_xx) / (dt^q / dx^2)
    tends to -coef * prod(k+i) * d^q u / dt^q (Tables atschemes-left/right)."""
    g = GOLD["leading_terms"][scheme]
    q = g["time"]["q"]
    coef = g["time"]["coef"][0] / g["time"]["coef"][1]
    s = order // 2
    T = s + 1
    ratios = {}
    for k in (1, 2):
        kp = 1
        for r_ in g["time"]["kroots"]:
            kp *= (k + r_)
        for N in (256, 512):
            h = 2 * math.pi / N
            dt = h
            npe = 8
            prob = Problem(ndim=1, n=(N,), pe=(npe,), dt=dt, order=order)
            o = Oracle(prob, DelayModel(L=4, T=T, mode="zero"), torch.zeros(prob.shape))
            n_now = 4 + T
            o.n = n_now
            x = torch.arange(N, dtype=torch.float64) * h
            o.hist = {l: torch.sin(x - l * dt).reshape(prob.shape) for l in range(0, n_now + 1)}
            K = torch.full((npe, 1, 2), k, dtype=torch.long)
            D = o.axis_derivative(o.hist[n_now], K, 0, o.taps2).reshape(-1) / h ** 2
            uxx = -torch.sin(x - n_now * dt)
            # d^q/dt^q sin(x - t)
            dq = [torch.sin, lambda z: -torch.cos(z), lambda z: -torch.sin(z), torch.cos][q % 4](x - n_now * dt)
            idx = torch.arange(npe) * (N // npe)         # points next to each low face
            pred = -coef * kp * dq[idx] * dt ** q / h ** 2
            err = (D - uxx)[idx]
            ratios[(k, N)] = float(((err - pred).abs().max()) / pred.abs().max())
    for k in (1, 2):
        assert ratios[(k, 512)] < 0.6 * ratios[(k, 256)] + 1e-3, ratios
        assert ratios[(k, 512)] < 0.05, ratios


def _slopes(errs):
    return [math.log(errs[i + 1] / errs[i]) / math.log(2) for i in range(len(errs) - 1)]


def _conv_errors(order, mode, T, L=3, P=8, tf=0.2, Ns=None, r_alpha=None):
    modes = W.make_modes([(3,), (4,), (5,)], [2.0, 0.5, 1.5], seed=7)   # Sec. 5.2 workload
    errs = []
    for N in Ns:
        dx = 2 * math.pi / N
        ra = r_alpha if r_alpha is not None else (0.1 if order == 2 else 0.05)
        dt = ra * dx * dx / 0.1
        steps = int(round(tf / dt))
        dt = tf / steps
        prob = Problem(ndim=1, n=(N,), pe=(P,), dt=dt, order=order, c=(1.0,), alpha=0.1,
                       integrator="euler" if order == 2 else "ab2")
        u0 = torch.from_numpy(W.eval_modes(modes, (N,), 1))
        o = _run(prob, DelayModel(L=L, T=T, mode=mode, seed=11), u0, steps)
        errs.append(error_norms(o.u, advected_modes(prob, modes, o.t))["l2"])
    return errs


@pytest.mark.slow
def test_convergence_order_second_order_case1():
    """Case 1 (AD, Euler, CD2, (1,2,2)b + (2,2,2)b), fixed P = 8, L = 3: slope -2
    for SYNC and AT, about -1 when the standard scheme is used asynchronously."""
    Ns = [64, 128, 256, 512]
    sy = _slopes(_conv_errors(2, "sync", 0, Ns=Ns))
    at = _slopes(_conv_errors(2, "rng", 0, Ns=Ns))
    st = _slopes(_conv_errors(2, "rng", 1, Ns=Ns))
    assert all(abs(s + 2) < 0.1 for s in sy), sy
    assert all(abs(s + 2) < 0.15 for s in at), at
    assert all(-1.4 < s < -0.8 for s in st), st


@pytest.mark.slow
def test_convergence_order_fourth_order_case4():
    """Case 4 (AD, AB2, CD4, (1,4,2) + (2,4,2)): slope -4; CD4 used asynchronously: about -1."""
    Ns = [64, 128, 256]
    sy = _slopes(_conv_errors(4, "sync", 0, Ns=Ns))
    at = _slopes(_conv_errors(4, "rng", 0, Ns=Ns))
    st = _slopes(_conv_errors(4, "rng", 1, Ns=Ns))
    assert all(abs(s + 4) < 0.2 for s in sy), sy
    assert all(abs(s + 4) < 0.25 for s in at), at
    assert all(-1.4 < s < -0.7 for s in st), st


def _mode_eigenvalue(prob, kappa):
    """Eigenvalue of the synchronous right-hand side on e^{i kappa x} (1-D)."""
    dx, s = prob.dx[0], prob.s
    ph = np.exp(1j * kappa * dx * np.arange(-s, s + 1))
    d1 = (_taps(1, prob.order) * ph).sum() / dx
    d2 = (_taps(2, prob.order) * ph).sum() / dx ** 2
    return -prob.c[0] * d1 + prob.alpha * d2


def test_ab3_from_exact_history_is_third_order_in_time():
    """Sec. 4.1 eq. time_disc with three levels: an explicit three-step Adams
    method u^{n+1} = u^n + dt (b0 f^n + b1 f^{n-1} + b2 f^{n-2}) is third-order
    accurate only for (b0, b1, b2) = (23, -16, 5)/12 (the order conditions
    b0 + b1 + b2 = 1, -(b1 + 2 b2) = 1/2, (b1 + 4 b2)/2 = 1/6 have that one
    solution). Started from the exact past right-hand sides of one Fourier
    mode, the oracle's error against the exact semi-discrete solution
    e^{lambda t} must fall by 8x per halving of dt."""
    kappa = 3
    N, tf = 32, 0.6
    errs = []
    for dt in (0.03, 0.015, 0.0075):
        prob = Problem(ndim=1, n=(N,), pe=(4,), dt=dt, order=4, integrator="ab3", c=(1.0,), alpha=0.1)
        lam = _mode_eigenvalue(prob, kappa)
        x = np.arange(N) * prob.dx[0]

        def exact(t):
            return torch.from_numpy(np.imag(np.exp(lam * t) * np.exp(1j * kappa * x)).reshape(prob.shape))

        o = Oracle(prob, DelayModel(mode="sync"), exact(0.0))
        K = delay_table(prob, DelayModel(mode="sync"), 0)
        o.fhist = [o.rhs(exact(-dt), K), o.rhs(exact(-2 * dt), K)]   # f^{-1}, f^{-2}
        steps = int(round(tf / dt))
        o.run(steps)
        errs.append(float((o.u - exact(steps * dt)).abs().max()))
    sl = _slopes(errs)
    assert all(-3.1 < v < -2.9 for v in sl), (errs, sl)


@pytest.mark.slow
def test_at_ab3_fourth_order_converges_at_slope_minus_four():
    """AB3 with the fourth-order AT scheme ((1,4,2) + (2,4,2), T = 3), delays
    L = 3 on 8 PEs, dt ~ dx^2: the spatial O(dx^4) error and the O(dt^2) =
    O(dx^4) of the Euler start-up give slope -4 against the exact advected
    decaying sine series (Sec. 5.2 workload)."""
    modes = W.make_modes([(3,), (4,), (5,)], [2.0, 0.5, 1.5], seed=7)
    tf = 0.1
    errs = {"sync": [], "rng": []}
    for N in (32, 64, 128):
        dx = 2 * math.pi / N
        steps = int(round(tf / (0.02 * dx * dx / 0.1)))
        prob = Problem(ndim=1, n=(N,), pe=(8,) if N >= 64 else (4,), dt=tf / steps, order=4,
                       integrator="ab3", c=(1.0,), alpha=0.1)
        u0 = torch.from_numpy(W.eval_modes(modes, (N,), 1))
        for mode in errs:
            o = _run(prob, DelayModel(L=3, mode=mode, seed=13), u0, steps)
            errs[mode].append(error_norms(o.u, advected_modes(prob, modes, o.t))["l2"])
    for mode, e in errs.items():
        sl = _slopes(e)
        assert all(-4.3 < v < -3.7 for v in sl), (mode, e, sl)


def test_first_configuration_against_analytic_solution():
    """N = 256, 8 PEs, L = 3, 1000 Euler steps, u0 = sin x: AT error equals the
    synchronous error to leading order and both are O(dx^2) small."""
    cfg = W.config_1d_advdiff()
    prob = Problem(ndim=1, n=cfg["n"], pe=cfg["pe"], dt=cfg["dt"], order=2, c=cfg["c"], alpha=cfg["alpha"])
    u0 = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], 1))
    sy = _run(prob, DelayModel(L=3, mode="sync"), u0, cfg["steps"])
    at = _run(prob, DelayModel(L=3, mode="rng", seed=cfg["seed"]), u0, cfg["steps"])
    ua = advected_modes(prob, cfg["modes"], sy.t)
    es = error_norms(sy.u, ua)["l2"]
    ea = error_norms(at.u, ua, boundary_mask(prob))["l2"]
    dx = prob.dx[0]
    assert es < 0.5 * dx * dx            # second order with a modest constant
    assert abs(ea - es) < 0.05 * es       # asynchrony costs <5% at this resolution


def test_three_d_with_x_only_field_and_delays_equals_one_d():
    """Dimension splitting: a field constant in y and z, delays only on x faces,
    evolves exactly like the 1-D problem on every (y, z) line."""
    N, P = 48, 4
    L, T = 3, 3
    steps = 15
    prob1 = Problem(ndim=1, n=(N,), pe=(P,), dt=2e-3, order=4, integrator="ab2", c=(1.0,), alpha=0.1)
    prob3 = Problem(ndim=3, n=(N, 8, 8), pe=(P, 2, 2), dt=2e-3, order=4, integrator="ab2", c=(1.0, 0.3, -0.2), alpha=0.1)
    rs = np.random.Generator(np.random.PCG64(9))
    k1 = rs.integers(0, L, size=(steps, P, 1, 2))
    k3 = np.zeros((steps, prob3.n_pe, 3, 2), dtype=np.int64)
    for p in range(prob3.n_pe):
        k3[:, p, 0, :] = k1[:, p % P, 0, :]
    u1 = torch.from_numpy(W.eval_modes(W.make_modes([(2,), (5,)], [1.0, 0.4], seed=2), (N,), 1))
    u3 = u1.reshape(1, 1, N).expand(8, 8, N).contiguous()
    a = _run(prob1, DelayModel(L=L, T=T, mode="host", host=k1), u1, steps).u
    b = _run(prob3, DelayModel(L=L, T=T, mode="host", host=k3), u3, steps).u
    assert float((b - a.reshape(1, 1, N)).abs().max()) < 1e-12


def _cole_hopf(x, t, amp, nu, nmodes=80):
    """Exact periodic solution of u_t + u u_x = nu u_xx, u(x,0) = amp sin x:
    u = -2 nu phi_x / phi with phi the heat solution from exp(amp cos x / 2 nu)."""
    from scipy.special import ive
    z = amp / (2 * nu)
    n = np.arange(nmodes)
    cn = np.where(n == 0, 1.0, 2.0) * ive(n, z)       # scaled Bessel I_n; common factor e^z cancels
    decay = np.exp(-nu * n ** 2 * t)
    num = (2 * nu * (n * cn * decay)[None, :] * np.sin(np.outer(x, n))).sum(1)
    den = ((cn * decay)[None, :] * np.cos(np.outer(x, n))).sum(1)
    return num / den


@pytest.mark.slow
@pytest.mark.parametrize("order,integ,want", [(4, "ab2", -4.0), (6, "rk2", -4.0)])
def test_burgers_converges_to_cole_hopf(order, integ, want):
    """Case 6-type Burgers (1-D): AT converges at the scheme's order against the
    exact Cole-Hopf solution; with Heun RK2 and dt ~ dx^2 the temporal
    O(dt^2) = O(dx^4) term dominates a sixth-order space error."""
    nu, amp, tf = 0.1, 0.5, 0.3
    errs = {"sync": [], "rng": []}
    Ns = [32, 64, 128]
    for N in Ns:
        dx = 2 * math.pi / N
        dt = 0.05 * dx * dx / nu
        steps = int(round(tf / dt))
        dt = tf / steps
        prob = Problem(ndim=1, n=(N,), pe=(4,), dt=dt, order=order, equation="burgers", alpha=nu, integrator=integ)
        x = np.arange(N) * dx
        u0 = torch.from_numpy(amp * np.sin(x).reshape(prob.shape))
        exact = _cole_hopf(x, tf, amp, nu)
        for mode in errs:
            # L = 3: with r_alpha = 0.05 larger L is outside the AT stability range
            o = _run(prob, DelayModel(L=3, mode=mode, seed=5), u0, steps)
            e = o.u.reshape(-1).numpy() - exact
            errs[mode].append(float(np.sqrt((e * e).mean())))
    for mode, e in errs.items():
        sl = _slopes(e)
        assert sl[-1] < want + 0.4, (mode, e, sl)
    assert errs["rng"][-1] < 2.0 * errs["sync"][-1]


def test_delay_table_uses_generator_and_clamp():
    prob = Problem(ndim=2, n=(16, 16), pe=(2, 2), dt=1e-3, order=4)
    dm = DelayModel(L=4, mode="rng", seed=1)
    thr = rng.thresholds(4)
    for n in (0, 1, 2, 3, 7):
        K = delay_table(prob, dm, n)
        for p in range(4):
            for a in range(2):
                for sd in range(2):
                    face = p * 4 + 2 * a + sd
                    want = rng.clamp_startup(rng.raw_delay(1, n, face, thr), n, 3)
                    assert int(K[p, a, sd]) == want


def test_invalid_problems_rejected():
    with pytest.raises(ValueError):
        Problem(ndim=1, n=(30,), pe=(4,), dt=1e-3)
    with pytest.raises(ValueError):
        Problem(ndim=1, n=(12,), pe=(4,), dt=1e-3, order=4)   # b = 3 < 2s
