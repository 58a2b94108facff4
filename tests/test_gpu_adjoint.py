"""GPU parity of the hand-written adjoint (at_adjoint) against the oracle's
gradients (reverse-mode autograd of the FP64 forward steps), and the full-size
gradient checks against central finite differences of the GPU forward (the
2-D advection-diffusion workload and the 512^3 Burgers workload).

Tolerances. FP64: relative L2 (and the element-wise measures) <= 1e-12 for
dJ/du0 and relative 1e-12 for dJ/dalpha, the forward's FP64 bar: both sides
are exact transposes of the same discrete map, evaluated in different orders,
so they differ by rounding only (measured: <= 1.8e-15 and <= 7.8e-14). FP32
bulk against the FP64 oracle: dJ/du0 <= 1e-5, the forward's FP32 bar (the
adjoint fields and the stored forward levels are rounded to FP32 every step;
measured <= 2.2e-7); dJ/dalpha 1e-4, a sum over all points and steps of mu
times the Laplacian of FP32-rounded levels, which cancels to a value small
against its terms (measured <= 2.9e-5, 1-D Burgers RK2). Finite differences
(FP32 forward, eps = 1e-3): 1e-3 relative.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.adjoint import gradients
from oracle.solver import DelayModel, Problem
from tests._cases import field_errors, initial_field, oracle_for, rel_l2, solver_for

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "1d_o2_euler_L3": dict(ndim=1, n=(64,), pe=(4,), order=2, integrator="euler", c=(1.0,), L=3, steps=37, every=8, ra=0.1),
    "1d_o4_ab2_L4_ragged": dict(ndim=1, n=(60,), pe=(5,), order=4, integrator="ab2", c=(0.7,), L=4, steps=33, every=5, ra=0.02),
    "1d_o6_ab2_L3": dict(ndim=1, n=(72,), pe=(4,), order=6, integrator="ab2", c=(1.0,), L=3, steps=25, every=7, ra=0.005),
    "1d_o4_T1_async_standard": dict(ndim=1, n=(48,), pe=(4,), order=4, integrator="ab2", c=(1.0,), L=3, T=1, steps=20, every=6, ra=0.02),
    "1d_o4_zero": dict(ndim=1, n=(48,), pe=(3,), order=4, integrator="ab2", c=(1.0,), L=3, mode="zero", steps=20, every=6, ra=0.02),
    "1d_o2_one_pe": dict(ndim=1, n=(32,), pe=(1,), order=2, integrator="euler", c=(1.0,), L=2, steps=15, every=4, ra=0.1),
    "2d_o4_ab2": dict(ndim=2, n=(40, 36), pe=(4, 3), order=4, integrator="ab2", c=(1.0, -0.5), L=4, steps=21, every=6, ra=0.02),
    "2d_o2_sync": dict(ndim=2, n=(32, 24), pe=(2, 2), order=2, integrator="euler", c=(1.0, 1.0), mode="sync", steps=15, every=4, ra=0.05),
    "3d_o4_ab2": dict(ndim=3, n=(24, 20, 16), pe=(2, 2, 2), order=4, integrator="ab2", c=(1.0, 1.0, 1.0), L=3, steps=9, every=4, ra=0.02),
    # 32 x 32 cross-sections: the forward runs on the 3-D fast path
    "3d_fast_o4_ab2": dict(ndim=3, n=(64, 64, 32), pe=(2, 2, 1), order=4, integrator="ab2", c=(1.0, -1.0, 0.5), L=4, steps=8, every=3, ra=0.02),
    # Heun RK2 (predictor ring) and the nonlinear Burgers right-hand side
    "1d_o6_rk2_burgers": dict(ndim=1, n=(96,), pe=(4,), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=3, steps=20, every=6, ra=0.01),
    "1d_o2_rk2_advdiff_L8": dict(ndim=1, n=(64,), pe=(4,), order=2, integrator="rk2", c=(1.0,), L=8, steps=25, every=7, ra=0.05),
    "2d_o4_rk2_burgers_sync": dict(ndim=2, n=(32, 24), pe=(2, 2), order=4, integrator="rk2", equation="burgers", alpha=0.05, mode="sync", steps=12, every=5, ra=0.01),
    "3d_o6_rk2_burgers": dict(ndim=3, n=(24, 24, 24), pe=(2, 2, 2), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=4, steps=6, every=4, ra=0.004),
    "3d_fast_o6_rk2_burgers": dict(ndim=3, n=(64, 64, 32), pe=(2, 2, 1), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=4, steps=6, every=4, ra=0.004),
    # PE cross-sections of 64 points: the column-streaming stage kernel
    "3d_o4_ab2_pe8x8": dict(ndim=3, n=(16, 16, 12), pe=(2, 2, 2), order=4, integrator="ab2", c=(0.5, -1.0, 1.0), L=4, steps=10, every=3, ra=0.02),
    "3d_o6_rk2_burgers_pe8x8": dict(ndim=3, n=(16, 16, 18), pe=(2, 2, 3), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=3, steps=8, every=3, ra=0.004),
}


def _case(name):
    c = dict(CASES[name])
    dx = 2 * math.pi / min(c["n"][: c["ndim"]])
    c["dt"] = c.pop("ra") * dx * dx / c.get("alpha", 0.1)
    return c


def _oracle_grads(case, u0, seed):
    prob = Problem(ndim=case["ndim"], n=case["n"], pe=case["pe"], dt=case["dt"], order=case["order"],
                   equation=case.get("equation", "advdiff"), c=case.get("c", (0.0, 0.0, 0.0)),
                   alpha=case.get("alpha", 0.1), integrator=case["integrator"])
    dm = DelayModel(L=case.get("L", 3), T=case.get("T", 0), mode=case.get("mode", "rng"), seed=case.get("seed", 0))
    return gradients(prob, dm, torch.as_tensor(u0), case.get("alpha", 0.1), case["steps"], torch.as_tensor(seed))


def _seed(case):
    n = tuple(case["n"]) + (1,) * (3 - len(case["n"]))
    return np.random.default_rng(11).standard_normal((n[2], n[1], n[0]))


def _gpu_grads(case, u0, seed, precision, every=None):
    s = solver_for(case, precision)
    s.set_state(torch.from_numpy(u0))
    g, ga = s.adjoint(case["steps"], torch.from_numpy(seed), every or case["every"])
    return s, g.cpu().to(torch.float64), ga


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adjoint_matches_oracle_gradients(name, precision):
    case = _case(name)
    _say(f"[adj] {name} {precision}: steps={case['steps']} every={case['every']}")
    u0 = initial_field(case)
    seed = _seed(case)
    gu_o, ga_o = _oracle_grads(case, u0, seed)
    s, gu, ga = _gpu_grads(case, u0, seed, precision)
    tol = 1e-12 if precision == "f64" else 1e-5
    err = rel_l2(gu, gu_o)
    _say(f"[adj]   du0 errors {field_errors(gu, gu_o, oracle_for(case, u0).prob)}   "
         f"dalpha {ga:.9e} vs {ga_o:.9e} (rel {abs(ga - ga_o) / abs(ga_o):.3e})")
    errs = field_errors(gu, gu_o, oracle_for(case, u0).prob)
    assert err <= tol and errs["max"] <= tol and errs["ib"] <= tol, errs
    assert ga == pytest.approx(ga_o, rel=tol if precision == "f64" else 1e-4)
    # the context ends at step N with the forward field of a plain run
    assert s.n_step == case["steps"]
    ref = solver_for(case, precision)
    ref.set_state(torch.from_numpy(u0))
    ref.step(case["steps"])
    assert torch.equal(s.state(), ref.state())


def test_adjoint_is_independent_of_the_checkpoint_interval():
    case = _case("2d_o4_ab2")
    u0, seed = initial_field(case), _seed(case)
    base = _gpu_grads(case, u0, seed, "f64", every=1)
    for every in (4, case["steps"], 1000):
        other = _gpu_grads(case, u0, seed, "f64", every=every)
        assert torch.equal(other[1], base[1]), every
        assert other[2] == base[2]


def test_adjoint_rejects_unsupported_problems():
    from paper_1702_00496_amd import ATError
    case = _case("1d_o2_euler_L3")
    for bad in (dict(integrator="ab3"), dict(scheme="space222")):
        c = dict(case, **bad)
        s = solver_for(c, "f64")
        s.set_state(torch.from_numpy(initial_field(c)))
        with pytest.raises(ATError):
            s.adjoint(5, torch.zeros(s.shape, dtype=torch.float64))
    s = solver_for(case, "f64")
    s.set_state(torch.from_numpy(initial_field(case)))
    s.step(1)
    with pytest.raises(ATError):   # the adjoint starts from step 0
        s.adjoint(5, torch.zeros(s.shape, dtype=torch.float64))


def test_autograd_function_matches_oracle():
    from paper_1702_00496_amd import evolve
    case = _case("2d_o4_ab2")
    spec = dict(ndim=case["ndim"], n=case["n"], pe=case["pe"], dt=case["dt"], order=case["order"],
                c=case["c"], integrator=case["integrator"], precision="f64", L=case["L"], seed=0)
    u0 = torch.from_numpy(initial_field(case)).cuda().requires_grad_(True)
    alpha = torch.tensor(0.1, dtype=torch.float64, requires_grad=True)
    target = torch.from_numpy(_seed(case)).cuda()
    uN = evolve(u0, alpha, case["steps"], every=5, **spec)
    J = 0.5 * ((uN - target) ** 2).sum()
    J.backward()
    seed = (uN - target).detach().cpu().numpy()
    gu_o, ga_o = _oracle_grads(case, initial_field(case), seed)
    assert rel_l2(u0.grad.cpu(), gu_o) <= 1e-12
    assert float(alpha.grad) == pytest.approx(ga_o, rel=1e-12)


def test_adjoint_full_2d_workload_against_finite_differences():
    """1024^2, 16^2 PEs of 64^2, fourth order, L = 4, AB2, 2000 steps,
    J = 1/2 sum (u_T - target)^2 dx^2, checkpoints every 64 steps. Reference:
    central differences (eps = 1e-3) of the FP64 GPU forward along 16
    unit-variance Gaussian directions and in alpha (eps = 1e-5). J is exactly
    quadratic in u0 (u_T is linear in u0), so the u0 differences are exact up
    to rounding. The FP64 adjoint must agree to 1e-7, the FP32-bulk adjoint to
    1e-3 relative to the largest directional derivative."""
    from paper_1702_00496_amd import Solver
    from oracle.analytic import advected_modes
    cfg = W.config_2d_advdiff()
    n = cfg["n"]
    dV = (2 * math.pi / n[0]) * (2 * math.pi / n[1])
    steps, every = cfg["steps"], 64
    u0 = torch.from_numpy(W.eval_modes(cfg["modes"], n, 2)).cuda()
    prob = Problem(ndim=2, n=n[:2], pe=cfg["pe"][:2], dt=cfg["dt"], order=4, c=cfg["c"][:2], alpha=cfg["alpha"])
    target = advected_modes(prob, cfg["target_modes"], steps * cfg["dt"]).cuda()

    def make(alpha, precision):
        return Solver(ndim=2, n=n, pe=cfg["pe"], dt=cfg["dt"], order=4, c=cfg["c"], alpha=alpha,
                      integrator="ab2", precision=precision, L=cfg["L"], seed=cfg["seed"])

    def J_of(u_init, alpha=cfg["alpha"], precision="f64"):
        s = make(alpha, precision)
        s.set_state(u_init)
        s.step(steps)
        d = s.state().to(torch.float64) - target
        return 0.5 * float((d * d).sum()) * dV, d * dV

    _say(f"[adj] full 2-D workload: {n[0]}x{n[1]}, {steps} steps, every {every}")
    dirs = W.gaussian_field((16,) + tuple(u0.shape), seed=5, unit_l2=False)
    dirs = [torch.from_numpy(d / np.sqrt((d ** 2).mean())).cuda() for d in dirs]
    eps = 1e-3
    fd = []
    for d in dirs:
        jp, _ = J_of(u0 + eps * d)
        jm, _ = J_of(u0 - eps * d)
        fd.append((jp - jm) / (2 * eps))
    ea = 1e-5
    fda = (J_of(u0, cfg["alpha"] + ea)[0] - J_of(u0, cfg["alpha"] - ea)[0]) / (2 * ea)
    scale = max(abs(v) for v in fd)
    for precision, tol in (("f64", 1e-7), ("f32", 1e-3)):
        _, seed = J_of(u0, precision=precision)
        s = make(cfg["alpha"], precision)
        s.set_state(u0)
        gu, ga = s.adjoint(steps, seed, every)
        gu = gu.to(torch.float64)
        worst = 0.0
        for i, d in enumerate(dirs):
            ad = float((gu * d).sum())
            worst = max(worst, abs(ad - fd[i]) / scale)
            _say(f"[adj]   {precision} direction {i}: adjoint {ad:.9e}  fd {fd[i]:.9e}")
        _say(f"[adj]   {precision} alpha: adjoint {ga:.9e}  fd {fda:.9e}   worst direction {worst:.2e}")
        assert worst <= tol, (precision, worst)
        assert ga == pytest.approx(fda, rel=tol)


def test_adjoint_full_burgers_workload_against_finite_differences():
    """512^3 viscous Burgers, 16^3 PEs of 32^3, sixth order (T = 4), L = 8,
    Heun RK2, 200 FP32 steps: gradient of the final energy
    J = 1/2 sum u_T^2 dx^3 with respect to u0 along 3 unit-variance Gaussian
    directions and to the viscosity, against central differences of the FP64
    GPU forward (eps = 1e-3 and 1e-5; J is not quadratic here, the O(eps^2)
    error stays below 1e-5 relative)."""
    from paper_1702_00496_amd import Solver
    cfg = W.config_3d_burgers()
    n = cfg["n"]
    dV = (2 * math.pi / n[0]) ** 3
    steps, every = cfg["steps"], 40
    u0 = torch.from_numpy(W.burgers_spectrum_field(n[0], 3, seed=cfg["seed"])).cuda()

    def make(alpha, precision):
        return Solver(ndim=3, n=n, pe=cfg["pe"], dt=cfg["dt"], order=6, equation="burgers", alpha=alpha,
                      integrator="rk2", precision=precision, L=cfg["L"], T=cfg["T"], seed=cfg["seed"])

    def J_of(u_init, alpha=cfg["alpha"], precision="f64"):
        s = make(alpha, precision)
        s.set_state(u_init)
        s.step(steps)
        u = s.state().to(torch.float64)
        del s
        return 0.5 * float((u * u).sum()) * dV, u * dV

    _say(f"[adj] full Burgers workload: {n[0]}^3, {steps} steps, every {every}")
    g = torch.Generator(device="cuda").manual_seed(5)
    dirs = [torch.randn(u0.shape, generator=g, device="cuda", dtype=torch.float64) for _ in range(3)]
    eps = 1e-3
    fd = []
    for d in dirs:
        fd.append((J_of(u0 + eps * d)[0] - J_of(u0 - eps * d)[0]) / (2 * eps))
        _say(f"[adj]   fd {fd[-1]:.9e}")
    ea = 1e-5
    fda = (J_of(u0, cfg["alpha"] + ea)[0] - J_of(u0, cfg["alpha"] - ea)[0]) / (2 * ea)
    _, seed = J_of(u0, precision="f32")
    s = make(cfg["alpha"], "f32")
    s.set_state(u0)
    gu, ga = s.adjoint(steps, seed, every)
    gu = gu.to(torch.float64)
    scale = max(abs(v) for v in fd)
    worst = 0.0
    for i, d in enumerate(dirs):
        ad = float((gu * d).sum())
        worst = max(worst, abs(ad - fd[i]) / scale)
        _say(f"[adj]   direction {i}: adjoint {ad:.9e}  fd {fd[i]:.9e}")
    _say(f"[adj]   nu: adjoint {ga:.9e}  fd {fda:.9e}   worst direction {worst:.2e}")
    assert worst <= 1e-3
    assert ga == pytest.approx(fda, rel=1e-3)


def _random_case(seed):
    """A seeded configuration the adjoint covers (time-expanded schemes;
    Euler, AB2, Heun RK2; advection-diffusion or Burgers; every delay mode)."""
    import random
    rng = random.Random(seed)
    ndim = rng.choice((1, 1, 2, 2, 3))
    order = rng.choice((2, 4, 6))
    s = order // 2
    n, pe = [], []
    for a in range(ndim):
        p = rng.randint(1, 4) if ndim < 3 else rng.randint(1, 2)
        n.append(p * rng.randint(2 * s, 2 * s + (10 if ndim == 1 else 4 if ndim == 2 else 2)))
        pe.append(p)
    equation = rng.choice(("advdiff", "advdiff", "burgers"))
    alpha = 0.05 if equation == "burgers" else 0.1
    dx = 2 * math.pi / max(n)
    case = dict(ndim=ndim, n=tuple(n), pe=tuple(pe), order=order, integrator=rng.choice(("euler", "ab2", "rk2")),
                equation=equation, c=tuple(round(rng.uniform(-1, 1), 3) for _ in range(ndim)), alpha=alpha,
                L=rng.randint(1, 6), T=rng.choice((0, 0, 1)), mode=rng.choice(("rng", "rng", "zero", "sync")),
                seed=rng.randint(0, 2 ** 31), steps=rng.randint(4, 20), every=rng.randint(2, 8),
                dt=min(0.005 * dx * dx / alpha, 0.02 * dx), ic_seed=rng.randint(0, 100))
    return case, rng.choice(("f64", "f32"))


@pytest.mark.parametrize("seed", range(48))
def test_adjoint_random_configuration_matches_oracle_gradients(seed):
    case, precision = _random_case(7000 + seed)
    _say(f"[adj] random {seed}: {case} {precision}")
    u0 = initial_field(case)
    sd = _seed(case)
    gu_o, ga_o = _oracle_grads(case, u0, sd)
    s, gu, ga = _gpu_grads(case, u0, sd, precision)
    tol = 1e-12 if precision == "f64" else 1e-5
    _say(f"[adj]   du0 errors {field_errors(gu, gu_o, oracle_for(case, u0).prob)}   "
         f"dalpha rel {abs(ga - ga_o) / max(abs(ga_o), 1e-300):.3e}")
    assert rel_l2(gu, gu_o) <= tol, (case, precision, rel_l2(gu, gu_o))
    assert ga == pytest.approx(ga_o, rel=tol if precision == "f64" else 1e-4), (case, precision, ga, ga_o)
