"""Pins of the oracle's gradients (reverse-mode autograd of its forward steps)
against finite differences of the forward steps themselves.

For advection-diffusion with the delays of every step fixed by the
generator, u^N is linear in u^0: central differences of the forward map are
exact up to rounding, so the full Jacobian can be built column by column on a
tiny grid and J^T seed compared with the reverse sweep. The alpha derivative
is checked by a central difference in alpha (error O(eps^2)).
"""
import math

import numpy as np
import pytest
import torch

from oracle.adjoint import forward, gradients
from oracle.solver import DelayModel, Problem


def _setup(ndim, n, pe, order, integ, L, mode="rng", ra=0.05, c=(1.0, -0.5, 0.3)):
    dx = 2 * math.pi / min(n)
    prob = Problem(ndim=ndim, n=n, pe=pe, dt=ra * dx * dx / 0.1, order=order, c=c[:ndim], alpha=0.1,
                   integrator=integ)
    dm = DelayModel(L=L, mode=mode, seed=7)
    rs = np.random.default_rng(3)
    u0 = torch.from_numpy(rs.standard_normal(prob.shape))
    seed = torch.from_numpy(rs.standard_normal(prob.shape))
    return prob, dm, u0, seed


@pytest.mark.parametrize("integ,order,L,mode", [("euler", 2, 3, "rng"), ("ab2", 4, 3, "rng"),
                                                ("ab2", 2, 2, "sync"), ("euler", 4, 4, "zero")])
def test_gradient_is_jacobian_transpose_times_seed(integ, order, L, mode):
    prob, dm, u0, seed = _setup(1, (16,), (2,), order, integ, L, mode)
    steps = 9
    gu, _ = gradients(prob, dm, u0, 0.1, steps, seed)
    eps = 1e-3
    jac = torch.zeros(16, 16, dtype=torch.float64)
    flat = u0.reshape(-1)
    for i in range(16):
        e = torch.zeros_like(flat)
        e[i] = eps
        up = forward(prob, dm, (flat + e).reshape(u0.shape), 0.1, steps).reshape(-1)
        um = forward(prob, dm, (flat - e).reshape(u0.shape), 0.1, steps).reshape(-1)
        jac[:, i] = (up - um) / (2 * eps)
    want = jac.T @ seed.reshape(-1)
    assert torch.allclose(gu.reshape(-1), want, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("ndim,n,pe,order,integ", [(2, (12, 10), (2, 2), 4, "ab2"), (3, (8, 8, 8), (2, 2, 2), 2, "euler")])
def test_gradient_matches_directional_differences(ndim, n, pe, order, integ):
    prob, dm, u0, seed = _setup(ndim, n, pe, order, integ, 3)
    steps = 7
    gu, ga = gradients(prob, dm, u0, 0.1, steps, seed)
    rs = np.random.default_rng(5)
    for _ in range(3):
        d = torch.from_numpy(rs.standard_normal(prob.shape))
        eps = 1e-3
        up = forward(prob, dm, u0 + eps * d, 0.1, steps)
        um = forward(prob, dm, u0 - eps * d, 0.1, steps)
        fd = float((seed * (up - um)).sum()) / (2 * eps)
        assert float((gu * d).sum()) == pytest.approx(fd, rel=1e-9, abs=1e-11)
    ea = 1e-5
    ja = float((seed * forward(prob, dm, u0, 0.1 + ea, steps)).sum())
    jb = float((seed * forward(prob, dm, u0, 0.1 - ea, steps)).sum())
    assert ga == pytest.approx((ja - jb) / (2 * ea), rel=1e-6)


def test_burgers_rk2_gradient_matches_directional_differences():
    """Nonlinear case (viscous Burgers, Heun RK2 with the predictor's own
    history): central differences with eps = 1e-6 carry an O(eps^2) error."""
    dx = 2 * math.pi / 48
    prob = Problem(ndim=1, n=(48,), pe=(4,), dt=0.01 * dx * dx / 0.05, order=4, equation="burgers",
                   alpha=0.05, integrator="rk2")
    dm = DelayModel(L=3, mode="rng", seed=9)
    rs = np.random.default_rng(4)
    u0 = torch.from_numpy(0.5 * np.sin(np.arange(48) * dx) + 0.1 * rs.standard_normal(48)).reshape(1, 1, 48)
    seed = torch.from_numpy(rs.standard_normal((1, 1, 48)))
    steps = 12
    gu, ga = gradients(prob, dm, u0, 0.05, steps, seed)
    for _ in range(3):
        d = torch.from_numpy(rs.standard_normal((1, 1, 48)))
        eps = 1e-6
        up = forward(prob, dm, u0 + eps * d, 0.05, steps)
        um = forward(prob, dm, u0 - eps * d, 0.05, steps)
        fd = float((seed * (up - um)).sum()) / (2 * eps)
        assert float((gu * d).sum()) == pytest.approx(fd, rel=1e-7)
    ea = 1e-6
    ja = float((seed * forward(prob, dm, u0, 0.05 + ea, steps)).sum())
    jb = float((seed * forward(prob, dm, u0, 0.05 - ea, steps)).sum())
    assert ga == pytest.approx((ja - jb) / (2 * ea), rel=1e-6)
