"""Pins of the oracle's exact solution, error measures and boundary set.

- The exact solution (Sec. 5.1 eq. ana_sol, reading: the phase is
  kappa . (x - c t) + phi) solves u_t + c . grad u = alpha lap u: checked with
  spectral space derivatives and a centred time difference, which a dropped
  kappa, a flipped sign of c or a wrong decay rate fails.
- Error measures (Sec. 4 averages, Sec. 5.1 pointwise error) on hand-computed
  arrays.
- The boundary set I_B (Sec. 2: points whose stencil reaches across a PE face)
  on a tiny grid written out by hand, and its size in 3-D by counting.
"""
import math

import pytest
import torch

from oracle.analytic import advected_modes
from oracle.norms import binned_mean_var, ensemble_mean_var, error_norms
from oracle.solver import Problem, boundary_mask


def _spectral_derivative(u, axis_dim, length, order):
    n = u.shape[axis_dim]
    k = torch.fft.fftfreq(n, d=length / n) * 2.0 * math.pi
    shape = [1, 1, 1]
    shape[axis_dim] = n
    k = k.reshape(shape).to(torch.complex128)
    uh = torch.fft.fft(u.to(torch.complex128), dim=axis_dim)
    return torch.fft.ifft(uh * (1j * k) ** order, dim=axis_dim).real


@pytest.mark.parametrize("ndim,c,modes", [
    (1, (1.0, 0.0, 0.0), [((2, 0, 0), 1.0, 0.3)]),
    (1, (-0.7, 0.0, 0.0), [((3, 0, 0), 2.0, 1.1), ((1, 0, 0), 0.5, 0.0)]),
    (3, (1.0, -0.5, 0.25), [((1, 2, 3), 1.0, 0.4), ((0, 0, 2), 1.5, 2.0)]),
])
def test_exact_solution_solves_advection_diffusion(ndim, c, modes):
    n = 16
    prob = Problem(ndim=ndim, n=(n,) * ndim, pe=(1,) * ndim, dt=1e-3, order=2,
                   c=c[:ndim], alpha=0.1)
    t, h = 0.37, 1e-4
    u = advected_modes(prob, modes, t)
    ut = (advected_modes(prob, modes, t + h) - advected_modes(prob, modes, t - h)) / (2 * h)
    resid = ut.clone()
    for a in range(ndim):
        dim = 2 - a
        resid += c[a] * _spectral_derivative(u, dim, prob.length, 1)
        resid -= prob.alpha * _spectral_derivative(u, dim, prob.length, 2)
    scale = float(ut.abs().max()) + 1.0
    assert float(resid.abs().max()) / scale < 1e-7


def test_exact_solution_at_t0_is_the_initial_series():
    prob = Problem(ndim=1, n=(8,), pe=(1,), dt=1e-3, order=2, c=(1.0,), alpha=0.1)
    u = advected_modes(prob, [((1, 0, 0), 1.0, 0.0)], 0.0).reshape(-1)
    x = torch.arange(8, dtype=torch.float64) * (2 * math.pi / 8)
    assert torch.allclose(u, torch.sin(x), atol=1e-15)


def test_error_norms_hand_computed():
    u = torch.tensor([3.0, -4.0, 0.0, 0.0], dtype=torch.float64).reshape(1, 1, 4)
    ref = torch.zeros_like(u)
    bmask = torch.tensor([True, False, False, True]).reshape(1, 1, 4)
    e = error_norms(u, ref, bmask)
    assert e["l1"] == pytest.approx(7.0 / 4.0, rel=1e-15)
    assert e["l2"] == pytest.approx(2.5, rel=1e-15)
    assert e["linf"] == 4.0
    assert e["l1_b"] == pytest.approx(1.5, rel=1e-15)
    assert e["l2_b"] == pytest.approx(math.sqrt(4.5), rel=1e-15)
    assert e["l1_i"] == pytest.approx(2.0, rel=1e-15)
    assert e["l2_i"] == pytest.approx(math.sqrt(8.0), rel=1e-15)


def test_ensemble_mean_and_unbiased_variance():
    m, v = ensemble_mean_var([1.0, 2.0, 3.0, 4.0])
    assert m == 2.5
    assert v == pytest.approx(5.0 / 3.0, rel=1e-15)


def test_binned_mean_and_variance_by_hand():
    """Six members in two order groups and two dx bins (edges 0.1, 0.2, 0.4):
    bin membership is half-open, a member outside every bin is dropped, a bin
    with one member has variance 0 and an empty bin counts 0."""
    dx = [0.1, 0.15, 0.2, 0.3, 0.4, 0.12]
    vals = [1.0, 3.0, 10.0, 14.0, 99.0, 5.0]
    groups = [0, 0, 0, 0, 0, 1]
    t = binned_mean_var(dx, vals, groups, [0.1, 0.2, 0.4], ngroups=2)
    assert t[0][0] == (2, 0.125, 2.0, 2.0)            # members 0, 1: mean 2, var ((1)^2 + (1)^2) / 1
    assert t[0][1][0] == 2 and t[0][1][2] == 12.0 and t[0][1][3] == 8.0   # members 2, 3 (0.4 excluded)
    assert t[0][1][1] == pytest.approx(0.25, rel=1e-15)
    assert t[1][0] == (1, 0.12, 5.0, 0.0)
    assert t[1][1] == (0, 0.0, 0.0, 0.0)


def test_boundary_set_one_d_by_hand():
    prob = Problem(ndim=1, n=(16,), pe=(2,), dt=1e-3, order=4, c=(1.0,), alpha=0.1)
    m = boundary_mask(prob).reshape(-1).nonzero().reshape(-1).tolist()
    assert m == [0, 1, 6, 7, 8, 9, 14, 15]


def test_boundary_set_three_d_count():
    b, s, pe = 8, 2, 2
    prob = Problem(ndim=3, n=(b * pe,) * 3, pe=(pe,) * 3, dt=1e-3, order=2 * s, c=(1.0, 1.0, 1.0),
                   alpha=0.1)
    m = boundary_mask(prob)
    assert int(m.sum()) == pe ** 3 * (b ** 3 - (b - 2 * s) ** 3)
