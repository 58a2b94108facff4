"""Gradients of a final-time function through the AT time steps (oracle).

Test infrastructure (oracle). Reverse-mode automatic differentiation (torch
autograd) of the oracle's own forward steps in float64, for the derivative of
J(u^N) with respect to the initial field u^0 and the diffusivity alpha. The
forward steps are those of ``oracle.solver`` (Sec. 2 eqs. general_deriv,
general_deriv_async; Sec. 3.4 Example 3 eq. cd4-at; Sec. 4.1 eqs. time_disc,
time_ab2); the delays of every step are fixed by the generator, so u^N is a
linear function of u^0 for advection-diffusion and a polynomial in alpha.
This route shares nothing with a hand-written transpose of the step.
"""
import torch

from .solver import Oracle


def forward(prob, dm, u0, alpha, nsteps, key=None):
    """u^N from u^0 (tensors may require grad)."""
    o = Oracle(prob, dm, u0, alpha=alpha, key=key)
    return o.run(nsteps)


def gradients(prob, dm, u0, alpha, nsteps, seed, key=None):
    """(dJ/du^0, dJ/dalpha) for the linear functional J = <seed, u^N>, whose
    gradient with respect to u^N is seed: the vector-Jacobian product that a
    reverse sweep started from lambda^N = seed returns."""
    u = torch.as_tensor(u0, dtype=torch.float64).clone().requires_grad_(True)
    a = torch.tensor(float(alpha), dtype=torch.float64, requires_grad=True)
    uN = forward(prob, dm, u, a, nsteps, key)
    J = (torch.as_tensor(seed, dtype=torch.float64) * uN).sum()
    gu, ga = torch.autograd.grad(J, (u, a))
    return gu.detach(), float(ga)

