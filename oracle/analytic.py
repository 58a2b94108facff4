"""Exact solution of linear advection-diffusion on a periodic box (oracle).

Test infrastructure (oracle). Sec. 5.1, eq. ana_sol: every Fourier mode of the
initial field (eq. IC) is advected with speed c and damped by exp(-alpha
|kappa|^2 t). The printed phase reads sin(kappa x + phi - c t); this oracle
takes sin(kappa . (x - c t) + phi), the solution of u_t + c . grad u =
alpha lap u (the two coincide for |kappa| = 1, the single-mode case of the
first configuration). With c = 0 it is the heat-equation solution.
"""
import math

import torch


def grid_axes(prob):
    """Node coordinates x_i = i * length / n per axis, broadcastable to (nz, ny, nx)."""
    xs = []
    for a in range(3):
        x = torch.arange(prob.n[a], dtype=torch.float64) * (prob.length / prob.n[a])
        shape = [1, 1, 1]
        shape[2 - a] = prob.n[a]
        xs.append(x.reshape(shape))
    return xs


def advected_modes(prob, modes, t):
    """u_a(x, t) = sum_kappa A exp(-alpha |kappa|^2 t) sin(kappa . (x - c t) + phi).

    ``modes``: iterable of (kappa (3 ints), amplitude, phase)."""
    xs = grid_axes(prob)
    out = torch.zeros(prob.shape, dtype=torch.float64)
    for kap, amp, phi in modes:
        k2 = sum(float(kv) ** 2 for kv in kap)
        arg = torch.zeros(prob.shape, dtype=torch.float64) + float(phi)
        for a in range(prob.ndim):
            arg = arg + float(kap[a]) * (xs[a] - prob.c[a] * t)
        out = out + float(amp) * math.exp(-prob.alpha * k2 * t) * torch.sin(arg)
    return out
