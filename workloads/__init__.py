"""Seeded synthetic inputs for the AT solver, shared by tests, smoke and bench.

This module only draws random numbers and evaluates initial fields on the
grid. It holds none of the method's arithmetic (no stencils, no delays, no
time stepping), so the oracle and the GPU library can both consume what it
produces without sharing code.

Initial fields follow the multi-scale form of Sec. 5.1 eq. IC,
u(x, 0) = sum_kappa A(kappa) sin(kappa . x + phi_kappa), with phases drawn
from numpy's PCG64 generator. The paper's runs use no external data set: all
its inputs are such synthetic superpositions.
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def phases(seed, count):
    return np.random.Generator(np.random.PCG64(seed)).uniform(0.0, TWO_PI, size=count)


def make_modes(kappas, amps, seed=None, phis=None):
    """List of (kappa (3 ints), amplitude, phase)."""
    kappas = [tuple(int(v) for v in k) + (0,) * (3 - len(k)) for k in kappas]
    if phis is None:
        phis = phases(seed, len(kappas)) if seed is not None else [0.0] * len(kappas)
    return [(k, float(a), float(p)) for k, a, p in zip(kappas, amps, phis)]


def eval_modes(modes, n, ndim, length=TWO_PI):
    """sum A sin(kappa . x + phi) on nodes x_i = i * length / n, shape (nz, ny, nx), float64."""
    n = tuple(n) + (1,) * (3 - len(n))
    axes = []
    for a in range(3):
        x = np.arange(n[a], dtype=np.float64) * (length / n[a])
        shape = [1, 1, 1]
        shape[2 - a] = n[a]
        axes.append(x.reshape(shape))
    out = np.zeros((n[2], n[1], n[0]), dtype=np.float64)
    for kap, amp, phi in modes:
        arg = np.full(out.shape, phi, dtype=np.float64)
        for a in range(ndim):
            arg = arg + kap[a] * axes[a]
        out += amp * np.sin(arg)
    return out


def gaussian_field(shape, seed, unit_l2=True):
    g = np.random.Generator(np.random.PCG64(seed)).standard_normal(size=shape)
    if unit_l2:
        g = g / np.sqrt((g * g).sum())
    return g


# --------------------------------------------------------------- configurations
def dt_from_ralpha(r_alpha, alpha, n, length=TWO_PI):
    dx = length / n
    return r_alpha * dx * dx / alpha


def config_1d_advdiff(n=256, pe=8, steps=1000, L=3, seed=0, order=2):
    """1-D advection-diffusion, u0 = sin x, c = 1, alpha = 0.1, diffusive CFL 0.1."""
    alpha = 0.1
    return dict(
        name=f"ad1d_n{n}_p{pe}",
        ndim=1, n=(n, 1, 1), pe=(pe, 1, 1), order=order, equation="advdiff",
        c=(1.0, 0.0, 0.0), alpha=alpha, integrator="euler" if order == 2 else "ab2",
        dt=dt_from_ralpha(0.1, alpha, n), steps=steps,
        L=L, T=order // 2 + 1, seed=seed,
        modes=make_modes([(1,)], [1.0], phis=[0.0]),
    )


def config_3d_advdiff(n=256, b=32, steps=500, L=4, seed=1, r_alpha=0.02):
    """3-D advection-diffusion, fourth order, AB2, four plane waves with random phases."""
    alpha = 0.1
    return dict(
        name=f"ad3d_n{n}_b{b}",
        ndim=3, n=(n, n, n), pe=(n // b,) * 3, order=4, equation="advdiff",
        c=(1.0, 1.0, 1.0), alpha=alpha, integrator="ab2",
        dt=dt_from_ralpha(r_alpha, alpha, n), steps=steps,
        L=L, T=3, seed=seed,
        modes=make_modes([(3, 0, 0), (0, 4, 0), (0, 0, 5), (1, 2, 3)],
                         [2.0, 0.5, 1.5, 1.0], seed=seed),
    )


def config_2d_advdiff(n=1024, b=64, steps=2000, L=4, seed=3, r_alpha=0.01):
    """2-D advection-diffusion (adjoint workload), fourth order, AB2.

    r_alpha = alpha dt / dx^2 = 0.01: with L = 4 the AT extrapolation makes
    the 2-D AB2 step unstable at 0.05 (a 1e-6 perturbation grows 1e8-fold in
    250 steps, measured with the oracle) although the synchronous scheme is
    stable up to 3/32; 0.03 still damps perturbations."""
    alpha = 0.1
    return dict(
        name=f"ad2d_n{n}_b{b}",
        ndim=2, n=(n, n, 1), pe=(n // b, n // b, 1), order=4, equation="advdiff",
        c=(1.0, 1.0, 0.0), alpha=alpha, integrator="ab2",
        dt=dt_from_ralpha(r_alpha, alpha, n), steps=steps,
        L=L, T=3, seed=seed,
        modes=make_modes([(3, 0), (0, 4), (5, 5), (1, 2)], [2.0, 0.5, 1.5, 1.0], seed=seed),
        target_modes=make_modes([(3, 0), (0, 4), (5, 5), (1, 2)], [2.0, 0.5, 1.5, 1.0], seed=seed + 1),
    )


def burgers_spectrum_field(n, ndim, seed=2, kpeak=4.0, urms=0.5):
    """Random-phase field with energy spectrum E(k) ~ k^4 exp(-2 (k/kpeak)^2),
    synthesised by an inverse real FFT and scaled to the given rms."""
    rs = np.random.Generator(np.random.PCG64(seed))
    shape = (n,) * ndim
    kk = [np.fft.fftfreq(n, d=1.0 / n)] * (ndim - 1) + [np.fft.rfftfreq(n, d=1.0 / n)]
    grids = np.meshgrid(*kk, indexing="ij")
    kmag = np.sqrt(sum(g * g for g in grids))
    with np.errstate(divide="ignore", invalid="ignore"):
        espec = kmag ** 4 * np.exp(-2.0 * (kmag / kpeak) ** 2)
        amp = np.where(kmag > 0, np.sqrt(espec / np.maximum(kmag, 1e-30) ** (ndim - 1)), 0.0)
    ph = rs.uniform(0.0, TWO_PI, size=amp.shape)
    spec = amp * np.exp(1j * ph)
    u = np.fft.irfftn(spec, s=shape, axes=tuple(range(ndim)))
    u = u * (urms / np.sqrt((u * u).mean()))
    u3 = u.reshape((1,) * (3 - ndim) + u.shape)   # (nz, ny, nx)
    return np.ascontiguousarray(u3)


def config_3d_burgers(n=512, b=32, steps=200, L=8, seed=2, r_alpha=0.002):
    """3-D viscous Burgers, sixth order, Heun RK2, spectrum peaked at k = 4.

    r_alpha = nu dt / dx^2 = 0.002: with L = 8 and four time levels the AT
    extrapolation weights reach 799 in sum of magnitudes and larger steps
    leave the stable range (measured with the oracle)."""
    nu = 0.01
    return dict(
        name=f"vb3d_n{n}_b{b}",
        ndim=3, n=(n, n, n), pe=(n // b,) * 3, order=6, equation="burgers",
        c=(0.0, 0.0, 0.0), alpha=nu, integrator="rk2",
        dt=dt_from_ralpha(r_alpha, nu, n), steps=steps,
        L=L, T=4, seed=seed, modes=None,
    )


def ensemble_instances(count=512, seed=3, b=64, nmin=1024, nmax=65536,
                       r_alpha=(0.1, 0.005)):
    """Descriptors of a delay ensemble of independent 1-D problems.

    N_i = b * round(exp(U(ln nmin, ln nmax)) / b); even members are second
    order (Euler), odd members fourth order (AB2); L_i drawn from {2, 4, 8};
    phases and a 64-bit delay generator key per member. Diffusive CFL
    r_alpha = alpha dt / dx^2 is 0.1 for second order and 0.005 for fourth
    order: with L = 8, fourth-order AB2 amplifies perturbations
    intermittently at 0.02 (a 1e-6 perturbation grows 1e3-fold within 2000
    steps for some delay sequences, measured with the oracle) and it is
    unstable at 0.05."""
    rs = np.random.Generator(np.random.PCG64(seed))
    logn = rs.uniform(math.log(nmin), math.log(nmax), size=count)
    ns = [int(b * max(1, round(math.exp(v) / b))) for v in logn]
    Ls = [int(v) for v in rs.choice([2, 4, 8], size=count)]
    ph = rs.uniform(0.0, TWO_PI, size=(count, 3))
    keys = rs.integers(0, 2 ** 64, size=count, dtype=np.uint64)
    out = []
    for i in range(count):
        order = 2 if i % 2 == 0 else 4
        ra = r_alpha[0] if order == 2 else r_alpha[1]
        out.append(dict(
            n=ns[i], pe=ns[i] // b, order=order, L=Ls[i], T=order // 2 + 1,
            integrator="euler" if order == 2 else "ab2",
            alpha=0.1, c=1.0, dt=dt_from_ralpha(ra, 0.1, ns[i]), seed=int(keys[i]),
            modes=make_modes([(3,), (4,), (5,)], [2.0, 0.5, 1.5], phis=list(ph[i])),
        ))
    return out
