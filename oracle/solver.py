"""AT finite-difference time stepping, FP64, full-field history (oracle).

Test infrastructure (oracle): plain torch CPU float64 operations, written for
readability, not speed. Shares no code with the product library.

What one step n -> n+1 computes:

1. Delays (Sec. 2, "asynchronous computing"; Sec. 5.1 simulation of delays).
   Every PE p draws, for each axis and each side, one delay k in [0, L-1]
   (uniform over all buffer points of that face, the "uniform delay" class of
   Table class). Start-up clamp: k <= max(0, n - T + 1).
2. Spatial derivatives (Sec. 2 eq. general_deriv; Sec. 3.4 Example 3 eq.
   cd4-at; Tables atschemes-left/right). Points whose stencil stays inside
   their PE (the set I_I) take the standard central difference CD_a on level
   n. A point of I_B, whose stencil reaches taps in the buffer set B across
   face sigma of its PE, takes
        sum_{m=0}^{T-1} c_m(k_sigma) * [ sum_o c_o V_o^{(m)} ],
   with V_o^{(m)} = u^n_{i+o} for taps inside the PE and u^{n-k-m}_{i+o} for
   taps across the face; c_m(k) solves the time-level system of Example 3
   (oracle.coeffs.time_level_weights). T = 1 is the asynchronous standard
   scheme of eq. general_deriv_async.
   Multi-dimensional problems apply this per axis with that axis' face delay
   (no mixed derivatives occur).
   Space-expanded single-level family (Tables atschemes-left/right, rows
   (2,1,2), (1,2,2)a, (2,2,2)a; Sec. 5.1 Cases 2 and 3), second-order CD
   only: the point next to a face whose delay k is positive takes an
   asymmetric stencil over own points at level n and 2 or 3 buffer points at
   the one level n-k (oracle.coeffs.space_expanded_at_stencil). Reading:
   these stencils are not the CD at k = 0 (Sec. 5.1 says so) and are used at
   "communication delayed" buffer points (caption of the convergence figure
   of Cases 2-5), so a face with k = 0 keeps the standard CD2; the paper's
   delay-free curve then has the synchronous slope -2, as it reports.
   Scheme "space212": first derivative (1,2,2)a, second (2,1,2);
   "space222": (1,2,2)a and (2,2,2)a.
3. Right-hand side (Sec. 5 eq. general): advection-diffusion
   f = -c . grad u + alpha lap u, viscous Burgers f = -u (sum_d du/dx_d) +
   alpha lap u.
4. Time update (Sec. 4.1 eqs. time_disc, time_ab2): Euler; AB2 (Euler at
   n = 0); AB3 (Euler, then AB2, then AB3); Heun RK2. The paper only treats
   linear multistep methods. Reading used for RK2: each stage is a field of
   its own with its own history, and every stage derivative is an AT
   derivative over that stage's past levels. Stage 1 uses levels of u,
   stage 2 levels of the predictor u* = u + dt f(u), both with the face's
   delay k of the step. With k = 0 this is the synchronous Heun method.

Layout: fields are (nz, ny, nx) float64 tensors, x fastest; axis 0 = x
(tensor dim 2), axis 1 = y (dim 1), axis 2 = z (dim 0). Grid nodes are
x_i = i * length / n. Everything is periodic.
"""
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Optional, Sequence
import math

import torch

from . import coeffs, rng


@dataclass
class Problem:
    ndim: int
    n: Sequence[int]                 # points per axis (x, y, z); unused axes = 1
    pe: Sequence[int]                # PEs per axis
    dt: float
    order: int = 2                   # spatial order a (2, 4, 6)
    equation: str = "advdiff"        # "advdiff" | "burgers"
    c: Sequence[float] = (0.0, 0.0, 0.0)
    alpha: float = 0.0               # diffusivity (viscosity for Burgers)
    integrator: str = "euler"        # "euler" | "ab2" | "ab3" | "rk2"
    length: float = 2.0 * math.pi

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n) + (1,) * (3 - len(self.n))
        self.pe = tuple(int(v) for v in self.pe) + (1,) * (3 - len(self.pe))
        self.c = tuple(float(v) for v in self.c) + (0.0,) * (3 - len(self.c))
        if self.ndim not in (1, 2, 3):
            raise ValueError("ndim must be 1, 2 or 3")
        s = self.order // 2
        for a in range(3):
            if self.n[a] % self.pe[a]:
                raise ValueError("points per axis must be a multiple of PEs per axis")
            if a < self.ndim and self.n[a] // self.pe[a] < 2 * s:
                raise ValueError("PE edge must hold at least 2s points")
            if a >= self.ndim and (self.n[a] != 1 or self.pe[a] != 1):
                raise ValueError("unused axes must have one point and one PE")

    @property
    def s(self):
        return self.order // 2

    @property
    def b(self):
        return tuple(self.n[a] // self.pe[a] for a in range(3))

    @property
    def dx(self):
        return tuple(self.length / self.n[a] for a in range(3))

    @property
    def n_pe(self):
        return self.pe[0] * self.pe[1] * self.pe[2]

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])


@dataclass
class DelayModel:
    L: int = 1
    T: int = 0                         # 0 -> order/2 + 1 (time-expanded AT)
    mode: str = "rng"                  # "rng" | "zero" | "sync" | "host"
    seed: int = 0
    weights: Optional[Sequence[int]] = None   # integer bin weights, None = uniform
    host: Optional[object] = None      # int array [nsteps, n_pe, ndim, 2] for mode "host"
    scheme: str = "time"               # "time" | "space212" | "space222" | "nonuniform212"

    def levels(self, order):
        if self.scheme != "time":   # single-level families
            return 1
        return self.T if self.T > 0 else order // 2 + 1


def delay_table(prob: Problem, dm: DelayModel, n: int, key: Optional[int] = None):
    """Delays used at step n: LongTensor [n_pe, ndim, 2] (after the start-up clamp)."""
    T = dm.levels(prob.order)
    K = torch.zeros((prob.n_pe, prob.ndim, 2), dtype=torch.long)
    if dm.mode in ("zero", "sync"):
        return K
    if dm.mode == "host":
        raw = torch.as_tensor(dm.host[n], dtype=torch.long).reshape(prob.n_pe, prob.ndim, 2)
        for p in range(prob.n_pe):
            for a in range(prob.ndim):
                for sd in range(2):
                    K[p, a, sd] = rng.clamp_startup(int(raw[p, a, sd]), n, T)
        return K
    thr = rng.thresholds(dm.L, dm.weights)
    k0 = dm.seed if key is None else key
    for p in range(prob.n_pe):
        for a in range(prob.ndim):
            for sd in range(2):
                face = p * 2 * prob.ndim + 2 * a + sd
                K[p, a, sd] = rng.clamp_startup(rng.raw_delay(k0, n, face, thr), n, T)
    return K


def point_delay_table(prob: Problem, dm: DelayModel, n: int, key: Optional[int] = None):
    """Delay of the second buffer point of every face at step n (non-uniform
    scheme): LongTensor [n_pe, ndim, 2]. The first buffer point takes the face
    delay of ``delay_table``; the second its own draw from the same generator
    with the face index shifted by the number of faces, n_pe * 2 * ndim."""
    K = torch.zeros((prob.n_pe, prob.ndim, 2), dtype=torch.long)
    if dm.mode in ("zero", "sync"):
        return K
    if dm.mode != "rng":
        raise ValueError("per-point delays come from the generator (mode rng) or are zero")
    thr = rng.thresholds(dm.L, dm.weights)
    k0 = dm.seed if key is None else key
    nfaces = prob.n_pe * 2 * prob.ndim
    for p in range(prob.n_pe):
        for a in range(prob.ndim):
            for sd in range(2):
                face = p * 2 * prob.ndim + 2 * a + sd
                K[p, a, sd] = rng.clamp_startup(rng.raw_delay(k0, n, nfaces + face, thr), n, 1)
    return K


def nonuniform_delays(k1, k2):
    """Delays (k1, k2) of the nearest and second buffer point as the
    non-uniform scheme uses them. Sec. 3.4 Example 1: eq. ex1-0 is singular
    where 3 k1 = k2 and is to be avoided by altering a delay; with k1 >= 1 the
    nearest point takes the next older level, k1 + 1 (always stored, and then
    3 k1 - k2 = 3). Both zero: the point is synchronous (None: the CD2 is used)."""
    if k1 == 0 and k2 == 0:
        return None
    if 3 * k1 == k2:
        k1 += 1
    return k1, k2


def _fr(x):
    return float(Fraction(x))


class Oracle:
    """One AT simulation. ``u0`` is a float64 tensor of shape prob.shape."""

    def __init__(self, prob: Problem, dm: DelayModel, u0, alpha=None, key=None):
        self.prob = prob
        self.dm = dm
        self.key = key
        self.T = dm.levels(prob.order)
        if self.T < 1 or self.T > 4:
            raise ValueError("T must be 1..4")
        if dm.mode != "sync" and dm.L < 1:
            raise ValueError("L must be >= 1")
        # alpha may be a tensor (for autograd) or a float
        self.alpha = prob.alpha if alpha is None else alpha
        self.taps1 = [_fr(c) for c in coeffs.central_difference(1, prob.order)]
        self.taps2 = [_fr(c) for c in coeffs.central_difference(2, prob.order)]
        # c_m(k) for every delay value
        self.wtab = {k: [_fr(c) for c in coeffs.time_level_weights(k, self.T)]
                     for k in range(0, max(dm.L, 1))}
        # space-expanded family: boundary stencils per derivative and side
        self.space = None
        self.nonuniform = None
        if dm.scheme == "nonuniform212":
            if prob.order != 2:
                raise ValueError("the non-uniform-delay scheme extends the second-order CD")
            if any(prob.b[a] < 2 for a in range(prob.ndim)):
                raise ValueError("nonuniform212 needs PE edges of at least 2 points")
            if dm.mode == "host":
                raise ValueError("nonuniform212 draws its per-point delays from the generator")
            self.nonuniform = {}     # (k1, k2) -> {d: {j: c}} at a right face, from eq. cond
        elif dm.scheme != "time":
            if dm.scheme not in ("space212", "space222"):
                raise ValueError(f"unknown scheme {dm.scheme}")
            if prob.order != 2:
                raise ValueError("the space-expanded schemes extend the second-order CD")
            depth = 3 if dm.scheme == "space222" else 2
            if any(prob.b[a] < depth for a in range(prob.ndim)):
                raise ValueError(f"{dm.scheme} needs PE edges of at least {depth} points")
            self.space = {(d, side): {key: _fr(c) for key, c in
                                      coeffs.space_expanded_at_stencil(d, dm.scheme, side).items()}
                          for d in (1, 2) for side in ("left", "right")}
        u0 = torch.as_tensor(u0, dtype=torch.float64)
        if tuple(u0.shape) != prob.shape:
            raise ValueError(f"u0 shape {tuple(u0.shape)} != {prob.shape}")
        self.hist = {0: u0}
        self.shist = {}          # RK2 predictor u* by level
        self.fhist = []          # f^{n-1}, f^{n-2} for the multistep methods
        self.n = 0
        self.delays = []         # delay table of every step taken

    # ---------------------------------------------------------------- history
    @staticmethod
    def level(hist, l):
        """Field at time level l of a history; before t = 0 the first level
        stands in (only reached with zero weight, see rng.clamp_startup)."""
        return hist[l] if l >= 0 else hist[0]

    # ------------------------------------------------------------ derivatives
    def _slab_delays(self, K, axis, side):
        """Delay of the consumer PE for every point of one boundary layer
        (shape = field shape with the axis replaced by its PE count)."""
        P = self.prob.pe
        b = self.prob.b
        kk = K[:, axis, side].reshape(P[2], P[1], P[0])   # [pz, py, px]
        dim = 2 - axis
        for a in range(3):
            d_ = 2 - a
            if a != axis:
                kk = kk.repeat_interleave(b[a], dim=d_)
        return kk

    def axis_derivative(self, centre, K, axis, taps, hist=None):
        """d-th derivative along ``axis`` (times dx^d), AT at I_B.

        ``centre`` is the field at level n; ``hist`` holds the past levels of
        the same quantity (default: the solution history)."""
        if self.nonuniform is not None and self.dm.mode != "sync":
            return self._nonuniform_axis_derivative(centre, K, axis, 1 if taps is self.taps1 else 2, hist)
        if self.space is not None and self.dm.mode != "sync":
            return self._space_axis_derivative(centre, K, axis, 1 if taps is self.taps1 else 2, hist)
        prob = self.prob
        hist = self.hist if hist is None else hist
        dim = 2 - axis
        s = prob.s
        N = prob.n[axis]
        b = prob.b[axis]
        # Standard central difference everywhere (eq. general_deriv).
        D = torch.zeros_like(centre)
        for o in range(-s, s + 1):
            D = D + taps[o + s] * torch.roll(centre, shifts=-o, dims=dim)
        if self.dm.mode == "sync":
            return D
        # Boundary layers: AT combination (eq. cd4-at and its table siblings).
        for side in (0, 1):
            layers = range(0, s) if side == 0 else range(b - s, b)
            Kslab = self._slab_delays(K, axis, side)
            for ell in layers:
                idx = torch.arange(prob.pe[axis]) * b + ell
                acc = torch.zeros_like(centre.index_select(dim, idx))
                for kd in range(0, self.dm.L):
                    mask = Kslab == kd
                    if not bool(mask.any()):
                        continue
                    w = self.wtab[kd]
                    val = torch.zeros_like(acc)
                    for m in range(self.T):
                        older = self.level(hist, self.n - kd - m)
                        st = torch.zeros_like(acc)
                        for o in range(-s, s + 1):
                            crossing = (ell + o < 0) if side == 0 else (ell + o >= b)
                            src = older if crossing else centre
                            st = st + taps[o + s] * src.index_select(dim, (idx + o) % N)
                        val = val + w[m] * st
                    acc = torch.where(mask, val, acc)
                D = D.index_copy(dim, idx, acc)
        return D

    def _space_axis_derivative(self, centre, K, axis, d, hist=None):
        """Space-expanded family: CD2 everywhere, the face-adjacent points
        (ell = 0 and ell = b - 1) of a face with delay k > 0 replaced by the
        asymmetric single-level stencil with buffer points at level n - k."""
        prob = self.prob
        hist = self.hist if hist is None else hist
        taps = self.taps1 if d == 1 else self.taps2
        dim = 2 - axis
        N = prob.n[axis]
        b = prob.b[axis]
        D = torch.zeros_like(centre)
        for o in (-1, 0, 1):
            D = D + taps[o + 1] * torch.roll(centre, shifts=-o, dims=dim)
        for side, ell, name in ((0, 0, "left"), (1, b - 1, "right")):
            Kslab = self._slab_delays(K, axis, side)
            idx = torch.arange(prob.pe[axis]) * b + ell
            acc = D.index_select(dim, idx)          # k = 0: the standard CD2
            for kd in range(1, self.dm.L):
                mask = Kslab == kd
                if not bool(mask.any()):
                    continue
                older = self.level(hist, self.n - kd)
                val = torch.zeros_like(acc)
                for (j, lev), c in self.space[(d, name)].items():
                    src = older if lev == "k" else centre
                    val = val + c * src.index_select(dim, (idx + j) % N)
                acc = torch.where(mask, val, acc)
            D = D.index_copy(dim, idx, acc)
        return D

    def _nonuniform_taps(self, k1, k2, d):
        """Right-face stencil {j: (level delay, c)} of the non-uniform scheme
        at the point i next to the face: points i-1, i at level n, i+1 at
        n-k1, i+2 at n-k2. d = 1: eq. cond with a = 2, r = 2 (Sec. 3.4 Example
        1, eq. ex1-0); d = 2: the same footprint with a = 1, r = 2 (the
        non-uniform form of the (2,1,2) row)."""
        key = (k1, k2)
        if key not in self.nonuniform:
            st = [(-1, 0), (0, 0), (1, k1), (2, k2)]
            tabs = {}
            for dd, a in ((1, 2), (2, 1)):
                status, c = coeffs.derive_scheme(st, dd, a, 2)
                if status != "unique":
                    raise AssertionError(f"non-uniform stencil {st} has no unique scheme")
                tabs[dd] = {j: (lev, _fr(c[(j, lev)])) for j, lev in st}
            self.nonuniform[key] = tabs
        return self.nonuniform[key][d]

    def _nonuniform_axis_derivative(self, centre, K, axis, d, hist=None):
        """Non-uniform-delay scheme: CD2 everywhere; at the face-adjacent
        points (ell = 0 and b - 1) the four-point stencil whose two buffer
        points carry their own delays (k1 nearest, k2 next). The left face is
        the mirror image (j -> -j, coefficients times (-1)^d)."""
        prob = self.prob
        hist = self.hist if hist is None else hist
        taps = self.taps1 if d == 1 else self.taps2
        dim = 2 - axis
        N = prob.n[axis]
        b = prob.b[axis]
        D = torch.zeros_like(centre)
        for o in (-1, 0, 1):
            D = D + taps[o + 1] * torch.roll(centre, shifts=-o, dims=dim)
        sgn_left = -1.0 if d == 1 else 1.0
        for side, ell in ((0, 0), (1, b - 1)):
            K1 = self._slab_delays(K, axis, side)
            K2 = self._slab_delays(self.K2, axis, side)
            idx = torch.arange(prob.pe[axis]) * b + ell
            acc = D.index_select(dim, idx)          # both delays 0: the standard CD2
            pairs = sorted(set(zip(K1.flatten().tolist(), K2.flatten().tolist())))
            for k1, k2 in pairs:
                kk = nonuniform_delays(k1, k2)
                if kk is None:
                    continue
                mask = (K1 == k1) & (K2 == k2)
                val = torch.zeros_like(acc)
                for j, (lev, c) in self._nonuniform_taps(kk[0], kk[1], d).items():
                    src = self.level(hist, self.n - lev) if lev > 0 else centre
                    jj = j if side == 1 else -j
                    cc = c if side == 1 else sgn_left * c
                    val = val + cc * src.index_select(dim, (idx + jj) % N)
                acc = torch.where(mask, val, acc)
            D = D.index_copy(dim, idx, acc)
        return D

    def rhs(self, centre, K, hist=None):
        """f = -c . grad u + alpha lap u, or -u sum_d u_{x_d} + alpha lap u."""
        prob = self.prob
        grad = []
        lap = []
        for a in range(prob.ndim):
            dx = prob.dx[a]
            grad.append(self.axis_derivative(centre, K, a, self.taps1, hist) / dx)
            lap.append(self.axis_derivative(centre, K, a, self.taps2, hist) / (dx * dx))
        L2 = lap[0]
        for t in lap[1:]:
            L2 = L2 + t
        if prob.equation == "advdiff":
            adv = prob.c[0] * grad[0]
            for a in range(1, prob.ndim):
                adv = adv + prob.c[a] * grad[a]
            return self.alpha * L2 - adv
        if prob.equation == "burgers":
            g = grad[0]
            for t in grad[1:]:
                g = g + t
            return self.alpha * L2 - centre * g
        raise ValueError(prob.equation)

    # ------------------------------------------------------------------ step
    def step(self):
        prob = self.prob
        n = self.n
        K = delay_table(prob, self.dm, n, self.key)
        self.delays.append(K)
        if self.nonuniform is not None:
            self.K2 = point_delay_table(prob, self.dm, n, self.key)
        u = self.hist[n]
        dt = prob.dt
        integ = prob.integrator
        if integ == "rk2":
            f1 = self.rhs(u, K)
            ustar = u + dt * f1
            self.shist[n] = ustar
            f2 = self.rhs(ustar, K, self.shist)
            unew = u + (0.5 * dt) * (f1 + f2)
        else:
            f = self.rhs(u, K)
            hist_f = [f] + self.fhist
            if integ == "euler" or len(hist_f) == 1:
                unew = u + dt * f
            elif integ == "ab2" or len(hist_f) == 2:
                unew = u + dt * (1.5 * hist_f[0] - 0.5 * hist_f[1])
            elif integ == "ab3":
                unew = u + dt * ((23.0 * hist_f[0] - 16.0 * hist_f[1] + 5.0 * hist_f[2]) / 12.0)
            else:
                raise ValueError(integ)
            depth = {"euler": 0, "ab2": 1, "ab3": 2}[integ]
            self.fhist = hist_f[:depth]
        self.n = n + 1
        self.hist[n + 1] = unew
        keep = self.n - (self.dm.L + self.T - 2)
        for h in (self.hist, self.shist):
            for l in [l for l in h if l < keep and l != 0]:
                del h[l]
        return unew

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()
        return self.hist[self.n]

    @property
    def u(self):
        return self.hist[self.n]

    @property
    def t(self):
        return self.n * self.prob.dt


def boundary_mask(prob: Problem):
    """True on I_B: points within s of a PE face along any axis (Sec. 2)."""
    s = prob.s
    m = torch.zeros(prob.shape, dtype=torch.bool)
    for a in range(prob.ndim):
        dim = 2 - a
        loc = torch.arange(prob.n[a]) % prob.b[a]
        near = (loc < s) | (loc >= prob.b[a] - s)
        shape = [1, 1, 1]
        shape[dim] = prob.n[a]
        m = m | near.reshape(shape).expand(prob.shape)
    return m
