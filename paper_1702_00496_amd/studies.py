"""Delay-statistics studies run on the ensemble kernel (Sec. 5.2).

Every realisation of a study is one member of a single ``Ensemble`` launch: a
periodic 1-D advection-diffusion problem (Sec. 5 eq. general) with the
initial sine series of Sec. 5.1 (eq. IC), its own delay generator key and the
delay law of its configuration. The average overall error <E> (Sec. 4) is the
mean over realisations of each member's space-averaged |E| against the exact
solution (Sec. 5.1 eq. ana_sol), computed in double on the device.

- ``moment_study``: <E> against L (or any delay law) for a time-expanded
  scheme with T levels, and the asynchronous part (<E> - <E>_s) / <E>_s
  relative to a synchronous member, next to the law of Sec. 5.2 eq.
  aveE_scaling_gen_kmom: <E> - <E>_s ~ E[k (k+1) ... (k+T-1)], i.e.
  <k^2> + <k> for T = 2 and <k^3> + 3<k^2> + 2<k> for T = 3 (with p_k = 1/L:
  L^2 - 1 and L^3 + 2L^2 - L - 2, eq. aveE_scaling_gen_L).
- ``delay_law_study``: the same for arbitrary delay laws p_k (several laws
  of one or more L side by side).
- ``pe_scaling_study``: <E> against the number of PEs P at fixed N (strong
  scaling: linear in P), at fixed P under refinement (asynchronous part
  ~ dx^{a+1}: slope -3 for a = 2) or at fixed P/N (weak scaling: ~ dx^a,
  slope -2), eq. aveE_scaling_gen2 (<E> ~ P dx^{a+1} sum gamma_m <k^m>).

Only argument marshalling and averaging happen here; the steps and the error
norms run in the library's kernels.
"""
import math

import numpy as np
import torch

from . import Ensemble

# Sec. 5.1 configuration of the 1-D experiments: kappa = {3, 4, 5},
# A = {2.0, 0.5, 1.5}
DEFAULT_MODES = ((3, 2.0), (4, 0.5), (5, 1.5))


def delay_law(L, T, weights=None):
    """E[k (k+1) ... (k+T-1)] for k drawn with bin weights (uniform if None)."""
    w = [1.0] * L if weights is None else [float(v) for v in weights]
    tot = sum(w)
    out = 0.0
    for k in range(L):
        term = 1.0
        for m in range(T):
            term *= k + m
        out += w[k] / tot * term
    return out


def _member_key(seed, tag, r):
    """Distinct 64-bit generator keys per (study seed, configuration, realisation)."""
    x = (seed * 0x9E3779B97F4A7C15 + tag * 0xBF58476D1CE4E5B9 + r * 0x94D049BB133111EB) & (2 ** 64 - 1)
    return x ^ (x >> 29)


def _initial_fields(members, modes):
    out = []
    for m in members:
        x = np.arange(m["n"], dtype=np.float64) * (2 * math.pi / m["n"])
        out.append(sum(a * np.sin(k * x) for k, a in modes))
    return torch.from_numpy(np.concatenate(out))


def run_members(members, steps, modes=DEFAULT_MODES, precision="f64", device="cuda", sync_ref=False):
    """Advance the members together for ``steps`` steps; per-member mean |E|,
    rms E and max |E| against the exact solution at t = steps * dt. With
    ``sync_ref`` the first member must be synchronous and every member of the
    same size is also measured against its final field (the asynchronous
    perturbation |u - u_s|): returns (exact norms, norms against u_s)."""
    ens = Ensemble(members, precision=precision, device=device)
    ens.set_state(_initial_fields(members, modes))
    ens.run(steps)
    kap = [k for k, _ in modes]
    amp = [a for _, a in modes]
    nrm = ens.norms(kap, amp, np.zeros((len(members), len(modes))))
    if not sync_ref:
        ens.close()
        return nrm
    parts = ens.split(ens.state().to(torch.float64))
    ref = torch.cat([parts[0] if m["n"] == members[0]["n"] else p for m, p in zip(members, parts)])
    rel = ens.norms(ref=ref)
    ens.close()
    return nrm, rel


def _dt(n, alpha, r_alpha):
    dx = 2 * math.pi / n
    return r_alpha * dx * dx / alpha


def moment_study(order=2, Ls=(2, 3, 4, 5, 6), realizations=64, n=128, pe=16, r_alpha=0.1, t_final=0.5,
                 c=1.0, alpha=0.1, weights=None, seed=0, precision="f64", device="cuda"):
    """<E> of the time-expanded scheme of ``order`` (T = order/2 + 1; Euler
    for order 2, AB2 for order 4) for every L in ``Ls`` (``weights``: one bin
    weight list per L, or None for p_k = 1/L), with ``realizations`` delay
    histories each and one synchronous member. Returns a dict with the
    members, and per L: E, E_sync, asynchronous = (E - E_sync) / E_sync (the
    paper's measure), law = E[k (k+1) ... (k+T-1)], ratio = asynchronous /
    law, and perturbation = the mean over histories of mean |u - u_s| with
    its ratio to the law (free of cancellation against the synchronous
    error)."""
    T = order // 2 + 1
    integ = "euler" if order == 2 else "ab2"
    dt = _dt(n, alpha, r_alpha)
    steps = int(round(t_final / dt))
    base = dict(n=n, pe=pe, order=order, integrator=integ, c=c, alpha=alpha, dt=dt)
    members = [dict(base, L=1, mode="sync", seed=0)]
    for i, L in enumerate(Ls):
        w = None if weights is None else weights[i]
        for r in range(realizations):
            members.append(dict(base, L=L, mode="rng", seed=_member_key(seed, L, r), weights=w))
    nrm, rel = run_members(members, steps, precision=precision, device=device, sync_ref=True)
    es = float(nrm[0, 0])
    rows = {}
    for i, L in enumerate(Ls):
        sl = slice(1 + i * realizations, 1 + (i + 1) * realizations)
        e = float(np.mean(nrm[sl, 0]))
        pert = float(np.mean(rel[sl, 0]))
        law = delay_law(L, T, None if weights is None else weights[i])
        a = (e - es) / es
        rows[L] = dict(E=e, E_sync=es, asynchronous=a, law=law, ratio=a / law if law else float("nan"),
                       perturbation=pert, perturbation_ratio=pert / law if law else float("nan"))
    return dict(order=order, T=T, steps=steps, dt=dt, members=members, per_L=rows)


def delay_law_study(order=2, laws=((3, (2, 5, 3)), (3, (5, 3, 2)), (3, (1, 1, 8)), (3, (8, 1, 1)), (4, (1, 2, 3, 4))),
                    realizations=64, n=128, pe=16, r_alpha=0.1, t_final=0.5, c=1.0, alpha=0.1, seed=0,
                    precision="f64", device="cuda"):
    """<E> for general delay laws p_k (Sec. 5.2 eq. aveE_scaling_gen_kmom: the
    asynchronous part follows E[k (k+1) ... (k+T-1)] for any p_k, not only
    p_k = 1/L): ``laws`` is a list of (L, bin weights); every law gets
    ``realizations`` delay histories and the configuration one synchronous
    member, all in one launch. Returns per law (in order): L, weights, E,
    E_sync, asynchronous = (E - E_sync) / E_sync, law = E[k (k+1) ...
    (k+T-1)], perturbation = mean over histories of mean |u - u_s| and its
    ratio to the law."""
    T = order // 2 + 1
    integ = "euler" if order == 2 else "ab2"
    dt = _dt(n, alpha, r_alpha)
    steps = int(round(t_final / dt))
    base = dict(n=n, pe=pe, order=order, integrator=integ, c=c, alpha=alpha, dt=dt)
    members = [dict(base, L=1, mode="sync", seed=0)]
    for i, (L, w) in enumerate(laws):
        for r in range(realizations):
            members.append(dict(base, L=L, mode="rng", seed=_member_key(seed, 5000 + i, r), weights=list(w)))
    nrm, rel = run_members(members, steps, precision=precision, device=device, sync_ref=True)
    es = float(nrm[0, 0])
    rows = []
    for i, (L, w) in enumerate(laws):
        sl = slice(1 + i * realizations, 1 + (i + 1) * realizations)
        e = float(np.mean(nrm[sl, 0]))
        pert = float(np.mean(rel[sl, 0]))
        law = delay_law(L, T, w)
        rows.append(dict(L=L, weights=list(w), E=e, E_sync=es, asynchronous=(e - es) / es, law=law,
                         perturbation=pert, perturbation_ratio=pert / law if law else float("nan")))
    return dict(order=order, T=T, steps=steps, dt=dt, members=members, per_law=rows)


def pe_scaling_study(order=2, configs=((512, 2), (512, 4), (512, 8), (512, 16), (512, 32)), L=3,
                     weights=(2, 5, 3), realizations=16, r_alpha=0.1, t_final=0.2, c=1.0, alpha=0.1,
                     seed=0, precision="f64", device="cuda"):
    """<E> for every (N, P) in ``configs`` (strong scaling: N fixed; weak:
    N/P fixed), with ``realizations`` delay histories each and one
    synchronous member per configuration; dt = r_alpha dx^2 / alpha per N and
    the same final time. Returns per (N, P): E, E_sync, E - E_sync and
    asynchronous = the mean over histories of mean |u - u_s| (the
    perturbation the delays cause, free of cancellation against the
    synchronous error)."""
    integ = "euler" if order == 2 else "ab2"
    members = []
    index = []
    for j, (n, p) in enumerate(configs):
        dt = _dt(n, alpha, r_alpha)
        base = dict(n=n, pe=p, order=order, integrator=integ, c=c, alpha=alpha, dt=dt)
        index.append((len(members), int(round(t_final / dt))))
        members.append(dict(base, L=1, mode="sync", seed=0))
        for r in range(realizations):
            members.append(dict(base, L=L, mode="rng", seed=_member_key(seed, 1000 + j, r), weights=list(weights)))
    # members of different N need different step counts: one launch per configuration
    rows = {}
    for j, (n, p) in enumerate(configs):
        start, steps = index[j]
        group = members[start: start + 1 + realizations]
        nrm, rel = run_members(group, steps, precision=precision, device=device, sync_ref=True)
        es = float(nrm[0, 0])
        e = float(np.mean(nrm[1:, 0]))
        rows[(n, p)] = dict(E=e, E_sync=es, difference=e - es, asynchronous=float(np.mean(rel[1:, 0])),
                            steps=steps)
    return dict(order=order, members=members, per_config=rows)


# ---------------------------------------------------------------- Cases 5, 6
def cole_hopf(x, t, amp, nu, nterms=None):
    """Exact solution of u_t + u u_x = nu u_xx on the periodic [0, 2 pi) with
    u(x, 0) = amp sin x (Cole-Hopf): with a = amp / (2 nu),
    theta = I_0(a) + 2 sum_n I_n(a) e^{-nu n^2 t} cos(n x) and
    u = -2 nu theta_x / theta (Bessel functions scaled by e^{-a}; the scale
    cancels in the ratio)."""
    from scipy.special import ive
    a = amp / (2.0 * nu)
    if nterms is None:
        nterms = int(max(40, 6 * a + 40))
    x = np.asarray(x, dtype=np.float64)
    theta = np.full_like(x, ive(0, a))
    dtheta = np.zeros_like(x)
    for n in range(1, nterms + 1):
        c = 2.0 * ive(n, a) * math.exp(-nu * n * n * t)
        theta += c * np.cos(n * x)
        dtheta -= c * n * np.sin(n * x)
    return -2.0 * nu * dtheta / theta


def _gpu_run(n, pe, order, integrator, equation, c, alpha, dt, steps, u0, L, weights, mode, seed, precision,
             scheme="time", T=0):
    from . import Solver
    s = Solver(ndim=1, n=(n,), pe=(pe,), dt=dt, order=order, equation=equation, c=(c,), alpha=alpha,
               integrator=integrator, precision=precision, L=L, T=T, mode=mode, seed=seed, weights=weights,
               scheme=scheme)
    s.set_graph(64)
    s.set_state(torch.as_tensor(u0).reshape(1, 1, n))
    s.step(steps)
    out = s.state().double().cpu().numpy().reshape(-1)
    s.close()
    return out


# The three arms of the Case 1 comparison (Sec. 5.2): the synchronous
# standard scheme, the standard scheme fed with delayed halos (T = 1), and the
# AT schemes (1,2,2)b/(2,2,2)b (T = 2).
CASE1_ARMS = {"synchronous": ("sync", 0), "asynchronous_standard": ("rng", 1), "at": ("rng", 0)}


def case1_study(n=128, pe=4, L=3, weights=(5, 3, 2), kappas=(2, 3, 5), amps=(1.0, 1.0, 1.0), c=1.0,
                alpha=0.1, r_alpha=0.1, times=(0.005, 0.05), conv_ns=(64, 128, 256, 512), conv_time=0.05,
                seed=3, precision="f64"):
    """Case 1 of the Sec. 5.1 table (advection-diffusion, Euler, CD2 with
    (1,2,2)b/(2,2,2)b) in the setting of the first experiment of Sec. 5.2:
    N = 128, kappa = {2, 3, 5}, P = 4, delays with p = {0.5, 0.3, 0.2}. For
    each time in ``times`` and each arm: mean |E|, max |E| at the points next
    to PE faces and max |E| elsewhere, against the exact advected decaying
    series (``per_time``); and the mean |E| at ``conv_time`` against N with
    its slopes (``convergence``). Amplitudes and times are not stated in the
    paper (readings)."""
    modes = tuple(zip(kappas, amps))

    def errors(n_, t):
        dt = _dt(n_, alpha, r_alpha)
        steps = max(1, int(round(t / dt)))
        dt = t / steps
        x = np.arange(n_) * (2 * math.pi / n_)
        u0 = sum(a * np.sin(k * x) for k, a in modes)
        exact = sum(a * math.exp(-alpha * k * k * t) * np.sin(k * (x - c * t)) for k, a in modes)
        b = n_ // pe
        face = (np.arange(n_) % b == 0) | (np.arange(n_) % b == b - 1)
        out = {}
        for arm, (mode, T) in CASE1_ARMS.items():
            u = _gpu_run(n_, pe, 2, "euler", "advdiff", c, alpha, dt, steps, u0, L, list(weights), mode, seed,
                         precision, T=T)
            e = np.abs(u - exact)
            out[arm] = dict(mean=float(e.mean()), face_max=float(e[face].max()), interior_max=float(e[~face].max()),
                            steps=steps, dt=dt)
        return out

    per_time = {t: errors(n, t) for t in times}
    conv = {arm: [] for arm in CASE1_ARMS}
    for n_ in conv_ns:
        r = errors(n_, conv_time)
        for arm in CASE1_ARMS:
            conv[arm].append(r[arm]["mean"])
    slopes = {arm: [math.log(v[i + 1] / v[i]) / math.log(conv_ns[i + 1] / conv_ns[i]) for i in range(len(v) - 1)]
              for arm, v in conv.items()}
    return dict(per_time=per_time, convergence=dict(ns=list(conv_ns), mean=conv, slopes=slopes))


CASE_CONFIGS = {
    # Sec. 5.1 table of cases: Case 2 = diffusion, Euler, CD2 with the
    # space-expanded (2,1,2); Case 3 = advection-diffusion, Euler, CD2 with
    # (1,2,2)a/(2,2,2)a; Case 4 = advection-diffusion, AB2, CD4 with
    # (1,4,2)/(2,4,2) (T = 3); Case 5 = diffusion, AB3, CD6 with (2,6,2)
    # (T = 4); Case 6 = viscous Burgers, AB2, CD4 with (1,4,2)/(2,4,2)
    "case2": dict(order=2, integrator="euler", equation="advdiff", c=0.0, alpha=0.1, r_alpha=0.05, t_final=0.05,
                  scheme="space212"),
    "case3": dict(order=2, integrator="euler", equation="advdiff", c=1.0, alpha=0.1, r_alpha=0.05, t_final=0.05,
                  scheme="space222"),
    "case4": dict(order=4, integrator="ab2", equation="advdiff", c=1.0, alpha=0.1, r_alpha=0.02, t_final=0.05),
    "case5": dict(order=6, integrator="ab3", equation="advdiff", c=0.0, alpha=0.1, r_alpha=0.01, t_final=0.1),
    "case6": dict(order=4, integrator="ab2", equation="burgers", c=0.0, alpha=0.1, r_alpha=0.02, t_final=0.5,
                  amp=1.0),
}


def convergence_study(case="case5", Ns=(32, 64, 128, 256), pe=4, L=3,
                      weight_sets=((1, 0, 0), (7, 2, 1), (4, 4, 2), (3, 5, 2)), realizations=2, seed=0,
                      precision="f64", T=0):
    """<E> against N for Cases 2-5 (exact: the decaying advected sine series of
    Sec. 5.1) or Case 6 (exact: Cole-Hopf for u0 = amp sin x), for every delay law in
    ``weight_sets`` (bin weights of k = 0, 1, ...; (1, 0, ...) is delay-free),
    dt = r_alpha dx^2 / alpha at a fixed final time. T = 1 runs the case's
    standard scheme fed with delayed halos instead of its AT schemes (Sec. 5.2,
    figure at-ord4-async). Returns per weight set the errors against N, their
    slopes, and the final fields (for moments)."""
    cfg = CASE_CONFIGS[case]
    out = {}
    for w in weight_sets:
        errs, fields = [], []
        for n in Ns:
            dx = 2 * math.pi / n
            steps = int(math.ceil(cfg["t_final"] / (cfg["r_alpha"] * dx * dx / cfg["alpha"])))
            dt = cfg["t_final"] / steps
            x = np.arange(n, dtype=np.float64) * dx
            if case != "case6":
                u0 = sum(a * np.sin(k * x) for k, a in DEFAULT_MODES)
                t = cfg["t_final"]
                exact = sum(a * math.exp(-cfg["alpha"] * k * k * t) * np.sin(k * (x - cfg["c"] * t))
                            for k, a in DEFAULT_MODES)
            else:
                u0 = cfg["amp"] * np.sin(x)
                exact = cole_hopf(x, cfg["t_final"], cfg["amp"], cfg["alpha"])
            e_r, f_r = [], []
            for r in range(realizations if sum(w[1:]) else 1):
                u = _gpu_run(n, pe, cfg["order"], cfg["integrator"], cfg["equation"], cfg["c"], cfg["alpha"], dt,
                             steps, u0, L, list(w), "rng", _member_key(seed, n, r), precision,
                             cfg.get("scheme", "time"), T=T)
                e_r.append(float(np.mean(np.abs(u - exact))))
                f_r.append(u)
            errs.append(float(np.mean(e_r)))
            fields.append(f_r)
        slopes = [math.log(errs[i + 1] / errs[i]) / math.log(Ns[i + 1] / Ns[i]) for i in range(len(Ns) - 1)]
        out[tuple(w)] = dict(E=errs, slopes=slopes, fields=fields)
    return dict(case=case, Ns=list(Ns), per_law=out)


def central_moments(u, dx):
    """Normalised central moments of u and of du/dx (spectral derivative of
    the periodic field): <(u - <u>)^2>, <(u - <u>)^3> / m2^{3/2},
    <(u - <u>)^4> / m2^2, for u and for du/dx (Sec. 5.2, Case 6 moments)."""
    n = u.size
    k = np.fft.rfftfreq(n, d=dx / (2 * math.pi))
    du = np.fft.irfft(1j * k * np.fft.rfft(u), n)

    def mom(v):
        d = v - v.mean()
        m2 = float(np.mean(d * d))
        return m2, float(np.mean(d ** 3)) / m2 ** 1.5, float(np.mean(d ** 4)) / m2 ** 2
    return dict(u=mom(u), dudx=mom(du))
