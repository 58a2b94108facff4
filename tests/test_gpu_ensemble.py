"""GPU parity of the delay ensemble (one persistent launch for all members and
steps) against the FP64 oracle run member by member.

Each member is an independent periodic 1-D advection-diffusion problem with
its own grid, PEs, scheme, L and generator key; the oracle runs it as a
single problem with the same key. Tolerances as for single problems:
relative L2 <= 1e-12 (FP64), <= 1e-5 (FP32 bulk, FP64 AT combination).
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.analytic import advected_modes
from oracle.norms import error_norms
from oracle.solver import DelayModel, Oracle, Problem
from tests._cases import check_field

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
KAPPAS, AMPS = (1, 2, 3), (1.0, 0.5, 0.25)

# ragged PE edges (12, 20), every order, both integrators, L from 1 to 8,
# non-uniform bins, the asynchronous standard scheme (T = 1), ZERO and SYNC
MEMBERS = [
    dict(n=128, pe=4, order=2, integrator="euler", L=3, mode="rng", c=1.0, ra=0.1, seed=11),
    dict(n=192, pe=6, order=4, integrator="ab2", L=4, mode="rng", c=-0.5, ra=0.02, seed=12),
    dict(n=96, pe=3, order=4, integrator="ab2", L=8, mode="rng", c=0.3, ra=0.005, seed=13),
    dict(n=60, pe=5, order=2, integrator="euler", L=2, mode="zero", c=1.0, ra=0.1, seed=14),
    dict(n=64, pe=4, order=4, integrator="ab2", L=1, mode="sync", c=1.0, ra=0.02, seed=15),
    dict(n=120, pe=6, order=6, integrator="ab2", L=3, mode="rng", c=0.7, ra=0.004, seed=16),
    dict(n=256, pe=4, order=2, integrator="euler", L=3, mode="rng", c=1.0, ra=0.1, seed=17, weights=[6, 3, 1]),
    dict(n=72, pe=6, order=4, integrator="ab2", L=3, T=1, mode="rng", c=1.0, ra=0.02, seed=18),
    dict(n=64, pe=1, order=4, integrator="euler", L=2, mode="rng", c=1.0, ra=0.02, seed=19),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _members(spec):
    out = []
    for m in spec:
        m = dict(m)
        ra = m.pop("ra")
        dx = 2 * math.pi / m["n"]
        m.setdefault("alpha", 0.1)
        m["dt"] = ra * dx * dx / m["alpha"]
        m.setdefault("T", 0)
        m.setdefault("length", 2 * math.pi)
        out.append(m)
    return out


def _phases(count, seed=21):
    return np.random.Generator(np.random.PCG64(seed)).uniform(0, 2 * math.pi, size=(count, len(KAPPAS)))


def _u0(members, phases):
    parts = []
    for m, ph in zip(members, phases):
        modes = W.make_modes([(k,) for k in KAPPAS], AMPS, phis=list(ph))
        parts.append(W.eval_modes(modes, (m["n"],), 1).reshape(-1))
    return np.concatenate(parts)


def _oracle(m, u0):
    prob = Problem(ndim=1, n=(m["n"],), pe=(m["pe"],), dt=m["dt"], order=m["order"], c=(m["c"],),
                   alpha=m["alpha"], integrator=m["integrator"])
    dm = DelayModel(L=m["L"], T=m["T"], mode=m["mode"], seed=m["seed"], weights=m.get("weights"))
    return Oracle(prob, dm, torch.as_tensor(u0, dtype=torch.float64).reshape(1, 1, -1))


def _ensemble(members, precision):
    from paper_1702_00496_amd import Ensemble
    return Ensemble(members, precision=precision)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_ensemble_matches_oracle_member_by_member(precision):
    members = _members(MEMBERS)
    ph = _phases(len(members))
    u0 = _u0(members, ph)
    steps = 60
    _say(f"[ens] parity {precision}: {len(members)} members, {steps} steps")
    ens = _ensemble(members, precision)
    ens.set_state(torch.from_numpy(u0))
    ens.run(steps)
    got = ens.split(ens.state().cpu())
    off = 0
    for i, m in enumerate(members):
        o = _oracle(m, u0[off:off + m["n"]])
        o.run(steps)
        err = check_field(got[i], o, TOL[precision], label=(i, m))
        _say(f"[ens]   member {i} n={m['n']} order={m['order']} {m['integrator']} L={m['L']} {m['mode']}: {err}")
        off += m["n"]


def _random_members(seed, count):
    """Seeded heterogeneous members: PE edges from the minimum 2s up, one to
    eight PEs, every order, both integrators, T from the default or 1..4, L
    1..8, optional bin weights, every delay mode; diffusive and advective
    time-step bounds keep each member from growing."""
    import random
    rng = random.Random(seed)
    out = []
    for i in range(count):
        order = rng.choice((2, 4, 6))
        s = order // 2
        pe = rng.randint(1, 8)
        n = pe * rng.randint(2 * s, 2 * s + 20)
        T = rng.choice((0, 0, 0, 1, 2, 3, 4))
        L = rng.randint(1, 3 if T > 2 else 8)
        dx = 2 * math.pi / n
        ra = {2: 0.05, 4: 0.01, 6: 0.004}[order]
        m = dict(n=n, pe=pe, order=order, integrator=rng.choice(("euler", "ab2")), L=L, T=T,
                 mode=rng.choice(("rng", "rng", "rng", "zero", "sync")), c=round(rng.uniform(-1, 1), 3),
                 alpha=0.1, seed=rng.randint(0, 2 ** 40), length=2 * math.pi,
                 dt=min(ra * dx * dx / 0.1, 0.05 * dx))
        if rng.random() < 0.4:
            m["weights"] = [rng.randint(1, 6) for _ in range(L)]
        out.append(m)
    return out


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_ensemble_random_members_match_oracle(precision):
    members = _random_members(4242, 40)
    ph = _phases(len(members), seed=5)
    u0 = _u0(members, ph)
    steps = 40
    _say(f"[ens] random members {precision}: {len(members)} members, {steps} steps")
    ens = _ensemble(members, precision)
    ens.set_state(torch.from_numpy(u0))
    ens.run(steps)
    got = ens.split(ens.state().cpu())
    off = 0
    for i, m in enumerate(members):
        o = _oracle(m, u0[off:off + m["n"]])
        o.run(steps)
        check_field(got[i], o, TOL[precision], label=(i, m))
        off += m["n"]


def test_ensemble_zero_delays_equal_synchronous_bitwise():
    base = [dict(m, mode="zero") for m in MEMBERS]
    sync = [dict(m, mode="sync") for m in MEMBERS]
    a_m, b_m = _members(base), _members(sync)
    u0 = torch.from_numpy(_u0(a_m, _phases(len(a_m))))
    out = []
    for mem in (a_m, b_m):
        e = _ensemble(mem, "f32")
        e.set_state(u0)
        e.run(50)
        out.append(e.state().cpu())
    assert torch.equal(out[0], out[1])


def test_ensemble_schedules_and_run_splits_are_bit_identical():
    members = _members(MEMBERS)
    u0 = torch.from_numpy(_u0(members, _phases(len(members))))
    ref = _ensemble(members, "f32")
    ref.set_state(u0)
    ref.run(40)
    want = ref.state().cpu()
    for g, t in ((1, 256), (4, 1024), (2, 512)):
        e = _ensemble(members, "f32")
        e.set_tuning(g, t)
        e.set_state(u0)
        e.run(40)
        assert torch.equal(e.state().cpu(), want), (g, t)
    # the same 40 steps as 15 + 25 and as a replayed 10-step graph
    e = _ensemble(members, "f32")
    e.set_state(u0)
    e.run(15)
    e.run(25)
    assert torch.equal(e.state().cpu(), want)
    e.set_state(u0)
    for _ in range(4):
        e.run(10)
    assert e.n_step == 40
    assert torch.equal(e.state().cpu(), want)


def test_ensemble_norms_match_oracle_norms():
    members = _members(MEMBERS)
    ph = _phases(len(members))
    u0 = _u0(members, ph)
    steps = 30
    ens = _ensemble(members, "f64")
    ens.set_state(torch.from_numpy(u0))
    ens.run(steps)
    got = ens.norms(KAPPAS, AMPS, ph)
    packed = ens.state().cpu()
    parts = ens.split(packed)
    refs = []
    for i, m in enumerate(members):
        prob = Problem(ndim=1, n=(m["n"],), pe=(m["pe"],), dt=m["dt"], order=m["order"], c=(m["c"],),
                       alpha=m["alpha"])
        modes = W.make_modes([(k,) for k in KAPPAS], AMPS, phis=list(ph[i]))
        ua = advected_modes(prob, modes, steps * m["dt"]).reshape(-1)
        refs.append(ua)
        e = error_norms(parts[i].to(torch.float64), ua)
        assert got[i, 0] == pytest.approx(e["l1"], rel=1e-9)
        assert got[i, 1] == pytest.approx(e["l2"], rel=1e-9)
        assert got[i, 2] == pytest.approx(e["linf"], rel=1e-9)
    # against a packed reference field the same numbers come back
    again = ens.norms(ref=torch.cat(refs))
    # (the two references differ by a few ulps of the O(1) field)
    assert np.allclose(again, got, rtol=1e-9, atol=1e-12)


def test_ensemble_rejects_bad_members():
    from paper_1702_00496_amd import ATError
    bad = _members([dict(n=100, pe=3, order=2, integrator="euler", L=3, mode="rng", c=1.0, ra=0.1, seed=1)])
    with pytest.raises(ATError):
        _ensemble(bad, "f32")


def test_ensemble_full_workload_properties():
    """The 512-member, 2000-step delay ensemble in FP32: finite everywhere,
    every member's error against the exact solution small, and the two
    smallest members equal to the FP64 oracle."""
    inst = W.ensemble_instances()
    members = [dict(n=m["n"], pe=m["pe"], order=m["order"], integrator=m["integrator"], L=m["L"], T=m["T"],
                    mode="rng", length=2 * math.pi, c=m["c"], alpha=m["alpha"], dt=m["dt"], seed=m["seed"])
               for m in inst]
    ph = np.array([[mo[2] for mo in m["modes"]] for m in inst])
    kap = [mo[0][0] for mo in inst[0]["modes"]]
    amp = [mo[1] for mo in inst[0]["modes"]]
    parts = [W.eval_modes(m["modes"], (m["n"],), 1).reshape(-1) for m in inst]
    u0 = np.concatenate(parts)
    steps = 2000
    _say(f"[ens] full workload: {len(members)} members, {u0.size} points, {steps} steps")
    ens = _ensemble(members, "f32")
    ens.set_state(torch.from_numpy(u0))
    ens.run(steps)
    err = ens.norms(kap, amp, ph)
    assert np.isfinite(err).all()
    # the delay error of these schemes is far below the field's O(1) size
    assert err[:, 1].max() < 1e-2, err[:, 1].max()
    got = ens.split(ens.state().cpu())
    small = sorted(range(len(members)), key=lambda i: members[i]["n"])[:2]
    for i in small:
        o = _oracle(members[i], parts[i])
        o.run(steps)
        r = check_field(got[i], o, TOL["f32"], label=(i, members[i]))
        _say(f"[ens]   member {i} n={members[i]['n']} order={members[i]['order']} L={members[i]['L']}: {r}")


def _workload_members():
    inst = W.ensemble_instances()
    members = [dict(n=m["n"], pe=m["pe"], order=m["order"], integrator=m["integrator"], L=m["L"], T=m["T"],
                    mode="rng", length=2 * math.pi, c=m["c"], alpha=m["alpha"], dt=m["dt"], seed=m["seed"])
               for m in inst]
    parts = [W.eval_modes(m["modes"], (m["n"],), 1).reshape(-1) for m in inst]
    return inst, members, parts


def test_ensemble_workload_largest_members_match_oracle():
    """The 512-member workload in its benchmark launch (every member, the
    default schedule), 200 steps in FP32: the three largest members (each
    above 60,000 points, the several-chunks-in-flight sweep), members of about
    16,000 and 4,000 points and the smallest one equal the FP64 oracle
    element by element."""
    inst, members, parts = _workload_members()
    steps = 200
    ens = _ensemble(members, "f32")
    ens.set_state(torch.from_numpy(np.concatenate(parts)))
    ens.run(steps)
    got = ens.split(ens.state().cpu())
    by_n = sorted(range(len(members)), key=lambda i: members[i]["n"])
    pick = by_n[-3:]
    for target in (16448, 4160):
        pick.append(min(by_n, key=lambda i: abs(members[i]["n"] - target)))
    pick.append(by_n[0])
    for i in pick:
        o = _oracle(members[i], parts[i])
        o.run(steps)
        e = check_field(got[i], o, TOL["f32"], label=(i, members[i]))
        _say(f"[ens]   member {i} n={members[i]['n']} order={members[i]['order']} L={members[i]['L']}: {e}")


def test_ensemble_bins_of_more_than_24_members_match_oracle():
    """One workgroup per CU and 6,400 small members: every workgroup's bin
    holds 25 members, more than its LDS batch of 24, so the launch runs the
    steps for one batch and then for the next. Members of the second batch
    (and a sample of the first) equal the FP64 oracle; the result equals the
    default schedule's bit for bit."""
    import random
    rng = random.Random(77)
    spec = []
    for i in range(6400):
        order = rng.choice((2, 4))
        pe = rng.choice((2, 3, 4))
        n = pe * rng.choice((4, 6, 8))
        dx = 2 * math.pi / n
        ra = 0.05 if order == 2 else 0.005
        spec.append(dict(n=n, pe=pe, order=order, integrator="euler" if order == 2 else "ab2",
                         L=rng.choice((2, 4, 8)) if order == 2 else rng.choice((2, 3)), mode="rng",
                         c=round(rng.uniform(-1, 1), 3), ra=min(ra, 0.005 / dx), seed=100 + i))
    members = _members(spec)
    ph = _phases(len(members), seed=8)
    u0 = torch.from_numpy(_u0(members, ph))
    steps = 24
    ens = _ensemble(members, "f32")
    ens.set_tuning(1, 1024)
    ens.set_state(u0)
    ens.run(steps)
    assert ens.bin_sizes().max() > 24, ens.bin_sizes().max()
    got_packed = ens.state().cpu()
    got = ens.split(got_packed)
    ref = _ensemble(members, "f32")
    ref.set_state(u0)
    ref.run(steps)
    assert torch.equal(ref.state().cpu(), got_packed)
    late = ens.members_beyond_batch(24)
    assert len(late) >= 256, len(late)
    off = np.concatenate([[0], np.cumsum([m["n"] for m in members])])
    check = sorted(set(late[::4]) | set(range(0, len(members), 211)))
    for i in check:
        o = _oracle(members[i], u0[off[i]:off[i + 1]].numpy())
        o.run(steps)
        check_field(got[i], o, TOL["f32"], label=(i, members[i]))
    _say(f"[ens] bins of {ens.bin_sizes().max()} members: {len(check)} members checked")


def test_ensemble_non_finite_member_reports_unstable():
    """A NaN in one member's field makes the ensemble norms return
    AT_EUNSTABLE."""
    from paper_1702_00496_amd import ATError, _lib
    members = _members(MEMBERS)
    ph = _phases(len(members))
    u0 = torch.from_numpy(_u0(members, ph))
    ens = _ensemble(members, "f32")
    ens.set_state(u0)
    ens.run(5)
    assert np.isfinite(ens.norms(KAPPAS, AMPS, ph)).all()
    u0[members[0]["n"] + 3] = float("nan")      # second member
    ens.set_state(u0)
    ens.run(5)
    with pytest.raises(ATError) as ei:
        ens.norms(KAPPAS, AMPS, ph)
    assert ei.value.status == _lib.AT_EUNSTABLE


def _dx_edges(members, nbins):
    dx = [m["length"] / m["n"] for m in members]
    lo, hi = min(dx), max(dx)
    return np.exp(np.linspace(np.log(lo), np.log(hi * (1 + 1e-9)), nbins + 1))


def test_ensemble_error_statistics_match_oracle_member_runs():
    """Mean and unbiased variance of the per-member RMS error against the exact
    solution, binned by grid spacing and grouped by order (the statistic the
    ensemble workload reports), from the FP64 ensemble against the same
    statistic over the FP64 oracle's member runs."""
    from oracle.norms import binned_mean_var
    import random
    rng = random.Random(31)
    spec = []
    for i in range(36):
        order = (2, 4)[i % 2]
        pe = rng.choice((4, 8))
        n = pe * rng.choice((8, 12, 16, 24, 32))
        spec.append(dict(n=n, pe=pe, order=order, integrator="euler" if order == 2 else "ab2",
                         L=rng.choice((2, 4, 8)), mode="rng", c=1.0, ra=0.1 if order == 2 else 0.005,
                         seed=500 + i))
    members = _members(spec)
    ph = _phases(len(members), seed=12)
    u0 = _u0(members, ph)
    steps = 150
    ens = _ensemble(members, "f64")
    ens.set_state(torch.from_numpy(u0))
    ens.run(steps)
    edges = _dx_edges(members, 4)
    got = ens.error_stats(edges, KAPPAS, AMPS, ph)
    off = 0
    rms, dxs, groups = [], [], []
    for i, m in enumerate(members):
        o = _oracle(m, u0[off:off + m["n"]])
        o.run(steps)
        modes = W.make_modes([(k,) for k in KAPPAS], AMPS, phis=list(ph[i]))
        ua = advected_modes(o.prob, modes, o.t)
        rms.append(error_norms(o.u, ua)["l2"])
        dxs.append(m["length"] / m["n"])
        groups.append(m["order"] // 2 - 1)
        off += m["n"]
    want = binned_mean_var(dxs, rms, groups, list(edges))
    # the RMS error is 1-Lipschitz in the field: each member's differs from the
    # oracle's by at most the RMS field difference, which the FP64 parity bar
    # puts below 1e-12 of the O(1) field (|u| <= 1.75 here)
    d = 1e-12 * 1.75
    for g in range(3):
        for j in range(len(edges) - 1):
            cnt, mdx, mean, var = want[g][j]
            assert got[g, j, 0] == cnt, (g, j)
            assert got[g, j, 1] == pytest.approx(mdx, rel=1e-14, abs=0)
            assert abs(got[g, j, 2] - mean) <= d, (g, j, got[g, j], want[g][j])
            assert abs(got[g, j, 3] - var) <= 2 * math.sqrt(var) * 2 * d + 4 * d * d, (g, j, got[g, j], want[g][j])
    assert got[:2, :, 0].sum() == len(members)


def test_ensemble_workload_error_statistics_equal_host_binning():
    """The 512-member workload after 2000 FP32 steps: the device's binned
    statistics equal the binning of its per-member norms done on the host."""
    from oracle.norms import binned_mean_var
    inst, members, parts = _workload_members()
    ens = _ensemble(members, "f32")
    ens.set_state(torch.from_numpy(np.concatenate(parts)))
    ens.run(2000)
    ph = np.array([[mo[2] for mo in m["modes"]] for m in inst])
    kap = [mo[0][0] for mo in inst[0]["modes"]]
    amp = [mo[1] for mo in inst[0]["modes"]]
    per = ens.norms(kap, amp, ph)
    edges = _dx_edges(members, 12)
    got = ens.error_stats(edges, kap, amp, ph)
    want = binned_mean_var([m["length"] / m["n"] for m in members], list(per[:, 1]),
                           [m["order"] // 2 - 1 for m in members], list(edges))
    for g in range(3):
        for j in range(12):
            cnt, mdx, mean, var = want[g][j]
            assert got[g, j, 0] == cnt
            assert got[g, j, 2] == pytest.approx(mean, rel=1e-12, abs=1e-300)
            assert got[g, j, 3] == pytest.approx(var, rel=1e-10, abs=1e-300)
    assert got[:, :, 0].sum() == len(members)
    _say(f"[ens] workload error table (order 2): {got[0, :, :].tolist()}")


def test_ensemble_autotune_restores_state_and_caches(tmp_path):
    """The ensemble autotuner times all nine (workgroups per CU, threads)
    candidates from the current state, keeps the fastest and leaves the state
    and step as they were (the continued run equals an untuned one bit for
    bit); a second ensemble of the same member shapes takes the choice from
    the JSON cache without timing."""
    from paper_1702_00496_amd import tuning
    members = _members(MEMBERS)
    u0 = torch.from_numpy(_u0(members, _phases(len(members))))
    ref = _ensemble(members, "f32")
    ref.set_state(u0)
    ref.run(30)
    want = ref.state().cpu()
    e = _ensemble(members, "f32")
    e.set_state(u0)
    e.run(10)
    path = str(tmp_path / "tuning.json")
    best, ms = e.autotune(nsteps=5, cache=path)
    assert len(ms) == 9 and best in ms and all(v > 0 for v in ms.values())
    assert e.tuning() == best and e.n_step == 10
    e.run(20)
    assert torch.equal(e.state().cpu(), want)
    ent = tuning.lookup(path, e.tuning_key())
    assert ent is not None and tuple(ent["variant"]) == best
    f = _ensemble([dict(m, seed=m["seed"] + 1) for m in members], "f32")
    f.set_state(2 * u0)
    assert f.tuning_key() == e.tuning_key()
    best2, ms2 = f.autotune(nsteps=5, cache=path)
    assert best2 == best and f.tuning() == best and ms2 == ms
