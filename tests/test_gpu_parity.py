"""GPU parity: the HIP library against the FP64 oracle, element by element.

Tolerances: relative L2 of the field difference <= 1e-12 for FP64 and <= 1e-5
for FP32 bulk (FP64 AT combination) against the FP64 oracle; delays bit-exact.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import rng as orng
from oracle.solver import delay_table
from tests._cases import check_field, initial_field, oracle_for, problem_for, rel_l2, solver_for

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _dt(case, r_alpha):
    # diffusive CFL on the finest axis
    dx = 2 * math.pi / max(v for v in case["n"][: case["ndim"]])
    return r_alpha * dx * dx / case.get("alpha", 0.1)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "1d_o2_euler_L3": dict(ndim=1, n=(256,), pe=(8,), order=2, integrator="euler", c=(1.0,), L=3, steps=300, ra=0.1),
    "1d_o4_ab2_ragged": dict(ndim=1, n=(120,), pe=(5,), order=4, integrator="ab2", c=(1.0,), L=4, steps=120, ra=0.02),
    "1d_o6_rk2_burgers": dict(ndim=1, n=(96,), pe=(4,), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=3, steps=80, ra=0.01),
    "1d_o4_ab3": dict(ndim=1, n=(60,), pe=(5,), order=4, integrator="ab3", c=(0.7,), L=3, steps=80, ra=0.02),
    "1d_o4_T1_async_standard": dict(ndim=1, n=(64,), pe=(4,), order=4, integrator="ab2", c=(1.0,), L=3, T=1, steps=80, ra=0.02),
    "1d_o2_weights": dict(ndim=1, n=(96,), pe=(6,), order=2, integrator="euler", c=(1.0,), L=3, weights=[6, 3, 1], steps=100, ra=0.1),
    "2d_o4_ab2_ragged": dict(ndim=2, n=(40, 36), pe=(4, 3), order=4, integrator="ab2", c=(1.0, -0.5), L=4, steps=40, ra=0.02),
    "2d_o2_euler": dict(ndim=2, n=(48, 32), pe=(3, 2), order=2, integrator="euler", c=(1.0, 1.0), L=2, steps=40, ra=0.05),
    "3d_o4_ab2_ragged": dict(ndim=3, n=(40, 36, 30), pe=(4, 3, 3), order=4, integrator="ab2", c=(1.0, 1.0, 1.0), L=4, steps=24, ra=0.02),
    "3d_o6_rk2_burgers": dict(ndim=3, n=(36, 36, 36), pe=(3, 3, 3), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=4, steps=16, ra=0.004),
    # 32 x 32 cross-sections take the 1024-thread 3-D path
    "3d_fast_o6_rk2_burgers": dict(ndim=3, n=(64, 64, 64), pe=(2, 2, 2), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=4, steps=10, ra=0.004),
    "3d_fast_o2_euler": dict(ndim=3, n=(64, 32, 64), pe=(2, 1, 2), order=2, integrator="euler", c=(1.0, 0.5, -0.5), L=3, steps=14, ra=0.05),
    "3d_fast_o4_ab3_px1": dict(ndim=3, n=(32, 64, 32), pe=(1, 2, 1), order=4, integrator="ab3", c=(1.0, 1.0, 1.0), L=4, steps=14, ra=0.01),
    "3d_fast_o4_ab2_bz16": dict(ndim=3, n=(64, 64, 48), pe=(2, 2, 3), order=4, integrator="ab2", c=(1.0, -1.0, 0.5), L=4, steps=12, ra=0.02),
    "3d_fast_o4_ab2_sync": dict(ndim=3, n=(64, 64, 32), pe=(2, 2, 1), order=4, integrator="ab2", c=(1.0, -1.0, 0.5), mode="sync", steps=12, ra=0.02),
    "3d_o2_euler_sync": dict(ndim=3, n=(32, 32, 32), pe=(2, 2, 2), order=2, integrator="euler", c=(1.0, 0.5, 0.25), mode="sync", steps=20, ra=0.05),
    # degenerate and extreme cases: the smallest PE edge b = 2s on every axis,
    # L = 1 (every delay 0), one PE per axis (a PE is its own neighbour), the
    # largest L and T, the 32 x 32 path with the thinnest PE (bz = 2s)
    "1d_o4_min_edge": dict(ndim=1, n=(16,), pe=(4,), order=4, integrator="ab2", c=(1.0,), L=3, steps=30, ra=0.02),
    "2d_o6_min_edge": dict(ndim=2, n=(18, 12), pe=(3, 2), order=6, integrator="euler", c=(1.0, -1.0), L=2, steps=20, ra=0.005),
    "3d_o2_min_edge": dict(ndim=3, n=(8, 6, 4), pe=(4, 3, 2), order=2, integrator="euler", c=(0.5, 1.0, -1.0), L=3, steps=20, ra=0.05),
    "1d_o2_L1": dict(ndim=1, n=(64,), pe=(4,), order=2, integrator="euler", c=(1.0,), L=1, steps=50, ra=0.1),
    "2d_o4_one_pe_per_axis": dict(ndim=2, n=(24, 20), pe=(1, 1), order=4, integrator="ab2", c=(1.0, 0.5), L=4, steps=30, ra=0.02),
    "1d_o6_L8_T4_rk2": dict(ndim=1, n=(96,), pe=(4,), order=6, integrator="rk2", c=(1.0,), L=8, steps=60, ra=0.002),
    # the 512^3 Burgers workload's scheme (sixth order, T = 4, L = 8, Heun RK2)
    # on the 32 x 32 path for long enough that delays reach 7 and ring
    # back-indices k + m reach 10 of the 12-slot ring
    "3d_fast_o6_L8_rk2_burgers": dict(ndim=3, n=(64, 64, 64), pe=(2, 2, 2), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=8, steps=28, ra=0.002),
    "3d_fast_o6_L8_rk2_burgers_pz1": dict(ndim=3, n=(64, 64, 32), pe=(2, 2, 1), order=6, integrator="rk2", equation="burgers", alpha=0.05, L=8, steps=20, ra=0.002),
    "3d_fast_o4_ab2_bz4": dict(ndim=3, n=(64, 64, 8), pe=(2, 2, 2), order=4, integrator="ab2", c=(1.0, -0.5, 0.5), L=4, steps=12, ra=0.02),
    # space-expanded single-level schemes (second-order CD): Case 2 (diffusion,
    # (2,1,2)) and Case 3 (advection-diffusion, (1,2,2)a + (2,2,2)a) with the
    # paper's p = {0.5, 0.3, 0.2}, then other integrators, shapes and the
    # thinnest PEs the stencils allow (b = 2 for (2,1,2), 3 for (2,2,2)a)
    "1d_o2_space212_case2": dict(ndim=1, n=(128,), pe=(16,), order=2, integrator="euler", c=(0.0,), L=3, weights=[5, 3, 2], scheme="space212", steps=200, ra=0.05),
    "1d_o2_space222_case3": dict(ndim=1, n=(128,), pe=(16,), order=2, integrator="euler", c=(1.0,), L=3, weights=[5, 3, 2], scheme="space222", steps=200, ra=0.05),
    "1d_o2_space222_ab2_min_edge": dict(ndim=1, n=(24,), pe=(8,), order=2, integrator="ab2", c=(1.0,), L=4, scheme="space222", steps=60, ra=0.05),
    "1d_o2_space212_min_edge": dict(ndim=1, n=(16,), pe=(8,), order=2, integrator="euler", c=(0.5,), L=3, scheme="space212", steps=60, ra=0.05),
    "2d_o2_space212_ragged": dict(ndim=2, n=(40, 36), pe=(4, 3), order=2, integrator="euler", c=(1.0, -0.5), L=3, scheme="space212", steps=40, ra=0.05),
    "2d_o2_space222_rk2": dict(ndim=2, n=(30, 24), pe=(3, 4), order=2, integrator="rk2", c=(1.0, 0.5), L=4, scheme="space222", steps=30, ra=0.05),
    "3d_o2_space222_ab2": dict(ndim=3, n=(24, 20, 18), pe=(2, 2, 3), order=2, integrator="ab2", c=(1.0, 1.0, -0.5), L=3, scheme="space222", steps=16, ra=0.05),
    "3d_o2_space212_burgers": dict(ndim=3, n=(20, 20, 20), pe=(2, 2, 2), order=2, integrator="ab2", equation="burgers", alpha=0.05, L=4, scheme="space212", steps=12, ra=0.02),
    # 32 x 32 cross-sections: the space-expanded schemes on the 3-D fast path
    "3d_fast_o2_space222": dict(ndim=3, n=(64, 64, 32), pe=(2, 2, 2), order=2, integrator="euler", c=(1.0, -0.5, 0.5), L=3, weights=[5, 3, 2], scheme="space222", steps=14, ra=0.05),
    "3d_fast_o2_space212_ab2": dict(ndim=3, n=(64, 32, 64), pe=(2, 1, 2), order=2, integrator="ab2", c=(0.5, 1.0, -1.0), L=4, scheme="space212", steps=14, ra=0.05),
    "3d_fast_o2_space222_rk2_burgers": dict(ndim=3, n=(64, 64, 24), pe=(2, 2, 2), order=2, integrator="rk2", equation="burgers", alpha=0.05, L=3, scheme="space222", steps=10, ra=0.02),
    "3d_fast_o2_space222_ab3_bz6": dict(ndim=3, n=(32, 64, 12), pe=(1, 2, 2), order=2, integrator="ab3", c=(1.0, 1.0, 1.0), L=4, scheme="space222", steps=12, ra=0.02),
    # deep PEs on the generic 3-D sweep: their planes are split into z-chunks
    # of several workgroups, with two solution buffers for AB2 (few PEs: down
    # to single-plane chunks, each reloading the strip-depth planes around it;
    # 4^3 PEs of 42 planes: 4 chunks of 11, the last one ragged)
    "3d_o4_ab2_chunked": dict(ndim=3, n=(40, 40, 48), pe=(2, 2, 1), order=4, integrator="ab2", c=(1.0, -0.5, 0.7), L=4, steps=10, ra=0.02),
    "3d_o6_rk2_chunked": dict(ndim=3, n=(30, 30, 40), pe=(1, 1, 2), order=6, integrator="rk2", c=(0.5, 0.5, 1.0), L=3, steps=8, ra=0.004),
    "3d_o4_ab2_chunk_ragged": dict(ndim=3, n=(48, 48, 168), pe=(4, 4, 4), order=4, integrator="ab2", c=(0.7, 1.0, -0.5), L=4, steps=6, ra=0.02),
    # non-uniform delays at the two buffer points (Sec. 3.4 Example 1); L = 8
    # and L = 5 with uniform bins reach the singular set 3 k1 = k2 many times
    "1d_o2_nonuniform_case2": dict(ndim=1, n=(128,), pe=(16,), order=2, integrator="euler", c=(0.0,), L=8, scheme="nonuniform212", steps=200, ra=0.05),
    "1d_o2_nonuniform_ab2_min_edge": dict(ndim=1, n=(16,), pe=(8,), order=2, integrator="ab2", c=(1.0,), L=4, scheme="nonuniform212", steps=60, ra=0.05),
    "2d_o2_nonuniform_rk2_ragged": dict(ndim=2, n=(40, 36), pe=(4, 3), order=2, integrator="rk2", c=(1.0, -0.5), L=6, scheme="nonuniform212", steps=30, ra=0.05),
    "3d_o2_nonuniform_burgers": dict(ndim=3, n=(20, 20, 20), pe=(2, 2, 2), order=2, integrator="ab2", equation="burgers", alpha=0.05, L=4, scheme="nonuniform212", steps=12, ra=0.02),
    "1d_o2_nonuniform_single_pe_L5": dict(ndim=1, n=(32,), pe=(1,), order=2, integrator="ab2", c=(1.0,), L=5, weights=[1, 1, 1, 3, 3], scheme="nonuniform212", steps=80, ra=0.05),
    "2d_o2_nonuniform_pe1x5_ab3": dict(ndim=2, n=(24, 40), pe=(1, 5), order=2, integrator="ab3", c=(0.5, 1.0), L=8, scheme="nonuniform212", steps=40, ra=0.02),
    "3d_o2_nonuniform_32x32_ab3": dict(ndim=3, n=(64, 64, 24), pe=(2, 2, 2), order=2, integrator="ab3", c=(1.0, 1.0, 1.0), L=5, scheme="nonuniform212", steps=12, ra=0.02),
}


def _case(name):
    c = dict(CASES[name])
    c["dt"] = _dt(c, c.pop("ra"))
    return c


_ORACLE_RUNS = {}


def _run_pair(case, precision):
    u0 = initial_field(case)
    steps = case["steps"]
    _say(f"[parity] {case} precision={precision}")
    s = solver_for(case, precision)
    s.set_state(torch.from_numpy(u0))
    s.step(steps)
    got = s.state().double().cpu()
    key = repr(sorted((k, repr(v)) for k, v in case.items()))
    if key not in _ORACLE_RUNS:       # both precisions compare with one oracle run
        o = oracle_for(case, u0)
        o.run(steps)
        _ORACLE_RUNS.clear()
        _ORACLE_RUNS[key] = o
    return got, _ORACLE_RUNS[key]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_field_parity(name, precision):
    case = _case(name)
    got, o = _run_pair(case, precision)
    check_field(got, o, TOL[precision], label=(name, precision))


@pytest.mark.parametrize("name", ["1d_o2_euler_L3", "2d_o4_ab2_ragged", "3d_o4_ab2_ragged", "3d_o6_rk2_burgers",
                                  "1d_o2_space222_case3", "2d_o2_nonuniform_rk2_ragged"])
def test_delays_bit_exact(name):
    case = _case(name)
    s = solver_for(case, "f64")
    steps = 40
    got = s.delays(0, steps)
    o = oracle_for(case, initial_field(case))
    for n in range(steps):
        want = delay_table(o.prob, o.dm, n).numpy()
        assert np.array_equal(got[n], want.reshape(got[n].shape)), n


@pytest.mark.parametrize("name", ["1d_o4_ab2_ragged", "2d_o4_ab2_ragged", "3d_o4_ab2_ragged", "3d_o6_rk2_burgers",
                                  "3d_fast_o6_rk2_burgers", "3d_fast_o4_ab2_bz16", "1d_o2_space222_case3",
                                  "2d_o2_space212_ragged", "3d_o2_space222_ab2", "3d_fast_o2_space222",
                                  "1d_o2_nonuniform_case2", "3d_o2_nonuniform_32x32_ab3", "3d_o4_ab2_chunked",
                                  "3d_o6_rk2_chunked", "3d_o4_ab2_chunk_ragged"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_zero_delays_equal_synchronous_bitwise(name, precision):
    case = _case(name)
    u0 = torch.from_numpy(initial_field(case))
    out = {}
    for mode in ("zero", "sync"):
        c = dict(case, mode=mode)
        s = solver_for(c, precision)
        s.set_state(u0)
        s.step(case["steps"])
        out[mode] = s.state()
    assert torch.equal(out["zero"], out["sync"])


@pytest.mark.parametrize("name", ["1d_o2_nonuniform_case2", "3d_o2_nonuniform_32x32_ab3"])
def test_nonuniform_cases_reach_the_singular_set(name):
    """The non-uniform parity cases draw (k1, k2) on the singular set 3 k1 = k2
    with k1 >= 1 (handled by the older level k1 + 1) and pairs with k1 != k2;
    their field parity is test_field_parity."""
    from oracle.solver import point_delay_table
    case = _case(name)
    o = oracle_for(case, initial_field(case))
    sing = unequal = 0
    for n in range(case["steps"]):
        K1 = delay_table(o.prob, o.dm, n)
        K2 = point_delay_table(o.prob, o.dm, n)
        sing += int(((3 * K1 == K2) & (K1 >= 1)).sum())
        unequal += int((K1 != K2).sum())
    assert sing >= 3 and unequal > 10 * sing, (sing, unequal)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_nonuniform_with_one_delay_level_is_the_synchronous_scheme(precision):
    """L = 1: every delay is 0, so no face takes the four-point stencil."""
    case = dict(_case("2d_o2_nonuniform_rk2_ragged"), L=1)
    u0 = torch.from_numpy(initial_field(case))
    out = {}
    for mode in ("rng", "sync"):
        s = solver_for(dict(case, mode=mode), precision)
        s.set_state(u0)
        s.step(case["steps"])
        out[mode] = s.state()
    assert torch.equal(out["rng"], out["sync"])


@pytest.mark.parametrize("name", ["2d_o2_nonuniform_rk2_ragged", "1d_o2_nonuniform_case2"])
def test_nonuniform_point_delays_bit_exact(name):
    """The device's second-point delays equal the generator's (the face
    delays are test_delays_bit_exact); other schemes have none."""
    from oracle.solver import point_delay_table
    from paper_1702_00496_amd import ATError
    case = _case(name)
    s = solver_for(case, "f64")
    steps = 60
    got = s.point_delays(0, steps)
    o = oracle_for(case, initial_field(case))
    for n in range(steps):
        want = point_delay_table(o.prob, o.dm, n).numpy()
        assert np.array_equal(got[n], want.reshape(got[n].shape)), n
    assert not np.array_equal(got, s.delays(0, steps))
    with pytest.raises(ATError, match="per-point"):
        solver_for(_case("1d_o2_space222_case3"), "f64").point_delays(0, 4)


def test_nonuniform_scheme_rejects_host_tables_and_other_orders():
    from paper_1702_00496_amd import ATError
    case = _case("1d_o2_nonuniform_ab2_min_edge")
    with pytest.raises(ATError, match="per-point"):
        solver_for(dict(case, mode="host", host=np.zeros((4, 8, 1, 2), dtype=np.int8)))
    with pytest.raises(ATError, match="order 2"):
        solver_for(dict(case, order=4, n=(32,), pe=(4,)))


def test_zero_steps_and_repeated_state_are_no_ops():
    case = _case("1d_o4_ab2_ragged")
    u0 = torch.from_numpy(initial_field(case))
    s = solver_for(case, "f64")
    s.set_state(u0)
    s.step(0)
    assert s.n_step == 0
    assert torch.equal(s.state().cpu(), u0.reshape(s.shape))
    s.step(7)
    a = s.state()
    s.set_state(u0)                       # back to step 0: the same 7 steps again
    s.step(3)
    s.step(0)
    s.step(4)
    assert torch.equal(s.state(), a)


def test_host_delay_table():
    case = _case("2d_o4_ab2_ragged")
    steps = case["steps"]
    npe = 12
    rs = np.random.Generator(np.random.PCG64(21))
    tab = rs.integers(0, case["L"], size=(steps, npe, 2, 2)).astype(np.int8)
    tab[:, 5, :, :] = case["L"] - 1          # one PE always maximally late
    case = dict(case, mode="host", host=tab)
    got, o = _run_pair(case, "f64")
    check_field(got, o, TOL["f64"], label="host delays")


def test_first_configuration_full_run():
    """N = 256, 8 PEs, L = 3, 1000 Euler steps, u0 = sin x (FP64)."""
    cfg = W.config_1d_advdiff()
    case = dict(ndim=1, n=cfg["n"][:1], pe=cfg["pe"][:1], order=2, integrator="euler", c=(1.0,),
                alpha=cfg["alpha"], dt=cfg["dt"], L=cfg["L"], seed=cfg["seed"], steps=cfg["steps"])
    u0 = W.eval_modes(cfg["modes"], cfg["n"], 1)
    s = solver_for(case, "f64")
    s.set_state(torch.from_numpy(u0))
    s.step(case["steps"])
    o = oracle_for(case, u0)
    o.run(case["steps"])
    check_field(s.state().cpu(), o, 1e-12, label="1-D workload")
    # error against the analytic decaying sine, computed by the library and by the oracle
    from oracle.analytic import advected_modes
    from oracle.norms import error_norms
    from oracle.solver import boundary_mask
    want = error_norms(o.u, advected_modes(o.prob, cfg["modes"], o.t), boundary_mask(o.prob))
    got = s.norms(modes=cfg["modes"])
    for k in ("l1", "l2", "linf", "l2_b", "l2_i", "l1_b", "l1_i"):
        assert abs(got[k] - want[k]) <= 1e-9 * want[k], (k, got[k], want[k])


@pytest.mark.parametrize("name", ["3d_o4_ab2_ragged", "3d_fast_o2_space222", "2d_o2_space212_ragged",
                                  "2d_o2_nonuniform_rk2_ragged", "3d_o4_ab2_chunked"])
def test_checkpoint_resume_bitwise(name):
    case = _case(name)
    u0 = torch.from_numpy(initial_field(case))
    a = solver_for(case, "f64")
    a.set_state(u0)
    a.step(30)
    ref = a.state()
    b = solver_for(case, "f64")
    b.set_state(u0)
    b.step(13)
    ck = b.save()
    b.step(5)                 # diverge, then restore
    b.load(ck)
    b.step(17)
    assert torch.equal(b.state(), ref)


@pytest.mark.parametrize("name", ["3d_o4_ab2_ragged", "3d_o6_rk2_burgers", "1d_o2_euler_L3", "3d_fast_o6_rk2_burgers",
                                  "3d_fast_o2_space222_rk2_burgers", "1d_o2_space222_case3",
                                  "3d_o2_nonuniform_32x32_ab3", "3d_o6_rk2_chunked"])
def test_graph_replay_equals_plain_launches(name):
    case = _case(name)
    u0 = torch.from_numpy(initial_field(case))
    a = solver_for(case, "f32")
    a.set_state(u0)
    a.step(21)
    b = solver_for(case, "f32")
    b.set_graph(4)
    b.set_state(u0)
    for _ in range(3):        # replays with eager work and syncs in between
        b.step(7)
        torch.cuda.synchronize()
        _ = b.state().sum().item()
    assert torch.isfinite(a.state()).all()
    assert torch.equal(a.state(), b.state())


def _full_case():
    cfg = W.config_3d_advdiff()
    return cfg, dict(ndim=3, n=cfg["n"], pe=cfg["pe"], order=4, integrator="ab2", c=cfg["c"],
                     alpha=cfg["alpha"], dt=cfg["dt"], L=cfg["L"], T=cfg["T"], seed=cfg["seed"])


def test_full_size_3d_workload_first_steps():
    """256^3, 8^3 PEs of 32^3, L = 4, AB2, in the graph launch configuration of
    the benchmark: the first 6 steps (every delay value 0..3 is reachable at
    step 5) against the oracle, FP64 and FP32 bulk."""
    cfg, case = _full_case()
    steps = 6
    u0 = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], 3))
    _say("[parity] full-size oracle run")
    o = oracle_for(case, u0)
    o.run(steps)
    for precision in ("f64", "f32"):
        s = solver_for(case, precision)
        s.set_graph(3)
        s.set_state(u0.cuda())
        s.step(steps)
        e = check_field(s.state().cpu(), o, TOL[precision], label=("full size", precision))
        _say(f"[parity] full size {precision}: {e}")
        d = s.delays(0, steps)
        for n in range(steps):
            assert np.array_equal(d[n], o.delays[n].numpy().reshape(d[n].shape))


@pytest.mark.parametrize("scheme", ["space222", "space212"])
def test_full_size_space_expanded_workload_first_steps(scheme):
    """The benchmark's space-expanded workload (256^3, 8^3 PEs of 32^3,
    second-order CD, Euler, L = 3 with p = {0.5, 0.3, 0.2}) in its graph
    launch configuration: the first 4 steps against the oracle, FP32 bulk."""
    cfg = W.config_3d_advdiff(n=256, b=32)
    dx = 2 * math.pi / 256
    case = dict(ndim=3, n=cfg["n"], pe=cfg["pe"], order=2, integrator="euler", c=(1.0, 1.0, 1.0), alpha=0.1,
                dt=0.05 * dx * dx / 0.1, L=3, weights=[5, 3, 2], seed=cfg["seed"], scheme=scheme)
    steps = 4
    u0 = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], 3))
    _say(f"[parity] full-size {scheme} oracle run")
    o = oracle_for(case, u0)
    o.run(steps)
    s = solver_for(case, "f32")
    s.set_graph(2)
    s.set_state(u0.cuda())
    s.step(steps)
    e = check_field(s.state().cpu(), o, TOL["f32"], label=("full size", scheme))
    _say(f"[parity] full size {scheme} f32: {e}")
    d = s.delays(0, steps)
    for n in range(steps):
        assert np.array_equal(d[n], o.delays[n].numpy().reshape(d[n].shape))


def test_full_size_3d_workload_full_run_properties():
    """All 500 steps at full size: the AT error against the exact solution
    matches the synchronous scheme's (fourth order, Sec. 5.2 Case 4); FP32
    bulk stays within 1e-5 of FP64; zero delays reproduce the synchronous
    scheme bit for bit."""
    cfg, case = _full_case()
    u0 = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], 3)).cuda()
    res = {}
    for key, precision, mode in [("at64", "f64", "rng"), ("at32", "f32", "rng"), ("sync64", "f64", "sync"),
                                 ("zero64", "f64", "zero")]:
        s = solver_for(dict(case, mode=mode), precision)
        s.set_graph(50)
        s.set_state(u0)
        s.step(cfg["steps"])
        res[key] = (s.state().double(), s.norms(modes=cfg["modes"]))
        _say(f"[parity] {key}: l2 error {res[key][1]['l2']:.4e}")
    assert torch.equal(res["zero64"][0], res["sync64"][0])
    e_at, e_sy = res["at64"][1]["l2"], res["sync64"][1]["l2"]
    assert abs(e_at - e_sy) <= 0.05 * e_sy
    check_field(res["at32"][0].cpu(), res["at64"][0].cpu(), 1e-5, prob=problem_for(case), label="f32 vs f64")


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_schedule_depths_bit_identical_and_autotune_restores_state(precision):
    case = _case("3d_fast_o4_ab2_bz16")
    u0 = torch.from_numpy(initial_field(case))
    outs = []
    from paper_1702_00496_amd import FAST_VARIANTS as VARIANTS
    for depth in VARIANTS:
        s = solver_for(case, precision)
        s.set_tuning(depth)
        assert s.tuning() == depth
        s.set_state(u0)
        s.step(9)
        outs.append(s.state())
    assert all(torch.equal(outs[0], o) for o in outs[1:])
    s = solver_for(case, precision)
    s.set_state(u0)
    s.step(4)
    before = s.state()
    best, ms = s.autotune(nsteps=3)
    assert best in VARIANTS and set(ms) == set(VARIANTS)
    assert torch.equal(s.state(), before) and s.n_step == 4
    s.step(5)
    assert torch.equal(s.state(), outs[0])


def test_autotune_cache_stores_then_applies_without_timing(tmp_path):
    """The first autotune of a problem class times the candidates and stores
    the winner; a second context of the same class (other data, other seed)
    takes it from the cache; another class misses."""
    from paper_1702_00496_amd import tuning
    case = _case("3d_fast_o4_ab2_bz16")
    path = str(tmp_path / "tuning.json")
    u0 = torch.from_numpy(initial_field(case))
    a = solver_for(case, "f32")
    a.set_state(u0)
    best, ms = a.autotune(nsteps=3, cache=path)
    ent = tuning.lookup(path, a.tuning_key())
    assert ent is not None and ent["variant"] == best and len(ent["ms"]) == len(ms)
    b = solver_for(dict(case, seed=99), "f32")
    b.set_state(2 * u0)
    assert b.tuning_key() == a.tuning_key()
    best2, ms2 = b.autotune(nsteps=3, cache=path)
    assert best2 == best and b.tuning() == best and ms2 == ms
    c = solver_for(case, "f64")
    assert c.tuning_key() != a.tuning_key() and tuning.lookup(path, c.tuning_key()) is None


def test_full_size_burgers_workload_properties():
    """512^3 viscous Burgers (16^3 PEs of 32^3, sixth order, T = 4, L = 8, Heun
    RK2) in the benchmark's launch configuration, 8 steps (delays up to 5
    reachable): the device delay draw equals the generator bit for bit; zero
    delays reproduce the synchronous scheme bit for bit; FP32 bulk stays
    within 1e-5 of FP64; the delays change the field (AT != synchronous) by
    far less than the field; the discrete energy does not grow (viscous
    Burgers dissipates)."""
    from oracle import rng as orng
    cfg = W.config_3d_burgers()
    case = dict(ndim=3, n=cfg["n"], pe=cfg["pe"], order=6, integrator="rk2", equation="burgers",
                alpha=cfg["alpha"], L=cfg["L"], T=cfg["T"], seed=cfg["seed"], dt=cfg["dt"])
    u0 = torch.from_numpy(W.burgers_spectrum_field(cfg["n"][0], 3, seed=cfg["seed"])).cuda()
    steps = 8
    res = {}
    for key, precision, mode in [("at32", "f32", "rng"), ("at64", "f64", "rng"), ("zero32", "f32", "zero"),
                                 ("sync32", "f32", "sync")]:
        s = solver_for(dict(case, mode=mode), precision)
        s.set_graph(4)
        s.set_state(u0)
        s.step(steps)
        res[key] = s.state().double().cpu()
        if key == "at32":
            d = s.delays(0, steps)
            npe = 16 ** 3
            thr = orng.thresholds(cfg["L"])
            for n in range(steps):
                for pid in (0, 1, 17, 300, npe - 1):
                    for f in range(6):
                        want = orng.clamp_startup(orng.raw_delay(cfg["seed"], n, pid * 6 + f, thr), n, cfg["T"])
                        assert d[n, pid, f // 2, f % 2] == want, (n, pid, f)
        del s
        torch.cuda.empty_cache()
        _say(f"[parity] burgers {key}: done")
    assert torch.equal(res["zero32"], res["sync32"])
    check_field(res["at32"], res["at64"], 1e-5, prob=problem_for(case), label="burgers f32 vs f64")
    diff = rel_l2(res["at64"], res["sync32"])
    _say(f"[parity] burgers AT vs synchronous: rel L2 {diff:.3e}")
    assert 0.0 < diff < 1e-3
    e0 = float((u0.double() ** 2).sum())
    assert float((res["at64"] ** 2).sum()) <= e0 * (1 + 1e-12)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_non_finite_field_reports_unstable(precision):
    """A field that holds a NaN (a blown-up run) makes the norm evaluation
    return AT_EUNSTABLE instead of numbers; a finite field of the same problem
    does not."""
    from paper_1702_00496_amd import ATError, _lib
    case = _case("3d_fast_o4_ab2_bz16")
    u0 = torch.from_numpy(initial_field(case))
    s = solver_for(case, precision)
    s.set_state(u0)
    s.step(3)
    modes = W.make_modes([(1, 2, 1)], [1.0], seed=4)
    assert all(math.isfinite(v) for v in s.norms(modes=modes).values())
    bad = u0.clone()
    bad[5, 7, 11] = float("nan")
    s.set_state(bad)
    s.step(3)
    with pytest.raises(ATError) as ei:
        s.norms(modes=modes)
    assert ei.value.status == _lib.AT_EUNSTABLE


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_generic_sweep_chunk_variants_bit_identical_and_autotuned(precision):
    """The generic 3-D sweep's z-chunk schedule variants (1, 2, 4, 8, 16
    chunks per PE) give the cost-model split's field bit for bit and the
    oracle's within the bar; the autotuner times exactly those variants on
    such a problem, restores the state and keeps the fastest."""
    from paper_1702_00496_amd import CHUNK_VARIANTS
    case = _case("3d_o4_ab2_chunked")
    u0 = torch.from_numpy(initial_field(case))
    ref = solver_for(case, precision)
    ref.set_state(u0)
    ref.step(case["steps"])
    want = ref.state()
    for v in CHUNK_VARIANTS:
        s = solver_for(case, precision)
        s.set_tuning(v)
        s.set_state(u0)
        s.step(case["steps"])
        assert torch.equal(s.state(), want), v
    o = oracle_for(case, u0.numpy())
    o.run(case["steps"])
    check_field(want.double().cpu(), o, TOL[precision], label="chunked")
    s = solver_for(case, precision)
    s.set_state(u0)
    s.step(3)
    before = s.state()
    best, ms = s.autotune(nsteps=3)
    assert best in CHUNK_VARIANTS and set(ms) == set(CHUNK_VARIANTS), (best, ms)
    assert torch.equal(s.state(), before) and s.n_step == 3
    s.step(case["steps"] - 3)
    assert torch.equal(s.state(), want)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_pe_major_fields_round_trip_and_variant_checks(precision):
    """Problems of the 32 x 32 path keep u PE-major inside the library: a
    [z][y][x] field set and read back comes out bit for bit through the
    16-byte vector copy and through the element-wise copy that unaligned
    caller buffers take; the state after steps does not depend on the
    alignment of the buffers; a schedule variant whose planes in flight do
    not divide the PE depth is refused (AT_EINVAL), and where the default's
    do not, the default is variant 1. Then the odd-depth problem matches the
    oracle within the bar."""
    import ctypes
    from paper_1702_00496_amd import ATError, _lib
    case = dict(ndim=3, n=(64, 32, 15), pe=(2, 1, 3), order=4, integrator="ab2", c=(1.0, -1.0, 0.5), L=4,
                steps=7)
    case["dt"] = _dt(case, 0.02)
    dtype = torch.float32 if precision == "f32" else torch.float64
    u0 = torch.from_numpy(initial_field(case)).to(dtype)
    s = solver_for(case, precision)
    assert s.tuning() == 1                      # bz = 5: two planes in flight do not divide it
    for v in (2, 4, 10, 18):
        with pytest.raises(ATError) as ei:
            s.set_tuning(v)
        assert ei.value.status == _lib.AT_EINVAL
    assert s.tuning() == 1
    s.set_tuning(17)                            # one plane in flight, alternating
    # unaligned caller buffers: one element into a larger allocation
    big = torch.empty(u0.numel() + 1, dtype=dtype, device="cuda")
    big[1:].copy_(u0.reshape(-1).cuda())
    raw = s._lib.at_set_state(s._ctx, ctypes.c_void_p(big[1:].data_ptr()))
    assert raw == _lib.AT_OK
    back = torch.empty(u0.numel() + 1, dtype=dtype, device="cuda")
    assert s._lib.at_get_state(s._ctx, ctypes.c_void_p(back[1:].data_ptr())) == _lib.AT_OK
    torch.cuda.synchronize()
    assert torch.equal(back[1:].cpu().reshape(u0.shape), u0)
    s.step(case["steps"])
    assert s._lib.at_get_state(s._ctx, ctypes.c_void_p(back[1:].data_ptr())) == _lib.AT_OK
    torch.cuda.synchronize()
    t = solver_for(case, precision)             # aligned buffers, default variant
    t.set_state(u0)
    assert torch.equal(t.state().cpu(), u0)
    t.step(case["steps"])
    want = t.state()
    assert torch.equal(back[1:].reshape(want.shape), want)
    o = oracle_for(case, u0.double().numpy())
    o.run(case["steps"])
    check_field(want.double().cpu(), o, TOL[precision], prob=problem_for(case), label="bz=5 PE-major")
