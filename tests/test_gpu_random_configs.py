"""Seeded random configurations against the oracle: dimension, ragged PE
shapes, order, scheme family, T, L and bin weights, integrator, equation,
delay mode and precision drawn together, so that combinations no hand-picked
case covers are still checked to the usual bar (relative L2 <= 1e-12 FP64,
<= 1e-5 FP32). Every configuration is one the library's validation accepts."""
import math
import random

import numpy as np
import pytest
import torch

from tests._cases import check_field, initial_field, oracle_for, solver_for

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def draw(seed):
    rng = random.Random(seed)
    ndim = rng.choice((1, 1, 2, 2, 3))
    scheme = rng.choice(("time", "time", "time", "space212", "space222", "nonuniform212"))
    order = 2 if scheme != "time" else rng.choice((2, 4, 6))
    s = order // 2
    depth = 3 if scheme == "space222" else (2 if scheme != "time" else s)
    need = max(2 * s, depth)
    n, pe = [], []
    for a in range(ndim):
        p = rng.choice((1, 2, 3, 4)) if ndim < 3 else rng.choice((1, 2, 3))
        b = rng.randint(need, need + (9 if ndim == 1 else 5 if ndim == 2 else 3))
        n.append(p * b)
        pe.append(p)
    equation = rng.choice(("advdiff", "advdiff", "burgers"))
    integrator = rng.choice(("euler", "ab2", "ab3", "rk2"))
    L = rng.randint(1, 6)
    T = 0 if scheme != "time" else rng.choice((0, 0, 1))
    weights = None if rng.random() < 0.5 else [rng.randint(1, 5) for _ in range(L)]
    c = tuple(round(rng.uniform(-1, 1), 3) for _ in range(ndim))
    alpha = 0.05 if equation == "burgers" else 0.1
    dx = 2 * math.pi / max(n)
    case = dict(ndim=ndim, n=tuple(n), pe=tuple(pe), order=order, integrator=integrator, equation=equation,
                c=c, alpha=alpha, L=L, T=T, weights=weights, scheme=scheme, seed=rng.randint(0, 2 ** 31),
                mode=rng.choice(("rng", "rng", "rng", "zero")), dt=min(0.005 * dx * dx / alpha, 0.02 * dx),
                steps=rng.randint(5, 25), ic_seed=rng.randint(0, 100))
    return case, rng.choice(("f64", "f32"))


@pytest.mark.parametrize("seed", range(64))
def test_random_configuration_matches_the_oracle(seed):
    case, precision = draw(1000 + seed)
    print(f"[random] seed {seed}: {case} {precision}", flush=True)
    u0 = initial_field(case)
    s = solver_for(case, precision)
    s.set_state(torch.from_numpy(u0))
    s.step(case["steps"])
    got = s.state().double().cpu()
    o = oracle_for(case, u0)
    o.run(case["steps"])
    check_field(got, o, TOL[precision], label=(case, precision))
    if case["mode"] == "rng":
        d = s.delays(0, case["steps"])
        for k in range(case["steps"]):
            assert np.array_equal(d[k], o.delays[k].numpy().reshape(d[k].shape)), k


def draw_deep(seed):
    """A 3-D problem for the generic sweep with deep PEs (16..40 planes, no
    32 x 32 cross-section, few PEs), so that its planes are split over
    several workgroups."""
    rng = random.Random(seed)
    scheme = rng.choice(("time", "time", "space212", "space222", "nonuniform212"))
    order = 2 if scheme != "time" else rng.choice((2, 4, 6))
    s = order // 2
    need = max(2 * s, 3 if scheme == "space222" else 2)
    pe = tuple(rng.choice((1, 2)) for _ in range(3))
    b = (rng.randint(need, 12), rng.randint(need, 12), rng.randint(16, 40))
    n = tuple(p * e for p, e in zip(pe, b))
    equation = rng.choice(("advdiff", "advdiff", "burgers"))
    alpha = 0.05 if equation == "burgers" else 0.1
    dx = 2 * math.pi / max(n)
    case = dict(ndim=3, n=n, pe=pe, order=order, integrator=rng.choice(("euler", "ab2", "ab3", "rk2")),
                equation=equation, c=tuple(round(rng.uniform(-1, 1), 3) for _ in range(3)), alpha=alpha,
                L=rng.randint(1, 5), T=0 if scheme != "time" else rng.choice((0, 0, 1)), weights=None,
                scheme=scheme, seed=rng.randint(0, 2 ** 31), mode=rng.choice(("rng", "rng", "zero", "sync")),
                dt=min(0.005 * dx * dx / alpha, 0.02 * dx), steps=rng.randint(3, 10), ic_seed=rng.randint(0, 100))
    return case, rng.choice(("f64", "f32"))


@pytest.mark.parametrize("seed", range(32))
def test_random_deep_generic_configuration_matches_the_oracle(seed):
    case, precision = draw_deep(3000 + seed)
    print(f"[random] deep seed {seed}: {case} {precision}", flush=True)
    u0 = initial_field(case)
    s = solver_for(case, precision)
    s.set_state(torch.from_numpy(u0))
    s.step(case["steps"])
    got = s.state().double().cpu()
    o = oracle_for(case, u0)
    o.run(case["steps"])
    check_field(got, o, TOL[precision], label=(case, precision))


def draw_wide(seed):
    """A deep-PE draw (as above) on up to 4 x 4 x 4 PEs of 8..48 planes, so
    that the split of each PE's planes into z-chunks meets the limit of one
    resident round and leaves ragged last chunks."""
    case, precision = draw_deep(seed)
    rng = random.Random(7 * seed + 1)
    pe = tuple(rng.choice((1, 2, 3, 4)) for _ in range(3))
    b = [e // p for e, p in zip(case["n"], case["pe"])]
    b[2] = rng.randint(8, 48)
    case["pe"] = pe
    case["n"] = tuple(p * e for p, e in zip(pe, b))
    dx = 2 * math.pi / max(case["n"])
    case["dt"] = min(0.005 * dx * dx / case["alpha"], 0.02 * dx)
    return case, precision


@pytest.mark.parametrize("seed", range(96))
def test_random_wide_generic_configuration_matches_the_oracle(seed):
    case, precision = draw_wide(7000 + seed)
    print(f"[random] wide seed {seed}: {case} {precision}", flush=True)
    u0 = initial_field(case)
    s = solver_for(case, precision)
    s.set_state(torch.from_numpy(u0))
    s.step(case["steps"])
    got = s.state().double().cpu()
    o = oracle_for(case, u0)
    o.run(case["steps"])
    check_field(got, o, TOL[precision], label=(case, precision))


@pytest.mark.parametrize("seed", range(12))
def test_random_configuration_checkpoint_and_graph_are_bitwise(seed):
    """Plain launches against a graph-replayed run that is checkpointed,
    driven past the checkpoint, restored and resumed: the same bits (one
    solution buffer or two, every integrator and scheme family)."""
    case, precision = (draw if seed % 2 == 0 else draw_deep)(5000 + seed)
    steps = case["steps"] + 6
    u0 = torch.from_numpy(initial_field(case))
    a = solver_for(case, precision)
    a.set_state(u0)
    a.step(steps)
    want = a.state()
    b = solver_for(case, precision)
    b.set_graph(3)
    b.set_state(u0)
    b.step(4)
    ck = b.save()
    b.step(5)
    b.load(ck)
    b.step(steps - 4)
    assert torch.equal(b.state(), want), (case, precision)
