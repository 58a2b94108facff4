"""Seeded random configurations of the 3-D path for 32 x 32 PE cross-sections
(the benchmark's kernel) against the oracle: z-depth, PEs per axis, order,
integrator, equation, scheme family, delay mode, precision and schedule
variant drawn together; relative L2 <= 1e-12 (FP64), <= 1e-5 (FP32), device
delays bit-exact. Every configuration is one the library accepts and runs on
that path (T = s + 1 for the time-expanded schemes, a variant whose z-chunk
divides the PE depth)."""
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
    scheme = rng.choice(("time", "time", "time", "space212", "space222"))
    order = 2 if scheme != "time" else rng.choice((2, 4, 6))
    depth = rng.choice((1, 2, 4, 9, 10, 12)) if scheme == "time" else rng.choice((1, 2))
    chunk = depth & 7
    bz = chunk * rng.randint(max(1, (2 * (order // 2) + chunk - 1) // chunk), max(1, 12 // chunk))
    bz = max(bz, 2 * (order // 2), 3 if scheme == "space222" else 2)
    if bz % chunk:
        bz += chunk - bz % chunk
    pe = (rng.choice((1, 2)), rng.choice((1, 2)), rng.choice((1, 2)))
    n = (32 * pe[0], 32 * pe[1], bz * pe[2])
    equation = rng.choice(("advdiff", "advdiff", "burgers"))
    alpha = 0.05 if equation == "burgers" else 0.1
    dx = 2 * math.pi / max(n)
    case = dict(ndim=3, n=n, pe=pe, order=order, integrator=rng.choice(("euler", "ab2", "ab3", "rk2")),
                equation=equation, c=tuple(round(rng.uniform(-1, 1), 3) for _ in range(3)), alpha=alpha,
                L=rng.randint(1, 5), T=0, scheme=scheme, mode=rng.choice(("rng", "rng", "zero", "sync")),
                seed=rng.randint(0, 2 ** 31), dt=min(0.005 * dx * dx / alpha, 0.02 * dx),
                steps=rng.randint(3, 9), ic_seed=rng.randint(0, 100))
    if rng.random() < 0.4:
        case["weights"] = [rng.randint(1, 5) for _ in range(case["L"])]
    precision = rng.choice(("f64", "f32"))
    # the alternating-direction twins of the 4-point variants
    if scheme == "time" and depth in (1, 2, 4) and rng.random() < 0.5:
        depth += 16
    return case, precision, depth


@pytest.mark.parametrize("seed", range(128))
def test_random_fast3d_configuration_matches_the_oracle(seed):
    case, precision, depth = draw(500 + seed)
    print(f"[fast3d] seed {seed}: {case} {precision} variant {depth}", flush=True)
    u0 = initial_field(case)
    s = solver_for(case, precision)
    s.set_tuning(depth)
    s.set_state(torch.from_numpy(u0))
    s.step(case["steps"])
    got = s.state().double().cpu()
    o = oracle_for(case, u0)
    o.run(case["steps"])
    check_field(got, o, TOL[precision], label=(case, precision, depth))
    if case["mode"] == "rng":
        d = s.delays(0, case["steps"])
        for k in range(case["steps"]):
            assert np.array_equal(d[k], o.delays[k].numpy().reshape(d[k].shape)), k
