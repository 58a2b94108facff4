"""The generic 3-D sweep over y-slices. A PE cross-section of more than 768
quads (here 64 x 64) is too large for one workgroup of the pipelined sweep,
so each z-chunk is swept by two workgroups, one per half of the rows, each
taking the other half's edge rows as level-n halo values. Checked against the
oracle element by element (relative L2 <= 1e-12 FP64, <= 1e-5 FP32) over the
delay modes, integrators, equations and z-chunk counts that route through
it (two solution buffers: 4 PEs; Heun with one)."""
import math

import pytest
import torch

from tests._cases import check_field, initial_field, oracle_for, solver_for

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}

# integrator, delay mode, precision, schedule variant (0: the cost model;
# 33 + k: 2^k z-chunks per PE), equation
CASES = [
    ("ab2", "rng", "f64", 0, "advdiff"),
    ("ab2", "rng", "f32", 36, "advdiff"),
    ("rk2", "rng", "f64", 34, "burgers"),
    ("ab3", "sync", "f32", 0, "advdiff"),
    ("euler", "zero", "f64", 40, "advdiff"),
    ("ab3", "rng", "f64", 33, "burgers"),
]


@pytest.mark.parametrize("integrator,mode,precision,variant,equation", CASES)
def test_y_sliced_generic_sweep_matches_the_oracle(integrator, mode, precision, variant, equation):
    n = (128, 128, 24)
    alpha = 0.05 if equation == "burgers" else 0.1
    dx = 2 * math.pi / max(n)
    case = dict(ndim=3, n=n, pe=(2, 2, 1), order=4, integrator=integrator, equation=equation,
                c=(0.7, -0.4, 0.3), alpha=alpha, L=4, T=0, mode=mode, seed=11, scheme="time",
                dt=min(0.005 * dx * dx / alpha, 0.02 * dx), steps=5, ic_seed=3)
    print(f"[slices] {case} {precision} variant {variant}", flush=True)
    u0 = initial_field(case)
    s = solver_for(case, precision)
    if variant:
        s.set_tuning(variant)
    s.set_state(torch.from_numpy(u0))
    s.step(case["steps"])
    got = s.state().double().cpu()
    o = oracle_for(case, u0)
    o.run(case["steps"])
    check_field(got, o, TOL[precision], label=(case, precision, variant))
