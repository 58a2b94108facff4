"""The pipelined form of the generic 3-D sweep on a cross-section whose
quad count (400 for 40 x 40) exceeds its halo item count (320): the
workgroup has 448 threads, and the 48 past the quads repeat the last quad
(the same values to the same addresses). Checked against the oracle element
by element (relative L2 <= 1e-12 FP64, <= 1e-5 FP32) for the integrators
whose history is rewritten in place (AB3's f^{n-2} buffer, Heun's u^n), the
delay modes and ragged z-chunk splits of the PE's 25 planes (4, 7 and 13
chunks)."""
import math

import pytest
import torch

from tests._cases import check_field, initial_field, oracle_for, solver_for

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}

# integrator, delay mode, precision, schedule variant (0: the cost model;
# 33 + k: 2^k z-chunks per PE, clamped so that no chunk is empty)
CASES = [
    ("ab3", "rng", "f64", 0),
    ("rk2", "rng", "f32", 36),
    ("ab2", "sync", "f32", 0),
    ("ab3", "zero", "f32", 40),
    ("euler", "rng", "f64", 48),
]


@pytest.mark.parametrize("integrator,mode,precision,variant", CASES)
def test_pipelined_sweep_with_idle_quad_threads_matches_the_oracle(integrator, mode, precision, variant):
    n = (80, 80, 25)
    dx = 2 * math.pi / max(n)
    case = dict(ndim=3, n=n, pe=(2, 2, 1), order=4, integrator=integrator, equation="advdiff",
                c=(0.6, -0.3, 0.4), alpha=0.1, L=4, T=0, mode=mode, seed=23, scheme="time",
                dt=min(0.005 * dx * dx / 0.1, 0.02 * dx), steps=6, ic_seed=5)
    print(f"[pipe] {case} {precision} variant {variant}", flush=True)
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
