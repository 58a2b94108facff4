"""The allocation-free norm entry point (at_norms_noalloc) against at_norms
through the C ABI: two calls in a row on one GPU, the second on a smaller
field, each with the exact-solution reference and with a reference field;
the results must be identical (same kernels, same reduction order)."""
import ctypes
import math

import numpy as np
import pytest
import torch

import workloads as W
from tests._cases import solver_for

pytestmark = pytest.mark.gpu


def _both(s, modes=None, ref=None):
    out = {}
    for name in ("at_norms", "at_norms_noalloc"):
        buf = (ctypes.c_double * 9)()
        fn = getattr(s._lib, name)
        if modes is not None:
            nm = len(modes)
            kap = (ctypes.c_int32 * (3 * nm))(*[int(k) for m in modes for k in (tuple(m[0]) + (0, 0, 0))[:3]])
            amp = (ctypes.c_double * nm)(*[float(m[1]) for m in modes])
            ph = (ctypes.c_double * nm)(*[float(m[2]) for m in modes])
            st = fn(s._ctx, nm, kap, amp, ph, None, buf)
        else:
            r = ref.to(device=s.device, dtype=torch.float64).contiguous()
            st = fn(s._ctx, 0, None, None, None, ctypes.c_void_p(r.data_ptr()), buf)
        assert st == 0, (name, st)
        out[name] = list(buf)
    return out["at_norms"], out["at_norms_noalloc"]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_norms_equal_workspace_norms(precision):
    cases = [
        dict(ndim=3, n=(96, 64, 64), pe=(3, 2, 2), order=4, integrator="ab2", c=(1.0, -0.5, 0.5), L=4, steps=7),
        dict(ndim=2, n=(40, 24), pe=(4, 3), order=2, integrator="euler", c=(1.0, 0.5), L=3, steps=9),
    ]
    for case in cases:     # the second call works on a smaller field than the first
        dx = 2 * math.pi / max(case["n"])
        case["dt"] = 0.02 * dx * dx / 0.1
        n3 = tuple(case["n"]) + (1,) * (3 - len(case["n"]))
        modes = W.make_modes([(1, 2, 1), (2, 1, 3)][: 2], [1.0, 0.5], seed=4)
        u0 = torch.from_numpy(W.eval_modes(modes, n3, case["ndim"]))
        s = solver_for(case, precision)
        s.set_state(u0)
        s.step(case["steps"])
        a, b = _both(s, modes=modes)
        assert a == b, (case, a, b)
        assert all(np.isfinite(a)) and a[1] > 0
        ref = u0.to(torch.float64) * 0.5
        a, b = _both(s, ref=ref)
        assert a == b, (case, a, b)
        s.close()
