"""Shared case builders for the GPU parity tests: one dict describes a problem;
the oracle and the HIP library are each constructed from it independently."""
import numpy as np
import torch

import workloads as W
from oracle.solver import DelayModel, Oracle, Problem, boundary_mask


def problem_for(case):
    return Problem(ndim=case["ndim"], n=case["n"], pe=case["pe"], dt=case["dt"], order=case["order"],
                   equation=case.get("equation", "advdiff"), c=case.get("c", (0.0, 0.0, 0.0)),
                   alpha=case.get("alpha", 0.1), integrator=case.get("integrator", "euler"))


def oracle_for(case, u0):
    prob = Problem(ndim=case["ndim"], n=case["n"], pe=case["pe"], dt=case["dt"], order=case["order"],
                   equation=case.get("equation", "advdiff"), c=case.get("c", (0.0, 0.0, 0.0)),
                   alpha=case.get("alpha", 0.1), integrator=case.get("integrator", "euler"))
    dm = DelayModel(L=case.get("L", 3), T=case.get("T", 0), mode=case.get("mode", "rng"),
                    seed=case.get("seed", 0), weights=case.get("weights"),
                    host=case.get("host"), scheme=case.get("scheme", "time"))
    return Oracle(prob, dm, torch.as_tensor(u0, dtype=torch.float64))


def solver_for(case, precision="f64"):
    from paper_1702_00496_amd import Solver
    host = case.get("host")
    return Solver(ndim=case["ndim"], n=case["n"], pe=case["pe"], dt=case["dt"], order=case["order"],
                  equation=case.get("equation", "advdiff"), c=case.get("c", (0.0, 0.0, 0.0)),
                  alpha=case.get("alpha", 0.1), integrator=case.get("integrator", "euler"),
                  precision=precision, L=case.get("L", 3), T=case.get("T", 0),
                  mode=case.get("mode", "rng"), seed=case.get("seed", 0),
                  weights=case.get("weights"), scheme=case.get("scheme", "time"),
                  host_delays=None if host is None else np.asarray(host, dtype=np.int8))


def initial_field(case):
    n = tuple(case["n"]) + (1,) * (3 - len(case["n"]))
    if case.get("equation") == "burgers":
        u = W.eval_modes(W.make_modes([(1, 2, 1), (2, 1, 3), (3, 1, 1)], [0.5, 0.3, 0.2], seed=case.get("ic_seed", 4)),
                         n, case["ndim"])
    else:
        u = W.eval_modes(W.make_modes([(1, 2, 1), (2, 1, 3), (3, 1, 2)], [1.0, 0.5, 0.25], seed=case.get("ic_seed", 4)),
                         n, case["ndim"])
    return u


def rel_l2(a, b):
    a = torch.as_tensor(a, dtype=torch.float64).reshape(-1)
    b = torch.as_tensor(b, dtype=torch.float64).reshape(-1)
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def field_errors(got, want, prob=None):
    """Relative errors of a field against the oracle's, element by element:
    ``l2`` = ||d||_2 / ||want||_2 over all points, ``max`` = max|d| / max|want|
    (relative Linf), and, when the problem is given, ``ib`` = the relative L2
    over the boundary set I_B only (points within s of a PE face, where the
    delayed levels enter)."""
    g = torch.as_tensor(got, dtype=torch.float64)
    w = torch.as_tensor(want, dtype=torch.float64)
    if prob is not None:
        g = g.reshape(prob.shape)
        w = w.reshape(prob.shape)
    d = g - w
    out = {"l2": float(torch.linalg.norm(d.reshape(-1)) / torch.linalg.norm(w.reshape(-1))),
           "max": float(d.abs().max() / w.abs().max())}
    if prob is not None:
        m = boundary_mask(prob)
        if bool(m.any()):
            out["ib"] = float(torch.linalg.norm(d[m]) / torch.linalg.norm(w[m]))
    return out


def check_field(got, want, tol, prob=None, label=""):
    """Assert every error of ``field_errors`` is within ``tol`` (and the field
    is finite); ``want`` may be an Oracle (its current level and problem are
    used). Returns the errors."""
    if isinstance(want, Oracle):
        prob = want.prob if prob is None else prob
        want = want.u
    g = torch.as_tensor(got, dtype=torch.float64)
    assert bool(torch.isfinite(g).all()), (label, "non-finite values")
    e = field_errors(g, want, prob)
    assert all(v <= tol for v in e.values()), (label, e, tol)
    return e
