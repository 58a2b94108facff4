"""Shared case builders for the GPU parity tests: one dict describes a problem;
the oracle and the HIP library are each constructed from it independently."""
import numpy as np
import torch

import workloads as W
from oracle.solver import DelayModel, Oracle, Problem


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
