"""Host-side checks of the C ABI: the library loads, exports every function
include/atfd.h declares, and validates arguments without a GPU."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "atfd.h")
LIB = os.path.join(ROOT, "paper_1702_00496_amd", "libatfd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(at_[a-z0-9_]+)\s*\(", text)))


def _lib():
    if not os.path.exists(LIB):
        pytest.fail("libatfd.so is not built (python -m paper_1702_00496_amd.build)")
    from paper_1702_00496_amd import _lib as L
    return L, L.load()


def test_every_declared_function_is_exported():
    _, lib = _lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    L, _ = _lib()
    assert set(declared_functions()) <= set(L.SIGNATURES), set(declared_functions()) - set(L.SIGNATURES)


def _prob(L, **kw):
    p = L.AtProblem()
    p.ndim = kw.get("ndim", 3)
    for a in range(3):
        p.n[a] = kw.get("n", (64, 64, 64))[a]
        p.pe[a] = kw.get("pe", (2, 2, 2))[a]
    p.length = 2 * math.pi
    p.alpha = 0.1
    p.dt = 1e-4
    p.order = kw.get("order", 4)
    p.integrator = L.INTEGRATORS[kw.get("integrator", "ab2")]
    p.precision = L.PRECISIONS[kw.get("precision", "f64")]
    return p


def _delay(mod, **kw):
    d = mod.AtDelay()
    d.L = kw.get("L", 4)
    d.T = kw.get("T", 0)
    d.mode = mod.MODES[kw.get("mode", "rng")]
    d.scheme = mod.SCHEMES[kw.get("scheme", "time")]
    return d


def _size(L, lib, p, d):
    v = ctypes.c_size_t(0)
    st = lib.at_workspace_size(ctypes.byref(p), ctypes.byref(d), ctypes.byref(v))
    return st, v.value


def test_workspace_size_accounts_for_fields_and_rings():
    L, lib = _lib()
    p, d = _prob(L), _delay(L)
    st, nb = _size(L, lib, p, d)
    assert st == L.AT_OK
    npts = 64 ** 3
    # one solution buffer (updated in place) + one AB2 history at 8 bytes,
    # plus L+T ring slots of 6 faces * s * 32^2 per PE for 8 PEs
    ring = (4 + 3) * 8 * 6 * 2 * 32 * 32 * 8
    assert nb >= 2 * npts * 8 + ring
    assert nb < 2 * npts * 8 + ring + 4 * 2 ** 20
    # the synchronous arm: two solution buffers, no ring
    d.mode = L.MODES["sync"]
    st, nb2 = _size(L, lib, p, d)
    assert st == L.AT_OK and 3 * npts * 8 <= nb2 < 3 * npts * 8 + 4 * 2 ** 20


@pytest.mark.parametrize("kw,dkw", [
    (dict(n=(64, 64, 60), pe=(2, 2, 8)), {}),           # 60 % 8 != 0
    (dict(n=(64, 64, 64), pe=(2, 2, 32)), {}),          # PE edge 2 < 2s
    (dict(order=3), {}),
    (dict(ndim=4), {}),
    (dict(ndim=1, n=(64, 2, 1), pe=(2, 1, 1)), {}),     # unused axis with n > 1
    ({}, dict(L=9)),
    ({}, dict(L=0)),
    ({}, dict(T=5)),
    (dict(n=(256, 256, 8), pe=(2, 2, 1)), {}),          # PE x*y extent too large
])
def test_invalid_arguments_are_rejected(kw, dkw):
    L, lib = _lib()
    st, _ = _size(L, lib, _prob(L, **kw), _delay(L, **dkw))
    assert st == L.AT_EINVAL
    assert lib.at_last_error(None)


def test_space_expanded_schemes_size_rings_by_strip_depth_and_validate():
    """The space-expanded schemes keep one level (T = 1: L + 1 ring slots) of
    2 ((2,1,2)) or 3 ((2,2,2)a) buffer points per face."""
    L, lib = _lib()
    p = _prob(L, ndim=1, n=(64, 1, 1), pe=(8, 1, 1), order=2, integrator="euler")
    npts = 64
    sizes = {}
    for scheme in ("time", "space212", "space222"):
        st, nb = _size(L, lib, p, _delay(L, L=3, scheme=scheme))
        assert st == L.AT_OK, scheme
        sizes[scheme] = nb
    # ring bytes: slots x PEs x (2 faces x depth) x 8 B, solution in place
    ring = {"time": (3 + 2) * 8 * 2 * 1 * 8, "space212": (3 + 1) * 8 * 2 * 2 * 8,
            "space222": (3 + 1) * 8 * 2 * 3 * 8}
    for scheme, nb in sizes.items():
        assert npts * 8 + ring[scheme] <= nb < npts * 8 + ring[scheme] + 4 * 2 ** 20
    assert sizes["space222"] - sizes["space212"] <= 4096 + ring["space222"]
    bad = [
        (dict(ndim=1, n=(64, 1, 1), pe=(8, 1, 1), order=4), dict(scheme="space222")),    # order 4
        (dict(ndim=1, n=(16, 1, 1), pe=(8, 1, 1), order=2), dict(scheme="space222")),    # PE edge 2 < 3
        (dict(ndim=1, n=(64, 1, 1), pe=(8, 1, 1), order=2), dict(scheme="space212", T=3)),
    ]
    for kw, dkw in bad:
        st, _ = _size(L, lib, _prob(L, **kw), _delay(L, L=3, **dkw))
        assert st == L.AT_EINVAL, (kw, dkw)
    d = _delay(L, L=3)
    d.scheme = 4
    st, _ = _size(L, lib, p, d)
    assert st == L.AT_EINVAL
    st, _ = _size(L, lib, _prob(L, ndim=1, n=(16, 1, 1), pe=(8, 1, 1), order=2), _delay(L, L=3, scheme="space212"))
    assert st == L.AT_OK


def test_nonuniform_scheme_sizes_two_deep_strips_and_validates():
    """The non-uniform-delay scheme keeps one level of 2 buffer points per face
    (the space212 ring) and takes no host delay table."""
    L, lib = _lib()
    p = _prob(L, ndim=1, n=(64, 1, 1), pe=(8, 1, 1), order=2, integrator="euler")
    st, a = _size(L, lib, p, _delay(L, L=3, scheme="space212"))
    st2, b = _size(L, lib, p, _delay(L, L=3, scheme="nonuniform212"))
    assert st == st2 == L.AT_OK and a == b
    st, _ = _size(L, lib, _prob(L, ndim=1, n=(64, 1, 1), pe=(8, 1, 1), order=4), _delay(L, L=3, scheme="nonuniform212"))
    assert st == L.AT_EINVAL
    st, _ = _size(L, lib, p, _delay(L, L=3, scheme="nonuniform212", T=2))
    assert st == L.AT_EINVAL


def test_host_delay_table_is_validated():
    L, lib = _lib()
    import numpy as np
    p = _prob(L, ndim=1, n=(64, 1, 1), pe=(4, 1, 1), order=2)
    d = _delay(L, mode="host")
    d.L = 3
    tab = np.zeros((5, 4, 1, 2), dtype=np.int8)
    tab[2, 1, 0, 1] = 3          # >= L
    d.host_delays = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    d.host_nsteps = 5
    st, _ = _size(L, lib, p, d)
    assert st == L.AT_EINVAL
    tab[2, 1, 0, 1] = 2
    st, _ = _size(L, lib, p, d)
    assert st == L.AT_OK


def _members(specs):
    L, _ = _lib()
    arr = (L.AtEnsMember * len(specs))()
    for i, sp in enumerate(specs):
        m = dict(n=128, pe=4, order=2, integrator=0, L=3, T=0, mode=0, length=2 * math.pi, c=1.0,
                 alpha=0.1, dt=1e-4, seed=i)
        m.update(sp)
        for k, v in m.items():
            setattr(arr[i], k, v)
    return arr


def test_ensemble_workspace_size_accounts_for_members():
    L, lib = _lib()
    arr = _members([{}, dict(n=256, pe=4, order=4, integrator=1, L=4)])
    size = ctypes.c_size_t(0)
    assert lib.at_ens_workspace_size(2, arr, 1, ctypes.byref(size)) == L.AT_OK
    # two fields + the AB2 history of 384 floats, rings of 5 and 7 slots
    ring = (5 * 4 * 2 * 1 + 7 * 4 * 2 * 2) * 4
    assert size.value >= 3 * 384 * 4 + ring
    size64 = ctypes.c_size_t(0)
    assert lib.at_ens_workspace_size(2, arr, 0, ctypes.byref(size64)) == L.AT_OK
    assert size64.value > size.value


@pytest.mark.parametrize("bad", [
    dict(n=100, pe=3),              # n not a multiple of pe
    dict(n=6, pe=2, order=4),       # PE edge 3 < 2s
    dict(order=5),
    dict(integrator=3),             # RK2 is not offered for ensembles
    dict(L=9),
    dict(T=5),
    dict(mode=2),                   # host delay tables are not offered for ensembles
    dict(dt=0.0),
])
def test_ensemble_invalid_members_are_rejected(bad):
    L, lib = _lib()
    arr = _members([{}, bad])
    size = ctypes.c_size_t(0)
    assert lib.at_ens_workspace_size(2, arr, 1, ctypes.byref(size)) == L.AT_EINVAL
    assert b"member 1" in lib.at_ens_last_error(None)


def test_ensemble_needs_members_and_precision():
    L, lib = _lib()
    arr = _members([{}])
    size = ctypes.c_size_t(0)
    assert lib.at_ens_workspace_size(0, arr, 1, ctypes.byref(size)) == L.AT_EINVAL
    assert lib.at_ens_workspace_size(1, arr, 7, ctypes.byref(size)) == L.AT_EINVAL
