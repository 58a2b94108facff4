"""Binding of the scheme-derivation calls of the C ABI (``at_derive_scheme``,
``at_search_scheme``): argument marshalling only. The order conditions, the
rank test and the exact elimination run in ``libatfd.so`` (host code, no GPU
needed); results come back as exact ``fractions.Fraction`` values.

A stencil is a list of (j, l) pairs: the scheme uses u_{i+j}^{n-l}
(Sec. 3.2 eq. general_deriv_at2); coefficients are dimensionless, the
derivative being sum c_{j,l} u_{i+j}^{n-l} / dx^d.
"""
import ctypes
from fractions import Fraction

from . import _lib

__all__ = ["derive_scheme", "search_scheme"]


def _info_dict(info):
    return {"status": _lib.DERIVE_STATUS[info.status], "order": info.order, "n_cond": info.n_cond,
            "n_unknown": info.n_unknown, "rank_a": info.rank_a, "rank_ab": info.rank_ab}


def derive_scheme(stencil, d, a, r):
    """Classify and solve eq. cond (Sec. 3.1) for an explicit stencil.

    Returns (status, coefficients, info): status 'unique', 'none' or
    'infinite'; coefficients a {(j, l): Fraction} for 'unique' (for
    'infinite' one member of the family, free entries zero; None for 'none');
    info holds the number of conditions and rank(A), rank(A|b).
    """
    lib = _lib.load()
    stencil = [(int(j), int(l)) for j, l in stencil]
    n = len(stencil)
    js = (ctypes.c_int32 * max(n, 1))(*[j for j, _ in stencil])
    ls = (ctypes.c_int32 * max(n, 1))(*[l for _, l in stencil])
    num = (ctypes.c_int64 * max(n, 1))()
    den = (ctypes.c_int64 * max(n, 1))()
    info = _lib.AtDerivation()
    _lib.check(lib.at_derive_scheme(d, a, r, n, js, ls, num, den, ctypes.byref(info)))
    out = _info_dict(info)
    if out["status"] == "none":
        return out["status"], None, out
    coefs = {stencil[i]: Fraction(num[i], den[i]) for i in range(n)}
    return out["status"], coefs, out


def search_scheme(d, a, r, s_min, k, T=1, with_centre=True, side="right", max_extent=12):
    """Smallest AT scheme with interior points -s_min..0 at level n and buffer
    points 1..s_max at levels n-k .. n-k-T+1 (mirrored for side='left').

    Returns (coefficients {(j, l): Fraction}, info) with info['order'] the
    accuracy reached, or (None, info) when no stencil up to max_extent gives one.
    """
    lib = _lib.load()
    cap = (s_min + 1) + max_extent * T
    n_out = ctypes.c_int32()
    js = (ctypes.c_int32 * cap)()
    ls = (ctypes.c_int32 * cap)()
    num = (ctypes.c_int64 * cap)()
    den = (ctypes.c_int64 * cap)()
    info = _lib.AtDerivation()
    sd = {"right": 1, "left": -1}.get(side, 0)    # anything else: the library rejects it
    _lib.check(lib.at_search_scheme(d, a, r, s_min, 1 if with_centre else 0, k, T, sd, max_extent, cap,
                                    ctypes.byref(n_out), js, ls, num, den, ctypes.byref(info)))
    out = _info_dict(info)
    if n_out.value == 0:
        return None, out
    return {(js[i], ls[i]): Fraction(num[i], den[i]) for i in range(n_out.value)}, out
