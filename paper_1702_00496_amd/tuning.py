"""Persistent cache of autotuned schedule variants (``at_autotune``).

A tuned variant depends on the device and on the problem's class, not on
its data: the key is (architecture, compute units, ndim, PE edges, order, T,
scheme, precision, integrator, equation, delay mode). Entries live in one
JSON file; writes replace the file atomically. Nothing here runs any part of
the method: the timing itself is ``at_autotune`` in the library.
"""
import json
import os
import tempfile

__all__ = ["default_path", "make_key", "make_ens_key", "lookup", "store"]


def default_path():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_1702_00496_amd", "tuning.json")


def make_key(arch, cus, ndim, edges, order, T, scheme, precision, integrator, equation, mode):
    b = "x".join(str(int(v)) for v in edges)
    return f"{arch}|cu{int(cus)}|dim{int(ndim)}|b{b}|o{int(order)}|T{int(T)}|{scheme}|{precision}|" \
           f"{integrator}|{equation}|{mode}"


def make_ens_key(arch, cus, members, precision):
    """Key of an ensemble's schedule: the device and the members' shapes and
    schemes (not their data, delay keys or coefficients)."""
    import hashlib
    h = hashlib.sha256()
    for m in members:
        h.update(f"{int(m['n'])},{int(m['pe'])},{int(m['order'])},{m.get('integrator', 'euler')},"
                 f"{int(m.get('L', 1))},{int(m.get('T', 0))},{m.get('mode', 'rng')};".encode())
    return f"{arch}|cu{int(cus)}|ensemble|{len(members)}|{precision}|{h.hexdigest()[:16]}"


def _load(path):
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def lookup(path, key):
    """The stored entry {"variant": int or [int, ...], "ms": {variant: ms}} or None."""
    ent = _load(path).get(key)
    if isinstance(ent, dict) and isinstance(ent.get("variant"), (int, list)):
        return ent
    return None


def store(path, key, variant, ms):
    data = _load(path)
    v = [int(x) for x in variant] if isinstance(variant, (list, tuple)) else int(variant)
    data[key] = {"variant": v, "ms": {str(k): float(x) for k, x in ms.items()}}
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuning.", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
