"""ctypes declarations of the libatfd C ABI (include/atfd.h).

Argument marshalling only: every computation happens in the HIP library.
Importing this module loads ``libatfd.so`` from this package directory and
raises if it is missing; there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libatfd.so")

AT_OK, AT_EINVAL, AT_ENOMEM, AT_EHIP, AT_EUNSTABLE, AT_ESTATE = range(6)
STATUS_NAMES = {0: "AT_OK", 1: "AT_EINVAL", 2: "AT_ENOMEM", 3: "AT_EHIP", 4: "AT_EUNSTABLE", 5: "AT_ESTATE"}
EQUATIONS = {"advdiff": 0, "burgers": 1}
INTEGRATORS = {"euler": 0, "ab2": 1, "ab3": 2, "rk2": 3}
PRECISIONS = {"f64": 0, "f32": 1}
MODES = {"rng": 0, "zero": 1, "host": 2, "sync": 3}
SCHEMES = {"time": 0, "space212": 1, "space222": 2, "nonuniform212": 3}


class AtProblem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("pe", ctypes.c_int32 * 3),
        ("n", ctypes.c_int64 * 3),
        ("length", ctypes.c_double),
        ("c", ctypes.c_double * 3),
        ("alpha", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("equation", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("precision", ctypes.c_int32),
    ]


class AtDelay(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("T", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("weights", ctypes.POINTER(ctypes.c_uint32)),
        ("host_delays", ctypes.POINTER(ctypes.c_int8)),
        ("host_nsteps", ctypes.c_int64),
    ]


class AtEnsMember(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("pe", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("T", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("length", ctypes.c_double),
        ("c", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("weights", ctypes.POINTER(ctypes.c_uint32)),
    ]


class AtDerivation(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in ("status", "order", "n_cond", "n_unknown", "rank_a", "rank_ab")]


DERIVE_STATUS = {0: "unique", 1: "none", 2: "infinite"}

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
SZ = ctypes.c_size_t
DP = ctypes.POINTER(ctypes.c_double)
IP = ctypes.POINTER(ctypes.c_int32)
LP = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes); the complete exported surface of include/atfd.h
SIGNATURES = {
    "at_version": (ctypes.c_char_p, []),
    "at_workspace_size": (I32, [ctypes.POINTER(AtProblem), ctypes.POINTER(AtDelay), ctypes.POINTER(SZ)]),
    "at_create": (I32, [ctypes.POINTER(AtProblem), ctypes.POINTER(AtDelay), P, SZ, P, ctypes.POINTER(P)]),
    "at_set_state": (I32, [P, P]),
    "at_step": (I32, [P, I64]),
    "at_set_graph": (I32, [P, I32]),
    "at_set_tuning": (I32, [P, I32]),
    "at_get_tuning": (I32, [P, ctypes.POINTER(I32)]),
    "at_autotune": (I32, [P, P, SZ, I32, ctypes.POINTER(I32), DP]),
    "at_get_state": (I32, [P, P]),
    "at_get_step": (I32, [P, ctypes.POINTER(I64)]),
    "at_get_delays": (I32, [P, I64, I64, ctypes.POINTER(ctypes.c_int8)]),
    "at_get_point_delays": (I32, [P, I64, I64, ctypes.POINTER(ctypes.c_int8)]),
    "at_norms": (I32, [P, I32, ctypes.POINTER(I32), DP, DP, P, DP]),
    "at_norms_noalloc": (I32, [P, I32, ctypes.POINTER(I32), DP, DP, P, DP]),
    "at_checkpoint_size": (I32, [P, ctypes.POINTER(SZ)]),
    "at_save": (I32, [P, P]),
    "at_load": (I32, [P, P]),
    "at_destroy": (I32, [P]),
    "at_last_error": (ctypes.c_char_p, [P]),
    "at_adjoint_scratch_size": (I32, [P, I64, I32, ctypes.POINTER(SZ)]),
    "at_adjoint": (I32, [P, I64, I32, P, P, SZ, P, DP]),
    "at_ens_workspace_size": (I32, [I32, ctypes.POINTER(AtEnsMember), I32, ctypes.POINTER(SZ)]),
    "at_ens_create": (I32, [I32, ctypes.POINTER(AtEnsMember), I32, P, SZ, P, ctypes.POINTER(P)]),
    "at_ens_set_state": (I32, [P, P]),
    "at_ens_run": (I32, [P, I64]),
    "at_ens_set_tuning": (I32, [P, I32, I32]),
    "at_ens_state_size": (I32, [P, ctypes.POINTER(SZ)]),
    "at_ens_autotune": (I32, [P, P, SZ, I64, ctypes.POINTER(I32), ctypes.POINTER(I32), DP]),
    "at_ens_get_tuning": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "at_ens_get_schedule": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "at_ens_get_state": (I32, [P, P]),
    "at_ens_get_step": (I32, [P, ctypes.POINTER(I64)]),
    "at_ens_norms": (I32, [P, I32, ctypes.POINTER(I32), DP, DP, P, DP]),
    "at_ens_error_stats": (I32, [P, I32, ctypes.POINTER(I32), DP, DP, P, I32, DP, DP]),
    "at_ens_destroy": (I32, [P]),
    "at_ens_last_error": (ctypes.c_char_p, [P]),
    "at_derive_scheme": (I32, [I32, I32, I32, I32, IP, IP, LP, LP, ctypes.POINTER(AtDerivation)]),
    "at_search_scheme": (I32, [I32, I32, I32, I32, I32, I32, I32, I32, I32, I32, IP, IP, IP, LP, LP,
                               ctypes.POINTER(AtDerivation)]),
}

_lib = None


def load():
    """Load libatfd.so (once). Raises OSError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_1702_00496_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ATError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, ctx=None, ens=False):
    if status != AT_OK:
        lib = load()
        msg = lib.at_ens_last_error(ctx) if ens else lib.at_last_error(ctx)
        raise ATError(status, msg.decode() if msg else "")
