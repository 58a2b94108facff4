"""Asynchrony-tolerant finite differences on MI355X: thin Python binding.

The numerical work is done by the HIP library ``libatfd.so`` through the C
ABI of ``include/atfd.h``. PyTorch only provides device memory (the caller-
owned workspace) and the current HIP stream. Nothing here computes any part
of the method.
"""
import ctypes
import math

import numpy as np
import torch

from . import _lib, tuning
from ._lib import ATError, AtDelay, AtEnsMember, AtProblem, check

ENS_TUNE_CANDIDATES = 9

__all__ = ["Solver", "Ensemble", "ATEvolve", "evolve", "ATError", "lib", "VARIANTS", "FAST_VARIANTS", "CHUNK_VARIANTS"]

# schedule variants of the 3-D 32x32 sweep (see at_set_tuning)
# schedule variants: the 32 x 32 3-D path's (planes in flight, points per
# thread, alternating sweep direction) and the generic 3-D sweep's z-chunk
# counts; at_autotune reports them in this order
FAST_VARIANTS = (1, 2, 4, 9, 10, 12, 17, 18, 20)
CHUNK_VARIANTS = (33, 34, 36, 40, 48)
VARIANTS = FAST_VARIANTS + CHUNK_VARIANTS


def lib():
    return _lib.load()


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _as_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One AT simulation context (``at_create`` .. ``at_destroy``)."""

    def __init__(self, ndim, n, pe, dt, order=2, equation="advdiff", c=(0.0, 0.0, 0.0), alpha=0.0,
                 integrator="euler", precision="f64", length=2.0 * math.pi, L=1, T=0, mode="rng",
                 seed=0, weights=None, host_delays=None, device="cuda", scheme="time"):
        L_ = _lib.load()
        n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        pe = tuple(int(v) for v in pe) + (1,) * (3 - len(pe))
        c = tuple(float(v) for v in c) + (0.0,) * (3 - len(c))
        self.ndim, self.n, self.pe = ndim, n, pe
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.shape = (n[2], n[1], n[0])
        self.device = torch.device(device)
        prob = AtProblem()
        prob.ndim = ndim
        for a in range(3):
            prob.pe[a] = pe[a]
            prob.n[a] = n[a]
            prob.c[a] = c[a]
        prob.length = length
        prob.alpha = alpha
        prob.dt = dt
        prob.equation = _lib.EQUATIONS[equation]
        prob.order = order
        prob.integrator = _lib.INTEGRATORS[integrator]
        prob.precision = _lib.PRECISIONS[precision]
        dl = AtDelay()
        dl.L = L
        dl.T = T
        dl.mode = _lib.MODES[mode]
        dl.scheme = _lib.SCHEMES[scheme]
        dl.seed = seed
        self._keep = []
        if weights is not None:
            w = (ctypes.c_uint32 * len(weights))(*[int(v) for v in weights])
            self._keep.append(w)
            dl.weights = ctypes.cast(w, ctypes.POINTER(ctypes.c_uint32))
        if host_delays is not None:
            hd = np.ascontiguousarray(host_delays, dtype=np.int8)
            self._keep.append(hd)
            dl.host_delays = hd.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
            dl.host_nsteps = hd.shape[0]
        self._prob, self._delay = prob, dl
        self._spec = dict(ndim=ndim, edges=tuple(n[a] // pe[a] for a in range(3)), order=order, T=T,
                          scheme=scheme, precision=precision, integrator=integrator, equation=equation,
                          mode=mode)
        nbytes = ctypes.c_size_t(0)
        check(L_.at_workspace_size(ctypes.byref(prob), ctypes.byref(dl), ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        check(L_.at_create(ctypes.byref(prob), ctypes.byref(dl), _as_ptr(self.workspace),
                           nbytes.value, _stream_ptr(), ctypes.byref(ctx)))
        self._ctx = ctx
        self._lib = L_

    # -- lifetime
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.at_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state
    def set_state(self, u0):
        u0 = u0.to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(u0.shape) != self.shape:
            raise ValueError(f"u0 shape {tuple(u0.shape)} != {self.shape}")
        self._u0_keep = u0
        check(self._lib.at_set_state(self._ctx, _as_ptr(u0)), self._ctx)

    def step(self, nsteps=1):
        check(self._lib.at_step(self._ctx, int(nsteps)), self._ctx)

    def set_graph(self, chunk):
        check(self._lib.at_set_graph(self._ctx, int(chunk)), self._ctx)

    def set_tuning(self, depth):
        check(self._lib.at_set_tuning(self._ctx, int(depth)), self._ctx)

    def tuning(self):
        v = ctypes.c_int32(0)
        check(self._lib.at_get_tuning(self._ctx, ctypes.byref(v)), self._ctx)
        return v.value

    def tuning_key(self):
        """Cache key of this problem class on the current device."""
        props = torch.cuda.get_device_properties(self.device)
        return tuning.make_key(getattr(props, "gcnArchName", props.name), props.multi_processor_count,
                               **self._spec)

    def autotune(self, nsteps=10, cache=None):
        """Time every schedule candidate on the current state (restored
        afterwards) and keep the fastest. Returns (depth, {depth: ms/step}).

        ``cache``: path of a JSON tuning cache (``tuning.default_path()`` for
        the per-user one). A stored entry for this problem class is applied
        without timing (its recorded times are returned); otherwise the
        result is timed and stored."""
        if cache is not None:
            ent = tuning.lookup(cache, self.tuning_key())
            if ent is not None:
                self.set_tuning(ent["variant"])
                return ent["variant"], {int(k): v for k, v in ent.get("ms", {}).items()}
        scratch = torch.empty(self.checkpoint_size(), dtype=torch.uint8, device=self.device)
        best = ctypes.c_int32(0)
        ms = (ctypes.c_double * len(VARIANTS))()
        check(self._lib.at_autotune(self._ctx, _as_ptr(scratch), scratch.numel(), int(nsteps),
                                    ctypes.byref(best), ms), self._ctx)
        times = {d: ms[i] for i, d in enumerate(VARIANTS) if ms[i] >= 0}
        if cache is not None:
            tuning.store(cache, self.tuning_key(), best.value, times)
        return best.value, times

    def state(self):
        out = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        check(self._lib.at_get_state(self._ctx, _as_ptr(out)), self._ctx)
        return out

    @property
    def n_step(self):
        v = ctypes.c_int64(0)
        check(self._lib.at_get_step(self._ctx, ctypes.byref(v)), self._ctx)
        return v.value

    def delays(self, n0, count):
        npe = self.pe[0] * self.pe[1] * self.pe[2]
        out = np.zeros((count, npe, self.ndim, 2), dtype=np.int8)
        check(self._lib.at_get_delays(self._ctx, int(n0), int(count),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))), self._ctx)
        return out

    def point_delays(self, n0, count):
        """Second-buffer-point delays of the non-uniform-delay scheme
        (``at_get_point_delays``), shaped like ``delays``."""
        npe = self.pe[0] * self.pe[1] * self.pe[2]
        out = np.zeros((count, npe, self.ndim, 2), dtype=np.int8)
        check(self._lib.at_get_point_delays(self._ctx, int(n0), int(count),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))), self._ctx)
        return out

    def norms(self, modes=None, ref=None):
        """Error norms vs Fourier modes [(kappa3, amp, phase)] or a float64 reference field."""
        out = (ctypes.c_double * 9)()
        if modes:
            nm = len(modes)
            kap = (ctypes.c_int32 * (3 * nm))(*[int(k) for m in modes for k in (tuple(m[0]) + (0, 0, 0))[:3]])
            amp = (ctypes.c_double * nm)(*[float(m[1]) for m in modes])
            ph = (ctypes.c_double * nm)(*[float(m[2]) for m in modes])
            st = self._lib.at_norms(self._ctx, nm, kap, amp, ph, None, out)
        else:
            ref = ref.to(device=self.device, dtype=torch.float64).contiguous()
            st = self._lib.at_norms(self._ctx, 0, None, None, None, _as_ptr(ref), out)
        check(st, self._ctx)
        keys = ["l1", "l2", "linf", "l1_b", "l2_b", "l1_i", "l2_i", "n_b", "n_i"]
        return dict(zip(keys, list(out)))

    # -- adjoint
    def adjoint(self, nsteps, seed, every=64):
        """dJ/du^0 and dJ/dalpha for J(u^N) with dJ/du^N = seed, N = nsteps steps
        from the state set at step 0 (at_adjoint). Leaves the solver at step N."""
        seed = seed.to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(seed.shape) != self.shape:
            raise ValueError(f"seed shape {tuple(seed.shape)} != {self.shape}")
        nbytes = ctypes.c_size_t(0)
        check(self._lib.at_adjoint_scratch_size(self._ctx, int(nsteps), int(every), ctypes.byref(nbytes)),
              self._ctx)
        scratch = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        grad = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        ga = ctypes.c_double(0.0)
        check(self._lib.at_adjoint(self._ctx, int(nsteps), int(every), _as_ptr(seed), _as_ptr(scratch),
                                   scratch.numel(), _as_ptr(grad), ctypes.byref(ga)), self._ctx)
        return grad, ga.value

    # -- checkpoints
    def checkpoint_size(self):
        v = ctypes.c_size_t(0)
        check(self._lib.at_checkpoint_size(self._ctx, ctypes.byref(v)), self._ctx)
        return v.value

    def save(self, buf=None):
        if buf is None:
            buf = torch.empty(self.checkpoint_size(), dtype=torch.uint8, device=self.device)
        check(self._lib.at_save(self._ctx, _as_ptr(buf)), self._ctx)
        return buf

    def load(self, buf):
        check(self._lib.at_load(self._ctx, _as_ptr(buf)), self._ctx)


class Ensemble:
    """Many independent 1-D AT problems advanced in one persistent launch
    (``at_ens_create`` .. ``at_ens_destroy``).

    ``members``: list of dicts with keys n, pe, order, integrator ("euler" |
    "ab2"), L, T (0 = order/2+1), mode ("rng" | "zero" | "sync"), length, c,
    alpha, dt, seed (the member's generator key), weights (optional)."""

    def __init__(self, members, precision="f32", device="cuda"):
        L_ = _lib.load()
        self.count = len(members)
        arr = (AtEnsMember * self.count)()
        self._keep = []
        self.sizes = []
        for i, m in enumerate(members):
            a = arr[i]
            a.n = int(m["n"])
            a.pe = int(m["pe"])
            a.order = int(m["order"])
            a.integrator = _lib.INTEGRATORS[m.get("integrator", "euler")]
            a.L = int(m.get("L", 1))
            a.T = int(m.get("T", 0))
            a.mode = _lib.MODES[m.get("mode", "rng")]
            a.length = float(m.get("length", 2.0 * math.pi))
            a.c = float(m.get("c", 0.0))
            a.alpha = float(m.get("alpha", 0.0))
            a.dt = float(m["dt"])
            a.seed = int(m.get("seed", 0)) & (2 ** 64 - 1)
            if m.get("weights") is not None:
                w = (ctypes.c_uint32 * len(m["weights"]))(*[int(v) for v in m["weights"]])
                self._keep.append(w)
                a.weights = ctypes.cast(w, ctypes.POINTER(ctypes.c_uint32))
            self.sizes.append(a.n)
        self._arr = arr
        self._members = [dict(m) for m in members]
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.device = torch.device(device)
        self.total = sum(self.sizes)
        prec = _lib.PRECISIONS[precision]
        nbytes = ctypes.c_size_t(0)
        check(L_.at_ens_workspace_size(self.count, arr, prec, ctypes.byref(nbytes)), None, ens=True)
        self.workspace = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        check(L_.at_ens_create(self.count, arr, prec, _as_ptr(self.workspace), nbytes.value,
                               _stream_ptr(), ctypes.byref(ctx)), None, ens=True)
        self._ctx = ctx
        self._lib = L_

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.at_ens_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        check(st, self._ctx, ens=True)

    def set_state(self, u0):
        """u0: packed 1-D tensor of all members' initial fields."""
        u0 = u0.to(device=self.device, dtype=self.dtype).contiguous().reshape(-1)
        if u0.numel() != self.total:
            raise ValueError(f"u0 has {u0.numel()} values, members need {self.total}")
        self._u0_keep = u0
        self._check(self._lib.at_ens_set_state(self._ctx, _as_ptr(u0)))

    def run(self, nsteps):
        self._check(self._lib.at_ens_run(self._ctx, int(nsteps)))

    def set_tuning(self, groups_per_cu=0, threads=0):
        self._check(self._lib.at_ens_set_tuning(self._ctx, int(groups_per_cu), int(threads)))

    def tuning(self):
        """(workgroups per CU, threads per workgroup) of the persistent launch."""
        g, t = ctypes.c_int32(0), ctypes.c_int32(0)
        self._check(self._lib.at_ens_get_tuning(self._ctx, ctypes.byref(g), ctypes.byref(t)))
        return g.value, t.value

    def tuning_key(self):
        props = torch.cuda.get_device_properties(self.device)
        return tuning.make_ens_key(getattr(props, "gcnArchName", props.name), props.multi_processor_count,
                                   self._members, "f64" if self.dtype == torch.float64 else "f32")

    def autotune(self, nsteps=50, cache=None):
        """Time every schedule candidate (``at_ens_autotune``) from the current
        state (restored afterwards) and keep the fastest. Returns
        ((groups_per_cu, threads), {(groups, threads): ms/step}). ``cache``: a
        JSON tuning cache path; a stored entry for these members' shapes is
        applied without timing."""
        if cache is not None:
            ent = tuning.lookup(cache, self.tuning_key())
            if ent is not None and isinstance(ent["variant"], list):
                g, t = ent["variant"]
                self.set_tuning(g, t)
                return (g, t), {tuple(int(x) for x in k.split("x")): v for k, v in ent.get("ms", {}).items()}
        sz = ctypes.c_size_t(0)
        self._check(self._lib.at_ens_state_size(self._ctx, ctypes.byref(sz)))
        scratch = torch.empty(max(int(sz.value), 1), dtype=torch.uint8, device=self.device)
        g, t = ctypes.c_int32(0), ctypes.c_int32(0)
        ms = (ctypes.c_double * ENS_TUNE_CANDIDATES)()
        self._check(self._lib.at_ens_autotune(self._ctx, _as_ptr(scratch), sz.value, int(nsteps),
                                              ctypes.byref(g), ctypes.byref(t), ms))
        times = {(gc, tc): ms[3 * i + j] for i, gc in enumerate((1, 2, 4)) for j, tc in enumerate((256, 512, 1024))}
        if cache is not None:
            tuning.store(cache, self.tuning_key(), [g.value, t.value],
                         {f"{a}x{b}": v for (a, b), v in times.items()})
        return (g.value, t.value), times

    def state(self):
        out = torch.empty(self.total, dtype=self.dtype, device=self.device)
        self._check(self._lib.at_ens_get_state(self._ctx, _as_ptr(out)))
        return out

    def schedule(self):
        """(bin_start, order): workgroup j runs members order[bin_start[j]:bin_start[j+1]]."""
        nb = ctypes.c_int32(0)
        self._check(self._lib.at_ens_get_schedule(self._ctx, ctypes.byref(nb), None, None))
        starts = (ctypes.c_int32 * (nb.value + 1))()
        order = (ctypes.c_int32 * self.count)()
        self._check(self._lib.at_ens_get_schedule(self._ctx, ctypes.byref(nb), starts, order))
        return np.array(starts[:], dtype=np.int64), np.array(order[:], dtype=np.int64)

    def bin_sizes(self):
        starts, _ = self.schedule()
        return np.diff(starts)

    def members_beyond_batch(self, batch=24):
        """Members that their workgroup runs after its first ``batch`` members."""
        starts, order = self.schedule()
        out = []
        for j in range(len(starts) - 1):
            out.extend(int(i) for i in order[starts[j] + batch:starts[j + 1]])
        return out

    def split(self, packed):
        return list(torch.split(packed, self.sizes))

    @property
    def n_step(self):
        v = ctypes.c_int64(0)
        self._check(self._lib.at_ens_get_step(self._ctx, ctypes.byref(v)))
        return v.value

    def norms(self, kappas=None, amps=None, phases=None, ref=None):
        """Per-member (mean|E|, rms E, max|E|) as a (count, 3) numpy array, vs the
        exact series (kappas, amps shared; phases [count][nmodes]) or a packed
        float64 reference field."""
        out = np.zeros((self.count, 3), dtype=np.float64)
        optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if kappas is not None:
            nm = len(kappas)
            kap = (ctypes.c_int32 * nm)(*[int(k) for k in kappas])
            amp = (ctypes.c_double * nm)(*[float(a) for a in amps])
            ph = np.ascontiguousarray(phases, dtype=np.float64).reshape(self.count, nm)
            st = self._lib.at_ens_norms(self._ctx, nm, kap, amp,
                                        ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, optr)
        else:
            ref = ref.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1)
            st = self._lib.at_ens_norms(self._ctx, 0, None, None, None, _as_ptr(ref), optr)
        self._check(st)
        return out


    def error_stats(self, dx_edges, kappas=None, amps=None, phases=None, ref=None):
        """Per order group (2, 4, 6) and dx bin: (count, mean dx, mean RMS error,
        unbiased variance of the RMS error) as a (3, nbins, 4) numpy array
        (``at_ens_error_stats``); the reference as for :meth:`norms`."""
        edges = np.ascontiguousarray(dx_edges, dtype=np.float64)
        nb = len(edges) - 1
        out = np.zeros((3, nb, 4), dtype=np.float64)
        optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        eptr = edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if kappas is not None:
            nm = len(kappas)
            kap = (ctypes.c_int32 * nm)(*[int(k) for k in kappas])
            amp = (ctypes.c_double * nm)(*[float(a) for a in amps])
            ph = np.ascontiguousarray(phases, dtype=np.float64).reshape(self.count, nm)
            st = self._lib.at_ens_error_stats(self._ctx, nm, kap, amp,
                                              ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None,
                                              nb, eptr, optr)
        else:
            ref = ref.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1)
            st = self._lib.at_ens_error_stats(self._ctx, 0, None, None, None, _as_ptr(ref), nb, eptr, optr)
        self._check(st)
        return out


class ATEvolve(torch.autograd.Function):
    """u^N = ATEvolve.apply(u0, alpha, spec, nsteps, every): N AT steps of the
    problem ``spec`` (Solver keyword arguments without alpha) from u0 with
    diffusivity alpha. The backward pass is the library's hand-written
    adjoint (at_adjoint), with checkpoints every ``every`` steps."""

    @staticmethod
    def forward(ctx, u0, alpha, spec, nsteps, every):
        a = float(alpha)
        s = Solver(alpha=a, **spec)
        s.set_state(u0.detach())
        s.step(int(nsteps))
        out = s.state()
        ctx.save_for_backward(u0.detach())
        ctx.alpha, ctx.spec, ctx.nsteps, ctx.every = a, spec, int(nsteps), int(every)
        ctx.alpha_is_tensor = torch.is_tensor(alpha)
        return out

    @staticmethod
    def backward(ctx, g):
        (u0,) = ctx.saved_tensors
        s = Solver(alpha=ctx.alpha, **ctx.spec)
        s.set_state(u0)
        gu, ga = s.adjoint(ctx.nsteps, g.contiguous(), ctx.every)
        galpha = torch.tensor(ga, dtype=torch.float64, device=u0.device) if ctx.alpha_is_tensor else None
        return gu.to(u0.dtype), galpha, None, None, None


def evolve(u0, alpha, nsteps, every=64, **spec):
    """Differentiable N-step AT evolution (see ATEvolve)."""
    return ATEvolve.apply(u0, alpha, spec, nsteps, every)
