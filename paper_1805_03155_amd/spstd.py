"""Thin ctypes binding of libspstd (the C ABI in include/spstd.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch provides the device workspace (a uint8 tensor) and the
stream.  Loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspstd.so")

FP64, FP32 = 0, 1
NYQ_FULL, NYQ_ZERO = 0, 1
SYMPLECTIC, RK4 = 0, 1
BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN = 0, 1, 2
LAP_SPECTRAL, LAP_FD3 = 0, 1
ALLOW_UNSTABLE = 0x1
EAGER = 0x2          # no step-chunk graphs
TIMING = 0x4         # pass kernels bracketed by HIP events (pass_times)
NO_RESIDENT = 0x8    # 1D and small 2D plans/batches use the pass kernels, not a resident kernel
AUTOTUNE = 0x10      # batches: time the candidate schedules at creation, keep the fastest
NO_MERGE = 0x20      # plans: step boundaries kept whole (neither merged nor chained)
NO_PLANES = 0x40     # 3D batches: separate z and x passes instead of one launch per x-z plane
NO_FOURSTEP = 0x80   # 1D batches of 8192/16384 points: one workgroup per row pair per x pass
PASS_KINDS = ("y", "z", "xab", "x", "yba")
MAX_PROBES = 64

STATUS = {0: "SPSTD_OK", 1: "SPSTD_ERR_ARG", 2: "SPSTD_ERR_UNSTABLE",
          3: "SPSTD_ERR_WORKSPACE", 4: "SPSTD_ERR_DEVICE", 5: "SPSTD_ERR_NONFINITE",
          6: "SPSTD_ERR_CAPACITY", 7: "SPSTD_ERR_SCRATCH"}


class SpstdError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{STATUS.get(code, code)}: {msg}")


P = ctypes.POINTER
c_d, c_i64, c_int, c_u32, c_sz = (ctypes.c_double, ctypes.c_int64, ctypes.c_int,
                                  ctypes.c_uint32, ctypes.c_size_t)


class Desc(ctypes.Structure):
    _fields_ = [("ndim", c_int), ("n", c_i64 * 3), ("dx", c_d * 3), ("hbar", c_d),
                ("mass", c_d), ("precision", c_int), ("method", c_int), ("m", c_int),
                ("c", P(c_d)), ("d", P(c_d)), ("dt", c_d), ("cfl_fraction", c_d),
                ("nyquist", c_int), ("nprobes", c_int), ("probe_idx", P(c_i64)),
                ("flags", c_u32), ("bc", c_int * 3), ("laplacian", c_int), ("neig", c_int)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("ndim", c_int), ("n", c_i64 * 3), ("precision", c_int), ("m", c_int),
                ("c", P(c_d)), ("d", P(c_d)), ("nyquist", c_int), ("capacity", c_int),
                ("nprobes", c_int), ("nsteps_max", c_i64), ("flags", c_u32),
                ("waves_per_block", c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("steps_done", c_i64), ("dt", c_d), ("xmax", c_d), ("rho", c_d),
                ("norm0", c_d), ("norm", c_d), ("substeps_per_step", c_d)]


EXPORTS = ["spstd_xmax", "spstd_stable_dt", "spstd_workspace_size", "spstd_plan",
           "spstd_step", "spstd_run", "spstd_plan_info", "spstd_device_fields",
           "spstd_get_state", "spstd_set_state", "spstd_spectrum", "spstd_pass_times",
           "spstd_energy", "spstd_eig_begin", "spstd_eig_read",
           "spstd_destroy", "spstd_strerror", "spstd_last_error",
           "spstd_batch_workspace_size", "spstd_batch_create", "spstd_batch_load",
           "spstd_batch_step", "spstd_batch_read", "spstd_batch_release",
           "spstd_batch_slot_info", "spstd_batch_destroy", "spstd_batch_last_error",
           "spstd_batch_schedule", "spstd_run_noalloc",
           "spstd_batch_group_workspace_size", "spstd_batch_group_create", "spstd_batch_group_step",
           "spstd_batch_group_schedule", "spstd_batch_group_set_schedule", "spstd_batch_group_destroy",
           "spstd_batch_group_last_error"]

_lib = None


def lib():
    """Load libspstd.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1805_03155_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        pd, pi64 = P(c_d), P(c_i64)
        L.spstd_xmax.argtypes = [c_int, pd, pd, pd]
        L.spstd_stable_dt.argtypes = [P(Desc), pd, pd]
        L.spstd_workspace_size.argtypes = [P(Desc), c_i64, P(c_sz)]
        L.spstd_plan.argtypes = [P(Desc), pd, pd, pd, ctypes.c_void_p, c_sz, c_i64,
                                 ctypes.c_void_p, P(ctypes.c_void_p)]
        L.spstd_step.argtypes = [ctypes.c_void_p, c_i64]
        L.spstd_run.argtypes = [ctypes.c_void_p, c_i64, pd, P(Stats)]
        L.spstd_plan_info.argtypes = [ctypes.c_void_p, P(Stats)]
        L.spstd_device_fields.argtypes = [ctypes.c_void_p] + [P(ctypes.c_void_p)] * 3 + [P(pd)]
        L.spstd_get_state.argtypes = [ctypes.c_void_p, pd, pd, pi64]
        L.spstd_set_state.argtypes = [ctypes.c_void_p, pd, pd, c_i64]
        L.spstd_spectrum.argtypes = [pd, c_i64, c_int, c_d, c_d, c_int, pd, pd, P(c_int)]
        L.spstd_pass_times.argtypes = [ctypes.c_void_p, pi64, pd, pd]
        L.spstd_energy.argtypes = [ctypes.c_void_p, pd]
        L.spstd_eig_begin.argtypes = [ctypes.c_void_p, pd, c_int, c_i64]
        L.spstd_eig_read.argtypes = [ctypes.c_void_p, c_int, pd, pd]
        L.spstd_destroy.argtypes = [ctypes.c_void_p]
        vp = ctypes.c_void_p
        L.spstd_run_noalloc.argtypes = [P(Desc), vp, vp, vp, c_i64, vp, vp]
        L.spstd_batch_workspace_size.argtypes = [P(BatchDesc), P(c_sz)]
        L.spstd_batch_create.argtypes = [P(BatchDesc), vp, c_sz, vp, P(vp)]
        L.spstd_batch_load.argtypes = [vp, c_int, pd, c_d, c_d, c_d, c_d, pd, pd, pd, pi64, pd]
        L.spstd_batch_step.argtypes = [vp, c_i64]
        L.spstd_batch_read.argtypes = [vp, c_int, pd, pd, pd, pi64]
        L.spstd_batch_release.argtypes = [vp, c_int]
        L.spstd_batch_slot_info.argtypes = [vp, c_int, P(c_int), pi64, pd]
        L.spstd_batch_schedule.argtypes = [vp, P(c_int), P(c_int), pd]
        L.spstd_batch_destroy.argtypes = [vp]
        L.spstd_batch_last_error.argtypes = [vp]
        L.spstd_batch_last_error.restype = ctypes.c_char_p
        L.spstd_batch_group_workspace_size.argtypes = [P(vp), c_int, P(c_sz)]
        L.spstd_batch_group_create.argtypes = [P(vp), c_int, c_u32, vp, c_sz, vp, P(vp)]
        L.spstd_batch_group_step.argtypes = [vp, c_i64]
        L.spstd_batch_group_schedule.argtypes = [vp, P(c_int), P(c_int), pd]
        L.spstd_batch_group_set_schedule.argtypes = [vp, c_int]
        L.spstd_batch_group_destroy.argtypes = [vp]
        L.spstd_batch_group_last_error.argtypes = [vp]
        L.spstd_batch_group_last_error.restype = ctypes.c_char_p
        L.spstd_strerror.argtypes = [c_int]
        L.spstd_strerror.restype = ctypes.c_char_p
        L.spstd_last_error.argtypes = [ctypes.c_void_p]
        L.spstd_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("spstd_strerror", "spstd_last_error", "spstd_batch_last_error",
                            "spstd_batch_group_last_error"):
                getattr(L, name).restype = c_int
        _lib = L
    return _lib


def _check(rc, plan=None, batch=None, group=None):
    if rc != 0:
        msg = lib().spstd_strerror(rc).decode()
        if plan:
            msg += " / " + lib().spstd_last_error(plan).decode()
        if batch:
            msg += " / " + lib().spstd_batch_last_error(batch).decode()
        if group:
            msg += " / " + lib().spstd_batch_group_last_error(group).decode()
        raise SpstdError(rc, msg)


def _dp(a):
    return a.ctypes.data_as(P(c_d)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()


def make_desc(n, dx, c=None, d=None, dt=0.0, cfl_fraction=0.5, hbar=1.0, mass=1.0,
              precision=FP64, method=SYMPLECTIC, nyquist=NYQ_FULL, probes=(), flags=0, bc=None,
              laplacian=LAP_SPECTRAL, neig=0):
    """Build a descriptor; the returned object keeps its arrays alive.
    bc: boundary per axis (BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN), default
    periodic."""
    desc = Desc()
    desc.ndim = len(n)
    for a in range(3):
        desc.n[a] = int(n[a]) if a < len(n) else 1
        desc.dx[a] = float(dx[a]) if a < len(dx) else 1.0
    desc.hbar, desc.mass = float(hbar), float(mass)
    desc.precision, desc.method, desc.nyquist = precision, method, nyquist
    keep = []
    if method == SYMPLECTIC:
        ca, da = _f64(c), _f64(d)
        keep += [ca, da]
        desc.m = len(ca)
        desc.c, desc.d = _dp(ca), _dp(da)
    else:
        desc.m = 0
    desc.dt, desc.cfl_fraction = float(dt), float(cfl_fraction)
    pidx = np.ascontiguousarray(np.asarray(probes, dtype=np.int64).ravel())
    keep.append(pidx)
    desc.nprobes = len(pidx)
    desc.probe_idx = pidx.ctypes.data_as(P(c_i64)) if len(pidx) else None
    desc.flags = flags
    for a in range(3):
        desc.bc[a] = int(bc[a]) if bc is not None and a < len(bc) else BC_PERIODIC
    desc.laplacian = laplacian
    desc.neig = int(neig)
    desc._keep = keep
    return desc


def xmax(c, d):
    ca, da = _f64(c), _f64(d)
    out = c_d()
    _check(lib().spstd_xmax(len(ca), _dp(ca), _dp(da), ctypes.byref(out)))
    return out.value


def stable_dt(desc, V):
    V = _f64(V)
    out = c_d()
    _check(lib().spstd_stable_dt(ctypes.byref(desc), _dp(V), ctypes.byref(out)))
    return out.value


def workspace_size(desc, nsteps_max):
    out = c_sz()
    _check(lib().spstd_workspace_size(ctypes.byref(desc), int(nsteps_max), ctypes.byref(out)))
    return out.value


def spectrum(series, dt, hbar=1.0, nlevels=4):
    """Eigenvalues from a probe series [nsamples, nprobes, 2] (host FP64)."""
    s = np.ascontiguousarray(series, dtype=np.float64)
    ns, npr = s.shape[0], s.shape[1]
    E = np.zeros(nlevels)
    A = np.zeros(nlevels)
    nf = c_int()
    _check(lib().spstd_spectrum(_dp(s.ravel()), ns, npr, float(dt), float(hbar), nlevels,
                                _dp(E), _dp(A), ctypes.byref(nf)))
    return E[: nf.value], A[: nf.value]


class Plan:
    """One solver instance with its device workspace (a torch uint8 tensor)."""

    def __init__(self, desc, V, psiR0, psiI0=None, nsteps_max=0, device="cuda",
                 stream=None):
        import torch
        self.desc = desc
        self.nsteps_max = int(nsteps_max)
        V, pr, pi = _f64(V), _f64(psiR0), _f64(psiI0)
        self.npoints = int(np.prod([desc.n[a] for a in range(3)]))
        nbytes = workspace_size(desc, self.nsteps_max)
        dev = torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        self._off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            rc = lib().spstd_plan(ctypes.byref(desc), _dp(V), _dp(pr), _dp(pi),
                                  ctypes.c_void_p(base + self._off), nbytes, self.nsteps_max,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(rc)
        self.h = h
        self._destroy = lib().spstd_destroy
        self.nprobes = desc.nprobes

    def __del__(self):
        # the destroy function is bound at creation: module globals may be
        # gone when the interpreter shuts down
        h, fn = getattr(self, "h", None), getattr(self, "_destroy", None)
        if h is not None and h.value and fn is not None:
            fn(h)
            self.h = None

    def step(self, nsteps):
        _check(lib().spstd_step(self.h, int(nsteps)), self.h)

    def run(self, nsteps):
        """Advance and return (probe series [(steps_done+1), P, 2], stats)."""
        st = Stats()
        lib().spstd_plan_info(self.h, ctypes.byref(st))
        total = st.steps_done + int(nsteps)
        out = np.zeros((total + 1, max(self.nprobes, 1), 2))
        _check(lib().spstd_run(self.h, int(nsteps), _dp(out.ravel()) if self.nprobes else None,
                               ctypes.byref(st)), self.h)
        return (out[:, : self.nprobes] if self.nprobes else None), st

    def pass_times(self):
        """{kind: (launches, total_ms, bytes_per_launch)} since the last call
        (plans made with the TIMING flag)."""
        k = len(PASS_KINDS)
        n = np.zeros(k, np.int64)
        ms = np.zeros(k)
        by = np.zeros(k)
        _check(lib().spstd_pass_times(self.h, n.ctypes.data_as(P(c_i64)), _dp(ms), _dp(by)),
               self.h)
        return {PASS_KINDS[i]: (int(n[i]), float(ms[i]), float(by[i])) for i in range(k)}

    def energy(self):
        """(kinetic, potential, norm) of the current state, each summed over
        the grid times the cell volume; <H> = (kinetic + potential) / norm."""
        out = np.zeros(3)
        _check(lib().spstd_energy(self.h, _dp(out)), self.h)
        return float(out[0]), float(out[1]), float(out[2])

    def eig_begin(self, energies, nsteps):
        """Accumulate the windowed Fourier sums of the next nsteps states at
        the given energies (plan made with neig >= len(energies))."""
        E = _f64(np.atleast_1d(energies))
        self._neig = len(E)
        _check(lib().spstd_eig_begin(self.h, _dp(E), len(E), int(nsteps)), self.h)

    def eig_read(self, k):
        """Accumulator k as a complex array of the grid's size."""
        re = np.zeros(self.npoints)
        im = np.zeros(self.npoints)
        _check(lib().spstd_eig_read(self.h, int(k), _dp(re), _dp(im)), self.h)
        return re + 1j * im

    def info(self):
        st = Stats()
        _check(lib().spstd_plan_info(self.h, ctypes.byref(st)), self.h)
        return st

    @property
    def dt(self):
        return self.info().dt

    def get_state(self):
        pr = np.zeros(self.npoints)
        pi = np.zeros(self.npoints)
        step = c_i64()
        _check(lib().spstd_get_state(self.h, _dp(pr), _dp(pi), ctypes.byref(step)), self.h)
        return pr, pi, step.value

    def set_state(self, psiR, psiI, step):
        _check(lib().spstd_set_state(self.h, _dp(_f64(psiR)), _dp(_f64(psiI)), int(step)), self.h)

    def device_fields(self):
        """(psiR, psiI, V) as torch views of the workspace (no copy)."""
        import torch
        ptrs = [ctypes.c_void_p() for _ in range(3)]
        pp = P(c_d)()
        _check(lib().spstd_device_fields(self.h, *[ctypes.byref(x) for x in ptrs],
                                         ctypes.byref(pp)), self.h)
        dt = torch.float64 if self.desc.precision == FP64 else torch.float32
        es = 8 if self.desc.precision == FP64 else 4
        base = self.ws.data_ptr()
        out = []
        for x in ptrs:
            off = x.value - base
            out.append(self.ws[off: off + es * self.npoints].view(dt))
        return tuple(out)


def run_noalloc(desc, V, psiR, psiI, nsteps, probes=None, stream=None):
    """spstd_run_noalloc: advance the device tensors psiR, psiI (in place)
    by nsteps steps with V, writing the probe series into the device tensor
    probes ([(nsteps+1), nprobes, 2] float64); no device memory is
    allocated.  desc needs an explicit dt."""
    import torch
    for t in (V, psiR, psiI):
        assert t.is_contiguous() and t.device.type == "cuda"
    st = stream if stream is not None else torch.cuda.current_stream(psiR.device)
    with torch.cuda.device(psiR.device):
        rc = lib().spstd_run_noalloc(ctypes.byref(desc), ctypes.c_void_p(V.data_ptr()),
                                     ctypes.c_void_p(psiR.data_ptr()), ctypes.c_void_p(psiI.data_ptr()),
                                     int(nsteps),
                                     ctypes.c_void_p(probes.data_ptr() if probes is not None else 0),
                                     ctypes.c_void_p(st.cuda_stream))
    _check(rc)


def plan_from_workload(w, precision=FP64, method=SYMPLECTIC, dt=0.0, nsteps_max=None,
                       nyquist=NYQ_FULL, flags=0, coeffs=None, device="cuda", stream=None,
                       laplacian=LAP_SPECTRAL, neig=0):
    """Plan for a workloads.Workload (same arrays the oracle is given)."""
    c, d = coeffs if coeffs is not None else w.coeffs
    desc = make_desc(w.n, w.dx, c, d, dt=dt, cfl_fraction=w.cfl_fraction, hbar=w.hbar,
                     mass=w.mass, precision=precision, method=method, nyquist=nyquist,
                     probes=w.probes, flags=flags, bc=w.bc, laplacian=laplacian, neig=neig)
    return Plan(desc, w.V, w.psiR, w.psiI,
                nsteps_max=w.steps if nsteps_max is None else nsteps_max,
                device=device, stream=stream)


def make_batch_desc(n, coeffs, capacity, nprobes=1, nsteps_max=0, precision=FP64,
                    nyquist=NYQ_FULL, flags=0, wpb=0):
    c, d = coeffs
    desc = BatchDesc()
    desc.ndim = len(n)
    for a in range(3):
        desc.n[a] = int(n[a]) if a < len(n) else 1
    ca, da = _f64(c), _f64(d)
    desc.precision, desc.m = precision, len(ca)
    desc.c, desc.d = _dp(ca), _dp(da)
    desc.nyquist, desc.capacity, desc.nprobes = nyquist, int(capacity), int(nprobes)
    desc.nsteps_max, desc.flags = int(nsteps_max), flags
    desc.waves_per_block = int(wpb)
    desc._keep = [ca, da]
    return desc


def batch_workspace_size(desc):
    out = c_sz()
    _check(lib().spstd_batch_workspace_size(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


class Batch:
    """Slots of independent instances of one shape, stepped together."""

    def __init__(self, n, coeffs, capacity, nprobes=1, nsteps_max=0, precision=FP64,
                 nyquist=NYQ_FULL, flags=0, device="cuda", stream=None, wpb=0):
        import torch
        self.desc = make_batch_desc(n, coeffs, capacity, nprobes, nsteps_max, precision,
                                    nyquist, flags, wpb)
        self.n = tuple(n)
        self.npoints = int(np.prod(n))
        self.nprobes = int(nprobes)
        self.capacity = int(capacity)
        nbytes = batch_workspace_size(self.desc)
        dev = torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            rc = lib().spstd_batch_create(ctypes.byref(self.desc),
                                          ctypes.c_void_p(base + (-base) % 256), nbytes,
                                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(rc)
        self.h = h
        self._destroy = lib().spstd_batch_destroy

    def __del__(self):
        h, fn = getattr(self, "h", None), getattr(self, "_destroy", None)
        if h is not None and h.value and fn is not None:
            fn(h)
            self.h = None

    def load(self, slot, dx, V, psiR, psiI=None, probes=(), dt=0.0, cfl_fraction=0.5,
             hbar=1.0, mass=1.0):
        """Load an instance into a free slot; returns the time step used."""
        dxa = _f64(list(dx) + [1.0] * (3 - len(dx)))
        pidx = np.ascontiguousarray(np.asarray(probes, dtype=np.int64).ravel())
        out = c_d()
        _check(lib().spstd_batch_load(self.h, int(slot), _dp(dxa), float(hbar), float(mass),
                                      float(dt), float(cfl_fraction), _dp(_f64(V)),
                                      _dp(_f64(psiR)), _dp(_f64(psiI)),
                                      pidx.ctypes.data_as(P(c_i64)) if len(pidx) else None,
                                      ctypes.byref(out)), batch=self.h)
        return out.value

    def load_workload(self, slot, w, dt=0.0):
        return self.load(slot, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt,
                         cfl_fraction=w.cfl_fraction, hbar=w.hbar, mass=w.mass)

    def step(self, nsteps):
        _check(lib().spstd_batch_step(self.h, int(nsteps)), batch=self.h)

    def schedule(self):
        """("resident" or "passes", pass-kernel waves per block (0: built-in),
        measured us/step at creation of (resident, passes at 2 waves/block,
        passes at 4), zeros where not tuned)."""
        r, w = c_int(), c_int()
        us = np.zeros(3)
        _check(lib().spstd_batch_schedule(self.h, ctypes.byref(r), ctypes.byref(w), _dp(us)))
        return ("resident" if r.value else "passes"), w.value, tuple(float(u) for u in us)

    def slot_info(self, slot):
        a, s, dt = c_int(), c_i64(), c_d()
        _check(lib().spstd_batch_slot_info(self.h, int(slot), ctypes.byref(a), ctypes.byref(s),
                                           ctypes.byref(dt)), batch=self.h)
        return bool(a.value), s.value, dt.value

    def read(self, slot, state=True):
        """(series [(steps+1), P, 2], psiR, psiI, steps) of one slot."""
        _, steps, _ = self.slot_info(slot)
        ser = np.zeros((steps + 1, max(self.nprobes, 1), 2))
        pr = np.zeros(self.npoints) if state else None
        pi = np.zeros(self.npoints) if state else None
        st = c_i64()
        _check(lib().spstd_batch_read(self.h, int(slot), _dp(ser.ravel()) if self.nprobes else None,
                                      _dp(pr), _dp(pi), ctypes.byref(st)), batch=self.h)
        return (ser[:, : self.nprobes] if self.nprobes else None), pr, pi, st.value

    def release(self, slot):
        _check(lib().spstd_batch_release(self.h, int(slot)), batch=self.h)


def group_ok(n, precision=FP64, resident=False):
    """Whether a batch of shape n can join a group (2D, axes of 128, 256 or
    512 points, pass kernels)."""
    return len(n) == 2 and all(k in (128, 256, 512) for k in n) and not resident


class BatchGroup:
    """2D batches of different shapes stepped together: one launch per pass
    for all of them (or, as the tuner may choose, their own kernels in
    turn).  While the group exists its members work on the group's stream."""

    def __init__(self, members, flags=0, device="cuda", stream=None):
        import torch
        self.members = list(members)
        arr = (ctypes.c_void_p * len(self.members))(*[b.h.value for b in self.members])
        self._arr = arr
        nb = c_sz()
        _check(lib().spstd_batch_group_workspace_size(arr, len(self.members), ctypes.byref(nb)))
        dev = torch.device(device)
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            rc = lib().spstd_batch_group_create(arr, len(self.members), int(flags),
                                                ctypes.c_void_p(base + (-base) % 256), nb.value,
                                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(rc)
        self.h = h
        self._destroy = lib().spstd_batch_group_destroy

    def __del__(self):
        h, fn = getattr(self, "h", None), getattr(self, "_destroy", None)
        if h is not None and h.value and fn is not None:
            fn(h)
            self.h = None

    def close(self):
        """Release the group; the members return to their own streams."""
        self.__del__()

    def step(self, nsteps):
        _check(lib().spstd_batch_group_step(self.h, int(nsteps)), group=self.h)

    def schedule(self):
        """(candidate in use, measured us/step per candidate)."""
        ch, nc = c_int(), c_int()
        us = np.zeros(64)
        _check(lib().spstd_batch_group_schedule(self.h, ctypes.byref(ch), ctypes.byref(nc), _dp(us)))
        return ch.value, tuple(float(u) for u in us[: nc.value])

    def set_schedule(self, choice):
        _check(lib().spstd_batch_group_set_schedule(self.h, int(choice)), group=self.h)
