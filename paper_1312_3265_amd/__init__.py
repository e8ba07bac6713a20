"""Python binding of liblq.so, the MI355X library for CG on the normal equations
of the Wilson and 2-flavour staggered Wilson Dirac matrices (include/lq.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels.  torch supplies device memory and the stream; the library never
allocates device memory itself.  Importing this package does not need a GPU;
calling into the library does, and raises if the built library is missing.

Fields cross the boundary in the canonical layout (see ``synth``): torch tensors
of shape (L4, L3, L2, L1, 4, 3) (Wilson) or (L4, L3, L2, L1, 3) (staggered
Wilson), complex128 (complex64 for the FP32/Q16 ``apply``).
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblq.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lq.h")

WILSON = 0
STAGGERED_WILSON = 1
OP_M, OP_MDAG, OP_MDAGM = 0, 1, 2
G55_CORNERS, G55_ONTHEFLY = 0, 1
F64, F32, Q16 = 0, 1, 2
FEAT_CORNERS, FEAT_F32, FEAT_Q16, FEAT_EO = 1, 2, 4, 8
OK, NOT_CONVERGED, STAGNATION = 0, 1, 2
FLAG_BREAKDOWN, FLAG_MAXITER, FLAG_STAGNATION = 1, 2, 4
WHERE_HOST, WHERE_DEVICE = 0, 1
ERR_ARG, ERR_WORKSPACE, ERR_DEVICE, ERR_BREAKDOWN, ERR_STATE = -1, -2, -3, -4, -5
SLOT_EMPTY, SLOT_RUNNING, SLOT_DONE, SLOT_FAILED = 0, 1, 2, 3


class LQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lq error {code}: {msg}")
        self.code = code


class Dirac(ctypes.Structure):
    _fields_ = [("formulation", ctypes.c_int32), ("g55_mode", ctypes.c_int32),
                ("mass", ctypes.c_double), ("r", ctypes.c_double)]


class Overlap(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("mass", ctypes.c_double), ("r", ctypes.c_double),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("degree", ctypes.c_int32),
                ("g55_mode", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("links", ctypes.c_int32),
                ("reliable_interval", ctypes.c_int32), ("poll_interval", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("max_restarts", ctypes.c_int32),
                ("reliable_delta", ctypes.c_double), ("evenodd", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("applications", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("iterated_residual", ctypes.c_double), ("true_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def header_symbols():
    """Function names declared in include/lq.h."""
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(lq_\w+)\s*\(", txt, re.M)))


def lib():
    """The loaded liblq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1312_3265_amd.build` (there is no fallback)")
    # torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
    # first makes the library bind to that same runtime, so device pointers and
    # streams from torch are valid in the library; loading the library first
    # would put a second runtime in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    c = ctypes
    P, I32, I64, D, SZ = c.c_void_p, c.c_int32, c.c_int64, c.c_double, c.c_size_t
    sig = {
        "lq_last_error": ([], c.c_char_p),
        "lq_version": ([], c.c_char_p),
        "lq_lattice_create": ([P, P, P], I32),
        "lq_lattice_destroy": ([P], None),
        "lq_lattice_volume": ([P], I64),
        "lq_gauge_bytes": ([P, c.c_uint32], SZ),
        "lq_gauge_create": ([P, P, I32, c.c_uint32, P, SZ, P, P], I32),
        "lq_gauge_destroy": ([P], None),
        "lq_gauge_su3_deviation": ([P, P], I32),
        "lq_gauge_plaquette": ([P, P, P], I32),
        "lq_apply_workspace_bytes": ([P, I32, I32, I32], SZ),
        "lq_apply": ([P, P, I32, I32, I32, P, P, P, SZ, P], I32),
        "lq_apply_noalloc_max_bytes": ([], SZ),
        "lq_apply_noalloc": ([P, P, I32, I32, I32, P, P, P], I32),
        "lq_schur_workspace_bytes": ([P, I32], SZ),
        "lq_schur_apply": ([P, P, I32, I32, I32, P, P, P, SZ, P], I32),
        "lq_pion_workspace_bytes": ([P], SZ),
        "lq_pion_correlator": ([P, I32, P, P, P, P, SZ, P], I32),
        "lq_spectrum_workspace_bytes": ([P, I32, I32, I32], SZ),
        "lq_spectrum": ([P, P, D, I32, I32, D, P, P, SZ, P, P, P, P, P], I32),
        "lq_time_dslash": ([P, P, I32, I32, I32, I32, I32, I32, I32, P, SZ, P, P], I32),
        "lq_time_dslash_workspace_bytes": ([P, I32, I32, I32, I32], SZ),
        "lq_tuned_launch": ([P, P, I32, I32, I32, P, P], I32),
        "lq_solve_workspace_bytes": ([P, I32, I32, P, I32], SZ),
        "lq_cg_solve": ([P, P, P, P, D, I32, P, P, SZ, P, P], I32),
        "lq_cg_solve_batch": ([P, I32, I32, D, I32, P, P, P, P, I32, P, P, SZ, P, P], I32),
        "lq_batch_create": ([P, I32, I32, D, I32, P, P, SZ, P], I32),
        "lq_batch_load": ([P, I32, P, D, D, I32, P], I32),
        "lq_batch_step": ([P, I32, P, P], I32),
        "lq_batch_fetch": ([P, I32, P, P, P], I32),
        "lq_batch_cancel": ([P, I32, P], I32),
        "lq_batch_destroy": ([P], None),
        "lq_batch_peek": ([P, I32, P, P], I32),
        "lq_lanczos_workspace_bytes": ([P, I32, I32, I32], SZ),
        "lq_overlap_workspace_bytes": ([P, I32], SZ),
        "lq_overlap_apply": ([P, P, P, P, P, SZ, P], I32),
        "lq_condition_number": ([P, P, I32, P, P, SZ, P, P, P, P, P, P, P], I32),
        "lq_critical_mass": ([P, I32, I32, D, D, D, I32, I32, I32, P, P, SZ, P, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc, allow_positive=False):
    if rc < 0 or (rc > 0 and not allow_positive):
        raise LQError(rc, lib().lq_last_error().decode())
    return rc


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _device_tensor(x, dtype, stream=None):
    """x as a contiguous device tensor of dtype.  A conversion or copy runs on
    torch's current stream; when the library will read the tensor on another
    `stream`, that stream first waits for the current one."""
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x.to(device="cuda", dtype=dtype)
    else:
        t = torch.from_numpy(x).to(device="cuda", dtype=dtype)
    t = t.contiguous()
    if stream is not None:
        cur = torch.cuda.current_stream()
        if stream != cur:
            stream.wait_stream(cur)
    return t


class Lattice:
    """A 4D lattice (dims = (L1, L2, L3, L4)) with fermion boundary signs."""

    def __init__(self, dims, bc=(1, 1, 1, 1)):
        self.dims = tuple(int(d) for d in dims)
        self.bc = tuple(int(b) for b in bc)
        h = ctypes.c_void_p()
        d = (ctypes.c_int32 * 4)(*self.dims)
        b = (ctypes.c_int32 * 4)(*self.bc)
        _check(lib().lq_lattice_create(d, b, ctypes.byref(h)))
        self._h = h
        self.volume = int(lib().lq_lattice_volume(h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lq_lattice_destroy(self._h)
            self._h = None


class Gauge:
    """Gauge field resident in HBM (library layout, FP64 plus requested copies).

    U: canonical complex128 field, a numpy array (uploaded by the library from
    host memory) or a torch tensor (passed as a device pointer)."""

    def __init__(self, lattice, U, features=FEAT_CORNERS | FEAT_F32 | FEAT_Q16, stream=None):
        import numpy as np
        torch = _torch()
        self.lattice = lattice
        self.features = features
        nbytes = int(lib().lq_gauge_bytes(lattice._h, features))
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        if isinstance(U, torch.Tensor):
            src, where = _device_tensor(U, torch.complex128, stream), WHERE_DEVICE
            ptr = _ptr(src)
        else:
            src, where = np.ascontiguousarray(U, dtype=np.complex128), WHERE_HOST
            ptr = ctypes.c_void_p(src.ctypes.data)
        if stream is not None:
            # the buffer was allocated on the current stream
            stream.wait_stream(torch.cuda.current_stream())
        h = ctypes.c_void_p()
        _check(lib().lq_gauge_create(lattice._h, ptr, where, features, _ptr(self.buf), nbytes,
                                     _stream(stream), ctypes.byref(h)))
        _stream_sync(stream)
        self._h = h
        self.nbytes = nbytes

    def plaquette(self, stream=None):
        out = ctypes.c_double()
        _check(lib().lq_gauge_plaquette(self._h, ctypes.byref(out), _stream(stream)))
        return out.value

    def su3_deviation(self):
        """max |row2 - conj(row0 x row1)| over the links (0 up to rounding for SU(3))."""
        out = ctypes.c_double()
        _check(lib().lq_gauge_su3_deviation(self._h, ctypes.byref(out)))
        return out.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lq_gauge_destroy(self._h)
            self._h = None


def _stream_sync(stream=None):
    torch = _torch()
    (stream or torch.cuda.current_stream()).synchronize()


def _field_shape(dims, formulation):
    L1, L2, L3, L4 = dims
    return (L4, L3, L2, L1, 4, 3) if formulation == WILSON else (L4, L3, L2, L1, 3)


def apply(gauge, formulation, mass, psi, op=OP_M, r=1.0, g55=G55_CORNERS, precision=F64,
          links=0, stream=None):
    """op(psi) with op in {M, M^dag, M^dag M}; returns a new device tensor."""
    torch = _torch()
    dt = torch.complex128 if precision == F64 else torch.complex64
    x = _device_tensor(psi, dt, stream)
    out = torch.empty_like(x)
    nb = int(lib().lq_apply_workspace_bytes(gauge._h, formulation, g55, precision))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = Dirac(formulation, g55, mass, r)
    _check(lib().lq_apply(gauge._h, ctypes.byref(d), op, precision, links, _ptr(x), _ptr(out),
                          _ptr(ws), nb, _stream(stream)))
    _stream_sync(stream)
    return out


def apply_noalloc(gauge, formulation, mass, psi, out, op=OP_M, r=1.0, g55=G55_CORNERS,
                  precision=F64, links=0, stream=None):
    """op(psi) into the caller's `out` (a device tensor like psi) through the
    allocation-free entry point (the library's fixed scratch; no device
    allocation in the call).  Asynchronous on `stream`."""
    torch = _torch()
    d = Dirac(formulation, g55, mass, r)
    _check(lib().lq_apply_noalloc(gauge._h, ctypes.byref(d), op, precision, links, _ptr(psi),
                                  _ptr(out), _stream(stream)))
    return out


def schur_apply(gauge, mass, psi, dagger=False, precision=F64, links=0, stream=None):
    """M^ psi_e (M^dag with dagger): the even-odd Schur complement of the
    Wilson matrix (r = 1) on the even sites of the full-lattice field psi;
    the odd sites of the result are zero.  Needs a gauge built with FEAT_EO."""
    torch = _torch()
    dt = torch.complex128 if precision == F64 else torch.complex64
    x = _device_tensor(psi, dt, stream)
    out = torch.empty_like(x)
    nb = int(lib().lq_schur_workspace_bytes(gauge._h, precision))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = Dirac(WILSON, G55_CORNERS, mass, 1.0)
    _check(lib().lq_schur_apply(gauge._h, ctypes.byref(d), int(dagger), precision, links, _ptr(x),
                                _ptr(out), _ptr(ws), nb, _stream(stream)))
    _stream_sync(stream)
    return out


def overlap_apply(gauge, psi, rho, mass, lo, hi, degree, r=1.0, g55=G55_CORNERS, stream=None):
    """D_ov(m) psi for the staggered overlap operator with kernel A = D_SW - rho
    (include/lq.h: lq_overlap_apply), (A^dag A)^{-1/2} by the Chebyshev
    interpolant of the given degree on [lo, hi]; returns a new device tensor."""
    torch = _torch()
    x = _device_tensor(psi, torch.complex128, stream)
    out = torch.empty_like(x)
    nb = int(lib().lq_overlap_workspace_bytes(gauge._h, g55))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    ov = Overlap(rho, mass, r, lo, hi, int(degree), g55)
    _check(lib().lq_overlap_apply(gauge._h, ctypes.byref(ov), _ptr(x), _ptr(out), _ptr(ws), nb,
                                  _stream(stream)))
    _stream_sync(stream)
    return out


def pion_correlator(lattice, props, stream=None):
    """(C, m_eff): the Wilson pion correlator of point-source propagators
    props (leading source axis, canonical Wilson fields) and its periodic
    effective mass, numpy arrays of length L4."""
    import numpy as np
    torch = _torch()
    p = _device_tensor(props, torch.complex128, stream)
    L4 = lattice.dims[3]
    corr = np.zeros(L4)
    meff = np.zeros(L4)
    nb = int(lib().lq_pion_workspace_bytes(lattice._h))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    _check(lib().lq_pion_correlator(lattice._h, p.shape[0], _ptr(p),
                                    corr.ctypes.data_as(ctypes.c_void_p),
                                    meff.ctypes.data_as(ctypes.c_void_p), _ptr(ws), nb,
                                    _stream(stream)))
    return corr, meff


def spectrum(gauge, formulation, mass, sigma, v0, steps=40, tol=1e-10, restarts=0, r=1.0,
             g55=G55_CORNERS, stream=None):
    """(eigenvalues, Ritz residual estimates) of M at `mass` nearest the real
    shift sigma by shift-invert Krylov-Schur with a basis of `steps` vectors
    and up to `restarts` restarts (numpy arrays, nearest first)."""
    import numpy as np
    torch = _torch()
    v = _device_tensor(v0, torch.complex128, stream)
    nb = int(lib().lq_spectrum_workspace_bytes(gauge._h, formulation, g55, steps))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = Dirac(formulation, g55, mass, r)
    re, im, res = np.zeros(steps), np.zeros(steps), np.zeros(steps)
    nev = ctypes.c_int32()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().lq_spectrum(gauge._h, ctypes.byref(d), float(sigma), steps, int(restarts),
                             float(tol), _ptr(v),
                             _ptr(ws), nb, ctypes.byref(nev), p(re), p(im), p(res),
                             _stream(stream)))
    k = nev.value
    return re[:k] + 1j * im[:k], res[:k]


def time_dslash(gauge, formulation, mass, dagger=False, r=1.0, g55=G55_CORNERS, precision=F64,
                links=0, nrhs=1, reps=50, rhs_per_thread=1, window=0, stream=None, kernel=None):
    """Average milliseconds per stencil launch (HIP events on the launch stream).
    kernel: 0 = t = M p + ||t||^2, 1 = plain M^dag, 2 = M^dag t with the CG
    update of r; 3, 4 = the even-odd pairs t = M^ p + ||t||^2 and M^dag t with
    the CG update (per pair); default 1 if dagger else 0."""
    torch = _torch()
    nb = int(lib().lq_time_dslash_workspace_bytes(gauge._h, formulation, g55, precision, nrhs))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = Dirac(formulation, g55, mass, r)
    ms = ctypes.c_double()
    sel = kernel if kernel is not None else (1 if dagger else 0)
    _check(lib().lq_time_dslash(gauge._h, ctypes.byref(d), sel, precision, links, nrhs,
                                rhs_per_thread, window, reps, _ptr(ws), nb, ctypes.byref(ms),
                                _stream(stream)))
    return ms.value


def tuned_launch(gauge, formulation, precision, links, nrhs, g55=G55_CORNERS):
    """(rhs_per_thread, window) the solvers' autotuner chose for batches of
    nrhs systems of this shape, or None if none has been tuned yet."""
    d = Dirac(formulation, g55, 0.0, 1.0)
    k, w = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().lq_tuned_launch(gauge._h, ctypes.byref(d), precision, links, nrhs,
                               ctypes.byref(k), ctypes.byref(w))
    if rc == ERR_STATE:
        return None
    _check(rc)
    return k.value, w.value


def solve_opts(precision=F64, links=0, reliable_interval=0, poll_interval=0, use_graph=0,
               max_restarts=0, reliable_delta=0.0, evenodd=0):
    return SolveOpts(precision, links, reliable_interval, poll_interval, use_graph, max_restarts,
                     reliable_delta, int(evenodd))


def solve_workspace_bytes(gauge, formulation, opts, nrhs, g55=G55_CORNERS):
    """Device bytes the solver needs for nrhs systems with these options."""
    return int(lib().lq_solve_workspace_bytes(gauge._h, formulation, g55, ctypes.byref(opts),
                                              nrhs))


def cg_solve(gauge, formulation, mass, chi, tol, maxiter=100000, r=1.0, g55=G55_CORNERS,
             opts=None, stream=None):
    """Solve (D+m)^dag (D+m) x = (D+m)^dag chi; returns (x, info dict)."""
    torch = _torch()
    c = _device_tensor(chi, torch.complex128, stream)
    x = torch.empty_like(c)
    opts = opts or solve_opts()
    nb = int(lib().lq_solve_workspace_bytes(gauge._h, formulation, g55, ctypes.byref(opts), 1))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = Dirac(formulation, g55, mass, r)
    info = SolveInfo()
    rc = lib().lq_cg_solve(gauge._h, ctypes.byref(d), _ptr(c), _ptr(x), tol, maxiter,
                           ctypes.byref(opts), _ptr(ws), nb, ctypes.byref(info), _stream(stream))
    if rc < 0 and rc != ERR_BREAKDOWN:
        _check(rc)
    return x, info.as_dict()


def cg_solve_batch(gauge, formulation, masses, chis, tols, maxiter=100000, r=1.0,
                   g55=G55_CORNERS, opts=None, stream=None, workspace=None):
    """Batched multi-RHS CG; chis has a leading RHS axis.  Returns (x, [info])."""
    torch = _torch()
    c = _device_tensor(chis, torch.complex128, stream)
    n = c.shape[0]
    x = torch.empty_like(c)
    opts = opts or solve_opts()
    nb = int(lib().lq_solve_workspace_bytes(gauge._h, formulation, g55, ctypes.byref(opts), n))
    ws = workspace if workspace is not None and workspace.numel() >= nb else \
        torch.empty(nb, dtype=torch.uint8, device="cuda")
    m = (ctypes.c_double * n)(*[float(v) for v in masses])
    t = (ctypes.c_double * n)(*[float(v) for v in tols])
    infos = (SolveInfo * n)()
    rc = lib().lq_cg_solve_batch(gauge._h, formulation, g55, r, n, m, _ptr(c), _ptr(x), t,
                                 maxiter, ctypes.byref(opts), _ptr(ws), nb, infos,
                                 _stream(stream))
    if rc < 0 and rc != ERR_BREAKDOWN:
        _check(rc)
    return x, [i.as_dict() for i in infos]


def condition_number(gauge, formulation, mass, v0, steps=200, r=1.0, g55=G55_CORNERS,
                     stream=None):
    """Lanczos (full reorthogonalisation) estimate of kappa of (D+m)^dag (D+m).

    Returns dict(lmin, lmax, kappa, alpha, beta, steps)."""
    torch = _torch()
    v = _device_tensor(v0, torch.complex128, stream)
    nb = int(lib().lq_lanczos_workspace_bytes(gauge._h, formulation, g55, steps))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = Dirac(formulation, g55, mass, r)
    lmin, lmax, kappa = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    a = (ctypes.c_double * steps)()
    b = (ctypes.c_double * max(steps - 1, 1))()
    nd = ctypes.c_int32()
    _check(lib().lq_condition_number(gauge._h, ctypes.byref(d), steps, _ptr(v), _ptr(ws), nb,
                                     ctypes.byref(lmin), ctypes.byref(lmax), ctypes.byref(kappa),
                                     a, b, ctypes.byref(nd), _stream(stream)))
    n = nd.value
    return dict(lmin=lmin.value, lmax=lmax.value, kappa=kappa.value, alpha=list(a[:n]),
                beta=list(b[:max(n - 1, 0)]), steps=n)


def critical_mass(gauge, formulation, v0, lo, hi, steps=200, ngrid=7, ngolden=8, r=1.0,
                  g55=G55_CORNERS, stream=None):
    """m_c = argmin_m of the Lanczos lowest Ritz value (scan + golden section)."""
    torch = _torch()
    v = _device_tensor(v0, torch.complex128, stream)
    nb = int(lib().lq_lanczos_workspace_bytes(gauge._h, formulation, g55, steps))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    mc, th = ctypes.c_double(), ctypes.c_double()
    _check(lib().lq_critical_mass(gauge._h, formulation, g55, r, lo, hi, ngrid, ngolden, steps,
                                  _ptr(v), _ptr(ws), nb, ctypes.byref(mc), ctypes.byref(th),
                                  _stream(stream)))
    return mc.value, th.value


class Batch:
    """Resident multi-slot solver for continuous batching (serving)."""

    def __init__(self, gauge, formulation, nslots, r=1.0, g55=G55_CORNERS, opts=None):
        torch = _torch()
        self.gauge = gauge
        self.formulation = formulation
        self.nslots = nslots
        self.opts = opts or solve_opts()
        nb = int(lib().lq_solve_workspace_bytes(gauge._h, formulation, g55,
                                                ctypes.byref(self.opts), nslots))
        self.ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        self.nbytes = nb
        h = ctypes.c_void_p()
        _check(lib().lq_batch_create(gauge._h, formulation, g55, r, nslots,
                                     ctypes.byref(self.opts), _ptr(self.ws), nb, ctypes.byref(h)))
        self._h = h
        self._states = (ctypes.c_int32 * nslots)()
        self._keep = {}

    def load(self, slot, chi, mass, tol, maxiter=100000, stream=None):
        torch = _torch()
        c = _device_tensor(chi, torch.complex128, stream)
        self._keep[slot] = c
        _check(lib().lq_batch_load(self._h, slot, _ptr(c), mass, tol, maxiter, _stream(stream)))

    def step(self, iterations, stream=None):
        _check(lib().lq_batch_step(self._h, iterations, self._states, _stream(stream)))
        return list(self._states)

    def fetch(self, slot, stream=None):
        torch = _torch()
        shape = _field_shape(self.gauge.lattice.dims, self.formulation)
        x = torch.empty(shape, dtype=torch.complex128, device="cuda")
        info = SolveInfo()
        _check(lib().lq_batch_fetch(self._h, slot, _ptr(x), ctypes.byref(info), _stream(stream)))
        self._keep.pop(slot, None)
        return x, info.as_dict()

    def cancel(self, slot, stream=None):
        """Discard a loaded slot (running or finished) and free it."""
        _check(lib().lq_batch_cancel(self._h, slot, _stream(stream)))
        self._keep.pop(slot, None)

    def peek(self, slot):
        """Slot progress as of the latest step (no device work)."""
        info = SolveInfo()
        sc = ctypes.c_double()
        _check(lib().lq_batch_peek(self._h, slot, ctypes.byref(info), ctypes.byref(sc)))
        d = info.as_dict()
        d.pop("seconds")
        d["scale"] = sc.value
        return d

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lq_batch_destroy(self._h)
            self._h = None
