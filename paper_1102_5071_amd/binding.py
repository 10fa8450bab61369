"""ctypes binding of libcfet.so (the C ABI in include/cfet.h).

Argument marshalling only: every step of the propagation runs in the
library's HIP kernels.  PyTorch supplies device memory (complex128 tensors on
the GPU) and the current HIP stream.  If the shared library is missing the
binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint32, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfet.so")

SCHEMES = {"CF2:1": 0, "CF4:2": 1, "CF4:3": 2, "CF4:3Opt": 3, "CF6:4": 4, "CF6:5": 5,
           "CF6:5b": 6, "CF6:6": 7, "CF6:5Imp": 8, "CF6:5Opt": 9, "CF6:6Opt": 10,
           "CF8:11": 11}
DRIVE_KINDS = {"cos": 0, "sin2cos": 1, "pwc": 2, "sechcos": 3}
ERRORS = {0: "CFET_OK", 1: "CFET_EINVAL", 2: "CFET_ENOMEM", 3: "CFET_EDEVICE",
          4: "CFET_ENONFINITE", 5: "CFET_EUNSUPPORTED", 6: "CFET_ENOCONV"}
VALIDATE_HERMITIAN = 0x1
PATH_FLAGS = {None: 0, "auto": 0, "multi": 0x10, "single": 0x20, "coop": 0x40,
              "sell": 0x10 | 0x100, "sell_uniform": 0x10 | 0x200, "sell_split": 0x10 | 0x800}
LAYOUT_FLAGS = {None: 0, "auto": 0, "sell": 0x100, "sell_uniform": 0x200, "sell_split": 0x800}
NO_REORDER = 0x400
KEEP_CSR = 0x4000
PATH_NAMES = {0: "none", 1: "multi", 2: "single", 3: "coop"}
LAYOUT_NAMES = {0: "csr", 1: "sell", 2: "sell_uniform", 3: "sell_split"}
# the kernel(s) of one Lanczos SpMV on the multi-kernel path, per layout
SPMV_KERNEL_NAMES = {0: "k_lz_spmv", 1: "k_sell_lz_spmv", 2: "k_sell_lz_spmv",
                     3: "k_tile_pass1+k_tile_pass2"}
MAX_KRYLOV = 64


class CfetError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _CSR(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("row_ptr", c_void_p), ("col", c_void_p),
                ("val", c_void_p)]


class _Drive(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("A", c_double), ("omega", c_double), ("phi", c_double),
                ("Tp", c_double), ("tc", c_double), ("tau", c_double), ("npieces", c_int32),
                ("t_edges", c_void_p), ("u", c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz_stored", c_int64), ("exponentials", c_int64),
                ("matvecs", c_int64), ("min_m_eff", c_int32), ("breakdowns", c_int32),
                ("path", c_int32), ("status", c_int32), ("last_norm", c_double),
                ("timed_launches", c_int64), ("timed_ms", c_double),
                ("segment_us", c_double * 4), ("layout", c_int32), ("reordered", c_int32),
                ("matrix_bytes", c_int64)]


class _DtChoice(ctypes.Structure):
    _fields_ = [("dt", c_double), ("nsteps", c_int64), ("c", c_double), ("dt1", c_double),
                ("dt2", c_double), ("diff", c_double), ("err_est", c_double),
                ("err_check", c_double), ("check_window", c_double), ("order", c_int32),
                ("n1", c_int32), ("n2", c_int32), ("check_n1", c_int32), ("check_n2", c_int32),
                ("rounds", c_int32)]


class _Instance(ctypes.Structure):
    _fields_ = [("h0", c_int32), ("nterms", c_int32), ("hk", c_int32 * 7),
                ("fk", _Drive * 7)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("ninst", c_int32), ("ngroups", c_int32), ("total_dim", c_int64),
                ("matvecs", c_int64), ("exponentials", c_int64), ("breakdowns", c_int64),
                ("early_stops", c_int64), ("min_m_eff", c_int32), ("max_m_eff", c_int32),
                ("status", c_int32), ("unroll", c_int32), ("graph", c_int32),
                ("block_threads", c_int32), ("tune_us", c_double * 12)]


BATCH_NO_GRAPH = 0x1000
BATCH_NO_AUTOTUNE = 0x2000

_LIB = None


def load():
    """Load libcfet.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1102_5071_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.cfet_version.restype = c_int32
    lib.cfet_last_error.restype = ctypes.c_char_p
    lib.cfet_last_error.argtypes = [c_void_p]
    lib.cfet_create.argtypes = [POINTER(_CSR), c_int32, POINTER(_CSR), POINTER(_Drive), c_uint32,
                                POINTER(c_void_p)]
    lib.cfet_propagate.argtypes = [c_void_p, c_void_p, c_double, c_double, c_int64, c_int32,
                                   c_int32, c_void_p]
    lib.cfet_propagate_static.argtypes = [c_void_p, c_void_p, c_double, c_double, c_int64,
                                          c_int32, c_int32, c_void_p]
    lib.cfet_gradient.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_double, c_int64,
                                  c_int32, c_int32, c_void_p, c_int32, POINTER(c_double),
                                  c_void_p, c_void_p]
    lib.cfet_propagate_chebyshev.argtypes = [c_void_p, c_void_p, c_double, c_double, c_int64,
                                             c_int32, c_double, c_void_p]
    lib.cfet_select_dt.argtypes = [c_void_p, c_void_p, c_double, c_double, c_int32, c_int32,
                                   c_double, c_int32, c_int32, c_double, c_double, c_int32,
                                   c_int32, POINTER(_DtChoice), c_void_p]
    lib.cfet_apply.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p]
    lib.cfet_stats.argtypes = [c_void_p, POINTER(_Stats)]
    lib.cfet_destroy.argtypes = [c_void_p]
    lib.cfet_scheme_info.argtypes = [c_int32, POINTER(c_int32), POINTER(c_int32), c_void_p,
                                     c_void_p]
    lib.cfet_step_weights.argtypes = [c_void_p, c_double, c_double, c_int64, c_int32, c_void_p,
                                      c_void_p]
    lib.cfet_profile.argtypes = [c_void_p, c_int32, c_int32]
    lib.cfet_tridiag_expm.argtypes = [c_void_p, c_void_p, c_int32, c_double, c_void_p, c_void_p,
                                      c_void_p]
    lib.cfet_batch_create.argtypes = [c_int32, POINTER(_CSR), c_int32, POINTER(_Instance),
                                      c_uint32, POINTER(c_void_p)]
    lib.cfet_batch_propagate.argtypes = [c_void_p, c_void_p, c_double, c_double, c_int64,
                                         c_int32, c_int32, c_double, c_void_p]
    lib.cfet_batch_stats.argtypes = [c_void_p, POINTER(_BatchStats)]
    lib.cfet_batch_set_layout.argtypes = [c_void_p, c_int32, c_int32]
    lib.cfet_batch_instance_matvecs.argtypes = [c_void_p, c_void_p]
    lib.cfet_batch_destroy.argtypes = [c_void_p]
    lib.cfet_batch_last_error.restype = ctypes.c_char_p
    lib.cfet_batch_last_error.argtypes = [c_void_p]
    for name in ("cfet_create", "cfet_propagate", "cfet_propagate_static", "cfet_gradient", "cfet_apply", "cfet_stats",
                 "cfet_destroy", "cfet_scheme_info", "cfet_step_weights", "cfet_tridiag_expm",
                 "cfet_profile", "cfet_batch_create", "cfet_batch_propagate", "cfet_batch_stats",
                 "cfet_batch_set_layout", "cfet_batch_instance_matvecs", "cfet_batch_destroy"):
        getattr(lib, name).restype = c_int32
    _LIB = lib
    return lib


def _check(code: int, ctx=None):
    if code != 0:
        lib = load()
        msg = lib.cfet_last_error(ctx).decode(errors="replace")
        raise CfetError(code, msg)


def scheme_id(scheme) -> int:
    return SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)


def scheme_info(scheme):
    """(x, g) as the library computes them (host-side call, no device work)."""
    lib = load()
    s = c_int32()
    M = c_int32()
    _check(lib.cfet_scheme_info(scheme_id(scheme), ctypes.byref(s), ctypes.byref(M), None, None))
    x = np.zeros(M.value)
    g = np.zeros(s.value * M.value)
    _check(lib.cfet_scheme_info(scheme_id(scheme), ctypes.byref(s), ctypes.byref(M),
                                x.ctypes.data, g.ctypes.data))
    return x, g.reshape(s.value, M.value)


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _csr_struct(m, keep):
    rp = m.row_ptr
    col = m.col
    val = m.val
    if isinstance(rp, np.ndarray):
        rp = np.ascontiguousarray(rp, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.complex128)
    keep.extend([rp, col, val])
    return _CSR(int(m.n), int(rp[-1]) if isinstance(rp, np.ndarray) else int(m.nnz),
                _ptr(rp), _ptr(col), _ptr(val))


def _drive_struct(d, keep):
    kind = DRIVE_KINDS[d["kind"]]
    edges = u = None
    npieces = 0
    if d["kind"] == "pwc":
        edges = np.ascontiguousarray(d["t_edges"], dtype=np.float64)
        u = np.ascontiguousarray(d["u"], dtype=np.float64)
        npieces = len(u)
        keep.extend([edges, u])
    return _Drive(kind, float(d.get("A", 0.0)), float(d.get("omega", 0.0)),
                  float(d.get("phi", 0.0)), float(d.get("Tp", 0.0)), float(d.get("tc", 0.0)),
                  float(d.get("tau", 1.0)), npieces, _ptr(edges), _ptr(u))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


class Propagator:
    """Owns a cfet context for H(t) = H0 + sum_k f_k(t) Hk[k]."""

    def __init__(self, H0, Hk, drives, validate_hermitian: bool = False, path=None,
                 layout=None, reorder: bool = True, keep_csr: bool = False):
        lib = load()
        keep = []
        self.nterms = len(Hk)
        if len(drives) != self.nterms:
            raise ValueError("one drive per driven term")
        h0 = _csr_struct(H0, keep)
        hk = (_CSR * self.nterms)(*[_csr_struct(h, keep) for h in Hk])
        dv = (_Drive * self.nterms)(*[_drive_struct(d, keep) for d in drives])
        ctx = c_void_p()
        flags = ((VALIDATE_HERMITIAN if validate_hermitian else 0) | PATH_FLAGS[path]
                 | LAYOUT_FLAGS[layout] | (0 if reorder else NO_REORDER)
                 | (KEEP_CSR if keep_csr else 0))
        code = lib.cfet_create(ctypes.byref(h0), self.nterms, hk, dv, flags, ctypes.byref(ctx))
        if code != 0:
            raise CfetError(code, lib.cfet_last_error(None).decode(errors="replace"))
        self._ctx = ctx
        self.n = int(H0.n)
        self._pwc_pieces = next((len(d["u"]) for d in drives if d["kind"] == "pwc"), 0)

    # -- helpers ---------------------------------------------------------
    def _check_vec(self, v):
        import torch
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.complex128
                and v.is_contiguous() and v.numel() == self.n):
            raise ValueError("expected a contiguous complex128 CUDA tensor of length n")

    def propagate(self, psi, t0: float, dt: float, nsteps: int, scheme, m: int, stream=None):
        """psi (complex128 CUDA tensor) is updated in place."""
        self._check_vec(psi)
        _check(load().cfet_propagate(self._ctx, c_void_p(psi.data_ptr()), float(t0), float(dt),
                                     int(nsteps), scheme_id(scheme), int(m),
                                     _stream_handle(stream)), self._ctx)
        return psi

    def propagate_static(self, psi, t0: float, dt: float, nsteps: int, scheme, m: int,
                         stream=None):
        """cfet_propagate_static: the multi-kernel propagation with the library's
        fixed device scratch (no allocation during the call)."""
        self._check_vec(psi)
        _check(load().cfet_propagate_static(self._ctx, c_void_p(psi.data_ptr()), float(t0),
                                            float(dt), int(nsteps), scheme_id(scheme), int(m),
                                            _stream_handle(stream)), self._ctx)
        return psi

    def propagate_chebyshev(self, psi, t0: float, dt: float, nsteps: int, scheme, tol: float,
                            stream=None):
        """cfet_propagate_chebyshev: the CFET steps with Chebyshev exponentials
        (series truncated at tol per exponential); psi updated in place."""
        self._check_vec(psi)
        _check(load().cfet_propagate_chebyshev(self._ctx, c_void_p(psi.data_ptr()), float(t0),
                                               float(dt), int(nsteps), scheme_id(scheme),
                                               float(tol), _stream_handle(stream)), self._ctx)
        return psi

    def apply(self, x, a: float, b, y=None, stream=None):
        import torch
        self._check_vec(x)
        if y is None:
            y = torch.empty_like(x)
        self._check_vec(y)
        bb = np.ascontiguousarray(np.atleast_1d(np.asarray(b, dtype=np.float64)))
        if bb.size != self.nterms:
            raise ValueError("need one weight per driven term")
        _check(load().cfet_apply(self._ctx, c_void_p(x.data_ptr()), c_void_p(y.data_ptr()),
                                 float(a), bb.ctypes.data, _stream_handle(stream)), self._ctx)
        return y

    def step_weights(self, t0: float, dt: float, nsteps: int, scheme):
        s = scheme_info(scheme)[1].shape[0]
        a = np.zeros(s)
        b = np.zeros(max(nsteps, 1) * s * self.nterms)
        _check(load().cfet_step_weights(self._ctx, float(t0), float(dt), int(nsteps),
                                        scheme_id(scheme), a.ctypes.data, b.ctypes.data),
               self._ctx)
        return a, b[:nsteps * s * self.nterms].reshape(nsteps, s, self.nterms)

    def stats(self) -> dict:
        st = _Stats()
        _check(load().cfet_stats(self._ctx, ctypes.byref(st)), self._ctx)
        out = {f[0]: getattr(st, f[0]) for f in _Stats._fields_}
        out["segment_us"] = list(out["segment_us"])
        return out

    def uses_sell(self) -> bool:
        """True when the multi-kernel path runs on a SELL-64 layout."""
        return self.stats()["layout"] in (1, 2)

    def profile(self, enable: bool, max_launches: int = 65536, segments: bool = True):
        """Event timing of the dominant kernel; segments: also the persistent
        kernels' segment timers (they lengthen those kernels slightly)."""
        mode = 0 if not enable else (1 if segments else 2)
        _check(load().cfet_profile(self._ctx, mode, int(max_launches)), self._ctx)

    def gradient(self, psi0, target, t0: float, dt: float, nsteps: int, scheme, m: int,
                 u=None, stream=None):
        """(F, dF/du): fidelity |<target|psi_N>|^2 of the CFET run from psi0 and its
        gradient with respect to the pieces of the piecewise-constant drive
        (u: optional amplitudes replacing those of the drive for this call)."""
        self._check_vec(psi0)
        self._check_vec(target)
        if u is None:
            K = self.pwc_pieces()
            uptr = None
        else:
            u = np.ascontiguousarray(u, dtype=np.float64)
            K = len(u)
            uptr = u.ctypes.data
        F = c_double()
        g = np.zeros(K)
        _check(load().cfet_gradient(self._ctx, c_void_p(psi0.data_ptr()),
                                    c_void_p(target.data_ptr()), float(t0), float(dt),
                                    int(nsteps), scheme_id(scheme), int(m), uptr, int(K),
                                    ctypes.byref(F), g.ctypes.data, _stream_handle(stream)),
               self._ctx)
        return F.value, g

    def select_dt(self, psi0, t0: float, window: float, n1: int, scheme, m: int,
                  T_total: float, eps: float, ratio: float = 2.5, checkpoints: int = 1,
                  verify: bool = True, refine: int = 0, stream=None) -> dict:
        """cfet_select_dt: the step for an accuracy goal eps over T_total from
        two probe runs of [t0, t0 + window] (n1 steps and the next count in
        the given ratio), optionally checked by two more runs and refined
        from them up to `refine` times."""
        self._check_vec(psi0)
        r = _DtChoice()
        _check(load().cfet_select_dt(self._ctx, c_void_p(psi0.data_ptr()), float(t0),
                                     float(window), int(n1), int(checkpoints), float(ratio),
                                     scheme_id(scheme), int(m), float(T_total), float(eps),
                                     1 if verify else 0, int(refine), ctypes.byref(r),
                                     _stream_handle(stream)), self._ctx)
        out = {f[0]: getattr(r, f[0]) for f in _DtChoice._fields_}
        if not verify:
            out["err_check"] = None
        return out

    def pwc_pieces(self) -> int:
        return self._pwc_pieces

    def close(self):
        if getattr(self, "_ctx", None):
            load().cfet_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BatchPropagator:
    """Owns a cfet batch: independent instances sharing scheme and time grid.

    ops: list of CSR operators; instances: list of dicts with keys h0 (operator
    index), hk (list of operator indices) and drives (one drive dict per hk
    entry).  States are passed as one complex128 CUDA tensor holding the
    instances one after another (see ``offsets``)."""

    def __init__(self, ops, instances, validate_hermitian: bool = False, graph: bool = True,
                 autotune: bool = True):
        lib = load()
        keep = []
        cops = (_CSR * len(ops))(*[_csr_struct(m, keep) for m in ops])
        insts = (_Instance * len(instances))()
        for t, inst in enumerate(instances):
            hk = list(inst["hk"])
            if len(hk) != len(inst["drives"]) or len(hk) > 7:
                raise ValueError("one drive per driven term, at most 7 terms")
            insts[t].h0 = int(inst["h0"])
            insts[t].nterms = len(hk)
            for k, (h, d) in enumerate(zip(hk, inst["drives"])):
                insts[t].hk[k] = int(h)
                insts[t].fk[k] = _drive_struct(d, keep)
        flags = ((VALIDATE_HERMITIAN if validate_hermitian else 0)
                 | (0 if graph else BATCH_NO_GRAPH) | (0 if autotune else BATCH_NO_AUTOTUNE))
        handle = c_void_p()
        code = lib.cfet_batch_create(len(ops), cops, len(instances), insts, flags,
                                     ctypes.byref(handle))
        if code != 0:
            raise CfetError(code, lib.cfet_batch_last_error(None).decode(errors="replace"))
        self._b = handle
        self.dims = [int(ops[i["h0"]].n) for i in instances]
        self.offsets = np.concatenate([[0], np.cumsum(self.dims)]).astype(np.int64)
        self.total = int(self.offsets[-1])

    def _check(self, code):
        if code != 0:
            raise CfetError(code, load().cfet_batch_last_error(self._b).decode(errors="replace"))

    def propagate(self, psi, t0: float, dt: float, nsteps: int, scheme, m: int,
                  tol: float = 0.0, stream=None):
        """psi: complex128 CUDA tensor of length sum(dims), updated in place."""
        import torch
        if not (isinstance(psi, torch.Tensor) and psi.is_cuda and psi.dtype == torch.complex128
                and psi.is_contiguous() and psi.numel() == self.total):
            raise ValueError("expected a contiguous complex128 CUDA tensor of length sum(dims)")
        self._check(load().cfet_batch_propagate(self._b, c_void_p(psi.data_ptr()), float(t0),
                                                float(dt), int(nsteps), scheme_id(scheme),
                                                int(m), float(tol), _stream_handle(stream)))
        return psi

    def stats(self) -> dict:
        st = _BatchStats()
        self._check(load().cfet_batch_stats(self._b, ctypes.byref(st)))
        out = {f[0]: getattr(st, f[0]) for f in _BatchStats._fields_}
        out["tune_us"] = list(out["tune_us"])
        return out

    def set_layout(self, block_threads: int, rows_per_lane: int):
        """Fix the row kernels' launch layout (cfet_batch_set_layout)."""
        self._check(load().cfet_batch_set_layout(self._b, int(block_threads), int(rows_per_lane)))

    def instance_matvecs(self):
        out = np.zeros(len(self.dims), dtype=np.int64)
        self._check(load().cfet_batch_instance_matvecs(self._b, out.ctypes.data))
        return out

    def split(self, psi):
        """Views of the instances' states in a packed tensor."""
        return [psi[self.offsets[t]:self.offsets[t + 1]] for t in range(len(self.dims))]

    def close(self):
        if getattr(self, "_b", None):
            load().cfet_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class _FidelityFn:
    """torch.autograd.Function for F(u) = |<target|psi_N(u)>|^2 (built lazily so
    that importing the binding does not import torch)."""
    _cls = None

    @classmethod
    def get(cls):
        if cls._cls is None:
            import torch

            class FidelityFunction(torch.autograd.Function):
                @staticmethod
                def forward(ctx, u, prop, psi0, target, t0, dt, nsteps, scheme, m):
                    F, g = prop.gradient(psi0, target, t0, dt, nsteps, scheme, m,
                                         u=u.detach().cpu().numpy())
                    ctx.save_for_backward(torch.from_numpy(g).to(u.device, u.dtype))
                    return u.new_tensor(F)

                @staticmethod
                def backward(ctx, gF):
                    (g,) = ctx.saved_tensors
                    return (gF * g,) + (None,) * 8

            cls._cls = FidelityFunction
        return cls._cls


def fidelity(u, prop, psi0, target, t0: float, dt: float, nsteps: int, scheme, m: int):
    """Differentiable F(u) = |<target|psi_N>|^2 for the piecewise-constant drive
    amplitudes u (a float64 torch tensor, CPU or CUDA): the forward call runs
    the CFET propagation and its adjoint on the GPU (cfet_gradient), backward
    returns dF/du."""
    return _FidelityFn.get().apply(u, prop, psi0, target, t0, dt, nsteps, scheme, m)


def tridiag_expm(alpha, beta, dt: float, stream=None):
    """c = exp(-i dt T) e_1 by the library's device kernel.  alpha, beta:
    float64 CUDA tensors (len k, k-1).  Returns (c, status)."""
    import torch
    k = alpha.numel()
    c = torch.empty(k, dtype=torch.complex128, device=alpha.device)
    status = torch.zeros(1, dtype=torch.int32, device=alpha.device)
    bptr = c_void_p(beta.data_ptr()) if beta is not None and beta.numel() > 0 else None
    _check(load().cfet_tridiag_expm(c_void_p(alpha.data_ptr()), bptr, int(k), float(dt),
                                    c_void_p(c.data_ptr()), c_void_p(status.data_ptr()),
                                    _stream_handle(stream)))
    return c, int(status.item())
