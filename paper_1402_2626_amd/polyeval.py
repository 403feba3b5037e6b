"""Python binding of the polyeval C ABI (``include/polyeval.h``).

Argument marshalling only: every step of the evaluation runs in the HIP
library.  PyTorch provides device memory and streams.  If the library is not
built, importing this module raises ``ImportError``; there is no fallback.

Tensors are float64 and limb-planar: ``x[P, 2, L, n]``, ``F[P, 2, L, N]``,
``J[P, 2, L, N, n]`` with L = 1 (double), 2 (double double), 4 (quad double).
A real system (level ``PE_REAL | L``) has one component instead of two:
``x[P, 1, L, n]`` and so on.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolyeval.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1402_2626_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

_c_int = ctypes.c_int32
_p = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)

PE_OK, PE_EINVAL, PE_ENOMEM, PE_EUNSUPPORTED, PE_EDEVICE, PE_ESINGULAR, PE_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
PE_REAL = 8  # level flag of real arithmetic

# every entry point of the C ABI with its ctypes signature
SIGNATURES = {
    "pe_abi_version": (_c_int, []),
    "pe_last_error": (ctypes.c_char_p, []),
    "pe_system_create": (_c_int, [ctypes.POINTER(_p), _c_int, _c_int, _c_int, _p, _p, _p, _p, _p, _p]),
    "pe_system_destroy": (_c_int, [_p]),
    "pe_system_info": (_c_int, [_p, _p]),
    "pe_system_set_shape": (_c_int, [_p, _c_int, _c_int, _p]),
    "pe_eval": (_c_int, [_p, _c_int, _p, _p, _p, _p]),
    "pe_eval_terms": (_c_int, [_p, _c_int, _p, _p, _p, _p]),
    "pe_eval_adjoint": (_c_int, [_p, _c_int, _p, _p, _p, _p]),
    "pe_eval_adjoint_static": (_c_int, [_p, _c_int, _p, _p, _p, _p]),
    "pe_batch_create": (_c_int, [ctypes.POINTER(_p), _c_int, _p, _p]),
    "pe_batch_destroy": (_c_int, [_p]),
    "pe_batch_layout": (_c_int, [_p, _p, _p, _p]),
    "pe_batch_info": (_c_int, [_p, _p]),
    "pe_batch_eval": (_c_int, [_p, _c_int, _p, _p, _p, _p]),
    "pe_newton_workspace_bytes": (ctypes.c_size_t, [_p, _c_int]),
    "pe_newton_step": (_c_int, [_p, _c_int, _p, _p, _p, _p]),
    "pe_batch_newton_workspace_bytes": (ctypes.c_size_t, [_p, _c_int]),
    "pe_batch_newton_step": (_c_int, [_p, _c_int, _p, _p, _p, _p]),
    "pe_homotopy_newton_step": (_c_int, [_p, _c_int, _p, _p, ctypes.c_double, _p, _p, _p]),
    "pe_homotopy_predict": (_c_int, [_p, _c_int, _p, _p, ctypes.c_double, _p, _p, _p]),
    "pe_homotopy_track": (_c_int, [_p, _c_int, _p, _p, _c_int, _c_int, _p, _p, _p]),
    "pe_lstsq_workspace_bytes": (ctypes.c_size_t, [_c_int, _c_int, _c_int, _c_int]),
    "pe_lstsq": (_c_int, [_c_int, _c_int, _c_int, _c_int, _p, _p, _p, _p, _p, _p, _p]),
    "pe_autotune": (_c_int, [_p, _c_int, _p]),
    "pe_set_plan_cache": (_c_int, [ctypes.c_char_p]),
}

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class PolyevalError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.pe_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def _check(status: int, where: str):
    if status != PE_OK:
        raise PolyevalError(status, where)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def abi_version() -> int:
    return int(_lib.pe_abi_version())


class System:
    """A polynomial system loaded on the current GPU."""

    def __init__(self, level: int, n_vars: int, poly_ptr, mon_ptr, var_idx, exps, coef, stream=None):
        self.code = int(level)                 # level code as passed to the library
        self.level = self.code & ~PE_REAL      # limbs per real part
        self.ncomp = 1 if self.code & PE_REAL else 2  # components per number
        self.n_vars = int(n_vars)
        self._poly_ptr = np.ascontiguousarray(poly_ptr, dtype=np.int64)
        self._mon_ptr = np.ascontiguousarray(mon_ptr, dtype=np.int64)
        self._var_idx = np.ascontiguousarray(var_idx, dtype=np.int32)
        self._exps = np.ascontiguousarray(exps, dtype=np.int32)
        self._coef = np.ascontiguousarray(coef, dtype=np.float64)
        self.n_polys = int(self._poly_ptr.shape[0] - 1)
        self.n_monomials = int(self._mon_ptr.shape[0] - 1)
        self.nnz = int(self._mon_ptr[-1]) if self.n_monomials > 0 else 0
        h = ctypes.c_void_p()
        st = _lib.pe_system_create(ctypes.byref(h), self.code, self.n_vars, self.n_polys,
                                   self._poly_ptr.ctypes.data, self._mon_ptr.ctypes.data,
                                   self._var_idx.ctypes.data, self._exps.ctypes.data,
                                   self._coef.ctypes.data, _stream(stream) if stream is not False else None)
        _check(st, "pe_system_create")
        self._h = h
        del self._var_idx, self._exps, self._coef, self._mon_ptr

    @classmethod
    def from_sparse(cls, s, stream=None) -> "System":
        """From a ``synth.PolySystem``."""
        return cls(s.level, s.n_vars, s.poly_ptr, s.mon_ptr, s.var_idx, s.exps, s.coef, stream)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        buf = (ctypes.c_int64 * 11)()
        _check(_lib.pe_system_info(self._h, buf), "pe_system_info")
        keys = ("level", "n", "N", "M", "nnz", "emax", "kmax", "device_bytes", "chunks_per_workgroup",
                "lds_bytes", "segment")
        return dict(zip(keys, list(buf)))

    def set_shape(self, chunks_per_workgroup: int = 0, segment: int = 0, stream=None):
        """Launch shape: chunks per workgroup (1, 2, 4; 0 = largest fitting)
        and variables per lane (0 = the level's default)."""
        _check(_lib.pe_system_set_shape(self._h, int(segment), int(chunks_per_workgroup), _stream(stream)),
               "pe_system_set_shape")

    def close(self):
        if getattr(self, "_h", None):
            _lib.pe_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- evaluation
    def _check_x(self, x):
        import torch
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float64 CUDA tensor")
        if x.dim() != 4 or tuple(x.shape[1:]) != (self.ncomp, self.level, self.n_vars):
            raise ValueError(f"x must have shape [P, {self.ncomp}, {self.level}, {self.n_vars}], got {tuple(x.shape)}")

    def eval(self, x, want_J: bool = True, out=None, stream=None):
        """F (and J) at the points x[P, 2, L, n]."""
        import torch
        self._check_x(x)
        P = x.shape[0]
        if out is None:
            F = torch.empty((P, self.ncomp, self.level, self.n_polys), dtype=torch.float64, device=x.device)
            J = torch.empty((P, self.ncomp, self.level, self.n_polys, self.n_vars), dtype=torch.float64,
                            device=x.device) if want_J else None
        else:
            F, J = out
        _check(_lib.pe_eval(self._h, P, _ptr(x), _ptr(F), _ptr(J), _stream(stream)), "pe_eval")
        return F, J

    def eval_terms(self, x, out=None, stream=None):
        """Every monomial's value V[P, 2, L, M] and partial derivatives
        G[P, 2, L, nnz] (input order), unsummed."""
        import torch
        self._check_x(x)
        P = x.shape[0]
        if out is None:
            V = torch.empty((P, self.ncomp, self.level, self.n_monomials), dtype=torch.float64, device=x.device)
            G = torch.empty((P, self.ncomp, self.level, self.nnz), dtype=torch.float64, device=x.device)
        else:
            V, G = out
        _check(_lib.pe_eval_terms(self._h, P, _ptr(x), _ptr(V), _ptr(G), _stream(stream)), "pe_eval_terms")
        return V, G

    def adjoint(self, x, v, out=None, stream=None):
        """g = J(x)^H v for x[P, 2, L, n], v[P, 2, L, N]."""
        import torch
        self._check_x(x)
        if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous() or \
                tuple(v.shape) != (x.shape[0], 2, self.level, self.n_polys):
            raise ValueError("v must be a contiguous float64 CUDA tensor [P, 2, L, N]")
        g = torch.empty_like(x) if out is None else out
        _check(_lib.pe_eval_adjoint(self._h, x.shape[0], _ptr(x), _ptr(v), _ptr(g), _stream(stream)),
               "pe_eval_adjoint")
        return g

    def adjoint_static(self, x, v, out=None, stream=None):
        """g = J(x)^H v through pe_eval_adjoint_static (no allocation in the
        library; calls on one GPU must not overlap)."""
        import torch
        self._check_x(x)
        if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous() or \
                tuple(v.shape) != (x.shape[0], 2, self.level, self.n_polys):
            raise ValueError("v must be a contiguous float64 CUDA tensor [P, 2, L, N]")
        g = torch.empty_like(x) if out is None else out
        _check(_lib.pe_eval_adjoint_static(self._h, x.shape[0], _ptr(x), _ptr(v), _ptr(g), _stream(stream)),
               "pe_eval_adjoint_static")
        return g

    def newton_workspace_bytes(self, P: int) -> int:
        return int(_lib.pe_newton_workspace_bytes(self._h, P))

    def newton_step(self, x, workspace=None, resid=None, stream=None):
        """One Gauss-Newton step in place on x[P, 2, L, n]; returns (x, resid[P, 2])."""
        import torch
        self._check_x(x)
        P = x.shape[0]
        if workspace is None:
            nbytes = self.newton_workspace_bytes(P)
            workspace = torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=x.device)
        if resid is None:
            resid = torch.empty((P, 2), dtype=torch.float64, device=x.device)
        _check(_lib.pe_newton_step(self._h, P, _ptr(x), _ptr(workspace), _ptr(resid), _stream(stream)),
               "pe_newton_step")
        return x, resid

    def _homotopy_args(self, x, c, workspace, resid):
        import torch
        self._check_x(x)
        P = x.shape[0]
        if c.dtype != torch.float64 or not c.is_cuda or not c.is_contiguous() or \
                tuple(c.shape) != (P, self.ncomp, self.level, self.n_polys):
            raise ValueError("c must be a contiguous float64 CUDA tensor [P, components, L, N]")
        if workspace is None:
            nbytes = self.newton_workspace_bytes(P)
            workspace = torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=x.device)
        if resid is None:
            resid = torch.empty((P, 2), dtype=torch.float64, device=x.device)
        return P, workspace, resid

    def homotopy_newton_step(self, x, c, t: float, workspace=None, resid=None, stream=None):
        """One Gauss-Newton step on f(x) - t c = 0, in place on x[P, 2, L, n]."""
        P, workspace, resid = self._homotopy_args(x, c, workspace, resid)
        _check(_lib.pe_homotopy_newton_step(self._h, P, _ptr(x), _ptr(c), float(t), _ptr(workspace), _ptr(resid),
                                            _stream(stream)), "pe_homotopy_newton_step")
        return x, resid

    def homotopy_predict(self, x, c, dt: float, workspace=None, resid=None, stream=None):
        """Euler predictor x += dx, J(x) dx = c dt, in place."""
        P, workspace, resid = self._homotopy_args(x, c, workspace, resid)
        _check(_lib.pe_homotopy_predict(self._h, P, _ptr(x), _ptr(c), float(dt), _ptr(workspace), _ptr(resid),
                                        _stream(stream)), "pe_homotopy_predict")
        return x, resid

    def homotopy_track(self, x, c, steps: int, corrector_iters: int = 3, workspace=None, resid=None, stream=None):
        """Track f(x) - t c = 0 from t = 1 (x = z with c = f(z)) to t = 0, in
        place on x[P, 2, L, n]."""
        P, workspace, resid = self._homotopy_args(x, c, workspace, resid)
        _check(_lib.pe_homotopy_track(self._h, P, _ptr(x), _ptr(c), int(steps), int(corrector_iters),
                                      _ptr(workspace), _ptr(resid), _stream(stream)), "pe_homotopy_track")
        return x, resid

    def autotune(self, P: int = 1, stream=None):
        _check(_lib.pe_autotune(self._h, P, _stream(stream)), "pe_autotune")


class Batch:
    """Several systems of one level evaluated in one persistent launch."""

    def __init__(self, systems, stream=None):
        self.systems = list(systems)
        if not self.systems:
            raise ValueError("empty batch")
        self.level = self.systems[0].level
        arr = (ctypes.c_void_p * len(self.systems))(*[s.handle.value for s in self.systems])
        h = ctypes.c_void_p()
        _check(_lib.pe_batch_create(ctypes.byref(h), len(self.systems), arr, _stream(stream)), "pe_batch_create")
        self._h = h
        S = len(self.systems)
        xo = np.zeros(S + 1, np.int64)
        fo = np.zeros(S + 1, np.int64)
        jo = np.zeros(S + 1, np.int64)
        _check(_lib.pe_batch_layout(self._h, xo.ctypes.data, fo.ctypes.data, jo.ctypes.data), "pe_batch_layout")
        self.x_off, self.F_off, self.J_off = xo, fo, jo

    def info(self) -> dict:
        v = np.zeros(4, np.int64)
        _check(_lib.pe_batch_info(self._h, v.ctypes.data), "pe_batch_info")
        return {"systems": int(v[0]), "level": int(v[1]), "segment": int(v[2]), "chunks_per_workgroup": int(v[3])}

    def close(self):
        if getattr(self, "_h", None):
            _lib.pe_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self, x, P: int, want_J: bool = True, out=None, stream=None):
        """x: flat float64 CUDA tensor of x_off[-1] * P doubles."""
        import torch
        if out is None:
            F = torch.empty(int(self.F_off[-1]) * P, dtype=torch.float64, device=x.device)
            J = torch.empty(int(self.J_off[-1]) * P, dtype=torch.float64, device=x.device) if want_J else None
        else:
            F, J = out
        _check(_lib.pe_batch_eval(self._h, P, _ptr(x), _ptr(F), _ptr(J), _stream(stream)), "pe_batch_eval")
        return F, J

    def newton_workspace_bytes(self, P: int) -> int:
        return int(_lib.pe_batch_newton_workspace_bytes(self._h, P))

    def newton_step(self, x, P: int, workspace=None, resid=None, stream=None):
        import torch
        if workspace is None:
            nbytes = self.newton_workspace_bytes(P)
            workspace = torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=x.device)
        if resid is None:
            resid = torch.empty((len(self.systems), P, 2), dtype=torch.float64, device=x.device)
        _check(_lib.pe_batch_newton_step(self._h, P, _ptr(x), _ptr(workspace), _ptr(resid), _stream(stream)),
               "pe_batch_newton_step")
        return x, resid


def lstsq(Ab, want_R: bool = False, want_Q: bool = False, workspace=None, stream=None):
    """Least-squares solution of A x = b for Ab[P, C, L, N, n + 1] (float64
    CUDA, column n = b; C = 2 complex, C = 1 real) by modified Gram-Schmidt
    on [A b].  Returns (x[P, C, L, n], resid[P, 2], R[P, C, L, n, n + 1] or
    None, Q[P, C, L, N, n] or None)."""
    import torch
    if Ab.dtype != torch.float64 or not Ab.is_cuda or not Ab.is_contiguous() or Ab.dim() != 5 or \
            Ab.shape[1] not in (1, 2):
        raise ValueError("Ab must be a contiguous float64 CUDA tensor [P, C, L, N, n + 1], C = 2 or 1")
    P, C, L, N, n1 = Ab.shape
    code = L | (PE_REAL if C == 1 else 0)
    n = n1 - 1
    dev = Ab.device
    x = torch.empty((P, C, L, n), dtype=torch.float64, device=dev)
    resid = torch.empty((P, 2), dtype=torch.float64, device=dev)
    R = torch.empty((P, C, L, n, n + 1), dtype=torch.float64, device=dev) if want_R else None
    Q = torch.empty((P, C, L, N, n), dtype=torch.float64, device=dev) if want_Q else None
    if workspace is None:
        nbytes = int(_lib.pe_lstsq_workspace_bytes(code, P, N, n))
        workspace = torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=dev)
    _check(_lib.pe_lstsq(code, P, N, n, _ptr(Ab), _ptr(x), _ptr(resid), _ptr(R), _ptr(Q), _ptr(workspace),
                         _stream(stream)), "pe_lstsq")
    return x, resid, R, Q


def set_plan_cache(path: str | None):
    _check(_lib.pe_set_plan_cache(None if path is None else path.encode()), "pe_set_plan_cache")
