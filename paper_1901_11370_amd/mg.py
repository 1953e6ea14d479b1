"""Python binding of the C ABI in ``include/mg.h`` (ctypes, argument marshalling only).

Every ``mg_*`` function below has the name, arguments and meaning of the C function;
the :class:`Tree` class bundles them with a torch-allocated device store and the
current torch stream.  All numerical work runs in the HIP kernels of
``libmg_gpu.so``; if that library is missing this module raises on import.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmg_gpu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1901_11370_amd/build.py "
                      "(there is no CPU fallback)")

# torch brings its own HIP runtime (same soname as the system one).  Loading torch
# first makes the library bind to that runtime, so device pointers and streams from
# torch and the library's launches share one runtime in the process.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

MG_OK, MG_ERR_ARG, MG_ERR_NOT_BALANCED, MG_ERR_DEVICE = 0, -1, -2, -3
MG_ERR_NOT_CONVERGED, MG_ERR_OOM, MG_ERR_STATE, MG_ERR_NAN = -4, -5, -6, -7
MG_BC_DIRICHLET, MG_BC_NEUMANN, MG_BC_PERIODIC = 0, 1, 2
MG_FP64, MG_MIXED = 0, 1
MG_SMOOTH_GSRB, MG_SMOOTH_JACOBI = 0, 1


class mg_bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32 * 6), ("value", ctypes.c_double * 6)]


class mg_domain(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("base_cells", ctypes.c_int32 * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("bc", mg_bc)]


class mg_params(ctypes.Structure):
    _fields_ = [("n_down", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_max_coarse", ctypes.c_int32),
                ("coarse_abs_tol", ctypes.c_double), ("coarse_rel_tol", ctypes.c_double),
                ("precision", ctypes.c_int32), ("variable_eps", ctypes.c_int32),
                ("ir_first_fmg", ctypes.c_int32), ("ir_vcycles", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("smoother", ctypes.c_int32), ("jacobi_weight", ctypes.c_double),
                ("helmholtz_lambda", ctypes.c_double), ("axisymmetric", ctypes.c_int32)]


mg_refine_fn = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int32), ctypes.c_int)

_P = ctypes.POINTER
_vp, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "mg_default_params": ([_P(mg_params)], ctypes.c_int),
    "mg_tree_create": ([_P(mg_domain), ctypes.c_int, ctypes.c_int, ctypes.c_int, mg_refine_fn, _vp,
                        _P(mg_params), _P(_vp)], ctypes.c_int),
    "mg_tree_destroy": ([_vp], None),
    "mg_tree_storage_bytes": ([_vp, _P(ctypes.c_size_t)], ctypes.c_int),
    "mg_tree_bind": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "mg_num_leaf_cells": ([_vp, _P(_i64)], ctypes.c_int),
    "mg_domain_leaf_cells": ([_vp, _P(_i64)], ctypes.c_int),
    "mg_num_levels": ([_vp, _P(ctypes.c_int)], ctypes.c_int),
    "mg_leaf_layout": ([_vp, _P(_i32)], ctypes.c_int),
    "mg_level_blocks": ([_vp, _P(_i32), _P(_i64)], ctypes.c_int),
    "mg_set_rhs": ([_vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_set_eps": ([_vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_set_phi": ([_vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_get_phi": ([_vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_set_homogeneous_bc": ([_vp, ctypes.c_int], ctypes.c_int),
    "mg_apply_operator": ([_vp, _vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_boundary_faces": ([_vp, _P(_i64), _P(_i64), _P(_i32)], ctypes.c_int),
    "mg_fold_dirichlet": ([_vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_vcycle": ([_vp, ctypes.c_int], ctypes.c_int),
    "mg_fmg": ([_vp, ctypes.c_int], ctypes.c_int),
    "mg_residual_norm": ([_vp, _P(_d), _P(_d)], ctypes.c_int),
    "mg_residual_norms_static": ([_vp, _vp], ctypes.c_int),
    "mg_domain_residual_norms": ([_vp, _P(_d), _P(_d)], ctypes.c_int),
    "mg_solve": ([_vp, _d, ctypes.c_int, ctypes.c_int, _P(ctypes.c_int)], ctypes.c_int),
    "mg_solve_stats": ([_vp, ctypes.c_int, _P(_d), _P(_d), _P(ctypes.c_int)], ctypes.c_int),
    "mg_face_gradient": ([_vp, _vp, _vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_divb_rhs": ([_vp, _vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "mg_divb_project": ([_vp, _vp, _vp, ctypes.c_int], ctypes.c_int),
    "mg_freespace_bc": ([_vp, ctypes.c_int, _vp, ctypes.c_int], ctypes.c_int),
    "mg_freespace_values": ([_vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "mg_freespace_guess": ([_vp, ctypes.c_int], ctypes.c_int),
    "mg_profile_enable": ([_vp, ctypes.c_int], ctypes.c_int),
    "mg_profile_read": ([_vp, _P(_i64), _P(_d), _P(_d)], ctypes.c_int),
    "mg_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "mg_last_error": ([_vp], ctypes.c_char_p),
}
EXPORTED = tuple(_SIGS)
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f


def torch_float64():
    import torch
    return torch.float64


class MGError(RuntimeError):
    def __init__(self, status, text=""):
        self.status = status
        msg = mg_strerror(status).decode()
        super().__init__(f"{msg} ({status})" + (f": {text}" if text else ""))


def _check(rc, handle=None, allow=()):
    if rc != MG_OK and rc not in allow:
        text = mg_last_error(handle).decode() if handle else ""
        raise MGError(rc, text)
    return rc


@dataclass
class Domain:
    """One independent box: ``base_cells`` cells on [lo, hi] with per-face boundary
    kinds/values (faces -x, +x, -y, +y, -z, +z)."""
    dim: int
    base_cells: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    bc_kind: Sequence[int]
    bc_value: Sequence[float] = field(default_factory=lambda: [0.0] * 6)

    def to_c(self) -> mg_domain:
        d = mg_domain()
        d.dim = self.dim
        for a in range(3):
            d.base_cells[a] = int(self.base_cells[a]) if a < self.dim else 1
            d.lo[a] = float(self.lo[a]) if a < self.dim else 0.0
            d.hi[a] = float(self.hi[a]) if a < self.dim else 1.0
        for f in range(6):
            d.bc.kind[f] = int(self.bc_kind[f]) if f < 2 * self.dim else MG_BC_PERIODIC
            d.bc.value[f] = float(self.bc_value[f]) if f < len(self.bc_value) else 0.0
        return d


def default_params(**kw) -> mg_params:
    p = mg_params()
    _check(mg_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Tree:
    """A forest of block trees bound to a torch-allocated device store."""

    def __init__(self, domains, bs: int = 16, max_refine: int = 0, refine: Optional[Callable] = None,
                 params: Optional[mg_params] = None, bind: bool = True, device: str = "cuda"):
        doms = (mg_domain * len(domains))(*[d.to_c() if isinstance(d, Domain) else d for d in domains])
        self.ndom = len(domains)
        self.dim = doms[0].dim
        self.params = params if params is not None else default_params()

        def _cb(ud, dom, level, origin, b):
            return 1 if refine(dom, level, (origin[0], origin[1], origin[2]), b) else 0

        self._cb = mg_refine_fn(_cb) if refine is not None else mg_refine_fn(0)
        h = _vp()
        _check(mg_tree_create(doms, len(domains), bs, max_refine, self._cb, None, ctypes.byref(self.params),
                              ctypes.byref(h)))
        self.h = h
        n = _i64()
        _check(mg_num_leaf_cells(self.h, ctypes.byref(n)), self.h)
        self.n_leaf = int(n.value)
        nb = ctypes.c_size_t()
        _check(mg_tree_storage_bytes(self.h, ctypes.byref(nb)), self.h)
        self.storage_bytes = int(nb.value)
        self.store = None
        if bind:
            self.bind(device)

    def bind(self, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("binding a tree needs a GPU")
        # one torch allocation; the caching allocator returns 512-byte aligned blocks
        self.store = torch.empty(self.storage_bytes + 256, dtype=torch.uint8, device=device)
        ptr = self.store.data_ptr()
        aligned = (ptr + 255) & ~255
        self.stream = torch.cuda.current_stream(self.store.device)
        _check(mg_tree_bind(self.h, _vp(aligned), self.storage_bytes, _vp(self.stream.cuda_stream)), self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and mg_tree_destroy is not None:   # None during interpreter shutdown
            mg_tree_destroy(h)
            self.h = None

    # -------------------------------------------------------------- structure
    def leaf_layout(self) -> np.ndarray:
        out = np.zeros((self.n_leaf, 5), dtype=np.int32)
        _check(mg_leaf_layout(self.h, out.ctypes.data_as(_P(_i32))), self.h)
        return out

    def domain_leaf_cells(self):
        out = np.zeros(self.ndom, dtype=np.int64)
        _check(mg_domain_leaf_cells(self.h, out.ctypes.data_as(_P(_i64))), self.h)
        return out

    def num_levels(self) -> int:
        n = ctypes.c_int()
        _check(mg_num_levels(self.h, ctypes.byref(n)), self.h)
        return n.value

    def level_blocks(self):
        n = self.num_levels()
        nb = np.zeros(n, dtype=np.int32)
        nc = np.zeros(n, dtype=np.int64)
        _check(mg_level_blocks(self.h, nb.ctypes.data_as(_P(_i32)), nc.ctypes.data_as(_P(_i64))), self.h)
        return nb, nc

    # ------------------------------------------------------------------ data
    def _arg(self, a):
        """(pointer, on_device, keepalive) for a leaf array (torch CUDA tensor or host)."""
        try:
            import torch
            if isinstance(a, torch.Tensor):
                if a.is_cuda:
                    a = a.detach().to(torch.float64).contiguous()
                    assert a.numel() == self.n_leaf
                    return _vp(a.data_ptr()), 1, a
                a = a.detach().numpy()
        except ImportError:
            pass
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.size == self.n_leaf
        return a.ctypes.data_as(_vp), 0, a

    def set_rhs(self, f):
        p, dev, keep = self._arg(f)
        _check(mg_set_rhs(self.h, p, dev), self.h)

    def set_eps(self, e):
        p, dev, keep = self._arg(e)
        _check(mg_set_eps(self.h, p, dev), self.h)

    def set_phi(self, phi):
        p, dev, keep = self._arg(phi)
        _check(mg_set_phi(self.h, p, dev), self.h)

    def get_phi(self, out=None):
        """Leaf phi: into ``out`` (torch CUDA tensor), else a new numpy array."""
        if out is not None:
            _check(mg_get_phi(self.h, _vp(out.data_ptr()), 1), self.h)
            return out
        a = np.zeros(self.n_leaf)
        _check(mg_get_phi(self.h, a.ctypes.data_as(_vp), 0), self.h)
        return a

    def apply_operator(self, phi, out=None):
        """L phi on the leaves (composite operator, the tree's eps and boundary values).
        phi a CUDA tensor: the result is a CUDA tensor (``out`` if given); else numpy."""
        p, dev, keep = self._arg(phi)
        if dev:
            import torch
            o = out if out is not None else torch.empty(self.n_leaf, dtype=torch.float64, device=self.store.device)
            _check(mg_apply_operator(self.h, p, _vp(o.data_ptr()), 1), self.h)
            return o
        o = np.zeros(self.n_leaf)
        _check(mg_apply_operator(self.h, p, o.ctypes.data_as(_vp), 0), self.h)
        return o

    def boundary_faces(self):
        """(leaf_cell, face) of every leaf-cell face on a physical Dirichlet face, in the
        order mg_fold_dirichlet takes its values."""
        n = _i64()
        _check(mg_boundary_faces(self.h, ctypes.byref(n), None, None), self.h)
        cells = np.zeros(n.value, dtype=np.int64)
        faces = np.zeros(n.value, dtype=np.int32)
        _check(mg_boundary_faces(self.h, ctypes.byref(n), cells.ctypes.data_as(_P(_i64)),
                                 faces.ctypes.data_as(_P(_i32))), self.h)
        return cells, faces

    def fold_dirichlet(self, values):
        """f_b -= 2 a / h^2 for the face values a (order of boundary_faces())."""
        p, dev, keep = self._arg_n(values)
        _check(mg_fold_dirichlet(self.h, p, dev), self.h)

    def _arg_n(self, a):
        """(pointer, on_device, keepalive) for an array of any length."""
        import torch
        if isinstance(a, torch.Tensor) and a.is_cuda:
            a = a.detach().to(torch.float64).contiguous()
            return _vp(a.data_ptr()), 1, a
        if isinstance(a, torch.Tensor):
            a = a.detach().numpy()
        a = np.ascontiguousarray(a, dtype=np.float64)
        return a.ctypes.data_as(_vp), 0, a

    def set_homogeneous_bc(self, on: bool):
        _check(mg_set_homogeneous_bc(self.h, 1 if on else 0), self.h)

    # ---------------------------------------------------------------- cycles
    def vcycle(self, n=1):
        _check(mg_vcycle(self.h, n), self.h)

    def fmg(self, n=1):
        _check(mg_fmg(self.h, n), self.h)

    def residual_norm(self):
        a, b = _d(), _d()
        _check(mg_residual_norm(self.h, ctypes.byref(a), ctypes.byref(b)), self.h, allow=(MG_ERR_NAN,))
        return a.value, b.value

    def domain_residual_norms(self):
        a = np.zeros(self.ndom)
        b = np.zeros(self.ndom)
        _check(mg_domain_residual_norms(self.h, a.ctypes.data_as(_P(_d)), b.ctypes.data_as(_P(_d))), self.h)
        return a, b

    def solve(self, rel_tol=1e-10, max_cycles=50, fmg_first=True, raise_on_fail=True):
        c = ctypes.c_int()
        rc = mg_solve(self.h, rel_tol, max_cycles, 1 if fmg_first else 0, ctypes.byref(c))
        if raise_on_fail:
            _check(rc, self.h)
        return c.value, rc

    def solve_stats(self):
        n = ctypes.c_int()
        _check(mg_solve_stats(self.h, 0, None, None, ctypes.byref(n)), self.h)
        r = np.zeros(max(n.value, 1))
        s = np.zeros(max(n.value, 1))
        _check(mg_solve_stats(self.h, n.value, r.ctypes.data_as(_P(_d)), s.ctypes.data_as(_P(_d)),
                              ctypes.byref(n)), self.h)
        return r[:n.value], s[:n.value]

    def face_gradient(self, phi, lam, out=None):
        p1, d1, k1 = self._arg(phi)
        p2, d2, k2 = self._arg(lam)
        if d1 != d2:
            raise ValueError("phi and lambda must both be on the device or both on the host")
        if d1:
            import torch
            o = out if out is not None else torch.empty(self.n_leaf, dtype=torch.float64, device=self.store.device)
            _check(mg_face_gradient(self.h, p1, p2, _vp(o.data_ptr()), 1), self.h)
            return o
        o = np.zeros(self.n_leaf)
        _check(mg_face_gradient(self.h, p1, p2, o.ctypes.data_as(_vp), 0), self.h)
        return o

    # ------------------------------------------------ divergence cleaning
    def _field(self, a, ncomp):
        """(pointer, on_device, array) for a (ncomp, n_leaf) float64 field, in place when
        it already is a contiguous float64 array or CUDA tensor."""
        try:
            import torch
            if isinstance(a, torch.Tensor) and a.is_cuda:
                if a.dtype != torch.float64 or not a.is_contiguous():
                    a = a.detach().to(torch.float64).contiguous()
                assert a.numel() == ncomp * self.n_leaf
                return _vp(a.data_ptr()), 1, a
        except ImportError:
            pass
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
            a = np.ascontiguousarray(np.asarray(a), dtype=np.float64)
        assert a.size == ncomp * self.n_leaf
        return a.ctypes.data_as(_vp), 0, a

    def divb_rhs(self, B, order=2):
        """f = div B (central differences of order 2 or 4), B of shape (dim, n_leaf)."""
        p, dev, keep = self._field(B, self.dim)
        _check(mg_divb_rhs(self.h, p, int(order), dev), self.h)

    def divb_project(self, B, e=None):
        """B <- B - grad phi and e <- e + (|B_new|^2 - |B_old|^2)/2 with the current phi.
        Works in place where the arrays allow it; returns (B, e)."""
        pb, db, b = self._field(B, self.dim)
        pe, de, ee = (None, db, None) if e is None else self._field(e, 1)
        if de != db:
            raise ValueError("B and e must both be on the device or both on the host")
        _check(mg_divb_project(self.h, pb, pe, db), self.h)
        return b, ee

    # ------------------------------------------------ free-space boundaries
    def freespace_values(self):
        n = _i64()
        _check(mg_freespace_values(self.h, ctypes.byref(n)), self.h)
        return int(n.value)

    def freespace_bc(self, coarsen=1, values=False, out=None):
        """Folds the free-space Dirichlet values of the current right-hand side into it
        (potential of the right-hand side restricted by 2^coarsen).  With values=True
        returns them (numpy, face-by-face order); with out (a CUDA float64 tensor of
        freespace_values() elements) writes them there on the device."""
        if out is not None:
            assert out.is_cuda and out.dtype == torch_float64() and out.numel() == self.freespace_values()
            _check(mg_freespace_bc(self.h, int(coarsen), _vp(out.data_ptr()), 1), self.h)
            return out
        if values:
            a = np.zeros(self.freespace_values())
            _check(mg_freespace_bc(self.h, int(coarsen), a.ctypes.data_as(_vp), 0), self.h)
            return a
        _check(mg_freespace_bc(self.h, int(coarsen), None, 0), self.h)
        return None

    def freespace_guess(self, coarsen=1):
        """phi = far-field potential of the current right-hand side (before freespace_bc)."""
        _check(mg_freespace_guess(self.h, int(coarsen)), self.h)

    # ------------------------------------------------------------- profiling
    def profile_enable(self, on=True):
        _check(mg_profile_enable(self.h, 1 if on else 0), self.h)

    def profile_read(self):
        n, ms, b = _i64(), _d(), _d()
        _check(mg_profile_read(self.h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)), self.h)
        return int(n.value), ms.value, b.value
