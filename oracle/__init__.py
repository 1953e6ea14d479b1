"""Reference FP64 CPU multigrid (test infrastructure only).

This package is the independent checker of the GPU library.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark import it; the product path never
does.  It wraps ``mg_oracle.c`` (plain C, built with ``-O2 -ffp-contract=off``) through
ctypes and shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("MG_ORACLE_LIB", os.path.join(_HERE, "libmg_oracle.so"))
_SRC = os.path.join(_HERE, "mg_oracle.c")

DIRICHLET, NEUMANN, PERIODIC = 0, 1, 2

REFINE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_int32), ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle into ``libmg_oracle.so`` next to its source."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o",
               _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        d, i32, i64, vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.og_create.restype = vp
        L.og_create.argtypes = [ctypes.c_int, P(i32), P(d), P(d), P(i32), P(d), ctypes.c_int,
                                ctypes.c_int, REFINE_FN, vp, ctypes.c_int, ctypes.c_int]
        L.og_destroy.argtypes = [vp]
        L.og_set_params.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d]
        for name in ("og_num_levels", "og_base_level", "og_num_leaf_blocks", "og_last_coarse_steps"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = ctypes.c_int
        L.og_num_leaf_cells.argtypes = [vp]
        L.og_num_leaf_cells.restype = i64
        L.og_level_info.argtypes = [vp, ctypes.c_int, P(i32), P(i32), P(i32)]
        L.og_leaf_layout.argtypes = [vp, P(i32)]
        for name in ("og_set_rhs", "og_set_eps", "og_set_phi", "og_get_phi", "og_leaf_residual"):
            getattr(L, name).argtypes = [vp, P(d)]
        L.og_vcycle.argtypes = [vp]
        L.og_fmg.argtypes = [vp]
        L.og_residual_norm.argtypes = [vp, P(d), P(d)]
        L.og_apply.argtypes = [vp, P(d), P(d)]
        L.og_face_gradient.argtypes = [vp, P(d), P(d), P(d)]
        L.og_face_gradient.restype = ctypes.c_int
        L.og_level_nblocks.argtypes = [vp, ctypes.c_int]
        L.og_level_nblocks.restype = ctypes.c_int
        L.og_block_meta.argtypes = [vp, ctypes.c_int, ctypes.c_int, P(i32), P(i32)]
        L.og_block_field.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(d)]
        L.og_set_block_field.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(d)]
        L.og_fill_ghosts_level.argtypes = [vp, ctypes.c_int]
        L.og_restrict_all.argtypes = [vp]
        L.og_correct_level.argtypes = [vp, ctypes.c_int]
        L.og_smooth_level.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.og_set_smoother.argtypes = [vp, ctypes.c_int, d]
        L.og_set_lambda.argtypes = [vp, d]
        L.og_set_axisymmetric.argtypes = [vp, ctypes.c_int]
        L.og_set_axisymmetric.restype = ctypes.c_int
        L.og_last_coarse_exit.argtypes = [vp]
        L.og_last_coarse_exit.restype = ctypes.c_int
        L.og_set_coarse_stall.argtypes = [vp, ctypes.c_int]
        L.og_coarse_solve.argtypes = [vp]
        L.og_set_threads.argtypes = [ctypes.c_int]
        L.og_set_threads.restype = ctypes.c_int
        L.og_boundary_faces.argtypes = [vp, P(d), P(i32)]
        L.og_boundary_faces.restype = i64
        L.og_set_boundary_values.argtypes = [vp, P(d)]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads of the reference solver's block loops (results do not depend on it)."""
    return int(lib().og_set_threads(int(n)))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class OracleTree:
    """One domain (one quadtree/octree) of the reference solver.

    ``refine(domain, level, origin, bs) -> bool`` is called for candidate blocks;
    ``level`` counts refinement levels above the base grid (0 = base) and ``origin``
    is the global index of the block's first cell on that level.
    """

    FIELDS = {"v": 0, "f": 1, "vold": 2, "r": 3, "eps": 4}

    def __init__(self, dim, base_cells, lo, hi, bc_kind, bc_value=None, bs=16,
                 max_refine=0, refine=None, domain_id=0, variable_eps=False):
        L = lib()
        self.dim = dim
        nf = 2 * dim
        bc_kind = np.asarray(list(bc_kind) + [PERIODIC] * (6 - nf), dtype=np.int32)
        bc_value = np.zeros(6) if bc_value is None else np.asarray(list(bc_value) + [0.0] * (6 - nf), dtype=np.float64)
        base = np.asarray(list(base_cells) + [1] * (3 - dim), dtype=np.int32)
        lo = np.asarray(list(lo) + [0.0] * (3 - dim), dtype=np.float64)
        hi = np.asarray(list(hi) + [1.0] * (3 - dim), dtype=np.float64)
        self._refine_py = refine

        def _cb(ud, dom, level, origin, bsz):
            o = (origin[0], origin[1], origin[2])
            return 1 if refine(dom, level, o, bsz) else 0

        self._cb = REFINE_FN(_cb) if refine is not None else REFINE_FN(0)
        self._h = L.og_create(dim, _ip(base), _dp(lo), _dp(hi), _ip(bc_kind), _dp(bc_value), bs,
                              max_refine, self._cb, None, domain_id, 1 if variable_eps else 0)
        if not self._h:
            raise ValueError("invalid tree arguments")
        self.lo, self.hi, self.base = lo, hi, base
        self.bc_kind, self.bc_value = bc_kind, bc_value
        self.n_leaf = int(L.og_num_leaf_cells(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().og_destroy(h)
            self._h = None

    # structure
    def set_params(self, n_down=2, n_up=2, n_max=1000, abs_tol=0.0, rel_tol=1e-8):
        lib().og_set_params(self._h, n_down, n_up, n_max, abs_tol, rel_tol)

    GSRB, JACOBI = 0, 1

    def set_smoother(self, kind, omega=2.0 / 3.0):
        lib().og_set_smoother(self._h, kind, omega)

    def set_lambda(self, lam):
        lib().og_set_lambda(self._h, lam)

    def set_axisymmetric(self, on=True):
        if lib().og_set_axisymmetric(self._h, 1 if on else 0) != 0:
            raise ValueError("axisymmetric form needs a 2D domain with lo[0] >= 0")

    @property
    def num_levels(self):
        return lib().og_num_levels(self._h)

    @property
    def base_level(self):
        return lib().og_base_level(self._h)

    def level_info(self, l):
        bs = ctypes.c_int32()
        nc = np.zeros(3, dtype=np.int32)
        nb = ctypes.c_int32()
        lib().og_level_info(self._h, l, ctypes.byref(bs), _ip(nc), ctypes.byref(nb))
        return int(bs.value), tuple(int(x) for x in nc), int(nb.value)

    def leaf_layout(self):
        out = np.zeros((self.n_leaf, 4), dtype=np.int32)
        lib().og_leaf_layout(self._h, _ip(out))
        return out

    @property
    def num_leaf_blocks(self):
        return lib().og_num_leaf_blocks(self._h)

    # data
    def _leaf(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == (self.n_leaf,)
        return a

    def set_rhs(self, f):
        f = self._leaf(f)
        lib().og_set_rhs(self._h, _dp(f))

    def set_eps(self, e):
        e = self._leaf(e)
        lib().og_set_eps(self._h, _dp(e))

    def set_phi(self, p):
        p = self._leaf(p)
        lib().og_set_phi(self._h, _dp(p))

    def get_phi(self):
        out = np.zeros(self.n_leaf)
        lib().og_get_phi(self._h, _dp(out))
        return out

    # cycles
    def vcycle(self, n=1):
        for _ in range(n):
            lib().og_vcycle(self._h)

    def fmg(self, n=1):
        for _ in range(n):
            lib().og_fmg(self._h)

    def residual_norm(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        lib().og_residual_norm(self._h, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def leaf_residual(self):
        out = np.zeros(self.n_leaf)
        lib().og_leaf_residual(self._h, _dp(out))
        return out

    def apply(self, phi):
        phi = self._leaf(phi)
        out = np.zeros(self.n_leaf)
        lib().og_apply(self._h, _dp(phi), _dp(out))
        return out

    @property
    def last_coarse_steps(self):
        return lib().og_last_coarse_steps(self._h)

    EXIT_TARGET, EXIT_NMAX, EXIT_STALL = 0, 1, 2

    @property
    def last_coarse_exit(self):
        return lib().og_last_coarse_exit(self._h)

    def set_coarse_stall(self, steps):
        """Stall window of the coarsest solve (default 8); 0: the paper's rule alone."""
        lib().og_set_coarse_stall(self._h, int(steps))

    def coarse_solve(self):
        """The coarsest-grid solve alone (level 0, current v and f)."""
        lib().og_coarse_solve(self._h)

    def boundary_faces(self):
        """(centres (n, 3), faces (n,)) of the physical Dirichlet faces of every level."""
        n = int(lib().og_boundary_faces(self._h, None, None))
        x = np.zeros((max(n, 1), 3))
        f = np.zeros(max(n, 1), dtype=np.int32)
        lib().og_boundary_faces(self._h, _dp(x), _ip(f))
        return x[:n], f[:n]

    def set_boundary_values(self, vals):
        """Dirichlet values per listed face (order of boundary_faces())."""
        n = int(lib().og_boundary_faces(self._h, None, None))
        v = np.ascontiguousarray(vals, dtype=np.float64)
        assert v.shape == (n,)
        lib().og_set_boundary_values(self._h, _dp(v))

    def set_boundary_function(self, fn):
        """Dirichlet values from fn(centres (n, dim), faces (n,)) -> (n,)."""
        x, f = self.boundary_faces()
        self.set_boundary_values(fn(x[:, :self.dim], f))

    def face_gradient(self, phi, lam):
        phi, lam = self._leaf(phi), self._leaf(lam)
        out = np.zeros(self.n_leaf)
        rc = lib().og_face_gradient(self._h, _dp(phi), _dp(lam), _dp(out))
        if rc != 0:
            raise ValueError("face gradient needs a uniform tree")
        return out

    def solve(self, rel_tol=1e-10, max_cycles=60, fmg_first=True):
        """FMG (optional) then V-cycles until the max-norm relative residual <= rel_tol."""
        hist = []
        if fmg_first:
            self.fmg()
            hist.append(self.residual_norm()[0])
        while (not hist or hist[-1] > rel_tol) and len(hist) < max_cycles:
            self.vcycle()
            hist.append(self.residual_norm()[0])
        return hist

    # inspection
    def level_nblocks(self, l):
        return lib().og_level_nblocks(self._h, l)

    def block_meta(self, l, ib):
        o = np.zeros(3, dtype=np.int32)
        hc = ctypes.c_int32()
        lib().og_block_meta(self._h, l, ib, _ip(o), ctypes.byref(hc))
        return tuple(int(x) for x in o), bool(hc.value)

    def block_field(self, l, ib, field):
        bs = self.level_info(l)[0]
        n = (bs + 2) ** self.dim
        out = np.zeros(n)
        lib().og_block_field(self._h, l, ib, self.FIELDS[field], _dp(out))
        return out.reshape((bs + 2,) * self.dim)  # [k][j][i] in 3D, [j][i] in 2D

    def set_block_field(self, l, ib, field, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        lib().og_set_block_field(self._h, l, ib, self.FIELDS[field], _dp(a))

    def fill_ghosts_level(self, l):
        lib().og_fill_ghosts_level(self._h, l)

    def restrict_all(self):
        lib().og_restrict_all(self._h)

    def correct_level(self, l):
        lib().og_correct_level(self._h, l)

    def smooth_level(self, l, n=1):
        lib().og_smooth_level(self._h, l, n)
