"""Driver of the FP64 oracle: forest -> tables -> Algorithm 1 loops in C.

Test infrastructure only (see the package docstring).

State convention: between coarse steps the oracle holds, as Algorithm 1
does, the post-streaming state on every I_L.  The initial state
f = f^eq(rho, u) is both post-streaming and post-collision, since collision
leaves an equilibrium unchanged.
"""

from __future__ import annotations

import ctypes
import os
import numpy as np

from . import build as _build
from .forest import Forest
from .tables import build_tables

Q = 19


class _Level(ctypes.Structure):
    _fields_ = [
        ("n_int", ctypes.c_int64), ("n_live", ctypes.c_int64), ("n_store", ctypes.c_int64),
        ("F", ctypes.c_void_p), ("G", ctypes.c_void_p),
        ("pull", ctypes.c_void_p), ("expl_src", ctypes.c_void_p),
        ("n_coal", ctypes.c_int64),
        ("coal_cell", ctypes.c_void_p), ("coal_dir", ctypes.c_void_p), ("coal_child", ctypes.c_void_p),
        ("omega", ctypes.c_double),
        ("poison_far", ctypes.c_int),
        ("trt", ctypes.c_int),
        ("lambda_o", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
        ("interp", ctypes.c_int),
        ("expl_oct", ctypes.c_void_p),
        ("expl_nbr", ctypes.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        lib.orc_coarse_steps.argtypes = [ctypes.POINTER(_Level), ctypes.c_int, ctypes.c_int]
        lib.orc_explode.argtypes = [ctypes.POINTER(_Level), ctypes.c_int]
        for name in ("orc_equilibrium", "orc_moments"):
            getattr(lib, name).argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_collide.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_double]
        lib.orc_collide_trt.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_void_p]
        lib.orc_lattice.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_stream_calls.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        if lib.orc_sizeof_level() != ctypes.sizeof(_Level):
            raise RuntimeError("oracle struct layout mismatch")
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def set_threads(n: int) -> int:
    """Host threads of the oracle's loops (n <= 0 leaves them); returns the
    previous maximum."""
    return int(_load().orc_set_threads(int(n)))


def lattice():
    """(e, w): the oracle's D3Q19 velocities (19, 3) and weights (19,)."""
    e = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    _load().orc_lattice(_ptr(e), _ptr(w))
    return e, w


def equilibrium(rho, u) -> np.ndarray:
    """eq. fequ for arrays rho (N,), u (N, 3); returns (N, 19)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
    out = np.empty((len(rho), Q), dtype=np.float64)
    _load().orc_equilibrium(len(rho), _ptr(rho), _ptr(u), _ptr(out))
    return out


def moments(f):
    """rho = sum f, u = sum e f / rho0 (rho0 = 1) for f (N, 19)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.empty(len(f))
    u = np.empty((len(f), 3))
    _load().orc_moments(len(f), _ptr(f), _ptr(rho), _ptr(u))
    return rho, u


def collide(f, omega: float) -> np.ndarray:
    """One SRT collision of every row of f (N, 19); returns a new array."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _load().orc_collide(len(f), _ptr(f), float(omega))
    return f


def collide_trt(f, lambda_e: float, lambda_o: float, accel=(0.0, 0.0, 0.0)) -> np.ndarray:
    """One TRT collision with a body force (section 2) of every row of f
    (N, 19); returns a new array."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    a = np.ascontiguousarray(accel, dtype=np.float64)
    _load().orc_collide_trt(len(f), _ptr(f), float(lambda_e), float(lambda_o), _ptr(a))
    return f


def lambda_o_level(lambda_e, lambda_eo):
    """eq. lambda_oL: the odd rate that keeps Lambda_eo (eq. lambda_eo) at
    the given value for the even rate lambda_e.  Exact for Fractions."""
    return (4 - 2 * lambda_e) / (2 + (4 * lambda_eo - 1) * lambda_e)


def accel_level(accel0, L: int):
    """eq. force_scaling: a_L = a_0 / 2^L (lattice units of level L)."""
    return [a / 2 ** L for a in accel0]


def omega_level(omega0, L: int):
    """eq. omega_scaling_0: omega_L = 2 w0 / (2^(L+1) + (1 - 2^L) w0).
    Exact if omega0 is a Fraction."""
    two_L = 2 ** L
    return 2 * omega0 / (2 * two_L + (1 - two_L) * omega0)


class RefinedOracle:
    """FP64 Algorithm-1 oracle on a 2:1 balanced forest."""

    def __init__(self, forest: Forest, omega0: float, coalescence: str = "virtual", lambda_eo=None,
                 accel0=None, interpolation: bool = False):
        """omega0: SRT omega_0, or with lambda_eo (TRT) the even rate
        lambda_e,0, scaled per level by eq. omega_scaling_0.  lambda_eo: TRT
        with lambda_o,L from eq. lambda_oL; accel0: constant lattice
        acceleration of level 0 (force term, a_L by eq. force_scaling).
        interpolation: explode with the limited linear reconstruction
        (refined_oracle.c, explode) instead of eq. ctof."""
        self.interpolation = bool(interpolation)
        self.forest = forest
        self.n = forest.n
        self.num_levels = forest.max_level + 1
        self.tables = build_tables(forest, coalescence)
        self._omega0 = omega0
        self._coalescence = coalescence
        self.omega = [float(omega_level(float(omega0), L)) for L in range(self.num_levels)]
        self.trt = lambda_eo is not None or accel0 is not None
        self.lambda_o = [float(lambda_o_level(w, lambda_eo)) if lambda_eo is not None else w for w in self.omega]
        a0 = [float(a) for a in (accel0 if accel0 is not None else (0.0, 0.0, 0.0))]
        self.accel = [accel_level(a0, L) for L in range(self.num_levels)]
        self.F = []
        self.G = []
        for t in self.tables:
            c = t.cells
            self.F.append(np.full((c.n_store, Q), np.nan))
            self.G.append(np.empty((c.n_live, Q)))
        self._levels = None
        self.poison_far = False
        self.steps_done = 0

    # -- sizes -----------------------------------------------------------------
    def n_int(self, L: int) -> int:
        return self.tables[L].cells.n_int

    def total_cells(self) -> int:
        return sum(self.n_int(L) for L in range(self.num_levels))

    def updates_per_coarse_step(self) -> int:
        return sum((2 ** L) * self.n_int(L) for L in range(self.num_levels))

    # -- state -------------------------------------------------------------------
    def init_pdfs(self, rho, u):
        """f = f^eq(rho, u) on every I_L; rho (N,), u (N, 3) in canonical order
        (level-major, blocks canonical, x fastest)."""
        rho = np.asarray(rho, dtype=np.float64)
        u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
        off = 0
        for L in range(self.num_levels):
            m = self.n_int(L)
            self.F[L][:] = np.nan
            if m:
                self.F[L][:m] = equilibrium(rho[off:off + m], u[off:off + m])
            off += m
        if off != len(rho):
            raise ValueError("rho/u length does not match the number of interior cells")

    def set_interior_pdfs(self, L: int, f):
        self.F[L][:self.n_int(L)] = f

    def interior_pdfs(self, L: int) -> np.ndarray:
        return self.F[L][:self.n_int(L)]

    def _build_levels(self):
        arr = (_Level * self.num_levels)()
        for L, t in enumerate(self.tables):
            c = t.cells
            lv = arr[L]
            lv.n_int, lv.n_live, lv.n_store = c.n_int, c.n_live, c.n_store
            lv.F = self.F[L].ctypes.data_as(ctypes.c_void_p)
            lv.G = _ptr(self.G[L])
            lv.pull = _ptr(t.pull)
            lv.expl_src = _ptr(t.expl_src)
            lv.n_coal = len(t.coal_cell)
            lv.coal_cell = _ptr(t.coal_cell)
            lv.coal_dir = _ptr(t.coal_dir)
            lv.coal_child = _ptr(t.coal_child)
            lv.omega = self.omega[L]
            lv.poison_far = int(self.poison_far)
            lv.trt = int(self.trt)
            lv.lambda_o = self.lambda_o[L]
            lv.accel = (ctypes.c_double * 3)(*self.accel[L])
            lv.interp = int(self.interpolation)
            lv.expl_oct = _ptr(t.expl_oct)
            lv.expl_nbr = _ptr(t.expl_nbr)
        self._levels = arr

    def step(self, steps: int = 1):
        """`steps` coarse time steps: NonUniformTimeStep(0) each."""
        self._build_levels()
        _load().orc_coarse_steps(self._levels, self.num_levels, int(steps))
        self.steps_done += steps

    def explode(self, L: int):
        """Only the explosion of level L >= 1 from the current level-(L-1)
        state: afterwards stored cells [n_int(L), n_store) hold E_L's values."""
        self._build_levels()
        _load().orc_explode(self._levels, int(L))

    def exploded(self, L: int):
        """(coordinates, values) of the explosion cells E_L of level L."""
        c = self.tables[L].cells
        return c.coords[c.n_int:], self.F[L][c.n_int:]

    def stream_calls(self, reset: bool = True) -> np.ndarray:
        """Stream(L) calls per level since the last reset."""
        out = np.zeros(self.num_levels, dtype=np.int64)
        _load().orc_stream_calls(_ptr(out), self.num_levels, int(reset))
        return out

    def regrid(self, flags, max_level: int):
        """New oracle on the regridded forest with the remapped state (see
        oracle/regrid.py); omega_0 and the coalescence reading are kept."""
        from .regrid import regrid_forest, remap_interior
        nf = regrid_forest(self.forest, flags, max_level)
        if self.trt:
            raise NotImplementedError("regrid of a TRT / forced state")
        new = RefinedOracle(nf, self._omega0, self._coalescence, interpolation=self.interpolation)
        pdfs = remap_interior(self.forest, [self.interior_pdfs(L) for L in range(self.num_levels)], nf)
        for L in range(new.num_levels):
            new.F[L][:] = np.nan
            new.F[L][:new.n_int(L)] = pdfs[L]
        return new

    # -- outputs -------------------------------------------------------------
    def moments(self):
        """(rho (N,), u (N, 3)) over all interior cells in canonical order;
        with a body force u = sum e f / rho0 + a_L / 2 (section 2, external
        forces)."""
        rs, us = [], []
        for L in range(self.num_levels):
            r, u = moments(self.interior_pdfs(L))
            rs.append(r)
            us.append(u + 0.5 * np.asarray(self.accel[L])[None, :])
        return np.concatenate(rs), np.concatenate(us)

    def level_weights(self) -> np.ndarray:
        """Cell volume 8^-L of every interior cell, canonical order."""
        return np.concatenate([np.full(self.n_int(L), 8.0 ** (-L)) for L in range(self.num_levels)])

    def mass(self):
        """Volume-weighted mass and momentum, sum_L 8^-L sum_{I_L} (f, e f)."""
        e, _ = lattice()
        M = 0.0
        J = np.zeros(3)
        for L in range(self.num_levels):
            f = self.interior_pdfs(L)
            M += 8.0 ** (-L) * f.sum()
            J += 8.0 ** (-L) * (f @ e.astype(np.float64)).sum(0)
        return M, J


def oracle_library_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "liborc_refined.so")
