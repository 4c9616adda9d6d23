"""Python binding of liblbm_refined.so (argument marshalling only).

Every computation runs in the HIP library; this module converts numpy
arrays and Python callables to the C ABI declared in include/lbm_refined.h
and raises LBMError on a negative status.  There is no fallback: if the
library is not built, loading it raises.
"""

from __future__ import annotations

import ctypes
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "liblbm_refined.so")

LBM_OK = 0
ERRORS = {
    -1: "LBM_E_INVALID", -2: "LBM_E_COVER", -3: "LBM_E_UNBALANCED", -4: "LBM_E_OOM",
    -5: "LBM_E_HIP", -6: "LBM_E_NONFINITE", -7: "LBM_E_STATE",
}
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}
SCHEDULE = {"graph": 0, "direct": 1, "per_block": 2}

REFINE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p)


class LBMError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class ForestDesc(ctypes.Structure):
    _fields_ = [
        ("root_blocks", ctypes.c_int * 3),
        ("cells_per_block", ctypes.c_int),
        ("max_level", ctypes.c_int),
        ("periodic", ctypes.c_int * 3),
        ("leaves", ctypes.POINTER(ctypes.c_int32)),
        ("num_leaves", ctypes.c_int64),
        ("refine", REFINE_FN),
        ("refine_user", ctypes.c_void_p),
        ("balance", ctypes.c_int),
        ("storage", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


_lib = None

# (name, argtypes) of every exported entry point
_SIGNATURES = {
    "lbm_create_block_forest": [ctypes.POINTER(ForestDesc), ctypes.POINTER(ctypes.c_void_p)],
    "lbm_destroy": [ctypes.c_void_p],
    "lbm_num_levels": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
    "lbm_num_blocks": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)],
    "lbm_num_cells": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)],
    "lbm_get_leaves": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_level_stats": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p],
    "lbm_set_level_omega": [ctypes.c_void_p, ctypes.c_double],
    "lbm_get_level_omega": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)],
    "lbm_set_trt_force": [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p],
    "lbm_init_pdfs": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_step_coarse": [ctypes.c_void_p, ctypes.c_int],
    "lbm_get_moments": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_get_moments_static": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_mass": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p],
    "lbm_set_schedule": [ctypes.c_void_p, ctypes.c_int],
    "lbm_set_coalescence_check": [ctypes.c_void_p, ctypes.c_int],
    "lbm_set_coalescence_fusion": [ctypes.c_void_p, ctypes.c_int],
    "lbm_set_level_fusion": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int],
    "lbm_get_level_fusion": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p],
    "lbm_set_explosion_interpolation": [ctypes.c_void_p, ctypes.c_int],
    "lbm_set_inplace": [ctypes.c_void_p, ctypes.c_int],
    "lbm_get_inplace": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_device_memory": [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "lbm_coalescence_check": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_set_launch": [ctypes.c_void_p, ctypes.c_int],
    "lbm_synchronize": [ctypes.c_void_p],
    "lbm_time_sweeps": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_time_launches": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p],
    "lbm_regrid": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64],
    "lbm_block_indicators": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_mlp_create": [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)],
    "lbm_mlp_destroy": [ctypes.c_void_p],
    "lbm_mlp_num_params": [ctypes.POINTER(ctypes.c_int)],
    "lbm_mlp_get_params": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_mlp_set_params": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_mlp_set_normalization": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p],
    "lbm_mlp_predict": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p],
    "lbm_mlp_gradient": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p],
    "lbm_mlp_train": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                      ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p],
    "lbm_set_level_launch": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int],
    "lbm_get_level_launch": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lbm_autotune": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p],
    "lbm_block_features": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_plain_targets": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_void_p],
    "lbm_mlp_fit_normalization": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64],
    "lbm_refinement_flags": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)],
    "lbm_get_pdfs": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_set_pdfs": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_lattice": [ctypes.c_void_p, ctypes.c_void_p],
    "lbm_build_leaves": [ctypes.POINTER(ForestDesc), ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
    "lbm_plan_level_stats": [ctypes.POINTER(ForestDesc), ctypes.c_int, ctypes.c_void_p],
    "lbm_probe_copy": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                       ctypes.POINTER(ctypes.c_double)],
    "lbm_probe_streams": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)],
}


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library missing at {path}; build it with `python -m paper_1508_07982_amd.build`")
        lib = ctypes.CDLL(path)
        for name, args in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.lbm_last_error.argtypes = []
        lib.lbm_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != LBM_OK:
        msg = load_library().lbm_last_error().decode(errors="replace")
        raise LBMError(rc, msg)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def lattice():
    e = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19, dtype=np.float64)
    _check(load_library().lbm_lattice(_ptr(e), _ptr(w)))
    return e, w


def _make_desc(roots, n, max_level, leaves, refine, balance, storage, device, stream, periodic=(True, True, True)):
    d = ForestDesc()
    roots = (roots,) * 3 if np.isscalar(roots) else tuple(roots)
    for a in range(3):
        d.root_blocks[a] = int(roots[a])
        d.periodic[a] = int(periodic[a])
    d.cells_per_block = int(n)
    d.max_level = int(max_level)
    keep = []
    if leaves is not None:
        arr = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
        keep.append(arr)
        d.leaves = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.num_leaves = len(arr)
    if refine is not None:
        cb = REFINE_FN(lambda L, x, y, z, user: int(bool(refine(L, x, y, z))))
        keep.append(cb)
        d.refine = cb
    d.balance = int(bool(balance))
    d.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.device = int(device)
    d.stream = ctypes.c_void_p(int(stream)) if stream else None
    return d, keep


def build_leaves(roots, n, max_level, leaves=None, refine=None, balance=True,
                 periodic=(True, True, True)) -> np.ndarray:
    """Host-only: the library's balanced forest, canonical leaf list (N, 4)."""
    d, keep = _make_desc(roots, n, max_level, leaves, refine, balance, "f32", 0, None, periodic)
    count = ctypes.c_int64(0)
    _check(load_library().lbm_build_leaves(ctypes.byref(d), None, 0, ctypes.byref(count)))
    out = np.zeros((count.value, 4), dtype=np.int32)
    _check(load_library().lbm_build_leaves(ctypes.byref(d), _ptr(out), count.value, ctypes.byref(count)))
    del keep
    return out


def plan_level_stats(roots, n, max_level, level, leaves=None, refine=None, balance=True, storage="f32",
                     periodic=(True, True, True)) -> dict:
    """Host-only: layout figures of one level of the forest the library would build."""
    d, keep = _make_desc(roots, n, max_level, leaves, refine, balance, storage, 0, None, periodic)
    out = np.zeros(8, dtype=np.int64)
    _check(load_library().lbm_plan_level_stats(ctypes.byref(d), int(level), _ptr(out)))
    del keep
    return _stats_dict(out)


def _stats_dict(out):
    keys = ("blocks", "coarse_blocks", "interior_cells", "fine_blocks", "work_tiles", "coalesced_pairs",
            "bytes_per_pdf", "cells_per_block")
    return {k: int(v) for k, v in zip(keys, out)}


class Forest:
    """A refined LBM simulation owned by the HIP library."""

    def __init__(self, roots, n, max_level, leaves=None, refine=None, balance=True, storage="f32",
                 device=0, stream=None, periodic=(True, True, True)):
        """periodic: per axis, True for a periodic axis, False for no-slip
        walls at both ends (section 2.2)."""
        self._lib = load_library()
        self.storage = storage
        self.n = int(n)
        d, keep = _make_desc(roots, n, max_level, leaves, refine, balance, storage, device, stream, periodic)
        h = ctypes.c_void_p()
        _check(self._lib.lbm_create_block_forest(ctypes.byref(d), ctypes.byref(h)))
        del keep
        self._h = h
        lv = ctypes.c_int()
        _check(self._lib.lbm_num_levels(self._h, ctypes.byref(lv)))
        self.num_levels = lv.value

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- sizes --------------------------------------------------------------------
    def num_cells(self, level: int = -1) -> int:
        v = ctypes.c_int64()
        _check(self._lib.lbm_num_cells(self._h, int(level), ctypes.byref(v)))
        return v.value

    def num_blocks(self, level: int = -1) -> int:
        v = ctypes.c_int64()
        _check(self._lib.lbm_num_blocks(self._h, int(level), ctypes.byref(v)))
        return v.value

    def leaves(self) -> np.ndarray:
        out = np.zeros((self.num_blocks(-1), 4), dtype=np.int32)
        _check(self._lib.lbm_get_leaves(self._h, _ptr(out)))
        return out

    def level_stats(self, level: int) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(self._lib.lbm_level_stats(self._h, int(level), _ptr(out)))
        return _stats_dict(out)

    def updates_per_coarse_step(self) -> int:
        return sum((2 ** L) * self.num_cells(L) for L in range(self.num_levels))

    # -- parameters and state --------------------------------------------------
    def set_level_omega(self, omega0: float):
        _check(self._lib.lbm_set_level_omega(self._h, float(omega0)))

    def set_trt_force(self, lambda_eo: float = 0.0, accel=None):
        """TRT with Lambda_eo = lambda_eo (0: lambda_o = lambda_e) and the
        level-0 lattice acceleration `accel` (3 values or None); call before
        init_pdfs.  lambda_eo = 0 without acceleration is SRT."""
        a = None if accel is None else np.ascontiguousarray(accel, dtype=np.float64).reshape(3)
        _check(self._lib.lbm_set_trt_force(self._h, float(lambda_eo), _ptr(a) if a is not None else None))

    def level_omega(self, level: int) -> float:
        v = ctypes.c_double()
        _check(self._lib.lbm_get_level_omega(self._h, int(level), ctypes.byref(v)))
        return v.value

    def set_schedule(self, schedule: str):
        _check(self._lib.lbm_set_schedule(self._h, SCHEDULE[schedule]))

    def set_explosion_interpolation(self, on: bool = True):
        """Limited linear reconstruction of exploded values (see the header)."""
        _check(self._lib.lbm_set_explosion_interpolation(self._h, int(bool(on))))

    def set_inplace(self, on: bool = True):
        """In-place (AA pattern) streaming on a forest whose leaves all lie
        on level 0: one PDF buffer instead of two (see the header)."""
        _check(self._lib.lbm_set_inplace(self._h, int(bool(on))))

    def inplace(self) -> bool:
        v = ctypes.c_int()
        _check(self._lib.lbm_get_inplace(self._h, ctypes.byref(v)))
        return bool(v.value)

    def set_coalescence_check(self, on: bool = True):
        _check(self._lib.lbm_set_coalescence_check(self._h, int(bool(on))))

    def set_coalescence_fusion(self, on: bool = True):
        """Every level: the coarser level's coalescence inside the level's
        second-substep launch (on, the default) or in a launch of its own
        (off); results are bitwise equal."""
        _check(self._lib.lbm_set_coalescence_fusion(self._h, int(bool(on))))

    def set_level_fusion(self, level: int, on: int):
        """The same for one level (on = 1, 0, or -1: the forest-wide setting)."""
        _check(self._lib.lbm_set_level_fusion(self._h, int(level), int(on)))

    def get_level_fusion(self, level: int) -> bool:
        v = ctypes.c_int()
        _check(self._lib.lbm_get_level_fusion(self._h, int(level), ctypes.byref(v)))
        return bool(v.value)

    def coalescence_check(self) -> dict:
        """FP64 accumulation-check figures since the last call (reset)."""
        out = np.zeros(3)
        _check(self._lib.lbm_coalescence_check(self._h, _ptr(out)))
        return {"max_abs_dev": float(out[0]), "max_bound_ratio": float(out[1]), "pairs": int(out[2])}

    def set_launch(self, persistent: int):
        _check(self._lib.lbm_set_launch(self._h, int(persistent)))

    def init_pdfs(self, rho, u):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        N = self.num_cells(-1)
        if rho.shape != (N,) or u.shape != (N, 3):
            raise ValueError(f"expected rho ({N},) and u ({N}, 3)")
        _check(self._lib.lbm_init_pdfs(self._h, _ptr(rho), _ptr(u)))

    def step_coarse(self, n_steps: int = 1):
        _check(self._lib.lbm_step_coarse(self._h, int(n_steps)))

    def time_sweeps(self, n_steps: int = 1):
        """Advance n_steps coarse steps with a HIP event pair around every
        sweep launch; returns {(level, substep): (mean ms, launches)}."""
        ms = np.zeros(2 * self.num_levels)
        cnt = np.zeros(2 * self.num_levels, dtype=np.int64)
        _check(self._lib.lbm_time_sweeps(self._h, int(n_steps), _ptr(ms), _ptr(cnt)))
        return {(i // 2, i % 2 + 1): (float(ms[i]), int(cnt[i])) for i in range(2 * self.num_levels) if cnt[i]}

    def time_launches(self, n_steps: int = 1):
        """As time_sweeps, plus {level: (mean ms, launches)} of the
        coalescence launches."""
        nl = self.num_levels
        ms = np.zeros(2 * nl)
        cnt = np.zeros(2 * nl, dtype=np.int64)
        cms = np.zeros(nl)
        ccnt = np.zeros(nl, dtype=np.int64)
        _check(self._lib.lbm_time_launches(self._h, int(n_steps), _ptr(ms), _ptr(cnt), _ptr(cms), _ptr(ccnt)))
        sweeps = {(i // 2, i % 2 + 1): (float(ms[i]), int(cnt[i])) for i in range(2 * nl) if cnt[i]}
        return sweeps, {L: (float(cms[L]), int(ccnt[L])) for L in range(nl) if ccnt[L]}

    def regrid(self, flags):
        """Split (> 0), merge (< 0) or keep (0) every leaf (canonical order)."""
        fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        if fl.shape != (self.num_blocks(-1),):
            raise ValueError("one flag per leaf expected")
        _check(self._lib.lbm_regrid(self._h, _ptr(fl), len(fl)))
        lv = ctypes.c_int()
        _check(self._lib.lbm_num_levels(self._h, ctypes.byref(lv)))
        self.num_levels = lv.value

    def block_indicators(self):
        """(features (nblocks, 12), crit (nblocks, 2) = (I_omega, I_neq))."""
        nb = self.num_blocks(-1)
        feat = np.zeros((nb, 12))
        crit = np.zeros((nb, 2))
        _check(self._lib.lbm_block_indicators(self._h, _ptr(feat), _ptr(crit)))
        return feat, crit

    def set_level_launch(self, level, persistent, order=0, split=1):
        _check(self._lib.lbm_set_level_launch(self._h, int(level), int(persistent), int(order), int(split)))

    def get_level_launch(self, level):
        """(persistent, order, split) of the level's sweep launches."""
        p, o, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.lbm_get_level_launch(self._h, int(level), ctypes.byref(p), ctypes.byref(o),
                                              ctypes.byref(s)))
        return p.value, o.value, s.value

    def autotune(self, n_steps=2, cache=None):
        """Pick each level's launch shape and coalescence fusion by timing;
        returns a list of {level, persistent, order, split, fuse,
        ms_per_level_step}.  With `cache` (a JSON file path) a choice stored
        for the same storage form, block size, level and block count is
        applied without timing, and new results are stored."""
        key = [f"{self.storage}/n{self.n}/L{L}/b{self.num_blocks(L)}" for L in range(self.num_levels)]
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if cache and all(k in table and "fuse" in table[k] for k in key):
            out = []
            for L, k in enumerate(key):
                e = table[k]
                self.set_level_launch(L, e["persistent"], e["order"], e["split"])
                self.set_level_fusion(L, e["fuse"])
                out.append(dict(e, level=L, cached=True))
            return out
        res = np.zeros(5 * self.num_levels)
        _check(self._lib.lbm_autotune(self._h, int(n_steps), _ptr(res)))
        out = [{"level": L, "persistent": int(res[5 * L]), "order": int(res[5 * L + 1]), "split": int(res[5 * L + 2]),
                "fuse": int(res[5 * L + 3]), "ms_per_level_step": float(res[5 * L + 4])} for L in range(self.num_levels)]
        if cache:
            for L, k in enumerate(key):
                table[k] = {c: out[L][c] for c in ("persistent", "order", "split", "fuse", "ms_per_level_step")}
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
        return out

    def block_features(self):
        """Features (nblocks, 12) from the fused single-pass kernel."""
        feat = np.zeros((self.num_blocks(-1), 12))
        _check(self._lib.lbm_block_features(self._h, _ptr(feat)))
        return feat

    def refinement_flags(self, theta_omega, theta_neq, mlp=None, delta=0.05):
        """Regrid flags per block from the criterion (mlp None) or the MLP;
        returns (flags, number of blocks decided by the fallback)."""
        flags = np.zeros(self.num_blocks(-1), dtype=np.int8)
        fb = ctypes.c_int32(0)
        _check(self._lib.lbm_refinement_flags(self._h, mlp._h if mlp is not None else None, float(theta_omega),
                                              float(theta_neq), float(delta), _ptr(flags), ctypes.byref(fb)))
        return flags, fb.value

    def synchronize(self):
        _check(self._lib.lbm_synchronize(self._h))

    def moments(self):
        N = self.num_cells(-1)
        rho = np.empty(N)
        u = np.empty((N, 3))
        _check(self._lib.lbm_get_moments(self._h, _ptr(rho), _ptr(u)))
        return rho, u

    def moments_static(self):
        """As moments(), through lbm_get_moments_static (no device
        allocation; calls overlapping on one device race)."""
        N = self.num_cells(-1)
        rho = np.empty(N)
        u = np.empty((N, 3))
        _check(self._lib.lbm_get_moments_static(self._h, _ptr(rho), _ptr(u)))
        return rho, u

    def mass(self):
        m = ctypes.c_double()
        j = np.zeros(3)
        _check(self._lib.lbm_mass(self._h, ctypes.byref(m), _ptr(j)))
        return m.value, j

    def get_pdfs(self) -> np.ndarray:
        h = np.empty((self.num_cells(-1), 19))
        _check(self._lib.lbm_get_pdfs(self._h, _ptr(h)))
        return h

    def set_pdfs(self, h):
        h = np.ascontiguousarray(h, dtype=np.float64)
        if h.shape != (self.num_cells(-1), 19):
            raise ValueError("expected (num_cells, 19)")
        _check(self._lib.lbm_set_pdfs(self._h, _ptr(h)))


def plain_targets(crit, theta_omega, theta_neq) -> np.ndarray:
    """Soft targets of the criterion: 1 refine-worthy, 0 coarsen-worthy, 0.5 keep."""
    crit = np.ascontiguousarray(crit, dtype=np.float64).reshape(-1, 2)
    t = np.zeros(len(crit))
    _check(load_library().lbm_plain_targets(_ptr(crit), len(crit), float(theta_omega), float(theta_neq), _ptr(t)))
    return t


class MLP:
    """The refinement surrogate 12 -> 64 -> 64 -> 1 owned by the HIP library."""

    def __init__(self, seed: int = 0, device: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib.lbm_mlp_create(int(device), int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int()
        _check(self._lib.lbm_mlp_num_params(ctypes.byref(n)))
        self.num_params = n.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        p = np.zeros(self.num_params, dtype=np.float32)
        _check(self._lib.lbm_mlp_get_params(self._h, _ptr(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(self._lib.lbm_mlp_set_params(self._h, _ptr(p)))

    def set_normalization(self, mean, std, fmin=None, fmax=None):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None for a in (mean, std, fmin, fmax)]
        _check(self._lib.lbm_mlp_set_normalization(self._h, *[_ptr(a) if a is not None else None for a in arrs]))

    def fit_normalization(self, X):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 12)
        _check(self._lib.lbm_mlp_fit_normalization(self._h, _ptr(X), len(X)))

    def predict(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 12)
        p = np.zeros(len(X), dtype=np.float32)
        _check(self._lib.lbm_mlp_predict(self._h, _ptr(X), len(X), _ptr(p)))
        return p

    def gradient(self, X, t) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 12)
        t = np.ascontiguousarray(t, dtype=np.float64)
        g = np.zeros(self.num_params, dtype=np.float32)
        _check(self._lib.lbm_mlp_gradient(self._h, _ptr(X), _ptr(t), len(X), _ptr(g)))
        return g

    def train(self, X, t, epochs=20, batch=256, lr=1e-3, seed=0) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 12)
        t = np.ascontiguousarray(t, dtype=np.float64)
        losses = np.zeros(max(epochs, 1))
        _check(self._lib.lbm_mlp_train(self._h, _ptr(X), _ptr(t), len(X), int(epochs), int(batch), float(lr),
                                       int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(losses)))
        return losses[:epochs]


def device_memory(device: int = 0):
    """(free bytes, total bytes) of a device (hipMemGetInfo)."""
    lib = load_library()
    fr, tot = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.lbm_device_memory(int(device), ctypes.byref(fr), ctypes.byref(tot)))
    return fr.value, tot.value


# ---- bandwidth probes (lbm_probe.h) ------------------------------------------

def probe_copy(dst_ptr: int, src_ptr: int, nbytes: int, iters: int = 5, nontemporal: bool = True,
               stream: int = 0) -> float:
    """Mean time in ms of a 16-byte-vector device copy of nbytes between two
    caller-owned device buffers (raw device addresses)."""
    lib = load_library()
    ms = ctypes.c_double()
    _check(lib.lbm_probe_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(nbytes), int(iters),
                              int(bool(nontemporal)), ctypes.c_void_p(stream or None), ctypes.byref(ms)))
    return ms.value


def probe_streams(dst_ptr: int, src_ptr: int, nblocks: int, n: int, elem_bytes: int, lanes: int = 256,
                  xcd: bool = False, iters: int = 5, stream: int = 0) -> float:
    """Mean launch time in ms of the sweep's access shape without arithmetic
    over nblocks blocks of 19 rows of n^3 elements (both buffers must hold
    nblocks * 19 * n^3 * elem_bytes bytes)."""
    lib = load_library()
    ms = ctypes.c_double()
    _check(lib.lbm_probe_streams(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(nblocks), int(n),
                                 int(elem_bytes), int(lanes), int(bool(xcd)), int(iters),
                                 ctypes.c_void_p(stream or None), ctypes.byref(ms)))
    return ms.value
