"""ctypes front end of the plain-C SEEDS oracle (``seeds_oracle.c``).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package. The product path
(``paper_1309_3848_amd``) never does.

The oracle is single-threaded C built with gcc; ``build()`` compiles it into
``oracle/libseeds_oracle.so``, and the same source with ``-fopenmp`` into
``oracle/libseeds_oracle_omp.so`` (the all-core CPU baseline: the units of a
phase are decided in parallel; results are identical to the serial build).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "seeds_oracle.c")
LIB = os.path.join(HERE, "libseeds_oracle.so")
LIB_OMP = os.path.join(HERE, "libseeds_oracle_omp.so")

RULE_INTERSECT = 0
RULE_EXACT = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no vector intrinsics), serial and
    all-core (-fopenmp) builds."""
    for lib_path, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(SRC):
            tmp = lib_path + ".tmp"
            subprocess.run(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-Wall", "-Wextra",
                            "-Wno-unknown-pragmas", *extra, "-o", tmp, SRC], check=True)
            os.replace(tmp, lib_path)
    return LIB


class Decision(ctypes.Structure):
    _fields_ = [("ux", ctypes.c_int32), ("uy", ctypes.c_int32), ("k", ctypes.c_int32),
                ("boundary", ctypes.c_int32), ("connect_ok", ctypes.c_int32),
                ("n", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("dropped", ctypes.c_int32), ("gain", ctypes.c_int64),
                ("aux", ctypes.c_int64), ("an", ctypes.c_int64), ("akl", ctypes.c_int64)]


_lib = None


def load(path: str) -> ctypes.CDLL:
    """Load an oracle build (the default one, or a variant built by a test)."""
    L = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.oracle_grid.argtypes = [I32, I32, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.oracle_grid.restype = I32
    L.oracle_quantise.argtypes = [P, I32, I32, I64, I32, P]
    L.oracle_create.argtypes = [P, I32, I32, I64, I32, I32, I32, I32, I32, I32]
    L.oracle_create.restype = P
    L.oracle_free.argtypes = [P]
    L.oracle_set_pixel_labels.argtypes = [P, P]
    L.oracle_set_pixel_labels.restype = I32
    L.oracle_next_phase.argtypes = [P]
    L.oracle_next_phase.restype = I32
    L.oracle_warm_start.argtypes = [P, P, ctypes.c_int64]
    L.oracle_warm_start.restype = I32
    L.oracle_set_unit_labels.argtypes = [P, I32, P]
    L.oracle_set_unit_labels.restype = I32
    L.oracle_decide_class.argtypes = [P, I32, P, I32]
    L.oracle_decide_class.restype = I32
    L.oracle_phase.argtypes = [P, I32]
    L.oracle_phase.restype = I32
    L.oracle_run.argtypes = [P, I32]
    L.oracle_run.restype = I32
    L.oracle_run_sequential.argtypes = [P]
    for f in ("oracle_num_superpixels", "oracle_level", "oracle_invalid_superpixels"):
        getattr(L, f).argtypes = [P]
        getattr(L, f).restype = I32
    L.oracle_unit_grid.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.oracle_grid_dims.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.oracle_unit_labels.argtypes = [P, P]
    L.oracle_pixel_labels.argtypes = [P, P]
    L.oracle_bins.argtypes = [P, P]
    L.oracle_histograms.argtypes = [P, P, P]
    L.oracle_energy.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.oracle_seeds.argtypes = [P, I32, I32, I64, I32, I32, I32, I32, I32, I32, I32, P, P, P]
    L.oracle_seeds.restype = I32
    L.oracle_quality.argtypes = [P, P, I32, I32, I32, I32, I32, P]
    L.oracle_quality.restype = I32
    L.oracle_threads.argtypes = []
    L.oracle_threads.restype = I32
    return L


def lib() -> ctypes.CDLL:
    """The oracle build. SEEDS_ORACLE_LIB may name another build of the same
    source (the mutation tests use it to plant mistakes)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("SEEDS_ORACLE_LIB")
        if alt:
            _lib = load(alt)
            return _lib
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = load(LIB)
    return _lib


_lib_omp = None


def lib_omp() -> ctypes.CDLL:
    """The all-core build (OpenMP over the units of a phase; threads from
    OMP_NUM_THREADS)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(LIB_OMP) or os.path.getmtime(LIB_OMP) < os.path.getmtime(SRC):
            build(force=True)
        _lib_omp = load(LIB_OMP)
    return _lib_omp


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def grid(H: int, W: int, K: int, L: int, cdll: ctypes.CDLL | None = None):
    """Superpixel grid (gx, gy) or None when the parameters are refused."""
    gx, gy = ctypes.c_int(), ctypes.c_int()
    if (cdll or lib()).oracle_grid(H, W, K, L, ctypes.byref(gx), ctypes.byref(gy)) != 0:
        return None
    return gx.value, gy.value


def quantise(rgb: np.ndarray, B: int, cdll: ctypes.CDLL | None = None) -> np.ndarray:
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    H, W, _ = rgb.shape
    out = np.empty((H, W), np.uint8)
    (cdll or lib()).oracle_quantise(_ptr(rgb), H, W, W * 3, B, _ptr(out))
    return out


class Oracle:
    """One image's oracle state: grid init, schedule cursor, histograms."""

    def __init__(self, rgb: np.ndarray, K: int, levels: int, bins: int = 5, iters: int = 4,
                 gamma: int = 1, rule: int = RULE_INTERSECT, cdll: ctypes.CDLL | None = None):
        self._L = cdll if cdll is not None else lib()
        self._rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        self.H, self.W, _ = self._rgb.shape
        self.B = bins
        self.nbins = bins ** 3
        h = self._L.oracle_create(_ptr(self._rgb), self.H, self.W, self.W * 3, K, levels, bins,
                                iters, gamma, rule)
        if not h:
            raise ValueError("oracle refused the parameters")
        self._h = ctypes.c_void_p(h)
        self.K = self._L.oracle_num_superpixels(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._L.oracle_free(h)
            self._h = None

    # -- schedule -------------------------------------------------------
    def run(self, max_phases: int = -1) -> int:
        return self._L.oracle_run(self._h, max_phases)

    def run_sequential(self) -> None:
        self._L.oracle_run_sequential(self._h)

    def phase(self, cls: int) -> int:
        return self._L.oracle_phase(self._h, cls)

    def next_phase(self) -> int:
        """Class of the next phase (state brought to its level), or -1."""
        return self._L.oracle_next_phase(self._h)

    def decide(self, cls: int):
        n = self._L.oracle_decide_class(self._h, cls, None, 0)
        arr = (Decision * max(n, 1))()
        self._L.oracle_decide_class(self._h, cls, arr, n)
        return [arr[i] for i in range(n)]

    def set_pixel_labels(self, labels: np.ndarray) -> None:
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        assert lab.shape == (self.H, self.W)
        if self._L.oracle_set_pixel_labels(self._h, _ptr(lab)) != 0:
            raise ValueError("label out of range")

    def warm_start(self, rgb: np.ndarray) -> None:
        """Next frame of a stream: keep the pixel labels, bin the new frame,
        recount; the next run() does I pixel sweeps."""
        img = np.ascontiguousarray(rgb, dtype=np.uint8)
        assert img.shape == (self.H, self.W, 3)
        if self._L.oracle_warm_start(self._h, _ptr(img), self.W * 3) != 0:
            raise ValueError("warm start needs a state at pixel level")

    def set_unit_labels(self, level: int, labels: np.ndarray) -> None:
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        s = 1 << level
        assert lab.shape == (-(-self.H // s), -(-self.W // s))
        if self._L.oracle_set_unit_labels(self._h, level, _ptr(lab)) != 0:
            raise ValueError("bad level or label")

    # -- state ----------------------------------------------------------
    @property
    def level(self) -> int:
        return self._L.oracle_level(self._h)

    @property
    def grid_dims(self):
        gx, gy = ctypes.c_int(), ctypes.c_int()
        self._L.oracle_grid_dims(self._h, ctypes.byref(gx), ctypes.byref(gy))
        return gx.value, gy.value

    def unit_labels(self) -> np.ndarray:
        uw, uh = ctypes.c_int(), ctypes.c_int()
        self._L.oracle_unit_grid(self._h, ctypes.byref(uw), ctypes.byref(uh))
        out = np.empty((uh.value, uw.value), np.int32)
        self._L.oracle_unit_labels(self._h, _ptr(out))
        return out

    def labels(self) -> np.ndarray:
        out = np.empty((self.H, self.W), np.int32)
        self._L.oracle_pixel_labels(self._h, _ptr(out))
        return out

    def bins(self) -> np.ndarray:
        out = np.empty((self.H, self.W), np.uint8)
        self._L.oracle_bins(self._h, _ptr(out))
        return out

    def histograms(self):
        hist = np.empty((self.K, self.nbins), np.int64)
        size = np.empty((self.K,), np.int64)
        self._L.oracle_histograms(self._h, _ptr(hist), _ptr(size))
        return hist, size

    def energy(self):
        Hc, Gc = ctypes.c_int64(), ctypes.c_int64()
        self._L.oracle_energy(self._h, ctypes.byref(Hc), ctypes.byref(Gc))
        return Hc.value, Gc.value

    def invalid_superpixels(self) -> int:
        return self._L.oracle_invalid_superpixels(self._h)


def seeds(rgb: np.ndarray, K: int, levels: int, bins: int = 5, iters: int = 4, gamma: int = 1,
          rule: int = RULE_INTERSECT, max_phases: int = -1, cdll: ctypes.CDLL | None = None):
    """One-shot oracle run: (labels HxW int32, hist Kx(B^3) int64, size K int64)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    H, W, _ = rgb.shape
    L = cdll or lib()
    gd = grid(H, W, K, levels, L)
    if gd is None:
        raise ValueError("oracle refused the parameters")
    Keff = gd[0] * gd[1]
    labels = np.empty((H, W), np.int32)
    hist = np.empty((Keff, bins ** 3), np.int64)
    size = np.empty((Keff,), np.int64)
    k = L.oracle_seeds(_ptr(rgb), H, W, W * 3, K, levels, bins, iters, gamma, rule,
                           max_phases, _ptr(labels), _ptr(hist), _ptr(size))
    if k < 0:
        raise ValueError("oracle refused the parameters")
    return labels, hist, size


def quality(labels: np.ndarray, truth: np.ndarray, K: int, R: int, eps: int = 2,
            cdll: ctypes.CDLL | None = None) -> dict:
    """Quality metrics of Sec. 6.1 as integer numerators (see oracle_quality):
    keys N, ue, asa, cue, br_hits, br_total."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    gt = np.ascontiguousarray(truth, dtype=np.int32)
    assert lab.shape == gt.shape and lab.ndim == 2
    out = np.zeros(6, np.int64)
    L = cdll or lib()
    if L.oracle_quality(_ptr(lab), _ptr(gt), lab.shape[0], lab.shape[1], K, R, eps, _ptr(out)) != 0:
        raise ValueError("label or segment out of range")
    return dict(zip(["N", "ue", "asa", "cue", "br_hits", "br_total"], (int(v) for v in out)))
