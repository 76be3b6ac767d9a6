"""ctypes driver for the oracle's C walk (walk.c).  Test infrastructure only.

Derives the medium coefficients from the optical depth (Eq. 1: OD = mu_ext l,
with l the cuboid's extent along the beam) and the albedo, then runs the FP64
walk over photon ranges split across host threads.  Each chunk fills its own
images; chunks are summed in chunk order, so a result depends only on the
chunk count, never on thread timing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import build as _build
from . import mie as _mie
from . import poly as _poly

N_SCALARS = 16
S = dict(face=slice(0, 6), absorbed=6, roulette_net=7, capped_w=8, events=9, photons=10,
         roulette_kills=11, capped=12, reflections=13, steps=14)
IREC_FIELDS = ("face", "cause", "k", "steps")
FREC_FIELDS = ("px", "py", "pz", "dx", "dy", "dz", "w", "L", "A")


class _Params(C.Structure):
    _fields_ = [("size", C.c_double * 3), ("n_med", C.c_double), ("n_out", C.c_double),
                ("mu_t", C.c_double), ("albedo", C.c_double),
                ("src_pos", C.c_double * 3), ("src_dir", C.c_double * 3),
                ("phase", C.c_int32), ("n_table", C.c_int32),
                ("table", C.POINTER(C.c_double)), ("g", C.c_double),
                ("seed", C.c_uint64), ("instance", C.c_uint32), ("max_steps", C.c_uint32),
                ("roulette_w", C.c_double), ("roulette_p", C.c_double),
                ("side_nx", C.c_int32), ("side_ny", C.c_int32),
                ("trans_nx", C.c_int32), ("trans_ny", C.c_int32), ("beam_radius", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        L.oracle_simulate.restype = C.c_int
        L.oracle_simulate.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_uint64, C.c_uint64,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_fresnel.restype = C.c_double
        L.oracle_fresnel.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_sample_v.restype = C.c_double
        L.oracle_sample_v.argtypes = [C.POINTER(_Params), C.c_double]
        L.oracle_rotate.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double]
        L.oracle_params_size.restype = C.c_size_t
        assert L.oracle_params_size() == C.sizeof(_Params), "oracle_params layout mismatch"
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class OracleResult:
    side: np.ndarray
    trans: np.ndarray
    side_w2: np.ndarray
    trans_w2: np.ndarray
    scalars: np.ndarray
    irec: Optional[np.ndarray] = None     # (4, n) int32
    frec: Optional[np.ndarray] = None     # (9, n) float64
    seconds: float = 0.0
    threads: int = 1

    def rec(self, name):
        if name in IREC_FIELDS:
            return self.irec[IREC_FIELDS.index(name)]
        return self.frec[FREC_FIELDS.index(name)]


class Walk:
    """Oracle walk for one medium.  ``table`` is an oracle MieTable."""

    def __init__(self, workload, table: Optional[_mie.MieTable] = None, *, g: Optional[float] = None,
                 table_v: Optional[np.ndarray] = None):
        w = workload
        self.w = w
        if table is None and table_v is None and (w.phase == 0 or g is None):
            table = (_poly.poly_table_from_workload(w) if getattr(w.particle, "n_bins", 1) > 1
                     else _mie.table_from_workload(w))
        self.table = table
        v = table_v if table_v is not None else (self.table.v if self.table is not None else np.zeros(2))
        self._v = np.ascontiguousarray(v, dtype=np.float64)
        p = _Params()
        for i in range(3):
            p.size[i] = w.size_mm[i]
            p.src_pos[i] = w.src_pos_mm[i]
            p.src_dir[i] = w.src_dir[i]
        p.n_med = w.particle.n_medium
        p.n_out = w.n_outside
        # Eq. 1: OD = mu_ext * l along the beam (z extent).
        p.mu_t = w.tau / w.size_mm[2]
        p.beam_radius = getattr(w, "beam_radius_mm", 0.0)
        p.albedo = w.albedo
        p.phase = w.phase
        p.n_table = len(self._v)
        p.table = self._v.ctypes.data_as(C.POINTER(C.c_double))
        if g is not None:
            p.g = g
        elif self.table is not None:
            p.g = self.table.g
        else:
            p.g = 0.0
        p.seed = w.seed
        p.instance = w.instance
        p.max_steps = w.max_steps
        p.roulette_w = w.roulette_w
        p.roulette_p = w.roulette_p
        p.side_nx = p.side_ny = w.side_px
        p.trans_nx = p.trans_ny = w.trans_px
        self.p = p

    def run(self, n_photons: Optional[int] = None, photon_offset: int = 0, ids: Optional[np.ndarray] = None,
            records: bool = False, threads: Optional[int] = None, chunks: Optional[int] = None) -> OracleResult:
        L = lib()
        w = self.w
        if ids is not None:
            ids = np.ascontiguousarray(ids, dtype=np.uint64)
            n = len(ids)
        else:
            n = w.n_photons if n_photons is None else n_photons
        threads = threads or min(os.cpu_count() or 1, 16)
        nchunk = chunks or threads
        nchunk = max(1, min(nchunk, max(n, 1)))
        bounds = [n * c // nchunk for c in range(nchunk + 1)]
        sy, sx = w.side_px, w.side_px
        ty, tx = w.trans_px, w.trans_px
        irec = np.zeros((4, n), dtype=np.int32) if records else None
        frec = np.zeros((9, n), dtype=np.float64) if records else None

        def job(c):
            lo, hi = bounds[c], bounds[c + 1]
            m = hi - lo
            out = dict(side=np.zeros((sy, sx)), trans=np.zeros((ty, tx)), side_w2=np.zeros((sy, sx)),
                       trans_w2=np.zeros((ty, tx)), scal=np.zeros(N_SCALARS))
            ir = np.zeros((4, m), dtype=np.int32) if records else None
            fr = np.zeros((9, m), dtype=np.float64) if records else None
            id_arr = ids[lo:hi] if ids is not None else None
            rc = L.oracle_simulate(C.byref(self.p), _ptr(id_arr), photon_offset + lo, m,
                                   _ptr(out["side"]), _ptr(out["trans"]), _ptr(out["side_w2"]),
                                   _ptr(out["trans_w2"]), _ptr(out["scal"]), _ptr(ir), _ptr(fr))
            if rc != 0:
                raise ValueError("oracle_simulate rejected its parameters")
            if records:
                irec[:, lo:hi] = ir
                frec[:, lo:hi] = fr
            return out

        t0 = time.perf_counter()
        if threads == 1 or nchunk == 1:
            outs = [job(c) for c in range(nchunk)]
        else:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                outs = list(ex.map(job, range(nchunk)))
        dt = time.perf_counter() - t0
        res = OracleResult(np.zeros((sy, sx)), np.zeros((ty, tx)), np.zeros((sy, sx)),
                           np.zeros((ty, tx)), np.zeros(N_SCALARS), irec, frec, dt, threads)
        for o in outs:      # fixed chunk order
            res.side += o["side"]
            res.trans += o["trans"]
            res.side_w2 += o["side_w2"]
            res.trans_w2 += o["trans_w2"]
            res.scalars += o["scal"]
        return res

    # Single-function probes of the walk's pieces, for the pins.
    def sample_v(self, u: float) -> float:
        return lib().oracle_sample_v(C.byref(self.p), float(u))


def philox_c(ctr, key):
    L = lib()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    L.oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(v) for v in out)


def fresnel(cos_i: float, n1: float, n2: float) -> float:
    return lib().oracle_fresnel(cos_i, n1, n2)


def rotate(d, cos_t, sin_t, cos_p, sin_p) -> np.ndarray:
    a = np.ascontiguousarray(d, dtype=np.float64).copy()
    lib().oracle_rotate(_ptr(a), cos_t, sin_t, cos_p, sin_p)
    return a
