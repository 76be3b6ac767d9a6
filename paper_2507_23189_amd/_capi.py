"""ctypes binding of libmcmie.so (include/mcmie.h).  Argument marshalling only:
every computation happens in the library's HIP kernels.  Device buffers are
torch tensors; work is enqueued on torch's current HIP stream."""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcmie.so")

MC_OK, MC_EINVAL, MC_EDEVICE, MC_ENOMEM, MC_EUNSUPPORTED = 0, -1, -2, -3, -4
MC_PHASE_MIE, MC_PHASE_HG = 0, 1
MC_MEDIUM_TAU, MC_MEDIUM_MU, MC_MEDIUM_CONCENTRATION = 0, 1, 2
MC_ACCUMULATE, MC_SIGMA, MC_RECORD, MC_FIX64, MC_MOMENTS, MC_MOMENTS_PIXEL2 = 1, 2, 4, 8, 16, 32
MC_EXIT_LOG = 64
MC_NOALLOC_SCRATCH_BYTES = 8 * (32 + (1 << 21))
MC_N_SCALARS = 20
MC_S_FACE, MC_S_ABSORBED, MC_S_ROULETTE_NET, MC_S_CAPPED_W, MC_S_EVENTS = 0, 6, 7, 8, 9
MC_S_PHOTONS, MC_S_ROULETTE_KILLS, MC_S_CAPPED, MC_S_REFLECTIONS, MC_S_STEPS, MC_S_RESERVED = 10, 11, 12, 13, 14, 15
MC_S_SIDE_W2, MC_S_SIDE_W2K, MC_S_SIDE_W2L = 16, 17, 18
MC_REC_I_N, MC_REC_F_N = 4, 9
MC_MAX_N_CDF, MC_MAX_N_ANGLES, MC_MAX_TERMS = 16384, 3001, 1024
MC_MAX_BATCH = 512
MC_MAX_BINS = 64
MC_METRICS_N, MC_MAX_ANNULI = 12, 2048
# Candidates mc_autotune_batch times, in its block-major order.
AUTOTUNE_BLOCKS, AUTOTUNE_CHUNKS = (256, 512, 1024), (256, 512, 1024, 2048, 4096)


class MieSpec(C.Structure):
    _fields_ = [("n_medium", C.c_double), ("m_re", C.c_double), ("m_im", C.c_double),
                ("diameter_um", C.c_double), ("wavelength_nm", C.c_double),
                ("n_angles", C.c_int32), ("n_cdf", C.c_int32)]


class _MieTableC(C.Structure):
    _fields_ = [("x", C.c_double), ("m_rel_re", C.c_double), ("m_rel_im", C.c_double),
                ("q_ext", C.c_double), ("q_sca", C.c_double), ("q_abs", C.c_double), ("g", C.c_double),
                ("sigma_ext_mm2", C.c_double), ("sigma_sca_mm2", C.c_double), ("sigma_abs_mm2", C.c_double),
                ("n_terms", C.c_int32), ("n_cdf", C.c_int32),
                ("inv_cdf", C.c_void_p), ("phase", C.c_void_p), ("cdf", C.c_void_p), ("coef", C.c_void_p),
                ("coef_capacity", C.c_int32), ("result", C.c_void_p), ("work", C.c_void_p)]


class MiePoly(C.Structure):
    """Lognormal size distribution of mie_table_build_poly (mie_poly_t)."""
    _fields_ = [("sigma_ln", C.c_double), ("n_bins", C.c_int32), ("reserved", C.c_int32),
                ("work", C.c_void_p), ("work_bytes", C.c_uint64)]


class Radial(C.Structure):
    """Centre (column, row) and outer radius in pixels of the radial analysis (mc_radial_t)."""
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("r_max", C.c_double)]


class Medium(C.Structure):
    """mc_medium_t: `input` selects tau + albedo, mu_sca + mu_abs, or a
    particle concentration with the cross-sections (MC_MEDIUM_*)."""
    _fields_ = [("input", C.c_int32), ("phase", C.c_int32), ("tau", C.c_double), ("albedo", C.c_double),
                ("mu_sca", C.c_double), ("mu_abs", C.c_double), ("concentration_per_mm3", C.c_double),
                ("mu_abs_host", C.c_double), ("n_cdf", C.c_int32), ("reserved", C.c_int32),
                ("inv_cdf", C.c_void_p), ("g", C.c_double), ("sigma_sca_mm2", C.c_double),
                ("sigma_abs_mm2", C.c_double)]


class Source(C.Structure):
    _fields_ = [("pos_mm", C.c_double * 3), ("dir", C.c_double * 3), ("beam_radius_mm", C.c_double)]


class Geometry(C.Structure):
    _fields_ = [("size_mm", C.c_double * 3), ("n_medium", C.c_double), ("n_outside", C.c_double)]


class Detector(C.Structure):
    _fields_ = [("side_nx", C.c_int32), ("side_ny", C.c_int32), ("trans_nx", C.c_int32),
                ("trans_ny", C.c_int32), ("flags", C.c_uint32)]


class Run(C.Structure):
    _fields_ = [("n_photons", C.c_uint64), ("photon_offset", C.c_uint64), ("seed", C.c_uint64),
                ("instance", C.c_uint32), ("max_steps", C.c_uint32), ("roulette_w", C.c_double),
                ("roulette_p", C.c_double), ("record_stride", C.c_uint64), ("block_size", C.c_int32),
                ("grid_blocks", C.c_int32), ("chunk", C.c_uint32), ("reserved", C.c_uint32),
                ("walk_events", C.c_void_p * 2), ("sim_events", C.c_void_p * 2)]

    def time_walk(self, start, end):
        """Have the library set torch.cuda.Events `start` and `end` to the
        start and end of the walk kernel (None, None: stop)."""
        self._set_events(self.walk_events, start, end)

    def time_sim(self, start, end):
        """Have the library set torch.cuda.Events `start` and `end` to the
        start of the call's first kernel and the end of its last (None, None:
        stop)."""
        self._set_events(self.sim_events, start, end)

    @staticmethod
    def _set_events(slots, start, end):
        for i, ev in enumerate((start, end)):
            if ev is None:
                slots[i] = None
                continue
            if not ev.cuda_event:
                ev.record()      # creates the underlying event
            slots[i] = ev.cuda_event


class BatchItem(C.Structure):
    """One medium of mc_simulate_batch (mc_batch_item_t)."""
    _fields_ = [("tau", C.c_double), ("albedo", C.c_double), ("inv_cdf", C.c_void_p), ("n_photons", C.c_uint64),
                ("instance", C.c_uint32), ("reserved", C.c_uint32)]


class _TallyC(C.Structure):
    _fields_ = [("side", C.c_void_p), ("trans", C.c_void_p), ("side_w2", C.c_void_p),
                ("trans_w2", C.c_void_p), ("scalars", C.c_void_p), ("rec_i", C.c_void_p),
                ("rec_f", C.c_void_p), ("rec_rows", C.c_uint64), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_uint64), ("side_wk", C.c_void_p), ("side_wl", C.c_void_p),
                ("side_w2k", C.c_void_p), ("side_w2l", C.c_void_p)]


class McError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded HIP library.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_23189_amd.build` "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        L.mie_table_build.argtypes = [C.POINTER(MieSpec), C.POINTER(_MieTableC), C.c_void_p]
        L.mie_table_enqueue.argtypes = [C.POINTER(MieSpec), C.POINTER(_MieTableC), C.c_void_p]
        L.mc_simulate.argtypes = [C.POINTER(Medium), C.POINTER(Source), C.POINTER(Geometry),
                                  C.POINTER(Detector), C.POINTER(Run), C.POINTER(_TallyC), C.c_void_p]
        L.mc_simulate_noalloc.argtypes = [C.POINTER(Medium), C.POINTER(Source), C.POINTER(Geometry),
                                          C.POINTER(Detector), C.POINTER(Run), C.POINTER(_TallyC), C.c_void_p]
        L.mc_grad.argtypes = [C.POINTER(Medium), C.POINTER(Geometry), C.POINTER(Detector), C.POINTER(_TallyC),
                              C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_double), C.c_void_p]
        L.mc_philox_blocks.argtypes = [C.c_uint64, C.c_uint32, C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32,
                                       C.c_void_p, C.c_void_p]
        L.mie_table_build_poly.argtypes = [C.POINTER(MieSpec), C.POINTER(MiePoly), C.POINTER(_MieTableC),
                                           C.c_void_p]
        L.mie_poly_work_bytes.argtypes = [C.POINTER(MieSpec), C.POINTER(MiePoly)]
        L.mie_poly_work_bytes.restype = C.c_uint64
        L.mc_lognormal_bins.argtypes = [C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.mc_metrics_work_bytes.argtypes = [C.c_int32, C.c_int32, C.POINTER(Radial)]
        L.mc_metrics_work_bytes.restype = C.c_uint64
        L.mc_image_metrics.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Radial),
                                       C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_double), C.c_void_p]
        L.mc_medium_coefficients.argtypes = [C.POINTER(Medium), C.POINTER(Geometry), C.POINTER(C.c_double)]
        L.mc_workspace_bytes.argtypes = [C.POINTER(Detector)]
        L.mc_workspace_bytes.restype = C.c_uint64
        L.mc_workspace_bytes_batch.argtypes = [C.POINTER(Detector), C.c_uint32]
        L.mc_workspace_bytes_batch.restype = C.c_uint64
        L.mc_workspace_bytes_batch_log.argtypes = [C.POINTER(Detector), C.c_uint32, C.c_uint64]
        L.mc_workspace_bytes_batch_log.restype = C.c_uint64
        L.mc_workspace_bytes_log.argtypes = [C.POINTER(Detector), C.c_uint64]
        L.mc_workspace_bytes_log.restype = C.c_uint64
        _batch_args = [C.POINTER(BatchItem), C.c_uint32, C.c_int32, C.POINTER(Source), C.POINTER(Geometry),
                       C.POINTER(Detector), C.POINTER(Run), C.POINTER(_TallyC)]
        L.mc_simulate_batch.argtypes = _batch_args + [C.c_void_p]
        L.mc_autotune_batch.argtypes = _batch_args + [C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_uint32),
                                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]
        L.mc_last_error.restype = C.c_char_p
        L.mc_version.restype = C.c_int
        for f in ("mie_table_build", "mie_table_enqueue", "mc_simulate", "mc_simulate_noalloc", "mc_grad", "mc_philox_blocks",
                  "mc_simulate_batch", "mc_autotune_batch", "mie_table_build_poly", "mc_lognormal_bins",
                  "mc_image_metrics", "mc_medium_coefficients"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != MC_OK:
        raise McError(rc, lib().mc_last_error().decode())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _require(t, name: str, dtypes, *, numel=None, min_numel=None, shape=None, optional=False):
    """Refuse, before any library call, a buffer the kernels would read or
    write out of bounds: it must be a contiguous tensor of one of `dtypes`
    with the stated element count or shape.  Raises ValueError; returns the
    tensor (None for an absent optional one).  Where it lives is checked
    afterwards, for all buffers of a call at once, by _on_one_gpu."""
    import torch
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if not isinstance(dtypes, (tuple, list)):
        dtypes = (dtypes,)
    if t.dtype not in dtypes:
        raise ValueError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} must hold at least {min_numel} elements, got {t.numel()}")
    return t


def _on_one_gpu(**named):
    """Every given tensor (None skipped) lives on the same GPU; returns it."""
    dev = None
    for name, t in named.items():
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError(f"{name} must be on a GPU, got {t.device}")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{name} is on {t.device}, other buffers of the call on {dev}")
    return dev


@dataclass
class MieTable:
    """Host scalars and device tensors written by mie_table_build."""
    x: float
    m_rel: complex
    q_ext: float
    q_sca: float
    q_abs: float
    g: float
    sigma_ext_mm2: float
    sigma_sca_mm2: float
    sigma_abs_mm2: float
    n_terms: int
    inv_cdf: "object"              # torch float32 (n_cdf,)
    phase: "object" = None         # torch float64 (n_angles,)
    cdf: "object" = None           # torch float64 (n_angles,)
    coef: "object" = None          # torch float64 (n_terms, 4): Re a, Im a, Re b, Im b
    result: "object" = None        # torch float64 (4,): Q_ext, Q_sca, g, n_terms (device)
    work: "object" = None          # torch float64 (n_angles,): the enqueued build's angle grid (kept alive here)


def mie_table_build(spec: MieSpec, device="cuda", *, phase=False, cdf=False, coef=False,
                    stream=None) -> MieTable:
    """Build the Mie table on the device (blocks until the scalars are back)."""
    import torch
    dev = torch.device(device)
    inv = torch.empty(max(int(spec.n_cdf), 1), dtype=torch.float32, device=dev)
    ph = torch.empty(max(int(spec.n_angles), 1), dtype=torch.float64, device=dev) if phase else None
    cd = torch.empty(max(int(spec.n_angles), 1), dtype=torch.float64, device=dev) if cdf else None
    co = torch.empty((MC_MAX_TERMS, 4), dtype=torch.float64, device=dev) if coef else None
    t = _MieTableC()
    t.inv_cdf, t.phase, t.cdf, t.coef = _ptr(inv), _ptr(ph), _ptr(cd), _ptr(co)
    t.coef_capacity = MC_MAX_TERMS if coef else 0
    with torch.cuda.device(dev):
        _check(lib().mie_table_build(C.byref(spec), C.byref(t), _stream(stream)))
    return MieTable(t.x, complex(t.m_rel_re, t.m_rel_im), t.q_ext, t.q_sca, t.q_abs, t.g, t.sigma_ext_mm2,
                    t.sigma_sca_mm2, t.sigma_abs_mm2, t.n_terms, inv, ph, cd,
                    co[: t.n_terms] if co is not None else None)


def mie_table_build_poly(spec: MieSpec, sigma_ln: float, n_bins: int, device="cuda", *, phase=False, cdf=False,
                         stream=None) -> MieTable:
    """Polydisperse table: lognormal diameters with median spec.diameter_um
    and width sigma_ln of ln d on n_bins Gauss-Hermite bins (blocks until the
    scalars are back)."""
    import torch
    dev = torch.device(device)
    inv = torch.empty(max(int(spec.n_cdf), 1), dtype=torch.float32, device=dev)
    ph = torch.empty(max(int(spec.n_angles), 1), dtype=torch.float64, device=dev) if phase else None
    cd = torch.empty(max(int(spec.n_angles), 1), dtype=torch.float64, device=dev) if cdf else None
    q = MiePoly(sigma_ln=float(sigma_ln), n_bins=int(n_bins))
    nbytes = int(lib().mie_poly_work_bytes(C.byref(spec), C.byref(q)))
    work = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=dev)
    q.work, q.work_bytes = _ptr(work), nbytes
    t = _MieTableC()
    t.inv_cdf, t.phase, t.cdf = _ptr(inv), _ptr(ph), _ptr(cd)
    with torch.cuda.device(dev):
        _check(lib().mie_table_build_poly(C.byref(spec), C.byref(q), C.byref(t), _stream(stream)))
    return MieTable(t.x, complex(t.m_rel_re, t.m_rel_im), t.q_ext, t.q_sca, t.q_abs, t.g, t.sigma_ext_mm2,
                    t.sigma_sca_mm2, t.sigma_abs_mm2, t.n_terms, inv, ph, cd)


def mc_lognormal_bins(median_um: float, sigma_ln: float, n_bins: int):
    """(diameters_um, probabilities) of the library's Gauss-Hermite bins (host)."""
    d = (C.c_double * max(int(n_bins), 1))()
    p = (C.c_double * max(int(n_bins), 1))()
    _check(lib().mc_lognormal_bins(float(median_um), float(sigma_ln), int(n_bins), d, p))
    return list(d)[: int(n_bins)], list(p)[: int(n_bins)]


def mie_table_enqueue(spec: MieSpec, device="cuda", *, inv_cdf=None, result=None, work=None,
                      stream=None) -> MieTable:
    """Enqueue the table build without waiting (efficiencies and g stay on
    the device in `result`).  Reuses the given buffers when passed; `work`
    (n_angles doubles) carries the angle grid between the two kernels and
    must not serve two builds in flight at once."""
    import torch
    dev = torch.device(device)
    inv = inv_cdf if inv_cdf is not None else torch.empty(max(int(spec.n_cdf), 1), dtype=torch.float32, device=dev)
    res = result if result is not None else torch.empty(4, dtype=torch.float64, device=dev)
    wk = work if work is not None else torch.empty(max(int(spec.n_angles), 1), dtype=torch.float64, device=dev)
    _require(inv, "inv_cdf", torch.float32, min_numel=max(int(spec.n_cdf), 1))
    _require(res, "result", torch.float64, min_numel=4)
    _require(wk, "work", torch.float64, min_numel=max(int(spec.n_angles), 1))
    _on_one_gpu(inv_cdf=inv, result=res, work=wk)
    t = _MieTableC()
    t.inv_cdf, t.result, t.work = _ptr(inv), _ptr(res), _ptr(wk)
    with torch.cuda.device(dev):
        _check(lib().mie_table_enqueue(C.byref(spec), C.byref(t), _stream(stream)))
    return MieTable(t.x, complex(t.m_rel_re, t.m_rel_im), t.q_ext, t.q_sca, t.q_abs, t.g, t.sigma_ext_mm2,
                    t.sigma_sca_mm2, t.sigma_abs_mm2, t.n_terms, inv, result=res, work=wk)


def mc_medium_coefficients(medium: Medium, geometry: Geometry) -> dict:
    """The coefficients the walk derives from `medium` (host only):
    mu_sca, mu_abs, mu_ext in 1/mm and the albedo."""
    out = (C.c_double * 4)()
    _check(lib().mc_medium_coefficients(C.byref(medium), C.byref(geometry), out))
    return dict(mu_sca=out[0], mu_abs=out[1], mu_ext=out[2], albedo=out[3])


def mc_workspace_bytes(det: Detector) -> int:
    return int(lib().mc_workspace_bytes(C.byref(det)))


def mc_workspace_bytes_log(det: Detector, n_photons: int) -> int:
    return int(lib().mc_workspace_bytes_log(C.byref(det), int(n_photons)))


def mc_workspace_bytes_batch(det: Detector, n_items: int) -> int:
    return int(lib().mc_workspace_bytes_batch(C.byref(det), int(n_items)))


def mc_workspace_bytes_batch_log(det: Detector, n_items: int, total_photons: int) -> int:
    return int(lib().mc_workspace_bytes_batch_log(C.byref(det), int(n_items), int(total_photons)))


@dataclass
class Tally:
    """Caller-owned device outputs and workspace of mc_simulate.  Images are
    float64, or int64 fixed point (weight * 2^32) when allocated with fix64."""
    side: "object"
    trans: "object"
    scalars: "object"
    workspace: "object" = None
    side_w2: "object" = None
    trans_w2: "object" = None
    rec_i: "object" = None          # (MC_REC_I_N, rows) int32
    rec_f: "object" = None          # (MC_REC_F_N, rows) float32
    side_wk: "object" = None        # MC_MOMENTS: float64, side-image shape
    side_wl: "object" = None
    side_w2k: "object" = None       # MC_MOMENTS_PIXEL2
    side_w2l: "object" = None

    @staticmethod
    def alloc(det: Detector, device="cuda", *, sigma=False, record_rows=0, fix64=False,
              moments=False, pixel2=False, log_photons=None, workspace=None) -> "Tally":
        """With det.flags & MC_EXIT_LOG, the workspace also holds an exit log
        sized for log_photons photons.  `workspace` (an int64 device tensor
        from a previous alloc) is shared instead of allocating one: walks
        enqueued one after another on one stream may share it."""
        import torch
        dev = torch.device(device)
        img = dict(dtype=torch.int64 if fix64 else torch.float64, device=dev)
        probe = Detector(det.side_nx, det.side_ny, det.trans_nx, det.trans_ny,
                         det.flags | (MC_SIGMA if sigma else 0))
        if det.flags & MC_EXIT_LOG:
            ws_bytes = mc_workspace_bytes_log(probe, int(log_photons or 0))
        else:
            ws_bytes = mc_workspace_bytes(probe)
        if workspace is None:
            workspace = torch.empty((ws_bytes + 7) // 8, dtype=torch.int64, device=dev)
        elif workspace.dtype != torch.int64 or workspace.numel() * 8 < ws_bytes:
            raise ValueError(f"shared workspace must be int64 with at least {ws_bytes} bytes")
        t = Tally(torch.empty((det.side_ny, det.side_nx), **img), torch.empty((det.trans_ny, det.trans_nx), **img),
                  torch.empty(MC_N_SCALARS, dtype=torch.float64, device=dev), workspace)
        if sigma:
            t.side_w2 = torch.empty_like(t.side)
            t.trans_w2 = torch.empty_like(t.trans)
        if moments:
            t.side_wk = torch.empty((det.side_ny, det.side_nx), dtype=torch.float64, device=dev)
            t.side_wl = torch.empty_like(t.side_wk)
        if moments and pixel2:
            t.side_w2k = torch.empty_like(t.side_wk)
            t.side_w2l = torch.empty_like(t.side_wk)
        if record_rows:
            t.rec_i = torch.empty((MC_REC_I_N, record_rows), dtype=torch.int32, device=dev)
            t.rec_f = torch.empty((MC_REC_F_N, record_rows), dtype=torch.float32, device=dev)
        return t

    @staticmethod
    def alloc_batch(det: Detector, n_items: int, device="cuda", *, sigma=False, fix64=False,
                    log_photons=None) -> "Tally":
        """Item-major outputs of mc_simulate_batch for n_items media; with
        det.flags & MC_EXIT_LOG the workspace also holds an exit log sized for
        log_photons photons over all items."""
        import torch
        dev = torch.device(device)
        img = dict(dtype=torch.int64 if fix64 else torch.float64, device=dev)
        probe = Detector(det.side_nx, det.side_ny, det.trans_nx, det.trans_ny,
                         det.flags | (MC_SIGMA if sigma else 0))
        if det.flags & MC_EXIT_LOG:
            ws_bytes = mc_workspace_bytes_batch_log(probe, n_items, int(log_photons or 0))
        else:
            ws_bytes = mc_workspace_bytes_batch(probe, n_items)
        if ws_bytes == 0:
            raise ValueError(f"invalid detector or n_items {n_items} (1..{MC_MAX_BATCH})")
        t = Tally(torch.empty((n_items, det.side_ny, det.side_nx), **img),
                  torch.empty((n_items, det.trans_ny, det.trans_nx), **img),
                  torch.empty((n_items, MC_N_SCALARS), dtype=torch.float64, device=dev),
                  torch.empty((ws_bytes + 7) // 8, dtype=torch.int64, device=dev))
        if sigma:
            t.side_w2 = torch.empty_like(t.side)
            t.trans_w2 = torch.empty_like(t.trans)
        return t

    def validate(self, det: Detector, n_items: Optional[int] = None, *, grad: bool = False,
                 need_workspace: bool = True, **extra):
        """Check every buffer the library will touch against `det` (and
        n_items media for a batched launch) before a call: dtypes, shapes and
        contiguity first, then that they (and the tensors in `extra`, already
        checked by the caller) share one GPU.  Raises ValueError; returns the
        device."""
        import torch
        lead = () if n_items is None else (int(n_items),)
        img_t = torch.int64 if det.flags & MC_FIX64 else torch.float64
        side_shape = lead + (det.side_ny, det.side_nx)
        trans_shape = lead + (det.trans_ny, det.trans_nx)
        used = {}
        if not grad:
            used["tally.side"] = _require(self.side, "tally.side", img_t, shape=side_shape)
            used["tally.trans"] = _require(self.trans, "tally.trans", img_t, shape=trans_shape)
        used["tally.scalars"] = _require(self.scalars, "tally.scalars", torch.float64,
                                         numel=MC_N_SCALARS * (1 if n_items is None else n_items))
        if need_workspace:
            used["tally.workspace"] = _require(self.workspace, "tally.workspace", torch.int64)
        if (det.flags & MC_SIGMA) and not grad:
            used["tally.side_w2"] = _require(self.side_w2, "tally.side_w2", img_t, shape=side_shape)
            used["tally.trans_w2"] = _require(self.trans_w2, "tally.trans_w2", img_t, shape=trans_shape)
        if det.flags & MC_MOMENTS or grad:
            for name in ("side_wk", "side_wl"):
                used[f"tally.{name}"] = _require(getattr(self, name), f"tally.{name}", torch.float64,
                                                 shape=side_shape)
        if det.flags & MC_MOMENTS_PIXEL2 or (grad and self.side_w2k is not None):
            for name in ("side_w2k", "side_w2l"):
                used[f"tally.{name}"] = _require(getattr(self, name), f"tally.{name}", torch.float64,
                                                 shape=side_shape)
        if (det.flags & MC_RECORD) and not grad and (self.rec_i is not None or self.rec_f is not None):
            ri = _require(self.rec_i, "tally.rec_i", torch.int32)
            if ri.dim() != 2 or ri.shape[0] != MC_REC_I_N:
                raise ValueError(f"tally.rec_i must have shape ({MC_REC_I_N}, rows)")
            used["tally.rec_i"] = ri
            used["tally.rec_f"] = _require(self.rec_f, "tally.rec_f", torch.float32, shape=(MC_REC_F_N, ri.shape[1]))
        return _on_one_gpu(**used, **extra)

    def _c(self) -> _TallyC:
        c = _TallyC()
        c.side, c.trans, c.scalars = _ptr(self.side), _ptr(self.trans), _ptr(self.scalars)
        c.side_w2, c.trans_w2 = _ptr(self.side_w2), _ptr(self.trans_w2)
        c.rec_i, c.rec_f = _ptr(self.rec_i), _ptr(self.rec_f)
        c.rec_rows = 0 if self.rec_i is None else int(self.rec_i.shape[1])
        c.workspace = _ptr(self.workspace)
        c.workspace_bytes = 0 if self.workspace is None else self.workspace.numel() * 8
        c.side_wk, c.side_wl = _ptr(self.side_wk), _ptr(self.side_wl)
        c.side_w2k, c.side_w2l = _ptr(self.side_w2k), _ptr(self.side_w2l)
        return c


def mc_simulate(medium: Medium, source: Source, geometry: Geometry, detector: Detector, run: Run,
                tally: Tally, stream=None) -> None:
    """Enqueue the photon walk on the stream (asynchronous)."""
    tally.validate(detector)
    tc = tally._c()
    _check(lib().mc_simulate(C.byref(medium), C.byref(source), C.byref(geometry), C.byref(detector),
                             C.byref(run), C.byref(tc), _stream(stream)))


def mc_simulate_noalloc(medium: Medium, source: Source, geometry: Geometry, detector: Detector, run: Run,
                        tally: Tally, stream=None) -> None:
    """mc_simulate with the library's own device scratch in place of a
    workspace (tally.workspace may be None): allocates nothing.  At most 2^21
    image pixels (2^20 with MC_SIGMA), no MC_EXIT_LOG; calls overlapping on
    one GPU race."""
    tally.validate(detector, need_workspace=False)
    tc = tally._c()
    tc.workspace, tc.workspace_bytes = None, 0
    _check(lib().mc_simulate_noalloc(C.byref(medium), C.byref(source), C.byref(geometry), C.byref(detector),
                                     C.byref(run), C.byref(tc), _stream(stream)))


def mc_grad(medium: Medium, geometry: Geometry, detector: Detector, tally: Tally, dloss_dside,
            d2loss_dside2=None, d2loss_uniform: float = 0.0, stream=None):
    """(dLoss/dmu_sca, dLoss/dmu_abs, dLoss/dconcentration) from the moments
    of `tally` (filled by mc_simulate with MC_MOMENTS), dLoss/dI of the side
    image (float64 device tensor) and, optionally, the loss's diagonal second
    derivative for the self-correlation correction: per pixel
    (`d2loss_dside2`, device tensor, needs MC_MOMENTS_PIXEL2) or one value for
    every pixel (`d2loss_uniform`).  Waits for the stream."""
    import torch
    n = detector.side_ny * detector.side_nx
    g = _require(dloss_dside, "dloss_dside", torch.float64, numel=n)
    h = _require(d2loss_dside2, "d2loss_dside2", torch.float64, numel=n, optional=True)
    tally.validate(detector, grad=True, dloss_dside=g, d2loss_dside2=h)
    out = (C.c_double * 3)()
    tc = tally._c()
    _check(lib().mc_grad(C.byref(medium), C.byref(geometry), C.byref(detector), C.byref(tc),
                         _ptr(dloss_dside), _ptr(d2loss_dside2), float(d2loss_uniform), out, _stream(stream)))
    return tuple(out)


def _batch_items(items) -> "C.Array":
    arr = (BatchItem * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def mc_simulate_batch(items, n_cdf: int, source: Source, geometry: Geometry, detector: Detector, run: Run,
                      tally: Tally, stream=None) -> None:
    """Enqueue the batched walk of `items` (a sequence of BatchItem, one per
    medium; outputs item-major in `tally`, see Tally.alloc_batch)."""
    arr = _batch_items(items)
    tally.validate(detector, len(items))
    tc = tally._c()
    _check(lib().mc_simulate_batch(arr, len(items), int(n_cdf), C.byref(source), C.byref(geometry),
                                   C.byref(detector), C.byref(run), C.byref(tc), _stream(stream)))


def mc_autotune_batch(items, n_cdf: int, source: Source, geometry: Geometry, detector: Detector, run: Run,
                      tally: Tally, sample_fraction: float = 0.0625, stream=None):
    """Time every (block size, chunk) candidate on a photon sample of the
    batch; returns (block_size, chunk, best_ms, {(block, chunk): ms}).  The
    tally is overwritten.  Waits for the stream."""
    arr = _batch_items(items)
    tally.validate(detector, len(items))
    tc = tally._c()
    blk, chk, best = C.c_int32(), C.c_uint32(), C.c_double()
    cand = (C.c_double * (len(AUTOTUNE_BLOCKS) * len(AUTOTUNE_CHUNKS)))()
    _check(lib().mc_autotune_batch(arr, len(items), int(n_cdf), C.byref(source), C.byref(geometry),
                                   C.byref(detector), C.byref(run), C.byref(tc), float(sample_fraction),
                                   C.byref(blk), C.byref(chk), C.byref(best), cand, _stream(stream)))
    table = {(b, c): cand[i * len(AUTOTUNE_CHUNKS) + j]
             for i, b in enumerate(AUTOTUNE_BLOCKS) for j, c in enumerate(AUTOTUNE_CHUNKS)}
    return blk.value, chk.value, best.value, table


def image_metrics(a, b, c=None, *, cx=None, cy=None, r_max=None, profiles=False, stream=None) -> dict:
    """Comparison measures of Tables 3 and 4 between images a and b (b the
    reference) and optionally c (float64 device tensors of one shape); the
    radial centre defaults to the image centre and r_max to half the shorter
    side.  Waits for the stream."""
    import torch
    if not isinstance(a, torch.Tensor) or a.dim() != 2:
        raise ValueError("a must be a 2-D torch tensor")
    _require(a, "a", torch.float64)
    _require(b, "b", torch.float64, shape=a.shape)
    _require(c, "c", torch.float64, shape=a.shape, optional=True)
    _on_one_gpu(a=a, b=b, c=c)
    ny, nx = (int(v) for v in a.shape)
    rad = Radial(nx / 2.0 if cx is None else cx, ny / 2.0 if cy is None else cy,
                 min(nx, ny) / 2.0 if r_max is None else r_max)
    nbytes = int(lib().mc_metrics_work_bytes(nx, ny, C.byref(rad)))
    if nbytes == 0:
        raise ValueError("invalid image shape or radial settings")
    work = torch.empty(nbytes // 8, dtype=torch.float64, device=a.device)
    n_r = int(math.ceil(rad.r_max))
    prof = torch.empty((4, n_r), dtype=torch.float64, device=a.device) if profiles else None
    out = (C.c_double * MC_METRICS_N)()
    _check(lib().mc_image_metrics(_ptr(a), _ptr(b), _ptr(c), nx, ny, C.byref(rad), _ptr(prof), _ptr(work), nbytes,
                                  out, _stream(stream)))
    res = dict(rmse=out[0], r=out[1], zone_rmse=[out[2], out[3], out[4]], radial_r=out[5], n_annuli=int(out[6]),
               max=[out[7], out[8], out[9]], better=out[10], pixels=int(out[11]))
    if profiles:
        res["profile_a"], res["profile_b"], res["profile_c"], res["count"] = prof[0], prof[1], prof[2], prof[3]
    return res


def mc_philox_blocks(seed: int, instance: int, ids, step0: int, n_steps: int, out, stream=None) -> None:
    """Fill `out` (uint32 viewed as int32, len(ids) * n_steps * 4) with the walk's Philox words."""
    import torch
    _require(ids, "ids", (torch.int64, torch.uint64))
    _require(out, "out", (torch.int32, torch.uint32), min_numel=int(ids.numel()) * int(n_steps) * 4)
    _on_one_gpu(ids=ids, out=out)
    _check(lib().mc_philox_blocks(seed, instance, _ptr(ids), int(ids.numel()), step0, n_steps, _ptr(out),
                                  _stream(stream)))


def mc_version() -> int:
    return lib().mc_version()
