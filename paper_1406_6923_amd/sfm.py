"""ctypes binding of libsfm.so (include/sfm.h) with the same entry-point names.

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are passed as torch tensors on the GPU (their data pointers are
borrowed for the duration of the stream work), host arrays as NumPy arrays,
streams as torch.cuda.Stream (default: the current stream).  A failing call
raises ``SfmError`` carrying the status and ``sfm_last_error``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsfm.so")

SFM_OK = 0
SFM_EINVAL = -1
SFM_EHIP = -2
SFM_ENOMEM = -3
SFM_EBREAKDOWN = -4
SFM_ESTATE = -5
SFM_EUNSTABLE = -6
SFM_ENOCONV = -7
STATUS_NAMES = {0: "SFM_OK", -1: "SFM_EINVAL", -2: "SFM_EHIP", -3: "SFM_ENOMEM",
                -4: "SFM_EBREAKDOWN", -5: "SFM_ESTATE", -6: "SFM_EUNSTABLE", -7: "SFM_ENOCONV"}
SFM_PREC_FP32 = 0
SFM_PREC_BF16_FP32ACC = 1
SFM_PREC_FP64 = 2


class sfm_config(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_int32 * 3), ("sub_cells", ctypes.c_int32 * 3), ("h", ctypes.c_double),
                ("m", ctypes.c_int32), ("k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("build_batch", ctypes.c_int32)]


class sfm_info(ctypes.Structure):
    _fields_ = [("n_subdomains", ctypes.c_int32), ("p", ctypes.c_int32), ("k", ctypes.c_int32),
                ("nsrc", ctypes.c_int32), ("nrec", ctypes.c_int32), ("has_roms", ctypes.c_int32),
                ("steps_done", ctypes.c_int64), ("coef_bytes", ctypes.c_int64),
                ("coef_bytes_algorithmic", ctypes.c_int64), ("state_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double), ("timed_steps", ctypes.c_int64),
                ("timed_main_ms", ctypes.c_double), ("timed_face_ms", ctypes.c_double),
                ("timed_record_ms", ctypes.c_double), ("rho_estimate", ctypes.c_double),
                ("rho_bound", ctypes.c_double), ("watchdog_checks", ctypes.c_int64)]


class SfmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

# name -> (restype, argtypes); mirrors include/sfm.h
SIGNATURES = {
    "sfm_create": (_I32, [ctypes.POINTER(sfm_config), ctypes.POINTER(_VP)]),
    "sfm_cnn_create": (_I32, [_I32, _I32, _I32, _I32, ctypes.c_uint64, ctypes.POINTER(_VP)]),
    "sfm_cnn_destroy": (None, [_VP]),
    "sfm_cnn_last_error": (ctypes.c_char_p, [_VP]),
    "sfm_cnn_info": (_I32, [_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I32), _VP, _VP]),
    "sfm_rom_inputs": (_I32, [_VP, _VP, _VP, _VP]),
    "sfm_rom_targets": (_I32, [_VP, _VP, _VP]),
    "sfm_ntd_error": (_I32, [_VP, _VP, _D, _VP, _VP]),
    "sfm_build_roms_surrogate": (_I32, [_VP, _VP, _D, _D, _VP, _I32, _VP, _I32, _VP, _VP, _VP, _VP, _VP]),
    "sfm_cnn_params": (_I32, [_VP, _VP, _VP]),
    "sfm_cnn_forward": (_I32, [_VP, _VP, _I32, _VP, _VP]),
    "sfm_cnn_backward": (_I32, [_VP, _VP, _VP, _VP]),
    "sfm_cnn_input_grad": (_I32, [_VP, _VP, _VP, _VP]),
    "sfm_surrogate_velocity_gradient": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "sfm_surrogate_predict": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "sfm_cnn_fit_scale": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP]),
    "sfm_cnn_train": (_I32, [_VP, _VP, _VP, _I64, _I32, _I32, ctypes.c_float, ctypes.c_uint64, _VP, _VP]),
    "sfm_create_boxes": (_I32, [ctypes.POINTER(sfm_config), _VP, _VP, ctypes.POINTER(_VP)]),
    "sfm_destroy": (None, [_VP]),
    "sfm_last_error": (ctypes.c_char_p, [_VP]),
    "sfm_query": (_I32, [_VP, ctypes.POINTER(sfm_info)]),
    "sfm_build_roms": (_I32, [_VP, _VP, _I32, _VP, _I32, _VP, _VP, _VP, _VP]),
    "sfm_build_roms_shifted": (_I32, [_VP, _D, _D, _I32, _VP, _I32, _VP, _I32, _VP, _VP, _VP,
                                      ctypes.POINTER(_I32), _VP]),
    "sfm_reset_state": (_I32, [_VP, _D, _VP]),
    "sfm_adjoint_gradient": (_I32, [_VP, _I32, _D, _VP, _VP, _I64, _I32, _VP, _VP, _VP]),
    "sfm_shots_init": (_I32, [_VP, _I32, _VP, _VP]),
    "sfm_shots_step": (_I32, [_VP, _I32, _D, _VP, _VP, _I64, _VP]),
    "sfm_shots_graph": (_I32, [_VP, _I32, ctypes.POINTER(_I64)]),
    "sfm_shots_get_state": (_I32, [_VP, _VP, _VP]),
    "sfm_shots_set_state": (_I32, [_VP, _VP, _VP]),
    "sfm_shots_timing": (_I32, [_VP, ctypes.POINTER(_I64), _VP]),
    "sfm_shots_tuning": (_I32, [_VP, ctypes.POINTER(_I32), _VP, _I32, ctypes.POINTER(_I32)]),
    "sfm_shots_select": (_I32, [_VP, _I32]),
    "sfm_load_roms": (_I32, [_VP, _VP, _VP, _I32, _VP, _VP, _I32, _VP, _VP]),
    "sfm_export_roms": (_I32, [_VP, _VP, _VP]),
    "sfm_export_projections": (_I32, [_VP, _VP, _VP]),
    "sfm_cfl_dt": (_I32, [_VP, _I32, ctypes.POINTER(_D), _VP]),
    "sfm_step": (_I32, [_VP, _I32, _D, _VP, _VP, _I64, _VP]),
    "sfm_set_watchdog": (_I32, [_VP, _I32, _D]),
    "sfm_dgemm_batched": (_I32, [_I32, _I32, _I32, _I32, _I32, _D, _VP, _I64, _I64, _VP, _I64, _I64, _D, _VP, _I64,
                                 _I64, _I32, _VP, _I64, _VP]),
    "sfm_cfl_dt_noalloc": (_I32, [_VP, _I32, ctypes.POINTER(_D), _VP]),
    "sfm_probe_fp64_matrix_rate": (_I32, [_I32, _I32, _VP, ctypes.POINTER(_D), _VP]),
    "sfm_record_receivers": (_I32, [_VP, _VP, _VP]),
    "sfm_apply_operator": (_I32, [_VP, _VP, _VP, _VP]),
    "sfm_set_timing": (_I32, [_VP, _I32]),
    "sfm_get_state": (_I32, [_VP, _VP, _VP, ctypes.POINTER(_I64)]),
    "sfm_set_state": (_I32, [_VP, _VP, _VP, _I64]),
    "sfm_set_levels": (_I32, [_VP, _VP]),
    "sfm_build_roms_levels": (_I32, [_VP, _VP, _VP, _I32, _VP, _I32, _VP, _VP, _VP, _VP]),
    "sfm_get_levels": (_I32, [_VP, _VP]),
    "sfm_fdtd_run": (_I32, [_VP, _D, _VP, _D, _I32, _I32, _VP, _VP, _I32, _VP, _VP, _I64, ctypes.POINTER(_D), _VP]),
    "sfm_fdtd_last_error": (ctypes.c_char_p, []),
    "sfm_step_plain": (_I32, [_VP, _I32, _D, _VP, _VP]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsfm.so (built in-tree by ``build_lib.build``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1406_6923_amd.build_lib`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ------------------------------------------------------------------ marshalling helpers
def _dev(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device arrays must be contiguous GPU tensors")
    return t.data_ptr()


def _host(a, dtype) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_VP)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _check(ctx, status: int):
    if status != SFM_OK:
        msg = load_library().sfm_last_error(ctx)
        raise SfmError(status, msg.decode() if msg else "")


# ------------------------------------------------------------------ entry points
def sfm_create(ncell, sub_cells, h: float, m: int, k: int, precision: int = SFM_PREC_FP32,
               build_batch: int = 0) -> int:
    """sub_cells: per axis one box size (equal boxes) or the list of box sizes (uneven boxes)."""
    lib = load_library()
    uneven = any(np.ndim(sc) > 0 for sc in sub_cells)
    even = [0, 0, 0] if uneven else [int(sc) for sc in sub_cells]
    cfg = sfm_config((ctypes.c_int32 * 3)(*ncell), (ctypes.c_int32 * 3)(*even), float(h), int(m), int(k),
                     int(precision), int(build_batch))
    out = _VP()
    if uneven:
        lists = [[int(sc)] * (int(n) // int(sc)) if np.ndim(sc) == 0 else [int(x) for x in sc]
                 for n, sc in zip(ncell, sub_cells)]
        nbox = np.array([len(x) for x in lists], dtype=np.int32)
        cells = np.array(sum(lists, []), dtype=np.int32)
        status = lib.sfm_create_boxes(ctypes.byref(cfg), _ptr(nbox), _ptr(cells), ctypes.byref(out))
    else:
        status = lib.sfm_create(ctypes.byref(cfg), ctypes.byref(out))
    _check(None, status)
    return out.value


def sfm_destroy(ctx: int) -> None:
    load_library().sfm_destroy(ctx)


def sfm_last_error(ctx: Optional[int]) -> str:
    msg = load_library().sfm_last_error(ctx)
    return msg.decode() if msg else ""


def sfm_query(ctx: int) -> dict:
    info = sfm_info()
    _check(ctx, load_library().sfm_query(ctx, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in sfm_info._fields_}


def sfm_build_roms(ctx: int, vel, src_ijk=None, rec_ijk=None, u0=None, v0=None, stream=None) -> None:
    src = _host(np.zeros((0, 3)) if src_ijk is None else src_ijk, np.int32).reshape(-1, 3)
    rec = _host(np.zeros((0, 3)) if rec_ijk is None else rec_ijk, np.int32).reshape(-1, 3)
    _check(ctx, load_library().sfm_build_roms(ctx, _dev(vel), len(src), _ptr(src), len(rec), _ptr(rec),
                                              _dev(u0), _dev(v0), _stream(stream)))


def sfm_build_roms_shifted(ctx: int, sigma: float, vel, src_ijk=None, rec_ijk=None, u0=None, v0=None,
                           cg_rtol: float = 1e-12, cg_max_iter: int = 5000, stream=None) -> int:
    """Finite-shift build; returns the largest inner CG iteration count."""
    src = _host(np.zeros((0, 3)) if src_ijk is None else src_ijk, np.int32).reshape(-1, 3)
    rec = _host(np.zeros((0, 3)) if rec_ijk is None else rec_ijk, np.int32).reshape(-1, 3)
    iters = _I32(0)
    _check(ctx, load_library().sfm_build_roms_shifted(ctx, float(sigma), float(cg_rtol), int(cg_max_iter), _dev(vel),
                                                      len(src), _ptr(src), len(rec), _ptr(rec), _dev(u0), _dev(v0),
                                                      ctypes.byref(iters), _stream(stream)))
    return int(iters.value)


def sfm_reset_state(ctx: int, dt: float, stream=None) -> None:
    _check(ctx, load_library().sfm_reset_state(ctx, float(dt), _stream(stream)))


def sfm_load_roms(ctx: int, gamma, gamma_hat, src_ijk=None, src_vec=None, rec_ijk=None, rec_rows=None) -> None:
    g = _host(gamma, np.float64)
    gh = _host(gamma_hat, np.float64)
    src = _host(np.zeros((0, 3)) if src_ijk is None else src_ijk, np.int32).reshape(-1, 3)
    rec = _host(np.zeros((0, 3)) if rec_ijk is None else rec_ijk, np.int32).reshape(-1, 3)
    sv = _host(src_vec, np.float64)
    rr = _host(rec_rows, np.float64)
    _check(ctx, load_library().sfm_load_roms(ctx, _ptr(g), _ptr(gh), len(src), _ptr(src), _ptr(sv), len(rec),
                                             _ptr(rec), _ptr(rr)))


def sfm_export_roms(ctx: int):
    info = sfm_query(ctx)
    S, k, p = info["n_subdomains"], info["k"], info["p"]
    g = np.empty((S, k, p, p))
    gh = np.empty((S, k, p, p))
    _check(ctx, load_library().sfm_export_roms(ctx, _ptr(g), _ptr(gh)))
    return g, gh


def sfm_export_projections(ctx: int):
    info = sfm_query(ctx)
    k, p = info["k"], info["p"]
    sv = np.empty((info["nsrc"], k, p))
    rr = np.empty((info["nrec"], k, p))
    _check(ctx, load_library().sfm_export_projections(ctx, _ptr(sv), _ptr(rr)))
    return sv, rr


def sfm_cfl_dt(ctx: int, iters: int = 200, stream=None) -> float:
    out = _D()
    _check(ctx, load_library().sfm_cfl_dt(ctx, int(iters), ctypes.byref(out), _stream(stream)))
    return out.value


def sfm_step(ctx: int, nsteps: int, dt: float, wavelet=None, traces=None, ld: Optional[int] = None,
             stream=None) -> None:
    if ld is None:
        ld = traces.shape[-1] if traces is not None else 0
    _check(ctx, load_library().sfm_step(ctx, int(nsteps), float(dt), _dev(wavelet), _dev(traces), int(ld),
                                        _stream(stream)))


def sfm_cfl_dt_noalloc(ctx: int, iters: int = 200, stream=None) -> float:
    out = _D()
    _check(ctx, load_library().sfm_cfl_dt_noalloc(ctx, int(iters), ctypes.byref(out), _stream(stream)))
    return out.value


def sfm_dgemm_batched(trans_a: bool, trans_b: bool, M: int, N: int, K: int, alpha: float, A, lda: int, stride_a: int,
                      B, ldb: int, stride_b: int, beta: float, C, ldc: int, stride_c: int, batch: int, work=None,
                      stream=None) -> None:
    """Column-major batched FP64 product on device tensors (see include/sfm.h)."""
    wb = work.numel() * work.element_size() if work is not None else 0
    st = load_library().sfm_dgemm_batched(int(bool(trans_a)), int(bool(trans_b)), int(M), int(N), int(K), float(alpha),
                                          _dev(A), int(lda), int(stride_a), _dev(B), int(ldb), int(stride_b),
                                          float(beta), _dev(C), int(ldc), int(stride_c), int(batch), _dev(work),
                                          int(wb), _stream(stream))
    if st != SFM_OK:
        raise SfmError(st, "sfm_dgemm_batched failed")


def sfm_probe_fp64_matrix_rate(out, blocks: int = 4096, iters: int = 2000, stream=None) -> float:
    """Sustained FP64 matrix-core TFLOP/s (out: device float64 tensor of >= blocks * 256)."""
    if out.numel() < blocks * 256:
        raise ValueError("out holds fewer than blocks * 256 doubles")
    tf = _D(0.0)
    st = load_library().sfm_probe_fp64_matrix_rate(int(blocks), int(iters), _dev(out), ctypes.byref(tf),
                                                   _stream(stream))
    if st != SFM_OK:
        raise SfmError(st, "sfm_probe_fp64_matrix_rate failed")
    return tf.value


def sfm_set_watchdog(ctx: int, every: int, max_norm: float = float("inf")) -> None:
    _check(ctx, load_library().sfm_set_watchdog(ctx, int(every), float(max_norm)))


def sfm_adjoint_gradient(ctx: int, nsteps: int, dt: float, wavelet, grad_traces, checkpoint_every: int = 100,
                         ld: Optional[int] = None, stream=None):
    """dJ/dGamma, dJ/dGamma-hat (FP64 [S][k][p][p] each) for trace gradient grad_traces [nrec][ld] (device)."""
    info = sfm_query(ctx)
    shape = (info["n_subdomains"], info["k"], info["p"], info["p"])
    g_gam = np.zeros(shape)
    g_hat = np.zeros(shape)
    if ld is None:
        ld = grad_traces.shape[-1]
    _check(ctx, load_library().sfm_adjoint_gradient(ctx, int(nsteps), float(dt), _dev(wavelet), _dev(grad_traces),
                                                    int(ld), int(checkpoint_every), _ptr(g_gam), _ptr(g_hat),
                                                    _stream(stream)))
    return g_gam, g_hat


def sfm_shots_init(ctx: int, nshot: int, shot_src=None, stream=None) -> None:
    arr = None if shot_src is None else _host(shot_src, np.int32).reshape(-1)
    if arr is not None and len(arr) != nshot:
        raise ValueError("shot_src needs one entry per shot")
    _check(ctx, load_library().sfm_shots_init(ctx, int(nshot), _ptr(arr) if arr is not None else None,
                                              _stream(stream)))


def sfm_shots_step(ctx: int, nsteps: int, dt: float, wavelet=None, traces=None, ld: Optional[int] = None,
                   stream=None) -> None:
    """wavelet: device float [nsteps][nshot]; traces: device float [nshot][nrec][ld] or None."""
    if ld is None:
        ld = traces.shape[-1] if traces is not None else 0
    _check(ctx, load_library().sfm_shots_step(ctx, int(nsteps), float(dt), _dev(wavelet), _dev(traces), int(ld),
                                              _stream(stream)))


def sfm_shots_get_state(ctx: int, nshot: int):
    info = sfm_query(ctx)
    u = np.empty((info["n_subdomains"], info["k"], info["p"], nshot), np.float32)
    d = np.empty_like(u)
    _check(ctx, load_library().sfm_shots_get_state(ctx, _ptr(u), _ptr(d)))
    return u, d


def sfm_shots_set_state(ctx: int, u, d) -> None:
    u = _host(u, np.float32)
    d = _host(d, np.float32)
    _check(ctx, load_library().sfm_shots_set_state(ctx, _ptr(u), _ptr(d)))


def sfm_shots_select(ctx: int, variant: int) -> None:
    """Force shot-kernel variant `variant` (order of sfm_shots_tuning), or -1 for the autotuner's."""
    _check(ctx, load_library().sfm_shots_select(ctx, int(variant)))


def sfm_shots_tuning(ctx: int, every_variant: bool = False):
    """(chosen waves per SIMD, [(waves, ms per step) of each variant]) from the last sfm_shots_init.
    Variants whose work-group limit is below this 6m were not run (time < 0): they are left out,
    unless every_variant, which lists all of them in variant order (the sfm_shots_select index)."""
    chosen, count = _I32(0), _I32(0)
    ms = np.zeros(16, np.float64)
    _check(ctx, load_library().sfm_shots_tuning(ctx, ctypes.byref(chosen), _ptr(ms), 8, ctypes.byref(count)))
    return int(chosen.value), [(int(ms[2 * v]), float(ms[2 * v + 1])) for v in range(count.value)
                               if every_variant or ms[2 * v + 1] >= 0]


def sfm_shots_timing(ctx: int):
    """(timed_steps, [main_ms, face_ms, record_ms]) summed since the last call."""
    n = _I64(0)
    ms = np.zeros(3, np.float64)
    _check(ctx, load_library().sfm_shots_timing(ctx, ctypes.byref(n), _ptr(ms)))
    return int(n.value), ms


def sfm_record_receivers(ctx: int, out, stream=None) -> None:
    _check(ctx, load_library().sfm_record_receivers(ctx, _dev(out), _stream(stream)))


def sfm_apply_operator(ctx: int, u, a, stream=None) -> None:
    _check(ctx, load_library().sfm_apply_operator(ctx, _dev(u), _dev(a), _stream(stream)))


def sfm_set_timing(ctx: int, enable, every: int = 1) -> None:
    """Time one step in `every` while enabled (False / 0 turns the timing off)."""
    _check(ctx, load_library().sfm_set_timing(ctx, int(every) if enable else 0))


def sfm_get_state(ctx: int):
    info = sfm_query(ctx)
    shape = (info["n_subdomains"], info["k"], info["p"])
    u = np.empty(shape, dtype=np.float32)
    d = np.empty(shape, dtype=np.float32)
    n = _I64()
    _check(ctx, load_library().sfm_get_state(ctx, _ptr(u), _ptr(d), ctypes.byref(n)))
    return u, d, n.value


def sfm_set_state(ctx: int, u_now=None, u_incr=None, n: int = 0) -> None:
    u = _host(u_now, np.float32)
    d = _host(u_incr, np.float32)
    _check(ctx, load_library().sfm_set_state(ctx, _ptr(u), _ptr(d), int(n)))


def sfm_shots_graph(ctx: int, enable: int = -1) -> int:
    """Enable (1) / disable (0) graph replay of shot windows, or query (-1); returns the replays so far."""
    n = _I64()
    _check(ctx, load_library().sfm_shots_graph(ctx, int(enable), ctypes.byref(n)))
    return n.value


def sfm_set_levels(ctx: int, k_per_sub=None) -> None:
    """Per-subdomain ROM levels (int per subdomain, 2..k); None restores k everywhere."""
    ks = None if k_per_sub is None else _host(np.asarray(k_per_sub), np.int32)
    _check(ctx, load_library().sfm_set_levels(ctx, _ptr(ks)))


def sfm_build_roms_levels(ctx: int, k_per_sub, vel, src_ijk=None, rec_ijk=None, u0=None, v0=None,
                          stream=None) -> None:
    ks = _host(np.asarray(k_per_sub), np.int32)
    src = _host(np.zeros((0, 3)) if src_ijk is None else src_ijk, np.int32).reshape(-1, 3)
    rec = _host(np.zeros((0, 3)) if rec_ijk is None else rec_ijk, np.int32).reshape(-1, 3)
    _check(ctx, load_library().sfm_build_roms_levels(ctx, _ptr(ks), _dev(vel), len(src), _ptr(src), len(rec),
                                                     _ptr(rec), _dev(u0), _dev(v0), _stream(stream)))


def sfm_get_levels(ctx: int) -> np.ndarray:
    out = np.empty(sfm_query(ctx)["n_subdomains"], dtype=np.int32)
    _check(ctx, load_library().sfm_get_levels(ctx, _ptr(out)))
    return out


def sfm_fdtd_run(ncell, h: float, vel, dt: float, nsteps: int, src_ijk=None, wavelet=None, rec_ijk=None,
                 traces=None, stream=None) -> float:
    """Fine-grid FDTD comparator; returns the wall time of the step loop in seconds."""
    lib = load_library()
    nc = _host(np.asarray(ncell), np.int32)
    src = _host(np.zeros((0, 3)) if src_ijk is None else src_ijk, np.int32).reshape(-1, 3)
    rec = _host(np.zeros((0, 3)) if rec_ijk is None else rec_ijk, np.int32).reshape(-1, 3)
    ld = traces.shape[-1] if traces is not None else 0
    secs = _D()
    status = lib.sfm_fdtd_run(_ptr(nc), float(h), _dev(vel), float(dt), int(nsteps), len(src), _ptr(src),
                              _dev(wavelet), len(rec), _ptr(rec), _dev(traces), int(ld), ctypes.byref(secs),
                              _stream(stream))
    if status != SFM_OK:
        raise SfmError(status, lib.sfm_fdtd_last_error().decode())
    return secs.value


def sfm_step_plain(ctx: int, nsteps: int, dt: float, wavelet=None, stream=None) -> None:
    _check(ctx, load_library().sfm_step_plain(ctx, int(nsteps), float(dt), _dev(wavelet), _stream(stream)))


class Sfm:
    """Owning handle around an sfm context (destroyed on close / garbage collection)."""

    def __init__(self, ncell, sub_cells, h, m, k, precision=SFM_PREC_FP32, build_batch=0):
        self.ctx = sfm_create(ncell, sub_cells, h, m, k, precision, build_batch)

    def close(self):
        if getattr(self, "ctx", None):
            sfm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def info(self):
        return sfm_query(self.ctx)


# ------------------------------------------------------------------ surrogate network
def _cnn_check(net, status: int):
    if status != SFM_OK:
        msg = load_library().sfm_cnn_last_error(net)
        raise SfmError(status, msg.decode() if msg else "")


class Cnn:
    """Owning handle around an sfm_cnn (the surrogate network); arguments as in include/sfm.h."""

    def __init__(self, n_in: int, channels: int, n_out: int, max_batch: int, seed: int = 0):
        lib = load_library()
        out = _VP()
        _cnn_check(None, lib.sfm_cnn_create(int(n_in), int(channels), int(n_out), int(max_batch), int(seed),
                                            ctypes.byref(out)))
        self.net = out.value
        self.n_in, self.channels, self.n_out, self.max_batch = n_in, channels, n_out, max_batch
        n, f = _I64(), _I32()
        nodes = np.zeros(5, np.int32)
        _cnn_check(self.net, lib.sfm_cnn_info(self.net, ctypes.byref(n), ctypes.byref(f), _ptr(nodes), None))
        self.n_params, self.features, self.nodes = int(n.value), int(f.value), nodes.tolist()

    def close(self):
        if getattr(self, "net", None):
            load_library().sfm_cnn_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _cnn_check(self.net, load_library().sfm_cnn_params(self.net, _ptr(out), None))
        return out

    def set_params(self, flat) -> None:
        arr = _host(flat, np.float32)
        if arr.size != self.n_params:
            raise ValueError(f"need {self.n_params} parameters")
        _cnn_check(self.net, load_library().sfm_cnn_params(self.net, None, _ptr(arr)))

    def forward(self, x, y=None, stream=None) -> None:
        _cnn_check(self.net, load_library().sfm_cnn_forward(self.net, _dev(x), int(x.shape[0]), _dev(y),
                                                            _stream(stream)))

    def backward(self, dy, grad, stream=None) -> None:
        _cnn_check(self.net, load_library().sfm_cnn_backward(self.net, _dev(dy), _dev(grad), _stream(stream)))

    def input_grad(self, dy, dx, stream=None) -> None:
        """dx = gradient of sum(dy * y) with respect to the inputs of the last forward pass."""
        _cnn_check(self.net, load_library().sfm_cnn_input_grad(self.net, _dev(dy), _dev(dx), _stream(stream)))

    def fit_scale(self, target, stream=None):
        mean = np.empty(self.n_out, np.float32)
        sd = np.empty(self.n_out, np.float32)
        _cnn_check(self.net, load_library().sfm_cnn_fit_scale(self.net, _dev(target), int(target.shape[0]), _ptr(mean),
                                                              _ptr(sd), _stream(stream)))
        return mean, sd

    def train(self, x, target, batch: int, epochs: int, lr: float, seed: int = 0, stream=None) -> np.ndarray:
        losses = np.zeros(max(epochs, 1), np.float64)
        _cnn_check(self.net, load_library().sfm_cnn_train(self.net, _dev(x), _dev(target), int(x.shape[0]),
                                                          int(batch), int(epochs), float(lr), int(seed),
                                                          _ptr(losses), _stream(stream)))
        return losses[:epochs]


def sfm_rom_inputs(ctx: int, vel, x, stream=None) -> None:
    _check(ctx, load_library().sfm_rom_inputs(ctx, _dev(vel), _dev(x), _stream(stream)))


def sfm_rom_targets(ctx: int, t, stream=None) -> None:
    _check(ctx, load_library().sfm_rom_targets(ctx, _dev(t), _stream(stream)))


def sfm_ntd_error(ctx: int, coef, f_peak: float, stream=None) -> np.ndarray:
    err = np.empty(sfm_query(ctx)["n_subdomains"], np.float64)
    _check(ctx, load_library().sfm_ntd_error(ctx, _dev(coef), float(f_peak), _ptr(err), _stream(stream)))
    return err


def sfm_surrogate_predict(ctx: int, net: "Cnn", vel, coef, stream=None) -> None:
    """coef (device float64 [S][2][k][p][p]) = the network's blocks, Gamma-hat_1 from the current ROMs."""
    _check(ctx, load_library().sfm_surrogate_predict(ctx, net.net, _dev(vel), _dev(coef), _stream(stream)))


def sfm_surrogate_velocity_gradient(ctx: int, net: "Cnn", vel, grad_gamma, grad_gamma_hat, grad_vel,
                                    stream=None) -> None:
    """grad_vel (device, nodes as vel) = dJ/dc through the network, from the block gradients
    grad_gamma / grad_gamma_hat (host float64 [S][k][p][p], as sfm_adjoint_gradient returns them)."""
    gg = _host(grad_gamma, np.float64)
    gh = _host(grad_gamma_hat, np.float64)
    info = sfm_query(ctx)
    need = info["n_subdomains"] * info["k"] * info["p"] ** 2
    if gg.size != need or gh.size != need:
        raise ValueError(f"block gradients need {need} entries each")
    _check(ctx, load_library().sfm_surrogate_velocity_gradient(ctx, net.net, _dev(vel), _ptr(gg), _ptr(gh),
                                                               _dev(grad_vel), _stream(stream)))


def sfm_build_roms_surrogate(ctx: int, net: "Cnn", tol: float, f_peak: float, vel, src_ijk=None, rec_ijk=None,
                             stream=None):
    """Returns (accepted [S] bool, ntd_err [S], seconds [4])."""
    src = _host(np.zeros((0, 3)) if src_ijk is None else src_ijk, np.int32).reshape(-1, 3)
    rec = _host(np.zeros((0, 3)) if rec_ijk is None else rec_ijk, np.int32).reshape(-1, 3)
    S = sfm_query(ctx)["n_subdomains"]
    acc = np.zeros(S, np.int32)
    err = np.zeros(S, np.float64)
    secs = np.zeros(4, np.float64)
    _check(ctx, load_library().sfm_build_roms_surrogate(ctx, net.net, float(tol), float(f_peak), _dev(vel), len(src),
                                                        _ptr(src), len(rec), _ptr(rec), _ptr(acc), _ptr(err),
                                                        _ptr(secs), _stream(stream)))
    return acc.astype(bool), err, secs
