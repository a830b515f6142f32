"""Python binding of the gfx950 HIP library ``libefwi.so`` (C ABI in ``include/efwi.h``).

Argument marshalling only: every step of the hot path runs in the library's HIP kernels.
Tensors are PyTorch device tensors (torch supplies device memory and the current HIP
stream); channel coordinates are host arrays. Importing this module fails loudly when the
library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libefwi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2305_14130_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

# status codes (efwi_status)
OK, E_INVAL, E_RANGE, E_CFL, E_WORKSPACE, E_HIP, E_NONFINITE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
CKPT_FP32, CKPT_BF16, CKPT_FP16 = 0, 1, 2
WS_FORWARD, WS_ADJOINT, WS_GRADIENT, WS_BATCH, WS_REGULARIZER = 0, 1, 2, 3, 4

EXPORTED = ["efwi_workspace_size", "efwi_validate", "efwi_model_forward", "efwi_model_adjoint",
            "efwi_shot_gradient", "efwi_shot_jt", "efwi_batch_gradient", "efwi_extension_regularizer",
            "efwi_status_string", "efwi_last_error", "efwi_version", "efwi_timing_enable",
            "efwi_timing_reset", "efwi_timing_query", "efwi_kernel_count", "efwi_kernel_name",
            "efwi_plan_interval", "efwi_set_tile_rows", "efwi_get_tile_rows", "efwi_autotune_workspace_size",
            "efwi_autotune", "efwi_batch_waves", "efwi_zoi_weights", "efwi_final_model",
            "efwi_pseudo_hessian", "efwi_das_field",
            "efwi_batch_gradient_grouped", "efwi_bspline_nodes", "efwi_bspline_expand",
            "efwi_bspline_adjoint", "efwi_shot_gradient_noalloc", "efwi_noalloc_scratch_bytes",
            "efwi_set_wave_cache_bytes", "efwi_get_wave_cache_bytes", "efwi_set_wave_lanes",
            "efwi_get_wave_lanes"]


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("nz", ctypes.c_int), ("ny", ctypes.c_int), ("nx", ctypes.c_int),
                ("dz", ctypes.c_float), ("dy", ctypes.c_float), ("dx", ctypes.c_float), ("dt", ctypes.c_float),
                ("nt", ctypes.c_int), ("npml", ctypes.c_int), ("pml_R", ctypes.c_float),
                ("pml_f0", ctypes.c_float), ("vp_max", ctypes.c_float), ("eps", ctypes.c_void_p)]


class _ShotC(ctypes.Structure):
    _fields_ = [("src_iz", ctypes.c_int), ("src_iy", ctypes.c_int), ("src_ix", ctypes.c_int),
                ("nch", ctypes.c_int), ("ch_iz", ctypes.POINTER(ctypes.c_int)),
                ("ch_iy", ctypes.POINTER(ctypes.c_int)), ("ch_ix", ctypes.POINTER(ctypes.c_int)),
                ("z0", ctypes.c_int), ("y0", ctypes.c_int), ("x0", ctypes.c_int),
                ("wz", ctypes.c_int), ("wy", ctypes.c_int), ("wx", ctypes.c_int),
                ("ckpt_interval", ctypes.c_int), ("ckpt_mode", ctypes.c_int),
                ("gauge", ctypes.c_int), ("decim", ctypes.c_int), ("rate", ctypes.c_int)]


@dataclass
class Shot:
    """One shot: source node, DAS channel nodes (full-model coordinates), window, checkpointing,
    DAS sampling (gauge channels, resampling factor, strain rate: see efwi_shot). The y
    fields are used on 3D grids only."""
    src_iz: int
    src_ix: int
    ch_iz: np.ndarray
    ch_ix: np.ndarray
    z0: int = 0
    x0: int = 0
    wz: int = 0
    wx: int = 0
    ckpt_interval: int = 0
    ckpt_mode: int = CKPT_FP32
    src_iy: int = 0
    ch_iy: np.ndarray = None
    y0: int = 0
    wy: int = 0
    gauge: int = 1
    decim: int = 1
    rate: bool = False
    _keep: list = field(default_factory=list, repr=False)

    @property
    def nch(self) -> int:
        return int(len(self.ch_iz))

    def data_shape(self, nt: int):
        """Shape of this shot's data for nt time steps: (nch, nt) for point strain, else
        (nch - gauge + 1, nt // decim)."""
        if self.nch == 0:
            return (0, nt // max(1, self.decim))
        return (self.nch - max(1, self.gauge) + 1, nt // max(1, self.decim))

    def c_struct(self) -> _ShotC:
        iz = np.ascontiguousarray(self.ch_iz, dtype=np.int32)
        ix = np.ascontiguousarray(self.ch_ix, dtype=np.int32)
        iy = None if self.ch_iy is None else np.ascontiguousarray(self.ch_iy, dtype=np.int32)
        self._keep[:] = [iz, ix, iy]
        ip = ctypes.POINTER(ctypes.c_int)
        return _ShotC(self.src_iz, self.src_iy, self.src_ix, len(iz), iz.ctypes.data_as(ip),
                      None if iy is None else iy.ctypes.data_as(ip), ix.ctypes.data_as(ip),
                      self.z0, self.y0, self.x0, self.wz, self.wy, self.wx, self.ckpt_interval, self.ckpt_mode,
                      int(self.gauge), int(self.decim), int(bool(self.rate)))


def make_grid(nz, nx, dz, dx, dt, nt, npml=0, pml_R=1e-3, pml_f0=10.0, vp_max=0.0, eps=None) -> Grid:
    """2D grid; eps: an FP32 device tensor [nz][nx] of Thomsen epsilon for a VTI medium
    (delta = eps / 2), kept alive by the grid, or None (isotropic)."""
    g = Grid(2, int(nz), 1, int(nx), float(dz), 1.0, float(dx), float(dt), int(nt), int(npml),
             float(pml_R), float(pml_f0), float(vp_max), None)
    if eps is not None:
        _f32(eps, "eps")
        if tuple(eps.shape) != (int(nz), int(nx)) or not eps.is_contiguous():
            raise ValueError("eps must be a contiguous [nz][nx] tensor")
        g.eps = eps.data_ptr()
        g._eps_ref = eps
    return g


def make_grid3d(nz, ny, nx, dz, dy, dx, dt, nt, npml=0, pml_R=1e-3, pml_f0=10.0, vp_max=0.0) -> Grid:
    return Grid(3, int(nz), int(ny), int(nx), float(dz), float(dy), float(dx), float(dt), int(nt), int(npml),
                float(pml_R), float(pml_f0), float(vp_max), None)


def n_components(grid: Grid) -> int:
    """Moment-tensor components of a source series: 3 in 2D (xx, zz, xz), 6 in 3D."""
    return 6 if grid.ndim == 3 else 3


_vp = ctypes.c_void_p
_lib.efwi_workspace_size.restype = ctypes.c_size_t
_lib.efwi_workspace_size.argtypes = [ctypes.c_int, ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(_ShotC)]
_lib.efwi_set_tile_rows.restype = ctypes.c_int
_lib.efwi_set_tile_rows.argtypes = [ctypes.c_int, ctypes.c_int]
_lib.efwi_get_tile_rows.restype = ctypes.c_int
_lib.efwi_get_tile_rows.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.efwi_set_wave_cache_bytes.restype = ctypes.c_int
_lib.efwi_set_wave_cache_bytes.argtypes = [ctypes.c_size_t]
_lib.efwi_get_wave_cache_bytes.restype = ctypes.c_size_t
_lib.efwi_get_wave_cache_bytes.argtypes = []
_lib.efwi_set_wave_lanes.restype = ctypes.c_int
_lib.efwi_set_wave_lanes.argtypes = [ctypes.c_int]
_lib.efwi_get_wave_lanes.restype = ctypes.c_int
_lib.efwi_get_wave_lanes.argtypes = []
_lib.efwi_autotune_workspace_size.restype = ctypes.c_size_t
_lib.efwi_autotune_workspace_size.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), ctypes.c_int]
_lib.efwi_autotune.restype = ctypes.c_int
_lib.efwi_autotune.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), _vp, _vp, ctypes.c_int, _vp,
                               ctypes.c_size_t, _vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_float)]
_lib.efwi_zoi_weights.restype = ctypes.c_int
_lib.efwi_final_model.restype = ctypes.c_int
_lib.efwi_batch_waves.restype = ctypes.c_int
_lib.efwi_batch_waves.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(_ShotC), ctypes.c_size_t,
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.efwi_plan_interval.restype = ctypes.c_int
_lib.efwi_plan_interval.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), ctypes.c_size_t]
_lib.efwi_validate.restype = ctypes.c_int
_lib.efwi_validate.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(_ShotC)]
_lib.efwi_model_forward.restype = ctypes.c_int
_lib.efwi_model_forward.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), _vp, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp]
_lib.efwi_model_adjoint.restype = ctypes.c_int
_lib.efwi_model_adjoint.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), _vp, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp]
_lib.efwi_shot_gradient.restype = ctypes.c_int
_lib.efwi_shot_gradient.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), _vp, _vp, _vp, _vp, _vp, _vp,
                                    _vp, ctypes.c_size_t, _vp]
_lib.efwi_shot_jt.restype = ctypes.c_int
_lib.efwi_shot_jt.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), _vp, _vp, _vp, _vp, _vp, _vp,
                              ctypes.c_size_t, _vp]
_lib.efwi_shot_gradient_noalloc.restype = ctypes.c_int
_lib.efwi_shot_gradient_noalloc.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), _vp, _vp, _vp, _vp, _vp,
                                            _vp, _vp]
_lib.efwi_noalloc_scratch_bytes.restype = ctypes.c_size_t
_lib.efwi_noalloc_scratch_bytes.argtypes = []
_lib.efwi_batch_gradient.restype = ctypes.c_int
_lib.efwi_batch_gradient.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(_ShotC), _vp, _vp, _vp,
                                     _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.efwi_extension_regularizer.restype = ctypes.c_int
_lib.efwi_extension_regularizer.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, _vp, _vp, _vp, ctypes.c_float, _vp,
                                            _vp, _vp, ctypes.c_size_t, _vp]
_lib.efwi_status_string.restype = ctypes.c_char_p
_lib.efwi_status_string.argtypes = [ctypes.c_int]
_lib.efwi_last_error.restype = ctypes.c_char_p
_lib.efwi_last_error.argtypes = []
_lib.efwi_version.restype = ctypes.c_char_p
_lib.efwi_version.argtypes = []
_lib.efwi_timing_enable.restype = ctypes.c_int
_lib.efwi_timing_enable.argtypes = [ctypes.c_int]
_lib.efwi_timing_reset.restype = ctypes.c_int
_lib.efwi_timing_reset.argtypes = []
_lib.efwi_timing_query.restype = ctypes.c_int
_lib.efwi_timing_query.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long),
                                   ctypes.POINTER(ctypes.c_double)]
_lib.efwi_kernel_count.restype = ctypes.c_int
_lib.efwi_kernel_count.argtypes = []
_lib.efwi_kernel_name.restype = ctypes.c_char_p
_lib.efwi_kernel_name.argtypes = [ctypes.c_int]


class EfwiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_lib.efwi_status_string(status).decode()}: {message}")
        self.status = status


def _check(rc: int):
    if rc != OK:
        raise EfwiError(rc, _lib.efwi_last_error().decode())


def version() -> str:
    return _lib.efwi_version().decode()


def timing_enable(sample_every: int) -> None:
    """Bracket every k-th launch of each kernel kind with HIP events (0 = off)."""
    _check(_lib.efwi_timing_enable(int(sample_every)))


def timing_reset() -> None:
    _check(_lib.efwi_timing_reset())


def timing_query() -> dict:
    """{kernel name: (launches, timed launches, mean ms per timed launch)}."""
    out = {}
    for k in range(_lib.efwi_kernel_count()):
        la, ti, ms = ctypes.c_long(), ctypes.c_long(), ctypes.c_double()
        _check(_lib.efwi_timing_query(k, ctypes.byref(la), ctypes.byref(ti), ctypes.byref(ms)))
        name = _lib.efwi_kernel_name(k).decode()
        out[name] = (la.value, ti.value, ms.value / ti.value if ti.value else 0.0)
    return out


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _f32(t, name):
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 device tensor")
    return t


# The C ABI takes raw pointers: every tensor is checked here, before its pointer is passed,
# for dtype, exact shape (or element count) and contiguity, and then all of a call's tensors
# for being device tensors on one device, so that a wrongly shaped or placed tensor raises
# instead of becoming an out-of-bounds device access. (Shapes are checked first so that the
# checks can be exercised without a GPU.)
def _arg(t, name, shape, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype:
        raise TypeError(f"{name} must be a {dtype} tensor")
    want = tuple(int(x) for x in shape)
    if tuple(t.shape) != want:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _opt(t, name, shape, dtype=torch.float32):
    return None if t is None else _arg(t, name, shape, dtype)


def _flat(t, name, numel, dtype=torch.float32):
    """A tensor of any shape holding exactly numel contiguous elements (concatenated data)."""
    if not isinstance(t, torch.Tensor) or t.dtype != dtype:
        raise TypeError(f"{name} must be a {dtype} tensor")
    if t.numel() != int(numel):
        raise ValueError(f"{name} holds {t.numel()} elements, expected {int(numel)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ws(ws):
    if not isinstance(ws, torch.Tensor) or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise TypeError("ws must be a contiguous uint8 tensor (see workspace())")
    return ws


def _device(**tensors):
    """The one device of a call's tensors (None entries are skipped)."""
    dev = None
    for name, t in tensors.items():
        if t is None:
            continue
        if not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{name} is on {t.device}, the call's other tensors on {dev}")
    return dev


def space(grid: Grid):
    """Grid points of one model parameter: (nz, nx), or (nz, ny, nx) in 3D."""
    return (grid.nz, grid.ny, grid.nx) if grid.ndim == 3 else (grid.nz, grid.nx)


def model_shape(grid: Grid):
    """(3, nz, nx) or (3, nz, ny, nx): a model (Vp, Vs, rho) or its gradient."""
    return (3,) + space(grid)


def _data_shape(grid: Grid, shot) -> tuple:
    return tuple(shot.data_shape(grid.nt))


def validate(grid: Grid, shots) -> None:
    arr = (_ShotC * len(shots))(*[s.c_struct() for s in shots])
    _check(_lib.efwi_validate(ctypes.byref(grid), len(shots), arr))


def workspace_size(kind: int, grid: Grid, shots) -> int:
    shots = list(shots)
    arr = (_ShotC * max(1, len(shots)))(*[s.c_struct() for s in shots])
    n = _lib.efwi_workspace_size(kind, ctypes.byref(grid), len(shots), arr)
    if n == 0 and kind != WS_REGULARIZER:
        raise EfwiError(_lib.efwi_validate(ctypes.byref(grid), len(shots), arr), _lib.efwi_last_error().decode())
    return int(n)


def plan_interval(grid: Grid, shot: Shot, budget_bytes: int) -> int:
    """Largest checkpoint interval whose gradient workspace fits the budget (nt: the whole
    forward history is kept and nothing is recomputed)."""
    sc = shot.c_struct()
    L = _lib.efwi_plan_interval(ctypes.byref(grid), ctypes.byref(sc), int(budget_bytes))
    _check(min(L, 0))
    return int(L)


def set_tile_rows(fwd_rows: int = 0, adj_rows: int = 0) -> None:
    """Rows of the fused forward / transposed step tiles (8, 12 or 16; 0 keeps a value)."""
    _check(_lib.efwi_set_tile_rows(int(fwd_rows), int(adj_rows)))


def set_wave_cache_bytes(nbytes: int) -> None:
    """Per-step state bound of a 2D wave (0: the default 256 MiB; -1: the workspace alone)."""
    _check(_lib.efwi_set_wave_cache_bytes(ctypes.c_size_t(nbytes if nbytes >= 0 else 2**64 - 1)))


def get_wave_cache_bytes() -> int:
    return int(_lib.efwi_get_wave_cache_bytes())


def set_wave_lanes(lanes: int) -> None:
    """Lanes of a 2D batch: 1, or 2 (waves alternate between two streams, each in half of
    the workspace); 0 restores the default."""
    _check(_lib.efwi_set_wave_lanes(int(lanes)))


def get_wave_lanes() -> int:
    return int(_lib.efwi_get_wave_lanes())


def get_tile_rows():
    f, a = ctypes.c_int(), ctypes.c_int()
    _check(_lib.efwi_get_tile_rows(ctypes.byref(f), ctypes.byref(a)))
    return f.value, a.value


def autotune(grid: Grid, shot: Shot, m, src, steps: int = 16, stream=None, times=None):
    """Time the shot's forward and transposed sweeps over `steps` steps for each tile height,
    keep the fastest for each (process-wide) and return (fwd_rows, adj_rows). With a dict
    `times`, also fill {rows: (forward ms, transposed ms)}."""
    _arg(m, "m", model_shape(grid))
    _arg(src, "src", (n_components(grid), grid.nt))
    _device(m=m, src=src)
    sc = shot.c_struct()
    need = _lib.efwi_autotune_workspace_size(ctypes.byref(grid), ctypes.byref(sc), int(steps))
    if need == 0:
        _check(_lib.efwi_validate(ctypes.byref(grid), 1, ctypes.byref(sc)))
        raise EfwiError(E_UNSUPPORTED, "autotune needs a 2D grid and steps >= 1")
    ws = workspace(need, m.device)
    f, a = ctypes.c_int(), ctypes.c_int()
    tm = (ctypes.c_float * 6)()
    _check(_lib.efwi_autotune(ctypes.byref(grid), ctypes.byref(sc), _ptr(m), _ptr(src), int(steps), _ptr(ws),
                              ws.numel(), _stream(stream), ctypes.byref(f), ctypes.byref(a), tm))
    if times is not None:
        for k, rows in enumerate((8, 12, 16)):
            times[rows] = (tm[2 * k], tm[2 * k + 1])
    return f.value, a.value


def recompute_fraction(grid: Grid, interval: int) -> float:
    """Share of the nt steps that the reverse sweep recomputes for a checkpoint interval
    (0: ceil(sqrt(nt))): every segment but the last, which the first sweep keeps."""
    nt = grid.nt
    L = interval if interval > 0 else int(np.ceil(np.sqrt(nt)))
    L = max(1, min(L, nt))
    return (-(-nt // L) - 1) * L / nt


def workspace(nbytes: int, device=None) -> torch.Tensor:
    return torch.empty(max(256, nbytes), dtype=torch.uint8, device=device or "cuda")


def model_forward(grid: Grid, shot: Shot, m, src, d=None, ws=None, stream=None):
    """d = K u(m): DAS data of one shot, shot.data_shape(nt) (point strain [nch][nt] by
    default)."""
    _arg(m, "m", model_shape(grid))
    dev = m.device
    _arg(src, "src", (n_components(grid), grid.nt))
    if d is None:
        d = torch.empty(shot.data_shape(grid.nt), dtype=torch.float32, device=dev)
    _arg(d, "d", _data_shape(grid, shot))
    _device(m=m, src=src, d=d, ws=ws)
    sc = shot.c_struct()
    need = _lib.efwi_workspace_size(WS_FORWARD, ctypes.byref(grid), 1, ctypes.byref(sc))
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_model_forward(ctypes.byref(grid), ctypes.byref(sc), _ptr(m), _ptr(src), _ptr(d), _ptr(ws),
                                   ws.numel(), _stream(stream)))
    return d


def model_adjoint(grid: Grid, shot: Shot, m, r, src_bar=None, ws=None, stream=None):
    """L^T r with respect to the [3][nt] source components."""
    _arg(m, "m", model_shape(grid))
    dev = m.device
    _arg(r, "r", _data_shape(grid, shot))
    if src_bar is None:
        src_bar = torch.empty((n_components(grid), grid.nt), dtype=torch.float32, device=dev)
    _arg(src_bar, "src_bar", (n_components(grid), grid.nt))
    _device(m=m, r=r, src_bar=src_bar, ws=ws)
    sc = shot.c_struct()
    need = _lib.efwi_workspace_size(WS_ADJOINT, ctypes.byref(grid), 1, ctypes.byref(sc))
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_model_adjoint(ctypes.byref(grid), ctypes.byref(sc), _ptr(m), _ptr(r), _ptr(src_bar),
                                   _ptr(ws), ws.numel(), _stream(stream)))
    return src_bar


def shot_gradient(grid: Grid, shot: Shot, m, src, d_obs, g=None, phi=None, d_out=None, ws=None, stream=None):
    """Misfit phi_s (device double) and gradient g_s [3][nz][nx] w.r.t. (Vp, Vs, rho)."""
    _arg(m, "m", model_shape(grid))
    dev = m.device
    _arg(src, "src", (n_components(grid), grid.nt))
    _arg(d_obs, "d_obs", _data_shape(grid, shot))
    if g is None:
        g = torch.empty_like(m)
    if phi is None:
        phi = torch.empty((), dtype=torch.float64, device=dev)
    _arg(g, "g", model_shape(grid))
    _flat(phi, "phi", 1, torch.float64)
    _opt(d_out, "d_out", _data_shape(grid, shot))
    _device(m=m, src=src, d_obs=d_obs, g=g, phi=phi, d_out=d_out, ws=ws)
    sc = shot.c_struct()
    need = _lib.efwi_workspace_size(WS_GRADIENT, ctypes.byref(grid), 1, ctypes.byref(sc))
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_shot_gradient(ctypes.byref(grid), ctypes.byref(sc), _ptr(m), _ptr(src), _ptr(d_obs), _ptr(g),
                                   _ptr(phi), _ptr(d_out), _ptr(ws), ws.numel(), _stream(stream)))
    return g, phi


def noalloc_scratch_bytes() -> int:
    """Scratch bytes of shot_gradient_noalloc (one library-owned array per GPU)."""
    return int(_lib.efwi_noalloc_scratch_bytes())


def shot_gradient_noalloc(grid: Grid, shot: Shot, m, src, d_obs, g, phi, d_out=None, stream=None):
    """shot_gradient for callers that cannot allocate: no workspace, the outputs g [3][...]
    and phi (float64, one element) passed in; the library's per-GPU scratch array instead
    (efwi_shot_gradient_noalloc). Allocates nothing."""
    _arg(m, "m", model_shape(grid))
    _arg(src, "src", (n_components(grid), grid.nt))
    _arg(d_obs, "d_obs", _data_shape(grid, shot))
    _arg(g, "g", model_shape(grid))
    _flat(phi, "phi", 1, torch.float64)
    _opt(d_out, "d_out", _data_shape(grid, shot))
    _device(m=m, src=src, d_obs=d_obs, g=g, phi=phi, d_out=d_out)
    sc = shot.c_struct()
    _check(_lib.efwi_shot_gradient_noalloc(ctypes.byref(grid), ctypes.byref(sc), _ptr(m), _ptr(src), _ptr(d_obs),
                                           _ptr(g), _ptr(phi), _ptr(d_out), _stream(stream)))
    return g, phi


def shot_jt(grid: Grid, shot: Shot, m, src, v, g=None, d_out=None, ws=None, stream=None):
    """g = J_s^T v for a data-space vector v [nch][nt] (backward of m -> d)."""
    _arg(m, "m", model_shape(grid))
    dev = m.device
    _arg(src, "src", (n_components(grid), grid.nt))
    _arg(v, "v", _data_shape(grid, shot))
    if g is None:
        g = torch.empty_like(m)
    _arg(g, "g", model_shape(grid))
    _opt(d_out, "d_out", _data_shape(grid, shot))
    _device(m=m, src=src, v=v, g=g, d_out=d_out, ws=ws)
    sc = shot.c_struct()
    need = _lib.efwi_workspace_size(WS_GRADIENT, ctypes.byref(grid), 1, ctypes.byref(sc))
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_shot_jt(ctypes.byref(grid), ctypes.byref(sc), _ptr(m), _ptr(src), _ptr(v), _ptr(g),
                             _ptr(d_out), _ptr(ws), ws.numel(), _stream(stream)))
    return g


def batch_gradient(grid: Grid, shots, m_ext, src, d_obs, g_ext=None, phi=None, ws=None, stream=None):
    """Data term of the extended misfit for all shots: g_ext[s] = J_s^T r_s on m_ext[s]."""
    shots = list(shots)
    ns = len(shots)
    _arg(m_ext, "m_ext", (ns,) + model_shape(grid))
    dev = m_ext.device
    _arg(src, "src", (ns, n_components(grid), grid.nt))
    _flat(d_obs, "d_obs", sum(int(np.prod(_data_shape(grid, s))) for s in shots))
    if g_ext is None:
        g_ext = torch.empty_like(m_ext)
    if phi is None:
        phi = torch.empty((ns,), dtype=torch.float64, device=dev)
    _arg(g_ext, "g_ext", (ns,) + model_shape(grid))
    _flat(phi, "phi", ns, torch.float64)
    _device(m_ext=m_ext, src=src, d_obs=d_obs, g_ext=g_ext, phi=phi, ws=ws)
    arr = (_ShotC * len(shots))(*[s.c_struct() for s in shots])
    need = _lib.efwi_workspace_size(WS_BATCH, ctypes.byref(grid), len(shots), arr)
    if need == 0:
        _check(_lib.efwi_validate(ctypes.byref(grid), len(shots), arr))
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_batch_gradient(ctypes.byref(grid), len(shots), arr, _ptr(m_ext), _ptr(src), _ptr(d_obs),
                                    _ptr(g_ext), _ptr(phi), _ptr(ws), ws.numel(), _stream(stream)))
    return g_ext, phi


def batch_gradient_grouped(grid: Grid, shots, groups, m_ext, src, d_obs, g_ext=None, phi=None, ws=None,
                           stream=None):
    """Data term with the model extended along groups of shots: shot s on m_ext[groups[s]],
    g_ext[k] = sum of the gradients of the shots of group k (efwi_batch_gradient_grouped)."""
    shots = list(shots)
    grp = np.ascontiguousarray(groups, dtype=np.int32)
    if grp.shape != (len(shots),):
        raise ValueError("one group index per shot")
    ns = len(shots)
    if not isinstance(m_ext, torch.Tensor) or m_ext.dim() < 1:
        raise TypeError("m_ext must be a [ng][3][...] tensor")
    ng = int(m_ext.shape[0])
    _arg(m_ext, "m_ext", (ng,) + model_shape(grid))
    dev = m_ext.device
    if ns and (grp.min() < 0 or grp.max() >= ng):
        raise ValueError(f"group indices must lie in [0, {ng})")
    _arg(src, "src", (ns, n_components(grid), grid.nt))
    _flat(d_obs, "d_obs", sum(int(np.prod(_data_shape(grid, s))) for s in shots))
    if g_ext is None:
        g_ext = torch.empty_like(m_ext)
    if phi is None:
        phi = torch.empty((ns,), dtype=torch.float64, device=dev)
    _arg(g_ext, "g_ext", (ng,) + model_shape(grid))
    _flat(phi, "phi", ns, torch.float64)
    _device(m_ext=m_ext, src=src, d_obs=d_obs, g_ext=g_ext, phi=phi, ws=ws)
    arr = (_ShotC * len(shots))(*[s.c_struct() for s in shots])
    need = _lib.efwi_workspace_size(WS_BATCH, ctypes.byref(grid), len(shots), arr)
    if need == 0:
        _check(_lib.efwi_validate(ctypes.byref(grid), len(shots), arr))
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_batch_gradient_grouped(ctypes.byref(grid), len(shots), arr,
                                            grp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), m_ext.shape[0],
                                            _ptr(m_ext), _ptr(src), _ptr(d_obs), _ptr(g_ext), _ptr(phi), _ptr(ws),
                                            ws.numel(), _stream(stream)))
    return g_ext, phi


def batch_waves(grid: Grid, shots, ws_bytes: int, with_lanes: bool = False):
    """The waves that batch_gradient advances for a workspace of ws_bytes, in order, each as
    the list of its shots' indices (see efwi_batch_waves); with_lanes: (waves, lanes)."""
    shots = list(shots)
    arr = (_ShotC * len(shots))(*[s.c_struct() for s in shots])
    n, lanes = ctypes.c_int(), ctypes.c_int()
    first = (ctypes.c_int * max(1, len(shots)))()
    order = (ctypes.c_int * max(1, len(shots)))()
    _check(_lib.efwi_batch_waves(ctypes.byref(grid), len(shots), arr, ctypes.c_size_t(ws_bytes), ctypes.byref(n),
                                 first, order, ctypes.byref(lanes)))
    starts = list(first[:n.value]) + [len(shots)]
    waves = [list(order[starts[w]:starts[w + 1]]) for w in range(n.value)]
    return (waves, lanes.value) if with_lanes else waves


def extension_regularizer(grid: Grid, m_ext, b, sink, eta, g_ext, phi=None, ws=None, stream=None):
    """phi_reg (device double) and g_ext += gradient of 1/2 eta^2 ||(I - S^T S_w) W m~||^2."""
    if not isinstance(m_ext, torch.Tensor) or m_ext.dim() < 1:
        raise TypeError("m_ext must be a [ns][3][...] tensor")
    ns = int(m_ext.shape[0])
    _arg(m_ext, "m_ext", (ns,) + model_shape(grid))
    dev = m_ext.device
    _arg(b, "b", (ns,) + space(grid))
    _arg(sink, "sink", (ns,) + space(grid), torch.uint8)
    _arg(g_ext, "g_ext", (ns,) + model_shape(grid))
    if phi is None:
        phi = torch.empty((), dtype=torch.float64, device=dev)
    _flat(phi, "phi", 1, torch.float64)
    _device(m_ext=m_ext, b=b, sink=sink, g_ext=g_ext, phi=phi, ws=ws)
    need = _lib.efwi_workspace_size(WS_REGULARIZER, ctypes.byref(grid), 0, None)
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_extension_regularizer(ctypes.byref(grid), ns, _ptr(m_ext), _ptr(b), _ptr(sink),
                                           float(eta), _ptr(g_ext), _ptr(phi), _ptr(ws), ws.numel(),
                                           _stream(stream)))
    return phi


class Zone(ctypes.Structure):
    """One source's zone of influence (efwi_zoi): sinkhole centre (z, y, x) and inverse
    covariance (zz, yy, xx, zy, zx, yx) in metres, active box (z0, z1, y0, y1, x0, x1), outer
    taper width."""
    _fields_ = [("src", ctypes.c_float * 3), ("icov", ctypes.c_float * 6), ("box", ctypes.c_float * 6),
                ("taper", ctypes.c_float)]


_lib.efwi_zoi_weights.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(Zone), ctypes.c_float,
                                  ctypes.c_float, _vp, _vp, _vp]
_lib.efwi_final_model.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
_lib.efwi_batch_gradient_grouped.restype = ctypes.c_int
_lib.efwi_batch_gradient_grouped.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(_ShotC),
                                             ctypes.POINTER(ctypes.c_int), ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp,
                                             ctypes.c_size_t, _vp]
_lib.efwi_bspline_nodes.restype = ctypes.c_int
_lib.efwi_bspline_nodes.argtypes = [ctypes.c_int, ctypes.c_int]
for _name in ("efwi_bspline_expand", "efwi_bspline_adjoint"):
    getattr(_lib, _name).restype = ctypes.c_int
    getattr(_lib, _name).argtypes = [ctypes.c_int] * 5 + [_vp, _vp, _vp]
_lib.efwi_das_field.restype = ctypes.c_int
_lib.efwi_das_field.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(_ShotC), _vp, _vp, _vp]
_lib.efwi_pseudo_hessian.restype = ctypes.c_int
_lib.efwi_pseudo_hessian.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(_ShotC), _vp, _vp,
                                     ctypes.c_float, _vp, _vp, _vp, ctypes.c_size_t, _vp]


def make_zone(src, icov, box, taper) -> Zone:
    return Zone((ctypes.c_float * 3)(*src), (ctypes.c_float * 6)(*icov), (ctypes.c_float * 6)(*box), float(taper))


def zoi_weights(grid: Grid, zones, n, nu, b=None, sink=None, device=None, stream=None):
    """ZOI weights b [Ns][...] (FP32) and sinkhole flags (uint8) of eq.(10) on the full grid."""
    zones = list(zones)
    shape = (grid.nz, grid.ny, grid.nx) if grid.ndim == 3 else (grid.nz, grid.nx)
    dev = device if device is not None else torch.device("cuda")
    if b is None:
        b = torch.empty((len(zones),) + shape, dtype=torch.float32, device=dev)
    if sink is None:
        sink = torch.empty((len(zones),) + shape, dtype=torch.uint8, device=b.device)
    _arg(b, "b", (len(zones),) + shape)
    _arg(sink, "sink", (len(zones),) + shape, torch.uint8)
    _device(b=b, sink=sink)
    arr = (Zone * len(zones))(*zones)
    _check(_lib.efwi_zoi_weights(ctypes.byref(grid), len(zones), arr, float(n), float(nu), _ptr(b), _ptr(sink),
                                 _stream(stream)))
    return b, sink


def final_model(grid: Grid, m_ext, b, sink, m_out=None, stream=None):
    """Physical model S_w W m~ of eq.(9), [3][...] FP32."""
    if not isinstance(m_ext, torch.Tensor) or m_ext.dim() < 1:
        raise TypeError("m_ext must be a [ns][3][...] tensor")
    ns = int(m_ext.shape[0])
    _arg(m_ext, "m_ext", (ns,) + model_shape(grid))
    dev = m_ext.device
    _arg(b, "b", (ns,) + space(grid))
    _arg(sink, "sink", (ns,) + space(grid), torch.uint8)
    if m_out is None:
        m_out = torch.empty(model_shape(grid), dtype=torch.float32, device=dev)
    _arg(m_out, "m_out", model_shape(grid))
    _device(m_ext=m_ext, b=b, sink=sink, m_out=m_out)
    _check(_lib.efwi_final_model(ctypes.byref(grid), m_ext.shape[0], _ptr(m_ext), _ptr(b), _ptr(sink), _ptr(m_out),
                                 _stream(stream)))
    return m_out


def bspline_nodes(n: int, spacing: int) -> int:
    """Cubic B-spline nodes along an axis of n cells with the given node spacing (cells)."""
    return int(_lib.efwi_bspline_nodes(int(n), int(spacing)))


def bspline_expand(c, nz: int, nx: int, dz_nodes: int, dx_nodes: int, out=None, stream=None):
    """Model planes [..][nz][nx] from cubic B-spline coefficients c [..][Nz][Nx]."""
    if not isinstance(c, torch.Tensor) or c.dim() < 2:
        raise TypeError("c must be a [..][Nz][Nx] tensor")
    lead = tuple(c.shape[:-2])
    _arg(c, "c", lead + (bspline_nodes(nz, dz_nodes), bspline_nodes(nx, dx_nodes)))
    if out is None:
        out = torch.empty(lead + (nz, nx), dtype=torch.float32, device=c.device)
    _arg(out, "out", lead + (nz, nx))
    _device(c=c, out=out)
    np_ = int(np.prod(lead)) if len(lead) else 1
    _check(_lib.efwi_bspline_expand(nz, nx, dz_nodes, dx_nodes, np_, _ptr(c), _ptr(out), _stream(stream)))
    return out


def bspline_adjoint(g, dz_nodes: int, dx_nodes: int, out=None, stream=None):
    """Coefficient gradients [..][Nz][Nx] from model-plane gradients g [..][nz][nx]."""
    if not isinstance(g, torch.Tensor) or g.dim() < 2:
        raise TypeError("g must be a [..][nz][nx] tensor")
    lead, (nz, nx) = tuple(g.shape[:-2]), tuple(g.shape[-2:])
    _arg(g, "g", lead + (nz, nx))
    shape = lead + (bspline_nodes(nz, dz_nodes), bspline_nodes(nx, dx_nodes))
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=g.device)
    _arg(out, "out", shape)
    _device(g=g, out=out)
    np_ = int(np.prod(lead)) if len(lead) else 1
    _check(_lib.efwi_bspline_adjoint(nz, nx, dz_nodes, dx_nodes, np_, _ptr(g), _ptr(out), _stream(stream)))
    return out


def das_field(grid: Grid, shot: Shot, e, out=None, stream=None):
    """Field data K e of the shot's DAS sampling from point strains e [nch][nt]."""
    _arg(e, "e", (shot.nch, grid.nt))
    if out is None:
        out = torch.empty(shot.data_shape(grid.nt), dtype=torch.float32, device=e.device)
    _arg(out, "out", _data_shape(grid, shot))
    _device(e=e, out=out)
    sc = shot.c_struct()
    _check(_lib.efwi_das_field(ctypes.byref(grid), ctypes.byref(sc), _ptr(e), _ptr(out), _stream(stream)))
    return out


def pseudo_hessian(grid: Grid, shots, m_ext, src, clip, h=None, p=None, ws=None, stream=None):
    """Approximate inverse pseudo-Hessian (efwi_pseudo_hessian): returns (h, p), the summed
    velocity autocorrelation and the clipped, scaled inverse, [nz][nx] FP32 each."""
    shots = list(shots)
    ns = len(shots)
    _arg(m_ext, "m_ext", (ns,) + model_shape(grid))
    dev = m_ext.device
    _arg(src, "src", (ns, n_components(grid), grid.nt))
    shape = space(grid)
    h = h if h is not None else torch.empty(shape, dtype=torch.float32, device=dev)
    p = p if p is not None else torch.empty(shape, dtype=torch.float32, device=dev)
    _arg(h, "h", shape), _arg(p, "p", shape)
    _device(m_ext=m_ext, src=src, h=h, p=p, ws=ws)
    arr = (_ShotC * len(shots))(*[s.c_struct() for s in shots])
    need = _lib.efwi_workspace_size(WS_BATCH, ctypes.byref(grid), len(shots), arr)
    if need == 0:
        _check(_lib.efwi_validate(ctypes.byref(grid), len(shots), arr))
    ws = _ws(ws if ws is not None else workspace(need, dev))
    _check(_lib.efwi_pseudo_hessian(ctypes.byref(grid), len(shots), arr, _ptr(m_ext), _ptr(src), float(clip), _ptr(h),
                                    _ptr(p), _ptr(ws), ws.numel(), _stream(stream)))
    return h, p

