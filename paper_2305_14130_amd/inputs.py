"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method (no propagation, staging, absorbing
boundary, misfit, gradient or regularizer): it only draws models, source and channel
geometry, moment tensors and source time functions from fixed seeds, in the shapes and
value distributions of the paper's guided-wave settings (a low-velocity reservoir layer
crossed by a horizontal DAS well with in-layer moment-tensor sources; the paper's field
data and its synthetic model's exact geometry are not available, so these stand in).

All arrays are NumPy float64 (the caller casts); models are [3][nz][nx] = (Vp, Vs, rho).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter


@dataclass
class Shot2D:
    src_iz: int
    src_ix: int
    M: np.ndarray              # (Mxx, Mzz, Mxz)
    ch_iz: np.ndarray          # [nch] int32
    ch_ix: np.ndarray          # [nch] int32
    # subdomain window into the full model (batched form); whole model when w* == 0
    z0: int = 0
    x0: int = 0
    wz: int = 0
    wx: int = 0


@dataclass
class Workload2D:
    name: str
    nz: int
    nx: int
    dz: float
    dx: float
    dt: float
    nt: int
    npml: int
    f0: float                  # Ricker central frequency
    vp_max: float
    stf: np.ndarray            # [nt] moment-rate s(t_{n+1/2})
    m_start: np.ndarray        # [3][nz][nx]
    m_true: np.ndarray         # [3][nz][nx]
    shots: list = field(default_factory=list)
    pml_R: float = 1e-3


def ricker(nt, dt, f0, amp=1.0):
    """Ricker wavelet with delay 1.5/f0 and unit peak, sampled at t_{n+1/2} = (n + 1/2) dt."""
    t = (np.arange(nt) + 0.5) * dt
    tau = t - 1.5 / f0
    a = (math.pi * f0 * tau) ** 2
    return amp * (1.0 - 2.0 * a) * np.exp(-a)


def smooth_random_field(shape, corr_cells, seed, max_abs):
    """White N(0,1) noise smoothed by a Gaussian of sigma = corr_cells / 2 (correlation
    ~exp(-r^2/corr^2)), rescaled so that max|field| = max_abs."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    s = gaussian_filter(w, sigma=corr_cells / 2.0, mode="reflect")
    return s * (max_abs / np.max(np.abs(s)))


def gaussian_blob(shape, cz, cx, sigma, amp):
    z = np.arange(shape[0])[:, None]
    x = np.arange(shape[1])[None, :]
    return amp * np.exp(-((z - cz) ** 2 + (x - cx) ** 2) / (2.0 * sigma ** 2))


# ---------------------------------------------------------------------------------------
# Parity workload: 100 x 200, dx = 5 m, three layers with a 20 m low-velocity layer.
# ---------------------------------------------------------------------------------------
def parity_2d(nt=1000, M0=1.0e16, blob_amp=0.03):
    nz, nx, h = 100, 200, 5.0
    vp = np.full((nz, nx), 3600.0)
    rho = np.full((nz, nx), 2450.0)
    vp[48:52] = 3000.0          # 4 cells = 20 m low-velocity layer (waveguide)
    rho[48:52] = 2300.0
    vp[52:] = 4500.0
    rho[52:] = 2600.0
    vs = vp / 1.7
    m_start = np.stack([vp, vs, rho])
    blob = gaussian_blob((nz, nx), 50, 110, 4.0, blob_amp)
    m_true = m_start.copy()
    m_true[0] *= 1.0 + blob
    m_true[1] *= 1.0 + blob
    ch_ix = (60 + 3 * np.arange(40)).astype(np.int32)
    ch_iz = np.full(40, 50, np.int32)
    shot = Shot2D(src_iz=50, src_ix=40, M=np.array([M0, M0, 0.0]), ch_iz=ch_iz, ch_ix=ch_ix)
    return Workload2D(name="parity-2d-100x200", nz=nz, nx=nx, dz=h, dx=h, dt=0.5e-3, nt=nt,
                      npml=20, f0=30.0, vp_max=4500.0, stf=ricker(nt, 0.5e-3, 30.0),
                      m_start=m_start, m_true=m_true, shots=[shot])


# ---------------------------------------------------------------------------------------
# Plain per-shot workload: 1000 x 3000, dx = 2.5 m, shale with a 15 m reservoir layer.
# ---------------------------------------------------------------------------------------
def _shale_model(nz, nx, h, res_top, res_bot, seed=14130, corr_m=50.0, anomalies=True):
    vp = np.full((nz, nx), 3800.0)
    ratio = np.full((nz, nx), 0.6)
    rho = np.full((nz, nx), 2550.0)
    vp[res_top:res_bot] = 3400.0
    ratio[res_top:res_bot] = 0.55
    rho[res_top:res_bot] = 2450.0
    vs = vp * ratio
    m = np.stack([vp, vs, rho])
    if anomalies:
        for k in range(3):
            m[k] = m[k] * (1.0 + smooth_random_field((nz, nx), corr_m / h, seed + k, 0.05))
    return m


def _mt_components(rng, M0):
    M = rng.uniform(-1.0, 1.0, 3)
    frob = math.sqrt(M[0] ** 2 + M[1] ** 2 + 2.0 * M[2] ** 2)
    return M * (M0 / frob)


def plain_2d(nz=1000, nx=3000, nt=4000, nshots=20, nch=1500, M0=1.0e16, anomalies=True):
    """Grid 1000 x 3000 at 2.5 m, nt = 4000 at 0.25 ms, 40-cell CPML, Ricker 60 Hz, 20
    moment-tensor sources in the layer, 1500 DAS e_xx channels along the well (iz = 500)."""
    h = 2.5
    res_top, res_bot = nz // 2 - 3, nz // 2 + 3
    m_true = _shale_model(nz, nx, h, res_top, res_bot, anomalies=anomalies)
    m_start = _shale_model(nz, nx, h, res_top, res_bot, anomalies=False)
    rng = np.random.default_rng(2305)
    iz = nz // 2
    ch_ix = (nx // 4 + np.arange(nch)).astype(np.int32)
    ch_iz = np.full(nch, iz, np.int32)
    shots = []
    span = max(1, (nx // 2) // max(1, nshots))
    for k in range(nshots):
        shots.append(Shot2D(src_iz=iz, src_ix=int(nx * 4 // 15 + span * k),
                            M=_mt_components(rng, M0), ch_iz=ch_iz, ch_ix=ch_ix))
    return Workload2D(name=f"plain-2d-{nz}x{nx}", nz=nz, nx=nx, dz=h, dx=h, dt=0.25e-3, nt=nt,
                      npml=40, f0=60.0, vp_max=3800.0 * 1.05, stf=ricker(nt, 0.25e-3, 60.0),
                      m_start=m_start, m_true=m_true, shots=shots)


def differentiation_2d(nz=1200, nx=4000, nt=8000, nshots=32, nch=2000, M0=1.0e16, anomalies=True):
    """The shale geology resampled to 2 m: grid 1200 x 4000, nt = 8000 at 0.2 ms, 40-cell
    CPML, Ricker 60 Hz, a reservoir of 8 cells (16 m) at mid depth, 32 moment-tensor sources
    along the well in the layer and 2000 DAS e_xx channels one cell apart (iz = nz / 2)."""
    h, dt = 2.0, 0.2e-3
    res_top, res_bot = nz // 2 - 4, nz // 2 + 4
    m_true = _shale_model(nz, nx, h, res_top, res_bot, anomalies=anomalies)
    m_start = _shale_model(nz, nx, h, res_top, res_bot, anomalies=False)
    rng = np.random.default_rng(2305)
    iz = nz // 2
    ch_ix = (nx // 4 + np.arange(nch)).astype(np.int32)
    ch_iz = np.full(nch, iz, np.int32)
    span = max(1, nch // max(1, nshots))
    shots = [Shot2D(src_iz=iz, src_ix=int(nx // 4 + span // 2 + span * k), M=_mt_components(rng, M0),
                    ch_iz=ch_iz, ch_ix=ch_ix) for k in range(nshots)]
    return Workload2D(name=f"differentiation-2d-{nz}x{nx}", nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, npml=40,
                      f0=60.0, vp_max=3800.0 * 1.05, stf=ricker(nt, dt, f0=60.0), m_start=m_start,
                      m_true=m_true, shots=shots)


def batched_2d(nshots=64, nt=4000, nz=1000, nx=3000, seed=64, M0=1.0e16, zrange=(400, 1000),
               xrange_=(800, 3000), npml=40):
    """64 shots on uneven subdomains (nz_s ~ U[400,1000], nx_s ~ U[800,3000]) cut around
    each source from the plain workload's model; channels are the well's channels inside
    each window's interior."""
    base = plain_2d(nz=nz, nx=nx, nt=nt, nshots=1, M0=M0)
    rng = np.random.default_rng(seed)
    mt_rng = np.random.default_rng(seed + 1)
    iz = nz // 2
    xs = np.linspace(nx / 6.0, nx * 5.0 / 6.0, nshots).round().astype(int)
    well_ix = base.shots[0].ch_ix
    shots = []
    for k in range(nshots):
        wz = int(rng.integers(zrange[0], zrange[1] + 1))
        wx = int(rng.integers(xrange_[0], xrange_[1] + 1))
        wz, wx = min(wz, nz), min(wx, nx)
        z0 = int(np.clip(iz - wz // 2, 0, nz - wz))
        x0 = int(np.clip(xs[k] - wx // 2, 0, nx - wx))
        lo, hi = x0 + npml + 2, x0 + wx - npml - 3
        sel = well_ix[(well_ix >= lo) & (well_ix <= hi)]
        shots.append(Shot2D(src_iz=iz, src_ix=int(xs[k]), M=_mt_components(mt_rng, M0),
                            ch_iz=np.full(len(sel), iz, np.int32), ch_ix=sel.astype(np.int32),
                            z0=z0, x0=x0, wz=wz, wx=wx))
    base.name = f"batched-2d-{nshots}shots"
    base.shots = shots
    return base


# ---------------------------------------------------------------------------------------
# Guided-wave synthetic of the paper's inversion tests (Synthetic examples): three layers
# with the starting-model parameters of Table 1 (top 4.5 / 2.3 km/s / 2.3 g/cc, middle
# waveguide 3.0 / 1.7 / 2.0, bottom 5.5 / 2.7 / 2.5) and smooth transitions, Gaussian Vp and
# Vs perturbations inside the waveguide, three sources in it with the same diagonal moment
# tensor (M_zz / M_xx = 0.75) and a 10 Hz Ricker time function. The paper's receivers are
# two-component geophones; here a horizontal DAS fiber along the waveguide records e_xx.
# The geometry (sizes, layer depths, anomaly positions) is this recipe's own.
# ---------------------------------------------------------------------------------------
def guided_wave_synthetic(nz=100, nx=400, h=5.0, dt=0.5e-3, nt=1600, npml=20, M0=1.0e16, mute_m=100.0,
                          source_errors=False, anomalies=((0, 130, 0.06), (0, 270, -0.05), (1, 200, 0.06))):
    from scipy.ndimage import gaussian_filter
    z = np.arange(nz) * h
    layer = np.zeros(nz, int)
    top, bot = 230.0, 270.0                     # 40 m waveguide
    layer[z >= top] = 1
    layer[z >= bot] = 2
    params = np.array([[4500.0, 2300.0, 2300.0], [3000.0, 1700.0, 2000.0], [5500.0, 2700.0, 2500.0]])
    m_start = np.empty((3, nz, nx))
    for k in range(3):
        col = gaussian_filter(params[layer, k], sigma=1.0, mode="nearest")
        m_start[k] = col[:, None]
    zc = int(round(0.5 * (top + bot) / h))
    m_true = m_start.copy()
    # relative Gaussian blobs (parameter, column, amplitude); by default a faster and a slower
    # Vp blob and a faster Vs blob between them
    for k, cx, amp in anomalies:
        m_true[k] *= 1.0 + gaussian_blob((nz, nx), zc, cx, 6.0, amp)
    src_ix = [100, 200, 300]
    all_ch = np.arange(30, nx - 30, 2).astype(np.int32)
    M = np.array([M0, 0.75 * M0, 0.0])              # (Mxx, Mzz, Mxz)
    stf = ricker(nt, dt, 10.0)
    shots = []
    for sx in src_ix:
        # channels closer than mute_m to the source are left out (near-field strain)
        ch_ix = all_ch[np.abs(all_ch - sx) * h >= mute_m]
        shots.append(Shot2D(src_iz=zc, src_ix=sx, M=M.copy(), ch_iz=np.full(len(ch_ix), zc, np.int32), ch_ix=ch_ix))
    w = Workload2D(name="guided-wave-synthetic", nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, npml=npml, f0=10.0,
                   vp_max=5500.0, stf=stf, m_start=m_start, m_true=m_true, shots=shots)
    if source_errors:
        w = with_source_errors(w)
    return w


def with_source_errors(w, shift_cells=1, mt_ratio=0.964, stf_error=0.165, seed=21):
    """The inverting side's wrong source parameters (inversion with source-related errors):
    every source one node to the left (the paper shifts 1 m on a finer grid), M_zz / M_xx set
    to mt_ratio at the same Frobenius norm, and the time function perturbed by a smooth
    random series of relative L2 size stf_error, smoothed over a quarter of the central
    period so that the error lies in the wavelet's band."""
    rng = np.random.default_rng(seed)
    shots = []
    for s in w.shots:
        fro = math.sqrt(s.M[0] ** 2 + s.M[1] ** 2 + 2.0 * s.M[2] ** 2)
        mxx = fro / math.sqrt(1.0 + mt_ratio ** 2)
        M = np.array([mxx, mt_ratio * mxx, 0.0])
        shots.append(Shot2D(src_iz=s.src_iz, src_ix=s.src_ix - shift_cells, M=M, ch_iz=s.ch_iz, ch_ix=s.ch_ix))
    from scipy.ndimage import gaussian_filter1d
    noise = gaussian_filter1d(rng.standard_normal(len(w.stf)), 0.25 / (w.f0 * w.dt))
    noise *= np.exp(-0.5 * ((np.arange(len(w.stf)) * w.dt - 1.5 / w.f0) / (1.0 / w.f0)) ** 2)
    noise *= stf_error * np.linalg.norm(w.stf) / np.linalg.norm(noise)
    return Workload2D(name=w.name + "-source-errors", nz=w.nz, nx=w.nx, dz=w.dz, dx=w.dx, dt=w.dt, nt=w.nt,
                      npml=w.npml, f0=w.f0, vp_max=w.vp_max, stf=w.stf + noise, m_start=w.m_start, m_true=w.m_true,
                      shots=shots, pml_R=w.pml_R)


def hard_sinkholes(nshots, nz, nx, src_iz, src_ix, a_z=8, a_x=40):
    """Hard source masks (uint8 [Ns][nz][nx]): 1 inside the ellipse |dz/a_z|^2 + |dx/a_x|^2 < 1
    around each source, and the matching ZOI weights b (0 inside, 1 elsewhere)."""
    z = np.arange(nz)[:, None]
    x = np.arange(nx)[None, :]
    sink = np.zeros((nshots, nz, nx), np.uint8)
    for s in range(nshots):
        sink[s] = (((z - src_iz[s]) / a_z) ** 2 + ((x - src_ix[s]) / a_x) ** 2) < 1.0
    b = np.where(sink > 0, 0.0, 1.0)
    return b, sink


def perturbed_extension(m, nshots, seed=77, rel=0.01, corr_cells=10.0):
    """Extended model m~ = S^T m plus per-shot smooth relative noise (so the consistency
    term is nonzero): [Ns][3][nz][nx]."""
    out = np.empty((nshots,) + m.shape)
    for s in range(nshots):
        for k in range(3):
            out[s, k] = m[k] * (1.0 + smooth_random_field(m.shape[1:], corr_cells, seed + 3 * s + k, rel))
    return out


@dataclass
class Shot3D:
    src_iz: int
    src_iy: int
    src_ix: int
    M: np.ndarray              # (Mxx, Myy, Mzz, Mxy, Mxz, Myz)
    ch_iz: np.ndarray
    ch_iy: np.ndarray
    ch_ix: np.ndarray


@dataclass
class Workload3D:
    name: str
    nz: int
    ny: int
    nx: int
    h: float
    dt: float
    nt: int
    npml: int
    f0: float
    vp_max: float
    stf: np.ndarray
    m_start: np.ndarray        # [3][nz][ny][nx]
    m_true: np.ndarray
    shots: list = field(default_factory=list)
    pml_R: float = 1e-3


def precision_3d(nz=300, ny=400, nx=400, nt=3000, nshots=8, nch_per_well=1000, h=5.0, dt=0.4e-3, npml=20,
                 f0=30.0, M0=1.0e16, seed=8, anomalies=True):
    """The shale geology at 5 m in 3D: background Vp 3800, Vs/Vp 0.6, rho 2550 with a 15 m
    (3-cell) reservoir Vp 3400, Vs/Vp 0.55, rho 2450 at mid depth, +-5% Gaussian-correlated
    anomalies (50 m) in the true model, moment-tensor shots (six components, seed 8) in the
    layer and two horizontal DAS wells along x at y = 3/8 and 5/8 of the width. A well holds
    at most one channel per interior node along x: on the 400-node axis that is 356 per well
    (712 in all), fewer than the nch_per_well = 1000 asked for, which is then capped."""
    res_top = nz // 2 - 1
    m = _shale_model(nz, nx, h, res_top, res_top + 3, anomalies=False)[:, :, None, :]
    m_start = np.repeat(m, ny, axis=2).transpose(0, 1, 2, 3)            # [3][nz][ny][nx]
    m_true = m_start.copy()
    if anomalies:   # (the timing sample of the full grid skips them: no observed data needed)
        for k in range(3):
            m_true[k] *= 1.0 + smooth_random_field((nz, ny, nx), 50.0 / h, 14130 + k, 0.05)
    iz = nz // 2
    wells = [int(ny * 3 // 8), int(ny * 5 // 8)]
    lo = npml + 2
    nch = min(nch_per_well, nx - 2 * lo)
    ch_ix = (lo + np.arange(nch) * max(1, (nx - 2 * lo) // nch)).astype(np.int32)
    ch_iz = np.full(2 * nch, iz, np.int32)
    ch_iy = np.concatenate([np.full(nch, wells[0]), np.full(nch, wells[1])]).astype(np.int32)
    ch_ix2 = np.concatenate([ch_ix, ch_ix]).astype(np.int32)
    rng = np.random.default_rng(seed)
    shots = []
    for s in range(nshots):
        M = rng.uniform(-1.0, 1.0, 6)
        M *= M0 / math.sqrt(M[0] ** 2 + M[1] ** 2 + M[2] ** 2 + 2 * (M[3] ** 2 + M[4] ** 2 + M[5] ** 2))
        sy = wells[s % 2] + (2 if s % 4 < 2 else -2)
        sx = int(lo + 4 + (nx - 2 * lo - 8) * (s + 0.5) / nshots)
        shots.append(Shot3D(src_iz=iz, src_iy=sy, src_ix=sx, M=M, ch_iz=ch_iz, ch_iy=ch_iy, ch_ix=ch_ix2))
    return Workload3D(name=f"precision-3d-{nz}x{ny}x{nx}", nz=nz, ny=ny, nx=nx, h=h, dt=dt, nt=nt, npml=npml,
                      f0=f0, vp_max=3800.0 * 1.05, stf=ricker(nt, dt, f0), m_start=m_start, m_true=m_true,
                      shots=shots)
