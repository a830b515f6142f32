"""FP64 oracle: 2D isotropic elastic propagation, DAS sampling, misfit and per-shot gradient.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). Parity of the GPU path is measured
against this module; it is pinned by the CPU tests (analytic Green's function, energy,
reciprocity, dot-product, finite differences, dense brute force).

Paper passages followed
-----------------------
* Forward problem, eq.(1): ``A(m) u_s = f_s`` with m = (Vp, Vs, rho). The paper gives no
  discretization. Reading taken: first-order velocity-stress system on a staggered grid,
  4th-order spatial differences (coefficients 9/8 and -1/24), leapfrog in time, CPML
  absorbing strips with kappa = 1.
* Point source, eq.(2), moment-tensor case ``-M grad(delta) w(t)``. In velocity-stress form
  this is a stress-rate injection ``d(sigma)/dt -= M s(t) delta(x - x_s)`` with s = dw/dt,
  delta -> 1/(dx dz). M_xz is spread 1/4 over the four shear nodes around the source.
* Sampling operator K_r, eq.(3): DAS horizontal strain e_xx at the channel's normal node,
  ``e_xx(t_{n+1}) = sum_{k<=n} dt * (D_x^- v_x^{k+1/2})``, recorded every time step.
* Misfit, eq.(4) and the data term of eq.(8): ``phi = 1/2 sum_c sum_n r[c,n]^2``,
  r = d - d_obs, no time weighting.
* Gradient, eq.(6): ``g_s = J_s^T (d_s - d_obs)``. Reading taken: the exact transpose of
  the discrete forward map (discretize-then-differentiate), so finite differences and
  dot-product tests hold to round-off. Each shot differentiates only its own m_s (eq.(8)).

Grid layout (all arrays ``[nz][nx]``, x fastest; values outside the array are zero)
------------------------------------------------------------------------------------
  sxx, szz at (i, j)        vx at (i, j+1/2)        vz at (i+1/2, j)
  sxz at (i+1/2, j+1/2)     i = z index, j = x index
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

C1 = 9.0 / 8.0
C2 = -1.0 / 24.0


@dataclass
class Grid2D:
    nz: int
    nx: int
    dz: float
    dx: float
    dt: float
    nt: int
    npml: int = 0
    pml_R: float = 1e-3
    pml_f0: float = 10.0
    vp_max: float = 0.0


# ---------------------------------------------------------------------------------------
# Staggered 4th-order differences (zero outside the array).
# ---------------------------------------------------------------------------------------
def _shift(f, k, axis):
    """Return g with g[..., j, ...] = f[..., j + k, ...] and zero where j + k is outside."""
    g = np.zeros_like(f)
    n = f.shape[axis]
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if k >= 0:
        src[axis] = slice(k, n)
        dst[axis] = slice(0, n - k)
    else:
        src[axis] = slice(0, n + k)
        dst[axis] = slice(-k, n)
    g[tuple(dst)] = f[tuple(src)]
    return g


def d_plus(f, h, axis):
    """Integer nodes -> half nodes: (D+ f)_{j+1/2} = [c1(f_{j+1}-f_j) + c2(f_{j+2}-f_{j-1})]/h."""
    return (C1 * (_shift(f, 1, axis) - f) + C2 * (_shift(f, 2, axis) - _shift(f, -1, axis))) / h


def d_minus(g, h, axis):
    """Half nodes -> integer nodes, array index j holding node j+1/2:
    (D- g)_j = [c1(g_{j+1/2}-g_{j-1/2}) + c2(g_{j+3/2}-g_{j-3/2})]/h."""
    return (C1 * (g - _shift(g, -1, axis)) + C2 * (_shift(g, 1, axis) - _shift(g, -2, axis))) / h


def _scatter(p, k, axis):
    """Transpose of ``_shift(., k)``: moves p[j] to index j + k (dropping what falls outside)."""
    return _shift(p, -k, axis)


def d_plus_T(p, h, axis):
    """Transpose of ``d_plus`` written as the explicit scatter of each stencil tap."""
    return (C1 * (_scatter(p, 1, axis) - p) + C2 * (_scatter(p, 2, axis) - _scatter(p, -1, axis))) / h


def d_minus_T(p, h, axis):
    """Transpose of ``d_minus`` written as the explicit scatter of each stencil tap."""
    return (C1 * (p - _scatter(p, -1, axis)) + C2 * (_scatter(p, 1, axis) - _scatter(p, -2, axis))) / h


# ---------------------------------------------------------------------------------------
# Model staging: m = (Vp, Vs, rho) -> (lambda+2mu, lambda, mu_xz, b_x, b_z).
# ---------------------------------------------------------------------------------------
def _clamped_plus1(n):
    return np.minimum(np.arange(n) + 1, n - 1)


def stage(vp, vs, rho):
    """Lame parameters at normal nodes, harmonic-mean shear modulus at shear nodes and
    arithmetic-mean buoyancy at velocity nodes. Edge neighbours are clamped to the last
    row/column; mu_xz = 0 if any of its four mu is 0."""
    vp, vs, rho = (np.asarray(a, np.float64) for a in (vp, vs, rho))
    nz, nx = vp.shape
    mu = rho * vs * vs
    lam2mu = rho * vp * vp
    lam = lam2mu - 2.0 * mu
    ip = _clamped_plus1(nz)
    jp = _clamped_plus1(nx)
    m00, m10, m01, m11 = mu, mu[ip, :], mu[:, jp], mu[ip][:, jp]
    allpos = (m00 > 0) & (m10 > 0) & (m01 > 0) & (m11 > 0)
    with np.errstate(divide="ignore"):
        inv = 1.0 / m00 + 1.0 / m10 + 1.0 / m01 + 1.0 / m11
        muxz = np.where(allpos, 4.0 / np.where(allpos, inv, 1.0), 0.0)
    bx = 2.0 / (rho + rho[:, jp])
    bz = 2.0 / (rho + rho[ip, :])
    return dict(lam2mu=lam2mu, lam=lam, mu=mu, muxz=muxz, bx=bx, bz=bz)


# ---------------------------------------------------------------------------------------
# CPML (unsplit, memory variables, kappa = 1).
# ---------------------------------------------------------------------------------------
def cpml_profile(n, h, npml, dt, vp_max, R, f0, half):
    """Coefficients (a, b) of psi <- b psi + a (D f) for the n nodes along one axis.

    Node coordinate (in cells) is j, or j + 1/2 for half nodes. The distance into the
    absorbing strip is xi = max(npml - x, x - (n - 1 - npml), 0) cells and r = min(xi/npml, 1).
    d = d0 r^2 with d0 = -3 vp_max ln(R) / (2 npml h), alpha = pi f0 (1 - r),
    b = exp(-(d + alpha) dt), a = d (b - 1) / (d + alpha)."""
    a = np.zeros(n)
    b = np.ones(n)
    if npml <= 0:
        return a, b
    x = np.arange(n, dtype=np.float64) + (0.5 if half else 0.0)
    xi = np.maximum(np.maximum(npml - x, x - (n - 1 - npml)), 0.0)
    r = np.minimum(xi / npml, 1.0)
    d0 = -3.0 * vp_max * np.log(R) / (2.0 * npml * h)
    d = d0 * r * r
    alpha = np.pi * f0 * (1.0 - r)
    b = np.exp(-(d + alpha) * dt)
    denom = d + alpha
    a = np.where(denom > 0, d * (b - 1.0) / np.where(denom > 0, denom, 1.0), 0.0)
    return a, b


def cpml_2d(g: Grid2D):
    """Profiles broadcast against [nz][nx]: x along the last axis, z along the first."""
    args = (g.npml, g.dt, g.vp_max, g.pml_R, g.pml_f0)
    axi, bxi = cpml_profile(g.nx, g.dx, *args, half=False)
    axh, bxh = cpml_profile(g.nx, g.dx, *args, half=True)
    azi, bzi = cpml_profile(g.nz, g.dz, *args, half=False)
    azh, bzh = cpml_profile(g.nz, g.dz, *args, half=True)
    return dict(axi=axi[None, :], bxi=bxi[None, :], axh=axh[None, :], bxh=bxh[None, :],
                azi=azi[:, None], bzi=bzi[:, None], azh=azh[:, None], bzh=bzh[:, None])


# The eight CPML memory variables: (derivative it corrects, profile used).
#   vx_x: D+x sxx at vx node (x half)   vx_z: D-z sxz at vx node (z int)
#   vz_x: D-x sxz at vz node (x int)    vz_z: D+z szz at vz node (z half)
#   xx_x: D-x vx at normal node (x int) zz_z: D-z vz at normal node (z int)
#   xz_z: D+z vx at shear node (z half) xz_x: D+x vz at shear node (x half)
PSI_PROFILE = dict(vx_x=("axh", "bxh"), vx_z=("azi", "bzi"), vz_x=("axi", "bxi"),
                   vz_z=("azh", "bzh"), xx_x=("axi", "bxi"), zz_z=("azi", "bzi"),
                   xz_z=("azh", "bzh"), xz_x=("axh", "bxh"))


def moment_tensor_series(M, stf):
    """Source components f[k][n] = M_k s(t_{n+1/2}) for k = xx, zz, xz (eq.(2), MT case)."""
    M = np.asarray(M, np.float64)
    return np.outer(M[:3], np.asarray(stf, np.float64))


# ---------------------------------------------------------------------------------------
# Forward propagation.
# ---------------------------------------------------------------------------------------
class Propagator2D:
    """Leapfrog velocity-stress time stepping for one shot (state kept in FP64)."""

    def __init__(self, grid: Grid2D, vp, vs, rho):
        self.g = grid
        self.med = stage(vp, vs, rho)
        self.pml = cpml_2d(grid)
        shape = (grid.nz, grid.nx)
        self.vx = np.zeros(shape)
        self.vz = np.zeros(shape)
        self.sxx = np.zeros(shape)
        self.szz = np.zeros(shape)
        self.sxz = np.zeros(shape)
        self.psi = {k: np.zeros(shape) for k in PSI_PROFILE}

    def _cpml(self, key, deriv):
        """psi <- b psi + a D ; returns the corrected derivative D + psi (kappa = 1)."""
        a, b = (self.pml[k] for k in PSI_PROFILE[key])
        self.psi[key] = b * self.psi[key] + a * deriv
        return deriv + self.psi[key]

    def velocity_half_step(self):
        """v^{n+1/2} = v^{n-1/2} + dt b (div sigma^n); returns the corrected divergences."""
        g, m = self.g, self.med
        qx = self._cpml("vx_x", d_plus(self.sxx, g.dx, 1)) + self._cpml("vx_z", d_minus(self.sxz, g.dz, 0))
        qz = self._cpml("vz_x", d_minus(self.sxz, g.dx, 1)) + self._cpml("vz_z", d_plus(self.szz, g.dz, 0))
        self.vx = self.vx + g.dt * m["bx"] * qx
        self.vz = self.vz + g.dt * m["bz"] * qz
        return qx, qz

    def stress_half_step(self):
        """sigma^{n+1} = sigma^n + dt C (strain rate of v^{n+1/2}); returns the corrected
        strain rates (pxx, pzz, pzx + pxz)."""
        g, m = self.g, self.med
        pxx = self._cpml("xx_x", d_minus(self.vx, g.dx, 1))
        pzz = self._cpml("zz_z", d_minus(self.vz, g.dz, 0))
        pzx = self._cpml("xz_z", d_plus(self.vx, g.dz, 0))
        pxz = self._cpml("xz_x", d_plus(self.vz, g.dx, 1))
        self.sxx = self.sxx + g.dt * (m["lam2mu"] * pxx + m["lam"] * pzz)
        self.szz = self.szz + g.dt * (m["lam"] * pxx + m["lam2mu"] * pzz)
        self.sxz = self.sxz + g.dt * m["muxz"] * (pzx + pxz)
        return pxx, pzz, pzx + pxz

    def inject(self, src_iz, src_ix, fxx, fzz, fxz):
        """Moment-tensor stress-rate injection at normal node (src_iz, src_ix)."""
        g = self.g
        w = g.dt / (g.dx * g.dz)
        self.sxx[src_iz, src_ix] -= w * fxx
        self.szz[src_iz, src_ix] -= w * fzz
        for i in (src_iz - 1, src_iz):
            for j in (src_ix - 1, src_ix):
                self.sxz[i, j] -= 0.25 * w * fxz

    def strain_rate_xx(self, ch_iz, ch_ix):
        """Uncorrected D-x vx at the channels' normal nodes."""
        return d_minus(self.vx, self.g.dx, 1)[ch_iz, ch_ix]


def forward(grid: Grid2D, vp, vs, rho, src_iz, src_ix, src, ch_iz, ch_ix, store=False, probe=None):
    """Run nt steps; return DAS data d[nch][nt] (strain e_xx at t_{n+1}).

    src: [3][nt] source components (xx, zz, xz) at t_{n+1/2}. With store=True also return
    the per-step corrected strain rates and divergences the gradient needs. ``probe`` is an
    optional callable(n, propagator) invoked after each full step (used by the tests)."""
    P = Propagator2D(grid, vp, vs, rho)
    ch_iz = np.asarray(ch_iz)
    ch_ix = np.asarray(ch_ix)
    nch = len(ch_iz)
    d = np.zeros((nch, grid.nt))
    e = np.zeros(nch)
    hist = [] if store else None
    for n in range(grid.nt):
        qx, qz = P.velocity_half_step()
        pxx, pzz, ps = P.stress_half_step()
        P.inject(src_iz, src_ix, src[0][n], src[1][n], src[2][n])
        e = e + grid.dt * P.strain_rate_xx(ch_iz, ch_ix)
        d[:, n] = e
        if store:
            hist.append((pxx, pzz, ps, qx, qz))
        if probe is not None:
            probe(n, P)
    if store:
        return d, hist, P
    return d


# ---------------------------------------------------------------------------------------
# Exact discrete transpose.
# ---------------------------------------------------------------------------------------
class Adjoint2D:
    """State of the exact discrete transpose of ``forward`` (adjoints of v, sigma, the CPML
    memory variables and the DAS accumulators), stepped backward one time step at a time."""

    def __init__(self, grid: Grid2D, vp, vs, rho, src_iz, src_ix, ch_iz, ch_ix, want_grad):
        g = grid
        self.g = g
        self.med = stage(vp, vs, rho)
        self.pml = cpml_2d(g)
        shape = (g.nz, g.nx)
        self.vxb, self.vzb = np.zeros(shape), np.zeros(shape)
        self.sxxb, self.szzb, self.sxzb = np.zeros(shape), np.zeros(shape), np.zeros(shape)
        self.psib = {k: np.zeros(shape) for k in PSI_PROFILE}
        self.ch_iz = np.asarray(ch_iz)
        self.ch_ix = np.asarray(ch_ix)
        self.src = (src_iz, src_ix)
        self.ebar = np.zeros(len(self.ch_iz))
        self.want_grad = want_grad
        if want_grad:
            self.glam, self.gmu, self.gmuxz = np.zeros(shape), np.zeros(shape), np.zeros(shape)
            self.gbx, self.gbz = np.zeros(shape), np.zeros(shape)

    def _cpml_T(self, key, ybar):
        a, b = (self.pml[k] for k in PSI_PROFILE[key])
        self.psib[key] = self.psib[key] + ybar
        xbar = ybar + a * self.psib[key]
        self.psib[key] = b * self.psib[key]
        return xbar

    def step(self, r_n, hist_n=None):
        """Transpose of time step n: r_n is r[:, n]; hist_n the forward quantities of step n
        (needed for the gradient). Returns the source-component adjoints (3,) of step n."""
        g, med = self.g, self.med
        iz, ix = self.src
        w = g.dt / (g.dx * g.dz)
        # DAS record: d[:, n] = e ; e += dt * D-x vx at channels
        self.ebar = self.ebar + r_n
        pch = np.zeros((g.nz, g.nx))
        np.add.at(pch, (self.ch_iz, self.ch_ix), g.dt * self.ebar)
        self.vxb = self.vxb + d_minus_T(pch, g.dx, 1)
        # source injection
        fbar = np.array([-w * self.sxxb[iz, ix], -w * self.szzb[iz, ix],
                         -0.25 * w * self.sxzb[iz - 1:iz + 1, ix - 1:ix + 1].sum()])
        # stress update
        sxxb, szzb, sxzb = self.sxxb, self.szzb, self.sxzb
        if self.want_grad:
            pxx, pzz, ps, qx, qz = hist_n
            self.glam += g.dt * (sxxb + szzb) * (pxx + pzz)
            self.gmu += 2.0 * g.dt * (sxxb * pxx + szzb * pzz)
            self.gmuxz += g.dt * sxzb * ps
        pxx_b = g.dt * (med["lam2mu"] * sxxb + med["lam"] * szzb)
        pzz_b = g.dt * (med["lam"] * sxxb + med["lam2mu"] * szzb)
        ps_b = g.dt * med["muxz"] * sxzb
        cT = self._cpml_T
        self.vxb = self.vxb + d_minus_T(cT("xx_x", pxx_b), g.dx, 1) + d_plus_T(cT("xz_z", ps_b), g.dz, 0)
        self.vzb = self.vzb + d_minus_T(cT("zz_z", pzz_b), g.dz, 0) + d_plus_T(cT("xz_x", ps_b), g.dx, 1)
        # velocity update
        if self.want_grad:
            self.gbx += g.dt * self.vxb * qx
            self.gbz += g.dt * self.vzb * qz
        qx_b = g.dt * med["bx"] * self.vxb
        qz_b = g.dt * med["bz"] * self.vzb
        self.sxxb = self.sxxb + d_plus_T(cT("vx_x", qx_b), g.dx, 1)
        self.sxzb = (self.sxzb + d_minus_T(cT("vx_z", qx_b), g.dz, 0)
                     + d_minus_T(cT("vz_x", qz_b), g.dx, 1))
        self.szzb = self.szzb + d_plus_T(cT("vz_z", qz_b), g.dz, 0)
        return fbar

    def gradients(self):
        return self.glam, self.gmu, self.gmuxz, self.gbx, self.gbz


def adjoint(grid: Grid2D, vp, vs, rho, src_iz, src_ix, ch_iz, ch_ix, r, hist=None):
    """Transpose of ``forward`` applied to r[nch][nt].

    Returns fbar[3][nt] = L^T r with respect to the source components, and, when the
    forward history ``hist`` is given, the parameter gradients (glam, gmu, gmuxz, gbx, gbz)
    of <d, r> with respect to (lambda, mu at normal nodes, mu_xz, b_x, b_z).

    Each forward sub-step y += T x becomes x_bar += T^T y_bar, taken in reverse order:
    DAS record, source injection, stress update (with its CPML variables), velocity update
    (with its CPML variables)."""
    A = Adjoint2D(grid, vp, vs, rho, src_iz, src_ix, ch_iz, ch_ix, want_grad=hist is not None)
    fbar = np.zeros((3, grid.nt))
    for n in range(grid.nt - 1, -1, -1):
        fbar[:, n] = A.step(r[:, n], hist[n] if hist is not None else None)
    if hist is not None:
        return fbar, A.gradients()
    return fbar


def chain_rule(vp, vs, rho, glam, gmu, gmuxz, gbx, gbz):
    """Gradients w.r.t. (lambda, mu, mu_xz, b_x, b_z) -> gradients w.r.t. (Vp, Vs, rho).

    mu_xz = 4 / sum_k(1/mu_k) over its four (clamped) corners: d mu_xz / d mu_k = mu_xz^2/(4 mu_k^2).
    b = 2/(rho_a + rho_b): d b / d rho_a = -b^2/2 (both terms land on one rho at a clamped edge).
    lambda = rho(Vp^2 - 2Vs^2), mu = rho Vs^2."""
    vp, vs, rho = (np.asarray(a, np.float64) for a in (vp, vs, rho))
    nz, nx = vp.shape
    med = stage(vp, vs, rho)
    mu, muxz, bx, bz = med["mu"], med["muxz"], med["bx"], med["bz"]
    ip = _clamped_plus1(nz)
    jp = _clamped_plus1(nx)
    I, J = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    gmu_tot = gmu.copy()
    with np.errstate(divide="ignore", invalid="ignore"):
        for (ci, cj) in ((I, J), (ip[I], J), (I, jp[J]), (ip[I], jp[J])):
            contrib = np.where(muxz > 0, gmuxz * muxz * muxz / (4.0 * mu[ci, cj] ** 2), 0.0)
            np.add.at(gmu_tot, (ci, cj), contrib)
    grho_b = np.zeros((nz, nx))
    for (ci, cj) in ((I, J), (I, jp[J])):
        np.add.at(grho_b, (ci, cj), -0.5 * gbx * bx * bx)
    for (ci, cj) in ((I, J), (ip[I], J)):
        np.add.at(grho_b, (ci, cj), -0.5 * gbz * bz * bz)
    g_vp = 2.0 * rho * vp * glam
    g_vs = 2.0 * rho * vs * (gmu_tot - 2.0 * glam)
    g_rho = (vp * vp - 2.0 * vs * vs) * glam + vs * vs * gmu_tot + grho_b
    return np.stack([g_vp, g_vs, g_rho])


def misfit(d, d_obs):
    """eq.(4) / data term of eq.(8): phi = 1/2 sum (d - d_obs)^2, and the residual."""
    r = np.asarray(d, np.float64) - np.asarray(d_obs, np.float64)
    return 0.5 * float(np.sum(r * r)), r


def model_forward(grid, m, src_iz, src_ix, src, ch_iz, ch_ix):
    """d = K u(m) for one shot; m is [3][nz][nx] = (Vp, Vs, rho)."""
    return forward(grid, m[0], m[1], m[2], src_iz, src_ix, src, ch_iz, ch_ix)


def model_adjoint(grid, m, src_iz, src_ix, ch_iz, ch_ix, r):
    """L^T r with respect to the [3][nt] source components."""
    return adjoint(grid, m[0], m[1], m[2], src_iz, src_ix, ch_iz, ch_ix, r)


def shot_gradient(grid, m, src_iz, src_ix, src, ch_iz, ch_ix, d_obs):
    """Per-shot data misfit and gradient g_s = J_s^T (d_s - d_obs) w.r.t. m_s = (Vp, Vs, rho).

    Returns (g[3][nz][nx], phi, d)."""
    d, hist, _ = forward(grid, m[0], m[1], m[2], src_iz, src_ix, src, ch_iz, ch_ix, store=True)
    phi, r = misfit(d, d_obs)
    _, gpar = adjoint(grid, m[0], m[1], m[2], src_iz, src_ix, ch_iz, ch_ix, r, hist=hist)
    return chain_rule(m[0], m[1], m[2], *gpar), phi, d


# ---------------------------------------------------------------------------------------
# Checkpointed gradient (the wavefield-recomputation schedule), optionally with 16-bit
# snapshots. Mirrors what the product path computes, so its compressed-checkpoint mode can
# be compared with this function at FP32 parity (and with ``shot_gradient`` for the error
# the compression itself causes).
# ---------------------------------------------------------------------------------------
STATE_FIELDS = ("vx", "vz", "sxx", "szz", "sxz")


def _snapshot(P, codec):
    from .checkpoint import roundtrip
    snap = {k: roundtrip(getattr(P, k), codec) for k in STATE_FIELDS}
    snap["psi"] = {k: roundtrip(v, codec) for k, v in P.psi.items()}
    return snap


def _restore(P, snap):
    for k in STATE_FIELDS:
        setattr(P, k, snap[k].copy())
    P.psi = {k: v.copy() for k, v in snap["psi"].items()}


def shot_gradient_checkpointed(grid, m, src_iz, src_ix, src, ch_iz, ch_ix, d_obs, interval, codec=None):
    """Per-shot gradient with the forward state snapshotted at the start of every segment of
    `interval` steps (each field encoded by ``checkpoint.roundtrip(., codec)``), the last
    segment's forward quantities kept from the first sweep, and every other segment
    recomputed from its (decoded) snapshot before its transposed steps. Segment 0 starts
    from the exact zero state. With codec None this equals ``shot_gradient`` to round-off.

    Returns (g[3][nz][nx], phi, d)."""
    g = grid
    L = max(1, min(int(interval), g.nt))
    nseg = (g.nt + L - 1) // L
    last0 = (nseg - 1) * L
    P = Propagator2D(g, m[0], m[1], m[2])
    ch_iz, ch_ix = np.asarray(ch_iz), np.asarray(ch_ix)
    d = np.zeros((len(ch_iz), g.nt))
    e = np.zeros(len(ch_iz))
    snaps = {}
    last_hist = []
    for n in range(g.nt):
        if n % L == 0 and 0 < n < last0:
            snaps[n // L] = _snapshot(P, codec)
        qx, qz = P.velocity_half_step()
        pxx, pzz, ps = P.stress_half_step()
        P.inject(src_iz, src_ix, src[0][n], src[1][n], src[2][n])
        e = e + g.dt * P.strain_rate_xx(ch_iz, ch_ix)
        d[:, n] = e
        if n >= last0:
            last_hist.append((pxx, pzz, ps, qx, qz))
    phi, r = misfit(d, d_obs)
    A = Adjoint2D(g, m[0], m[1], m[2], src_iz, src_ix, ch_iz, ch_ix, want_grad=True)
    for k in range(nseg - 1, -1, -1):
        n0, n1 = k * L, min(g.nt, (k + 1) * L)
        if k == nseg - 1:
            hist = last_hist
        else:
            Q = Propagator2D(g, m[0], m[1], m[2])
            if k > 0:
                _restore(Q, snaps[k])
            hist = []
            for n in range(n0, n1):
                qx, qz = Q.velocity_half_step()
                pxx, pzz, ps = Q.stress_half_step()
                Q.inject(src_iz, src_ix, src[0][n], src[1][n], src[2][n])
                hist.append((pxx, pzz, ps, qx, qz))
        for n in range(n1 - 1, n0 - 1, -1):
            A.step(r[:, n], hist[n - n0])
    return chain_rule(m[0], m[1], m[2], *A.gradients()), phi, d
