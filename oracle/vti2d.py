"""FP64 oracle: 2D elastic propagation in a VTI medium (vertical symmetry axis), as in the
field example's starting model (Thomsen epsilon from the data, delta = epsilon / 2,
density and anisotropy kept fixed while Vp0 and Vs0 are inverted).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings and definitions
------------------------
* Stiffness in the x-z plane from Thomsen's parameters (the textbook definitions written
  out): c33 = rho Vp0^2, c55 = mu = rho Vs0^2, c11 = c33 (1 + 2 eps),
  c13 = sqrt((c33 - c55)(c33 (1 + 2 delta) - c55)) - c55 with delta = eps / 2.
* The scheme is the isotropic one (``elastic2d``: staggering, CPML, source, DAS) with the
  normal-stress update sigma_xx += dt (c11 p_xx + c13 p_zz), sigma_zz += dt (c13 p_xx +
  c33 p_zz); the shear update keeps the harmonic mean of mu at the shear node.
* Gradients: with respect to (c11, c13, c33) at the normal nodes, mu_xz and the
  buoyancies, then, at fixed eps, with respect to (Vp0, Vs0, rho): c11, c13 depend on Vp0
  only through c33 and on Vs0 only through mu.
With eps = 0 every function equals its isotropic counterpart.
"""
from __future__ import annotations

import numpy as np

from . import elastic2d as E


def stage_vti(vp0, vs0, rho, eps):
    med = E.stage(vp0, vs0, rho)
    eps = np.asarray(eps, np.float64) * np.ones_like(med["mu"])
    c33, mu = med["lam2mu"], med["mu"]
    med["c33"] = c33
    med["c11"] = c33 * (1.0 + 2.0 * eps)
    med["c13"] = np.sqrt((c33 - mu) * (c33 * (1.0 + eps) - mu)) - mu
    med["eps"] = eps
    return med


class PropagatorVTI(E.Propagator2D):
    def __init__(self, grid, vp0, vs0, rho, eps):
        super().__init__(grid, vp0, vs0, rho)
        self.med = stage_vti(vp0, vs0, rho, eps)

    def stress_half_step(self):
        g, m = self.g, self.med
        pxx = self._cpml("xx_x", E.d_minus(self.vx, g.dx, 1))
        pzz = self._cpml("zz_z", E.d_minus(self.vz, g.dz, 0))
        pzx = self._cpml("xz_z", E.d_plus(self.vx, g.dz, 0))
        pxz = self._cpml("xz_x", E.d_plus(self.vz, g.dx, 1))
        self.sxx = self.sxx + g.dt * (m["c11"] * pxx + m["c13"] * pzz)
        self.szz = self.szz + g.dt * (m["c13"] * pxx + m["c33"] * pzz)
        self.sxz = self.sxz + g.dt * m["muxz"] * (pzx + pxz)
        return pxx, pzz, pzx + pxz


def forward(grid, m, eps, src_iz, src_ix, src, ch_iz, ch_ix, store=False, probe=None):
    """As ``elastic2d.forward`` in the VTI medium; m = (Vp0, Vs0, rho)."""
    P = PropagatorVTI(grid, m[0], m[1], m[2], eps)
    ch_iz, ch_ix = np.asarray(ch_iz), np.asarray(ch_ix)
    d = np.zeros((len(ch_iz), grid.nt))
    e = np.zeros(len(ch_iz))
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
    return (d, hist, P) if store else d


class AdjointVTI(E.Adjoint2D):
    """Exact transpose of ``forward``: the isotropic transpose with the VTI normal block."""

    def __init__(self, grid, m, eps, src_iz, src_ix, ch_iz, ch_ix, want_grad):
        super().__init__(grid, m[0], m[1], m[2], src_iz, src_ix, ch_iz, ch_ix, want_grad)
        self.med = stage_vti(m[0], m[1], m[2], eps)
        if want_grad:
            shape = (grid.nz, grid.nx)
            self.g11, self.g13, self.g33 = np.zeros(shape), np.zeros(shape), np.zeros(shape)

    def step(self, r_n, hist_n=None):
        g, med = self.g, self.med
        iz, ix = self.src
        w = g.dt / (g.dx * g.dz)
        self.ebar = self.ebar + r_n
        pch = np.zeros((g.nz, g.nx))
        np.add.at(pch, (self.ch_iz, self.ch_ix), g.dt * self.ebar)
        self.vxb = self.vxb + E.d_minus_T(pch, g.dx, 1)
        fbar = np.array([-w * self.sxxb[iz, ix], -w * self.szzb[iz, ix],
                         -0.25 * w * self.sxzb[iz - 1:iz + 1, ix - 1:ix + 1].sum()])
        sxxb, szzb, sxzb = self.sxxb, self.szzb, self.sxzb
        if self.want_grad:
            pxx, pzz, ps, qx, qz = hist_n
            self.g11 += g.dt * sxxb * pxx
            self.g33 += g.dt * szzb * pzz
            self.g13 += g.dt * (sxxb * pzz + szzb * pxx)
            self.gmuxz += g.dt * sxzb * ps
        pxx_b = g.dt * (med["c11"] * sxxb + med["c13"] * szzb)
        pzz_b = g.dt * (med["c13"] * sxxb + med["c33"] * szzb)
        ps_b = g.dt * med["muxz"] * sxzb
        cT = self._cpml_T
        self.vxb = self.vxb + E.d_minus_T(cT("xx_x", pxx_b), g.dx, 1) + E.d_plus_T(cT("xz_z", ps_b), g.dz, 0)
        self.vzb = self.vzb + E.d_minus_T(cT("zz_z", pzz_b), g.dz, 0) + E.d_plus_T(cT("xz_x", ps_b), g.dx, 1)
        if self.want_grad:
            self.gbx += g.dt * self.vxb * qx
            self.gbz += g.dt * self.vzb * qz
        qx_b = g.dt * med["bx"] * self.vxb
        qz_b = g.dt * med["bz"] * self.vzb
        self.sxxb = self.sxxb + E.d_plus_T(cT("vx_x", qx_b), g.dx, 1)
        self.sxzb = (self.sxzb + E.d_minus_T(cT("vx_z", qx_b), g.dz, 0)
                     + E.d_minus_T(cT("vz_x", qz_b), g.dx, 1))
        self.szzb = self.szzb + E.d_plus_T(cT("vz_z", qz_b), g.dz, 0)
        return fbar


def adjoint(grid, m, eps, src_iz, src_ix, ch_iz, ch_ix, r, hist=None):
    A = AdjointVTI(grid, m, eps, src_iz, src_ix, ch_iz, ch_ix, want_grad=hist is not None)
    fbar = np.zeros((3, grid.nt))
    for n in range(grid.nt - 1, -1, -1):
        fbar[:, n] = A.step(r[:, n], hist[n] if hist is not None else None)
    if hist is not None:
        return fbar, (A.g11, A.g13, A.g33, A.gmuxz, A.gbx, A.gbz)
    return fbar


def chain_rule(m, eps, g11, g13, g33, gmuxz, gbx, gbz):
    """(c11, c13, c33, mu_xz, b_x, b_z) gradients -> (Vp0, Vs0, rho) at fixed eps.

    d c13 / d c33 and d c13 / d mu from c13 = R - mu, R^2 = (c33 - mu)(c33 (1 + eps) - mu);
    the total c33 gradient g33 + (1 + 2 eps) g11 + (d c13/d c33) g13 and the direct mu
    gradient (d c13/d mu) g13 then enter the isotropic chain rule as its lambda and mu
    gradients (c33 = lambda + 2 mu there)."""
    med = stage_vti(m[0], m[1], m[2], eps)
    c33, mu, e = med["c33"], med["mu"], med["eps"]
    A, B = c33 - mu, c33 * (1.0 + e) - mu
    R = np.sqrt(A * B)
    with np.errstate(divide="ignore", invalid="ignore"):
        dc13_dc33 = np.where(R > 0, (B + A * (1.0 + e)) / (2.0 * R), 0.0)
        dc13_dmu = np.where(R > 0, -(A + B) / (2.0 * R), 0.0) - 1.0
    g33_tot = g33 + (1.0 + 2.0 * e) * g11 + dc13_dc33 * g13
    gmu_direct = dc13_dmu * g13
    return E.chain_rule(m[0], m[1], m[2], g33_tot, gmu_direct + 2.0 * g33_tot, gmuxz, gbx, gbz)


def model_forward(grid, m, eps, src_iz, src_ix, src, ch_iz, ch_ix):
    return forward(grid, m, eps, src_iz, src_ix, src, ch_iz, ch_ix)


def shot_gradient(grid, m, eps, src_iz, src_ix, src, ch_iz, ch_ix, d_obs):
    """(g[3][nz][nx] w.r.t. (Vp0, Vs0, rho), phi, d) for one shot in the VTI medium."""
    d, hist, _ = forward(grid, m, eps, src_iz, src_ix, src, ch_iz, ch_ix, store=True)
    phi, r = E.misfit(d, d_obs)
    _, grads = adjoint(grid, m, eps, src_iz, src_ix, ch_iz, ch_ix, r, hist=hist)
    return chain_rule(m, eps, *grads), phi, d
