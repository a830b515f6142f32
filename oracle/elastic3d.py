"""FP64 oracle: 3D isotropic elastic propagation, DAS sampling, misfit and per-shot gradient.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The same readings as ``elastic2d`` (the paper gives no discretization) carried to three
dimensions: first-order velocity-stress system (eq.(1), m = (Vp, Vs, rho)) on the standard
3D staggered grid, 4th-order differences, leapfrog, CPML (kappa = 1) on every face, the
moment-tensor source of eq.(2) with six components, DAS e_xx at the channels (eq.(3)), the
L2 misfit (eq.(4)) and the gradient J^T r (eq.(6)) as the exact transpose of the discrete
forward map.

Grid layout (arrays ``[nz][ny][nx]``, axes z = 0, y = 1, x = 2; zero outside):
  sxx, syy, szz at (i, k, j)      vx at (i, k, j+1/2)   vy at (i, k+1/2, j)   vz at (i+1/2, k, j)
  sxy at (i, k+1/2, j+1/2)        sxz at (i+1/2, k, j+1/2)                 syz at (i+1/2, k+1/2, j)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .elastic2d import cpml_profile, d_minus, d_minus_T, d_plus, d_plus_T, misfit

X, Y, Z = 2, 1, 0


@dataclass
class Grid3D:
    nz: int
    ny: int
    nx: int
    dz: float
    dy: float
    dx: float
    dt: float
    nt: int
    npml: int = 0
    pml_R: float = 1e-3
    pml_f0: float = 10.0
    vp_max: float = 0.0

    def h(self, axis):
        return {X: self.dx, Y: self.dy, Z: self.dz}[axis]


def _cl(n):
    return np.minimum(np.arange(n) + 1, n - 1)


def _harmonic(mus):
    allpos = np.all([m > 0 for m in mus], axis=0)
    with np.errstate(divide="ignore"):
        inv = sum(1.0 / m for m in mus)
        return np.where(allpos, len(mus) / np.where(allpos, inv, 1.0), 0.0)


def stage(vp, vs, rho):
    """Lame parameters at normal nodes, harmonic-mean shear moduli at the three shear node
    types (4 clamped corners each), arithmetic-mean buoyancy at the three velocity nodes."""
    vp, vs, rho = (np.asarray(a, np.float64) for a in (vp, vs, rho))
    nz, ny, nx = vp.shape
    mu = rho * vs * vs
    lam2mu = rho * vp * vp
    iz, iy, ix = _cl(nz), _cl(ny), _cl(nx)
    sh = lambda f, a, b, c: f[a][:, b][:, :, c]
    I, K, J = np.arange(nz), np.arange(ny), np.arange(nx)
    muxy = _harmonic([mu, sh(mu, I, iy, J), sh(mu, I, K, ix), sh(mu, I, iy, ix)])
    muxz = _harmonic([mu, sh(mu, iz, K, J), sh(mu, I, K, ix), sh(mu, iz, K, ix)])
    muyz = _harmonic([mu, sh(mu, iz, K, J), sh(mu, I, iy, J), sh(mu, iz, iy, J)])
    bx = 2.0 / (rho + sh(rho, I, K, ix))
    by = 2.0 / (rho + sh(rho, I, iy, J))
    bz = 2.0 / (rho + sh(rho, iz, K, J))
    return dict(lam2mu=lam2mu, lam=lam2mu - 2.0 * mu, mu=mu, muxy=muxy, muxz=muxz, muyz=muyz,
                bx=bx, by=by, bz=bz)


def cpml_3d(g: Grid3D):
    args = (g.npml, g.dt, g.vp_max, g.pml_R, g.pml_f0)
    out = {}
    for ax, n, h, shape in ((X, g.nx, g.dx, (1, 1, -1)), (Y, g.ny, g.dy, (1, -1, 1)), (Z, g.nz, g.dz, (-1, 1, 1))):
        for half in (False, True):
            a, b = cpml_profile(n, h, *args, half=half)
            out[(ax, half)] = (a.reshape(shape), b.reshape(shape))
    return out


# The 18 CPML memory variables: name -> (source field, axis, forward operator '+'/'-').
# Velocity side (stress divergence terms) and stress side (strain-rate terms); the profile
# is taken at the node's half/integer coordinate along the derivative's axis, which is
# half exactly when the operator is D+ (integer -> half node).
VEL_TERMS = {
    "vx": (("sxx", X, "+"), ("sxy", Y, "-"), ("sxz", Z, "-")),
    "vy": (("sxy", X, "-"), ("syy", Y, "+"), ("syz", Z, "-")),
    "vz": (("sxz", X, "-"), ("syz", Y, "-"), ("szz", Z, "+")),
}
NORMAL_TERMS = {"xx": ("vx", X), "yy": ("vy", Y), "zz": ("vz", Z)}         # all D-
SHEAR_TERMS = {"sxy": (("vx", Y), ("vy", X)), "sxz": (("vx", Z), ("vz", X)),  # all D+
               "syz": (("vy", Z), ("vz", Y))}
SHEAR_MU = {"sxy": "muxy", "sxz": "muxz", "syz": "muyz"}
FIELDS = ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")


def _D(op):
    return d_plus if op == "+" else d_minus


def _DT(op):
    return d_plus_T if op == "+" else d_minus_T


def moment_tensor_series(M, stf):
    """Source components f[k][n] = M_k s(t_{n+1/2}), k = xx, yy, zz, xy, xz, yz (eq.(2))."""
    return np.outer(np.asarray(M, np.float64)[:6], np.asarray(stf, np.float64))


def _shear_nodes(name, iz, iy, ix):
    """The four shear nodes of type `name` around normal node (iz, iy, ix)."""
    if name == "sxy":
        return [(iz, k, j) for k in (iy - 1, iy) for j in (ix - 1, ix)]
    if name == "sxz":
        return [(i, iy, j) for i in (iz - 1, iz) for j in (ix - 1, ix)]
    return [(i, k, ix) for i in (iz - 1, iz) for k in (iy - 1, iy)]


class Propagator3D:
    def __init__(self, grid: Grid3D, vp, vs, rho):
        self.g = grid
        self.med = stage(vp, vs, rho)
        self.pml = cpml_3d(grid)
        shape = (grid.nz, grid.ny, grid.nx)
        for f in FIELDS:
            setattr(self, f, np.zeros(shape))
        self.psi = {}

    def _cpml(self, key, axis, half, deriv):
        a, b = self.pml[(axis, half)]
        self.psi[key] = b * self.psi.get(key, 0.0) + a * deriv
        return deriv + self.psi[key]

    def velocity_half_step(self):
        g, m = self.g, self.med
        qs = {}
        for v, terms in VEL_TERMS.items():
            q = 0.0
            for (src, ax, op) in terms:
                q = q + self._cpml(f"{v}:{src}", ax, op == "+", _D(op)(getattr(self, src), g.h(ax), ax))
            qs[v] = q
            setattr(self, v, getattr(self, v) + g.dt * m["b" + v[1]] * q)
        return qs

    def stress_half_step(self):
        g, m = self.g, self.med
        p = {c: self._cpml(f"p{c}", ax, False, d_minus(getattr(self, v), g.h(ax), ax))
             for c, (v, ax) in NORMAL_TERMS.items()}
        tr = p["xx"] + p["yy"] + p["zz"]
        for c in ("xx", "yy", "zz"):
            s = "s" + c
            setattr(self, s, getattr(self, s) + g.dt * (m["lam"] * tr + (m["lam2mu"] - m["lam"]) * p[c]))
        ps = {}
        for s, terms in SHEAR_TERMS.items():
            t = 0.0
            for (v, ax) in terms:
                t = t + self._cpml(f"{s}:{v}", ax, True, d_plus(getattr(self, v), g.h(ax), ax))
            ps[s] = t
            setattr(self, s, getattr(self, s) + g.dt * m[SHEAR_MU[s]] * t)
        return p, ps

    def inject(self, iz, iy, ix, f):
        """f = (f_xx, f_yy, f_zz, f_xy, f_xz, f_yz) at t_{n+1/2}."""
        g = self.g
        w = g.dt / (g.dx * g.dy * g.dz)
        self.sxx[iz, iy, ix] -= w * f[0]
        self.syy[iz, iy, ix] -= w * f[1]
        self.szz[iz, iy, ix] -= w * f[2]
        for name, fk in (("sxy", f[3]), ("sxz", f[4]), ("syz", f[5])):
            arr = getattr(self, name)
            for node in _shear_nodes(name, iz, iy, ix):
                arr[node] -= 0.25 * w * fk

    def strain_rate_xx(self, ch):
        return d_minus(self.vx, self.g.dx, X)[ch]


def forward(grid, m, src_pos, src, ch, store=False, probe=None):
    """DAS data d[nch][nt]; ch = (ch_iz, ch_iy, ch_ix). With store=True also the per-step
    corrected strain rates and divergences."""
    P = Propagator3D(grid, m[0], m[1], m[2])
    ch = tuple(np.asarray(c) for c in ch)
    d = np.zeros((len(ch[0]), grid.nt))
    e = np.zeros(len(ch[0]))
    hist = [] if store else None
    for n in range(grid.nt):
        qs = P.velocity_half_step()
        p, ps = P.stress_half_step()
        P.inject(*src_pos, src[:, n])
        e = e + grid.dt * P.strain_rate_xx(ch)
        d[:, n] = e
        if store:
            hist.append((p, ps, qs))
        if probe is not None:
            probe(n, P)
    return (d, hist) if store else d


def adjoint(grid, m, src_pos, ch, r, hist=None):
    """Exact transpose of ``forward``: fbar[6][nt] = L^T r w.r.t. the source components, and
    with ``hist`` the gradients w.r.t. the staged parameters (lambda, mu, the three shear
    moduli, the three buoyancies) as a dict."""
    g = grid
    med = stage(*m)
    pml = cpml_3d(g)
    shape = (g.nz, g.ny, g.nx)
    bar = {f: np.zeros(shape) for f in FIELDS}
    psib = {}
    ch = tuple(np.asarray(c) for c in ch)
    ebar = np.zeros(len(ch[0]))
    fbar = np.zeros((6, g.nt))
    grads = {k: np.zeros(shape) for k in ("lam", "mu", "muxy", "muxz", "muyz", "bx", "by", "bz")} if hist else None
    iz, iy, ix = src_pos
    w = g.dt / (g.dx * g.dy * g.dz)

    def cpml_T(key, axis, half, ybar):
        a, b = pml[(axis, half)]
        psib[key] = psib.get(key, 0.0) + ybar
        xbar = ybar + a * psib[key]
        psib[key] = b * psib[key]
        return xbar

    for n in range(g.nt - 1, -1, -1):
        # DAS record transpose
        ebar = ebar + r[:, n]
        pch = np.zeros(shape)
        np.add.at(pch, ch, g.dt * ebar)
        bar["vx"] = bar["vx"] + d_minus_T(pch, g.dx, X)
        # source injection transpose
        fbar[0, n] = -w * bar["sxx"][iz, iy, ix]
        fbar[1, n] = -w * bar["syy"][iz, iy, ix]
        fbar[2, n] = -w * bar["szz"][iz, iy, ix]
        for q, name in ((3, "sxy"), (4, "sxz"), (5, "syz")):
            fbar[q, n] = -0.25 * w * sum(bar[name][node] for node in _shear_nodes(name, iz, iy, ix))
        # stress update transpose
        sb = {c: bar["s" + c] for c in ("xx", "yy", "zz")}
        trb = sb["xx"] + sb["yy"] + sb["zz"]
        if hist:
            p, ps, qs = hist[n]
            tr = p["xx"] + p["yy"] + p["zz"]
            grads["lam"] += g.dt * trb * tr
            grads["mu"] += 2.0 * g.dt * (sb["xx"] * p["xx"] + sb["yy"] * p["yy"] + sb["zz"] * p["zz"])
            for s in SHEAR_TERMS:
                grads[SHEAR_MU[s]] += g.dt * bar[s] * ps[s]
        for c, (v, ax) in NORMAL_TERMS.items():
            pb = g.dt * (med["lam"] * trb + (med["lam2mu"] - med["lam"]) * sb[c])
            bar[v] = bar[v] + d_minus_T(cpml_T(f"p{c}", ax, False, pb), g.h(ax), ax)
        for s, terms in SHEAR_TERMS.items():
            tb = g.dt * med[SHEAR_MU[s]] * bar[s]
            for (v, ax) in terms:
                bar[v] = bar[v] + d_plus_T(cpml_T(f"{s}:{v}", ax, True, tb), g.h(ax), ax)
        # velocity update transpose
        for v, terms in VEL_TERMS.items():
            if hist:
                grads["b" + v[1]] += g.dt * bar[v] * qs[v]
            qb = g.dt * med["b" + v[1]] * bar[v]
            for (src, ax, op) in terms:
                bar[src] = bar[src] + _DT(op)(cpml_T(f"{v}:{src}", ax, op == "+", qb), g.h(ax), ax)
    return (fbar, grads) if hist else fbar


def chain_rule(m, grads):
    """(lambda, mu, mu_xy, mu_xz, mu_yz, b_x, b_y, b_z) gradients -> (Vp, Vs, rho) gradients.
    Each shear modulus is the harmonic mean of four clamped corners (d mu_s / d mu_k =
    mu_s^2 / (4 mu_k^2)); each buoyancy the inverse mean density of two clamped nodes
    (d b / d rho = -b^2 / 2)."""
    vp, vs, rho = (np.asarray(a, np.float64) for a in m)
    nz, ny, nx = vp.shape
    med = stage(vp, vs, rho)
    mu = med["mu"]
    iz, iy, ix = _cl(nz), _cl(ny), _cl(nx)
    I, K, J = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    corners = {"muxy": [(I, K, J), (I, iy[K], J), (I, K, ix[J]), (I, iy[K], ix[J])],
               "muxz": [(I, K, J), (iz[I], K, J), (I, K, ix[J]), (iz[I], K, ix[J])],
               "muyz": [(I, K, J), (iz[I], K, J), (I, iy[K], J), (iz[I], iy[K], J)]}
    gmu = grads["mu"].copy()
    with np.errstate(divide="ignore", invalid="ignore"):
        for name, cs in corners.items():
            ms = med[name]
            for c in cs:
                np.add.at(gmu, c, np.where(ms > 0, grads[name] * ms * ms / (4.0 * mu[c] ** 2), 0.0))
    grho = np.zeros_like(gmu)
    pairs = {"bx": [(I, K, J), (I, K, ix[J])], "by": [(I, K, J), (I, iy[K], J)], "bz": [(I, K, J), (iz[I], K, J)]}
    for name, cs in pairs.items():
        for c in cs:
            np.add.at(grho, c, -0.5 * grads[name] * med[name] ** 2)
    gl = grads["lam"]
    return np.stack([2.0 * rho * vp * gl, 2.0 * rho * vs * (gmu - 2.0 * gl),
                     (vp * vp - 2.0 * vs * vs) * gl + vs * vs * gmu + grho])


def model_forward(grid, m, src_pos, src, ch):
    return forward(grid, m, src_pos, src, ch)


def model_adjoint(grid, m, src_pos, ch, r):
    return adjoint(grid, m, src_pos, ch, r)


def shot_gradient(grid, m, src_pos, src, ch, d_obs):
    """(g[3][nz][ny][nx], phi, d) for one shot, full forward history."""
    d, hist = forward(grid, m, src_pos, src, ch, store=True)
    phi, r = misfit(d, d_obs)
    _, grads = adjoint(grid, m, src_pos, ch, r, hist=hist)
    return chain_rule(m, grads), phi, d


# ---------------------------------------------------------------------------------------
# Checkpointed gradient: the wavefield-recomputation schedule, optionally with 16-bit
# snapshots, so that the compressed-checkpoint modes can be compared with this function at
# FP32 parity (and with ``shot_gradient`` for the error the compression itself causes).
# ---------------------------------------------------------------------------------------
def _snapshot(P, codec):
    from .checkpoint import roundtrip
    snap = {f: roundtrip(getattr(P, f), codec) for f in FIELDS}
    snap["psi"] = {k: roundtrip(v, codec) for k, v in P.psi.items()}
    return snap


def _restore(P, snap):
    for f in FIELDS:
        setattr(P, f, snap[f].copy())
    P.psi = {k: v.copy() for k, v in snap["psi"].items()}


class _RecomputedHistory:
    """The forward quantities of step n, as ``adjoint`` asks for them (n descending): the
    last segment's from the first sweep, every other segment's recomputed from its (decoded)
    snapshot when its first step is asked for; segment 0 starts from the exact zero state."""

    def __init__(self, grid, m, src_pos, src, L, snaps, last0, last_hist):
        self.grid, self.m, self.src_pos, self.src, self.L = grid, m, src_pos, src, L
        self.snaps, self.last0, self.last_hist = snaps, last0, last_hist
        self.k, self.seg = None, None

    def __bool__(self):
        return True

    def __getitem__(self, n):
        if n >= self.last0:
            return self.last_hist[n - self.last0]
        k = n // self.L
        if k != self.k:
            Q = Propagator3D(self.grid, *self.m)
            if k > 0:
                _restore(Q, self.snaps[k])
            self.seg = []
            for j in range(k * self.L, min(self.grid.nt, (k + 1) * self.L)):
                qs = Q.velocity_half_step()
                p, ps = Q.stress_half_step()
                Q.inject(*self.src_pos, self.src[:, j])
                self.seg.append((p, ps, qs))
            self.k = k
        return self.seg[n - k * self.L]


def shot_gradient_checkpointed(grid, m, src_pos, src, ch, d_obs, interval, codec=None):
    """``shot_gradient`` with the forward state (nine fields and the CPML memory variables)
    snapshotted at the start of every segment of `interval` steps but the first and the last,
    each field encoded by ``checkpoint.roundtrip(., codec)``; the last segment's forward
    quantities are kept from the first sweep and the others recomputed from their snapshots
    during the transposed sweep. With codec None this equals ``shot_gradient`` to round-off.

    Returns (g[3][nz][ny][nx], phi, d)."""
    g = grid
    L = max(1, min(int(interval), g.nt))
    nseg = (g.nt + L - 1) // L
    last0 = (nseg - 1) * L
    P = Propagator3D(g, m[0], m[1], m[2])
    ch = tuple(np.asarray(c) for c in ch)
    d = np.zeros((len(ch[0]), g.nt))
    e = np.zeros(len(ch[0]))
    snaps, last_hist = {}, []
    for n in range(g.nt):
        if n % L == 0 and 0 < n < last0:
            snaps[n // L] = _snapshot(P, codec)
        qs = P.velocity_half_step()
        p, ps = P.stress_half_step()
        P.inject(*src_pos, src[:, n])
        e = e + g.dt * P.strain_rate_xx(ch)
        d[:, n] = e
        if n >= last0:
            last_hist.append((p, ps, qs))
    phi, r = misfit(d, d_obs)
    hist = _RecomputedHistory(g, m, src_pos, src, L, snaps, last0, last_hist)
    _, grads = adjoint(g, m, src_pos, ch, r, hist=hist)
    return chain_rule(m, grads), phi, d
