"""Outer loop of the source-extended FWI and of the conventional FWI it is compared with
(Model extension along sources, eqs.(8)-(9); Synthetic examples, eqs.(13)-(14)).

* ``lbfgs``: limited-memory BFGS (two-loop recursion) with a line search that satisfies the
  strong Wolfe conditions (bracketing, then zoom with safeguarded cubic interpolation), as in
  Nocedal and Wright, Numerical Optimization, Algorithms 7.4, 3.5 and 3.6. It stops when the
  convergence rate of eq.(13), (Phi_k - Phi_{k+1}) / Phi_k, falls below a threshold (0.1%
  in the paper) or when no step satisfying the conditions is found.
* ``ExtendedFWI`` / ``ConventionalFWI``: objectives and gradients from the library:
  the data term of every shot on its own component (efwi.batch_gradient) plus the
  consistency term (efwi.extension_regularizer), or every shot on one common model.
  Unknowns are relative perturbations x = m / m_start - 1 of Vp and Vs (density is kept,
  as in the paper's synthetic), one copy per source in the extended case.
* ``final_model``: the physical model S_w W m~ of eq.(9) (efwi.final_model).
* ``cosine_similarity``: eq.(14).
* The two alternatives the paper compares with: conventional FWI with a near-offset mute and
  an approximate inverse pseudo-Hessian as l-BFGS's initial inverse Hessian
  (``lbfgs(h0=...)``, efwi.pseudo_hessian), and conventional FWI whose per-shot gradients
  are mapped by S_w W before the solver sees them, eq.(15) (``PreconditionedFWI``).

Only the optimizer's vector algebra (dot products, axpy on flat device tensors) runs in
PyTorch; every wave propagation, gradient, regularizer and extension operator is the HIP
library's.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import efwi


def cosine_similarity(a, b) -> float:
    """eq.(14): v1^T v2 / (||v1|| ||v2||), in FP64."""
    a = np.asarray(a.detach().cpu() if torch.is_tensor(a) else a, np.float64).ravel()
    b = np.asarray(b.detach().cpu() if torch.is_tensor(b) else b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def convergence_rate(phi_prev: float, phi: float) -> float:
    """eq.(13): relative decrease of the objective over one iteration."""
    return (phi_prev - phi) / phi_prev


@dataclass
class Record:
    phi: list = field(default_factory=list)        # objective after each iteration (0: start)
    rate: list = field(default_factory=list)       # eq.(13) per iteration
    evaluations: int = 0
    stop: str = ""


def _dot(a, b) -> float:
    return float(torch.dot(a.reshape(-1).double(), b.reshape(-1).double()))


def _cubic_min(a0, f0, d0, a1, f1, d1):
    """Minimizer of the cubic interpolating (a0, f0, d0) and (a1, f1, d1), or None."""
    if not all(np.isfinite(v) for v in (f0, d0, f1, d1)) or a0 == a1:
        return None
    d_1 = d0 + d1 - 3.0 * (f0 - f1) / (a0 - a1)
    rad = d_1 * d_1 - d0 * d1
    if rad < 0.0:
        return None
    d_2 = np.sign(a1 - a0) * np.sqrt(rad)
    den = d1 - d0 + 2.0 * d_2
    return None if den == 0.0 else a1 - (a1 - a0) * (d1 + d_2 - d_1) / den


def wolfe_search(fg, x, f0, g0, d, alpha, c1=1e-4, c2=0.9, max_evals=20, record=None):
    """Step length along d satisfying the strong Wolfe conditions
    f(x + a d) <= f0 + c1 a g0.d and |g(x + a d).d| <= c2 |g0.d|.
    Returns (a, f, g) or None when no such step is found within max_evals evaluations."""
    dg0 = _dot(g0, d)
    if not dg0 < 0.0:
        return None

    def ev(a):
        f, g = fg(x + a * d)
        if record is not None:
            record.evaluations += 1
        if not np.isfinite(f):      # a step into an unphysical model: treat as too long
            return float("inf"), g, 0.0
        return f, g, _dot(g, d)

    def zoom(lo, f_lo, dg_lo, hi, f_hi, dg_hi, left):
        for _ in range(left):
            a = _cubic_min(lo, f_lo, dg_lo, hi, f_hi, dg_hi)
            w = hi - lo
            if a is None or not (min(lo, hi) + 0.1 * abs(w) <= a <= max(lo, hi) - 0.1 * abs(w)):
                a = lo + 0.5 * w                       # bisection when the cubic is unusable
            f, g, dg = ev(a)
            if f > f0 + c1 * a * dg0 or f >= f_lo:
                hi, f_hi, dg_hi = a, f, dg
            else:
                if abs(dg) <= -c2 * dg0:
                    return a, f, g
                if dg * (hi - lo) >= 0.0:
                    hi, f_hi, dg_hi = lo, f_lo, dg_lo
                lo, f_lo, dg_lo = a, f, dg
        return None

    a_prev, f_prev, dg_prev = 0.0, f0, dg0
    a = alpha
    for i in range(max_evals):
        f, g, dg = ev(a)
        if f > f0 + c1 * a * dg0 or (i > 0 and f >= f_prev):
            return zoom(a_prev, f_prev, dg_prev, a, f, dg, max_evals - i - 1)
        if abs(dg) <= -c2 * dg0:
            return a, f, g
        if dg >= 0.0:
            return zoom(a, f, dg, a_prev, f_prev, dg_prev, max_evals - i - 1)
        a_prev, f_prev, dg_prev = a, f, dg
        a = 2.0 * a
    return None


def lbfgs(fg, x0, max_iter=100, rate_tol=1e-3, memory=10, first_step=None, callback=None, h0=None):
    """Minimize f with l-BFGS; fg(x) -> (f: float, g: tensor like x). first_step: the
    largest |change| of x the first line search starts from (the later ones start from the
    unit quasi-Newton step). h0: an optional positive diagonal D (tensor like x) for the
    initial inverse Hessian, used as gamma_k D with gamma_k = s^T y / (y^T D y) of the latest
    pair (D alone before the first pair); None is the identity. Returns (x, Record)."""
    rec = Record()
    x = x0.clone()
    f, g = fg(x)
    rec.evaluations += 1
    rec.phi.append(f)
    S, Y, R = [], [], []
    for it in range(max_iter):
        # two-loop recursion: d = -H g
        q = g.clone()
        alphas = []
        for s, y, r in zip(reversed(S), reversed(Y), reversed(R)):
            a = r * _dot(s, q)
            alphas.append(a)
            q -= a * y
        if h0 is not None:
            if S:
                q *= h0 * (_dot(S[-1], Y[-1]) / _dot(Y[-1], h0 * Y[-1]))
            else:
                q *= h0
        elif S:
            q *= _dot(S[-1], Y[-1]) / _dot(Y[-1], Y[-1])
        for (s, y, r), a in zip(zip(S, Y, R), reversed(alphas)):
            b = r * _dot(y, q)
            q += (a - b) * s
        d = -q
        if S:
            alpha = 1.0
        else:
            scale = float(d.abs().max())
            alpha = (first_step / scale) if (first_step and scale > 0.0) else 1.0
        found = wolfe_search(fg, x, f, g, d, alpha, record=rec)
        if found is None:
            rec.stop = "line search failed"
            break
        a, f_new, g_new = found
        s, y = a * d, g_new - g
        sy = _dot(s, y)
        if sy > 0.0:                                   # keep the pair only if curvature is positive
            S.append(s)
            Y.append(y)
            R.append(1.0 / sy)
            if len(S) > memory:
                del S[0], Y[0], R[0]
        x = x + s
        rate = convergence_rate(f, f_new)
        f, g = f_new, g_new
        rec.phi.append(f)
        rec.rate.append(rate)
        if callback is not None:
            callback(it, x, f)
        if rate < rate_tol:
            rec.stop = "convergence rate below %g" % rate_tol
            break
    else:
        rec.stop = "iteration limit"
    return x, rec


class _Problem:
    """Shared set-up: grid, shots, sources, observed data and the starting model, and the
    parameterization of the unknowns: relative Vp, Vs perturbations on the grid, or, with
    ``bspline=(dz_nodes, dx_nodes)``, their cubic B-spline coefficients (efwi.bspline_*; the
    field example's smoothing regularization); ``mask`` [nz][nx] multiplies the gradients on
    the grid (the field example restricts the update to the reservoir layer)."""

    def __init__(self, w, d_obs, device=None, bspline=None, mask=None):
        self.dev = device if device is not None else torch.device("cuda")
        self.w = w
        self.grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)
        self.shots = [efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, ckpt_interval=w.nt) for s in w.shots]
        self.ns = len(self.shots)
        self.src = torch.tensor(np.stack([np.outer(s.M, w.stf) for s in w.shots]), dtype=torch.float32,
                                device=self.dev)
        self.d_obs = d_obs
        self.m0 = torch.tensor(w.m_start, dtype=torch.float32, device=self.dev)
        self.ws = efwi.workspace(efwi.workspace_size(efwi.WS_BATCH, self.grid, self.shots), self.dev)
        self.data_phi = None
        self.bspline = None if bspline is None else (int(bspline[0]), int(bspline[1]))
        self.mask = mask

    def _xshape(self):
        if self.bspline is None:
            return (self.w.nz, self.w.nx)
        return (efwi.bspline_nodes(self.w.nz, self.bspline[0]), efwi.bspline_nodes(self.w.nx, self.bspline[1]))

    def _rel(self, x):
        """Relative perturbations on the grid from the unknowns."""
        if self.bspline is None:
            return x
        return efwi.bspline_expand(x.contiguous(), self.w.nz, self.w.nx, *self.bspline)

    def _grad_x(self, g_rel):
        """Gradient with respect to the unknowns from the one on the grid's relative
        perturbations: mask, then the B-spline transpose."""
        if self.mask is not None:
            g_rel = g_rel * self.mask
        if self.bspline is None:
            return g_rel.contiguous()
        return efwi.bspline_adjoint(g_rel.contiguous(), *self.bspline)

    def _data(self, m_ext):
        g, phi = efwi.batch_gradient(self.grid, self.shots, m_ext, self.src, self.d_obs, ws=self.ws)
        return g, float(phi.sum())


class ExtendedFWI(_Problem):
    """eq.(8): sum_s 1/2 ||d_s(m_s) - d_obs_s||^2 + 1/2 eta^2 ||(I - S^T S_w) W m~||^2 over
    x [nc][2][nz][nx] (relative Vp, Vs perturbations of every component). With ``groups``
    (one index per shot) the model is extended along groups of sources: shot s runs on
    component groups[s], nc = max(groups) + 1, and b, sink hold one zone per group."""

    def __init__(self, w, d_obs, b, sink, eta, device=None, groups=None, bspline=None, mask=None):
        super().__init__(w, d_obs, device, bspline, mask)
        self.b, self.sink, self.eta = b, sink, eta
        self.groups = None if groups is None else [int(k) for k in groups]
        self.nc = self.ns if groups is None else max(self.groups) + 1
        self.rws = efwi.workspace(efwi.workspace_size(efwi.WS_REGULARIZER, self.grid, []), self.dev)

    def _data(self, m_ext):
        if self.groups is None:
            return super()._data(m_ext)
        g, phi = efwi.batch_gradient_grouped(self.grid, self.shots, self.groups, m_ext, self.src, self.d_obs,
                                             ws=self.ws)
        return g, float(phi.sum())

    def x0(self):
        return torch.zeros((self.nc, 2) + self._xshape(), dtype=torch.float32, device=self.dev)

    def model(self, x):
        m = self.m0.unsqueeze(0).repeat(self.nc, 1, 1, 1)
        m[:, :2] *= 1.0 + self._rel(x)
        return m.contiguous()

    def __call__(self, x):
        m = self.model(x)
        g, phi_d = self._data(m)
        phi_r = efwi.extension_regularizer(self.grid, m, self.b, self.sink, self.eta, g, ws=self.rws)
        self.data_phi = phi_d
        return phi_d + float(phi_r), self._grad_x(g[:, :2] * self.m0[:2])

    def final(self, x):
        """eq.(9): the physical model S_w W m~."""
        return efwi.final_model(self.grid, self.model(x), self.b, self.sink)


class ConventionalFWI(_Problem):
    """Conventional misfit: every shot on the one model m, x [2][...] (grid or B-spline
    coefficients)."""

    def x0(self):
        return torch.zeros((2,) + self._xshape(), dtype=torch.float32, device=self.dev)

    def model(self, x):
        m = self.m0.clone()
        m[:2] *= 1.0 + self._rel(x)
        return m

    def __call__(self, x):
        m = self.model(x)
        g, phi = self._data(m.unsqueeze(0).repeat(self.ns, 1, 1, 1).contiguous())
        self.data_phi = phi
        return phi, self._grad_x(g.sum(0)[:2] * self.m0[:2])

    def final(self, x):
        return self.model(x)


class PreconditionedFWI(ConventionalFWI):
    """Conventional misfit, but the solver receives the heuristic gradient of eq.(15): the
    per-shot gradients g_s (each shot on the common model) stacked as an extended vector and
    mapped by S_w W (efwi.final_model with the zones' weights and sinkholes) instead of
    summed. The objective is unchanged, so the direction need not descend."""

    def __init__(self, w, d_obs, b, sink, device=None, bspline=None, mask=None):
        super().__init__(w, d_obs, device, bspline, mask)
        self.b, self.sink = b, sink

    def __call__(self, x):
        m = self.model(x)
        g, phi = self._data(m.unsqueeze(0).repeat(self.ns, 1, 1, 1).contiguous())
        self.data_phi = phi
        gbar = efwi.final_model(self.grid, g, self.b, self.sink)
        return phi, self._grad_x(gbar[:2] * self.m0[:2])


def inverse_pseudo_hessian(prob, clip):
    """The diagonal initial inverse Hessian of the mute + pseudo-Hessian method for a
    conventional problem over x [2][nz][nx]: efwi.pseudo_hessian at the starting model with
    the inverting side's sources, the same weight for Vp and Vs. The unknowns must be on the
    grid (no B-spline parameterization)."""
    if prob.bspline is not None:
        raise ValueError("the diagonal pseudo-Hessian acts on grid unknowns, not on B-spline coefficients")
    m_ext = prob.m0.unsqueeze(0).repeat(prob.ns, 1, 1, 1).contiguous()
    _, p = efwi.pseudo_hessian(prob.grid, prob.shots, m_ext, prob.src, clip, ws=prob.ws)
    return p.unsqueeze(0).repeat(2, 1, 1).contiguous()


def synthetic_comparison(source_errors=False, eta_rel=1.0, max_iter=60, rate_tol=1e-3, nt=1600, mute_m=100.0,
                         device=None, log=None, methods=("conventional", "extended"), ph_mute_m=200.0,
                         ph_clip=0.01, sink_m=(20.0, 100.0), anomalies=None, shift_cells=1):
    """Conventional and extended FWI on the guided-wave synthetic (inputs.guided_wave_synthetic):
    noise-free data from the true model and the true sources, inverted with the exact or the
    perturbed source parameters; returns the iterations, stop reasons and the cosine
    similarity (eq.(14)) of the inverted Vp and Vs perturbations with the true ones, over the
    model without its absorbing strips. eta^2 = eta_rel * Phi_data(start) / ||0.01 m_start||^2
    summed over the components (Vp, Vs), i.e. a uniform 1% inconsistency costs eta_rel times
    the starting data misfit. ``methods`` may also name the paper's two alternatives:
    "mute_pseudo_hessian" (channels within ph_mute_m of a source dropped, the approximate
    inverse pseudo-Hessian with clip fraction ph_clip as the initial inverse Hessian) and
    "gradient_preconditioning" (eq.(15) with the extended FWI's zones). ``sink_m`` gives the
    sinkholes' vertical and horizontal semi-axes in metres; ``anomalies`` the true model's
    blobs (inputs.guided_wave_synthetic); ``shift_cells`` the assumed sources' shift to the
    left in the source-error protocol."""
    from . import inputs
    dev = device if device is not None else torch.device("cuda")
    kw = {} if anomalies is None else {"anomalies": anomalies}
    w_true = inputs.guided_wave_synthetic(nt=nt, mute_m=mute_m, **kw)
    w = inputs.with_source_errors(w_true, shift_cells=shift_cells) if source_errors else w_true
    grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    m_true = T(w_true.m_true)
    d_obs = torch.cat([efwi.model_forward(grid, efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix), m_true,
                                          T(np.outer(s.M, w_true.stf))) for s in w_true.shots])
    # zones of influence around the assumed source positions: an elliptical sinkhole
    # (20 m vertical, 100 m horizontal semi-axes) in a zone covering the whole model
    zones = [efwi.make_zone((s.src_iz * w.dz, 0.0, s.src_ix * w.dx), (1 / sink_m[0] ** 2, 0.0, 1 / sink_m[1] ** 2, 0.0, 0.0, 0.0),
                            (0.0, (w.nz - 1) * w.dz, 0.0, 0.0, 0.0, (w.nx - 1) * w.dx), 0.0) for s in w.shots]
    b, sink = efwi.zoi_weights(grid, zones, 2.0, 0.9, device=dev)
    out = {"source_errors": source_errors, "eta_rel": eta_rel, "mute_m": mute_m, "sink_m": list(sink_m)}
    P = w.npml + 1
    interior = (slice(None), slice(P, w.nz - P), slice(P, w.nx - P))
    true_pert = (w_true.m_true[:2] - w.m_start[:2]) / w.m_start[:2]
    conv = ConventionalFWI(w, d_obs, dev)
    phi0, _ = conv(conv.x0())
    m_sc = conv.m0[:2].double()
    eta = float(np.sqrt(eta_rel * phi0 / float(conv.ns * torch.sum((0.01 * m_sc) ** 2))))
    problems = {"conventional": lambda: (conv, None), "extended": lambda: (ExtendedFWI(w, d_obs, b, sink, eta, dev), None),
                "gradient_preconditioning": lambda: (PreconditionedFWI(w, d_obs, b, sink, dev), None)}

    def muted():
        wt = inputs.guided_wave_synthetic(nt=nt, mute_m=ph_mute_m, **kw)
        wm = inputs.with_source_errors(wt, shift_cells=shift_cells) if source_errors else wt
        dm = torch.cat([efwi.model_forward(grid, efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix), m_true,
                                           T(np.outer(s.M, wt.stf))) for s in wt.shots])
        prob = ConventionalFWI(wm, dm, dev)
        return prob, inverse_pseudo_hessian(prob, ph_clip)

    problems["mute_pseudo_hessian"] = muted
    for name in methods:
        prob, h0 = problems[name]()
        x, rec = lbfgs(prob, prob.x0(), max_iter=max_iter, rate_tol=rate_tol, first_step=0.01, h0=h0)
        m = prob.final(x).cpu().numpy().astype(np.float64)
        pert = (m[:2] - w.m_start[:2]) / w.m_start[:2]
        prob(x)   # the data misfit of the accepted iterate (the last evaluation may be a rejected trial)
        out[name] = {"iterations": len(rec.rate), "evaluations": rec.evaluations, "stop": rec.stop,
                     "phi": [rec.phi[0], rec.phi[-1]], "data_phi_final": prob.data_phi,
                     "cs_vp": cosine_similarity(pert[0][interior[1:]], true_pert[0][interior[1:]]),
                     "cs_vs": cosine_similarity(pert[1][interior[1:]], true_pert[1][interior[1:]])}
        if log:
            log(f"{name}: {out[name]}")
    return out
