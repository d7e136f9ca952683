"""Kinetic reference for electrons radiating in a static magnetic field
perpendicular to their motion (cases 1 and 3 of the paper's Sec. 5.1, whose
expected curves come from evolving the electron distribution function rather
than from particles).

TEST INFRASTRUCTURE ONLY (part of the oracle; shares nothing with the HIP
library).

Model, for u perpendicular to B with E = 0: the rotation keeps |u|, so
chi = |u| c B / E_s depends on |u| only; the QS rate W(|u|) and the photon
fraction distribution P(chi, xi) are those of the oracle's tables (Sec. 2.2
rate, Sec. 3.2 table interpolation), and collinear emission of
gamma_gamma = (gamma - 1) xi moves |u| to |u| - gamma_gamma (momentum
conservation).  With the optical-depth method the waiting time is
memoryless, and W is constant between events in this geometry, so each
time step of length dt emits with probability 1 - exp(-W dt) independently
of the past (at most one event per step, tau redrawn): the particle loop is
exactly a discrete Markov chain in |u|.  This module evolves that chain's
distribution on a fine grid in ln|u|:
  * the never-emitted part stays an exact atom at u0;
  * a jump from the atom is spread over the grid with the exact CDF
    differences at the cell edges; a jump from a cell starts at the cell's
    centre (the only discretisation);
  * photons are tallied on their own energy grid the same way.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def implied_cdf(table: "O.Table", chi: float, xi: np.ndarray) -> np.ndarray:
    """P(xi' <= xi) for the QS table's inverse-CDF sampling at chi: rows
    interpolated linearly in ln chi (chi clamped to the table), ln P linear
    in ln xi between the stored knots, P ~ xi^(1/3) below xi_min, 1 at xi = 1
    (Sec. 3.2 sampling, read in the forward direction)."""
    t = table
    c = min(max(chi, t.chi_min), t.chi_max)
    l0, l1 = np.log(t.chi_min), np.log(t.chi_max)
    d = (l1 - l0) / (t.n_chi - 1)
    n = int(np.floor((np.log(c) - l0) / d))
    n = min(max(n, 0), t.n_chi - 2)
    f = (np.log(c) - (l0 + n * d)) / d
    row = t.cdf[n] + f * (t.cdf[n + 1] - t.cdf[n])            # ln P at the knots
    lmin = np.log(t.frac_min)
    lx = lmin * (1.0 - np.arange(t.n_frac) / (t.n_frac - 1))  # ln xi at the knots
    xi = np.asarray(xi, dtype=np.float64)
    out = np.empty_like(xi)
    with np.errstate(divide="ignore"):
        lxi = np.log(xi)
    below = lxi < lmin
    out[below] = np.exp(row[0] + (lxi[below] - lmin) / 3.0)
    mid = ~below & (xi < 1.0)
    out[mid] = np.exp(np.interp(lxi[mid], lx, row))
    out[xi >= 1.0] = 1.0
    out[xi <= 0.0] = 0.0
    return out


class StaticFieldChain:
    """Distribution of |u| (and the photon energy tally) after k steps."""

    def __init__(self, qs: "O.Table", b_norm: float, u0: float, dt: float, edges_u: np.ndarray,
                 edges_photon: np.ndarray):
        self.qs, self.b, self.u0, self.dt = qs, float(b_norm), float(u0), float(dt)
        self.eu = np.asarray(edges_u, dtype=np.float64)
        self.ep = np.asarray(edges_photon, dtype=np.float64)
        self.centres = np.sqrt(self.eu[:-1] * self.eu[1:])
        self.atom = 1.0
        self.cells = np.zeros(len(self.eu) - 1)
        self.photons = np.zeros(len(self.ep) - 1)
        self._jump_atom = self._jump_row(self.u0)
        self._p_atom = self._emit_prob(self.u0)
        self._rows = [self._jump_row(u) for u in self.centres]
        self._p_cells = np.array([self._emit_prob(u) for u in self.centres])

    def _emit_prob(self, u):
        g = np.sqrt(1.0 + u * u)
        return -np.expm1(-self.qs.rate(u * self.b, g) * self.dt)

    def _jump_row(self, u):
        """(destination masses over the |u| cells, photon masses over the
        photon cells) for one emission from |u| = u."""
        g = np.sqrt(1.0 + u * u)
        gm1 = u * u / (g + 1.0)
        chi = u * self.b
        # |u'| = u - gm1 xi  <=>  xi = (u - |u'|)/gm1 ; |u'| decreasing in xi
        xi_e = np.clip((u - self.eu) / gm1, 0.0, 1.0)
        cdf_e = implied_cdf(self.qs, chi, xi_e)
        dest = cdf_e[:-1] - cdf_e[1:]
        xi_p = np.clip(self.ep / gm1, 0.0, 1.0)
        cdf_p = implied_cdf(self.qs, chi, xi_p)
        ph = cdf_p[1:] - cdf_p[:-1]
        return dest, ph

    def step(self):
        new = self.cells * (1.0 - self._p_cells)
        photons = self.photons.copy()
        pa = self.atom * self._p_atom
        new += pa * self._jump_atom[0]
        photons += pa * self._jump_atom[1]
        moving = self.cells * self._p_cells
        for i in np.nonzero(moving > 0)[0]:
            d, p = self._rows[i]
            new += moving[i] * d
            photons += moving[i] * p
        self.atom *= 1.0 - self._p_atom
        self.cells = new
        self.photons = photons

    def run(self, steps: int):
        for _ in range(steps):
            self.step()
        return self
