"""Coarse-graining transform and the paper's scalar formulas, in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 2.4 of arXiv:2211.06142:
  eq 14      k = d_g / d_p
  eq 15-16   n_CG = n_p / n_g = k^3
  eq 19-20   rho_g = rho_p, m_g = k^3 m_p
  eq 22-24   F_c,g = k^2 F_c,p  =>  gamma_g = k gamma_p
  eq 27-28   W_g = k^3 W_p      =>  E*_g = E*_p
  eq 29-30   delta_g = k delta_p, a_g = k a_p
  eq 31-34   damping scales k^2 => beta_g = beta_p, e_g = e_p
  eq 35      mu_g = mu_p
  Table 3    only the surface energy changes
SSW / SSP (Fig. 3 and the PSD paragraph of section 3.1): SSW multiplies every
diameter by k; SSP uses one size, k times the mean diameter of the fine system.
"""
import math

import numpy as np


def scale_material(fine, k):
    """Grain-scale material from the fine one (Table 3).  fine: dict with
    rho, E, nu, e, mu, mu_roll, gamma.  Returns a new dict with k_cg = k."""
    if k < 1.0:
        raise ValueError("coarse-grain factor k must be >= 1 (eq 14)")
    g = dict(fine)
    g["gamma"] = k * fine["gamma"]      # eq 24
    g["k_cg"] = k
    return g


def ssw_diameters(d_fine, k):
    """SSW: every diameter times k (polydispersity kept)."""
    return k * np.asarray(d_fine, dtype=np.float64)


def mean_diameter(d_fine):
    """Mass-equivalent mean diameter (sum d^3 / N)^(1/3) of a number sample."""
    d = np.asarray(d_fine, dtype=np.float64)
    return float(np.cbrt(np.mean(d ** 3)))


def mean_diameter_mass_fractions(diam, mass_frac):
    """Mass-equivalent mean diameter of a PSD given by mass fractions
    (Table 2 layout): number of particles of class i is proportional to
    w_i / d_i^3, so (sum n_i d_i^3 / sum n_i)^(1/3) = (sum w_i / sum w_i/d_i^3)^(1/3)."""
    d = np.asarray(diam, dtype=np.float64)
    w = np.asarray(mass_frac, dtype=np.float64)
    return float((w.sum() / np.sum(w / d ** 3)) ** (1.0 / 3.0))


def ssp_diameter(d_fine, k):
    """SSP: one monodisperse size, k times the mean diameter."""
    return k * mean_diameter(d_fine)


def grain_count(n_fine, k):
    """eq 15-16: n_g = n_p / k^3."""
    return n_fine / k ** 3


def rayleigh_dt(R_mean, rho, E, nu):
    """eq 37-38 with the shear modulus G = E / (2 (1 + nu))."""
    G = E / (2.0 * (1.0 + nu))
    beta_r = 0.8766 + 0.163 * nu
    return math.pi * R_mean / beta_r * math.sqrt(rho / G)


def unresolved_ok(x_cfd, d_mean):
    """eq 36: x_cfd / d_mean > 3."""
    return x_cfd / d_mean > 3.0


def dimensionless_production(t, M):
    """eq 39-40: t_d = t / t_end and M_d(t) = int_0^t M / int_0^t_end M
    (trapezoid rule on the sampled M(t))."""
    t = np.asarray(t, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (M[1:] + M[:-1]) * np.diff(t))])
    return t / t[-1], cum / cum[-1]


def rmsre(ref, model):
    """eq 41 with the square inside the root: sqrt(mean(((ref - model)/ref)^2)) * 100."""
    ref = np.asarray(ref, dtype=np.float64)
    model = np.asarray(model, dtype=np.float64)
    return float(np.sqrt(np.mean(((ref - model) / ref) ** 2)) * 100.0)


def speedup(t_fine, t_coarse):
    """eq 43."""
    return t_fine / t_coarse
