"""Simultaneous angular fit over categories (oracle test infrastructure).

Example 2 of the paper (Ipanema-beta, arXiv:1706.01420) fits the angular x
decay-time PDF in several bins of the KK mass at once, with one data set per
bin and flavour, each category normalised on its own, the P-wave and mixing
parameters shared and the S-wave fraction and phase free per bin (its S-P
interference factor C_SP is a constant of the bin).  The joint NLL is the sum
of the categories' NLLs, each evaluated with its own parameters.

Parameter layout (SIM_SHARED first, then per bin b):
    fL, fpe, dpa, dpe, G, DG, DM, phis, mu_m, sigma_m,  Fs_0, dS_0,  Fs_1, dS_1, ...
A category is (model, cols, w, bin, settings) with model 3 (untagged sample
of B_s) or 4 (tagged, with the qd column); settings as models.pdf (its
normalisation weights xi and its bin's c_sp).
"""
import math

import numpy as np

from . import nll as N

SIM_SHARED = ("fL", "fpe", "dpa", "dpe", "G", "DG", "DM", "phis", "mu_m", "sigma_m")


def nparams(nbins):
    return len(SIM_SHARED) + 2 * nbins


def category_index(b):
    """Positions in the simultaneous vector of the 12 per-category parameters
    (fL, fpe, Fs, dpa, dpe, dS, G, DG, DM, phis, mu_m, sigma_m) of bin b."""
    s = len(SIM_SHARED)
    return [0, 1, s + 2 * b, 2, 3, s + 2 * b + 1, 4, 5, 6, 7, 8, 9]


def category_theta(theta, b):
    return [theta[i] for i in category_index(b)]


def nll(cats, theta):
    """Sum of the categories' NLLs; +inf if any is +inf."""
    tot = []
    for model, cols, w, b, settings in cats:
        f = N.nll(model, cols, category_theta(theta, b), w, settings)
        if not math.isfinite(f):
            return math.inf
        tot.append(f)
    return math.fsum(tot)


def nll_grad(cats, theta):
    """(NLL, gradient): each category's 12-component gradient, added at the
    positions its parameters take in the simultaneous vector."""
    K = len(theta)
    fs, g = [], np.zeros(K)
    for model, cols, w, b, settings in cats:
        f, gc = N.nll_grad(model, cols, category_theta(theta, b), w, settings)
        if not math.isfinite(f):
            return math.inf, np.full(K, np.nan)
        fs.append(f)
        for j, i in enumerate(category_index(b)):
            g[i] += gc[j]
    return math.fsum(fs), g
