"""Synthetic photon cross-section tables (inputs to both the HIP path and the oracle).

The paper's engine reads Livermore evaluated photon data (Sec. 2.4.1); those
tables are not available here, so every run uses a synthetic stand-in with
the same structure: per material, three partial mass attenuation
coefficients mu/rho [cm^2/g] (photoelectric, incoherent, coherent) tabulated
on a grid uniform in ln E.

Per element (Z, A, E_K) and energy E [keV], in cm^2/atom:
  * incoherent: Z * sigma_KN(E), the free-electron Klein-Nishina total cross
    section (textbook closed form);
  * photoelectric: C_pe Z^4 E^-3, divided by 7.5 below the K edge;
  * coherent: C_coh Z^2 E^-2;
  * pair production (optional fourth partial): C_pair Z^2 (1 - 2 m_e c^2 / E)^3
    above the threshold 2 m_e c^2, a negligible floor below it (the tables keep
    every partial positive; both transport codes drop the pair partial at or
    below the threshold).
A material's mu/rho is sum_i w_i (N_A / A_i) sigma_i.
"""
from __future__ import annotations

import math

import numpy as np

R_E_CM = 2.8179403262e-13       # classical electron radius [cm]
MEC2_KEV = 510.99895            # electron rest energy [keV]
N_A = 6.02214076e23
C_PE = 4.6e-23
C_COH = 3.5e-23
C_PAIR = 1.31e-27   # ~1.3e-3 cm^2/g for Ge at 2 MeV
PAIR_FLOOR = 1e-40  # cm^2/atom below the threshold
K_EDGE_JUMP = 7.5

# (Z, A, K-edge keV or None)
ELEMENTS = {
    "H": (1, 1.008, None),
    "C": (6, 12.011, None),
    "N": (7, 14.007, None),
    "O": (8, 15.999, None),
    "Al": (13, 26.9815, 1.5596),
    "Si": (14, 28.085, 1.8389),
    "Ar": (18, 39.948, 3.2059),
    "Cu": (29, 63.546, 8.979),
    "Ge": (32, 72.630, 11.103),
}

# name -> (composition by mass fraction, nominal density g/cm^3)
MATERIALS = {
    "vacuum": ({}, 0.0),
    "Ge": ({"Ge": 1.0}, 5.32),
    "Al": ({"Al": 1.0}, 2.699),
    "Cu": ({"Cu": 1.0}, 8.96),
    "air": ({"N": 0.755, "O": 0.232, "Ar": 0.013}, 1.205e-3),
    "water": ({"H": 0.1119, "O": 0.8881}, 1.0),
    "soil": ({"O": 0.5326, "Si": 0.4674}, 1.6),
    "PP": ({"C": 0.8563, "H": 0.1437}, 0.90),
}

# default grid: 1024 points uniform in ln E over [1 keV, 3 MeV]
GRID_N = 1024
GRID_E0 = 1.0
GRID_E1 = 3000.0


def grid(n=GRID_N, e0=GRID_E0, e1=GRID_E1):
    lnE0 = math.log(e0)
    dlnE = (math.log(e1) - lnE0) / (n - 1)
    return lnE0, dlnE, n


def grid_energies(lnE0, dlnE, n):
    return np.exp(lnE0 + dlnE * np.arange(n))


def sigma_kn(E_keV):
    """Klein-Nishina total cross section per electron [cm^2] (textbook form)."""
    k = np.asarray(E_keV, dtype=np.float64) / MEC2_KEV
    l = np.log1p(2.0 * k)
    a = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k)
    b = l / (2.0 * k) - (1.0 + 3.0 * k) / (1.0 + 2.0 * k) ** 2
    return 2.0 * math.pi * R_E_CM ** 2 * (a + b)


def element_sigmas(sym, E_keV):
    Z, A, EK = ELEMENTS[sym]
    E = np.asarray(E_keV, dtype=np.float64)
    s_c = Z * sigma_kn(E)
    jump = np.ones_like(E) if EK is None else np.where(E >= EK, 1.0, 1.0 / K_EDGE_JUMP)
    s_pe = C_PE * Z ** 4 * E ** -3 * jump
    s_coh = C_COH * Z ** 2 * E ** -2
    return s_pe, s_c, s_coh


def element_pair(sym, E_keV):
    Z, _, _ = ELEMENTS[sym]
    E = np.asarray(E_keV, dtype=np.float64)
    x = np.clip(1.0 - 2.0 * MEC2_KEV / E, 0.0, None)
    return np.where(E > 2.0 * MEC2_KEV, C_PAIR * Z ** 2 * x ** 3, PAIR_FLOOR)


def pair_attenuation(composition, E_keV):
    """Pair-production mu/rho [cm^2/g] for a mass-fraction mix."""
    E = np.asarray(E_keV, dtype=np.float64)
    out = np.zeros_like(E)
    for sym, w in composition.items():
        _, A, _ = ELEMENTS[sym]
        out += w * N_A / A * element_pair(sym, E)
    return out


def mass_attenuation(composition, E_keV):
    """(photo, compton, coherent) mu/rho [cm^2/g] for a mass-fraction mix."""
    E = np.asarray(E_keV, dtype=np.float64)
    out = [np.zeros_like(E), np.zeros_like(E), np.zeros_like(E)]
    for sym, w in composition.items():
        _, A, _ = ELEMENTS[sym]
        for i, s in enumerate(element_sigmas(sym, E)):
            out[i] += w * N_A / A * s
    return tuple(out)


def material_table(name, lnE0=None, dlnE=None, n=None, coherent=True, pair=False):
    """Tabulated (photo, compton, coherent[, pair]) mu/rho on the ln E grid."""
    if lnE0 is None:
        lnE0, dlnE, n = grid()
    comp, _ = MATERIALS[name]
    E = grid_energies(lnE0, dlnE, n)
    pe, c, coh = mass_attenuation(comp, E)
    if not coherent:
        coh = np.zeros_like(coh)
    if pair:
        return pe, c, coh, pair_attenuation(comp, E) if comp else np.zeros_like(pe)
    return pe, c, coh


def constant_table(photo=0.0, compton=0.0, coherent=0.0, n=GRID_N, pair=None):
    """Energy-independent synthetic partials, for closed-form tests (pair, when
    given, is a fourth partial; transport drops it at or below 2 m_e c^2)."""
    t = (np.full(n, float(photo)), np.full(n, float(compton)), np.full(n, float(coherent)))
    return t if pair is None else t + (np.full(n, float(pair)),)
