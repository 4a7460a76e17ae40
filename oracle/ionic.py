"""Barreto-Cressman-type ionic model (Section 2), vectorised over points.

The paper names the model and its states (intracellular Na, extracellular K,
intracellular Ca and gating variables) and defers the equations to the cited
works.  Reading used on both sides: the five-state single-neuron model with
states y = (n, h, [K]_o, [Na]_i, [Ca]_i), potential V = u in mV, time in ms:

    m_inf = a_m / (a_m + b_m)
    I_Na  = -g_Na m_inf^3 h (V - V_Na) - g_NaL (V - V_Na)
    I_K   = -(g_K n^4 + g_AHP Ca/(1 + Ca)) (V - V_K) - g_KL (V - V_K)
    I_Cl  = -g_ClL (V - V_Cl)
    dq/dt = phi (a_q (1 - q) - b_q q),  q in {n, h}
    d[K]_o/dt  = (-gamma I_K - 2 beta I_pump - I_glia - I_diff) / tau
    d[Na]_i/dt = (gamma I_Na / beta - 3 I_pump) / tau
    d[Ca]_i/dt = -ca_coef g_Ca (V - V_Ca) / (1 + exp(-(V + 25)/2.5)) - Ca / ca_tau

with the pump, glial and bath terms, Nernst potentials and rate functions
below.  The monodomain current is f(u, y) = -(I_Na + I_K + I_Cl) (so that
C_m du/dt = -f in a single cell, matching the sign of eq. (1)), and the ODE
right-hand side of eq. (1) is m(u, y) = -dy/dt.

The removable singularity x / (1 - exp(-x)) at x = 0 is evaluated by the
series 1 + x/2 + x^2/12 for |x| < 1e-4.

Constants: ``pdg_inputs.params`` (recalled, not verified against the cited
source; physiological fidelity is parity unpinned, the ODE integration is
pinned against scipy's adaptive integrator in the tests).
"""
from __future__ import annotations

import numpy as np

(G_NA, G_NAL, G_K, G_KL, G_AHP, G_CLL, G_CA, V_CA, PHI, TAU, BETA, RHO, G_GLIA, EPS,
 K_BATH, CL_I, CL_O, NERNST, GAMMA, CA_TAU, CA_COEF, K_I0, NA_I0, NA_O0) = range(24)


def _xexp(x):
    """x / (1 - exp(-x)) with its removable singularity at 0."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-4
    safe = np.where(small, 1.0, x)
    out = safe / (1.0 - np.exp(-safe))
    ser = 1.0 + x / 2.0 + x * x / 12.0
    return np.where(small, ser, out)


def rates(V):
    am = _xexp(0.1 * (V + 30.0))
    bm = 4.0 * np.exp(-(V + 55.0) / 18.0)
    an = 0.1 * _xexp(0.1 * (V + 34.0))
    bn = 0.125 * np.exp(-(V + 44.0) / 80.0)
    ah = 0.07 * np.exp(-(V + 44.0) / 20.0)
    bh = 1.0 / (1.0 + np.exp(-(V + 14.0) / 10.0))
    return am, bm, an, bn, ah, bh


def currents(V, y, prm):
    n, h, ko, nai, cai = y
    if np.any(ko <= 0) or np.any(nai <= 0):
        raise FloatingPointError("ionic: non-positive concentration before a logarithm")
    ki = prm[K_I0] + (prm[NA_I0] - nai)
    nao = prm[NA_O0] - prm[BETA] * (nai - prm[NA_I0])
    if np.any(ki <= 0) or np.any(nao <= 0):
        raise FloatingPointError("ionic: non-positive concentration before a logarithm")
    vna = prm[NERNST] * np.log(nao / nai)
    vk = prm[NERNST] * np.log(ko / ki)
    vcl = prm[NERNST] * np.log(prm[CL_I] / prm[CL_O])
    am, bm, an, bn, ah, bh = rates(V)
    minf = am / (am + bm)
    ina = -prm[G_NA] * minf ** 3 * h * (V - vna) - prm[G_NAL] * (V - vna)
    ik = -(prm[G_K] * n ** 4 + prm[G_AHP] * cai / (1.0 + cai)) * (V - vk) - prm[G_KL] * (V - vk)
    icl = -prm[G_CLL] * (V - vcl)
    return ina, ik, icl, (an, bn, ah, bh)


def f_ion(V, y, prm):
    """Ionic current density f(u, y) of eq. (1)."""
    ina, ik, icl, _ = currents(V, y, prm)
    return -(ina + ik + icl)


def dydt(V, y, prm):
    """Time derivative of the ionic state, dy/dt = -m(u, y); returns [5, ...]."""
    n, h, ko, nai, cai = y
    ina, ik, _, (an, bn, ah, bh) = currents(V, y, prm)
    ipump = prm[RHO] / (1.0 + np.exp((25.0 - nai) / 3.0)) / (1.0 + np.exp(5.5 - ko))
    iglia = prm[G_GLIA] / (1.0 + np.exp((18.0 - ko) / 2.5))
    idiff = prm[EPS] * (ko - prm[K_BATH])
    dn = prm[PHI] * (an * (1.0 - n) - bn * n)
    dh = prm[PHI] * (ah * (1.0 - h) - bh * h)
    dko = (-prm[GAMMA] * ik - 2.0 * prm[BETA] * ipump - iglia - idiff) / prm[TAU]
    dna = (prm[GAMMA] * ina / prm[BETA] - 3.0 * ipump) / prm[TAU]
    dca = -prm[CA_COEF] * prm[G_CA] * (V - prm[V_CA]) / (1.0 + np.exp(-(V + 25.0) / 2.5)) - cai / prm[CA_TAU]
    return np.stack([dn, dh, dko, dna, dca])


def m_ion(V, y, prm):
    """m(u, y) of eq. (1): dy/dt + m = 0."""
    return -dydt(V, y, prm)


def gate_steady_state(V):
    am, bm, an, bn, ah, bh = rates(np.asarray(V, dtype=np.float64))
    return an / (an + bn), ah / (ah + bh)
