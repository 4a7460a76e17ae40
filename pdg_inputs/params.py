"""Shared parameter tables (data only).

The paper names the Barreto-Cressman ionic model and its state variables
(intracellular Na, extracellular K, intracellular Ca, gating variables;
Section 2) but defers its equations and constants to the cited works.  The
table below is the reading both implementations use: a five-state
Cressman-type single-neuron model (n, h, [K]_o, [Na]_i, [Ca]_i).  Its constants
are recalled from the published model and are not verified against that source;
both sides read this one table, so GPU/oracle parity does not depend on them.

The order of ``IONIC_NAMES`` is the order of the parameter vector passed
through the C-ABI.
"""
from __future__ import annotations

import numpy as np

IONIC_NAMES = (
    "g_Na",     # 0  fast Na conductance            mS/cm^2
    "g_NaL",    # 1  Na leak
    "g_K",      # 2  delayed-rectifier K
    "g_KL",     # 3  K leak
    "g_AHP",    # 4  Ca-gated K (after-hyperpolarisation)
    "g_ClL",    # 5  Cl leak
    "g_Ca",     # 6  Ca conductance in the Ca balance
    "V_Ca",     # 7  Ca reversal potential           mV
    "phi",      # 8  gate time-scale factor
    "tau",      # 9  concentration time scale        ms
    "beta",     # 10 intra/extracellular volume ratio
    "rho",      # 11 pump strength
    "G_glia",   # 12 glial uptake strength
    "eps",      # 13 diffusion-to-bath rate
    "k_bath",   # 14 bath K concentration            mM
    "Cl_i",     # 15 intracellular Cl                mM
    "Cl_o",     # 16 extracellular Cl                mM
    "nernst",   # 17 RT/F factor of the Nernst potentials (mV)
    "gamma",    # 18 current-to-concentration factor
    "ca_tau",   # 19 Ca decay time                   ms
    "ca_coef",  # 20 Ca influx factor
    "K_i0",     # 21 reference intracellular K        mM
    "Na_i0",    # 22 reference intracellular Na       mM
    "Na_o0",    # 23 reference extracellular Na       mM
)

IONIC_DEFAULT = np.array([
    100.0, 0.0175, 40.0, 0.05, 0.01, 0.05, 0.1, 120.0,
    3.0, 1000.0, 7.0, 1.25, 66.0, 1.2, 4.0,
    6.0, 130.0, 26.64, 0.33, 80.0, 0.002,
    140.0, 18.0, 144.0,
], dtype=np.float64)

N_IONIC_PARAMS = len(IONIC_NAMES)
N_STATES = 5
STATE_NAMES = ("n", "h", "K_o", "Na_i", "Ca_i")

#: resting membrane potential used for initial data (mV)
U_REST = -70.0
#: initial ionic state: gates near their steady state at U_REST, rest
#: concentrations of the model.  Plain numbers (the oracle's tests check that
#: the two gate values sit within 1e-3 of the gates' steady state at U_REST).
Y_REST = np.array([0.0552, 0.9860, 4.0, 18.0, 0.0], dtype=np.float64)
