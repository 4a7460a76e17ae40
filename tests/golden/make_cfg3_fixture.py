"""Writes ``cfg3_step1.json``: the FP64 oracle's first time step of eq. (4)
on the cfg3 workload (3-D, p = 3, 659,920 dofs, 512 subdomains + P1 coarse,
fibre field 10:1), as sampled entries of U^1 plus whole-vector norms.

The oracle takes about 14 min of setup and 9 min for the step on 8 host
cores, too long for a test, so its result is stored.  Only ``oracle/`` and
``pdg_inputs/`` are called: every stored value is the oracle's.

Usage: ``python tests/golden/make_cfg3_fixture.py``.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.monodomain import Monodomain  # noqa: E402
from pdg_inputs import problems  # noqa: E402

N_SAMPLES = 2048
SAMPLE_SEED = 31


def main(out=os.path.join(HERE, "cfg3_step1.json")):
    t0 = time.time()
    pr = problems.cfg3()
    print(f"cfg3: {pr.n_elem} elements, {pr.n_dof} dofs; oracle setup", flush=True)
    md = Monodomain(pr)
    t1 = time.time()
    print(f"setup {t1 - t0:.0f} s; step 1", flush=True)
    U0, Up0, Y0 = md.initial_state()
    _, I = md.ionic_update(U0, Up0, Y0)
    b = md.rhs(U0, I)
    U1, _, _, info = md.step(U0, Up0, Y0)
    t2 = time.time()
    print(f"step {t2 - t1:.0f} s, {info.iters} iterations", flush=True)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(pr.n_dof, N_SAMPLES, replace=False))
    k = info.iters
    rec = {
        "what": "FP64 oracle, first Crank-Nicolson step of eq. (4) on the cfg3 workload "
                "(pdg_inputs.problems.cfg3), PCG with the two-level additive Schwarz "
                "preconditioner of eq. (5) (FP64 Cholesky solves) from x0 = U^0 to relres 1e-10",
        "script": "tests/golden/make_cfg3_fixture.py",
        "n_dof": int(pr.n_dof),
        "iters": int(k),
        "bnorm": float(np.linalg.norm(b)),
        # recurrence residual norms at the last two iterations (for the
        # one-iteration tie-break of the parity tests)
        "resnorm_last": [float(info.resnorms[k - 1]), float(info.resnorms[k])],
        "norm_U1": float(np.linalg.norm(U1)),
        "norm_dU": float(np.linalg.norm(U1 - U0)),
        "sample_seed": SAMPLE_SEED,
        "idx": [int(i) for i in idx],
        "U1": [float(v) for v in U1[idx]],
        "U0": [float(v) for v in U0[idx]],
        "oracle_seconds": {"setup": round(t1 - t0, 1), "step": round(t2 - t1, 1)},
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=0)
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
