"""Write tests/golden/<config>_oracle.json: FP64 oracle results for a
synthetic workload, used by the GPU parity tests at full size.

Calls only the oracle package (and the seeded input generator).  Stored:
kept NAF count and the eigenvalues around the cut, the Laplace grid of the
oracle, QP energies and Z factors in the sum-over-states form (no Laplace
transform) and in the Laplace form with the oracle's grid, Sigma on the Pade
nodes and W_nm at sampled frequencies (both invariant under rotations of
the NAF basis, so any correct eigensolver reproduces them).

usage: python tests/golden/make_golden.py medium
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from gwsynth import get_config, make_problem  # noqa: E402
from oracle import grids  # noqa: E402
from oracle.g0w0 import g0w0_problem  # noqa: E402


def main(name: str):
    cfg = get_config(name)
    t0 = time.time()
    prob = make_problem(cfg)
    print(f"generated {name} in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    sos = g0w0_problem(prob)
    print(f"SOS chain in {time.time() - t0:.1f} s", flush=True)
    lo, hi = grids.lt_bounds(prob.eps, cfg.n_fc, cfg.n_occ, sos.omega[0])
    x, w, err = grids.lt_grid(cfg.n_lt, lo, hi)
    t0 = time.time()
    lt = g0w0_problem(prob, lt=(x, w), U=sos.U)
    print(f"LT chain in {time.time() - t0:.1f} s", flush=True)
    n = sos.n_naf
    jsel = sorted(set([0, len(sos.omega) // 2, len(sos.omega) - 1]))
    out = {
        "config": name,
        "n_naf": int(n),
        "eig_near_cut": sos.lam[max(0, n - 5):n + 5].tolist(),
        "eig_top": sos.lam[:5].tolist(),
        "lt_x": x.tolist(), "lt_w": w.tolist(), "lt_err_norm": float(err),
        "lt_bounds": [float(lo), float(hi)],
        "qp": prob.qp.tolist(),
        "eps_qp_sos": sos.eps_qp.tolist(), "z_sos": sos.z.tolist(),
        "eps_qp_lt": lt.eps_qp.tolist(), "z_lt": lt.z.tolist(),
        "sigma_sos_re": sos.sigma.real.tolist(), "sigma_sos_im": sos.sigma.imag.tolist(),
        "sigma_lt_re": lt.sigma.real.tolist(), "sigma_lt_im": lt.sigma.imag.tolist(),
        "w_freq_index": jsel,
        "W_lt_sel": lt.W[jsel].tolist(),
        "W_sos_sel": sos.W[jsel].tolist(),
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "medium")
