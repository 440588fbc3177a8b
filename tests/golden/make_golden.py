"""Write tests/golden/<config>_oracle.json: FP64 oracle results for a
synthetic workload, used by the GPU parity tests at full size.

Calls only the oracle package (and the seeded input generator).  Stored:
kept NAF count and the eigenvalues around the cut, the Laplace grid of the
oracle, QP energies and Z factors in the sum-over-states form (no Laplace
transform) and in the Laplace form with the oracle's grid, Sigma on the Pade
nodes, W_nm at sampled frequencies and the trace and Frobenius norm of every
Laplace matrix M^m (all invariant under rotations of the NAF basis, so any
correct eigensolver reproduces them).

Workloads whose raw tensors do not fit in host memory ("large") are
streamed: the NAF metric (Eq. 11) is a sum over rows, accumulated over
occupied-index chunks of the generator, and the transformation (Eq. 13) is
applied chunk by chunk; everything after the transformation is the oracle's
chain unchanged.

"medium_sweep" stores the sum-over-states QP energies of the medium
workload at F = 32, 64 and 128 imaginary frequencies (the references of the
grid sweep, Fig. 4 and Sec. 3).

usage: python tests/golden/make_golden.py medium|large|medium_literal|medium_sweep
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
from gwsynth.problem import ProblemStream  # noqa: E402
from oracle import grids, naf  # noqa: E402
from oracle.g0w0 import g0w0_naf, g0w0_problem  # noqa: E402

STREAMED = {"large"}


def _log(t0, msg):
    print(f"[{time.time() - t0:7.1f} s] {msg}", flush=True)


def _streamed_naf(cfg, t0, chunk=16):
    """NAF metric, basis and transformed tensors of a streamed workload."""
    src = ProblemStream(cfg)
    o, v, A = cfg.n_act_occ, cfg.n_virt, cfg.n_aux
    _log(t0, "QP rows generated")
    K = np.zeros((A, A))
    for i0 in range(0, o, chunk):
        i1 = min(o, i0 + chunk)
        K += naf.naf_metric(src.oo_chunk(i0, i1), src.ov_chunk(i0, i1))
        _log(t0, f"metric: occupied {i1}/{o}")
    lam, U = naf.naf_basis(K, cfg.eps_naf, cfg.max_keep)
    del K
    n = U.shape[1]
    _log(t0, f"NAF basis: {n} of {A} kept")
    Rt_ov = np.empty((o * v, n))
    for i0 in range(0, o, chunk):
        i1 = min(o, i0 + chunk)
        Rt_ov[i0 * v:i1 * v] = naf.naf_transform(src.ov_chunk(i0, i1), U)
        _log(t0, f"transform: occupied {i1}/{o}")
    Rt_qp = naf.naf_transform(src.R_qp, U)
    return src.eps, src.qp, lam, U, Rt_ov, Rt_qp


def sweep_references(t0, F_list=(32, 64, 128)):
    """Sum-over-states QP energies of the medium workload at several F."""
    cfg = get_config("medium")
    prob = make_problem(cfg)
    _log(t0, "generated medium")
    common = dict(n_pade=cfg.n_pade, x0=cfg.x0, eta=cfg.eta)
    out = {"config": "medium_sweep", "qp": np.asarray(prob.qp).tolist(), "F": list(F_list)}
    base = None
    for F in F_list:
        if base is None:
            base = g0w0_problem(prob, n_freq=F)
            res = base
        else:
            res = g0w0_naf(prob.eps, cfg.n_fc, cfg.n_occ, prob.qp, base.Rt_ov, base.Rt_qp,
                           lam=base.lam, U=base.U, n_freq=F, **common)
        out[f"eps_qp_sos_F{F}"] = res.eps_qp.tolist()
        out[f"z_sos_F{F}"] = res.z.tolist()
        _log(t0, f"sum-over-states chain at F = {F} done")
    path = os.path.join(HERE, "medium_sweep_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    _log(t0, f"wrote {path}")


def main(name: str):
    if name == "medium_sweep":
        return sweep_references(time.time())
    cfg = get_config(name)
    t0 = time.time()
    common = dict(n_freq=cfg.n_freq, n_pade=cfg.n_pade, x0=cfg.x0, eta=cfg.eta)
    if name in STREAMED:
        eps, qp, lam, U, Rt_ov, Rt_qp = _streamed_naf(cfg, t0)
        sos = g0w0_naf(eps, cfg.n_fc, cfg.n_occ, qp, Rt_ov, Rt_qp, lam=lam, U=U, **common)
    else:
        prob = make_problem(cfg)
        eps, qp = prob.eps, prob.qp
        _log(t0, f"generated {name}")
        sos = g0w0_problem(prob)
        lam, U, Rt_ov, Rt_qp = sos.lam, sos.U, sos.Rt_ov, sos.Rt_qp
        del prob
    _log(t0, "sum-over-states chain done")
    lo, hi = grids.lt_bounds(eps, cfg.n_fc, cfg.n_occ, sos.omega[0])
    x, w, err = grids.lt_grid(cfg.n_lt, lo, hi)
    lt = g0w0_naf(eps, cfg.n_fc, cfg.n_occ, qp, Rt_ov, Rt_qp, lam=lam, U=U, lt=(x, w),
                  keep=True, **common)
    _log(t0, "Laplace chain done")
    n = sos.n_naf
    jsel = sorted(set([0, len(sos.omega) // 2, len(sos.omega) - 1]))
    if name in STREAMED:
        jsel = jsel[:2]
    out = {
        "config": name,
        "n_naf": int(n),
        "eig_near_cut": lam[max(0, n - 5):n + 5].tolist(),
        "eig_top": lam[:5].tolist(),
        "lt_x": x.tolist(), "lt_w": w.tolist(), "lt_err_norm": float(err),
        "lt_bounds": [float(lo), float(hi)],
        "qp": np.asarray(qp).tolist(),
        "eps_qp_sos": sos.eps_qp.tolist(), "z_sos": sos.z.tolist(),
        "eps_qp_lt": lt.eps_qp.tolist(), "z_lt": lt.z.tolist(),
        "sigma_sos_re": sos.sigma.real.tolist(), "sigma_sos_im": sos.sigma.imag.tolist(),
        "sigma_lt_re": lt.sigma.real.tolist(), "sigma_lt_im": lt.sigma.imag.tolist(),
        "w_freq_index": jsel,
        "W_lt_sel": lt.W[jsel].tolist(),
        "W_sos_sel": sos.W[jsel].tolist(),
        "M_trace": [float(np.trace(m)) for m in lt.M],
        "M_fro": [float(np.linalg.norm(m)) for m in lt.M],
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    _log(t0, f"wrote {path}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "medium")
