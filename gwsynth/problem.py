"""Seeded synthetic orbital energies and RI three-index tensors.

Recipe (all draws seeded; orbital indices are absolute, 0 = lowest):

* Energies: the ``n_fc`` frozen-core orbitals sit exactly at ``e_core``.
  Active occupied energies are sorted U(e_occ_range) draws with the HOMO
  pinned at the top of the range; virtual energies are sorted
  U(e_virt_range) draws with the LUMO and the highest virtual pinned at the
  ends of the range.
* Tensor: B^P_pq = c * sum_j U_Pj s_j V_j(pq) for p <= q, mirrored for
  p > q, with U a Haar-random orthogonal n_aux x n_aux matrix and
  s_j = exp(-j / tau).
  - ``exact_orthonormal`` (the tiny molecule): V has exactly orthonormal
    rows over every unique orbital pair (frozen core included), c = 1.
  - otherwise V_j(pq) = G_j(pq) / sqrt(n_all) with G a counter-based
    (SplitMix64) uniform on [-sqrt 3, sqrt 3] keyed on (pair, j), so any
    block of rows can be generated on its own and blocks agree; n_all is
    the number of unordered pairs over all orbitals, so the rows are nearly
    orthonormal over the pairs as in the tiny molecule, and c = 1.  Unless
    the configuration fixes tau, it is chosen so that about naf_target
    natural auxiliary functions exceed eps_naf (see ``decay_length``).

Only the blocks the hot path reads are materialised, over active orbitals:
``R_oo`` [o][o][A], ``R_ov`` [o*v][A] (i-major: row i*v + a) and ``R_qp``
[Q][M][A] (rows n in the QP set, m over all active orbitals).
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

from .configs import Config

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64_uniform(key: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 (Steele, Lea & Flood 2014) evaluated at state
    key + (counter + 1) * golden; returns doubles in [0, 1)."""
    with np.errstate(over="ignore"):
        z = (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = z + np.uint64(key & 0xFFFFFFFFFFFFFFFF)
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _seed_key(seed: int) -> int:
    return (seed * 0xD1B54A32D192ED03 + 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF


@dataclasses.dataclass
class Problem:
    cfg: Config
    eps: np.ndarray      # [n_occ + n_virt] all orbital energies (Ha)
    qp: np.ndarray       # absolute indices of the QP states (all active)
    R_oo: np.ndarray     # [o][o][A]
    R_ov: np.ndarray     # [o*v][A], row i*v + a
    R_qp: np.ndarray     # [Q][M][A], m over active orbitals
    c_scale: float

    @property
    def n_occ(self):
        return self.cfg.n_occ

    @property
    def n_fc(self):
        return self.cfg.n_fc

    @property
    def n_virt(self):
        return self.cfg.n_virt

    @property
    def n_aux(self):
        return self.cfg.n_aux


def _energies(cfg: Config, rng: np.random.Generator) -> np.ndarray:
    o = cfg.n_act_occ
    lo, hi = cfg.e_occ_range
    occ = np.sort(np.concatenate([rng.uniform(lo, hi, size=o - 1), [hi]]))
    vlo, vhi = cfg.e_virt_range
    virt = np.sort(np.concatenate([[vlo], rng.uniform(vlo, vhi, size=cfg.n_virt - 2), [vhi]]))
    core = np.full(cfg.n_fc, cfg.e_core)
    return np.concatenate([core, occ, virt])


def decay_length(cfg: Config) -> float:
    """Decay length tau of s_j = exp(-j / tau).  With unit-variance pair
    functions normalised over all n_all orbital pairs (c = 1, as for the tiny
    molecule), the NAF metric has expected eigenvalues
    2 f exp(-2 j / tau), f = (o^2 + 2 o v) / n_all; tau puts the eigenvalue
    midway between j = naf_target - 1 and naf_target at eps_naf (1e-2 when
    eps_naf is 0), unless the configuration fixes tau."""
    if cfg.tau > 0:
        return cfg.tau
    o, v = cfg.n_act_occ, cfg.n_virt
    n_tot = cfg.n_occ + cfg.n_virt
    f = (o * o + 2 * o * v) / (n_tot * (n_tot + 1) / 2.0)
    eps = cfg.eps_naf if cfg.eps_naf > 0 else 1e-2
    return (2 * cfg.naf_target - 1) / math.log(2 * f / eps)


def _haar(n: int, rng: np.random.Generator) -> np.ndarray:
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))[None, :]


def _pair_index(p: np.ndarray, q: np.ndarray, n: int) -> np.ndarray:
    """Index of the unordered pair {p, q} among the n(n+1)/2 pairs."""
    a = np.minimum(p, q).astype(np.int64)
    b = np.maximum(p, q).astype(np.int64)
    return a * n - (a * (a - 1)) // 2 + (b - a)


class _RowSource:
    """Rows B[pair, :] of the synthetic tensor for arbitrary orbital pairs."""

    def __init__(self, cfg: Config, rng: np.random.Generator):
        self.cfg = cfg
        A = cfg.n_aux
        self.n_tot = cfg.n_occ + cfg.n_virt
        self.U = _haar(A, rng)
        if cfg.exact_orthonormal:
            s = np.exp(-np.arange(A) / cfg.tau)
            n_pairs = self.n_tot * (self.n_tot + 1) // 2
            if n_pairs < A:
                raise ValueError("exact_orthonormal needs n_pairs >= n_aux")
            g = rng.standard_normal((n_pairs, A))
            vt, _ = np.linalg.qr(g)          # [n_pairs][A], orthonormal columns
            self.c = 1.0
            self.all_rows = (vt * (self.c * s)[None, :]) @ self.U.T
        else:
            n_all = self.n_tot * (self.n_tot + 1) / 2.0
            self.c = cfg.c_scale
            self.tau = decay_length(cfg)
            s = np.exp(-np.arange(A) / self.tau)
            self.colscale = (self.c / math.sqrt(n_all)) * s * math.sqrt(3.0)
            self.key = _seed_key(cfg.seed)
            self.all_rows = None

    def _g_block(self, idx: np.ndarray) -> np.ndarray:
        A = self.cfg.n_aux
        j = np.arange(A, dtype=np.uint64)
        ctr = idx.astype(np.uint64)[:, None] * np.uint64(A) + j[None, :]
        return (2.0 * splitmix64_uniform(self.key, ctr) - 1.0) * self.colscale[None, :]

    def rows(self, p: np.ndarray, q: np.ndarray, dtype=np.float64,
             block: int = 16384, sub: int = 1024) -> np.ndarray:
        """B rows for orbital pairs (p[r], q[r]) (absolute indices)."""
        import concurrent.futures
        idx = _pair_index(np.asarray(p), np.asarray(q), self.n_tot)
        if self.all_rows is not None:
            return self.all_rows[idx].astype(dtype)
        A = self.cfg.n_aux
        out = np.empty((idx.size, A), dtype=dtype)
        UT = self.U.T
        workers = min(16, os.cpu_count() or 1)
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            for b0 in range(0, idx.size, block):
                bi = idx[b0:b0 + block]
                parts = list(ex.map(self._g_block,
                                    [bi[s0:s0 + sub] for s0 in range(0, bi.size, sub)]))
                out[b0:b0 + bi.size] = np.concatenate(parts) @ UT
        return out


def _qp_states(cfg: Config) -> np.ndarray:
    nf, no, nv = cfg.n_fc, cfg.n_occ, cfg.n_virt
    homo, lumo = no - 1, no
    qp = np.concatenate([np.arange(homo - cfg.n_qp_occ + 1, homo + 1),
                         np.arange(lumo, lumo + cfg.n_qp_virt)])
    if qp.min() < nf or qp.max() >= no + nv:
        raise ValueError("QP states must be active orbitals")
    return qp


class ProblemStream:
    """The problem of ``make_problem(cfg)`` with the occupied-occupied and
    occupied-virtual blocks produced in occupied-index chunks on the host
    (same draws, same rows), for shapes whose whole tensor does not fit in
    host memory.  ``R_qp`` is materialised."""

    def __init__(self, cfg: Config, dtype=np.float64):
        if cfg.exact_orthonormal:
            raise ValueError("the exactly orthonormal (tiny) recipe is not streamed")
        rng = np.random.default_rng(cfg.seed)
        self.cfg = cfg
        self.eps = _energies(cfg, rng)
        self.src = _RowSource(cfg, rng)
        self.qp = _qp_states(cfg)
        self.dtype = dtype
        nf, no, nv = cfg.n_fc, cfg.n_occ, cfg.n_virt
        act = np.arange(nf, no + nv)
        qn, qm = np.meshgrid(self.qp, act, indexing="ij")
        self.R_qp = self.src.rows(qn.ravel(), qm.ravel(), dtype).reshape(
            self.qp.size, cfg.n_act, cfg.n_aux)

    def oo_chunk(self, i0: int, i1: int) -> np.ndarray:
        """Rows (i, j), active occupied i in [i0, i1) and every active
        occupied j: [(i1 - i0)][o][A]."""
        c = self.cfg
        occ = np.arange(c.n_fc, c.n_occ)
        vi, vj = np.meshgrid(occ[i0:i1], occ, indexing="ij")
        return self.src.rows(vi.ravel(), vj.ravel(), self.dtype).reshape(
            i1 - i0, c.n_act_occ, c.n_aux)

    def ov_chunk(self, i0: int, i1: int) -> np.ndarray:
        """Rows i*v + a for active occupied i in [i0, i1): [(i1-i0)*v][A]."""
        c = self.cfg
        occ = np.arange(c.n_fc + i0, c.n_fc + i1)
        virt = np.arange(c.n_occ, c.n_occ + c.n_virt)
        vi, va = np.meshgrid(occ, virt, indexing="ij")
        return self.src.rows(vi.ravel(), va.ravel(), self.dtype)


def make_problem(cfg: Config, dtype=np.float64) -> Problem:
    """Build the synthetic problem for ``cfg`` (deterministic in cfg.seed)."""
    rng = np.random.default_rng(cfg.seed)
    eps = _energies(cfg, rng)
    src = _RowSource(cfg, rng)
    nf, no, nv = cfg.n_fc, cfg.n_occ, cfg.n_virt
    o, M, A = cfg.n_act_occ, cfg.n_act, cfg.n_aux
    act = np.arange(nf, no + nv)
    occ = np.arange(nf, no)
    virt = np.arange(no, no + nv)
    qp = _qp_states(cfg)

    # Unique pairs needed by the three blocks, generated once.
    pi, pj = np.meshgrid(occ, occ, indexing="ij")
    oo_p, oo_q = pi.ravel(), pj.ravel()
    vi, va = np.meshgrid(occ, virt, indexing="ij")
    ov_p, ov_q = vi.ravel(), va.ravel()
    qn, qm = np.meshgrid(qp, act, indexing="ij")
    qp_p, qp_q = qn.ravel(), qm.ravel()

    all_p = np.concatenate([oo_p, ov_p, qp_p])
    all_q = np.concatenate([oo_q, ov_q, qp_q])
    key = _pair_index(all_p, all_q, src.n_tot)
    uniq, inv = np.unique(key, return_inverse=True)
    # recover one (p, q) per unique key
    first = np.zeros(uniq.size, dtype=np.int64)
    first[inv[::-1]] = np.arange(key.size)[::-1]
    rows = src.rows(all_p[first], all_q[first], dtype=dtype)

    n_oo, n_ov = oo_p.size, ov_p.size
    R_oo = rows[inv[:n_oo]].reshape(o, o, A)
    R_ov = rows[inv[n_oo:n_oo + n_ov]].reshape(o * nv, A)
    R_qp = rows[inv[n_oo + n_ov:]].reshape(qp.size, M, A)
    del rows
    return Problem(cfg=cfg, eps=eps, qp=qp, R_oo=np.ascontiguousarray(R_oo),
                   R_ov=np.ascontiguousarray(R_ov),
                   R_qp=np.ascontiguousarray(R_qp), c_scale=src.c)
