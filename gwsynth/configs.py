"""Workload shapes for the synthetic LT-AC G0W0 problems.

The shapes mirror the paper's systems: small GW100-sized molecules, water
clusters of a few thousand basis functions, the WW-6 dye and the BODIPY
tetramer (Sec. 4: water clusters 430-4300 basis functions, WW-6 with 5583
basis / 13802 auxiliary functions, BODIPY tetramer with 7412 basis
functions).  No geometry, basis set or SCF enters; every tensor is drawn
from a seeded generator (see ``problem.py``).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_occ: int            # occupied orbitals, frozen core included
    n_fc: int             # frozen-core orbitals (lowest occupied)
    n_virt: int           # virtual orbitals
    n_aux: int            # auxiliary functions before NAF truncation
    eps_naf: float        # NAF eigenvalue threshold (strict ">")
    max_keep: int         # cap on kept NAFs (0 = no cap)
    naf_target: int       # NAF count the tensor scale is tuned to give
    tau: float            # singular-value decay s_j = exp(-j / tau); 0 = derived
                          # from naf_target (gwsynth.problem.decay_length)
    n_lt: int             # Laplace points
    n_freq: int           # imaginary-frequency integration points
    n_pade: int           # Pade points
    n_qp_occ: int         # QP states HOMO-(n_qp_occ-1) .. HOMO
    n_qp_virt: int        # QP states LUMO .. LUMO+(n_qp_virt-1)
    seed: int
    exact_orthonormal: bool = False  # tiny: exactly orthonormal pair rows
    c_scale: float = 1.0  # overall scale c of the tensor (B = c sum_j U s_j V_j)
    eta: float = 1e-3     # real-axis broadening (Ha)
    x0: float = 0.5       # modified Gauss-Legendre scale (Ha)
    e_core: float = -20.0
    e_occ_range: tuple = (-20.0, -0.3)
    e_virt_range: tuple = (0.05, 5.0)

    @property
    def n_act_occ(self) -> int:
        return self.n_occ - self.n_fc

    @property
    def n_act(self) -> int:
        return self.n_act_occ + self.n_virt

    @property
    def n_qp(self) -> int:
        return self.n_qp_occ + self.n_qp_virt

    def with_(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


# A tiny molecule, no NAF truncation (threshold 0): every auxiliary
# function is kept and the NAF transform is orthogonal.
TINY = Config(name="tiny", n_occ=10, n_fc=2, n_virt=40, n_aux=150,
              eps_naf=0.0, max_keep=0, naf_target=150, tau=30.0,
              n_lt=8, n_freq=32, n_pade=16, n_qp_occ=1, n_qp_virt=1,
              seed=1, exact_orthonormal=True)

# ~1000 basis functions (a water cluster of ~25 molecules in size).
MEDIUM = Config(name="medium", n_occ=100, n_fc=30, n_virt=900, n_aux=3000,
                eps_naf=1e-2, max_keep=0, naf_target=1500, tau=0.0,
                n_lt=10, n_freq=60, n_pade=16, n_qp_occ=5, n_qp_virt=5,
                seed=2)

# ~2500 basis functions.
LARGE = Config(name="large", n_occ=300, n_fc=80, n_virt=2200, n_aux=7000,
               eps_naf=1e-2, max_keep=0, naf_target=3500, tau=0.0,
               n_lt=12, n_freq=80, n_pade=16, n_qp_occ=10, n_qp_virt=10,
               seed=3)

# ~7400 basis functions (the size of the BODIPY tetramer).
PAPER = Config(name="paper", n_occ=950, n_fc=250, n_virt=6700, n_aux=20000,
               eps_naf=1e-2, max_keep=0, naf_target=9000, tau=0.0,
               n_lt=14, n_freq=100, n_pade=16, n_qp_occ=5, n_qp_virt=5,
               seed=4)



def _scale_for_target(cfg: Config) -> float:
    """Scale c that puts the expected NAF-metric eigenvalue
    c^2 2 f exp(-2 j / tau), f = (o^2 + 2 o v) / n_all, at eps_naf midway
    between j = naf_target - 1 and naf_target, for a fixed decay tau."""
    o, v = cfg.n_act_occ, cfg.n_virt
    n_tot = cfg.n_occ + cfg.n_virt
    f = (o * o + 2 * o * v) / (n_tot * (n_tot + 1) / 2.0)
    return float(np.sqrt(cfg.eps_naf / (2 * f) * np.exp((2 * cfg.naf_target - 1) / cfg.tau)))


# The medium shape with the decay exp(-j/400) taken literally; the scale c
# then has to grow (c ~ 5.9) for about 1500 functions to pass the threshold.
# Used only to report the Laplace error of that regime next to the derived
# decay of MEDIUM.
MEDIUM_LITERAL = MEDIUM.with_(name="medium_literal", tau=400.0)
MEDIUM_LITERAL = MEDIUM_LITERAL.with_(c_scale=_scale_for_target(MEDIUM_LITERAL))

CONFIGS = {c.name: c for c in (TINY, MEDIUM, LARGE, PAPER, MEDIUM_LITERAL)}


def get_config(name: str) -> Config:
    return CONFIGS[name]


def batched_configs(n_mol: int = 64) -> list[Config]:
    """Molecules of uneven size: n_occ ~ U{20..120}, v = 8 n_occ,
    n_aux = 3 (n_occ + n_virt), half the auxiliary functions kept."""
    out = []
    for b in range(n_mol):
        seed = 1000 + b
        rng = np.random.default_rng(seed)
        n = int(rng.integers(20, 121))
        v = 8 * n
        a = 3 * (n + v)
        out.append(Config(name=f"batched{b}", n_occ=n, n_fc=0, n_virt=v,
                          n_aux=a, eps_naf=0.0, max_keep=a // 2,
                          naf_target=a // 2, tau=a / 7.5, n_lt=8, n_freq=48,
                          n_pade=16, n_qp_occ=1, n_qp_virt=1, seed=seed))
    return out
