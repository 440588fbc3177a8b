"""Device twin of the synthetic problem generator.

Same recipe and same draws as ``problem.py`` (energies and the Haar matrix U
come from the identical host random stream; the pair functions G_j(pq) are
the same counter-based SplitMix64 uniforms), evaluated with torch on a
device so the large configurations do not need tens of GB of host rows:
B rows = (2 u - 1) * colscale @ U^T, computed in FP64 and rounded to the
requested dtype, exactly as the host generator does.  The arithmetic here is
input generation only; none of the method's steps appears.

Rows are produced in blocks, so the occupied-virtual block can also be
streamed in occupied-index chunks (``ov_chunk``) for shapes whose full
tensor would not fit in device memory.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .configs import Config
import math

from .problem import (_GOLDEN, _MIX1, _MIX2, _RowSource, _energies, _pair_index, _seed_key,
                      decay_length)


def _signed(c: int) -> int:
    c &= 0xFFFFFFFFFFFFFFFF
    return c - (1 << 64) if c >= (1 << 63) else c


_G = _signed(int(_GOLDEN))
_M1 = _signed(int(_MIX1))
_M2 = _signed(int(_MIX2))


def splitmix64_uniform_torch(key: int, counters):
    """SplitMix64 (Steele, Lea & Flood 2014) at state key + (counter+1)*golden,
    on int64 tensors (two's-complement wrap-around equals the unsigned
    arithmetic; logical right shifts are arithmetic shifts masked to the
    remaining bits).  Returns float64 in [0, 1)."""
    import torch
    z = (counters + 1) * _G + _signed(key)
    z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * _M1
    z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * _M2
    z = z ^ ((z >> 31) & ((1 << 33) - 1))
    return ((z >> 11) & ((1 << 53) - 1)).to(torch.float64) * (1.0 / 9007199254740992.0)


class DeviceRowSource:
    """Rows B[pair, :] generated on ``device`` (torch)."""

    def __init__(self, cfg: Config, rng: np.random.Generator, device,
                 haar_on_device: bool = False):
        """``haar_on_device``: draw the same Gaussian matrix on the host but
        take its QR on the device (for n_aux in the tens of thousands); U
        then differs from the host generator's by rounding only."""
        import torch
        if cfg.exact_orthonormal:
            raise ValueError("the exactly orthonormal (tiny) recipe is host-only")
        self.device = torch.device(device)
        if haar_on_device:
            A = cfg.n_aux
            z = torch.as_tensor(rng.standard_normal((A, A)), device=self.device)
            q, r = torch.linalg.qr(z)
            del z
            U = q * torch.sign(torch.diagonal(r))[None, :]
            del q, r
            self.UT = U.T.contiguous()
            del U
            host = _RowSource.__new__(_RowSource)
            host.cfg = cfg
            host.n_tot = cfg.n_occ + cfg.n_virt
            n_all = host.n_tot * (host.n_tot + 1) / 2.0
            host.c = cfg.c_scale
            tau = decay_length(cfg)
            s = np.exp(-np.arange(A) / tau)
            host.colscale = (host.c / math.sqrt(n_all)) * s * math.sqrt(3.0)
        else:
            host = _RowSource(cfg, rng)       # consumes the same draws as the host path
            self.UT = torch.as_tensor(host.U.T.copy(), device=self.device)
        self.cfg = cfg
        self.n_tot = host.n_tot
        self.key = _seed_key(cfg.seed)
        self.c = host.c
        self.colscale = torch.as_tensor(host.colscale, device=self.device)
        self.j = torch.arange(cfg.n_aux, dtype=torch.int64, device=self.device)

    def rows_from_index(self, idx, out, block: int = 4096):
        """out[r] = B row of pair index idx[r]; ``out`` is a [len(idx)][A]
        tensor (any float dtype, any row stride) on the device."""
        import torch
        idx = torch.as_tensor(idx, dtype=torch.int64, device=self.device)
        A = self.cfg.n_aux
        for b0 in range(0, idx.numel(), block):
            bi = idx[b0:b0 + block]
            ctr = bi[:, None] * A + self.j[None, :]
            g = (2.0 * splitmix64_uniform_torch(self.key, ctr) - 1.0) * self.colscale[None, :]
            del ctr
            out[b0:b0 + bi.numel()] = (g @ self.UT).to(out.dtype)
            del g
        return out

    def rows(self, p, q, dtype, block: int = 4096):
        import torch
        idx = _pair_index(np.asarray(p), np.asarray(q), self.n_tot)
        out = torch.empty((idx.size, self.cfg.n_aux), dtype=dtype, device=self.device)
        return self.rows_from_index(idx, out, block)


@dataclasses.dataclass
class DeviceProblem:
    cfg: Config
    eps: np.ndarray
    qp: np.ndarray
    R_oo: object          # torch [o][o][A] or None
    R_ov: object          # torch [o*v][A] or None (stream with ov_chunk)
    R_qp: object          # torch [Q][M][A]
    c_scale: float
    src: DeviceRowSource

    def oo_chunk(self, i0: int, i1: int, dtype, out=None):
        """Rows (i, j) of the occupied-occupied block for active occupied i in
        [i0, i1) and every active occupied j, as a [(i1-i0)*o][A] tensor."""
        import torch
        c = self.cfg
        occ = np.arange(c.n_fc, c.n_occ)
        vi, vj = np.meshgrid(occ[i0:i1], occ, indexing="ij")
        idx = _pair_index(vi.ravel(), vj.ravel(), self.src.n_tot)
        if out is None:
            out = torch.empty((idx.size, c.n_aux), dtype=dtype, device=self.src.device)
        return self.src.rows_from_index(idx, out)

    def ov_chunk(self, i0: int, i1: int, dtype, out=None):
        """Rows i*v + a of the occupied-virtual block for active occupied
        i in [i0, i1), as a [(i1-i0)*v][A] tensor (or into ``out``)."""
        import torch
        c = self.cfg
        occ = np.arange(c.n_fc + i0, c.n_fc + i1)
        virt = np.arange(c.n_occ, c.n_occ + c.n_virt)
        vi, va = np.meshgrid(occ, virt, indexing="ij")
        idx = _pair_index(vi.ravel(), va.ravel(), self.src.n_tot)
        if out is None:
            out = torch.empty((idx.size, c.n_aux), dtype=dtype, device=self.src.device)
        return self.src.rows_from_index(idx, out)


def make_problem_device(cfg: Config, device="cuda", dtype=None, with_ov: bool = True,
                        block: int = 4096, with_oo: bool = True,
                        haar_on_device: bool = False, with_qp: bool = True) -> DeviceProblem:
    """The problem of ``make_problem(cfg)`` with its tensors generated on
    ``device`` (default dtype float64).  ``with_ov=False`` / ``with_oo=False``
    leave the occupied-virtual / occupied-occupied blocks to be streamed with
    ``DeviceProblem.ov_chunk`` / ``oo_chunk``; ``with_qp=False`` skips the
    QP rows (R_qp is then None)."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    rng = np.random.default_rng(cfg.seed)
    eps = _energies(cfg, rng)
    src = DeviceRowSource(cfg, rng, device, haar_on_device)
    nf, no, nv = cfg.n_fc, cfg.n_occ, cfg.n_virt
    o, M, A = cfg.n_act_occ, cfg.n_act, cfg.n_aux
    act = np.arange(nf, no + nv)
    occ = np.arange(nf, no)
    virt = np.arange(no, no + nv)
    homo, lumo = no - 1, no
    qp = np.concatenate([np.arange(homo - cfg.n_qp_occ + 1, homo + 1),
                         np.arange(lumo, lumo + cfg.n_qp_virt)])
    if qp.min() < nf or qp.max() >= no + nv:
        raise ValueError("QP states must be active orbitals")
    R_oo = None
    if with_oo:
        pi, pj = np.meshgrid(occ, occ, indexing="ij")
        R_oo = src.rows(pi.ravel(), pj.ravel(), dtype, block).reshape(o, o, A)
    R_ov = None
    if with_ov:
        vi, va = np.meshgrid(occ, virt, indexing="ij")
        R_ov = src.rows(vi.ravel(), va.ravel(), dtype, block)
    R_qp = None
    if with_qp:
        qn, qm = np.meshgrid(qp, act, indexing="ij")
        R_qp = src.rows(qn.ravel(), qm.ravel(), dtype, block).reshape(qp.size, M, A)
    return DeviceProblem(cfg=cfg, eps=eps, qp=qp, R_oo=R_oo, R_ov=R_ov, R_qp=R_qp,
                         c_scale=src.c, src=src)
