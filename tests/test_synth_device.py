"""The device twin of the generator (run here with torch on the CPU) draws
the same numbers and builds the same rows as the host generator."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gwsynth import get_config, make_problem  # noqa: E402
from gwsynth.device import make_problem_device, splitmix64_uniform_torch  # noqa: E402
from gwsynth.problem import splitmix64_uniform  # noqa: E402


def test_splitmix64_twin_is_bit_identical():
    ctr = np.concatenate([np.arange(0, 5000), np.array([2**40 + 7, 2**62 - 1, 123456789012])])
    for key in (0, 1, 0xFFFFFFFFFFFFFFFF, 0x632BE59BD9B4E019):
        a = splitmix64_uniform(key, ctr)
        b = splitmix64_uniform_torch(key, torch.as_tensor(ctr, dtype=torch.int64)).numpy()
        assert np.array_equal(a, b)
        assert a.min() >= 0.0 and a.max() < 1.0


def test_device_problem_matches_host_problem():
    cfg = get_config("medium").with_(n_occ=12, n_fc=4, n_virt=30, n_aux=64, naf_target=32,
                                     n_qp_occ=2, n_qp_virt=2)
    h = make_problem(cfg)
    d = make_problem_device(cfg, device="cpu", block=100)
    assert np.array_equal(h.eps, d.eps) and np.array_equal(h.qp, d.qp)
    for name in ("R_oo", "R_ov", "R_qp"):
        a, b = getattr(h, name), getattr(d, name).numpy()
        assert a.shape == b.shape
        assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a)), name
    o, v = cfg.n_act_occ, cfg.n_virt
    ch = d.ov_chunk(3, 6, torch.float32).numpy()
    assert np.max(np.abs(ch - h.R_ov[3 * v:6 * v])) <= 1e-6 * np.max(np.abs(h.R_ov))
    assert o * v == h.R_ov.shape[0]
    oc = d.oo_chunk(2, 5, torch.float64).numpy()
    assert np.max(np.abs(oc - h.R_oo[2:5].reshape(-1, cfg.n_aux))) <= 1e-14 * np.max(np.abs(a))


def test_haar_on_device_matches_host_qr():
    cfg = get_config("medium").with_(n_occ=12, n_fc=4, n_virt=30, n_aux=64, naf_target=32,
                                     n_qp_occ=2, n_qp_virt=2)
    h = make_problem(cfg)
    d = make_problem_device(cfg, device="cpu", haar_on_device=True)
    assert np.array_equal(h.eps, d.eps)
    a, b = h.R_ov, d.R_ov.numpy()
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_host_stream_matches_host_problem():
    """The host stream (occupied chunks, for workloads whose whole tensor does
    not fit in memory) draws the same rows as make_problem, bitwise; the
    scale c enters every row linearly."""
    from gwsynth.problem import ProblemStream
    cfg = get_config("medium").with_(n_occ=12, n_fc=4, n_virt=30, n_aux=64, naf_target=32,
                                     n_qp_occ=2, n_qp_virt=2)
    h = make_problem(cfg)
    s = ProblemStream(cfg)
    o, v, A = cfg.n_act_occ, cfg.n_virt, cfg.n_aux
    assert np.array_equal(h.eps, s.eps) and np.array_equal(h.qp, s.qp)
    assert np.array_equal(h.R_qp, s.R_qp)
    assert np.array_equal(h.R_ov[3 * v:7 * v], s.ov_chunk(3, 7))
    assert np.array_equal(h.R_oo[2:5], s.oo_chunk(2, 5))
    h2 = make_problem(cfg.with_(c_scale=2.5))
    assert np.max(np.abs(h2.R_ov - 2.5 * h.R_ov)) <= 1e-14 * np.max(np.abs(h2.R_ov))
    d2 = make_problem_device(cfg.with_(c_scale=2.5), device="cpu")
    assert np.max(np.abs(d2.R_ov.numpy() - h2.R_ov)) <= 1e-14 * np.max(np.abs(h2.R_ov))
