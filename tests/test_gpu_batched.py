"""GPU parity of the batched calls, the graph capture and the batched G0W0
driver.

Each batched twin runs several uneven problems (ragged sizes, an empty
chunk, padded rows) in one launch per kernel and is compared, job by job,
with the oracle on the same inputs.  Captured graphs are replayed several
times with eager work in between; every replay must reproduce the eager
result exactly.  The batched G0W0 of the 64-molecule workload is checked
against the oracle (same Laplace grids) on its smallest molecules and, for
all 64, the FP32 graph against the per-molecule FP64 path.
"""
import sys

import numpy as np
import pytest

from bounds import assert_quadform_close
from conftest import HARTREE_MEV

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from oracle import grids, pade, rpa, sigma  # noqa: E402
from oracle.g0w0 import g0w0_problem  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_04508_amd import gwlt
    return gwlt


@pytest.fixture(scope="module")
def ctx(gw):
    c = gw.Context(0)
    yield c
    c.close()


def dev(a, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dt).contiguous()


def rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _lt_case(seed, o, v, N, L):
    rng = np.random.default_rng(seed)
    eps_i = -np.sort(rng.uniform(0.3, 20.0, max(o, 1)))[::-1][:o]
    eps_a = np.sort(rng.uniform(0.05, 5.0, v))
    R = rng.standard_normal((o * v, N)) / np.sqrt(N)
    lo = (eps_a[0] - (eps_i[-1] if o else -0.3)) ** 2
    x, w, _ = grids.lt_grid(L, lo, 1e4)
    return eps_i, eps_a, R, x, w


# (o, v, N, row stride or 0)
CHI_SHAPES = [(8, 40, 150, 0), (13, 389, 300, 0), (3, 7, 129, 0), (0, 11, 64, 0),
              (5, 50, 256, 384), (2, 600, 97, 0)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("bf16x3", 1e-4)])
def test_polarizability_batched_matches_oracle(gw, ctx, prec, tol):
    _say(f"polarizability batched {prec}")
    L = 4
    jobs, refs, Ms = [], [], []
    for s, (o, v, N, ld) in enumerate(CHI_SHAPES):
        eps_i, eps_a, R, x, w = _lt_case(100 + s, o, v, N, L)
        d = (eps_a[None, :] - eps_i[:, None]).ravel()
        refs.append(rpa.m_lt(R, d, x, w) if o else np.zeros((L, N, N)))
        M = torch.full((L, N, N), float("nan"), dtype=torch.float64, device="cuda")
        Ms.append(M)
        dt = torch.float64 if prec == "fp64" else torch.float32
        if ld:
            Rd = torch.full((o * v, ld), 1e30, dtype=dt, device="cuda")
            Rd[:, :N] = dev(R, prec)
            Rd = Rd[:, :N]
        else:
            Rd = dev(R, prec) if o else None
        jobs.append(dict(n_naf=N, n_i=o, n_virt=v, x_lt=x, w_lt=w, eps_i=eps_i, eps_a=eps_a,
                         R_chunk=Rd, M=M))
    gw.gw_polarizability_lt_batched(ctx, prec, L, jobs, 0, 1)
    gw.gw_sync(ctx)
    for s, (M, ref) in enumerate(zip(Ms, refs)):
        Mh = M.cpu().numpy()
        assert np.all(np.isfinite(Mh)), s
        assert np.array_equal(Mh, np.transpose(Mh, (0, 2, 1)))
        for m in range(L):
            if CHI_SHAPES[s][0] == 0:
                assert np.all(Mh[m] == 0.0)
            else:
                assert rel_fro(Mh[m], ref[m]) < tol, (s, m, rel_fro(Mh[m], ref[m]))


def _spd_m(seed, L, N):
    rng = np.random.default_rng(seed)
    M = np.empty((L, N, N))
    for m in range(L):
        X = rng.standard_normal((N + 20, N)) / np.sqrt(N) * 0.3 / (m + 1)
        M[m] = X.T @ X
    return M


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 2e-7)])
def test_screen_batched_matches_oracle(gw, ctx, prec, tol):
    _say(f"screen batched {prec}")
    L = 3
    shapes = [(150, 5), (333, 3), (64, 2), (1, 2), (200, 4), (65, 1)]
    jobs, refs, Ws = [], [], []
    for s, (N, F) in enumerate(shapes):
        M = _spd_m(30 + s, L, N)
        x = np.array([0.05, 0.5, 3.0]) * (1.0 + 0.1 * s)
        om, _ = grids.modified_gauss_legendre(F, 0.5 + 0.1 * s)
        refs.append(rpa.screen(rpa.pi_lt(M, x, om)))
        W = torch.zeros((F, N, N), dtype=torch.float64 if prec == "fp64" else torch.float32,
                        device="cuda")
        Ws.append(W)
        jobs.append(dict(n_naf=N, x_lt=x, M=dev(M, "fp64"), omega=om, W_hat=W))
    gw.gw_screen_batched(ctx, prec, L, jobs)
    gw.gw_sync(ctx)
    for s, (W, ref) in enumerate(zip(Ws, refs)):
        Wh = W.double().cpu().numpy()
        for j in range(len(ref)):
            # W^ = A^-1 - 1 cancels digits where Pi is small (high frequencies):
            # its error is relative to W^ plus a floor relative to A^-1 itself
            d = np.linalg.norm(Wh[j] - ref[j])
            bound = tol * np.linalg.norm(ref[j]) + 1e-13 * np.linalg.norm(ref[j] + np.eye(len(ref[j])))
            assert d <= bound, (s, j, d, bound)
            assert np.array_equal(Wh[j], Wh[j].T)


@pytest.mark.parametrize("width", [128, 256, 64])
def test_screen_batched_each_width_matches_oracle(gw, ctx, width):
    """The sweep at each outer width, pinned through gw_autotune_restrict, on
    matrices whose 128-tile counts differ (6, 3, 2, 1), so their sweeps end
    at different steps: at width 128 the update of each step is split over
    two streams (the next panel's row and column, then the rest) and the
    panel and pivot buffers alternate by step."""
    _say(f"screen batched width {width}")
    L = 3
    shapes = [(700, 3), (300, 2), (129, 2), (1, 1), (640, 2)]
    jobs, refs, Ws = [], [], []
    for s, (N, F) in enumerate(shapes):
        M = _spd_m(60 + s, L, N)
        x = np.array([0.05, 0.5, 3.0]) * (1.0 + 0.1 * s)
        om, _ = grids.modified_gauss_legendre(F, 0.5 + 0.1 * s)
        refs.append(rpa.screen(rpa.pi_lt(M, x, om)))
        W = torch.zeros((F, N, N), dtype=torch.float64, device="cuda")
        Ws.append(W)
        jobs.append(dict(n_naf=N, x_lt=x, M=dev(M, "fp64"), omega=om, W_hat=W))
    gw.gw_autotune(ctx, 2)
    gw.gw_autotune(ctx, 0)
    gw.gw_autotune_restrict(ctx, "screen", 1024, width)
    try:
        gw.gw_screen_batched(ctx, "fp64", L, jobs)
        gw.gw_sync(ctx)
    finally:
        gw.gw_autotune_restrict(ctx, "screen", 0)
        gw.gw_autotune(ctx, 1)
    for s, (W, ref) in enumerate(zip(Ws, refs)):
        Wh = W.cpu().numpy()
        for j in range(len(ref)):
            d = np.linalg.norm(Wh[j] - ref[j])
            bound = 1e-11 * np.linalg.norm(ref[j]) + 1e-13 * np.linalg.norm(ref[j] + np.eye(len(ref[j])))
            assert d <= bound, (s, j, d, bound)
            assert np.array_equal(Wh[j], Wh[j].T)


def test_screen_batched_reports_non_spd(gw, ctx):
    good = _spd_m(5, 1, 40)
    bad = -np.eye(70)[None] * 10.0
    Wg = torch.zeros((2, 40, 40), dtype=torch.float64, device="cuda")
    Wb = torch.zeros((1, 70, 70), dtype=torch.float64, device="cuda")
    jobs = [dict(n_naf=40, x_lt=[0.1], M=dev(good, "fp64"), omega=[0.2, 0.3], W_hat=Wg),
            dict(n_naf=70, x_lt=[0.1], M=dev(bad, "fp64"), omega=[0.2], W_hat=Wb)]
    gw.gw_screen_batched(ctx, "fp64", 1, jobs)
    with pytest.raises(gw.GwError) as ei:
        gw.gw_sync(ctx)
    assert ei.value.status == gw.GW_ENOTSPD
    gw.gw_sync(ctx)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6), ("bf16x3", 1e-4)])
def test_sigma_batched_matches_oracle(gw, ctx, prec, tol):
    _say(f"sigma batched {prec}")
    shapes = [(3, 70, 333, 2), (2, 45, 128, 3), (1, 200, 257, 1), (2, 9, 64, 2)]
    jobs, refs, outs, inputs = [], [], [], []
    for s, (Q, Mo, N, F) in enumerate(shapes):
        rng = np.random.default_rng(200 + s)
        R = rng.standard_normal((Q, Mo, N)) / np.sqrt(N)
        X = rng.standard_normal((F, N, N)) / np.sqrt(N)
        What = -np.einsum("fij,fkj->fik", X, X) / 4.0
        eps_m = np.sort(rng.uniform(-2, 2, Mo))
        om, wom = grids.modified_gauss_legendre(F, 0.5)
        op, _ = grids.modified_gauss_legendre(5, 0.5)
        eF = 0.05 * s
        W_ref = rpa.w_diag(R, What)
        S_ref = sigma.sigma_iw(W_ref, eps_m, eF, om, wom, op)
        refs.append((W_ref, S_ref))
        inputs.append((R, What))
        sig = torch.zeros((Q, len(op), 2), dtype=torch.float64, device="cuda")
        Wnm = torch.zeros((F, Q, Mo), dtype=torch.float64, device="cuda")
        outs.append((sig, Wnm))
        jobs.append(dict(n_naf=N, n_qp=Q, n_mo=Mo, eps_mo=eps_m, eps_F=eF, R_qp=dev(R, prec),
                         omega=om, w_omega=wom, W_hat=dev(What, prec), omega_pade=op,
                         sigma_iw=sig, W_nm=Wnm))
    gw.gw_sigma_diag_batched(ctx, prec, jobs, 0)
    gw.gw_sync(ctx)
    for s, ((W_ref, S_ref), (sig, Wnm)) in enumerate(zip(refs, outs)):
        R, What = inputs[s]
        assert_quadform_close(Wnm.cpu().numpy(), W_ref, R.reshape(-1, R.shape[-1]), What, prec,
                              rounded_inputs=prec != "fp64")
        sh = sig.cpu().numpy()
        S = sh[..., 0] + 1j * sh[..., 1]
        assert np.max(np.abs(S - S_ref)) < 10 * tol * np.max(np.abs(S_ref)), s


def test_qp_batched_matches_oracle(gw, ctx, tiny_problem, tiny_sos):
    p, r = tiny_problem, tiny_sos
    c = p.cfg
    sig = torch.as_tensor(np.stack([r.sigma.real, r.sigma.imag], -1)).cuda().contiguous()
    jobs = []
    statics = [np.array([0.003, -0.002]), None, np.array([0.0, 0.01])]
    for s in statics:
        jobs.append(dict(eps_n=p.eps[p.qp], static_n=s, eps_F=r.eps_f,
                         omega_pade=r.omega_pade, sigma_iw=sig))
    outs = gw.gw_qp_solve_batched(ctx, jobs, c.eta, 1e-10, 200)
    zn = 1j * r.omega_pade
    for s, (E, Z, S) in zip(statics, outs):
        for q, n in enumerate(p.qp):
            a = pade.thiele_coefficients(zn, r.sigma[q])
            cn = 0.0 if s is None else s[q]
            Eo, Zo, ok = pade.qp_solve(p.eps[n], cn, r.eps_f, zn, a, c.eta, tol=1e-10,
                                       max_iter=200)
            assert S[q] == 0 and ok
            assert abs(E[q] - Eo) < 1e-9 and abs(Z[q] - Zo) < 1e-6


def test_graph_capture_replays(gw, ctx):
    """Capture polarizability + screening + self-energy, replay three times
    with eager work in between: every replay equals the eager result; a
    replay after the input changed in place equals the eager result on the
    new input."""
    _say("graph capture")
    o, v, N, L, F, Q, Mo = 6, 90, 140, 3, 4, 2, 40
    eps_i, eps_a, R, x, w = _lt_case(7, o, v, N, L)
    rng = np.random.default_rng(8)
    Rq = rng.standard_normal((Q, Mo, N)) / np.sqrt(N)
    eps_m = np.sort(rng.uniform(-2, 2, Mo))
    om, wom = grids.modified_gauss_legendre(F, 0.5)
    op, _ = grids.modified_gauss_legendre(6, 0.5)
    Rd = dev(R * 0.3, "fp32")
    Rqd = dev(Rq, "fp32")
    M = torch.zeros((L, N, N), dtype=torch.float64, device="cuda")
    W = torch.zeros((F, N, N), dtype=torch.float32, device="cuda")
    sig = torch.zeros((Q, len(op), 2), dtype=torch.float64, device="cuda")

    def seq():
        gw.gw_polarizability_lt(ctx, "fp32", N, x, w, o, v, eps_i, eps_a, Rd, 0, 1, M)
        gw.gw_screen(ctx, "fp32", N, x, M, om, W)
        gw.gw_sigma_diag(ctx, "fp32", N, Q, Mo, eps_m, 0.01, Rqd, om, wom, W, op, 0, sig)

    seq()                                      # eager: sizes the workspace
    gw.gw_sync(ctx)
    ref = (M.clone(), W.clone(), sig.clone())
    gw.gw_graph_begin(ctx)
    seq()
    g = gw.gw_graph_end(ctx)
    try:
        other = torch.zeros((L, 64, 64), dtype=torch.float64, device="cuda")
        for rep in range(3):
            M.zero_(); W.zero_(); sig.zero_()
            gw.gw_graph_launch(ctx, g)
            gw.gw_sync(ctx)
            assert torch.equal(M, ref[0]) and torch.equal(W, ref[1]) and torch.equal(sig, ref[2]), rep
            # eager work on other data between replays
            e2, a2, R2, x2, w2 = _lt_case(50 + rep, 3, 20, 64, L)
            gw.gw_polarizability_lt(ctx, "fp32", 64, x2, w2, 3, 20, e2, a2, dev(R2, "fp32"), 0, 1,
                                    other)
            gw.gw_sync(ctx)
        # the graph reads its device inputs in place
        Rd.mul_(0.5)
        gw.gw_graph_launch(ctx, g)
        gw.gw_sync(ctx)
        got = (M.clone(), W.clone(), sig.clone())
        seq()
        gw.gw_sync(ctx)
        assert torch.equal(got[0], M) and torch.equal(got[1], W) and torch.equal(got[2], sig)
        assert not torch.equal(got[0], ref[0])
        # synchronising calls are refused while capturing
        gw.gw_graph_begin(ctx)
        with pytest.raises(gw.GwError) as ei:
            gw.gw_qp_solve(ctx, [-0.5], None, 0.0, op, sig, 1e-3)
        assert ei.value.status == gw.GW_EUNSUPPORTED
        g2 = gw.gw_graph_end(ctx)
        g2.close()
    finally:
        g.close()


# ------------------------------------------------------------------ batched G0W0

@pytest.fixture(scope="module")
def batch64():
    from gwsynth import batched_configs
    from gwsynth.device import make_problem_device
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _say("generating the 64-molecule batch on the device")
    probs = [make_problem_device(c, device="cuda", dtype=torch.float64) for c in batched_configs()]
    torch.cuda.synchronize()
    yield probs
    del probs
    torch.cuda.empty_cache()


def _mols(probs, prec):
    out = []
    for p in probs:
        cast = (lambda t: t) if prec == "fp64" else (lambda t: t.to(torch.float32).contiguous())
        out.append(dict(cfg=p.cfg, eps=p.eps, qp=p.qp, R_oo=cast(p.R_oo), R_ov=cast(p.R_ov),
                        R_qp=cast(p.R_qp)))
    return out


def test_g0w0_batched_vs_per_molecule(gw, ctx, batch64):
    probs = batch64
    params = gw.batch_params_for(probs[0].cfg)
    _say("per-molecule fp64")
    E64 = []
    for p in probs:
        E, Z, S, sig, st = gw.gw_g0w0(ctx, "fp64", gw.params_for(p.cfg), p.eps, p.qp, None,
                                      p.R_oo, p.R_ov, p.R_qp)
        assert np.all(S == 0)
        E64.append((E, st.n_naf))
    _say("batched fp64 (eager)")
    res, stats = gw.gw_g0w0_batched(ctx, "fp64", params, _mols(probs, "fp64"), graph=False)
    for (E, Z, S, _, n), (Er, nr) in zip(res, E64):
        assert n == nr and np.all(S == 0)
        assert np.max(np.abs(E - Er)) * HARTREE_MEV < 1e-6
    mols32 = _mols(probs, "fp32")
    for prec, tol in (("fp32", 1.0), ("bf16x3", 1.0)):
        for rep in range(3):
            res, stats = gw.gw_g0w0_batched(ctx, prec, params, mols32, graph=True)
            _say(f"batched {prec} graph rep {rep}: total {stats.t_total_ms:.1f} ms "
                 f"(NAF {stats.t_naf_ms:.1f}), replayed {stats.graph_replayed}")
            assert stats.graph_replayed == (1 if rep > 0 else 0)
            d = max(np.max(np.abs(E - Er)) for (E, _, _, _, _), (Er, _) in zip(res, E64))
            _say(f"  max |E - E_fp64| = {d * HARTREE_MEV:.2e} meV")
            assert d * HARTREE_MEV < tol
            assert all(np.all(S == 0) for (_, _, S, _, _) in res)
            if rep == 0:
                first = [E.copy() for (E, _, _, _, _) in res]
            else:
                assert all(np.array_equal(E, F0) for (E, _, _, _, _), F0 in zip(res, first))


def test_g0w0_batched_smallest_against_oracle(gw, ctx, batch64):
    """The three smallest molecules of the batch through the batched driver
    against the oracle taking the same Laplace grids (the precision part)."""
    from gwsynth import make_problem
    probs = sorted(batch64, key=lambda p: p.cfg.n_occ)[:3]
    params = gw.batch_params_for(probs[0].cfg)
    res, _ = gw.gw_g0w0_batched(ctx, "fp32", params, _mols(probs, "fp32"), graph=False)
    for p, (E, Z, S, _, n) in zip(probs, res):
        hp = make_problem(p.cfg)
        c = hp.cfg
        om0 = grids.modified_gauss_legendre(c.n_freq, c.x0)[0][0]
        lo, hi = grids.lt_bounds(hp.eps, c.n_fc, c.n_occ, om0)
        x, w, _ = grids.lt_grid(c.n_lt, lo, hi)
        ref = g0w0_problem(hp, lt=(x, w))
        assert n == ref.n_naf
        err = np.abs(E - ref.eps_qp) * HARTREE_MEV
        _say(f"  n_occ={c.n_occ}: precision part {err.max():.2e} meV")
        assert np.all(err < 1.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_naf_batched_matches_single(gw, ctx, prec):
    """Batched metric + bucketed padded eigensolves against the oracle's
    metric and eigenvalues, and the kept subspaces against the oracle's
    projector, for uneven jobs."""
    from oracle import naf as onaf
    _say(f"naf batched {prec}")
    rng = np.random.default_rng(71)
    shapes = [(150, 300, 600), (97, 40, 250), (130, 0, 700), (64, 100, 64)]
    jobs, refs = [], []
    for A, n_oo, n_ov in shapes:
        s = np.exp(-np.arange(A) / (A / 6.0))
        Roo = rng.standard_normal((n_oo, A)) * s / np.sqrt(A)
        Rov = rng.standard_normal((n_ov, A)) * s / np.sqrt(A)
        dt = np.float64 if prec == "fp64" else np.float32
        K_ref = onaf.naf_metric(Roo.astype(dt).astype(np.float64), Rov.astype(dt).astype(np.float64))
        lam = np.sort(np.linalg.eigvalsh(K_ref))[::-1]
        keep = A // 2
        cut = 0.5 * (lam[keep - 1] + lam[keep])
        _, U_ref = onaf.naf_basis(K_ref, cut)
        refs.append((K_ref, lam, U_ref, cut))
        jobs.append(dict(n_aux=A, R_oo=dev(Roo, prec) if n_oo else None, R_ov=dev(Rov, prec),
                         K=torch.zeros((A, A), dtype=torch.float64, device="cuda"),
                         U=torch.zeros((A, A), dtype=torch.float64, device="cuda"),
                         eps_naf=cut, max_keep=0))
    out = gw.gw_naf_compress_batched(ctx, prec, jobs)
    for (n, ev), (K_ref, lam, U_ref, cut), j in zip(out, refs, jobs):
        A = j["n_aux"]
        assert n == A // 2
        dK = 1e-13 if prec == "fp64" else 1e-6
        assert np.max(np.abs(ev - lam)) <= dK * 10 * lam[0]
        Uh = j["U"].cpu().numpy()[:n].T
        assert np.allclose(Uh.T @ Uh, np.eye(n), atol=1e-12)
        P, P_ref = Uh @ Uh.T, U_ref @ U_ref.T
        gap = lam[n - 1] - lam[n]
        assert np.linalg.norm(P - P_ref) <= np.sqrt(2) * (dK * 10 * lam[0] * A) / (0.5 * gap)
    # transform: batched equals single-call output bitwise (same kernel)
    Rin = [dev(rng.standard_normal((333, j["n_aux"])), prec) for j in jobs]
    outs_b = [torch.zeros((333, 128 * ((n + 127) // 128)), dtype=r.dtype, device="cuda")
              for (n, _), r in zip(out, Rin)]
    gw.gw_naf_apply_batched(ctx, prec, [dict(n_aux=j["n_aux"], n_naf=n, U=j["U"], R_in=r, R_out=o)
                                        for j, (n, _), r, o in zip(jobs, out, Rin, outs_b)])
    for j, (n, _), r, o in zip(jobs, out, Rin, outs_b):
        o1 = torch.zeros_like(o)
        gw.gw_naf_apply(ctx, prec, j["n_aux"], n, j["U"], r, o1)
        gw.gw_sync(ctx)
        assert torch.equal(o, o1)


def test_reserve_then_capture_without_eager_run(gw):
    """On a fresh context, gw_reserve sizes the workspace so the calls can be
    captured without ever running eagerly; the replay matches an eager run
    on a second context."""
    o, v, N, L, F, Q, Mo = 5, 70, 130, 3, 3, 2, 30
    eps_i, eps_a, R, x, w = _lt_case(9, o, v, N, L)
    rng = np.random.default_rng(10)
    Rq = rng.standard_normal((Q, Mo, N)) / np.sqrt(N)
    eps_m = np.sort(rng.uniform(-2, 2, Mo))
    om, wom = grids.modified_gauss_legendre(F, 0.5)
    op, _ = grids.modified_gauss_legendre(5, 0.5)
    Rd, Rqd = dev(R * 0.3, "fp32"), dev(Rq, "fp32")

    def run(c):
        M = torch.zeros((L, N, N), dtype=torch.float64, device="cuda")
        W = torch.zeros((F, N, N), dtype=torch.float32, device="cuda")
        sig = torch.zeros((Q, len(op), 2), dtype=torch.float64, device="cuda")

        def seq():
            gw.gw_polarizability_lt(c, "fp32", N, x, w, o, v, eps_i, eps_a, Rd, 0, 1, M)
            gw.gw_screen(c, "fp32", N, x, M, om, W)
            gw.gw_sigma_diag(c, "fp32", N, Q, Mo, eps_m, 0.01, Rqd, om, wom, W, op, 0, sig)
        return M, W, sig, seq

    c1 = gw.Context(0)
    try:
        gw.gw_reserve(c1, "fp32", n_naf=N, n_occ_act=o, n_virt=v, n_mo=Mo, n_qp=Q, n_lt=L,
                      n_w=F, n_pade=len(op))
        M1, W1, s1, seq1 = run(c1)
        gw.gw_graph_begin(c1)
        seq1()
        g = gw.gw_graph_end(c1)
        gw.gw_graph_launch(c1, g)
        gw.gw_sync(c1)
        c2 = gw.Context(0)
        M2, W2, s2, seq2 = run(c2)
        seq2()
        gw.gw_sync(c2)
        c2.close()
        assert torch.equal(M1, M2) and torch.equal(W1, W2) and torch.equal(s1, s2)
        g.close()
    finally:
        c1.close()
