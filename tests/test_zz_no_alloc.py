"""gw_sigma_diag_noalloc (the entry point for callers that cannot allocate):
through the C ABI it gives what gw_sigma_diag gives on the same inputs,
bitwise, and the oracle's W_nm and Sigma to the precision's tolerance, on
two calls in a row, the second with a smaller input; sizes beyond its fixed
scratch are rejected before anything is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from oracle import rpa, sigma  # noqa: E402


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


def _dev(a, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dt).contiguous()


def _case(seed, Q, Mo, N, F, Pd):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((Q, Mo, N)) / np.sqrt(N)
    X = rng.standard_normal((F, N + 7, N)) / np.sqrt(N)
    What = -np.einsum("fki,fkj->fij", X, X) / 4.0        # symmetric negative definite
    eps_m = np.sort(rng.uniform(-2.0, 3.0, Mo))
    om = np.sort(rng.uniform(0.05, 4.0, F))
    wom = rng.uniform(0.1, 1.0, F)
    omp = np.linspace(0.05, 2.0, Pd)
    return R, What, eps_m, 0.1, om, wom, omp


def _run(gw, ctx, fn, prec, case, acc_from=None):
    R, What, eps_m, eF, om, wom, omp = case
    Q, Mo, N = R.shape
    F = len(om)
    sig = torch.zeros((Q, len(omp), 2), dtype=torch.float64, device="cuda")
    if acc_from is not None:
        sig.copy_(acc_from)
    Wnm = torch.full((F, Q, Mo), np.nan, dtype=torch.float64, device="cuda")
    fn(ctx, prec, N, Q, Mo, eps_m, eF, _dev(R, prec), om, wom, _dev(What, prec), omp,
       int(acc_from is not None), sig, Wnm)
    gw.gw_sync(ctx)
    return sig.cpu().numpy(), Wnm.cpu().numpy()


def _oracle(case):
    R, What, eps_m, eF, om, wom, omp = case
    W = rpa.w_diag(R, What)
    return W, sigma.sigma_iw(W, eps_m, eF, om, wom, omp)


TOL = {"fp64": 1e-11, "fp32": 2e-6, "bf16x3": 1e-4}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_allocating_entry_point(gw, ctx, prec):
    big = _case(1, 3, 301, 333, 3, 8)      # ragged: 903 rows, 333 aux functions
    small = _case(2, 2, 70, 129, 2, 8)     # smaller second call
    for case in (big, small):
        s_ref, w_ref = _run(gw, ctx, gw.gw_sigma_diag, prec, case)
        s_na, w_na = _run(gw, ctx, gw.gw_sigma_diag_noalloc, prec, case)
        assert np.array_equal(s_na, s_ref)
        assert np.array_equal(w_na, w_ref)
        W_or, S_or = _oracle(case)
        tol = TOL[prec]
        # per row (n, m) across frequencies: relative to that row's largest |W_nm|
        err = np.abs(w_na - W_or).max(axis=0) / np.abs(W_or).max(axis=0)
        assert err.max() < tol, err.max()
        S = s_na[..., 0] + 1j * s_na[..., 1]
        assert np.max(np.abs(S - S_or)) < tol * 10 * np.max(np.abs(S_or))


def test_noalloc_accumulates_and_rejects_oversize(gw, ctx):
    case = _case(3, 2, 90, 150, 4, 6)
    R, What, eps_m, eF, om, wom, omp = case
    first = (R, What[:2], eps_m, eF, om[:2], wom[:2], omp)
    second = (R, What[2:], eps_m, eF, om[2:], wom[2:], omp)
    s1, _ = _run(gw, ctx, gw.gw_sigma_diag_noalloc, "fp64", first)
    s2, _ = _run(gw, ctx, gw.gw_sigma_diag_noalloc, "fp64", second,
                 acc_from=torch.as_tensor(s1).cuda())
    _, S_or = _oracle(case)
    assert np.max(np.abs(s2[..., 0] + 1j * s2[..., 1] - S_or)) < 1e-12 * np.max(np.abs(S_or))
    # 50 frequencies x 16 column slices x 12000 rows x 8 B = 77 MB of partials
    Q, Mo, N, F = 4, 3000, 1024, 50
    Rb = torch.zeros((Q, Mo, N), dtype=torch.float64, device="cuda")
    Wb = torch.zeros((F, N, N), dtype=torch.float64, device="cuda")
    sig = torch.zeros((Q, 4, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GwError) as ei:
        gw.gw_sigma_diag_noalloc(ctx, "fp64", N, Q, Mo, np.zeros(Mo), 0.0, Rb,
                                 np.linspace(0.1, 4.0, F), np.ones(F), Wb,
                                 np.linspace(0.1, 1.0, 4), 0, sig)
    assert ei.value.status == gw.GW_EINVAL
    assert "scratch" in str(ei.value)
