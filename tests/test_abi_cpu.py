"""CPU tests of the C ABI: the library loads and exports every declared
symbol, the host-side grids (rows a1 and a3) match the oracle, and argument
errors come back as status codes.  No device work is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from oracle import grids

gwlt = pytest.importorskip("paper_2307_04508_amd.gwlt")


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "gwlt.h")).read()
    return sorted(set(re.findall(r"^(?:gw_status|const char\*)\s+(gw_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gwlt.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(gwlt.EXPORTS)


@pytest.mark.parametrize("n", [1, 2, 7, 32, 33, 128])
def test_mgl_grid_matches_oracle(n):
    om, wt = gwlt.gw_freq_grid_mgl(n, 0.5)
    o2, w2 = grids.modified_gauss_legendre(n, 0.5)
    # nodes near t = 1 are amplified by 1 / (1 - t) under the mapping
    assert np.allclose(om, o2, rtol=1e-10, atol=1e-15)
    assert np.allclose(wt, w2, rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("k,lo,hi", [(8, 0.1225, 1e4), (10, 0.1225, 1e4), (12, 0.1225, 1e4),
                                     (6, 0.05, 300.0), (4, 2.0, 1e3)])
def test_minimax_grid_matches_oracle(k, lo, hi):
    x, w, e = gwlt.gw_lt_grid_minimax(k, lo, hi)
    xo, wo, eo = grids.lt_grid(k, lo, hi)
    assert np.allclose(x, xo, rtol=1e-9)
    assert np.allclose(w, wo, rtol=1e-9)
    assert abs(e - eo) < 1e-9 * eo


@pytest.mark.parametrize("k", [14, 16])
def test_minimax_grid_equioscillates_large_k(k):
    al, om, e = gwlt.gw_minimax_inverse(k, 8.16e4)
    pts, vals = grids._extrema(8.16e4, al, om, k, n_grid=40000)
    assert pts.size == 2 * k + 1
    assert np.all(np.sign(vals[1:]) == -np.sign(vals[:-1]))
    assert np.max(np.abs(vals)) - np.min(np.abs(vals)) < 1e-8 * e


def test_minimax_grid_matches_oracle_beyond_16_points():
    # k = 17 at R = 1e6: the level sits near 2e-7, where rounding in the error
    # curve (about 1e-15 near t = 1) limits how sharply equioscillation shows
    al, om, e = gwlt.gw_minimax_inverse(17, 1e6)
    ao, oo, eo = grids.minimax_inverse(17, 1e6)
    assert np.allclose(al, ao, rtol=1e-7)
    assert np.allclose(om, oo, rtol=1e-7)
    assert abs(e - abs(eo)) < 1e-7 * e


@pytest.mark.parametrize("k,R", [(18, 1e6), (20, 1e8)])
def test_minimax_grid_equioscillates_beyond_16_points(k, R):
    al, om, e = gwlt.gw_minimax_inverse(k, R)
    pts, vals = grids._extrema(R, al, om, k, n_grid=40000)
    assert pts.size == 2 * k + 1
    assert np.all(np.sign(vals[1:]) == -np.sign(vals[:-1]))
    assert np.max(np.abs(vals)) - np.min(np.abs(vals)) < 1e-14 + 1e-8 * e


@pytest.mark.parametrize("eps_lt", [1e-4, 1e-6, 1e-7])
def test_lt_grid_auto_takes_the_smallest_grid(eps_lt):
    lo, hi = 0.0904, 1.2e4
    n, x, w, e = gwlt.gw_lt_grid_auto(eps_lt, lo, hi)
    assert e <= eps_lt
    x2, w2, e2 = gwlt.gw_lt_grid_minimax(n, lo, hi)
    assert np.array_equal(x, x2) and np.array_equal(w, w2) and e == e2
    if n > 1:
        assert gwlt.gw_lt_grid_minimax(n - 1, lo, hi)[2] > eps_lt


def test_lt_grid_auto_reports_an_unreachable_target():
    with pytest.raises(gwlt.GwError) as ei:
        gwlt.gw_lt_grid_auto(1e-9, 0.0904, 1.2e4, max_lt=6)
    assert ei.value.status == gwlt.GW_ENOCONV


def test_prepare_matches_oracle(tiny_problem):
    p = tiny_problem
    c = p.cfg
    eF, lo, hi = gwlt.gw_prepare(c.n_occ, c.n_fc, c.n_virt, p.eps, 0.01)
    lo2, hi2 = grids.lt_bounds(p.eps, c.n_fc, c.n_occ, 0.01)
    assert eF == pytest.approx(0.5 * (p.eps[c.n_occ - 1] + p.eps[c.n_occ]), abs=1e-15)
    assert lo == pytest.approx(lo2, rel=1e-15) and hi == pytest.approx(hi2, rel=1e-15)


def test_argument_errors_are_status_codes():
    with pytest.raises(gwlt.GwError) as ei:
        gwlt.gw_freq_grid_mgl(0, 0.5)
    assert ei.value.status == gwlt.GW_EINVAL
    with pytest.raises(gwlt.GwError) as ei:
        gwlt.gw_lt_grid_minimax(21, 1.0, 10.0)
    assert ei.value.status == gwlt.GW_EINVAL
    with pytest.raises(gwlt.GwError):
        gwlt.gw_prepare(3, 3, 5, np.zeros(8), 0.0)        # n_fc == n_occ
    lib = gwlt._lib
    assert lib.gw_polarizability_lt(None, 0, 1, 1, None, None, 0, 1, None, None, None, 0, 0, 0,
                                    None) == gwlt.GW_EINVAL
    assert lib.gw_screen(None, 0, 1, 1, None, None, 1, None, None) == gwlt.GW_EINVAL
    assert lib.gw_sync(None) == gwlt.GW_EINVAL
    assert lib.gw_autotune_save(None, b"/nonexistent/t.txt") == gwlt.GW_EINVAL
    n = ctypes.c_int(7)
    assert lib.gw_autotune_load(None, b"/nonexistent/t.txt", ctypes.byref(n)) == gwlt.GW_EINVAL
    assert lib.gw_autotune_restrict(None, b"syrk", 2, 0) == gwlt.GW_EINVAL
    assert b"NULL" in lib.gw_last_error(None) or lib.gw_last_error(None) != b""


def test_binding_uses_a_single_hip_runtime():
    """The library is bound to torch's HIP runtime: after the binding is
    imported only one libamdhip64 is mapped in the process (a second one
    would own neither torch's tensors nor its streams)."""
    with open("/proc/self/maps") as f:
        libs = {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    assert len({os.path.realpath(p) for p in libs}) == 1, libs


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the binding next to no libgwlt.so refuses to import: there
    is no CPU fallback to route calls to."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "gwpkg"
    pkg.mkdir()
    (pkg / "__init__.py").write_text("")
    shutil.copy(os.path.join(ROOT, "paper_2307_04508_amd", "gwlt.py"), pkg / "gwlt.py")
    res = subprocess.run([sys.executable, "-c", "import gwpkg.gwlt"], cwd=tmp_path,
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "ImportError" in res.stderr and "libgwlt.so not found" in res.stderr


def test_product_code_never_reaches_the_oracle():
    """Nothing in the package (binding, build script, HIP and C++ sources)
    imports, loads or names the oracle package."""
    pkg = os.path.join(ROOT, "paper_2307_04508_amd")
    pat = re.compile(r"^\s*(?:from|import)\s+oracle\b|\boracle[./]", re.M)
    hits = []
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h", ".inc")):
                p = os.path.join(dirpath, f)
                if pat.search(open(p, encoding="utf-8", errors="replace").read()):
                    hits.append(p)
    assert hits == []
