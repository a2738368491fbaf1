"""The C-ABI library loads on the CPU host and exports every entry point
declared in include/mls2mc.h; argument validation that happens before any
device work returns EINVAL with a message (no GPU needed for these)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mls2mc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mls2mc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_1709_09763_amd as P
    return P.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["mls2mc_kl_field", "mls2mc_forward", "mls2mc_loglik", "mls2mc_next_step",
              "mls2mc_resample", "mls2mc_pcn_step", "mls2mc_create", "mls2mc_destroy",
              "mls2mc_run", "mls2mc_gather", "mls2mc_forward_field", "mls2mc_philox_fill"]:
        assert n in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_size_queries(L):
    import paper_1709_09763_amd as P
    assert P.mls2mc_n_elem(4) == 512
    assert P.mls2mc_n_unknowns(9) == 511 ** 2
    assert "gfx950" in P.mls2mc_version()


@pytest.mark.parametrize("field,val,msg", [
    ("l_min", 0, "l_min"), ("l_max", 11, "l_max"), ("K", 0, "K"), ("sigma2", -1.0, "sigma2"),
    ("corr_len", 0.0, "corr_len"), ("m", 0, "m"), ("sigma_n", 0.0, "sigma_n"),
    ("precision", 7, "precision"), ("cov", 5, "covariance"), ("kl_quad", 16, "kl_quad"),
    ("bc", 3, "boundary-value"),
])
def test_create_rejects_bad_problems(L, field, val, msg):
    import paper_1709_09763_amd as P
    pr = P.Problem(3, 6, 10, 1.0, 0.3, 3, 0.01, 0, 0.0, 0)
    setattr(pr, field, val)
    h = C.c_void_p()
    rc = L.mls2mc_create(C.byref(pr), C.byref(h))
    assert rc == 1
    assert h.value is None
    assert msg in P.mls2mc_last_error()


def test_flow_cell_is_fp64_only(L):
    import paper_1709_09763_amd as P
    pr = P.Problem(3, 6, 10, 1.0, 0.3, 3, 0.01, P.MIXED, 0.0, 0, 0, 0, P.BC_FLOW_CELL)
    h = C.c_void_p()
    assert L.mls2mc_create(C.byref(pr), C.byref(h)) == 1
    assert "FP64 only" in P.mls2mc_last_error()


@pytest.mark.parametrize("quad,K,msg", [(15, 10, "kl_quad"), (2, 1, "kl_quad"), (130, 10, "kl_quad"),
                                        (4, 17, "K exceeds")])
def test_create_rejects_bad_matern_grids(L, quad, K, msg):
    import paper_1709_09763_amd as P
    pr = P.Problem(3, 6, K, 1.0, 0.3, 3, 0.01, 0, 0.0, 0, P.COV_MATERN32, quad)
    h = C.c_void_p()
    assert L.mls2mc_create(C.byref(pr), C.byref(h)) == 1
    assert h.value is None
    assert msg in P.mls2mc_last_error()


def test_null_context_is_rejected(L):
    assert L.mls2mc_forward(None, 4, 1, None, None, None, None, None) == 1
    assert L.mls2mc_resample(None, 4, None, None, None, None) == 1
    assert L.mls2mc_destroy(None) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1709_09763_amd._lib as lib
    monkeypatch.setattr(lib, "_lib", None)
    monkeypatch.setattr(lib, "library_path", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        lib.lib()
