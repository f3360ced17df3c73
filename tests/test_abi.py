"""CPU checks of the C-ABI library: it loads, exports every declared entry point, and the
host-side argument checks answer without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1901_11095_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not B.is_built():
        B.build()
    from paper_1901_11095_amd import sal
    return sal.load()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "sal.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sal_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    from paper_1901_11095_amd import sal
    assert set(sal.EXPORTS) == set(names)


def test_default_params(lib):
    from paper_1901_11095_amd import sal
    p = sal.default_params(16)
    assert (p.L, p.d, p.sigma, list(p.rays)) == (16, 16, 4.0, [3, 12, 48])
    assert p.a == p.b == p.c == 1.0 / 3.0 and p.normalize == 1 and p.precision == sal.FP32


@pytest.mark.parametrize("fields,status", [
    ({"L": 1}, 1), ({"d": 1}, 1), ({"sigma": 0.0}, 1), ({"precision": 9}, 1), ({"L": 21}, 2),
    ({"L": 32}, 2), ({"L": 12, "precision": 2}, 2), ({"L": 5, "precision": 2}, 2), ({"L": 4, "precision": 1}, 2),
    ({"stride": 0}, 1), ({"stride": 3, "precision": 2}, 2), ({"stride": 4}, 1), ({"stride": 5}, 1),
    ({"L": 4, "stride": 2}, 1), ({"rays": 1 << 26}, 1),
])
def test_create_rejects(lib, fields, status):
    """Invalid parameters are rejected before any device call (a stride neither below L/2 nor
    equal to L); cube sides above 20 and 16-bit forms other than at L = 8 and 16 or with
    strides above 2 are unsupported."""
    from paper_1901_11095_amd import sal
    p = sal.default_params(8)
    for k, v in fields.items():
        if k == "rays":
            p.rays[0] = v
        else:
            setattr(p, k, v)
    h = ctypes.c_void_p()
    st = lib.sal_create(ctypes.byref(p), 0, ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert len(lib.sal_last_error(None)) > 0


def test_create_rejects_empty_rays(lib):
    from paper_1901_11095_amd import sal
    p = sal.default_params(8)
    p.rays[1] = 0
    h = ctypes.c_void_p()
    assert lib.sal_create(ctypes.byref(p), 0, ctypes.byref(h)) == sal.SAL_E_INVAL


def test_null_arguments(lib):
    from paper_1901_11095_amd import sal
    assert lib.sal_create(None, 0, None) == sal.SAL_E_INVAL
    assert lib.sal_saliency(None, None, 8, 8, 8, None, None, None, None, None, 0, None) == sal.SAL_E_INVAL
    lib.sal_destroy(None)


def test_product_path_never_touches_the_oracle():
    """The package and the C sources neither import, load nor name the oracle."""
    pkg = os.path.join(ROOT, "paper_1901_11095_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b|liboracle|sal_oracle", txt), f
