"""CPU-side checks of the library: it loads, exports every declared symbol,
and its host-only pieces behave (no GPU calls)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(fe):
    names = declared_functions()
    assert len(names) >= 13
    L = fe.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(fe.EXPORTED) == set(names)


def test_version(fe):
    assert fe.version() >= 300


def test_dense_symeig_closed_form_path(fe):
    """Path graph P_n: eigenvalues 2 cos(pi k / (n + 1))."""
    n = 40
    a = np.zeros((n, n))
    i = np.arange(n - 1)
    a[i, i + 1] = a[i + 1, i] = 1.0
    w, z = fe.fe_dense_symeig(a)
    want = 2 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1))
    assert np.allclose(np.sort(w), np.sort(want), atol=1e-13)
    assert np.allclose(z.T @ z, np.eye(n), atol=1e-13)
    assert np.allclose(a @ z, z * w, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 128])
def test_dense_symeig_random(fe, n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n))
    a = a + a.T
    w, z = fe.fe_dense_symeig(a)
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(a), atol=1e-12 * max(1, np.abs(a).max()) * n)
    assert np.allclose(a @ z, z * w, atol=1e-11 * n)


def test_dense_symeig_repeated_and_zero(fe):
    a = np.diag([3.0, 3.0, 0.0, -3.0, 0.0])
    w, z = fe.fe_dense_symeig(a)
    assert np.allclose(np.sort(w), [-3, 0, 0, 3, 3])
    assert np.allclose(a @ z, z * w)


def test_csr_build_validates_before_touching_the_device(fe):
    with pytest.raises(fe.FeError) as e:
        fe.fe_csr_build(4, np.array([0, 9], np.int32), np.array([1, 2], np.int32))
    assert e.value.status == fe.FE_EINVAL
    with pytest.raises(fe.FeError) as e:
        fe.fe_csr_build(0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert e.value.status == fe.FE_EINVAL
    with pytest.raises(fe.FeError) as e:
        fe.fe_csr_from_csr(3, np.array([0, 2, 1, 1]), np.array([1, 2], np.int32))
    assert e.value.status == fe.FE_EINVAL
    with pytest.raises(fe.FeError) as e:  # row not strictly increasing
        fe.fe_csr_from_csr(3, np.array([0, 2, 2, 2]), np.array([2, 1], np.int32))
    assert e.value.status == fe.FE_EINVAL
