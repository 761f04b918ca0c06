"""CPU-side checks of the library: it loads, exports every declared symbol,
and its host-only pieces behave (no GPU calls)."""
import ctypes
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


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a struct declared in include/fe.h, from gcc."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    body = "\n".join(f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields)
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"fe.h\"\nint main(void) {\n"
                   f'  printf("%zu\\n", sizeof({struct}));\n{body}\n  return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("cls,struct", [("KsOpts", "fe_ks_opts"), ("KsReport", "fe_ks_report")])
def test_binding_structs_match_header(cls, struct, tmp_path):
    """The ctypes mirrors of the option and report structs have the C layout."""
    from paper_1602_01421_amd import fe as F
    C = getattr(F, cls)
    names = [f[0] for f in C._fields_]
    size, offs = _c_layout(struct, names, tmp_path)
    assert ctypes.sizeof(C) == size
    assert [getattr(C, f).offset for f in names] == offs
