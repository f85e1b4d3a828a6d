"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2509_01099_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "islbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(islbm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(pkg.EXPORTS)


def test_library_exports_every_mlp_symbol():
    """The warm-start network kernels declared in include/islbm_mlp.h."""
    text = open(os.path.join(ROOT, "include", "islbm_mlp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    syms = sorted(set(re.findall(r"\b(islbm_[a-z0-9_]+)\s*\(", text)))
    assert len(syms) >= 8
    lib = pkg.load()
    for s in syms:
        assert hasattr(lib, s), s


def test_options_struct_matches_header():
    text = open(os.path.join(ROOT, "include", "islbm.h")).read()
    body = text[text.index("typedef struct {\n  double u_f;"):text.index("} islbm_options;")]
    names = re.findall(r"\b([a-z_]+)(?:\[4\])?;", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    flat = []
    for line in re.sub(r"/\*.*?\*/", "", body, flags=re.S).split(";"):
        flat += re.findall(r"([a-z_]+)(?:\[\d\])?\s*$", line.strip().split(" ", 1)[-1]) or []
    fields = [f for f, _ in pkg.islbm_options._fields_]
    for f in fields:
        assert f in body, f
    assert names  # the struct body parsed


@pytest.mark.parametrize("kind,a", [("uniform", 0), ("erf", 1.5), ("cosine", 0), ("tanh", 1.5)])
def test_mesh_spacing_matches_oracle_mesh(kind, a):
    n = 77
    sp = pkg.islbm_mesh_spacing(kind, n, a)
    x = oracle.mesh(kind, n, a)
    assert np.allclose(sp, np.diff(x), rtol=0, atol=1e-15)
    assert sp[0] == sp[-1]


def test_query_bytes():
    fb, gb = pkg.islbm_query_bytes(2, [100, 50], pkg.ISLBM_FP32)
    assert fb == 9 * 128 * 50 * 4 and gb == 5 * 128 * 50 * 4
    fb, gb = pkg.islbm_query_bytes(3, [256, 256, 256], pkg.ISLBM_FP16DEV)
    assert fb == 19 * 256 ** 3 * 2 and gb == 7 * 256 ** 3 * 2
    fb, gb = pkg.islbm_query_bytes(2, [100, 50], pkg.ISLBM_FP32SR)   # FP32 storage
    assert fb == 9 * 128 * 50 * 4 and gb == 5 * 128 * 50 * 4
    with pytest.raises(pkg.IslbmError):
        pkg.islbm_query_bytes(2, [2, 50], pkg.ISLBM_FP32)
    with pytest.raises(pkg.IslbmError):
        pkg.islbm_query_bytes(2, [100, 50], 5)                     # unknown storage


def _create(n, sp, Ra=1e6, Pr=0.71, lattice=2, opt=None):
    try:
        pkg.islbm_create(lattice, n, sp, Ra, Pr, opt)
    except pkg.IslbmError as e:
        return e.code
    return 0


def test_create_validates_before_the_device():
    sp = pkg.islbm_mesh_spacing("erf", 20)
    assert _create([20, 20], [sp, sp], Ra=-1) == pkg.ISLBM_EINVAL
    assert _create([20, 20], [sp, sp], Pr=0) == pkg.ISLBM_EINVAL
    assert _create([20, 20], [sp, sp], lattice=4) == pkg.ISLBM_EINVAL
    assert _create([2, 20], [sp[:3], sp], lattice=2) == pkg.ISLBM_EINVAL
    bad = sp.copy()
    bad[5] = 0.5 * bad[0]                     # spacing below the lattice unit
    assert _create([20, 20], [bad, sp]) == pkg.ISLBM_EMESH
    ghost = sp.copy()
    ghost[-1] *= 1.5                          # ghost spacing differs from Delta
    assert _create([20, 20], [ghost, sp]) == pkg.ISLBM_EMESH
    other = pkg.islbm_mesh_spacing("erf", 30)  # different lattice unit on y
    assert _create([20, 30], [sp, other]) == pkg.ISLBM_EMESH
    # a_T > 1 is refused before any device work
    assert _create([20, 20], [sp, sp], Ra=1.0) == pkg.ISLBM_EPARAM


def test_create_without_device_reports_edevice():
    sp = pkg.islbm_mesh_spacing("erf", 20)
    code = _create([20, 20], [sp, sp])
    import torch

    if not torch.cuda.is_available():
        assert code == pkg.ISLBM_EDEVICE
        assert "device" in pkg.load().islbm_last_error(None).decode()


def test_strerror_and_null_handling():
    lib = pkg.load()
    assert lib.islbm_strerror(0) == b"ok"
    assert lib.islbm_strerror(-2).startswith(b"mesh")
    assert lib.islbm_strerror(7) == b"unknown status"
    lib.islbm_destroy(None)                  # no-op
    assert lib.islbm_step(None, 1) == pkg.ISLBM_EINVAL
    assert lib.islbm_plan_steps(None, 20) == pkg.ISLBM_EINVAL
    assert lib.islbm_time_steps_split(None, 2, None, None, None) == pkg.ISLBM_EINVAL
    assert lib.islbm_copy_bytes(None, None, 16, None) == pkg.ISLBM_EINVAL
    assert lib.islbm_nu_re(None, None) == pkg.ISLBM_EINVAL
    assert lib.islbm_steady_change(None, None, None, None) == pkg.ISLBM_EINVAL
    assert lib.islbm_time(None) == -1
