"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, and validates host-side arguments without touching a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hgf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def hgf():
    import paper_2203_05526_amd as pkg
    from paper_2203_05526_amd import hgf as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_2203_05526_amd import build
        build.build()
    pkg.load_library()
    return pkg


def test_exports_every_declared_symbol(hgf):
    from paper_2203_05526_amd import hgf as mod
    lib = ctypes.CDLL(mod.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(mod.EXPORTED) <= set(names)


def test_version_and_params(hgf):
    assert "gfx950" in hgf.version()
    s = synth.random_system((3, 4, 2), 0)
    S = hgf.define_system(s)
    assert S.num_params() == 3 + 3 + 3 * 3
    assert len(hgf.param_names(3)) == S.num_params()


@pytest.mark.parametrize("field,value", [
    ("gamma1", -0.1), ("gamma_phi", -1.0), ("n_th", -0.5), ("kerr", np.nan), ("detuning", np.inf),
])
def test_define_system_rejects_bad_parameters(hgf, field, value):
    s = synth.random_system((3, 2), 0)
    getattr(s, field)[0] = value
    with pytest.raises(hgf.HgfError) as e:
        hgf.define_system(s)
    assert e.value.status == "HGF_EINVAL"


def test_define_system_rejects_bad_shapes(hgf):
    s = synth.random_system((3, 2), 0)
    s.cross_kerr[0, 1] += 1.0  # not symmetric
    with pytest.raises(hgf.HgfError):
        hgf.define_system(s)
    with pytest.raises(hgf.HgfError):
        hgf.System((0,), [0.0], [0.0], [0.0], [0.1], [0.1], [0.0])
    with pytest.raises(hgf.HgfError):
        hgf.System((40,), [0.0], [0.0], [0.0], [0.1], [0.1], [0.0])
    with pytest.raises(hgf.HgfError):
        hgf.System(tuple([2] * 17), *[[0.0] * 17] * 2, [0.0] * 289, *[[0.1] * 17] * 3)


def test_null_arguments_are_rejected(hgf):
    from paper_2203_05526_amd import hgf as mod
    lib = mod.load_library()
    out = ctypes.c_void_p()
    assert lib.hgf_define_system(None, ctypes.byref(out)) == -1
    assert b"NULL" in lib.hgf_last_error()
    assert lib.hgf_evolve(None, 1.0, 0.1, 0, None) == -1
    assert lib.hgf_clear_error(None) == -1
    assert lib.hgf_num_params(None) == -1
    assert lib.hgf_get_tile_config(None, 0, None) == -1
    assert lib.hgf_set_tile_config(None, 0, None) == -1
    assert lib.hgf_autotune(None, 1, 1e-3, None, 0, None) == -1
    assert lib.hgf_reconstruct(None, 3, None, None) == -1
    assert b"NULL" in lib.hgf_last_error()
    assert lib.hgf_set_threshold(None, 1e-6) == -1
    assert lib.hgf_get_info(None, None) == -1
    two = (ctypes.c_double * 2)()
    assert lib.hgf_expectation_noalloc(None, None, two, None) == -1
    assert lib.hgf_expectation(None, None, two, None) == -1
    assert lib.hgf_evolve_batch(None, 1, None, None, None) == -1
    assert b"bad batch arguments" in lib.hgf_last_error()


def test_allocator_hook_arguments(hgf):
    """hgf_set_allocator takes both callbacks or neither (no device call is made)."""
    from paper_2203_05526_amd import hgf as mod
    lib = mod.load_library()
    alloc = mod._ALLOC_FN(lambda n, d, u: None)
    assert lib.hgf_set_allocator(alloc, mod._FREE_FN(), None) == -1
    assert b"both" in lib.hgf_last_error()
    assert lib.hgf_set_allocator(mod._ALLOC_FN(), mod._FREE_FN(), None) == 0


def test_dissipator_validation(hgf):
    """Secular dissipator options are validated when the system is defined."""
    args = ((3, 2), [0.0, 0.0], [0.0, 0.0], [0.0] * 4, [0.1, 0.1], [0.1, 0.1], [0.0, 0.0])
    hgf.System(*args, dissipator="secular")
    hgf.System(*args, dissipator="secular", n_th_levels=[0.1, 0.2, 0.0])
    with pytest.raises(hgf.HgfError):
        hgf.System(*args, dissipator="lindblad", n_th_levels=[0.1, 0.2, 0.0])
    with pytest.raises(hgf.HgfError):
        hgf.System(*args, dissipator="secular", n_th_levels=[0.1, -0.2, 0.0])
    with pytest.raises(hgf.HgfError):
        hgf.System(*args, dissipator="secular", n_th_levels=[0.1, 0.2])


def test_network_validation(hgf):
    """Drive and exchange are validated when the system is defined (no GPU)."""
    args = ((3, 2), [0.0, 0.0], [0.0, 0.0], [0.0] * 4, [0.1, 0.1], [0.1, 0.1], [0.0, 0.0])
    assert hgf.System(*args, drive=[1.0 + 0.5j, 0.0], exchange=[[0.0, 2.0], [2.0, 0.0]]).network
    with pytest.raises(hgf.HgfError):
        hgf.System(*args, exchange=[[0.0, 2.0], [1.0, 0.0]])  # not symmetric
    with pytest.raises(hgf.HgfError):
        hgf.System(*args, drive=[np.nan, 0.0])
    with pytest.raises(hgf.HgfError):
        hgf.System(*args, drive=[1.0])  # wrong length
    n = 9  # the full (k, l) grid has 2N axes: at most 8 modes
    with pytest.raises(hgf.HgfError):
        hgf.System((2,) * n, [0.0] * n, [0.0] * n, [0.0] * (n * n), [0.1] * n, [0.0] * n, [0.0] * n,
                   drive=[1.0] + [0.0] * (n - 1))


def test_over_large_operators_are_rejected_before_device_work(hgf):
    """Sector grids whose point count would overflow (16 modes at cutoff 16:
    16^16 = 2^64 points) or exceed the library's 2^32-point cap are refused
    with HGF_EINVAL by a host-side check that runs before any device call."""
    n = 16
    S = hgf.System((16,) * n, [0.0] * n, [0.0] * n, [0.0] * (n * n), [0.1] * n, [0.0] * n, [0.0] * n)
    with pytest.raises(hgf.HgfError) as e:
        hgf.map_operator(S, factors=[np.eye(16)] * n)
    assert e.value.status == "HGF_EINVAL" and "2^32" in str(e.value)
    # sparse input: one term in the diagonal sector (16^16 points)
    ks = np.zeros((1, n), dtype=np.int32)
    with pytest.raises(hgf.HgfError) as e:
        hgf.map_operator(S, sparse=(ks, ks, np.array([1.0])))
    assert e.value.status == "HGF_EINVAL" and "2^32" in str(e.value)
    # gradient requests go through the same check
    with pytest.raises(hgf.HgfError) as e:
        hgf.grad(S, synth.fock_state([0] * n), 0.1, 0.01, factors=[np.eye(16)] * n)
    assert e.value.status == "HGF_EINVAL"
    # just over the cap in total over sectors: 8 modes at cutoff 16 with
    # bidiagonal factors (sum over the two diagonals 16 + 15 = 31 per mode,
    # 31^8 = 8.5e11 points in total, 16^8 = 2^32 in the diagonal sector alone)
    n = 8
    S = hgf.System((16,) * n, [0.0] * n, [0.0] * n, [0.0] * (n * n), [0.1] * n, [0.0] * n, [0.0] * n)
    fac = np.eye(16) + np.eye(16, k=1)
    with pytest.raises(hgf.HgfError) as e:
        hgf.map_operator(S, factors=[fac] * n)
    assert e.value.status == "HGF_EINVAL"
    # the full (k, l) grid of a network: 8 modes at cutoff 32 (2^80 points)
    S = hgf.System((32,) * n, [0.0] * n, [0.0] * n, [0.0] * (n * n), [0.1] * n, [0.0] * n, [0.0] * n,
                   drive=[1.0] + [0.0] * (n - 1))
    with pytest.raises(hgf.HgfError) as e:
        hgf.map_operator(S, factors=[np.eye(32)] * n)
    assert e.value.status == "HGF_EINVAL" and "2^28" in str(e.value)
