"""Operator-level output (Eq. (11)): the number-basis matrix elements of the
evolved operator on the lowest levels of every mode, through the C ABI,
against the oracle's matrix, and the paper's operator error on the
three-level truncation against a half-step reference."""

import itertools

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgf():
    return library()


def block(cutoff, M, levels):
    """Rows and columns of M whose occupations are all below `levels`, in the
    order of the reconstruction (last mode fastest)."""
    idx = [np.ravel_multi_index(k, cutoff) for k in itertools.product(range(levels), repeat=len(cutoff))]
    return M[np.ix_(idx, idx)]


def eps_r(M, M_ref):
    """Relative operator error: Frobenius norm of the difference over that of
    the reference (the matrix taken as a vector of its elements)."""
    return np.linalg.norm(M - M_ref) / np.linalg.norm(M_ref)


def dense_operator(cutoff, seed):
    rng = np.random.default_rng(seed)
    dim = int(np.prod(cutoff))
    return rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
@pytest.mark.parametrize("cutoff,levels", [((3, 3, 3), 3), ((4, 5, 4), 3), ((6, 7), 2), ((5,), 5)])
def test_reconstruct_matches_oracle_matrix(hgf, cutoff, levels, precision, tol):
    announce(f"reconstruct {cutoff} levels={levels} {precision}")
    s = synth.random_system(cutoff, 301, scale=3.0, n_th=0.2)
    M0 = dense_operator(cutoff, 301)
    op = hgf.map_operator(hgf.define_system(s), dense=M0, precision=precision)
    T, dt = 0.05, 1e-3
    hgf.evolve(op, T, dt)
    got = hgf.reconstruct(op, levels)
    ref = block(cutoff, oracle.dense_from_sectors(cutoff, oracle.evolve(s, oracle.sectors_from_dense(cutoff, M0),
                                                                          T, dt)), levels)
    assert got.shape == ref.shape
    assert eps_r(got, ref) < tol
    # before any step: the input matrix itself
    op0 = hgf.map_operator(hgf.define_system(s), dense=M0, precision="fp64")
    assert eps_r(hgf.reconstruct(op0, levels), block(cutoff, M0, levels)) < 1e-15


def test_reconstruct_real_grid_and_sparse_sectors(hgf):
    """A real observable on the diagonal sector (held as a real grid) and an
    operator with few sectors: absent sectors read as zero."""
    cutoff = (4, 6, 5)
    announce("reconstruct real grid")
    s = synth.random_system(cutoff, 302, scale=2.0, n_th=0.3)
    fac = synth.parity_factors(cutoff)
    op = hgf.map_operator(hgf.define_system(s), factors=fac, precision="mixed")
    assert op.info()["real_functions"] == 1
    hgf.evolve(op, 0.1, 1e-3)
    got = hgf.reconstruct(op, 3)
    ref = block(cutoff, oracle.dense_from_sectors(cutoff, oracle.evolve(s, oracle.product_sectors(fac), 0.1, 1e-3)),
                3)
    assert eps_r(got, ref) < 1e-5
    assert np.all(got[~np.eye(got.shape[0], dtype=bool)] == 0)  # diagonal sector only


def test_reconstruct_split_layout(hgf):
    """Split layout (G = g0 (c_x c_y x^p y^q + R) per monomial, several
    functions per sector) equals the merged layout and the oracle."""
    cutoff = (3, 4)
    announce("reconstruct split")
    s = synth.random_system(cutoff, 303, scale=2.0)
    M0 = dense_operator(cutoff, 303)
    M0 = M0 + M0.conj().T
    k = np.array([np.unravel_index(i, cutoff) for i in range(12) for _ in range(12)])
    l = np.array([np.unravel_index(j, cutoff) for _ in range(12) for j in range(12)])
    S = hgf.define_system(s)
    sp = hgf.map_operator(S, sparse=(k, l, M0.reshape(-1)), layout="split")
    mg = hgf.map_operator(S, dense=M0)
    T, dt = 0.1, 2.5e-4
    for op in (sp, mg):
        hgf.evolve(op, T, dt)
    a, b = hgf.reconstruct(sp, 3), hgf.reconstruct(mg, 3)
    ref = block(cutoff, oracle.dense_from_sectors(cutoff, oracle.evolve(s, oracle.sectors_from_dense(cutoff, M0),
                                                                          T, dt)), 3)
    assert eps_r(b, ref) < 1e-10
    assert eps_r(a, ref) < 1e-9  # split and merged steps agree to RK4's truncation error


def test_three_level_error_against_half_step_reference(hgf):
    """The paper's accuracy measure: the operator on the three-level truncation
    against a reference run with half the step.  Off-diagonal sectors carry the
    Kerr phases, so the RK4 error is visible; it falls by 2^4 per halving, and
    the GPU's figure equals the oracle's."""
    cutoff = (5, 5)
    announce("three-level eps_r")
    s = synth.random_system(cutoff, 304, scale=20.0, n_th=0.1)
    fac = synth.quadrature_factors(cutoff)
    S = hgf.define_system(s)
    T = 0.02
    mats, refs = [], []
    for dt in (4e-4, 2e-4, 1e-4):
        op = hgf.map_operator(S, factors=fac, precision="fp64")
        hgf.evolve(op, T, dt)
        mats.append(hgf.reconstruct(op, 3))
        refs.append(block(cutoff, oracle.dense_from_sectors(cutoff, oracle.evolve(s, oracle.product_sectors(fac),
                                                                                    T, dt)), 3))
    e1, e2 = eps_r(mats[0], mats[1]), eps_r(mats[1], mats[2])
    assert 1e-12 < e2 < e1
    assert 12.0 < e1 / e2 < 20.0
    assert abs(e1 - eps_r(refs[0], refs[1])) < 1e-3 * e1


def test_reconstruct_arguments(hgf):
    cutoff = (3, 4)
    s = synth.random_system(cutoff, 305)
    op = hgf.map_operator(hgf.define_system(s), dense=np.eye(12, dtype=np.complex128))
    for bad in (0, 4):
        with pytest.raises(hgf.HgfError) as e:
            hgf.reconstruct(op, bad)
        assert e.value.status == "HGF_EINVAL"
    big = synth.random_system((6,) * 10, 306)
    opb = hgf.map_operator(hgf.define_system(big), factors=synth.parity_factors((6,) * 10), precision="mixed")
    with pytest.raises(hgf.HgfError) as e:
        hgf.reconstruct(opb, 3)  # 3^20 elements
    assert e.value.status == "HGF_EINVAL"
    assert np.allclose(hgf.reconstruct(opb, 1), 1.0)  # <0|parity|0> = 1
