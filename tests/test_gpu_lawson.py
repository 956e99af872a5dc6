"""Integrating-factor (Lawson) RK4 on the GPU (scheme HGF_LAWSON_RK4) against
the oracle's integrating-factor RK4 in the number basis, plus its defining
properties: exact without jumps, and stable where classical RK4 is not."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, gpu_number_grids, library, max_rel_err, oracle_number_grids, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def hgf():
    return library()


def dense_operator(cutoff, seed):
    rng = np.random.default_rng(seed)
    dim = int(np.prod(cutoff))
    return rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))


def stiff_system(cutoff, seed):
    """Kerr phases of hundreds of rad/us against jump rates of order 1/us."""
    s = synth.random_system(cutoff, seed, scale=1.0, n_th=0.3)
    s.kerr = -300.0 + 50.0 * np.arange(len(cutoff))
    return s


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
def test_lawson_matches_oracle(hgf, precision, tol, dissipator):
    cutoff = (3, 4, 3)
    announce(f"lawson {dissipator} {precision}")
    s = synth.random_system(cutoff, 401, scale=3.0, n_th=0.2)
    if dissipator == "secular":
        s.dissipator = "secular"
        s.n_th_levels = np.random.default_rng(401).uniform(0.0, 0.5, size=sum(c - 1 for c in cutoff))
    M = dense_operator(cutoff, 401)
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
    assert op.info()["n_functions"] == 5 * 7 * 5  # many launches per step: graph chunks below 64 steps
    T, dt = 0.06, 1e-3
    hgf.evolve(op, T, dt, scheme="lawson")
    ref = oracle_number_grids(cutoff, oracle.evolve_lawson(s, oracle.sectors_from_dense(cutoff, M), T, dt))
    assert max_rel_err(gpu_number_grids(op, cutoff), ref) < tol


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_lawson_real_grid(hgf, precision, tol):
    """A real observable on the diagonal sector, held as a real grid."""
    cutoff = (5, 6, 4)
    announce(f"lawson real grid {precision}")
    s = synth.random_system(cutoff, 402, scale=3.0, n_th=0.3)
    fac = synth.parity_factors(cutoff)
    op = hgf.map_operator(hgf.define_system(s), factors=fac, precision=precision)
    assert op.info()["real_functions"] == 1
    T, dt = 0.1, 1e-3
    hgf.evolve(op, T, dt, scheme="lawson")
    ref = oracle_number_grids(cutoff, oracle.evolve_lawson(s, oracle.product_sectors(fac), T, dt))
    assert max_rel_err(gpu_number_grids(op, cutoff), ref) < tol


def test_lawson_exact_without_jumps(hgf):
    """gamma1 = 0: each coefficient is multiplied by exp(D T), whatever the
    step (here |D| dt ~ 10, far outside classical RK4's stability region)."""
    cutoff = (4, 3)
    announce("lawson without jumps")
    s = synth.random_system(cutoff, 403, scale=40.0)
    s.gamma1 = np.zeros(2)
    M = dense_operator(cutoff, 403)
    ops = oracle.sectors_from_dense(cutoff, M)
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision="fp64")
    with pytest.raises(hgf.HgfError) as e:
        hgf.evolve(op, 0.1, 0.05)
    assert e.value.status == "HGF_EUNSTABLE"
    hgf.evolve(op, 0.1, 0.05, scheme="lawson")
    ref = oracle_number_grids(cutoff, oracle.evolve_lawson(s, ops, 0.1, 0.05))
    assert max_rel_err(gpu_number_grids(op, cutoff), ref) < 1e-12
    # and that equals exp(D T) A(0) for the diagonal coefficient D of each element
    E = np.array([sum(s.detuning[j] * k[j] + 0.5 * s.kerr[j] * k[j] * (k[j] - 1) for j in range(2))
                  + s.cross_kerr[0, 1] * k[0] * k[1] for k in np.ndindex(*cutoff)])
    occ = np.array(list(np.ndindex(*cutoff)))
    D = 1j * (E[:, None] - E[None, :])
    for j in range(2):
        D -= s.gamma_phi[j] * (occ[:, None, j] - occ[None, :, j]) ** 2
    exact = oracle.sectors_from_dense(cutoff, np.exp(D * 0.1) * M)
    assert max_rel_err(gpu_number_grids(op, cutoff), oracle_number_grids(cutoff, exact)) < 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_lawson_where_rk4_is_unstable(hgf, precision, tol):
    """Stiff Kerr phases in off-diagonal sectors (the product of quadratures
    spans 2^N of them): classical RK4 refuses the step, the integrating-factor
    scheme takes it, matches the oracle's scheme, and stays within 1e-5 of a
    converged solution (oracle RK4 at a 100 x smaller step, itself within
    about 3e-7; classical RK4 needs a 40 x smaller step than this one to come
    within 1e-5)."""
    cutoff = (6, 5, 6)
    announce(f"lawson stiff {precision}")
    s = stiff_system(cutoff, 404)
    fac = synth.quadrature_factors(cutoff)
    S = hgf.define_system(s)
    op = hgf.map_operator(S, factors=fac, precision=precision)
    T, dt = 0.02, 1e-3
    with pytest.raises(hgf.HgfError) as e:
        hgf.evolve(op, T, dt)
    assert e.value.status == "HGF_EUNSTABLE"
    hgf.evolve(op, T, dt, scheme="lawson")
    got = gpu_number_grids(op, cutoff)
    assert max_rel_err(got, oracle_number_grids(cutoff, oracle.evolve_lawson(s, oracle.product_sectors(fac), T,
                                                                              dt))) < tol
    fine_ops = oracle.evolve(s, oracle.product_sectors(fac), T, dt / 100)
    assert max_rel_err(got, oracle_number_grids(cutoff, fine_ops)) < 1e-5
    st = synth.coherent_state([0.5, 0.3 + 0.2j, 0.4j])
    assert rel(hgf.expectation(op, st), oracle.expectation(cutoff, fine_ops, st)) < 1e-5


def test_lawson_step_sizes_compose(hgf):
    """Two calls with different steps (the per-step factor tables are rebuilt)
    equal the oracle's two-step sequence; RK4 and Lawson calls mix."""
    cutoff = (4, 5)
    announce("lawson composition")
    s = synth.random_system(cutoff, 405, scale=3.0, n_th=0.2)
    M = dense_operator(cutoff, 405)
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision="fp64")
    hgf.evolve(op, 0.02, 1e-3, scheme="lawson")
    hgf.evolve(op, 0.02, 5e-4, scheme="lawson")
    hgf.evolve(op, 0.01, 1e-3)
    a = oracle.evolve_lawson(s, oracle.sectors_from_dense(cutoff, M), 0.02, 1e-3)
    a = oracle.evolve_lawson(s, a, 0.02, 5e-4)
    a = oracle.evolve(s, a, 0.01, 1e-3)
    assert max_rel_err(gpu_number_grids(op, cutoff), oracle_number_grids(cutoff, a)) < FP64_TOL
    assert op.info()["steps_done"] == 20 + 40 + 10


def test_lawson_errors(hgf):
    cutoff = (3, 4)
    s = synth.random_system(cutoff, 406)
    S = hgf.define_system(s)
    one = np.array([[1, 2]])
    sp = hgf.map_operator(S, sparse=(one, one, np.array([1.0 + 0j])), layout="split")
    with pytest.raises(hgf.HgfError) as e:
        hgf.evolve(sp, 0.01, 1e-3, scheme="lawson")
    assert e.value.status == "HGF_EUNSUPPORTED"
    from paper_2203_05526_amd import hgf as mod
    op = hgf.map_operator(S, dense=np.eye(12, dtype=np.complex128))
    assert mod._lib.hgf_evolve(op.handle, 0.01, 1e-3, 2, None) == -6  # HGF_EUNSUPPORTED
    # jump rates too large for the step: unstable for either scheme
    s.gamma1 = np.array([5e3, 5e3])
    op2 = hgf.map_operator(hgf.define_system(s), dense=np.eye(12, dtype=np.complex128))
    with pytest.raises(hgf.HgfError) as e:
        hgf.evolve(op2, 0.01, 1e-3, scheme="lawson")
    assert e.value.status == "HGF_EUNSTABLE"
