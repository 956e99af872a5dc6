"""The secular dissipator (Eq. (15): one lowering and one raising channel per
transition n <-> n+1 with per-transition bath occupations) on the GPU path,
against the FP64 oracle: every kernel form (resident, tiled, grouped,
generic, split layout) and the gradient."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, gpu_grids, gpu_number_grids, library, max_rel_err, oracle_number_grids, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def hgf():
    return library()


def secular_system(cutoff, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    s = synth.random_system(cutoff, seed, scale=scale, n_th=0.2)
    s.dissipator = "secular"
    s.n_th_levels = rng.uniform(0.0, 0.6, size=sum(c - 1 for c in cutoff))
    return s


def dense_operator(cutoff, seed):
    rng = np.random.default_rng(seed)
    dim = int(np.prod(cutoff))
    return rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("cutoff,seed,kernel", [((4, 5), 201, "resident"), ((3, 4, 3, 4, 3), 202, "tiled"),
                                                ((3, 4, 3, 4, 3), 203, "generic")])
def test_secular_matches_oracle(hgf, cutoff, seed, kernel, precision, tol):
    announce(f"secular {cutoff} {kernel} {precision}")
    s = secular_system(cutoff, seed)
    M = dense_operator(cutoff, seed)
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
    nf = op.info()["n_functions"]
    if kernel == "generic":
        for i in range(nf):
            if op.tile_config(i)["resident"] == 0:
                op.set_tile_config(i, 0)
    kinds = {(op.tile_config(i)["resident"], op.tile_config(i)["nfast"] > 0) for i in range(nf)}
    if kernel == "resident":
        assert kinds == {(1, True)}
    elif kernel == "tiled":
        assert (0, True) in kinds
    else:
        assert (0, False) in kinds
    T, dt = 0.05, 1e-3
    hgf.evolve(op, T, dt)
    ref = oracle_number_grids(cutoff, oracle.evolve(s, oracle.sectors_from_dense(cutoff, M), T, dt))
    assert max_rel_err(gpu_number_grids(op, cutoff), ref) < tol


def test_secular_batch_and_split_layout(hgf):
    """Grouped launches (a batch of two secular systems of one shape) and the
    split layout (point sources with per-level down-jump coefficients)."""
    cutoff = (3, 4, 3, 4, 3)
    announce("secular batch + split")
    systems = [secular_system(cutoff, 210 + i) for i in range(2)]
    M = dense_operator(cutoff, 210)
    M[np.abs(M) < 1.5] = 0.0
    ops = [hgf.map_operator(hgf.define_system(s), dense=M, precision="fp64") for s in systems]
    T, dt = 0.04, 1e-3
    hgf.evolve_batch(ops, [T, T], [dt, dt])
    for op, s in zip(ops, systems):
        ref = oracle_number_grids(cutoff, oracle.evolve(s, oracle.sectors_from_dense(cutoff, M), T, dt))
        assert max_rel_err(gpu_number_grids(op, cutoff), ref) < FP64_TOL
    # split layout: one monomial, compared through the expectation value.  The
    # separable part takes its own scalar RK4, so split and merged steps agree
    # to RK4's truncation error only: a finer step keeps that below 1e-9.
    s = systems[0]
    dt = 2.5e-4
    k, l = np.array([[1, 2, 0, 1, 2]]), np.array([[1, 2, 0, 1, 2]])
    sp = hgf.map_operator(hgf.define_system(s), sparse=(k, l, np.array([1.0 + 0j])), layout="split",
                          precision="fp64")
    hgf.evolve(sp, T, dt)
    st = synth.coherent_state([0.6, 0.4 + 0.2j, 0.8, 0.3, 0.5j])
    ref_ops = oracle.evolve(s, oracle.sparse_sectors(cutoff, k, l, np.array([1.0 + 0j])), T, dt)
    assert rel(hgf.expectation(sp, st), oracle.expectation(cutoff, ref_ops, st)) < 1e-9


def test_secular_gradient_matches_oracle_sensitivities(hgf):
    cutoff = (3, 4, 3)
    announce("secular gradient")
    s = secular_system(cutoff, 220, scale=2.0)
    M = dense_operator(cutoff, 220)
    M = M + M.conj().T
    S = hgf.define_system(s)
    st = synth.coherent_state([0.5, 0.3 + 0.4j, 0.7])
    T, dt = 0.1, 1e-3
    ops = oracle.sectors_from_dense(cutoff, M)
    fin, sens = oracle.evolve_sens(s, ops, T, dt)
    ref_val = oracle.expectation(cutoff, fin, st)
    ref_grad = np.array([oracle.expectation(cutoff, sp, st) for sp in sens])
    val, g = hgf.grad(S, st, T, dt, dense=M, checkpoint_every=7)
    assert rel(val, ref_val) < FP64_TOL
    assert np.max(np.abs(g - ref_grad)) / np.max(np.abs(ref_grad)) < FP64_TOL


def test_secular_equals_lindblad_on_populations(hgf):
    """One bath occupation for every transition: on the diagonal sector the
    two dissipators give the same functions (to rounding)."""
    cutoff = (5, 6, 4)
    announce("secular vs lindblad on populations")
    s = synth.random_system(cutoff, 230, scale=3.0, n_th=0.3)
    sec = s.copy()
    sec.dissipator = "secular"
    rng = np.random.default_rng(230)
    fac = [np.diag(rng.uniform(0.5, 1.5, size=c)).astype(np.complex128) for c in cutoff]
    a = hgf.map_operator(hgf.define_system(s), factors=fac, precision="fp64")
    b = hgf.map_operator(hgf.define_system(sec), factors=fac, precision="fp64")
    hgf.evolve(a, 0.05, 1e-3)
    hgf.evolve(b, 0.05, 1e-3)
    assert max_rel_err(gpu_grids(b), gpu_grids(a)) < 1e-13
