"""The driven, exchange-coupled network (Eq. (16) in the drive frame) on the
GPU: one full (k, l) grid per operator, against the oracle's full-matrix RK4,
read through hgf_reconstruct and hgf_expectation."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, library

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def hgf():
    return library()


def network_system(cutoff, seed, dissipator="lindblad", scale=2.0):
    rng = np.random.default_rng(seed)
    s = synth.random_system(cutoff, seed, scale=scale, n_th=0.2)
    n = len(cutoff)
    s.drive = (rng.normal(size=n) + 1j * rng.normal(size=n)) * 3.0
    J = np.zeros((n, n))
    for i in range(n - 1):
        J[i, i + 1] = J[i + 1, i] = rng.uniform(1.0, 4.0)
    s.exchange = J
    if dissipator == "secular":
        s.dissipator = "secular"
        s.n_th_levels = rng.uniform(0.0, 0.5, size=sum(c - 1 for c in cutoff))
    return s


def rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def state_vector(cutoff, alphas):
    v = np.ones(1, dtype=np.complex128)
    for a, c in zip(alphas, oracle.state_amplitudes(cutoff, synth.coherent_state(alphas))):
        v = np.kron(v, c)
    return v


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("cutoff,seed,dissipator", [((4, 4), 501, "lindblad"), ((3, 3, 3), 502, "secular"),
                                                    ((6,), 503, "lindblad"), ((3, 4), 504, "lindblad")])
def test_network_matches_oracle(hgf, cutoff, seed, dissipator, precision, tol):
    announce(f"network {cutoff} {dissipator} {precision}")
    s = network_system(cutoff, seed, dissipator)
    dim = int(np.prod(cutoff))
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
    assert op.info()["n_functions"] == 1 and op.info()["total_points"] == dim * dim
    T, dt = 0.05, 2.5e-4
    hgf.evolve(op, T, dt)
    ref = oracle.evolve_full(s, M, T, dt)
    L = min(cutoff)
    got = hgf.reconstruct(op, L)
    idx = [np.ravel_multi_index(k, cutoff) for k in np.ndindex(*(L,) * len(cutoff))]
    assert rel_fro(got, ref[np.ix_(idx, idx)]) < tol
    alphas = [0.5 + 0.2j * j for j in range(len(cutoff))]
    c = state_vector(cutoff, alphas)
    want = np.conj(c) @ ref @ c
    J = hgf.expectation(op, synth.coherent_state(alphas))
    assert abs(J - want) / abs(want) < (10 * tol if precision == "mixed" else tol)


def test_network_maximum_modes(hgf):
    """Eight modes (16 grid axes, the limit) of two levels each, both
    dissipators' tables through the coordinate packing, against the oracle."""
    cutoff = (2,) * 8
    announce("network 8 modes")
    for dissipator in ("lindblad", "secular"):
        s = network_system(cutoff, 509, dissipator, scale=1.0)
        rng = np.random.default_rng(509)
        M = rng.normal(size=(256, 256)) + 1j * rng.normal(size=(256, 256))
        op = hgf.map_operator(hgf.define_system(s), dense=M, precision="fp64")
        assert op.info()["total_points"] == 2 ** 16
        T, dt = 0.01, 5e-4
        hgf.evolve(op, T, dt)
        ref = oracle.evolve_full(s, M, T, dt)
        assert rel_fro(hgf.reconstruct(op, 2), ref) < FP64_TOL


def test_qubit_chain_driven_on_one_end(hgf):
    """Table I's structure: a chain of anharmonic modes (three levels each),
    the first driven on resonance, nearest-neighbour exchange, weak decay; the
    observable prod_j (a_j + a_j^+) (the Hermitian form of the test operator
    prod_j a_j)."""
    cutoff = (3, 3, 3, 3)
    announce("qubit chain")
    n = len(cutoff)
    two_pi = 2 * np.pi
    s = synth.System(cutoff, np.zeros(n), np.full(n, -2 * two_pi * 250.0), np.zeros((n, n)),
                     np.full(n, 0.02), np.zeros(n), np.zeros(n))
    s.drive = np.array([two_pi * 125.0] + [0.0] * (n - 1), dtype=np.complex128)
    J = np.zeros((n, n))
    for i in range(n - 1):
        J[i, i + 1] = J[i + 1, i] = two_pi * 10.0
    s.exchange = J
    fac = synth.quadrature_factors(cutoff)
    op = hgf.map_operator(hgf.define_system(s), factors=fac, precision="fp64")
    T, dt = 2e-3, 1e-5
    hgf.evolve(op, T, dt)
    M0 = np.ones((1, 1), dtype=np.complex128)
    for f in fac:
        M0 = np.kron(M0, f)
    ref = oracle.evolve_full(s, M0, T, dt)
    assert rel_fro(hgf.reconstruct(op, 3), ref) < FP64_TOL
    alphas = [0.3, 0.2j, 0.1, 0.0]
    c = state_vector(cutoff, alphas)
    want = np.conj(c) @ ref @ c
    assert abs(hgf.expectation(op, synth.coherent_state(alphas)) - want) < 1e-10 * max(1.0, abs(want))


def test_network_in_a_batch(hgf):
    """A network operator (one full grid on the untiled kernel) and sector
    operators evolved in one batch equal their separate evolves."""
    announce("network batch")
    a = network_system((3, 4), 505)
    b = synth.random_system((4, 5, 3), 506, scale=2.0)
    Ma = np.random.default_rng(505).normal(size=(12, 12)) + 0j
    fb = synth.parity_factors((4, 5, 3))
    ops1 = [hgf.map_operator(hgf.define_system(a), dense=Ma, precision="mixed"),
            hgf.map_operator(hgf.define_system(b), factors=fb, precision="mixed")]
    ops2 = [hgf.map_operator(hgf.define_system(a), dense=Ma, precision="mixed"),
            hgf.map_operator(hgf.define_system(b), factors=fb, precision="mixed")]
    hgf.evolve_batch(ops1, [0.02, 0.03], [1e-3, 1e-3])
    hgf.evolve(ops2[0], 0.02, 1e-3)
    hgf.evolve(ops2[1], 0.03, 1e-3)
    for x, y in zip(ops1, ops2):
        assert np.array_equal(hgf.reconstruct(x, 3), hgf.reconstruct(y, 3))


def test_network_unsupported_paths(hgf):
    announce("network errors")
    s = network_system((3, 3), 507)
    S = hgf.define_system(s)
    M = np.eye(9, dtype=np.complex128)
    one = np.array([[1, 2]])
    with pytest.raises(hgf.HgfError) as e:
        hgf.map_operator(S, sparse=(one, one, np.array([1.0 + 0j])), layout="split")
    assert e.value.status == "HGF_EUNSUPPORTED"
    op = hgf.map_operator(S, dense=M)
    for call in (lambda: hgf.evolve(op, 0.01, 1e-3, scheme="lawson"),
                 lambda: op.function(0),
                 lambda: hgf.grad(S, synth.coherent_state([0.1, 0.2]), 0.01, 1e-3, dense=M)):
        with pytest.raises(hgf.HgfError) as e:
            call()
        assert e.value.status == "HGF_EUNSUPPORTED"
    with pytest.raises(hgf.HgfError) as e:
        op.set_tile_config(0, 2)
    assert e.value.status == "HGF_EINVAL"
    with pytest.raises(hgf.HgfError) as e:
        hgf.evolve(op, 0.1, 0.1)  # far outside RK4's stability region
    assert e.value.status == "HGF_EUNSTABLE"
    # zero drive and exchange arrays keep the sector form
    z = synth.random_system((3, 3), 508)
    z.drive = np.zeros(2, dtype=np.complex128)
    z.exchange = np.zeros((2, 2))
    R = np.random.default_rng(508).normal(size=(9, 9)) + 0j
    assert hgf.map_operator(hgf.define_system(z), dense=R).info()["n_functions"] == 25  # 5 x 5 sectors
