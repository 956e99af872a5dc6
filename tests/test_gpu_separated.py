"""The separated form of Eqs. (9a)-(9c) on the GPU (layouts HGF_SEPARATED:
R on the diagonal k = l, and HGF_SEPARATED_EXACT: R on the whole box),
against the oracle's separated form (the same classical RK4 on the joint
state (Gx_i, Gy_i, R), written from the paper's equations and pinned by its
fourth-order convergence to the dense expm).  FP64, tolerance 1e-10 relative
(max-normalised over the number-basis matrix) and on expectation values."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, library, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def hgf():
    return library()


def _matrix_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _product(factors):
    A = np.ones((1, 1), dtype=np.complex128)
    for f in factors:
        A = np.kron(A, f)
    return A


@pytest.mark.parametrize("layout", ["separated", "separated_exact"])
@pytest.mark.parametrize("modes,cutoff", [(1, 6), (2, 6), (3, 4)])
def test_table1_chain_matches_oracle(hgf, layout, modes, cutoff):
    """The paper's network example (Table I: chain at the drive frequency,
    drive on mode 1, secular dissipator at zero temperature), operator
    prod_j a_j (one monomial per nonzero g_{p,q}(0): (cutoff - 1)^N),
    w_q t / pi = 10 in 100 RK4 steps."""
    w = synth.table1_network(modes, cutoff)
    s = w.system
    announce(f"separated {layout}: Table I, {modes} modes, cutoff {cutoff}")
    op = hgf.map_operator(hgf.define_system(s), factors=w.factors, layout=layout)
    info = op.info()
    nm = (cutoff - 1) ** modes
    dim = cutoff ** modes
    assert info["n_functions"] == 2 * nm + 1
    assert info["total_points"] == 2 * nm * dim + (dim if layout == "separated" else dim * dim)
    hgf.evolve(op, w.t_total, w.dt)
    monos = oracle.monomials(s, _product(w.factors))
    assert len(monos) == nm
    gx, gy, r = oracle.evolve_separated(s, monos, w.t_total, w.dt, "z" if layout == "separated" else "full")
    ref = oracle.separated_matrix(s, monos, gx, gy, r)
    got = hgf.reconstruct(op, cutoff)
    assert _matrix_err(got, ref) < FP64_TOL
    st = w.states[0]
    amps = oracle.state_amplitudes(s.cutoff, st)
    c = amps[0]
    for a in amps[1:]:
        c = np.kron(c, a)
    assert rel(hgf.expectation(op, st), np.conj(c) @ ref @ c) < FP64_TOL


@pytest.mark.parametrize("layout", ["separated", "separated_exact"])
@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
def test_random_network_matches_oracle(hgf, layout, dissipator):
    """A random driven, exchange-coupled two-mode network with thermal jumps
    and dephasing, and a random operator over all (k, l) (every coefficient a
    monomial)."""
    cutoff = (3, 4)
    rng = np.random.default_rng(401)
    s = synth.random_system(cutoff, 401, scale=2.0, n_th=0.2)
    s.gamma_phi = np.array([0.4, 0.3])
    s.drive = np.array([1.5 - 2.0j, 0.7 + 1.1j])
    s.exchange = np.array([[0.0, 2.5], [2.5, 0.0]])
    if dissipator == "secular":
        s.dissipator = "secular"
        s.n_th_levels = rng.uniform(0.0, 0.5, size=2 + 3)
    announce(f"separated {layout}: random network, {dissipator}")
    dim = 12
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    op = hgf.map_operator(hgf.define_system(s), dense=A0, layout=layout)
    T, dt = 0.2, 1e-3
    hgf.evolve(op, T, dt)
    monos = oracle.monomials(s, A0)
    gx, gy, r = oracle.evolve_separated(s, monos, T, dt, "z" if layout == "separated" else "full")
    ref = oracle.separated_matrix(s, monos, gx, gy, r)
    assert _matrix_err(hgf.reconstruct(op, 3), ref[np.ix_(*[_levels(cutoff, 3)] * 2)]) < FP64_TOL
    st = synth.coherent_state([0.6 + 0.2j, 0.5])
    c = np.kron(*oracle.state_amplitudes(cutoff, st))
    assert rel(hgf.expectation(op, st), np.conj(c) @ ref @ c) < FP64_TOL


def _levels(cutoff, L):
    """Flat indices (over the cutoff box) of the points with every occupation below L."""
    import itertools
    return [int(np.ravel_multi_index(k, cutoff)) for k in itertools.product(*[range(L)] * len(cutoff))]


def test_separated_layout_rules(hgf):
    """FP64 only; R on the whole box is refused beyond 2^28 points; an evolve
    split into two calls equals one call."""
    w = synth.table1_network(2, 5)
    S = hgf.define_system(w.system)
    with pytest.raises(hgf.HgfError) as e:
        hgf.map_operator(S, factors=w.factors, layout="separated", precision="mixed")
    assert e.value.status == "HGF_EUNSUPPORTED"
    a = hgf.map_operator(S, factors=w.factors, layout="separated")
    b = hgf.map_operator(S, factors=w.factors, layout="separated")
    hgf.evolve(a, w.t_total, w.dt)
    hgf.evolve(b, w.t_total / 2, w.dt)
    hgf.evolve(b, w.t_total / 2, w.dt)
    assert np.array_equal(hgf.reconstruct(a, 5), hgf.reconstruct(b, 5))
    assert a.info()["steps_done"] == 100


@pytest.mark.parametrize("layout", ["separated", "separated_exact"])
def test_ragged_three_modes_sparse_operator_with_drop_tol(hgf, layout):
    """Three modes of unequal cutoffs (3, 4, 5) in a driven exchange chain
    under the Lindblad dissipator at finite temperature, a sparse random
    operator, and drop_tol keeping part of its monomials (the same ones on
    both sides: the threshold sits in a wide gap of the |g_{p,q}(0)|)."""
    cutoff = (3, 4, 5)
    s = synth.random_system(cutoff, 402, scale=2.0, n_th=0.15)
    s.gamma_phi = np.array([0.2, 0.5, 0.3])
    s.drive = np.array([0.0, 1.2 + 0.4j, -0.6j])
    s.exchange = np.array([[0.0, 1.7, 0.0], [1.7, 0.0, -2.2], [0.0, -2.2, 0.0]])
    ks, ls, vals = synth.random_sparse_operator(cutoff, 40, 402)
    dim = int(np.prod(cutoff))
    A0 = np.zeros((dim, dim), dtype=np.complex128)
    for k, l, v in zip(ks, ls, vals):
        A0[np.ravel_multi_index(k, cutoff), np.ravel_multi_index(l, cutoff)] += v
    g = np.sort(np.array([abs(m[2]) for m in oracle.monomials(s, A0)]))
    gaps = g[1:] / g[:-1]
    idx = np.arange(len(gaps))
    i = int(np.argmax(np.where((idx >= len(g) // 3) & (idx < 2 * len(g) // 3), gaps, 0.0)))
    assert gaps[i] > 1.01
    drop = float(np.sqrt(g[i] * g[i + 1]))
    monos = oracle.monomials(s, A0, drop_tol=drop)
    assert 0 < len(monos) < len(g)
    announce(f"separated {layout}: ragged 3 modes, {len(monos)} of {len(g)} monomials")
    op = hgf.map_operator(hgf.define_system(s), sparse=(ks, ls, vals), layout=layout, drop_tol=drop)
    assert op.info()["n_functions"] == 2 * len(monos) + 1
    T, dt = 0.1, 1e-3
    hgf.evolve(op, T, dt)
    gx, gy, r = oracle.evolve_separated(s, monos, T, dt, "z" if layout == "separated" else "full")
    ref = oracle.separated_matrix(s, monos, gx, gy, r)
    assert _matrix_err(hgf.reconstruct(op, 3), ref[np.ix_(*[_levels(cutoff, 3)] * 2)]) < FP64_TOL
    st = synth.coherent_state([0.4, 0.7 - 0.3j, 0.5j])
    amps = oracle.state_amplitudes(cutoff, st)
    c = np.kron(np.kron(amps[0], amps[1]), amps[2])
    assert rel(hgf.expectation(op, st), np.conj(c) @ ref @ c) < FP64_TOL


def test_separated_zero_operator_and_noalloc_refusal(hgf):
    """With every coefficient below drop_tol there is no monomial: R stays
    zero; the allocation-free expectation refuses the separated layouts."""
    w = synth.table1_network(2, 4)
    S = hgf.define_system(w.system)
    op = hgf.map_operator(S, factors=w.factors, layout="separated", drop_tol=1e9)
    assert op.info()["n_functions"] == 1
    hgf.evolve(op, w.t_total, w.dt)
    assert np.all(hgf.reconstruct(op, 4) == 0)
    assert hgf.expectation(op, w.states[0]) == 0
    op2 = hgf.map_operator(S, factors=w.factors, layout="separated")
    with pytest.raises(hgf.HgfError) as e:
        hgf.expectation_noalloc(op2, w.states[0])
    assert e.value.status == "HGF_EUNSUPPORTED"
