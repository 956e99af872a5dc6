"""The tiled stage kernel of a network operator (tiles: the (k, l) block of the
last two modes in LDS, the other modes' terms from per-tile records) against
the oracle's full-matrix RK4 and against the untiled kernel."""

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


def all_pairs_network(cutoff, seed, dissipator="lindblad"):
    """Drive on every mode, exchange between every pair (so the records hold
    slow-slow and slow-fast exchange terms and the kernel the fast pair),
    cross-Kerr between every pair."""
    rng = np.random.default_rng(seed)
    s = synth.random_system(cutoff, seed, scale=2.0, n_th=0.2)
    n = len(cutoff)
    s.drive = (rng.normal(size=n) + 1j * rng.normal(size=n)) * 3.0
    J = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            J[i, j] = J[j, i] = rng.uniform(-4.0, 4.0)
    s.exchange = J
    if dissipator == "secular":
        s.dissipator = "secular"
        s.n_th_levels = rng.uniform(0.0, 0.5, size=sum(c - 1 for c in cutoff))
    return s


def rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def random_matrix(dim, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))


# tiles of 256 (4 x 4 levels), 400 (5 x 4, ragged) and 576 points; 9 to 36 tiles (the tiled
# kernel is then asked for: by default it takes grids of at least 256 tiles)
SHAPES = [((4, 4, 4), 601, "lindblad"), ((3, 5, 4), 602, "secular"), ((2, 3, 4, 4), 603, "lindblad"),
          ((3, 2, 4, 6), 604, "secular")]


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("cutoff,seed,dissipator", SHAPES)
def test_tiled_network_matches_oracle(hgf, cutoff, seed, dissipator, precision, tol):
    announce(f"tiled network {cutoff} {dissipator} {precision}")
    s = all_pairs_network(cutoff, seed, dissipator)
    dim = int(np.prod(cutoff))
    M = random_matrix(dim, seed)
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
    assert op.tile_config(0)["nfast"] == 0  # fewer than 256 tiles: untiled by default
    op.set_tile_config(0, 4)
    cfg = op.tile_config(0)
    assert cfg["nfast"] == 4 and cfg["tile_points"] == (cutoff[-2] * cutoff[-1]) ** 2
    T, dt = 0.02, 2.5e-4
    hgf.evolve(op, T, dt)
    ref = oracle.evolve_full(s, M, T, dt)
    L = min(cutoff)
    idx = [np.ravel_multi_index(k, cutoff) for k in np.ndindex(*(L,) * len(cutoff))]
    assert rel_fro(hgf.reconstruct(op, L), ref[np.ix_(idx, idx)]) < tol
    # every level through an expectation value
    alphas = [0.6 - 0.3j * j for j in range(len(cutoff))]
    c = np.ones(1, dtype=np.complex128)
    for a in oracle.state_amplitudes(cutoff, synth.coherent_state(alphas)):
        c = np.kron(c, a)
    want = np.conj(c) @ ref @ c
    got = hgf.expectation(op, synth.coherent_state(alphas))
    assert abs(got - want) / abs(want) < (10 * tol if precision == "mixed" else tol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tiled_and_untiled_network_kernels_agree(hgf, precision):
    """Every tiled launch shape (workgroup size, walk order, workgroups per CU)
    gives the same grid bit for bit (each point's arithmetic is the same), and
    the untiled kernel the same grid up to rounding."""
    cutoff = (3, 3, 4, 5)
    announce(f"tiled vs untiled network {cutoff} {precision}")
    s = all_pairs_network(cutoff, 611, "secular")
    dim = int(np.prod(cutoff))
    M = random_matrix(dim, 611)
    T, dt = 0.01, 5e-4
    shapes = [dict(), dict(threads=512), dict(threads=128, walk_block=2), dict(walk_block=3, wgs_per_cu=1)]
    grids = []
    for sh in shapes:
        op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
        op.set_tile_config(0, 4, **sh)
        cfg = op.tile_config(0)
        assert cfg["nfast"] == 4
        for k, v in sh.items():
            assert cfg[k] == v, (k, cfg)
        hgf.evolve(op, T, dt)
        grids.append(hgf.reconstruct(op, min(cutoff)))
    for g in grids[1:]:
        assert np.array_equal(g, grids[0])
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
    assert op.tile_config(0)["nfast"] == 0
    hgf.evolve(op, T, dt)
    assert rel_fro(grids[0], hgf.reconstruct(op, min(cutoff))) < (1e-13 if precision == "fp64" else 1e-6)


def test_tiled_network_table1_four_modes(hgf):
    """The paper's network example at four modes, cutoff 6 (the bench's tile
    of 1296 points, 1296 tiles), ten RK4 steps against the oracle."""
    announce("tiled network Table I, 4 modes")
    w = synth.table1_network(4, 6)
    op = hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="fp64")
    assert op.tile_config(0)["nfast"] == 4 and op.tile_config(0)["tile_points"] == 1296
    steps = 10
    hgf.evolve(op, steps * w.dt, w.dt)
    M0 = np.ones((1, 1), dtype=np.complex128)
    for f in w.factors:
        M0 = np.kron(M0, f)
    ref = oracle.evolve_full(w.system, M0, steps * w.dt, w.dt)
    assert rel_fro(hgf.reconstruct(op, 6), ref) < FP64_TOL


def test_tiled_network_table1_five_modes_against_untiled(hgf):
    """Five modes, cutoff 6 (60,466,176 points, the bench's grid and launch
    shape): two steps of the tiled kernel, FP64 and mixed, against the untiled
    FP64 kernel (itself checked against the oracle on smaller grids), on the
    three lowest levels and the expectation value."""
    announce("tiled network Table I, 5 modes")
    w = synth.table1_network(5, 6)
    out = {}
    for prec, nfast in (("fp64", 4), ("mixed", 4), ("fp64", 0)):
        op = hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision=prec)
        if nfast == 0:
            op.set_tile_config(0, 0)
        assert op.tile_config(0)["nfast"] == nfast
        hgf.evolve(op, 2 * w.dt, w.dt)
        out[prec, nfast] = (hgf.reconstruct(op, 3), hgf.expectation(op, w.states[0]))
        del op
    ref = out["fp64", 0]
    for key, tol in ((("fp64", 4), 1e-13), (("mixed", 4), MIXED_TOL)):
        assert rel_fro(out[key][0], ref[0]) < tol, key
        assert abs(out[key][1] - ref[1]) <= 10 * tol * abs(ref[1]), key


def test_network_modes_reordered_for_tiles(hgf):
    """A drive on one mode and a chain of exchanges: the grid holds the driven
    mode and its busiest partner in the tiles (here modes 1 and 2, 16 x 16
    points; in the given order the last two modes would give tiles of 64
    points, too small to tile), with ragged cutoffs; the readout and the
    expectation value come back in the caller's mode order."""
    cutoff = (3, 4, 4, 2)
    announce(f"network mode order {cutoff}")
    rng = np.random.default_rng(631)
    s = synth.random_system(cutoff, 631, scale=2.0, n_th=0.1)
    n = len(cutoff)
    s.drive = np.array([0.0, 2.5 - 1.5j, 0.0, 0.0])
    J = np.zeros((n, n))
    for i in range(n - 1):
        J[i, i + 1] = J[i + 1, i] = rng.uniform(1.0, 3.0)
    s.exchange = J
    dim = int(np.prod(cutoff))
    M = random_matrix(dim, 631)
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
        op.set_tile_config(0, 4)  # in the given order the tiles would hold 64 points: not feasible
        cfg = op.tile_config(0)
        assert cfg["nfast"] == 4 and cfg["tile_points"] == 256
        T, dt = 0.02, 2.5e-4
        hgf.evolve(op, T, dt)
        ref = oracle.evolve_full(s, M, T, dt)
        L = min(cutoff)
        idx = [np.ravel_multi_index(k, cutoff) for k in np.ndindex(*(L,) * n)]
        assert rel_fro(hgf.reconstruct(op, L), ref[np.ix_(idx, idx)]) < tol
        alphas = [0.7, 0.4j, -0.5, 0.3 + 0.3j]
        c = np.ones(1, dtype=np.complex128)
        for a in oracle.state_amplitudes(cutoff, synth.coherent_state(alphas)):
            c = np.kron(c, a)
        want = np.conj(c) @ ref @ c
        got = hgf.expectation(op, synth.coherent_state(alphas))
        assert abs(got - want) / abs(want) < (10 * tol if precision == "mixed" else tol)


def test_tiled_network_in_a_batch(hgf):
    """A network operator on the tiled kernel and a sector operator evolved in
    one batch equal their separate evolves bit for bit."""
    announce("tiled network batch")
    a = all_pairs_network((3, 3, 4, 5), 641, "secular")
    b = synth.random_system((4, 5, 3), 642, scale=2.0)
    Ma = random_matrix(180, 641)
    fb = synth.parity_factors((4, 5, 3))
    runs = []
    for batched in (True, False):
        ops = [hgf.map_operator(hgf.define_system(a), dense=Ma, precision="mixed"),
               hgf.map_operator(hgf.define_system(b), factors=fb, precision="mixed")]
        ops[0].set_tile_config(0, 4)
        if batched:
            hgf.evolve_batch(ops, [0.02, 0.03], [1e-3, 1e-3])
        else:
            hgf.evolve(ops[0], 0.02, 1e-3)
            hgf.evolve(ops[1], 0.03, 1e-3)
        runs.append([hgf.reconstruct(op, 3) for op in ops])
    for x, y in zip(*runs):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("cutoff,precision,tol,points", [((2, 8, 8), "mixed", MIXED_TOL, 4096),
                                                         ((3, 7, 7), "fp64", FP64_TOL, 2401)])
def test_tiled_network_largest_tiles(hgf, cutoff, precision, tol, points):
    """The largest tiles the kernel takes: 8 x 8 levels (4096 points, eight
    lane rounds of 512 lanes; mixed precision, whose LDS allows it) and 7 x 7
    levels in FP64, against the oracle."""
    announce(f"tiled network largest tiles {cutoff} {precision}")
    s = all_pairs_network(cutoff, 651, "lindblad")
    dim = int(np.prod(cutoff))
    M = random_matrix(dim, 651)
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
    op.set_tile_config(0, 4)
    cfg = op.tile_config(0)
    assert cfg["nfast"] == 4 and cfg["tile_points"] == points
    assert (points + cfg["threads"] - 1) // cfg["threads"] <= 8
    T, dt = 0.01, 2.5e-4
    hgf.evolve(op, T, dt)
    ref = oracle.evolve_full(s, M, T, dt)
    L = min(cutoff)
    idx = [np.ravel_multi_index(k, cutoff) for k in np.ndindex(*(L,) * len(cutoff))]
    assert rel_fro(hgf.reconstruct(op, L), ref[np.ix_(idx, idx)]) < tol
    alphas = [0.5, 0.3 - 0.4j, 0.6j]
    c = np.ones(1, dtype=np.complex128)
    for a in oracle.state_amplitudes(cutoff, synth.coherent_state(alphas)):
        c = np.kron(c, a)
    want = np.conj(c) @ ref @ c
    assert abs(hgf.expectation(op, synth.coherent_state(alphas)) - want) / abs(want) < 10 * tol
    if precision == "fp64":  # 8 x 8 levels do not fit the FP64 tile's LDS
        s8 = all_pairs_network((2, 8, 8), 652)
        op8 = hgf.map_operator(hgf.define_system(s8), dense=random_matrix(128, 652), precision="fp64")
        with pytest.raises(hgf.HgfError) as e:
            op8.set_tile_config(0, 4)
        assert e.value.status == "HGF_EINVAL"


def test_tiled_network_six_modes_all_pairs(hgf):
    """Six modes (cutoffs 3, 3, 3, 3, 4, 4: 1,679,616 points, 6,561 tiles of
    256, tiled by default), a drive on every mode and exchange between every
    pair, secular dissipator: the records then hold four slow modes' jumps and
    drives, six slow-slow and eight slow-fast exchange pairs.  Ten steps
    against the oracle, FP64 and mixed."""
    cutoff = (3, 3, 3, 3, 4, 4)
    announce(f"tiled network six modes {cutoff}")
    s = all_pairs_network(cutoff, 661, "secular")
    dim = int(np.prod(cutoff))
    M = random_matrix(dim, 661)
    T, dt = 0.005, 5e-4
    ref = oracle.evolve_full(s, M, T, dt)
    alphas = [0.3, -0.2j, 0.25, 0.1 + 0.1j, 0.4, -0.3]
    c = np.ones(1, dtype=np.complex128)
    for a in oracle.state_amplitudes(cutoff, synth.coherent_state(alphas)):
        c = np.kron(c, a)
    want = np.conj(c) @ ref @ c
    L = min(cutoff)
    idx = [np.ravel_multi_index(k, cutoff) for k in np.ndindex(*(L,) * len(cutoff))]
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        op = hgf.map_operator(hgf.define_system(s), dense=M, precision=precision)
        cfg = op.tile_config(0)
        assert cfg["nfast"] == 4 and cfg["tile_points"] == 256
        hgf.evolve(op, T, dt)
        assert rel_fro(hgf.reconstruct(op, L), ref[np.ix_(idx, idx)]) < tol
        assert abs(hgf.expectation(op, synth.coherent_state(alphas)) - want) / abs(want) < 10 * tol
        del op


def test_network_tile_config_errors(hgf):
    s = all_pairs_network((3, 4, 4), 621)
    M = random_matrix(48, 621)
    op = hgf.map_operator(hgf.define_system(s), dense=M, precision="fp64")
    op.set_tile_config(0, 4)
    before = op.tile_config(0)
    for bad in [dict(nfast=3), dict(nfast=4, xblock=2), dict(nfast=4, pipe=1), dict(nfast=4, resident=1),
                dict(nfast=4, threads=193), dict(nfast=4, threads=576)]:
        with pytest.raises(hgf.HgfError) as e:
            op.set_tile_config(0, **bad)
        assert e.value.status == "HGF_EINVAL", bad
        assert op.tile_config(0) == before
    # two modes: no slow mode to tile over, the untiled kernel only
    s2 = all_pairs_network((4, 4), 622)
    op2 = hgf.map_operator(hgf.define_system(s2), dense=random_matrix(16, 622), precision="fp64")
    assert op2.tile_config(0)["nfast"] == 0
    with pytest.raises(hgf.HgfError) as e:
        op2.set_tile_config(0, 4)
    assert e.value.status == "HGF_EINVAL"


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", MIXED_TOL)])
def test_tiled_network_harmonic_chain_closed_form(hgf, precision, tol):
    """The five-mode, cutoff-6 grid of the bench (60,466,176 points, default
    tiled launch) with the Kerr terms set to zero and the Lindblad dissipator:
    the first moments then obey the closed linear equation
    d<a>/dt = -(i H1 + Gamma/2) <a> - i Omega (H1: detunings and exchange,
    Gamma: decay rates), so from the vacuum <a_k>(T) = [-i M^-1 (1 - exp(-M T)) Omega]_k
    with M = i H1 + Gamma/2.  A weak drive keeps the field near 0.1, where the
    six-level truncation is far below the tolerance."""
    import scipy.linalg
    n, nc = 5, 6
    announce(f"tiled network harmonic chain closed form {precision}")
    w = synth.table1_network(n, nc)
    s = w.system.copy()
    s.kerr = np.zeros(n)
    s.dissipator = "lindblad"
    s.n_th = np.zeros(n)
    s.drive = np.array([-1j * 2 * np.pi * 12.5] + [0.0] * (n - 1), dtype=np.complex128)
    H1 = np.diag(s.detuning).astype(np.complex128) + s.exchange
    M = 1j * H1 + np.diag(s.gamma1) / 2
    T, dt = w.t_total, w.dt
    field = -1j * np.linalg.solve(M, (np.eye(n) - scipy.linalg.expm(-M * T)) @ s.drive)
    a = np.diag(np.sqrt(np.arange(1, nc, dtype=float)), 1).astype(np.complex128)
    vacuum = synth.fock_state([0] * n)
    for k in (0, n - 1):
        fac = [a if j == k else np.eye(nc, dtype=np.complex128) for j in range(n)]
        op = hgf.map_operator(hgf.define_system(s), factors=fac, precision=precision)
        assert op.tile_config(0)["nfast"] == 4
        hgf.evolve(op, T, dt)
        got = hgf.expectation(op, vacuum)
        assert abs(got - field[k]) < tol * np.max(np.abs(field)), (k, got, field[k])
        del op
