"""Thresholded representation (hgf_set_threshold): after every RK4 step the
coefficients with |g| <= threshold are dropped.  Checked against the same
truncation applied step by step to the oracle's results (the full-grid
network and the separated form), with the peak count of kept coefficients."""

import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgf():
    return library()


def _product(factors):
    A = np.ones((1, 1), dtype=np.complex128)
    for f in factors:
        A = np.kron(A, f)
    return A


def _fac(cutoff):
    dim = int(np.prod(cutoff))
    return np.array([math.sqrt(float(np.prod([math.factorial(int(x)) for x in np.unravel_index(K, cutoff)])))
                     for K in range(dim)])


def test_threshold_full_grid_matches_truncated_oracle(hgf):
    """Table I chain, 2 modes at cutoff 5: the full (k, l) grid truncated at
    |g| <= 1e-5 after each step, against the oracle's full-matrix RK4 step
    followed by the same truncation of g = A / sqrt(k! l!)."""
    w = synth.table1_network(2, 5)
    s = w.system
    thr = 1e-5
    announce("threshold, full grid")
    op = hgf.map_operator(hgf.define_system(s), factors=w.factors)
    hgf.set_threshold(op, thr)
    hgf.evolve(op, w.t_total, w.dt)
    fac = _fac(s.cutoff)
    scale = np.outer(fac, fac)
    A = _product(w.factors)
    peak = 0
    for _ in range(w.n_steps):
        A = oracle.evolve_full(s, A, w.dt, w.dt)
        g = A / scale
        g[np.abs(g) <= thr] = 0.0
        peak = max(peak, int(np.count_nonzero(g)))
        A = g * scale
    got = hgf.reconstruct(op, 5)
    assert float(np.max(np.abs(got - A)) / np.max(np.abs(A))) < 1e-9
    g = got / scale
    assert np.all((g == 0) | (np.abs(g) > thr))
    assert op.info()["stored_peak"] == peak
    assert 0 < peak < g.size
    # below three modes the tile is the whole grid
    assert op.info()["tile_points"] == g.size and op.info()["stored_tiles_peak"] == 1


def test_threshold_tiles_three_mode_network(hgf):
    """Table I chain, 3 modes at cutoff 4: the kept coefficients and the kept
    tiles.  The stage kernel's tile is the (k, l) block of the two fastest
    positions; for this chain the drive and the 1-2 exchange put modes 1 and 2
    there, so a tile is one (k_3, l_3) pair of mode 3."""
    w = synth.table1_network(3, 4)
    s = w.system
    thr = 1e-4
    announce("threshold tiles, 3-mode network")
    op = hgf.map_operator(hgf.define_system(s), factors=w.factors)
    hgf.set_threshold(op, thr)
    hgf.evolve(op, w.t_total, w.dt)
    fac = _fac(s.cutoff)
    scale = np.outer(fac, fac)
    A = _product(w.factors)
    peak = tpeak = 0
    for _ in range(w.n_steps):
        A = oracle.evolve_full(s, A, w.dt, w.dt)
        g = A / scale
        g[np.abs(g) <= thr] = 0.0
        peak = max(peak, int(np.count_nonzero(g)))
        occ = np.any(g.reshape((4,) * 6) != 0, axis=(0, 1, 3, 4))  # (k_3, l_3)
        tpeak = max(tpeak, int(np.count_nonzero(occ)))
        A = g * scale
    got = hgf.reconstruct(op, 4)
    assert float(np.max(np.abs(got - A)) / np.max(np.abs(A))) < 1e-9
    info = op.info()
    assert info["stored_peak"] == peak
    assert info["tile_points"] == 4 ** 4
    assert info["stored_tiles_peak"] == tpeak
    assert 0 < tpeak <= 16


def test_threshold_separated_matches_truncated_oracle(hgf):
    """The separated form (R on the diagonal), 2 modes at cutoff 5, every
    Gx, Gy and R coefficient truncated at |g| <= 1e-5 after each step."""
    w = synth.table1_network(2, 5)
    s = w.system
    thr = 1e-5
    announce("threshold, separated")
    op = hgf.map_operator(hgf.define_system(s), factors=w.factors, layout="separated")
    hgf.set_threshold(op, thr)
    hgf.evolve(op, w.t_total, w.dt)
    monos = oracle.monomials(s, _product(w.factors))
    state = None
    peak = tpeak = 0
    for _ in range(w.n_steps):
        gx, gy, r = oracle.evolve_separated(s, monos, w.dt, w.dt, "z", state=state)
        for a in (gx, gy, r):
            a[np.abs(a) <= thr] = 0.0
        peak = max(peak, int(np.count_nonzero(gx) + np.count_nonzero(gy) + np.count_nonzero(r)))
        # tiles: one grid each (Gx_i, Gy_i, the diagonal R)
        tiles = sum(int(np.any(a.reshape(len(monos), -1) != 0, axis=1).sum()) for a in (gx, gy)) + int(np.any(r != 0))
        tpeak = max(tpeak, tiles)
        state = (gx, gy, r)
    ref = oracle.separated_matrix(s, monos, *state)
    got = hgf.reconstruct(op, 5)
    assert float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))) < 1e-9
    assert op.info()["stored_peak"] == peak
    assert 0 < peak < op.info()["total_points"]
    assert op.info()["tile_points"] == 25
    assert op.info()["stored_tiles_peak"] == tpeak


def test_threshold_switches(hgf):
    """Threshold 0 turns the truncation off (the same result as never set);
    negative thresholds are refused; a batch refuses a truncated member;
    sector operators are not truncated."""
    w = synth.table1_network(2, 4)
    S = hgf.define_system(w.system)
    a = hgf.map_operator(S, factors=w.factors)
    b = hgf.map_operator(S, factors=w.factors)
    hgf.set_threshold(b, 1e-3)
    hgf.set_threshold(b, 0.0)
    hgf.evolve(a, w.t_total, w.dt)
    hgf.evolve(b, w.t_total, w.dt)
    assert np.array_equal(hgf.reconstruct(a, 4), hgf.reconstruct(b, 4))
    assert a.info()["stored_peak"] == -1
    with pytest.raises(hgf.HgfError) as e:
        hgf.set_threshold(a, -1.0)
    assert e.value.status == "HGF_EINVAL"
    hgf.set_threshold(b, 1e-6)
    with pytest.raises(hgf.HgfError) as e:  # truncation runs step by step in hgf_evolve only
        hgf.evolve_batch([a, b], [w.t_total] * 2, [w.dt] * 2)
    assert e.value.status == "HGF_EUNSUPPORTED"
    s = synth.random_system((3, 3), 1)
    c = hgf.map_operator(hgf.define_system(s), factors=[np.eye(3), np.eye(3)])
    with pytest.raises(hgf.HgfError) as e:
        hgf.set_threshold(c, 1e-3)
    assert e.value.status == "HGF_EUNSUPPORTED"
