"""The resident integrator of small network operators (the whole (k, l) grid
twice in LDS, one workgroup per operator, every step of a call in one
launch) against the oracle's full-matrix RK4 and against the untiled stage
kernel, alone, in a batch and under a threshold."""

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


def _network(cutoff, seed, dissipator="lindblad"):
    """Drive on every mode, exchange and cross-Kerr between every pair,
    thermal jumps and dephasing."""
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


def _err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("cutoff,dissipator", [((6,), "lindblad"), ((5, 5), "secular"), ((3, 3, 3), "lindblad")])
def test_resident_network_matches_oracle_and_untiled(hgf, precision, tol, cutoff, dissipator):
    """One to three modes (grids of 36, 625 and 729 points), a dense random
    operator, 40 RK4 steps: the resident form (the default for these grids)
    against the oracle, and against the untiled kernel (the same stencil
    arithmetic, so the two agree to the last bits)."""
    s = _network(cutoff, 61 + len(cutoff), dissipator)
    dim = int(np.prod(cutoff))
    rng = np.random.default_rng(61)
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    announce(f"resident network {cutoff} {dissipator} {precision}")
    S = hgf.define_system(s)
    a = hgf.map_operator(S, dense=A0, precision=precision)
    cfg = a.tile_config(0)
    assert cfg["resident"] == 1 and cfg["nfast"] == 0 and a.info()["untiled_functions"] == 0
    b = hgf.map_operator(S, dense=A0, precision=precision)
    b.set_tile_config(0, 0)
    assert b.tile_config(0)["resident"] == 0 and b.info()["untiled_functions"] == 1
    T, dt = 0.04, 1e-3
    hgf.evolve(a, T, dt)
    hgf.evolve(b, T, dt)
    L = max(cutoff)
    ga, gb = hgf.reconstruct(a, L), hgf.reconstruct(b, L)
    ref = oracle.evolve_full(s, A0, T, dt)
    assert _err(ga, ref) < tol
    assert _err(ga, gb) < (1e-13 if precision == "fp64" else 1e-6)


def test_resident_network_batch_threshold_and_switches(hgf):
    """A batch of three resident networks and one on the untiled kernel equals
    the members evolved one at a time; a threshold runs the resident form step
    by step; the resident form can be switched off and on again, and is
    refused for a grid beyond LDS."""
    announce("resident networks in a batch")
    w = synth.table1_network(2, 5)
    S = hgf.define_system(w.system)
    ops = [hgf.map_operator(S, factors=w.factors) for _ in range(4)]
    ops[3].set_tile_config(0, 0)
    alone = [hgf.map_operator(S, factors=w.factors) for _ in range(4)]
    alone[3].set_tile_config(0, 0)
    hgf.evolve_batch(ops, [w.t_total] * 4, [w.dt] * 4)
    for op in alone:
        hgf.evolve(op, w.t_total, w.dt)
    for x, y in zip(ops, alone):
        assert np.array_equal(hgf.reconstruct(x, 5), hgf.reconstruct(y, 5))
    # threshold: the resident form advanced one step at a time, truncated in
    # between (its values against the truncated oracle: tests/test_gpu_threshold.py);
    # here only that it advanced: near the untruncated result (|g| <= 1e-5
    # dropped, scaled by up to sqrt(4! 4!) in the number basis), not at the start
    t = hgf.map_operator(S, factors=w.factors)
    hgf.set_threshold(t, 1e-5)
    hgf.evolve(t, w.t_total, w.dt)
    assert 0 < t.info()["stored_peak"] < t.info()["total_points"]
    start = hgf.reconstruct(hgf.map_operator(S, factors=w.factors), 5)
    assert _err(hgf.reconstruct(t, 5), hgf.reconstruct(alone[0], 5)) < 0.05
    assert _err(hgf.reconstruct(t, 5), start) > 0.5
    # switches
    ops[3].set_tile_config(0, 0, resident=1)
    assert ops[3].tile_config(0)["resident"] == 1
    big = hgf.map_operator(hgf.define_system(synth.table1_network(3, 6).system),
                           factors=synth.table1_network(3, 6).factors)
    assert big.tile_config(0)["resident"] == 0
    with pytest.raises(hgf.HgfError) as e:
        big.set_tile_config(0, 0, resident=1)  # 46,656 points: beyond LDS
    assert e.value.status == "HGF_EINVAL"
