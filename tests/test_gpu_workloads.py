"""Full-horizon parity of the benchmark workloads against the FP64 oracle.

On the diagonal sector (every observable of these workloads lies there) the
generator is a constant plus a sum of commuting single-mode generators, so a
product observable evolves into the product of single-mode solutions, exact
up to RK4's O(h^5) splitting term (below 1e-20 per step at these step
sizes).  The references are therefore products of single-mode oracle runs at
the full horizon, at any number of modes.

* 10 Kerr modes at cutoff 6 (6^10 points), parity-weighted projector, T = 2 us,
  dt = 0.05 ns (4e4 steps), in the launch shape the benchmark times: mixed
  precision within 1e-5 and FP64 within 1e-10, at sampled grid points (in the
  number basis) and through the expectation value.
* The 96-member batch (64 x 6 modes at cutoff 8, 32 uneven systems of 2-5
  modes at cutoffs 6-20), T = 1 us, dt = 0.1 ns (1e4 steps) in one grouped
  evolve: every member's expectation value within 1e-5 (mixed).
"""

import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, library, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def hgf():
    return library()


def single_mode_runs(system, factors, state, steps, dt):
    """Per mode: the number-basis diagonal of the evolved factor and its
    expectation value in the mode's state (oracle, one thread)."""
    diag, vals = [], []
    for j, nc in enumerate(system.cutoff):
        sj = synth.System((nc,), system.detuning[j:j + 1], system.kerr[j:j + 1], np.zeros((1, 1)),
                          system.gamma1[j:j + 1], system.gamma_phi[j:j + 1], system.n_th[j:j + 1])
        out = oracle.evolve_steps(sj, oracle.product_sectors([factors[j]]), steps, dt, nthreads=1)
        diag.append(out[(0,)].copy())
        vals.append(oracle.expectation((nc,), out, (state[0], [state[1][j]])))
    return diag, vals


@pytest.fixture(scope="module")
def c4_reference():
    w = synth.large_c4()
    steps = w.n_steps
    assert steps == 40000
    announce("10-mode workload: single-mode oracle references at the full horizon")
    diag, vals = single_mode_runs(w.system, w.factors, w.states[0], steps, w.dt)
    return w, diag, complex(np.prod(vals))


def _check_c4(hgf, w, diag, Jref, op, tol):
    d, e, grid, _ = op.function(0)
    assert d == (0,) * 10 and e == (6,) * 10
    rng = np.random.default_rng(7)
    idx = rng.integers(0, 6, size=(50000, 10))
    idx = np.concatenate([idx, np.array(np.unravel_index(np.arange(64), (2,) * 6 + (1,) * 4)).T])
    ref = np.ones(len(idx), dtype=np.complex128)
    for j in range(10):
        ref *= diag[j][idx[:, j]]
    fact = np.array([float(math.factorial(m)) for m in range(6)])
    got = grid[tuple(idx.T)] * np.prod(fact[idx], axis=1)  # number basis: g * prod_j k_j!
    err_pts = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    J = hgf.expectation(op, w.states[0])
    err_J = rel(J, Jref)
    announce(f"  sampled points {err_pts:.2e}, expectation {err_J:.2e} ({J} vs {Jref})")
    assert err_pts < tol
    assert err_J < tol


@pytest.mark.parametrize("precision,tol", [("mixed", MIXED_TOL), ("fp64", FP64_TOL)])
def test_ten_mode_workload_full_horizon(hgf, c4_reference, precision, tol):
    w, diag, Jref = c4_reference
    announce(f"10-mode workload, 4e4 steps, {precision}")
    op = hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision=precision)
    hgf.autotune([op], w.dt)  # the launch shape the benchmark times
    announce(f"  shape {op.tile_config(0)}")
    hgf.evolve(op, w.t_total, w.dt)
    assert op.info()["steps_done"] == 40000
    _check_c4(hgf, w, diag, Jref, op, tol)


def test_batch_workload_full_horizon(hgf):
    ws = synth.batch_c2()
    assert len(ws) == 96
    announce("batch workload: 96 members, 1e4 steps, one grouped evolve (mixed)")
    ops = [hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="mixed") for w in ws]
    hgf.autotune(ops, ws[0].dt)
    hgf.evolve_batch(ops, [w.t_total for w in ws], [w.dt for w in ws])
    worst = 0.0
    for i, (w, op) in enumerate(zip(ws, ops)):
        assert op.info()["steps_done"] == w.n_steps == 10000
        _, vals = single_mode_runs(w.system, w.factors, w.states[0], w.n_steps, w.dt)
        Jref = complex(np.prod(vals))
        err = rel(hgf.expectation(op, w.states[0]), Jref)
        worst = max(worst, err)
        assert err < MIXED_TOL, (i, w.name, err)
    announce(f"  worst member error {worst:.2e}")
