"""The gradient (hgf_grad: discrete adjoint of the RK4 steps on the transposed
generator, checkpointed) on the paths the workloads run: the LDS-tiled stage
kernel with slow-axis neighbour tiles, both dissipators; the full 4-mode
cutoff-16 workload against factorised single-mode oracle sensitivities with
its exact zeros; central finite differences of the forward evolve; and the
torch.autograd.Function built on it.

Tolerances: 1e-10 relative (FP64) against the oracle's forward
sensitivities, as max |g - ref| / max |ref| over the parameters; central
differences (h = 1e-6 relative) agree to their own truncation and
cancellation error, 1e-6 relative."""

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


def tridiagonal_factors(cutoff, seed):
    """Hermitian per-mode factors (a + a^+) + diag(r): sectors d_j in {-1, 0, 1}."""
    rng = np.random.default_rng(seed)
    return [q + np.diag(rng.uniform(-1.0, 1.0, size=c)) for q, c in zip(synth.quadrature_factors(cutoff), cutoff)]


def oracle_value_and_grad(s, ops, T, dt, st):
    fin, sens = oracle.evolve_sens(s, ops, T, dt)
    return oracle.expectation(s.cutoff, fin, st), np.array([oracle.expectation(s.cutoff, sp, st) for sp in sens])


def grad_err(g, ref):
    return float(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))


def slow_axis_system(dissipator, seed):
    s = synth.random_system((5, 5, 5, 5), seed, scale=2.0, n_th=0.2)
    if dissipator == "secular":
        rng = np.random.default_rng(seed)
        s.dissipator = "secular"
        s.n_th_levels = rng.uniform(0.0, 0.6, size=4 * 4)
    return s


@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
@pytest.mark.parametrize("max_nfast", [1, 2])
def test_gradient_with_slow_axes_matches_oracle(hgf, monkeypatch, dissipator, max_nfast):
    """4 modes at cutoff 5 with tridiagonal Hermitian factors (81 sectors of
    up to 625 points), the tiled kernel held to 1 or 2 fast axes: the forward
    and adjoint stencils read 3 or 2 slow axes of neighbour tiles, and the
    transposed tables of those axes enter every reverse step."""
    monkeypatch.setenv("HGF_MAX_NFAST", str(max_nfast))
    announce(f"gradient, slow axes (nfast <= {max_nfast}), {dissipator}")
    s = slow_axis_system(dissipator, 301 + max_nfast)
    fac = tridiagonal_factors(s.cutoff, 301)
    S = hgf.define_system(s)
    probe = hgf.map_operator(S, factors=fac, precision="fp64")
    cfgs = [probe.tile_config(i) for i in range(probe.info()["n_functions"])]
    assert any(c["resident"] == 0 and 0 < c["nfast"] <= max_nfast and c["blocks"] > 0 for c in cfgs)
    del probe
    st = synth.coherent_state([0.6 + 0.2j, 0.9, -0.4j, 0.5])
    T, dt = 0.02, 1e-3
    ref_val, ref_grad = oracle_value_and_grad(s, oracle.product_sectors(fac), T, dt, st)
    assert np.min(np.abs(ref_grad)) > 1e-6 * np.max(np.abs(ref_grad))  # every parameter matters here
    for ce in (1, 7, 100):
        val, g = hgf.grad(S, st, T, dt, factors=fac, checkpoint_every=ce)
        assert rel(val, ref_val) < FP64_TOL, ce
        assert grad_err(g, ref_grad) < FP64_TOL, (ce, grad_err(g, ref_grad))


def test_gradient_six_modes_default_tiles(hgf):
    """6 modes at cutoff 4 with the product of quadratures (64 sectors of
    3^6 points): the default shape tiles the four trailing axes and leaves two
    slow axes."""
    cutoff = (4,) * 6
    announce("gradient, 6 modes, quadratures, default tiles")
    s = synth.random_system(cutoff, 311, scale=2.0, n_th=0.2)
    fac = synth.quadrature_factors(cutoff)
    S = hgf.define_system(s)
    probe = hgf.map_operator(S, factors=fac, precision="fp64")
    cfg = probe.tile_config(0)
    assert cfg["resident"] == 0 and cfg["nfast"] == 4 and cfg["blocks"] > 0
    del probe
    st = synth.coherent_state([0.5, 0.4j, 0.7, 0.3 - 0.3j, 0.6, 0.2])
    T, dt = 0.01, 1e-3
    ref_val, ref_grad = oracle_value_and_grad(s, oracle.product_sectors(fac), T, dt, st)
    val, g = hgf.grad(S, st, T, dt, factors=fac, checkpoint_every=4)
    assert rel(val, ref_val) < FP64_TOL
    assert grad_err(g, ref_grad) < FP64_TOL


def _single_mode(s, j):
    return synth.System((s.cutoff[j],), s.detuning[j:j + 1], s.kerr[j:j + 1], np.zeros((1, 1)),
                        s.gamma1[j:j + 1], s.gamma_phi[j:j + 1], s.n_th[j:j + 1])


def test_gradient_workload_factorises(hgf):
    """The 4-mode cutoff-16 workload as the benchmark runs it (bitstring
    projector, coherent state, T = 5 us, dt = 0.1 ns, checkpoints every 100
    steps; the tiled kernel with two fast and two slow axes).  On the
    diagonal sector the generator is a sum of commuting single-mode
    generators, so J = prod_j J_j and dJ/dgamma1_j = J'_j prod_{i != j} J_i
    with single-mode oracle sensitivities (exact up to RK4's O(h^5) splitting
    term, ~1e-22 per step here).  K, chi, Delta and gamma_phi do not enter the
    diagonal sector: those 18 partials are zero."""
    w = synth.grad_c3()
    s = w.system
    st = w.states[0]
    n = 4
    announce("gradient workload (4 x 16, 5e4 steps) vs factorised oracle")
    Js, dJ = [], []
    for j in range(n):
        sj = _single_mode(s, j)
        fin, sens = oracle.evolve_sens(sj, oracle.product_sectors([w.factors[j]]), w.t_total, w.dt, nthreads=1)
        c = ("coherent", [st[1][j]])
        Js.append(oracle.expectation((16,), fin, c))
        dJ.append([oracle.expectation((16,), sp, c) for sp in sens])  # K, Delta, gamma1, gamma_phi
    J = np.prod(Js)
    P = n + n * (n - 1) // 2 + 3 * n
    ref = np.zeros(P, dtype=np.complex128)
    for j in range(n):
        ref[n + 6 + n + j] = dJ[j][2] * np.prod([Js[i] for i in range(n) if i != j])
        # the oracle's own zeros (to its rounding)
        assert max(abs(dJ[j][0]), abs(dJ[j][1]), abs(dJ[j][3])) <= 1e-14 * abs(dJ[j][2])
    val, g = hgf.grad(hgf.define_system(s), st, w.t_total, w.dt, factors=w.factors,
                      checkpoint_every=w.extra["checkpoint_every"])
    assert rel(val, J) < FP64_TOL, (val, J)
    gam = slice(n + 6 + n, n + 6 + 2 * n)
    assert grad_err(g[gam], ref[gam]) < FP64_TOL, grad_err(g[gam], ref[gam])
    zeros = np.ones(P, dtype=bool)
    zeros[gam] = False
    assert zeros.sum() == 18
    assert np.max(np.abs(g[zeros])) <= 1e-14 * np.max(np.abs(g))


@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
@pytest.mark.parametrize("cutoff,ce", [((5, 5, 5, 5), 7), ((9, 3, 7), 100), ((16,), 13), ((32, 32), 9)])
def test_gradient_on_chip_matches_launches_and_oracle(hgf, monkeypatch, dissipator, cutoff, ce):
    """Sectors of at most four axes and 1024 points run the whole gradient on
    chip (the resident integrator for the forward pass and each segment's
    recompute, one launch for each segment's reverse sweep and products,
    the next recompute beside each sweep); it agrees with the same run in
    sequence bit for bit, with the stage-launch path (HGF_RESIDENT=0) to
    rounding and with the oracle's forward sensitivities at 1e-10."""
    announce(f"gradient on chip {cutoff} ce={ce} {dissipator}")
    s = synth.random_system(cutoff, 351, scale=2.0, n_th=0.2)
    if dissipator == "secular":
        rng = np.random.default_rng(351)
        s.dissipator = "secular"
        s.n_th_levels = rng.uniform(0.0, 0.6, size=sum(c - 1 for c in cutoff))
    fac = tridiagonal_factors(cutoff, 351) if max(cutoff) <= 16 else \
        [np.diag(np.random.default_rng(352 + j).normal(size=c)) + 0j for j, c in enumerate(cutoff)]
    st = synth.coherent_state([0.5 + 0.2j, 0.7, -0.3j, 0.4][:len(cutoff)])
    T, dt = 0.03, 1e-3
    S = hgf.define_system(s)
    out = {}
    for res in ("1", "0"):
        monkeypatch.setenv("HGF_RESIDENT", res)
        out[res] = hgf.grad(S, st, T, dt, factors=fac, checkpoint_every=ce)
    monkeypatch.delenv("HGF_RESIDENT")
    # the next segment's recompute beside the sweep, or in sequence: the same bits
    monkeypatch.setenv("HGF_GRAD_OVERLAP", "0")
    seq = hgf.grad(S, st, T, dt, factors=fac, checkpoint_every=ce)
    monkeypatch.delenv("HGF_GRAD_OVERLAP")
    assert seq[0] == out["1"][0] and np.array_equal(seq[1], out["1"][1])
    assert rel(out["1"][0], out["0"][0]) < 1e-12
    assert grad_err(out["1"][1], out["0"][1]) < 1e-12
    if np.prod(cutoff) <= 1024 and max(cutoff) <= 16:
        ref_val, ref_grad = oracle_value_and_grad(s, oracle.product_sectors(fac), T, dt, st)
        assert rel(out["1"][0], ref_val) < FP64_TOL
        assert grad_err(out["1"][1], ref_grad) < FP64_TOL


def test_small_gradient_workload_matches_stored_oracle(hgf):
    """The small off-diagonal gradient workload of the benchmark (4 Kerr
    modes, cutoff 5, product of quadratures, 2,000 steps, on chip) against
    the oracle's value and sensitivities stored by tests/golden/make_golden.py."""
    import json
    import os
    announce("small gradient workload vs stored oracle")
    w = synth.grad_c3b(cutoff=5, t_total=0.02, dt=1e-5)
    with open(os.path.join(os.path.dirname(__file__), "golden", "small_gradient.json")) as fh:
        ref = json.load(fh)
    assert ref["steps"] == w.n_steps
    val, g = hgf.grad(hgf.define_system(w.system), w.states[0], w.t_total, w.dt, factors=w.factors,
                      checkpoint_every=100)
    assert rel(val, complex(*ref["value"])) < FP64_TOL
    assert grad_err(g, np.array([complex(*x) for x in ref["grad"]])) < FP64_TOL


def test_gradient_thirteen_modes_products(hgf, monkeypatch):
    """13 modes at cutoff 2 with a bitstring projector (one 8,192-point
    sector): the parameter products run once per segment in chunks of four
    modes (0-3, 4-7, 8-11, 12), and step by step in one pass when the stages
    are not stored (HGF_GRAD_STORE=0); both give the same bits, and the
    gamma1 partials match factorised single-mode oracle sensitivities while
    the other 117 partials (K, chi, Delta, gamma_phi) are zero on the
    diagonal sector."""
    n = 13
    cutoff = (2,) * n
    announce("gradient, 13 modes, segment products vs per step vs factorised oracle")
    s = synth.random_system(cutoff, 341, scale=2.0, n_th=0.3)
    rng = np.random.default_rng(341)
    bits = rng.integers(0, 2, size=n)
    fac = synth.projector_factors(cutoff, bits)
    alpha = rng.uniform(0.2, 0.8, size=n) * np.exp(1j * rng.uniform(0, 2 * np.pi, size=n))
    st = synth.coherent_state(list(alpha))
    T, dt = 0.05, 1e-3
    S = hgf.define_system(s)
    out = []
    for store in (None, "0"):
        if store is None:
            monkeypatch.delenv("HGF_GRAD_STORE", raising=False)
        else:
            monkeypatch.setenv("HGF_GRAD_STORE", store)
        out.append(hgf.grad(S, st, T, dt, factors=fac, checkpoint_every=7))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])
    val, g = out[0]
    Js, dg = [], []
    for j in range(n):
        fin, sens = oracle.evolve_sens(_single_mode(s, j), oracle.product_sectors([fac[j]]), T, dt, nthreads=1)
        c = ("coherent", [alpha[j]])
        Js.append(oracle.expectation((2,), fin, c))
        dg.append(oracle.expectation((2,), sens[2], c))  # single-mode parameters: K, Delta, gamma1, gamma_phi
    P = n + n * (n - 1) // 2 + 3 * n
    assert len(g) == P
    ref = np.zeros(P, dtype=np.complex128)
    gam = slice(n + n * (n - 1) // 2 + n, n + n * (n - 1) // 2 + 2 * n)
    ref[gam] = [dg[j] * np.prod([Js[i] for i in range(n) if i != j]) for j in range(n)]
    assert rel(val, np.prod(Js)) < FP64_TOL
    assert grad_err(g[gam], ref[gam]) < FP64_TOL, grad_err(g[gam], ref[gam])
    zeros = np.ones(P, dtype=bool)
    zeros[gam] = False
    assert np.max(np.abs(g[zeros])) <= 1e-14 * np.max(np.abs(g))


def test_gradient_matches_central_differences(hgf):
    """dJ/dtheta from the reverse sweep against central differences of the
    forward evolve (FP64), h_i = 1e-6 max(|theta_i|, 1), on the slow-axis
    system with off-diagonal sectors (every parameter enters)."""
    announce("gradient vs central differences")
    s = slow_axis_system("lindblad", 321)
    fac = tridiagonal_factors(s.cutoff, 321)
    st = synth.coherent_state([0.6 + 0.2j, 0.9, -0.4j, 0.5])
    T, dt = 0.02, 1e-3
    val, g = hgf.grad(hgf.define_system(s), st, T, dt, factors=fac, checkpoint_every=5)
    theta = hgf.params_vector(s)
    n = 4

    def J(th):
        t = s.copy()
        t.kerr[:] = th[:n]
        q = n
        for i in range(n):
            for j in range(i + 1, n):
                t.cross_kerr[i, j] = t.cross_kerr[j, i] = th[q]
                q += 1
        t.detuning[:] = th[q:q + n]
        t.gamma1[:] = th[q + n:q + 2 * n]
        t.gamma_phi[:] = th[q + 2 * n:q + 3 * n]
        op = hgf.map_operator(hgf.define_system(t), factors=fac, precision="fp64")
        hgf.evolve(op, T, dt)
        return hgf.expectation(op, st)

    assert rel(J(theta), val) < 1e-12
    fd = np.zeros(len(theta), dtype=np.complex128)
    for p in range(len(theta)):
        h = 1e-6 * max(abs(theta[p]), 1.0)
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd[p] = (J(tp) - J(tm)) / (2 * h)
    assert grad_err(g, fd) < 1e-6, grad_err(g, fd)


def test_autograd_function(hgf):
    """expectation_of_params: value and gradient on the device of theta, the
    gradient equal to hgf_grad's and to central differences of the value;
    a forward without a gradient request runs the plain evolve; a
    non-Hermitian observable is refused."""
    import torch

    from paper_2203_05526_amd.autograd import expectation_of_params
    announce("autograd.Function")
    cutoff = (4, 5)
    s = synth.random_system(cutoff, 331, scale=2.0, n_th=0.2)
    fac = tridiagonal_factors(cutoff, 331)
    st = synth.coherent_state([0.6 + 0.2j, 0.8])
    spec = {"cutoff": cutoff, "n_th": s.n_th, "state": st, "t_total": 0.05, "dt": 1e-3, "factors": fac,
            "checkpoint_every": 10}
    theta = torch.tensor(hgf.params_vector(s), dtype=torch.float64, device="cuda", requires_grad=True)
    J = expectation_of_params(theta, spec)
    assert J.device == theta.device and J.dtype == torch.float64
    (gr,) = torch.autograd.grad(J, theta)
    assert gr.device == theta.device
    val, g = hgf.grad(hgf.define_system(s), st, 0.05, 1e-3, factors=fac, checkpoint_every=10)
    assert J.item() == val.real
    assert np.array_equal(gr.cpu().numpy(), g.real)
    with torch.no_grad():
        J0 = expectation_of_params(theta, spec)
        assert abs(float(J0) - val.real) < 1e-12 * abs(val.real)
        fd = []
        for p in range(theta.numel()):
            h = 1e-6 * max(abs(float(theta[p])), 1.0)
            e = torch.zeros_like(theta)
            e[p] = h
            fd.append((float(expectation_of_params(theta + e, spec)) - float(expectation_of_params(theta - e, spec)))
                      / (2 * h))
    fd = np.array(fd)
    assert np.max(np.abs(gr.cpu().numpy() - fd)) / np.max(np.abs(fd)) < 1e-6
    # a non-Hermitian observable has a complex expectation value
    bad = dict(spec, factors=[np.triu(f) for f in fac])
    with pytest.raises(ValueError):
        expectation_of_params(theta, bad)
