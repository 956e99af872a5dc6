"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check uses a closed form,
an invariant, an independent dense construction (Kronecker-product
superoperator + scipy expm), or the exact polynomial of classical RK4.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from tests import pinlib


def small_system(seed=0, cutoff=(3, 4), **kw):
    return synth.random_system(cutoff, seed, **kw)


# --------------------------------------------------------------- invariants

def test_identity_is_stationary(oracle_lib):
    """Adjoint master equation, Eq. (3): L^dagger(I) = 0 (trace preservation)."""
    s = small_system(1, (4, 3, 3))
    ops = {(0, 0, 0): np.ones(s.cutoff, dtype=np.complex128)}
    r = oracle.rhs(s, ops)
    assert np.max(np.abs(r[(0, 0, 0)])) < 1e-12
    out = oracle.evolve(s, ops, 0.2, 1e-3)
    assert np.max(np.abs(out[(0, 0, 0)] - 1.0)) < 1e-12


def test_hermiticity_preserved(oracle_lib):
    """Eq. (3) maps Hermitian operators to Hermitian operators: sector -d is the
    conjugate transpose of sector d at all times."""
    s = small_system(2, (3, 4))
    rng = np.random.default_rng(5)
    dim = 12
    M = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    M = M + M.conj().T
    ops = oracle.sectors_from_dense(s.cutoff, M)
    out = oracle.evolve(s, ops, 0.3, 1e-3)
    Mt = oracle.dense_from_sectors(s.cutoff, out)
    assert np.max(np.abs(Mt - Mt.conj().T)) < 1e-13 * np.max(np.abs(Mt))
    assert pinlib.rel(Mt, M) > 1e-3  # it did evolve


def test_sectors_do_not_leak(oracle_lib):
    """Every term of the master equation shifts k and l together, so the full
    operator evolved as one object equals its sectors evolved separately."""
    s = small_system(3, (3, 3))
    rng = np.random.default_rng(6)
    M = rng.normal(size=(9, 9)) + 1j * rng.normal(size=(9, 9))
    ops = oracle.sectors_from_dense(s.cutoff, M)
    whole = oracle.dense_from_sectors(s.cutoff, oracle.evolve(s, ops, 0.1, 1e-3))
    parts = np.zeros_like(whole)
    for d, box in ops.items():
        parts += oracle.dense_from_sectors(s.cutoff, oracle.evolve(s, {d: box}, 0.1, 1e-3))
    assert pinlib.rel(parts, whole) < 1e-14


# ------------------------------------------------------- dense expm pin

@pytest.mark.parametrize("cutoff,seed", [((3, 3), 11), ((4,), 12), ((2, 3, 2), 13)])
def test_against_dense_superoperator_expm(oracle_lib, cutoff, seed):
    """The oracle's RK4 result equals exp(S T) applied to A(0), with S the
    adjoint Liouvillian built from Kronecker products, within RK4's error."""
    s = small_system(seed, cutoff, n_th=0.3)
    rng = np.random.default_rng(seed)
    dim = int(np.prod(cutoff))
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    ops = oracle.sectors_from_dense(cutoff, A0)
    T, dt = 0.5, 1e-3
    got = oracle.dense_from_sectors(cutoff, oracle.evolve(s, ops, T, dt))
    ref = pinlib.expm_evolve(s, A0, T)
    assert pinlib.rel(got, ref) < 1e-10


def test_rk4_converges_at_fourth_order(oracle_lib):
    """Halving dt cuts the error against the exact exponential ~16x
    (the reference-method recipe of the paper uses half the time step)."""
    s = small_system(21, (3, 3), scale=20.0, n_th=0.2)
    rng = np.random.default_rng(21)
    A0 = rng.normal(size=(9, 9)) + 1j * rng.normal(size=(9, 9))
    ops = oracle.sectors_from_dense(s.cutoff, A0)
    T = 0.2
    ref = pinlib.expm_evolve(s, A0, T)
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        got = oracle.dense_from_sectors(s.cutoff, oracle.evolve(s, ops, T, dt))
        errs.append(pinlib.rel(got, ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


# ------------------------------------------------------- closed forms

def test_no_jumps_matches_rk4_polynomial(oracle_lib):
    """With gamma1 = 0 only the diagonal rates remain: each element gets
    R(lambda h)^M with R the RK4 stability polynomial and
    lambda = i(E_k - E_l) - gamma_phi (k - l)^2, exactly (up to rounding)."""
    s = small_system(31, (4, 3))
    s.gamma1[:] = 0.0
    rng = np.random.default_rng(31)
    A0 = rng.normal(size=(12, 12)) + 1j * rng.normal(size=(12, 12))
    ops = oracle.sectors_from_dense(s.cutoff, A0)
    h, M = 2e-3, 150
    got = oracle.dense_from_sectors(s.cutoff, oracle.evolve_steps(s, ops, M, h))
    ref = np.zeros_like(A0)
    for ki in range(12):
        k = np.unravel_index(ki, s.cutoff)
        for li in range(12):
            l = np.unravel_index(li, s.cutoff)

            def E(v):
                e = sum(s.detuning[j] * v[j] + 0.5 * s.kerr[j] * v[j] * (v[j] - 1) for j in range(2))
                return e + s.cross_kerr[0, 1] * v[0] * v[1]

            lam = 1j * (E(k) - E(l)) - sum(s.gamma_phi[j] * (k[j] - l[j]) ** 2 for j in range(2))
            ref[ki, li] = pinlib.rk4_polynomial(lam * h) ** M * A0[ki, li]
    assert pinlib.rel(got, ref) < 1e-13


def test_number_operator_closed_form(oracle_lib):
    """<a^+a>(t) = e^{-gamma t} <a^+a>(0) + n_th (1 - e^{-gamma t}) for a damped
    mode with thermal bath (the closed form the damped oscillator obeys)."""
    nc = 24
    g, nth = 0.7, 0.05
    s = synth.System((nc,), np.array([0.3]), np.array([-4.0]), np.zeros((1, 1)),
                     np.array([g]), np.array([0.4]), np.array([nth]))
    ops = {(0,): np.arange(nc, dtype=np.complex128)}
    T = 1.3
    out = oracle.evolve(s, ops, T, 1e-3)
    for alpha in (0.0, 0.8, 1.2 + 0.5j):
        got = oracle.expectation(s.cutoff, out, ("coherent", [alpha])).real
        ref = math.exp(-g * T) * abs(alpha) ** 2 + nth * (1 - math.exp(-g * T))
        assert abs(got - ref) < 1e-11


def test_single_mode_zero_temperature_projector(oracle_lib):
    """n_th = 0: <n| P1(T) |n> = n e^{-gT} (1 - e^{-gT})^{n-1} (binomial
    thinning of a Fock state) and, for a coherent state, s e^{-s} with
    s = |alpha|^2 e^{-gT} (Poisson thinning).  Kerr and dephasing do not
    change populations."""
    nc = 30
    g = 0.02
    s = synth.System((nc,), np.array([0.0]), np.array([synth.TWO_PI * -200.0]), np.zeros((1, 1)),
                     np.array([g]), np.array([0.01]), np.array([0.0]))
    ops = oracle.product_sectors(synth.projector_factors((nc,), (1,)))
    T = 10.0
    out = oracle.evolve(s, ops, T, 1e-2)
    e = math.exp(-g * T)
    for n in range(0, 6):
        got = oracle.expectation(s.cutoff, out, ("fock", [n])).real
        ref = n * e * (1 - e) ** (n - 1) if n >= 1 else 0.0
        assert abs(got - ref) < 1e-12
    a = 1.1
    got = oracle.expectation(s.cutoff, out, ("coherent", [a])).real
    sv = a * a * e
    assert abs(got - sv * math.exp(-sv)) < 1e-12


def test_single_mode_thermal_projector(oracle_lib):
    """n_th > 0, coherent state: the damped state is a displaced thermal state
    with amplitude beta = alpha e^{-gT/2} and occupation nt = n_th (1 - e^{-gT});
    its |1> population is e^{-|b|^2/(1+nt)} [nt/(1+nt)^2 + |b|^2/(1+nt)^3]."""
    nc = 30
    g, nth = 0.5, 0.2
    s = synth.System((nc,), np.array([0.7]), np.array([-3.0]), np.zeros((1, 1)),
                     np.array([g]), np.array([0.3]), np.array([nth]))
    ops = oracle.product_sectors(synth.projector_factors((nc,), (1,)))
    T = 1.5
    out = oracle.evolve(s, ops, T, 1e-3)
    for alpha in (0.6, 1.0 - 0.4j):
        got = oracle.expectation(s.cutoff, out, ("coherent", [alpha])).real
        b2 = abs(alpha) ** 2 * math.exp(-g * T)
        nt = nth * (1 - math.exp(-g * T))
        ref = math.exp(-b2 / (1 + nt)) * (nt / (1 + nt) ** 2 + b2 / (1 + nt) ** 3)
        assert abs(got - ref) < 1e-11


# ------------------------------------------------------- structure

def test_product_observable_factorises(oracle_lib):
    """On the diagonal sector the generator is a sum of commuting single-mode
    generators, so a product observable in a product state gives the product
    of single-mode expectation values (up to RK4's O(h^5) splitting term)."""
    s = small_system(41, (5, 4, 6), n_th=0.1)
    bits = (1, 0, 2)
    alpha = (0.7, 1.1j, 0.5 - 0.2j)
    ops = oracle.product_sectors(synth.projector_factors(s.cutoff, bits))
    out = oracle.evolve(s, ops, 1.0, 1e-3)
    J = oracle.expectation(s.cutoff, out, ("coherent", alpha))
    prod = 1.0
    for j in range(3):
        sj = synth.System((s.cutoff[j],), s.detuning[j:j + 1], s.kerr[j:j + 1], np.zeros((1, 1)),
                          s.gamma1[j:j + 1], s.gamma_phi[j:j + 1], s.n_th[j:j + 1])
        oj = oracle.evolve(sj, oracle.product_sectors([synth.projector_factors(
            (s.cutoff[j],), (bits[j],))[0]]), 1.0, 1e-3)
        prod *= oracle.expectation(sj.cutoff, oj, ("coherent", [alpha[j]]))
    assert abs(J - prod) < 1e-12 * abs(prod)


def test_diagonal_sector_ignores_hamiltonian_and_dephasing(oracle_lib):
    s = small_system(51, (4, 5), n_th=0.1)
    ops = oracle.product_sectors(synth.projector_factors(s.cutoff, (1, 2)))
    a = oracle.evolve(s, ops, 0.7, 1e-3)
    s2 = s.copy()
    s2.kerr[:] = 0
    s2.detuning[:] = 0
    s2.cross_kerr[:] = 0
    s2.gamma_phi[:] = 0
    b = oracle.evolve(s2, ops, 0.7, 1e-3)
    assert pinlib.rel(a[(0, 0)], b[(0, 0)]) < 1e-14


# ------------------------------------------------------- coefficient maps

@pytest.mark.parametrize("nc", [1, 4, 7])
def test_coefficient_maps(nc):
    """Eq. (6) and the inner sum of Eq. (11) are inverse maps; the basis of
    Eqs. (7)-(8) with r = 1 is T_{k,l} = sqrt(k! l!) |k><l| on the truncated
    space, so g_{k,l} = <k|A|l> / sqrt(k! l!)."""
    f = synth.random_normal_coeffs(nc, 7 + nc)
    g = oracle.g_from_f(f)
    assert np.max(np.abs(oracle.f_from_g(g) - f)) < 1e-12 * np.max(np.abs(f))
    A = oracle.number_from_normal(f)
    scale = np.array([[math.sqrt(math.factorial(k) * math.factorial(l)) for l in range(nc)]
                      for k in range(nc)])
    assert np.max(np.abs(g * scale - A)) < 1e-11 * np.max(np.abs(A))
    for k in range(nc):
        for l in range(nc):
            T = oracle.basis_T(k, l, nc)
            ref = np.zeros((nc, nc))
            ref[k, l] = scale[k, l]
            assert np.max(np.abs(T - ref)) < 1e-10 * scale[k, l]
    # Eq. (7): A = sum g_kl T_kl
    recon = sum(g[k, l] * oracle.basis_T(k, l, nc) for k in range(nc) for l in range(nc))
    assert np.max(np.abs(recon - A)) < 1e-10 * max(1.0, np.max(np.abs(A)))


@pytest.mark.parametrize("cutoff,seed", [((4, 3), 71), ((3, 5, 2), 72)])
def test_generating_coefficients_and_sector_grid(cutoff, seed):
    """The oracle's coefficient map (number-basis sectors -> g of Eqs. (6)-(8))
    and its sector slicing (m = min(k, l), extent Nc_j - |d_j|), checked
    against a product operator built from normal-ordered per-mode
    coefficients: Eq. (2) by matrix products gives the number-basis operator,
    Eq. (6) by its sum gives every g_{k,l} = prod_j g_j[k_j, l_j], and each
    sector grid point m is compared with the product at k = m + u, l = m + v
    (u_j = max(0, -d_j), v_j = max(0, d_j)), looped over explicitly."""
    import itertools
    fs = [synth.random_normal_coeffs(nc, seed + j) for j, nc in enumerate(cutoff)]
    gs = [oracle.g_from_f(f) for f in fs]
    ops = oracle.product_sectors([oracle.number_from_normal(f) for f in fs])
    gco = oracle.generating_coefficients(cutoff, ops)
    assert set(gco) == set(ops)
    assert any(min(d) < 0 for d in ops) and any(max(d) > 0 for d in ops)
    scale = max(float(np.max(np.abs(g))) for g in gs) ** len(cutoff)
    for d, box in gco.items():
        grid = oracle.sector_grid(cutoff, d, box)
        ext = tuple(nc - abs(dj) for nc, dj in zip(cutoff, d))
        assert grid.shape == ext
        for m in itertools.product(*[range(e) for e in ext]):
            k = [mj + max(0, -dj) for mj, dj in zip(m, d)]
            l = [mj + max(0, dj) for mj, dj in zip(m, d)]
            ref = np.prod([g[kj, lj] for g, kj, lj in zip(gs, k, l)])
            assert abs(grid[m] - ref) < 1e-12 * scale, (d, m)


def test_sector_grid_hand_sliced():
    """One sector sliced by hand: cutoff (3, 4), d = (1, -2) keeps k_0 in
    {0, 1} (l_0 = k_0 + 1 < 3) and k_1 in {2, 3} (l_1 = k_1 - 2 >= 0)."""
    box = np.arange(12, dtype=np.complex128).reshape(3, 4) * (1 + 0.5j)
    grid = oracle.sector_grid((3, 4), (1, -2), box)
    assert grid.shape == (2, 2)
    assert np.array_equal(grid, np.array([[box[0, 2], box[0, 3]], [box[1, 2], box[1, 3]]]))
    assert np.array_equal(oracle.sector_grid((3, 4), (0, 0), box), box)
    assert oracle.sector_grid((3, 4), (-2, 3), box).shape == (1, 1)
    assert oracle.sector_grid((3, 4), (-2, 3), box)[0, 0] == box[2, 0]


# ------------------------------------------------------- sensitivities

@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
def test_sensitivities_match_finite_differences(oracle_lib, dissipator):
    """Forward sensitivities of the discrete RK4 map against central finite
    differences of the oracle's own expectation value."""
    s = small_system(61, (3, 4), n_th=0.2)
    if dissipator == "secular":
        s = with_secular(s, np.random.default_rng(62))
    rng = np.random.default_rng(61)
    A0 = rng.normal(size=(12, 12)) + 1j * rng.normal(size=(12, 12))
    A0 = A0 + A0.conj().T
    ops = oracle.sectors_from_dense(s.cutoff, A0)
    state = ("coherent", (0.6 + 0.2j, 0.9))
    T, dt = 0.2, 2e-3
    _, sens = oracle.evolve_sens(s, ops, T, dt)
    n = s.n_modes
    names = []
    for j in range(n):
        names.append(("kerr", j))
    for i in range(n):
        for j in range(i + 1, n):
            names.append(("chi", (i, j)))
    for j in range(n):
        names.append(("detuning", j))
    for j in range(n):
        names.append(("gamma1", j))
    for j in range(n):
        names.append(("gamma_phi", j))
    assert len(names) == oracle.num_params(n) == len(sens)
    for p, (field, idx) in enumerate(names):
        def J(delta):
            s2 = s.copy()
            if field == "chi":
                s2.cross_kerr[idx] += delta
                s2.cross_kerr[idx[::-1]] += delta
            else:
                getattr(s2, field)[idx] += delta
            return oracle.expectation(s2.cutoff, oracle.evolve(s2, ops, T, dt), state)

        h = 1e-5
        fd = (J(h) - J(-h)) / (2 * h)
        an = oracle.expectation(s.cutoff, sens[p], state)
        assert abs(an - fd) < 1e-7 * max(1.0, abs(fd)), (field, idx, an, fd)


# ------------------------------------------------------- secular dissipator (Eq. (15))

def with_secular(s, rng, constant=False):
    """The same system with the secular dissipator; per-transition bath
    occupations drawn at random (or n_th for every transition)."""
    s2 = s.copy()
    s2.dissipator = "secular"
    if not constant:
        s2.n_th_levels = rng.uniform(0.0, 0.5, size=sum(c - 1 for c in s.cutoff))
    return s2


@pytest.mark.parametrize("cutoff,seed", [((3, 3), 91), ((5,), 92), ((2, 3, 2), 93)])
def test_secular_against_dense_superoperator_expm(oracle_lib, cutoff, seed):
    """Secular form: the oracle's element-wise right-hand side integrated with
    RK4 equals exp(S T) with S built from the paper's transition jump
    operators |n><n+1|, |n+1><n| as Kronecker products."""
    rng = np.random.default_rng(seed)
    s = with_secular(small_system(seed, cutoff, n_th=0.2), rng)
    dim = int(np.prod(cutoff))
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    ops = oracle.sectors_from_dense(cutoff, A0)
    T, dt = 0.5, 1e-3
    got = oracle.dense_from_sectors(cutoff, oracle.evolve(s, ops, T, dt))
    ref = pinlib.expm_evolve(s, A0, T)
    assert pinlib.rel(got, ref) < 1e-10


def test_secular_equals_lindblad_on_the_diagonal_sector(oracle_lib):
    """With one bath occupation for every transition the secular and Lindblad
    forms agree on populations (the diagonal sector) and differ on coherences,
    where the secular form has no jump terms."""
    s = small_system(94, (4, 3), n_th=0.3)
    sec = with_secular(s, None, constant=True)
    rng = np.random.default_rng(94)
    diag = {(0, 0): rng.normal(size=s.cutoff) + 1j * rng.normal(size=s.cutoff)}
    assert pinlib.rel(oracle.rhs(sec, diag)[(0, 0)], oracle.rhs(s, diag)[(0, 0)]) < 1e-14
    off = {(1, 0): rng.normal(size=s.cutoff) + 1j * rng.normal(size=s.cutoff)}
    assert pinlib.rel(oracle.rhs(sec, off)[(1, 0)], oracle.rhs(s, off)[(1, 0)]) > 1e-3


def test_secular_identity_and_thermal_state_are_stationary(oracle_lib):
    """Secular form with level-dependent bath occupations: the identity is a
    fixed point of the adjoint equation (trace preservation), and the state
    with detailed-balance populations p_{n+1} / p_n = nbar_n / (nbar_n + 1)
    per mode is stationary: <psi| L^+(A) |psi>-weights vanish for every A."""
    rng = np.random.default_rng(95)
    s = with_secular(small_system(95, (4, 5), n_th=0.2), rng)
    ones = {(0, 0): np.ones(s.cutoff, dtype=np.complex128)}
    assert np.max(np.abs(oracle.rhs(s, ones)[(0, 0)])) < 1e-13
    # thermal populations, a product over modes
    pops = []
    for j, nc in enumerate(s.cutoff):
        nb = pinlib.transition_occupations(s, j)
        p = np.ones(nc)
        for t in range(nc - 1):
            p[t + 1] = p[t] * nb[t] / (nb[t] + 1.0)
        pops.append(p / p.sum())
    rho = np.einsum("i,j->ij", *pops)
    dim = int(np.prod(s.cutoff))
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    dA = oracle.dense_from_sectors(s.cutoff, oracle.rhs(s, oracle.sectors_from_dense(s.cutoff, A0)))
    rate = np.sum(rho.reshape(-1) * np.diag(dA))
    assert abs(rate) < 1e-12 * np.max(np.abs(dA))
    # a non-thermal population distribution is not stationary
    assert abs(np.sum(np.ones(dim) / dim * np.diag(dA))) > 1e-6


def test_secular_coherence_decays_without_feeding(oracle_lib):
    """Zero-temperature secular form, one mode: a coherence |k><l| (k != l)
    evolves into a multiple of itself, exp((i (E_k - E_l) - gamma1 (k + l) / 2
    - gamma_phi (k - l)^2) t) in the continuous limit (the Lindblad form would
    also feed |k+1><l+1|); checked against RK4's polynomial of that rate."""
    s = synth.System((6,), np.array([0.7]), np.array([-2.0]), np.zeros((1, 1)), np.array([0.9]),
                     np.array([0.3]), np.array([0.0]), "secular")
    T, dt = 0.3, 1e-3
    steps = oracle.n_steps(T, dt)
    for k, l in ((3, 1), (0, 4), (5, 2)):
        A = np.zeros((6, 6), dtype=np.complex128)
        A[k, l] = 1.0
        out = oracle.dense_from_sectors((6,), oracle.evolve(s, oracle.sectors_from_dense((6,), A), T, dt))
        E = lambda m: 0.7 * m + 0.5 * (-2.0) * m * (m - 1)
        lam = 1j * (E(k) - E(l)) - 0.9 * (k + l) / 2 - 0.3 * (k - l) ** 2
        expect = pinlib.rk4_polynomial(lam * dt) ** steps
        assert abs(out[k, l] - expect) < 1e-13
        out[k, l] = 0.0
        assert np.max(np.abs(out)) == 0.0


# --------------------------------------------------------------- integrating-factor RK4

def test_lawson_exact_without_jumps(oracle_lib):
    """With no emission or absorption (gamma1 = 0) the right-hand side of
    Eq. (3) is diagonal element by element, D[k,l] = i(E_k - E_l) -
    sum_j gamma_phi_j (k_j - l_j)^2, and the integrating-factor step takes it
    exactly: A(T) = exp(D T) A(0) whatever the step size."""
    cutoff = (4, 3)
    s = small_system(120, cutoff, scale=40.0)
    s.gamma1 = np.zeros(2)
    rng = np.random.default_rng(120)
    dim = 12
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    E = np.real(np.diag(pinlib.hamiltonian(s)))
    occ = np.array([np.unravel_index(i, cutoff) for i in range(dim)])
    D = 1j * (E[:, None] - E[None, :])
    for j in range(2):
        D -= s.gamma_phi[j] * (occ[:, None, j] - occ[None, :, j]) ** 2
    T = 0.1
    got = oracle.dense_from_sectors(cutoff, oracle.evolve_lawson(s, oracle.sectors_from_dense(cutoff, A0), T, 0.05))
    assert pinlib.rel(got, np.exp(D * T) * A0) < 1e-13
    # classical RK4 at this step is far off (|D| dt ~ 10)
    rk = oracle.dense_from_sectors(cutoff, oracle.evolve(s, oracle.sectors_from_dense(cutoff, A0), T, 0.05))
    assert pinlib.rel(rk, np.exp(D * T) * A0) > 1.0


@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
def test_lawson_converges_to_expm_at_fourth_order(oracle_lib, dissipator):
    """Stiff Kerr phases with weak jumps: against exp(S T) of the Kronecker
    superoperator the integrating-factor result converges at fourth order
    (error / 16 per halving of dt) and at a step where classical RK4 is
    unstable it is already accurate."""
    cutoff = (5, 4)
    rng = np.random.default_rng(121)
    s = small_system(121, cutoff, scale=1.0, n_th=0.3)
    s.kerr = np.array([-300.0, -250.0])
    s.cross_kerr = np.array([[0.0, -20.0], [-20.0, 0.0]])
    if dissipator == "secular":
        s = with_secular(s, rng)
    dim = 20
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    ops = oracle.sectors_from_dense(cutoff, A0)
    T = 0.2
    ref = pinlib.expm_evolve(s, A0, T)
    # the jump terms oscillate in the interaction picture at the neighbours'
    # phase difference (K d ~ 300 rad/us): the fourth-order regime starts at
    # a step of a few thousandths of a microsecond
    errs = [pinlib.rel(oracle.dense_from_sectors(cutoff, oracle.evolve_lawson(s, ops, T, dt)), ref)
            for dt in (0.002, 0.001, 0.0005)]
    assert errs[0] < 1e-5
    assert 12.0 < errs[0] / errs[1] < 20.0 and 12.0 < errs[1] / errs[2] < 20.0
    rk = oracle.dense_from_sectors(cutoff, oracle.evolve(s, ops, T, 0.002))
    assert not np.all(np.isfinite(rk)) or pinlib.rel(rk, ref) > 1.0


# --------------------------------------------------------------- driven, exchange-coupled network (full matrix)

def network(seed, cutoff, dissipator="lindblad"):
    rng = np.random.default_rng(seed)
    s = small_system(seed, cutoff, scale=2.0, n_th=0.2)
    n = len(cutoff)
    s.drive = rng.normal(size=n) * 3.0 + 1j * rng.normal(size=n) * 3.0
    J = np.zeros((n, n))
    for i in range(n - 1):
        J[i, i + 1] = J[i + 1, i] = rng.uniform(1.0, 4.0)
    s.exchange = J
    if dissipator == "secular":
        s = with_secular(s, rng)
    return s


@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
@pytest.mark.parametrize("cutoff,seed", [((3, 4), 130), ((2, 3, 2), 131), ((6,), 132)])
def test_network_against_dense_superoperator_expm(oracle_lib, cutoff, seed, dissipator):
    """Drive Omega_j a_j^+ + h.c. and exchange J_ij (a_i^+ a_j + h.c.) (Eq. (16)
    in the drive frame): the oracle's element-wise full-matrix right-hand side,
    integrated with RK4, equals exp(S T) of the Kronecker superoperator."""
    s = network(seed, cutoff, dissipator)
    dim = int(np.prod(cutoff))
    rng = np.random.default_rng(seed)
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    T, dt = 0.3, 1.25e-4
    got = oracle.evolve_full(s, A0, T, dt)
    assert pinlib.rel(got, pinlib.expm_evolve(s, A0, T)) < 1e-10  # RK4 error <= 5e-12 at this step
    # one right-hand side against the superoperator itself
    assert pinlib.rel(oracle.rhs_full(s, A0), (pinlib.adjoint_superop(s) @ A0.reshape(-1)).reshape(A0.shape)) < 1e-13


def test_network_identity_stationary_and_hermiticity(oracle_lib):
    """Eq. (3) with the network Hamiltonian: L^+(I) = 0 and A = A^+ stays
    Hermitian; the sector oracle refuses coupled sectors."""
    cutoff = (3, 3, 2)
    s = network(133, cutoff)
    dim = 18
    assert np.max(np.abs(oracle.rhs_full(s, np.eye(dim)))) < 1e-12
    rng = np.random.default_rng(133)
    M = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    M = M + M.conj().T
    out = oracle.evolve_full(s, M, 0.2, 1e-3)
    assert np.max(np.abs(out - out.conj().T)) < 1e-12 * np.max(np.abs(out))
    with pytest.raises(ValueError):
        oracle.evolve(s, oracle.sectors_from_dense(cutoff, M), 0.1, 1e-3)


def _annihilation(nc):
    return np.diag(np.sqrt(np.arange(1, nc, dtype=float)), 1).astype(np.complex128)


def test_network_driven_damped_mode_closed_form(oracle_lib):
    """A resonantly driven, damped mode (Eq. (16), one mode, H = Delta n +
    Omega a^+ + conj(Omega) a, emission at gamma1): the Heisenberg equation
    d<a>/dt = -(gamma1/2 + i Delta) <a> - i Omega gives, from the vacuum,
    <a>(t) = -i Omega / (gamma1/2 + i Delta) (1 - exp(-(gamma1/2 + i Delta) t)).
    Checked on a(T) from the oracle's full-matrix RK4 (cutoff 14: the field
    stays near 0.17, the truncation is far below the tolerance)."""
    nc, delta, g1, om = 14, 2.0, 1.0, 0.3 + 0.2j
    s = synth.System((nc,), np.array([delta]), np.zeros(1), np.zeros((1, 1)), np.array([g1]), np.zeros(1),
                     np.zeros(1))
    s.drive = np.array([om])
    s.exchange = np.zeros((1, 1))
    T, dt = 2.0, 1e-3
    aT = oracle.evolve_full(s, _annihilation(nc), T, dt)
    z = g1 / 2 + 1j * delta
    want = -1j * om / z * (1 - np.exp(-z * T))
    assert abs(aT[0, 0] - want) < 1e-10 * abs(want)
    # <a^+ a> in the same state: |<a>|^2 (the state stays coherent)
    n_op = _annihilation(nc).conj().T @ _annihilation(nc)
    nT = oracle.evolve_full(s, n_op, T, dt)
    assert abs(nT[0, 0] - abs(want) ** 2) < 1e-10 * abs(want) ** 2


def test_network_exchange_swaps_a_coherent_field(oracle_lib):
    """Two lossless modes coupled by exchange J (a_1^+ a_2 + a_2^+ a_1): the
    Heisenberg equations da_1/dt = -i J a_2, da_2/dt = -i J a_1 give, for the
    state |alpha> (x) |0>, <a_1>(t) = alpha cos(J t) and <a_2>(t) =
    -i alpha sin(J t).  The excitation number is conserved, so at cutoff 12 and
    |alpha| = 0.4 the truncation is negligible."""
    nc, J, alpha = 12, 3.0, 0.4 - 0.1j
    s = synth.System((nc, nc), np.zeros(2), np.zeros(2), np.zeros((2, 2)), np.zeros(2), np.zeros(2), np.zeros(2))
    s.drive = np.zeros(2, dtype=np.complex128)
    s.exchange = np.array([[0.0, J], [J, 0.0]])
    T, dt = 0.7, 5e-4
    a = _annihilation(nc)
    eye = np.eye(nc, dtype=np.complex128)
    c = np.kron(*oracle.state_amplitudes((nc, nc), synth.coherent_state([alpha, 0.0])))
    for op, want in ((np.kron(a, eye), alpha * np.cos(J * T)), (np.kron(eye, a), -1j * alpha * np.sin(J * T))):
        opT = oracle.evolve_full(s, op, T, dt)
        got = np.conj(c) @ opT @ c
        assert abs(got - want) < 1e-9 * abs(alpha), (got, want)


# --------------------------------------------- separated form (Eqs. (9a)-(9c))

def _product(factors):
    A = np.ones((1, 1), dtype=np.complex128)
    for f in factors:
        A = np.kron(A, f)
    return A


@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
@pytest.mark.parametrize("cutoff,seed", [((4,), 140), ((3, 3), 141)])
def test_separated_form_converges_to_expm(oracle_lib, cutoff, seed, dissipator):
    """G = Gx Gy + R per initial monomial (Eq. (10)), with R on the whole
    (k, l) box, is exact in continuous time: its RK4 result converges to
    exp(S T) of the independently built Kronecker superoperator at fourth
    order (error / 16 per halving of the step), for a driven, exchange-coupled
    network with dephasing and a random operator over all (k, l)."""
    s = network(seed, cutoff, dissipator)
    s.gamma_phi = np.full(len(cutoff), 0.4)
    dim = int(np.prod(cutoff))
    rng = np.random.default_rng(seed)
    A0 = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    monos = oracle.monomials(s, A0)
    assert len(monos) == dim * dim
    T = 0.3
    ref = pinlib.expm_evolve(s, A0, T)
    errs = []
    for steps in (40, 80, 160):
        gx, gy, r = oracle.evolve_separated(s, monos, T, T / steps, "full")
        errs.append(pinlib.rel(oracle.separated_matrix(s, monos, gx, gy, r), ref))
    assert errs[-1] < 1e-7, errs
    for a, b in zip(errs, errs[1:]):
        assert 10.0 < a / b < 24.0, errs


def test_separated_form_without_dissipation_keeps_R_zero(oracle_lib):
    """Without jumps and dephasing P = 0: R stays exactly zero and G = Gx Gy
    (for both representations of R)."""
    cutoff = (3, 4)
    s = network(142, cutoff)
    s.gamma1[:] = 0.0
    s.gamma_phi[:] = 0.0
    A0 = _product([oracle.adag_matrix(3).conj().T, oracle.adag_matrix(4)])
    monos = oracle.monomials(s, A0)
    for mode in ("full", "z"):
        gx, gy, r = oracle.evolve_separated(s, monos, 0.2, 2.5e-4, mode)
        assert np.max(np.abs(r)) == 0.0
    ref = pinlib.expm_evolve(s, A0, 0.2)
    assert pinlib.rel(oracle.separated_matrix(s, monos, gx, gy, r), ref) < 1e-9


@pytest.mark.parametrize("dissipator", ["lindblad", "secular"])
def test_separated_z_grid_exact_without_drive_and_exchange(oracle_lib, dissipator):
    """With no drive and no exchange the one-sided operators Kx, Ky are
    diagonal, so a diagonal initial operator keeps Gx Gy diagonal in each
    mode, the source P(Gx Gy) feeds only the diagonal, and R is a function of
    x_j y_j alone: R on the z-grid equals R on the whole box."""
    cutoff = (4, 3)
    s = network(143, cutoff, dissipator)
    s.drive = np.zeros(2, dtype=np.complex128)
    s.exchange = np.zeros((2, 2))
    s.gamma_phi = np.full(2, 0.5)
    rng = np.random.default_rng(143)
    A0 = np.diag(rng.normal(size=12) + 1j * rng.normal(size=12))
    monos = oracle.monomials(s, A0)
    gx, gy, r = oracle.evolve_separated(s, monos, 0.3, 1e-3, "full")
    gx2, gy2, rz = oracle.evolve_separated(s, monos, 0.3, 1e-3, "z")
    assert np.max(np.abs(r - np.diag(np.diag(r)))) == 0.0
    assert np.max(np.abs(np.diag(r) - rz.reshape(-1))) < 1e-14 * np.max(np.abs(r))
    assert pinlib.rel(oracle.separated_matrix(s, monos, gx2, gy2, rz),
                      pinlib.expm_evolve(s, A0, 0.3)) < 1e-9
