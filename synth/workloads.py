"""Seeded workloads for the damped Kerr-network adjoint master equation.

Units: time in microseconds, angular frequencies in rad/us (2*pi * 1 MHz is
2*pi rad/us), decay rates in 1/us.  Every draw uses numpy's PCG64
(``numpy.random.default_rng(seed)``) in the fixed order

    K[N], detuning[N], T1[N], Tphi[N], chi[i<j, lexicographic],
    bitstring[N], |alpha|[N], arg(alpha)[N]

so that a seed names one system.  The rates handed on are gamma1 = 1/T1 and
gamma_phi = 1/Tphi; how those rates enter the dissipators is decided by the
consumers, not here.  Per-mode observable factors are plain matrices in the
truncated number basis; states are described by occupations or coherent
amplitudes only.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class System:
    """Parameters of N Kerr-coupled damped modes (rotating frame).

    H = sum_j [detuning_j n_j + (kerr_j/2) a_j^+ a_j^+ a_j a_j]
        + sum_{i<j} cross_kerr[i,j] n_i n_j
    gamma1_j, gamma_phi_j, n_th_j describe the baths of mode j.
    """

    cutoff: Tuple[int, ...]
    detuning: np.ndarray
    kerr: np.ndarray
    cross_kerr: np.ndarray  # (N, N), symmetric, zero diagonal
    gamma1: np.ndarray
    gamma_phi: np.ndarray
    n_th: np.ndarray
    # "lindblad" (emission/absorption channels a, a^+) or "secular" (one channel
    # per transition n <-> n+1); n_th_levels (secular only, optional): the bath
    # occupation of every transition, sum_j (cutoff_j - 1) values, modes in order
    dissipator: str = "lindblad"
    n_th_levels: Optional[np.ndarray] = None
    # driven, exchange-coupled network (optional): complex drive amplitudes
    # Omega_j (H += Omega_j a_j^+ + conj(Omega_j) a_j, static in the drive
    # frame) and a symmetric exchange matrix J (H += sum_{i<j} J_ij (a_i^+ a_j + h.c.))
    drive: Optional[np.ndarray] = None
    exchange: Optional[np.ndarray] = None

    @property
    def n_modes(self) -> int:
        return len(self.cutoff)

    def copy(self) -> "System":
        return System(tuple(self.cutoff), self.detuning.copy(), self.kerr.copy(),
                      self.cross_kerr.copy(), self.gamma1.copy(),
                      self.gamma_phi.copy(), self.n_th.copy(), self.dissipator,
                      None if self.n_th_levels is None else self.n_th_levels.copy(),
                      None if self.drive is None else self.drive.copy(),
                      None if self.exchange is None else self.exchange.copy())


@dataclass
class Workload:
    name: str
    system: System
    # observable: tensor product of per-mode matrices (list of (Nc_j, Nc_j)),
    # or a sum of several such products (list of lists).
    factors: List[np.ndarray]
    states: List[Tuple[str, np.ndarray]]
    t_total: float
    dt: float
    bitstring: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n_steps(self) -> int:
        return int(round(self.t_total / self.dt))

    @property
    def points(self) -> int:
        return int(np.prod(self.system.cutoff))


# ---------------------------------------------------------------- observables

def projector_factors(cutoff: Sequence[int], bits: Sequence[int]) -> List[np.ndarray]:
    """Per-mode factors of the projector |b><b| onto an occupation string."""
    out = []
    for nc, b in zip(cutoff, bits):
        m = np.zeros((nc, nc), dtype=np.complex128)
        m[int(b), int(b)] = 1.0
        out.append(m)
    return out


def parity_factors(cutoff: Sequence[int]) -> List[np.ndarray]:
    """Per-mode factors of (|0><0| - |1><1|), the qubit-subspace Z parity."""
    out = []
    for nc in cutoff:
        m = np.zeros((nc, nc), dtype=np.complex128)
        m[0, 0] = 1.0
        m[1, 1] = -1.0
        out.append(m)
    return out


def quadrature_factors(cutoff: Sequence[int]) -> List[np.ndarray]:
    """Per-mode factors of (a + a^+) in the truncated number basis."""
    out = []
    for nc in cutoff:
        m = np.zeros((nc, nc), dtype=np.complex128)
        for n in range(1, nc):
            m[n - 1, n] = np.sqrt(n)
            m[n, n - 1] = np.sqrt(n)
        out.append(m)
    return out


def annihilation_factors(cutoff: Sequence[int]) -> List[np.ndarray]:
    """Per-mode truncated annihilation operators a_j (the product is the test
    operator prod_j a_j of the network example)."""
    return [np.diag(np.sqrt(np.arange(1, c, dtype=float)), 1).astype(np.complex128) for c in cutoff]


def table1_network(n_modes: int, cutoff: int = 6) -> Workload:
    """The network example's parameters: a chain of anharmonic modes, each at
    the drive frequency (zero detuning in the drive frame), anharmonicity
    eta = 2 pi 250 MHz (K = 2 eta), the first driven with Omega = 2 pi 125 MHz
    (i Omega a e^{i w t} + h.c. is -i conj(Omega) a^+ + h.c. in the drive
    frame), nearest-neighbour exchange J = 2 pi 10 MHz, decay kappa = 0.02/us
    under the secular dissipator at zero bath temperature; observable
    prod_j a_j; horizon w_q t / pi = 10 with w_q = 2 pi 3500 MHz."""
    n = n_modes
    two_pi = TWO_PI
    sysm = System((cutoff,) * n, np.zeros(n), np.full(n, 2 * two_pi * 250.0), np.zeros((n, n)),
                  np.full(n, 0.02), np.zeros(n), np.zeros(n), dissipator="secular")
    sysm.drive = np.array([-1j * two_pi * 125.0] + [0.0] * (n - 1), dtype=np.complex128)
    J = np.zeros((n, n))
    for i in range(n - 1):
        J[i, i + 1] = J[i + 1, i] = two_pi * 10.0
    sysm.exchange = J
    t_total = 10 * np.pi / (two_pi * 3500.0)
    return Workload(f"network of {n} driven anharmonic modes (Table I), cutoff {cutoff}", sysm,
                    annihilation_factors(sysm.cutoff), [coherent_state([0.5] * n)], t_total, t_total / 100)


def fock_state(occ: Sequence[int]) -> Tuple[str, np.ndarray]:
    return ("fock", np.asarray(occ, dtype=np.int64))


def coherent_state(alpha: Sequence[complex]) -> Tuple[str, np.ndarray]:
    return ("coherent", np.asarray(alpha, dtype=np.complex128))


# ---------------------------------------------------------------- systems

def _draw(rng: np.random.Generator, n: int, alpha_range=(0.5, 1.5)):
    kerr = TWO_PI * rng.uniform(-250.0, -150.0, size=n)
    detuning = TWO_PI * rng.uniform(-5.0, 5.0, size=n)
    t1 = rng.uniform(30.0, 100.0, size=n)
    tphi = rng.uniform(50.0, 200.0, size=n)
    chi = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            chi[i, j] = chi[j, i] = TWO_PI * rng.uniform(-1.0, -0.1)
    bits = rng.integers(0, 2, size=n)
    amp = rng.uniform(alpha_range[0], alpha_range[1], size=n)
    phase = rng.uniform(0.0, TWO_PI, size=n)
    return kerr, detuning, t1, tphi, chi, bits, amp * np.exp(1j * phase)


def seeded_system(cutoff: Sequence[int], seed: int, n_th: float = 0.01,
                  alpha_range=(0.5, 1.5)):
    """Draw one system with the distributions of the 3-mode workload.

    Returns (System, bitstring, alpha)."""
    n = len(cutoff)
    rng = np.random.default_rng(seed)
    kerr, det, t1, tphi, chi, bits, alpha = _draw(rng, n, alpha_range)
    sysm = System(tuple(int(c) for c in cutoff), det, kerr, chi, 1.0 / t1,
                  1.0 / tphi, np.full(n, float(n_th)))
    return sysm, bits, alpha


def single_mode_c0() -> Workload:
    """One Kerr mode: K/2pi = -200 MHz, T1 = 50 us, Tphi = 100 us, n_th = 0.01,
    cutoff 16, observable |1><1|, T = 1 us, dt = 0.1 ns."""
    sysm = System((16,), np.zeros(1), np.array([TWO_PI * -200.0]), np.zeros((1, 1)),
                  np.array([1.0 / 50.0]), np.array([1.0 / 100.0]), np.array([0.01]))
    return Workload("one Kerr mode, cutoff 16, |1><1|", sysm,
                    projector_factors((16,), (1,)),
                    [fock_state([1]), coherent_state([1.0])], 1.0, 1e-4,
                    bitstring=np.array([1]))


def three_mode_c1(seed: int = 1) -> Workload:
    sysm, bits, alpha = seeded_system((12, 12, 12), seed)
    return Workload("3 Kerr modes, cutoff 12, bitstring projector", sysm,
                    projector_factors(sysm.cutoff, bits),
                    [coherent_state(alpha), fock_state(bits)], 10.0, 1e-4,
                    bitstring=bits)


def batch_c2(n_even: int = 64, n_uneven: int = 32) -> List[Workload]:
    """64 systems of 6 modes at cutoff 8 (seeds 1000...) and 32 systems of
    2-5 modes with per-mode cutoffs 6-20 (the following seeds)."""
    out = []
    for i in range(n_even):
        sysm, bits, alpha = seeded_system((8,) * 6, 1000 + i)
        out.append(Workload(f"6 modes cutoff 8 seed {1000 + i}", sysm,
                            projector_factors(sysm.cutoff, bits),
                            [coherent_state(alpha)], 1.0, 1e-4, bitstring=bits))
    for i in range(n_uneven):
        seed = 1000 + n_even + i
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 6))
        cut = tuple(int(c) for c in rng.integers(6, 21, size=n))
        sysm, bits, alpha = seeded_system(cut, seed)
        out.append(Workload(f"{n} modes cutoffs {cut} seed {seed}", sysm,
                            projector_factors(sysm.cutoff, bits),
                            [coherent_state(alpha)], 1.0, 1e-4, bitstring=bits))
    return out


def grad_c3(seed: int = 3) -> Workload:
    sysm, bits, alpha = seeded_system((16,) * 4, seed)
    return Workload("4 Kerr modes, cutoff 16, bitstring projector", sysm,
                    projector_factors(sysm.cutoff, bits),
                    [coherent_state(alpha)], 5.0, 1e-4, bitstring=bits,
                    extra={"checkpoint_every": 100})


def grad_c3b(seed: int = 3, cutoff: int = 8, t_total: float = 0.02,
             dt: float = 1e-6) -> Workload:
    """Off-diagonal companion of the gradient workload: observable
    prod_j (a_j + a_j^+), which spans 2^N occupation-difference sectors."""
    sysm, bits, alpha = seeded_system((cutoff,) * 4, seed)
    return Workload(f"4 Kerr modes, cutoff {cutoff}, product of quadratures", sysm,
                    quadrature_factors(sysm.cutoff),
                    [coherent_state(alpha)], t_total, dt, bitstring=bits)


def large_c4(seed: int = 4) -> Workload:
    sysm, bits, alpha = seeded_system((6,) * 10, seed, alpha_range=(0.3, 1.0))
    return Workload("10 Kerr modes, cutoff 6, parity-weighted projector", sysm,
                    parity_factors(sysm.cutoff),
                    [coherent_state(alpha)], 2.0, 5e-5, bitstring=bits)


# ---------------------------------------------------------------- test inputs

def random_system(cutoff: Sequence[int], seed: int, n_th: float = 0.05,
                  scale: float = 1.0) -> System:
    """A random system for unit tests: rates of order `scale` (1/us)."""
    rng = np.random.default_rng(seed)
    n = len(cutoff)
    chi = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            chi[i, j] = chi[j, i] = scale * rng.uniform(-1.0, 1.0)
    return System(tuple(int(c) for c in cutoff),
                  scale * rng.uniform(-1.0, 1.0, size=n),
                  scale * rng.uniform(-2.0, 2.0, size=n),
                  chi,
                  scale * rng.uniform(0.2, 1.0, size=n),
                  scale * rng.uniform(0.1, 0.5, size=n),
                  rng.uniform(0.5, 1.5, size=n) * n_th)


def random_product_operator(cutoff: Sequence[int], seed: int) -> List[np.ndarray]:
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(nc, nc)) + 1j * rng.normal(size=(nc, nc)) for nc in cutoff]


def random_sparse_operator(cutoff: Sequence[int], n_terms: int, seed: int):
    """Random (k, l, value) triples in the truncated number basis."""
    rng = np.random.default_rng(seed)
    n = len(cutoff)
    ks = np.stack([rng.integers(0, nc, size=n_terms) for nc in cutoff], axis=1)
    ls = np.stack([rng.integers(0, nc, size=n_terms) for nc in cutoff], axis=1)
    vals = rng.normal(size=n_terms) + 1j * rng.normal(size=n_terms)
    return ks.astype(np.int32), ls.astype(np.int32), vals


def random_normal_coeffs(nc: int, seed: int) -> np.ndarray:
    """Random normal-ordered coefficients f[p, q] of one mode."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(nc, nc)) + 1j * rng.normal(size=(nc, nc))
