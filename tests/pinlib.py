"""Independent constructions used to pin the oracle.

The dense superoperator here is built from Kronecker products of the
truncated ladder-operator matrices, a different route from the oracle's
element-wise formula, so a dropped term, a wrong sign or a transposed index in
either one shows up as a mismatch.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def ladder(nc: int) -> np.ndarray:
    a = np.zeros((nc, nc), dtype=np.complex128)
    for n in range(1, nc):
        a[n - 1, n] = np.sqrt(n)
    return a


def embed(op: np.ndarray, j: int, cutoff) -> np.ndarray:
    out = np.ones((1, 1), dtype=np.complex128)
    for i, nc in enumerate(cutoff):
        out = np.kron(out, op if i == j else np.eye(nc))
    return out


def hamiltonian(system) -> np.ndarray:
    cutoff = system.cutoff
    dim = int(np.prod(cutoff))
    H = np.zeros((dim, dim), dtype=np.complex128)
    a = [embed(ladder(nc), j, cutoff) for j, nc in enumerate(cutoff)]
    drive = getattr(system, "drive", None)
    exch = getattr(system, "exchange", None)
    for j in range(system.n_modes):
        ad = a[j].conj().T
        H += system.detuning[j] * ad @ a[j] + 0.5 * system.kerr[j] * ad @ ad @ a[j] @ a[j]
        for i in range(j):
            H += system.cross_kerr[i, j] * (a[i].conj().T @ a[i]) @ (ad @ a[j])
            if exch is not None:
                H += exch[i, j] * (a[i].conj().T @ a[j] + ad @ a[i])
        if drive is not None:
            H += drive[j] * ad + np.conj(drive[j]) * a[j]
    return H


def transition_occupations(system, j: int) -> np.ndarray:
    """Bath occupation of every transition n <-> n+1 of mode j (secular form)."""
    nc = system.cutoff[j]
    lv = getattr(system, "n_th_levels", None)
    if lv is None:
        return np.full(nc - 1, system.n_th[j])
    off = sum(c - 1 for c in system.cutoff[:j])
    return np.asarray(lv[off:off + nc - 1], dtype=float)


def jump_channels(system):
    """(rate, L) for every channel of every mode: the Lindblad form (a, a^+,
    n), or the secular form of Eq. (15) (one lowering and one raising jump per
    transition n <-> n+1, plus dephasing n)."""
    cutoff = system.cutoff
    out = []
    secular = getattr(system, "dissipator", "lindblad") == "secular"
    for j, nc in enumerate(cutoff):
        a = embed(ladder(nc), j, cutoff)
        n = a.conj().T @ a
        if secular:
            nbar = transition_occupations(system, j)
            for t in range(nc - 1):
                down = np.zeros((nc, nc), dtype=np.complex128)
                down[t, t + 1] = 1.0  # |t><t+1|
                out.append((system.gamma1[j] * (t + 1) * (nbar[t] + 1), embed(down, j, cutoff)))
                out.append((system.gamma1[j] * (t + 1) * nbar[t], embed(down.T.copy(), j, cutoff)))
        else:
            out.append((system.gamma1[j] * (1 + system.n_th[j]), a))
            out.append((system.gamma1[j] * system.n_th[j], a.conj().T))
        out.append((2 * system.gamma_phi[j], n))
    return out


def adjoint_superop(system) -> np.ndarray:
    """Matrix S with vec(dA/dt) = S vec(A) for the adjoint master equation,
    row-major vec: vec(P X Q) = kron(P, Q^T) vec(X)."""
    H = hamiltonian(system)
    dim = H.shape[0]
    eye = np.eye(dim)
    S = 1j * (np.kron(H, eye) - np.kron(eye, H.T))
    for kap, L in jump_channels(system):
        Ld = L.conj().T
        LdL = Ld @ L
        S += 0.5 * kap * (2 * np.kron(Ld, L.T) - np.kron(LdL, eye) - np.kron(eye, LdL.T))
    return S


def expm_evolve(system, A0: np.ndarray, t: float) -> np.ndarray:
    S = adjoint_superop(system)
    v = scipy.linalg.expm(S * t) @ A0.reshape(-1)
    return v.reshape(A0.shape)


def rk4_polynomial(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.reshape(-1))
    return float(np.linalg.norm((a - b).reshape(-1)) / (den if den > 0 else 1.0))
