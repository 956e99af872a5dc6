"""Plain FP64 CPU oracle for the adjoint Lindblad master equation of damped
Kerr-coupled bosonic modes.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this package; the product library never does, and this
package never imports the product library.

The heavy loop (the element-wise right-hand side of the adjoint master
equation, Eq. (3), and classical RK4) is the C file ``adjoint_me.c`` next to
this one; this module builds it with gcc, loads it with ctypes and adds the
plain numpy pieces: sector bookkeeping, states, the expectation value, and the
coefficient maps of Eqs. (6) and (11) with the basis of Eqs. (7)-(8).

Operators are dictionaries ``{d: box}``: ``d`` is the occupation difference
l - k (a tuple of ints), ``box`` a complex128 array of shape ``cutoff`` whose
entry at k is the number-basis element A[k, k + d] (zero where k + d leaves
the truncated space).
"""

from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from typing import Dict, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adjoint_me.c")
_LIB = os.path.join(_HERE, "_adjoint_me.so")
_lib = None

Sectors = Dict[Tuple[int, ...], np.ndarray]


def build() -> str:
    """Compile the C oracle with gcc (OpenMP, IEEE arithmetic)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp",
           _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    ip, dp, vp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    sysargs = [ctypes.c_int, ip, dp, dp, dp, dp, dp, dp, ctypes.c_int, dp]
    lib.oracle_rhs.argtypes = sysargs + [ctypes.c_int, ip, vp, vp, ctypes.c_int]
    lib.oracle_evolve.argtypes = sysargs + [ctypes.c_int, ip, vp, ctypes.c_long,
                                            ctypes.c_double, ctypes.c_int]
    lib.oracle_evolve_lawson.argtypes = sysargs + [ctypes.c_int, ip, vp, ctypes.c_long,
                                            ctypes.c_double, ctypes.c_int]
    lib.oracle_evolve_sens.argtypes = sysargs + [ctypes.c_int, ip, vp, vp, ctypes.c_long,
                                                 ctypes.c_double, ctypes.c_int]
    lib.oracle_rhs_full.argtypes = sysargs + [dp, dp, vp, vp, ctypes.c_int]
    lib.oracle_evolve_full.argtypes = sysargs + [dp, dp, vp, ctypes.c_long, ctypes.c_double, ctypes.c_int]
    lib.oracle_evolve_separated.argtypes = sysargs + [dp, dp, ctypes.c_int, ip, ip, vp, ctypes.c_int, vp, vp, vp,
                                                      ctypes.c_long, ctypes.c_double, ctypes.c_int]
    lib.oracle_num_params.argtypes = [ctypes.c_int]
    lib.oracle_max_threads.argtypes = []
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _sysargs(system):
    n = system.n_modes
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(np.asarray(x, dtype=dt).reshape(-1))
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int if dt == np.int32 else ctypes.c_double))

    secular = getattr(system, "dissipator", "lindblad") == "secular"
    levels = getattr(system, "n_th_levels", None)
    args = [n, arr(system.cutoff, np.int32), arr(system.detuning, np.float64),
            arr(system.kerr, np.float64), arr(system.cross_kerr, np.float64),
            arr(system.gamma1, np.float64), arr(system.gamma_phi, np.float64),
            arr(system.n_th, np.float64), 1 if secular else 0,
            arr(levels, np.float64) if (secular and levels is not None) else None]
    return args, keep


def _network_args(system, keep):
    """Drive (2N doubles, re/im) and exchange (N*N) pointers, or NULL."""
    out = []
    for x, dt in ((getattr(system, "drive", None), np.complex128), (getattr(system, "exchange", None), np.float64)):
        if x is None:
            out.append(None)
            continue
        a = np.ascontiguousarray(np.asarray(x, dtype=dt).reshape(-1))
        if dt == np.complex128:
            a = a.view(np.float64)
        keep.append(a)
        out.append(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def is_network(system) -> bool:
    """True when drive or exchange is present: the sectors are coupled and
    only the full-matrix functions apply."""
    d, x = getattr(system, "drive", None), getattr(system, "exchange", None)
    return (d is not None and np.any(np.asarray(d) != 0)) or (x is not None and np.any(np.asarray(x) != 0))


def _require_sectors(system):
    if is_network(system):
        raise ValueError("drive and exchange couple the sectors: use the full-matrix functions")


def rhs_full(system, A: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """One evaluation of the right-hand side of Eq. (3) on the full matrix A,
    with the network Hamiltonian of Eq. (16) (drive, exchange)."""
    lib = _load()
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    out = np.zeros_like(A)
    args, keep = _sysargs(system)
    rc = lib.oracle_rhs_full(*args, *_network_args(system, keep), A.ctypes.data, out.ctypes.data, nthreads)
    if rc:
        raise RuntimeError(f"oracle_rhs_full failed ({rc})")
    return out


def evolve_full(system, A: np.ndarray, t_total: float, dt: float, nthreads: int = 0) -> np.ndarray:
    """A(T) from the full matrix A(0) by classical RK4 with step dt."""
    lib = _load()
    A = np.array(A, dtype=np.complex128, order="C")
    args, keep = _sysargs(system)
    rc = lib.oracle_evolve_full(*args, *_network_args(system, keep), A.ctypes.data, n_steps(t_total, dt),
                                float(dt), nthreads)
    if rc:
        raise RuntimeError(f"oracle_evolve_full failed ({rc})")
    return A


def monomials(system, A: np.ndarray, drop_tol: float = 0.0):
    """The initial monomials of Eq. (10) for the full number-basis matrix A:
    (p, q, g_pq(0)) for every coefficient g_{p,q} = A[p, q] / sqrt(p! q!)
    (Eqs. (6)-(8) with o1 = a^+, o2 = a) with |g_pq| > drop_tol, p and q as
    occupation tuples."""
    cutoff = tuple(system.cutoff)
    dim = int(np.prod(cutoff))
    out = []
    for K in range(dim):
        k = np.unravel_index(K, cutoff)
        for L in range(dim):
            if A[K, L] == 0:
                continue
            l = np.unravel_index(L, cutoff)
            sc = math.sqrt(float(np.prod([math.factorial(int(x)) for x in k + l])))
            g = complex(A[K, L]) / sc
            if abs(g) > drop_tol:
                out.append((tuple(int(x) for x in k), tuple(int(x) for x in l), g))
    return out


def evolve_separated(system, monos, t_total: float, dt: float, rmode: str = "full", nthreads: int = 0,
                     state=None):
    """The separated form G = Gx Gy + R of Eqs. (9a)-(9c) for every monomial
    (p, q, c) of `monos` (Gx(0) = x^p, Gy(0) = y^q, R(0) = 0), classical RK4
    on the joint state.  Returns (gx [nmono, *cutoff], gy [nmono, *cutoff],
    r): r is the sum over the monomials of c R, on the full (k, l) box
    ([dim, dim], rmode "full") or on its diagonal k = l ([*cutoff], rmode "z",
    the approximation by a function of x_j y_j).  `state` = (gx, gy, r) as
    returned continues from that state instead of the initial monomials."""
    lib = _load()
    cutoff = tuple(system.cutoff)
    n = len(cutoff)
    dim = int(np.prod(cutoff))
    nm = len(monos)
    P = np.ascontiguousarray(np.array([m[0] for m in monos], dtype=np.int32).reshape(nm, n))
    Q = np.ascontiguousarray(np.array([m[1] for m in monos], dtype=np.int32).reshape(nm, n))
    C = np.ascontiguousarray(np.array([m[2] for m in monos], dtype=np.complex128))
    gx = np.zeros((nm, dim), dtype=np.complex128)
    gy = np.zeros((nm, dim), dtype=np.complex128)
    for i in range(nm):
        gx[i, np.ravel_multi_index(P[i], cutoff)] = 1.0
        gy[i, np.ravel_multi_index(Q[i], cutoff)] = 1.0
    rm = {"full": 0, "z": 1}[rmode]
    r = np.zeros((dim, dim) if rm == 0 else (dim,), dtype=np.complex128)
    if state is not None:
        gx = np.array(state[0], dtype=np.complex128).reshape(nm, dim)
        gy = np.array(state[1], dtype=np.complex128).reshape(nm, dim)
        r = np.array(state[2], dtype=np.complex128).reshape(r.shape)
    args, keep = _sysargs(system)
    rc = lib.oracle_evolve_separated(*args, *_network_args(system, keep), nm,
                                     P.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                     Q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), C.ctypes.data, rm,
                                     gx.ctypes.data, gy.ctypes.data, r.ctypes.data, n_steps(t_total, dt), float(dt),
                                     nthreads)
    if rc:
        raise RuntimeError(f"oracle_evolve_separated failed ({rc})")
    return gx.reshape((nm,) + cutoff), gy.reshape((nm,) + cutoff), (r if rm == 0 else r.reshape(cutoff))


def separated_matrix(system, monos, gx, gy, r) -> np.ndarray:
    """The full number-basis matrix of G = sum_i c_i Gx_i Gy_i + R (Eq. (11)
    with the coefficient map of Eqs. (6)-(8)): M[k, l] = sqrt(k! l!) g(k, l)."""
    cutoff = tuple(system.cutoff)
    dim = int(np.prod(cutoff))
    g = np.zeros((dim, dim), dtype=np.complex128)
    for i, (_, _, c) in enumerate(monos):
        g += c * np.outer(gx[i].reshape(dim), gy[i].reshape(dim))
    r = np.asarray(r)
    if r.shape == (dim, dim):
        g += r
    else:
        g += np.diag(r.reshape(dim))
    fac = np.array([math.sqrt(float(np.prod([math.factorial(int(x)) for x in np.unravel_index(K, cutoff)])))
                    for K in range(dim)])
    return g * np.outer(fac, fac)


def _pack(system, ops: Sectors):
    keys = sorted(ops.keys())
    n = system.n_modes
    d = np.ascontiguousarray(np.array(keys, dtype=np.int32).reshape(len(keys), n))
    A = np.ascontiguousarray(np.stack([np.asarray(ops[k], dtype=np.complex128).reshape(system.cutoff)
                                       for k in keys]))
    return keys, d, A


def num_params(n: int) -> int:
    """K[N], chi[i<j], Delta[N], gamma1[N], gamma_phi[N]."""
    return n + n * (n - 1) // 2 + 3 * n


def rhs(system, ops: Sectors, nthreads: int = 0) -> Sectors:
    """One evaluation of the right-hand side of Eq. (3) on every sector."""
    _require_sectors(system)
    lib = _load()
    keys, d, A = _pack(system, ops)
    out = np.zeros_like(A)
    args, keep = _sysargs(system)
    rc = lib.oracle_rhs(*args, len(keys), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                        A.ctypes.data, out.ctypes.data, nthreads)
    if rc:
        raise RuntimeError(f"oracle_rhs failed ({rc})")
    return {k: out[i] for i, k in enumerate(keys)}


def n_steps(t_total: float, dt: float) -> int:
    m = int(round(t_total / dt))
    if m < 0 or abs(m * dt - t_total) > 1e-9 * max(1.0, abs(t_total)):
        raise ValueError("t_total must be a non-negative integer multiple of dt")
    return m


def evolve(system, ops: Sectors, t_total: float, dt: float, nthreads: int = 0) -> Sectors:
    """A(T) from A(0) by classical RK4 with step dt (same scheme as the paper's
    fourth-order Runge-Kutta integration)."""
    _require_sectors(system)
    lib = _load()
    keys, d, A = _pack(system, ops)
    args, keep = _sysargs(system)
    rc = lib.oracle_evolve(*args, len(keys), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           A.ctypes.data, n_steps(t_total, dt), float(dt), nthreads)
    if rc:
        raise RuntimeError(f"oracle_evolve failed ({rc})")
    return {k: A[i] for i, k in enumerate(keys)}


def evolve_lawson(system, ops: Sectors, t_total: float, dt: float, nthreads: int = 0) -> Sectors:
    """A(T) from A(0) by the integrating-factor (Lawson) RK4: the diagonal
    part of the right-hand side of Eq. (3) taken exactly, the jump terms by
    classical RK4 in the interaction picture."""
    lib = _load()
    keys, d, A = _pack(system, ops)
    args, keep = _sysargs(system)
    rc = lib.oracle_evolve_lawson(*args, len(keys), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  A.ctypes.data, n_steps(t_total, dt), float(dt), nthreads)
    if rc:
        raise RuntimeError(f"oracle_evolve_lawson failed ({rc})")
    return {k: A[i] for i, k in enumerate(keys)}


def evolve_steps(system, ops: Sectors, steps: int, dt: float, nthreads: int = 0) -> Sectors:
    lib = _load()
    keys, d, A = _pack(system, ops)
    args, keep = _sysargs(system)
    rc = lib.oracle_evolve(*args, len(keys), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           A.ctypes.data, int(steps), float(dt), nthreads)
    if rc:
        raise RuntimeError(f"oracle_evolve failed ({rc})")
    return {k: A[i] for i, k in enumerate(keys)}


def evolve_sens(system, ops: Sectors, t_total: float, dt: float, nthreads: int = 0):
    """A(T) and dA(T)/dtheta_p for every parameter (forward sensitivities of
    the discrete RK4 map).  Returns (A_T, [S_p])."""
    lib = _load()
    keys, d, A = _pack(system, ops)
    P = num_params(system.n_modes)
    S = np.zeros((P,) + A.shape, dtype=np.complex128)
    args, keep = _sysargs(system)
    rc = lib.oracle_evolve_sens(*args, len(keys), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                A.ctypes.data, S.ctypes.data, n_steps(t_total, dt), float(dt),
                                nthreads)
    if rc:
        raise RuntimeError(f"oracle_evolve_sens failed ({rc})")
    a_t = {k: A[i] for i, k in enumerate(keys)}
    sens = [{k: S[p, i] for i, k in enumerate(keys)} for p in range(P)]
    return a_t, sens


# ------------------------------------------------------------------ operators

def product_sectors(factors: Sequence[np.ndarray]) -> Sectors:
    """Sectors of the tensor product of per-mode matrices M_j:
    A[k, l] = prod_j M_j[k_j, l_j]."""
    cutoff = tuple(m.shape[0] for m in factors)
    per_mode = []
    for m in factors:
        nc = m.shape[0]
        ds = [dj for dj in range(-nc + 1, nc) if np.any(np.diagonal(m, offset=dj) != 0)]
        per_mode.append(ds)
    out: Sectors = {}
    for d in itertools.product(*per_mode):
        box = np.ones(cutoff, dtype=np.complex128)
        for j, (m, dj) in enumerate(zip(factors, d)):
            nc = m.shape[0]
            col = np.zeros(nc, dtype=np.complex128)
            for k in range(nc):
                if 0 <= k + dj < nc:
                    col[k] = m[k, k + dj]
            shape = [1] * len(cutoff)
            shape[j] = nc
            box = box * col.reshape(shape)
        out[tuple(int(x) for x in d)] = box
    return out


def sparse_sectors(cutoff: Sequence[int], ks, ls, vals) -> Sectors:
    """Sectors of sum_t vals[t] |k_t><l_t| (repeated (k, l) pairs add up)."""
    out: Sectors = {}
    for k, l, v in zip(np.asarray(ks), np.asarray(ls), np.asarray(vals)):
        d = tuple(int(b - a) for a, b in zip(k, l))
        box = out.setdefault(d, np.zeros(tuple(cutoff), dtype=np.complex128))
        box[tuple(int(a) for a in k)] += v
    return out


def dense_from_sectors(cutoff: Sequence[int], ops: Sectors) -> np.ndarray:
    """Full number-basis matrix (small systems only), index order C-style."""
    dim = int(np.prod(cutoff))
    M = np.zeros((dim, dim), dtype=np.complex128)
    for d, box in ops.items():
        for k in itertools.product(*[range(c) for c in cutoff]):
            l = tuple(a + b for a, b in zip(k, d))
            if all(0 <= x < c for x, c in zip(l, cutoff)):
                M[np.ravel_multi_index(k, cutoff), np.ravel_multi_index(l, cutoff)] = box[k]
    return M


def sectors_from_dense(cutoff: Sequence[int], M: np.ndarray, tol: float = 0.0) -> Sectors:
    out: Sectors = {}
    for ki in range(M.shape[0]):
        k = np.unravel_index(ki, cutoff)
        for li in range(M.shape[1]):
            if abs(M[ki, li]) <= tol:
                continue
            l = np.unravel_index(li, cutoff)
            d = tuple(int(b - a) for a, b in zip(k, l))
            box = out.setdefault(d, np.zeros(tuple(cutoff), dtype=np.complex128))
            box[tuple(int(a) for a in k)] = M[ki, li]
    return out


# ------------------------------------------------------------------ states

def mode_amplitudes(nc: int, kind: str, value) -> np.ndarray:
    """Number-basis amplitudes c_n of one mode's state.

    fock: c = delta_{n, value}.
    coherent: c_n = alpha^n / sqrt(n!), renormalised on the truncated space.
    """
    if kind == "fock":
        c = np.zeros(nc, dtype=np.complex128)
        c[int(value)] = 1.0
        return c
    if kind == "coherent":
        alpha = complex(value)
        c = np.array([alpha ** n / math.sqrt(math.factorial(n)) for n in range(nc)],
                     dtype=np.complex128)
        return c / np.linalg.norm(c)
    raise ValueError(kind)


def state_amplitudes(cutoff: Sequence[int], state) -> List[np.ndarray]:
    kind, vals = state
    if kind == "product":
        return [np.asarray(v, dtype=np.complex128) for v in vals]
    return [mode_amplitudes(nc, kind, v) for nc, v in zip(cutoff, vals)]


def expectation(cutoff: Sequence[int], ops: Sectors, state) -> complex:
    """<psi0| A |psi0> = sum_{k,l} conj(c_k) A[k,l] c_l for a product state."""
    amps = state_amplitudes(cutoff, state)
    total = 0.0 + 0.0j
    for d, box in ops.items():
        left = np.ones((1,) * len(cutoff), dtype=np.complex128)
        right = np.ones((1,) * len(cutoff), dtype=np.complex128)
        for j, (c, dj) in enumerate(zip(amps, d)):
            nc = len(c)
            shifted = np.zeros(nc, dtype=np.complex128)
            for k in range(nc):
                if 0 <= k + dj < nc:
                    shifted[k] = c[k + dj]
            shape = [1] * len(cutoff)
            shape[j] = nc
            left = left * np.conj(c).reshape(shape)
            right = right * shifted.reshape(shape)
        total += complex(np.sum(left * box * right))
    return total


# ------------------------------------------------------- coefficient maps

def adag_matrix(nc: int) -> np.ndarray:
    m = np.zeros((nc, nc), dtype=np.complex128)
    for n in range(1, nc):
        m[n, n - 1] = math.sqrt(n)
    return m


def number_from_normal(f: np.ndarray) -> np.ndarray:
    """Single mode: the matrix of sum_{p,q} f[p,q] (a^+)^p a^q on the
    truncated space (Eq. (2) with o1 = a^+, o2 = a), by matrix products."""
    nc = f.shape[0]
    ad = adag_matrix(nc)
    a = ad.conj().T
    out = np.zeros((nc, nc), dtype=np.complex128)
    for p in range(nc):
        for q in range(nc):
            if f[p, q] != 0:
                out += f[p, q] * np.linalg.matrix_power(ad, p) @ np.linalg.matrix_power(a, q)
    return out


def g_from_f(f: np.ndarray, r: complex = 1.0) -> np.ndarray:
    """Eq. (6): g[k,l] = sum_{j=0}^{min(k,l)} r^{-j}/j! f[k-j, l-j]."""
    nc0, nc1 = f.shape
    g = np.zeros_like(f, dtype=np.complex128)
    for k in range(nc0):
        for l in range(nc1):
            g[k, l] = sum(r ** (-j) / math.factorial(j) * f[k - j, l - j]
                          for j in range(min(k, l) + 1))
    return g


def f_from_g(g: np.ndarray, r: complex = 1.0) -> np.ndarray:
    """Inverse of Eq. (6), the inner sum of Eq. (11):
    f[k,l] = sum_{j=0}^{min(k,l)} (-r)^{-j}/j! g[k-j, l-j]."""
    nc0, nc1 = g.shape
    f = np.zeros_like(g, dtype=np.complex128)
    for k in range(nc0):
        for l in range(nc1):
            f[k, l] = sum((-r) ** (-j) / math.factorial(j) * g[k - j, l - j]
                          for j in range(min(k, l) + 1))
    return f


def basis_T(k: int, l: int, nc: int, r: complex = 1.0) -> np.ndarray:
    """Eq. (8) on the truncated space: T_{k,l} = sum_j (-r)^{-j}/j! (a^+)^{k+j} a^{l+j}."""
    ad = adag_matrix(nc)
    a = ad.conj().T
    out = np.zeros((nc, nc), dtype=np.complex128)
    for j in range(nc):
        if k + j >= nc or l + j >= nc:
            break
        out += (-r) ** (-j) / math.factorial(j) * (np.linalg.matrix_power(ad, k + j)
                                                   @ np.linalg.matrix_power(a, l + j))
    return out


def generating_coefficients(cutoff: Sequence[int], ops: Sectors) -> Sectors:
    """g[k, l] = <k|A|l> / sqrt(prod_j k_j! l_j!): the coefficients of A in the
    basis T_{k,l} of Eqs. (7)-(8) with o1 = a^+, o2 = a (r = 1)."""
    out: Sectors = {}
    for d, box in ops.items():
        scale = np.ones(tuple(cutoff))
        for j, (nc, dj) in enumerate(zip(cutoff, d)):
            s = np.array([math.sqrt(math.factorial(k) * math.factorial(k + dj)) if 0 <= k + dj < nc else 1.0
                          for k in range(nc)])
            shape = [1] * len(cutoff)
            shape[j] = nc
            scale = scale * s.reshape(shape)
        out[d] = box / scale
    return out


def sector_grid(cutoff: Sequence[int], d: Sequence[int], box: np.ndarray) -> np.ndarray:
    """The part of a k-box where l = k + d stays inside the truncated space,
    indexed by m = min(k, l) (extent Nc_j - |d_j| per mode)."""
    sl = tuple(slice(max(0, -dj), max(0, -dj) + nc - abs(dj)) for nc, dj in zip(cutoff, d))
    return box[sl]
