"""Helpers shared by the GPU tests: comparison of library functions with the
oracle's number-basis sectors (the oracle result is rescaled to the g
coefficients by the oracle's own routine)."""

from __future__ import annotations

import sys

import numpy as np

import oracle


def announce(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def library():
    import paper_2203_05526_amd as hgf
    hgf.load_library()
    return hgf


def oracle_grids(cutoff, ops):
    """{d: m-grid of g} from oracle number-basis sectors."""
    g = oracle.generating_coefficients(cutoff, ops)
    return {d: oracle.sector_grid(cutoff, d, box) for d, box in g.items()}


def gpu_grids(op):
    out = {}
    for i in range(op.info()["n_functions"]):
        d, e, grid, _ = op.function(i)
        assert d not in out
        out[d] = grid
    return out


def max_rel_err(got: dict, ref: dict) -> float:
    """max |got - ref| / max |ref| over all sectors (sectors absent on one side
    count as zero there)."""
    scale = max(float(np.max(np.abs(v))) for v in ref.values())
    err = 0.0
    for d in set(got) | set(ref):
        a = got.get(d)
        b = ref.get(d)
        if a is None:
            a = np.zeros_like(b)
        if b is None:
            b = np.zeros_like(a)
        assert a.shape == b.shape, (d, a.shape, b.shape)
        err = max(err, float(np.max(np.abs(a - b))))
    return err / scale


def rel(a: complex, b: complex) -> float:
    return abs(a - b) / max(abs(b), 1e-300)


def number_scale(cutoff, d):
    """sqrt(prod_j k_j! l_j!) over the grid of sector d (m = min(k, l))."""
    import math
    scale = np.ones(tuple(nc - abs(dj) for nc, dj in zip(cutoff, d)))
    for j, (nc, dj) in enumerate(zip(cutoff, d)):
        u, v = max(0, -dj), max(0, dj)
        s = np.array([math.sqrt(math.factorial(m + u) * math.factorial(m + v)) for m in range(nc - abs(dj))])
        shape = [1] * len(cutoff)
        shape[j] = len(s)
        scale = scale * s.reshape(shape)
    return scale


def gpu_number_grids(op, cutoff):
    """Library functions converted back to number-basis elements
    <k|A|l> = g_{k,l} sqrt(k! l!), where every entry of a generic operator is
    of order one (a comparison of g alone hides errors at high occupation)."""
    return {d: g * number_scale(cutoff, d) for d, g in gpu_grids(op).items()}


def oracle_number_grids(cutoff, ops):
    return {d: oracle.sector_grid(cutoff, d, box) for d, box in ops.items()}
