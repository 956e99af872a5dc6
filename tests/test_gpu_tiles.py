"""Launch shapes of the tiled RK4 stage kernel and the autotuner that picks
them: every shape computes the same RK4 steps (to rounding) and matches the
FP64 oracle; the autotuner's cache round-trips; infeasible shapes are
rejected without changing the operator."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import announce, gpu_number_grids, library, max_rel_err, oracle_number_grids

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def hgf():
    return library()


def _shapes(tile_points):
    """(threads, xblock, pipe, wgs_per_cu, walk_block) samples for one tile
    size: the default workgroup, the smallest and the largest feasible one,
    odd XCD blocks, blocked walk orders (blocks of 2 and 3, with interleaved
    XCD blocks, and blocks wider than some axes)."""
    ths = [t for t in range(64, 513, 64) if -(-tile_points // t) <= 8]
    return [(0, 0, 0, 0, 0), (ths[0], 3, 1, 0, 2), (ths[-1], 128, 0, 1, 0), (ths[len(ths) // 2], 1, 1, 2, 3),
            (0, 0, 0, 0, 4), (ths[-1], 5, 0, 0, 3)]


def _apply(hgf, op, nfast, threads, xblock, pipe, wgs=0, walk=0):
    """Set the shape on every function where it is feasible; returns how many took it."""
    took = 0
    for i in range(op.info()["n_functions"]):
        try:
            op.set_tile_config(i, nfast, threads, xblock, pipe, wgs, walk_block=walk)
            took += 1
        except hgf.HgfError as e:
            assert e.status == "HGF_EINVAL"
    return took


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["real-diagonal", "complex-bidiagonal"])
def test_forced_tile_shapes_agree_and_match_oracle(hgf, precision, kind):
    cutoff = (3, 6, 6, 6, 6) if kind == "real-diagonal" else (3, 5, 4, 6, 3)
    announce(f"forced tile shapes {kind} {precision}")
    s = synth.random_system(cutoff, 51, scale=3.0, n_th=0.3)
    rng = np.random.default_rng(51)
    if kind == "real-diagonal":
        fac = [np.diag(rng.uniform(0.5, 1.5, size=c)).astype(np.complex128) for c in cutoff]
    else:
        fac = [np.triu(np.tril(rng.normal(size=(c, c)) + 1j * rng.normal(size=(c, c)), 1)) for c in cutoff]
    S = hgf.define_system(s)
    T, dt = 0.02, 1e-3
    ref = oracle_number_grids(cutoff, oracle.evolve(s, oracle.product_sectors(fac), T, dt))
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    same = 1e-13 if precision == "fp64" else 1e-6
    base = hgf.map_operator(S, factors=fac, precision=precision)
    hgf.evolve(base, T, dt)
    base_grids = gpu_number_grids(base, cutoff)
    assert max_rel_err(base_grids, ref) < tol
    tried = 0
    for nfast in (1, 2, 3, 4):
        tile = int(np.prod(cutoff[len(cutoff) - nfast:]))
        for threads, xblock, pipe, wgs, walk in _shapes(tile):
            op = hgf.map_operator(S, factors=fac, precision=precision)
            if _apply(hgf, op, nfast, threads, xblock, pipe, wgs, walk) == 0:
                continue
            shape = (nfast, threads, xblock, pipe, wgs, walk)
            announce(f"  nfast={nfast} threads={threads} xblock={xblock} pipe={pipe} wgs_per_cu={wgs} walk={walk}")
            hgf.evolve(op, T, dt)
            got = gpu_number_grids(op, cutoff)
            assert max_rel_err(got, ref) < tol, shape
            assert max_rel_err(got, base_grids) < same, shape
            if walk and nfast < len(cutoff):
                assert any(op.tile_config(i)["walk_block"] == walk for i in range(op.info()["n_functions"]))
                # the walk order moves no arithmetic: the same numbers as the row-major walk
                rm = hgf.map_operator(S, factors=fac, precision=precision)
                _apply(hgf, rm, nfast, threads, xblock, pipe, wgs, 0)
                hgf.evolve(rm, T, dt)
                assert max_rel_err(got, gpu_number_grids(rm, cutoff)) == 0.0, shape
            tried += 1
    assert tried >= 10
    if kind == "complex-bidiagonal":  # the untiled kernel too
        op = hgf.map_operator(S, factors=fac, precision=precision)
        assert _apply(hgf, op, 0, 0, 0, 0) == op.info()["n_functions"]
        assert op.tile_config(0)["nfast"] == 0
        hgf.evolve(op, T, dt)
        assert max_rel_err(gpu_number_grids(op, cutoff), ref) < tol


def test_tile_config_rejects_infeasible_shapes(hgf):
    cutoff = (3, 6, 6, 6, 6)
    announce("tile config errors")
    s = synth.random_system(cutoff, 52, scale=3.0)
    S = hgf.define_system(s)
    fac = [np.eye(c, dtype=np.complex128) * 0.5 for c in cutoff]
    op = hgf.map_operator(S, factors=fac, precision="mixed")
    assert op.info()["real_functions"] == 1
    before = op.tile_config(0)
    assert before["nfast"] >= 1 and before["blocks"] > 0
    bad = [(0, 0, 0, 0),      # a real grid needs the tiled kernel
           (4, 100, 0, 0),    # not a multiple of 64
           (4, 128, 0, 0),    # 1296-point tile in more than 8 lane rounds
           (4, 1024, 0, 0),   # above 512 lanes
           (6, 0, 0, 0),      # more fast axes than the grid has
           (4, 256, 0, 2),    # pipe is 0 or 1
           (4, 256, 0, 0, 64),  # more resident workgroups than fit on a CU
           (4, 256, 0, 0, 0, 0, -2)]  # negative walk block
    for cfg in bad:
        with pytest.raises(hgf.HgfError) as e:
            op.set_tile_config(0, *cfg)
        assert e.value.status == "HGF_EINVAL", cfg
        assert op.tile_config(0) == before
    with pytest.raises(hgf.HgfError) as e:
        op.set_tile_config(3, 4)
    assert e.value.status == "HGF_EINVAL"
    one = np.ones((1, len(cutoff)), dtype=np.int32)
    sp = hgf.map_operator(S, sparse=(one, one, np.array([1.0 + 0j])), layout="split", precision="fp64")
    with pytest.raises(hgf.HgfError) as e:
        sp.set_tile_config(0, 2)
    assert e.value.status == "HGF_EUNSUPPORTED"


def test_autotune_cache_and_results(hgf, tmp_path):
    """The autotuner measures each distinct shape once, writes the cache,
    leaves the evolved states unchanged, and a later call applies the cached
    shapes without measuring."""
    announce("autotune")
    cache = str(tmp_path / "tune.txt")
    T, dt = 0.02, 1e-3
    cases = []
    for cutoff, seed in (((3, 6, 6, 6, 6), 53), ((2, 4, 5, 7, 3), 54)):
        s = synth.random_system(cutoff, seed, scale=3.0, n_th=0.2)
        rng = np.random.default_rng(seed)
        fac = [np.diag(rng.uniform(0.5, 1.5, size=c)).astype(np.complex128) for c in cutoff]
        S = hgf.define_system(s)
        ref = oracle_number_grids(cutoff, oracle.evolve(s, oracle.product_sectors(fac), T, dt))
        cases.append((cutoff, S, fac, ref))
    ops = [hgf.map_operator(S, factors=fac, precision="mixed") for _, S, fac, _ in cases]
    twin = hgf.map_operator(cases[0][1], factors=cases[0][2], precision="mixed")
    hgf.autotune(ops + [twin], dt, cache=cache)
    lines = open(cache).read().splitlines()
    # two grid shapes, and at least the two functions of the first shape share
    # an axis split: one grouped launch, tuned as a whole (the shapes tuned
    # per grid decide whether the third function joins that group)
    assert len(lines) == 3, lines
    shape_line = [ln for ln in lines if ":mixed:real:3x6x6x6x6 " in ln]
    assert len(shape_line) == 1
    assert any(":mixed:real:2x4x5x7x3 " in ln for ln in lines)
    group_line = [ln for ln in lines if ":group:" in ln]
    assert len(group_line) == 1 and (":m2:" in group_line[0] or ":m3:" in group_line[0]), lines
    for op in ops:
        cfg = op.tile_config(0)
        assert cfg["stage_us"] > 0.0 and cfg["blocks"] > 0
    assert twin.tile_config(0) == ops[0].tile_config(0)
    for op, (cutoff, _, _, ref) in zip(ops, cases):
        hgf.evolve(op, T, dt)
        assert max_rel_err(gpu_number_grids(op, cutoff), ref) < MIXED_TOL
    # cached shapes are applied to new operators without measuring
    fresh = hgf.map_operator(cases[0][1], factors=cases[0][2], precision="mixed")
    hgf.autotune([fresh], dt, cache=cache, mode="cached_only")
    a = fresh.tile_config(0)
    fields = shape_line[0].split()[1:7]
    assert [a[k] for k in ("nfast", "threads", "xblock", "pipe", "wgs_per_cu", "walk_block")] == [
        int(v) for v in fields]
    # force re-measures and rewrites the entry in place
    hgf.autotune([fresh], dt, cache=cache, mode="force")
    assert len(open(cache).read().splitlines()) == 3
    hgf.evolve(fresh, T, dt)
    assert max_rel_err(gpu_number_grids(fresh, cases[0][0]), cases[0][3]) < MIXED_TOL
    # no cache path: measure and apply only
    nocache = hgf.map_operator(cases[1][1], factors=cases[1][2], precision="mixed")
    hgf.autotune([nocache], dt)
    assert nocache.tile_config(0)["stage_us"] > 0.0
    # a single-tile grid runs on the resident integrator: nothing to tune
    small = hgf.map_operator(hgf.define_system(synth.random_system((4, 5, 7), 55)),
                             factors=[np.eye(c, dtype=np.complex128) for c in (4, 5, 7)], precision="mixed")
    assert small.tile_config(0)["resident"] == 1
    hgf.autotune([small], dt, cache=cache)
    assert small.tile_config(0)["stage_us"] == 0.0
    assert len(open(cache).read().splitlines()) == 3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_integrator_large_sectors(hgf, monkeypatch, precision):
    """Sectors of 7^4 points (product of quadratures on 4 modes at cutoff 8):
    more points than one tile of the stage kernel, so they run on the
    resident integrator by their own layout, with two padded copies of
    73,728 B (mixed) or 147,456 B (FP64, five lane rounds of 512 lanes) of
    LDS; equal to the grouped stage launches (to rounding) and the oracle."""
    announce(f"resident 7^4 sectors {precision}")
    w = synth.grad_c3b()
    S = hgf.define_system(w.system)
    T = 200 * w.dt
    ops = {}
    for res in ("1", "0"):
        monkeypatch.setenv("HGF_RESIDENT", res)
        op = hgf.map_operator(S, factors=w.factors, precision=precision)
        nf = op.info()["n_functions"]
        assert nf == 16
        cfgs = [op.tile_config(i) for i in range(nf)]
        assert all(c["resident"] == (res == "1") and c["tile_points"] < 2401 for c in cfgs)
        hgf.evolve(op, T, w.dt)
        ops[res] = op
    monkeypatch.delenv("HGF_RESIDENT")
    cutoff = w.system.cutoff
    a, b = gpu_number_grids(ops["1"], cutoff), gpu_number_grids(ops["0"], cutoff)
    assert max_rel_err(a, b) < (1e-13 if precision == "fp64" else 1e-6)
    ref = oracle_number_grids(cutoff, oracle.evolve(w.system, oracle.product_sectors(w.factors), T, w.dt))
    assert max_rel_err(a, ref) < (FP64_TOL if precision == "fp64" else MIXED_TOL)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_integrator_matches_stage_launches(hgf, precision):
    """Grids that are one tile are integrated on chip by one workgroup through
    all steps of a call.  The result equals the per-stage launches (to
    rounding) and the oracle, for the 3-mode workload (one real sector) and
    for a random operator whose 35 sectors all run in one resident launch."""
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    same = 1e-13 if precision == "fp64" else 1e-6
    announce(f"resident 3-mode {precision}")
    w = synth.three_mode_c1()
    S = hgf.define_system(w.system)
    ops = {}
    for res in (1, 0):
        op = hgf.map_operator(S, factors=w.factors, precision=precision)
        assert op.tile_config(0)["resident"] == 1  # the default for a single-tile grid
        if res == 0:
            op.set_tile_config(0, 3, 0, 0, 0, 0, 0)
            assert op.tile_config(0)["resident"] == 0
        hgf.evolve(op, 0.05, w.dt)
        hgf.evolve(op, 0.03, w.dt)  # a second call continues from the stored state
        ops[res] = op
    a, b = gpu_number_grids(ops[1], w.system.cutoff), gpu_number_grids(ops[0], w.system.cutoff)
    assert max_rel_err(a, b) < same
    ref = oracle_number_grids(w.system.cutoff, oracle.evolve(w.system, oracle.product_sectors(w.factors), 0.08, w.dt))
    assert max_rel_err(a, ref) < tol
    assert ops[1].info()["steps_done"] == 800

    announce(f"resident multi-sector {precision}")
    cutoff = (4, 5, 3)
    s = synth.random_system(cutoff, 71, scale=3.0, n_th=0.2)
    rng = np.random.default_rng(71)
    fac = [rng.normal(size=(c, c)) + 1j * rng.normal(size=(c, c)) for c in cutoff]
    S = hgf.define_system(s)
    op = hgf.map_operator(S, factors=fac, precision=precision)
    nf = op.info()["n_functions"]
    assert nf == 7 * 9 * 5
    assert all(op.tile_config(i)["resident"] == 1 for i in range(nf))
    T, dt = 0.05, 1e-3
    hgf.evolve(op, T, dt)
    ref = oracle_number_grids(cutoff, oracle.evolve(s, oracle.product_sectors(fac), T, dt))
    assert max_rel_err(gpu_number_grids(op, cutoff), ref) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_workgroup_sizes(hgf, precision):
    """The resident integrator's workgroup size, set through
    hgf_set_tile_config: every size that covers the 3-mode grid (1,728
    points) in at most four lane rounds gives the same result
    bit for bit (each point's arithmetic does not depend on it); other sizes
    are rejected and leave the function as it was."""
    w = synth.three_mode_c1()
    S = hgf.define_system(w.system)
    announce(f"resident workgroup sizes {precision}")
    sizes = (448, 512) if precision == "fp64" else (448, 576, 896, 1024)
    grids = []
    for th in sizes:
        op = hgf.map_operator(S, factors=w.factors, precision=precision)
        op.set_tile_config(0, 3, th, 0, 0, 0, 1)
        cfg = op.tile_config(0)
        assert cfg["resident"] == 1 and cfg["threads"] == th, cfg
        hgf.evolve(op, 0.02, w.dt)
        grids.append(op.function(0)[2])
    for g in grids[1:]:
        assert np.array_equal(g, grids[0])
    op = hgf.map_operator(S, factors=w.factors, precision=precision)
    before = op.tile_config(0)
    for th in (100, 384 if precision == "fp64" else 320, 2048):
        with pytest.raises(hgf.HgfError) as e:
            op.set_tile_config(0, 3, th, 0, 0, 0, 1)
        assert e.value.status == "HGF_EINVAL", th
        assert op.tile_config(0) == before


def test_resident_members_in_a_batch(hgf):
    """A batch mixing resident members (small grids) with tiled ones advances
    each member as its own evolve does and matches the oracle."""
    announce("resident members in a batch")
    shapes = [(6, 7), (3, 4, 5), (2, 6, 6, 6, 3), (9,), (3, 3, 3, 3, 3)]
    T, dt = [0.02, 0.03, 0.01, 0.04, 0.02], 1e-3
    systems, facs = [], []
    for i, c in enumerate(shapes):
        systems.append(synth.random_system(c, 80 + i, scale=3.0, n_th=0.2))
        rng = np.random.default_rng(80 + i)
        facs.append([np.triu(np.tril(rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k)), 1)) for k in c])
    batch = [hgf.map_operator(hgf.define_system(s), factors=f, precision="mixed") for s, f in zip(systems, facs)]
    single = [hgf.map_operator(hgf.define_system(s), factors=f, precision="mixed") for s, f in zip(systems, facs)]
    kinds = {op.tile_config(0)["resident"] for op in batch}
    assert kinds == {0, 1}
    hgf.evolve_batch(batch, T, [dt] * len(batch))
    for op, t in zip(single, T):
        hgf.evolve(op, t, dt)
    for op_b, op_s, c, s, f, t in zip(batch, single, shapes, systems, facs, T):
        a, b = gpu_number_grids(op_b, c), gpu_number_grids(op_s, c)
        assert max_rel_err(a, b) < 1e-6, c
        ref = oracle_number_grids(c, oracle.evolve(s, oracle.product_sectors(f), t, dt))
        assert max_rel_err(a, ref) < MIXED_TOL, c


def test_untiled_functions_reported(hgf, monkeypatch):
    """hgf_get_info counts the functions that run on the untiled stage kernel:
    none on a grid the tiled kernel takes, all of them when the untiled
    kernel is forced, and that count follows a forced shape (nfast 0)."""
    announce("untiled functions in hgf_get_info")
    cutoff = (4, 6, 6, 6, 6)  # one diagonal sector of 5184 points: tiled, not resident
    s = synth.random_system(cutoff, 52)
    rng = np.random.default_rng(52)
    # complex diagonal entries: a complex grid (the untiled kernel takes no real grids)
    fac = [np.diag(rng.uniform(0.5, 1.5, size=c) * np.exp(1j * rng.uniform(0, 6.3, size=c))) for c in cutoff]
    S = hgf.define_system(s)
    op = hgf.map_operator(S, factors=fac, precision="fp64")
    info = op.info()
    assert info["untiled_functions"] == 0
    op.set_tile_config(0, 0)
    assert op.info()["untiled_functions"] == 1
    monkeypatch.setenv("HGF_STAGE_KERNEL", "generic")
    op2 = hgf.map_operator(S, factors=fac, precision="fp64")
    i2 = op2.info()
    assert i2["untiled_functions"] == i2["n_functions"] > 0


def test_stream_ceiling_helper(hgf):
    """The streaming-ceiling helper times the four stages on fresh buffers and
    refuses empty or over-large sizes."""
    announce("stream ceiling helper")
    us = hgf.stream_ceiling("mixed", True, 1 << 20, 3)
    assert len(us) == 4 and all(u > 0 for u in us)
    assert us[3] >= us[0] * 0.8  # stage 4 moves the most bytes
    for args in (("fp64", False, 0, 3), ("mixed", True, 1 << 20, 0), ("fp64", False, 1 << 29, 1)):
        with pytest.raises(hgf.HgfError) as e:
            hgf.stream_ceiling(*args)
        assert e.value.status == "HGF_EINVAL"
