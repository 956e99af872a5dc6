"""Python binding of libhgf (ctypes): argument marshalling only.

Every numerical step runs in the HIP library; this module converts Python
and numpy arguments into the C structures of ``include/hgf.h`` and passes
torch's current HIP stream.  It fails loudly when the library is missing.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgf.so")

HGF_FP64, HGF_MIXED = 0, 1
HGF_MERGED, HGF_SPLIT, HGF_SEPARATED, HGF_SEPARATED_EXACT = 0, 1, 2, 3
HGF_OP_PRODUCT, HGF_OP_SPARSE, HGF_OP_DENSE = 0, 1, 2
HGF_BASIS_NUMBER, HGF_BASIS_NORMAL = 0, 1
HGF_PSI_FOCK, HGF_PSI_COHERENT, HGF_PSI_PRODUCT = 0, 1, 2

STATUS = {0: "HGF_OK", -1: "HGF_EINVAL", -2: "HGF_ENOMEM", -3: "HGF_EDEVICE", -4: "HGF_EUNSTABLE",
          -5: "HGF_ENONFINITE", -6: "HGF_EUNSUPPORTED", -7: "HGF_ESTATE"}

EXPORTED = ["hgf_define_system", "hgf_destroy_system", "hgf_num_params", "hgf_map_operator",
            "hgf_destroy_operator", "hgf_evolve", "hgf_evolve_batch", "hgf_expectation", "hgf_expectation_noalloc",
            "hgf_reconstruct", "hgf_grad", "hgf_set_threshold", "hgf_stream_ceiling",
            "hgf_get_info", "hgf_get_function", "hgf_last_error", "hgf_version"]


class HgfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_i32p = ctypes.POINTER(ctypes.c_int32)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)
_f64p = ctypes.POINTER(ctypes.c_double)


class _SystemDesc(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int32), ("cutoff", _i32p), ("detuning", _f64p), ("kerr", _f64p),
                ("cross_kerr", _f64p), ("gamma1", _f64p), ("gamma_phi", _f64p), ("n_th", _f64p),
                ("dissipator", ctypes.c_int32), ("n_th_levels", _f64p), ("drive", _f64p), ("exchange", _f64p)]


HGF_DISS_LINDBLAD, HGF_DISS_SECULAR = 0, 1
_DISS = {"lindblad": HGF_DISS_LINDBLAD, "secular": HGF_DISS_SECULAR}


class _OperatorDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("basis", ctypes.c_int32), ("values", _f64p),
                ("indices", _i32p), ("n_terms", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("drop_tol", ctypes.c_double)]


class _StateDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("fock", _i32p), ("alpha", _f64p), ("amps", _f64p)]


class _Info(ctypes.Structure):
    _fields_ = [("n_functions", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("total_points", ctypes.c_int64), ("steps_done", ctypes.c_int64),
                ("time_us", ctypes.c_double), ("fp32_underflow", ctypes.c_int64),
                ("error_state", ctypes.c_int32), ("real_functions", ctypes.c_int32),
                ("stored_peak", ctypes.c_int64), ("untiled_functions", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("stored_tiles_peak", ctypes.c_int64),
                ("tile_points", ctypes.c_int64)]


class _TileConfig(ctypes.Structure):
    _fields_ = [("nfast", ctypes.c_int32), ("threads", ctypes.c_int32), ("xblock", ctypes.c_int32),
                ("pipe", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32), ("resident", ctypes.c_int32),
                ("walk_block", ctypes.c_int32), ("blocks", ctypes.c_int32), ("tile_points", ctypes.c_int32), ("stage_us", ctypes.c_double)]


TUNE_FLAGS = {"default": 0, "cached_only": 1, "force": 2}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhgf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhgf.so not found at {path}; build it with "
                           "`python -m paper_2203_05526_amd.build`")
    # torch brings its own HIP runtime; load it first so that libhgf binds to
    # the same one and torch's streams and allocator are valid for it
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.hgf_define_system.argtypes = [ctypes.POINTER(_SystemDesc), ctypes.POINTER(vp)]
    lib.hgf_destroy_system.argtypes = [vp]
    lib.hgf_destroy_system.restype = None
    lib.hgf_num_params.argtypes = [vp]
    lib.hgf_map_operator.argtypes = [vp, ctypes.POINTER(_OperatorDesc), ctypes.POINTER(vp)]
    lib.hgf_destroy_operator.argtypes = [vp]
    lib.hgf_destroy_operator.restype = None
    lib.hgf_evolve.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp]
    lib.hgf_clear_error.argtypes = [vp]
    lib.hgf_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
    lib.hgf_evolve_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, _f64p, _f64p, vp]
    lib.hgf_expectation.argtypes = [vp, ctypes.POINTER(_StateDesc), _f64p, vp]
    lib.hgf_expectation_noalloc.argtypes = [vp, ctypes.POINTER(_StateDesc), _f64p, vp]
    lib.hgf_reconstruct.argtypes = [vp, ctypes.c_int32, _f64p, vp]
    lib.hgf_grad.argtypes = [vp, ctypes.POINTER(_OperatorDesc), ctypes.POINTER(_StateDesc),
                             ctypes.c_double, ctypes.c_double, ctypes.c_int32, _f64p, _f64p, vp]
    lib.hgf_get_info.argtypes = [vp, ctypes.POINTER(_Info)]
    lib.hgf_set_threshold.argtypes = [vp, ctypes.c_double]
    lib.hgf_get_function.argtypes = [vp, ctypes.c_int32, _i32p, _i32p, _f64p, ctypes.c_int64, _f64p, vp]
    lib.hgf_get_tile_config.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(_TileConfig)]
    lib.hgf_set_tile_config.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(_TileConfig)]
    lib.hgf_autotune.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_double, ctypes.c_char_p,
                                 ctypes.c_int32, vp]
    lib.hgf_last_error.restype = ctypes.c_char_p
    lib.hgf_last_error.argtypes = []
    lib.hgf_version.restype = ctypes.c_char_p
    lib.hgf_version.argtypes = []
    lib.hgf_stream_ceiling.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), vp]
    for name in EXPORTED:
        if not hasattr(lib, name):
            raise RuntimeError(f"libhgf.so does not export {name}")
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = _lib.hgf_last_error().decode()
        raise HgfError(rc, msg)


def _stream(stream) -> Optional[int]:
    """A hipStream_t as an integer: an explicit int, a torch stream, or torch's
    current stream on the current device."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream) or None
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))


def _i32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1))


def _cplx_flat(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(-1))
    return a.view(np.float64)


# ------------------------------------------------------------------ system

class System:
    """A handle on hgf_system (copy of the parameters, validated)."""

    def __init__(self, cutoff, detuning, kerr, cross_kerr, gamma1, gamma_phi, n_th, dissipator="lindblad",
                 n_th_levels=None, drive=None, exchange=None):
        lib = load_library()
        n = len(cutoff)
        self.n_modes = n
        self.cutoff = tuple(int(c) for c in cutoff)
        self._arrays = [_i32(cutoff), _f64(detuning), _f64(kerr), _f64(cross_kerr), _f64(gamma1),
                        _f64(gamma_phi), _f64(n_th)]
        for a, ln in zip(self._arrays, (n, n, n, n * n, n, n, n)):
            if a.size != ln:
                raise HgfError(-1, "system array has the wrong length")
        levels = None
        if n_th_levels is not None:
            levels = _f64(n_th_levels)
            if levels.size != sum(c - 1 for c in self.cutoff):
                raise HgfError(-1, "n_th_levels needs sum(cutoff - 1) values")
            self._arrays.append(levels)
        net = []
        for x, ln in ((drive, n), (exchange, n * n)):
            if x is None:
                net.append(None)
                continue
            a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128 if ln == n else np.float64).reshape(-1))
            if a.size != ln:
                raise HgfError(-1, "drive needs N complex values and exchange N*N values")
            a = a.view(np.float64) if ln == n else a
            self._arrays.append(a)
            net.append(a.ctypes.data_as(_f64p))
        self.network = any(x is not None for x in net)
        d = _SystemDesc(n, *(a.ctypes.data_as(_i32p if i == 0 else _f64p) for i, a in enumerate(self._arrays[:7])),
                        _DISS[dissipator], levels.ctypes.data_as(_f64p) if levels is not None else None, *net)
        h = ctypes.c_void_p()
        _check(lib.hgf_define_system(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def num_params(self) -> int:
        return int(_lib.hgf_num_params(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hgf_destroy_system(self._h)
            self._h = None


def define_system(system) -> System:
    """hgf_define_system from an object with cutoff, detuning, kerr,
    cross_kerr, gamma1, gamma_phi and n_th (e.g. ``synth.System``)."""
    return System(system.cutoff, system.detuning, system.kerr, system.cross_kerr, system.gamma1,
                  system.gamma_phi, system.n_th, getattr(system, "dissipator", "lindblad"),
                  getattr(system, "n_th_levels", None), getattr(system, "drive", None),
                  getattr(system, "exchange", None))


# ------------------------------------------------------------------ operators

_PREC = {"fp64": HGF_FP64, "mixed": HGF_MIXED}
_LAYOUT = {"merged": HGF_MERGED, "split": HGF_SPLIT, "separated": HGF_SEPARATED, "separated_exact": HGF_SEPARATED_EXACT}
_BASIS = {"number": HGF_BASIS_NUMBER, "normal": HGF_BASIS_NORMAL}


def _operator_desc(system: System, factors=None, sparse=None, basis="number", precision="fp64",
                   layout="merged", drop_tol=0.0, dense=None):
    keep = []
    if sum(x is not None for x in (factors, sparse, dense)) != 1:
        raise HgfError(-1, "give exactly one of factors=, sparse= or dense=")
    if dense is not None:
        dim = int(np.prod(system.cutoff))
        if np.shape(dense) != (dim, dim):
            raise HgfError(-1, "dense operator shape does not match the truncated space")
        vals = _cplx_flat(dense)
        keep.append(vals)
        d = _OperatorDesc(HGF_OP_DENSE, _BASIS[basis], vals.ctypes.data_as(_f64p), None, 0,
                          _PREC[precision], _LAYOUT[layout], float(drop_tol))
    elif factors is not None:
        if len(factors) != system.n_modes:
            raise HgfError(-1, "one factor per mode is needed")
        for f, nc in zip(factors, system.cutoff):
            if np.shape(f) != (nc, nc):
                raise HgfError(-1, "factor shape does not match the cutoff")
        vals = np.concatenate([_cplx_flat(f) for f in factors])
        keep.append(vals)
        d = _OperatorDesc(HGF_OP_PRODUCT, _BASIS[basis], vals.ctypes.data_as(_f64p), None, 0,
                          _PREC[precision], _LAYOUT[layout], float(drop_tol))
    else:
        ks, ls, values = sparse
        ks = np.asarray(ks, dtype=np.int32).reshape(-1, system.n_modes)
        ls = np.asarray(ls, dtype=np.int32).reshape(-1, system.n_modes)
        idx = _i32(np.concatenate([ks, ls], axis=1))
        vals = _cplx_flat(values)
        keep += [idx, vals]
        d = _OperatorDesc(HGF_OP_SPARSE, _BASIS[basis], vals.ctypes.data_as(_f64p), idx.ctypes.data_as(_i32p),
                          ks.shape[0], _PREC[precision], _LAYOUT[layout], float(drop_tol))
    return d, keep


class Operator:
    def __init__(self, handle, system: System):
        self._h = handle
        self.system = system

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _Info()
        _check(_lib.hgf_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    def function(self, idx: int, stream=None):
        """(sector d, extents, grid as complex128 ndarray, split info or None)."""
        n = self.system.n_modes
        d = np.zeros(n, dtype=np.int32)
        e = np.zeros(n, dtype=np.int32)
        _check(_lib.hgf_get_function(self._h, idx, d.ctypes.data_as(_i32p), e.ctypes.data_as(_i32p), None, 0,
                                     None, None))
        grid = np.zeros(int(np.prod(e)), dtype=np.complex128)
        extra = np.zeros(4 * n + 6)
        _check(_lib.hgf_get_function(self._h, idx, None, None, grid.view(np.float64).ctypes.data_as(_f64p),
                                     grid.size, extra.ctypes.data_as(_f64p), _stream(stream)))
        split = {"p": extra[:n].astype(int), "q": extra[n:2 * n].astype(int),
                 "g0": complex(extra[2 * n], extra[2 * n + 1]),
                 "cx": complex(extra[2 * n + 2], extra[2 * n + 3]),
                 "cy": complex(extra[2 * n + 4], extra[2 * n + 5])}
        return tuple(int(x) for x in d), tuple(int(x) for x in e), grid.reshape(tuple(e)), split

    def tile_config(self, idx: int) -> dict:
        """hgf_get_tile_config: launch shape of function ``idx``."""
        c = _TileConfig()
        _check(_lib.hgf_get_tile_config(self._h, idx, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in _TileConfig._fields_}

    def set_tile_config(self, idx: int, nfast: int, threads: int = 0, xblock: int = 0, pipe: int = 0,
                        wgs_per_cu: int = 0, resident: int = 0, walk_block: int = 0) -> None:
        """hgf_set_tile_config: force the launch shape of function ``idx``."""
        c = _TileConfig(nfast, threads, xblock, pipe, wgs_per_cu, resident, walk_block, 0, 0, 0.0)
        _check(_lib.hgf_set_tile_config(self._h, idx, ctypes.byref(c)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hgf_destroy_operator(self._h)
            self._h = None


def map_operator(system: System, factors=None, sparse=None, basis="number", precision="fp64",
                 layout="merged", drop_tol=0.0, dense=None) -> Operator:
    """hgf_map_operator: ``factors`` is a list of per-mode (Nc, Nc) matrices of
    a product operator; ``sparse`` is (k[T, N], l[T, N], values[T]); ``dense``
    is a (D, D) matrix over the whole truncated space (D = prod Nc, last mode
    fastest)."""
    d, keep = _operator_desc(system, factors, sparse, basis, precision, layout, drop_tol, dense)
    h = ctypes.c_void_p()
    _check(_lib.hgf_map_operator(system.handle, ctypes.byref(d), ctypes.byref(h)))
    return Operator(h, system)


SCHEMES = {"rk4": 0, "lawson": 1}  # HGF_RK4, HGF_LAWSON_RK4


def evolve(op: Operator, t_total: float, dt: float, stream=None, scheme: str = "rk4") -> None:
    """hgf_evolve with scheme "rk4" (classical RK4) or "lawson" (integrating-factor RK4)."""
    _check(_lib.hgf_evolve(op.handle, float(t_total), float(dt), SCHEMES[scheme], _stream(stream)))


def set_threshold(op: Operator, threshold: float) -> None:
    """hgf_set_threshold: after every step, drop the coefficients with |g| <=
    threshold (0 turns it off); op.info()["stored_peak"] reports the largest
    number kept since."""
    _check(_lib.hgf_set_threshold(op.handle, float(threshold)))


def clear_error(op: Operator) -> None:
    """hgf_clear_error: leave the error state after HGF_ENONFINITE."""
    _check(_lib.hgf_clear_error(op.handle))


_hooks = None  # keeps the ctypes callbacks alive while registered


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device allocations through torch's caching
    allocator (hgf_set_allocator), or back to hipMalloc.  Blocks allocated
    while the hook is set return to torch when freed; at interpreter exit the
    hook is removed first, so that later frees do not call back into a
    finalising interpreter."""
    global _hooks
    import torch

    if not enable:
        _check(_lib.hgf_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        _hooks = None
        return

    def alloc(nbytes, device, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device),
                                                      stream=torch.cuda.current_stream(int(device)))
        except Exception:
            return None

    def free(ptr, device, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    hooks = (_ALLOC_FN(alloc), _FREE_FN(free))
    _check(_lib.hgf_set_allocator(hooks[0], hooks[1], None))
    if _hooks is None:
        import atexit
        atexit.register(_drop_hooks)
    _hooks = hooks


def _drop_hooks() -> None:
    global _hooks
    if _hooks is not None and _lib is not None:
        _lib.hgf_set_allocator(_ALLOC_FN(), _FREE_FN(), None)
        _hooks = None


def evolve_batch(ops: Sequence[Operator], t_total, dt, stream=None) -> None:
    n = len(ops)
    arr = (ctypes.c_void_p * n)(*[o.handle.value for o in ops])
    t = _f64(np.broadcast_to(np.asarray(t_total, dtype=np.float64), (n,)))
    h = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)))
    _check(_lib.hgf_evolve_batch(arr, n, t.ctypes.data_as(_f64p), h.ctypes.data_as(_f64p), _stream(stream)))


def autotune(ops: Sequence[Operator], dt: float, cache: Optional[str] = None, mode: str = "default",
             stream=None) -> None:
    """hgf_autotune: measure (or load from the text cache ``cache``) the
    fastest stage-kernel launch shape of every grid shape among ``ops`` for
    steps of ``dt``; mode is "default", "cached_only" or "force"."""
    n = len(ops)
    arr = (ctypes.c_void_p * max(n, 1))(*[o.handle.value for o in ops])
    path = cache.encode() if cache else None
    _check(_lib.hgf_autotune(arr, n, float(dt), path, TUNE_FLAGS[mode], _stream(stream)))


def _state_desc(system: System, state):
    kind, vals = state
    keep = []
    if kind == "fock":
        a = _i32(vals)
        keep.append(a)
        return _StateDesc(HGF_PSI_FOCK, a.ctypes.data_as(_i32p), None, None), keep
    if kind == "coherent":
        a = _cplx_flat(vals)
        keep.append(a)
        return _StateDesc(HGF_PSI_COHERENT, None, a.ctypes.data_as(_f64p), None), keep
    if kind == "product":
        a = np.concatenate([_cplx_flat(v) for v in vals])
        keep.append(a)
        return _StateDesc(HGF_PSI_PRODUCT, None, None, a.ctypes.data_as(_f64p)), keep
    raise HgfError(-1, f"unknown state kind {kind}")


def expectation(op: Operator, state, stream=None) -> complex:
    d, keep = _state_desc(op.system, state)
    out = np.zeros(2)
    _check(_lib.hgf_expectation(op.handle, ctypes.byref(d), out.ctypes.data_as(_f64p), _stream(stream)))
    return complex(out[0], out[1])


def expectation_noalloc(op: Operator, state, stream=None) -> complex:
    """hgf_expectation_noalloc: the same value as expectation(), with every
    device buffer taken from the library's static device scratch (no device
    allocation; operators needing more than its 4 MiB are refused)."""
    d, keep = _state_desc(op.system, state)
    out = np.zeros(2)
    _check(_lib.hgf_expectation_noalloc(op.handle, ctypes.byref(d), out.ctypes.data_as(_f64p), _stream(stream)))
    return complex(out[0], out[1])


def reconstruct(op: Operator, levels: int, stream=None) -> np.ndarray:
    """hgf_reconstruct: <k|A(t)|l> for all occupations below ``levels``, as a
    (levels^N, levels^N) complex matrix (last mode fastest)."""
    n = op.system.n_modes
    ln = int(levels) ** n
    out = np.zeros(2 * ln * ln)
    _check(_lib.hgf_reconstruct(op.handle, int(levels), out.ctypes.data_as(_f64p), _stream(stream)))
    return out.view(np.complex128).reshape(ln, ln)


def grad(system: System, state, t_total: float, dt: float, factors=None, sparse=None, basis="number",
         checkpoint_every: int = 100, stream=None, dense=None) -> Tuple[complex, np.ndarray]:
    """hgf_grad: (J, dJ/dtheta) with theta = K[N], chi[i<j], Delta[N], gamma1[N], gamma_phi[N]."""
    od, keep = _operator_desc(system, factors, sparse, basis, "fp64", "merged", 0.0, dense)
    sd, keep2 = _state_desc(system, state)
    P = system.num_params()
    val = np.zeros(2)
    g = np.zeros(2 * P)
    _check(_lib.hgf_grad(system.handle, ctypes.byref(od), ctypes.byref(sd), float(t_total), float(dt),
                         int(checkpoint_every), val.ctypes.data_as(_f64p), g.ctypes.data_as(_f64p),
                         _stream(stream)))
    return complex(val[0], val[1]), g.view(np.complex128).copy()


def version() -> str:
    return load_library().hgf_version().decode()


def stream_ceiling(precision: str, real: bool, points: int, reps: int = 10, stream=None) -> List[float]:
    """hgf_stream_ceiling: microseconds per launch of each Horner stage when its
    operands are streamed once per point with no neighbour reads (the stage
    kernel's streaming ceiling; a measurement helper)."""
    us = (ctypes.c_double * 4)()
    _check(_lib.hgf_stream_ceiling(_PREC[precision], 1 if real else 0, int(points), int(reps), us,
                                   _stream(stream)))
    return [us[i] for i in range(4)]


def param_names(n: int) -> List[str]:
    names = [f"kerr[{j}]" for j in range(n)]
    names += [f"chi[{i},{j}]" for i in range(n) for j in range(i + 1, n)]
    names += [f"detuning[{j}]" for j in range(n)]
    names += [f"gamma1[{j}]" for j in range(n)]
    names += [f"gamma_phi[{j}]" for j in range(n)]
    return names


def params_vector(system) -> np.ndarray:
    """theta in hgf_num_params order from a parameter object."""
    n = len(system.cutoff)
    chi = [system.cross_kerr[i][j] for i in range(n) for j in range(i + 1, n)]
    return np.concatenate([np.asarray(system.kerr, float), np.asarray(chi, float),
                           np.asarray(system.detuning, float), np.asarray(system.gamma1, float),
                           np.asarray(system.gamma_phi, float)])
