"""MI355X (gfx950) generating-function solver for the adjoint Lindblad master
equation of damped Kerr-coupled bosonic modes (arXiv:2203.05526).

The numerical work runs in the HIP library ``libhgf.so`` (C ABI in
``include/hgf.h``); this package is its Python binding.
"""

from .hgf import (  # noqa: F401
    HgfError,
    Operator,
    System,
    autotune,
    clear_error,
    define_system,
    evolve,
    evolve_batch,
    expectation,
    expectation_noalloc,
    reconstruct,
    set_threshold,
    stream_ceiling,
    grad,
    load_library,
    map_operator,
    param_names,
    params_vector,
    use_torch_allocator,
    version,
)
