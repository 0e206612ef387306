"""K-GRAPE hot path on MI355X (gfx950): Krylov-Lanczos propagation of an open
XXZ spin chain under piecewise-constant control and the GRAPE gradient
(Larocca & Wisniacki, arXiv 2010.03598).

The compute lives in libkgrape.so (hand-written HIP kernels behind the C ABI of
include/kgrape.h); this package is its Python binding.
"""

from ._lib import (KG_C64, KG_C128, KG_HC_SX, KG_HC_SZ, KgError, LIB_PATH,  # noqa: F401
                   load as load_library)
from .autograd import GrapeFidelity, fidelity  # noqa: F401
from .api import (XXZ, GrapeResult, Krylov, Workspace, debug_index_map, profile,  # noqa: F401
                  grape_ascent_update, grape_forward, grape_gradient, grape_gradient_columns,
                  krylov_expv, new_states,
                  states_bytes, xxz_apply)
from .reduced import (ReducedBasis, ReducedWorkspace, grape_forward_pe,  # noqa: F401
                      grape_gradient_pe, krylov_expv_pe, pe_dim, pe_states, pe_tables_host,
                      xxz_pe_apply)

__all__ = [
    "XXZ", "Krylov", "Workspace", "GrapeResult", "xxz_apply", "krylov_expv", "grape_forward",
    "grape_gradient_columns",
    "grape_gradient", "grape_ascent_update", "debug_index_map", "new_states", "states_bytes",
    "KG_C64", "KG_C128", "KG_HC_SX", "KG_HC_SZ", "KgError", "load_library", "LIB_PATH", "profile",
    "GrapeFidelity", "fidelity", "ReducedBasis", "ReducedWorkspace", "pe_dim", "pe_states",
    "pe_tables_host", "xxz_pe_apply", "krylov_expv_pe", "grape_forward_pe", "grape_gradient_pe",
]
