"""MI355X evaluator of the smoothed level-set function of a triangulated solid
(Vico, Greengard, O'Neil, Rachh): Phi / grad Phi at targets and the Newton
chart projection onto Phi = 1/2, as HIP kernels for gfx950 behind the C ABI
of include/lss.h.  This module is argument marshalling only."""
from ._binding import (Context, LssError, load_library, library_path, FP64, MIXED,
                       FAR_DIRECT, FAR_FMM, NODE_CONVERGED, NODE_MAXITER, NODE_NOBRACKET,
                       NODE_DEGENERATE_H, TRI6, EXPORTED_SYMBOLS, default_rule)

__all__ = ["Context", "LssError", "load_library", "library_path", "FP64", "MIXED",
           "FAR_DIRECT", "FAR_FMM", "NODE_CONVERGED", "NODE_MAXITER", "NODE_NOBRACKET",
           "NODE_DEGENERATE_H", "TRI6", "EXPORTED_SYMBOLS", "default_rule"]
