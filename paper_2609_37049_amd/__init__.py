"""libdisco for MI355X: the hot path of the subtraction method for
disconnected diagrams (Wilson-clover D and D_Lambda inversions on
distillation sources, perambulators, loops, correlators) as HIP kernels for
gfx950 behind a C ABI (include/disco.h).  This package holds the HIP sources
(csrc/), the in-tree build, and a thin ctypes binding."""
from .binding import (  # noqa: F401
    Context, Domains, Net, DiscoError, SolverParams, SolverStats, TrainParams, TrainStats, lib, exported_symbols,
    F64, F32, BF16, G_1, G_5, G_X, G_Y, G_Z, G_TILDE, EPI_DOTAUX, EPI_NORM, EPI_DOTIN, EPI_DOTAUXIN, CGNR_F64, BICGSTAB_DC, FGMRES_NN, BICGSTAB_RU, K_STENCIL, K_NN, K_STENCIL_F64, K_STENCIL_F32, K_STENCIL_BF16, K_MFMA, OPT_GRAPHS, OPT_STAGE, OPT_EO, OPT_TILE_Y, OPT_TILE_T, OPT_NARROW,
    K_STENCIL_EO_F64, K_STENCIL_EO_F32, K_STENCIL_EO_BF16,
    OK, EINVAL, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, ESTATE,
)
