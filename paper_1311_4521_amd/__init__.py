"""MI355X-native Wilson hopping matrix, even-odd twisted-mass operator and CG.

The computation lives in ``libtmhop.so`` (hand-written HIP for gfx950, C-ABI
in ``include/tmhop.h``); ``tmhop`` is its ctypes binding.
"""

from .tmhop import (EO, F16, F16_R12, F32, F32_R12, F64, F64_R12, OE, TMARCH, XSLAB, Lattice, TmhError, autotune_hop, autotune_mrhs,
                    batch_cg_solve, cg_solve, gauge_export, gauge_import, hop_apply, hop_apply_mrhs,
                    hop_force, lattice_create, norm2, profile_enable, profile_read, qtm_apply, qtm_apply_noalloc,
                    qtm_force,
                    scalar_prod_r, solve_full, spinor_export, spinor_import, status_string)

__all__ = ["EO", "OE", "XSLAB", "TMARCH", "F64", "F32", "F64_R12", "F32_R12", "F16", "F16_R12", "Lattice", "TmhError", "lattice_create",
           "gauge_import", "spinor_import", "spinor_export", "gauge_export", "hop_apply", "qtm_apply",
           "qtm_apply_noalloc",
           "cg_solve", "hop_force", "qtm_force", "solve_full", "hop_apply_mrhs", "batch_cg_solve",
           "autotune_mrhs", "autotune_hop", "profile_enable", "profile_read",
           "scalar_prod_r", "norm2", "status_string"]
