"""MI355X (gfx950) library for the Earth Mover's Distance misfit of seismic gathers
in the dynamic (Beckmann) formulation, solved by PDHG with linesearch
(Yong et al., arXiv 1808.07284, Sections 2.1-2.3, Algorithm 1).

The compute path is the C ABI of libemd_mi355x.so (include/emd_mi355x.h) over
hand-written HIP kernels; this package only marshals arguments into it.
"""
from ._lib import (EMDError, F32, F64, GATHER_STATUS, LS_FIXED, LS_L1, LS_L2,  # noqa: F401
                   MASS_BALANCE, MASS_NONE, MASS_UNIT)
from .api import (INFO_DTYPE, EMDMisfit, Multigrid, Plan, SolverParams, coarse_descs,  # noqa: F401
                  emd_adjoint_source, emd_decompose_noalloc,
                  emd_decompose, emd_misfit, emd_pdhg_solve, emd_pdhg_solve_replay,
                  emd_pdhg_solve_resume, info_numpy, lsd_misfit, prolong, residual_history, resolve_failed,
                  restrict, solver_state,
                  WarmStart)
