"""MI355X-native Picard / PCG hot path of the RichardsFOAM method
(Orgogozo et al., arXiv:1809.10895) behind the C ABI of include/rf.h, and
the column ensemble of include/rf_ensemble.h.

    from paper_1809_10895_amd import Solver, Ensemble, workloads
"""
from .binding import (Ensemble, Guess, RF_DIRICHLET, RF_FLUX, RF_FREE_DRAINAGE, RF_GARDNER, RF_NOFLOW,  # noqa: F401
                      RF_PRECOND_JACOBI, RF_PRECOND_ZLINE, RF_VGM, RF_XMAX, RF_XMIN, RF_YMAX,
                      RF_YMIN, RF_ZMAX, RF_ZMIN, RfError, Solver, default_options, load_library)
