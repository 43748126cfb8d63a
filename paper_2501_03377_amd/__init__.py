"""MI355X-native tensor-structured PCG for the finite-difference Poisson
equation (arXiv 2501.03377): a HIP library with a C ABI (include/kpcg.h)
and this thin Python binding."""

from .kpcg import (Plan, Server, Ticket, KpError, KpResult, kp_basis_1d, kp_lowrank_table, kp_version, kp_strerror, BC, PREC,
                   KP_OK, KP_NOT_CONVERGED, KP_EINVAL, KP_ENOMEM, KP_EHIP, KP_ENONFINITE,
                   KP_EBREAKDOWN, KP_EBUSY, KP_FLAG_WARM_START, KP_FLAG_NO_PRECOND, KP_FLAG_FLEX_BETA, KP_FLAG_RESIDUAL_ONLY,
                   KP_FLAG_NO_GRAPH, KP_FLAG_DIAGNOSTICS, KP_FLAG_ANORM_STOP, DIAG_COLUMNS)

__all__ = ["Plan", "Server", "Ticket", "KpError", "KpResult", "kp_basis_1d", "kp_lowrank_table", "kp_version", "kp_strerror", "BC", "PREC",
           "KP_OK", "KP_NOT_CONVERGED", "KP_EINVAL", "KP_ENOMEM", "KP_EHIP", "KP_ENONFINITE",
           "KP_EBREAKDOWN", "KP_EBUSY", "KP_FLAG_WARM_START", "KP_FLAG_NO_PRECOND", "KP_FLAG_FLEX_BETA", "KP_FLAG_RESIDUAL_ONLY",
           "KP_FLAG_NO_GRAPH", "KP_FLAG_DIAGNOSTICS", "KP_FLAG_ANORM_STOP", "DIAG_COLUMNS"]
