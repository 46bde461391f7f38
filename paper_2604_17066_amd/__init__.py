"""MI355X (gfx950) implementation of the Stage-2 hot path of the Reference-state
System Reliability method (Byun, Ryu & Song, arXiv 2604.17066).

The compute lives in librsr.so (HIP kernels behind the C ABI of
include/rsr.h); this package only marshals arguments.  Importing the package
does not need a GPU; creating a Context does, and there is no CPU fallback.
"""
from ._abi import (  # noqa: F401
    RSR_OK, RSR_EINVAL, RSR_ENOMEM, RSR_EHIP, RSR_EUNSUPPORTED, RSR_LABEL, RSR_COUNT, RSR_AUTO,
    RSR_POPCOUNT, RSR_MFMA, RSR_MFMA_FP4, RSR_PERSIST, RSR_UNKNOWN_ONLY, RSR_ALL,
    RSR_SYS_HOST_CALLBACK,
    RSRError, lib,
)
from .api import (  # noqa: F401
    Context, Model, Refs, System, Buffers, Plan, alloc_samples, rsr_sample, rsr_classify,
    rsr_eval_unknown, rsr_estimate, rsr_grad, rsr_importance, rsr_boundary_search, stage1, stage2,
)
from .autograd import RSRProbability, rsr_probability  # noqa: F401
