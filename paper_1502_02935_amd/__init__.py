"""MI355X-native ideal-MHD TVD-MUSCL step (HIP kernels behind a C ABI).

    from paper_1502_02935_amd import Sim, config_from_problem
"""
from ._lib import (MHD_FP32, MHD_FP64, BC_INFLOW, BC_OUTFLOW, BC_PERIODIC,  # noqa: F401
                   RECON_FIRST, RECON_KAPPA, RECON_PAPER, MHDError, load)
from .sim import MHDConfig, Sim, config_from_problem, hlld_batch, recon_batch  # noqa: F401
from .sim import workspace_bytes, mlp_forward, MlpTrainer  # noqa: F401
