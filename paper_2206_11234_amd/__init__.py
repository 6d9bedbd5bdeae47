"""MI355X-native importance-sampled first-passage engine for stochastic inflation.

Method: Jackson, Assadullahi, Koyama, Vennin, Wands, arXiv:2206.11234.
The hot path (Euler-Maruyama stepping with a drift bias and its importance
weight, first passage, weighted N-histogram with log-sum-exp merges) runs in
hand-written HIP kernels for gfx950 behind the C ABI of include/pyfpt.h;
this package is the thin Python binding over it.
"""
from ._lib import (BIAS_MLP, BIAS_NOISE_SCALED, BIAS_NONE, BIAS_POWER, POT_FLAT, POT_QUADRATIC,
                   POT_QUADRATIC_BUMP, ST_CENSORED, ST_ENDED, ST_ESCAPED, PyfptError)
from .api import (COMBINE_NO_EXTRAPOLATION, Dump, Records, Result, combine, device_cus, layout, mlp_forward, proposal_loss_grad, proposal_records,
                  run, run_batch, run_single_abi, train_proposal)

__all__ = ["COMBINE_NO_EXTRAPOLATION", "combine", "run", "run_batch", "run_single_abi", "layout", "device_cus", "mlp_forward", "proposal_records",
           "proposal_loss_grad", "train_proposal", "Result", "Dump", "Records", "PyfptError",
           "POT_QUADRATIC", "POT_QUADRATIC_BUMP", "POT_FLAT", "BIAS_NONE", "BIAS_NOISE_SCALED", "BIAS_POWER",
           "BIAS_MLP", "ST_ENDED", "ST_CENSORED", "ST_ESCAPED"]
