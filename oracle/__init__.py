"""Plain FP64 CPU oracle for randUTV (Alg. 3), randUTV_boosted (Alg. 2),
powerURV (Alg. 1) and the RSVD.

TEST INFRASTRUCTURE, not product code. Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import, call or run anything in this package. It shares no code with the HIP
library in ``paper_2106_13402_amd`` and never imports it.
"""
from .philox import gaussian, philox4x64_10
from .hqr import apply_q, form_q, hqr
from .small_svd import canonical_signs, small_svd
from .randutv import randutv, randutv_partial
from .randutv_boosted import randutv_boosted
from .powerurv import powerurv
from .rsvd import rsvd
from . import metrics

__all__ = [
    "gaussian", "philox4x64_10", "hqr", "apply_q", "form_q",
    "small_svd", "canonical_signs", "randutv", "randutv_partial", "randutv_boosted", "powerurv", "rsvd", "metrics",
]
