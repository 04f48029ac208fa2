"""MI355X click-pattern probabilities of a lossy Gaussian boson sampler.

The computation lives in libgbs.so (HIP, gfx950); see include/gbs.h for the C
ABI and gbs.py for the Python binding.  torch_api.py wraps the device calls as
a torch.autograd.Function.
"""
from .gbs import (Context, Plan, GBSError, load, LIB_PATH, GBS_PREC_FP64,  # noqa: F401
                  GBS_PREC_MIXED)
