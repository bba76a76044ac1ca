"""MI355X codon-constrained McCaskill partition function (HIP library + binding).

The compute path is ``libcdz.so`` (hand-written HIP for gfx950, C ABI in
``include/cdz.h``); this package only marshals arguments to it
(:mod:`.binding`), builds it (:mod:`.build`), wraps the adjoint as a
``torch.autograd.Function`` (:mod:`.autograd`) and draws seeded synthetic
inputs (:mod:`.inputs`).
"""
from . import inputs  # noqa: F401
from .binding import (CdzError, cdz_backward_dev, cdz_create, cdz_forward_dev,  # noqa: F401
                      cdz_last_error, cdz_last_timings, cdz_marginals, cdz_partition,
                      cdz_sample, cdz_status_string)
