"""MI355X (gfx950) implementation of the SARABANDE 3/4PCF hot path (arXiv 2210.10206).

The computation runs in the HIP library ``libsarabande_hip.so`` (C ABI in
``include/sarabande_hip.h``); this package only marshals arguments and owns
device memory through torch.
"""
from ._lib import SbError, load  # noqa: F401


def __getattr__(name):
    # torch-dependent front end, imported on first use
    if name in ("Plan", "measure", "ZetaFn", "normalization"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
