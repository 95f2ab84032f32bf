"""MI355X (gfx950) CNT-GW hot path: entropic Gromov-Wasserstein solves for
conditionally-negative-type penalties (Algorithm 1 of "Gromov-Wasserstein at
Scale, Beyond Squared Norms"), with the N x M cost never stored.

The compute runs in ``libgwmi.so`` (hand-written HIP kernels behind the C ABI
of ``include/gw.h``); this package only marshals arguments.
"""
from . import _lib  # noqa: F401
from ._lib import GWError, LIB_PATH, load, seeded_landmarks  # noqa: F401


def __getattr__(name):
    # torch-dependent parts load lazily so that the C ABI can be inspected
    # without a GPU
    if name in ("Context", "make_params"):
        from . import api
        return getattr(api, name)
    if name in ("GWLoss", "gw_loss"):
        from . import autograd
        return getattr(autograd, name)
    if name in ("Server",):
        from . import serve
        return getattr(serve, name)
    raise AttributeError(name)
