"""MI355X (gfx950) log-polar hyperbolic Radon transform.

The transform runs in libhrt.so (HIP kernels behind the C ABI of
include/hrt.h); this package only marshals arguments."""
from ._lib import HrtError, load as load_library  # noqa: F401


def __getattr__(name):
    # torch-dependent parts load lazily so that the C ABI can be used without
    # importing torch
    if name in ("Plan", "HRTFunction", "hrt_forward", "describe"):
        from . import hrt
        return getattr(hrt, name)
    raise AttributeError(name)
