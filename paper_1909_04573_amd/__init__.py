"""MI355X (gfx950) SDA camera-fingerprint path: HIP kernels behind the C ABI
of include/prnu.h, with a thin ctypes binding in :mod:`.prnu`."""
from . import prnu  # noqa: F401

__all__ = ["prnu"]
