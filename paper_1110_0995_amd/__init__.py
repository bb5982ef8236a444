"""MI355X (gfx950) D3Q19 lattice-Boltzmann + immersed-boundary cell-flow step.

The hot path runs in the HIP library ``liblbmibm.so`` (C ABI in
``include/lbmibm.h``); ``lbm.Lattice`` / ``lbm.Mesh`` are its thin Python
front end, ``scenario`` builds the seeded synthetic inputs.
"""

__all__ = ["scenario", "lbm", "build"]


def __getattr__(name):
    if name in ("Lattice", "Mesh"):
        from . import lbm
        return getattr(lbm, name)
    raise AttributeError(name)
