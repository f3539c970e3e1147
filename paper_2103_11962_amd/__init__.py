"""Regional multigrid preconditioned CG for semi-structured grids on MI355X (HIP, gfx950).

``regmg`` is the ctypes binding of the C ABI declared in ``include/regmg.h``.
"""
from . import regmg  # noqa: F401
