"""MI355X (gfx950) implementation of the lattice Omega_GW path of arXiv 2605.27231.

The computation lives in the HIP library ``libsigw.so`` behind the C ABI of
``include/sigw.h``; this package holds its build script, a ctypes binding
with the same entry-point names, and the batching/serving layers on top.
"""
from ._lib import SigwError, lib  # noqa: F401
from .api import Plan, plan_desc, sigw_kernel_table, sigw_kernel_table_w, sigw_plan_footprint  # noqa: F401

__all__ = ["Plan", "plan_desc", "sigw_kernel_table", "sigw_kernel_table_w", "sigw_plan_footprint", "SigwError",
           "lib"]
