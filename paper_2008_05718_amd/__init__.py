"""Exact Brandes betweenness centrality on one AMD Instinct MI355X (gfx950).

The computation lives in the HIP library ``libbc.so`` (C ABI in
``include/bc.h``); ``binding`` wraps it with ctypes.  ``workloads`` builds the
seeded synthetic input graphs.  Importing the package loads nothing; the first
call into ``binding`` loads libbc.so and fails loudly if it is not built.
"""
__all__ = ["binding", "workloads", "build"]
