"""MI355X-native hydrodynamic (nonlocal Drude / GNOR) FDTD.

The compute path lives in the HIP library ``libgnorfdtd.so`` (C-ABI, see
``include/gnor_fdtd.h``); :mod:`paper_2005_06997_amd.binding` marshals
arguments to it.  :mod:`paper_2005_06997_amd.workloads` draws the seeded
synthetic problems.
"""
__all__ = ["binding", "workloads"]
