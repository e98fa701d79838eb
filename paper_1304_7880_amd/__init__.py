"""MI355X-native weighted-density lattice Boltzmann (WDLB) step.

The GPU library (libwdlb.so, hand-written HIP for gfx950 behind a C ABI) is
loaded lazily by :mod:`paper_1304_7880_amd.wdlb`; importing the package or
its seeded :mod:`workloads` touches no GPU.
"""
__all__ = ["wdlb", "workloads"]
