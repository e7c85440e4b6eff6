"""MI355X-native matrix-free element loop of the Cahn-Hilliard Navier-Stokes
method of Khanwale et al. (arXiv 1912.12453).

The compute path is the C-ABI library ``libchns.so`` (hand-written HIP for
gfx950); :mod:`.chns` is its thin ctypes binding and :mod:`.workloads` holds
the seeded synthetic inputs.
"""
__all__ = ["chns", "workloads"]
