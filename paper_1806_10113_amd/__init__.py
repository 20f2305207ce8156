"""tgo: task-group ordering on MI355X.

Exact evaluation of the temporal execution model of Lazaro-Munoz et al.
(Section 4) over launch orderings of offloaded task groups, and the ordering
heuristic of Section 5.1, as HIP kernels for gfx950 behind the C ABI in
include/tgo.h.  ``tgo`` holds the ctypes binding, ``workloads`` the seeded
input generators.
"""
__all__ = ["tgo", "workloads"]
