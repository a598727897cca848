"""MI355X (gfx950) simplified string method for atomistic spin lattices.

Modules: ssm (binding of libssm.so, the C ABI in include/ssm.h), inputs
(seeded synthetic strings and workloads), build (in-tree HIP build).
"""
__all__ = ["ssm", "inputs", "build"]
