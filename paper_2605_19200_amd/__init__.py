"""MI355X (gfx950) engine for spatially accelerated generalized winding numbers
on curved boundaries: rational Bezier curves in 2D and trimmed rational
bicubic patches in 3D.

Submodules are imported lazily so that the seeded input generators
(`workloads`) can be used without loading the HIP library.
"""

__all__ = ["gwn", "workloads", "serve"]
