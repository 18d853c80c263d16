"""MI355X (gfx950) implementation of the AIMx matvec and its batched solver.

* ``binding``  -- ctypes wrapper of ``libaimx.so`` (C ABI: include/aim.h)
* ``build``    -- in-tree hipcc build of the library
* ``inputs``   -- seeded synthetic meshes and vectors (no method arithmetic)

Importing the package loads nothing; ``binding.load_library()`` raises if
the library has not been built.
"""
__all__ = ["binding", "build", "inputs"]
