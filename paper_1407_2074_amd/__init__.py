"""MI355X-native multi-channel brick-octree ray caster.

The compute path is a C-ABI shared library of hand-written HIP kernels for gfx950
(``liboctree_rc.so``, declared in ``include/octree_rc.h``); this package only marshals
arguments into it.  Importing the package does not load the library: ``octree`` and the other
submodules do, and they raise if it is missing instead of falling back to anything else.
"""

__all__ = ["synth"]
