"""MI355X-native particle update: CIC/TSC gather, Boris / drag / tracer push,
moment deposit and cell-tile sort, behind the C ABI declared in include/pl.h.

Importing the package loads nothing; ``paper_2602_23434_amd.binding`` loads the
HIP library (libpl.so) and fails loudly when it has not been built.
"""

__all__ = ["inputs", "binding"]
