"""MI355X (gfx950) STAP hot path: HIP kernels behind a C ABI (libstap.so).

``paper_2203_06233_amd.stap`` is the Python binding; ``build`` compiles the
library in-tree.
"""
__all__ = ["stap", "build"]
