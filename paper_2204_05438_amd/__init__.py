"""MI355X (gfx950) terminal-edge-region polygonal mesher: HIP kernels behind a
C ABI (include/polylla.h) and a thin ctypes binding (lib.py)."""

__all__ = ["lib", "build"]
