"""Sequential CPU oracle of the terminal-edge-region polygonal mesh method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only callers. The product path (the HIP library and
its Python binding) never imports or links it, and the two share no code.
"""
from .run import build, oracle_lepp, oracle_mesh, oracle_on, HE, TRI, VTX, STATS  # noqa: F401
