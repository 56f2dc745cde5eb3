"""FP64 CPU oracle for the real-space static polarizability build.

TEST INFRASTRUCTURE ONLY.  This package is imported by the test-suite, by the
package smoke check and by the benchmark's CPU-baseline leg, and by nothing
else: the GPU library never imports, links or calls it, and it shares no code
with the GPU path (its only inputs come from the seeded generator `gwsynth`).

Parity status of each function is stated in its docstring; all of them are
pinned by closed forms, invariants or independent routes in the CPU tests.
"""
from .gw_oracle import *  # noqa: F401,F403
