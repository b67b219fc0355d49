"""CPU oracle for linear elliptical slice sampling (arXiv 2407.10449).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code
with the HIP implementation; both consume the same seeded inputs from the
`synth` package.
"""
from . import philox, ess  # noqa: F401
