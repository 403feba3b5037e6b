"""CPU oracle for polynomial system evaluation and differentiation.

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import, call or link
anything in this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path:
its only common import is the seeded input generator, which holds no
evaluation arithmetic.

The oracle computes in exact dyadic arithmetic (Python integers scaled by
powers of two), so its F and J are the exact values of the polynomials and
their partial derivatives at the given point, with no rounding at all.
"""
from .exact import *  # noqa: F401,F403
