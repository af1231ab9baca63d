"""FP64 CPU reference of the occupancy pass. TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU baseline import this
package; the product library never does.
"""
from . import oracle, literal  # noqa: F401
