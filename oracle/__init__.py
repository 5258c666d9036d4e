"""CPU oracle (TEST INFRASTRUCTURE ONLY): plain float64 reference of the saddle-point solve.

Only the tests, the entry module's smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.
"""
