"""CPU oracle for the GiFt hot path -- test infrastructure only.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The device library never does, and this package
never imports the device library.
"""
