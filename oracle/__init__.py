"""CPU oracle for the density-fitted GW hot path.

Test infrastructure only: plain fp64 numpy forms of the paper's equations,
used by the tests, the smoke check and the CPU-baseline timing.  The product
library never imports, links or runs anything in this package.
"""
