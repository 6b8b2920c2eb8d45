"""CPU oracle of the vacancy-jump AKMC path.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product (the HIP
library under paper_2604_24091_amd/ and its binding) never imports it.
"""
