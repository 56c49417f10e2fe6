"""CPU oracle for the decentralized detection / precoding hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg import this package; the product library never does, and the
two share no code.  ``dbp_oracle`` is the FP64 oracle (Algorithms 1-3 and the
centralized closed forms), ``rational`` the exact-arithmetic cross-check for tiny
instances, ``ml`` the brute-force maximum-likelihood detector.
"""
