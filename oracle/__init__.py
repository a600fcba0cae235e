"""FP64 CPU oracle for the DARC hot path.

Test infrastructure: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  The HIP product path never imports it and shares
no code with it.
"""
