"""FP64 CPU oracle for overlap-save HFSO variable-bandwidth filtering.

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.
"""
