"""FP64 CPU oracle for the RBF neural-field path.

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU library and its binding never do.
"""
