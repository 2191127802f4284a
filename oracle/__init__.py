"""CPU test oracle for the reverse-mode energy gradient (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import
this package. The GPU library neither imports nor links it.
"""
