"""CPU oracle for the MOMENTI motif search (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library never does, and the
two share no code: this side is plain C (``momenti_oracle.c``) driven through
ctypes, double precision, sequential, following the paper step by step.
"""
from .oracle import *  # noqa: F401,F403
