"""CPU oracle for ParRep on CTMC reaction networks -- TEST INFRASTRUCTURE ONLY.

A plain, slow C implementation (``parrep_oracle.c``) of the paper's Algorithm 1
with a ctypes front end (``oracle.py``).  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it; the
GPU library and its binding never do.
"""
