"""ORACLE -- test infrastructure only.

Serial FP64 CPU reference of the hybrid pseudopotential phase-change LBM time
step with conjugate heat transfer (arXiv:1911.10747, Section 2).  Used by
tests/, the smoke check and the benchmark's CPU-baseline leg; never by the
product path, with which it shares no code.
"""
