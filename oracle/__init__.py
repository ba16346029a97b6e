"""Exact CPU reference of the Ozaki-II p-bit GEMM.

TEST INFRASTRUCTURE ONLY: imported by the tests, by __graft_entry__.smoke()
and by the cpu_baseline leg of bench.py, never by the GPU path.
"""
