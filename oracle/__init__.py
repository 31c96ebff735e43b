"""CPU oracle for the interval subdivision hot path -- TEST INFRASTRUCTURE ONLY.

Imported only by tests/, __graft_entry__.smoke() and the CPU-baseline leg of
bench.py.  The product package never imports it.
"""
