"""CPU oracle of TRPL+K — test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
import anything under this package.  The HIP library never calls it.
"""
