import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def feasible_lattices(max_L=120, max_lam2=4, require_p1=False):
    """All (L, a, M, lam1, lam2) with L <= max_L that satisfy the lattice
    conditions a | L, M | L, L lam1/(lam2 a) and L lam1/(lam2 M) integers."""
    from math import gcd
    out = []
    for L in range(2, max_L + 1):
        divs = [d for d in range(1, L + 1) if L % d == 0]
        for a in divs:
            for M in divs:
                if a == L or M == 1:
                    continue
                for lam2 in range(1, max_lam2 + 1):
                    for lam1 in range(0, lam2):
                        if gcd(lam1, lam2) != 1:
                            continue
                        if ((L // a) * lam1) % lam2 or ((L // M) * lam1) % lam2:
                            continue
                        if require_p1 and M % a:
                            continue
                        out.append((L, a, M, lam1, lam2))
    return out


# Degenerate lattices: one time position (a = L), one channel (M = 1), a = 1,
# M = L, p = L / gcd(L, 1) = 48 with columns of one value, and L = 1.
DEGENERATE_LATTICES = [(48, 48, 12, 0, 1), (48, 4, 1, 0, 1), (48, 1, 12, 0, 1), (48, 1, 48, 0, 1),
                       (96, 2, 48, 1, 2), (1, 1, 1, 0, 1), (48, 48, 1, 0, 1), (48, 1, 1, 0, 1)]
