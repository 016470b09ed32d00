"""D3Q27 lattice (Sec. II B, Fig. 1; weights Eq. (17)).

Direction ordering used throughout the oracle:
    i = 9*(cx+1) + 3*(cy+1) + (cz+1),  cx,cy,cz in {-1,0,1}
so the rest direction is i = 13 and the opposite of i is 26 - i.  The paper
fixes no ordering; this one is a data-layout convention only.
"""
from fractions import Fraction

import torch

Q = 27
REST = 13
CS2 = Fraction(1, 3)          # c_s^2 = c^2/3 with c = 1 (Sec. II B)

# velocities as python ints
C = [(cx, cy, cz) for cx in (-1, 0, 1) for cy in (-1, 0, 1) for cz in (-1, 0, 1)]


def weight_exact(c):
    """Eq. (17): the weight depends only on |c_i|^2."""
    n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2]
    return {0: Fraction(8, 27), 1: Fraction(2, 27), 2: Fraction(1, 54), 3: Fraction(1, 216)}[n2]


W_EXACT = [weight_exact(c) for c in C]
OPP = [C.index((-c[0], -c[1], -c[2])) for c in C]

C_T = torch.tensor(C, dtype=torch.float64)            # (27, 3)
W_T = torch.tensor([float(w) for w in W_EXACT], dtype=torch.float64)   # (27,)
