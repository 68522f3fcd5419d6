"""D3Q19 lattice for the oracle (test infrastructure only).

The paper uses the D3Q19 velocity set with 19 velocities c_0 ... c_18 and the
standard D3Q19 weights with squared sound speed c_s^2 = 1/3 (Sec. 2, text
around Eq. LBE and Eq. local_eq); it cites these rather than printing them, so
the standard values are written out here:

    c_0 = 0                                  w = 1/3
    c_1..c_6   = +-e_x, +-e_y, +-e_z          w = 1/18
    c_7..c_18  = (+-1,+-1,0), (+-1,0,+-1),
                 (0,+-1,+-1)                  w = 1/36

The ordering (opposite pairs adjacent) is this project's choice.

The MRT transformation matrix is the d'Humieres et al. (2002) D3Q19 basis that
the paper takes from its MRT reference (Sec. 2, the MRT collision operator
paragraph).  Rows, 0-based here:

    0  rho            1                      10 3 pi_xx   (3c^2-5)(3cx^2-c^2)
    1  e              19c^2-30               11 p_ww      cy^2-cz^2
    2  eps            (21c^4-53c^2+24)/2     12 pi_ww     (3c^2-5)(cy^2-cz^2)
    3  j_x            cx                     13 p_xy      cx cy
    4  q_x            (5c^2-9)cx             14 p_yz      cy cz
    5  j_y            cy                     15 p_xz      cx cz
    6  q_y            (5c^2-9)cy             16 m_x       (cy^2-cz^2)cx
    7  j_z            cz                     17 m_y       (cz^2-cx^2)cy
    8  q_z            (5c^2-9)cz             18 m_z       (cx^2-cy^2)cz
    9  3 p_xx         3cx^2-c^2

Pins (tests/test_lattice.py): the isotropy identities up to fourth order in
exact rationals, failure at sixth order, the opposite map, orthogonality of
the MRT rows and their known squared norms.
"""
from fractions import Fraction

import torch

Q = 19
CS2 = 1.0 / 3.0

C_INT = (
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
)


def weight_fraction(c):
    """Exact D3Q19 weight of velocity c as a Fraction."""
    n = sum(abs(k) for k in c)
    return {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}[n]


W_FRAC = tuple(weight_fraction(c) for c in C_INT)


def velocities():
    """[19, 3] float64 tensor of lattice velocities (cx, cy, cz)."""
    return torch.tensor(C_INT, dtype=torch.float64)


def weights():
    """[19] float64 tensor of lattice weights."""
    return torch.tensor([float(w) for w in W_FRAC], dtype=torch.float64)


def opposite():
    """Index of -c_a for every a."""
    idx = {c: a for a, c in enumerate(C_INT)}
    return tuple(idx[(-c[0], -c[1], -c[2])] for c in C_INT)


def mrt_rows_int():
    """The 19 d'Humieres rows as lists of integers (one entry per velocity)."""
    rows = []
    for fn in (
        lambda x, y, z, c2: 1,
        lambda x, y, z, c2: 19 * c2 - 30,
        lambda x, y, z, c2: (21 * c2 * c2 - 53 * c2 + 24) // 2,
        lambda x, y, z, c2: x,
        lambda x, y, z, c2: (5 * c2 - 9) * x,
        lambda x, y, z, c2: y,
        lambda x, y, z, c2: (5 * c2 - 9) * y,
        lambda x, y, z, c2: z,
        lambda x, y, z, c2: (5 * c2 - 9) * z,
        lambda x, y, z, c2: 3 * x * x - c2,
        lambda x, y, z, c2: (3 * c2 - 5) * (3 * x * x - c2),
        lambda x, y, z, c2: y * y - z * z,
        lambda x, y, z, c2: (3 * c2 - 5) * (y * y - z * z),
        lambda x, y, z, c2: x * y,
        lambda x, y, z, c2: y * z,
        lambda x, y, z, c2: x * z,
        lambda x, y, z, c2: (y * y - z * z) * x,
        lambda x, y, z, c2: (z * z - x * x) * y,
        lambda x, y, z, c2: (x * x - y * y) * z,
    ):
        rows.append([fn(x, y, z, x * x + y * y + z * z) for (x, y, z) in C_INT])
    return rows


def mrt_matrix():
    """[19, 19] float64 MRT matrix M (moments m = M f)."""
    return torch.tensor(mrt_rows_int(), dtype=torch.float64)


# 0-based row classes of the d'Humieres basis.
CONSERVED_ROWS = (0, 3, 5, 7)          # rho, j_x, j_y, j_z
BULK_ROWS = (1,)                        # e (energy): bulk viscosity
SHEAR_ROWS = (9, 11, 13, 14, 15)        # 3p_xx, p_ww, p_xy, p_yz, p_xz
GHOST_ROWS = (2, 4, 6, 8, 10, 12, 16, 17, 18)


def mrt_rates(tau, s_bulk, s_ghost, s_conserved=1.0):
    """Diagonal of Lambda: shear rows 1/tau, bulk s_bulk, ghost s_ghost.

    The paper lists s_2 = s_10 = s_12 = s_14 = s_15 = s_16 = omega (1-based
    d'Humieres rows: e, 3p_xx, p_ww, p_xy, p_yz, p_xz) with every other rate 1
    (Sec. 2, MRT paragraph).  Its choice is s_bulk = 1/tau, s_ghost = 1 here;
    the conserved-row rate has no effect on the result.
    """
    lam = [None] * Q
    for rows, val in ((CONSERVED_ROWS, s_conserved), (BULK_ROWS, s_bulk),
                      (SHEAR_ROWS, 1.0 / tau), (GHOST_ROWS, s_ghost)):
        for r in rows:
            lam[r] = torch.as_tensor(val, dtype=torch.float64)
    # torch.stack keeps autograd through tau (and the other rates) when they
    # are tensors.
    return torch.stack(lam)
