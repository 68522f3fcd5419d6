"""Pins of the oracle's D3Q19 tables against exact mathematics.

The velocity set and weights are the standard D3Q19 ones the paper uses
(Sec. 2); the MRT basis is the d'Humieres (2002) one of the paper's MRT
reference.  These checks would catch a wrong weight, a missing or duplicated
velocity, or a typo in a basis polynomial.
"""
from fractions import Fraction
from itertools import product

from oracle import lattice


def _moment(order_idx):
    s = Fraction(0)
    for c, w in zip(lattice.C_INT, lattice.W_FRAC):
        term = w
        for i in order_idx:
            term *= c[i]
        s += term
    return s


def test_velocity_set_is_d3q19():
    assert len(set(lattice.C_INT)) == 19
    norms = sorted(sum(abs(k) for k in c) for c in lattice.C_INT)
    assert norms == [0] + [1] * 6 + [2] * 12
    assert all(max(abs(k) for k in c) <= 1 for c in lattice.C_INT)


def test_isotropy_exact_rationals():
    cs2 = Fraction(1, 3)
    assert _moment(()) == 1
    for i in range(3):
        assert _moment((i,)) == 0
    for i, j in product(range(3), repeat=2):
        assert _moment((i, j)) == (cs2 if i == j else 0)
    for idx in product(range(3), repeat=3):
        assert _moment(idx) == 0
    for i, j, k, l in product(range(3), repeat=4):
        d = lambda a, b: 1 if a == b else 0  # noqa: E731
        expect = cs2 * cs2 * (d(i, j) * d(k, l) + d(i, k) * d(j, l) + d(i, l) * d(j, k))
        assert _moment((i, j, k, l)) == expect
    for idx in product(range(3), repeat=5):
        assert _moment(idx) == 0


def test_sixth_order_isotropy_fails():
    # D3Q19 is not sixth-order isotropic: sum w cx^6 = 1/3, while an
    # isotropic tensor would need 15 c_s^6 = 5/9.
    assert _moment((0,) * 6) == Fraction(1, 3)
    assert Fraction(15, 27) != Fraction(1, 3)


def test_opposite_is_involution():
    opp = lattice.opposite()
    for a, c in enumerate(lattice.C_INT):
        assert opp[opp[a]] == a
        assert lattice.C_INT[opp[a]] == (-c[0], -c[1], -c[2])


def test_mrt_rows_orthogonal_with_known_norms():
    rows = lattice.mrt_rows_int()
    # Squared norms of the d'Humieres D3Q19 basis.
    norms = [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
    for i in range(19):
        for j in range(19):
            dot = sum(a * b for a, b in zip(rows[i], rows[j]))
            assert dot == (norms[i] if i == j else 0), (i, j, dot)


def test_mrt_rows_are_the_named_moments():
    rows = lattice.mrt_rows_int()
    c = lattice.C_INT
    assert rows[0] == [1] * 19
    assert rows[3] == [v[0] for v in c]
    assert rows[5] == [v[1] for v in c]
    assert rows[7] == [v[2] for v in c]
    assert rows[13] == [v[0] * v[1] for v in c]
    assert rows[14] == [v[1] * v[2] for v in c]
    assert rows[15] == [v[0] * v[2] for v in c]


def test_rate_classes_partition_rows():
    all_rows = (lattice.CONSERVED_ROWS + lattice.BULK_ROWS + lattice.SHEAR_ROWS
                + lattice.GHOST_ROWS)
    assert sorted(all_rows) == list(range(19))
