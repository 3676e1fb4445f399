"""Index arithmetic of the 2D stage's ghost centres, checked on the host.

The stage kernel skips a centre beyond a wall or outflow side in phase 2 and
copies it afterwards, with the image's signs, from its image centre in the
same tile's LDS region.  This re-derives that arithmetic (tile origin, the
20 x (TY + 4) centre grid of the region, the margin of four ghost lattice
lines, the lattice images of each side kind) for every tile height the
library builds, grids from 4 cells (the smallest the boundary accepts)
upward and every combination of side kinds, and checks that each ghost's
image lies in the region and is a centre that phase 2 computes, never a
ghost itself."""
import pytest

PER, OUT, NOSLIP, SYM = 0, 1, 2, 3
TX, MARGIN = 16, 4


def axis_image(X, twon, lo, hi):
    """lattice image of coordinate X on an axis of 2n half cells"""
    if lo == PER:
        return X % twon
    if X < 0:
        return (1 if X & 1 else 0) if lo == OUT else -X
    if X > twon:
        return (twon - 1 if (X - twon) & 1 else twon) if hi == OUT else 2 * twon - X
    return X


def check_grid(TY, n1, n2, bcx, bcy):
    WA, HA = 2 * TX + 9, 2 * TY + 9
    Xl, Yl = 2 * n1, 2 * n2
    bad = 0
    for tj in range(n2 // TY + 1):
        for ti in range(n1 // TX + 1):
            X0, Y0 = 2 * TX * ti, 2 * TY * tj
            centres = [(X0 - 3 + 2 * (c % (TX + 4)), Y0 - 3 + 2 * (c // (TX + 4)))
                       for c in range((TX + 4) * (TY + 4))]

            def in_region(X, Y):
                return X <= Xl + MARGIN and Y <= Yl + MARGIN

            def ghost(X, Y):
                return (((X < 0 or X > Xl) and bcx[0] != PER)
                        or ((Y < 0 or Y > Yl) and bcy[0] != PER))

            computed = {(X, Y) for X, Y in centres if in_region(X, Y) and not ghost(X, Y)}
            for X, Y in centres:
                if not in_region(X, Y) or not ghost(X, Y):
                    continue
                Xi = X if bcx[0] == PER else axis_image(X, Xl, *bcx)
                Yi = Y if bcy[0] == PER else axis_image(Y, Yl, *bcy)
                lx, ly = Xi - X0 + 4, Yi - Y0 + 4
                if not (0 <= lx < WA and 0 <= ly < HA and (Xi, Yi) in computed):
                    bad += 1
    return bad


SIDES = [(PER, PER), (NOSLIP, NOSLIP), (OUT, OUT), (SYM, OUT), (OUT, NOSLIP)]


@pytest.mark.parametrize("TY", [5, 7, 10, 14])
def test_every_ghost_centre_image_is_a_computed_centre_of_the_region(TY):
    for n1 in (4, 5, 15, 16, 17, 33, 40):
        for n2 in (4, 6, 7, 8, 13, 14, 15, 29):
            for bcx in SIDES:
                for bcy in SIDES:
                    assert check_grid(TY, n1, n2, bcx, bcy) == 0, (TY, n1, n2, bcx, bcy)


def test_a_one_cell_grid_would_break_it():
    """why the boundary requires n >= 4: with one cell a mirrored ghost's
    image is itself beyond the opposite wall"""
    assert check_grid(7, 1, 1, (PER, PER), (NOSLIP, SYM)) > 0
