"""Host emulation of the integer index arithmetic the kernels use to order
their tiles and to wrap periodic coordinates, transcribed from the device
code: every ordering is a bijection onto the tiles of the grid, and every
coordinate handed to the one-correction periodic wrap lies within one period
either side of the grid (the wrap is exact there), for all grid sizes the
library accepts (at least 4 cells per axis)."""
import itertools

import pytest


def wrap1(t, n):
    """t mod n by one correction either way (valid for -n <= t < 2n)."""
    t = t + n if t < 0 else t
    return t - n if t >= n else t


def tile_coords(lin, nt, fast):
    """Tile `fast` varies fastest, then the lower of the other two axes."""
    a1 = 1 if fast == 0 else 0
    a2 = 1 if fast == 2 else 2
    t = [0, 0, 0]
    t[fast] = lin % nt[fast]
    lin //= nt[fast]
    t[a1] = lin % nt[a1]
    t[a2] = lin // nt[a1]
    return tuple(t)


def fp32_flux_tile_coords(lin, nt, d2):
    """FP32 flux tiles: x-tile pairs first, then t2, when t2 is not x and the
    x-tile count is even; otherwise t2 tiles adjacent."""
    if d2 != 0 and nt[0] % 2 == 0:
        xh = lin & 1
        r = lin >> 1
        t = [0, 0, 0]
        t[d2] = r % nt[d2]
        r //= nt[d2]
        t[0] = 2 * (r % (nt[0] >> 1)) + xh
        t[3 - d2] = r // (nt[0] >> 1)
        return tuple(t)
    return tile_coords(lin, nt, d2)


def test_wrap1_is_modulo_within_one_period():
    for period in (4, 5, 7, 16, 33):
        for t in range(-period, 2 * period):
            assert wrap1(t, period) == t % period


@pytest.mark.parametrize("d", [0, 1, 2])
def test_fp32_flux_tile_order_is_a_bijection(d):
    """Every FP32 flux tile is visited exactly once (even and odd x-tile
    counts, ragged grids), and where the pair order applies the two tiles of
    a pair run back to back and t2 neighbours two blocks apart."""
    d2 = (d + 2) % 3
    for nx, ny, nz in itertools.product((4, 16, 20, 33, 40), (5, 12, 17), (4, 9, 16)):
        # FP32 tiles: 16 faces along x, 4 along y, one z plane
        nt = ((nx + 15) // 16, (ny + 3) // 4, nz)
        total = nt[0] * nt[1] * nt[2]
        seen = [fp32_flux_tile_coords(lin, nt, d2) for lin in range(total)]
        assert len(set(seen)) == total
        assert all(0 <= seen[i][a] < nt[a] for i in range(total) for a in range(3))
        if d2 != 0 and nt[0] % 2 == 0:
            for lin in range(0, total, 2):
                a, b = seen[lin], seen[lin + 1]
                assert a[0] % 2 == 0 and b[0] == a[0] + 1 and a[1:] == b[1:]
            for lin in range(total - 2):
                a, b = seen[lin], seen[lin + 2]
                if a[d2] + 1 < nt[d2]:
                    assert b[d2] == a[d2] + 1 and b[0] == a[0] and b[3 - d2] == a[3 - d2]


def test_staged_flux_rows_stay_within_one_period():
    """flux4_kernel (x and z faces): the block at t2 tile tc stages rows
    t = 4 tc - 2 + r, r = 0..7, for tc < ceil(n / 4).  For every n >= 4 they
    lie in [-n, 2n), so the one-correction wrap is the periodic wrap."""
    for n in range(4, 700):
        ntile = (n + 3) // 4
        lo = -2
        hi = 4 * (ntile - 1) - 2 + 7
        assert -n <= lo and hi < 2 * n, n
        for tc in (0, ntile - 1):
            for r in range(8):
                t = 4 * tc - 2 + r
                assert wrap1(t, n) == t % n


def test_y_face_staged_columns_need_the_division_only_below_9():
    """flux4y_kernel: the block at x tile tc stages columns
    x = 16 tc - 2 + min(e, 19), e = 0..31, for tc < ceil(n_x / 16).  They lie
    in [-n_x, 2 n_x) exactly when n_x > 8, the condition under which the
    kernel takes the one-correction wrap (narrower grids take the division)."""
    for n in range(4, 700):
        ntile = (n + 15) // 16
        xs = [16 * tc - 2 + min(e, 19) for tc in range(ntile) for e in range(32)]
        inside = all(-n <= x < 2 * n for x in xs)
        assert inside == (n > 8), n
        if n > 8:
            assert all(wrap1(x, n) == x % n for x in xs)


def test_cell_coordinates_stay_within_one_period():
    """The ghost cells the reconstruction (normal stencils 3 cells either
    side, t1 halo of 2) and the statistics (4th-order differences, 2 cells
    either side) ask for lie within three cells of the grid: inside one
    period either side for every axis of at least 4 cells."""
    for n in range(4, 64):
        for c in range(-3, n + 3):
            assert wrap1(c, n) == c % n
