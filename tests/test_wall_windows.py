"""Host check of the general three-step kernel's LDS windows (WallWindows in
csrc/lbm13_kernels.hip): every read the wall fix-ups make of a reflected
population (sec. 7 path reversal, as fix_link applies it: tangential
coordinate kept, normal coordinate mirrored in the wall half a spacing outside
the last node) must land in the window the producing level writes, for every
tile of the grid of whole tiles from the domain's origin, every domain size up
to a few tiles and every wall configuration.  The rule below is the kernel's;
the check enumerates the fix-ups of wall_fixups."""
import itertools

import pytest

VX = (0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0)
VY = (0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2)
OPP = (0, 3, 4, 1, 2, 7, 8, 5, 6, 11, 12, 9, 10)
# links replaced at each wall: (first-layer only, every layer within two nodes)
FIXED = {"W": ((1, 5, 8), (9,)), "E": ((3, 6, 7), (11,)), "S": ((2, 5, 6), (10,)), "N": ((4, 7, 8), (12,))}
STEP3_SHAPES = ((64, 16), (32, 32), (64, 8), (32, 16), (32, 8))


def window(i, last):
    """(xlo, xhi, ylo, yhi): slots kept past the reading level's region."""
    vx, vy = VX[i], VY[i]
    xhi = (3 if vx == 2 else 1) if vx > 0 else 0
    yhi = (3 if vy == 2 else 1) if vy > 0 else 0
    xlo = (-vx if last else (1 if vy else 0)) if vx < 0 else 0
    ylo = (-vy if last else (1 if vx else 0)) if vy < 0 else 0
    return xlo, xhi, ylo, yhi


def reflected(wall, I, x, y, nx, ny):
    """Node whose population OPP[I] replaces link I of node (x, y) (fix_link)."""
    px, py = x, y
    if wall == "W":
        px = -1 + VX[I] - x
    elif wall == "E":
        px = 2 * nx - 1 + VX[I] - x
    elif wall == "S":
        py = -1 + VY[I] - y
    else:
        py = 2 * ny - 1 + VY[I] - y
    return px, py


def fixups(x, y, nx, ny, xwall, ywall):
    """(wall, link) pairs wall_fixups replaces at node (x, y), in its order."""
    out = []
    if ywall and y < 2:
        out += [("S", I) for I in (FIXED["S"][0] if y == 0 else ()) + FIXED["S"][1]]
    if ywall and y >= ny - 2:
        out += [("N", I) for I in (FIXED["N"][0] if y == ny - 1 else ()) + FIXED["N"][1]]
    if xwall and x < 2:
        out += [("W", I) for I in (FIXED["W"][0] if x == 0 else ()) + FIXED["W"][1]]
    if xwall and x >= nx - 2:
        out += [("E", I) for I in (FIXED["E"][0] if x == nx - 1 else ()) + FIXED["E"][1]]
    return out


def check_domain(tw, th, nx, ny, xwall, ywall):
    """Every fix-up read of the second and third levels of every tile."""
    misses = []
    for x0, y0 in itertools.product(range(0, nx, tw), range(0, ny, th)):
        tw3, th3 = min(tw, nx - x0), min(th, ny - y0)
        for last, (ox, oy), (w, h), reach in ((False, (x0 - 2, y0 - 2), (tw + 4, th + 4), 2),
                                              (True, (x0, y0), (tw, th), 0)):
            # the level's nodes: its region within reach of the tile's nodes,
            # inside the domain on a walled axis
            xs = range(max(ox, 0) if xwall else ox, min(x0 + tw3 + reach, nx) if xwall else x0 + tw3 + reach)
            ys = range(max(oy, 0) if ywall else oy, min(y0 + th3 + reach, ny) if ywall else y0 + th3 + reach)
            # the level before it computes these nodes
            pxs = range(max(ox - 2, 0) if xwall else ox - 2, min(x0 + tw3 + reach + 2, nx) if xwall else x0 + tw3 + reach + 2)
            pys = range(max(oy - 2, 0) if ywall else oy - 2, min(y0 + th3 + reach + 2, ny) if ywall else y0 + th3 + reach + 2)
            for x, y in itertools.product(xs, ys):
                for wall, I in fixups(x, y, nx, ny, xwall, ywall):
                    px, py = reflected(wall, I, x, y, nx, ny)
                    i = OPP[I]
                    ux, uy = px - ox + VX[i], py - oy + VY[i]
                    xlo, xhi, ylo, yhi = window(i, last)
                    ok = -xlo <= ux < w + xhi and -ylo <= uy < h + yhi and px in pxs and py in pys
                    if not ok:
                        misses.append((tw, th, nx, ny, x0, y0, "L3" if last else "L2", wall, I, x, y))
    return misses


@pytest.mark.parametrize("tw,th", STEP3_SHAPES)
def test_reflected_reads_stay_in_the_windows_x_walls(tw, th):
    misses = []
    for nx in range(2, 3 * tw + 8):
        misses += check_domain(tw, th, nx, th + 3, True, False)
    assert not misses, misses[:5]


@pytest.mark.parametrize("tw,th", STEP3_SHAPES)
def test_reflected_reads_stay_in_the_windows_y_walls(tw, th):
    misses = []
    for ny in range(2, 3 * th + 8):
        misses += check_domain(tw, th, tw + 3, ny, False, True)
    assert not misses, misses[:5]


@pytest.mark.parametrize("tw,th", STEP3_SHAPES)
def test_reflected_reads_stay_in_the_windows_closed(tw, th):
    """Walls on all four sides (corners, where a diagonal is replaced at both
    walls), sizes around one and two tiles and the smallest domains."""
    sizes_x = sorted(set(range(2, 9)) | set(range(tw - 3, tw + 4)) | set(range(2 * tw - 3, 2 * tw + 4)))
    sizes_y = sorted(set(range(2, 9)) | set(range(th - 3, th + 4)) | set(range(2 * th - 3, 2 * th + 4)))
    misses = []
    for nx, ny in itertools.product(sizes_x, sizes_y):
        misses += check_domain(tw, th, nx, ny, True, True)
    assert not misses, misses[:5]


def test_a_narrower_rule_misses_reads():
    """The check has teeth: one slot less past the high edge for the speed-2
    populations (two instead of three) misses the reflected read of a
    second-layer node when a tile ends three nodes before the East wall."""
    global window
    keep = window

    def narrower(i, last):
        xlo, xhi, ylo, yhi = keep(i, last)
        return xlo, min(xhi, 2), ylo, min(yhi, 2)
    window = narrower
    try:
        assert check_domain(32, 16, 32 + 3, 19, True, False)
        assert not check_domain(32, 16, 32 + 4, 19, True, False)
    finally:
        window = keep
