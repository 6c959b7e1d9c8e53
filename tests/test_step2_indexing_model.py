"""Host model of the two-step kernel's pull and bounce-back indexing.

The two-step kernel (two lattice steps per pass, phase A into an LDS ring of
rows, phase B from it) picks the word each population is pulled from by lane
arithmetic, lane shifts, the ring's outside-cell slots and per-row bit masks
of the solid cells; a mistake there shows only next to solid cells, and only
for some positions of them relative to the strips and lanes.  This model
re-enacts that index logic on the CPU, in the kernel's own terms (its
direction tables, read from the source; its geometry tests; the masks its
`solids` builds and the bit its `solid` tests; phase A's row loads, lane
shifts, edge words and outside cells; phase B's ring reads; the store mask;
the ring slots of both phases), and checks, for every fluid cell and
direction, that the word it lands on is the one the pull-stream step with
halfway bounce-back (paper Section 2 and Appendix A) defines: the population
f_i at x - c_i if that cell is fluid, else the cell's own f_opp(i); rows
beyond a wall bounce back; an open channel's ends pull from its ghost
columns.  The solid cells come from the oracle's geometry (square and grid
bars), independently of the masks the model rebuilds.

Words are named ("t", i, x, y) for the state the launch reads (step t),
("u", i, x, y) for phase A's results (step t + 1) and ("in", i, y) /
("out", i, y) for the inlet and outlet ghost columns.
"""
import os
import re

import numpy as np
import pytest

from oracle import open_channel as ooc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tables():
    src = open(os.path.join(ROOT, "paper_2005_09323_amd", "csrc", "common.hpp")).read()
    out = {}
    for name in ("CX", "CY", "OPP"):
        m = re.search(r"constexpr int %s\[9\] = \{([^}]*)\};" % name, src)
        out[name] = [int(v) for v in m.group(1).split(",")]
    return out["CX"], out["CY"], out["OPP"]


CX, CY, OPP = _tables()
STRIP = 256


class Geometry:
    """One member: nx x ny, square (sx0, sy0, ss) (ss = 0: none), open channel
    with grid bars (gx0, bar) (bar = 0: none) or periodic in x."""

    def __init__(self, nx, ny, square, open_=False, gx0=0, bar=0):
        self.nx, self.ny = nx, ny
        self.sx0, self.sy0, self.ss = square
        self.open, self.gx0, self.bar = open_, gx0, bar
        sol = np.zeros((ny, nx), dtype=bool)
        if self.ss:
            sol[self.sy0:self.sy0 + self.ss, self.sx0:self.sx0 + self.ss] = True
        if open_ and bar:
            sol |= ooc.grid_mask(ny, nx, ooc.OpenChannel(0.05, gx0, bar, nx, 1.0))
        self.solid = sol  # the definition's solid cells (oracle geometry)

    # -- the definition ------------------------------------------------------
    def expected(self, x, y, i, step):
        """Word a fluid cell (x, y) pulls for direction i from the state `step`."""
        xs, ys = x - CX[i], y - CY[i]
        if ys < 0 or ys >= self.ny:
            return (step, OPP[i], x, y)
        if self.open:
            if xs < 0:
                return ("in", i, ys)
            if xs >= self.nx:
                return ("out", i, ys)
        else:
            xs %= self.nx
        if self.solid[ys, xs]:
            return (step, OPP[i], x, y)
        return (step, i, xs, ys)


class Kernel:
    """The kernel's index logic for one member, transcribed."""

    def __init__(self, g: Geometry):
        self.g = g

    # geometry helpers (common.hpp)
    def in_square(self, x, y):
        g = self.g
        return 0 <= x - g.sx0 < g.ss and 0 <= y - g.sy0 < g.ss

    def grid_row(self, y):
        g = self.g
        r = y - (g.bar >> 1)
        return g.bar > 0 and r >= 0 and r % (2 * g.bar) < g.bar

    # per strip
    def strip(self, tx):
        g = self.g
        base = STRIP * tx
        s = dict(base=base, left_end=base == 0, right_end=base + STRIP == g.nx)
        s["xl"] = (g.nx if s["left_end"] else base) - 1
        s["xr"] = 0 if s["right_end"] else base + STRIP
        s["sq_cols"] = g.ss > 0 and base <= g.sx0 + g.ss and base + STRIP - 1 >= g.sx0 - 1
        s["grid_cols"] = self.grid_cols(base)
        return s

    def grid_cols(self, base):
        g = self.g
        return g.open and g.bar > 0 and base <= g.gx0 + g.bar + 1 and base + STRIP - 1 >= g.gx0 - 2

    def grow(self, s, yy):
        return self.g.open and s["grid_cols"] and 0 <= yy < self.g.ny and self.grid_row(yy)

    def rows3(self, s, yy):
        if not self.g.open:
            return 0
        return (1 if self.grow(s, yy - 1) else 0) | (2 if self.grow(s, yy) else 0) | (4 if self.grow(s, yy + 1) else 0)

    def lane_masks(self, s, x0):
        g = self.g
        gcols = 0
        if s["grid_cols"]:
            for j in range(6):
                gcols |= (1 if 0 <= x0 - 1 + j - g.gx0 < g.bar else 0) << j
        sqcols = 0
        if g.open and s["sq_cols"]:
            for j in range(6):
                sqcols |= (1 if 0 <= x0 - 1 + j - g.sx0 < g.ss else 0) << j
        return gcols, sqcols

    def solids(self, yy, near, g3, gcols, sqcols):
        g = self.g
        mk = 0
        for j in range(3):
            row = gcols if (g3 >> j) & 1 else 0
            if near and 0 <= yy - 1 + j - g.sy0 < g.ss:
                row |= sqcols
            mk |= row << (6 * j)
        return mk

    def solid(self, mk, x0, dx, yy, j, near):
        if self.g.open:
            return (mk >> (6 * j + dx + 1)) & 1 != 0
        return near and self.in_square(x0 + dx, yy)

    # phase A: the lane's four cells of row y at step t + 1
    def phase_a(self, s, lane, y):
        g = self.g
        x0 = s["base"] + 4 * lane
        near_sq = s["sq_cols"] and g.sy0 - 1 <= y <= g.sy0 + g.ss
        gA = self.rows3(s, y)
        near_a = near_sq or gA != 0
        gcols, sqcols = self.lane_masks(s, x0)
        mk = self.solids(y, near_sq, gA, gcols, sqcols) if g.open else 0

        def raw(i, k):  # the row load of direction i, element k (load_row)
            ys = y - CY[i]
            if ys < 0 or ys >= g.ny:
                return ("t", OPP[i], x0 + k, y)
            return ("t", i, x0 + k, ys)

        def edge(i):  # the edge word of a +-x mover (load_row)
            ys = y - CY[i]
            if CX[i] == 1:
                return ("in", i, ys) if (g.open and s["left_end"]) else ("t", i, s["xl"], ys)
            return ("out", i, ys) if (g.open and s["right_end"]) else ("t", i, s["xr"], ys)

        out = {}
        for k in range(4):
            for i in range(9):
                ys = y - CY[i]
                wall = ys < 0 or ys >= g.ny
                if wall or CX[i] == 0:
                    w = raw(i, k)
                elif CX[i] == 1:  # f4{lane == 0 ? e : shr1(v.w), v.x, v.y, v.z}
                    w = raw(i, k - 1) if k >= 1 else (edge(i) if lane == 0 else ("t", i, x0 - 1, ys))
                else:  # f4{v.y, v.z, v.w, lane == 63 ? e : shl1(v.x)}
                    w = raw(i, k + 1) if k <= 2 else (edge(i) if lane == 63 else ("t", i, x0 + 4, ys))
                out[(x0 + k, i)] = w
            if near_a and not self.solid(mk, x0, k, y, 1, near_sq):
                for i in range(1, 9):
                    ys = y - CY[i]
                    if ys < 0 or ys >= g.ny:
                        continue
                    if self.solid(mk, x0, k - CX[i], ys, 1 - CY[i], near_sq):
                        # ownv: the rows of the +-x movers' opposites are loaded already
                        out[(x0 + k, i)] = raw(OPP[i], k) if CY[OPP[i]] == 0 else ("t", OPP[i], x0 + k, y)
        return out

    # phase A: the outside cell of lane 0 (left) or 1 (right) of row y
    def outside(self, s, lane, y):
        g = self.g
        xh = s["xr"] if lane & 1 else s["xl"]
        own_h = not g.open or not (s["right_end"] if lane & 1 else s["left_end"])
        if not own_h:
            return None
        gA = self.rows3(s, y)
        out = {}
        for i in range(9):
            ys = y - CY[i]
            if g.open:
                xs = xh - CX[i]
                bounce = ys < 0 or ys >= g.ny or self.in_square(xs, ys) or (
                    0 <= xs - g.gx0 < g.bar and (gA >> (1 - CY[i])) & 1)
            else:  # load_cell<false>: periodic in x, the square only
                xs = (xh - CX[i]) % g.nx
                bounce = ys < 0 or ys >= g.ny or self.in_square(xs, ys)
            out[i] = ("t", OPP[i], xh, y) if bounce else ("t", i, xs, ys)
        # stored into the ring unless the kernel finds the cell solid
        stored = not (self.in_square(xh, y) or (g.open and 0 <= xh - g.gx0 < g.bar and (gA >> 1) & 1))
        return xh, out, stored

    # phase B: the lane's four cells of row r at step t + 2 (words of step t + 1)
    def phase_b(self, s, lane, r, ring_edge):
        g = self.g
        x0 = s["base"] + 4 * lane
        near_sq = s["sq_cols"] and g.sy0 - 1 <= r <= g.sy0 + g.ss
        gB = self.rows3(s, r)
        near_b = near_sq or gB != 0
        gcols, sqcols = self.lane_masks(s, x0)
        mkb = self.solids(r, near_sq, gB, gcols, sqcols) if g.open and near_b else 0
        out = {}
        for k in range(4):
            for i in range(9):
                rsrc = r - CY[i]
                if rsrc < 0 or rsrc >= g.ny:
                    w = ("u", OPP[i], x0 + k, r)
                elif CX[i] == 1:
                    if k >= 1:
                        w = ("u", i, x0 + k - 1, rsrc)
                    elif lane > 0:
                        w = ("u", i, x0 - 1, rsrc)
                    else:
                        w = ring_edge("left", i, rsrc)
                elif CX[i] == -1:
                    if k <= 2:
                        w = ("u", i, x0 + k + 1, rsrc)
                    elif lane < 63:
                        w = ("u", i, x0 + 4, rsrc)
                    elif g.open and s["right_end"]:
                        w = ("out", i, rsrc)  # built from the velocity ring
                    else:
                        w = ring_edge("right", i, rsrc)
                else:
                    w = ("u", i, x0 + k, rsrc)
                out[(x0 + k, i)] = w
        if near_b:
            for k in range(4):
                if self.solid(mkb, x0, k, r, 1, near_sq):
                    continue
                for i in range(1, 9):
                    rsrc = r - CY[i]
                    if rsrc < 0 or rsrc >= g.ny:
                        continue
                    if self.solid(mkb, x0, k - CX[i], rsrc, 1 - CY[i], near_sq):
                        out[(x0 + k, i)] = ("u", OPP[i], x0 + k, r)
        smask = (mkb >> 7) & 0xF
        if not g.open and near_b:
            for k in range(4):
                smask |= (1 if self.solid(0, x0, k, r, 1, near_sq) else 0) << k
        return out, smask


def check_member(g: Geometry, rows=None):
    """Every fluid cell's words in both phases against the definition; phase
    B's stores against the solid cells.  Returns the mismatches."""
    kern = Kernel(g)
    bad = []
    rows = range(g.ny) if rows is None else rows
    for tx in range(g.nx // STRIP):
        s = kern.strip(tx)
        for y in rows:
            # phase A: the strip's cells and its two outside cells, step t -> t + 1
            ring = {}
            for lane in range(64):
                for (x, i), w in kern.phase_a(s, lane, y).items():
                    ring[(x, i)] = w
            for lane in (0, 1):
                o = kern.outside(s, lane, y)
                if o is None:
                    continue
                xh, words, stored = o
                if g.solid[y, xh]:
                    continue
                if not stored:
                    bad.append(("outside cell not stored", tx, xh, y))
                for i, w in words.items():
                    if w != g.expected(xh, y, i, "t"):
                        bad.append(("A outside", tx, xh, y, i, w, g.expected(xh, y, i, "t")))
            for (x, i), w in ring.items():
                if not g.solid[y, x] and w != g.expected(x, y, i, "t"):
                    bad.append(("A", tx, x, y, i, w, g.expected(x, y, i, "t")))
        for r in rows:
            # phase B, step t + 1 -> t + 2: a ring-edge word is the outside cell's
            # result if phase A stored it, else whatever the slot held before
            def ring_edge(side, i, rsrc, s=s):
                lane = 0 if side == "left" else 1
                if g.open and side == "left" and s["left_end"]:
                    return ("in", i, rsrc)
                xh, _, stored = kern.outside(s, lane, rsrc)
                return ("u", i, xh, rsrc) if stored else ("stale", side, rsrc)

            for lane in range(64):
                words, smask = kern.phase_b(s, lane, r, ring_edge)
                x0 = s["base"] + 4 * lane
                for k in range(4):
                    x = x0 + k
                    if bool((smask >> k) & 1) != bool(g.solid[r, x]):
                        bad.append(("B store mask", tx, x, r))
                    if g.solid[r, x]:
                        continue
                    for i in range(9):
                        w, e = words[(x, i)], g.expected(x, r, i, "u")
                        if w != e:
                            bad.append(("B", tx, x, r, i, w, e))
    return bad


def ring_slots_ok(ny, nw, lag, split_rows=None):
    """The ring's row slots (y % (nw + 1 + lag)) and the outlet's velocity ring
    (y & 15): every row phase B reads is the one phase A last wrote there."""
    rrows = nw + 1 + lag
    segs = [(0, ny)] if split_rows is None else [(a, min(a + split_rows, ny)) for a in range(0, ny, split_rows)]
    for ya, yb in segs:
        ya0, ya1 = (max(ya - lag, 0), min(yb + lag, ny)) if split_rows else (0, ny)
        iters = (yb + lag - ya0 + nw - 1) // nw if split_rows else (ny + lag - 1) // nw + 1
        slot, vslot = {}, {}
        for j in range(iters):
            for wv in range(nw):
                y = ya0 + j * nw + wv
                if y < ya1:
                    slot[y % rrows] = y
                    vslot[y & 15] = y
            for wv in range(nw):
                r = ya0 + j * nw + wv - lag
                if not (ya <= r < yb):
                    continue
                for rs in (r - 1, r, r + 1):
                    if 0 <= rs < ny and slot.get(rs % rrows) != rs:
                        return False
                if lag == 2:  # the outlet ghost of row rsrc reads rows rsrc - 1 .. rsrc + 1, clamped
                    for rs in (r - 1, r, r + 1):
                        if 0 <= rs < ny:
                            for v in (max(rs - 1, 0), rs, min(rs + 1, ny - 1)):
                                if vslot.get(v & 15) != v:
                                    return False
    return True


# ---------------------------------------------------------------------------


def test_model_reads_the_words_the_definition_names_on_the_papers_channel():
    """512 x 128, square 16 at the centre, grid of 8-cell bars from x = 32."""
    g = Geometry(512, 128, (248, 56, 16), open_=True, gx0=32, bar=8)
    assert check_member(g) == []


def test_model_on_the_grid_geometry_of_the_open_channel_tests():
    """The geometry of the GPU tests' grid runs, OpenParams(0.05, 12, 6, ...),
    on a two-step lattice (nx a multiple of 256), with the square near it."""
    for square in [(70, 19, 8), (20, 10, 6), (24, 3, 5)]:
        g = Geometry(512, 48, square, open_=True, gx0=12, bar=6)
        assert check_member(g) == [], square


@pytest.mark.parametrize("open_", [False, True])
def test_model_squares_at_every_offset_from_a_strip_seam(open_):
    """Squares whose edges fall on every column from 6 left to 6 right of the
    seam between two strips and of a lane boundary, near the walls and not."""
    for sx0 in list(range(242, 262)) + list(range(3, 9)):
        for ss, sy0 in [(2, 1), (5, 9), (3, 24 - 3 - 1)]:
            g = Geometry(512, 24, (sx0, sy0, ss), open_=open_, gx0=0, bar=0)
            rows = range(max(sy0 - 2, 0), min(sy0 + ss + 2, 24))
            assert check_member(g, rows) == [], (sx0, sy0, ss)


def test_model_grid_bars_at_every_offset_from_a_strip_seam():
    """Grid bars whose first or last column falls on every column from 6 left
    to 6 right of the seam at x = 256 (and of the inlet end), for bar sizes 1
    to 4: in particular a bar ending two columns left of the seam, or starting
    two columns right of it, which only the strips' outside cells touch."""
    for bar in (1, 2, 3, 4):
        for gx0 in sorted(set(list(range(248 - bar, 264)) + list(range(1, 8)))):
            g = Geometry(512, 20, (400, 6, 4), open_=True, gx0=gx0, bar=bar)
            assert check_member(g) == [], (gx0, bar)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_model_on_seeded_random_geometries(seed):
    """The seeded sweep of the GPU bounce-back test, square and grid drawn the
    same way, every row checked."""
    rng = np.random.default_rng(seed)
    for case in range(4):
        nx, ny, s = 512, int(rng.integers(20, 48)), int(rng.integers(2, 9))
        square = (int(rng.integers(24, nx - s - 4)), int(rng.integers(1, ny - s - 1)), s)
        open_, gx0, bar = False, 0, 0
        if case % 2:
            bar = int(rng.integers(2, 7))
            gx0 = int(rng.integers(2, square[0] - bar - 3))
            rng.integers(300, nx - 20)  # the sponge column of the GPU test (unused here)
            open_ = True
        assert check_member(Geometry(nx, ny, square, open_, gx0, bar)) == [], (seed, case)


def test_model_finds_a_planted_mask_mistake(monkeypatch):
    """The model is not vacuous: with the strips' grid-column range one column
    narrower, [base - 1, base + 256] (what the strip's own cells need; the
    kernel used it for the outside cells too), a bar ending two columns left
    of a seam is missed, and the model reports the outside cell that pulls
    from the bar instead of bouncing back, and the strip-edge cell of phase B
    that takes the outside cell's wrong result."""
    g = Geometry(512, 20, (400, 6, 4), open_=True, gx0=253, bar=2)  # bars at 253, 254; seam at 256
    assert check_member(g) == []

    def narrow(self, base):
        return self.g.open and self.g.bar > 0 and base <= self.g.gx0 + self.g.bar and base + STRIP - 1 >= self.g.gx0 - 1

    monkeypatch.setattr(Kernel, "grid_cols", narrow)
    bad = check_member(g)
    assert any(b[0] == "A outside" and b[2] == 255 for b in bad), bad[:3]


@pytest.mark.parametrize("nw", [2, 4, 8])
@pytest.mark.parametrize("lag", [1, 2])
def test_ring_slots_hold_the_rows_phase_b_reads(nw, lag):
    for ny in (1, 2, 3, 7, 16, 33, 128):
        assert ring_slots_ok(ny, nw, lag), ny
        for split in (1, 2, 5, 16):
            assert ring_slots_ok(ny, nw, lag, split), (ny, split)


def _c_rem(a, b):
    """C's a % b (the sign of a)."""
    r = abs(a) % b
    return -r if a < 0 else r


def test_grid_row_phase_matches_the_row_test():
    """The kernel does not test rows for the grid directly: each wave carries the phase
    (y - bar/2) mod 2 bar of its phase-A row, set once by a division and advanced by NW rows per
    iteration, and derives the bits for rows y - 1, y, y + 1 (phase A) and for r = y - LAG
    (phase B) from it.  They equal the direct row test on every row, wave, lag and row range."""
    def direct(ny, bar, yy):
        r = yy - (bar >> 1)
        return 0 <= yy < ny and bar > 0 and r >= 0 and r % (2 * bar) < bar

    def bits_direct(ny, bar, yy):
        return sum((1 << k) for k, d in enumerate((-1, 0, 1)) if direct(ny, bar, yy + d))

    def bits_phase(ny, bar, yy, ph):
        gper, ghalf = 2 * bar, bar >> 1
        grow = lambda y, p: ghalf <= y < ny and p < bar
        pm = gper - 1 if ph == 0 else ph - 1
        pp = 0 if ph + 1 == gper else ph + 1
        return (1 if grow(yy - 1, pm) else 0) | (2 if grow(yy, ph) else 0) | (4 if grow(yy + 1, pp) else 0)

    checked = 0
    for bar in range(1, 10):
        gper, ghalf = 2 * bar, bar >> 1
        for ny in (1, 2, 5, 37, 128):
            for nw in (2, 4, 8):
                for lag in (1, 2):
                    for split in (None, 5, 16):
                        segs = [(0, ny)] if split is None else [(a, min(a + split, ny)) for a in range(0, ny, split)]
                        for ya, yb in segs:
                            ya0, ya1 = (max(ya - lag, 0), min(yb + lag, ny)) if split else (0, ny)
                            iters = (yb + lag - ya0 + nw - 1) // nw if split else (ny + lag - 1) // nw + 1
                            for wv in range(nw):
                                r0 = _c_rem(ya0 + wv - ghalf, gper)
                                gph = r0 + gper if r0 < 0 else r0
                                for j in range(iters):
                                    y = ya0 + j * nw + wv
                                    if y < ya1:
                                        assert bits_phase(ny, bar, y, gph) == bits_direct(ny, bar, y)
                                        checked += 1
                                    r = y - lag
                                    phb = gph - lag
                                    phb += gper if phb < 0 else 0
                                    phb += gper if phb < 0 else 0
                                    if ya <= r < yb:
                                        assert bits_phase(ny, bar, r, phb) == bits_direct(ny, bar, r), (bar, ny, nw, lag, r)
                                        checked += 1
                                    gph += nw
                                    while gph >= gper:
                                        gph -= gper
    assert checked > 10000
