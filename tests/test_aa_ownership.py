"""Slot ownership of one odd AA step, replayed on the CPU.

The stepping kernel updates the population store in place; an odd step reads
slot 26-i at x - c_i and writes slot i at x + c_i, and the boundary rules
redirect some of these accesses (inlet equilibrium, outflow ghost plane,
bounce-back and free-slip walls, extra writes for the slots no fluid cell
pushes). This module replays, cell by cell, the addresses that the open-domain
launch pair touches: the 32-bit fast path over every cell off the z walls
(periodic index wrap, then the inflow/outflow rules per lane, with its
pre-loads from wrapped positions that the x = 0 and x = nx-1 lanes replace)
and the general-path kernel over the two wall planes, and checks:

  1. every slot has at most one writer over both launches;
  2. a slot whose loaded value a cell uses is written by no other cell (so
     neither the order of threads inside a launch nor the order of the two
     launches matters);
  3. every slot the next (even) step reads is written exactly once;
  4. with 16-bit storage on whole 256-wide rows, the staged stores (each lane
     stores the value aimed at its own x) write the same slots, each from
     inside the workgroup that owns it.

A mistake planted in the replay (pushes out of the box through x = 0 no longer
dropped) breaks rule 1 on the outlet-side slots of x = nx-1, which the
zero-gradient extra writes fill. The geometries are those of the GPU boundary
and degenerate-case parity tests. Pure host logic, no GPU."""
import itertools

import pytest

PER, INOUT, NOSLIP, FREESLIP = "periodic", "inout", "noslip", "freeslip"


def cx(i):
    return i % 3 - 1


def cy(i):
    return (i // 3) % 3 - 1


def cz(i):
    return i // 9 - 1


def refl_z(i):
    return i - 18 * cz(i)


def wrap(v, n):
    return v % n


class Replay:
    """Slot accesses of one odd step: writes[slot] = [writer cells],
    used_reads[slot] = [reader cells], discarded = pre-loads replaced by a
    boundary value."""

    def __init__(self, nx, ny, nz, bc_x, bc_zlo, bc_zhi, drop_x0_pushes=True):
        self.n = (nx, ny, nz)
        self.bc_x, self.bc_zlo, self.bc_zhi = bc_x, bc_zlo, bc_zhi
        self.drop_x0_pushes = drop_x0_pushes
        self.writes, self.used_reads, self.discarded = {}, {}, []

    def _w(self, slot, cell):
        self.writes.setdefault(slot, []).append(cell)

    def _r(self, slot, cell):
        self.used_reads.setdefault(slot, []).append(cell)

    # fast path: every cell off the z walls, z wraps (periodic z) or stays in
    def fast_cell(self, x, y, z):
        nx, ny, nz = self.n
        cell = (x, y, z)
        xo = self.bc_x == INOUT
        for i in range(27):
            src = (26 - i, wrap(x - cx(i), nx), wrap(y - cy(i), ny), wrap(z - cz(i), nz))
            replaced = xo and ((x == 0 and cx(i) == 1) or (x == nx - 1 and cx(i) == -1))
            if replaced:
                self.discarded.append((src, cell))
            else:
                self._r(src, cell)
        for i in range(27):
            if xo and cx(i) == -1 and x == 0 and self.drop_x0_pushes:
                continue
            if xo and cx(i) == 1 and x == nx - 1:
                continue
            self._w((i, wrap(x + cx(i), nx), wrap(y + cy(i), ny), wrap(z + cz(i), nz)), cell)
        if xo:
            self.extras(x, y, z)

    def extras(self, x, y, z):
        """slots no fluid cell pushes: inlet equilibrium at x = 0, zero-gradient
        copy at x = nx-1 (the z rules resolved first, as in the kernel)"""
        nx, ny, nz = self.n
        cell = (x, y, z)
        if x == 0:
            for i in [k for k in range(27) if cx(k) == 1]:
                sz = z - cz(i)
                if cz(i) != 0 and not 0 <= sz < nz and (self.bc_zlo if sz < 0 else self.bc_zhi) == NOSLIP:
                    continue
                self._w((i, 0, y, z), cell)
        if x == nx - 1:
            for j in [k for k in range(27) if cx(k) == -1]:
                ty, tz = wrap(y + cy(j), ny), z + cz(j)
                if cz(j) != 0 and not 0 <= tz < nz:
                    bc = self.bc_zlo if tz < 0 else self.bc_zhi
                    if bc == NOSLIP:
                        continue
                    if bc == FREESLIP:
                        self._w((refl_z(j), x, ty, z), cell)
                        continue
                    tz = wrap(tz, nz)
                self._w((j, x, ty, tz), cell)

    # general path (the wall planes): per-direction boundary rules
    def general_cell(self, x, y, z):
        nx, ny, nz = self.n
        cell = (x, y, z)
        for i in range(27):
            sx, sy, sz = x - cx(i), y - cy(i), z - cz(i)
            ii = i
            if cz(i) != 0 and not 0 <= sz < nz:
                bc = self.bc_zlo if sz < 0 else self.bc_zhi
                if bc == NOSLIP:
                    self._r((i, x, y, z), cell)
                    continue
                if bc == FREESLIP:
                    ii, sz = refl_z(i), z
                else:
                    sz = wrap(sz, nz)
            sy = wrap(sy, ny)
            if cx(i) != 0 and not 0 <= sx < nx:
                if self.bc_x == PER:
                    sx = wrap(sx, nx)
                else:
                    continue  # inlet value or ghost plane: no store slot
            self._r((26 - ii, sx, sy, sz), cell)
        for i in range(27):
            tx, ty, tz = x + cx(i), y + cy(i), z + cz(i)
            jj = i
            if cz(i) != 0 and not 0 <= tz < nz:
                bc = self.bc_zlo if tz < 0 else self.bc_zhi
                if bc == NOSLIP:
                    self._w((26 - i, x, y, z), cell)
                    continue
                if bc == FREESLIP:
                    jj, tz = refl_z(i), z
                else:
                    tz = wrap(tz, nz)
            ty = wrap(ty, ny)
            if cx(i) != 0 and not 0 <= tx < nx:
                if self.bc_x != PER:
                    continue
                tx = wrap(tx, nx)
            self._w((jj, tx, ty, tz), cell)
        if self.bc_x == INOUT:
            self.extras(x, y, z)

    def run(self, general_everywhere=False):
        nx, ny, nz = self.n
        walls = self.bc_zlo != PER
        for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
            on_wall = walls and z in (0, nz - 1)
            if general_everywhere or on_wall:
                self.general_cell(x, y, z)
            else:
                self.fast_cell(x, y, z)
        return self


def check(rep):
    nx, ny, nz = rep.n
    multi = {s: w for s, w in rep.writes.items() if len(w) > 1}
    assert not multi, f"slots with several writers: {list(multi.items())[:3]}"
    for slot, readers in rep.used_reads.items():
        assert len(readers) == 1, (slot, readers)
        writers = rep.writes.get(slot, [])
        assert all(w == readers[0] for w in writers), (slot, readers, writers)
    missing = [(i, x, y, z) for i in range(27) for z in range(nz) for y in range(ny) for x in range(nx)
               if (i, x, y, z) not in rep.writes]
    assert not missing, f"{len(missing)} slots of the next step unwritten, e.g. {missing[:3]}"


GEOMS = [
    ((20, 12, 10), INOUT, PER, PER),
    ((20, 12, 10), PER, NOSLIP, NOSLIP),
    ((20, 12, 10), PER, FREESLIP, FREESLIP),
    ((20, 12, 10), PER, NOSLIP, FREESLIP),
    ((20, 12, 10), INOUT, NOSLIP, FREESLIP),
    ((20, 12, 10), INOUT, NOSLIP, NOSLIP),
    ((20, 12, 10), INOUT, FREESLIP, FREESLIP),
    ((2, 3, 2), INOUT, NOSLIP, FREESLIP),
    ((3, 2, 4), PER, NOSLIP, NOSLIP),
    ((2, 5, 3), INOUT, PER, PER),
    ((37, 9, 6), INOUT, NOSLIP, FREESLIP),
]


@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: f"{g[0][0]}x{g[0][1]}x{g[0][2]}-{g[1]}-{g[2]}-{g[3]}")
@pytest.mark.parametrize("general", [False, True], ids=["fast+walls", "general"])
def test_odd_step_slot_ownership(geom, general):
    shape, bx, zlo, zhi = geom
    check(Replay(*shape, bx, zlo, zhi).run(general_everywhere=general))


def test_discarded_preloads_are_the_boundary_slots():
    """The x = 0 and x = nx-1 lanes of the fast path first load from wrapped
    positions, then replace those values by the inlet equilibrium or the ghost
    plane: those loads land exactly on the slots the other boundary's extra
    writes fill in the same step (harmless: the values are never used)."""
    rep = Replay(20, 12, 10, INOUT, NOSLIP, FREESLIP).run()
    assert rep.discarded
    for (slot, cell) in rep.discarded:
        i, x = slot[0], slot[1]
        assert (cell[0] == 0 and x == 19 and cx(i) == -1) or (cell[0] == 19 and x == 0 and cx(i) == 1)


def test_planted_undropped_x0_push_breaks_ownership():
    """Pushes out of the box through x = 0, if not dropped, wrap onto the
    outlet-side slots of x = nx-1 that the zero-gradient extra writes fill:
    two writers per slot."""
    rep = Replay(20, 12, 10, INOUT, NOSLIP, FREESLIP, drop_x0_pushes=False).run()
    with pytest.raises(AssertionError, match="several writers"):
        check(rep)
    doubled = [s for s, w in rep.writes.items() if len(w) > 1]
    assert doubled and all(s[1] == 19 and cx(s[0]) == -1 for s in doubled)


def test_staged_stores_write_the_same_slots_inside_the_workgroup():
    """16-bit storage on whole 256-wide rows stores the 18 x-shifted
    directions through LDS: lane t stores the value aimed at its own x
    (lanes 0 and 255 also the pushes across the tile edges x0 - 1 and
    x0 + 256). The slots equal the direct pushes', and each is stored by a
    lane of the tile that produced the value."""
    nx, ny, nz = 512, 3, 3
    for bc_x in (PER, INOUT):
        direct = Replay(nx, ny, nz, bc_x, PER, PER)
        staged = {}
        for z, y in itertools.product(range(nz), range(ny)):
            for x0 in range(0, nx, 256):
                for t in range(256):
                    x = x0 + t
                    for i in range(27):
                        if cx(i) == 0:
                            continue
                        # the push of lane t for direction i targets x + c_x; the
                        # storing lane is the one whose own x that is, or the
                        # edge lane for the pushes across the tile edge
                        tx = x + cx(i)
                        if bc_x == INOUT and not 0 <= tx < nx:
                            continue  # dropped at the box faces
                        if x0 <= tx < x0 + 256:
                            store_lane = tx - x0
                        else:
                            store_lane = 255 if cx(i) == -1 else 0
                        slot = (i, wrap(tx, nx), wrap(y + cy(i), ny), wrap(z + cz(i), nz))
                        staged.setdefault(slot, []).append(((x0, y, z), store_lane))
        direct.run()
        shifted = {s: w for s, w in direct.writes.items()
                   if cx(s[0]) != 0 and not (bc_x == INOUT and (w[0][0] in (0, nx - 1)) and s[1] in (0, nx - 1)
                                             and len(w) == 1 and _is_extra(s, w[0], nx))}
        for slot, writers in shifted.items():
            assert slot in staged, slot
            assert len(staged[slot]) == 1, (slot, staged[slot])
            (tile, lane) = staged[slot][0]
            producer = writers[0]
            assert (producer[0] // 256) * 256 == tile[0] and producer[1:] == tile[1:], (slot, producer, tile)
        assert len(staged) == len(shifted)


def _is_extra(slot, cell, nx):
    """a slot filled by an inlet / outlet extra write (not a push)"""
    i, x = slot[0], slot[1]
    return (cell[0] == 0 and x == 0 and cx(i) == 1) or (cell[0] == nx - 1 and x == nx - 1 and cx(i) == -1)
