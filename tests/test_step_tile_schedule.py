"""Host replay of the step kernel's LDS schedule (csrc/sgn_fused.hpp, step_tile).

A model of the kernel's index arithmetic, phase by phase as its barriers
separate them: staging (every thread writes its share of the region),
then for each of the four stages an evaluation phase (LDS reads only: the
two or three owned nodes per thread, then up to two ring nodes) and a write-back
phase (the stage just formed replaces the one read).  For every tile of a
grid the replay checks that

  * every LDS read and write stays inside the staged region, rows [0, RY) and
    columns [0, RX) -- so with padded rows the pad column is never touched and
    the padded and unpadded layouts are relabelings of the same slots;
  * every read finds the version of the stage being evaluated (the staged
    state for k1, Y_s for k_s), written in an earlier phase; the bathymetry
    plane is written once, at staging;
  * no slot is written twice in one write-back phase;
  * node 1 shares its centre and lower neighbour with node 0's upper
    neighbour and centre, and node 2 its lower neighbour with node 1's centre,
    exactly when the kernel relies on it;
  * ring slots 0 .. RING3-1 cover the rings at distance 1..3 once each.

The replay covers the manufactured-source instances too: the source is added
to the rates in registers and touches no LDS, so their schedule is the one
replayed here.  No GPU needed."""

import itertools

import pytest

PER, REF = 0, 1
THREADS = 256
HALO = 4
SHAPES = {8: 64, 16: 32, 24: 32}  # tile height -> width: 64 x 8, 32 x 16, 32 x 24
PLANES = 7          # h u v w eta b 1/h
B_PLANE = 5


def stencil(i, n, bc):
    """(om, op): LDS offsets of the left/right neighbours (closure rows at walls)."""
    om, op = -1, 1
    if bc == REF:
        if i == 0:
            om = 0
        if i == n - 1:
            op = 0
    return om, op


def on_axis(g, n, bc):
    return True if bc == PER else 0 <= g < n


def ring_count(tx, ty, d):
    return 2 * (tx + 2 * d) + 2 * (ty + 2 * d - 2)


def ring_node(m, tx, ty):
    r1 = ring_count(tx, ty, 1)
    r2 = r1 + ring_count(tx, ty, 2)
    if m < r1:
        d = 1
    elif m < r2:
        d, m = 2, m - r1
    else:
        d, m = 3, m - r2
    w = tx + 2 * d
    hs = ty + 2 * d - 2
    if m < w:
        return -d, m - d
    if m < 2 * w:
        return ty - 1 + d, m - w - d
    if m < 2 * w + hs:
        return m - 2 * w - d + 1, -d
    return m - 2 * w - hs - d + 1, tx - 1 + d


class Lds:
    def __init__(self, rx, ry, pad):
        self.rx, self.ry, self.row = rx, ry, rx + pad
        self.version = {}

    def slot(self, f, r, c):
        assert 0 <= r < self.ry and 0 <= c < self.rx, ("outside the staged region", f, r, c)
        return (f * self.ry + r) * self.row + c

    def write(self, f, r, c, ver, seen):
        s = self.slot(f, r, c)
        assert s not in seen, ("written twice in one phase", f, r, c)
        seen.add(s)
        self.version[s] = ver

    def read_node(self, r, c, want):
        for f in range(PLANES):
            s = self.slot(f, r, c)
            assert s in self.version, ("read before written", f, r, c)
            got = self.version[s]
            assert got == (0 if f == B_PLANE else want), ("stale stage", f, r, c, got, want)


def replay_tile(nx, ny, bcx, bcy, ty, pad, i0, j0, skip_slot=None):
    tx = SHAPES[ty]
    no = tx * ty // THREADS  # owned nodes per thread
    rx, ry = tx + 2 * HALO, ty + 2 * HALO
    rings = [ring_count(tx, ty, 1)]
    rings += [rings[0] + ring_count(tx, ty, 2), rings[0] + ring_count(tx, ty, 2) + ring_count(tx, ty, 3)]
    ring3 = rings[2]
    assert ring3 <= 2 * THREADS
    lds = Lds(rx, ry, pad)

    # staging: version 0 (the step's input state) everywhere in the region
    seen = set()
    for idx in range(rx * ry):
        rr, cc = divmod(idx, rx)
        for f in range(PLANES):
            lds.write(f, rr, cc, 0, seen)

    # thread map
    own = []
    for tid in range(THREADS):
        lx, ly0 = tid % tx, no * (tid // tx)
        i, j = i0 + lx, j0 + ly0
        own.append((lx, ly0, i, j, [on_axis(i, nx, bcx) and on_axis(j + k, ny, bcy) for k in range(no)]))
    ring = []
    for tid in range(THREADS):
        for k in (0, 1):
            m = tid + k * THREADS
            if m < ring3 and m != skip_slot:
                r, c = ring_node(m, tx, ty)
                ring.append((m, r, c, on_axis(i0 + c, nx, bcx) and on_axis(j0 + r, ny, bcy)))

    for st in (1, 2, 3, 4):
        want = st - 1
        ring_lim = rings[3 - st] if st < 4 else 0
        # evaluation phase: reads only
        for lx, ly0, i, j, od in own:
            run = [od[k] if st < 4 else (i < nx and j + k < ny) for k in range(no)]
            if not run[0]:
                continue
            r, c = ly0 + HALO, lx + HALO
            om, op = stencil(i, nx, bcx)
            ym0, yp0 = stencil(j, ny, bcy)
            for rr, cc in ((r, c), (r + yp0, c), (r, c + om), (r, c + op), (r + ym0, c)):
                lds.read_node(rr, cc, want)
            if run[1]:
                ym1, yp1 = stencil(j + 1, ny, bcy)
                # node 1's centre is node 0's upper neighbour, its lower neighbour node 0's centre
                assert r + yp0 == r + 1 and (r + 1) + ym1 == r, (i, j)
                for rr, cc in ((r + 1, c + om), (r + 1, c + op), (r + 1 + yp1, c)):
                    lds.read_node(rr, cc, want)
                if no == 3 and run[2]:
                    ym2, yp2 = stencil(j + 2, ny, bcy)
                    # node 2's lower neighbour is node 1's centre; its own centre is read again
                    assert (r + 2) + ym2 == r + 1, (i, j)
                    for rr, cc in ((r + 2, c), (r + 2, c + om), (r + 2, c + op), (r + 2 + yp2, c)):
                        lds.read_node(rr, cc, want)
            elif no == 3:
                assert not run[2], (i, j)  # node 2 in the domain implies node 1 in the domain
            if st == 4:
                for k in range(no):
                    if run[k]:
                        lds.slot(B_PLANE, ly0 + k + HALO, lx + HALO)  # epilogues read b of the owned node
        if st == 4:
            break
        for m, rr, cc, ok in ring:
            if m >= ring_lim or not ok:
                continue
            om, op = stencil(i0 + cc, nx, bcx)
            ym, yp = stencil(j0 + rr, ny, bcy)
            r, c = rr + HALO, cc + HALO
            for a, b in ((r, c), (r, c + om), (r, c + op), (r + ym, c), (r + yp, c)):
                lds.read_node(a, b, want)
        # write-back phase: the stage just formed (every plane but b)
        seen = set()
        for lx, ly0, i, j, od in own:
            for k in range(no):
                if od[k]:
                    for f in range(PLANES):
                        if f != B_PLANE:
                            lds.write(f, ly0 + k + HALO, lx + HALO, st, seen)
        for m, rr, cc, ok in ring:
            if m < ring_lim and ok:
                for f in range(PLANES):
                    if f != B_PLANE:
                        lds.write(f, rr + HALO, cc + HALO, st, seen)


def tiles(nx, ny, ty):
    tx = SHAPES[ty]
    for j0 in range(0, ny, ty):
        for i0 in range(0, nx, tx):
            yield i0, j0


@pytest.mark.parametrize("ty", [8, 16, 24])
def test_ring_map_covers_each_ring_node_once(ty):
    tx = SHAPES[ty]
    total = sum(ring_count(tx, ty, d) for d in (1, 2, 3))
    got = [ring_node(m, tx, ty) for m in range(total)]
    assert len(set(got)) == total
    expect = {(r, c) for r in range(-3, ty + 3) for c in range(-3, tx + 3)
              if not (0 <= r < ty and 0 <= c < tx)}
    assert set(got) == expect


@pytest.mark.parametrize("ty,pad", list(itertools.product([8, 16, 24], [0, 1])))
@pytest.mark.parametrize("bcx,bcy", [(REF, REF), (PER, PER), (REF, PER), (PER, REF)])
def test_schedule_40x40(ty, pad, bcx, bcy):
    """The grid of the manufactured-solution tests (40 x 40): every tile."""
    for i0, j0 in tiles(40, 40, ty):
        replay_tile(40, 40, bcx, bcy, ty, pad, i0, j0)


@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("nx,ny", [(4, 4), (5, 9), (70, 257), (129, 33), (33, 25), (40, 49)])
def test_schedule_ragged_and_tiny(ty, nx, ny):
    for bcx, bcy in ((REF, REF), (PER, PER)):
        for i0, j0 in tiles(nx, ny, ty):
            replay_tile(nx, ny, bcx, bcy, ty, 1, i0, j0)


def test_replay_detects_a_stale_neighbour():
    """The replay is sharp: leaving out one ring-3 node at stage 1 leaves a stale
    value that a ring-2 evaluation reads at stage 2."""
    ty, tx = 8, SHAPES[8]
    last = ring_count(tx, ty, 1) + ring_count(tx, ty, 2) + ring_count(tx, ty, 3) - 1
    replay_tile(200, 200, PER, PER, ty, 1, 64, 64)
    with pytest.raises(AssertionError, match="stale stage"):
        replay_tile(200, 200, PER, PER, ty, 1, 64, 64, skip_slot=last)
