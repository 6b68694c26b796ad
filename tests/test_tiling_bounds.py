"""CPU replay of the index arithmetic of the 3D step kernel (step3_kernel,
load3, the Neumann mirror loads) and of the two-step 2D kernel
(step2_body: the prefetched rows, the LDS rings, the delayed stores) for
every kernel variant the library lists, on lattices smaller than one tile,
one z slice group or one two-step window, and on ragged ones.

Each replay walks the launch grid the host builds (blocks, XCD-contiguous
item order, threads, z slices or row passes) with the formulas of the
kernel source and asserts that every global load and store offset lies
inside the q planes, every statistics slot inside the item table, every
LDS index inside its array, and, for the rings, that each row read from
LDS is the row the update wants (no slot was overwritten too early).
The variant table is read from the library (lbm_stefan_variant_name), so
a variant added to the table is replayed too; nothing runs on a GPU.
"""
import itertools
import os
import re

import numpy as np
import pytest


@pytest.fixture(scope="module")
def names():
    from paper_2505_13097_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2505_13097_amd import build
        build.build(verbose=False)
    from paper_2505_13097_amd import variant_names
    return {q: variant_names(q, "f64") for q in (5, 9, 7, 19)}


def _dirs3(q):
    """velocity set of D3Q7 (faces) or D3Q19 (faces and edges)"""
    out = [(0, 0, 0)]
    for v in itertools.product((-1, 0, 1), repeat=3):
        nz = sum(abs(c) for c in v)
        if nz == 1 or (q == 19 and nz == 2):
            out.append(v)
    assert len(out) == q
    return out


def _dirs2(q):
    out = [(0, 0)]
    for v in itertools.product((-1, 0, 1), repeat=2):
        nz = sum(abs(c) for c in v)
        if nz == 1 or (q == 9 and nz == 2):
            out.append(v)
    assert len(out) == q
    return out


# ---------------------------------------------------------------------
# 3D: step3_kernel

def _parse3(name):
    m = re.fullmatch(r"(\d+)x(\d+)/npt(\d+)/z(\d+)(/nt)?(/s)?", name)
    tw, by, npt, cz = (int(m.group(k)) for k in range(1, 5))
    return tw // npt, by, npt, cz


# the 3D item order's bands of rows (kBand3Rows of lattice3d.hpp)
BAND3_ROWS = 128


def replay3(q, nx, ny, nz, bx, by, npt, cz, periodic=(0, 0, 0),
            neu=(0, 0, 0, 0, 0, 0), bad_fast=False, x_off=0, x_lim=None,
            out=None, bad_row=False):
    """Every offset step3_kernel touches; returns the number checked.
    bad_fast: widen the fast path's x guard by one (a planted mistake).
    x_off, x_lim: the split step's column range (tiles from x_off, no
    update from x_lim on); out, if given, receives the stores per node
    ([z][y][x]).  The interior-row path (xrow: both x faces Dirichlet or
    bounce-back, so neither periodic nor Neumann here) is replayed for the
    rows off the y and z faces of tiles off the fast path; bad_row: its x
    sources left unclamped (a planted mistake)."""
    xrow = nx >= 3 and not periodic[0] and not neu[0] and not neu[1]
    P = nx * ny * nz
    n = (nx, ny, nz)
    tw = bx * npt
    x_lim = nx if x_lim is None else x_lim
    tiles = (-(-(x_lim - x_off) // tw), -(-ny // by), -(-nz // cz))
    nitems = tiles[0] * tiles[1] * tiles[2]
    per_xcd = (nitems + 7) // 8
    dirs = _dirs3(q)
    assert bx % 64 == 0 and bx * by <= 256      # __launch_bounds__(256)
    checked = 0
    seen = np.zeros(nitems, dtype=int)
    tyy, txx = np.meshgrid(np.arange(by), np.arange(bx), indexing="ij")

    def check(i, cx, cy, cz_):
        """node (cx, cy, cz_) of plane i: each coordinate inside its axis,
        the flat offset inside the planes"""
        nonlocal checked
        for v, m in ((cx, nx), (cy, ny), (cz_, nz)):
            v = np.asarray(v)
            assert v.min() >= 0 and v.max() < m, (v.min(), v.max(), m)
        off = i * P + (np.asarray(cz_) * ny + cy) * nx + cx
        assert off.min() >= 0 and off.max() < q * P
        checked += np.size(off)

    for b in range(8 * per_xcd):
        t = (b & 7) * per_xcd + (b >> 3)
        if t >= nitems:
            continue
        seen[t] += 1                      # the block's statistics slot
        tx = t % tiles[0]
        r = t // tiles[0]
        # bands of tile rows, each through all its z chunks (set_tiling3)
        band = max(1, BAND3_ROWS // by)
        per = band * tiles[2]
        bi, rr = r // per, r % per
        bw = min(band, tiles[1] - bi * band)
        ty, tz = bi * band + rr % bw, rr // bw
        x0, y0 = x_off + tx * tw, ty * by
        z0, z1 = tz * cz, min(tz * cz + cz, nz)
        fxy = (x0 >= 1 and x0 + tw <= nx - (0 if bad_fast else 1) and
               x0 + tw <= x_lim and y0 >= 1 and y0 + by <= ny - 1)
        for z in range(z0, z1):
            fast = fxy and 1 <= z <= nz - 2
            for k in range(npt):
                x = (x0 + txx + k * bx).ravel()
                y = (y0 + tyy).ravel()
                if not fast and xrow and 1 <= z <= nz - 2:
                    # rows off the y and z faces (a wave is one row): every
                    # lane loads, at its column clamped into the row, the x
                    # sources clamped too; lanes inside the row and before
                    # x_lim store
                    row = (y >= 1) & (y <= ny - 2)
                    xc = np.minimum(x[row], nx - 1)
                    yr = y[row]
                    if xc.size:
                        st = x[row] < min(nx, x_lim)
                        if out is not None:
                            np.add.at(out, (np.full(st.sum(), z), yr[st],
                                            x[row][st]), 1)
                        for i, e in enumerate(dirs):
                            check(i, xc, yr, np.full_like(xc, z))
                            sx = xc - e[0]
                            if e[0] != 0 and not bad_row:
                                sx = np.clip(sx, 0, nx - 1)
                            check(i, sx, yr - e[1], np.full_like(xc, z - e[2]))
                    x, y = x[~row], y[~row]
                if not fast:
                    keep = (x < x_lim) & (y < ny)
                    x, y = x[keep], y[keep]
                if x.size == 0:
                    continue
                if out is not None:
                    np.add.at(out, (np.full_like(x, z), y, x), 1)
                c = (x, y, np.full_like(x, z))
                # neighbours: unclamped on the fast path, wrapped or
                # clamped elsewhere (neighbours3)
                m, p = [], []
                for a in range(3):
                    mm, pp = c[a] - 1, c[a] + 1
                    if not fast:
                        mm = np.where(mm < 0, mm + n[a] if periodic[a] else 0,
                                      mm)
                        pp = np.where(pp >= n[a], pp - n[a] if periodic[a]
                                      else n[a] - 1, pp)
                    m.append(mm)
                    p.append(pp)
                for i, e in enumerate(dirs):
                    check(i, x, y, z)             # own populations, store
                    s = [m[a] if e[a] == 1 else (p[a] if e[a] == -1 else c[a])
                         for a in range(3)]
                    check(i, s[0], s[1], s[2])
                if not fast and any(neu):
                    # mirror_m0_3: sources of the mirror node, clamped
                    mir = [c[a].copy() for a in range(3)]
                    on = np.zeros(x.size, dtype=bool)
                    for a in range(3):
                        if neu[2 * a]:
                            hit = c[a] == 0
                            mir[a] = np.where(hit, 1, mir[a])
                            on |= hit
                        if neu[2 * a + 1]:
                            hit = c[a] == n[a] - 1
                            mir[a] = np.where(hit, n[a] - 2, mir[a])
                            on |= hit
                    for i, e in enumerate(dirs):
                        s = []
                        for a in range(3):
                            v = mir[a][on] - e[a]
                            v = np.where(v < 0, v + n[a] if periodic[a] else 0,
                                         v)
                            v = np.where(v >= n[a], v - n[a] if periodic[a]
                                         else n[a] - 1, v)
                            s.append(v)
                        if s[0].size:
                            check(i, s[0], s[1], s[2])
    assert np.all(seen == 1)              # every item once, one slot each
    return checked


SHAPES3 = [(12, 9, 7), (3, 3, 3), (4, 3, 5), (65, 5, 9), (130, 6, 10)]


@pytest.mark.parametrize("q", [7, 19])
def test_3d_kernel_offsets_inside_planes(names, q):
    for name in names[q]:
        bx, by, npt, cz = _parse3(name)
        for shape in SHAPES3:
            for per in ((0, 0, 0), (1, 0, 1)):
                assert replay3(q, *shape, bx, by, npt, cz, per) > 0
            # the freezing octant's Neumann faces (x+, y+, z+)
            replay3(q, *shape, bx, by, npt, cz, (0, 0, 0),
                    (0, 1, 0, 1, 0, 1))


# the 3D split step: front strip of FRONT3_COLUMNS columns with the tiling
# of FRONT3 (kFront3Columns, kFront3Variant of lattice3d.hpp)
FRONT3_COLUMNS = 64
FRONT3 = (64, 4, 1, 32)


@pytest.mark.parametrize("q", [7, 19])
def test_3d_split_step_stores_every_node_once(names, q):
    """Split variants: the front strip (columns below 64) and the quiet
    and full passes (tiles from column 64) store every node once, every
    access inside the planes."""
    split = [n for n in names[q] if n.endswith("/s")]
    assert split
    for name in split:
        bx, by, npt, cz = _parse3(name)
        for shape in [(129, 6, 10), (200, 5, 7), (130, 3, 3), (320, 9, 4)]:
            nx, ny, nz = shape
            assert nx > 2 * FRONT3_COLUMNS
            for per in ((0, 0, 0), (0, 1, 1)):
                out = np.zeros((nz, ny, nx), dtype=int)
                replay3(q, *shape, *FRONT3, per, x_lim=FRONT3_COLUMNS,
                        out=out)
                replay3(q, *shape, bx, by, npt, cz, per,
                        x_off=FRONT3_COLUMNS, out=out)
                assert np.all(out == 1), (name, shape)


@pytest.mark.parametrize("q", [7, 19])
def test_3d_step_stores_every_node_once(names, q):
    """The plain 3D step of every variant: the fast path, the interior-row
    path (rows off the y and z faces of tiles holding an x face or a ragged
    end) and the bounds-checked path together store every node once, with
    the interior-row path on (Dirichlet or bounce-back x faces) and off
    (a periodic x axis, a Neumann x face)."""
    for name in names[q]:
        if name.endswith("/s"):
            continue
        bx, by, npt, cz = _parse3(name)
        # (70, 300, 6): several bands of rows and a ragged last band
        for shape in SHAPES3 + [(300, 7, 6), (70, 300, 6)]:
            for per, neu in (((0, 0, 0), (0,) * 6), ((0, 1, 1), (0,) * 6),
                             ((1, 0, 0), (0,) * 6),
                             ((0, 0, 0), (0, 1, 0, 0, 1, 0))):
                out = np.zeros(shape[::-1], dtype=int)
                replay3(q, *shape, bx, by, npt, cz, per, neu, out=out)
                assert np.all(out == 1), (name, shape, per, neu)


def test_3d_replay_detects_an_unclamped_row_source():
    """The replay itself: with the interior-row path's x sources left
    unclamped, the x = 0 node's +x pull reads column -1, and the replay
    says so."""
    replay3(7, 130, 6, 6, 128, 1, 2, 4)
    with pytest.raises(AssertionError):
        replay3(7, 130, 6, 6, 128, 1, 2, 4, bad_row=True)


def test_3d_replay_detects_an_overrun():
    """The replay itself: with the fast path's x guard one node too wide
    (x0 + tw <= nx instead of nx - 1) the +x pull of the last column leaves
    the lattice, and the replay says so."""
    replay3(7, 128, 6, 6, 64, 2, 1, 4)
    with pytest.raises(AssertionError):
        replay3(7, 128, 6, 6, 64, 2, 1, 4, bad_fast=True)


# ---------------------------------------------------------------------
# 2D two-step kernel: step2_body

def _parse_t2(name):
    m = re.fullmatch(r"(\d+)x(\d+)/t2s?(/r(\d+))?(/nt)?", name)
    return int(m.group(1)), int(m.group(2)), int(m.group(4) or 1)


def replay_t2(q, nx, ny, win, by, rows, px, py, two=True, ring_rows=None,
              shift=0, skip_strip0=False, out=None):
    """Every offset and LDS row step2_body touches; returns the number of
    global accesses checked.  ring_rows: ring size other than the kernel's
    BY + 2 (a planted mistake).  shift: the descriptor's x_shift (a narrow
    first strip); skip_strip0: the blocks of strip 0 exit (the split
    schedule's front strips), and out, if given, receives the count of
    stores per node instead of the every-node-once check."""
    P = nx * ny
    ring = by + 2 if ring_rows is None else ring_rows
    nstrips = (nx + shift + win - 5) // (win - 4)
    nseg = -(-ny // rows)
    nitems = nstrips * nseg
    per_xcd = (nitems + 7) // 8
    assert win % 64 == 0 and win * by <= 1024
    dirs = _dirs2(q)
    seen = np.zeros(nitems, dtype=int)
    written = np.zeros((ny, nx), dtype=int)   # stores of the launch
    checked = 0

    def gcheck(j, gx, gy):
        nonlocal checked
        assert 0 <= gx < nx and 0 <= gy < ny, (gx, gy)
        assert 0 <= j * P + gy * nx + gx < q * P
        checked += 1

    def lrow(r):
        if 0 <= r < ny:
            return r
        return r % ny if py else -1

    for bidx in range(8 * per_xcd):
        item = (bidx & 7) * per_xcd + (bidx >> 3)
        if item >= nitems:
            continue
        seen[item] += 1
        strip, seg = item % nstrips, item // nstrips
        if skip_strip0 and strip == 0:
            continue
        s0 = seg * rows
        s1 = min(s0 + rows, ny)
        base = s0 - 12
        iters = (s1 - s0 + 4 + by - 1) // by
        # ring contents: the lattice row (window row index) in each slot
        l0 = [None] * ring
        l1 = [None] * ring
        for t in range(win):
            x = strip * (win - 4) - 2 + t - shift
            assert -2 - shift <= x <= nx + win   # the window may overhang
        cols = []
        for t in range(win):
            x = strip * (win - 4) - 2 + t - shift
            gx, col = x, 0 <= x < nx
            if not col and px:
                gx, col = x % nx, True
            own_col = 2 <= t < win - 2 and 0 <= x < nx
            cols.append((x, gx, col, own_col))
        # first prefetch
        for ty in range(by):
            gr = lrow(s0 - 2 + ty)
            for t in range(win):
                x, gx, col, _ = cols[t]
                for j in range(q):
                    gcheck(j, gx if col else 0, 0 if gr < 0 else gr)
        pend = []                        # stores waiting for the next pass
        for i in range(iters):
            a = s0 - 2 + i * by
            for ty in range(by):
                slot = a + ty - base
                assert slot >= 0          # the unsigned modulo is the slot
                l0[slot % ring] = a + ty
            for (wx, wy) in pend:
                for j in range(q):
                    gcheck(j, wx, wy)
            pend = []
            if i + 1 < iters:
                for ty in range(by):
                    gr = lrow(a + by + ty)
                    for t in range(win):
                        x, gx, col, _ = cols[t]
                        for j in range(q):
                            gcheck(j, gx if col else 0, 0 if gr < 0 else gr)
            # step n + 1 (barrier before: the ring holds rows a .. a+by-1)
            new_l1 = {}
            for ty in range(by):
                rb = a - 1 + ty
                gb = lrow(rb)
                for t in range(win):
                    x, gx, col, own_col = cols[t]
                    if two:
                        if not (1 <= t < win - 1 and col and gb >= 0 and
                                s0 - 1 <= rb <= s1):
                            continue
                    elif not (own_col and s0 <= rb < s1):
                        continue
                    for (ex, ey) in dirs:
                        rr = rb - ey
                        assert 0 <= t - ex < win
                        # a source row outside a non-periodic lattice is
                        # read from LDS and masked: only real rows must be
                        # the ones wanted
                        if lrow(rr) >= 0:
                            assert l0[(rr - base) % ring] == rr, (rr, l0)
                    if two:
                        new_l1[(rb - base) % ring] = rb
                    else:
                        pend.append((x, rb))
                        written[rb, x] += 1
            for k, v in new_l1.items():
                l1[k] = v
            # step n + 2 (after the second barrier)
            if two:
                for ty in range(by):
                    c = a - 2 + ty
                    for t in range(win):
                        x, gx, col, own_col = cols[t]
                        if not (own_col and s0 <= c < s1):
                            continue
                        for (ex, ey) in dirs:
                            rr = c - ey
                            assert 0 <= t - ex < win
                            if lrow(rr) >= 0:
                                assert l1[(rr - base) % ring] == rr, (rr, l1)
                        pend.append((x, c))
                        written[c, x] += 1
        for (wx, wy) in pend:
            for j in range(q):
                gcheck(j, wx, wy)
    assert np.all(seen == 1)
    if out is not None:
        out += written
    else:
        assert np.all(written == 1)      # every node stored exactly once
    return checked


# the split two-step schedule of the batched form: front strips of
# FRONT_COLUMNS columns (the whole lattice if at most 64 columns wide),
# both steps by batch_front_kernel (front2_body) in segments of
# FRONT_ROWS[storage bytes] rows (kFrontColumns of host_util.hpp,
# front_rows of kernels.hpp)
FRONT_COLUMNS = 60
FRONT_ROWS = {4: 10, 8: 6}


def front_cols(nx):
    return nx if nx <= 64 else FRONT_COLUMNS


def replay_front(q, nx, ny, py, rows, x_lim, x_cnt):
    """front2_body over every segment: returns the count of step n + 2
    stores and of statistics contributions per node at each step; checks
    every global load and store inside the lattice, every LDS index inside
    the buffer, and that each LDS value a step n + 2 update pulls (and is
    not masked) was computed at step n + 1 in the same block."""
    W, RR = 64, rows + 2
    assert (RR * W) % 256 == 0 and x_lim <= W and x_cnt <= x_lim <= nx
    dirs = _dirs2(q)
    stored = np.zeros((ny, nx), dtype=int)
    counted1 = np.zeros((ny, nx), dtype=int)
    for seg in range(-(-ny // rows)):
        y0, y1 = seg * rows, min(seg * rows + rows, ny)
        have = {}
        for n in range(RR * W):
            r, x = n >> 6, n & (W - 1)
            yy = y0 - 1 + r
            gy = yy if 0 <= yy < ny else (yy % ny if py else -1)
            if x < x_lim and gy >= 0 and yy <= y1:
                assert 0 <= x < nx and 0 <= gy < ny     # load_node
                assert 0 <= r < RR
                have[(r, x)] = gy
                if y0 <= yy < y1 and x < x_cnt:
                    counted1[gy, x] += 1
        for n in range(rows * W):
            r, x = n >> 6, n & (W - 1)
            y = y0 + r
            if not (x < x_cnt and y < y1):
                continue
            for (ex, ey) in dirs:
                sx, sy = x - ex, y - ey
                inside = 0 <= sx < nx and (0 <= sy < ny or py)
                lr, lc = r + 1 - ey, (x - ex) & (W - 1)
                assert 0 <= lr < RR and 0 <= lc < W
                if inside:
                    assert have.get((lr, lc)) == sy % ny, (x, y, ex, ey)
            assert 0 <= x < nx and 0 <= y < ny             # store
            stored[y, x] += 1
    return stored, counted1


@pytest.mark.parametrize("q", [5, 9])
def test_split_schedule_updates_every_node_once(names, q):
    """The front kernel plus the shifted two-step strips (the quiet and
    full passes skip strip 0) store every node of step n + 2 exactly once
    and count it once per step."""
    t2s = [n for n in names[q] if "/t2s" in n]
    assert t2s
    for name in t2s:
        win, by, rows = _parse_t2(name)
        for (nx, ny) in SHAPES2 + [(59, 7), (60, 9), (61, 5), (62, 66),
                                   (64, 30), (65, 14), (124, 13),
                                   (183, 10), (184, 3), (185, 33)]:
            wf = front_cols(nx)
            shift = win - 4 - wf
            for py in (False, True):
                for sb in (4, 8):
                    s2, c1 = replay_front(q, nx, ny, py, FRONT_ROWS[sb],
                                          min(wf + 1, nx), min(wf, nx))
                    assert np.all(c1[:, :wf] == 1) and not c1[:, wf:].any()
                out = np.zeros((ny, nx), dtype=int)
                replay_t2(q, nx, ny, win, by, rows, False, py, True,
                          shift=shift, skip_strip0=True, out=out)
                assert not out[:, :wf].any()
                assert np.all(out + s2 == 1), (name, nx, ny)
                # odd single steps: the full kernel over every strip
                replay_t2(q, nx, ny, win, by, rows, False, py, False,
                          shift=shift)


def test_front_replay_detects_a_short_halo():
    """The replay itself: without the halo row above, a step n + 2 pull
    would read a value not computed in the block."""
    replay_front(5, 40, 20, False, 14, 21, 20)
    with pytest.raises(AssertionError):
        replay_front_short(5, 40, 20, False, 14, 21, 20)


def replay_front_short(q, nx, ny, py, rows, x_lim, x_cnt):
    """replay_front with step n + 1 computed for the segment's rows and the
    row below only (a planted mistake)"""
    W = 64
    dirs = _dirs2(q)
    for seg in range(-(-ny // rows)):
        y0, y1 = seg * rows, min(seg * rows + rows, ny)
        have = {}
        for r in range(rows + 1):
            for x in range(min(x_lim, W)):
                yy = y0 - 1 + r
                if 0 <= yy < ny:
                    have[(r, x)] = yy
        for r in range(y1 - y0):
            for x in range(x_cnt):
                y = y0 + r
                for (ex, ey) in dirs:
                    sx, sy = x - ex, y - ey
                    if 0 <= sx < nx and 0 <= sy < ny:
                        assert have.get((r + 1 - ey, (x - ex) & 63)) == sy


SHAPES2 = [(3, 3), (5, 4), (3, 40), (124, 5), (125, 6), (126, 3), (252, 9),
           (253, 17), (130, 70)]


@pytest.mark.parametrize("q", [5, 9])
def test_two_step_kernel_offsets_inside_planes(names, q):
    t2 = [n for n in names[q] if "/t2" in n]
    assert t2
    for name in t2:
        win, by, rows = _parse_t2(name)
        for (nx, ny) in SHAPES2:
            for px, py in ((False, False), (True, True), (False, True)):
                for two in (True, False):
                    assert replay_t2(q, nx, ny, win, by, rows, px, py,
                                     two) > 0


def test_two_step_replay_detects_a_short_ring():
    """The replay itself: a ring of BY + 1 rows loses a row the second step
    still needs."""
    replay_t2(5, 40, 20, 128, 2, 16, False, False)
    with pytest.raises(AssertionError):
        replay_t2(5, 40, 20, 128, 2, 16, False, False, ring_rows=3)
