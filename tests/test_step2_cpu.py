"""Host-side checks of the two-step kernel's index maps (no GPU).

The two-step kernel walks its tiles (64 x 16 or 32 x 32 nodes with 4 per
thread in phase B, or, for FP64, 64 x 8 with 2) in vertical strips of up to
512 nodes across, collides step n + 1 on each tile's region (the tile's
nodes inside the lattice and a one-node halo: at most 66 x 18, 34 x 34 or
66 x 10 nodes, less for a tile at the lattice's right or lower edge) and
writes slot i of a region node straight into the LDS entry of the tile node
that pulls it (Eq. 10), or, next to a bounce-back wall, the node's own
reversed slot into the entry its absent neighbour would fill.  These tests
restate that arithmetic and check that the walk visits every tile once,
that every LDS entry phase B reads is written exactly once, by the source
the pull with half-way bounce-back names, that the region row of a region
node comes out exact from its float product, that the multiply-and-shift
divisions of the walk equal integer division (restated, and the kernels'
own code built for the host from tests/host_walk.hip), and that
phase B's stores cover each row and its padding up to the next multiple of
4 exactly once.
"""
import ctypes
import os
import random
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
STRIP_NODES = 512
SHAPES = [(64, 16), (32, 32), (64, 8), (32, 16)]
TW, TH = 64, 16


def strip_tile(t, tiles_x, tiles_y, sw):
    full = tiles_x // sw
    in_full = full * sw * tiles_y
    if t < in_full:
        st, i = divmod(t, sw * tiles_y)
        ty, c = divmod(i, sw)
        return st * sw + c, ty
    w = tiles_x - full * sw
    ty, c = divmod(t - in_full, w)
    return full * sw + c, ty


@pytest.mark.parametrize("tw,th", SHAPES)
@pytest.mark.parametrize("nx,ny", [(1, 1), (64, 16), (65, 17), (300, 70), (1030, 9), (4096, 64),
                                   (520, 200), (64 * 13, 16 * 5)])
def test_strip_walk_visits_every_tile_once(nx, ny, tw, th):
    tiles_x, tiles_y = (nx + tw - 1) // tw, (ny + th - 1) // th
    sw = min(tiles_x, STRIP_NODES // tw)
    seen = [strip_tile(t, tiles_x, tiles_y, sw) for t in range(tiles_x * tiles_y)]
    assert sorted(seen) == sorted((x, y) for x in range(tiles_x) for y in range(tiles_y))
    # Within a full strip the tile above is sw tiles earlier.
    if tiles_y > 1 and tiles_x >= sw:
        assert seen[sw] == (seen[0][0], seen[0][1] + 1)


def fast_div(d):
    """The kernel's divisor d >= 1 as (m, sh): m = ceil(2^(31+s) / d) with
    2^(s-1) < d <= 2^s, sh = 31 + s."""
    s = 0
    while s < 31 and (1 << s) < d:
        s += 1
    return -(-(1 << (31 + s)) // d), 31 + s


def div_by(n, f):
    m, sh = f
    assert 0 <= m < 1 << 32 and 0 <= n < 1 << 31
    return ((n * m) & ((1 << 64) - 1)) >> sh


def test_fast_division_is_exact_below_2_31():
    rng = random.Random(7)
    divisors = list(range(1, 3000)) + [(1 << k) + o for k in range(12, 31) for o in (-1, 0, 1)]
    divisors += [rng.randrange(1, 1 << 31) for _ in range(300)] + [(1 << 31) - 1]
    for d in divisors:
        f = fast_div(d)
        ns = {0, 1, d - 1, d, d + 1, 2 * d - 1, (1 << 31) - 1, (1 << 31) - 1 - d}
        ns |= {rng.randrange(0, 1 << 31) for _ in range(20)}
        ns |= {q * d + r for q in (1, 7, (1 << 31) // d - 1) for r in (0, d - 1)}
        for n in ns:
            if 0 <= n < 1 << 31:
                assert div_by(n, f) == n // d, (d, n)


@pytest.fixture(scope="module")
def walk_lib(tmp_path_factory):
    """tests/host_walk.hip: the kernels' strip walk and divisions built for the host."""
    out = tmp_path_factory.mktemp("host_walk") / "libhost_walk.so"
    subprocess.check_call([HIPCC, "--offload-host-only", "-O2", "-std=c++17", "-fPIC", "-shared",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1705_11092_amd", "csrc"),
                           "-o", str(out), os.path.join(ROOT, "tests", "host_walk.hip")],
                          stderr=subprocess.DEVNULL)
    h = ctypes.CDLL(str(out))
    h.host_div_by.argtypes = [ctypes.c_uint32, ctypes.c_int]
    h.host_div_by.restype = ctypes.c_int
    ip = ctypes.POINTER(ctypes.c_int)
    h.host_strip_walk.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, ip, ip]
    return h


def test_kernel_division_is_exact_below_2_31(walk_lib):
    """The kernels' own multiply-and-shift division, compiled for the host."""
    rng = random.Random(11)
    divisors = list(range(1, 600)) + [(1 << k) + o for k in range(10, 31) for o in (-1, 0, 1)]
    divisors += [rng.randrange(1, 1 << 31) for _ in range(100)] + [(1 << 31) - 1]
    for d in divisors:
        ns = {0, 1, d - 1, d, d + 1, (1 << 31) - 1, (1 << 31) - 1 - d}
        ns |= {rng.randrange(0, 1 << 31) for _ in range(10)}
        ns |= {q * d + r for q in (1, 3, (1 << 31) // d - 1) for r in (0, d - 1)}
        for n in ns:
            if 0 <= n < 1 << 31:
                assert walk_lib.host_div_by(d, n) == n // d, (d, n)


@pytest.mark.parametrize("tw,th", SHAPES)
@pytest.mark.parametrize("nx,ny", [(1, 1), (65, 17), (300, 70), (1030, 9), (4096, 4096), (520, 200),
                                   (32768, 32768)])
def test_kernel_strip_walk_names_the_strip_walk_tile(walk_lib, nx, ny, tw, th):
    """The kernels' prepared walk, compiled for the host, against strip_tile."""
    tiles_x, tiles_y = (nx + tw - 1) // tw, (ny + th - 1) // th
    sw = min(tiles_x, STRIP_NODES // tw)
    n = tiles_x * tiles_y
    full = tiles_x // sw
    in_full = full * sw * tiles_y
    ts = range(n) if n <= 20000 else sorted(t for t in {0, n - 1, in_full - 1, in_full} | set(range(0, n, 997)) if 0 <= t < n)
    t = np.ascontiguousarray(np.array(list(ts), dtype=np.int32))
    tx = np.zeros_like(t)
    ty = np.zeros_like(t)
    ip = ctypes.POINTER(ctypes.c_int)
    walk_lib.host_strip_walk(tiles_x, tiles_y, sw, t.ctypes.data_as(ip), len(t), tx.ctypes.data_as(ip),
                             ty.ctypes.data_as(ip))
    for k in range(len(t)):
        assert (int(tx[k]), int(ty[k])) == strip_tile(int(t[k]), tiles_x, tiles_y, sw), (int(t[k]), nx, ny)


@pytest.mark.parametrize("tw,th", SHAPES)
@pytest.mark.parametrize("nx,ny", [(1, 1), (65, 17), (300, 70), (1030, 9), (4096, 4096), (520, 200),
                                   (32768, 32768)])
def test_strip_walk_with_prepared_divisions(nx, ny, tw, th):
    """The single-lattice walk (divisions by sw * tiles_y, sw and the last
    strip's width prepared on the host) names the same tile as strip_tile."""
    tiles_x, tiles_y = (nx + tw - 1) // tw, (ny + th - 1) // th
    sw = min(tiles_x, STRIP_NODES // tw)
    full = tiles_x // sw
    in_full, w = full * sw * tiles_y, tiles_x - full * sw
    by_strip, by_sw, by_w = fast_div(sw * tiles_y), fast_div(sw), fast_div(w if w > 0 else 1)
    n = tiles_x * tiles_y
    ts = range(n) if n <= 20000 else sorted(t for t in {0, n - 1, in_full - 1, in_full} | set(range(0, n, 997)) if 0 <= t < n)
    for t in ts:
        if t < in_full:
            st = div_by(t, by_strip)
            i = t - st * (sw * tiles_y)
            ty = div_by(i, by_sw)
            got = (st * sw + (i - ty * sw), ty)
        else:
            i = t - in_full
            ty = div_by(i, by_w)
            got = (full * sw + (i - ty * w), ty)
        assert got == strip_tile(t, tiles_x, tiles_y, sw), (t, nx, ny)


def _phase_a_writes(nx, ny, bc, x0, y0, tw=TW, th=TH):
    """Map (slot, tile row, tile column) -> (source x, source y, source slot)
    as phase A writes it, from the region's row and column tables."""
    rw = min(tw, nx - x0) + 2
    rh = min(th, ny - y0) + 2
    rows = []
    for rr in range(rh):
        y = y0 - 1 + rr
        beyond = bool(bc) and (y < 0 or y >= ny)
        if beyond:
            y = 0 if y < 0 else ny - 1
        rows.append((y % ny, beyond))
    cols = [(x0 - 1 + cc) % nx for cc in range(rw)]
    writes = {}
    for rr in range(rh):
        y, beyond = rows[rr]
        if beyond:
            continue
        for cc in range(rw):
            x = cols[cc]
            a, b = rr - 1, cc - 1
            for i in range(9):
                ai, bi = a + EY[i], b + EX[i]
                if 0 <= ai < th and 0 <= bi < tw:
                    assert (i, ai, bi) not in writes, "written twice"
                    writes[(i, ai, bi)] = (x, y, i)
            lo, hi = bc and y == 0, bc and y == ny - 1
            if (lo or hi) and 0 <= a < th and 0 <= b < tw:
                for i in range(9):
                    if (EY[i] == 1 and lo) or (EY[i] == -1 and hi):
                        assert (i, a, b) not in writes, "wall entry written twice"
                        writes[(i, a, b)] = (x, y, OPP[i])
    return writes


@pytest.mark.parametrize("tw,th", SHAPES)
@pytest.mark.parametrize("nx,ny,bc", [(300, 70, 1), (300, 70, 0), (65, 17, 1), (33, 1, 1), (70, 2, 1),
                                      (2, 2, 0), (19, 1, 0), (1, 17, 1), (129, 33, 1), (200, 40, 0),
                                      (40, 100, 0), (31, 33, 1)])
def test_lds_entries_hold_the_pulled_values(nx, ny, bc, tw, th):
    tiles_x, tiles_y = (nx + tw - 1) // tw, (ny + th - 1) // th
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            x0, y0 = tx * tw, ty * th
            writes = _phase_a_writes(nx, ny, bc, x0, y0, tw, th)
            for r in range(th):
                y = y0 + r
                if y >= ny:
                    continue
                for c in range(tw):
                    x = x0 + c
                    if x >= nx:
                        continue
                    for i in range(9):
                        ys = y - EY[i]
                        if bc and (ys < 0 or ys >= ny):
                            want = (x, y, OPP[i])  # half-way bounce-back
                        else:
                            want = ((x - EX[i]) % nx, ys % ny, i)
                        assert writes.get((i, r, c)) == want, (nx, ny, bc, tx, ty, r, c, i)


@pytest.mark.parametrize("tw,th", SHAPES)
def test_region_row_from_float_product_is_exact(tw, th):
    # rr = (int)((j + 1/2) * fl(1/rw)) in FP32 for every region size the
    # kernel meets and every index a thread takes (j < 5 * 256).
    import numpy as np
    for rw in range(3, tw + 3):
        inv = np.float32(1.0) / np.float32(rw)
        for rh in range(3, th + 3):
            n = rw * rh
            j = np.arange(min(n, 5 * 256), dtype=np.int64)
            rr = ((j.astype(np.float32) + np.float32(0.5)) * inv).astype(np.int64)
            assert np.array_equal(rr, j // rw), (rw, rh)


@pytest.mark.parametrize("npt,tw", [(4, 64), (4, 32), (2, 64), (2, 32)])
def test_phase_b_stores_cover_each_row_and_its_padding_once(npt, tw):
    # Phase B: the thread with nodes [c, c + npt) of a row stores them when
    # c < nx, with copies of the last real node past nx; with npt = 2 the
    # thread that holds the row's last node also fills the rest of its
    # group of 4 (a second store of 2 at c + 2).
    for nx in range(1, 140):
        written = []
        for x0 in range(0, nx, tw):
            for c in range(0, tw, npt):
                if x0 + c >= nx:
                    continue
                written += range(x0 + c, x0 + c + npt)
                if npt == 2:
                    full = x0 + c + npt <= nx
                    if (full and x0 + c + 2 == nx and nx % 4) or (not full and (x0 + c) % 4 == 0):
                        written += range(x0 + c + 2, x0 + c + 4)
        want = list(range((nx + 3) // 4 * 4))
        assert sorted(written) == want, (npt, nx)


@pytest.mark.parametrize("tw,th", SHAPES)
def test_packed_phase_b_covers_the_tile_once(tw, th):
    # A batch tile at a lattice's right edge with `we` columns in the
    # lattice maps thread t to row t // lpr and group t % lpr (lpr = the
    # groups of npt nodes across `we`), the row from the float product
    # (t + 1/2) * fl(1/lpr); every node of the tile inside the lattice is
    # one thread's, once.
    import numpy as np
    npt = tw * th // 256
    lpr_full = tw // npt
    for we in range(1, tw + 1):
        lpr = (we + npt - 1) // npt
        t = np.arange(256)
        if lpr < lpr_full:
            rb = ((t.astype(np.float32) + np.float32(0.5)) * (np.float32(1.0) / np.float32(lpr))).astype(np.int64)
            assert np.array_equal(rb, t // lpr), (tw, th, we)
        else:
            rb = t // lpr_full
        cb = (t - rb * (lpr if lpr < lpr_full else lpr_full)) * npt
        seen = {}
        for r, c in zip(rb.tolist(), cb.tolist()):
            if r >= th or c >= we:
                continue
            for k in range(npt):
                seen[(r, c + k)] = seen.get((r, c + k), 0) + 1
        want = {(r, x) for r in range(th) for x in range(we)}
        assert want <= set(seen) and all(v == 1 for v in seen.values()), (tw, th, we)


def _own_node_writes(nx, ny, bc, x0, y0, tw, th, npt, pack):
    """The 16-bit storage types' pair step: thread t owns its phase-B nodes
    in phase A too (slot 0 stays in its registers), and the region's ring
    (the nodes around the tile's part in the lattice) is collided one node
    per thread.  Map (slot 1..8, tile row, tile column) -> source, as those
    writes fill it, checking each entry is written once and in bounds, and
    that every tile node in the lattice is one thread's."""
    import numpy as np
    we, he = min(tw, nx - x0), min(th, ny - y0)
    lpr_full = tw // npt
    writes, owners = {}, {}

    def put(key, val):
        assert 1 <= key[0] <= 8 and 0 <= key[1] < th and 0 <= key[2] < tw
        assert key not in writes, ("written twice", key)
        writes[key] = val

    def to_lds(a, b, x, y):
        for i in range(1, 9):
            ai, bi = a + EY[i], b + EX[i]
            if 0 <= ai < th and 0 <= bi < tw:
                put((i, ai, bi), (x, y, i))
        if bc:
            lo, hi = y == 0, y == ny - 1
            if (lo or hi) and 0 <= a < th and 0 <= b < tw:
                for i in range(1, 9):
                    if (EY[i] == 1 and lo) or (EY[i] == -1 and hi):
                        put((i, a, b), (x, y, OPP[i]))

    for t in range(256):
        rb, cb = t // lpr_full, (t % lpr_full) * npt
        if pack:
            lpr = (we + npt - 1) // npt
            if lpr < lpr_full:
                rb = int((np.float32(t) + np.float32(0.5)) * (np.float32(1.0) / np.float32(lpr)))
                cb = (t - rb * lpr) * npt
        if not (rb < he and cb < we):
            continue
        for k in range(npt):
            if cb + k < we:
                assert (rb, cb + k) not in owners
                owners[(rb, cb + k)] = t
                to_lds(rb, cb + k, x0 + cb + k, y0 + rb)
    rw, rh = we + 2, he + 2
    nring = 2 * rw + 2 * he
    assert nring <= 256
    for k in range(nring):
        if k < 2 * rw:
            rr, cc = (0, k) if k < rw else (rh - 1, k - rw)
        else:
            j = k - 2 * rw
            rr, cc = (1 + j, 0) if j < he else (1 + j - he, rw - 1)
        y = y0 - 1 + rr
        if bc and (y < 0 or y >= ny):
            continue
        to_lds(rr - 1, cc - 1, (x0 - 1 + cc) % nx, y % ny)
    assert set(owners) == {(r, c) for r in range(he) for c in range(we)}
    return writes


@pytest.mark.parametrize("tw,th", SHAPES)
@pytest.mark.parametrize("pack", [False, True])
@pytest.mark.parametrize("nx,ny,bc", [(300, 70, 1), (300, 70, 0), (65, 17, 1), (33, 1, 1), (70, 2, 1),
                                      (2, 2, 0), (19, 1, 0), (1, 17, 1), (129, 33, 1), (200, 40, 0),
                                      (40, 100, 0), (31, 33, 1), (1, 1, 0), (1, 1, 1), (4, 3, 1)])
def test_own_node_pair_step_fills_the_pulled_values(nx, ny, bc, tw, th, pack):
    npt = tw * th // 256
    tiles_x, tiles_y = (nx + tw - 1) // tw, (ny + th - 1) // th
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            x0, y0 = tx * tw, ty * th
            writes = _own_node_writes(nx, ny, bc, x0, y0, tw, th, npt, pack)
            for r in range(min(th, ny - y0)):
                for c in range(min(tw, nx - x0)):
                    x, y = x0 + c, y0 + r
                    for i in range(1, 9):
                        ys = y - EY[i]
                        if bc and (ys < 0 or ys >= ny):
                            want = (x, y, OPP[i])
                        else:
                            want = ((x - EX[i]) % nx, ys % ny, i)
                        assert writes.get((i, r, c)) == want, (nx, ny, bc, tx, ty, r, c, i)
