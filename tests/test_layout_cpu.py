"""Host-side checks of the step's memory accesses (no GPU).

The step kernel loads, for every group of VEC nodes and every direction, one
vector of VEC elements starting at x0 - dx in the source run (pull form, or
either phase of in-place streaming), then patches the x-periodic wraps.  These
tests restate that index arithmetic (row blocks, half-way bounce-back rows,
the in-place slot reversal) and check, against the library's own buffer size,
that every such vector lies inside the buffer, and that a real node's lane
holds its true source element except where the kernel patches it (the row's
first node for dx = +1, its last for dx = -1).
"""
import pytest

EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
EB = {"f64": 8, "f32": 4, "f16": 2}
VECS = {"f64": (2, 1), "f32": (4, 2, 1), "f16": (8, 4, 2)}


def _pitch(nx, eb):
    # Runs padded to 8 elements, or, above 64 nodes, to 128-byte lines.
    a = max(8, 128 // eb) if nx > 64 else 8
    return (nx + a - 1) // a * a


def _row_shift(nx, ny, eb):
    # Rows per block R = 2^k: runs of one direction in a block reach 16 KB,
    # or R reaches the height.
    run, sh = _pitch(nx, eb) * eb, 0
    while (run << sh) < 16384 and (2 << sh) <= ny:
        sh += 1
    return sh


def _check(nx, ny, storage, vec, bc, inplace, buffer_bytes):
    eb = EB[storage]
    P, rs = _pitch(nx, eb), _row_shift(nx, ny, eb)
    R = 1 << rs
    rows = (ny + R - 1) // R * R
    total = buffer_bytes // eb
    assert buffer_bytes - 9 * rows * P * eb == 64, "row blocks or tail guard disagree with the library"
    dstride, bstride = R * P, 9 * R * P

    def row_base(y):
        return (y >> rs) * bstride + (y & (R - 1)) * P

    def source_of(i, y):
        d, r, dx = i, y - EY[i], EX[i]
        if r < 0 or r >= ny:
            if bc:
                d, r, dx = OPP[i], y, 0
            else:
                r = r + ny if r < 0 else r - ny
        return d, r, dx

    for phase in ((0, 1) if inplace else (0,)):
        for y in range(ny):
            for x0 in range(0, P, vec):
                for i in range(9):
                    if inplace and phase == 0:
                        d, r, dx = i, y, 0
                    else:
                        d, r, dx = source_of(i, y)
                        if inplace:
                            d = OPP[d]
                    base = d * dstride + row_base(r)
                    lo = base + x0 - dx
                    assert 0 <= lo and lo + vec <= total, (nx, ny, storage, vec, bc, inplace, phase, y, x0, i)
                    for k in range(vec):
                        x = x0 + k
                        if x >= nx:
                            continue  # padding lane: never stored as loaded
                        if lo + k != base + (x - dx) % nx:
                            assert (x == 0 and dx == 1) or (x == nx - 1 and dx == -1), \
                                (nx, ny, storage, vec, phase, y, x0, i, k)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_step_vector_loads_stay_in_the_buffer(storage):
    from paper_1705_11092_amd import clbm
    widths = list(range(1, 34)) + [63, 64, 65, 127, 1030]
    for nx in widths:
        for ny in (1, 2, 3, 9, 23):
            nbytes = clbm.buffer_bytes(nx, ny, storage)
            for vec in VECS[storage]:
                for bc in (0, 1):
                    for inplace in (False, True):
                        _check(nx, ny, storage, vec, bc, inplace, nbytes)
