"""A CPU model of the row codes of the restricted system B on the five- and
nine-point stencils (the grid-order form of B = A[Omega, Omega], Algorithm 1
step 4): each row stores two 16-bit offsets to the number of members before
the cells straight below and above it plus the slots' presence bits, and
only the values of its upper slots; a lower coupling is the neighbour's
entry in the mirrored slot.

The model encodes as the gather does and decodes as the kernels' row loader
does, on random domains of small grids (one-row, one-column and one-cell
grids included), and checks that
  * every decoded column is the member's local number, and absent slots
    decode to no member;
  * the mirrored slot of each lower member decodes back to the row;
  * the value read through the mirrored slot equals the row's own coupling
    bit for bit, on half-stored stencil coefficients.
Host logic only: no GPU, no library call."""
import numpy as np
import pytest

# slot offsets (dx, dy) in ascending column order
SLOTS = {
    5: [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)],
    9: [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)],
}


def half_stencil(nx, ny, nb, rng):
    """Coefficients of a half-stored stencil: per cell C and its couplings
    to the east, north (and north-east, north-west on nine points)."""
    n = nx * ny
    co = {k: rng.standard_normal(n) for k in ("C", "E", "N", "NE", "NW")}
    return co


def coupling(co, nx, ny, i, dx, dy):
    """a(i, j) for j = i + (dx, dy), read as the stencil stores it: a lower
    or left neighbour's coupling is that neighbour's forward entry."""
    x, y = i % nx, i // nx
    if (dx, dy) == (0, 0):
        return co["C"][i]
    j = i + dy * nx + dx
    table = {(1, 0): ("E", i), (-1, 0): ("E", j), (0, 1): ("N", i), (0, -1): ("N", j),
             (1, 1): ("NE", i), (-1, -1): ("NE", j), (-1, 1): ("NW", i), (1, -1): ("NW", j)}
    name, at = table[(dx, dy)]
    assert 0 <= x + dx < nx and 0 <= y + dy < ny
    return co[name][at]


def encode(nx, ny, nb, member, co):
    """Row codes, presence bits, stored upper values and the full rows of B
    (for the check) of the domain `member` (bool per cell), as the gather
    builds them."""
    idx = np.flatnonzero(member)
    inv = -np.ones(nx * ny, dtype=np.int64)
    inv[idx] = np.arange(idx.size)
    mid = nb // 2
    K = idx.size
    off = np.zeros(K, dtype=np.uint32)
    mask = np.zeros(K, dtype=np.uint8)
    upper = np.zeros((mid + 1, K))
    cols = -np.ones((K, nb), dtype=np.int64)
    full = np.zeros((K, nb))
    for k, i in enumerate(idx):
        x, y = i % nx, i // nx
        cs = [-1] * nb
        a = [0.0] * nb
        for sl, (dx, dy) in enumerate(SLOTS[nb]):
            if 0 <= x + dx < nx and 0 <= y + dy < ny:
                j = i + dy * nx + dx
                if inv[j] >= 0:
                    cs[sl] = int(inv[j])
                    a[sl] = coupling(co, nx, ny, i, dx, dy)
        m = 0
        for sl in range(nb):
            if sl != mid and cs[sl] >= 0:
                m |= 1 << (sl if sl < mid else sl - 1)
        if nb == 9:
            ps = cs[0] + 1 if cs[0] >= 0 else cs[1] if cs[1] >= 0 else cs[2] if cs[2] >= 0 else k
            pn = cs[6] + 1 if cs[6] >= 0 else cs[7] if cs[7] >= 0 else cs[8] if cs[8] >= 0 else k
        else:
            ps = cs[0] if cs[0] >= 0 else k
            pn = cs[4] if cs[4] >= 0 else k
        assert -32768 <= ps - k <= 32767 and -32768 <= pn - k <= 32767
        off[k] = ((ps - k) & 0xFFFF) | (((pn - k) & 0xFFFF) << 16)
        mask[k] = m
        upper[:, k] = a[mid:]
        cols[k] = cs
        full[k] = a
    return off, mask, upper, cols, full


def i16(v):
    v = int(v) & 0xFFFF
    return v - 0x10000 if v >= 0x8000 else v


def decode(nb, off, mask, k):
    """The columns of row k as the row loader derives them (-1: absent)."""
    mid = nb // 2
    so, no = k + i16(off[k]), k + i16(off[k] >> 16)
    m = int(mask[k])
    has = lambda sl: (m >> (sl if sl < mid else sl - 1)) & 1
    if nb == 9:
        c = [so - 1 if has(0) else -1, so if has(1) else -1, so + has(1) if has(2) else -1,
             k - 1 if has(3) else -1, k, k + 1 if has(5) else -1,
             no - 1 if has(6) else -1, no if has(7) else -1, no + has(7) if has(8) else -1]
    else:
        c = [so if has(0) else -1, k - 1 if has(1) else -1, k, k + 1 if has(3) else -1,
             no if has(4) else -1]
    return c


def load_values(nb, upper, c, k):
    """B's row k as the row loader reads it: its upper slots, and each lower
    slot from the member's mirrored slot."""
    mid = nb // 2
    vals = [0.0] * nb
    for sl in range(mid, nb):
        vals[sl] = upper[sl - mid, k]
    for sl in range(mid):
        j = c[sl]
        vals[sl] = upper[nb - 1 - sl - mid, j] if j >= 0 else 0.0
    return vals


GRIDS = [(1, 1), (1, 7), (7, 1), (2, 2), (5, 4), (13, 9), (31, 6)]


@pytest.mark.parametrize("nb", [5, 9])
@pytest.mark.parametrize("nx,ny", GRIDS)
@pytest.mark.parametrize("density", [0.0, 0.3, 0.7, 1.0])
def test_row_codes_decode_to_the_members(nb, nx, ny, density):
    rng = np.random.default_rng(1000 * nx + 10 * ny + int(10 * density) + nb)
    for trial in range(3):
        member = rng.random(nx * ny) < density
        co = half_stencil(nx, ny, nb, rng)
        off, mask, upper, cols, full = encode(nx, ny, nb, member, co)
        K = cols.shape[0]
        mid = nb // 2
        for k in range(K):
            c = decode(nb, off, mask, k)
            assert c == cols[k].tolist(), (nb, nx, ny, k)
            # every lower member's mirrored slot points back at row k
            for sl in range(mid):
                j = c[sl]
                if j >= 0:
                    assert decode(nb, off, mask, j)[nb - 1 - sl] == k
            # and its value there is the row's own coupling, to the bit
            vals = load_values(nb, upper, c, k)
            assert np.array_equal(np.array(vals), full[k])


def test_the_model_sees_a_wrong_mirror():
    """A loader that took the lower values from the wrong slot (the member's
    own slot s instead of the mirrored one) is caught by the value check."""
    nb, nx, ny = 9, 6, 5
    rng = np.random.default_rng(7)
    member = np.ones(nx * ny, dtype=bool)
    co = half_stencil(nx, ny, nb, rng)
    off, mask, upper, cols, full = encode(nx, ny, nb, member, co)
    mid = nb // 2
    wrong = 0
    for k in range(cols.shape[0]):
        c = decode(nb, off, mask, k)
        for sl in range(mid):
            j = c[sl]
            if j >= 0 and upper[(mid + 1 + sl) % (mid + 1), j] != full[k][sl]:
                wrong += 1
    assert wrong > 0
