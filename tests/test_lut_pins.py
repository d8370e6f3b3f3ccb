"""Pins of the library's lower-star lookup table (paper Sec. 3.2-3.3) against the oracle.

The table classifies the cells of each lower star L(v) by reducing L(v) on its own.  Its
claim is that every pair it forms inside L(v) is a pair of the global reduction, and that the
cells it leaves unpaired (KEEP edges and squares, ROOT top cells, local minima) are paired
outside L(v).  These tests read entries through the C ABI (ph_lut_entry, no GPU) and check
both claims cell by cell against the oracle's full pairing (all dimensions, zero-persistence
pairs kept), which knows nothing of lower stars or tables.  Also pinned: the number of
distinct configurations after the collapse rule of Sec. 3.3 (47 in 2D, 15935 in 3D).
"""
import itertools

import numpy as np
import pytest

import oracle
import synthetic as S

fc = pytest.importorskip("paper_2606_04801_amd")
try:
    fc.lib()
except (ImportError, OSError) as e:  # library not built: the build check reports it
    pytest.skip("library not built: %s" % e, allow_module_level=True)

# local offsets (dz, dy, dx) numbered by dimension, then lexicographically (code 0 = vertex)
CODES = [(0, 0, 0)] + sorted((o for o in itertools.product((-1, 0, 1), repeat=3) if any(o)),
                             key=lambda o: (sum(1 for t in o if t), o))
EDGE3 = CODES[1:7]
SQ3 = CODES[7:19]
# 2D mask bit order: up, left, right, down, up-left, up-right, down-left, down-right
NB2 = [(-1, 0), (0, -1), (0, 1), (1, 0), (-1, -1), (-1, 1), (1, -1), (1, 1)]
EDGE2 = NB2[:4]


def test_config_counts():
    assert fc.lut_config_count(2) == 47
    assert fc.lut_config_count(3) == 15935


def test_entry_rejects_bad_masks():
    with pytest.raises(fc.PHError):
        fc.lut_entry(2, 256)
    with pytest.raises(fc.PHError):
        fc.lut_entry(3, 1 << 26)
    with pytest.raises(fc.PHError):
        fc.lut_entry(4, 0)


class Pairing:
    """Full oracle pairing of one image with cell geometry helpers (doubled grid)."""

    def __init__(self, img):
        self.img = img
        self.shape3 = (1,) + img.shape if img.ndim == 2 else img.shape
        D, H, W = self.shape3
        self.G = (2 * D - 1, 2 * H - 1, 2 * W - 1)
        pairs = oracle.diagram(img, dims=tuple(range(img.ndim)), method=oracle.FULL, keep_zero=True)
        self.death_of, self.birth_of, self.lsv = {}, {}, {}
        for p in pairs:
            b, d = int(p["birth_cell"]), int(p["death_cell"])
            self.lsv[b] = int(p["birth_vertex"])
            if d >= 0:
                self.death_of[b] = d
                self.birth_of[d] = b
                self.lsv[d] = int(p["death_vertex"])
        f = img.reshape(-1)
        self.f = f

    def cell(self, v, off):
        D, H, W = self.shape3
        z, r = divmod(v, H * W)
        y, x = divmod(r, W)
        Z, Y, X = 2 * z + off[0], 2 * y + off[1], 2 * x + off[2]
        if not (0 <= Z < self.G[0] and 0 <= Y < self.G[1] and 0 <= X < self.G[2]):
            return None
        return (Z * self.G[1] + Y) * self.G[2] + X

    def coords(self, c):
        Z, r = divmod(c, self.G[1] * self.G[2])
        Y, X = divmod(r, self.G[2])
        return Z, Y, X

    def before(self, a, b):
        """vertex a precedes vertex b in the refined order (value, then pixel index)."""
        fa, fb = float(self.f[a]), float(self.f[b])
        return fa < fb or (fa == fb and a < b)

    def nbr(self, v, d):
        D, H, W = self.shape3
        z, r = divmod(v, H * W)
        y, x = divmod(r, W)
        zz, yy, xx = z + d[0], y + d[1], x + d[2]
        if 0 <= zz < D and 0 <= yy < H and 0 <= xx < W:
            return (zz * H + yy) * W + xx
        return None

    def paired_inside(self, v, c):
        """c is paired (either way) with a cell whose last vertex is v."""
        o = self.death_of.get(c, self.birth_of.get(c))
        return o is not None and self.lsv.get(o) == v


def other_cofacet_octant(P, v, facet, top):
    """Octant (relative to v) of the cofacet of `facet` other than `top`."""
    Fz, Fy, Fx = P.coords(facet)
    Tz, Ty, Tx = P.coords(top)
    Oz, Oy, Ox = 2 * Fz - Tz, 2 * Fy - Ty, 2 * Fx - Tx      # reflect top across the facet
    D, H, W = P.shape3
    z, r = divmod(v, H * W)
    y, x = divmod(r, W)
    return (Oz - 2 * z, Oy - 2 * y, Ox - 2 * x)


def check_2d(img):
    P = Pairing(img)
    H, W = img.shape
    for v in range(H * W):
        mask = 0
        for b, (dy, dx) in enumerate(NB2):
            n = P.nbr(v, (0, dy, dx))
            if n is not None and P.before(n, v):
                mask |= 1 << b
        e = fc.lut_entry(2, mask)
        direct, keep, present, root = e & 7, (e >> 3) & 15, (e >> 7) & 15, (e >> 11) & 15
        vc = P.cell(v, (0, 0, 0))
        edges = mask & 15
        assert direct == 7 or (edges >> direct) & 1, (v, mask, "direct edge not in L(v)")
        assert (direct == 7) == (edges == 0), (v, mask, "minimum iff no lower edge")
        assert keep & ~edges == 0 and (direct == 7 or not (keep >> direct) & 1), (v, mask, "keep")
        assert root & ~present == 0, (v, mask, "root")
        if direct == 7:                                    # local minimum: killed outside L(v)
            assert not P.paired_inside(v, vc), (v, mask)
        else:
            ec = P.cell(v, (0,) + EDGE2[direct])
            assert P.death_of.get(vc) == ec, (v, mask, "direct")
        for i, (dy, dx) in enumerate(EDGE2):
            if not (mask >> i) & 1:
                continue
            ec = P.cell(v, (0, dy, dx))
            assert P.lsv[ec] == v
            if i == direct:
                continue
            if (keep >> i) & 1:
                assert not P.paired_inside(v, ec), (v, mask, i, "keep edge paired inside")
            else:                                          # pruned: killed by a square of L(v)
                sq = P.death_of.get(ec)
                assert sq is not None and P.lsv[sq] == v, (v, mask, i, "pruned edge")
        for q in range(4):
            off = (0, 1 if q >> 1 else -1, 1 if q & 1 else -1)
            sc = P.cell(v, off)
            inside = sc is not None and P.lsv[sc] == v
            assert bool((present >> q) & 1) == inside, (v, mask, q, "square presence")
            if not inside:
                continue
            killed = P.birth_of[sc]                        # squares are never positive (H2 = 0)
            if (root >> q) & 1:
                assert P.lsv[killed] != v, (v, mask, q, "root square paired inside")
            else:
                assert P.lsv[killed] == v, (v, mask, q, "local square paired outside")
                t = (e >> (15 + 2 * q)) & 3
                o = other_cofacet_octant(P, v, killed, sc)
                assert o == (0, 1 if t >> 1 else -1, 1 if t & 1 else -1), (v, mask, q, "link")


def check_3d(img):
    P = Pairing(img)
    D, H, W = img.shape
    for v in range(D * H * W):
        mask = 0
        for k, off in enumerate(CODES[1:]):
            n = P.nbr(v, off)
            if n is not None and P.before(n, v):
                mask |= 1 << k
        e = fc.lut_entry(3, mask)
        direct, keep_e, keep_s = e & 7, (e >> 3) & 63, (e >> 9) & 0xFFF
        root, present_c = (e >> 21) & 0xFF, (e >> 53) & 0xFF
        vc = P.cell(v, (0, 0, 0))
        edges = mask & 63
        assert direct == 7 or (edges >> direct) & 1, (v, mask, "direct edge not in L(v)")
        assert (direct == 7) == (edges == 0), (v, mask, "minimum iff no lower edge")
        assert keep_e & ~edges == 0 and (direct == 7 or not (keep_e >> direct) & 1), (v, mask, "keep")
        assert root & ~present_c == 0, (v, mask, "root")
        if direct == 7:
            assert not P.paired_inside(v, vc), (v, mask)
        else:
            assert P.death_of.get(vc) == P.cell(v, EDGE3[direct]), (v, mask, "direct")
        for i, off in enumerate(EDGE3):
            ec = P.cell(v, off)
            if ec is None or P.lsv[ec] != v:
                assert not (mask >> i) & 1 or ec is None
                continue
            if i == direct:
                continue
            if (keep_e >> i) & 1:
                assert not P.paired_inside(v, ec), (v, mask, i, "keep edge")
            else:
                assert P.paired_inside(v, ec), (v, mask, i, "pruned edge")
        for s, off in enumerate(SQ3):
            sc = P.cell(v, off)
            if sc is None or P.lsv[sc] != v:
                assert not (keep_s >> s) & 1, (v, mask, s, "keep square outside L(v)")
                continue
            if (keep_s >> s) & 1:
                assert not P.paired_inside(v, sc), (v, mask, s, "keep square")
            else:
                assert P.paired_inside(v, sc), (v, mask, s, "square not paired inside")
        for c in range(8):
            off = (1 if c >> 2 else -1, 1 if (c >> 1) & 1 else -1, 1 if c & 1 else -1)
            cc = P.cell(v, off)
            inside = cc is not None and P.lsv[cc] == v
            assert bool((present_c >> c) & 1) == inside, (v, mask, c, "cube presence")
            if not inside:
                continue
            killed = P.birth_of[cc]                        # cubes are never positive (H3 = 0)
            if (root >> c) & 1:
                assert P.lsv[killed] != v, (v, mask, c, "root cube")
            else:
                assert P.lsv[killed] == v, (v, mask, c, "local cube")
                t = (e >> (29 + 3 * c)) & 7
                o = other_cofacet_octant(P, v, killed, cc)
                assert o == (1 if t >> 2 else -1, 1 if (t >> 1) & 1 else -1, 1 if t & 1 else -1), \
                    (v, mask, c, "link")


@pytest.mark.parametrize("seed", range(6))
def test_lut_2d_against_oracle(seed):
    rng = np.random.default_rng(seed)
    for k in range(4):
        shape = tuple(int(x) for x in rng.integers(2, 8, size=2))
        lev = int(rng.choice([2, 3, 1 << 20]))
        check_2d(S.levels(shape, lev, 500 + 10 * seed + k))


@pytest.mark.parametrize("seed", range(4))
def test_lut_3d_against_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    for k in range(2):
        shape = tuple(int(x) for x in rng.integers(2, 5, size=3))
        lev = int(rng.choice([2, 3, 1 << 20]))
        check_3d(S.levels(shape, lev, 700 + 10 * seed + k))


def test_lut_3d_fields():
    check_3d(S.grf((5, 5, 5), 1.0, 11))
    check_3d(S.quantize_u8(S.grf((4, 5, 6), 1.5, 12)))
