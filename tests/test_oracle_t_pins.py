"""Pins of the oracle's T-filtration (pixels as top cells, paper Sec. 2.2) against facts that
do not come from its own code:

* connectivity: the sublevel complex at t is the union of the closed pixels with f <= t, so
  its H0 counts the components of {f <= t} under 8-adjacency (26 in 3D), and its top
  homology the components of {f > t} under 4-adjacency (6 in 3D) that do not touch the image
  border (scipy's labelling does the counting);
* Alexander duality with the V-filtration, cell by cell: the T complex of f is the dual cell
  complex of the V complex of g = -f, point-reflected and framed by a ring of -inf pixels.
  A T pair (s, t) of dimension k is the V pair (t*, s*) of dimension d-1-k, with values
  negated; the frame's own top class is the T essential class.  The reflection turns the V
  tie-break (larger value, then larger index, enters later) into the T one (smaller value,
  then smaller index, enters first), so even the cells chosen under ties agree;
* small cases worked by hand.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import synthetic as S


def T(img, **kw):
    return oracle.diagram(img, filtration="T", **kw)


def test_diagonal_pixels_touch():
    """Two pixels that share only a corner are one component under T, two under V."""
    a = np.array([[0, 1], [1, 0]], np.float32)
    t = T(a)
    assert len(t) == 1 and t["dim"][0] == 0 and t["death_cell"][0] == -1
    v = oracle.diagram(a)
    assert len(v[v["dim"] == 0]) == 2


def test_ring_around_a_pixel():
    """A ring of 0 around a pixel of 5: one loop born at 0, filled when the centre enters,
    whose top cell sits at doubled coordinates (3, 3) of the 7x7 grid."""
    a = np.zeros((3, 3), np.float32)
    a[1, 1] = 5
    t = T(a)
    assert list(t["dim"]) == [0, 1]
    assert (t["birth"][1], t["death"][1]) == (0.0, 5.0)
    assert t["death_cell"][1] == 3 * 7 + 3 and t["death_vertex"][1] == 4


def test_diagonal_gap_is_not_a_hole():
    """Under T a loop needs 4-connected background: a background pixel enclosed only
    diagonally still makes a hole (its sides are in the complex), but two background pixels
    meeting at a corner whose other two pixels are foreground are separated there."""
    a = np.array([[0, 0, 0, 0],
                  [0, 9, 0, 0],
                  [0, 0, 9, 0],
                  [0, 0, 0, 0]], np.float32)
    t = T(a)
    h1 = t[t["dim"] == 1]
    assert sorted(zip(h1["birth"], h1["death"])) == [(0.0, 9.0), (0.0, 9.0)]


def betti_from_pairs(pairs, dim, t):
    p = pairs[pairs["dim"] == dim]
    return int(((p["birth"] <= t) & (t < p["death"])).sum())


def betti_from_labels(img, t):
    nd = img.ndim
    _, b0 = ndimage.label(img <= t, structure=np.ones((3,) * nd, bool))
    lab, nb = ndimage.label(img > t, structure=ndimage.generate_binary_structure(nd, 1))
    border = set()
    for ax in range(nd):
        for side in (0, -1):
            border |= set(np.unique(np.take(lab, side, axis=ax)).tolist())
    holes = len(set(range(1, nb + 1)) - border)
    return b0, holes


@pytest.mark.parametrize("nd", [2, 3])
def test_betti_numbers_match_connectivity(nd):
    rng = np.random.default_rng(40 + nd)
    for k in range(60 if nd == 2 else 40):
        shape = tuple(int(x) for x in rng.integers(1, 12 if nd == 2 else 7, size=nd))
        img = S.levels(shape, int(rng.choice([2, 3, 6, 1 << 20])), 900 + 10 * nd + k)
        pairs = T(img)
        top = nd - 1
        for t in np.unique(img):
            b0, bt = betti_from_labels(img, t)
            assert betti_from_pairs(pairs, 0, t) == b0, (shape, k, t)
            assert betti_from_pairs(pairs, top, t) == bt, (shape, k, t)
        assert betti_from_pairs(pairs, 0, np.float32(img.min()) - 1) == 0


def dual_image(f):
    """g = -f point-reflected, framed by one ring of -inf pixels."""
    g = np.full(tuple(e + 2 for e in f.shape), -np.inf, np.float32)
    g[(slice(1, -1),) * f.ndim] = -f[(slice(None, None, -1),) * f.ndim]
    return g


def t_from_v(f, v):
    """The T pairs of f that duality predicts from the V pairs v of dual_image(f), in the T
    output order (dimension, then death key, essential class last)."""
    nd = f.ndim
    n = np.array((1,) * (3 - nd) + f.shape)           # pixel extents, leading 1 for images
    P = n + np.where(np.arange(3) < 3 - nd, 0, 2)     # framed extents
    dv = np.where(np.arange(3) < 3 - nd, 1, 2 * P - 1)   # V doubled extents
    dt = np.where(np.arange(3) < 3 - nd, 1, 2 * n + 1)   # T doubled extents
    fl = f.reshape(-1)

    def coords(i, ext):
        c = []
        for e in ext[::-1]:
            c.append(i % e)
            i //= e
        return c[::-1]

    def is_frame(vtx):
        c = coords(int(vtx), P)
        return any(not (1 <= c[k] <= P[k] - 2) for k in range(3 - nd, 3))

    def pixel(vtx):
        c = coords(int(vtx), P)
        q = [0 if k < 3 - nd else n[k] - c[k] for k in range(3)]
        assert all(0 <= q[k] < n[k] for k in range(3))
        return int((q[0] * n[1] + q[1]) * n[2] + q[2])

    def cell(ci):
        c = coords(int(ci), dv)
        x = [0 if k < 3 - nd else 2 * n[k] + 1 - c[k] for k in range(3)]
        assert all(0 <= x[k] < dt[k] for k in range(3))
        return int((x[0] * dt[1] + x[1]) * dt[2] + x[2])

    out = []
    for vd in (nd - 1, 0):                            # V top -> T H0, V H0 -> T top
        for p in v[v["dim"] == vd][::-1]:
            if p["death_cell"] < 0:                   # the frame's component: no T class
                assert vd == 0 and is_frame(p["birth_vertex"])
                continue
            b_pix = pixel(p["death_vertex"])
            b_cell = cell(p["death_cell"])
            if vd == nd - 1 and is_frame(p["birth_vertex"]):
                out.append((0, fl[b_pix], np.float32(np.inf), b_cell, -1, b_pix, -1))
                assert p["birth"] == -np.inf
                continue
            d_pix = pixel(p["birth_vertex"])
            assert fl[b_pix] == -p["death"] and fl[d_pix] == -p["birth"]
            out.append((nd - 1 - vd, fl[b_pix], fl[d_pix], b_cell, cell(p["birth_cell"]), b_pix, d_pix))
    return np.array(out, dtype=oracle.PAIR_DTYPE)


def same(a, b):
    if len(a) != len(b):
        return "count %d != %d" % (len(a), len(b))
    for name in a.dtype.names:
        x, y = np.asarray(a[name]), np.asarray(b[name])
        if x.dtype == np.float32:
            x, y = x.view(np.uint32), y.view(np.uint32)
        bad = np.nonzero(x != y)[0]
        if len(bad):
            return "%s differs at %d: %r vs %r" % (name, bad[0], a[bad[0]], b[bad[0]])
    return None


@pytest.mark.parametrize("nd", [2, 3])
def test_alexander_duality_with_v_cell_by_cell(nd):
    rng = np.random.default_rng(70 + nd)
    for k in range(80 if nd == 2 else 50):
        shape = tuple(int(x) for x in rng.integers(1, 11 if nd == 2 else 6, size=nd))
        img = S.levels(shape, int(rng.choice([2, 3, 5, 1 << 20])), 3000 + 10 * nd + k)
        msg = same(T(img), t_from_v(img, oracle.diagram(dual_image(img))))
        assert msg is None, (shape, k, msg)


def test_duality_with_special_values():
    a = np.array([[0.0, -0.0, 1.0, -np.inf], [-np.inf, 0.5, -0.0, 0.0], [1e-45, -1e-45, 3.0, 0.0]],
                 np.float32)
    assert same(T(a), t_from_v(a, oracle.diagram(dual_image(a)))) is None
    v = np.stack([a, a[::-1], a]).astype(np.float32)
    assert same(T(v), t_from_v(v, oracle.diagram(dual_image(v)))) is None


def test_full_and_split_reductions_agree():
    rng = np.random.default_rng(5)
    for k in range(30):
        nd = 2 + (k % 2)
        shape = tuple(int(x) for x in rng.integers(1, 8 if nd == 2 else 5, size=nd))
        img = S.levels(shape, 3, 7000 + k)
        a = T(img, method=oracle.FULL)
        a = a[(a["dim"] == 0) | (a["dim"] == nd - 1)]
        assert same(a, T(img, method=oracle.SPLIT)) is None


def t_death_key(img, cell):
    """Refined T key of a cell of the T doubled grid (extents 2n+1, an image seen as one
    layer): (value, pixel index of the entry top cell, dimension, cell index), the entry top
    cell being the (value, index)-smallest pixel whose closed cell contains it."""
    a = img.reshape((1,) * (3 - img.ndim) + img.shape)
    n = a.shape
    d = [1 if img.ndim == 2 and k == 0 else 2 * n[k] + 1 for k in range(3)]
    z, rem = divmod(int(cell), d[1] * d[2])
    y, x = divmod(rem, d[2])
    co = (z, y, x)
    choices = []
    for k in range(3):
        c = co[k]
        if img.ndim == 2 and k == 0:
            choices.append([0])
        elif c % 2:
            choices.append([(c - 1) // 2])
        else:
            choices.append([p for p in (c // 2 - 1, c // 2) if 0 <= p < n[k]])
    best = min((float(a[i, j, l]) + 0.0, (i * n[1] + j) * n[2] + l)
               for i in choices[0] for j in choices[1] for l in choices[2])
    dim = sum(1 for k in range(3 - img.ndim, 3) if co[k] % 2 == 1)
    return best + (dim, int(cell))


def test_t_output_order_is_death_key_essential_last():
    """T pairs come by (dim, refined T key of the death cell), the essential class last in
    H0; the key is recomputed here from the T definition (Sec. 2.2) and reading T1.  Tied
    inputs make the death key order differ from the death cell index and from the birth
    order, so a sort on either fails."""
    witnessed = 0
    for k in range(60):
        nd = 2 + (k % 2)
        rng = np.random.default_rng(8300 + k)
        shape = tuple(int(x) for x in rng.integers(4, 10 if nd == 2 else 6, size=nd))
        img = S.levels(shape, int(rng.choice([2, 3, 4])), 8400 + k)
        pr = T(img)
        key = [(int(p["dim"]), 1, ()) if p["death_cell"] < 0 else
               (int(p["dim"]), 0, t_death_key(img, p["death_cell"])) for p in pr]
        assert key == sorted(key) and len(set(key)) == len(key), (shape, k)
        assert int((pr["death_cell"] < 0).sum()) == 1 and pr["death_cell"][(pr["dim"] == 0).sum() - 1] == -1
        for d in (0, nd - 1):
            sel = pr[(pr["dim"] == d) & (pr["death_cell"] >= 0)]
            if len(sel) > 1:
                witnessed += sel["death_cell"].tolist() != sorted(sel["death_cell"].tolist())
    assert witnessed >= 5, "the inputs never separate the death key order from the cell index"
