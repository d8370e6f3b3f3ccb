"""Independent, test-only references used to pin the oracle.

Nothing here is imported by the oracle or by the GPU library, and nothing here imports them.
The code is deliberately different from the oracle's: it enumerates cells with numpy, uses
F2 ranks of bit-packed Python integers, and implements textbook special cases.

  * ``persistent_betti_multiset``: value pairs from ranks of persistent homology groups
    (no pairing algorithm at all), so it fixes the (birth, death) value multiset of every
    dimension independently of any tie-break.
  * ``pairing_lemma_pairs``: exact index pairs from the pairing lemma
    r(i,j) - r(i+1,j) + r(i+1,j-1) - r(i,j-1) = 1 on the boundary matrix in refined order.
  * ``kruskal_h0``: H0 by sequential Kruskal with the elder rule over all edges.
  * ``dual_union_find_top``: top-dimension pairs by union-find on the dual graph (top cells
    plus one cell at infinity, facets taken in reverse order; paper Sec. 3.1 / Appendix A).
  * ``product_field`` / ``product_bars``: an image or volume f = max(g_0(i_0), g_1(i_1), ...)
    of 1D sequences is a product filtration; by the Kuenneth formula over a field its
    barcode is fixed by the factors' 1D H0 bars: H0 is every combination
    [max of births, min of deaths) of non-zero length and no higher dimension has a bar
    (each factor has only H0, and the torsion terms of the max-product are empty).  This
    gives the value multiset at any size, e.g. for a 2^27-voxel volume.
"""
from __future__ import annotations

import itertools

import numpy as np


class Complex:
    """Doubled-grid cubical complex of an image/volume; 2D input is seen as (1,H,W)."""

    def __init__(self, img: np.ndarray, ndim: int | None = None):
        img = np.asarray(img, dtype=np.float32)
        self.ndim = img.ndim if ndim is None else ndim
        e = (1,) * (3 - img.ndim) + img.shape
        self.e = e
        self.img = img.reshape(e)
        self.vals = self.img.ravel()
        self.d = tuple(2 * x - 1 for x in e)
        n = int(np.prod(self.d))
        self.n = n
        co = np.stack(np.unravel_index(np.arange(n), self.d), axis=1)
        self.co = co
        self.dim = (co % 2).sum(axis=1)
        # vertex order: value (IEEE, -0 == +0), then pixel index
        v = self.vals.astype(np.float64) + 0.0
        pix = np.arange(self.vals.size)
        order = np.lexsort((pix, v))
        vrank = np.empty(self.vals.size, np.int64)
        vrank[order] = np.arange(self.vals.size)
        self.vrank = vrank
        lsv = np.empty(n, np.int64)
        for c in range(n):
            best, br = -1, -1
            for vv in self.vertices(c):
                if vrank[vv] > br:
                    br, best = vrank[vv], vv
            lsv[c] = best
        self.lsv = lsv
        self.f = self.vals[lsv]
        # refined order: (rank of lower-star vertex, dim, cellidx)
        self.order = np.lexsort((np.arange(n), self.dim, vrank[lsv]))
        self.pos = np.empty(n, np.int64)
        self.pos[self.order] = np.arange(n)

    def vertices(self, c):
        co = self.co[c]
        ch = [(x // 2, x // 2 + 1) if x % 2 else (x // 2,) for x in co]
        for z, y, x in itertools.product(*ch):
            yield (z * self.e[1] + y) * self.e[2] + x

    def cidx(self, co):
        return (co[0] * self.d[1] + co[1]) * self.d[2] + co[2]

    def facets(self, c):
        co = list(self.co[c])
        out = []
        for k in range(3):
            if co[k] % 2:
                for s in (-1, 1):
                    t = list(co)
                    t[k] += s
                    out.append(self.cidx(t))
        return out

    def cofacets(self, c):
        co = list(self.co[c])
        out = []
        for k in range(3):
            if co[k] % 2 == 0:
                for s in (-1, 1):
                    t = list(co)
                    t[k] += s
                    if 0 <= t[k] < self.d[k]:
                        out.append(self.cidx(t))
        return out

    def cells_of_dim(self, p):
        return np.nonzero(self.dim == p)[0]


# ----------------------------------------------------------------------- F2 rank --

def f2_rank(rows) -> int:
    """Rank over F2 of a list of row bitmasks (Python ints)."""
    basis = {}
    r = 0
    for x in rows:
        while x:
            h = x.bit_length() - 1
            if h in basis:
                x ^= basis[h]
            else:
                basis[h] = x
                r += 1
                break
    return r


def _boundary_rows(cx: Complex, p: int, row_cells, col_cells):
    """Rows (bitmask over col positions) of d_p restricted to the given cells."""
    cindex = {int(c): i for i, c in enumerate(col_cells)}
    rows = {int(r): 0 for r in row_cells}
    for c in col_cells:
        for fc in cx.facets(int(c)):
            if fc in rows:
                rows[fc] ^= 1 << cindex[int(c)]
    return rows


def persistent_betti_multiset(img, ndim=None):
    """{(p, birth value, death value or inf): multiplicity} from persistent Betti numbers.

    beta_p^{s,t} = n_p(K_s) - rank d_p|K_s - rank d_{p+1}|K_t + rank (rows of d_{p+1}|K_t
    outside K_s); multiplicities by inclusion-exclusion over consecutive values.
    """
    cx = Complex(img, ndim)
    vals = np.unique(cx.f.astype(np.float64) + 0.0)
    m = len(vals)
    top = cx.ndim

    def beta(p, s, t):
        if s < 0:
            return 0
        Ks = set(np.nonzero(cx.f <= vals[s])[0].tolist())
        Kt = set(np.nonzero(cx.f <= vals[t])[0].tolist())
        cp_s = [c for c in Ks if cx.dim[c] == p]
        n_ps = len(cp_s)
        if p > 0:
            rows = _boundary_rows(cx, p, [c for c in Ks if cx.dim[c] == p - 1], cp_s)
            rk_p = f2_rank(rows.values())
        else:
            rk_p = 0
        cq_t = [c for c in Kt if cx.dim[c] == p + 1]
        rows_t = _boundary_rows(cx, p + 1, [c for c in Kt if cx.dim[c] == p], cq_t)
        rk_q = f2_rank(rows_t.values())
        rk_out = f2_rank([v for r, v in rows_t.items() if r not in Ks])
        return n_ps - rk_p - rk_q + rk_out

    out = {}
    for p in range(0, top + 1):
        B = [[beta(p, s, t) if t >= s else 0 for t in range(m)] for s in range(-1, m)]
        b = lambda s, t: B[s + 1][t]
        for i in range(m):
            for j in range(i + 1, m):
                mu = b(i, j - 1) - b(i - 1, j - 1) - b(i, j) + b(i - 1, j)
                if mu:
                    out[(p, float(vals[i]), float(vals[j]))] = mu
            mu_inf = b(i, m - 1) - b(i - 1, m - 1)
            if mu_inf:
                out[(p, float(vals[i]), float("inf"))] = mu_inf
    return out


def multiset_of(pairs, dims=None):
    out = {}
    for p in pairs:
        d = int(p["dim"])
        if dims is not None and d not in dims:
            continue
        k = (d, float(p["birth"]) + 0.0, float(p["death"]) + 0.0)
        out[k] = out.get(k, 0) + 1
    return out


# ---------------------------------------------------------------- pairing lemma --

def pairing_lemma_pairs(img, ndim=None):
    """All (birth cell, death cell) pairs, zero persistence included, from the lemma."""
    cx = Complex(img, ndim)
    n = cx.n
    cols = []   # column j (refined position) as bitmask over row positions
    for j in range(n):
        c = int(cx.order[j])
        m = 0
        for fc in cx.facets(c):
            m |= 1 << int(cx.pos[fc])
        cols.append(m)

    def r(i, j):
        if i >= n or j < 0:
            return 0
        mask = ~((1 << i) - 1)
        return f2_rank([cols[t] & mask for t in range(j + 1)])

    pairs = set()
    for j in range(n):
        for i in range(j):
            if r(i, j) - r(i + 1, j) + r(i + 1, j - 1) - r(i, j - 1) == 1:
                pairs.add((int(cx.order[i]), int(cx.order[j])))
    return pairs, cx


# ---------------------------------------------------------------------- Kruskal --

def kruskal_h0(img, ndim=None, keep_zero=False):
    """H0 pairs (birth cell, death cell) by sequential Kruskal, elder rule."""
    cx = Complex(img, ndim)
    parent = {}

    def find(x):
        while parent.get(x, x) != x:
            x = parent[x]
        return x

    edges = sorted(cx.cells_of_dim(1).tolist(), key=lambda c: cx.pos[c])
    vcell = lambda v: cx.cidx([2 * x for x in np.unravel_index(v, cx.e)])
    out = []
    for e in edges:
        a, b = [int(x) for x in cx.vertices(e)]
        ra, rb = find(a), find(b)
        if ra == rb:
            continue
        young, old = (ra, rb) if cx.vrank[ra] > cx.vrank[rb] else (rb, ra)
        parent[young] = old
        if keep_zero or cx.vals[young] != cx.f[e]:
            out.append((vcell(young), int(e)))
    roots = {find(v) for v in range(cx.vals.size)}
    for r in roots:
        out.append((vcell(r), -1))
    return sorted(out)


# ----------------------------------------------------------------- dual union-find --

def dual_union_find_top(img, ndim=None, keep_zero=False):
    """Top-dimension pairs (facet cell, top cell) by union-find on the dual graph."""
    cx = Complex(img, ndim)
    D = cx.ndim
    INF = -1
    parent = {}

    def find(x):
        while parent.get(x, x) != x:
            x = parent[x]
        return x

    def elder(a, b):          # dual age: larger refined position is elder; inf eldest
        if a == INF:
            return True
        if b == INF:
            return False
        return cx.pos[a] > cx.pos[b]

    facs = sorted(cx.cells_of_dim(D - 1).tolist(), key=lambda c: -cx.pos[c])
    out = []
    for s in facs:
        cof = [c for c in cx.cofacets(s) if cx.dim[c] == D]
        if len(cof) == 0:
            continue
        ends = cof + [INF] if len(cof) == 1 else cof
        r1, r2 = find(ends[0]), find(ends[1])
        if r1 == r2:
            continue
        young, old = (r2, r1) if elder(r1, r2) else (r1, r2)
        parent[young] = old
        if keep_zero or cx.f[s] != cx.f[young]:
            out.append((int(s), int(young)))
    return sorted(out)


def bars_1d(g):
    """H0 bars (birth, death) of a 1D sequence under the V-filtration (an edge enters at the
    larger of its two values), by union-find with the elder rule; the essential bar last."""
    g = [float(x) for x in g]
    n = len(g)
    parent = list(range(n))
    born = {}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    events = [(g[t], 0, t) for t in range(n)] + [(max(g[t], g[t + 1]), 1, t) for t in range(n - 1)]
    out = []
    for v, kind, t in sorted(events):
        if kind == 0:
            born[t] = (g[t], t)
            continue
        a, b = find(t), find(t + 1)
        if born[a] < born[b]:
            a, b = b, a                       # a: the younger root, which dies
        out.append((born[a][0], v))
        parent[a] = b
    out.append((born[find(0)][0], float("inf")))
    return out


def product_field(gs):
    """f[i_0, i_1, ...] = max_k g_k[i_k] as float32 (gs: 2 or 3 sequences, slowest axis first)."""
    gs = [np.asarray(g, np.float32) for g in gs]
    f = gs[0].reshape((-1,) + (1,) * (len(gs) - 1))
    for k, g in enumerate(gs[1:], 1):
        shape = [1] * len(gs)
        shape[k] = -1
        f = np.maximum(f, g.reshape(shape))
    return np.ascontiguousarray(f, dtype=np.float32)


def product_bars(gs):
    """Sorted (dim, birth, death) multiset of product_field(gs), non-zero persistence only."""
    out = []
    for tr in itertools.product(*[bars_1d(g) for g in gs]):
        b = max(x[0] for x in tr)
        d = min(x[1] for x in tr)
        if d > b:
            out.append((0, b, d))
    return sorted(out)
