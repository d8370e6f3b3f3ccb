/*
 * cubical_oracle.c -- plain CPU reference for V- and T-filtration cubical persistence over F2.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this file or the
 * library built from it; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU library.
 *
 * What it computes (the plain definition, no pruning, no lookup table, no union-find):
 *   - the cubical complex on the pixel grid: cells are products of elementary
 *     intervals, dimension = number of non-degenerate factors (paper Sec. 2.2);
 *   - the V-filtration f(cell) = max over the cell's vertices of the pixel value
 *     (paper Sec. 2.2, lower-star filtration);
 *   - the fully refined order (paper Sec. 2.3): first by the lower-star vertex under
 *     the vertex order (value, then row-major pixel index as first-order tie-break),
 *     then by dimension, then by the cell's linear index on the doubled grid
 *     (second-order tie-break inside the lower star);
 *   - persistence pairs by the standard column reduction of the boundary matrix
 *     over F2 in that order (paper Sec. 2.1);
 *   - pairs whose birth and death values are equal are omitted (paper Sec. 2.3).
 *
 * Two reduction routes, which give identical pairs:
 *   OR_FULL  : reduce the whole boundary matrix, every dimension.
 *   OR_SPLIT : reduce only the blocks needed for the requested dimensions.  H0 comes
 *              from the vertex-edge block.  The top dimension's pairs come from the
 *              anti-transposed (coboundary) block of the top cells, reduced in reverse
 *              order, which yields the same pairs as the boundary block (the homology /
 *              cohomology duality the paper's Sec. 3.1 and Appendix A rely on).  Other
 *              middle dimensions use their boundary block.  In this route the only
 *              essential class reported is the one of H0 (the grid is contractible).
 *
 * T-filtration (or_diagram_t; paper Sec. 2.2, its dual construction): the pixels are the
 * top cells of a complex on (H+1)x(W+1) [(D+1)x(H+1)x(W+1)] vertices.  A cell's value is
 * the minimum over the top cells that contain it; the first-order tie-break is the top cell
 * through which the cell enters, i.e. the minimum of those top cells under the pixel order
 * (value, then row-major pixel index): the pseudo lower star the paper's Sec. 3.3 names for
 * this case.  The rest of the order (dimension, then doubled-grid cell index) and the
 * reduction are those of the V case.  birth_vertex / death_vertex name the pixel whose
 * value the cell takes.  Output order: by dimension, then by the death cell's position in
 * the refined order, essential classes last.  Pixel (i,j[,k]) is the top cell at doubled
 * coordinates (2i+1, 2j+1[, 2k+1]); the doubled grid has extents 2e+1 (1 on the leading
 * axis of an image).
 *
 * Cell indexing: a 2D image of extents (H,W) is treated as a (1,H,W) volume.  Cell
 * coordinates live on the doubled grid (2H-1, 2W-1) [(2D-1, 2H-1, 2W-1) in 3D]; a
 * coordinate is odd where the cell has a non-degenerate factor.  cellidx is the
 * row-major linear index on that grid, pixidx the row-major pixel index.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "cubical_oracle.h"

typedef struct {
    int ndim;          /* 2 or 3: dimension of the complex the caller asks for */
    int tmode;         /* 0: V-filtration (pixels are vertices), 1: T (pixels are top cells) */
    int64_t e[3];      /* pixel extents, slowest first, padded to 3 with leading 1 */
    int64_t d[3];      /* doubled extents: 2e-1 (V), 2e+1 (T; 1 on the leading axis in 2D) */
    int64_t nvox;
    int64_t ncell;
    const float *img;
    int64_t *vrank;    /* vertex rank under (value, pixidx) */
} grid_t;

/* ---------------------------------------------------------------- vertex order -- */

typedef struct { float v; int64_t p; } vkey_t;

static int cmp_vkey(const void *a, const void *b) {
    const vkey_t *x = (const vkey_t *)a, *y = (const vkey_t *)b;
    /* IEEE comparison: -0 and +0 compare equal, so the pixel index decides. */
    if (x->v < y->v) return -1;
    if (x->v > y->v) return 1;
    if (x->p < y->p) return -1;
    if (x->p > y->p) return 1;
    return 0;
}

static int build_vertex_ranks(grid_t *g) {
    vkey_t *k = (vkey_t *)malloc(sizeof(vkey_t) * (size_t)g->nvox);
    if (!k) return OR_ENOMEM;
    for (int64_t i = 0; i < g->nvox; ++i) { k[i].v = g->img[i]; k[i].p = i; }
    qsort(k, (size_t)g->nvox, sizeof(vkey_t), cmp_vkey);
    g->vrank = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->nvox);
    if (!g->vrank) { free(k); return OR_ENOMEM; }
    for (int64_t r = 0; r < g->nvox; ++r) g->vrank[k[r].p] = r;
    free(k);
    return OR_OK;
}

/* ------------------------------------------------------------------ cell facts -- */

static void cell_coords(const grid_t *g, int64_t c, int64_t co[3]) {
    co[2] = c % g->d[2]; c /= g->d[2];
    co[1] = c % g->d[1]; c /= g->d[1];
    co[0] = c;
}

static int64_t cell_index(const grid_t *g, const int64_t co[3]) {
    return (co[0] * g->d[1] + co[1]) * g->d[2] + co[2];
}

static int cell_dim(const int64_t co[3]) {
    return (int)((co[0] & 1) + (co[1] & 1) + (co[2] & 1));
}

/* The vertex of the cell that enters last: the maximum, under the vertex order, of
 * the cell's vertices (floor / ceil halves of each odd coordinate). */
static int64_t cell_lsv(const grid_t *g, const int64_t co[3]) {
    int64_t best = -1, bestr = -1;
    for (int m = 0; m < 8; ++m) {
        int64_t v[3];
        int ok = 1;
        for (int k = 0; k < 3; ++k) {
            int bit = (m >> k) & 1;
            if (co[k] & 1) v[k] = co[k] / 2 + bit;
            else { v[k] = co[k] / 2; if (bit) ok = 0; }
        }
        if (!ok) continue;
        int64_t p = (v[0] * g->e[1] + v[1]) * g->e[2] + v[2];
        if (g->vrank[p] > bestr) { bestr = g->vrank[p]; best = p; }
    }
    return best;
}

/* T-filtration: the top cell through which the cell enters -- the minimum, under the pixel
 * order, of the top cells containing it.  An odd coordinate is fixed; an even coordinate c
 * on an axis of the complex takes the neighbours c-1 and c+1 that lie inside the grid. */
static int64_t cell_entry_top(const grid_t *g, const int64_t co[3]) {
    int64_t best = -1, bestr = -1;
    const int k0 = 3 - g->ndim;                        /* first axis of the complex */
    for (int m = 0; m < 8; ++m) {
        int64_t t[3];
        int ok = 1;
        for (int k = 0; k < 3; ++k) {
            int bit = (m >> k) & 1;
            if (k < k0) { t[k] = 0; if (bit) ok = 0; continue; }
            if (co[k] & 1) { t[k] = co[k]; if (bit) ok = 0; }
            else t[k] = co[k] + (bit ? 1 : -1);
            if (t[k] < 0 || t[k] >= g->d[k]) ok = 0;
        }
        if (!ok) continue;
        int64_t q[3];
        for (int k = 0; k < 3; ++k) q[k] = k < k0 ? 0 : (t[k] - 1) / 2;
        int64_t p = (q[0] * g->e[1] + q[1]) * g->e[2] + q[2];
        if (bestr < 0 || g->vrank[p] < bestr) { bestr = g->vrank[p]; best = p; }
    }
    return best;
}

/* The pixel whose value the cell takes and whose rank orders it first. */
static int64_t cell_pixel(const grid_t *g, const int64_t co[3]) {
    return g->tmode ? cell_entry_top(g, co) : cell_lsv(g, co);
}

/* Key of the fully refined order: (rank of lower-star vertex, dim, cellidx). */
typedef struct { int64_t r; int64_t dim; int64_t c; } ckey_t;

static int cmp_ckey(const void *a, const void *b) {
    const ckey_t *x = (const ckey_t *)a, *y = (const ckey_t *)b;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->dim != y->dim) return x->dim < y->dim ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return 0;
}

static ckey_t key_of(const grid_t *g, int64_t c) {
    int64_t co[3];
    cell_coords(g, c, co);
    ckey_t k;
    k.r = g->vrank[cell_pixel(g, co)];
    k.dim = cell_dim(co);
    k.c = c;
    return k;
}

/* Facets: move one odd coordinate by -1 or +1.  Returns the count. */
static int facets(const grid_t *g, int64_t c, int64_t out[6]) {
    int64_t co[3];
    cell_coords(g, c, co);
    int n = 0;
    for (int k = 0; k < 3; ++k) {
        if (!(co[k] & 1)) continue;
        for (int s = -1; s <= 1; s += 2) {
            int64_t t[3] = {co[0], co[1], co[2]};
            t[k] += s;
            out[n++] = cell_index(g, t);
        }
    }
    return n;
}

/* Cofacets: move one even coordinate by -1 or +1, staying inside the grid. */
static int cofacets(const grid_t *g, int64_t c, int64_t out[6]) {
    int64_t co[3];
    cell_coords(g, c, co);
    int n = 0;
    for (int k = 0; k < 3; ++k) {
        if (co[k] & 1) continue;
        for (int s = -1; s <= 1; s += 2) {
            int64_t t[3] = {co[0], co[1], co[2]};
            t[k] += s;
            if (t[k] < 0 || t[k] >= g->d[k]) continue;
            out[n++] = cell_index(g, t);
        }
    }
    return n;
}

/* ------------------------------------------------------------- sparse columns -- */
/* A column is a sorted array of row positions (ascending).  Addition over F2 is the
 * symmetric difference. */

typedef struct { int64_t *v; int64_t n, cap; } col_t;

static int col_push(col_t *c, int64_t x) {
    if (c->n == c->cap) {
        int64_t nc = c->cap ? 2 * c->cap : 4;
        int64_t *nv = (int64_t *)realloc(c->v, sizeof(int64_t) * (size_t)nc);
        if (!nv) return OR_ENOMEM;
        c->v = nv; c->cap = nc;
    }
    c->v[c->n++] = x;
    return OR_OK;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* dst := dst + src over F2 (both sorted). */
static int col_add(col_t *dst, const col_t *src) {
    int64_t alloc = dst->n + src->n + 1;
    int64_t *out = (int64_t *)malloc(sizeof(int64_t) * (size_t)alloc);
    if (!out) return OR_ENOMEM;
    int64_t i = 0, j = 0, n = 0;
    while (i < dst->n || j < src->n) {
        if (j >= src->n || (i < dst->n && dst->v[i] < src->v[j])) out[n++] = dst->v[i++];
        else if (i >= dst->n || src->v[j] < dst->v[i]) out[n++] = src->v[j++];
        else { ++i; ++j; }            /* equal entries cancel */
    }
    free(dst->v);
    dst->v = out; dst->n = n; dst->cap = alloc;
    return OR_OK;
}

/* ------------------------------------------------------------------- results -- */

typedef struct { or_pair *p; int64_t n, cap; } plist_t;

static int plist_push(plist_t *L, or_pair x) {
    if (L->n == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 64;
        or_pair *np = (or_pair *)realloc(L->p, sizeof(or_pair) * (size_t)nc);
        if (!np) return OR_ENOMEM;
        L->p = np; L->cap = nc;
    }
    L->p[L->n++] = x;
    return OR_OK;
}

/* Record pair (birth cell b, death cell d; d < 0 for an essential class) when its
 * dimension is requested and, unless keep_zero, its persistence is not zero. */
static int emit(const grid_t *g, plist_t *L, uint32_t dims_mask, int keep_zero,
                int64_t b, int64_t d) {
    int64_t co[3];
    cell_coords(g, b, co);
    int dim = cell_dim(co);
    if (!((dims_mask >> dim) & 1u)) return OR_OK;
    or_pair x;
    memset(&x, 0, sizeof x);
    x.dim = dim;
    x.birth_cell = b;
    x.birth_vertex = cell_pixel(g, co);
    x.birth = g->img[x.birth_vertex];
    if (d >= 0) {
        int64_t cd[3];
        cell_coords(g, d, cd);
        x.death_cell = d;
        x.death_vertex = cell_pixel(g, cd);
        x.death = g->img[x.death_vertex];
        if (!keep_zero && x.birth == x.death) return OR_OK;   /* zero persistence */
    } else {
        x.death_cell = -1;
        x.death_vertex = -1;
        x.death = INFINITY;
    }
    return plist_push(L, x);
}

/* ------------------------------------------------------------ full reduction -- */

static int reduce_full(const grid_t *g, uint32_t dims_mask, int keep_zero, plist_t *L) {
    int64_t n = g->ncell;
    ckey_t *k = (ckey_t *)malloc(sizeof(ckey_t) * (size_t)n);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *pivot = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);  /* row pos -> column pos */
    col_t *R = (col_t *)calloc((size_t)n, sizeof(col_t));
    char *paired = (char *)calloc((size_t)n, 1);
    int rc = OR_OK;
    if (!k || !pos || !pivot || !R || !paired) { rc = OR_ENOMEM; goto done; }
    for (int64_t c = 0; c < n; ++c) k[c] = key_of(g, c);
    qsort(k, (size_t)n, sizeof(ckey_t), cmp_ckey);
    for (int64_t i = 0; i < n; ++i) { pos[k[i].c] = i; pivot[i] = -1; }

    for (int64_t j = 0; j < n; ++j) {                 /* columns left to right */
        int64_t f[6];
        int nf = facets(g, k[j].c, f);
        for (int t = 0; t < nf; ++t)
            if ((rc = col_push(&R[j], pos[f[t]])) != OR_OK) goto done;
        qsort(R[j].v, (size_t)R[j].n, sizeof(int64_t), cmp_i64);
        while (R[j].n > 0) {
            int64_t low = R[j].v[R[j].n - 1];
            if (pivot[low] < 0) break;
            if ((rc = col_add(&R[j], &R[pivot[low]])) != OR_OK) goto done;
        }
        if (R[j].n > 0) {
            int64_t low = R[j].v[R[j].n - 1];
            pivot[low] = j;
            paired[low] = paired[j] = 1;
            if ((rc = emit(g, L, dims_mask, keep_zero, k[low].c, k[j].c)) != OR_OK) goto done;
        }
    }
    /* Essential classes: cells whose reduced column is zero and that kill nothing. */
    for (int64_t j = 0; j < n; ++j)
        if (!paired[j] && R[j].n == 0)
            if ((rc = emit(g, L, dims_mask, keep_zero, k[j].c, -1)) != OR_OK) goto done;
done:
    if (R) for (int64_t j = 0; j < n; ++j) free(R[j].v);
    free(R); free(k); free(pos); free(pivot); free(paired);
    return rc;
}

/* ---------------------------------------------------------- split reduction -- */

/* Sorted list of all cells of one dimension in the fully refined order. */
static int cells_of_dim(const grid_t *g, int dim, ckey_t **out, int64_t *cnt) {
    int64_t m = 0;
    for (int64_t c = 0; c < g->ncell; ++c) {
        int64_t co[3];
        cell_coords(g, c, co);
        if (cell_dim(co) == dim) ++m;
    }
    ckey_t *k = (ckey_t *)malloc(sizeof(ckey_t) * (size_t)(m ? m : 1));
    if (!k) return OR_ENOMEM;
    int64_t i = 0;
    for (int64_t c = 0; c < g->ncell; ++c) {
        int64_t co[3];
        cell_coords(g, c, co);
        if (cell_dim(co) == dim) k[i++] = key_of(g, c);
    }
    qsort(k, (size_t)m, sizeof(ckey_t), cmp_ckey);
    *out = k; *cnt = m;
    return OR_OK;
}

/* Boundary block d_{p+1}: columns = (p+1)-cells ascending, rows = p-cells.
 * Emits the H_p pairs; for p = 0 also the essential vertices. */
static int reduce_boundary_block(const grid_t *g, int p, uint32_t dims_mask, int keep_zero,
                                 plist_t *L) {
    ckey_t *rows = NULL, *cols = NULL;
    int64_t nr = 0, nc = 0;
    int rc;
    if ((rc = cells_of_dim(g, p, &rows, &nr)) != OR_OK) return rc;
    if ((rc = cells_of_dim(g, p + 1, &cols, &nc)) != OR_OK) { free(rows); return rc; }
    int64_t *rpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->ncell);
    int64_t *pivot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr ? nr : 1));
    col_t *R = (col_t *)calloc((size_t)(nc ? nc : 1), sizeof(col_t));
    char *rowpaired = (char *)calloc((size_t)(nr ? nr : 1), 1);
    if (!rpos || !pivot || !R || !rowpaired) { rc = OR_ENOMEM; goto done; }
    for (int64_t i = 0; i < nr; ++i) { rpos[rows[i].c] = i; pivot[i] = -1; }
    for (int64_t j = 0; j < nc; ++j) {
        int64_t f[6];
        int nf = facets(g, cols[j].c, f);
        for (int t = 0; t < nf; ++t)
            if ((rc = col_push(&R[j], rpos[f[t]])) != OR_OK) goto done;
        qsort(R[j].v, (size_t)R[j].n, sizeof(int64_t), cmp_i64);
        while (R[j].n > 0) {
            int64_t low = R[j].v[R[j].n - 1];
            if (pivot[low] < 0) break;
            if ((rc = col_add(&R[j], &R[pivot[low]])) != OR_OK) goto done;
        }
        if (R[j].n > 0) {
            int64_t low = R[j].v[R[j].n - 1];
            pivot[low] = j;
            rowpaired[low] = 1;
            if ((rc = emit(g, L, dims_mask, keep_zero, rows[low].c, cols[j].c)) != OR_OK) goto done;
        }
    }
    if (p == 0)
        for (int64_t i = 0; i < nr; ++i)
            if (!rowpaired[i])
                if ((rc = emit(g, L, dims_mask, keep_zero, rows[i].c, -1)) != OR_OK) goto done;
done:
    if (R) for (int64_t j = 0; j < nc; ++j) free(R[j].v);
    free(R); free(rows); free(cols); free(rpos); free(pivot); free(rowpaired);
    return rc;
}

/* Coboundary block of the top dimension D, anti-transposed: columns are the (D-1)-cells
 * taken in DEScending refined order, each holding the forward positions of its top-cell
 * cofacets; the pivot of a column is its smallest forward position (the last row in the
 * reversed order).  A non-zero reduced column of facet s with pivot tau gives the pair
 * (s, tau), the same pair the boundary block d_D gives. */
static int reduce_coboundary_top(const grid_t *g, int D, uint32_t dims_mask, int keep_zero,
                                 plist_t *L) {
    ckey_t *facs = NULL, *tops = NULL;
    int64_t nf = 0, nt = 0;
    int rc;
    if ((rc = cells_of_dim(g, D - 1, &facs, &nf)) != OR_OK) return rc;
    if ((rc = cells_of_dim(g, D, &tops, &nt)) != OR_OK) { free(facs); return rc; }
    int64_t *tpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->ncell);
    int64_t *pivot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt ? nt : 1));
    col_t *R = (col_t *)calloc((size_t)(nf ? nf : 1), sizeof(col_t));
    if (!tpos || !pivot || !R) { rc = OR_ENOMEM; goto done; }
    for (int64_t i = 0; i < nt; ++i) { tpos[tops[i].c] = i; pivot[i] = -1; }
    for (int64_t j = nf - 1; j >= 0; --j) {           /* reverse order */
        int64_t cf[6];
        int ncf = cofacets(g, facs[j].c, cf);
        for (int t = 0; t < ncf; ++t) {
            int64_t co[3];
            cell_coords(g, cf[t], co);
            if (cell_dim(co) != D) continue;
            if ((rc = col_push(&R[j], tpos[cf[t]])) != OR_OK) goto done;
        }
        qsort(R[j].v, (size_t)R[j].n, sizeof(int64_t), cmp_i64);
        while (R[j].n > 0) {
            int64_t low = R[j].v[0];                   /* smallest forward position */
            if (pivot[low] < 0) break;
            if ((rc = col_add(&R[j], &R[pivot[low]])) != OR_OK) goto done;
        }
        if (R[j].n > 0) {
            int64_t low = R[j].v[0];
            pivot[low] = j;
            if ((rc = emit(g, L, dims_mask, keep_zero, facs[j].c, tops[low].c)) != OR_OK) goto done;
        }
    }
done:
    if (R) for (int64_t j = 0; j < nf; ++j) free(R[j].v);
    free(R); free(facs); free(tops); free(tpos); free(pivot);
    return rc;
}

/* ----------------------------------------------------------- output ordering -- */

static const grid_t *g_sort_grid;   /* comparator context (qsort has none) */

static int cmp_pair(const void *a, const void *b) {
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    if (x->dim != y->dim) return x->dim < y->dim ? -1 : 1;
    ckey_t kx = key_of(g_sort_grid, x->birth_cell), ky = key_of(g_sort_grid, y->birth_cell);
    return cmp_ckey(&kx, &ky);
}

/* T-filtration order: dimension, then the death cell's key, essential classes last. */
static int cmp_pair_t(const void *a, const void *b) {
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    if (x->dim != y->dim) return x->dim < y->dim ? -1 : 1;
    if ((x->death_cell < 0) != (y->death_cell < 0)) return x->death_cell < 0 ? 1 : -1;
    if (x->death_cell < 0) return 0;
    ckey_t kx = key_of(g_sort_grid, x->death_cell), ky = key_of(g_sort_grid, y->death_cell);
    return cmp_ckey(&kx, &ky);
}

/* ------------------------------------------------------------------ entry ---- */

static int diagram(const float *img, int32_t ndim, const int64_t *ext, uint32_t dims_mask,
                   int32_t method, int32_t keep_zero, int tmode, or_pair **out, int64_t *count) {
    *out = NULL;
    *count = 0;
    if (!img || !ext || (ndim != 2 && ndim != 3)) return OR_EINVAL;
    grid_t g;
    memset(&g, 0, sizeof g);
    g.ndim = ndim;
    g.tmode = tmode;
    g.e[0] = 1;
    for (int k = 0; k < ndim; ++k) {
        if (ext[k] < 1) return OR_EINVAL;
        g.e[3 - ndim + k] = ext[k];
    }
    if (ndim == 2) g.e[0] = 1;
    g.nvox = g.e[0] * g.e[1] * g.e[2];
    for (int k = 0; k < 3; ++k) g.d[k] = tmode ? 2 * g.e[k] + 1 : 2 * g.e[k] - 1;
    if (tmode && ndim == 2) g.d[0] = 1;
    g.ncell = g.d[0] * g.d[1] * g.d[2];
    g.img = img;
    for (int64_t i = 0; i < g.nvox; ++i)
        if (isnan(img[i])) return OR_ENAN;

    int rc = build_vertex_ranks(&g);
    if (rc != OR_OK) return rc;
    plist_t L = {0, 0, 0};
    if (method == OR_FULL) {
        rc = reduce_full(&g, dims_mask, keep_zero, &L);
    } else if (method == OR_SPLIT) {
        for (int p = 0; p < ndim && rc == OR_OK; ++p) {
            if (!((dims_mask >> p) & 1u)) continue;
            if (p == ndim - 1 && p > 0) rc = reduce_coboundary_top(&g, ndim, dims_mask, keep_zero, &L);
            else rc = reduce_boundary_block(&g, p, dims_mask, keep_zero, &L);
        }
    } else {
        rc = OR_EINVAL;
    }
    if (rc == OR_OK && L.n > 1) {
        g_sort_grid = &g;
        qsort(L.p, (size_t)L.n, sizeof(or_pair), tmode ? cmp_pair_t : cmp_pair);
        g_sort_grid = NULL;
    }
    free(g.vrank);
    if (rc != OR_OK) { free(L.p); return rc; }
    *out = L.p;
    *count = L.n;
    return OR_OK;
}

int or_diagram(const float *img, int32_t ndim, const int64_t *ext, uint32_t dims_mask,
               int32_t method, int32_t keep_zero, or_pair **out, int64_t *count) {
    return diagram(img, ndim, ext, dims_mask, method, keep_zero, 0, out, count);
}

int or_diagram_t(const float *img, int32_t ndim, const int64_t *ext, uint32_t dims_mask,
                 int32_t method, int32_t keep_zero, or_pair **out, int64_t *count) {
    return diagram(img, ndim, ext, dims_mask, method, keep_zero, 1, out, count);
}

void or_free(void *p) { free(p); }

/* Reference gradient: g = 0, then, in output order, the birth gradient of every pair goes
 * to its birth vertex and the death gradient of every pair with a finite death goes to its
 * death vertex (FP32 accumulation). */
int or_gradient(const or_pair *pairs, int64_t n, const float *grad_birth,
                const float *grad_death, float *grad_img, int64_t nvox) {
    for (int64_t i = 0; i < nvox; ++i) grad_img[i] = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        if (pairs[i].birth_vertex < 0 || pairs[i].birth_vertex >= nvox) return OR_EINVAL;
        grad_img[pairs[i].birth_vertex] += grad_birth[i];
        if (pairs[i].death_vertex >= 0) {
            if (pairs[i].death_vertex >= nvox) return OR_EINVAL;
            grad_img[pairs[i].death_vertex] += grad_death[i];
        }
    }
    return OR_OK;
}
