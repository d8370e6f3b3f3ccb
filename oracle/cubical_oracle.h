/* cubical_oracle.h -- TEST INFRASTRUCTURE ONLY: plain CPU reference for V- and T-filtration
 * cubical persistence over F2.  Not part of, and never linked into, the GPU library. */
#ifndef CUBICAL_ORACLE_H
#define CUBICAL_ORACLE_H
#include <stdint.h>

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENAN = -2, OR_ENOMEM = -4 };
enum { OR_FULL = 0, OR_SPLIT = 1 };

typedef struct {
    int32_t dim;            /* homology dimension of the pair */
    float birth;            /* value of the birth cell (copy of a pixel value) */
    float death;            /* value of the death cell, +inf for an essential class */
    int64_t birth_cell;     /* doubled-grid linear index of the birth cell */
    int64_t death_cell;     /* doubled-grid linear index of the death cell, -1 if essential */
    int32_t birth_vertex;   /* pixel index of the birth cell's last-entering vertex */
    int32_t death_vertex;   /* same for the death cell, -1 if essential */
} or_pair;

/* img: row-major pixels, ext[ndim] extents (slowest first).  dims_mask bit p asks for H_p.
 * On success *out holds *count pairs sorted by (dim, birth key); free with or_free. */
int or_diagram(const float *img, int32_t ndim, const int64_t *ext, uint32_t dims_mask,
               int32_t method, int32_t keep_zero, or_pair **out, int64_t *count);
/* The same for the T-filtration (pixels are the top cells); pairs sorted by (dim, death
 * key), essential classes last; birth_vertex / death_vertex name the pixel whose value the
 * cell takes. */
int or_diagram_t(const float *img, int32_t ndim, const int64_t *ext, uint32_t dims_mask,
                 int32_t method, int32_t keep_zero, or_pair **out, int64_t *count);
void or_free(void *p);
int or_gradient(const or_pair *pairs, int64_t n, const float *grad_birth,
                const float *grad_death, float *grad_img, int64_t nvox);
#endif
