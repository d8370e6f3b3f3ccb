/*
 * flashcubical.h -- C ABI of the gfx950 library for V-filtration cubical persistence over F2
 * on 2D images and 3D volumes (H0 and the top dimension: H1 for images, H2 for volumes).
 *
 * Method (Le Breton, Szustakowski, Piraud, "Fast Cubical Persistent Homology on 2D and 3D
 * Images via Union-Find, Pruning, and Lookup Tables"):
 *   - cells, V-filtration and persistence pairs as defined in Sec. 2.1-2.2;
 *   - the fully refined order of Sec. 2.3: a cell is ordered by its last-entering vertex
 *     (pixel value, then row-major pixel index), then by dimension, then by its index on
 *     the doubled grid; pairs of equal birth and death value are not reported;
 *   - lookup-table classification and pruning of each vertex's lower star (Sec. 3.2, 3.3),
 *     union-find for H0 and union-find on the dual graph with a cell at infinity for the top
 *     dimension (Sec. 3.1, Appendix A), as assembled in Sec. 4.1 (2D) and Sec. 4.2 steps 1-3
 *     (3D), and with PH_H1 the middle dimension of a volume (Sec. 4.2 steps 4-5).  A volume
 *     with an extent of 1 is still a volume (empty H2; its H1 needs PH_H1).
 *
 * Conventions shared by every entry point:
 *   - Pixel layout: row-major, last axis fastest.  2D extents are (H, W), 3D (D, H, W); every
 *     extent >= 1, and the voxel count of one instance is at most 2^27 (a 512^3 volume; under
 *     PH_TFILT the framed extents, each + 2, count).
 *   - pixidx: row-major pixel index.  Cell index: row-major index on the doubled grid
 *     (2H-1, 2W-1) or (2D-1, 2H-1, 2W-1), a coordinate being odd where the cell spans that
 *     axis.
 *   - Output pairs, per instance, are sorted by (dim, birth cell in the refined order):
 *     H0 first (its essential class, death = +inf, death_cell = death_vertex = -1, is the
 *     first pair), then the top dimension.  birth and death are bit copies of input pixels.
 *   - Memory: every pointer named d_* is device memory owned by the caller; h_* is host
 *     memory.  The library allocates nothing per call.  It owns only its lookup tables,
 *     built on the host and copied once per device on first use into device buffers it
 *     keeps until the process ends (about 1.2 MB per device), and the workspace array of
 *     ph_diagram_noalloc (PH_NOALLOC_SCRATCH_MIB per device, part of its code object).
 *   - Streams: all work is enqueued on `stream`.  ph_diagram, ph_diagram_batch and
 *     ph_backward never synchronise with the host, so a sequence of them can be captured in a
 *     HIP graph; results are valid once the stream has reached them.  ph_autotune and the
 *     inspection helpers do wait.
 *   - Errors: argument errors found on the host are returned synchronously (PH_EINVAL,
 *     PH_ENOMEM for a too-small workspace, PH_EHIP for a failed HIP call).  Errors found
 *     by the kernels are written to the per-instance status word (PH_ENAN for a NaN pixel,
 *     PH_ECAPACITY when the pairs exceed the capacity: the true count is still written and
 *     the first `capacity` pairs in output order are stored, PH_ELISTS when the lists outgrow
 *     a PH_LIST_FRACTION, PH_EINTERNAL if a bounded loop ran out of iterations).
 *   - Calls that share a workspace must not overlap in time.
 *   - FLASHCUBICAL_TRACE=1 in the environment names every kernel launch on stderr and waits
 *     for it (a debugging aid: it synchronises, so it must not be set during graph capture).
 */
#ifndef FLASHCUBICAL_H
#define FLASHCUBICAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PH_OK = 0,
    PH_EINVAL = -1,
    PH_ENAN = -2,
    PH_ECAPACITY = -3,
    PH_ENOMEM = -4,
    PH_EHIP = -5,
    PH_EINTERNAL = -6,
    PH_ELISTS = -7
};

/* flags: which dimensions to report (H0 is always computed; 2D needs it for the top), and the
 * element type of the input (float32 unless one of PH_IN_U8, PH_IN_U16 is set; setting both
 * is PH_EINVAL).  An integer input gives bitwise the results of the same values as float32
 * (every 8- and 16-bit integer is exactly a float32); it reads 1 or 2 bytes per voxel and
 * always uses the default tiles.
 *
 * PH_TFILT selects the T-filtration (paper Sec. 2.2, its dual construction; the extension
 * the paper's Sec. 6 names): the pixels are the top cells of a complex on (n+1) vertices per
 * axis, and a cell enters with the first top cell that contains it (value = minimum over the
 * top cells containing it; ties go to the smaller pixel index, then lower dimension, then
 * smaller doubled-grid index).  By Alexander duality this complex is the dual cell complex of
 * the V complex of the negated, point-reflected image framed by one ring of -inf pixels:
 * the library computes that V diagram with the same kernels and maps every pair back (the
 * dual of a T pair (s, t) of dimension k is the V pair (t*, s*) of dimension d-1-k).  Under
 * PH_TFILT:
 *   - PH_H0 / PH_HTOP name the T dimensions; both V dimensions are always computed;
 *   - cells are indices on the T doubled grid, extents 2n+1 per axis (1 on the leading axis
 *     of an image); pixel (i, j[, k]) is the top cell (2i+1, 2j+1[, 2k+1]); birth_vertex /
 *     death_vertex name the pixel whose value the cell takes;
 *   - pairs come by dimension, then by the death cell's position in the filtration order,
 *     the essential class last;
 *   - a +inf pixel is reported as PH_ENAN (it would tie the frame);
 *   - ph_capacity_bound and ph_workspace_bytes of the same flags account for the frame: pass
 *     the shape with every extent grown by 2 to ph_capacity_bound (ph_capacity_bound_flags
 *     does it itself).
 *
 * PH_H1 adds H1 of every volume of the call (Sec. 4.2 steps 4-5; images ignore it, their H1
 * is the top dimension).  The cells left unpaired by the lookup table, the H0 union-find and
 * the dual union-find form a reduced problem: rows are the KEEP edges H0 left positive,
 * columns the KEEP squares the dual union-find left unpaired.  Each column is first expressed
 * in those rows by adding the reduced columns the table knows for every pair inside one lower
 * star (legal column operations: each added column precedes the column), then the columns are
 * reduced over F2 in square order.  The H1 pairs of non-zero persistence are reported between
 * H0 and H2, in the same order and with the same fields as the other dimensions (under
 * PH_TFILT: the T-filtration's H1, by duality, by death key).  Internal limits (a column's
 * running sum beyond 2048 live edges (columns beyond 512 take a second pass with larger
 * tables), its boundary in critical cells beyond 64 edges, the columns' pool beyond 4 entries
 * per KEEP-square slot) are reported as PH_EINTERNAL.  Volumes
 * run the 3D classify pass on the default tiles under PH_H1. */
enum { PH_H0 = 1, PH_HTOP = 2, PH_IN_U8 = 4, PH_IN_U16 = 8, PH_TFILT = 16, PH_H1 = 32, PH_WIDE = 64 };

/* PH_WIDE (not in the paper, a scheduling choice): the union-finds (H0 and the top dimension)
 * of an instance of 2^20 or more voxels with more than 20,440 nodes (too many for one
 * workgroup's LDS) start with 16 of their parallel rounds spread over the whole GPU (two
 * launches a round), then finish in one workgroup as without the flag.  The pairs are the
 * same.  It pays for inputs with many critical cells (noise: about a sixth of the pixels are
 * H0 nodes); a smooth field rarely has that many nodes, and then the extra launches (a few
 * microseconds each) are spent for nothing. */

/* List fraction (flags bits 8-15; not in the paper, a sizing choice).  The workspace holds, per
 * instance, the lists of cells that survive pruning (KEEP edges, KEEP squares, H0 nodes, dual
 * nodes) and the sort, union-find and H1 arrays sized by them.  By default every list is sized
 * for the worst case (every edge kept), which never overflows but costs about 160 B per pixel
 * for images and 240 B per voxel for volumes.  PH_LIST_FRACTION(k), k = 1..255, sizes each list
 * to k/256 of its worst case (at least 4096 entries, never more than the worst case); the
 * per-pixel arrays (forest links) keep their size.  Smooth fields keep well under 1 % of their
 * cells, so PH_LIST_FRACTION(1) fits them in a tenth of the workspace; noise keeps about a sixth
 * of the edges.  Pass the same flags to ph_workspace_bytes and to the call.  An instance whose
 * lists outgrow their capacities gets the status PH_ELISTS and no pairs; ph_work_counters
 * still reports its true list sizes (KEEP edges, KEEP squares, H0 nodes, dual nodes), from which
 * a sufficient fraction follows.  Results that fit are bitwise those of the worst-case sizing. */
#define PH_LIST_FRACTION(k) ((uint32_t)((k) & 0xFF) << 8)

typedef struct {
    int32_t ndim;       /* 2 or 3 */
    int32_t ext[3];     /* extents, slowest first; ext[2] unused when ndim == 2 */
} ph_shape;

/* Structure-of-arrays output, device pointers, caller-owned.  Each array holds at least the
 * capacity of the call (sum of capacities for a batch). */
typedef struct {
    int8_t *dim;            /* homology dimension: 0, ndim-1, or 1 for a volume under PH_H1 */
    float *birth;           /* value of the birth cell */
    float *death;           /* value of the death cell; +inf for the essential class */
    int64_t *birth_cell;    /* doubled-grid index of the birth cell */
    int64_t *death_cell;    /* doubled-grid index of the death cell; -1 if essential */
    int32_t *birth_vertex;  /* pixel giving the birth cell its value (its last vertex) */
    int32_t *death_vertex;  /* same for the death cell; -1 if essential */
} ph_pairs;

/* Optional launch tuning; NULL picks the autotuned choice for the batch's size class (see
 * ph_autotune), else the defaults.
 * The choice never changes results, only speed. */
typedef struct {
    int32_t tile2d;     /* 0: 64x16, 1: 32x32, 2: 128x8 vertices per workgroup */
    int32_t tile3d;     /* 0: 16x8x8, 1: 32x8x4, 2: 8x8x16 (x, y, z) voxels per workgroup */
} ph_tuning;

/* Upper bound of the pairs of one instance: pixels + top cells (H0 pairs <= pixels, top
 * pairs <= top cells).  A capacity of this size can never overflow. */
int64_t ph_capacity_bound(ph_shape shape);

/* The same bound for a call with the given flags: under PH_TFILT that of the framed dual image
 * (every extent + 2), and under PH_H1 a volume's H1 pairs are added (at most its squares
 * minus its cubes).  0 for an invalid shape. */
int64_t ph_capacity_bound_flags(ph_shape shape, uint32_t flags);

/* Workspace bytes needed by a batch of n instances with the given host shapes (also valid
 * for n = 1 and ph_diagram) under the given flags (PH_TFILT: the framed extents; PH_H1: the
 * volumes' H1 arrays; PH_LIST_FRACTION(k): the lists at k/256 of their worst case).
 * Returns 0 for invalid shapes. */
size_t ph_workspace_bytes(const ph_shape *h_shapes, int32_t n, uint32_t flags);

/* Persistence diagram of one image or volume (Sec. 4.1 / Sec. 4.2 steps 1-3).
 *   d_img     : device, row-major pixels of `shape`, of the element type the flags name.
 *   out       : device SoA arrays with room for `capacity` pairs.
 *   d_count   : device int64, receives the number of pairs (even beyond capacity).
 *   d_status  : device int32, receives PH_OK or a kernel-detected error.
 *   d_ws      : device workspace of ws_bytes >= ph_workspace_bytes(&shape, 1, flags).
 * Returns PH_OK when the work was enqueued. */
int ph_diagram(const void *d_img, ph_shape shape, uint32_t flags, ph_pairs out,
               int64_t capacity, int64_t *d_count, int32_t *d_status, void *d_ws,
               size_t ws_bytes, void *stream);

/* ph_diagram for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Arguments and results as for
 * ph_diagram, without a workspace argument: the workspace is a library-owned device array of
 * PH_NOALLOC_SCRATCH_MIB MiB per device, set up (its device address taken, the tables
 * uploaded) by ph_init_device, which must have run on the current device first; the array
 * lives until the process ends.  The call itself allocates nothing (no hipMalloc, hipFree,
 * host heap), writes no memset, and never waits for the stream.
 * Errors: PH_EINVAL if ph_init_device has not run on the current device, PH_ENOMEM (with a
 * message on stderr) if ph_workspace_bytes(&shape, 1, flags) exceeds the array; otherwise as
 * ph_diagram.  Every call on one device shares that device's array and leaves its contents
 * behind (the kernels clear what must start at zero): calls that overlap in time on one
 * device, on any streams, race and must not be made. */
#define PH_NOALLOC_SCRATCH_MIB 64
int ph_diagram_noalloc(const void *d_img, ph_shape shape, uint32_t flags, ph_pairs out,
                       int64_t capacity, int64_t *d_count, int32_t *d_status, void *stream);

/* Diagrams of n instances (1 <= n <= 65535) of uneven sizes and mixed 2D/3D in one set of launches:
 * persistent kernels walk a per-instance table built on the device from d_shapes.
 *   d_imgs     : all pixels concatenated (element type as the flags name); instance i
 *                starts at element d_img_off[i].
 *   d_shapes   : device copy of h_shapes (n entries); h_shapes sizes the launch grids.
 *   out        : shared SoA output; instance i writes from element d_out_off[i] and has
 *                capacity d_out_off[i+1] - d_out_off[i] (d_out_off has n+1 entries).
 *   d_counts, d_status : n entries each.
 *   tuning     : NULL = default/autotuned tiles.
 * The pairs of each instance are bitwise those of a single ph_diagram call on it. */
int ph_diagram_batch(int32_t n, const void *d_imgs, const int64_t *d_img_off,
                     const ph_shape *d_shapes, const ph_shape *h_shapes, uint32_t flags,
                     ph_pairs out, const int64_t *d_out_off, int64_t *d_counts,
                     int32_t *d_status, const ph_tuning *tuning, void *d_ws, size_t ws_bytes,
                     void *stream);

/* ph_diagram_batch that also clears the gradient buffer a later ph_backward_scatter fills (not
 * part of the paper: the zero fill of ph_backward, moved into the classify passes, which visit
 * every pixel anyway).
 *   d_grad_img : device float32, packed like d_imgs (instance i from element d_img_off[i]);
 *                every pixel of every instance is set to 0.0f, in the caller's layout also
 *                under PH_TFILT; elements outside the instances are left as they are.
 * Otherwise (arguments, pairs, errors) as ph_diagram_batch; PH_EINVAL if d_grad_img is null.
 * After an error return the buffer may be cleared in part or not at all. */
int ph_diagram_batch_grad(int32_t n, const void *d_imgs, const int64_t *d_img_off,
                          const ph_shape *d_shapes, const ph_shape *h_shapes, uint32_t flags,
                          ph_pairs out, const int64_t *d_out_off, int64_t *d_counts,
                          int32_t *d_status, const ph_tuning *tuning, void *d_ws, size_t ws_bytes,
                          float *d_grad_img, void *stream);

/* Autotuner (not part of the paper): runs the batch once per candidate tile choice (the 2D
 * choices if the batch holds images, the 3D ones if it holds volumes), one warm-up and `reps`
 * timed runs each, writes the fastest to *best and remembers it for the batch's size class
 * (which dimensions it holds and the binary order of magnitude of its mean instance size):
 * later ph_diagram_batch calls with tuning == NULL in that class use it.  Arguments as for
 * ph_diagram_batch; the outputs hold the last run's results.  Waits for the stream (not for
 * use during graph capture).  Tile choices never change results, only speed.  With an integer
 * input (PH_IN_U8, PH_IN_U16) or PH_TFILT it runs the batch once on the default tiles, writes
 * those to *best and records nothing (a T batch with tuning == NULL takes the defaults). */
int ph_autotune(int32_t n, const void *d_imgs, const int64_t *d_img_off, const ph_shape *d_shapes,
                const ph_shape *h_shapes, uint32_t flags, ph_pairs out, const int64_t *d_out_off,
                int64_t *d_counts, int32_t *d_status, void *d_ws, size_t ws_bytes, int32_t reps,
                ph_tuning *best, void *stream);

/* Gradient of pair values with respect to the pixels (not part of the paper; 1 <= n <= 65535): for every
 * stored pair j of instance i, d_grad_birth[j] is added to the birth pixel and, if the death
 * is finite, d_grad_death[j] to the death pixel; all other pixels get 0.
 *   pairs, d_counts : as written by ph_diagram(_batch) for n instances.
 *   d_out_off  : device, n+1 entries: instance i's pairs (and gradients) are entries
 *                [d_out_off[i], d_out_off[i+1]); counts beyond that capacity are clamped.
 *   d_grad_img : device float32, total_voxels entries, instance i from d_img_off[i]
 *                (device, n entries).  Overwritten.
 * Additions to one pixel are atomic, so their rounding order is not fixed. */
int ph_backward(int32_t n, ph_pairs pairs, const int64_t *d_out_off, const int64_t *d_counts,
                const float *d_grad_birth, const float *d_grad_death, float *d_grad_img,
                const int64_t *d_img_off, int64_t total_voxels, void *stream);

/* ph_backward without its zero fill (not part of the paper): the pair gradients are added to
 * d_grad_img as it stands, so it must hold zeros first, as ph_diagram_batch_grad leaves it;
 * pixels no pair names keep their value.  Arguments and errors as ph_backward; the result on a
 * buffer so cleared is bitwise that of ph_backward. */
int ph_backward_scatter(int32_t n, ph_pairs pairs, const int64_t *d_out_off, const int64_t *d_counts,
                        const float *d_grad_birth, const float *d_grad_death, float *d_grad_img,
                        const int64_t *d_img_off, int64_t total_voxels, void *stream);

/* Host-side view of the lookup table (Sec. 3.3), for inspection and tests.
 * ndim 2: raw_mask has 8 bits (neighbours up, left, right, down, up-left, up-right,
 * down-left, down-right); ndim 3: 26 bits, neighbour at offset code k+1 of the local cell
 * list (offsets ordered by number of non-zero coordinates, then lexicographically, slowest
 * axis first).  Bit set = that neighbour precedes the vertex.  *entry receives the
 * classification of the vertex's lower star L(v) by the relative reduction of L(v):
 *   2D (edges i = 0..3: up, left, right, down; squares q = 0..3: quadrant bits
 *   (dy > 0) << 1 | (dx > 0)):
 *     bits 0-2   edge paired with the vertex (7: none, the vertex is a local minimum)
 *     bits 3-6   KEEP edges (unpaired inside L(v))
 *     bits 7-10  squares of L(v)
 *     bits 11-14 ROOT squares (unpaired inside L(v))
 *     bits 15-22 for each other square q of L(v), 2 bits at 15 + 2q: quadrant of the other
 *                cofacet of the edge that q is paired with
 *   3D (edges i = 0..5 at codes 1..6; squares s = 0..11 at codes 7..18; cubes c = 0..7:
 *   octant bits (dz > 0) << 2 | (dy > 0) << 1 | (dx > 0)):
 *     bits 0-2   edge paired with the vertex (7: none)
 *     bits 3-8   KEEP edges
 *     bits 9-20  KEEP squares
 *     bits 21-28 ROOT cubes
 *     bits 29-52 for each other cube c of L(v), 3 bits at 29 + 3c: octant of the other
 *                cofacet of the square that c is paired with
 *     bits 53-60 cubes of L(v)
 * Returns PH_OK or PH_EINVAL. */
int ph_lut_entry(int32_t ndim, uint32_t raw_mask, uint64_t *entry);

/* Number of distinct lower-star configurations after collapsing irrelevant diagonal
 * neighbours (Sec. 3.3): 47 for 2D, 15935 for 3D. */
int32_t ph_lut_config_count(int32_t ndim);

/* Upload the lookup tables to the current device now (they are otherwise uploaded on first
 * use), verify the device copy, and take the device address of the workspace array of
 * ph_diagram_noalloc; PH_OK, PH_EHIP or PH_EINTERNAL. */
int ph_init_device(void);

/* Text report (into buf, len bytes) of the current device's per-block LDS and thread limits
 * and each kernel's static LDS, registers and launch size; returns PH_OK when every kernel
 * fits, PH_EHIP otherwise.  Launches nothing. */
int ph_device_report(char *buf, size_t len);

/* Per-kernel timing.  ph_profile(1) clears earlier records and makes every following launch
 * of this library record a pair of HIP events around it on its stream; ph_profile(0) stops
 * recording.  Not for use while a stream is being captured into a graph.
 * ph_profile_read waits for the recorded events, writes up to max per-kernel totals (kernels in
 * launch-pipeline order, only those launched), sets *count to the number of kernels seen, and
 * clears the records.  Returns PH_OK, PH_EINVAL or PH_EHIP. */
typedef struct {
    char name[32];
    int32_t launches;
    double total_ms;
} ph_kernel_time;
int ph_profile(int32_t enable);
int ph_profile_read(ph_kernel_time *out, int32_t max, int32_t *count);

/* Work counters of the last call that used workspace d_ws for n instances (the same n), for
 * sizing and diagnostics: 16 int32 per instance written to h_out (host), in order KEEP edges,
 * KEEP squares (3D), H0 nodes (local minima), dual nodes (ROOT top cells + the cell at
 * infinity), H0 union-find rounds, dual union-find rounds, edges finished sequentially, the
 * instance's error word, and under PH_H1: H1 columns, columns reduced one by one (their
 * lowest row occurs in an earlier column), the most steps one column's expression in
 * critical cells took, the pool entries used, the columns that needed the large tables, and
 * the reduction's rounds (or, when it ran one column at a time, its column additions); then
 * the forest links followed to resolve the KEEP edges' endpoints (H0) and the facets'
 * cofacets (top dimension).  Copies synchronously; PH_OK, PH_EINVAL or PH_EHIP. */
int ph_work_counters(const void *d_ws, int32_t n, int32_t *h_out);

/* Library version string. */
const char *ph_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FLASHCUBICAL_H */
