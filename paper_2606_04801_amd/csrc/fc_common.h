// fc_common.h -- definitions shared by the host code and the gfx950 kernels of the library.
//
// Local cells.  The lower star L(v) of a vertex v (paper Sec. 2.3) is made of cells of the
// doubled grid at offsets delta in {-1,0,1}^3 from 2v.  The 27 offsets are numbered by a
// "code" in the order the refined filtration uses inside one lower star: by dimension, then
// lexicographically with the slowest axis first (which is the doubled-grid index order).
//   code 0      : the vertex itself
//   codes 1..6  : edges   (-1,0,0) (0,-1,0) (0,0,-1) (0,0,1) (0,1,0) (1,0,0)
//   codes 7..18 : squares with two non-zero coordinates, lexicographic
//   codes 19..26: cubes (+-1,+-1,+-1), lexicographic; cube index c = code-19 is the octant
//                 bits (dz>0)<<2 | (dy>0)<<1 | (dx>0)
// A 2D image is the plane dz = 0: edges codes 2..5 (up, left, right, down), squares codes
// 11..14 (up-left, up-right, down-left, down-right); square index q = code-11 is the
// quadrant bits (dy>0)<<1 | (dx>0).
//
// Cell keys.  Every cell is named by a 64-bit key
//     ord32(f(v)) << 32 | pixidx(v) << 5 | code
// where v is the cell's last-entering vertex.  Unsigned comparison of keys of one instance
// is exactly the fully refined order of Sec. 2.3 restricted to one dimension; ord32 is a
// monotone map of float32 bits to uint32 with -0 mapped like +0.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define FC_HD __host__ __device__ __forceinline__
#else
#define FC_HD inline
#endif

namespace fc {

constexpr int kCodeBits = 5;
constexpr int kPixBits = 27;                       // pixel index field: voxels per instance <= 2^27
constexpr uint64_t kPixMask = (1ull << kPixBits) - 1;

// offsets (dz, dy, dx) of the 27 local cells, in code order
constexpr int8_t kOff[27][3] = {
    {0, 0, 0},
    {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {0, 0, 1}, {0, 1, 0}, {1, 0, 0},
    {-1, -1, 0}, {-1, 0, -1}, {-1, 0, 1}, {-1, 1, 0}, {0, -1, -1}, {0, -1, 1},
    {0, 1, -1}, {0, 1, 1}, {1, -1, 0}, {1, 0, -1}, {1, 0, 1}, {1, 1, 0},
    {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}, {1, -1, 1},
    {1, 1, -1}, {1, 1, 1}};

// Offsets as arithmetic on packed constants (2 bits per code and axis), so device code needs
// no table in memory: off_of(code, axis) = kOff[code][axis].
constexpr uint64_t pack_axis(int a) {
    uint64_t k = 0;
    for (int c = 0; c < 27; ++c) k |= (uint64_t)(kOff[c][a] + 1) << (2 * c);
    return k;
}
constexpr uint64_t kOffPackZ = pack_axis(0), kOffPackY = pack_axis(1), kOffPackX = pack_axis(2);
FC_HD int off_of(int code, int axis) {
    const uint64_t k = axis == 0 ? kOffPackZ : (axis == 1 ? kOffPackY : kOffPackX);
    return (int)((k >> (2 * code)) & 3u) - 1;
}

FC_HD uint32_t ord32(uint32_t u) {
    if (u == 0x80000000u) u = 0;                   // -0 ranks with +0
    return (u >> 31) ? ~u : (u | 0x80000000u);
}
// ord32 of the bits of a float that is not -0: a float plus +0.0 (which turns -0 into +0 and
// leaves every other value, subnormals and NaNs included, as it was) qualifies
FC_HD uint32_t ord32_no_neg0(uint32_t u) { return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u); }

FC_HD uint64_t make_key(uint32_t ord, uint32_t pix, uint32_t code) {
    return ((uint64_t)ord << 32) | ((uint64_t)pix << kCodeBits) | code;
}
FC_HD uint32_t key_pix(uint64_t k) { return (uint32_t)((k >> kCodeBits) & kPixMask); }
FC_HD uint32_t key_code(uint64_t k) { return (uint32_t)(k & 31u); }
FC_HD uint32_t key_ord(uint64_t k) { return (uint32_t)(k >> 32); }

// ---------------------------------------------------------------- LUT entry layouts --
// 2D entry (uint32), indexed by the raw 8-bit neighbour mask:
//   [0:3)   direct edge index 0..3 (edge code 2+i), 7 = none (v is a local minimum)
//   [3:7)   KEEP edges (critical in L(v), go to the H0 union-find)
//   [7:11)  squares present in L(v)
//   [11:15) ROOT squares (critical: dual union-find nodes)
//   [15:23) link quadrant of each non-ROOT square, 2 bits per square
// 3D entry (uint64), found through the two-level index below:
//   [0:3)   direct edge index 0..5 (edge code 1+i), 7 = none
//   [3:9)   KEEP edges
//   [9:21)  KEEP squares (critical: go to the dual union-find)
//   [21:29) ROOT cubes
//   [29:53) link octant of each non-ROOT cube, 3 bits per cube
//   [53:61) cubes present in L(v)
constexpr uint32_t kNoDirect = 7;
constexpr int kL2Keep = 3, kL2Present = 7, kL2Root = 11, kL2Link = 15;
constexpr int kL3Keep = 3, kL3KeepSq = 9, kL3Root = 21, kL3Link = 29, kL3Present = 53;
constexpr int kL3Configs = 15935;
constexpr int kL2Configs = 47;

// 3D two-level index.  Level 1 is indexed by (6 face bits | 12 square bits << 6) of the raw
// neighbour mask and holds (base << 8 | possible-cube mask) of the canonical configuration
// (squares kept only where both faces are present); level 2 at base + (the raw cube bits
// compressed through the possible mask) holds the entry.
constexpr int kL1Size = 1 << 18;

// square index s = code-7: the two face (edge) indices it spans
constexpr int8_t kSqFace[12][2] = {{0, 1}, {0, 2}, {0, 3}, {0, 4}, {1, 2}, {1, 3},
                                   {2, 4}, {3, 4}, {5, 1}, {5, 2}, {5, 3}, {5, 4}};
// cube index c: its three square indices
constexpr int8_t kCubeSq[8][3] = {{0, 1, 4}, {0, 2, 5}, {3, 1, 6}, {3, 2, 7},
                                  {8, 9, 4}, {8, 10, 5}, {11, 9, 6}, {11, 10, 7}};

// ---------------------------------------------------------- per-instance geometry --
struct Geom {
    int64_t N;      // vertices
    int64_t E;      // edges
    int64_t S;      // squares
    int64_t C;      // cubes
    int64_t T;      // top cells (squares in 2D, cubes in 3D)
    int64_t F;      // facet list capacity kept apart from the edges (3D squares, 2D none)
    int64_t FAC;    // facets walked by the dual union-find (2D edges, 3D squares)
};

FC_HD Geom geom(int ndim, int64_t D, int64_t H, int64_t W) {
    Geom g;
    g.N = D * H * W;
    g.E = (D - 1) * H * W + D * (H - 1) * W + D * H * (W - 1);
    g.S = (D - 1) * (H - 1) * W + (D - 1) * H * (W - 1) + D * (H - 1) * (W - 1);
    g.C = (D - 1) * (H - 1) * (W - 1);
    if (ndim == 2) { g.T = (H - 1) * (W - 1); g.F = 0; g.FAC = g.E; }
    else { g.T = g.C; g.F = g.S; g.FAC = g.S; }
    return g;
}

// Instance descriptor, built on the device by the plan kernel (and on the host for sizing).
struct Inst {
    int32_t ndim, D, H, W;
    int64_t N, T, E, F, FAC;
    int64_t src_off;           // offset of the instance's pixels in the caller's input (elements)
    int64_t out_off, out_cap;
    int64_t tile_base;         // first tile of this instance in its (2D or 3D) classify grid
    int32_t tx, ty, tz;        // tiles along x, y, z
    int32_t tfilt;             // 1: T-filtration, the grid is the framed dual image (extents + 2),
                               // read from the caller's pixels on the fly (see tf_value)
    int32_t h1;                // 1: a volume whose H1 is computed too (Sec. 4.2 steps 4-5)
    int32_t lists;             // list capacities in 1/256 of the worst case (0: the worst case)
    int64_t M0cap, MTcap;      // capacities of the H0 and dual node lists (worst: N, T + 1)
    // byte offsets of the per-instance arrays inside the workspace
    int64_t o_par0, o_parT, o_keyE, o_ea, o_eb, o_neg0, o_keyF, o_fa, o_fb, o_killer;
    int64_t o_n0key, o_n0sorted, o_nTkey, o_uf0, o_moe0, o_death0, o_ufT, o_moeT;
    int64_t o_live, o_live2, o_ra, o_rb, o_scratch;
    // H1 of a volume: per-vertex configuration index and first sorted KEEP edge, per KEEP
    // square its H1 column (start and length in the pool, -1 if paired in H2), per KEEP edge
    // its pivot column and the first column holding it, and the pool of column entries
    int64_t o_cfg3, o_kpos, o_h1b, o_h1n, o_piv, o_first, o_pool, o_retry;
    int64_t pool_cap;          // int32 entries of the pool
    int64_t end;
};

// counters per instance (int32 each).  The four list counters that every classify tile
// advances with an atomic each sit on cache lines of their own (128 B apart), so the atomics
// of one tile, and of the tiles of one instance, do not queue behind each other on one line.
enum {
    CNT_E = 0, CNT_F = 32, CNT_M0 = 64, CNT_MT = 96,
    CNT_ERR = 128, CNT_ROUNDS0, CNT_ROUNDST, CNT_SEQ,
    CNT_H1COLS, CNT_H1UNSAFE, CNT_H1ROUNDS, CNT_H1RETRY, CNT_H1ADDS, CNT_HOPS0, CNT_HOPST,
    CNT_WLIVE0 = 144, CNT_WLIVET = 146,  // wide union-find rounds: live edges of a round, two slots by parity
    CNT_OSEC0 = 148, CNT_OSECT,          // wide output: pairs of the H0 and the top-dimension lists
    CNT_H1POOL = 160, CNT_WORDS = 192
};
// pool entries per KEEP-square slot of an H1 volume: room for the Morse boundaries of the
// columns (a few entries each) and the reduced forms of the columns that need reduction
constexpr int64_t kH1PoolPerSquare = 4;

FC_HD int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Capacity of a list whose worst case is `worst` entries, under a list fraction of k / 256
// (k = 0: the worst case): at least kListFloor entries, never above the worst case.
constexpr int64_t kListFloor = 4096;
FC_HD int64_t list_cap(int64_t worst, int k) {
    if (k <= 0 || worst <= kListFloor) return worst;
    const int64_t c = (worst * k + 255) / 256;
    return c < kListFloor ? kListFloor : (c > worst ? worst : c);
}

// Unused bytes left after every workspace array (0 in the library; the CPU emulation build of
// the tests sets it so that a run past the end of an array lands in poisoned memory).
#ifndef FC_ARRAY_GAP
#define FC_ARRAY_GAP 0
#endif

// Fill the array offsets of one instance starting at byte `at`; returns the end offset.
FC_HD int64_t layout(Inst &I, int64_t at) {
    const int64_t N = I.N, T = I.T, E = I.E, F = I.F, FAC = I.FAC, M0 = I.M0cap, MT = I.MTcap;
    const int64_t L = (E > F ? E : F) > 0 ? (E > F ? E : F) : 1;
    int64_t SCR = L > M0 ? L : M0;
    auto take = [&](int64_t bytes) {
        int64_t o = at;
        at = align256(at + (bytes > 0 ? bytes : 1) + FC_ARRAY_GAP);
        return o;
    };
    I.o_par0 = take(4 * N);
    I.o_parT = take(4 * T);
    I.o_keyE = take(8 * E);
    I.o_ea = take(4 * E);
    I.o_eb = take(4 * E);
    I.o_neg0 = take(4 * E);
    I.o_keyF = take(8 * F);
    I.o_fa = take(4 * FAC);
    I.o_fb = take(4 * FAC);
    I.o_killer = take(4 * FAC);
    I.o_n0key = take(8 * M0);
    I.o_n0sorted = take(8 * M0);
    I.o_nTkey = take(8 * MT);
    I.o_uf0 = take(4 * M0);
    I.o_moe0 = take(4 * M0);
    I.o_death0 = take(4 * M0);
    I.o_ufT = take(4 * MT);
    I.o_moeT = take(4 * MT);
    // live, live2 and ra, rb are two contiguous regions: each is also the merge scratch of one
    // long sorted list (KEEP squares: at most L keys; node keys: at most SCR)
    I.o_live = take(8 * L);
    I.o_live2 = I.o_live + 4 * L;     // the dual's live edges (it runs beside H0 in volumes)
    I.o_ra = take(8 * SCR);
    I.o_rb = I.o_ra + 4 * L;
    I.o_scratch = take(8 * SCR);
    const bool h1 = I.h1 && I.ndim == 3;
    I.pool_cap = h1 ? kH1PoolPerSquare * F : 0;
    I.o_cfg3 = h1 ? take(2 * N) : 0;
    I.o_kpos = h1 ? take(4 * N) : 0;
    I.o_h1b = h1 ? take(4 * F) : 0;
    I.o_h1n = h1 ? take(4 * F) : 0;
    I.o_piv = h1 ? take(4 * E) : 0;
    I.o_first = h1 ? take(4 * E) : 0;
    I.o_pool = h1 ? take(4 * I.pool_cap) : 0;
    I.o_retry = h1 ? take(4 * F) : 0;       // columns too large for the first pass's tables
    I.end = at;
    return at;
}

}  // namespace fc

namespace fc {

// 3D: canonical level-1 index and present-cube mask from the raw 26-bit neighbour mask.
// A cell of L(v) is present when every neighbour spanned by it precedes v (Sec. 3.3: a
// diagonal neighbour only matters when the adjacent ones are present).
FC_HD uint32_t canon3d(uint32_t raw, uint32_t *cubes) {
    uint32_t face = raw & 63u;
    uint32_t sq = 0;
#pragma unroll
    for (int s = 0; s < 12; ++s) {
        uint32_t need = (1u << kSqFace[s][0]) | (1u << kSqFace[s][1]);
        if (((raw >> (6 + s)) & 1u) && (face & need) == need) sq |= 1u << s;
    }
    uint32_t cb = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        uint32_t need = (1u << kCubeSq[c][0]) | (1u << kCubeSq[c][1]) | (1u << kCubeSq[c][2]);
        if (((raw >> (18 + c)) & 1u) && (sq & need) == need) cb |= 1u << c;
    }
    *cubes = cb;
    return face | (sq << 6);
}

// possible cubes given the present squares
FC_HD uint32_t possible_cubes(uint32_t sq) {
    uint32_t cb = 0;
    for (int c = 0; c < 8; ++c) {
        uint32_t need = (1u << kCubeSq[c][0]) | (1u << kCubeSq[c][1]) | (1u << kCubeSq[c][2]);
        if ((sq & need) == need) cb |= 1u << c;
    }
    return cb;
}

// gather the bits of `bits` selected by `mask` into the low bits (software pext)
FC_HD uint32_t compress8(uint32_t bits, uint32_t mask) {
    uint32_t out = 0, k = 0;
    for (int c = 0; c < 8; ++c)
        if ((mask >> c) & 1u) { out |= ((bits >> c) & 1u) << k; ++k; }
    return out;
}

}  // namespace fc
