// fc_kernels.hip -- gfx950 kernels and C ABI of the cubical persistence library.
//
// Pipeline of one call (each step a kernel over every instance of the batch):
//   plan      : per-instance table (sizes, tiles, workspace offsets), counters cleared
//   classify  : LDS-tiled stencil over the pixels; per vertex the neighbour mask is looked
//               up in the lower-star table (Sec. 3.3) and the lower star is pruned
//               (Sec. 3.2): DIRECT edges and locally paired top cells become forest links
//               resolved inside the tile, critical cells are appended to compact lists
//   sort      : KEEP edges (and 3D KEEP squares) sorted by their refined-order keys
//   resolve   : endpoints / cofacets of the sorted cells mapped to union-find nodes
//   uf        : H0 union-find with the elder rule over the KEEP edges (Sec. 4.1 step 3,
//               Sec. 4.2 step 2), by parallel rounds of safe merges (see uf_body)
//   resolve   : cofacets of the facets left for the top dimension (2D: the edges H0 did not
//               use, the cross-pruning of Sec. 3.2 / Sec. 4.1 step 4)
//   uf (dual) : union-find on the dual graph with the cell at infinity, facets in decreasing
//               order (Sec. 3.1, Appendix A)
//   output    : pairs of non-zero persistence, sorted by (dim, birth key), written SoA
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/flashcubical.h"
#include "fc_common.h"

namespace fc {

int build_lut2d(uint32_t *lut, char *err, int errlen);
int build_lut3d(uint32_t *l1, uint64_t *l2, uint16_t *h1e, uint16_t *h1s, char *err, int errlen);

// The lookup tables live in device buffers the library allocates once per device and passes
// to the kernels as arguments; device code reads no variable of its own code object.
struct Luts {
    const uint32_t *l2d;   // 256 entries (2D)
    const uint32_t *l1;    // kL1Size entries (3D level 1)
    const uint64_t *l2;    // kL3Configs entries (3D level 2)
    const uint16_t *h1e;   // 8 per 3D entry: an edge's partner combination (3D H1)
    const uint16_t *h1s;   // 16 per 3D entry: a KEEP square's own combination (3D H1)
    const uint8_t *pext;   // 256: [mask nibble << 4 | bits nibble] -> compress8(bits, mask)
};

constexpr int32_t kLocal = 0x40000000;     // LDS link to an entry of the same tile
constexpr int32_t kUnset = 0x7FFFFFFF;     // LDS cube slot not yet written
constexpr int kMaxChase = 1 << 22;         // bound of every pointer walk
constexpr int kUfThreads = 1024;
constexpr int kUfLdsNodes = 5120;          // union-find nodes kept in LDS with their keys (40 KiB + 40 KiB)
constexpr int kUfLdsEdges = 4096;          // union-find live edges kept in LDS (3 x 16 KiB)
constexpr int kUfLdsWords = 40880;         // the union-find's LDS (160 KiB less its other shared words), int32
constexpr int kUfLdsNodesOnly = kUfLdsWords / 2;   // nodes whose par, moe alone fit in LDS
constexpr int kSortThreads = 1024;
constexpr int kSortCap = 4096;             // keys sorted entirely in LDS (32 KiB)
constexpr int kMaxRounds = 48;             // parallel rounds before the sequential finish
constexpr int kWideRounds = 32;            // union-find rounds over many workgroups (PH_WIDE)
constexpr int64_t kWideVoxels = 1 << 20;   // ... for instances of this many voxels
constexpr int kWideBlocks = 2048, kWideThreads = 256;
constexpr int32_t kFired = 1 << 30;        // wide rounds: an edge fired this round (above every node index)
constexpr int32_t kInf = 0x7FFFFFFF;
constexpr int kMaxInstances = 65535;       // instances of one call: the y extent of a grid
// Halo key of a pixel outside the image.  Pixel keys are capped one below it (only the NaN bit
// pattern 0x7FFFFFFF would reach it, and NaN input is an error), so an outside neighbour never
// precedes a vertex and the stencil needs no bounds checks.
constexpr uint32_t kOutside = 0xFFFFFFFFu;

// ------------------------------------------------------------------ workspace map --
FC_HD int64_t off_tb2(int n) { return align256((int64_t)n * (int64_t)sizeof(Inst)); }
FC_HD int64_t off_tb3(int n) { return off_tb2(n) + align256((int64_t)(n + 1) * 8); }
FC_HD int64_t off_cnt(int n) { return off_tb3(n) + align256((int64_t)(n + 1) * 8); }
FC_HD int64_t header_bytes(int n) { return off_cnt(n) + align256((int64_t)n * CNT_WORDS * 4); }

struct Tiles { int tw2, th2, tw3, th3, td3; };

// lists: the list fraction (k / 256 of the worst case, 0 for the worst case); I.E, I.F and
// I.FAC are the capacities of the KEEP-edge, KEEP-square and facet lists from then on
FC_HD void fill_inst(Inst &I, const ph_shape &s, const Tiles &tl, int lists = 0) {
    I.ndim = s.ndim;
    if (s.ndim == 2) { I.D = 1; I.H = s.ext[0]; I.W = s.ext[1]; }
    else { I.D = s.ext[0]; I.H = s.ext[1]; I.W = s.ext[2]; }
    Geom g = geom(I.ndim, I.D, I.H, I.W);
    I.N = g.N; I.T = g.T;
    I.lists = lists;
    I.E = list_cap(g.E, lists);
    I.F = list_cap(g.F, lists);
    I.FAC = I.ndim == 2 ? I.E : I.F;                 // the facets the dual walks: KEEP edges / squares
    I.M0cap = list_cap(g.N, lists);
    I.MTcap = list_cap(g.T + 1, lists);
    if (s.ndim == 2) {
        I.tx = (I.W + tl.tw2 - 1) / tl.tw2; I.ty = (I.H + tl.th2 - 1) / tl.th2; I.tz = 1;
    } else {
        I.tx = (I.W + tl.tw3 - 1) / tl.tw3; I.ty = (I.H + tl.th3 - 1) / tl.th3;
        I.tz = (I.D + tl.td3 - 1) / tl.td3;
    }
    I.tfilt = 0;
    I.h1 = 0;
}

// list fraction k of the flags (PH_LIST_FRACTION(k): capacities k / 256 of the worst case)
inline int list_fraction(uint32_t flags) { return (int)((flags >> 8) & 0xFFu); }

// T-filtration: the framed dual image has one more pixel on each side of every axis
FC_HD ph_shape framed(ph_shape s) {
    for (int k = 0; k < s.ndim; ++k) s.ext[k] += 2;
    return s;
}

// One thread per instance, in chunks of the block: each instance's table entry, with its
// workspace offset and first tile found by a block-wide prefix sum over the chunk.  An
// instance's arrays start on a 256-byte boundary, so its layout is its size-only layout
// shifted by its offset.
constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void k_plan(int n, const ph_shape *__restrict__ d_shapes, ph_shape single,
                       const int64_t *__restrict__ d_img_off, const int64_t *__restrict__ d_out_off,
                       int64_t single_cap, Tiles tl, uint8_t *__restrict__ ws,
                       int64_t *__restrict__ d_counts, int32_t *__restrict__ d_status,
                       int64_t want_t2, int64_t want_t3, int64_t ws_bytes, int tfilt, int h1, int lists) {
    __shared__ int64_t s_scan[2][3][kPlanThreads];   // bytes, 2D tiles, 3D tiles (double buffer)
    __shared__ int64_t s_run[3];
    if (blockIdx.x != 0) return;
    const int t = threadIdx.x;
    Inst *tab = (Inst *)ws;
    int64_t *tb2 = (int64_t *)(ws + off_tb2(n));
    int64_t *tb3 = (int64_t *)(ws + off_tb3(n));
    int32_t *cnt = (int32_t *)(ws + off_cnt(n));
    if (t == 0) { s_run[0] = header_bytes(n); s_run[1] = 0; s_run[2] = 0; }
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += kPlanThreads) {
        const int i = c0 + t;
        Inst I;
        bool ok = true;
        int64_t v[3] = {0, 0, 0};
        if (i < n) {
            ph_shape s = d_shapes ? d_shapes[i] : single;
            ok = (s.ndim == 2 || s.ndim == 3) && s.ext[0] >= 1 && s.ext[1] >= 1 && (s.ndim == 2 || s.ext[2] >= 1);
            if (!ok) s = ph_shape{2, {1, 1, 1}};
            if (tfilt) s = framed(s);
            fill_inst(I, s, tl, lists);
            if (I.N > (1ll << kPixBits)) {
                ok = false;
                s = ph_shape{2, {1, 1, 1}};
                fill_inst(I, tfilt ? framed(s) : s, tl, lists);
            }
            I.tfilt = tfilt;
            I.h1 = h1 && I.ndim == 3;
            v[0] = layout(I, 0);
            if (I.ndim == 2) v[1] = (int64_t)I.tx * I.ty;
            else v[2] = (int64_t)I.tx * I.ty * I.tz;
        }
        // the counter words of this chunk's instances set to zero by the whole block, a word a
        // thread, in coalesced stores (the barriers of the scan order them before each
        // instance's own non-zero words below)
        {
            const int c1 = n - c0 < kPlanThreads ? n : c0 + kPlanThreads;
            for (int64_t w = (int64_t)c0 * CNT_WORDS + t; w < (int64_t)c1 * CNT_WORDS; w += kPlanThreads) cnt[w] = 0;
        }
        // inclusive Hillis-Steele scan of the three sizes over the block
        int b = 0;
        for (int k = 0; k < 3; ++k) s_scan[0][k][t] = v[k];
        __syncthreads();
        for (int off = 1; off < kPlanThreads; off <<= 1) {
            for (int k = 0; k < 3; ++k)
                s_scan[b ^ 1][k][t] = s_scan[b][k][t] + (t >= off ? s_scan[b][k][t - off] : 0);
            b ^= 1;
            __syncthreads();
        }
        if (i < n) {
            const int64_t at = s_run[0] + s_scan[b][0][t] - v[0];
            I.src_off = d_img_off ? d_img_off[i] : 0;
            I.out_off = d_out_off ? d_out_off[i] : 0;
            I.out_cap = d_out_off ? d_out_off[i + 1] - d_out_off[i] : single_cap;
            tb2[i] = s_run[1] + s_scan[b][1][t] - v[1];
            tb3[i] = s_run[2] + s_scan[b][2][t] - v[2];
            I.tile_base = I.ndim == 2 ? tb2[i] : tb3[i];
            layout(I, at);
            tab[i] = I;
            cnt[i * CNT_WORDS + CNT_MT] = 1;           // dual node 0 is the cell at infinity
            if (!ok || I.out_cap < 0) cnt[i * CNT_WORDS + CNT_ERR] = PH_EINVAL;
            d_counts[i] = 0;
            d_status[i] = PH_OK;
        }
        __syncthreads();
        if (t == kPlanThreads - 1)
            for (int k = 0; k < 3; ++k) s_run[k] += s_scan[b][k][t];
        __syncthreads();
    }
    if (t == 0) {
        tb2[n] = s_run[1];
        tb3[n] = s_run[2];
    }
    // the launch grids were sized from the host shapes: a device table that disagrees with
    // them (or outgrows the workspace) disables every instance
    if (s_run[1] != want_t2 || s_run[2] != want_t3 || s_run[0] > ws_bytes)
        for (int i = t; i < n; i += kPlanThreads) cnt[i * CNT_WORDS + CNT_ERR] = PH_EINVAL;
}

// true when an earlier kernel recorded an error for this instance: later kernels skip it
__device__ __forceinline__ bool failed(const int32_t *cnt) {
    return __hip_atomic_load(&cnt[CNT_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}
// the same decision taken once for the whole block (every thread must call it)
__device__ __forceinline__ bool block_failed(const int32_t *cnt) {
    return __syncthreads_or(failed(cnt) ? 1 : 0) != 0;
}

// Workgroups are dealt to the 8 XCDs of the chip round-robin (workgroup w runs on XCD w % 8),
// and each XCD has its own L2.  Tiles are renumbered so that every XCD gets one contiguous run
// of tiles: neighbouring tiles share halo rows, which then hit the same L2.  A bijection of
// [0, g) for any grid size g.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t w, int64_t g) {
    const int64_t base = g / kXcds, rem = g % kXcds;
    const int64_t x = w % kXcds, local = w / kXcds;
    return x * base + (x < rem ? x : rem) + local;
}

// Instance owning `tile`: the largest i with tb[i] <= tile (tb ascending, tb[0] = 0,
// tb[n] = all tiles).  Every wave searches on its own, 64 probes per step, so a batch of up to
// 64 instances costs one dependent load and 65535 instances three.
__device__ __forceinline__ int find_inst(const int64_t *tb, int n, int64_t tile) {
    const int lane = __lane_id();
    int lo = 0, hi = n;                            // tb[lo] <= tile < tb[hi]
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) >> 6;
        const int probe = lo + lane * step;
        const bool le = probe < hi && tb[probe] <= tile;
        const uint64_t m = __ballot(le);           // lanes 0.. set up to the owner's step
        const int last = 63 - __builtin_clzll(m);  // lane 0 always qualifies (tb[lo] <= tile)
        lo += last * step;
        hi = lo + step < hi ? lo + step : hi;
    }
    return lo;
}

// Barrier for LDS traffic only.  The global stores of a block are read by later kernels,
// never by the block's other threads, so the barrier does not wait for them to complete.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The classify passes go on after a list overflow (PH_ELISTS), writing nothing beyond the
// capacities, so that the list counts they reserve are the instance's true sizes; any other
// error stops them.  One thread reads the word and the block takes its answer through LDS
// (s_flag), so every thread decides alike.  Every thread must call it.
__device__ __forceinline__ bool block_failed_classify(const int32_t *cnt, int *s_flag) {
    if (threadIdx.x == 0) {
        const int e = __hip_atomic_load(&cnt[CNT_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = e != 0 && e != PH_ELISTS;
    }
    lds_barrier();
    return *s_flag != 0;
}
// The same in two steps, so that the word's load is in flight while the block does other work:
// err_word (thread 0 reads the word, the others 0), then block_failed_from with its value.
__device__ __forceinline__ int err_word(const int32_t *cnt) {
    return threadIdx.x == 0 ? __hip_atomic_load(&cnt[CNT_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
}
__device__ __forceinline__ bool block_failed_from(int e, int *s_flag) {
    if (threadIdx.x == 0) *s_flag = e != 0 && e != PH_ELISTS;
    lds_barrier();
    return *s_flag != 0;
}

template <typename T>
__device__ __forceinline__ T *arr(uint8_t *ws, int64_t off) { return (T *)(ws + off); }

__device__ __forceinline__ void set_err(int32_t *cnt, int code) {
    atomicCAS(&cnt[CNT_ERR], 0, code);
}
// A list outgrew its capacity: PH_ELISTS under a list fraction, else (the worst case cannot
// overflow) an internal error
__device__ __forceinline__ void list_overflow(const Inst &I, int32_t *cnt) {
    set_err(cnt, I.lists ? PH_ELISTS : PH_EINTERNAL);
}

// Links inside a classify tile.  A slot holds a final value (a node, a link out of the tile,
// the cell at infinity) or kLocal | s, a link to slot s of the same tile.  A top-cell slot that
// no vertex of the tile writes keeps its initial value, the cell's own global index: a link
// that reaches it ends there, at a cell of another tile.  Pointer jumping (jump_links) replaces
// every local link by its target's value until none is left.
__device__ __forceinline__ bool is_local(int32_t v) { return v >= kLocal; }

// Offset of octant t = (z y x bits), t < 8, of the eight cubes around a vertex from the slot
// of the first (t = 0), in a slot box of rows PW and layers PW * PH.  When every offset fits a
// byte the eight are picked with one byte permute; t itself is the selector: its upper bytes
// are zero and pick byte 0 of the low word, the first octant's offset, which is zero.
template <int PW, int PH>
__device__ __forceinline__ int oct_slot(uint32_t t) {
    constexpr uint32_t L = PH * PW;
    if constexpr (L + PW + 1 < 256) {
        constexpr uint32_t lo = 0u | 1u << 8 | (uint32_t)PW << 16 | (uint32_t)(PW + 1) << 24;
        constexpr uint32_t hi = L | (L + 1) << 8 | (L + PW) << 16 | (L + PW + 1) << 24;
        return (int)__builtin_amdgcn_perm(hi, lo, t);
    } else {
        return (int)((t >> 2) * L + ((t >> 1) & 1u) * PW + (t & 1u));
    }
}

// Offset of square q = (y x bits), q < 4, of the four squares around a vertex from the slot of
// the first (q = 0), in rows of PW slots; picked with a byte permute (q as the selector, as in
// oct_slot) when every offset fits a byte.
template <int PW>
__device__ __forceinline__ int quad_slot(uint32_t q) {
    if constexpr (PW + 1 < 256) {
        return (int)__builtin_amdgcn_perm(0u, 0u | 1u << 8 | (uint32_t)PW << 16 | (uint32_t)(PW + 1) << 24, q);
    } else {
        return (int)((q >> 1) * PW + (q & 1u));
    }
}

// link to slot s of the tile when bit t of inimg is set, else -1 (the cell at infinity):
// kp = kLocal | pos0 with s = pos0 + off; a sign-extended bit field and one bit select
__device__ __forceinline__ int32_t dual_link(uint32_t inimg, uint32_t t, int32_t kp, int off) {
    const int32_t m = -(int32_t)((inimg >> t) & 1u);                 // 0 or -1
    return ((kp + off) & m) | ~m;
}

// 2 raw + (a < b), or with LE 2 raw + (a <= b), unsigned: the compare sets VCC and an add with
// carry shifts it in (two vector instructions; compiled code takes a compare, a select and a
// merge).  A vector read of VCC as carry right after a vector compare wrote it needs no wait
// states (the same pairing as the add and add-with-carry of a 64-bit sum).  The CPU emulation
// build of the kernels computes the same in C.
template <bool LE>
__device__ __forceinline__ uint32_t shift_in_less(uint32_t raw, uint32_t a, uint32_t b) {
#if defined(__AMDGCN__)
    uint32_t r;
    if (LE)
        asm("v_cmp_le_u32_e32 vcc, %1, %2\n\tv_addc_co_u32_e32 %0, vcc, %3, %3, vcc"
            : "=v"(r) : "v"(a), "v"(b), "v"(raw) : "vcc");
    else
        asm("v_cmp_lt_u32_e32 vcc, %1, %2\n\tv_addc_co_u32_e32 %0, vcc, %3, %3, vcc"
            : "=v"(r) : "v"(a), "v"(b), "v"(raw) : "vcc");
    return r;
#else
    return raw + raw + (uint32_t)(LE ? a <= b : a < b);
#endif
}

// v clamped into [0, hi]
__device__ __forceinline__ int clamp0(int v, int hi) {
    const int a = v > 0 ? v : 0;
    return a < hi ? a : hi;
}

// T-filtration (Sec. 2.2): the kernels run the V construction on the framed dual image of the
// caller's pixels, whose pixel (z, y, x) holds minus the caller's pixel at the point reflection
// (sD - z, sH - y, sW - x) of the inner box (s* = framed extent - 2; an image has no frame
// along z) and -inf on the frame.  Its V complex is the dual cell complex of the caller's T
// complex with the frame added; the reflection turns the V tie-break (a larger index enters
// later) into the T one read backwards.  Nothing is stored: the classify passes and 3D H1 read
// the caller's pixels through this map.  f is the caller's pixel, inner whether the framed
// pixel lies inside the frame.  A +inf pixel would tie the frame: it becomes NaN, which the
// classify pass reports as PH_ENAN.
__device__ __forceinline__ float tf_value(float f, bool inner) {
    return !inner ? __int_as_float(0xff800000)                                    // -inf
                  : (f == __int_as_float(0x7f800000) ? __int_as_float(0x7fc00000) : -f);
}
template <bool B> using tf_tag = std::integral_constant<bool, B>;
__device__ __forceinline__ int32_t slot_get(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void slot_put(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// OR of a flag over the block with one LDS-only barrier.  Successive calls alternate between
// the two halves of s_any[8] (parity): every wave rewrites its flag on each call, and a wave can
// only rewrite a half after every wave has passed the barrier of the call in between, so no
// flag is overwritten while still being read.
__device__ __forceinline__ bool block_any(bool flag, int *s_any, int parity) {
    static_assert(256 / 64 <= 4, "one flag per wave of the block");
    const bool w = __ballot(flag) != 0;
    if (__lane_id() == 0) s_any[parity * 4 + (threadIdx.x >> 6)] = w ? 1 : 0;
    lds_barrier();
    const int *a = s_any + parity * 4;
    return (a[0] | a[1] | a[2] | a[3]) != 0;
}

// Pointer jumping over a tile's vertex slots sp0[256 N0] and top-cell slots spT[ST NT].  A
// thread owns the vertex slots threadIdx.x + 256 k and the top-cell slots threadIdx.x + ST k
// and holds their values in v0, vT (a thread without top-cell slots holds finals there); it
// alone writes them.  Every round it replaces each local value by its target's value and
// publishes it; a barrier ends the round, so chains at least halve every round.  Reads within
// a round may already see other slots' new values, which only helps: a value only ever moves
// along its own chain.  Slots are read and written whole, as relaxed atomics.  A chain visits
// each slot at most once, which bounds the rounds.  All threads of the block must call it.
template <int N0, int NT, int ST>
__device__ __forceinline__ void jump_links(int32_t *sp0, int32_t *spT, int32_t (&v0)[N0], int32_t (&vT)[NT],
                                           int *s_any, int32_t *cnt) {
    const int tid = threadIdx.x;
    bool any = true;                                // a thread whose slots are all final stays so
    for (int round = 0; round <= 256 * (N0 + NT); ++round) {
        if (any) {
            any = false;
#pragma unroll
            for (int k = 0; k < N0; ++k) {
                if (is_local(v0[k])) {
                    // kLocal | s, s clamped to the last slot; times 4 it wraps to the offset 4 s
                    const uint32_t u = (uint32_t)v0[k], hi = (uint32_t)kLocal + 256u * N0 - 1u;
                    const uint32_t t = (u < hi ? u : hi) - (uint32_t)kLocal;
                    v0[k] = slot_get(&sp0[t]);
                    slot_put(&sp0[tid + 256 * k], v0[k]);
                    any |= is_local(v0[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                if (is_local(vT[k])) {
                    const uint32_t u = (uint32_t)vT[k], hi = (uint32_t)kLocal + ST * NT - 1u;
                    const uint32_t t = (u < hi ? u : hi) - (uint32_t)kLocal;
                    vT[k] = slot_get(&spT[t]);
                    slot_put(&spT[tid + ST * k], vT[k]);
                    any |= is_local(vT[k]);
                }
            }
        }
        if (!block_any(any, s_any, round & 1)) return;
    }
    set_err(cnt, PH_EINTERNAL);
}

// Block-wide reservation of slots in up to four per-instance lists at once.  Each thread
// passes its counts packed 16 bits per list (every block total stays below 2^16: a tile has
// 1024 vertices and at most 12 kept cells each of one kind); the block scans them once and
// lane k of wave 0 reserves list k's block total with a single atomic, all lists' atomics in
// flight together, so a tile costs one atomic per non-empty list instead of one per wave and
// pass, and one round trip to L2.  lists8 holds the lists' counter words, a byte each (list k
// in bits 8k..8k+7).  Returns the thread's exclusive prefix (packed the same way); the lists'
// first slots are left in s_base.  All threads call it.
// Inclusive sum of x over the lanes of a wave up to each lane, with data-parallel-primitive
// moves: sums inside each row of 16 lanes (row shifts by 1, 2, 4 and 8 lanes, a lane shifted in
// from outside the row reading 0), then the totals carried up (lane 15 of row 0 and 2 added
// to rows 1 and 3, lane 31 to rows 2 and 3).  All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);   // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return x;
}

template <int NLIST>
__device__ __forceinline__ uint64_t block_alloc(int32_t *cnt, uint32_t lists8, uint64_t packed,
                                                uint64_t *s_scan, int32_t *s_base) {
    const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // the 16-bit fields never carry: each block total stays below 2^16, so the two 32-bit
    // halves are summed apart
    const uint64_t x = (uint64_t)wave_incl_sum((uint32_t)(packed >> 32)) << 32 | wave_incl_sum((uint32_t)packed);
    if (lane == 63) s_scan[wid] = x;
    lds_barrier();
    uint64_t pre = 0;                                // the block's entries before this wave's
    for (int w = 0; w < wid; ++w) pre += s_scan[w];
    if (wid == 0 && lane < NLIST) {
        // lane k of wave 0 takes list k's block of entries: the atomics are in flight together
        uint64_t tot = 0;
        for (int w = 0; w < nw; ++w) tot += s_scan[w];
        const int li = (int)((lists8 >> (8 * lane)) & 0xFFu);   // counter word of list `lane`
        const int t = (int)((tot >> (16 * lane)) & 0xFFFFu);
        s_base[lane] = t ? atomicAdd(&cnt[li], t) : 0;
    }
    lds_barrier();
    return pre + x - packed;
}

// ph_diagram_batch_grad: the caller's gradient of one classify tile's pixels (TD layers of TH
// rows of TW, 1024 in all) set to zero for ph_backward_scatter; under the T-filtration only the
// inner pixels of the framed grid are the caller's, at the reflected index.  Where the rows
// start on 16-byte boundaries (the gradient base of the instance and W a multiple of 4) each
// thread clears four neighbours of a row with one store; else four pixels 256 apart.  The
// tile's pixels per thread go with the index computed once: 256 is a whole number of layers
// (3D tiles) or rows (2D tiles), so only z (or y) moves between them.
template <int TW, int TH, int TD>
__device__ __forceinline__ void clear_grad_tile(float *__restrict__ g, int tfilt, int D, int H, int W, int z0,
                                                int y0, int x0) {
    static_assert(TW * TH * TD == 1024 && TW % 4 == 0, "a tile is 1024 pixels in rows of whole quads");
    constexpr int LAY = TD > 1 ? TW * TH : TW;     // pixels per step of the moving coordinate
    static_assert(256 % LAY == 0, "a block covers whole layers (3D) or rows (2D)");
    constexpr int DM = 256 / LAY;                  // steps of the moving coordinate per pass
    const int HW = H * W, t = threadIdx.x;
    if (!tfilt && (((uintptr_t)g & 15) | (uintptr_t)(W & 3)) == 0) {
        constexpr int Q = TW / 4;
        const int lx = (t % Q) * 4, r = t / Q, ly = r % TH, lz = r / TH;
        const int gz = z0 + lz, gy = y0 + ly, gx = x0 + lx;
        if (gz < D && gy < H && gx < W)            // W % 4 == 0: the quad lies in the row
            *(float4 *)(g + (uint32_t)(gz * HW + gy * W + gx)) = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const int lx = t % TW, ly = (t / TW) % TH, lz = t / (TW * TH);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    // the moving coordinate m (z in 3D, y in 2D), its range, the fixed ones' test, the index
    // at the first pass and its step between passes
    int m, mlo, mhi, idx, step;
    bool fixed_in;
    if (!tfilt) {
        m = TD > 1 ? gz : gy;
        mlo = 0;
        mhi = (TD > 1 ? D : H) - 1;
        fixed_in = gx < W && (TD > 1 ? gy < H : true);
        idx = gz * HW + gy * W + gx;
        step = DM * (TD > 1 ? HW : W);
    } else {
        const int sH = H - 2, sW = W - 2;
        m = TD > 1 ? gz : gy;
        mlo = 1;
        mhi = (TD > 1 ? D : H) - 2;
        fixed_in = gx >= 1 && gx <= sW && (TD > 1 ? gy >= 1 && gy <= sH : true);
        idx = TD > 1 ? ((D - 2 - gz) * sH + (sH - gy)) * sW + (sW - gx) : (sH - gy) * sW + (sW - gx);
        step = -DM * (TD > 1 ? sH * sW : sW);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int mk = m + k * DM;
        if (fixed_in && mk >= mlo && mk <= mhi) g[(uint32_t)(idx + k * step)] = 0.0f;
    }
}

// ================================================================ classify 2D ====
template <int TW, int TH, typename T>
__global__ __launch_bounds__(256) void k_classify2d(const T *__restrict__ imgs,
                                                    uint8_t *__restrict__ ws, int n, Luts lut,
                                                    float *__restrict__ grad) {
    static_assert((TW * TH) % 256 == 0, "tile must be a multiple of the block");
    constexpr int KW = TW + 2, PW = TW + 1, NP = (TH + 1) * (TW + 1);
    constexpr int NIT = TH * TW / 256, NKT = (NP + 255) / 256;
    __shared__ uint32_t skey[(TH + 2) * KW];
    __shared__ int32_t sp0[TH * TW];
    __shared__ int32_t spT[256 * NKT];           // padded to whole rounds of the block
    constexpr int NRT = (256 * NKT + PW - 1) / PW;   // slot rows, padding included
    __shared__ int2 s_row[NRT];
    __shared__ int s_nan;
    __shared__ uint64_t s_scan[4];
    __shared__ int32_t s_base[4];
    __shared__ int s_any[8];
    __shared__ int2 s_dir[4];
    __shared__ int s_fail;

    const Inst *tab = (const Inst *)ws;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int i = find_inst((const int64_t *)(ws + off_tb2(n)), n, tile);
    // the instance's record copied before the kernel's first store or atomic: its fields load as
    // scalar loads in one batch (after a store they would be vector loads where first used)
    const Inst I = tab[i];
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    const int err = err_word(cnt);
    const int H = I.H, W = I.W;
    const int lt = (int)(tile - I.tile_base);
    const int ty = lt / I.tx, tx = lt - ty * I.tx;
    const int y0 = ty * TH, x0 = tx * TW;
    // before the error check: an instance that fails still has its gradient cleared
    if (grad) clear_grad_tile<TW, TH, 1>(grad + I.src_off, I.tfilt, 1, H, W, 0, y0, x0);
    if (block_failed_from(err, &s_fail)) return;
    const T *img = imgs + I.src_off;
    int32_t *par0 = arr<int32_t>(ws, I.o_par0);
    int32_t *parT = arr<int32_t>(ws, I.o_parT);
    uint64_t *keyE = arr<uint64_t>(ws, I.o_keyE);
    uint64_t *n0key = arr<uint64_t>(ws, I.o_n0key);
    uint64_t *nTkey = arr<uint64_t>(ws, I.o_nTkey);

    if (threadIdx.x == 0) s_nan = 0;
    int nan = 0;
    // The halo box is TH + 2 rows of KW keys.  Wave w loads rows w, w + 4, ... in whole
    // 64-column chunks, so a row's y, its clamp and whether it lies in the image are the same
    // for the wave; the KW % 64 columns left over are loaded one key per thread.  Every load of
    // the thread is issued before the first is used: the addresses are clamped into the image
    // and outside pixels replaced afterwards.  Clamped loads read a pixel of the instance: a
    // NaN there is one of the instance's own.  Under the T-filtration the image is the framed
    // dual one, read through the reflection (tf_value).
    auto halo = [&](auto tf) {
        constexpr bool TF = decltype(tf)::value;
        constexpr int NR = TH + 2, NFC = KW / 64, REM = KW - 64 * NFC;
        constexpr int ITEMS = NR * NFC, PERW = (ITEMS + 3) / 4;     // (row, chunk) items
        constexpr int NREM = NR * REM, NLR = (NREM + 255) / 256;   // left-over keys
        const int sH = H - 2, sW = W - 2;                           // T: the caller's extents
        const int lane = __lane_id(), w = threadIdx.x >> 6;
        auto at = [&](int gy, int gx) -> uint32_t {                // clamped source offset
            return TF ? (uint32_t)(clamp0(sH - gy, sH - 1) * sW + clamp0(sW - gx, sW - 1))
                      : (uint32_t)(clamp0(gy, H - 1) * W + clamp0(gx, W - 1));
        };
        auto put = [&](int idx, float v, int gy, int gx) {
            if constexpr (TF) v = tf_value(v, gy >= 1 && gy <= H - 2 && gx >= 1 && gx <= W - 2);
            nan |= v != v;
            const uint32_t o = ord32_no_neg0(__float_as_uint(v + 0.0f));
            const bool in = (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
            skey[idx] = in ? (o < kOutside ? o : kOutside - 1u) : kOutside;
        };
        float f[PERW > 0 ? PERW : 1], fr[NLR > 0 ? NLR : 1];
#pragma unroll
        for (int k = 0; k < PERW; ++k) {
            const int j = w + 4 * k, r = j / (NFC > 0 ? NFC : 1), ch = j - r * NFC;
            if (j < ITEMS) f[k] = (float)img[at(y0 - 1 + r, x0 - 1 + ch * 64 + lane)];
        }
#pragma unroll
        for (int k = 0; k < NLR; ++k) {
            const int q = threadIdx.x + 256 * k, r = q / (REM > 0 ? REM : 1), c = 64 * NFC + q - r * REM;
            if (q < NREM) fr[k] = (float)img[at(y0 - 1 + r, x0 - 1 + c)];
        }
#pragma unroll
        for (int k = 0; k < PERW; ++k) {
            const int j = w + 4 * k, r = j / (NFC > 0 ? NFC : 1), ch = j - r * NFC;
            if (j < ITEMS) put(r * KW + ch * 64 + lane, f[k], y0 - 1 + r, x0 - 1 + ch * 64 + lane);
        }
#pragma unroll
        for (int k = 0; k < NLR; ++k) {
            const int q = threadIdx.x + 256 * k, r = q / (REM > 0 ? REM : 1), c = 64 * NFC + q - r * REM;
            if (q < NREM) put(r * KW + c, fr[k], y0 - 1 + r, x0 - 1 + c);
        }
    };
    if (I.tfilt) halo(tf_tag<true>{});
    else halo(tf_tag<false>{});
    // square slots start unset (padding final); after pass 2 the slots no vertex of the tile
    // wrote get their square's global index (see is_local).  s_row[r]: global index of the
    // first square of slot row r (x = x0 - 1) and whether the row lies in the image.
#pragma unroll
    for (int k = 0; k < NKT; ++k) spT[threadIdx.x + 256 * k] = threadIdx.x + 256 * k < NP ? kUnset : 0;
    for (int r = threadIdx.x; r < NRT; r += 256) {
        const int sy = y0 - 1 + r;
        s_row[r] = make_int2(sy * (W - 1) + x0 - 1, r <= TH && (unsigned)sy < (unsigned)(H - 1));
    }
    if (threadIdx.x < 4) {
        // direct edge 2 + d (d = 0..3: up, left, right, down): the step to the neighbour's slot
        // in the tile (low word) and to its pixel in the image (high word)
        const int d = threadIdx.x;
        s_dir[d] = d == 0 ? make_int2(-TW, -W) : d == 1 ? make_int2(-1, -1) : d == 2 ? make_int2(1, 1)
                                                                                  : make_int2(TW, W);
    }
    lds_barrier();
    if (nan) s_nan = 1;

    // neighbours in mask-bit order: up, left, right, down, UL, UR, DL, DR
    constexpr int NDY[8] = {-1, 0, 0, 1, -1, -1, 1, 1};
    constexpr int NDX[8] = {0, -1, 1, 0, -1, 1, -1, 1};
    constexpr bool NBEFORE[8] = {true, true, false, false, true, true, false, false};

    // pass 1: every vertex of the thread through the table; counts of the cells it keeps
    constexpr uint32_t kValid = 1u << 31;           // above every field of a 2D entry
    uint32_t ev[NIT];
    uint32_t c_min = 0, c_edge = 0, c_root = 0;     // cells the thread keeps, by list
    // the 3x3 neighbourhood of vertex threadIdx.x + 256 it starts at skey[nb0 + it * kRows * KW]
    static_assert(256 % TW == 0, "a block covers whole tile rows");
    constexpr int kRows = 256 / TW;
    const int nb0 = (threadIdx.x / TW) * KW + threadIdx.x % TW;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int l = threadIdx.x + it * 256;
        const int r = l / TW, c = l - r * TW, gy = y0 + r, gx = x0 + c;
        const uint32_t *nb = skey + nb0 + it * kRows * KW;
        // branch-free (see the 3D kernel): a pixel outside the image is computed and dropped
        const bool in = gy < H && gx < W;
        const uint32_t kv = nb[KW + 1];
        uint32_t mask = 0;                              // bit b: neighbour b comes before v
#pragma unroll
        for (int b = 7; b >= 0; --b) {                  // outside neighbours hold kOutside
            const uint32_t kn = nb[(1 + NDY[b]) * KW + 1 + NDX[b]];
            mask = NBEFORE[b] ? shift_in_less<true>(mask, kn, kv) : shift_in_less<false>(mask, kn, kv);
        }
        const uint32_t e = in ? lut.l2d[mask] | kValid : 0u;
        // (an entry outside the image is 0 and counts nothing)
        c_min += (e & 7u) == kNoDirect ? 1u : 0u;
        c_edge += __popc((e >> kL2Keep) & 15u);
        c_root += __popc((e >> kL2Root) & 15u);
        ev[it] = e;
    }
    constexpr uint32_t lists8 = CNT_M0 | CNT_E << 8 | CNT_MT << 16;
    const uint64_t packed = c_min | c_edge << 16 | (uint64_t)c_root << 32;
    const uint64_t pre = block_alloc<3>(cnt, lists8, packed, s_scan, s_base);
    int id0 = s_base[0] + (int)(pre & 0xFFFFu);
    int kb = s_base[1] + (int)((pre >> 16) & 0xFFFFu);
    int rb = s_base[2] + (int)((pre >> 32) & 0xFFFFu);

    // pass 2: forest links, node keys and compact lists at the reserved slots.  Vertex
    // threadIdx.x + 256 it lies at row r0 + it kRows, column c0 of the tile; bit d of out_x:
    // the direct edge 2 + d leaves the tile sideways
    const int r0 = threadIdx.x / TW, c0 = threadIdx.x % TW;
    const uint32_t out_x = (c0 == 0 ? 2u : 0u) | (c0 == TW - 1 ? 4u : 0u);
    static_assert(NIT >= 2, "the first and last rows of the tile fall to different iterations");
    const uint32_t out_first = out_x | (r0 == 0 ? 1u : 0u);               // it = 0: r = r0
    const uint32_t out_last = out_x | (r0 == kRows - 1 ? 8u : 0u);        // it = NIT - 1
#pragma unroll 1                                    // rolled: fewer live registers, more waves per SIMD
    for (int it = 0; it < NIT; ++it) {
        const uint32_t e = ev[it];
        const int l = threadIdx.x + it * 256;
        if (!(e & kValid)) {                       // outside the image: a final slot value
            sp0[l] = 0;
            continue;
        }
        const int r = r0 + it * kRows, c = c0, gy = y0 + r, gx = x0 + c;
        const uint32_t kv = skey[(r + 1) * KW + c + 1];
        const uint32_t pv = (uint32_t)(gy * W + gx);
        const uint32_t direct = e & 7u;
        const uint32_t keep = (e >> kL2Keep) & 15u;
        const uint32_t present = (e >> kL2Present) & 15u;
        const uint32_t root = (e >> kL2Root) & 15u;

        // H0 forest: link to the other end of the DIRECT edge, or become a node
        if (direct == kNoDirect) {
            int id = id0++;
            if (id >= I.M0cap) { list_overflow(I, cnt); id = 0; }
            sp0[l] = -(id + 1);
            n0key[id] = make_key(kv, pv, 0);
        } else {
            // a link to the neighbour across the direct edge: its slot, or its pixel when it
            // lies outside the tile
            const uint32_t out = it == 0 ? out_first : (it == NIT - 1 ? out_last : out_x);
            const int2 dd = s_dir[direct];
            sp0[l] = (out >> direct) & 1u ? (int32_t)pv + dd.y : kLocal | (l + dd.x);
        }
        // KEEP edges -> compact list
        for (uint32_t m = keep; m; m &= m - 1) {
            const int b = __builtin_ctz(m);
            if (kb < I.E) keyE[kb] = make_key(kv, pv, 2 + b); else list_overflow(I, cnt);
            ++kb;
        }
        // squares of L(v): ROOT -> dual node, the others -> dual link.  Square q = (y x bits)
        // has its first corner at v - (1,1) + q and its slot at pos0 + quad_slot(q); it lies in
        // the image when both corner coordinates do.
        if (present) {
            const int pos0 = r * PW + c;
            const uint32_t inimg = ((gy >= 1 ? 0x3u : 0u) | (gy <= H - 2 ? 0xCu : 0u)) &
                                   ((gx >= 1 ? 0x5u : 0u) | (gx <= W - 2 ? 0xAu : 0u));
            for (uint32_t m = root & present; m; m &= m - 1) {
                const int q = __builtin_ctz(m);
                if (rb >= I.MTcap) { list_overflow(I, cnt); rb = 0; }
                spT[pos0 + quad_slot<PW>(q)] = -(rb + 1);
                nTkey[rb] = make_key(kv, pv, 11 + q);
                ++rb;
            }
            for (uint32_t m = present & ~root; m; m &= m - 1) {
                const int q = __builtin_ctz(m);
                const uint32_t t = (e >> (kL2Link + 2 * q)) & 3u;
                spT[pos0 + quad_slot<PW>(q)] = dual_link(inimg, t, kLocal | pos0, quad_slot<PW>(t));
            }
        }
    }
    lds_barrier();

    // resolve links inside the tile (see jump_links)
    int32_t v0[NIT], vT[NKT];
#pragma unroll
    for (int k = 0; k < NKT; ++k) {
        const int p = threadIdx.x + 256 * k, pr = p / PW, pc = p - pr * PW;
        vT[k] = spT[p];
        if (vT[k] == kUnset) spT[p] = vT[k] = s_row[pr].x + pc;
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) v0[k] = sp0[threadIdx.x + 256 * k];
    lds_barrier();
    jump_links<NIT, NKT, 256>(sp0, spT, v0, vT, s_any, cnt);

#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int l = threadIdx.x + 256 * k, r = l / TW, c = l - r * TW, gy = y0 + r, gx = x0 + c;
        if (gy < H && gx < W) par0[(uint32_t)(gy * W + gx)] = v0[k];
    }
#pragma unroll
    for (int k = 0; k < NKT; ++k) {
        const int p = threadIdx.x + 256 * k, pr = p / PW, pc = p - pr * PW;
        const int32_t v = vT[k];
        const int2 row = s_row[pr];
        const int32_t gidx = row.x + pc;
        if (p >= NP || v == gidx) continue;          // not a square of this tile
        // a square is only ever marked for a vertex whose lower star holds it, so it lies in
        // the image; the check keeps a corrupted table from writing outside parT
        if (row.y && (unsigned)(x0 - 1 + pc) < (unsigned)(W - 1)) parT[gidx] = v;
        else set_err(cnt, PH_EINTERNAL);
    }
    if (threadIdx.x == 0 && s_nan) set_err(cnt, PH_ENAN);
}

// ================================================================ classify 3D ====
// 256 threads; at least seven workgroups per compute unit are asked for, and at 52 registers
// without spills the kernel runs eight (32 waves).  The instance's record is copied before the
// first store, so its fields sit in scalar registers: read after a store, they were vector
// loads into vector registers, and the kernel needed 72 registers and ran seven workgroups,
// 9 % slower on the batched step.  Asking for eight makes the 32 x 8 x 4 tile spill scalar
// registers.
template <int TW, int TH, int TD, typename T, bool H1 = false>
__global__ __launch_bounds__(256, 7) void k_classify3d(const T *__restrict__ imgs,
                                                    uint8_t *__restrict__ ws, int n, Luts lut,
                                                    float *__restrict__ grad) {
    static_assert((TW * TH * TD) % 256 == 0, "tile must be a multiple of the block");
    constexpr int KW = TW + 2, KH = TH + 2, KD = TD + 2;
    constexpr int PW = TW + 1, PH = TH + 1, PD = TD + 1, NP = PW * PH * PD;
    constexpr int NV = TW * TH * TD, NIT = NV / 256;
    // Cube slots: the slot box is PD * PH rows of PW.  A group of PW consecutive threads owns
    // one row, GT rows at a time (slots threadIdx.x + k STT of the thread), so a thread keeps
    // its column and steps its row, and the row's global cube index, by constants.
    constexpr int GT = 256 / PW, STT = GT * PW, NRT = PD * PH, NKT = (NRT + GT - 1) / GT;
    static_assert(NKT * STT >= NP, "cube slots cover the box");
    __shared__ uint32_t skey[KD * KH * KW];
    __shared__ int32_t sp0[NV];
    __shared__ int32_t spT[NKT * STT];
    __shared__ int s_nan;
    __shared__ uint64_t s_scan[4];
    __shared__ int32_t s_base[4];
    __shared__ int s_any[8];
    __shared__ uint8_t s_pext[256];              // [mask nibble << 4 | bits nibble]: compress8 of the two
    __shared__ int2 s_row[NKT * GT];
    __shared__ int2 s_dir[6];
    __shared__ int s_fail;

    const Inst *tab = (const Inst *)ws;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int i = find_inst((const int64_t *)(ws + off_tb3(n)), n, tile);
    // the instance's record copied before the kernel's first store or atomic: its fields load as
    // scalar loads in one batch (after a store they would be vector loads where first used)
    const Inst I = tab[i];
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    const int err = err_word(cnt);
    const int D = I.D, H = I.H, W = I.W;
    const int lt = (int)(tile - I.tile_base);
    const int tz = lt / (I.tx * I.ty), rem = lt - tz * I.tx * I.ty;
    const int ty = rem / I.tx, tx = rem - ty * I.tx;
    const int z0 = tz * TD, y0 = ty * TH, x0 = tx * TW;
    // before the error check: an instance that fails still has its gradient cleared
    if (grad) clear_grad_tile<TW, TH, TD>(grad + I.src_off, I.tfilt, D, H, W, z0, y0, x0);
    if (block_failed_from(err, &s_fail)) return;
    const T *img = imgs + I.src_off;
    int32_t *par0 = arr<int32_t>(ws, I.o_par0);
    int32_t *parT = arr<int32_t>(ws, I.o_parT);
    uint64_t *keyE = arr<uint64_t>(ws, I.o_keyE);
    uint64_t *keyF = arr<uint64_t>(ws, I.o_keyF);
    uint64_t *n0key = arr<uint64_t>(ws, I.o_n0key);
    uint64_t *nTkey = arr<uint64_t>(ws, I.o_nTkey);
    const int64_t HW = (int64_t)H * W;
    const int64_t TH1W1 = (int64_t)(H - 1) * (W - 1);

    if (threadIdx.x == 0) s_nan = 0;
    int nan = 0;
    constexpr int KP = KH * KW;                    // keys in one layer of the halo box
    if constexpr (KP <= 256 && 2 * KP > 256) {
        // One thread per (y, x) of a halo layer, stepping through the KD layers: the layer's
        // z, its clamp and whether it lies in the volume are the same for the whole block, so
        // a key costs its load, its order bits and the inside select.  Clamped loads read a
        // voxel of the instance: a NaN there is one of the instance's own.
        const int yy = threadIdx.x / KW, c = threadIdx.x - yy * KW;
        const int gx = x0 - 1 + c, gy = y0 - 1 + yy;
        auto halo = [&](auto tf) {
            constexpr bool TF = decltype(tf)::value;
            const int sD = D - 2, sH = H - 2, sW = W - 2;   // T: the caller's extents
            const uint32_t off = TF ? (uint32_t)(clamp0(sH - gy, sH - 1) * sW + clamp0(W - 2 - gx, W - 3))
                                    : (uint32_t)(clamp0(gy, H - 1) * W + clamp0(gx, W - 1));
            const bool inyx = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H;
            const bool inner_yx = gx >= 1 && gx <= W - 2 && gy >= 1 && gy <= H - 2;
            float f[KD];
#pragma unroll
            for (int k = 0; k < KD; ++k) {
                const int gz = z0 - 1 + k;
                const uint32_t layer = TF ? (uint32_t)(clamp0(sD - gz, sD - 1) * sH * sW)
                                          : (uint32_t)(clamp0(gz, D - 1) * (int)HW);
                f[k] = (float)img[layer + off];
            }
#pragma unroll
            for (int k = 0; k < KD; ++k) {
                const int gz = z0 - 1 + k;
                float v = f[k];
                if constexpr (TF) v = tf_value(v, inner_yx && gz >= 1 && gz <= D - 2);
                nan |= v != v;
                const uint32_t o = ord32_no_neg0(__float_as_uint(v + 0.0f));
                const bool in = inyx && (unsigned)gz < (unsigned)D;
                skey[threadIdx.x + k * KP] = in ? (o < kOutside ? o : kOutside - 1u) : kOutside;
            }
        };
        if (threadIdx.x < KP) {
            if (I.tfilt) halo(tf_tag<true>{});
            else halo(tf_tag<false>{});
        }
    } else {
        // The halo box is KD * KH rows of KW keys.  A group of KW consecutive threads loads
        // one row, kGroups rows at a time, so a thread keeps its column and steps its row by a
        // constant.  Every load of the thread is issued before the first is used: addresses
        // are clamped into the volume (offsets fit 32 bits: an instance has <= 2^27 voxels)
        // and outside voxels replaced afterwards.  Under the T-filtration the volume is the
        // framed dual one, read through the reflection (tf_value).
        constexpr int kGroups = 256 / KW, NR = KD * KH, NL = (NR + kGroups - 1) / kGroups;
        const int g = threadIdx.x / KW, c = threadIdx.x - g * KW;
        const int gx = x0 - 1 + c;
        const bool inx = (unsigned)gx < (unsigned)W && g < kGroups;
        auto halo = [&](auto tf) {
            constexpr bool TF = decltype(tf)::value;
            const int cx = TF ? clamp0(W - 2 - gx, W - 3) : clamp0(gx, W - 1);   // T: reflected
            float f[NL];
            uint32_t inside = 0;                            // bit k: row g + k kGroups, in the volume
            uint32_t inner = 0;                             // T: and inside the frame
            int zz = g / KH, yy = g - zz * KH;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int gz = z0 - 1 + zz, gy = y0 - 1 + yy;
                if constexpr (TF) {
                    const int sD = D - 2, sH = H - 2, sW = W - 2;   // the caller's extents
                    const int cz = clamp0(sD - gz, sD - 1), cy = clamp0(sH - gy, sH - 1);
                    f[k] = (float)img[(uint32_t)((cz * sH + cy) * sW + cx)];
                    if (gx >= 1 && gx <= W - 2 && gz >= 1 && gz <= D - 2 && gy >= 1 && gy <= H - 2) inner |= 1u << k;
                } else {
                    const int cz = clamp0(gz, D - 1), cy = clamp0(gy, H - 1);
                    f[k] = (float)img[(uint32_t)(cz * (int)HW + cy * W + cx)];
                }
                if (inx && (unsigned)gz < (unsigned)D && (unsigned)gy < (unsigned)H) inside |= 1u << k;
                yy += kGroups % KH;
                zz += kGroups / KH;
                if (yy >= KH) { yy -= KH; ++zz; }
            }
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                if (g >= kGroups || g + k * kGroups >= NR) break;   // threads past the last group load only
                float v = f[k];
                if constexpr (TF) v = tf_value(v, (inner >> k) & 1u);
                const uint32_t o = ord32(__float_as_uint(v));
                const bool in = (inside >> k) & 1u;
                nan |= in && v != v;
                skey[threadIdx.x + k * kGroups * KW] = in ? (o < kOutside ? o : kOutside - 1u) : kOutside;
            }
        };
        if (I.tfilt) halo(tf_tag<true>{});
        else halo(tf_tag<false>{});
    }
    // cube slots start unset (padding rows final); after pass 2 the slots no vertex of the
    // tile wrote get their cube's global index (see is_local).  s_row[r]: global index of the
    // first cube of slot row r (x = x0 - 1) and whether the row lies in the image.
    const int gT = threadIdx.x / PW;
#pragma unroll
    for (int k = 0; k < NKT; ++k)
        if (gT < GT) spT[threadIdx.x + k * STT] = gT + k * GT < NRT ? kUnset : 0;
    for (int r = threadIdx.x; r < NKT * GT; r += 256) {
        const int pz = r / PH, py = r - pz * PH, cz = z0 - 1 + pz, cy = y0 - 1 + py;
        s_row[r] = make_int2(cz * (int)TH1W1 + cy * (W - 1) + x0 - 1,
                             r < NRT && (unsigned)cz < (unsigned)(D - 1) && (unsigned)cy < (unsigned)(H - 1));
    }
    s_pext[threadIdx.x] = lut.pext[threadIdx.x];
    if (threadIdx.x < 6) {
        // direct edge 1 + d (d = 0..5: -z, -y, -x, +x, +y, +z): the step to the neighbour's
        // slot in the tile (low word) and to its voxel in the volume (high word)
        const int d = threadIdx.x, sgn = d < 3 ? -1 : 1, axis = d < 3 ? d : 5 - d;
        const int sdel = axis == 0 ? TH * TW : (axis == 1 ? TW : 1);
        const int gdel = axis == 0 ? (int)HW : (axis == 1 ? W : 1);
        s_dir[d] = make_int2(sgn * sdel, sgn * gdel);
    }
    lds_barrier();
    if (nan) s_nan = 1;

    // pass 1: every vertex of the thread through the table; counts of the cells it keeps
    constexpr uint64_t kValid = 1ull << 63;         // above every field of a 3D entry
    uint64_t ev[NIT];
    uint32_t c_min = 0, c_edge = 0, c_sq = 0, c_root = 0;   // cells the thread keeps, by list
    bool bad = false;                 // a table index out of range (a corrupted table)
    // the 3x3x3 neighbourhood of vertex threadIdx.x + 256 it starts at skey[nb0 + it * kLayers * KH * KW]
    static_assert(256 % (TH * TW) == 0, "a block covers whole tile layers");
    constexpr int kLayers = 256 / (TH * TW);
    const int nb0 = ((threadIdx.x / (TH * TW)) * KH + (threadIdx.x / TW) % TH) * KW + threadIdx.x % TW;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int l = threadIdx.x + it * 256;
        const int lz = l / (TH * TW), lrem = l - lz * TH * TW, ly = lrem / TW, lx = lrem - ly * TW;
        const int gz = z0 + lz, gy = y0 + ly, gx = x0 + lx;
        const uint32_t *nb = skey + nb0 + it * kLayers * KH * KW;
        // branch-free, so the vertices of the thread form one scheduling region: a vertex
        // outside the image (partial tiles) is computed on its clamped halo keys and dropped
        const bool in = gz < D && gy < H && gx < W;
        const uint32_t kv = nb[(KH + 1) * KW + 1];
        // bit code - 1 of raw: the neighbour at kOff[code] comes before v (ties by position);
        // shifted in from the top code down
        uint32_t raw = 0;
#pragma unroll
        for (int code = 26; code >= 1; --code) {        // outside neighbours hold kOutside
            const int dz = kOff[code][0], dy = kOff[code][1], dx = kOff[code][2];
            const bool before = dz < 0 || (dz == 0 && (dy < 0 || (dy == 0 && dx < 0)));
            const uint32_t kn = nb[((1 + dz) * KH + 1 + dy) * KW + 1 + dx];
            raw = before ? shift_in_less<true>(raw, kn, kv) : shift_in_less<false>(raw, kn, kv);
        }
        // level 1 holds the canonical configuration for every raw square set; the cube bits
        // are compressed through its possible-cube mask one nibble at a time
        const uint32_t l1 = lut.l1[raw & (uint32_t)(kL1Size - 1)];
        const uint32_t cb = raw >> 18;
        const uint32_t lo = s_pext[((l1 & 15u) << 4) | (cb & 15u)];
        const uint32_t hi = s_pext[(l1 & 0xF0u) | (cb >> 4)];
        const uint32_t idx2 = (l1 >> 8) + lo + (hi << __popc(l1 & 15u));
        const bool ok = idx2 < (uint32_t)kL3Configs;
        bad |= !ok;                                    // the entry read instead is refused below
        uint64_t e = lut.l2[ok ? idx2 : 0u];
        e = in ? e | kValid : 0;
        if (H1 && in)                                  // 3D H1 looks the configurations up again
            arr<uint16_t>(ws, I.o_cfg3)[(uint32_t)gz * (uint32_t)HW + (uint32_t)(gy * W + gx)] = (uint16_t)(ok ? idx2 : 0u);
        // (an entry outside the volume is 0 and counts nothing)
        c_min += (e & 7u) == kNoDirect ? 1u : 0u;
        c_edge += __popc((uint32_t)(e >> kL3Keep) & 63u);
        c_sq += __popc((uint32_t)(e >> kL3KeepSq) & 4095u);
        c_root += __popc((uint32_t)(e >> kL3Root) & 255u);
        ev[it] = e;
    }
    if (bad) set_err(cnt, PH_EINTERNAL);
    constexpr uint32_t lists8 = CNT_M0 | CNT_E << 8 | CNT_F << 16 | (uint32_t)CNT_MT << 24;
    const uint64_t packed = c_min | c_edge << 16 | (uint64_t)(c_sq | c_root << 16) << 32;
    const uint64_t pre = block_alloc<4>(cnt, lists8, packed, s_scan, s_base);
    int id0 = s_base[0] + (int)(pre & 0xFFFFu);
    int kb = s_base[1] + (int)((pre >> 16) & 0xFFFFu);
    int fb = s_base[2] + (int)((pre >> 32) & 0xFFFFu);
    int rb = s_base[3] + (int)((pre >> 48) & 0xFFFFu);

    // pass 2: forest links, node keys and compact lists at the reserved slots
    const int64_t capN = I.M0cap, capE = I.E, capF = I.F, capT = I.MTcap;
    // vertex threadIdx.x + 256 it lies at (lz0 + it kLayers, ly0, lx0) of the tile; bit d of
    // out_yx: the direct edge 1 + d along y or x leaves the tile
    const int lz0 = threadIdx.x / (TH * TW), ly0 = (threadIdx.x / TW) % TH, lx0 = threadIdx.x % TW;
    const uint32_t out_yx = (ly0 == 0 ? 2u : 0u) | (lx0 == 0 ? 4u : 0u) | (lx0 == TW - 1 ? 8u : 0u) |
                            (ly0 == TH - 1 ? 16u : 0u);
    static_assert(NIT >= 2, "the first and last layers of the tile fall to different iterations");
    const uint32_t out_first = out_yx | (lz0 == 0 ? 1u : 0u);              // it = 0: lz = lz0
    const uint32_t out_last = out_yx | (lz0 == kLayers - 1 ? 32u : 0u);    // it = NIT - 1
#pragma unroll 1                                    // rolled: fewer live registers, more waves per SIMD
    for (int it = 0; it < NIT; ++it) {
        const uint64_t e = ev[it];
        const int l = threadIdx.x + it * 256;
        if (!(e & kValid)) {                       // outside the volume: a final slot value
            sp0[l] = 0;
            continue;
        }
        const int lz = lz0 + it * kLayers, ly = ly0, lx = lx0;
        const int gz = z0 + lz, gy = y0 + ly, gx = x0 + lx;
        const uint32_t kv = skey[((lz + 1) * KH + ly + 1) * KW + lx + 1];
        const uint32_t pv = (uint32_t)gz * (uint32_t)HW + (uint32_t)(gy * W + gx);   // < 2^27
        const uint32_t direct = (uint32_t)(e & 7u);
        const uint32_t keep = (uint32_t)((e >> kL3Keep) & 63u);
        const uint32_t keepsq = (uint32_t)((e >> kL3KeepSq) & 4095u);
        const uint32_t root = (uint32_t)((e >> kL3Root) & 255u);
        const uint32_t present = (uint32_t)((e >> kL3Present) & 255u);
        const uint32_t links = (uint32_t)(e >> kL3Link) & 0xFFFFFFu;

        if (direct == kNoDirect) {
            int64_t id = id0++;
            if (id >= capN) { list_overflow(I, cnt); id = 0; }
            sp0[l] = -(int32_t)(id + 1);
            n0key[id] = make_key(kv, pv, 0);
        } else {
            // a link to the neighbour across the direct edge: its slot, or its voxel when it
            // lies outside the tile
            const uint32_t out = it == 0 ? out_first : (it == NIT - 1 ? out_last : out_yx);
            const int2 dd = s_dir[direct];
            sp0[l] = (out >> direct) & 1u ? (int32_t)pv + dd.y : kLocal | (l + dd.x);
        }
        for (uint32_t m = keep; m; m &= m - 1) {
            const int b = __builtin_ctz(m);
            if (kb < capE) keyE[kb] = make_key(kv, pv, 1 + b); else list_overflow(I, cnt);
            ++kb;
        }
        for (uint32_t m = keepsq; m; m &= m - 1) {
            const int q = __builtin_ctz(m);
            if (fb < capF) keyF[fb] = make_key(kv, pv, 7 + q); else list_overflow(I, cnt);
            ++fb;
        }
        if (present) {
            // the eight cubes around v: octant t = (z y x bits) has its first corner at
            // v - (1,1,1) + t, its slot at pos0 + the octant's slot offset, and lies inside the
            // image when every corner coordinate does
            const int pos0 = (lz * PH + ly) * PW + lx;
            const uint32_t okx = (gx >= 1 ? 1u : 0u) | (gx <= W - 2 ? 2u : 0u);
            const uint32_t oky = (gy >= 1 ? 1u : 0u) | (gy <= H - 2 ? 2u : 0u);
            const uint32_t okz = (gz >= 1 ? 1u : 0u) | (gz <= D - 2 ? 2u : 0u);
            const uint32_t inimg = ((okx & 1u ? 0x55u : 0u) | (okx & 2u ? 0xAAu : 0u)) &
                                   ((oky & 1u ? 0x33u : 0u) | (oky & 2u ? 0xCCu : 0u)) &
                                   ((okz & 1u ? 0x0Fu : 0u) | (okz & 2u ? 0xF0u : 0u));
            // root cubes become dual nodes, every other cube of L(v) a dual link (two loops:
            // roots are rare, so most waves skip the first)
            for (uint32_t m = root & present; m; m &= m - 1) {
                const int b = __builtin_ctz(m);
                if (rb >= capT) { list_overflow(I, cnt); rb = 0; }
                spT[pos0 + oct_slot<PW, PH>(b)] = -(rb + 1);
                nTkey[rb] = make_key(kv, pv, 19 + b);
                ++rb;
            }
            for (uint32_t m = present & ~root; m; m &= m - 1) {
                const int b = __builtin_ctz(m);
                const uint32_t t = (links >> (3 * b)) & 7u;
                spT[pos0 + oct_slot<PW, PH>(b)] = dual_link(inimg, t, kLocal | pos0, oct_slot<PW, PH>(t));
            }
        }
    }
    lds_barrier();

    // the thread's cube slots (column cT of rows gT + k GT)
    const int cT = threadIdx.x - gT * PW;
    int32_t v0[NIT], vT[NKT];
#pragma unroll
    for (int k = 0; k < NKT; ++k) {
        vT[k] = gT < GT ? spT[threadIdx.x + STT * k] : 0;
        if (vT[k] == kUnset) spT[threadIdx.x + STT * k] = vT[k] = s_row[gT + k * GT].x + cT;
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) v0[k] = sp0[threadIdx.x + 256 * k];
    lds_barrier();
    jump_links<NIT, NKT, STT>(sp0, spT, v0, vT, s_any, cnt);

#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int l = threadIdx.x + 256 * k;
        const int lz = l / (TH * TW), lrem = l - lz * TH * TW, ly = lrem / TW, lx = lrem - ly * TW;
        const int gz = z0 + lz, gy = y0 + ly, gx = x0 + lx;
        if (gz < D && gy < H && gx < W) par0[(uint32_t)(gz * (int)HW + gy * W + gx)] = v0[k];
    }
    {
        // the thread's cube slots again; a slot still holding its own index belongs to
        // another tile
        const bool inx = (unsigned)(x0 - 1 + cT) < (unsigned)(W - 1);
#pragma unroll
        for (int k = 0; k < NKT; ++k) {
            if (gT >= GT || gT + k * GT >= NRT) continue;   // no slot, or a padding row
            const int32_t v = vT[k];
            const int2 row = s_row[gT + k * GT];
            const int32_t gidx = row.x + cT;
            if (v != gidx) {
                if (inx && row.y) parT[gidx] = v;
                else set_err(cnt, PH_EINTERNAL);
            }
        }
    }
    if (threadIdx.x == 0 && s_nan) set_err(cnt, PH_ENAN);
}

// ===================================================================== block scan ==
// Exclusive scan of a 0/1 flag over a block of kUfThreads threads; returns the prefix and
// writes the block total to *total.  All threads must call it.
// Barrier of the block; LDS_ONLY: orders LDS accesses only, for phases that exchange nothing
// through global memory (their global stores are not read back inside the kernel).
template <bool LDS_ONLY>
__device__ __forceinline__ void block_sync() {
    if (LDS_ONLY) lds_barrier();
    else __syncthreads();
}

template <bool LDS_ONLY = false>
__device__ __forceinline__ int block_flag_scan(int flag, int *s_wsum, int *total) {
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const uint64_t b = __ballot(flag);
    const int pre = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) s_wsum[wid] = __popcll(b);
    block_sync<LDS_ONLY>();
    const int nw = blockDim.x >> 6;
    int base = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        int v = s_wsum[w];
        if (w < wid) base += v;
        tot += v;
    }
    block_sync<LDS_ONLY>();
    *total = tot;
    return base + pre;
}

// ======================================================================== sort ====
// Sort one list per instance ascending.  which: 0 = KEEP edges (in place), 1 = KEEP squares
// (in place), 2 = H0 node keys copied to a sorted array.  Lists that fit in LDS are sorted
// there by a bitonic network; longer ones are sorted in LDS-sized runs by the same network
// and the runs merged pairwise in global memory, a tile of outputs at a time through LDS
// (merge path: each tile's share of the two runs is found by one binary search per tile).
// Keys are unique (the pixel and code are part of them), so every order is total.

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of s[0, P) ascending (P a power of two, 2 <= P <= 4 * blockDim.x; s holds
// 4 * blockDim.x keys, padding included) by the whole block.  Thread t holds keys 4t .. 4t + 3
// in registers.  A compare-exchange whose partner is in the same thread is done in registers,
// in the same wave by lane shuffles, and only one in another wave goes through LDS: those
// stages alternate between s and s2, with one barrier each.  On return x holds the thread's
// four keys of the sorted sequence.  All threads of the block must call it.
__device__ void bitonic_regs(uint64_t *s, uint64_t *s2, int P, uint64_t (&x)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = s[4 * t + e];
    bool flip = false;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t y[4];
            if (j >= 256) {                          // partner in another wave
                uint64_t *b = flip ? s2 : s;
                flip = !flip;
#pragma unroll
                for (int e = 0; e < 4; ++e) b[4 * t + e] = x[e];
                lds_barrier();
#pragma unroll
                for (int e = 0; e < 4; ++e) y[e] = b[(4 * t + e) ^ j];
            } else if (j >= 4) {                     // another lane of the wave
#pragma unroll
                for (int e = 0; e < 4; ++e) y[e] = shfl_xor64(x[e], j >> 2);
            } else if (j == 2) {
                y[0] = x[2]; y[1] = x[3]; y[2] = x[0]; y[3] = x[1];
            } else {
                y[0] = x[1]; y[1] = x[0]; y[2] = x[3]; y[3] = x[2];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 4 * t + e;
                const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                const bool lt = x[e] < y[e];
                x[e] = keep_min == lt ? x[e] : y[e];
            }
        }
    }
}

// Sort of one list of instance I (WHICH: 0 KEEP edges, 1 KEEP squares, 2 node keys), m keys,
// by the whole block.  The list is a template argument, so each instantiation is straight-line
// code: with the list chosen by a run-time argument, the gfx950 build of an earlier sort kernel
// took the node-key branch without setting the scalar register pair that holds the count's
// address, and loaded the count from near address 0.  The caller loads every count first.
// a list the wide sort kernels take under PH_WIDE (k_sort_runs, k_sort_merge)
__device__ __forceinline__ bool sort_is_wide(const Inst &I, int m) {
    return I.N >= kWideVoxels && m > kSortCap && !I.h1;
}

template <int WHICH>
__device__ __forceinline__ void sort_list(uint8_t *__restrict__ ws, const Inst &I, int32_t *cnt, int m,
                                          uint64_t *s, uint64_t *s2) {
    uint64_t *src = arr<uint64_t>(ws, WHICH == 0 ? I.o_keyE : (WHICH == 1 ? I.o_keyF : I.o_n0key));
    uint64_t *dst = WHICH == 2 ? arr<uint64_t>(ws, I.o_n0sorted) : src;
    const int64_t cap = WHICH == 0 ? I.E : (WHICH == 1 ? I.F : I.M0cap);
    if (m > cap) { if (threadIdx.x == 0) set_err(cnt, PH_EINTERNAL); return; }
    if (m <= 0) return;
    if (m <= kSortCap) {
        static_assert(kSortCap == 4 * kSortThreads, "four keys per thread");
        int P = 2;
        while (P < m) P <<= 1;
        for (int t = threadIdx.x; t < kSortCap; t += blockDim.x) s[t] = t < m ? src[t] : ~0ull;
        __syncthreads();
        uint64_t x[4];
        bitonic_regs(s, s2, P, x);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * (int)threadIdx.x + e < m) dst[4 * threadIdx.x + e] = x[e];
        __syncthreads();                         // s, s2 are free for the caller's next sort
        return;
    }
    // long list: LDS-sized runs, then merge passes between dst and the list's own scratch
    uint64_t *scr = arr<uint64_t>(ws, WHICH == 0 ? I.o_scratch : (WHICH == 1 ? I.o_live : I.o_ra));
    for (int base = 0; base < m; base += kSortCap) {
        const int len = (m - base) < kSortCap ? (m - base) : kSortCap;
        int P = 2;
        while (P < len) P <<= 1;
        for (int t = threadIdx.x; t < kSortCap; t += blockDim.x) s[t] = t < len ? src[base + t] : ~0ull;
        __syncthreads();
        uint64_t x[4];
        bitonic_regs(s, s2, P, x);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * (int)threadIdx.x + e < len) dst[base + 4 * threadIdx.x + e] = x[e];
        __syncthreads();
    }
    const uint64_t *a = dst;
    uint64_t *b = scr;
    int *s_split = (int *)s2;                        // split points of a batch of tiles
    for (int64_t w = kSortCap; w < m; w <<= 1) {
        const int64_t ntiles = (m + kSortCap - 1) / kSortCap;
        for (int64_t tb = 0; tb < ntiles; tb += kSortThreads) {
            const int64_t nb = ntiles - tb < kSortThreads ? ntiles - tb : kSortThreads;
            // tile k starts at output o = (tb + k) T of its pair [ps, ps + 2w): the number of
            // left-run keys among the pair's first o - ps outputs (merge path); k = nb too, the
            // batch's end (used only when the batch's last tile ends inside its pair)
            for (int k = threadIdx.x; k <= nb; k += blockDim.x) {
                const int64_t o = (tb + k) * kSortCap, ps = o / (2 * w) * (2 * w);
                if (o >= m) { s_split[k] = 0; continue; }   // past the list: never read
                const int64_t la = (m - ps) < w ? (m - ps) : w;
                const int64_t lb = (m - ps - la) < w ? (m - ps - la) : w;
                const int64_t d = o - ps;
                int64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (a[ps + mid] < a[ps + w + d - 1 - mid]) lo = mid + 1;
                    else hi = mid;
                }
                s_split[k] = (int)lo;
            }
            __syncthreads();
            for (int64_t k = 0; k < nb; ++k) {
                const int64_t o0 = (tb + k) * kSortCap, ps = o0 / (2 * w) * (2 * w);
                const int64_t la = (m - ps) < w ? (m - ps) : w;
                const int64_t lb = (m - ps - la) < w ? (m - ps - la) : w;
                const int64_t pend = ps + la + lb;
                const int64_t o1 = o0 + kSortCap < pend ? o0 + kSortCap : pend;
                const int64_t i0 = s_split[k], j0 = o0 - ps - i0;
                // the tile's end: the next tile's split inside the same pair, else the pair's end
                const int64_t i1 = o1 == pend ? la : s_split[k + 1];
                const int na = (int)(i1 - i0), nt = (int)(o1 - o0), nb2 = nt - na;
                for (int t = threadIdx.x; t < nt; t += blockDim.x)
                    s[t] = t < na ? a[ps + i0 + t] : a[ps + w + j0 + (t - na)];
                __syncthreads();
                // thread t writes outputs 4t .. 4t + 3 of the tile: its split in LDS, then a
                // short sequential merge
                const int d = 4 * (int)threadIdx.x;
                if (d < nt) {
                    int lo = d > nb2 ? d - nb2 : 0, hi = d < na ? d : na;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s[mid] < s[na + d - 1 - mid]) lo = mid + 1;
                        else hi = mid;
                    }
                    int ia = lo, ib = d - lo;
                    for (int e = 0; e < 4 && d + e < nt; ++e) {
                        const bool take_a = ib >= nb2 || (ia < na && s[ia] < s[na + ib]);
                        b[o0 + d + e] = take_a ? s[ia++] : s[na + ib++];
                    }
                }
                __syncthreads();
            }
        }
        const uint64_t *t = a;
        a = b;
        b = (uint64_t *)t;
    }
    if (a != dst)
        for (int64_t t = threadIdx.x; t < m; t += blockDim.x) dst[t] = a[t];
    __syncthreads();
}

// The three sorts of every instance in one launch: block (i, w) sorts list w of instance i, so
// the lists of all instances are sorted side by side.  A list longer than the LDS merges
// through scratch of its own: the sort scratch (KEEP edges), the live-edge arrays (KEEP
// squares) and the root arrays (node keys), which the union-find only uses afterwards.
// wide: the call sorts long lists with k_sort_runs and k_sort_merge (sort_is_wide), which this
// launch leaves to them.
__global__ __launch_bounds__(kSortThreads) void k_sort_lists(uint8_t *__restrict__ ws, int n, int wide) {
    __shared__ uint64_t s[kSortCap];
    __shared__ uint64_t s2[kSortCap];
    const int i = blockIdx.x, w = blockIdx.y;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    if (block_failed(cnt)) return;
    const int mE = cnt[CNT_E], mF = cnt[CNT_F], mN = cnt[CNT_M0];
    if (wide) {                                  // (an oversized count stays sort_list's error)
        const int m = w == 0 ? mE : (w == 1 ? mF : mN);
        if (sort_is_wide(I, m) && m <= (w == 0 ? I.E : (w == 1 ? I.F : I.M0cap))) return;
    }
    if (w == 0) {
        sort_list<0>(ws, I, cnt, mE, s, s2);
        if (I.h1 && I.ndim == 3) {
            // 3D H1: the sorted position of each vertex's first KEEP edge (a vertex's KEEP edges
            // are adjacent in the sorted list, by code)
            const uint64_t *kE = arr<uint64_t>(ws, I.o_keyE);
            int32_t *kpos = arr<int32_t>(ws, I.o_kpos);
            for (int t = threadIdx.x; t < mE; t += blockDim.x) {
                const uint32_t wv = key_pix(kE[t]);
                if ((t == 0 || key_pix(kE[t - 1]) != wv) && wv < I.N) kpos[wv] = t;
            }
        }
    } else if (w == 1) {
        sort_list<1>(ws, I, cnt, mF, s, s2);
    } else {
        sort_list<2>(ws, I, cnt, mN, s, s2);
    }
}

// ------------------------------------------------------------------ wide sort --
// Under PH_WIDE a list longer than kSortCap keys of an instance of kWideVoxels or more voxels
// (not under PH_H1) is sorted by the whole GPU: k_sort_runs sorts each of its kSortCap-key runs
// in a workgroup of its own, then pass p of k_sort_merge merges the pairs of runs of
// kSortCap << p keys, one workgroup an output tile of kSortCap keys (the merge-path tiles of
// sort_list), from the list's output to its scratch on even passes and back on odd ones.
// The first pass with nothing to merge copies a result left in the scratch back.  Grids
// (blocks, n, 3): blockIdx.z = the list (KEEP edges, KEEP squares, H0 node keys).
struct SortLists {
    uint64_t *src, *dst, *scr;
    int64_t cap;
    int m;
};
__device__ __forceinline__ SortLists sort_lists_of(uint8_t *__restrict__ ws, const Inst &I, const int32_t *cnt, int w) {
    SortLists L;
    L.src = arr<uint64_t>(ws, w == 0 ? I.o_keyE : (w == 1 ? I.o_keyF : I.o_n0key));
    L.dst = w == 2 ? arr<uint64_t>(ws, I.o_n0sorted) : L.src;
    L.scr = arr<uint64_t>(ws, w == 0 ? I.o_scratch : (w == 1 ? I.o_live : I.o_ra));
    L.cap = w == 0 ? I.E : (w == 1 ? I.F : I.M0cap);
    L.m = cnt[w == 0 ? CNT_E : (w == 1 ? CNT_F : CNT_M0)];
    return L;
}

// the list this block works on, or m = 0 (s_flag: the instance failed earlier)
__device__ __forceinline__ SortLists sort_wide_list(uint8_t *__restrict__ ws, int n, int *s_flag) {
    const int i = blockIdx.y;
    const Inst &I = ((const Inst *)ws)[i];
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    if (threadIdx.x == 0) *s_flag = failed(cnt);
    __syncthreads();
    SortLists L = sort_lists_of(ws, I, cnt, blockIdx.z);
    if (*s_flag || !sort_is_wide(I, L.m) || L.m > L.cap) L.m = 0;   // (an oversized count: k_sort_lists reports it)
    return L;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_runs(uint8_t *__restrict__ ws, int n) {
    __shared__ uint64_t s[kSortCap];
    __shared__ uint64_t s2[kSortCap];
    __shared__ int s_flag;
    const SortLists L = sort_wide_list(ws, n, &s_flag);
    const int m = L.m;
    for (int64_t base = (int64_t)blockIdx.x * kSortCap; base < m; base += (int64_t)gridDim.x * kSortCap) {
        const int len = (int)((m - base) < kSortCap ? (m - base) : kSortCap);
        int P = 2;
        while (P < len) P <<= 1;
        for (int t = threadIdx.x; t < kSortCap; t += blockDim.x) s[t] = t < len ? L.src[base + t] : ~0ull;
        __syncthreads();
        uint64_t x[4];
        bitonic_regs(s, s2, P, x);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * (int)threadIdx.x + e < len) L.dst[base + 4 * threadIdx.x + e] = x[e];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_merge(uint8_t *__restrict__ ws, int n, int pass) {
    __shared__ uint64_t s[kSortCap];
    __shared__ int64_t s_split[2];
    __shared__ int s_flag;
    const SortLists L = sort_wide_list(ws, n, &s_flag);
    const int64_t m = L.m;
    if (m == 0) return;
    int np = 0;                                  // merge passes the list needs
    while (((int64_t)kSortCap << np) < m) ++np;
    if (pass >= np) {
        if (pass == np && (np & 1))             // the last merge wrote the scratch
            for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
                L.dst[t] = L.scr[t];
        return;
    }
    const int64_t w = (int64_t)kSortCap << pass;
    const uint64_t *a = pass & 1 ? L.scr : L.dst;
    uint64_t *b = pass & 1 ? L.dst : L.scr;
    const int64_t ntiles = (m + kSortCap - 1) / kSortCap;
    for (int64_t k = blockIdx.x; k < ntiles; k += gridDim.x) {
        // tile k: outputs [o0, o1) of its pair [ps, ps + la + lb); its first and last splits
        // (left-run keys among the pair's first o - ps outputs, by merge path)
        const int64_t o0 = k * kSortCap, ps = o0 / (2 * w) * (2 * w);
        const int64_t la = (m - ps) < w ? (m - ps) : w;
        const int64_t lb = (m - ps - la) < w ? (m - ps - la) : w;
        const int64_t pend = ps + la + lb;
        const int64_t o1 = o0 + kSortCap < pend ? o0 + kSortCap : pend;
        if (threadIdx.x < 2) {
            const int64_t o = threadIdx.x == 0 ? o0 : o1;
            int64_t split = la;
            if (o < pend) {
                const int64_t d = o - ps;
                int64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (a[ps + mid] < a[ps + w + d - 1 - mid]) lo = mid + 1;
                    else hi = mid;
                }
                split = lo;
            }
            s_split[threadIdx.x] = split;
        }
        __syncthreads();
        const int64_t i0 = s_split[0], j0 = o0 - ps - i0;
        const int na = (int)(s_split[1] - i0), nt = (int)(o1 - o0), nb2 = nt - na;
        for (int t = threadIdx.x; t < nt; t += blockDim.x)
            s[t] = t < na ? a[ps + i0 + t] : a[ps + w + j0 + (t - na)];
        __syncthreads();
        // thread t writes outputs 4t .. 4t + 3 of the tile: its split in LDS, then a short
        // sequential merge
        const int d = 4 * (int)threadIdx.x;
        if (d < nt) {
            int lo = d > nb2 ? d - nb2 : 0, hi = d < na ? d : na;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s[mid] < s[na + d - 1 - mid]) lo = mid + 1;
                else hi = mid;
            }
            int ia = lo, ib = d - lo;
            for (int e = 0; e < 4 && d + e < nt; ++e) {
                const bool take_a = ib >= nb2 || (ia < na && s[ia] < s[na + ib]);
                b[o0 + d + e] = take_a ? s[ia++] : s[na + ib++];
            }
        }
        __syncthreads();
    }
}

// ===================================================================== resolve ====
// Follow forest links from entries x0 and x1 to their root node ids, both walks at once so
// their loads are in flight together; -1 (and an error) if a link leaves [0, size) or a node
// id is not below nodes; a walk not run yields 0.
__device__ __forceinline__ void chase2(const int32_t *__restrict__ p, int64_t x0, int64_t x1, bool run0, bool run1,
                                       int64_t size, int nodes, int32_t *cnt, int &r0, int &r1, int &hops) {
    r0 = 0;
    r1 = 0;
    bool a0 = run0, a1 = run1;
    for (int it = 0; (a0 || a1) && it < kMaxChase; ++it) {
        if (a0 && (x0 < 0 || x0 >= size)) { set_err(cnt, PH_EINTERNAL); r0 = -1; a0 = false; }
        if (a1 && (x1 < 0 || x1 >= size)) { set_err(cnt, PH_EINTERNAL); r1 = -1; a1 = false; }
        hops += (int)a0 + (int)a1;
        const int32_t v0 = a0 ? p[x0] : 0, v1 = a1 ? p[x1] : 0;
        if (a0) {
            if (v0 >= 0) x0 = v0;
            else {
                a0 = false;
                r0 = -(v0 + 1);
                if (r0 >= nodes) { set_err(cnt, PH_EINTERNAL); r0 = -1; }
            }
        }
        if (a1) {
            if (v1 >= 0) x1 = v1;
            else {
                a1 = false;
                r1 = -(v1 + 1);
                if (r1 >= nodes) { set_err(cnt, PH_EINTERNAL); r1 = -1; }
            }
        }
    }
    if (a0) { set_err(cnt, PH_EINTERNAL); r0 = -1; }
    if (a1) { set_err(cnt, PH_EINTERNAL); r1 = -1; }
}

// Add a per-thread count to a counter with one atomic per wave (all lanes of the wave call it).
__device__ __forceinline__ void wave_count(int32_t *counter, int v) {
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if (__lane_id() == 0 && v) atomicAdd(counter, v);
}

// H0: the two endpoints of every sorted KEEP edge of instance i, as H0 nodes (local minima).
// The blocks of one instance are blockIdx.x of gridDim.x; the links followed are counted.
__device__ __forceinline__ void resolve_edges(uint8_t *__restrict__ ws, int n, int i) {
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    if (failed(cnt)) return;
    const int m = cnt[CNT_E], M0 = cnt[CNT_M0];
    if (m > I.E) { set_err(cnt, PH_EINTERNAL); return; }
    const uint64_t *keyE = arr<uint64_t>(ws, I.o_keyE);
    const int32_t *par0 = arr<int32_t>(ws, I.o_par0);
    int32_t *ea = arr<int32_t>(ws, I.o_ea), *eb = arr<int32_t>(ws, I.o_eb);
    const int64_t HW = (int64_t)I.H * I.W;
    int hops = 0;
    for (int r0 = blockIdx.x * 256; r0 < m; r0 += gridDim.x * 256) {    // whole waves iterate
        const int r = r0 + threadIdx.x;
        if (r >= m) continue;
        const uint64_t k = keyE[r];
        const int64_t v = key_pix(k);
        const int code = key_code(k);
        if (code < 1 || code > 6) { set_err(cnt, PH_EINTERNAL); ea[r] = eb[r] = -1; continue; }
        const int64_t u = v + off_of(code, 0) * HW + off_of(code, 1) * (int64_t)I.W + off_of(code, 2);
        int a, b;
        chase2(par0, v, u, true, true, I.N, M0, cnt, a, b, hops);
        ea[r] = a;
        eb[r] = b;
    }
    wave_count(&cnt[CNT_HOPS0], hops);
}

// Top dimension: the two cofacets of every facet of instance i walked by the dual union-find,
// as dual nodes (0 = the cell at infinity).  2D walks the KEEP edges that H0 did not use.
__device__ __forceinline__ void resolve_facets(uint8_t *__restrict__ ws, int n, int i) {
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    if (failed(cnt)) return;
    const bool is2d = I.ndim == 2;
    const int m = is2d ? cnt[CNT_E] : cnt[CNT_F], MT = cnt[CNT_MT];
    if (m > (is2d ? I.E : I.F) || MT > I.MTcap) { set_err(cnt, PH_EINTERNAL); return; }
    const uint64_t *key = arr<uint64_t>(ws, is2d ? I.o_keyE : I.o_keyF);
    const int32_t *neg0 = arr<int32_t>(ws, I.o_neg0);
    const int32_t *parT = arr<int32_t>(ws, I.o_parT);
    int32_t *fa = arr<int32_t>(ws, I.o_fa), *fb = arr<int32_t>(ws, I.o_fb);
    const int D = I.D, H = I.H, W = I.W;
    const int64_t HW = (int64_t)H * W;
    int hops = 0;
    for (int r0 = blockIdx.x * 256; r0 < m; r0 += gridDim.x * 256) {    // whole waves iterate
        const int r = r0 + threadIdx.x;
        if (r >= m) continue;
        if (is2d && neg0[r]) { fa[r] = -1; fb[r] = -1; continue; }   // cross-pruned
        const uint64_t k = key[r];
        const int64_t v = key_pix(k);
        const int code = key_code(k);
        if (v >= I.N || (is2d ? (code < 2 || code > 5) : (code < 7 || code > 18))) {
            set_err(cnt, PH_EINTERNAL);
            fa[r] = fb[r] = -1;
            continue;
        }
        const int vz = (int)(v / HW), vrem = (int)(v - vz * HW), vy = vrem / W, vx = vrem - vy * W;
        int axis = -1;
        for (int a = is2d ? 1 : 0; a < 3; ++a)
            if (off_of(code, a) == 0) axis = a;
        int64_t top[2];
        bool in[2];
        for (int t = 0; t < 2; ++t) {
            int o[3] = {off_of(code, 0), off_of(code, 1), off_of(code, 2)};
            o[axis] = t ? 1 : -1;
            // top cell at doubled offset o from 2v: its first corner is v + (o - 1) / 2; a
            // cofacet outside the image is the cell at infinity (node 0)
            const int cz = is2d ? 0 : vz + (o[0] - 1) / 2;
            const int cy = vy + (o[1] - 1) / 2, cx = vx + (o[2] - 1) / 2;
            in[t] = cy >= 0 && cy < H - 1 && cx >= 0 && cx < W - 1 && (is2d || (cz >= 0 && cz < D - 1));
            top[t] = ((int64_t)cz * (H - 1) + cy) * (W - 1) + cx;
        }
        int a, b;
        chase2(parT, top[0], top[1], in[0], in[1], I.T, MT, cnt, a, b, hops);
        fa[r] = a;
        fb[r] = b;
    }
    wave_count(&cnt[CNT_HOPST], hops);
}

// Resolve passes, blockIdx.y = instance.  Stage 0: blockIdx.z = 0 the KEEP edges of every
// instance, z = 1 (with the top dimension) the facets of the volumes, whose dual does not wait
// for H0.  Stage 1: the facets of the images, which need the edges H0 used.
__global__ __launch_bounds__(256) void k_resolve(uint8_t *__restrict__ ws, int n, int stage, int htop) {
    const int i = blockIdx.y;
    const bool vol = ((const Inst *)ws)[i].ndim == 3;
    if (stage == 0 && blockIdx.z == 0) resolve_edges(ws, n, i);
    else if (stage == 0 && htop && vol) resolve_facets(ws, n, i);
    else if (stage == 1 && !vol) resolve_facets(ws, n, i);
}

// ================================================================== union-find ====
// Elder-rule union-find over m sorted edges (H0) or facets taken in decreasing order (dual).
// Exact parallel rounds: every current component computes its minimum outgoing edge (in the
// walk order).  A component whose minimum outgoing edge reaches a component with an elder
// representative dies on that edge.  This is the pairing sequential Kruskal makes: the
// component's own side at that edge is exactly itself (no earlier edge leaves it), and the
// other side already contains the elder representative (components only merge along edges
// taken before their own outgoing ones, so every member is joined to its representative by
// earlier edges).  The globally first live edge always fires, so rounds make progress; the
// few edges left after kMaxRounds are finished in order by one thread, which is exact for
// the same reason.
// Node-array access: LDS arrays are coherent inside the block; global ones are read with
// device-scope loads so a value another wave wrote (or an atomic updated) is never served
// from a stale L1 line.
template <bool GLOBAL>
__device__ __forceinline__ int32_t ld_node(int32_t *p) {
    if (GLOBAL) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <bool GLOBAL>
__device__ __forceinline__ void st_node(int32_t *p, int32_t v) {
    if (GLOBAL) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The round loop.  GN: the node arrays (par, moe) live in global memory, else in LDS; GL: the
// live-edge arrays (walk position q, and the current roots A, B of the edge's two ends) live in
// global memory, else in LDS; KG: the node keys are read from global memory, else copied to
// LDS (s_key).  A fired edge is marked by complementing its q; compaction keeps the edges whose
// ends still lie in different components and moves them down in place.
// cont (global arrays only): the instance went through the wide rounds (k_uf_wide): par,
// the deaths and the killers hold their state, and A[q], B[q] each edge's roots there (A[q] < 0:
// done); the rounds go on from it.
template <bool DUAL, bool GN, bool GL, bool KG = GN>
__device__ __forceinline__ void uf_body(uint8_t *__restrict__ ws, int n, int32_t *par, int32_t *moe,
                                        int32_t *live, int32_t *A, int32_t *B, uint64_t *s_key, int *s_wsum,
                                        bool cont = false) {
    const int i = blockIdx.x;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    const bool is2d = I.ndim == 2;
    const int m = DUAL ? (is2d ? cnt[CNT_E] : cnt[CNT_F]) : cnt[CNT_E];
    const int M = DUAL ? cnt[CNT_MT] : cnt[CNT_M0];
    const int32_t *ea = arr<int32_t>(ws, DUAL ? I.o_fa : I.o_ea);
    const int32_t *eb = arr<int32_t>(ws, DUAL ? I.o_fb : I.o_eb);
    const uint64_t *gkey = arr<uint64_t>(ws, DUAL ? I.o_nTkey : I.o_n0key);
    const uint64_t *nkey = KG ? gkey : s_key;       // node keys, else copied to LDS with the nodes
    int32_t *neg0 = arr<int32_t>(ws, I.o_neg0);
    int32_t *death0 = arr<int32_t>(ws, I.o_death0);
    int32_t *killer = arr<int32_t>(ws, I.o_killer);

    // elder(x, y): x entered earlier in the walk order
    auto elder = [&](int x, int y) -> bool {
        if (DUAL) return x == 0 || (y != 0 && nkey[x] > nkey[y]);
        return nkey[x] < nkey[y];
    };
    auto find = [&](int x) -> int {
        for (int it = 0; it < kMaxChase; ++it) {
            const int p = ld_node<GN>(&par[x]);
            if (p == x) return x;
            const int g = ld_node<GN>(&par[p]);
            if (g != p) st_node<GN>(&par[x], g);       // path halving (any ancestor is valid)
            x = g;
        }
        set_err(cnt, PH_EINTERNAL);
        return x;
    };
    auto edge_of = [&](int q) { return DUAL ? m - 1 - q : q; };
    // all state in LDS: the round barriers order LDS only (the rounds' global stores, the
    // deaths and killers, are each written once and read after the kernel)
    constexpr bool kLds = !GN && !GL;
    auto fire = [&](int dead, int into, int r) {
        st_node<GN>(&par[dead], into);
        if (DUAL) killer[r] = dead;
        else { death0[dead] = r; neg0[r] = 1; }
    };

    for (int x = threadIdx.x; x < M; x += blockDim.x) {
        if (!cont) st_node<GN>(&par[x], x);
        st_node<GN>(&moe[x], kInf);
        if (!KG) s_key[x] = gkey[x];
    }
    if (cont) {
    } else if (DUAL) {
        for (int r = threadIdx.x; r < m; r += blockDim.x) killer[r] = -1;
    } else {
        for (int r = threadIdx.x; r < m; r += blockDim.x) neg0[r] = 0;
        for (int x = threadIdx.x; x < M; x += blockDim.x) death0[x] = -1;
    }
    __syncthreads();                                // the init stores land before any round's

    // live list: walk positions q whose edge joins two different nodes (after the wide
    // rounds: whose edge is not done; compacted in place)
    int L = 0;
    for (int base = 0; base < m; base += blockDim.x) {
        const int q = base + threadIdx.x;
        int flag = 0, a = 0, b = 0;
        if (q < m && cont) {
            a = A[q];
            b = B[q];
            flag = a >= 0 && !(a & kFired);
        } else if (q < m) {
            const int r = edge_of(q);
            a = ea[r];
            b = eb[r];
            flag = a >= 0 && b >= 0 && a < M && b < M && a != b;
        }
        int tot;
        const int pos = block_flag_scan<kLds>(flag, s_wsum, &tot);
        if (flag) { live[L + pos] = q; A[L + pos] = a; B[L + pos] = b; }
        L += tot;
    }
    block_sync<kLds>();

    int round = 0;
    for (; round < kMaxRounds && L > 0; ++round) {
        for (int t = threadIdx.x; t < L; t += blockDim.x) {
            const int q = live[t];
            const int x = find(A[t]), y = find(B[t]);
            A[t] = x;
            B[t] = y;
            if (x != y) { atomicMin(&moe[x], q); atomicMin(&moe[y], q); }
        }
        block_sync<kLds>();
        for (int t = threadIdx.x; t < L; t += blockDim.x) {
            const int x = A[t], y = B[t];
            if (x == y) continue;
            const int q = live[t];
            int dead = -1, into = -1;
            if (ld_node<GN>(&moe[x]) == q && elder(y, x)) { dead = x; into = y; }
            else if (ld_node<GN>(&moe[y]) == q && elder(x, y)) { dead = y; into = x; }
            if (dead >= 0) {
                fire(dead, into, edge_of(q));
                live[t] = ~q;
            }
        }
        block_sync<kLds>();
        for (int t = threadIdx.x; t < L; t += blockDim.x) {
            st_node<GN>(&moe[A[t]], kInf);
            st_node<GN>(&moe[B[t]], kInf);
        }
        block_sync<kLds>();
        int L2 = 0;
        for (int base = 0; base < L; base += blockDim.x) {
            const int t = base + threadIdx.x;
            int flag = 0, q = 0, a = 0, b = 0;
            if (t < L) {
                q = live[t];
                a = A[t];
                b = B[t];
                flag = a != b && q >= 0;
            }
            int tot;
            const int pos = block_flag_scan<kLds>(flag, s_wsum, &tot);   // every read of the chunk is done
            if (flag) { live[L2 + pos] = q; A[L2 + pos] = a; B[L2 + pos] = b; }
            L2 += tot;
        }
        block_sync<kLds>();
        L = L2;
    }
    if (threadIdx.x == 0) {
        cnt[DUAL ? CNT_ROUNDST : CNT_ROUNDS0] = round + (cont ? cnt[DUAL ? CNT_ROUNDST : CNT_ROUNDS0] : 0);
        if (L > 0) cnt[CNT_SEQ] += L;
        for (int t = 0; t < L; ++t) {               // sequential finish, walk order
            const int q = live[t];
            const int x = find(A[t]), y = find(B[t]);
            if (x == y) continue;
            const int dead = elder(y, x) ? x : y, into = dead == x ? y : x;
            fire(dead, into, edge_of(q));
        }
    }
}

// ------------------------------------------------------------- wide union-find --
// Under PH_WIDE an instance of kWideVoxels or more voxels with more nodes than one
// workgroup's LDS holds (kUfLdsNodesOnly) first runs up to kWideRounds of the rounds above
// spread over kWideBlocks workgroups, one phase a launch; k_unionfind then goes on from there
// in one workgroup (uf_body with cont) if edges are left.  Phase 0 of round r counts the
// edges it finds live (CNT_WLIVE0 / CNT_WLIVET + r % 2, one atomic a workgroup); a round that
// finds none ends the work, and the later launches return at once.  An edge keeps its walk position q: A[q], B[q] hold its two
// roots; A[q] = -1 once it is done (both ends in one component), A[q] | kFired in the round it
// fires.  Round r lowers moe_r, one of two node arrays taken in turn (moe, and the live-edge
// array the continuation fills later), to the edges' q.  Phase 0 of round r first restores to
// kInf the entries of the other array that round r - 1 lowered (the two roots each edge still
// names), then finds each live edge's roots and lowers theirs; phase 1 fires each root whose
// minimum edge reaches an elder root.  These are the rounds of uf_body, taken by the whole grid.
__device__ __forceinline__ bool uf_is_wide(const Inst &I, int M, int m) {
    const int64_t L = I.E > I.F ? I.E : I.F;      // the second node array is a live-edge array
    return I.N >= kWideVoxels && M > kUfLdsNodesOnly && M <= L;
}

// phase -1: initialise; 0, 1: the two phases of round `round`.  Grid (kWideBlocks, n, side)
template <bool DUAL>
__device__ __forceinline__ void uf_wide(uint8_t *__restrict__ ws, int n, int phase, int round, int *s_flag) {
    const int i = blockIdx.y;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    const int M = DUAL ? cnt[CNT_MT] : cnt[CNT_M0];
    const int m = DUAL ? (I.ndim == 2 ? cnt[CNT_E] : cnt[CNT_F]) : cnt[CNT_E];
    if (threadIdx.x == 0) *s_flag = failed(cnt);
    lds_barrier();
    if (*s_flag || !uf_is_wide(I, M, m)) return;
    if (M > (DUAL ? I.MTcap : I.M0cap) || m > (DUAL && I.ndim == 3 ? I.F : I.E)) {
        if (threadIdx.x == 0 && blockIdx.x == 0 && phase < 0) set_err(cnt, PH_EINTERNAL);
        return;
    }
    // wlive[r % 2]: nonzero when round r found a live edge.  Phase 1 of round r clears the
    // other slot for round r + 1 (phase 0 of round r read it last); a round that found none
    // leaves both at 0, so every later launch returns here.  One thread of a workgroup reads
    // the flags (a word every workgroup reads at once is a hot spot).
    int32_t *wlive = cnt + (DUAL ? CNT_WLIVET : CNT_WLIVE0);
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (phase >= 0) {
        if (phase == 1 && t0 == 0) __hip_atomic_store(&wlive[(round + 1) & 1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();                             // every thread has read s_flag[0]
        if (threadIdx.x == 0) {
            const int slot = phase == 0 ? (round - 1) & 1 : round & 1;
            s_flag[0] = (phase == 0 && round == 0) ||
                        __hip_atomic_load(&wlive[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        }
        __syncthreads();
        if (!s_flag[0]) return;
    }
    int32_t *par = arr<int32_t>(ws, DUAL ? I.o_ufT : I.o_uf0);
    int32_t *moe_even = arr<int32_t>(ws, DUAL ? I.o_moeT : I.o_moe0);
    int32_t *moe_odd = arr<int32_t>(ws, DUAL ? I.o_live2 : I.o_live);
    int32_t *cur = round & 1 ? moe_odd : moe_even, *prev = round & 1 ? moe_even : moe_odd;
    const int64_t L = I.E > I.F ? I.E : I.F;
    int32_t *A = DUAL ? arr<int32_t>(ws, I.o_scratch) : arr<int32_t>(ws, I.o_ra);
    int32_t *B = DUAL ? arr<int32_t>(ws, I.o_scratch) + L : arr<int32_t>(ws, I.o_rb);
    const uint64_t *nkey = arr<uint64_t>(ws, DUAL ? I.o_nTkey : I.o_n0key);
    int32_t *neg0 = arr<int32_t>(ws, I.o_neg0);
    int32_t *death0 = arr<int32_t>(ws, I.o_death0);
    int32_t *killer = arr<int32_t>(ws, I.o_killer);
    const int stride = gridDim.x * blockDim.x;
    auto edge_of = [&](int q) { return DUAL ? m - 1 - q : q; };
    if (phase < 0) {
        const int32_t *ea = arr<int32_t>(ws, DUAL ? I.o_fa : I.o_ea);
        const int32_t *eb = arr<int32_t>(ws, DUAL ? I.o_fb : I.o_eb);
        if (t0 < 2) wlive[t0] = 0;
        if (t0 == 0) cnt[DUAL ? CNT_ROUNDST : CNT_ROUNDS0] = 0;
        for (int x = t0; x < M; x += stride) {
            par[x] = x;
            moe_even[x] = kInf;
            moe_odd[x] = kInf;
            if (!DUAL) death0[x] = -1;
        }
        for (int q = t0; q < m; q += stride) {
            const int r = edge_of(q), a = ea[r], b = eb[r];
            const bool ok = a >= 0 && b >= 0 && a < M && b < M && a != b;
            A[q] = ok ? a : -1;
            B[q] = b;
            if (DUAL) killer[r] = -1;
            else neg0[r] = 0;
        }
        return;
    }
    auto elder = [&](int x, int y) -> bool {
        if (DUAL) return x == 0 || (y != 0 && nkey[x] > nkey[y]);
        return nkey[x] < nkey[y];
    };
    // Phase 0 changes par only by path halving, which keeps every link pointing to an
    // ancestor, and lowers moe only: a stale read of either (through the workgroup's cache) is
    // an older ancestor or a higher moe, so the roots found and the atomics taken stay right.
    auto find = [&](int x) -> int {
        for (int it = 0; it < kMaxChase; ++it) {
            const int p = ld_node<false>(&par[x]);
            if (p == x) return x;
            const int g = ld_node<false>(&par[p]);
            if (g != p) st_node<true>(&par[x], g);     // path halving (any ancestor is valid)
            x = g;
        }
        set_err(cnt, PH_EINTERNAL);
        return x;
    };
    int live = 0;
    // The eldest node (the cell at infinity; for H0 the node of the least key, first of the
    // sorted node keys) never dies, so its moe is never needed: its component, which grows
    // to hold most edges' ends, would otherwise take one atomic per edge on one word.
    int eldest = 0;
    if (!DUAL) {
        if (threadIdx.x == 0) {
            const uint64_t k0 = arr<uint64_t>(ws, I.o_n0sorted)[0];
            const uint32_t p0 = key_pix(k0);
            const int id = p0 < (uint32_t)I.N ? -(arr<int32_t>(ws, I.o_par0)[p0] + 1) : -1;
            s_flag[1] = id >= 0 && id < M ? id : -1;     // -1: every root takes its atomics
        }
        __syncthreads();
        eldest = s_flag[1];
    }
    for (int q = t0; q < m; q += stride) {
        const int a = A[q];
        if (a < 0) continue;
        if (phase == 0) {
            const int b = B[q];
            if (round > 0) {                        // the entries round - 1 lowered
                prev[a & ~kFired] = kInf;
                prev[b] = kInf;
            }
            if (a & kFired) { A[q] = -1; continue; }
            const int x = find(a), y = find(b);
            if (x == y) { A[q] = -1; continue; }
            A[q] = x;
            B[q] = y;
            ++live;
            // a root's moe is settled early by its first edges: read before the atomic
            if (x != eldest && q < ld_node<false>(&cur[x])) atomicMin(&cur[x], q);
            if (y != eldest && q < ld_node<false>(&cur[y])) atomicMin(&cur[y], q);
        } else {
            const int x = a, y = B[q];
            int dead = -1, into = -1;
            if (cur[x] == q && elder(y, x)) { dead = x; into = y; }
            else if (cur[y] == q && elder(x, y)) { dead = y; into = x; }
            if (dead >= 0) {
                st_node<true>(&par[dead], into);
                const int r = edge_of(q);
                if (DUAL) killer[r] = dead;
                else { death0[dead] = r; neg0[r] = 1; }
                A[q] = a | kFired;
            }
        }
    }
    if (phase == 0 && __syncthreads_or(live > 0) && threadIdx.x == 0) {
        // the flag and the rounds counter, written only while not yet set (read first)
        if (__hip_atomic_load(&wlive[round & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            __hip_atomic_store(&wlive[round & 1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int32_t *rc = &cnt[DUAL ? CNT_ROUNDST : CNT_ROUNDS0];
        if (__hip_atomic_load(rc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < round + 1) atomicMax(rc, round + 1);
    }
}

// blockIdx.y = instance; stage and blockIdx.z choose H0 or the dual as in k_unionfind
__global__ __launch_bounds__(kWideThreads) void k_uf_wide(uint8_t *__restrict__ ws, int n, int stage, int htop,
                                                          int phase, int round) {
    __shared__ int s_flag[2];                    // the instance failed; the eldest H0 node
    const bool vol = ((const Inst *)ws)[blockIdx.y].ndim == 3;
    if (stage == 0 && blockIdx.z == 0) uf_wide<false>(ws, n, phase, round, s_flag);
    else if ((stage == 0 && htop && vol) || (stage == 1 && !vol)) uf_wide<true>(ws, n, phase, round, s_flag);
}

// Instances with at most kUfLdsNodes nodes keep par, moe and the node keys in LDS, and with
// at most kUfLdsEdges edges their live-edge arrays too; up to kUfLdsNodesOnly nodes keep par
// and moe in the whole LDS (keys and live edges in the workspace); larger ones use the
// workspace for everything.  The H0 and dual union-finds of one volume run side by side: the
// dual keeps its live edges in the free second live array and its roots in the sort scratch
// (8 max(L, N) bytes).  s_lds: kUfLdsWords int32 words, 8-byte aligned.
template <bool DUAL>
__device__ __forceinline__ void uf_run(uint8_t *__restrict__ ws, int n, int32_t *s_lds, int *s_wsum, bool wide) {
    const int i = blockIdx.x;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    const int32_t *cnt = (const int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    const int M = DUAL ? cnt[CNT_MT] : cnt[CNT_M0];
    const int m = DUAL ? (I.ndim == 2 ? cnt[CNT_E] : cnt[CNT_F]) : cnt[CNT_E];
    if (block_failed(cnt)) return;
    if (M < 1 || M > (DUAL ? I.MTcap : I.M0cap) || m > (DUAL && I.ndim == 3 ? I.F : I.E)) {
        if (threadIdx.x == 0) set_err((int32_t *)cnt, PH_EINTERNAL);
        return;
    }
    int32_t *gpar = arr<int32_t>(ws, DUAL ? I.o_ufT : I.o_uf0), *gmoe = arr<int32_t>(ws, DUAL ? I.o_moeT : I.o_moe0);
    const int64_t L = I.E > I.F ? I.E : I.F;
    int32_t *glive = arr<int32_t>(ws, DUAL ? I.o_live2 : I.o_live);
    int32_t *ga = DUAL ? arr<int32_t>(ws, I.o_scratch) : arr<int32_t>(ws, I.o_ra);
    int32_t *gb = DUAL ? arr<int32_t>(ws, I.o_scratch) + L : arr<int32_t>(ws, I.o_rb);
    // LDS carve for the small case: par, moe (kUfLdsNodes each), live, A, B (kUfLdsEdges each),
    // then the node keys (8-byte aligned: the offset is even)
    int32_t *s_par = s_lds, *s_moe = s_lds + kUfLdsNodes, *s_live = s_lds + 2 * kUfLdsNodes;
    int32_t *s_a = s_live + kUfLdsEdges, *s_b = s_a + kUfLdsEdges;
    uint64_t *s_key = (uint64_t *)(s_b + kUfLdsEdges);
    static_assert((2 * kUfLdsNodes + 3 * kUfLdsEdges) % 2 == 0, "node keys 8-byte aligned");
    static_assert(2 * kUfLdsNodes + 3 * kUfLdsEdges + 2 * kUfLdsNodes <= kUfLdsWords, "LDS carve");
    if (wide && uf_is_wide(I, M, m)) {
        // the wide rounds' last round found no live edge: nothing is left
        if (cnt[(DUAL ? CNT_WLIVET : CNT_WLIVE0) + ((kWideRounds - 1) & 1)] == 0) return;
        uf_body<DUAL, true, true>(ws, n, gpar, gmoe, glive, ga, gb, nullptr, s_wsum, true);
    }
    else if (M <= kUfLdsNodes && m <= kUfLdsEdges) uf_body<DUAL, false, false>(ws, n, s_par, s_moe, s_live, s_a, s_b, s_key, s_wsum);
    else if (M <= kUfLdsNodes) uf_body<DUAL, false, true>(ws, n, s_par, s_moe, glive, ga, gb, s_key, s_wsum);
    else if (M <= kUfLdsNodesOnly)
        uf_body<DUAL, false, true, true>(ws, n, s_lds, s_lds + kUfLdsNodesOnly, glive, ga, gb, nullptr, s_wsum);
    else uf_body<DUAL, true, true>(ws, n, gpar, gmoe, glive, ga, gb, nullptr, s_wsum);
}

// Union-find passes, blockIdx.x = instance.  Stage 0: blockIdx.y = 0 H0 of every instance,
// y = 1 (with the top dimension) the dual of the volumes; stage 1: the dual of the images.
// wide: the call ran the wide rounds (k_uf_wide) before this launch.
__global__ __launch_bounds__(kUfThreads) void k_unionfind(uint8_t *__restrict__ ws, int n, int stage, int htop, int wide) {
    __shared__ __align__(8) int32_t s_lds[kUfLdsWords];
    __shared__ int s_wsum[kUfThreads / 64];
    const bool vol = ((const Inst *)ws)[blockIdx.x].ndim == 3;
    if (stage == 0 && blockIdx.y == 0) uf_run<false>(ws, n, s_lds, s_wsum, wide != 0);
    else if ((stage == 0 && htop && vol) || (stage == 1 && !vol)) uf_run<true>(ws, n, s_lds, s_wsum, wide != 0);
}

// ======================================================================= 3D H1 ====
// H1 of a volume (Sec. 4.2 steps 4-5): the cells not already paired.  Rows are the positive
// edges; columns the KEEP squares the dual union-find left unpaired (squares paired in H2 are
// dropped, as are zero-persistence pairs inside one lower star).  Every edge paired inside its
// lower star L(w) with a square tau has a reduced column known from the table: the sum of the
// boundaries of the squares of L(w) that tau's relative reduction added (tau's combination),
// whose last entry is that edge.  A column sigma in L(v) starts as the sum of the boundaries of
// its own combination (the squares of L(v) its relative reduction added), which has no entry
// in L(v).  From then on every locally paired entry lies in an earlier lower star, so its
// partner precedes sigma: adding the partner's reduced column is a legal column operation in
// any order.  Each entry that turns present is queued and classified once it comes out of the
// queue; a locally paired one still present gets its partner's reduced column added (which
// removes it and adds only entries below it, so the work ends); entries that can never be a
// pivot (negative edges: paired with their vertex, or H0-negative KEEP edges) are dropped.
// What is left are KEEP edges that H0 left positive: the column's boundary in the complex of
// critical cells.  A standard reduction of those small columns, in square order, then gives
// exactly the pairs of the full boundary-matrix reduction.
//
// One single-wave workgroup per column at a time, 64 queued entries per step; the column is an
// F2 set of edge keys in an open-addressing table in LDS (toggling a key is adding the edge).
constexpr int kH1Slots = 1024;             // table slots (and queue entries) of the first pass
constexpr int kH1BigSlots = 4096;          // the same for the columns the first pass could not hold
constexpr int kH1MaxBoundary = 64;         // entries of one column's boundary in critical cells
constexpr int kH1MaxChunks = 1 << 20;
// A column holds edges by their id, pixel << 5 | code (the low 32 bits of the edge key: the
// pixel is the edge's last vertex, the code 1..6 sits in the low 3 bits); bits 3 and 4 of a
// table entry carry the slot state.  An id is below 2^32 - 1, so the empty slot cannot occur.
constexpr uint32_t kH1Empty = ~0u;
constexpr uint32_t kH1Present = 1u << 3, kH1Final = 1u << 4, kH1Flags = kH1Present | kH1Final;

template <int SLOTS>
__device__ __forceinline__ uint32_t h1_hash(uint32_t id) {
    constexpr int BITS = SLOTS == 512 ? 9 : (SLOTS == 1024 ? 10 : (SLOTS == 2048 ? 11 : 12));
    static_assert((1 << BITS) == SLOTS, "power-of-two table");
    const uint32_t x = (id >> kCodeBits) * 8u + (id & 7u);   // pixel, code
    return (x * 2654435761u) >> (32 - BITS);
}

// The LDS state of one column: an open-addressing table of edge keys (a key's slot keeps its
// state: present in the column, classified, known negative), and a FIFO of keys that turned
// present while unclassified (each is looked at once it comes out).
template <int SLOTS>
struct H1Col {
    uint32_t *tab;
    uint32_t *alt;                 // second table the big tables compact into (unused below 2048)
    uint32_t *queue;
    uint32_t *neg;                 // bit per slot: the key there is a negative edge
    int *used, *tail, *over;
    int head;                      // queue position of the chunk being processed (uniform)

    __device__ __forceinline__ bool is_neg(uint32_t h) const { return (neg[h >> 5] >> (h & 31)) & 1u; }
    __device__ __forceinline__ void enqueue(uint32_t key) {
        const int t = atomicAdd(tail, 1);
        if (t - head >= SLOTS) atomicOr(over, 1);
        else queue[t & (SLOTS - 1)] = key;
    }
    // add edge `key` to the column (toggle its presence); negative edges are left out for good
    __device__ __forceinline__ void toggle(uint32_t key) {
        uint32_t h = h1_hash<SLOTS>(key);
        for (int probe = 0; probe < SLOTS; ++probe, h = (h + 1) & (SLOTS - 1)) {
            uint32_t v = __hip_atomic_load(&tab[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (v == kH1Empty) {
                v = atomicCAS(&tab[h], kH1Empty, key | kH1Present);
                if (v == kH1Empty) {
                    atomicAdd(used, 1);
                    enqueue(key);
                    return;
                }
            }
            if ((v & ~kH1Flags) == key) {
                if ((v & kH1Final) && is_neg(h)) return;
                const uint32_t old = atomicXor(&tab[h], kH1Present);
                if (!(old & kH1Present) && !(old & kH1Final)) enqueue(key);
                return;
            }
        }
        atomicOr(over, 1);
    }
    // slot of `key`, or -1
    __device__ __forceinline__ int find(uint32_t key) const {
        uint32_t h = h1_hash<SLOTS>(key);
        for (int probe = 0; probe < SLOTS; ++probe, h = (h + 1) & (SLOTS - 1)) {
            const uint32_t v = __hip_atomic_load(&tab[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (v == kH1Empty) return -1;
            if ((v & ~kH1Flags) == key) return (int)h;
        }
        return -1;
    }
    __device__ __forceinline__ void reinsert(uint32_t *t, uint32_t x) {
        uint32_t h = h1_hash<SLOTS>(x & ~kH1Flags);
        for (int probe = 0; probe < SLOTS; ++probe, h = (h + 1) & (SLOTS - 1))
            if (atomicCAS(&t[h], kH1Empty, x) == kH1Empty) break;
        atomicAdd(used, 1);
    }
    // rebuild the table with its live entries (present, not negative); all lanes call it
    __device__ __forceinline__ void compact() {
        const int lane = threadIdx.x;
        if constexpr (SLOTS >= 2048) {              // through the second table
            lds_barrier();                          // every lane has read *used
            for (int k = lane; k < SLOTS; k += 64) alt[k] = kH1Empty;
            if (lane == 0) *used = 0;
            lds_barrier();
            for (int k = lane; k < SLOTS; k += 64) {
                const uint32_t x = tab[k];
                if (x != kH1Empty && (x & kH1Present) && !((x & kH1Final) && is_neg(k))) reinsert(alt, x);
            }
            lds_barrier();
            for (int k = lane; k < SLOTS / 32; k += 64) neg[k] = 0;
            uint32_t *t = tab;
            tab = alt;
            alt = t;
            lds_barrier();
            return;
        }
        constexpr int PER = SLOTS / 64;
        uint32_t keep[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = lane + 64 * j;
            const uint32_t x = tab[k];
            keep[j] = (x != kH1Empty && (x & kH1Present) && !((x & kH1Final) && is_neg(k))) ? x : kH1Empty;
        }
        lds_barrier();
#pragma unroll
        for (int j = 0; j < PER; ++j) tab[lane + 64 * j] = kH1Empty;
        for (int k = lane; k < SLOTS / 32; k += 64) neg[k] = 0;
        if (lane == 0) *used = 0;
        lds_barrier();
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (keep[j] != kH1Empty) reinsert(tab, keep[j]);
        lds_barrier();
    }
};

// The voxel values 3D H1 compares: the caller's, or under the T-filtration those of the framed
// dual volume (extents D, H, W), read through the reflection (tf_value).
template <typename T>
struct VoxVals {
    const T *img;
    int tf, D, H, W;
    __device__ __forceinline__ float at(uint32_t p) const {
        if (!tf) return (float)img[p];
        const int HW = H * W, z = (int)(p / (uint32_t)HW), rem = (int)p - z * HW, y = rem / W, x = rem - y * W;
        const bool inner = z >= 1 && z <= D - 2 && y >= 1 && y <= H - 2 && x >= 1 && x <= W - 2;
        const int sD = D - 2, sH = H - 2, sW = W - 2;
        return tf_value(inner ? (float)img[(uint32_t)(((sD - z) * sH + (sH - y)) * sW + (sW - x))] : 0.0f, inner);
    }
};

// order key of voxel p: ord32 of its value, then p (the vertex order of Sec. 2.3)
template <typename T>
__device__ __forceinline__ uint64_t vox_key(const VoxVals<T> &img, uint32_t p) {
    return ((uint64_t)ord32(__float_as_uint(img.at(p))) << 32) | p;
}
// key of the edge between voxels a and b = a + the unit offset of edge code code_ab, from
// their order keys: its last vertex is the later one, the code is seen from there
__device__ __forceinline__ uint64_t edge_key_of(uint64_t ka, uint64_t kb, uint32_t code_ab) {
    const bool a_last = ka > kb;
    const uint64_t k = a_last ? ka : kb;
    return (k & 0xFFFFFFFF00000000ull) | ((k & 0xFFFFFFFFull) << kCodeBits) | (a_last ? code_ab : 7u - code_ab);
}

// Add the boundary of square slot q of L(w) to the column, every occurrence of edge `skip` left
// out: its two edges at w (w is their last vertex) and the two opposite ones, whose last
// vertices are looked up.
template <int SLOTS, typename T>
__device__ __forceinline__ void h1_square(H1Col<SLOTS> &col, const VoxVals<T> &img, uint32_t w, int q, int W, int HW,
                                          uint32_t skip) {
    const int c = 7 + q;
    const int a1 = off_of(c, 0) ? 0 : 1;            // the two axes the square spans, slowest first
    const int a2 = off_of(c, 2) ? 2 : 1;
    const int s1 = off_of(c, a1), s2 = off_of(c, a2);
    const int st1 = a1 == 0 ? HW : W, st2 = a2 == 2 ? 1 : W;
    const uint32_t c1 = s1 < 0 ? 1 + a1 : 6 - a1, c2 = s2 < 0 ? 1 + a2 : 6 - a2;
    const uint32_t pa = (uint32_t)((int)w + s1 * st1), pb = (uint32_t)((int)w + s2 * st2);
    const uint32_t pab = (uint32_t)((int)pa + s2 * st2);
    const uint64_t ka = vox_key(img, pa), kb = vox_key(img, pb), kab = vox_key(img, pab);
    const uint32_t w5 = w << kCodeBits;
    const uint32_t e[4] = {w5 | c1, w5 | c2, (uint32_t)edge_key_of(ka, kab, c2), (uint32_t)edge_key_of(kb, kab, c1)};
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (e[k] != skip) col.toggle(e[k]);
}

// Class of the edge with id `key` (no state bits): 0 negative (paired with its vertex, or a KEEP
// edge H0 used), 1 a KEEP edge left positive by H0 (*rr: its sorted position), 2 paired in its
// lower star (*comb: its partner's combination), -1 inconsistent data.
__device__ __forceinline__ int h1_class(uint32_t key, const uint16_t *cfg3, const int32_t *kpos,
                                        const int32_t *neg0, int64_t N, int mE, const Luts &lut,
                                        uint32_t *comb, int *rr) {
    const uint32_t w = key >> kCodeBits, c = key & 31u;
    if (w >= N || c < 1 || c > 6) return -1;
    const uint32_t cfg = cfg3[w];
    const int32_t kp = kpos[w];                      // meaningful only if w has KEEP edges
    if (cfg >= (uint32_t)kL3Configs) return -1;
    const uint64_t ent = lut.l2[cfg];
    const uint32_t cm = lut.h1e[cfg * 8 + (c - 1)];
    if ((uint32_t)(ent & 7u) == c - 1) return 0;
    const uint32_t keep = (uint32_t)(ent >> kL3Keep) & 63u;
    if ((keep >> (c - 1)) & 1u) {
        const int r = kp + __popc(keep & ((1u << (c - 1)) - 1u));
        if (kp < 0 || r >= mE) return -1;
        *rr = r;
        return neg0[r] ? 0 : 1;
    }
    *comb = cm;
    return cm ? 2 : -1;
}

// One workgroup of 64 threads per column at a time, blockIdx.y = instance.  Pass 0 takes every
// KEEP square in turn (a square paired in H2 is no column: h1n = -1) with tables of kH1Slots;
// a column whose live entries outgrow them is put on the instance's retry list, which pass 1
// goes through with kH1BigSlots.  The column's boundary in critical cells (sorted descending)
// goes to the pool, its start and length to h1b, h1n.
template <typename T, int SLOTS>
__global__ __launch_bounds__(64) void k_h1_morse(const T *__restrict__ imgs, uint8_t *__restrict__ ws, int n,
                                                 Luts lut, int pass) {
    __shared__ uint32_t s_tab[SLOTS];
    __shared__ uint32_t s_tab2[SLOTS >= 2048 ? SLOTS : 1];
    __shared__ uint32_t s_queue[SLOTS];
    __shared__ uint32_t s_neg[SLOTS / 32];
    __shared__ int s_used, s_tail, s_over, s_nb;
    __shared__ int32_t s_bnd[kH1MaxBoundary];
    const int i = blockIdx.y;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    if (I.ndim != 3 || !I.h1) return;
    if (block_failed(cnt)) return;
    const int lane = threadIdx.x;
    const int mF = cnt[CNT_F], mE = cnt[CNT_E];
    if (mF > I.F || mE > I.E) {
        if (lane == 0) set_err(cnt, PH_EINTERNAL);
        return;
    }
    const VoxVals<T> img{imgs + I.src_off, I.tfilt, I.D, I.H, I.W};
    const int W = I.W, HW = I.H * I.W;
    const uint64_t *keyF = arr<uint64_t>(ws, I.o_keyF);
    const int32_t *killer = arr<int32_t>(ws, I.o_killer);
    const uint16_t *cfg3 = arr<uint16_t>(ws, I.o_cfg3);
    const int32_t *kpos = arr<int32_t>(ws, I.o_kpos);
    const int32_t *neg0 = arr<int32_t>(ws, I.o_neg0);
    int32_t *h1b = arr<int32_t>(ws, I.o_h1b), *h1n = arr<int32_t>(ws, I.o_h1n);
    int32_t *pool = arr<int32_t>(ws, I.o_pool);
    int32_t *retry = arr<int32_t>(ws, I.o_retry);
    const int ncols = pass == 0 ? mF : cnt[CNT_H1RETRY];
    H1Col<SLOTS> col{s_tab, s_tab2, s_queue, s_neg, &s_used, &s_tail, &s_over, 0};
    int cols = 0, max_chunks = 0;
    for (int k = blockIdx.x; k < ncols; k += gridDim.x) {
        const int r = pass == 0 ? k : retry[k];
        if (r < 0 || r >= mF) {
            if (lane == 0) set_err(cnt, PH_EINTERNAL);
            return;
        }
        if (pass == 0 && killer[r] >= 0) {           // paired in H2: not a column
            if (lane == 0) h1n[r] = -1;
            continue;
        }
        lds_barrier();                               // the previous column's last reads are done
        col.tab = s_tab;
        col.alt = s_tab2;
        for (int t = lane; t < SLOTS; t += 64) s_tab[t] = kH1Empty;
        for (int t = lane; t < SLOTS / 32; t += 64) s_neg[t] = 0;
        if (lane == 0) { s_used = 0; s_tail = 0; s_over = 0; s_nb = 0; }
        col.head = 0;
        lds_barrier();
        // the column's own combination: the sum of its boundaries leaves L(v)
        const uint64_t ks = keyF[r];
        const uint32_t v = key_pix(ks), cs = key_code(ks);
        bool ok = cs >= 7 && cs <= 18 && v < I.N;
        const uint32_t cfg = ok ? cfg3[v] : 0u;
        ok = ok && cfg < (uint32_t)kL3Configs;
        const uint32_t comb = ok ? lut.h1s[cfg * 16 + (cs - 7)] : 0u;
        ok = ok && ((comb >> (cs - 7)) & 1u);
        if (ok && lane < 12 && ((comb >> lane) & 1u)) h1_square(col, img, v, lane, W, HW, kH1Empty);
        lds_barrier();
        bool bad = __ballot(!ok) != 0;
        int chunk = 0;
        for (; !bad && chunk < kH1MaxChunks; ++chunk) {
            if (s_over) break;                       // uniform: read after a barrier
            if (s_used > SLOTS * 3 / 4) {
                col.compact();
                if (s_used > SLOTS / 2) { if (lane == 0) s_over = 1; lds_barrier(); break; }
            }
            const int tail = s_tail;
            if (col.head >= tail) break;             // every key that turned present was looked at
            const uint32_t key = col.head + lane < tail ? s_queue[(col.head + lane) & (SLOTS - 1)] : kH1Empty;
            lds_barrier();
            bool err = false;
            uint32_t tasks = 0;                          // squares of a claimed entry's partner
            if (key != kH1Empty) {
                const int h = col.find(key);
                const uint32_t x = h >= 0 ? col.tab[h] : 0u;
                if (h >= 0 && (x & kH1Present) && !(x & kH1Final)) {
                    uint32_t cm = 0;
                    int rr = -1;
                    const int cl = h1_class(key, cfg3, kpos, neg0, I.N, mE, lut, &cm, &rr);
                    if (cl == 0) {
                        atomicOr(&s_neg[h >> 5], 1u << (h & 31));
                        atomicOr(&col.tab[h], kH1Final);
                        atomicAnd(&col.tab[h], ~kH1Present);
                    } else if (cl == 1) {
                        atomicOr(&col.tab[h], kH1Final);
                    } else if (cl == 2) {
                        // claim the entry; its partner's reduced column (without it) is added
                        // below, one square per lane
                        const uint32_t old = atomicAnd(&col.tab[h], ~kH1Present);
                        if ((old & kH1Present) && !(old & kH1Final)) tasks = cm;
                    } else {
                        err = true;
                    }
                }
            }
            // the claimed entries' squares, spread over the lanes 64 at a time: square g of the
            // wave's list belongs to the lane whose exclusive prefix is the largest one <= g
            const int ntask = __popc(tasks);
            int off = ntask;                             // inclusive prefix over the lanes
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(off, d, 64);
                if (lane >= d) off += y;
            }
            const int total = __shfl(off, 63, 64);
            off -= ntask;
            for (int r0 = 0; r0 < total; r0 += 64) {
                const int g = r0 + lane;
                int owner = 0;
                for (int st = 32; st > 0; st >>= 1) {
                    const int cand = owner + st < 64 ? owner + st : 63;
                    const int co = __shfl(off, cand, 64);
                    if (owner + st < 64 && co <= g) owner = cand;
                }
                uint32_t m = (uint32_t)__shfl((int)tasks, owner, 64);
                const uint32_t okey = (uint32_t)__shfl((int)key, owner, 64);
                const int kth = g - __shfl(off, owner, 64);
                if (g < total) {
                    for (int j = 0; j < kth; ++j) m &= m - 1;
                    h1_square(col, img, okey >> kCodeBits, __builtin_ctz(m), W, HW, okey);
                }
            }
            col.head = col.head + 64 < tail ? col.head + 64 : tail;
            lds_barrier();
            bad |= __ballot(err) != 0;
        }
        if (!bad && chunk >= kH1MaxChunks) bad = true;
        if (!bad && s_over) {
            if (pass == 0) {                         // too large for these tables: the second pass
                if (lane == 0) retry[atomicAdd(&cnt[CNT_H1RETRY], 1)] = r;
                continue;
            }
            bad = true;
        }
        if (bad) {
            if (lane == 0) set_err(cnt, PH_EINTERNAL);
            return;
        }
        ++cols;
        max_chunks = chunk > max_chunks ? chunk : max_chunks;
        // the entries left are KEEP edges H0 left positive: their sorted positions
        for (int win = 0; win < SLOTS; win += 64) {
            const int h = win + lane;
            const uint32_t x = col.tab[h];
            if (x != kH1Empty && (x & kH1Present) && (x & kH1Final) && !col.is_neg(h)) {
                uint32_t cm = 0;
                int rr = -1;
                const int cl = h1_class(x & ~kH1Flags, cfg3, kpos, neg0, I.N, mE, lut, &cm, &rr);
                const int at = atomicAdd(&s_nb, 1);
                if (cl == 1 && at < kH1MaxBoundary) s_bnd[at] = rr;
                else atomicOr(&s_nb, 1 << 30);       // marks the column bad
            }
        }
        lds_barrier();
        const int nb = s_nb;
        if (nb <= 0 || nb > kH1MaxBoundary) {        // a negative square has a non-empty boundary
            if (lane == 0) set_err(cnt, PH_EINTERNAL);
            return;
        }
        // sort the boundary descending (ascending bitonic over the 64 lanes, stored backwards)
        int x = lane < nb ? s_bnd[lane] : 0x7FFFFFFF;
        for (int kk = 2; kk <= 64; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const int y = __shfl_xor(x, j, 64);
                const bool keep_min = ((lane & j) == 0) == ((lane & kk) == 0);
                x = keep_min ? (x < y ? x : y) : (x > y ? x : y);
            }
        int off = 0;
        if (lane == 0) off = atomicAdd(&cnt[CNT_H1POOL], nb);
        off = __shfl(off, 0, 64);
        if ((int64_t)off + nb > I.pool_cap) {
            if (lane == 0) set_err(cnt, PH_EINTERNAL);
            return;
        }
        if (lane < nb) pool[off + nb - 1 - lane] = x;
        if (lane == 0) { h1b[r] = off; h1n[r] = nb; }
        lds_barrier();
    }
    if (lane == 0 && cols) {
        atomicAdd(&cnt[CNT_H1COLS], cols);
        atomicMax(&cnt[CNT_H1ROUNDS], max_chunks);
    }
}

// Reduction of the H1 columns of one volume per workgroup, in square order.  A column whose
// lowest row appears in no earlier column keeps that row for good ("safe"): it is paired at
// once, in parallel.  The other ("unsafe") columns are reduced together in rounds: each adds
// the column of smallest index that has the same lowest row (its form at the start of the
// round), so every addition takes an earlier column and every column's lowest row only goes
// down; when no two columns share a lowest row the matrix is reduced, and the pairs are those
// of the sequential reduction.  The rounds run in LDS when the instance fits (rows, columns,
// entries), else one thread reduces the unsafe columns in order out of the workspace.
// piv[row] = the column paired with that KEEP edge.
constexpr int kRedRows = 4096;             // KEEP edges of an instance reduced in LDS
constexpr int kRedPool = 6144;             // column entries of one LDS buffer
constexpr int kRedList = 2048;             // unsafe columns held in LDS
constexpr int kRedRounds = 1 << 16;

__device__ __forceinline__ uint64_t red_ref(int r, int off, int len) {    // min by column index
    return ((uint64_t)(uint32_t)r << 32) | ((uint64_t)(uint32_t)off << 16) | (uint32_t)len;
}

__global__ __launch_bounds__(kUfThreads) void k_h1_reduce(uint8_t *__restrict__ ws, int n) {
    __shared__ int s_wsum[kUfThreads / 64];
    __shared__ uint64_t s_claim[kRedRows];          // per row: smallest column (index, start, length) with it lowest
    __shared__ int32_t s_buf[2][kRedPool];          // unsafe columns' entries, this round and the next
    __shared__ int32_t s_ul[kRedList], s_off[kRedList], s_len[kRedList];
    __shared__ int s_top, s_any, s_fail;
    const int i = blockIdx.x;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    if (I.ndim != 3 || !I.h1) return;
    if (block_failed(cnt)) return;
    const int mF = cnt[CNT_F], mE = cnt[CNT_E];
    int32_t *h1b = arr<int32_t>(ws, I.o_h1b), *h1n = arr<int32_t>(ws, I.o_h1n);
    int32_t *piv = arr<int32_t>(ws, I.o_piv), *first = arr<int32_t>(ws, I.o_first);
    int32_t *pool = arr<int32_t>(ws, I.o_pool);
    for (int t = threadIdx.x; t < mE; t += blockDim.x) {
        piv[t] = -1;
        first[t] = 0x7FFFFFFF;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < mF; r += blockDim.x) {
        const int b = h1b[r], m = h1n[r];
        for (int k = 0; m > 0 && k < m; ++k) {
            const int e = pool[b + k];
            if (e < 0 || e >= mE) set_err(cnt, PH_EINTERNAL);
            else atomicMin(&first[e], r);
        }
    }
    __syncthreads();
    // safe columns are paired; the unsafe ones, in order, into the list
    int32_t *list = arr<int32_t>(ws, I.o_ea);         // (H0's endpoints are done; E >= F)
    int L = 0;
    for (int base = 0; base < mF; base += blockDim.x) {
        const int r = base + threadIdx.x;
        int flag = 0;
        if (r < mF && h1n[r] > 0) {
            const int low = pool[h1b[r]];
            if (low >= 0 && low < mE && first[low] == r) piv[low] = r;
            else flag = 1;
        }
        int tot;
        const int pos = block_flag_scan(flag, s_wsum, &tot);
        if (flag) list[L + pos] = r;
        L += tot;
    }
    if (threadIdx.x == 0) cnt[CNT_H1UNSAFE] = L;
    __syncthreads();
    // the unsafe columns' entries into LDS buffer 0 (a block-wide prefix sum of their lengths)
    bool lds = mE <= kRedRows && L <= kRedList;
    if (lds) {
        int at = 0;
        for (int base = 0; base < L; base += blockDim.x) {
            const int u = base + threadIdx.x;
            const int len = u < L ? h1n[list[u]] : 0;
            // exclusive scan of len over the chunk
            int x = len;
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(x, d, 64);
                if (__lane_id() >= d) x += y;
            }
            if (__lane_id() == 63) s_wsum[threadIdx.x >> 6] = x;
            __syncthreads();
            int wbase = 0, tot = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                if (w < (int)(threadIdx.x >> 6)) wbase += s_wsum[w];
                tot += s_wsum[w];
            }
            __syncthreads();
            if (u < L) {
                s_ul[u] = list[u];
                s_off[u] = at + wbase + x - len;
                s_len[u] = len;
            }
            at += tot;
        }
        __syncthreads();                             // the list, starts and lengths are written
        lds = at <= kRedPool;
        if (lds)
            for (int u = 0; u < L; ++u) {            // every thread copies its share of each column
                const int b = h1b[s_ul[u]];
                for (int k = threadIdx.x; k < s_len[u]; k += blockDim.x) s_buf[0][s_off[u] + k] = pool[b + k];
            }
        __syncthreads();
    }
    if (lds) {
        int cur = 0, round = 0;
        for (; round < kRedRounds; ++round) {
            // claims: for each unsafe column's lowest row, the smallest unsafe column with it
            for (int u = threadIdx.x; u < L; u += blockDim.x) s_claim[s_buf[cur][s_off[u]]] = ~0ull;
            if (threadIdx.x == 0) { s_top = 0; s_any = 0; s_fail = 0; }
            __syncthreads();
            for (int u = threadIdx.x; u < L; u += blockDim.x)
                atomicMin((unsigned long long *)&s_claim[s_buf[cur][s_off[u]]],
                          (unsigned long long)red_ref(s_ul[u], s_off[u], s_len[u]));
            __syncthreads();
            // each column adds the safe pivot of its lowest row if there is one, else the
            // claimant when that is an earlier column; the result goes to the other buffer
            for (int u = threadIdx.x; u < L; u += blockDim.x) {
                const int32_t *A = s_buf[cur] + s_off[u];
                const int na = s_len[u], low = A[0], r = s_ul[u];
                const int sp = piv[low];             // a safe column with this lowest row
                const uint64_t cl = s_claim[low];
                const int cr = (int)(cl >> 32);
                const int32_t *C = nullptr;
                int nc = 0;
                if (sp >= 0) { C = pool + h1b[sp]; nc = h1n[sp]; }
                else if (cr < r) { C = s_buf[cur] + (int)((cl >> 16) & 0xFFFFu); nc = (int)(cl & 0xFFFFu); }
                const int room = na + nc;
                const int dst = atomicAdd(&s_top, room);
                if (dst + room > kRedPool) { s_fail = 1; continue; }
                int32_t *B = s_buf[cur ^ 1] + dst;
                int a = 0, k = 0, nb = 0;
                while (a < na || k < nc) {           // A + C over F2, both descending
                    const int32_t ck = k < nc ? C[k] : -1;
                    if (k >= nc || (a < na && A[a] > ck)) B[nb++] = A[a++];
                    else if (a >= na || ck > A[a]) { B[nb++] = ck; ++k; }
                    else { ++a; ++k; }
                }
                if (nb == 0) s_fail = 2;             // a negative square reduces to a non-zero column
                if (nc) s_any = 1;
                s_off[u] = dst;
                s_len[u] = nb;
            }
            __syncthreads();
            if (s_fail) break;
            cur ^= 1;
            if (!s_any) break;
            __syncthreads();
        }
        if (s_fail == 2 || round >= kRedRounds) {
            if (threadIdx.x == 0) set_err(cnt, PH_EINTERNAL);
            return;
        }
        if (!s_fail) {
            // reduced: the lowest rows are distinct
            for (int u = threadIdx.x; u < L; u += blockDim.x) piv[s_buf[cur][s_off[u]]] = s_ul[u];
            if (threadIdx.x == 0) cnt[CNT_H1ADDS] = round;
            return;
        }
        // out of LDS room: the one-by-one pass below starts again from the columns in the
        // workspace (the rounds wrote nothing there, and piv holds the safe pivots only)
    }
    if (threadIdx.x != 0) return;
    // one thread, in order, out of the workspace: two work buffers of up to mE entries in the
    // sort scratch (2 max(E, F, N) int32, free now)
    int32_t *A = arr<int32_t>(ws, I.o_scratch), *B = A + I.E;
    int adds = 0;
    for (int u = 0; u < L; ++u) {
        const int r = list[u];
        int na = h1n[r];
        for (int k = 0; k < na; ++k) A[k] = pool[h1b[r] + k];
        bool changed = false;
        for (int it = 0; na > 0 && it < kMaxChase; ++it) {
            const int low = A[0];
            const int j = piv[low];
            if (j < 0) break;
            // A := A + column j over F2, both descending
            const int *C = pool + h1b[j];
            const int nc = h1n[j];
            int a = 0, c = 0, nb = 0;
            while (a < na || c < nc) {
                if (c >= nc || (a < na && A[a] > C[c])) B[nb++] = A[a++];
                else if (a >= na || C[c] > A[a]) B[nb++] = C[c++];
                else { ++a; ++c; }
            }
            int32_t *t = A; A = B; B = t;
            na = nb;
            changed = true;
            ++adds;
        }
        if (na <= 0) { set_err(cnt, PH_EINTERNAL); return; }
        if (changed) {
            const int off = atomicAdd(&cnt[CNT_H1POOL], na);
            if ((int64_t)off + na > I.pool_cap) { set_err(cnt, PH_EINTERNAL); return; }
            for (int k = 0; k < na; ++k) pool[off + k] = A[k];
            h1b[r] = off;
            h1n[r] = na;
        }
        piv[A[0]] = r;
    }
    cnt[CNT_H1ADDS] = adds;
}

// ====================================================================== output ====
__device__ __forceinline__ int64_t cell_index(const Inst &I, int64_t v, int code) {
    const int64_t HW = (int64_t)I.H * I.W;
    const int64_t z = v / HW, rem = v - z * HW, y = rem / I.W, x = rem - y * I.W;
    const int64_t Z = 2 * z + off_of(code, 0), Y = 2 * y + off_of(code, 1), X = 2 * x + off_of(code, 2);
    return (Z * (2 * (int64_t)I.H - 1) + Y) * (2 * (int64_t)I.W - 1) + X;
}

// An instance under PH_WIDE of kWideVoxels or more voxels (not under PH_H1) has its pairs
// written by the whole GPU: mode 1 (grid (kWideBlocks, n)) counts the pairs of every chunk of
// kUfThreads list entries of each section into the live-edge array (free once the union-finds
// are done), k_output_scan turns the counts into each chunk's first position and the section
// totals (CNT_OSEC0, CNT_OSECT), and mode 2 (the same grid) writes every chunk's pairs there.
// Mode 0 (grid n) writes the other instances' pairs as one workgroup and, for the wide ones,
// only their count and status.
__device__ __forceinline__ bool out_is_wide(const Inst &I, uint32_t flags) {
    return (flags & PH_WIDE) && I.N >= kWideVoxels && !I.h1;
}

__global__ __launch_bounds__(kUfThreads) void k_output(const void *__restrict__ imgs,
                                                      uint8_t *__restrict__ ws, int n, uint32_t flags,
                                                      ph_pairs out, int64_t *__restrict__ d_counts,
                                                      int32_t *__restrict__ d_status, int mode) {
    __shared__ int s_wsum[kUfThreads / 64];
    const int i = mode == 0 ? blockIdx.x : blockIdx.y;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    const bool wide = out_is_wide(I, flags);
    if (mode != 0 && !wide) return;
    // pixel value as float32, from the caller's input of the element type the flags name
    auto img = [&](int64_t p) -> float {
        const int64_t q = I.src_off + p;
        if (flags & PH_IN_U8) return (float)((const uint8_t *)imgs)[q];
        if (flags & PH_IN_U16) return (float)((const uint16_t *)imgs)[q];
        return ((const float *)imgs)[q];
    };
    const int32_t *par0 = arr<int32_t>(ws, I.o_par0);
    const int32_t *death0 = arr<int32_t>(ws, I.o_death0);
    const int32_t *killer = arr<int32_t>(ws, I.o_killer);
    const uint64_t *keyE = arr<uint64_t>(ws, I.o_keyE);
    const uint64_t *n0s = arr<uint64_t>(ws, I.o_n0sorted);
    const uint64_t *nTkey = arr<uint64_t>(ws, I.o_nTkey);
    const bool is2d = I.ndim == 2;
    const uint64_t *fkey = arr<uint64_t>(ws, is2d ? I.o_keyE : I.o_keyF);
    const int M0 = cnt[CNT_M0], MT = cnt[CNT_MT], mE = cnt[CNT_E];
    const int mf = is2d ? cnt[CNT_E] : cnt[CNT_F];
    const int64_t cap = I.out_cap, o = I.out_off;
    int64_t P = 0;
    if (block_failed(cnt)) {
        if (threadIdx.x == 0 && mode == 0) { d_counts[i] = 0; d_status[i] = cnt[CNT_ERR]; }
        return;
    }
    // chunks of kUfThreads entries: this block's first and step (mode 0: all, in order);
    // wide: per-chunk counts, then first positions, H0 section first (ch0), then the top's (chT)
    const int c_first = mode == 0 ? 0 : blockIdx.x, c_step = mode == 0 ? 1 : gridDim.x;
    int32_t *ch0 = arr<int32_t>(ws, I.o_live);
    int32_t *chT = ch0 + (M0 + kUfThreads - 1) / kUfThreads;
    // a pixel index and a cell code read back from a key must name a cell of this instance
    auto key_ok = [&](uint64_t k, int lo, int hi) {
        const int c = (int)key_code(k);
        return key_pix(k) < (uint64_t)I.N && c >= lo && c <= hi;
    };

    // T-filtration: the V pairs are those of the framed dual image (extents D, H, W; the
    // caller's are sD, sH, sW).  Its pixel p is the caller's pixel at the point reflection
    // (-1 on the frame); its doubled-grid coordinate X on an axis is the T coordinate 2s+1-X.
    const bool tf = (flags & PH_TFILT) != 0;
    const bool vol = I.ndim == 3;
    const int64_t sD = vol ? I.D - 2 : 1, sH = I.H - 2, sW = I.W - 2;
    auto src_px = [&](int64_t v) -> int32_t {
        const int64_t HW = (int64_t)I.H * I.W;
        const int64_t z = v / HW, rem = v - z * HW, y = rem / I.W, x = rem - y * I.W;
        if ((vol && (z < 1 || z > I.D - 2)) || y < 1 || y > I.H - 2 || x < 1 || x > I.W - 2) return -1;
        return (int32_t)((((vol ? sD - z : 0) * sH) + (sH - y)) * sW + (sW - x));
    };
    auto t_cell = [&](int64_t v, int code) -> int64_t {
        const int64_t HW = (int64_t)I.H * I.W;
        const int64_t z = v / HW, rem = v - z * HW, y = rem / I.W, x = rem - y * I.W;
        const int64_t Z = vol ? 2 * sD + 1 - (2 * z + off_of(code, 0)) : 0;
        const int64_t Y = 2 * sH + 1 - (2 * y + off_of(code, 1)), X = 2 * sW + 1 - (2 * x + off_of(code, 2));
        if (Z < 0 || Z > 2 * sD || Y < 0 || Y > 2 * sH || X < 0 || X > 2 * sW) return -1;
        return (Z * (2 * sH + 1) + Y) * (2 * sW + 1) + X;
    };

    auto put = [&](int64_t pos, int dim, float bv, float dv, int64_t bc, int32_t bpix, int64_t dc, int32_t dpix) {
        if (pos >= cap) return;
        const int64_t j = o + pos;
        out.dim[j] = (int8_t)dim;
        out.birth[j] = bv;
        out.death[j] = dv;
        out.birth_cell[j] = bc;
        out.death_cell[j] = dc;
        out.birth_vertex[j] = bpix;
        out.death_vertex[j] = dpix;
    };
    const float kInf = __int_as_float(0x7f800000);
    // A section's k-th pair (in the order of its list) goes to start + k, or, with rev >= 0
    // pairs in the section, to start + rev - 1 - k.  With write false the section only counts.
    auto place = [](int64_t start, int64_t rev, int64_t k) { return rev >= 0 ? start + rev - 1 - k : start + k; };

    // H0 pairs of the V complex, by birth key (under the T-filtration: its top pairs)
    auto sec_h0 = [&](bool write, int64_t start, int64_t rev) -> int64_t {
        int64_t Q = 0;
        for (int base = c_first * blockDim.x; base < M0; base += c_step * blockDim.x) {
            const int j = base + threadIdx.x;
            int flag = 0;
            uint64_t nk = 0, ek = 0;
            int d = -1;
            if (j < M0) {
                nk = n0s[j];
                const int32_t pv = key_ok(nk, 0, 0) ? par0[key_pix(nk)] : 0;
                const int id = -(pv + 1);
                if (pv >= 0 || id >= M0) { set_err(cnt, PH_EINTERNAL); }
                else {
                    d = death0[id];
                    if (d < 0) flag = !tf;                    // essential (the frame's, under T)
                    else if (d >= mE || !key_ok(ek = keyE[d], 1, 6)) set_err(cnt, PH_EINTERNAL);
                    else flag = key_ord(ek) != key_ord(nk);
                }
            }
            int tot;
            const int pos = block_flag_scan(flag, s_wsum, &tot);
            if (mode == 1) {
                if (threadIdx.x == 0) ch0[base / blockDim.x] = tot;
                continue;
            }
            if (mode == 2) Q = ch0[base / blockDim.x];
            if (flag && write) {
                const int32_t bp = (int32_t)key_pix(nk);
                const int64_t at = place(start, rev, Q + pos);
                if (d < 0) put(at, 0, img(bp), kInf, cell_index(I, bp, 0), bp, -1, -1);
                else if (!tf) {
                    const int32_t dp = (int32_t)key_pix(ek);
                    put(at, 0, img(bp), img(dp), cell_index(I, bp, 0), bp, cell_index(I, dp, key_code(ek)), dp);
                } else {
                    const int32_t dp = (int32_t)key_pix(ek), sb = src_px(dp), sd = src_px(bp);
                    const int64_t cb = t_cell(dp, key_code(ek)), cd = t_cell(bp, 0);
                    if (sb < 0 || sd < 0 || cb < 0 || cd < 0) set_err(cnt, PH_EINTERNAL);
                    else put(at, I.ndim - 1, img(sb), img(sd), cb, sb, cd, sd);
                }
            }
            Q += tot;
        }
        return Q;
    };
    // top-dimension pairs of the V complex, by birth key (under the T-filtration: its H0
    // pairs; the one born on the frame is the essential class)
    auto sec_top = [&](bool write, int64_t start, int64_t rev) -> int64_t {
        int64_t Q = 0;
        for (int base = c_first * blockDim.x; base < mf; base += c_step * blockDim.x) {
            const int r = base + threadIdx.x;
            int flag = 0;
            uint64_t fk = 0, tk = 0;
            if (r < mf) {
                const int x = killer[r];
                if (x >= MT || x == 0) set_err(cnt, PH_EINTERNAL);
                else if (x > 0) {
                    fk = fkey[r];
                    tk = nTkey[x];
                    if (!key_ok(fk, is2d ? 2 : 7, is2d ? 5 : 18) || !key_ok(tk, is2d ? 11 : 19, is2d ? 14 : 26))
                        set_err(cnt, PH_EINTERNAL);
                    else flag = key_ord(fk) != key_ord(tk);
                }
            }
            int tot;
            const int pos = block_flag_scan(flag, s_wsum, &tot);
            if (mode == 1) {
                if (threadIdx.x == 0) chT[base / blockDim.x] = tot;
                continue;
            }
            if (mode == 2) Q = chT[base / blockDim.x];
            if (flag && write) {
                const int32_t bp = (int32_t)key_pix(fk), dp = (int32_t)key_pix(tk);
                const int64_t at = place(start, rev, Q + pos);
                if (!tf) {
                    put(at, I.ndim - 1, img(bp), img(dp), cell_index(I, bp, key_code(fk)), bp,
                        cell_index(I, dp, key_code(tk)), dp);
                } else {
                    const int32_t sb = src_px(dp), sd = src_px(bp);
                    const int64_t cb = t_cell(dp, key_code(tk));
                    if (sb < 0 || cb < 0) set_err(cnt, PH_EINTERNAL);
                    else if (sd < 0) put(at, 0, img(sb), kInf, cb, sb, -1, -1);
                    else {
                        const int64_t cd = t_cell(bp, key_code(fk));
                        if (cd < 0) set_err(cnt, PH_EINTERNAL);
                        else put(at, 0, img(sb), img(sd), cb, sb, cd, sd);
                    }
                }
            }
            Q += tot;
        }
        return Q;
    };

    // H1 pairs of a volume (KEEP edge r paired with column piv[r]), by birth key (under the
    // T-filtration: its H1 pairs, the dual of each, by death key)
    const bool h1 = I.h1 && vol;
    const int32_t *piv = h1 ? arr<int32_t>(ws, I.o_piv) : nullptr;
    auto sec_h1 = [&](bool write, int64_t start, int64_t rev) -> int64_t {
        int64_t Q = 0;
        for (int base = 0; base < mE; base += blockDim.x) {
            const int r = base + threadIdx.x;
            int flag = 0;
            uint64_t ek = 0, sk = 0;
            if (r < mE) {
                const int j = piv[r];
                if (j >= mf) set_err(cnt, PH_EINTERNAL);
                else if (j >= 0) {
                    ek = keyE[r];
                    sk = fkey[j];
                    if (!key_ok(ek, 1, 6) || !key_ok(sk, 7, 18)) set_err(cnt, PH_EINTERNAL);
                    else flag = key_ord(ek) != key_ord(sk);
                }
            }
            int tot;
            const int pos = block_flag_scan(flag, s_wsum, &tot);
            if (flag && write) {
                const int32_t bp = (int32_t)key_pix(ek), dp = (int32_t)key_pix(sk);
                const int64_t at = place(start, rev, Q + pos);
                if (!tf) {
                    put(at, 1, img(bp), img(dp), cell_index(I, bp, key_code(ek)), bp, cell_index(I, dp, key_code(sk)), dp);
                } else {
                    const int32_t sb = src_px(dp), sd = src_px(bp);
                    const int64_t cb = t_cell(dp, key_code(sk)), cd = t_cell(bp, key_code(ek));
                    if (sb < 0 || sd < 0 || cb < 0 || cd < 0) set_err(cnt, PH_EINTERNAL);
                    else put(at, 1, img(sb), img(sd), cb, sb, cd, sd);
                }
            }
            Q += tot;
        }
        return Q;
    };

    if (wide) {
        // section sizes from k_output_scan (mode 1 counts; mode 0 only reports)
        const int64_t nh0 = cnt[CNT_OSEC0], ntop = cnt[CNT_OSECT];
        if (mode == 1) {
            if (flags & (tf ? PH_HTOP : PH_H0)) sec_h0(false, 0, -1);
            if (flags & (tf ? PH_H0 : PH_HTOP)) sec_top(false, 0, -1);
            return;
        }
        if (!tf) {
            const int64_t a0 = (flags & PH_H0) ? nh0 : 0;
            if (mode == 2) {
                if (flags & PH_H0) sec_h0(true, 0, -1);
                if (flags & PH_HTOP) sec_top(true, a0, -1);
                return;
            }
            P = a0 + ((flags & PH_HTOP) ? ntop : 0);
        } else {
            const int64_t c0 = (flags & PH_H0) ? ntop : 0, ct = (flags & PH_HTOP) ? nh0 : 0;
            if (mode == 2) {
                if (flags & PH_H0) sec_top(true, 0, c0);
                if (flags & PH_HTOP) sec_h0(true, c0, ct);
                return;
            }
            P = c0 + ct;
        }
    } else if (!tf) {
        if (flags & PH_H0) P += sec_h0(true, P, -1);
        if (h1) P += sec_h1(true, P, -1);
        if (flags & PH_HTOP) P += sec_top(true, P, -1);
    } else {
        // T order: by dimension, then by death key, so each section is written backwards
        const int64_t c0 = (flags & PH_H0) ? sec_top(false, 0, -1) : 0;
        const int64_t c1 = h1 ? sec_h1(false, 0, -1) : 0;
        const int64_t ct = (flags & PH_HTOP) ? sec_h0(false, 0, -1) : 0;
        if (flags & PH_H0) sec_top(true, 0, c0);
        if (h1) sec_h1(true, c0, c1);
        if (flags & PH_HTOP) sec_h0(true, c0 + c1, ct);
        P = c0 + c1 + ct;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        d_counts[i] = P;
        int st = __hip_atomic_load(&cnt[CNT_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (st == 0 && P > cap) st = PH_ECAPACITY;
        d_status[i] = st;
    }
}

// Between modes 1 and 2 of k_output: each wide instance's chunk counts become the chunks'
// first positions inside their section (exclusive sums), and the section totals go to
// CNT_OSEC0 (H0 list) and CNT_OSECT (top list).  One workgroup an instance.
__global__ __launch_bounds__(kUfThreads) void k_output_scan(uint8_t *__restrict__ ws, int n, uint32_t flags) {
    __shared__ int32_t s_w[kUfThreads / 64];
    __shared__ int64_t s_run;
    const int i = blockIdx.x;
    const Inst I = ((const Inst *)ws)[i];           // one batch of loads, before any atomic
    int32_t *cnt = (int32_t *)(ws + off_cnt(n)) + i * CNT_WORDS;
    if (!out_is_wide(I, flags) || block_failed(cnt)) return;
    const int M0 = cnt[CNT_M0], mf = I.ndim == 2 ? cnt[CNT_E] : cnt[CNT_F];
    const int n0 = (M0 + kUfThreads - 1) / kUfThreads, nt = (mf + kUfThreads - 1) / kUfThreads;
    int32_t *ch = arr<int32_t>(ws, I.o_live);
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    for (int sec = 0; sec < 2; ++sec) {
        int32_t *c = sec == 0 ? ch : ch + n0;
        const int nc = sec == 0 ? n0 : nt;
        if (threadIdx.x == 0) s_run = 0;
        __syncthreads();
        for (int base = 0; base < nc; base += blockDim.x) {
            const int k = base + threadIdx.x;
            const uint32_t v = k < nc ? (uint32_t)c[k] : 0u;
            const uint32_t incl = wave_incl_sum(v);
            if (lane == 63) s_w[wid] = (int32_t)incl;
            __syncthreads();
            int32_t before = 0, total = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                if (w < wid) before += s_w[w];
                total += s_w[w];
            }
            const int64_t run = s_run;
            if (k < nc) c[k] = (int32_t)(run + before + incl - v);
            __syncthreads();                     // every thread has read s_w and s_run
            if (threadIdx.x == 0) s_run = run + total;
            __syncthreads();
        }
        if (threadIdx.x == 0) cnt[sec == 0 ? CNT_OSEC0 : CNT_OSECT] = (int32_t)s_run;
        __syncthreads();
    }
}

// ==================================================================== backward ====
__global__ void k_zero(float *__restrict__ g, int64_t nv) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nv; t += (int64_t)gridDim.x * blockDim.x)
        g[t] = 0.0f;
}

__global__ void k_scatter(ph_pairs pr, const int64_t *__restrict__ d_out_off,
                          const int64_t *__restrict__ d_counts, const float *__restrict__ gb,
                          const float *__restrict__ gd, float *__restrict__ g,
                          const int64_t *__restrict__ d_img_off, int n, int64_t total) {
    const int i = blockIdx.y;
    const int64_t nvox = (i + 1 < n ? d_img_off[i + 1] : total) - d_img_off[i];
    const int64_t o = d_out_off[i];
    int64_t cnt = d_counts[i];
    const int64_t cap = d_out_off[i + 1] - o;
    if (cnt > cap) cnt = cap;
    float *gi = g + d_img_off[i];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < cnt; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = o + t;
        const int32_t bv = pr.birth_vertex[j], dv = pr.death_vertex[j];
        if (bv >= 0 && bv < nvox) atomicAdd(&gi[bv], gb[j]);
        if (dv >= 0 && dv < nvox) atomicAdd(&gi[dv], gd[j]);
    }
}

// ================================================================== host side ====
namespace {

std::once_flag g_lut_once;
int g_lut_status = PH_OK;
uint32_t g_h_lut2d[256];
std::vector<uint32_t> g_h_l1;
std::vector<uint64_t> g_h_l2;
std::vector<uint16_t> g_h_h1e, g_h_h1s;
int g_cfg2d = 0, g_cfg3d = 0;
std::mutex g_dev_mu;
bool g_dev_ready[64] = {false};
Luts g_dev_lut[64];                 // per-device table buffers, kept until the process ends

void build_host_luts() {
    char err[256] = {0};
    g_h_l1.assign(kL1Size, 0);
    g_h_l2.assign(kL3Configs, 0);
    g_h_h1e.assign((size_t)kL3Configs * 8, 0);
    g_h_h1s.assign((size_t)kL3Configs * 16, 0);
    g_cfg2d = build_lut2d(g_h_lut2d, err, sizeof err);
    if (g_cfg2d != kL2Configs) { fprintf(stderr, "flashcubical: 2D table: %s\n", err); g_lut_status = PH_EINTERNAL; return; }
    g_cfg3d = build_lut3d(g_h_l1.data(), g_h_l2.data(), g_h_h1e.data(), g_h_h1s.data(), err, sizeof err);
    if (g_cfg3d != kL3Configs) { fprintf(stderr, "flashcubical: 3D table: %s\n", err); g_lut_status = PH_EINTERNAL; return; }
}

int host_luts() {
    std::call_once(g_lut_once, build_host_luts);
    return g_lut_status;
}

// Every kernel must fit the device: static LDS within the per-block limit and the block
// size we launch within the kernel's limit.  A kernel that cannot launch would leave later
// kernels reading unwritten workspace, so the library refuses to run instead.
struct KInfo { const char *name; const void *fn; int threads; };

// A failed HIP call of the set-up path is named on stderr: the caller only sees PH_EHIP.
bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    fprintf(stderr, "flashcubical: %s failed: %s\n", what, hipGetErrorString(e));
    return false;
}

int check_kernels(int dev, char *report, size_t len) {
    const KInfo ks[] = {
        {"k_plan", (const void *)k_plan, kPlanThreads},
        {"k_classify2d<64,16>", (const void *)k_classify2d<64, 16, float>, 256},
        {"k_classify2d<32,32>", (const void *)k_classify2d<32, 32, float>, 256},
        {"k_classify2d<128,8>", (const void *)k_classify2d<128, 8, float>, 256},
        {"k_classify2d<64,16,u8>", (const void *)k_classify2d<64, 16, uint8_t>, 256},
        {"k_classify2d<64,16,u16>", (const void *)k_classify2d<64, 16, uint16_t>, 256},
        {"k_classify3d<16,8,8>", (const void *)k_classify3d<16, 8, 8, float>, 256},
        {"k_classify3d<32,8,4>", (const void *)k_classify3d<32, 8, 4, float>, 256},
        {"k_classify3d<8,8,16>", (const void *)k_classify3d<8, 8, 16, float>, 256},
        {"k_classify3d<16,8,8,u8>", (const void *)k_classify3d<16, 8, 8, uint8_t>, 256},
        {"k_classify3d<16,8,8,u16>", (const void *)k_classify3d<16, 8, 8, uint16_t>, 256},
        {"k_sort_lists", (const void *)k_sort_lists, kSortThreads},
        {"k_resolve", (const void *)k_resolve, 256},
        {"k_unionfind", (const void *)k_unionfind, kUfThreads},
        {"k_uf_wide", (const void *)k_uf_wide, kWideThreads},
        {"k_sort_runs", (const void *)k_sort_runs, kSortThreads},
        {"k_sort_merge", (const void *)k_sort_merge, kSortThreads},
        {"k_output_scan", (const void *)k_output_scan, kUfThreads},
        {"k_output", (const void *)k_output, kUfThreads},
        {"k_zero", (const void *)k_zero, 256},
        {"k_scatter", (const void *)k_scatter, 256},
        {"k_classify3d<16,8,8,h1>", (const void *)k_classify3d<16, 8, 8, float, true>, 256},
        {"k_classify3d<16,8,8,u8,h1>", (const void *)k_classify3d<16, 8, 8, uint8_t, true>, 256},
        {"k_classify3d<16,8,8,u16,h1>", (const void *)k_classify3d<16, 8, 8, uint16_t, true>, 256},
        {"k_h1_morse", (const void *)k_h1_morse<float, kH1Slots>, 64},
        {"k_h1_morse<u8>", (const void *)k_h1_morse<uint8_t, kH1Slots>, 64},
        {"k_h1_morse<u16>", (const void *)k_h1_morse<uint16_t, kH1Slots>, 64},
        {"k_h1_morse<big>", (const void *)k_h1_morse<float, kH1BigSlots>, 64},
        {"k_h1_morse<u8,big>", (const void *)k_h1_morse<uint8_t, kH1BigSlots>, 64},
        {"k_h1_morse<u16,big>", (const void *)k_h1_morse<uint16_t, kH1BigSlots>, 64},
        {"k_h1_reduce", (const void *)k_h1_reduce, kUfThreads},
    };
    int maxsh = 0, maxthr = 0;
    if (!hip_ok(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute") ||
        !hip_ok(hipDeviceGetAttribute(&maxthr, hipDeviceAttributeMaxThreadsPerBlock, dev), "hipDeviceGetAttribute"))
        return PH_EHIP;
    size_t used = 0;
    auto put = [&](const char *fmt, auto... a) {
        if (!report || used >= len) return;
        int k = snprintf(report + used, len - used, fmt, a...);
        if (k > 0) used += (size_t)k;
    };
    put("device %d: max shared per block %d, max threads per block %d\n", dev, maxsh, maxthr);
    int rc = PH_OK;
    for (const KInfo &k : ks) {
        hipFuncAttributes at;
        if (!hip_ok(hipFuncGetAttributes(&at, k.fn), k.name)) { put("%s: attributes unavailable\n", k.name); rc = PH_EHIP; continue; }
        const bool ok = (int)at.sharedSizeBytes <= maxsh && at.maxThreadsPerBlock >= k.threads && k.threads <= maxthr;
        put("%s: lds %d B, regs %d, max threads %d, launch %d %s\n", k.name, (int)at.sharedSizeBytes,
            at.numRegs, at.maxThreadsPerBlock, k.threads, ok ? "ok" : "DOES NOT FIT");
        if (!ok) rc = PH_EHIP;
    }
    return rc;
}

int device_luts() {
    int rc = host_luts();
    if (rc != PH_OK) return rc;
    int dev = 0;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice") || dev < 0 || dev >= 64) return PH_EHIP;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_dev_ready[dev]) return PH_OK;
    // one device buffer holds every table, each part 256-byte aligned
    const size_t n2d = sizeof g_h_lut2d, n1 = sizeof(uint32_t) * kL1Size, n2 = sizeof(uint64_t) * kL3Configs;
    const size_t ne = sizeof(uint16_t) * g_h_h1e.size(), ns = sizeof(uint16_t) * g_h_h1s.size();
    const size_t o1 = align256(n2d), o2 = o1 + align256(n1), oe = o2 + align256(n2), os = oe + align256(ne);
    const size_t op = os + align256(ns);
    uint8_t h_pext[256];
    for (uint32_t k = 0; k < 256; ++k) h_pext[k] = (uint8_t)compress8(k & 15u, k >> 4);
    uint8_t *buf = nullptr;
    if (!hip_ok(hipMalloc((void **)&buf, op + sizeof h_pext), "hipMalloc (tables)")) return PH_EHIP;
    if (!hip_ok(hipMemcpy(buf, g_h_lut2d, n2d, hipMemcpyHostToDevice), "hipMemcpy (tables)") ||
        !hip_ok(hipMemcpy(buf + o1, g_h_l1.data(), n1, hipMemcpyHostToDevice), "hipMemcpy (tables)") ||
        !hip_ok(hipMemcpy(buf + o2, g_h_l2.data(), n2, hipMemcpyHostToDevice), "hipMemcpy (tables)") ||
        !hip_ok(hipMemcpy(buf + oe, g_h_h1e.data(), ne, hipMemcpyHostToDevice), "hipMemcpy (tables)") ||
        !hip_ok(hipMemcpy(buf + os, g_h_h1s.data(), ns, hipMemcpyHostToDevice), "hipMemcpy (tables)") ||
        !hip_ok(hipMemcpy(buf + op, h_pext, sizeof h_pext, hipMemcpyHostToDevice), "hipMemcpy (tables)")) {
        (void)hipFree(buf);
        return PH_EHIP;
    }
    g_dev_lut[dev] = Luts{(const uint32_t *)buf, (const uint32_t *)(buf + o1), (const uint64_t *)(buf + o2),
                          (const uint16_t *)(buf + oe), (const uint16_t *)(buf + os), buf + op};
    rc = check_kernels(dev, nullptr, 0);
    if (rc != PH_OK) return rc;
    g_dev_ready[dev] = true;
    return PH_OK;
}

bool valid_shape(const ph_shape &s) {
    if (s.ndim != 2 && s.ndim != 3) return false;
    int64_t nv = 1;
    for (int k = 0; k < s.ndim; ++k) {
        if (s.ext[k] < 1) return false;
        nv *= s.ext[k];                            // <= 2^27 * 2^31 before the check: no overflow
        if (nv > (1ll << kPixBits)) return false;  // pixel indices must fit the key's 27 bits
    }
    return true;
}

const int kTile2[3][2] = {{64, 16}, {32, 32}, {128, 8}};
const int kTile3[3][3] = {{16, 8, 8}, {32, 8, 4}, {8, 8, 16}};

Tiles tiles_of(const ph_tuning *t) {
    int a = t ? t->tile2d : 0, b = t ? t->tile3d : 0;
    if (a < 0 || a > 2) a = 0;
    if (b < 0 || b > 2) b = 0;
    return Tiles{kTile2[a][0], kTile2[a][1], kTile3[b][0], kTile3[b][1], kTile3[b][2]};
}

// total workspace bytes and classify grid sizes for a list of host shapes
int64_t plan_host(const ph_shape *h, int n, const Tiles &tl, int64_t *t2, int64_t *t3, bool tfilt, bool h1,
                  int lists) {
    int64_t at = header_bytes(n);
    *t2 = 0;
    *t3 = 0;
    for (int i = 0; i < n; ++i) {
        Inst I;
        fill_inst(I, tfilt ? framed(h[i]) : h[i], tl, lists);
        I.tfilt = tfilt;
        I.h1 = h1 && I.ndim == 3;
        if (I.ndim == 2) *t2 += (int64_t)I.tx * I.ty;
        else *t3 += (int64_t)I.tx * I.ty * I.tz;
        at = layout(I, at);
    }
    return at;
}

int64_t max_voxels(const ph_shape *h, int n) {
    int64_t m = 1;
    for (int i = 0; i < n; ++i) {
        int64_t v = 1;
        for (int a = 0; a < h[i].ndim; ++a) v *= h[i].ext[a];
        if (v > m) m = v;
    }
    return m;
}

int64_t max_list(const ph_shape *h, int n) {
    int64_t m = 1;
    for (int i = 0; i < n; ++i) {
        Inst I;
        fill_inst(I, h[i], Tiles{64, 16, 16, 8, 8});
        int64_t l = I.E > I.F ? I.E : I.F;
        if (l > m) m = l;
    }
    return m;
}

template <int A, int B, typename T = float>
void launch2d(int64_t tiles, const void *imgs, uint8_t *ws, int n, Luts lut, hipStream_t st, float *grad) {
    hipLaunchKernelGGL((k_classify2d<A, B, T>), dim3((unsigned)tiles), dim3(256), 0, st, (const T *)imgs, ws, n, lut,
                       grad);
}
template <int A, int B, int C, typename T = float, bool H1 = false>
void launch3d(int64_t tiles, const void *imgs, uint8_t *ws, int n, Luts lut, hipStream_t st, float *grad) {
    hipLaunchKernelGGL((k_classify3d<A, B, C, T, H1>), dim3((unsigned)tiles), dim3(256), 0, st, (const T *)imgs, ws, n,
                       lut, grad);
}

Luts current_luts() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    return g_dev_lut[dev];
}

// ------------------------------------------------------------------ autotuning --
// Tile choices found fastest by ph_autotune, per size class of a batch: which dimensions it
// holds and the binary order of magnitude of its mean instance size.  A batch call without an
// explicit tuning uses the entry of its class, else the defaults.  Tiles never change results.
using SizeClass = std::tuple<int, int, int>;
std::mutex g_tune_mu;
std::map<SizeClass, ph_tuning> g_tune;

SizeClass size_class(const ph_shape *h, int n) {
    int has2 = 0, has3 = 0;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        int64_t v = 1;
        for (int k = 0; k < h[i].ndim; ++k) v *= h[i].ext[k];
        total += v;
        (h[i].ndim == 2 ? has2 : has3) = 1;
    }
    int64_t mean = total / (n > 0 ? n : 1);
    int bucket = 0;
    while (mean > 1) { mean >>= 1; ++bucket; }
    return SizeClass{has2, has3, bucket};
}

bool tuned_for(const ph_shape *h, int n, ph_tuning *t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(size_class(h, n));
    if (it == g_tune.end()) return false;
    *t = it->second;
    return true;
}

// ------------------------------------------------------------------- profiling --
// Optional per-launch timing with HIP events on the launch stream (not for use while the
// stream is being captured into a graph).
enum KernelId {
    K_PLAN, K_CLASSIFY2D, K_CLASSIFY3D, K_SORT, K_RESOLVE, K_UF, K_RESOLVE_2D, K_UF_2D, K_H1MORSE, K_H1MORSE2, K_H1REDUCE,
    K_OUTPUT, K_ZERO, K_SCATTER, K_UFWIDE, K_UFWIDE_2D, K_SORTWIDE, K_OUTWIDE, K_COUNT
};
const char *const kKernelNames[K_COUNT] = {
    "k_plan", "k_classify2d", "k_classify3d", "k_sort", "k_resolve", "k_unionfind",
    "k_resolve(2d top)", "k_unionfind(2d top)", "k_h1_morse", "k_h1_morse(large)", "k_h1_reduce", "k_output", "k_zero", "k_scatter",
    "k_uf_wide", "k_uf_wide(2d top)", "k_sort_wide", "k_output_wide"};

struct ProfRec { int kid; hipEvent_t a, b; };
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

hipEvent_t prof_mark(hipStream_t st) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    if (hipEventRecord(e, st) != hipSuccess) { (void)hipEventDestroy(e); return nullptr; }
    return e;
}

void prof_push(int kid, hipEvent_t a, hipEvent_t b) {
    if (!a || !b) {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        return;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(ProfRec{kid, a, b});
}

bool prof_enabled() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on;
}

// FLASHCUBICAL_TRACE=1: name every launch on stderr before it is made and wait for it after,
// so that a failing kernel is the last one named.
bool trace_enabled() {
    static const bool on = [] {
        const char *e = getenv("FLASHCUBICAL_TRACE");
        return e && e[0] == '1' && e[1] == 0;
    }();
    return on;
}

int trace_before(int kid) {
    fprintf(stderr, "flashcubical: launch %s\n", kKernelNames[kid]);
    fflush(stderr);
    return PH_OK;
}

int trace_after(int kid, hipStream_t st) {
    const hipError_t e = hipStreamSynchronize(st);
    fprintf(stderr, "flashcubical: %s %s\n", kKernelNames[kid], e == hipSuccess ? "done" : "FAILED");
    fflush(stderr);
    return e == hipSuccess ? PH_OK : PH_EHIP;
}

// d_grad: with ph_diagram_batch_grad, the caller's gradient buffer the classify passes set to
// zero (packed like the inputs); else null
int run(int n, const void *d_imgs, const int64_t *d_img_off, const ph_shape *d_shapes,
        const ph_shape *h_shapes, ph_shape single, uint32_t flags, ph_pairs out,
        const int64_t *d_out_off, int64_t single_cap, int64_t *d_counts, int32_t *d_status,
        const ph_tuning *tuning, void *d_ws, size_t ws_bytes, hipStream_t st, float *d_grad = nullptr) {
    if (n < 1 || n > kMaxInstances || !d_imgs || !h_shapes || !d_counts || !d_status || !d_ws) return PH_EINVAL;
    if (!out.dim || !out.birth || !out.death || !out.birth_cell || !out.death_cell ||
        !out.birth_vertex || !out.death_vertex)
        return PH_EINVAL;
    // under the T-filtration the kernels below run on the framed dual images (extents + 2),
    // which they read from the caller's pixels through the reflection (tf_value)
    const bool tf = (flags & PH_TFILT) != 0;
    // (a single instance keeps its framed shape on the stack: the no-allocation entry point
    // allocates nothing, on the host either)
    ph_shape framed_one;
    std::vector<ph_shape> framed_many;
    ph_shape *framed_shapes = &framed_one;
    if (tf && n > 1) {
        framed_many.resize(n);
        framed_shapes = framed_many.data();
    }
    if (tf)
        for (int i = 0; i < n; ++i) framed_shapes[i] = framed(h_shapes[i]);
    const ph_shape *hs = tf ? framed_shapes : h_shapes;
    bool any2 = false, any3 = false;
    for (int i = 0; i < n; ++i) {
        if (!valid_shape(h_shapes[i]) || !valid_shape(hs[i])) return PH_EINVAL;
        (h_shapes[i].ndim == 3 ? any3 : any2) = true;
    }
    if (!(flags & (PH_H0 | PH_HTOP | PH_H1))) return PH_EINVAL;
    if ((flags & PH_IN_U8) && (flags & PH_IN_U16)) return PH_EINVAL;
    const int elem = (flags & PH_IN_U8) ? 1 : ((flags & PH_IN_U16) ? 2 : 0);   // 0 float32, 1 u8, 2 u16
    if (elem != 0) tuning = nullptr;               // integer inputs use the default tiles
    const bool h1 = (flags & PH_H1) != 0;
    ph_tuning h1_tuning;
    if (h1 && tuning && tuning->tile3d != 0) {     // 3D H1 plans and runs the default 3D tile
        h1_tuning = *tuning;
        h1_tuning.tile3d = 0;
        tuning = &h1_tuning;
    }
    int rc = device_luts();
    if (rc != PH_OK) return rc;
    const Tiles tl = tiles_of(tuning);
    int64_t t2, t3;
    const int lists = list_fraction(flags);
    const int64_t need = plan_host(h_shapes, n, tl, &t2, &t3, tf, h1, lists);   // frames them itself
    if ((int64_t)ws_bytes < need) return PH_ENOMEM;
    if (t2 >= (1ll << 31) || t3 >= (1ll << 31)) return PH_EINVAL;
    uint8_t *ws = (uint8_t *)d_ws;
    const int tile2 = tuning ? tuning->tile2d : 0, tile3 = tuning ? tuning->tile3d : 0;

    // Each launch is checked on its own: the error a failed launch leaves behind would be
    // overwritten by the next successful call.
    const bool prof = prof_enabled(), trace = trace_enabled();
#define FC_LAUNCH(KID, ...)                                                   \
    do {                                                                      \
        if (trace) trace_before(KID);                                         \
        hipEvent_t ev_a = prof ? prof_mark(st) : nullptr;                     \
        (void)hipGetLastError();                                              \
        __VA_ARGS__;                                                          \
        if (hipGetLastError() != hipSuccess) {                                \
            if (ev_a) (void)hipEventDestroy(ev_a);                            \
            return PH_EHIP;                                                   \
        }                                                                     \
        if (prof) prof_push(KID, ev_a, prof_mark(st));                        \
        if (trace && trace_after(KID, st) != PH_OK) return PH_EHIP;           \
    } while (0)
    FC_LAUNCH(K_PLAN, hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, st, n, d_shapes, single, d_img_off, d_out_off,
                                 single_cap, tl, ws, d_counts, d_status, t2, t3, (int64_t)ws_bytes, tf ? 1 : 0,
                                 h1 ? 1 : 0, lists));
    const int64_t ml = max_list(hs, n), mv = max_voxels(hs, n);
    const void *cimgs = d_imgs;                    // what the classify passes read
    const Luts lut = current_luts();
    if (t2 > 0) {
        if (elem == 1) FC_LAUNCH(K_CLASSIFY2D, (launch2d<64, 16, uint8_t>(t2, cimgs, ws, n, lut, st, d_grad)));
        else if (elem == 2) FC_LAUNCH(K_CLASSIFY2D, (launch2d<64, 16, uint16_t>(t2, cimgs, ws, n, lut, st, d_grad)));
        else if (tile2 == 1) FC_LAUNCH(K_CLASSIFY2D, launch2d<32, 32>(t2, cimgs, ws, n, lut, st, d_grad));
        else if (tile2 == 2) FC_LAUNCH(K_CLASSIFY2D, launch2d<128, 8>(t2, cimgs, ws, n, lut, st, d_grad));
        else FC_LAUNCH(K_CLASSIFY2D, launch2d<64, 16>(t2, cimgs, ws, n, lut, st, d_grad));
    }
    if (t3 > 0 && h1) {                            // 3D H1 keeps every configuration: default tiles
        if (elem == 1) FC_LAUNCH(K_CLASSIFY3D, (launch3d<16, 8, 8, uint8_t, true>(t3, cimgs, ws, n, lut, st, d_grad)));
        else if (elem == 2) FC_LAUNCH(K_CLASSIFY3D, (launch3d<16, 8, 8, uint16_t, true>(t3, cimgs, ws, n, lut, st, d_grad)));
        else FC_LAUNCH(K_CLASSIFY3D, (launch3d<16, 8, 8, float, true>(t3, cimgs, ws, n, lut, st, d_grad)));
    } else if (t3 > 0) {
        if (elem == 1) FC_LAUNCH(K_CLASSIFY3D, (launch3d<16, 8, 8, uint8_t>(t3, cimgs, ws, n, lut, st, d_grad)));
        else if (elem == 2) FC_LAUNCH(K_CLASSIFY3D, (launch3d<16, 8, 8, uint16_t>(t3, cimgs, ws, n, lut, st, d_grad)));
        else if (tile3 == 1) FC_LAUNCH(K_CLASSIFY3D, launch3d<32, 8, 4>(t3, cimgs, ws, n, lut, st, d_grad));
        else if (tile3 == 2) FC_LAUNCH(K_CLASSIFY3D, launch3d<8, 8, 16>(t3, cimgs, ws, n, lut, st, d_grad));
        else FC_LAUNCH(K_CLASSIFY3D, launch3d<16, 8, 8>(t3, cimgs, ws, n, lut, st, d_grad));
    }
    // resolve grid: the lists are a small share of the voxels for any field that is not noise,
    // so 256 threads per 64Ki voxels of the largest instance; the loops stride over the rest
    int64_t rb = (mv + 65535) / 65536;
    if (rb > (ml + 255) / 256) rb = (ml + 255) / 256;
    if ((flags & PH_WIDE) && mv >= kWideVoxels) rb = (mv + 4095) / 4096;   // noise: lists of a sixth of the pixels
    const unsigned rblocks = (unsigned)(rb < 1 ? 1 : (rb > 1024 ? 1024 : rb));
    // PH_WIDE: the union-finds and the long lists of instances of kWideVoxels or more voxels
    // are spread over the whole GPU (each instance's kernels decide for themselves, from its
    // counts)
    const int wide = (flags & PH_WIDE) && mv >= kWideVoxels ? 1 : 0;
    FC_LAUNCH(K_SORT, hipLaunchKernelGGL(k_sort_lists, dim3(n, 3), dim3(kSortThreads), 0, st, ws, n, wide));
    if (wide) {
        int64_t runs = (ml + kSortCap - 1) / kSortCap;
        const unsigned sb = (unsigned)std::min<int64_t>(512, runs);   // workgroups per list: runs, then tiles
        FC_LAUNCH(K_SORTWIDE, hipLaunchKernelGGL(k_sort_runs, dim3(sb, n, 3), dim3(kSortThreads), 0, st, ws, n));
        int passes = 0;
        while (((int64_t)kSortCap << passes) < ml) ++passes;
        for (int p = 0; p <= passes; ++p)         // the last one only copies back
            FC_LAUNCH(K_SORTWIDE, hipLaunchKernelGGL(k_sort_merge, dim3(sb, n, 3), dim3(kSortThreads), 0, st, ws, n, p));
    }
    // volumes: the dual (resolve, union-find) beside H0; images: the dual after H0
    // T's H0 is the V top; 3D H1 needs the squares the dual union-find pairs
    const int htop = (tf || (flags & PH_HTOP) || (h1 && any3)) ? 1 : 0;
    const unsigned side = htop && any3 ? 2 : 1;
    FC_LAUNCH(K_RESOLVE, hipLaunchKernelGGL(k_resolve, dim3(rblocks, n, side), dim3(256), 0, st, ws, n, 0, htop));
    auto wide_rounds = [&](int stage, unsigned sides, int kid) -> int {
        for (int ph = -1, r = 0; r < kWideRounds; ph == 1 ? (ph = 0, ++r) : ++ph) {
            FC_LAUNCH(kid, hipLaunchKernelGGL(k_uf_wide, dim3(kWideBlocks, n, sides), dim3(kWideThreads), 0, st, ws, n,
                                              stage, htop, ph, r));
        }
        return PH_OK;
    };
    if (wide && wide_rounds(0, side, K_UFWIDE) != PH_OK) return PH_EHIP;
    FC_LAUNCH(K_UF, hipLaunchKernelGGL(k_unionfind, dim3(n, side), dim3(kUfThreads), 0, st, ws, n, 0, htop, wide));
    if (htop && any2) {
        FC_LAUNCH(K_RESOLVE_2D, hipLaunchKernelGGL(k_resolve, dim3(rblocks, n), dim3(256), 0, st, ws, n, 1, htop));
        if (wide && wide_rounds(1, 1, K_UFWIDE_2D) != PH_OK) return PH_EHIP;
        FC_LAUNCH(K_UF_2D, hipLaunchKernelGGL(k_unionfind, dim3(n), dim3(kUfThreads), 0, st, ws, n, 1, htop, wide));
    }
    if (h1 && any3) {
        // one 64-thread workgroup per 512 voxels of the largest volume (at most 8192 per
        // instance), each taking columns in turn: short-lived workgroups, so the hardware
        // balances the columns' uneven costs (per 4096 voxels measured 13 % slower)
        const unsigned hb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (mv + 511) / 512));
        // pass 1 (64 workgroups per instance) takes the columns pass 0 could not hold
        if (elem == 1) {
            FC_LAUNCH(K_H1MORSE, hipLaunchKernelGGL((k_h1_morse<uint8_t, kH1Slots>), dim3(hb, n), dim3(64), 0, st, (const uint8_t *)cimgs, ws, n, lut, 0));
            FC_LAUNCH(K_H1MORSE2, hipLaunchKernelGGL((k_h1_morse<uint8_t, kH1BigSlots>), dim3(64, n), dim3(64), 0, st, (const uint8_t *)cimgs, ws, n, lut, 1));
        } else if (elem == 2) {
            FC_LAUNCH(K_H1MORSE, hipLaunchKernelGGL((k_h1_morse<uint16_t, kH1Slots>), dim3(hb, n), dim3(64), 0, st, (const uint16_t *)cimgs, ws, n, lut, 0));
            FC_LAUNCH(K_H1MORSE2, hipLaunchKernelGGL((k_h1_morse<uint16_t, kH1BigSlots>), dim3(64, n), dim3(64), 0, st, (const uint16_t *)cimgs, ws, n, lut, 1));
        } else {
            FC_LAUNCH(K_H1MORSE, hipLaunchKernelGGL((k_h1_morse<float, kH1Slots>), dim3(hb, n), dim3(64), 0, st, (const float *)cimgs, ws, n, lut, 0));
            FC_LAUNCH(K_H1MORSE2, hipLaunchKernelGGL((k_h1_morse<float, kH1BigSlots>), dim3(64, n), dim3(64), 0, st, (const float *)cimgs, ws, n, lut, 1));
        }
        FC_LAUNCH(K_H1REDUCE, hipLaunchKernelGGL(k_h1_reduce, dim3(n), dim3(kUfThreads), 0, st, ws, n));
    }
    if (wide) {                                   // PH_WIDE: large instances' pairs by the whole GPU
        FC_LAUNCH(K_OUTWIDE, hipLaunchKernelGGL(k_output, dim3(kWideBlocks / 4, n), dim3(kUfThreads), 0, st, d_imgs, ws, n,
                                                flags, out, d_counts, d_status, 1));
        FC_LAUNCH(K_OUTWIDE, hipLaunchKernelGGL(k_output_scan, dim3(n), dim3(kUfThreads), 0, st, ws, n, flags));
        FC_LAUNCH(K_OUTWIDE, hipLaunchKernelGGL(k_output, dim3(kWideBlocks / 4, n), dim3(kUfThreads), 0, st, d_imgs, ws, n,
                                                flags, out, d_counts, d_status, 2));
    }
    FC_LAUNCH(K_OUTPUT, hipLaunchKernelGGL(k_output, dim3(n), dim3(kUfThreads), 0, st, d_imgs, ws, n, flags, out, d_counts,
                                 d_status, 0));
    return PH_OK;
}

// Device address of the no-allocation workspace on each device (see `scratch` below), taken
// by ph_init_device; null until then.
void *g_scratch_dev[64] = {nullptr};

}  // namespace
}  // namespace fc

// Workspace of ph_diagram_noalloc: one array per device, in the library's code object, held
// until the process ends.  In host code `scratch` names a host-side stand-in, not device
// memory: only the address hipGetSymbolAddress returns for the current device is ever passed
// to a kernel (fc::g_scratch_dev).
constexpr size_t kScratchBytes = (size_t)PH_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// ====================================================================== C ABI ====

namespace fc {
namespace {
// ph_backward and ph_backward_scatter: the zero fill (zero) then the scatter
int backward(int32_t n, ph_pairs pairs, const int64_t *d_out_off, const int64_t *d_counts,
             const float *d_grad_birth, const float *d_grad_death, float *d_grad_img,
             const int64_t *d_img_off, int64_t total_voxels, void *stream, bool zero) {
    if (n < 1 || n > fc::kMaxInstances || !d_counts || !d_grad_birth || !d_grad_death || !d_grad_img || total_voxels < 1 ||
        !pairs.birth_vertex || !pairs.death_vertex)
        return PH_EINVAL;
    if (!d_out_off || !d_img_off) return PH_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int rc = fc::device_luts();
    if (rc != PH_OK) return rc;
    const bool prof = fc::prof_enabled(), trace = fc::trace_enabled();
    if (zero) {
        const int64_t zb = (total_voxels + 255) / 256;
        if (trace) fc::trace_before(fc::K_ZERO);
        hipEvent_t z0 = prof ? fc::prof_mark(st) : nullptr;
        (void)hipGetLastError();
        hipLaunchKernelGGL(fc::k_zero, dim3((unsigned)(zb < 8192 ? zb : 8192)), dim3(256), 0, st, d_grad_img,
                           total_voxels);
        if (hipGetLastError() != hipSuccess) {
            if (z0) (void)hipEventDestroy(z0);
            return PH_EHIP;
        }
        if (prof) fc::prof_push(fc::K_ZERO, z0, fc::prof_mark(st));
        if (trace && fc::trace_after(fc::K_ZERO, st) != PH_OK) return PH_EHIP;
    }
    if (trace) fc::trace_before(fc::K_SCATTER);
    hipEvent_t s0 = prof ? fc::prof_mark(st) : nullptr;
    // pairs are a small share of the voxels for any field that is not noise: one 256-thread
    // block per 64Ki voxels of the mean instance (1..64 per instance); the loop strides over the rest
    int64_t sb = (total_voxels / n + 65535) / 65536;
    sb = sb < 1 ? 1 : (sb > 64 ? 64 : sb);
    hipLaunchKernelGGL(fc::k_scatter, dim3((unsigned)sb, n), dim3(256), 0, st, pairs, d_out_off, d_counts,
                       d_grad_birth, d_grad_death, d_grad_img, d_img_off, (int)n, total_voxels);
    const bool ok = hipGetLastError() == hipSuccess;
    if (prof) fc::prof_push(fc::K_SCATTER, s0, ok ? fc::prof_mark(st) : nullptr);
    if (ok && trace && fc::trace_after(fc::K_SCATTER, st) != PH_OK) return PH_EHIP;
    return ok ? PH_OK : PH_EHIP;
}
}  // namespace
}  // namespace fc

extern "C" {

int64_t ph_capacity_bound(ph_shape s) {
    if (!fc::valid_shape(s)) return 0;
    fc::Inst I;
    fc::fill_inst(I, s, fc::Tiles{64, 16, 16, 8, 8});
    return I.N + I.T;
}

int64_t ph_capacity_bound_flags(ph_shape s, uint32_t flags) {
    if (flags & PH_TFILT) s = fc::framed(s);
    if (!fc::valid_shape(s)) return 0;
    fc::Inst I;
    fc::fill_inst(I, s, fc::Tiles{64, 16, 16, 8, 8});
    const fc::Geom g = fc::geom(I.ndim, I.D, I.H, I.W);
    // H1 pairs of a volume: at most its negative squares, S - C (= E - V + 1 by Euler)
    return I.N + I.T + ((flags & PH_H1) && I.ndim == 3 ? g.S - g.C : 0);
}

size_t ph_workspace_bytes(const ph_shape *h_shapes, int32_t n, uint32_t flags) {
    const bool tf = (flags & PH_TFILT) != 0;
    if (!h_shapes || n < 1) return 0;
    for (int i = 0; i < n; ++i)
        if (!fc::valid_shape(h_shapes[i]) || (tf && !fc::valid_shape(fc::framed(h_shapes[i])))) return 0;
    int64_t t2, t3, best = 0;
    for (int a = 0; a < 3; ++a)                      // large enough for every tile choice
        for (int b = 0; b < 3; ++b) {
            ph_tuning t{a, b};
            int64_t need = fc::plan_host(h_shapes, n, fc::tiles_of(&t), &t2, &t3, tf, (flags & PH_H1) != 0,
                                         fc::list_fraction(flags));
            if (need > best) best = need;
        }
    return (size_t)best;
}

int ph_diagram(const void *d_img, ph_shape shape, uint32_t flags, ph_pairs out, int64_t capacity,
               int64_t *d_count, int32_t *d_status, void *d_ws, size_t ws_bytes, void *stream) {
    if (capacity < 0) return PH_EINVAL;
    return fc::run(1, d_img, nullptr, nullptr, &shape, shape, flags, out, nullptr, capacity, d_count,
                   d_status, nullptr, d_ws, ws_bytes, (hipStream_t)stream);
}

int ph_diagram_noalloc(const void *d_img, ph_shape shape, uint32_t flags, ph_pairs out, int64_t capacity,
                       int64_t *d_count, int32_t *d_status, void *stream) {
    if (capacity < 0) return PH_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return PH_EHIP;
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(fc::g_dev_mu);
        ws = fc::g_scratch_dev[dev];             // set with the tables by ph_init_device
    }
    if (!ws) return PH_EINVAL;
    const int rc = fc::run(1, d_img, nullptr, nullptr, &shape, shape, flags, out, nullptr, capacity, d_count,
                           d_status, nullptr, ws, kScratchBytes, (hipStream_t)stream);
    if (rc == PH_ENOMEM)
        fprintf(stderr, "flashcubical: ph_diagram_noalloc: the instance needs more than the %d MiB of the "
                        "library's workspace (ph_workspace_bytes gives its need)\n", PH_NOALLOC_SCRATCH_MIB);
    return rc;
}

int ph_diagram_batch(int32_t n, const void *d_imgs, const int64_t *d_img_off, const ph_shape *d_shapes,
                     const ph_shape *h_shapes, uint32_t flags, ph_pairs out, const int64_t *d_out_off,
                     int64_t *d_counts, int32_t *d_status, const ph_tuning *tuning, void *d_ws,
                     size_t ws_bytes, void *stream) {
    if (!d_img_off || !d_shapes || !d_out_off || !h_shapes || n < 1) return PH_EINVAL;
    ph_shape dummy{2, {1, 1, 1}};
    ph_tuning tuned;
    // the recorded choices are those of V batches of the size class: a T batch takes the defaults
    if (!tuning && !(flags & PH_TFILT) && fc::tuned_for(h_shapes, n, &tuned)) tuning = &tuned;
    return fc::run(n, d_imgs, d_img_off, d_shapes, h_shapes, dummy, flags, out, d_out_off, 0, d_counts,
                   d_status, tuning, d_ws, ws_bytes, (hipStream_t)stream);
}

int ph_diagram_batch_grad(int32_t n, const void *d_imgs, const int64_t *d_img_off, const ph_shape *d_shapes,
                          const ph_shape *h_shapes, uint32_t flags, ph_pairs out, const int64_t *d_out_off,
                          int64_t *d_counts, int32_t *d_status, const ph_tuning *tuning, void *d_ws,
                          size_t ws_bytes, float *d_grad_img, void *stream) {
    if (!d_img_off || !d_shapes || !d_out_off || !h_shapes || n < 1 || !d_grad_img) return PH_EINVAL;
    ph_shape dummy{2, {1, 1, 1}};
    ph_tuning tuned;
    if (!tuning && !(flags & PH_TFILT) && fc::tuned_for(h_shapes, n, &tuned)) tuning = &tuned;
    return fc::run(n, d_imgs, d_img_off, d_shapes, h_shapes, dummy, flags, out, d_out_off, 0, d_counts,
                   d_status, tuning, d_ws, ws_bytes, (hipStream_t)stream, d_grad_img);
}

int ph_autotune(int32_t n, const void *d_imgs, const int64_t *d_img_off, const ph_shape *d_shapes,
                const ph_shape *h_shapes, uint32_t flags, ph_pairs out, const int64_t *d_out_off,
                int64_t *d_counts, int32_t *d_status, void *d_ws, size_t ws_bytes, int32_t reps,
                ph_tuning *best, void *stream) {
    if (!d_img_off || !d_shapes || !d_out_off || !h_shapes || n < 1 || reps < 1 || !best) return PH_EINVAL;
    ph_shape dummy0{2, {1, 1, 1}};
    if (flags & (PH_IN_U8 | PH_IN_U16 | PH_TFILT)) {
        // integer inputs and T batches take the default tiles: nothing to time, nothing
        // recorded for the size class (float32 V batches of the class keep their own choice)
        *best = ph_tuning{0, 0};
        return fc::run(n, d_imgs, d_img_off, d_shapes, h_shapes, dummy0, flags, out, d_out_off, 0, d_counts,
                       d_status, best, d_ws, ws_bytes, (hipStream_t)stream);
    }
    const fc::SizeClass cls = fc::size_class(h_shapes, n);
    const int n2 = std::get<0>(cls) ? 3 : 1, n3 = std::get<1>(cls) ? 3 : 1;
    hipStream_t st = (hipStream_t)stream;
    ph_shape dummy{2, {1, 1, 1}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return PH_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return PH_EHIP; }
    float best_ms = -1.f;
    int rc = PH_OK;
    for (int a = 0; a < n2 && rc == PH_OK; ++a)
        for (int b = 0; b < n3 && rc == PH_OK; ++b) {
            const ph_tuning t{a, b};
            rc = fc::run(n, d_imgs, d_img_off, d_shapes, h_shapes, dummy, flags, out, d_out_off, 0, d_counts,
                         d_status, &t, d_ws, ws_bytes, st);              // warm-up
            if (rc != PH_OK) break;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = PH_EHIP; break; }
            for (int r = 0; r < reps && rc == PH_OK; ++r)
                rc = fc::run(n, d_imgs, d_img_off, d_shapes, h_shapes, dummy, flags, out, d_out_off, 0,
                             d_counts, d_status, &t, d_ws, ws_bytes, st);
            if (rc != PH_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = PH_EHIP; break; }
            if (best_ms < 0.f || ms < best_ms) { best_ms = ms; *best = t; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PH_OK) return rc;
    std::lock_guard<std::mutex> lk(fc::g_tune_mu);
    fc::g_tune[cls] = *best;
    return PH_OK;
}

int ph_backward(int32_t n, ph_pairs pairs, const int64_t *d_out_off, const int64_t *d_counts,
                const float *d_grad_birth, const float *d_grad_death, float *d_grad_img,
                const int64_t *d_img_off, int64_t total_voxels, void *stream) {
    return fc::backward(n, pairs, d_out_off, d_counts, d_grad_birth, d_grad_death, d_grad_img, d_img_off,
                        total_voxels, stream, true);
}

int ph_backward_scatter(int32_t n, ph_pairs pairs, const int64_t *d_out_off, const int64_t *d_counts,
                        const float *d_grad_birth, const float *d_grad_death, float *d_grad_img,
                        const int64_t *d_img_off, int64_t total_voxels, void *stream) {
    return fc::backward(n, pairs, d_out_off, d_counts, d_grad_birth, d_grad_death, d_grad_img, d_img_off,
                        total_voxels, stream, false);
}

int ph_lut_entry(int32_t ndim, uint32_t raw_mask, uint64_t *entry) {
    if (!entry) return PH_EINVAL;
    int rc = fc::host_luts();
    if (rc != PH_OK) return rc;
    if (ndim == 2) {
        if (raw_mask > 255u) return PH_EINVAL;
        *entry = fc::g_h_lut2d[raw_mask];
        return PH_OK;
    }
    if (ndim == 3) {
        if (raw_mask >> 26) return PH_EINVAL;
        uint32_t cubes;
        const uint32_t idx1 = fc::canon3d(raw_mask, &cubes);
        const uint32_t l1 = fc::g_h_l1[idx1];
        *entry = fc::g_h_l2[(l1 >> 8) + fc::compress8(cubes, l1 & 255u)];
        return PH_OK;
    }
    return PH_EINVAL;
}

int32_t ph_lut_config_count(int32_t ndim) {
    if (fc::host_luts() != PH_OK) return -1;
    return ndim == 2 ? fc::g_cfg2d : ndim == 3 ? fc::g_cfg3d : -1;
}

const char *ph_version(void) { return "flashcubical-gfx950 0.1"; }

int ph_work_counters(const void *d_ws, int32_t n, int32_t *h_out) {
    if (!d_ws || n < 1 || !h_out) return PH_EINVAL;
    std::vector<int32_t> c((size_t)n * fc::CNT_WORDS);
    if (hipMemcpy(c.data(), (const uint8_t *)d_ws + fc::off_cnt(n), c.size() * sizeof(int32_t),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return PH_EHIP;
    const int pick[16] = {fc::CNT_E, fc::CNT_F, fc::CNT_M0, fc::CNT_MT, fc::CNT_ROUNDS0, fc::CNT_ROUNDST,
                          fc::CNT_SEQ, fc::CNT_ERR, fc::CNT_H1COLS, fc::CNT_H1UNSAFE, fc::CNT_H1ROUNDS,
                          fc::CNT_H1POOL, fc::CNT_H1RETRY, fc::CNT_H1ADDS, fc::CNT_HOPS0, fc::CNT_HOPST};
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 16; ++k) h_out[i * 16 + k] = c[(size_t)i * fc::CNT_WORDS + pick[k]];
    return PH_OK;
}

int ph_profile(int32_t enable) {
    std::vector<fc::ProfRec> old;
    {
        std::lock_guard<std::mutex> lk(fc::g_prof_mu);
        if (enable) old.swap(fc::g_prof);
        fc::g_prof_on = enable != 0;
    }
    for (auto &r : old) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    return PH_OK;
}

int ph_profile_read(ph_kernel_time *out, int32_t max, int32_t *count) {
    if (!count || max < 0 || (max > 0 && !out)) return PH_EINVAL;
    std::vector<fc::ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(fc::g_prof_mu);
        recs.swap(fc::g_prof);
    }
    double ms[fc::K_COUNT] = {0};
    int32_t nl[fc::K_COUNT] = {0};
    int rc = PH_OK;
    for (auto &r : recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) rc = PH_EHIP;
        else { ms[r.kid] += t; nl[r.kid] += 1; }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    int32_t k = 0;
    for (int i = 0; i < fc::K_COUNT; ++i) {
        if (nl[i] == 0) continue;
        if (k < max) {
            memset(&out[k], 0, sizeof out[k]);
            snprintf(out[k].name, sizeof out[k].name, "%s", fc::kKernelNames[i]);
            out[k].launches = nl[i];
            out[k].total_ms = ms[i];
        }
        ++k;
    }
    *count = k;
    return rc;
}

/* Report of the device limits and of every kernel's resources; launches nothing. */
int ph_device_report(char *buf, size_t len) {
    if (!buf || len == 0) return PH_EINVAL;
    buf[0] = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PH_EHIP;
    return fc::check_kernels(dev, buf, len);
}

/* Copy the lookup tables to the current device (normally done on first use) and read them
 * back; PH_OK when the device copy equals the host tables. */
int ph_init_device(void) {
    int rc = fc::device_luts();
    if (rc != PH_OK) return rc;
    {
        int dev = 0;
        if (!fc::hip_ok(hipGetDevice(&dev), "hipGetDevice") || dev < 0 || dev >= 64) return PH_EHIP;
        std::lock_guard<std::mutex> lk(fc::g_dev_mu);
        if (!fc::g_scratch_dev[dev]) {
            void *p = nullptr;
            if (!fc::hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress (scratch)") || !p)
                return PH_EHIP;
            fc::g_scratch_dev[dev] = p;
        }
    }
    std::vector<uint32_t> l2d(256), l1(fc::kL1Size);
    std::vector<uint64_t> l2(fc::kL3Configs);
    std::vector<uint16_t> he(fc::g_h_h1e.size()), hs(fc::g_h_h1s.size());
    const fc::Luts t = fc::current_luts();
    if (!fc::hip_ok(hipMemcpy(l2d.data(), t.l2d, 256 * sizeof(uint32_t), hipMemcpyDeviceToHost), "hipMemcpy (read-back)") ||
        !fc::hip_ok(hipMemcpy(l1.data(), t.l1, l1.size() * sizeof(uint32_t), hipMemcpyDeviceToHost), "hipMemcpy (read-back)") ||
        !fc::hip_ok(hipMemcpy(l2.data(), t.l2, l2.size() * sizeof(uint64_t), hipMemcpyDeviceToHost), "hipMemcpy (read-back)") ||
        !fc::hip_ok(hipMemcpy(he.data(), t.h1e, he.size() * sizeof(uint16_t), hipMemcpyDeviceToHost), "hipMemcpy (read-back)") ||
        !fc::hip_ok(hipMemcpy(hs.data(), t.h1s, hs.size() * sizeof(uint16_t), hipMemcpyDeviceToHost), "hipMemcpy (read-back)"))
        return PH_EHIP;
    if (memcmp(l2d.data(), fc::g_h_lut2d, 256 * sizeof(uint32_t)) || l1 != fc::g_h_l1 || l2 != fc::g_h_l2 ||
        he != fc::g_h_h1e || hs != fc::g_h_h1s)
        return PH_EINTERNAL;
    return PH_OK;
}

}  // extern "C"
