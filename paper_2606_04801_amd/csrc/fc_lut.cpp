// fc_lut.cpp -- host generator of the lower-star lookup tables (paper Sec. 3.3).
//
// For every configuration of preceding neighbours of a vertex v, the lower star L(v) (the
// cells whose last vertex is v) is fixed, and so is everything the paper stores for it:
// which cells are paired inside L(v) and with what, in the fully refined order.  We compute
// that by reducing the RELATIVE boundary matrix of L(v): each cell's boundary restricted to
// the cells of L(v), columns and rows in the order of L(v) (dimension, then cell index).  A
// pair found there is a pair of the whole filtration (the part of a column outside L(v)
// precedes every row of L(v), so it never decides a pivot), and the unpaired cells of L(v)
// are the ones left to the global union-finds.  Classes produced:
//   vertex : paired with its first edge (DIRECT, the H0 link) or a local minimum;
//   edge   : DIRECT / paired with a square (pruned: positive, Sec. 3.2) / KEEP;
//   square (3D facet) : paired with an edge (H1, irrelevant here) / paired with a cube /
//            KEEP (goes to the dual union-find);
//   top cell : paired with a facet in L(v) (LOCAL) / ROOT (node of the dual union-find).
// A LOCAL top cell needs the dual-graph link the global walk would make when it dies: the
// cofacet on the other side of its killing facet.  We get it by running the dual union-find
// of Sec. 3.1 on L(v) alone (facets in decreasing order, cells outside L(v) merged into one
// elder node), and we check that it pairs exactly like the reduction.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "fc_common.h"

namespace fc {
namespace {

int code_of(int dz, int dy, int dx) {
    for (int c = 0; c < 27; ++c)
        if (kOff[c][0] == dz && kOff[c][1] == dy && kOff[c][2] == dx) return c;
    return -1;
}

int dim_of(int c) {
    return (kOff[c][0] != 0) + (kOff[c][1] != 0) + (kOff[c][2] != 0);
}

struct Local {
    int partner[27];   // paired cell code, -1 if critical / absent
    bool birth[27];    // true when the cell is the positive member of its pair
    int link[27];      // for top cells paired in L(v): code of the cofacet across (may be absent)
    uint32_t comb[27]; // cells of L(v) (bit per code) whose boundaries sum to the reduced column
};

// Relative reduction of L(v); `present` has bit c for each cell code in L(v).
bool reduce_local(uint32_t present, Local &L, char *err, int errlen) {
    uint32_t R[27] = {0};
    int pivot_of[27];
    for (int c = 0; c < 27; ++c) {
        pivot_of[c] = -1; L.partner[c] = -1; L.birth[c] = false; L.link[c] = -1; L.comb[c] = 0;
    }
    for (int c = 0; c < 27; ++c) {                 // code order = order inside L(v)
        if (!((present >> c) & 1u)) continue;
        uint32_t col = 0;
        for (int k = 0; k < 3; ++k) {
            if (kOff[c][k] == 0) continue;
            int f[3] = {kOff[c][0], kOff[c][1], kOff[c][2]};
            f[k] = 0;                               // the facet that still contains v
            int fc_ = code_of(f[0], f[1], f[2]);
            if (!((present >> fc_) & 1u)) { snprintf(err, errlen, "L(v) not closed"); return false; }
            col |= 1u << fc_;
        }
        uint32_t comb = 1u << c;
        while (col) {
            int low = 31 - __builtin_clz(col);
            if (pivot_of[low] < 0) break;
            col ^= R[pivot_of[low]];
            comb ^= L.comb[pivot_of[low]];
        }
        L.comb[c] = comb;
        if (col) {
            int low = 31 - __builtin_clz(col);
            pivot_of[low] = c;
            R[c] = col;
            L.partner[low] = c;
            L.partner[c] = low;
            L.birth[low] = true;
        }
    }
    return true;
}

// Dual union-find restricted to L(v); fills L.link for top cells and checks the pairs.
bool dual_links(uint32_t present, bool is2d, Local &L, char *err, int errlen) {
    const int D = is2d ? 2 : 3;
    const int EXT = 27;
    int parent[28];
    for (int c = 0; c < 28; ++c) parent[c] = c;
    auto find = [&](int x) { while (parent[x] != x) x = parent[x]; return x; };
    for (int s = 26; s >= 1; --s) {                // facets, decreasing order
        if (!((present >> s) & 1u) || dim_of(s) != D - 1) continue;
        int k = -1;                                  // the in-plane axis the facet does not span
        for (int a = is2d ? 1 : 0; a < 3; ++a)
            if (kOff[s][a] == 0) k = a;
        int cof[2], node[2];
        for (int t = 0; t < 2; ++t) {
            int o[3] = {kOff[s][0], kOff[s][1], kOff[s][2]};
            o[k] = t ? 1 : -1;
            cof[t] = code_of(o[0], o[1], o[2]);
            node[t] = ((present >> cof[t]) & 1u) ? cof[t] : EXT;
        }
        int r0 = find(node[0]), r1 = find(node[1]);
        if (r0 == r1) continue;
        // the younger in the dual order is the one entering later in the reverse walk:
        // the smaller code; the outside node is the eldest
        int young = (r0 == EXT) ? r1 : (r1 == EXT) ? r0 : (r0 < r1 ? r0 : r1);
        int other = (young == r0) ? r1 : r0;
        int across = (find(node[0]) == young) ? cof[1] : cof[0];
        if (L.partner[young] != s || L.birth[young]) {
            snprintf(err, errlen, "dual pairing disagrees with the reduction (facet %d, cell %d)", s, young);
            return false;
        }
        L.link[young] = across;
        parent[young] = other;
    }
    for (int c = 1; c < 27; ++c)                     // every locally paired top cell got a link
        if (((present >> c) & 1u) && dim_of(c) == D && L.partner[c] >= 0 && L.link[c] < 0) {
            snprintf(err, errlen, "top cell %d paired without a dual link", c);
            return false;
        }
    return true;
}

bool entry2d(uint32_t present, uint32_t *out, char *err, int errlen) {
    Local L;
    if (!reduce_local(present, L, err, errlen) || !dual_links(present, true, L, err, errlen)) return false;
    static const int ecode[4] = {2, 3, 4, 5}, qcode[4] = {11, 12, 13, 14};
    uint32_t e = kNoDirect;
    if (L.partner[0] >= 0) {
        for (int i = 0; i < 4; ++i) if (L.partner[0] == ecode[i]) e = i;
        if (e == kNoDirect) { snprintf(err, errlen, "vertex paired with a non-edge"); return false; }
    }
    for (int i = 0; i < 4; ++i) {
        int c = ecode[i];
        if (!((present >> c) & 1u)) continue;
        if (L.partner[c] < 0) e |= 1u << (kL2Keep + i);                   // KEEP
    }
    for (int q = 0; q < 4; ++q) {
        int c = qcode[q];
        if (!((present >> c) & 1u)) continue;
        e |= 1u << (kL2Present + q);
        if (L.partner[c] < 0) { e |= 1u << (kL2Root + q); continue; }     // ROOT
        int t = L.link[c];
        uint32_t quad = ((kOff[t][1] > 0) << 1) | (kOff[t][2] > 0);
        e |= quad << (kL2Link + 2 * q);
    }
    *out = e;
    return true;
}

// H1 rows of a 3D configuration (Sec. 4.2 steps 4-5): per edge slot i of L(v) paired with a
// square tau of L(v), the squares of L(v) (12-bit mask, bit s = code 7 + s) whose boundaries
// sum to tau's reduced column, whose last entry is that edge; per square slot s that stays
// critical, the squares whose boundaries sum to zero inside L(v) (s itself and the earlier
// columns its reduction added).  0 where the slot has no such role.
bool h1rows(const Local &L, uint32_t present, uint16_t *edge, uint16_t *square, char *err, int errlen) {
    for (int i = 0; i < 8; ++i) edge[i] = 0;
    for (int s = 0; s < 16; ++s) square[s] = 0;
    for (int i = 0; i < 6; ++i) {
        const int c = 1 + i, t = L.partner[c];
        if (!((present >> c) & 1u) || t < 7) continue;        // absent, critical or paired with v
        if (t > 18 || !L.birth[c]) { snprintf(err, errlen, "edge %d paired with cell %d", c, t); return false; }
        edge[i] = (uint16_t)((L.comb[t] >> 7) & 0xFFFu);
        if (L.comb[t] & ~(0xFFFu << 7)) { snprintf(err, errlen, "square combination leaves the squares"); return false; }
    }
    for (int s = 0; s < 12; ++s) {
        const int c = 7 + s;
        if (!((present >> c) & 1u) || L.partner[c] >= 0) continue;
        square[s] = (uint16_t)((L.comb[c] >> 7) & 0xFFFu);
        if (L.comb[c] & ~(0xFFFu << 7)) { snprintf(err, errlen, "square combination leaves the squares"); return false; }
    }
    return true;
}

bool entry3d(uint32_t present, uint64_t *out, uint16_t *h1e, uint16_t *h1s, char *err, int errlen) {
    Local L;
    if (!reduce_local(present, L, err, errlen) || !dual_links(present, false, L, err, errlen)) return false;
    if (!h1rows(L, present, h1e, h1s, err, errlen)) return false;
    uint64_t e = kNoDirect;
    if (L.partner[0] >= 0) e = (uint64_t)(L.partner[0] - 1);
    for (int i = 0; i < 6; ++i) {
        int c = 1 + i;
        if (((present >> c) & 1u) && L.partner[c] < 0) e |= 1ull << (kL3Keep + i);
    }
    for (int s = 0; s < 12; ++s) {
        int c = 7 + s;
        if (((present >> c) & 1u) && L.partner[c] < 0) e |= 1ull << (kL3KeepSq + s);
    }
    for (int b = 0; b < 8; ++b) {
        int c = 19 + b;
        if (!((present >> c) & 1u)) continue;
        e |= 1ull << (kL3Present + b);
        if (L.partner[c] < 0) { e |= 1ull << (kL3Root + b); continue; }
        int t = L.link[c];
        uint64_t oct = ((uint64_t)(kOff[t][0] > 0) << 2) | ((kOff[t][1] > 0) << 1) | (kOff[t][2] > 0);
        e |= oct << (kL3Link + 3 * b);
    }
    *out = e;
    return true;
}

}  // namespace

// 2D: 256 entries indexed by the raw mask (bit i: neighbour of code {2,3,4,5,11,12,13,14}[i]).
// Returns the number of distinct lower-star configurations, or -1 on error.
int build_lut2d(uint32_t *lut, char *err, int errlen) {
    static const int ncode[8] = {2, 3, 4, 5, 11, 12, 13, 14};
    std::vector<uint32_t> seen;
    for (uint32_t m = 0; m < 256; ++m) {
        uint32_t present = 1u;                      // the vertex
        for (int i = 0; i < 4; ++i) if ((m >> i) & 1u) present |= 1u << ncode[i];
        for (int q = 0; q < 4; ++q) {               // a square needs its diagonal and both sides
            int c = ncode[4 + q];
            int dy = kOff[c][1], dx = kOff[c][2];
            int ey = code_of(0, dy, 0), ex = code_of(0, 0, dx);
            if (((m >> (4 + q)) & 1u) && ((present >> ey) & 1u) && ((present >> ex) & 1u)) present |= 1u << c;
        }
        if (!entry2d(present, &lut[m], err, errlen)) return -1;
        bool dup = false;
        for (uint32_t p : seen) dup |= (p == present);
        if (!dup) seen.push_back(present);
    }
    return (int)seen.size();
}

// 3D: level 1 (2^18 words) and level 2 (kL3Configs entries), and the H1 rows of every level-2
// entry (h1e: 8 uint16 per entry, h1s: 16 uint16 per entry; see h1rows).  Returns the config
// count or -1.
int build_lut3d(uint32_t *l1, uint64_t *l2, uint16_t *h1e, uint16_t *h1s, char *err, int errlen) {
    memset(l1, 0, sizeof(uint32_t) * kL1Size);
    uint32_t next = 0;
    for (uint32_t face = 0; face < 64; ++face) {
        uint32_t relsq = 0;                          // squares whose two faces are present
        for (int s = 0; s < 12; ++s) {
            uint32_t need = (1u << kSqFace[s][0]) | (1u << kSqFace[s][1]);
            if ((face & need) == need) relsq |= 1u << s;
        }
        for (uint32_t sq = 0; sq < 4096; ++sq) {
            if (sq & ~relsq) continue;               // only canonical square sets
            uint32_t poss = possible_cubes(sq);
            uint32_t idx1 = face | (sq << 6);
            uint32_t n2 = 1u << __builtin_popcount(poss);
            if (next + n2 > (uint32_t)kL3Configs) { snprintf(err, errlen, "too many 3D configurations"); return -1; }
            l1[idx1] = (next << 8) | poss;
            for (uint32_t cb = 0; cb < 256; ++cb) {
                if (cb & ~poss) continue;
                uint32_t present = 1u;
                for (int i = 0; i < 6; ++i) if ((face >> i) & 1u) present |= 1u << (1 + i);
                for (int s = 0; s < 12; ++s) if ((sq >> s) & 1u) present |= 1u << (7 + s);
                for (int c = 0; c < 8; ++c) if ((cb >> c) & 1u) present |= 1u << (19 + c);
                uint32_t slot = next + compress8(cb, poss);
                if (!entry3d(present, &l2[slot], h1e + 8 * (size_t)slot, h1s + 16 * (size_t)slot, err, errlen)) return -1;
            }
            next += n2;
        }
    }
    // every other square set maps to the entry of its canonical set (the squares whose two
    // faces are present), so the kernels index level 1 with the raw face and square bits
    for (uint32_t face = 0; face < 64; ++face) {
        uint32_t relsq = 0;
        for (int s = 0; s < 12; ++s) {
            uint32_t need = (1u << kSqFace[s][0]) | (1u << kSqFace[s][1]);
            if ((face & need) == need) relsq |= 1u << s;
        }
        for (uint32_t sq = 0; sq < 4096; ++sq)
            if (sq & ~relsq) l1[face | (sq << 6)] = l1[face | ((sq & relsq) << 6)];
    }
    return (int)next;
}

}  // namespace fc
