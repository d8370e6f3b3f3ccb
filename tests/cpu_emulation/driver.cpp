// Runs the library's kernels on the CPU (through the emulated HIP runtime) for the test suite.
//
//   driver in.bin out.bin
//
// in.bin (little-endian): int32 n, uint32 flags, int32 mode (0: ph_diagram, n must be 1;
// 1: ph_diagram_batch; 2: ph_autotune then ph_diagram_batch), int32 tile2d, int32 tile3d
// (-1: no tuning argument), int32 backward (1: also run ph_backward for the loss
// sum over finite pairs of (death - birth)^2; 2: the same gradient from ph_diagram_batch_grad,
// on a gradient buffer full of NaNs, then ph_backward_scatter; mode 1 or 2 only), int32
// capacity per instance (-1: the bound);
// then n x (int32 ndim, int32 ext[3]); then the pixels of all instances, float32,
// concatenated.
// out.bin: per instance int64 count, int32 status, then the stored pairs as int32 dim,
// float32 birth, float32 death, int64 birth_cell, int64 death_cell, int32 birth_vertex,
// int32 death_vertex; then, with backward, the float32 gradient of all pixels.
//
// Under AddressSanitizer the workspace gaps between the per-instance arrays (and the unused
// tail) are poisoned as soon as the plan kernel has written the instance table, so a kernel
// that runs past the end of one of its arrays is reported even when it stays inside the
// workspace allocation.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <array>
#include <vector>

#include "hip/hip_runtime.h"
#include "flashcubical.h"
#include "fc_common.h"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#if __has_feature(memory_sanitizer)
#include <sanitizer/msan_interface.h>
#define EMU_MSAN_DRIVER 1
#endif
#endif
#ifdef __SANITIZE_ADDRESS__
#define EMU_ASAN 1
#endif
#ifdef EMU_ASAN
#include <sanitizer/asan_interface.h>
#endif

// the emulated runtime's globals and fiber switch live in runtime.cpp

namespace {

uint8_t *g_ws = nullptr;
size_t g_wsb = 0;
int g_n = 0;
bool g_guarded = false;

int64_t a256(int64_t x) { return (x + 255) & ~(int64_t)255; }

void poison(int64_t from, int64_t to) {
#ifdef EMU_ASAN
    if (to > from) __asan_poison_memory_region(g_ws + from, (size_t)(to - from));
#else
    (void)from;
    (void)to;
#endif
}

// layout of the workspace header and arrays, restated from the header comments of fc_common.h
void guard_workspace(const void *) {
    if (g_guarded) return;                        // the first launch of a call is the plan kernel
    g_guarded = true;
    const int n = g_n;
    const int64_t tb2 = a256((int64_t)n * (int64_t)sizeof(fc::Inst));
    const int64_t tb3 = tb2 + a256((int64_t)(n + 1) * 8), cn = tb3 + a256((int64_t)(n + 1) * 8);
    const int64_t hdr = cn + a256((int64_t)n * fc::CNT_WORDS * 4);
    poison((int64_t)n * (int64_t)sizeof(fc::Inst), tb2);
    poison(tb2 + (int64_t)(n + 1) * 8, tb3);
    poison(tb3 + (int64_t)(n + 1) * 8, cn);
    poison(cn + (int64_t)n * fc::CNT_WORDS * 4, hdr);
    int64_t expect = hdr;
    for (int i = 0; i < n; ++i) {
        const fc::Inst &I = ((const fc::Inst *)g_ws)[i];
        const int64_t N = I.N, T = I.T, E = I.E, F = I.F, FAC = I.FAC;
        const int64_t L = (E > F ? E : F) > 0 ? (E > F ? E : F) : 1, SCR = L > N ? L : N;
        std::vector<std::array<int64_t, 2>> a = {
            {I.o_par0, 4 * N}, {I.o_parT, 4 * T}, {I.o_keyE, 8 * E}, {I.o_ea, 4 * E},
            {I.o_eb, 4 * E}, {I.o_neg0, 4 * E}, {I.o_keyF, 8 * F}, {I.o_fa, 4 * FAC},
            {I.o_fb, 4 * FAC}, {I.o_killer, 4 * FAC}, {I.o_n0key, 8 * N},
            {I.o_n0sorted, 8 * N}, {I.o_nTkey, 8 * (T + 1)}, {I.o_uf0, 4 * N},
            {I.o_moe0, 4 * N}, {I.o_death0, 4 * N}, {I.o_ufT, 4 * (T + 1)},
            {I.o_moeT, 4 * (T + 1)}, {I.o_live, 8 * L}, {I.o_ra, 8 * L},
            {I.o_scratch, 8 * SCR}};
        if (I.h1 && I.ndim == 3) {                                   // 3D H1
            const int64_t h1arr[][2] = {{I.o_cfg3, 2 * N}, {I.o_kpos, 4 * N}, {I.o_h1b, 4 * F}, {I.o_h1n, 4 * F},
                                        {I.o_piv, 4 * E}, {I.o_first, 4 * E}, {I.o_pool, 4 * I.pool_cap},
                                        {I.o_retry, 4 * F}};
            for (const auto &x : h1arr) a.push_back({x[0], x[1]});
        }
        const int na = (int)a.size();
        if (a[0][0] != expect) { fprintf(stderr, "driver: unexpected workspace layout\n"); abort(); }
        for (int k = 0; k < na; ++k) {
            const int64_t next = k + 1 < na ? a[k + 1][0] : I.end;
            poison(a[k][0] + a[k][1], next);
        }
        expect = I.end;
    }
    poison(expect, (int64_t)g_wsb);
}

void unguard() {
#ifdef EMU_ASAN
    __asan_unpoison_memory_region(g_ws, g_wsb);
#endif
    g_guarded = false;
}

template <typename T> void uninit(T *p, size_t count) {
#ifdef EMU_MSAN_DRIVER
    __msan_poison(p, count * sizeof(T));
#else
    (void)p;
    (void)count;
#endif
}

// Every buffer a kernel receives is device memory of the emulated runtime (hipMalloc), as on
// the GPU; only h_shapes stays in host memory.
template <typename T> T *dev_alloc(size_t count) {
    void *p = nullptr;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) { fprintf(stderr, "driver: hipMalloc\n"); exit(2); }
    return (T *)p;
}
template <typename T> T *dev_copy(const std::vector<T> &v) {
    T *p = dev_alloc<T>(v.size());
    if (!v.empty()) memcpy(p, v.data(), v.size() * sizeof(T));
    return p;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 3) { fprintf(stderr, "usage: driver in.bin out.bin\n"); return 2; }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[7];
    if (fread(hdr, 4, 7, f) != 7) return 2;
    const int n = hdr[0], mode = hdr[2], backward = hdr[5];
    const uint32_t flags = (uint32_t)hdr[1];
    std::vector<ph_shape> shapes(n);
    std::vector<int64_t> img_off(n + 1, 0), out_off(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        int32_t s[4];
        if (fread(s, 4, 4, f) != 4) return 2;
        shapes[i].ndim = s[0];
        int64_t nv = 1;
        for (int k = 0; k < 3; ++k) {
            shapes[i].ext[k] = s[1 + k];
            if (k < s[0]) nv *= s[1 + k];
        }
        img_off[i + 1] = img_off[i] + nv;
        out_off[i + 1] = out_off[i] + (hdr[6] >= 0 ? hdr[6] : ph_capacity_bound_flags(shapes[i], flags));
    }
    std::vector<float> img(img_off[n]);
    if (fread(img.data(), 4, img.size(), f) != img.size()) return 2;
    fclose(f);

    const int64_t cap = out_off[n];
    g_wsb = ph_workspace_bytes(shapes.data(), n, flags);
    uint8_t *ws = dev_alloc<uint8_t>(g_wsb);
    for (size_t k = 0; k < g_wsb; ++k) ws[k] = (uint8_t)(k * 2654435761u >> 13);   // garbage
    uninit(ws, g_wsb);
    g_ws = ws;
    g_n = n;
    float *d_img = dev_copy(img);
    int64_t *d_img_off = dev_copy(img_off), *d_out_off = dev_copy(out_off);
    ph_shape *d_shapes = dev_copy(shapes);
    int8_t *dim = dev_alloc<int8_t>(cap);
    float *birth = dev_alloc<float>(cap), *death = dev_alloc<float>(cap);
    int64_t *bcell = dev_alloc<int64_t>(cap), *dcell = dev_alloc<int64_t>(cap), *counts = dev_alloc<int64_t>(n);
    int32_t *bvert = dev_alloc<int32_t>(cap), *dvert = dev_alloc<int32_t>(cap), *status = dev_alloc<int32_t>(n);
    uninit(dim, cap); uninit(birth, cap); uninit(death, cap); uninit(bcell, cap); uninit(dcell, cap);
    uninit(bvert, cap); uninit(dvert, cap); uninit(counts, n); uninit(status, n);
    ph_pairs out{dim, birth, death, bcell, dcell, bvert, dvert};
    ph_tuning tune{hdr[3], hdr[4]};
    const ph_tuning *tp = hdr[3] >= 0 ? &tune : nullptr;
    float *grad = nullptr;
    if (backward) {
        grad = dev_alloc<float>(img.size());
        uninit(grad, img.size());
    }
    if (backward == 2) {
        if (mode == 0) return 2;
        for (size_t k = 0; k < img.size(); ++k) grad[k] = __builtin_nanf("");
    }
    emu_after_launch = guard_workspace;
    int rc;
    if (mode == 0) {
        if (n != 1) return 2;
        rc = ph_diagram(d_img, shapes[0], flags, out, cap, counts, status, ws, g_wsb, nullptr);
    } else {
        if (mode == 2) {
            ph_tuning best{0, 0};
            rc = ph_autotune(n, d_img, d_img_off, d_shapes, shapes.data(), flags, out, d_out_off, counts, status,
                             ws, g_wsb, 1, &best, nullptr);
            unguard();
            if (rc != PH_OK) { fprintf(stderr, "driver: autotune rc %d\n", rc); return 3; }
        }
        if (backward == 2)
            rc = ph_diagram_batch_grad(n, d_img, d_img_off, d_shapes, shapes.data(), flags, out, d_out_off, counts,
                                       status, tp, ws, g_wsb, grad, nullptr);
        else
            rc = ph_diagram_batch(n, d_img, d_img_off, d_shapes, shapes.data(), flags, out, d_out_off, counts,
                                  status, tp, ws, g_wsb, nullptr);
    }
    unguard();
    emu_after_launch = nullptr;
    if (rc != PH_OK) { fprintf(stderr, "driver: rc %d\n", rc); return 3; }
    if (getenv("EMU_STATS")) {                    // per-instance work counters, for sizing studies
        const int64_t cn = a256((int64_t)n * (int64_t)sizeof(fc::Inst)) + 2 * a256((int64_t)(n + 1) * 8);
        for (int i = 0; i < n; ++i) {
            const int32_t *c = (const int32_t *)(ws + cn) + i * fc::CNT_WORDS;
            const fc::Inst &I = ((const fc::Inst *)ws)[i];
            fprintf(stderr, "stats %d N %ld keepE %d keepF %d minima %d roots %d rounds0 %d roundsT %d seq %d\n", i,
                    (long)I.N, c[fc::CNT_E], c[fc::CNT_F], c[fc::CNT_M0], c[fc::CNT_MT], c[fc::CNT_ROUNDS0],
                    c[fc::CNT_ROUNDST], c[fc::CNT_SEQ]);
        }
    }

    if (backward) {
        std::vector<float> gb(cap, 0.f), gd(cap, 0.f);
        for (int i = 0; i < n; ++i)
            for (int64_t j = 0; j < counts[i] && j < out_off[i + 1] - out_off[i]; ++j) {
                const int64_t k = out_off[i] + j;
                if (dcell[k] < 0) continue;
                const float d = death[k] - birth[k];
                gb[k] = -2.f * d;
                gd[k] = 2.f * d;
            }
        float *d_gb = dev_copy(gb), *d_gd = dev_copy(gd);
        rc = (backward == 2 ? ph_backward_scatter : ph_backward)(n, out, d_out_off, counts, d_gb, d_gd, grad,
                                                                 d_img_off, (int64_t)img.size(), nullptr);
        if (rc != PH_OK) { fprintf(stderr, "driver: backward rc %d\n", rc); return 3; }
    }

    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    for (int i = 0; i < n; ++i) {
        fwrite(&counts[i], 8, 1, o);
        fwrite(&status[i], 4, 1, o);
        const int64_t m = counts[i] < out_off[i + 1] - out_off[i] ? counts[i] : out_off[i + 1] - out_off[i];
        for (int64_t j = 0; j < m && (status[i] == PH_OK || status[i] == PH_ECAPACITY); ++j) {
            const int64_t k = out_off[i] + j;
            const int32_t dm = dim[k];
            fwrite(&dm, 4, 1, o); fwrite(&birth[k], 4, 1, o); fwrite(&death[k], 4, 1, o);
            fwrite(&bcell[k], 8, 1, o); fwrite(&dcell[k], 8, 1, o);
            fwrite(&bvert[k], 4, 1, o); fwrite(&dvert[k], 4, 1, o);
        }
    }
    if (backward) fwrite(grad, 4, img.size(), o);
    fclose(o);
    return 0;
}
