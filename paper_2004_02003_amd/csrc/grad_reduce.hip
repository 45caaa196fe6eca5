// Deterministic reduction of the adjoint's grid-gradient records.
//
// The reverse sweep writes one record per accumulator flush into a slot fixed
// by (flush rank, seed): the 8 corner gradients (x 3 components) of one cell
// of one grid level, keyed by parity colour | level | cell (unused slots carry
// a key above every colour).  A stable radix sort (radix.hip) orders the
// records by key;
// then, one colour at a time (a contiguous range of the sorted keys), each
// (level, cell) group is summed in slot order (the flush's rank, then the
// seed id) and added to the grid's 8 corners with plain loads and stores.
// Two different cells of one colour differ by at least two cells along some
// axis, so their corner sets are disjoint and the stores of one colour never
// collide; the colours are applied in a fixed order.  The result does not
// depend on thread timing, unlike FP32 atomics, and each corner costs one
// read and one write per group instead of one memory-side atomic per
// contribution.
#include "bto_internal.h"

namespace bto {

// Before a sweep: every slot unused, and each slot's sort value its own index
// (written here in one coalesced pass rather than by the sweep's scattered
// record stores).
__global__ __launch_bounds__(BLOCK) void grad_clear_kernel(uint64_t* key, uint32_t* idx, uint64_t n, uint64_t empty) {
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (uint64_t)gridDim.x * BLOCK) {
        key[i] = empty;
        idx[i] = (uint32_t)i;
    }
}

// bounds[c] = first sorted slot of colour c (c = 0..8; colour 8 = unused slots).
__global__ __launch_bounds__(BLOCK) void grad_bounds_kernel(const uint64_t* key, uint64_t n, int colour_shift,
                                                            uint32_t* bounds) {
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i <= n; i += (uint64_t)gridDim.x * BLOCK) {
        const uint64_t c = i < n ? (key[i] >> colour_shift) : 9;
        const uint64_t cp = i > 0 ? (key[i - 1] >> colour_shift) : 0;
        const uint64_t lo = i > 0 ? cp + 1 : 0;
        for (uint64_t q = lo; q <= c && q <= 8; ++q) bounds[q] = (uint32_t)i;
    }
}

__global__ __launch_bounds__(BLOCK) void grad_apply_kernel(const uint64_t* key, const uint32_t* idx, const float* val,
                                                           const uint32_t* bounds, int colour, uint64_t cell_mask,
                                                           int level_shift, uint64_t level_mask, float* const* gf,
                                                           Geom g) {
    // a group is one (colour, level, cell): a run of equal keys
    const uint32_t lo = bounds[colour], hi = bounds[colour + 1];
    for (uint32_t i = lo + blockIdx.x * BLOCK + threadIdx.x; i < hi; i += gridDim.x * BLOCK) {
        const uint64_t k = key[i];
        if (i > lo && key[i - 1] == k) continue;  // not the first record of its group
        float s[24];
#pragma unroll
        for (int q = 0; q < 24; ++q) s[q] = 0.f;
        for (uint32_t j = i; j < hi && key[j] == k; ++j) {
            const float4* v = reinterpret_cast<const float4*>(val + 24 * (size_t)idx[j]);
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float4 x = v[q];
                s[4 * q + 0] += x.x;
                s[4 * q + 1] += x.y;
                s[4 * q + 2] += x.z;
                s[4 * q + 3] += x.w;
            }
        }
        const uint32_t base = (uint32_t)(k & cell_mask);
        const int level = (int)((k >> level_shift) & level_mask);
        float* grid = in_global(gf[level]);
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    float* p = grid + 3 * ((uint64_t)base + (uint64_t)q + (uint64_t)g.sy * b + (uint64_t)g.sz * c);
                    const int m = 3 * (q + 2 * b + 4 * c);
                    p[0] += s[m + 0];
                    p[1] += s[m + 1];
                    p[2] += s[m + 2];
                }
    }
}

static int key_bits(const GradRec& r) { return r.level_bits + r.cell_bits + 3; }

size_t grad_sort_temp_bytes(uint64_t n, int) { return radix_temp_bytes(n); }

static unsigned grid_of(uint64_t n) {
    const uint64_t b = (n + BLOCK - 1) / BLOCK;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

hipError_t launch_grad_clear(const GradRec& r, uint64_t n, hipStream_t s) {
    // unused slots: the colour field reads 8, above every real colour
    const uint64_t empty = (uint64_t)8 << (key_bits(r) - 3);
    hipLaunchKernelGGL(grad_clear_kernel, dim3(grid_of(n)), dim3(BLOCK), 0, s, r.key, r.idx, n, empty);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const GradRec& r, uint64_t n, uint64_t* key_out, uint32_t* idx_out, uint32_t* bounds,
                              void* temp, size_t temp_bytes, float* const* gf, const Geom& g, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int colour_shift = key_bits(r) - 3;
    (void)temp_bytes;
    // one more bit than the key fields: the unused-slot marker; the sorted
    // pairs end in (key_out, idx_out) or, after an even number of passes, in
    // the records' own arrays
    bool in_alt = false;
    hipError_t e = launch_radix_sort_pairs(r.key, r.idx, key_out, idx_out, n, key_bits(r) + 1, temp, &in_alt, s);
    if (e != hipSuccess) return e;
    if (!in_alt) {
        key_out = r.key;
        idx_out = r.idx;
    }
    hipLaunchKernelGGL(grad_bounds_kernel, dim3(grid_of(n + 1)), dim3(BLOCK), 0, s, key_out, n, colour_shift, bounds);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t cell_mask = (1ull << r.cell_bits) - 1ull;
    const uint64_t level_mask = (1ull << r.level_bits) - 1ull;
    for (int colour = 0; colour < 8; ++colour) {
        hipLaunchKernelGGL(grad_apply_kernel, dim3(grid_of(n / 8 + 1)), dim3(BLOCK), 0, s, key_out, idx_out, r.val,
                           bounds, colour, cell_mask, r.cell_bits, level_mask, gf, g);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace bto
