// Deterministic reduction of the adjoint's grid-gradient records.
//
// The reverse sweep appends one record per accumulator flush: the 8 corner
// gradients (x 3 components) of one cell of one grid level, keyed by
// parity colour | level | cell | seed id.  A stable radix sort orders the
// records by key; then, one colour at a time, each (level, cell) group is
// summed in key order (by seed id, then flush order) and added to the grid's
// 8 corners with plain loads and stores.  Two different cells of one colour
// differ by at least two cells along some axis, so their corner sets are
// disjoint and the stores of one colour never collide; the colours are
// applied in a fixed order.  The result does not depend on thread timing,
// unlike FP32 atomics, and each corner costs one read and one write per
// group instead of one memory-side atomic per contribution.
#include <rocprim/device/device_radix_sort.hpp>

#include "bto_internal.h"

namespace bto {

__global__ __launch_bounds__(BLOCK) void grad_apply_kernel(const uint64_t* key, const uint32_t* idx, const float* val,
                                                           uint32_t n, uint64_t colour, int colour_shift,
                                                           int pid_bits, uint64_t cell_mask, int level_shift,
                                                           uint64_t level_mask, float* const* gf, Geom g) {
    // a group is one (colour, level, cell): the key without its seed-id bits
    const int group_shift = pid_bits;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const uint64_t k = key[i];
        if ((k >> colour_shift) != colour) continue;
        const uint64_t group = k >> group_shift;
        if (i > 0 && (key[i - 1] >> group_shift) == group) continue;  // not the first record of its group
        float s[24];
#pragma unroll
        for (int q = 0; q < 24; ++q) s[q] = 0.f;
        for (uint32_t j = i; j < n && (key[j] >> group_shift) == group; ++j) {
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
        const uint32_t base = (uint32_t)((k >> pid_bits) & cell_mask);
        const int level = (int)((k >> level_shift) & level_mask);
        float* grid = gf[level];
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

size_t grad_sort_temp_bytes(uint32_t cap, int bits) {
    size_t bytes = 0;
    if (rocprim::radix_sort_pairs(nullptr, bytes, (uint64_t*)nullptr, (uint64_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, (size_t)cap, 0u, (unsigned)bits) != hipSuccess)
        return 0;
    return bytes;
}

hipError_t launch_grad_reduce(const GradRec& r, uint32_t n, uint64_t* key_out, uint32_t* idx_out, void* temp,
                              size_t temp_bytes, float* const* gf, const Geom& g, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int colour_shift = r.level_bits + r.cell_bits + r.pid_bits;
    const int bits = colour_shift + 3;
    size_t bytes = temp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(temp, bytes, r.key, key_out, r.idx, idx_out, (size_t)n, 0u,
                                             (unsigned)bits, s);
    if (e != hipSuccess) return e;
    const uint64_t cell_mask = (r.cell_bits >= 64) ? ~0ull : ((1ull << r.cell_bits) - 1ull);
    const uint64_t level_mask = (1ull << r.level_bits) - 1ull;
    const unsigned blocks = (unsigned)((n + BLOCK - 1) / BLOCK);
    for (uint64_t colour = 0; colour < 8; ++colour) {
        hipLaunchKernelGGL(grad_apply_kernel, dim3(blocks), dim3(BLOCK), 0, s, key_out, idx_out, r.val, n, colour,
                           colour_shift, r.pid_bits, cell_mask, r.cell_bits + r.pid_bits, level_mask, gf, g);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace bto
