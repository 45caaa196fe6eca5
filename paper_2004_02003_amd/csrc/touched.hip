// Touched grid points per step: the exact count behind the per-unit byte
// figure of a seeding whose particles rarely share cells (stride 4 and up).
//
// The seeds walk the interval one step per launch with the adjoint's forward
// arithmetic (FP64 position from the seed's world coordinates, rk4_step on
// the same corner values).  Every cell a stage samples marks the eight corner
// points of the level it reads in one bitmap per level; after the step a
// second kernel adds up the set bits and clears the words for the next step.
#include "bto_internal.h"

namespace bto {

// A register cell cache that also marks, on every reload, the corner points
// of the cell it loads (atomicOr into a bitmap of the block's points).
template <int DT>
struct MarkCache : CellCache<DT> {
    uint32_t* bits;
};

template <int DT, class C>
__device__ __forceinline__ bool fetch(const Geom& g, const char* V, const C& c, MarkCache<DT>& k) {
    const uint32_t b = c.base;
    if (k.base != b) {
        const uint32_t sy = (uint32_t)g.sy, sz = (uint32_t)g.sz;
        const uint32_t row[4] = {b, b + sy, b + sz, b + sy + sz};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (uint32_t q = 0; q < 2; ++q) {
                const uint32_t p = row[r] + q;
                atomicOr(&k.bits[p >> 5], 1u << (p & 31u));
            }
        }
    }
    ensure<DT>(g, V, b, static_cast<CellCache<DT>&>(k));
    return true;
}

__global__ __launch_bounds__(BLOCK) void touch_init_kernel(const TouchArgs a) {
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < a.P; p += (int64_t)gridDim.x * BLOCK) {
        double x[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = (a.seed_xyz[3 * p + d] - a.origin[d]) * a.g.inv_sp[d];
            a.x[3 * p + d] = x[d];
        }
        a.alive[p] = inside(a.g, x) ? 1u : 0u;
    }
}

template <int DT, int MODE>
__global__ __launch_bounds__(BLOCK) void touch_step_kernel(const TouchArgs a) {
    const char* V0 = in_global(a.f0);
    const char* V1 = in_global(a.f1);
    const int lane = threadIdx.x % WAVE;
    uint32_t entering = 0;
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < a.P; p += (int64_t)gridDim.x * BLOCK) {
        if (!a.alive[p]) continue;
        ++entering;
        double x[3] = {a.x[3 * p], a.x[3 * p + 1], a.x[3 * p + 2]};
        MarkCache<DT> A, B;
        A.base = B.base = NO_CELL;
        A.bits = a.bits0;
        B.bits = a.bits1;
        const auto no_exit = [](const double*) {};
        const int status = rk4_step<DT, MODE>(a.g, V0, V1, a.h, x, A, B, no_exit);
        if (status == S_VALID) {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.x[3 * p + d] = x[d];
        } else {
            a.alive[p] = 0u;
        }
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) entering += __shfl_xor(entering, o);
    if (lane == 0 && entering) atomicAdd(a.out + 2, (unsigned long long)entering);
}

// Set bits of a bitmap into *out; every word is cleared for the next step.
__global__ __launch_bounds__(BLOCK) void touch_count_kernel(uint32_t* bits, size_t words, unsigned long long* out) {
    const int lane = threadIdx.x % WAVE;
    uint32_t n = 0;
    for (size_t w = (size_t)blockIdx.x * BLOCK + threadIdx.x; w < words; w += (size_t)gridDim.x * BLOCK) {
        n += (uint32_t)__popc(bits[w]);
        bits[w] = 0u;
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) n += __shfl_xor(n, o);
    if (lane == 0 && n) atomicAdd(out, (unsigned long long)n);
}

__global__ void touch_zero_kernel(unsigned long long* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

static unsigned grid_of(size_t n) {
    size_t g = (n + BLOCK - 1) / BLOCK;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

hipError_t launch_touch_init(const TouchArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(touch_init_kernel, dim3(grid_of((size_t)a.P)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int DT>
static hipError_t touch_step_dt(const TouchArgs& a, int mode, hipStream_t s) {
    const dim3 g(grid_of((size_t)a.P)), b(BLOCK);
    switch (mode) {
    case MODE_LINEAR: hipLaunchKernelGGL((touch_step_kernel<DT, MODE_LINEAR>), g, b, 0, s, a); break;
    case MODE_FROZEN: hipLaunchKernelGGL((touch_step_kernel<DT, MODE_FROZEN>), g, b, 0, s, a); break;
    case MODE_LINEAR | MODE_FP64:
        hipLaunchKernelGGL((touch_step_kernel<DT, MODE_LINEAR | MODE_FP64>), g, b, 0, s, a);
        break;
    case MODE_FROZEN | MODE_FP64:
        hipLaunchKernelGGL((touch_step_kernel<DT, MODE_FROZEN | MODE_FP64>), g, b, 0, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_touch_step(const TouchArgs& a, int dtype, int mode, hipStream_t s) {
    switch (dtype) {
    case DT_F32: return touch_step_dt<DT_F32>(a, mode, s);
    case DT_F16: return touch_step_dt<DT_F16>(a, mode, s);
    case DT_BF16: return touch_step_dt<DT_BF16>(a, mode, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_touch_count(uint32_t* bits, size_t words, unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(touch_count_kernel, dim3(grid_of(words)), dim3(BLOCK), 0, s, bits, words, out);
    return hipGetLastError();
}

hipError_t launch_touch_zero(unsigned long long* p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(touch_zero_kernel, dim3(grid_of(n)), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace bto
