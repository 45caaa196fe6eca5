// Spatial re-sort of live particles ("rebin", part of particle management).
//
// Particles start in lattice order, so the 64 lanes of a wavefront read nearby
// cells and share cache lines; as the flow disperses them that locality
// decays and every lane touches its own lines.  Between advection launches the
// live particles of each XCD segment are re-ordered by the 32x2x2-cell bin
// that holds them, bins in x-fastest order (a wavefront's particles then lie
// along a few grid rows, so each of a cell's row loads covers long runs of
// contiguous memory -- the same reason the lattice is seeded x-fastest), with
// a counting sort:
//   count   - per particle, atomically increment its (segment, bin) counter;
//             the old value is the particle's rank inside the bin;
//   scan    - exclusive prefix sum over all bins (segment-major; radix.hip);
//   scatter - move each particle to its segment base + bin offset + rank, and
//             zero its bin for the next rebin.
// Order inside a bin is unspecified; results do not depend on particle
// order.
#include "bto_internal.h"

namespace bto {

__device__ __forceinline__ int segment_of(const Segs& sg, int64_t i) {
    int seg = 0;
#pragma unroll
    for (int x = 1; x < NSEG; ++x) seg += (i >= sg.base[x]) ? 1 : 0;
    return seg;
}

__global__ __launch_bounds__(BLOCK) void rebin_count_kernel(const RebinArgs a) {
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < a.P; i += (int64_t)gridDim.x * BLOCK) {
        const int seg = segment_of(a.segs, i);
        if (i - a.segs.base[seg] >= (int64_t)a.count[seg * CSTRIDE]) continue;  // slot beyond the segment's live count
        const uint32_t c = a.pos[i].cell;
        const uint32_t key = (c & 1023u) / REBIN_BIN[0] +
                             a.nbx * (((c >> 10) & 1023u) / REBIN_BIN[1] + a.nby * (((c >> 20) & 1023u) / REBIN_BIN[2]));
        const uint32_t bin = (uint32_t)seg * a.nbins + key;
        a.bin[i] = bin;
        a.rank[i] = atomicAdd(&a.hist[bin], 1u);
    }
}

__global__ __launch_bounds__(BLOCK) void rebin_scatter_kernel(const RebinArgs a) {
    uint32_t start[NSEG];
    uint32_t acc = 0;
#pragma unroll
    for (int x = 0; x < NSEG; ++x) {
        start[x] = acc;
        acc += a.count[x * CSTRIDE];
    }
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < a.P; i += (int64_t)gridDim.x * BLOCK) {
        const int seg = segment_of(a.segs, i);
        if (i - a.segs.base[seg] >= (int64_t)a.count[seg * CSTRIDE]) continue;
        const uint32_t bin = a.bin[i];
        const int64_t dst = a.segs.base[seg] + (int64_t)(a.offs[bin] - start[seg]) + a.rank[i];
        a.out_pos[dst] = a.pos[i];
        a.out_id[dst] = a.id[i];
        a.hist[bin] = 0u;  // every particle of the bin writes the same zero
    }
}

static int grid_of(int64_t n) {
    int64_t b = (n + BLOCK - 1) / BLOCK;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

size_t rebin_temp_bytes(int64_t nbins_total) { return scan_temp_bytes((uint64_t)nbins_total); }

hipError_t launch_rebin(const RebinArgs& a, hipStream_t s) {
    if (a.P == 0) return hipSuccess;
    hipLaunchKernelGGL(rebin_count_kernel, dim3(grid_of(a.P)), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(a.hist, a.offs, (uint64_t)NSEG * a.nbins, a.temp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rebin_scatter_kernel, dim3(grid_of(a.P)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace bto
