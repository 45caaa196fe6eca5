// Kernels of the per-block BTO path around the advection: lattice and
// explicit seeding, counter setup, and the seed-ordered flow-map writer.
#include "bto_internal.h"

namespace bto {

// ---------------------------------------------------------------------------
// Seeding.
// ---------------------------------------------------------------------------

// Slot order of the lattice.  Default: octant-major -- the lattice is split
// in two per axis and each octant fills one XCD segment, in natural x-fastest
// order inside it (a wavefront's lanes lie along grid rows, so each of a
// cell's four row loads covers long contiguous runs of the grid, and each
// XCD keeps a compact octant of the block).  Alternatives for experiments:
// brick-major -- bricks of B0 x B1 x B2 = 64 lattice points (one wavefront)
// in x-fastest brick order, x-fastest inside a brick (64 x 1 x 1 is the plain
// natural order, the segments then being z-slabs); bricks on the high faces
// may be partial and slot(id) is the closed-form prefix count -- and Morton
// order of 4 x 4 x 4 bricks.
__device__ __forceinline__ int64_t brick_slot(const int32_t m[3], const int32_t B[3], int a, int b, int c) {
    const int bx = a / B[0], by = b / B[1], bz = c / B[2];
    const int lx = a % B[0], ly = b % B[1], lz = c % B[2];
    const int cx = min(B[0], m[0] - B[0] * bx), cy = min(B[1], m[1] - B[1] * by), cz = min(B[2], m[2] - B[2] * bz);
    return (int64_t)m[0] * m[1] * B[2] * bz + (int64_t)m[0] * B[1] * by * cz + (int64_t)B[0] * bx * cy * cz +
           lx + cx * (ly + cy * lz);
}

// When the lattice is a cube of 4 * 2^k points per axis the bricks are laid
// out in Morton order instead, so that each eighth of the slots (one XCD
// segment) is a compact octant of the block rather than a slab.
__device__ __forceinline__ uint32_t spread3b(uint32_t v) {
    v &= 0xFFu;
    v = (v | (v << 8)) & 0x0000F00Fu;
    v = (v | (v << 4)) & 0x000C30C3u;
    v = (v | (v << 2)) & 0x00249249u;
    return v;
}

__global__ __launch_bounds__(BLOCK) void seed_lattice_kernel(const SeedLatticeArgs a) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < a.P; t += (int64_t)gridDim.x * BLOCK) {
        const int ia = (int)(t % a.m[0]);
        const int ib = (int)((t / a.m[0]) % a.m[1]);
        const int ic = (int)(t / ((int64_t)a.m[0] * a.m[1]));
        const double x[3] = {a.off[0] + (double)a.stride * ia, a.off[1] + (double)a.stride * ib,
                             a.off[2] + (double)a.stride * ic};
        int64_t slot;
        if (a.octant) {
            // octant-major: octant o = (x high) + 2 (y high) + 4 (z high), x-fastest inside it
            const int hx = ia >= a.half[0], hy = ib >= a.half[1], hz = ic >= a.half[2];
            const int lx = ia - hx * a.half[0], ly = ib - hy * a.half[1], lz = ic - hz * a.half[2];
            const int sx = hx ? a.m[0] - a.half[0] : a.half[0];
            const int sy = hy ? a.m[1] - a.half[1] : a.half[1];
            slot = a.oct_base[hx + 2 * hy + 4 * hz] + lx + (int64_t)sx * (ly + (int64_t)sy * lz);
        } else if (a.morton) {
            slot = (int64_t)(spread3b(ia >> 2) | (spread3b(ib >> 2) << 1) | (spread3b(ic >> 2) << 2)) * 64 +
                   ((ia & 3) + 4 * ((ib & 3) + 4 * (ic & 3)));
        } else {
            slot = brick_slot(a.m, a.brick, ia, ib, ic);
        }
        a.pos[slot] = pack(x);
        a.id[slot] = (uint32_t)t;
#pragma unroll
        for (int d = 0; d < 3; ++d) a.seed_xyz[3 * t + d] = a.origin[d] + a.spacing[d] * x[d];
        a.rec_meta[t] = META_LIVE;
    }
}

__global__ __launch_bounds__(BLOCK) void seed_explicit_kernel(const SeedExplicitArgs a) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < a.P; t += (int64_t)gridDim.x * BLOCK) {
        double x[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double w = a.xyz[3 * t + d];
            a.seed_xyz[3 * t + d] = w;
            x[d] = (w - a.origin[d]) * a.inv_sp[d];
        }
        const int seg = (int)((t * NSEG) / a.P);
        const bool in = inside(a.g, x);
        // slots in the segment: one atomic per wavefront and segment (a wavefront's
        // seeds span one or two segments), ranks from the ballot
        const int lane = threadIdx.x % WAVE;
        const unsigned long long below = (1ull << lane) - 1ull;
        unsigned long long pending = __ballot(in);
        uint32_t k = 0;
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int lseg = __shfl(seg, leader);
            const unsigned long long same = __ballot(in && seg == lseg) & pending;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&a.count[lseg * CSTRIDE], (uint32_t)__popcll(same));
            base = __shfl(base, leader);
            if (in && seg == lseg) k = base + (uint32_t)__popcll(same & below);
            pending &= ~same;
        }
        if (in) {
            a.pos[a.segs.base[seg] + k] = pack(x);
            a.id[a.segs.base[seg] + k] = (uint32_t)t;
            a.rec_meta[t] = META_LIVE;
        } else {
            // outside the block from the start: terminated at step 0, end = seed
            PState s;
            s.cell = 0;
            s.q[0] = s.q[1] = s.q[2] = 0u;
            a.rec_pos[t] = s;  // position taken from seed_xyz by the writer
            a.rec_meta[t] = (S_TERMINATED << META_SHIFT) | META_OUTSIDE;
        }
    }
}

struct CountValues {
    uint32_t v[3 * NSEG];
};

__global__ void set_counts_kernel(uint32_t* counts, const CountValues vals, int n, unsigned long long* psteps) {
    const int t = threadIdx.x;
    if (t < n) counts[t * CSTRIDE] = vals.v[t];
    if (t < NSEG && psteps) psteps[t * PSTRIDE] = 0ull;
}

// ---------------------------------------------------------------------------
// Flow-map writer.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void write_world(const FlowmapArgs& a, int64_t id, const PState& st) {
    double x[3];
    unpack(st, x);
#pragma unroll
    for (int d = 0; d < 3; ++d) a.out_end[3 * id + d] = a.origin[d] + a.spacing[d] * x[d];
}

// Seeds whose particle has ended (terminated or invalid).
__global__ __launch_bounds__(BLOCK) void flowmap_records_kernel(const FlowmapArgs a) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < a.P; t += (int64_t)gridDim.x * BLOCK) {
        if (a.out_seed) {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.out_seed[3 * t + d] = a.seed_xyz[3 * t + d];
        }
        const int32_t meta = a.rec_meta[t];
        if (meta == META_LIVE) continue;
        if (meta & META_OUTSIDE) {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.out_end[3 * t + d] = a.seed_xyz[3 * t + d];
        } else {
            write_world(a, t, a.rec_pos[t]);
        }
        a.out_flag[t] = (uint8_t)(meta >> META_SHIFT);
        a.out_exit[t] = meta & META_STEP;
    }
}

// Particles still advancing: valid, exit step = steps done.
__global__ __launch_bounds__(BLOCK) void flowmap_live_kernel(const FlowmapArgs a) {
    const int seg = blockIdx.x % NSEG;
    const int r = blockIdx.x / NSEG;
    const int R = gridDim.x / NSEG;
    const uint32_t cnt = a.count[seg * CSTRIDE];
    const int64_t sbase = a.segs.base[seg];
    for (uint32_t i = (uint32_t)r * BLOCK + threadIdx.x; i < cnt; i += (uint32_t)R * BLOCK) {
        const uint32_t id = a.id[sbase + i];
        write_world(a, id, a.pos[sbase + i]);
        a.out_flag[id] = (uint8_t)S_VALID;
        a.out_exit[id] = a.steps_done;
    }
}

// Exit points: world coordinates of the point where a terminated trajectory
// left the block (when the advection recorded it); NaN for every other seed.
__global__ __launch_bounds__(BLOCK) void exit_points_kernel(const FlowmapArgs a) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < a.P; t += (int64_t)gridDim.x * BLOCK) {
        const int32_t meta = a.rec_meta[t];
        double w[3] = {__builtin_nan(""), __builtin_nan(""), __builtin_nan("")};
        if (meta != META_LIVE && (meta & META_EXITPT)) {
            double x[3], f[3];
            unpack(a.rec_pos[t], x);
            const float4 o = a.rec_out[t];
            const double y[3] = {x[0] + (double)o.x, x[1] + (double)o.y, x[2] + (double)o.z};
            exit_face(a.g, x, y, f);
#pragma unroll
            for (int d = 0; d < 3; ++d) w[d] = a.origin[d] + a.spacing[d] * f[d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) a.out_face[3 * t + d] = w[d];
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static int grid_for(int64_t n) {
    int64_t b = (n + BLOCK - 1) / BLOCK;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

hipError_t launch_seed_lattice(const SeedLatticeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(seed_lattice_kernel, dim3(grid_for(a.P)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_seed_explicit(const SeedExplicitArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(seed_explicit_kernel, dim3(grid_for(a.P)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_set_counts(uint32_t* counts, const uint32_t* values, int n, unsigned long long* psteps,
                             hipStream_t s) {
    CountValues v;
    for (int q = 0; q < 3 * NSEG; ++q) v.v[q] = q < n ? values[q] : 0u;
    hipLaunchKernelGGL(set_counts_kernel, dim3(1), dim3(64), 0, s, counts, v, n, psteps);
    return hipGetLastError();
}

hipError_t launch_exit_points(const FlowmapArgs& a, hipStream_t s) {
    const int64_t nb = (a.P + BLOCK - 1) / BLOCK;
    const int grid = (int)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096);
    hipLaunchKernelGGL(exit_points_kernel, dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// Checkpoint of the live particles (recorded for the adjoint at the start of
// a launch): the unpacked FP64 position, i.e. exactly the state the next
// advection launch resumes from.
__global__ __launch_bounds__(BLOCK) void ckpt_store_kernel(const CkptArgs a) {
    const int seg = blockIdx.x % NSEG;
    const int r = blockIdx.x / NSEG;
    const int R = gridDim.x / NSEG;
    const uint32_t cnt = a.count[seg * CSTRIDE];
    const int64_t sbase = a.segs.base[seg];
    for (uint32_t i = (uint32_t)r * BLOCK + threadIdx.x; i < cnt; i += (uint32_t)R * BLOCK) {
        const uint32_t id = a.id[sbase + i];
        double x[3];
        unpack(a.pos[sbase + i], x);
#pragma unroll
        for (int d = 0; d < 3; ++d) a.out[3 * (size_t)id + d] = x[d];
    }
}

hipError_t launch_ckpt_store(const CkptArgs& a, int R, hipStream_t s) {
    hipLaunchKernelGGL(ckpt_store_kernel, dim3(R * NSEG), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_flowmap(const FlowmapArgs& a, int R, hipStream_t s) {
    hipLaunchKernelGGL(flowmap_records_kernel, dim3(grid_for(a.P)), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || R == 0) return e;  // R == 0: live particles written by the caller
    hipLaunchKernelGGL(flowmap_live_kernel, dim3(R * NSEG), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace bto
