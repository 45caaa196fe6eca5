// Kernels of the per-block BTO path: seeding, the fused RK4 advection with
// boundary termination and live-particle compaction, and the flow-map writer.
#include "bto_internal.h"

namespace bto {

// ---------------------------------------------------------------------------
// Seeding.
// ---------------------------------------------------------------------------

// Lattice points are stored brick-major: bricks of 4x4x4 lattice points (one
// wavefront) in x-fastest brick order, x-fastest inside a brick, so that a
// wavefront's particles share cache lines of the field.  Bricks on the high
// faces may be partial; slot(id) is the closed-form prefix count.
__device__ __forceinline__ int64_t brick_slot(const int32_t m[3], int a, int b, int c) {
    const int bx = a >> 2, by = b >> 2, bz = c >> 2;
    const int lx = a & 3, ly = b & 3, lz = c & 3;
    const int cx = min(4, m[0] - 4 * bx), cy = min(4, m[1] - 4 * by), cz = min(4, m[2] - 4 * bz);
    return (int64_t)m[0] * m[1] * 4 * bz + (int64_t)m[0] * 4 * by * cz + (int64_t)4 * bx * cy * cz +
           lx + cx * (ly + cy * lz);
}

__global__ __launch_bounds__(BLOCK) void seed_lattice_kernel(const SeedLatticeArgs a) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < a.P; t += (int64_t)gridDim.x * BLOCK) {
        const int ia = (int)(t % a.m[0]);
        const int ib = (int)((t / a.m[0]) % a.m[1]);
        const int ic = (int)(t / ((int64_t)a.m[0] * a.m[1]));
        const double x[3] = {a.off[0] + (double)a.stride * ia, a.off[1] + (double)a.stride * ib,
                             a.off[2] + (double)a.stride * ic};
        const int64_t slot = brick_slot(a.m, ia, ib, ic);
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
        if (inside(a.g, x)) {
            const uint32_t k = atomicAdd(&a.count[seg], 1u);
            a.pos[a.segs.base[seg] + k] = pack(x);
            a.id[a.segs.base[seg] + k] = (uint32_t)t;
            a.rec_meta[t] = META_LIVE;
        } else {
            // outside the block from the start: terminated at step 0, end = seed
            PState s;
            s.cell = 0;
            s.f[0] = s.f[1] = s.f[2] = 0.f;
            a.rec_pos[t] = s;  // position taken from seed_xyz by the writer
            a.rec_meta[t] = (S_TERMINATED << META_SHIFT) | 0 | (1 << 27);
        }
    }
}

struct CountValues {
    uint32_t v[3 * NSEG];
};

__global__ void set_counts_kernel(uint32_t* counts, const CountValues vals, int n, unsigned long long* psteps) {
    const int t = threadIdx.x;
    if (t < n) counts[t] = vals.v[t];
    if (t < NSEG && psteps) psteps[t] = 0ull;
}

// ---------------------------------------------------------------------------
// Fused advection: K RK4 steps per particle, then compaction of survivors.
// ---------------------------------------------------------------------------
template <int DT, int MODE>
__global__ __launch_bounds__(BLOCK) void advect_kernel(const AdvectArgs a) {
    constexpr int W = BLOCK / WAVE;
    const int seg = blockIdx.x % NSEG;
    const int r = blockIdx.x / NSEG;
    const int R = gridDim.x / NSEG;
    const int wave = threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    __shared__ uint32_t s_cnt[W];
    __shared__ uint32_t s_base;
    if (blockIdx.x == 0 && threadIdx.x < NSEG) a.clear_count[threadIdx.x] = 0u;

    const uint32_t cnt = a.in_count[seg];
    const int64_t sbase = a.segs.base[seg];
    uint32_t my_steps = 0;

    // Block-uniform loop over batches of BLOCK particles of this segment, so
    // the barriers below are reached by every wave the same number of times.
    for (uint32_t bb = (uint32_t)r * BLOCK; bb < cnt; bb += (uint32_t)R * BLOCK) {
        const uint32_t i = bb + threadIdx.x;
        const bool alive = i < cnt;
        Stepper<DT> stp;
        stp.x[0] = stp.x[1] = stp.x[2] = 0.0;
        uint32_t id = 0;
        int status = S_VALID;
        int s = 0;
        if (alive) {
            const PState ps = a.in_pos[sbase + i];
            id = a.in_id[sbase + i];
            unpack(ps, stp.x);
            stepper_init(stp);
            // two steps per iteration: the slots swap roles, so nothing is copied
            for (s = 0; s < a.K; ++s) {
                status = rk4_step<DT, MODE>(a.g, a.f[s], a.f[s + 1], a.h[s], stp.x, stp.A, stp.B);
                if (status != S_VALID) break;
                stp.A.base = NO_CELL;
                if (MODE != MODE_LINEAR) stp.B.base = NO_CELL;
                if (++s >= a.K) break;
                status = rk4_step<DT, MODE>(a.g, a.f[s], a.f[s + 1], a.h[s], stp.x, stp.B, stp.A);
                if (status != S_VALID) break;
                stp.B.base = NO_CELL;
                if (MODE != MODE_LINEAR) stp.A.base = NO_CELL;
            }
            my_steps += (status == S_VALID) ? (uint32_t)a.K : (uint32_t)(s + 1);
        }
        const double* x = stp.x;
        const bool keep = alive && status == S_VALID;
        // survivors: wave ballot, block prefix over the waves, one atomic per block
        const unsigned long long m = __ballot(keep);
        if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t c = s_cnt[w];
                s_cnt[w] = tot;
                tot += c;
            }
            s_base = tot ? atomicAdd(&a.out_count[seg], tot) : 0u;
        }
        __syncthreads();
        if (keep) {
            const uint32_t off = s_base + s_cnt[wave] +
                                 __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            a.out_pos[sbase + off] = pack(x);
            a.out_id[sbase + off] = id;
        }
        if (alive && !keep) {
            a.rec_pos[id] = pack(x);
            a.rec_meta[id] = (status << META_SHIFT) | (a.step0 + s);
        }
        __syncthreads();  // s_cnt / s_base are reused by the next batch
    }
    // block total of attempted particle-steps, one atomic per block into the segment's counter
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) my_steps += __shfl_xor(my_steps, o);
    if (lane == 0) s_cnt[wave] = my_steps;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) tot += s_cnt[w];
        if (tot) atomicAdd(&a.psteps[seg], tot);
    }
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
        if (meta & (1 << 27)) {  // seeded outside the block
#pragma unroll
            for (int d = 0; d < 3; ++d) a.out_end[3 * t + d] = a.seed_xyz[3 * t + d];
        } else {
            write_world(a, t, a.rec_pos[t]);
        }
        a.out_flag[t] = (uint8_t)(meta >> META_SHIFT);
        a.out_exit[t] = meta & ((1 << 27) - 1);
    }
}

// Particles still advancing: valid, exit step = steps done.
__global__ __launch_bounds__(BLOCK) void flowmap_live_kernel(const FlowmapArgs a) {
    const int seg = blockIdx.x % NSEG;
    const int r = blockIdx.x / NSEG;
    const int R = gridDim.x / NSEG;
    const uint32_t cnt = a.count[seg];
    const int64_t sbase = a.segs.base[seg];
    for (uint32_t i = (uint32_t)r * BLOCK + threadIdx.x; i < cnt; i += (uint32_t)R * BLOCK) {
        const uint32_t id = a.id[sbase + i];
        write_world(a, id, a.pos[sbase + i]);
        a.out_flag[id] = (uint8_t)S_VALID;
        a.out_exit[id] = a.steps_done;
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

template <int DT, int MODE>
static hipError_t launch_advect_t(const AdvectArgs& a, int R, hipStream_t s) {
    hipLaunchKernelGGL((advect_kernel<DT, MODE>), dim3(R * NSEG), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_advect_m(const AdvectArgs& a, int mode, int R, hipStream_t s) {
    return mode == MODE_LINEAR ? launch_advect_t<DT, MODE_LINEAR>(a, R, s) : launch_advect_t<DT, MODE_FROZEN>(a, R, s);
}

hipError_t launch_advect(const AdvectArgs& a, int dtype, int mode, int R, hipStream_t s) {
    switch (dtype) {
    case DT_F32: return launch_advect_m<DT_F32>(a, mode, R, s);
    case DT_F16: return launch_advect_m<DT_F16>(a, mode, R, s);
    default: return launch_advect_m<DT_BF16>(a, mode, R, s);
    }
}

template <int DT, int MODE>
static int occ_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, advect_kernel<DT, MODE>, BLOCK, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

template <int DT>
static int occ_m(int mode) {
    return mode == MODE_LINEAR ? occ_t<DT, MODE_LINEAR>() : occ_t<DT, MODE_FROZEN>();
}

int advect_max_blocks_per_cu(int dtype, int mode) {
    switch (dtype) {
    case DT_F32: return occ_m<DT_F32>(mode);
    case DT_F16: return occ_m<DT_F16>(mode);
    default: return occ_m<DT_BF16>(mode);
    }
}

hipError_t launch_flowmap(const FlowmapArgs& a, int R, hipStream_t s) {
    hipLaunchKernelGGL(flowmap_records_kernel, dim3(grid_for(a.P)), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(flowmap_live_kernel, dim3(R * NSEG), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace bto
