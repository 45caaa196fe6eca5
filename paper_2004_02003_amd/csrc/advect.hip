// The fused RK4 advection kernel with boundary termination and live-particle
// compaction (the hot kernel of the path).
#include "bto_internal.h"

namespace bto {

// ---------------------------------------------------------------------------
// Fused advection: K RK4 steps per particle, then compaction of survivors.
// ---------------------------------------------------------------------------
template <int DT, int LPP> struct CacheOf { using T = CellCache<DT>; };
template <> struct CacheOf<DT_F32, 2> { using T = PairCache; };

template <int DT, int MODE, int LPP>
__global__ __launch_bounds__(BLOCK) void advect_kernel(const AdvectArgs a) {
    using Cache = typename CacheOf<DT, LPP>::T;
    constexpr int W = BLOCK / WAVE;
    constexpr int PPB = BLOCK / LPP;  // particles per workgroup batch
    const int seg = blockIdx.x % NSEG;
    const int r = blockIdx.x / NSEG;
    const int R = gridDim.x / NSEG;
    const int wave = threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    const uint32_t half = LPP == 2 ? (threadIdx.x & 1u) : 0u;
    const bool owner = half == 0;  // the lane that writes the particle's results
    __shared__ uint32_t s_cnt[W];
    __shared__ uint32_t s_base;
    if (blockIdx.x == 0 && threadIdx.x < NSEG) a.clear_count[threadIdx.x] = 0u;

    const uint32_t cnt = a.in_count[seg];
    const int64_t sbase = a.segs.base[seg];
    uint32_t my_steps = 0;

    // Block-uniform loop over batches of PPB particles of this segment, so
    // the barriers below are reached by every wave the same number of times.
    for (uint32_t bb = (uint32_t)r * PPB; bb < cnt; bb += (uint32_t)R * PPB) {
        const uint32_t i = bb + threadIdx.x / LPP;
        const bool alive = i < cnt;
        double x[3] = {0.0, 0.0, 0.0};
        Cache A, B;
        A.base = B.base = NO_CELL;
        if constexpr (LPP == 2) A.h = B.h = half;
        uint32_t id = 0;
        int status = S_VALID;
        int s = 0;
        if (alive) {
            const PState ps = a.in_pos[sbase + i];
            id = a.in_id[sbase + i];
            unpack(ps, x);
            // two steps per iteration: the slots swap roles, so nothing is copied
            for (s = 0; s < a.K; ++s) {
                status = rk4_step<DT, MODE>(a.g, a.f[s], a.f[s + 1], a.h[s], x, A, B);
                if (status != S_VALID) break;
                A.base = NO_CELL;
                if (MODE != MODE_LINEAR) B.base = NO_CELL;
                if (++s >= a.K) break;
                status = rk4_step<DT, MODE>(a.g, a.f[s], a.f[s + 1], a.h[s], x, B, A);
                if (status != S_VALID) break;
                B.base = NO_CELL;
                if (MODE != MODE_LINEAR) A.base = NO_CELL;
            }
            if (owner) my_steps += (status == S_VALID) ? (uint32_t)a.K : (uint32_t)(s + 1);
        }
        const bool keep = alive && status == S_VALID;
        // survivors: wave ballot, block prefix over the waves, one atomic per block
        const unsigned long long m = __ballot(keep && owner);
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
        if (keep && owner) {
            const uint32_t off = s_base + s_cnt[wave] +
                                 __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            a.out_pos[sbase + off] = pack(x);
            a.out_id[sbase + off] = id;
        }
        if (alive && !keep && owner) {
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
// Launchers.
// ---------------------------------------------------------------------------
template <int DT, int MODE, int LPP>
static hipError_t launch_advect_t(const AdvectArgs& a, int R, hipStream_t s) {
    hipLaunchKernelGGL((advect_kernel<DT, MODE, LPP>), dim3(R * NSEG), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_advect_m(const AdvectArgs& a, int mode, int lpp, int R, hipStream_t s) {
    if constexpr (DT == DT_F32) {
        if (lpp == 2)
            return mode == MODE_LINEAR ? launch_advect_t<DT, MODE_LINEAR, 2>(a, R, s)
                                       : launch_advect_t<DT, MODE_FROZEN, 2>(a, R, s);
    }
    return mode == MODE_LINEAR ? launch_advect_t<DT, MODE_LINEAR, 1>(a, R, s)
                               : launch_advect_t<DT, MODE_FROZEN, 1>(a, R, s);
}

hipError_t launch_advect(const AdvectArgs& a, int dtype, int mode, int lpp, int R, hipStream_t s) {
    switch (dtype) {
    case DT_F32: return launch_advect_m<DT_F32>(a, mode, lpp, R, s);
    case DT_F16: return launch_advect_m<DT_F16>(a, mode, 1, R, s);
    default: return launch_advect_m<DT_BF16>(a, mode, 1, R, s);
    }
}

template <int DT, int MODE, int LPP>
static int occ_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, advect_kernel<DT, MODE, LPP>, BLOCK, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int DT>
static int occ_m(int mode, int lpp) {
    if constexpr (DT == DT_F32) {
        if (lpp == 2) return mode == MODE_LINEAR ? occ_t<DT, MODE_LINEAR, 2>() : occ_t<DT, MODE_FROZEN, 2>();
    }
    return mode == MODE_LINEAR ? occ_t<DT, MODE_LINEAR, 1>() : occ_t<DT, MODE_FROZEN, 1>();
}

int advect_max_blocks_per_cu(int dtype, int mode, int lpp) {
    switch (dtype) {
    case DT_F32: return occ_m<DT_F32>(mode, lpp);
    case DT_F16: return occ_m<DT_F16>(mode, 1);
    default: return occ_m<DT_BF16>(mode, 1);
    }
}

}  // namespace bto
