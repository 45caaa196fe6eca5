// The fused RK4 advection kernel with boundary termination and live-particle
// compaction (the hot kernel of the path).
#include "bto_internal.h"

namespace bto {

// ---------------------------------------------------------------------------
// Fused advection: K RK4 steps per particle, then compaction of survivors.
// ---------------------------------------------------------------------------
template <int DT, int LPP> struct CacheOf { using T = CellCache<DT>; };
template <> struct CacheOf<DT_F32, 2> { using T = PairCache; };

template <int DT, int MODE, int LPP, int REC>
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
    if (blockIdx.x == 0 && threadIdx.x < NSEG) a.clear_count[threadIdx.x * CSTRIDE] = 0u;

    const uint32_t cnt = a.in_count[seg * CSTRIDE];
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
            // a terminated particle's outside point, kept as its offset from x
            const auto on_exit = [&](const double* y) {
                if constexpr (REC)
                    a.rec_out[id] = make_float4((float)(y[0] - x[0]), (float)(y[1] - x[1]), (float)(y[2] - x[2]), 0.f);
            };
            // two steps per iteration: the slots swap roles, so nothing is copied
            for (s = 0; s < a.K; ++s) {
                status = rk4_step<DT, MODE>(a.g, a.f[s], a.f[s + 1], a.h[s], x, A, B, on_exit);
                if (status != S_VALID) break;
                A.base = NO_CELL;
                if (is_frozen<MODE>) B.base = NO_CELL;
                if (++s >= a.K) break;
                status = rk4_step<DT, MODE>(a.g, a.f[s], a.f[s + 1], a.h[s], x, B, A, on_exit);
                if (status != S_VALID) break;
                B.base = NO_CELL;
                if (is_frozen<MODE>) A.base = NO_CELL;
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
            s_base = tot ? atomicAdd(&a.out_count[seg * CSTRIDE], tot) : 0u;
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
            a.rec_meta[id] = (status << META_SHIFT) | (a.step0 + s) | (REC && status == S_TERMINATED ? META_EXITPT : 0);
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
        if (tot) atomicAdd(&a.psteps[seg * PSTRIDE], tot);
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// Every compiled variant: storage type, time mode, lanes per particle (two
// only for FP32), exit-point recording.
template <int DT_, int MODE_, int LPP_, int REC_>
struct Variant {
    static constexpr int DT = DT_, MODE = MODE_, LPP = LPP_, REC = REC_;
};

template <int DT, int LPP, int MODE, class F>
static auto with_rec(int rec, F&& f) {
    return rec ? f(Variant<DT, MODE, LPP, 1>{}) : f(Variant<DT, MODE, LPP, 0>{});
}

template <int DT, int LPP, class F>
static auto with_mode_rec(int mode, int rec, F&& f) {
    if constexpr (LPP == 2) {  // two lanes per particle: the FP32 sampler only
        return (mode & MODE_FROZEN) ? with_rec<DT, LPP, MODE_FROZEN>(rec, f) : with_rec<DT, LPP, MODE_LINEAR>(rec, f);
    } else {
        switch (mode) {
        case MODE_LINEAR: return with_rec<DT, LPP, MODE_LINEAR>(rec, f);
        case MODE_FROZEN: return with_rec<DT, LPP, MODE_FROZEN>(rec, f);
        case MODE_LINEAR | MODE_FP64: return with_rec<DT, LPP, MODE_LINEAR | MODE_FP64>(rec, f);
        default: return with_rec<DT, LPP, MODE_FROZEN | MODE_FP64>(rec, f);
        }
    }
}

template <class F>
static auto with_variant(int dtype, int mode, int lpp, int rec, F&& f) {
    switch (dtype) {
    // two lanes per particle only with the FP32 sampler
    case DT_F32:
        return lpp == 2 && !(mode & MODE_FP64) ? with_mode_rec<DT_F32, 2>(mode, rec, f)
                                               : with_mode_rec<DT_F32, 1>(mode, rec, f);
    case DT_F16: return with_mode_rec<DT_F16, 1>(mode, rec, f);
    default: return with_mode_rec<DT_BF16, 1>(mode, rec, f);
    }
}

hipError_t launch_advect(const AdvectArgs& a, int dtype, int mode, int lpp, int rec, int R, hipStream_t s) {
    return with_variant(dtype, mode, lpp, rec, [&](auto v) {
        using V = decltype(v);
        hipLaunchKernelGGL((advect_kernel<V::DT, V::MODE, V::LPP, V::REC>), dim3(R * NSEG), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    });
}

int advect_max_blocks_per_cu(int dtype, int mode, int lpp, int rec) {
    return with_variant(dtype, mode, lpp, rec, [](auto v) {
        using V = decltype(v);
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, advect_kernel<V::DT, V::MODE, V::LPP, V::REC>, BLOCK,
                                                         0) != hipSuccess)
            return 1;
        return nb > 0 ? nb : 1;
    });
}

}  // namespace bto
