// Tile layout of the live particles: the in situ step in tile order.
//
// Live particles are kept in buckets, one per tile of cells (a particle
// belongs to the tile of its sampling cell); tiles run along a Hilbert curve
// in cell space, one eighth of the curve per XCD, so neighbouring tiles run
// close in time on one XCD and share the grid lines of their common faces in
// its L2.  One step is two launches:
//   tile_gather_kernel  one workgroup per tile: advance every particle of the
//   (tiles = 2)         tile one RK4 step, gathering the grid values, and
//                       write each survivor into the bucket of the tile it
//                       ends in (next step's buffers);
//   tile_stage_kernel   the same with the tile's cells plus a halo of H cells
//   (tiles = 1)         of level n (and n+1) first staged in LDS with
//                       coalesced row loads and sampled from there; a
//                       particle whose stage point needs a cell outside the
//                       staged box is deferred: appended unchanged to this
//                       step's list;
//   tile_list_kernel    advance the list (deferred particles, and those that
//                       did not fit their bucket in the previous step) with
//                       global gathers, into the same next-step buckets.
// All sample with the same arithmetic on the same FP32 corner values, so a
// particle's step does not depend on which kernel took it.
//
// Buffers (context-owned): two bucket arrays (ping-pong) of nbuckets x cap
// slots of state + seed id, bucket b holding the tile that workgroup b runs
// (so a workgroup loads its tile id, particle count and particles at once); a
// ring of three bucket-count arrays (the launch pair of a step reads ring slot
// s, appends to s+1 and clears s+2); the list
// in the context's ping-pong particle buffers with a ring of three counts;
// per-XCD live and particle-step counters as in the segment layout.
#include <type_traits>

#include "bto_internal.h"

namespace bto {

// Tile of a position's sampling cell (the cell locate() picks).
__device__ __forceinline__ uint32_t tile_key(const Geom& g, const TileGeom& tg, const double x[3]) {
    uint32_t t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int v = (int)floor(x[d]);
        v = v > g.n[d] - 2 ? g.n[d] - 2 : v;
        v = v < 0 ? 0 : v;
        t[d] = (uint32_t)v / (uint32_t)tg.T[d];
    }
    return t[0] + (uint32_t)tg.nt[0] * (t[1] + (uint32_t)tg.nt[1] * t[2]);
}

// Write survivors to the bucket of their tile (key: tile id): one returning
// atomic per (wavefront, destination tile) on the bucket's count, lane slots
// from the ballot.  Slots beyond the bucket's capacity go to the next list instead
// (one atomic per wavefront).  Wave-uniform control flow.
__device__ __forceinline__ void scatter_survivors(bool surv, uint32_t key, const PState& st, uint32_t id,
                                                  const TileOut& o) {
    const int lane = threadIdx.x % WAVE;
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long pending = __ballot(surv);
    uint32_t slot = 0;
    uint32_t bkt = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t lk = __shfl(key, leader);
        const bool mine = surv && key == lk;
        const unsigned long long same = __ballot(mine) & pending;
        uint32_t base = 0, lb = 0;
        if (lane == leader) {
            lb = (uint32_t)o.slot_of[lk];
            base = atomicAdd(&o.tc[lb], (uint32_t)__popcll(same));
        }
        base = __shfl(base, leader);
        lb = __shfl(lb, leader);
        if (mine) {
            slot = base + (uint32_t)__popcll(same & below);
            bkt = lb;
        }
        pending &= ~same;
    }
    const bool over = surv && slot >= o.cap;
    if (surv && !over) {
        const size_t q = (size_t)bkt * o.cap + slot;
        o.bpos[q] = st;
        o.bid[q] = id;
    }
    const unsigned long long om = __ballot(over);
    if (om) {
        const int leader = __ffsll((long long)om) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(o.list_count, (uint32_t)__popcll(om));
        base = __shfl(base, leader);
        if (over) {
            const uint32_t k = base + (uint32_t)__popcll(om & below);
            o.list_pos[k] = st;
            o.list_id[k] = id;
        }
    }
}

// Append particles to a list, one atomic per wavefront (wave-uniform).
__device__ __forceinline__ void append_list(bool on, const PState& st, uint32_t id, PState* pos, uint32_t* ids,
                                            uint32_t* count) {
    const int lane = threadIdx.x % WAVE;
    const unsigned long long m = __ballot(on);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (on) {
        const uint32_t k = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        pos[k] = st;
        ids[k] = id;
    }
}

// Workgroup totals of particle-steps and survivors into the XCD's counters
// (NT threads per workgroup).
template <int NT>
__device__ __forceinline__ void add_totals(uint32_t steps, uint32_t surv, unsigned long long* psteps,
                                           uint32_t* live, uint32_t* s_red, int W = NT / WAVE) {
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        steps += __shfl_xor(steps, o);
        surv += __shfl_xor(surv, o);
    }
    __syncthreads();
    if (lane == 0) {
        s_red[wave] = steps;
        s_red[NT / WAVE + wave] = surv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ts = 0;
        uint32_t tl = 0;
        for (int w = 0; w < W; ++w) {
            ts += s_red[w];
            tl += s_red[NT / WAVE + w];
        }
        const int xcd = blockIdx.x % NSEG;
        if (ts) atomicAdd(&psteps[xcd * PSTRIDE], ts);
        if (tl) atomicAdd(&live[xcd * CSTRIDE], tl);
    }
}

__device__ __forceinline__ void end_record(const TileStepArgs& a, int status, uint32_t id, const double x[3], int rec) {
    a.rec_pos[id] = pack(x);
    a.rec_meta[id] = (status << META_SHIFT) | a.step0 | (rec && status == S_TERMINATED ? META_EXITPT : 0);
}

__device__ __forceinline__ void tile_coords(const Geom& g, const TileGeom& tg, const double x[3], int t[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int v = (int)floor(x[d]);
        v = v > g.n[d] - 2 ? g.n[d] - 2 : v;
        v = v < 0 ? 0 : v;
        t[d] = v / tg.T[d];
    }
}

// Bucket of each neighbour of tile ts (direction (dx, dy, dz) in -1..1 at
// index (dz + 1) * 9 + (dy + 1) * 3 + dx + 1; -1 outside the block), loaded
// by the first 27 threads at the start of a workgroup and kept in a register
// until the scatter (so the load overlaps the step instead of stalling the
// first barrier).
__device__ __forceinline__ int32_t neighbour_bucket(const TileGeom& tg, const TileOut& o, const int ts[3]) {
    int32_t b = -1;
    if (threadIdx.x < 27) {
        const int d = (int)threadIdx.x;
        const int q[3] = {ts[0] + d % 3 - 1, ts[1] + (d / 3) % 3 - 1, ts[2] + d / 9 - 1};
        if (q[0] >= 0 && q[0] < tg.nt[0] && q[1] >= 0 && q[1] < tg.nt[1] && q[2] >= 0 && q[2] < tg.nt[2])
            b = o.slot_of[q[0] + tg.nt[0] * (q[1] + tg.nt[1] * q[2])];
    }
    return b;
}

// Survivors of one workgroup batch into the buckets of the next step.  A
// survivor ends in its own tile or a neighbour (direction dx, dy, dz in
// -1..1) unless it jumped further: ranks per direction from LDS atomics, then
// one global atomic per (batch, destination tile) reserves the slots.
// Survivors that jumped further take one global atomic each; slots beyond the
// bucket's capacity go to the next list.  Block-uniform (barriers inside);
// nb: the neighbour bucket of direction threadIdx.x (threads 0..26, from
// neighbour_bucket), stored to s_nb before the first barrier.
__device__ __forceinline__ void scatter_block(bool surv, const int ts[3], const int td[3], const PState& st,
                                              uint32_t id, const TileGeom& tg, const TileOut& o, uint32_t* s_hist,
                                              uint32_t* s_base, int32_t* s_nb, int32_t nb) {
    int dir = 27;
    if (surv) {
        const int dx = td[0] - ts[0], dy = td[1] - ts[1], dz = td[2] - ts[2];
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) dir = (dz + 1) * 9 + (dy + 1) * 3 + dx + 1;
    }
    if (threadIdx.x < 27) {
        s_hist[threadIdx.x] = 0u;
        s_nb[threadIdx.x] = nb;
    }
    __syncthreads();
    uint32_t rank = 0;
    if (surv && dir < 27) rank = atomicAdd(&s_hist[dir], 1u);
    __syncthreads();
    if (threadIdx.x < 27) {
        const uint32_t c = s_hist[threadIdx.x];
        s_base[threadIdx.x] = c ? atomicAdd(&o.tc[s_nb[threadIdx.x]], c) : 0u;
    }
    __syncthreads();
    bool over = false;
    if (surv) {
        uint32_t bkt, slot;
        if (dir < 27) {
            bkt = (uint32_t)s_nb[dir];
            slot = s_base[dir] + rank;
        } else {
            bkt = (uint32_t)o.slot_of[td[0] + tg.nt[0] * (td[1] + tg.nt[1] * td[2])];
            slot = atomicAdd(&o.tc[bkt], 1u);
        }
        over = slot >= o.cap;
        if (!over) {
            const size_t q = (size_t)bkt * o.cap + slot;
            o.bpos[q] = st;
            o.bid[q] = id;
        }
    }
    append_list(over, st, id, o.list_pos, o.list_id, o.list_count);
}

// ---------------------------------------------------------------------------
// The staging box of tile t: the tile's cells plus a halo of H cells, clipped
// to the block (lo: first point per axis, ext: points per axis, <= S).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_box(const Geom& g, const TileGeom& tg, int t, int tc[3], int lo[3], int ext[3]) {
    tc[0] = t % tg.nt[0];
    tc[1] = (t / tg.nt[0]) % tg.nt[1];
    tc[2] = t / (tg.nt[0] * tg.nt[1]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int l = tc[d] * tg.T[d] - tg.H;
        const int h = tc[d] * tg.T[d] + tg.T[d] + tg.H;
        lo[d] = l < 0 ? 0 : l;
        const int hi = h > g.n[d] - 1 ? g.n[d] - 1 : h;
        ext[d] = hi - lo[d] + 1;
    }
}

// Grid values of one staging box held in registers between their loads and
// their stores to LDS: every load of the box is issued at once (one round
// trip), one point per thread per pass, rows of the box contiguous in x.
template <int DT, int MODE, int S>
struct StageRegs {
    static constexpr int NPT = S * S * S;
    static constexpr int KP = (NPT + BLOCK - 1) / BLOCK;
    static constexpr int NL = is_frozen<MODE> ? 1 : 2;
    static constexpr int EB = DT == DT_F32 ? 16 : 8;  // LDS bytes per staged point
    static constexpr uint32_t PLANE = (uint32_t)NPT * EB;
    using Pt = typename std::conditional<DT == DT_F32, Pt32, Pt16>::type;
    Pt v[NL][KP];
    uint32_t ok;

    __device__ __forceinline__ void load(const Geom& g, const char* V0, const char* V1, const int lo[3],
                                         const int ext[3]) {
        ok = 0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int p = threadIdx.x + k * BLOCK;
            const int lx = p % S, ly = (p / S) % S, lz = p / (S * S);
            if (p < NPT && lx < ext[0] && ly < ext[1] && lz < ext[2]) {
                ok |= 1u << k;
                const uint64_t gp = (uint64_t)(lo[0] + lx) + (uint64_t)g.sy * (uint32_t)(lo[1] + ly) +
                                    (uint64_t)g.sz * (uint32_t)(lo[2] + lz);
                v[0][k] = *reinterpret_cast<const Pt*>(V0 + gp * sizeof(Pt));
                if constexpr (NL == 2) v[NL - 1][k] = *reinterpret_cast<const Pt*>(V1 + gp * sizeof(Pt));
            }
        }
    }

    __device__ __forceinline__ void store(char* lds) const {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            if (ok & (1u << k)) {
                const int p = threadIdx.x + k * BLOCK;
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    if constexpr (DT == DT_F32) {
                        *reinterpret_cast<float4*>(lds + l * PLANE + (size_t)p * EB) =
                            make_float4(v[l][k].v[0], v[l][k].v[1], v[l][k].v[2], 0.f);
                    } else {
                        *reinterpret_cast<uint2*>(lds + l * PLANE + (size_t)p * EB) =
                            make_uint2(v[l][k].xy, (uint32_t)v[l][k].z);
                    }
                }
            }
        }
    }
};

// One RK4 step of up to one batch of a tile's particles and the move of the
// survivors to their next buckets (block-uniform).
template <int DT, int MODE, int REC, class CA>
__device__ __forceinline__ void tile_batch(const TileStepArgs& a, bool alive, const PState& st, uint32_t id,
                                           const int tc[3], const char* V0, const char* V1, CA& A, CA& B,
                                           uint32_t& my_steps, uint32_t& my_surv, uint32_t* s_hist,
                                           uint32_t* s_base, int32_t* s_nb, int32_t nb) {
    double x[3] = {0.0, 0.0, 0.0};
    int status = S_DEFER;
    if (alive) {
        unpack(st, x);
        const auto on_exit = [&](const double* y) {
            if constexpr (REC)
                a.rec_out[id] = make_float4((float)(y[0] - x[0]), (float)(y[1] - x[1]), (float)(y[2] - x[2]), 0.f);
        };
        A.base = B.base = NO_CELL;
        status = rk4_step<DT, MODE>(a.g, V0, V1, a.h, x, A, B, on_exit);
        if (status != S_DEFER) ++my_steps;
        if (status == S_TERMINATED || status == S_INVALID) end_record(a, status, id, x, REC);
    }
    const bool surv = alive && status == S_VALID;
    const bool defer = alive && status == S_DEFER;
    my_surv += surv ? 1u : 0u;
    int td[3] = {0, 0, 0};
    if (surv) tile_coords(a.g, a.tg, x, td);
    scatter_block(surv, tc, td, surv ? pack(x) : st, id, a.tg, a.out, s_hist, s_base, s_nb, nb);
    append_list(defer, st, id, a.list_pos, a.list_id, a.list_count);
}

// Lanes of one batch reordered by the (z, y) row of their cell inside the
// tile (counting sort in LDS), so that the lanes of a wavefront share grid
// rows: each row load of the sampler then touches a few cache lines per
// wavefront instead of one per lane.  Block-uniform.
constexpr int SORT_ROWS_MAX = 16 * 16;  // rows of the largest tile (y, z sides <= 16)
template <int NT>
struct SortLds {
    uint32_t off[SORT_ROWS_MAX + 64];
    PState pos[NT];
    uint32_t id[NT];
};

template <int NT>
__device__ __forceinline__ void sort_rows(const TileGeom& tg, const int tc[3], bool on, PState& st, uint32_t& id,
                                          SortLds<NT>& s, int nthr = NT) {
    const int Ty = tg.T[1], Tz = tg.T[2];
    const int nrow = Ty * Tz;  // bin nrow: lanes without a particle, last
    uint32_t key = (uint32_t)nrow;
    if (on) {
        int ly = (int)((st.cell >> 10) & 1023u) - tc[1] * Ty;
        int lz = (int)(st.cell >> 20) - tc[2] * Tz;
        ly = ly < 0 ? 0 : (ly > Ty - 1 ? Ty - 1 : ly);
        lz = lz < 0 ? 0 : (lz > Tz - 1 ? Tz - 1 : lz);
        key = (uint32_t)(lz * Ty + ly);
    }
    for (int i = threadIdx.x; i <= nrow; i += nthr) s.off[i] = 0u;
    __syncthreads();
    const uint32_t rank = atomicAdd(&s.off[key], 1u);
    __syncthreads();
    if (threadIdx.x < WAVE) {
        // exclusive scan of the nrow + 1 bin counts by one wavefront
        constexpr int PER = (SORT_ROWS_MAX + WAVE) / WAVE;
        uint32_t v[PER], sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = threadIdx.x * PER + k;
            v[k] = i <= nrow ? s.off[i] : 0u;
            sum += v[k];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o);
            if ((int)threadIdx.x >= o) incl += u;
        }
        uint32_t run = incl - sum;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = threadIdx.x * PER + k;
            if (i <= nrow) s.off[i] = run;
            run += v[k];
        }
    }
    __syncthreads();
    const uint32_t dst = s.off[key] + rank;
    s.pos[dst] = st;
    s.id[dst] = id;
    __syncthreads();
    st = s.pos[threadIdx.x];
    id = s.id[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Gathering tile step: one workgroup of NT threads per tile, the particles
// gather from the grids (through L2, which the tile order keeps warm).
// ---------------------------------------------------------------------------
template <int DT, int MODE, int REC, int NT>
__global__ __launch_bounds__(NT) void tile_gather_kernel(const TileStepArgs a) {
    __shared__ uint32_t s_red[2 * (NT / WAVE)];
    __shared__ uint32_t s_hist[32], s_base[32];
    __shared__ int32_t s_nb[32];
    __shared__ SortLds<NT> s_sort;
    if (blockIdx.x == 0 && threadIdx.x < NSEG) a.live_clear[threadIdx.x * CSTRIDE] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == NSEG) *a.list_clear = 0u;
    // bucket b = this workgroup: its tile, count and first particles load at once
    const uint32_t b = blockIdx.x;
    const int32_t t = a.order[b];
    uint32_t cnt = a.tc_in[b];
    const size_t bin = (size_t)b * a.out.cap;
    PState st0{};
    uint32_t id0 = 0;
    if (threadIdx.x < a.out.cap) {  // in the bucket even when beyond its count
        st0 = a.in_pos[bin + threadIdx.x];
        id0 = a.in_id[bin + threadIdx.x];
    }
    if (t < 0) return;
    if (threadIdx.x == 0) a.tc_clear[b] = 0u;
    cnt = cnt < a.out.cap ? cnt : a.out.cap;
    if (cnt == 0) return;
    // A tile with fewer particles than threads: the wavefronts past its count
    // end here, so they hold no wave slot while the tile runs (s_barrier then
    // waits for the surviving wavefronts only).  The wave index is taken from
    // the first lane so that the branch is scalar: the whole wavefront ends.
    int nw = NT / WAVE;
    if (cnt < (uint32_t)NT) {
        nw = (int)((cnt + WAVE - 1) / WAVE);
        if (__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)) >= nw) return;
    }
    int tc[3], lo[3], ext[3];
    tile_box(a.g, a.tg, t, tc, lo, ext);
    const int32_t nb = neighbour_bucket(a.tg, a.out, tc);
    if (cnt <= NT) sort_rows<NT>(a.tg, tc, threadIdx.x < cnt, st0, id0, s_sort, nw * WAVE);
    const char* V0 = in_global(a.f0);
    const char* V1 = in_global(a.f1);
    uint32_t my_steps = 0, my_surv = 0;
    for (uint32_t bb = 0; bb < cnt; bb += NT) {
        const uint32_t i = bb + threadIdx.x;
        const bool alive = i < cnt;
        PState st = st0;
        uint32_t id = id0;
        if (bb && alive) {
            st = a.in_pos[bin + i];
            id = a.in_id[bin + i];
        }
        CellCache<DT> A, B;
        tile_batch<DT, MODE, REC>(a, alive, st, id, tc, V0, V1, A, B, my_steps, my_surv, s_hist, s_base, s_nb, nb);
    }
    add_totals<NT>(my_steps, my_surv, a.psteps, a.live_out, s_red, nw);
}

// ---------------------------------------------------------------------------
// Staged tile step: one workgroup per tile stages the tile's cells plus a halo
// of H cells of both levels in LDS (every load of the box issued at once),
// then advances the tile's particles sampling from LDS.  Particles whose stage
// points need cells beyond the staged box are deferred to the list.
// ---------------------------------------------------------------------------
template <int DT, int MODE, int REC, int S>
__global__ __launch_bounds__(BLOCK) void tile_stage_kernel(const TileStepArgs a) {
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t s_red[2 * (BLOCK / WAVE)];
    __shared__ uint32_t s_hist[32], s_base[32];
    __shared__ int32_t s_nb[32];
    using SR = StageRegs<DT, MODE, S>;
    if (blockIdx.x == 0 && threadIdx.x < NSEG) a.live_clear[threadIdx.x * CSTRIDE] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == NSEG) *a.list_clear = 0u;
    const uint32_t b = blockIdx.x;
    const int32_t t = a.order[b];
    uint32_t cnt = a.tc_in[b];
    const size_t bin = (size_t)b * a.out.cap;
    PState st0{};
    uint32_t id0 = 0;
    if (threadIdx.x < a.out.cap) {  // in the bucket even when beyond its count
        st0 = a.in_pos[bin + threadIdx.x];
        id0 = a.in_id[bin + threadIdx.x];
    }
    if (t < 0) return;
    if (threadIdx.x == 0) a.tc_clear[b] = 0u;
    cnt = cnt < a.out.cap ? cnt : a.out.cap;
    if (cnt == 0) return;
    int tc[3], lo[3], ext[3];
    tile_box(a.g, a.tg, t, tc, lo, ext);
    const int32_t nb = neighbour_bucket(a.tg, a.out, tc);
    {
        SR sr;
        sr.load(a.g, in_global(a.f0), in_global(a.f1), lo, ext);
        sr.store(lds);
    }
    __syncthreads();
    LdsCache<DT> A, B;
    A.plane = lds;
    B.plane = lds + (is_frozen<MODE> ? 0u : SR::PLANE);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A.lo[d] = B.lo[d] = lo[d];
        A.lim[d] = B.lim[d] = ext[d] - 2;
    }
    A.S = B.S = S;
    uint32_t my_steps = 0, my_surv = 0;
    for (uint32_t bb = 0; bb < cnt; bb += BLOCK) {
        const uint32_t i = bb + threadIdx.x;
        const bool alive = i < cnt;
        PState st = st0;
        uint32_t id = id0;
        if (bb && alive) {
            st = a.in_pos[bin + i];
            id = a.in_id[bin + i];
        }
        tile_batch<DT, MODE, REC>(a, alive, st, id, tc, nullptr, nullptr, A, B, my_steps, my_surv, s_hist, s_base,
                                  s_nb, nb);
    }
    add_totals<BLOCK>(my_steps, my_surv, a.psteps, a.live_out, s_red);
}

// ---------------------------------------------------------------------------
// The list: deferred particles of this step and bucket overflows of the last
// one, advanced with global gathers into the next step's buckets.
// ---------------------------------------------------------------------------
template <int DT, int MODE, int REC>
__global__ __launch_bounds__(BLOCK) void tile_list_kernel(const TileListArgs a) {
    __shared__ uint32_t s_red[2 * (BLOCK / WAVE)];
    const uint32_t n = *a.in_count;
    uint32_t my_steps = 0, my_surv = 0;
    const char* V0 = in_global(a.s.f0);
    const char* V1 = in_global(a.s.f1);
    // wave-uniform loop over the list
    const uint32_t wave_g = (blockIdx.x * BLOCK + threadIdx.x) / WAVE;
    const uint32_t nwaves = gridDim.x * (BLOCK / WAVE);
    for (uint32_t w0 = wave_g * WAVE; w0 < n; w0 += nwaves * WAVE) {
        const uint32_t i = w0 + threadIdx.x % WAVE;
        const bool alive = i < n;
        double x[3] = {0.0, 0.0, 0.0};
        uint32_t id = 0;
        int status = S_INVALID;
        if (alive) {
            const PState st = a.in_pos[i];
            id = a.in_id[i];
            unpack(st, x);
            CellCache<DT> A, B;
            A.base = B.base = NO_CELL;
            const auto on_exit = [&](const double* y) {
                if constexpr (REC)
                    a.s.rec_out[id] = make_float4((float)(y[0] - x[0]), (float)(y[1] - x[1]), (float)(y[2] - x[2]), 0.f);
            };
            status = rk4_step<DT, MODE>(a.s.g, V0, V1, a.s.h, x, A, B, on_exit);
            ++my_steps;
            if (status != S_VALID) end_record(a.s, status, id, x, REC);
        }
        const bool surv = alive && status == S_VALID;
        my_surv += surv ? 1u : 0u;
        const uint32_t key = surv ? tile_key(a.s.g, a.s.tg, x) : 0u;
        scatter_survivors(surv, key, pack(x), id, a.s.out);
    }
    add_totals<BLOCK>(my_steps, my_surv, a.s.psteps, a.s.live_out, s_red);
}

// ---------------------------------------------------------------------------
// Segment layout -> buckets (once per interval, before the first tile step):
// every live particle of the segments into the bucket of its tile, overflow
// into the list of the coming step.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void tile_bin_kernel(const TileBinArgs a) {
    const int seg = blockIdx.x % NSEG;
    const int r = blockIdx.x / NSEG;
    const int R = gridDim.x / NSEG;
    const uint32_t cnt = a.count[seg * CSTRIDE];
    const int64_t sbase = a.segs.base[seg];
    for (uint32_t b0 = (uint32_t)r * BLOCK; b0 < cnt; b0 += (uint32_t)R * BLOCK) {
        const uint32_t i = b0 + threadIdx.x;
        const bool alive = i < cnt;
        PState st{};
        uint32_t id = 0, key = 0;
        if (alive) {
            st = a.pos[sbase + i];
            id = a.id[sbase + i];
            double x[3];
            unpack(st, x);
            key = tile_key(a.g, a.tg, x);
        }
        scatter_survivors(alive, key, st, id, a.out);
    }
}

// Zero n words (tile and list counts before the first tile step).
__global__ void tile_fill_kernel(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// Live particles of the tile layout (buckets and the pending list), by seed
// id: end position for the flow map (flowmap args) or FP64 position for a
// checkpoint (out != null).
__global__ __launch_bounds__(BLOCK) void tile_live_kernel(const TileLiveArgs a) {
    const uint64_t total = (uint64_t)a.ntiles * a.cap;
    for (uint64_t q = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; q < total + a.list_n_max;
         q += (uint64_t)gridDim.x * BLOCK) {
        PState st;
        uint32_t id;
        if (q < total) {
            const uint32_t t = (uint32_t)(q / a.cap), k = (uint32_t)(q % a.cap);  // bucket, slot
            const uint32_t c = a.tc[t];
            if (k >= c || k >= a.cap) continue;
            st = a.bpos[q];
            id = a.bid[q];
        } else {
            const uint64_t k = q - total;
            if (k >= *a.list_count) continue;
            st = a.list_pos[k];
            id = a.list_id[k];
        }
        double x[3];
        unpack(st, x);
        if (a.ckpt) {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.ckpt[3 * (size_t)id + d] = x[d];
        } else {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.out_end[3 * (size_t)id + d] = a.origin[d] + a.spacing[d] * x[d];
            a.out_flag[id] = (uint8_t)S_VALID;
            a.out_exit[id] = a.steps_done;
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <int DT, int MODE, int REC>
static hipError_t launch_tile_step_t(const TileStepArgs& a, int stage, hipStream_t s) {
    constexpr int S = DT == DT_F32 ? TILE_S_F32 : TILE_S_16;
    using SR = StageRegs<DT, MODE, S>;
    constexpr size_t lds = (size_t)SR::NL * SR::PLANE;
    if (!stage) {
        hipLaunchKernelGGL((tile_gather_kernel<DT, MODE, REC, GATHER_NT>), dim3(a.order_len), dim3(GATHER_NT), 0, s, a);
        return hipGetLastError();
    }
    // LDS beyond the default limit: raise the kernel's dynamic-LDS limit (on
    // the current device) before the launch
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_stage_kernel<DT, MODE, REC, S>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        (void)hipGetLastError();
    hipLaunchKernelGGL((tile_stage_kernel<DT, MODE, REC, S>), dim3(a.order_len), dim3(BLOCK), lds, s, a);
    return hipGetLastError();
}

template <int DT, int MODE, int REC>
static hipError_t launch_tile_list_t(const TileListArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((tile_list_kernel<DT, MODE, REC>), dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <class F>
static hipError_t tile_dispatch(int dtype, int mode, int rec, F&& f) {
    auto by_rec = [&](auto dt, auto md) {
        return rec ? f(dt, md, std::integral_constant<int, 1>{}) : f(dt, md, std::integral_constant<int, 0>{});
    };
    auto by_mode = [&](auto dt) {
        switch (mode) {
        case MODE_LINEAR: return by_rec(dt, std::integral_constant<int, MODE_LINEAR>{});
        case MODE_FROZEN: return by_rec(dt, std::integral_constant<int, MODE_FROZEN>{});
        case MODE_LINEAR | MODE_FP64: return by_rec(dt, std::integral_constant<int, MODE_LINEAR | MODE_FP64>{});
        default: return by_rec(dt, std::integral_constant<int, MODE_FROZEN | MODE_FP64>{});
        }
    };
    switch (dtype) {
    case DT_F32: return by_mode(std::integral_constant<int, DT_F32>{});
    case DT_F16: return by_mode(std::integral_constant<int, DT_F16>{});
    default: return by_mode(std::integral_constant<int, DT_BF16>{});
    }
}

hipError_t launch_tile_step(const TileStepArgs& a, int dtype, int mode, int rec, int stage, hipStream_t s) {
    return tile_dispatch(dtype, mode, rec, [&](auto dt, auto md, auto rc) {
        return launch_tile_step_t<decltype(dt)::value, decltype(md)::value, decltype(rc)::value>(a, stage, s);
    });
}

hipError_t launch_tile_list(const TileListArgs& a, int dtype, int mode, int rec, int grid, hipStream_t s) {
    return tile_dispatch(dtype, mode, rec, [&](auto dt, auto md, auto rc) {
        return launch_tile_list_t<decltype(dt)::value, decltype(md)::value, decltype(rc)::value>(a, grid, s);
    });
}

hipError_t launch_tile_bin(const TileBinArgs& a, int R, hipStream_t s) {
    hipLaunchKernelGGL(tile_bin_kernel, dim3(R * NSEG), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tile_fill(uint32_t* p, size_t n, hipStream_t s) {
    size_t g = (n + BLOCK - 1) / BLOCK;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(tile_fill_kernel, dim3((unsigned)g), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_tile_live(const TileLiveArgs& a, hipStream_t s) {
    const uint64_t total = (uint64_t)a.ntiles * a.cap + a.list_n_max;
    uint64_t g = (total + BLOCK - 1) / BLOCK;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(tile_live_kernel, dim3((unsigned)g), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace bto
