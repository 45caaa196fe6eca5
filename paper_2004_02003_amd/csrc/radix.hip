// Device-wide exclusive scan of 32-bit counts and a stable LSD radix sort of
// (64-bit key, 32-bit value) pairs, for the two reorderings of the path: the
// grid-gradient records (sorted by colour | level | cell, equal keys kept in
// slot order) and the rebin's bin offsets.
//
// Scan: each workgroup scans a chunk of 4,096 counts and writes the chunk's
// total; one workgroup scans the totals; each chunk then adds its offset.
//
// Sort, per 8-bit digit from the lowest: a histogram of the digit per tile of
// 4,096 pairs (digit-major: count[digit][tile]), its exclusive scan (the first
// output slot of every (digit, tile)), and a scatter.  In the scatter
// wavefront w of a tile takes the tile's pairs [1024 w, 1024 w + 1024) in 16
// rounds of 64 consecutive pairs; lanes with equal digits find each other with
// one ballot per digit bit, and a pair's slot is its (digit, tile) base, plus
// the counts of its digit in the tile's earlier wavefronts, earlier rounds and
// lower lanes -- the input order, so equal keys keep their order.  A pair's
// rank among its round's equal digits and the group's size are found once, in
// the counting pass, and kept packed in one register per round.
#include "bto_internal.h"

namespace bto {

constexpr int SCAN_CHUNK = 4096;          // counts per scan workgroup (256 threads x 16)
constexpr int RADIX_BITS = 8;
constexpr int RADIX_BINS = 1 << RADIX_BITS;
constexpr int BINS_PER_THREAD = RADIX_BINS / BLOCK;  // 1
constexpr int SORT_ROUNDS = 16;           // rounds of 64 pairs per wavefront
constexpr int SORT_TILE = BLOCK * SORT_ROUNDS;  // 4,096 pairs per workgroup
static_assert(RADIX_BINS % BLOCK == 0, "whole digits per thread");

// ---------------------------------------------------------------------------
// Scan.
// ---------------------------------------------------------------------------
// Exclusive scan of one 4,096-count chunk by one workgroup; the chunk's total
// goes to totals[chunk] (if non-null); add: an offset per chunk (or null).
// launch_exclusive_scan reads `in` twice, so in and out must not overlap.
__global__ __launch_bounds__(BLOCK) void scan_chunk_kernel(const uint32_t* in, uint32_t* out, uint64_t n,
                                                           uint32_t* totals, const uint32_t* add) {
    __shared__ uint32_t s_wave[BLOCK / WAVE];
    constexpr int PER = SCAN_CHUNK / BLOCK;  // 16 consecutive counts per thread
    const uint64_t c0 = (uint64_t)blockIdx.x * SCAN_CHUNK + (uint64_t)threadIdx.x * PER;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = c0 + k < n ? in[c0 + k] : 0u;
        sum += v[k];
    }
    // exclusive scan of the per-thread sums: within the wavefront, then over the wavefronts
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == WAVE - 1) s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        const uint32_t t = s_wave[w];
        before += w < wave ? t : 0u;
        total += t;
    }
    uint32_t run = before + incl - sum + (add ? add[blockIdx.x] : 0u);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (c0 + k < n) out[c0 + k] = run;
        run += v[k];
    }
    if (totals && threadIdx.x == 0) totals[blockIdx.x] = total;
}

// Exclusive scan of the chunk totals (any count) by one workgroup, in place.
__global__ __launch_bounds__(BLOCK) void scan_totals_kernel(uint32_t* t, uint32_t n) {
    __shared__ uint32_t s_wave[BLOCK / WAVE];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    if (threadIdx.x == 0) s_carry = 0u;
    __syncthreads();
    for (uint32_t b = 0; b < n; b += BLOCK) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t x = i < n ? t[i] : 0u;
        uint32_t incl = x;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == WAVE - 1) s_wave[wave] = incl;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / WAVE; ++w) {
            before += w < wave ? s_wave[w] : 0u;
            total += s_wave[w];
        }
        const uint32_t carry = s_carry;
        if (i < n) t[i] = carry + before + incl - x;
        __syncthreads();  // every thread has read s_wave and s_carry
        if (threadIdx.x == 0) s_carry = carry + total;
        __syncthreads();
    }
}

size_t scan_temp_bytes(uint64_t n) {
    const uint64_t chunks = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return (size_t)(chunks > 0 ? chunks : 1) * sizeof(uint32_t);
}

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t n, void* temp, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t chunks = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    uint32_t* totals = static_cast<uint32_t*>(temp);
    if (chunks == 1) {
        hipLaunchKernelGGL(scan_chunk_kernel, dim3(1), dim3(BLOCK), 0, s, in, out, n, nullptr, nullptr);
        return hipGetLastError();
    }
    // chunk totals first (the chunk-local scans written to out by this pass
    // are rewritten with their offsets by the third pass)
    hipLaunchKernelGGL(scan_chunk_kernel, dim3((unsigned)chunks), dim3(BLOCK), 0, s, in, out, n, totals, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(BLOCK), 0, s, totals, (uint32_t)chunks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // out holds each chunk's local exclusive scan: add the chunk offsets
    hipLaunchKernelGGL(scan_chunk_kernel, dim3((unsigned)chunks), dim3(BLOCK), 0, s, in, out, n, nullptr, totals);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Radix sort.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void radix_hist_kernel(const uint64_t* key, uint64_t n, int shift,
                                                           uint32_t* hist, uint32_t ntiles) {
    __shared__ uint32_t s_h[RADIX_BINS];
#pragma unroll
    for (int j = 0; j < BINS_PER_THREAD; ++j) s_h[threadIdx.x + j * BLOCK] = 0u;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * SORT_TILE;
#pragma unroll 4
    for (int k = 0; k < SORT_ROUNDS; ++k) {
        const uint64_t i = t0 + (uint64_t)k * BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&s_h[(uint32_t)(key[i] >> shift) & (RADIX_BINS - 1)], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BINS_PER_THREAD; ++j) {
        const uint32_t d = threadIdx.x + j * BLOCK;
        hist[(uint64_t)d * ntiles + blockIdx.x] = s_h[d];
    }
}

// Lanes of the wavefront whose digit equals this lane's (among the lanes in
// `active`).
__device__ __forceinline__ unsigned long long digit_peers(uint32_t d, unsigned long long active) {
    unsigned long long m = active;
#pragma unroll
    for (int b = 0; b < RADIX_BITS; ++b) {
        const unsigned long long bal = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

__global__ __launch_bounds__(BLOCK) void radix_scatter_kernel(const uint64_t* key, const uint32_t* val, uint64_t n,
                                                              int shift, const uint32_t* offs, uint32_t ntiles,
                                                              uint64_t* key_out, uint32_t* val_out) {
    constexpr int W = BLOCK / WAVE;
    __shared__ uint32_t s_cnt[W][RADIX_BINS];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < BINS_PER_THREAD; ++j) s_cnt[w][threadIdx.x + j * BLOCK] = 0u;
    __syncthreads();
    const uint64_t w0 = (uint64_t)blockIdx.x * SORT_TILE + (uint64_t)wave * (WAVE * SORT_ROUNDS);
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint64_t k[SORT_ROUNDS];
    uint32_t v[SORT_ROUNDS];
    uint32_t rg[SORT_ROUNDS];  // rank among the round's equal digits | group size << 8 (0: no pair)
    // counts of each digit in this wavefront's 1,024 pairs
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const uint64_t i = w0 + (uint64_t)r * WAVE + lane;
        const bool ok = i < n;
        k[r] = ok ? key[i] : 0ull;
        v[r] = ok ? val[i] : 0u;
        const uint32_t d = (uint32_t)(k[r] >> shift) & (RADIX_BINS - 1);
        const unsigned long long peers = digit_peers(d, __ballot(ok));
        const uint32_t rank = (uint32_t)__popcll(peers & lt), size = (uint32_t)__popcll(peers);
        rg[r] = ok ? rank | (size << 8) : 0u;
        if (ok && rank == 0u) s_cnt[wave][d] += size;  // the group's lowest lane
    }
    __syncthreads();
    // base of each digit for each wavefront of the tile
#pragma unroll
    for (int j = 0; j < BINS_PER_THREAD; ++j) {
        const uint32_t d = threadIdx.x + j * BLOCK;
        uint32_t run = offs[(uint64_t)d * ntiles + blockIdx.x];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t c = s_cnt[w][d];
            s_cnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const uint32_t d = (uint32_t)(k[r] >> shift) & (RADIX_BINS - 1);
        const uint32_t size = rg[r] >> 8, rank = rg[r] & 0xFFu;
        const uint32_t base = s_cnt[wave][d];  // read by every lane of the group before the lowest one adds
        if (size) {
            key_out[base + rank] = k[r];
            val_out[base + rank] = v[r];
        }
        if (size && rank == 0u) s_cnt[wave][d] = base + size;
    }
}

size_t radix_temp_bytes(uint64_t n) {
    const uint64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    const uint64_t cnt = (tiles > 0 ? tiles : 1) * RADIX_BINS;
    return (size_t)(2 * cnt) * sizeof(uint32_t) + scan_temp_bytes(cnt) + 256;
}

hipError_t launch_radix_sort_pairs(uint64_t* key, uint32_t* val, uint64_t* key_alt, uint32_t* val_alt, uint64_t n,
                                   int bits, void* temp, bool* result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (n == 0) return hipSuccess;
    if (n > 0xFFFFFFFFull) return hipErrorInvalidValue;
    const uint64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    const uint64_t cnt = tiles * RADIX_BINS;
    uint32_t* hist = static_cast<uint32_t*>(temp);
    uint32_t* offs = hist + cnt;
    void* stemp = offs + cnt;
    uint64_t* ka = key;
    uint32_t* va = val;
    uint64_t* kb = key_alt;
    uint32_t* vb = val_alt;
    bool alt = false;
    for (int shift = 0; shift < bits; shift += RADIX_BITS) {
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)tiles), dim3(BLOCK), 0, s, ka, n, shift, hist,
                           (uint32_t)tiles);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = launch_exclusive_scan(hist, offs, cnt, stemp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)tiles), dim3(BLOCK), 0, s, ka, va, n, shift, offs,
                           (uint32_t)tiles, kb, vb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ka, kb);
        std::swap(va, vb);
        alt = !alt;
    }
    *result_in_alt = alt;
    return hipSuccess;
}

}  // namespace bto
