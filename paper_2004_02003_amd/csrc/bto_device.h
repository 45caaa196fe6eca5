// Device-side building blocks of the BTO advection path for gfx950.
//
// Particle state between launches: the grid cell (10 bits per axis, packed in
// one dword) plus the offset inside it as three 32-bit fixed-point fractions
// -- one 16-byte record, loaded and stored as a single dwordx4.  Inside a
// launch the position lives in FP64 registers (cell + offset is exact in
// FP64), so stage points and the step update are formed in FP64 and the
// boundary test is exact; the velocity sampler runs in FP32 (or FP64 on
// request).  Storing a position between launches rounds it by at most 2^-33
// cells.
//
// Velocity grids stay in the caller's layout (AoS xyz per point, x fastest).
// The sampler reads each cell as four x-rows of two adjacent points (24 bytes
// for float32, 12 bytes for float16/bfloat16), one vector access per row;
// gfx950 under ROCm runs with unaligned global access enabled, so the
// 2-byte-aligned 12-byte rows of 16-bit grids need no padding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace bto {

constexpr int KMAX = 128;  // RK4 steps fused into one launch (one per cycle)
constexpr int NSEG = 8;    // particle segments, one per XCD
constexpr int WAVE = 64;
constexpr int BLOCK = 256;

enum : int { S_VALID = 0, S_TERMINATED = 1, S_INVALID = 2 };
// Internal outcome of a step sampled from a staged tile: a stage point needs
// grid values outside the staged box, so the step is left undone (x kept at
// the step's start) and redone from the global grids.  Never recorded.
constexpr int S_DEFER = 3;
// Adjoint statuses of seeds whose recomputation contradicts a recorded forward.
constexpr int ADJ_DROPPED = 3, ADJ_DROPPED_PARTIAL = 4;
enum : int { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };
enum : int { MODE_LINEAR = 0, MODE_FROZEN = 1 };
// Mode bit: extended-precision sampling.  In-cell offsets, sums and stage
// velocities in FP64; trilinear weights applied in FP32 to the corner
// differences from the cell's base corner (trilerp / trilerp_mid for double).
constexpr int MODE_FP64 = 2;
template <int MODE>
constexpr bool is_frozen = (MODE & MODE_FROZEN) != 0;
// Arithmetic type of the sampler in a mode.
template <int MODE>
using SampleT = typename std::conditional<(MODE & MODE_FP64) != 0, double, float>::type;
// Per-seed record of an ended particle: flag << 28 | bits below | exit step.
constexpr int32_t META_LIVE = -1;          // record slot of a particle still advancing
constexpr int META_SHIFT = 28;
constexpr int32_t META_OUTSIDE = 1 << 27;  // seeded outside the block
constexpr int32_t META_EXITPT = 1 << 26;   // exit point recorded (terminated in a step)
constexpr int32_t META_STEP = (1 << 26) - 1;

struct __align__(16) PState {
    uint32_t cell;  // cx | cy << 10 | cz << 20
    uint32_t q[3];  // offset inside the cell in units of 2^-32 (fixed point, [0, 1))
};

constexpr double OFFSET_UNIT = 1.0 / 4294967296.0;  // 2^-32

// The position cell + q * 2^-32 is exact in FP64 (10 + 32 bits).
__device__ __forceinline__ void unpack(const PState& s, double x[3]) {
    x[0] = (double)(s.cell & 1023u) + (double)s.q[0] * OFFSET_UNIT;
    x[1] = (double)((s.cell >> 10) & 1023u) + (double)s.q[1] * OFFSET_UNIT;
    x[2] = (double)((s.cell >> 20) & 1023u) + (double)s.q[2] * OFFSET_UNIT;
}

// Nearest representable state (error <= 2^-33 cells per axis): an offset that
// rounds up to a whole cell moves to the next cell.  x must be inside the
// block (0 <= x_d <= n_d - 1 <= 1023).
__device__ __forceinline__ PState pack(const double x[3]) {
    PState s;
    uint32_t c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double fl = floor(x[d]);
        const double r = rint((x[d] - fl) * 4294967296.0);  // exact product, integer in [0, 2^32]
        const bool carry = r >= 4294967296.0;
        c[d] = (uint32_t)(int)fl + (carry ? 1u : 0u);
        s.q[d] = carry ? 0u : (uint32_t)r;
    }
    s.cell = c[0] | (c[1] << 10) | (c[2] << 20);
    return s;
}

// ---------------------------------------------------------------------------
// Block geometry in cell units.
// ---------------------------------------------------------------------------
struct Geom {
    int32_t n[3];        // grid points per axis
    double nmax[3];      // n - 1: the closed box is [0, nmax]
    double inv_sp[3];    // 1 / spacing: world velocity -> cells per unit time
    uint32_t sy, sz;     // point strides of y and z (n <= 1024 per axis)
};

__device__ __forceinline__ bool inside(const Geom& g, const double p[3]) {
    return p[0] >= 0.0 && p[0] <= g.nmax[0] && p[1] >= 0.0 && p[1] <= g.nmax[1] &&
           p[2] >= 0.0 && p[2] <= g.nmax[2];
}

// Sampling cell i_d = min(floor(p_d), n_d - 2) and offset f_d = p_d - i_d,
// rounded to the sampler's type R (FP32 unless sampling in FP64).
template <class R>
struct CellR {
    uint32_t base;  // point index of corner (i, j, k)
    int i[3];       // the cell indices (i, j, k)
    R f[3];
};
using Cell = CellR<float>;

template <class R = float>
__device__ __forceinline__ CellR<R> locate(const Geom& g, const double p[3]) {
    CellR<R> c;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int v = (int)floor(p[d]);
        v = v > g.n[d] - 2 ? g.n[d] - 2 : v;
        c.i[d] = v;
        c.f[d] = (R)(p[d] - (double)v);
    }
    c.base = (uint32_t)c.i[0] + g.sy * (uint32_t)c.i[1] + g.sz * (uint32_t)c.i[2];
    return c;
}

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return fma(a, b, c); }

// ---------------------------------------------------------------------------
// Corner values of one cell of one grid level, held in registers across the
// RK4 stages (and across steps: the level n+1 corners of step n are the level
// n corners of step n+1).  Four x-rows of two adjacent points; row r has
// y-offset (r & 1) and z-offset (r >> 1); value (r, q) is component q % 3 of
// point q / 3.  16-bit grids are converted to FP32 once, when loaded.
// ---------------------------------------------------------------------------
constexpr uint32_t NO_CELL = 0xFFFFFFFFu;

struct __attribute__((packed, aligned(4))) Row32 { float v[6]; };

// Value (r, q) of a row of two 16-bit points packed as three dwords
// (x0|y0, z0|x1, y1|z1), converted to FP32 (exact).
template <int DT>
__device__ __forceinline__ float dec16(uint32_t w, int hi) {
    const uint32_t h = hi ? (w >> 16) : (w & 0xFFFFu);
    if constexpr (DT == DT_F16) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
    } else {
        return __uint_as_float(h << 16);
    }
}

// A row of two 16-bit points (12 bytes at a 2-byte-aligned offset: half of
// the rows start off a dword boundary) as three dwords, through one 4-aligned
// 16-byte load that holds it, shifted into place in registers.  The window
// starts at most at lim (the grid's size in bytes minus 16), so it never
// reads beyond the grid.  Misaligned 12-byte loads cost the texture path
// more than the aligned 16 bytes (6% on the 512^3 f16 in situ step).
__device__ __forceinline__ void load_row16(const char* V, uint32_t pt, uint64_t lim, uint32_t w[3]) {
    const uint64_t off = (uint64_t)pt * 6u;
    uint64_t st = off & ~3ull;
    st = st < lim ? st : lim;
    const uint4 q = *reinterpret_cast<const uint4*>(V + st);
    const uint32_t sh = (uint32_t)(off - st) * 8u;  // 0, 16 or (clamped at the end) 32
    w[0] = (uint32_t)((((uint64_t)q.y << 32) | q.x) >> sh);
    w[1] = (uint32_t)((((uint64_t)q.z << 32) | q.y) >> sh);
    w[2] = (uint32_t)((((uint64_t)q.w << 32) | q.z) >> sh);
}

template <int DT>
struct CellCache {
    uint32_t base;
    float R[4][6];
    __device__ __forceinline__ float v(int r, int q) const { return R[r][q]; }
    __device__ __forceinline__ void load_row(const char* V, uint32_t pt, int r, uint64_t) {
        const Row32 x = *reinterpret_cast<const Row32*>(V + (uint64_t)pt * 12u);
#pragma unroll
        for (int q = 0; q < 6; ++q) R[r][q] = x.v[q];
    }
};

// 16-bit grids: the rows stay packed in registers (12 instead of 24 per
// level) and are converted to FP32 where the sampler reads them.
template <>
struct CellCache<DT_F16> {
    uint32_t base;
    uint32_t W[4][3];
    __device__ __forceinline__ float v(int r, int q) const { return dec16<DT_F16>(W[r][q >> 1], q & 1); }
    __device__ __forceinline__ void load_row(const char* V, uint32_t pt, int r, uint64_t lim) {
        load_row16(V, pt, lim, W[r]);
    }
};

template <>
struct CellCache<DT_BF16> {
    uint32_t base;
    uint32_t W[4][3];
    __device__ __forceinline__ float v(int r, int q) const { return dec16<DT_BF16>(W[r][q >> 1], q & 1); }
    __device__ __forceinline__ void load_row(const char* V, uint32_t pt, int r, uint64_t lim) {
        load_row16(V, pt, lim, W[r]);
    }
};

template <int DT>
__device__ __forceinline__ void ensure(const Geom& g, const char* V, uint32_t base, CellCache<DT>& c) {
    if (c.base != base) {
        const uint64_t lim = 6ull * (uint64_t)g.sz * (uint64_t)g.n[2] - 16ull;  // 16-bit rows only
        c.load_row(V, base, 0, lim);
        c.load_row(V, base + g.sy, 1, lim);
        c.load_row(V, base + g.sz, 2, lim);
        c.load_row(V, base + g.sy + g.sz, 3, lim);
        c.base = base;
    }
}

// Trilinear corner weights w[r][x] (row r as above, x-offset x), times `scale`.
template <class R>
__device__ __forceinline__ void corner_weights(const R f[3], R scale, R w[4][2]) {
    const R wz0 = ((R)1 - f[2]) * scale, wz1 = f[2] * scale;
    const R wy0 = (R)1 - f[1], wy1 = f[1];
    const R yz[4] = {wy0 * wz0, wy1 * wz0, wy0 * wz1, wy1 * wz1};
    const R wx0 = (R)1 - f[0], wx1 = f[0];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        w[r][0] = yz[r] * wx0;
        w[r][1] = yz[r] * wx1;
    }
}

// Trilinear interpolation of one level, in the arithmetic of R (the corner
// values are FP32 numbers, exact in either type).
template <class CA, class R>
__device__ __forceinline__ void trilerp(const CA& A, const R f[3], R out[3]) {
    R w[4][2];
    corner_weights<R>(f, (R)1, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        R acc = w[0][0] * (R)A.v(0, c);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r) acc = fmar(w[r][0], (R)A.v(r, c), acc);
            acc = fmar(w[r][1], (R)A.v(r, 3 + c), acc);
        }
        out[c] = acc;
    }
}

// The extended-precision sampler (MODE_FP64, R = double).  The weights and
// the corner differences stay in FP32; the base corner, the sum and the stage
// velocity are FP64: v = b + sum_i w_i (v_i - b) with b the cell's first
// corner.  The base enters with coefficient exactly 1, so the weights' and
// the sum's rounding scale with the differences across the cell, not with the
// velocity itself -- close to a sampler entirely in FP64 at a fraction of its
// conversions and registers.
template <class CA>
__device__ __forceinline__ void trilerp(const CA& A, const double f[3], double out[3]) {
    const float ff[3] = {(float)f[0], (float)f[1], (float)f[2]};
    float w[4][2];
    corner_weights<float>(ff, 1.f, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float b = A.v(0, c);
        float acc = w[0][1] * (A.v(0, 3 + c) - b);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            acc = fmaf(w[r][0], A.v(r, c) - b, acc);
            acc = fmaf(w[r][1], A.v(r, 3 + c) - b, acc);
        }
        out[c] = (double)b + (double)acc;
    }
}

// The same at the time midpoint: base (b_A + b_B) / 2, differences of both levels.
template <class CA>
__device__ __forceinline__ void trilerp_mid(const CA& A, const CA& B, const double f[3], double out[3]) {
    const float ff[3] = {(float)f[0], (float)f[1], (float)f[2]};
    float w[4][2];
    corner_weights<float>(ff, 0.5f, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float ba = A.v(0, c), bb = B.v(0, c);
        float acc = w[0][1] * ((A.v(0, 3 + c) - ba) + (B.v(0, 3 + c) - bb));
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            acc = fmaf(w[r][0], (A.v(r, c) - ba) + (B.v(r, c) - bb), acc);
            acc = fmaf(w[r][1], (A.v(r, 3 + c) - ba) + (B.v(r, 3 + c) - bb), acc);
        }
        out[c] = 0.5 * ((double)ba + (double)bb) + (double)acc;
    }
}

// Trilinear interpolation of the time midpoint (A + B) / 2 of two levels:
// the factor 1/2 is folded into the weights.
template <class CA, class R>
__device__ __forceinline__ void trilerp_mid(const CA& A, const CA& B, const R f[3], R out[3]) {
    R w[4][2];
    corner_weights<R>(f, (R)0.5, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        R acc = w[0][0] * (R)A.v(0, c);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r) acc = fmar(w[r][0], (R)A.v(r, c), acc);
            acc = fmar(w[r][0], (R)B.v(r, c), acc);
            acc = fmar(w[r][1], (R)A.v(r, 3 + c), acc);
            acc = fmar(w[r][1], (R)B.v(r, 3 + c), acc);
        }
        out[c] = acc;
    }
}

// ---------------------------------------------------------------------------
// Two lanes per particle (FP32 grids).  The pair (lanes 2m, 2m+1) carries the
// same particle; lane h = lane & 1 keeps and loads only the x-corner h of
// each of the cell's four rows: 12 bytes, one dwordx3 load per row, and the
// pair's loads are adjacent in memory, so a wavefront's row load covers one
// contiguous run with half the cache-line accesses per particle of the
// one-lane layout.  Each lane forms the partial trilinear sum over its
// corners and adds its partner's with one DPP lane swap; both then hold the
// same velocity (a + b == b + a), so positions and decisions stay identical.
// ---------------------------------------------------------------------------
struct __attribute__((packed, aligned(4))) Pt32 { float v[3]; };

struct PairCache {
    uint32_t base;
    uint32_t h;      // x-corner of this lane (0 or 1)
    float R[4][3];   // corner (h, row) of each row r
    __device__ __forceinline__ void load_row(const char* V, uint32_t pt, int r) {
        const Pt32 x = *reinterpret_cast<const Pt32*>(V + (uint64_t)(pt + h) * 12u);
        R[r][0] = x.v[0];
        R[r][1] = x.v[1];
        R[r][2] = x.v[2];
    }
};

template <int DT>
__device__ __forceinline__ void ensure(const Geom& g, const char* V, uint32_t base, PairCache& c) {
    if (c.base != base) {
        c.load_row(V, base, 0);
        c.load_row(V, base + g.sy, 1);
        c.load_row(V, base + g.sz, 2);
        c.load_row(V, base + g.sy + g.sz, 3);
        c.base = base;
    }
}

__device__ __forceinline__ float pair_sum(float v) {
    // quad_perm(1, 0, 3, 2): the partner lane's value
    const int o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false);
    return v + __int_as_float(o);
}

__device__ __forceinline__ void pair_weights(const PairCache& A, const float f[3], float scale, float w[4]) {
    const float wx = (A.h ? f[0] : 1.f - f[0]) * scale;
    const float wz0 = (1.f - f[2]) * wx, wz1 = f[2] * wx;
    w[0] = (1.f - f[1]) * wz0;
    w[1] = f[1] * wz0;
    w[2] = (1.f - f[1]) * wz1;
    w[3] = f[1] * wz1;
}

__device__ __forceinline__ void trilerp(const PairCache& A, const float f[3], float out[3]) {
    float w[4];
    pair_weights(A, f, 1.f, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = w[0] * A.R[0][c];
#pragma unroll
        for (int r = 1; r < 4; ++r) acc = fmaf(w[r], A.R[r][c], acc);
        out[c] = pair_sum(acc);
    }
}

__device__ __forceinline__ void trilerp_mid(const PairCache& A, const PairCache& B, const float f[3], float out[3]) {
    float w[4];
    pair_weights(A, f, 0.5f, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = w[0] * A.R[0][c];
        acc = fmaf(w[0], B.R[0][c], acc);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            acc = fmaf(w[r], A.R[r][c], acc);
            acc = fmaf(w[r], B.R[r][c], acc);
        }
        out[c] = pair_sum(acc);
    }
}

// Trilinear value and its derivatives with respect to the in-cell offset
// (d v_c / d f_d, which equals d v_c / d p_d in cell units); MID averages the
// two levels per corner first (time midpoint).
template <bool MID, class CA>
__device__ __forceinline__ void trilerp_grad(const CA& A, const CA& B, const float f[3], float v[3],
                                             float G[3][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float lo[4], hi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lo[r] = MID ? 0.5f * (A.v(r, c) + B.v(r, c)) : A.v(r, c);
            hi[r] = MID ? 0.5f * (A.v(r, 3 + c) + B.v(r, 3 + c)) : A.v(r, 3 + c);
        }
        float a[4], dx[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[r] = lerp(lo[r], hi[r], f[0]);
            dx[r] = hi[r] - lo[r];
        }
        const float b0 = lerp(a[0], a[1], f[1]);
        const float b1 = lerp(a[2], a[3], f[1]);
        v[c] = lerp(b0, b1, f[2]);
        G[c][0] = lerp(lerp(dx[0], dx[1], f[1]), lerp(dx[2], dx[3], f[1]), f[2]);
        G[c][1] = lerp(a[1] - a[0], a[3] - a[2], f[2]);
        G[c][2] = b1 - b0;
    }
}

// ---------------------------------------------------------------------------
// Grid levels staged in LDS for one tile of cells (the tile kernels): every
// grid point of the staging box, S points per axis starting at point lo,
// x fastest, one entry per point -- (x, y, z, 0) as FP32 (16 bytes) for FP32
// grids, as the stored 16-bit values (8 bytes) otherwise; one plane per
// level.  A cell is available when both of its corner points along every axis
// lie in the staged part of the box (lim = staged points - 2 per axis).  The
// values handed to the sampler are the same FP32 numbers a global row load
// produces, so a step sampled from LDS is bit-identical to one sampled from
// the grids.
// ---------------------------------------------------------------------------
template <int DT>
struct LdsCache {
    uint32_t base;  // grid point index of the cached cell (NO_CELL: none)
    // FP32: the values; 16-bit: each row packed as three dwords as in CellCache
    typename std::conditional<DT == DT_F32, float[4][6], uint32_t[4][3]>::type R;
    const char* plane;  // this level's plane in LDS
    int lo[3], lim[3];
    int S;
    __device__ __forceinline__ float v(int r, int q) const {
        if constexpr (DT == DT_F32) {
            return R[r][q];
        } else {
            return dec16<DT>(R[r][q >> 1], q & 1);
        }
    }
    __device__ __forceinline__ void load_row(uint32_t li, int r) {
        if constexpr (DT == DT_F32) {
            const float4 a = *reinterpret_cast<const float4*>(plane + (size_t)li * 16u);
            const float4 b = *reinterpret_cast<const float4*>(plane + (size_t)li * 16u + 16u);
            R[r][0] = a.x;
            R[r][1] = a.y;
            R[r][2] = a.z;
            R[r][3] = b.x;
            R[r][4] = b.y;
            R[r][5] = b.z;
        } else {
            // entries (x0|y0, z0|0, x1|y1, z1|0) -> (x0|y0, z0|x1, y1|z1)
            const uint4 a = *reinterpret_cast<const uint4*>(plane + (size_t)li * 8u);
            R[r][0] = a.x;
            R[r][1] = (a.y & 0xFFFFu) | (a.z << 16);
            R[r][2] = (a.z >> 16) | (a.w << 16);
        }
    }
};

// Bring a cell's corner values into the cache.  Global caches always succeed;
// an LDS cache fails when the cell lies outside the staged box.
template <int DT, class Cache, class C>
__device__ __forceinline__ bool fetch(const Geom& g, const char* V, const C& c, Cache& k) {
    ensure<DT>(g, V, c.base, k);
    return true;
}

template <int DT, class C>
__device__ __forceinline__ bool fetch(const Geom&, const char*, const C& c, LdsCache<DT>& k) {
    if (k.base == c.base) return true;
    const int lx = c.i[0] - k.lo[0], ly = c.i[1] - k.lo[1], lz = c.i[2] - k.lo[2];
    if ((unsigned)lx > (unsigned)k.lim[0] || (unsigned)ly > (unsigned)k.lim[1] || (unsigned)lz > (unsigned)k.lim[2])
        return false;
    const uint32_t li = (uint32_t)lx + (uint32_t)k.S * ((uint32_t)ly + (uint32_t)k.S * (uint32_t)lz);
    const uint32_t S = (uint32_t)k.S, S2 = S * S;
    k.load_row(li, 0);
    k.load_row(li + S, 1);
    k.load_row(li + S2, 2);
    k.load_row(li + S + S2, 3);
    k.base = c.base;
    return true;
}

template <class R>
__device__ __forceinline__ bool finite3(const R k[3]) {
    return __builtin_isfinite(k[0]) && __builtin_isfinite(k[1]) && __builtin_isfinite(k[2]);
}

// Per-lane stepping state: FP64 position plus the two cached levels.
template <int DT>
struct Stepper {
    double x[3];
    CellCache<DT> A;  // level n   (cycle of the step's start)
    CellCache<DT> B;  // level n+1
};

template <int DT>
__device__ __forceinline__ void stepper_init(Stepper<DT>& st) {
    st.A.base = NO_CELL;
    st.B.base = NO_CELL;
}

// One classic RK4 step of one cycle: stage times t, t+h/2, t+h/2, t+h with the
// field linear in time between V0 (cycle n) and V1 (cycle n+1), or V0 only
// when frozen.  Each stage velocity is checked finite right after sampling;
// each later stage point and the end point are checked inside the block, in
// order.  On any event x is left at the step's start.
// Where the segment from the inside point x to the outside point y first meets
// the box surface: the smallest fraction over the faces y violates (ties to
// the lowest axis), that axis set exactly to its face value, the others
// clamped into the box against rounding.  The exit location of a terminated
// trajectory (its last inside position and the stage or end point that
// terminated it).
__device__ __forceinline__ void exit_face(const Geom& g, const double x[3], const double y[3], double f[3]) {
    double tau = INFINITY, fv = 0.0;
    int axis = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double t = INFINITY, v = 0.0;
        if (y[d] < 0.0) {
            t = (0.0 - x[d]) / (y[d] - x[d]);
        } else if (y[d] > g.nmax[d]) {
            t = (g.nmax[d] - x[d]) / (y[d] - x[d]);
            v = g.nmax[d];
        }
        if (t < tau) {
            tau = t;
            axis = d;
            fv = v;
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double q = fma(tau, y[d] - x[d], x[d]);
        f[d] = d == axis ? fv : fmin(fmax(q, 0.0), g.nmax[d]);
    }
}

// One RK4 step.  On termination x keeps the last inside position and
// `on_exit(y)` is called with the outside point that ended the particle.  With
// LDS caches the step may return S_DEFER (x unchanged) before any event.
template <int DT, int MODE, class Cache, class OnExit>
__device__ __forceinline__ int rk4_step(const Geom& g, const char* V0, const char* V1, double h, double* x,
                                        Cache& LA, Cache& LB, OnExit&& on_exit) {
    using R = SampleT<MODE>;
    const double hs[3] = {h * g.inv_sp[0], h * g.inv_sp[1], h * g.inv_sp[2]};
    R k1[3], k2[3], k3[3], k4[3];
    double y[3];
    CellR<R> c;

    c = locate<R>(g, x);
    if (!fetch<DT>(g, V0, c, LA)) return S_DEFER;
    trilerp(LA, c.f, k1);
    if (!finite3(k1)) return S_INVALID;
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = fma(0.5 * hs[d], (double)k1[d], x[d]);
    if (!inside(g, y)) {
        on_exit(y);
        return S_TERMINATED;
    }

    c = locate<R>(g, y);
    if (!fetch<DT>(g, V0, c, LA)) return S_DEFER;
    if (!is_frozen<MODE>) {
        if (!fetch<DT>(g, V1, c, LB)) return S_DEFER;
        trilerp_mid(LA, LB, c.f, k2);
    } else {
        trilerp(LA, c.f, k2);
    }
    if (!finite3(k2)) return S_INVALID;
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = fma(0.5 * hs[d], (double)k2[d], x[d]);
    if (!inside(g, y)) {
        on_exit(y);
        return S_TERMINATED;
    }

    c = locate<R>(g, y);
    if (!fetch<DT>(g, V0, c, LA)) return S_DEFER;
    if (!is_frozen<MODE>) {
        if (!fetch<DT>(g, V1, c, LB)) return S_DEFER;
        trilerp_mid(LA, LB, c.f, k3);
    } else {
        trilerp(LA, c.f, k3);
    }
    if (!finite3(k3)) return S_INVALID;
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = fma(hs[d], (double)k3[d], x[d]);
    if (!inside(g, y)) {
        on_exit(y);
        return S_TERMINATED;
    }

    c = locate<R>(g, y);
    if (!is_frozen<MODE>) {
        if (!fetch<DT>(g, V1, c, LB)) return S_DEFER;
        trilerp(LB, c.f, k4);
    } else {
        if (!fetch<DT>(g, V0, c, LA)) return S_DEFER;
        trilerp(LA, c.f, k4);
    }
    if (!finite3(k4)) return S_INVALID;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R ks = (k1[d] + k4[d]) + (R)2 * (k2[d] + k3[d]);
        y[d] = fma(hs[d] * (1.0 / 6.0), (double)ks, x[d]);
    }
    if (!inside(g, y)) {
        on_exit(y);
        return S_TERMINATED;
    }
    x[0] = y[0];
    x[1] = y[1];
    x[2] = y[2];
    return S_VALID;
}

// Stepping with two cache slots whose roles alternate: step s reads level n
// from slot s % 2 and level n+1 from the other slot, which then holds the
// next step's level n, so no corner values are ever copied.
template <int DT, int MODE>
__device__ __forceinline__ int rk4_step_alt(const Geom& g, const char* V0, const char* V1, double h, int s,
                                            Stepper<DT>& st) {
    int status;
    const auto no_exit = [](const double*) {};
    if ((s & 1) == 0) {
        status = rk4_step<DT, MODE>(g, V0, V1, h, st.x, st.A, st.B, no_exit);
        if (!is_frozen<MODE>) st.A.base = NO_CELL;  // will receive level n+2
    } else {
        status = rk4_step<DT, MODE>(g, V0, V1, h, st.x, st.B, st.A, no_exit);
        if (!is_frozen<MODE>) st.B.base = NO_CELL;
    }
    if (is_frozen<MODE>) st.A.base = st.B.base = NO_CELL;
    return status;
}

}  // namespace bto
