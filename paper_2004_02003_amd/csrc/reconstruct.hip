// Post hoc side of the flow map on the seed lattice: placing per-block flow
// maps into one lattice, rebuilding terminated entries by the one-dimensional
// linear interpolation of Eq. (1) (Section 3.2; Eq. (2) shows the rebuilt
// value changes no later linear interpolation), and the accuracy metric of
// Eq. (5) and Eq. (6) (Section 4).
//
// Layout: lattice entries in x-fastest order, end positions as 3 doubles per
// entry, states as bytes (0 missing, 1 known, 2 rebuilt).  The rebuild runs
// one pass per axis (x, then y, then z); a pass gives each lattice line to one
// wavefront, which fills every run of unknown entries that has known entries
// on both sides.  Lines of one pass are disjoint, so a pass needs no
// synchronisation beyond the kernel boundary.
#include <mutex>

#include "bto_internal.h"

namespace bto {

constexpr uint8_t ST_MISSING = 0, ST_KNOWN = 1, ST_REBUILT = 2;

__global__ __launch_bounds__(BLOCK) void recon_init_kernel(int64_t P, double* end, const uint8_t* flag,
                                                           uint8_t* state) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < P; t += (int64_t)gridDim.x * BLOCK) {
        const bool known = flag[t] == (uint8_t)S_VALID;
        state[t] = known ? ST_KNOWN : ST_MISSING;
        if (!known) {
            const double nan = __builtin_nan("");
            end[3 * t] = nan;
            end[3 * t + 1] = nan;
            end[3 * t + 2] = nan;
        }
    }
}

// One pass along the lattice axis with point stride `st` and length `len`
// (at most 1024: a lattice line never exceeds the grid's points per axis);
// lines are indexed by the other two axes (count n_a along the first, strides
// s_a, s_b).  One wavefront per line: the line is read in chunks of 64
// entries, a ballot per chunk marks the known ones, and every unknown entry
// finds its nearest known neighbours from the ballot masks (below: highest set
// bit under its lane, carried across chunks left to right; above: lowest set
// bit over its lane, carried right to left).  All states are read before any
// entry is written, so only entries known at the start of the pass bracket.
constexpr int LINE_CHUNKS = 16;  // 16 x 64 = 1024 entries

__global__ __launch_bounds__(BLOCK) void recon_pass_kernel(int64_t n_lines, int32_t n_a, int64_t s_a, int64_t s_b,
                                                           int32_t len, int64_t st, double* end, uint8_t* state) {
#pragma clang fp contract(off)  // Eq. (1) rounded as written: two products, one sum
    const int64_t line = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (line >= n_lines) return;  // whole wavefronts leave together
    const int64_t a = line % n_a, b = line / n_a;
    const int64_t base = a * s_a + b * s_b;
    const int nchunk = (len + WAVE - 1) / WAVE;
    unsigned long long mask[LINE_CHUNKS];
#pragma unroll
    for (int c = 0; c < LINE_CHUNKS; ++c) {
        mask[c] = 0ull;
        if (c < nchunk) {
            const int i = c * WAVE + lane;
            const bool known = i < len && state[base + (int64_t)i * st] != ST_MISSING;
            mask[c] = __ballot(known);
        }
    }
    // nearest known index below each of this lane's entries (-1: none)
    int lo[LINE_CHUNKS];
    int carry = -1;
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int c = 0; c < LINE_CHUNKS; ++c) {
        lo[c] = -1;
        if (c < nchunk) {
            const unsigned long long m = mask[c] & below;
            lo[c] = m ? c * WAVE + 63 - __clzll((long long)m) : carry;
            if (mask[c]) carry = c * WAVE + 63 - __clzll((long long)mask[c]);
        }
    }
    // nearest known index above, then Eq. (1) for the unknown entries between
    carry = -1;
    const unsigned long long above = lane == 63 ? 0ull : ~((2ull << lane) - 1ull);
#pragma unroll
    for (int c = LINE_CHUNKS - 1; c >= 0; --c) {
        if (c >= nchunk) continue;
        const unsigned long long m = mask[c] & above;
        const int hi = m ? c * WAVE + __ffsll((long long)m) - 1 : carry;
        if (mask[c]) carry = c * WAVE + __ffsll((long long)mask[c]) - 1;
        const int i = c * WAVE + lane;
        const bool missing = i < len && !((mask[c] >> lane) & 1ull);
        if (missing && lo[c] >= 0 && hi >= 0) {
            // Eq. (1): L(x1) = (x1 - x0)/(x2 - x0) f(x2) + (x2 - x1)/(x2 - x0) f(x0)
            const double span = (double)(hi - lo[c]);
            const double w2 = (double)(i - lo[c]) / span;
            const double w0 = (double)(hi - i) / span;
            const int64_t q0 = base + (int64_t)lo[c] * st, q2 = base + (int64_t)hi * st, r = base + (int64_t)i * st;
#pragma unroll
            for (int d = 0; d < 3; ++d) end[3 * r + d] = w2 * end[3 * q2 + d] + w0 * end[3 * q0 + d];
            state[r] = ST_REBUILT;
        }
    }
}

// Eq. (5) partial sums: per workgroup the sum and maximum of |b - m| over the
// entries m keeps (flag valid) and b covers, and the counts of covered and
// uncovered such entries.
struct ErrPart {
    double sum, max;
    unsigned long long n, uncovered;
};

__global__ __launch_bounds__(BLOCK) void err_partial_kernel(int64_t P, const double* b, const uint8_t* bstate,
                                                            const double* m, const uint8_t* mflag, ErrPart* part) {
    double sum = 0.0, mx = 0.0;
    unsigned long long n = 0, unc = 0;
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < P; t += (int64_t)gridDim.x * BLOCK) {
        if (mflag[t] != (uint8_t)S_VALID) continue;
        if (bstate[t] == ST_MISSING) {
            ++unc;
            continue;
        }
        const double dx = b[3 * t] - m[3 * t], dy = b[3 * t + 1] - m[3 * t + 1], dz = b[3 * t + 2] - m[3 * t + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        sum += d;
        mx = fmax(mx, d);
        ++n;
    }
    __shared__ double s_sum[BLOCK], s_max[BLOCK];
    __shared__ unsigned long long s_n[BLOCK], s_u[BLOCK];
    s_sum[threadIdx.x] = sum;
    s_max[threadIdx.x] = mx;
    s_n[threadIdx.x] = n;
    s_u[threadIdx.x] = unc;
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
            s_max[threadIdx.x] = fmax(s_max[threadIdx.x], s_max[threadIdx.x + o]);
            s_n[threadIdx.x] += s_n[threadIdx.x + o];
            s_u[threadIdx.x] += s_u[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = ErrPart{s_sum[0], s_max[0], s_n[0], s_u[0]};
}

// Fixed-order sum of the partials (deterministic for a given grid): each of
// BLOCK threads sums a strided subset in order, then a fixed tree in LDS.
__global__ __launch_bounds__(BLOCK) void err_final_kernel(int nparts, const ErrPart* part, ErrPart* out) {
    double sum = 0.0, mx = 0.0;
    unsigned long long n = 0, unc = 0;
    for (int i = threadIdx.x; i < nparts; i += BLOCK) {
        sum += part[i].sum;
        mx = fmax(mx, part[i].max);
        n += part[i].n;
        unc += part[i].uncovered;
    }
    __shared__ double s_sum[BLOCK], s_max[BLOCK];
    __shared__ unsigned long long s_n[BLOCK], s_u[BLOCK];
    s_sum[threadIdx.x] = sum;
    s_max[threadIdx.x] = mx;
    s_n[threadIdx.x] = n;
    s_u[threadIdx.x] = unc;
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
            s_max[threadIdx.x] = fmax(s_max[threadIdx.x], s_max[threadIdx.x + o]);
            s_n[threadIdx.x] += s_n[threadIdx.x + o];
            s_u[threadIdx.x] += s_u[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = ErrPart{s_sum[0], s_max[0], s_n[0], s_u[0]};
}

// Copy a block's seed-ordered flow map (lattice mb, x fastest) into a larger
// lattice M at lattice offset off, adding `shift` to the positions (block
// coordinates -> domain coordinates).
__global__ __launch_bounds__(BLOCK) void place_kernel(int32_t mb0, int32_t mb1, int64_t Pb, int32_t M0, int32_t M1,
                                                      int32_t o0, int32_t o1, int32_t o2, double sh0, double sh1,
                                                      double sh2, const double* src_xyz, const uint8_t* src_flag,
                                                      double* dst_xyz, uint8_t* dst_flag) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < Pb; t += (int64_t)gridDim.x * BLOCK) {
        const int64_t i = t % mb0, j = (t / mb0) % mb1, k = t / ((int64_t)mb0 * mb1);
        const int64_t q = (i + o0) + (int64_t)M0 * ((j + o1) + (int64_t)M1 * (k + o2));
        dst_xyz[3 * q] = src_xyz[3 * t] + sh0;
        dst_xyz[3 * q + 1] = src_xyz[3 * t + 1] + sh1;
        dst_xyz[3 * q + 2] = src_xyz[3 * t + 2] + sh2;
        dst_flag[q] = src_flag[t];
    }
}

static int grid_for(int64_t n) {
    const int64_t nb = (n + BLOCK - 1) / BLOCK;
    return (int)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096);
}

hipError_t launch_reconstruct(const int32_t m[3], double* end, const uint8_t* flag, uint8_t* state, hipStream_t s) {
    const int64_t P = (int64_t)m[0] * m[1] * m[2];
    hipLaunchKernelGGL(recon_init_kernel, dim3(grid_for(P)), dim3(BLOCK), 0, s, P, end, flag, state);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t sx = 1, sy = m[0], sz = (int64_t)m[0] * m[1];
    // x pass: lines over (y, z); y pass: lines over (x, z); z pass: lines over (x, y)
    struct Pass { int32_t len; int64_t st; int32_t n_a; int64_t s_a; int32_t n_b; int64_t s_b; };
    const Pass passes[3] = {{m[0], sx, m[1], sy, m[2], sz}, {m[1], sy, m[0], sx, m[2], sz}, {m[2], sz, m[0], sx, m[1], sy}};
    for (const Pass& p : passes) {
        const int64_t lines = (int64_t)p.n_a * p.n_b;
        if (p.len < 3 || lines == 0) continue;
        if (p.len > LINE_CHUNKS * WAVE) return hipErrorInvalidValue;
        const int64_t nb = (lines * WAVE + BLOCK - 1) / BLOCK;  // one wavefront per line
        hipLaunchKernelGGL(recon_pass_kernel, dim3((unsigned)nb), dim3(BLOCK), 0, s, lines, p.n_a, p.s_a, p.s_b, p.len,
                           p.st, end, state);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int err_parts_for(int64_t P) { return grid_for(P) < 1024 ? grid_for(P) : 1024; }

size_t err_scratch_bytes(int64_t P) { return sizeof(ErrPart) * (size_t)(err_parts_for(P) + 1); }

hipError_t launch_flowmap_error(int64_t P, const double* b, const uint8_t* bstate, const double* m, const uint8_t* mflag,
                                void* scratch, double out4[4], hipStream_t s) {
    const int parts = err_parts_for(P);
    ErrPart* part = static_cast<ErrPart*>(scratch);
    hipLaunchKernelGGL(err_partial_kernel, dim3(parts), dim3(BLOCK), 0, s, P, b, bstate, m, mflag, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(err_final_kernel, dim3(1), dim3(BLOCK), 0, s, parts, part, part + parts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ErrPart r;
    e = hipMemcpyAsync(&r, part + parts, sizeof r, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    out4[0] = r.sum;
    out4[1] = r.max;
    out4[2] = (double)r.n;
    out4[3] = (double)r.uncovered;
    return hipSuccess;
}

// Fixed device scratch of the allocation-free accuracy metric: room for the
// largest partial-sum grid (1,024 workgroups) plus the final record, which
// covers every entry count.  Each GPU holds its own copy at its own address,
// found once per device with hipGetSymbolAddress; host code uses only that
// address (the array's name on the host is a stand-in, not device memory).
// Every call on one GPU shares the array: calls that overlap on one GPU race.
constexpr size_t ERR_STATIC_BYTES = 1025 * sizeof(ErrPart);
static __device__ __align__(256) char scratch[ERR_STATIC_BYTES];
constexpr int ERR_STATIC_MAX_DEVICES = 64;

hipError_t err_static_scratch(void** ptr, size_t* bytes) {
    static std::mutex mu;
    static void* addr[ERR_STATIC_MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= ERR_STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = ERR_STATIC_BYTES;
    return hipSuccess;
}

hipError_t launch_place(const int32_t mb[3], const int32_t M[3], const int32_t off[3], const double shift[3],
                        const double* src_xyz, const uint8_t* src_flag, double* dst_xyz, uint8_t* dst_flag,
                        hipStream_t s) {
    const int64_t Pb = (int64_t)mb[0] * mb[1] * mb[2];
    hipLaunchKernelGGL(place_kernel, dim3(grid_for(Pb)), dim3(BLOCK), 0, s, mb[0], mb[1], Pb, M[0], M[1], off[0], off[1],
                       off[2], shift[0], shift[1], shift[2], src_xyz, src_flag, dst_xyz, dst_flag);
    return hipGetLastError();
}

}  // namespace bto
