// Input generator (device side): the divergence-free Fourier-mode turbulence
// grid of one cycle, written straight into device memory in a storage
// precision.  Same tables and the same FP64 operations in the same order as
// the host evaluator in turb.c, with floating-point contraction off, so every
// grid value (and its rounding to the storage type) is bit-identical to the
// host's.  Input preparation only; no advection arithmetic here.
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace {

__device__ double round_sig(double x, int bits, int emin) {
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e);
    int ex = e - 1;
    if (ex < emin) ex = emin;
    const int q = ex - (bits - 1);
    return ldexp(rint(ldexp(x, -q)), q);
}

__device__ uint16_t f16_bits(double r) {  // r is exactly representable in binary16
    const _Float16 h = (_Float16)(float)r;
    return __builtin_bit_cast(uint16_t, h);
}

__device__ uint16_t bf16_bits(double r) {  // r is exactly representable in bfloat16
    const float f = (float)r;
    return (uint16_t)(__builtin_bit_cast(uint32_t, f) >> 16);
}

struct DevTables {
    int32_t nx, ny, nz, M;
    const double *exr, *exi, *eyr, *eyi, *ezr, *ezi, *pr, *pi, *amp;
};

constexpr int MMAX = 256;

// One workgroup per (j, k) row; threads over i.
__global__ __launch_bounds__(256) void turb_row_kernel(const DevTables T, int32_t c, int32_t dtype, void* out) {
    __shared__ double cr_s[MMAX], ci_s[MMAX], a_s[3 * MMAX];
    const int row = blockIdx.x;
    const int j = row % T.ny, k = row / T.ny;
    for (int m = threadIdx.x; m < T.M; m += blockDim.x) {
        const double yr = T.eyr[(size_t)m * T.ny + j], yi = T.eyi[(size_t)m * T.ny + j];
        const double zr = T.ezr[(size_t)m * T.nz + k], zi = T.ezi[(size_t)m * T.nz + k];
        const double tr = yr * zr - yi * zi;
        const double ti = yr * zi + yi * zr;
        const double qr = T.pr[(size_t)c * T.M + m], qi = T.pi[(size_t)c * T.M + m];
        cr_s[m] = tr * qr - ti * qi;
        ci_s[m] = tr * qi + ti * qr;
        a_s[3 * m] = T.amp[3 * m];
        a_s[3 * m + 1] = T.amp[3 * m + 1];
        a_s[3 * m + 2] = T.amp[3 * m + 2];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < T.nx; i += blockDim.x) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int m = 0; m < T.M; ++m) {
            const double re = T.exr[(size_t)m * T.nx + i] * cr_s[m] - T.exi[(size_t)m * T.nx + i] * ci_s[m];
            s0 += a_s[3 * m] * re;
            s1 += a_s[3 * m + 1] * re;
            s2 += a_s[3 * m + 2] * re;
        }
        const size_t o = ((size_t)row * T.nx + i) * 3;
        const double v[3] = {s0, s1, s2};
        if (dtype == 0) {
            for (int d = 0; d < 3; ++d) static_cast<double*>(out)[o + d] = v[d];
        } else if (dtype == 1) {
            for (int d = 0; d < 3; ++d) static_cast<float*>(out)[o + d] = (float)v[d];
        } else if (dtype == 2) {
            for (int d = 0; d < 3; ++d) static_cast<uint16_t*>(out)[o + d] = f16_bits(round_sig(v[d], 11, -14));
        } else {
            for (int d = 0; d < 3; ++d) static_cast<uint16_t*>(out)[o + d] = bf16_bits(round_sig(v[d], 8, -126));
        }
    }
}

}  // namespace

// Tables are device pointers laid out as in turb.c; out is a device grid
// (nz, ny, nx, 3) of dtype 0 f64, 1 f32, 2 binary16 bits, 3 bfloat16 bits.
extern "C" int turb_grid_dev(int32_t nx, int32_t ny, int32_t nz, int32_t M, const double* exr, const double* exi,
                             const double* eyr, const double* eyi, const double* ezr, const double* ezi,
                             const double* pr, const double* pi, const double* amp, int32_t c, int32_t dtype,
                             void* out, void* stream) {
    if (M > MMAX || M < 1 || nx < 1 || ny < 1 || nz < 1 || !out) return -1;
    DevTables T{nx, ny, nz, M, exr, exi, eyr, eyi, ezr, ezi, pr, pi, amp};
    hipLaunchKernelGGL(turb_row_kernel, dim3((unsigned)(ny * nz)), dim3(256), 0, (hipStream_t)stream, T, c, dtype,
                       out);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
