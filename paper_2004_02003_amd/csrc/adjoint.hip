// Discrete adjoint of the per-block RK4 advection (gradients of end positions
// with respect to seed positions and velocity grids), with checkpointing, and
// the FTLE of flow-map Jacobians.
//
// One lane per seed.  Forward: the same RK4 stepping as the advection kernel,
// storing the FP64 position every `k` steps (checkpoints) -- or none at all
// when the advection recorded the checkpoints (then the per-seed records give
// which seeds stayed inside for the whole interval).  Backward: for each
// k-step segment in reverse, recompute its steps from the checkpoint (storing
// each step's start), then walk them backwards: recompute the four stage
// points with the sampler gradients G_s (on the cell chosen by the floor/clamp
// rule) and apply the transposed stage recurrences to every cotangent vector.
// Grid gradients leave as records for the sorted, deterministic reduction
// (grad_reduce.hip), or as FP32 atomics when no record buffer is given (their
// summation order is then not fixed).  Terminated and invalid seeds contribute nothing (the
// loss covers only the basis flows that stay inside the block).
#include "bto_internal.h"

namespace bto {

struct StageRec {
    uint32_t base[4];
    float f[4][3];
    float G[4][3][3];  // d k~_r / d y_d in cells (k~ = velocity in cells per unit time)
};

// One RK4 step that also records every stage's cell, offsets and sampler
// gradient.  The stage velocities and positions come from the same sampler
// calls in the same order as rk4_step (so the step is bit-identical to the
// forward's and takes the same decisions); the gradient G of each stage is
// taken separately on the same corner values.  Returns the same status.
template <int DT, int MODE>
__device__ __forceinline__ int rk4_step_rec(const Geom& g, const char* V0, const char* V1, double h,
                                            Stepper<DT>& st, StageRec& rec) {
    const double hs[3] = {h * g.inv_sp[0], h * g.inv_sp[1], h * g.inv_sp[2]};
    float k[4][3];
    double y[3] = {st.x[0], st.x[1], st.x[2]};
    const double coef[3] = {0.5, 0.5, 1.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (s > 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) y[d] = fma(coef[s - 1] * hs[d], (double)k[s - 1][d], st.x[d]);
            if (!inside(g, y)) return S_TERMINATED;
        }
        const Cell c = locate(g, y);
        rec.base[s] = c.base;
#pragma unroll
        for (int d = 0; d < 3; ++d) rec.f[s][d] = c.f[d];
        float G[3][3], unused[3];
        if (is_frozen<MODE> || s == 0) {
            ensure<DT>(g, V0, c.base, st.A);
            trilerp(st.A, c.f, k[s]);
            trilerp_grad<false>(st.A, st.A, c.f, unused, G);
        } else if (s == 3) {
            ensure<DT>(g, V1, c.base, st.B);
            trilerp(st.B, c.f, k[s]);
            trilerp_grad<false>(st.B, st.B, c.f, unused, G);
        } else {
            ensure<DT>(g, V0, c.base, st.A);
            ensure<DT>(g, V1, c.base, st.B);
            trilerp_mid(st.A, st.B, c.f, k[s]);
            trilerp_grad<true>(st.A, st.B, c.f, unused, G);
        }
        if (!finite3(k[s])) return S_INVALID;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) rec.G[s][r][d] = (float)g.inv_sp[r] * G[r][d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float ks = (k[0][d] + k[3][d]) + 2.0f * (k[1][d] + k[2][d]);
        y[d] = fma(hs[d] * (1.0 / 6.0), (double)ks, st.x[d]);
    }
    if (!inside(g, y)) return S_TERMINATED;
    st.x[0] = y[0];
    st.x[1] = y[1];
    st.x[2] = y[2];
    return S_VALID;
}

__device__ __forceinline__ void gT(const float G[3][3], const float v[3], float out[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) out[d] = G[0][d] * v[0] + G[1][d] * v[1] + G[2][d] * v[2];
}


// Grid-gradient accumulator: the 8 corner gradients of one cell of one grid
// level, summed in registers while consecutive stage contributions hit the
// same cell and level, and flushed only when the cell or level changes (and at
// the end of each checkpoint segment).  In the reverse sweep a level receives
// its contributions from two consecutive steps (level n from step n's first
// three stages and from step n-1's last three), so a particle that stays in
// its cell flushes once per level.  A flush appends a record for the sorted,
// deterministic reduction (or, without records or when they are full, adds the
// values to the grid with FP32 atomics).
struct GradAcc {
    uint32_t base;
    int level;
    uint32_t nrec;  // records written by this seed
    float v[8][3];
};

__device__ __forceinline__ void acc_flush(const Geom& g, float* const* gf, const GradRec& R, uint32_t pid,
                                          GradAcc& A) {
    if (A.base == NO_CELL) return;
    if (R.key && A.nrec < R.per_seed) {
        // the seed's next record slot: no counter, and the lanes of a wavefront
        // that flush together write neighbouring slots
        const uint64_t slot = (uint64_t)(A.nrec++) * R.P + pid;
        const uint32_t i = A.base % g.sy, j = (A.base / g.sy) % (uint32_t)g.n[1], k = A.base / g.sz;
        const uint64_t colour = (uint64_t)((i & 1u) | ((j & 1u) << 1) | ((k & 1u) << 2));
        R.key[slot] = (colour << (R.level_bits + R.cell_bits)) | ((uint64_t)A.level << R.cell_bits) |
                      (uint64_t)A.base;  // the slot's sort value, its index, was written by the clear
        float4* out = reinterpret_cast<float4*>(R.val + 24 * (size_t)slot);
#pragma unroll
        for (int q = 0; q < 6; ++q)
            out[q] = make_float4(A.v[(4 * q) / 3][(4 * q) % 3], A.v[(4 * q + 1) / 3][(4 * q + 1) % 3],
                                 A.v[(4 * q + 2) / 3][(4 * q + 2) % 3], A.v[(4 * q + 3) / 3][(4 * q + 3) % 3]);
        A.base = NO_CELL;
        return;
    }
    float* grid = in_global(gf[A.level]);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                float* p = grid + 3 * ((uint64_t)A.base + (uint64_t)q + (uint64_t)g.sy * b + (uint64_t)g.sz * c);
                const int k = q + 2 * b + 4 * c;
                unsafeAtomicAdd(p + 0, A.v[k][0]);
                unsafeAtomicAdd(p + 1, A.v[k][1]);
                unsafeAtomicAdd(p + 2, A.v[k][2]);
            }
    A.base = NO_CELL;
}

__device__ __forceinline__ void acc_add(const Geom& g, float* const* gf, const GradRec& R, uint32_t pid, GradAcc& A,
                                        int level, uint32_t base, const float f[3], float coef, const float lam[3]) {
    if (A.base != base || A.level != level) {
        acc_flush(g, gf, R, pid, A);
        A.base = base;
        A.level = level;
#pragma unroll
        for (int k = 0; k < 8; ++k) A.v[k][0] = A.v[k][1] = A.v[k][2] = 0.f;
    }
    const float wx[2] = {1.f - f[0], f[0]}, wy[2] = {1.f - f[1], f[1]}, wz[2] = {1.f - f[2], f[2]};
    const float l[3] = {(float)g.inv_sp[0] * lam[0] * coef, (float)g.inv_sp[1] * lam[1] * coef,
                        (float)g.inv_sp[2] * lam[2] * coef};
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float w = wx[q] * wy[b] * wz[c];
                const int k = q + 2 * b + 4 * c;
                A.v[k][0] = fmaf(w, l[0], A.v[k][0]);
                A.v[k][1] = fmaf(w, l[1], A.v[k][1]);
                A.v[k][2] = fmaf(w, l[2], A.v[k][2]);
            }
}

// One wavefront per workgroup: the adjoint holds about 280 registers per lane
// (one wavefront per SIMD), so a seed set of a few tens of thousands fills
// only a fraction of the SIMDs; single-wavefront workgroups spread those
// wavefronts over every CU (and its L1 and texture pipeline) instead of
// packing four of them onto each of the first P/256 CUs.
constexpr int ADJ_BLOCK = WAVE;

template <int DT, int MODE, int NCOT>
__global__ __launch_bounds__(ADJ_BLOCK) void adjoint_kernel(const AdjointArgs a) {
    const int64_t p = (int64_t)blockIdx.x * ADJ_BLOCK + threadIdx.x;
    if (p >= a.P) return;
    const int N = a.N, K = a.k;
    const int nseg = (N + K - 1) / K;
    // checkpoints and recomputed step starts, slot-major ([slot][seed][xyz]), so a
    // wavefront's 64 positions of one slot are one contiguous 1.5 KB run
    const size_t P3 = (size_t)a.P * 3;
    const size_t CK = (size_t)a.ck_stride;
    double* ck = a.ckpt + (size_t)p * 3;
    double* buf = a.buf + (size_t)p * 3;
    // grids, steps and gradient grids are given from step f_base on
    const auto F = [&](int n) { return in_global(a.f[n - a.f_base]); };
    const auto H = [&](int n) { return a.h[n - a.f_base]; };

    Stepper<DT> st;
    stepper_init(st);
    int status;
    if (a.rec_meta) {
        // forward recorded by the advection: its checkpoints are in place and
        // the record says whether the seed stayed inside for the whole interval
        const int32_t meta = a.rec_meta[p];
        status = meta == META_LIVE ? S_VALID : (int)((uint32_t)meta >> META_SHIFT);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) st.x[d] = (a.seed_xyz[3 * p + d] - a.origin[d]) * a.g.inv_sp[d];
        status = inside(a.g, st.x) ? S_VALID : S_TERMINATED;
        for (int n = 0; n < N && status == S_VALID; ++n) {
            if (n % K == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) ck[CK * (size_t)(n / K) + d] = st.x[d];
            }
            status = rk4_step_alt<DT, MODE>(a.g, F(n), F(n + 1), H(n), n, st);
        }
    }
    // a seed dropped by the call of a later segment stays dropped
    const int prior = a.drop ? (int)a.drop[p] : 0;
    const bool first = a.sg_first == nseg - 1, last = a.sg_last == 0;

    float lam[NCOT][3];
#pragma unroll
    for (int c = 0; c < NCOT; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float* src = first ? a.cot : a.lam;
            lam[c][d] = status == S_VALID && !prior ? src[(p * NCOT + c) * 3 + d] * (first ? (float)a.sp[d] : 1.f)
                                                    : 0.f;
        }

    GradAcc acc;
    acc.base = NO_CELL;
    acc.level = -1;
    acc.nrec = 0;
    // A recomputed step that does not stay inside contradicts the forward that
    // called the seed valid: possible only when the forward was taken by the
    // advection with other rounding (recorded checkpoints; launches cut inside a
    // checkpoint segment, two lanes per particle, the tile layout).  Such a seed
    // is dropped.
    bool mismatch = false;
    if (status == S_VALID && !prior) {
        for (int sg = a.sg_first; sg >= a.sg_last && !mismatch; --sg) {
            const int n0 = sg * K;
            const int n1 = (n0 + K < N) ? n0 + K : N;
            stepper_init(st);
#pragma unroll
            for (int d = 0; d < 3; ++d) st.x[d] = ck[CK * (size_t)sg + d];
            for (int n = n0; n < n1 && !mismatch; ++n) {
#pragma unroll
                for (int d = 0; d < 3; ++d) buf[P3 * (size_t)(n - n0) + d] = st.x[d];
                if (n + 1 < n1) mismatch = rk4_step_alt<DT, MODE>(a.g, F(n), F(n + 1), H(n), n - n0, st) != S_VALID;
            }
            for (int n = n1 - 1; n >= n0 && !mismatch; --n) {
                Stepper<DT> sr;
                stepper_init(sr);
#pragma unroll
                for (int d = 0; d < 3; ++d) sr.x[d] = buf[P3 * (size_t)(n - n0) + d];
                StageRec rec;
                if (rk4_step_rec<DT, MODE>(a.g, F(n), F(n + 1), H(n), sr, rec) != S_VALID) {
                    mismatch = true;
                    break;
                }
                const float h = (float)H(n);
                const int lv = n - a.f_base;  // grid level of cycle n in the gradient grids
#pragma unroll
                for (int c = 0; c < NCOT; ++c) {
                    float lk[4][3], ly[4][3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) lk[3][d] = (h / 6.f) * lam[c][d];
                    gT(rec.G[3], lk[3], ly[3]);
#pragma unroll
                    for (int d = 0; d < 3; ++d) lk[2][d] = (h / 3.f) * lam[c][d] + h * ly[3][d];
                    gT(rec.G[2], lk[2], ly[2]);
#pragma unroll
                    for (int d = 0; d < 3; ++d) lk[1][d] = (h / 3.f) * lam[c][d] + (0.5f * h) * ly[2][d];
                    gT(rec.G[1], lk[1], ly[1]);
#pragma unroll
                    for (int d = 0; d < 3; ++d) lk[0][d] = (h / 6.f) * lam[c][d] + (0.5f * h) * ly[1][d];
                    gT(rec.G[0], lk[0], ly[0]);
                    if (c == 0 && a.grad_f) {
                        if (is_frozen<MODE>) {
#pragma unroll
                            for (int s = 0; s < 4; ++s) acc_add(a.g, a.grad_f, a.grec, (uint32_t)p, acc, lv, rec.base[s], rec.f[s], 1.f, lk[s]);
                        } else {
                            // level n+1 first (it already holds step n+1's share), then level n
                            acc_add(a.g, a.grad_f, a.grec, (uint32_t)p, acc, lv + 1, rec.base[1], rec.f[1], 0.5f, lk[1]);
                            acc_add(a.g, a.grad_f, a.grec, (uint32_t)p, acc, lv + 1, rec.base[2], rec.f[2], 0.5f, lk[2]);
                            acc_add(a.g, a.grad_f, a.grec, (uint32_t)p, acc, lv + 1, rec.base[3], rec.f[3], 1.f, lk[3]);
                            acc_add(a.g, a.grad_f, a.grec, (uint32_t)p, acc, lv, rec.base[0], rec.f[0], 1.f, lk[0]);
                            acc_add(a.g, a.grad_f, a.grec, (uint32_t)p, acc, lv, rec.base[1], rec.f[1], 0.5f, lk[1]);
                            acc_add(a.g, a.grad_f, a.grec, (uint32_t)p, acc, lv, rec.base[2], rec.f[2], 0.5f, lk[2]);
                        }
                    }
#pragma unroll
                    for (int d = 0; d < 3; ++d) lam[c][d] += ly[0][d] + ly[1][d] + ly[2][d] + ly[3][d];
                }
            }
            if (a.grad_f && !mismatch) acc_flush(a.g, a.grad_f, a.grec, (uint32_t)p, acc);  // keep it out of the next recompute
        }
    }
    int drop = prior;
    if (mismatch) {
        // no gradient from this seed: its pending sums are dropped and this
        // call's grid records withdrawn; contributions already in the grids
        // (added with atomics after its record slots ran out, or by the call
        // of a later segment) cannot be, and the status says so
#pragma unroll
        for (int c = 0; c < NCOT; ++c) lam[c][0] = lam[c][1] = lam[c][2] = 0.f;
        bool withdrawn = true;
        if (a.grad_f) {
            if (a.grec.key) {
                const uint32_t kept = acc.nrec < a.grec.per_seed ? acc.nrec : a.grec.per_seed;
                const uint64_t unused = (uint64_t)8 << (a.grec.level_bits + a.grec.cell_bits);  // colour 8
                for (uint32_t j = 0; j < kept; ++j) a.grec.key[(uint64_t)j * a.grec.P + (uint64_t)p] = unused;
                withdrawn = acc.nrec <= a.grec.per_seed;
            } else {
                withdrawn = false;
            }
            withdrawn = withdrawn && first;
        }
        drop = withdrawn ? ADJ_DROPPED : ADJ_DROPPED_PARTIAL;
    }
    if (a.drop && drop != prior) a.drop[p] = (uint8_t)drop;
    if (last) {
        if (a.status_out) a.status_out[p] = (uint8_t)(drop ? drop : status);
#pragma unroll
        for (int c = 0; c < NCOT; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) a.grad_seed[(p * NCOT + c) * 3 + d] = lam[c][d] * (float)a.g.inv_sp[d];
    } else {
#pragma unroll
        for (int c = 0; c < NCOT; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) a.lam[(p * NCOT + c) * 3 + d] = lam[c][d];
    }
}

// ---------------------------------------------------------------------------
// FTLE: sigma = ln sqrt(lambda_max(J^T J)) / |T| per seed, from row-major
// Jacobians (3x3 FP32).  The largest eigenvalue of the symmetric 3x3 matrix
// C = J^T J comes from the closed-form trigonometric solution of its
// characteristic cubic, evaluated in FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void ftle_kernel(const float* jac, int64_t P, double inv_T, float* out) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= P) return;
    double J[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) J[r][c] = (double)jac[9 * p + 3 * r + c];
    double C[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[i][j] = J[0][i] * J[0][j] + J[1][i] * J[1][j] + J[2][i] * J[2][j];
    const double p1 = C[0][1] * C[0][1] + C[0][2] * C[0][2] + C[1][2] * C[1][2];
    const double q = (C[0][0] + C[1][1] + C[2][2]) / 3.0;
    const double p2 = (C[0][0] - q) * (C[0][0] - q) + (C[1][1] - q) * (C[1][1] - q) + (C[2][2] - q) * (C[2][2] - q) +
                      2.0 * p1;
    double lmax;
    if (p2 <= 0.0) {
        lmax = q;
    } else {
        const double pp = sqrt(p2 / 6.0);
        double B[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) B[i][j] = (C[i][j] - (i == j ? q : 0.0)) / pp;
        double detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                      B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                      B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
        double r = detB / 2.0;
        r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
        const double phi = acos(r) / 3.0;
        lmax = q + 2.0 * pp * cos(phi);
    }
    out[p] = (float)(0.5 * log(lmax) * inv_T);
}

// ---------------------------------------------------------------------------
template <int DT, int MODE, int NCOT>
static hipError_t launch_adj_t(const AdjointArgs& a, hipStream_t s) {
    const int64_t blocks = (a.P + ADJ_BLOCK - 1) / ADJ_BLOCK;
    hipLaunchKernelGGL((adjoint_kernel<DT, MODE, NCOT>), dim3((unsigned)blocks), dim3(ADJ_BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int DT, int MODE>
static hipError_t launch_adj_m(const AdjointArgs& a, hipStream_t s) {
    return a.ncot == 1 ? launch_adj_t<DT, MODE, 1>(a, s) : launch_adj_t<DT, MODE, 3>(a, s);
}

template <int DT>
static hipError_t launch_adj_d(const AdjointArgs& a, int mode, hipStream_t s) {
    return mode == MODE_LINEAR ? launch_adj_m<DT, MODE_LINEAR>(a, s) : launch_adj_m<DT, MODE_FROZEN>(a, s);
}

hipError_t launch_adjoint(const AdjointArgs& a, int dtype, int mode, hipStream_t s) {
    if (a.P == 0) return hipSuccess;
    switch (dtype) {
    case DT_F32: return launch_adj_d<DT_F32>(a, mode, s);
    case DT_F16: return launch_adj_d<DT_F16>(a, mode, s);
    default: return launch_adj_d<DT_BF16>(a, mode, s);
    }
}

hipError_t launch_ftle(const float* jac, int64_t P, double inv_T, float* out, hipStream_t s) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(ftle_kernel, dim3((unsigned)((P + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, jac, P, inv_T, out);
    return hipGetLastError();
}

}  // namespace bto
