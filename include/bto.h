/*
 * bto.h -- C-ABI of the per-block Boundary Termination Optimization (BTO)
 * advection library for AMD Instinct MI355X (gfx950).
 *
 * The method (Sane et al., "Scalable In Situ Lagrangian Flow Map Extraction",
 * Section 3.1): on one process's block of a time-varying velocity field,
 * seed basis-flow particles on a uniform lattice, advance each with one
 * fourth-order Runge-Kutta step per simulation cycle, terminate every particle
 * whose trajectory reaches the block boundary, and at the end of the interval
 * store the flow map F_{t0}^{t}(x0) (Section 2.1) of the particles that stayed
 * inside.  No communication is involved: every block is independent.
 *
 * Conventions shared by every entry point
 *  - Coordinates: world coordinates at the boundary.  A block has n[d] grid
 *    points per axis (n[d] >= 2, n[d] <= 1024), point (i,j,k) at
 *    origin + spacing * (i,j,k).  The block is the closed box spanned by its
 *    grid points; a point on a face is inside.
 *  - Velocity grids: one per cycle, array-of-structures (vx,vy,vz) per point,
 *    x fastest then y then z: element ((k*n[1] + j)*n[0] + i)*3 + d.  Storage
 *    type float32, float16 or bfloat16 (bto_dtype); values in world units per
 *    unit time.  Between cycles n and n+1 the field is linear in time; inside
 *    a cell it is trilinear in space.
 *  - Memory: every d_* pointer is device memory of the context's device.
 *    Velocity grids are borrowed: they must stay alive and unchanged until the
 *    work enqueued on `stream` has completed.  Outputs are caller-allocated.
 *    The context owns all particle state.
 *  - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *    Calls only enqueue work and return, unless stated otherwise.
 *  - Errors: arguments are validated before anything is enqueued.  Return
 *    codes below; bto_last_error gives the message of the last failure.  An
 *    asynchronous device fault surfaces as BTO_EHIP on a later call.
 *  - Threads: one context per host thread at a time.
 */
#ifndef BTO_H
#define BTO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bto_ctx bto_ctx;

enum bto_status {
    BTO_OK = 0,
    BTO_EINVAL = -1, /* bad argument (null pointer, size, time order, dtype) */
    BTO_ENOMEM = -2, /* device allocation failed                             */
    BTO_EHIP = -3,   /* HIP runtime error (launch failure, earlier fault)    */
    BTO_ESTATE = -4, /* call out of order (e.g. advect before seed)          */
    BTO_ERANGE = -5  /* count above the context's capacity                   */
};

typedef enum { BTO_F32 = 0, BTO_F16 = 1, BTO_BF16 = 2 } bto_dtype;

/* Time interpolation inside one RK4 step (flags of bto_advect_interval).
 * LINEAR: stage velocities at t_n, t_n + h/2, t_n + h/2, t_n + h interpolate
 * linearly between the grids of cycles n and n+1.  FROZEN: every stage reads
 * the grid of cycle n (the single-time-step in situ constraint of Section 2.2). */
enum { BTO_TIME_LINEAR = 0, BTO_TIME_FROZEN = 1 };

/* Flag bit of bto_advect_interval, OR-ed with the time mode: record, for every
 * particle that this call terminates, the point where its trajectory left the
 * block (read back with bto_exit_points).  Off by default: it costs a few
 * percent of advection throughput. */
enum { BTO_RECORD_EXIT = 2 };

/* Flag bit of bto_advect_interval and bto_adjoint_interval.  On advection:
 * record checkpoints for the adjoint -- the FP64 position (cell units) of
 * every live particle at each step of the interval that is a multiple of the
 * tuning's ckpt_every (counted from the seeding), taken at launch boundaries
 * (launches are cut so that one starts at each such step).  The context holds
 * ceil(steps / ckpt_every) x max_particles x 24 bytes for them, grown on demand
 * (a growth synchronizes `stream`).  On the adjoint: take the forward
 * trajectory from those checkpoints and the recorded flags instead of
 * recomputing it (every advect call of the interval must have recorded, with
 * one ckpt_every). */
enum { BTO_RECORD_CKPT = 1 << 4 };

/* Flag bit of bto_advect_interval: extended-precision sampling.  In-cell
 * offsets, the interpolation sums and the stage velocities are FP64; the
 * trilinear weights are applied in FP32 to the differences of the corner
 * values from the cell's base corner, which enters the FP64 sum with
 * coefficient 1 (grid values and positions are unchanged: the stored values
 * and FP64 positions).  The sampler's rounding then scales with the field's
 * variation across a cell instead of its magnitude, close to a sampler
 * entirely in FP64, at a few more ALU operations per step;
 * lanes_per_particle 2 does not apply.  The adjoint always samples in FP32
 * (it rejects the flag). */
enum { BTO_SAMPLE_FP64 = 1 << 5 };

/* Per-seed outcome in the flow map. */
enum { BTO_VALID = 0, BTO_TERMINATED = 1, BTO_INVALID = 2 };

/* Adjoint only (d_status of bto_adjoint_interval): a seed the recorded forward
 * called valid but whose recomputed steps leave the block -- possible only
 * with BTO_RECORD_CKPT when the advection rounded differently from the
 * adjoint's recomputation (launches cut inside a checkpoint segment, two
 * lanes per particle, the tile layout).  Its gradient rows are zero and its
 * grid-gradient records are withdrawn (DROPPED); DROPPED_PARTIAL: some of its
 * grid contributions had already been added with atomics and stay in. */
enum { BTO_ADJ_DROPPED = 3, BTO_ADJ_DROPPED_PARTIAL = 4 };

typedef struct {
    int32_t n[3];        /* grid points per axis                    */
    double origin[3];    /* world position of grid point (0,0,0)    */
    double spacing[3];   /* grid spacing per axis (> 0)             */
} bto_block;

typedef struct {
    int64_t n_seeds;         /* seeds placed by the last bto_seed*                    */
    int64_t n_live;          /* particles still advancing                             */
    int64_t particle_steps;  /* RK4 steps attempted since seeding (live particles,    */
                             /* including each particle's terminating step)           */
    int32_t steps_done;      /* steps advanced in the current interval                */
    int32_t reserved;
} bto_stats_t;

/* Create a context for one block on HIP device `device`, with room for
 * `max_particles` seeds (device memory ~100 B per seed is allocated here).
 * Returns BTO_EINVAL for bad sizes, BTO_ENOMEM if allocation fails. */
int bto_create(const bto_block *blk, int64_t max_particles, int32_t device, bto_ctx **out);

/* Release the context and its device memory (synchronizes its device). */
int bto_destroy(bto_ctx *ctx);

/* Message of the last failing call on this context (never NULL). */
const char *bto_last_error(const bto_ctx *ctx);

/* Start a new interval with a uniform seed lattice (the 1:X data reduction of
 * Section 2.3: one seed per stride^3 grid points).  Seed coordinate per axis,
 * in cell units from the block origin: offset[d] + stride * m, m = 0, 1, ...
 * while <= n[d] - 1; offset3 == NULL means (stride - 1) / 2 on every axis.
 * Seed ids are the lattice linear index, x fastest.  *n_seeds_out (may be
 * NULL) receives the count.  BTO_ERANGE if it exceeds max_particles. */
int bto_seed(bto_ctx *ctx, int32_t stride, const double *offset3, int64_t *n_seeds_out, void *stream);

/* Start a new interval with caller-given seeds: d_xyz is n x 3 doubles (world
 * coordinates, device memory), seed id = row index.  Seeds outside the block
 * are TERMINATED at exit step 0. */
int bto_seed_explicit(bto_ctx *ctx, const double *d_xyz, int64_t n, void *stream);

/* Advance every live particle by n_steps RK4 steps (Section 3.1), one per
 * cycle, terminating at the block boundary.  d_fields is a HOST array of
 * n_steps + 1 device pointers to velocity grids of the consecutive cycles
 * c0 .. c0 + n_steps, times (host) their n_steps + 1 strictly increasing
 * times; step s uses h = times[s+1] - times[s].  May be called repeatedly
 * within one interval (e.g. once per cycle with two grids): steps accumulate
 * and exit steps count from the seeding.  flags: BTO_TIME_LINEAR or
 * BTO_TIME_FROZEN, optionally | BTO_RECORD_EXIT and | BTO_RECORD_CKPT.
 * Termination rule: the stage points y2, y3, y4 and the
 * step's end point are tested in that order; the first outside the block
 * terminates the particle in that step with its position frozen at the last
 * inside position; a non-finite velocity sample flags it INVALID likewise. */
int bto_advect_interval(bto_ctx *ctx, const void *const *d_fields, const double *times, int32_t n_steps,
                        int32_t dtype, int32_t flags, void *stream);

/* Write the interval's flow map in seed-id order (Section 2.3: end positions
 * saved at the end of the interval).  Per seed: d_seed_xyz (n x 3 doubles,
 * may be NULL), d_end_xyz (n x 3 doubles, world coordinates; for terminated
 * and invalid seeds the last inside position), d_flag (BTO_VALID /
 * BTO_TERMINATED / BTO_INVALID), d_exit_step (step of termination, or the
 * interval's step count for valid seeds).  If n_valid_out is non-NULL the call
 * synchronizes `stream` and returns the number of valid seeds.  The particle
 * state is left unchanged (more steps may follow).  An interval seeded with
 * no seeds writes nothing, and its output pointers may then be NULL.
 * BTO_ESTATE before seeding. */
int bto_flowmap_out(bto_ctx *ctx, double *d_seed_xyz, double *d_end_xyz, uint8_t *d_flag,
                    int32_t *d_exit_step, int64_t *n_valid_out, void *stream);

/* Exit points of the interval so far, in seed-id order: for every seed
 * terminated during a step, the world coordinates of the point where its
 * trajectory left the block (storing termination locations on the boundary
 * is the future work named in the paper's conclusion).  The exit point is
 * where the straight segment from the particle's last inside position to
 * the first outside point (the RK4 stage or step end that terminated it)
 * meets the block surface; one coordinate lies exactly on a face.
 * d_exit_xyz: n x 3 doubles on the device, written on `stream` (async);
 * NaN for valid and invalid seeds, for seeds outside the block at seeding
 * and for particles terminated by a call made without BTO_RECORD_EXIT.
 * May be NULL for an interval without seeds.  BTO_ESTATE before seeding. */
int bto_exit_points(bto_ctx *ctx, double *d_exit_xyz, void *stream);

/* Counters of the current interval.  Synchronizes `stream`. */
int bto_stats(bto_ctx *ctx, bto_stats_t *out, void *stream);

/* Launch-shape tuning of the advection (none of it changes which events
 * happen; end positions agree to FP32 rounding), and the checkpoint spacing:
 *   steps_per_launch    RK4 steps fused into one kernel launch, 1..128
 *                       (default 32; launches are balanced to equal lengths);
 *   rebin_every         re-sort the live particles by 32x2x2-cell bin, bins in
 *                       x-fastest order, every this many steps (restores cache
 *                       locality as the flow mixes them; 0 = never, the default);
 *   blocks_per_cu       cap on resident advection workgroups per compute unit
 *                       (0 = as many as the register budget allows);
 *   lanes_per_particle  1 (default) or 2.  With 2 and FP32 storage, the two
 *                       lanes of a pair each load and weight one x-corner of
 *                       every cell row and add their partial sums; this halves
 *                       the cache lines a wavefront touches per row load at the
 *                       cost of doubled per-particle ALU work, which pays on
 *                       incoherent (mixed) particle sets.  16-bit storage
 *                       always uses 1;
 *   ckpt_every          steps between the checkpoints that BTO_RECORD_CKPT
 *                       records (>= 1, default 10);
 *   tiles               0 (default), 1 or 2.  With 1 or 2, every RK4 step is
 *                       its own pair of launches over the live particles kept
 *                       in buckets by tile of cells, one workgroup per tile,
 *                       tiles along a Hilbert curve in cell space with one
 *                       eighth of them per XCD; each survivor goes into the bucket of the tile it
 *                       ends in, so the particles stay sorted by tile.  With 2
 *                       (tiles of 32 x 8 x 8 cells, long along x) the
 *                       particles gather from the grids.
 *                       With 1 the workgroup first stages its tile's cells
 *                       plus a 2-cell halo of both grid levels in LDS with
 *                       coalesced loads and samples from there (12^3-cell
 *                       tiles for 16-bit storage, 8^3 for FP32, so that two
 *                       workgroups fit a CU's LDS); particles whose stage
 *                       points leave the staged box are advanced from the
 *                       grids by the second launch.  Results are identical to
 *                       the default layout run one step per launch.  Pays for
 *                       large blocks advanced one cycle per call (the in situ
 *                       form).  Set before bto_seed* (it is latched for the
 *                       interval); with 1, every advect call of the interval
 *                       must use storage types of one tile size (BTO_EINVAL
 *                       otherwise).  steps_per_launch, rebin_every,
 *                       blocks_per_cu and lanes_per_particle do not apply.

 * Defaults come from the environment variables BTO_STEPS_PER_LAUNCH,
 * BTO_REBIN_EVERY, BTO_BLOCKS_PER_CU, BTO_LANES_PER_PARTICLE and BTO_TILES
 * when the context is created.  BTO_EINVAL for values out of range; takes
 * effect on the next advect call (tiles: on the next seeding). */
typedef struct {
    int32_t steps_per_launch;
    int32_t rebin_every;
    int32_t blocks_per_cu;
    int32_t lanes_per_particle;
    int32_t ckpt_every;
    int32_t tiles;
} bto_tuning;

int bto_set_tuning(bto_ctx *ctx, const bto_tuning *t);
int bto_get_tuning(const bto_ctx *ctx, bto_tuning *t);

/* Discrete adjoint of the interval: gradients of end positions with respect
 * to seed positions (the flow-map Jacobian, hence FTLE -- the paper's FTLE
 * use of flow maps, Results section) and to the velocity grids.
 * For the seeds of the current interval (bto_seed*), recompute the RK4
 * advection through d_fields / times (same meaning as bto_advect_interval,
 * all n_steps + 1 grids resident), storing each particle's position every
 * ckpt_every steps, then sweep back segment by segment: recompute the
 * segment's steps from its checkpoint and apply the transposed stage
 * recurrences of RK4 with the trilinear sampler's gradient on the cell chosen
 * by the floor/clamp rule.
 *   d_cot_end  (n_seeds x n_cot x 3 floats, world units): cotangents of the
 *              end positions; n_cot = 1 (a scalar loss L = sum c . x_end) or
 *              3 (one per axis: d_grad_seed then holds the 3x3 flow-map
 *              Jacobian dx_end/dx_0 per seed, row-major).
 *   d_grad_seed (n_seeds x n_cot x 3 floats): d L / d x_0 per cotangent.
 *              (d_cot_end and d_grad_seed may be NULL when n_seeds is 0.)
 *   d_grad_fields: NULL, or a HOST array of n_steps + 1 device pointers to
 *              float32 grids shaped like the velocity grids (non-overlapping;
 *              if one pointer repeats, the atomic path below is used);
 *              d L / d V_c is ADDED to them.  Each particle's contributions
 *              to one cell of one grid are summed, recorded, sorted by
 *              (cell parity, grid, cell, seed) and added in that order, so
 *              the result is deterministic.  A seed has room for
 *              2 (n_steps + 1) + 2 records (fewer if all records would pass
 *              about 4 GiB); its further ones, and all of them with
 *              BTO_GRAD_ATOMICS=1 in the environment at context creation,
 *              are added with FP32 atomics instead, in no fixed order.
 *              Only with n_cot = 1.
 *   d_status (n_seeds bytes, may be NULL): BTO_VALID / BTO_TERMINATED /
 *              BTO_INVALID from the recomputed forward (or the recorded
 *              flags), BTO_ADJ_DROPPED / BTO_ADJ_DROPPED_PARTIAL for seeds
 *              dropped by the adjoint (see there).
 * flags: BTO_TIME_LINEAR or BTO_TIME_FROZEN, optionally | BTO_RECORD_CKPT:
 * then the forward pass is not recomputed; the checkpoints and flags that the
 * interval's advection recorded are used (the grids, times and mode must be
 * those of that advection).  BTO_ESTATE unless every advect call since the
 * seeding recorded with one ckpt_every; BTO_EINVAL unless n_steps equals the
 * steps advected and ckpt_every the recorded spacing.  d_status then holds
 * the recorded flags.
 * Seeds that do not stay inside the block for the whole interval contribute
 * nothing: their gradient rows are zero.  Scratch of about
 * n_seeds * (n_steps / ckpt_every + ckpt_every) * 24 bytes is held by the
 * context.  The call waits for its small host-to-device tables to be copied
 * (it synchronizes `stream` once before the launch). */
int bto_adjoint_interval(bto_ctx *ctx, const void *const *d_fields, const double *times, int32_t n_steps,
                         int32_t dtype, int32_t flags, const float *d_cot_end, int32_t n_cot, float *d_grad_seed,
                         float *const *d_grad_fields, uint8_t *d_status, int32_t ckpt_every, void *stream);

/* The same adjoint one checkpoint segment per call, for intervals whose grids
 * are not all resident (the in situ form keeps two; a segment needs its
 * ckpt_every + 1).  The interval must have been advected with
 * BTO_RECORD_CKPT on every call (checkpoints every ckpt_every steps, as for
 * bto_adjoint_interval with BTO_RECORD_CKPT).  Segment s covers steps
 * s*k .. min((s+1)*k, N) - 1 (k the recorded spacing, N the steps advected);
 * call it for s = nseg - 1 down to 0 (nseg = ceil(N / k)), with
 *   d_fields / times  the k_s + 1 grids and times of cycles s*k .. s*k + k_s
 *                     (k_s the segment's steps), device pointers / host;
 *   d_cot_end         the end cotangents as for bto_adjoint_interval (read by
 *                     the first call, s = nseg - 1; may be NULL later);
 *   n_cot             1 or 3, the same on every call;
 *   d_grad_seed       written by the last call (s = 0; may be NULL before);
 *   d_grad_fields     NULL, or (n_cot = 1) the k_s + 1 FP32 gradient grids of
 *                     the segment's cycles, accumulated; the first grid of
 *                     segment s is the last of segment s - 1, so pass the same
 *                     buffer for it in both calls;
 *   d_status          NULL, or n_seeds bytes written by the last call (the
 *                     recorded flags, BTO_ADJ_DROPPED*).
 * The context carries the cotangents between the calls (n_seeds x 36 bytes).
 * Results equal bto_adjoint_interval's with BTO_RECORD_CKPT (for grid
 * gradients: up to the order in which two segments' sums meet on their
 * shared grid).  BTO_ESTATE without a complete checkpoint record, or when a
 * call is out of order (each call must sweep the segment below the previous
 * one; any advect or seed call ends the sequence); BTO_EINVAL for a segment
 * index out of range or null pointers that are needed. */
int bto_adjoint_segment(bto_ctx *ctx, int32_t segment, const void *const *d_fields, const double *times,
                        int32_t dtype, int32_t flags, const float *d_cot_end, int32_t n_cot, float *d_grad_seed,
                        float *const *d_grad_fields, uint8_t *d_status, void *stream);

/* Finite-time Lyapunov exponent per seed from row-major 3x3 Jacobians:
 * sigma = ln sqrt(lambda_max(J^T J)) / |T| (d_jac: n x 9 floats, d_out: n floats). */
int bto_ftle(bto_ctx *ctx, const float *d_jac, int64_t n, double T, float *d_out, void *stream);

/* Grid points touched per step by the context's seeds: the count behind the
 * per-unit byte figure of the advection's roofline (its input-side bytes per
 * step are the points of level n and of level n + 1 that the step's stage
 * points sample, times the bytes per point).  At the stride-2 lattice density
 * this is about 8 points per live particle per level; sparser seedings share
 * fewer corners and are counted here exactly.  A diagnostic that is not part of
 * the paper's method: the RK4 step and the trilinear sampler are those of
 * Section 3.1's advection worklet, and the count is the
 * bookkeeping of its reads.
 *   d_fields / times  n_steps + 1 grids (device) and times (host), as for
 *                     bto_advect_interval; dtype, flags likewise
 *                     (BTO_TIME_LINEAR / BTO_TIME_FROZEN, optionally
 *                     | BTO_SAMPLE_FP64);
 *   d_counts          3 x n_steps unsigned 64-bit counters, device, written:
 *                     per step n, the distinct points of level n sampled, the
 *                     distinct points of level n + 1 sampled, and the particles
 *                     entering the step.
 * The seeds walk the interval from their seeded positions with the adjoint's
 * forward (FP64 positions kept between steps), one step per launch, each
 * sampled cell marking its eight corners in a bitmap of the block's points
 * per level.  The context's own advection state is not touched.  Allocates
 * n_seeds x 25 bytes plus two bitmaps (one bit per grid point) for the call
 * and synchronizes the stream before it returns.  BTO_ESTATE before seeding;
 * BTO_EINVAL for null pointers, non-increasing times or unknown flags. */
int bto_touched_points(bto_ctx *ctx, const void *const *d_fields, const double *times, int32_t n_steps,
                       int32_t dtype, int32_t flags, unsigned long long *d_counts, void *stream);

/* ---- Post hoc side of the seed-lattice flow map (no context needed) ---- */

/* Place one block's seed-ordered flow map (lattice mb[3] points per axis, x
 * fastest: d_src_xyz mb0*mb1*mb2 x 3 doubles, d_src_flag bytes) into a larger
 * lattice of M[3] points at lattice offset off[3] (d_dst_xyz, d_dst_flag, same
 * layout), adding shift3 (host, 3 doubles, may be NULL) to every position, so
 * that the flow maps of neighbouring blocks form one lattice in one frame.
 * Device pointers; async on `stream`.  BTO_EINVAL if the block does not fit. */
int bto_place_block(const int32_t mb[3], const int32_t M[3], const int32_t off[3], const double *shift3,
                    const double *d_src_xyz, const uint8_t *d_src_flag, double *d_dst_xyz, uint8_t *d_dst_flag,
                    void *stream);

/* Rebuild the terminated entries of a lattice flow map (Section 3.2): every
 * entry whose d_flag is not BTO_VALID is replaced by the linear interpolation
 * of Eq. (1) between the nearest valid entries on both sides of it along one
 * lattice line (Eq. (2): the rebuilt value changes no later linear
 * interpolation).  Lines are taken one axis at a time, x then y then z; a pass
 * may use values rebuilt by an earlier pass, never values rebuilt in the same
 * pass.  m[3]: lattice points per axis (x fastest); d_end_xyz: m0*m1*m2 x 3
 * doubles, updated in place (entries left unrebuilt become NaN); d_state:
 * bytes out, 0 missing, 1 valid, 2 rebuilt.  Device pointers; async.
 * BTO_EINVAL for null pointers or more than 1024 lattice points on an axis. */
int bto_reconstruct_lattice(const int32_t m[3], double *d_end_xyz, const uint8_t *d_flag, uint8_t *d_state,
                            void *stream);

/* Accuracy of a BTO flow map b against a communicating one m (Section 4,
 * Eq. (5) and Eq. (6)): over the n entries that m keeps (d_m_flag BTO_VALID)
 * and b covers (d_b_state nonzero), out5[0] = mean |b - m| (the total average
 * L2 norm), out5[1] = maximum |b - m|, out5[2] = entries compared, out5[3] =
 * entries m keeps that b leaves missing, out5[4] = (cell - mean) / cell * 100
 * (Accuracy%, cell = the grid cell side in the same units).  out5 is host
 * memory; synchronizes `stream`.  Deterministic for a given n. */
int bto_flowmap_error(int64_t n, const double *d_b_xyz, const uint8_t *d_b_state, const double *d_m_xyz,
                      const uint8_t *d_m_flag, double cell, double *out5, void *stream);

/* bto_flowmap_error without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as bto_flowmap_error,
 * bit-identical to it; its partial sums live in a fixed device array of
 * 1,025 records (32,800 bytes) that the library keeps on each GPU it runs on
 * until the process ends, enough for every n (BTO_ERANGE would report an n
 * whose partials did not fit).  Every call on one GPU shares that array and
 * finds it as the previous call left it (each call writes every record it
 * reads, so nothing needs clearing): calls that overlap on one GPU, from
 * several host threads or on several streams, race and must be serialized by
 * the caller.  out5 is host memory; synchronizes `stream`. */
int bto_flowmap_error_static(int64_t n, const double *d_b_xyz, const uint8_t *d_b_state, const double *d_m_xyz,
                             const uint8_t *d_m_flag, double cell, double *out5, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BTO_H */
