// Host <-> kernel interface of the BTO library (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bto_device.h"

namespace bto {

// Per-segment counters (live counts, particle-step totals) lie one 128-byte
// line apart, counter x of a slot at index x * CSTRIDE (32-bit) or x * PSTRIDE
// (64-bit).  Every workgroup of a launch adds into them; device-scope atomics
// are carried out at the memory side, and spreading the counters over lines
// lets the segments' atomics proceed in parallel there.
constexpr int CSTRIDE = 32;
constexpr int PSTRIDE = 16;

// Live particles are split into NSEG contiguous segments of the ping-pong
// buffers.  Workgroup b of a launch works on segment b % NSEG: consecutive
// workgroups are dispatched round-robin over the 8 XCDs, so each XCD keeps
// one spatially compact slab of particles (and of the field) in its own L2.
// Pointers read from a device array (the grid tables) are generic to the
// compiler, which then emits flat memory instructions for every gather and
// atomic through them; flat instructions also count against the scalar-load
// counter, so their waits and those of scalar loads merge.  Every grid lives in
// global memory: rebuilding the pointer in the global address space (through
// its integer value, which no pass folds back into the generic pointer) lets
// the compiler emit the global forms.
template <class T>
__device__ __forceinline__ T* in_global(T* p) {
    using G = __attribute__((address_space(1))) T*;
    return (T*)(G)(uintptr_t)p;
}

struct Segs {
    int64_t base[NSEG];  // first slot of each segment
};

struct AdvectArgs {
    const char* f[KMAX + 1];  // grids of cycles c0 .. c0 + K
    double h[KMAX];           // step sizes
    Geom g;
    int32_t K;                // steps in this launch
    int32_t step0;            // steps already done in the interval
    Segs segs;
    const PState* in_pos;
    const uint32_t* in_id;
    PState* out_pos;
    uint32_t* out_id;
    const uint32_t* in_count;   // NSEG live counts entering the launch
    uint32_t* out_count;        // NSEG counts of survivors (zero on entry)
    uint32_t* clear_count;      // NSEG counts cleared for the launch after next
    PState* rec_pos;            // per seed id: final state of ended particles
    int32_t* rec_meta;          // per seed id: flag << 28 | exit step
    float4* rec_out;            // per seed id: outside point - last inside position (terminated only)
    unsigned long long* psteps; // NSEG counters of attempted particle-steps
};

struct SeedLatticeArgs {
    int32_t m[3];        // lattice points per axis
    double off[3];       // lattice offset (cells)
    int32_t stride;
    int32_t morton;      // bricks in Morton order (power-of-two cube of bricks)
    int32_t octant;      // octant-major order: segment x = lattice octant x, x-fastest inside
    int32_t half[3];     // octant split per axis: indices < half[d] are the low half
    int64_t oct_base[NSEG];  // first slot of each octant
    int32_t brick[3];    // lattice points per brick and axis (product 64)
    int64_t P;
    Segs segs;
    double origin[3], spacing[3];
    PState* pos;
    uint32_t* id;
    double* seed_xyz;    // per seed id, world coordinates
    int32_t* rec_meta;
};

struct SeedExplicitArgs {
    const double* xyz;   // world
    int64_t P;
    Geom g;
    Segs segs;
    double origin[3], inv_sp[3];
    PState* pos;
    uint32_t* id;
    uint32_t* count;     // NSEG, zero on entry
    double* seed_xyz;
    PState* rec_pos;
    int32_t* rec_meta;
};

struct FlowmapArgs {
    int64_t P;
    int32_t steps_done;
    Segs segs;
    const uint32_t* count;
    const PState* pos;
    const uint32_t* id;
    const PState* rec_pos;
    const int32_t* rec_meta;
    const float4* rec_out;
    Geom g;
    const double* seed_xyz;
    double origin[3], spacing[3];
    double* out_seed;    // may be null
    double* out_end;
    uint8_t* out_flag;
    int32_t* out_exit;
    double* out_face;    // exit points (bto_exit_points)
};

// Grid-gradient records for the deterministic reduction: each accumulator
// flush writes (key, 8 x 3 corner gradients) instead of adding them to the
// grid with atomics; key = parity colour | level | cell (bit widths below,
// colour on top; colour field 8 marks an unused slot).  The j-th flush of seed
// p goes to slot j * P + p, a position fixed by (j, p) alone, so the stable
// sort leaves each group's records in an order that does not depend on thread
// timing.  A seed's flushes beyond per_seed fall back to atomics.  key == null:
// atomics.
struct GradRec {
    uint64_t* key;
    uint32_t* idx;              // record index (the sort's values)
    float* val;                 // per_seed * P x 24 floats
    uint32_t per_seed;
    uint32_t P;
    int32_t cell_bits, level_bits;
};

struct AdjointArgs {
    const char* const* f;       // device array: N + 1 grids
    const double* h;            // device array: N step sizes
    Geom g;
    int32_t N;                  // steps
    int32_t k;                  // checkpoint every k steps
    int32_t ncot;               // cotangent vectors per seed (1 or 3)
    int64_t P;
    const double* seed_xyz;     // P x 3 world
    double origin[3], sp[3];
    const float* cot;           // P x ncot x 3, d L / d x_end (world)
    float* grad_seed;           // P x ncot x 3, d L / d x_0 (world)
    float* const* grad_f;       // device array of N + 1 FP32 grids (accumulated) or null
    double* ckpt;               // ceil(N/k) slots of ck_stride doubles ([slot][seed][xyz], cell units)
    int64_t ck_stride;          // doubles per checkpoint slot (>= 3 P)
    double* buf;                // k x P x 3 scratch (slot-major)
    uint8_t* status_out;        // P (may be null): status of the recomputed forward
    const int32_t* rec_meta;    // non-null: take the forward from recorded checkpoints and these records
    GradRec grec;               // grid-gradient records (grec.key null: atomics)
    // Segments swept by this launch, sg_first down to sg_last (the whole
    // interval: nseg - 1 .. 0).  f, h and grad_f hold the grids, steps and
    // gradient grids from step f_base on.  lam (P x ncot x 3, cell units)
    // carries the cotangents from one launch to the next (read unless sg_first
    // is the last segment, written unless sg_last is 0); drop (P bytes, may be
    // null for a single launch) marks seeds dropped by an earlier launch.
    int32_t sg_first, sg_last;
    int32_t f_base;
    float* lam;
    uint8_t* drop;
};

// Checkpoint of the live particles for the adjoint: FP64 positions (cell
// units) by seed id into one slot.
struct CkptArgs {
    Segs segs;
    const uint32_t* count;     // NSEG live counts
    const PState* pos;
    const uint32_t* id;
    double* out;               // slot base: [seed id][xyz]
};

// Rebin bins: REBIN_BIN[0] x REBIN_BIN[1] x REBIN_BIN[2] cells, x fastest.
constexpr int REBIN_BIN[3] = {32, 2, 2};

struct RebinArgs {
    int64_t P;                 // slots covered by the segments
    Segs segs;
    const uint32_t* count;     // NSEG live counts
    const PState* pos;         // current buffers
    const uint32_t* id;
    PState* out_pos;           // the other ping-pong buffers
    uint32_t* out_id;
    uint32_t* bin;             // per slot: (segment, brick) bin
    uint32_t* rank;            // per slot: rank inside the bin
    uint32_t* hist;            // NSEG * nbins counts (all zero between rebins)
    uint32_t* offs;            // NSEG * nbins exclusive prefix sums
    uint32_t nbins;            // bins per segment
    uint32_t nbx, nby;         // bins along x and y
    void* temp;
    size_t temp_bytes;
};

// ---------------------------------------------------------------------------
// Tile layout of the live particles (tile-staged advection, tiles.hip).
// ---------------------------------------------------------------------------
constexpr int TILE_H = 2;       // halo cells staged around a tile
constexpr int TILE_S_16 = 17;   // staging box side in points, 16-bit grids (tile of 12 cells)
constexpr int TILE_S_F32 = 13;  // FP32 grids (tile of 8 cells)

// Tile sides in cells.  Staged tiles are cubes sized so that two workgroups'
// boxes fit a CU's LDS.  Gathering tiles are 32 x 8 x 8 cells for every
// storage type: 256 seeds at stride 2, one per thread of the workgroup, on
// rows long in x (the grid's contiguous axis), whose lines the particles of
// a row share (8% faster than 12^3 cubes on the 512^3 f16 step).
constexpr int TILE_GATHER[3] = {32, 8, 8};
constexpr int GATHER_NT = 256;  // threads per workgroup of the gathering tile step

__host__ __device__ constexpr int tile_side(int dtype, int staged, int axis) {
    return staged ? (dtype == DT_F32 ? TILE_S_F32 : TILE_S_16) - 1 - 2 * TILE_H : TILE_GATHER[axis];
}

struct __attribute__((packed, aligned(2))) Pt16 {
    uint32_t xy;
    uint16_t z;
};

struct TileGeom {
    int32_t T[3];       // tile sides (cells)
    int32_t H;          // halo of a staged tile (cells)
    int32_t nt[3];      // tiles per axis
};

struct TileOut {
    uint32_t* tc;       // bucket counts of the next step (appended)
    const int32_t* slot_of;  // bucket of each tile id
    PState* bpos;       // next step's buckets: nbuckets x cap
    uint32_t* bid;
    uint32_t cap;
    PState* list_pos;   // next step's list (bucket overflow)
    uint32_t* list_id;
    uint32_t* list_count;
};

struct TileStepArgs {
    const char* f0;           // grid of cycle n
    const char* f1;           // grid of cycle n + 1
    double h;
    Geom g;
    TileGeom tg;
    int32_t step0;            // index of this step in the interval
    const int32_t* order;     // tile of bucket b = workgroup b (-1: none); b = k * NSEG + x is the
                              // k-th tile of XCD x's run
    int32_t order_len;        // buckets (a multiple of NSEG)
    const uint32_t* tc_in;    // this step's bucket counts
    uint32_t* tc_clear;       // bucket counts cleared for the step after next
    const PState* in_pos;     // this step's buckets
    const uint32_t* in_id;
    TileOut out;
    PState* list_pos;         // this step's list (deferred particles appended)
    uint32_t* list_id;
    uint32_t* list_count;
    uint32_t* list_clear;     // list count cleared for the step after next
    PState* rec_pos;
    int32_t* rec_meta;
    float4* rec_out;
    unsigned long long* psteps;
    uint32_t* live_out;       // NSEG survivor counts of the next step
    uint32_t* live_clear;     // NSEG counts cleared for the step after next
};

struct TileListArgs {
    TileStepArgs s;
    const PState* in_pos;     // this step's list
    const uint32_t* in_id;
    const uint32_t* in_count;
};

struct TileBinArgs {
    Geom g;
    TileGeom tg;
    Segs segs;
    const uint32_t* count;    // NSEG live counts of the segments
    const PState* pos;
    const uint32_t* id;
    TileOut out;              // buckets and list of the coming step
};

struct TileLiveArgs {
    uint32_t ntiles, cap;     // buckets, slots per bucket
    const uint32_t* tc;
    const PState* bpos;
    const uint32_t* bid;
    const PState* list_pos;
    const uint32_t* list_id;
    const uint32_t* list_count;
    uint64_t list_n_max;
    int32_t steps_done;
    double origin[3], spacing[3];
    double* out_end;          // flow map (ckpt == null)
    uint8_t* out_flag;
    int32_t* out_exit;
    double* ckpt;             // checkpoint slot base: [seed id][xyz] (cell units)
};

// One workgroup per order entry; stage = 1: sample LDS-staged tiles, 0: gather
// from the grids.
hipError_t launch_tile_step(const TileStepArgs& a, int dtype, int mode, int rec, int stage, hipStream_t s);
hipError_t launch_tile_list(const TileListArgs& a, int dtype, int mode, int rec, int grid, hipStream_t s);
hipError_t launch_tile_bin(const TileBinArgs& a, int blocks_per_seg, hipStream_t s);
hipError_t launch_tile_fill(uint32_t* p, size_t n, hipStream_t s);
hipError_t launch_tile_live(const TileLiveArgs& a, hipStream_t s);

hipError_t launch_seed_lattice(const SeedLatticeArgs& a, hipStream_t s);
hipError_t launch_seed_explicit(const SeedExplicitArgs& a, hipStream_t s);
hipError_t launch_set_counts(uint32_t* counts, const uint32_t* values, int n, unsigned long long* psteps,
                             hipStream_t s);
hipError_t launch_advect(const AdvectArgs& a, int dtype, int mode, int lanes_per_particle, int record_exit,
                         int blocks_per_seg, hipStream_t s);
hipError_t launch_exit_points(const FlowmapArgs& a, hipStream_t s);
hipError_t launch_reconstruct(const int32_t m[3], double* end, const uint8_t* flag, uint8_t* state, hipStream_t s);
size_t err_scratch_bytes(int64_t P);
hipError_t launch_flowmap_error(int64_t P, const double* b, const uint8_t* bstate, const double* m, const uint8_t* mflag,
                                void* scratch, double out4[4], hipStream_t s);
// This GPU's copy of the fixed scratch of the allocation-free metric (looked
// up on the first call on each device) and its size in bytes.
hipError_t err_static_scratch(void** ptr, size_t* bytes);
hipError_t launch_place(const int32_t mb[3], const int32_t M[3], const int32_t off[3], const double shift[3],
                        const double* src_xyz, const uint8_t* src_flag, double* dst_xyz, uint8_t* dst_flag,
                        hipStream_t s);
hipError_t launch_flowmap(const FlowmapArgs& a, int blocks_per_seg, hipStream_t s);
hipError_t launch_ckpt_store(const CkptArgs& a, int blocks_per_seg, hipStream_t s);

// Touched grid points per step (diagnostic walk of the seeds, one step per
// launch).
struct TouchArgs {
    Geom g;
    const char* f0;                 // grids of the step's two cycles
    const char* f1;
    double h;                       // step size
    int64_t P;                      // seeds
    const double* seed_xyz;         // P x 3 world
    double origin[3];
    double* x;                      // P x 3 positions, cell units
    uint8_t* alive;                 // P
    uint32_t* bits0;                // bitmaps of the block's points: level n,
    uint32_t* bits1;                //   level n + 1
    unsigned long long* out;        // the step's counters: points of level n, n + 1, particles entering
};
hipError_t launch_touch_init(const TouchArgs& a, hipStream_t s);
hipError_t launch_touch_step(const TouchArgs& a, int dtype, int mode, hipStream_t s);
hipError_t launch_touch_count(uint32_t* bits, size_t words, unsigned long long* out, hipStream_t s);
hipError_t launch_touch_zero(unsigned long long* p, size_t n, hipStream_t s);
int advect_max_blocks_per_cu(int dtype, int mode, int lanes_per_particle, int record_exit);
hipError_t launch_adjoint(const AdjointArgs& a, int dtype, int mode, hipStream_t s);
size_t grad_sort_temp_bytes(uint64_t n, int bits);
// Mark all n record slots unused (before the adjoint sweep writes them).
hipError_t launch_grad_clear(const GradRec& r, uint64_t n, hipStream_t s);
// Sort the n record slots by key and add each (level, cell) group's sum to the
// grids, one parity colour at a time (no two cells of one colour share a corner).
hipError_t launch_grad_reduce(const GradRec& r, uint64_t n, uint64_t* key_out, uint32_t* idx_out, uint32_t* bounds,
                              void* temp, size_t temp_bytes, float* const* gf, const Geom& g, hipStream_t s);
hipError_t launch_ftle(const float* jac, int64_t P, double inv_T, float* out, hipStream_t s);
size_t rebin_temp_bytes(int64_t nbins_total);

// Device-wide exclusive scan of n counts (in != out; temp: scan_temp_bytes)
// and stable LSD radix sort of (key, value) pairs on the low `bits` key bits,
// ping-ponging between (key, val) and (key_alt, val_alt); *result_in_alt says
// which pair of arrays holds the sorted result (temp: radix_temp_bytes).
size_t scan_temp_bytes(uint64_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t n, void* temp, hipStream_t s);
size_t radix_temp_bytes(uint64_t n);
hipError_t launch_radix_sort_pairs(uint64_t* key, uint32_t* val, uint64_t* key_alt, uint32_t* val_alt, uint64_t n,
                                   int bits, void* temp, bool* result_in_alt, hipStream_t s);
hipError_t launch_rebin(const RebinArgs& a, hipStream_t s);

}  // namespace bto
