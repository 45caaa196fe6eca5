// C-ABI of the per-block BTO library: context, argument validation and the
// launch sequence.  Every step of the path runs in the kernels of advect.hip
// (and adjoint.hip); this file only owns memory and enqueues work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bto.h"
#include "bto_internal.h"

using namespace bto;

// the three slots of live counts, ahead of the particle-step counters
static constexpr size_t COUNT_BYTES = 3 * NSEG * CSTRIDE * sizeof(uint32_t);

struct bto_ctx {
    bto_block blk;
    Geom geom;
    int device = 0;
    int64_t cap = 0;
    int cus_per_xcd = 32;
    int steps_per_launch = 32;    // fused steps per advect launch, <= KMAX (BTO_STEPS_PER_LAUNCH)
    int blocks_per_cu_cap = 0;    // cap on resident advect workgroups per CU (BTO_BLOCKS_PER_CU; 0 = occupancy)
    int rebin_every = 0;          // re-sort live particles every this many steps (BTO_REBIN_EVERY; 0 = never)
    int lanes_per_particle = 1;   // FP32 grids: 1 or 2 lanes per particle (BTO_LANES_PER_PARTICLE)
    int morton_seed = 0;          // Morton brick order at seeding when possible (BTO_MORTON_SEED)
    int octant_seed = 1;          // octant-major seeding, one lattice octant per XCD segment (BTO_OCTANT_SEED=0: slabs)
    int brick[3] = {64, 1, 1};    // lattice points per seeding brick (BTO_BRICK="bx,by,bz", product 64)
    int steps_since_rebin = 0;
    uint32_t* rebin_buf = nullptr;  // 4 x cap keys/values
    void* rebin_temp = nullptr;
    size_t rebin_temp_bytes = 0;
    // particle state (ping-pong)
    PState* pos[2] = {nullptr, nullptr};
    uint32_t* id[2] = {nullptr, nullptr};
    int cur = 0;
    // per-seed records
    PState* rec_pos = nullptr;
    int32_t* rec_meta = nullptr;
    float4* rec_out = nullptr;        // terminated particles: outside point - last inside position
    double* seed_xyz = nullptr;
    // counters: ring of 3 x NSEG live counts, then NSEG particle-step counters
    // (each counter in a line of its own: CSTRIDE, PSTRIDE)
    uint32_t* counts = nullptr;
    unsigned long long* psteps = nullptr;
    int slot = 0;           // ring slot holding the current live counts
    // interval bookkeeping (host)
    bool seeded = false;
    int64_t n_seeds = 0;
    int32_t steps_done = 0;
    Segs segs{};
    int64_t seg_cap[NSEG] = {0};
    // adjoint scratch (grown on demand)
    void* adj_scratch = nullptr;
    size_t adj_bytes = 0;
    // checkpoints recorded by BTO_RECORD_CKPT advection: ck_slots slots of cap x 3 doubles
    int ckpt_every = 10;          // tuning: spacing of recorded checkpoints
    double* ck_rec = nullptr;
    int64_t ck_slots = 0;
    int ck_k = 0;                 // spacing recorded in this interval (0: nothing advected yet)
    bool ck_ok = false;           // every advect call since the seeding recorded, with spacing ck_k
    // segment-by-segment adjoint: cotangents carried between the calls, dropped-seed marks
    void* seg_buf = nullptr;
    size_t seg_bytes = 0;
    int seg_next = -1;            // segment the next bto_adjoint_segment call must sweep (-1: none)
    int seg_ncot = 0;
    // grid-gradient records of the adjoint (sorted reduction), grown on demand
    void* grec_buf = nullptr;
    size_t grec_bytes = 0;
    bool grad_atomics = false;    // BTO_GRAD_ATOMICS=1: add grid gradients with FP32 atomics instead
    // tile layout (tile-staged steps; tuning `tiles`, latched at seeding)
    int tiles = 0;
    bool tile_on = false;         // this interval advances in the tile layout
    bool tile_layout = false;     // live particles are in the buckets (else in the segments)
    TileGeom tg{};
    uint32_t ntiles = 0, tcap = 0;
    int tile_grid = 0;            // workgroups of a tile step (8 x the largest octant of tiles)
    void* tile_buf = nullptr;     // [order | slot of tile | 3 x bucket counts, 3 list counts | buckets x 2]
    size_t tile_bytes = 0;
    int32_t* tile_order = nullptr;  // tile of each bucket (= workgroup)
    int32_t* tile_slot = nullptr;   // bucket of each tile
    uint32_t* tcount = nullptr;     // 3 x buckets counts
    uint32_t* lcount = nullptr;
    PState* bpos[2] = {nullptr, nullptr};
    uint32_t* bid[2] = {nullptr, nullptr};
    int tb = 0;                   // bucket buffer of the current step
    std::string err;
};

static int fail(bto_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

static int hip_fail(bto_ctx* c, hipError_t e, const char* where) {
    return fail(c, BTO_EHIP, "%s: %s", where, hipGetErrorString(e));
}

// Pending asynchronous errors (a fault in earlier work) surface here.
static int check_pending(bto_ctx* c) {
    hipError_t e = hipPeekAtLastError();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return hip_fail(c, e, "earlier HIP error");
    }
    return BTO_OK;
}

static void set_segments(bto_ctx* c, int64_t P) {
    for (int x = 0; x < NSEG; ++x) c->segs.base[x] = (x * P + NSEG - 1) / NSEG;
    for (int x = 0; x < NSEG; ++x) c->seg_cap[x] = (x + 1 < NSEG ? c->segs.base[x + 1] : P) - c->segs.base[x];
}

static int blocks_per_seg(const bto_ctx* c, int64_t max_seg, int per_cu) {
    int64_t need = (max_seg + BLOCK - 1) / BLOCK;
    int64_t lim = (int64_t)c->cus_per_xcd * per_cu;
    if (need < 1) need = 1;
    return (int)(need < lim ? need : lim);
}

extern "C" {

int bto_create(const bto_block* blk, int64_t max_particles, int32_t device, bto_ctx** out) {
    if (!blk || !out) return BTO_EINVAL;
    *out = nullptr;
    for (int d = 0; d < 3; ++d) {
        if (blk->n[d] < 2 || blk->n[d] > 1024) return BTO_EINVAL;
        if (!(blk->spacing[d] > 0.0) || !std::isfinite(blk->spacing[d]) || !std::isfinite(blk->origin[d]))
            return BTO_EINVAL;
    }
    if (max_particles < 1 || max_particles > (int64_t)0xFFFFFFFFll) return BTO_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return BTO_EINVAL;
    bto_ctx* c = new (std::nothrow) bto_ctx();
    if (!c) return BTO_ENOMEM;
    c->blk = *blk;
    c->device = device;
    c->cap = max_particles;
    for (int d = 0; d < 3; ++d) {
        c->geom.n[d] = blk->n[d];
        c->geom.nmax[d] = (double)(blk->n[d] - 1);
        c->geom.inv_sp[d] = 1.0 / blk->spacing[d];
    }
    c->geom.sy = (uint32_t)blk->n[0];
    c->geom.sz = (uint32_t)blk->n[0] * (uint32_t)blk->n[1];
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return BTO_EINVAL;
    }
    if (const char* e = std::getenv("BTO_STEPS_PER_LAUNCH")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= KMAX) c->steps_per_launch = v;
    }
    if (const char* e = std::getenv("BTO_BLOCKS_PER_CU")) c->blocks_per_cu_cap = std::atoi(e);
    if (const char* e = std::getenv("BTO_REBIN_EVERY")) c->rebin_every = std::atoi(e) > 0 ? std::atoi(e) : 0;
    if (const char* e = std::getenv("BTO_MORTON_SEED")) c->morton_seed = std::atoi(e) != 0;
    if (const char* e = std::getenv("BTO_OCTANT_SEED")) c->octant_seed = std::atoi(e) != 0;
    if (const char* e = std::getenv("BTO_LANES_PER_PARTICLE")) c->lanes_per_particle = std::atoi(e) == 2 ? 2 : 1;
    if (const char* e = std::getenv("BTO_GRAD_ATOMICS")) c->grad_atomics = std::atoi(e) != 0;
    if (const char* e = std::getenv("BTO_TILES")) {
        const int v = std::atoi(e);
        c->tiles = v >= 0 && v <= 2 ? v : 0;
    }
    if (const char* e = std::getenv("BTO_BRICK")) {
        int b0 = 0, b1 = 0, b2 = 0;
        if (std::sscanf(e, "%d,%d,%d", &b0, &b1, &b2) == 3 && b0 > 0 && b1 > 0 && b2 > 0 && b0 * b1 * b2 == 64) {
            c->brick[0] = b0;
            c->brick[1] = b1;
            c->brick[2] = b2;
        }
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount >= NSEG)
        c->cus_per_xcd = prop.multiProcessorCount / NSEG;
    const size_t P = (size_t)max_particles;
    bool ok = true;
    for (int q = 0; q < 2 && ok; ++q) {
        ok = ok && hipMalloc(&c->pos[q], P * sizeof(PState)) == hipSuccess;
        ok = ok && hipMalloc(&c->id[q], P * sizeof(uint32_t)) == hipSuccess;
    }
    ok = ok && hipMalloc(&c->rec_pos, P * sizeof(PState)) == hipSuccess;
    ok = ok && hipMalloc(&c->rec_meta, P * sizeof(int32_t)) == hipSuccess;
    ok = ok && hipMalloc(&c->rec_out, P * sizeof(float4)) == hipSuccess;
    ok = ok && hipMalloc(&c->seed_xyz, P * 3 * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&c->counts, COUNT_BYTES + NSEG * PSTRIDE * sizeof(unsigned long long)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        bto_destroy(c);
        return BTO_ENOMEM;
    }
    c->psteps = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(c->counts) + COUNT_BYTES);
    *out = c;
    return BTO_OK;
}

int bto_destroy(bto_ctx* c) {
    if (!c) return BTO_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (int q = 0; q < 2; ++q) {
        if (c->pos[q]) (void)hipFree(c->pos[q]);
        if (c->id[q]) (void)hipFree(c->id[q]);
    }
    if (c->rec_pos) (void)hipFree(c->rec_pos);
    if (c->rec_meta) (void)hipFree(c->rec_meta);
    if (c->rec_out) (void)hipFree(c->rec_out);
    if (c->seed_xyz) (void)hipFree(c->seed_xyz);
    if (c->counts) (void)hipFree(c->counts);
    if (c->adj_scratch) (void)hipFree(c->adj_scratch);
    if (c->ck_rec) (void)hipFree(c->ck_rec);
    if (c->grec_buf) (void)hipFree(c->grec_buf);
    if (c->rebin_buf) (void)hipFree(c->rebin_buf);
    if (c->rebin_temp) (void)hipFree(c->rebin_temp);
    if (c->tile_buf) (void)hipFree(c->tile_buf);
    if (c->seg_buf) (void)hipFree(c->seg_buf);
    delete c;
    return BTO_OK;
}

const char* bto_last_error(const bto_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

static int begin(bto_ctx* c) {
    if (!c) return BTO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, BTO_EHIP, "hipSetDevice failed");
    return check_pending(c);
}

static int start_interval(bto_ctx* c, int64_t P, const uint32_t* seg_counts, hipStream_t s) {
    uint32_t vals[3 * NSEG] = {0};
    for (int x = 0; x < NSEG; ++x) vals[x] = seg_counts ? seg_counts[x] : 0u;
    hipError_t e = launch_set_counts(c->counts, vals, 3 * NSEG, c->psteps, s);
    if (e != hipSuccess) return hip_fail(c, e, "set_counts launch");
    c->slot = 0;
    c->cur = 0;
    c->seeded = true;
    c->n_seeds = P;
    c->steps_done = 0;
    c->steps_since_rebin = 0;
    c->ck_k = 0;
    c->ck_ok = true;
    c->tile_on = c->tiles != 0;
    c->tile_layout = false;
    c->seg_next = -1;
    return BTO_OK;
}

// ---------------------------------------------------------------------------
// Tile layout.
// ---------------------------------------------------------------------------
// Index of (x, y, z) along a 3-D Hilbert curve over [0, 2^bits)^3, in
// Skilling's transpose form ("Programming the Hilbert curve", 2004): undo the
// excess work of the axes from the top bit down, Gray-encode across the axes,
// then interleave the bits from the most significant.  Consecutive indices
// are unit steps in space.
static uint64_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int bits) {
    uint32_t X[3] = {x, y, z};
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int j = bits - 1; j >= 0; --j)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> j) & 1u);
    return h;
}


// Tile geometry of storage type dtype, buckets sized for the current seeds,
// and the tile order: workgroups run round-robin over the 8 XCDs, and XCD x
// takes the x-th eighth of the tiles in Morton order (neighbouring tiles run
// close in time on one XCD and share their halo lines in its L2).
static int tile_setup(bto_ctx* c, int dtype, hipStream_t s) {
    TileGeom tg{};
    tg.H = TILE_H;
    uint64_t ntiles = 1;
    for (int d = 0; d < 3; ++d) {
        tg.T[d] = tile_side(dtype, c->tiles == 1, d);
        const int cells = c->blk.n[d] - 1;
        tg.nt[d] = (cells + tg.T[d] - 1) / tg.T[d];
        ntiles *= (uint64_t)tg.nt[d];
    }
    if (ntiles > 0xFFFFFFFFull / 2) return fail(c, BTO_ERANGE, "too many tiles");
    uint64_t per = ((uint64_t)c->n_seeds + ntiles - 1) / ntiles;
    uint64_t cap = 2 * per + 32;
    if (cap < 64) cap = 64;
    cap = (cap + 31) & ~(uint64_t)31;
    if ((ntiles + NSEG) * cap > 0xFFFFFFFFull) return fail(c, BTO_ERANGE, "tile buckets exceed 2^32 slots");
    // the same geometry and bucket size as the last interval: everything is in place
    if (c->tile_buf && std::memcmp(&c->tg, &tg, sizeof tg) == 0 && c->ntiles == (uint32_t)ntiles &&
        c->tcap == (uint32_t)cap)
        return BTO_OK;
    // workgroup order: all tiles along a Hilbert curve, cut into NSEG equal
    // contiguous runs, run x for XCD x; order[k * NSEG + x] = k-th tile of run x.
    // The curve runs in cell space: a tile's coordinates are scaled by its
    // side over the shortest side, so a run of the curve is a compact region
    // of cells even for tiles long along x (on the 512^3 f16 step: Morton
    // order on tile indices 0.877 ms, Morton in cell space 0.833 ms, Hilbert
    // in cell space 0.823 ms).
    const int tmin = std::min(tg.T[0], std::min(tg.T[1], tg.T[2]));
    int hbits = 1;
    for (int d = 0; d < 3; ++d)
        while ((1u << hbits) < (uint32_t)(tg.nt[d] * (tg.T[d] / tmin))) ++hbits;
    std::vector<std::pair<uint64_t, int32_t>> mt;
    mt.reserve((size_t)ntiles);
    for (int tz = 0; tz < tg.nt[2]; ++tz)
        for (int ty = 0; ty < tg.nt[1]; ++ty)
            for (int tx = 0; tx < tg.nt[0]; ++tx) {
                const uint32_t px = (uint32_t)(tx * (tg.T[0] / tmin)), py = (uint32_t)(ty * (tg.T[1] / tmin)),
                               pz = (uint32_t)(tz * (tg.T[2] / tmin));
                const uint64_t key = hilbert3(px, py, pz, hbits);
                mt.push_back({key, tx + tg.nt[0] * (ty + tg.nt[1] * tz)});
            }
    std::sort(mt.begin(), mt.end());
    const size_t longest = ((size_t)ntiles + NSEG - 1) / NSEG;
    const int grid = (int)(longest * NSEG);
    std::vector<int32_t> order((size_t)grid, -1);
    for (int x = 0; x < NSEG; ++x) {
        const size_t b = (size_t)ntiles * x / NSEG, e = (size_t)ntiles * (x + 1) / NSEG;
        for (size_t k = b; k < e; ++k) order[(k - b) * NSEG + x] = mt[k].second;
    }
    // bucket b holds the tile of workgroup b, so there are `grid` buckets
    std::vector<int32_t> slot_of((size_t)ntiles, -1);
    for (int b = 0; b < grid; ++b)
        if (order[(size_t)b] >= 0) slot_of[(size_t)order[(size_t)b]] = b;
    const size_t o_bytes = ((size_t)grid * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t s_bytes = ((size_t)ntiles * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t c_bytes = ((3 * (size_t)grid + 3) * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t b_bytes = (size_t)grid * cap * (sizeof(PState) + sizeof(uint32_t));
    const size_t need = o_bytes + s_bytes + c_bytes + 2 * b_bytes;
    if (need > c->tile_bytes) {
        if (c->tile_buf) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(c, e, "tile buffers sync");
            (void)hipFree(c->tile_buf);
            c->tile_buf = nullptr;
            c->tile_bytes = 0;
        }
        if (hipMalloc(&c->tile_buf, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, BTO_ENOMEM, "tile buffers of %zu bytes", need);
        }
        c->tile_bytes = need;
    }
    char* q = static_cast<char*>(c->tile_buf);
    c->tile_order = reinterpret_cast<int32_t*>(q);
    c->tile_slot = reinterpret_cast<int32_t*>(q + o_bytes);
    c->tcount = reinterpret_cast<uint32_t*>(q + o_bytes + s_bytes);
    c->lcount = c->tcount + 3 * (size_t)grid;
    char* b = q + o_bytes + s_bytes + c_bytes;
    for (int k = 0; k < 2; ++k) {
        c->bpos[k] = reinterpret_cast<PState*>(b + k * b_bytes);
        c->bid[k] = reinterpret_cast<uint32_t*>(b + k * b_bytes + (size_t)grid * cap * sizeof(PState));
    }
    hipError_t e = hipMemcpyAsync(c->tile_order, order.data(), (size_t)grid * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->tile_slot, slot_of.data(), (size_t)ntiles * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the tables are host temporaries
    if (e != hipSuccess) return hip_fail(c, e, "tile order upload");
    c->tg = tg;
    c->ntiles = (uint32_t)ntiles;
    c->tcap = (uint32_t)cap;
    c->tile_grid = grid;
    return BTO_OK;
}

// Move the live particles of the segments into the buckets of the coming
// step (all tile and list counts zeroed first; the count ring keeps its slot).
static int tile_enter(bto_ctx* c, int dtype, int max_seg_blocks, hipStream_t s) {
    int rc = tile_setup(c, dtype, s);
    if (rc) return rc;
    hipError_t e = launch_tile_fill(c->tcount, 3 * (size_t)c->tile_grid + 3, s);
    if (e != hipSuccess) return hip_fail(c, e, "tile count fill");
    TileBinArgs a{};
    a.g = c->geom;
    a.tg = c->tg;
    a.segs = c->segs;
    a.count = c->counts + NSEG * CSTRIDE * c->slot;
    a.pos = c->pos[c->cur];
    a.id = c->id[c->cur];
    c->tb = 0;
    c->cur = 1 - c->cur;  // the list of the coming step lives in the other particle buffer
    a.out.tc = c->tcount + (size_t)c->slot * c->tile_grid;
    a.out.slot_of = c->tile_slot;
    a.out.bpos = c->bpos[c->tb];
    a.out.bid = c->bid[c->tb];
    a.out.cap = c->tcap;
    a.out.list_pos = c->pos[c->cur];
    a.out.list_id = c->id[c->cur];
    a.out.list_count = c->lcount + c->slot;
    e = launch_tile_bin(a, max_seg_blocks, s);
    if (e != hipSuccess) return hip_fail(c, e, "tile bin launch");
    c->tile_layout = true;
    return BTO_OK;
}

// Live particles of the tile layout, by seed id: flow-map entries (out_end
// non-null) or FP64 positions into a checkpoint slot (ckpt non-null).
static int tile_live(bto_ctx* c, double* out_end, uint8_t* out_flag, int32_t* out_exit, double* ckpt,
                     hipStream_t s) {
    TileLiveArgs a{};
    a.ntiles = (uint32_t)c->tile_grid;
    a.cap = c->tcap;
    a.tc = c->tcount + (size_t)c->slot * c->tile_grid;
    a.bpos = c->bpos[c->tb];
    a.bid = c->bid[c->tb];
    a.list_pos = c->pos[c->cur];
    a.list_id = c->id[c->cur];
    a.list_count = c->lcount + c->slot;
    a.list_n_max = (uint64_t)c->n_seeds;
    a.steps_done = c->steps_done;
    for (int d = 0; d < 3; ++d) {
        a.origin[d] = c->blk.origin[d];
        a.spacing[d] = c->blk.spacing[d];
    }
    a.out_end = out_end;
    a.out_flag = out_flag;
    a.out_exit = out_exit;
    a.ckpt = ckpt;
    hipError_t e = launch_tile_live(a, s);
    return e == hipSuccess ? BTO_OK : hip_fail(c, e, "tile live launch");
}

// One RK4 step of every live particle in the tile layout: the tile launch,
// then the list launch; the rings advance by one.
static int tile_step(bto_ctx* c, const void* f0, const void* f1, double h, int dtype, int mode, int rec,
                     hipStream_t s) {
    const int sl = c->slot, sl1 = (c->slot + 1) % 3, sl2 = (c->slot + 2) % 3;
    TileStepArgs a{};
    a.f0 = static_cast<const char*>(f0);
    a.f1 = static_cast<const char*>(f1);
    a.h = h;
    a.g = c->geom;
    a.tg = c->tg;
    a.step0 = c->steps_done;
    a.order = c->tile_order;
    a.order_len = c->tile_grid;
    a.tc_in = c->tcount + (size_t)sl * c->tile_grid;
    a.tc_clear = c->tcount + (size_t)sl2 * c->tile_grid;
    a.in_pos = c->bpos[c->tb];
    a.in_id = c->bid[c->tb];
    a.out.tc = c->tcount + (size_t)sl1 * c->tile_grid;
    a.out.slot_of = c->tile_slot;
    a.out.bpos = c->bpos[1 - c->tb];
    a.out.bid = c->bid[1 - c->tb];
    a.out.cap = c->tcap;
    a.out.list_pos = c->pos[1 - c->cur];
    a.out.list_id = c->id[1 - c->cur];
    a.out.list_count = c->lcount + sl1;
    a.list_pos = c->pos[c->cur];
    a.list_id = c->id[c->cur];
    a.list_count = c->lcount + sl;
    a.list_clear = c->lcount + sl2;
    a.rec_pos = c->rec_pos;
    a.rec_meta = c->rec_meta;
    a.rec_out = c->rec_out;
    a.psteps = c->psteps;
    a.live_out = c->counts + NSEG * CSTRIDE * sl1;
    a.live_clear = c->counts + NSEG * CSTRIDE * sl2;
    hipError_t e = launch_tile_step(a, dtype, mode, rec, c->tiles == 1 ? 1 : 0, s);
    if (e != hipSuccess) return hip_fail(c, e, "tile step launch");
    TileListArgs l{};
    l.s = a;
    l.in_pos = c->pos[c->cur];
    l.in_id = c->id[c->cur];
    l.in_count = c->lcount + sl;
    int64_t lg = c->n_seeds / (BLOCK * 32);
    lg = lg < 64 ? 64 : (lg > 1024 ? 1024 : lg);
    e = launch_tile_list(l, dtype, mode, rec, (int)lg, s);
    if (e != hipSuccess) return hip_fail(c, e, "tile list launch");
    c->slot = sl1;
    c->cur = 1 - c->cur;
    c->tb = 1 - c->tb;
    c->steps_done += 1;
    return BTO_OK;
}

// Room for checkpoint slots 0 .. slots - 1 (keeps the recorded ones).
static int ensure_ckpt_slots(bto_ctx* c, int64_t slots, hipStream_t s) {
    if (slots <= c->ck_slots) return BTO_OK;
    int64_t want = c->ck_slots * 2 > slots ? c->ck_slots * 2 : slots;
    const size_t slot_bytes = (size_t)c->cap * 3 * sizeof(double);
    double* nb = nullptr;
    if (hipMalloc(&nb, (size_t)want * slot_bytes) != hipSuccess) {
        (void)hipGetLastError();
        want = slots;
        if (hipMalloc(&nb, (size_t)want * slot_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, BTO_ENOMEM, "checkpoint record of %lld slots", (long long)slots);
        }
    }
    if (c->ck_rec) {
        hipError_t e = hipMemcpyAsync(nb, c->ck_rec, (size_t)c->ck_slots * slot_bytes, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipFree(nb);
            return hip_fail(c, e, "checkpoint record growth");
        }
        (void)hipFree(c->ck_rec);
    }
    c->ck_rec = nb;
    c->ck_slots = want;
    return BTO_OK;
}

// Re-sort the live particles of every segment by 32x2x2-cell bin, bins in x-fastest order.
static int rebin(bto_ctx* c, hipStream_t s) {
    uint32_t nb[3];
    for (int d = 0; d < 3; ++d) nb[d] = (uint32_t)((c->blk.n[d] + REBIN_BIN[d] - 1) / REBIN_BIN[d]);
    const uint32_t nbins = nb[0] * nb[1] * nb[2];
    if (!c->rebin_buf) {
        const size_t tb = rebin_temp_bytes((int64_t)NSEG * nbins);
        if (tb == 0) return fail(c, BTO_EHIP, "rebin: scan storage query failed");
        const size_t words = (size_t)c->cap * 2 + (size_t)NSEG * nbins * 2;
        if (hipMalloc(&c->rebin_buf, words * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&c->rebin_temp, tb) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, BTO_ENOMEM, "rebin buffers");
        }
        // the bin counts start at zero once; each rebin leaves them zero again
        if (hipMemset(c->rebin_buf + (size_t)c->cap * 2, 0, (size_t)NSEG * nbins * sizeof(uint32_t)) != hipSuccess)
            return fail(c, BTO_EHIP, "rebin: clearing bin counts failed");
        c->rebin_temp_bytes = tb;
    }
    RebinArgs a{};
    a.P = c->n_seeds;
    a.segs = c->segs;
    a.count = c->counts + NSEG * CSTRIDE * c->slot;
    a.pos = c->pos[c->cur];
    a.id = c->id[c->cur];
    a.out_pos = c->pos[1 - c->cur];
    a.out_id = c->id[1 - c->cur];
    a.bin = c->rebin_buf;
    a.rank = c->rebin_buf + c->cap;
    a.hist = c->rebin_buf + 2 * (size_t)c->cap;
    a.offs = a.hist + (size_t)NSEG * nbins;
    a.nbins = nbins;
    a.nbx = nb[0];
    a.nby = nb[1];
    a.temp = c->rebin_temp;
    a.temp_bytes = c->rebin_temp_bytes;
    hipError_t e = launch_rebin(a, s);
    if (e != hipSuccess) return hip_fail(c, e, "rebin");
    c->cur = 1 - c->cur;
    c->steps_since_rebin = 0;
    return BTO_OK;
}

int bto_seed(bto_ctx* c, int32_t stride, const double* offset3, int64_t* n_seeds_out, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (stride < 1) return fail(c, BTO_EINVAL, "stride must be >= 1 (got %d)", stride);
    SeedLatticeArgs a{};
    int64_t P = 1;
    for (int d = 0; d < 3; ++d) {
        const double off = offset3 ? offset3[d] : (stride - 1) / 2.0;
        if (!std::isfinite(off) || off < 0.0) return fail(c, BTO_EINVAL, "lattice offset must be finite and >= 0");
        a.off[d] = off;
        a.m[d] = off > (double)(c->blk.n[d] - 1) ? 0 : (int32_t)std::floor((c->blk.n[d] - 1 - off) / stride) + 1;
        P *= a.m[d];
        a.origin[d] = c->blk.origin[d];
        a.spacing[d] = c->blk.spacing[d];
    }
    if (P > c->cap) return fail(c, BTO_ERANGE, "lattice has %lld seeds, capacity is %lld", (long long)P,
                                (long long)c->cap);
    a.stride = stride;
    a.P = P;
    for (int d = 0; d < 3; ++d) a.brick[d] = c->brick[d];
    {
        // Morton brick order needs a cube of 4 * 2^k lattice points per axis (<= 4 * 256)
        const int32_t mb = a.m[0] / 4;
        const bool pow2 = mb >= 1 && mb <= 256 && (mb & (mb - 1)) == 0;
        a.morton = (a.m[0] == a.m[1] && a.m[1] == a.m[2] && a.m[0] % 4 == 0 && pow2 && c->morton_seed) ? 1 : 0;
    }
    set_segments(c, P);
    if (c->octant_seed && !a.morton) {
        // one lattice octant per segment (each XCD keeps a compact octant of the block)
        a.octant = 1;
        int64_t size[NSEG];
        for (int d = 0; d < 3; ++d) a.half[d] = (a.m[d] + 1) / 2;
        for (int o = 0; o < NSEG; ++o) {
            size[o] = 1;
            for (int d = 0; d < 3; ++d) size[o] *= ((o >> d) & 1) ? a.m[d] - a.half[d] : a.half[d];
        }
        int64_t acc = 0;
        for (int o = 0; o < NSEG; ++o) {
            a.oct_base[o] = acc;
            c->segs.base[o] = acc;
            c->seg_cap[o] = size[o];
            acc += size[o];
        }
    }
    a.segs = c->segs;
    a.pos = c->pos[0];
    a.id = c->id[0];
    a.seed_xyz = c->seed_xyz;
    a.rec_meta = c->rec_meta;
    hipStream_t s = (hipStream_t)stream;
    uint32_t cnt[NSEG];
    for (int x = 0; x < NSEG; ++x) cnt[x] = (uint32_t)c->seg_cap[x];
    rc = start_interval(c, P, cnt, s);
    if (rc) return rc;
    if (P > 0) {
        hipError_t e = launch_seed_lattice(a, s);
        if (e != hipSuccess) return hip_fail(c, e, "seed launch");
    }
    if (n_seeds_out) *n_seeds_out = P;
    return BTO_OK;
}

int bto_seed_explicit(bto_ctx* c, const double* d_xyz, int64_t n, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !d_xyz)) return fail(c, BTO_EINVAL, "null seed array or negative count");
    if (n > c->cap) return fail(c, BTO_ERANGE, "%lld seeds, capacity is %lld", (long long)n, (long long)c->cap);
    set_segments(c, n);
    hipStream_t s = (hipStream_t)stream;
    rc = start_interval(c, n, nullptr, s);
    if (rc) return rc;
    if (n == 0) return BTO_OK;
    SeedExplicitArgs a{};
    a.xyz = d_xyz;
    a.P = n;
    a.g = c->geom;
    a.segs = c->segs;
    for (int d = 0; d < 3; ++d) {
        a.origin[d] = c->blk.origin[d];
        a.inv_sp[d] = 1.0 / c->blk.spacing[d];
    }
    a.pos = c->pos[0];
    a.id = c->id[0];
    a.count = c->counts;  // slot 0
    a.seed_xyz = c->seed_xyz;
    a.rec_pos = c->rec_pos;
    a.rec_meta = c->rec_meta;
    hipError_t e = launch_seed_explicit(a, s);
    if (e != hipSuccess) return hip_fail(c, e, "seed_explicit launch");
    return BTO_OK;
}

int bto_advect_interval(bto_ctx* c, const void* const* d_fields, const double* times, int32_t n_steps,
                        int32_t dtype, int32_t flags, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (!d_fields || !times) return fail(c, BTO_EINVAL, "null field or time array");
    if (n_steps <= 0) return fail(c, BTO_EINVAL, "n_steps must be > 0 (got %d)", n_steps);
    if (dtype < BTO_F32 || dtype > BTO_BF16) return fail(c, BTO_EINVAL, "unknown dtype %d", dtype);
    const int tmode = flags & ~(BTO_RECORD_EXIT | BTO_RECORD_CKPT | BTO_SAMPLE_FP64);
    if (tmode != BTO_TIME_LINEAR && tmode != BTO_TIME_FROZEN) return fail(c, BTO_EINVAL, "unknown flags %d", flags);
    const int mode = tmode | ((flags & BTO_SAMPLE_FP64) ? MODE_FP64 : 0);
    const int rec = (flags & BTO_RECORD_EXIT) ? 1 : 0;
    const bool rec_ck = (flags & BTO_RECORD_CKPT) != 0;
    for (int32_t q = 0; q <= n_steps; ++q)
        if (!d_fields[q]) return fail(c, BTO_EINVAL, "field pointer %d is null", q);
    for (int32_t q = 0; q < n_steps; ++q)
        if (!(times[q + 1] > times[q]) || !std::isfinite(times[q + 1]) || !std::isfinite(times[q]))
            return fail(c, BTO_EINVAL, "times must be finite and strictly increasing (index %d)", q);
    if (!c->seeded) return fail(c, BTO_ESTATE, "advect called before seeding");
    if ((int64_t)c->steps_done + n_steps > META_STEP) return fail(c, BTO_ERANGE, "interval too long");
    c->seg_next = -1;  // more steps: a segment-by-segment adjoint starts over
    hipStream_t s = (hipStream_t)stream;
    // checkpoint record: complete only if every call of the interval records with one spacing
    if (rec_ck) {
        if (c->ck_k == 0) c->ck_k = c->ckpt_every;
        if (c->ck_k != c->ckpt_every) c->ck_ok = false;
    } else {
        c->ck_ok = false;
    }
    const bool store_ck = rec_ck && c->ck_ok;
    if (store_ck && c->n_seeds > 0) {
        rc = ensure_ckpt_slots(c, ((int64_t)c->steps_done + n_steps - 1) / c->ck_k + 1, s);
        if (rc) return rc;
    }
    if (c->n_seeds == 0) {
        c->steps_done += n_steps;
        return BTO_OK;
    }
    int64_t max_seg = 0;
    for (int x = 0; x < NSEG; ++x) max_seg = c->seg_cap[x] > max_seg ? c->seg_cap[x] : max_seg;
    if (c->tile_on) {
        if (c->tile_layout && tile_side(dtype, c->tiles == 1, 0) != c->tg.T[0])
            return fail(c, BTO_EINVAL, "this interval's tile layout has %d-cell tiles; storage type %d needs %d",
                        c->tg.T[0], dtype, tile_side(dtype, c->tiles == 1, 0));
        if (!c->tile_layout) {
            rc = tile_enter(c, dtype, blocks_per_seg(c, max_seg, 4), s);
            if (rc) return rc;
        }
        for (int32_t q = 0; q < n_steps; ++q) {
            if (store_ck && c->steps_done % c->ck_k == 0) {
                rc = tile_live(c, nullptr, nullptr, nullptr,
                               c->ck_rec + (size_t)(c->steps_done / c->ck_k) * (size_t)c->cap * 3, s);
                if (rc) return rc;
            }
            rc = tile_step(c, d_fields[q], d_fields[q + 1], times[q + 1] - times[q], dtype, mode, rec, s);
            if (rc) return rc;
        }
        return BTO_OK;
    }
    const int lpp = dtype == BTO_F32 ? c->lanes_per_particle : 1;
    int per_cu = advect_max_blocks_per_cu(dtype, mode, lpp, rec);
    if (c->blocks_per_cu_cap > 0 && c->blocks_per_cu_cap < per_cu) per_cu = c->blocks_per_cu_cap;
    const int R = blocks_per_seg(c, max_seg * lpp, per_cu);
    // launches of (nearly) equal length, at most steps_per_launch steps each
    int kmax = c->steps_per_launch;
    if (c->rebin_every > 0 && c->rebin_every < kmax) kmax = c->rebin_every;
    const int nl = (n_steps + kmax - 1) / kmax;
    for (int32_t l = 0, q0 = 0; q0 < n_steps; ++l) {
        int K = n_steps / nl + (l < n_steps % nl ? 1 : 0);
        if (store_ck) {
            // launches end at checkpoint steps; equal lengths between two of them
            const int to_ck = c->ck_k - c->steps_done % c->ck_k;
            const int seg = to_ck < n_steps - q0 ? to_ck : n_steps - q0;
            const int parts = (seg + kmax - 1) / kmax;
            K = (seg + parts - 1) / parts;
        }
        if (c->rebin_every > 0 && c->steps_since_rebin >= c->rebin_every) {
            rc = rebin(c, s);
            if (rc) return rc;
        }
        if (store_ck && c->steps_done % c->ck_k == 0) {
            CkptArgs ca{};
            ca.segs = c->segs;
            ca.count = c->counts + NSEG * CSTRIDE * c->slot;
            ca.pos = c->pos[c->cur];
            ca.id = c->id[c->cur];
            ca.out = c->ck_rec + (size_t)(c->steps_done / c->ck_k) * (size_t)c->cap * 3;
            hipError_t e = launch_ckpt_store(ca, blocks_per_seg(c, max_seg, 4), s);
            if (e != hipSuccess) return hip_fail(c, e, "checkpoint store launch");
        }
        AdvectArgs a{};
        for (int q = 0; q <= K; ++q) a.f[q] = static_cast<const char*>(d_fields[q0 + q]);
        for (int q = 0; q < K; ++q) a.h[q] = times[q0 + q + 1] - times[q0 + q];
        a.g = c->geom;
        a.K = K;
        a.step0 = c->steps_done;
        a.segs = c->segs;
        a.in_pos = c->pos[c->cur];
        a.in_id = c->id[c->cur];
        a.out_pos = c->pos[1 - c->cur];
        a.out_id = c->id[1 - c->cur];
        a.in_count = c->counts + NSEG * CSTRIDE * c->slot;
        a.out_count = c->counts + NSEG * CSTRIDE * ((c->slot + 1) % 3);
        a.clear_count = c->counts + NSEG * CSTRIDE * ((c->slot + 2) % 3);
        a.rec_pos = c->rec_pos;
        a.rec_meta = c->rec_meta;
        a.rec_out = c->rec_out;
        a.psteps = c->psteps;
        hipError_t e = launch_advect(a, dtype, mode, lpp, rec, R, s);
        if (e != hipSuccess) return hip_fail(c, e, "advect launch");
        c->cur = 1 - c->cur;
        c->slot = (c->slot + 1) % 3;
        c->steps_done += K;
        c->steps_since_rebin += K;
        q0 += K;
    }
    return BTO_OK;
}

int bto_flowmap_out(bto_ctx* c, double* d_seed_xyz, double* d_end_xyz, uint8_t* d_flag, int32_t* d_exit_step,
                    int64_t* n_valid_out, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (!c->seeded) return fail(c, BTO_ESTATE, "flowmap_out called before seeding");
    // an interval without seeds writes nothing: its (empty) outputs may be null
    if (c->n_seeds > 0 && (!d_end_xyz || !d_flag || !d_exit_step)) return fail(c, BTO_EINVAL, "null output pointer");
    hipStream_t s = (hipStream_t)stream;
    if (c->n_seeds > 0) {
        FlowmapArgs a{};
        a.P = c->n_seeds;
        a.steps_done = c->steps_done;
        a.segs = c->segs;
        a.count = c->counts + NSEG * CSTRIDE * c->slot;
        a.pos = c->pos[c->cur];
        a.id = c->id[c->cur];
        a.rec_pos = c->rec_pos;
        a.rec_meta = c->rec_meta;
        a.seed_xyz = c->seed_xyz;
        for (int d = 0; d < 3; ++d) {
            a.origin[d] = c->blk.origin[d];
            a.spacing[d] = c->blk.spacing[d];
        }
        a.out_seed = d_seed_xyz;
        a.out_end = d_end_xyz;
        a.out_flag = d_flag;
        a.out_exit = d_exit_step;
        int64_t max_seg = 0;
        for (int x = 0; x < NSEG; ++x) max_seg = c->seg_cap[x] > max_seg ? c->seg_cap[x] : max_seg;
        // the segment writer only when the live particles are in the segments
        hipError_t e = launch_flowmap(a, c->tile_layout ? 0 : blocks_per_seg(c, max_seg, 4), s);
        if (e != hipSuccess) return hip_fail(c, e, "flowmap launch");
        if (c->tile_layout) {
            rc = tile_live(c, d_end_xyz, d_flag, d_exit_step, nullptr, s);
            if (rc) return rc;
        }
    }
    if (n_valid_out) {
        bto_stats_t st;
        rc = bto_stats(c, &st, stream);
        if (rc) return rc;
        *n_valid_out = st.n_live;
    }
    return BTO_OK;
}

int bto_exit_points(bto_ctx* c, double* d_exit_xyz, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (!c->seeded) return fail(c, BTO_ESTATE, "exit_points called before seeding");
    if (c->n_seeds > 0 && !d_exit_xyz) return fail(c, BTO_EINVAL, "null output pointer");
    if (c->n_seeds > 0) {
        FlowmapArgs a{};
        a.P = c->n_seeds;
        a.rec_pos = c->rec_pos;
        a.rec_meta = c->rec_meta;
        a.rec_out = c->rec_out;
        a.g = c->geom;
        for (int d = 0; d < 3; ++d) {
            a.origin[d] = c->blk.origin[d];
            a.spacing[d] = c->blk.spacing[d];
        }
        a.out_face = d_exit_xyz;
        hipError_t e = launch_exit_points(a, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(c, e, "exit points launch");
    }
    return BTO_OK;
}

static bool lattice_ok(const int32_t m[3]) {
    return m && m[0] >= 1 && m[1] >= 1 && m[2] >= 1 && (int64_t)m[0] * m[1] * m[2] <= ((int64_t)1 << 40);
}

int bto_reconstruct_lattice(const int32_t m[3], double* d_end_xyz, const uint8_t* d_flag, uint8_t* d_state,
                            void* stream) {
    if (!lattice_ok(m) || !d_end_xyz || !d_flag || !d_state) return BTO_EINVAL;
    if (m[0] > 1024 || m[1] > 1024 || m[2] > 1024) return BTO_EINVAL;  // one line fits one wavefront's chunks
    return launch_reconstruct(m, d_end_xyz, d_flag, d_state, (hipStream_t)stream) == hipSuccess ? BTO_OK : BTO_EHIP;
}

int bto_flowmap_error(int64_t n, const double* d_b_xyz, const uint8_t* d_b_state, const double* d_m_xyz,
                      const uint8_t* d_m_flag, double cell, double* out5, void* stream) {
    if (n < 1 || !d_b_xyz || !d_b_state || !d_m_xyz || !d_m_flag || !out5 || !(cell > 0.0)) return BTO_EINVAL;
    void* scratch = nullptr;
    if (hipMalloc(&scratch, err_scratch_bytes(n)) != hipSuccess) return BTO_ENOMEM;
    double r[4];
    const hipError_t e = launch_flowmap_error(n, d_b_xyz, d_b_state, d_m_xyz, d_m_flag, scratch, r, (hipStream_t)stream);
    (void)hipFree(scratch);
    if (e != hipSuccess) return BTO_EHIP;
    const double mean = r[2] > 0 ? r[0] / r[2] : 0.0;
    out5[0] = mean;
    out5[1] = r[1];
    out5[2] = r[2];
    out5[3] = r[3];
    out5[4] = (cell - mean) / cell * 100.0;
    return BTO_OK;
}

int bto_flowmap_error_static(int64_t n, const double* d_b_xyz, const uint8_t* d_b_state, const double* d_m_xyz,
                             const uint8_t* d_m_flag, double cell, double* out5, void* stream) {
    if (n < 1 || !d_b_xyz || !d_b_state || !d_m_xyz || !d_m_flag || !out5 || !(cell > 0.0)) return BTO_EINVAL;
    void* scratch = nullptr;
    size_t have = 0;
    if (err_static_scratch(&scratch, &have) != hipSuccess) return BTO_EHIP;
    if (err_scratch_bytes(n) > have) return BTO_ERANGE;
    double r[4];
    if (launch_flowmap_error(n, d_b_xyz, d_b_state, d_m_xyz, d_m_flag, scratch, r, (hipStream_t)stream) != hipSuccess)
        return BTO_EHIP;
    const double mean = r[2] > 0 ? r[0] / r[2] : 0.0;
    out5[0] = mean;
    out5[1] = r[1];
    out5[2] = r[2];
    out5[3] = r[3];
    out5[4] = (cell - mean) / cell * 100.0;
    return BTO_OK;
}

int bto_place_block(const int32_t mb[3], const int32_t M[3], const int32_t off[3], const double shift3[3],
                    const double* d_src_xyz, const uint8_t* d_src_flag, double* d_dst_xyz, uint8_t* d_dst_flag,
                    void* stream) {
    if (!lattice_ok(mb) || !lattice_ok(M) || !off || !d_src_xyz || !d_src_flag || !d_dst_xyz || !d_dst_flag)
        return BTO_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (off[d] < 0 || off[d] + mb[d] > M[d]) return BTO_EINVAL;
    const double zero[3] = {0.0, 0.0, 0.0};
    return launch_place(mb, M, off, shift3 ? shift3 : zero, d_src_xyz, d_src_flag, d_dst_xyz, d_dst_flag,
                        (hipStream_t)stream) == hipSuccess
               ? BTO_OK
               : BTO_EHIP;
}

int bto_stats(bto_ctx* c, bto_stats_t* out, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (!out) return fail(c, BTO_EINVAL, "null output");
    std::memset(out, 0, sizeof *out);
    out->n_seeds = c->n_seeds;
    out->steps_done = c->steps_done;
    if (!c->seeded) return BTO_OK;
    hipStream_t s = (hipStream_t)stream;
    uint32_t cnt[NSEG * CSTRIDE];
    unsigned long long psv[NSEG * PSTRIDE];
    hipError_t e = hipMemcpyAsync(cnt, c->counts + NSEG * CSTRIDE * c->slot, sizeof cnt, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(psv, c->psteps, sizeof psv, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "stats readback");
    int64_t live = 0;
    for (int x = 0; x < NSEG; ++x) live += cnt[x * CSTRIDE];
    unsigned long long ps = 0;
    for (int x = 0; x < NSEG; ++x) ps += psv[x * PSTRIDE];
    out->n_live = live;
    out->particle_steps = (int64_t)ps;
    return BTO_OK;
}

}  // extern "C"

// The adjoint launch over checkpoint segments sg_first .. sg_last with the
// grids, steps and gradient grids of steps f_base .. f_base + n_local (arguments
// validated by the callers).  Checkpoints: recomputed into the scratch (whole
// interval only) or the ones the advection recorded (use_ck).
static int adjoint_run(bto_ctx* c, const void* const* d_fields, const double* times, int32_t n_local, int32_t N,
                       int32_t dtype, int mode, bool use_ck, const float* d_cot_end, int32_t n_cot,
                       float* d_grad_seed, float* const* d_grad_fields, uint8_t* d_status, int32_t ckpt_every,
                       int32_t sg_first, int32_t sg_last, int32_t f_base, float* lam, uint8_t* drop,
                       hipStream_t s) {
    const int K = ckpt_every < N ? ckpt_every : N;
    const int nseg = (N + K - 1) / K;
    const size_t P = (size_t)c->n_seeds;
    const size_t tab =
        ((size_t)(n_local + 1) * 2 * sizeof(void*) + (size_t)n_local * sizeof(double) + 255) & ~(size_t)255;
    // checkpoint slots live in the scratch unless they were recorded
    const size_t need = tab + P * 3 * sizeof(double) * ((use_ck ? 0 : (size_t)nseg) + (size_t)K);
    hipError_t e;
    if (need > c->adj_bytes) {
        if (c->adj_scratch) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(c, e, "adjoint scratch sync");
            (void)hipFree(c->adj_scratch);
            c->adj_scratch = nullptr;
            c->adj_bytes = 0;
        }
        if (hipMalloc(&c->adj_scratch, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, BTO_ENOMEM, "adjoint scratch of %zu bytes", need);
        }
        c->adj_bytes = need;
    }
    char* base = static_cast<char*>(c->adj_scratch);
    std::vector<char> host(tab, 0);
    const void** hf = reinterpret_cast<const void**>(host.data());
    void** hg = reinterpret_cast<void**>(host.data() + (size_t)(n_local + 1) * sizeof(void*));
    double* hh = reinterpret_cast<double*>(host.data() + (size_t)(n_local + 1) * 2 * sizeof(void*));
    for (int32_t q = 0; q <= n_local; ++q) {
        hf[q] = d_fields[q];
        hg[q] = d_grad_fields ? (void*)d_grad_fields[q] : nullptr;
    }
    for (int32_t q = 0; q < n_local; ++q) hh[q] = times[q + 1] - times[q];
    e = hipMemcpyAsync(base, host.data(), tab, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint tables upload");
    AdjointArgs a{};
    a.f = reinterpret_cast<const char* const*>(base);
    a.grad_f = d_grad_fields ? reinterpret_cast<float* const*>(base + (size_t)(n_local + 1) * sizeof(void*)) : nullptr;
    a.h = reinterpret_cast<const double*>(base + (size_t)(n_local + 1) * 2 * sizeof(void*));
    a.g = c->geom;
    a.N = N;
    a.k = K;
    a.ncot = n_cot;
    a.P = (int64_t)P;
    a.seed_xyz = c->seed_xyz;
    for (int d = 0; d < 3; ++d) {
        a.origin[d] = c->blk.origin[d];
        a.sp[d] = c->blk.spacing[d];
    }
    a.cot = d_cot_end;
    a.grad_seed = d_grad_seed;
    if (use_ck) {
        a.ckpt = c->ck_rec;
        a.ck_stride = c->cap * 3;
        a.buf = reinterpret_cast<double*>(base + tab);
        a.rec_meta = c->rec_meta;
    } else {
        a.ckpt = reinterpret_cast<double*>(base + tab);
        a.ck_stride = (int64_t)P * 3;
        a.buf = a.ckpt + P * 3 * (size_t)nseg;
        a.rec_meta = nullptr;
    }
    a.status_out = d_status;
    a.sg_first = sg_first;
    a.sg_last = sg_last;
    a.f_base = f_base;
    a.lam = lam;
    a.drop = drop;
    // grid gradients: records for the sorted reduction, unless the key does not fit
    a.grec = GradRec{};
    uint64_t* key_out = nullptr;
    uint32_t* idx_out = nullptr;
    uint32_t* bounds = nullptr;
    void* sort_temp = nullptr;
    size_t sort_bytes = 0;
    uint64_t n_slots = 0;
    bool grads_distinct = true;  // the colour passes store without atomics: one buffer per grid
    if (d_grad_fields) {
        std::vector<const void*> gp(d_grad_fields, d_grad_fields + n_local + 1);
        std::sort(gp.begin(), gp.end());
        grads_distinct = std::adjacent_find(gp.begin(), gp.end()) == gp.end();
    }
    if (d_grad_fields && !c->grad_atomics && grads_distinct) {
        auto bits_for = [](uint64_t v) {  // bits to hold 0 .. v
            int b = 1;
            while (b < 64 && (v >> b) != 0) ++b;
            return b;
        };
        const uint64_t npts = (uint64_t)c->geom.n[0] * (uint64_t)c->geom.n[1] * (uint64_t)c->geom.n[2];
        GradRec r{};
        r.P = (uint32_t)P;
        r.cell_bits = bits_for(npts - 1);
        r.level_bits = bits_for((uint64_t)n_local);
        const int kb = r.cell_bits + r.level_bits + 3;
        const uint64_t per = 2 * sizeof(uint64_t) + 2 * sizeof(uint32_t) + 24 * sizeof(float);
        const uint64_t max_slots = ((uint64_t)4 << 30) / per;  // at most ~4 GiB of records
        // about one flush per seed and level when particles keep their cells, plus cell changes
        uint64_t ps = 2 * (uint64_t)(n_local + 1) + 2;
        if (ps * P > max_slots) ps = max_slots / P;
        if (kb + 1 <= 64 && ps >= 1) {
            r.per_seed = (uint32_t)ps;
            n_slots = ((uint64_t)P * ps + 15) & ~(uint64_t)15;  // keeps every array 128-byte aligned
            sort_bytes = grad_sort_temp_bytes(n_slots, kb + 1);
            const size_t temp_r = (sort_bytes + 255) & ~(size_t)255;
            const size_t need_r = temp_r + (size_t)n_slots * per + 256;
            if (need_r > c->grec_bytes) {
                if (c->grec_buf) {
                    e = hipStreamSynchronize(s);
                    if (e != hipSuccess) return hip_fail(c, e, "gradient records sync");
                    (void)hipFree(c->grec_buf);
                    c->grec_buf = nullptr;
                    c->grec_bytes = 0;
                }
                if (hipMalloc(&c->grec_buf, need_r) != hipSuccess) {
                    (void)hipGetLastError();
                    c->grec_buf = nullptr;
                } else {
                    c->grec_bytes = need_r;
                }
            }
            if (c->grec_buf && sort_bytes > 0) {
                // [sort temp | keys | sorted keys | indices | sorted indices | values | colour bounds]
                char* q = static_cast<char*>(c->grec_buf);
                sort_temp = q;
                r.key = reinterpret_cast<uint64_t*>(q + temp_r);
                key_out = r.key + n_slots;
                r.idx = reinterpret_cast<uint32_t*>(key_out + n_slots);
                idx_out = r.idx + n_slots;
                r.val = reinterpret_cast<float*>(idx_out + n_slots);
                bounds = reinterpret_cast<uint32_t*>(r.val + 24 * (size_t)n_slots);
                e = launch_grad_clear(r, n_slots, s);
                if (e != hipSuccess) return hip_fail(c, e, "gradient record clear");
                a.grec = r;
            }
        }
    }
    e = launch_adjoint(a, dtype, mode, s);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint launch");
    if (a.grec.key) {
        e = launch_grad_reduce(a.grec, n_slots, key_out, idx_out, bounds, sort_temp, sort_bytes, a.grad_f, c->geom, s);
        if (e != hipSuccess) return hip_fail(c, e, "gradient reduction");
    }
    return BTO_OK;
}

extern "C" {

int bto_adjoint_interval(bto_ctx* c, const void* const* d_fields, const double* times, int32_t n_steps,
                         int32_t dtype, int32_t flags, const float* d_cot_end, int32_t n_cot, float* d_grad_seed,
                         float* const* d_grad_fields, uint8_t* d_status, int32_t ckpt_every, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (!d_fields || !times) return fail(c, BTO_EINVAL, "null field or time array");
    if (n_steps <= 0) return fail(c, BTO_EINVAL, "n_steps must be > 0 (got %d)", n_steps);
    if (dtype < BTO_F32 || dtype > BTO_BF16) return fail(c, BTO_EINVAL, "unknown dtype %d", dtype);
    const int mode = flags & ~BTO_RECORD_CKPT;
    const bool use_ck = (flags & BTO_RECORD_CKPT) != 0;
    if (mode != BTO_TIME_LINEAR && mode != BTO_TIME_FROZEN) return fail(c, BTO_EINVAL, "unknown flags %d", flags);
    if (n_cot != 1 && n_cot != 3) return fail(c, BTO_EINVAL, "n_cot must be 1 or 3 (got %d)", n_cot);
    if (d_grad_fields && n_cot != 1) return fail(c, BTO_EINVAL, "grid gradients need n_cot == 1");
    if (ckpt_every < 1) return fail(c, BTO_EINVAL, "ckpt_every must be >= 1");
    for (int32_t q = 0; q <= n_steps; ++q) {
        if (!d_fields[q]) return fail(c, BTO_EINVAL, "field pointer %d is null", q);
        if (d_grad_fields && !d_grad_fields[q]) return fail(c, BTO_EINVAL, "grad field pointer %d is null", q);
    }
    for (int32_t q = 0; q < n_steps; ++q)
        if (!(times[q + 1] > times[q]) || !std::isfinite(times[q + 1]) || !std::isfinite(times[q]))
            return fail(c, BTO_EINVAL, "times must be finite and strictly increasing (index %d)", q);
    if (!c->seeded) return fail(c, BTO_ESTATE, "adjoint called before seeding");
    // per-seed arrays may be null only when there are no seeds
    if (c->n_seeds > 0 && (!d_cot_end || !d_grad_seed)) return fail(c, BTO_EINVAL, "null cotangent or gradient array");
    if (use_ck) {
        if (!c->ck_ok || c->ck_k == 0)
            return fail(c, BTO_ESTATE, "no complete checkpoint record (advect every call of the interval with BTO_RECORD_CKPT)");
        if (n_steps != c->steps_done)
            return fail(c, BTO_EINVAL, "n_steps %d differs from the %d steps advected", n_steps, c->steps_done);
        if (ckpt_every != c->ck_k)
            return fail(c, BTO_EINVAL, "ckpt_every %d differs from the recorded spacing %d", ckpt_every, c->ck_k);
    }
    if (c->n_seeds == 0) return BTO_OK;
    const int K = ckpt_every < n_steps ? ckpt_every : n_steps;
    const int nseg = (n_steps + K - 1) / K;
    c->seg_next = -1;  // a whole-interval adjoint ends any segment sequence
    return adjoint_run(c, d_fields, times, n_steps, n_steps, dtype, mode, use_ck, d_cot_end, n_cot, d_grad_seed,
                       d_grad_fields, d_status, ckpt_every, nseg - 1, 0, 0, nullptr, nullptr, (hipStream_t)stream);
}

int bto_adjoint_segment(bto_ctx* c, int32_t segment, const void* const* d_fields, const double* times,
                        int32_t dtype, int32_t flags, const float* d_cot_end, int32_t n_cot, float* d_grad_seed,
                        float* const* d_grad_fields, uint8_t* d_status, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (!d_fields || !times) return fail(c, BTO_EINVAL, "null field or time array");
    if (dtype < BTO_F32 || dtype > BTO_BF16) return fail(c, BTO_EINVAL, "unknown dtype %d", dtype);
    const int mode = flags & ~BTO_RECORD_CKPT;
    if (mode != BTO_TIME_LINEAR && mode != BTO_TIME_FROZEN) return fail(c, BTO_EINVAL, "unknown flags %d", flags);
    if (n_cot != 1 && n_cot != 3) return fail(c, BTO_EINVAL, "n_cot must be 1 or 3 (got %d)", n_cot);
    if (d_grad_fields && n_cot != 1) return fail(c, BTO_EINVAL, "grid gradients need n_cot == 1");
    if (!c->seeded) return fail(c, BTO_ESTATE, "adjoint called before seeding");
    if (!c->ck_ok || c->ck_k == 0 || c->steps_done == 0)
        return fail(c, BTO_ESTATE, "no complete checkpoint record (advect every call of the interval with BTO_RECORD_CKPT)");
    const int N = c->steps_done;
    const int K = c->ck_k < N ? c->ck_k : N;
    const int nseg = (N + K - 1) / K;
    if (segment < 0 || segment >= nseg) return fail(c, BTO_EINVAL, "segment %d outside 0..%d", segment, nseg - 1);
    const bool first = segment == nseg - 1;
    if (first) {
        if (!d_cot_end && c->n_seeds > 0) return fail(c, BTO_EINVAL, "the last segment needs the end cotangents");
    } else if (c->seg_next != segment || c->seg_ncot != n_cot) {
        return fail(c, BTO_ESTATE, "segments must be swept from %d down to 0 with one n_cot (expected %d)", nseg - 1,
                    c->seg_next);
    }
    if (segment == 0 && !d_grad_seed && c->n_seeds > 0)
        return fail(c, BTO_EINVAL, "segment 0 needs the seed-gradient output");
    const int n0 = segment * K, n1 = n0 + K < N ? n0 + K : N;
    const int nl = n1 - n0;
    for (int32_t q = 0; q <= nl; ++q) {
        if (!d_fields[q]) return fail(c, BTO_EINVAL, "field pointer %d is null", q);
        if (d_grad_fields && !d_grad_fields[q]) return fail(c, BTO_EINVAL, "grad field pointer %d is null", q);
    }
    for (int32_t q = 0; q < nl; ++q)
        if (!(times[q + 1] > times[q]) || !std::isfinite(times[q + 1]) || !std::isfinite(times[q]))
            return fail(c, BTO_EINVAL, "times must be finite and strictly increasing (index %d)", q);
    hipStream_t s = (hipStream_t)stream;
    if (c->n_seeds == 0) {
        c->seg_next = segment - 1;
        c->seg_ncot = n_cot;
        return BTO_OK;
    }
    // cotangents carried between the calls and the dropped-seed marks
    const size_t lam_bytes = ((size_t)c->n_seeds * 3 * 3 * sizeof(float) + 255) & ~(size_t)255;
    const size_t need = lam_bytes + (((size_t)c->n_seeds + 3) & ~(size_t)3);
    if (need > c->seg_bytes) {
        if (c->seg_buf) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(c, e, "segment state sync");
            (void)hipFree(c->seg_buf);
            c->seg_buf = nullptr;
            c->seg_bytes = 0;
        }
        if (hipMalloc(&c->seg_buf, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, BTO_ENOMEM, "segment state of %zu bytes", need);
        }
        c->seg_bytes = need;
    }
    float* lam = static_cast<float*>(c->seg_buf);
    uint8_t* drop = reinterpret_cast<uint8_t*>(static_cast<char*>(c->seg_buf) + lam_bytes);
    if (first) {
        hipError_t e = launch_tile_fill(reinterpret_cast<uint32_t*>(drop), ((size_t)c->n_seeds + 3) / 4, s);
        if (e != hipSuccess) return hip_fail(c, e, "segment state clear");
    }
    rc = adjoint_run(c, d_fields, times, nl, N, dtype, mode, true, d_cot_end, n_cot, d_grad_seed, d_grad_fields,
                     d_status, c->ck_k, segment, segment, n0, lam, drop, s);
    if (rc) return rc;
    c->seg_next = segment - 1;
    c->seg_ncot = n_cot;
    return BTO_OK;
}

int bto_ftle(bto_ctx* c, const float* d_jac, int64_t n, double T, float* d_out, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!d_jac || !d_out))) return fail(c, BTO_EINVAL, "null argument or negative count");
    if (!(T != 0.0) || !std::isfinite(T)) return fail(c, BTO_EINVAL, "T must be finite and non-zero");
    hipError_t e = launch_ftle(d_jac, n, 1.0 / std::fabs(T), d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "ftle launch");
    return BTO_OK;
}

int bto_touched_points(bto_ctx* c, const void* const* d_fields, const double* times, int32_t n_steps,
                       int32_t dtype, int32_t flags, unsigned long long* d_counts, void* stream) {
    int rc = begin(c);
    if (rc) return rc;
    if (!d_fields || !times || !d_counts) return fail(c, BTO_EINVAL, "null argument");
    if (n_steps <= 0) return fail(c, BTO_EINVAL, "n_steps must be > 0 (got %d)", n_steps);
    if (dtype < BTO_F32 || dtype > BTO_BF16) return fail(c, BTO_EINVAL, "unknown dtype %d", dtype);
    const int base_mode = flags & ~BTO_SAMPLE_FP64;
    if (base_mode != BTO_TIME_LINEAR && base_mode != BTO_TIME_FROZEN)
        return fail(c, BTO_EINVAL, "unknown flags %d", flags);
    const int mode = (base_mode == BTO_TIME_FROZEN ? MODE_FROZEN : MODE_LINEAR) |
                     ((flags & BTO_SAMPLE_FP64) ? MODE_FP64 : 0);
    for (int32_t q = 0; q <= n_steps; ++q)
        if (!d_fields[q]) return fail(c, BTO_EINVAL, "field pointer %d is null", q);
    for (int32_t q = 0; q < n_steps; ++q)
        if (!(times[q + 1] > times[q]) || !std::isfinite(times[q + 1]) || !std::isfinite(times[q]))
            return fail(c, BTO_EINVAL, "times must be finite and strictly increasing (index %d)", q);
    if (!c->seeded) return fail(c, BTO_ESTATE, "touched points counted before seeding");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_touch_zero(d_counts, (size_t)n_steps * 3, s);
    if (e != hipSuccess) return hip_fail(c, e, "touched points: clear counters");
    const int64_t P = c->n_seeds;
    if (P == 0) return BTO_OK;
    const size_t npts = (size_t)c->geom.n[0] * (size_t)c->geom.n[1] * (size_t)c->geom.n[2];
    const size_t words = (npts + 31) / 32;
    const size_t xb = ((size_t)P * 3 * sizeof(double) + 255) & ~(size_t)255;
    const size_t ab = ((size_t)P + 255) & ~(size_t)255;
    const size_t bb = ((words * sizeof(uint32_t)) + 255) & ~(size_t)255;
    char* buf = nullptr;
    e = hipMalloc(&buf, xb + ab + 2 * bb);
    if (e != hipSuccess) return hip_fail(c, e, "touched points: scratch allocation");
    TouchArgs a{};
    a.g = c->geom;
    a.P = P;
    a.seed_xyz = c->seed_xyz;
    for (int d = 0; d < 3; ++d) a.origin[d] = c->blk.origin[d];
    a.x = reinterpret_cast<double*>(buf);
    a.alive = reinterpret_cast<uint8_t*>(buf + xb);
    a.bits0 = reinterpret_cast<uint32_t*>(buf + xb + ab);
    a.bits1 = reinterpret_cast<uint32_t*>(buf + xb + ab + bb);
    e = launch_tile_fill(a.bits0, 2 * bb / sizeof(uint32_t), s);
    if (e == hipSuccess) e = launch_touch_init(a, s);
    for (int32_t n = 0; n < n_steps && e == hipSuccess; ++n) {
        a.f0 = static_cast<const char*>(d_fields[n]);
        a.f1 = static_cast<const char*>(d_fields[n + 1]);
        a.h = times[n + 1] - times[n];
        a.out = d_counts + 3 * (size_t)n;
        e = launch_touch_step(a, dtype, mode, s);
        if (e == hipSuccess) e = launch_touch_count(a.bits0, words, a.out, s);
        if (e == hipSuccess) e = launch_touch_count(a.bits1, words, a.out + 1, s);
    }
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(c, e, "touched points launch");
    if (e2 != hipSuccess) return hip_fail(c, e2, "touched points");
    return BTO_OK;
}

int bto_set_tuning(bto_ctx* c, const bto_tuning* t) {
    if (!c) return BTO_EINVAL;
    if (!t) return fail(c, BTO_EINVAL, "null tuning");
    if (t->steps_per_launch < 1 || t->steps_per_launch > KMAX)
        return fail(c, BTO_EINVAL, "steps_per_launch must be in 1..%d", KMAX);
    if (t->rebin_every < 0) return fail(c, BTO_EINVAL, "rebin_every must be >= 0");
    if (t->blocks_per_cu < 0) return fail(c, BTO_EINVAL, "blocks_per_cu must be >= 0");
    if (t->lanes_per_particle != 1 && t->lanes_per_particle != 2)
        return fail(c, BTO_EINVAL, "lanes_per_particle must be 1 or 2");
    if (t->ckpt_every < 1) return fail(c, BTO_EINVAL, "ckpt_every must be >= 1");
    if (t->tiles < 0 || t->tiles > 2) return fail(c, BTO_EINVAL, "tiles must be 0, 1 or 2");
    c->tiles = t->tiles;
    c->lanes_per_particle = t->lanes_per_particle;
    c->ckpt_every = t->ckpt_every;
    c->steps_per_launch = t->steps_per_launch;
    c->rebin_every = t->rebin_every;
    c->blocks_per_cu_cap = t->blocks_per_cu;
    return BTO_OK;
}

int bto_get_tuning(const bto_ctx* c, bto_tuning* t) {
    if (!c || !t) return BTO_EINVAL;
    t->steps_per_launch = c->steps_per_launch;
    t->rebin_every = c->rebin_every;
    t->blocks_per_cu = c->blocks_per_cu_cap;
    t->lanes_per_particle = c->lanes_per_particle;
    t->ckpt_every = c->ckpt_every;
    t->tiles = c->tiles;
    return BTO_OK;
}

}  // extern "C"
