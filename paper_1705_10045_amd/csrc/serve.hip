// Serving pool (include/lbm_mi355x.h, lbm_pool_*): many independent D3Q19 FP32 simulations
// resident in one HBM arena and advanced together.
//
// Device side: a slot table (one SlotDesc per slot) and a flat work list of tiles: slot s owns
// the global tile indices [tile_begin, tile_begin + ntiles).  One step of every active slot is
// one launch of k_pool_step per kind of request present (periodic or with walls or gravity,
// BGK or MRT) over a fixed grid that walks the work list, followed by k_pool_advance, which
// flips each slot's buffer parity, counts its steps down and retires it when done or when its
// error word is set.  steps_per_run such steps are captured into a HIP graph, one graph per set
// of kinds, each captured once on first use; admissions and collections only rewrite the slot
// table between replays.
//
// Host side: first-fit allocation of slot buffers inside one arena allocated at creation
// (admission by footprint never calls the allocator of the runtime), tickets, and the
// completion bookkeeping read back after each replay.
//
// Overlap: replays run on the pool's stream; admissions (upload, initial state) and
// collections (moments, download) run on a second stream of the same (default) priority.  A
// replay may be left in flight (lbm_pool_run_async): the slot table travels through pinned
// host buffers, the next call waits for the replay and its readback, and only then rewrites
// the device table.  Meanwhile admissions touch only free arena blocks and slots that the
// replay in flight does not advance, and collections only finished (inactive) slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/lbm_mi355x.h"
#include "kernels.hpp"
#include "sim.hpp"
#include "step_kernel.hpp"

namespace lbm {

constexpr int kPoolTX = 32, kPoolTY = 16;  // tile of the FP32 D3Q19 step, one moment slot per
constexpr int kPoolThreads = 768;          // thread, LDS stash as in the single-simulation launch
constexpr int kPoolChunk = 16;             // z planes per tile: uniform tile work in the mix
constexpr int kPoolGrid = 256;             // persistent workgroups: one per compute unit
constexpr int kPoolMaxEdge = 128;

struct SlotDesc {
    float* buf[2];
    StepGeom geom;
    Phys phys;
    int tile_begin;
    int ntiles;
    int parity;        // buf[parity] holds the current state
    int active;        // 1 while steps remain and no error was flagged
    int kind;          // launch that serves the slot: kind_of(ext, mrt), ext 0 periodic, 1 walls
                       // or gravity (kExtWalls), 2 a tabulated EOS (kExtTable), mrt the MRT
                       // collision
    const double* eos_p;     // tabulated EOS: the request's copy of the table in the arena
    const double* eos_coex;
    long long remaining;
    long long steps_done;
};

struct PoolHeader {
    int nslots;        // slots [0, nslots) are searched by the step kernel
    int total_tiles;
    int kind_tiles[6]; // tiles of the requests of each kind (SlotDesc::kind)
};

constexpr int kPoolKinds = 6;
__host__ __device__ constexpr int kind_of(int ext, bool mrt) { return ext + (mrt ? 3 : 0); }

// One launch per kind of request (EXTK: kExtNone for periodic boxes, kExtWalls with walls or
// gravity, kExtTable with a tabulated EOS; MRT: the MRT collision instead of BGK), each skipping
// the other kinds' tiles, so the common periodic BGK step keeps the registers of its own
// instantiation.
template <int EXTK, bool MRT>
__global__ void __launch_bounds__(kPoolThreads)
k_pool_step(const SlotDesc* __restrict__ slots, const PoolHeader* __restrict__ hdr,
            const double* __restrict__ table, double s0, double inv_ds, int* __restrict__ errs)
{
    constexpr int kKind = kind_of(EXTK == kExtNone ? 0 : (EXTK == kExtWalls ? 1 : 2), MRT);
    if (hdr->kind_tiles[kKind] == 0) return;
    __shared__ TileLds<19, float, float, kPoolTX, kPoolTY, true> lds;
    const int total = hdr->total_tiles;
    const int nslots = hdr->nslots;
    // XCD-aware order: each XCD walks contiguous runs of the work list, so neighbouring tiles
    // of one request share that XCD's L2
    for (int t = xcd_logical_block(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
        // slot owning tile t: last slot with tile_begin <= t (binary search, workgroup-uniform)
        int lo = 0, hi = nslots - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (slots[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        const SlotDesc& d = slots[lo];
        if (!d.active || t - d.tile_begin >= d.ntiles || d.kind != kKind) continue;
        // workgroup-uniform copies, so the stores of the step cannot alias them
        const StepGeom g = d.geom;
        const Phys ph = d.phys;
        const int parity = d.parity;
        const int local = t - d.tile_begin;
        const float* src = d.buf[parity];
        float* dst = d.buf[1 - parity];
        StepAux aux;
        aux.maxwell = table;
        aux.tab_s0 = s0;
        aux.tab_inv_ds = inv_ds;
        aux.err = errs + lo;
        aux.eos_p = d.eos_p;
        aux.eos_coex = d.eos_coex;
        aux.partials = nullptr;
        // each request's own collision: MRT, or BGK with tau = 1 (with the density prefetch)
        // or general; all share the workgroup's LDS
        if constexpr (MRT)
            step_tile<19, float, float, kPoolTX, kPoolTY, kPoolThreads, false, kAddrBuf, kMrt, true, EXTK>(
                lds, src, dst, g, ph, aux, local);
        else if (ph.omega == 1.0)
            step_tile<19, float, float, kPoolTX, kPoolTY, kPoolThreads, true, kAddrBuf, kTauOne, true, EXTK>(
                lds, src, dst, g, ph, aux, local);
        else
            step_tile<19, float, float, kPoolTX, kPoolTY, kPoolThreads, false, kAddrBuf, kTauAny, true, EXTK>(
                lds, src, dst, g, ph, aux, local);
    }
}

__global__ void k_pool_advance(SlotDesc* __restrict__ slots, const PoolHeader* __restrict__ hdr,
                               const int* __restrict__ errs)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= hdr->nslots) return;
    SlotDesc& d = slots[s];
    if (!d.active) return;
    d.parity ^= 1;
    d.steps_done += 1;
    d.remaining -= 1;
    if (d.remaining <= 0 || errs[s] != 0) d.active = 0;
}

}  // namespace lbm

using namespace lbm;

struct PoolSlot {
    bool used = false;
    long long ticket = -1;
    size_t offset = 0, bytes = 0;
    lbm_params params;
    long long nsteps = 0;
};

struct lbm_pool {
    int device = 0;
    hipStream_t stream = nullptr;            // replays
    bool own_stream = false;
    hipStream_t side = nullptr;              // admissions and collections
    SlotDesc* h_up = nullptr;                // pinned: the table as uploaded before a replay
    PoolHeader* h_hdr = nullptr;             // pinned: its header
    SlotDesc* h_rb = nullptr;                // pinned: the table read back after a replay
    int* h_errs = nullptr;                   // pinned: the error words read back after a replay
    hipEvent_t done = nullptr;               // end of the replay in flight and of its readback
    bool in_flight = false;
    std::vector<long long> launched;         // ticket in each slot when that replay was launched
    size_t budget = 0, in_use = 0;
    char* arena = nullptr;
    std::map<size_t, size_t> free_blocks;   // offset -> size, coalesced
    int max_slots = 0, steps_per_run = 1;
    std::vector<PoolSlot> slots;
    std::vector<SlotDesc> table;             // host mirror of the device slot table
    SlotDesc* d_slots = nullptr;
    PoolHeader* d_hdr = nullptr;
    int* d_errs = nullptr;
    double* d_table = nullptr;
    double tab_s0 = 0, tab_inv_ds = 0;
    double* d_staging = nullptr;             // initial fields of a request (5 n doubles)
    double* d_scratch = nullptr;             // moment scratch (10 n doubles)
    double* d_red = nullptr;                 // reduction partials (kPoolRedBlocks x 5)
    double* d_totals = nullptr;              // per slot: totals at admission, then at the end
    // one graph per set of request kinds present (bit k: a slot of SlotDesc::kind k is
    // active), captured on first use, so a replay launches only the kinds it serves
    hipGraph_t graph[1 << kPoolKinds] = {};
    hipGraphExec_t exec[1 << kPoolKinds] = {};
    int kinds = 0;                           // kind set of the uploaded table
    bool dirty = true;
    long long next_ticket = 1;
    std::map<long long, int> ticket_slot;
    std::map<long long, lbm_status> finished;  // collected-or-not results by ticket
};

namespace {

const size_t kAlign = 256;
// blocks of the per-slot reductions (a pool state has at most kPoolMaxEdge^3 nodes)
const int kPoolRedBlocks = 1024;

// FP64 totals of a slot's populations (as lbm_reduce) into out[0..4], on the side stream
hipError_t slot_reduce(lbm_pool* p, const SlotDesc& d, const lbm_params& prm, int parity, double* out)
{
    const long long n = (long long)prm.nx * prm.ny * prm.nz;
    int blocks = reduce_blocks(n);
    if (blocks > kPoolRedBlocks) blocks = kPoolRedBlocks;
    return launch_reduce(19, 4, d.buf[parity], plane_elements(prm), d.geom.plane, p->d_red, blocks, out, p->side);
}

bool arena_alloc(lbm_pool* p, size_t bytes, size_t& off)
{
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = p->free_blocks.begin(); it != p->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            off = it->first;
            const size_t rest = it->second - bytes;
            p->free_blocks.erase(it);
            if (rest) p->free_blocks[off + bytes] = rest;
            p->in_use += bytes;
            return true;
        }
    }
    return false;
}

void arena_free(lbm_pool* p, size_t off, size_t bytes)
{
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    p->in_use -= bytes;
    auto it = p->free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != p->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        p->free_blocks.erase(nx);
    }
    if (it != p->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            p->free_blocks.erase(it);
        }
    }
}

StepGeom pool_geometry(const lbm_params& p)
{
    StepGeom g;
    g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
    g.pitch = row_pitch(p.nx, 4);
    g.plane = padded_plane(plane_elements(p));
    g.ntx = (p.nx + kPoolTX - 1) / kPoolTX;
    g.nty = (p.ny + kPoolTY - 1) / kPoolTY;
    g.chunk = kPoolChunk < p.nz ? kPoolChunk : p.nz;
    g.nchunks = (p.nz + g.chunk - 1) / g.chunk;
    g.resident = 0;
    return g;
}

// Rebuild the work list (tile prefix over slots in index order) and upload the table.
lbm_status upload_table(lbm_pool* p)
{
    int total = 0, nslots = 0, kind_tiles[kPoolKinds] = {}, kinds = 0;
    for (int s = 0; s < p->max_slots; ++s) {
        SlotDesc& d = p->table[s];
        d.tile_begin = total;
        if (p->slots[s].used && d.active) {
            d.ntiles = d.geom.ntx * d.geom.nty * d.geom.nchunks;
            total += d.ntiles;
            kind_tiles[d.kind] += d.ntiles;
            kinds |= 1 << d.kind;
            nslots = s + 1;
        } else {
            d.ntiles = 0;
        }
    }
    // staged in pinned memory: the copies are truly asynchronous, and the host mirror may change
    // (admissions) before they have run; the pinned copy is rewritten only after the next
    // replay, which the stream orders after these copies, has completed
    p->h_hdr->nslots = nslots;
    p->h_hdr->total_tiles = total;
    for (int k = 0; k < kPoolKinds; ++k) p->h_hdr->kind_tiles[k] = kind_tiles[k];
    memcpy(p->h_up, p->table.data(), sizeof(SlotDesc) * p->max_slots);
    hipError_t e = hipMemcpyAsync(p->d_slots, p->h_up, sizeof(SlotDesc) * p->max_slots,
                                  hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_hdr, p->h_hdr, sizeof(PoolHeader), hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pool table upload");
    p->kinds = kinds;
    p->dirty = false;
    return LBM_OK;
}

// Captures steps_per_run steps of the kinds in `kinds` (one launch per kind, then the advance)
// into the graph of that kind set.  Called with no replay in flight on the pool's stream.
lbm_status capture_graph(lbm_pool* p, int kinds)
{
    hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture begin");
    const int adv_blocks = (p->max_slots + 255) / 256;
    for (int i = 0; i < p->steps_per_run; ++i) {
#define LBM_POOL_LAUNCH(EXTK, MRT)                                                                       \
    if (kinds & (1 << kind_of(EXTK == kExtNone ? 0 : (EXTK == kExtWalls ? 1 : 2), MRT)))                  \
        hipLaunchKernelGGL((k_pool_step<EXTK, MRT>), dim3(kPoolGrid), dim3(kPoolThreads), 0, p->stream,      \
                           p->d_slots, p->d_hdr, p->d_table, p->tab_s0, p->tab_inv_ds, p->d_errs);
        LBM_POOL_LAUNCH(kExtNone, false)
        LBM_POOL_LAUNCH(kExtWalls, false)
        LBM_POOL_LAUNCH(kExtTable, false)
        LBM_POOL_LAUNCH(kExtNone, true)
        LBM_POOL_LAUNCH(kExtWalls, true)
        LBM_POOL_LAUNCH(kExtTable, true)
#undef LBM_POOL_LAUNCH
        hipLaunchKernelGGL(k_pool_advance, dim3(adv_blocks), dim3(256), 0, p->stream, p->d_slots,
                           p->d_hdr, p->d_errs);
    }
    e = hipStreamEndCapture(p->stream, &p->graph[kinds]);
    if (e != hipSuccess) return hip_fail(e, "graph capture end");
    e = hipGraphInstantiate(&p->exec[kinds], p->graph[kinds], nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    return LBM_OK;
}

// Waits for the replay in flight and its readback, then takes over the new state of every slot
// that the replay advanced (slots admitted or collected meanwhile keep their host state) and
// records the requests that finished or left the EOS domain.
lbm_status finish_replay(lbm_pool* p)
{
    if (!p->in_flight) return LBM_OK;
    p->in_flight = false;
    const hipError_t e = hipEventSynchronize(p->done);
    if (e != hipSuccess) return hip_fail(e, "pool replay");
    for (int s = 0; s < p->max_slots; ++s) {
        PoolSlot& ps = p->slots[s];
        if (!ps.used || ps.ticket != p->launched[s]) continue;
        SlotDesc& d = p->table[s];
        const SlotDesc& r = p->h_rb[s];
        d.parity = r.parity;
        d.active = r.active;
        d.remaining = r.remaining;
        d.steps_done = r.steps_done;
        if (!p->finished.count(ps.ticket)) {
            if (p->h_errs[s]) p->finished[ps.ticket] = LBM_EUNSTABLE;
            else if (!r.active) p->finished[ps.ticket] = LBM_OK;
        }
        // a slot that finished no longer contributes tiles: rebuild the work list
        if (!r.active) p->dirty = true;
    }
    return LBM_OK;
}

// Waits for the previous replay (if any), refreshes the table and enqueues the next replay
// with the readback of its table behind it.
lbm_status launch_replay(lbm_pool* p)
{
    lbm_status st = finish_replay(p);
    if (st != LBM_OK) return st;
    if (p->dirty) {
        st = upload_table(p);
        if (st != LBM_OK) return st;
    }
    bool any = false;
    for (int s = 0; s < p->max_slots; ++s) any = any || (p->slots[s].used && p->table[s].active);
    if (!any) return LBM_OK;
    if (!p->exec[p->kinds]) {
        st = capture_graph(p, p->kinds);
        if (st != LBM_OK) return st;
    }
    for (int s = 0; s < p->max_slots; ++s) p->launched[s] = p->slots[s].used ? p->slots[s].ticket : -1;
    hipError_t e = hipGraphLaunch(p->exec[p->kinds], p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_rb, p->d_slots, sizeof(SlotDesc) * p->max_slots, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_errs, p->d_errs, sizeof(int) * p->max_slots, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipEventRecord(p->done, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pool replay launch");
    p->in_flight = true;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_pool_create(size_t hbm_budget_bytes, int max_slots, int steps_per_run, void* stream,
                           lbm_pool** out)
{
    clear_error();
    if (!out) { set_error("out is NULL"); return LBM_EINVAL; }
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096 || steps_per_run < 1 || steps_per_run > 1000 ||
        hbm_budget_bytes < ((size_t)1 << 20)) {
        set_error("pool needs 1 <= max_slots <= 4096, 1 <= steps_per_run <= 1000, budget >= 1 MiB");
        return LBM_EINVAL;
    }
    double rv, rl;
    if (!host_band_limits(0.8, rv, rl)) { set_error("Maxwell table unavailable"); return LBM_EDEVICE; }
    lbm_pool* p = new lbm_pool();
    if (hipError_t e = hipGetDevice(&p->device); e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    if (stream) {
        p->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete p; return hip_fail(e, "hipStreamCreate"); }
        p->own_stream = true;
    }
    p->budget = hbm_budget_bytes / kAlign * kAlign;
    p->max_slots = max_slots;
    p->steps_per_run = steps_per_run;
    p->slots.assign(max_slots, PoolSlot());
    p->table.assign(max_slots, SlotDesc());
    memset(p->table.data(), 0, sizeof(SlotDesc) * max_slots);
    p->launched.assign(max_slots, -1);
    const long long nmax = (long long)kPoolMaxEdge * kPoolMaxEdge * kPoolMaxEdge;
    hipError_t e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_up, sizeof(SlotDesc) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_rb, sizeof(SlotDesc) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_hdr, sizeof(PoolHeader), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_errs, sizeof(int) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&p->arena, p->budget);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_slots, sizeof(SlotDesc) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_hdr, sizeof(PoolHeader));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_errs, sizeof(int) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_staging, sizeof(double) * 5 * nmax);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_scratch, sizeof(double) * 10 * nmax);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_red, sizeof(double) * 5 * kPoolRedBlocks);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_totals, sizeof(double) * 10 * max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_table, sizeof(double) * 2 * kMaxwellPoints);
    if (e != hipSuccess) { lbm_status r = hip_fail(e, "pool allocation"); lbm_pool_destroy(p); return r; }
    p->free_blocks[0] = p->budget;
    // table of the band limits, the same one every simulation uses
    std::vector<double> tab(2 * kMaxwellPoints);
    const double s_lo = std::sqrt(1.0 - kLatentTmax), s_hi = std::sqrt(1.0 - kLatentTmin);
    const double ds = (s_hi - s_lo) / (kMaxwellPoints - 1);
    for (int i = 0; i < kMaxwellPoints; ++i) {
        const double Tr = 1.0 - (s_lo + i * ds) * (s_lo + i * ds);
        host_band_limits(Tr < kLatentTmin ? kLatentTmin : Tr, tab[2 * i], tab[2 * i + 1]);
    }
    p->tab_s0 = s_lo;
    p->tab_inv_ds = 1.0 / ds;
    e = hipMemcpyAsync(p->d_table, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_errs, 0, sizeof(int) * max_slots, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) { lbm_status r = hip_fail(e, "pool setup"); lbm_pool_destroy(p); return r; }
    // the graph of the common kind set (periodic BGK requests only) up front
    lbm_status st = upload_table(p);
    if (st == LBM_OK) st = capture_graph(p, 1);
    if (st != LBM_OK) { lbm_pool_destroy(p); return st; }
    *out = p;
    return LBM_OK;
}

lbm_status lbm_pool_submit(lbm_pool* p, const lbm_params* params, const double* rho0, const double* u0,
                           const double* T0, long long nsteps, long long* ticket)
{
    clear_error();
    if (!p || !ticket || nsteps < 1) { set_error("bad pool, ticket pointer or step count"); return LBM_EINVAL; }
    lbm_status st = validate_params(params);
    if (st != LBM_OK) return st;
    if (params->lattice != 19 || params->storage_bytes != 4 || params->nx > kPoolMaxEdge ||
        params->ny > kPoolMaxEdge || params->nz > kPoolMaxEdge) {
        set_error("pool requests must be D3Q19, FP32 storage, edges <= %d", kPoolMaxEdge);
        return LBM_EINVAL;
    }
    st = validate_fields(*params, rho0, u0, T0);
    if (st != LBM_OK) return st;
    int slot = -1;
    for (int s = 0; s < p->max_slots; ++s)
        if (!p->slots[s].used) { slot = s; break; }
    if (slot < 0) { set_error("no free slot"); return LBM_EBUSY; }
    const size_t half = state_bytes(*params);
    const size_t half_al = (half + kAlign - 1) / kAlign * kAlign;
    // a tabulated EOS travels with the request: its own copy beside the two buffers
    const bool table = params->eos == LBM_EOS_TABLE;
    const size_t np = table ? (size_t)params->eos_nrho * params->eos_nT : 0;
    const size_t nc = table ? 2 * (size_t)params->eos_nT : 0;
    const size_t table_al = (sizeof(double) * (np + nc) + kAlign - 1) / kAlign * kAlign;
    const size_t bytes = 2 * half_al + table_al;
    size_t off = 0;
    if (lbm_status sd = use_device(p->device); sd != LBM_OK) return sd;
    if (!arena_alloc(p, bytes, off)) {
        set_error("request needs %zu bytes; %zu of %zu in use", bytes, p->in_use, p->budget);
        return LBM_EBUSY;
    }
    PoolSlot& ps = p->slots[slot];
    ps.used = true;
    ps.offset = off;
    ps.bytes = bytes;
    ps.params = *params;
    ps.params.eos_p = nullptr;     // the caller's table pointers are not kept
    ps.params.eos_coex = nullptr;
    ps.nsteps = nsteps;
    ps.ticket = p->next_ticket++;
    SlotDesc& d = p->table[slot];
    memset(&d, 0, sizeof(d));
    d.buf[0] = (float*)(p->arena + off);
    d.buf[1] = (float*)(p->arena + off + half_al);
    d.geom = pool_geometry(*params);
    d.phys = make_phys(*params);
    d.parity = 0;
    d.active = 1;
    const bool ext = params->walls || params->gravity[0] != 0.0 || params->gravity[1] != 0.0 ||
                     params->gravity[2] != 0.0;
    d.kind = kind_of(table ? 2 : (ext ? 1 : 0), params->collision == LBM_COLLISION_MRT);
    d.eos_p = nullptr;
    d.eos_coex = nullptr;
    if (table) {
        d.eos_p = (const double*)(p->arena + off + 2 * half_al);
        d.eos_coex = d.eos_p + np;
    }
    d.remaining = nsteps;
    const long long n = (long long)params->nx * params->ny * params->nz;
    // on the side stream: a replay in flight does not touch this free arena block or this
    // slot's error word (the slot is not active on the device)
    hipError_t e = hipMemsetAsync(p->arena + off, 0, 2 * half_al, p->side);
    if (e == hipSuccess && table)
        e = hipMemcpyAsync((void*)d.eos_p, params->eos_p, sizeof(double) * np, hipMemcpyHostToDevice, p->side);
    if (e == hipSuccess && table)
        e = hipMemcpyAsync((void*)d.eos_coex, params->eos_coex, sizeof(double) * nc, hipMemcpyHostToDevice, p->side);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_errs + slot, 0, sizeof(int), p->side);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_staging, rho0, sizeof(double) * n, hipMemcpyHostToDevice, p->side);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_staging + n, u0, sizeof(double) * 3 * n, hipMemcpyHostToDevice, p->side);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_staging + 4 * n, T0, sizeof(double) * n, hipMemcpyHostToDevice, p->side);
    if (e == hipSuccess)
        e = launch_init(19, 4, d.buf[0], p->d_staging, p->d_staging + n, p->d_staging + 4 * n, params->nx,
                        params->ny, params->nz, d.geom.pitch, d.geom.plane, params->c_v, params->walls,
                        p->side);
    // the totals of the initial state, kept for lbm_pool_totals
    if (e == hipSuccess) e = slot_reduce(p, d, *params, 0, p->d_totals + 10 * slot);
    // the staging buffer is reused by the next submission, and the next replay must find the
    // initial state in place: wait for this upload (not for the replay in flight)
    if (e == hipSuccess) e = hipStreamSynchronize(p->side);
    if (e != hipSuccess) {
        arena_free(p, off, bytes);
        ps = PoolSlot();
        return hip_fail(e, "request upload");
    }
    p->ticket_slot[ps.ticket] = slot;
    p->dirty = true;
    *ticket = ps.ticket;
    return LBM_OK;
}

lbm_status lbm_pool_run_async(lbm_pool* p)
{
    clear_error();
    if (!p) { set_error("pool is NULL"); return LBM_EINVAL; }
    if (lbm_status sd = use_device(p->device); sd != LBM_OK) return sd;
    return launch_replay(p);
}

lbm_status lbm_pool_run(lbm_pool* p)
{
    clear_error();
    if (!p) { set_error("pool is NULL"); return LBM_EINVAL; }
    if (lbm_status sd = use_device(p->device); sd != LBM_OK) return sd;
    lbm_status st = launch_replay(p);
    if (st == LBM_OK) st = finish_replay(p);
    return st;
}

lbm_status lbm_pool_poll(lbm_pool* p, long long ticket, int* done, lbm_status* result)
{
    clear_error();
    if (!p || !done) { set_error("NULL argument"); return LBM_EINVAL; }
    auto it = p->ticket_slot.find(ticket);
    if (it == p->ticket_slot.end()) { set_error("unknown ticket %lld", ticket); return LBM_EINVAL; }
    auto f = p->finished.find(ticket);
    *done = f != p->finished.end();
    if (result) *result = *done ? f->second : LBM_OK;
    return LBM_OK;
}

lbm_status lbm_pool_collect(lbm_pool* p, long long ticket, double* rho, double* u_star, double* E, double* T)
{
    clear_error();
    if (!p) { set_error("pool is NULL"); return LBM_EINVAL; }
    auto it = p->ticket_slot.find(ticket);
    if (it == p->ticket_slot.end()) { set_error("unknown ticket %lld", ticket); return LBM_EINVAL; }
    auto f = p->finished.find(ticket);
    if (f == p->finished.end()) { set_error("ticket %lld has not finished", ticket); return LBM_EBUSY; }
    const int s = it->second;
    PoolSlot& ps = p->slots[s];
    const SlotDesc& d = p->table[s];
    if (lbm_status sd = use_device(p->device); sd != LBM_OK) return sd;
    const long long n = (long long)ps.params.nx * ps.params.ny * ps.params.nz;
    double* scr = p->d_scratch;
    double* d_us = scr + 7 * n;
    int* d_err = p->d_errs + s;
    // on the side stream: the slot has finished, so a replay in flight does not advance it
    hipError_t e = launch_moments(19, 4, d.buf[d.parity], scr, ps.params.nx, ps.params.ny, ps.params.nz,
                                  d.geom.pitch, d.geom.plane, d.phys, d.eos_p, d_err, nullptr,
                                  u_star ? d_us : nullptr, nullptr, nullptr, p->side);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, scr, sizeof(double) * n, hipMemcpyDeviceToHost, p->side);
    if (e == hipSuccess && u_star) e = hipMemcpyAsync(u_star, d_us, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, p->side);
    if (e == hipSuccess && E) e = hipMemcpyAsync(E, scr + 4 * n, sizeof(double) * n, hipMemcpyDeviceToHost, p->side);
    if (e == hipSuccess && T) e = hipMemcpyAsync(T, scr + 5 * n, sizeof(double) * n, hipMemcpyDeviceToHost, p->side);
    if (e == hipSuccess) e = hipStreamSynchronize(p->side);
    if (e != hipSuccess) return hip_fail(e, "collect");
    const lbm_status result = f->second;
    arena_free(p, ps.offset, ps.bytes);
    p->ticket_slot.erase(it);
    p->finished.erase(f);
    ps = PoolSlot();
    memset(&p->table[s], 0, sizeof(SlotDesc));
    p->dirty = true;
    if (result != LBM_OK) set_error("request %lld left the EOS domain", ticket);
    return result;
}

lbm_status lbm_pool_totals(lbm_pool* p, long long ticket, double initial[5], double final_[5])
{
    clear_error();
    if (!p) { set_error("pool is NULL"); return LBM_EINVAL; }
    auto it = p->ticket_slot.find(ticket);
    if (it == p->ticket_slot.end()) { set_error("unknown ticket %lld", ticket); return LBM_EINVAL; }
    if (p->finished.find(ticket) == p->finished.end()) {
        set_error("ticket %lld has not finished", ticket);
        return LBM_EBUSY;
    }
    const int s = it->second;
    const SlotDesc& d = p->table[s];
    if (lbm_status sd = use_device(p->device); sd != LBM_OK) return sd;
    double h[10];
    double* d_tot = p->d_totals + 10 * s;
    // on the side stream: the slot has finished, so a replay in flight does not advance it
    hipError_t e = slot_reduce(p, d, p->slots[s].params, d.parity, d_tot + 5);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d_tot, sizeof(h), hipMemcpyDeviceToHost, p->side);
    if (e == hipSuccess) e = hipStreamSynchronize(p->side);
    if (e != hipSuccess) return hip_fail(e, "slot totals");
    if (initial) memcpy(initial, h, sizeof(double) * 5);
    if (final_) memcpy(final_, h + 5, sizeof(double) * 5);
    return LBM_OK;
}

lbm_status lbm_pool_stats(const lbm_pool* p, long long out[4])
{
    if (!p || !out) { set_error("NULL argument"); return LBM_EINVAL; }
    long long active = 0, free_slots = 0;
    for (int s = 0; s < p->max_slots; ++s) {
        if (p->slots[s].used && p->table[s].active) ++active;
        if (!p->slots[s].used) ++free_slots;
    }
    out[0] = active;
    out[1] = (long long)p->in_use;
    out[2] = (long long)p->budget;
    out[3] = free_slots;
    return LBM_OK;
}

lbm_status lbm_pool_destroy(lbm_pool* p)
{
    if (!p) return LBM_OK;
    // release everything even if the device reports an error: nothing here can be retried
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->side) (void)hipStreamSynchronize(p->side);
    for (int k = 0; k < (1 << kPoolKinds); ++k) {
        if (p->exec[k]) (void)hipGraphExecDestroy(p->exec[k]);
        if (p->graph[k]) (void)hipGraphDestroy(p->graph[k]);
    }
    if (p->arena) (void)hipFree(p->arena);
    if (p->d_slots) (void)hipFree(p->d_slots);
    if (p->d_hdr) (void)hipFree(p->d_hdr);
    if (p->d_errs) (void)hipFree(p->d_errs);
    if (p->d_staging) (void)hipFree(p->d_staging);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    if (p->d_red) (void)hipFree(p->d_red);
    if (p->d_totals) (void)hipFree(p->d_totals);
    if (p->d_table) (void)hipFree(p->d_table);
    if (p->h_up) (void)hipHostFree(p->h_up);
    if (p->h_rb) (void)hipHostFree(p->h_rb);
    if (p->h_hdr) (void)hipHostFree(p->h_hdr);
    if (p->h_errs) (void)hipHostFree(p->h_errs);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return LBM_OK;
}

}  // extern "C"
