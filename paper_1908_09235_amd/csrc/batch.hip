// Batched and served forms (include/lbm2p.h, lbm_batch_* and lbm_server_*).
//
// A batch holds independent instances, each a full domain (its own
// geometry, parameters and state) carved out of one device arena.  A step
// of the batch is three launches on the compute stream: the boundary pass
// over the link blocks of every instance, the main pass over the tiles of
// every instance (persistent workgroups over per-XCD tile queues, or one
// workgroup per tile), and a per-instance reduction that records the total
// mass and advances the instance's step counter.  The instance tables live
// in device memory, so the launches are captured once into a graph of
// several steps and replayed while instances join and leave.  Instances
// are built on a second stream, so a new instance is prepared while the
// running ones compute.
//
// The server keeps a FIFO of requests; each scheduling round waits for
// the chunk of steps in flight, retires finished instances, launches the
// next chunk for everything resident, and while that chunk runs admits
// queued requests as arena memory allows (admission by device footprint).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/lbm2p.h"
#include "domain.hpp"
#include "launch.hpp"

using namespace lbm;

namespace {

constexpr int kQueues = 8;
constexpr int kBoundaryGrid = 1024;
constexpr int kReduceGrid = 512;

}  // namespace

struct lbm_batch {
    lbm_batch_desc bd{};
    Arena arena;
    hipStream_t stream = nullptr;  // compute
    hipStream_t setup = nullptr;   // instance construction and read-out
    bool own_stream = false;
    int ncu = 0;
    int tile_w = 256, tile_h = 16, persistent = 1;
    int ring = 3;  // rows of loads per lane of the main pass (2, 3, 4)
    int graph_steps = 32;

    std::vector<lbm_domain*> inst;        // per slot (nullptr: free)
    std::vector<BState> state;            // host mirror, valid after a sync
    std::vector<char> joined;             // slot is in the device tables
    bool dirty = true;                    // tables must be rebuilt
    bool inflight = false;

    // device tables
    BInst* d_inst = nullptr;
    BState* d_state = nullptr;
    int2* d_tiles = nullptr;
    int* d_qnext = nullptr;
    int* d_qbound = nullptr;
    int2* d_lblk = nullptr;
    int* d_nlblk = nullptr;
    int tiles_cap = 0, lblk_cap = 0;
    long long ntiles = 0, nlblk = 0;
    // pinned staging for table uploads (reused only after a sync)
    BInst* h_inst = nullptr;
    BState* h_state = nullptr;
    int2* h_tiles = nullptr;
    int2* h_lblk = nullptr;
    int* h_small = nullptr;  // qbound[9], nlblk

    hipGraphExec_t graph = nullptr;
    // tile_w, persistent, main grid, steps, save_f, boundary grid, reduce
    // grid, ring
    int graph_key[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct lbm_server {
    lbm_batch* b = nullptr;
    long long chunk = 64;
    struct Req {
        long long id;
        lbm_desc copy;  // its arrays stay the caller's until admission
        long long steps;
    };
    std::deque<Req> queue;
    std::unordered_map<long long, int> slot_of;  // admitted id -> slot
    std::vector<long long> id_of;                // slot -> id (or -1)
    std::vector<char> finished;                  // slot finished (not released)
    long long next_id = 0, admitted = 0, chunks = 0, rejected = 0;
};

namespace {

template <typename T>
int dmalloc(T** p, size_t n) {
    if (hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return LBM_ENOMEM;
    }
    return LBM_OK;
}

template <typename T>
int hmalloc(T** p, size_t n) {
    if (hipHostMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n, 1) * sizeof(T),
                      hipHostMallocDefault) != hipSuccess) {
        *p = nullptr;
        return LBM_ENOMEM;
    }
    return LBM_OK;
}

void drop_graph(lbm_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

void free_batch(lbm_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (lbm_domain* d : b->inst)
        if (d) domain_free(d);
    drop_graph(b);
    for (void* p : {(void*)b->d_inst, (void*)b->d_state, (void*)b->d_tiles, (void*)b->d_qnext,
                    (void*)b->d_qbound, (void*)b->d_lblk, (void*)b->d_nlblk})
        if (p) (void)hipFree(p);
    for (void* p : {(void*)b->h_inst, (void*)b->h_state, (void*)b->h_tiles, (void*)b->h_lblk,
                    (void*)b->h_small})
        if (p) (void)hipHostFree(p);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->setup) (void)hipStreamDestroy(b->setup);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int grow_tables(lbm_batch* b, long long tiles, long long lblk) {
    if (tiles > b->tiles_cap) {
        const int cap = (int)std::max<long long>(tiles, 2LL * b->tiles_cap);
        if (b->d_tiles) (void)hipFree(b->d_tiles);
        if (b->h_tiles) (void)hipHostFree(b->h_tiles);
        b->d_tiles = nullptr;
        b->h_tiles = nullptr;
        if (dmalloc(&b->d_tiles, cap) || hmalloc(&b->h_tiles, cap)) return LBM_ENOMEM;
        b->tiles_cap = cap;
        drop_graph(b);  // the graph holds the old table address
    }
    if (lblk > b->lblk_cap) {
        const int cap = (int)std::max<long long>(lblk, 2LL * b->lblk_cap);
        if (b->d_lblk) (void)hipFree(b->d_lblk);
        if (b->h_lblk) (void)hipHostFree(b->h_lblk);
        b->d_lblk = nullptr;
        b->h_lblk = nullptr;
        if (dmalloc(&b->d_lblk, cap) || hmalloc(&b->h_lblk, cap)) return LBM_ENOMEM;
        b->lblk_cap = cap;
        drop_graph(b);
    }
    return LBM_OK;
}

BInst make_inst(lbm_domain* d) {
    BInst I{};
    I.f[0] = d->f[0];
    I.f[1] = d->f[1];
    I.flags = d->flags;
    I.side_mom_bytes = (unsigned)(3 * std::max(d->nslots, 1) * 8);
    I.side_f_bytes = (unsigned)(9 * (d->save_f ? std::max(d->nslots, 1) : 1) * 8);
    I.side_idx = d->side_idx;
    I.psiw = d->psiw;
    I.side_mom = d->side_mom;
    I.side_f = d->side_f;
    I.partial = d->partial;
    I.nx = d->nx;
    I.ny = d->ny;
    I.pitch = d->pitch;
    I.nsegs = d->nsegs;
    I.nstrips = d->nstrips;
    I.np = d->nblocks;
    I.plane = d->plane;
    I.ph = d->ph64;
    I.nslot = d->nslot_links;
    I.fix = d->fix;
    I.lnode = d->lnode;
    I.lmeta = d->lmeta;
    I.lghost = d->lghost;
    I.lxf = d->lxf;
    I.lxff = d->lxff;
    I.lslotb = d->lslotb;
    I.lslotf = d->lslotf;
    I.lc = d->lc;
    I.luw = d->luw;
    I.rref = d->ph64.rref;
    I.lref = d->lref;
    I.hist = d->hist;
    I.cap = d->cap;
    I.unstable = d->unstable;
    return I;
}

// Rebuild and upload the instance, tile and link-block tables.  Only with
// nothing in flight on the compute stream.
int rebuild(lbm_batch* b) {
    const int n = (int)b->inst.size();
    long long tiles = 0, lblk = 0;
    for (int i = 0; i < n; ++i) {
        lbm_domain* d = b->inst[i];
        if (!d) continue;
        if (domain_set_tiles(d, b->tile_w, b->tile_h) != LBM_OK) return LBM_EINVAL;
        tiles += d->nblocks;
        lblk += (d->nslot_links + 255) / 256;
    }
    int rc = grow_tables(b, tiles, lblk);
    if (rc) return rc;
    long long k = 0, m = 0;
    for (int i = 0; i < n; ++i) {
        lbm_domain* d = b->inst[i];
        b->joined[i] = d != nullptr;
        if (!d) {
            b->h_inst[i] = BInst{};
            b->h_state[i] = BState{0, 0};
            continue;
        }
        b->h_inst[i] = make_inst(d);
        b->h_state[i] = b->state[i];
        for (int t = 0; t < d->nblocks; ++t) b->h_tiles[k++] = make_int2(i, t);
        for (int t = 0; t < (d->nslot_links + 255) / 256; ++t) b->h_lblk[m++] = make_int2(i, t);
    }
    b->ntiles = tiles;
    b->nlblk = lblk;
    // queue q serves a contiguous run of the tile list
    for (int q = 0; q <= kQueues; ++q) b->h_small[q] = (int)(tiles * q / kQueues);
    b->h_small[kQueues + 1] = (int)lblk;
    hipStream_t s = b->stream;
    if (hipMemcpyAsync(b->d_inst, b->h_inst, n * sizeof(BInst), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(b->d_state, b->h_state, n * sizeof(BState), hipMemcpyHostToDevice, s) ||
        (tiles && hipMemcpyAsync(b->d_tiles, b->h_tiles, tiles * sizeof(int2),
                                 hipMemcpyHostToDevice, s)) ||
        (lblk && hipMemcpyAsync(b->d_lblk, b->h_lblk, lblk * sizeof(int2),
                                hipMemcpyHostToDevice, s)) ||
        hipMemcpyAsync(b->d_qbound, b->h_small, (kQueues + 1) * sizeof(int),
                       hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(b->d_nlblk, b->h_small + kQueues + 1, sizeof(int),
                       hipMemcpyHostToDevice, s))
        return LBM_EDEVICE;
    b->dirty = false;
    return LBM_OK;
}

BatchLaunch launch_of(lbm_batch* b) {
    BatchLaunch L{};
    L.args.inst = b->d_inst;
    L.args.state = b->d_state;
    L.args.tiles = b->d_tiles;
    L.args.qnext = b->d_qnext;
    L.args.qbound = b->d_qbound;
    L.args.lblk = b->d_lblk;
    L.args.nlblk = b->d_nlblk;
    L.args.ninst = (int)b->inst.size();
    L.args.tile_h = b->tile_h;
    L.args.persistent = b->persistent;
    L.eos = b->bd.eos;
    L.storage = b->bd.storage;
    L.tile_w = b->tile_w;
    L.ring = b->bd.storage == LBM_STORE_F16NODE ? 3 : b->ring;
    L.save_f = false;
    for (lbm_domain* d : b->inst)
        if (d && d->save_f) L.save_f = true;
    if (b->persistent) {
        const int occ = b->bd.storage == LBM_STORE_F64
                            ? batch_occupancy_f64(b->bd.eos, b->bd.storage, b->tile_w, L.save_f,
                                                  b->ring)
                            : batch_occupancy_f32(b->bd.eos, b->bd.storage, b->tile_w, L.save_f,
                                                  b->ring);
        // no more workgroups than tiles: a small batch would otherwise pay
        // for queue tickets of workgroups that find nothing to do
        L.main_grid = (int)std::min<long long>((long long)b->ncu * std::max(occ, 1),
                                               std::max<long long>(b->ntiles, 1));
    } else {
        L.main_grid = (int)std::max<long long>(b->ntiles, 1);
    }
    L.bnd_grid = (int)std::min<long long>(kBoundaryGrid, std::max<long long>(b->nlblk, 1));
    L.red_grid = std::min<int>(kReduceGrid, std::max<int>((int)b->inst.size(), 1));
    L.stream = b->stream;
    return L;
}

void launch_step(lbm_batch* b, const BatchLaunch& L) {
    if (b->bd.storage == LBM_STORE_F64) launch_batch_f64(L);
    else launch_batch_f32(L);
    launch_batch_reduce(L);
}

// Enqueue n steps on the compute stream: whole graphs of graph_steps steps,
// the rest as plain launches.
int enqueue(lbm_batch* b, long long n) {
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    if (b->ntiles == 0) return LBM_OK;
    const BatchLaunch L = launch_of(b);
    const int G = b->graph_steps;
    long long done = 0;
    if (G > 0 && n >= G) {
        const int key[8] = {b->tile_w, b->persistent, L.main_grid, G, L.save_f ? 1 : 0,
                            L.bnd_grid, L.red_grid, L.ring};
        if (b->graph && std::memcmp(key, b->graph_key, sizeof key) != 0) drop_graph(b);
        if (!b->graph) {
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return LBM_EDEVICE;
            for (int k = 0; k < G; ++k) launch_step(b, L);
            if (hipStreamEndCapture(b->stream, &g) != hipSuccess) return LBM_EDEVICE;
            const hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b->graph = nullptr;
                return LBM_EDEVICE;
            }
            std::memcpy(b->graph_key, key, sizeof key);
        }
        for (; done + G <= n; done += G)
            if (hipGraphLaunch(b->graph, b->stream) != hipSuccess) return LBM_EDEVICE;
    }
    for (; done < n; ++done) launch_step(b, L);
    if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
    b->inflight = true;
    return LBM_OK;
}

// Wait for the compute stream and refresh the host mirror of the states
// and the per-instance domain bookkeeping.
int sync_batch(lbm_batch* b) {
    const int n = (int)b->inst.size();
    if (b->inflight) {
        if (hipMemcpyAsync(b->h_state, b->d_state, n * sizeof(BState), hipMemcpyDeviceToHost,
                           b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess)
            return LBM_EDEVICE;
        for (int i = 0; i < n; ++i)
            if (b->joined[i] && b->inst[i]) b->state[i] = b->h_state[i];
        b->inflight = false;
    }
    for (int i = 0; i < n; ++i) {
        lbm_domain* d = b->inst[i];
        if (!d) continue;
        d->t = b->state[i].t;
        d->cur = (int)(d->t & 1);
        d->pending = false;
        d->pending_t = d->t;
    }
    return LBM_OK;
}

int batch_add(lbm_batch* b, const lbm_desc* desc, long long steps, int* slot) {
    if (desc->storage != b->bd.storage || desc->eos != b->bd.eos) return LBM_EINVAL;
    int s = -1;
    for (int i = 0; i < (int)b->inst.size(); ++i)
        if (!b->inst[i]) {
            s = i;
            break;
        }
    if (s < 0) return LBM_ENOMEM;  // no free slot
    lbm_desc c = *desc;
    c.stream = b->setup;
    c.tile_w = b->tile_w;
    c.tile_h = b->tile_h;
    lbm_domain* d = nullptr;
    int rc = domain_create(&c, &b->arena, &d);
    if (rc) return rc;
    // A reused slot may still be listed in the device tables, with the
    // stopped state of its previous instance, until the next rebuild: the
    // launches skip it, and its device state is not read back meanwhile.
    b->inst[s] = d;
    b->state[s] = BState{0, steps};
    b->joined[s] = 0;
    b->dirty = true;
    *slot = s;
    return LBM_OK;
}

int batch_remove(lbm_batch* b, int slot) {
    lbm_domain* d = b->inst[slot];
    // a joined instance may be read by queued work unless it has stopped
    if (b->joined[slot] && b->inflight && b->state[slot].remaining > 0) {
        int rc = sync_batch(b);
        if (rc) return rc;
    }
    domain_free(d);
    b->inst[slot] = nullptr;
    b->state[slot] = BState{0, 0};
    b->dirty = true;
    return LBM_OK;
}

bool valid_slot(lbm_batch* b, int slot) {
    return b && slot >= 0 && slot < (int)b->inst.size() && b->inst[slot];
}

}  // namespace

extern "C" {

int lbm_batch_create(const lbm_batch_desc* bd, lbm_batch** out) {
    if (!bd || !out) return LBM_EINVAL;
    if (bd->storage < LBM_STORE_F64 || bd->storage > LBM_STORE_F16NODE) return LBM_EINVAL;
    if (bd->eos < LBM_EOS_NONE || bd->eos > LBM_EOS_CS) return LBM_EINVAL;
    if (bd->max_instances < 1 || bd->max_instances > (1 << 20)) return LBM_EINVAL;
    if (bd->tile_w != 0 && bd->tile_w != 64 && bd->tile_w != 128 && bd->tile_w != 256)
        return LBM_EINVAL;
    if (bd->tile_h < 0 || (bd->tile_h > 0 && bd->tile_h < 8)) return LBM_EINVAL;
    if (bd->persistent < 0 || bd->persistent > 1) return LBM_EINVAL;
    if (bd->ring != 0 && (bd->ring < 2 || bd->ring > 4)) return LBM_EINVAL;
    if (bd->storage == LBM_STORE_F16NODE && bd->ring != 0 && bd->ring != 3) return LBM_EINVAL;
    if (bd->arena_bytes <= 0) return LBM_EINVAL;
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ENOMEM;
    b->bd = *bd;
    b->tile_w = bd->tile_w ? bd->tile_w : 256;
    b->tile_h = bd->tile_h ? bd->tile_h : 16;
    b->persistent = bd->persistent;
    b->ring = bd->ring ? bd->ring : 3;
    b->graph_steps = bd->graph_steps == 0 ? 32 : std::max(bd->graph_steps, 0);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        free_batch(b);
        return LBM_EDEVICE;
    }
    b->ncu = prop.multiProcessorCount;
    b->stream = static_cast<hipStream_t>(bd->stream);
    if (!b->stream) {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            free_batch(b);
            return LBM_EDEVICE;
        }
        b->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&b->setup, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
        free_batch(b);
        return LBM_EDEVICE;
    }
    const int n = bd->max_instances;
    int rc = b->arena.init((size_t)bd->arena_bytes);
    if (!rc) rc = dmalloc(&b->d_inst, n);
    if (!rc) rc = dmalloc(&b->d_state, n);
    if (!rc) rc = dmalloc(&b->d_qnext, kQueues * kQueueStride);
    if (!rc) rc = dmalloc(&b->d_qbound, kQueues + 1);
    if (!rc) rc = dmalloc(&b->d_nlblk, 1);
    if (!rc) rc = hmalloc(&b->h_inst, n);
    if (!rc) rc = hmalloc(&b->h_state, n);
    if (!rc) rc = hmalloc(&b->h_small, kQueues + 2);
    if (!rc) rc = grow_tables(b, 1024, 1024);
    if (rc) {
        free_batch(b);
        return rc;
    }
    if (hipMemsetAsync(b->d_qnext, 0, kQueues * kQueueStride * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_state, 0, n * sizeof(BState), b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        free_batch(b);
        return LBM_EDEVICE;
    }
    b->inst.assign(n, nullptr);
    b->state.assign(n, BState{0, 0});
    b->joined.assign(n, 0);
    *out = b;
    return LBM_OK;
}

int lbm_batch_add(lbm_batch* b, const lbm_desc* d, int64_t steps, int32_t* slot) {
    if (!b || !d || !slot || steps < 0) return LBM_EINVAL;
    if (d->open_x != 0) return LBM_EINVAL;  // batched instances are periodic
    int s = -1;
    int rc = batch_add(b, d, steps, &s);
    if (rc == LBM_OK) *slot = s;
    return rc;
}

int lbm_batch_run(lbm_batch* b, int64_t n) {
    if (!b || n < 0) return LBM_EINVAL;
    if (n == 0) return LBM_OK;
    if (b->inflight) {
        int rc = sync_batch(b);
        if (rc) return rc;
    }
    return enqueue(b, n);
}

int lbm_batch_sync(lbm_batch* b) {
    if (!b) return LBM_EINVAL;
    return sync_batch(b);
}

int lbm_batch_status(lbm_batch* b, int32_t slot, int64_t* t, int64_t* remaining,
                     int64_t* unstable_step) {
    if (!valid_slot(b, slot)) return LBM_EINVAL;
    int rc = sync_batch(b);
    if (rc) return rc;
    if (t) *t = b->state[slot].t;
    if (remaining) *remaining = b->state[slot].remaining;
    if (unstable_step) {
        int64_t u = -1;
        rc = lbm_unstable_step(b->inst[slot], &u);
        if (rc) return rc;
        *unstable_step = u;
    }
    return LBM_OK;
}

int lbm_batch_moments(lbm_batch* b, int32_t slot, double* rho, double* ux, double* uy) {
    if (!valid_slot(b, slot)) return LBM_EINVAL;
    int rc = sync_batch(b);
    if (rc) return rc;
    return lbm_moments(b->inst[slot], rho, ux, uy);
}

int lbm_batch_mass_history(lbm_batch* b, int32_t slot, double* out, int64_t cap,
                           int64_t* n_written) {
    if (!valid_slot(b, slot)) return LBM_EINVAL;
    int rc = sync_batch(b);
    if (rc) return rc;
    return lbm_mass_history(b->inst[slot], out, cap, n_written);
}

int lbm_batch_remove(lbm_batch* b, int32_t slot) {
    if (!valid_slot(b, slot)) return LBM_EINVAL;
    return batch_remove(b, slot);
}

int lbm_batch_tune(lbm_batch* b, int64_t steps_per_trial, int32_t out[5]) {
    if (!b || steps_per_trial < 1 || !out) return LBM_EINVAL;
    int rc = sync_batch(b);
    if (rc) return rc;
    if (b->dirty && (rc = rebuild(b))) return rc;
    if (b->ntiles == 0) {
        // nothing to time: the shape stays as it is
        out[0] = b->tile_w;
        out[1] = b->tile_h;
        out[2] = b->persistent;
        out[3] = 0;
        out[4] = b->ring;
        return LBM_OK;
    }
    const int tws[3] = {64, 128, 256}, ths[3] = {8, 16, 32}, rings[3] = {2, 3, 4};
    const int nring = b->bd.storage == LBM_STORE_F16NODE ? 1 : 3;
    float best = -1.0f;
    int bw = b->tile_w, bh = b->tile_h, bp = b->persistent, br = b->ring;
    const int G = b->graph_steps;
    b->graph_steps = 0;  // time plain launches (no capture per candidate)
    for (int ri = 0; ri < nring && !rc; ++ri)
        for (int p = 0; p <= 1 && !rc; ++p)
            for (int wi = 0; wi < 3 && !rc; ++wi)
                for (int hi = 0; hi < 3 && !rc; ++hi) {
                const int tw = tws[wi], th = ths[hi];
                b->tile_w = tw;
                b->tile_h = th;
                b->persistent = p;
                b->ring = nring == 1 ? 3 : rings[ri];
                b->dirty = true;
                if ((rc = enqueue(b, 1))) break;  // rebuild, warm up
                if (hipEventRecord(b->ev0, b->stream) != hipSuccess) rc = LBM_EDEVICE;
                if (!rc) rc = enqueue(b, steps_per_trial);
                if (!rc && hipEventRecord(b->ev1, b->stream) != hipSuccess) rc = LBM_EDEVICE;
                if (!rc) rc = sync_batch(b);
                // (the stop event is waited for on its own: a run that
                // launched nothing leaves no batch work to wait for)
                if (!rc && hipEventSynchronize(b->ev1) != hipSuccess) rc = LBM_EDEVICE;
                float ms = 0.0f;
                if (!rc && hipEventElapsedTime(&ms, b->ev0, b->ev1) != hipSuccess) rc = LBM_EDEVICE;
                if (rc) break;
                if (best < 0.0f || ms < best) {
                    best = ms;
                    bw = tw;
                    bh = th;
                    bp = p;
                    br = b->ring;
                }
            }
    b->graph_steps = G;
    b->tile_w = bw;
    b->tile_h = bh;
    b->persistent = bp;
    b->ring = br;
    b->dirty = true;
    if (rc) return rc;
    out[0] = bw;
    out[1] = bh;
    out[2] = bp;
    out[3] = (int32_t)(best * 1000.0f / (float)steps_per_trial);  // us per step
    out[4] = br;
    return LBM_OK;
}

int lbm_batch_info(lbm_batch* b, int64_t out[8]) {
    if (!b || !out) return LBM_EINVAL;
    long long n = 0, tiles = 0, lblk = 0;
    for (lbm_domain* d : b->inst) {
        if (!d) continue;
        ++n;
        const int sc = strip_cols(b->tile_w);
        tiles += ((d->nx + sc - 1) / sc) * (long long)((d->ny + b->tile_h - 1) / b->tile_h);
        lblk += (d->nslot_links + 255) / 256;
    }
    out[0] = n;
    out[1] = tiles;
    out[2] = lblk;
    out[3] = (int64_t)b->arena.capacity();
    out[4] = (int64_t)b->arena.used();
    out[5] = b->tile_w;
    out[6] = b->tile_h;
    out[7] = b->persistent;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) { free_batch(b); }

// ------------------------------------------------------------------ server
int lbm_server_create(const lbm_batch_desc* bd, int64_t chunk_steps, lbm_server** out) {
    if (!bd || !out || chunk_steps < 1) return LBM_EINVAL;
    lbm_server* s = new (std::nothrow) lbm_server();
    if (!s) return LBM_ENOMEM;
    int rc = lbm_batch_create(bd, &s->b);
    if (rc) {
        delete s;
        return rc;
    }
    s->chunk = chunk_steps;
    s->id_of.assign(bd->max_instances, -1);
    s->finished.assign(bd->max_instances, 0);
    *out = s;
    return LBM_OK;
}

int lbm_server_submit(lbm_server* s, const lbm_desc* d, int64_t steps, int64_t* id) {
    if (!s || !d || !id || steps < 1) return LBM_EINVAL;
    if (d->storage != s->b->bd.storage || d->eos != s->b->bd.eos) return LBM_EINVAL;
    if (d->open_x != 0) return LBM_EINVAL;
    lbm_server::Req r{s->next_id++, *d, steps};
    s->queue.push_back(r);
    *id = r.id;
    return LBM_OK;
}

int lbm_server_progress(lbm_server* s, int64_t* done_ids, int64_t cap, int64_t* n_done) {
    if (!s || !n_done || cap < 0 || (cap > 0 && !done_ids)) return LBM_EINVAL;
    lbm_batch* b = s->b;
    *n_done = 0;
    // 1. the chunk in flight
    int rc = sync_batch(b);
    if (rc) return rc;
    // finished requests are reported at most cap at a time; the others stay
    // unreported (they run no more steps) for the next calls
    long long nd = 0;
    for (int i = 0; i < (int)b->inst.size() && nd < cap; ++i) {
        if (!b->inst[i] || s->finished[i] || !b->joined[i]) continue;
        if (b->state[i].remaining <= 0) {
            s->finished[i] = 1;
            done_ids[nd++] = s->id_of[i];
        }
    }
    // 2. the next chunk for everything resident
    bool any = false;
    for (int i = 0; i < (int)b->inst.size(); ++i)
        if (b->inst[i] && b->state[i].remaining > 0) any = true;
    if (any) {
        if ((rc = enqueue(b, s->chunk))) return rc;
        ++s->chunks;
    }
    // 3. while it runs, admit queued requests in arrival order as memory allows
    while (!s->queue.empty()) {
        lbm_server::Req& r = s->queue.front();
        int slot = -1;
        rc = batch_add(b, &r.copy, r.steps, &slot);
        if (rc == LBM_ENOMEM) {
            // wait for memory or a slot, unless nothing resident could free any
            bool resident = false;
            for (lbm_domain* d : b->inst) resident = resident || d != nullptr;
            if (resident) break;
        }
        if (rc) {
            ++s->rejected;
            s->queue.pop_front();
            continue;
        }
        s->id_of[slot] = r.id;
        s->slot_of[r.id] = slot;
        s->finished[slot] = 0;
        ++s->admitted;
        s->queue.pop_front();
    }
    *n_done = nd;
    return LBM_OK;
}

int lbm_server_result(lbm_server* s, int64_t id, double* rho, double* ux, double* uy,
                      double mass[2], int64_t* steps_done, int64_t* unstable_step) {
    if (!s) return LBM_EINVAL;
    auto it = s->slot_of.find(id);
    if (it == s->slot_of.end()) return LBM_EINVAL;
    const int slot = it->second;
    if (!s->finished[slot]) return LBM_EINVAL;
    lbm_domain* d = s->b->inst[slot];
    // read-out on the setup stream; the compute stream skips this instance
    d->t = s->b->state[slot].t;
    d->cur = (int)(d->t & 1);
    d->pending = false;
    int rc = LBM_OK;
    if (rho || ux || uy) rc = lbm_moments(d, rho, ux, uy);
    if (!rc && mass) {
        std::vector<double> h((size_t)std::min<long long>(d->t + 1, d->cap));
        int64_t n = 0;
        rc = lbm_mass_history(d, h.data(), (int64_t)h.size(), &n);
        if (!rc) {
            mass[0] = d->t + 1 <= d->cap ? h[0] : NAN;  // M(0) if still in the ring
            mass[1] = h[(size_t)n - 1];
        }
    }
    if (!rc && steps_done) *steps_done = d->t;
    if (!rc && unstable_step) rc = lbm_unstable_step(d, unstable_step);
    return rc;
}

int lbm_server_release(lbm_server* s, int64_t id) {
    if (!s) return LBM_EINVAL;
    auto it = s->slot_of.find(id);
    if (it == s->slot_of.end()) return LBM_EINVAL;
    const int slot = it->second;
    if (!s->finished[slot]) return LBM_EINVAL;
    int rc = batch_remove(s->b, slot);
    if (rc) return rc;
    s->slot_of.erase(it);
    s->id_of[slot] = -1;
    s->finished[slot] = 0;
    return LBM_OK;
}

int lbm_server_info(lbm_server* s, int64_t out[8]) {
    if (!s || !out) return LBM_EINVAL;
    long long running = 0, fin = 0;
    for (int i = 0; i < (int)s->b->inst.size(); ++i) {
        if (!s->b->inst[i]) continue;
        if (s->finished[i]) ++fin;
        else ++running;
    }
    out[0] = (int64_t)s->queue.size();
    out[1] = running;
    out[2] = fin;
    out[3] = (int64_t)s->b->arena.used();
    out[4] = (int64_t)s->b->arena.capacity();
    out[5] = s->chunks;
    out[6] = s->admitted;
    out[7] = s->rejected;
    return LBM_OK;
}

void lbm_server_destroy(lbm_server* s) {
    if (!s) return;
    free_batch(s->b);
    delete s;
}

}  // extern "C"
