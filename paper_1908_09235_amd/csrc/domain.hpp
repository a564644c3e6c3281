// Host-side state of one domain, shared by the single-domain API
// (lbm2p.hip) and the batched and served forms (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <map>
#include <vector>

#include "../../include/lbm2p.h"
#include "launch.hpp"

namespace lbm {

// Device memory carved out of one hipMalloc: first fit over 256-byte
// granules with a coalescing free list.  Bookkeeping is host-only, so
// taking and returning memory never synchronises the device; the caller
// returns a block only once no queued work uses it.
class Arena {
  public:
    ~Arena();
    int init(size_t bytes);  // lbm_status
    void* alloc(size_t bytes);  // nullptr if nothing fits
    void release(void* p);
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t largest_free() const;

  private:
    char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    std::map<size_t, size_t> live_;  // offset -> bytes
};

}  // namespace lbm

struct lbm_domain {
    int nx = 0, ny = 0, pitch = 0;
    long long plane = 0;
    int storage = 0, eos = 0, coll = 0, rule = 0, fix = 0;
    int tile_w = 0, tile_h = 0, nstrips = 0, nsegs = 0, nblocks = 0;
    size_t esize = 8;
    size_t fbytes = 0;  // one state buffer: nine planes (+ the FP16 per-node
                        // form's FP32 density plane)
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t* flags = nullptr;
    float* psiw = nullptr;  // FP16 storage: psi_w of solid nodes in FP32
    int* side_idx = nullptr;
    double* side_mom = nullptr;
    double* side_f = nullptr;
    int nslots = 0;
    bool save_f = false;
    double* partial = nullptr;
    double* hist = nullptr;
    long long* unstable = nullptr;
    double* mom_out = nullptr;
    int* lref = nullptr;   // per link: side slot whose density encodes its ghost
    int open_x = 0;        // velocity inlet at x = 0, outlet at x = nx - 1
    double inlet_u = 0.0;
    double* force = nullptr;   // wall force partials, two per link block
    unsigned long long* negrest = nullptr;  // scheme A: negative rest count
    unsigned long long* degen = nullptr;    // scheme B / Bao: cancelled sums count
    bool force_valid = false;  // a boundary pass has written them
    int nb = 0, nl = 0;
    int nslot_links = 0;
    int *lnode = nullptr, *lmeta = nullptr, *lghost = nullptr, *lxf = nullptr,
        *lxff = nullptr, *lslotb = nullptr, *lslotf = nullptr;
    double *lc = nullptr, *luw = nullptr;
    long long cap = 0, t = 0;
    long long* clock = nullptr;  // device: step of the last recorded mass
    // Two steps per pass (k_main2): fused = 2 when in use (1: every step
    // is its own pass); eligible when the form allows it.
    int fused = 1;
    bool fusable = false;
    int tile_h2 = 0, nstrips2 = 0, nsegs2 = 0, nblocks2 = 0;
    int* node_link = nullptr;    // per node (pitch layout): first link slot + 1, or 0
    int* tile_order = nullptr;   // tile of each workgroup of the two-step pass
    std::vector<int> bnd_x, bnd_y;  // host: the boundary nodes (tile weights)
    double* partial2 = nullptr;  // masses of the second step of a pass
    int pending_steps = 0;       // steps of the last pass whose masses are pending
    // After a two-step pass f*(t - 1) is not in memory: the buffer that
    // held f*(t - 2) still does, with the ghosts of step t - 1, and the
    // moments at t and the wall force of the last step are read from a
    // replay of step t - 1 into these buffers.
    bool last_fused = false;
    bool replay_valid = false;
    void* frep = nullptr;
    double* side_mom_rep = nullptr;
    bool pending = false;
    long long pending_t = 0;
    hipStream_t stream = nullptr;
    int device = 0;              // the GPU the domain lives on
    // Captured runs of 2^k steps (k = 0 .. kGraphLevels - 1), per parity of
    // the buffer that holds f*(t) when the run starts; built on first use
    // on a capture stream of the domain's own and replayed on `stream`.
    static constexpr int kGraphLevels = 6;
    hipGraphExec_t graphs[2][kGraphLevels] = {};
    hipStream_t cap_stream = nullptr;
    bool graphs_off = false;     // capture failed once: plain launches
    lbm::Phys<double> ph64{};
    lbm::Phys<float> ph32{};
    size_t bytes = 0;
    long long fluid = 0, fallbacks = 0;
    std::vector<void*> allocs;
    lbm::Arena* arena = nullptr;  // sub-allocate from it instead of hipMalloc
    int partial_cap = 0;          // partials held (enough for 64 x 8 tiles)
    int prof = 0;                 // record every prof-th step (0: off)
    int nrec = 0;
    std::vector<hipEvent_t> ev;
    double main_ms = 0, bnd_ms = 0;
    long long main_n = 0, bnd_n = 0;
};

namespace lbm {

// Build a domain from a descriptor (all device work on desc->stream, which
// is synchronised before returning).  With an arena, device memory comes
// from it.
int domain_create(const lbm_desc* desc, Arena* arena, lbm_domain** out);
void domain_free(lbm_domain* d);
// The tile shape of the main pass (tile_w 64/128/256, tile_h >= 1 with at
// most partial_cap tiles); the next launch uses it.
int domain_set_tiles(lbm_domain* d, int tile_w, int tile_h);
Ctx domain_ctx(lbm_domain* d);
// The buffer the moments at the current time are pulled from: f*(t - 1)
// with the ghosts of step t (after a two-step pass, rebuilt by a replay of
// step t - 1 into the domain's replay buffer; also forms the wall force of
// the last step).  Enqueued on the domain's stream; allocates nothing.
const void* moments_source(lbm_domain* d);

}  // namespace lbm
