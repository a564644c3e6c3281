// Launch interface between the host API and the kernels.  Each storage
// precision is compiled in its own translation unit (launch_f64.hip with
// exact left-to-right rounding, launch_f32.hip with fused multiply-adds).
#pragma once

#include <hip/hip_runtime.h>

#include "fused.hpp"

namespace lbm {

struct Ctx {
    int nx, ny, pitch;
    long long plane;
    int eos;
    int storage;  // lbm_storage
    int tile_w, tile_h, nsegs, nstrips, nblocks;
    const uint8_t* flags;
    float* psiw;  // FP16 storage: psi_w of solid nodes in FP32 (else null)
    const int* side_idx;
    double* side_mom;
    double* side_f;
    unsigned side_mom_bytes, side_f_bytes;
    bool save_f;  // boundary nodes save pre-collision populations (Zhao-Yong)
    double* partial;
    double* mom_out;
    const float* ref;  // init: density plane of the buffer being filled (or null)
    Phys<double> ph;  // converted to the compute type by the launcher
    hipStream_t stream;
    // two steps per pass (k_main2)
    int tile_h2, nsegs2, nstrips2, nblocks2;
    const int* node_link;
    const int* tile_order;  // two-step pass: tile of each workgroup
    double* partial2;
    const int* lmeta;
    const double* lc;
    const double* luw;
    unsigned long long* negrest;
    unsigned long long* degen;
    int fix;
    // when set, the main, two-step and boundary launches record their own
    // start and end on these events (the dispatch's timestamps, without
    // the launch latency that events recorded around a launch include)
    hipEvent_t ev_start, ev_stop;
};

// one main pass src -> dst (or the moments of src when moments is set)
void launch_main_f64(const Ctx& c, const void* src, void* dst, bool moments);
void launch_main_f32(const Ctx& c, const void* src, void* dst, bool moments);
// two steps per pass src -> dst (storage forms with FP32 or FP16
// populations and one reference density; see fused.hpp)
void launch_main2_f32(const Ctx& c, const void* src, void* dst);
// one boundary pass on cur
void launch_boundary_f64(const Ctx& c, void* cur, const BndArgs& b, int nblocks);
void launch_boundary_f32(const Ctx& c, void* cur, const BndArgs& b, int nblocks);
// psi at walls into plane 0 of both buffers, and f(0) = f_eq(rho0, u0)
// scattered into buf
void launch_init_f64(const Ctx& c, const double* rho_wall, const double* rho0,
                     const double* ux0, const double* uy0, void* buf, void* other);
void launch_init_f32(const Ctx& c, const double* rho_wall, const double* rho0,
                     const double* ux0, const double* uy0, void* buf, void* other);
// the last main pass's partials (two arrays if it made two steps) into
// hist[(clock + 1) % cap], clock += 1 per step
void launch_reduce(const Ctx& c, bool two, long long cap, long long* clock, double* hist,
                   long long* unstable);

// One step of a batch: boundary and main passes (per storage precision),
// then the per-instance reduction.
struct BatchLaunch {
    BatchArgs args;
    int eos, storage;
    int tile_w;     // main-pass workgroup size
    int main_grid;  // persistent: workgroups; otherwise: tiles
    bool save_f;    // some instance saves pre-collision populations
    int bnd_grid;
    int ring;       // rows of loads per lane of the main pass (2, 3, 4)
    int red_grid;
    hipStream_t stream;
};
void launch_batch_f64(const BatchLaunch& L);
void launch_batch_f32(const BatchLaunch& L);
void launch_batch_reduce(const BatchLaunch& L);
// resident workgroups per CU of the batched main kernel
int batch_occupancy_f64(int eos, int storage, int tile_w, bool save_f, int ring);
int batch_occupancy_f32(int eos, int storage, int tile_w, bool save_f, int ring);

}  // namespace lbm
