// FP32 storage with FP64 arithmetic (LBM_STORE_F32) or FP32 arithmetic
// (LBM_STORE_F32_ARITH32); FP32 or FP16 deviations g = f - w rho_ref with
// FP32 arithmetic (LBM_STORE_F32DEV, LBM_STORE_F16DEV); FP16 deviations
// from a per-node reference (LBM_STORE_F16NODE).  Built with
// -ffp-contract=off: every product and sum rounds as written (the FP16
// per-node decode fuses its multiply-adds explicitly), so that a kernel's
// arithmetic does not depend on what the compiler would contract where,
// and the two-steps-per-pass kernel rounds exactly as two single steps.
#include "launch_impl.hpp"

namespace lbm {

void launch_main_f32(const Ctx& c, const void* src, void* dst, bool moments) {
    switch (c.storage) {
    case 2: main_any<float, float>(c, src, dst, moments); break;
    case 3: main_any<float, float, 1>(c, src, dst, moments); break;
    case 4: main_any<_Float16, float, 1>(c, src, dst, moments); break;
    case 5: main_any<_Float16, float, 2>(c, src, dst, moments); break;
    default: main_any<float, double>(c, src, dst, moments);
    }
}
void launch_main2_f32(const Ctx& c, const void* src, void* dst) {
    switch (c.storage) {
    case 2: main2_any<float, float, 0>(c, src, dst); break;
    case 3: main2_any<float, float, 1>(c, src, dst); break;
    case 4: main2_any<_Float16, float, 1>(c, src, dst); break;
    default: main2_any<float, double, 0>(c, src, dst);
    }
}
void launch_boundary_f32(const Ctx& c, void* cur, const BndArgs& b, int nblocks) {
    switch (c.storage) {
    case 3: boundary_any<float, 1>(c, cur, b, nblocks); break;
    case 4: boundary_any<_Float16, 1>(c, cur, b, nblocks); break;
    case 5: boundary_any<_Float16, 2>(c, cur, b, nblocks); break;
    default: boundary_any<float>(c, cur, b, nblocks);
    }
}
void launch_init_f32(const Ctx& c, const double* rw, const double* r0, const double* u0,
                     const double* v0, void* buf, void* other) {
    switch (c.storage) {
    case 2: case 3: init_any<float, float>(c, rw, r0, u0, v0, buf, other); break;
    case 4: case 5: init_any<_Float16, float>(c, rw, r0, u0, v0, buf, other); break;
    default: init_any<float, double>(c, rw, r0, u0, v0, buf, other);
    }
}

void launch_batch_f32(const BatchLaunch& L) {
    switch (L.storage) {
    case 2: batch_any<float, float, 0>(L); break;
    case 3: batch_any<float, float, 1>(L); break;
    case 4: batch_any<_Float16, float, 1>(L); break;
    case 5: batch_any<_Float16, float, 2>(L); break;
    default: batch_any<float, double, 0>(L);
    }
}
int batch_occupancy_f32(int eos, int storage, int tile_w, bool save_f, int ring) {
    switch (storage) {
    case 2: return occupancy_any<float, float, 0>(eos, tile_w, save_f, ring);
    case 3: return occupancy_any<float, float, 1>(eos, tile_w, save_f, ring);
    case 4: return occupancy_any<_Float16, float, 1>(eos, tile_w, save_f, ring);
    case 5: return occupancy_any<_Float16, float, 2>(eos, tile_w, save_f, ring);
    default: return occupancy_any<float, double, 0>(eos, tile_w, save_f, ring);
    }
}

}  // namespace lbm
