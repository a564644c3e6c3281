// FP32 storage with FP64 arithmetic (LBM_STORE_F32) or FP32 arithmetic
// (LBM_STORE_F32_ARITH32); FP32 or FP16 deviations g = f - w rho_ref with
// FP32 arithmetic (LBM_STORE_F32DEV, LBM_STORE_F16DEV).  Built with fused
// multiply-adds allowed.
#include "launch_impl.hpp"

namespace lbm {

void launch_main_f32(const Ctx& c, const void* src, void* dst, bool moments) {
    switch (c.storage) {
    case 2: main_any<float, float>(c, src, dst, moments); break;
    case 3: main_any<float, float, true>(c, src, dst, moments); break;
    case 4: main_any<_Float16, float, true>(c, src, dst, moments); break;
    default: main_any<float, double>(c, src, dst, moments);
    }
}
void launch_boundary_f32(const Ctx& c, void* cur, const BndArgs& b, int nblocks) {
    switch (c.storage) {
    case 3: boundary_any<float, true>(c, cur, b, nblocks); break;
    case 4: boundary_any<_Float16, true>(c, cur, b, nblocks); break;
    default: boundary_any<float>(c, cur, b, nblocks);
    }
}
void launch_init_f32(const Ctx& c, const double* rw, const double* r0, const double* u0,
                     const double* v0, void* buf) {
    switch (c.storage) {
    case 2: case 3: init_any<float, float>(c, rw, r0, u0, v0, buf); break;
    case 4: init_any<_Float16, float>(c, rw, r0, u0, v0, buf); break;
    default: init_any<float, double>(c, rw, r0, u0, v0, buf);
    }
}

void launch_batch_f32(const BatchLaunch& L) {
    switch (L.storage) {
    case 2: batch_any<float, float, false>(L); break;
    case 3: batch_any<float, float, true>(L); break;
    case 4: batch_any<_Float16, float, true>(L); break;
    default: batch_any<float, double, false>(L);
    }
}
int batch_occupancy_f32(int eos, int storage, int tile_w) {
    switch (storage) {
    case 2: return occupancy_any<float, float, false>(eos, tile_w);
    case 3: return occupancy_any<float, float, true>(eos, tile_w);
    case 4: return occupancy_any<_Float16, float, true>(eos, tile_w);
    default: return occupancy_any<float, double, false>(eos, tile_w);
    }
}

}  // namespace lbm
