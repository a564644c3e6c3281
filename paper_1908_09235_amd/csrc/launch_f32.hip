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

}  // namespace lbm
