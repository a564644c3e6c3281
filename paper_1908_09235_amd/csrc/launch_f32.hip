// FP32 storage, with FP64 arithmetic (LBM_STORE_F32) or FP32 arithmetic
// (LBM_STORE_F32_ARITH32).  Built with fused multiply-adds allowed.
#include "launch_impl.hpp"

namespace lbm {

void launch_main_f32(const Ctx& c, const void* src, void* dst, bool moments) {
    if (c.storage == 2) main_any<float, float>(c, src, dst, moments);
    else main_any<float, double>(c, src, dst, moments);
}
void launch_boundary_f32(const Ctx& c, void* cur, const BndArgs& b, int nblocks) {
    boundary_any<float>(c, cur, b, nblocks);
}
void launch_init_f32(const Ctx& c, const double* rw, const double* r0, const double* u0,
                     const double* v0, void* buf) {
    if (c.storage == 2) init_any<float, float>(c, rw, r0, u0, v0, buf);
    else init_any<float, double>(c, rw, r0, u0, v0, buf);
}

}  // namespace lbm
