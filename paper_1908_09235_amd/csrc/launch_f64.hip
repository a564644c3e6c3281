// FP64 storage and arithmetic.  Built with -ffp-contract=off: every product
// and sum rounds as written, in the order the method's formulas give it.
#include "launch_impl.hpp"

namespace lbm {

void launch_main_f64(const Ctx& c, const void* src, void* dst, bool moments) {
    main_any<double, double>(c, src, dst, moments);
}
void launch_boundary_f64(const Ctx& c, void* cur, const BndArgs& b, int nblocks) {
    boundary_any<double>(c, cur, b, nblocks);
}
void launch_init_f64(const Ctx& c, const double* rw, const double* r0, const double* u0,
                     const double* v0, void* buf, void* other) {
    init_any<double, double>(c, rw, r0, u0, v0, buf, other);
}
void launch_reduce(const Ctx& c, bool two, long long cap, long long* clock, double* hist,
                   long long* unstable) {
    hipLaunchKernelGGL(k_reduce<0>, dim3(1), dim3(256), 0, c.stream, c.partial,
                       two ? c.partial2 : nullptr, two ? c.nblocks2 : c.nblocks, hist, cap,
                       clock, unstable);
}

void launch_batch_f64(const BatchLaunch& L) { batch_any<double, double, 0>(L); }
void launch_batch_reduce(const BatchLaunch& L) {
    hipLaunchKernelGGL(k_reduce_batch<0>, dim3(L.red_grid), dim3(256), 0, L.stream, L.args);
}
int batch_occupancy_f64(int eos, int, int tile_w, bool save_f, int ring) {
    return occupancy_any<double, double, 0>(eos, tile_w, save_f, ring);
}

}  // namespace lbm
