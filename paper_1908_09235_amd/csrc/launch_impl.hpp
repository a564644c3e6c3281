// Launcher bodies, instantiated once per storage precision.
#pragma once

#include <hip/hip_ext.h>

#include "launch.hpp"

namespace lbm {

template <typename R>
Phys<R> convert(const Phys<double>& d) {
    return phys_as<R>(d);
}

// A launch on c.stream, timed by the dispatch itself when c carries events.
template <typename K, typename... A>
void launch_on(const Ctx& c, K kernel, dim3 grid, dim3 block, A... args) {
    if (c.ev_start)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, c.stream, c.ev_start, c.ev_stop, 0u,
                              args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, c.stream, args...);
}

template <typename S, typename R, int EOS, bool MOM, int DEV, bool SAVEF>
void main_t(const Ctx& c, const S* src, S* dst) {
    MainArgs<S> a{};
    a.src = src;
    a.dst = dst;
    a.flags = c.flags;
    a.side_idx = c.side_idx;
    a.psiw = c.psiw;
    a.side_mom = c.side_mom;
    a.side_f = c.side_f;
    a.partial = c.partial;
    a.mom_out = c.mom_out;
    a.nx = c.nx;
    a.ny = c.ny;
    a.pitch = c.pitch;
    a.plane = c.plane;
    a.tile_h = c.tile_h;
    a.nsegs = c.nsegs;
    a.nstrips = c.nstrips;
    a.side_mom_bytes = c.side_mom_bytes;
    a.side_f_bytes = c.side_f_bytes;
    launch_on(c, k_main<S, R, EOS, MOM, DEV, SAVEF>, dim3(c.nblocks), dim3(c.tile_w), a,
              convert<R>(c.ph));
}

template <typename S, typename R, bool MOM, int DEV, bool SAVEF>
void main_e(const Ctx& c, const S* s, S* t) {
    if (c.eos == EOS_NONE) main_t<S, R, EOS_NONE, MOM, DEV, SAVEF>(c, s, t);
    else if (c.eos == EOS_EXP) main_t<S, R, EOS_EXP, MOM, DEV, SAVEF>(c, s, t);
    else main_t<S, R, EOS_CS, MOM, DEV, SAVEF>(c, s, t);
}

template <typename S, typename R, int DEV = 0>
void main_any(const Ctx& c, const void* src, void* dst, bool moments) {
    const S* s = static_cast<const S*>(src);
    S* t = static_cast<S*>(dst);
    if (moments) main_e<S, R, true, DEV, false>(c, s, t);
    else if (c.save_f) main_e<S, R, false, DEV, true>(c, s, t);
    else main_e<S, R, false, DEV, false>(c, s, t);
}

template <typename S, typename R, int EOS, int DEV>
void main2_t(const Ctx& c, const S* src, S* dst) {
    Main2Args<S> a{};
    a.src = src;
    a.dst = dst;
    a.flags = c.flags;
    a.side_idx = c.side_idx;
    a.node_link = c.node_link;
    a.order = c.tile_order;
    a.psiw = c.psiw;
    a.side_mom = c.side_mom;
    a.partial1 = c.partial;
    a.partial2 = c.partial2;
    a.lmeta = c.lmeta;
    a.lc = c.lc;
    a.luw = c.luw;
    a.negrest = c.negrest;
    a.degen = c.degen;
    a.fix = c.fix;
    a.nx = c.nx;
    a.ny = c.ny;
    a.pitch = c.pitch;
    a.plane = c.plane;
    a.tile_h = c.tile_h2;
    a.nsegs = c.nsegs2;
    a.nstrips = c.nstrips2;
    a.side_mom_bytes = c.side_mom_bytes;
    launch_on(c, k_main2<S, R, EOS, DEV>, dim3(c.nblocks2), dim3(kF2Lanes), a,
              convert<R>(c.ph));
}

template <typename S, typename R, int DEV>
void main2_any(const Ctx& c, const void* src, void* dst) {
    const S* s = static_cast<const S*>(src);
    S* t = static_cast<S*>(dst);
    if (c.eos == EOS_NONE) main2_t<S, R, EOS_NONE, DEV>(c, s, t);
    else if (c.eos == EOS_EXP) main2_t<S, R, EOS_EXP, DEV>(c, s, t);
    else main2_t<S, R, EOS_CS, DEV>(c, s, t);
}

template <typename S, int DEV = 0>
void boundary_any(const Ctx& c, void* cur, const BndArgs& b, int nblocks) {
    launch_on(c, k_boundary<S, DEV>, dim3(nblocks), dim3(256), static_cast<S*>(cur), b);
}

template <typename S, typename R>
void init_any(const Ctx& c, const double* rw, const double* r0, const double* u0,
              const double* v0, void* buf, void* other) {
    const dim3 g((c.nx + 255) / 256, c.ny);
    const Phys<R> ph = convert<R>(c.ph);
    S* b0 = static_cast<S*>(buf);
    S* b1 = static_cast<S*>(other);
    if (c.eos == EOS_EXP)
        hipLaunchKernelGGL((k_psi_wall<S, R, EOS_EXP>), g, dim3(256), 0, c.stream, b0, b1, c.psiw, rw,
                           c.flags, c.nx, c.ny, c.pitch, ph);
    else if (c.eos == EOS_CS)
        hipLaunchKernelGGL((k_psi_wall<S, R, EOS_CS>), g, dim3(256), 0, c.stream, b0, b1, c.psiw, rw,
                           c.flags, c.nx, c.ny, c.pitch, ph);
    else
        hipLaunchKernelGGL((k_psi_wall<S, R, EOS_NONE>), g, dim3(256), 0, c.stream, b0, b1, c.psiw, rw,
                           c.flags, c.nx, c.ny, c.pitch, ph);
    hipLaunchKernelGGL(k_init_scatter<S>, g, dim3(256), 0, c.stream, b0, c.flags, r0, u0, v0,
                       c.nx, c.ny, c.pitch, c.plane, c.ph.rref, c.ref);
}

template <typename S, typename R, int DEV, bool SAVEF, int RING>
void batch_main_r(const BatchLaunch& L) {
    if (L.eos == EOS_EXP)
        hipLaunchKernelGGL((k_main_batch<S, R, EOS_EXP, DEV, SAVEF, RING>), dim3(L.main_grid),
                           dim3(L.tile_w), 0, L.stream, L.args);
    else if (L.eos == EOS_CS)
        hipLaunchKernelGGL((k_main_batch<S, R, EOS_CS, DEV, SAVEF, RING>), dim3(L.main_grid),
                           dim3(L.tile_w), 0, L.stream, L.args);
    else
        hipLaunchKernelGGL((k_main_batch<S, R, EOS_NONE, DEV, SAVEF, RING>), dim3(L.main_grid),
                           dim3(L.tile_w), 0, L.stream, L.args);
}

// rows of loads per lane: the ring L.ring (the FP16 per-node form: 3 only)
template <typename S, typename R, int DEV, bool SAVEF>
void batch_main(const BatchLaunch& L) {
    if constexpr (DEV == 2) {
        batch_main_r<S, R, DEV, SAVEF, 3>(L);
    } else {
        if (L.ring == 2) batch_main_r<S, R, DEV, SAVEF, 2>(L);
        else if (L.ring == 4) batch_main_r<S, R, DEV, SAVEF, 4>(L);
        else batch_main_r<S, R, DEV, SAVEF, 3>(L);
    }
}

template <typename S, typename R, int DEV>
void batch_any(const BatchLaunch& L) {
    hipLaunchKernelGGL((k_boundary_batch<S, DEV>), dim3(L.bnd_grid), dim3(256), 0, L.stream,
                       L.args);
    if (L.save_f) batch_main<S, R, DEV, true>(L);
    else batch_main<S, R, DEV, false>(L);
}

template <typename S, typename R, int DEV, bool SAVEF, int RING>
int occupancy_e(int eos, int tile_w) {
    int n = 0;
    hipError_t e;
    if (eos == EOS_EXP)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(k_main_batch<S, R, EOS_EXP, DEV, SAVEF, RING>),
            tile_w, 0);
    else if (eos == EOS_CS)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(k_main_batch<S, R, EOS_CS, DEV, SAVEF, RING>),
            tile_w, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(k_main_batch<S, R, EOS_NONE, DEV, SAVEF, RING>),
            tile_w, 0);
    return e == hipSuccess ? n : 0;
}

template <typename S, typename R, int DEV>
int occupancy_any(int eos, int tile_w, bool save_f, int ring) {
    if constexpr (DEV != 2) {
        if (ring == 2)
            return save_f ? occupancy_e<S, R, DEV, true, 2>(eos, tile_w)
                          : occupancy_e<S, R, DEV, false, 2>(eos, tile_w);
        if (ring == 4)
            return save_f ? occupancy_e<S, R, DEV, true, 4>(eos, tile_w)
                          : occupancy_e<S, R, DEV, false, 4>(eos, tile_w);
    }
    return save_f ? occupancy_e<S, R, DEV, true, 3>(eos, tile_w)
                  : occupancy_e<S, R, DEV, false, 3>(eos, tile_w);
}

}  // namespace lbm
