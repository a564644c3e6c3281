// Launcher bodies, instantiated once per storage precision.
#pragma once

#include "launch.hpp"

namespace lbm {

template <typename R>
Phys<R> convert(const Phys<double>& d) {
    Phys<R> p;
    p.G = R(d.G);
    p.gx = R(d.gx);
    p.gy = R(d.gy);
    p.e0 = R(d.e0);
    p.e1 = R(d.e1);
    p.e2 = R(d.e2);
    p.e3 = R(d.e3);
    p.p2G = R(d.p2G);
    p.rref = R(d.rref);
    for (int i = 0; i < 9; ++i) p.s[i] = R(d.s[i]);
    return p;
}

template <typename S, typename R, int EOS, bool MOM, bool DEV>
void main_t(const Ctx& c, const S* src, S* dst) {
    MainArgs<S> a{};
    a.src = src;
    a.dst = dst;
    a.flags = c.flags;
    a.psiw = c.psiw;
    a.side_idx = c.side_idx;
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
    hipLaunchKernelGGL((k_main<S, R, EOS, MOM, DEV>), dim3(c.nblocks), dim3(c.tile_w), 0,
                       c.stream, a, convert<R>(c.ph));
}

template <typename S, typename R, bool MOM, bool DEV>
void main_s(const Ctx& c, const void* src, void* dst) {
    const S* s = static_cast<const S*>(src);
    S* t = static_cast<S*>(dst);
    if (c.eos == EOS_NONE) main_t<S, R, EOS_NONE, MOM, DEV>(c, s, t);
    else if (c.eos == EOS_EXP) main_t<S, R, EOS_EXP, MOM, DEV>(c, s, t);
    else main_t<S, R, EOS_CS, MOM, DEV>(c, s, t);
}

template <typename S, typename R, bool DEV = false>
void main_any(const Ctx& c, const void* src, void* dst, bool moments) {
    if (moments) main_s<S, R, true, DEV>(c, src, dst);
    else main_s<S, R, false, DEV>(c, src, dst);
}

template <typename S, bool DEV = false>
void boundary_any(const Ctx& c, void* cur, const BndArgs& b, int nblocks) {
    hipLaunchKernelGGL((k_boundary<S, DEV>), dim3(nblocks), dim3(256), 0, c.stream,
                       static_cast<S*>(cur), b);
}

template <typename S, typename R>
void init_any(const Ctx& c, const double* rw, const double* r0, const double* u0,
              const double* v0, void* buf) {
    const dim3 g((c.nx + 255) / 256, c.ny);
    const Phys<R> ph = convert<R>(c.ph);
    R* psiw = static_cast<R*>(c.psiw);
    if (c.eos == EOS_EXP)
        hipLaunchKernelGGL((k_psi_wall<R, EOS_EXP>), g, dim3(256), 0, c.stream, psiw, rw,
                           c.flags, c.nx, c.ny, c.pitch, ph);
    else if (c.eos == EOS_CS)
        hipLaunchKernelGGL((k_psi_wall<R, EOS_CS>), g, dim3(256), 0, c.stream, psiw, rw,
                           c.flags, c.nx, c.ny, c.pitch, ph);
    else
        hipLaunchKernelGGL((k_psi_wall<R, EOS_NONE>), g, dim3(256), 0, c.stream, psiw, rw,
                           c.flags, c.nx, c.ny, c.pitch, ph);
    hipLaunchKernelGGL(k_init_scatter<S>, g, dim3(256), 0, c.stream, static_cast<S*>(buf),
                       c.flags, r0, u0, v0, c.nx, c.ny, c.pitch, c.plane, c.ph.rref);
}

}  // namespace lbm
