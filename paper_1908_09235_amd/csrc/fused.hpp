// Two time steps per pass.
//
// One launch advances f*(t) to f*(t + 2): the populations of the
// intermediate step never reach HBM, so a node's populations are read and
// written once per two updates instead of twice.  The boundary pass of
// step t (k_boundary) has written the incoming populations of step t + 1
// into the ghost slots of f*(t), as for a single step; the wall rules and
// the corrections of step t + 2 (Eqs. 7-15, 18, 20-23) are evaluated
// inside the pass from f*(t + 1) and the moments of t + 1, with the same
// arithmetic as the boundary pass (link_value), and enter the pull of
// step t + 2 directly.  Every value is computed exactly as two single
// steps compute it, so the results are bit-identical to them.
//
// Layout of the work: a workgroup is one wavefront of 64 lanes that owns a
// strip of 56 columns (lane j holds column x0 - 4 + j; the four columns
// on either side only feed the strip's interior) and marches upward
// through the rows of its segment.  Per row it pulls f(t + 1) from HBM (two
// rows of loads in flight, as in the single-step kernel) and forms
// psi(t + 1); collides step t + 1 one row behind into LDS rings of three
// rows of f*(t + 1), of the moments of t + 1 and of the flags; evaluates
// the wall rules of the boundary nodes of the row before that, pulls its
// f(t + 2) from the ring and forms psi(t + 2); and collides step t + 2 one
// row later still, storing f*(t + 2) of the strip's own columns and rows.
// Row k of the march is absolute row y0 - 3 + k.  The three-row rings keep
// the LDS per wavefront small enough for more wavefronts per CU; the
// quadratic interpolation rule, which reads a fluid node two rows from the
// boundary node (x_ff), falls outside them and is not fused.
#pragma once

#include "kernels.hpp"

namespace lbm {

constexpr int kF2Lanes = 64;                         // one wavefront
constexpr int kF2Halo = 4;                           // feed-only columns per side
constexpr int kF2Cols = kF2Lanes - 2 * kF2Halo;      // columns a strip updates

template <typename S>
struct Main2Args {
    const S* __restrict__ src;            // f*(t), ghosts of step t + 1 written
    S* __restrict__ dst;                  // f*(t + 2)
    const uint8_t* __restrict__ flags;
    const int* __restrict__ side_idx;     // per node (pitch layout), flagged only
    const int* __restrict__ node_link;    // per node: first link slot + 1, or 0
    const int* __restrict__ order;        // tile of each workgroup (null: XCD order)
    const float* __restrict__ psiw;       // FP16 storage: psi_w of solid nodes
    double* __restrict__ side_mom;        // moments of t + 2 of flagged nodes
    double* __restrict__ partial1;        // per workgroup: mass at t + 1
    double* __restrict__ partial2;        // per workgroup: mass at t + 2
    const int* __restrict__ lmeta;        // link tables (see BndArgs)
    const double* __restrict__ lc;
    const double* __restrict__ luw;
    unsigned long long* __restrict__ negrest;
    unsigned long long* __restrict__ degen;
    int fix;
    int nx, ny, pitch;
    long long plane;
    int tile_h, nsegs, nstrips;
    unsigned side_mom_bytes;
};

template <typename S>
struct Row2Load {
    S f[9];
    uint8_t fl;
    int si;     // side slot (flagged nodes)
    int nl;     // first link slot + 1 (boundary nodes), else 0
    float pw;   // FP16 storage: psi_w of a solid node in FP32
};

// The pulled populations of step t + 2 of one row, in the stored form.
template <typename S>
struct Pull2 {
    S f[9];
};

// (at least three wavefronts per SIMD: 168 registers; the Carnahan-Starling
// variants fit without spilling in FP32 storage, the FP16 ones spill 12
// bytes per lane and still run faster than at two wavefronts)
template <typename S, typename R, int EOS, int DEV>
__global__ __launch_bounds__(kF2Lanes) __attribute__((amdgpu_waves_per_eu(3))) void k_main2(
    Main2Args<S> a, Phys<R> ph) {
    static_assert(DEV == 0 || DEV == 1, "per-node references are not fused");
    // ring rows of f*(t + 1), of the moments of t + 1 and of the flags: the
    // rows m - 1 .. m + 1 around the row m being pulled, the newest being
    // the row just collided
    constexpr int N1 = 3, NM = 3;
    __shared__ S fs1[N1][9][kF2Lanes];
    // moments of t + 1 in the arithmetic type: rho (its deviation from the
    // reference density with one reference; psi of the wall density at a
    // solid node), u_x, u_y -- the wall rules widen them to FP64 exactly
    __shared__ R mo1[NM][3][kF2Lanes];
    __shared__ R ps1[3][kF2Lanes];
    __shared__ R ps2[3][kF2Lanes];
    // per lane and ring row: flags | (first link slot + 1) << 8, and the
    // side slot (kept in LDS rather than carried in registers, so that no
    // loaded value is copied around the loop while loads are in flight)
    __shared__ int mfl[NM][kF2Lanes];
    __shared__ int msi[NM][kF2Lanes];
    constexpr unsigned ES = sizeof(S);

    const unsigned pitch = (unsigned)a.pitch;
    const unsigned pb = (unsigned)(a.plane * ES);
    const rsrc_t rs = make_rsrc(a.src, 9u * pb);
    const rsrc_t rd = make_rsrc(a.dst, 9u * pb);
    const rsrc_t rfl = make_rsrc(a.flags, pitch * (unsigned)a.ny);
    const rsrc_t rsi = make_rsrc(a.side_idx, pitch * (unsigned)a.ny * 4u);
    const rsrc_t rnl = make_rsrc(a.node_link, pitch * (unsigned)a.ny * 4u);
    const rsrc_t rsm = make_rsrc(a.side_mom, a.side_mom_bytes);
    const rsrc_t rpw = make_rsrc(a.psiw, ES == 2 ? pitch * (unsigned)a.ny * 4u : 0u);

    const int j = threadIdx.x;
    const int tile = a.order ? a.order[blockIdx.x] : xcd_tile(blockIdx.x, gridDim.x);
    const int seg = tile / a.nstrips, strip = tile - seg * a.nstrips;
    const int x0 = (int)(((unsigned long long)strip * (unsigned)a.nx) / (unsigned)a.nstrips);
    const int ncols =
        (int)(((unsigned long long)(strip + 1) * (unsigned)a.nx) / (unsigned)a.nstrips) - x0;
    const bool outc = j >= kF2Halo && j < kF2Halo + ncols;
    int xi = (x0 - kF2Halo + j) % a.nx;
    xi = xi < 0 ? xi + a.nx : xi;
    const unsigned x = (unsigned)xi;
    const unsigned xm = x == 0 ? a.nx - 1 : x - 1;
    const unsigned xp = x == (unsigned)a.nx - 1 ? 0 : x + 1;
    const int y0 = seg * a.tile_h;
    const int H = min(a.tile_h, a.ny - y0);
    auto row_of = [&](int k) {
        int y = (y0 - 3 + k) % a.ny;
        return y < 0 ? y + a.ny : y;
    };
    // neighbouring lanes (clamped: the edge lanes only feed the interior)
    auto lane = [](int l) { return l < 0 ? 0 : (l > kF2Lanes - 1 ? kF2Lanes - 1 : l); };
    auto r1 = [](int k) { return (k + 2 * N1) % N1; };
    auto rm = [](int k) { return (k + 2 * NM) % NM; };
    auto r3 = [](int k) { return (k + 6) % 3; };

    // ---- step t + 1: loads, psi, collision (as main_tile)
    uint8_t nfl;
    auto load_flags = [&](int k) { nfl = bload<uint8_t>(rfl, x, (unsigned)row_of(k) * pitch); };
    // pulled rows 0 .. H + 5 feed psi(t + 1); later ones move nothing
    auto issue = [&](int k, Row2Load<S>& L) {
        const int y = row_of(k);
        const bool rv = k <= H + 5;
        const uint8_t fl = rv ? nfl : uint8_t(FL_SOLID);
        L.fl = fl;
        load_flags(k + 1);
        const bool fluid = !(fl & FL_SOLID);
        const unsigned r0 = (unsigned)y * pitch * ES;
        const unsigned rmo = (unsigned)(y == 0 ? a.ny - 1 : y - 1) * pitch * ES;
        const unsigned rpo = (unsigned)(y == a.ny - 1 ? 0 : y + 1) * pitch * ES;
        const unsigned vc = fluid ? x * ES : kOOB, vm = fluid ? xm * ES : kOOB,
                       vp = fluid ? xp * ES : kOOB;
        // plane 0 of the node itself: the rest population, or psi_w if solid
        L.f[0] = bload<S>(rs, rv ? x * ES : kOOB, r0);
        L.f[1] = bload<S>(rs, vm, 1 * pb + r0);
        L.f[2] = bload<S>(rs, vc, 2 * pb + rmo);
        L.f[3] = bload<S>(rs, vp, 3 * pb + r0);
        L.f[4] = bload<S>(rs, vc, 4 * pb + rpo);
        L.f[5] = bload<S>(rs, vm, 5 * pb + rmo);
        L.f[6] = bload<S>(rs, vp, 6 * pb + rmo);
        L.f[7] = bload<S>(rs, vp, 7 * pb + rpo);
        L.f[8] = bload<S>(rs, vm, 8 * pb + rpo);
        if constexpr (ES == 2)
            L.pw = bload<float>(rpw, (rv && !fluid) ? x * 4u : kOOB, (unsigned)y * pitch * 4u);
        // side slot and first link (+ 1) of a flagged node; every lane
        // issues both loads (an offset out of range reads 0), so that the
        // number of loads in flight is the same on every path and the
        // waits before a use stay exact
        const bool side = fluid && (fl & FL_SAVE_MOM);
        const unsigned so = side ? x * 4u : kOOB;
        L.si = bload<int>(rsi, so, (unsigned)y * pitch * 4u);
        L.nl = bload<int>(rnl, so, (unsigned)y * pitch * 4u);
    };
    auto decode = [&](const S* g, R f[9]) {
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = R(g[q]);
    };
    auto psi_w = [&](const Row2Load<S>& L) { return ES == 2 ? R(L.pw) : R(L.f[0]); };
    auto publish1 = [&](const Row2Load<S>& L, int k) {
        R f[9];
        decode(L.f, f);
        const R rho = DEV == 1 ? ph.rref + dens<R>(f) : dens<R>(f);
        ps1[r3(k)][j] = (L.fl & FL_SOLID) ? psi_w(L) : psi_of<EOS, R>(rho, ph);
    };
    auto psis = [&](R(*ring)[kF2Lanes], int km, int k0, int kp, R ps[9]) {
        const int cl = lane(j - 1), cr = lane(j + 1);
        ps[0] = ring[k0][j];
        ps[1] = ring[k0][cr];
        ps[2] = ring[kp][j];
        ps[3] = ring[k0][cl];
        ps[4] = ring[km][j];
        ps[5] = ring[kp][cr];
        ps[6] = ring[kp][cl];
        ps[7] = ring[km][cl];
        ps[8] = ring[km][cr];
    };

    double msum1 = 0.0, msum2 = 0.0;
    Pull2<S> fcur{}, fnxt{};      // pulled f(t + 2) of rows k - 2 and k - 1

    // the wall rules of step t + 2 for the boundary node of lane j in row m
    // (march index), applied to its pulled populations f
    auto links = [&](int m, int nl, bool own, Pull2<S>& f) {
        const bool bnd = nl > 0;
        if (!__builtin_amdgcn_ballot_w64(bnd)) return;
        const int slot = r1(m);
        auto fst = [&](int q, int row, int l) {
            const double v = double(fs1[r1(row)][q][lane(l)]);
            return DEV == 1 ? v + wt(q) * double(ph.rref) : v;
        };
        const double m0 = double(mo1[rm(m)][0][j]);
        const double rho_b = DEV == 1 ? double(ph.rref) + m0 : m0;
        const double ubx = double(mo1[rm(m)][1][j]), uby = double(mo1[rm(m)][2][j]);
        const int i0 = bnd ? nl - 1 : 0;
        const int len = bnd ? (a.lmeta[i0] >> 8) & 15 : 0;
        auto eval = [&](int i, double& fab, double& ch, double& bk, double& wl, int& d) {
            const int meta = a.lmeta[i];
            d = meta & 15;
            const int kind = (meta >> 4) & 15;
            double c[7];
#pragma unroll
            for (int q = 0; q < 7; ++q) c[q] = a.lc[8 * i + q];
            const double uwx = a.luw[2 * i], uwy = a.luw[2 * i + 1];
            const int od = opp(d), dx = cx(d), dy = cy(d);
            fab = fst(d, m, j);
            return link_value(kind, d, c, uwx, uwy, fab, rho_b, ubx, uby, ch, bk, wl,
                              [&](int what) -> double {
                                  switch (what) {
                                  case LV_OD_B: return fst(od, m, j);
                                  case LV_D_F: return fst(d, m - dy, j - dx);
                                  // (x_ff lies two rows away, outside the
                                  // ring: the quadratic rule is not fused)
                                  case LV_D_FF: return NAN;
                                  case LV_OD_F: return fst(od, m - dy, j - dx);
                                  case LV_UFX: return double(mo1[rm(m - dy)][1][lane(j - dx)]);
                                  case LV_UFY: return double(mo1[rm(m - dy)][2][lane(j - dx)]);
                                  default: return 0.0;  // LV_PRE: Zhao-Yong is not fused
                                  }
                              });
        };
        double rho_s = NAN;
        double out_sum = 0.0, in_sum = 0.0;
        if (a.fix == 2 || a.fix == 3) {
            // scheme B, Eq. 22 (chi inside the sums), or Bao et al., Eq. 23
            double num = 0.0, den = 0.0, mag = 0.0;
            for (int l = 0; l < len; ++l) {
                double fab, ch, bk, wl;
                int d;
                (void)eval(i0 + l, fab, ch, bk, wl, d);
                if (a.fix == 2) {
                    num += ch * fab;
                    den += ch * bk;
                    mag += fabs(ch * bk);
                } else {
                    num += fab;
                    den += bk;
                    mag += fabs(bk);
                }
            }
            if (den != 0.0 && fabs(den) > 1e-12 * mag) rho_s = num / den;
            else if (bnd && own && mag > 0.0 && a.degen) atomicAdd(a.degen, 1ull);
        }
        for (int l = 0; l < len; ++l) {
            double fab, ch, bk, wl;
            int d;
            double r = eval(i0 + l, fab, ch, bk, wl, d);
            if (!isnan(rho_s)) r = (1.0 - ch) * fab + ch * (rho_s * bk) - wl;
            out_sum += fab;
            in_sum += r + wl;
            // the incoming population, as the ghost slot would hold it
            const S g = S(r - (DEV == 1 ? wt(d) * double(ph.rref) : 0.0));
            const int od = opp(d);
#pragma unroll
            for (int q = 1; q < 9; ++q)
                if (q == od) f.f[q] = g;
        }
        if (bnd && a.fix == 1) {
            // Eq. (15) without the wall momentum, added to the rest
            // population (Eq. 18)
            const double v = double(fs1[slot][0][j]) + (out_sum - in_sum);
            f.f[0] = S(v);
            if (own && a.negrest) {
                const double f0 = DEV == 1 ? v + wt(0) * double(ph.rref) : v;
                if (f0 < 0.0) atomicAdd(a.negrest, 1ull);
            }
        }
    };

    // row k of the march: psi(t + 1) of row k + 1; step t + 1 of row k;
    // wall rules, pull and psi of step t + 2 of row k - 1; step t + 2 of
    // row k - 2; then the loads of row k + 3 into Lc
    auto step = [&](int k, Row2Load<S>& Lc, Row2Load<S>& Ln) {
        publish1(Ln, k + 1);
        __syncthreads();
        // -- step t + 1, row k (absolute rows y0 - 2 .. y0 + H + 1)
        if (k <= H + 4) {
            const bool fluid = !(Lc.fl & FL_SOLID);
            R fc[9];
            decode(Lc.f, fc);
            R ps[9];
            psis(ps1, r3(k - 1), r3(k), r3(k + 1), ps);
            R rho, drho, ux, uy, Fx, Fy;
            node_moments<R, EOS, DEV>(fc, ps, ph, rho, drho, ux, uy, Fx, Fy);
            const double rho_d = DEV == 1 ? double(ph.rref) + double(drho) : double(rho);
            msum1 += (fluid && outc && k >= 3 && k < H + 3) ? rho_d : 0.0;
            R dh[9];
            collide<R>(fc, rho, drho, ux, uy, Fx, Fy, ph, dh);
            const int s = r1(k);
#pragma unroll
            for (int q = 0; q < 9; ++q) fs1[s][q][j] = fluid ? S(fc[q] + dh[q]) : S(0);
            // (a solid node keeps psi of its wall density in the density slot)
            mo1[rm(k)][0][j] = fluid ? (DEV == 1 ? drho : rho) : psi_w(Lc);
            mo1[rm(k)][1][j] = fluid ? ux : R(0);
            mo1[rm(k)][2][j] = fluid ? uy : R(0);
            mfl[rm(k)][j] = int(Lc.fl) | (Lc.nl << 8);
            msi[rm(k)][j] = Lc.si;
        }
        __syncthreads();
        // -- step t + 2: wall rules, pull and psi of row m = k - 1
        // (absolute rows y0 - 1 .. y0 + H)
        const int m = k - 1;
        if (m >= 2 && m <= H + 3) {
            const int mf = mfl[rm(m)][j];
            const bool fluid = !(mf & FL_SOLID);
#pragma unroll
            for (int q = 0; q < 9; ++q) fnxt.f[q] = fs1[r1(m - cy(q))][q][lane(j - cx(q))];
            links(m, fluid ? (mf >> 8) : 0, outc && m >= 3 && m < H + 3, fnxt);
            R f[9];
            decode(fnxt.f, f);
            const R rho = DEV == 1 ? ph.rref + dens<R>(f) : dens<R>(f);
            ps2[r3(m)][j] = fluid ? psi_of<EOS, R>(rho, ph) : mo1[rm(m)][0][j];
        }
        __syncthreads();
        // -- step t + 2, row n = k - 2 (absolute rows y0 .. y0 + H - 1)
        const int n = k - 2;
        if (n >= 3 && n < H + 3) {
            const int nf = mfl[rm(n)][j];
            const bool live = outc && !(nf & FL_SOLID);
            R fc[9];
            decode(fcur.f, fc);
            R ps[9];
            psis(ps2, r3(n - 1), r3(n), r3(n + 1), ps);
            R rho, drho, ux, uy, Fx, Fy;
            node_moments<R, EOS, DEV>(fc, ps, ph, rho, drho, ux, uy, Fx, Fy);
            const double rho_d = DEV == 1 ? double(ph.rref) + double(drho) : double(rho);
            msum2 += live ? rho_d : 0.0;
            const bool sm = live && (nf & FL_SAVE_MOM);
            if (__builtin_amdgcn_ballot_w64(sm)) {
                const unsigned so = sm ? (unsigned)msi[rm(n)][j] * 24u : kOOB;
                bstore(rho_d, rsm, so, 0u);
                bstore(double(ux), rsm, so + 8u, 0u);
                bstore(double(uy), rsm, so + 16u, 0u);
            }
            R dh[9];
            collide<R>(fc, rho, drho, ux, uy, Fx, Fy, ph, dh);
            const unsigned r0 = (unsigned)row_of(n) * pitch * ES;
            const unsigned vo = live ? x * ES : kOOB;
#pragma unroll
            for (int q = 0; q < 9; ++q) bstore(S(fc[q] + dh[q]), rd, vo, q * pb + r0);
        }
        fcur = fnxt;
        issue(k + 3, Lc);  // Lc is free again
    };

    Row2Load<S> A, B, C;
    load_flags(0);
    issue(0, C);
    issue(1, A);
    issue(2, B);
    publish1(C, 0);
    issue(3, C);
    publish1(A, 1);
    // a whole number of three-row rotations over rows 1 .. H + 4
    const int K3 = (H + 4 + 2) / 3 * 3;
    for (int k = 1; k < 1 + K3; k += 3) {
        step(k, A, B);
        step(k + 1, B, C);
        step(k + 2, C, A);
    }

    // fixed-order wavefront reductions of the two mass partials
    double v1 = msum1, v2 = msum2;
    for (int off = 32; off > 0; off >>= 1) {
        v1 += __shfl_down(v1, off, 64);
        v2 += __shfl_down(v2, off, 64);
    }
    if (j == 0) {
        a.partial1[tile] = v1;
        a.partial2[tile] = v2;
    }
}

}  // namespace lbm
