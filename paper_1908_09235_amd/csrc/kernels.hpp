// Kernels of one time step.
//
// State between steps: buffer `cur` holds the post-collision populations
// f*(t) in structure-of-arrays layout, nine planes of ny rows of `pitch`
// elements.  A step is two launches:
//
//   k_boundary(cur): one thread per boundary node.  For each of the node's
//     cut links it evaluates the wall rule (Eqs. 7-14) from f*(t) and the
//     node's saved moments, then the leak of Eq. (15) and the correction of
//     scheme A, B or Bao, and writes each incoming population into the
//     solid neighbour's slot of the opposite direction (the "ghost" slot:
//     the only slot a pull from the fluid node reads there).  Scheme A adds
//     the leak to the node's own rest population.
//
//   k_main(cur -> nxt): pull-streaming (Eq. 3) of all nine populations,
//     density, pseudopotential, the force of Eq. (16), the velocity of
//     Eq. (5) and collision (Eq. 2), fused.  A workgroup owns a strip of
//     tile_w columns and marches down tile_h rows, keeping psi of three
//     consecutive rows in a four-slot LDS ring; the two halo columns of the
//     strip are recomputed by two lanes.  Solid nodes are neither loaded nor
//     stored.  Boundary nodes (and the x_f nodes that MLS reads) save their
//     moments, and under Zhao-Yong their pre-collision populations, for the
//     next k_boundary.  Each workgroup writes one FP64 partial of the total
//     mass; the next launch reduces the partials in a fixed order.
#pragma once

#include "lattice.hpp"

namespace lbm {

constexpr int kMaxTileW = 256;

enum : uint8_t { FL_SOLID = 1, FL_SAVE_MOM = 2, FL_SAVE_F = 4 };

// wavefronts are handed to the 8 XCDs round robin; map consecutive
// workgroup ids of one XCD to consecutive tiles (vertically adjacent
// segments of a strip) so that they share that XCD's L2
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int xcd = b & 7, idx = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename S>
struct MainArgs {
    const S* __restrict__ src;
    S* __restrict__ dst;
    const uint8_t* __restrict__ flags;  // per node (pitch layout)
    const void* __restrict__ psiw;      // per node, compute type, solid only
    const int* __restrict__ side_idx;   // per node, flagged only
    double* __restrict__ side_mom;      // [slot][3]: rho, ux, uy
    double* __restrict__ side_f;        // [slot][9]: pre-collision f
    double* __restrict__ partial;       // per workgroup
    double* __restrict__ mom_out;       // moments mode: rho, ux, uy planes
    int nx, ny, pitch;
    long long plane;                    // elements per population plane
    int tile_h, nsegs;
};

template <typename R, int EOS>
struct NodeCtx {
    const uint8_t* flags;
    const R* psiw;
    Phys<R> ph;
};

template <typename S, typename R>
__device__ __forceinline__ void pull9(const S* __restrict__ src, long long plane,
                                      int rm, int r0, int rp, int x, int xm,
                                      int xp, R f[9]) {
    // f_a(x, y) = f*_a(x - e_a, y): rows rm = y-1, r0 = y, rp = y+1
    f[0] = R(src[0 * plane + r0 + x]);
    f[1] = R(src[1 * plane + r0 + xm]);
    f[2] = R(src[2 * plane + rm + x]);
    f[3] = R(src[3 * plane + r0 + xp]);
    f[4] = R(src[4 * plane + rp + x]);
    f[5] = R(src[5 * plane + rm + xm]);
    f[6] = R(src[6 * plane + rm + xp]);
    f[7] = R(src[7 * plane + rp + xp]);
    f[8] = R(src[8 * plane + rp + xm]);
}

template <typename R>
__device__ __forceinline__ R dens(const R f[9]) {
    return f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
}

// pull one node and return its psi (solid nodes: the wall value, no loads)
template <typename S, typename R, int EOS>
__device__ __forceinline__ R pull_psi(const MainArgs<S>& a, const R* psiw,
                                      const Phys<R>& ph, int y, int x,
                                      uint8_t& fl, R f[9]) {
    const int ym = y == 0 ? a.ny - 1 : y - 1;
    const int yp = y == a.ny - 1 ? 0 : y + 1;
    const int xm = x == 0 ? a.nx - 1 : x - 1;
    const int xp = x == a.nx - 1 ? 0 : x + 1;
    const int r0 = y * a.pitch;
    fl = a.flags[r0 + x];
    if (fl & FL_SOLID) return psiw[r0 + x];
    pull9<S, R>(a.src, a.plane, ym * a.pitch, r0, yp * a.pitch, x, xm, xp, f);
    return psi_of<EOS, R>(dens<R>(f), ph);
}

// MOMENTS: write rho, u at every node instead of colliding and storing
template <typename S, typename R, int EOS, int COLL, bool MOMENTS>
__global__ __launch_bounds__(256) void k_main(MainArgs<S> a, Phys<R> ph) {
    __shared__ R ring[4][kMaxTileW + 2];
    __shared__ double wsum[kMaxTileW / 64];
    const R* psiw = static_cast<const R*>(a.psiw);

    const int tid = threadIdx.x;
    const int W = blockDim.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int strip = tile / a.nsegs, seg = tile - strip * a.nsegs;
    const int x0 = strip * W;
    const int ncols = min(W, a.nx - x0);
    const bool act = tid < ncols;
    const int x = act ? x0 + tid : x0;
    const bool halo = tid < 2;
    const int hx = tid == 0 ? (x0 == 0 ? a.nx - 1 : x0 - 1)
                            : (x0 + ncols == a.nx ? 0 : x0 + ncols);
    const int hcol = tid == 0 ? 0 : ncols + 1;
    const int y0 = seg * a.tile_h;
    const int y1 = min(y0 + a.tile_h, a.ny);

    R fc[9], fn[9], fh[9];
    uint8_t flc = 0, fln = 0, flh = 0;
    double msum = 0.0;

    // prologue: psi of rows y0-1 (slot 0) and y0 (slot 1)
    {
        const int y = y0 == 0 ? a.ny - 1 : y0 - 1;
        if (act) ring[0][tid + 1] = pull_psi<S, R, EOS>(a, psiw, ph, y, x, fln, fn);
        if (halo) ring[0][hcol] = pull_psi<S, R, EOS>(a, psiw, ph, y, hx, flh, fh);
        if (act) ring[1][tid + 1] = pull_psi<S, R, EOS>(a, psiw, ph, y0, x, flc, fc);
        if (halo) ring[1][hcol] = pull_psi<S, R, EOS>(a, psiw, ph, y0, hx, flh, fh);
    }

    for (int k = 0, y = y0; y < y1; ++k, ++y) {
        const int yn = y == a.ny - 1 ? 0 : y + 1;
        const int sm = k & 3, s0 = (k + 1) & 3, sp = (k + 2) & 3;
        if (act) ring[sp][tid + 1] = pull_psi<S, R, EOS>(a, psiw, ph, yn, x, fln, fn);
        if (halo) ring[sp][hcol] = pull_psi<S, R, EOS>(a, psiw, ph, yn, hx, flh, fh);
        __syncthreads();
        if (act && !(flc & FL_SOLID)) {
            const int c = tid + 1;
            const R rho = dens<R>(fc);
            R Fx = R(0), Fy = R(0);
            if constexpr (EOS != EOS_NONE) {
                // Eq. (16): F = -G psi(x) sum_a w_a psi(x + e_a) e_a
                const R p1 = ring[s0][c + 1], p2 = ring[sp][c], p3 = ring[s0][c - 1];
                const R p4 = ring[sm][c], p5 = ring[sp][c + 1], p6 = ring[sp][c - 1];
                const R p7 = ring[sm][c - 1], p8 = ring[sm][c + 1];
                const R w1 = R(wf(1)), w5 = R(wf(5));
                R sx, sy;
                if constexpr (sizeof(R) == 8) {
                    // the sum in direction order
                    sx = w1 * p1 - w1 * p3 + w5 * p5 - w5 * p6 - w5 * p7 + w5 * p8;
                    sy = w1 * p2 - w1 * p4 + w5 * p5 + w5 * p6 - w5 * p7 - w5 * p8;
                } else {
                    // opposite neighbours paired first: exactly zero where psi
                    // is uniform and exactly odd under reflection, also when
                    // products fuse into multiply-adds
                    sx = w1 * (p1 - p3) + w5 * ((p5 - p7) + (p8 - p6));
                    sy = w1 * (p2 - p4) + w5 * ((p5 - p7) + (p6 - p8));
                }
                const R pc = ring[s0][c];
                Fx = -ph.G * pc * sx;
                Fy = -ph.G * pc * sy;
            }
            Fx = Fx + rho * ph.gx;
            Fy = Fy + rho * ph.gy;
            // Eq. (5)
            const R mx = fc[1] - fc[3] + fc[5] - fc[6] - fc[7] + fc[8];
            const R my = fc[2] - fc[4] + fc[5] + fc[6] - fc[7] - fc[8];
            const R ux = (mx + Fx / R(2)) / rho;
            const R uy = (my + Fy / R(2)) / rho;
            const int idx = y * a.pitch + x;
            if constexpr (MOMENTS) {
                const int o = y * a.nx + x;
                a.mom_out[o] = double(rho);
                a.mom_out[(long long)a.nx * a.ny + o] = double(ux);
                a.mom_out[2LL * a.nx * a.ny + o] = double(uy);
            } else {
                if (sizeof(R) == 8) {
                    msum += double(rho);
                } else {
                    double r = 0.0;
#pragma unroll
                    for (int q = 0; q < 9; ++q) r += double(fc[q]);
                    msum += r;
                }
                if (flc & (FL_SAVE_MOM | FL_SAVE_F)) {
                    const int slot = a.side_idx[idx];
                    if (flc & FL_SAVE_MOM) {
                        a.side_mom[3 * slot + 0] = double(rho);
                        a.side_mom[3 * slot + 1] = double(ux);
                        a.side_mom[3 * slot + 2] = double(uy);
                    }
                    if (flc & FL_SAVE_F) {
#pragma unroll
                        for (int q = 0; q < 9; ++q) a.side_f[9 * slot + q] = double(fc[q]);
                    }
                }
                collide<COLL, R>(fc, rho, ux, uy, Fx, Fy, ph);
#pragma unroll
                for (int q = 0; q < 9; ++q) a.dst[q * a.plane + idx] = S(fc[q]);
            }
        } else if (MOMENTS && act) {
            const int o = y * a.nx + x;
            a.mom_out[o] = 0.0;
            a.mom_out[(long long)a.nx * a.ny + o] = 0.0;
            a.mom_out[2LL * a.nx * a.ny + o] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) fc[q] = fn[q];
        flc = fln;
    }

    if constexpr (!MOMENTS) {
        // fixed-order block reduction of the mass partial
        double v = msum;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((tid & 63) == 0) wsum[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < (W + 63) / 64; ++w) t += wsum[w];
            a.partial[blockIdx.x] = t;
        }
    }
}

// Sum the main kernel's partials in a fixed order into the history ring.
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partial,
                                                int np, double* __restrict__ hist,
                                                long long slot, long long t,
                                                long long* __restrict__ unstable) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int i = tid; i < np; i += 256) v += partial[i];
    red[tid] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        const double m = red[0];
        hist[slot] = m;
        if (!isfinite(m) && *unstable < 0) *unstable = t;
    }
}

template <int Unused = 0>
__global__ __launch_bounds__(256) void k_reduce(const double* partial, int np,
                                                double* hist, long long slot,
                                                long long t, long long* unstable) {
    reduce_partials(partial, np, hist, slot, t, unstable);
}

// ---------------------------------------------------------------- boundary
enum : int {
    LK_HALFWAY = 0,  // f*_a(x_b) - wall
    LK_CHI_UB = 1,   // Eq. 7/8 with u_s = u_b            (FH q < 1/2)
    LK_CHI_UF = 2,   // Eq. 7/8 with u_s = u_f            (MLS q < 1/2)
    LK_CHI_EXT = 3,  // Eq. 7/8 with u_s of Eq. 10        (q >= 1/2)
    LK_LIN_F = 4,    // c1 f*_a(x_b) + c2 f*_a(x_f)
    LK_LIN_B = 5,    // c1 f*_a(x_b) + c2 f*_abar(x_b)
    LK_QUAD_F = 6,   // c1 f*_a(x_b) + c2 f*_a(x_f) - c3 f*_a(x_ff)
    LK_QUAD_B = 7,   // c1 f*_a(x_b) + c2 f*_abar(x_b) - c3 f*_abar(x_f)
    LK_ZY = 8        // c1 f*_abar(x_b) + c2 f_a(x_b)
};

struct BndArgs {
    int nb;                          // boundary nodes
    const int* __restrict__ bnode;   // node index (pitch layout)
    const int* __restrict__ bslot;   // side slot of the node
    const int* __restrict__ bstart;  // CSR into links, nb + 1
    const int* __restrict__ ldir;
    const int* __restrict__ lkind;
    const int* __restrict__ lghost;  // node index of x_s
    const int* __restrict__ lxf;     // node index of x_f (or -1)
    const int* __restrict__ lxff;    // node index of x_ff (or -1)
    const int* __restrict__ lslotf;  // side slot of x_f (or -1)
    const double* __restrict__ lc;   // [link][8]: c1 c2 c3 chi cb uwq_x uwq_y pad
    const double* __restrict__ luw;  // [link][2]: wall velocity
    const double* __restrict__ side_mom;
    const double* __restrict__ side_f;
    long long plane;
    int fix;                         // 0 none, 1 A, 2 B, 3 Bao
    // reduction of the previous main launch's mass partials (last block)
    const double* __restrict__ partial;
    int np;
    double* __restrict__ hist;
    long long slot, t;
    long long* __restrict__ unstable;
    int do_reduce;
};

template <typename S>
__global__ __launch_bounds__(256) void k_boundary(S* __restrict__ A, BndArgs b) {
    if (blockIdx.x == gridDim.x - 1) {
        if (b.do_reduce) reduce_partials(b.partial, b.np, b.hist, b.slot, b.t, b.unstable);
        return;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.nb) return;
    const int node = b.bnode[i];
    const int k0 = b.bstart[i], k1 = b.bstart[i + 1];
    const double* mom = b.side_mom + 3 * b.bslot[i];
    const double rho_b = mom[0], ubx = mom[1], uby = mom[2];
    const long long P = b.plane;

    double inc[8], fab[8], chi[8], br[8], wall[8];
    int n = 0;
    for (int k = k0; k < k1; ++k, ++n) {
        const int d = b.ldir[k];
        const int od = opp(d);
        const double* c = b.lc + 8 * k;
        const double ex = double(cx(d)), ey = double(cy(d));
        const double fa_b = double(A[d * P + node]);
        const double uwx = b.luw[2 * k], uwy = b.luw[2 * k + 1];
        // momentum of a moving wall, Ladd / Mei et al.: 2 w_a rho_b e.u_w / c_s^2
        const double wl = 2.0 * wt(d) * rho_b * 3.0 * (ex * uwx + ey * uwy);
        double r = 0.0, ch = 0.0, bk = 0.0;
        const int kind = b.lkind[k];
        if (kind == LK_HALFWAY) {
            r = fa_b - wl;
        } else if (kind <= LK_CHI_EXT) {
            double usx, usy;
            if (kind == LK_CHI_UB) {
                usx = ubx; usy = uby;
            } else if (kind == LK_CHI_UF) {
                const double* mf = b.side_mom + 3 * b.lslotf[k];
                usx = mf[1]; usy = mf[2];
            } else {
                usx = c[4] * ubx + c[5];
                usy = c[4] * uby + c[6];
            }
            ch = c[3];
            const double eus = edot<double>(d, usx, usy);
            const double eub = edot<double>(d, ubx, uby);
            const double ub2 = ubx * ubx + uby * uby;
            bk = wt(d) * (1.0 + 3.0 * eus + 4.5 * (eub * eub) - 1.5 * ub2);
            r = (1.0 - ch) * fa_b + ch * (rho_b * bk) - wl;
        } else if (kind == LK_LIN_F) {
            r = c[0] * fa_b + c[1] * double(A[d * P + b.lxf[k]]);
        } else if (kind == LK_LIN_B) {
            r = c[0] * fa_b + c[1] * double(A[od * P + node]);
        } else if (kind == LK_QUAD_F) {
            r = c[0] * fa_b + c[1] * double(A[d * P + b.lxf[k]]) -
                c[2] * double(A[d * P + b.lxff[k]]);
        } else if (kind == LK_QUAD_B) {
            r = c[0] * fa_b + c[1] * double(A[od * P + node]) -
                c[2] * double(A[od * P + b.lxf[k]]);
        } else {  // LK_ZY
            const double fpre = b.side_f[9 * b.bslot[i] + d];
            r = c[0] * double(A[od * P + node]) + c[1] * fpre;
        }
        inc[n] = r;
        fab[n] = fa_b;
        chi[n] = ch;
        br[n] = bk;
        wall[n] = wl;
    }
    if (b.fix == 2 || b.fix == 3) {
        // scheme B, Eq. 22 (chi inside the sums) or Bao et al., Eq. 23
        double num = 0.0, den = 0.0, mag = 0.0;
        for (int m = 0; m < n; ++m) {
            if (b.fix == 2) {
                num += chi[m] * fab[m];
                den += chi[m] * br[m];
                mag += fabs(chi[m] * br[m]);
            } else {
                num += fab[m];
                den += br[m];
                mag += fabs(br[m]);
            }
        }
        if (den != 0.0 && fabs(den) > 1e-12 * mag) {
            const double rho_s = num / den;
            for (int m = 0; m < n; ++m)
                inc[m] = (1.0 - chi[m]) * fab[m] + chi[m] * (rho_s * br[m]) - wall[m];
        }
    }
    // Eq. (15) without the wall momentum, written back as incoming values
    double out_sum = 0.0, in_sum = 0.0;
    n = 0;
    for (int k = k0; k < k1; ++k, ++n) {
        const int d = b.ldir[k];
        out_sum += fab[n];
        in_sum += inc[n] + wall[n];
        A[opp(d) * P + b.lghost[k]] = S(inc[n]);
    }
    if (b.fix == 1) {
        // Eq. (18)
        const double f0 = double(A[node]);
        A[node] = S(f0 + (out_sum - in_sum));
    }
}

// f(0) = f_eq(rho0, u0), stored where the first pull reads it:
// buffer[a][x - e_a] = f_a(0)(x)
template <typename S>
__global__ void k_init_scatter(S* __restrict__ B, const uint8_t* __restrict__ flags,
                               const double* __restrict__ rho0,
                               const double* __restrict__ ux0,
                               const double* __restrict__ uy0, int nx, int ny,
                               int pitch, long long plane) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx || y >= ny) return;
    if (flags[y * pitch + x] & FL_SOLID) return;
    const int o = y * nx + x;
    const double r = rho0[o], ux = ux0[o], uy = uy0[o];
    const double usq = ux * ux + uy * uy;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double eu = edot<double>(a, ux, uy);
        const double f = wt(a) * r * (1.0 + 3.0 * eu + 4.5 * (eu * eu) - 1.5 * usq);
        int xs = x - cx(a), ys = y - cy(a);
        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
        B[a * plane + ys * pitch + xs] = S(f);
    }
}

// psi of the virtual wall density at solid nodes
template <typename R, int EOS>
__global__ void k_psi_wall(R* __restrict__ psiw, const double* __restrict__ rho_wall,
                           const uint8_t* __restrict__ flags, int nx, int ny,
                           int pitch, Phys<R> ph) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx || y >= ny) return;
    const int i = y * pitch + x;
    psiw[i] = (flags[i] & FL_SOLID) ? psi_of<EOS, R>(R(rho_wall[y * nx + x]), ph) : R(0);
}

}  // namespace lbm
